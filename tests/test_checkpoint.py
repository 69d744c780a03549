"""Checkpoints: save/load round trip and the mesh/prep hash check (CPU)."""
import numpy as np
import pytest
import torch

from paper_2102_12933_amd import fdu
from paper_2102_12933_amd.checkpoint import load_state, prep_hash, save_state
from paper_2102_12933_amd.inputs import make_mesh, vortex_state


def test_round_trip_and_hash(tmp_path):
    m = make_mesh(12, L=10.0, periodic=True, seed=2)
    prep = fdu.Prep(m, deg=3, reorder=2)
    w = torch.from_numpy(vortex_state(m))
    p = str(tmp_path / "ck.npz")
    save_state(p, prep, w, step=17, t=1.25)
    w2, step, t = load_state(p, prep, device="cpu")
    assert torch.equal(w2, w) and step == 17 and t == 1.25
    other = fdu.Prep(make_mesh(12, L=10.0, periodic=True, seed=3), deg=3, reorder=2)
    with pytest.raises(ValueError, match="another mesh"):
        load_state(p, other, device="cpu")
    assert prep_hash(fdu.Prep(m, deg=3, reorder=1)) != prep_hash(prep)
