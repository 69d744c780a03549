"""Save and resume solver states.

A checkpoint is a ``.npz`` file holding the state (library numbering, the
solver's precision), the step count, the time, and a hash of everything the
state's meaning depends on: the mesh (coordinates, edges, triangles, ghost
data) and the prep settings (degree, level, vertex order, artificial edges).
Loading into a prep with a different hash raises.  Files are read with
``allow_pickle=False``.
"""
from __future__ import annotations

import hashlib

import numpy as np
import torch


def prep_hash(prep) -> str:
    """SHA-256 (hex, 16 chars) of a prep's mesh and settings."""
    m = prep.mesh
    h = hashlib.sha256()
    for a in (m.xy, m.edges, m.tri, m.ghost_src, m.ghost_refl):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    h.update(repr((str(m.periodic), tuple(m.box), prep.deg, prep.level, prep.reorder,
                   bool(getattr(prep, "artificial", False)))).encode())
    return h.hexdigest()[:16]


def save_state(path: str, prep, w: torch.Tensor, step: int = 0, t: float = 0.0) -> None:
    """Write the state w ([nv_total, 4], library numbering) with step, time and hash."""
    np.savez(path, w=w.detach().cpu().numpy(), step=np.int64(step), t=np.float64(t),
             hash=np.array(prep_hash(prep)))


def load_state(path: str, prep, device="cuda"):
    """(w on device, step, t) from a checkpoint written for the same mesh and prep."""
    with np.load(path, allow_pickle=False) as f:
        saved = str(f["hash"])
        if saved != prep_hash(prep):
            raise ValueError(f"checkpoint was written for another mesh or prep ({saved} != {prep_hash(prep)})")
        w = torch.from_numpy(f["w"].copy()).to(device)
        return w, int(f["step"]), float(f["t"])
