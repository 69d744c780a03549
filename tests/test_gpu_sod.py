"""Shock tubes on the GPU path (through the C ABI), against the oracle:

* the two-dimensional shock tube of Sec. 3.2 (periodic [-1, 1]^2 shifted to
  [0, 2]^2, high-pressure square |x|, |y| < 0.25) on the regular diagonalized
  mesh at the paper's spacing (50 x 50, h = 0.04): ten SSP-RK3 steps equal the
  oracle's ten steps, and the run to t = 0.6 at CFL 0.5 stays physical, with
  the final state's residual equal to the oracle's at sampled vertices;
* the same on a 101 x 101 mesh (h = 0.02), and on a jittered lattice with
  degree-3 one-level stencils (the nearly neutral configuration of the linear
  stability study);
* the rotated Sod problem with walls on the regular 1025 x 1025 mesh: 200
  chained SSP-RK3 steps at CFL 0.2 stay physical, and the final state's
  residual equals the oracle's at sampled vertices (near the waves, walls,
  corners, at random).  At CFL 0.5 the first stage already drives the energy
  negative at the vertex where the interface meets a reflecting wall (the
  oracle does the same from 129^2 on; tests/test_oracle_sod.py)."""
import numpy as np
import pytest
import torch

from oracle.solver import Oracle
from paper_2102_12933_amd.inputs import make_mesh, sod_state, square_sod_state
from tests._helpers import rel_err_per_component

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _fdu():
    from paper_2102_12933_amd import fdu
    return fdu


def _setup(m, deg):
    fdu = _fdu()
    prep = fdu.Prep(m, deg=deg, reorder=2)
    perm = prep.arrays()["perm"]
    return fdu.Solver(prep, device=0), perm


def _run(s, w, tend, cfl, max_steps=100000):
    """Chained SSP-RK3 steps to tend (the last step clipped); returns (t, steps)."""
    scratch = torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    t, n = 0.0, 0
    while t < tend - 1e-12 and n < max_steps:
        s.cfl_dt(w, cfl, dt)
        d = min(dt.item(), tend - t)
        dt.fill_(d)
        s.rk_step(w, scratch, dt)
        t += d
        n += 1
    return t, n


def _sampled_residual_err(m, deg, w_dev, perm, s, sample):
    w_in = np.empty((m.nv, 4))
    w_in[perm] = w_dev.cpu().numpy()
    R = s.residual(w_dev).cpu().numpy()
    iperm = np.argsort(perm)
    Ro = Oracle(m, deg=deg, vertices=sample).residual(torch.from_numpy(w_in)).numpy()
    return rel_err_per_component(R[iperm[sample]], Ro)


def test_square_sod_ten_steps_equal_the_oracle():
    m = make_mesh(50, L=2.0, periodic=True, jitter=0.0, diag="uniform")
    s, perm = _setup(m, 5)
    o = Oracle(m, deg=5)
    w0 = square_sod_state(m)
    w = torch.from_numpy(np.ascontiguousarray(w0[perm])).cuda()
    scratch = torch.empty(2 * m.nv, 4, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    wo = torch.from_numpy(w0.copy())
    for _ in range(10):
        s.rk_step(w, scratch, dt, cfl=0.5)
        wo = o.rk3_step(wo, o.cfl_dt(wo, 0.5))
    err = rel_err_per_component(w.cpu().numpy(), wo.numpy()[perm])
    print("square Sod 50^2, 10 steps: rel err", err)
    assert err.max() <= TOL


@pytest.mark.parametrize("N,jitter,deg", [(50, 0.0, 5), (101, 0.0, 5), (50, 0.15, 3)])
def test_square_sod_runs_to_t06(N, jitter, deg):
    m = make_mesh(N, L=2.0, periodic=True, jitter=jitter, diag="uniform", seed=0)
    s, perm = _setup(m, deg)
    w = torch.from_numpy(np.ascontiguousarray(square_sod_state(m)[perm])).cuda()
    t, n = _run(s, w, 0.6, 0.5)
    nbad, first = s.check_state(w)
    print(f"square Sod {N}^2 jitter {jitter} deg {deg}: t = {t:.4f} in {n} steps, bad rows {nbad}")
    assert abs(t - 0.6) < 1e-12 and nbad == 0
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([rng.choice(m.nv_real, 200, replace=False), [0, m.nv_real - 1]]))
    err = _sampled_residual_err(m, deg, w, perm, s, sample)
    print("final state residual rel err (sampled)", err)
    assert err.max() <= TOL


@pytest.mark.slow
def test_rotated_sod_200_chained_steps_regular_1025():
    m = make_mesh(1025, L=1.0, periodic=False, jitter=0.0, diag="uniform", ghost_layers=4)
    s, perm = _setup(m, 5)
    w = torch.from_numpy(np.ascontiguousarray(sod_state(m)[perm])).cuda()
    scratch = torch.empty(2 * m.nv, 4, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    for _ in range(200):
        s.rk_step(w, scratch, dt, cfl=0.2)
    nbad, _ = s.check_state(w)
    print("rotated Sod 1025^2 regular, 200 steps at CFL 0.2: bad rows", nbad, "last dt", dt.item())
    assert nbad == 0
    rng = np.random.default_rng(2)
    a = np.deg2rad(30.0)
    xy = m.xy[:m.nv_real]
    sd = (xy[:, 0] - 0.5) * np.cos(a) + (xy[:, 1] - 0.5) * np.sin(a)
    near = np.nonzero(np.abs(sd) < 0.1)[0]
    wall = np.nonzero((xy[:, 1] < 1e-12) | (xy[:, 1] > 1 - 1e-12))[0]
    sample = np.unique(np.concatenate([rng.choice(near, 250, replace=False), rng.choice(m.nv_real, 100, replace=False),
                                       rng.choice(wall, 50, replace=False), [0, 1024, 1025 * 1024, m.nv_real - 1]]))
    err = _sampled_residual_err(m, 5, w, perm, s, sample)
    print("final state residual rel err (sampled)", err)
    assert err.max() <= TOL
