"""Full-field parity at the benchmark's size: the 1025^2 rotated-Sod mesh
(1,050,625 real vertices, Hilbert order, degree-5 two-level stencils), every
real vertex of the GPU residual against the oracle, in FP64 (1e-12) and in
FP32 storage (1e-5, the oracle fed the same FP32-representable state).

The state is the one after one SSP-RK3 step (CFL 0.2) from the Sod data, so
the WENO weights see smeared, not only piecewise-constant, data.  Building the
oracle's stencils and weights takes about 0.6 ms per vertex, so the reference
is computed by a pool of CPU processes (the oracle only; the GPU is not used by
them), each building the oracle for a block of vertices."""
import os
import time

import numpy as np
import pytest
import torch

from tests._helpers import rel_err_per_component

pytestmark = pytest.mark.gpu

N_FULL = 1025
_MESH = {}


def _mesh(N):
    from paper_2102_12933_amd.inputs import make_mesh
    if N not in _MESH:
        _MESH[N] = make_mesh(N, L=1.0, periodic=False, seed=0, ghost_layers=4)
    return _MESH[N]


def _oracle_block(args):
    """Worker: oracle residuals of the given real vertices for each state file."""
    N, verts, paths = args
    torch.set_num_threads(1)
    from oracle.solver import Oracle
    o = Oracle(_mesh(N), deg=5, vertices=verts)
    out = []
    for p in paths:
        w = torch.from_numpy(np.load(p))
        out.append(o.residual(w).numpy())
    return verts, out


def oracle_residuals(N, states, tmpdir, workers=16, blocks=48, log=print):
    """Oracle residual of every real vertex for each state (input numbering),
    from `workers` processes over `blocks` vertex blocks."""
    import concurrent.futures as cf
    import multiprocessing as mp

    m = _mesh(N)
    paths = []
    for i, w in enumerate(states):
        p = os.path.join(str(tmpdir), f"state{i}.npy")
        np.save(p, np.ascontiguousarray(w))
        paths.append(p)
    out = [np.empty((m.nv_real, 4)) for _ in states]
    chunks = np.array_split(np.arange(m.nv_real), blocks)
    t0 = time.time()
    done = 0
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for verts, res in ex.map(_oracle_block, [(N, c, paths) for c in chunks]):
            for o, r in zip(out, res):
                o[verts] = r
            done += len(verts)
            log(f"oracle: {done}/{m.nv_real} vertices ({time.time() - t0:.0f} s)")
    return out


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_full_field_residual_fp64_and_fp32(tmp_path):
    from paper_2102_12933_amd import fdu
    from paper_2102_12933_amd.inputs import sod_state

    def log(msg):
        print(msg, flush=True)

    m = _mesh(N_FULL)
    prep = fdu.Prep(m, deg=5, reorder=2)
    perm = prep.arrays()["perm"]
    iperm = np.argsort(perm)
    s = fdu.Solver(prep, device=0)
    w0 = torch.from_numpy(np.ascontiguousarray(sod_state(m)[perm])).cuda()
    w1, w2, w3 = (torch.empty_like(w0) for _ in range(3))
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    s.cfl_dt(w0, 0.2, dt)
    s.rk_stage(0, w0, w0, w1, dt)
    s.rk_stage(1, w0, w1, w2, dt)
    s.rk_stage(2, w0, w2, w3, dt)
    R64 = s.residual(w3).cpu().numpy()
    w_in = np.empty((m.nv, 4))
    w_in[perm] = w3.cpu().numpy()
    # FP32 storage: the same state rounded to FP32, default variants of the FP32 solver
    w32 = w_in.astype(np.float32).astype(np.float64)
    s32 = fdu.Solver(prep, device=0, precision="f32")
    R32 = s32.residual(torch.from_numpy(np.ascontiguousarray(w32[perm]).astype(np.float32)).cuda())
    R32 = R32.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    log(f"GPU residuals done (variants fp64 {s.variants()}, fp32 {s32.variants()})")
    ref64, ref32 = oracle_residuals(N_FULL, [w_in, w32], tmp_path,
                                    workers=min(16, os.cpu_count() or 1), log=log)
    nr = m.nv_real
    e64 = rel_err_per_component(R64[iperm[:nr]], ref64)
    e32 = rel_err_per_component(R32[iperm[:nr]], ref32)
    log(f"1025^2 all {nr} real vertices: fp64 rel err {e64}, fp32 storage rel err {e32}")
    assert e64.max() <= 1e-12
    assert e32.max() <= 1e-5
