"""Why the FP32 variant stores in FP32 but computes in FP64 (CPU study on the
oracle's formulas).  The same residual evaluated with every table and every
operation in FP32 is compared with FP64 arithmetic on the same FP32-rounded
state:
  * with the Appendix's eps = 1e-40 (below FP32's normal range) the nonlinear
    WENO weights degenerate and the residual is off by ~1e-3 relative;
  * with a representable eps the error is a few 1e-6 on a 33^2 mesh and grows
    about like 1/h (the divergence weights scale like 1/h and multiply
    differences of O(h)), passing 1e-5 from 65^2 on.
So FP32 arithmetic cannot meet a 1e-5 relative bar at the workload sizes,
while FP32 storage with FP64 arithmetic does (tests/test_gpu_fp32.py)."""
import numpy as np
import torch

from oracle.solver import Oracle
from paper_2102_12933_amd.inputs import make_mesh, vortex_state


def _fp32_copy(o):
    """The same oracle object with its tables cast to FP32 (geometry-only
    tensors of the divergence and of both WENO sides)."""
    for obj in (o, o.wenoL, o.wenoR):
        for name, val in list(vars(obj).items()):
            if isinstance(val, torch.Tensor) and val.dtype == torch.float64:
                setattr(obj, name, val.float())
    return o


def _rel_err(N, eps):
    m = make_mesh(N, L=10.0, periodic=True, jitter=0.15, seed=0)
    w = vortex_state(m, beta=5.0, mach=0.5)
    w32 = w.astype(np.float32)
    o = Oracle(m, deg=5, weno_eps=eps)
    R64 = o.residual(torch.from_numpy(w32.astype(np.float64))).numpy()
    R32 = _fp32_copy(o).residual(torch.from_numpy(w32))
    assert R32.dtype == torch.float32
    R32 = R32.double().numpy()
    return (np.abs(R32 - R64).max(0) / np.abs(R64).max(0)).max()


def test_subnormal_eps_breaks_fp32_weights():
    assert _rel_err(33, 1e-40) > 1e-3
    assert _rel_err(33, 1e-20) < 1e-5


def test_fp32_arithmetic_error_grows_with_resolution():
    e33, e65 = _rel_err(33, 1e-20), _rel_err(65, 1e-20)
    assert 1e-7 < e33 < e65
    assert e65 > 1e-5
