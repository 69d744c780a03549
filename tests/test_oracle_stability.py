"""Linear stability of the semi-discrete scheme, from the oracle's Jacobian.

At a uniform state every WENO smoothness indicator vanishes and its gradient
too, so the residual's Jacobian there is that of the linear scheme (optimal
weights).  Its eigenvalues say whether the method of lines can grow errors.
These tests record what the spectrum shows on small periodic meshes (h = 1,
free stream (u, v) = (0.5, 0.3), c = 1), to explain which configurations
can be run for long times:

* regular diagonalized mesh, degree 3 on one-level stencils: no eigenvalue
  with a positive real part (rounding level);
* the same lattice with the quad diagonals drawn at random (no jitter): a real
  eigenvalue of about +0.1/h.  It stays when the edge states are replaced by the
  mean of the edge's end states (no WENO, no upwinding, no 1D stencil), so the
  growing mode lives in the least-squares divergence of Sec. 2.2.1 on irregular
  connectivity, not in the edge interpolation (the edge-side readings, Roe or
  Rusanov, characteristic or conservative variables, Catmull-Rom or chordal
  arcs, move it by a few percent only);
* jittered lattice with uniform diagonals: degree 3 one-level is nearly
  neutral, degree 5 two-level has a growing mode of about +0.1/h, matching which
  of them run the paper's square shock tube to t = 0.6 (tests/test_oracle_sod.py).

WENO eps is 1e-6 here only so that autograd through the weights stays finite
(at eps = 1e-40 the derivative of 1/(beta + eps) overflows); at a uniform
state the weights and their derivatives do not depend on eps.
"""
import numpy as np
import pytest
import torch

from oracle.solver import Oracle
from paper_2102_12933_amd.inputs import make_mesh, primitive_to_conservative


def _max_real_eigenvalue(N, jitter, diag, deg, level, central_edges=False):
    m = make_mesh(N, L=float(N), periodic=True, jitter=jitter, diag=diag, seed=0)
    o = Oracle(m, deg=deg, level=level, weno_eps=1e-6)
    if central_edges:
        def mean_of_ends(w):
            W6 = w[o.sten_t]
            a = 0.5 * (W6[:, 2] + W6[:, 3])
            return a, a
        o.edge_states = mean_of_ends
    q = primitive_to_conservative(np.array(1.0), np.array(0.5), np.array(0.3), np.array(1.0 / 1.4))
    w = torch.from_numpy(np.tile(q, (m.nv, 1)))
    J = torch.autograd.functional.jacobian(o.residual, w, vectorize=True).reshape(w.numel(), w.numel())
    ev = np.linalg.eigvals(J.numpy())
    return float(ev.real.max()), float(np.abs(ev).max())


@pytest.mark.slow
def test_regular_mesh_has_no_growing_mode():
    re, rho = _max_real_eigenvalue(12, 0.0, "uniform", 3, 1)
    assert rho > 1.0 and re <= 1e-12 * rho, (re, rho)


@pytest.mark.slow
def test_random_diagonals_grow_in_the_divergence():
    re, _ = _max_real_eigenvalue(12, 0.0, "random", 3, 1)
    re_c, _ = _max_real_eigenvalue(12, 0.0, "random", 3, 1, central_edges=True)
    assert re > 0.05 and re_c > 0.05, (re, re_c)


@pytest.mark.slow
def test_jittered_uniform_diagonals_degree_three_vs_five():
    re3, _ = _max_real_eigenvalue(12, 0.15, "uniform", 3, 1)
    re5, _ = _max_real_eigenvalue(12, 0.15, "uniform", 5, 2)
    assert re3 < 2e-3 and re5 > 0.05, (re3, re5)
