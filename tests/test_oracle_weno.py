"""Pins of the oracle's non-uniform WENO5 (Appendix) against facts fixed by the
paper and by interpolation theory, independent of the oracle's own formulas."""
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle.nuweno import NUWeno5, linear_weights, substencil_coefficients, uniform_weno5

HERE = os.path.dirname(__file__)


def random_stencils(n, seed=0, jitter=0.5):
    """Five points around a midpoint at 0 with x_i = -x_{i+1}; others moved by up
    to jitter * spacing (the Sec. 2.3.2 perturbation)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 2.0, n)
    x = np.stack([-2.5 * d, -1.5 * d, -0.5 * d, 0.5 * d, 1.5 * d], 1)
    x[:, [0, 1, 4]] += rng.uniform(-jitter, jitter, (n, 3)) * d[:, None]
    return x


def lagrange_at_zero(nodes):
    """Lagrange basis values at 0 by solving the Vandermonde system V^T l = e_0."""
    V = np.vander(nodes, increasing=True)          # V[m, p] = x_m^p
    e0 = np.zeros(len(nodes))
    e0[0] = 1.0
    return np.linalg.solve(V.T, e0)


def test_substencil_coefficients_are_lagrange_basis():
    x = random_stencils(200, seed=1)
    sub = substencil_coefficients(x)
    for i in range(x.shape[0]):
        for k in range(3):
            np.testing.assert_allclose(sub[i, k], lagrange_at_zero(x[i, k:k + 3]), rtol=1e-12, atol=1e-13)


def test_linear_weights_sum_to_one_and_rebuild_S5():
    x = random_stencils(500, seed=2)
    C = linear_weights(x)
    np.testing.assert_allclose(C.sum(1), 1.0, atol=1e-14)
    sub = substencil_coefficients(x)
    for i in range(x.shape[0]):
        comb = np.zeros(5)
        for k in range(3):
            comb[k:k + 3] += C[i, k] * sub[i, k]
        np.testing.assert_allclose(comb, lagrange_at_zero(x[i]), rtol=1e-11, atol=1e-12)


def read_golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "uniform_weno5.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *rest = line.split()
            vals[key] = [float(Fraction(r)) for r in rest]
    return vals


def test_uniform_special_case_matches_textbook():
    g = read_golden()
    x = np.array([[-2.5, -1.5, -0.5, 0.5, 1.5]]) * 0.37
    np.testing.assert_allclose(linear_weights(x)[0], g["C"], rtol=0, atol=1e-15)
    sub = substencil_coefficients(x)[0]
    for k in range(3):
        np.testing.assert_allclose(sub[k] * 8, g[f"S{k}x8"], atol=1e-13)
    w = NUWeno5(x)
    eye = torch.eye(5, dtype=torch.float64).reshape(1, 5, 5)
    lin = w.linear(eye)[0].numpy()
    np.testing.assert_allclose(lin * 128, g["S5x128"], atol=1e-12)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_linear_scheme_reproduces_degree_4(deg):
    x = random_stencils(300, seed=3)
    rng = np.random.default_rng(deg)
    c = rng.normal(size=deg + 1)
    u = torch.from_numpy(np.polyval(c, x))
    w = NUWeno5(x)
    np.testing.assert_allclose(w.linear(u).numpy(), c[-1], rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_nonlinear_scheme_reproduces_degree_2(deg):
    x = random_stencils(300, seed=4)
    rng = np.random.default_rng(10 + deg)
    c = rng.normal(size=deg + 1)
    u = torch.from_numpy(np.polyval(c, x))
    np.testing.assert_allclose(NUWeno5(x)(u).numpy(), c[-1], rtol=1e-11, atol=1e-11)


def test_smoothness_indicator_equals_quadrature_of_definition():
    x = random_stencils(100, seed=5)
    rng = np.random.default_rng(6)
    u = rng.normal(size=(100, 5))
    beta = NUWeno5(x).smoothness(torch.from_numpy(u)).numpy()
    gx, gw = np.polynomial.legendre.leggauss(8)
    for i in range(100):
        a, b = x[i, 2], x[i, 3]
        dx = b - a
        t = 0.5 * (a + b) + 0.5 * (b - a) * gx
        for k in range(3):
            q = np.polyfit(x[i, k:k + 3], u[i, k:k + 3], 2)
            d1 = np.polyval(np.polyder(q, 1), t)
            d2 = np.polyval(np.polyder(q, 2), t)
            ref = 0.5 * (b - a) * np.sum(gw * (dx * d1 ** 2 + dx ** 3 * d2 ** 2))
            assert abs(beta[i, k] - ref) <= 1e-10 * max(1.0, abs(ref))


def test_smoothness_indicator_uniform_closed_form():
    """Hand-derived on x = (-5/2..3/2): beta_0 = (u0 - 3u1 + 2u2)^2 + 13/12 (u0 - 2u1 + u2)^2,
    beta_1 = (u3 - u2)^2 + 13/12 (u1 - 2u2 + u3)^2, beta_2 = (u3 - u2)^2 + 13/12 (u2 - 2u3 + u4)^2."""
    rng = np.random.default_rng(7)
    u = rng.normal(size=(50, 5))
    x = np.tile([-2.5, -1.5, -0.5, 0.5, 1.5], (50, 1))
    beta = NUWeno5(x).smoothness(torch.from_numpy(u)).numpy()
    u0, u1, u2, u3, u4 = u.T
    ref = np.stack([(u0 - 3 * u1 + 2 * u2) ** 2 + 13 / 12 * (u0 - 2 * u1 + u2) ** 2,
                    (u3 - u2) ** 2 + 13 / 12 * (u1 - 2 * u2 + u3) ** 2,
                    (u3 - u2) ** 2 + 13 / 12 * (u2 - 2 * u3 + u4) ** 2], 1)
    np.testing.assert_allclose(beta, ref, rtol=1e-12, atol=1e-13)


def test_discontinuity_gets_no_weight():
    """A jump inside S_0 and S_1 only leaves S_2 (ENO property): omega_2 -> 1."""
    x = random_stencils(50, seed=8, jitter=0.3)
    u = torch.from_numpy(np.where(np.arange(5)[None, :] <= 1, 1.0, 0.0) * np.ones((50, 1)))
    om = NUWeno5(x).weights(u).numpy()
    np.testing.assert_allclose(om[:, 2], 1.0, atol=1e-12)


def _order(hs, errs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def test_sin_perturbed_stencils_order():
    """Sec. 2.3.2: sin x, five points moved randomly by up to 50% of the spacing:
    NU-WENO5 keeps fifth order, standard WENO5 drops to near first order."""
    hs = 2.0 ** -np.arange(2, 7)
    rng = np.random.default_rng(9)
    nu_err, u_err = [], []
    for h in hs:
        xc = rng.uniform(0, 2 * np.pi, 400)
        x = np.tile(np.array([-2.5, -1.5, -0.5, 0.5, 1.5]) * h, (400, 1))
        x[:, [0, 1, 4]] += rng.uniform(-0.5, 0.5, (400, 3)) * h
        u = torch.from_numpy(np.sin(xc[:, None] + x))
        exact = np.sin(xc)
        nu_err.append(np.abs(NUWeno5(x)(u).numpy() - exact).mean())
        u_err.append(np.abs(uniform_weno5(400)(u).numpy() - exact).mean())
    assert abs(_order(hs, nu_err) - 5.0) < 0.6, nu_err
    assert abs(_order(hs, u_err) - 1.0) < 0.4, u_err


def test_middle_substencils_are_shared_by_the_two_sides():
    """The left state of an edge interpolates on (L3, L2, L1, R1, R2), the right
    state on the mirrored (R3, R2, R1, L1, L2).  The left's sub-stencils
    (L2, L1, R1) and (L1, R1, R2) are the right's (R1, L1, L2) and (R2, R1, L1):
    the same quadratics, evaluated at the same midpoint, with smoothness
    indicators integrated over the same middle edge, so their values and
    indicators agree between the sides (the edge kernel evaluates them once)."""
    rng = np.random.default_rng(11)
    n = 200
    d = rng.uniform(0.5, 2.0, n)                       # middle-edge length
    gaps = rng.uniform(0.3, 3.0, (n, 4)) * d[:, None]
    s = np.stack([-d / 2 - gaps[:, 0] - gaps[:, 1], -d / 2 - gaps[:, 1], -d / 2,
                  d / 2, d / 2 + gaps[:, 2], d / 2 + gaps[:, 2] + gaps[:, 3]], 1)
    u = torch.from_numpy(rng.normal(size=(n, 6)))
    left = NUWeno5(s[:, 0:5])
    right = NUWeno5(-s[:, ::-1][:, 0:5])
    ul, ur = u[:, 0:5], torch.flip(u, [1])[:, 0:5]
    vl, _ = left._sub_values(ul)
    vr, _ = right._sub_values(ur)
    bl, br = left.smoothness(ul), right.smoothness(ur)
    for kl, kr in ((1, 2), (2, 1)):
        assert torch.allclose(vl[:, kl], vr[:, kr], rtol=1e-12, atol=1e-12)
        assert torch.allclose(bl[:, kl], br[:, kr], rtol=1e-11, atol=1e-13)
    # the outer ones are not shared
    assert not torch.allclose(vl[:, 0], vr[:, 0], rtol=1e-3)
