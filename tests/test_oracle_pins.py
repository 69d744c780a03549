"""Pins of oracle functions that the scheme-level tests leave open, each checked
against something other than the oracle's own formula:

* the SSP-RK3 stage form (Sec. 3, the Shu-Osher scheme): for a linear residual
  R(w) = lambda w the three stages take the closed-form values 1 + z,
  1 + z/2 + z^2/4 and 1 + z + z^2/2 + z^3/6 (z = lambda dt), and the stages
  chained on the real residual reproduce the full step;
* the residual's vector-Jacobian product: dot test and central finite
  differences of the residual itself (no autograd on the checking side);
* the positivity fallback (an addition to the paper's scheme): an edge whose
  interpolated density is negative on both sides takes its end vertex states;
* Harten's entropy fix of the Roe flux: value delta/2 at a zero eigenvalue and
  a C1 junction with |lambda| at |lambda| = delta.
"""
import numpy as np
import pytest
import torch

from oracle import euler
from oracle.solver import Oracle
from paper_2102_12933_amd.inputs import make_mesh, primitive_to_conservative, sod_state, vortex_state


def _linear_oracle(lam):
    m = make_mesh(6, L=1.0, periodic=True)
    o = Oracle(m, deg=3)
    A = torch.tensor([[lam.real, -lam.imag], [lam.imag, lam.real]], dtype=torch.float64)
    o._full_residual = lambda w: w @ A.T
    return o


@pytest.mark.parametrize("lam,dt", [(-0.7 + 0.4j, 0.9), (0.3 - 1.1j, 0.5), (-2.0 + 0.0j, 0.6)])
def test_rk3_stages_closed_form(lam, dt):
    """Each stage of the stage form against its closed-form multiplier (a
    swapped a_k / b_k pair or a wrong stage input changes these values)."""
    o = _linear_oracle(lam)
    z = lam * dt
    w0 = torch.tensor([[1.0, 0.0]], dtype=torch.float64)
    w1 = o.rk3_stage(0, w0, w0, dt)
    w2 = o.rk3_stage(1, w0, w1, dt)
    w3 = o.rk3_stage(2, w0, w2, dt)
    for got, ref in ((w1, 1 + z), (w2, 1 + z / 2 + z * z / 4), (w3, 1 + z + z * z / 2 + z ** 3 / 6)):
        np.testing.assert_allclose([got[0, 0].item(), got[0, 1].item()], [ref.real, ref.imag], rtol=1e-14, atol=1e-15)
    # stage 0 ignores w_n: any w_n gives the same first stage
    junk = torch.tensor([[123.0, -7.0]], dtype=torch.float64)
    assert torch.equal(o.rk3_stage(0, junk, w0, dt), w1)


def test_rk3_stages_compose_the_step():
    """On the real residual (walled Sod and periodic vortex), three stages in a
    row equal rk3_step to rounding."""
    for m, w in ((make_mesh(14, periodic=False, seed=4, ghost_layers=4), None),
                 (make_mesh(14, L=10.0, periodic=True, seed=4), "vortex")):
        o = Oracle(m, deg=5)
        w0 = torch.from_numpy(vortex_state(m, beta=5.0, mach=0.5) if w else sod_state(m))
        dt = o.cfl_dt(w0, 0.4)
        w1 = o.rk3_stage(0, w0, w0, dt)
        w2 = o.rk3_stage(1, w0, w1, dt)
        w3 = o.rk3_stage(2, w0, w2, dt)
        ref = o.rk3_step(w0, dt)
        nr = m.nv_real
        err = (w3[:nr] - ref[:nr]).abs().max(0).values / ref[:nr].abs().max(0).values
        assert float(err.max()) <= 1e-15, err


def _smooth_walled_state(m, seed):
    """A smooth, positive state on a walled mesh (no discontinuity, so the
    residual is differentiable everywhere)."""
    rng = np.random.default_rng(seed)
    x, y = m.xy[:, 0], m.xy[:, 1]
    a = rng.uniform(0.5, 1.5, 5)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * a[0] * x) * np.cos(2 * np.pi * a[1] * y)
    u = 0.3 * np.cos(2 * np.pi * a[2] * y)
    v = 0.2 * np.sin(2 * np.pi * a[3] * x)
    p = 1.0 + 0.1 * np.cos(2 * np.pi * a[4] * (x + y))
    return primitive_to_conservative(rho, u, v, p)


@pytest.mark.parametrize("case", ["vortex", "walled"])
def test_residual_vjp_dot_test_and_central_differences(case):
    """(dR/dw)^T Rbar from residual_vjp against directional derivatives of the
    residual by central differences, on a 12^2 mesh at WENO eps = 1e-6 (with
    eps = 1e-40 the nonlinear weights are not differentiable where the data are
    near uniform): <vjp(v), u> = <v, J u> for random u, v, and the transposed
    product equals the finite-difference Jacobian applied column by column on a
    few unit directions.  Step h = 1e-7 relative to each component's scale:
    at eps = 1e-6 the weights of the nearly uniform far field are strongly
    nonlinear, and the O(h^2) error of central differences is 6e-6 relative at
    h = 1e-6 and 6e-8 at h = 1e-7 (measured: the differences converge to the
    product as h^2 down to h = 1e-8)."""
    if case == "vortex":
        m = make_mesh(12, L=10.0, periodic=True, seed=5)
        w0 = vortex_state(m, beta=5.0, mach=0.5)
    else:
        m = make_mesh(12, periodic=False, seed=5, ghost_layers=4)
        w0 = _smooth_walled_state(m, 5)
    o = Oracle(m, deg=5, weno_eps=1e-6)
    w = torch.from_numpy(w0)
    nr = m.nv_real
    rng = np.random.default_rng(11)
    scale = np.abs(w0[:nr]).max(0)
    h = 1e-7
    for trial in range(3):
        u = np.zeros_like(w0)
        u[:nr] = rng.standard_normal((nr, 4)) * scale       # ghost rows are overwritten by the fill
        v = rng.standard_normal((nr, 4))
        ut = torch.from_numpy(u)
        with torch.no_grad():
            Ju = (o.residual(w + h * ut) - o.residual(w - h * ut)) / (2 * h)
        lhs = float((torch.from_numpy(v) * Ju).sum())
        g = o.residual_vjp(w, torch.from_numpy(v))
        rhs = float((g * ut).sum())
        assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + np.abs(v).sum() * float(Ju.abs().max()) * 1e-3), (trial, lhs, rhs)
    # column checks: unit perturbations of single state entries
    for (vi, k) in ((0, 0), (nr // 2, 1), (nr - 1, 3), (7, 2)):
        e = torch.zeros_like(w)
        e[vi, k] = scale[k]
        with torch.no_grad():
            col = (o.residual(w + h * e) - o.residual(w - h * e)) / (2 * h)
        vv = torch.from_numpy(rng.standard_normal((nr, 4)))
        g = o.residual_vjp(w, vv)
        ref = float((vv * col).sum())
        got = float(g[vi, k]) * scale[k]
        assert abs(got - ref) <= 1e-6 * (float((vv.abs() * col.abs()).sum()) + 1e-30), (vi, k, got, ref)


def test_positivity_fallback_takes_end_vertex_states():
    """A density dip on the two middle vertices of a straight, equally spaced
    edge stencil (regular mesh): densities (1, 1, d, d, 1, 1) with one
    temperature and zero velocity.  Every quadratic sub-stencil of NU-WENO5 is
    negative at the midpoint (through (-1.5, 1), (-0.5, d), (0.5, d) it is
    d - (1 - d)/8 there; the outer two are lower still), so both interpolated
    states have negative density whatever the nonlinear weights, and the
    fallback returns the end vertex states exactly.  Without the fallback the
    same edge keeps the negative densities."""
    N = 12
    m = make_mesh(N, L=float(N), periodic=True, jitter=0.0, diag="uniform")
    o = Oracle(m, deg=5)
    off = Oracle(m, deg=5, positivity=False)
    # an edge along x in the middle row: vertices (i, j) -> (i + 1, j), id = i N + j
    a, b = 5 * N + 6, 6 * N + 6
    k = int(np.nonzero((o.sten6[:, 2] == a) & (o.sten6[:, 3] == b))[0][0])
    assert list(o.sten6[k]) == [3 * N + 6, 4 * N + 6, a, b, 7 * N + 6, 8 * N + 6]
    d = 0.02
    rho = np.ones(m.nv)
    rho[[a, b]] = d
    w = torch.from_numpy(primitive_to_conservative(rho, np.zeros(m.nv), np.zeros(m.nv), 0.8 * rho))
    wl_off, wr_off = off.edge_states(w)
    assert float(wl_off[k, 0]) < 0 and float(wr_off[k, 0]) < 0
    wl, wr = o.edge_states(w)
    assert torch.equal(wl[k], w[a]) and torch.equal(wr[k], w[b])
    # edges whose interpolated states are physical are left alone
    ok = (o._physical(wl_off) & o._physical(wr_off)).numpy()
    assert ok.sum() > 0
    assert torch.equal(wl[ok], wl_off[ok]) and torch.equal(wr[ok], wr_off[ok])
    # the flux of the fallback edge is the exact normal flux of the common end state
    r = o.edge_fluxes(w)
    np.testing.assert_allclose(r[k].numpy(), euler.normal_flux(w[a], o.n_e[k]).numpy(), rtol=1e-14, atol=1e-15)


def test_harten_entropy_fix_values():
    """|lambda| -> (lambda^2 + delta^2) / (2 delta) inside |lambda| < delta:
    delta/2 at lambda = 0, and value and slope continuous at |lambda| = delta
    (so the modified eigenvalue is C1, as the adjoint needs)."""
    delta = torch.tensor([0.37], dtype=torch.float64)
    assert float(euler.harten(torch.zeros(1, dtype=torch.float64), delta)) == pytest.approx(0.185, rel=1e-15)
    for s in (1.0, -1.0):
        inside = torch.tensor([s * 0.37 * (1 - 1e-9)], dtype=torch.float64, requires_grad=True)
        outside = torch.tensor([s * 0.37 * (1 + 1e-9)], dtype=torch.float64, requires_grad=True)
        vi, vo = euler.harten(inside, delta), euler.harten(outside, delta)
        assert abs(vi.item() - 0.37) < 1e-9 and abs(vo.item() - 0.37) < 1e-9
        (gi,) = torch.autograd.grad(vi, inside)
        (go,) = torch.autograd.grad(vo, outside)
        assert abs(float(gi) - s) < 1e-8 and float(go) == s
    # below delta the fix is strictly above |lambda| and increasing in |lambda|
    x = torch.linspace(0, 0.37, 50, dtype=torch.float64)
    y = euler.harten(x, delta)
    assert bool((y[:-1] >= x[:-1]).all()) and bool((torch.diff(y) > 0).all())


def test_roe_flux_enters_the_entropy_fix():
    """A transonic pair (Roe-averaged u_n - c inside (-delta, delta)): the Roe
    flux with the fix differs from the flux without it exactly by the change of
    dissipation on the sonic wave, (fix(l) - |l|) alpha_1 r_1 / 2, where alpha_1
    is the sonic wave's strength; the other three waves are untouched."""
    rho, p = 1.0, 1.0
    c = np.sqrt(1.4 * p / rho)
    n = torch.tensor([1.0, 0.0], dtype=torch.float64)
    wl = torch.from_numpy(primitive_to_conservative(np.array(1.0), np.array(0.98 * c), np.array(0.1), np.array(1.0)))
    wr = torch.from_numpy(primitive_to_conservative(np.array(0.9), np.array(1.03 * c), np.array(0.1), np.array(0.85)))
    u, v, H, cr = euler.roe_average(wl, wr)
    lam = euler.eigenvalues(u, v, cr, n)
    delta = 0.1 * cr
    assert abs(float(lam[0])) < float(delta)                     # sonic wave inside the fix
    assert bool((lam[1:].abs() > delta).all())
    f_fix = euler.roe_flux(wl, wr, n, delta_frac=0.1)
    f_raw = euler.roe_flux(wl, wr, n, delta_frac=1e-30)           # delta -> 0: no fix anywhere
    R = euler.right_eigenvectors(u, v, H, cr, n)
    alpha = torch.linalg.solve(R, wr - wl)
    l1 = float(lam[0])
    fix = (l1 * l1 + float(delta) ** 2) / (2 * float(delta))
    expect = -0.5 * (fix - abs(l1)) * alpha[0] * R[:, 0]
    np.testing.assert_allclose((f_fix - f_raw).numpy(), expect.numpy(), rtol=1e-10, atol=1e-15)
