"""GPU tests of the hand-written adjoint (through the C ABI): residual VJP and
SSP-RK3 step VJP against the oracle's autograd VJP (1e-12 relative), a
finite-difference check, and the unrolled-gradient workload: isentropic vortex,
20 SSP-RK3 steps at a fixed dt, checkpoints every 5 steps, gradient of the
domain-integrated entropy deviation J = sum_v A_v (p_v / rho_v^gamma - 1) with
respect to the initial state and to the vortex strength, against central
finite differences (h = 1e-6) and, on a small mesh, the oracle's VJP.

All adjoint cases use WENO eps = 1e-6: with the paper's eps = 1e-40 the
smoothness indicators of near-uniform flow (the vortex far field) sit at
rounding level, the nonlinear weights switch sub-stencils on perturbations of
order 1e-15, and the derivative there is rounding noise (finite differences of
the residual do not converge as h -> 0; they do with eps = 1e-6 or with the
linear weights)."""
import numpy as np
import pytest
import torch

from oracle.solver import Oracle
from paper_2102_12933_amd.inputs import make_mesh, vertex_areas, vortex_state
from tests._helpers import rel_err_per_component
from tests.test_gpu_parity import perturbed_sod

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _fdu():
    from paper_2102_12933_amd import fdu
    return fdu


ADJ_EPS = 1e-6


class AdjCase:
    def __init__(self, N, periodic, ghosts, deg, state, seed=0, **params):
        fdu = _fdu()
        params.setdefault("weno_eps", ADJ_EPS)
        self.m = make_mesh(N, L=10.0 if periodic else 1.0, periodic=periodic, seed=seed, ghost_layers=ghosts)
        self.prep = fdu.Prep(self.m, deg=deg, reorder=1)
        self.perm = self.prep.arrays()["perm"]
        self.s = fdu.Solver(self.prep, device=0, **params)
        self.s.enable_adjoint()
        okw = {"weno_eps": params["weno_eps"]}
        if "positivity" in params:
            okw["positivity"] = bool(params["positivity"])
        if "weno_power" in params:
            okw["weno_power"] = params["weno_power"]
        if "riemann" in params:
            okw["riemann"] = "roe" if params["riemann"] == 0 else "rusanov"
        if params.get("interpolation"):
            okw["interpolation"] = "conservative"
        if params.get("uniform_weno"):
            okw["weno"] = "uniform"
        self.o = Oracle(self.m, deg=deg, **okw)
        self.w0 = vortex_state(self.m, beta=5.0, mach=0.5) if state == "vortex" else perturbed_sod(self.m)

    def dev(self, a):
        return torch.from_numpy(np.ascontiguousarray(a[self.perm])).cuda()


CASES = [(20, True, 0, 5, "vortex", {}), (24, True, 0, 3, "vortex", {}), (16, False, 4, 5, "sod", {}),
         (16, False, 4, 5, "sod", dict(positivity=0)), (18, True, 0, 5, "vortex", dict(weno_power=2)),
         (18, True, 0, 5, "vortex", dict(riemann=1)), (16, False, 4, 5, "sod", dict(interpolation=1)),
         (18, True, 0, 5, "vortex", dict(uniform_weno=1))]


@pytest.mark.parametrize("N,per,G,deg,state,params", CASES)
def test_residual_vjp_matches_oracle(N, per, G, deg, state, params):
    c = AdjCase(N, per, G, deg, state, **params)
    rng = np.random.default_rng(N)
    Rbar = rng.normal(size=(c.m.nv_real, 4))
    wb = c.s.residual_vjp(c.dev(c.w0), c.dev(np.concatenate([Rbar, np.zeros((c.m.ng, 4))]))[:c.m.nv_real].contiguous())
    ref = c.o.residual_vjp(torch.from_numpy(c.w0), torch.from_numpy(Rbar)).numpy()
    err = rel_err_per_component(wb.cpu().numpy(), ref[c.perm])
    print(N, per, deg, state, params, "residual vjp rel err", err)
    assert err.max() <= TOL


@pytest.mark.parametrize("N,per,G,deg,state", [(16, True, 0, 5, "vortex"), (14, False, 4, 5, "sod")])
def test_rk_step_vjp_matches_oracle(N, per, G, deg, state):
    c = AdjCase(N, per, G, deg, state)
    dt = 0.5 * c.o.cfl_dt(torch.from_numpy(c.w0), 0.3)
    rng = np.random.default_rng(1)
    ybar = np.concatenate([rng.normal(size=(c.m.nv_real, 4)), np.zeros((c.m.ng, 4))])
    x = torch.from_numpy(c.w0.copy()).requires_grad_(True)
    y = c.o.rk3_step(x, dt)
    (ref,) = torch.autograd.grad(y[:c.m.nv_real], x, torch.from_numpy(ybar[:c.m.nv_real]))
    wn = c.dev(c.w0)
    out = torch.empty_like(wn)
    scratch = torch.empty(4 * c.m.nv, 4, dtype=torch.float64, device="cuda")
    c.s.rk_step_vjp(wn, c.dev(ybar), out, scratch, dt)
    err = rel_err_per_component(out.cpu().numpy(), ref.numpy()[c.perm])
    print("rk step vjp rel err", err)
    assert err.max() <= TOL


def test_residual_vjp_finite_difference():
    c = AdjCase(20, True, 0, 5, "vortex", seed=4)
    rng = np.random.default_rng(2)
    d = rng.normal(size=c.w0.shape) * np.array([1e-2, 1e-2, 1e-2, 1e-2])
    Rbar = rng.normal(size=(c.m.nv_real, 4))
    h = 1e-6
    Rp = c.s.residual(c.dev(c.w0 + h * d)).cpu().numpy()
    Rm = c.s.residual(c.dev(c.w0 - h * d)).cpu().numpy()
    fd = np.sum(Rbar[c.perm[:c.m.nv_real]] * (Rp - Rm) / (2 * h))
    wb = c.s.residual_vjp(c.dev(c.w0), c.dev(np.concatenate([Rbar, np.zeros((c.m.ng, 4))]))[:c.m.nv_real].contiguous())
    ad = np.sum(wb.cpu().numpy() * d[c.perm])
    assert abs(ad - fd) <= 1e-5 * abs(ad), (ad, fd)


def smooth_direction(m, rng, kmax=3):
    """Seeded random perturbation of the initial state made of low Fourier modes
    of the periodic box (resolved on the mesh), one field per component."""
    x = 2 * np.pi * m.xy[:, 0] / m.box[0]
    y = 2 * np.pi * m.xy[:, 1] / m.box[1]
    d = np.zeros((m.nv, 4))
    for c in range(4):
        for kx in range(kmax + 1):
            for ky in range(-kmax, kmax + 1):
                a, b = rng.normal(size=2)
                d[:, c] += a * np.cos(kx * x + ky * y) + b * np.sin(kx * x + ky * y)
    return d


def _entropy_functional(solver, areas_dev, gamma=1.4):
    def J(w):
        wr = w[:solver.nv_real]
        rho = wr[:, 0]
        p = (gamma - 1.0) * (wr[:, 3] - 0.5 * (wr[:, 1] ** 2 + wr[:, 2] ** 2) / rho)
        return torch.sum(areas_dev * (p / rho ** gamma - 1.0))
    return J


def _unrolled_grad_check(N, nsteps, ckpt, oracle_check):
    from paper_2102_12933_amd.autograd import rk_unroll
    from paper_2102_12933_amd.inputs import vortex_state
    fdu = _fdu()
    m = make_mesh(N, L=10.0, periodic=True, seed=0)
    prep = fdu.Prep(m, deg=5, reorder=1)
    perm = prep.arrays()["perm"]
    s = fdu.Solver(prep, device=0, weno_eps=ADJ_EPS)
    s.enable_adjoint()
    beta = 5.0
    w0 = vortex_state(m, beta=beta, mach=0.5)
    w0d = torch.from_numpy(w0[perm]).cuda()
    dt = float(s.cfl_dt(w0d, 0.5).item())            # frozen at its t = 0 value
    A = torch.from_numpy(vertex_areas(m)[perm][:m.nv_real]).cuda()
    J = _entropy_functional(s, A)
    x = w0d.clone().requires_grad_(True)
    val = J(rk_unroll(s, x, nsteps, dt, ckpt))
    (g,) = torch.autograd.grad(val, x)
    g = g.cpu().numpy()

    def Jfwd(wi):
        with torch.no_grad():
            return float(J(rk_unroll(s, torch.from_numpy(wi).cuda(), nsteps, dt, ckpt)))

    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(2):
        d = smooth_direction(m, rng)[perm]
        fd = (Jfwd(w0[perm] + h * d) - Jfwd(w0[perm] - h * d)) / (2 * h)
        ad = float(np.sum(g * d))
        print(f"N={N} direction: adjoint {ad:.12e} fd {fd:.12e}")
        assert abs(ad - fd) <= 1e-5 * abs(ad)
    # vortex strength through the initial state: dw0/dbeta by complex step
    cs = 1e-30
    from paper_2102_12933_amd.inputs import primitive_to_conservative, vortex_primitive
    wc = primitive_to_conservative(*vortex_primitive(m.xy, 0.0, beta=beta + 1j * cs, mach=0.5, box=m.box,
                                                     periodic=True, center=(5.0, 5.0)))
    dw_db = np.imag(wc)[perm] / cs
    ad_b = float(np.sum(g * dw_db))
    hb = 1e-6
    fd_b = (Jfwd(vortex_state(m, beta=beta + hb, mach=0.5)[perm]) - Jfwd(vortex_state(m, beta=beta - hb, mach=0.5)[perm])) / (2 * hb)
    print(f"N={N} dJ/dbeta adjoint {ad_b:.12e} fd {fd_b:.12e}")
    assert abs(ad_b - fd_b) <= 1e-5 * abs(ad_b)
    if oracle_check:
        o = Oracle(m, deg=5, weno_eps=ADJ_EPS)
        xo = torch.from_numpy(w0.copy()).requires_grad_(True)
        w = xo
        for _ in range(nsteps):
            w = o.rk3_step(w, dt)
        Ao = torch.from_numpy(vertex_areas(m)[:m.nv_real])
        wr = w[:m.nv_real]
        rho = wr[:, 0]
        p = 0.4 * (wr[:, 3] - 0.5 * (wr[:, 1] ** 2 + wr[:, 2] ** 2) / rho)
        (go,) = torch.autograd.grad(torch.sum(Ao * (p / rho ** 1.4 - 1.0)), xo)
        err = rel_err_per_component(g, go.numpy()[perm])
        print("unrolled gradient vs oracle", err)
        assert err.max() <= 1e-11


def test_unrolled_gradient_small_vs_oracle():
    _unrolled_grad_check(20, 20, 5, oracle_check=True)


@pytest.mark.slow
def test_unrolled_gradient_257():
    """Adjoint workload at 257^2 (66,049 vertices): 20 steps, checkpoints every 5."""
    _unrolled_grad_check(257, 20, 5, oracle_check=False)


@pytest.mark.slow
@pytest.mark.parametrize("workload", ["vortex257", "sod1025"])
def test_residual_vjp_sampled_at_full_size(workload):
    """The residual VJP at the workloads' full sizes, in the bench's launch
    shape (Hilbert order, default kernels): a cotangent supported on a sample
    of vertices (near the Sod interface, walls, corners, at random) makes
    (dR/dw)^T Rbar depend only on the residual at the sample, which the
    oracle computes there and differentiates by autograd; the GPU's whole
    output field (every row) is compared with it.  The adjoint workload (257^2
    jittered periodic vortex) and the headline mesh (1025^2 walled rotated Sod
    with a smooth perturbation, where the positivity fallback and the mirror
    ghosts enter the VJP)."""
    fdu = _fdu()
    if workload == "vortex257":
        m = make_mesh(257, L=10.0, periodic=True, seed=0)
        w0 = vortex_state(m, beta=5.0, mach=0.5)
        rng = np.random.default_rng(11)
        sample = np.unique(rng.choice(m.nv_real, 300, replace=False))
    else:
        m = make_mesh(1025, L=1.0, periodic=False, seed=0, ghost_layers=4)
        w0 = perturbed_sod(m)
        rng = np.random.default_rng(12)
        a = np.deg2rad(30.0)
        xy = m.xy[:m.nv_real]
        sd = (xy[:, 0] - 0.5) * np.cos(a) + (xy[:, 1] - 0.5) * np.sin(a)
        near = np.nonzero(np.abs(sd) < 0.01)[0]
        wall = np.nonzero((xy[:, 1] < 1e-12) | (xy[:, 1] > 1 - 1e-12) | (xy[:, 0] < 1e-12) | (xy[:, 0] > 1 - 1e-12))[0]
        sample = np.unique(np.concatenate([rng.choice(near, 150, replace=False), rng.choice(m.nv_real, 100, replace=False),
                                           rng.choice(wall, 60, replace=False), [0, 1024, 1025 * 1024, m.nv_real - 1]]))
    prep = fdu.Prep(m, deg=5, reorder=2)
    perm = prep.arrays()["perm"]
    s = fdu.Solver(prep, device=0, weno_eps=ADJ_EPS)
    s.enable_adjoint()
    Rbar = np.zeros((m.nv, 4))
    Rbar[sample] = rng.normal(size=(len(sample), 4))

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a[perm])).cuda()

    wb = s.residual_vjp(dev(w0), dev(Rbar)[:m.nv_real].contiguous()).cpu().numpy()
    o = Oracle(m, deg=5, vertices=sample, weno_eps=ADJ_EPS)
    ref = o.residual_vjp(torch.from_numpy(w0), torch.from_numpy(Rbar[sample])).numpy()
    err = rel_err_per_component(wb, ref[perm])
    print(workload, "sampled residual VJP rel err", err, "sample", len(sample),
          "rows touched", int(np.count_nonzero(np.abs(ref).sum(1))))
    assert err.max() <= TOL


@pytest.mark.parametrize("N,per,G,deg,state", [(16, True, 0, 5, "vortex"), (14, False, 4, 5, "sod")])
def test_step_vjp_with_given_stages_equals_step_vjp(N, per, G, deg, state):
    """fdu_rk_step_vjp_stages, given the stage states of the forward stages at
    the same dt, equals fdu_rk_step_vjp (which recomputes them) bit for bit;
    aliased stage states are refused."""
    fdu = _fdu()
    c = AdjCase(N, per, G, deg, state)
    dt = 0.5 * c.o.cfl_dt(torch.from_numpy(c.w0), 0.3)
    rng = np.random.default_rng(3)
    ybar = c.dev(np.concatenate([rng.normal(size=(c.m.nv_real, 4)), np.zeros((c.m.ng, 4))]))
    wn = c.dev(c.w0)
    out1 = torch.empty_like(wn)
    c.s.rk_step_vjp(wn.clone(), ybar, out1, torch.empty(4 * c.m.nv, 4, dtype=torch.float64, device="cuda"), dt)
    dt_dev = torch.full((1,), dt, dtype=torch.float64, device="cuda")
    w0, w1, w2 = wn.clone(), torch.empty_like(wn), torch.empty_like(wn)
    c.s.rk_stage(0, w0, w0, w1, dt_dev)
    c.s.rk_stage(1, w0, w1, w2, dt_dev)
    out2 = torch.empty_like(wn)
    scratch2 = torch.empty(2 * c.m.nv, 4, dtype=torch.float64, device="cuda")
    c.s.rk_step_vjp_stages(w0, w1, w2, ybar, out2, scratch2, dt)
    assert torch.equal(out1, out2)
    with pytest.raises(fdu.FduError, match="INVALID_ARG"):
        c.s.rk_step_vjp_stages(w0, w1, w1, ybar, out2, scratch2, dt)
    with pytest.raises(fdu.FduError, match="INVALID_ARG"):
        c.s.rk_step_vjp_stages(w0, w1, w2, ybar, w1, scratch2, dt)
