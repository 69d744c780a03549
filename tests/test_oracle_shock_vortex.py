"""Shock-vortex inputs and the boundary pieces they need (CPU): the channel mesh
periodic in y, Dirichlet ghosts, the Rankine-Hugoniot states of the stationary
shock and the isentropic vortex of Sec. 3.3, and prep == oracle on a channel."""
import numpy as np
import pytest
import torch

from oracle import euler
from oracle.geometry import min_image
from oracle.solver import Oracle
from paper_2102_12933_amd.inputs import (GAMMA, make_channel_mesh, normal_shock_states, primitive_to_conservative,
                                         shock_vortex_state)


def test_channel_mesh_counts_and_y_periodicity():
    Nx, Ny, G = 12, 10, 3
    m = make_channel_mesh(Nx, Ny, -3.0, 2.5, -1.0, 1.5, jitter=0.1, seed=4, ghost_layers=G)
    assert m.nv_real == Nx * Ny and m.ng == 2 * G * Ny
    real_edges = np.all(m.edges < m.nv_real, 1).sum()
    assert real_edges == Nx * Ny - Ny + Nx * Ny + (Nx - 1) * Ny   # x-links, y-links (wrapping), diagonals
    assert len(m.tri) == 2 * (Nx - 1 + 2 * G) * Ny
    # y wraps, x does not
    d = min_image(m, np.array([[5.4, 2.4], [-5.4, -2.4]]))
    np.testing.assert_allclose(d, [[5.4, -0.1], [-5.4, 0.1]], atol=1e-12)
    # every edge is short after the minimum image
    e = min_image(m, m.xy[m.edges[:, 1]] - m.xy[m.edges[:, 0]])
    assert np.sqrt((e ** 2).sum(1)).max() < 2.0 * max(5.5 / (Nx - 1), 2.5 / Ny)
    # ghosts mirror across x walls: same y, x reflected
    gx = m.xy[m.nv_real:, 0]
    sx = m.xy[m.ghost_src, 0]
    left = gx < -3.0
    np.testing.assert_allclose(gx[left], -6.0 - sx[left], atol=1e-12)
    np.testing.assert_allclose(gx[~left], 5.0 - sx[~left], atol=1e-12)
    np.testing.assert_allclose(m.xy[m.nv_real:, 1], m.xy[m.ghost_src, 1], atol=1e-12)
    assert np.all(m.ghost_refl == 4)


@pytest.mark.parametrize("mach", [1.2, 2.0, 3.5])
def test_normal_shock_rankine_hugoniot(mach):
    """The downstream state conserves the x-fluxes of mass, momentum and energy
    (Euler fluxes of Sec. 2.1), is subsonic, and has higher entropy."""
    up, down = normal_shock_states(mach)
    wu = torch.from_numpy(primitive_to_conservative(*[np.array([q]) for q in up]))
    wd = torch.from_numpy(primitive_to_conservative(*[np.array([q]) for q in down]))
    fu, _ = euler.fluxes(wu, GAMMA)
    fd, _ = euler.fluxes(wd, GAMMA)
    np.testing.assert_allclose(fd.numpy(), fu.numpy(), rtol=1e-13, atol=1e-13)
    rho, u, _, p = down
    assert abs(u) / np.sqrt(GAMMA * p / rho) < 1.0
    assert p / rho ** GAMMA > up[3] / up[0] ** GAMMA
    # the trivial solution (no jump) is excluded
    assert rho > up[0] * (1 + 0.1 * (mach - 1))


def test_shock_vortex_initial_state_and_ghost_states():
    m = make_channel_mesh(81, 80, -65.0, 15.0, -40.0, 40.0, ghost_layers=4)
    w, gs = shock_vortex_state(m)
    rho, u, v, p = [x.numpy() for x in euler.primitives(torch.from_numpy(w), GAMMA)]
    up, down = normal_shock_states(1.2)
    x, y = m.xy[:, 0], m.xy[:, 1]
    right = x > 0
    np.testing.assert_allclose(p[right], rho[right] ** GAMMA / GAMMA, rtol=1e-13)   # isentropic vortex
    far = right & ((x - 4) ** 2 + y ** 2 > 100)
    np.testing.assert_allclose(rho[far], up[0], rtol=1e-12)
    np.testing.assert_allclose(u[far], up[1], atol=1e-12)
    np.testing.assert_allclose(rho[~right], down[0], rtol=1e-14)
    near = right & ((x - 4) ** 2 + y ** 2 < 4)
    assert rho[near].min() < 0.8                                  # a strong vortex core
    # the vortex velocity is a rotation about its centre: (u - U, v) is normal to (x - xc, y - yc)
    dx, dy = x[right] - 4.0, y[right]
    np.testing.assert_allclose((u[right] - up[1]) * dx + v[right] * dy, 0.0, atol=1e-12)
    # Dirichlet ghosts: downstream state on the left wall, upstream state on the right
    gx = m.xy[m.nv_real:, 0]
    wu = primitive_to_conservative(*[np.array(q) for q in up])
    wd = primitive_to_conservative(*[np.array(q) for q in down])
    np.testing.assert_allclose(gs[gx > 0], np.broadcast_to(wu, gs[gx > 0].shape))
    np.testing.assert_allclose(gs[gx < 0], np.broadcast_to(wd, gs[gx < 0].shape))
    o = Oracle(m, deg=3, ghost_state=gs)
    wf = o.fill_ghosts(torch.from_numpy(w)).numpy()
    np.testing.assert_array_equal(wf[m.nv_real:], gs)


def test_prep_matches_oracle_on_a_channel():
    from paper_2102_12933_amd import fdu
    m = make_channel_mesh(14, 12, -3.0, 3.0, -2.0, 2.0, jitter=0.15, seed=7, diag="random", ghost_layers=4)
    A = fdu.Prep(m, deg=5, reorder=2).arrays()
    o = Oracle(m, deg=5, ghost_state=np.ones((m.ng, 4)))
    perm = A["perm"]
    fe = A["flux_edge"]
    assert np.array_equal(np.sort(fe), o.edges)
    loc = np.searchsorted(o.edges, fe)
    assert np.array_equal(perm[A["sten6"]], o.sten6[loc])
    d = o.s[loc, 3] - o.s[loc, 2]
    geo_o = np.stack([o.s[loc, 0] / d, o.s[loc, 1] / d, o.s[loc, 4] / d, o.s[loc, 5] / d,
                      o.dir[loc, 0], o.dir[loc, 1]], 1)
    np.testing.assert_allclose(A["geo"], geo_o, rtol=0, atol=1e-13)
    W = o.W
    for i in range(A["nv_real"]):
        O = perm[i]
        a0, a1 = A["vptr"][i], A["vptr"][i + 1]
        b0, b1 = W["vptr"][O], W["vptr"][O + 1]
        cols = perm[A["vcol"][a0:a1]]
        srt = np.argsort(cols)
        assert np.array_equal(cols[srt], W["vcol"][b0:b1])
        scale = np.abs(W["wf"][b0:b1]).max()
        assert np.abs(A["wfg"][a0:a1][srt, 0] - W["wf"][b0:b1]).max() <= 1e-12 * scale
