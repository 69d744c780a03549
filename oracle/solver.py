"""The oracle's residual, boundary treatment, time step and SSP-RK3 (FP64 CPU).

Per residual evaluation, in the paper's order (abstract; Sec. 2.2, 2.3):
  0. ghost fill (walls only; reading below);
  1. for every edge a divergence stencil uses: gather the six states of its 1D
     stencil, project them on the characteristic variables of the edge
     direction, interpolate left and right midpoint states with NU-WENO5 along
     the curve-length coordinate (the right state on the mirrored stencil),
     return to conservative variables and take the numerical flux r_k along
     the edge direction;
  2. for every vertex O: div = sum_j [wf_j (f_j - f_O) + wg_j (g_j - g_O)]
     + sum_k we_k (r_k - n_k . F_O)  (the differenced right-hand side R of
     Sec. 2.2.1 times the weight row), and the residual dw/dt = -div.
SSP-RK3 of Shu and Osher (the third-order TVD Runge-Kutta scheme Sec. 3 cites):
  w1 = w + dt R(w);  w2 = 3/4 w + 1/4 (w1 + dt R(w1));  w' = 1/3 w + 2/3 (w2 + dt R(w2)).
Addition (not in the paper; ``positivity=False`` turns it off): where an
interpolated midpoint state has rho <= 0 or p <= 0 (the WENO quadratics can
overshoot on stencils that cross a discontinuity twice), that side of the edge
falls back to its end vertex state (w_L = w_L1, w_R = w_R1).
Ablation switches (the comparisons of Sec. 2.3.1-2.3.2, defaults = the paper's
scheme): ``interpolation="conservative"`` interpolates the conservative
variables directly instead of the characteristic ones; ``weno="uniform"`` uses
standard WENO5 (equally spaced nodes) whatever the spacing along the stencil.
Dirichlet boundaries (the paper's inflow/outflow condition): ghosts flagged
Dirichlet (bit 2 of ghost_refl) take given states (``ghost_state``).
Readings: dt = CFL * min_v h_v / (|u_v| + c_v) over real vertices, h_v the
shortest edge at v (the paper names the CFL number but no formula).  Walls (not
in the paper, which has periodic and Dirichlet boundaries only): ghost states
copy their mirror source, with the momentum components normal to a reflecting
wall negated (parity unpinned).
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

from . import euler
from .geometry import arc_coordinates, min_image, neighbour_table, select_1d_stencils
from .lsq import Topology, artificial_edges, ls_weights
from .nuweno import NUWeno5, WENO_EPS, WENO_POWER, uniform_weno5


class Oracle:
    def __init__(self, mesh, deg: int = 5, level=None, vertices=None, gamma: float = euler.GAMMA,
                 weno_eps: float = WENO_EPS, weno_power: int = WENO_POWER,
                 entropy_frac: float = 0.1, riemann: str = "roe", positivity: bool = True,
                 interpolation: str = "characteristic", weno: str = "nonuniform", artificial: bool = False,
                 ghost_state=None):
        if interpolation not in ("characteristic", "conservative") or weno not in ("nonuniform", "uniform"):
            raise ValueError("interpolation: characteristic|conservative, weno: nonuniform|uniform")
        self.interpolation = interpolation
        self.ghost_state = None if ghost_state is None else torch.as_tensor(np.asarray(ghost_state, np.float64))
        self.mesh = mesh
        self.positivity = positivity
        self.gamma = gamma
        self.entropy_frac = entropy_frac
        self.riemann = riemann
        self.deg = deg
        self.all_vertices = vertices is None
        self.vertices = np.arange(mesh.nv_real) if vertices is None else np.asarray(vertices, np.int64)
        if np.any(self.vertices >= mesh.nv_real):
            raise ValueError("residuals are defined on real vertices only")
        self.topo = Topology(mesh)
        # artificial edges (all real vertices decide, so a subset of vertices sees
        # the same edge ids as the whole mesh); the edge list becomes mesh + them
        self.artificial = (artificial_edges(self.topo, np.arange(mesh.nv_real), deg, level) if artificial
                           else np.zeros((0, 2), np.int64))
        self.all_edges = np.concatenate([mesh.edges.astype(np.int64), self.artificial], 0)
        mesh_e = replace(mesh, edges=self.all_edges)
        self.W = ls_weights(mesh_e, self.topo, self.vertices, deg, level, self.artificial if artificial else None)
        self.edges = np.unique(self.W["ecol"])                      # edges whose flux is needed
        nbtab, _ = neighbour_table(mesh)                             # continuation along the mesh's edges
        self.sten6 = select_1d_stencils(mesh_e, self.edges, nbtab)
        self.s, self.dir = arc_coordinates(mesh, self.sten6)
        if weno == "uniform":        # standard WENO5 whatever the node spacing (Sec. 2.3.2 comparison)
            self.wenoL = uniform_weno5(len(self.edges), weno_eps, weno_power)
            self.wenoR = uniform_weno5(len(self.edges), weno_eps, weno_power)
        else:
            self.wenoL = NUWeno5(self.s[:, 0:5], weno_eps, weno_power)
            self.wenoR = NUWeno5(-self.s[:, [5, 4, 3, 2, 1]], weno_eps, weno_power)
        W = self.W
        nsel = len(self.vertices)
        self.v_row = torch.from_numpy(np.repeat(np.arange(nsel), np.diff(W["vptr"])))
        self.e_row = torch.from_numpy(np.repeat(np.arange(nsel), np.diff(W["eptr"])))
        self.v_col = torch.from_numpy(W["vcol"])
        self.e_loc = torch.from_numpy(np.searchsorted(self.edges, W["ecol"]))
        self.wf = torch.from_numpy(W["wf"])
        self.wg = torch.from_numpy(W["wg"])
        self.we = torch.from_numpy(W["we"])
        self.n_e = torch.from_numpy(self.dir)                       # [ne_needed, 2]
        self.vt = torch.from_numpy(self.vertices)
        self.sten_t = torch.from_numpy(self.sten6)

    # ---------------------------------------------------------------- boundary
    def fill_ghosts(self, w: torch.Tensor) -> torch.Tensor:
        m = self.mesh
        if m.ng == 0:
            return w
        src = torch.from_numpy(m.ghost_src.astype(np.int64))
        refl = torch.from_numpy(m.ghost_refl.astype(np.int64))
        g = w[src]
        sx = 1.0 - 2.0 * (refl & 1).to(w.dtype)
        sy = 1.0 - 2.0 * ((refl >> 1) & 1).to(w.dtype)
        g = torch.stack([g[:, 0], sx * g[:, 1], sy * g[:, 2], g[:, 3]], -1)
        dirichlet = torch.from_numpy((m.ghost_refl & 4) != 0)
        if bool(dirichlet.any()):                   # Dirichlet ghosts take the given states
            if self.ghost_state is None:
                raise ValueError("the mesh has Dirichlet ghosts: pass ghost_state")
            g = torch.where(dirichlet[:, None], self.ghost_state.to(w.dtype), g)
        return torch.cat([w[:m.nv_real], g], 0)

    # ---------------------------------------------------------------- edges
    def edge_states(self, w: torch.Tensor):
        """Interpolated (w_L, w_R) at the midpoints of the needed edges."""
        W6 = w[self.sten_t]                                         # [ne,6,4]
        if self.interpolation == "conservative":                     # ablation: no projection
            wL = self.wenoL(W6[:, 0:5])
            wR = self.wenoR(W6[:, [5, 4, 3, 2, 1]])
        else:
            R, L = euler.char_basis(W6[:, 2], W6[:, 3], self.n_e, self.gamma)
            C6 = torch.einsum("eij,esj->esi", L, W6)                 # characteristic values
            cL = self.wenoL(C6[:, 0:5])
            cR = self.wenoR(C6[:, [5, 4, 3, 2, 1]])
            wL = torch.einsum("eij,ej->ei", R, cL)
            wR = torch.einsum("eij,ej->ei", R, cR)
        if self.positivity:
            wL = torch.where(self._physical(wL)[:, None], wL, W6[:, 2])
            wR = torch.where(self._physical(wR)[:, None], wR, W6[:, 3])
        return wL, wR

    def _physical(self, q):
        rho, _, _, p = euler.primitives(q, self.gamma)
        return (rho > 0) & (p > 0)

    def edge_fluxes(self, w: torch.Tensor) -> torch.Tensor:
        """Numerical flux projections r_k [ne_needed, 4] (edge order: self.edges)."""
        w = self.fill_ghosts(w)
        wL, wR = self.edge_states(w)
        if self.riemann == "roe":
            return euler.roe_flux(wL, wR, self.n_e, self.gamma, self.entropy_frac)
        return euler.rusanov_flux(wL, wR, self.n_e, self.gamma)

    # ---------------------------------------------------------------- residual
    def divergence(self, f: torch.Tensor, g: torch.Tensor, r: torch.Tensor) -> torch.Tensor:
        """Least-squares df/dx + dg/dy at the selected vertices from vertex fluxes
        f, g [nv, m] and edge flux projections r [ne_needed, m] (Sec. 2.2.1)."""
        fO, gO = f[self.vt], g[self.vt]
        tv = self.wf[:, None] * (f[self.v_col] - fO[self.v_row]) + self.wg[:, None] * (g[self.v_col] - gO[self.v_row])
        n = self.n_e[self.e_loc]
        te = self.we[:, None] * (r[self.e_loc] - (n[:, 0:1] * fO[self.e_row] + n[:, 1:2] * gO[self.e_row]))
        div = torch.zeros(len(self.vertices), f.shape[1], dtype=f.dtype)
        return div.index_add(0, self.v_row, tv).index_add(0, self.e_row, te)

    def residual(self, w: torch.Tensor) -> torch.Tensor:
        """dw/dt = -(df/dx + dg/dy) at the selected real vertices [nsel, 4]."""
        w = self.fill_ghosts(w)
        r = self.edge_fluxes(w)
        f, g = euler.fluxes(w, self.gamma)
        return -self.divergence(f, g, r)

    def edge_midpoints(self) -> np.ndarray:
        """Midpoints [ne_needed, 2] of the needed edges (unwrapped from their L1 end)."""
        m = self.mesh
        a = self.sten6[:, 2]
        return m.xy[a] + 0.5 * min_image(m, m.xy[self.sten6[:, 3]] - m.xy[a])

    # ---------------------------------------------------------------- time
    def cfl_dt(self, w: torch.Tensor, cfl: float) -> float:
        m = self.mesh
        d = min_image(m, m.xy[m.edges[:, 1]] - m.xy[m.edges[:, 0]])
        le = np.sqrt((d * d).sum(-1))
        hv = np.full(m.nv, np.inf)
        np.minimum.at(hv, m.edges[:, 0], le)
        np.minimum.at(hv, m.edges[:, 1], le)
        rho, u, v, p = euler.primitives(w[:m.nv_real].detach(), self.gamma)
        c = torch.sqrt(self.gamma * p / rho)
        s = torch.sqrt(u * u + v * v) + c
        return float(cfl * torch.min(torch.from_numpy(hv[:m.nv_real]) / s))

    def _full_residual(self, w):
        if not self.all_vertices:
            raise ValueError("time stepping needs the residual at every real vertex")
        R = self.residual(w)
        return torch.cat([R, torch.zeros(self.mesh.ng, 4, dtype=w.dtype)], 0)

    def rk3_step(self, w: torch.Tensor, dt: float) -> torch.Tensor:
        w1 = w + dt * self._full_residual(w)
        w2 = 0.75 * w + 0.25 * (w1 + dt * self._full_residual(w1))
        return w / 3.0 + 2.0 / 3.0 * (w2 + dt * self._full_residual(w2))

    def rk3_stage(self, k: int, w_n: torch.Tensor, w_prev: torch.Tensor, dt: float) -> torch.Tensor:
        """Stage k (0, 1, 2) of SSP-RK3: a_k w^n + b_k (w_prev + dt R(w_prev))."""
        a, b = [(0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)][k]
        return a * w_n + b * (w_prev + dt * self._full_residual(w_prev))

    # ---------------------------------------------------------------- adjoint
    def residual_vjp(self, w: torch.Tensor, Rbar: torch.Tensor) -> torch.Tensor:
        """(dR/dw)^T Rbar by autograd through the whole residual."""
        x = w.detach().clone().requires_grad_(True)
        R = self.residual(x)
        (g,) = torch.autograd.grad(R, x, Rbar)
        return g
