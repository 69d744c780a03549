"""Seeded synthetic workloads: triangulated 2D meshes and initial flow states.

This module is the only code shared by the oracle and the GPU path.  It holds
none of the scheme's arithmetic (no stencils, no interpolation, no fluxes, no
least squares): it only produces the inputs the paper's test problems are posed
on (Sec. 3) as plain arrays.

Meshes (stand-ins for the paper's diagonalized structured meshes, Sec. 3.1, and
its general triangulations, Sec. 2.2.3 and 3.1):
  * an N x N lattice of vertices, each quad split along one diagonal;
  * the diagonal is either always the main one ("uniform", the paper's regular
    diagonalized mesh) or drawn from a seeded bit per quad ("random");
  * vertices are moved by a seeded uniform jitter of up to +-jitter*h per
    coordinate (all vertices when periodic, interior ones otherwise).
RNG contract: ``numpy.random.default_rng(seed)`` draws the jitter ``[N*N, 2]``
first, then the diagonal bits ``[nq, nq]`` (nq = N periodic, N-1 otherwise).

Non-periodic meshes may carry a mirror ghost layer ``ghost_layers`` deep: ghost
vertex positions and ghost triangles are the mirror images of the interior ones
across the walls x=0, x=L, y=0, y=L.  Each ghost records its source vertex and
which momentum components a reflecting wall negates (``ghost_refl`` bit 0: m_x,
bit 1: m_y); filling ghost states from those is the solver's job.  Bit 2 marks a
Dirichlet ghost: its state is a given boundary value (an array the caller
passes beside the mesh), not a copy of its source.

Channel meshes (``make_channel_mesh``) are periodic in y only (``periodic ==
"y"``), with walls at x0 and x1 and mirror ghosts across those two walls.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4  # ratio of specific heats used throughout the paper (Sec. 2.1)


@dataclass
class Mesh:
    xy: np.ndarray          # [nv_total, 2] float64 vertex coordinates
    nv_real: int            # vertices [0, nv_real) are real, the rest ghosts
    tri: np.ndarray         # [T, 3] int32 counter-clockwise triangles
    edges: np.ndarray       # [E, 2] int32, a < b, lexicographic order
    periodic: object        # True (both directions), False, or "y" (y only)
    box: tuple              # (Lx, Ly) domain size
    h: float                # nominal lattice spacing
    N: int
    ghost_src: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    ghost_refl: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int8))
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return self.xy.shape[0]

    @property
    def ne(self) -> int:
        return self.edges.shape[0]

    @property
    def ng(self) -> int:
        return self.nv - self.nv_real


def _quad_tris(v00, v10, v01, v11, bit):
    """Two CCW triangles per quad; bit 1 splits along v00-v11, bit 0 along v10-v01."""
    t_main = np.stack([np.stack([v00, v10, v11], -1), np.stack([v00, v11, v01], -1)], 1)
    t_anti = np.stack([np.stack([v00, v10, v01], -1), np.stack([v10, v11, v01], -1)], 1)
    t = np.where(bit[:, None, None] == 1, t_main, t_anti)
    return t.reshape(-1, 3)


def _edges_from_tris(tri: np.ndarray) -> np.ndarray:
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], 0)
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def make_mesh(N: int, L: float = 1.0, periodic: bool = True, jitter: float = 0.15,
              seed: int = 0, diag: str = "random", ghost_layers: int = 0,
              reflect_x: bool = False, reflect_y: bool = True) -> Mesh:
    """Jittered triangulated N x N lattice on [0, L]^2.

    periodic: x_i = i L / N, N*N unique vertices, 2 N^2 triangles, 3 N^2 edges.
    non-periodic: x_i = i L / (N-1), walls at 0 and L, optional mirror ghosts.
    reflect_x / reflect_y: whether the walls normal to x / y reflect momentum
    (recorded in ``ghost_refl``; a non-reflecting wall is a plain copy).
    """
    if N < 3:
        raise ValueError("N must be >= 3")
    if diag not in ("random", "uniform"):
        raise ValueError("diag must be 'random' or 'uniform'")
    rng = np.random.default_rng(seed)
    h = L / N if periodic else L / (N - 1)
    jit = rng.uniform(-jitter * h, jitter * h, size=(N * N, 2)) if jitter > 0 else np.zeros((N * N, 2))
    nq = N if periodic else N - 1
    if diag == "random":
        bits = rng.integers(0, 2, size=(nq, nq)).astype(np.int8)
    else:
        bits = np.ones((nq, nq), np.int8)

    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    base = np.stack([ii * h, jj * h], -1).reshape(-1, 2).astype(np.float64)
    if periodic:
        if ghost_layers:
            raise ValueError("periodic meshes take no ghost layer")
        xy = base + jit
        vid = (ii * N + jj)
        qi, qj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        qi, qj = qi.ravel(), qj.ravel()
        ip, jp = (qi + 1) % N, (qj + 1) % N
        tri = _quad_tris(vid[qi, qj], vid[ip, qj], vid[qi, jp], vid[ip, jp], bits[qi, qj])
        mesh = Mesh(xy=xy, nv_real=N * N, tri=tri.astype(np.int32), edges=_edges_from_tris(tri),
                    periodic=True, box=(L, L), h=h, N=N)
        mesh.meta = dict(N=N, L=L, periodic=True, jitter=jitter, seed=seed, diag=diag)
        return mesh

    interior = ((ii > 0) & (ii < N - 1) & (jj > 0) & (jj < N - 1)).reshape(-1)
    xy_real = base.copy()
    xy_real[interior] += jit[interior]
    G = int(ghost_layers)
    if G > N - 1:
        raise ValueError("ghost_layers must be <= N-1")
    M = N + 2 * G
    # extended lattice index e in [0, M) <-> lattice index e - G in [-G, N-1+G]
    lat = np.arange(M) - G
    src = np.where(lat < 0, -lat, np.where(lat > N - 1, 2 * (N - 1) - lat, lat))
    outside = (lat < 0) | (lat > N - 1)
    EI, EJ = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    li, lj = lat[EI], lat[EJ]
    real = (~outside[EI]) & (~outside[EJ])
    ids = np.full((M, M), -1, np.int64)
    ids[real] = li[real] * N + lj[real]
    ng = int((~real).sum())
    ids[~real] = N * N + np.arange(ng)
    # ghost positions: mirror the source vertex across the crossed walls
    gi, gj = li[~real], lj[~real]
    si, sj = src[EI][~real], src[EJ][~real]
    sid = si * N + sj
    gx = xy_real[sid, 0].copy()
    gy = xy_real[sid, 1].copy()
    gx = np.where(gi < 0, -gx, np.where(gi > N - 1, 2 * L - gx, gx))
    gy = np.where(gj < 0, -gy, np.where(gj > N - 1, 2 * L - gy, gy))
    xy = np.concatenate([xy_real, np.stack([gx, gy], -1)], 0)
    crossed_x = (gi < 0) | (gi > N - 1)
    crossed_y = (gj < 0) | (gj > N - 1)
    refl = (crossed_x & reflect_x).astype(np.int8) | ((crossed_y & reflect_y).astype(np.int8) << 1)
    # quads of the extended lattice mirror the real quads; each crossed wall flips the diagonal
    qlat = np.arange(M - 1) - G
    qsrc = np.where(qlat < 0, -qlat - 1, np.where(qlat > N - 2, 2 * N - 3 - qlat, qlat))
    qout = ((qlat < 0) | (qlat > N - 2)).astype(np.int8)
    QI, QJ = np.meshgrid(np.arange(M - 1), np.arange(M - 1), indexing="ij")
    QI, QJ = QI.ravel(), QJ.ravel()
    qbit = bits[qsrc[QI], qsrc[QJ]] ^ ((qout[QI] + qout[QJ]) & 1).astype(np.int8)
    tri = _quad_tris(ids[QI, QJ], ids[QI + 1, QJ], ids[QI, QJ + 1], ids[QI + 1, QJ + 1], qbit)
    mesh = Mesh(xy=xy, nv_real=N * N, tri=tri.astype(np.int32), edges=_edges_from_tris(tri),
                periodic=False, box=(L, L), h=h, N=N,
                ghost_src=sid.astype(np.int32), ghost_refl=refl)
    mesh.meta = dict(N=N, L=L, periodic=False, jitter=jitter, seed=seed, diag=diag,
                     ghost_layers=G, reflect_x=reflect_x, reflect_y=reflect_y)
    return mesh


def make_channel_mesh(Nx: int, Ny: int, x0: float, x1: float, y0: float, y1: float, jitter: float = 0.0,
                      seed: int = 0, diag: str = "uniform", ghost_layers: int = 4, wall: str = "dirichlet") -> Mesh:
    """Jittered triangulated lattice on [x0, x1] x [y0, y1), periodic in y.

    x_i = x0 + i (x1 - x0) / (Nx - 1), i < Nx (walls at x0 and x1);
    y_j = y0 + j (y1 - y0) / Ny, j < Ny (periodic).  Vertices off the two walls
    are jittered (RNG: jitter [Nx*Ny, 2], then diagonal bits [Nx-1, Ny]).  A
    mirror ghost layer ``ghost_layers`` deep lies across each wall; ``wall``:
    "dirichlet" (ghost_refl bit 2: given boundary states), "reflect" (bit 0) or
    "copy" (0).  Vertex id = i Ny + j.
    """
    if Nx < 3 or Ny < 3:
        raise ValueError("Nx, Ny must be >= 3")
    if diag not in ("random", "uniform") or wall not in ("dirichlet", "reflect", "copy"):
        raise ValueError("diag: random|uniform, wall: dirichlet|reflect|copy")
    rng = np.random.default_rng(seed)
    hx, hy = (x1 - x0) / (Nx - 1), (y1 - y0) / Ny
    jit = (rng.uniform(-jitter, jitter, size=(Nx * Ny, 2)) * np.array([hx, hy])) if jitter > 0 \
        else np.zeros((Nx * Ny, 2))
    bits = rng.integers(0, 2, size=(Nx - 1, Ny)).astype(np.int8) if diag == "random" \
        else np.ones((Nx - 1, Ny), np.int8)
    ii, jj = np.meshgrid(np.arange(Nx), np.arange(Ny), indexing="ij")
    xy_real = np.stack([x0 + ii * hx, y0 + jj * hy], -1).reshape(-1, 2).astype(np.float64)
    inner = ((ii > 0) & (ii < Nx - 1)).reshape(-1)
    xy_real[inner] += jit[inner]
    G = int(ghost_layers)
    if G > Nx - 1:
        raise ValueError("ghost_layers must be <= Nx-1")
    M = Nx + 2 * G
    lat = np.arange(M) - G                                     # extended x index in [-G, Nx-1+G]
    src = np.where(lat < 0, -lat, np.where(lat > Nx - 1, 2 * (Nx - 1) - lat, lat))
    outside = (lat < 0) | (lat > Nx - 1)
    EI, EJ = np.meshgrid(np.arange(M), np.arange(Ny), indexing="ij")
    li = lat[EI]
    real = ~outside[EI]
    ids = np.full((M, Ny), -1, np.int64)
    ids[real] = li[real] * Ny + EJ[real]
    ng = int((~real).sum())
    ids[~real] = Nx * Ny + np.arange(ng)
    gi, gj = li[~real], EJ[~real]
    sid = src[EI][~real] * Ny + gj
    gx = xy_real[sid, 0].copy()
    gx = np.where(gi < 0, 2 * x0 - gx, 2 * x1 - gx)
    xy = np.concatenate([xy_real, np.stack([gx, xy_real[sid, 1]], -1)], 0)
    flag = {"dirichlet": 4, "reflect": 1, "copy": 0}[wall]
    refl = np.full(ng, flag, np.int8)
    qlat = np.arange(M - 1) - G
    qsrc = np.where(qlat < 0, -qlat - 1, np.where(qlat > Nx - 2, 2 * Nx - 3 - qlat, qlat))
    qout = ((qlat < 0) | (qlat > Nx - 2)).astype(np.int8)
    QI, QJ = np.meshgrid(np.arange(M - 1), np.arange(Ny), indexing="ij")
    QI, QJ = QI.ravel(), QJ.ravel()
    qbit = bits[qsrc[QI], QJ] ^ qout[QI]
    jp = (QJ + 1) % Ny
    tri = _quad_tris(ids[QI, QJ], ids[QI + 1, QJ], ids[QI, jp], ids[QI + 1, jp], qbit)
    mesh = Mesh(xy=xy, nv_real=Nx * Ny, tri=tri.astype(np.int32), edges=_edges_from_tris(tri),
                periodic="y", box=(x1 - x0, y1 - y0), h=min(hx, hy), N=Nx,
                ghost_src=sid.astype(np.int32), ghost_refl=refl)
    mesh.meta = dict(Nx=Nx, Ny=Ny, x0=x0, x1=x1, y0=y0, y1=y1, jitter=jitter, seed=seed, diag=diag,
                     ghost_layers=G, wall=wall)
    return mesh


# ----------------------------------------------------------------------------
# Initial states (conservative variables w = [rho, rho u, rho v, rho E], Sec. 2.1)
# ----------------------------------------------------------------------------

def primitive_to_conservative(rho, u, v, p, gamma: float = GAMMA) -> np.ndarray:
    """w from (rho, u, v, p) with E = e + (u^2+v^2)/2 and p = (gamma-1) rho e (Sec. 2.1)."""
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)], -1)


def _wrap(d, L):
    return d - L * np.round(d / L)


def _wrap_mesh(mesh, d):
    """Displacements [..., 2] to their nearest periodic image on the mesh's box."""
    d = np.array(d, dtype=np.float64, copy=True)
    if mesh.periodic is True:
        d[..., 0] = _wrap(d[..., 0], mesh.box[0])
    if mesh.periodic is True or mesh.periodic == "y":
        d[..., 1] = _wrap(d[..., 1], mesh.box[1])
    return d


def vortex_primitive(xy: np.ndarray, t=0.0, beta: float = 5.0, mach: float = 0.5,
                     angle_deg: float = 45.0, center=(5.0, 5.0), box=(10.0, 10.0),
                     periodic: bool = True, gamma: float = GAMMA):
    """Isentropic vortex of Sec. 3.1 convected by a free stream of Mach ``mach``
    (rho_inf = p_inf = 1, so |U_inf| = mach*sqrt(gamma)) at ``angle_deg``.

    ``t`` may be complex (complex-step differentiation in time); the minimum
    image is taken on its real part.
    """
    a = np.deg2rad(angle_deg)
    U = mach * np.sqrt(gamma) * np.array([np.cos(a), np.sin(a)])
    cx = center[0] + U[0] * t
    cy = center[1] + U[1] * t
    dx = xy[:, 0] - cx
    dy = xy[:, 1] - cy
    if periodic:
        dx = dx - box[0] * np.round(np.real(dx) / box[0])
        dy = dy - box[1] * np.round(np.real(dy) / box[1])
    r2 = dx * dx + dy * dy
    rho = (1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)) ** (1.0 / (gamma - 1.0))
    amp = beta / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    u = U[0] - amp * dy
    v = U[1] + amp * dx
    p = rho ** gamma
    return rho, u, v, p


def vortex_state(mesh_or_xy, t: float = 0.0, **kw) -> np.ndarray:
    xy, kw = _xy_and_box(mesh_or_xy, kw)
    return primitive_to_conservative(*vortex_primitive(xy, t, **kw), gamma=kw.get("gamma", GAMMA))


def vortex_state_dt(mesh_or_xy, t: float = 0.0, step: float = 1e-30, **kw) -> np.ndarray:
    """Exact d w / d t of the convected vortex, by complex-step differentiation."""
    xy, kw = _xy_and_box(mesh_or_xy, kw)
    g = kw.get("gamma", GAMMA)
    rho, u, v, p = vortex_primitive(xy, t + 1j * step, **kw)
    w = primitive_to_conservative(rho, u, v, p, gamma=g)
    return np.imag(w) / step


def _xy_and_box(mesh_or_xy, kw):
    kw = dict(kw)
    if isinstance(mesh_or_xy, Mesh):
        kw.setdefault("box", mesh_or_xy.box)
        kw.setdefault("periodic", mesh_or_xy.periodic)
        if "center" not in kw:
            kw["center"] = (0.5 * mesh_or_xy.box[0], 0.5 * mesh_or_xy.box[1])
        return mesh_or_xy.xy, kw
    return mesh_or_xy, kw


def sod_state(mesh_or_xy, angle_deg: float = 30.0, center=(0.5, 0.5),
              left=(1.0, 0.0, 0.0, 1.0), right=(0.125, 0.0, 0.0, 0.1),
              gamma: float = GAMMA) -> np.ndarray:
    """Planar Sod data with the interface through ``center`` and normal at
    ``angle_deg`` from +x: ``left`` where (x - c).n < 0, ``right`` otherwise."""
    xy = mesh_or_xy.xy if isinstance(mesh_or_xy, Mesh) else mesh_or_xy
    a = np.deg2rad(angle_deg)
    s = (xy[:, 0] - center[0]) * np.cos(a) + (xy[:, 1] - center[1]) * np.sin(a)
    lt = s < 0
    prim = [np.where(lt, left[k], right[k]) for k in range(4)]
    return primitive_to_conservative(*prim, gamma=gamma)


def square_sod_state(mesh_or_xy, half: float = 0.25, center=None,
                     inside=(1.0, 0.0, 0.0, 1.0), outside=(0.125, 0.0, 0.0, 0.1),
                     gamma: float = GAMMA) -> np.ndarray:
    """Two-dimensional shock tube of Sec. 3.2: ``inside`` in the square
    |x - cx| < half, |y - cy| < half, ``outside`` elsewhere.  The paper's domain
    is the periodic box [-1, 1]^2 with the square at its centre; on a periodic
    mesh of [0, 2]^2 the default centre is the box centre, which is the same
    problem shifted by (1, 1)."""
    if isinstance(mesh_or_xy, Mesh):
        xy = mesh_or_xy.xy
        if center is None:
            center = (0.5 * mesh_or_xy.box[0], 0.5 * mesh_or_xy.box[1])
    else:
        xy = mesh_or_xy
        if center is None:
            raise ValueError("pass center with bare coordinates")
    sq = (np.abs(xy[:, 0] - center[0]) < half) & (np.abs(xy[:, 1] - center[1]) < half)
    prim = [np.where(sq, inside[k], outside[k]) for k in range(4)]
    return primitive_to_conservative(*prim, gamma=gamma)


def normal_shock_states(mach: float = 1.2, gamma: float = GAMMA):
    """Primitive (rho, u, v, p) on both sides of a stationary normal shock at x = 0
    with the flow in -x: upstream (x > 0) rho = 1, p = 1/gamma (sound speed 1),
    u = -mach; downstream from the Rankine-Hugoniot relations."""
    M2 = mach * mach
    r = (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)          # density ratio
    pr = 1.0 + 2.0 * gamma / (gamma + 1.0) * (M2 - 1.0)            # pressure ratio
    up = (1.0, -mach, 0.0, 1.0 / gamma)
    down = (r, -mach / r, 0.0, pr / gamma)
    return up, down


def shock_vortex_state(mesh, mach: float = 1.2, mv: float = 1.0, center=(4.0, 0.0), gamma: float = GAMMA):
    """Shock-vortex interaction (Sec. 3.3): a stationary Mach-``mach`` normal shock
    at x = 0 (flow in -x, upstream at x > 0) and an isentropic vortex of strength
    ``mv`` centred upstream at ``center``:
      rho = (1 - (gamma-1)/2 mv^2 exp(1 - r^2))^(1/(gamma-1)),  p = rho^gamma / gamma,
      (du, dv) = mv exp((1 - r^2)/2) (-(y - yc), x - xc),
    superposed on the upstream state (the exponent's factor reads (gamma-1)).
    Returns (w [nv, 4], ghost_state [ng, 4]): the Dirichlet ghosts left of x = 0
    hold the downstream state, those right of it the upstream state."""
    up, down = normal_shock_states(mach, gamma)
    xy = mesh.xy
    dx, dy = xy[:, 0] - center[0], xy[:, 1] - center[1]
    if mesh.periodic == "y":
        dy = _wrap(dy, mesh.box[1])
    r2 = dx * dx + dy * dy
    rho_v = (1.0 - 0.5 * (gamma - 1.0) * mv * mv * np.exp(1.0 - r2)) ** (1.0 / (gamma - 1.0))
    amp = mv * np.exp(0.5 * (1.0 - r2))
    upstream = xy[:, 0] > 0.0
    rho = np.where(upstream, up[0] * rho_v, down[0])
    u = np.where(upstream, up[1] - amp * dy, down[1])
    v = np.where(upstream, up[2] + amp * dx, down[2])
    p = np.where(upstream, rho_v ** gamma / gamma, down[3])
    w = primitive_to_conservative(rho, u, v, p, gamma=gamma)
    gx = xy[mesh.nv_real:, 0]
    gs = np.where((gx > 0.0)[:, None], primitive_to_conservative(*[np.array(q) for q in up], gamma=gamma)[None, :],
                  primitive_to_conservative(*[np.array(q) for q in down], gamma=gamma)[None, :])
    return w, np.ascontiguousarray(gs)


def batch_specs(n: int = 64, n_min: int = 65, n_max: int = 513, seed: int = 42,
                beta_range=(2.0, 6.0), mach_range=(0.3, 0.8), mesh_seed0: int = 1000):
    """Instance table of the batched vortex workload: N_i ~ U{n_min..n_max},
    mesh seed 1000+i, strength ~ U[2,6], free-stream Mach ~ U[0.3,0.8]."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_min, n_max + 1, size=n)
    betas = rng.uniform(*beta_range, size=n)
    machs = rng.uniform(*mach_range, size=n)
    return [dict(N=int(Ns[i]), seed=mesh_seed0 + i, beta=float(betas[i]), mach=float(machs[i]))
            for i in range(n)]


def vertex_areas(mesh) -> np.ndarray:
    """Median-dual-like vertex areas: one third of the areas of the triangles
    incident to each vertex ([nv] float64; ghost triangles count for their
    vertices too, callers take the real rows)."""
    t = mesh.tri.astype(np.int64)
    p0 = mesh.xy[t[:, 0]]
    d1 = mesh.xy[t[:, 1]] - p0
    d2 = mesh.xy[t[:, 2]] - p0
    if mesh.periodic:
        d1, d2 = _wrap_mesh(mesh, d1), _wrap_mesh(mesh, d2)
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    A = np.zeros(mesh.nv)
    for k in range(3):
        np.add.at(A, t[:, k], area / 3.0)
    return A
