"""Mesh geometry for the oracle: adjacency, minimum-image vectors, the 1D
curvilinear six-point stencil of every edge and its arc-length coordinates.

Paper: Sec. 2.3.1 (through each edge, a chain of connected edges chosen to be
the smoothest available; Catmull-Rom curves that leave the middle edge tangentially; WENO
along the curve-length coordinate).

Readings of what the paper leaves open:
  * stencil choice: L1 = the smaller-id endpoint, R1 = the other.  Each
    continuation vertex is the neighbour that maximises the cosine between the
    new segment and the previous one (cosines within 1e-12 tie; the smaller id
    wins).  Already chosen stencil vertices are excluded.
  * curve: on each side a cubic Hermite curve through (L1, L2, L3) with
    tangents m(L1) = |L2-L1| (L1-R1)/|R1-L1| (the middle-edge direction),
    m(L2) = (L3-L1)/2 (Catmull-Rom), m(L3) = L3-L2; segment lengths by
    16-point Gauss-Legendre quadrature of |H'(u)|.  (parity unpinned: the
    paper fixes neither the tangent magnitudes nor the end condition; only
    straight stencils, where every reading gives the chord lengths, are pinned.)
"""
from __future__ import annotations

import numpy as np

TIE_TOL = 1e-12


def min_image(mesh, d: np.ndarray) -> np.ndarray:
    """Displacement vectors d [..., 2] reduced to the nearest periodic image
    (mesh.periodic: True = both directions, "y" = y only, False = none)."""
    if mesh.periodic is False or mesh.periodic is None:
        return d
    L = np.asarray(mesh.box, dtype=np.float64)
    out = np.array(d, dtype=np.float64, copy=True)
    if mesh.periodic == "y":
        out[..., 1] -= L[1] * np.round(out[..., 1] / L[1])
        return out
    return out - L * np.round(out / L)


def vec(mesh, a, b) -> np.ndarray:
    """Vector from vertex a to vertex b (minimum image when periodic)."""
    return min_image(mesh, mesh.xy[b] - mesh.xy[a])


def neighbour_lists(mesh):
    """Sorted neighbour id arrays per vertex, from the edge list."""
    e = mesh.edges
    nb = [[] for _ in range(mesh.nv)]
    for a, b in e:
        nb[a].append(int(b))
        nb[b].append(int(a))
    return [np.array(sorted(x), dtype=np.int64) for x in nb]


def neighbour_table(mesh):
    """Padded neighbour table [nv, maxdeg] (ascending ids, -1 padding) and degrees."""
    e = mesh.edges.astype(np.int64)
    a = np.concatenate([e[:, 0], e[:, 1]])
    b = np.concatenate([e[:, 1], e[:, 0]])
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    deg = np.bincount(a, minlength=mesh.nv)
    maxdeg = int(deg.max())
    start = np.concatenate([[0], np.cumsum(deg)[:-1]])
    pos = np.arange(a.size) - start[a]
    tab = np.full((mesh.nv, maxdeg), -1, dtype=np.int64)
    tab[a, pos] = b
    return tab, deg


def _continue(mesh, nbtab, cur, prev_dir, exclude):
    """Vectorised continuation step: for each row pick the neighbour q of cur[i]
    maximising cos(q - cur, prev_dir), excluding ids listed in exclude[i]."""
    cand = nbtab[cur]                                   # [n, maxdeg]
    valid = cand >= 0
    for ex in exclude:
        valid &= cand != ex[:, None]
    cq = np.where(valid, cand, 0)
    d = min_image(mesh, mesh.xy[cq] - mesh.xy[cur][:, None, :])
    num = d[..., 0] * prev_dir[:, None, 0] + d[..., 1] * prev_dir[:, None, 1]
    den = np.sqrt((d * d).sum(-1)) * np.sqrt((prev_dir * prev_dir).sum(-1))[:, None]
    den = np.where(valid, den, 1.0)
    cos = np.where(valid, num / den, -np.inf)
    cmax = cos.max(axis=1)
    if not np.all(np.isfinite(cmax)):
        raise ValueError("an edge has no admissible stencil continuation")
    near = valid & (cos >= cmax[:, None] - TIE_TOL)
    ids = np.where(near, cand, np.iinfo(np.int64).max)
    return ids.min(axis=1), cmax


def select_1d_stencils(mesh, edge_ids=None, nbtab=None):
    """Six-point stencils [n, 6] = (L3, L2, L1, R1, R2, R3) for the given edges."""
    if edge_ids is None:
        edge_ids = np.arange(mesh.ne)
    if nbtab is None:
        nbtab, _ = neighbour_table(mesh)
    e = mesh.edges[edge_ids].astype(np.int64)
    L1 = np.minimum(e[:, 0], e[:, 1])
    R1 = np.maximum(e[:, 0], e[:, 1])
    L2, cl2 = _continue(mesh, nbtab, L1, vec(mesh, R1, L1), [R1])
    R2, cr2 = _continue(mesh, nbtab, R1, vec(mesh, L1, R1), [L1])
    L3, cl3 = _continue(mesh, nbtab, L2, vec(mesh, L1, L2), [L1, R1, R2])
    R3, cr3 = _continue(mesh, nbtab, R2, vec(mesh, R1, R2), [R1, L1, L2])
    st = np.stack([L3, L2, L1, R1, R2, R3], axis=1)
    srt = np.sort(st, axis=1)
    if np.any(srt[:, 1:] == srt[:, :-1]):
        raise ValueError("a 1D stencil repeats a vertex")
    return st


def gauss_legendre_01(n: int = 16):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def hermite_length(P0, P1, m0, m1, n: int = 16):
    """Arc length of the cubic Hermite segment H(u), u in [0,1], with end points
    P0, P1 and end tangents m0, m1 (all [k, 2])."""
    u, wq = gauss_legendre_01(n)
    u = u[:, None, None]
    dH = ((6 * u * u - 6 * u) * P0 + (3 * u * u - 4 * u + 1) * m0
          + (-6 * u * u + 6 * u) * P1 + (3 * u * u - 2 * u) * m1)
    speed = np.sqrt((dH * dH).sum(-1))                  # [n, k]
    return (wq[:, None] * speed).sum(0)


def arc_coordinates(mesh, sten6):
    """Curve-length coordinates s [n, 6] of the six stencil points with the
    middle-edge midpoint at 0 (s[2] = -d/2, s[3] = +d/2), and the unit
    middle-edge direction n [n, 2] (from L1 to R1)."""
    L3, L2, L1, R1, R2, R3 = (sten6[:, k] for k in range(6))
    # unwrapped positions relative to L1
    pL1 = np.zeros((sten6.shape[0], 2))
    pR1 = vec(mesh, L1, R1)
    pL2 = vec(mesh, L1, L2)
    pL3 = pL2 + vec(mesh, L2, L3)
    pR2 = pR1 + vec(mesh, R1, R2)
    pR3 = pR2 + vec(mesh, R2, R3)
    d = np.sqrt((pR1 * pR1).sum(-1))
    t = pR1 / d[:, None]

    def side(P1, P2, P3, tangent_dir):
        l12 = np.sqrt(((P2 - P1) ** 2).sum(-1))
        m1 = l12[:, None] * tangent_dir
        m2 = 0.5 * (P3 - P1)
        m3 = P3 - P2
        return hermite_length(P1, P2, m1, m2), hermite_length(P2, P3, m2, m3)

    aL, bL = side(pL1, pL2, pL3, -t)
    aR, bR = side(pR1, pR2, pR3, t)
    s = np.stack([-0.5 * d - aL - bL, -0.5 * d - aL, -0.5 * d,
                  0.5 * d, 0.5 * d + aR, 0.5 * d + aR + bR], axis=1)
    return s, t
