"""Least-squares flux divergence weights (Sec. 2.2.1) on one- and two-level
divergence stencils (Sec. 2.2.2), for the oracle.

Around vertex O the two flux components are modelled as f = f0 + p(x,y)^T a and
g = g0 + p(x,y)^T b with p = [x, y, x^2, xy, y^2, x^3, ...] (all monomials of
degree 1..deg, in that order).  Each stencil vertex j gives two rows
([p(x_j), 0] and [0, p(x_j)]), each stencil edge k one row
([n_xk p(x_k), n_yk p(x_k)], x_k its midpoint, n_k its unit direction from the
smaller-id end to the larger-id end).  With [a; b] = A^+ R (A^+ by SVD, as the
paper does) the divergence at O is a_1 + b_2 = (r_a1 + r_b2) R, so the weights
are the sum of the two rows of A^+ belonging to a_1 and b_2; they depend only on
the geometry.  Coordinates are scaled by h_O (mean length of the edges at O)
before the SVD, and the weights divided by h_O afterwards.

Stencils:
  one-level  vertices N(O); edges of the triangles incident to O (spokes + ring).
  two-level  union of the one-level stencils of O and of every J in N(O),
             without O itself (18 vertices and 42 edges on a regular mesh).
Short one-level stencils (fewer than deg(deg+3)+4 conditions; the paper only
says "not enough edges").  Default reading: replace it by the two-level one.
With artificial edges (Sec. 2.2.2, figures of the one-level stencils with
dashed edges): O is joined to the far vertex K of the triangle across each of
its ring edges (J_a, J_b) when K is not yet a neighbour of O; those K and the
new edges O-K join O's one-level stencil, and only if that is still short is
the two-level stencil used.  Artificial edges get ids after the mesh's edges,
in lexicographic order of their (smaller, larger) end ids; the neighbour graph
(and so every two-level stencil and every edge's 1D stencil continuation) is
that of the mesh's own edges.
"""
from __future__ import annotations

import numpy as np

from .geometry import min_image


RANK_TOL = 1e-10


def monomial_exponents(deg: int):
    """(i, j) exponent pairs of x^i y^j, degree 1..deg, in the paper's order."""
    out = []
    for d in range(1, deg + 1):
        for j in range(d + 1):
            out.append((d - j, j))
    return out


def conditions_needed(deg: int) -> int:
    """Unknowns of the coupled system for polynomials of degree deg: deg(deg+3)."""
    return deg * (deg + 3)


class Topology:
    """CSR incidence: vertex -> neighbours, vertex -> triangles, triangle -> edges."""

    def __init__(self, mesh):
        self.mesh = mesh
        nv = mesh.nv
        e = mesh.edges.astype(np.int64)
        self.ekey = e[:, 0] * nv + e[:, 1]               # sorted (edges are lexicographic)
        a = np.concatenate([e[:, 0], e[:, 1]])
        b = np.concatenate([e[:, 1], e[:, 0]])
        o = np.lexsort((b, a))
        self.nb_ptr = np.concatenate([[0], np.cumsum(np.bincount(a, minlength=nv))])
        self.nb_col = b[o]
        t = mesh.tri.astype(np.int64)
        tv = t.reshape(-1)
        tt = np.repeat(np.arange(t.shape[0]), 3)
        o = np.lexsort((tt, tv))
        self.vt_ptr = np.concatenate([[0], np.cumsum(np.bincount(tv, minlength=nv))])
        self.vt_col = tt[o]
        pairs = np.stack([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], 1)  # [T,3,2]
        lo = pairs.min(-1)
        hi = pairs.max(-1)
        key = lo * nv + hi
        self.tri_edges = np.searchsorted(self.ekey, key)
        assert np.all(self.ekey[self.tri_edges] == key)

    def nbrs(self, v):
        return self.nb_col[self.nb_ptr[v]:self.nb_ptr[v + 1]]

    def tris(self, v):
        return self.vt_col[self.vt_ptr[v]:self.vt_ptr[v + 1]]

    def one_level(self, O):
        verts = set(int(x) for x in self.nbrs(O))
        edges = set(int(x) for x in self.tri_edges[self.tris(O)].reshape(-1))
        return verts, edges

    def across_vertices(self, O):
        """Far vertex of the triangle on the other side of each ring edge of O
        (ring edge = side of a triangle at O not touching O), when it is not O
        itself or a neighbour of O."""
        t = self.mesh.tri
        nb = set(int(x) for x in self.nbrs(O))
        out = set()
        for tr in self.tris(O):
            a, b = [int(x) for x in t[tr] if x != O]
            other = (set(int(x) for x in self.tris(a)) & set(int(x) for x in self.tris(b))) - {int(tr)}
            for to in other:
                K = [int(x) for x in t[to] if x != a and x != b][0]
                if K != O and K not in nb:
                    out.add(K)
        return out

    def two_level(self, O):
        verts, edges = set(), set()
        for J in [O] + [int(x) for x in self.nbrs(O)]:
            v, e = self.one_level(J)
            verts |= v
            edges |= e
        verts.discard(O)
        return verts, edges


def artificial_edges(topo: Topology, vertices, deg: int, level=None) -> np.ndarray:
    """[n, 2] artificial edges (smaller id first, lexicographic order) that the
    one-level stencils of the given real vertices need."""
    if level is None:
        level = 2 if deg > 3 else 1
    pairs = set()
    if level == 1:
        for O in vertices:
            O = int(O)
            v, e = topo.one_level(O)
            if 2 * len(v) + len(e) < conditions_needed(deg) + 4:
                for K in topo.across_vertices(O):
                    pairs.add((min(O, K), max(O, K)))
    return np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)


def divergence_stencil(topo: Topology, O: int, deg: int, level=None, art=None):
    """Sorted (vertex ids, edge ids) of the divergence stencil of O.  art: the
    artificial edges (array [n, 2], ids topo's edge count + row), or None."""
    if level is None:
        level = 2 if deg > 3 else 1
    if level == 1:
        v, e = topo.one_level(O)
        if 2 * len(v) + len(e) < conditions_needed(deg) + 4 and art is not None and len(art):
            ne = len(topo.ekey)
            for K in topo.across_vertices(O):
                row = np.nonzero((art[:, 0] == min(O, K)) & (art[:, 1] == max(O, K)))[0]
                v.add(K)
                e.add(ne + int(row[0]))
        if 2 * len(v) + len(e) < conditions_needed(deg) + 4:
            v, e = topo.two_level(O)
    else:
        v, e = topo.two_level(O)
    return np.array(sorted(v), dtype=np.int64), np.array(sorted(e), dtype=np.int64)


def _assemble(mesh, O, verts, edges, exps, hO):
    """Least-squares matrices A of Sec. 2.2.1 for a group of vertices O [g] whose
    stencils have equal sizes (verts [g, nV], edges [g, nE]), in coordinates
    scaled by hO [g].  Rows: f/g interleaved per stencil vertex, then one row
    per stencil edge.  Returns [g, 2 nV + nE, 2 M]."""
    M = len(exps)
    xO = mesh.xy[O][:, None, :]
    xv = min_image(mesh, mesh.xy[verts] - xO) / hO[:, None, None]
    ea = mesh.edges[edges, 0].astype(np.int64)
    eb = mesh.edges[edges, 1].astype(np.int64)
    pa = min_image(mesh, mesh.xy[ea] - xO)
    dab = min_image(mesh, mesh.xy[eb] - mesh.xy[ea])
    xe = (pa + 0.5 * dab) / hO[:, None, None]
    ne = dab / np.sqrt((dab * dab).sum(-1))[..., None]
    Pv = np.stack([xv[..., 0] ** i * xv[..., 1] ** j for (i, j) in exps], -1)   # [g, nV, M]
    Pe = np.stack([xe[..., 0] ** i * xe[..., 1] ** j for (i, j) in exps], -1)   # [g, nE, M]
    g, nV, nE = verts.shape[0], verts.shape[1], edges.shape[1]
    A = np.zeros((g, 2 * nV + nE, 2 * M))
    A[:, 0:2 * nV:2, :M] = Pv
    A[:, 1:2 * nV:2, M:] = Pv
    A[:, 2 * nV:, :M] = ne[..., 0:1] * Pe
    A[:, 2 * nV:, M:] = ne[..., 1:2] * Pe
    return A


def mean_incident_length(mesh, topo: Topology, O: int) -> float:
    nb = topo.nbrs(O)
    d = min_image(mesh, mesh.xy[nb] - mesh.xy[O])
    return float(np.sqrt((d * d).sum(-1)).mean())


def ls_weights(mesh, topo: Topology, vertices, deg: int, level=None, art=None):
    """Divergence weights of the given vertices as CSR arrays:
    vptr, vcol, wf, wg (vertex part) and eptr, ecol, we (edge part).
    With artificial edges (art), mesh.edges must list the mesh's edges followed
    by them.

    The weight row is r_a1 + r_b2 of the SVD pseudo-inverse
    A^+ = V diag(1/sigma) U^T (zero for sigma < RANK_TOL sigma_max), divided
    by h_O."""
    exps = monomial_exponents(deg)
    M = len(exps)
    vertices = np.asarray(vertices, dtype=np.int64)
    sten = [divergence_stencil(topo, int(O), deg, level, art) for O in vertices]
    hO = np.array([mean_incident_length(mesh, topo, int(O)) for O in vertices])
    nV = np.array([len(v) for v, _ in sten], dtype=np.int64)
    nE = np.array([len(e) for _, e in sten], dtype=np.int64)
    wv = [None] * len(vertices)
    wev = [None] * len(vertices)
    groups = {}
    for i, key in enumerate(zip(nV.tolist(), nE.tolist())):
        groups.setdefault(key, []).append(i)
    for (a, b), idx in groups.items():
        idx = np.array(idx)
        V = np.stack([sten[i][0] for i in idx])
        E = np.stack([sten[i][1] for i in idx])
        A = _assemble(mesh, vertices[idx], V, E, exps, hO[idx])
        U, S, Vt = np.linalg.svd(A, full_matrices=False)
        # pseudo-inverse: singular values below RANK_TOL * sigma_max count as zero
        # (exactly symmetric stencils, e.g. mirror-ghost corners, are rank deficient)
        Sinv = np.where(S > RANK_TOL * S[:, :1], 1.0 / S, 0.0)
        coef = (Vt[:, :, 0] + Vt[:, :, M + 1]) * Sinv                    # [g, n]
        rho = np.einsum("gk,gmk->gm", coef, U)                           # [g, m]
        # the divergence must still be determined: A^T rho = e_a1 + e_b2
        e = np.zeros(2 * M)
        e[0] = e[M + 1] = 1.0
        resid = np.abs(np.einsum("gmn,gm->gn", A, rho) - e).max(1)
        if np.any(resid > 1e-8):
            bad = vertices[idx][resid > 1e-8]
            raise ValueError(f"divergence not determined by the stencil of vertex {int(bad[0])}")
        rho = rho / hO[idx][:, None]
        for t, i in enumerate(idx):
            wv[i] = rho[t, :2 * a]
            wev[i] = rho[t, 2 * a:]
    vptr = np.concatenate([[0], np.cumsum(nV)]).astype(np.int64)
    eptr = np.concatenate([[0], np.cumsum(nE)]).astype(np.int64)
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if len(xs) else np.zeros(0, dt)
    wvc = cat(wv, np.float64)
    return dict(vptr=vptr, vcol=cat([v for v, _ in sten], np.int64),
                wf=wvc[0::2].copy(), wg=wvc[1::2].copy(),
                eptr=eptr, ecol=cat([e for _, e in sten], np.int64),
                we=cat(wev, np.float64))
