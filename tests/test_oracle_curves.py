"""Accuracy of midpoint interpolation along curves (Sec. 2.3.3): fifth order
when a fixed smooth curve is refined, near first order when a Catmull-Rom
curve stencil is scaled down (the reason the scheme degrades on general
unstructured meshes, Sec. 3.1)."""
import os

import numpy as np
import torch

from oracle.geometry import arc_coordinates
from oracle.nuweno import NUWeno5, uniform_weno5
from paper_2102_12933_amd.inputs import Mesh

HERE = os.path.dirname(__file__)


def _nodes():
    vals = {}
    with open(os.path.join(HERE, "golden", "refining_curve_nodes.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, *r = line.split()
            vals[k] = np.array([float(t) for t in r])
    return vals["x"], vals["y"]


def _order(hs, errs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def test_refining_curve_fifth_order():
    """The quintic through the printed nodes is the curve; each original interval is
    split into k pieces whose interior nodes are moved by up to 30% of the piece
    (seeded), so stencils stay non-uniform as they are refined."""
    X, Y = _nodes()
    poly = np.polyfit(X, Y, 5)
    dpoly = np.polyder(poly)
    f = lambda x: np.sin(x) * np.cos(np.polyval(poly, x))
    gx, gw = np.polynomial.legendre.leggauss(30)

    def arclen(a, b):
        t = 0.5 * (a + b) + 0.5 * (b - a) * gx
        return 0.5 * (b - a) * np.sum(gw * np.sqrt(1 + np.polyval(dpoly, t) ** 2))

    def point_at(s_target, a, b):
        lo, hi = a, b
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if arclen(a, mid) < s_target:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    rng = np.random.default_rng(11)
    hs, nl_err, lin_err, u_err = [], [], [], []
    for lev in range(4, 8):
        k = 2 ** lev
        pieces = []
        for i in range(5):
            t = np.linspace(X[i], X[i + 1], k + 1)[:-1]
            t[1:] += rng.uniform(-0.3, 0.3, k - 1) * (X[i + 1] - X[i]) / k
            pieces.append(t)
        xs = np.concatenate(pieces + [[X[-1]]])
        S = np.concatenate([[0.0], np.cumsum([arclen(xs[i], xs[i + 1]) for i in range(len(xs) - 1)])])
        rows = np.arange(2, len(xs) - 3)
        t = np.array([f(point_at(0.5 * (S[i + 1] - S[i]), xs[i], xs[i + 1])) for i in rows])
        sl = np.stack([S[rows + o] for o in (-2, -1, 0, 1, 2)], 1) - 0.5 * (S[rows] + S[rows + 1])[:, None]
        u = torch.from_numpy(np.stack([f(xs[rows + o]) for o in (-2, -1, 0, 1, 2)], 1))
        w = NUWeno5(sl)
        nl_err.append(np.abs(w(u).numpy() - t).mean())
        lin_err.append(np.abs(w.linear(u).numpy() - t).mean())
        u_err.append(np.abs(uniform_weno5(len(rows))(u).numpy() - t).mean())
        hs.append(S[-1] / (len(xs) - 1))
    assert _order(hs[-2:], lin_err[-2:]) > 4.2, lin_err
    assert _order(hs, nl_err) > 3.5, nl_err
    assert _order(hs, u_err) < 1.5, u_err


def test_scaled_catmull_rom_curve_first_order():
    base = np.array([[-2.3, 0.35], [-1.25, 0.15], [-0.5, 0.0], [0.5, 0.0], [1.55, 0.45], [2.2, 1.35]])
    f = lambda p: np.sin(p[..., 0] + 0.3) * np.cos(p[..., 1] - 0.2)
    scales = 2.0 ** -np.arange(3, 9)
    errs = []
    for sc in scales:
        xy = base * sc + np.array([0.4, -0.7])
        m = Mesh(xy=xy, nv_real=6, tri=np.zeros((0, 3), np.int32), edges=np.zeros((0, 2), np.int32),
                 periodic=False, box=(1.0, 1.0), h=sc, N=0)
        s, _ = arc_coordinates(m, np.arange(6)[None, :])
        u = torch.from_numpy(f(xy[:5])[None, :])
        target = f(0.5 * (xy[2] + xy[3]))
        errs.append(abs(NUWeno5(s[:, :5]).linear(u).item() - target))
    assert abs(_order(scales, errs) - 1.0) < 0.35, errs
