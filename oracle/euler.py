"""2D Euler pieces for the oracle (torch FP64, differentiable).

Sec. 2.1: w = [rho, rho u, rho v, rho E], f = [rho u, rho u^2 + p, rho u v,
(rho E + p) u], g = [rho v, rho v u, rho v^2 + p, (rho E + p) v],
p = (gamma - 1) rho e, E = e + (u^2 + v^2)/2, gamma = 1.4.

The characteristic variables of the edge interpolation (Sec. 2.3.1, Appendix)
and the numerical flux at the edge midpoint use the eigenvectors of the flux
Jacobian projected on the edge direction n:
    A_n = n_x df/dw + n_y dg/dw = R diag(u_n - c, u_n, u_n, u_n + c) R^{-1}.
Readings (the paper names neither the averaging for the characteristic frame
nor the Riemann solver of its scheme; it names Roe's solver for its structured
comparison scheme): the frame is taken at the Roe average of the edge's two end
vertices; the flux is Roe's, with Harten's entropy fix |l| -> (l^2 + d^2)/(2 d)
for |l| < d, d = 0.1 * c_roe, on all four waves.  (parity unpinned beyond the
consistency, symmetry and Roe-property checks of the tests.)
"""
from __future__ import annotations

import torch

GAMMA = 1.4


def primitives(w, gamma=GAMMA):
    rho = w[..., 0]
    u = w[..., 1] / rho
    v = w[..., 2] / rho
    p = (gamma - 1.0) * (w[..., 3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def fluxes(w, gamma=GAMMA):
    """(f, g), each [..., 4]."""
    rho, u, v, p = primitives(w, gamma)
    rE = w[..., 3]
    f = torch.stack([rho * u, rho * u * u + p, rho * u * v, (rE + p) * u], -1)
    g = torch.stack([rho * v, rho * v * u, rho * v * v + p, (rE + p) * v], -1)
    return f, g


def normal_flux(w, n, gamma=GAMMA):
    f, g = fluxes(w, gamma)
    return n[..., 0:1] * f + n[..., 1:2] * g


def roe_average(wl, wr, gamma=GAMMA):
    """Roe-averaged u, v, H, c of two states."""
    rl, ul, vl, pl = primitives(wl, gamma)
    rr, ur, vr, pr = primitives(wr, gamma)
    Hl = (wl[..., 3] + pl) / rl
    Hr = (wr[..., 3] + pr) / rr
    sl, sr = torch.sqrt(rl), torch.sqrt(rr)
    u = (sl * ul + sr * ur) / (sl + sr)
    v = (sl * vl + sr * vr) / (sl + sr)
    H = (sl * Hl + sr * Hr) / (sl + sr)
    c = torch.sqrt((gamma - 1.0) * (H - 0.5 * (u * u + v * v)))
    return u, v, H, c


def right_eigenvectors(u, v, H, c, n):
    """R [..., 4, 4] with columns r1..r4 for waves u_n - c, u_n, u_n (shear), u_n + c."""
    nx, ny = n[..., 0], n[..., 1]
    tx, ty = -ny, nx
    un = u * nx + v * ny
    ut = u * tx + v * ty
    q2 = 0.5 * (u * u + v * v)
    one = torch.ones_like(u)
    zero = torch.zeros_like(u)
    r1 = torch.stack([one, u - c * nx, v - c * ny, H - c * un], -1)
    r2 = torch.stack([one, u, v, q2], -1)
    r3 = torch.stack([zero, tx, ty, ut], -1)
    r4 = torch.stack([one, u + c * nx, v + c * ny, H + c * un], -1)
    return torch.stack([r1, r2, r3, r4], -1)


def eigenvalues(u, v, c, n):
    un = u * n[..., 0] + v * n[..., 1]
    return torch.stack([un - c, un, un, un + c], -1)


def char_basis(wa, wb, n, gamma=GAMMA):
    """(R, L = R^{-1}) at the Roe average of wa, wb in direction n."""
    u, v, H, c = roe_average(wa, wb, gamma)
    R = right_eigenvectors(u, v, H, c, n)
    return R, torch.linalg.inv(R)


def harten(lam, delta):
    a = torch.abs(lam)
    return torch.where(a < delta, (lam * lam + delta * delta) / (2.0 * delta), a)


def roe_flux(wl, wr, n, gamma=GAMMA, delta_frac=0.1):
    """Roe flux along n: (F_n(wl) + F_n(wr))/2 - R |Lambda| R^{-1} (wr - wl) / 2."""
    u, v, H, c = roe_average(wl, wr, gamma)
    R = right_eigenvectors(u, v, H, c, n)
    L = torch.linalg.inv(R)
    lam = harten(eigenvalues(u, v, c, n), (delta_frac * c).unsqueeze(-1))
    alpha = (L @ (wr - wl).unsqueeze(-1)).squeeze(-1)
    diss = (R @ (lam * alpha).unsqueeze(-1)).squeeze(-1)
    return 0.5 * (normal_flux(wl, n, gamma) + normal_flux(wr, n, gamma)) - 0.5 * diss


def rusanov_flux(wl, wr, n, gamma=GAMMA):
    """Local Lax-Friedrichs flux along n (switchable alternative)."""
    _, ul, vl, pl = primitives(wl, gamma)
    _, ur, vr, pr = primitives(wr, gamma)
    cl = torch.sqrt(gamma * pl / wl[..., 0])
    cr = torch.sqrt(gamma * pr / wr[..., 0])
    sl = torch.abs(ul * n[..., 0] + vl * n[..., 1]) + cl
    sr = torch.abs(ur * n[..., 0] + vr * n[..., 1]) + cr
    s = torch.maximum(sl, sr).unsqueeze(-1)
    return 0.5 * (normal_flux(wl, n, gamma) + normal_flux(wr, n, gamma)) - 0.5 * s * (wr - wl)
