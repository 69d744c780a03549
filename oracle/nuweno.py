"""Non-uniform fifth-order WENO interpolation at an edge midpoint (Appendix).

Five points x_{i-2} .. x_{i+2} with the midpoint of [x_i, x_{i+1}] at the origin
(x_i = -x_{i+1}).  The three sub-stencils S0 = {i-2, i-1, i}, S1 = {i-1, i, i+1},
S2 = {i, i+1, i+2} give quadratic interpolants evaluated at 0 (eqs. A1-A3, the
a/b/c coefficient formulas written out below), combined with the linear weights
C_k (closed forms printed in the Appendix, summing to one).  The nonlinear
weights are omega_k = alpha_k / sum(alpha), alpha_k = C_k / (beta_k + eps)^q with
q = 1 and eps = 1e-40 as printed, and the smoothness indicator

    beta_k = sum_{l=1,2} int_{x_i}^{x_{i+1}} dx^(2l-1) (d^l u_k / dx^l)^2 dx.

Reading: dx is the integration interval x_{i+1} - x_i (the paper leaves it
undefined).  The oracle evaluates beta_k from the definition: the quadratic's
monomial coefficients come from solving its 3x3 Vandermonde system, and the
polynomial integrals are taken in closed form.

Geometry-only quantities are numpy arrays; values are torch tensors (FP64) so
autograd can differentiate the nonlinear weights.
"""
from __future__ import annotations

import numpy as np
import torch

WENO_EPS = 1e-40
WENO_POWER = 1


def substencil_coefficients(x: np.ndarray) -> np.ndarray:
    """[n, 3, 3]: coefficient of node S_k[m] in the S_k interpolant at 0 (eqs. A1-A3)."""
    xm2, xm1, x0, xp1, xp2 = (x[:, k] for k in range(5))
    a0 = xm1 * x0 * (x0 - xm1)
    a1 = -xm2 * x0 * (x0 - xm2)
    a2 = xm2 * xm1 * (xm1 - xm2)
    d0 = (xm1 - xm2) * (x0 - xm2) * (x0 - xm1)
    b0 = x0 * xp1 * (xp1 - x0)
    b1 = -xm1 * xp1 * (xp1 - xm1)
    b2 = x0 * xm1 * (x0 - xm1)
    d1 = (x0 - xm1) * (xp1 - xm1) * (xp1 - x0)
    c0 = xp1 * xp2 * (xp2 - xp1)
    c1 = -x0 * xp2 * (xp2 - x0)
    c2 = xp1 * x0 * (xp1 - x0)
    d2 = (xp1 - x0) * (xp2 - x0) * (xp2 - xp1)
    return np.stack([np.stack([a0, a1, a2], -1) / d0[:, None],
                     np.stack([b0, b1, b2], -1) / d1[:, None],
                     np.stack([c0, c1, c2], -1) / d2[:, None]], 1)


def linear_weights(x: np.ndarray) -> np.ndarray:
    """[n, 3]: optimal linear weights C_0, C_1, C_2 (Appendix, eq. C_K)."""
    xm2, xm1, x0, xp1, xp2 = (x[:, k] for k in range(5))
    C0 = xp1 * xp2 / ((xp1 - xm2) * (xp2 - xm2))
    C1 = -xm2 * (-xm2 - xm1 + xp1 + xp2) * xp2 / ((xp1 - xm2) * (xp2 - xm2) * (xp2 - xm1))
    C2 = xm2 * xm1 / ((xp2 - xm2) * (xp2 - xm1))
    return np.stack([C0, C1, C2], -1)


class NUWeno5:
    """Geometry of a batch of five-point stencils, ready to interpolate values."""

    def __init__(self, x: np.ndarray, eps: float = WENO_EPS, power: int = WENO_POWER):
        x = np.asarray(x, dtype=np.float64)
        self.x = x
        self.eps = eps
        self.power = power
        self.sub = torch.from_numpy(substencil_coefficients(x))          # [n,3,3]
        self.C = torch.from_numpy(linear_weights(x))                     # [n,3]
        # Vandermonde inverses: monomial coefficients (q0, q1, q2) of each sub-stencil quadratic
        V = np.stack([np.stack([np.ones_like(x[:, k:k + 3]), x[:, k:k + 3], x[:, k:k + 3] ** 2], -1)
                      for k in range(3)], 1)                             # [n,3(k),3(node),3(pow)]
        self.Vinv = torch.from_numpy(np.linalg.inv(V))                   # [n,3,3(pow),3(node)]
        a, b = x[:, 2], x[:, 3]
        self.a = torch.from_numpy(a)
        self.b = torch.from_numpy(b)
        self.dx = torch.from_numpy(b - a)

    def _sub_values(self, u):
        """u [n, 5, *] -> sub-stencil interpolants [n, 3, *] and node triples [n, 3, 3, *]."""
        trip = torch.stack([u[:, k:k + 3] for k in range(3)], 1)         # [n,3,3,*]
        extra = u.dim() - 2
        sub = self.sub.reshape(self.sub.shape + (1,) * extra)
        return (sub * trip).sum(2), trip

    def smoothness(self, u):
        """beta_k [n, 3, *] from the definition (closed-form polynomial integrals)."""
        _, trip = self._sub_values(u)
        extra = u.dim() - 2
        Vinv = self.Vinv.reshape(self.Vinv.shape + (1,) * extra)
        q = (Vinv * trip.unsqueeze(2)).sum(3)                            # [n,3,3(pow),*]
        q1, q2 = q[:, :, 1], q[:, :, 2]
        sh = (-1, 1) + (1,) * extra
        a, b, dx = self.a.reshape(sh), self.b.reshape(sh), self.dx.reshape(sh)
        # int_a^b (q1 + 2 q2 x)^2 dx  and  int_a^b (2 q2)^2 dx
        i1 = q1 * q1 * (b - a) + 2.0 * q1 * q2 * (b * b - a * a) + (4.0 / 3.0) * q2 * q2 * (b ** 3 - a ** 3)
        i2 = 4.0 * q2 * q2 * (b - a)
        return dx * i1 + dx ** 3 * i2

    def linear(self, u):
        """Linear (optimal-weight) interpolant sum_k C_k u_k at 0."""
        ut, _ = self._sub_values(u)
        extra = u.dim() - 2
        C = self.C.reshape(self.C.shape + (1,) * extra)
        return (C * ut).sum(1)

    def weights(self, u):
        beta = self.smoothness(u)
        extra = u.dim() - 2
        C = self.C.reshape(self.C.shape + (1,) * extra)
        alpha = C / (beta + self.eps) ** self.power
        return alpha / alpha.sum(1, keepdim=True)

    def __call__(self, u):
        """Nonlinear interpolant sum_k omega_k u_k at the midpoint."""
        ut, _ = self._sub_values(u)
        return (self.weights(u) * ut).sum(1)


def uniform_weno5(n: int, eps: float = WENO_EPS, power: int = WENO_POWER) -> NUWeno5:
    """Standard (uniform) WENO5 midpoint interpolation: the same construction on
    equally spaced coordinates, whatever the true node positions are."""
    x = np.tile(np.array([-2.5, -1.5, -0.5, 0.5, 1.5]), (n, 1))
    return NUWeno5(x, eps, power)
