"""Pins of the oracle's Euler pieces against the flux definition of Sec. 2.1:
the eigen-decomposition must rebuild the flux Jacobian (computed here by
autograd of the flux), the Roe flux must be consistent, conservative under edge
reversal, satisfy Roe's property and reduce to pure upwinding when supersonic."""
import numpy as np
import pytest
import torch

from oracle import euler


def states(n, seed=0, mach=0.8):
    g = torch.Generator().manual_seed(seed)
    rho = 0.5 + torch.rand(n, generator=g, dtype=torch.float64)
    p = 0.3 + torch.rand(n, generator=g, dtype=torch.float64)
    c = torch.sqrt(1.4 * p / rho)
    u = mach * c * (2 * torch.rand(n, generator=g, dtype=torch.float64) - 1)
    v = mach * c * (2 * torch.rand(n, generator=g, dtype=torch.float64) - 1)
    return torch.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)], -1)


def directions(n, seed=1):
    a = torch.rand(n, generator=torch.Generator().manual_seed(seed), dtype=torch.float64) * 2 * np.pi
    return torch.stack([torch.cos(a), torch.sin(a)], -1)


def test_flux_definition_values():
    w = torch.tensor([[2.0, 2.0 * 0.3, 2.0 * -0.4, 1.0 / 0.4 + 0.5 * 2.0 * 0.25]], dtype=torch.float64)
    f, g = euler.fluxes(w)
    # rho=2, u=.3, v=-.4, p=1, rhoE=2.75
    np.testing.assert_allclose(f[0].numpy(), [0.6, 2 * 0.09 + 1, 2 * 0.3 * -0.4, (2.75 + 1) * 0.3], rtol=1e-14)
    np.testing.assert_allclose(g[0].numpy(), [-0.8, 2 * -0.4 * 0.3, 2 * 0.16 + 1, (2.75 + 1) * -0.4], rtol=1e-14)


def test_eigendecomposition_rebuilds_flux_jacobian():
    w = states(20)
    n = directions(20)
    for i in range(20):
        J = torch.autograd.functional.jacobian(lambda x: euler.normal_flux(x, n[i]), w[i])
        R, L = euler.char_basis(w[i], w[i], n[i])
        _, u, v, p = euler.primitives(w[i])
        c = torch.sqrt(1.4 * p / w[i, 0])
        lam = euler.eigenvalues(u, v, c, n[i])
        A = R @ torch.diag(lam) @ L
        np.testing.assert_allclose(A.numpy(), J.numpy(), rtol=1e-12, atol=1e-12)


def test_roe_flux_consistency_and_reversal():
    wl, wr, n = states(50, 2), states(50, 3), directions(50)
    np.testing.assert_allclose(euler.roe_flux(wl, wl, n).numpy(), euler.normal_flux(wl, n).numpy(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(euler.roe_flux(wr, wl, -n).numpy(), -euler.roe_flux(wl, wr, n).numpy(), rtol=1e-12, atol=1e-12)


def test_roe_property():
    wl, wr, n = states(50, 4), states(50, 5), directions(50)
    u, v, H, c = euler.roe_average(wl, wr)
    R = euler.right_eigenvectors(u, v, H, c, n)
    lam = euler.eigenvalues(u, v, c, n)
    A = R @ torch.diag_embed(lam) @ torch.linalg.inv(R)
    lhs = euler.normal_flux(wr, n) - euler.normal_flux(wl, n)
    rhs = (A @ (wr - wl).unsqueeze(-1)).squeeze(-1)
    np.testing.assert_allclose(lhs.numpy(), rhs.numpy(), rtol=1e-11, atol=1e-12)


def test_supersonic_flux_is_upwind():
    wl = states(30, 6, mach=0.0)
    rho, _, _, p = euler.primitives(wl)
    c = torch.sqrt(1.4 * p / rho)
    n = directions(30)
    u = 2.5 * c
    wl = torch.stack([rho, rho * u * n[:, 0], rho * u * n[:, 1], p / 0.4 + 0.5 * rho * u * u], -1)
    wr = wl * torch.tensor([1.01, 1.02, 1.02, 1.015], dtype=torch.float64)
    np.testing.assert_allclose(euler.roe_flux(wl, wr, n).numpy(), euler.normal_flux(wl, n).numpy(), rtol=1e-12, atol=1e-12)


def test_rusanov_consistency():
    wl, n = states(10, 7), directions(10)
    np.testing.assert_allclose(euler.rusanov_flux(wl, wl, n).numpy(), euler.normal_flux(wl, n).numpy(), rtol=1e-13)
