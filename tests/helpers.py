"""Test-side helpers: gauge transforms and lattice shifts on natural-layout numpy arrays.

These act on inputs only (they build transformed inputs for the covariance
tests); they do not implement any step of the smearing method.
"""
from __future__ import annotations

import numpy as np

# axis of a [Lt][Lz][Ly][Lx] array that carries spatial direction mu = x, y, z
_AXIS4 = {0: 3, 1: 2, 2: 1}
# axis of a one-slice [Lz][Ly][Lx] array that carries spatial direction mu
_AXIS3 = {0: 2, 1: 1, 2: 0}


def shift4(a: np.ndarray, mu: int, k: int) -> np.ndarray:
    """b(x) = a(x + k mu^) for a field indexed [Lt][Lz][Ly][Lx][...] (periodic)."""
    return np.roll(a, -k, axis=_AXIS4[mu])


def shift3(a: np.ndarray, mu: int, k: int) -> np.ndarray:
    """b(x) = a(x + k mu^) for a one-slice field indexed [Lz][Ly][Lx][...] (periodic)."""
    return np.roll(a, -k, axis=_AXIS3[mu])


def dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def transform_links(U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """U_mu(x) -> G(x) U_mu(x) G^dag(x + mu^) for the spatial mu (t links copied)."""
    out = U.copy()
    for mu in range(3):
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ dag(shift4(G, mu, 1))
    return out


def transform_twolinks(W: np.ndarray, G: np.ndarray) -> np.ndarray:
    """W_mu(x) -> G(x) W_mu(x) G^dag(x + 2mu^), W indexed [Lt][Lz][Ly][Lx][3][3][3]."""
    out = np.empty_like(W)
    for mu in range(3):
        out[..., mu, :, :] = G @ W[..., mu, :, :] @ dag(shift4(G, mu, 2))
    return out


def transform_vector(psi: np.ndarray, G_slice: np.ndarray) -> np.ndarray:
    """psi(x) -> G(x) psi(x) on one slice; psi [..][Lz][Ly][Lx][3], G_slice [Lz][Ly][Lx][3][3]."""
    return np.einsum('...ab,...b->...a', G_slice, psi)


def parity_class(L3, x0=(0, 0, 0)) -> np.ndarray:
    """Boolean [Lz][Ly][Lx] mask of sites x with x_mu - x0_mu even in every direction."""
    Lx, Ly, Lz = L3
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing='ij')
    return ((x - x0[0]) % 2 == 0) & ((y - x0[1]) % 2 == 0) & ((z - x0[2]) % 2 == 0)
