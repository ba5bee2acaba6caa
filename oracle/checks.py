"""Closed forms that pin the FP64 oracle (test infrastructure only).

On the unit gauge field (all links 1) the two-link Laplacian of eq. tlLapl1
reduces to a free lattice operator,

    4 Lap = sum_mu (S_mu - 2),      (S_mu psi)(x) = psi(x + 2mu^) + psi(x - 2mu^),

so one smearing step of eq. tlSmear is  T = (1 - 6c) + c sum_mu S_mu  with
c = sigma / (4n), and the smeared point source is T^n applied to a delta
function.  Two independent evaluations of T^n delta are given here:

* ``free_kernel_dft``: diagonalise T by plane waves.  A plane wave
  exp(i p.x) is an eigenvector of Lap with eigenvalue -sum_mu sin^2(p_mu), so
  T^n delta_{x0}(x) = V^-1 sum_p exp(i p.(x - x0)) (1 - (sigma/n) sum_mu sin^2 p_mu)^n
  with p_mu = 2 pi k / L_mu (evaluated with numpy's inverse FFT).
* ``free_kernel_walks``: expand T^n with the multinomial theorem; S_mu^k
  delta counts the periodic +-2 walks of k steps along mu, which is a sum of
  binomial coefficients.  All terms are positive, so the sum is accurate to
  rounding; ``free_kernel_walks_exact`` does the same sum in integers.

Neither evaluation shares code with the C oracle.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb, factorial, lgamma, log, exp
from typing import Sequence

import numpy as np


def _dims(L3: Sequence[int]):
    Lx, Ly, Lz = (int(v) for v in L3)
    return Lx, Ly, Lz


def plane_wave_eigenvalue(k: Sequence[int], L3: Sequence[int]) -> float:
    """Eigenvalue of the free two-link Laplacian on exp(i p.x), p_mu = 2 pi k_mu / L_mu."""
    return -sum(np.sin(2 * np.pi * kk / LL) ** 2 for kk, LL in zip(k, L3))


def free_kernel_dft(L3: Sequence[int], n: int, sigma: float, x0: Sequence[int] = (0, 0, 0)) -> np.ndarray:
    """Free-field smeared point source, scalar profile [Lz][Ly][Lx] (Fourier form)."""
    Lx, Ly, Lz = _dims(L3)
    pz = 2 * np.pi * np.arange(Lz) / Lz
    py = 2 * np.pi * np.arange(Ly) / Ly
    px = 2 * np.pi * np.arange(Lx) / Lx
    s2 = (np.sin(pz)[:, None, None] ** 2 + np.sin(py)[None, :, None] ** 2
          + np.sin(px)[None, None, :] ** 2)
    lam = 1.0 - (sigma / n) * s2
    k = np.fft.ifftn(lam ** n).real
    return np.roll(k, shift=(x0[2], x0[1], x0[0]), axis=(0, 1, 2))


def plane_wave_eigenvalue_onelink(k: Sequence[int], L3: Sequence[int]) -> float:
    """Eigenvalue of the free one-link Laplacian H - 6 on exp(i p.x): -4 sum_mu sin^2(p_mu / 2)."""
    return float(-4.0 * sum(np.sin(np.pi * k[i] / L3[i]) ** 2 for i in range(3)))


def free_kernel_onelink_dft(L3: Sequence[int], n: int, sigma: float, x0: Sequence[int] = (0, 0, 0)) -> np.ndarray:
    """Free-field point source after (1 + (sigma/n)(H - 6))^n, scalar profile [Lz][Ly][Lx]."""
    Lx, Ly, Lz = _dims(L3)
    s2 = (np.sin(np.pi * np.arange(Lz) / Lz)[:, None, None] ** 2
          + np.sin(np.pi * np.arange(Ly) / Ly)[None, :, None] ** 2
          + np.sin(np.pi * np.arange(Lx) / Lx)[None, None, :] ** 2)
    lam = 1.0 - (sigma / n) * 4.0 * s2
    k = np.fft.ifftn(lam ** n).real
    return np.roll(k, shift=(x0[2], x0[1], x0[0]), axis=(0, 1, 2))


def walk_counts(L: int, kmax: int) -> np.ndarray:
    """B[k, x] = number of k-step walks with steps +-2 from 0 ending at x (mod L)."""
    B = np.zeros((kmax + 1, L), dtype=np.float64)
    for k in range(kmax + 1):
        for j in range(k + 1):
            B[k, (2 * (2 * j - k)) % L] += comb(k, j)
    return B


def free_kernel_walks(L3: Sequence[int], n: int, sigma: float, x0: Sequence[int] = (0, 0, 0)) -> np.ndarray:
    """Free-field smeared point source [Lz][Ly][Lx] (multinomial sum of +-2 walks)."""
    Lx, Ly, Lz = _dims(L3)
    c = sigma / (4.0 * n)
    a = 1.0 - 6.0 * c
    if not (a > 0 and c > 0):
        raise ValueError("closed form implemented for 0 < sigma/n < 2/3")
    Bx, By, Bz = walk_counts(Lx, n), walk_counts(Ly, n), walk_counts(Lz, n)
    out = np.zeros((Lz, Ly, Lx))
    lf = [lgamma(k + 1) for k in range(n + 1)]
    for k3 in range(n + 1):
        C = np.zeros((n + 1, n + 1))
        for k2 in range(n + 1 - k3):
            for k1 in range(n + 1 - k3 - k2):
                k0 = n - k1 - k2 - k3
                C[k1, k2] = exp(lf[n] - lf[k0] - lf[k1] - lf[k2] - lf[k3]
                                + k0 * log(a) + (n - k0) * log(c))
        plane = By.T @ C.T @ Bx            # [y][x] = sum_{k1,k2} C[k1,k2] By[k2,y] Bx[k1,x]
        out += Bz[k3][:, None, None] * plane[None, :, :]
    return np.roll(out, shift=(x0[2], x0[1], x0[0]), axis=(0, 1, 2))


def free_kernel_walks_exact(L3: Sequence[int], n: int, sigma: Fraction) -> dict:
    """Exact rational free-field kernel: {(x, y, z): Fraction} for the point source at 0."""
    Lx, Ly, Lz = _dims(L3)
    sigma = Fraction(sigma)
    c = sigma / (4 * n)
    a = 1 - 6 * c
    def counts(L):
        B = [[0] * L for _ in range(n + 1)]
        for k in range(n + 1):
            for j in range(k + 1):
                B[k][(2 * (2 * j - k)) % L] += comb(k, j)
        return B
    Bx, By, Bz = counts(Lx), counts(Ly), counts(Lz)
    out = {}
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                out[(x, y, z)] = Fraction(0)
    for k1 in range(n + 1):
        for k2 in range(n + 1 - k1):
            for k3 in range(n + 1 - k1 - k2):
                k0 = n - k1 - k2 - k3
                m = factorial(n) // (factorial(k0) * factorial(k1) * factorial(k2) * factorial(k3))
                coef = m * a ** k0 * c ** (k1 + k2 + k3)
                for z in range(Lz):
                    if Bz[k3][z] == 0:
                        continue
                    for y in range(Ly):
                        if By[k2][y] == 0:
                            continue
                        byz = Bz[k3][z] * By[k2][y]
                        for x in range(Lx):
                            if Bx[k1][x]:
                                out[(x, y, z)] += coef * byz * Bx[k1][x]
    return out


def dense_operator(apply, shape) -> np.ndarray:
    """Matrix of a linear map on complex arrays of ``shape`` (columns = images of unit vectors)."""
    n = int(np.prod(shape))
    D = np.empty((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1.0
        D[:, j] = np.asarray(apply(e.reshape(shape))).reshape(n)
    return D


def max_rel(a: np.ndarray, ref: np.ndarray) -> float:
    """max_x |a(x) - ref(x)| / max_x |ref(x)| over colour vectors (last axis = colour)."""
    d = np.sqrt(np.sum(np.abs(np.asarray(a) - np.asarray(ref)) ** 2, axis=-1))
    r = np.sqrt(np.sum(np.abs(np.asarray(ref)) ** 2, axis=-1))
    m = r.max()
    return float(d.max() / m) if m > 0 else float(d.max())


def l2_rel(a: np.ndarray, ref: np.ndarray) -> float:
    num = np.linalg.norm(np.asarray(a).ravel() - np.asarray(ref).ravel())
    den = np.linalg.norm(np.asarray(ref).ravel())
    return float(num / den) if den > 0 else float(num)
