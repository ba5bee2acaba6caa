"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each ``pin_*`` function takes an oracle handle and raises AssertionError when
the oracle disagrees with a closed form, an invariant, a special case or a
brute-force evaluation.  ``tests/test_oracle.py`` runs them on the real oracle;
``tests/test_oracle_mutants.py`` runs them on deliberately broken copies of
the oracle source to show that every planted mistake is caught.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

from oracle import checks
from paper_2301_05518_amd import synth
from tests import helpers as H

TOL = 1e-13
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(k):
    return np.random.default_rng([20230113, k])


def _haar_links(L, seed):
    return synth.gauge_field(L, "haar", seed)


# ------------------------------------------------------------- two-link product

def pin_twolinks_unit(orc):
    """Unit links give unit two-link products (Sec. 2, definition of V_mu)."""
    W = orc.build_twolinks(synth.unit_gauge((4, 3, 5, 2)))
    assert np.abs(W - np.eye(3)).max() == 0.0


def pin_twolinks_diagonal_phases(orc):
    """Diagonal phase links: V_mu(x) = diag(exp(i(theta(x) + theta(x+mu^)))) exactly."""
    L = (5, 4, 6, 3)
    theta = _rng(1).uniform(-np.pi, np.pi, size=(L[3], L[2], L[1], L[0], 4, 3))
    U = np.zeros(theta.shape[:-1] + (3, 3), np.complex128)
    for a in range(3):
        U[..., a, a] = np.exp(1j * theta[..., a])
    W = orc.build_twolinks(U)
    for mu in range(3):
        expect = theta[..., mu, :] + H.shift4(theta[..., mu, :], mu, 1)
        ref = np.zeros(W.shape[:4] + (3, 3), np.complex128)
        for a in range(3):
            ref[..., a, a] = np.exp(1j * expect[..., a])
        assert np.abs(W[..., mu, :, :] - ref).max() < TOL


def pin_twolinks_su3(orc):
    """Products of SU(3) links are SU(3): unitary and unit determinant."""
    W = orc.build_twolinks(_haar_links((4, 4, 4, 2), 11))
    eye = np.eye(3)
    assert np.abs(W @ H.dag(W) - eye).max() < TOL
    assert np.abs(np.linalg.det(W) - 1.0).max() < TOL


def pin_twolinks_third_row(orc):
    """A product of SU(3) links has third row conj(row0 x row1), the identity behind the
    twelve-real two-link storage; links scaled off SU(3) break it (so the storage is valid
    for special unitary links only)."""
    U = _haar_links((5, 4, 3, 2), 14)
    W = orc.build_twolinks(U)
    rebuilt = np.conj(np.cross(W[..., 0, :], W[..., 1, :]))
    assert np.abs(rebuilt - W[..., 2, :]).max() < TOL
    Ws = orc.build_twolinks(1.1 * U)
    rebuilt = np.conj(np.cross(Ws[..., 0, :], Ws[..., 1, :]))
    assert np.abs(rebuilt - Ws[..., 2, :]).max() > 0.1


def pin_twolinks_covariance(orc):
    """Gauge covariance: U -> G U G^dag(x+mu^) gives W -> G(x) W G^dag(x+2mu^).

    Fixes the operand order of the product and the neighbour it reads.
    """
    L = (4, 6, 5, 2)
    U = _haar_links(L, 12)
    G = synth.gauge_transform(L, 13)
    W = orc.build_twolinks(U)
    WG = orc.build_twolinks(H.transform_links(U, G))
    assert np.abs(WG - H.transform_twolinks(W, G)).max() < TOL


# ------------------------------------------------------------- Laplacian

def _random_w(L, seed, unitary=True):
    """A two-link-shaped field that is not a product of links (tests the Laplacian alone)."""
    if unitary:
        w = synth.su3_haar(_rng(seed), L[3] * L[2] * L[1] * L[0] * 3)
    else:
        w = synth.random_field(_rng(seed), (L[3] * L[2] * L[1] * L[0] * 3, 3, 3))
    return w.reshape(L[3], L[2], L[1], L[0], 3, 3, 3)


def pin_lap_forms_agree(orc):
    """Eq. tlLapl1 (precomputed W) equals eq. tlLapl2 (two one-link transports)."""
    for L in ((6, 4, 8, 3), (4, 4, 4, 1), (5, 3, 7, 2), (2, 1, 3, 1)):
        U = _haar_links(L, 20 + L[0])
        W = orc.build_twolinks(U)
        for t in range(L[3]):
            psi = synth.random_field(_rng(21 + t), (L[2], L[1], L[0], 3))
            a = orc.laplacian(W, t, psi)
            b = orc.laplacian_oneplusone(U, t, psi)
            assert checks.max_rel(a, b) < TOL


def pin_lap_plane_waves(orc):
    """Unit links: exp(i p.x) e_c is an eigenvector with eigenvalue -sum_mu sin^2 p_mu.

    At L_mu = 4 the +2 and -2 neighbours coincide and both hops must count.
    """
    for L3 in ((4, 6, 8), (8, 4, 5), (3, 4, 2)):
        Lx, Ly, Lz = L3
        W = orc.build_twolinks(synth.unit_gauge(L3 + (1,)))
        z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing='ij')
        for k in ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 2, 3), (Lx - 1, 1, Lz // 2)):
            k = (k[0] % Lx, k[1] % Ly, k[2] % Lz)
            phase = np.exp(2j * np.pi * (k[0] * x / Lx + k[1] * y / Ly + k[2] * z / Lz))
            for c in range(3):
                psi = np.zeros((Lz, Ly, Lx, 3), np.complex128)
                psi[..., c] = phase
                out = orc.laplacian(W, 0, psi)
                lam = checks.plane_wave_eigenvalue(k, L3)
                assert np.abs(out - lam * psi).max() < TOL


def pin_lap_hermitian(orc):
    """<phi, Lap psi> = <Lap phi, psi>, also for non-unitary two-link fields."""
    for unitary in (True, False):
        L = (6, 4, 5, 2)
        W = _random_w(L, 30 + unitary, unitary)
        for t in range(L[3]):
            phi = synth.random_field(_rng(31), (L[2], L[1], L[0], 3))
            psi = synth.random_field(_rng(32), (L[2], L[1], L[0], 3))
            lhs = np.vdot(phi, orc.laplacian(W, t, psi))
            rhs = np.vdot(orc.laplacian(W, t, phi), psi)
            assert abs(lhs - rhs) < TOL * abs(lhs)


def pin_lap_covariance(orc):
    """Lap[W^G](G psi) = G Lap[W](psi) with W^G(x) = G(x) W(x) G^dag(x+2mu^)."""
    L = (4, 6, 6, 2)
    W = _random_w(L, 40)
    G = synth.gauge_transform(L, 41)
    WG = H.transform_twolinks(W, G)
    for t in range(L[3]):
        psi = synth.random_field(_rng(42), (L[2], L[1], L[0], 3))
        a = orc.laplacian(WG, t, H.transform_vector(psi, G[t]))
        b = H.transform_vector(orc.laplacian(W, t, psi), G[t])
        assert checks.max_rel(a, b) < TOL


def pin_lap_sublattice_and_slice(orc):
    """Taste preservation: hops of two sites keep each parity sublattice to itself.

    Also: the result on slice t depends only on the links of slice t.
    """
    L = (6, 8, 4, 3)
    U = _haar_links(L, 50)
    W = orc.build_twolinks(U)
    rng = _rng(51)
    for x0 in ((0, 0, 0), (1, 0, 1), (1, 1, 1)):
        mask = H.parity_class(L[:3], x0)
        psi = synth.random_field(rng, (L[2], L[1], L[0], 3)) * mask[..., None]
        out = orc.laplacian(W, 1, psi)
        assert np.abs(out[~mask]).max() == 0.0
        assert np.abs(out[mask]).max() > 0.1
    U2 = U.copy()
    U2[0] = synth.gauge_field(L, "haar", 52)[0]
    U2[2] = synth.gauge_field(L, "haar", 53)[2]
    U2[..., 3, :, :] = np.eye(3)
    psi = synth.random_field(rng, (L[2], L[1], L[0], 3))
    a = orc.laplacian(W, 1, psi)
    b = orc.laplacian(orc.build_twolinks(U2), 1, psi)
    assert np.abs(a - b).max() == 0.0


def pin_lap_dense_nsd(orc):
    """Dense 4^3 matrix: Hermitian, spectrum in [-3, 0] for unitary links; free field exact."""
    L = (4, 4, 4, 1)
    W = orc.build_twolinks(_haar_links(L, 60))
    D = checks.dense_operator(lambda v: orc.laplacian(W, 0, v), (4, 4, 4, 3))
    assert np.abs(D - D.conj().T).max() < TOL
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= -3.0 - 1e-12 and ev.max() <= 1e-12
    # free field: the dense spectrum is the plane-wave spectrum, 3-fold for colour
    W1 = orc.build_twolinks(synth.unit_gauge(L))
    D1 = checks.dense_operator(lambda v: orc.laplacian(W1, 0, v), (4, 4, 4, 3))
    ev1 = np.sort(np.linalg.eigvalsh(D1))
    pw = sorted(checks.plane_wave_eigenvalue((kx, ky, kz), (4, 4, 4))
                for kz in range(4) for ky in range(4) for kx in range(4) for _ in range(3))
    assert np.abs(ev1 - np.array(pw)).max() < 1e-12


# ------------------------------------------------------------- smearing

def pin_smear_free_field(orc):
    """Unit links: the smeared point source equals the exact free kernel (both closed forms)."""
    cases = (((8, 8, 8), 20, 2.0, (0, 0, 0)), ((4, 6, 10), 7, 1.5, (1, 2, 3)),
             ((5, 4, 3), 9, 3.0, (2, 1, 0)))
    for L3, n, sigma, x0 in cases:
        W = orc.build_twolinks(synth.unit_gauge(L3 + (2,)))
        for c in range(3):
            src = synth.point_source(L3, c, x0)
            out = orc.smear(W, 1, n, sigma, src)
            k1 = checks.free_kernel_dft(L3, n, sigma, x0)
            k2 = checks.free_kernel_walks(L3, n, sigma, x0)
            ref = np.zeros_like(out)
            ref[..., c] = k2
            assert np.abs(k1 - k2).max() < 1e-14 * np.abs(k2).max()
            assert checks.max_rel(out, ref) < TOL


def pin_smear_golden_free(orc):
    """Fig. 1a quantity: |psi(x, y, 0, 0)| of a free-field smeared point source, exact values."""
    path = os.path.join(GOLDEN, "free_point_8x8x8_n20_sigma2.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    W = orc.build_twolinks(synth.unit_gauge((8, 8, 8, 1)))
    out = orc.smear(W, 0, 20, 2.0, synth.point_source((8, 8, 8), 0))
    norms = orc.site_norms(out)
    peak = max(float(Fraction(r[3])) for r in rows)
    for x, y, z, val in rows:
        assert abs(norms[int(z), int(y), int(x)] - float(Fraction(val))) < TOL * peak


def pin_smear_dense_power(orc):
    """4^3 random links: smearing equals matrix_power(1 + (sigma/n) D, n) applied to psi."""
    L = (4, 4, 4, 2)
    W = orc.build_twolinks(_haar_links(L, 70))
    D = checks.dense_operator(lambda v: orc.laplacian(W, 1, v), (4, 4, 4, 3))
    n, sigma = 6, 1.2
    T = np.linalg.matrix_power(np.eye(D.shape[0]) + (sigma / n) * D, n)
    psi = synth.random_field(_rng(71), (4, 4, 4, 3))
    out = orc.smear(W, 1, n, sigma, psi)
    assert checks.max_rel(out, (T @ psi.ravel()).reshape(psi.shape)) < TOL


def pin_smear_special_cases(orc):
    """sigma=0 is the identity; n=1 is psi + sigma Lap psi; the map is linear."""
    L = (6, 4, 6, 2)
    W = orc.build_twolinks(_haar_links(L, 80))
    rng = _rng(81)
    psi = synth.random_field(rng, (6, 4, 6, 3))
    phi = synth.random_field(rng, (6, 4, 6, 3))
    assert np.abs(orc.smear(W, 1, 5, 0.0, psi) - psi).max() == 0.0
    one = orc.smear(W, 1, 1, 0.7, psi)
    assert checks.max_rel(one, psi + 0.7 * orc.laplacian(W, 1, psi)) < TOL
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lin = orc.smear(W, 1, 8, 2.0, a * psi + b * phi)
    ref = a * orc.smear(W, 1, 8, 2.0, psi) + b * orc.smear(W, 1, 8, 2.0, phi)
    assert checks.max_rel(lin, ref) < TOL


def pin_smear_covariance_and_contraction(orc):
    """smear(G U, G psi) = G smear(U, psi); for sigma/n <= 2/3 the norm does not grow."""
    L = (6, 6, 4, 2)
    U = _haar_links(L, 90)
    G = synth.gauge_transform(L, 91)
    psi = synth.random_field(_rng(92), (4, 6, 6, 3))
    W = orc.build_twolinks(U)
    WG = orc.build_twolinks(H.transform_links(U, G))
    a = orc.smear(WG, 0, 10, 4.0, H.transform_vector(psi, G[0]))
    s = orc.smear(W, 0, 10, 4.0, psi)
    assert checks.max_rel(a, H.transform_vector(s, G[0])) < TOL
    assert np.linalg.norm(s) <= np.linalg.norm(psi)
    assert np.linalg.norm(s) > 0.01 * np.linalg.norm(psi)


def pin_smear_batch(orc):
    """A batch of right-hand sides on different slices equals one-by-one smearing."""
    L = (4, 6, 4, 3)
    W = orc.build_twolinks(_haar_links(L, 95))
    psi = synth.random_field(_rng(96), (4, 4, 6, 4, 3))
    ts = [2, 0, 2, 1]
    out = orc.smear_batch(W, ts, 5, 1.0, psi)
    for r, t in enumerate(ts):
        assert np.abs(out[r] - orc.smear(W, t, 5, 1.0, psi[r])).max() == 0.0


# ------------------------------------------------------------- one-link smearing (Sec. 2)

def pin_onelink_plane_waves(orc):
    """Unit links: exp(i p.x) e_c is an eigenvector of H with eigenvalue 2 sum_mu cos p_mu and
    of nabla^2 = H - 6 with eigenvalue -4 sum_mu sin^2(p_mu / 2).  At L_mu = 1, 2 the two
    neighbours coincide and both hops count."""
    for L3 in ((4, 6, 8), (5, 3, 7), (1, 2, 3)):
        Lx, Ly, Lz = L3
        U = synth.unit_gauge(L3 + (1,))
        z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing='ij')
        for k in ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 2, 3), (Lx - 1, 1, Lz // 2)):
            k = (k[0] % Lx, k[1] % Ly, k[2] % Lz)
            phase = np.exp(2j * np.pi * (k[0] * x / Lx + k[1] * y / Ly + k[2] * z / Lz))
            psi = np.zeros((Lz, Ly, Lx, 3), np.complex128)
            psi[..., 1] = phase
            lam_h = 2.0 * sum(np.cos(2 * np.pi * k[i] / L3[i]) for i in range(3))
            assert np.abs(orc.hop_onelink(U, 0, psi) - lam_h * psi).max() < TOL
            lam = checks.plane_wave_eigenvalue_onelink(k, L3)
            assert np.abs(orc.laplacian_onelink(U, 0, psi) - lam * psi).max() < TOL


def pin_onelink_dense(orc):
    """Dense 4x4x3 matrices with SU(3) links: nabla^2 Hermitian with spectrum in [-12, 0],
    and H = nabla^2 + 6 entry by entry (two independent code paths)."""
    L = (4, 4, 3, 1)
    U = _haar_links(L, 70)
    D = checks.dense_operator(lambda v: orc.laplacian_onelink(U, 0, v), (3, 4, 4, 3))
    Hm = checks.dense_operator(lambda v: orc.hop_onelink(U, 0, v), (3, 4, 4, 3))
    assert np.abs(D - D.conj().T).max() < TOL
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= -12.0 - 1e-12 and ev.max() <= 1e-12
    assert np.abs(Hm - (D + 6.0 * np.eye(D.shape[0]))).max() < TOL


def pin_onelink_covariance_and_slice(orc):
    """nabla^2[U^G](G psi) = G nabla^2[U](psi); the result on slice t reads only the spatial
    links of slice t."""
    L = (4, 5, 6, 2)
    U = _haar_links(L, 71)
    G = synth.gauge_transform(L, 72)
    UG = H.transform_links(U, G)
    for t in range(L[3]):
        psi = synth.random_field(_rng(73 + t), (L[2], L[1], L[0], 3))
        a = orc.laplacian_onelink(UG, t, H.transform_vector(psi, G[t]))
        b = H.transform_vector(orc.laplacian_onelink(U, t, psi), G[t])
        assert checks.max_rel(a, b) < TOL
    U2 = U.copy()
    U2[0] = synth.gauge_field(L, "haar", 74)[0]
    U2[..., 3, :, :] = np.eye(3)
    psi = synth.random_field(_rng(75), (L[2], L[1], L[0], 3))
    assert np.abs(orc.laplacian_onelink(U, 1, psi) - orc.laplacian_onelink(U2, 1, psi)).max() == 0.0


def pin_gsmear_identity(orc):
    """The rewriting that follows eq. gsmear: (1 + alpha H)^n = (1 + 6 alpha)^n (1 + alpha' nabla^2)^n
    with alpha' = alpha / (1 + 6 alpha), i.e. the Laplacian-form smearing with sigma = n alpha'.
    Also sigma = 0 is the identity and n = 1 is psi + sigma nabla^2 psi."""
    L = (6, 5, 4, 2)
    U = _haar_links(L, 76)
    psi = synth.random_field(_rng(77), (L[2], L[1], L[0], 3))
    for alpha, n in ((0.05, 7), (0.1, 12), (-0.02, 5)):
        a = orc.gsmear_hop(U, 1, n, alpha, psi)
        ap = alpha / (1.0 + 6.0 * alpha)
        b = (1.0 + 6.0 * alpha) ** n * orc.smear_onelink(U, 1, n, n * ap, psi)
        assert checks.max_rel(a, b) < 1e-12
    assert np.abs(orc.smear_onelink(U, 0, 9, 0.0, psi) - psi).max() == 0.0
    one = orc.smear_onelink(U, 0, 1, 0.13, psi)
    assert checks.max_rel(one, psi + 0.13 * orc.laplacian_onelink(U, 0, psi)) < TOL
    ts = [1, 0, 1]
    batch = np.stack([psi, 2 * psi, 1j * psi])
    out = orc.smear_onelink_batch(U, ts, 4, 0.3, batch)
    for r in range(3):
        assert np.abs(out[r] - orc.smear_onelink(U, ts[r], 4, 0.3, batch[r])).max() == 0.0


def pin_onelink_free_field(orc):
    """Unit links: a smeared point source equals the plane-wave closed form."""
    L3 = (8, 6, 10)
    U = synth.unit_gauge(L3 + (1,))
    for c, x0 in ((0, (0, 0, 0)), (2, (1, 2, 3))):
        psi = synth.point_source(L3, c, x0)
        out = orc.smear_onelink(U, 0, 12, 1.5, psi)
        ref = np.zeros_like(out)
        ref[..., c] = checks.free_kernel_onelink_dft(L3, 12, 1.5, x0)
        assert np.abs(out - ref).max() < TOL


# ------------------------------------------------------------- reductions

def pin_reductions(orc):
    """FP64 norms and inner products against closed forms.

    A normalised plane wave has unit norm; <phi, psi> is conjugate-linear in
    phi and linear in psi; site norms square-sum to the total norm.
    """
    Lx, Ly, Lz = 6, 4, 5
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing='ij')
    wave = np.exp(2j * np.pi * (x / Lx + 2 * y / Ly - z / Lz)) / np.sqrt(Lx * Ly * Lz)
    psi = np.zeros((Lz, Ly, Lx, 3), np.complex128)
    psi[..., 1] = wave
    assert abs(orc.norm2(psi) - 1.0) < TOL
    psi[..., 2] = 2j * wave
    assert abs(orc.norm2(psi) - 5.0) < TOL
    rng = _rng(100)
    a = synth.random_field(rng, (Lz, Ly, Lx, 3))
    b = synth.random_field(rng, (Lz, Ly, Lx, 3))
    ab = orc.dot(a, b)
    assert abs(orc.dot(1j * a, b) - (-1j) * ab) < TOL * abs(ab)
    assert abs(orc.dot(a, 1j * b) - 1j * ab) < TOL * abs(ab)
    assert abs(orc.dot(b, a) - np.conj(ab)) < TOL * abs(ab)
    assert abs(orc.dot(a, a) - orc.norm2(a)) < TOL * orc.norm2(a)
    sn = orc.site_norms(a)
    assert abs(np.sum(sn ** 2) - orc.norm2(a)) < TOL * orc.norm2(a)
    e = np.zeros((Lz, Ly, Lx, 3), np.complex128)
    e[1, 2, 3] = (3.0, 4.0j, 0.0)
    sn = orc.site_norms(e)
    assert sn[1, 2, 3] == 5.0 and sn.sum() == 5.0


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
