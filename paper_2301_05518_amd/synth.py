"""Seeded synthetic inputs for two-link staggered Gaussian smearing.

This module only draws inputs: gauge links, gauge transforms, sources and
source time slices.  It holds none of the smearing method's arithmetic (no
two-link product, no Laplacian, no smearing step), so that the independent
FP64 oracle and the HIP library can both be fed from it without sharing any
of the method's code.

Array conventions (all complex128, C order, host numpy arrays):

* gauge field ``U``: ``[Lt][Lz][Ly][Lx][mu][a][b]`` with ``mu`` = 0,1,2,3 for
  x, y, z, t.  ``U[..., mu, :, :]`` at site x is the link U_mu(x) that
  transports a colour vector from x+mu^ to x (the hopping operator of Sec. 2).
* colour-vector field on one time slice: ``[Lz][Ly][Lx][3]``; a batch of
  right-hand sides stacks these as ``[n_rhs][Lz][Ly][Lx][3]``.
* geometry ``L = (Lx, Ly, Lz, Lt)``.

Every random draw goes through ``numpy.random.default_rng([seed, *keys])``
(PCG64 behind a SeedSequence), so each time slice of a gauge field can be
drawn on its own and the result does not depend on the number of worker
threads used.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

BASE_SEED = 2301055180
STREAM_LINKS = 0
STREAM_SOURCES = 1
STREAM_GAUGE_TRANSFORM = 2


def seed_for(config_index: int, stream: int) -> int:
    """Seed of one random stream of one workload (links, sources, transform)."""
    return BASE_SEED + 10 * int(config_index) + int(stream)


def rng_for(seed: int, *keys: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), *[int(k) for k in keys]])


# ---------------------------------------------------------------- SU(3) draws

def _complex_normal(rng: np.random.Generator, shape, std: float = 1.0) -> np.ndarray:
    z = rng.standard_normal(tuple(shape) + (2,))
    return std * (z[..., 0] + 1j * z[..., 1])


def _cross(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.stack(
        [a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
         a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
         a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def su3_from_rows(r1: np.ndarray, r2: np.ndarray) -> np.ndarray:
    """Special-unitary matrix whose first two rows span (r1, r2).

    Gram-Schmidt on the two rows, then row 3 = conj(row1 x row2), which makes
    the determinant exactly |row1 x row2|^2 = 1.  Used both to draw Haar SU(3)
    matrices and to reunitarise nearly unitary ones.
    """
    u1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    proj = np.sum(np.conj(u1) * r2, axis=-1, keepdims=True)
    v = r2 - proj * u1
    u2 = v / np.linalg.norm(v, axis=-1, keepdims=True)
    u3 = np.conj(_cross(u1, u2))
    return np.stack([u1, u2, u3], axis=-2)


def reunitarise(m: np.ndarray) -> np.ndarray:
    return su3_from_rows(m[..., 0, :], m[..., 1, :])


def su3_haar(rng: np.random.Generator, n: int) -> np.ndarray:
    """n SU(3) matrices, Haar distributed.

    The first two rows of a Haar U(3) matrix are Gram-Schmidt of two complex
    Gaussian rows; completing them with det = 1 gives the Haar measure on
    SU(3).  This is the "near-Haar" link recipe of the large workloads.
    """
    z = _complex_normal(rng, (n, 2, 3))
    return su3_from_rows(z[:, 0, :], z[:, 1, :])


def su3_exp_antiherm(rng: np.random.Generator, n: int, std: float = 0.3) -> np.ndarray:
    """n SU(3) matrices exp(A), A traceless anti-Hermitian, then reunitarised.

    A = (M - M^dag)/2 minus its trace part, where Re M and Im M are i.i.d.
    N(0, std^2).  exp(A) is taken through the eigendecomposition of the
    Hermitian matrix iA.
    """
    m = _complex_normal(rng, (n, 3, 3), std)
    a = 0.5 * (m - np.conj(np.swapaxes(m, -1, -2)))
    tr = np.trace(a, axis1=-2, axis2=-1) / 3.0
    a = a - tr[:, None, None] * np.eye(3)
    lam, vec = np.linalg.eigh(1j * a)
    expa = np.einsum('nij,nj,nkj->nik', vec, np.exp(-1j * lam), np.conj(vec))
    return reunitarise(expa)


def unit_gauge(L: Sequence[int]) -> np.ndarray:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    u = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def gauge_slice(L: Sequence[int], kind: str, seed: int, t: int) -> np.ndarray:
    """Links of time slice t, shape [Lz][Ly][Lx][4][3][3]; drawn from (seed, t)."""
    Lx, Ly, Lz, _ = (int(v) for v in L)
    n = Lz * Ly * Lx * 4
    rng = rng_for(seed, t)
    if kind == "haar":
        u = su3_haar(rng, n)
    elif kind == "exp":
        u = su3_exp_antiherm(rng, n, 0.3)
    elif kind == "unit":
        u = np.zeros((n, 3, 3), np.complex128)
        u[:, 0, 0] = u[:, 1, 1] = u[:, 2, 2] = 1.0
    else:
        raise ValueError(f"unknown link recipe {kind!r}")
    return u.reshape(Lz, Ly, Lx, 4, 3, 3)


def gauge_field(L: Sequence[int], kind: str, seed: int,
                workers: int = 1, out: np.ndarray | None = None) -> np.ndarray:
    """Whole gauge field [Lt][Lz][Ly][Lx][4][3][3]; slice t drawn from (seed, t)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    if out is None:
        out = np.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)

    def one(t):
        out[t] = gauge_slice(L, kind, seed, t)

    if workers <= 1 or Lt == 1:
        for t in range(Lt):
            one(t)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(Lt)))
    return out


def gauge_transform(L: Sequence[int], seed: int) -> np.ndarray:
    """Random SU(3) matrix G(x) per site, shape [Lt][Lz][Ly][Lx][3][3]."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    g = su3_haar(rng_for(seed, 0), Lt * Lz * Ly * Lx)
    return g.reshape(Lt, Lz, Ly, Lx, 3, 3)


# ---------------------------------------------------------------- sources

def point_source(L3: Sequence[int], colour: int, x0: Sequence[int] = (0, 0, 0)) -> np.ndarray:
    """1+0i at spatial site x0 = (x, y, z) in colour c, zero elsewhere."""
    Lx, Ly, Lz = (int(v) for v in L3)
    p = np.zeros((Lz, Ly, Lx, 3), dtype=np.complex128)
    p[x0[2], x0[1], x0[0], colour] = 1.0
    return p


def wall_source(L3: Sequence[int], colour: int) -> np.ndarray:
    """1+0i on every site of the slice in colour c (colour wall source)."""
    Lx, Ly, Lz = (int(v) for v in L3)
    p = np.zeros((Lz, Ly, Lx, 3), dtype=np.complex128)
    p[..., colour] = 1.0
    return p


def z2_source(rng: np.random.Generator, L3: Sequence[int], colour: int) -> np.ndarray:
    """Real +-1 (probability 1/2 each) on every site in colour c, zero elsewhere."""
    Lx, Ly, Lz = (int(v) for v in L3)
    p = np.zeros((Lz, Ly, Lx, 3), dtype=np.complex128)
    p[..., colour] = rng.integers(0, 2, size=(Lz, Ly, Lx)) * 2.0 - 1.0
    return p


def random_field(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian field (Re, Im ~ N(0,1)) of any shape."""
    return _complex_normal(rng, shape)


def random_slices(rng: np.random.Generator, Lt: int, k: int) -> list[int]:
    return sorted(int(t) for t in rng.choice(Lt, size=k, replace=False))


# ---------------------------------------------------------------- workloads

@dataclass
class Lattice:
    """One lattice of a workload and the right-hand sides smeared on it."""
    L: tuple                      # (Lx, Ly, Lz, Lt)
    links: str                    # "exp" | "haar" | "unit"
    link_seed: int
    t_of_rhs: list                # time slice of every RHS
    sources: list = field(default_factory=list)   # (kind, colour[, x0]) per RHS
    source_seed: int = 0

    @property
    def V3(self) -> int:
        return self.L[0] * self.L[1] * self.L[2]

    def source(self, r: int) -> np.ndarray:
        kind, colour = self.sources[r][0], self.sources[r][1]
        L3 = self.L[:3]
        if kind == "point":
            return point_source(L3, colour, self.sources[r][2] if len(self.sources[r]) > 2 else (0, 0, 0))
        if kind == "wall":
            return wall_source(L3, colour)
        if kind == "z2":
            return z2_source(rng_for(self.source_seed, r), L3, colour)
        raise ValueError(kind)

    def sources_array(self) -> np.ndarray:
        return np.stack([self.source(r) for r in range(len(self.t_of_rhs))])

    def links_array(self, workers: int = 1) -> np.ndarray:
        return gauge_field(self.L, self.links, self.link_seed, workers=workers)


@dataclass
class Workload:
    name: str
    lattices: list
    n_steps: int
    sigma: float
    precisions: tuple             # storage precisions the workload is run in

    @property
    def rhs_site_updates(self) -> int:
        return sum(l.V3 * len(l.t_of_rhs) for l in self.lattices) * self.n_steps


def workload(index: int) -> Workload:
    """The five seeded synthetic workloads (index 0..4), smallest first.

    0: 8^3x8, exp-of-anti-Hermitian links, 1 point source (colour 0, t=0),
       N=20, sigma=2, FP64.
    1: 32^3x64, Haar links, 3 colour point sources at the origin of t=0,
       N=40, sigma=4, FP64.
    2: 48^3x96, Haar links, 3 colour point sources on t=0, N=40, sigma=5,
       FP32 and FP16 with a per-site scale.
    3: 64^3x96, Haar links, 3 colour wall sources on each of the 8 slices
       t = 0, 12, ..., 84 (24 RHS), N=60, sigma=6, FP32.
    4: uneven batch 24^3x48 + 32^3x64 + 48^3x96, Haar links, 1/2/4 random
       slices per lattice x 3 colour-diluted Z2 sources, N=40, sigma=4, BF16.
    5: sink smearing of a whole propagator: 64^3x96, Haar links, 3 colour
       walls on every one of the 96 slices (288 RHS) with one two-link field
       for all slices, N=60, sigma=6, FP32.
    """
    s = lambda stream: seed_for(index + 1, stream)  # noqa: E731
    if index == 0:
        lat = Lattice((8, 8, 8, 8), "exp", s(STREAM_LINKS), [0], [("point", 0)], s(STREAM_SOURCES))
        return Workload("8^3x8 fp64 point N=20 sigma=2", [lat], 20, 2.0, ("f64",))
    if index == 1:
        lat = Lattice((32, 32, 32, 64), "haar", s(STREAM_LINKS), [0, 0, 0],
                      [("point", c) for c in range(3)], s(STREAM_SOURCES))
        return Workload("32^3x64 fp64 3 colour points N=40 sigma=4", [lat], 40, 4.0, ("f64",))
    if index == 2:
        lat = Lattice((48, 48, 48, 96), "haar", s(STREAM_LINKS), [0, 0, 0],
                      [("point", c) for c in range(3)], s(STREAM_SOURCES))
        return Workload("48^3x96 fp32/fp16s 3 colour points N=40 sigma=5", [lat], 40, 5.0, ("f32", "f16s"))
    if index == 3:
        ts = [12 * k for k in range(8)]
        t_of_rhs = [t for t in ts for _ in range(3)]
        srcs = [("wall", c) for _ in ts for c in range(3)]
        lat = Lattice((64, 64, 64, 96), "haar", s(STREAM_LINKS), t_of_rhs, srcs, s(STREAM_SOURCES))
        return Workload("64^3x96 fp32 3 colour walls x 8 slices N=60 sigma=6", [lat], 60, 6.0, ("f32",))
    if index == 4:
        rng = rng_for(s(STREAM_SOURCES), 0)
        lats = []
        for j, (L, k) in enumerate((((24, 24, 24, 48), 1), ((32, 32, 32, 64), 2), ((48, 48, 48, 96), 4))):
            ts = random_slices(rng, L[3], k)
            t_of_rhs = [t for t in ts for _ in range(3)]
            srcs = [("z2", c) for _ in ts for c in range(3)]
            lats.append(Lattice(L, "haar", s(STREAM_LINKS) + 1000 * j, t_of_rhs, srcs,
                                s(STREAM_SOURCES) + 1000 * (j + 1)))
        return Workload("uneven 24^3x48+32^3x64+48^3x96 bf16 Z2 N=40 sigma=4", lats, 40, 4.0, ("bf16",))
    if index == 5:
        ts = list(range(96))
        t_of_rhs = [t for t in ts for _ in range(3)]
        srcs = [("wall", c) for _ in ts for c in range(3)]
        lat = Lattice((64, 64, 64, 96), "haar", s(STREAM_LINKS), t_of_rhs, srcs, s(STREAM_SOURCES))
        return Workload("64^3x96 fp32 sink smearing: 3 colour walls x 96 slices N=60 sigma=6", [lat], 60, 6.0,
                        ("f32",))
    raise IndexError(index)
