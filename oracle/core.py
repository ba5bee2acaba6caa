"""ctypes wrapper over the FP64 C oracle (test infrastructure only).

All arrays are host numpy complex128 in the natural layouts documented in
``oracle.c``:  U [Lt][Lz][Ly][Lx][4][3][3], two-link field
[Lt][Lz][Ly][Lx][3][3][3], one-slice colour vectors [Lz][Ly][Lx][3].
Test infrastructure: only the tests, the package smoke check and the
benchmark's CPU-baseline leg use it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_c_int4 = ctypes.c_int * 4
_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Handle on one compiled copy of the oracle library."""

    def __init__(self, path: str | None = None):
        path = path or _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            if path == _build.LIB:
                _build.build()
        self.path = path
        self.lib = ctypes.CDLL(path)
        l = self.lib
        vp = ctypes.c_void_p
        l.or_build_twolinks.argtypes = [_c_int4, vp, vp]
        l.or_lap_twolink.argtypes = [_c_int4, vp, ctypes.c_int, vp, vp]
        l.or_lap_oneplusone.argtypes = [_c_int4, vp, ctypes.c_int, vp, vp]
        l.or_smear.argtypes = [_c_int4, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp]
        l.or_smear_batch.argtypes = [_c_int4, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_double, vp]
        l.or_hop_onelink.argtypes = [_c_int4, vp, ctypes.c_int, vp, vp]
        l.or_lap_onelink.argtypes = [_c_int4, vp, ctypes.c_int, vp, vp]
        l.or_gsmear_hop.argtypes = [_c_int4, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp]
        l.or_smear_onelink.argtypes = [_c_int4, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp]
        l.or_smear_onelink_batch.argtypes = [_c_int4, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_double, vp]
        l.or_norm2.argtypes = [ctypes.c_long, vp]
        l.or_norm2.restype = ctypes.c_double
        l.or_dot.argtypes = [ctypes.c_long, vp, vp, _dp, _dp]
        l.or_site_norms.argtypes = [ctypes.c_long, vp, vp]

    # -- helpers
    @staticmethod
    def _geom(U_or_W: np.ndarray):
        Lt, Lz, Ly, Lx = U_or_W.shape[:4]
        return _c_int4(Lx, Ly, Lz, Lt), (Lx, Ly, Lz, Lt)

    @staticmethod
    def _c128(a: np.ndarray) -> np.ndarray:
        return np.ascontiguousarray(a, dtype=np.complex128)

    # -- the method
    def build_twolinks(self, U: np.ndarray) -> np.ndarray:
        """W_mu(x) = U_mu(x) U_mu(x+mu^) for mu = x, y, z; shape [Lt][Lz][Ly][Lx][3][3][3]."""
        U = self._c128(U)
        assert U.shape[4:] == (4, 3, 3)
        g, _ = self._geom(U)
        W = np.empty(U.shape[:4] + (3, 3, 3), np.complex128)
        self.lib.or_build_twolinks(g, _ptr(U), _ptr(W))
        return W

    def laplacian(self, W: np.ndarray, t: int, psi: np.ndarray) -> np.ndarray:
        """Two-link Laplacian (first form, with W) on slice t."""
        W = self._c128(W)
        psi = self._c128(psi)
        g, L = self._geom(W)
        assert psi.shape == (L[2], L[1], L[0], 3)
        out = np.empty_like(psi)
        self.lib.or_lap_twolink(g, _ptr(W), int(t), _ptr(psi), _ptr(out))
        return out

    def laplacian_oneplusone(self, U: np.ndarray, t: int, psi: np.ndarray) -> np.ndarray:
        """Two-link Laplacian (second form: two one-link transports, no W) on slice t."""
        U = self._c128(U)
        psi = self._c128(psi)
        g, L = self._geom(U)
        assert psi.shape == (L[2], L[1], L[0], 3)
        out = np.empty_like(psi)
        self.lib.or_lap_oneplusone(g, _ptr(U), int(t), _ptr(psi), _ptr(out))
        return out

    def smear(self, W: np.ndarray, t: int, n: int, sigma: float, psi: np.ndarray) -> np.ndarray:
        """(1 + (sigma/n) Lap)^n psi on slice t; returns a new array."""
        W = self._c128(W)
        out = self._c128(psi).copy()
        g, L = self._geom(W)
        assert out.shape == (L[2], L[1], L[0], 3)
        self.lib.or_smear(g, _ptr(W), int(t), int(n), float(sigma), _ptr(out))
        return out

    def smear_batch(self, W: np.ndarray, t_of_rhs, n: int, sigma: float, psi: np.ndarray) -> np.ndarray:
        W = self._c128(W)
        out = self._c128(psi).copy()
        g, L = self._geom(W)
        ts = np.ascontiguousarray(t_of_rhs, dtype=np.int32)
        assert out.shape == (len(ts), L[2], L[1], L[0], 3)
        self.lib.or_smear_batch(g, _ptr(W), len(ts), _ptr(ts), int(n), float(sigma), _ptr(out))
        return out

    # -- one-link operators (Sec. 2: H, nabla^2 = H - 6, eq. gsmear)
    def _slice_op(self, fn, U, t, psi):
        U = self._c128(U)
        psi = self._c128(psi)
        g, L = self._geom(U)
        assert U.shape[4:] == (4, 3, 3) and psi.shape == (L[2], L[1], L[0], 3)
        out = np.empty_like(psi)
        fn(g, _ptr(U), int(t), _ptr(psi), _ptr(out))
        return out

    def hop_onelink(self, U: np.ndarray, t: int, psi: np.ndarray) -> np.ndarray:
        """H psi on slice t."""
        return self._slice_op(self.lib.or_hop_onelink, U, t, psi)

    def laplacian_onelink(self, U: np.ndarray, t: int, psi: np.ndarray) -> np.ndarray:
        """nabla^2 psi = (H - 6) psi on slice t."""
        return self._slice_op(self.lib.or_lap_onelink, U, t, psi)

    def gsmear_hop(self, U: np.ndarray, t: int, n: int, alpha: float, psi: np.ndarray) -> np.ndarray:
        """(1 + alpha H)^n psi on slice t (eq. gsmear without C)."""
        U = self._c128(U)
        out = self._c128(psi).copy()
        g, L = self._geom(U)
        assert out.shape == (L[2], L[1], L[0], 3)
        self.lib.or_gsmear_hop(g, _ptr(U), int(t), int(n), float(alpha), _ptr(out))
        return out

    def smear_onelink(self, U: np.ndarray, t: int, n: int, sigma: float, psi: np.ndarray) -> np.ndarray:
        """(1 + (sigma/n) nabla^2)^n psi on slice t."""
        U = self._c128(U)
        out = self._c128(psi).copy()
        g, L = self._geom(U)
        assert out.shape == (L[2], L[1], L[0], 3)
        self.lib.or_smear_onelink(g, _ptr(U), int(t), int(n), float(sigma), _ptr(out))
        return out

    def smear_onelink_batch(self, U: np.ndarray, t_of_rhs, n: int, sigma: float, psi: np.ndarray) -> np.ndarray:
        U = self._c128(U)
        out = self._c128(psi).copy()
        g, L = self._geom(U)
        ts = np.ascontiguousarray(t_of_rhs, dtype=np.int32)
        assert out.shape == (len(ts), L[2], L[1], L[0], 3)
        self.lib.or_smear_onelink_batch(g, _ptr(U), len(ts), _ptr(ts), int(n), float(sigma), _ptr(out))
        return out

    # -- reductions
    def norm2(self, psi: np.ndarray) -> float:
        psi = self._c128(psi)
        return float(self.lib.or_norm2(psi.size // 3, _ptr(psi)))

    def dot(self, phi: np.ndarray, psi: np.ndarray) -> complex:
        phi = self._c128(phi)
        psi = self._c128(psi)
        assert phi.shape == psi.shape
        re, im = ctypes.c_double(), ctypes.c_double()
        self.lib.or_dot(psi.size // 3, _ptr(phi), _ptr(psi), ctypes.byref(re), ctypes.byref(im))
        return complex(re.value, im.value)

    def site_norms(self, psi: np.ndarray) -> np.ndarray:
        psi = self._c128(psi)
        out = np.empty(psi.shape[:-1], np.float64)
        self.lib.or_site_norms(psi.size // 3, _ptr(psi), _ptr(out))
        return out


_default: Oracle | None = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
