"""Two-link staggered Gaussian smearing on AMD Instinct MI355X (gfx950).

Thin Python binding over ``libtwolink.so`` (C ABI in ``include/twolink.h``).
It only marshals arguments: every step of the smearing path runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.

Method: Gottlieb, Jeong, Strelchenko, "Two-link Staggered Quark Smearing in
QUDA", arXiv:2301.05518 -- two-link product (Sec. 2), two-link Laplacian
(eq. tlLapl1), smearing (eq. tlSmear), precomputed two-links reused for every
source and sink (Sec. 3).

Layouts (torch tensors on the context's device):
  gauge field U  complex128 [Lt][Lz][Ly][Lx][4][3][3]
  colour vectors complex128 [n_rhs][Lz][Ly][Lx][3]
  two-link field uint8 buffer of ``twolinks_bytes(L, prec, n_slices)`` bytes

Precisions: "f64", "f32", "f16s", "bf16" (colour vectors and two-links), each
also as "<prec>-w12": two-links stored as their first two rows only (12 reals),
the third rebuilt in the kernels, valid for SU(3) gauge links only.  A suffix
"-onelink" (after "-w12" if both) selects one-link Gaussian smearing (Sec. 2):
the field then comes from Context.pack_links and the operators hop one site
(nabla^2 = H - 6, 0 <= sigma/n <= 1/6).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Sequence

from . import _lib
from ._lib import PREC, TL_AUTOTUNE, TL_GRAPH, TL_ONE_STEP, TL_ONELINK, TL_PLAIN, TL_W12, TwolinkError  # noqa: F401

__all__ = ["Context", "Job", "Plan", "TwolinkError", "PREC", "TL_PLAIN", "TL_GRAPH", "TL_AUTOTUNE", "TL_ONE_STEP", "TL_W12", "TL_ONELINK",
           "twolinks_bytes", "library"]


def library():
    return _lib.load()


def _geom(L: Sequence[int]) -> _lib.Geom:
    g = _lib.Geom()
    for i in range(4):
        g.L[i] = int(L[i])
    return g


def _prec(p) -> int:
    if isinstance(p, str):
        if p not in PREC:
            raise ValueError(f"unknown precision {p!r}; one of {list(PREC)}")
        return PREC[p]
    return int(p)


def _check_w_format(W, prec, name: str):
    """A two-link buffer built by Context.build_twolinks remembers its format; a mismatch
    (other precision, or 12- vs 18-real storage) would be read as garbage."""
    built = getattr(W, "_tl_prec", None)
    if built is not None and built != _prec(prec):
        raise ValueError(f"{name} was built with precision code {built}, used with {_prec(prec)}")


def _i32(values):
    if values is None:
        return None, 0
    arr = (ctypes.c_int32 * len(values))(*[int(v) for v in values])
    return arr, len(values)


def twolinks_bytes(L: Sequence[int], prec="f32", n_slices: int | None = None) -> int:
    n = int(L[3]) if n_slices is None else int(n_slices)
    return int(_lib.load().tl_twolinks_bytes(ctypes.byref(_geom(L)), _prec(prec), n))


def _ptr(t) -> int:
    return int(t.data_ptr())


def _need(t, dtype: str, numel: int, name: str, at_least: bool = False, device: int | None = None):
    """The C ABI takes raw pointers: check dtype, device, layout and size here."""
    import torch
    want = getattr(torch, dtype)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    if t.dtype != want:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if (t.numel() < numel) if at_least else (t.numel() != numel):
        raise ValueError(f"{name} has {t.numel()} elements, expected {'>= ' if at_least else ''}{numel}")


def _v3(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2])


@dataclass
class Job:
    """One lattice's right-hand sides: psi [n_rhs][Lz][Ly][Lx][3] complex128, smeared in place."""
    L: tuple
    W: object                     # uint8 tensor from Context.build_twolinks
    t_of_rhs: Sequence[int]
    psi: object
    w_slices: Sequence[int] | None = None


class Context:
    """A library context on one device, queueing on a torch stream (default: the current one)."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        if device >= 0:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            sp = ctypes.c_void_p(stream.cuda_stream)
            self._torch_stream = stream
        else:
            sp = ctypes.c_void_p(None)
            self._torch_stream = None
        rc = self.lib.tl_create(ctypes.byref(h), int(device), sp)
        if rc != 0:
            raise TwolinkError(rc, self.lib.tl_last_error(None).decode())
        self.h = h

    # -- plumbing
    def _check(self, rc: int):
        if rc != 0:
            raise TwolinkError(rc, self.lib.tl_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.tl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        self._check(self.lib.tl_sync(self.h))

    def stats(self) -> dict:
        """The context's counters: graphs captured, tuning sweeps and cache hits, kept tl_smear plans reused."""
        st = _lib.CtxStats()
        self._check(self.lib.tl_get_stats(self.h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in st._fields_}

    def set_stream(self, stream):
        """Queue later work on a torch stream of the context's device (tl_set_stream: the new
        stream first waits for what the context queued on the old one)."""
        self._check(self.lib.tl_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))
        self._torch_stream = stream

    def _torch_device(self):
        import torch
        return torch.device("cuda", self.device)

    # -- the path
    def build_twolinks(self, L, U, prec="f32", slices=None, W=None):
        """Two-link field W_mu(x) = U_mu(x) U_mu(x+mu^) (FP64 math, stored in prec)."""
        return self._links(self.lib.tl_build_twolinks, L, U, prec, slices, W)

    def pack_links(self, L, U, prec="f32-onelink", slices=None, W=None):
        """One-link field U_mu(x) for one-link smearing (prec must end in "-onelink")."""
        return self._links(self.lib.tl_pack_links, L, U, prec, slices, W)

    def _links(self, fn, L, U, prec, slices, W):
        import torch
        n = int(L[3]) if slices is None else len(slices)
        nbytes = twolinks_bytes(L, prec, n)
        _need(U, "complex128", _v3(L) * int(L[3]) * 36, "U", device=self.device)
        if W is None:
            W = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self._torch_device())
        _need(W, "uint8", nbytes, "W", at_least=True, device=self.device)
        arr, ns = _i32(slices)
        self._check(fn(self.h, ctypes.byref(_geom(L)), ctypes.c_void_p(_ptr(U)),
                       arr, ns if slices is not None else 0, _prec(prec), ctypes.c_void_p(_ptr(W))))
        W._tl_prec = _prec(prec)
        return W

    def laplacian(self, L, W, prec, t, psi_in, out=None, w_slices=None):
        import torch
        _need(psi_in, "complex128", _v3(L) * 3, "psi_in", device=self.device)
        if out is None:
            out = torch.empty_like(psi_in)
        _need(out, "complex128", _v3(L) * 3, "out", device=self.device)
        nw = int(L[3]) if w_slices is None else len(w_slices)
        _check_w_format(W, prec, "W")
        _need(W, "uint8", twolinks_bytes(L, prec, nw), "W", at_least=True, device=self.device)
        arr, n = _i32(w_slices)
        self._check(self.lib.tl_laplacian(self.h, ctypes.byref(_geom(L)), ctypes.c_void_p(_ptr(W)), arr, n,
                                          _prec(prec), int(t), ctypes.c_void_p(_ptr(psi_in)),
                                          ctypes.c_void_p(_ptr(out))))
        return out

    def _jobs(self, jobs: Sequence[Job], prec):
        arr = (_lib.Job * len(jobs))()
        keep = []
        for i, j in enumerate(jobs):
            _need(j.psi, "complex128", len(j.t_of_rhs) * _v3(j.L) * 3, f"jobs[{i}].psi", device=self.device)
            nw = int(j.L[3]) if j.w_slices is None else len(j.w_slices)
            _check_w_format(j.W, prec, f"jobs[{i}].W")
            _need(j.W, "uint8", twolinks_bytes(j.L, prec, nw), f"jobs[{i}].W", at_least=True, device=self.device)
            ts, nt = _i32(j.t_of_rhs)
            ws, nw = _i32(j.w_slices)
            keep += [ts, ws]
            arr[i].g = _geom(j.L)
            arr[i].W = _ptr(j.W)
            arr[i].w_slices = ws
            arr[i].n_w_slices = nw
            arr[i].n_rhs = nt
            arr[i].t_of_rhs = ts
            arr[i].psi = _ptr(j.psi)
        return arr, keep

    def smear(self, jobs: Sequence[Job], n_steps: int, sigma: float, prec="f32", flags: int = 0):
        arr, keep = self._jobs(jobs, prec)
        self._check(self.lib.tl_smear(self.h, arr, len(jobs), int(n_steps), float(sigma), _prec(prec),
                                      int(flags)))

    def stream_time(self, buf, n_in: int = 4, kinds: int = 2, grid: int = 0, reps: int = 5) -> float:
        """ms per launch of the streaming probe over a uint8 device buffer (tl_stream_time)."""
        _need(buf, "uint8", 1, "buf", at_least=True, device=self.device)
        ms = ctypes.c_double()
        self._check(self.lib.tl_stream_time(self.h, ctypes.c_void_p(_ptr(buf)), buf.numel(), int(n_in), int(kinds),
                                            int(grid), int(reps), ctypes.byref(ms)))
        return ms.value

    def plan(self, jobs: Sequence[Job], n_steps: int, sigma: float, prec="f32", flags: int = 0) -> "Plan":
        return Plan(self, jobs, n_steps, sigma, prec, flags)

    def reduce(self, kind: str, psi, phi=None, out=None):
        """FP64 reductions of complex128 fields [n_rhs][...][3]: 'norm2', 'dot' (<phi, psi>), 'site_norm'."""
        return self._reduce(self.lib.tl_reduce, kind, psi, phi, out)

    def reduce_noalloc(self, kind: str, psi, phi=None, out=None):
        """As reduce, through tl_reduce_noalloc (no library allocation; pass `out`, a float64 tensor
        of n_rhs, 2 n_rhs or n_rhs * n_sites entries, to allocate nothing here either)."""
        return self._reduce(self.lib.tl_reduce_noalloc, kind, psi, phi, out)

    def _reduce(self, fn, kind: str, psi, phi, out):
        import torch
        k = {"norm2": 0, "dot": 1, "site_norm": 2}[kind]
        n_rhs = psi.shape[0]
        n_sites = psi[0].numel() // 3
        _need(psi, "complex128", n_rhs * n_sites * 3, "psi", device=self.device)
        if k == 1:
            if phi is None or phi.shape != psi.shape:
                raise ValueError("dot needs phi of psi's shape")
            _need(phi, "complex128", n_rhs * n_sites * 3, "phi", device=self.device)
        size = {0: n_rhs, 1: 2 * n_rhs, 2: n_rhs * n_sites}[k]
        if out is None:
            out = torch.empty(size, dtype=torch.float64, device=psi.device)
        _need(out, "float64", size, "out", device=self.device)
        self._check(fn(self.h, k, n_sites, n_rhs, ctypes.c_void_p(_ptr(psi)),
                       ctypes.c_void_p(_ptr(phi) if phi is not None else None),
                       ctypes.c_void_p(_ptr(out))))
        if k == 1:
            return torch.complex(out[0::2], out[1::2])
        if k == 2:
            return out.view(psi.shape[:-1])
        return out


class Plan:
    """Resident smearing plan: packed fields, work list, tuned tiling, optional HIP graph."""

    def __init__(self, ctx: Context, jobs, n_steps, sigma, prec, flags):
        self.ctx = ctx
        self.jobs = list(jobs)
        self.prec = prec
        arr, self._keep = ctx._jobs(self.jobs, prec)
        self._arr = arr
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.tl_plan_create(ctx.h, arr, len(self.jobs), int(n_steps), float(sigma), _prec(prec),
                                          int(flags), ctypes.byref(h)))
        self.h = h
        self.n_rhs = sum(len(j.t_of_rhs) for j in self.jobs)

    def load(self):
        self.ctx._check(self.ctx.lib.tl_plan_load(self.h))

    def run(self):
        self.ctx._check(self.ctx.lib.tl_plan_run(self.h))

    def store(self):
        self.ctx._check(self.ctx.lib.tl_plan_store(self.h))

    def reduce(self, kind: str, other: "Plan | None" = None):
        """FP64 reductions of the resident fields, RHS in job order ('dot' is <other, self>)."""
        import torch
        k = {"norm2": 0, "dot": 1, "site_norm": 2}[kind]
        sites = sum(j.psi[0].numel() // 3 * len(j.t_of_rhs) for j in self.jobs)
        size = {0: self.n_rhs, 1: 2 * self.n_rhs, 2: sites}[k]
        out = torch.empty(size, dtype=torch.float64, device=self.ctx._torch_device())
        self.ctx._check(self.ctx.lib.tl_plan_reduce(self.h, k, other.h if other is not None else None,
                                                    ctypes.c_void_p(_ptr(out))))
        if k == 1:
            return torch.complex(out[0::2], out[1::2])
        return out

    def time(self, reps: int = 3) -> float:
        ms = ctypes.c_double()
        self.ctx._check(self.ctx.lib.tl_plan_time(self.h, int(reps), ctypes.byref(ms)))
        return ms.value

    def info(self) -> dict:
        inf = _lib.PlanInfo()
        self.ctx._check(self.ctx.lib.tl_plan_get_info(self.h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in inf._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tl_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
