"""Test-side numpy readers of the packed storage formats of libtwolink.

Written from the format description (planes of fixed-width words per site,
reals in (re, im) order; F16S = half times an FP32 per-site scale), not from
the library's code, so that the GPU's stored two-link field can be compared
with the oracle's product element by element, and the colour-vector storage
rounding can be checked bit for bit.
"""
from __future__ import annotations

import numpy as np

W_BYTES = {"f64": 144, "f32": 72, "f16s": 40, "bf16": 36,
           "f64-w12": 96, "f32-w12": 48, "f16s-w12": 24, "bf16-w12": 24}
V_BYTES = {"f64": 48, "f32": 24, "f16s": 16, "bf16": 12}


def padded(v3: int) -> int:
    return (v3 + 63) // 64 * 64


def _bf16_to_f32(u16: np.ndarray) -> np.ndarray:
    return (u16.astype(np.uint32) << 16).view(np.float32)


def decode_twolinks(raw: np.ndarray, L, prec: str, n_slots: int) -> np.ndarray:
    """Packed two-link bytes -> complex128 [slot][Lz][Ly][Lx][mu][3][3].

    Twelve-real forms ("<prec>-w12") hold rows 0 and 1 only; row 2 comes back as NaN."""
    Lx, Ly, Lz = L[:3]
    v3 = Lx * Ly * Lz
    vp = padded(v3)
    wb = W_BYTES[prec]
    raw = np.ascontiguousarray(raw[: n_slots * 3 * vp * wb]).reshape(n_slots, 3, vp * wb)
    reals = np.empty((n_slots, 3, v3, 18), np.float64)
    for s in range(n_slots):
        for mu in range(3):
            blk = raw[s, mu]
            if prec == "f64":
                planes = blk.view(np.float64).reshape(9, vp, 2)[:, :v3, :]
                reals[s, mu] = planes.transpose(1, 0, 2).reshape(v3, 18)
            elif prec == "f32":
                p4 = blk[: 64 * vp].view(np.float32).reshape(4, vp, 4)[:, :v3, :].transpose(1, 0, 2).reshape(v3, 16)
                p2 = blk[64 * vp: 72 * vp].view(np.float32).reshape(vp, 2)[:v3]
                reals[s, mu] = np.concatenate([p4, p2], axis=1)
            elif prec == "bf16":
                p8 = blk[: 32 * vp].view(np.uint16).reshape(2, vp, 8)[:, :v3, :].transpose(1, 0, 2).reshape(v3, 16)
                p2 = blk[32 * vp: 36 * vp].view(np.uint16).reshape(vp, 2)[:v3]
                reals[s, mu] = _bf16_to_f32(np.concatenate([p8, p2], axis=1))
            elif prec.endswith("-w12"):
                base = prec[:-4]
                reals[s, mu, :, 12:] = np.nan
                if base == "f64":
                    reals[s, mu, :, :12] = blk.view(np.float64).reshape(6, vp, 2)[:, :v3, :].transpose(1, 0, 2).reshape(v3, 12)
                elif base == "f32":
                    reals[s, mu, :, :12] = blk.view(np.float32).reshape(3, vp, 4)[:, :v3, :].transpose(1, 0, 2).reshape(v3, 12)
                else:
                    p8 = blk[: 16 * vp].view(np.uint16).reshape(vp, 8)[:v3]
                    p4 = blk[16 * vp: 24 * vp].view(np.uint16).reshape(vp, 4)[:v3]
                    bits = np.concatenate([p8, p4], axis=1)
                    if base == "bf16":
                        reals[s, mu, :, :12] = _bf16_to_f32(bits)
                    else:
                        reals[s, mu, :, :12] = bits.view(np.float16).astype(np.float64)
            elif prec == "f16s":
                p8 = blk[: 32 * vp].view(np.float16).reshape(2, vp, 8)[:, :v3, :].transpose(1, 0, 2).reshape(v3, 16)
                tail = blk[32 * vp: 40 * vp].reshape(vp, 8)[:v3]
                h2 = tail[:, :4].copy().view(np.float16).reshape(v3, 2)
                scale = tail[:, 4:].copy().view(np.float32).reshape(v3, 1)
                reals[s, mu] = np.concatenate([p8, h2], axis=1).astype(np.float32) * scale
            else:
                raise ValueError(prec)
    c = reals[..., 0::2] + 1j * reals[..., 1::2]          # [slot][mu][v3][9]
    c = c.transpose(0, 2, 1, 3).reshape(n_slots, Lz, Ly, Lx, 3, 3, 3)
    return c


def f32_to_bf16_rne(x: np.ndarray) -> np.ndarray:
    """float32 -> bf16 bits with round-to-nearest-even (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def storage_round_vectors(psi: np.ndarray, prec: str) -> np.ndarray:
    """What storing complex128 colour vectors [..][3] in `prec` and reading them back gives."""
    re = np.stack([psi.real, psi.imag], axis=-1).reshape(psi.shape[:-1] + (6,))
    if prec == "f64":
        out = re
    elif prec == "f32":
        out = re.astype(np.float32).astype(np.float64)
    elif prec == "bf16":
        out = _bf16_to_f32(f32_to_bf16_rne(re.astype(np.float32))).astype(np.float64)
    elif prec == "f16s":
        f = re.astype(np.float32)
        mx = np.max(np.abs(f), axis=-1, keepdims=True)
        pre = np.where(mx < np.float32(2.0 ** -126), np.float32(2.0 ** 64), np.float32(1.0))
        safe = np.where(mx > 0, mx * pre, np.float32(1.0))
        inv = np.where(mx > 0, np.float32(1.0) / safe, np.float32(0.0)).astype(np.float32)
        h = ((f * pre) * inv).astype(np.float16)
        out = (h.astype(np.float32) * mx).astype(np.float64)
    else:
        raise ValueError(prec)
    out = out.reshape(psi.shape[:-1] + (3, 2))
    return out[..., 0] + 1j * out[..., 1]


# ---------------------------------------------------------------- link storage model

def _f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, np.float64).astype(np.float32)


def _bf16_round(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 (nearest) -> bf16 (nearest even), back to float64."""
    return _bf16_to_f32(f32_to_bf16_rne(_f32(x))).astype(np.float64)


def _half_round(x: np.ndarray) -> np.ndarray:
    """FP64 -> IEEE half (nearest even, one rounding), back to float64."""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def storage_round_links(m: np.ndarray, prec: str) -> np.ndarray:
    """What storing complex128 3x3 link matrices [..][3][3] in `prec` and reading them back gives.

    From the format description: FP32 and BF16 round every real to nearest (BF16 through
    FP32); F16S divides the 18 reals of a matrix by s = max |real| (rounded to FP32), forms the
    quotient in FP64, rounds it once to half, and decodes half * s in FP32.  The
    twelve-real forms ("<prec>-w12") store rows 0 and 1 (16-bit ones with no scale) and the
    reader rebuilds row 2 as conj(row0 x row1), evaluated here in FP64."""
    base, w12 = (prec[:-4], True) if prec.endswith("-w12") else (prec, False)
    re = np.stack([m.real, m.imag], axis=-1).reshape(m.shape[:-2] + (18,))
    if w12:
        rows = re[..., :12]
        if base == "f64":
            r = rows.copy()
        elif base == "f32":
            r = _f32(rows).astype(np.float64)
        elif base == "bf16":
            r = _bf16_round(rows)
        elif base == "f16s":
            r = _half_round(rows)
        else:
            raise ValueError(prec)
        c = (r[..., 0::2] + 1j * r[..., 1::2]).reshape(m.shape[:-2] + (2, 3))
        a, b = c[..., 0, :], c[..., 1, :]
        third = np.conj(np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                                  a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                                  a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1))
        return np.concatenate([c, third[..., None, :]], axis=-2)
    if base == "f64":
        out = re
    elif base == "f32":
        out = _f32(re).astype(np.float64)
    elif base == "bf16":
        out = _bf16_round(re)
    elif base == "f16s":
        s = _f32(np.max(np.abs(re), axis=-1, keepdims=True))
        inv = np.where(s > 0, 1.0 / np.where(s > 0, s.astype(np.float64), 1.0), 0.0)
        h = (re * inv).astype(np.float16)
        out = (h.astype(np.float32) * s).astype(np.float64)
    else:
        raise ValueError(prec)
    c = out[..., 0::2] + 1j * out[..., 1::2]
    return c.reshape(m.shape)


def ulp(x: np.ndarray, fmt: str) -> np.ndarray:
    """Spacing of the storage format's numbers at magnitude |x| (float64 array)."""
    p, emin = {"f32": (23, -126), "bf16": (7, -126), "half": (10, -14)}[fmt]
    ax = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.where(ax > 0, np.maximum(e, emin), emin)
    return np.exp2(e - p)
