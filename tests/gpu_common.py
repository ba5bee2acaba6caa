"""Shared helpers of the GPU tests: run the HIP path through the C ABI, run the oracle."""
from __future__ import annotations

import sys

import numpy as np

from oracle import checks

# Tolerances (max-rel and L2-rel against the FP64 oracle).
#   FP64: the target of the method, 1e-12.
#   Mixed precision, n smearing steps: each step is a contraction for
#   sigma/n <= 2/3 (|alpha| + 6 beta = 1 and |W| = 1), stores the vectors
#   once (relative error <= u) and adds FP32 arithmetic and two-link
#   rounding errors of about u more, so the error after n steps is at most
#   about 2 (n + 1) u times the initial size.  Smooth fields (wall sources)
#   accumulate their rounding errors coherently, so the linear bound is
#   the right one.  u = 2^-24 (FP32), 2^-11 relative to the per-site
#   maximum (F16S), 2^-8 (BF16).  Wrong hops, signs or indices give O(1)
#   errors; the single-application Laplacian bound (16 u, allowing a
#   four-fold cancellation between -6 psi and the hops) pins those tightly.
UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16s": 2.0 ** -11, "bf16": 2.0 ** -8}

# Twelve-real two-links ("<prec>-w12"): the rebuilt third row inherits the
# rounding of the two stored unit rows (about u each through the cross
# product) plus four rounded operations per entry, up to about 4u, so the
# two-link term of the per-step budget grows from u to about 4u: 2 u per
# step becomes 5 u (n-step bound 5 (n + 1) u), and the Laplacian bound grows
# by the same factor 2.5.  FP64 keeps its 1e-12 target.
W12_FACTOR = 2.5


def _split(prec: str):
    return (prec[:-4], True) if prec.endswith("-w12") else (prec, False)


def tol(prec: str, n: int) -> float:
    base, w12 = _split(prec)
    if base == "f64":
        return 1e-12
    return 2.0 * (n + 1) * UNIT_ROUNDOFF[base] * (W12_FACTOR if w12 else 1.0)


def tol_lap(prec: str) -> float:
    base, w12 = _split(prec)
    return 1e-14 if base == "f64" else 16.0 * UNIT_ROUNDOFF[base] * (W12_FACTOR if w12 else 1.0)


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def errors(out, ref):
    return checks.max_rel(out, ref), checks.l2_rel(out, ref)


def gpu_smear(ctx, lattices, n, sigma, prec, flags=0, w_slices=None, return_jobs=False):
    """lattices: list of (L, U numpy, t_of_rhs, psi numpy). Returns smeared psi per lattice (numpy)."""
    import torch
    import paper_2301_05518_amd as tl
    jobs = []
    for L, U, ts, psi in lattices:
        W = ctx.build_twolinks(L, to_dev(U), prec, slices=w_slices)
        jobs.append(tl.Job(tuple(L), W, list(ts), to_dev(psi), w_slices))
    ctx.smear(jobs, n, sigma, prec, flags)
    torch.cuda.synchronize()
    outs = [j.psi.cpu().numpy() for j in jobs]
    return (outs, jobs) if return_jobs else outs
