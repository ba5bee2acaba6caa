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


def tol(prec: str, n: int) -> float:
    if prec == "f64":
        return 1e-12
    return 2.0 * (n + 1) * UNIT_ROUNDOFF[prec]


def tol_lap(prec: str) -> float:
    return 1e-14 if prec == "f64" else 16.0 * UNIT_ROUNDOFF[prec]


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
