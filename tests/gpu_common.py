"""Shared helpers of the GPU tests: run the HIP path through the C ABI, run the oracle."""
from __future__ import annotations

import sys

import numpy as np

from oracle import checks

# Tolerances (max-rel and L2-rel against the FP64 oracle).
#   FP64: the target of the method, 1e-12.
#   Mixed precision: n steps, each a contraction for sigma/n <= 2/3, each
#   storing the vectors once with relative rounding error <= u after one
#   rounding of the two-link field.  Worst case the errors add linearly,
#   (n + 1) u; rounding errors of independent sites and steps add like a
#   random walk, sqrt(n + 1) u.  The bar is 4 sqrt(n + 1) u with the storage
#   unit roundoff u = 2^-24 (FP32), 2^-11 relative to the per-site maximum
#   (F16S), 2^-8 (BF16); a wrong hop, sign or index gives O(1) errors.
UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16s": 2.0 ** -11, "bf16": 2.0 ** -8}


def tol(prec: str, n: int) -> float:
    if prec == "f64":
        return 1e-12
    return 4.0 * (n + 1) ** 0.5 * UNIT_ROUNDOFF[prec]


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
