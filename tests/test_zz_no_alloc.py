"""tl_reduce_noalloc through the C ABI against tl_reduce: bit-identical FP64 results on two
calls in a row, the second smaller (the fixed partial-sum area keeps the first call's
contents), for every reduction kind; a size beyond the fixed area is refused."""
import numpy as np
import pytest

from paper_2301_05518_amd import synth
from tests.gpu_common import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2301_05518_amd as tl
    c = tl.Context(0)
    yield c
    c.close()


def fields(k, n_rhs, L3):
    rng = np.random.default_rng([6600, k])
    psi = synth.random_field(rng, (n_rhs, L3[2], L3[1], L3[0], 3))
    phi = synth.random_field(rng, (n_rhs, L3[2], L3[1], L3[0], 3))
    return to_dev(psi), to_dev(phi), psi, phi


def test_noalloc_equals_reduce_twice(ctx, orc, torch):
    # first call: 6 RHS of 40x36x30 sites (43200 sites, 11 blocks of partial sums each);
    # second: 2 RHS of 9x7x5 (one block) -- it must not read the first call's leftovers
    for k, (n_rhs, L3) in enumerate([(6, (40, 36, 30)), (2, (9, 7, 5))]):
        psi, phi, psi_h, phi_h = fields(k, n_rhs, L3)
        for kind in ("norm2", "dot", "site_norm"):
            other = phi if kind == "dot" else None
            want = ctx.reduce(kind, psi, other)
            size = {"norm2": n_rhs, "dot": 2 * n_rhs, "site_norm": psi.numel() // 3}[kind]
            out = torch.full((size,), float("nan"), dtype=torch.float64, device="cuda")
            got = ctx.reduce_noalloc(kind, psi, other, out=out)
            torch.cuda.synchronize()
            log(f"call {k} {kind}: {n_rhs} RHS of {L3}")
            assert not torch.isnan(out).any()
            assert torch.equal(got, want), kind
        n2 = ctx.reduce_noalloc("norm2", psi).cpu().numpy()
        for r in range(n_rhs):
            assert abs(n2[r] - orc.norm2(psi_h[r])) <= 1e-13 * n2[r]


def test_noalloc_full_area_then_refusal(ctx, torch):
    """The largest first pass the fixed area holds (1024 RHS x 64 blocks of 4096 sites, 12.9 GB
    of fields), then a size one block beyond it, refused before any device work."""
    import ctypes
    n_rhs, n_sites = 1024, 64 * 4096
    g = torch.Generator(device="cuda").manual_seed(6601)
    psi = torch.randn((n_rhs, n_sites, 3), dtype=torch.complex128, device="cuda", generator=g)
    log(f"full area: {n_rhs} RHS x {n_sites} sites")
    want = ctx.reduce("norm2", psi)
    got = ctx.reduce_noalloc("norm2", psi)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    lib = ctx.lib
    out = torch.empty(n_rhs, dtype=torch.float64, device="cuda")
    rc = lib.tl_reduce_noalloc(ctx.h, 0, n_sites + 1, n_rhs, ctypes.c_void_p(psi.data_ptr()), None,
                               ctypes.c_void_p(out.data_ptr()))
    assert rc == -2 and b"fixed area" in lib.tl_last_error(ctx.h)     # TL_ERR_SHAPE, nothing queued
    del psi
    torch.cuda.empty_cache()
