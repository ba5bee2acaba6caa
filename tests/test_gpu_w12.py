"""GPU parity of the twelve-real two-link storage ("<prec>-w12"): two rows of each
W_mu(x) stored, the third rebuilt in the kernels (valid for SU(3) links, Sec. 2).

Against the FP64 oracle, which always uses the full product; the stored rows are
also compared with the eighteen-real build bit for bit where both round the same way.
"""
import numpy as np
import pytest

from paper_2301_05518_amd import synth
from tests import packed
from tests.gpu_common import errors, gpu_smear, log, to_dev, tol, tol_lap

pytestmark = pytest.mark.gpu

W12 = ["f64-w12", "f32-w12", "f16s-w12", "bf16-w12"]


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


def rng(k):
    return np.random.default_rng([7117, k])


def haar(L, seed):
    return synth.gauge_field(L, "haar", 4100 + seed)


@pytest.mark.parametrize("prec", W12)
def test_build_stores_two_rows(ctx, orc, torch, prec):
    L = (10, 6, 7, 2)
    log(f"build {prec} {L}")
    U = haar(L, 1)
    Ud = to_dev(U)
    got = packed.decode_twolinks(ctx.build_twolinks(L, Ud, prec).cpu().numpy(), L, prec, L[3])
    assert np.isnan(got[..., 2, :]).all()
    ref = orc.build_twolinks(U)
    base = prec[:-4]
    bound = {"f64": 1e-14, "f32": 2.0 ** -24, "f16s": 2.0 ** -11 * 1.01, "bf16": 2.0 ** -8 * 1.01}[base]
    d = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))[..., :2, :].max()
    assert d <= bound, d
    if base != "f16s":   # same rounding as the eighteen-real form (F16S there carries a scale)
        full = packed.decode_twolinks(ctx.build_twolinks(L, Ud, base).cpu().numpy(), L, base, L[3])
        assert np.array_equal(got[..., :2, :], full[..., :2, :])


@pytest.mark.parametrize("prec", W12)
def test_laplacian_w12(ctx, orc, torch, prec):
    for k, L in enumerate([(4, 4, 4, 1), (17, 9, 5, 2), (2, 3, 5, 1), (8, 8, 8, 2)]):
        U = haar(L, 10 + k)
        W = ctx.build_twolinks(L, to_dev(U), prec)
        Wo = orc.build_twolinks(U)
        for t in range(L[3]):
            psi = synth.random_field(rng(10 * k + t), (L[2], L[1], L[0], 3))
            out = ctx.laplacian(L, W, prec, t, to_dev(psi)).cpu().numpy()
            ref = orc.laplacian(Wo, t, psi)
            mr, l2 = errors(out, ref)
            log(f"laplacian {prec} {L} t={t}: max-rel {mr:.3e}")
            assert mr < tol_lap(prec) and l2 < tol_lap(prec)


@pytest.mark.parametrize("prec", W12)
def test_smear_w12(ctx, orc, torch, prec):
    L = (16, 16, 16, 2)
    n, sigma = 40, 5.0
    U = haar(L, 20)
    psi = np.stack([synth.point_source(L[:3], c) for c in range(3)] + [synth.z2_source(rng(21), L[:3], 1)])
    ts = [0, 0, 0, 1]
    ref = orc.smear_batch(orc.build_twolinks(U), ts, n, sigma, psi)
    out = gpu_smear(ctx, [(L, U, ts, psi)], n, sigma, prec, 6)[0]
    mr, l2 = errors(out, ref)
    log(f"16^3 {prec} N={n}: max-rel {mr:.3e} l2-rel {l2:.3e} (bar {tol(prec, n):.2e})")
    assert mr < tol(prec, n) and l2 < tol(prec, n)


VARIANT_TILES = ["0,64,1,0", "0,128,3,256", "1,64,4,0", "2,64,4,0", "2,128,3,0", "3,64,2,0", "3,128,5,0",
                 "4,64,1,0", "4,256,3,16", "5,512,16,0", "5,256,3,0", "5,256,5,0,1", "6,512,16,0",
                 "6,256,3,0", "6,512,1,8", "6,256,2,0,1", "7,512,16,0", "7,256,3,0", "7,512,1,8", "7,256,2,0,1",
                 "7,512,16,0,1,1", "5,256,5,0,0,1", "2,64,4,0,1,1"]


@pytest.mark.parametrize("prec", W12)
def test_step_variants_bit_identical_w12(ctx, orc, torch, prec, monkeypatch):
    """Every variant rebuilds the third row with the same operations (variant 6 after its
    barrier), so all tilings give the same bits."""
    cases = [((10, 6, 13, 3), [0, 2, 0, 0]), ((8, 4, 1, 2), [1])]
    if prec == "f64-w12":
        cases = [((10, 6, 13, 3), [0, 2]), ((8, 4, 1, 2), [1])]   # LDS kernels: FP64 groups of one RHS
    lats = []
    for k, (L, ts) in enumerate(cases):
        U = haar(L, 30 + k)
        psi = synth.random_field(rng(30 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    outs = {}
    for tile in VARIANT_TILES:
        monkeypatch.setenv("TL_TILE", tile)
        log(f"variants {prec}: tile {tile}")
        outs[tile] = gpu_smear(ctx, lats, 7, 2.5, prec)
    for tile in VARIANT_TILES:
        for a, b in zip(outs[tile], outs[VARIANT_TILES[0]]):
            assert np.array_equal(a, b), tile
    for (L, U, ts, psi), o in zip(lats, outs[VARIANT_TILES[0]]):
        ref = orc.smear_batch(orc.build_twolinks(U), ts, 7, 2.5, psi)
        mr, l2 = errors(o, ref)
        assert mr < tol(prec, 7) and l2 < tol(prec, 7)


def test_fp64_w12_close_to_full(ctx, torch):
    """FP64: rebuilding the third row changes the result only at rounding level."""
    L = (12, 12, 12, 1)
    U = haar(L, 40)
    psi = synth.random_field(rng(40), (3, L[2], L[1], L[0], 3))
    a = gpu_smear(ctx, [(L, U, [0, 0, 0], psi)], 20, 3.0, "f64")[0]
    b = gpu_smear(ctx, [(L, U, [0, 0, 0], psi)], 20, 3.0, "f64-w12")[0]
    mr, _ = errors(b, a)
    assert mr < 1e-13


def test_format_mismatch_is_refused(ctx, torch):
    import paper_2301_05518_amd as tl
    L = (8, 8, 8, 1)
    U = to_dev(haar(L, 50))
    psi = to_dev(synth.random_field(rng(50), (1, 8, 8, 8, 3)))
    W = ctx.build_twolinks(L, U, "f32")
    with pytest.raises(ValueError, match="built with precision code"):
        ctx.smear([tl.Job(L, W, [0], psi)], 2, 1.0, "f32-w12")
    W12 = ctx.build_twolinks(L, U, "f32-w12")
    with pytest.raises(ValueError, match="built with precision code"):
        ctx.laplacian(L, W12, "f32", 0, psi[0])
