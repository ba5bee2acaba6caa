"""GPU parity of one-link Gaussian smearing (Sec. 2: H, nabla^2 = H - 6, eq. gsmear and the
rewriting with C' and alpha' that follows it), through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest

from oracle import checks
from paper_2301_05518_amd import synth
from tests import packed
from tests.gpu_common import errors, log, to_dev, tol, tol_lap

pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "f16s", "bf16"]


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
    return np.random.default_rng([9231, k])


def haar(L, seed):
    return synth.gauge_field(L, "haar", 5200 + seed)


def smear1(ctx, torch, lattices, n, sigma, prec, flags=0):
    """lattices: list of (L, U, t_of_rhs, psi); one-link smearing on the GPU."""
    import paper_2301_05518_amd as tl
    jobs = []
    for L, U, ts, psi in lattices:
        W = ctx.pack_links(L, to_dev(U), prec)
        jobs.append(tl.Job(tuple(L), W, list(ts), to_dev(psi)))
    ctx.smear(jobs, n, sigma, prec, flags)
    torch.cuda.synchronize()
    return [j.psi.cpu().numpy() for j in jobs]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32-w12"])
def test_pack_stores_the_links(ctx, torch, prec):
    L = (6, 5, 7, 2)
    U = haar(L, 1)
    got = packed.decode_twolinks(ctx.pack_links(L, to_dev(U), prec + "-onelink").cpu().numpy(), L, prec, L[3])
    ref = U[..., :3, :, :]
    rows = 2 if prec.endswith("-w12") else 3
    base = prec.split("-")[0]
    if base == "f64":
        assert np.array_equal(got[..., :rows, :], ref[..., :rows, :])
    else:
        bound = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8 * 1.01}[base]
        d = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))[..., :rows, :].max()
        assert d <= bound


@pytest.mark.parametrize("prec", PRECS + ["f32-w12"])
def test_laplacian_onelink(ctx, orc, torch, prec):
    for k, L in enumerate([(4, 4, 4, 1), (17, 9, 5, 2), (1, 2, 3, 1), (2, 3, 5, 1), (8, 8, 8, 2)]):
        U = haar(L, 10 + k)
        W = ctx.pack_links(L, to_dev(U), prec + "-onelink")
        for t in range(L[3]):
            psi = synth.random_field(rng(10 * k + t), (L[2], L[1], L[0], 3))
            out = ctx.laplacian(L, W, prec + "-onelink", t, to_dev(psi)).cpu().numpy()
            ref = orc.laplacian_onelink(U, t, psi)
            mr, l2 = errors(out, ref)
            log(f"one-link laplacian {prec} {L} t={t}: max-rel {mr:.3e}")
            assert mr < tol_lap(prec) and l2 < tol_lap(prec)


@pytest.mark.parametrize("prec", PRECS + ["f32-w12"])
def test_smear_onelink(ctx, orc, torch, prec):
    L = (16, 16, 16, 2)
    n, sigma = 40, 4.0
    U = haar(L, 20)
    psi = np.stack([synth.point_source(L[:3], c) for c in range(3)] + [synth.z2_source(rng(21), L[:3], 1)])
    ts = [0, 0, 0, 1]
    ref = orc.smear_onelink_batch(U, ts, n, sigma, psi)
    out = smear1(ctx, torch, [(L, U, ts, psi)], n, sigma, prec + "-onelink", 6)[0]
    mr, l2 = errors(out, ref)
    log(f"one-link 16^3 {prec} N={n}: max-rel {mr:.3e} l2-rel {l2:.3e} (bar {tol(prec, n):.2e})")
    assert mr < tol(prec, n) and l2 < tol(prec, n)


def test_gsmear_hopping_form(ctx, orc, torch):
    """C (1 + alpha H)^n psi (eq. gsmear) from the Laplacian-form kernels: sigma = n alpha', times (1 + 6 alpha)^n."""
    L = (10, 8, 12, 2)
    U = haar(L, 30)
    psi = synth.random_field(rng(30), (2, L[2], L[1], L[0], 3))
    n, alpha = 15, 0.08
    ap = alpha / (1.0 + 6.0 * alpha)
    out = smear1(ctx, torch, [(L, U, [0, 1], psi)], n, n * ap, "f64-onelink")[0] * (1.0 + 6.0 * alpha) ** n
    for r, t in enumerate([0, 1]):
        ref = orc.gsmear_hop(U, t, n, alpha, psi[r])
        assert checks.max_rel(out[r], ref) < 1e-12


def test_free_field_closed_form(ctx, torch):
    L3 = (12, 10, 8)
    U = synth.unit_gauge(L3 + (1,))
    psi = synth.point_source(L3, 1, (3, 2, 1))[None]
    out = smear1(ctx, torch, [(L3 + (1,), U, [0], psi)], 20, 2.5, "f64-onelink")[0][0]
    ref = np.zeros_like(out)
    ref[..., 1] = checks.free_kernel_onelink_dft(L3, 20, 2.5, (3, 2, 1))
    assert np.abs(out - ref).max() < 1e-13


TILES = ["0,64,1,0", "0,128,3,256", "0,256,2,0,1,1", "4,64,1,0", "4,256,3,16", "4,128,2,0,1,1", "0,64,5,7,0,1",
         "7,512,16,0", "7,256,3,0,1,1", "7,512,1,8,0,1", "7,64,4,0,1,0", "7,512,5,4,1,1"]


@pytest.mark.parametrize("prec", PRECS + ["bf16-w12"])
def test_variants_bit_identical_onelink(ctx, orc, torch, prec, monkeypatch):
    # every lattice has a full-row tiling (Ly with a divisor >= 4) for variant 7; FP64 groups
    # of one RHS there
    cases = [((10, 8, 13, 3), [0, 2, 0, 0]), ((5, 4, 2, 1), [0, 0]), ((3, 4, 1, 2), [1])]
    if prec == "f64":
        cases = [((10, 8, 13, 3), [0, 2]), ((5, 4, 2, 1), [0]), ((3, 4, 1, 2), [1])]
    lats = []
    for k, (L, ts) in enumerate(cases):
        U = haar(L, 40 + k)
        psi = synth.random_field(rng(40 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    outs = {}
    for tile in TILES:
        monkeypatch.setenv("TL_TILE", tile)
        outs[tile] = smear1(ctx, torch, lats, 7, 0.9, prec + "-onelink")
    for tile in TILES:
        for a, b in zip(outs[tile], outs[TILES[0]]):
            assert np.array_equal(a, b), tile
    for (L, U, ts, psi), o in zip(lats, outs[TILES[0]]):
        ref = orc.smear_onelink_batch(U, ts, 7, 0.9, psi)
        mr, l2 = errors(o, ref)
        assert mr < tol(prec, 7) and l2 < tol(prec, 7)


def test_refusals(ctx, torch, monkeypatch):
    import paper_2301_05518_amd as tl
    L = (8, 8, 8, 1)
    U = to_dev(haar(L, 50))
    psi = to_dev(synth.random_field(rng(50), (1, 8, 8, 8, 3)))
    with pytest.raises(tl.TwolinkError, match="TL_ERR_PRECISION"):
        ctx.build_twolinks(L, U, "f32-onelink")
    W1 = ctx.pack_links(L, U, "f32-onelink")
    with pytest.raises(ValueError, match="built with precision code"):
        ctx.smear([tl.Job(L, W1, [0], psi)], 2, 0.2, "f32")
    monkeypatch.setenv("TL_TILE", "6,512,4,0")
    with pytest.raises(tl.TwolinkError, match="TL_ERR_UNSUPPORTED"):
        ctx.smear([tl.Job(L, W1, [0], psi)], 2, 0.2, "f32-onelink")
    monkeypatch.delenv("TL_TILE")
    with pytest.raises(tl.TwolinkError, match="TL_ERR_ARG"):
        ctx.smear([tl.Job(L, W1, [0], psi)], 2, 0.5, "f32-onelink")   # sigma/n = 1/4 > 1/6
