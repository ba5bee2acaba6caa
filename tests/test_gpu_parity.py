"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle, at
sizes the oracle finishes in seconds: ragged tiles, odd extents, L = 1, 2, 4,
every precision, every launch mode."""
import os

import numpy as np
import pytest

from oracle import checks
from paper_2301_05518_amd import synth
from tests import helpers as H
from tests import packed
from tests.gpu_common import errors, gpu_smear, log, to_dev, tol, tol_lap

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
    return np.random.default_rng([4242, k])


def haar(L, seed):
    return synth.gauge_field(L, "haar", seed)


# ------------------------------------------------------------------ build

BUILD_SHAPES = [(6, 5, 7, 3), (4, 4, 4, 2), (17, 9, 5, 2), (1, 2, 3, 2), (64, 3, 2, 1)]


@pytest.mark.parametrize("L", BUILD_SHAPES, ids=[str(s) for s in BUILD_SHAPES])
def test_build_fp64_equals_product(ctx, orc, torch, L):
    log(f"build f64 {L}")
    U = haar(L, 1 + L[0])
    W = ctx.build_twolinks(L, to_dev(U), "f64")
    torch.cuda.synchronize()
    got = packed.decode_twolinks(W.cpu().numpy(), L, "f64", L[3])
    ref = orc.build_twolinks(U)
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16"])
def test_build_storage_rounding(ctx, orc, torch, prec):
    L = (10, 6, 7, 2)
    log(f"build {prec} {L}")
    U = haar(L, 7)
    W = ctx.build_twolinks(L, to_dev(U), prec)
    torch.cuda.synchronize()
    got = packed.decode_twolinks(W.cpu().numpy(), L, prec, L[3])
    ref = orc.build_twolinks(U)
    # one rounding of entries of modulus <= 1 (SU(3)): half an ulp at 1 plus FP32 double-rounding slack
    bound = {"f32": 2.0 ** -24, "f16s": 2.0 ** -11 * 1.01, "bf16": 2.0 ** -8 * 1.01}[prec]
    d = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag)).max()
    assert d <= bound, d


def test_build_slice_subset(ctx, orc, torch):
    L = (6, 4, 5, 4)
    U = haar(L, 3)
    W = ctx.build_twolinks(L, to_dev(U), "f64", slices=[2, 0, 3])
    torch.cuda.synchronize()
    got = packed.decode_twolinks(W.cpu().numpy(), L, "f64", 3)
    ref = orc.build_twolinks(U)
    for slot, t in enumerate([2, 0, 3]):
        assert np.abs(got[slot] - ref[t]).max() < 1e-14


# ------------------------------------------------------------------ Laplacian

LAP_SHAPES = [(4, 4, 4, 1), (2, 3, 5, 2), (1, 1, 1, 1), (1, 6, 2, 1), (17, 9, 5, 2), (8, 8, 8, 3), (33, 2, 4, 1)]


@pytest.mark.parametrize("L", LAP_SHAPES, ids=[str(s) for s in LAP_SHAPES])
def test_laplacian_fp64(ctx, orc, torch, L):
    log(f"laplacian f64 {L}")
    U = haar(L, 11)
    Ud = to_dev(U)
    W = ctx.build_twolinks(L, Ud, "f64")
    Wo = orc.build_twolinks(U)
    for t in range(L[3]):
        psi = synth.random_field(rng(t), (L[2], L[1], L[0], 3))
        out = ctx.laplacian(L, W, "f64", t, to_dev(psi))
        torch.cuda.synchronize()
        ref = orc.laplacian(Wo, t, psi)
        assert checks.max_rel(out.cpu().numpy(), ref) < 1e-14


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16"])
def test_laplacian_mixed(ctx, orc, torch, prec):
    L = (12, 10, 9, 2)
    U = haar(L, 12)
    W = ctx.build_twolinks(L, to_dev(U), prec)
    psi = synth.random_field(rng(5), (L[2], L[1], L[0], 3))
    out = ctx.laplacian(L, W, prec, 1, to_dev(psi)).cpu().numpy()
    ref = orc.laplacian(orc.build_twolinks(U), 1, psi)
    mr, l2 = errors(out, ref)
    log(f"laplacian {prec}: max-rel {mr:.3e} l2-rel {l2:.3e}")
    assert mr < tol_lap(prec) and l2 < tol_lap(prec)


def test_laplacian_subset_slot(ctx, orc, torch):
    L = (6, 6, 4, 5)
    U = haar(L, 13)
    W = ctx.build_twolinks(L, to_dev(U), "f64", slices=[4, 1])
    psi = synth.random_field(rng(6), (4, 6, 6, 3))
    out = ctx.laplacian(L, W, "f64", 1, to_dev(psi), w_slices=[4, 1]).cpu().numpy()
    ref = orc.laplacian(orc.build_twolinks(U), 1, psi)
    assert checks.max_rel(out, ref) < 1e-14


# ------------------------------------------------------------------ smearing, FP64

def test_smear_point_source_8cube(ctx, orc, torch):
    """8^3x8, exp-of-anti-Hermitian links, point source, N=20, sigma=2 (the small workload)."""
    wl = synth.workload(0)
    lat = wl.lattices[0]
    U = lat.links_array()
    psi = lat.sources_array()
    out = gpu_smear(ctx, [(lat.L, U, lat.t_of_rhs, psi)], wl.n_steps, wl.sigma, "f64")[0]
    ref = orc.smear_batch(orc.build_twolinks(U), lat.t_of_rhs, wl.n_steps, wl.sigma, psi)
    mr, l2 = errors(out, ref)
    log(f"8^3x8 f64 N=20: max-rel {mr:.3e} l2-rel {l2:.3e}")
    assert mr < 1e-12 and l2 < 1e-12


MODES = {"batched": 0, "plain": 1, "graph": 2, "autotune": 4, "graph+autotune": 6, "plain+autotune": 5}


def test_smear_modes_bit_identical(ctx, orc, torch):
    """Every launch mode gives the same bits; all match the oracle."""
    import paper_2301_05518_amd as tl
    L = (10, 6, 9, 4)
    ts = [1, 3, 1, 1, 3, 0, 1]          # groups of 4, 2 and 1 RHS
    U = haar(L, 21)
    psi = synth.random_field(rng(21), (len(ts), L[2], L[1], L[0], 3))
    ref = orc.smear_batch(orc.build_twolinks(U), ts, 9, 3.0, psi)
    outs = {}
    for name, flags in MODES.items():
        outs[name] = gpu_smear(ctx, [(L, U, ts, psi)], 9, 3.0, "f64", flags)[0]
        mr, l2 = errors(outs[name], ref)
        log(f"mode {name}: max-rel {mr:.3e}")
        assert mr < 1e-12 and l2 < 1e-12
    for name in MODES:
        assert np.array_equal(outs[name], outs["batched"]), name


def test_plain_autotune_uneven_batch(ctx, orc, torch):
    """Plain launches (one RHS per launch) of an uneven batch, tuned over every lattice shape of
    the batch: the same bits as batched launches, and the oracle's result."""
    lats = []
    for k, (L, ts) in enumerate([((10, 6, 9, 2), [0, 1, 1]), ((8, 8, 6, 1), [0, 0]), ((6, 4, 5, 2), [1])]):
        U = haar(L, 60 + k)
        psi = synth.random_field(rng(60 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    plain = gpu_smear(ctx, lats, 7, 2.5, "f64", MODES["plain+autotune"])
    batched = gpu_smear(ctx, lats, 7, 2.5, "f64", MODES["batched"])
    for (L, U, ts, psi), a, b in zip(lats, plain, batched):
        assert np.array_equal(a, b), L
        ref = orc.smear_batch(orc.build_twolinks(U), ts, 7, 2.5, psi)
        mr, l2 = errors(a, ref)
        log(f"plain+autotune {L}: max-rel {mr:.3e}")
        assert mr < 1e-12 and l2 < 1e-12


def test_side_stream_and_second_context(ctx, orc, torch):
    """A context on a non-default torch stream (and a second context on the same device)
    gives the same bits as the default-stream context; the caller orders the streams."""
    import paper_2301_05518_amd as tl
    L = (12, 8, 10, 2)
    ts = [0, 1, 0]
    U = haar(L, 23)
    psi = synth.random_field(rng(23), (len(ts), L[2], L[1], L[0], 3))
    ref = gpu_smear(ctx, [(L, U, ts, psi)], 6, 2.0, "f32", 6)[0]
    side = torch.cuda.Stream()
    c2 = tl.Context(0, stream=side)
    try:
        with torch.cuda.stream(side):
            Ud, pd = to_dev(U), to_dev(psi)
            W = c2.build_twolinks(L, Ud, "f32")
            c2.smear([tl.Job(L, W, ts, pd)], 6, 2.0, "f32", 6)
        side.synchronize()
        assert np.array_equal(pd.cpu().numpy(), ref)
    finally:
        c2.close()


@pytest.mark.parametrize("kinds", [0, 1, 2, 3])
def test_stream_probe_sums_planes(ctx, torch, kinds):
    """The streaming probe writes its last plane as the sum of the others (any load/store kind)."""
    n_in, words = 4, 10000 + 37
    vals = torch.arange(n_in * words * 4, dtype=torch.float32, device="cuda").remainder_(97.0)
    buf = torch.zeros((n_in + 1) * words * 16 + 48, dtype=torch.uint8, device="cuda")
    buf[: n_in * words * 16].view(torch.float32).copy_(vals)
    ms = ctx.stream_time(buf, n_in=n_in, kinds=kinds, grid=7, reps=2)
    torch.cuda.synchronize()
    assert ms > 0.0
    planes = buf[: (n_in + 1) * words * 16].view(torch.float32).view(n_in + 1, words * 4)
    assert torch.equal(planes[n_in], planes[:n_in].sum(dim=0))


def test_stream_switch_orders_scratch(orc, torch):
    """tl_set_stream between two Laplacians of different shapes: the second call reuses the
    context scratch (its table upload and pack) while the first may still run on the old
    stream; the switch makes the new stream wait, so both results are right."""
    import paper_2301_05518_amd as tl
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    c = tl.Context(0, stream=s1)
    try:
        La, Lb = (48, 48, 40, 1), (10, 6, 8, 1)
        Ua, Ub = haar(La, 31), haar(Lb, 32)
        pa = synth.random_field(rng(31), (La[2], La[1], La[0], 3))
        pb = synth.random_field(rng(32), (Lb[2], Lb[1], Lb[0], 3))
        da, db = to_dev(pa), to_dev(pb)
        Wa = c.build_twolinks(La, to_dev(Ua), "f64")
        Wb = c.build_twolinks(Lb, to_dev(Ub), "f64")
        oa, ob = torch.empty_like(da), torch.empty_like(db)
        torch.cuda.synchronize()
        c.laplacian(La, Wa, "f64", 0, da, out=oa)
        c.set_stream(s2)
        c.laplacian(Lb, Wb, "f64", 0, db, out=ob)
        torch.cuda.synchronize()
        assert checks.max_rel(oa.cpu().numpy(), orc.laplacian(orc.build_twolinks(Ua), 0, pa)) < 1e-14
        assert checks.max_rel(ob.cpu().numpy(), orc.laplacian(orc.build_twolinks(Ub), 0, pb)) < 1e-14
    finally:
        c.close()


VARIANT_TILES = ["0,64,1,0", "0,128,3,256", "1,64,4,0", "1,128,5,512", "2,64,4,0", "2,128,3,0",
                 "2,192,16,256", "2,64,1,8", "3,64,1,0", "3,64,2,0", "3,128,5,0", "3,256,16,0", "3,64,4,8",
                 "4,64,1,0", "4,256,3,16", "4,128,2,0", "2,64,16,0,1", "0,64,2,0,1", "4,64,2,0,1",
                 "5,512,16,0", "5,256,3,0", "5,512,1,8", "5,256,5,0,1", "5,64,2,0",
                 "6,512,16,0", "6,256,3,0", "6,512,1,8", "6,256,2,0,1", "6,64,4,0",
                 "7,512,16,0", "7,256,3,0", "7,512,1,8", "7,256,2,0,1", "7,64,4,0", "7,512,5,4",
                 # odd steps reversed (tile order and march directions)
                 "0,64,2,5,0,1", "2,64,4,0,1,1", "3,128,5,0,0,1", "4,128,2,3,0,1", "5,256,3,0,1,1",
                 "6,512,1,8,0,1", "7,512,16,0,1,1", "7,256,3,5,0,1"]


@pytest.mark.parametrize("prec", PRECS)
def test_step_variants_bit_identical(ctx, orc, torch, prec, monkeypatch):
    """Every kernel variant and tiling (ragged xy tiles, ragged and alternating z chunks,
    persistent grids) gives the same bits as the direct kernel."""
    # every lattice has a full-row tiling (Ly with a divisor >= 4) so the LDS variant applies;
    # 8x4 makes the halo rows wrap onto the tile itself
    cases = [((10, 6, 13, 3), [0, 2, 0, 0]), ((5, 7, 2, 1), [0, 0]), ((8, 4, 1, 2), [1])]
    lats = []
    for k, (L, ts) in enumerate(cases):
        U = haar(L, 25 + k)
        psi = synth.random_field(rng(25 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    outs = {}
    # the LDS-staged kernel takes FP64 groups of one RHS only (these lattices have wider groups)
    tiles = [t for t in VARIANT_TILES if not (prec == "f64" and t[:2] in ("5,", "6,", "7,"))]
    for tile in tiles:
        monkeypatch.setenv("TL_TILE", tile)
        log(f"variants {prec}: tile {tile}")
        outs[tile] = gpu_smear(ctx, lats, 7, 2.5, prec)
    for tile in tiles:
        for a, b in zip(outs[tile], outs[VARIANT_TILES[0]]):
            assert np.array_equal(a, b), tile
    for (L, U, ts, psi), o in zip(lats, outs[VARIANT_TILES[0]]):
        ref = orc.smear_batch(orc.build_twolinks(U), ts, 7, 2.5, psi)
        mr, l2 = errors(o, ref)
        assert mr < tol(prec, 7) and l2 < tol(prec, 7)


ROW64_TILES = ["0,64,1,0", "5,512,3,0", "6,256,2,0,1", "7,512,4,0", "7,256,3,5,0,1", "7,512,2,3,1,1",
               "7,256,16,0,1,0"]


# (lattice, RHS slices, tilings): 256-thread tiles have no row tiling when Ly = 6
ROW64_CASES = [((64, 8, 6, 2), [0, 0, 1, 0], ROW64_TILES),
               ((64, 6, 5, 1), [0, 0, 0], ["0,64,1,0", "5,512,3,0", "7,512,4,0", "7,512,2,3,1,1", "7,512,5,0,0,1"])]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ROW64_CASES, ids=["64x8x6", "64x6x5"])
def test_step_variants_rows_of_64(ctx, orc, torch, prec, case, monkeypatch):
    """Rows of 64 sites (one wave per row, the benchmark's row length): the LDS-staged
    variants, whose FP32 and F16S forms take the backward x two-link from the neighbouring
    lane, give the direct kernel's bits.  Ly = 6 leaves two idle waves in a 512-thread tile
    (they still take part in the lane exchange); Lz = 5 makes a single chain."""
    L, ts, tiles = case
    if prec == "f64":   # the LDS-staged FP64 kernels take groups of one RHS
        ts = [L[3] - 1]
    U = haar(L, 60)
    psi = synth.random_field(rng(60), (len(ts), L[2], L[1], L[0], 3))
    outs = {}
    for tile in tiles:
        monkeypatch.setenv("TL_TILE", tile)
        log(f"rows of 64 {prec} {L}: tile {tile}")
        outs[tile] = gpu_smear(ctx, [(L, U, ts, psi)], 6, 2.0, prec)[0]
    for tile in tiles[1:]:
        assert np.array_equal(outs[tile], outs[tiles[0]]), tile
    ref = orc.smear_batch(orc.build_twolinks(U), ts, 6, 2.0, psi)
    mr, l2 = errors(outs[tiles[0]], ref)
    assert mr < tol(prec, 6) and l2 < tol(prec, 6)


@pytest.mark.parametrize("prec", ["f32-onelink", "f16s-onelink", "f32-w12-onelink"])
def test_onelink_rows_of_64(ctx, orc, torch, prec, monkeypatch):
    """One-link fields on rows of 64 sites: the pipelined variant takes the backward x link
    from the lane one to the left and gives the direct kernel's bits."""
    import paper_2301_05518_amd as tl
    L = (64, 6, 7, 2)
    ts = [0, 0, 1]
    U = haar(L, 61)
    psi = synth.random_field(rng(61), (len(ts), L[2], L[1], L[0], 3))
    outs = {}
    for tile in ("0,64,1,0", "7,512,4,0", "7,512,3,5,0,1", "7,512,2,0,1,1"):
        monkeypatch.setenv("TL_TILE", tile)
        log(f"one-link rows of 64 {prec}: tile {tile}")
        jobs = [tl.Job(L, ctx.pack_links(L, to_dev(U), prec), ts, to_dev(psi))]
        ctx.smear(jobs, 5, 0.5, prec)
        torch.cuda.synchronize()
        outs[tile] = jobs[0].psi.cpu().numpy()
    for tile, o in outs.items():
        assert np.array_equal(o, outs["0,64,1,0"]), tile
    ref = orc.smear_onelink_batch(U, ts, 5, 0.5, psi)
    base = prec.replace("-onelink", "")
    mr, l2 = errors(outs["0,64,1,0"], ref)
    assert mr < tol(base, 5) and l2 < tol(base, 5)


def test_lds_variant_fp64_single_rhs(ctx, orc, torch, monkeypatch):
    """The LDS-staged kernel at FP64 (groups of one RHS) matches the direct kernel bit for bit;
    forcing it on a wider FP64 group is refused before any launch."""
    import paper_2301_05518_amd as tl
    lats = []
    for k, (L, ts) in enumerate((((12, 8, 10, 2), [0, 1]), ((6, 5, 7, 1), [0]))):
        U = haar(L, 27 + k)
        psi = synth.random_field(rng(27 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    outs = []
    for tile in ("0,64,1,0", "5,512,4,0", "5,256,16,8,1", "6,512,4,0", "6,256,3,8,1", "7,512,4,0", "7,256,3,8,1"):
        monkeypatch.setenv("TL_TILE", tile)
        outs.append(gpu_smear(ctx, lats, 6, 2.0, "f64"))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    monkeypatch.setenv("TL_TILE", "5,512,4,0")
    L = (12, 8, 10, 1)
    with pytest.raises(tl.TwolinkError, match="TL_ERR_UNSUPPORTED"):
        gpu_smear(ctx, [(L, haar(L, 29), [0, 0], synth.random_field(rng(29), (2, 10, 8, 12, 3)))], 6, 2.0, "f64")


def test_smear_uneven_batch_fp64(ctx, orc, torch):
    shapes = [((6, 4, 8, 3), [0, 2]), ((9, 7, 5, 2), [1, 1, 1]), ((4, 4, 4, 1), [0])]
    lats, refs = [], []
    for k, (L, ts) in enumerate(shapes):
        U = haar(L, 30 + k)
        psi = synth.random_field(rng(30 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
        refs.append(orc.smear_batch(orc.build_twolinks(U), ts, 12, 4.0, psi))
    for flags in (0, 6):
        outs = gpu_smear(ctx, lats, 12, 4.0, "f64", flags)
        for o, r in zip(outs, refs):
            assert checks.max_rel(o, r) < 1e-12


def test_free_field_closed_form(ctx, torch):
    """Unit links: the GPU result equals the exact free kernel (Fourier form), no C oracle involved."""
    for L, n, sigma, x0 in (((8, 8, 8, 2), 20, 2.0, (0, 0, 0)), ((12, 6, 10, 1), 15, 3.0, (3, 1, 7))):
        U = synth.unit_gauge(L)
        psi = np.stack([synth.point_source(L[:3], c, x0) for c in range(3)])
        out = gpu_smear(ctx, [(L, U, [L[3] - 1] * 3, psi)], n, sigma, "f64")[0]
        k = checks.free_kernel_dft(L[:3], n, sigma, x0)
        for c in range(3):
            ref = np.zeros_like(out[c])
            ref[..., c] = k
            assert checks.max_rel(out[c], ref) < 1e-13


def test_gauge_covariance(ctx, torch):
    L = (8, 6, 6, 2)
    U = haar(L, 40)
    G = synth.gauge_transform(L, 41)
    psi = synth.random_field(rng(40), (2, L[2], L[1], L[0], 3))
    a = gpu_smear(ctx, [(L, H.transform_links(U, G), [0, 1], np.stack([H.transform_vector(psi[0], G[0]),
                                                                          H.transform_vector(psi[1], G[1])]))],
                  10, 4.0, "f64")[0]
    b = gpu_smear(ctx, [(L, U, [0, 1], psi)], 10, 4.0, "f64")[0]
    for r in range(2):
        assert checks.max_rel(a[r], H.transform_vector(b[r], G[r])) < 1e-12


def test_repeated_runs_and_parity(ctx, orc, torch):
    """Two runs of an odd number of steps = one smearing with twice the steps (same sigma/n)."""
    import paper_2301_05518_amd as tl
    L = (6, 8, 6, 2)
    U = haar(L, 50)
    psi = synth.random_field(rng(50), (3, L[2], L[1], L[0], 3))
    Wo = orc.build_twolinks(U)
    for flags in (0, 2):
        W = ctx.build_twolinks(L, to_dev(U), "f64")
        p = to_dev(psi)
        plan = ctx.plan([tl.Job(L, W, [1, 1, 0], p)], 5, 1.5, "f64", flags)
        plan.load()
        plan.run()
        plan.run()
        plan.store()
        torch.cuda.synchronize()
        ref = orc.smear_batch(Wo, [1, 1, 0], 10, 3.0, psi)
        assert checks.max_rel(p.cpu().numpy(), ref) < 1e-12
        plan.close()


# ------------------------------------------------------------------ mixed precision

@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16"])
def test_smear_mixed_precision(ctx, orc, torch, prec):
    L = (16, 16, 16, 2)
    n, sigma = 40, 5.0
    U = haar(L, 60)
    psi = np.stack([synth.point_source(L[:3], c) for c in range(3)] + [synth.z2_source(rng(61), L[:3], 1)])
    ts = [0, 0, 0, 1]
    ref = orc.smear_batch(orc.build_twolinks(U), ts, n, sigma, psi)
    out = gpu_smear(ctx, [(L, U, ts, psi)], n, sigma, prec, 6)[0]
    mr, l2 = errors(out, ref)
    log(f"16^3 {prec} N={n}: max-rel {mr:.3e} l2-rel {l2:.3e} (bar {tol(prec, n):.2e})")
    assert mr < tol(prec, n) and l2 < tol(prec, n)


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16"])
def test_point_source_tails_stay_finite(ctx, orc, torch, prec):
    """A point source smeared over a large slice reaches FP32-subnormal values far away."""
    L = (40, 40, 40, 1)
    U = haar(L, 65)
    psi = synth.point_source(L[:3], 0)[None]
    out = gpu_smear(ctx, [(L, U, [0], psi)], 40, 5.0, prec, 6)[0]
    assert np.isfinite(out).all()
    ref = orc.smear_batch(orc.build_twolinks(U), [0], 40, 5.0, psi)
    mr, l2 = errors(out, ref)
    log(f"40^3 point {prec}: max-rel {mr:.3e} l2-rel {l2:.3e}")
    assert mr < tol(prec, 40) and l2 < tol(prec, 40)


@pytest.mark.parametrize("prec", PRECS)
def test_zero_steps_is_storage_roundtrip(ctx, torch, prec):
    """n = 0: pack then unpack; equals storing in the precision, bit for bit."""
    L = (7, 5, 3, 2)
    U = haar(L, 70)
    psi = synth.random_field(rng(70), (3, L[2], L[1], L[0], 3)) * np.array([1.0, 1e-3, 30.0])[:, None, None, None, None]
    psi[1, 0, 0, 0] = 0.0          # an all-zero site (F16S scale 0)
    psi[2, 1, 1, 1] = (3e-40, -1e-41j, 0.0)   # largest component an FP32 subnormal
    psi[2, 1, 1, 2] = (1e-30, 2e-31, 0.0)
    out = gpu_smear(ctx, [(L, U, [0, 1, 0], psi)], 0, 0.0, prec)[0]
    assert np.array_equal(out, packed.storage_round_vectors(psi, prec))


@pytest.mark.parametrize("prec", PRECS)
def test_storage_roundtrip_large(ctx, torch, prec):
    """The round trip on 147k reals with per-site magnitudes over four decades.  For F16S the
    quotient v * RN(1/s) is rounded to FP32 and then to half; rounding the exact product once,
    to half, gives a different code in about one real in 10^4, so this size tells the two apart."""
    L = (32, 16, 16, 1)
    U = haar(L, 71)
    r = rng(71)
    psi = synth.random_field(r, (3, L[2], L[1], L[0], 3))
    psi *= np.exp2(r.uniform(-6.0, 6.0, size=psi.shape[:-1]))[..., None]
    out = gpu_smear(ctx, [(L, U, [0, 0, 0], psi)], 0, 0.0, prec)[0]
    want = packed.storage_round_vectors(psi, prec)
    if prec == "f16s":
        re = np.stack([psi.real, psi.imag], -1).reshape(psi.shape[:-1] + (6,)).astype(np.float32)
        mx = np.abs(re).max(-1, keepdims=True)
        once = (re.astype(np.float64) * (np.float32(1.0) / mx).astype(np.float64)).astype(np.float16)
        twice = (re * (np.float32(1.0) / mx)).astype(np.float16)
        log(f"f16s: {int(np.sum(once != twice))} reals where one rounding would differ")
    assert np.array_equal(out, want)


# ------------------------------------------------------------------ reductions

def test_reduce_natural(ctx, orc, torch):
    psi = synth.random_field(rng(80), (3, 5, 6, 7, 3))
    phi = synth.random_field(rng(81), (3, 5, 6, 7, 3))
    n2 = ctx.reduce("norm2", to_dev(psi)).cpu().numpy()
    dt = ctx.reduce("dot", to_dev(psi), to_dev(phi)).cpu().numpy()
    sn = ctx.reduce("site_norm", to_dev(psi)).cpu().numpy()
    for r in range(3):
        assert abs(n2[r] - orc.norm2(psi[r])) < 1e-13 * n2[r]
        d = orc.dot(phi[r], psi[r])
        assert abs(dt[r] - d) < 1e-13 * abs(d)
        assert np.abs(sn[r] - orc.site_norms(psi[r])).max() < 1e-14 * sn[r].max()
    again = ctx.reduce("norm2", to_dev(psi)).cpu().numpy()
    assert np.array_equal(n2, again)        # fixed summation order


def test_plan_reductions(ctx, orc, torch):
    import paper_2301_05518_amd as tl
    L = (8, 6, 10, 2)
    U = haar(L, 90)
    psi = synth.random_field(rng(90), (3, L[2], L[1], L[0], 3))
    Wo = orc.build_twolinks(U)
    ref = orc.smear_batch(Wo, [1, 0, 1], 8, 2.0, psi)
    W = ctx.build_twolinks(L, to_dev(U), "f64")
    a = ctx.plan([tl.Job(L, W, [1, 0, 1], to_dev(psi))], 8, 2.0, "f64", 0)
    b = ctx.plan([tl.Job(L, W, [1, 0, 1], to_dev(psi))], 8, 2.0, "f64", 0)
    a.load(); a.run()
    b.load()
    n2 = a.reduce("norm2").cpu().numpy()
    sn = a.reduce("site_norm").cpu().numpy().reshape(3, L[2], L[1], L[0])
    dt = a.reduce("dot", b).cpu().numpy()        # <psi_initial, psi_smeared>
    for r in range(3):
        assert abs(n2[r] - orc.norm2(ref[r])) < 1e-12 * n2[r]
        assert np.abs(sn[r] - orc.site_norms(ref[r])).max() < 1e-12 * sn[r].max()
        d = orc.dot(psi[r], ref[r])
        assert abs(dt[r] - d) < 1e-12 * abs(d)
    a.close(); b.close()


# ------------------------------------------------------------------ error paths (host-forced)

@pytest.mark.parametrize("mode", ["alloc", "launch"])
def test_fault_hooks(torch, mode, monkeypatch):
    """TL_FAULT makes the library take its error paths without running a kernel."""
    import paper_2301_05518_amd as tl
    monkeypatch.setenv("TL_FAULT", mode)
    c = tl.Context(0)
    L = (4, 4, 4, 1)
    U = to_dev(synth.unit_gauge(L))
    W = torch.zeros(tl.twolinks_bytes(L, "f64"), dtype=torch.uint8, device="cuda")
    p = to_dev(synth.point_source(L[:3], 0)[None])
    if mode == "launch":
        with pytest.raises(tl.TwolinkError, match="TL_ERR_HIP"):
            c.build_twolinks(L, U, "f64", W=W)
    with pytest.raises(tl.TwolinkError, match="TL_ERR_NOMEM" if mode == "alloc" else "TL_ERR_HIP"):
        c.smear([tl.Job(L, W, [0], p)], 4, 1.0, "f64")
    c.close()
