"""Two smearing steps per launch (step variant 8) against one-step launches of the direct
kernel: bit for bit on every storage form, for even step counts and odd ones (which end
with one launch of the one-step companion tiling), y and z chains of odd and even length,
a y chain of one row, rows of 64 sites (backward x two-link from the neighbouring lane),
ragged z chunks, persistent grids, nontemporal stores and reversed odd launches; then the
autotuner's pick, graph replays (the resident buffer flips once per launch) and the refusals."""
import numpy as np
import pytest

from paper_2301_05518_amd import synth
from tests.gpu_common import errors, log, to_dev, tol

pytestmark = pytest.mark.gpu

DIRECT = "0,64,1,0"

# (lattice, RHS slices): Ly = 6 (two y chains of 3 rows) with Lz = 13 (one z chain of 13);
# Ly = 7 (one y chain of 7); Lz = 1; Ly = 2 (y chains of one row, every chain row of a tile
# wraps onto it); rows of 64 sites
CASES = [((10, 6, 13, 3), [0, 2, 0, 0]), ((5, 7, 2, 1), [0, 0]), ((8, 4, 1, 2), [1]),
         ((12, 2, 8, 1), [0, 0]), ((64, 8, 6, 2), [0, 0, 1, 0])]

# blocks of at least three rows of 64; the last names its one-step companion
FUSE_TILES = ["8,512,4,0", "8,256,3,0,1", "8,448,1,8", "8,192,16,0,0,1", "8,512,2,5,1,1",
              "8,384,5,0,0,0;4,128,2,0,0,1"]

PRECS = ["f64", "f32", "f16s", "bf16", "f32-w12", "bf16-w12"]


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
    return np.random.default_rng([4343, k])


def lattices(prec, seed0):
    out = []
    for k, (L, ts) in enumerate(CASES):
        if prec.startswith("f64"):   # the LDS-staged FP64 kernels take groups of one RHS
            ts = sorted(set(ts))
        U = synth.gauge_field(L, "haar", seed0 + k)
        psi = synth.random_field(rng(seed0 + k), (len(ts), L[2], L[1], L[0], 3))
        out.append((L, U, ts, psi))
    return out


def smear(ctx, torch, lats, n, sigma, prec, flags=0, variant=None):
    """Smear through a plan; variant: the step variant the plan must have run."""
    import paper_2301_05518_amd as tl
    jobs = []
    for L, U, ts, psi in lats:
        links = ctx.pack_links if prec.endswith("-onelink") else ctx.build_twolinks
        jobs.append(tl.Job(tuple(L), links(L, to_dev(U), prec), list(ts), to_dev(psi)))
    plan = ctx.plan(jobs, n, sigma, prec, flags)
    try:
        plan.load()
        plan.run()
        plan.store()
        torch.cuda.synchronize()
        info = plan.info()
    finally:
        plan.close()
    if variant is not None:
        assert info["variant"] == variant and info["steps_per_launch"] == (2 if variant == 8 else 1), info
    return [j.psi.cpu().numpy() for j in jobs]


@pytest.mark.parametrize("n", [6, 7])
@pytest.mark.parametrize("prec", PRECS)
def test_two_steps_bit_identical(ctx, orc, torch, prec, n, monkeypatch):
    lats = lattices(prec, 10)
    monkeypatch.setenv("TL_TILE", DIRECT)
    ref = smear(ctx, torch, lats, n, 2.5, prec, variant=0)
    for tile in FUSE_TILES:
        monkeypatch.setenv("TL_TILE", tile)
        log(f"two steps per launch {prec} n={n}: tile {tile}")
        out = smear(ctx, torch, lats, n, 2.5, prec, variant=8)
        for (L, _, _, _), a, b in zip(lats, out, ref):
            assert np.array_equal(a, b), (tile, L)
    for (L, U, ts, psi), o in zip(lats, ref):
        mr, l2 = errors(o, orc.smear_batch(orc.build_twolinks(U), ts, n, 2.5, psi))
        assert mr < tol(prec, n) and l2 < tol(prec, n), L


# every lattice with rows of 64 sites: the kernel built for that row length (backward x
# two-links from the neighbouring lane where the form allows it)
ROW64_CASES = [((64, 8, 6, 2), [0, 0, 1, 0]), ((64, 6, 5, 1), [0, 0, 0]), ((64, 2, 4, 1), [0])]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16", "f32-w12", "f16s-w12", "f32-onelink",
                                  "f16s-onelink"])
def test_two_steps_rows_of_64(ctx, orc, torch, prec, monkeypatch):
    lats = []
    for k, (L, ts) in enumerate(ROW64_CASES):
        if prec.startswith("f64"):
            ts = sorted(set(ts))
        U = synth.gauge_field(L, "haar", 40 + k)
        psi = synth.random_field(rng(40 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    n, sigma = (5, 0.5) if prec.endswith("-onelink") else (7, 2.5)
    monkeypatch.setenv("TL_TILE", DIRECT)
    ref = smear(ctx, torch, lats, n, sigma, prec, variant=0)
    for tile in ("8,512,4,0", "8,384,3,0,1,1", "8,192,1,8,0,1", "8,448,16,5,1,0", "8,512,2,3,0,1"):
        monkeypatch.setenv("TL_TILE", tile)
        log(f"two steps per launch, rows of 64, {prec}: tile {tile}")
        out = smear(ctx, torch, lats, n, sigma, prec, variant=8)
        for (L, _, _, _), a, b in zip(lats, out, ref):
            assert np.array_equal(a, b), (tile, L)
    for (L, U, ts, psi), o in zip(lats, ref):
        if prec.endswith("-onelink"):
            r = orc.smear_onelink_batch(U, ts, n, sigma, psi)
            base = prec.replace("-onelink", "")
        else:
            r = orc.smear_batch(orc.build_twolinks(U), ts, n, sigma, psi)
            base = prec
        mr, l2 = errors(o, r)
        assert mr < tol(base, n) and l2 < tol(base, n), L


@pytest.mark.parametrize("prec", ["f32-onelink", "f16s-onelink"])
def test_two_steps_onelink(ctx, orc, torch, prec, monkeypatch):
    """One-link fields (hops of one site): the chains are all rows and all planes."""
    lats = lattices(prec, 20)
    monkeypatch.setenv("TL_TILE", DIRECT)
    ref = smear(ctx, torch, lats, 5, 0.5, prec, variant=0)
    for tile in ("8,512,4,0", "8,256,3,8,1,1", "8,192,1,0,0,1"):
        monkeypatch.setenv("TL_TILE", tile)
        log(f"two steps per launch {prec}: tile {tile}")
        out = smear(ctx, torch, lats, 5, 0.5, prec, variant=8)
        for (L, _, _, _), a, b in zip(lats, out, ref):
            assert np.array_equal(a, b), (tile, L)
    base = prec.replace("-onelink", "")
    for (L, U, ts, psi), o in zip(lats, ref):
        mr, l2 = errors(o, orc.smear_onelink_batch(U, ts, 5, 0.5, psi))
        assert mr < tol(base, 5) and l2 < tol(base, 5), L


def test_plan_runs_flip_buffers(ctx, orc, torch, monkeypatch):
    """Graph replays and eager runs of a plan whose launches each run two steps: with n = 6
    (three launches) every run leaves its result in the other resident buffer, with n = 4
    (two) in the same one; load, run and store three times in a row and compare each result."""
    import paper_2301_05518_amd as tl
    L = (64, 8, 6, 1)
    U = synth.gauge_field(L, "haar", 31)
    psi = synth.random_field(rng(31), (3, 6, 8, 64, 3))
    for n in (6, 4):
        monkeypatch.setenv("TL_TILE", DIRECT)
        ref = smear(ctx, torch, [(L, U, [0, 0, 0], psi)], n, 2.0, "f32")[0]
        monkeypatch.setenv("TL_TILE", "8,512,2,0,1,1")
        for flags in (tl.TL_GRAPH, 0):
            job = tl.Job(L, ctx.build_twolinks(L, to_dev(U), "f32"), [0, 0, 0], to_dev(psi))
            plan = ctx.plan([job], n, 2.0, "f32", flags)
            for rep in range(3):
                job.psi.copy_(to_dev(psi))
                plan.load()
                plan.run()
                plan.store()
                torch.cuda.synchronize()
                assert plan.info()["steps_per_launch"] == 2 and plan.info()["variant"] == 8
                assert np.array_equal(job.psi.cpu().numpy(), ref), (n, flags, rep)
            plan.close()


def test_autotune_includes_two_steps(ctx, orc, torch, monkeypatch):
    """The autotuner's pick, one or two steps per launch, gives the direct kernel's bits; its
    one-step companion serves an odd step count."""
    import paper_2301_05518_amd as tl
    monkeypatch.delenv("TL_TILE", raising=False)
    L = (64, 16, 12, 2)
    U = synth.gauge_field(L, "haar", 32)
    psi = synth.random_field(rng(32), (3, 12, 16, 64, 3))
    for n in (8, 9):
        monkeypatch.setenv("TL_TILE", DIRECT)
        ref = smear(ctx, torch, [(L, U, [1, 1, 1], psi)], n, 3.0, "f32")[0]
        monkeypatch.delenv("TL_TILE")
        job = tl.Job(L, ctx.build_twolinks(L, to_dev(U), "f32"), [1, 1, 1], to_dev(psi))
        plan = ctx.plan([job], n, 3.0, "f32", tl.TL_GRAPH | tl.TL_AUTOTUNE)
        plan.load()
        plan.run()
        plan.store()
        torch.cuda.synchronize()
        info = plan.info()
        log(f"autotune n={n}: variant {info['variant']}, {info['steps_per_launch']} step(s) per launch")
        assert info["steps_per_launch"] == (2 if info["variant"] == 8 else 1)
        assert np.array_equal(job.psi.cpu().numpy(), ref), n
        plan.close()
    # TL_ONE_STEP keeps the tuning to one step per launch
    job = tl.Job(L, ctx.build_twolinks(L, to_dev(U), "f32"), [1, 1, 1], to_dev(psi))
    plan = ctx.plan([job], 8, 3.0, "f32", tl.TL_AUTOTUNE | tl.TL_ONE_STEP)
    plan.load()
    plan.run()
    plan.store()
    torch.cuda.synchronize()
    assert plan.info()["steps_per_launch"] == 1 and plan.info()["variant"] != 8
    plan.close()


def test_two_steps_refusals(ctx, torch, monkeypatch):
    """Two steps per launch are refused before any launch for TL_PLAIN (one step per launch)
    and for FP64 groups of more than one RHS."""
    import paper_2301_05518_amd as tl
    L = (12, 8, 10, 1)
    U = synth.gauge_field(L, "haar", 33)
    psi = synth.random_field(rng(33), (2, 10, 8, 12, 3))
    monkeypatch.setenv("TL_TILE", "8,512,4,0")
    with pytest.raises(tl.TwolinkError, match="TL_ERR_UNSUPPORTED"):
        smear(ctx, torch, [(L, U, [0, 0], psi)], 4, 2.0, "f32", tl.TL_PLAIN)
    with pytest.raises(tl.TwolinkError, match="TL_ERR_UNSUPPORTED"):
        smear(ctx, torch, [(L, U, [0, 0], psi)], 4, 2.0, "f64")


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16"])
def test_nan_source_detected_and_confined(ctx, torch, prec, monkeypatch):
    """A NaN in one source is caught by the plan's FP64 norms and stays in its own RHS: the
    RHS sharing its two-link loads (same slice, same group) and the RHS of another slice come
    out bit for bit as without it, under one-step tilings and the two-step kernel."""
    import paper_2301_05518_amd as tl
    L = (64, 8, 6, 2)
    ts = [0, 0, 0, 1]
    U = synth.gauge_field(L, "haar", 34)
    psi = synth.random_field(rng(34), (len(ts), 6, 8, 64, 3))
    bad = psi.copy()
    bad[1, 3, 2, 17, 1] = complex(np.nan, 0.0)
    for tile in (DIRECT, "7,512,4,0,1,1", "8,384,3,0,1,1"):
        monkeypatch.setenv("TL_TILE", tile)
        outs, norms = [], []
        for src in (psi, bad):
            job = tl.Job(L, ctx.build_twolinks(L, to_dev(U), prec), ts, to_dev(src))
            plan = ctx.plan([job], 6, 2.0, prec, tl.TL_GRAPH)
            plan.load()
            plan.run()
            norms.append(plan.reduce("norm2").cpu().numpy())
            plan.store()
            torch.cuda.synchronize()
            outs.append(job.psi.cpu().numpy())
            plan.close()
        log(f"NaN source {prec} tile {tile}: norms {norms[1]}")
        assert np.isnan(norms[1][1]) and np.isnan(outs[1][1]).any()
        for r in (0, 2, 3):
            assert np.isfinite(norms[1][r]) and norms[1][r] == norms[0][r], (tile, r)
            assert np.array_equal(outs[1][r], outs[0][r]), (tile, r)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_split_groups_bit_identical(ctx, orc, torch, prec, monkeypatch):
    """Tilings that give every RHS its own tiles (TL_TILE width field 1: the slice's two-links
    loaded once per RHS) compute the same bits as the plan's groups of up to four RHS; FP64,
    whose LDS-staged kernels take one RHS per group, runs them on split groups."""
    import paper_2301_05518_amd as tl
    L1, L2 = (64, 8, 6, 2), (10, 6, 7, 2)
    lats = []
    for k, (L, ts) in enumerate(((L1, [0, 0, 0, 1, 1]), (L2, [1, 1, 1, 1]))):
        U = synth.gauge_field(L, "haar", 50 + k)
        psi = synth.random_field(rng(50 + k), (len(ts), L[2], L[1], L[0], 3))
        lats.append((L, U, ts, psi))
    monkeypatch.setenv("TL_TILE", DIRECT)
    ref = smear(ctx, torch, lats, 6, 2.0, prec, variant=0)
    tiles = ["0,64,1,0,0,0,1", "4,128,2,3,1,1,1", "7,512,4,0,1,1,1", "5,256,3,0,0,0,1"]
    if prec != "f64":
        tiles += ["8,384,3,0,1,1,1", "8,384,3,0,1,1,2"]
    for tile in tiles:
        monkeypatch.setenv("TL_TILE", tile)
        log(f"split groups {prec}: tile {tile}")
        job_out = smear(ctx, torch, lats, 6, 2.0, prec, variant=int(tile[0]))
        for (L, _, _, _), a, b in zip(lats, job_out, ref):
            assert np.array_equal(a, b), (tile, L)
    for (L, U, ts, psi), o in zip(lats, ref):
        mr, l2 = errors(o, orc.smear_batch(orc.build_twolinks(U), ts, 6, 2.0, psi))
        assert mr < tol(prec, 6) and l2 < tol(prec, 6), L


def test_plan_info_reports_split_width(ctx, torch, monkeypatch):
    import paper_2301_05518_amd as tl
    L = (12, 8, 6, 1)
    U = synth.gauge_field(L, "haar", 52)
    psi = synth.random_field(rng(52), (3, 6, 8, 12, 3))
    for tile, w in (("4,128,2,0,0,0,1", 1), ("4,128,2,0,0,0", 3)):
        monkeypatch.setenv("TL_TILE", tile)
        job = tl.Job(L, ctx.build_twolinks(L, to_dev(U), "f32"), [0, 0, 0], to_dev(psi))
        plan = ctx.plan([job], 4, 1.0, "f32")
        plan.load()
        plan.run()
        torch.cuda.synchronize()
        info = plan.info()
        assert info["group_width"] == 3 and info["tile_width"] == w, info
        plan.close()
