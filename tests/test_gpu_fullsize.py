"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (graph + autotune, two-links built for the source slices).

The oracle computes whole slices (one smeared output site depends on the
whole slice after n >= L/4 steps), so each test compares every site of a
sample of right-hand sides, each against an oracle run on that RHS's slice.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import checks, core
from paper_2301_05518_amd import synth
from tests.gpu_common import errors, log, tol

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


def run_workload(ctx, torch, index, prec, flags, sample):
    """Smear workload `index` on the GPU; compare `sample` RHS indices per lattice with the oracle."""
    import paper_2301_05518_amd as tl
    wl = synth.workload(index)
    dev = torch.device("cuda", 0)
    orc = core.get()
    jobs, lats = [], []
    for lat in wl.lattices:
        Lx, Ly, Lz, Lt = lat.L
        slices = sorted(set(lat.t_of_rhs))
        # only the source slices' links are read when W is built for those slices
        U = torch.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=torch.complex128, device=dev)
        keep = set(lat.t_of_rhs[r] for r in sample(len(lat.t_of_rhs)))   # the oracle needs these
        host = {}
        with ThreadPoolExecutor(max_workers=16) as ex:
            futs = {t: ex.submit(synth.gauge_slice, lat.L, lat.links, lat.link_seed, t) for t in slices}
            for t in slices:
                u = futs[t].result()
                U[t].copy_(torch.from_numpy(u))
                if t in keep:
                    host[t] = u
        if prec.endswith("-onelink"):
            W = ctx.pack_links(lat.L, U, prec, slices=slices)
        else:
            W = ctx.build_twolinks(lat.L, U, prec, slices=slices)
        psi = torch.from_numpy(lat.sources_array()).to(dev)
        jobs.append(tl.Job(lat.L, W, lat.t_of_rhs, psi, slices))
        lats.append((lat, host))
        del U
    log(f"workload {index} ({wl.name}) {prec}: smearing on the GPU")
    ctx.smear(jobs, wl.n_steps, wl.sigma, prec, flags)
    torch.cuda.synchronize()
    worst = 0.0
    for (lat, host), job in zip(lats, jobs):
        for r in sample(len(lat.t_of_rhs)):
            t = lat.t_of_rhs[r]
            if prec.endswith("-onelink"):
                ref = orc.smear_onelink(host[t][None], 0, wl.n_steps, wl.sigma, lat.source(r))
            else:
                ref = orc.smear(orc.build_twolinks(host[t][None]), 0, wl.n_steps, wl.sigma, lat.source(r))
            got = job.psi[r].cpu().numpy()
            mr, l2 = errors(got, ref)
            log(f"  {lat.L} RHS {r} (t={t}): max-rel {mr:.3e} l2-rel {l2:.3e}")
            if not (np.isfinite(mr) and np.isfinite(l2)):
                worst = float("inf")
            else:
                worst = max(worst, mr, l2)
    return worst, wl.n_steps


def test_workload1_fp64_32cube(ctx, torch):
    """32^3x64, 3 colour point sources, N=40, FP64: every RHS, batched and plain launches."""
    for flags in (6, 1):
        worst, n = run_workload(ctx, torch, 1, "f64", flags, lambda k: range(k))
        assert worst < tol("f64", n)


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_workload2_48cube(ctx, torch, prec):
    """48^3x96, 3 colour point sources, N=40, FP32 and F16S: every RHS."""
    worst, n = run_workload(ctx, torch, 2, prec, 6, lambda k: range(k))
    assert worst < tol(prec, n)


def test_workload3_64cube_24rhs(ctx, torch):
    """64^3x96, 24 colour wall sources on 8 slices, N=60, FP32: 4 RHS sampled over slices and colours."""
    worst, n = run_workload(ctx, torch, 3, "f32", 6, lambda k: [0, 7, 14, k - 1])
    assert worst < tol("f32", n)


@pytest.mark.parametrize("prec", ["f16s", "bf16"])
def test_workload3_16bit_storage(ctx, torch, prec):
    """Workload 3 stored in F16S and BF16 (tuned, graph): 2 RHS sampled against the oracle."""
    worst, n = run_workload(ctx, torch, 3, prec, 6, lambda k: [5, k - 1])
    log(f"workload 3 in {prec}: worst {worst:.3e} (bar {tol(prec, n):.2e})")
    assert worst < tol(prec, n)


def test_workload3_w12(ctx, torch):
    """Workload 3 with twelve-real two-links (FP32 rows, third row rebuilt): 3 RHS sampled."""
    worst, n = run_workload(ctx, torch, 3, "f32-w12", 6, lambda k: [0, 11, k - 1])
    assert worst < tol("f32-w12", n)


def test_workload3_onelink(ctx, torch):
    """Workload 3's sources under one-link smearing (same sigma, hops of one site), FP32: 3 RHS sampled."""
    worst, n = run_workload(ctx, torch, 3, "f32-onelink", 6, lambda k: [0, 13, k - 1])
    assert worst < tol("f32", n)


def test_workload4_uneven_bf16(ctx, torch):
    """Uneven batch 24^3x48 + 32^3x64 + 48^3x96, Z2 sources, N=40, BF16: first and last RHS of each lattice."""
    worst, n = run_workload(ctx, torch, 4, "bf16", 6, lambda k: sorted({0, k - 1}))
    assert worst < tol("bf16", n)


def test_workload5_sink_smearing_288rhs(ctx, torch):
    """64^3x96, 3 colour walls on all 96 slices (288 RHS) with one two-link field, N=60, FP32:
    RHS on the first, a middle and the last slice."""
    worst, n = run_workload(ctx, torch, 5, "f32", 6, lambda k: [0, 143, k - 1])
    assert worst < tol("f32", n)


def test_64cube_odd_steps_two_step_launches(ctx, torch, monkeypatch):
    """A 64^3 slice with 3 colour walls and an odd step count (n = 7): three two-step launches
    and one launch of the named one-step companion give the bits of seven one-step launches
    and of the autotuned plan; every RHS against the oracle."""
    import paper_2301_05518_amd as tl
    L = (64, 64, 64, 1)
    n, sigma = 7, 0.7
    u = synth.gauge_slice(L, "haar", 2301055100, 0)
    psi = np.zeros((3, 64, 64, 64, 3), dtype=np.complex128)
    for c in range(3):
        psi[c, ..., c] = 1.0
    Ud = torch.from_numpy(u[None]).cuda()
    runs = {"two-step + companion": ("8,384,4,0,1,1;7,512,16,0,1,1", tl.TL_GRAPH),
            "one-step": ("7,512,16,0,1,1", tl.TL_GRAPH),
            "autotuned": (None, tl.TL_GRAPH | tl.TL_AUTOTUNE)}
    outs = {}
    for name, (tile, flags) in runs.items():
        if tile is None:
            monkeypatch.delenv("TL_TILE", raising=False)
        else:
            monkeypatch.setenv("TL_TILE", tile)
        W = ctx.build_twolinks(L, Ud, "f32")
        job = tl.Job(L, W, [0, 0, 0], torch.from_numpy(psi).cuda())
        plan = ctx.plan([job], n, sigma, "f32", flags)
        plan.load()
        plan.run()
        plan.store()
        torch.cuda.synchronize()
        info = plan.info()
        log(f"64^3 n=7 {name}: variant {info['variant']}, {info['steps_per_launch']} step(s) per launch")
        if name == "two-step + companion":
            assert info["variant"] == 8 and info["steps_per_launch"] == 2
        outs[name] = job.psi.cpu().numpy()
        plan.close()
    for name in runs:
        assert np.array_equal(outs[name], outs["one-step"]), name
    orc = core.get()
    Wo = orc.build_twolinks(u[None])
    worst = 0.0
    for c in range(3):
        ref = orc.smear(Wo, 0, n, sigma, psi[c])
        mr, l2 = errors(outs["one-step"][c], ref)
        worst = max(worst, mr, l2)
    log(f"  max-rel/l2 {worst:.3e}")
    assert worst < tol("f32", n)


def test_workload3_two_step_plan_equals_one_step_all_rhs(ctx, torch):
    """The benchmark's workload (64^3x96, 24 colour walls on 8 slices, n = 60, FP32) as the
    autotuned plan runs it (two steps per launch) and with one step per launch (TL_ONE_STEP):
    every site of every RHS bit for bit."""
    import paper_2301_05518_amd as tl
    wl = synth.workload(3)
    lat = wl.lattices[0]
    dev = torch.device("cuda", 0)
    slices = sorted(set(lat.t_of_rhs))
    Lx, Ly, Lz, Lt = lat.L
    U = torch.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=torch.complex128, device=dev)
    with ThreadPoolExecutor(max_workers=16) as ex:
        futs = {t: ex.submit(synth.gauge_slice, lat.L, lat.links, lat.link_seed, t) for t in slices}
        for t in slices:
            U[t].copy_(torch.from_numpy(futs[t].result()))
    src = torch.from_numpy(lat.sources_array()).to(dev)
    W = ctx.build_twolinks(lat.L, U, "f32", slices=slices)
    del U
    outs, infos = [], []
    for flags in (tl.TL_GRAPH | tl.TL_AUTOTUNE, tl.TL_GRAPH | tl.TL_AUTOTUNE | tl.TL_ONE_STEP):
        job = tl.Job(lat.L, W, lat.t_of_rhs, src.clone(), slices)
        plan = ctx.plan([job], wl.n_steps, wl.sigma, "f32", flags)
        plan.load()
        plan.run()
        plan.store()
        torch.cuda.synchronize()
        infos.append(plan.info())
        outs.append(job.psi)
        plan.close()
    log(f"workload 3: tuned {infos[0]['variant']} x{infos[0]['steps_per_launch']}, "
        f"one-step {infos[1]['variant']} x{infos[1]['steps_per_launch']}")
    assert infos[1]["steps_per_launch"] == 1
    assert torch.equal(outs[0], outs[1])
