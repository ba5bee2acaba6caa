"""Seeded random cases through the C ABI: ragged shapes, uneven RHS patterns, every storage
precision and link form, random tilings of every step variant (one and two steps per launch).
Each tiling must give the direct kernel's bits; the direct kernel must match the FP64 oracle
within the precision's bound."""
import numpy as np
import pytest

from paper_2301_05518_amd import synth
from tests.gpu_common import errors, gpu_smear, log, to_dev, tol

pytestmark = pytest.mark.gpu

N_CASES = 64
FORMS = ["f64", "f32", "f16s", "bf16", "f32-w12", "bf16-w12", "f64-onelink", "f32-onelink", "f16s-w12-onelink"]


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


def draw_case(k):
    rng = np.random.default_rng([77011, k])
    form = FORMS[k % len(FORMS)]
    extents = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 13, 16, 17, 24]
    L = tuple(int(rng.choice(extents)) for _ in range(3)) + (int(rng.integers(1, 4)),)
    n_rhs = int(rng.integers(1, 8))
    ts = [int(t) for t in rng.integers(0, L[3], size=n_rhs)]
    if form.startswith("f64"):
        ts = sorted(set(ts))          # FP64 LDS kernels take groups of one RHS
    n = int(rng.integers(1, 9))
    one = form.endswith("onelink")
    sigma = float(rng.uniform(0.05, 1.0 / 6.0 if one else 2.0 / 3.0)) * n
    variants = [0, 4, 7] if one else [0, 1, 2, 3, 4, 5, 6, 7]
    tiles = []
    for _ in range(3):
        v = int(rng.choice(variants))
        block = int(rng.choice([64, 128, 256, 512] if v >= 5 else [64, 128, 192, 256]))
        tz = int(rng.integers(1, 17))
        grid = int(rng.choice([0, 0, 3, 8, 64]))
        tiles.append(f"{v},{block},{tz},{grid},{int(rng.integers(0, 2))},{int(rng.integers(0, 2))}")
    # and a two-step tiling (variant 8: two steps per launch, a one-step launch for an odd last step)
    block = int(rng.choice([192, 256, 320, 384, 448, 512]))
    tz, grid = int(rng.integers(1, 17)), int(rng.choice([0, 0, 3, 8, 64]))
    tiles.append(f"8,{block},{tz},{grid},{int(rng.integers(0, 2))},{int(rng.integers(0, 2))}")
    if k >= 24 and k % 4 == 0:   # rows of 64 sites: the two-step kernels built for that row length
        L = (64,) + L[1:]
        tiles += ["8,512,4,0,1,1", "8,384,3,0,0,1"]
    return form, L, ts, n, sigma, tiles


@pytest.mark.parametrize("k", range(N_CASES))
def test_random_case(ctx, orc, torch, k, monkeypatch):
    import paper_2301_05518_amd as tl
    form, L, ts, n, sigma, tiles = draw_case(k)
    U = synth.gauge_field(L, "haar", 91000 + k)
    psi = synth.random_field(np.random.default_rng([77012, k]), (len(ts), L[2], L[1], L[0], 3))
    log(f"case {k}: {form} L={L} ts={ts} n={n} sigma={sigma:.3f} tiles={tiles}")
    lat = [(L, U, ts, psi)]

    def run(tile):
        monkeypatch.setenv("TL_TILE", tile)
        if form.endswith("onelink"):
            jobs = [tl.Job(L, ctx.pack_links(L, to_dev(U), form), ts, to_dev(psi))]
            ctx.smear(jobs, n, sigma, form)
            torch.cuda.synchronize()
            return jobs[0].psi.cpu().numpy()
        return gpu_smear(ctx, lat, n, sigma, form)[0]

    ref_gpu = run("0,64,1,0")
    for tile in tiles:
        try:
            out = run(tile)
        except tl.TwolinkError as e:   # a tiling that does not apply to this case (no row tiling, FP64 width)
            assert "TL_ERR_UNSUPPORTED" in str(e)
            log(f"  tile {tile}: not applicable")
            continue
        assert np.array_equal(out, ref_gpu), tile
    if form.endswith("onelink"):
        ref = orc.smear_onelink_batch(U, ts, n, sigma, psi)
    else:
        ref = orc.smear_batch(orc.build_twolinks(U), ts, n, sigma, psi)
    mr, l2 = errors(ref_gpu, ref)
    base = form.replace("-onelink", "")
    log(f"  max-rel {mr:.3e} l2-rel {l2:.3e} (bar {tol(base, n):.2e})")
    assert mr < tol(base, n) and l2 < tol(base, n)
