"""Caches for library callers: tl_smear(TL_GRAPH) keeps the plan and captured graph of a job
list and replays it on a repeated call; TL_TUNE_CACHE carries autotuning results to a fresh
process."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2301_05518_amd import synth
from tests.gpu_common import log, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def inputs(k):
    L = (12, 10, 8, 2)
    U = synth.gauge_field(L, "haar", 8100 + k)
    psi = synth.random_field(np.random.default_rng([8101, k]), (3, L[2], L[1], L[0], 3))
    return L, U, [1, 0, 1], psi


@pytest.mark.parametrize("n", [6, 5])
def test_repeated_smear_replays_the_kept_graph(torch, n):
    import paper_2301_05518_amd as tl
    L, U, ts, psi = inputs(n)
    ca, cb = tl.Context(0), tl.Context(0)
    try:
        Wa, Wb = ca.build_twolinks(L, to_dev(U), "f32"), cb.build_twolinks(L, to_dev(U), "f32")
        pa, pb = to_dev(psi), to_dev(psi)
        ja, jb = [tl.Job(L, Wa, ts, pa)], [tl.Job(L, Wb, ts, pb)]
        ca.smear(ja, n, 2.0, "f32", tl.TL_GRAPH)
        first = ca.stats()
        for _ in range(2):
            ca.smear(ja, n, 2.0, "f32", tl.TL_GRAPH)
        again = ca.stats()
        log(f"n={n}: after one call {first}, after three {again}")
        assert first["graphs_captured"] == 1 and first["smear_plan_hits"] == 0
        assert again["graphs_captured"] == 1 and again["smear_plan_hits"] == 2
        for _ in range(3):          # the same three smearings, eager launches, no plan kept
            cb.smear(jb, n, 2.0, "f32", 0)
        torch.cuda.synchronize()
        assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())
        # another field is another job list: a new plan and graph
        pc = to_dev(psi)
        ca.smear([tl.Job(L, Wa, ts, pc)], n, 2.0, "f32", tl.TL_GRAPH)
        assert ca.stats()["graphs_captured"] == 2
        # five distinct job lists displace the first (four are kept)
        extra = [to_dev(psi) for _ in range(3)]
        for q in extra:
            ca.smear([tl.Job(L, Wa, ts, q)], n, 2.0, "f32", tl.TL_GRAPH)
        before = ca.stats()["graphs_captured"]
        ca.smear(ja, n, 2.0, "f32", tl.TL_GRAPH)
        assert ca.stats()["graphs_captured"] == before + 1
    finally:
        ca.close()
        cb.close()


CHILD = r"""
import json, sys
sys.path.insert(0, ROOT)
import numpy as np, torch
import paper_2301_05518_amd as tl
from paper_2301_05518_amd import synth
L = (16, 12, 8, 2)
U = synth.gauge_field(L, "haar", 8200)
psi = synth.random_field(np.random.default_rng([8201]), (3, L[2], L[1], L[0], 3))
c = tl.Context(0)
W = c.build_twolinks(L, torch.from_numpy(U).cuda(), PREC)
p = c.plan([tl.Job(L, W, [0, 0, 1], torch.from_numpy(psi).cuda())], 8, 2.0, PREC, tl.TL_AUTOTUNE | tl.TL_GRAPH)
p.load()
p.run()
torch.cuda.synchronize()
info = p.info()
print(json.dumps({"stats": c.stats(), "tile": [info[k] for k in ("variant", "block", "tz", "grid", "nt", "flip",
                                                                   "tile_width", "group_width")]}))
"""


def test_tune_cache_file_skips_the_sweep_in_a_fresh_process(torch, tmp_path):
    cache = tmp_path / "tune.json"
    env = dict(os.environ, TL_TUNE_CACHE=str(cache))
    code = CHILD.replace("ROOT", repr(ROOT)).replace("PREC", repr("bf16"))
    runs = []
    for k in range(2):
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert res.returncode == 0, res.stderr[-2000:]
        runs.append(json.loads(res.stdout.strip().splitlines()[-1]))
        log(f"process {k}: {runs[-1]}")
    assert runs[0]["stats"]["tune_sweeps"] == 1 and runs[0]["stats"]["tune_hits"] == 0
    assert runs[1]["stats"]["tune_sweeps"] == 0 and runs[1]["stats"]["tune_hits"] == 1
    assert runs[0]["tile"] == runs[1]["tile"]
    rec = json.loads(cache.read_text())
    assert len(rec) == 1
    # "variant,block,tz,grid,nt,flip[,width]", then ";" and the one-step companion of a two-step tiling
    main = list(rec.values())[0].split(";")[0]
    f = [int(x) for x in main.split(",")]
    assert len(f) in (6, 7)
    width = f[6] if len(f) == 7 and f[6] > 0 else runs[0]["tile"][7]
    assert f[:3] + f[4:6] == [runs[0]["tile"][i] for i in (0, 1, 2, 4, 5)]   # the plan reports min(grid, tiles)
    assert width == runs[0]["tile"][6]


def test_tune_cache_entry_that_does_not_apply_is_tuned_again(torch, tmp_path):
    """A cache file entry naming a valid tiling that this plan cannot run (an FP64 plan with two
    RHS per group, and an LDS-staged variant, which takes FP64 groups of one RHS) is dropped:
    the plan is tuned again and the file gets the new winner."""
    cache = tmp_path / "tune.json"
    env = dict(os.environ, TL_TUNE_CACHE=str(cache))
    code = CHILD.replace("ROOT", repr(ROOT)).replace("PREC", repr("f64"))

    def child():
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert res.returncode == 0, res.stderr[-2000:]
        return json.loads(res.stdout.strip().splitlines()[-1])

    first = child()
    rec = json.loads(cache.read_text())
    assert len(rec) == 1 and first["tile"][7] == 2
    key = list(rec)[0]
    cache.write_text(json.dumps({key: "7,512,4,0,0,0"}))
    second = child()
    log(f"first {first}, second {second}")
    assert second["stats"]["tune_sweeps"] == 1 and second["stats"]["tune_hits"] == 0
    if second["tile"][0] >= 5:   # an LDS-staged winner runs every RHS on its own tiles
        assert second["tile"][6] == 1
    assert json.loads(cache.read_text())[key] != "7,512,4,0,0,0"
