"""Host logic of bench.py, on the CPU: the one-GPU refusal, the counter summary and the
accuracy report against the oracle."""
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    msg = json.loads(res.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _write_counters(d, counter, rows):
    os.makedirs(d)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_summary(tmp_path):
    """Only the most-dispatched step-kernel instance is counted; each counter is scaled by
    what it reads for the 1 GiB calibration copy (KiB per dispatch in the files)."""
    main = "void tl::(anonymous namespace)::step_zpipe<1, 3, true>(tl::StepGroup const*, int)"
    other = "void tl::(anonymous namespace)::step_zpipe<5, 3, true>(tl::StepGroup const*, int)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = (1 << 30) // 1024
    fetch = [(main, 300000)] * 6 + [(other, 100)] * 3 + [(copy, gib_kib // 2), (copy, 4)]
    write = [(main, 150000)] * 6 + [(other, 100)] * 3 + [(copy, gib_kib)]
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    rec = bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "workloadX", "7,512,16,256,1,1",
                                   path=str(out))
    assert rec["kernel"] == "step_zpipe<1, 3, true>"
    f, w = rec["counters"]["FETCH_SIZE"], rec["counters"]["WRITE_SIZE"]
    assert f["launches"] == 6 and w["launches"] == 6
    assert abs(f["scale"] - 2.0) < 1e-12 and abs(w["scale"] - 1.0) < 1e-12   # small copy ignored
    assert abs(rec["bytes_per_launch"] - (300000 * 1024 * 2.0 + 150000 * 1024)) < 1e-3
    assert json.load(open(out))["workloadX"]["tile"] == "7,512,16,256,1,1"
    # a second tiling keeps the first one's record under its own key
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "workloadX", "8,384,16,256,1,1",
                             path=str(out))
    allrec = json.load(open(out))
    assert allrec["workloadX"]["tile"] == "8,384,16,256,1,1"
    assert allrec["workloadX|7,512,16,256,1,1"]["tile"] == "7,512,16,256,1,1"


def test_accuracy_against_the_oracle():
    """The accuracy field compares the library's result with the oracle's on the sampled RHS:
    zero for the oracle's own result, the planted relative error for a scaled one."""
    import numpy as np
    import torch
    from paper_2301_05518_amd import synth
    wl = synth.workload(0)
    lat = wl.lattices[0]
    U = bench.links_on_device(torch, lat, torch.device("cpu"), 1)
    _, none = bench.cpu_baseline(lat, wl, U, 1)
    assert none is None
    from oracle import core
    orc = core.get()
    ref = orc.smear(orc.build_twolinks(U[0:1].numpy()), 0, wl.n_steps, wl.sigma, lat.source(0))
    cpu, acc = bench.cpu_baseline(lat, wl, U, 1, gpu_out=np.stack([ref]))
    assert cpu["kind"] == "oracle" and acc["max_rel"] == 0.0 and acc["l2_rel"] == 0.0
    _, acc = bench.cpu_baseline(lat, wl, U, 1, gpu_out=np.stack([ref * (1 + 1e-3)]))
    assert abs(acc["max_rel"] - 1e-3) < 1e-9 and abs(acc["l2_rel"] - 1e-3) < 1e-9


def test_source_hash_ignores_comments_only():
    """The traffic record stays valid across comment and layout edits and not across code edits."""
    assert bench.code_of("int a; // note\n/* block\n comment */  int   b;\n") == "int a; int b;"
    files = {n: f"// {n}\nint f_{len(n)}(int x) {{ return x; }}\n" for n in bench.STEP_SOURCES}
    h0 = bench.kernel_source_hash(files.__getitem__)
    files["tl_step.h"] = files["tl_step.h"].replace("// tl_step.h", "/* reworded */")
    assert bench.kernel_source_hash(files.__getitem__) == h0
    files["tl_step.h"] = files["tl_step.h"].replace("return x;", "return x + 1;")
    assert bench.kernel_source_hash(files.__getitem__) != h0
