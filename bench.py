#!/usr/bin/env python3
"""Benchmark of the two-link smearing path on one MI355X.

One timed step is one pass of the whole path over a batch of synthetic
input already resident in HBM: two-link build (FP64 product, stored in the
batch precision, for the slices the sources live on), packing of the
complex128 sources into the resident storage format, n smearing steps (one
persistent fused launch per step, all right-hand sides together, replayed
from a HIP graph), FP64 norms of every smeared field, and unpacking back to
complex128.  The plan (resident buffers, work list, tuned tiling, captured
graph) is created once before timing and reused by every pass.

Default workload: 64^3x96 lattice, Haar SU(3) links, 3 colour wall sources
on each of 8 time slices (24 RHS), n = 60, sigma = 6, FP32 storage and
arithmetic.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload 3] [--no-cpu] [--no-plain]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
METRIC = "smeared site-updates/s per RHS + % HBM roofline; FP64 vs batched mixed precision"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-w12", action="store_true",
                    help="skip the twelve-real measurement (profiling runs: one step-kernel instance)")
    ap.add_argument("--cpu-rhs", type=int, default=24, help="RHS in the CPU oracle sample")
    ap.add_argument("--flags", type=int, default=6, help="plan flags (2 graph | 4 autotune)")
    ap.add_argument("--onelink", action="store_true",
                    help="one-link Gaussian smearing (hops of one site, nabla^2 = H - 6) instead of two-link")
    ap.add_argument("--w12", action="store_true",
                    help="twelve-real two-link storage (two rows stored, third rebuilt; SU(3) links)")
    ap.add_argument("--tile", default=None, help="fixed step tiling 'variant,block,tz,grid' (no tuning)")
    ap.add_argument("--prec", choices=("f64", "f32", "f16s", "bf16"), default=None,
                    help="storage precision instead of the workload's first one (e.g. f16s for workload 2)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (their rates, roofline fractions and oracle errors)")
    ap.add_argument("--build-only", action="store_true",
                    help="time only the two-link build of every slice of the workload's first lattice "
                         "(profiling runs of the build kernel)")
    ap.add_argument("--oracle-sample", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script into "
                         "profiles/traffic.json and exit")
    return ap.parse_args()


STEP_SOURCES = ("tl_step.h", "tl_step_f64.hip", "tl_step_f32.hip", "tl_step_f16s.hip", "tl_step_bf16.hip",
                "tl_format.h", "tl_internal.h")


def code_of(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed: what the compiler
    sees (these files hold no string literal containing a comment marker)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(read=None) -> str:
    """Hash of the code (comments and layout aside) of the sources that define the smearing
    step kernels, the kernel the traffic counters measure; the build, pack and reduction
    kernels live elsewhere.  read(name) returns a file's text (default: the working tree)."""
    if read is None:
        def read(name):
            with open(os.path.join(ROOT, "paper_2301_05518_amd", "csrc", name)) as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(code_of(read(f)).encode())
    return h.hexdigest()[:16]


def workload_key(args) -> str:
    return (f"workload{args.workload}" + (f"-{args.prec}" if args.prec else "") + ("-w12" if args.w12 else "")
            + ("-onelink" if args.onelink else ""))


def measured_traffic(workload_key: str, tile: str):
    """HBM bytes per step-kernel launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source with the same tiling (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        allrec = json.load(open(path))
    except (ValueError, OSError):
        return None
    # a record per tiling ("<workload>|<tile>"); the plain workload key holds the latest one
    for rec in (allrec.get(f"{workload_key}|{tile}"), allrec.get(workload_key)):
        if rec and rec.get("kernel_source_hash") == kernel_source_hash() and rec.get("tile") == tile:
            return rec.get("bytes_per_launch")
    return None


COPY_BYTES = 1 << 30          # known-size device copy used to calibrate the byte counters


def _counter_rows(d, counter):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") == counter:
                    rows.append(row)
    return rows


def summarize_counters(fetch_dir, write_dir, workload_key, tile, path=None):
    """Per-launch HBM bytes of the step kernel from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for a plain copy of COPY_BYTES."""
    out = {}
    kernel = None
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        # the step-kernel instance with the most dispatches (the plan the run timed)
        names = [r["Kernel_Name"] for r in rows if "step_" in r["Kernel_Name"]]
        if names and kernel is None:
            kernel = max(set(names), key=names.count)
        step = [float(r["Counter_Value"]) * 1024 for r in rows if r["Kernel_Name"] == kernel]
        copy = [float(r["Counter_Value"]) * 1024 for r in rows
                if "copyBuffer" in r["Kernel_Name"] or "copy_kernel" in r["Kernel_Name"]]
        # the calibration copies only (FETCH_SIZE reads about half of their bytes; host-to-device
        # copies read zero on these counters)
        copy = [c for c in copy if c > 0.1 * COPY_BYTES]
        if not step or not copy:
            raise SystemExit(f"no step-kernel or calibration-copy dispatches with {counter} in {d}")
        scale = COPY_BYTES / (sum(copy) / len(copy))
        out[counter] = {"raw_bytes_per_launch": sum(step) / len(step), "launches": len(step),
                        "copy_raw_bytes": sum(copy) / len(copy), "scale": scale,
                        "bytes_per_launch": sum(step) / len(step) * scale}
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    allrec = json.load(open(path)) if os.path.exists(path) else {}
    allrec[workload_key] = {
        "kernel_source_hash": kernel_source_hash(), "tile": tile,
        "kernel": kernel.replace("void ", "").replace("tl::(anonymous namespace)::", "").split("(")[0],
        "bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"],
        "counters": out,
    }
    allrec[f"{workload_key}|{tile}"] = allrec[workload_key]
    with open(path, "w") as fh:
        json.dump(allrec, fh, indent=1)
    print(json.dumps(allrec[workload_key], indent=1))
    return allrec[workload_key]


def links_on_device(torch, lat, dev, workers):
    """Gauge field [Lt][Lz][Ly][Lx][4][3][3] on the GPU, drawn slice by slice on the host."""
    from paper_2301_05518_amd import synth
    Lx, Ly, Lz, Lt = lat.L
    U = torch.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=torch.complex128, device=dev)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(synth.gauge_slice, lat.L, lat.links, lat.link_seed, t) for t in range(Lt)]
        for t, f in enumerate(futs):
            U[t].copy_(torch.from_numpy(f.result()))
    return U


def cpu_baseline(lat, wl, U_dev, n_rhs_sample, onelink=False, gpu_out=None):
    """The FP64 oracle as it stands, on a bounded sample of the same workload; with gpu_out (the
    library's result for the sampled RHS from the sources, numpy) also the error of that result
    against the oracle's, compared after the timed region."""
    from oracle import checks, core
    orc = core.get()
    ts = lat.t_of_rhs[:n_rhs_sample]
    slices = sorted(set(ts))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    updates = 0
    refs = {}
    for t in slices:
        u = U_dev[t:t + 1].cpu().numpy()
        Wt = None if onelink else orc.build_twolinks(u)
        for r, tr in enumerate(ts):
            if tr != t:
                continue
            if onelink:
                refs[r] = orc.smear_onelink(u, 0, wl.n_steps, wl.sigma, lat.source(r))
            else:
                refs[r] = orc.smear(Wt, 0, wl.n_steps, wl.sigma, lat.source(r))
            updates += lat.V3 * wl.n_steps
    dt = time.perf_counter() - t0
    sample = (f"{len(ts)} of {len(lat.t_of_rhs)} RHS ({len(slices)} slices, {lat.L[0]}^3) x {wl.n_steps} "
              f"steps{'' if onelink else ' incl. their two-link builds'}, FP64, {dt:.1f} s")
    cpu = {"value": updates / dt, "unit": "RHS-site-updates/s", "cores": threads, "kind": "oracle",
           "sample": sample}
    acc = None
    if gpu_out is not None:
        mr = max(checks.max_rel(gpu_out[r], refs[r]) for r in refs)
        l2 = max(checks.l2_rel(gpu_out[r], refs[r]) for r in refs)
        acc = {"max_rel": mr, "l2_rel": l2, "against": "FP64 oracle",
               "sample": f"RHS 0..{len(ts) - 1} of lattice 0 (worst over the sample), one pass from the sources"}
    return cpu, acc


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample_child():
    """Child process (no GPU): the oracle on one RHS of the benchmark workload, whatever threads
    OMP_NUM_THREADS gives it; prints one JSON line."""
    from oracle import core
    from paper_2301_05518_amd import synth
    wl = synth.workload(3)
    lat = wl.lattices[0]
    t = lat.t_of_rhs[0]
    orc = core.get()
    u = synth.gauge_slice(lat.L, lat.links, lat.link_seed, t)[None]
    t0 = time.perf_counter()
    W = orc.build_twolinks(u)
    orc.smear(W, 0, wl.n_steps, wl.sigma, lat.source(0))
    dt = time.perf_counter() - t0
    print(json.dumps({"value": lat.V3 * wl.n_steps / dt, "seconds": dt,
                      "sample": f"RHS 0 (one 64^3 slice) x {wl.n_steps} steps incl. its two-link build, FP64"}))


def oracle_single_thread():
    """The oracle's single-thread rate, timed in a child process with OMP_NUM_THREADS=1."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample"], env=env,
                         capture_output=True, text=True, timeout=300)
    if res.returncode != 0:
        log(f"[bench] single-thread oracle sample failed: {res.stderr[-500:]}")
        return None
    rec = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": rec["value"], "unit": "RHS-site-updates/s", "cores": 1, "sample": rec["sample"],
            "seconds": round(rec["seconds"], 2)}


STEP_KINDS = 2    # the step kernels' load and store kinds: cached loads, nontemporal stores


def stream_ceiling(ctx, torch, dev, nbytes):
    """Streaming probe of the library (tl_stream_time): four input planes, one output plane, the
    step's read/write mix, over nbytes in all; every load/store kind and three grid sizes."""
    nbytes = max(nbytes // (5 * 256) * 5 * 256, 5 * 256)
    buf = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    kinds_name = {0: "cached loads, cached stores", 1: "nontemporal loads, cached stores",
                  2: "cached loads, nontemporal stores", 3: "nontemporal loads, nontemporal stores"}
    rows = []
    for kinds in range(4):
        for per_cu in (4, 16, 64):
            ms = ctx.stream_time(buf, n_in=4, kinds=kinds, grid=per_cu * n_cu, reps=5)
            rows.append({"kinds": kinds_name[kinds], "grid": per_cu * n_cu,
                         "GBs": round(nbytes / (ms * 1e-3) / 1e9, 1), "step_kinds": kinds == STEP_KINDS})
    del buf
    torch.cuda.empty_cache()
    best = max(rows, key=lambda r: r["GBs"])
    same = max((r for r in rows if r["step_kinds"]), key=lambda r: r["GBs"])
    return {"ceiling_GBs": best["GBs"], "ceiling_kinds": best["kinds"], "step_kinds_GBs": same["GBs"],
            "bytes": nbytes, "mix": "4 reads : 1 write", "configs": rows}


def compact_lattice(lat):
    """The lattice cut down to the slices its RHS live on: links of those slices only (drawn as in
    the full field), the RHS's slices renumbered.  A step on a slice never reads another slice,
    so the smearing work and its result are those of the full lattice."""
    from paper_2301_05518_amd import synth
    slices = sorted(set(lat.t_of_rhs))
    U = np.stack([synth.gauge_slice(lat.L, lat.links, lat.link_seed, t) for t in slices])
    L = tuple(lat.L[:3]) + (len(slices),)
    return L, U, [slices.index(t) for t in lat.t_of_rhs]


TILE_KEYS = ("variant", "block", "tz", "grid", "nt", "flip")


def tile_text(info) -> str:
    """A plan's tiling as TL_TILE reads it (the RHS-per-group field when groups are split)."""
    t = ",".join(str(info[k]) for k in TILE_KEYS)
    return t + (f",{info['tile_width']}" if info["tile_width"] != info["group_width"] else "")


def tile_dict(info) -> dict:
    return {**{k: info[k] for k in TILE_KEYS}, "width": info["tile_width"]}


KERNEL_NAMES = ["step_direct", "step_zmarch", "step_zring", "step_zfront", "step_rolled", "step_zlds", "step_zchain",
                "step_zpipe", "step_fuse2"]


def measure_workload(ctx, torch, tl, dev, index, prec, plain=False, passes=5):
    """Step and pass rates, roofline fraction and oracle error of one of the other workloads."""
    from oracle import checks, core
    from paper_2301_05518_amd import synth
    wl = synth.workload(index)
    orc = core.get()
    lats = [compact_lattice(lat) for lat in wl.lattices]
    srcs = [lat.sources_array() for lat in wl.lattices]
    jobs = []
    for (L, U, ts), src in zip(lats, srcs):
        Ud = torch.from_numpy(U).to(dev)
        jobs.append((L, Ud, ts, torch.from_numpy(src).to(dev)))
    tjobs = [tl.Job(L, ctx.build_twolinks(L, Ud, prec), ts, psi) for L, Ud, ts, psi in jobs]
    plan = ctx.plan(tjobs, wl.n_steps, wl.sigma, prec, tl.TL_GRAPH | tl.TL_AUTOTUNE)
    # one pass from the sources, checked against the oracle on every RHS
    plan.load()
    plan.run()
    plan.store()
    torch.cuda.synchronize()
    mr = l2 = 0.0
    outs = [j.psi.cpu().numpy() for j in tjobs]
    oracle_s = 0.0
    for (L, U, ts), out, src in zip(lats, outs, srcs):
        t0 = time.perf_counter()
        Wo = orc.build_twolinks(U)
        refs = [orc.smear(Wo, t, wl.n_steps, wl.sigma, src[r]) for r, t in enumerate(ts)]
        oracle_s += time.perf_counter() - t0
        for r, ref in enumerate(refs):
            mr = max(mr, checks.max_rel(out[r], ref))
            l2 = max(l2, checks.l2_rel(out[r], ref))

    def one_pass():
        for (L, Ud, ts, _), j in zip(jobs, tjobs):
            ctx.build_twolinks(L, Ud, prec, W=j.W)
        plan.load()
        plan.run()
        plan.reduce("norm2")
        plan.store()

    one_pass()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(passes):
        one_pass()
    e1.record()
    e1.synchronize()
    pass_ms = e0.elapsed_time(e1) / passes
    step_ms = plan.time(reps=5)
    info = plan.info()
    # algorithmic bytes: those of every RHS-site-update (W, the input and the output once each)
    spl = info["steps_per_launch"]
    launch_ms = step_ms * wl.n_steps / ((wl.n_steps + spl - 1) // spl)
    gbs = info["bytes_per_step"] / (step_ms * 1e-3) / 1e9
    rec = {"workload": wl.name, "storage": prec, "rhs": sum(len(ts) for _, _, ts in lats),
           "step_us": round(step_ms * 1e3, 2), "launch_us": round(launch_ms * 1e3, 2), "steps_per_launch": spl,
           "pass_ms": round(pass_ms, 4),
           "value": wl.rhs_site_updates / (pass_ms * 1e-3),
           "smear_only_rate": info["rhs_sites"] / (step_ms * 1e-3),
           "algorithmic_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
           "working_set_MB": round(info["bytes_per_step"] / 1e6, 1),
           "max_rel": mr, "l2_rel": l2,
           "tile": tile_dict(info),
           "oracle": {"value": wl.rhs_site_updates / oracle_s, "unit": "RHS-site-updates/s",
                      "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                      "seconds": round(oracle_s, 2),
                      "sample": "every RHS x every step, with the two-link build of its slices, FP64"}}
    plan.close()
    if plain:
        pj = [tl.Job(L, ctx.build_twolinks(L, Ud, "f64"), ts, psi) for L, Ud, ts, psi in jobs]
        p64 = ctx.plan(pj, wl.n_steps, wl.sigma, "f64", tl.TL_PLAIN | tl.TL_AUTOTUNE)
        p64.load()
        launch_ms = p64.time(reps=1)
        pinfo = p64.info()
        plain_ms = launch_ms * pinfo["launches_per_step"] * wl.n_steps
        rec["plain_fp64_smear_ms"] = round(plain_ms, 4)
        rec["speedup_over_plain_fp64"] = round(plain_ms / (step_ms * wl.n_steps), 3)
        p64.close()
    del jobs, tjobs
    torch.cuda.empty_cache()
    log(f"[bench]   {wl.name} {prec}: step {rec['step_us']} us ({rec['frac']:.3f} of HBM, "
        f"{rec['working_set_MB']} MB/step), pass {rec['pass_ms']} ms, max-rel {mr:.2e}")
    return rec


def build_only(args):
    """Two-link build of every slice of the workload's first lattice, timed with HIP events (the
    command that profiles the build kernel alone), plus the calibration copy for the counters."""
    import torch
    import paper_2301_05518_amd as tl
    from paper_2301_05518_amd import synth
    dev = torch.device("cuda", 0)
    wl = synth.workload(args.workload)
    lat = wl.lattices[0]
    prec = (args.prec or wl.precisions[0]) + ("-w12" if args.w12 else "")
    log(f"[bench] build only: {lat.L}, {prec}")
    U = links_on_device(torch, lat, dev, min(16, os.cpu_count() or 1))
    ctx = tl.Context(0)
    W = ctx.build_twolinks(lat.L, U, prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ctx.build_twolinks(lat.L, U, prec, W=W)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nbytes = lat.V3 * lat.L[3] * 3 * 144 + tl.twolinks_bytes(lat.L, prec, lat.L[3])
    ca = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    torch.empty_like(ca).copy_(ca)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": "build_twolinks", "lattice": list(lat.L), "storage": prec, "ms": round(ms, 4),
                      "algorithmic_bytes": nbytes, "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                      "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}), flush=True)
    ctx.close()


def main():
    args = parse()
    if args.oracle_sample:
        oracle_sample_child()
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, workload_key(args), args.tile)
        return
    if args.tile:
        os.environ["TL_TILE"] = args.tile
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU: the path shards by time slice with no "
                                   "exchange, but multi-GPU runs are not implemented; use --gpus 1"}))
        sys.exit(2)
    if args.build_only:
        build_only(args)
        return

    import torch
    import paper_2301_05518_amd as tl
    from paper_2301_05518_amd import synth

    dev = torch.device("cuda", 0)
    wl = synth.workload(args.workload)
    base = args.prec or wl.precisions[0]
    form = ("-w12" if args.w12 else "") + ("-onelink" if args.onelink else "")
    prec = base + form

    def links(lat, U, pr, slices=None, W=None):
        """Two-link field, or the packed links for one-link smearing."""
        fn = ctx.pack_links if pr.endswith("-onelink") else ctx.build_twolinks
        return fn(lat.L, U, pr, slices=slices, W=W)

    workers = min(16, os.cpu_count() or 1)
    log(f"[bench] workload {args.workload}: {wl.name}; drawing inputs")
    t_in = time.perf_counter()
    jobs_in = []
    for lat in wl.lattices:
        U = links_on_device(torch, lat, dev, workers)
        psi = torch.from_numpy(lat.sources_array()).to(dev)
        slices = sorted(set(lat.t_of_rhs))
        jobs_in.append((lat, U, psi, slices))
    torch.cuda.synchronize()
    U_first = jobs_in[0][1]
    log(f"[bench] inputs resident in HBM ({time.perf_counter() - t_in:.1f} s)")

    ctx = tl.Context(0)
    jobs = []
    for lat, U, psi, slices in jobs_in:
        W = links(lat, U, prec, slices)
        jobs.append(tl.Job(lat.L, W, lat.t_of_rhs, psi, slices))
    plan = ctx.plan(jobs, wl.n_steps, wl.sigma, prec, args.flags)
    n_rhs = sum(len(l.t_of_rhs) for l in wl.lattices)

    run_events = []   # HIP events around the smearing launches of each timed pass

    def one_pass(timed=False):
        for (lat, U, _, slices), j in zip(jobs_in, jobs):
            links(lat, U, prec, slices, j.W)
        plan.load()
        if timed:   # the library queues on torch's current stream, where these events go
            ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ea.record()
            plan.run()
            eb.record()
            run_events.append((ea, eb))
        else:
            plan.run()
        norms = plan.reduce("norm2")
        plan.store()
        return norms

    # the result of one pass from the sources, for the accuracy check against the oracle
    # (the later passes start from the previous pass's output: same work, other values)
    n_sample = min(args.cpu_rhs, len(wl.lattices[0].t_of_rhs))
    first_out = None
    if not args.no_cpu:
        one_pass()
        torch.cuda.synchronize()
        first_out = jobs[0].psi[:n_sample].cpu().numpy()

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    log("[bench] warm; timing")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        norms = one_pass(timed=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    updates = wl.rhs_site_updates
    value = updates / (ms_per_step * 1e-3)
    finite = bool(torch.isfinite(norms).all().item())
    log(f"[bench] pass {ms_per_step:.3f} ms -> {value:.4e} RHS-site-updates/s")

    # achievable streaming bandwidth: a plain device copy of a known size (also the
    # calibration dispatch for the byte counters of a rocprofv3 --pmc run)
    ca = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        cb.copy_(ca)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * COPY_BYTES * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    torch.cuda.empty_cache()
    # achievable rate of the step's read/write mix: the library's streaming probe over as many
    # bytes as one step moves
    ceiling = stream_ceiling(ctx, torch, dev, int(plan.info()["bytes_per_step"]))
    log(f"[bench] streaming probe: best {ceiling['ceiling_GBs']} GB/s ({ceiling['ceiling_kinds']}), "
        f"{ceiling['step_kinds_GBs']} GB/s with the step's load and store kinds")

    # dominant kernel: the smearing step.  Its average launch duration comes from the HIP events
    # around the smearing launches inside the timed passes above (the n launches of a pass
    # replayed from the graph, gaps between them included); back-to-back replays outside the
    # timed region are reported beside it.
    info = plan.info()
    # one launch runs spl steps (2: the two-step kernel, which reads W and its input once and
    # writes only the second step's output); the algorithmic bytes are those of the RHS-site-
    # updates it performs, 120 B each at FP32 and three RHS per W load (W, the input and the
    # output once per update), so a two-step launch counts two steps' bytes against its time
    spl = info["steps_per_launch"]
    launches = max(1, info["launches_per_step"] * ((wl.n_steps + spl - 1) // spl))
    step_ms = sum(a.elapsed_time(b) for a, b in run_events) / len(run_events) / launches
    isolated_ms = plan.time(reps=3) * wl.n_steps / launches
    algo_bytes = info["bytes_per_step"] * spl
    achieved = algo_bytes / (step_ms * 1e-3) / 1e9
    key = workload_key(args)
    tile = tile_text(info)
    traffic = measured_traffic(key, tile)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[info["variant"]], "steps_per_launch": spl,
                "algorithmic_bytes_per_launch": algo_bytes,
                # what one launch must move at the least (W once, its input and its output once),
                # and the share of HBM bandwidth the launch's counted traffic uses
                "launch_min_bytes": info["bytes_per_step"],
                "traffic_GBs": round(traffic / (step_ms * 1e-3) / 1e9, 1) if traffic else None,
                "traffic_frac": round(traffic / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "avg_launch_ms": round(step_ms, 5), "isolated_launch_ms": round(isolated_ms, 5),
                "copy_GBs": round(copy_gbs, 1), "ceiling_GBs": ceiling["ceiling_GBs"],
                # the rate of the launch's counted traffic (else of its least bytes) over the best stream
                "frac_of_ceiling": round((traffic or info["bytes_per_step"]) / (step_ms * 1e-3) / 1e9
                                         / ceiling["ceiling_GBs"], 4),
                "ceiling": {k: ceiling[k] for k in ("ceiling_kinds", "step_kinds_GBs", "bytes", "mix", "configs")}}
    log(f"[bench] step kernel ({spl} step(s) per launch) {step_ms * 1e3:.1f} us per launch, "
        f"{achieved:.0f} GB/s algorithmic")
    if spl == 2 and not args.no_extra:
        # the fastest one-step tiling on the same resident data, for comparison
        p1 = ctx.plan(jobs, wl.n_steps, wl.sigma, prec, args.flags | tl.TL_ONE_STEP)
        p1.load()
        ms1 = p1.time(reps=3)
        i1 = p1.info()
        a1 = i1["bytes_per_step"] / (ms1 * 1e-3) / 1e9
        roofline["one_step"] = {"kernel": KERNEL_NAMES[i1["variant"]], "launch_ms": round(ms1, 5),
                                "achieved": round(a1, 1), "frac": round(a1 / HBM_PEAK_GBS, 4),
                                "tile": tile_text(i1)}
        p1.close()
        log(f"[bench] fastest one-step tiling: {roofline['one_step']}")

    # the pieces of a pass, timed alone on the same stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=3):
        fn()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    build_ms = timed(lambda: [links(lat, U, prec, s, j.W)
                              for (lat, U, _, s), j in zip(jobs_in, jobs)])
    pack_ms = timed(plan.load)
    unpack_ms = timed(plan.store)
    norm_ms = timed(lambda: plan.reduce("norm2"))
    smear_ms = step_ms * launches
    lat0, U0 = jobs_in[0][0], jobs_in[0][1]
    Wall = links(lat0, U0, prec)
    build_all_ms = timed(lambda: links(lat0, U0, prec, W=Wall), reps=2)
    # the build's own roofline: U's three spatial links read once (FP64), W written once
    build_bytes = lat0.V3 * lat0.L[3] * 3 * 144 + tl.twolinks_bytes(lat0.L, prec, lat0.L[3])
    build_gbs = build_bytes / (build_all_ms * 1e-3) / 1e9
    del Wall
    torch.cuda.empty_cache()
    smear_rate = info["rhs_sites"] * wl.n_steps / (smear_ms * 1e-3)

    # plain FP64: one RHS per launch, RHS in succession, eager launches
    plain = None
    if not args.no_plain:
        pjobs = []
        for (lat, U, psi, slices) in jobs_in:
            W64 = links(lat, U, "f64" + form.replace("-w12", ""), slices)
            pjobs.append(tl.Job(lat.L, W64, lat.t_of_rhs, psi, slices))
        # one RHS per launch, RHS in succession, eager launches, FP64 storage; its tiling tuned
        # for that case like the batched plan's, so the speedup compares tuned with tuned
        p64 = ctx.plan(pjobs, wl.n_steps, wl.sigma, "f64" + form.replace("-w12", ""), tl.TL_PLAIN | tl.TL_AUTOTUNE)
        p64.load()
        launch_ms = p64.time(reps=1)
        pinfo = p64.info()
        plain_ms = launch_ms * pinfo["launches_per_step"] * wl.n_steps
        plain_rate = pinfo["rhs_sites"] * wl.n_steps / (plain_ms * 1e-3)
        plain = {"smear_ms": round(plain_ms, 3), "rate": plain_rate,
                 "launch_us": round(launch_ms * 1e3, 2),
                 "tile": tile_dict(pinfo),
                 "achieved_GBs": round(pinfo["bytes_per_step"] / (plain_ms / wl.n_steps * 1e-3) / 1e9, 1),
                 "speedup_of_batched": round(smear_rate / plain_rate, 3)}
        p64.close()
        del pjobs
        torch.cuda.empty_cache()
        log(f"[bench] plain fp64 {plain_rate:.3e} /s; batched {prec} is {smear_rate / plain_rate:.2f}x")

    # the same smearing with twelve-real two-links (rows 0, 1 stored, row 2 rebuilt), its own
    # tuned plan on the same resident inputs: reported beside the headline, not as `value`
    w12 = None
    if not args.w12 and not args.no_w12:
        wprec = base + "-w12" + form
        wjobs = [tl.Job(lat.L, links(lat, U, wprec, slices), lat.t_of_rhs, psi, slices)
                 for (lat, U, psi, slices) in jobs_in]
        pw = ctx.plan(wjobs, wl.n_steps, wl.sigma, wprec, args.flags)
        pw.load()
        w_ms = pw.time(reps=3)
        winfo = pw.info()
        w12 = {"storage": wprec, "step_ms": round(w_ms, 5),
               "algorithmic_bytes_per_launch": winfo["bytes_per_step"],
               "achieved_GBs": round(winfo["bytes_per_step"] / (w_ms * 1e-3) / 1e9, 1),
               "frac": round(winfo["bytes_per_step"] / (w_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "smear_only_rate": winfo["rhs_sites"] / (w_ms * 1e-3),
               "tile": tile_dict(winfo)}
        pw.close()
        del wjobs
        torch.cuda.empty_cache()
        log(f"[bench] twelve-real two-links: step {w_ms * 1e3:.1f} us")

    # the other workloads: each on the slices its RHS live on, in its own tuned graph plan
    extra = None
    if not args.no_extra and args.workload == 3 and not args.onelink and not args.w12 and not args.prec:
        log("[bench] other workloads")
        del jobs_in, jobs
        plan.close()
        torch.cuda.empty_cache()
        extra = {}
        for key, index, pr, pl in (("8^3x8_f64", 0, "f64", False), ("32^3x64_f64", 1, "f64", True),
                                   ("48^3x96_f32", 2, "f32", True), ("48^3x96_f16s", 2, "f16s", True),
                                   ("uneven_bf16", 4, "bf16", True)):
            extra[key] = measure_workload(ctx, torch, tl, dev, index, pr, plain=pl)

    cpu = accuracy = None
    if not args.no_cpu:
        log("[bench] CPU oracle sample")
        cpu, accuracy = cpu_baseline(wl.lattices[0], wl, U_first, n_sample, args.onelink, first_out)
        cpu["cpu_model"] = cpu_model()
        if not args.onelink:
            cpu["single_thread"] = oracle_single_thread()
        log(f"[bench] oracle {cpu['value']:.3e} /s on {cpu['cores']} threads; "
            f"max-rel {accuracy['max_rel']:.2e} against it")

    lat = wl.lattices[0]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RHS-site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": base,
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "lattices": [list(l.L) for l in wl.lattices],
            "rhs": n_rhs,
            "n_smear": wl.n_steps,
            "sigma": wl.sigma,
            "storage": prec,
            "accumulate": "f64" if base == "f64" else "f32",
            "operator": "one-link Laplacian H - 6" if args.onelink else "two-link Laplacian (eq. tlLapl1)",
            "pass": "build(source slices) + pack + n steps + FP64 norms + unpack",
            "tile": {**tile_dict(info), "n_tiles": info["n_tiles"], "group_width": info["group_width"]},
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "breakdown_ms": {"build": round(build_ms, 4), "pack": round(pack_ms, 4), "smear": round(smear_ms, 4),
                         "norms": round(norm_ms, 4), "unpack": round(unpack_ms, 4),
                         "build_all_slices": round(build_all_ms, 4)},
        "build_roofline": {"bound": "hbm", "achieved": round(build_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(build_gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": build_bytes,
                           "slices": lat0.L[3]},
        "smear_only_rate": smear_rate,
        "plain_fp64": plain,
        "twelve_real": w12,
        "workloads": extra,
        "finite": finite,
    }
    print(json.dumps(out), flush=True)
    if extra is None:
        plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
