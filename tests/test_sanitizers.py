"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: the FP64 oracle under its pins,
and the host code of the C-ABI library (argument validation on a host-only context).  The GPU
code is built as usual: sanitizers here instrument host code only."""
import os
import shutil
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2301_05518_amd")


def gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()


def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    obuild.build(obuild.SRC, lib, extra=["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                          "-fno-omit-frame-pointer", "-g"])
    asan, ubsan = gcc_runtime("libasan.so"), gcc_runtime("libubsan.so")
    if not (os.path.exists(asan) and os.path.exists(ubsan)):
        pytest.skip("gcc sanitizer runtimes not installed")
    code = (
        "import sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from oracle.core import Oracle\n"
        "from tests import oracle_pins\n"
        f"o = Oracle({lib!r})\n"
        "for p in oracle_pins.ALL_PINS:\n"
        "    p(o)\n"
        "print('pins passed:', len(oracle_pins.ALL_PINS))\n"
    )
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "pins passed" in res.stdout
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2301_05518_amd import build as lbuild
    objdir = os.path.join(PKG, "_build")
    device_objs = [os.path.join(objdir, f.replace(".hip", ".o")) for f in lbuild.SOURCES if f != "tl_runtime.hip"]
    if not all(os.path.exists(o) for o in device_objs):
        pytest.skip("library objects not built (run the package build first)")
    clangxx = os.path.join(os.path.dirname(os.path.realpath(lbuild.HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    clangxx = clangxx if os.path.exists(clangxx) else shutil.which("amdclang++") or shutil.which("clang++")
    if clangxx is None:
        pytest.skip("no clang++ for the host driver")
    # the runtime's host code instrumented (each sanitizer flag applies to the host pass only)
    san_host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    rt_obj = str(tmp_path / "tl_runtime_san.o")
    subprocess.run([lbuild.HIPCC, *lbuild.FLAGS, *san_host, "-c", os.path.join(lbuild.CSRC, "tl_runtime.hip"),
                    "-o", rt_obj], check=True, capture_output=True, text=True)
    lib = str(tmp_path / "libtwolink_san.so")
    subprocess.run([lbuild.HIPCC, f"--offload-arch={lbuild.ARCH}", "-shared", "-fPIC", "-o", lib, rt_obj,
                    *device_objs], check=True, capture_output=True, text=True)
    exe = str(tmp_path / "abi_host_check")
    subprocess.run([clangxx, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_host_check.cpp"),
                    "-o", exe, lib, f"-Wl,-rpath,{tmp_path}"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, (res.stdout + res.stderr)[-3000:]
    assert "all passed" in res.stdout
    # the tuning-cache reader (run by tl_create, also on a host-only context) on valid and
    # malformed files: truncated, unbalanced quotes, overflowing or surplus fields, an empty
    # companion tiling, binary bytes, an empty file
    caches = [b'{"k|1": "8,384,32,256,1,1;7,512,16,256,1,1", "k|2": "4,128,1,256,1,0,1"}',
              b'{"k": "8,384', b'"', b'{"k": "99999999999999999999,1,2,3"}',
              b'{"k": "8,384,32,256,1,1;"}', b'{"k": "1,2,3,4,5,6,7,8,9,10"}', b'{"k": "-5,64,1,0"}',
              bytes(range(256)) * 4, b'']
    for i, content in enumerate(caches):
        f = tmp_path / f"tune{i}.json"
        f.write_bytes(content)
        res = subprocess.run([exe], env=dict(env, TL_TUNE_CACHE=str(f)), capture_output=True, text=True,
                             timeout=300)
        assert res.returncode == 0 and "all passed" in res.stdout, (i, (res.stdout + res.stderr)[-3000:])
