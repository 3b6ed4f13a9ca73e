"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the C oracle and the library's host code (the argument validation,
workspace layout and launch set-up of sdtw_api.hip; its device code and the
tile-variant objects are the ordinary ones) with -fsanitize=address,undefined
into _build/sanitize, then runs the CPU tests that exercise them -- every
validation path of the C ABI, the workspace queries and the oracle's pins --
in a child process with the sanitizer runtime preloaded.  Any sanitizer
report fails the test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
CSRC = os.path.join(ROOT, "paper_2403_06931_amd", "csrc")
LLVM = "/opt/rocm/llvm"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

TEST_FILES = ["test_abi_cpu.py", "test_oracle_bruteforce.py", "test_oracle_invariants.py",
              "test_oracle_grad.py", "test_oracle_pruned.py", "test_oracle_quant.py",
              "test_oracle_f16.py"]


def _asan_runtime():
    hits = glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux",
                                  "libclang_rt.asan-x86_64.so"))
    return hits[0] if hits else None


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise AssertionError(" ".join(cmd) + "\n" + res.stdout[-4000:] + res.stderr[-4000:])


def _build_oracle():
    lib = os.path.join(OUT, "liboracle.so")
    _run([os.path.join(LLVM, "bin", "clang"), "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
          "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-Wl,-rpath," + os.path.join(LLVM, "lib"),
          "-o", lib, os.path.join(ROOT, "oracle", "sdtw_oracle.c"), "-lm"])
    return lib


def _build_library():
    """sdtw_api.hip with sanitized host code, linked with the ordinary
    tile-variant objects of the regular build."""
    sys.path.insert(0, CSRC)
    try:
        import build as lib_build
    finally:
        sys.path.pop(0)
    objs = sorted(glob.glob(os.path.join(lib_build.OBJ_DIR, "sdtw_variant_*.o")))
    if len(objs) != len(lib_build.variants()):
        lib_build.build()
        objs = sorted(glob.glob(os.path.join(lib_build.OBJ_DIR, "sdtw_variant_*.o")))
    api_obj = os.path.join(OUT, "sdtw_api_sanitized.o")
    flags = [f for f in lib_build.FLAGS if f != "-O3"]
    _run([HIPCC, *flags, "-O1", "-g",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-omit-frame-pointer",
          "-c", lib_build.API_SOURCE, "-o", api_obj])
    lib = os.path.join(OUT, "libsdtw.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fvisibility=hidden",
          api_obj, *objs, "-o", lib])
    return lib


def test_cpu_tests_clean_under_sanitizers():
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    os.makedirs(OUT, exist_ok=True)
    oracle_lib = _build_oracle()
    sdtw_lib = _build_library()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "SDTW_LIBRARY": sdtw_lib,
        "SDTW_ORACLE_LIBRARY": oracle_lib,
        "CUDA_VISIBLE_DEVICES": "", "HIP_VISIBLE_DEVICES": "",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           *[os.path.join(ROOT, "tests", f) for f in TEST_FILES]]
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-6000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert " passed" in out
