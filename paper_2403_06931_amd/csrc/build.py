"""Build step for libsdtw.so (HIP, gfx950).

Compiles the C-ABI library in-tree with hipcc:
  -O3 -ffp-contract=off          every product and sum rounded on its own (no FMA),
                                 so results are bit-identical to a plain FP32 DP;
  -fno-fast-math                 subnormals kept, IEEE min/max;
  -target-feature -packed-fp32-ops   no packed FP32 instructions.
"""
import concurrent.futures as cf
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsdtw.so")
API_SOURCE = os.path.join(HERE, "sdtw_api.hip")
VARIANT_SOURCE = os.path.join(HERE, "sdtw_variant_tu.hip")
VARIANT_LIST = os.path.join(HERE, "sdtw_variants.inc")
OBJ_DIR = os.path.join(os.path.dirname(os.path.dirname(HERE)), "_build", "sdtw")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + HERE,
]


def variants():
    """(index, R, T, W, KS, XL) entries of the X-macro list in sdtw_variants.inc."""
    text = open(VARIANT_LIST).read()
    return [tuple(int(x) for x in m.groups())
            for m in re.finditer(r"X\((\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)\)", text)]


# hipcc's host pass does not know the packed-fp32 feature and says so
_NOISE = "is not a recognized feature for this target"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if _NOISE not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every translation unit (in parallel) and link libsdtw.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    units = [(API_SOURCE, os.path.join(OBJ_DIR, "sdtw_api.o"), [])]
    for i, r, t, w, ks, xl in variants():
        units.append((VARIANT_SOURCE, os.path.join(OBJ_DIR, f"sdtw_variant_{i}.o"),
                      [f"-DSDTW_VARIANT_INDEX={i}", f"-DSDTW_R={r}", f"-DSDTW_T={t}",
                       f"-DSDTW_W={w}", f"-DSDTW_KS={ks}", f"-DSDTW_XL={xl}"]))
    jobs = jobs or min(len(units), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, [HIPCC, *FLAGS, *defs, "-c", src, "-o", obj], verbose)
                for src, obj, defs in units]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fvisibility=hidden",
          *[obj for _, obj, _ in units], "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
