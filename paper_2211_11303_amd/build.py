"""Build libhlu.so for gfx950 in-tree (hipcc, no JIT caches).

Usage: python -m paper_2211_11303_amd.build   (or call build())
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhlu.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["mesh.cpp", "structure.cpp", "plan.cpp", "chain_sched.cpp", "api.cpp", "gmres.cpp", "batch.cpp",
           "server.cpp", "autotune.cpp", "hinverse.cpp",
           "kernels_hlu.hip",
           "kernels_vec.hip", "kernels_chain.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(HERE, "..", "include")]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# sources (libhlu_asan.so): every -fsanitize flag applies to the host pass
# only, the device code is built as usual.  For CPU runs of the host logic
# (planner, schedules, assembly) with the ASan runtime preloaded; see
# tests/test_lib_asan.py.
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
ASAN_OUT = os.path.join(HERE, "libhlu_asan.so")
ASAN_BUILD_DIR = os.path.join(HERE, "_build_asan")


def _compile(src, sanitize=False):
    bdir = ASAN_BUILD_DIR if sanitize else BUILD_DIR
    obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
    flags = COMMON + (SAN_HOST if sanitize else [])
    cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + flags + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{errs}")
    return obj


def build(verbose=False, sanitize=False):
    bdir, out = (ASAN_BUILD_DIR, ASAN_OUT) if sanitize else (BUILD_DIR, OUT)
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950"] + (SAN_HOST if sanitize else []) + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stderr)
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--asan" in sys.argv)
    sys.exit(0)
