"""The host logic of the library (assembly, cluster and block trees, the
task planner, the persistent-solve schedules, the Schulz-inverse plans)
under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU library tests
run against the host-sanitized build (paper_2211_11303_amd/build.py
--asan, every -fsanitize applied to the host pass only) in a child process
with the sanitizer runtime preloaded; any report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if not os.path.exists(clang):
        return None
    r = subprocess.run([clang, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_host_logic_under_sanitizers():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime in this image")
    sys.path.insert(0, ROOT)
    from paper_2211_11303_amd import build
    lib = build.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HLU_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_lib_cpu.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
