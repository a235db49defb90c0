"""The library's host code (validation, layout, task listing and planning of
products, renormalisation steps, out-of-HBM plans and spin-adapted problems)
under AddressSanitizer and UndefinedBehaviorSanitizer: the sources are built
once more with the sanitizers on the host side only, and
``sanitized_host_checks.py`` runs in a child process with the sanitizer
runtime preloaded.  No GPU needed."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_sanitizers(tmp_path):
    rt = _runtime()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or the sanitizer runtime not available")
    sys.path.insert(0, ROOT)
    from paper_2305_05581_amd.build import SOURCES, CSRC, ARCH
    common = ["-O1", "-g", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-I", os.path.join(ROOT, "include")]
    objs = [str(tmp_path / s.replace(".hip", ".o")) for s in SOURCES]

    def compile_one(i):
        cmd = [HIPCC] + common + ["-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)

    with ThreadPoolExecutor(max_workers=4) as ex:
        for r in ex.map(compile_one, range(len(SOURCES))):
            assert r.returncode == 0, r.stdout.decode()[-2000:]
    lib = str(tmp_path / "libtns_sanitized.so")
    r = subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", "-o", lib] + objs,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    assert r.returncode == 0, r.stdout.decode()[-2000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitized_host_checks.py"), lib], env=env,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=600)
    out = r.stdout.decode()
    assert r.returncode == 0 and "sanitized host checks passed" in out, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
