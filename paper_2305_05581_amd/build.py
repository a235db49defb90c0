"""Build the gfx950 shared library ``libtns.so`` in the package directory.

    python -m paper_2305_05581_amd.build

Every source under ``csrc/`` is compiled for gfx950 only; packed FP32
instructions are disabled (``-packed-fp32-ops``).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtns.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
SOURCES = ["tasklist.hip", "fwd.hip", "apply.hip", "davidson.hip", "peak.hip", "renorm.hip", "ttcache.hip", "su2.hip"]


def flags():
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
            "-I", os.path.join(HERE, "..", "include")]


def build(verbose=False, jobs=4):
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = []
    procs = []
    for s in srcs:
        o = os.path.join(CSRC, s.replace(".hip", ".o"))
        cmd = [HIPCC] + flags() + ["-c", os.path.join(CSRC, s), "-o", o]
        objs.append(o)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode())
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        if verbose and out:
            sys.stderr.write(out.decode())
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout.decode())
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
