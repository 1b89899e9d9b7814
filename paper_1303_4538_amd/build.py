"""Build libsip.so in-tree with hipcc for gfx950.

    python -m paper_1303_4538_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["sip_kernels.hip", "sip_api.hip", "sip_server.hip", "sip_blocks.hip", "sip_sched.cpp", "sip_host.cpp"]
OUT = os.path.join(HERE, "libsip.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


def hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose=False):
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", tmp] + srcs + [
        "-lpthread", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libsip.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
