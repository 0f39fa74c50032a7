"""Build libfsmp.so (the sampler) and liblds_probe.so (the LDS bandwidth probe that
bench.py uses for its roofline) in-tree with hipcc for gfx950 (MI355X).

    python -m paper_2403_03156_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfsmp.so")
PROBE_LIB = os.path.join(HERE, "liblds_probe.so")
SOURCES = ["fsmp_api.hip", "fsmp_kernels.hip", "fsmp_server.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def _compile(out, srcs, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _compile(LIB, sources(), verbose)
    _compile(PROBE_LIB, [os.path.join(CSRC, "lds_probe.hip")], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
