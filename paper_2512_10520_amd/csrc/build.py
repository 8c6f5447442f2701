"""Build libmt.so (HIP, gfx950) next to the Python package.

    python -m paper_2512_10520_amd.csrc.build [--verbose]

Every HIP source is compiled with FMA contraction off (fused multiply-adds
are explicit in the source, so inlined copies of the step agree bit for bit)
and with packed FP32 instructions disabled.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libmt.so")
SOURCES = ["mt_api.hip", "mt_kernels.hip"]
# Measurement helper (gather microbenchmark), a library of its own.
GBENCH_LIB = os.path.join(PKG, "libmt_gbench.so")
GBENCH_SOURCES = ["gbench.hip"]
ARCH = os.environ.get("MT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _compile(sources, out, verbose):
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", HERE,
           "-o", out + ".tmp"] + [os.path.join(HERE, s) for s in sources]
    if verbose:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    """Compile libmt.so (the transport) and libmt_gbench.so (measurement)."""
    _compile(SOURCES, LIB, verbose)
    _compile(GBENCH_SOURCES, GBENCH_LIB, False)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
