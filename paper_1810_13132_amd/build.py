"""Build libvbdr.so (HIP, gfx950) and the stream generator in-tree.

    python -m paper_1810_13132_amd.build
"""
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libvbdr.so")
ARCH = os.environ.get("VBDR_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def hip_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
            # keep the compiler from forming packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def build_hip(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, n) for n in ("vbdr.hip", "vbdr_learn.hip", "vbdr_batch.hip")]
    cmd = [hipcc()] + hip_flags() + ["-shared", "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_all(verbose: bool = False):
    from paper_1810_13132_amd import synth
    synth.build(verbose=verbose)
    return build_hip(verbose=verbose)


if __name__ == "__main__":
    build_all(verbose=True)
