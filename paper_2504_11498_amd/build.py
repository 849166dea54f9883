"""Build libmrep.so in-tree for gfx950 (hipcc for the kernels, g++ for the host
decomposition, which is compiled without floating-point contraction so that its
FP64 arithmetic is deterministic)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmrep.so")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # packed FP32 instructions are disabled for all device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# the screen's minimum over MFMA results: no NaN canonicalisation, MFMA results in VGPRs
SCREEN_FLAGS = ["-fno-honor-nans", "-mllvm", "-amdgpu-mfma-vgpr-form=1"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    host_o = os.path.join(BUILD, "mrep_host.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-I", INC, "-c",
          os.path.join(CSRC, "mrep_host.cpp"), "-o", host_o])
    dev_o = os.path.join(BUILD, "mrep_device.o")
    _run(["hipcc", *HIP_FLAGS, "-I", INC, "-c", os.path.join(CSRC, "mrep_device.hip"), "-o", dev_o])
    scr_o = os.path.join(BUILD, "mrep_screen.o")
    _run(["hipcc", *HIP_FLAGS, *SCREEN_FLAGS, "-I", INC, "-c", os.path.join(CSRC, "mrep_screen.hip"), "-o", scr_o])
    nn_o = os.path.join(BUILD, "mrep_nn.o")
    _run(["hipcc", *HIP_FLAGS, "-I", INC, "-c", os.path.join(CSRC, "mrep_nn.hip"), "-o", nn_o])
    surf_o = os.path.join(BUILD, "mrep_surf.o")
    _run(["hipcc", *HIP_FLAGS, "-I", INC, "-c", os.path.join(CSRC, "mrep_surf.hip"), "-o", surf_o])
    clip_o = os.path.join(BUILD, "mrep_clip.o")
    _run(["hipcc", *HIP_FLAGS, "-I", INC, "-c", os.path.join(CSRC, "mrep_clip.hip"), "-o", clip_o])
    spans_o = os.path.join(BUILD, "mrep_spans.o")
    _run(["hipcc", *HIP_FLAGS, "-I", INC, "-c", os.path.join(CSRC, "mrep_spans.hip"), "-o", spans_o])
    # the device decomposition repeats the host's arithmetic bit for bit: no contraction
    ddec_o = os.path.join(BUILD, "mrep_ddecomp.o")
    _run(["hipcc", *HIP_FLAGS, "-ffp-contract=off", "-I", INC, "-c", os.path.join(CSRC, "mrep_ddecomp.hip"), "-o",
          ddec_o])
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", dev_o, scr_o, nn_o, surf_o, clip_o, spans_o, ddec_o, host_o, "-o", tmp,
          "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
