"""Build libmc.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import shutil
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("mc_kernels.hip", "mc_mlp.hip", "mc_api.hip")]
HEADERS = [os.path.join(_HERE, "csrc", f) for f in ("mc_device.h", "mc_internal.h", "mc_physics.h", "mc_mlp.h")] + [
    os.path.join(os.path.dirname(_HERE), "include", "mc.h")]
OUT = os.path.join(_HERE, "libmc.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # interpolation, macroscopic sums and kinematics must round as written
    "-ffp-contract=off",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def library_path() -> str:
    return OUT


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source into libmc.so (always recompiles)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = OUT + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, OUT)
    return OUT
