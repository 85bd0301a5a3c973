"""Builds libmbcontract.so (HIP, gfx950) in-tree, and synth/libsynth.so."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmbcontract.so")
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "--offload-arch=gfx950"
# packed FP32 instructions stay off; hipcc forms none by itself with this
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def _compile(src, obj, kind):
    if kind == "host":   # plain C++ (no HIP): the host compiler
        cmd = ["g++"] + COMMON + ["-c", src, "-o", obj]
    else:
        cmd = [HIPCC, ARCH] + COMMON + (DEVICE_FLAGS if kind == "hip" else []) + ["-c", src, "-o", obj]
    _run(cmd)


def build_library(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    units = [("termlist.cpp", "host"), ("capi.cpp", "hipapi"), ("batch.cpp", "hipapi"), ("blocks.hip", "hip"),
             ("contract.hip", "hip"), ("contract_f32.hip", "hip"), ("contract_f32b.hip", "hip"), ("contract_f32b_m6.hip", "hip"),
             ("contract_f64.hip", "hip"), ("contract_f32_m6.hip", "hip"), ("contract_f64_m6.hip", "hip"),
             ("errest.hip", "hip"),
             ("noalloc.hip", "hip")]
    objs = [os.path.join(BUILD_DIR, name + ".o") for name, _ in units]
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(units), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_compile, os.path.join(CSRC, name), obj, kind) for (name, kind), obj in zip(units, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_synth(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, "synth.hip.o")
    _run([HIPCC, ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off"] + DEVICE_FLAGS +
         ["-c", os.path.join(ROOT, "synth", "synth.hip"), "-o", obj])
    tmp = SYNTH_LIB + ".tmp"
    _run([HIPCC, ARCH, "-shared", "-fPIC", "-o", tmp, obj])
    os.replace(tmp, SYNTH_LIB)
    if verbose:
        print("built", SYNTH_LIB)
    return SYNTH_LIB


def build_all(verbose: bool = False):
    build_library(verbose)
    build_synth(verbose)


if __name__ == "__main__":
    build_all(verbose=True)
