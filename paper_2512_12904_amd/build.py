"""Build steps for the in-tree native libraries.

libhqc_gpu.so   hipcc, gfx950: kernels + C ABI (include/hqc_gpu.h)
libhqc_synth.so gcc: seeded input generator
"""
import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GPU_SO = os.path.join(HERE, "libhqc_gpu.so")
GPU_SOURCES = [os.path.join(CSRC, "hqc_kernels.hip"), os.path.join(CSRC, "hqc_encrypt.hip"),
               os.path.join(CSRC, "hqc_kem.hip"), os.path.join(CSRC, "hqc_ring.hip"),
               os.path.join(CSRC, "hqc_tune.hip"),
               os.path.join(CSRC, "hqc_capi.cpp")]
GPU_HEADERS = [os.path.join(CSRC, "hqc_internal.h"), os.path.join(CSRC, "hqc_internal_enc.h"),
               os.path.join(CSRC, "hqc_device.h"),
               os.path.join(ROOT, "include", "hqc_gpu.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def build_gpu(verbose=False, jobs=None):
    """Compile the HIP library for gfx950 (cross-compiles without a GPU): each
    source to an object in parallel (the sources share no device symbols),
    then one shared-library link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc()] + HIPCC_FLAGS + inc + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL)
        return obj

    n = jobs or max(1, min(len(GPU_SOURCES), os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(n) as ex:
        objs = list(ex.map(compile_one, GPU_SOURCES))
    tmp = GPU_SO + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL)
    os.replace(tmp, GPU_SO)
    return GPU_SO


def gpu_stale():
    if not os.path.exists(GPU_SO):
        return True
    t = os.path.getmtime(GPU_SO)
    return any(os.path.getmtime(s) > t for s in GPU_SOURCES + GPU_HEADERS)


def build_synth():
    from . import synth
    synth.build()


def build_all(verbose=False):
    build_synth()
    build_gpu(verbose=verbose)
