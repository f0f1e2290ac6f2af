"""Build the HIP library in-tree: hipcc for gfx950 -> paper_2312_00229_amd/libweno_zoom.so.

Flags: -O3, FP contraction off (every fused multiply-add in the kernels is
written explicitly, so the operation sequence -- and hence every bit of the
result -- is the same in all kernels that share the device code), packed FP32
disabled, C++17."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libweno_zoom.so")
SOURCES = ["weno_api.hip", "weno_bwd.hip", "weno_resample.hip"]
ARCH = os.environ.get("WENO_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [
        hipcc(),
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-shared",
        "-ffp-contract=off",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result",
        "-I" + INCLUDE,
        "-I" + CSRC,
        *srcs,
        "-o", tmp,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % LIB)
    os.replace(tmp, LIB)
    return LIB


def build_asan(out_dir: str, verbose: bool = False) -> str:
    """The same library with AddressSanitizer on its HOST code only (device
    code is built as usual), for the ABI checks on the CPU: the three sources
    are compiled in parallel and linked into out_dir/libweno_zoom_asan.so.
    Load it through WENO_ZOOM_LIB with the sanitizer runtime preloaded
    (asan_runtime())."""
    os.makedirs(out_dir, exist_ok=True)
    common = [hipcc(), "--offload-arch=" + ARCH, "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
              "-Xarch_host", "-fsanitize=address",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
              "-I" + INCLUDE, "-I" + CSRC]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(common + ["-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed building the sanitizer objects")
    lib = os.path.join(out_dir, "libweno_zoom_asan.so")
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address", *objs,
           "-o", lib]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=True)
    return lib


def asan_runtime() -> str:
    """Path of the AddressSanitizer runtime of ROCm's clang."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    res = subprocess.run([clang, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                         check=True)
    return res.stdout.strip()


if __name__ == "__main__":
    print(build(verbose=True))
