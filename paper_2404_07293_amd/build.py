"""Build the HIP library libscw.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2404_07293_amd.build [--jobs N]
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libscw.so")

SOURCES = [
    "lapack.cpp",
    "setup.cpp",
    "api.cpp",
    "tune.cpp",
    "kernels_setup.hip",
    "kernels_synth.hip",
    "kernels_mfma.hip",
    "kernels_batch.hip",
    "surrogate.cpp",
    "kernels_surrogate.hip",
    "noalloc.hip",
    "kernels_eig.hip",
    "kernels_surrogate_bf16.hip",
    "eig.cpp",
]

ARCH = "gfx950"


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return [
        "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-result",
        "-I" + os.path.join(HERE, "..", "include"),
    ]


# Per-file code-generation options. The bf16 surrogate kernels keep their
# matrix-core accumulators in ordinary vector registers: their epilogues read
# every accumulator once (bias, GELU, rounding), which in accumulation
# registers costs one extra move per value, and the smaller register total
# leaves room for more waves per SIMD.
FILE_FLAGS = {
    "kernels_surrogate_bf16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def compile_one(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + flags() + FILE_FLAGS.get(src, []) + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs=8, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-ldl", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host AddressSanitizer / UndefinedBehaviorSanitizer build of the library's
# sources linked with the ABI driver tests/sanitize/abi_check.cpp into one
# executable. The sanitizers instrument host code only (each -fsanitize= is
# bound to the host pass); device code is compiled as in the library.
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_EXE = os.path.join(SAN_DIR, "abi_check")
SAN_DRIVER = os.path.join(HERE, "..", "tests", "sanitize", "abi_check.cpp")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(jobs=8, verbose=False):
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        cmd = ([hipcc()] + flags() + FILE_FLAGS.get(os.path.basename(src), []) + SAN_FLAGS +
               ["-I" + CSRC, "-x", "hip", "-c", path, "-o", obj])
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout,
                                                                 r.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, srcs + [os.path.abspath(SAN_DRIVER)]))
    tmp = SAN_EXE + ".tmp"
    cmd = ([hipcc(), "--offload-arch=" + ARCH] + SAN_FLAGS + ["-o", tmp] + objs +
           ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-ldl", "-lpthread"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, SAN_EXE)
    if verbose:
        print("built", SAN_EXE)
    return SAN_EXE


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--sanitize", action="store_true",
                    help="also build the host-sanitizer ABI driver")
    args = ap.parse_args(argv)
    build(args.jobs, verbose=True)
    if args.sanitize:
        build_sanitized(args.jobs, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
