"""Build libsem.so (HIP, gfx950) in-tree with hipcc.

Every .hip / .cpp file under csrc/ is compiled for gfx950 and linked into
paper_2405_05640_amd/libsem.so.  Host OpenMP (mesh setup) comes from the ROCm
LLVM runtime, found through an rpath.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsem.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-fopenmp",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-I" + os.path.join(HERE, "..", "include")]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _obj(src, outdir):
    return os.path.join(outdir, os.path.basename(src) + ".o")


def build(verbose=False, jobs=8):
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    srcs = sources()

    def compile_one(src):
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", src, "-o", _obj(src, outdir)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stderr))
        if r.stderr.strip() and verbose:
            print(r.stderr)
        return src

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    llvm_lib = os.path.join(ROCM, "llvm", "lib")
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-fopenmp", "-o", tmp] + \
        [_obj(s, outdir) for s in srcs] + ["-Wl,-rpath," + llvm_lib, "-L" + llvm_lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
