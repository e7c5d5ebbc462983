"""Build the HIP library libtmul.so in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtmul.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("tmul.hip", "k1_full.hip", "k1_lo.hip", "k1_hi.hip", "k0_small.hip", "fp32c.hip",
                     "serve.cpp", "mulmod.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", f)
                  for f in ("kernels.hpp", "fft_tile.hpp", "dfloat.hpp", "plan.hpp", "dispatch.hpp")] \
    + [os.path.join(ROOT, "include", "tmul.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions are kept out of every GPU build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False):
    """Compile libtmul.so (always recompiles): one object per source, in
    parallel, then one shared-library link."""
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    tmpdir = tempfile.mkdtemp(prefix="tmul_build_")
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
        cmd = [hipcc] + HIPCC_FLAGS + inc + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for pr, cmd in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmpdir)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
