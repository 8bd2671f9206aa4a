"""Build libbms.so (the HIP library behind include/bms.h) for gfx950.

Compiles every source under csrc/ with hipcc and links them into
paper_1808_01829_amd/libbms.so. Always recompiles (objects go to _build/).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build", "bms")
OUT = os.path.join(HERE, "libbms.so")

ARCH = "gfx950"
# packed FP32 instructions are disabled for every device pass
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


# per-file device options: the Gram kernels keep their matrix-core
# accumulators in ordinary VGPRs (with accumulation registers the loop-carried
# accumulators are copied between the two files every iteration, which
# doubles their register use and halves the resident waves)
FILE_FLAGS = {
    "blas.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src, verbose):
    obj = os.path.join(OBJ, src + ".o")
    cmd = (["hipcc"] + CFLAGS + FILE_FLAGS.get(src, []) +
           ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, err


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(lambda s: _compile(s, verbose), srcs))
    for obj, err in res:
        if err and verbose:
            print(err, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in res]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
