"""Build libcgks.so in-tree with hipcc for gfx950."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcgks.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["cgks.hip", "cgks_batch.hip", "cgks_batch_f32.hip"]
# per-source flags: the batched FP32 face kernels without machine
# loop-invariant code motion (it would hold the flux's FP64 constants in
# vector registers across their persistent loop)
EXTRA_FLAGS = {"cgks_batch_f32.hip": ["-mllvm", "-disable-machine-licm"]}

HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
               # multiply-adds fused only within a source expression: every
               # kernel that inlines the same device function then does the
               # same arithmetic (batched jobs equal the jobs alone, bit for bit)
               "-ffp-contract=on",
               # no packed FP32 instructions anywhere in this library
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")


def build(verbose=False):
    """Regenerate the constant tables and compile the library (always): one
    object per source, compiled in parallel, linked into one shared library."""
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_tables.py")],
                          stdout=None if verbose else subprocess.DEVNULL)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc] + HIPCC_FLAGS + EXTRA_FLAGS.get(s, []) + ["-c", "-o", o, os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(len(cmds)) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
