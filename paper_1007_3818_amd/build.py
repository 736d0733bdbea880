"""Build libgamer_hydro.so (HIP, gfx950) in-tree, next to this file.

    python -m paper_1007_3818_amd.build [-v]

Every HIP translation unit is compiled for gfx950 only.  Packed FP32 vector
instructions are disabled (``-packed-fp32-ops``); the host pass of hipcc warns
that it does not know that feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgamer_hydro.so")
SOURCES = ["solver.hip", "ctu.hip", "aux_kernels.hip", "amr.hip", "rtvd.hip", "abi.hip"]
HEADERS = ["internal.h", "device_math.h", "euler.h"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


# hipcc's host pass does not know the GPU target feature above and says so once
# per compile; that line is dropped, everything else is shown
_HARMLESS = "'-packed-fp32-ops' is not a recognized feature for this target"


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msg = "\n".join(l for l in r.stdout.splitlines() if _HARMLESS not in l)
    if msg.strip():
        print(msg, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, extra=None, out=None, bdir=None) -> str:
    """Compile every source and link the library (to `out`, default in-tree).
    `extra` adds compiler flags, e.g. -D tunables of a tuning variant."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    bdir = bdir or os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *FLAGS, *(extra or []), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
        objs.append(obj)
    target = out or LIB
    tmp = target + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    extra = [a for a in sys.argv[1:] if a != "-v"]
    print(build(verbose="-v" in sys.argv, extra=extra))
