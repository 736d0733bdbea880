"""Operation counts of the oracle's step -- TEST AND MEASUREMENT INFRASTRUCTURE.

The oracle's unchanged C sources are compiled as C++ with ``counted_double.hpp``
force-included, which turns their ``double`` into a type that counts every
add/subtract, multiply, divide and square root (and, apart, comparisons,
|x|, min and max).  Running a step on a workload then gives the arithmetic the
method does per cell-update as the oracle states it, which the benchmark's
roofline model uses.  The counting build shares nothing with the HIP library.

    python -m oracle.flopcount      # counts on the benchmark workloads' groups
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.dirname(HERE)
SRCS = [os.path.join(ORACLE, f) for f in ("gamer_oracle.c", "gamer_ctu.c", "gamer_rtvd.c")]
LIB = os.path.join(HERE, "libgamer_oracle_counted.so")
KINDS = ("add", "mul", "div", "sqrt", "cmp")

_lib = None


def build(verbose=False):
    """Compile the counting build of the oracle (g++, -O1, no contraction)."""
    hdr = os.path.join(HERE, "counted_double.hpp")
    flags = ["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-w"]
    objs = []
    for src in SRCS:  # the oracle's sources, with the counting type forced in
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        objs.append(obj)
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [*flags, "-include", hdr, "-x", "c++", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    tmp = LIB + ".tmp"
    cmd = [*flags, "-shared", os.path.join(HERE, "driver.cpp"), *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        deps = SRCS + [os.path.join(HERE, f) for f in ("counted_double.hpp", "driver.cpp")]
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in deps):
            build()
        L = ctypes.CDLL(LIB)
        P, D, I, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
        L.fc_hydro_solve.argtypes = [P, I64, D, D, D, D, I, P, P, P]
        L.fc_hydro_stages.argtypes = [P, I64, D, D, D, D, P, P]
        L.fc_ctu_solve.argtypes = [P, I64, D, D, D, D, P, P, P]
        L.fc_rtvd_solve.argtypes = [P, I64, D, D, D, I, P, P, P]
        for f in (L.fc_hydro_solve, L.fc_hydro_stages, L.fc_ctu_solve, L.fc_rtvd_solve):
            f.restype = I
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _result(counts, extra):
    out = dict(zip(KINDS, (int(c) for c in counts)))
    out["flops"] = out["add"] + out["mul"] + out["div"] + out["sqrt"]
    out.update(extra)
    return out


def hydro_step(padded, dt, dh, gamma, theta=1.5, char_limiting=False):
    """Counts of one MUSCL-Hancock + Roe step on padded groups (n, 5, 20, 20, 20);
    also returns the new state, so a caller can check it against the oracle."""
    a = np.ascontiguousarray(padded, dtype=np.float64)
    n = a.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    fb = np.zeros(2, dtype=np.int64)
    cnt = np.zeros(5, dtype=np.uint64)
    rc = _load().fc_hydro_solve(_ptr(a), n, dt, dh, gamma, theta, int(char_limiting), _ptr(out), _ptr(fb),
                                _ptr(cnt))
    if rc != 0:
        raise RuntimeError(f"counted oracle step failed ({rc})")
    return _result(cnt, {"fallbacks": (int(fb[0]), int(fb[1])), "cells": n * 4096}), out


STAGES = ("prim", "slopes", "predictor", "riemann", "update", "cfl_speed", "sums")


def hydro_stages(padded, dt, dh, gamma, theta=1.5):
    """Counts of the same step split by stage, plus the step's epilogue on the
    new state (the CFL signal-speed maximum and the conserved sums, which the
    GPU step also computes).  Returns ({stage: counts}, new state)."""
    a = np.ascontiguousarray(padded, dtype=np.float64)
    n = a.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    cnt = np.zeros((7, 5), dtype=np.uint64)
    _load().fc_hydro_stages(_ptr(a), n, dt, dh, gamma, theta, _ptr(out), _ptr(cnt))
    return {s: _result(cnt[k], {"cells": n * 4096}) for k, s in enumerate(STAGES)}, out


def ctu_step(padded, dt, dh, gamma, theta=1.5):
    a = np.ascontiguousarray(padded, dtype=np.float64)
    n = a.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    fb = np.zeros(2, dtype=np.int64)
    cnt = np.zeros(5, dtype=np.uint64)
    rc = _load().fc_ctu_solve(_ptr(a), n, dt, dh, gamma, theta, _ptr(out), _ptr(fb), _ptr(cnt))
    if rc != 0:
        raise RuntimeError(f"counted CTU step failed ({rc})")
    return _result(cnt, {"fallbacks": (int(fb[0]), int(fb[1])), "cells": n * 4096}), out


def rtvd_step(padded3, dt, dh, gamma, order=0):
    """padded3: groups with three ghost cells, (n, 5, 22, 22, 22)."""
    a = np.ascontiguousarray(padded3, dtype=np.float64)
    n = a.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    bad = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(5, dtype=np.uint64)
    rc = _load().fc_rtvd_solve(_ptr(a), n, dt, dh, gamma, order, _ptr(out), _ptr(bad), _ptr(cnt))
    if rc != 0:
        raise RuntimeError(f"counted relaxing-TVD step failed ({rc})")
    return _result(cnt, {"bad": int(bad[0]), "cells": n * 4096}), out
