"""The benchmark's flop model: operation counts of the oracle's step from its
instrumented build (oracle/flopcount), CPU only.

  * the counting number type counts each +, -, *, / and sqrt once, on a
    snippet of known operation count;
  * the instrumented build computes bitwise the same new state as the plain
    oracle (so it counts the oracle's own arithmetic, not something else);
  * the per-cell counts that bench.py uses are what the instrumented oracle
    counts on the stated samples of workloads 5 and 2.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import bench
import oracle
from oracle import flopcount as fc
from oracle.flopcount.__main__ import GAMMA, sample

HERE = os.path.dirname(os.path.abspath(__file__))


def test_counting_type_counts_each_operation(tmp_path):
    src = tmp_path / "snippet.c"
    src.write_text(
        "double snippet(double a, double b) {\n"
        "    double c = a * b + a / b - sqrt(a);\n"   # mul, div, add, sub, sqrt
        "    if (c < 0.0) c = -c;\n"                  # one comparison, a sign change
        "    c += fabs(b) * 2.0;\n"                   # abs (not a flop), mul, add
        "    return fmin(c, 1e300);\n"                # min (not a flop)
        "}\n")
    drv = tmp_path / "drv.cpp"
    drv.write_text(
        '#include "counted_double.hpp"\n#undef double\n#undef malloc\n'
        "namespace flopcount { uint64_t ops[5]; }\n"
        "cdouble snippet(cdouble, cdouble);\n"
        'extern "C" double run(double a, double b, uint64_t *out) {\n'
        "    for (auto &o : flopcount::ops) o = 0;\n"
        "    double r = snippet(cdouble(a), cdouble(b)).v;\n"
        "    for (int k = 0; k < 5; ++k) out[k] = flopcount::ops[k];\n"
        "    return r;\n}\n")
    hdr = os.path.join(os.path.dirname(fc.__file__), "counted_double.hpp")
    lib = tmp_path / "snip.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-w", "-include", hdr, "-x", "c++", "-c", str(src),
                    "-o", str(tmp_path / "s.o")], check=True)
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-I", os.path.dirname(hdr), str(drv),
                    str(tmp_path / "s.o"), "-o", str(lib)], check=True)
    L = ctypes.CDLL(str(lib))
    L.run.restype = ctypes.c_double
    L.run.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    out = np.zeros(5, dtype=np.uint64)
    a, b = 2.0, 0.5
    r = L.run(a, b, out.ctypes.data)
    c = a * b + a / b - np.sqrt(a)
    c = -c if c < 0 else c
    assert r == min(c + abs(b) * 2.0, 1e300)
    assert out.tolist() == [3, 2, 1, 1, 3]  # add/sub, mul, div, sqrt, compare/abs/min


def test_counting_build_equals_plain_oracle():
    pad, dt, dh = sample(256, 4, 2)
    pad = pad[:3]
    counts, got = fc.hydro_step(pad, dt, dh, GAMMA)
    want, _, fb = oracle.hydro_solve(pad, dt, dh, GAMMA)
    assert np.array_equal(got, want)
    assert counts["fallbacks"] == fb
    _, got2 = fc.hydro_stages(pad, dt, dh, GAMMA)
    assert np.array_equal(got2, want)
    cc, got3 = fc.ctu_step(pad, dt, dh, GAMMA)
    want3, _, _ = oracle.hydro_solve(pad, dt, dh, GAMMA, coupling="ctu")
    assert np.array_equal(got3, want3)


@pytest.mark.parametrize("workload", [5, 2])
def test_bench_flop_model_is_the_counted_one(workload):
    n, kmax = (1024, 8) if workload == 5 else (256, 4)
    pad, dt, dh = sample(n, kmax, workload)
    st, _ = fc.hydro_stages(pad, dt, dh, GAMMA)
    total = sum(v["flops"] for v in st.values())
    assert total / (32 * 4096) == bench.FLOPS_PER_CELL[workload]
    if workload == 2:
        c, _ = fc.ctu_step(pad, dt, dh, GAMMA)
        epi = st["cfl_speed"]["flops"] + st["sums"]["flops"]
        assert (c["flops"] + epi) / (32 * 4096) == bench.CTU_FLOPS_PER_CELL
        pad3, dt3, dh3 = sample(256, 4, 2, ghost=3)
        r, _ = fc.rtvd_step(pad3, dt3, dh3, GAMMA, order=0)
        assert r["flops"] / (32 * 4096) == bench.RTVD_FLOPS_PER_CELL
