"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a temporary copy of the oracle's C
sources, builds that copy with the oracle's own build function, and runs the
pins that must catch the mistake in a child process whose `oracle` package
loads the mutant library: the run must fail on a test, not on the build or on
loading.  A control copy without a mistake must pass two pin files through the
same route, so that a failing run is the mistake's doing.  The mistakes are the
ones the pins were written against: the unsplit coupling of the Hancock
predictor (Sec. 2, half-step prediction), the value and the sides of the
Harten-Hyman entropy fix (Roe's solver), the limiter's central difference, the
sign of Roe's dissipation, the predictor's half step, the relaxing scheme's
half step, the CTU correction's sign, the characteristic limiter's projections, and the coarse/fine correction's area
average and sign and the restriction's average (the Python part of the oracle,
loaded from the copy in place of `oracle.amr`).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
SOURCES = ("gamer_oracle.c", "gamer_rtvd.c", "gamer_ctu.c")
PY_SOURCES = ("amr.py",)  # Python parts of the oracle, loaded from the copy in place of oracle.amr

# (what the mistake is, file, [(text, replacement)], pins that must catch it)
MUTANTS = [
    ("no unsplit coupling: every face state keeps only the last direction's flux difference",
     "gamer_oracle.c", [("S[v] += fm[v] - fp[v];", "S[v] = fm[v] - fp[v];")],
     ["tests/test_oracle_unsplit.py"]),
    ("entropy fix with the modulus delta instead of (lambda^2 + delta^2) / (2 delta)",
     "gamer_oracle.c", [("absl[0] = (lam * lam + delta * delta) / (2.0 * delta);", "absl[0] = delta;"),
                        ("absl[4] = (lam * lam + delta * delta) / (2.0 * delta);", "absl[4] = delta;")],
     ["tests/test_oracle_entropy.py"]),
    ("entropy fix of wave 5 with its two sides swapped",
     "gamer_oracle.c", [("double lleft = us + cs, lright = uR + cR, lam = r.lambda[4];",
                         "double lleft = uR + cR, lright = us + cs, lam = r.lambda[4];")],
     ["tests/test_oracle_entropy.py"]),
    ("limiter's central difference not halved",
     "gamer_oracle.c", [("0.5 * fabs(a + b)", "fabs(a + b)")],
     ["tests/test_oracle_pins.py"]),
    ("Roe dissipation added instead of subtracted",
     "gamer_oracle.c", [("F[m] = 0.5 * (FL[m] + FR[m]) - 0.5 * diss;", "F[m] = 0.5 * (FL[m] + FR[m]) + 0.5 * diss;")],
     ["tests/test_oracle_pins.py"]),
    ("Hancock predictor over dt instead of dt/2",
     "gamer_oracle.c", [("double coef = dt / (2.0 * dh);", "double coef = dt / dh;")],
     ["tests/test_oracle_unsplit.py", "tests/test_oracle_flows.py"]),
    ("relaxing scheme's half step over dt instead of dt/2",
     "gamer_rtvd.c", [("- 0.5 * dtdx * (F[i * RV + v]", "- dtdx * (F[i * RV + v]")],
     ["tests/test_oracle_rtvd.py"]),
    ("CTU transverse correction added instead of subtracted",
     "gamer_ctu.c", [("u[v] = dst[eidx(v, i, j, k)] - hdt * corr[v];",
                      "u[v] = dst[eidx(v, i, j, k)] + hdt * corr[v];")],
     ["tests/test_oracle_ctu.py"]),
    ("Roe averages weighted by density instead of its square root",
     "gamer_oracle.c", [("double sl = sqrt(wl[0]), sr = sqrt(wr[0]);", "double sl = wl[0], sr = wr[0];")],
     ["tests/test_oracle_pins.py"]),
    ("HLLE's state-difference term with the states swapped",
     "gamer_oracle.c", [("SL * SR * (R[m] - L[m])", "SL * SR * (L[m] - R[m])")],
     ["tests/test_oracle_pins.py"]),
    ("update reading the y fluxes with their transverse indices transposed",
     "gamer_oracle.c", [("double dfy = FL(1, v, j + 1, k, i) - FL(1, v, j, k, i);",
                         "double dfy = FL(1, v, j + 1, i, k) - FL(1, v, j, i, k);")],
     ["tests/test_oracle_pins.py", "tests/test_oracle_unsplit.py", "tests/test_oracle_flows.py"]),
    ("CFL signal speed with one sound speed instead of three",
     "gamer_oracle.c", [("+ fabs(w[3]) + 3.0 * cs;", "+ fabs(w[3]) + cs;")],
     ["tests/test_oracle_pins.py"]),
    ("characteristic limiting with the acoustic waves' velocity components swapped",
     "gamer_oracle.c", [("dW[n] = c / rho * (m[4] - m[0]);", "dW[n] = c / rho * (m[0] - m[4]);")],
     ["tests/test_oracle_char.py"]),
    ("characteristic limiting with the entropy wave's pressure term added",
     "gamer_oracle.c", [("la[1] = a[0] - a[4] / c2;", "la[1] = a[0] + a[4] / c2;"),
                        ("lb[1] = b[0] - b[4] / c2;", "lb[1] = b[0] + b[4] / c2;")],
     ["tests/test_oracle_char.py"]),
    ("coarse/fine correction with the fine fluxes averaged over 2 instead of 4 faces",
     "amr.py", [("+ Ff[:, 1::2, 1::2]) / 4.0", "+ Ff[:, 1::2, 1::2]) / 2.0")],
     ["tests/test_oracle_amr.py"]),
    ("coarse/fine correction with its sign flipped on the wrong side",
     "amr.py", [("if side == 1:\n                delta = -delta", "if side == 0:\n                delta = -delta")],
     ["tests/test_oracle_amr.py"]),
    ("restriction averaging over 4 instead of 8 fine cells",
     "amr.py", [("= blk / 8.0", "= blk / 4.0")],
     ["tests/test_oracle_amr.py"]),
]

# Child process: point the oracle's build at the copy, build it (exit 3 if that
# fails), load it (exit 4 if another library got loaded), then run the pins.
DRIVER = r"""
import os, sys
sys.path.insert(0, {root!r})
import oracle, oracle.build as b
b.LIB = {lib!r}
b.SRCS = {srcs!r}
try:
    b.build()
except Exception as e:
    print("BUILD FAILED", e, flush=True)
    sys.exit(3)
lib = oracle._lib()
if os.path.realpath(lib._name) != os.path.realpath({lib!r}):
    print("LOADED", lib._name, flush=True)
    sys.exit(4)
import importlib.util
spec = importlib.util.spec_from_file_location("oracle.amr", {amr!r})
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle.amr"] = mod
spec.loader.exec_module(mod)
oracle.amr = mod
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", *{targets!r}]))
"""


def _run(tmp_path, name, edits, targets):
    d = tmp_path / name
    d.mkdir()
    for f in SOURCES + PY_SOURCES:
        shutil.copy(os.path.join(ORACLE, f), d / f)
    for fname, pairs in edits:
        p = d / fname
        text = p.read_text()
        for old, new in pairs:
            assert text.count(old) == 1, (fname, old)
            text = text.replace(old, new)
        p.write_text(text)
    lib = str(d / "libgamer_oracle_mutant.so")
    code = DRIVER.format(root=ROOT, lib=lib, srcs=[str(d / f) for f in SOURCES], amr=str(d / "amr.py"),
                         targets=targets)
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    return r.returncode, r.stdout[-3000:] + r.stderr[-3000:]


def test_control_copy_passes(tmp_path):
    rc, out = _run(tmp_path, "control", [], ["tests/test_oracle_pins.py", "tests/test_oracle_amr.py"])
    assert rc == 0, out


@pytest.mark.parametrize("what,fname,pairs,targets", MUTANTS, ids=[m[0][:40] for m in MUTANTS])
def test_mutant_fails_a_pin(tmp_path, what, fname, pairs, targets):
    rc, out = _run(tmp_path, "mutant", [(fname, pairs)], targets)
    # pytest's exit code 1: tests ran and at least one failed
    assert rc == 1, f"{what}: exit {rc}\n{out}"
    print(f"[mutant] {what}: caught", flush=True)
