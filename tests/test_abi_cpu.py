"""Host-side checks of the C ABI (no GPU needed): the library builds and loads,
exports every symbol the header declares, and rejects bad arguments before it
touches the device."""
import ctypes
import os
import re

import pytest

from paper_1007_3818_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gamer_hydro.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gamer_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_native.LIB_PATH):
        from paper_1007_3818_amd import build
        build.build()
    return _native.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) == 38
    for n in names:
        assert hasattr(lib, n), n
        assert n in _native.SIGNATURES, n
    assert set(_native.SIGNATURES) == set(names)


def test_opts_struct_layout():
    # gamer_opts: double theta, int32 variant, int32 grid, int32 limiting, int32 zseg,
    # uint64_t *bad_count_dev
    assert ctypes.sizeof(_native.GamerOpts) == 32
    assert _native.GamerOpts.variant.offset == 8 and _native.GamerOpts.grid.offset == 12
    assert _native.GamerOpts.limiting.offset == 16 and _native.GamerOpts.zseg.offset == 20
    assert _native.GamerOpts.bad_count_dev.offset == 24


def test_opts_struct_layout_matches_header(tmp_path):
    """The C compiler's layout of gamer_opts from the public header."""
    import subprocess
    src = tmp_path / "o.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gamer_hydro.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu", sizeof(gamer_opts),'
                   ' offsetof(gamer_opts, variant), offsetof(gamer_opts, grid),'
                   ' offsetof(gamer_opts, limiting), offsetof(gamer_opts, zseg),'
                   ' offsetof(gamer_opts, bad_count_dev)); return 0; }\n')
    exe = tmp_path / "o"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    O = _native.GamerOpts
    assert got == [ctypes.sizeof(O), O.variant.offset, O.grid.offset, O.limiting.offset, O.zseg.offset,
                   O.bad_count_dev.offset]


def test_solver_variants(lib):
    th, wv = ctypes.c_int(0), ctypes.c_int(0)
    pth = ctypes.cast(ctypes.byref(th), ctypes.c_void_p)
    pwv = ctypes.cast(ctypes.byref(wv), ctypes.c_void_p)
    for f32 in (0, 1):
        n = lib.gamer_solver_variants(f32)
        assert n >= 1
        for v in range(n):
            assert lib.gamer_solver_variant_shape(f32, v, pth, pwv) == 0
            assert th.value in (256, 320) and 1 <= wv.value <= 8
        assert lib.gamer_solver_variant_shape(f32, n, pth, pwv) == _native.GAMER_EINVAL
        assert lib.gamer_solver_variant_shape(f32, 0, None, pwv) == _native.GAMER_EINVAL


def test_version(lib):
    assert lib.gamer_version() >= 200


def _rc(fn, *args):
    return fn(*args)


P = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def test_solve_argument_errors(lib):
    f = lib.gamer_hydro_solve
    assert f(None, 4, 0.1, 0.1, 1.4, None, P) == _native.GAMER_EINVAL
    assert b"NULL" in lib.gamer_last_error()
    assert f(P, 4, 0.1, 0.1, 1.4, None, None) == _native.GAMER_EINVAL
    assert f(P, -1, 0.1, 0.1, 1.4, None, P) == _native.GAMER_EINVAL
    assert f(P, 4, 0.0, 0.1, 1.4, None, P) == _native.GAMER_EINVAL
    assert f(P, 4, float("nan"), 0.1, 1.4, None, P) == _native.GAMER_EINVAL
    assert f(P, 4, 0.1, -1.0, 1.4, None, P) == _native.GAMER_EINVAL
    assert f(P, 4, 0.1, 0.1, 1.0, None, P) == _native.GAMER_EINVAL
    assert f(P, 4, 0.1, 0.1, float("inf"), None, P) == _native.GAMER_EINVAL
    # zero groups: a successful no-op, even with NULL arrays
    assert f(None, 0, 0.1, 0.1, 1.4, None, None) == _native.GAMER_OK
    assert lib.gamer_hydro_solve_f32(None, 0, 0.1, 0.1, 1.4, None, None) == _native.GAMER_OK


def test_batched_argument_errors(lib):
    f = lib.gamer_hydro_solve_batched
    assert f(P, 4, None, None, P, 1, 1.4, None, P, None, None, None) == _native.GAMER_EINVAL  # no dt_dev
    assert f(P, 4, None, P, None, 1, 1.4, None, P, None, None, None) == _native.GAMER_EINVAL  # no dh_dev
    assert f(P, 4, None, P, P, 0, 1.4, None, P, None, None, None) == _native.GAMER_EINVAL
    assert f(P, 4, None, P, P, 33, 1.4, None, P, None, None, None) == _native.GAMER_EINVAL
    bad = _native.GamerOpts(1.5, 0, 0, 0, 0, 0x1004)  # misaligned counter
    assert f(P, 4, None, P, P, 1, 1.4, None, P, None, ctypes.byref(bad), None) == _native.GAMER_EINVAL
    assert b"bad_count_dev" in lib.gamer_last_error()
    bad = _native.GamerOpts(2.5, 0, 0)
    assert f(P, 4, None, P, P, 1, 1.4, None, P, None, ctypes.byref(bad), None) == _native.GAMER_EINVAL
    bad = _native.GamerOpts(0.5, 0, 0)
    assert f(P, 4, None, P, P, 1, 1.4, None, P, None, ctypes.byref(bad), None) == _native.GAMER_EINVAL
    bad = _native.GamerOpts(1.5, 99, 0)
    assert f(P, 4, None, P, P, 1, 1.4, None, P, None, ctypes.byref(bad), None) == _native.GAMER_EINVAL
    assert b"variant" in lib.gamer_last_error()
    bad = _native.GamerOpts(1.5, -1, 0)
    assert f(P, 4, None, P, P, 1, 1.4, None, P, None, ctypes.byref(bad), None) == _native.GAMER_EINVAL
    bad = _native.GamerOpts(1.5, 0, -4)
    assert f(P, 4, None, P, P, 1, 1.4, None, P, None, ctypes.byref(bad), None) == _native.GAMER_EINVAL


def test_limiting_and_mixed_argument_errors(lib):
    E = _native.GAMER_EINVAL
    Q = ctypes.c_void_p(0x2000)
    # a bad limiting value or a negative z-segment length: every solver entry point
    for lim, zseg in ((2, 0), (-1, 0), (0, -1)):
        bad = _native.GamerOpts(1.5, 0, 0, lim, zseg)
        assert lib.gamer_hydro_solve_batched(P, 4, None, P, P, 1, 1.4, None, Q, None,
                                             ctypes.byref(bad), None) == E
        assert lib.gamer_hydro_solve_periodic_mixed(P, 2, 2, 2, P, P, 1.4, None, Q, None,
                                                    ctypes.byref(bad)) == E
    # a z-segment length is for the periodic entry points only
    bad = _native.GamerOpts(1.5, 0, 0, 0, 3)
    assert lib.gamer_hydro_solve_batched(P, 4, None, P, P, 1, 1.4, None, Q, None, ctypes.byref(bad), None) == E
    assert b"zseg" in lib.gamer_last_error()
    assert lib.gamer_ctu_solve_batched(P, 4, None, P, P, 1, 1.4, None, Q, None, ctypes.byref(bad), None, 0) == E
    f = lib.gamer_hydro_solve_batched_mixed
    assert f(P, 4, None, None, P, 1, 1.4, None, Q, None, None, None) == E  # no dt_dev
    assert f(P, 4, None, P, None, 1, 1.4, None, Q, None, None, None) == E  # no dh_dev
    assert f(P, 4, None, P, P, 0, 1.4, None, Q, None, None, None) == E
    assert f(None, 4, None, P, P, 1, 1.4, None, Q, None, None, None) == E
    bad = _native.GamerOpts(1.5, lib.gamer_solver_variants(1), 0, 0, 0)  # float variants index
    assert f(P, 4, None, P, P, 1, 1.4, None, Q, None, ctypes.byref(bad), None) == E
    g = lib.gamer_hydro_solve_periodic_mixed
    assert g(P, 0, 2, 2, P, P, 1.4, None, Q, None, None) == E
    assert g(P, 2, 2, 2, P, P, 1.4, None, P, None, None) == E


def test_ctu_argument_errors(lib):
    E = _native.GAMER_EINVAL
    Q = ctypes.c_void_p(0x2000)
    W = ctypes.c_void_p(0x4000)
    need = lib.gamer_ctu_workspace_bytes(8, 0)
    assert need >= 8 * (6 * 5 * 18 ** 3 + 3 * 5 * 18 ** 3) * 8  # predicted states, transverse fluxes
    assert lib.gamer_ctu_workspace_bytes(0, 1) == 0
    pipe = ctypes.byref(_native.GamerOpts(1.5, 1, 0, 0, 0))  # variant 1: the pipeline through a workspace
    for f in (lib.gamer_ctu_solve_batched, lib.gamer_ctu_solve_batched_f32):
        for o in (None, pipe):  # checks common to the fused sweep and the pipeline
            assert f(P, -1, None, P, P, 1, 1.4, None, Q, None, o, W, need) == E
            assert f(P, 8, None, P, P, 1, 1.0, None, Q, None, o, W, need) == E
            assert f(None, 8, None, P, P, 1, 1.4, None, Q, None, o, W, need) == E
            assert f(P, 8, None, None, P, 1, 1.4, None, Q, None, o, W, need) == E
            assert f(P, 8, None, P, P, 0, 1.4, None, Q, None, o, W, need) == E
        # the pipeline's workspace: missing, short, misaligned
        assert f(P, 8, None, P, P, 1, 1.4, None, Q, None, pipe, None, need) == E
        assert f(P, 8, None, P, P, 1, 1.4, None, Q, None, pipe, W, 1000) == E
        assert f(P, 8, None, P, P, 1, 1.4, None, Q, None, pipe, ctypes.c_void_p(0x4010), need) == E
        for bad in (_native.GamerOpts(1.5, 2, 0, 0, 0), _native.GamerOpts(1.5, 0, 8, 0, 0),
                    _native.GamerOpts(1.5, 0, 0, 1, 0), _native.GamerOpts(3.0, 0, 0, 0, 0),
                    _native.GamerOpts(1.5, 0, 0, 0, 0, 0x1002)):
            assert f(P, 8, None, P, P, 1, 1.4, None, Q, None, ctypes.byref(bad), W, need) == E
        assert f(None, 0, None, None, None, 1, 1.4, None, None, None, None, None, 0) == _native.GAMER_OK


def test_rtvd_argument_errors(lib):
    E = _native.GAMER_EINVAL
    Q = ctypes.c_void_p(0x2000)
    W = ctypes.c_void_p(0x4000)
    need = lib.gamer_rtvd_workspace_bytes(8, 0)
    assert need == 8 * 5 * (16 * 22 * 22 + 16 * 16 * 22) * 8
    assert lib.gamer_rtvd_workspace_bytes(8, 1) == need // 2
    assert lib.gamer_rtvd_workspace_bytes(0, 0) == 0
    for f in (lib.gamer_rtvd_solve_batched, lib.gamer_rtvd_solve_batched_f32):
        assert f(P, -1, None, P, P, 1, 1.4, 0, W, need, Q) == E
        assert f(P, 8, None, P, P, 1, 1.4, 2, W, need, Q) == E            # order
        assert f(P, 8, None, P, P, 1, 1.0, 0, W, need, Q) == E            # gamma
        assert f(None, 8, None, P, P, 1, 1.4, 0, W, need, Q) == E
        assert f(P, 8, None, None, P, 1, 1.4, 0, W, need, Q) == E
        assert f(P, 8, None, P, P, 0, 1.4, 0, W, need, Q) == E            # n_levels
        assert f(P, 8, None, P, P, 1, 1.4, 0, None, need, Q) == E         # no workspace
        assert f(P, 8, None, P, P, 1, 1.4, 0, W, 100, Q) == E             # short workspace
        assert b"workspace" in lib.gamer_last_error()
        assert f(P, 8, None, P, P, 1, 1.4, 0, ctypes.c_void_p(0x4008), need, Q) == E  # misaligned
        assert f(P, 8, None, P, P, 1, 1.4, 0, W, need, P) == E            # aliased
        assert f(None, 0, None, None, None, 1, 1.4, 0, None, 0, None) == _native.GAMER_OK
    for f in (lib.gamer_rtvd_solve_periodic, lib.gamer_rtvd_solve_periodic_f32):
        assert f(P, 0, 2, 2, P, P, 1.4, 0, W, need, Q) == E
        assert f(P, 1 << 25, 1, 1, P, P, 1.4, 0, W, need, Q) == E
        assert f(P, 2, 2, 2, P, P, 1.4, 0, W, need, P) == E
        # the first x sweep's grid: 44 work-groups per group along x, gy and gz as grid rows
        for shape in ((381301, 1, 1), (1, 65536, 1), (1, 1, 65536)):
            assert f(P, *shape, P, P, 1.4, 0, W, need, Q) == E
            assert b"relaxing TVD" in lib.gamer_last_error()


def test_periodic_argument_errors(lib):
    Q = ctypes.c_void_p(0x2000)
    for f in (lib.gamer_hydro_solve_periodic, lib.gamer_hydro_solve_periodic_f32):
        assert f(P, 0, 1, 1, P, P, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert f(P, 1, -2, 1, P, P, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert f(P, 1 << 25, 1, 1, P, P, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert f(P, 1 << 11, 1 << 11, 1 << 10, P, P, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert b"too large" in lib.gamer_last_error()
        assert f(None, 2, 2, 2, P, P, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert f(P, 2, 2, 2, None, P, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert f(P, 2, 2, 2, P, None, 1.4, None, Q, None, None) == _native.GAMER_EINVAL
        assert f(P, 2, 2, 2, P, P, 1.4, None, None, None, None) == _native.GAMER_EINVAL
        assert f(P, 2, 2, 2, P, P, 1.4, None, P, None, None) == _native.GAMER_EINVAL
        assert b"different" in lib.gamer_last_error()
        assert f(P, 2, 2, 2, P, P, 0.9, None, Q, None, None) == _native.GAMER_EINVAL
        bad = _native.GamerOpts(1.5, 7, 0)
        assert f(P, 2, 2, 2, P, P, 1.4, None, Q, None, ctypes.byref(bad)) == _native.GAMER_EINVAL
        bad = _native.GamerOpts(3.0, 0, 0)
        assert f(P, 2, 2, 2, P, P, 1.4, None, Q, None, ctypes.byref(bad)) == _native.GAMER_EINVAL


def test_cf_face_struct_layout(tmp_path):
    """gamer_cf_face as the C compiler lays it out equals the numpy record type
    the binding builds (offsets and size), compiled from the public header."""
    import subprocess
    from paper_1007_3818_amd.amr import CF_FACE_DTYPE
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "gamer_hydro.h"\n'
        "int main(void) { printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(gamer_cf_face),"
        " offsetof(gamer_cf_face, coarse_group), offsetof(gamer_cf_face, fine_group),"
        " offsetof(gamer_cf_face, dir), offsetof(gamer_cf_face, coarse_face),"
        " offsetof(gamer_cf_face, side), offsetof(gamer_cf_face, qs), offsetof(gamer_cf_face, qf));"
        " return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    f = CF_FACE_DTYPE.fields
    want = [CF_FACE_DTYPE.itemsize] + [f[n][1] for n in
                                       ("coarse_group", "fine_group", "dir", "coarse_face", "side", "qs", "qf")]
    assert got == want


def test_amr_argument_errors(lib):
    E = _native.GAMER_EINVAL
    A16 = ctypes.c_void_p(0x1000)
    A8 = ctypes.c_void_p(0x1008)
    for f in (lib.gamer_flux_accumulate, lib.gamer_flux_accumulate_f32):
        assert f(P, -1, P, 1, A16) == E
        assert f(None, 0, None, 1, None) == _native.GAMER_OK
        assert f(None, 2, P, 1, A16) == E
        assert f(P, 2, None, 1, A16) == E
        assert f(P, 2, P, 1, None) == E
        assert f(P, 2, P, 1, A8) == E
        assert b"aligned" in lib.gamer_last_error()
    for f in (lib.gamer_flux_correct, lib.gamer_flux_correct_f32):
        assert f(P, -1, P, P, 1, P, 1, P, P, None) == E
        assert f(P, 1, P, P, -1, P, 1, P, P, None) == E
        assert f(P, 1, P, P, 1, P, -5, P, P, None) == E
        assert f(None, 1, None, None, 1, None, 0, None, None, None) == _native.GAMER_OK
        assert f(None, 1, P, P, 1, P, 1, P, P, None) == E
        assert f(P, 1, P, P, 1, None, 1, P, P, None) == E
        assert f(P, 1, P, P, 1, P, 1, None, P, None) == E
        assert f(P, 1, P, P, 1, P, 1, P, None, None) == E
        assert f(P, 1, P, P, 1, ctypes.c_void_p(0x1004), 1, P, P, None) == E
        assert f(P, 1, P, P, 1, P, (1 << 32) + 1, P, P, None) == E
    for f in (lib.gamer_restrict, lib.gamer_restrict_f32):
        assert f(P, P, -1, P, 1, None) == E
        assert f(P, P, 1, P, -1, None) == E
        assert f(P, P, (1 << 27) + 1, P, 1, None) == E
        assert f(None, None, 0, None, 0, None) == _native.GAMER_OK
        assert f(None, P, 1, P, 1, None) == E
        assert f(P, None, 1, P, 1, None) == E
        assert f(P, P, 1, None, 1, None) == E


def test_other_entry_point_errors(lib):
    assert lib.gamer_step_reduce(P, 4, None, P, 1, 0.0, P, None) == _native.GAMER_EINVAL
    assert lib.gamer_step_reduce(P, 4, None, None, 1, 0.5, P, None) == _native.GAMER_EINVAL
    assert lib.gamer_step_reduce(P, 4, None, P, 40, 0.5, P, None) == _native.GAMER_EINVAL
    assert lib.gamer_step_reduce(None, 4, None, P, 1, 0.5, P, None) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt(P, 4, 0.0, 1.4, 0.5, P, 1) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt(P, 4, 0.1, 1.4, -0.5, P, 1) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt(P, 4, 0.1, 1.4, 0.5, None, 1) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt(None, 4, 0.1, 1.4, 0.5, P, 1) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt(None, 0, 0.1, 1.4, 0.5, None, 0) == _native.GAMER_OK
    # the allocation-free variant: every check comes before any device call
    big = _native.NOALLOC_MAX_GROUPS + 1
    assert lib.gamer_cfl_dt_noalloc(P, big, 0.1, 1.4, 0.5, P) == _native.GAMER_EINVAL
    assert b"above the fixed scratch" in lib.gamer_last_error()
    assert lib.gamer_cfl_dt_noalloc(P, -1, 0.1, 1.4, 0.5, P) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt_noalloc(P, 4, 0.0, 1.4, 0.5, P) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt_noalloc(P, 4, 0.1, 1.0, 0.5, P) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt_noalloc(P, 4, 0.1, 1.4, 0.5, None) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt_noalloc(None, 4, 0.1, 1.4, 0.5, P) == _native.GAMER_EINVAL
    assert lib.gamer_cfl_dt_noalloc(None, 0, 0.1, 1.4, 0.5, None) == _native.GAMER_OK
    assert lib.gamer_conserved_sums(P, 4, 0.0, P, 1) == _native.GAMER_EINVAL
    assert lib.gamer_conserved_sums(P, 4, 0.1, None, 1) == _native.GAMER_EINVAL
    assert lib.gamer_group_stats(P, 4, 1.0, P) == _native.GAMER_EINVAL
    assert lib.gamer_group_stats(None, 4, 1.4, P) == _native.GAMER_EINVAL
    assert lib.gamer_pack_periodic(P, 0, 1, 1, P) == _native.GAMER_EINVAL
    assert lib.gamer_pack_periodic(None, 1, 1, 1, P) == _native.GAMER_EINVAL
    assert lib.gamer_pack_periodic_f32(P, 1, 1, 1, None) == _native.GAMER_EINVAL


def test_stream_is_per_thread_state(lib):
    import threading
    assert lib.gamer_set_stream(ctypes.c_void_p(0x1234)) == 0
    seen = []
    t = threading.Thread(target=lambda: seen.append(lib.gamer_get_stream()))
    t.start()
    t.join()
    assert lib.gamer_get_stream() == 0x1234
    assert seen == [None]
    lib.gamer_set_stream(None)


def test_binding_rejects_host_tensors():
    import torch
    from paper_1007_3818_amd import hydro
    with pytest.raises(ValueError):
        hydro.hydro_solve(torch.zeros((1, 5, 20, 20, 20), dtype=torch.float64), 0.1, 0.1, 1.4)
    with pytest.raises(TypeError):
        hydro.hydro_solve(torch.zeros((1, 5, 20, 20, 20), dtype=torch.float16), 0.1, 0.1, 1.4)
