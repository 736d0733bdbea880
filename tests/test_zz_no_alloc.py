"""The allocation-free CFL entry point (gamer_cfl_dt_noalloc) through the C
ABI, against gamer_cfl_dt on the same groups: bitwise the same time step (the
same kernels in the same order), on consecutive calls whose second batch is
smaller than the first (the fixed scratch keeps the first call's stats), at
the largest batch the fixed scratch holds, and beside a non-physical cell
(NaN in both).  Sizes above the limit are rejected before any device work."""
import pytest
import torch

from paper_1007_3818_amd import _native, hydro, workloads as W

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def _pair(groups, dh, cfl=0.5):
    want = hydro.cfl_dt(groups, dh, G53, cfl, device_out=True)
    got = torch.full((1,), float("nan"), dtype=torch.float64, device=groups.device)
    hydro.cfl_dt_noalloc(groups, dh, G53, cfl, out=got)
    torch.cuda.synchronize()
    return float(got.item()), float(want.item())


def test_noalloc_matches_allocating_call_twice(gpu):
    print("[noalloc] 64^3 log-normal (64 groups), then 16 of them", flush=True)
    st, dh = W.cosmo_like(n=64)
    st = st.to(gpu)
    got, want = _pair(st, dh)
    assert got == want and 0.0 < got < float("inf"), (got, want)
    small = st[16:32].contiguous()
    got2, want2 = _pair(small, dh, cfl=0.4)
    assert got2 == want2 and 0.0 < got2 < float("inf"), (got2, want2)
    # the smaller batch's own value, not the first call's
    assert got2 != got


def test_noalloc_at_the_limit_and_with_a_bad_cell(gpu):
    n = _native.NOALLOC_MAX_GROUPS
    print(f"[noalloc] {n} uniform groups (the fixed scratch's limit)", flush=True)
    W_ = torch.tensor([0.9, 0.3, -0.2, 0.1, 1.2], dtype=torch.float64)
    U = W.conserved(*W_, G53)
    st = U.to(gpu)[None, :, None, None, None].expand(n, 5, 16, 16, 16).contiguous()
    got, want = _pair(st, 1.0 / 1024)
    assert got == want, (got, want)
    cs = (G53 * 1.2 / 0.9) ** 0.5
    exact = 0.5 / 1024 / (0.3 + 0.2 + 0.1 + 3 * cs)
    assert abs(got - exact) <= 4e-15 * exact
    del st
    torch.cuda.empty_cache()
    print("[noalloc] 5 groups with one non-physical cell", flush=True)
    st = U.to(gpu)[None, :, None, None, None].expand(5, 5, 16, 16, 16).contiguous()
    st[3, 4, 7, 8, 9] = -1.0  # E < 0: p < 0
    got, want = _pair(st, 0.1)
    assert got != got and want != want  # NaN in both


def test_noalloc_rejects_sizes_above_the_limit(gpu):
    st = torch.zeros((1, 5, 16, 16, 16), dtype=torch.float64, device=gpu)
    out = torch.zeros(1, dtype=torch.float64, device=gpu)
    lib = _native.lib()
    rc = lib.gamer_cfl_dt_noalloc(st.data_ptr(), _native.NOALLOC_MAX_GROUPS + 1, 0.1, G53, 0.5, out.data_ptr())
    assert rc == _native.GAMER_EINVAL
    assert float(out.item()) == 0.0
