"""Streams and graphs around the batched step, through the binding.

  * The batched step (solve + reduce) captured once in a HIP graph and replayed
    four times, with eager library work and synchronisations between the
    replays: every replay's new state, group stats, time step and totals equal
    the eager step's, bitwise.
  * Two batches stepped at the same time on two streams (the solver keeps no
    state between launches and uses no library scratch): each result equals the
    same step run alone, bitwise.
"""
import pytest
import torch

from paper_1007_3818_amd import hydro, workloads as W

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def _batch(gpu, n=64, seed_workload=2, dtype=torch.float64):
    st, dh = W.smooth_modes(n=n, kmax=2, workload=seed_workload)
    g = n // 16
    s = st.to(dtype).to(gpu)
    return s, hydro.pack_periodic(s, g, g, g), dh


def test_graph_replays_equal_eager_step(gpu):
    for dtype in (torch.float64, torch.float32):
        s, pad, dh = _batch(gpu, dtype=dtype)
        n = pad.shape[0]
        dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
        dt_dev = torch.empty(1, dtype=torch.float64, device=gpu)
        stats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
        totals = torch.empty(7, dtype=torch.float64, device=gpu)
        out = torch.empty_like(s)
        hydro.group_stats(s, G53, out=stats)
        hydro.step_reduce(stats, None, dh_dev, 0.5, dt_out=dt_dev, totals_out=totals)
        dt0 = dt_dev.clone()

        def step():
            hydro.hydro_solve_batched(pad, None, dt_dev, dh_dev, G53, out=out, group_stats=stats)
            hydro.step_reduce(stats, None, dh_dev, 0.5, dt_out=dt_dev, totals_out=totals)

        step()
        torch.cuda.synchronize()
        want = [t.clone() for t in (out, stats, dt_dev, totals)]
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                step()
        torch.cuda.current_stream().wait_stream(side)
        other = torch.empty((n, 8), dtype=torch.float64, device=gpu)
        for r in range(4):
            # eager work between replays: another stats pass, clearing the outputs
            hydro.group_stats(s, G53, out=other)
            out.zero_()
            stats.zero_()
            totals.zero_()
            dt_dev.copy_(dt0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            got = (out, stats, dt_dev, totals)
            for name, a, b in zip(("state", "stats", "dt", "totals"), got, want):
                assert torch.equal(a, b), (dtype, r, name)
        print(f"[graph] {dtype}: 4 replays equal the eager step bitwise", flush=True)
        del graph


def test_two_streams_at_once(gpu):
    s1, p1, dh1 = _batch(gpu, n=64, seed_workload=2)
    s2, p2, dh2 = _batch(gpu, n=64, seed_workload=4)
    dts = [torch.tensor([0.3 * dh], dtype=torch.float64, device=gpu) for dh in (dh1, dh2)]
    dhs = [torch.tensor([dh], dtype=torch.float64, device=gpu) for dh in (dh1, dh2)]
    alone = [hydro.hydro_solve_batched(p, None, dt, dh_, G53) for p, dt, dh_ in zip((p1, p2), dts, dhs)]
    torch.cuda.synchronize()
    outs = [torch.empty_like(a) for a in alone]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    for k in range(3):  # a few rounds, so that the launches overlap
        for i, st in enumerate(streams):
            with torch.cuda.stream(st):
                hydro.hydro_solve_batched((p1, p2)[i], None, dts[i], dhs[i], G53, out=outs[i])
    torch.cuda.synchronize()
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)
