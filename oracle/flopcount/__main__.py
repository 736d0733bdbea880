"""Count the oracle's arithmetic per cell-update on samples of the benchmark
workloads (TEST AND MEASUREMENT INFRASTRUCTURE; see the package docstring).

    python -m oracle.flopcount

Samples: 32 groups spread evenly over the group index of each grid, their
padded inputs evaluated directly from the seeded workload, one step at the
sample's own CFL time step (C = 0.5).  Prints one JSON object.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import flopcount as fc  # noqa: E402
from paper_1007_3818_amd import workloads as W  # noqa: E402

GAMMA = 5.0 / 3.0
SAMPLE = 32


def sample_ids(n):
    g = (n // 16) ** 3
    return np.linspace(0, g - 1, SAMPLE).round().astype(np.int64)


def sample(n, kmax, workload, ghost=2):
    pad = W.smooth_modes_padded(sample_ids(n), n=n, kmax=kmax, workload=workload, ghost=ghost).numpy()
    c = slice(ghost, ghost + 16)
    dt = oracle.cfl_dt(np.ascontiguousarray(pad[:, :, c, c, c]), 1.0 / n, GAMMA, 0.5)
    return pad, dt, 1.0 / n


def per_cell(counts):
    cells = counts["cells"]
    return {k: counts[k] / cells for k in (*fc.KINDS, "flops")}


def main():
    res = {}
    pad, dt, dh = sample(1024, 8, 5)
    c, _ = fc.hydro_step(pad, dt, dh, GAMMA)
    res["muscl_hancock_roe workload 5 (1024^3)"] = {"per_cell": per_cell(c), "fallbacks": c["fallbacks"]}
    st, _ = fc.hydro_stages(pad, dt, dh, GAMMA)
    res["muscl_hancock_roe workload 5 (1024^3), by stage"] = {k: per_cell(v) for k, v in st.items()}
    pad, dt, dh = sample(256, 4, 2)
    c, _ = fc.hydro_step(pad, dt, dh, GAMMA)
    res["muscl_hancock_roe workload 2 (256^3)"] = {"per_cell": per_cell(c), "fallbacks": c["fallbacks"]}
    c, _ = fc.ctu_step(pad, dt, dh, GAMMA)
    res["ctu workload 2 (256^3)"] = {"per_cell": per_cell(c), "fallbacks": c["fallbacks"]}
    pad3, dt3, dh3 = sample(256, 4, 2, ghost=3)
    c, _ = fc.rtvd_step(pad3, dt3, dh3, GAMMA, order=0)
    res["relaxing_tvd workload 2 (256^3)"] = {"per_cell": per_cell(c), "bad": c["bad"]}
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
