"""Writes the extended-precision references of the long runs on the largest grids, as sampled
values (the full states are too large to keep): the 1023^2 workload over all its 1000 steps, and
the batched workload's instances with n = 511 and n = 1023 over their 500 steps.

Each reference is oracle.sfac_oracle.extended_solve (the two-level step of eq. (finalstrang)
through Remark 1's diagonalisation, every table and operation in numpy's longdouble) on the
seeded input of paper_2209_08437_amd.workloads; nothing else is called. The files hold the
state's largest |u| (the scale of the relative max-norm) and 2048 seeded sample positions with
their values rounded to float64, plus the position of the largest |u|.

    python tests/golden/make_extended_references.py          # about 20 minutes on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import sfac_oracle as O  # noqa: E402
from paper_2209_08437_amd import workloads as W  # noqa: E402

SAMPLES = 2048


def cases():
    b = W.batched_2d()
    return [("extended_large_2d_1023.json", "the 2D single large instance (N = 1023, 1000 steps)", W.large_2d_1023()),
            ("extended_batched_2d_37.json", "instance 37 of the batched workload (seed 4; n = 1023, 500 steps)", b[37]),
            ("extended_batched_2d_40.json", "instance 40 of the batched workload (seed 4; n = 511, 500 steps)", b[40])]


def write(name, what, inst):
    t = time.time()
    x = O.extended_solve(inst.u0, inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau, inst.steps)
    flat = x.reshape(-1)
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([rng.choice(flat.size, SAMPLES, replace=False), [int(np.abs(flat).argmax())]]))
    out = {
        "source": f"extended-precision reference of {what}: oracle extended_solve (eq. (finalstrang), "
                  f"Remark 1, numpy longdouble), written by tests/golden/make_extended_references.py",
        "ns": list(inst.ns), "alphas": list(inst.alphas), "eps": inst.eps, "tau": inst.tau, "steps": inst.steps,
        "longdouble_eps": float(np.finfo(np.longdouble).eps),
        "max_abs": float(np.abs(flat).max()),
        "index": [int(i) for i in idx],
        "value": [float(flat[i]) for i in idx],
    }
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: {inst.ns} x {inst.steps} steps in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    want = sys.argv[1:]
    for name, what, inst in cases():
        if not want or name in want:
            write(name, what, inst)
