"""Per-step record of max|u| (sfac_plan_trace / sfac_plan_read_trace) against the oracle.

The maximum norm after every step is what Example 4 (Sec. 5) follows; Theorem 1 bounds it by
1. The record must hold, for step k, the largest |u| of the state after step k: against the
oracle's states to the FP64 parity tolerance, against the sticky sfac_plan_flags maximum
exactly, and bitwise the same whether the steps run in one call or several, with graph
chunks or single steps.
"""
import numpy as np
import pytest
from conftest import progress

from oracle import sfac_oracle as O
from paper_2209_08437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    progress(msg)   # past the output capture: long tests show they are alive


def _oracle_maxes(u0, ns, alphas, eps, hs, tau, steps):
    out = []
    O.two_level_solve(u0, ns, alphas, eps, hs, tau, steps, observe=lambda k, u: out.append(np.abs(u).max()))
    return np.array(out)


@pytest.mark.parametrize("which", ["plain_2d_63", "3d_small"])
def test_trace_matches_oracle_per_step(sfac_lib, which):
    import torch
    from paper_2209_08437_amd import sfac
    if which == "plain_2d_63":
        inst = W.plain_2d_63()
        ns, alphas, eps, hs, tau, u0 = inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau, inst.u0
    else:
        ns, alphas, eps, tau = (17, 9, 33), (1.3, 1.6, 1.9), 0.3, 0.02
        hs = W.mesh_widths(ns)
        u0 = W.uniform_field(tuple(reversed(ns)), -0.95, 0.95, seed=41)
    steps = 100
    ref = _oracle_maxes(u0, ns, alphas, eps, hs, tau, steps)
    _say(f"case trace {which}")
    u = torch.tensor(u0, device="cuda")
    with sfac.Plan(ns, alphas, eps, tau, hs, "f64") as p:
        p.trace(150)
        p.step(u, 70)                 # two 32-step graph replays and six one-step replays
        p.step(u, 30)
        vals, count = p.read_trace()
        _, max_abs = p.flags()
    assert count == steps and len(vals) == steps
    rel = np.abs(vals - ref).max() / np.abs(ref).max()
    _say(f"  max rel diff to the oracle {rel:.2e}; max|u| {vals.max():.6f}")
    assert rel <= 1e-12
    assert vals.max() == max_abs              # the same folded maximum as the sticky status
    assert np.all(vals <= 1.0)


def test_trace_capacity_restart_and_stop(sfac_lib):
    import torch
    from paper_2209_08437_amd import sfac
    inst = W.plain_2d_63()
    args = (inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, "f64")
    u = torch.tensor(inst.u0, device="cuda")
    with sfac.Plan(*args) as p:
        p.trace(100)
        p.step(u, 60)
        full, n = p.read_trace()
    assert n == 60 and len(full) == 60
    # a smaller record: steps beyond it are counted, not recorded; single-step calls give the
    # same bits as graph chunks
    u = torch.tensor(inst.u0, device="cuda")
    with sfac.Plan(*args) as p:
        p.trace(25)
        for _ in range(60):
            p.step(u, 1)
        part, n = p.read_trace()
        assert n == 60 and len(part) == 25
        assert np.array_equal(part, full[:25])
        # the pass timing is not part of the record; a restart zeroes it
        p.time_passes(u, 3)
        assert p.read_trace()[1] == 60
        p.trace(10)
        p.step(u, 4)
        vals, n = p.read_trace()
        assert n == 4 and len(vals) == 4 and np.all(vals > 0)
        # stop: no record, stepping goes on
        p.trace(0)
        p.step(u, 5)
        vals, n = p.read_trace()
        assert n == 0 and len(vals) == 0


def test_trace_fp32(sfac_lib):
    import torch
    from paper_2209_08437_amd import sfac
    inst = W.plain_2d_63()
    ref = _oracle_maxes(inst.u0, inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau, inst.steps)
    u = torch.tensor(inst.u0.astype(np.float32), device="cuda")
    with sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, "f32") as p:
        p.trace(inst.steps)
        p.step(u, inst.steps)
        vals, n = p.read_trace()
    assert n == inst.steps
    e = float(np.abs(vals - ref).max() / np.abs(ref).max())
    print(f"  fp32 per-step max|u| rel err {e:.3e}", flush=True)
    assert e <= 5e-5   # the FP32 parity bound of the state (increment form)
