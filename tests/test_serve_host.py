"""Scheduling logic of the solve server, on the CPU: a stand-in executor steps states with the
oracle and advances a simulated clock by a modelled device time, so admission, continuous
batching, rejection and latency accounting are checked without a GPU."""
import numpy as np
import pytest

from oracle import sfac_oracle as O
from paper_2209_08437_amd import serve, workloads as W


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class OracleExecutor:
    """Steps with the CPU oracle; each grouped step costs `per_point_step` simulated seconds per
    grid-point-step plus a fixed tick overhead."""

    def __init__(self, clock, per_point_step=1e-7, overhead=1e-3):
        self.clock = clock
        self.rate = per_point_step
        self.overhead = overhead
        self.log = []

    def bytes_needed(self, inst, dtype):
        return int(np.prod(inst.ns)) * (8 if dtype == "f64" else 4)

    def admit(self, inst, dtype):
        ops = O.axis_operators(inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau)
        return {"inst": inst, "ops": ops, "u": np.array(inst.u0, dtype=np.float64)}

    def step(self, handles, nsteps):
        self.log.append([(id(h), k) for h, k in zip(handles, nsteps)])
        work = 0
        for h, k in zip(handles, nsteps):
            h["u"] = O.two_level_solve(h["u"], None, None, None, None, h["inst"].tau, k, ops=h["ops"])
            work += int(np.prod(h["inst"].ns)) * k
        self.clock.t += self.overhead + work * self.rate

    def retire(self, handle):
        return handle["u"], 0, float(np.abs(handle["u"]).max())


def _requests(count=10, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for rid in range(count):
        t += float(rng.exponential(0.002))
        d = 2 if rid % 3 else 3
        n = int(rng.integers(4, 12)) if d == 3 else int(rng.integers(6, 30))
        ns = (n,) * d
        inst = W.Instance(ns, tuple(float(a) for a in rng.uniform(1.1, 1.9, d)), float(rng.uniform(0.02, 0.2)),
                          float(rng.uniform(1e-3, 1e-2)), W.mesh_widths(ns), int(rng.integers(3, 40)))
        inst.u0 = W.uniform_field(inst.shape, -0.9, 0.9, seed=100 + rid)
        out.append(W.Request(rid, t, inst, "f64" if rid % 2 else "f32"))
    return out


def test_all_complete_with_results_equal_to_lone_solves():
    clock = SimClock()
    ex = OracleExecutor(clock)
    reqs = _requests()
    srv = serve.Server(ex, budget_bytes=10 ** 9, tick_steps=7, clock=clock, sleep=clock.sleep)
    tickets, summ = srv.run(reqs)
    assert summ["completed"] == len(reqs) and summ["rejected"] == 0
    for r, tk in zip(sorted(reqs, key=lambda r: r.rid), tickets):
        i = r.inst
        alone = O.two_level_solve(i.u0, i.ns, i.alphas, i.eps, i.hs, i.tau, i.steps)
        assert np.array_equal(tk.result, alone)          # ticks split the steps; bitwise the same
        assert tk.latency >= 0 and tk.admitted >= tk.arrival
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
    # admission cost (plan tables and upload) is timed per admitted request
    assert 0 <= summ["admit_p50_ms"] <= summ["admit_max_ms"]
    assert summ["p50_queue_wait_s"] >= 0


def test_budget_limits_admission_and_oversize_is_rejected():
    clock = SimClock()
    ex = OracleExecutor(clock)
    reqs = _requests(12, seed=5)
    sizes = [ex.bytes_needed(r.inst, r.dtype) for r in reqs]
    budget = max(sizes) - 1                      # the largest requests do not fit, the rest do
    too_big = {r.rid for r, s in zip(reqs, sizes) if s > budget}
    assert too_big and len(too_big) < len(reqs)
    srv = serve.Server(ex, budget_bytes=budget, tick_steps=5, clock=clock, sleep=clock.sleep)
    tickets, summ = srv.run(reqs)
    assert summ["peak_bytes"] <= budget
    for tk in tickets:
        assert tk.rejected == (tk.rid in too_big)
        assert (tk.finished is None) == (tk.rid in too_big)
    assert summ["completed"] == len(reqs) - len(too_big)


def test_fifo_admission_and_continuous_joining():
    clock = SimClock()
    ex = OracleExecutor(clock, per_point_step=1e-5)
    reqs = _requests(8, seed=7)
    srv = serve.Server(ex, budget_bytes=10 ** 9, tick_steps=3, max_active=3, clock=clock, sleep=clock.sleep)
    tickets, summ = srv.run(reqs)
    order = sorted(tickets, key=lambda t: t.arrival)
    adm = [t.admitted for t in order]
    assert adm == sorted(adm)                       # first come, first served
    assert summ["peak_active"] == 3
    # somebody was admitted while earlier requests were still running (joined mid-flight)
    joined = any(b.admitted < a.finished and b.admitted > a.admitted for a in order for b in order)
    assert joined
    # every grouped step advanced each active request by at most the tick size
    assert all(k <= 3 for tick in ex.log for _, k in tick)


def test_server_refuses_negative_steps_and_flags_untouched_states():
    """A request with negative steps is refused without stopping the stream; a zero-step
    request returns its initial state with the flags the library would set for it."""
    from paper_2209_08437_amd import sfac
    clock = SimClock()
    ex = OracleExecutor(clock)
    reqs = _requests(4, seed=9)
    reqs[1].inst.steps = -2
    reqs[2].inst.steps = 0
    reqs[2].inst.u0 = reqs[2].inst.u0 * 1.5            # |u0| > 1: outside the DMP's premise
    srv = serve.Server(ex, budget_bytes=10 ** 9, tick_steps=5, clock=clock, sleep=clock.sleep)
    tickets, summ = srv.run(reqs)
    assert tickets[1].rejected and tickets[1].finished is None
    assert summ["completed"] == 3 and summ["rejected"] == 1
    t2 = tickets[2]
    assert np.array_equal(t2.result, reqs[2].inst.u0)
    assert t2.flags == sfac.FLAG_ABOVE_ONE and t2.max_abs == np.abs(reqs[2].inst.u0).max() > 1
    bad = np.array(reqs[2].inst.u0)
    bad[0, 0] = np.nan
    f, m = serve.initial_flags(bad)
    assert f & sfac.FLAG_NONFINITE and f & sfac.FLAG_ABOVE_ONE and np.isfinite(m)
    assert serve.initial_flags(np.zeros((3, 3))) == (0, 0.0)
    for i in (0, 3):
        inst = reqs[i].inst
        alone = O.two_level_solve(inst.u0, inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau, inst.steps)
        assert np.array_equal(tickets[i].result, alone)


def test_online_service_futures_from_several_threads():
    """Service: submissions from two threads, results through futures, bitwise equal to lone
    solves; an oversize request fails its future alone; close() drains; no submit afterwards."""
    import threading
    clock = SimClock()
    reqs = _requests(count=12, seed=11)
    big = W.Instance((40, 40), (1.5, 1.5), 0.1, 0.01, W.mesh_widths((40, 40)), 5)
    big.u0 = W.uniform_field(big.shape, -0.5, 0.5, seed=1)
    zero = W.Instance((9, 9), (1.5, 1.5), 0.1, 0.01, W.mesh_widths((9, 9)), 0)
    zero.u0 = W.uniform_field(zero.shape, -0.5, 0.5, seed=2)
    futs = {}
    need = max(int(np.prod(r.inst.ns)) * 8 for r in reqs)
    budget = 12000                    # every small request fits (a few at a time); the big one never
    assert need <= budget < 8 * 40 * 40
    with serve.Service(lambda: OracleExecutor(clock), budget_bytes=budget, tick_steps=5) as svc:
        def worker(part):
            for r in part:
                futs[r.rid] = svc.submit(r.inst, r.dtype)
        threads = [threading.Thread(target=worker, args=(reqs[i::2],)) for i in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        f_big = svc.submit(big, "f64")
        f_zero = svc.submit(zero, "f32")
        with pytest.raises(ValueError):
            svc.submit(zero, "bf16")
        neg = W.Instance((9, 9), (1.5, 1.5), 0.1, 0.01, W.mesh_widths((9, 9)), -1)
        neg.u0 = zero.u0
        with pytest.raises(ValueError, match="steps"):
            svc.submit(neg, "f64")
    with pytest.raises(RuntimeError):
        svc.submit(zero, "f64")
    for r in reqs:
        i = r.inst
        out, flags, vmax = futs[r.rid].result(timeout=0)
        alone = O.two_level_solve(i.u0, i.ns, i.alphas, i.eps, i.hs, i.tau, i.steps)
        assert np.array_equal(out, alone) and flags == 0 and vmax == np.abs(alone).max()
    with pytest.raises(ValueError, match="budget"):
        f_big.result(timeout=0)
    assert np.array_equal(f_zero.result(timeout=0)[0], zero.u0)
    st = svc.stats()
    assert st["submitted"] == 14 and st["completed"] == 13 and st["rejected"] == 1 and st["failed"] == 0
    assert st["peak_bytes"] <= budget


def test_online_service_step_failure_reaches_futures():
    """A failing grouped step fails the futures of the requests in it and the service goes on."""
    clock = SimClock()

    class Flaky(OracleExecutor):
        calls = 0

        def step(self, handles, nsteps):
            Flaky.calls += 1
            if Flaky.calls == 1:
                raise RuntimeError("device step failed")
            super().step(handles, nsteps)

    r1, r2 = _requests(count=2, seed=5)
    with serve.Service(lambda: Flaky(clock), budget_bytes=10 ** 9, tick_steps=100) as svc:
        f1 = svc.submit(r1.inst, "f64")
        with pytest.raises(RuntimeError, match="device step failed"):
            f1.result(timeout=30)
        f2 = svc.submit(r2.inst, "f64")
        out, _, _ = f2.result(timeout=30)
    i = r2.inst
    assert np.array_equal(out, O.two_level_solve(i.u0, i.ns, i.alphas, i.eps, i.hs, i.tau, i.steps))
    assert svc.stats()["failed"] == 1


def test_online_service_reports_executor_start_failure():
    def broken():
        raise RuntimeError("no device")
    with pytest.raises(RuntimeError, match="no device"):
        serve.Service(broken, budget_bytes=1)


def test_online_service_refuses_device_executors():
    """Device executors stay off the online service (see Service's docstring)."""
    class DeviceStandIn(OracleExecutor):
        on_device = True

    with pytest.raises(RuntimeError, match="not enabled for device executors"):
        serve.Service(serve.GpuExecutor, budget_bytes=1)
    with pytest.raises(RuntimeError, match="not enabled for device executors"):
        serve.Service(lambda: DeviceStandIn(SimClock()), budget_bytes=1)
