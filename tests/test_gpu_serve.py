"""The solve server on the GPU: a short mixed stream (2D and 3D, FP64 and FP32, uneven sizes
and step counts) under a memory budget that forces queueing; every served result must be
bitwise equal to the same solve run alone with its own plan, and FP64 results must match the
oracle."""
import sys

import numpy as np
import pytest

from oracle import sfac_oracle as O
from paper_2209_08437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stream(count=10, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for rid in range(count):
        t += float(rng.exponential(0.01))
        d = 3 if rid % 3 == 0 else 2
        n = int(rng.integers(8, 34)) if d == 3 else int(rng.integers(31, 131))
        ns = (n,) * d
        inst = W.Instance(ns, tuple(float(a) for a in rng.uniform(1.1, 1.9, d)), float(rng.uniform(0.02, 0.2)),
                          float(rng.uniform(1e-3, 1e-2)), W.mesh_widths(ns), int(rng.integers(5, 41)))
        inst.u0 = W.uniform_field(inst.shape, -0.9, 0.9, seed=200 + rid)
        out.append(W.Request(rid, t, inst, "f64" if rid % 2 else "f32"))
    return out


def test_served_results_equal_lone_solves(sfac_lib):
    import torch
    from paper_2209_08437_amd import serve, sfac
    reqs = _stream()
    ex = serve.GpuExecutor()
    sizes = [ex.bytes_needed(r.inst, r.dtype) for r in reqs]
    budget = max(sizes) + sorted(sizes)[len(sizes) // 2]     # forces some requests to wait
    print(f"case served stream of {len(reqs)} requests, budget {budget} B", flush=True)
    srv = serve.Server(ex, budget_bytes=budget, tick_steps=8)
    tickets, summ = srv.run(reqs)
    print({k: summ[k] for k in ("completed", "ticks", "peak_active", "p50_latency_s", "p99_latency_s")}, flush=True)
    assert summ["completed"] == len(reqs) and summ["rejected"] == 0
    assert summ["peak_bytes"] <= budget
    for r, tk in zip(sorted(reqs, key=lambda r: r.rid), tickets):
        i = r.inst
        tdt = torch.float64 if r.dtype == "f64" else torch.float32
        u = torch.tensor(i.u0, dtype=tdt, device="cuda")
        with sfac.Plan(i.ns, i.alphas, i.eps, i.tau, i.hs, r.dtype) as p:
            p.step(u, i.steps)
        torch.cuda.synchronize()
        alone = u.double().cpu().numpy()
        assert np.array_equal(tk.result, alone), r.rid
        assert tk.flags == 0 and tk.max_abs <= 1.0
        if r.dtype == "f64" and r.rid < 6:
            ref = O.two_level_solve(i.u0, i.ns, i.alphas, i.eps, i.hs, i.tau, i.steps)
            assert np.abs(tk.result - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.timeout(600)
def test_served_full_size_requests_equal_lone_solves(sfac_lib):
    """Requests at the served stream's largest sizes (a 255^3 FP64 and a 1023^2 FP32 solve)
    beside small ones, under a budget that holds both large ones at once: each result bitwise
    equal to its lone solve."""
    import torch
    from paper_2209_08437_amd import autotune, serve, sfac
    rng = np.random.default_rng(77)
    reqs = []
    specs = [((255, 255, 255), "f64", 30), ((1023, 1023), "f32", 60), ((40, 40, 40), "f32", 25),
             ((300, 300), "f64", 45), ((31, 31, 31), "f64", 12)]
    t = 0.0
    for rid, (ns, dt, steps) in enumerate(specs):
        t += 0.002
        inst = W.Instance(ns, tuple(float(a) for a in rng.uniform(1.1, 1.9, len(ns))), float(rng.uniform(0.02, 0.2)),
                          float(rng.uniform(1e-3, 1e-2)), W.mesh_widths(ns), steps)
        inst.u0 = W.uniform_field(inst.shape, -0.9, 0.9, seed=300 + rid)
        reqs.append(W.Request(rid, t, inst, dt))
    ex = serve.GpuExecutor()
    sizes = [ex.bytes_needed(r.inst, r.dtype) for r in reqs]
    print(f"case served full-size requests, bytes {sizes}", flush=True)
    srv = serve.Server(ex, budget_bytes=sum(sizes), tick_steps=20)
    tickets, summ = srv.run(reqs)
    ex.close()
    assert summ["completed"] == len(reqs) and summ["peak_bytes"] <= sum(sizes)
    for r, tk in zip(reqs, tickets):
        i = r.inst
        tdt = torch.float64 if r.dtype == "f64" else torch.float32
        u = torch.tensor(i.u0, dtype=tdt, device="cuda")
        # the server's plans take the packaged schedule of their shape (1023^2 has one)
        sched = autotune.lookup(i.ns, r.dtype) or {}
        with sfac.Plan(i.ns, i.alphas, i.eps, i.tau, i.hs, r.dtype, **sched) as p:
            p.step(u, i.steps)
        torch.cuda.synchronize()
        assert np.array_equal(tk.result, u.double().cpu().numpy()), r.rid
        assert tk.flags == 0 and tk.max_abs <= 1.0


@pytest.mark.skip(reason="the one run of the online service with the device executor on its worker thread "
                         "ended in a host segmentation fault whose cause has not been found; the service "
                         "refuses device executors until it is")
def test_online_service_results_equal_lone_solves(sfac_lib):
    """The online form: submissions from two threads, the worker thread owning the device
    executor; each future's state is bitwise the lone solve's."""
    import threading
    import torch
    from paper_2209_08437_amd import serve, sfac
    reqs = _stream(count=8, seed=23)
    ex0 = serve.GpuExecutor()
    sizes = [ex0.bytes_needed(r.inst, r.dtype) for r in reqs]
    ex0.close()
    budget = max(sizes) + min(sizes)
    print(f"case online service, {len(reqs)} requests, budget {budget} B", flush=True)
    futs = {}
    with serve.Service(serve.GpuExecutor, budget_bytes=budget, tick_steps=6) as svc:
        def worker(part):
            for r in part:
                futs[r.rid] = svc.submit(r.inst, r.dtype)
        threads = [threading.Thread(target=worker, args=(reqs[i::2],)) for i in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        results = {rid: f.result(timeout=120) for rid, f in futs.items()}
    st = svc.stats()
    print(st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["peak_bytes"] <= budget
    for r in reqs:
        i = r.inst
        tdt = torch.float64 if r.dtype == "f64" else torch.float32
        u = torch.tensor(i.u0, dtype=tdt, device="cuda")
        with sfac.Plan(i.ns, i.alphas, i.eps, i.tau, i.hs, r.dtype) as p:
            p.step(u, i.steps)
        torch.cuda.synchronize()
        out, flags, vmax = results[r.rid]
        assert np.array_equal(out, u.double().cpu().numpy()), r.rid
        assert flags == 0 and vmax <= 1.0
