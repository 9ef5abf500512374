"""Throughput of the two-level Strang step on one MI355X: grid-point-steps per second.

A bench step is one time step of the solver (J^Q_{tau/2}, e^{tau/2 C} e^{tau S} e^{tau/2 C}
along every axis, J^Q_{tau/2}) over the whole grid of the workload. The default workload is
the largest single-GPU instance: 3D, N = 255 per axis (16.6 M points), alpha = (1.2, 1.5, 1.8),
eps = 0.08, tau = 5e-3, FP64, and the default K = 200 timed steps is its full run. The state is
resident in HBM before the timed region starts; the timed region is one sfac_step call of K
steps (HIP graph replays: K / 32 replays of a 32-step graph and one replay per set bit of the
rest, all captured beforehand by untimed runs of K steps from a copy of the initial state, kept
up for a quarter of a second so that the device's clocks are up) bracketed by device
synchronizations.

Each axis pass runs the schedule (method, kernel, elements per thread, lines per block) that
the autotuner picked on an MI355X for this shape, read from the table that ships with the
package (`--tune-cache none` tunes afresh on the device at hand).

Besides the headline value the JSON line carries: the FP32 rate of the same workload, the 2D
1023^2 instance (FP64 and FP32) and the 64-instance batched workload (FP32 and FP64 grouped
launches against the same instances on plain FP64 plans one after another) as sub-objects, the
roofline of the dominant launch of each single instance, the CPU oracle timed on a bounded sample with the max-norm error of the GPU results
against it (the 63^3 subsample of the 3D instance over all its steps, and the 1023^2 instance
over all its steps), and the one-level scheme with the exact exponential that the paper
compares the two-level scheme with, run on the GPU over the same steps.

Roofline. Each axis pass does the conventional FFT count of flops on every point: 6 transforms
of 5 L log2 L flops per complex line of 2 real lines, i.e. 15 log2 N flops per point, plus 9 for
the three spectrum scalings and the two psi twiddles, plus the nonlinear half-steps (about 20
flops per point per step, split over the d passes). Steps alternate their axis order (1..d, then
d..1), so at every step boundary one launch covers the same axis twice: it reads and writes the
state once (2 x points x element bytes) for two passes' flops. In steady state two steps of the
3D instance launch axis 2 twice, axis 3 once (two passes) and axis 1 once (two passes); two steps
of a 2D instance launch each axis once (two passes). The roofline object describes the launch
that takes the largest share of that time. Whichever of its algorithmic bytes and flops takes
longer at the published peaks (8 TB/s HBM; 78.6 FP64 / 157.3 FP32 TFLOP/s vector) bounds it: a
single 3D N = 255 FP64 pass moves 16 B per point for 136 flops (8.5 flop/B, below the 9.8 flop/B
ridge), bound by HBM; a fused one does 272 flops on the same bytes, and a fused 2D N = 1023 one
338, bound by arithmetic. `achieved` is the algorithmic flops (or bytes) per launch over the
launch's mean duration, measured here with HIP events around a graph of back-to-back launches of
that kind on the plan's stream. `traffic` is the HBM bytes per launch measured with hardware
counters (rocprofv3 FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy kernel) when the
committed record matches the current kernel sources.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point-steps/s (N^d·steps/s) FP64 vs FP32 + HBM GB/s; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}     # MI355X published vector peaks
MFMA_F64_PEAK_TFLOPS = 78.6                         # MI355X published dense FP64 matrix peak
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from paper_2209_08437_amd import workloads as W
    if name == "large_2d_1023":
        return W.large_2d_1023(), "2D single large instance: [-1,1]^2, N=1023 per axis, alpha=(1.3,1.7), eps=0.05, tau=1e-3, 1000 steps, u0 = 0.9 tanh of a smoothed seeded normal field"
    if name == "large_3d_255":
        return W.large_3d_255(), "3D single instance: [-1,1]^3, N=255 per axis, alpha=(1.2,1.5,1.8), eps=0.08, tau=5e-3, 200 steps, u0 uniform in [-0.5,0.5]"
    if name == "plain_2d_63":
        return W.plain_2d_63(), "2D plain method: [-1,1]^2, N=63 per axis, alpha=(1.5,1.5), eps=0.1, tau=0.01, 100 steps, u0 uniform in [-0.9,0.9]"
    raise SystemExit(f"unknown workload {name}")


def pass_flops(inst, axis):
    """Algorithmic flops of one pass along `axis` (0-based) over the whole grid."""
    import math
    return inst.points * (15.0 * math.log2(inst.ns[axis]) + 9.0 + 20.0 / inst.dims)


def gpu_rate(inst, dtype, steps, warmup, pass_reps, tune=True, tune_cache=None, with_diagnostics=True):
    import numpy as np
    import torch
    from paper_2209_08437_amd import autotune, sfac
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u0 = torch.tensor(inst.u0, dtype=tdt, device="cuda")
    u = u0.clone()
    sched = {}
    if tune:
        if tune_cache == "none":
            best = autotune.tune(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype, use_cache=False)
        elif tune_cache:
            best = autotune.tune(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype, path=tune_cache)
        else:
            best = autotune.tune(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype,
                                 path=autotune.PACKAGED, save=False)
        sched = {k: best[k] for k in ("method", "elems_log2", "lines_per_block", "kernel")}
        log(f"[bench] {dtype}: tuned schedule {sched} (pass us {[round(x * 1e3, 1) for x in best['ms']]})")
    # plan creation: host tables in long double, one device allocation, upload (first step
    # captures the step graphs and is timed apart from it)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plan = sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype, **sched)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - tp) * 1e3
    methods = [plan.method(a + 1) for a in range(inst.dims)]
    log(f"[bench] {dtype}: methods per axis {methods}; warmup {warmup} steps")
    tp = time.perf_counter()
    plan.step(u, warmup)
    torch.cuda.synchronize()
    warm_ms = (time.perf_counter() - tp) * 1e3
    log(f"[bench] {dtype}: plan created in {plan_ms:.2f} ms; {warmup} warm-up steps (graph capture included) "
        f"{warm_ms:.2f} ms")
    # the step graphs the timed call replays (a 32-step chunk and one graph per set bit of the
    # rest) are captured before it by untimed runs of the same step count from the same state
    # buffer (graphs belong to a state address), which is then reset; the runs go on for a
    # quarter of a second, so that the device's clocks have ramped up under load when the timed
    # region starts (after idling, a short timed call otherwise runs up to 20% slow)
    t_prime = time.perf_counter() + 0.25
    for _ in range(1000):
        u.copy_(u0)
        plan.step(u, steps)
        torch.cuda.synchronize()
        if time.perf_counter() > t_prime:
            break
    u.copy_(u0)
    plan.reset_flags()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    plan.step(u, steps)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    gpu_ms = ev0.elapsed_time(ev1)
    flags, vmax = plan.flags()
    log(f"[bench] {dtype}: {steps} steps in {wall * 1e3:.2f} ms wall ({gpu_ms:.2f} ms events), "
        f"max|u| {vmax:.6f}, flags {flags}")
    # the same timed region repeated (state reset from u0 outside each), for the spread
    reps = []
    for _ in range(5):
        u.copy_(u0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.step(u, steps)
        e1.record()
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / steps)
    # per-pass kernel durations: each axis' pass launched pass_reps times back to back from a
    # captured graph, HIP events around the replay on the plan's stream (on a scratch copy)
    uu = u0.clone()
    pass_ms = plan.time_passes(uu, pass_reps)
    # the launches that cover axis 1 and axis d twice (a step's last pass and the next one's
    # first, as the steps run them at every step boundary)
    fused_ms = plan.time_fused(uu, pass_reps)
    del uu
    torch.cuda.synchronize()
    state = u.double().cpu().numpy()
    diag = diagnostics(plan, u0, u, min(steps, 200)) if with_diagnostics else None
    result = {
        "wall_s": wall, "gpu_ms": gpu_ms, "flags": flags, "max_abs": vmax,
        "pass_ms": pass_ms, "fused_ms": fused_ms, "methods": methods, "state": state, "schedule": sched,
        "plan_create_ms": plan_ms, "warmup_ms": warm_ms, "diagnostics": diag, "repeat_ms_per_step": reps,
    }
    plan.close()
    return result


def diagnostics(plan, u0, u, k):
    """Outside the timed region: the discrete energy (Sec. 5, Example 5) of the initial and final
    states and the time of one evaluation, and what recording max|u| after every step (Example 4)
    adds to a step, from k graph-replayed steps with and without the record."""
    import torch
    from paper_2209_08437_amd import sfac
    try:
        e_start = plan.energy(u0)                 # the first call builds the energy tables
        t = time.perf_counter()
        e_end = plan.energy(u)
        energy_ms = (time.perf_counter() - t) * 1e3

        def timed(trace):
            plan.trace(k if trace else 0)
            w = u0.clone()
            plan.step(w, k)                       # captures the step graphs
            torch.cuda.synchronize()
            plan.trace(k if trace else 0)         # restart the record
            w.copy_(u0)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            plan.step(w, k)
            ev[1].record()
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]) / k, (plan.read_trace() if trace else None)

        plain_ms, _ = timed(False)
        trace_ms, (rec, n) = timed(True)
        plan.trace(0)
        return {"energy_start": e_start, "energy_end": e_end, "energy_call_ms": round(energy_ms, 3),
                "trace_steps": n, "trace_max_abs": float(rec.max()) if len(rec) else None,
                "trace_overhead_us_per_step": round((trace_ms - plain_ms) * 1e3, 2)}
    except sfac.SfacError as err:
        return {"unavailable": str(err)}


def step_launches(dims, fused_ms):
    """The launches of two consecutive steps in steady state, as (axis 0-based, passes per launch,
    launches per two steps): the step boundaries fuse the last pass of a step with the first of
    the next (axis d after a step in the order 1..d, axis 1 after one in the order d..1); an axis
    whose kernel does not fuse (fused time 0) runs its two passes as two launches."""
    if dims == 1:
        return [(0, 2, 1)] if fused_ms[0] > 0 else [(0, 1, 2)]
    out = []
    for a in range(dims):
        end = 0 if a == 0 else (1 if a == dims - 1 else None)
        if end is not None and fused_ms[end] > 0:
            out.append((a, 2, 1))
        else:
            out.append((a, 1, 2))
    return out


def pass_roofline(inst, dtype, r, workload_name):
    """Roofline of the dominant launch of the step: of the launches two steps make in steady
    state (step_launches), the one that takes the largest share of their time. A launch reads
    and writes the state once; a fused launch does two passes' flops on those bytes. The bound
    is whichever of its algorithmic bytes and algorithmic flops takes longer at the published
    peaks; `achieved` is that quantity per launch over the mean launch duration. The other
    figure is reported beside it, and `traffic` is the counter-measured HBM bytes per launch when
    the committed record matches."""
    from paper_2209_08437_amd import profiling
    esize = 8 if dtype == "f64" else 4
    pass_ms = r["pass_ms"]
    fused_ms = r["fused_ms"]
    mix = step_launches(inst.dims, fused_ms)

    def launch_ms(a, passes):
        return (fused_ms[0 if a == 0 else 1] if passes == 2 else pass_ms[a])

    a, passes, _ = max(mix, key=lambda m: m[2] * launch_ms(m[0], m[1]))
    ms = launch_ms(a, passes)
    step_ms = sum(m[2] * launch_ms(m[0], m[1]) for m in mix) / 2.0
    fl = passes * pass_flops(inst, a)
    byt = 2 * inst.points * esize
    sec = ms * 1e-3
    peak_tf = VALU_PEAK_TFLOPS[dtype]
    tf = fl / sec / 1e12
    gbps = byt / sec / 1e9
    hbm = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbps / HBM_PEAK_GBS, 4)}
    alu = {"bound": "alu", "achieved": round(tf, 3), "peak": peak_tf, "unit": "TFLOP/s",
           "frac": round(tf / peak_tf, 4)}
    hbm_bound = byt / (HBM_PEAK_GBS * 1e9) >= fl / (peak_tf * 1e12)
    out = dict(hbm if hbm_bound else alu)
    rec = profiling.load_traffic(TRAFFIC_RECORD, workload_name, dtype, r["schedule"] or None)
    traffic = None
    if rec:
        hit = [x for x in rec["per_axis"] if x["axis"] == a + 1 and x.get("twice", False) == (passes == 2)]
        traffic = hit[0]["bytes"] if hit else None
    meth, length = r["methods"][a]
    out.update({
        "traffic": traffic,
        "kernel": f"{meth} axis pass ({'double' if esize == 8 else 'float'}, transform length {length}), "
                  f"axis {a + 1}" + (", two passes per launch (a step boundary between)" if passes == 2 else ""),
        "algorithmic_bytes_per_launch": byt, "flops_per_launch": round(fl),
        "mean_launch_ms": round(ms, 5), "pass_ms": [round(x, 5) for x in pass_ms],
        "fused_ms": [round(x, 5) for x in fused_ms],
        "launches_per_two_steps": [{"axis": m[0] + 1, "passes": m[1], "launches": m[2]} for m in mix],
        "step_ms_from_launches": round(step_ms, 5),
        "timing": "HIP events around a graph of back-to-back launches of each launch kind on the plan's stream",
        "alu" if hbm_bound else "hbm": alu if hbm_bound else hbm,
        "traffic_record": (f"profiles/traffic.json ({rec['profile']})" if rec else
                           "none for the current kernel sources"),
    })
    return out


def one_level_exact(inst, steps, two_level_state, two_level_ms, workload_name, pass_reps):
    """The one-level scheme (eq. (strang)) with e^{tau B} per axis as a dense FP64 product on the
    GPU (SFAC_METHOD_EXACT) over the bench's steps: plan creation (host eigendecomposition),
    step time, the products' flop rate (2 N flops per point and axis), the max-norm distance
    of its final state from the two-level scheme's, and the roofline of the dense product with
    the longest mean duration (HIP events around each product on the plan's stream, against
    the FP64 matrix-core peak; traffic from the committed counter record when it matches)."""
    import numpy as np
    import torch
    from paper_2209_08437_amd import sfac
    if max(inst.ns) > 1024:
        return {"unavailable": "N above 1024"}
    u0 = torch.tensor(inst.u0, dtype=torch.float64, device="cuda")
    u = u0.clone()
    t = time.perf_counter()
    plan = sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, "f64", method="exact")
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t) * 1e3
    try:
        plan.step(u, 5)
        u.copy_(u0)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        plan.step(u, steps)
        ev[1].record()
        torch.cuda.synchronize()
        step_ms = ev[0].elapsed_time(ev[1]) / steps
        flags, vmax = plan.flags()
        prod_ms = plan.time_passes(u0.clone(), pass_reps)
    finally:
        plan.close()
    flops = sum(2.0 * n * inst.points for n in inst.ns)
    a = max(range(inst.dims), key=lambda i: prod_ms[i])
    fl = 2.0 * inst.ns[a] * inst.points
    tf = fl / (prod_ms[a] * 1e-3) / 1e12
    from paper_2209_08437_amd import profiling
    rec = profiling.load_traffic(TRAFFIC_RECORD, workload_name, "exact")
    roof = {"bound": "mfma", "achieved": round(tf, 3), "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / MFMA_F64_PEAK_TFLOPS, 4),
            "traffic": rec["per_axis"][a]["bytes"] if rec and len(rec["per_axis"]) > a else None,
            "kernel": f"exact_gemm (FP64 matrix cores), axis {a + 1}", "flops_per_launch": fl,
            "algorithmic_bytes_per_launch": 8 * (2 * inst.points + inst.ns[a] ** 2),
            "product_ms": [round(x, 5) for x in prod_ms]}
    diff = float(np.abs(u.cpu().numpy() - two_level_state).max())
    log(f"[bench] one-level exact: {step_ms * 1e3:.1f} us/step ({flops / step_ms / 1e9:.1f} TFLOP/s products), "
        f"plan {create_ms:.0f} ms, max|diff| to two-level {diff:.3e}")
    return {"ms_per_step": round(step_ms, 5), "plan_create_ms": round(create_ms, 1),
            "product_flops_per_step": flops, "product_TFLOPs": round(flops / step_ms / 1e9, 3),
            "two_level_speedup": round(step_ms / two_level_ms, 2),
            "max_abs_diff_vs_two_level": diff, "max_abs": vmax, "flags": flags, "roofline": roof}


def batched_run(args):
    """All instances of the batched workload stepped together (sfac_batch_step), against the
    same instances stepped one after another with plain FP64 plans."""
    import numpy as np
    import torch
    from paper_2209_08437_amd import autotune, sfac, workloads as W
    insts = W.batched_2d(count=args.batch_count, steps=args.steps or 500)
    steps = insts[0].steps
    pts = sum(i.points for i in insts)
    res = {}
    finals = {}
    for dt in ("f32", "f64"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        sched = None
        if not args.no_tune:
            path = None if args.tune_cache in (None, "none") else args.tune_cache
            sched = autotune.schedules(insts, dt, path=path)
            log(f"[bench] batched {dt}: schedules for {len(set(tuple(i.ns) for i in insts))} shapes")
        states = [torch.tensor(i.u0, dtype=tdt, device="cuda") for i in insts]
        b = sfac.Batch(insts, dt, schedules=sched)
        b.step(states, min(args.warmup, steps))
        # the step graphs of the timed call (they belong to the states' addresses) are captured by
        # an untimed run of the same steps on the same buffers, which are then reset
        for u, i in zip(states, insts):
            u.copy_(torch.tensor(i.u0, dtype=tdt, device="cuda"))
        b.step(states, steps)
        torch.cuda.synchronize()
        for u, i in zip(states, insts):
            u.copy_(torch.tensor(i.u0, dtype=tdt, device="cuda"))
        b.reset_flags()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(states, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        vmax = max(b.flags(k)[1] for k in range(len(insts)))
        flags = 0
        for k in range(len(insts)):
            flags |= b.flags(k)[0]
        res[dt] = {"value": pts * steps / wall, "wall_s": wall, "max_abs": vmax, "flags": flags}
        finals[dt] = [u.double().cpu().numpy() for u in states]
        log(f"[bench] batched {len(insts)} instances {dt}: {steps} steps in {wall * 1e3:.1f} ms")
        b.close()
    # plain FP64 path: one plan per instance, stepped one after another
    plans = [sfac.Plan(i.ns, i.alphas, i.eps, i.tau, i.hs, "f64") for i in insts]
    states = [torch.tensor(i.u0, dtype=torch.float64, device="cuda") for i in insts]
    for p, u in zip(plans, states):
        p.step(u, min(args.warmup, steps))
    for p, u, i in zip(plans, states, insts):     # graphs of the timed call, captured untimed
        u.copy_(torch.tensor(i.u0, dtype=torch.float64, device="cuda"))
        p.step(u, steps)
        u.copy_(torch.tensor(i.u0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, u in zip(plans, states):
        p.step(u, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res["f64_sequential"] = {"value": pts * steps / wall, "wall_s": wall}
    for p in plans:
        p.close()
    sizes = sorted(set(i.ns[0] for i in insts))
    return {
        "metric": METRIC, "value": round(res["f32"]["value"], 1), "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(res["f32"]["wall_s"] * 1e3 / steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched grouped solve (shared launches per kernel variant): {len(insts)} independent 2D instances, n from "
                               f"{sizes}, alpha_l ~ U(1.1,1.9), eps ~ U(0.02,0.2), tau ~ U(1e-3,1e-2), {steps} steps",
                   "points": pts},
        "batched_f64": round(res["f64"]["value"], 1),
        "plain_f64_sequential": round(res["f64_sequential"]["value"], 1),
        "speedup_f32_batched_vs_plain_f64": round(res["f32"]["value"] / res["f64_sequential"]["value"], 3),
        "max_abs": max(res["f32"]["max_abs"], res["f64"]["max_abs"]),
        "flags": res["f32"]["flags"] | res["f64"]["flags"],
        "f32_rel_err_vs_f64_gpu_max": float(max(np.abs(a - r).max() / np.abs(r).max()
                                                for a, r in zip(finals["f32"], finals["f64"]))),
        "schedules": "autotuned (MI355X table, missing shapes tuned on the device)" if not args.no_tune
                     else "automatic",
    }


class _StreamExecutor:
    """The device executor for long served streams: a request's initial state is drawn from its
    seed when it is admitted (not held for the whole stream) and results are not read back
    (flags and max|u| only), so host memory stays bounded."""

    def __init__(self):
        from paper_2209_08437_amd import serve
        self.ex = serve.GpuExecutor(keep_states=False)
        self.on_device = True

    def bytes_needed(self, inst, dtype):
        return self.ex.bytes_needed(inst, dtype)

    def admit(self, inst, dtype):
        from paper_2209_08437_amd import workloads as W
        inst.u0 = W.uniform_field(inst.shape, -0.9, 0.9, inst.seed)
        try:
            return self.ex.admit(inst, dtype)
        finally:
            inst.u0 = None

    def step(self, handles, nsteps):
        self.ex.step(handles, nsteps)

    def retire(self, handle):
        return self.ex.retire(handle)

    def close(self):
        self.ex.close()


def _serve(reqs, args):
    from paper_2209_08437_amd import serve
    ex = _StreamExecutor()
    def progress(done, total):
        if done % 100 == 0 or done == total:
            log(f"[bench]   {done}/{total} requests finished")
    srv = serve.Server(ex, budget_bytes=int(args.serve_budget_gb * 2 ** 30), tick_steps=args.tick_steps,
                       progress=progress)
    tickets, summ = srv.run(reqs)
    ex.close()
    return tickets, summ, srv


def sustainable_rate(args):
    """Highest arrival rate the server keeps up with, by bisection on the logarithm of the rate:
    a stream of args.serve_probe_count requests of the served workload's mix is served at each
    trial rate; the server keeps up when it serves at least 90% of the offered grid-point-steps
    per second (the rest is the drain of the last requests). Each trial runs in a process of its
    own (one server, one executor per process), started before this process touches the GPU."""
    import math
    import subprocess
    lo, hi = args.serve_rate_lo, args.serve_rate
    trials = []
    for k in range(args.serve_bisect):
        r = math.sqrt(lo * hi)
        cmd = [sys.executable, os.path.abspath(__file__), "--workload", "served", "--serve-count",
               str(args.serve_probe_count), "--serve-rate", repr(r), "--serve-seed", str(50 + k), "--serve-bisect",
               "0", "--serve-budget-gb", repr(args.serve_budget_gb), "--tick-steps", str(args.tick_steps)]
        res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
        if res.returncode != 0:
            log(res.stderr[-2000:])
            raise SystemExit(f"served probe at {r:.2f} req/s failed with status {res.returncode}")
        summ = json.loads(res.stdout.strip().splitlines()[-1])
        ratio = summ["served_fraction_of_offered"]
        ok = ratio >= 0.9
        trials.append({"rate": round(r, 2), "served_over_offered": round(ratio, 3), "keeps_up": ok,
                       "p50_latency_s": summ["p50_latency_s"], "p99_latency_s": summ["p99_latency_s"],
                       "makespan_s": round(summ["summary"]["makespan_s"], 2)})
        log(f"[bench] served probe at {r:.1f} req/s: served/offered {ratio:.3f}, p99 {summ['p99_latency_s']:.2f} s")
        if ok:
            lo = r
        else:
            hi = r
    return {"sustainable_rate_req_per_s": round(lo, 2), "first_rate_not_sustained": round(hi, 2),
            "probe_requests": args.serve_probe_count, "criterion": "served >= 0.9 x offered grid-point-steps/s",
            "trials": trials}


def served_run(args):
    """The served workload: the seeded Poisson stream (mean args.serve_rate req/s) of
    args.serve_count requests through the continuous-batching server, then the highest
    sustainable arrival rate by bisection."""
    from paper_2209_08437_amd import workloads as W
    sustainable = sustainable_rate(args) if args.serve_bisect > 0 else None
    reqs = W.served_stream(count=args.serve_count, rate=args.serve_rate, seed=args.serve_seed, materialize=False)
    n3 = sum(1 for r in reqs if r.inst.dims == 3)
    nf = sum(1 for r in reqs if r.dtype == "f32")
    log(f"[bench] serving {len(reqs)} requests ({n3} 3D, {nf} FP32) arriving over {reqs[-1].arrival:.1f} s")
    tickets, summ, srv = _serve(reqs, args)
    bad = sum(1 for t in tickets if t.flags)
    vmax = max((t.max_abs for t in tickets if t.finished is not None), default=0.0)
    log(f"[bench] served {summ['completed']}/{len(reqs)} requests in {summ['makespan_s']:.2f} s, "
        f"p50 {summ['p50_latency_s']:.3f} s p99 {summ['p99_latency_s']:.3f} s")
    out = {
        "metric": METRIC, "value": round(summ["throughput_gps"], 1), "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"served solve stream: {len(reqs)} requests of the seeded Poisson stream "
                               f"(mean {args.serve_rate:g} req/s; {n3} 3D n in [31,255], {len(reqs) - n3} 2D n in "
                               f"[63,1023]; steps in [50,2000]; {nf} FP32, {len(reqs) - nf} FP64)",
                   "budget_bytes": srv.budget, "tick_steps": srv.tick_steps},
        "p50_latency_s": summ["p50_latency_s"], "p99_latency_s": summ["p99_latency_s"],
        "offered_gps": summ["offered_gps"], "served_fraction_of_offered": summ["throughput_gps"] / summ["offered_gps"],
        "requests_flagged": bad, "max_abs": vmax,
        "summary": {k: v for k, v in summ.items() if k not in ("p50_latency_s", "p99_latency_s")},
    }
    if sustainable is not None:
        out["sustainable"] = sustainable
    return out


def cpu_leg(inst, seconds, checks=()):
    """The CPU oracle as it stands: (1) timed on a bounded sample of the workload (table set-up,
    the dense per-axis exponentials, timed apart; then as many whole steps as fit the budget, on
    all host threads and on one); (2) the max-norm error of GPU results against it: each check is
    (name, instance, {dtype: final GPU state}) and the oracle runs the instance's full step count."""
    import numpy as np
    from oracle import sfac_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    ops = O.axis_operators(inst.ns, inst.alphas, inst.eps, inst.hs, inst.tau)
    setup = time.perf_counter() - t0
    u = np.array(inst.u0, dtype=np.float64)
    t0 = time.perf_counter()
    u = O.two_level_step(u, ops, inst.tau)
    one = time.perf_counter() - t0
    k = max(1, min(inst.steps - 1, int(seconds / max(one, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(k):
        u = O.two_level_step(u, ops, inst.tau)
    dt = time.perf_counter() - t0
    pts = inst.points
    out = {
        "value": pts * k / dt, "unit": "grid-point-steps/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{k} steps of the same {'x'.join(map(str, inst.ns))} workload after 1 untimed step "
                  f"(dense per-axis exponentials, numpy/OpenBLAS FP64); table set-up {setup:.2f} s not included",
    }
    # the same oracle on one thread, over a fifth of the budget
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            u = O.two_level_step(u, ops, inst.tau)
            one1 = time.perf_counter() - t0
            k1 = max(1, min(inst.steps - 1, int(seconds / 5 / max(one1, 1e-6))))
            t0 = time.perf_counter()
            for _ in range(k1):
                u = O.two_level_step(u, ops, inst.tau)
            dt1 = time.perf_counter() - t0
        out["single_thread"] = {"value": pts * k1 / dt1, "unit": "grid-point-steps/s", "cores": 1,
                                "sample": f"{k1} steps after 1 untimed step"}
    except ImportError:
        pass
    acc = {}
    for name, cinst, states in checks:
        t0 = time.perf_counter()
        ref = O.two_level_solve(cinst.u0, cinst.ns, cinst.alphas, cinst.eps, cinst.hs, cinst.tau, cinst.steps)
        scale = float(np.abs(ref).max())
        acc[name] = {"steps": cinst.steps, "grid": list(cinst.ns), "oracle_s": round(time.perf_counter() - t0, 2),
                     "oracle_max_abs": scale}
        for dt_, st in states.items():
            acc[name][f"{dt_}_rel_err_vs_oracle"] = float(np.abs(st - ref).max() / scale)
        log(f"[bench] oracle check {name}: " + ", ".join(f"{k2} {v:.3e}" for k2, v in acc[name].items()
                                                          if k2.endswith("oracle")))
    return out, acc


def sub_workload(name, steps, args):
    """FP64 and FP32 runs of another single-instance workload, for a sub-object of the line."""
    inst, desc = workload(name)
    steps = steps if steps is not None else inst.steps
    r64 = gpu_rate(inst, "f64", steps, args.warmup, args.pass_reps, tune=not args.no_tune,
                   tune_cache=args.tune_cache, with_diagnostics=False)
    r32 = gpu_rate(inst, "f32", steps, args.warmup, args.pass_reps, tune=not args.no_tune,
                   tune_cache=args.tune_cache, with_diagnostics=False)
    out = {"workload": desc, "steps": steps}
    for dt_, r in (("f64", r64), ("f32", r32)):
        out[dt_] = {"value": round(inst.points * steps / r["wall_s"], 1), "unit": "grid-point-steps/s",
                    "ms_per_step": round(r["wall_s"] * 1e3 / steps, 5), "max_abs": r["max_abs"], "flags": r["flags"],
                    "schedule": r["schedule"], "roofline": pass_roofline(inst, dt_, r, name)}
    return inst, out, {"f64": r64["state"], "f32": r32["state"]}


def subsample_states(big, args):
    """GPU FP64 and FP32 results of the 63^3 companion of the 3D instance (all its steps)."""
    import torch
    from paper_2209_08437_amd import sfac, workloads as W
    inst = W.subsample_3d_63(big)
    states = {}
    for dt_ in ("f64", "f32"):
        tdt = torch.float64 if dt_ == "f64" else torch.float32
        u = torch.tensor(inst.u0, dtype=tdt, device="cuda")
        with sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dt_) as p:
            p.step(u, inst.steps)
            flags, vmax = p.flags()
        states[dt_] = u.double().cpu().numpy()
        log(f"[bench] 63^3 subsample {dt_}: {inst.steps} steps, max|u| {vmax:.6f}, flags {flags}")
    return inst, states


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="large_3d_255")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="skip the 1023^2 and batched sub-objects of the 3D line")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched sub-object of the 3D line")
    ap.add_argument("--no-oracle-checks", action="store_true",
                    help="skip the oracle runs behind the error figures (the 1023^2 one takes about a minute)")
    ap.add_argument("--no-exact", action="store_true", help="skip the one-level exact-exponential comparison")
    ap.add_argument("--pass-reps", type=int, default=20)
    ap.add_argument("--no-tune", action="store_true", help="default schedules instead of autotuned ones")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: tune only shapes missing from it and add them (default: "
                         "the schedules measured on an MI355X that ship with the package, read only; "
                         "'none': tune every axis afresh)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrival rate of the served stream (req/s)")
    ap.add_argument("--serve-bisect", type=int, default=6,
                    help="bisection steps for the highest sustainable arrival rate (0: skip)")
    ap.add_argument("--serve-rate-lo", type=float, default=2.0)
    ap.add_argument("--serve-probe-count", type=int, default=150)
    ap.add_argument("--serve-seed", type=int, default=5, help="seed of the served stream")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--tick-steps", type=int, default=50)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 512 MiB buffer 20 times (a plain copy kernel of known traffic, "
                         "larger than every cache level, to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the slab decomposition over several GPUs is designed, not implemented)", flush=True)
        sys.exit(2)
    from paper_2209_08437_amd import sfac, build_lib
    if not os.path.exists(sfac.LIB_PATH):
        build_lib.build()
    if args.workload == "served":
        # its rate probes run as child processes, started before this process touches the GPU
        print(json.dumps(served_run(args)), flush=True)
        return
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.workload == "batched_2d":
        print(json.dumps(batched_run(args)), flush=True)
        return
    inst, desc = workload(args.workload)
    steps = args.steps if args.steps is not None else inst.steps
    if args.copy_probe:
        a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_copy": a.numel() * a.element_size(), "copies": 20}))
        return
    esize = 8 if args.dtype == "f64" else 4
    pts = inst.points
    main_r = gpu_rate(inst, args.dtype, steps, args.warmup, args.pass_reps, tune=not args.no_tune,
                      tune_cache=args.tune_cache)
    value = pts * steps / main_r["wall_s"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(main_r["wall_s"] * 1e3 / steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc, "grid": list(inst.ns), "points": pts,
                   "methods": [m for m, _ in main_r["methods"]], "schedule": main_r["schedule"],
                   "effective_GBps": round(value * 2 * inst.dims * esize / 1e9, 2),
                   "plan_create_ms": round(main_r["plan_create_ms"], 3),
                   "warmup_ms": round(main_r["warmup_ms"], 3)},
        "roofline": pass_roofline(inst, args.dtype, main_r, args.workload),
    }
    out["roofline"]["step_ms_timed_region"] = round(main_r["gpu_ms"] / steps, 5)
    checks = []
    r32 = None
    if not args.no_fp32 and args.dtype == "f64":
        r32 = gpu_rate(inst, "f32", steps, args.warmup, args.pass_reps, tune=not args.no_tune,
                       tune_cache=args.tune_cache, with_diagnostics=False)
        import numpy as np
        ref = main_r["state"]
        out["fp32"] = {"value": round(pts * steps / r32["wall_s"], 1), "unit": "grid-point-steps/s",
                       "ms_per_step": round(r32["wall_s"] * 1e3 / steps, 5),
                       "speedup_vs_fp64": round(main_r["wall_s"] / r32["wall_s"], 3),
                       "rel_err_vs_fp64_gpu": float(np.abs(r32["state"] - ref).max() / np.abs(ref).max()),
                       "max_abs": r32["max_abs"], "flags": r32["flags"], "schedule": r32["schedule"],
                       "plan_create_ms": round(r32["plan_create_ms"], 3),
                       "roofline": pass_roofline(inst, "f32", r32, args.workload)}
    import statistics
    rp = main_r["repeat_ms_per_step"]
    out["repeats"] = {"n": len(rp), "median_ms_per_step": round(statistics.median(rp), 5),
                      "min_ms_per_step": round(min(rp), 5), "max_ms_per_step": round(max(rp), 5),
                      "note": "the timed region repeated after it (HIP events, state reset outside); value is the first"}
    out["max_abs"] = main_r["max_abs"]
    out["flags"] = main_r["flags"]
    out["diagnostics"] = main_r["diagnostics"]
    if args.workload == "large_3d_255" and steps == inst.steps and not (args.no_cpu or args.no_oracle_checks):
        # the 63^3 companion run whose error against the oracle the CPU leg reports
        sub_inst, sstates = subsample_states(inst, args)
        checks.append(("subsample_3d_63", sub_inst, sstates))
    if args.workload == "large_3d_255" and not args.no_sub:
        c2_inst, out["large_2d_1023"], c2_states = sub_workload("large_2d_1023", None, args)
        checks.append(("large_2d_1023", c2_inst, c2_states))
    if args.workload == "large_3d_255" and not args.no_sub and not args.no_batched:
        b = batched_run(args)
        out["batched_2d"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "steps", "dtype", "batched_f64",
                                               "plain_f64_sequential", "speedup_f32_batched_vs_plain_f64",
                                               "f32_rel_err_vs_f64_gpu_max", "max_abs", "flags", "schedules")}
        out["batched_2d"]["workload"] = b["config"]["workload"]
    if args.dtype == "f64" and not args.no_exact:
        out["one_level_exact"] = one_level_exact(inst, steps, main_r["state"], main_r["wall_s"] * 1e3 / steps,
                                                 args.workload, args.pass_reps)
    if not args.no_cpu:
        log(f"[bench] timing the CPU oracle for about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"], acc = cpu_leg(inst, args.cpu_seconds, [] if args.no_oracle_checks else checks)
        if acc:
            out["accuracy_vs_oracle"] = acc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
