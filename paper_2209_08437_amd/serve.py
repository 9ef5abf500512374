"""Continuous-batching solve server on one GPU.

Requests (an instance of the fractional Allen-Cahn problem, a step count and an arithmetic
type) arrive over time. The server admits queued requests first-come first-served while their
device memory (state + tables) fits a budget, keeps every admitted state on the device, and in
each tick advances all admitted requests together by up to `tick_steps` steps with one grouped
step (sfac_group_step: one launch per pass and kernel variant for all of them, FP64 and FP32
mixed). Finished requests are read back and retired at the tick boundary, which frees memory
for queued ones; requests that arrive while others run join at the next tick. A request larger
than the whole budget is rejected.

Splitting a solve into ticks and sharing launches with other requests does not change its
result: every state sees exactly the kernels and order of a lone sfac_step call.

The executor does the device work; `GpuExecutor` uses the library. Anything with the same four
methods can stand in (the tests use a CPU stand-in to check the scheduling).
"""
from collections import deque
from dataclasses import dataclass, field
import math
import time

import numpy as np


@dataclass
class Ticket:
    """Life of one request: stream times in seconds from the start of the run."""
    rid: int
    arrival: float
    points: int
    steps: int
    dtype: str
    admitted: float = None
    finished: float = None
    rejected: bool = False
    result: object = field(default=None, repr=False)
    flags: int = 0
    max_abs: float = 0.0

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class GpuExecutor:
    """Device side of the server: one plan and one device-resident state per admitted request,
    one group for the grouped steps, all on one stream. Plans take the autotuned schedule of
    their shape when the schedule table (`schedule_table`: a cache file path; default the
    packaged MI355X table; False for automatic schedules only) holds it; nothing is tuned
    while serving."""

    def __init__(self, stream=None, schedule_table=None):
        import torch
        from . import autotune, sfac
        self.torch = torch
        self.sfac = sfac
        self.autotune = autotune
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.group = sfac.Group(self.stream)
        self.table = {} if schedule_table is False else autotune.load_table(schedule_table)

    def bytes_needed(self, inst, dtype):
        esize = 8 if dtype == "f64" else 4
        tables = 0
        for n in inst.ns:
            m = 2
            while m < 2 * n - 1:
                m *= 2
            tables += 4 * m * 2 * esize + 1024        # twiddles, two spectra, alignment
        return int(np.prod(inst.ns)) * esize + tables + 256

    def admit(self, inst, dtype):
        torch = self.torch
        tdt = torch.float64 if dtype == "f64" else torch.float32
        sched = self.autotune.lookup(inst.ns, dtype, table=self.table) if self.table else None
        with torch.cuda.stream(self.stream):
            plan = self.sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype,
                                  stream=self.stream, use_graph=False, **(sched or {}))
            u = torch.as_tensor(np.asarray(inst.u0), dtype=tdt).to("cuda", non_blocking=False)
        return (plan, u)

    def step(self, handles, nsteps):
        plans = [h[0] for h in handles]
        states = [h[1] for h in handles]
        self.group.step(plans, states, nsteps)
        self.stream.synchronize()

    def retire(self, handle):
        plan, u = handle
        flags, vmax = plan.flags()
        out = u.double().cpu().numpy()
        plan.close()
        return out, flags, vmax


class Server:
    """Admission by device-memory budget, FIFO, continuous batching in ticks of `tick_steps`."""

    def __init__(self, executor, budget_bytes, tick_steps=50, max_active=256,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.tick_steps = int(tick_steps)
        self.max_active = int(max_active)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests):
        """Serve `requests` (objects with rid, arrival, inst, dtype; arrival in seconds from the
        start) in real time. Returns (tickets in request order, summary dict)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        tickets = {r.rid: Ticket(r.rid, r.arrival, int(np.prod(r.inst.ns)), int(r.inst.steps), r.dtype)
                   for r in reqs}
        queue = deque()
        active = []          # [ticket, handle, remaining steps, bytes]
        used = 0
        nxt = 0
        ticks = 0
        peak_active = 0
        peak_bytes = 0
        t0 = self.clock()
        busy = 0.0
        admit_s = []         # per admitted request: plan tables, device upload of state and tables
        while nxt < len(reqs) or queue or active:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            # admission: first come first served while the head fits the budget
            while queue and len(active) < self.max_active:
                r = queue[0]
                need = self.ex.bytes_needed(r.inst, r.dtype)
                tk = tickets[r.rid]
                if need > self.budget:
                    queue.popleft()
                    tk.rejected = True
                    continue
                if used + need > self.budget:
                    break
                queue.popleft()
                tk.admitted = self.clock() - t0
                if tk.steps == 0:
                    tk.finished = tk.admitted
                    tk.result = np.array(r.inst.u0, dtype=np.float64, copy=True)
                    continue
                ta = self.clock()
                handle = self.ex.admit(r.inst, r.dtype)
                admit_s.append(self.clock() - ta)
                active.append([tk, handle, tk.steps, need])
                used += need
            peak_active = max(peak_active, len(active))
            peak_bytes = max(peak_bytes, used)
            if active:
                k = [min(self.tick_steps, a[2]) for a in active]
                ts = self.clock()
                self.ex.step([a[1] for a in active], k)
                busy += self.clock() - ts
                ticks += 1
                still = []
                for a, kk in zip(active, k):
                    a[2] -= kk
                    if a[2] == 0:
                        tk = a[0]
                        tk.result, tk.flags, tk.max_abs = self.ex.retire(a[1])
                        tk.finished = self.clock() - t0
                        used -= a[3]
                    else:
                        still.append(a)
                active = still
            elif nxt < len(reqs) and not queue:
                wait = reqs[nxt].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(wait)
        makespan = self.clock() - t0
        done = [t for t in tickets.values() if t.finished is not None]
        lat = np.array([t.latency for t in done]) if done else np.zeros(0)
        wait = np.array([t.admitted - t.arrival for t in done]) if done else np.zeros(0)
        adm = np.array(admit_s)
        work = sum(t.points * t.steps for t in done)
        span_arrivals = (reqs[-1].arrival - reqs[0].arrival) if len(reqs) > 1 else 0.0
        offered = sum(t.points * t.steps for t in tickets.values())
        summary = {
            "requests": len(reqs), "completed": len(done),
            "rejected": sum(t.rejected for t in tickets.values()),
            "makespan_s": makespan, "busy_s": busy, "ticks": ticks,
            "throughput_gps": work / makespan if makespan > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
            "offered_gps": offered / span_arrivals if span_arrivals > 0 else math.inf,
            "peak_active": peak_active, "peak_bytes": peak_bytes, "budget_bytes": self.budget,
            "p50_queue_wait_s": float(np.percentile(wait, 50)) if len(wait) else None,
            "admit_p50_ms": float(np.percentile(adm, 50)) * 1e3 if len(adm) else None,
            "admit_max_ms": float(adm.max()) * 1e3 if len(adm) else None,
            "admit_total_s": float(adm.sum()),
        }
        return [tickets[r.rid] for r in sorted(reqs, key=lambda r: r.rid)], summary
