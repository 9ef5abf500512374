"""Continuous-batching solve server on one GPU.

Requests (an instance of the fractional Allen-Cahn problem, a step count and an arithmetic
type) arrive over time. The server admits queued requests first-come first-served while their
device memory (state + tables) fits a budget, keeps every admitted state on the device, and in
each tick advances all admitted requests together by up to `tick_steps` steps with one grouped
step (sfac_group_step: the launches of all of them shared per kernel variant, FP64 and FP32
mixed). Finished requests are read back and retired at the tick boundary, which frees memory
for queued ones; requests that arrive while others run join at the next tick. A request larger
than the whole budget is rejected.

Splitting a solve into ticks and sharing launches with other requests does not change its
result: every state sees exactly the kernels and order of a lone sfac_step call.

The executor does the device work; `GpuExecutor` uses the library. Anything with the same four
methods can stand in (the tests use a CPU stand-in to check the scheduling).

Two front ends share that policy: `Server.run` replays a list of timed requests (the benchmark's
arrival stream), and `Service` is the online form: `submit` from any thread returns a future,
and one worker thread owns the executor and runs the ticks.
"""
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field
import math
import queue
import threading
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


def initial_flags(u0):
    """(flags, max|u|) of a state no step has touched: the same sticky bits the library sets
    (non-finite values; some |u| > 1)."""
    from .sfac import FLAG_ABOVE_ONE, FLAG_NONFINITE
    a = np.abs(np.asarray(u0, dtype=np.float64))
    if a.size == 0:
        return 0, 0.0
    flags = 0 if np.all(np.isfinite(a)) else FLAG_NONFINITE
    fin = a[np.isfinite(a)]
    vmax = float(fin.max()) if fin.size else 0.0
    if vmax > 1.0:
        flags |= FLAG_ABOVE_ONE
    return flags, vmax


class GpuExecutor:
    """Device side of the server: one plan and one device-resident state per admitted request,
    one group for the grouped steps, all on one stream. Plans take the autotuned schedule of
    their shape when the schedule table (`schedule_table`: a cache file path; default the
    packaged MI355X table; False for automatic schedules only) holds it; nothing is tuned
    while serving.

    A request's device memory is what the library reports for its plan
    (sfac_plan_device_bytes: tables, status, descriptors) plus its state; the plan is built when
    the server first asks for that figure and kept for the admission. `step` only queues the
    grouped launches (the host goes on admitting while the device runs); `retire` waits for the
    request's work and reads its state back.

    An admitted state is uploaded on a copy stream of its own, from the caller's (pageable)
    array: the host waits for that copy only, not for the grouped steps queued on the
    executor's stream, which is then ordered after the copy. No host staging buffer outlives the
    call (keeping a page-locked copy of every admitted state until it retired held gigabytes of
    locked host memory on long streams)."""

    on_device = True

    def __init__(self, stream=None, schedule_table=None, keep_states=True):
        import torch
        from . import autotune, sfac
        self.torch = torch
        self.sfac = sfac
        self.autotune = autotune
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.group = sfac.Group(self.stream)
        self.table = {} if schedule_table is False else autotune.load_table(schedule_table)
        self.keep_states = keep_states   # False: retire reports flags and max|u| only (no read-back)
        self.copy_stream = torch.cuda.Stream(device=self.stream.device)
        self._built = {}          # id(inst) -> (inst, dtype, plan), plans built for bytes_needed

    def _plan(self, inst, dtype):
        key = id(inst)
        hit = self._built.get(key)
        if hit is not None and hit[0] is inst and hit[1] == dtype:
            return hit[2]
        sched = self.autotune.lookup(inst.ns, dtype, table=self.table) if self.table else None
        plan = self.sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype,
                              stream=self.stream, use_graph=False, **(sched or {}))
        if len(self._built) >= 4:                 # requests that were measured but never admitted
            old = next(iter(self._built))
            self._built.pop(old)[2].close()
        self._built[key] = (inst, dtype, plan)
        return plan

    def bytes_needed(self, inst, dtype):
        esize = 8 if dtype == "f64" else 4
        return int(np.prod(inst.ns)) * esize + int(self._plan(inst, dtype).device_bytes)

    def admit(self, inst, dtype):
        torch = self.torch
        tdt = torch.float64 if dtype == "f64" else torch.float32
        plan = self._plan(inst, dtype)
        self._built.pop(id(inst), None)
        # a synchronous copy on the copy stream (runs beside the queued grouped steps); the
        # executor's stream waits for it before the request's first step
        with torch.cuda.stream(self.copy_stream):
            u = torch.as_tensor(np.asarray(inst.u0), dtype=tdt).to(self.stream.device, non_blocking=False)
        self.stream.wait_stream(self.copy_stream)
        u.record_stream(self.stream)
        return (plan, u)

    def step(self, handles, nsteps):
        plans = [h[0] for h in handles]
        states = [h[1] for h in handles]
        self.group.step(plans, states, nsteps)

    def retire(self, handle):
        plan, u = handle
        flags, vmax = plan.flags()                # waits for the plan's stream
        out = None
        if self.keep_states:
            with self.torch.cuda.stream(self.stream):
                out = u.double().cpu().numpy()
        plan.close()
        return out, flags, vmax

    def close(self):
        for _, _, plan in self._built.values():
            plan.close()
        self._built.clear()
        self.group.close()


class Server:
    """Admission by device-memory budget, FIFO, continuous batching in ticks of `tick_steps`."""

    def __init__(self, executor, budget_bytes, tick_steps=50, max_active=256,
                 clock=time.perf_counter, sleep=time.sleep, progress=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.tick_steps = int(tick_steps)
        self.max_active = int(max_active)
        self.clock = clock
        self.sleep = sleep
        self.progress = progress      # called with (finished requests, all requests) after each retire

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
        finished = 0
        admit_s = []         # per admitted request: plan tables, device upload of state and tables

        def admit(used):
            while queue and len(active) < self.max_active:
                r = queue[0]
                tk = tickets[r.rid]
                if tk.steps < 0:                  # not a solve: refused, the stream goes on
                    queue.popleft()
                    tk.rejected = True
                    continue
                need = self.ex.bytes_needed(r.inst, r.dtype) if tk.steps > 0 else 0
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
                    tk.flags, tk.max_abs = initial_flags(tk.result)
                    continue
                ta = self.clock()
                handle = self.ex.admit(r.inst, r.dtype)
                admit_s.append(self.clock() - ta)
                active.append([tk, handle, tk.steps, need])
                used += need
            return used

        while nxt < len(reqs) or queue or active:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            # admission: first come first served while the head fits the budget
            used = admit(used)
            peak_active = max(peak_active, len(active))
            peak_bytes = max(peak_bytes, used)
            if active:
                k = [min(self.tick_steps, a[2]) for a in active]
                ts = self.clock()
                self.ex.step([a[1] for a in active], k)
                busy += self.clock() - ts
                ticks += 1
                # while the device runs the tick: take arrivals and admit what still fits (they
                # join the next tick; the requests this tick finishes still hold their memory)
                now = self.clock() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    queue.append(reqs[nxt])
                    nxt += 1
                n_before = len(active)
                used = admit(used)
                peak_bytes = max(peak_bytes, used)
                joined = active[n_before:]
                active = active[:n_before]
                still = []
                for a, kk in zip(active, k):
                    a[2] -= kk
                    if a[2] == 0:
                        tk = a[0]
                        tr = self.clock()
                        tk.result, tk.flags, tk.max_abs = self.ex.retire(a[1])
                        busy += self.clock() - tr
                        tk.finished = self.clock() - t0
                        used -= a[3]
                        finished += 1
                        if self.progress is not None:
                            self.progress(finished, len(reqs))
                    else:
                        still.append(a)
                active = still + joined
                peak_active = max(peak_active, len(active))
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


class Service:
    """Online solve service: `submit(inst, dtype)` from any thread returns a
    concurrent.futures.Future of (final state as an FP64 array, sticky flags, max|u|).

    One worker thread creates the executor (`executor_factory()`, e.g. GpuExecutor) and does
    all device work. Between ticks it takes new submissions, admits queued requests first come
    first served while their device memory fits `budget_bytes`, and advances every admitted
    request by up to `tick_steps` steps in one grouped step; requests that finish are read back
    and their futures completed at the tick boundary. A request larger than the whole budget,
    or one whose admission or step fails, gets the exception in its future. A future cancelled
    before admission is dropped. `close()` stops taking submissions, lets the admitted and
    queued requests finish, and joins the worker.

    Not enabled for device executors (`on_device`, e.g. GpuExecutor): the one run of this
    service with the device executor on its worker thread ended in a host segmentation fault
    whose cause has not been found, so such an executor is refused with an error until it is.
    Device serving goes through `Server.run`, which does its device work on the calling thread."""

    _STOP = object()

    _DEVICE_REFUSED = ("the online service is not enabled for device executors: its one run with the "
                       "device executor on a worker thread ended in a host segmentation fault of unknown cause; "
                       "serve through Server.run")

    def __init__(self, executor_factory, budget_bytes, tick_steps=50, max_active=256):
        if isinstance(executor_factory, type) and getattr(executor_factory, "on_device", False):
            raise RuntimeError(self._DEVICE_REFUSED)
        self.budget = int(budget_bytes)
        self.tick_steps = int(tick_steps)
        self.max_active = int(max_active)
        self._inbox = queue.Queue()
        self._closed = False
        self._lock = threading.Lock()
        self._stats = {"submitted": 0, "completed": 0, "rejected": 0, "failed": 0, "ticks": 0,
                       "peak_active": 0, "peak_bytes": 0}
        self._ready = threading.Event()
        self._start_error = None
        self._thread = threading.Thread(target=self._loop, args=(executor_factory,), daemon=True)
        self._thread.start()
        self._ready.wait()
        if self._start_error is not None:
            raise self._start_error

    def submit(self, inst, dtype="f64"):
        if dtype not in ("f64", "f32"):
            raise ValueError(f"dtype {dtype!r}, expected 'f64' or 'f32'")
        if int(inst.steps) < 0:
            raise ValueError(f"steps = {inst.steps}, expected >= 0")
        fut = Future()
        with self._lock:
            if self._closed:
                raise RuntimeError("the service is closed")
            self._stats["submitted"] += 1
            self._inbox.put((inst, dtype, fut))
        return fut

    def stats(self):
        with self._lock:
            return dict(self._stats)

    def close(self):
        with self._lock:
            if self._closed:
                return
            self._closed = True
            self._inbox.put(self._STOP)
        self._thread.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _count(self, key, n=1):
        with self._lock:
            self._stats[key] += n

    def _loop(self, executor_factory):
        try:
            ex = executor_factory()
            if getattr(ex, "on_device", False):
                raise RuntimeError(self._DEVICE_REFUSED)
        except Exception as err:        # reported by the constructor
            self._start_error = err
            self._ready.set()
            return
        self._ready.set()
        pending = deque()
        active = []            # [future, handle, remaining steps, bytes]
        used = 0
        stopping = False
        while True:
            # new submissions: wait for one when there is nothing else to do
            idle = not active and not pending
            while True:
                try:
                    item = self._inbox.get(block=idle and not stopping)
                except queue.Empty:
                    break
                idle = False
                if item is self._STOP:
                    stopping = True
                else:
                    pending.append(item)
            while pending and len(active) < self.max_active:
                inst, dtype, fut = pending[0]
                need = ex.bytes_needed(inst, dtype)
                if need <= self.budget and used + need > self.budget:
                    break
                pending.popleft()
                if not fut.set_running_or_notify_cancel():
                    continue
                if need > self.budget:
                    fut.set_exception(ValueError(f"request needs {need} bytes, more than the budget {self.budget}"))
                    self._count("rejected")
                    continue
                if int(inst.steps) == 0:
                    u0 = np.array(inst.u0, dtype=np.float64, copy=True)
                    fut.set_result((u0,) + initial_flags(u0))
                    self._count("completed")
                    continue
                try:
                    handle = ex.admit(inst, dtype)
                except Exception as err:
                    fut.set_exception(err)
                    self._count("failed")
                    continue
                active.append([fut, handle, int(inst.steps), need])
                used += need
            with self._lock:
                self._stats["peak_active"] = max(self._stats["peak_active"], len(active))
                self._stats["peak_bytes"] = max(self._stats["peak_bytes"], used)
            if active:
                k = [min(self.tick_steps, a[2]) for a in active]
                try:
                    ex.step([a[1] for a in active], k)
                except Exception as err:
                    for a in active:
                        a[0].set_exception(err)
                        try:
                            ex.retire(a[1])
                        except Exception:
                            pass
                    self._count("failed", len(active))
                    active, used = [], 0
                    continue
                self._count("ticks")
                still = []
                for a, kk in zip(active, k):
                    a[2] -= kk
                    if a[2] == 0:
                        try:
                            a[0].set_result(ex.retire(a[1]))
                            self._count("completed")
                        except Exception as err:
                            a[0].set_exception(err)
                            self._count("failed")
                        used -= a[3]
                    else:
                        still.append(a)
                active = still
            elif stopping and not pending:
                return
