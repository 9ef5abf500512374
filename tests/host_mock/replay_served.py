"""Replays served streams through serve.Server against a host build of the library (mock HIP
runtime, sanitizers): the call sequence of the device executor (a plan per request, grouped
steps with cached step graphs, flags, destroy), with a simulated clock. Usage:
    replay_served.py LIBRARY COUNT:RATE:SEED[:TICK_STEPS] ...
Prints one line per stream; exits non-zero (the mock or a sanitizer aborts) on misuse. When the
mock injects failures (MOCK_FAIL_EVERY), the executor counts the library's errors and goes on:
plan creation is retried, a failed grouped step or status read is skipped."""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import numpy as np  # noqa: E402

from paper_2209_08437_amd import autotune, serve, sfac, workloads as W  # noqa: E402


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class HostExecutor:
    """GpuExecutor's calls, with states in the mock's memory and a modelled step time."""
    on_device = True

    def __init__(self, L, clock, gps=5e10):
        self.L, self.clock, self.gps = L, clock, gps
        self.group = sfac.Group(stream=0)
        self.table = autotune.load_table()
        self._built = {}
        self.errors = 0

    def _tolerate(self, fn, tries=1):
        """fn(); a library error is counted and, within `tries`, retried"""
        for k in range(tries):
            try:
                return fn()
            except sfac.SfacError:
                self.errors += 1
                if k + 1 == tries:
                    raise

    def _plan(self, inst, dtype):
        hit = self._built.get(id(inst))
        if hit is not None and hit[0] is inst and hit[1] == dtype:
            return hit[2]
        sched = autotune.lookup(inst.ns, dtype, table=self.table)
        plan = self._tolerate(lambda: sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype, stream=0,
                                                use_graph=False, **(sched or {})), tries=8)
        if len(self._built) >= 4:
            self._built.pop(next(iter(self._built)))[2].close()
        self._built[id(inst)] = (inst, dtype, plan)
        return plan

    def bytes_needed(self, inst, dtype):
        return int(np.prod(inst.ns)) * (8 if dtype == "f64" else 4) + int(self._plan(inst, dtype).device_bytes)

    def admit(self, inst, dtype):
        plan = self._plan(inst, dtype)
        self._built.pop(id(inst), None)
        u = None
        for _ in range(8):
            u = self.L.mock_alloc(int(np.prod(inst.ns)) * (8 if dtype == "f64" else 4))
            if u:
                break
        assert u
        return (plan, u, inst)

    def step(self, handles, nsteps):
        n = len(handles)
        hs = (ctypes.c_void_p * n)(*[h[0]._h.value for h in handles])
        ptrs = (ctypes.c_void_p * n)(*[h[1] for h in handles])
        steps = (ctypes.c_int64 * n)(*[int(x) for x in nsteps])
        try:
            sfac._check(self.L.sfac_group_step(self.group._h, n, hs, ptrs, steps))
        except sfac.SfacError:
            self.errors += 1
        self.clock.t += 2e-4 + sum(int(np.prod(h[2].ns)) * k for h, k in zip(handles, nsteps)) / self.gps

    def retire(self, handle):
        plan, u, _ = handle
        try:
            f, m = plan.flags()
        except sfac.SfacError:
            self.errors += 1
            f, m = 0, 0.0
        plan.close()
        self.L.mock_free(u)
        return None, f, m

    def close(self):
        for _, _, p in self._built.values():
            p.close()
        self.group.close()


def main():
    sfac.LIB_PATH = sys.argv[1]
    L = sfac.lib()
    L.mock_alloc.restype = ctypes.c_void_p
    L.mock_alloc.argtypes = [ctypes.c_size_t]
    L.mock_free.argtypes = [ctypes.c_void_p]
    for name in ("mock_live_allocations", "mock_live_streams", "mock_live_graphs", "mock_injected_failures"):
        getattr(L, name).restype = ctypes.c_size_t
    for spec in sys.argv[2:]:
        fields = spec.split(":")
        count, rate, seed = fields[:3]
        tick = int(fields[3]) if len(fields) > 3 else 50
        clock = Clock()
        ex = HostExecutor(L, clock)
        reqs = W.served_stream(count=int(count), rate=float(rate), seed=int(seed), materialize=False)
        srv = serve.Server(ex, budget_bytes=16 << 30, tick_steps=tick, clock=clock, sleep=clock.sleep)
        _, summ = srv.run(reqs)
        ex.close()
        print(f"stream {spec}: completed {summ['completed']} ticks {summ['ticks']} peak_active "
              f"{summ['peak_active']} injected {L.mock_injected_failures()} errors {ex.errors} left: allocations "
              f"{L.mock_live_allocations()} streams {L.mock_live_streams()} graphs {L.mock_live_graphs()}",
              flush=True)


if __name__ == "__main__":
    main()
