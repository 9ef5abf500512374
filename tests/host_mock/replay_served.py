"""Replays served streams through serve.Server against a host build of the library (mock HIP
runtime, sanitizers): the call sequence of the device executor (a plan per request, grouped
steps with cached step graphs, flags, destroy), with a simulated clock. Usage:
    replay_served.py LIBRARY COUNT:RATE:SEED ...
Prints one line per stream; exits non-zero (the mock or a sanitizer aborts) on misuse."""
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

    def _plan(self, inst, dtype):
        hit = self._built.get(id(inst))
        if hit is not None and hit[0] is inst and hit[1] == dtype:
            return hit[2]
        sched = autotune.lookup(inst.ns, dtype, table=self.table)
        plan = sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype, stream=0, use_graph=False,
                         **(sched or {}))
        if len(self._built) >= 4:
            self._built.pop(next(iter(self._built)))[2].close()
        self._built[id(inst)] = (inst, dtype, plan)
        return plan

    def bytes_needed(self, inst, dtype):
        return int(np.prod(inst.ns)) * (8 if dtype == "f64" else 4) + int(self._plan(inst, dtype).device_bytes)

    def admit(self, inst, dtype):
        plan = self._plan(inst, dtype)
        self._built.pop(id(inst), None)
        u = self.L.mock_alloc(int(np.prod(inst.ns)) * (8 if dtype == "f64" else 4))
        assert u
        return (plan, u, inst)

    def step(self, handles, nsteps):
        n = len(handles)
        hs = (ctypes.c_void_p * n)(*[h[0]._h.value for h in handles])
        ptrs = (ctypes.c_void_p * n)(*[h[1] for h in handles])
        steps = (ctypes.c_int64 * n)(*[int(x) for x in nsteps])
        sfac._check(self.L.sfac_group_step(self.group._h, n, hs, ptrs, steps))
        self.clock.t += 2e-4 + sum(int(np.prod(h[2].ns)) * k for h, k in zip(handles, nsteps)) / self.gps

    def retire(self, handle):
        plan, u, _ = handle
        f, m = plan.flags()
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
    for name in ("mock_live_allocations", "mock_live_streams", "mock_live_graphs"):
        getattr(L, name).restype = ctypes.c_size_t
    for spec in sys.argv[2:]:
        count, rate, seed = spec.split(":")
        clock = Clock()
        ex = HostExecutor(L, clock)
        reqs = W.served_stream(count=int(count), rate=float(rate), seed=int(seed), materialize=False)
        srv = serve.Server(ex, budget_bytes=16 << 30, tick_steps=50, clock=clock, sleep=clock.sleep)
        _, summ = srv.run(reqs)
        ex.close()
        print(f"stream {spec}: completed {summ['completed']} ticks {summ['ticks']} peak_active "
              f"{summ['peak_active']} left: allocations {L.mock_live_allocations()} streams "
              f"{L.mock_live_streams()} graphs {L.mock_live_graphs()}", flush=True)


if __name__ == "__main__":
    main()
