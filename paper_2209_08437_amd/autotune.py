"""Autotuner for the axis-pass schedules.

For one problem shape it times candidate schedules of every axis pass on the device and keeps
the fastest: the method (embedded or diagonal, where both apply), the diagonal kernel (generic
or register-resident two-step), the number of elements each thread holds in the embedded kernel
(4, 8 or 16: more threads per line and more radix passes, or fewer threads and fewer passes) and
the number of line pairs per thread block. Timing uses
sfac_plan_time_passes (HIP events around each pass on the plan's stream), so only the device
work is measured. Results are cached in a JSON file keyed by (axis length, lines in the pass,
stride class, dtype), so a shape is tuned once per machine; `SFAC_TUNE_CACHE` names the file
(default ~/.cache/sfac_autotune.json).

All candidates compute the same operator and pass the same parity tests; they differ in speed
and in rounding order only.
"""
import itertools
import json
import os

import numpy as np


# schedules measured on an MI355X for the benchmark shapes (written by this tuner, read only)
PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def cache_path():
    return os.environ.get("SFAC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sfac_autotune.json"))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def axis_key(ns, axis, dtype):
    """Cache key of one axis pass: its length, the number of lines, and whether they are
    contiguous (axis 1) or strided."""
    n = ns[axis]
    lines = int(np.prod(ns)) // n
    return f"{dtype}:n{n}:lines{lines}:{'contig' if axis == 0 else 'strided'}"


# N = A B pairs of the register-resident diagonal kernel (the library's list)
DIAG2_PAIRS = ((3, 5), (5, 7), (7, 9), (9, 11), (11, 13), (13, 15), (15, 17), (5, 9), (7, 11))


def candidates(n):
    """Schedules worth timing for an axis of n interior nodes:
    (method, elems_log2, lines_per_block, kernel); kernel 4 is the embedded method with LDS-staged
    tiles."""
    from . import sfac
    out = []
    for le, lpb in itertools.product((3, 4), (0, 1, 2, 4)):
        out.append(("embed", le, lpb, 0))
    m = 2
    while m < 2 * n - 1:
        m *= 2
    if 64 <= m <= 2048:
        for lpb in (0, 1, 2):
            out.append(("embed", 2, lpb, 0))
    if m >= 64:
        # tiles staged through LDS: strided passes read runs of several line pairs
        for le in ((2, 3, 4) if m <= 2048 else (3, 4)):
            for lpb in (0, 2, 4):
                out.append(("embed", le, lpb, 4))
    pair = [(a, b) for a, b in DIAG2_PAIRS if a * b == n]
    if pair:
        full = 256 // max(pair[0])          # lines of a whole 256-thread block
        for lpb in sorted({0, 2, 3, 4, 5, 6, 7, 10, full}):
            out.append(("diag", 0, lpb, 2))
        lpw = 64 // max(pair[0])
        for w in (0, 1, 2, 4):
            out.append(("diag", 0, w * lpw, 3))
    try:
        sfac.axis_tables(n, 1.5, 0.1, 0.01, 0.1, "diag")
        out.append(("diag", 0, 0, 1))
    except sfac.SfacError:
        pass
    return out


def _step_ms(ns, alphas, eps, tau, hs, dtype, sched, u0, steps=50, trials=5):
    """Mean step time (ms) of a plan with this schedule, replaying its step graphs: the least of
    `trials` timed runs of `steps` steps after as many warm-up steps."""
    import torch
    from . import sfac
    with sfac.Plan(ns, alphas, eps, tau, hs, dtype, **sched) as p:
        u = u0.clone()
        p.step(u, steps)
        torch.cuda.synchronize()
        best = None
        for _ in range(trials):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            p.step(u, steps)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / steps
            best = t if best is None else min(best, t)
    return best


def tune(ns, alphas, eps, tau, hs, dtype="f64", reps=10, use_cache=True, verbose=False, path=None, save=True,
         tie=0.03):
    """Best schedule per axis for this shape: returns dict(method=[...], elems_log2=[...],
    lines_per_block=[...], kernel=[...], ms=[...]) ready to pass to sfac.Plan as keyword arguments
    (after dropping 'ms'). `path` names the cache file (default: cache_path()); with save=False
    shapes missing from it are tuned but the file is left as it is.

    Candidates are timed per pass (events around each launch). Those within `tie` of an axis'
    best are then timed again as whole steps replayed from graphs, the way plans run, with every
    axis of the same cache key (e.g. both strided axes in 3D) on the candidate; the fastest step
    wins. Per-pass timing alone cannot see how consecutive passes overlap."""
    import torch
    from . import sfac
    path = path or cache_path()
    cache = _load_cache(path) if use_cache else {}
    dims = len(ns)
    best = {"method": [None] * dims, "elems_log2": [0] * dims, "lines_per_block": [0] * dims,
            "kernel": [0] * dims, "ms": [None] * dims}
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(0)
    u0 = torch.tensor(rng.uniform(-0.9, 0.9, size=tuple(reversed(ns))), dtype=tdt, device="cuda")
    fresh = {}          # key -> candidate timings of the keys tuned here
    for a in range(dims):
        key = axis_key(ns, a, dtype)
        if key in cache and len(cache[key]) == 5:
            m, le, lpb, kern, ms = cache[key]
        else:
            results = []
            for m, le, lpb, kern in candidates(ns[a]):
                meth = [None] * dims
                meth[a] = m
                les = [0] * dims
                les[a] = le
                lp = [0] * dims
                lp[a] = lpb
                kk = [0] * dims
                kk[a] = kern
                try:
                    p = sfac.Plan(ns, alphas, eps, tau, hs, dtype, method=meth, elems_log2=les, lines_per_block=lp,
                                  kernel=kk, use_graph=False)
                except sfac.SfacError:
                    continue
                u = u0.clone()
                p.time_passes(u, 2)
                t = p.time_passes(u, reps)[a]
                p.close()
                results.append((t, m, le, lpb, kern))
                if verbose:
                    print(f"  axis {a + 1} {m} kernel {kern} elems 2^{le} lines/block {lpb or 'auto'}: "
                          f"{t * 1e3:.1f} us", flush=True)
            ms, m, le, lpb, kern = min(results)
            cache[key] = [m, le, lpb, kern, ms]
            fresh[key] = sorted(results)
        best["method"][a] = m
        best["elems_log2"][a] = le
        best["lines_per_block"][a] = lpb
        best["kernel"][a] = kern
        best["ms"][a] = ms
    for key, results in fresh.items():
        close = [r for r in results if r[0] <= results[0][0] * (1.0 + tie)]
        if len(close) < 2:
            continue
        axes = [a for a in range(dims) if axis_key(ns, a, dtype) == key]
        timed = []
        for cand in close:
            t, m, le, lpb, kern = cand
            sched = {k: list(best[k]) for k in SCHEDULE_KEYS}
            for a in axes:
                sched["method"][a], sched["elems_log2"][a] = m, le
                sched["lines_per_block"][a], sched["kernel"][a] = lpb, kern
            step = _step_ms(ns, alphas, eps, tau, hs, dtype, sched, u0)
            timed.append((step, cand))
            if verbose:
                print(f"  step with axes {[a + 1 for a in axes]} on {m} kernel {kern} elems 2^{le} "
                      f"lines/block {lpb or 'auto'}: {step * 1e3:.1f} us", flush=True)
        t, m, le, lpb, kern = min(timed)[1]
        cache[key] = [m, le, lpb, kern, t]
        for a in axes:
            best["method"][a], best["elems_log2"][a] = m, le
            best["lines_per_block"][a], best["kernel"][a], best["ms"][a] = lpb, kern, t
    if use_cache and save:
        _save_cache(path, cache)
    return best


SCHEDULE_KEYS = ("method", "elems_log2", "lines_per_block", "kernel")


def load_table(path=None):
    """A schedule cache file as a dict (default: the packaged MI355X table); {} if unreadable."""
    return _load_cache(path or PACKAGED)


def lookup(ns, dtype, path=None, table=None):
    """The cached schedule of this shape (dict of SCHEDULE_KEYS, per-axis lists) if every axis is
    in the cache (`table` as returned by load_table, else the file `path`, default the packaged
    MI355X table), else None. Launches nothing."""
    cache = table if table is not None else _load_cache(path or PACKAGED)
    dims = len(ns)
    out = {k: [None if k == "method" else 0] * dims for k in SCHEDULE_KEYS}
    for a in range(dims):
        rec = cache.get(axis_key(ns, a, dtype))
        if not rec or len(rec) != 5:
            return None
        out["method"][a], out["elems_log2"][a], out["lines_per_block"][a], out["kernel"][a] = rec[:4]
    return out


def schedules(instances, dtype="f64", path=None, tune_missing=True, reps=10):
    """Schedules for a batch: one per instance, looked up by shape in the cache file `path`
    (default: the packaged MI355X table); shapes it lacks are tuned on the device once per
    distinct shape (not written back) if tune_missing, else left automatic (None)."""
    path = path or PACKAGED
    done = {}
    out = []
    for inst in instances:
        key = (tuple(inst.ns), dtype)
        if key not in done:
            sch = lookup(inst.ns, dtype, path)
            if sch is None and tune_missing:
                best = tune(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype, reps=reps, path=path,
                            save=False)
                sch = {k: best[k] for k in SCHEDULE_KEYS}
            done[key] = sch
        out.append(done[key])
    return out


def _main():
    """Tune every distinct shape of the named workloads for both arithmetic types into a cache
    file (the packaged MI355X table is written this way, on one MI355X):
    python -m paper_2209_08437_amd.autotune --out FILE large_2d_1023 large_3d_255 plain_2d_63 batched_2d
    Shapes already in FILE are kept; --fresh starts from an empty file."""
    import argparse
    import time
    from . import workloads as W
    ap = argparse.ArgumentParser(description=_main.__doc__)
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--out", required=True)
    ap.add_argument("--fresh", action="store_true")
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args()
    if a.fresh and os.path.exists(a.out):
        os.remove(a.out)
    seen = set()
    for name in a.workloads:
        made = getattr(W, name)()
        insts = made if isinstance(made, list) else [made]
        for dt in ("f64", "f32"):
            for inst in insts:
                key = (tuple(inst.ns), dt)
                if key in seen:
                    continue
                seen.add(key)
                t0 = time.perf_counter()
                best = tune(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dt, reps=a.reps, path=a.out)
                print(f"{name} {dt} {tuple(inst.ns)}: {{{', '.join(f'{k}: {best[k]}' for k in SCHEDULE_KEYS)}}} "
                      f"pass us {[round(x * 1e3, 1) for x in best['ms']]} ({time.perf_counter() - t0:.1f} s)",
                      flush=True)


if __name__ == "__main__":
    _main()
