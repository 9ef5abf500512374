"""Helpers for the committed rocprofv3 summaries (text under profiles/).

* `source_hash()` fingerprints the kernel sources, so that a counter-derived HBM traffic figure
  is used only while the kernels it was measured on are unchanged.
* `stats_markdown()` turns a `--kernel-trace --stats` CSV into a short markdown table.
* `sq_markdown()` summarises shader-sequencer counter runs (VALU and LDS work, waits, occupancy).
* `traffic_from_pmc()` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of a workload and
  the same two counters read on a plain copy kernel of known size into calibrated HBM bytes
  per launch of each axis-pass kernel (or of the one-level scheme's dense products).
* `exact_axis_means()` and `mfma_markdown()` summarise the dense products' trace and their
  matrix-core counters.

The launches a summary describes are the timed ones of sfac_plan_time_passes (one pass of one
axis per launch) and sfac_plan_time_fused (two passes over axis 1 or axis d per launch, as the
steps run them at every step boundary): each block of them follows a marker kernel
pass_timing_mark<k> whose number names it (the axis for single passes, FUSED_MARK + the axis
for the fused launches, 0 after the last). Dispatches outside the marked blocks (the steps,
whose axis order alternates from step to step) are not attributed.
"""
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
PASS_KERNEL_TAGS = ("_pass_single", "_pass_multi")


KERNEL_SOURCES = ("sfac_kernels.hip", "sfac_kernels.hpp", "sfac_fft.hpp", "sfac_embed.hpp", "sfac_diag2.hpp")


_COMMENT_OR_STRING = re.compile(r'"(?:\\.|[^"\\\n])*"|//[^\n]*|/\*.*?\*/', re.S)


def code_text(text):
    """Source text with comments removed (string literals kept), lines stripped, blank lines
    dropped: what the compiler sees, up to layout."""
    text = _COMMENT_OR_STRING.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", text)
    return "\n".join(line.strip() for line in text.splitlines() if line.strip())


def source_hash(read=None):
    """SHA-256 over the names and code text (code_text) of the device-code sources, first 16 hex
    digits; comment-only edits leave it unchanged. `read(name)` returns a source's text (default:
    the files under csrc/)."""
    if read is None:
        def read(name):
            with open(os.path.join(CSRC, name), encoding="utf-8") as f:
                return f.read()
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        h.update(code_text(read(name)).encode())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def short_name(name):
    """Kernel name without the namespaces and the argument list."""
    s = name.replace("(anonymous namespace)::", "").split("(")[0]
    for p in ("void ", "sfac::"):
        s = s.replace(p, "")
    return s.strip()


MARK_TAG = "pass_timing_mark<"
FUSED_MARK = 10          # marker number of the fused launches of axis a: FUSED_MARK + a


def slot_of(axis, twice, dims):
    """Label of the launches of `axis` (0-based): one pass (twice False) or two (twice True)."""
    return axis + (dims if twice else 0)


def slot_axis(slot, dims):
    """(axis 0-based, twice) of a label."""
    return (slot - dims, True) if slot >= dims else (slot, False)


def axis_labels(names, dims, tags=PASS_KERNEL_TAGS, periodic=False):
    """Label (slot_of) of every dispatch named by `tags` in a time-ordered list of kernel names
    that lies in a marked block of timed launches, None for the others: a marker
    pass_timing_mark<k> opens the block of single passes of axis k (1..3) or of the fused
    launches of axis k - FUSED_MARK, pass_timing_mark<0> closes the last. With `periodic`
    (the one-level scheme's dense products, one per axis in the order 1..d every step), the
    dispatches outside the blocks take their place in that order, counted per element type."""
    out = []
    count = {}
    timing = None
    for nm in names:
        if MARK_TAG in nm:
            k = int(nm.split(MARK_TAG, 1)[1].split(">", 1)[0])
            if k == 0:
                timing = None
            elif k > FUSED_MARK:
                timing = slot_of(k - FUSED_MARK - 1, True, dims)
            else:
                timing = slot_of(k - 1, False, dims)
            out.append(None)
        elif any(t in nm for t in tags):
            if timing is None and periodic:
                et = "double" if "<double" in nm else "float"
                k = count.get(et, 0)
                out.append(k % dims)
                count[et] = k + 1
            else:
                out.append(timing)
        else:
            out.append(None)
    return out


def slot_name(slot, dims):
    a, twice = slot_axis(slot, dims)
    return f"{a + 1}{' (two passes)' if twice else ''}"


def trace_axis_means(trace_csv, dims):
    """Mean duration (us) per (kernel, axis, one or two passes) of the timed pass-kernel dispatches
    in a kernel trace, one list per element type; the label comes from axis_labels."""
    rows = sorted(_rows(trace_csv), key=lambda r: int(r["Start_Timestamp"]))
    labels = axis_labels([r["Kernel_Name"] for r in rows], dims)
    seq = {}
    for r, a in zip(rows, labels):
        if a is None:
            continue
        k = r["Kernel_Name"]
        et = "double" if "<double" in k else "float"
        seq.setdefault(et, [[] for _ in range(2 * dims)])[a].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), short_name(k)))
    out = {}
    for et, per in seq.items():
        res = []
        for sl in range(2 * dims):
            xs = [x for x, _ in per[sl]]
            if not xs:
                continue
            a, twice = slot_axis(sl, dims)
            res.append({"axis": a + 1, "twice": twice, "kernel": per[sl][0][1], "dispatches": len(xs),
                        "mean_us": sum(xs) / len(xs) / 1e3, "min_us": min(xs) / 1e3, "max_us": max(xs) / 1e3})
        out[et] = res
    return out


def exact_axis_means(trace_csv, ns):
    """The one-level scheme's dense products in a kernel trace: mean duration (us) per axis (the
    d-periodic dispatch order) and the flop rate, 2 N_axis flops per grid point."""
    rows = sorted(_rows(trace_csv), key=lambda r: int(r["Start_Timestamp"]))
    v = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows if "exact_gemm" in r["Kernel_Name"]]
    pts = 1
    for n in ns:
        pts *= n
    out = []
    for a in range(len(ns)):
        xs = v[a::len(ns)]
        if not xs:
            continue
        mean = sum(xs) / len(xs) / 1e3
        out.append({"axis": a + 1, "dispatches": len(xs), "mean_us": mean, "min_us": min(xs) / 1e3,
                    "max_us": max(xs) / 1e3, "tflops": 2.0 * ns[a] * pts / (mean * 1e-6) / 1e12})
    return out


def stats_markdown(stats_csv, top=8):
    rows = _rows(stats_csv)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | average us | min us | max us | share % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


EXACT_KERNEL_TAGS = ("exact_gemm",)


def _pass_counters(pmc_csv, counter, dims, tags=PASS_KERNEL_TAGS):
    """Mean counter value (KiB) per label (slot_of) over the timed dispatches of the kernels
    named by `tags` (the axis passes by default) in one --pmc run."""
    rows = [r for r in _rows(pmc_csv) if r["Counter_Name"] == counter]
    per_dispatch = {}
    names = {}
    for r in rows:
        if not (any(t in r["Kernel_Name"] for t in tags) or MARK_TAG in r["Kernel_Name"]):
            continue
        d = int(r["Dispatch_Id"])
        per_dispatch[d] = per_dispatch.get(d, 0.0) + float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    order = sorted(per_dispatch)
    labels = axis_labels([names[d] for d in order], dims, tags, periodic=tags == EXACT_KERNEL_TAGS)
    sums = [0.0] * (2 * dims)
    counts = [0] * (2 * dims)
    kern = [None] * (2 * dims)
    for d, a in zip(order, labels):
        if a is None:
            continue
        sums[a] += per_dispatch[d]
        counts[a] += 1
        kern[a] = short_name(names[d])
    return [s / c if c else None for s, c in zip(sums, counts)], counts, kern


def _copy_counter(pmc_csv, counter):
    """Mean counter value (KiB) over the copy kernel's dispatches of a --copy-probe run."""
    vals = {}
    for r in _rows(pmc_csv):
        if r["Counter_Name"] != counter or any(t in r["Kernel_Name"] for t in PASS_KERNEL_TAGS + EXACT_KERNEL_TAGS):
            continue
        d = int(r["Dispatch_Id"])
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    # the probe's copies are its largest dispatches; take those
    big = sorted(vals.values())[-20:]
    return sum(big) / len(big)


def traffic_from_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, dims, tags=PASS_KERNEL_TAGS):
    """Calibrated HBM bytes per launch of the pass kernels (or the kernels named by `tags`):
    counter KiB x 1024 x (copy bytes / copy counter bytes)."""
    f, nf, kf = _pass_counters(fetch_csv, "FETCH_SIZE", dims, tags)
    w, nw, _ = _pass_counters(write_csv, "WRITE_SIZE", dims, tags)
    cf = _copy_counter(copy_fetch_csv, "FETCH_SIZE") * 1024.0
    cw = _copy_counter(copy_write_csv, "WRITE_SIZE") * 1024.0
    scale_f = copy_bytes / cf
    scale_w = copy_bytes / cw
    per_axis = []
    for sl in range(2 * dims):
        if f[sl] is None or w[sl] is None:
            continue
        a, twice = slot_axis(sl, dims)
        fb = f[sl] * 1024.0 * scale_f
        wb = w[sl] * 1024.0 * scale_w
        per_axis.append({"axis": a + 1, "twice": twice, "kernel": kf[sl], "dispatches": nf[sl],
                         "fetch_kib_raw": round(f[sl], 1), "write_kib_raw": round(w[sl], 1),
                         "fetch_bytes": round(fb), "write_bytes": round(wb), "bytes": round(fb + wb)})
    return {"copy_bytes": copy_bytes, "copy_fetch_kib_raw": round(cf / 1024.0, 1),
            "copy_write_kib_raw": round(cw / 1024.0, 1), "fetch_scale": scale_f, "write_scale": scale_w,
            "per_axis": per_axis}


# Shader-sequencer counters of the pass kernels, two passes of eight (FP64 runs of bench.py)
SQ_SETS = (("A", "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS "
                 "SQ_WAIT_INST_ANY SQ_INSTS_VALU"),
           ("B", "SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU "
                 "SQ_ACTIVE_INST_ANY SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64"))
SQ_COMMAND = ("timeout -s KILL 90 rocprofv3 --pmc $COUNTERS --output-format csv -d $O/$SET_$W -o run -- "
              "python3 $R/bench.py --workload $W --dtype f64 --no-cpu --no-fp32 --no-exact --no-sub --steps 10 --warmup 2 "
              "--pass-reps 2")
# MI355X: 256 CUs of 4 SIMDs; a SIMD issues one wavefront VALU instruction (FP64, or FP32 unpacked) every
# 4 cycles at 2.4 GHz
VALU_WAVE_INSTR_PER_US = 256 * 4 / 4 * 2400.0


def sq_axis_means(csv_path, dims, tags=PASS_KERNEL_TAGS):
    """Mean value per label (slot_of) of every counter in one --pmc run, over the timed dispatches
    of the kernels named by `tags` (the pass kernels by default; a dispatch's rows are summed),
    with the kernel name of each; labels without dispatches are left out."""
    per, names = {}, {}
    for r in _rows(csv_path):
        if not (any(t in r["Kernel_Name"] for t in tags) or MARK_TAG in r["Kernel_Name"]):
            continue
        d = int(r["Dispatch_Id"])
        c = per.setdefault(d, {})
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    order = sorted(per)
    labels = axis_labels([names[d] for d in order], dims, tags, periodic=tags == EXACT_KERNEL_TAGS)
    names = {d: short_name(n) for d, n in names.items()}
    out = {}
    for sl in range(2 * dims):
        ds = [d for d, lab in zip(order, labels) if lab == sl]
        if not ds:
            continue
        keys = set().union(*(per[d] for d in ds))
        out[sl] = {"kernel": names[ds[0]], "dispatches": len(ds),
                   **{k: sum(per[d].get(k, 0.0) for d in ds) / len(ds) for k in keys}}
    return out


def sq_markdown(directory, workload, dims):
    """Markdown summary of the SQ_SETS runs of one workload."""
    runs = [sq_axis_means(os.path.join(directory, f"{name}_{workload}", "run_counter_collection.csv"), dims)
            for name, _ in SQ_SETS]
    axes = [(sl, {**runs[0][sl], **runs[1].get(sl, {})}) for sl in sorted(runs[0])]
    lines = [f"# Shader-sequencer counters, workload {workload} (FP64)", "",
             "Commands (run from /tmp on one MI355X; `$R` is the repository root, `$O` the output directory):", "",
             "```"]
    for name, counters in SQ_SETS:
        lines.append(SQ_COMMAND.replace("$COUNTERS", counters).replace("$SET", name).replace("$W", workload))
    lines += ["```", "",
              "Per axis, means over the timed launches of a run (sfac_plan_time_passes: one pass per launch; "
              "sfac_plan_time_fused: two passes over the axis per launch, as the steps run them). "
              "Wave-cycle counters are accumulated per wavefront in the same units, so their ratios are shares "
              "of a wavefront's lifetime. VALU issue time: the VALU instructions at one wavefront instruction "
              "per SIMD every 4 cycles on 1024 SIMDs at 2.4 GHz.", "",
              "| axis | kernel | waves | VALU instr. | VALU issue us | FMA / ADD F64 | VALU share | LDS-wait share | "
              "any-wait share | LDS instr. | bank conflicts | VMEM rd / wr |",
              "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for sl, c in axes:
        wc = c.get("SQ_WAVE_CYCLES", 0.0) or float("nan")
        lines.append(
            f"| {slot_name(sl, dims)} | `{c['kernel']}` | {c.get('SQ_WAVES', 0):.0f} | {c.get('SQ_INSTS_VALU', 0):.3g} | "
            f"{c.get('SQ_INSTS_VALU', 0) / VALU_WAVE_INSTR_PER_US:.1f} | "
            f"{c.get('SQ_INSTS_VALU_FMA_F64', 0):.3g} / {c.get('SQ_INSTS_VALU_ADD_F64', 0):.3g} | "
            f"{c.get('SQ_ACTIVE_INST_VALU', 0) / wc:.3f} | {c.get('SQ_WAIT_INST_LDS', 0) / wc:.3f} | "
            f"{c.get('SQ_WAIT_INST_ANY', 0) / wc:.3f} | {c.get('SQ_INSTS_LDS', 0):.3g} | "
            f"{c.get('SQ_LDS_BANK_CONFLICT', 0):.3g} | {c.get('SQ_INSTS_VMEM_RD', 0):.3g} / "
            f"{c.get('SQ_INSTS_VMEM_WR', 0):.3g} |")
    lines += ["", f"Device-code source hash: `{source_hash()}`.", ""]
    return "\n".join(lines)


# Matrix-core counters of the one-level scheme's dense products (bench.py runs with the exact
# comparison on)
MFMA_COUNTERS = ("SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU_MFMA_F64 SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_LDS "
                 "SQ_LDS_BANK_CONFLICT SQ_INSTS_VMEM_RD")
MFMA_COMMAND = ("timeout -s KILL 120 rocprofv3 --pmc " + MFMA_COUNTERS + " --output-format csv -d $O/$W -o run -- "
                "python3 $R/bench.py --workload $W --no-cpu --no-fp32 --no-sub --steps 10 --warmup 2 --pass-reps 2")
SIMDS = 1024                      # MI355X: 256 CUs of 4 SIMDs
CLOCK_MHZ = 2400.0


def mfma_markdown(directory, workloads):
    """Markdown summary of the matrix-core counter runs of the exact-exponential products: per
    workload and axis, FP64 MFMA instructions per dispatch, cycles per instruction, and the share
    of every SIMD's time the matrix core is busy over the dispatch's mean duration (taken from
    the trace of the same counter run)."""
    lines = ["# Matrix-core counters of the one-level scheme's dense products (`exact_gemm`, FP64)", "",
             "Commands (run from /tmp on one MI355X; `$R` is the repository root, `$O` the output directory):", "",
             "```"]
    lines += [MFMA_COMMAND.replace("$W", w) for w, _ in workloads]
    lines += ["```", "",
              "Per axis, means over the product dispatches of a run. The MFMA-busy share is "
              "SQ_VALU_MFMA_BUSY_CYCLES over (1024 SIMDs x the dispatch's duration in 2.4 GHz cycles); "
              "the duration is the mean of the same dispatches' timestamps in the counter run, which counter "
              "collection lengthens (the kernel-trace means in axis_pass_*.md are the plain durations).", "",
              "| workload | axis | kernel | waves | MFMA F64 instr. | cycles per MFMA | mean us | MFMA-busy share | "
              "LDS instr. | bank conflicts |", "|---|---|---|---|---|---|---|---|---|---|"]
    for w, dims in workloads:
        path = os.path.join(directory, w, "run_counter_collection.csv")
        means = sq_axis_means(path, dims, tags=EXACT_KERNEL_TAGS)
        # durations per axis from the rows' timestamps (one value per dispatch)
        spans = {}
        for r in _rows(path):
            if any(t in r["Kernel_Name"] for t in EXACT_KERNEL_TAGS):
                spans[int(r["Dispatch_Id"])] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        order = sorted(spans)
        for a in range(dims):
            c = means.get(a, {"kernel": None})
            ds = order[a::dims]
            us = sum(spans[d] for d in ds) / len(ds) / 1e3 if ds else float("nan")
            n = c.get("SQ_INSTS_VALU_MFMA_F64", 0.0)
            busy = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
            lines.append(f"| {w} | {a + 1} | `{c['kernel']}` | {c.get('SQ_WAVES', 0):.0f} | {n:.4g} | "
                         f"{busy / n if n else float('nan'):.1f} | {us:.2f} | "
                         f"{busy / (SIMDS * us * CLOCK_MHZ):.3f} | {c.get('SQ_INSTS_LDS', 0):.3g} | "
                         f"{c.get('SQ_LDS_BANK_CONFLICT', 0):.3g} |")
    lines += ["", f"Device-code source hash: `{source_hash()}`.", ""]
    return "\n".join(lines)


def load_traffic(path, workload, dtype, schedule=None):
    """The committed traffic record of (workload, dtype), or None if absent, if the kernel
    sources changed since it was measured, or if it was measured with another schedule."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    rec = data.get(f"{workload}:{dtype}")
    if not rec or rec.get("source_hash") != source_hash():
        return None
    if schedule is not None and rec.get("schedule") != schedule:
        return None
    return rec


# the commands that make the profiles of one workload W (run from /tmp; R is the repository root,
# O the output directory; DT is f64 and f32 in turn)
COMMANDS = """\
python3 -m paper_2209_08437_amd.autotune --fresh --out $R/paper_2209_08437_amd/tuned_mi355x.json large_2d_1023 large_3d_255 plain_2d_63 batched_2d   # the packaged schedule table, tuned on an MI355X beforehand; every run below uses it
rocprofv3 --kernel-trace --stats --output-format csv -d $O/trace_$W -o run -- python3 $R/bench.py --workload $W --no-cpu --no-sub
rocprofv3 --pmc FETCH_SIZE --output-format csv -d $O/FETCH_SIZE_$W_$DT -o run -- python3 $R/bench.py --workload $W --dtype $DT --no-cpu --no-fp32 --no-sub --steps 20 --warmup 2 --pass-reps 2
rocprofv3 --pmc WRITE_SIZE --output-format csv -d $O/WRITE_SIZE_$W_$DT -o run -- python3 $R/bench.py --workload $W --dtype $DT --no-cpu --no-fp32 --no-sub --steps 20 --warmup 2 --pass-reps 2
rocprofv3 --pmc FETCH_SIZE --output-format csv -d $O/copy_FETCH_SIZE -o run -- python3 $R/bench.py --copy-probe
rocprofv3 --pmc WRITE_SIZE --output-format csv -d $O/copy_WRITE_SIZE -o run -- python3 $R/bench.py --copy-probe"""


def _schedules(err_log):
    """Tuned schedule per dtype from the '[bench] <dtype>: tuned schedule {...}' lines of bench.py."""
    import ast
    out = {}
    try:
        for line in open(err_log):
            if "tuned schedule" in line:
                dt = line.split("]")[1].split(":")[0].strip()
                out[dt] = ast.literal_eval(line[line.index("{"):line.index("}") + 1])
    except OSError:
        pass
    return out


BATCH_TRACE_COMMAND = ("rocprofv3 --kernel-trace --stats --output-format csv -d $O/trace_batched_2d -o run -- "
                       "python3 $R/bench.py --workload batched_2d --no-cpu")


def busy_intervals(intervals):
    """Total length of the union of (start, end) intervals."""
    busy, cur_s, cur_e = 0, None, None
    for s, e in sorted(intervals):
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        busy += cur_e - cur_s
    return busy


def grouped_gaps(trace_csv):
    """Per arithmetic type, over the window of the grouped (multi-instance) pass dispatches of a
    kernel trace: wall time, the time at least one kernel runs, the idle remainder (what a
    single persistent launch could at most take back), and the sum of kernel durations over the
    busy time (how many launches overlap on average)."""
    rows = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    out = {}
    for tag, name in (("<float", "f32"), ("<double", "f64")):
        multi = [k for k in rows if "_multi" in k[2] and tag in k[2]]
        if not multi:
            continue
        t0, t1 = min(k[0] for k in multi), max(k[1] for k in multi)
        win = [k for k in rows if k[0] >= t0 and k[1] <= t1]
        busy = busy_intervals([(s, e) for s, e, _ in win])
        total = sum(e - s for s, e, _ in win)
        out[name] = {"dispatches": len(multi), "others": len(win) - len(multi), "wall_ms": (t1 - t0) / 1e6,
                     "busy_ms": busy / 1e6, "idle_ms": (t1 - t0 - busy) / 1e6,
                     "idle_frac": (t1 - t0 - busy) / (t1 - t0), "overlap": total / busy}
    return out


def batch_trace_markdown(directory):
    """Markdown summary of the kernel trace of the batched workload."""
    d = os.path.join(directory, "trace_batched_2d")
    bench = json.load(open(os.path.join(directory, "bench_batched_2d.json")))
    steps = bench["steps"] + bench["warmup"]
    lines = ["# Grouped launches, workload batched_2d", "",
             "Command (run from /tmp on one MI355X; `$R` is the repository root, `$O` the output directory):", "",
             "```", BATCH_TRACE_COMMAND, "```", "", "## Kernel trace (`--kernel-trace --stats`)", "",
             stats_markdown(os.path.join(d, "run_kernel_stats.csv"), top=12), "",
             "## Idle time between grouped launches", "",
             f"Over the window of each arithmetic's grouped pass dispatches ({steps} steps of all 64 instances: "
             "warm-up and timed region), the time during which no kernel runs is the most that one persistent "
             "launch per step could take back; the sum of kernel durations over the busy time is the mean number "
             "of launches running at once (the step graph fans a pass's launches out over several streams).", "",
             "| dtype | grouped dispatches | wall ms | busy ms | idle ms | idle share | us idle per step | "
             "launches at once |", "|---|---|---|---|---|---|---|---|"]
    for dt, g in grouped_gaps(os.path.join(d, "run_kernel_trace.csv")).items():
        lines.append(f"| {dt} | {g['dispatches']} | {g['wall_ms']:.2f} | {g['busy_ms']:.2f} | {g['idle_ms']:.2f} | "
                     f"{g['idle_frac']:.3f} | {g['idle_ms'] * 1e3 / steps:.1f} | {g['overlap']:.2f} |")
    lines += ["", f"bench.py in the same session (under the profiler): FP32 {bench['ms_per_step'] * 1e3:.1f} us per step "
              f"of all 64 instances, FP64 {bench['config']['points'] / bench['batched_f64'] * 1e6:.1f} us.", "",
              f"Device-code source hash: `{source_hash()}`.", ""]
    return "\n".join(lines)


def _main():
    """Write the markdown summary of one workload's profiles and update the traffic record."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", required=True, help="directory holding the rocprofv3 outputs")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--dims", type=int, required=True)
    ap.add_argument("--out", help="markdown summary to write")
    ap.add_argument("--traffic", help="JSON traffic record to update")
    ap.add_argument("--sq", help="write the SQ counter summary (SQ_SETS runs) to this file instead")
    ap.add_argument("--mfma", help="write the matrix-core counter summary of the exact products (MFMA_COMMAND runs of "
                                   "large_2d_1023 and large_3d_255 under --dir) to this file instead")
    ap.add_argument("--batch-trace", help="write the summary of the batched workload's kernel trace "
                                          "(BATCH_TRACE_COMMAND under --dir) to this file instead")
    a = ap.parse_args()
    if a.batch_trace:
        with open(a.batch_trace, "w") as f:
            f.write(batch_trace_markdown(a.dir))
        return
    if a.mfma:
        with open(a.mfma, "w") as f:
            f.write(mfma_markdown(a.dir, [("large_2d_1023", 2), ("large_3d_255", 3)]))
        return
    d, w = a.dir, a.workload
    if a.sq:
        with open(a.sq, "w") as f:
            f.write(sq_markdown(d, w, a.dims))
        return
    if not (a.out and a.traffic):
        ap.error("--out and --traffic are required without --sq")
    bench = json.load(open(os.path.join(d, f"bench_{w}.json")))
    lines = [f"# Axis-pass kernels, workload {w}", ""]
    lines += ["Commands (run from /tmp on one MI355X; `$R` is the repository root, `$O` the output "
              "directory, `$DT` f64 and f32 in turn):", "", "```"]
    lines += [COMMANDS.replace("$W", w), "```", ""]
    lines += ["## Kernel trace (`--kernel-trace --stats`)", "",
              stats_markdown(os.path.join(d, f"trace_{w}", "run_kernel_stats.csv")), ""]
    means = trace_axis_means(os.path.join(d, f"trace_{w}", "run_kernel_trace.csv"), a.dims)
    lines += ["Per axis, the timed launches (sfac_plan_time_passes: one pass per launch; sfac_plan_time_fused: "
              "two passes over the axis per launch, the step boundary in between, as the steps run them):", "",
              "| element | axis | kernel | dispatches | mean us | min us | max us |", "|---|---|---|---|---|---|---|"]
    for et, res in means.items():
        for r in res:
            lines.append(f"| {et} | {r['axis']}{' (two passes)' if r['twice'] else ''} | `{r['kernel']}` | "
                         f"{r['dispatches']} | {r['mean_us']:.2f} | {r['min_us']:.2f} | {r['max_us']:.2f} |")
    ex = exact_axis_means(os.path.join(d, f"trace_{w}", "run_kernel_trace.csv"), bench["config"]["grid"])
    if ex:
        lines += ["", "One-level scheme with the exact exponential (`exact_gemm`, FP64 matrix cores; "
                  "2 N flops per point and axis; peak 78.6 TFLOP/s):", "",
                  "| axis | dispatches | mean us | min us | max us | TFLOP/s | frac |", "|---|---|---|---|---|---|---|"]
        for r in ex:
            lines.append(f"| {r['axis']} | {r['dispatches']} | {r['mean_us']:.2f} | {r['min_us']:.2f} | "
                         f"{r['max_us']:.2f} | {r['tflops']:.1f} | {r['tflops'] / 78.6:.3f} |")
        one = bench.get("one_level_exact", {})
        if "ms_per_step" in one:
            lines += ["", f"bench.py in the same session: {one['ms_per_step'] * 1e3:.1f} us per one-level step "
                      f"({one['product_TFLOPs']} TFLOP/s over the step), plan creation {one['plan_create_ms']:.0f} ms."]
    def launches(roof):
        return (f"pass us {[round(x * 1e3, 2) for x in roof['pass_ms']]}, two-pass launches (axis 1, axis d) us "
                f"{[round(x * 1e3, 2) for x in roof.get('fused_ms', [])]}")
    lines += ["", f"bench.py in the same session (no profiler): FP64 {bench['ms_per_step'] * 1e3:.2f} us/step, "
              f"{launches(bench['roofline'])}; FP32 {bench['fp32']['ms_per_step'] * 1e3:.2f} us/step, "
              f"{launches(bench['fp32']['roofline'])} (0: that axis' kernel does not fuse).", ""]
    scheds = _schedules(os.path.join(d, f"bench_{w}.err"))
    rec_all = {}
    try:
        rec_all = json.load(open(a.traffic))
    except (OSError, ValueError):
        pass
    lines += ["## HBM traffic (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`)", "",
              "Counters in KiB per dispatch, calibrated on a plain copy of 512 MiB (bench.py --copy-probe): "
              "bytes = KiB x 1024 x (copy bytes / copy counter bytes).", "",
              "| dtype | axis | kernel | FETCH KiB | WRITE KiB | calibrated bytes | algorithmic bytes | ratio |",
              "|---|---|---|---|---|---|---|---|"]
    for dt, es in (("f64", 8), ("f32", 4)):
        t = traffic_from_pmc(os.path.join(d, f"FETCH_SIZE_{w}_{dt}", "run_counter_collection.csv"),
                             os.path.join(d, f"WRITE_SIZE_{w}_{dt}", "run_counter_collection.csv"),
                             os.path.join(d, "copy_FETCH_SIZE", "run_counter_collection.csv"),
                             os.path.join(d, "copy_WRITE_SIZE", "run_counter_collection.csv"), 512 << 20, a.dims)
        pts = 1
        for n in bench["config"]["grid"]:
            pts *= n
        alg = 2 * pts * es
        for r in t["per_axis"]:
            lines.append(f"| {dt} | {r['axis']}{' (two passes)' if r['twice'] else ''} | `{r['kernel']}` | "
                         f"{r['fetch_kib_raw']} | {r['write_kib_raw']} | {r['bytes']} | {alg} | {r['bytes'] / alg:.3f} |")
        rec_all[f"{w}:{dt}"] = {"source_hash": source_hash(), "profile": os.path.basename(a.out),
                                "algorithmic_bytes": alg, "schedule": scheds.get(dt), **t}
    ex_t = None
    try:
        ex_t = traffic_from_pmc(os.path.join(d, f"FETCH_SIZE_{w}_f64", "run_counter_collection.csv"),
                                os.path.join(d, f"WRITE_SIZE_{w}_f64", "run_counter_collection.csv"),
                                os.path.join(d, "copy_FETCH_SIZE", "run_counter_collection.csv"),
                                os.path.join(d, "copy_WRITE_SIZE", "run_counter_collection.csv"), 512 << 20, a.dims,
                                tags=EXACT_KERNEL_TAGS)
    except (TypeError, ZeroDivisionError, OSError):
        ex_t = None
    if ex_t and ex_t["per_axis"] and all(r["dispatches"] for r in ex_t["per_axis"]):
        grid = bench["config"]["grid"]
        pts = 1
        for n in grid:
            pts *= n
        lines += ["", "One-level scheme's dense products (`exact_gemm`, FP64; algorithmic bytes: read the state and "
                  "e^{tau B}, write the product):", "",
                  "| axis | FETCH KiB | WRITE KiB | calibrated bytes | algorithmic bytes | ratio |", "|---|---|---|---|---|---|"]
        for r in ex_t["per_axis"]:
            alg = 8 * (2 * pts + grid[r["axis"] - 1] ** 2)
            r["algorithmic_bytes"] = alg
            lines.append(f"| {r['axis']} | {r['fetch_kib_raw']} | {r['write_kib_raw']} | {r['bytes']} | {alg} | "
                         f"{r['bytes'] / alg:.3f} |")
        rec_all[f"{w}:exact"] = {"source_hash": source_hash(), "profile": os.path.basename(a.out),
                                 "schedule": None, **ex_t}
    lines += ["", f"Copy calibration: FETCH_SIZE read {t['copy_fetch_kib_raw']} KiB and WRITE_SIZE "
              f"{t['copy_write_kib_raw']} KiB per 512 MiB copy (scales {t['fetch_scale']:.4f}, "
              f"{t['write_scale']:.4f}).", f"Device-code source hash: `{source_hash()}`.", ""]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    with open(a.traffic, "w") as f:
        json.dump(rec_all, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    _main()
