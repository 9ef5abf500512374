"""Host tests of the profile helpers: the device-code fingerprint that keys the committed HBM
traffic record, the counter calibration and the per-axis attribution of pass dispatches."""
import csv
import json
import os

import pytest

from paper_2209_08437_amd import profiling as P

PASS = "void sfac::(anonymous namespace)::embed_pass_single<double, 11, 3, false, false>(sfac::PassDesc<double>)"
TWICE = "void sfac::(anonymous namespace)::embed_pass_single<double, 11, 3, false, true>(sfac::PassDesc<double>)"
COPY = "__amd_rocclr_copyBuffer"


def MARK(k):
    return f"void sfac::(anonymous namespace)::pass_timing_mark<{k}>()"


def _sources():
    out = {}
    for name in P.KERNEL_SOURCES:
        with open(os.path.join(P.CSRC, name), encoding="utf-8") as f:
            out[name] = f.read()
    return out


def test_code_text_drops_comments_and_keeps_strings():
    text = 'int a = 1; // one\n/* two\n   lines */ const char* s = "x // y /* z */";\n\n   b();  \n'
    assert P.code_text(text) == 'int a = 1;\nconst char* s = "x // y /* z */";\nb();'


def test_source_hash_follows_code_not_comments():
    src = _sources()
    base = P.source_hash(lambda n: src[n])
    assert base == P.source_hash()
    name = "sfac_kernels.hip"
    # a comment edited, added and a blank line inserted: same code, same fingerprint
    edited = src[name].replace("//", "// edited:", 1) + "\n\n// trailing note\n"
    assert P.source_hash(lambda n: edited if n == name else src[n]) == base
    # a code edit changes it
    assert "kBlockThreads" in src["sfac_kernels.hpp"]
    code = src["sfac_kernels.hpp"].replace("kBlockThreads", "kBlockThreadz", 1)
    assert P.source_hash(lambda n: code if n == "sfac_kernels.hpp" else src[n]) != base


def _write_pmc(path, rows):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))


def _timed_2d(counter, vals, extra=()):
    """Counter rows of a 2D run: step dispatches (not attributed), then the timed blocks of
    sfac_plan_time_passes (axis 1, axis 2) and sfac_plan_time_fused (axis 1, axis 2), two
    launches each, behind their markers; `vals` holds the eight launches' values."""
    rows = [(1, PASS, counter, 5000.0), (2, TWICE, counter, 5000.0)]          # steps: ignored
    names = [MARK(1), PASS, PASS, MARK(2), PASS, PASS, MARK(11), TWICE, TWICE, MARK(12), TWICE, TWICE, MARK(0)]
    it = iter(vals)
    for i, nm in enumerate(names, start=3):
        rows.append((i, nm, counter, 0.0 if "mark" in nm else next(it)))
    return rows + list(extra)


def test_traffic_calibration_and_axis_attribution(tmp_path):
    # a 2D run: each dispatch's counter may be reported in several parts (as per-XCD rows) that
    # must be summed; a copy kernel is not a pass kernel; only the marked blocks count
    # the first timed launch (dispatch 4) comes in two rows: 60 + 40
    fetch = _timed_2d("FETCH_SIZE", [60.0, 110.0, 200.0, 210.0, 300.0, 300.0, 400.0, 400.0],
                      extra=[(4, PASS, "FETCH_SIZE", 40.0), (99, COPY, "FETCH_SIZE", 9999.0)])
    write = _timed_2d("WRITE_SIZE", [300.0, 320.0, 400.0, 420.0, 500.0, 500.0, 600.0, 600.0])
    copy_bytes = 1 << 20
    # the copy probe: 20 large copies whose FETCH counter reads half the copied bytes and whose
    # WRITE counter reads all of them, plus one small unrelated dispatch
    cf = [(i, COPY, "FETCH_SIZE", copy_bytes / 2 / 1024) for i in range(1, 21)] + [(21, COPY, "FETCH_SIZE", 1.0)]
    cw = [(i, COPY, "WRITE_SIZE", copy_bytes / 1024) for i in range(1, 21)] + [(21, COPY, "WRITE_SIZE", 1.0)]
    paths = {}
    for key, rows in (("f", fetch), ("w", write), ("cf", cf), ("cw", cw)):
        paths[key] = str(tmp_path / f"{key}.csv")
        _write_pmc(paths[key], rows)
    t = P.traffic_from_pmc(paths["f"], paths["w"], paths["cf"], paths["cw"], copy_bytes, 2)
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    a1, a2, f1, f2 = t["per_axis"]
    assert [(r["axis"], r["twice"]) for r in t["per_axis"]] == [(1, False), (2, False), (1, True), (2, True)]
    assert (a1["dispatches"], a2["dispatches"], f1["dispatches"]) == (2, 2, 2)
    assert a1["fetch_kib_raw"] == 105.0 and a2["fetch_kib_raw"] == 205.0 and f2["fetch_kib_raw"] == 400.0
    assert a1["write_kib_raw"] == 310.0 and a2["write_kib_raw"] == 410.0 and f1["write_kib_raw"] == 500.0
    assert a1["bytes"] == round(105.0 * 1024 * 2 + 310.0 * 1024)
    assert a2["bytes"] == round(205.0 * 1024 * 2 + 410.0 * 1024)
    assert a1["kernel"] == "embed_pass_single<double, 11, 3, false, false>"
    assert f1["kernel"] == "embed_pass_single<double, 11, 3, false, true>"


def test_trace_axis_means(tmp_path):
    path = str(tmp_path / "trace.csv")
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [(PASS, 0, 900), (MARK(1), 900, 1000), (PASS, 1000, 3000), (PASS, 3000, 7000), (COPY, 7000, 9000),
            (MARK(2), 8990, 9000), (PASS, 9000, 12000), (PASS, 12000, 17000),
            (MARK(12), 16990, 17000), (TWICE, 17000, 25000), (MARK(0), 24990, 25000), (PASS, 25000, 26000)]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in reversed(rows):     # unordered on disk: sorted by start time
            w.writerow(dict(zip(fields, r)))
    m = P.trace_axis_means(path, 2)["double"]
    assert [(r["axis"], r["twice"], r["dispatches"]) for r in m] == [(1, False, 2), (2, False, 2), (2, True, 1)]
    assert m[0]["mean_us"] == pytest.approx(3.0) and m[1]["mean_us"] == pytest.approx(4.0)
    assert m[0]["min_us"] == pytest.approx(2.0) and m[1]["max_us"] == pytest.approx(5.0)
    assert m[2]["mean_us"] == pytest.approx(8.0)


def test_axis_labels_follow_timing_marks():
    """Only the timed launches are attributed: blocks announced by pass_timing_mark<axis> (one pass
    per launch) or pass_timing_mark<FUSED_MARK + axis> (two passes over the axis per launch), the
    last closed by pass_timing_mark<0>; step dispatches, whose axis order alternates, get None.
    The one-level scheme's products (periodic) take the d-periodic order outside the blocks."""
    A = "void sfac::(anonymous namespace)::diag2_pass_single<double, 15, 17, true, false>(sfac::PassDesc<double>)"
    B = "void sfac::(anonymous namespace)::diag2_pass_single<double, 15, 17, false, false>(sfac::PassDesc<double>)"
    T = "void sfac::(anonymous namespace)::diag2_pass_single<double, 15, 17, true, true>(sfac::PassDesc<double>)"
    names = [A, B, T, COPY,
             MARK(1), A, A, MARK(2), B, B, MARK(3), B, B, MARK(11), T, MARK(13), T, T, MARK(0),
             A, T, B]
    got = P.axis_labels(names, 3)
    assert got == [None, None, None, None,
                   None, 0, 0, None, 1, 1, None, 2, 2, None, 3, None, 5, 5, None,
                   None, None, None]
    assert [P.slot_axis(s, 3) for s in (0, 2, 3, 5)] == [(0, False), (2, False), (0, True), (2, True)]
    G = "void sfac::(anonymous namespace)::exact_gemm<2, 16>(double const*)"
    assert P.axis_labels([G, G, G, G, G], 2, tags=P.EXACT_KERNEL_TAGS, periodic=True) == [0, 1, 0, 1, 0]


def test_trace_axis_means_with_timed_blocks(tmp_path):
    path = str(tmp_path / "trace.csv")
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    mark = lambda a: f"void sfac::(anonymous namespace)::pass_timing_mark<{a}>()"
    rows = [(PASS, 0, 2000), (PASS, 2000, 6000),                                    # one step
            (mark(1), 6000, 6100), (PASS, 6100, 8100), (PASS, 8100, 10100),       # axis 1 timed
            (mark(2), 10100, 10200), (PASS, 10200, 14200), (mark(0), 14200, 14300),
            (PASS, 14300, 16300), (PASS, 16300, 20300)]                          # one more step: ignored
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))
    m = P.trace_axis_means(path, 2)["double"]
    assert [r["dispatches"] for r in m] == [2, 1]
    assert m[0]["mean_us"] == pytest.approx(2.0) and m[1]["mean_us"] == pytest.approx(4.0)


def test_traffic_record_used_only_for_current_code_and_schedule(tmp_path):
    sched = {"method": ["embed", "embed"], "elems_log2": [3, 3], "lines_per_block": [4, 4], "kernel": [0, 0]}
    rec = {"source_hash": P.source_hash(), "schedule": sched, "per_axis": [{"axis": 1, "bytes": 1}]}
    path = str(tmp_path / "traffic.json")
    with open(path, "w") as f:
        json.dump({"w:f64": rec, "old:f64": dict(rec, source_hash="0" * 16)}, f)
    assert P.load_traffic(path, "w", "f64", sched)["per_axis"][0]["bytes"] == 1
    assert P.load_traffic(path, "w", "f64") is not None
    assert P.load_traffic(path, "w", "f32", sched) is None
    assert P.load_traffic(path, "old", "f64", sched) is None
    assert P.load_traffic(path, "w", "f64", dict(sched, lines_per_block=[0, 0])) is None
    assert P.load_traffic(str(tmp_path / "missing.json"), "w", "f64") is None



def test_sq_axis_means(tmp_path):
    # a 2D run: per-XCD rows of a dispatch are summed, other kernels and step dispatches skipped,
    # labels without timed dispatches left out
    rows = [(1, PASS, "SQ_WAVES", 7.0), (2, MARK(1), "SQ_WAVES", 1.0),
            (3, PASS, "SQ_WAVES", 1000.0), (3, PASS, "SQ_WAVES", 1048.0), (3, PASS, "SQ_INSTS_VALU", 10.0),
            (4, PASS, "SQ_WAVES", 2048.0), (4, PASS, "SQ_INSTS_VALU", 20.0),
            (5, COPY, "SQ_WAVES", 5.0), (6, MARK(12), "SQ_WAVES", 1.0),
            (7, TWICE, "SQ_WAVES", 2048.0), (7, TWICE, "SQ_INSTS_VALU", 30.0),
            (8, TWICE, "SQ_WAVES", 2048.0), (8, TWICE, "SQ_INSTS_VALU", 50.0), (9, MARK(0), "SQ_WAVES", 1.0)]
    path = str(tmp_path / "sq.csv")
    _write_pmc(path, rows)
    m = P.sq_axis_means(path, 2)
    assert sorted(m) == [0, 3]
    a1, f2 = m[0], m[3]
    assert a1["dispatches"] == f2["dispatches"] == 2
    assert a1["SQ_WAVES"] == 2048.0 and f2["SQ_WAVES"] == 2048.0
    assert a1["SQ_INSTS_VALU"] == 15.0 and f2["SQ_INSTS_VALU"] == 40.0
    assert a1["kernel"] == "embed_pass_single<double, 11, 3, false, false>"


def test_exact_axis_means(tmp_path):
    # a 2D one-level run: products alternate axis 1, axis 2; other kernels are skipped
    path = str(tmp_path / "trace.csv")
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    gemm = "sfac::(anonymous namespace)::exact_gemm(double const*, double const*, double*, int, int, int)"
    nl = "sfac::(anonymous namespace)::exact_nl(double*, double const*, long long, double, int)"
    rows = [(nl, 0, 500), (gemm, 1000, 3000), (gemm, 3000, 7000), (nl, 7000, 7500),
            (gemm, 9000, 13000), (gemm, 13000, 19000), (PASS, 20000, 21000)]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))
    a1, a2 = P.exact_axis_means(path, [100, 50])
    assert a1["dispatches"] == a2["dispatches"] == 2
    assert a1["mean_us"] == pytest.approx(3.0) and a2["mean_us"] == pytest.approx(5.0)
    assert a1["tflops"] == pytest.approx(2 * 100 * 5000 / 3e-6 / 1e12)
    assert a2["tflops"] == pytest.approx(2 * 50 * 5000 / 5e-6 / 1e12)


def test_exact_traffic_attribution(tmp_path):
    # a 2D run with both the pass kernels and the one-level products: each kind is attributed on
    # its own, and neither counts as the copy probe
    gemm = "void sfac::(anonymous namespace)::exact_gemm<1, 32>(double const*, double const*, double*)"
    fetch = [(1, PASS, "FETCH_SIZE", 100.0), (2, PASS, "FETCH_SIZE", 200.0),
             (3, gemm, "FETCH_SIZE", 50.0), (3, gemm, "FETCH_SIZE", 50.0), (4, gemm, "FETCH_SIZE", 300.0),
             (5, gemm, "FETCH_SIZE", 110.0), (6, gemm, "FETCH_SIZE", 290.0)]
    write = [(1, PASS, "WRITE_SIZE", 10.0), (2, PASS, "WRITE_SIZE", 20.0),
             (3, gemm, "WRITE_SIZE", 30.0), (4, gemm, "WRITE_SIZE", 40.0),
             (5, gemm, "WRITE_SIZE", 30.0), (6, gemm, "WRITE_SIZE", 40.0)]
    copy_bytes = 1 << 20
    cf = [(i, COPY, "FETCH_SIZE", copy_bytes / 1024) for i in range(1, 21)] + [(21, gemm, "FETCH_SIZE", 1e9)]
    cw = [(i, COPY, "WRITE_SIZE", copy_bytes / 1024) for i in range(1, 21)] + [(21, gemm, "WRITE_SIZE", 1e9)]
    paths = {}
    for key, rows in (("f", fetch), ("w", write), ("cf", cf), ("cw", cw)):
        paths[key] = str(tmp_path / f"{key}.csv")
        _write_pmc(paths[key], rows)
    ex = P.traffic_from_pmc(paths["f"], paths["w"], paths["cf"], paths["cw"], copy_bytes, 2, tags=P.EXACT_KERNEL_TAGS)
    assert ex["fetch_scale"] == pytest.approx(1.0) and ex["write_scale"] == pytest.approx(1.0)
    a1, a2 = ex["per_axis"]
    assert a1["fetch_kib_raw"] == 105.0 and a2["fetch_kib_raw"] == 295.0
    assert a1["write_kib_raw"] == 30.0 and a2["write_kib_raw"] == 40.0
    assert a1["kernel"] == "exact_gemm<1, 32>"
    ps = P.traffic_from_pmc(paths["f"], paths["w"], paths["cf"], paths["cw"], copy_bytes, 2)
    assert ps["per_axis"] == []           # pass dispatches outside the timed blocks are not attributed


def test_mfma_markdown(tmp_path):
    # one 2D run with two product dispatches per axis (rows per XCD summed) and a pass kernel in
    # between that is not counted; one 3D run absent from the summary's other table is not needed
    gemm = "void sfac::(anonymous namespace)::exact_gemm<1, 32>(double const*)"
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for d, (t0, t1) in enumerate([(0, 10000), (20000, 30000), (40000, 50000), (60000, 70000)], start=1):
        rows += [(d, gemm, "SQ_INSTS_VALU_MFMA_F64", 500.0, t0, t1), (d, gemm, "SQ_INSTS_VALU_MFMA_F64", 500.0, t0, t1),
                 (d, gemm, "SQ_VALU_MFMA_BUSY_CYCLES", 64000.0, t0, t1), (d, gemm, "SQ_WAVES", 64.0, t0, t1)]
    rows.append((9, PASS, "SQ_INSTS_VALU_MFMA_F64", 1e9, 0, 1))
    for w in ("large_2d_1023", "large_3d_255"):
        os.makedirs(tmp_path / w)
        with open(tmp_path / w / "run_counter_collection.csv", "w", newline="") as f:
            wr = csv.DictWriter(f, fieldnames=fields)
            wr.writeheader()
            for r in rows:
                wr.writerow(dict(zip(fields, r)))
    md = P.mfma_markdown(str(tmp_path), [("large_2d_1023", 2)])
    line = [l for l in md.splitlines() if l.startswith("| large_2d_1023 | 1 |")][0]
    cells = [c.strip() for c in line.split("|")]
    assert cells[5] == "1000" and cells[6] == "64.0" and cells[7] == "10.00"
    # busy share: 64000 / (1024 SIMDs x 10 us x 2400 cycles per us)
    assert float(cells[8]) == pytest.approx(64000 / (1024 * 10 * 2400), abs=1e-3)
