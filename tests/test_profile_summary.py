"""Host logic of the rocprofv3 summary: marker windows, evaluation split, span
alignment, copy calibration and the derived busy fractions, on synthetic
CSVs of known content."""
import csv
import json

import pytest

from paper_2303_08169_amd import profile_summary as ps

SPANS = ["neighbor_check_rebuild", "edge_list", "geometry", "fwd.latent1.0", "tp_fwd1", "forces"]
# one evaluation: the spans' kernels, edge_list and forces launching two kernels each
EVAL = [("nq::(anonymous namespace)::k_displacement(double const*)", 1.0),
        ("nq::(anonymous namespace)::k_edge_count(double const*)", 2.0),
        ("nq::(anonymous namespace)::k_scan_block(int const*)", 3.0),
        ("nq::(anonymous namespace)::k_geometry(int)", 4.0),
        ("void nq::(anonymous namespace)::k_gemm_ws<2, 3, 8>(nq::A)", 50.0),
        ("void nq::(anonymous namespace)::k_tp_fwd<2, 2, true>(nq::T)", 6.0),
        ("nq::(anonymous namespace)::k_forces(long)", 7.0),
        ("nq::(anonymous namespace)::k_total_energy(long)", 8.0)]
PRE = [("nq::(anonymous namespace)::k_gemm<2, 1>(x)", 99.0),     # autotuning before the window
       ("at::native::spin_kernel(long)", 0.0)]
POST = [("at::native::spin_kernel(long)", 0.0), ("__amd_rocclr_copyBuffer", 5.0)]


def _counter_csv(path, counter, evals, scale=1.0):
    seq = PRE + EVAL * evals + POST
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, v) in enumerate(seq):
            # two rows per dispatch (e.g. two XCDs) that the reader adds up
            w.writerow([i + 1, name, counter, v * scale / 2])
            w.writerow([i + 1, name, counter, v * scale / 2])


def _trace_csv(path, evals):
    seq = PRE + EVAL * evals + POST
    t = 1000
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Correlation_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, (name, v) in enumerate(seq):
            w.writerow([i + 1, name, t, t + int(v * 1000)])
            t += int(v * 1000) + 10


def _copy_csv(path, counter, kib):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerow([1, "at::native::fill_kernel", counter, 3.0])
        w.writerow([2, "__amd_rocclr_copyBuffer", counter, kib])
        w.writerow([3, "__amd_rocclr_copyBuffer", counter, kib])


def _setup(tmp_path, evals=3):
    spans = tmp_path / "spans.json"
    spans.write_text(json.dumps({"workload": "w", "precision": "bf16x3", "path": "layered", "evals": evals,
                                 "edges": 100, "spans": SPANS, "span_counts": [evals] * len(SPANS),
                                 "source_sha256": "abc"}))
    _trace_csv(tmp_path / "trace.csv", evals)
    _counter_csv(tmp_path / "fetch.csv", "FETCH_SIZE", evals)
    _counter_csv(tmp_path / "write.csv", "WRITE_SIZE", evals, scale=2.0)
    _copy_csv(tmp_path / "cf.csv", "FETCH_SIZE", 512.0)     # a 1 MiB copy read as half
    _copy_csv(tmp_path / "cw.csv", "WRITE_SIZE", 1024.0)
    return spans


def test_spans_counters_and_calibration(tmp_path):
    spans = _setup(tmp_path)
    out = tmp_path / "out.json"
    ps.main(["--spans", str(spans), "--trace", str(tmp_path / "trace.csv"), "--fetch", str(tmp_path / "fetch.csv"),
             "--write", str(tmp_path / "write.csv"), "--copy-fetch", str(tmp_path / "cf.csv"),
             "--copy-write", str(tmp_path / "cw.csv"), "--copy-bytes", str(1 << 20),
             "--json", str(out), "--md", str(tmp_path / "out.md")])
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    s = rec["spans"]
    # edge_list owns k_edge_count and k_scan_block; forces owns k_forces and k_total_energy
    assert s["edge_list"]["kernels"] == ["k_edge_count", "k_scan_block"]
    assert s["forces"]["kernels"] == ["k_forces", "k_total_energy"]
    assert s["edge_list"]["fetch_kib"] == pytest.approx(5.0)
    assert s["fwd.latent1.0"]["avg_ms_trace"] == pytest.approx(50.0 * 1e-3)
    # bytes: 1024 * (FETCH * 2 + WRITE * 1); WRITE was recorded at twice the FETCH values
    assert s["fwd.latent1.0"]["hbm_bytes_per_launch"] == pytest.approx(1024 * (50 * 2 + 100))
    per_eval = sum(v for _, v in EVAL)
    assert rec["hbm_bytes_per_step"] == pytest.approx(1024 * (per_eval * 2 + 2 * per_eval))
    assert "fwd.latent1.0" in (tmp_path / "out.md").read_text()


def test_sq_fractions(tmp_path):
    spans = _setup(tmp_path, evals=2)
    sq = tmp_path / "sq.csv"
    with open(sq, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        seq = PRE + EVAL * 2 + POST
        for i, (name, v) in enumerate(seq):
            # 8 XCDs x 1000 cycles; MFMA busy on a quarter of 1024 SIMDs for the whole kernel
            w.writerow([i + 1, name, "GRBM_GUI_ACTIVE", 8000.0])
            w.writerow([i + 1, name, "SQ_VALU_MFMA_BUSY_CYCLES", 256 * 1000.0])
            w.writerow([i + 1, name, "SQ_ACTIVE_INST_VALU", 128 * 1000.0])
            w.writerow([i + 1, name, "SQ_WAIT_INST_ANY", 30.0])
            w.writerow([i + 1, name, "SQ_WAVE_CYCLES", 100.0])
    agent = tmp_path / "agent.csv"
    agent.write_text("Name,Simd_Count,Cu_Count,Num_Xcc\ngfx950,1024,256,8\n")
    out = tmp_path / "o.json"
    ps.main(["--spans", str(spans), "--trace", str(tmp_path / "trace.csv"), "--sq", str(sq), "--agent", str(agent),
             "--json", str(out), "--md", str(tmp_path / "o.md")])
    r = json.loads(out.read_text())["spans"]["tp_fwd1"]
    assert r["mfma_busy"] == pytest.approx(0.25)
    assert r["valu_busy"] == pytest.approx(0.5)
    assert r["wait_any"] == pytest.approx(0.3)


def test_missing_marker_or_wrong_count_is_an_error(tmp_path):
    spans = _setup(tmp_path, evals=3)
    d = json.loads(spans.read_text())
    d["evals"] = 4
    d["span_counts"] = [4] * len(SPANS)
    spans.write_text(json.dumps(d))
    with pytest.raises(ValueError, match="expected 4"):
        ps.main(["--spans", str(spans), "--trace", str(tmp_path / "trace.csv"), "--json", str(tmp_path / "x.json"),
                 "--md", str(tmp_path / "x.md")])


def test_chunked_evaluations_are_keyed_by_kernel(tmp_path):
    spans = _setup(tmp_path, evals=3)
    d = json.loads(spans.read_text())
    d["span_counts"][3] = 6    # a span that runs twice per evaluation (two centre chunks)
    spans.write_text(json.dumps(d))
    out = tmp_path / "k.json"
    ps.main(["--spans", str(spans), "--trace", str(tmp_path / "trace.csv"), "--fetch", str(tmp_path / "fetch.csv"),
             "--write", str(tmp_path / "write.csv"), "--copy-fetch", str(tmp_path / "cf.csv"),
             "--copy-write", str(tmp_path / "cw.csv"), "--copy-bytes", str(1 << 20),
             "--json", str(out), "--md", str(tmp_path / "k.md")])
    rec = json.loads(out.read_text())
    assert rec["keyed_by"] == "kernel" and "spans" not in rec
    k = rec["kernels"]
    assert set(k) == {"k_displacement", "k_edge_count", "k_scan_block", "k_geometry", "k_gemm_ws", "k_tp_fwd",
                      "k_forces", "k_total_energy"}
    assert k["k_gemm_ws"]["launches_per_eval"] == 1 and k["k_gemm_ws"]["avg_ms_trace"] == pytest.approx(0.05)
    assert k["k_gemm_ws"]["hbm_bytes_per_launch"] == pytest.approx(1024 * (50 * 2 + 100))
    per_eval = sum(v for _, v in EVAL)
    assert rec["hbm_bytes_per_step"] == pytest.approx(1024 * (per_eval * 2 + 2 * per_eval))


def test_span_kernel_names():
    assert ps.span_kernels("fwd.twobody") == ("k_tb_fwd",)
    assert ps.span_kernels("bwd.twobody") == ("k_tb_bwd",)
    assert ps.span_kernels("fwd.twobody.0") == ("k_gemm", "k_gemm_ws")
    assert ps.span_kernels("tp_bwd1") == ("k_tp_bwd", "k_tp_bwd_last32")
    with pytest.raises(ValueError):
        ps.span_kernels("no_such_span")
