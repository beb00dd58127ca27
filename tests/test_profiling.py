"""Host logic of the profiling helpers: counter scaling by the copy probe,
the recorded launch shape, and the kernel-trace table (synthetic CSV files
in the layout rocprofv3 writes)."""

import csv

import pytest

from paper_2307_06305_amd import profiling as P


def _counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def _fake_runs(tmp_path, g_da=2, g_csr=2):
    da = P.kernel_name("da", f"stream_g{g_da}_t4096")
    cs = P.kernel_name("csr", f"stream_g{g_csr}_t2048")
    copy = "damn::kern::stream_copy(...)"
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    # the copy of 1 MiB reads as 512 KiB on FETCH_SIZE and 1024 KiB on WRITE_SIZE
    _counters(f, "FETCH_SIZE", [(copy, 512.0), (da, 300.0), (da, 302.0), (cs, 400.0)])
    _counters(w, "WRITE_SIZE", [(copy, 1024.0), (da, 16.0), (da, 16.0), (cs, 16.0)])
    return f, w


def test_kernel_names_follow_the_launch():
    assert P.stream_launch("stream_g4_t1024") == (4, 1024, 1)
    assert P.stream_launch("paired_g8_t2048") == (8, 2048, 2)
    assert P.kernel_name("da", "stream_g4_t1024") == \
        "spmv_stream<short, double, true, 4, false, double, 2, 1>"
    assert P.kernel_name("csr", "stream_g1_t2048") == \
        "spmv_stream<int, double, false, 1, false, double, 2, 1>"
    assert P.kernel_name("da", "paired_g4_t2048") == \
        "spmv_stream<short, double, true, 4, false, double, 2, 2>"
    for bad in ("vector_l4_u2", "pairs_g4_t2048"):
        with pytest.raises(ValueError):
            P.stream_launch(bad)


def test_summary_scales_by_the_copy_probe(tmp_path):
    f, w = _fake_runs(tmp_path)
    s = P.summarize(str(f), str(w), 1 << 20, "stream_g2_t4096", "stream_g2_t2048")
    assert s["fetch_scale"] == pytest.approx(0.5) and s["write_scale"] == pytest.approx(1.0)
    da = s["kernels"]["da"]
    assert da["launch"] == "stream_g2_t4096" and da["dispatches"] == [2, 2]
    # mean of the two dispatches, KiB -> bytes, divided by the probe's factor
    assert da["hbm_read_bytes"] == pytest.approx(301.0 * 1024 / 0.5)
    assert da["hbm_bytes"] == pytest.approx(301.0 * 2048 + 16.0 * 1024)
    assert s["kernels"]["csr"]["hbm_bytes"] == pytest.approx(400.0 * 2048 + 16.0 * 1024)


def test_recorded_traffic_needs_the_same_launch_and_sources(tmp_path):
    f, w = _fake_runs(tmp_path)
    s = P.summarize(str(f), str(w), 1 << 20)
    out = tmp_path / "traffic.md"
    P.write_summary(s, str(out), "rocprofv3 ...")
    want = 301.0 * 2048 + 16.0 * 1024
    assert P.read_traffic(str(out), "da") == pytest.approx(want)
    assert P.read_traffic(str(out), "da", launch=P.DA_LAUNCH) == pytest.approx(want)
    assert P.read_traffic(str(out), "da", launch="stream_g4_t4096") is None
    # a summary taken from other kernel sources is not used
    text = out.read_text().replace(s["source_sha256"], "0" * 64)
    out.write_text(text)
    assert P.read_traffic(str(out), "da") is None
    assert P.read_traffic(str(tmp_path / "missing.md"), "da") is None


def test_missing_kernel_is_an_error(tmp_path):
    f, w = _fake_runs(tmp_path, g_da=4)
    with pytest.raises(KeyError):
        P.summarize(str(f), str(w), 1 << 20, "stream_g2_t4096")


def test_trace_table_orders_by_total_time(tmp_path):
    path = tmp_path / "stats.csv"
    cols = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"]
    rows = [("void a_kernel(int)", 10, 1000, 100, 10.0, 90, 110),
            ("void b_kernel(int)", 2, 8000, 4000, 80.0, 3900, 4100),
            ("c_kernel", 5, 1000, 200, 10.0, 150, 250)]
    with open(path, "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(cols)
        wr.writerows(rows)
    st = P.kernel_stats(str(path))
    assert [r[0] for r in st][:1] == ["b_kernel"]
    assert st[0][1:3] == (2, 4.0)
    assert [r[0] for r in P.kernel_stats(str(path), ["c_"])] == ["c_kernel"]
    out = tmp_path / "trace.md"
    P.write_trace_summary(str(path), str(out), "title", "cmd", "notes")
    text = out.read_text()
    assert "| `b_kernel` | 2 | 4.0 |" in text


def test_source_hash_ignores_comments_only():
    a = "int f(int x) {  // twice\n  return 2 * x; /* note */\n}\n"
    b = "// header\nint f(int x) {\n  return 2 * x;\n}\n"
    c = "int f(int x) {\n  return 3 * x;\n}\n"
    assert P._code_only(a) == P._code_only(b)
    assert P._code_only(a) != P._code_only(c)


def test_counter_table_keeps_workloads_apart(tmp_path):
    """Means per dispatch by counter, one column per workload and kernel:
    the same kernel symbol in two workloads stays two columns."""
    k = "void damn::kern::spmv_stream<int, double, false, 4, false, double, 2, 1>(args)"
    a1, a2, b1 = tmp_path / "a1.csv", tmp_path / "a2.csv", tmp_path / "b1.csv"
    _counters(a1, "TCC_HIT_sum", [(k, 10.0), (k, 20.0), ("other(x)", 5.0)])
    _counters(a2, "TCC_MISS_sum", [(k, 4.0)])
    _counters(b1, "TCC_HIT_sum", [(k, 100.0)])
    m = P.counter_means([str(a1), str(a2)])
    name = "damn::kern::spmv_stream<int, double, false, 4, false, double, 2, 1>"
    assert m[name] == {"TCC_HIT_sum": 15.0, "TCC_MISS_sum": 4.0}
    out = tmp_path / "c.md"
    P.write_counter_summary([f"wl-a={a1},{a2}", f"wl-b={b1}"], str(out), "t", "cmd", "",
                            ["spmv_stream"])
    text = out.read_text()
    assert "wl-a: `" in text and "wl-b: `" in text and "other" not in text
    row = [ln for ln in text.splitlines() if ln.startswith("| TCC_HIT_sum |")][0]
    assert row == "| TCC_HIT_sum | 15 | 100 |"


def test_dispatch_groups_split_by_grid(tmp_path):
    """Launches of one kernel with different grids (the read probe's one-pass
    and many-pass launches) are averaged apart; durations in microseconds."""
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size_X", "Start_Timestamp",
                                          "End_Timestamp"])
        w.writeheader()
        for grid, dur in ((256, 10_000), (256, 12_000), (4096, 150_000), (4096, 148_000)):
            w.writerow({"Kernel_Name": "void damn::kern::stream_lds<2>(args)",
                        "Grid_Size_X": grid, "Start_Timestamp": 1000, "End_Timestamp": 1000 + dur})
        w.writerow({"Kernel_Name": "other(x)", "Grid_Size_X": 1, "Start_Timestamp": 0,
                    "End_Timestamp": 5})
    g = P.dispatch_groups(str(path), ["stream_lds"])
    assert g == [("damn::kern::stream_lds<2>", 256, 2, 11.0, 10.0),
                 ("damn::kern::stream_lds<2>", 4096, 2, 149.0, 148.0)]
