"""CPU: the rocprofv3 summariser behind the committed counter and trace
summaries (and so behind the bench line's `traffic`): kernel-name parsing,
the copy calibration of FETCH_SIZE / WRITE_SIZE, the grouping of the mixed
memory-pattern probe's dispatches, kernel-trace statistics and the files
written, on small synthetic rocprofv3 outputs."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1712_09494_amd import profile_summary as ps  # noqa: E402

COPY_BYTES = float(1 << 29)


def write_pmc(d, rows):
    """rows: (dispatch id, kernel name, counter, value)."""
    os.makedirs(os.path.join(d, "box"), exist_ok=True)
    with open(os.path.join(d, "box", "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Agent_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (disp, name, cname, val) in enumerate(rows):
            w.writerow([i, disp, 1, name, cname, val])


def write_trace(d, rows):
    """rows: (name, calls, total ns, min ns, max ns)."""
    os.makedirs(os.path.join(d, "box"), exist_ok=True)
    with open(os.path.join(d, "box", "run_kernel_stats.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        for name, calls, tot, mn, mx in rows:
            w.writerow([name, calls, tot, tot / calls, 0, mn, mx, 0])


FOP = "void ht::bucketed_fop_kernel<8, 4, 1, false, false>(ht::DevTable, unsigned long const*, unsigned long, " \
      "unsigned char*)"
PROBE = "void ht::cuckoo_probe_kernel<1, false, false>(ht::DevTable, unsigned long const*, unsigned long)"
COPY = "void ht::(anonymous namespace)::probe_copy_kernel(ulong2 const*, ulong2*, unsigned long)"


def mix(same):
    return f"void ht::probe_mix_kernel<{'true' if same else 'false'}>(unsigned long*, unsigned long, unsigned int)"


def test_short_names():
    assert ps.short_name(FOP) == "bucketed_fop_kernel"
    assert ps.short_name(PROBE) == "cuckoo_probe_kernel"
    assert ps.short_name(COPY) == "probe_copy_kernel"
    assert ps.short_name(mix(True)) == "probe_mix_kernel<true>"
    assert ps.short_name("void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<long>>(int)") \
        == "vectorized_elementwise_kernel"


def test_copy_calibration_scales_each_kernel(tmp_path):
    # the copy reads and writes COPY_BYTES but FETCH_SIZE shows half of it
    # (a 2x factor) and WRITE_SIZE all of it; a kernel's bytes follow
    half_kib = COPY_BYTES / 1024 / 2
    write_pmc(str(tmp_path / "p1"), [(1, COPY, "FETCH_SIZE", half_kib), (2, FOP, "FETCH_SIZE", 1000.0),
                                     (3, FOP, "FETCH_SIZE", 3000.0)])
    write_pmc(str(tmp_path / "p2"), [(1, COPY, "WRITE_SIZE", COPY_BYTES / 1024), (2, FOP, "WRITE_SIZE", 500.0),
                                     (3, FOP, "WRITE_SIZE", 700.0)])
    s = ps.summarise(ps.read_pmc([str(tmp_path / "p1"), str(tmp_path / "p2")], 6, ["a", "b"]), COPY_BYTES)
    assert s["fetch_scale"] == pytest.approx(2.0)
    assert s["write_scale"] == pytest.approx(1.0)
    k = s["kernels"]["bucketed_fop_kernel"]
    assert k["dispatches"] == 2
    assert k["hbm_read_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)      # mean of 1000 and 3000 KiB, x 2
    assert k["hbm_write_bytes"] == pytest.approx(600.0 * 1024)
    assert k["hbm_bytes"] == pytest.approx(2000.0 * 1024 * 2.0 + 600.0 * 1024)
    cal = s["kernels"]["probe_copy_kernel"]
    assert cal["hbm_read_bytes"] == pytest.approx(COPY_BYTES)
    assert cal["hbm_write_bytes"] == pytest.approx(COPY_BYTES)


def test_no_calibration_gives_no_bytes(tmp_path):
    write_pmc(str(tmp_path / "p"), [(1, FOP, "FETCH_SIZE", 10.0), (1, FOP, "WRITE_SIZE", 5.0)])
    s = ps.summarise(ps.read_pmc([str(tmp_path / "p")], 6, []), COPY_BYTES)
    assert s["fetch_scale"] is None and s["write_scale"] is None
    assert "hbm_bytes" not in s["kernels"]["bucketed_fop_kernel"]


def test_mix_dispatches_grouped_per_compared_kernel(tmp_path):
    # 12 dispatches of each form: the first 6 belong to the first kernel
    # named, the next 6 to the second; a dispatch with several counters
    # (several rows) counts once
    rows = []
    for i in range(12):
        for same in (False, True):
            disp = 100 + 2 * i + int(same)
            rows.append((disp, mix(same), "TCC_HIT_sum", float(i)))
            rows.append((disp, mix(same), "TCC_MISS_sum", 10.0))
    write_pmc(str(tmp_path / "p"), rows)
    pmc = ps.read_pmc([str(tmp_path / "p")], 6, ["bucketed_fop", "cuckoo_probe"])
    assert set(pmc) == {f"probe_mix[{f},{k}]" for f in ("same_line", "other_line")
                        for k in ("bucketed_fop", "cuckoo_probe")}
    s = ps.summarise(pmc, COPY_BYTES)["kernels"]
    assert s["probe_mix[same_line,bucketed_fop]"]["TCC_HIT_sum"] == pytest.approx(2.5)    # mean of 0..5
    assert s["probe_mix[other_line,cuckoo_probe]"]["TCC_HIT_sum"] == pytest.approx(8.5)  # mean of 6..11
    assert s["probe_mix[same_line,cuckoo_probe]"]["l2_hit_rate"] == pytest.approx(8.5 / 18.5)


def test_trace_statistics_merge_instances(tmp_path):
    write_trace(str(tmp_path / "kt"), [(FOP, 10, 500_000.0, 40_000.0, 60_000.0),
                                       (FOP.replace("<8,", "<16,"), 10, 700_000.0, 50_000.0, 90_000.0),
                                       (PROBE, 20, 800_000.0, 30_000.0, 45_000.0)])
    st = ps.read_trace(str(tmp_path / "kt"))
    fop = st["bucketed_fop_kernel"]
    assert fop["calls"] == 20
    assert fop["avg_us"] == pytest.approx(60.0)          # 1.2 ms over 20 calls
    assert fop["min_ns"] == 40_000.0 and fop["max_ns"] == 90_000.0
    assert fop["share"] == pytest.approx(1.2 / 2.0)
    assert st["cuckoo_probe_kernel"]["avg_us"] == pytest.approx(40.0)


def test_command_line_writes_summaries_with_source_hash(tmp_path):
    half_kib = COPY_BYTES / 1024 / 2
    write_pmc(str(tmp_path / "p1"), [(1, COPY, "FETCH_SIZE", half_kib), (2, PROBE, "FETCH_SIZE", 100_000.0)])
    write_pmc(str(tmp_path / "p2"), [(1, COPY, "WRITE_SIZE", COPY_BYTES / 1024), (2, PROBE, "WRITE_SIZE", 50_000.0)])
    write_trace(str(tmp_path / "kt"), [(PROBE, 4, 240_000.0, 55_000.0, 65_000.0)])
    (tmp_path / "cmds.txt").write_text("rocprofv3 --pmc FETCH_SIZE -- prog\nrocprofv3 --pmc WRITE_SIZE -- prog\n")
    out = tmp_path / "out"
    out.mkdir()
    subprocess.run([sys.executable, "-m", "paper_1712_09494_amd.profile_summary", "--workload", "unit_case",
                    "--pmc", str(tmp_path / "p1"), str(tmp_path / "p2"), "--trace", str(tmp_path / "kt"),
                    "--commands-file", str(tmp_path / "cmds.txt"), "--outdir", str(out)], cwd=ROOT, check=True)
    res = json.loads((out / "counters_unit_case.json").read_text())
    assert res["kernel_source_sha256"] == ps.source_hash()
    assert res["commands"][0].startswith("rocprofv3 --pmc FETCH_SIZE")
    k = res["kernels"]["cuckoo_probe_kernel"]
    assert k["hbm_bytes"] == pytest.approx(100_000.0 * 1024 * 2 + 50_000.0 * 1024)
    md = (out / "counters_unit_case.md").read_text()
    assert "| cuckoo_probe_kernel | 1 | 204.80 | 51.20 |" in md
    assert ps.source_hash() in md
    trace_md = [p for p in os.listdir(out) if p.startswith("kernel_trace_")]
    assert trace_md == ["kernel_trace_unit_case.md"]
    assert "| cuckoo_probe_kernel | 4 | 60.00 |" in (out / trace_md[0]).read_text()
