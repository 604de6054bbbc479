"""The profile-summary tool behind profiles/: kernel-name normalisation, the
kernel-time table, and the traffic record's calibration against the
reference copy (synthetic rocprofv3-style CSV files; no GPU)."""
import csv
import json

from paper_1505_08019_amd import prof

PASS = "void fft2::pass_kernel<0, 10, 2, 3, false>(fft2::PassArgs)"
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float>, std::array<char*, 3ul> >(int)"


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_normalise():
    assert prof.normalise(PASS) == "pass_kernel<0,10,2,3,false>"
    assert prof.normalise("fft2::split_pass1<2, 1>(fft2::SplitArgs)") == "split_pass1<2,1>"


def test_stats_table_lists_focus_first(tmp_path):
    fields = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"]
    rows = [{"Name": "big_kernel(int)", "Calls": 10, "TotalDurationNs": 9e6, "AverageNs": 9e5, "Percentage": 90,
             "MinNs": 8e5, "MaxNs": 1e6},
            {"Name": PASS, "Calls": 100, "TotalDurationNs": 7e5, "AverageNs": 7e3, "Percentage": 7, "MinNs": 5e3,
             "MaxNs": 9e3}]
    src = tmp_path / "stats.csv"
    _write(src, fields, rows)
    text = prof.stats_md(str(src), str(tmp_path / "k.md"), "cmd --x", focus=("pass_kernel<0,10,2,3,false>",))
    body = [l for l in text.splitlines() if l.startswith("| `")]
    assert body[0].startswith("| `pass_kernel<0,10,2,3,false>` | 100 | 7.00 |")
    assert body[1].startswith("| `big_kernel` | 10 | 900.00 |")
    assert "    cmd --x" in text


def test_traffic_scales_by_the_reference_copy(tmp_path):
    """The copy reads and writes COPY_BYTES once; whatever each counter reads
    for it sets that counter's scale, applied to every other kernel."""
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    copy_kib = prof.COPY_BYTES / 1024.0
    fetch = [{"Kernel_Name": COPY, "Counter_Name": "FETCH_SIZE", "Counter_Value": copy_kib / 2},  # reads half
             {"Kernel_Name": PASS, "Counter_Name": "FETCH_SIZE", "Counter_Value": 4096.0},
             {"Kernel_Name": PASS, "Counter_Name": "FETCH_SIZE", "Counter_Value": 4104.0}]
    write = [{"Kernel_Name": COPY, "Counter_Name": "WRITE_SIZE", "Counter_Value": copy_kib},
             {"Kernel_Name": PASS, "Counter_Name": "WRITE_SIZE", "Counter_Value": 8192.0},
             {"Kernel_Name": PASS, "Counter_Name": "WRITE_SIZE", "Counter_Value": 8192.0}]
    _write(tmp_path / "f.csv", fields, fetch)
    _write(tmp_path / "w.csv", fields, write)
    rec = prof.traffic_json(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "t.json"), "cmd")
    assert rec["copy_reference"]["fetch_scale"] == 2.0 and rec["copy_reference"]["write_scale"] == 1.0
    k = rec["kernels"]["pass_kernel<0,10,2,3,false>"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == int(4100.0 * 1024 * 2) and k["write_bytes"] == 8192 * 1024
    assert k["hbm_bytes_per_launch"] == k["fetch_bytes"] + k["write_bytes"]
    assert rec["source_hash"] == prof.kernel_source_hash()
    assert json.load(open(tmp_path / "t.json"))["kernels"] == rec["kernels"]



def test_sq_table_ratios(tmp_path):
    """Per-dispatch averages of each SQ counter, and the activity counters as
    fractions of SQ_WAVE_CYCLES."""
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = []
    for v in (1000.0, 3000.0):  # two dispatches: wave cycles average 2000
        rows.append({"Kernel_Name": PASS, "Counter_Name": "SQ_WAVE_CYCLES", "Counter_Value": v})
    for c, v in (("SQ_ACTIVE_INST_VALU", 500.0), ("SQ_WAIT_INST_ANY", 1000.0), ("SQ_INSTS_VALU", 2e6)):
        rows += [{"Kernel_Name": PASS, "Counter_Name": c, "Counter_Value": v}] * 2
    _write(tmp_path / "sq.csv", fields, rows)
    text = prof.sq_md(str(tmp_path / "sq.csv"), str(tmp_path / "sq.md"), "cmd --y", "test")
    body = [l for l in text.splitlines() if l.startswith("| `")]
    assert len(body) == 1
    cells = [c.strip() for c in body[0].strip("|").split("|")]
    head = [l for l in text.splitlines() if l.startswith("| kernel")][0]
    cols = [c.strip() for c in head.strip("|").split("|")]
    got = dict(zip(cols, cells))
    assert got["dispatches"] == "2" and got["SQ_WAVE_CYCLES"] == "2000" and got["SQ_INSTS_VALU"] == "2M"
    assert got["active VALU / wave cycles"] == "0.25" and got["wait / wave cycles"] == "0.50"
    assert "    cmd --y" in text
