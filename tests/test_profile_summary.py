"""rocprofv3 summaries: kernel statistics, per-dispatch counter means and the
traffic record (counter KiB scaled by a calibration kernel), on small
synthetic CSV files in the profiler's column layout."""
import hashlib
import json

from paper_2604_01397_amd import profile_summary as ps

STATS_HEADER = "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs,StdDev\n"
PMC_HEADER = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"


def _write(path, header, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    path.write_text(header + "".join(",".join(str(c) for c in r) + "\n" for r in rows))


def _pmc(tmp_path, name, counter, rows):
    # rows: (dispatch, kernel, value); two hardware instances per dispatch
    out = []
    for d, k, v in rows:
        out.append((d, k, counter, v / 2))
        out.append((d, k, counter, v / 2))
    _write(tmp_path / name / "x_counter_collection.csv", PMC_HEADER, out)
    return str(tmp_path / name)


def test_stats_table(tmp_path, capsys):
    _write(tmp_path / "kt" / "kt_kernel_stats.csv", STATS_HEADER,
           [("k_check", 4, 4000000, 1000000, 80.0, 900000, 1100000, 1),
            ("k_apply", 4, 1000000, 250000, 20.0, 200000, 300000, 1)])
    assert ps.main(["--stats", str(tmp_path / "kt"), "--match", "check"]) == 0
    out = capsys.readouterr().out
    assert "`k_check` | 4 | 4.000 | 1000.00" in out and "k_apply" not in out


def test_counters_sum_instances(tmp_path):
    d = _pmc(tmp_path, "f", "FETCH_SIZE", [(1, "k_check", 100.0), (2, "k_check", 300.0)])
    cs = ps.counters(d)
    assert sorted(cs["k_check"]["FETCH_SIZE"]) == [100.0, 300.0]


def test_traffic_record(tmp_path):
    fetch = _pmc(tmp_path, "fetch", "FETCH_SIZE", [(1, "k_check<float>", 1000.0),
                                                   (2, "k_check<float>", 3000.0),
                                                   (3, "k_apply", 5.0)])
    write = _pmc(tmp_path, "write", "WRITE_SIZE", [(1, "k_check<float>", 10.0),
                                                   (2, "k_check<float>", 30.0)])
    # calibration: a kernel moving 1 MiB each way; FETCH_SIZE reads half of it
    cf = _pmc(tmp_path, "cf", "FETCH_SIZE", [(1, "neg_kernel", 512.0)])
    cw = _pmc(tmp_path, "cw", "WRITE_SIZE", [(1, "neg_kernel", 1024.0)])
    src = tmp_path / "a.hip"
    src.write_text("kernel source")
    rec_path = tmp_path / "rec.txt"
    assert ps.main(["--record", str(rec_path), "--pmc", fetch, write, "--kernel", "k_check",
                    "--cal-kernel", "neg_kernel", "--cal-fetch", cf, "--cal-write", cw,
                    "--cal-bytes", str(1 << 20), "--algo-bytes", "1234", "--workload", "w",
                    "--sources", str(src)]) == 0
    rec = json.loads(rec_path.read_text())
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["dispatches"] == 2
    assert rec["fetch_bytes_per_launch"] == 2000 * 1024 * 2
    assert rec["write_bytes_per_launch"] == 20 * 1024
    assert rec["traffic_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert rec["source_sha256"] == hashlib.sha256(b"kernel source").hexdigest()
    assert rec["algorithmic_bytes_per_launch"] == 1234
