"""Host-side arithmetic of bench.py: the algorithmic byte counts behind
``roofline`` and ``correction_frac``, and the rule that the committed HBM
traffic record is used only while the check kernel's sources are unchanged.
"""
import json
import os
import shutil

import bench


def test_correction_bytes_of_the_512cube_workload():
    # the 512^3 float32 workload as a bench run reports it: n vertices, K
    # critical points, 30 changing iterations, 128 105 269 targets in all
    n, K, its, targets = 512 ** 3, 27_845_957, 30, 128_105_269
    b = 4
    setup = 13 * n                      # read f and g_hat, write g', one code byte
    dense = 30 * (5 * n + n // 8 + 4 * K)
    edits = 14 * targets                # value, count, final-edit count; value, count written
    sort = 4 * 2 * (4 + 4) * K          # four 8-bit passes over (key, slot), read and written
    assert bench.algorithmic_bytes(n, b, K, its, targets) == setup + dense + edits + sort
    assert bench.algorithmic_bytes(n, b, K, its, targets) == 29_297_935_998


def test_check_bytes_per_vertex_formula_is_the_documented_one():
    # (b + 1) + 1/8 + b K / n: a float64 field with no critical points moves
    # 9.125 B per checked vertex, a float32 field whose vertices are all
    # critical 9.125 as well
    assert bench.algorithmic_bytes(8, 8, 0, 1, 0) - bench.algorithmic_bytes(8, 8, 0, 0, 0) == 73
    assert bench.algorithmic_bytes(8, 4, 8, 1, 0) - bench.algorithmic_bytes(8, 4, 8, 0, 0) == 73


def _copy_record(tmp_path):
    with open(bench.TRAFFIC_RECORD) as fh:
        rec = json.load(fh)
    for src in rec["sources"]:
        dst = tmp_path / src
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copyfile(os.path.join(bench.ROOT, src), dst)
    rel = os.path.relpath(bench.TRAFFIC_RECORD, bench.ROOT)
    (tmp_path / rel).parent.mkdir(parents=True, exist_ok=True)
    shutil.copyfile(bench.TRAFFIC_RECORD, tmp_path / rel)
    return rec, str(tmp_path / rel)


def test_traffic_record_is_used_only_for_unchanged_sources(tmp_path, monkeypatch):
    rec, record = _copy_record(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", record)
    # the record's own hash, recomputed over the copied sources
    import hashlib
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update((tmp_path / src).read_bytes())
    if h.hexdigest() == rec["source_sha256"]:
        assert bench.measured_traffic(512) == rec["traffic_bytes_per_launch"]
    assert bench.measured_traffic(256) is None          # another workload
    victim = tmp_path / rec["sources"][0]
    victim.write_bytes(victim.read_bytes() + b"\n")     # any change to a source
    assert bench.measured_traffic(512) is None
    os.remove(record)                                   # no record at all
    assert bench.measured_traffic(512) is None
