"""Host-side helpers of bench.py: the kernel-source hash that keys the committed counter summaries
ignores comments and layout but not code, and the counter ingest reads rocprofv3's CSV layout."""
import csv
import json
import os

import bench


def test_code_hash_ignores_comments_and_layout(tmp_path):
    a = tmp_path / "a.hip"
    a.write_text('int f(int x) {  // add one\n    return x + 1; /* block\ncomment */ }\nconst char* s = "// kept";\n')
    b = tmp_path / "b.hip"
    b.write_text('int f(int x) { return x + 1; }\n\n// another comment\nconst char* s = "// kept";\n')
    c = tmp_path / "c.hip"
    c.write_text('int f(int x) { return x + 2; }\nconst char* s = "// kept";\n')
    d = tmp_path / "d.hip"
    d.write_text('int f(int x) { return x + 1; }\nconst char* s = "// changed";\n')
    h = lambda p: bench.kernel_source_hash([str(p)])
    assert h(a) == h(b)
    assert h(a) != h(c)
    assert h(a) != h(d)


def test_ingest_counters_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    # one pass directory per counter, rows as rocprofv3 --pmc -f csv writes them
    fields = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = {"FETCH_SIZE": [("k_sweep_fused2q<true, true>", 1000.0), ("k_sweep_fused2q<true, true>", 1200.0),
                           ("direct_copy_kernel_cuda", 131072.0)],
            "WRITE_SIZE": [("k_sweep_fused2q<true, true>", 2000.0), ("k_sweep_fused2q<true, true>", 2000.0),
                           ("direct_copy_kernel_cuda", 262144.0)]}
    dirs = []
    for counter, entries in rows.items():
        d = tmp_path / counter
        d.mkdir()
        with open(d / "pmc_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=fields)
            w.writeheader()
            for i, (k, v) in enumerate(entries):
                w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": counter,
                            "Counter_Value": v})
        dirs.append(str(d))
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    e = bench.ingest_counters("fused_L16384", "fused", 16384, dirs, "k_sweep_fused2q<true", None, 1 << 28, "cmd")
    # a 2^28-byte copy reads 131072 KiB in FETCH_SIZE: the read counter is scaled x2, writes x1
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["fetch_kib_raw"] == 1100.0 and e["write_kib_raw"] == 2000.0
    assert e["hbm_bytes_per_launch"] == 1024 * (1100 * 2 + 2000)
    assert e["source_hash"] == bench.kernel_source_hash()
    assert json.load(open(out))["fused_L16384"]["command"] == "cmd"
    # the cubic lattice's record is keyed to the hash of its own sources as well, which measured_counters checks
    e3 = bench.ingest_counters("int8_3d_L1024", "int8", 1024, dirs, "k_sweep_fused2q<true", None, 1 << 28, "cmd",
                               2.0 * 1024 ** 3)
    assert e3["source_hash"] == bench.kernel_source_hash(bench.KERNEL_SOURCES_3D)
    assert bench.measured_traffic("int8_3d", 1024) == e3["hbm_bytes_per_launch"]


def test_fused_passes_cover_every_sweep_and_end_in_the_first_buffer():
    # the two-sweep and one-sweep passes alternate between two buffers, so they must come in an even
    # number for the chain to end where it started; an odd count makes its first sweep in place
    assert bench.fused_passes(0) == (0, 0, 0)
    assert bench.fused_passes(1) == (0, 0, 1)
    assert bench.fused_passes(2) == (0, 2, 0)
    assert bench.fused_passes(4) == (2, 0, 0)
    assert bench.fused_passes(7) == (2, 2, 1)
    for n in range(64):
        pairs, singles, in_place = bench.fused_passes(n)
        assert 2 * pairs + singles + in_place == n
        assert (pairs + singles) % 2 == 0 and pairs % 2 == 0 and in_place == n % 2
        assert singles in (0, 2)
