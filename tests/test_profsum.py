"""CPU tests of the rocprofv3 summary helper: counter scaling by the calibration copy and the
rule that measured traffic is reported only for unchanged kernel sources."""
import csv

from paper_2603_11531_amd import profsum

FIELDS = ["Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_pmc_scales_by_the_copy_and_sums_kernels(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # the copy of 1 MiB reads back half its bytes on FETCH_SIZE and all of them on WRITE_SIZE
    _csv(fetch, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0), ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 1.0),
                 ("k_a<x>", "FETCH_SIZE", 100.0), ("k_a<x>", "FETCH_SIZE", 300.0), ("k_b", "FETCH_SIZE", 10.0)])
    _csv(write, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0), ("k_a<x>", "WRITE_SIZE", 50.0),
                 ("k_b", "WRITE_SIZE", 4.0)])
    text = profsum.pmc(str(fetch), str(write), None, ["k_a", "k_b"], 1.0, "cmd")
    kv = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith(" "))
    # k_a: fetch mean 200 KiB x 2 + write 50 KiB; k_b: 10 x 2 + 4
    assert float(kv["traffic_bytes_per_launch"]) == (400 + 50 + 20 + 4) * 1024.0
    assert kv["source_sha256"] == profsum.source_hash()


def test_traffic_is_dropped_when_sources_change(tmp_path):
    p = tmp_path / "s.txt"
    p.write_text(f"source_sha256: {profsum.source_hash()}\ntraffic_bytes_per_launch: 1234\n")
    assert profsum.read_traffic(str(p)) == 1234.0
    p.write_text("source_sha256: 0000000000000000\ntraffic_bytes_per_launch: 1234\n")
    assert profsum.read_traffic(str(p)) is None
    assert profsum.read_traffic(str(tmp_path / "missing.txt")) is None


def test_summary_counters_are_parsed_back(tmp_path):
    p = tmp_path / "s.txt"
    p.write_text(f"source_sha256: {profsum.source_hash(profsum.SOURCES['bin'])}\ntraffic_bytes_per_launch: 10\n\n"
                 "SQ / GRBM counters per dispatch (mean over dispatches):\n"
                 "  chunk_write_kernel     SQ_INSTS_VALU                    123.0\n"
                 "  chunk_write_kernel     GRBM_GUI_ACTIVE                  800.0\n")
    traffic, sq = profsum.read_summary(str(p), profsum.SOURCES["bin"])
    assert traffic == 10.0
    assert sq == {("chunk_write_kernel", "SQ_INSTS_VALU"): 123.0, ("chunk_write_kernel", "GRBM_GUI_ACTIVE"): 800.0}
    assert profsum.read_summary(str(p), profsum.SOURCES["blend"]) is None
