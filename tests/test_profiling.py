"""CPU checks of the profile summarizer used for profiles/ (no GPU): it reads
rocprofv3 CSV output, scales counters by the copy kernel's reading, and the
benchmark's traffic figure is withheld once the walk's sources change."""
import csv
import os

import pytest

from paper_1710_07745_amd import profiling


def write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_scaling(tmp_path, capsys):
    copy = 256 << 20
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    # the copy kernel reads half its bytes on FETCH_SIZE (KiB) and all on WRITE_SIZE
    write_counters(fd, [["__amd_rocclr_copyBuffer", "FETCH_SIZE", copy / 2048],
                        ["k_walk<3>(args)", "FETCH_SIZE", 100.0],
                        ["k_walk<3>(args)", "FETCH_SIZE", 300.0],
                        ["k_walk<3>(args)", "FETCH_SIZE", 200.0]])
    write_counters(wd, [["__amd_rocclr_copyBuffer", "WRITE_SIZE", copy / 1024],
                        ["k_walk<3>(args)", "WRITE_SIZE", 50.0]])
    profiling.main(["traffic", fd, wd, "--kernel", "k_walk<3>", "--copy-bytes", str(copy),
                    "--alg-bytes", "1024"])
    out = dict(ln.split(":", 1) for ln in capsys.readouterr().out.splitlines() if not ln.startswith("#"))
    assert float(out["fetch_scale"]) == pytest.approx(2.0)
    assert float(out["write_scale"]) == pytest.approx(1.0)
    # medians 200 and 50 KiB -> 2 * 200 KiB + 50 KiB
    assert float(out["traffic_bytes_per_launch"]) == pytest.approx((2 * 200 + 50) * 1024)
    assert out["source_sha256"].strip() == profiling.walk_source_hash()


def test_read_traffic_needs_matching_sources(tmp_path):
    p = tmp_path / "t.txt"
    p.write_text(f"source_sha256: {profiling.walk_source_hash()}\ntraffic_bytes_per_launch: 1234\n")
    assert profiling.read_traffic(str(p)) == 1234.0
    p.write_text("source_sha256: deadbeef\ntraffic_bytes_per_launch: 1234\n")
    assert profiling.read_traffic(str(p)) is None
    assert profiling.read_traffic(str(tmp_path / "missing.txt")) is None


def test_committed_traffic_summary_parses():
    path = os.path.join(profiling.ROOT, "profiles", "f32_walk_4096_traffic.txt")
    kv = dict(ln.split(":", 1) for ln in open(path) if ":" in ln and not ln.startswith("#"))
    assert float(kv["traffic_bytes_per_launch"]) > float(kv["algorithmic_bytes_per_launch"]) > 0


def test_valu_summary(tmp_path, capsys):
    d = str(tmp_path / "v")
    write_counters(d, [["k_walk<3>(args)", "SQ_INSTS_VALU", 9000.0],
                       ["k_walk<3>(args)", "SQ_INSTS_VALU", 8000.0],
                       ["k_walk<3>(args)", "SQ_INSTS_VALU", 8500.0],
                       ["k_walk<3>(args)", "SQ_WAVES", 10.0],
                       ["other", "SQ_INSTS_VALU", 1.0]])
    profiling.main(["valu", d, "--kernel", "k_walk<3>"])
    out = dict(ln.split(":", 1) for ln in capsys.readouterr().out.splitlines() if not ln.startswith("#"))
    assert float(out["valu_insts_per_launch"]) == 8500.0
    assert float(out["valu_insts_per_wave"]) == 850.0
    p = tmp_path / "valu.txt"
    p.write_text("\n".join(f"{k}:{v}" for k, v in out.items()) + "\n")
    assert profiling.read_valu(str(p)) == 8500.0
    p.write_text("source_sha256: 0\nvalu_insts_per_launch: 8500\n")
    assert profiling.read_valu(str(p)) is None


def test_counters_table(tmp_path, capsys):
    d = str(tmp_path / "c")
    write_counters(d, [["k_a(x)", "SQ_WAVES", 4.0], ["k_a(x)", "SQ_WAVES", 6.0], ["k_a(x)", "SQ_WAVES", 5.0],
                       ["k_a(x)", "SQ_WAIT_ANY", 9.0], ["k_b(y)", "SQ_WAVES", 1.0]])
    profiling.main(["counters", d, "--kernel", "k_a", "--kernel", "k_b"])
    lines = [ln.split() for ln in capsys.readouterr().out.splitlines() if not ln.startswith("#")]
    assert lines[0] == ["kernel", "SQ_WAIT_ANY", "SQ_WAVES"]
    assert lines[1] == ["k_a", "9", "5"]
    assert lines[2] == ["k_b", "-", "1"]


def test_traffic_table_uses_the_largest_copy(tmp_path, capsys):
    """Several kernels of one run pair; the calibration is the largest copy of
    the run (a small upload copy in the same run must not be taken for it)."""
    copy = 256 << 20
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    write_counters(fd, [["__amd_rocclr_copyBuffer", "FETCH_SIZE", 4.0],
                        ["__amd_rocclr_copyBuffer", "FETCH_SIZE", copy / 2048],
                        ["__amd_rocclr_copyBuffer", "FETCH_SIZE", 3.0],
                        ["k_a, b<1, 2>(x)", "FETCH_SIZE", 10000.0],
                        ["k_c(y)", "FETCH_SIZE", 1.0]])
    write_counters(wd, [["__amd_rocclr_copyBuffer", "WRITE_SIZE", copy / 1024],
                        ["__amd_rocclr_copyBuffer", "WRITE_SIZE", 2.0],
                        ["k_a, b<1, 2>(x)", "WRITE_SIZE", 5000.0],
                        ["k_c(y)", "WRITE_SIZE", 1.0]])
    profiling.main(["traffic-table", fd, wd, "--copy-bytes", str(copy),
                    "--kernel", "k_a, b<1, 2>=25600000", "--kernel", "k_c=0"])
    rows = [ln for ln in capsys.readouterr().out.splitlines() if not ln.startswith("#")]
    assert rows[0].split()[0] == "kernel"
    a = rows[1].split()
    # fetch 2 x 10000 KiB, write 5000 KiB: 20.48 + 5.12 MB against 25.6 MB
    assert a[-5:] == ["20.5", "5.1", "25.6", "25.6", "1.00"]
    assert rows[2].split()[-1] == "-"
