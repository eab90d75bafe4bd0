"""The benchmark's measurement logic on the CPU, with synthetic profiler
output: how counter runs become per-launch HBM bytes and instruction counts
(scaled by a plain copy), which resource a roofline record calls binding and
how its fraction follows from the committed counters, the kernel names it
looks them up by, the kernel-trace summary, and the refusal of more than one
GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads  # noqa: E402

RES = "prc::k_resident<float, 0, false, true>"
COPY = "void __amd_rocclr_copyBuffer(unsigned char*, unsigned char*, unsigned long)"


def write_counters(folder, ctr, rows):
    os.makedirs(os.path.join(folder, ctr), exist_ok=True)
    with open(os.path.join(folder, ctr, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Counter_Name", "Kernel_Name",
                                           "Grid_Size", "Counter_Value"])
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow(dict(Dispatch_Id=i, Counter_Name=ctr, Kernel_Name=name, Grid_Size=grid,
                            Counter_Value=value))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_runs_become_per_launch_bytes_and_instructions(tmp_path, monkeypatch):
    """A copy that reads back half of its 256 MiB in FETCH_SIZE (KiB) sets a
    scale of 2 for reads; resident dispatches split into the first five
    (20-step launches) and the rest (the tuner's 1000-step launches)."""
    kib = bench.PMC_COPY_BYTES / 1024.0
    grid = 262144  # threads of the resident launch (its dispatches are told apart by name)
    short = [(RES, grid, 1000.0 + k) for k in range(bench.PMC_SHORT_LAUNCHES)]
    long_ = [(RES, grid, 50000.0), (RES, grid, 52000.0)]
    big = workloads.CAVITY_4096x2048_F32
    sweep = "void prc::k_sweep2<float, 0, 64, 16, false, true, true>(float const*, float*)"
    pmc = tmp_path / "pmc"
    write_counters(pmc, "FETCH_SIZE", [(COPY, 1 << 20, kib / 2)] + short + long_ +
                   [(sweep, big.nx * big.ny, 300000.0)])
    write_counters(pmc, "WRITE_SIZE", [(COPY, 1 << 20, kib)] + short + long_ +
                   [(sweep, big.nx * big.ny, 290000.0)])
    os.makedirs(pmc / "SQ", exist_ok=True)
    with open(pmc / "SQ" / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Counter_Name", "Kernel_Name",
                                           "Grid_Size", "Counter_Value"])
        w.writeheader()
        i = 0
        for ctr in bench.SQ_COUNTERS:
            for n, g, _ in short + long_:
                w.writerow(dict(Dispatch_Id=i, Counter_Name=ctr, Kernel_Name=n, Grid_Size=g,
                                Counter_Value=7.0))
                i += 1
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.traffic_from_counters(str(pmc))
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))
    assert rec["copy_scale"]["FETCH_SIZE"] == pytest.approx(2.0)
    assert rec["copy_scale"]["WRITE_SIZE"] == pytest.approx(1.0)
    small = rec["per_launch"]["1024x512_f32"]
    s20, s1000 = small[RES + "@20"], small[RES + "@1000"]
    assert s20["dispatches"] == bench.PMC_SHORT_LAUNCHES and s1000["dispatches"] == 2
    mean_short = sum(v for _, _, v in short) / len(short)
    assert s20["fetch_bytes"] == round(mean_short * 1024 * 2)
    assert s20["write_bytes"] == round(mean_short * 1024)
    assert s20["hbm_bytes"] == s20["fetch_bytes"] + s20["write_bytes"]
    assert s1000["fetch_bytes"] == round(51000.0 * 1024 * 2)
    assert s20["valu_insts"] == 7 and s1000["lds_insts"] == 7
    inst = "prc::k_sweep2<float, 0, 64, 16, false, true, true>"
    assert rec["per_launch"]["4096x2048_f32"][inst]["hbm_bytes"] == round(
        300000.0 * 1024 * 2) + round(290000.0 * 1024)


def fake_counters(tmp_path, monkeypatch, counters, source_hash=None):
    from paper_2208_03562_amd import build
    (tmp_path / "profiles").mkdir(exist_ok=True)
    rec = {"source_hash": source_hash or build.source_hash(),
           "per_launch": {"1024x512_f32": {RES + "@20": counters}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))


RESIDENT_RUN = dict(tile=9, chunk_steps=20, chunk_us=80.0, chunk_kernel_us=79.0, sweep_us=4.0)


def test_roofline_binds_to_the_larger_measured_fraction(tmp_path, monkeypatch):
    """VALU: 0.6 x 614.4 G/s over 80 us; HBM: 2.4e8 B over 80 us = 3 TB/s
    (0.375 of 8 TB/s): VALU binds, frac 0.6; the algorithmic rate is 72 B x
    nodes x 20 steps over the same 80 us."""
    w = workloads.CAVITY_1024x512_F32
    valu = 0.6 * 614.4e9 * 80e-6
    fake_counters(tmp_path, monkeypatch, {"hbm_bytes": 240_000_000, "valu_insts": valu,
                                          "lds_insts": valu / 6})
    rec = bench.roofline_of(w, dict(RESIDENT_RUN), "f32")
    assert rec["kernel"] == RES and rec["steps_per_launch"] == 20
    assert rec["bound"] == "alu" and rec["frac"] == pytest.approx(0.6, abs=1e-4)
    assert rec["fractions"]["hbm"] == pytest.approx(0.375, abs=1e-4)
    assert rec["peak"] == bench.VALU_PEAK_GINST_S
    nodes = w.nx * w.ny
    assert rec["algorithmic_bytes"] == 72 * nodes * 20
    assert rec["algorithmic_gbs"] == pytest.approx(72 * nodes * 20 / 80e-6 / 1e9, rel=1e-4)
    assert rec["valu_insts_per_node_update"] == pytest.approx(valu * 64 / (nodes * 20), abs=0.1)
    assert rec["traffic"] == 240_000_000 and rec["kernel_us"] == 80.0
    assert rec["kernel_only_us"] == 79.0


def test_roofline_binds_to_hbm_when_bytes_dominate(tmp_path, monkeypatch):
    fake_counters(tmp_path, monkeypatch, {"hbm_bytes": 560_000_000, "valu_insts": 1.0e6})
    rec = bench.roofline_of(workloads.CAVITY_1024x512_F32, dict(RESIDENT_RUN), "f32")
    assert rec["bound"] == "hbm" and rec["unit"] == "GB/s"
    assert rec["frac"] == pytest.approx(560e6 / 80e-6 / 1e9 / 8000.0, abs=1e-4)


def test_counters_of_other_code_are_not_used(tmp_path, monkeypatch):
    """Counters taken on another build of the library (another source hash)
    leave traffic null and the record on the algorithmic byte rate, said so
    in its unit."""
    fake_counters(tmp_path, monkeypatch, {"hbm_bytes": 1, "valu_insts": 1}, source_hash="0" * 16)
    rec = bench.roofline_of(workloads.CAVITY_1024x512_F32, dict(RESIDENT_RUN), "f32")
    assert rec["traffic"] is None and "fractions" not in rec
    assert rec["frac"] == rec["algorithmic_frac"] and "no counters" in rec["unit"]


def test_sweep_kernel_names():
    big = 2 * 4096 * 2048 * 9 * 4
    small = 1024 * 512 * 9 * 4
    assert bench.sweep_kernel_name("f32", 0, 9, small) == RES
    assert bench.sweep_kernel_name("f16", 0, 7, big) == \
        "prc::k_sweep2<__half, 0, 64, 16, false, true, true>"
    assert bench.sweep_kernel_name("f32", 0, 7, small) == \
        "prc::k_sweep2<float, 0, 64, 16, false, true, false>"
    assert bench.sweep_kernel_name("f64", 0, 6, big) == \
        "prc::k_sweep2<double, 0, 32, 16, false, true, false>"
    assert bench.sweep_kernel_name("bf16", 0, 2, big) == \
        "prc::k_sweep<__hip_bfloat16, 0, 128, 4, false, true>"


def test_trace_summary_splits_resident_launches_by_length(tmp_path, capsys):
    rows = [(RES, 262144, d) for d in (3500, 3510, 3490)] + \
           [(RES, 262144, d) for d in (82, 84)] + [("void prc::k_x(int)", 128, 10)]
    with open(tmp_path / "bench_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size_X", "Start_Timestamp",
                                           "End_Timestamp"])
        w.writeheader()
        t = 0
        for name, grid, us in rows:
            w.writerow(dict(Kernel_Name=name, Grid_Size_X=grid, Start_Timestamp=t,
                            End_Timestamp=t + us * 1000))
            t += us * 1000 + 5000
    bench.trace_summary(str(tmp_path))
    lines = [l for l in capsys.readouterr().out.splitlines() if l.startswith("| `")]
    assert len(lines) == 3
    long_, short = lines[0].split("|"), lines[1].split("|")
    assert int(long_[3]) == 3 and float(long_[4]) == pytest.approx(3500.0)
    assert int(short[3]) == 2 and float(short[4]) == pytest.approx(83.0)
