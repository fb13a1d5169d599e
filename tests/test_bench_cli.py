"""bench.py command line on the CPU: one GPU only, and the JSON fields the
measurement contract names (checked on the source, no GPU run)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_contract_fields_present():
    src = open(os.path.join(ROOT, "bench.py")).read()
    for key in ('"metric"', '"value"', '"unit"', '"n_gpus"', '"steps"', '"warmup"',
                '"ms_per_step"', '"higher_is_better"', '"scaling"', '"vs_baseline"', '"dtype"',
                '"data"', '"config"', '"roofline"', '"bound"', '"achieved"', '"peak"', '"frac"',
                '"traffic"', '"cpu_baseline"', '"cores"', '"kind"', '"sample"'):
        assert key in src, key


def test_counter_summary_scaling_and_issue_shares(tmp_path):
    # synthetic rocprofv3 counter CSV: the 2 GiB copy first, then two
    # dispatches of a kernel; FETCH_SIZE of the copy reads half its bytes
    # (scale 2), WRITE_SIZE all of them (scale 1); the issue shares are
    # instructions x 4 cycles over 1024 SIMDs x 2.4 GHz x the duration
    sys.path.insert(0, ROOT)
    import bench
    copy_kib = (2 << 30) / 1024.0
    rows = []
    did = 0

    def add(name, counter, value, t0, t1, grid=4096):
        nonlocal did
        did += 1
        rows.append(dict(Dispatch_Id=did, Kernel_Name=name, Counter_Name=counter,
                         Counter_Value=value, Grid_Size=grid, Start_Timestamp=t0,
                         End_Timestamp=t1))

    add("__amd_rocclr_copyBuffer", "FETCH_SIZE", copy_kib / 2, 0, 10)
    add("__amd_rocclr_copyBuffer", "WRITE_SIZE", copy_kib, 0, 10)
    t = 1_000_000  # ns
    for k in range(2):
        add("k_demo<1>", "FETCH_SIZE", 1000.0, 0, t)
        add("k_demo<1>", "WRITE_SIZE", 500.0, 0, t)
        add("k_demo<1>", "SQ_WAVES", 2048.0, 0, t)
        add("k_demo<1>", "SQ_INSTS_VALU", 0.25 * 1024 * 2.4e9 * 1e-3 / 4, 0, t)
        add("k_demo<1>", "SQ_INSTS_SALU", 0.10 * 1024 * 2.4e9 * 1e-3 / 4, 0, t)
    path = tmp_path / "c.csv"
    import csv
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)
    out = tmp_path / "s.json"
    bench.summarize_pmc("k_demo", str(out), [str(path)], ["cmd"], alg_bytes=3 * 1024 * 1024)
    import json
    d = json.load(open(out))
    assert abs(d["FETCH_SIZE"]["scale"] - 2.0) < 1e-12
    assert abs(d["WRITE_SIZE"]["scale"] - 1.0) < 1e-12
    assert abs(d["hbm_bytes_per_launch"] - (1000 * 1024 * 2 + 500 * 1024)) < 1e-6
    assert abs(d["ratio_hbm_to_algorithmic"] - 2500 * 1024 / (3 * 1024 * 1024)) < 1e-12
    assert abs(d["valu_issue_frac"] - 0.25) < 1e-9
    assert abs(d["salu_issue_frac"] - 0.10) < 1e-9
    assert abs(d["valu_insts_per_wave"] - 0.25 * 1024 * 2.4e9 * 1e-3 / 4 / 2048) < 1e-6
