"""The benchmark's host logic (CPU): the one-GPU contract, the kernel classes the roofline
object is computed for, the traffic file written from rocprofv3 counter tables and read back
only for the kernel sources it was taken on, and that the committed traffic file belongs to
the current kernel sources."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


@pytest.mark.parametrize("name,cls", [
    ("void aaq::k_sweep<float, 2, false, false, 1, 12, 393310u>(aaq::SweepArgs<float>)", "sweep_2state"),
    ("void aaq::k_sweep<float, 1, false, false, 0, 12, 10u>(aaq::SweepArgs<float>)", "sweep_1state"),
    ("void aaq::k_sweep<double, 2, false, true, 1, 13, 524410u>(aaq::SweepArgs<double>)", "sweep_2state"),
    ("void aaq::k_bsweep<float, 2, true, 1, 12>(aaq::BatchArgs<float>)", "sweep_2state"),
    ("void aaq::k_bsweep<float, 1, false, 0, 13>(aaq::BatchArgs<float>)", "sweep_1state"),
    # batched steps compiled per shape: two states when the shape loads or creates lambda
    ("void aaq::k_bsweep_k<float, 1, 12, 265u>(aaq::BatchArgs<float>)", "sweep_1state"),      # first
    ("void aaq::k_bsweep_k<float, 0, 12, 14u>(aaq::BatchArgs<float>)", "sweep_2state"),       # plain backward
    ("void aaq::k_bsweep_k<float, 1, 13, 524410u>(aaq::BatchArgs<float>)", "sweep_2state"),   # turnaround
    ("void aaq::k_bsweep_k<float, 1, 12, 65562u>(aaq::BatchArgs<float>)", "sweep_1state"),    # forward boundary
    ("aaq::k_reduce(double const*, void const*, int const*, double*)", "reduce"),
    ("void aaq::k_bsweep_out<float>(aaq::BatchArgs<float>)", "reduce"),
    ("void aaq::k_tables<float>(aaq::TableArgs<float>)", "tables"),
    ("void aaq::k_plan_tables<float>(aaq::PlanTableArgs<float>)", "tables"),
    ("void aaq::k_units<float, 2, 10>(aaq::UnitArgs<float>)", "units"),
    ("void aaq::k_zz_pass<float>(float2 const*, unsigned long, int, int)", "zz_pass"),
    ("__amd_rocclr_copyBuffer", None),
])
def test_kernel_class(name, cls):
    assert bench.kernel_class(name) == cls


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, kib) in enumerate(rows):
            w.writerow([i + 1, name, counter, kib])


def test_traffic_file_round_trip(tmp_path):
    two = "void aaq::k_sweep<float, 2, false, false, 0, 12, 78u>(aaq::SweepArgs<float>)"
    one = "void aaq::k_sweep<float, 1, false, false, 0, 12, 10u>(aaq::SweepArgs<float>)"
    copy = "__amd_rocclr_copyBuffer"
    # the copy of 512 MiB reads as half its bytes on FETCH_SIZE and as all of them on WRITE_SIZE
    _counter_csv(tmp_path / "fetch.csv", "FETCH_SIZE", [(copy, 4), (copy, 262144), (two, 100), (two, 300), (one, 50)])
    _counter_csv(tmp_path / "write.csv", "WRITE_SIZE", [(copy, 4), (copy, 524288), (two, 200), (two, 200), (one, 70)])
    out = tmp_path / "traffic.json"
    bench.write_traffic(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"), out_path=str(out))
    t = json.load(open(out))
    assert t["kernel_sha"] == bench.kernel_hash()
    assert t["factors"]["FETCH_SIZE"]["factor"] == pytest.approx(2.0)
    assert t["factors"]["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    k2 = t["kernels"]["sweep_2state"]
    assert k2["launches"] == 2
    assert k2["fetch_bytes_per_launch"] == pytest.approx(2.0 * 200 * 1024)
    assert k2["write_bytes_per_launch"] == pytest.approx(200 * 1024)
    assert k2["hbm_bytes_per_launch"] == pytest.approx(600 * 1024)
    assert bench.load_traffic("sweep_2state", path=str(out)) == pytest.approx(600 * 1024)
    assert bench.load_traffic("sweep_1state", path=str(out)) == pytest.approx((100 + 70) * 1024)
    assert bench.load_traffic("units", path=str(out)) is None
    # counters taken on other kernel sources are not reported
    t["kernel_sha"] = "0" * 16
    json.dump(t, open(out, "w"))
    assert bench.load_traffic("sweep_2state", path=str(out)) is None
    assert bench.load_traffic("sweep_2state", path=str(tmp_path / "missing.json")) is None


def test_committed_traffic_is_for_the_current_kernel_sources():
    """profiles/traffic.json (and the profile summaries beside it) were taken on the kernel
    sources in the tree: otherwise the benchmark line reports no measured traffic."""
    t = json.load(open(bench.TRAFFIC_JSON))
    assert t["kernel_sha"] == bench.kernel_hash()
    for cls in ("sweep_1state", "sweep_2state"):
        assert bench.load_traffic(cls) > 0
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("sweep_") and name.endswith(".md"):
            assert f"kernel_sha {bench.kernel_hash()}" in open(os.path.join(ROOT, "profiles", name)).read(), name
