"""Host logic of bench.py: profile summaries and the traffic lookup."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

ADV = "void mdeos::(anonymous namespace)::k_advance<512, 1, 4096, false, 4, false>(mdeos::AdvanceParams)"
COPY = "void at::native::vectorized_elementwise_kernel<4, neg>(int)"
FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
          "Start_Timestamp", "End_Timestamp"]


def _counters(d, name, values):
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        wr = csv.DictWriter(f, FIELDS)
        wr.writeheader()
        for i, (k, v) in enumerate(values):
            wr.writerow(dict(Correlation_Id=i, Dispatch_Id=i + 1, Kernel_Name=k, Counter_Name=name,
                             Counter_Value=v, Start_Timestamp=0, End_Timestamp=1))


def test_pmc_summary_calibrates_and_round_trips(tmp_path, monkeypatch):
    copy = 1 << 30
    # warmup launch, 2 timed launches, then the calibration copy
    _counters(str(tmp_path / "f"), "FETCH_SIZE", [(ADV, 999.0), (ADV, 100.0), (ADV, 300.0), (COPY, 2 * 1048576.0)])
    _counters(str(tmp_path / "w"), "WRITE_SIZE", [(ADV, 5.0), (ADV, 10.0), (ADV, 30.0), (COPY, 1048576.0)])
    log = tmp_path / "b.log"
    log.write_text("# noise\n" + json.dumps({
        "steps": 2, "value": 1.0, "unit": "EOS evals/s", "config": {"workload": "w"},
        "roofline": {"kernel_ms": 10.0, "achieved": 1, "unit": "TFLOP/s", "frac": 0.1, "peak": 1,
                     "state_bytes_per_launch": 1e6},
        "copy_calibration": {"bytes": copy}}) + "\n")
    text = bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(log), ["cmd1", "cmd2"])
    # fetch: mean 200 KiB x (2^30 / 2 GiB) = 100 KiB; write: mean 20 KiB x 1 = 20 KiB
    want = (200 * 1024 * 0.5) + (20 * 1024 * 1.0)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_advance_cfgX_fp64_traffic.md").write_text(text)
    got = bench.traffic_from_profile("cfgX", "fp64", str(prof))
    assert got == pytest.approx(want, rel=1e-6)
    # a changed kernel source invalidates the stored figure
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.traffic_from_profile("cfgX", "fp64", str(prof)) is None


def test_traffic_absent_profile_is_null(tmp_path):
    assert bench.traffic_from_profile("nothing", "fp64", str(tmp_path)) is None


def test_energy_steps_count():
    from paper_2508_06012_amd import workloads as wl
    s = wl.cfg2().sched
    # multiples of 10 in 1..2000, plus none extra (w0 = 1000, rescales 500, 1000 are multiples)
    assert bench.energy_steps(s) == 200


def test_multi_gpu_request_exits_with_message(capsys, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err


def test_failed_serving_leg_is_reported_not_fatal(monkeypatch):
    """A serving leg runs in a child process; when it fails (here: no device
    in this process's environment), the leg comes back as an error entry with
    the child's exit status, and the caller goes on."""
    monkeypatch.setenv("HIP_VISIBLE_DEVICES", "-1")  # the child sees no device, on any host
    leg = bench.serve_leg_child(2000.0, 1)
    assert leg["rate_qps"] == 2000.0 and leg["continuum_steps"] == 1
    assert "error" in leg and ("exit status" in leg["error"] or "signal" in leg["error"]), leg
