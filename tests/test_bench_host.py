"""Host-side logic of bench.py (CPU): the served block's stream prefix, the
guard on the stored traffic figure, the issue-model peaks, the CPU-sized
oracle timing and the one-GPU contract."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_served_prefix_is_a_budgeted_prefix_of_the_stream(bench):
    import workloads

    stream = workloads.served_stream(100)
    rate = 8.7e12
    sizes = []
    for budget in (10.0, 120.0, 230.0, 400.0, 1e6):
        p = bench.served_prefix(100, budget, rate)
        assert 4 <= len(p) <= 100
        assert [a.spec for a in p] == [a.spec for a in stream[:len(p)]]  # a prefix, same draws
        sizes.append(len(p))
    assert sizes == sorted(sizes) and sizes[0] == 4 and sizes[-1] == 100


def test_stored_traffic_only_for_its_kernel_and_workload(bench):
    t = bench.MEASURED_TRAFFIC
    assert bench.measured_traffic("mixture-100k", t["kernel"]) is None
    assert bench.measured_traffic(t["workload"], "k_lscv_units_f32<16>") is None
    v = bench.measured_traffic(t["workload"], t["kernel"])
    assert v is None or v == pytest.approx(t["fetch_bytes"] + t["write_bytes"])


def test_issue_model_peaks(bench):
    # one LSCV term: 3 plain FP32 instructions and one exp2; a psi_r pair:
    # 5 + r/2 plain and one exp2, three stages of equal pair count
    cu, f = 256, 2.4e9
    assert bench.LSCV_PEAK == pytest.approx(1.0 / (3 / (cu * 128 * f) + 1 / (cu * 32 * f)))
    assert bench.LSCV_PEAK == pytest.approx(11.2347e12, rel=1e-4)
    assert bench.LSCV_PEAK_UNPACKED == pytest.approx(7.86432e12, rel=1e-5)
    assert bench.PSI_PLAIN == (9, 8, 7)
    assert bench.PSI_PEAK == pytest.approx(6.5536e12, rel=1e-4)
    assert bench.PSI_PEAK_UNPACKED == pytest.approx(3.93216e12, rel=1e-5)
    assert bench.FP32_PEAK_TFLOPS == 157.3


def test_plain_1k_oracle_times(bench):
    t = bench.plain_1k_oracle_times(reps=1)
    assert t["one_core_s"] > 0 and t["all_cores_s"] > 0 and t["cores"] >= 1
    import oracle

    assert oracle.num_threads() == t["cores"]  # thread count restored


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
