"""Host-side parts of bench.py, checked without a GPU: the refusal of more than
one GPU, the operation count behind the roofline, the paper's fit of the GPU
cost per template (Sec. III) and the source check of the traffic figure."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    env = dict(os.environ, WORLD_SIZE="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, env=env)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_valu_operations_per_evaluation():
    # a run of L templates: 6 index operations for its first bin, one add per template
    assert bench.valu_ops_per_eval("L5_J4_W4_K8_O4") == pytest.approx(11.0 / 5.0)
    assert bench.valu_ops_per_eval("L3_J6_W4_K8") == pytest.approx(3.0)
    assert bench.valu_ops_per_eval("L1_J4_W4_K16") == 7.0


def test_paper_cost_fit():
    """log10 c = -(5/3) log10 n + log10 N / (1 + (1e6/n)^(5/6)): at n = 1e6 the
    denominator is 2, so c = 1e-10 sqrt(N); the values the benchmark quotes."""
    assert bench.paper_cost_per_template(10 ** 6, 10 ** 4) == pytest.approx(1e-8, rel=1e-12)
    assert bench.paper_cost_per_template(10 ** 6, 10 ** 3) == pytest.approx(1e-10 * 10 ** 1.5, rel=1e-12)
    assert bench.paper_cost_per_template(10 ** 5, 10 ** 4) == pytest.approx(1.5088e-8, rel=1e-4)
    assert bench.paper_cost_per_template(10 ** 7, 10 ** 4) == pytest.approx(6.6277e-9, rel=1e-4)


def test_traffic_figure_is_tied_to_its_tile_and_source():
    t = bench.measured_traffic("L5_J4_W4_K8_O4")
    assert t is None or t > 4.0e9  # at least the statistics written
    assert bench.measured_traffic("L3_J6_W4_K8") is None
    with open(os.path.join(ROOT, "profiles", "eval_grid_allsky_band_traffic.txt")) as fh:
        text = fh.read()
    assert ("source_sha256: " + bench.kernel_source_hash()) in text or t is None


def test_cpu_baseline_reports_model_and_one_thread():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
    r = bench.cpu_baseline_one_thread(n_sky=1)
    assert r["cores"] == 1 and r["value"] > 1e7, r
    assert "first 1 sky points" in r["sample"]
