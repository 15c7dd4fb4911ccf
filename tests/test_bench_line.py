"""The benchmark's output contract, on the CPU: the last stdout line is one
compact JSON object with the metric, the roofline and the CPU baseline, and
stays small however large the per-section record grows; more than one GPU
is refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _full_line():
    big = {f"k{i}": {"kernel_ms": 1.0 * i, "status_counts": {"FEASIBLE": i, "CONVERGED": 3},
                     "table": list(range(50))} for i in range(200)}
    return {
        "metric": "L-BFGS descents/sec and pair-evals/sec at n=1000, batched FP32 vs plain, to E<1e-20",
        "value": 10800.0, "unit": "descents/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 23.7, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "dtype_note": "FP64 in the verify", "data": "synthetic",
        "config": {"workload": "256 random starts, n=1000, R=34.6, m=10, max_iter=5000",
                   "instances": 256, "n": 1000, "R": 34.6, "list_cutoff": 2.3},
        "pair_evals_per_s": 2.7e10, "feasible_fraction": 0.98, "descent_ms_events_median": 23.6,
        "plain_descents_per_s": 156.0, "batched_over_plain": 69.0, "plain_instances": 256,
        "roofline_descent": {"kernel": "lbfgs_descend_kernel", "bound": "alu", "achieved": 2.1,
                             "peak": 157.3, "unit": "TFLOP/s", "frac": 0.0137, "traffic": 4.67e6,
                             "avg_launch_ms": 23.6, "busy_cu_share": 0.25, "extra": big},
        "roofline_sweep": {"kernel": "energy_grad_kernel", "bound": "hbm", "achieved": 4552.0,
                           "peak": 8000.0, "unit": "GB/s", "frac": 0.569, "traffic": 1.977e9,
                           "per_launch_bytes": 1907408896, "avg_launch_ms": 0.419,
                           "instances": 65536, "listed_pairs": 149041152, "other_list_forms": big},
        "cpu_baseline": {"value": 37.5, "unit": "descents/s", "cores": 16, "kind": "oracle",
                         "sample": "256 of the 256 starts", "single_thread_descent": big},
        "kbatch": big, "learned_proposal": big, "tau64_ablation": big,
    }


def test_compact_line_is_small_and_complete():
    out = bench.compact_line(_full_line(), "gpurun_out/bench_sections.json")
    text = json.dumps(out)
    assert len(text) < 2048, len(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in out, k
    assert "workload" in out["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in out["roofline"], k
    assert out["roofline"]["frac"] == pytest.approx(out["roofline"]["achieved"] / out["roofline"]["peak"], rel=1e-3)
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in out["cpu_baseline"], k
    assert out["cpu_baseline"]["kind"] == "oracle"
    json.loads(text)   # one line of valid JSON
    assert "\n" not in text


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
