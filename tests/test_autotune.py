"""Autotuner: cache keys and storage (CPU), and a small measured tuning run
on the GPU whose choice must be one of the candidates and keep the outcomes."""
import numpy as np
import pytest

import synth


def test_workload_key_and_cache_roundtrip(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2303_02650_amd import autotune as AT
    k1 = AT.workload_key("descent", np.array([1000, 700]), np.array([34.6, 29.0]))
    k2 = AT.workload_key("descent", np.array([600, 1000]), np.array([26.0, 34.6]))
    assert k1.startswith("descent|") and "n<=1024" in k1
    assert AT.workload_key("descent", np.array([20]), np.array([5.2])).split("|")[2] == "n<=32"
    p = str(tmp_path / "tune.json")
    AT.store(k1, {"best": {"cutoff": 2.4}}, p)
    AT.store("other", {"best": {}}, p)
    data = AT.load_cache(p)
    assert data[k1]["best"]["cutoff"] == 2.4 and "other" in data
    assert AT.load_cache(str(tmp_path / "missing.json")) == {}


@pytest.mark.gpu
def test_tune_descent_small(tmp_path):
    import paper_2303_02650_amd as P
    from paper_2303_02650_amd import autotune as AT
    rs = synth.C3_restarts()
    base = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4)
    out = AT.tune_descent(rs.offset, rs.R, rs.xy, base, sample=8, reps=1)
    assert len(out["table"]) == len(AT.DESCENT_CANDIDATES) and out["instances"] == 8
    assert out["best"] in out["table"]
    assert all(t["iters_max"] <= 300 for t in out["table"])
    assert out["best"]["us_per_iter"] == min(t["us_per_iter"] for t in out["table"])
    Pt, entry, cached = AT.tuned_descent_params(rs.offset, rs.R, rs.xy, base,
                                                path=str(tmp_path / "t.json"), sample=8, reps=1)
    assert not cached and Pt.cutoff == entry["best"]["cutoff"]
    Pt2, _, cached2 = AT.tuned_descent_params(rs.offset, rs.R, rs.xy, base,
                                              path=str(tmp_path / "t.json"))
    assert cached2 and Pt2 == Pt
