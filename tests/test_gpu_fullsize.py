"""Full-size checks in the launch configurations the benchmark times: the
main step (256 starts of n = 1000 at R = 34.6 in one persistent launch,
FP32 with the contact margin 1e-4, FP64 near E = 0) and the HBM sweep
(65536 instances of n = 1000, one launch).  Sampled outputs are recomputed
by the oracle one by one; the rest is checked through properties that hold
at any size."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2303_02650_amd as P
    assert torch.cuda.is_available()
    return P


def test_main_step_full_size_sampled(P):
    inst = synth.C2(256)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy = torch.from_numpy(inst.xy.reshape(-1).copy()).cuda()
    prm = P.DescentParams(max_iter=5000, g_tol=1e-6, ftol=1e-7, ftol_window=20,
                          contact_margin=1e-4, tau64=1e-4)
    res = P.results(P.lbfgs_descend(d, xy, prm))
    e64, mp, mc, feas = (t.cpu().numpy() for t in P.verify(d, xy))
    x = xy.cpu().numpy().reshape(-1, 2)
    # properties of every result
    assert set(np.unique(res["status"])) <= {1, 2, 3, 5}
    assert (res["iters"] <= 5000).all() and (res["evals"] >= res["iters"]).all()
    assert (res["E32"] >= 0).all() and np.isfinite(res["E32"]).all()
    assert feas.mean() >= 0.9
    # FEASIBLE claims hold in FP64, and feasible means E64 < 1e-20
    assert (feas[res["status"] == 1] == 1).all()
    assert ((e64 < 1e-20) == (feas == 1)).all()
    # sampled instances against the oracle
    for b in range(0, 256, 37):
        xb = x[inst.offset[b]:inst.offset[b + 1]]
        v = oracle.verify(xb, float(inst.R[b]))
        assert e64[b] == pytest.approx(v["E"], rel=1e-12, abs=1e-300)
        assert bool(feas[b]) == bool(v["feasible"])
        assert mp[b] == pytest.approx(v["max_pair_overlap"], rel=1e-12, abs=1e-15)
        assert mc[b] == pytest.approx(v["max_cont_overlap"], rel=1e-12, abs=1e-15)
        # the reported FP32 energy is the energy of circles of radius 1 + 1e-4
        E_m = oracle.energy(xb.astype(np.float64), float(inst.R[b]), rad=1.0 + 1e-4)
        assert res["E32"][b] == pytest.approx(E_m, rel=1e-3, abs=1e-7)


def test_sweep_full_size_sampled(P):
    base = synth.C2(4)
    reps = 65536 // base.B
    big = synth.pack([base.instance(b) for b in range(base.B)] * reps, list(base.R) * reps)
    d = P.DeviceInstances.from_host(big.offset, big.R)
    xy = torch.from_numpy(big.xy.reshape(-1)).cuda()
    row, col = P.build_neighbors(d, xy, 2.3, 0.0, True)
    E, g = P.energy_grad(d, xy, row, col)
    E = E.cpu().numpy()
    g = g.cpu().numpy().reshape(-1, 2)
    # replicas give the same bits wherever they sit in the launch
    for b in range(base.B):
        assert np.unique(E[b::base.B]).size == 1
    rows = row.cpu().numpy()
    for b in range(base.B):
        xb = base.instance(b)
        E64, _, _, g64 = oracle.energy_grad(xb.astype(np.float64), float(base.R[b]))
        for r in (0, reps // 2, reps - 1):
            k = r * base.B + b
            assert abs(E[k] - E64) <= 1e-5 * E64
            o0, o1 = big.offset[k], big.offset[k + 1]
            gk = g[o0:o1]
            assert np.linalg.norm(gk - g64) <= 1e-5 * np.linalg.norm(g64)
        # listed entries equal the oracle's pair count (both orientations)
        o0 = big.offset[b]
        n = big.offset[b + 1] - o0
        assert rows[o0 + n] - rows[o0] == 2 * oracle.neighbors(xb, 2.3)[0].size
