"""The framework of Alg. 4 on the GPU: on the proven optima (n = 2, 3, 7:
R = 2, 1 + 2/sqrt(3), 3) it reaches the optimal radius; the record only
improves, every recorded layout is overlap-free for unit circles at its
radius by the oracle's FP64 check, and runs are reproducible."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    from paper_2303_02650_amd.framework import Framework
    assert torch.cuda.is_available()
    return Framework


@pytest.mark.parametrize("n,R_opt", [(2, 2.0), (3, 1.0 + 2.0 / math.sqrt(3.0)), (7, 3.0)])
def test_reaches_proven_optima(F, n, R_opt):
    fw = F(n, [R_opt * 1.05] * 8, M=8, s_iter=20, seed=n)
    info = fw.run(rounds=3)
    Rb = np.array(info["R_best"])
    assert np.isfinite(Rb).all()
    # the descents work on circles of radius 1 + 1e-4 (contact margin), so
    # the adjusted radius sits that fraction above the optimum
    assert R_opt - 1e-6 <= Rb.min() <= R_opt * (1 + 1e-4) + 5e-5
    assert (Rb >= R_opt - 1e-6).all()                 # nothing below a proven optimum
    x = fw.x_best.cpu().numpy().reshape(-1, 2)
    for c in range(fw.C):
        v = oracle.verify(x[c * n:(c + 1) * n], float(np.float32(Rb[c])))
        assert v["E"] < 1e-20, (c, v)


def test_record_only_improves_and_is_reproducible(F):
    n = 40
    Rb = [math.sqrt(n / 0.8)] * 6
    runs = []
    for _ in range(2):
        fw = F(n, Rb, M=10, s_iter=10, seed=5)
        R0 = fw.R_best.copy()
        info = fw.run(rounds=3)
        runs.append((np.array(info["R_best"]), fw.x_best.cpu().numpy()))
        assert (np.array(info["R_best"]) <= R0).all()
        means = [h["R_best_mean"] for h in info["history"]]
        assert all(b <= a for a, b in zip(means, means[1:]))
        x = fw.x_best.cpu().numpy().reshape(-1, 2)
        for c in range(fw.C):
            assert oracle.verify(x[c * n:(c + 1) * n], float(np.float32(info["R_best"][c])))["E"] < 1e-20
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_time_limit_stops(F):
    fw = F(20, [5.3] * 2, M=4, s_iter=5, seed=1)
    info = fw.run(seconds=0.0)
    assert info["rounds"] == 0


def test_tightened_radii_are_the_smallest_fp32_containers(F):
    """Adjusted radii keep up to the contact margin of slack; the FP64
    tightening replaces them by the FP32 value just above max_i |c_i| + 1
    where the unit circles stay overlap-free, so recorded radii are never
    below that bound, are FP64-feasible, and some sit within one FP32 ulp of
    it."""
    n = 40
    fw = F(n, [math.sqrt(n / 0.8)] * 6, M=10, s_iter=10, seed=5)
    info = fw.run(rounds=2)
    assert info["tightened"] > 0
    x = fw.x_best.cpu().numpy().reshape(-1, 2)
    tight = 0
    for c in range(fw.C):
        xc = x[c * n:(c + 1) * n]
        Rc = info["R_best"][c]
        assert Rc == float(np.float32(Rc))
        Rmin = float((np.hypot(xc[:, 0].astype(np.float64), xc[:, 1].astype(np.float64)) + 1.0).max())
        assert Rc >= Rmin - 1e-12
        assert oracle.verify(xc, Rc)["E"] < 1e-20
        tight += Rc - Rmin <= float(np.spacing(np.float32(Rc)))
    assert tight >= 1
