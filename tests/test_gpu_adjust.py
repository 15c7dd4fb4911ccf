"""GPU container adjustment (Sec. 4.2, Eq. 12, Alg. 2) against the oracle's:
early iterations of the first round, the proven optimal radii, and n = 1000
layouts checked in FP64 at the returned radii."""
import math

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


def run(P, inst, params, lam=1e-4, rounds=35):
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    R, out = P.adjust_container(d, xy, params, lam, rounds)
    return xy.cpu().numpy().reshape(-1, 2), R.cpu().numpy(), P.results(out), d, xy


def hexagon(scale):
    return np.array([[0.0, 0.0]] + [[2 * scale * math.cos(k * math.pi / 3),
                                     2 * scale * math.sin(k * math.pi / 3)] for k in range(6)])


def triangle(scale):
    r = 2 * scale / math.sqrt(3)
    return np.array([[r * math.cos(a), r * math.sin(a)] for a in (0.3, 0.3 + 2 * math.pi / 3,
                                                                   0.3 + 4 * math.pi / 3)])


@pytest.mark.parametrize("name,xy,R0,Ropt", [
    ("n2", np.array([[1.1, 0.2], [-1.1, -0.2]]), 2.5, 2.0),
    ("n3", triangle(1.1), 2.6, 1 + 2 / math.sqrt(3)),
    ("n7", hexagon(1.1), 3.6, 3.0),
])
def test_proven_optima(P, name, xy, R0, Ropt):
    inst = synth.pack([xy], [R0])
    prm = P.DescentParams(g_tol=1e-7, ftol=0.0, contact_margin=0.0)
    x, R, res, d, xyd = run(P, inst, prm)
    assert res["iters"][0] > 0
    assert abs(R[0] - Ropt) < 2e-5, (name, R[0], Ropt, res)
    # the oracle reaches the same optimum from the same start
    _, Ro, _ = oracle.adjust_container(xy, R0)
    assert abs(Ro - Ropt) < 1e-8


@pytest.mark.parametrize("margin", [0.0, 1e-4])
def test_first_iterations_follow_the_oracle(P, margin):
    """With a contact margin mu the GPU's circles have radius 1 + mu, in the
    pair and the containment terms alike: the oracle's radius."""
    rng = np.random.default_rng(3)
    xy = synth.disk_uniform(30, 6.5, rng)
    inst = synth.pack([xy], [6.5])
    for iters in (1, 2, 4):
        prm = P.DescentParams(max_iter=iters, g_tol=0.0, ftol=0.0, contact_margin=margin)
        x, R, res, d, xyd = run(P, inst, prm, rounds=1)
        po = oracle.DescentParams(max_iter=iters, g_tol=0.0, ftol=0.0, rad=1.0 + margin)
        xo, Ro, ro = oracle.adjust_container(inst.xy.astype(np.float64), 6.5, po, 1e-4, 1)
        assert res["iters"][0] == ro["iters"] == iters
        assert abs(R[0] - Ro) <= 1e-5 * max(1.0, abs(Ro)), (iters, R[0], Ro)
        np.testing.assert_allclose(x, xo, rtol=0, atol=2e-4)


def test_deterministic_and_zero_rounds(P):
    inst = synth.C2(4)
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4)
    a = run(P, inst, prm, rounds=6)
    b = run(P, inst, prm, rounds=6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    z = run(P, inst, prm, rounds=0)
    assert np.array_equal(z[0], inst.xy) and np.allclose(z[1], inst.R.astype(np.float32))


def test_n1000_layouts_shrink_and_stay_feasible(P):
    """Descend 16 C2 starts at R = 34.6, then adjust the container: the
    radius shrinks for most of them (it grows a little where circles of
    radius 1 + margin still overlap after the descent, which the adjustment
    resolves) and unit circles are FP64-feasible at the returned radius (the
    margin leaves the slack for FP32 rounding)."""
    inst = synth.C2(16)
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    P.lbfgs_descend(d, xy, prm)
    R, out = P.adjust_container(d, xy, prm, 1e-4, 35)
    R = R.cpu().numpy().astype(np.float64)
    res = P.results(out)
    assert (res["status"] != 6).all()
    d2 = P.DeviceInstances.from_host(inst.offset, R)
    e64, mp, mc, feas = P.verify(d2, xy)
    feas = feas.cpu().numpy()
    assert (R < 34.6).mean() >= 0.75 and R.max() < 34.7, R
    assert feas.mean() >= 0.9, (feas, e64.cpu().numpy())
    # FP64 check by the oracle on one of them
    b = int(np.argmax(feas))
    xb = xy.cpu().numpy().reshape(-1, 2)[inst.offset[b]:inst.offset[b + 1]]
    v = oracle.verify(xb, float(R[b]))
    assert v["feasible"] and v["E"] < 1e-20
