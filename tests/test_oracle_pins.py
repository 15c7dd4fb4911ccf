"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks it against a
closed form, a finite difference, an invariance, a library routine or the
paper's dense BFGS update (Eq. 11), chosen so that a dropped term, a wrong
sign, a wrong index or a transposed operand in the oracle fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def closed_form_layouts():
    """Layouts of tests/golden/closed_forms.json, built from their text."""
    cases = json.load(open(GOLD))["cases"]
    out = []
    for c in cases:
        n = c["n"]
        if n == 2:
            xy = np.array([[-1.0, 0.0], [1.0, 0.0]])
            R = c["R"]
        elif n == 3:
            r = 2.0 / math.sqrt(3.0)  # circumradius of the side-2 triangle
            xy = np.array([[r * math.cos(a), r * math.sin(a)]
                           for a in (math.pi / 2, math.pi / 2 + 2 * math.pi / 3,
                                     math.pi / 2 + 4 * math.pi / 3)])
            R = 1.0 + 2.0 / math.sqrt(3.0)
        else:
            xy = np.array([[0.0, 0.0]] + [[2 * math.cos(k * math.pi / 3), 2 * math.sin(k * math.pi / 3)]
                                          for k in range(6)])
            R = c["R"]
        out.append((n, xy, R))
    return out


# --------------------------------------------------------------------------
# Energy (Def. 3.1, Def. 3.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", closed_form_layouts(), ids=lambda c: f"n{c[0]}")
def test_closed_form_optima_have_zero_energy(case):
    n, xy, R = case
    E, Ep, Ec, g = oracle.energy_grad(xy, R)
    assert E < 1e-20
    # shrinking the container by delta must cost energy: the optimum is tight
    E2 = oracle.energy(xy, R - 1e-3)
    assert E2 > 1e-8


def test_two_circles_container_closed_form():
    # two circles touching at (+-1, 0): container overlap of each is delta
    for delta in (1e-3, 0.1, 0.5):
        E, Ep, Ec, _ = oracle.energy_grad(np.array([[-1.0, 0.0], [1.0, 0.0]]), 2.0 - delta)
        assert Ep == 0.0
        assert Ec == pytest.approx(2 * delta * delta, rel=1e-12)


def test_pair_overlap_closed_form_any_direction():
    rng = np.random.default_rng(5)
    for _ in range(20):
        l = rng.uniform(0.01, 1.99)
        th = rng.uniform(0, 2 * np.pi)
        c = rng.uniform(-3, 3, size=2)
        xy = np.array([c, c + l * np.array([np.cos(th), np.sin(th)])])
        E, Ep, Ec, _ = oracle.energy_grad(xy, 1e6)
        assert Ec == 0.0
        assert Ep == pytest.approx((2 - l) ** 2, rel=1e-9)
    # no overlap at or beyond contact
    xy = np.array([[0.0, 0.0], [2.0, 0.0]])
    assert oracle.energy(xy, 1e6) == 0.0


def test_single_circle_containment_closed_form():
    for rho, R in ((3.0, 3.5), (3.0, 4.0), (3.0, 4.5), (0.0, 0.5)):
        E = oracle.energy(np.array([[rho * 0.6, rho * 0.8]]), R)
        assert E == pytest.approx(max(0.0, rho + 1 - R) ** 2, rel=1e-12, abs=0)


def test_chain_spacing_closed_form():
    # k circles on a line spaced s: only neighbours overlap when 1 < s < 2
    for k, s in ((5, 1.9), (12, 1.5), (8, 2.0 + 1e-9)):
        xy = np.stack([np.arange(k) * s, np.zeros(k)], axis=1)
        xy -= xy.mean(axis=0)
        E, Ep, Ec, _ = oracle.energy_grad(xy, 1e3)
        assert Ep == pytest.approx((k - 1) * max(0.0, 2 - s) ** 2, rel=1e-10, abs=0)


def test_hex_lattice_zero_iff_spacing_at_least_two():
    def hexpatch(spacing, rows=7):
        pts = []
        for r in range(-rows, rows + 1):
            for c in range(-rows, rows + 1):
                pts.append(((c + 0.5 * (r % 2)) * spacing, r * spacing * math.sqrt(3) / 2))
        return np.array(pts)
    loose = hexpatch(2.0 + 1e-6)
    R = np.sqrt((loose ** 2).sum(1)).max() + 1.0 + 1e-3
    assert oracle.energy(loose, R) == 0.0
    tight = hexpatch(2.0 - 1e-3)
    Rt = np.sqrt((tight ** 2).sum(1)).max() + 1.0 + 1e-3
    E, Ep, Ec, _ = oracle.energy_grad(tight, Rt)
    assert Ec == 0.0 and Ep > 0.0
    # every nearest-neighbour pair overlaps by 1e-3: count them independently
    tree = cKDTree(tight)
    nn_pairs = len(tree.query_pairs(2.0 - 1e-3 + 1e-9))
    assert Ep == pytest.approx(nn_pairs * 1e-6, rel=1e-6)


def test_energy_nonnegative_and_feasible_iff_zero():
    for seed in range(5):
        inst = synth.instance_set(1, 40, 6.0, seed)
        E = oracle.energy(inst.xy.astype(np.float64), 6.0)
        assert E >= 0.0
        v = oracle.verify(inst.xy, 6.0)
        # feasibility by direct geometry (scipy distance and norms)
        xy = inst.xy.astype(np.float64)
        tree = cKDTree(xy)
        overlap = len(tree.query_pairs(2.0 - 1e-12)) > 0
        outside = (np.sqrt((xy ** 2).sum(1)) + 1 > 6.0).any()
        assert (E == 0.0) == (not overlap and not outside)
        assert v["feasible"] == (E < 1e-20)


# --------------------------------------------------------------------------
# Gradient
# --------------------------------------------------------------------------

def _fd_grad(xy, R, h=1e-6):
    g = np.zeros_like(xy)
    for i in range(xy.shape[0]):
        for c in range(2):
            a = xy.copy(); a[i, c] += h
            b = xy.copy(); b[i, c] -= h
            g[i, c] = (oracle.energy(a, R) - oracle.energy(b, R)) / (2 * h)
    return g


def _away_from_kinks(xy, R, margin=1e-3):
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    iu = np.triu_indices(xy.shape[0], 1)
    rho = np.sqrt((xy ** 2).sum(1))
    return (np.abs(d[iu] - 2) > margin).all() and (d[iu] > margin).all() and \
        (np.abs(rho + 1 - R) > margin).all()


@pytest.mark.parametrize("seed", range(4))
def test_gradient_matches_central_differences(seed):
    rng = synth.rng_for(100 + seed)
    R = 4.0
    xy = synth.disk_uniform(12, R + 0.7, rng)  # some circles poke out
    assert _away_from_kinks(xy, R)
    E, Ep, Ec, g = oracle.energy_grad(xy, R)
    assert Ep > 0 and Ec > 0
    fd = _fd_grad(xy, R)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_pair_forces_sum_to_zero_and_no_torque():
    rng = synth.rng_for(7)
    xy = synth.disk_uniform(60, 6.0, rng)
    E, Ep, Ec, g = oracle.energy_grad(xy, 1e6)  # huge container: pair part only
    assert Ec == 0.0 and Ep > 0
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * np.abs(g).sum()
    torque = (xy[:, 0] * g[:, 1] - xy[:, 1] * g[:, 0]).sum()
    assert abs(torque) < 1e-11 * np.abs(g).sum()


def test_invariances():
    rng = synth.rng_for(11)
    R = 7.0
    xy = synth.disk_uniform(50, R + 0.5, rng)
    E, Ep, Ec, g = oracle.energy_grad(xy, R)
    # rotation about the origin: E unchanged, g rotates
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    E2, Ep2, Ec2, g2 = oracle.energy_grad(xy @ Q.T, R)
    assert E2 == pytest.approx(E, rel=1e-12)
    assert np.allclose(g2, g @ Q.T, rtol=1e-9, atol=1e-12)
    # translation: the pair part is unchanged
    _, Ep3, _, _ = oracle.energy_grad(xy + np.array([3.0, -2.0]), R)
    assert Ep3 == pytest.approx(Ep, rel=1e-12)
    # relabelling: E unchanged, g permutes
    perm = rng.permutation(xy.shape[0])
    E4, _, _, g4 = oracle.energy_grad(xy[perm], R)
    assert E4 == pytest.approx(E, rel=1e-12)
    assert np.allclose(g4, g[perm], rtol=1e-10, atol=1e-13)


def test_inflated_radius_equals_rescaled_problem():
    # circles of radius r in a container R are unit circles in R/r after
    # scaling lengths by 1/r: E_r(x; R) = r^2 E_1(x/r; R/r)
    rng = synth.rng_for(3)
    xy = synth.disk_uniform(30, 5.5, rng)
    r = 1.0 + 1e-2
    E_r, _, _, g_r = oracle.energy_grad(xy, 5.0, rad=r)
    E_1, _, _, g_1 = oracle.energy_grad(xy / r, 5.0 / r)
    assert E_r == pytest.approx(r * r * E_1, rel=1e-12)
    assert np.allclose(g_r, r * g_1, rtol=1e-10, atol=1e-14)


# --------------------------------------------------------------------------
# Batch energy (Eq. 7)
# --------------------------------------------------------------------------

def test_batch_energy_identities():
    rng = synth.rng_for(21)
    R = 6.0
    xy = synth.disk_uniform(45, R + 0.3, rng)
    E, Ep, Ec, g = oracle.energy_grad(xy, R)
    batches = rng.integers(0, 4, size=xy.shape[0])
    total = 0.0
    within = 0.0
    for b in range(4):
        mask = (batches == b).astype(np.int32)
        Eb, gb = oracle.batch_energy_grad(xy, R, mask)
        # gradient of the batch energy is the full gradient restricted to B_p
        assert np.allclose(gb[mask == 1], g[mask == 1], rtol=1e-12, atol=1e-14)
        assert (gb[mask == 0] == 0).all()
        total += Eb
        within += oracle.energy(xy[mask == 1], R)  # pairs inside B_p + containment
    cross = E - within
    # every cross pair is counted by both of its batches, inner pairs once
    assert total == pytest.approx(E + cross, rel=1e-12)


def test_batch_energy_depends_only_on_batch_terms():
    # moving a circle outside B_p changes E(x_p) only through pairs with B_p;
    # finite differences of E(x_p) w.r.t. x_p equal the restricted gradient
    rng = synth.rng_for(22)
    R = 5.0
    xy = synth.disk_uniform(25, R + 0.4, rng)
    assert _away_from_kinks(xy, R)
    mask = (np.arange(25) % 3 == 0).astype(np.int32)
    _, gb = oracle.batch_energy_grad(xy, R, mask)
    h = 1e-6
    for i in np.flatnonzero(mask):
        for c in range(2):
            a = xy.copy(); a[i, c] += h
            b = xy.copy(); b[i, c] -= h
            fd = (oracle.batch_energy_grad(a, R, mask)[0] - oracle.batch_energy_grad(b, R, mask)[0]) / (2 * h)
            assert fd == pytest.approx(gb[i, c], rel=1e-5, abs=1e-9)


# --------------------------------------------------------------------------
# Neighbor pairs (Gamma of Sec. 4.3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_neighbors_match_kdtree(seed):
    inst = synth.instance_set(1, 700, 29.0, seed)
    xy32 = inst.xy
    pi, pj = oracle.neighbors(xy32, 2.3)
    assert (pi < pj).all()
    order = np.lexsort((pj, pi))
    assert (order == np.arange(len(pi))).all()  # ordered by i then j
    ref = cKDTree(xy32.astype(np.float64)).query_pairs(2.3, output_type="ndarray")
    ref = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
    assert len(ref) == len(pi)
    assert (ref[:, 0] == pi).all() and (ref[:, 1] == pj).all()


def test_neighbors_strict_cutoff_and_degenerate():
    xy = np.array([[0, 0], [2.5, 0], [0, 2.25], [0, 0]], dtype=np.float32)
    pi, pj = oracle.neighbors(xy, 2.3)
    assert set(zip(pi.tolist(), pj.tolist())) == {(0, 2), (0, 3), (2, 3)}
    pi, pj = oracle.neighbors(np.zeros((0, 2), np.float32), 2.3)
    assert len(pi) == 0
    pi, pj = oracle.neighbors(np.zeros((1, 2), np.float32), 2.3)
    assert len(pi) == 0


# --------------------------------------------------------------------------
# Inverse-Hessian product (Eq. 10-11)
# --------------------------------------------------------------------------

def _dense_eq11(S, Y, g):
    """H g with H from Eq. 11 applied to each stored pair, oldest first,
    starting from gamma I (gamma from the newest pair)."""
    dim = g.shape[0]
    s, y = S[-1], Y[-1]
    H = (s @ y) / (y @ y) * np.eye(dim)
    I = np.eye(dim)
    for u, v in zip(S, Y):
        beta = v @ u
        H = (I - np.outer(u, v) / beta) @ H @ (I - np.outer(v, u) / beta) + np.outer(u, u) / beta
    return H @ g


@pytest.mark.parametrize("k", [1, 2, 5, 10])
def test_two_loop_equals_dense_bfgs_update(k):
    rng = np.random.default_rng(k)
    dim = 14
    A = rng.normal(size=(dim, dim))
    A = A @ A.T + dim * np.eye(dim)  # SPD model Hessian: s^T y > 0
    S = rng.normal(size=(k, dim))
    Y = S @ A.T + 0.01 * rng.normal(size=(k, dim))
    g = rng.normal(size=dim)
    r = oracle.two_loop(S, Y, g)
    ref = _dense_eq11(S, Y, g)
    assert np.allclose(r, ref, rtol=1e-10, atol=1e-12)


def test_two_loop_without_history_is_identity():
    g = np.arange(6.0)
    assert np.array_equal(oracle.two_loop(np.zeros((0, 6)), np.zeros((0, 6)), g), g)


def test_two_loop_secant_condition():
    # the BFGS update makes H y_newest = s_newest
    rng = np.random.default_rng(3)
    dim, k = 10, 4
    A = rng.normal(size=(dim, dim)); A = A @ A.T + np.eye(dim)
    S = rng.normal(size=(k, dim)); Y = S @ A.T
    assert np.allclose(oracle.two_loop(S, Y, Y[-1]), S[-1], rtol=1e-9, atol=1e-11)


# --------------------------------------------------------------------------
# Descent (Alg. 1, k = 1, L-BFGS reading)
# --------------------------------------------------------------------------

def test_descent_energy_non_increasing_and_counts():
    inst = synth.C1()
    xy0 = inst.xy.astype(np.float64)
    P = oracle.DescentParams(max_iter=2000)
    x, res, tr = oracle.descend(xy0, 5.2, P, trace=True)
    assert res["iters"] == len(tr) - 1
    assert (np.diff(tr) <= 0).all()
    assert res["E"] == pytest.approx(oracle.energy(x, 5.2), rel=1e-12, abs=1e-300)
    assert res["status"] in ("FEASIBLE", "STATIONARY", "MAX_ITER", "STALLED")


def test_descent_on_quadratic_pair_reaches_contact():
    # two overlapping circles in a big container: the minimum separates them
    xy = np.array([[-0.3, 0.1], [0.4, -0.2]])
    x, res, _ = oracle.descend(xy, 50.0)
    assert res["status"] == "FEASIBLE"
    d = np.linalg.norm(x[0] - x[1])
    assert d >= 2.0 - 1e-10


@pytest.mark.parametrize("case", closed_form_layouts(), ids=lambda c: f"n{c[0]}")
def test_descent_closed_form_radius_bounds(case):
    n, _, Rstar = case
    reached_above = 0
    for seed in range(16):
        xy0 = synth.disk_uniform(n, Rstar + 1e-3, synth.rng_for(seed))
        _, res_hi, _ = oracle.descend(xy0, Rstar + 1e-3)
        reached_above += res_hi["status"] == "FEASIBLE"
        _, res_lo, _ = oracle.descend(xy0, Rstar - 1e-3)
        # below the proven optimum no layout is feasible
        assert res_lo["E"] > 1e-20 and res_lo["status"] != "FEASIBLE"
    assert reached_above >= 1


def test_descent_status_max_iter_and_ftol():
    inst = synth.C1()
    xy0 = inst.xy.astype(np.float64)
    _, res, _ = oracle.descend(xy0, 5.2, oracle.DescentParams(max_iter=3))
    assert res["iters"] <= 3
    if res["status"] == "MAX_ITER":
        assert res["iters"] == 3


def test_verify_specific_overlaps():
    xy = np.array([[0, 0], [1.5, 0], [0, 4.0]], dtype=np.float32)
    v = oracle.verify(xy, 5.5)
    assert v["max_pair_overlap"] == pytest.approx(0.5)
    assert v["max_cont_overlap"] == pytest.approx(0.0 + max(0, 4 + 1 - 5.5))
    assert v["E"] == pytest.approx(0.25)
    v = oracle.verify(xy, 4.5)
    assert v["max_cont_overlap"] == pytest.approx(0.5)
    assert not v["feasible"]


def test_neighbors_boundary_against_exact_rationals():
    # pairs whose exact squared distance (rational arithmetic on the FP32
    # inputs) lies within 1e-7 relative of cutoff^2 on either side, but not
    # so close that the one rounding of the FP64 sum could flip the decision
    from fractions import Fraction
    rng = np.random.default_rng(9)
    c2 = 2.3 * 2.3
    c2q = Fraction(c2)
    pts, want = [], []
    while len(pts) < 400:
        a = rng.uniform(-30, 30, size=2).astype(np.float32)
        th = rng.uniform(0, 2 * np.pi)
        l = 2.3 * (1 + rng.uniform(-5e-8, 5e-8))
        b = (a.astype(np.float64) + l * np.array([np.cos(th), np.sin(th)])).astype(np.float32)
        dx = Fraction(float(a[0])) - Fraction(float(b[0]))
        dy = Fraction(float(a[1])) - Fraction(float(b[1]))
        l2 = dx * dx + dy * dy
        rel = abs(float((l2 - c2q) / c2q))
        if rel < 1e-14 or rel > 1e-7:
            continue
        pts.append((a, b))
        want.append(l2 < c2q)
    assert 50 < sum(want) < 350
    for (a, b), w in zip(pts, want):
        pi, pj = oracle.neighbors(np.stack([a, b]), 2.3)
        assert (len(pi) == 1) == w


def test_descent_sufficient_decrease_with_large_c1():
    # with c1 = 0.4 an accepted step must cut E by a visible amount: the
    # trace never rises and falls strictly while far from a minimum (near
    # one, FP64 steps can leave E unchanged and are accepted with equality)
    for seed in range(3):
        xy0 = synth.disk_uniform(30, 6.0, synth.rng_for(seed))
        P = oracle.DescentParams(max_iter=200, c1=0.4)
        _, res, tr = oracle.descend(xy0, 6.0, P, trace=True)
        assert len(tr) > 25
        assert (np.diff(tr) <= 0).all()
        assert (np.diff(tr[:20]) < 0).all()


def test_nonfinite_position_leaves_energy_undefined():
    xy = synth.disk_uniform(6, 4.0, synth.rng_for(4))
    xy[3, 1] = np.inf
    E, Ep, Ec, g = oracle.energy_grad(xy, 4.0)
    assert np.isnan(E) and np.isnan(g).all()
    xy[3, 1] = np.nan
    v = oracle.verify(xy.astype(np.float32), 4.0)
    assert np.isnan(v["E"]) and not v["feasible"]
