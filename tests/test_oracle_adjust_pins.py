"""Pins of the container adjustment (Sec. 4.2, Eq. 12, Alg. 2) in the oracle.

U = E + lambda R^2 is checked against the separately pinned energy, dU/dR by
central finite differences, and the whole algorithm against the proven
optimal radii (n = 2: 2, n = 3: 1 + 2/sqrt 3, n = 7: 3), reached from
oversized containers, and from random starts as a lower bound: no feasible
layout has a smaller radius than the optimum.
"""
import math

import numpy as np
import pytest

import oracle


def z_of(xy, R):
    return np.concatenate([np.asarray(xy, dtype=np.float64).reshape(-1), [R]])


def test_U_is_E_plus_penalty_and_shares_its_x_gradient():
    rng = np.random.default_rng(0)
    xy = rng.uniform(-3, 3, (12, 2))
    for lam in (0.0, 1e-4, 0.3):
        U, g = oracle.container_energy(z_of(xy, 3.2), 1.0, lam)
        E, _, _, gE = oracle.energy_grad(xy, 3.2)
        assert U == pytest.approx(E + lam * 3.2 ** 2, rel=1e-14)
        np.testing.assert_allclose(g[:-1], gE.reshape(-1), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("lam", [0.0, 1e-4, 0.05])
def test_dU_dR_finite_differences(lam):
    rng = np.random.default_rng(1)
    xy = rng.uniform(-3.5, 3.5, (15, 2))        # several circles cross the boundary
    R = 3.7
    _, g = oracle.container_energy(z_of(xy, R), 1.0, lam)
    h = 1e-6
    up, _ = oracle.container_energy(z_of(xy, R + h), 1.0, lam)
    dn, _ = oracle.container_energy(z_of(xy, R - h), 1.0, lam)
    fd = (up - dn) / (2 * h)
    assert abs(g[-1]) > 1e-3
    assert g[-1] == pytest.approx(fd, rel=1e-7)
    # closed form of the R component
    rho = np.sqrt((xy ** 2).sum(1))
    d0 = np.maximum(rho + 1.0 - R, 0.0)
    assert g[-1] == pytest.approx(-2 * d0.sum() + 2 * lam * R, rel=1e-13)


def hexagon():
    return np.array([[0.0, 0.0]] + [[2 * math.cos(k * math.pi / 3), 2 * math.sin(k * math.pi / 3)]
                                    for k in range(6)])


def triangle():
    r = 2 / math.sqrt(3)
    return np.array([[r * math.cos(a), r * math.sin(a)] for a in (0, 2 * math.pi / 3, 4 * math.pi / 3)])


@pytest.mark.parametrize("name,xy,R0,Ropt", [
    ("n2 from R=2.5", np.array([[1.0, 0.0], [-1.0, 0.0]]), 2.5, 2.0),
    ("n2 from R=1.6", np.array([[0.7, 0.0], [-0.7, 0.0]]), 1.6, 2.0),
    ("n3 from R=2.6", triangle() * 1.1, 2.6, 1 + 2 / math.sqrt(3)),
    ("n7 from R=3.6", hexagon() * 1.1, 3.6, 3.0),
])
def test_reaches_proven_optimum(name, xy, R0, Ropt):
    x, R, r = oracle.adjust_container(xy, R0)
    assert r["rounds"] == 35
    assert R == pytest.approx(Ropt, abs=1e-8), (name, R, r)
    assert r["E"] < 1e-20


@pytest.mark.parametrize("seed", range(4))
def test_random_starts_are_feasible_and_not_below_the_optimum(seed):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-3, 3, (7, 2))
    x, R, r = oracle.adjust_container(xy, 4.0)
    assert r["E"] < 1e-20
    assert R >= 3.0 - 1e-9
    assert R < 4.0


def test_zero_rounds_leave_the_input():
    xy = np.array([[1.0, 0.0], [-1.0, 0.0]])
    x, R, r = oracle.adjust_container(xy, 2.5, rounds=0)
    assert R == 2.5 and np.array_equal(x, xy) and r["iters"] == 0
