"""Pins of the oracle's geometric batch descent (Alg. 1, Eq. 7)."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_one_batch_follows_whole_descent():
    # with k = 1 the batch method is the plain quasi-Newton descent (Sec. 6.4
    # notes GBO degenerates to the non-batch method for k = 1)
    inst = synth.C1()
    xy0 = inst.xy.astype(np.float64)
    P = oracle.DescentParams(max_iter=40)
    xw, rw, tw = oracle.descend(xy0, 5.2, P, trace=True)
    xg, rg, tg = oracle.gbo_descend(xy0, 5.2, P, blocks=1, max_outer=40, trace=True)
    assert rg["outer"] == rw["iters"]
    assert np.allclose(tg, tw, rtol=1e-9, atol=1e-12)
    assert np.allclose(xg, xw, rtol=1e-9, atol=1e-9)


def test_colour_schedule_equals_sequential_when_colours_do_not_touch():
    inst = synth.C4(1)
    xy0 = inst.xy.astype(np.float64)
    P = oracle.DescentParams()
    xj, rj, tj = oracle.gbo_descend(xy0, 34.4, P, blocks=4, max_outer=3, jacobi=True, trace=True)
    xs, rs, ts = oracle.gbo_descend(xy0, 34.4, P, blocks=4, max_outer=3, jacobi=False, trace=True)
    assert np.array_equal(xj, xs) and np.array_equal(tj, ts)


def test_partition_is_a_proper_four_colouring_of_blocks():
    inst = synth.C4(1)
    xy = inst.xy.astype(np.float64)
    R, blocks = 34.4, 4
    b, c = oracle.gbo_batches(xy, R, blocks)
    S = 2 * R / blocks
    bx, by = b % blocks, b // blocks
    # every circle lies in its block's square (clamped at the border)
    lo_x, lo_y = -R + bx * S, -R + by * S
    inside_x = ((xy[:, 0] >= lo_x - 1e-12) | (bx == 0)) & ((xy[:, 0] < lo_x + S) | (bx == blocks - 1))
    inside_y = ((xy[:, 1] >= lo_y - 1e-12) | (by == 0)) & ((xy[:, 1] < lo_y + S) | (by == blocks - 1))
    assert inside_x.all() and inside_y.all()
    # blocks that touch (8-neighbourhood) never share a colour
    col = {}
    for p, cc in zip(b, c):
        assert col.setdefault(int(p), int(cc)) == cc
    for p, cp in col.items():
        for q, cq in col.items():
            if p != q and abs(p % blocks - q % blocks) <= 1 and abs(p // blocks - q // blocks) <= 1:
                assert cp != cq


@pytest.mark.parametrize("blocks", [2, 4])
def test_batch_descent_never_raises_energy(blocks):
    inst = synth.C2(1)
    P = oracle.DescentParams()
    _, res, tr = oracle.gbo_descend(inst.xy.astype(np.float64), 34.6, P, blocks=blocks,
                                    max_outer=25, trace=True)
    assert len(tr) == 26
    assert (np.diff(tr) <= 1e-12 * tr[0]).all()
    assert tr[-1] < 0.2 * tr[0]


def test_batch_descent_closed_form_reaches_feasible():
    Rstar = 3.0
    hits = 0
    for seed in range(12):
        xy0 = synth.disk_uniform(7, Rstar + 1e-3, synth.rng_for(seed))
        _, res, _ = oracle.gbo_descend(xy0, Rstar + 1e-3, oracle.DescentParams(), blocks=2,
                                       max_outer=3000)
        hits += res["status"] == "FEASIBLE"
        _, lo, _ = oracle.gbo_descend(xy0, Rstar - 1e-3, oracle.DescentParams(), blocks=2,
                                      max_outer=3000)
        assert lo["status"] != "FEASIBLE"
    assert hits >= 1


def test_steps_are_limited_by_the_line_search_only():
    # one batch, one visit from a start with large overlaps: Alg. 1 takes the
    # step the backtracking search accepts, alpha * p with alpha0 =
    # 1 / max(1, ||g||) and halvings -- the same as the whole-instance
    # descent's first step -- however far it moves a circle
    inst = synth.C1()
    x0 = inst.xy.astype(np.float64)
    x, res, _ = oracle.gbo_descend(x0, 5.2, oracle.DescentParams(), blocks=1, max_outer=1)
    xw, _, _ = oracle.descend(x0, 5.2, oracle.DescentParams(max_iter=1))
    assert np.allclose(x, xw, rtol=0, atol=1e-12)
    assert np.hypot(*(x - x0).T).max() > 0.15
