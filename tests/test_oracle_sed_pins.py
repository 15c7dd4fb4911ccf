"""Pins of the SED oracle (Sec. 5, Alg. 5): the Philox4x64-10 generator
against numpy's own Philox bit generator, the perturbation and selection
uniforms recomputed from numpy's words, J against its definition, the
selection rule against exact softmax probabilities, and the SED loop's
invariants."""
import math

import numpy as np
import pytest

import oracle
import synth


def numpy_block(counter, key):
    """numpy's Philox (4x64, 10 rounds) advances the counter before its first
    block: start it one below to get the block at `counter`."""
    c = list(counter)
    assert c[0] >= 1
    c[0] -= 1
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [((1, 0, 0, 0), (0, 0)), ((5, 7, 9, 11), (123, 456)),
                                         ((2 ** 63, 0, 17, 3), (2 ** 64 - 1, 0)),
                                         ((12345, 2 ** 40, 7, 2 ** 32 - 1), (99, 2 ** 63))])
def test_philox_matches_numpy(counter, key):
    assert oracle.philox(counter, key) == numpy_block(counter, key)


def test_shift_from_numpy_words():
    n, seed, chain, it, cand = 37, 4242, 5, 11, 3
    r = oracle.sed_shift(n, seed, chain, it, cand).reshape(-1)
    ref = np.empty(2 * n, dtype=np.float32)
    for k in range(2 * n):
        blk = k // 4
        if blk == 0:
            # counter word 0 is 0 for the first block: compute it with the
            # oracle's block function, pinned above against numpy
            w = oracle.philox((0, cand, it, chain), (seed, 0))[k % 4]
        else:
            w = numpy_block((blk, cand, it, chain), (seed, 0))[k % 4]
        u = np.float32(w >> 40) * np.float32(2.0 ** -24)
        ref[k] = np.float32(np.float32(u * np.float32(1.6)) - np.float32(0.8))
    assert np.array_equal(r.view(np.uint32), ref.view(np.uint32))
    assert (r >= -0.8).all() and (r < 0.8).all()


def test_shift_statistics_and_counter_layout():
    n = 4000
    a = oracle.sed_shift(n, 1, 0, 0, 0).reshape(-1)
    assert abs(a.mean()) < 0.02 and abs(a.var() - 1.6 ** 2 / 12) < 0.01
    # every component of the counter changes the draw
    for args in ((1, 1, 0, 0), (1, 0, 1, 0), (1, 0, 0, 1), (2, 0, 0, 0)):
        assert not np.array_equal(a[:64], oracle.sed_shift(32, *args).reshape(-1))
    xy = synth.disk_uniform(32, 6.0, synth.rng_for(0)).astype(np.float32)
    p = oracle.sed_perturb(xy, 1, 0, 0, 0)
    assert np.array_equal(p, (xy + oracle.sed_shift(32, 1, 0, 0, 0)).astype(np.float32))


def test_selection_uniform_from_numpy():
    for seed, chain, it in ((0, 0, 0), (7, 3, 12), (2 ** 40, 255, 499)):
        w = numpy_block((2 ** 63, 0, it, chain), (seed, 0))[0]
        assert oracle.sed_uniform(seed, chain, it) == (w >> 11) * 2.0 ** -53


def test_J_definition():
    for E in (0.5, 0.09, 2e-5, 3.7e-13, 8e-26, 5.0, 123.0):
        assert oracle.sed_J(E, 400) == math.ceil(-math.log10(E))
    assert oracle.sed_J(0.0, 25) == 25 and oracle.sed_J(1e-300, 25) == 25


def test_select_argmin_branch():
    E = [3e-4, 1e-6, 1e-6, 2e-3]
    assert oracle.sed_select(E, 1e-5, 0.99) == 1          # lowest index among the minima
    assert oracle.sed_select([5e-3], 1e-5, 0.3) == 0


def test_select_softmax_probabilities():
    E = [3e-4, 2e-6, 5e-3, 7e-5]                          # all above E_cur: softmax branch
    J = [math.ceil(-math.log10(e)) for e in E]
    w = np.exp(np.array(J, dtype=float) - max(J))
    p = w / w.sum()
    us = (np.arange(20000) + 0.5) / 20000
    counts = np.bincount([oracle.sed_select(E, 1e-9, u) for u in us], minlength=4) / len(us)
    np.testing.assert_allclose(counts, p, atol=1e-4)


def test_sed_loop_invariants():
    P = oracle.DescentParams(ftol=1e-9, ftol_window=20, max_iter=2000)
    xy = synth.disk_uniform(14, 4.3, synth.rng_for(5))
    x, r = oracle.sed(xy, 4.3, P, s_iter=6, seed=11)
    assert r["E_best"] <= r["E_start"] and r["iterations"] <= 6
    assert r["descents"] >= 1 + r["iterations"]
    assert oracle.energy(x, 4.3) == pytest.approx(r["E_best"], rel=1e-12, abs=1e-300)
    x2, r2 = oracle.sed(xy, 4.3, P, s_iter=6, seed=11)
    assert r2 == r and np.array_equal(x, x2)
    # a start that the first descent already makes feasible ends at once
    xs, rs = oracle.sed(synth.disk_uniform(7, 3.6, synth.rng_for(1)), 3.6, P, s_iter=10)
    assert rs["E_start"] <= 1e-25 and rs["iterations"] == 0 and rs["descents"] == 1
