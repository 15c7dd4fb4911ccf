"""The restart fixture (tests/golden/c3_restarts.npz) against its recipe."""
import os
import sys

import numpy as np

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_fixture_shapes_follow_recipe():
    inst = synth.C3_restarts()
    z = np.load(os.path.join(GOLD, "c3_restarts.npz"), allow_pickle=False)
    ns, Rs = synth.C3_sizes(256)
    assert inst.B == 256
    assert np.array_equal(inst.n, ns)
    assert np.allclose(inst.R, np.sqrt(ns / 0.84), rtol=0, atol=1e-12)
    assert np.isfinite(inst.xy).all()
    moved = z["moved"]
    per = np.bincount(np.searchsorted(inst.offset, moved, side="right") - 1, minlength=256)
    assert np.array_equal(per, np.maximum(1, np.round(0.05 * ns)).astype(int))
    # relocated circles sit inside the disk of radius R - 1
    inst_of = np.searchsorted(inst.offset, moved, side="right") - 1
    rho = np.hypot(inst.xy[moved, 0], inst.xy[moved, 1])
    assert (rho <= inst.R[inst_of] - 1 + 1e-4).all()
    # restarts overlap (the moved circles land inside a jammed packing)
    for b in range(0, 256, 37):
        assert oracle.energy(inst.instance(b).astype(np.float64), inst.R[b]) > 0


def test_fixture_regenerates_bit_exactly():
    sys.path.insert(0, GOLD)
    import make_c3_restarts as mk
    inst = synth.C3_restarts()
    starts = synth.C3(256)
    for b in (3, 200):
        _, x, res, idx, dest = mk.one((b, starts.instance(b), float(starts.R[b])))
        again = synth.apply_relocation(x, idx, dest).astype(np.float32)
        assert np.array_equal(again, inst.instance(b))
