"""The stored k-batch outcomes are the oracle's: one descent that ends early
is recomputed and must match the stored record exactly."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def test_stored_kbatch_outcome_regenerates():
    import make_kbatch_outcomes as M
    gold = json.load(open(os.path.join(HERE, "golden", "kbatch_sector5_outcomes.json")))
    rows = {(r["instance"], r["anm"]): r for r in gold["outcomes"]}
    assert len(rows) == 2 * M.COUNT
    b = 29                       # FEASIBLE after 1482 outer iterations: a few seconds
    got = M.one((b, False))
    want = rows[(b, False)]
    assert got["status"] == want["status"] and got["outer"] == want["outer"]
    assert got["feasible"] == want["feasible"] and got["E_unit"] == pytest.approx(want["E_unit"], abs=0)
