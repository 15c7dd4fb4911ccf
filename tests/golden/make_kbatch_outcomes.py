"""Writes tests/golden/kbatch_sector5_outcomes.json: the outcomes of the FP64
oracle's k-batch descent (Alg. 1 over five sector batches, Sec. 4.1) on the
32 random starts of n = 1000 at R = 34.4 (seed 3) that the GPU finish test
descends, with the GPU test's settings: circles of radius 1 + 1e-4 (the
contact margin), a relative decrease below 1e-7 over 20 outer iterations
or ||g|| <= 1e-12 ends a descent, at most 5000 outer iterations; the
neighbor lists are all pairs (anm = false) or ANM with l_cut = 4 (anm =
true).  Every final layout is checked for unit circles in FP64 (feasible:
E < 1e-20).  Calls only oracle/ and synth/.

    python tests/golden/make_kbatch_outcomes.py [--procs 8]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kbatch_sector5_outcomes.json")
COUNT, K, MARGIN = 32, 5, 1e-4


def partition(inst, b):
    return oracle.partition(inst.instance(b), "sector", K, seed=5, instance=b)


def one(args):
    b, anm = args
    inst = synth.C4(COUNT)
    x0 = inst.instance(b).astype(np.float64)
    P = oracle.DescentParams(g_tol=1e-12, ftol=1e-7, rad=1.0 + MARGIN)
    x, r, _ = oracle.gbo_seq_descend(x0, float(inst.R[b]), partition(inst, b), K, P,
                                     max_outer=5000, anm=anm, lcut=4.0 if anm else 2.3)
    v = oracle.verify(x.astype(np.float32), float(inst.R[b]))
    return {"instance": b, "anm": anm, "status": r["status"], "outer": r["outer"],
            "E_unit": v["E"], "feasible": bool(v["feasible"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args()
    oracle.lib()
    jobs = [(b, anm) for anm in (False, True) for b in range(COUNT)]
    with mp.get_context("fork").Pool(a.procs) as pool:
        rows = pool.map(one, jobs, chunksize=1)
    out = {"workload": f"{COUNT} random starts, n=1000, R=34.4 (seed 3), sector partition, k={K}",
           "settings": {"rad": 1.0 + MARGIN, "ftol": 1e-7, "ftol_window": 20, "g_tol": 1e-12,
                        "max_outer": 5000, "feasible": "unit circles, FP64 E < 1e-20 at the final FP32-rounded layout"},
           "outcomes": rows}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    for anm in (False, True):
        sel = [r for r in rows if r["anm"] == anm]
        print(f"anm={anm}: feasible {sum(r['feasible'] for r in sel)}/{len(sel)}, "
              f"MAX_ITER {sum(r['status'] == 'MAX_ITER' for r in sel)}")


if __name__ == "__main__":
    main()
