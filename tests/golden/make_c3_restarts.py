"""Writes tests/golden/c3_restarts.npz: the restart inputs of the batched
restart workload (256 instances, n ~ U{300..1000} from seed 2, R =
sqrt(n / 0.84)).

Each start (uniform in the disk of radius R - 1) is descended to a local
minimum by the FP64 oracle (L-BFGS, m = 10, at most 5000 iterations, stop at
E < 1e-20, ||g|| <= 1e-12 or a relative decrease below 1e-7 over 20
iterations), then round(0.05 n) distinct circles are moved to uniform
points in the disk of radius R - 1 -- the perturbation step of the paper's
solution-space exploring heuristic (Alg. 5) in the relocation form.  Calls
only oracle/ and synth/.

    python tests/golden/make_c3_restarts.py [--count 256] [--procs 8]
"""
import argparse
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_restarts.npz")


def one(args):
    b, xy, R = args
    P = oracle.DescentParams(max_iter=5000, g_tol=1e-12, ftol=1e-7, ftol_window=20)
    x, res, _ = oracle.descend(xy.astype(np.float64), R, P)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2, b, 5])))
    idx, dest = synth.relocation_draws(x.shape[0], R, 0.05, rng)
    return b, x, res, idx, dest


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    starts = synth.C3(a.count)
    oracle.lib()
    jobs = [(b, starts.instance(b), float(starts.R[b])) for b in range(a.count)]
    with mp.get_context("fork").Pool(a.procs) as pool:
        out = sorted(pool.map(one, jobs, chunksize=1), key=lambda t: t[0])
    restarts = [synth.apply_relocation(x, idx, dest) for _, x, _, idx, dest in out]
    packed = synth.pack(restarts, starts.R)
    moved = np.concatenate([idx + packed.offset[b] for b, (_, _, _, idx, _) in enumerate(out)])
    status = np.array([r["status"] for _, _, r, _, _ in out])
    E = np.array([r["E"] for _, _, r, _, _ in out])
    np.savez_compressed(OUT, xy=packed.xy, offset=packed.offset, R=packed.R,
                        moved=moved.astype(np.int32), converged_E=E,
                        converged_status=status.astype("U12"))
    print(f"wrote {OUT}: {a.count} instances, {packed.total_n} circles; converged states "
          f"{dict(zip(*np.unique(status, return_counts=True)))}, median E {np.median(E):.3e}")


if __name__ == "__main__":
    main()
