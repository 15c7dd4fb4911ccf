"""Seeded synthetic inputs for the circle-packing descent.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It only draws random numbers and packs arrays: it contains none
of the method's arithmetic (no energy, no gradient, no neighbor logic).

Recipe (one instance):
  * n unit circles, container radius R;
  * centres uniform in the disk of radius R - 1:
    u = rng.random((n, 2)), r = (R - 1) sqrt(u0), theta = 2 pi u1;
  * rng = numpy Generator(PCG64(seed)); instance b of a batch uses the b-th
    child of ``SeedSequence(seed).spawn(count)``.

The paper starts from centres uniform in the square [-R_b, R_b]^2 (Sec. 5.1);
the disk of radius R - 1 keeps every start inside the container, which is
the layout the benchmark workloads use.  ``square_uniform`` gives the paper's
layout for tests that want it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "disk_uniform", "square_uniform", "Instances", "pack", "instance_set",
    "relocation_draws", "apply_relocation", "rng_for", "candidates",
    "C1", "C2", "C3", "C4", "C5",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def disk_uniform(n: int, R: float, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in the disk of radius R - 1, float64 (n, 2)."""
    u = rng.random((n, 2))
    r = (R - 1.0) * np.sqrt(u[:, 0])
    th = 2.0 * math.pi * u[:, 1]
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def square_uniform(n: int, R: float, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in the square [-R, R]^2 (the paper's random layout)."""
    return rng.uniform(-R, R, size=(n, 2))


@dataclass
class Instances:
    """A packed batch of instances.

    xy      float32 (total_n, 2), instance b owns rows offset[b]:offset[b+1]
    offset  int32 (B+1,)
    R       float64 (B,)  (the FP32 copy is R.astype(float32))
    """
    xy: np.ndarray
    offset: np.ndarray
    R: np.ndarray

    @property
    def B(self) -> int:
        return int(self.R.shape[0])

    @property
    def n(self) -> np.ndarray:
        return np.diff(self.offset).astype(np.int32)

    @property
    def total_n(self) -> int:
        return int(self.offset[-1])

    @property
    def max_n(self) -> int:
        return int(self.n.max()) if self.B else 0

    def instance(self, b: int) -> np.ndarray:
        return self.xy[self.offset[b]:self.offset[b + 1]]


def pack(xys, Rs) -> Instances:
    """Pack per-instance (n_b, 2) arrays into one Instances (FP32 positions)."""
    xys = [np.asarray(a, dtype=np.float64).reshape(-1, 2) for a in xys]
    ns = [a.shape[0] for a in xys]
    offset = np.zeros(len(xys) + 1, dtype=np.int32)
    offset[1:] = np.cumsum(ns)
    xy = np.concatenate(xys, axis=0).astype(np.float32) if xys else np.zeros((0, 2), np.float32)
    return Instances(xy=np.ascontiguousarray(xy), offset=offset,
                     R=np.asarray(Rs, dtype=np.float64).reshape(-1))


def instance_set(count: int, n, R, seed: int) -> Instances:
    """count instances; n and R are ints/floats or callables of (b, rng)."""
    children = np.random.SeedSequence(seed).spawn(count)
    xys, Rs = [], []
    for b, ss in enumerate(children):
        rng = np.random.Generator(np.random.PCG64(ss))
        nb = int(n(b, rng)) if callable(n) else int(n)
        Rb = float(R(b, nb)) if callable(R) else float(R)
        xys.append(disk_uniform(nb, Rb, rng))
        Rs.append(Rb)
    return pack(xys, Rs)


def relocation_draws(n: int, R: float, frac: float, rng: np.random.Generator):
    """The random draws of one restart: round(frac*n) distinct circles
    (uniform without replacement) and as many destinations uniform in the
    disk of radius R - 1."""
    k = max(1, int(round(frac * n))) if n > 0 else 0
    idx = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
    dest = disk_uniform(k, R, rng)
    return idx, dest


def candidates(inst: "Instances", count: int, rng: np.random.Generator):
    """Candidate relocations of the learned proposal: per instance, count
    pairs (circle index uniform in [0, n_b), destination uniform in the disk
    of radius R_b - 1).  Returns cand_circle int32 [B, count] (local indices)
    and cand_dest float32 [B, count, 2]."""
    B = inst.B
    cc = np.zeros((B, count), dtype=np.int32)
    cd = np.zeros((B, count, 2), dtype=np.float32)
    for b in range(B):
        nb = int(inst.offset[b + 1] - inst.offset[b])
        if nb > 0:
            cc[b] = rng.integers(0, nb, size=count)
        cd[b] = disk_uniform(count, float(inst.R[b]), rng)
    return cc, cd


def apply_relocation(xy: np.ndarray, idx: np.ndarray, dest: np.ndarray) -> np.ndarray:
    out = np.array(xy, copy=True)
    out[idx] = dest.astype(out.dtype)
    return out


# ---------------------------------------------------------------------------
# Workload shapes.  Densities follow the paper's instance range
# (n = 300 .. 1000 at near-best-known density n / R^2 ~ 0.84).
# ---------------------------------------------------------------------------

def C1() -> Instances:
    """n = 20, R = 5.2, seed 0 (one instance)."""
    return pack([disk_uniform(20, 5.2, rng_for(0))], [5.2])


def C2(count: int = 1) -> Instances:
    """n = 1000, R = 34.6.  count = 1 is the single seed-1 instance; larger
    counts spawn independent children of seed 1."""
    if count == 1:
        return pack([disk_uniform(1000, 34.6, rng_for(1))], [34.6])
    return instance_set(count, 1000, 34.6, seed=1)


def C3_sizes(count: int = 256, seed: int = 2):
    """n_b ~ U{300..1000}, R_b = sqrt(n_b / 0.84)."""
    rng = rng_for(seed)
    ns = rng.integers(300, 1001, size=count)
    return ns.astype(np.int32), np.sqrt(ns / 0.84)


def C3(count: int = 256) -> Instances:
    """Random starts of the C3 shapes (seed 2); the converged-then-relocated
    restarts are built from these by a committed fixture script."""
    ns, Rs = C3_sizes(count)
    children = np.random.SeedSequence(2).spawn(count)
    xys = [disk_uniform(int(nb), float(Rb), np.random.Generator(np.random.PCG64(ss)))
           for nb, Rb, ss in zip(ns, Rs, children)]
    return pack(xys, Rs)


def C4(count: int = 64) -> Instances:
    """n = 1000, R = 34.4, seed 3."""
    return instance_set(count, 1000, 34.4, seed=3)


def C5(count: int = 128) -> Instances:
    """n = 1000, R = 34.4 (learned-proposal evaluation shape), seed 5."""
    return instance_set(count, 1000, 34.4, seed=5)


def C3_restarts(path: str | None = None) -> Instances:
    """The batched restart workload: 256 oracle-converged C3 packings with
    5% of their circles relocated (tests/golden/c3_restarts.npz, written by
    tests/golden/make_c3_restarts.py)."""
    import os
    p = path or os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "tests", "golden", "c3_restarts.npz")
    z = np.load(p, allow_pickle=False)
    return Instances(xy=np.ascontiguousarray(z["xy"]), offset=z["offset"].astype(np.int32),
                     R=z["R"].astype(np.float64))
