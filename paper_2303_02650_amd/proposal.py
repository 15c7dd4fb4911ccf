"""Host-side driver of the learned proposal for SED's perturbation step
(Sec. 5, Alg. 5): SED perturbs the current layout, descends again and keeps
the result when its energy is lower.  Here a perturbation relocates k = 5 %
of the circles; a candidate is (circle i, destination q uniform in the disk
of radius R - 1), a network scores candidates from local features and the
k best-scored distinct circles move.  Uniform random choice among the same
candidates is the fallback, and the descent's final FP64 energy decides.

This module only sequences library calls; every computation runs in
libpecc's kernels (descent, FP64 verify, features, network forward, Adam
training, proposal, acceptance).  The random draws of the method (which
circles, which destinations) are made here with numpy and passed in.

  generate_samples  accept/reject outcomes of random relocations of
                    converged, infeasible layouts: one row of features per
                    relocated circle, labelled 1 when the restart's final
                    FP64 energy is below the energy before the move (every
                    move of a restart shares its label)
  train             Adam on the mean BCE loss over shuffled minibatches
  SsedArm           one SED chain per instance: propose, descend, verify,
                    accept
  compare           paired learned-vs-random chains on the same instances
                    with the same candidates per step
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import (DescentParams, DeviceInstances, MlpTrainer, accept, features,
               init_params, lbfgs_descend, mlp_forward, pecc_lbfgs_descend_workspace_size,
               propose, verify, RESULT_DTYPE)

E_FEASIBLE = 1e-20


def ssed_params(max_iter: int = 5000) -> DescentParams:
    """Descent settings of the restarts: FP32 working-precision stop, contact
    margin 1e-4, FP64 sufficient-decrease test below E = 3e-6."""
    return DescentParams(max_iter=max_iter, g_tol=1e-6, ftol=1e-7, ftol_window=20,
                         contact_margin=1e-4, tau64=3e-6)


def disk_points(rng: np.random.Generator, count: int, R: float) -> np.ndarray:
    u = rng.random((count, 2))
    r = (R - 1.0) * np.sqrt(u[:, 0])
    th = 2.0 * math.pi * u[:, 1]
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def draw_candidates(rng: np.random.Generator, n: np.ndarray, R: np.ndarray, count: int,
                    distinct: bool = False):
    """count candidates per instance: circle indices (distinct when asked,
    then count <= n) and destinations uniform in the disk of radius R - 1."""
    B = len(n)
    cc = np.zeros((B, count), dtype=np.int32)
    cd = np.zeros((B, count, 2), dtype=np.float32)
    for b in range(B):
        if distinct:
            cc[b] = rng.choice(int(n[b]), size=count, replace=False)
        else:
            cc[b] = rng.integers(0, int(n[b]), size=count)
        cd[b] = disk_points(rng, count, float(R[b]))
    return cc, cd


class _Batch:
    """Equal-n instances on the device plus descent buffers."""

    def __init__(self, n: int, R: np.ndarray, xy: torch.Tensor, params: DescentParams):
        self.n = n
        self.R = np.asarray(R, dtype=np.float64)
        B = len(self.R)
        self.inst = DeviceInstances.from_host(np.arange(B + 1, dtype=np.int32) * n, self.R,
                                              device=xy.device)
        self.xy = xy.reshape(-1).contiguous()
        self.P = params
        self.ws = torch.empty(pecc_lbfgs_descend_workspace_size(self.inst), dtype=torch.uint8,
                              device=xy.device)
        self.out = torch.empty(B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=xy.device)

    @property
    def B(self) -> int:
        return len(self.R)

    def descend(self, xy: torch.Tensor) -> torch.Tensor:
        """Descend xy in place; return the FP64 energies of unit circles."""
        lbfgs_descend(self.inst, xy, self.P, self.ws, self.out)
        e, _, _, _ = verify(self.inst, xy)
        return e


def generate_samples(n_restarts: int, R_range=(34.3, 34.6), n: int = 1000, frac: float = 0.05,
                     batch: int = 512, chain: int = 8, seed: int = 0, device="cuda",
                     params: DescentParams | None = None, log=None):
    """Features [rows, 8] and labels [rows] (device FP32) from at least
    n_restarts random relocations of converged infeasible layouts."""
    P = params or ssed_params()
    rng = np.random.default_rng(seed)
    k = max(1, int(round(frac * n)))
    feats, labels = [], []
    done = 0
    stats = {"restarts": 0, "accepted": 0, "starts": 0, "start_feasible": 0}
    while done < n_restarts:
        Rs = rng.uniform(R_range[0], R_range[1], size=batch)
        xy0 = np.concatenate([disk_points(rng, n, R) for R in Rs]).astype(np.float32)
        full = _Batch(n, Rs, torch.from_numpy(xy0).to(device), P)
        e = full.descend(full.xy)
        stats["starts"] += batch
        e_h = e.cpu().numpy()
        stats["start_feasible"] += int((e_h < E_FEASIBLE).sum())
        live = np.nonzero(e_h >= E_FEASIBLE)[0]
        xy_all = full.xy.view(batch, n, 2)
        for _ in range(chain):
            if len(live) == 0 or done >= n_restarts:
                break
            sel = torch.from_numpy(live).to(device)
            sub = _Batch(n, Rs[live], xy_all.index_select(0, sel).clone(), P)
            e_sub = e.index_select(0, sel).clone()
            cc, cd = draw_candidates(rng, np.full(len(live), n), Rs[live], k, distinct=True)
            ccd, cdd = torch.from_numpy(cc.reshape(-1)).to(device), torch.from_numpy(cd.reshape(-1)).to(device)
            f = features(sub.inst, sub.xy, ccd, cdd)          # before the move
            xy_new, _ = propose(sub.inst, sub.xy, ccd, cdd, None, k)
            e_new = sub.descend(xy_new)
            acc = accept(sub.inst, sub.xy, e_sub, xy_new, e_new)
            feats.append(f)
            labels.append(acc.to(torch.float32).repeat_interleave(k))
            xy_all.index_copy_(0, sel, sub.xy.view(-1, n, 2))
            e.index_copy_(0, sel, e_sub)
            e_h = e.cpu().numpy()
            acc_h = acc.cpu().numpy()
            stats["restarts"] += len(live)
            stats["accepted"] += int(acc_h.sum())
            done += len(live)
            live = live[e_h[live] >= E_FEASIBLE]
        if log:
            log(f"samples: {done} restarts, accept rate {stats['accepted'] / max(1, stats['restarts']):.3f}")
    return torch.cat(feats), torch.cat(labels), stats


def train(feats: torch.Tensor, labels: torch.Tensor, epochs: int = 16, batch_rows: int = 8192,
          lr: float = 2e-3, seed: int = 0):
    """Adam over shuffled minibatches; returns (params, per-epoch mean loss)."""
    dev = feats.device
    T = MlpTrainer(init_params(seed, device=dev), lr=lr, max_rows=batch_rows)
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    N = feats.shape[0]
    hist = []
    for _ in range(epochs):
        perm = torch.randperm(N, generator=g).to(dev)
        losses = []
        for a in range(0, N - batch_rows + 1, batch_rows):
            idx = perm[a:a + batch_rows]
            losses.append(T.train_step(feats.index_select(0, idx), labels.index_select(0, idx)).clone())
        hist.append(torch.stack(losses).mean().item() if losses else float("nan"))
    return T.params, hist


class SsedArm:
    """One SED chain per instance from a common converged start."""

    def __init__(self, batch: _Batch, xy: torch.Tensor, e: torch.Tensor, scorer: torch.Tensor | None):
        self.b = batch
        self.xy = xy.clone()
        self.e = e.clone()
        self.scorer = scorer
        self.xy_new = torch.empty_like(self.xy)

    def step(self, ccd: torch.Tensor, cdd: torch.Tensor, k: int):
        s = None
        if self.scorer is not None:
            s = mlp_forward(self.scorer, features(self.b.inst, self.xy, ccd, cdd))
        propose(self.b.inst, self.xy, ccd, cdd, s, k, xy_out=self.xy_new)
        e_new = self.b.descend(self.xy_new)
        return accept(self.b.inst, self.xy, self.e, self.xy_new, e_new)


@dataclass
class Comparison:
    first_feasible_learned: np.ndarray    # descents until first FP64-feasible layout (D+2: never)
    first_feasible_random: np.ndarray
    start_feasible: np.ndarray
    budget: int
    seconds: float

    def summary(self, boot: int = 2000, seed: int = 0) -> dict:
        L, Rn = self.first_feasible_learned, self.first_feasible_random
        cap = self.budget + 1
        d = (Rn - L).astype(np.float64)
        rng = np.random.default_rng(seed)
        bs = [d[rng.integers(0, len(d), len(d))].mean() for _ in range(boot)] if len(d) else [0.0]
        return {
            "instances": int(len(L)),
            "budget_descents": int(cap),
            "start_feasible": float(self.start_feasible.mean()),
            "feasible_learned": float((L <= cap).mean()),
            "feasible_random": float((Rn <= cap).mean()),
            "mean_descents_learned": float(np.minimum(L, cap + 1).mean()),
            "mean_descents_random": float(np.minimum(Rn, cap + 1).mean()),
            "mean_saving": float(d.mean()) if len(d) else 0.0,
            "saving_ci95": [float(np.quantile(bs, 0.025)), float(np.quantile(bs, 0.975))],
            "learned_better": int((d > 0).sum()),
            "random_better": int((d < 0).sum()),
            "seconds": self.seconds,
        }


def compare(scorer: torch.Tensor, R: float = 34.4, n: int = 1000, instances: int = 128,
            budget: int = 16, cands: int = 4096, frac: float = 0.05, seed: int = 5,
            xy0: np.ndarray | None = None, device="cuda", params: DescentParams | None = None):
    """Paired chains: each instance descends once from its start (shared),
    then both arms take up to `budget` relocate-descend-accept steps with the
    same candidates.  Descents to the first feasible layout count the first
    descent as 1 (never: budget + 2)."""
    P = params or ssed_params()
    rng = np.random.default_rng(seed)
    k = max(1, int(round(frac * n)))
    Rs = np.full(instances, R)
    if xy0 is None:
        xy0 = np.concatenate([disk_points(rng, n, R) for _ in range(instances)])
    xy0 = torch.from_numpy(np.asarray(xy0, dtype=np.float32).reshape(-1)).to(device)
    t0 = time.time()
    b = _Batch(n, Rs, xy0, P)
    e0 = b.descend(b.xy)
    start = (e0 < E_FEASIBLE).cpu().numpy()
    arms = [SsedArm(b, b.xy, e0, scorer), SsedArm(b, b.xy, e0, None)]
    first = [np.where(start, 1, budget + 2) for _ in arms]
    for s in range(budget):
        cc, cd = draw_candidates(rng, np.full(instances, n), Rs, cands)
        ccd = torch.from_numpy(cc.reshape(-1)).to(device)
        cdd = torch.from_numpy(cd.reshape(-1)).to(device)
        for a, arm in enumerate(arms):
            arm.step(ccd, cdd, k)
            feas = (arm.e < E_FEASIBLE).cpu().numpy()
            first[a] = np.where((first[a] > budget + 1) & feas, s + 2, first[a])
    torch.cuda.synchronize()
    return Comparison(first[0], first[1], start, budget, time.time() - t0)
