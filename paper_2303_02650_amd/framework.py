"""Host-side driver of the framework for solving PECC (Sec. 5.1, Alg. 4) over
a batch of independent runs ("chains"), each with its own reference radius
R_b.  It only sequences library calls and keeps the best record:

  start      x* = random layout in [-R_b, R_b]^2, descended at R_b
             (pecc_lbfgs_descend), then the container adjustment of Alg. 2
             (pecc_adjust_container) gives (x*, R*);
  rounds     per round: R = min(R_b, R*); SED (Alg. 5) from a new random
             layout at R (SedChains: descent, J-controlled candidates,
             Eq. 18 selection, stop at E <= 1e-25); the adjustment of its
             best layout gives (x, R'); the record takes (x, R') when R' <
             R* and the unit circles are overlap-free at R' in FP64
             (pecc_verify with R' as the FP64 radius).

Every adjusted radius is then tightened in FP64: the descents work on
circles of radius 1 + contact_margin, so R' keeps up to that margin of
slack; the smallest container of the layout's unit circles,
max_i |c_i| + 1 rounded up to an FP32 value, replaces R' where the unit
circles are pairwise overlap-free in FP64 (pecc_verify_tighten).

The random layouts are drawn here with numpy (chain c, round t: a PCG64
stream seeded by (seed, t, c)) and passed to the library as inputs; SED
draws its perturbations with Philox inside the library (seed + round).  Rounds run until ``rounds``
are done or ``seconds`` have passed (the paper's cut-off time T_cut).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import (DescentParams, DeviceInstances, RESULT_DTYPE, adjust_container,
               pecc_lbfgs_descend, pecc_lbfgs_descend_workspace_size, pecc_verify_tighten)
from .sed import SedChains


def _random_layouts(n: int, R: np.ndarray, seed: int, round_: int) -> np.ndarray:
    """Uniform layouts in [-R_c, R_c]^2 (the initial layouts of Alg. 4 and Alg. 5)."""
    out = []
    for c, Rc in enumerate(R):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, round_, c])))
        out.append(rng.uniform(-float(Rc), float(Rc), size=(n, 2)))
    return np.concatenate(out).astype(np.float32)


class Framework:
    def __init__(self, n: int, R_b, params: DescentParams | None = None, M: int = 25,
                 s_iter: int = 500, e_stop: float = 1e-25, seed: int = 0, device="cuda"):
        self.n, self.M, self.s_iter, self.e_stop, self.seed = n, M, s_iter, e_stop, seed
        self.R_b = np.asarray(R_b, dtype=np.float64).reshape(-1)
        self.C = self.R_b.size
        self.params = params or DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4)
        self.dev = torch.device(device)
        self.offset = np.arange(self.C + 1, dtype=np.int32) * n
        self.rounds = 0
        self.history = []
        # start: descent and container adjustment of a random layout
        x = torch.from_numpy(_random_layouts(n, self.R_b, seed, 0)).to(self.dev).reshape(-1)
        inst = self._instances(self.R_b)
        out = torch.empty(self.C * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=self.dev)
        ws = torch.empty(pecc_lbfgs_descend_workspace_size(inst), dtype=torch.uint8, device=self.dev)
        pecc_lbfgs_descend(inst, x, self.params.c(), out, ws)
        self.tightened = 0
        R_adj, _ = adjust_container(inst, x, self.params)
        R_t, ok = self._tighten(x, R_adj)
        self.R_best = np.where(ok, R_t, np.inf)
        self.x_best = x.clone()
        self.R_initial = self.R_best.copy()

    def _instances(self, R: np.ndarray) -> DeviceInstances:
        return DeviceInstances.from_host(self.offset, np.asarray(R, dtype=np.float32))

    def _tighten(self, x: torch.Tensor, R_adj: torch.Tensor):
        """Each adjusted radius replaced by the smallest FP32 container of
        the layout's unit circles (max_i |c_i| + 1 rounded up) where they are
        pairwise overlap-free in FP64 and it is smaller, with FP64
        feasibility at the returned radius (pecc_verify_tighten)."""
        off = torch.from_numpy(self.offset).to(self.dev)
        Rf = R_adj.float().contiguous()
        inst = DeviceInstances(offset=off, R=Rf, R64=Rf.double(), max_n=self.n,
                               total_n=self.C * self.n)
        R_out = torch.empty(self.C, dtype=torch.float32, device=self.dev)
        feas = torch.empty(self.C, dtype=torch.int32, device=self.dev)
        pecc_verify_tighten(inst, x, 1e-20, R_out, feas)
        Rn = R_out.cpu().numpy().astype(np.float64)
        self.tightened += int((Rn < Rf.cpu().numpy().astype(np.float64)).sum())
        return Rn, feas.cpu().numpy().astype(bool)

    def step(self) -> dict:
        """One round of Alg. 4 for every chain."""
        t = self.rounds + 1
        R = np.minimum(self.R_b, self.R_best)
        inst = self._instances(R)
        x0 = torch.from_numpy(_random_layouts(self.n, R, self.seed, t)).to(self.dev).reshape(-1)
        sed = SedChains(inst, x0, self.params, M=self.M, e_stop=self.e_stop, seed=self.seed + t)
        info = sed.run(self.s_iter)
        x = sed.xy_best.clone()
        R_adj, _ = adjust_container(inst, x, self.params)
        Rn, ok = self._tighten(x, R_adj)
        better = ok & (Rn < self.R_best)
        if better.any():
            sel = torch.from_numpy(np.repeat(better, 2 * self.n)).to(self.dev)
            self.x_best = torch.where(sel, x, self.x_best)
            self.R_best = np.where(better, Rn, self.R_best)
        self.rounds = t
        rec = {"round": t, "sed_iterations": info["iterations"], "sed_descents": info["descents"],
               "sed_feasible": float((sed.E_best.cpu().numpy() <= self.e_stop).mean()),
               "improved": int(better.sum()), "R_best_mean": float(np.mean(self.R_best))}
        self.history.append(rec)
        return rec

    def run(self, rounds: int | None = None, seconds: float | None = None) -> dict:
        t0 = time.perf_counter()
        while True:
            if rounds is not None and self.rounds >= rounds:
                break
            if seconds is not None and time.perf_counter() - t0 >= seconds:
                break
            if rounds is None and seconds is None:
                break
            self.step()
        torch.cuda.synchronize()
        return {"rounds": self.rounds, "seconds": time.perf_counter() - t0,
                "R_initial": self.R_initial.tolist(), "R_best": self.R_best.tolist(),
                "tightened": self.tightened, "history": self.history}
