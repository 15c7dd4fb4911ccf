"""Host-side driver of SED (Sec. 5, Alg. 5) over a batch of independent
chains at fixed radii.  It only sequences library calls: per SED iteration
pecc_sed_plan (candidate counts from J), pecc_sed_perturb (Philox shifts),
one pecc_lbfgs_descend over the packed candidate batch, pecc_verify (FP64
energies of unit circles) and pecc_sed_select (Eq. 18 and the best record).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import (DescentParams, DeviceInstances, PECC_SED_MAX_CAND, RESULT_DTYPE, lbfgs_descend,
               pecc_lbfgs_descend_workspace_size, pecc_sed_perturb, pecc_sed_plan,
               pecc_sed_select, pecc_verify, results, verify)


class SedChains:
    """State of B chains: current and best layouts and FP64 energies, and the
    candidate batch (B*M slots) the iterations reuse."""

    def __init__(self, inst: DeviceInstances, xy: torch.Tensor, params: DescentParams | None = None,
                 M: int = 25, e_stop: float = 1e-25, seed: int = 0):
        assert 1 <= M <= PECC_SED_MAX_CAND
        dev = xy.device
        self.inst, self.M, self.e_stop, self.seed = inst, M, e_stop, seed
        self.P = (params or DescentParams()).c()
        self.xy = xy.reshape(-1).contiguous()
        # Alg. 5 begins by descending the starts
        out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        ws = torch.empty(pecc_lbfgs_descend_workspace_size(inst), dtype=torch.uint8, device=dev)
        from . import pecc_lbfgs_descend
        pecc_lbfgs_descend(inst, self.xy, self.P, out, ws)
        self.E_cur, _, _, _ = verify(inst, self.xy)
        self.E_start = self.E_cur.clone()
        self.E_best = self.E_cur.clone()
        self.xy_best = self.xy.clone()
        S = inst.B * M
        self.m = torch.zeros(inst.B, dtype=torch.int32, device=dev)
        self.cand_off = torch.zeros(S + 1, dtype=torch.int32, device=dev)
        self.cand_R = torch.zeros(S, dtype=torch.float32, device=dev)
        self.cand_R64 = torch.zeros(S, dtype=torch.float64, device=dev)
        self.cand_xy = torch.zeros(2 * M * max(1, inst.total_n), dtype=torch.float32, device=dev)
        self.cand = DeviceInstances(offset=self.cand_off, R=self.cand_R, R64=self.cand_R64,
                                    max_n=inst.max_n, total_n=M * inst.total_n)
        self.cand_out = torch.empty(S * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self.cand_ws = torch.empty(pecc_lbfgs_descend_workspace_size(self.cand), dtype=torch.uint8,
                                   device=dev)
        self.cand_E = torch.zeros(S, dtype=torch.float64, device=dev)
        self.chosen = torch.zeros(inst.B, dtype=torch.int32, device=dev)
        self.iterations = 0
        self.descents = inst.B
        # bookkeeping: descents per chain so far, and at its first layout
        # with E <= e_stop (-1: not yet)
        self.desc_chain = torch.ones(inst.B, dtype=torch.int64, device=dev)
        self.first_feasible = torch.where(self.E_best <= e_stop, 1, -1).to(torch.int64)

    def step(self) -> int:
        """One SED iteration of every active chain; returns the number of
        candidates descended (0: every chain has stopped)."""
        it = self.iterations
        pecc_sed_plan(self.inst, self.E_cur, self.E_best, self.M, self.e_stop, self.m,
                      self.cand_off, self.cand_R, self.cand_R64)
        active = int(self.m.sum().item())
        if active == 0:
            return 0
        pecc_sed_perturb(self.inst, self.xy, self.M, self.m, self.cand_off, self.seed, it,
                         self.cand_xy)
        from . import pecc_lbfgs_descend
        pecc_lbfgs_descend(self.cand, self.cand_xy, self.P, self.cand_out, self.cand_ws)
        pecc_verify(self.cand, self.cand_xy, 1e-20, self.cand_E, None, None, None)
        pecc_sed_select(self.inst, self.M, self.m, self.cand_off, self.cand_xy, self.cand_E,
                        self.seed, it, self.xy, self.E_cur, self.xy_best, self.E_best, self.chosen)
        self.iterations += 1
        self.descents += active
        self.desc_chain += self.m.to(torch.int64)
        newly = (self.E_best <= self.e_stop) & (self.first_feasible < 0)
        self.first_feasible = torch.where(newly, self.desc_chain, self.first_feasible)
        return active

    def run(self, s_iter: int) -> dict:
        t0 = time.perf_counter()
        for _ in range(s_iter):
            if self.step() == 0:
                break
        torch.cuda.synchronize()
        return {"iterations": self.iterations, "descents": self.descents,
                "seconds": time.perf_counter() - t0}
