"""Measured autotuner for the descent's neighbor-list and cell parameters and
for the block grid of the geometric batch descent.

The knobs change how the work is organised, not what is computed:

  * list cutoff c and rebuild distance s = (c - 2) / 2 (the skin reading of
    the neighbor maintenance of Sec. 4.3): a pair that overlaps stays listed
    between rebuilds for any c > 2, so a larger c means fewer rebuilds and
    more swept pairs, a smaller one the opposite;
  * cell side h >= c of the grid the lists are built from;
  * blocks per axis of the geometric batches (batch size versus the number
    of colour phases of Alg. 1).

A circle's pair terms are summed in list order, which the cell side
changes, so two settings can round differently in the last FP32 bits and a
descent can end on a different, equally valid layout; the tuning table
is timed at a fixed iteration budget (cost per iteration), and the
geometric batch grid, which does change the schedule, is only eligible when
its FP64-feasible fraction is not below the best one's by more than
`max_feasible_drop`.

Results are cached as JSON keyed by GPU architecture, n bucket and density
bucket, in $PECC_TUNE_CACHE (default ~/.cache/pecc/tune.json).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, replace

import numpy as np
import torch

from . import (DescentParams, DeviceInstances, RESULT_DTYPE, pecc_gbo_descend,
               pecc_gbo_descend_workspace_size, pecc_lbfgs_descend,
               pecc_lbfgs_descend_workspace_size, pecc_verify, results)

# (cutoff, rebuild distance, cell side; 0 = the cutoff)
DESCENT_CANDIDATES = [(2.3, 0.15, 0.0), (2.2, 0.10, 0.0), (2.4, 0.20, 0.0), (2.6, 0.30, 0.0),
                      (2.8, 0.40, 0.0), (3.0, 0.50, 0.0), (2.3, 0.15, 2.9), (2.4, 0.20, 3.0)]
GBO_CANDIDATES = [4, 5, 6]


def cache_path() -> str:
    return os.environ.get("PECC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pecc", "tune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def workload_key(kind: str, n: np.ndarray, R: np.ndarray) -> str:
    """kind | arch | n bucket (next power of two of the largest n) | density
    bucket (n / R^2 to 0.02)."""
    n = np.asarray(n, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    nb = 1 << max(0, int(math.ceil(math.log2(max(1.0, float(n.max()))))))
    rho = float(np.mean(n / np.maximum(R, 1e-9) ** 2))
    return f"{kind}|{_arch()}|n<={nb}|rho~{round(rho / 0.02) * 0.02:.2f}"


def load_cache(path: str | None = None) -> dict:
    p = path or cache_path()
    try:
        with open(p) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    p = path or cache_path()
    data = load_cache(p)
    data[key] = entry
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _subset(offset, R, xy, sample):
    offset = np.asarray(offset, dtype=np.int64)
    B = len(offset) - 1
    k = min(B, sample)
    idx = np.linspace(0, B - 1, k).round().astype(np.int64)      # spread over the batch
    parts = [np.asarray(xy).reshape(-1, 2)[offset[b]:offset[b + 1]] for b in idx]
    off = np.zeros(k + 1, dtype=np.int32)
    off[1:] = np.cumsum([p.shape[0] for p in parts])
    return off, np.asarray(R, dtype=np.float64)[idx], np.concatenate(parts).astype(np.float32)


def _time_runs(run, reps):
    run()                                   # warm-up (and the outcome)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_descent(offset, R, xy, base: DescentParams, sample: int = 64, reps: int = 2,
                 candidates=DESCENT_CANDIDATES, tune_iters: int = 300, device="cuda") -> dict:
    """Time pecc_lbfgs_descend on a sample of the workload for each setting
    at a fixed iteration budget (tune_iters), so that the cost per iteration
    (rebuild frequency against swept pairs) decides, not how long the
    slowest trajectory happens to run.  Returns {"best": {...}, "table":
    [...]}; the first candidate is the reference."""
    off, Rs, x0 = _subset(offset, R, xy, sample)
    inst = DeviceInstances.from_host(off, Rs, device=device)
    xin = torch.from_numpy(x0.reshape(-1)).to(device)
    xw = torch.empty_like(xin)
    ws = torch.empty(pecc_lbfgs_descend_workspace_size(inst), dtype=torch.uint8, device=device)
    out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=device)
    table = []
    for cutoff, skin, cell in candidates:
        P = replace(base, cutoff=cutoff, skin_half=skin, cell_size=cell, max_iter=tune_iters)
        Pc = P.c()

        def run():
            xw.copy_(xin)
            pecc_lbfgs_descend(inst, xw, Pc, out, ws)

        ms = _time_runs(run, reps)
        res = results(out)
        it = int(res["iters"].max())
        table.append({"cutoff": cutoff, "skin_half": skin, "cell_size": cell, "ms": ms,
                      "us_per_iter": 1e3 * ms / max(1, it), "iters_max": it,
                      "rebuilds_per_iter": float(res["rebuilds"].sum() / max(1, res["iters"].sum())),
                      "pairs_per_eval": float(res["pair_evals"].sum() / max(1, res["evals"].sum()))})
    best = min(table, key=lambda t: t["us_per_iter"])
    return {"best": best, "table": table, "instances": int(inst.B), "tune_iters": tune_iters}


def tune_gbo(offset, R, xy, base: DescentParams, sample: int = 16, candidates=GBO_CANDIDATES,
             max_feasible_drop: float = 0.05, device="cuda") -> dict:
    """Time pecc_gbo_descend for each blocks-per-axis count; instances whose
    batches overflow the per-batch capacity report BAD_INSTANCE and make the
    setting ineligible."""
    off, Rs, x0 = _subset(offset, R, xy, sample)
    inst = DeviceInstances.from_host(off, Rs, device=device)
    xin = torch.from_numpy(x0.reshape(-1)).to(device)
    xw = torch.empty_like(xin)
    out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=device)
    e64 = torch.empty(inst.B, dtype=torch.float64, device=device)
    feas = torch.empty(inst.B, dtype=torch.int32, device=device)
    Pc = base.c()
    table = []
    for blocks in candidates:
        ws = torch.empty(pecc_gbo_descend_workspace_size(inst, blocks), dtype=torch.uint8,
                         device=device)

        def run():
            xw.copy_(xin)
            pecc_gbo_descend(inst, xw, Pc, blocks, 0, out, ws)

        ms = _time_runs(run, 1)
        pecc_verify(inst, xw, 1e-20, e64, None, None, feas)
        res = results(out)
        table.append({"blocks": blocks, "ms": ms, "feasible": float(feas.cpu().numpy().mean()),
                      "bad": int((res["status"] == 7).sum()),
                      "outer_iters_mean": float(res["iters"].mean())})
    ref = max(t["feasible"] for t in table if t["bad"] == 0) if any(t["bad"] == 0 for t in table) else 0.0
    ok = [t for t in table if t["bad"] == 0 and t["feasible"] >= ref - max_feasible_drop]
    best = min(ok, key=lambda t: t["ms"]) if ok else table[0]
    return {"best": best, "table": table, "instances": int(inst.B)}


def tuned_descent_params(offset, R, xy, base: DescentParams, tune_if_missing: bool = True,
                         path: str | None = None, **kw):
    """(params, entry, cached): base with the cached or freshly tuned list
    and cell settings for this workload's key."""
    n = np.diff(np.asarray(offset))
    key = workload_key("descent", n, R)
    entry = load_cache(path).get(key)
    cached = entry is not None
    if entry is None:
        if not tune_if_missing:
            return base, None, False
        entry = tune_descent(offset, R, xy, base, **kw)
        entry["base"] = asdict(base)
        store(key, entry, path)
    b = entry["best"]
    return replace(base, cutoff=b["cutoff"], skin_half=b["skin_half"],
                   cell_size=b["cell_size"]), entry, cached
