#!/usr/bin/env python3
"""Benchmark of the PECC penalty-energy descent on one MI355X.

A step is one pass of the whole hot path over one batch: 256 random starts
of n = 1000 unit circles in a container of radius R = 34.6 (centres uniform
in the disk of radius R - 1, independent children of seed 1) are reset into
the work buffer, every instance descends with L-BFGS in one persistent
launch (cell-grid neighbor lists, skin-triggered rebuilds, FP32 sweep, FP64
sufficient-decrease test near E = 0) and the FP64 verify checks every final
layout.  The step is captured once as HIP graphs and replayed.

Printed JSON line: descents/s of the batched path (value), the plain
single-instance path on a sample of the same instances, pair-evals/s, the
fraction of descents that end FP64-feasible (E < 1e-20), the roofline of the
descent kernel and of the standalone list sweep at an HBM-sized batch, and
the FP64 oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3         # MI355X vector FP32, TFLOP/s
FP64_PEAK_TFLOPS = 78.6          # MI355X vector FP64, TFLOP/s
BF16_PEAK_TFLOPS = 2500.0        # MI355X dense BF16 matrix cores, TFLOP/s
MLP_FLOPS_PER_ROW = 2 * (8 * 64 + 64 * 64 + 64)   # multiply-adds of the 8-64-64-1 network
COPY_BYTES = 1 << 30             # calibration copy: 1 GiB read + 1 GiB written
# HBM bytes per launch of the uint16-list sweep at 65536 x n=1000, from two
# rocprofv3 counter runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the scales
# measured on the 1 GiB copy): profiles/energy_grad_kernel_traffic_65536x1000.md.
# Valid for the kernel as profiled; None for other batch sizes.
SWEEP_TRAFFIC_BYTES_65536 = 1.9769e9
# HBM bytes per launch of lbfgs_descend_kernel for the 256-instance main step
# (same counter runs): profiles/lbfgs_descend_kernel_traffic_256x1000.md.
DESCENT_TRAFFIC_BYTES_256 = 4.77e6
# Instruction counters of the same launch (SQ_INSTS_VALU per wave per
# evaluation, SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES):
# profiles/lbfgs_descend_kernel_sq_counters_256x1000.md.  Valid for the
# kernel as profiled.
DESCENT_VALU_PER_WAVE_EVAL_256 = 1164
DESCENT_VALU_ACTIVE_SHARE_256 = 0.332

N_CIRCLES, R_C2, BATCH = 1000, 34.6, 256


def kbatch_study(P, a, dev, stream):
    """Alg. 1 with k equal batches of the sector, annulus, fence and random
    partitions, batches visited in order, on random starts of n = 1000 at
    R = 34.4: descents per second, outer iterations and the converged FP64
    energy for every (partition, k), and the ratio of the best k's time to
    k = 1's (the quantities of the paper's partition and batch-number
    study).  One launch per setting covers every start; with more starts
    than compute units the rate reflects the mean descent time."""
    import torch
    import synth
    c4 = synth.C4(a.kbatch_instances)
    d = P.DeviceInstances.from_host(c4.offset, c4.R)
    x0 = torch.from_numpy(c4.xy.reshape(-1)).to(dev)
    x = torch.empty_like(x0)
    ws = torch.empty(P.pecc_gbo_kbatch_descend_workspace_size(d), dtype=torch.uint8, device=dev)
    out = torch.empty(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    e64 = torch.empty(d.B, dtype=torch.float64, device=dev)
    feas = torch.empty(d.B, dtype=torch.int32, device=dev)
    bo = torch.empty(d.total_n, dtype=torch.int32, device=dev)
    ks = [int(v) for v in a.kbatch_ks.split(",") if v]
    dks = [int(v) for v in a.kbatch_dense_ks.split(",") if v]

    def one(kind, k, anm=False):
        prm = descent_params(P, a.max_iter)
        if anm:
            prm.cutoff = 4.0
        pc = prm.c()
        P.pecc_partition(d, x0, P.PARTITIONS[kind], k, 17, bo)
        x.copy_(x0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.pecc_gbo_kbatch_descend(d, x, bo, k, 1 if anm else 0, pc, out, ws)
        e1.record(stream)
        P.pecc_verify(d, x, 1e-20, e64, None, None, feas)
        torch.cuda.synchronize()
        r = P.results(out)
        ms = e0.elapsed_time(e1)
        return {"kernel_ms": ms, "descents_per_s": d.B / (ms / 1e3),
                "outer_iters_mean": float(r["iters"].mean()),
                "evals_mean": float(r["evals"].mean()),
                "rebuilds_mean": float(r["rebuilds"].mean()),
                "E64_mean": float(e64.cpu().numpy().mean()),
                "feasible_fraction": float(feas.cpu().numpy().mean()),
                "status_counts": {P.STATUS[s]: int((r["status"] == s).sum()) for s in np.unique(r["status"])}}

    one("sector", 5)                                  # warm-up
    table = {}
    for kind in P.PARTITIONS:
        for k in ks:
            if kind != "sector" and k == 1:
                continue                              # k = 1 is one batch for every kind
            table[f"{kind}_k{k}"] = one(kind, k)
            print(f"[bench] kbatch {kind} k={k}: {table[f'{kind}_k{k}']['kernel_ms']:.1f} ms, "
                  f"E64 mean {table[f'{kind}_k{k}']['E64_mean']:.3g}", file=sys.stderr, flush=True)
    table["sector_k5_anm_lcut4"] = one("sector", 5, anm=True)
    if 1 in ks:
        table["sector_k1_anm_lcut4"] = one("sector", 1, anm=True)
    summary = {}
    if 1 in ks:
        t1 = table["sector_k1"]["kernel_ms"]
        for kind in P.PARTITIONS:
            cand = {k: table[f"{kind}_k{k}"]["kernel_ms"] for k in ks if k > 1 and f"{kind}_k{k}" in table}
            if cand:
                kb = min(cand, key=cand.get)
                summary[kind] = {"best_k": kb, "best_ms": cand[kb], "ratio_to_k1": cand[kb] / t1}
    # the paper's dense per-batch matrices: sector batches, fewer starts
    dense = {}
    if a.kbatch_dense_instances > 0:
        cd = synth.C4(a.kbatch_dense_instances)
        dd = P.DeviceInstances.from_host(cd.offset, cd.R)
        xd0 = torch.from_numpy(cd.xy.reshape(-1)).to(dev)
        xd = torch.empty_like(xd0)
        bod = torch.empty(dd.total_n, dtype=torch.int32, device=dev)
        outd = torch.empty(dd.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        e64d = torch.empty(dd.B, dtype=torch.float64, device=dev)
        feasd = torch.empty(dd.B, dtype=torch.int32, device=dev)
        pc = descent_params(P, a.max_iter).c()
        for k in dks:
            mb = -(-1000 // k)
            wsd = torch.empty(P.pecc_gbo_kbatch_bfgs_workspace_size(dd, mb), dtype=torch.uint8,
                              device=dev)
            P.pecc_partition(dd, xd0, P.PARTITIONS["sector"], k, 17, bod)
            xd.copy_(xd0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.pecc_gbo_kbatch_bfgs_descend(dd, xd, bod, k, 0, mb, pc, outd, wsd)
            e1.record(stream)
            P.pecc_verify(dd, xd, 1e-20, e64d, None, None, feasd)
            torch.cuda.synchronize()
            r = P.results(outd)
            ms = e0.elapsed_time(e1)
            # matrix bytes: per visit one read and one write (the pass that
            # forms H g and applies the pending update of Eq. 11), counting
            # every visit as updating its matrix
            vis = float(r["iters"].astype(np.float64).sum()) * k
            mbytes = vis * 2 * 4 * (2 * 1000 / k) ** 2
            dense[f"sector_k{k}"] = {
                "kernel_ms": ms, "descents_per_s": dd.B / (ms / 1e3),
                "matrix_bytes_per_instance": 4 * k * (2 * mb) ** 2,
                "matrix_GBs_if_every_visit_updates": mbytes / (ms / 1e3) / 1e9,
                "outer_iters_mean": float(r["iters"].mean()), "outer_iters_max": int(r["iters"].max()),
                "evals_mean": float(r["evals"].mean()),
                "E64_mean": float(e64d.cpu().numpy().mean()),
                "feasible_fraction": float(feasd.cpu().numpy().mean()),
                "status_counts": {P.STATUS[s]: int((r["status"] == s).sum()) for s in np.unique(r["status"])}}
            del wsd
            print(f"[bench] kbatch dense sector k={k}: {ms:.1f} ms", file=sys.stderr, flush=True)
        if 1 in dks:
            t1 = dense["sector_k1"]["kernel_ms"]
            cand = {k: dense[f"sector_k{k}"]["kernel_ms"] for k in dks if k > 1}
            if cand:
                kb = min(cand, key=cand.get)
                dense["best"] = {"best_k": kb, "best_ms": cand[kb], "ratio_to_k1": cand[kb] / t1}
        dense["workload"] = (f"{dd.B} random starts, n=1000, R=34.4 (seed 3); sector batches, one "
                             f"dense FP32 inverse-Hessian matrix per batch (Eq. 8-11)")
        if a.dense_rate_iters > 0:
            dense["matrix_pass_rate"] = dense_pass_rate(P, a, dev, stream)
    whole = descent_params(P, a.max_iter).c()
    x.copy_(x0)
    wws = torch.empty(P.pecc_lbfgs_descend_workspace_size(d), dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    P.pecc_lbfgs_descend(d, x, whole, out, wws)
    e1.record(stream)
    torch.cuda.synchronize()
    return {"workload": f"{d.B} random starts, n=1000, R=34.4 (seed 3); k equal batches of each "
                        f"partition visited in order, one L-BFGS iteration per visit; cutoff 2.3 "
                        f"with skin 0.15, or ANM with l_cut 4",
            "settings": table, "best_k_by_partition": summary, "dense_bfgs": dense,
            "whole_instance_descent_ms": e0.elapsed_time(e1)}


def dense_pass_rate(P, a, dev, stream):
    """Matrix throughput of the dense k = 1 descent with every start busy for
    the whole launch: g_tol = ftol = 0, so each start runs the same number of
    outer iterations (a.dense_rate_iters, unless a line search stalls) and
    each workgroup streams its 2000 x 2000 FP32 matrix for the whole
    kernel.  Matrix bytes: the first two visits do not touch the matrix
    (H = I, no update known yet), the third writes it without reading it,
    every later one reads and writes it once; per start (2 t - 5) x 16 MB for
    t outer iterations.  With B <= compute units one workgroup runs per CU,
    so bytes / kernel time / B is the rate of one CU."""
    import torch
    import synth
    out = {}
    for B in (64, a.kbatch_dense_instances):
        if B <= 0 or str(B) in out:
            continue
        c = synth.C4(B)
        d = P.DeviceInstances.from_host(c.offset, c.R)
        x = torch.from_numpy(c.xy.reshape(-1)).to(dev)
        bo = torch.zeros(d.total_n, dtype=torch.int32, device=dev)
        res_b = torch.empty(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        ws = torch.empty(P.pecc_gbo_kbatch_bfgs_workspace_size(d, 1000), dtype=torch.uint8, device=dev)
        prm = descent_params(P, a.dense_rate_iters)
        prm.g_tol = 0.0
        prm.ftol = 0.0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.pecc_gbo_kbatch_bfgs_descend(d, x, bo, 1, 0, 1000, prm.c(), res_b, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        it = P.results(res_b)["iters"].astype(np.int64)
        mat = 2000 * 2000 * 4
        byts = float(np.maximum(2 * it - 5, 0).sum()) * mat
        busy = min(B, torch.cuda.get_device_properties(dev).multi_processor_count)
        out[str(B)] = {"starts": B, "outer_iters_min": int(it.min()), "outer_iters_max": int(it.max()),
                       "kernel_ms": ms, "matrix_bytes": byts, "GBs": byts / ms / 1e6,
                       "busy_cus": busy, "GBs_per_busy_cu": byts / ms / 1e6 / busy}
        print(f"[bench] dense k=1 matrix pass, {B} starts x {int(it.max())} outer iterations: "
              f"{ms:.1f} ms, {byts / ms / 1e9:.3f} TB/s, {byts / ms / 1e6 / busy:.1f} GB/s per CU",
              file=sys.stderr, flush=True)
        del ws
    return out


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--max-iter", type=int, default=5000)
    ap.add_argument("--plain-sample", type=int, default=0,
                    help="instances timed one call each (0: every instance of the batch)")
    ap.add_argument("--sweep-batch", type=int, default=65536, help="instances in the HBM sweep test")
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--pipeline-streams", type=int, default=4,
                    help="streams of the pipelined main-step measurement (1: skip)")
    ap.add_argument("--no-tau", action="store_true", help="skip the tau64 ablation")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the standalone sweep roofline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain single-instance path")
    ap.add_argument("--no-restarts", action="store_true", help="skip the batched restart workload")
    ap.add_argument("--no-gbo", action="store_true", help="skip the geometric batch workload")
    ap.add_argument("--no-lp", action="store_true", help="skip the learned-proposal workload")
    ap.add_argument("--no-adjust", action="store_true", help="skip the container adjustment")
    ap.add_argument("--no-sed", action="store_true", help="skip the SED chains")
    ap.add_argument("--no-kbatch", action="store_true", help="skip the k-batch partition study")
    ap.add_argument("--no-framework", action="store_true", help="skip the Alg. 4 framework runs")
    ap.add_argument("--framework-rounds", type=int, default=3)
    ap.add_argument("--framework-sed-iters", type=int, default=10)
    ap.add_argument("--tune", action="store_true",
                    help="main step with the autotuner's list cutoff / skin (default 2.3 / 0.15: "
                         "the tuner's early-iteration cost does not predict the tail-bound step)")
    ap.add_argument("--kbatch-ks", default="1,2,3,5,7,10,15", help="batch counts of the study")
    ap.add_argument("--kbatch-dense-ks", default="1,2,5,6,10", help="batch counts, dense matrices")
    ap.add_argument("--kbatch-dense-instances", type=int, default=256,
                    help="random starts of the dense-matrix study (0: skip)")
    ap.add_argument("--dense-rate-iters", type=int, default=200,
                    help="outer iterations of the fixed-length dense k = 1 throughput runs (0: skip)")
    ap.add_argument("--kbatch-instances", type=int, default=512,
                    help="random starts per setting (more than the CUs: the rate reflects the mean)")
    ap.add_argument("--sed-iters", type=int, default=10, help="SED iterations of the chains")
    ap.add_argument("--lp-restarts", type=int, default=20000, help="restarts of training data")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle descents (0: the whole batch)")
    ap.add_argument("--cpu-cores", type=int, default=0, help="oracle processes (0: host cores, max 16)")
    ap.add_argument("--sections-out", default=os.path.join("gpurun_out", "bench_sections.json"),
                    help="file that receives every section of the run as JSON ('' : none)")
    return ap.parse_args(argv)


def descent_params(P, max_iter):
    # FP32 working-precision stop: relative decrease below 1e-7 over 20
    # iterations, or ||g||_2 <= 1e-6.  The contact margin 1e-4 (about 26 FP32
    # ulps of a coordinate near |x| = 35) lets the FP32 descent aim inside the
    # set that the FP64 check of unit circles calls feasible.  The
    # sufficient-decrease test moves to FP64 once E < 3e-6: on twelve 256-start
    # workloads that keeps the FP64-feasible counts of 1e-4 (within two starts
    # on each) at less cost, while never moving (0) loses feasible layouts.
    return P.DescentParams(max_iter=max_iter, g_tol=1e-6, ftol=1e-7, ftol_window=20,
                           contact_margin=1e-4, tau64=3e-6)


def algorithmic_flops(res, n, m):
    """Flops the method needs for the recorded work:
    10 per listed pair (i<j) and 10 per circle per evaluation, and the
    L-BFGS two-loop (16 m n) plus the curvature update (8 n) per iteration."""
    return float((10.0 * res["pair_evals"] + 10.0 * n * res["evals"]
                  + (16.0 * m * n + 8.0 * n) * res["iters"]).sum())


def _oracle_descent(args):
    xy, R, max_iter = args
    import oracle
    P = oracle.DescentParams(max_iter=max_iter, g_tol=1e-12, ftol=1e-7, ftol_window=20)
    t0 = time.perf_counter()
    _, res, _ = oracle.descend(xy.astype(np.float64), R, P)
    return time.perf_counter() - t0, res


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(inst, max_iter, sample, cores, gpu_pairs_per_eval=None):
    import multiprocessing as mp
    import oracle
    import synth
    oracle.lib()   # built before the pool forks
    # one descent on one thread at the C1 and C2 shapes
    single = {}
    for tag, one in (("C1_n20", synth.C1()), ("C2_n1000", synth.C2(1))):
        dt, res = _oracle_descent((one.instance(0), float(one.R[0]), 2000 if tag == "C1_n20" else max_iter))
        single[tag] = {"seconds": dt, "iters": res["iters"], "status": res["status"]}
    jobs = [(inst.instance(b), float(inst.R[b]), max_iter) for b in range(sample)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        out = pool.map(_oracle_descent, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    iters = sum(r["iters"] for _, r in out)
    evals = sum(r["evals"] for _, r in out)
    n = inst.instance(0).shape[0]
    feas = sum(r["status"] == "FEASIBLE" for _, r in out)
    return {"value": sample / wall, "unit": "descents/s", "cores": cores, "kind": "oracle",
            "sample": (f"{sample} of the {inst.B} n={n} R={inst.R[0]} starts, FP64 brute-force "
                       f"L-BFGS descents over {cores} processes; {iters} iterations, "
                       f"{evals} evaluations of n(n-1)/2 = {n * (n - 1) // 2} pairs; "
                       f"{feas} feasible; wall {wall:.1f} s"),
            "pair_evals_per_s_bruteforce": evals * n * (n - 1) / 2 / wall,
            "pair_evals_per_s_list_equivalent": (evals * gpu_pairs_per_eval / wall
                                                 if gpu_pairs_per_eval else None),
            "list_equivalent_note": "oracle evaluations x the GPU run's mean listed pairs (i<j) per evaluation",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_thread_descent": single}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(instances are independent: a multi-GPU run would shard the batch with no "
              "exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2303_02650_amd as P
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] {P.version()} on {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)

    inst = synth.C2(a.batch)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy0 = torch.from_numpy(inst.xy.reshape(-1)).to(dev)
    xy = torch.empty_like(xy0)
    params = descent_params(P, a.max_iter)
    main_tune = None
    if a.tune:
        # list cutoff / rebuild distance / cell side measured on a 64-start
        # sample of this workload (cost per iteration; same outcomes)
        from dataclasses import replace
        from paper_2303_02650_amd import autotune as AT
        main_tune = AT.tune_descent(inst.offset, inst.R, inst.xy, params, sample=64, reps=2)
        tb = main_tune["best"]
        params = replace(params, cutoff=tb["cutoff"], skin_half=tb["skin_half"],
                         cell_size=tb["cell_size"])
        print(f"[bench] main-step autotune: {tb}", file=sys.stderr, flush=True)
    ws = torch.empty(P.pecc_lbfgs_descend_workspace_size(d), dtype=torch.uint8, device=dev)
    out = torch.empty(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    e64 = torch.empty(d.B, dtype=torch.float64, device=dev)
    mp_ = torch.empty_like(e64)
    mc_ = torch.empty_like(e64)
    feas = torch.empty(d.B, dtype=torch.int32, device=dev)
    Pc = params.c()

    def descend_once():
        xy.copy_(xy0)
        P.pecc_lbfgs_descend(d, xy, Pc, out, ws)

    def verify_once():
        P.pecc_verify(d, xy, 1e-20, e64, mp_, mc_, feas)

    # eager warm-up (also primes the library's device queries), then capture
    descend_once(); verify_once()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    g_desc, g_ver = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g_desc, stream=side):
            descend_once()
        with torch.cuda.graph(g_ver, stream=side):
            verify_once()
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        g_desc.replay(); g_ver.replay()
    torch.cuda.synchronize()
    print(f"[bench] warm-up done ({a.warmup} steps)", file=sys.stderr, flush=True)

    # ---- timed region: K steps --------------------------------------------
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in evs:
        e0.record(stream)
        g_desc.replay()
        e1.record(stream)
        g_ver.replay()
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    desc_ms = [e0.elapsed_time(e1) for e0, e1, _ in evs]
    ver_ms = [e1.elapsed_time(e2) for _, e1, e2 in evs]
    ms_per_step = wall * 1e3 / a.steps
    res = P.results(out)
    f = feas.cpu().numpy()
    value = a.batch / (ms_per_step / 1e3)
    pair_evals = int(res["pair_evals"].sum())
    status_counts = {P.STATUS[s]: int((res["status"] == s).sum()) for s in np.unique(res["status"])}
    print(f"[bench] timed {a.steps} steps: {ms_per_step:.2f} ms/step, descent kernel "
          f"{np.mean(desc_ms):.2f} ms, verify {np.mean(ver_ms):.3f} ms; status {status_counts}",
          file=sys.stderr, flush=True)

    # roofline of the descent kernel: algorithmic flops / kernel time
    flops = algorithmic_flops(res, N_CIRCLES, params.m)
    t_desc = float(np.mean(desc_ms)) / 1e3
    achieved_tf = flops / t_desc / 1e12
    roof = {"kernel": "lbfgs_descend_kernel", "bound": "alu", "achieved": achieved_tf,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved_tf / FP32_PEAK_TFLOPS,
            "traffic": DESCENT_TRAFFIC_BYTES_256 if (a.batch == 256 and a.max_iter == 5000) else None,
            "per_launch_flops": flops, "avg_launch_ms": t_desc * 1e3,
            # the running kernel is bound by vector-instruction issue, most
            # of which are not algorithmic flops (counter profile)
            "valu_instructions_per_wave_eval": DESCENT_VALU_PER_WAVE_EVAL_256 if a.batch == 256 else None,
            "valu_active_share_of_wave_time": DESCENT_VALU_ACTIVE_SHARE_256 if a.batch == 256 else None,
            "busy_cu_share": float(res["iters"].mean() / max(1, res["iters"].max()))}
    # the same fraction over the CU time the descents actually hold (one
    # instance per CU; a CU idles once its descent has ended)
    roof["frac_of_busy_cus"] = roof["frac"] / max(roof["busy_cu_share"], 1e-9)

    line = {
        # value: descents/s of the batched step; pair-evals/s and the plain
        # path's rate are the other quantities of the metric, reported beside it
        "metric": "L-BFGS descents/sec and pair-evals/sec at n=1000, batched FP32 vs plain, to E<1e-20",
        "value": value, "unit": "descents/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "dtype_note": "FP64 in the verify and in the sufficient-decrease test near E = 0",
        "data": "synthetic",
        "config": {"workload": f"{a.batch} random starts, n={N_CIRCLES}, R={R_C2}, m=10, "
                               f"max_iter={a.max_iter}",
                   "instances": a.batch, "n": N_CIRCLES, "R": R_C2,
                   "list_cutoff": params.cutoff, "skin_half": params.skin_half,
                   "cell_size": params.cell_size},
        "pair_evals_per_s": pair_evals / (ms_per_step / 1e3),
        "step_ms_events_median": float(np.median(np.array(desc_ms) + np.array(ver_ms))),
        "descent_ms_events_median": float(np.median(desc_ms)),
        "feasible_fraction": float(f.mean()),
        "status_counts": status_counts,
        "iters_mean": float(res["iters"].mean()), "evals_mean": float(res["evals"].mean()),
        "E64_final_mean": float(e64.cpu().numpy().mean()),
        "roofline_descent": roof,
        # the FP64 verify of the same step: 5 FP64 flops per pair distance
        # (two differences, two squares, a sum) over all n(n-1)/2 pairs
        "roofline_verify": {
            "kernel": "verify_kernel", "bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
            "per_launch_flops": 5.0 * a.batch * N_CIRCLES * (N_CIRCLES - 1) / 2,
            "avg_launch_ms": float(np.mean(ver_ms)),
            "achieved": 5.0 * a.batch * N_CIRCLES * (N_CIRCLES - 1) / 2 / (float(np.mean(ver_ms)) / 1e3) / 1e12},
    }
    line["roofline_verify"]["frac"] = line["roofline_verify"]["achieved"] / FP64_PEAK_TFLOPS
    if main_tune is not None:
        line["autotune"] = {"chosen": main_tune["best"], "sample_instances": 64,
                            "table": main_tune["table"]}

    # ---- ablation of the FP64 threshold of the sufficient-decrease test ----
    # The FP64 regime starts once min(E32, E1) < tau64; tau64 = 0 keeps every
    # test in FP32.  Same starts, one launch each, FP64 verify of the results.
    if not a.no_tau:
        from dataclasses import replace
        abl = {}
        xt_ = torch.empty_like(xy0)
        outt = torch.empty_like(out)
        e64t, feast = torch.empty_like(e64), torch.empty_like(feas)
        for tau in (0.0, 1e-7, 1e-6, 3e-6, 1e-5, 1e-4, 1e-3):
            pt = replace(params, tau64=tau).c()
            xt_.copy_(xy0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.pecc_lbfgs_descend(d, xt_, pt, outt, ws)
            e1.record(stream)
            P.pecc_verify(d, xt_, 1e-20, e64t, None, None, feast)
            torch.cuda.synchronize()
            rt = P.results(outt)
            abl[f"{tau:g}"] = {
                "kernel_ms": e0.elapsed_time(e1), "feasible_fraction": float(feast.float().mean().item()),
                "iters_mean": float(rt["iters"].mean()), "iters_max": int(rt["iters"].max()),
                "E64_mean": float(e64t.mean().item()),
                "status_counts": {P.STATUS[v]: int((rt["status"] == v).sum()) for v in np.unique(rt["status"])}}
            print(f"[bench] tau64 {tau:g}: {abl[f'{tau:g}']['kernel_ms']:.1f} ms, feasible "
                  f"{abl[f'{tau:g}']['feasible_fraction']:.3f}", file=sys.stderr, flush=True)
        line["tau64_ablation"] = {"workload": "the main step's 256 starts, one launch per tau64",
                                  "by_tau64": abl}
        # the contact margin: the descent works on circles of radius 1 + mu;
        # feasibility is decided for unit circles in FP64
        mab = {}
        for mu in (0.0, 1e-5, 1e-4, 1e-3):
            pt = replace(params, contact_margin=mu).c()
            xt_.copy_(xy0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.pecc_lbfgs_descend(d, xt_, pt, outt, ws)
            e1.record(stream)
            P.pecc_verify(d, xt_, 1e-20, e64t, None, None, feast)
            torch.cuda.synchronize()
            rt = P.results(outt)
            mab[f"{mu:g}"] = {
                "kernel_ms": e0.elapsed_time(e1), "feasible_fraction": float(feast.float().mean().item()),
                "iters_mean": float(rt["iters"].mean()),
                "status_counts": {P.STATUS[v]: int((rt["status"] == v).sum()) for v in np.unique(rt["status"])}}
            print(f"[bench] contact margin {mu:g}: {mab[f'{mu:g}']['kernel_ms']:.1f} ms, feasible "
                  f"{mab[f'{mu:g}']['feasible_fraction']:.3f}", file=sys.stderr, flush=True)
        line["contact_margin_ablation"] = {"workload": "the main step's 256 starts, one launch per margin",
                                           "by_margin": mab}

    # ---- container adjustment (Alg. 2) of the 256 descended layouts --------
    if not a.no_adjust:
        xa = xy.clone()                   # the main step's final layouts
        Ra = torch.empty(d.B, dtype=torch.float32, device=dev)
        outa = torch.empty_like(out)
        P.pecc_adjust_container(d, xa, Pc, 1e-4, 35, Ra, outa, ws)       # warm-up
        torch.cuda.synchronize()
        xa.copy_(xy)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.pecc_adjust_container(d, xa, Pc, 1e-4, 35, Ra, outa, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ta = e0.elapsed_time(e1)
        Rh = Ra.cpu().numpy().astype(np.float64)
        da = P.DeviceInstances.from_host(inst.offset, Rh)
        ea, _, _, fa = P.verify(da, xa)
        ra = P.results(outa)
        line["adjust_container"] = {
            "workload": "the 256 descended C2 layouts, 35 rounds, lambda 1e-4 halved each round, "
                        "contact margin 1e-4; feasibility of unit circles checked in FP64 at the returned radii",
            "kernel_ms": ta, "radii_per_s": d.B / (ta / 1e3),
            "R_start": R_C2, "R_mean": float(Rh.mean()), "R_min": float(Rh.min()),
            "R_max": float(Rh.max()), "feasible_fraction": float(fa.cpu().numpy().mean()),
            "iters_mean": float(ra["iters"].mean()), "iters_max": int(ra["iters"].max())}
        print(f"[bench] adjust: {ta:.1f} ms, R mean {Rh.mean():.4f} min {Rh.min():.4f}",
              file=sys.stderr, flush=True)

    # ---- plain single-instance path (one call per instance, no graph) ------
    if not a.no_plain:
        k = min(a.plain_sample or a.batch, a.batch)
        subs = []
        for b in range(k):
            one = synth.pack([inst.instance(b)], [inst.R[b]])
            db = P.DeviceInstances.from_host(one.offset, one.R)
            x0 = torch.from_numpy(one.xy.reshape(-1)).to(dev)
            subs.append((db, x0, torch.empty_like(x0),
                         torch.empty(P.pecc_lbfgs_descend_workspace_size(db), dtype=torch.uint8, device=dev),
                         torch.empty(P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)))
        for db, x0, xw, wsb, ob in subs[:1]:       # warm-up
            xw.copy_(x0); P.pecc_lbfgs_descend(db, xw, Pc, ob, wsb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for db, x0, xw, wsb, ob in subs:
            xw.copy_(x0)
            P.pecc_lbfgs_descend(db, xw, Pc, ob, wsb)
            torch.cuda.synchronize()
        plain_wall = time.perf_counter() - t0
        plain_rate = k / plain_wall
        # the plain calls descend the same starts as the batched step: every
        # final layout must equal the batched one bit for bit
        xb_all = xy.view(-1, 2)
        same = all(torch.equal(xw.view(-1, 2), xb_all[int(inst.offset[b]):int(inst.offset[b + 1])])
                   for b, (_, _, xw, _, _) in enumerate(subs))
        plain_iters = np.array([int(P.results(ob)["iters"][0]) for *_, ob in subs])
        line["plain_descents_per_s"] = plain_rate
        line["batched_over_plain"] = value / plain_rate
        line["plain_instances"] = k
        line["plain_iters_mean"] = float(plain_iters.mean())
        line["plain_results_equal_batched"] = bool(same)
        print(f"[bench] plain: {k} descents in {plain_wall:.3f} s (iterations mean "
              f"{plain_iters.mean():.0f} vs the batch's {res['iters'][:k].mean():.0f}); layouts equal "
              f"to the batched step's: {same}", file=sys.stderr, flush=True)
        del subs

    # ---- batched restarts: 256 converged packings, 5% relocated ------------
    if not a.no_restarts:
        rs = synth.C3_restarts()
        dr = P.DeviceInstances.from_host(rs.offset, rs.R)
        r0 = torch.from_numpy(rs.xy.reshape(-1)).to(dev)
        rx = torch.empty_like(r0)
        rws = torch.empty(P.pecc_lbfgs_descend_workspace_size(dr), dtype=torch.uint8, device=dev)
        rout = torch.empty(dr.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        rf = torch.empty(dr.B, dtype=torch.int32, device=dev)
        re64 = torch.empty(dr.B, dtype=torch.float64, device=dev)

        # measured choice of list cutoff / rebuild distance / cell side on a
        # 64-instance sample of the workload (same outcomes, different cost)
        from dataclasses import replace
        from paper_2303_02650_amd import autotune as AT
        tune = AT.tune_descent(rs.offset, rs.R, rs.xy, params, sample=64, reps=2)
        tb = tune["best"]
        Pr = replace(params, cutoff=tb["cutoff"], skin_half=tb["skin_half"],
                     cell_size=tb["cell_size"]).c()
        print(f"[bench] restarts autotune: {tb}", file=sys.stderr, flush=True)

        def restart_once():
            rx.copy_(r0)
            P.pecc_lbfgs_descend(dr, rx, Pr, rout, rws)
            P.pecc_verify(dr, rx, 1e-20, re64, None, None, rf)

        restart_once()
        torch.cuda.synchronize()
        g_rs = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g_rs, stream=side):
                restart_once()
        torch.cuda.synchronize()
        g_rs.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            g_rs.replay()
        torch.cuda.synchronize()
        rms = (time.perf_counter() - t0) * 1e3 / a.steps
        rr = P.results(rout)
        line["restarts"] = {
            "workload": f"{dr.B} restarts, n in [300,1000], R = sqrt(n/0.84), 5% relocated",
            "descents_per_s": dr.B / (rms / 1e3), "ms_per_step": rms,
            "pair_evals_per_s": float(rr["pair_evals"].sum()) / (rms / 1e3),
            "feasible_fraction": float(rf.cpu().numpy().mean()),
            "status_counts": {P.STATUS[s]: int((rr["status"] == s).sum()) for s in np.unique(rr["status"])},
            "iters_mean": float(rr["iters"].mean()), "iters_max": int(rr["iters"].max()),
            "autotune": {"chosen": {k: tb[k] for k in ("cutoff", "skin_half", "cell_size")},
                         "sample_instances": tune["instances"], "table": tune["table"]}}
        if not a.no_plain:
            # plain path on a sample of the restarts: one call per instance, no graph
            kp = min(a.plain_sample or dr.B, dr.B)
            pl = []
            for b in range(kp):
                one = synth.pack([rs.instance(b)], [rs.R[b]])
                db = P.DeviceInstances.from_host(one.offset, one.R)
                x1 = torch.from_numpy(one.xy.reshape(-1)).to(dev)
                pl.append((db, x1, torch.empty_like(x1),
                           torch.empty(P.pecc_lbfgs_descend_workspace_size(db), dtype=torch.uint8, device=dev),
                           torch.empty(P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)))
            db, x1, xw, wsb, ob = pl[0]
            xw.copy_(x1); P.pecc_lbfgs_descend(db, xw, Pr, ob, wsb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for db, x1, xw, wsb, ob in pl:
                xw.copy_(x1)
                P.pecc_lbfgs_descend(db, xw, Pr, ob, wsb)
                torch.cuda.synchronize()
            prate = kp / (time.perf_counter() - t0)
            line["restarts"]["plain_descents_per_s"] = prate
            line["restarts"]["batched_over_plain"] = line["restarts"]["descents_per_s"] / prate
            line["restarts"]["plain_instances"] = kp
        print(f"[bench] restarts: {rms:.2f} ms/step", file=sys.stderr, flush=True)

    # ---- geometric batch descent: 64 x n=1000, R=34.4, 4 x 4 blocks -------
    if not a.no_gbo:
        c4 = synth.C4(64)
        dg = P.DeviceInstances.from_host(c4.offset, c4.R)
        g0 = torch.from_numpy(c4.xy.reshape(-1)).to(dev)
        gx = torch.empty_like(g0)
        gws = torch.empty(P.pecc_gbo_descend_workspace_size(dg, 4), dtype=torch.uint8, device=dev)
        gout = torch.empty(dg.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        gf = torch.empty(dg.B, dtype=torch.int32, device=dev)
        ge = torch.empty(dg.B, dtype=torch.float64, device=dev)
        from paper_2303_02650_amd import autotune as AT
        gtune = AT.tune_gbo(c4.offset, c4.R, c4.xy, descent_params(P, a.max_iter), sample=16)
        gblocks = int(gtune["best"]["blocks"])
        gws = torch.empty(P.pecc_gbo_descend_workspace_size(dg, gblocks), dtype=torch.uint8, device=dev)
        print(f"[bench] gbo autotune: {gtune['best']}", file=sys.stderr, flush=True)
        gbo = {"autotune": {"chosen_blocks": gblocks, "table": gtune["table"]}}
        for tag, margin, fp64 in (("fp32", 1e-4, 0), ("fp32_margin0", 0.0, 0), ("fp64sweep_margin0", 0.0, 1)):
            gp = descent_params(P, a.max_iter)
            gp.contact_margin = margin
            gpc = gp.c()
            gx.copy_(g0)
            P.pecc_gbo_descend(dg, gx, gpc, gblocks, fp64, gout, gws)      # warm-up
            torch.cuda.synchronize()
            ts = []
            for _ in range(max(1, min(a.steps, 3))):
                gx.copy_(g0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                P.pecc_gbo_descend(dg, gx, gpc, gblocks, fp64, gout, gws)
                e1.record(stream)
                P.pecc_verify(dg, gx, 1e-20, ge, None, None, gf)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            gr = P.results(gout)
            e64 = ge.cpu().numpy()
            ent = {"descents_per_s": dg.B / (np.mean(ts) / 1e3), "kernel_ms": float(np.mean(ts)),
                   "feasible_fraction": float(gf.cpu().numpy().mean()),
                   "outer_iters_mean": float(gr["iters"].mean()),
                   # trials that moved a batch circle beyond the skin (swept
                   # over the cell grid: Alg. 1 does not limit the step)
                   "cell_evals_mean": float(gr["cell_evals"].mean()),
                   "evals_mean": float(gr["evals"].mean()),
                   "status_counts": {P.STATUS[s]: int((gr["status"] == s).sum()) for s in np.unique(gr["status"])},
                   "E64_median": float(np.median(e64))}
            if margin == 0.0:
                rel = np.abs(gr["E32"].astype(np.float64) - e64) / np.maximum(e64, 1e-300)
                ent["reported_E_rel_err_vs_fp64_median"] = float(np.median(rel[e64 > 0])) if (e64 > 0).any() else 0.0
                ent["reported_E_rel_err_vs_fp64_max"] = float(rel[e64 > 0].max()) if (e64 > 0).any() else 0.0
            gbo[tag] = ent
            print(f"[bench] gbo {tag}: {np.mean(ts):.1f} ms", file=sys.stderr, flush=True)
        # the whole-instance descent on the same 64 instances, for comparison
        wws = torch.empty(P.pecc_lbfgs_descend_workspace_size(dg), dtype=torch.uint8, device=dev)
        wp = descent_params(P, a.max_iter).c()
        gx.copy_(g0)
        P.pecc_lbfgs_descend(dg, gx, wp, gout, wws)
        torch.cuda.synchronize()
        gx.copy_(g0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.pecc_lbfgs_descend(dg, gx, wp, gout, wws)
        e1.record(stream)
        P.pecc_verify(dg, gx, 1e-20, ge, None, None, gf)
        torch.cuda.synchronize()
        wr = P.results(gout)
        gbo["lbfgs_whole_instance"] = {
            "descents_per_s": dg.B / (e0.elapsed_time(e1) / 1e3), "kernel_ms": e0.elapsed_time(e1),
            "feasible_fraction": float(gf.cpu().numpy().mean()),
            "iters_mean": float(wr["iters"].mean()),
            "E64_median": float(np.median(ge.cpu().numpy()))}
        line["gbo"] = {"workload": f"64 random starts, n=1000, R=34.4, {gblocks} x {gblocks} blocks "
                                   f"(~{1000 // (gblocks * gblocks)} circles per batch)",
                       **gbo}

    # ---- k-batch descent (Alg. 1) over the four partitions of Sec. 4.1 -----
    if not a.no_kbatch:
        line["kbatch"] = kbatch_study(P, a, dev, stream)

    # ---- learned proposal: 128 x n=1000, R=34.4, 4096 candidates ----------
    if not a.no_lp:
        from paper_2303_02650_amd import proposal as PR
        t0 = time.perf_counter()
        F, Y, st = PR.generate_samples(a.lp_restarts, R_range=(34.3, 34.6), seed=1)
        torch.cuda.synchronize()
        t_gen = time.perf_counter() - t0
        print(f"[bench] lp: {F.shape[0]} samples from {st['restarts']} restarts in {t_gen:.1f} s",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        scorer, hist = PR.train(F, Y, epochs=16, batch_rows=8192, lr=2e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        # kernel timings at the evaluation shape on one converged state
        c5 = synth.C5(128)
        B5, C5c, k5 = c5.B, 4096, 50
        b5 = PR._Batch(1000, c5.R, torch.from_numpy(c5.xy.reshape(-1)).to(dev), PR.ssed_params())
        e5 = b5.descend(b5.xy)
        cc, cd = PR.draw_candidates(np.random.default_rng(7), np.full(B5, 1000), c5.R, C5c)
        ccd, cdd = torch.from_numpy(cc.reshape(-1)).to(dev), torch.from_numpy(cd.reshape(-1)).to(dev)
        feats = torch.empty(B5 * C5c, 8, dtype=torch.float32, device=dev)
        logits = torch.empty(B5 * C5c, dtype=torch.float32, device=dev)
        xy_new = torch.empty_like(b5.xy)
        sel = torch.empty(B5, k5, dtype=torch.int32, device=dev)
        rows = B5 * C5c
        stages = {
            "features": lambda: P.pecc_features(b5.inst, b5.xy, C5c, ccd, cdd, feats),
            "mlp_forward": lambda: P.pecc_mlp_forward(scorer, feats, rows, logits),
            "propose": lambda: P.pecc_propose(b5.inst, b5.xy, C5c, ccd, cdd, logits, k5, sel, xy_new),
        }
        tms = {}
        for name, fn in stages.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            tms[name] = e0.elapsed_time(e1) / reps
        xs = xy_new.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        e_new = b5.descend(xs)
        acc = P.accept(b5.inst, b5.xy.clone(), e5.clone(), xs, e_new)
        e1.record(stream)
        torch.cuda.synchronize()
        tms["descend_verify_accept"] = e0.elapsed_time(e1)
        T = P.MlpTrainer(scorer, max_rows=8192)
        xb8, yb8 = F[:8192].contiguous(), Y[:8192].contiguous()
        T.train_step(xb8, yb8)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(20):
            T.train_step(xb8, yb8)
        e1.record(stream)
        torch.cuda.synchronize()
        t_step = e0.elapsed_time(e1) / 20
        cmp = PR.compare(scorer, R=34.4, instances=128, budget=16, seed=6, xy0=c5.xy).summary()
        fwd_tf = MLP_FLOPS_PER_ROW * rows / (tms["mlp_forward"] / 1e3) / 1e12
        line["learned_proposal"] = {
            "workload": "128 x n=1000, R=34.4 (seed 5), 4096 candidates per instance, top-50 "
                        "distinct; training data from random relocations of converged "
                        "n=1000 layouts, R in [34.3, 34.6]",
            "training_samples": int(F.shape[0]), "training_label_mean": float(Y.mean().item()),
            "sample_generation_s": t_gen, "restarts_per_s": st["restarts"] / t_gen,
            "training_s": t_train, "training_loss_per_epoch": hist,
            "train_step_ms_8192_rows": t_step, "train_rows_per_s": 8192 / (t_step / 1e3),
            "ssed_step_ms": tms, "candidates_scored_per_s": rows / ((tms["features"] + tms["mlp_forward"]) / 1e3),
            "roofline_mlp_forward": {"kernel": "mlp_forward_kernel", "bound": "mfma",
                                     "achieved": fwd_tf, "peak": BF16_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": fwd_tf / BF16_PEAK_TFLOPS,
                                     "traffic": None, "per_launch_flops": MLP_FLOPS_PER_ROW * rows,
                                     "avg_launch_ms": tms["mlp_forward"]},
            "vs_random": cmp}
        print(f"[bench] lp: train {t_train:.1f} s, stages {tms}, vs random {cmp}", file=sys.stderr,
              flush=True)
        del F, Y

    # ---- SED (Alg. 5): 128 chains, n=1000, R=34.4 ---------------------------
    if not a.no_sed:
        from paper_2303_02650_amd.sed import SedChains
        c5 = synth.C5(128)
        d5 = P.DeviceInstances.from_host(c5.offset, c5.R)
        x5 = torch.from_numpy(c5.xy.reshape(-1)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch = SedChains(d5, x5, descent_params(P, a.max_iter), M=25, seed=17)
        info = ch.run(a.sed_iters)
        e_start = ch.E_start.cpu().numpy()
        e_best = ch.E_best.cpu().numpy()
        line["sed"] = {
            "workload": f"128 chains, n=1000, R=34.4 (seed 5), {a.sed_iters} SED iterations, "
                        "J-controlled candidates (M=25), x+r perturbation r in U(-0.8,0.8), "
                        "Eq. 18 selection",
            "seconds": time.perf_counter() - t0, "iterations": info["iterations"],
            "descents": info["descents"],
            "descents_per_s": info["descents"] / (time.perf_counter() - t0),
            "feasible_after_first_descent": float((e_start <= 1e-25).mean()),
            "feasible_after_sed": float((e_best <= 1e-25).mean()),
            "E_best_median": float(np.median(e_best)), "E_start_median": float(np.median(e_start))}
        ff = ch.first_feasible.cpu().numpy()
        line["sed"]["mean_descents_to_first_feasible"] = float(ff[ff > 0].mean()) if (ff > 0).any() else None
        print(f"[bench] sed: {line['sed']}", file=sys.stderr, flush=True)
        del ch

    # ---- the framework of Alg. 4: 64 runs of n = 1000 ----------------------
    if not a.no_framework:
        from paper_2303_02650_amd.framework import Framework
        Rb = float(np.sqrt(1000 / 0.85))
        t0 = time.perf_counter()
        fw = Framework(1000, [Rb] * 64, descent_params(P, a.max_iter), M=25,
                       s_iter=a.framework_sed_iters, seed=23)
        t_init = time.perf_counter() - t0
        info = fw.run(rounds=a.framework_rounds)
        Rbest = np.array(info["R_best"])
        line["framework"] = {
            "workload": f"64 runs of n=1000, reference radius R_b = sqrt(1000/0.85) = {Rb:.4f} "
                        f"(a synthetic stand-in: density 0.85), {a.framework_rounds} rounds of SED "
                        f"({a.framework_sed_iters} iterations, M=25) + container adjustment",
            "seconds_initial": t_init, "seconds_rounds": info["seconds"],
            "R_initial_mean": float(np.mean(info["R_initial"])),
            "R_best_mean": float(Rbest.mean()), "R_best_min": float(Rbest.min()),
            "density_best_mean": float(np.mean(1000 / Rbest ** 2)),
            "below_R_b_fraction": float((Rbest < Rb).mean()),
            "history": info["history"]}
        print(f"[bench] framework: R {np.mean(info['R_initial']):.4f} -> {Rbest.mean():.4f} "
              f"(min {Rbest.min():.4f}) in {info['seconds']:.1f} s", file=sys.stderr, flush=True)

    # ---- standalone list sweep at an HBM-sized batch -----------------------
    if not a.no_sweep:
        # the C3 shape (256 random starts, n in [300, 1000]): ~5 MB, cache
        # resident, so its rate is an effective one, not an HBM figure
        c3 = synth.C3(256)
        dc3 = P.DeviceInstances.from_host(c3.offset, c3.R)
        xc3 = torch.from_numpy(c3.xy.reshape(-1)).to(dev)
        rc3, cc3 = P.build_neighbors(dc3, xc3, 2.3, 0.0, P.LIST_LOCAL16)
        Ec3 = torch.empty(dc3.B, dtype=torch.float32, device=dev)
        gc3 = torch.empty_like(xc3)
        for _ in range(5):
            P.pecc_energy_grad(dc3, xc3, rc3, cc3, cc3.numel(), P.LIST_LOCAL16, 1.0, Ec3, gc3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(100):
            P.pecc_energy_grad(dc3, xc3, rc3, cc3, cc3.numel(), P.LIST_LOCAL16, 1.0, Ec3, gc3)
        e1.record(stream)
        torch.cuda.synchronize()
        t3 = e0.elapsed_time(e1) / 1e3 / 100
        tn3 = dc3.total_n
        b3 = 8 * tn3 + 8 * tn3 + 4 * (tn3 + dc3.B) + 2 * cc3.numel() + 4 * dc3.B
        line["sweep_c3_effective"] = {
            "kernel": "energy_grad_kernel", "instances": dc3.B, "circles": tn3,
            "per_launch_bytes": b3, "avg_launch_ms": t3 * 1e3,
            "effective_GBs": b3 / t3 / 1e9, "pair_evals_per_s": (cc3.numel() // 2) / t3,
            "note": "cache-resident working set: an effective rate, not an HBM figure"}
        del c3, dc3, xc3, rc3, cc3, Ec3, gc3
        torch.cuda.empty_cache()          # fresh allocations for the 2.5 GB of sweep buffers
        reps = a.sweep_batch // a.batch
        big = synth.pack([inst.instance(b) for b in range(a.batch)] * reps, list(inst.R) * reps)
        dbig = P.DeviceInstances.from_host(big.offset, big.R)
        xb = torch.from_numpy(big.xy.reshape(-1)).to(dev)
        # the compact list: uint16 instance-local indices, both orientations
        # (2 bytes per entry, 4 per listed pair)
        row, col = P.build_neighbors(dbig, xb, 2.3, 0.0, P.LIST_LOCAL16)
        E = torch.empty(dbig.B, dtype=torch.float32, device=dev)
        g = torch.empty_like(xb)
        # first touches of the fresh output buffers are slower, and the clocks
        # take some tens of launches to settle
        for _ in range(40):
            P.pecc_energy_grad(dbig, xb, row, col, col.numel(), P.LIST_LOCAL16, 1.0, E, g)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.sweep_reps):
            P.pecc_energy_grad(dbig, xb, row, col, col.numel(), P.LIST_LOCAL16, 1.0, E, g)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / a.sweep_reps
        tn = dbig.total_n
        npairs = col.numel() // 2
        # per instance 8n (positions) + 8n (gradient) + 4(n+1) (row) + 4P
        # (P listed pairs) + 4 (E)
        bytes_alg = 8 * tn + 8 * tn + 4 * (tn + dbig.B) + 4 * npairs + 4 * dbig.B
        # the other list forms at the same shape, for comparison
        forms = {}
        for fname, form in (("int32_each_pair_once", P.LIST_HALF), ("int32_both_orientations", P.LIST_FULL)):
            rf_, cf_ = P.build_neighbors(dbig, xb, 2.3, 0.0, form)
            for _ in range(3):
                P.pecc_energy_grad(dbig, xb, rf_, cf_, cf_.numel(), form, 1.0, E, g)
            e0.record(stream)
            for _ in range(5):
                P.pecc_energy_grad(dbig, xb, rf_, cf_, cf_.numel(), form, 1.0, E, g)
            e1.record(stream)
            torch.cuda.synchronize()
            tf = e0.elapsed_time(e1) / 1e3 / 5
            bf = 16 * tn + 4 * (tn + dbig.B) + 4 * cf_.numel() + 4 * dbig.B
            forms[fname] = {"avg_launch_ms": tf * 1e3, "list_bytes_per_launch": bf,
                            "GBs_on_these_bytes": bf / tf / 1e9,
                            "GBs_on_4P_bytes": bytes_alg / tf / 1e9}
            del rf_, cf_
        print(f"[bench] sweep list forms: {forms}", file=sys.stderr, flush=True)
        gbs = bytes_alg / t / 1e9
        # plain device copy of a known size: measured copy bandwidth, and the
        # reference dispatch that scales the profiler's byte counters
        cal_src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        cal_dst = torch.empty_like(cal_src)
        cal_dst.copy_(cal_src)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            cal_dst.copy_(cal_src)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 2 * COPY_BYTES / (e0.elapsed_time(e1) / 5 / 1e3) / 1e9
        del cal_src, cal_dst
        line["roofline_sweep"] = {
            "kernel": "energy_grad_kernel", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": SWEEP_TRAFFIC_BYTES_65536 if dbig.B == 65536 else None,
            "copy_GBs_measured": copy_gbs,
            "per_launch_bytes": bytes_alg, "avg_launch_ms": t * 1e3,
            "instances": dbig.B, "listed_pairs": int(npairs),
            "list_form": "uint16 instance-local indices, both orientations",
            "pair_evals_per_s": npairs / t, "other_list_forms": forms}
        print(f"[bench] sweep: {dbig.B} instances, {bytes_alg / 1e9:.2f} GB in {t * 1e3:.3f} ms "
              f"= {gbs:.0f} GB/s", file=sys.stderr, flush=True)
        del big, dbig, xb, row, col, E, g

    # ---- the same steps pipelined over streams -----------------------------
    # Consecutive steps (each the same 256 starts: reset, one persistent
    # launch, its verify, own buffers) on a ring of streams: a launch's
    # workgroups leave their CU once its queue is empty, so the next
    # launches' work fills the CUs that a step's slowest descents leave idle.
    # Every descent runs to its end and every result is checked against the
    # timed step's.  Last of the GPU sections, so that its extra streams
    # cannot touch the graph replays of the others.  Plain launches, not graph replays: replays of captured
    # graphs on more streams than the device has hardware queues were seen
    # to overlap consecutive replays on one stream.
    if a.pipeline_streams > 1:
        sets = []
        for _ in range(a.pipeline_streams):
            f64 = [torch.empty(d.B, dtype=torch.float64, device=dev) for _ in range(3)]
            sets.append((torch.cuda.Stream(), torch.empty_like(xy0), torch.empty_like(out),
                         torch.empty_like(ws), *f64, torch.empty_like(feas)))
        torch.cuda.synchronize()
        kp = a.steps * a.pipeline_streams
        t0 = time.perf_counter()
        for k in range(kp):
            st, xs, outs, wss, e64s, mps, mcs, fes = sets[k % len(sets)]
            with torch.cuda.stream(st):
                xs.copy_(xy0)
                P.pecc_lbfgs_descend(d, xs, Pc, outs, wss)
                P.pecc_verify(d, xs, 1e-20, e64s, mps, mcs, fes)
        torch.cuda.synchronize()
        wall_p = time.perf_counter() - t0
        same = all(torch.equal(xs, xy) and torch.equal(outs, out) and torch.equal(fes, feas)
                   for _, xs, outs, _, _, _, _, fes in sets)
        line["pipelined"] = {
            "streams": len(sets), "steps": kp, "ms_per_step": wall_p * 1e3 / kp,
            "descents_per_s": a.batch * kp / wall_p, "results_equal_to_timed_step": bool(same),
            "note": "the same step on a ring of streams; not the headline value"}
        print(f"[bench] pipelined over {len(sets)} streams: {wall_p * 1e3 / kp:.2f} ms/step, "
              f"results equal: {same}", file=sys.stderr, flush=True)

    # ---- FP64 oracle on the host cores (bounded sample) --------------------
    if not a.no_cpu:
        cores = a.cpu_cores or max(1, min(16, len(os.sched_getaffinity(0))))
        sample = min(a.cpu_sample or a.batch, a.batch)
        print(f"[bench] oracle CPU baseline: {sample} descents on {cores} processes ...",
              file=sys.stderr, flush=True)
        line["cpu_baseline"] = run_cpu_baseline(inst, a.max_iter, sample, cores,
                                                gpu_pairs_per_eval=pair_evals / max(1, int(res["evals"].sum())))

    if a.sections_out:
        os.makedirs(os.path.dirname(os.path.abspath(a.sections_out)), exist_ok=True)
        with open(a.sections_out, "w") as fh:
            json.dump(line, fh, indent=1)
        print(f"[bench] every section written to {a.sections_out}", file=sys.stderr, flush=True)
    print(json.dumps(compact_line(line, a.sections_out)), flush=True)


def _pick(d, keys):
    return {k: d[k] for k in keys if k in d}


def compact_line(line, sections_file=None):
    """The one JSON line of the run: the headline metric, the plain path,
    the sweep's HBM roofline (with the descent kernel's ALU fraction beside
    it) and the CPU baseline.  Every other section goes to the sections
    file; this line stays well under 2 KB."""
    out = _pick(line, ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                       "higher_is_better", "scaling", "vs_baseline", "dtype", "data"))
    out["config"] = _pick(line.get("config", {}), ("workload", "instances", "n", "R"))
    out.update(_pick(line, ("pair_evals_per_s", "feasible_fraction", "descent_ms_events_median",
                            "plain_descents_per_s", "batched_over_plain", "plain_instances")))
    desc = line.get("roofline_descent")
    desc_c = _pick(desc, ("kernel", "bound", "achieved", "peak", "unit", "frac", "avg_launch_ms",
                          "busy_cu_share")) if desc else None
    sweep = line.get("roofline_sweep")
    if sweep:
        roof = _pick(sweep, ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                             "per_launch_bytes", "avg_launch_ms", "instances", "listed_pairs"))
        roof["descent"] = desc_c
        out["roofline"] = roof
    elif desc_c:
        out["roofline"] = desc_c
    cpu = line.get("cpu_baseline")
    if cpu:
        out["cpu_baseline"] = _pick(cpu, ("value", "unit", "cores", "kind", "sample"))
    if sections_file:
        out["sections_file"] = sections_file
    return out


if __name__ == "__main__":
    main()
