"""FP64 CPU oracle for the circle-packing penalty-energy descent.

TEST INFRASTRUCTURE ONLY.  The oracle is the independent checker of the HIP
library: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the GPU path.

The arithmetic lives in ``pecc_oracle.c`` (plain C, FP64, brute force over all
pairs, built with ``-O2 -ffp-contract=off``); this module only marshals numpy
arrays through ctypes.  Each function names the part of the paper it follows:

  energy_grad        Def. 3.1 / Def. 3.2 (Eq. 3, Eq. 5) and their gradient
  batch_energy_grad  Eq. 7 (batch energy of Sec. 4.1)
  neighbors          Gamma(i) of Sec. 4.3, FP64 predicate on FP32 inputs
  two_loop           H g for the inverse update of Eq. 10-11 (limited memory)
  descend            Alg. 1 with one batch, L-BFGS reading of Eq. 8-11
  gbo_descend        Alg. 1 with geometric batches (2D grid blocks, 4 colours)
  verify             Eq. 1-2 checked through E (Eq. 5) in FP64
  container_energy   U of Eq. 12 (radius as a variable) and its gradient
  adjust_container   Alg. 2: 35 minimisations of U with lambda halved

The solution-space exploring and descent heuristic (Sec. 5, Alg. 5) lives in
``pecc_oracle_sed.c``: philox (Philox4x64-10), sed_shift / sed_perturb,
sed_uniform, sed_J, sed_select, sed.

The k-batch partitions of Sec. 4.1, the batch descent of Alg. 1 with the
batches visited in order and the adaptive neighbor maintenance of Alg. 3
live in ``pecc_oracle_part.c``: partition (sector, annulus, fence, random),
gamma_energy (E over a neighbor structure built elsewhere), gbo_seq_descend.

The learned proposal of the perturbation step (Sec. 5, Alg. 5) lives in
``pecc_oracle_lp.c``; the network is the project's own definition:

  bf16_round         FP32 -> BF16 round-to-nearest-even
  features           8 local features of a candidate (circle, destination)
  mlp_forward        8 -> 64 -> 64 -> 1 erf-GELU network, FP64
  mlp_grad           mean BCE-with-logits loss and its gradient, FP64
  adam               one Adam step, FP64
  propose            top-k distinct circles by score, and their relocation
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "pecc_oracle.c"), os.path.join(_HERE, "pecc_oracle_lp.c"),
         os.path.join(_HERE, "pecc_oracle_sed.c"), os.path.join(_HERE, "pecc_oracle_part.c")]
_HDRS = [os.path.join(_HERE, "pecc_oracle_types.h")]
_LIB = os.path.join(_HERE, "_pecc_oracle.so")

STATUS = {0: "RUNNING", 1: "FEASIBLE", 2: "STATIONARY", 3: "CONVERGED",
          4: "STALLED", 5: "MAX_ITER", 6: "NONFINITE"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no contraction)."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _stale() -> bool:
    return not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                           for f in _SRCS + _HDRS)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        L = C.CDLL(_LIB)
        dp, fp, ip = C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int32)
        L.oracle_energy_grad.restype = C.c_double
        L.oracle_energy_grad.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp, dp, dp]
        L.oracle_batch_energy_grad.restype = C.c_double
        L.oracle_batch_energy_grad.argtypes = [C.c_int, dp, C.c_double, C.c_double, ip, dp]
        L.oracle_neighbors.restype = C.c_int64
        L.oracle_neighbors.argtypes = [C.c_int, fp, C.c_double, ip, ip, C.c_int64]
        L.oracle_two_loop.restype = None
        L.oracle_two_loop.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp]
        L.oracle_descend.restype = C.c_int
        L.oracle_descend.argtypes = [C.c_int, dp, C.c_double, C.c_void_p, C.c_void_p, dp]
        L.oracle_verify.restype = C.c_int
        L.oracle_verify.argtypes = [C.c_int, fp, C.c_double, C.c_double, dp]
        L.oracle_gbo_batches.restype = C.c_int
        L.oracle_gbo_batches.argtypes = [C.c_int, dp, C.c_double, C.c_int, ip, ip]
        L.oracle_gbo_descend.restype = C.c_int
        L.oracle_gbo_descend.argtypes = [C.c_int, dp, C.c_double, C.c_void_p, C.c_void_p,
                                         C.c_void_p, dp]
        L.oracle_container_energy.restype = C.c_double
        L.oracle_container_energy.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp]
        L.oracle_adjust_container.restype = C.c_int
        L.oracle_adjust_container.argtypes = [C.c_int, dp, dp, C.c_void_p, C.c_double, C.c_int,
                                              C.c_void_p]
        u64 = C.c_uint64
        L.oracle_philox4x64.restype = None
        L.oracle_philox4x64.argtypes = [C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
        L.oracle_sed_shift.restype = None
        L.oracle_sed_shift.argtypes = [C.c_int, u64, C.c_int32, C.c_int32, C.c_int32, fp]
        L.oracle_sed_perturb.restype = None
        L.oracle_sed_perturb.argtypes = [C.c_int, fp, u64, C.c_int32, C.c_int32, C.c_int32, fp]
        L.oracle_sed_uniform.restype = C.c_double
        L.oracle_sed_uniform.argtypes = [u64, C.c_int32, C.c_int32]
        L.oracle_sed_J.restype = C.c_int
        L.oracle_sed_J.argtypes = [C.c_double, C.c_int]
        L.oracle_sed_select.restype = C.c_int
        L.oracle_sed_select.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_int]
        L.oracle_sed.restype = C.c_int
        L.oracle_sed.argtypes = [C.c_int, dp, C.c_double, C.c_void_p, C.c_int, C.c_int, C.c_double,
                                 u64, C.c_int32, C.c_void_p]
        i64 = C.c_int64
        L.oracle_bf16_round.restype = None
        L.oracle_partition.argtypes = [C.c_int, fp, C.c_int, C.c_int, u64, C.c_int32, ip]
        L.oracle_partition.restype = C.c_int
        L.oracle_gamma_energy.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double]
        L.oracle_gamma_energy.restype = C.c_double
        L.oracle_gbo_seq_descend.argtypes = [C.c_int, dp, C.c_double, C.c_void_p, ip, C.c_int,
                                             C.c_void_p, C.c_void_p, dp, dp]
        L.oracle_bfgs_update.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_bfgs_update.restype = None
        L.oracle_gbo_seq_descend.restype = C.c_int
        L.oracle_bf16_round.argtypes = [i64, fp, fp]
        L.oracle_features.restype = C.c_int
        L.oracle_features.argtypes = [C.c_int, fp, C.c_double, C.c_int, ip, fp, dp]
        L.oracle_mlp_forward.restype = None
        L.oracle_mlp_forward.argtypes = [dp, C.c_int, i64, dp, dp]
        L.oracle_mlp_grad.restype = C.c_double
        L.oracle_mlp_grad.argtypes = [dp, C.c_int, i64, dp, dp, dp]
        L.oracle_adam.restype = None
        L.oracle_adam.argtypes = [C.c_int, dp, dp, dp, dp, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_double]
        L.oracle_propose.restype = C.c_int
        L.oracle_propose.argtypes = [C.c_int, fp, C.c_int, ip, fp, fp, C.c_int, ip, fp]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def energy_grad(xy, R: float, rad: float = 1.0):
    """E, E_pair, E_cont and dE/dx (shape (n, 2)) at FP64 positions xy (n, 2)."""
    xy, p = _d(np.asarray(xy).reshape(-1, 2))
    n = xy.shape[0]
    g = np.zeros((n, 2), dtype=np.float64)
    ep, ec = C.c_double(), C.c_double()
    E = lib().oracle_energy_grad(n, p, float(R), float(rad), C.byref(ep), C.byref(ec),
                                 g.ctypes.data_as(C.POINTER(C.c_double)))
    return E, ep.value, ec.value, g


def energy(xy, R: float, rad: float = 1.0) -> float:
    xy, p = _d(np.asarray(xy).reshape(-1, 2))
    return lib().oracle_energy_grad(xy.shape[0], p, float(R), float(rad), None, None, None)


def batch_energy_grad(xy, R: float, mask, rad: float = 1.0):
    """Eq. 7 batch energy of the circles with mask != 0 and its gradient."""
    xy, p = _d(np.asarray(xy).reshape(-1, 2))
    m = np.ascontiguousarray(mask, dtype=np.int32)
    g = np.zeros_like(xy)
    E = lib().oracle_batch_energy_grad(xy.shape[0], p, float(R), float(rad),
                                       m.ctypes.data_as(C.POINTER(C.c_int32)),
                                       g.ctypes.data_as(C.POINTER(C.c_double)))
    return E, g


def neighbors(xy32, cutoff: float = 2.3):
    """Half pair set {(i, j): i < j, l_ij < cutoff} (FP64 test on FP32 input),
    ordered by i then j; returns int32 arrays (pi, pj)."""
    xy, p = _f(np.asarray(xy32, dtype=np.float32).reshape(-1, 2))
    n = xy.shape[0]
    L = lib()
    cnt = L.oracle_neighbors(n, p, float(cutoff), None, None, 0)
    pi = np.zeros(max(cnt, 1), dtype=np.int32)
    pj = np.zeros(max(cnt, 1), dtype=np.int32)
    L.oracle_neighbors(n, p, float(cutoff), pi.ctypes.data_as(C.POINTER(C.c_int32)),
                       pj.ctypes.data_as(C.POINTER(C.c_int32)), cnt)
    return pi[:cnt], pj[:cnt]


def two_loop(S, Y, g):
    """r = H g for the stored pairs S, Y (k rows, oldest first)."""
    S, ps = _d(np.atleast_2d(S))
    Y, py = _d(np.atleast_2d(Y))
    g, pg = _d(np.asarray(g).reshape(-1))
    k = S.shape[0] if S.size else 0
    r = np.zeros_like(g)
    lib().oracle_two_loop(g.shape[0], k, ps, py, pg, r.ctypes.data_as(C.POINTER(C.c_double)))
    return r


class _Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("max_iter", C.c_int32), ("max_halvings", C.c_int32),
                ("ftol_window", C.c_int32), ("c1", C.c_double), ("eps_curv", C.c_double),
                ("e_feasible", C.c_double), ("g_tol", C.c_double), ("ftol", C.c_double),
                ("rad", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("evals", C.c_int32),
                ("resets", C.c_int32), ("E", C.c_double), ("gnorm", C.c_double)]


@dataclass
class DescentParams:
    """Descent constants.  Defaults: memory m = 10, the paper's MaxIter = 5000
    and gradient stop 1e-12 (Sec. 6.1, Alg. 1), feasibility E < 1e-20."""
    m: int = 10
    max_iter: int = 5000
    max_halvings: int = 40
    ftol_window: int = 20
    c1: float = 1e-4
    eps_curv: float = 1e-8
    e_feasible: float = 1e-20
    g_tol: float = 1e-12
    ftol: float = 0.0
    rad: float = 1.0


def descend(xy, R: float, params: DescentParams | None = None, trace: bool = False):
    """Whole-instance L-BFGS descent in FP64.  Returns (xy_final, result, trace)."""
    P = params or DescentParams()
    x, px = _d(np.array(np.asarray(xy).reshape(-1, 2), dtype=np.float64, copy=True))
    cp = _Params(**asdict(P))
    cr = _Result()
    tr = np.zeros(P.max_iter + 1, dtype=np.float64) if trace else None
    rc = lib().oracle_descend(x.shape[0], px, float(R), C.byref(cp), C.byref(cr),
                              tr.ctypes.data_as(C.POINTER(C.c_double)) if trace else None)
    if rc != 0:
        raise RuntimeError(f"oracle_descend failed ({rc})")
    res = {"status": STATUS[cr.status], "iters": cr.iters, "evals": cr.evals,
           "resets": cr.resets, "E": cr.E, "gnorm": cr.gnorm}
    if trace:
        tr = tr[:cr.iters + 1]
    return x, res, tr


def verify(xy32, R: float, tol: float = 1e-20):
    """FP64 feasibility of FP32 positions: E, max pair overlap, max container
    overlap, feasible flag."""
    xy, p = _f(np.asarray(xy32, dtype=np.float32).reshape(-1, 2))
    out = np.zeros(3, dtype=np.float64)
    f = lib().oracle_verify(xy.shape[0], p, float(R), float(tol),
                            out.ctypes.data_as(C.POINTER(C.c_double)))
    return {"E": out[0], "max_pair_overlap": out[1], "max_cont_overlap": out[2],
            "feasible": bool(f)}


class _GboParams(C.Structure):
    _fields_ = [("blocks", C.c_int32), ("max_outer", C.c_int32), ("jacobi", C.c_int32),
                ("pad", C.c_int32)]


class _GboResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer", C.c_int32), ("visits", C.c_int32),
                ("evals", C.c_int32), ("stalled_visits", C.c_int32), ("pad", C.c_int32),
                ("E", C.c_double), ("gsum", C.c_double)]


def gbo_batches(xy, R: float, blocks: int):
    """Batch id and colour of every circle for a blocks x blocks grid."""
    xy, px = _d(np.asarray(xy).reshape(-1, 2))
    b = np.zeros(xy.shape[0], dtype=np.int32)
    c = np.zeros(xy.shape[0], dtype=np.int32)
    lib().oracle_gbo_batches(xy.shape[0], px, float(R), int(blocks),
                             b.ctypes.data_as(C.POINTER(C.c_int32)),
                             c.ctypes.data_as(C.POINTER(C.c_int32)))
    return b, c


def gbo_descend(xy, R: float, params: DescentParams | None = None, blocks: int = 4,
                max_outer: int = 5000, jacobi: bool = True, trace: bool = False):
    """Geometric batch descent (Alg. 1 over grid blocks, Eq. 7) in FP64 over
    all pairs; no step is limited but by the line search.  Returns
    (xy_final, result, trace)."""
    P = params or DescentParams()
    x, px = _d(np.array(np.asarray(xy).reshape(-1, 2), dtype=np.float64, copy=True))
    cp = _Params(**asdict(P))
    gp = _GboParams(int(blocks), int(max_outer), 1 if jacobi else 0, 0)
    cr = _GboResult()
    tr = np.zeros(max_outer + 1, dtype=np.float64) if trace else None
    rc = lib().oracle_gbo_descend(x.shape[0], px, float(R), C.byref(cp), C.byref(gp), C.byref(cr),
                                  tr.ctypes.data_as(C.POINTER(C.c_double)) if trace else None)
    if rc != 0:
        raise RuntimeError(f"oracle_gbo_descend failed ({rc})")
    res = {"status": STATUS[cr.status], "outer": cr.outer, "visits": cr.visits,
           "evals": cr.evals, "stalled_visits": cr.stalled_visits, "E": cr.E, "gsum": cr.gsum}
    if trace:
        tr = tr[:cr.outer + 1]
    return x, res, tr


# ---------------------------------------------------------------------------
# Container adjustment (Sec. 4.2, Eq. 12, Alg. 2)
# ---------------------------------------------------------------------------
class _AdjResult(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("iters", C.c_int32), ("evals", C.c_int32),
                ("last_status", C.c_int32), ("R", C.c_double), ("E", C.c_double)]


def container_energy(z, rad: float = 1.0, lam: float = 1e-4):
    """(U, grad (2n+1,)) at z = [x1, y1, ..., xn, yn, R]."""
    z, pz = _d(np.asarray(z).reshape(-1))
    n = (z.size - 1) // 2
    g = np.zeros(z.size, dtype=np.float64)
    U = lib().oracle_container_energy(n, pz, float(rad), float(lam),
                                      g.ctypes.data_as(C.POINTER(C.c_double)))
    return U, g


def adjust_container(xy, R: float, params: DescentParams | None = None, lambda0: float = 1e-4,
                     rounds: int = 35):
    """Alg. 2 in FP64.  Returns (xy_final (n, 2), R_final, result dict)."""
    P = params or DescentParams()
    x, px = _d(np.array(np.asarray(xy).reshape(-1, 2), dtype=np.float64, copy=True))
    Rv = C.c_double(float(R))
    cp = _Params(**asdict(P))
    cr = _AdjResult()
    rc = lib().oracle_adjust_container(x.shape[0], px, C.byref(Rv), C.byref(cp), float(lambda0),
                                       int(rounds), C.byref(cr))
    if rc != 0:
        raise RuntimeError(f"oracle_adjust_container failed ({rc})")
    return x, Rv.value, {"rounds": cr.rounds, "iters": cr.iters, "evals": cr.evals,
                         "last_status": STATUS[cr.last_status], "R": cr.R, "E": cr.E}


# ---------------------------------------------------------------------------
# SED (Sec. 5, Alg. 5) and its random numbers (pecc_oracle_sed.c)
# ---------------------------------------------------------------------------
def philox(counter, key):
    """Philox4x64-10 block at counter (4 words) and key (2 words)."""
    c = (C.c_uint64 * 4)(*[int(v) & (2 ** 64 - 1) for v in counter])
    k = (C.c_uint64 * 2)(*[int(v) & (2 ** 64 - 1) for v in key])
    o = (C.c_uint64 * 4)()
    lib().oracle_philox4x64(c, k, o)
    return [int(v) for v in o]


def sed_shift(n: int, seed: int, chain: int, it: int, cand: int):
    r = np.zeros(2 * n, dtype=np.float32)
    lib().oracle_sed_shift(n, seed, chain, it, cand, r.ctypes.data_as(C.POINTER(C.c_float)))
    return r.reshape(-1, 2)


def sed_perturb(xy32, seed: int, chain: int, it: int, cand: int):
    xy, px = _f(np.asarray(xy32, dtype=np.float32).reshape(-1, 2))
    out = np.zeros_like(xy)
    lib().oracle_sed_perturb(xy.shape[0], px, seed, chain, it, cand,
                             out.ctypes.data_as(C.POINTER(C.c_float)))
    return out


def sed_uniform(seed: int, chain: int, it: int) -> float:
    return lib().oracle_sed_uniform(seed, chain, it)


def sed_J(E: float, jmax: int = 25) -> int:
    return lib().oracle_sed_J(float(E), int(jmax))


def sed_select(E, E_cur: float, u: float, jmax: int = 25) -> int:
    E, pE = _d(np.asarray(E).reshape(-1))
    return lib().oracle_sed_select(E.size, pE, float(E_cur), float(u), int(jmax))


class _SedResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("descents", C.c_int32), ("E_best", C.c_double),
                ("E_start", C.c_double)]


def sed(xy, R: float, params: DescentParams | None = None, s_iter: int = 500, m_max: int = 25,
        e_stop: float = 1e-25, seed: int = 0, chain: int = 0):
    """Alg. 5 in FP64 from the start xy; returns (best layout, result dict)."""
    P = params or DescentParams()
    x, px = _d(np.array(np.asarray(xy).reshape(-1, 2), dtype=np.float64, copy=True))
    cp = _Params(**asdict(P))
    cr = _SedResult()
    rc = lib().oracle_sed(x.shape[0], px, float(R), C.byref(cp), int(s_iter), int(m_max),
                          float(e_stop), int(seed), int(chain), C.byref(cr))
    if rc != 0:
        raise RuntimeError(f"oracle_sed failed ({rc})")
    return x, {"iterations": cr.iterations, "descents": cr.descents, "E_best": cr.E_best,
               "E_start": cr.E_start}


# ---------------------------------------------------------------------------
# Learned proposal (pecc_oracle_lp.c)
# ---------------------------------------------------------------------------
N_FEATURES, N_HIDDEN, N_PARAMS = 8, 64, 4801
# offsets of W1 [64][8], b1, W2 [64][64], b2, W3 [64], b3 in the flat vector
PARAM_SLICES = {"W1": (0, 512), "b1": (512, 576), "W2": (576, 4672), "b2": (4672, 4736),
                "W3": (4736, 4800), "b3": (4800, 4801)}


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def bf16_round(w):
    """FP32 -> BF16 (round to nearest even), returned as float32."""
    w, pw = _f(np.asarray(w, dtype=np.float32).reshape(-1))
    out = np.empty_like(w)
    lib().oracle_bf16_round(w.size, pw, out.ctypes.data_as(C.POINTER(C.c_float)))
    return out


def features(xy32, R: float, cand_circle, cand_dest):
    """(ncand, 8) FP64 features of candidates (circle index, destination)."""
    xy, px = _f(np.asarray(xy32, dtype=np.float32).reshape(-1, 2))
    cc, pc = _i(np.asarray(cand_circle).reshape(-1))
    cd, pd = _f(np.asarray(cand_dest, dtype=np.float32).reshape(-1, 2))
    out = np.zeros((cc.size, 8), dtype=np.float64)
    rc = lib().oracle_features(xy.shape[0], px, float(R), cc.size, pc, pd,
                               out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ValueError("candidate circle index out of range")
    return out


def mlp_forward(params, x, round_bf16: bool = True):
    """Logits (rows,) of the network at parameters ``params`` (4801,)."""
    p, pp = _d(np.asarray(params).reshape(-1))
    assert p.size == N_PARAMS
    x, px = _d(np.asarray(x).reshape(-1, N_FEATURES))
    z = np.zeros(x.shape[0], dtype=np.float64)
    lib().oracle_mlp_forward(pp, 1 if round_bf16 else 0, x.shape[0], px,
                             z.ctypes.data_as(C.POINTER(C.c_double)))
    return z


def mlp_grad(params, x, y, round_bf16: bool = True):
    """(loss, grad (4801,)) of the mean BCE-with-logits loss."""
    p, pp = _d(np.asarray(params).reshape(-1))
    assert p.size == N_PARAMS
    x, px = _d(np.asarray(x).reshape(-1, N_FEATURES))
    y, py = _d(np.asarray(y).reshape(-1))
    g = np.zeros(N_PARAMS, dtype=np.float64)
    loss = lib().oracle_mlp_grad(pp, 1 if round_bf16 else 0, x.shape[0], px, py,
                                 g.ctypes.data_as(C.POINTER(C.c_double)))
    return loss, g


def adam(params, m, v, grad, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step on copies; returns (params, m, v)."""
    p, pp = _d(np.array(params, dtype=np.float64, copy=True).reshape(-1))
    m, pm = _d(np.array(m, dtype=np.float64, copy=True).reshape(-1))
    v, pv = _d(np.array(v, dtype=np.float64, copy=True).reshape(-1))
    g, pg = _d(np.asarray(grad).reshape(-1))
    lib().oracle_adam(p.size, pp, pm, pv, pg, int(t), float(lr), float(b1), float(b2), float(eps))
    return p, m, v


def propose(xy32, cand_circle, cand_dest, scores, k: int):
    """Top-k distinct circles; returns (selected candidate indices, relocated xy)."""
    xy, px = _f(np.asarray(xy32, dtype=np.float32).reshape(-1, 2))
    cc, pc = _i(np.asarray(cand_circle).reshape(-1))
    cd, pd = _f(np.asarray(cand_dest, dtype=np.float32).reshape(-1, 2))
    if scores is not None:
        sc, ps = _f(np.asarray(scores, dtype=np.float32).reshape(-1))
    else:
        ps = None
    sel = np.zeros(max(int(k), 1), dtype=np.int32)
    out = np.zeros_like(xy)
    cnt = lib().oracle_propose(xy.shape[0], px, cc.size, pc, pd, ps, int(k),
                               sel.ctypes.data_as(C.POINTER(C.c_int32)),
                               out.ctypes.data_as(C.POINTER(C.c_float)))
    return sel[:cnt], out


# ---------------------------------------------------------------------------
# Partitions (Sec. 4.1), sequential batch descent (Alg. 1), ANM (Alg. 3)
# ---------------------------------------------------------------------------
PARTITIONS = {"sector": 0, "annulus": 1, "fence": 2, "random": 3}


def partition(xy32, kind: str, k: int, seed: int = 0, instance: int = 0):
    """batch_of (int32 [n]) of the k-batch partition `kind` of FP32 positions."""
    x, px = _f(np.asarray(xy32).reshape(-1, 2))
    out = np.zeros(x.shape[0], dtype=np.int32)
    rc = lib().oracle_partition(x.shape[0], px, PARTITIONS[kind], int(k), int(seed) & (2 ** 64 - 1),
                                int(instance), out.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc != 0:
        raise ValueError(f"oracle_partition failed ({rc})")
    return out


def gamma_energy(ref, xy, R: float, lcut: float = 4.0) -> float:
    """E of xy over the neighbor structure built at ref with l_cut."""
    r, pr = _d(np.asarray(ref).reshape(-1, 2))
    x, px = _d(np.asarray(xy).reshape(-1, 2))
    return lib().oracle_gamma_energy(r.shape[0], pr, px, float(R), float(lcut))


class _SeqParams(C.Structure):
    _fields_ = [("max_outer", C.c_int32), ("anm", C.c_int32), ("lcut", C.c_double),
                ("dense", C.c_int32), ("pad", C.c_int32)]


def bfgs_update(H, u, v):
    """Eq. 11 applied to a symmetric H (returns a new array)."""
    H = np.array(H, dtype=np.float64, copy=True, order="C")
    u, pu = _d(np.asarray(u).reshape(-1))
    v, pv = _d(np.asarray(v).reshape(-1))
    lib().oracle_bfgs_update(u.size, H.ctypes.data_as(C.POINTER(C.c_double)), pu, pv)
    return H


class _SeqResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer", C.c_int32), ("visits", C.c_int32),
                ("evals", C.c_int32), ("stalled_visits", C.c_int32), ("anm_checks", C.c_int32),
                ("anm_changes", C.c_int32), ("pad", C.c_int32), ("E", C.c_double),
                ("gsum", C.c_double)]


def gbo_seq_descend(xy, R: float, batch_of, k: int, params: DescentParams | None = None,
                    max_outer: int = 5000, anm: bool = False, lcut: float = 4.0,
                    trace: bool = False, dense: bool = False, xtrace: bool = False):
    """Alg. 1 with the given partition, batches visited in order, FP64
    (dense: the paper's per-batch inverse-Hessian matrices).  Returns
    (xy_final, result, trace), and the positions at the top of every outer
    iteration as a fourth item when xtrace is set."""
    P = params or DescentParams()
    x, px = _d(np.array(np.asarray(xy).reshape(-1, 2), dtype=np.float64, copy=True))
    bo = np.ascontiguousarray(np.asarray(batch_of), dtype=np.int32)
    if bo.size != x.shape[0]:
        raise ValueError("batch_of needs one entry per circle")
    cp = _Params(**asdict(P))
    sp = _SeqParams(int(max_outer), 1 if anm else 0, float(lcut), 1 if dense else 0, 0)
    cr = _SeqResult()
    tr = np.zeros(max_outer + 1, dtype=np.float64) if trace else None
    xt = np.zeros((max_outer + 1, x.shape[0], 2), dtype=np.float64) if xtrace else None
    rc = lib().oracle_gbo_seq_descend(x.shape[0], px, float(R), C.byref(cp),
                                      bo.ctypes.data_as(C.POINTER(C.c_int32)), int(k),
                                      C.byref(sp), C.byref(cr),
                                      tr.ctypes.data_as(C.POINTER(C.c_double)) if trace else None,
                                      xt.ctypes.data_as(C.POINTER(C.c_double)) if xtrace else None)
    if rc != 0:
        raise RuntimeError(f"oracle_gbo_seq_descend failed ({rc})")
    res = {"status": STATUS[cr.status], "outer": cr.outer, "visits": cr.visits,
           "evals": cr.evals, "stalled_visits": cr.stalled_visits,
           "anm_checks": cr.anm_checks, "anm_changes": cr.anm_changes, "E": cr.E,
           "gsum": cr.gsum}
    if trace:
        tr = tr[:cr.outer + 1]
    if xtrace:
        return x, res, tr, xt[:cr.outer + 1]
    return x, res, tr
