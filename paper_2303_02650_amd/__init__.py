"""Python binding of libpecc (MI355X penalty-energy descent for PECC).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libpecc.so``.  Tensors are torch tensors on the GPU; the binding
passes their device pointers and the current torch stream to the C ABI
declared in ``include/pecc.h`` and raises ``PeccError`` on a non-zero return.
The library must have been built (``python paper_2303_02650_amd/build.py``);
importing this package without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, asdict, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpecc.so")

PECC_MAX_N = 1024
PECC_MAX_M = 10
PECC_NOALLOC_MAX_INSTANCES = 65536
# neighbor-list forms (PECC_LIST_*)
LIST_HALF, LIST_FULL, LIST_LOCAL16 = 0, 1, 2
STATUS = {0: "RUNNING", 1: "FEASIBLE", 2: "STATIONARY", 3: "CONVERGED", 4: "STALLED",
          5: "MAX_ITER", 6: "NONFINITE", 7: "BAD_INSTANCE"}


class PeccError(RuntimeError):
    pass


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with python paper_2303_02650_amd/build.py")
_lib = C.CDLL(LIB_PATH)


class pecc_instances(C.Structure):
    _fields_ = [("num_instances", C.c_int32), ("max_n", C.c_int32), ("total_n", C.c_int64),
                ("offset", C.c_void_p), ("R", C.c_void_p), ("R64", C.c_void_p)]


class pecc_descent_params(C.Structure):
    _fields_ = [("m", C.c_int32), ("max_iter", C.c_int32), ("max_halvings", C.c_int32),
                ("ftol_window", C.c_int32), ("c1", C.c_float), ("eps_curv", C.c_float),
                ("cutoff", C.c_float), ("skin_half", C.c_float), ("cell_size", C.c_float),
                ("g_tol", C.c_float), ("ftol", C.c_float), ("contact_margin", C.c_float),
                ("e_feasible", C.c_double), ("tau64", C.c_double)]


RESULT_DTYPE = np.dtype([("status", np.int32), ("iters", np.int32), ("evals", np.int32),
                         ("rebuilds", np.int32), ("pair_evals", np.int64), ("E32", np.float32),
                         ("gnorm", np.float32), ("E64", np.float64), ("cell_evals", np.int32),
                         ("reserved", np.int32)])
assert RESULT_DTYPE.itemsize == 48

class pecc_adam_params(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


PECC_FEATURES = 8
PECC_MLP_PARAMS = 4801

_P = C.POINTER
_V = C.c_void_p
_sig = {
    "pecc_last_error": (C.c_char_p, []),
    "pecc_version": (C.c_char_p, []),
    "pecc_build_neighbors_workspace_size": (C.c_int, [_P(pecc_instances), _P(C.c_size_t)]),
    "pecc_build_neighbors": (C.c_int, [_P(pecc_instances), C.c_void_p, C.c_double, C.c_float,
                                       C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_void_p, C.c_size_t, C.c_void_p]),
    "pecc_energy_grad": (C.c_int, [_P(pecc_instances), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_int64, C.c_int32, C.c_float, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "pecc_descent_params_default": (None, [_P(pecc_descent_params)]),
    "pecc_lbfgs_descend_workspace_size": (C.c_int, [_P(pecc_instances), _P(C.c_size_t)]),
    "pecc_lbfgs_descend": (C.c_int, [_P(pecc_instances), C.c_void_p, _P(pecc_descent_params),
                                     C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "pecc_lbfgs_descend_noalloc": (C.c_int, [_P(pecc_instances), C.c_void_p,
                                             _P(pecc_descent_params), C.c_void_p, C.c_void_p]),
    "pecc_verify": (C.c_int, [_P(pecc_instances), C.c_void_p, C.c_double, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pecc_verify_tighten": (C.c_int, [_P(pecc_instances), C.c_void_p, C.c_double, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "pecc_gbo_descend_workspace_size": (C.c_int, [_P(pecc_instances), C.c_int32, _P(C.c_size_t)]),
    "pecc_gbo_descend": (C.c_int, [_P(pecc_instances), C.c_void_p, _P(pecc_descent_params),
                                   C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.c_void_p]),
    "pecc_partition": (C.c_int, [_P(pecc_instances), _V, C.c_int32, C.c_int32, C.c_uint64, _V, _V]),
    "pecc_gbo_kbatch_descend_workspace_size": (C.c_int, [_P(pecc_instances), _P(C.c_size_t)]),
    "pecc_gbo_kbatch_descend": (C.c_int, [_P(pecc_instances), _V, _V, C.c_int32, C.c_int32,
                                          _P(pecc_descent_params), _V, _V, C.c_size_t, _V]),
    "pecc_gbo_kbatch_bfgs_workspace_size": (C.c_int, [_P(pecc_instances), C.c_int32,
                                                      _P(C.c_size_t)]),
    "pecc_gbo_kbatch_bfgs_descend": (C.c_int, [_P(pecc_instances), _V, _V, C.c_int32, C.c_int32,
                                               C.c_int32, _P(pecc_descent_params), _V, _V,
                                               C.c_size_t, _V]),
    "pecc_adjust_container_workspace_size": (C.c_int, [_P(pecc_instances), _P(C.c_size_t)]),
    "pecc_adjust_container": (C.c_int, [_P(pecc_instances), _V, _P(pecc_descent_params), C.c_float,
                                        C.c_int32, _V, _V, _V, C.c_size_t, _V]),
    "pecc_sed_plan": (C.c_int, [_P(pecc_instances), _V, _V, C.c_int32, C.c_double, _V, _V, _V, _V,
                                _V]),
    "pecc_sed_perturb": (C.c_int, [_P(pecc_instances), _V, C.c_int32, _V, _V, C.c_uint64, C.c_int32,
                                   _V, _V]),
    "pecc_sed_select": (C.c_int, [_P(pecc_instances), C.c_int32, _V, _V, _V, _V, C.c_uint64,
                                  C.c_int32, _V, _V, _V, _V, _V, _V]),
    "pecc_features": (C.c_int, [_P(pecc_instances), _V, C.c_int32, _V, _V, _V, _V]),
    "pecc_mlp_forward": (C.c_int, [_V, _V, C.c_int64, _V, _V]),
    "pecc_mlp_grad_workspace_size": (C.c_int, [C.c_int64, _P(C.c_size_t)]),
    "pecc_mlp_grad": (C.c_int, [_V, _V, _V, C.c_int64, _V, _V, _V, C.c_size_t, _V]),
    "pecc_mlp_adam": (C.c_int, [_V, _V, _V, _V, _V, _P(pecc_adam_params), _V]),
    "pecc_mlp_train_step": (C.c_int, [_V, _V, _V, _V, _P(pecc_adam_params), _V, _V, C.c_int64,
                                      _V, _V, _V, C.c_size_t, _V]),
    "pecc_propose": (C.c_int, [_P(pecc_instances), _V, C.c_int32, _V, _V, _V, C.c_int32, _V, _V,
                               _V]),
    "pecc_accept": (C.c_int, [_P(pecc_instances), _V, _V, _V, _V, _V, _V]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(rc: int):
    if rc != 0:
        raise PeccError(f"libpecc error {rc}: {_lib.pecc_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def version() -> str:
    return _lib.pecc_version().decode()


# ---------------------------------------------------------------------------
# Instances on the device
# ---------------------------------------------------------------------------
@dataclass
class DeviceInstances:
    """Device copy of a packed batch (offsets, radii) plus host sizes."""
    offset: torch.Tensor      # int32 [B+1]
    R: torch.Tensor           # float32 [B]
    R64: torch.Tensor         # float64 [B]
    max_n: int
    total_n: int
    _c: pecc_instances = field(default=None, repr=False)

    @property
    def B(self) -> int:
        return int(self.R.shape[0])

    def c(self) -> pecc_instances:
        if self._c is None:
            self._c = pecc_instances(self.B, self.max_n, self.total_n, self.offset.data_ptr(),
                                     self.R.data_ptr(), self.R64.data_ptr())
        return self._c

    @staticmethod
    def from_host(offset, R, device="cuda") -> "DeviceInstances":
        off = np.asarray(offset, dtype=np.int32)
        R = np.asarray(R, dtype=np.float64)
        n = np.diff(off)
        return DeviceInstances(offset=torch.from_numpy(off).to(device),
                               R=torch.from_numpy(R.astype(np.float32)).to(device),
                               R64=torch.from_numpy(R).to(device),
                               max_n=int(n.max()) if len(n) else 0, total_n=int(off[-1]))


# ---------------------------------------------------------------------------
# C ABI, same names
# ---------------------------------------------------------------------------
def pecc_build_neighbors_workspace_size(inst: DeviceInstances) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_build_neighbors_workspace_size(C.byref(inst.c()), C.byref(b)))
    return b.value


def pecc_build_neighbors(inst, xy, cutoff, cell_size, form, row, col, capacity, num_pairs,
                         workspace, stream=None):
    _check(_lib.pecc_build_neighbors(C.byref(inst.c()), _ptr(xy), float(cutoff), float(cell_size),
                                     int(form), _ptr(row), _ptr(col), int(capacity),
                                     _ptr(num_pairs), _ptr(workspace),
                                     workspace.numel() * workspace.element_size(),
                                     _stream(stream)))


def pecc_energy_grad(inst, xy, row, col, col_len, form, rad, energy, grad, stream=None):
    _check(_lib.pecc_energy_grad(C.byref(inst.c()), _ptr(xy), _ptr(row), _ptr(col),
                                 int(col_len), int(form), float(rad), _ptr(energy), _ptr(grad),
                                 _stream(stream)))


def pecc_lbfgs_descend_workspace_size(inst: DeviceInstances) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_lbfgs_descend_workspace_size(C.byref(inst.c()), C.byref(b)))
    return b.value


def pecc_lbfgs_descend(inst, xy, params: pecc_descent_params, out, workspace, stream=None):
    _check(_lib.pecc_lbfgs_descend(C.byref(inst.c()), _ptr(xy), C.byref(params), _ptr(out),
                                   _ptr(workspace), workspace.numel() * workspace.element_size(),
                                   _stream(stream)))


def pecc_lbfgs_descend_noalloc(inst, xy, params: pecc_descent_params, out, stream=None):
    _check(_lib.pecc_lbfgs_descend_noalloc(C.byref(inst.c()), _ptr(xy), C.byref(params), _ptr(out),
                                           _stream(stream)))


def pecc_gbo_descend_workspace_size(inst: DeviceInstances, blocks: int) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_gbo_descend_workspace_size(C.byref(inst.c()), int(blocks), C.byref(b)))
    return b.value


def pecc_gbo_descend(inst, xy, params: pecc_descent_params, blocks, sweep_fp64, out, workspace,
                     stream=None):
    _check(_lib.pecc_gbo_descend(C.byref(inst.c()), _ptr(xy), C.byref(params), int(blocks),
                                 int(sweep_fp64), _ptr(out), _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), _stream(stream)))


def pecc_verify(inst, xy, tol, energy64, max_pair, max_cont, feasible, stream=None):
    _check(_lib.pecc_verify(C.byref(inst.c()), _ptr(xy), float(tol), _ptr(energy64),
                            _ptr(max_pair), _ptr(max_cont), _ptr(feasible), _stream(stream)))


def pecc_verify_tighten(inst, xy, tol, R_out, feasible, stream=None):
    _check(_lib.pecc_verify_tighten(C.byref(inst.c()), _ptr(xy), float(tol), _ptr(R_out),
                                    _ptr(feasible), _stream(stream)))


# ---------------------------------------------------------------------------
# Conveniences (allocation + the calls above)
# ---------------------------------------------------------------------------
@dataclass
class DescentParams:
    m: int = 10
    max_iter: int = 5000
    max_halvings: int = 40
    ftol_window: int = 20
    c1: float = 1e-4
    eps_curv: float = 1e-8
    cutoff: float = 2.3
    skin_half: float = 0.15
    cell_size: float = 0.0
    g_tol: float = 1e-6
    ftol: float = 1e-7
    contact_margin: float = 0.0
    e_feasible: float = 1e-20
    tau64: float = 3e-6

    def c(self) -> pecc_descent_params:
        return pecc_descent_params(**asdict(self))


def default_params() -> DescentParams:
    p = pecc_descent_params()
    _lib.pecc_descent_params_default(C.byref(p))
    return DescentParams(**{k: getattr(p, k) for k, _ in pecc_descent_params._fields_})


def build_neighbors(inst: DeviceInstances, xy: torch.Tensor, cutoff: float = 2.3,
                    cell_size: float = 0.0, form: int = LIST_HALF, capacity: int | None = None):
    """Returns (row int32 [total_n+1], col [num_pairs]) in the list form
    ``form`` (LIST_HALF / LIST_FULL: int32 global indices; LIST_LOCAL16:
    instance-local indices held in an int16 tensor, values below 1024;
    False / True stand for LIST_HALF / LIST_FULL)."""
    form = int(form)
    dev = xy.device
    dt = torch.int16 if form == LIST_LOCAL16 else torch.int32
    row = torch.empty(inst.total_n + 1, dtype=torch.int32, device=dev)
    npairs = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(pecc_build_neighbors_workspace_size(inst), dtype=torch.uint8, device=dev)
    cap = capacity if capacity is not None else max(16, 8 * inst.total_n)
    col = torch.empty(max(cap, 1), dtype=dt, device=dev)
    pecc_build_neighbors(inst, xy, cutoff, cell_size, form, row, col, cap, npairs, ws)
    need = int(npairs.item())
    if need > cap:
        col = torch.empty(need, dtype=dt, device=dev)
        pecc_build_neighbors(inst, xy, cutoff, cell_size, form, row, col, need, npairs, ws)
    return row, col[:need]


def energy_grad(inst: DeviceInstances, xy: torch.Tensor, row: torch.Tensor, col: torch.Tensor,
                rad: float = 1.0, want_grad: bool = True, form: int | None = None):
    """E [B] and grad [2 total_n]; the list form defaults to LIST_LOCAL16
    for an int16 col and LIST_HALF for an int32 one (a list with both
    orientations read as LIST_HALF gives the same pairs)."""
    if form is None:
        form = LIST_LOCAL16 if col.dtype == torch.int16 else LIST_HALF
    E = torch.empty(inst.B, dtype=torch.float32, device=xy.device)
    g = torch.empty_like(xy) if want_grad else None
    pecc_energy_grad(inst, xy, row, col, col.numel(), form, rad, E, g)
    return E, g


def lbfgs_descend(inst: DeviceInstances, xy: torch.Tensor, params: DescentParams | None = None,
                  workspace: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """Descends every instance in place; returns the device result buffer
    (uint8 [B*40]); ``results()`` turns it into a numpy record array."""
    P = (params or DescentParams()).c()
    if out is None:
        out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=xy.device)
    if workspace is None:
        workspace = torch.empty(pecc_lbfgs_descend_workspace_size(inst), dtype=torch.uint8,
                                device=xy.device)
    pecc_lbfgs_descend(inst, xy, P, out, workspace)
    return out


def gbo_descend(inst: DeviceInstances, xy: torch.Tensor, params: DescentParams | None = None,
                blocks: int = 4, sweep_fp64: bool = False, workspace: torch.Tensor | None = None,
                out: torch.Tensor | None = None):
    """Geometric batch descent of every instance in place; returns the
    device result buffer (see ``results``)."""
    P = (params or DescentParams()).c()
    if out is None:
        out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=xy.device)
    if workspace is None:
        workspace = torch.empty(pecc_gbo_descend_workspace_size(inst, blocks), dtype=torch.uint8,
                                device=xy.device)
    pecc_gbo_descend(inst, xy, P, blocks, sweep_fp64, out, workspace)
    return out


PARTITIONS = {"sector": 0, "annulus": 1, "fence": 2, "random": 3}
PECC_MAX_BATCHES = 16


def pecc_partition(inst, xy, kind: int, k: int, seed: int, batch_of, stream=None):
    _check(_lib.pecc_partition(C.byref(inst.c()), _ptr(xy), int(kind), int(k),
                               int(seed) & (2 ** 64 - 1), _ptr(batch_of), _stream(stream)))


def partition(inst: DeviceInstances, xy: torch.Tensor, kind: str = "sector", k: int = 5,
              seed: int = 0) -> torch.Tensor:
    """k-batch partition of every instance (Sec. 4.1): int32 batch ids."""
    out = torch.empty(inst.total_n, dtype=torch.int32, device=xy.device)
    pecc_partition(inst, xy, PARTITIONS[kind], k, seed, out)
    return out


def pecc_gbo_kbatch_descend_workspace_size(inst: DeviceInstances) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_gbo_kbatch_descend_workspace_size(C.byref(inst.c()), C.byref(b)))
    return b.value


def pecc_gbo_kbatch_descend(inst, xy, batch_of, k: int, anm: int, params: pecc_descent_params,
                            out, workspace, stream=None):
    _check(_lib.pecc_gbo_kbatch_descend(C.byref(inst.c()), _ptr(xy), _ptr(batch_of), int(k),
                                        int(anm), C.byref(params), _ptr(out), _ptr(workspace),
                                        workspace.numel() * workspace.element_size(),
                                        _stream(stream)))


def gbo_kbatch_descend(inst: DeviceInstances, xy: torch.Tensor, batch_of: torch.Tensor, k: int,
                       params: DescentParams | None = None, anm: bool = False,
                       workspace: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """Alg. 1 over the partition batch_of (k batches, visited in order) of
    every instance, in place; anm selects the neighbor maintenance of Alg. 3
    (l_cut = params.cutoff).  Returns the device result buffer."""
    P = (params or DescentParams()).c()
    if out is None:
        out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=xy.device)
    if workspace is None:
        workspace = torch.empty(pecc_gbo_kbatch_descend_workspace_size(inst), dtype=torch.uint8,
                                device=xy.device)
    pecc_gbo_kbatch_descend(inst, xy, batch_of, k, 1 if anm else 0, P, out, workspace)
    return out


def pecc_gbo_kbatch_bfgs_workspace_size(inst: DeviceInstances, max_batch: int) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_gbo_kbatch_bfgs_workspace_size(C.byref(inst.c()), int(max_batch), C.byref(b)))
    return b.value


def pecc_gbo_kbatch_bfgs_descend(inst, xy, batch_of, k: int, anm: int, max_batch: int,
                                 params: pecc_descent_params, out, workspace, stream=None):
    _check(_lib.pecc_gbo_kbatch_bfgs_descend(C.byref(inst.c()), _ptr(xy), _ptr(batch_of), int(k),
                                             int(anm), int(max_batch), C.byref(params), _ptr(out),
                                             _ptr(workspace),
                                             workspace.numel() * workspace.element_size(),
                                             _stream(stream)))


def gbo_kbatch_bfgs_descend(inst: DeviceInstances, xy: torch.Tensor, batch_of: torch.Tensor,
                            k: int, max_batch: int, params: DescentParams | None = None,
                            anm: bool = False, workspace: torch.Tensor | None = None,
                            out: torch.Tensor | None = None):
    """The k-batch descent with dense per-batch BFGS matrices (Eq. 8-11), in
    place; max_batch bounds every batch's size.  Returns the result buffer."""
    P = (params or DescentParams()).c()
    if out is None:
        out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=xy.device)
    if workspace is None:
        workspace = torch.empty(pecc_gbo_kbatch_bfgs_workspace_size(inst, max_batch),
                                dtype=torch.uint8, device=xy.device)
    pecc_gbo_kbatch_bfgs_descend(inst, xy, batch_of, k, 1 if anm else 0, max_batch, P, out,
                                 workspace)
    return out


def pecc_adjust_container_workspace_size(inst: DeviceInstances) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_adjust_container_workspace_size(C.byref(inst.c()), C.byref(b)))
    return b.value


def pecc_adjust_container(inst, xy, params: pecc_descent_params, lambda0, rounds, R_out, out,
                          workspace, stream=None):
    _check(_lib.pecc_adjust_container(C.byref(inst.c()), _ptr(xy), C.byref(params), float(lambda0),
                                      int(rounds), _ptr(R_out), _ptr(out), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(),
                                      _stream(stream)))


def adjust_container(inst: DeviceInstances, xy: torch.Tensor, params: DescentParams | None = None,
                     lambda0: float = 1e-4, rounds: int = 35):
    """Container adjustment (Alg. 2) in place on xy; returns (R_out float32
    [B], device result buffer)."""
    P = (params or DescentParams()).c()
    out = torch.empty(inst.B * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=xy.device)
    ws = torch.empty(pecc_adjust_container_workspace_size(inst), dtype=torch.uint8, device=xy.device)
    R_out = torch.empty(inst.B, dtype=torch.float32, device=xy.device)
    pecc_adjust_container(inst, xy, P, lambda0, rounds, R_out, out, ws)
    return R_out, out


PECC_SED_MAX_CAND = 64


def pecc_sed_plan(chains, E_cur, E_best, M, e_stop, m, cand_offset, cand_R, cand_R64, stream=None):
    _check(_lib.pecc_sed_plan(C.byref(chains.c()), _ptr(E_cur), _ptr(E_best), int(M), float(e_stop),
                              _ptr(m), _ptr(cand_offset), _ptr(cand_R), _ptr(cand_R64),
                              _stream(stream)))


def pecc_sed_perturb(chains, xy, M, m, cand_offset, seed, it, cand_xy, stream=None):
    _check(_lib.pecc_sed_perturb(C.byref(chains.c()), _ptr(xy), int(M), _ptr(m), _ptr(cand_offset),
                                 int(seed) & (2 ** 64 - 1), int(it), _ptr(cand_xy), _stream(stream)))


def pecc_sed_select(chains, M, m, cand_offset, cand_xy, cand_E, seed, it, xy_cur, E_cur, xy_best,
                    E_best, chosen, stream=None):
    _check(_lib.pecc_sed_select(C.byref(chains.c()), int(M), _ptr(m), _ptr(cand_offset),
                                _ptr(cand_xy), _ptr(cand_E), int(seed) & (2 ** 64 - 1), int(it),
                                _ptr(xy_cur), _ptr(E_cur), _ptr(xy_best), _ptr(E_best),
                                _ptr(chosen), _stream(stream)))


def results(out: torch.Tensor) -> np.ndarray:
    return out.cpu().numpy().view(RESULT_DTYPE)


def verify(inst: DeviceInstances, xy: torch.Tensor, tol: float = 1e-20):
    dev = xy.device
    e = torch.empty(inst.B, dtype=torch.float64, device=dev)
    mp = torch.empty_like(e)
    mc = torch.empty_like(e)
    f = torch.empty(inst.B, dtype=torch.int32, device=dev)
    pecc_verify(inst, xy, tol, e, mp, mc, f)
    return e, mp, mc, f


# ---------------------------------------------------------------------------
# Learned proposal (same names as the C ABI, then conveniences)
# ---------------------------------------------------------------------------
def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def pecc_features(inst, xy, cands_per_inst, cand_circle, cand_dest, features, stream=None):
    _check(_lib.pecc_features(C.byref(inst.c()), _ptr(xy), int(cands_per_inst), _ptr(cand_circle),
                              _ptr(cand_dest), _ptr(features), _stream(stream)))


def pecc_mlp_forward(params, features, rows, logits, stream=None):
    _check(_lib.pecc_mlp_forward(_ptr(params), _ptr(features), int(rows), _ptr(logits),
                                 _stream(stream)))


def pecc_mlp_grad_workspace_size(rows: int) -> int:
    b = C.c_size_t()
    _check(_lib.pecc_mlp_grad_workspace_size(int(rows), C.byref(b)))
    return b.value


def pecc_mlp_grad(params, features, labels, rows, loss, grad, workspace, stream=None):
    _check(_lib.pecc_mlp_grad(_ptr(params), _ptr(features), _ptr(labels), int(rows), _ptr(loss),
                              _ptr(grad), _ptr(workspace), _nbytes(workspace), _stream(stream)))


def pecc_mlp_adam(params, m, v, grad, step, hp: pecc_adam_params, stream=None):
    _check(_lib.pecc_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), _ptr(step), C.byref(hp),
                              _stream(stream)))


def pecc_mlp_train_step(params, m, v, step, hp: pecc_adam_params, features, labels, rows, loss,
                        grad, workspace, stream=None):
    _check(_lib.pecc_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), _ptr(step), C.byref(hp),
                                    _ptr(features), _ptr(labels), int(rows), _ptr(loss), _ptr(grad),
                                    _ptr(workspace), _nbytes(workspace), _stream(stream)))


def pecc_propose(inst, xy, cands_per_inst, cand_circle, cand_dest, scores, k, selected, xy_out,
                 stream=None):
    _check(_lib.pecc_propose(C.byref(inst.c()), _ptr(xy), int(cands_per_inst), _ptr(cand_circle),
                             _ptr(cand_dest), _ptr(scores), int(k), _ptr(selected), _ptr(xy_out),
                             _stream(stream)))


def pecc_accept(inst, xy_cur, e_cur, xy_new, e_new, accepted, stream=None):
    _check(_lib.pecc_accept(C.byref(inst.c()), _ptr(xy_cur), _ptr(e_cur), _ptr(xy_new),
                            _ptr(e_new), _ptr(accepted), _stream(stream)))


def features(inst: DeviceInstances, xy: torch.Tensor, cand_circle: torch.Tensor,
             cand_dest: torch.Tensor) -> torch.Tensor:
    """FP32 features [B*C, 8] of C candidates per instance."""
    C_ = cand_circle.numel() // inst.B
    out = torch.empty(inst.B * C_, PECC_FEATURES, dtype=torch.float32, device=xy.device)
    pecc_features(inst, xy, C_, cand_circle, cand_dest, out)
    return out


def mlp_forward(params: torch.Tensor, feats: torch.Tensor) -> torch.Tensor:
    rows = feats.shape[0]
    z = torch.empty(rows, dtype=torch.float32, device=feats.device)
    pecc_mlp_forward(params, feats, rows, z)
    return z


def mlp_grad(params: torch.Tensor, feats: torch.Tensor, labels: torch.Tensor,
             workspace: torch.Tensor | None = None):
    """(loss [1], grad [4801]) of the mean BCE-with-logits loss."""
    rows = feats.shape[0]
    dev = params.device
    if workspace is None:
        workspace = torch.empty(pecc_mlp_grad_workspace_size(rows), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    grad = torch.empty(PECC_MLP_PARAMS, dtype=torch.float32, device=dev)
    pecc_mlp_grad(params, feats, labels, rows, loss, grad, workspace)
    return loss, grad


class MlpTrainer:
    """FP32 master parameters, Adam moments and the device step counter."""

    def __init__(self, params: torch.Tensor, lr: float = 1e-3, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, max_rows: int = 8192):
        dev = params.device
        self.params = params.detach().to(torch.float32).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.hp = pecc_adam_params(lr, beta1, beta2, eps)
        self.ws = torch.empty(pecc_mlp_grad_workspace_size(max_rows), dtype=torch.uint8,
                              device=dev)
        self.max_rows = max_rows

    def train_step(self, feats: torch.Tensor, labels: torch.Tensor):
        rows = feats.shape[0]
        assert rows <= self.max_rows
        pecc_mlp_train_step(self.params, self.m, self.v, self.step, self.hp, feats, labels, rows,
                            self.loss, self.grad, self.ws)
        return self.loss


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-style random initial parameters (zero biases)."""
    g = np.random.default_rng(seed)
    p = np.zeros(PECC_MLP_PARAMS, dtype=np.float32)
    p[0:512] = g.normal(0, np.sqrt(2 / 8), 512)
    p[576:4672] = g.normal(0, np.sqrt(2 / 64), 4096)
    p[4736:4800] = g.normal(0, np.sqrt(1 / 64), 64)
    return torch.from_numpy(p).to(device)


def propose(inst: DeviceInstances, xy: torch.Tensor, cand_circle: torch.Tensor,
            cand_dest: torch.Tensor, scores: torch.Tensor | None, k: int,
            xy_out: torch.Tensor | None = None):
    """(relocated layout, selected candidate indices [B, k])."""
    C_ = cand_circle.numel() // inst.B
    if xy_out is None:
        xy_out = torch.empty_like(xy)
    sel = torch.empty(inst.B, max(k, 1), dtype=torch.int32, device=xy.device)
    pecc_propose(inst, xy, C_, cand_circle, cand_dest, scores, k, sel, xy_out)
    return xy_out, sel[:, :k]


def accept(inst: DeviceInstances, xy_cur: torch.Tensor, e_cur: torch.Tensor,
           xy_new: torch.Tensor, e_new: torch.Tensor) -> torch.Tensor:
    acc = torch.empty(inst.B, dtype=torch.int32, device=xy_cur.device)
    pecc_accept(inst, xy_cur, e_cur, xy_new, e_new, acc)
    return acc
