"""Host-side checks of the C ABI: the library loads, exports every entry
point include/pecc.h declares, and rejects bad arguments before any GPU work
(no compute call is made here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pecc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pecc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def P():
    import paper_2303_02650_amd as P
    return P


def test_every_declared_symbol_is_exported(P):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(P._lib, name), name
        assert name in P.EXPORTED, f"binding lacks {name}"


def test_version(P):
    assert "gfx950" in P.version()


def _fake_inst(P, B=2, max_n=10, total_n=20):
    # non-null dummy device pointers: validation must fail before any use
    return P.pecc_instances(B, max_n, total_n, 0x1000, 0x2000, 0)


def _rc(fn, *args):
    return fn(*args)


def test_descend_rejects_bad_params(P):
    inst = _fake_inst(P)
    out = C.c_void_p(0x3000)
    ws = C.c_void_p(0x4000)
    for field, bad in [("m", 0), ("m", 11), ("max_iter", -1), ("ftol_window", 0),
                       ("ftol_window", 64), ("c1", 0.0), ("c1", 1.0), ("contact_margin", -1.0),
                       ("skin_half", 0.0), ("cutoff", 1.9), ("cell_size", 1.0)]:
        p = P.DescentParams()
        setattr(p, field, bad)
        rc = P._lib.pecc_lbfgs_descend(C.byref(inst), C.c_void_p(0x5000), C.byref(p.c()), out, ws,
                                       1 << 20, None)
        assert rc == -1, (field, bad, rc)
        assert len(P._lib.pecc_last_error()) > 0
    # workspace too small
    p = P.DescentParams().c()
    rc = P._lib.pecc_lbfgs_descend(C.byref(inst), C.c_void_p(0x5000), C.byref(p), out, ws, 4, None)
    assert rc == -2
    # margin that eats the whole skin
    p = P.DescentParams(contact_margin=0.2).c()
    rc = P._lib.pecc_lbfgs_descend(C.byref(inst), C.c_void_p(0x5000), C.byref(p), out, ws, 1 << 20,
                                   None)
    assert rc == -1 and b"cutoff" in P._lib.pecc_last_error()


def test_instances_validation(P):
    p = P.DescentParams().c()
    for inst in [P.pecc_instances(0, 10, 20, 0x1000, 0x2000, 0),
                 P.pecc_instances(2, 2000, 20, 0x1000, 0x2000, 0),
                 P.pecc_instances(2, 10, -1, 0x1000, 0x2000, 0),
                 P.pecc_instances(2, 10, 20, 0, 0x2000, 0),
                 P.pecc_instances(2, 10, 20, 0x1000, 0, 0)]:
        rc = P._lib.pecc_lbfgs_descend(C.byref(inst), C.c_void_p(0x5000), C.byref(p),
                                       C.c_void_p(0x3000), C.c_void_p(0x4000), 1 << 20, None)
        assert rc == -1
    assert P._lib.pecc_lbfgs_descend(None, None, None, None, None, 0, None) == -1


def test_build_and_sweep_validation(P):
    inst = _fake_inst(P)
    size = C.c_size_t()
    assert P._lib.pecc_build_neighbors_workspace_size(C.byref(inst), C.byref(size)) == 0
    assert size.value >= 16
    args = dict(xy=C.c_void_p(0x10), cutoff=2.3, cell=0.0, full=1, row=C.c_void_p(0x20),
                col=C.c_void_p(0x30), cap=100, npairs=C.c_void_p(0x40), ws=C.c_void_p(0x50),
                wsb=size.value)

    def call(**kw):
        a = dict(args, **kw)
        return P._lib.pecc_build_neighbors(C.byref(inst), a["xy"], a["cutoff"], a["cell"],
                                           a["full"], a["row"], a["col"], a["cap"], a["npairs"],
                                           a["ws"], a["wsb"], None)
    assert call(cutoff=0.0) == -1
    assert call(cell=1.0) == -1
    assert call(row=None) == -1
    assert call(cap=-1) == -1
    assert call(col=None) == -1
    assert call(wsb=1) == -2
    assert call(ws=None) == -2
    # energy/grad
    E = C.c_void_p(0x60)
    f = P._lib.pecc_energy_grad
    assert f(C.byref(inst), C.c_void_p(0x10), C.c_void_p(0x20), C.c_void_p(0x30), 10, 0, 0.0, E, None, None) == -1
    assert f(C.byref(inst), C.c_void_p(0x10), None, C.c_void_p(0x30), 10, 0, 1.0, E, None, None) == -1
    assert f(C.byref(inst), C.c_void_p(0x10), C.c_void_p(0x20), None, 10, 0, 1.0, E, None, None) == -1
    assert f(C.byref(inst), C.c_void_p(0x10), C.c_void_p(0x20), C.c_void_p(0x30), -1, 0, 1.0, E, None, None) == -1
    assert f(C.byref(inst), C.c_void_p(0x10), C.c_void_p(0x20), C.c_void_p(0x30), 10, 0, 1.0, None, None, None) == -1
    # unknown list form; a 16-bit list at an odd address
    assert f(C.byref(inst), C.c_void_p(0x10), C.c_void_p(0x20), C.c_void_p(0x30), 10, 3, 1.0, E, None, None) == -1
    assert f(C.byref(inst), C.c_void_p(0x10), C.c_void_p(0x20), C.c_void_p(0x31), 10, 2, 1.0, E, None, None) == -1
    assert call(full=3) == -1
    assert call(full=2, col=C.c_void_p(0x31)) == -1
    # verify
    assert P._lib.pecc_verify(C.byref(inst), C.c_void_p(0x10), 1e-20, None, None, None, None, None) == -1
    vt = P._lib.pecc_verify_tighten
    assert vt(C.byref(inst), C.c_void_p(0x10), 1e-20, None, C.c_void_p(0x70), None) == -1
    assert vt(C.byref(inst), C.c_void_p(0x10), 1e-20, C.c_void_p(0x70), None, None) == -1
    assert vt(C.byref(inst), None, 1e-20, C.c_void_p(0x70), C.c_void_p(0x80), None) == -1


def test_default_params_match_header(P):
    d = P.default_params()
    assert d.m == 10 and d.max_iter == 5000 and d.max_halvings == 40
    assert abs(d.cutoff - 2.3) < 1e-6 and abs(d.skin_half - 0.15) < 1e-7
    assert d.e_feasible == 1e-20 and d.tau64 == 3e-6


def test_learned_proposal_entry_points_reject_bad_arguments(P):
    inst = _fake_inst(P)
    ptr = C.c_void_p(0x5000)
    L = P._lib
    assert L.pecc_features(C.byref(inst), ptr, -1, ptr, ptr, ptr, None) == -1
    assert L.pecc_features(C.byref(inst), None, 4, ptr, ptr, ptr, None) == -1
    assert L.pecc_mlp_forward(ptr, ptr, -1, ptr, None) == -1
    assert L.pecc_mlp_forward(None, ptr, 10, ptr, None) == -1
    b = C.c_size_t()
    assert L.pecc_mlp_grad_workspace_size(-1, C.byref(b)) == -1
    assert L.pecc_mlp_grad_workspace_size(8192, C.byref(b)) == 0 and b.value > 0
    assert L.pecc_mlp_grad(ptr, ptr, ptr, 8192, ptr, ptr, ptr, b.value - 1, None) == -2
    assert L.pecc_mlp_grad(ptr, ptr, None, 8192, ptr, ptr, ptr, b.value, None) == -1
    bad = [P.pecc_adam_params(-1.0, 0.9, 0.999, 1e-8), P.pecc_adam_params(1e-3, 1.0, 0.999, 1e-8),
           P.pecc_adam_params(1e-3, 0.9, 0.999, 0.0)]
    for hp in bad:
        assert L.pecc_mlp_adam(ptr, ptr, ptr, ptr, ptr, C.byref(hp), None) == -1
    good = P.pecc_adam_params(1e-3, 0.9, 0.999, 1e-8)
    assert L.pecc_mlp_adam(ptr, ptr, ptr, ptr, None, C.byref(good), None) == -1
    assert L.pecc_mlp_train_step(ptr, ptr, ptr, ptr, C.byref(bad[0]), ptr, ptr, 10, ptr, ptr, ptr,
                                 b.value, None) == -1
    assert L.pecc_propose(C.byref(inst), ptr, 4, ptr, ptr, None, -1, ptr, ptr, None) == -1
    assert L.pecc_propose(C.byref(inst), ptr, 4, ptr, ptr, None, 3, ptr, None, None) == -1
    assert L.pecc_accept(C.byref(inst), ptr, None, ptr, ptr, None, None) == -1
    assert b"pecc_accept" in L.pecc_last_error()


def test_adjust_container_rejects_bad_arguments(P):
    inst = _fake_inst(P)
    ptr = C.c_void_p(0x5000)
    prm = P.default_params().c()
    L = P._lib
    b = C.c_size_t()
    assert L.pecc_adjust_container_workspace_size(C.byref(inst), C.byref(b)) == 0
    args = lambda lam, rounds, rout: (C.byref(inst), ptr, C.byref(prm), lam, rounds, rout, ptr, ptr,
                                      b.value, None)
    assert L.pecc_adjust_container(*args(-1.0, 35, ptr)) == -1
    assert L.pecc_adjust_container(*args(float("nan"), 35, ptr)) == -1
    assert L.pecc_adjust_container(*args(1e-4, 65, ptr)) == -1
    assert L.pecc_adjust_container(*args(1e-4, -1, ptr)) == -1
    assert L.pecc_adjust_container(*args(1e-4, 35, None)) == -1
    assert L.pecc_adjust_container(C.byref(inst), ptr, C.byref(prm), 1e-4, 35, ptr, ptr, ptr,
                                   b.value - 1, None) == -2
