"""The descent entry point that allocates nothing (its work queue in a
library-held array) against pecc_lbfgs_descend, through the C ABI: two
calls in a row, the second with fewer and smaller instances, each equal to
the workspace entry point's result bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2303_02650_amd as P
    assert torch.cuda.is_available()
    return P


def descend_both(P, inst, params):
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    x0 = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    xa, xb = x0.clone(), x0.clone()
    oa = torch.zeros(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    ob = torch.full_like(oa, 0xAB)
    ws = torch.empty(P.pecc_lbfgs_descend_workspace_size(d), dtype=torch.uint8, device="cuda")
    P.pecc_lbfgs_descend(d, xa, params, oa, ws)
    P.pecc_lbfgs_descend_noalloc(d, xb, params, ob)
    torch.cuda.synchronize()
    return xa, xb, oa, ob


def test_noalloc_descent_equals_workspace_descent_twice(P):
    params = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4, max_iter=3000).c()
    first = synth.C3(40)                            # n in [300, 1000]
    xa, xb, oa, ob = descend_both(P, first, params)
    assert torch.equal(xa, xb) and torch.equal(oa, ob)
    # a second call, smaller in both instance count and sizes: the queue left
    # by the first call must not leak into it
    rng = synth.rng_for(3)
    small = synth.pack([synth.disk_uniform(n, np.sqrt(n / 0.84), rng) for n in (20, 64, 7, 150)],
                       [np.sqrt(n / 0.84) for n in (20, 64, 7, 150)])
    xa, xb, oa, ob = descend_both(P, small, params)
    assert torch.equal(xa, xb) and torch.equal(oa, ob)
    res = P.results(ob)
    assert set(res["status"].tolist()) <= {1, 2, 3, 4, 5}


def test_noalloc_rejects_more_instances_than_its_array(P):
    import ctypes as C
    n = P.PECC_NOALLOC_MAX_INSTANCES + 1
    inst = P.pecc_instances(n, 10, 10 * n, 0x1000, 0x2000, 0)
    rc = P._lib.pecc_lbfgs_descend_noalloc(C.byref(inst), C.c_void_p(0x3000),
                                           C.byref(P.DescentParams().c()), C.c_void_p(0x4000), None)
    assert rc == -1 and b"exceed" in P._lib.pecc_last_error()
