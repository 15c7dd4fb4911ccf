"""HIP-graph capture of the library's calls: every replay must reproduce the
eager result bit for bit (the kernels are deterministic), with eager work and
synchronisations between replays."""
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


def capture(fn):
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            fn()
    torch.cuda.synchronize()
    return g


def test_descent_and_verify_graph_replays(P):
    inst = synth.C2(16)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    x0 = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    x = torch.empty_like(x0)
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4).c()
    ws = torch.empty(P.pecc_lbfgs_descend_workspace_size(d), dtype=torch.uint8, device="cuda")
    out = torch.empty(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    e64 = torch.empty(d.B, dtype=torch.float64, device="cuda")
    feas = torch.empty(d.B, dtype=torch.int32, device="cuda")

    def step():
        x.copy_(x0)
        P.pecc_lbfgs_descend(d, x, prm, out, ws)
        P.pecc_verify(d, x, 1e-20, e64, None, None, feas)

    step()
    torch.cuda.synchronize()
    ref = (x.clone(), out.clone(), e64.clone(), feas.clone())
    g = capture(step)
    row, col = P.build_neighbors(d, x0)
    for rep in range(3):
        x.zero_(); out.zero_(); e64.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, ref[0]) and torch.equal(out, ref[1]), rep
        assert torch.equal(e64, ref[2]) and torch.equal(feas, ref[3]), rep
        P.energy_grad(d, x0, row, col)            # eager work between replays
        torch.cuda.synchronize()


def test_proposal_step_graph_replays(P):
    inst = synth.C2(8)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    cc, cd = synth.candidates(inst, 2048, synth.rng_for(41))
    ccd, cdd = torch.from_numpy(cc.reshape(-1)).cuda(), torch.from_numpy(cd.reshape(-1)).cuda()
    params = P.init_params(3)
    feats = torch.empty(d.B * 2048, 8, dtype=torch.float32, device="cuda")
    logits = torch.empty(d.B * 2048, dtype=torch.float32, device="cuda")
    xy_new = torch.empty_like(xy)
    sel = torch.empty(d.B, 50, dtype=torch.int32, device="cuda")

    def step():
        P.pecc_features(d, xy, 2048, ccd, cdd, feats)
        P.pecc_mlp_forward(params, feats, d.B * 2048, logits)
        P.pecc_propose(d, xy, 2048, ccd, cdd, logits, 50, sel, xy_new)

    step()
    torch.cuda.synchronize()
    ref = (feats.clone(), logits.clone(), sel.clone(), xy_new.clone())
    g = capture(step)
    for rep in range(3):
        feats.zero_(); logits.zero_(); sel.zero_(); xy_new.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = (feats, logits, sel, xy_new)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), rep
        P.mlp_forward(params, feats[:100])           # eager work between replays
        torch.cuda.synchronize()


def test_train_step_graph_replays_advance_like_eager(P):
    rng = np.random.default_rng(42)
    x = torch.from_numpy(rng.normal(size=(4096, 8)).astype(np.float32)).cuda()
    y = torch.from_numpy((rng.random(4096) < 0.5).astype(np.float32)).cuda()
    p0 = P.init_params(5)
    eager = P.MlpTrainer(p0, lr=1e-3, max_rows=4096)
    for _ in range(3):
        eager.train_step(x, y)
    torch.cuda.synchronize()
    T = P.MlpTrainer(p0, lr=1e-3, max_rows=4096)
    g = capture(lambda: T.train_step(x, y))
    # capturing does not run the work: the state is still the initial one
    assert T.step.item() == 0 and torch.equal(T.params, p0)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        P.mlp_forward(T.params, x[:64])              # eager work between replays
        torch.cuda.synchronize()
    assert T.step.item() == 3
    assert torch.equal(T.params, eager.params) and torch.equal(T.m, eager.m)
    assert torch.equal(T.v, eager.v)


def test_partition_and_kbatch_descents_graph_replays(P):
    inst = synth.C1()
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    x0 = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    x_l, x_d = torch.empty_like(x0), torch.empty_like(x0)
    bo = torch.empty(d.total_n, dtype=torch.int32, device="cuda")
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4).c()
    ws_l = torch.empty(P.pecc_gbo_kbatch_descend_workspace_size(d), dtype=torch.uint8, device="cuda")
    ws_d = torch.empty(P.pecc_gbo_kbatch_bfgs_workspace_size(d, 7), dtype=torch.uint8, device="cuda")
    out_l = torch.empty(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    out_d = torch.empty_like(out_l)

    def step():
        P.pecc_partition(d, x0, P.PARTITIONS["sector"], 3, 0, bo)
        x_l.copy_(x0)
        x_d.copy_(x0)
        P.pecc_gbo_kbatch_descend(d, x_l, bo, 3, 0, prm, out_l, ws_l)
        P.pecc_gbo_kbatch_bfgs_descend(d, x_d, bo, 3, 0, 7, prm, out_d, ws_d)

    step()
    torch.cuda.synchronize()
    ref = (bo.clone(), x_l.clone(), out_l.clone(), x_d.clone(), out_d.clone())
    g = capture(step)
    for rep in range(3):
        bo.fill_(-1); x_l.zero_(); x_d.zero_(); out_l.zero_(); out_d.zero_()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((bo, x_l, out_l, x_d, out_d), ref):
            assert torch.equal(a, b), rep
        P.partition(d, x0, "fence", 2)                   # eager work between replays
        torch.cuda.synchronize()


def test_concurrent_launches_on_several_streams_match_sequential(P):
    """The same descents and verifies issued on four streams at once (own
    buffers per stream, two rounds, plain launches): every stream's results
    equal the sequential run's bit for bit, whichever workgroups and CUs the
    overlapping persistent launches got."""
    inst = synth.C2(64)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    x0 = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4).c()
    nws = P.pecc_lbfgs_descend_workspace_size(d)

    def buffers():
        return (torch.empty_like(x0), torch.zeros(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8,
                                                  device="cuda"),
                torch.empty(nws, dtype=torch.uint8, device="cuda"),
                torch.zeros(d.B, dtype=torch.float64, device="cuda"),
                torch.zeros(d.B, dtype=torch.int32, device="cuda"))

    def step(b):
        x, out, ws, e64, feas = b
        x.copy_(x0)
        P.pecc_lbfgs_descend(d, x, prm, out, ws)
        P.pecc_verify(d, x, 1e-20, e64, None, None, feas)

    ref = buffers()
    step(ref)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(4)]
    sets = [buffers() for _ in streams]
    for _ in range(2):
        for st, b in zip(streams, sets):
            with torch.cuda.stream(st):
                step(b)
    torch.cuda.synchronize()
    for k, b in enumerate(sets):
        for got, want in zip(b[:2] + b[3:], ref[:2] + ref[3:]):
            assert torch.equal(got, want), k


def test_back_to_back_replays_like_the_benchmark(P):
    """The benchmark's timed loop: K steps, each a replay of the captured
    reset + descent graph and of the captured verify graph, back to back on
    one stream with events between them and no host synchronisation.  Every
    step's results (copied aside on the same stream) equal the eager step's
    bit for bit."""
    inst = synth.C2(64)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    x0 = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    x = torch.empty_like(x0)
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, ftol_window=20, contact_margin=1e-4,
                          tau64=1e-5).c()
    ws = torch.empty(P.pecc_lbfgs_descend_workspace_size(d), dtype=torch.uint8, device="cuda")
    out = torch.empty(d.B * P.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    e64 = torch.empty(d.B, dtype=torch.float64, device="cuda")
    mp_ = torch.empty_like(e64)
    mc_ = torch.empty_like(e64)
    feas = torch.empty(d.B, dtype=torch.int32, device="cuda")

    def descend_once():
        x.copy_(x0)
        P.pecc_lbfgs_descend(d, x, prm, out, ws)

    def verify_once():
        P.pecc_verify(d, x, 1e-20, e64, mp_, mc_, feas)

    descend_once(); verify_once()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (x, out, e64, mp_, mc_, feas)]
    g_desc, g_ver = capture(descend_once), capture(verify_once)
    K = 6
    hist = [[torch.empty_like(t) for t in ref] for _ in range(K)]
    for t in (x, out, e64, mp_, mc_, feas):
        t.zero_()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    for k, (e0, e1, e2) in enumerate(evs):
        e0.record(stream)
        g_desc.replay()
        e1.record(stream)
        g_ver.replay()
        e2.record(stream)
        for h, t in zip(hist[k], (x, out, e64, mp_, mc_, feas)):
            h.copy_(t)
    torch.cuda.synchronize()
    for k in range(K):
        for h, r in zip(hist[k], ref):
            assert torch.equal(h, r), k
        assert evs[k][0].elapsed_time(evs[k][1]) > 0.0
