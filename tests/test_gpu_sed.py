"""GPU SED (Sec. 5, Alg. 5) against the oracle: the plan (J-controlled
candidate counts and the packed candidate layout), the Philox perturbation
and the Eq. 18 selection bit for bit on identical inputs; whole chains
statistically (FP32 and FP64 descents part ways after a few steps)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2303_02650_amd as P
    assert torch.cuda.is_available()
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def chains():
    a = synth.C2(1)
    r = synth.C3_restarts()
    c1 = synth.C1()
    return synth.pack([a.instance(0), r.instance(3), c1.instance(0), r.instance(9)],
                      [a.R[0], r.R[3], c1.R[0], r.R[9]])


def plan(P, inst, E_cur, E_best, M, e_stop=1e-25):
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    S = inst.B * M
    m = torch.zeros(inst.B, dtype=torch.int32, device="cuda")
    off = torch.zeros(S + 1, dtype=torch.int32, device="cuda")
    cR = torch.zeros(S, dtype=torch.float32, device="cuda")
    cR64 = torch.zeros(S, dtype=torch.float64, device="cuda")
    P.pecc_sed_plan(d, dev(E_cur), dev(E_best), M, e_stop, m, off, cR, cR64)
    return d, m, off, cR, cR64


def test_plan_counts_and_layout(P):
    inst = chains()
    E_cur = np.array([3.2e-7, 0.7, 0.0, 2e-3])
    E_best = np.array([3.2e-7, 0.5, 0.0, 1e-30])       # chain 2 and 3 have stopped
    M = 12
    d, m, off, cR, cR64 = plan(P, inst, E_cur, E_best, M)
    ref_m = [0 if eb <= 1e-25 else max(1, oracle.sed_J(ec, M)) for ec, eb in zip(E_cur, E_best)]
    assert m.cpu().numpy().tolist() == ref_m == [7, 1, 0, 0]
    n = inst.n
    sizes = [n[b] if j < ref_m[b] else 0 for b in range(inst.B) for j in range(M)]
    assert np.array_equal(off.cpu().numpy(), np.concatenate([[0], np.cumsum(sizes)]))
    assert np.array_equal(cR64.cpu().numpy(), np.repeat(inst.R, M))


def test_perturbation_matches_oracle(P):
    inst = chains()
    M, seed, it = 5, 987654321, 13
    E_cur = np.array([2e-3, 0.4, 1e-9, 0.02])
    d, m, off, cR, cR64 = plan(P, inst, E_cur, np.full(4, 1.0), M)
    cand = torch.zeros(2 * int(off[-1].item()) + 2, dtype=torch.float32, device="cuda")
    P.pecc_sed_perturb(d, dev(inst.xy.reshape(-1)), M, m, off, seed, it, cand)
    cand = cand.cpu().numpy()
    offh = off.cpu().numpy()
    mh = m.cpu().numpy()
    for b in range(inst.B):
        for j in range(mh[b]):
            c = b * M + j
            got = cand[2 * offh[c]:2 * offh[c + 1]].reshape(-1, 2)
            ref = oracle.sed_perturb(inst.instance(b), seed, b, it, j)
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (b, j)


@pytest.mark.parametrize("case", ["argmin", "softmax", "stopped"])
def test_selection_matches_oracle(P, case):
    inst = chains()
    M, seed, it = 6, 55, 4
    rng = np.random.default_rng(8)
    E_cur = np.array([1e-6, 1e-4, 3e-3, 2e-5])
    E_best = np.array([1e-6, 1e-5, 1e-3, 2e-5]) if case != "stopped" else np.array([1e-6, 0.0, 1e-3, 2e-5])
    d, m, off, cR, cR64 = plan(P, inst, E_cur, E_best, M)
    S = inst.B * M
    # candidate layouts: distinct values per slot so that the copied one is identifiable
    total = int(off[-1].item())
    cand = torch.from_numpy(rng.normal(size=2 * max(total, 1)).astype(np.float32)).cuda()
    if case == "argmin":
        cE = rng.uniform(1e-8, 1e-3, S)              # some candidate beats every E_cur
    else:
        cE = rng.uniform(5e-3, 1e-1, S)              # none does: the softmax(J) draw
    cE[2::3] = cE[1::3]                               # ties
    xy_cur = dev(inst.xy.reshape(-1).copy())
    xy_best = dev(inst.xy.reshape(-1).copy())
    Ec, Eb = dev(E_cur), dev(E_best)
    chosen = torch.zeros(inst.B, dtype=torch.int32, device="cuda")
    P.pecc_sed_select(d, M, m, off, cand, dev(cE), seed, it, xy_cur, Ec, xy_best, Eb, chosen)
    mh, offh, ch = m.cpu().numpy(), off.cpu().numpy(), chosen.cpu().numpy()
    candh = cand.cpu().numpy()
    for b in range(inst.B):
        if mh[b] == 0:
            assert ch[b] == -1
            continue
        k = oracle.sed_select(cE[b * M:b * M + mh[b]], E_cur[b], oracle.sed_uniform(seed, b, it), M)
        assert ch[b] == k, (b, ch[b], k)
        c = b * M + k
        seg = candh[2 * offh[c]:2 * offh[c + 1]]
        o = inst.offset
        assert np.array_equal(xy_cur.cpu().numpy()[2 * o[b]:2 * o[b + 1]], seg)
        assert Ec.cpu().numpy()[b] == cE[c]
        better = cE[c] < E_best[b]
        assert Eb.cpu().numpy()[b] == (cE[c] if better else E_best[b])
        expect_best = seg if better else inst.xy.reshape(-1)[2 * o[b]:2 * o[b + 1]]
        assert np.array_equal(xy_best.cpu().numpy()[2 * o[b]:2 * o[b + 1]], expect_best)


def test_chains_improve_and_stop(P):
    """32 chains of n = 20 at R = 4.95 (density 0.82): every chain's best
    energy is at most its start and some improve, and the whole run is
    reproducible."""
    from paper_2303_02650_amd.sed import SedChains
    inst = synth.instance_set(32, 20, 4.95, seed=21)
    prm = P.DescentParams(g_tol=1e-6, ftol=1e-7, contact_margin=1e-4)
    runs = []
    for _ in range(2):
        d = P.DeviceInstances.from_host(inst.offset, inst.R)
        ch = SedChains(d, dev(inst.xy.reshape(-1).copy()), prm, M=25, seed=3)
        info = ch.run(40)
        runs.append((ch.E_best.cpu().numpy(), ch.xy_best.cpu().numpy(), info, ch.E_start.cpu().numpy(),
                     ch.m.cpu().numpy()))
    Eb, xb, info, E0, m = runs[0]
    assert np.array_equal(Eb, runs[1][0]) and np.array_equal(xb, runs[1][1])
    assert (Eb <= E0).all() and (Eb < E0).any()
    assert info["iterations"] <= 40 and info["descents"] > 32
    # the best records are what they claim: FP64 energies of unit circles
    for b in range(0, 32, 5):
        x = xb.reshape(-1, 2)[inst.offset[b]:inst.offset[b + 1]]
        v = oracle.verify(x, float(inst.R[b]))
        assert v["E"] == pytest.approx(Eb[b], rel=1e-9, abs=1e-300)
