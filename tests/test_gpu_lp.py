"""GPU parity of the learned-proposal kernels against the oracle.

Features: counts bit-exact, the rest within FP32 rounding of the FP64 oracle.
Network forward and gradient: relative error in norm <= 1e-2 against the
FP64 oracle over the same BF16-rounded weights (BF16 products with FP32
accumulation).  Adam: the FP32 update against the FP64 update on the same
inputs.  Proposal: bit-exact on identical FP32 scores.
"""
import math

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


def instances():
    """C2 seed 1, two C3 restart layouts (converged + relocated) and a tiny one."""
    a = synth.C2(1)
    r = synth.C3_restarts()
    xs = [a.instance(0), r.instance(0), r.instance(5), synth.C1().instance(0)]
    Rs = [a.R[0], r.R[0], r.R[5], synth.C1().R[0]]
    return synth.pack(xs, Rs)


def rand_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(oracle.N_PARAMS, dtype=np.float32)
    p[0:512] = rng.normal(0, math.sqrt(2 / 8), 512)
    p[512:576] = rng.normal(0, 0.1, 64)
    p[576:4672] = rng.normal(0, math.sqrt(2 / 64), 4096)
    p[4672:4736] = rng.normal(0, 0.1, 64)
    p[4736:4800] = rng.normal(0, math.sqrt(1 / 64), 64)
    p[4800] = 0.1
    return p


def feature_like_rows(seed, rows):
    """Rows in the range real features take (energies, counts, gaps, densities)."""
    rng = np.random.default_rng(seed)
    x = np.stack([rng.random(rows), rng.integers(0, 7, rows), rng.random(rows) - 0.05,
                  rng.integers(0, 14, rows) / (16 * math.pi), rng.random(rows),
                  rng.integers(0, 7, rows), rng.random(rows) - 0.05,
                  rng.integers(0, 14, rows) / (16 * math.pi)], axis=1)
    return x.astype(np.float32)


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------
def test_features_match_oracle(P):
    inst = instances()
    C = 1500                      # two chunks of 1024, ragged second
    cc, cd = synth.candidates(inst, C, synth.rng_for(21))
    cc[0, 7] = -1                 # invalid indices give NaN rows
    cc[1, 9] = inst.n[1]
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    f = P.features(d, dev(inst.xy.reshape(-1)), dev(cc.reshape(-1)), dev(cd.reshape(-1))).cpu().numpy()
    f = f.reshape(inst.B, C, 8)
    for b in range(inst.B):
        ok = (cc[b] >= 0) & (cc[b] < inst.n[b])
        ref = oracle.features(inst.instance(b), inst.R[b], cc[b][ok], cd[b][ok])
        got = f[b][ok]
        for col in (1, 5):
            assert np.array_equal(got[:, col], ref[:, col]), (b, col)
        for col in (3, 7):
            assert np.array_equal(np.round(got[:, col] * 16 * math.pi), np.round(ref[:, col] * 16 * math.pi))
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-6)
        assert np.isnan(f[b][~ok]).all()


def test_features_deterministic(P):
    inst = synth.C2(2)
    cc, cd = synth.candidates(inst, 4096, synth.rng_for(22))
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    args = (dev(inst.xy.reshape(-1)), dev(cc.reshape(-1)), dev(cd.reshape(-1)))
    a = P.features(d, *args)
    b = P.features(d, *args)
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rows", [1, 17, 4133])
def test_forward_matches_oracle(P, rows):
    p = rand_params(1)
    x = feature_like_rows(2, rows)
    z = P.mlp_forward(dev(p), dev(x)).cpu().numpy().astype(np.float64)
    ref = oracle.mlp_forward(p.astype(np.float64), x.astype(np.float64))
    assert np.linalg.norm(z - ref) <= 1e-2 * np.linalg.norm(ref)
    assert np.abs(z - ref).max() <= 1e-2 * (1 + np.abs(ref).max())


def test_forward_on_real_features(P):
    inst = synth.C2(1)
    cc, cd = synth.candidates(inst, 2000, synth.rng_for(23))
    x = oracle.features(inst.instance(0), inst.R[0], cc[0], cd[0]).astype(np.float32)
    p = rand_params(3)
    z = P.mlp_forward(dev(p), dev(x)).cpu().numpy().astype(np.float64)
    ref = oracle.mlp_forward(p.astype(np.float64), x.astype(np.float64))
    assert np.linalg.norm(z - ref) <= 1e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("rows", [5, 3000])
def test_grad_matches_oracle(P, rows):
    p = rand_params(4)
    x = feature_like_rows(5, rows)
    y = (np.random.default_rng(6).random(rows) < 0.4).astype(np.float32)
    loss, g = P.mlp_grad(dev(p), dev(x), dev(y))
    L, ref = oracle.mlp_grad(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    assert loss.item() == pytest.approx(L, rel=1e-3)
    g = g.cpu().numpy().astype(np.float64)
    for name, (a, b) in oracle.PARAM_SLICES.items():
        err = np.linalg.norm(g[a:b] - ref[a:b])
        assert err <= 1e-2 * np.linalg.norm(ref[a:b]) + 1e-12, name


def test_grad_empty_and_deterministic(P):
    p = dev(rand_params(7))
    x = dev(feature_like_rows(8, 2049))
    y = dev((np.arange(2049) % 3 == 0).astype(np.float32))
    l1, g1 = P.mlp_grad(p, x, y)
    l2, g2 = P.mlp_grad(p, x, y)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)
    l0, g0 = P.mlp_grad(p, x[:0], y[:0])
    assert l0.item() == 0.0 and not g0.any()


def test_adam_matches_oracle(P):
    rng = np.random.default_rng(9)
    p0 = rand_params(10)
    T = P.MlpTrainer(dev(p0), lr=3e-3)
    p, m, v = p0.astype(np.float64), np.zeros(oracle.N_PARAMS), np.zeros(oracle.N_PARAMS)
    for t in range(1, 4):
        g = (rng.normal(size=oracle.N_PARAMS) * 10.0 ** rng.integers(-6, 0, oracle.N_PARAMS)).astype(np.float32)
        P.pecc_mlp_adam(T.params, T.m, T.v, dev(g), T.step, T.hp)
        p, m, v = oracle.adam(p, m, v, g.astype(np.float64), t, lr=3e-3)
    got = T.params.cpu().numpy().astype(np.float64)
    tol = 4 * np.spacing(np.abs(p).astype(np.float32)).astype(np.float64) + 1e-5 * 3e-3
    assert (np.abs(got - p) <= tol).all()
    assert T.step.item() == 3


def test_train_step_is_grad_then_adam(P):
    p0 = dev(rand_params(11))
    x = dev(feature_like_rows(12, 700))
    y = dev((np.arange(700) % 2).astype(np.float32))
    A = P.MlpTrainer(p0, lr=1e-3)
    B = P.MlpTrainer(p0, lr=1e-3)
    for _ in range(3):
        A.train_step(x, y)
        loss, g = P.mlp_grad(B.params, x, y)
        P.pecc_mlp_adam(B.params, B.m, B.v, g, B.step, B.hp)
    assert torch.equal(A.params, B.params) and torch.equal(A.m, B.m) and torch.equal(A.v, B.v)


def test_training_learns_a_separable_rule(P):
    # label = 1 where the destination's overlap feature is below 0.5
    x = feature_like_rows(13, 8192)
    y = (x[:, 4] < 0.5).astype(np.float32)
    xd, yd = dev(x), dev(y)
    T = P.MlpTrainer(P.init_params(0), lr=3e-3, max_rows=1024)
    first = None
    for it in range(400):
        a = (it * 1024) % 8192
        loss = T.train_step(xd[a:a + 1024], yd[a:a + 1024]).item()
        first = loss if first is None else first
    z = P.mlp_forward(T.params, xd).cpu().numpy()
    acc = ((z > 0) == (y > 0.5)).mean()
    assert loss < 0.5 * first and acc > 0.95, (first, loss, acc)


# ---------------------------------------------------------------------------
# Proposal and acceptance
# ---------------------------------------------------------------------------
def proposal_case(seed, C=600, k=50):
    inst = instances()
    rng = synth.rng_for(seed)
    cc, cd = synth.candidates(inst, C, rng)
    scores = np.round(rng.normal(size=(inst.B, C)), 1).astype(np.float32)   # many ties
    scores[:, ::11] = -0.0
    scores[:, 1::11] = 0.0
    cc[2, 3] = -5                 # ignored
    return inst, cc, cd, scores, k


@pytest.mark.parametrize("mode", ["scores", "random", "nan"])
def test_propose_matches_oracle(P, mode):
    inst, cc, cd, scores, k = proposal_case(31)
    if mode == "nan":
        scores[1, 17] = np.nan    # instance 1 falls back to random, the others keep scores
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    sc = None if mode == "random" else dev(scores.reshape(-1))
    xy_out, sel = P.propose(d, dev(inst.xy.reshape(-1)), dev(cc.reshape(-1)), dev(cd.reshape(-1)),
                            sc, k)
    xy_out = xy_out.cpu().numpy().reshape(-1, 2)
    sel = sel.cpu().numpy()
    for b in range(inst.B):
        s_b = None if mode == "random" else scores[b]
        ref_sel, ref_xy = oracle.propose(inst.instance(b), cc[b], cd[b], s_b, k)
        got = sel[b][sel[b] >= 0]
        assert np.array_equal(got, ref_sel), b
        assert (sel[b][len(ref_sel):] == -1).all()
        assert np.array_equal(xy_out[inst.offset[b]:inst.offset[b + 1]], ref_xy), b


def test_propose_k_beyond_distinct_circles(P):
    inst = synth.C1()                                 # n = 20
    cc, cd = synth.candidates(inst, 64, synth.rng_for(32))
    scores = np.random.default_rng(33).normal(size=64).astype(np.float32)
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy_out, sel = P.propose(d, dev(inst.xy.reshape(-1)), dev(cc.reshape(-1)), dev(cd.reshape(-1)),
                            dev(scores), 40)
    ref_sel, ref_xy = oracle.propose(inst.instance(0), cc[0], cd[0], scores, 40)
    sel = sel.cpu().numpy()[0]
    assert len(ref_sel) == len(set(cc[0].tolist())) < 40
    assert np.array_equal(sel[:len(ref_sel)], ref_sel) and (sel[len(ref_sel):] == -1).all()
    assert np.array_equal(xy_out.cpu().numpy().reshape(-1, 2), ref_xy)


def test_accept_keeps_lower_energy(P):
    inst = instances()
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    cur = dev(inst.xy.reshape(-1))
    new = cur + 1.0
    e_cur = dev(np.array([1.0, 2.0, 0.0, 5.0]))
    e_new = dev(np.array([0.5, 2.0, 1e-30, np.nan]))
    acc = P.accept(d, cur, e_cur, new, e_new).cpu().numpy()
    assert acc.tolist() == [1, 0, 0, 0]
    assert e_cur.cpu().numpy().tolist() == [0.5, 2.0, 0.0, 5.0]
    out = cur.cpu().numpy().reshape(-1, 2)
    o = inst.offset
    assert np.array_equal(out[o[0]:o[1]], inst.instance(0) + 1.0)
    assert np.array_equal(out[o[1]:], inst.xy[o[1]:])


# ---------------------------------------------------------------------------
# The trained proposal against random proposals (statistical; parity unpinned)
# ---------------------------------------------------------------------------
def test_paired_arms_without_network_are_identical(P):
    from paper_2303_02650_amd import proposal as PR
    inst = synth.C5(16)
    s = PR.compare(None, R=34.4, instances=16, budget=3, seed=9, xy0=inst.xy).summary()
    assert s["mean_saving"] == 0.0 and s["learned_better"] == s["random_better"] == 0


def test_learned_proposal_needs_fewer_descents_than_random(P):
    """Trained on accept/reject outcomes of random relocations of converged
    n = 1000 layouts (R in [34.3, 34.6]), evaluated on 128 fresh instances at
    R = 34.4: descents until the first FP64-feasible layout, paired against
    random proposals drawn from the same candidates."""
    from paper_2303_02650_amd import proposal as PR
    F, Y, st = PR.generate_samples(20000, R_range=(34.3, 34.6), seed=1)
    assert F.shape[0] >= 20000 * 50 and 0.2 < Y.mean().item() < 0.8
    scorer, hist = PR.train(F, Y, epochs=16)
    assert hist[-1] < hist[0]
    s = PR.compare(scorer, R=34.4, instances=128, budget=16, seed=6,
                   xy0=synth.C5(128).xy).summary()
    print(s)
    assert s["mean_saving"] > 0 and s["saving_ci95"][0] > 0, s
    assert s["feasible_learned"] >= s["feasible_random"], s
