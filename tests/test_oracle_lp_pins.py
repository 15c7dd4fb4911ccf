"""Pins of the learned-proposal oracle (features, network, Adam, top-k).

Each function is pinned to something other than itself: torch's own BF16
conversion, GELU, BCE-with-logits, autograd and Adam on the CPU in FP64;
central finite differences; closed forms on lattices and on a zero network;
SciPy's KD-tree for the neighbor counts; the oracle's separately pinned total
energy for the overlap-energy feature; a sort-based restatement of the
proposal rule.
"""
import math

import numpy as np
import pytest
import torch

import oracle

S = oracle.PARAM_SLICES


def rand_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, scale, oracle.N_PARAMS).astype(np.float32)
    return p.astype(np.float64)


def torch_net(params, round_bf16=True):
    """The same network out of torch modules (FP64 CPU)."""
    p = torch.tensor(params, dtype=torch.float64)

    def w(name):
        a, b = S[name]
        t = p[a:b].clone()
        if round_bf16 and name.startswith("W"):
            t = t.float().to(torch.bfloat16).double()
        return t

    l1 = torch.nn.Linear(8, 64).double()
    l2 = torch.nn.Linear(64, 64).double()
    l3 = torch.nn.Linear(64, 1).double()
    with torch.no_grad():
        l1.weight.copy_(w("W1").view(64, 8)); l1.bias.copy_(w("b1"))
        l2.weight.copy_(w("W2").view(64, 64)); l2.bias.copy_(w("b2"))
        l3.weight.copy_(w("W3").view(1, 64)); l3.bias.copy_(w("b3"))
    net = torch.nn.Sequential(l1, torch.nn.GELU(approximate="none"), l2,
                              torch.nn.GELU(approximate="none"), l3)
    return net, (l1, l2, l3)


def flat_grad(layers):
    l1, l2, l3 = layers
    return np.concatenate([l1.weight.grad.reshape(-1), l1.bias.grad, l2.weight.grad.reshape(-1),
                           l2.bias.grad, l3.weight.grad.reshape(-1),
                           l3.bias.grad]).astype(np.float64)


def rand_x(seed, rows=64):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.5, (rows, 8))


# ---------------------------------------------------------------------------
# BF16 rounding
# ---------------------------------------------------------------------------
def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    w = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8),
                         3.4e38, np.inf, -np.inf, 1e-45]]).astype(np.float32)
    ours = oracle.bf16_round(w)
    ref = torch.from_numpy(w).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1).
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: the even one is 1 + 2^-6.
    out = oracle.bf16_round(np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8], np.float32))
    assert out[0] == 1.0 and out[1] == 1 + 2 ** -6
    assert np.isnan(oracle.bf16_round(np.array([np.nan], np.float32))[0])


# ---------------------------------------------------------------------------
# Network forward / backward
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("round_bf16", [True, False])
def test_forward_matches_torch(round_bf16):
    p, x = rand_params(1), rand_x(2)
    net, _ = torch_net(p, round_bf16)
    ref = net(torch.tensor(x)).detach().numpy().reshape(-1)
    z = oracle.mlp_forward(p, x, round_bf16)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_grad_matches_torch_autograd():
    p, x = rand_params(3), rand_x(4, rows=96)
    y = (np.random.default_rng(5).random(96) < 0.4).astype(np.float64)
    net, layers = torch_net(p, True)
    z = net(torch.tensor(x)).reshape(-1)
    loss = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(y))
    loss.backward()
    ref = flat_grad(layers)
    L, g = oracle.mlp_grad(p, x, y, True)
    assert L == pytest.approx(loss.item(), rel=1e-12)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


def test_grad_finite_differences():
    # Without the BF16 rounding the loss is smooth in the parameters.
    p, x = rand_params(6, 0.3), rand_x(7, rows=16)
    y = np.array([0, 1] * 8, dtype=np.float64)
    L0, g = oracle.mlp_grad(p, x, y, False)
    rng = np.random.default_rng(8)
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(6, b - a), replace=False)
                          for a, b in S.values()])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (oracle.mlp_grad(pp, x, y, False)[0] - oracle.mlp_grad(pm, x, y, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])), (k, fd, g[k])


def test_rounded_equals_unrounded_on_bf16_weights():
    p = rand_params(9)
    p[:4800] = oracle.bf16_round(p[:4800].astype(np.float32))   # biases too: all representable
    x, y = rand_x(10, 32), np.ones(32)
    assert np.array_equal(oracle.mlp_forward(p, x, True), oracle.mlp_forward(p, x, False))
    assert np.array_equal(oracle.mlp_grad(p, x, y, True)[1], oracle.mlp_grad(p, x, y, False)[1])


def test_zero_network_closed_form():
    # W1 = W2 = W3 = 0: z = b3 for every row; only b3 and W3 receive gradient.
    p = np.zeros(oracle.N_PARAMS)
    rng = np.random.default_rng(11)
    p[S["b1"][0]:S["b1"][1]] = rng.normal(size=64)
    p[S["b2"][0]:S["b2"][1]] = b2 = rng.normal(size=64)
    p[4800] = b3 = 0.7
    x, y = rand_x(12, 40), (rng.random(40) < 0.3).astype(float)
    L, g = oracle.mlp_grad(p, x, y, True)
    ybar = y.mean()
    sig = 1.0 / (1.0 + math.exp(-b3))
    assert L == pytest.approx(math.log1p(math.exp(b3)) - ybar * b3, rel=1e-14)
    assert g[4800] == pytest.approx(sig - ybar, rel=1e-13)
    gelu_b2 = np.array([0.5 * t * (1 + math.erf(t / math.sqrt(2))) for t in b2])
    np.testing.assert_allclose(g[S["W3"][0]:S["W3"][1]], (sig - ybar) * gelu_b2, rtol=1e-12)
    assert not g[:S["W3"][0]].any()


def test_loss_stable_for_large_logits():
    p = np.zeros(oracle.N_PARAMS)
    p[4800] = 800.0                                    # exp(800) overflows a double
    L, g = oracle.mlp_grad(p, np.zeros((2, 8)), np.array([0.0, 1.0]))
    assert L == pytest.approx(400.0, rel=1e-14)        # (800 + 0) / 2
    assert g[4800] == pytest.approx(0.5, rel=1e-14)


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------
def test_adam_first_step_closed_form():
    g = np.array([3.0, -2e-3, 0.0, 1e-9])
    p, m, v = oracle.adam(np.ones(4), np.zeros(4), np.zeros(4), g, t=1, lr=0.01, eps=1e-8)
    # bias-corrected first step: lr * g / (|g| + eps)
    np.testing.assert_allclose(p, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15)


def test_adam_matches_torch():
    rng = np.random.default_rng(13)
    p0 = rng.normal(size=300)
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(300), np.zeros(300)
    for t in range(1, 8):
        g = rng.normal(size=300) * (0.1 ** (t % 3))
        w.grad = torch.tensor(g)
        opt.step()
        p, m, v = oracle.adam(p, m, v, g, t, lr=3e-3)
    np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------
def hex_lattice(spacing, radius):
    pts = []
    k = int(radius / spacing) + 2
    for a in range(-k, k + 1):
        for b in range(-k, k + 1):
            x = spacing * (a + 0.5 * b)
            y = spacing * (math.sqrt(3) / 2) * b
            if x * x + y * y <= radius * radius:
                pts.append((x, y))
    return np.array(pts)


def test_features_hex_lattice():
    # Spacing 2 (1 + 1e-6): interior circles nearly touch 6 neighbours (no
    # overlap), the next shell is at 2 sqrt 3 (inside 4), the third just
    # beyond 4: 6 within 2.3 and 12 within 4.
    xy = hex_lattice(2.0 * (1 + 1e-6), 12.0).astype(np.float32)
    R = 40.0
    centre = int(np.argmin((xy.astype(np.float64) ** 2).sum(1)))
    f = oracle.features(xy, R, [centre], xy[[centre]])[0]
    assert f[0] == pytest.approx(0.0, abs=1e-15)       # E = 0 -> log10(1e-20)/20 + 1 = 0
    assert f[1] == 6 and f[5] == 6
    assert f[3] == pytest.approx(12 / (16 * math.pi), rel=1e-15)
    assert f[2] == pytest.approx((R - 1) / R, rel=1e-15)
    assert np.array_equal(f[:4], f[4:])                 # destination = own position, i lifted out


def test_features_two_circles_and_container():
    R = 10.0
    xy = np.array([[0.0, 0.0], [1.5, 0.0]], np.float32)
    f = oracle.features(xy, R, [0], [[0.0, 0.0]])[0]
    e = (2 - 1.5) ** 2
    assert f[0] == pytest.approx(math.log10(e + 1e-20) / 20 + 1, rel=1e-14)
    assert f[1] == 1 and f[3] == pytest.approx(1 / (16 * math.pi))
    # destination outside the container, far from circle 1: containment only
    rho = 9.5
    g = oracle.features(xy, R, [0], [[0.0, -rho]])[0]
    assert g[4] == pytest.approx(math.log10((rho + 1 - R) ** 2 + 1e-20) / 20 + 1, rel=1e-14)
    assert g[5] == 0 and g[7] == 0
    assert g[6] == pytest.approx((R - 1 - rho) / R, rel=1e-14)


def test_feature_counts_match_kdtree():
    from scipy.spatial import cKDTree
    import synth
    inst = synth.C2(1)
    xy = inst.xy
    R = float(inst.R[0])
    rng = np.random.default_rng(14)
    cc = rng.integers(0, 1000, 300).astype(np.int32)
    dest = synth.disk_uniform(300, R, rng).astype(np.float32)
    f = oracle.features(xy, R, cc, dest)
    tree = cKDTree(xy.astype(np.float64))
    for k in range(300):
        i = cc[k]
        for (px, py), base in ((xy[i], 0), (dest[k], 4)):
            p = np.array([px, py], np.float64)
            near = [j for j in tree.query_ball_point(p, 2.3 + 1e-9) if j != i]
            far = [j for j in tree.query_ball_point(p, 4.0 + 1e-9) if j != i]
            # drop exact-boundary hits (the oracle's compares are strict)
            d2 = lambda j: float(((xy[j].astype(np.float64) - p) ** 2).sum())
            near = [j for j in near if d2(j) < 5.29]
            far = [j for j in far if d2(j) < 16.0]
            assert f[k, base + 1] == len(near)
            assert f[k, base + 3] == pytest.approx(len(far) / (16 * math.pi), rel=1e-15)


def test_source_energy_sums_to_total_energy():
    # Summing the source overlap energy over all circles counts each pair
    # twice and each containment term once: 2 E_pair + E_cont.
    import synth
    inst = synth.C1()
    xy = inst.xy
    R = float(inst.R[0])
    n = xy.shape[0]
    f = oracle.features(xy, R, np.arange(n), xy)
    e_i = 10 ** (20 * (f[:, 0] - 1)) - 1e-20
    _, ep, ec, _ = oracle.energy_grad(xy.astype(np.float64), R)
    assert e_i.sum() == pytest.approx(2 * ep + ec, rel=1e-9)


def test_features_reject_bad_index():
    with pytest.raises(ValueError):
        oracle.features(np.zeros((3, 2), np.float32), 5.0, [3], [[0, 0]])


# ---------------------------------------------------------------------------
# Proposal (top-k distinct)
# ---------------------------------------------------------------------------
def propose_by_sort(n, cc, scores, k):
    """The rule restated with a sort: best candidate per circle, then the
    circles ordered by (-score, candidate index)."""
    best = {}
    for c, i in enumerate(cc):
        s = 0.0 if scores is None else float(scores[c])
        if i not in best or s > best[i][0]:
            best[i] = (s, c)
    order = sorted(best.values(), key=lambda t: (-t[0], t[1]))
    return np.array([c for _, c in order[:k]], dtype=np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_propose_matches_sort(seed):
    rng = np.random.default_rng(seed)
    n, C, k = 200, 800, 10
    xy = rng.normal(size=(n, 2)).astype(np.float32)
    cc = rng.integers(0, n, C).astype(np.int32)
    dest = rng.normal(size=(C, 2)).astype(np.float32)
    scores = np.round(rng.normal(size=C), 1).astype(np.float32)   # many ties
    scores[::7] = -0.0
    scores[1::7] = 0.0
    sel, out = oracle.propose(xy, cc, dest, scores, k)
    ref = propose_by_sort(n, cc, scores, k)
    assert np.array_equal(sel, ref)
    assert len(set(cc[sel])) == k
    exp = xy.copy()
    exp[cc[sel]] = dest[sel]
    assert np.array_equal(out, exp)


def test_propose_random_fallback():
    rng = np.random.default_rng(3)
    n, C, k = 50, 120, 8
    xy = rng.normal(size=(n, 2)).astype(np.float32)
    cc = rng.integers(0, n, C).astype(np.int32)
    dest = rng.normal(size=(C, 2)).astype(np.float32)
    first = []
    for c, i in enumerate(cc):
        if i not in [cc[j] for j in first]:
            first.append(c)
    sel, _ = oracle.propose(xy, cc, dest, None, k)
    assert np.array_equal(sel, first[:k])
    bad = rng.normal(size=C).astype(np.float32)
    bad[5] = np.nan
    sel2, _ = oracle.propose(xy, cc, dest, bad, k)
    assert np.array_equal(sel2, sel)


def test_propose_fewer_circles_than_k():
    xy = np.zeros((5, 2), np.float32)
    cc = np.array([1, 1, 3], np.int32)
    sel, out = oracle.propose(xy, cc, np.ones((3, 2), np.float32),
                              np.array([0.1, 0.5, 0.2], np.float32), 4)
    assert np.array_equal(sel, [1, 2])
    assert np.array_equal(out[[1, 3]], np.ones((2, 2))) and not out[[0, 2, 4]].any()
