"""Pins of the partition, sequential batch descent and ANM oracle (Sec. 4.1,
Alg. 1, Sec. 4.3, Alg. 3).

Partitions: sizes floor(n/k) / ceil(n/k) with the larger batches first, and
the order of every kind recomputed with numpy's own routines (arctan2,
hypot, stable sorts, numpy's Philox).  Batch descent: the colour-major
visit of the grid batches equals the grid batch descent without a
displacement cap bit for bit; one batch follows the whole-instance
descent; E never increases.  ANM: with a neighbor structure that holds
every pair the descent equals the exact one and the checks follow the
doubling schedule in closed form; energies over Gamma equal the exact
energy while no circle has moved by 1 or more since Gamma was built."""
import math

import numpy as np
import pytest

import oracle
import synth

KINDS = list(oracle.PARTITIONS)


def disk_points(n, R, seed):
    rng = np.random.default_rng(seed)
    u = rng.random((n, 2))
    r = (R - 1.0) * np.sqrt(u[:, 0])
    t = 2.0 * np.pi * u[:, 1]
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1).astype(np.float32)


def cut(order, n, k):
    """batch_of from an ascending order: consecutive runs, larger first."""
    q, r = divmod(n, k)
    sizes = [q + 1] * r + [q] * (k - r)
    b = np.empty(n, dtype=np.int32)
    pos = 0
    for p, s in enumerate(sizes):
        b[order[pos:pos + s]] = p
        pos += s
    return b


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n,k", [(1000, 5), (300, 3), (17, 4), (3, 5), (1, 1), (64, 1), (101, 15)])
def test_partition_sizes(kind, n, k):
    xy = disk_points(n, math.sqrt(n / 0.84) + 1.0, n * 31 + k)
    b = oracle.partition(xy, kind, k, seed=3)
    assert b.dtype == np.int32 and b.min() >= 0 and b.max() < k
    q, r = divmod(n, k)
    assert np.bincount(b, minlength=k).tolist() == [q + 1] * r + [q] * (k - r)


@pytest.mark.parametrize("n,k", [(1000, 5), (300, 7), (97, 2)])
def test_sector_annulus_fence_match_numpy(n, k):
    xy = disk_points(n, math.sqrt(n / 0.84), 5 + n)
    x, y = xy[:, 0].astype(np.float64), xy[:, 1].astype(np.float64)
    idx = np.arange(n)
    assert np.array_equal(oracle.partition(xy, "sector", k), cut(np.lexsort((idx, np.arctan2(y, x))), n, k))
    assert np.array_equal(oracle.partition(xy, "annulus", k), cut(np.lexsort((idx, np.hypot(x, y))), n, k))
    assert np.array_equal(oracle.partition(xy, "fence", k), cut(np.lexsort((idx, x)), n, k))


def test_sector_axis_points_and_ties():
    # angles: (0,-1) -pi/2, (1,-1e-30) just below 0, origin 0, (1,0) 0,
    # (1,1) pi/4, (-1,1e-30) just below pi, (-1,0) pi, (-2,0) pi
    pts = np.array([[-1, 0], [1, 1], [0, -1], [-2, 0], [1, 0], [0, 0], [-1, 1e-30], [1, -1e-30],
                    [2, 2]], dtype=np.float32)
    b = oracle.partition(pts, "sector", len(pts))     # one circle per batch: the rank
    # (1,1) and (2,2) have equal angles: lower index first
    expect = [2, 7, 4, 5, 1, 8, 6, 0, 3]
    assert b.tolist() == np.argsort(expect).tolist()


def numpy_word0(counter, key):
    c = list(counter)
    c[0] -= 1
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return int(bg.random_raw(4)[0])


@pytest.mark.parametrize("instance", [0, 3])
def test_random_partition_from_numpy_philox(instance):
    n, k, seed = 200, 6, 987654321
    xy = disk_points(n, 16.0, 1)
    keys = [oracle.philox((0, instance, 0, 2 ** 62), (seed, 0))[0]]   # counter word 0 = 0
    keys += [numpy_word0((i, instance, 0, 2 ** 62), (seed, 0)) for i in range(1, n)]
    order = sorted(range(n), key=lambda i: (keys[i], i))
    assert np.array_equal(oracle.partition(xy, "random", k, seed=seed, instance=instance),
                          cut(np.array(order), n, k))
    # positions play no part; the seed and the instance do
    assert np.array_equal(oracle.partition(xy * 0.5, "random", k, seed=seed, instance=instance),
                          oracle.partition(xy, "random", k, seed=seed, instance=instance))
    assert not np.array_equal(oracle.partition(xy, "random", k, seed=seed + 1, instance=instance),
                              oracle.partition(xy, "random", k, seed=seed, instance=instance))


def test_partition_rejects_bad_arguments():
    xy = disk_points(10, 4.0, 0)
    with pytest.raises(ValueError):
        oracle.partition(xy, "sector", 0)
    with pytest.raises(KeyError):
        oracle.partition(xy, "spiral", 3)


def grid_relabelled(x, R, blocks):
    """Grid batches renumbered colour-major (colour, then block index)."""
    import ctypes as C
    n = len(x)
    bo = np.zeros(n, np.int32)
    co = np.zeros(n, np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    oracle.lib().oracle_gbo_batches(n, x.ctypes.data_as(C.POINTER(C.c_double)), float(R), blocks,
                                    bo.ctypes.data_as(C.POINTER(C.c_int32)),
                                    co.ctypes.data_as(C.POINTER(C.c_int32)))
    used = sorted(set(bo.tolist()), key=lambda p: (int(co[bo == p][0]), p))
    lab = {p: r for r, p in enumerate(used)}
    return np.array([lab[p] for p in bo], np.int32), len(used)


@pytest.mark.parametrize("which", ["C2", "C4"])
def test_colour_major_visits_equal_grid_descent(which):
    inst = synth.C2(1) if which == "C2" else synth.C4(1)
    x, R = inst.instance(0).astype(np.float64), float(inst.R[0])
    b, k = grid_relabelled(x, R, 4)
    P = oracle.DescentParams(g_tol=0.0)
    xa, ra, ta = oracle.gbo_seq_descend(x, R, b, k, P, max_outer=4, trace=True)
    xb, rb, tb = oracle.gbo_descend(x, R, P, blocks=4, max_outer=4, jacobi=False,
                                    trace=True)
    assert np.array_equal(xa, xb) and np.array_equal(ta, tb)
    assert (ra["visits"], ra["evals"], ra["gsum"]) == (rb["visits"], rb["evals"], rb["gsum"])


def test_one_batch_follows_whole_descent():
    # one batch: Eq. 7 is Eq. 5 and every visit is an L-BFGS iteration; only
    # the order of the energy's summation differs
    inst = synth.C2(1)
    x, R = inst.instance(0).astype(np.float64), float(inst.R[0])
    P = oracle.DescentParams(g_tol=0.0, max_iter=25)
    xa, ra, _ = oracle.gbo_seq_descend(x, R, np.zeros(len(x), np.int32), 1, P, max_outer=25)
    xb, rb, _ = oracle.descend(x, R, P)
    assert ra["outer"] == rb["iters"] == 25 and ra["visits"] == 25
    assert np.abs(xa - xb).max() < 1e-9
    assert ra["E"] == pytest.approx(rb["E"], rel=1e-9)


@pytest.mark.parametrize("kind", KINDS)
def test_energy_never_increases(kind):
    inst = synth.C4(1)
    x32 = inst.instance(0)
    b = oracle.partition(x32, kind, 5, seed=11)
    _, res, tr = oracle.gbo_seq_descend(x32.astype(np.float64), float(inst.R[0]), b, 5,
                                        oracle.DescentParams(g_tol=0.0), max_outer=40, trace=True)
    assert res["outer"] == 40 and res["visits"] == 200
    assert (np.diff(tr) <= 0.0).all()
    assert tr[-1] < 0.2 * tr[0]


def test_anm_with_every_pair_is_exact_and_doubles():
    inst = synth.C1()
    x, R = inst.instance(0).astype(np.float64), float(inst.R[0])
    b = oracle.partition(inst.instance(0), "sector", 3)
    P = oracle.DescentParams(g_tol=0.0)
    T = 37
    xa, ra, ta = oracle.gbo_seq_descend(x, R, b, 3, P, max_outer=T, anm=True, lcut=4.0 * R,
                                        trace=True)
    xb, rb, tb = oracle.gbo_seq_descend(x, R, b, 3, P, max_outer=T, anm=False, trace=True)
    assert np.array_equal(xa, xb) and np.array_equal(ta, tb)
    # Gamma never changes: checks at calls 1, 3, 7, 15, 31 (len doubling)
    assert ra["outer"] == T
    assert ra["anm_changes"] == 0 and ra["anm_checks"] == int(math.floor(math.log2(T + 1))) == 5


def test_anm_schedule_on_a_stationary_pair():
    # two unit circles in a container of radius 1.5: the symmetric minimum
    # (+-5/6, 0) has E = 1/3; nothing leaves Gamma (l_cut 4)
    a = 5.0 / 6.0
    x = np.array([[-a, 0.0], [a, 0.0]])
    b = np.array([0, 1], np.int32)
    P = oracle.DescentParams(g_tol=0.0, e_feasible=0.0)
    _, res, tr = oracle.gbo_seq_descend(x, 1.5, b, 2, P, max_outer=100, anm=True, lcut=4.0,
                                        trace=True)
    assert tr[0] == pytest.approx(1.0 / 3.0, rel=1e-12)
    assert res["anm_changes"] == 0
    assert res["anm_checks"] == int(math.floor(math.log2(res["outer"] + 1)))


def test_gamma_energy_exact_until_a_circle_moves_by_one():
    inst = synth.C2(1)
    ref = inst.instance(0).astype(np.float64)
    R = float(inst.R[0])
    assert oracle.gamma_energy(ref, ref, R, 4.0) == oracle.energy(ref, R)
    rng = np.random.default_rng(4)
    d = rng.normal(size=ref.shape)
    d *= (0.999 * rng.random((len(ref), 1))) / np.linalg.norm(d, axis=1, keepdims=True)
    moved = ref + d                                   # every circle moved by < 1
    assert oracle.gamma_energy(ref, moved, R, 4.0) == oracle.energy(moved, R)
    # one circle jumps onto a far circle: the new overlap is not in Gamma
    far = ref.copy()
    i = int(np.argmin(np.hypot(ref[:, 0], ref[:, 1])))
    j = int(np.argmax(np.hypot(ref[:, 0] - ref[i, 0], ref[:, 1] - ref[i, 1])))
    far[i] = ref[j] + np.array([0.5, 0.0])
    assert oracle.gamma_energy(ref, far, R, 4.0) < oracle.energy(far, R) - 1.0


# ---------------------------------------------------------------------------
# The paper's dense inverse-Hessian update (Eq. 10-11) and the dense batch
# descent that uses it
# ---------------------------------------------------------------------------
def eq11(H, u, v):
    """Eq. 11 as printed: (I - u v'/b) H (I - v u'/b) + u u'/b, b = v'u."""
    b = float(v @ u)
    I = np.eye(len(u))
    return (I - np.outer(u, v) / b) @ H @ (I - np.outer(v, u) / b) + np.outer(u, u) / b


@pytest.mark.parametrize("d", [1, 4, 37])
def test_bfgs_update_is_eq11(d):
    rng = np.random.default_rng(d)
    A = rng.normal(size=(d, d))
    H = A @ A.T + d * np.eye(d)
    u = rng.normal(size=d)
    v = u + 0.3 * rng.normal(size=d)
    if v @ u <= 0:
        v = -v
    Hn = oracle.bfgs_update(H, u, v)
    assert np.allclose(Hn, eq11(H, u, v), rtol=1e-12, atol=1e-12 * np.abs(H).max())
    assert np.allclose(Hn @ v, u, rtol=1e-10, atol=1e-12)          # secant condition
    assert np.allclose(Hn, Hn.T, rtol=0, atol=1e-12 * np.abs(Hn).max())
    assert np.linalg.eigvalsh(Hn).min() > 0                          # stays positive definite


@pytest.mark.parametrize("k", [1, 2])
def test_dense_steps_follow_eq8_to_eq11(k):
    """Every visit moves its batch by -alpha H_p g(x_p), alpha a power of two
    times alpha0, with H_p rebuilt here from the visited steps by the printed
    Eq. 11 (numpy products) starting from I."""
    inst = synth.C1()
    x0, R = inst.instance(0).astype(np.float64), float(inst.R[0])
    b = oracle.partition(inst.instance(0), "sector", k)
    T = 12
    _, res, _, xs = oracle.gbo_seq_descend(x0, R, b, k, oracle.DescentParams(g_tol=0.0),
                                           max_outer=T, dense=True, xtrace=True)
    assert res["outer"] == T and res["stalled_visits"] == 0
    H = {p: np.eye(2 * int((b == p).sum())) for p in range(k)}
    updated = {p: False for p in range(k)}
    for t in range(T):
        cur = xs[t].copy()
        for p in range(k):
            m = b == p
            g = oracle.energy_grad(cur, R)[3][m].reshape(-1)
            d = -H[p] @ g
            nxt = cur.copy()
            nxt[m] = xs[t + 1][m]
            step = (nxt[m] - cur[m]).reshape(-1)
            alpha = float(step @ d) / float(d @ d)
            assert np.abs(step - alpha * d).max() <= 1e-8 * np.abs(step).max(), (t, p)
            a0 = 1.0 if updated[p] else 1.0 / max(1.0, float(np.linalg.norm(g)))
            j = np.log2(a0 / alpha)
            assert abs(j - round(j)) < 1e-6 and round(j) >= 0, (t, p, alpha)
            y = oracle.energy_grad(nxt, R)[3][m].reshape(-1) - g
            if step @ y > 1e-8 * (y @ y):
                H[p] = eq11(H[p], step, y)
                updated[p] = True
            cur = nxt
