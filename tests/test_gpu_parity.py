"""GPU parity of libpecc against the FP64 oracle (run on an MI355X).

Neighbor sets: bit-exact.  Energy and gradient: |E32 - E64| <= 1e-5 E64 and
||g32 - g64||_2 <= 1e-5 ||g64||_2 per instance at workload input states
(random layouts with O(1) overlaps).  FP64 verify: 1e-12 relative (only the
summation order differs).  Descent: early iterations follow the oracle's
trajectory; whole descents are compared by outcome.
"""
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


def to_dev(P, inst: synth.Instances):
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    xy = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    return d, xy


def mixed_batch(seed=0, sizes=(0, 1, 2, 17, 64, 333, 700, 1000, 1024, 513)):
    rng = synth.rng_for(seed)
    xys, Rs = [], []
    for n in sizes:
        R = float(np.sqrt(max(n, 1) / 0.84)) if n > 3 else 3.0
        xys.append(synth.disk_uniform(n, R, rng))
        Rs.append(R)
    return synth.pack(xys, Rs)


def crowded_batch():
    # 35 circles inside a disk of radius 0.6: each has more than 24
    # neighbors within the cutoff, which the descent's list cannot hold
    rng = synth.rng_for(8)
    core = synth.disk_uniform(35, 1.6, rng)
    rest = synth.disk_uniform(25, 8.0, rng)
    return synth.pack([np.concatenate([core, rest])], [8.0])


def tight_batch():
    # circles far denser than any packing: several thousand listed pairs per
    # instance (up to ~23k), more than the sweep stages in LDS at once
    rng = synth.rng_for(12)
    sizes_R = ((1024, 13.0), (600, 10.0), (300, 30.0))
    return synth.pack([synth.disk_uniform(n, R, rng) for n, R in sizes_R], [R for _, R in sizes_R])


BATCHES = {
    "C1": lambda: synth.C1(),
    "crowded": crowded_batch,
    "tight": tight_batch,
    "C2": lambda: synth.C2(1),
    "mixed": lambda: mixed_batch(0),
    "C3starts": lambda: synth.C3(24),
    "C4x8": lambda: synth.C4(8),
    "C3restarts": lambda: synth.C3_restarts(),
}


# ---------------------------------------------------------------------------
# neighbor lists
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(BATCHES))
@pytest.mark.parametrize("form", [0, 1, 2])
def test_neighbor_sets_bit_exact(P, name, form):
    inst = BATCHES[name]()
    d, xy = to_dev(P, inst)
    row, col = P.build_neighbors(d, xy, 2.3, 0.0, form)
    assert col.dtype == (torch.int16 if form == P.LIST_LOCAL16 else torch.int32)
    full = form != P.LIST_HALF
    row = row.cpu().numpy()
    col = col.cpu().numpy().astype(np.int64)
    assert row[0] == 0 and row[-1] == len(col)
    for b in range(inst.B):
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        pi, pj = oracle.neighbors(inst.instance(b), 2.3)
        want = {}
        for i, j in zip(pi.tolist(), pj.tolist()):
            want.setdefault(i, []).append(j)
            if full:
                want.setdefault(j, []).append(i)
        base = 0 if form == P.LIST_LOCAL16 else o0      # local indices need no offset
        for i in range(o1 - o0):
            got = col[row[o0 + i]:row[o0 + i + 1]] - base
            w = sorted(want.get(i, []))
            assert got.tolist() == w, (name, b, i)


def test_neighbor_cell_sizes_agree(P):
    inst = synth.C2(1)
    d, xy = to_dev(P, inst)
    r0, c0 = P.build_neighbors(d, xy, 2.3, 0.0, True)
    for h in (2.5, 3.45, 7.0):
        r, c = P.build_neighbors(d, xy, 2.3, h, True)
        assert torch.equal(r, r0) and torch.equal(c, c0)


def test_neighbor_capacity_overflow_reports_need(P):
    inst = synth.C2(1)
    d, xy = to_dev(P, inst)
    row_full, col_full = P.build_neighbors(d, xy, 2.3, 0.0, False)
    need = col_full.numel()
    row = torch.empty(inst.total_n + 1, dtype=torch.int32, device="cuda")
    col = torch.full((need // 2,), -7, dtype=torch.int32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(P.pecc_build_neighbors_workspace_size(d), dtype=torch.uint8, device="cuda")
    P.pecc_build_neighbors(d, xy, 2.3, 0.0, 0, row, col, need // 2, npairs, ws)
    assert int(npairs.item()) == need
    assert torch.equal(row, row_full)
    # rows that end within the capacity are complete; the row that crosses
    # it holds some of its entries; nothing is written beyond capacity
    r = row.cpu().numpy()
    cut = r[np.searchsorted(r, need // 2, side="right") - 1]
    assert torch.equal(col[:cut], col_full[:cut])
    assert (col[cut:] != -7).all()


def test_neighbor_degenerate_layouts(P):
    # coincident circles, circles far outside the container, one cell
    xy = np.array([[0, 0], [0, 0], [0, 0], [50, 50], [50.5, 50], [-40, 3], [1.0, 0.5]])
    inst = synth.pack([xy, np.zeros((0, 2)), np.array([[1e3, -1e3]])], [3.0, 5.0, 2.0])
    d, x = to_dev(P, inst)
    row, col = P.build_neighbors(d, x, 2.3, 0.0, False)
    row = row.cpu().numpy(); col = col.cpu().numpy()
    pi, pj = oracle.neighbors(inst.instance(0), 2.3)
    got = [(i, int(j)) for i in range(7) for j in col[row[i]:row[i + 1]]]
    assert got == list(zip(pi.tolist(), pj.tolist()))


# ---------------------------------------------------------------------------
# energy and gradient
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(BATCHES))
@pytest.mark.parametrize("form", [0, 2])
def test_energy_grad_within_1e5(P, name, form):
    inst = BATCHES[name]()
    d, xy = to_dev(P, inst)
    row, col = P.build_neighbors(d, xy, 2.3, 0.0, form)
    E, g = P.energy_grad(d, xy, row, col, form=form)
    E = E.cpu().numpy()
    g = g.cpu().numpy().reshape(-1, 2)
    worst = 0.0
    for b in range(inst.B):
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        E64, _, _, g64 = oracle.energy_grad(inst.instance(b).astype(np.float64), inst.R[b])
        if o1 - o0 == 0:
            assert E[b] == 0.0
            continue
        errE = abs(E[b] - E64) / max(E64, 1e-30)
        errg = np.linalg.norm(g[o0:o1] - g64) / max(np.linalg.norm(g64), 1e-30)
        worst = max(worst, errE, errg)
        if E64 > 1e-3:   # workload states: O(1) overlaps
            assert errE <= 1e-5, (name, b, errE)
            assert errg <= 1e-5, (name, b, errg)
    print(f"{name}: worst relative error vs FP64 {worst:.3e}")


@pytest.mark.parametrize("name", ["C2", "mixed", "crowded", "tight", "C3restarts"])
def test_energy_grad_list_forms_agree(P, name):
    """The three list forms hold the same pairs.  The two with both
    orientations (int32 global, uint16 local) run the same sweep: the same
    bits.  The half list forms each pair's term once (the product rounded
    before it is added, where the other sweep fuses the multiply-add) and
    adds the same terms in another order: equal to FP32 rounding."""
    inst = BATCHES[name]()
    d, xy = to_dev(P, inst)
    rh, ch = P.build_neighbors(d, xy, 2.3, 0.0, P.LIST_HALF)
    rf, cf = P.build_neighbors(d, xy, 2.3, 0.0, P.LIST_FULL)
    rl, cl = P.build_neighbors(d, xy, 2.3, 0.0, P.LIST_LOCAL16)
    assert cf.numel() == 2 * ch.numel() == cl.numel() and torch.equal(rf, rl)
    Eh, gh = P.energy_grad(d, xy, rh, ch, form=P.LIST_HALF)
    Ef, gf = P.energy_grad(d, xy, rf, cf, form=P.LIST_FULL)
    El, gl = P.energy_grad(d, xy, rl, cl, form=P.LIST_LOCAL16)
    assert torch.equal(Ef, El) and torch.equal(gf, gl)
    gh64, gf64 = gh.cpu().numpy().astype(np.float64), gf.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gh64 - gf64) <= 1e-6 * np.linalg.norm(gf64)
    Eh, Ef = Eh.cpu().numpy().astype(np.float64), Ef.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Eh - Ef) <= 1e-6 * np.abs(Ef)), (Eh, Ef)
    # a list with both orientations read as a half list: the same pairs,
    # the same bits as the half list itself
    Ex, gx = P.energy_grad(d, xy, rf, cf, form=P.LIST_HALF)
    assert torch.equal(gx, gh)
    # the tight batch's lists take several LDS chunks of the half-list sweep
    # (3024 entries) and overflow the staged segment of the full-list sweep
    # (6128 entries), which then reads the list from global memory
    if name == "tight":
        rows = rh.cpu().numpy()
        per = [rows[inst.offset[b + 1]] - rows[inst.offset[b]] for b in range(inst.B)]
        assert max(per) > 3 * 3024 and 2 * max(per) > 6128, per


def test_energy_grad_decreasing_rows_give_nan(P):
    inst = synth.C2(2)
    d, xy = to_dev(P, inst)
    row, col = P.build_neighbors(d, xy, 2.3, 0.0, False)
    bad = row.clone()
    bad[5], bad[6] = row[6] + 3, row[5]           # row 5 of instance 0 ends before it starts
    E = torch.empty(2, dtype=torch.float32, device="cuda")
    g = torch.zeros_like(xy)
    P.pecc_energy_grad(d, xy, bad, col, col.numel(), P.LIST_HALF, 1.0, E, g)
    E2, _ = P.energy_grad(d, xy, row, col)
    assert torch.isnan(E[0]) and E[1] == E2[1]


def test_energy_grad_margin_radius(P):
    inst = synth.C2(1)
    d, xy = to_dev(P, inst)
    row, col = P.build_neighbors(d, xy, 2.3, 0.0, False)
    E, g = P.energy_grad(d, xy, row, col, rad=1.05)
    E64, _, _, g64 = oracle.energy_grad(inst.xy.astype(np.float64), inst.R[0], rad=1.05)
    assert abs(E.item() - E64) <= 1e-5 * E64
    assert np.linalg.norm(g.cpu().numpy().reshape(-1, 2) - g64) <= 1e-5 * np.linalg.norm(g64)


def test_energy_grad_deterministic(P):
    inst = synth.C4(8)
    d, xy = to_dev(P, inst)
    for form in (P.LIST_HALF, P.LIST_LOCAL16):
        row, col = P.build_neighbors(d, xy, 2.3, 0.0, form)
        E1, g1 = P.energy_grad(d, xy, row, col, form=form)
        E2, g2 = P.energy_grad(d, xy, row, col, form=form)
        assert torch.equal(E1, E2) and torch.equal(g1, g2)


def test_energy_grad_bad_rows_give_nan(P):
    inst = synth.C1()
    d, xy = to_dev(P, inst)
    row, col = P.build_neighbors(d, xy, 2.3, 0.0, True)
    E, _ = P.energy_grad(d, xy, row, col[:1].clone() if col.numel() > 1 else col, form=P.LIST_FULL)
    # a col_len shorter than the list makes the instance's range invalid
    E2 = torch.empty(1, dtype=torch.float32, device="cuda")
    P.pecc_energy_grad(d, xy, row, col, max(0, col.numel() - 1), P.LIST_FULL, 1.0, E2, None)
    if col.numel() > 0:
        assert torch.isnan(E2).all()


# ---------------------------------------------------------------------------
# FP64 verify
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(BATCHES))
def test_verify_fp64(P, name):
    inst = BATCHES[name]()
    d, xy = to_dev(P, inst)
    e, mp, mc, f = [t.cpu().numpy() for t in P.verify(d, xy)]
    for b in range(inst.B):
        v = oracle.verify(inst.instance(b), inst.R[b])
        assert e[b] == pytest.approx(v["E"], rel=1e-12, abs=1e-300)
        assert mp[b] == v["max_pair_overlap"]
        assert mc[b] == pytest.approx(v["max_cont_overlap"], rel=1e-15, abs=0)
        assert bool(f[b]) == v["feasible"]


def test_verify_closed_forms(P):
    import math
    r3 = 2 / math.sqrt(3)
    tri = np.array([[r3 * math.cos(a), r3 * math.sin(a)]
                    for a in (math.pi / 2, math.pi / 2 + 2 * math.pi / 3, math.pi / 2 + 4 * math.pi / 3)])
    hexa = np.array([[0, 0]] + [[2 * math.cos(k * math.pi / 3), 2 * math.sin(k * math.pi / 3)]
                                for k in range(6)])
    inst = synth.pack([np.array([[-1.0, 0], [1.0, 0]]), tri, hexa, np.array([[-1.0, 0], [1.0, 0]])],
                      [2.0, 1 + 2 / math.sqrt(3) + 1e-6, 3.0 + 1e-6, 1.999])
    d, xy = to_dev(P, inst)
    e, mp, mc, f = [t.cpu().numpy() for t in P.verify(d, xy)]
    for b in range(4):
        v = oracle.verify(inst.instance(b), inst.R[b])
        assert bool(f[b]) == v["feasible"]
        assert e[b] == pytest.approx(v["E"], rel=1e-12, abs=1e-300)
    assert f[0] == 1 and f[3] == 0


def _tight_expected(xy, R):
    """Smallest FP32 container of FP32 positions by the oracle: rho_max =
    max_i fl(|c_i| + 1) (the oracle's containment overlap at radius 0),
    rounded up to FP32; taken when the unit circles fit there (oracle FP64
    check) and it is below R."""
    if len(xy) == 0:
        return np.float32(R), oracle.verify(xy, R)["feasible"]
    rho = oracle.verify(xy, 0.0)["max_cont_overlap"]
    rt = np.float32(rho)
    if float(rt) < rho:
        rt = np.nextafter(rt, np.float32(np.inf))
    assert float(rt) >= rho and float(np.nextafter(rt, np.float32(0))) < rho
    if float(rt) < R and oracle.verify(xy, float(rt))["feasible"]:
        return rt, True
    return np.float32(R), oracle.verify(xy, R)["feasible"]


def test_verify_tighten_gives_smallest_fp32_container(P):
    import math
    s = 1 + 1e-6
    hexa = np.array([[0, 0]] + [[2 * s * math.cos(k * math.pi / 3), 2 * s * math.sin(k * math.pi / 3)]
                                for k in range(6)])
    g = np.array([[2.5 * i - 5.0, 2.5 * j - 5.0] for i in range(5) for j in range(5)])
    rng = synth.rng_for(11)
    g = g + rng.uniform(-0.2, 0.2, size=g.shape)               # pairwise >= 2.1 apart
    pair_over = np.array([[-0.9, 0.0], [0.9, 0.0]])            # overlapping
    bad = np.array([[0.0, 0.0], [np.inf, 0.0]])
    layouts = [(hexa, 3.01), (hexa, 2.9), (g, 12.0), (pair_over, 3.0), (np.zeros((0, 2)), 1.5),
               (np.array([[-1.000001, 0.0], [1.000001, 0.0]]), 2.5), (bad, 4.0)]
    inst = synth.pack([xy for xy, _ in layouts], [R for _, R in layouts])
    d, xy = to_dev(P, inst)
    R_out = torch.empty(inst.B, dtype=torch.float32, device="cuda")
    feas = torch.empty(inst.B, dtype=torch.int32, device="cuda")
    P.pecc_verify_tighten(d, xy, 1e-20, R_out, feas)
    Ro, fo = R_out.cpu().numpy(), feas.cpu().numpy()
    for b in range(inst.B - 1):
        rt, ok = _tight_expected(inst.instance(b), float(inst.R[b]))
        assert Ro[b] == rt, (b, Ro[b], rt)
        assert bool(fo[b]) == ok, b
        assert bool(fo[b]) == oracle.verify(inst.instance(b), float(Ro[b]))["feasible"], b
    assert Ro[-1] == np.float32(4.0) and fo[-1] == 0          # a non-finite coordinate
    # tightened: the hexagon at 3.01, the grid, the spaced pair; kept: the rest
    assert Ro[0] < np.float32(3.01) and Ro[2] < 12.0 and Ro[5] < 2.5
    assert Ro[1] == np.float32(2.9) and fo[1] == 0
    assert Ro[3] == np.float32(3.0) and fo[3] == 0
    assert Ro[4] == np.float32(1.5) and fo[4] == 1


# ---------------------------------------------------------------------------
# descent
# ---------------------------------------------------------------------------
def gpu_params(P, **kw):
    base = dict(g_tol=0.0, ftol=0.0)
    base.update(kw)
    return P.DescentParams(**base)


def run_gpu(P, inst, params):
    d, xy = to_dev(P, inst)
    out = P.lbfgs_descend(d, xy, params)
    res = P.results(out)
    return xy.cpu().numpy().reshape(-1, 2), res


def c3_subset():
    full = synth.C3_restarts()
    pick = [0, 17, 101, 255]
    return synth.pack([full.instance(b) for b in pick], full.R[pick])


BATCHES["C3sub"] = c3_subset


def follow_oracle(P, inst, iters, m=10, tau64=0.0, tol_per_iter=2e-5, name=""):
    """The first iterations of the GPU descent against the FP64 oracle's:
    the same number of accepted iterations, positions within tol_per_iter x
    iters (relative to the layout's extent), the same energy to 1e-4."""
    xg, res = run_gpu(P, inst, gpu_params(P, max_iter=iters, tau64=tau64, m=m))
    worst = 0.0
    for b in range(inst.B):
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        n = o1 - o0
        x64, r64, tr = oracle.descend(inst.instance(b).astype(np.float64), inst.R[b],
                                      oracle.DescentParams(max_iter=iters, g_tol=0.0, m=m), trace=True)
        if n == 0:
            continue
        if r64["E"] < 1e-10:
            # the overlap vanished: FP32 reaches E = 0 in its own number of
            # steps; both sides must end (numerically) overlap-free
            assert oracle.energy(xg[o0:o1].astype(np.float64), inst.R[b]) < 1e-10
            continue
        assert res["iters"][b] == r64["iters"], (name, b, res[b], r64)
        scale = max(1.0, float(np.abs(x64).max()))
        err = np.abs(xg[o0:o1] - x64).max() / scale
        worst = max(worst, err)
        assert err < tol_per_iter * max(1, iters), (name, b, err)
        assert res["E32"][b] == pytest.approx(r64["E"], rel=1e-4, abs=1e-6)
    return worst


@pytest.mark.parametrize("name", ["C1", "C2", "mixed", "crowded", "C3sub"])
@pytest.mark.parametrize("iters", [1, 2, 3, 6])
def test_descent_first_iterations_follow_oracle(P, name, iters):
    follow_oracle(P, BATCHES[name](), iters, name=name)


@pytest.mark.parametrize("name", ["C1", "C2", "C3sub"])
@pytest.mark.parametrize("m,iters", [(2, 4), (2, 8), (3, 6), (3, 8), (1, 5)])
def test_descent_history_eviction_follows_oracle(P, name, m, iters):
    """Memory m below the iteration count: the history keeps the newest m
    pairs (Eq. 10-11 over the last m), so the oldest pair leaves the
    two-loop several times within the run."""
    follow_oracle(P, BATCHES[name](), iters, m=m, name=name)


@pytest.mark.parametrize("name", ["C2", "C3sub"])
@pytest.mark.parametrize("iters", [12, 16])
def test_descent_full_history_follows_oracle(P, name, iters):
    """Past m = 10 iterations: every iteration after the tenth evicts the
    oldest pair of a full history."""
    follow_oracle(P, BATCHES[name](), iters, name=name)


def near_feasible_batch():
    # seven circles a little off the hexagonal optimum of n = 7 (R = 3)
    # in a container 1e-3 wider, and the C3 restarts' first two instances
    # after a short FP64 descent (small overlaps, E far below 1)
    rng = synth.rng_for(21)
    hexa = np.array([[0.0, 0.0]] + [[2 * np.cos(k * np.pi / 3), 2 * np.sin(k * np.pi / 3)]
                                    for k in range(6)])
    hexa = hexa * (1.0 - 2e-4) + rng.uniform(-1e-4, 1e-4, hexa.shape)
    xs, Rs = [hexa], [3.0 + 1e-3]
    rs = synth.C3_restarts()
    for b in (0, 1):
        x, _, _ = oracle.descend(rs.instance(b).astype(np.float64), rs.R[b],
                                 oracle.DescentParams(max_iter=200))
        xs.append(x)
        Rs.append(float(rs.R[b]))
    return synth.pack(xs, Rs)


@pytest.mark.parametrize("iters", [1, 3, 6])
def test_descent_fp64_regime_follows_oracle(P, iters):
    """With tau64 above every start energy the GPU tests sufficient decrease
    on FP64 energies from the first iteration (its FP32 directions, the
    oracle's FP64 decisions): the trajectories agree like the FP32 ones."""
    inst = near_feasible_batch()
    E0 = [oracle.energy(inst.instance(b).astype(np.float64), inst.R[b]) for b in range(inst.B)]
    assert max(E0) < 1.0 and min(E0) > 1e-12, E0
    follow_oracle(P, inst, iters, tau64=10.0, name="near-feasible")


def test_descent_batch_equals_single(P):
    inst = synth.C3(6)
    params = gpu_params(P, max_iter=300)
    xb, rb = run_gpu(P, inst, params)
    for b in range(inst.B):
        one = synth.pack([inst.instance(b)], [inst.R[b]])
        x1, r1 = run_gpu(P, one, params)
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        assert np.array_equal(xb[o0:o1], x1)
        assert rb[b].tobytes() == r1[0].tobytes()


def test_descent_deterministic(P):
    inst = synth.C4(4)
    params = gpu_params(P, max_iter=500)
    x1, r1 = run_gpu(P, inst, params)
    x2, r2 = run_gpu(P, inst, params)
    assert np.array_equal(x1, x2) and r1.tobytes() == r2.tobytes()


def test_descent_energy_matches_reported(P):
    inst = synth.C4(4)
    xg, res = run_gpu(P, inst, P.DescentParams(max_iter=400))
    for b in range(inst.B):
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        E64 = oracle.energy(xg[o0:o1].astype(np.float64), inst.R[b])
        assert res["E32"][b] == pytest.approx(E64, rel=1e-4)
        assert res["iters"][b] <= 400
        assert res["pair_evals"][b] > 0 and res["rebuilds"][b] >= 1


@pytest.mark.parametrize("case", ["n2", "n3", "n7"])
def test_descent_closed_forms_reach_feasible(P, case):
    import math
    n, Rstar = {"n2": (2, 2.0), "n3": (3, 1 + 2 / math.sqrt(3)), "n7": (7, 3.0)}[case]
    xys = [synth.disk_uniform(n, Rstar + 1e-3, synth.rng_for(s)) for s in range(16)]
    inst = synth.pack(xys, [Rstar + 1e-3] * 16)
    # FP32 positions resolve overlaps only to ~1e-7; a contact margin of 1e-5
    # makes the FP32 descent aim inside the feasible set, FP64 decides
    params = P.DescentParams(max_iter=3000, contact_margin=1e-5)
    xg, res = run_gpu(P, inst, params)
    feas = res["status"] == 1
    assert feas.sum() >= 1
    # every FEASIBLE claim holds under the FP64 oracle
    for b in np.flatnonzero(feas):
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        assert oracle.verify(xg[o0:o1], Rstar + 1e-3)["feasible"]
    inst_lo = synth.pack(xys, [Rstar - 1e-3] * 16)
    _, res_lo = run_gpu(P, inst_lo, params)
    assert (res_lo["status"] != 1).all()


def test_descent_whole_runs_match_oracle_outcomes(P):
    # small instances: both descend to a local minimum from the same start;
    # compare final energies (trajectories may part in late iterations)
    xys = [synth.disk_uniform(20, 5.2, synth.rng_for(s)) for s in range(12)]
    inst = synth.pack(xys, [5.2] * 12)
    xg, res = run_gpu(P, inst, P.DescentParams(max_iter=2000))
    close = 0
    for b in range(12):
        _, r64, _ = oracle.descend(inst.instance(b).astype(np.float64), 5.2,
                                   oracle.DescentParams(max_iter=2000, ftol=1e-7))
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        e_gpu = oracle.energy(xg[o0:o1].astype(np.float64), 5.2)
        if abs(e_gpu - r64["E"]) <= 1e-3 * max(r64["E"], 1e-12) or (e_gpu < 1e-12 and r64["E"] < 1e-12):
            close += 1
    assert close >= 9


def test_descent_edge_instances(P):
    xy_nan = synth.disk_uniform(5, 3.0, synth.rng_for(1)); xy_nan[2, 0] = np.nan
    inst = synth.pack([np.zeros((0, 2)), np.array([[0.3, 0.1]]), xy_nan,
                       np.array([[5.0, 0.0]])], [2.0, 2.0, 3.0, 2.0])
    xg, res = run_gpu(P, inst, P.DescentParams(max_iter=200))
    assert res["status"][0] == 1            # empty: E = 0
    assert res["status"][1] == 1            # one circle well inside
    assert res["status"][2] == 6            # NaN input
    assert res["status"][3] in (1, 2, 3)    # pulled back to the wall
    assert np.hypot(*xg[-1]) <= 1.0 + 1e-6


def test_descent_bad_instance_reported(P):
    # an instance larger than PECC_MAX_N is refused per instance
    big = synth.disk_uniform(1100, 36.0, synth.rng_for(2))
    small = synth.disk_uniform(10, 4.0, synth.rng_for(3))
    inst = synth.pack([small, big], [4.0, 36.0])
    d = P.DeviceInstances.from_host(inst.offset, inst.R)
    d.max_n = 1024   # host bound is a promise the device re-checks
    xy = torch.from_numpy(inst.xy.reshape(-1)).cuda()
    out = P.lbfgs_descend(d, xy, P.DescentParams(max_iter=50))
    res = P.results(out)
    assert res["status"][1] == 7
    assert res["status"][0] in (1, 2, 3, 4, 5)


def test_nonfinite_positions_give_nan_everywhere(P):
    xy = synth.disk_uniform(6, 4.0, synth.rng_for(4)); xy[3, 1] = np.nan
    inst = synth.pack([xy, synth.disk_uniform(5, 4.0, synth.rng_for(5))], [4.0, 4.0])
    d, x = to_dev(P, inst)
    row, col = P.build_neighbors(d, x, 2.3, 0.0, True)
    E, _ = P.energy_grad(d, x, row, col)
    e, mp, mc, f = [t.cpu().numpy() for t in P.verify(d, x)]
    assert np.isnan(E[0].item()) and np.isfinite(E[1].item())
    assert np.isnan(e[0]) and np.isnan(mp[0]) and np.isnan(mc[0]) and f[0] == 0
    assert np.isfinite(e[1])


def test_c3_restart_batch_descends(P):
    inst = synth.C3_restarts()
    xg, res = run_gpu(P, inst, P.DescentParams(max_iter=5000, contact_margin=1e-4))
    assert set(np.unique(res["status"])) <= {1, 2, 3, 4, 5}
    d, xy = to_dev(P, inst)
    xy.copy_(torch.from_numpy(xg.reshape(-1)))
    e64, _, _, f = [t.cpu().numpy() for t in P.verify(d, xy)]
    # every FEASIBLE claim is confirmed by the FP64 oracle on a sample
    for b in np.flatnonzero(res["status"] == 1)[:8]:
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        assert oracle.verify(xg[o0:o1], inst.R[b])["feasible"]
    assert (f == (res["status"] == 1)).all()


def test_descent_stalls_when_no_step_passes(P):
    """c1 = 0.999 asks the first trial to realise almost all of the linear
    decrease, which a curved energy never does at a full step; with no
    halving allowed the line search fails at once: STALLED after 0
    iterations, positions unchanged -- on the GPU as in the oracle."""
    inst = mixed_batch(3, sizes=(20, 333, 1000))
    prm = gpu_params(P, max_iter=50, c1=0.999, max_halvings=0)
    xg, res = run_gpu(P, inst, prm)
    for b in range(inst.B):
        o0, o1 = inst.offset[b], inst.offset[b + 1]
        x64, r64, _ = oracle.descend(inst.instance(b).astype(np.float64), inst.R[b],
                                     oracle.DescentParams(max_iter=50, g_tol=0.0, c1=0.999,
                                                          max_halvings=0))
        assert r64["status"] == "STALLED" and r64["iters"] == 0, r64
        assert P.STATUS[res["status"][b]] == "STALLED" and res["iters"][b] == 0, res[b]
        assert np.array_equal(xg[o0:o1], inst.instance(b))
