"""GPU parity: the HIP path through the C ABI against the CPU oracle.

* direct sum vs the FP64 oracle;
* plan internals (tree cells, point sets, geometry, proxies, interaction
  lists) vs the oracle's tree and traversal: integers bit-exact, geometry to
  rounding;
* eval stages (proxy weights, proxy potentials, near field) and results vs the
  oracle FMM to rounding (same algorithm, other summation order), and vs the
  direct-sum oracle within the approximation gate;
* degenerate cases, distinct sets, adaptive trees, determinism, FP32 form.
"""

import math

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from workloads import cubed_sphere_grid, random_sphere_points, real_y43, real_y41
from oracle import direct as odirect
from oracle import fmm as F
from gates import elem_max

pytestmark = pytest.mark.gpu

DEV = "cuda"


def tdev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _announce(msg):
    print("\n[gpu case] " + msg, flush=True)


# ------------------------------------------------------------------ direct

# The biharmonic kernel is smooth and nearly constant (pi^2/24 at coincidence),
# so against the zero-mean field Y_4,3 its sum cancels to about 1/400 of
# sum |G w|: rounding of the terms is magnified by that factor.
CANCEL = {1: 1.0, 2: 1.0, 3: 1.0, 4: 20.0, 5: 1.0}


@pytest.mark.parametrize("kernel", [1, 2, 3, 4, 5])
def test_direct_matches_oracle(kernel):
    _announce("direct config-1 grid kernel %d" % kernel)
    P, A = cubed_sphere_grid(32)
    w = real_y43(P) * A
    ref = odirect(kernel, P, P, w)
    got = host(cs.direct(tdev(P), tdev(P), tdev(w), kernel=kernel))
    c = CANCEL[kernel]
    print("fp64 rel_l2 %.3e rel_max %.3e" % (rel_l2(got, ref), rel_max(got, ref)), flush=True)
    assert rel_l2(got, ref) < 1e-13 * c and rel_max(got, ref) < 1e-12 * c
    got32 = host(cs.direct(tdev(P), tdev(P), tdev(w), kernel=kernel, fp32=True))
    print("fp32 rel_l2 %.3e" % rel_l2(got32, ref), flush=True)
    assert rel_l2(got32, ref) < 2e-6 * c


def test_direct_distinct_and_ragged():
    _announce("direct distinct sets, ragged sizes")
    S, A = cubed_sphere_grid(8)
    X = random_sphere_points(1001, 5)
    X[:3] = S[[0, 7, 100]]  # exact coincidences are skipped
    w = np.random.default_rng(1).standard_normal(S.shape[0])
    for k in (1, 2, 3, 4, 5):
        ref = odirect(k, X, S, w)
        got = host(cs.direct(tdev(X), tdev(S), tdev(w), kernel=k))
        assert rel_max(got, ref) < 1e-12 * CANCEL[k]
    one = host(cs.direct(tdev(X[:1]), tdev(S[:1]), tdev(w[:1]), kernel=1))
    assert one[0] == 0.0  # the only source coincides with the target


# ------------------------------------------------------------------ plan internals

def _compare_tree(plan, otree, which, gtol=4e-16):
    c = plan.cells(which)
    n = len(otree.cells)
    assert c["level"].shape[0] == n
    lv = np.array([C.level for C in otree.cells])
    fc = np.array([C.face for C in otree.cells])
    ii = np.array([C.i for C in otree.cells])
    jj = np.array([C.j for C in otree.cells])
    cnt = np.array([C.count for C in otree.cells])
    ch0 = np.array([-1 if C.is_leaf else C.children[0].id for C in otree.cells])
    assert np.array_equal(c["level"], lv)
    assert np.array_equal(c["face"], fc)
    assert np.array_equal(c["ci"], ii) and np.array_equal(c["cj"], jj)
    assert np.array_equal(c["count"], cnt)
    assert np.array_equal(c["child0"], ch0)
    perm = plan.permutation(which)
    assert np.array_equal(np.sort(perm), np.arange(perm.shape[0]))
    for k, C in enumerate(otree.cells):
        got = np.sort(perm[c["begin"][k]:c["begin"][k] + c["count"][k]])
        assert np.array_equal(got, np.sort(C.idx))
    cen = np.array([C.center for C in otree.cells])
    rad = np.array([C.radius for C in otree.cells])
    assert np.max(np.abs(c["center"] - cen)) < gtol
    if gtol <= 4e-16:
        assert np.max(np.abs(c["radius"] - rad) / rad) < 1e-14
    else:  # shrunk boxes: radii down to ~1e-7 (one point), compare absolutely
        assert np.max(np.abs(c["radius"] - rad)) < gtol
    prox = plan.proxies(which)
    oprox = np.array([C.proxies for C in otree.cells])
    assert np.max(np.abs(prox - oprox)) < gtol


def _compare_lists(plan, ofmm):
    got = plan.lists()
    for kind in ("PP", "PC", "CP", "CC"):
        t, s = got[kind]
        mine = sorted(zip(t.tolist(), s.tolist()))
        ref = sorted((T.id, S.id) for T, S in ofmm.lists[kind])
        assert mine == ref, kind


CASES = {
    # name: (targets, sources or None, kernel, p, theta, leaf)
    "config1": lambda: (cubed_sphere_grid(32)[0], None, 1, 8, 0.7, 64),
    "grid_E64_leaf128": lambda: (cubed_sphere_grid(64)[0], None, 1, 6, 0.7, 128),
    "ragged_leaf50": lambda: (cubed_sphere_grid(32)[0], None, 3, 5, 0.6, 50),
    "distinct_random": lambda: (random_sphere_points(3000, 41), cubed_sphere_grid(16)[0], 2, 6, 0.6, 40),
    "clustered": lambda: (_clustered(), None, 1, 4, 0.5, 12),
    "tiny_p1_leaf1": lambda: (cubed_sphere_grid(2)[0], None, 1, 1, 0.5, 1),
    "biharmonic_E32": lambda: (cubed_sphere_grid(32)[0], None, 4, 8, 0.7, 64),
    "sal_distinct": lambda: (random_sphere_points(2000, 43), cubed_sphere_grid(16)[0], 5, 6, 0.6, 40),
    # distinct sets sharing points: the source grid points near +x among the
    # targets (their leaves keep the zero test), random points elsewhere
    "distinct_coincident": lambda: (np.concatenate([_grid16_near_x(), random_sphere_points(2000, 44)]),
                                    cubed_sphere_grid(16)[0], 1, 6, 0.6, 40),
    # leaves of more than 64 points: the near field's block path
    "random_leaf100": lambda: (random_sphere_points(6000, 47), None, 1, 6, 0.7, 100),
    # 6,144 leaves of 9 points: the one-wave-per-leaf path and the symmetric
    # PP pairs (both forms); the smaller cases keep the block path
    "grid_E96_leaf16": lambda: (cubed_sphere_grid(96)[0], None, 1, 4, 0.7, 16),
    # the same leaves for Biot-Savart (one direction at a time: no symmetric
    # pairs for its vector kernel)
    "bs_grid_E96_leaf16": lambda: (cubed_sphere_grid(96)[0], None, 2, 4, 0.7, 16),
    # high degrees: P2M with two leaves per block (p >= 12), L2P of three
    # components at p = 12 (LDS near its limit); PC (p = 14) and CC (p = 12) present
    "high_p14": lambda: (cubed_sphere_grid(32)[0], None, 1, 14, 0.5, 64),
    "bs_p12": lambda: (cubed_sphere_grid(32)[0], None, 2, 12, 0.6, 64),
    # the largest degree the library takes (p = 16: 289 proxies a cell)
    "max_p16": lambda: (cubed_sphere_grid(24)[0], None, 3, 16, 0.6, 64),
    # cluster shrinking (paper §3): boxes from the points, per-cell operators;
    # a clustered cloud, distinct sets (both trees shrunk), and the
    # one-wave-per-leaf near field with symmetric pairs
    "clustered_shrink": lambda: (_clustered(), None, 1, 4, 0.5, 12, True),
    "distinct_shrink": lambda: (random_sphere_points(3000, 41), cubed_sphere_grid(16)[0], 2, 6,
                                0.6, 40, True),
    "grid_E96_leaf16_shrink": lambda: (cubed_sphere_grid(96)[0], None, 3, 4, 0.7, 16, True),
}


def _case(name):
    c = CASES[name]()
    return c if len(c) == 7 else c + (False,)


def _grid16_near_x():
    P = cubed_sphere_grid(16)[0]
    return P[P[:, 0] > 0.9]


def _clustered():
    X = random_sphere_points(2500, 9)
    X = X[X[:, 2] > 0.3]
    return np.concatenate([X, random_sphere_points(300, 10)])


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    name = request.param
    T, S, k, p, th, leaf, shrink = _case(name)
    _announce("plan case %s: n_t=%d n_s=%s kernel=%d p=%d theta=%g leaf=%d shrink=%s"
              % (name, T.shape[0], None if S is None else S.shape[0], k, p, th, leaf, shrink))
    ofmm = F.FMM(T, S, k, p, th, leaf, shrink=shrink)
    plan = cs.Plan(tdev(T), None if S is None else tdev(S), kernel=k, p=p, theta=th,
                   leaf_size=leaf, shrink=shrink)
    plan.shrink_case = shrink
    yield name, T, S, k, p, th, leaf, ofmm, plan
    plan.close()


def test_tree_and_geometry(case):
    name, T, S, k, p, th, leaf, ofmm, plan = case
    # shrunk boxes come from the points' angles (atan on two sides: an ulp)
    gtol = 2e-15 if plan.shrink_case else 4e-16
    _compare_tree(plan, ofmm.ttree, 0, gtol)
    if S is not None:
        _compare_tree(plan, ofmm.stree, 1, gtol)


def test_lists(case):
    name, T, S, k, p, th, leaf, ofmm, plan = case
    _compare_lists(plan, ofmm)
    st = plan.stats()
    assert st["n_pp"] == len(ofmm.lists["PP"]) and st["n_cc"] == len(ofmm.lists["CC"])
    # kernel evaluations per list, counted from the oracle's lists
    K = (p + 1) ** 2
    want = {}
    for kind in ("PP", "PC", "CP", "CC"):
        ev = 0
        for Tc, Sc in ofmm.lists[kind]:
            nt = Tc.count if kind in ("PP", "PC") else K
            ns = Sc.count if kind in ("PP", "CP") else K
            ev += nt * ns
            if kind == "PP" and S is None and Tc.id == Sc.id:
                ev -= Tc.count
        want[kind] = ev
    assert (st["evals_pp"], st["evals_pc"], st["evals_cp"], st["evals_cc"]) == \
        (want["PP"], want["PC"], want["CP"], want["CC"])
    assert st["max_leaf_t"] == max(C.count for C in ofmm.ttree.cells if C.is_leaf)
    # same-set plans: PP entries of distinct leaves split into pairs that hold
    # both ways (evaluated once per pair) and one-way entries
    pp = set((Tc.id, Sc.id) for Tc, Sc in ofmm.lists["PP"])
    p32 = cs.Plan(tdev(T), None if S is None else tdev(S), kernel=k, p=p, theta=th,
                  leaf_size=leaf, fp32=True, shrink=plan.shrink_case)
    s32 = p32.stats()
    p32.close()
    if S is None:
        both = sum(1 for a, b in pp if a != b and (b, a) in pp)
        one = sum(1 for a, b in pp if a != b and (b, a) not in pp)
        assert both % 2 == 0
        assert (st["pp_sym_pairs"], st["pp_one_way"]) == (both // 2, one)  # FP64 form
        # FP32 form: a pair whose entries are close (exact differences) stays
        # two one-way entries; the close rule is symmetric, so pairs split whole
        lost = both // 2 - s32["pp_sym_pairs"]
        assert lost >= 0 and s32["pp_one_way"] == one + 2 * lost
        assert s32["pp_close"] >= 2 * lost
    else:
        assert (st["pp_sym_pairs"], st["pp_one_way"]) == (0, 0)
        assert (s32["pp_sym_pairs"], s32["pp_one_way"]) == (0, 0)
    if name == "distinct_coincident":
        # some target leaves hold a point equal to a source point, others not
        leaves = [C for C in ofmm.ttree.cells if C.is_leaf and C.count > 0]
        src = set(map(tuple, S))
        hit = sum(1 for C in leaves if any(tuple(T[i]) in src for i in C.idx))
        assert 0 < hit < len(leaves)


def test_cases_cover_both_near_field_paths():
    """Many leaves of at most 64 points take the one-wave-per-leaf near field
    (and the symmetric PP pairs), the others the block path: the parity cases
    hold both."""
    got = {}
    for name in ("config1", "random_leaf100", "grid_E96_leaf16"):
        T, S, k, p, th, leaf, _ = _case(name)
        pl = cs.Plan(tdev(T), None if S is None else tdev(S), kernel=k, p=p, theta=th,
                     leaf_size=leaf, fp32=True)
        got[name] = pl.stats()
        pl.close()
    assert got["config1"]["near_wave"] == 0 and got["random_leaf100"]["near_wave"] == 0
    assert got["random_leaf100"]["max_leaf_t"] > 64
    assert got["grid_E96_leaf16"]["near_wave"] == 1 and got["grid_E96_leaf16"]["pp_close"] == 0
    assert got["grid_E96_leaf16"]["pp_sym_pairs"] > 0


def test_stages_and_result(case):
    name, T, S, k, p, th, leaf, ofmm, plan = case
    src = T if S is None else S
    rng = np.random.default_rng(3)
    w = rng.standard_normal(src.shape[0])
    ref, stg = ofmm.evaluate(w, stages=True)
    out, wbar, psi, near = plan.eval_stages(tdev(w))
    out, wbar, psi, near = host(out), host(wbar), host(psi), host(near)
    # proxy weights after the upward pass
    ow = np.array([stg["wbar"][C.id].reshape(-1) for C in ofmm.stree.cells])
    assert rel_max(wbar, ow) < 1e-13
    # proxy potentials after the downward pass at the leaves that hold targets
    # (the library accumulates them per leaf; other cells keep their own sums)
    vd = 3 if k == 2 else 1
    n1 = p + 1
    c = CANCEL[k]
    op = np.zeros((vd, len(ofmm.ttree.cells), n1 * n1))
    for cid, val in stg["psi"].items():
        op[:, cid, :] = np.asarray(val).reshape(n1 * n1, vd).T
    full = np.array([C.count > 0 and C.is_leaf for C in ofmm.ttree.cells])
    if np.any(op[:, full] != 0):
        assert rel_max(psi[:, full], op[:, full]) < 1e-12 * c
    # near field (PP + PC)
    onear = stg["near"]
    assert rel_max(near, onear) < 1e-12 * c
    # the whole result, vs the oracle FMM and vs the direct sum
    assert rel_max(out, ref) < 1e-12 * c
    d = odirect(k, T, src, w)
    assert rel_l2(out, d) < 1e-3


def test_fp32_form_close_to_fp64(case):
    name, T, S, k, p, th, leaf, ofmm, plan = case
    src = T if S is None else S
    w = np.random.default_rng(4).standard_normal(src.shape[0])
    plan32 = cs.Plan(tdev(T), None if S is None else tdev(S), kernel=k, p=p, theta=th,
                     leaf_size=leaf, fp32=True, shrink=plan.shrink_case)
    a = host(plan.eval(tdev(w)))
    b = host(plan32.eval(tdev(w)))
    plan32.close()
    print("fp32 vs fp64 rel_l2 %.3e elem_max %.3e" % (rel_l2(b, a), elem_max(b, a)), flush=True)
    assert rel_l2(b, a) < 5e-6 * CANCEL[k]
    assert elem_max(b, a) < 5e-5 * CANCEL[k]


def test_fp32_near_field_matches_oracle(case):
    """FP32 form near field (PP + PC) against the oracle's near field: same-set
    plans with leaves of at most 64 points evaluate each symmetric PP pair once
    for both directions; the others one direction at a time."""
    name, T, S, k, p, th, leaf, ofmm, plan = case
    src = T if S is None else S
    w = np.random.default_rng(5).standard_normal(src.shape[0])
    ref, stg = ofmm.evaluate(w, stages=True)
    plan32 = cs.Plan(tdev(T), None if S is None else tdev(S), kernel=k, p=p, theta=th,
                     leaf_size=leaf, fp32=True, shrink=plan.shrink_case)
    out, wbar, psi, near = plan32.eval_stages(tdev(w))
    near = host(near)
    again = host(plan32.eval(tdev(w)))
    assert np.array_equal(again, host(plan32.eval(tdev(w))))  # deterministic
    plan32.close()
    err = rel_l2(near, stg["near"])
    em = elem_max(near, stg["near"])
    print("fp32 near field rel_l2 %.3e elem_max %.3e" % (err, em), flush=True)
    assert err < 2e-6 * CANCEL[k]
    assert em < 5e-5 * CANCEL[k]


def _straddling_points(delta):
    """Four points at +-delta across the central line of the face around +x
    (xi = 0 or eta = 0, whichever axis carries it), which is a cell edge at
    every level: two pairs of points in neighbouring leaves, 2 delta apart."""
    Q = np.array([[1.0, delta, 0.3], [1.0, -delta, 0.3], [1.0, 0.3, delta], [1.0, 0.3, -delta]])
    return Q / np.linalg.norm(Q, axis=1, keepdims=True)


def test_fp32_close_pairs_across_leaf_edges():
    """Points 2e-5 apart in neighbouring leaves: the expanded squared distance
    |t|^2 + |s|^2 - 2 t.s of the FP32 form cannot resolve them (its rounding is
    ~1e-9 against a squared distance of 4e-10), so the plan detects the small
    edge gap and those entries take exact differences; the pair's targets then
    match the oracle to FP32 coordinate resolution."""
    _announce("grid E=32 + 4 points straddling a leaf edge, 1/r, FP32 near field")
    G = cubed_sphere_grid(32)[0]
    P = np.concatenate([G, _straddling_points(1e-5)])
    w = np.random.default_rng(6).standard_normal(P.shape[0])
    o = F.FMM(P, None, 3, 6, 0.7, 64)
    ref, stg = o.evaluate(w, stages=True)
    pl = cs.Plan(tdev(P), None, kernel=3, p=6, theta=0.7, leaf_size=64, fp32=True)
    st = pl.stats()
    out, wbar, psi, near = pl.eval_stages(tdev(w))
    near, out = host(near)[:, 0], host(out)
    pl.close()
    assert st["pp_close"] > 0
    assert np.all(np.isfinite(out))
    on = stg["near"][:, 0]
    q = np.arange(G.shape[0], P.shape[0])
    err = np.abs(near[q] - on[q]) / np.abs(on[q])
    print("straddling targets rel err", err, flush=True)
    assert np.all(err < 1e-2)
    n = G.shape[0]
    assert rel_l2(near[:n], on[:n]) < 2e-6
    # the grid alone keeps its points 1/8 of a half leaf width from the edges
    pg = cs.Plan(tdev(G), None, kernel=3, p=6, theta=0.7, leaf_size=64, fp32=True)
    assert pg.stats()["pp_close"] == 0
    pg.close()


@pytest.mark.parametrize("kernel", [1, 3])
def test_fp32_random_points(kernel):
    """Uniform random points: close pairs in the same or neighbouring leaves
    limit the FP32 form to its coordinate resolution (a pair at distance d
    carries a relative error of about ulp(leaf size) / d in its kernel value),
    here ~1e-5 of the 1/r near field; the result stays finite."""
    _announce("random points n=20000 leaf 40 kernel %d, FP32 near field" % kernel)
    P = random_sphere_points(20000, 4)
    w = np.random.default_rng(4).standard_normal(P.shape[0])
    o = F.FMM(P, None, kernel, 6, 0.7, 40)
    ref, stg = o.evaluate(w, stages=True)
    pl = cs.Plan(tdev(P), None, kernel=kernel, p=6, theta=0.7, leaf_size=40, fp32=True)
    st = pl.stats()
    out, wbar, psi, near = pl.eval_stages(tdev(w))
    near, out = host(near), host(out)
    pl.close()
    assert st["pp_close"] > 0
    on = stg["near"]
    print("rel_l2 %.3e max %.3e" % (rel_l2(near, on), rel_max(near, on)), flush=True)
    assert np.all(np.isfinite(out))
    assert rel_l2(near, on) < 3e-5 and rel_max(near, on) < 1e-4


@pytest.mark.parametrize("kernel", [1, 2, 3])
def test_fp32_random_points_wave_path(kernel):
    """Many small leaves of uniform random points: the one-wave-per-leaf near
    field, its close entries in exact differences and one way, the others as
    symmetric pairs where they hold both ways, against the oracle's near field
    at the bound of the block-path case above; repeatable bitwise."""
    _announce("random points n=50000 leaf 32 kernel %d, FP32 wave path" % kernel)
    P = random_sphere_points(50000, 4)
    w = np.random.default_rng(4).standard_normal(P.shape[0])
    o = F.FMM(P, None, kernel, 6, 0.7, 32)
    ref, stg = o.evaluate(w, stages=True)
    pl = cs.Plan(tdev(P), None, kernel=kernel, p=6, theta=0.7, leaf_size=32, fp32=True)
    st = pl.stats()
    out, wbar, psi, near = pl.eval_stages(tdev(w))
    near2 = host(pl.eval_stages(tdev(w))[3])
    near, out = host(near), host(out)
    pl.close()
    assert st["pp_close"] > 0 and st["near_wave"] == 1
    on = stg["near"]
    print("rel_l2 %.3e max %.3e" % (rel_l2(near, on), rel_max(near, on)), flush=True)
    assert np.all(np.isfinite(out))
    assert rel_l2(near, on) < 3e-5 and rel_max(near, on) < 1e-4
    assert np.array_equal(near, near2)


def test_deterministic(case):
    name, T, S, k, p, th, leaf, ofmm, plan = case
    src = T if S is None else S
    w = tdev(np.random.default_rng(5).standard_normal(src.shape[0]))
    a = host(plan.eval(w))
    b = host(plan.eval(w))
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ whole method

@pytest.mark.parametrize("kernel", [1, 2, 3, 4, 5])
def test_degenerate_all_pp_equals_direct(kernel):
    _announce("degenerate theta->0 and leaf>=N, kernel %d" % kernel)
    P, A = cubed_sphere_grid(8)
    w = real_y41(P) * A
    ref = host(cs.direct(tdev(P), tdev(P), tdev(w), kernel=kernel))
    for th, leaf in ((1e-9, 16), (0.7, P.shape[0])):
        pl = cs.Plan(tdev(P), None, kernel=kernel, p=4, theta=th, leaf_size=leaf)
        st = pl.stats()
        assert st["n_pc"] == st["n_cp"] == st["n_cc"] == 0
        got = host(pl.eval(tdev(w)))
        pl.close()
        assert rel_l2(got, ref) < 1e-14 * CANCEL[kernel]


def test_config1_gate_and_eigenrelation():
    _announce("config 1 end to end")
    P, A = cubed_sphere_grid(32)
    f = real_y43(P)
    w = f * A
    pl = cs.Plan(tdev(P), None, kernel=1, p=8, theta=0.7, leaf_size=64)
    fs = host(pl.eval(tdev(w)))
    pl.close()
    ds = odirect(1, P, P, w)
    assert rel_l2(fs, ds) < 1e-6
    e = math.sqrt(np.sum((fs - f / 20) ** 2 * A) / np.sum((f / 20) ** 2 * A))
    assert e < 4e-2


def test_single_point_and_empty_faces():
    _announce("single point, one populated face")
    X = np.array([[0.0, 0.0, 1.0]])
    pl = cs.Plan(tdev(X), None, kernel=1, p=3, theta=0.5, leaf_size=4)
    assert host(pl.eval(tdev(np.array([2.0]))))[0] == 0.0
    pl.close()
    Y = random_sphere_points(500, 2)
    Y = Y[Y[:, 2] > 0.9]  # all on the +z face
    w = np.random.default_rng(2).standard_normal(Y.shape[0])
    pl = cs.Plan(tdev(Y), None, kernel=3, p=5, theta=0.5, leaf_size=4)
    got = host(pl.eval(tdev(w)))
    pl.close()
    assert rel_l2(got, odirect(3, Y, Y, w)) < 1e-4


def test_plan_rejects_points_off_the_sphere():
    _announce("off-sphere rejection")
    X = random_sphere_points(100, 3)
    X[5] *= 1.001
    with pytest.raises(cs.CsfmmError) as ei:
        cs.Plan(tdev(X), None, kernel=1, p=4, theta=0.5, leaf_size=8)
    assert ei.value.status == -2


@pytest.mark.parametrize("name", ["config1", "high_p14", "bs_p12", "max_p16", "distinct_random"])
def test_m2m_row_kernel_matches_the_oracle(name, monkeypatch):
    """The row-blocked M2M (levels of 8,192 parents or more at full size) forced
    onto every level of small trees: the proxy weights and the result match the
    oracle's as tightly as the default per-tile kernel's do, and the two
    kernels agree to rounding (the same product, summed in another order)."""
    T, S, k, p, th, leaf, shrink = _case(name)
    _announce("row-blocked M2M on case %s (p=%d)" % (name, p))
    ofmm = F.FMM(T, S, k, p, th, leaf)
    src = T if S is None else S
    w = np.random.default_rng(8).standard_normal(src.shape[0])
    ref, stg = ofmm.evaluate(w, stages=True)
    plan = cs.Plan(tdev(T), None if S is None else tdev(S), kernel=k, p=p, theta=th, leaf_size=leaf)
    out0, wbar0 = (host(x) for x in plan.eval_stages(tdev(w))[:2])
    monkeypatch.setenv("CSFMM_M2M_ROWS_MIN", "0")
    out1, wbar1 = (host(x) for x in plan.eval_stages(tdev(w))[:2])
    plan.close()
    scale = np.max(np.abs(wbar0))
    print("wbar rows vs tiles %.3e, out rows vs tiles %.3e" % (
        np.max(np.abs(wbar1 - wbar0)) / scale, rel_max(out1, out0)), flush=True)
    assert np.max(np.abs(wbar1 - wbar0)) <= 1e-13 * scale
    ow = np.array([stg["wbar"][C.id].reshape(-1) for C in ofmm.stree.cells])
    assert rel_max(wbar1, ow) < 1e-13
    assert rel_max(out1, out0) < 1e-12
    assert rel_l2(out1, ref) < 1e-12 * CANCEL[k]
