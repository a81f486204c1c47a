"""Pins of the oracle's version of the paper's guide (Sec. 5.5, 5.6): the vMF
lobe against its closed-form normalisation and moments, the tree against a
brute-force restatement of its split and overlap rule, the leaf
distributions against direct weighted sums, the defensive sampling law
against its mixture probabilities, and the P(n)-factored reciprocal
probability against the number of admissible chains."""
import math
import types

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import scenes as S
from tests.test_oracle_pins import strip_solutions


def ep64(xD, xL, n=1, types_=0, nD=(0, 0, 1), obj1=-1):
    xD = np.atleast_2d(np.asarray(xD, np.float64))
    xL = np.atleast_2d(np.asarray(xL, np.float64))
    N = max(len(xD), len(xL))
    xD = np.ascontiguousarray(np.broadcast_to(xD, (N, 3)).T)
    xL = np.ascontiguousarray(np.broadcast_to(xL, (N, 3)).T)
    nd = np.ascontiguousarray(np.broadcast_to(np.asarray(nD, np.float64), (N, 3)).T)
    return types.SimpleNamespace(xD=xD, nD=nd, xL=xL, length=np.full(N, n, np.uint8),
                                 types=np.full(N, types_, np.uint8), obj1=np.full(N, obj1, np.int32), n=N)


def ks(x, cdf):
    x = np.sort(x)
    n = len(x)
    F = cdf(x)
    return max(np.max(np.arange(1, n + 1) / n - F), np.max(F - np.arange(n) / n))


# ---------------------------------------------------------------------------
# the vMF lobe (Eq. vMF)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kappa", [0.5, 8.0, 200.0, 1e5])
def test_vmf_density_integrates_to_one(oracle_lib, kappa):
    # integral over the sphere = 2 pi int_{-1}^{1} f(c) dc, with the grid
    # refined geometrically towards c = 1 where a sharp lobe lives
    mu = np.array([0.3, -0.2, 0.9])
    mu /= np.linalg.norm(mu)
    b1 = np.cross(mu, [1.0, 0, 0])
    b1 /= np.linalg.norm(b1)
    t = np.concatenate([[0.0], np.geomspace(1e-12, 2.0, 20000)])   # t = 1 - c
    f = np.array([O.vmf_pdf(mu, kappa, (1 - ti) * mu + math.sqrt(max(0.0, 1 - (1 - ti) ** 2)) * b1) for ti in t])
    integral = 2 * math.pi * np.trapezoid(f, t)
    assert abs(integral - 1.0) < 1e-5


@pytest.mark.parametrize("kappa", [0.5, 8.0, 200.0, 1e5])
def test_vmf_sampling_follows_the_lobe(oracle_lib, kappa):
    mu = np.array([-0.6, 0.0, 0.8])
    N = 40000
    g = np.random.default_rng(3)
    w = O.vmf_sample(mu, kappa, g.random((N, 2)))
    assert np.allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-12)
    c = w @ mu
    # mean cosine coth(kappa) - 1/kappa; cosine CDF (e^{k c} - e^{-k}) / (e^k - e^{-k})
    mean = 1.0 / math.tanh(kappa) - 1.0 / kappa
    sd = math.sqrt(max(np.var(c), 1e-30))
    assert abs(c.mean() - mean) < 5 * sd / math.sqrt(N)
    def cdf(x):
        return (np.exp(kappa * (x - 1)) - math.exp(-2 * kappa)) / (1 - math.exp(-2 * kappa))
    assert ks(c, cdf) < 1.95 / math.sqrt(N)
    # azimuth uniform about mu
    b1 = np.cross(mu, [0.0, 1.0, 0.0])
    b1 /= np.linalg.norm(b1)
    b2 = np.cross(mu, b1)
    phi = (np.arctan2(w @ b2, w @ b1) + np.pi) / (2 * np.pi)
    assert ks(phi, lambda x: x) < 1.95 / math.sqrt(N)


# ---------------------------------------------------------------------------
# the tree (Sec. 5.6)
# ---------------------------------------------------------------------------

def random_records(N, seed=0, lo=0.0, hi=4.0):
    g = np.random.default_rng(seed)
    xD = g.uniform(lo, hi, (N, 3))
    xL = np.column_stack([g.uniform(lo, hi, N), g.uniform(lo, hi, N), g.normal(2.0, 0.3, N).clip(lo, hi)])
    w = g.normal(size=(N, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    n = g.integers(1, 4, N)
    t = g.integers(0, 2, N) * (n > 1)
    wt = g.uniform(0.1, 2.0, N)
    wt[::97] = 0.0            # zero weight: not a sample
    return O.sample_records(xD, xL, w, wt, n, t)


def brute_node_sets(rec, lo, hi, eps, thr, max_depth):
    """The tree restated recursively: node -> (box, member ids, own ids)."""
    P = rec[:, :6].astype(np.float64)
    valid = (rec[:, 9] > 0) & np.all((P >= lo) & (P <= hi), 1)
    out = []

    def rec_node(blo, bhi, members, own, depth):
        k = len(out)
        out.append((blo.copy(), bhi.copy(), members, own, depth, None))
        if not (len(members) > thr) or depth >= max_depth:
            return
        ax = int(np.argmax(bhi - blo))
        mid = 0.5 * (blo[ax] + bhi[ax])
        dil = eps * (mid - blo[ax])
        v = P[members, ax]
        lm = members[(v >= blo[ax] - dil) & (v < mid + dil)]
        rm = members[(v >= mid - dil) & (v < bhi[ax] + dil)]
        lown = np.intersect1d(own, members[v < mid])
        rown = np.intersect1d(own, members[v >= mid])
        out[k] = out[k][:5] + ((ax, mid),)
        llo, lhi, rlo, rhi = blo.copy(), bhi.copy(), blo.copy(), bhi.copy()
        lhi[ax] = mid
        rlo[ax] = mid
        return (llo, lhi, lm, lown), (rlo, rhi, rm, rown)

    # breadth first, children left then right
    queue = [(np.array(lo, float), np.array(hi, float), np.nonzero(valid)[0], np.nonzero(valid)[0], 0)]
    while queue:
        blo, bhi, m, o, d = queue.pop(0)
        kids = rec_node(blo, bhi, m, o, d)
        if kids:
            for c in kids:
                queue.append((*c, d + 1))
    return out, valid.sum()


@pytest.mark.parametrize("eps", [0.0, 0.1])
def test_tree_matches_brute_force_restatement(oracle_lib, eps):
    N = 6000
    rec = random_records(N)
    lo, hi = np.zeros(6), np.full(6, 4.0)
    t = O.STree(rec, lo, hi, eps=eps)
    d = t.nodes()
    want, n_valid = brute_node_sets(rec, lo, hi, eps, math.sqrt((rec[:, 9] > 0).sum()), 20)
    assert len(want) == len(d["axis"])
    own_total = 0
    for k, (blo, bhi, members, own, depth, split) in enumerate(want):
        ids, own_flags = t.node_entries(k, d["n_entries"][k])
        assert np.array_equal(ids, members), k
        assert set(ids[own_flags == 1]) == set(own), k
        assert np.allclose(d["lo"][k], blo) and np.allclose(d["hi"][k], bhi)
        if split is None:
            assert d["axis"][k] == -1
            assert d["n_entries"][k] <= math.sqrt(n_valid) or d["depth"][k] >= 20
            own_total += d["n_own"][k]
        else:
            assert (d["axis"][k], d["mid"][k]) == split
    assert own_total == n_valid       # every sample is own in exactly one leaf
    if eps == 0.0:
        leaves = d["axis"] < 0
        assert np.array_equal(d["n_entries"][leaves], d["n_own"][leaves])


def test_leaf_histograms_and_lobe_footprints(oracle_lib):
    N = 4000
    rec = random_records(N, seed=1)
    lo, hi = np.zeros(6), np.full(6, 4.0)
    t = O.STree(rec, lo, hi, eps=0.1, sigma_min=1e-3, sigma_lone=0.1)
    d = t.nodes()
    L = t.lobes()
    for k in np.nonzero(d["axis"] < 0)[0][:40]:
        ids, _ = t.node_entries(k, d["n_entries"][k])
        r = rec[ids].astype(np.float64)
        assert abs(d["W"][k] - r[:, 9].sum()) < 1e-9 * max(1, r[:, 9].sum())
        for n in range(1, 9):
            assert abs(d["Wn"][k, n - 1] - r[r[:, 10] == n, 9].sum()) < 1e-9
        # lobes: groups by (n, tau), samples in id order, kappa = 1 / sigma^2
        q = d["lobe0"][k]
        keys = sorted(set(zip(r[:, 10].astype(int), r[:, 11].astype(int))))
        for (n, ty) in keys:
            sel = ids[(r[:, 10] == n) & (r[:, 11] == ty)]
            dirs = rec[sel, 6:9].astype(np.float64)
            dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
            for a in range(len(sel)):
                assert L["n"][q] == n and L["type"][q] == ty
                assert np.allclose(L["mu"][q], dirs[a], atol=1e-12)
                assert L["w"][q] == pytest.approx(float(rec[sel[a], 9]))
                if len(sel) == 1:
                    sig = 0.1
                else:
                    cosang = np.clip(np.delete(dirs, a, 0) @ dirs[a], -1, 1)
                    sig = max(float(np.arccos(cosang.max())), 1e-3)
                assert L["kappa"][q] == pytest.approx(1.0 / sig ** 2, rel=1e-6)
                q += 1


# ---------------------------------------------------------------------------
# defensive sampling of n, tau and w_D (Sec. 5.5)
# ---------------------------------------------------------------------------

def single_leaf_tree(records, **kw):
    return O.STree(records, [-10.0] * 6, [10.0] * 6, thr_scale=1e9, **kw)


def test_sampled_length_and_type_follow_the_defensive_mixture(oracle_lib):
    # one leaf: lengths 1 and 2 with weights 1 and 3; at n = 1 types R / T
    # with weights 1 / 3.  P_0(n) puts 0.8 on n = 1, 0.2 on n = 3.  A dielectric
    # plane: p_0 decides the type by a fair coin at the plane.
    sc = S.plane_scene(W.MAT_DIELECTRIC, ior=1.5, half=4.0)
    osc = O.Scene(sc)
    xD, xL = np.array([0.2, 0.1, -1.0]), np.array([-0.3, 0.2, 2.0])
    wdir = np.array([0.0, 0.0, 1.0])
    rec = O.sample_records(np.tile(xD, (4, 1)), np.tile(xL, (4, 1)), np.tile(wdir, (4, 1)),
                           [0.25, 0.75, 1.5, 1.5], [1, 1, 2, 2], [0, 1, 3, 3])
    p0n = np.array([0.8, 0.0, 0.2, 0, 0, 0, 0, 0])
    alpha = 0.5
    t = single_leaf_tree(rec, p0n=p0n, alpha=alpha, p_transmit=0.5)
    N = 40000
    ep = ep64(xD, np.tile(xL, (N, 1)), obj1=0)
    n, ty, pn, prim, pos, st = O.stree_sample_seeds(osc, t, ep)
    Pe = np.array([1.0, 3.0, 0, 0, 0, 0, 0, 0]) / 4.0
    Pn = alpha * p0n + (1 - alpha) * Pe
    cnt = np.bincount(n, minlength=9)[1:]
    m = Pn > 0
    chi2 = float((((cnt[m] - N * Pn[m]) ** 2) / (N * Pn[m])).sum())
    assert chi2 < 16.3, (cnt, N * Pn)          # 0.1% point of chi-square(2)
    assert np.allclose(pn, Pn[n - 1], rtol=1e-12)
    # type at n = 1: p_0 (coin, 1/2) or P_e(T | 1) = 3/4
    one = n == 1
    pT = alpha * 0.5 + (1 - alpha) * 0.75
    k = int((ty[one] == 1).sum())
    assert abs(k / one.sum() - pT) < 4 * math.sqrt(pT * (1 - pT) / one.sum())
    # n = 3 (prior only) cannot be deduced on a single plane
    assert np.all(st[n == 3] == O.SEED_INVALID) and np.all(st[n == 1] == 0)


def test_sampled_directions_follow_the_lobes(oracle_lib):
    # alpha = 0: every (w_D, tau) comes from the learned mixture.  Two groups
    # at n = 1 (R with weight 1 along d1, T with weight 3 along d2), one
    # sample each, so each lobe has the lone-sample footprint sigma_lone:
    # tau follows 1 : 3 and w_D the lobe of its group (vMF cosine law).
    sc = S.plane_scene(W.MAT_DIELECTRIC, ior=1.5, half=50.0, z=1.0, normal_up=False)
    osc = O.Scene(sc)
    xD, xL = np.zeros(3), np.array([0.0, 0.0, 3.0])
    d1 = np.array([0.3, 0.0, 1.0])
    d2 = np.array([-0.3, 0.1, 1.0])
    d1 /= np.linalg.norm(d1)
    d2 /= np.linalg.norm(d2)
    rec = O.sample_records(np.tile(xD, (2, 1)), np.tile(xL, (2, 1)), np.stack([d1, d2]), [1.0, 3.0], [1, 1], [0, 1])
    sig = 0.05
    t = single_leaf_tree(rec, alpha=0.0, sigma_lone=sig)
    kappa = 1.0 / sig ** 2
    N = 30000
    ep = ep64(xD, np.tile(xL, (N, 1)), obj1=0)
    n, ty, pn, prim, pos, st = O.stree_sample_seeds(osc, t, ep)
    assert np.all(st == 0) and np.all(n == 1)
    k = int((ty == 1).sum())
    assert abs(k / N - 0.75) < 4 * math.sqrt(0.75 * 0.25 / N)
    w = pos[:, 0, :].T - xD
    w /= np.linalg.norm(w, axis=1, keepdims=True)

    def cdf(x):
        return (np.exp(kappa * (x - 1)) - math.exp(-2 * kappa)) / (1 - math.exp(-2 * kappa))
    for tau, d in ((0, d1), (1, d2)):
        c = w[ty == tau] @ d
        assert ks(c, cdf) < 1.95 / math.sqrt(len(c))


# ---------------------------------------------------------------------------
# P(n) factored out of the reciprocal probability (Sec. 5.8)
# ---------------------------------------------------------------------------

def test_inverse_probability_with_sampled_length_counts_solutions(oracle_lib):
    # lengths drawn 30% n = 1 / 70% n = 2 on the mirror strip: restricted to
    # the sampled n = 1 configurations, E[1{n = 1, converged} K / P(n)] is
    # the number of one-bounce solutions, enumerated in closed form; an
    # estimate that forgot the P(n) factor would give 0.3 of it
    sc = S.strip_scene(W.MAT_MIRROR)
    osc = O.Scene(sc)
    xD = np.array([-1.3, 0.0, 0.9])
    xL = np.array([1.1, 0.0, 1.4])
    n_sol = len(strip_solutions(sc, xD, xL))
    empty = O.sample_records(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0),
                             np.zeros(0))
    t = single_leaf_tree(empty, p0n=np.array([0.3, 0.7, 0, 0, 0, 0, 0, 0]), alpha=0.5)
    M = 8000
    ep = ep64(xD, np.tile(xL, (M, 1)), obj1=0)
    n, ty, pn, prim, pos, st = O.stree_sample_seeds(osc, t, ep)
    assert np.allclose(pn[n == 1], 0.3) and np.allclose(pn[n == 2], 0.7)
    wep = types.SimpleNamespace(**{**vars(ep), "length": n, "types": ty})
    r = O.walk(osc, wep, prim, pos.astype(np.float32), st)
    trials, ip, trunc, pn2 = O.stree_inv_prob(osc, t, wep, n, ty, r["prim"], r["pos"], r["status"], max_trials=100000)
    conv = r["status"] == O.CONVERGED
    assert not trunc[conv].any()
    assert np.allclose(ip[conv], trials[conv] / pn2[conv])
    est = np.where(conv & (n == 1), ip, 0.0)
    se = est.std() / math.sqrt(M)
    assert abs(est.mean() - n_sol) < 4 * se, (est.mean(), n_sol, se)
