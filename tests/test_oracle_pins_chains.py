"""Pins of the oracle's seed deduction, mixture pick, direction cone, stall
path and refractive solution sets against what geometry fixes.

Each test compares the oracle with an independent statement of the same
fact: Snell's invariant across parallel interfaces and the unfolded mirror
path (Eq. deduction), the law of the component pick of a Gaussian mixture
(Sec. 5.5), the directions of every admissible chain found from the paper's
hemisphere initialization (Sec. 6.4), the closed-form mirror point reached
through the FP64 acceptance of a stalled walk, and the meridian-plane root
count of a two-refraction path through a ball lens (the finite solution set
of Sec. 4).
"""
import math
import types

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import scenes as S


def ep64(xD, xL, n=1, types_=0, nD=(0, 0, 1), obj1=-1):
    xD = np.atleast_2d(np.asarray(xD, np.float64))
    xL = np.atleast_2d(np.asarray(xL, np.float64))
    N = max(len(xD), len(xL))
    xD = np.ascontiguousarray(np.broadcast_to(xD, (N, 3)).T)
    xL = np.ascontiguousarray(np.broadcast_to(xL, (N, 3)).T)
    nd = np.ascontiguousarray(np.broadcast_to(np.asarray(nD, np.float64), (N, 3)).T)
    n = np.broadcast_to(np.asarray(n), (N,))
    t = np.broadcast_to(np.asarray(types_), (N,))
    return types.SimpleNamespace(xD=xD, nD=nd, xL=xL, length=np.ascontiguousarray(n, np.uint8),
                                 types=np.ascontiguousarray(t, np.uint8), obj1=np.full(N, obj1, np.int32), n=N)


# ---------------------------------------------------------------------------
# Eq. deduction for n >= 2: flat parallel interfaces and parallel mirrors
# ---------------------------------------------------------------------------

def stack_index_at(z):
    """Index of refraction at height z in the slab stack (glass inside slab k:
    -0.5 k - 0.25 < z < -0.5 k, air elsewhere)."""
    for k in range(W.SLAB_COUNT):
        top = -W.SLAB_GAP * k
        if top - W.SLAB_THICK < z < top:
            return 1.5
    return 1.0


def snell_invariant_chain(xD, wD, n):
    """Vertices of the ray from xD along wD (pointing up) through interfaces
    n, n-1, ..., 1 of a flat slab stack, from Snell's invariant: the
    tangential part of eta w is the same in every layer.  Returns None when
    the ray is totally reflected ("tir") or leaves the stack's [0, 4]^2
    footprint ("out") before reaching interface 1."""
    eta0 = stack_index_at(xD[2])
    th = eta0 * wD[:2]                     # conserved tangential component of eta w
    x = np.array(xD, np.float64)
    pts = []
    for i in range(n):
        zk = W.interface_z(n - i)
        eta = stack_index_at(0.5 * (x[2] + zk))
        s2 = float(th @ th) / eta ** 2
        if s2 >= 1.0:
            return "tir"
        w = np.array([th[0] / eta, th[1] / eta, math.sqrt(1.0 - s2)])
        x = x + w * ((zk - x[2]) / w[2])
        if not (0.0 < x[0] < 4.0 and 0.0 < x[1] < 4.0):
            return "out"
        pts.append(x.copy())
    return np.array(pts)


@pytest.mark.parametrize("cone_deg", [40.0, 65.0])
def test_deduction_through_flat_slabs_follows_snell_invariant(oracle_lib, cone_deg):
    sc = W.slab_stack_scene(amp=0.0)
    osc = O.Scene(sc)
    g = np.random.default_rng(11)
    N = 4000
    n = g.integers(2, 9, N)
    zs = np.array([W.interface_z(k) - 0.5 * W.SLAB_THICK for k in range(1, 9)])
    xD = np.stack([g.uniform(1.0, 3.0, N), g.uniform(1.0, 3.0, N), zs[n - 1]], 1)
    ep = ep64(xD, [2.0, 2.0, 3.0], n=n, types_=(1 << n) - 1, obj1=W.P0_DIRECTION)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(cone_deg)))
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    # the sampled direction w_D of every chain, also where the deduction
    # fails: the same draws (same chain counters) with n = 1 stop at the
    # first interface, which every launch direction reaches
    ep1 = ep64(xD, [2.0, 2.0, 3.0], n=1, types_=1, obj1=W.P0_DIRECTION)
    _, pos1, st1 = O.sample_seeds(osc, ep1, prm=prm)
    assert np.all(st1 == 0)
    n_tir = n_ok = 0
    for c in range(N):
        x1 = pos1[:, 0, c]
        wD = (x1 - xD[c]) / np.linalg.norm(x1 - xD[c])
        want = snell_invariant_chain(xD[c], wD, int(n[c]))
        if isinstance(want, str):
            n_tir += want == "tir"
            assert st[c] == O.SEED_INVALID, c
            continue
        n_ok += 1
        assert st[c] == 0, c
        got = pos[:, :n[c], c].T
        assert np.abs(got - want).max() < 1e-12, (c, got, want)
        # objects: interface n - i + 1 (object n - i) holds vertex i
        objs = [osc.src.tri_obj[p] for p in prim[:n[c], c]]
        assert objs == [int(n[c]) - 1 - i for i in range(n[c])]
    assert n_ok > N // 2
    if cone_deg > 60:
        # the wide cone reaches total internal reflection for chains starting
        # in glass (critical angle 41.8 degrees), so both branches are pinned
        assert n_tir > 50
    else:
        assert n_tir == 0


def two_mirror_scene(half=50.0, gap=2.0):
    """Mirror at z = 0 facing up (object 0) and mirror at z = gap facing down
    (object 1)."""
    v = np.array([[-half, -half, 0], [half, -half, 0], [half, half, 0], [-half, half, 0],
                  [-half, -half, gap], [half, -half, gap], [half, half, gap], [-half, half, gap]], np.float64)
    t = np.array([[0, 1, 2], [0, 2, 3], [4, 6, 5], [4, 7, 6]])
    n = np.array([[0, 0, 1.0]] * 4 + [[0, 0, -1.0]] * 4)
    return W._finish("two_mirrors", v, n, t, np.array([0, 0, 1, 1]), [W.MAT_MIRROR, W.MAT_MIRROR], [1.0, 1.0],
                     np.zeros((0, 4)), [], 2 * half)


def test_deduction_between_parallel_mirrors_unfolds_to_a_line(oracle_lib):
    # Between two parallel mirrors the reflected path unfolds into a straight
    # line: vertex i lies at horizontal offset (z-distance travelled) * tan
    # of the launch angle, alternately on the upper and the lower mirror.
    sc = two_mirror_scene()
    osc = O.Scene(sc)
    g = np.random.default_rng(12)
    N = 2000
    n = g.integers(1, 9, N)
    xD = np.stack([g.uniform(-1, 1, N), g.uniform(-1, 1, N), np.full(N, 1.0)], 1)
    ep = ep64(xD, [0.0, 0.0, 1.5], n=n, types_=0, obj1=W.P0_DIRECTION)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(60)))
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    assert np.all(st == 0)
    for c in range(N):
        wD = pos[:, 0, c] - xD[c]
        wD /= np.linalg.norm(wD)
        slope = wD[:2] / wD[2]
        travelled = 1.0
        for i in range(n[c]):
            z = 2.0 if i % 2 == 0 else 0.0
            want = np.array([xD[c, 0] + slope[0] * travelled, xD[c, 1] + slope[1] * travelled, z])
            assert np.abs(pos[:, i, c] - want).max() < 1e-12, (c, i)
            assert osc.src.tri_obj[prim[i, c]] == (1 if i % 2 == 0 else 0)
            travelled += 2.0


# ---------------------------------------------------------------------------
# component pick of the guided mixture
# ---------------------------------------------------------------------------

def test_guided_component_pick_follows_the_mixture_weights(oracle_lib):
    # Eight components with distinct weights, means and covariances, far
    # apart: the share of seeds near each mean must follow pi (chi-square,
    # 7 degrees of freedom), and each cluster's covariance must be its own
    # component's (an index shift between pi, mu and Sigma fails here).
    sc = S.plane_scene(W.MAT_MIRROR, half=2.0)
    osc = O.Scene(sc)
    K, res = 8, 2
    pi = np.arange(1, K + 1, dtype=np.float64)
    pi /= pi.sum()
    ang = 2 * np.pi * np.arange(K) / K
    mu = np.stack([1.2 * np.cos(ang), 1.2 * np.sin(ang)], 1)
    sd = 0.02 + 0.01 * np.arange(K)
    cov = np.stack([sd ** 2, 0.3 * sd ** 2, 0.5 * sd ** 2], 1)
    cells = res ** 3
    gd = O.Guide([-5, -5, -5], [5, 5, 5], res, K, 0, np.ones(cells, np.int32), np.tile(pi, (cells, 1)),
                 np.tile(mu, (cells, 1, 1)), np.tile(cov, (cells, 1, 1)))
    N = 40000
    ep = ep64([0.0, 0.0, 1.0], np.tile([0.0, 0.0, 2.0], (N, 1)), obj1=0)
    prim, pos, st = O.sample_seeds(osc, ep, guide=gd, alpha=0.0)
    assert np.all(st == 0)
    xy = pos[:2, 0, :].T
    lab = np.argmin(((xy[:, None, :] - mu[None]) ** 2).sum(-1), 1)
    cnt = np.bincount(lab, minlength=K)
    chi2 = float((((cnt - N * pi) ** 2) / (N * pi)).sum())
    assert chi2 < 24.3, (chi2, cnt, N * pi)   # 0.1% point of chi-square(7)
    for j in range(K):
        d = xy[lab == j] - mu[j]
        c = np.cov(d.T)
        want = np.array([[cov[j, 0], cov[j, 1]], [cov[j, 1], cov[j, 2]]])
        m = cnt[j]
        assert np.abs(d.mean(0)).max() < 5 * sd[j] / math.sqrt(m)
        assert np.abs(c - want).max() < 6 * sd[j] ** 2 * math.sqrt(2.0 / m), j


# ---------------------------------------------------------------------------
# the direction cone of the slab workloads covers every admissible chain
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_slab_cone_covers_every_admissible_first_direction(oracle_lib):
    # The paper's direction initialization draws w_D on the whole hemisphere
    # (Sec. 6.4).  The slab workloads restrict it to a cone of
    # SEED_CONE_DEG about +z, which keeps p_0 covering every admissible chain
    # (unbiasedness needs T > 0 => p > 0, Sec. 4) only if no admissible chain
    # leaves x_D outside the cone.  Dense hemisphere seeding on a grid of
    # shading points, for every length, finds the admissible chains; all of
    # their first directions must lie inside the cone, with margin.
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    grid = np.array([0.5, 2.0, 3.5])
    zs = np.array([W.interface_z(k) - 0.5 * W.SLAB_THICK for k in range(1, 9)])
    M = 1200
    rows = []
    for n in range(2, 9):
        for x in grid:
            for y in grid:
                rows.append((n, x, y))
    N = len(rows) * M
    n = np.repeat([r[0] for r in rows], M)
    xD = np.stack([np.repeat([r[1] for r in rows], M), np.repeat([r[2] for r in rows], M), zs[n - 1]], 1)
    ep = ep64(xD, [2.0, 2.0, 3.0], n=n, types_=(1 << n) - 1, obj1=W.P0_DIRECTION)
    prm_h = O.params(sc.scale, cone_cos=0.0)
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm_h)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st, polish=False, prm=prm_h)
    conv = r["status"] == O.CONVERGED
    assert conv.sum() > 2000
    w = r["pos"][:, 0, :].T - xD
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip(w[conv, 2], -1, 1)))
    assert ang.max() < W.SEED_CONE_DEG - 4.0, ang.max()
    # every solution the hemisphere finds is also found from the cone
    cc = math.cos(math.radians(W.SEED_CONE_DEG))
    prm_c = O.params(sc.scale, cone_cos=cc)
    prim2, pos2, st2 = O.sample_seeds(osc, ep, prm=prm_c)
    r2 = O.walk(osc, ep, prim2, pos2.astype(np.float32), st2, polish=False, prm=prm_c)
    conv2 = r2["status"] == O.CONVERGED
    row = np.arange(N) // M
    hemi = set(zip(row[conv], r["sol"][conv]))
    cone = set(zip(row[conv2], r2["sol"][conv2]))
    assert len(hemi - cone) <= 0.02 * len(hemi), (len(hemi - cone), len(hemi))


# ---------------------------------------------------------------------------
# the stalled-walk path: FP64 check accepts the chain at the closed form
# ---------------------------------------------------------------------------

def test_stalled_walk_is_accepted_by_the_fp64_check_at_the_mirror_point(oracle_lib):
    # With a residual tolerance of 0 no FP32-style convergence test can pass:
    # every walk that reaches the solution ends when a full step within the
    # vertex tolerance no longer lowers the residual (the stall), and the FP64
    # check must then accept it at the mirror-image point of the plane.
    sc = S.plane_scene(W.MAT_MIRROR)
    osc = O.Scene(sc)
    g = np.random.default_rng(13)
    N = 300
    xD = np.stack([g.uniform(-2, 2, N), g.uniform(-2, 2, N), g.uniform(0.3, 2, N)], 1)
    xL = np.stack([g.uniform(-2, 2, N), g.uniform(-2, 2, N), g.uniform(0.5, 3, N)], 1)
    ep = ep64(xD, xL)
    prim, pos, st = O.sample_seeds(osc, ep)
    base = O.walk(osc, ep, prim, pos.astype(np.float32), st, polish=False)
    stall = O.walk(osc, ep, prim, pos.astype(np.float32), st, polish=False,
                   prm=O.params(sc.scale, tol_residual=0.0))
    conv = stall["status"] == O.CONVERGED
    assert np.array_equal(conv, base["status"] == O.CONVERGED)
    assert conv.mean() > 0.9
    # the stall path runs the FP64 polish (reported as `polished` even though
    # polishing was switched off); a plain convergence would not
    via_stall = conv & (stall["polished"] == 1)
    assert via_stall.sum() > 0.9 * conv.sum()
    assert not np.any(base["polished"][conv])
    img = xL * np.array([1, 1, -1.0])
    t = xD[:, 2] / (xD[:, 2] - img[:, 2])
    x1 = xD + (img - xD) * t[:, None]
    err = np.linalg.norm(stall["pos"][:, 0, :].T - x1, axis=1)
    assert err[conv].max() < 1e-12
    assert stall["residual"][conv].max() < 1e-10


# ---------------------------------------------------------------------------
# ball lens: the number of two-refraction chains by receiver radius
# ---------------------------------------------------------------------------

def ball_lens_paths(rho, eta=1.5, zD=-1.5, zL=3.0, n_grid=20001):
    """Two-refraction paths from the axial light (0, 0, zL) through the unit
    glass ball to the receiver point (rho, 0, zD).  By symmetry every such
    path lies in the meridian plane y = 0: trace the light's rays by launch
    angle in that plane (Snell's law in vector form at both crossings) and
    bisect the landing offset x(psi) = rho.  Returns each root as the chain
    (x_1, x_2) counted from the receiver: the light's exit point, then its
    entry point."""
    def trace(psi):
        d = np.array([math.sin(psi), -math.cos(psi)])
        o = np.array([0.0, zL])
        b = o @ d
        disc = b * b - (o @ o - 1.0)
        if disc <= 0:
            return None
        p1 = o + d * (-b - math.sqrt(disc))
        n1 = p1.copy()
        c1 = -(d @ n1)
        e = 1.0 / eta
        k = 1 - e * e * (1 - c1 * c1)
        d2 = e * d + (e * c1 - math.sqrt(k)) * n1
        p2 = p1 + d2 * (-2.0 * (p1 @ d2))
        n2 = -p2
        c2 = -(d2 @ n2)
        k2 = 1 - eta * eta * (1 - c2 * c2)
        if k2 <= 0:
            return None
        d3 = eta * d2 + (eta * c2 - math.sqrt(k2)) * n2
        if d3[1] >= 0:
            return None
        t = (zD - p2[1]) / d3[1]
        return p2[0] + t * d3[0], p1, p2

    lim = math.asin(1.0 / zL)
    psis = np.linspace(-lim, lim, n_grid)[1:-1]
    vals = []
    for p in psis:
        r = trace(p)
        vals.append(np.nan if r is None else r[0] - rho)
    vals = np.array(vals)
    out = []
    for k in range(len(psis) - 1):
        if not (np.isfinite(vals[k]) and np.isfinite(vals[k + 1])) or vals[k] * vals[k + 1] > 0:
            continue
        a, b, fa = psis[k], psis[k + 1], vals[k]
        for _ in range(100):
            m = 0.5 * (a + b)
            fm = trace(m)[0] - rho
            if (fm > 0) == (fa > 0):
                a, fa = m, fm
            else:
                b = m
        _, p1, p2 = trace(0.5 * (a + b))
        out.append((np.array([p2[0], 0.0, p2[1]]), np.array([p1[0], 0.0, p1[1]])))
    return out


def ball_lens_scene(eta=1.5):
    v, n, t, o = W._empty_mesh()
    return W._finish("ball_lens", v, n, t, o, [W.MAT_DIELECTRIC], [eta], [[0.0, 0.0, 0.0, 1.0]], [0], 2.0)


def oracle_solutions(osc, xD, xL, M):
    ep = ep64(xD, np.tile(xL, (M, 1)), n=2, types_=3, obj1=0)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    found = []
    for c in np.nonzero(conv)[0]:
        p = r["pos"][:, :2, c].T
        if not any(np.abs(p - q).max() < 1e-6 for q in found):
            found.append(p)
    return found, ep, r


@pytest.mark.parametrize("rho,count", [(0.08, 3), (0.15, 3), (0.5, 1), (1.2, 1), (2.6, 0)])
def test_ball_lens_solution_count_by_receiver_radius(oracle_lib, rho, count):
    sc = ball_lens_scene()
    osc = O.Scene(sc)
    xD = np.array([rho, 0.0, -1.5])
    xL = np.array([0.0, 0.0, 3.0])
    want = ball_lens_paths(rho)
    assert len(want) == count
    found, _, _ = oracle_solutions(osc, xD, xL, 6000)
    assert len(found) == count
    for x1, x2 in want:
        best = min(max(np.abs(q[0] - x1).max(), np.abs(q[1] - x2).max()) for q in found)
        assert best < 1e-9


def test_ball_lens_mean_inverse_probability_counts_three_chains(oracle_lib):
    # E[1{converged} K] = number of admissible chains (here 3, inside the fold)
    sc = ball_lens_scene()
    osc = O.Scene(sc)
    xD = np.array([0.1, 0.0, -1.5])
    xL = np.array([0.0, 0.0, 3.0])
    assert len(ball_lens_paths(0.1)) == 3
    M = 3000
    _, ep, r = oracle_solutions(osc, xD, xL, M)
    trials, ip, trunc = O.inv_prob(osc, ep, r["prim"], r["pos"], r["status"], max_trials=200000)
    assert not trunc.any()
    est = np.where(r["status"] == O.CONVERGED, ip, 0.0)
    se = est.std() / math.sqrt(M)
    assert abs(est.mean() - 3.0) < 4 * se, (est.mean(), se)


# ---------------------------------------------------------------------------
# validation of external chains (used on the GPU's converged chains)
# ---------------------------------------------------------------------------

def test_validate_accepts_float32_solutions_and_rejects_wrong_type(oracle_lib):
    eta = 1.5
    sc = S.plane_scene(W.MAT_DIELECTRIC, ior=eta)
    osc = O.Scene(sc)
    g = np.random.default_rng(14)
    N = 200
    xD = np.stack([g.uniform(-1.5, 1.5, N), g.uniform(-1.5, 1.5, N), g.uniform(-2, -0.3, N)], 1)
    xL = np.stack([g.uniform(-1.5, 1.5, N), g.uniform(-1.5, 1.5, N), g.uniform(0.5, 3, N)], 1)
    ep = ep64(xD, xL, n=1, types_=1)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    assert conv.sum() > 50
    pos32 = r["pos"].astype(np.float32).astype(np.float64)
    v = O.validate(osc, ep, r["prim"], pos32)
    assert np.all(v["ok"][conv] == 1)
    assert v["residual"][conv].max() < 1e-10
    assert v["moved"][conv].max() < 1e-5
    assert np.all(v["side"][conv] == 1) and np.all(v["visible"][conv] == 1)
    for c in np.nonzero(conv)[0]:
        assert np.linalg.norm(pos32[:, 0, c] + 0 - snell_point_flat(xD[c], xL[c], eta)) < 1e-6
    # the same vertices read as a reflection: the polish moves them far (or
    # the side test fails), so the chain is not accepted as an R solution
    ep_r = ep64(xD, xL, n=1, types_=0)
    w = O.validate(osc, ep_r, r["prim"], pos32)
    bad = (w["residual"] > 1e-10) | (w["moved"] > 1e-4 * sc.scale) | (w["side"] == 0)
    assert np.all(bad[conv])


def snell_point_flat(xD, xL, eta):
    """Refraction point on z = 0 by bisection on Snell's law in the plane of incidence."""
    dh = xL[:2] - xD[:2]
    D = np.linalg.norm(dh)
    u = dh / D
    hD, hL = abs(xD[2]), abs(xL[2])
    a, b = 0.0, D
    for _ in range(200):
        m = 0.5 * (a + b)
        f = eta * m / math.hypot(m, hD) - (D - m) / math.hypot(D - m, hL)
        a, b = (m, b) if f < 0 else (a, m)
    s = 0.5 * (a + b)
    return np.array([xD[0] + u[0] * s, xD[1] + u[1] * s, 0.0])
