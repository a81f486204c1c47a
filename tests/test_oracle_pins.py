"""Pins of the FP64 oracle against what the geometry and mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (numpy's Philox), brute force, a closed form, a 1-D root enumeration,
a textbook identity, an exact EM invariant or a statistical law.
"""
import math
import types

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import scenes as S


def ep64(xD, xL, n=1, types_=0, nD=(0, 0, 1), obj1=-1):
    """Endpoints kept in float64 (the oracle takes FP64 endpoints)."""
    xD = np.atleast_2d(np.asarray(xD, np.float64))
    xL = np.atleast_2d(np.asarray(xL, np.float64))
    N = max(len(xD), len(xL))
    xD = np.ascontiguousarray(np.broadcast_to(xD, (N, 3)).T)
    xL = np.ascontiguousarray(np.broadcast_to(xL, (N, 3)).T)
    nd = np.ascontiguousarray(np.broadcast_to(np.asarray(nD, np.float64), (N, 3)).T)
    return types.SimpleNamespace(xD=xD, nD=nd, xL=xL, length=np.full(N, n, np.uint8),
                                 types=np.full(N, types_, np.uint8), obj1=np.full(N, obj1, np.int32), n=N)


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("key,ctr", [((0, 0), (1, 0, 0, 0)), ((5, 7), (2, 2, 3, 4)),
                                     ((2 ** 63 + 5, 11), (2 ** 64 - 1, 3, 0, 9))])
def test_philox_matches_numpy(oracle_lib, key, ctr):
    # numpy's Philox is Philox4x64-10; it increments its 256-bit counter
    # before each block, so counter c - 1 yields the block for c.
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array([ctr[0] - 1, *ctr[1:]], np.uint64))
    want = bg.random_raw(4)
    got = O.philox(key[0], ctr, key1=key[1])
    assert list(got) == list(want)


def test_uniform_extraction_from_numpy_words(oracle_lib):
    for chain, trial, attempt in [(1, 0, 0), (17, 3, 2), (2 ** 40, 65, 8)]:
        bg = np.random.Philox(key=np.array([9, 0], np.uint64),
                              counter=np.array([chain - 1, trial, attempt, 0], np.uint64))
        halves = []
        for w in bg.random_raw(4):
            halves += [int(w) >> 32, int(w) & 0xFFFFFFFF]
        want = np.array([(h >> 8) / 2.0 ** 24 for h in halves])
        got = O.uniforms(9, chain, trial, attempt)
        assert np.array_equal(got, want)
        assert np.all((got >= 0) & (got < 1))


# ---------------------------------------------------------------------------
# ray casting: BVH traversal equals brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scene_fn", [W.icosphere_glass_scene, W.slab_stack_scene,
                                      lambda: W.water_scene(res=96)])
def test_bvh_matches_brute_force(oracle_lib, scene_fn):
    sc = scene_fn()
    osc = O.Scene(sc)
    g = np.random.default_rng(1)
    lo = sc.verts.min(0) - 1.0 if sc.n_tris else np.array([-3, -3, -3.0])
    hi = sc.verts.max(0) + 1.0 if sc.n_tris else np.array([3, 3, 3.0])
    n = 1500
    o = g.uniform(lo, hi, (n, 3))
    tgt = g.uniform(lo, hi, (n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p1, t1 = O.raycast(osc, o, d, tmin=1e-7)
    p2, t2 = O.raycast(osc, o, d, tmin=1e-7, brute=True)
    assert np.array_equal(p1, p2)
    assert np.array_equal(t1, t2)
    assert (p1 != O.PRIM_NONE).mean() > 0.2


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def great_circle_reflection(xD, xL, grid=4000):
    """All reflection points on the unit sphere for endpoints xD, xL: they lie
    on the great circle through O, xD, xL; bracket the tangential component
    of the half vector on a grid and bisect."""
    u = xD / np.linalg.norm(xD)
    v = xL - u * (xL @ u)
    v /= np.linalg.norm(v)

    def g(ph):
        p = np.cos(ph) * u + np.sin(ph) * v
        t = -np.sin(ph) * u + np.cos(ph) * v
        h = (xD - p) / np.linalg.norm(xD - p) + (xL - p) / np.linalg.norm(xL - p)
        return h @ t, p, h @ p

    phis = np.linspace(-np.pi, np.pi, grid + 1)
    vals = np.array([g(ph)[0] for ph in phis])
    out = []
    for k in np.nonzero(np.sign(vals[:-1]) * np.sign(vals[1:]) < 0)[0]:
        a, b = phis[k], phis[k + 1]
        fa = vals[k]
        for _ in range(80):
            m = 0.5 * (a + b)
            fm = g(m)[0]
            if np.sign(fm) == np.sign(fa):
                a, fa = m, fm
            else:
                b = m
        _, p, hp = g(0.5 * (a + b))
        if hp > 0 and p @ xD > 1 and p @ xL > 1:   # visible from both endpoints
            out.append(p)
    return out


def test_sphere_mirror_matches_great_circle_root(oracle_lib):
    sc = W.sphere_mirror_scene()
    ep = W.sphere_mirror_endpoints(1024)
    osc = O.Scene(sc)
    prim, pos, st = O.sample_seeds(osc, ep)
    assert np.all(st == 0)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    has = np.zeros(ep.n, bool)
    for c in range(ep.n):
        sols = great_circle_reflection(ep.xD[:, c].astype(np.float64), ep.xL[:, c].astype(np.float64), 1500)
        has[c] = len(sols) > 0
        if conv[c]:
            assert len(sols) == 1
            assert np.linalg.norm(r["pos"][:, 0, c] - sols[0]) < 1e-9
    # a convex mirror has at most one reflection point; existence <=> the
    # visible caps overlap, which holds for about 47% of these configurations
    assert 0.40 < has.mean() < 0.55
    assert not np.any(conv & ~has)
    assert conv.sum() > 100


def test_plane_mirror_image_point_and_G(oracle_lib):
    sc = S.plane_scene(W.MAT_MIRROR)
    osc = O.Scene(sc)
    g = np.random.default_rng(2)
    N = 400
    xD = np.stack([g.uniform(-2, 2, N), g.uniform(-2, 2, N), g.uniform(0.3, 2, N)], 1)
    xL = np.stack([g.uniform(-2, 2, N), g.uniform(-2, 2, N), g.uniform(0.5, 3, N)], 1)
    nD = g.normal(size=(N, 3))
    nD /= np.linalg.norm(nD, axis=1, keepdims=True)
    ep = ep64(xD, xL, nD=(0, 0, 1))
    ep.nD = np.ascontiguousarray(nD.T)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    assert conv.mean() > 0.9
    img = xL * np.array([1, 1, -1.0])
    t = xD[:, 2] / (xD[:, 2] - img[:, 2])
    x1 = xD + (img - xD) * t[:, None]
    err = np.linalg.norm(r["pos"][:, 0, :].T - x1, axis=1)
    assert err[conv].max() < 1e-10
    d = np.linalg.norm(img - xD, axis=1)
    w = (x1 - xD) / np.linalg.norm(x1 - xD, axis=1, keepdims=True)
    G = np.abs(np.sum(nD * w, 1)) / d ** 2
    assert np.allclose(r["G"][conv], G[conv], rtol=1e-9)
    assert np.all(r["kappa"][conv] == 1.0)


def snell_plane_point(xD, xL, eta_D, eta_L):
    """Refraction point on the plane z = 0 between xD (medium eta_D) and xL
    (medium eta_L): Snell's law in the plane of incidence is monotone in the
    horizontal offset s, so bisection finds the unique root."""
    dh = xL[:2] - xD[:2]
    D = np.linalg.norm(dh)
    u = dh / D
    hD, hL = abs(xD[2]), abs(xL[2])

    def f(s):
        return eta_D * s / math.hypot(s, hD) - eta_L * (D - s) / math.hypot(D - s, hL)

    a, b = 0.0, D
    for _ in range(200):
        m = 0.5 * (a + b)
        if f(m) < 0:
            a = m
        else:
            b = m
    s = 0.5 * (a + b)
    return np.array([xD[0] + u[0] * s, xD[1] + u[1] * s, 0.0])


def fresnel_by_angles(ti, tt):
    # Fresnel's sine and tangent laws (an independent form of the equations)
    rs = -math.sin(ti - tt) / math.sin(ti + tt)
    rp = math.tan(ti - tt) / math.tan(ti + tt)
    return 0.5 * (rs * rs + rp * rp)


def test_plane_refraction_snell_root_and_fresnel(oracle_lib):
    eta = 1.5
    sc = S.plane_scene(W.MAT_DIELECTRIC, ior=eta)
    osc = O.Scene(sc)
    g = np.random.default_rng(3)
    N = 300
    xD = np.stack([g.uniform(-1.5, 1.5, N), g.uniform(-1.5, 1.5, N), g.uniform(-2, -0.3, N)], 1)
    xL = np.stack([g.uniform(-1.5, 1.5, N), g.uniform(-1.5, 1.5, N), g.uniform(0.5, 3, N)], 1)
    ep = ep64(xD, xL, n=1, types_=1, nD=(0, 0, 1))
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    assert conv.mean() > 0.4
    for c in np.nonzero(conv)[0]:
        p = snell_plane_point(xD[c], xL[c], eta, 1.0)
        assert np.linalg.norm(r["pos"][:, 0, c] - p) < 1e-9
        wi = (xD[c] - p) / np.linalg.norm(xD[c] - p)
        wo = (xL[c] - p) / np.linalg.norm(xL[c] - p)
        ti, tt = math.acos(abs(wi[2])), math.acos(abs(wo[2]))
        assert abs(r["kappa"][c] - (1 - fresnel_by_angles(ti, tt))) < 1e-9


def test_fresnel_normal_incidence(oracle_lib):
    # at normal incidence F = ((eta - 1) / (eta + 1))^2
    eta = 1.5
    osc = O.Scene(S.plane_scene(W.MAT_DIELECTRIC, ior=eta, half=1.0))
    ep = ep64([[0.2, 0.1, -1.0]], np.tile([0.2, 0.1, 2.0], (64, 1)), n=1, types_=1)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    assert conv.sum() > 5
    assert np.abs(r["kappa"][conv] - (1 - ((eta - 1) / (eta + 1)) ** 2)).max() < 1e-12


# ---------------------------------------------------------------------------
# invariants on the synthetic workloads
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,n", [("sphere_mirror", 2048), ("icosphere_tt", 4096), ("water_caustic", 4096),
                                    ("slab_uneven", 4096)])
def test_converged_residual_below_1e_10(oracle_lib, name, n):
    scene_fn, ep_fn = W.WORKLOADS[name]
    sc = scene_fn() if name != "water_caustic" else W.water_scene(res=128)
    ep = ep_fn(n)
    osc = O.Scene(sc)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)))
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st, prm=prm)
    conv = r["status"] == O.CONVERGED
    assert conv.sum() > 50
    assert r["residual"][conv].max() < 1e-10
    assert np.all(r["polished"][conv] == 1)
    # the reversal symmetry of reflection / refraction: walking the converged
    # chain backwards (x_L <-> x_D) is admissible too
    assert np.all(np.isfinite(r["G"][conv])) and np.all(r["G"][conv] > 0)


def test_reversed_chain_is_admissible(oracle_lib):
    # reflection and refraction are symmetric under reversal: the converged
    # chain read from x_L to x_D satisfies the constraints as well
    sc = W.icosphere_glass_scene()
    osc = O.Scene(sc)
    ep = W.icosphere_endpoints(2048)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = np.nonzero(r["status"] == O.CONVERGED)[0][:200]
    assert len(conv) > 50
    for c in conv:
        C, J, fr = O.constraint(osc, 2, 3, ep.xL[:, c].astype(np.float64), ep.xD[:, c].astype(np.float64),
                                r["prim"][[1, 0], c], r["pos"][:, [1, 0], c].T)
        assert np.abs(C).max() < 1e-9


def test_jacobian_matches_central_differences(oracle_lib):
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    ep = W.slab_uneven_endpoints(4096)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)))
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    checked = 0
    for c in np.nonzero((st == 0) & (ep.length >= 2))[0][:60]:
        n = int(ep.length[c])
        pr = prim[:n, c]
        p = pos[:, :n, c].T.copy()
        xD, xL = ep.xD[:, c].astype(np.float64), ep.xL[:, c].astype(np.float64)
        C0, J, _ = O.constraint(osc, n, int(ep.types[c]), xD, xL, pr, p)
        h = 1e-6
        Jfd = np.zeros_like(J)
        for k in range(2 * n):
            y = np.zeros(2 * n)
            y[k] = h
            Cp, _, _ = O.constraint(osc, n, int(ep.types[c]), xD, xL, pr, O.offset_positions(osc, pr, p, y))
            y[k] = -h
            Cm, _, _ = O.constraint(osc, n, int(ep.types[c]), xD, xL, pr, O.offset_positions(osc, pr, p, y))
            Jfd[:, k] = (Cp - Cm) / (2 * h)
        assert np.abs(J - Jfd).max() < 1e-6 * max(1.0, np.abs(J).max())
        # block tridiagonal: C_i depends only on vertices i-1, i, i+1
        for i in range(n):
            for j in range(n):
                if abs(i - j) > 1:
                    assert np.all(J[2 * i:2 * i + 2, 2 * j:2 * j + 2] == 0)
        checked += 1
    assert checked > 20


# ---------------------------------------------------------------------------
# brute-force enumeration on a y-invariant scene, and E[K] = 1/p
# ---------------------------------------------------------------------------

def strip_solutions(sc, xD, xL):
    """Every reflection point of the y-invariant strip for endpoints in the
    plane y = 0: along y = 0 the mesh is piecewise linear in x with linearly
    blended vertex normals, so each segment is scanned for sign changes of the
    half vector's tangential component and bisected."""
    nx = sc.verts.shape[0] // 2
    P = sc.verts[:nx].astype(np.float64)
    N = sc.normals[:nx].astype(np.float64)
    out = []

    def g(i, s):
        p = P[i] * (1 - s) + P[i + 1] * s
        p[1] = 0.0
        n = N[i] * (1 - s) + N[i + 1] * s
        n /= np.linalg.norm(n)
        h = (xD - p) / np.linalg.norm(xD - p) + (xL - p) / np.linalg.norm(xL - p)
        return h[0] * n[2] - h[2] * n[0], p, h @ n

    for i in range(nx - 1):
        ss = np.linspace(0, 1, 33)
        vals = np.array([g(i, s)[0] for s in ss])
        for k in np.nonzero(np.sign(vals[:-1]) * np.sign(vals[1:]) < 0)[0]:
            a, b, fa = ss[k], ss[k + 1], vals[k]
            for _ in range(80):
                m = 0.5 * (a + b)
                fm = g(i, m)[0]
                if np.sign(fm) == np.sign(fa):
                    a, fa = m, fm
                else:
                    b = m
            _, p, hn = g(i, 0.5 * (a + b))
            if hn > 0:
                out.append(p)
    # keep the points whose two segments clear the profile (visibility)
    keep = []
    xs = P[:, 0]
    zs = P[:, 2]
    for p in out:
        ok = True
        for q in (xD, xL):
            ts = np.linspace(1e-4, 1 - 1e-4, 4000)
            seg = p[None, :] + (q - p)[None, :] * ts[:, None]
            ok &= bool(np.all(seg[:, 2] > np.interp(seg[:, 0], xs, zs) + 1e-9))
        if ok:
            keep.append(p)
    return keep


def test_dense_seeding_finds_exactly_the_enumerated_solutions(oracle_lib):
    sc = S.strip_scene(W.MAT_MIRROR)
    osc = O.Scene(sc)
    xD = np.array([-1.3, 0.0, 0.9])
    xL = np.array([1.1, 0.0, 1.4])
    want = strip_solutions(sc, xD, xL)
    assert len(want) >= 3
    M = 20000
    ep = ep64(xD, np.tile(xL, (M, 1)), obj1=0)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    conv = r["status"] == O.CONVERGED
    found = []
    for c in np.nonzero(conv)[0]:
        p = r["pos"][:, 0, c]
        if not any(np.linalg.norm(p - q) < 1e-6 for q in found):
            found.append(p)
    assert len(found) == len(want)
    for p in want:
        assert min(np.linalg.norm(p - q) for q in found) < 1e-8


def test_mean_bernoulli_inverse_probability_counts_solutions(oracle_lib):
    # E[ 1{converged} K ] = sum_j p_j (1 / p_j) = number of admissible chains
    sc = S.strip_scene(W.MAT_MIRROR)
    osc = O.Scene(sc)
    xD = np.array([-1.3, 0.0, 0.9])
    xL = np.array([1.1, 0.0, 1.4])
    n_sol = len(strip_solutions(sc, xD, xL))
    M = 6000
    ep = ep64(xD, np.tile(xL, (M, 1)), obj1=0)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    trials, ip, trunc = O.inv_prob(osc, ep, r["prim"], r["pos"], r["status"], max_trials=100000)
    assert not trunc.any()
    est = np.where(r["status"] == O.CONVERGED, ip, 0.0)
    se = est.std() / math.sqrt(M)
    assert abs(est.mean() - n_sol) < 4 * se + 1e-9, (est.mean(), n_sol, se)
    # with repeats the estimate is the average of independent K's
    t2, ip2, _ = O.inv_prob(osc, ep, r["prim"], r["pos"], r["status"], max_trials=100000, repeats=4)
    conv = r["status"] == O.CONVERGED
    assert np.all(ip2[conv] * 4 == t2[conv])


# ---------------------------------------------------------------------------
# generalized geometric term: finite differences of the re-solved chain
# ---------------------------------------------------------------------------

def onb(n):
    sign = math.copysign(1.0, n[2])
    a = -1.0 / (sign + n[2])
    b = n[0] * n[1] * a
    return (np.array([1 + sign * n[0] ** 2 * a, sign * b, -sign * n[0]]),
            np.array([b, sign + n[1] ** 2 * a, -n[1]]))


@pytest.mark.parametrize("which", ["sphere", "icosphere", "refract_plane"])
def test_G_matches_finite_differences(oracle_lib, which):
    if which == "sphere":
        sc, ep = W.sphere_mirror_scene(), W.sphere_mirror_endpoints(256)
    elif which == "icosphere":
        sc, ep = W.icosphere_glass_scene(), W.icosphere_endpoints(2048)
    else:
        sc = S.plane_scene(W.MAT_DIELECTRIC, 1.5)
        g = np.random.default_rng(5)
        xD = np.stack([g.uniform(-1, 1, 64), g.uniform(-1, 1, 64), g.uniform(-2, -0.3, 64)], 1)
        xL = np.stack([g.uniform(-1, 1, 64), g.uniform(-1, 1, 64), g.uniform(0.5, 3, 64)], 1)
        ep = ep64(xD, xL, n=1, types_=1)
    osc = O.Scene(sc)
    prim, pos, st = O.sample_seeds(osc, ep)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    idx = np.nonzero(r["status"] == O.CONVERGED)[0][:25]
    assert len(idx) >= 10
    h = 1e-5
    for c in idx:
        n = int(ep.length[c])
        xD = ep.xD[:, c].astype(np.float64)
        xL = ep.xL[:, c].astype(np.float64)
        nD = ep.nD[:, c].astype(np.float64)
        xn = r["pos"][:, n - 1, c]
        t1, t2 = onb((xn - xL) / np.linalg.norm(xn - xL))
        dw = []
        for t in (t1, t2):
            ws = []
            for sgn in (1, -1):
                e = ep64(xD, xL + sgn * h * t, n=n, types_=int(ep.types[c]), nD=nD)
                rr = O.walk(osc, e, r["prim"][:, [c]], r["pos"][:, :, [c]].astype(np.float32))
                assert rr["status"][0] == O.CONVERGED
                x1 = rr["pos"][:, 0, 0]
                ws.append((x1 - xD) / np.linalg.norm(x1 - xD))
            dw.append((ws[0] - ws[1]) / (2 * h))
        w = (r["pos"][:, 0, c] - xD) / np.linalg.norm(r["pos"][:, 0, c] - xD)
        G_fd = abs(nD @ w) * abs(w @ np.cross(dw[0], dw[1]))
        assert abs(G_fd - r["G"][c]) <= 2e-5 * r["G"][c], (which, c, G_fd, r["G"][c])


# ---------------------------------------------------------------------------
# seed distributions
# ---------------------------------------------------------------------------

def ks_uniform(x):
    x = np.sort(x)
    n = len(x)
    return max(np.max(np.arange(1, n + 1) / n - x), np.max(x - np.arange(n) / n))


def test_sphere_cap_seeds_uniform(oracle_lib):
    sc = W.sphere_mirror_scene()
    osc = O.Scene(sc)
    N = 20000
    ep = ep64([0.3, -0.4, -2.2], np.tile([0, 0, 3.0], (N, 1)))
    prim, pos, st = O.sample_seeds(osc, ep)
    p = pos[:, 0, :].T
    assert np.allclose(np.linalg.norm(p, axis=1), 1.0, atol=1e-12)
    ax = ep.xD[:, 0] / np.linalg.norm(ep.xD[:, 0])
    cmax = 1.0 / np.linalg.norm(ep.xD[:, 0])
    ct = p @ ax
    assert ct.min() >= cmax - 1e-12
    # cos(theta) uniform on [cmax, 1]: KS statistic below the 1e-3 critical value
    assert ks_uniform((ct - cmax) / (1 - cmax)) < 1.95 / math.sqrt(N)


def test_surface_seeds_uniform_on_plane(oracle_lib):
    sc = S.plane_scene(W.MAT_MIRROR, half=2.0)
    osc = O.Scene(sc)
    N = 20000
    ep = ep64([0.1, 0.2, 1.0], np.tile([0.0, 0.0, 2.0], (N, 1)), obj1=0)
    prim, pos, st = O.sample_seeds(osc, ep)
    assert np.all(st == 0)
    x = (pos[0, 0] + 2) / 4
    y = (pos[1, 0] + 2) / 4
    assert ks_uniform(x) < 1.95 / math.sqrt(N)
    assert ks_uniform(y) < 1.95 / math.sqrt(N)
    # triangle choice proportional to area (two equal halves)
    assert abs((prim[0] == 0).mean() - 0.5) < 4 * 0.5 / math.sqrt(N)


def test_direction_seeds_uniform_in_cone(oracle_lib):
    sc = S.plane_scene(W.MAT_MIRROR, half=50.0, z=1.0, normal_up=False)
    osc = O.Scene(sc)
    N = 20000
    cc = math.cos(math.radians(40))
    ep = ep64([0.0, 0.0, 0.0], np.tile([0.0, 0.0, -2.0], (N, 1)), obj1=W.P0_DIRECTION)
    prim, pos, st = O.sample_seeds(osc, ep, prm=O.params(100.0, cone_cos=cc))
    assert np.all(st == 0)
    w = pos[:, 0, :].T / np.linalg.norm(pos[:, 0, :].T, axis=1, keepdims=True)
    assert w[:, 2].min() >= cc - 1e-12
    assert ks_uniform((w[:, 2] - cc) / (1 - cc)) < 1.95 / math.sqrt(N)
    phi = (np.arctan2(w[:, 1], w[:, 0]) + np.pi) / (2 * np.pi)
    assert ks_uniform(phi) < 1.95 / math.sqrt(N)


def one_cell_guide(mu, cov, alpha_target=0):
    res, K = 2, 8
    cells = res ** 3
    valid = np.zeros(cells, np.int32)
    valid[:] = 1
    pi = np.zeros((cells, K))
    pi[:, 0] = 1.0
    mus = np.zeros((cells, K, 2))
    mus[:, :, :] = mu
    covs = np.zeros((cells, K, 3))
    covs[:, :, :] = cov
    return O.Guide([-5, -5, -5], [5, 5, 5], res, K, 0, valid, pi, mus, covs)


def test_guided_seeds_follow_the_gaussian(oracle_lib):
    sc = S.plane_scene(W.MAT_MIRROR, half=2.0)
    osc = O.Scene(sc)
    N = 20000
    mu = np.array([0.3, -0.2])
    cov = np.array([0.04, 0.01, 0.02])
    gd = one_cell_guide(mu, cov)
    ep = ep64([0.0, 0.0, 1.0], np.tile([0.0, 0.0, 2.0], (N, 1)), obj1=0)
    prim, pos, st = O.sample_seeds(osc, ep, guide=gd, alpha=0.0)
    xy = pos[:2, 0, :].T
    Sig = np.array([[cov[0], cov[1]], [cov[1], cov[2]]])
    assert np.allclose(xy.mean(0), mu, atol=4 * math.sqrt(0.04 / N))
    assert np.allclose(np.cov(xy.T), Sig, atol=4 * 0.04 * math.sqrt(2 / N))
    # alpha = 0.5: half of the seeds come from the uniform p_0
    prim, pos, st = O.sample_seeds(osc, ep, guide=gd, alpha=0.5)
    xy = pos[:2, 0, :].T
    far = np.abs(xy - mu).max(1) > 1.0    # beyond 5 sigma of the Gaussian
    # the uniform half lands outside the 2 x 2 box around mu (inside the
    # 4 x 4 plane) with probability 1 - 4/16
    assert abs(far.mean() - 0.5 * 0.75) < 4 * math.sqrt(0.25 / N)


# ---------------------------------------------------------------------------
# weighted EM
# ---------------------------------------------------------------------------

def em_samples(n, g, centres, spread, lo, hi):
    k = g.integers(0, len(centres), n)
    uv = np.asarray(centres)[k] + g.normal(scale=spread, size=(n, 2))
    xD = np.stack([g.uniform(lo[0], hi[0], n), g.uniform(lo[1], hi[1], n), g.uniform(lo[2], hi[2], n)], 1)
    w = g.uniform(0.1, 2.0, n)
    return np.concatenate([xD, uv, w[:, None], np.zeros((n, 2))], 1).astype(np.float32)


def weighted_ll(s, gd, cell=0):
    uv, w = s[:, 3:5].astype(np.float64), s[:, 5].astype(np.float64)
    dens = np.zeros(len(s))
    for j in range(gd.comps):
        if gd.pi[cell, j] <= 0:
            continue
        a, b, c = gd.cov[cell, j]
        det = a * c - b * b
        d = uv - gd.mu[cell, j]
        q = (c * d[:, 0] ** 2 - 2 * b * d[:, 0] * d[:, 1] + a * d[:, 1] ** 2) / det
        dens += gd.pi[cell, j] * np.exp(-0.5 * q) / (2 * np.pi * math.sqrt(det))
    return float(np.sum(w * np.log(dens)))


def test_em_initialization_closed_form(oracle_lib):
    g = np.random.default_rng(7)
    lo, hi = [0, 0, 0], [1, 1, 1]
    s = em_samples(500, g, [[0, 0], [1, 1]], 0.2, lo, hi)
    reg = 1e-4
    gd = O.fit_guide(s, lo, hi, res=1, iters=0, reg=reg)
    uv, w = s[:, 3:5].astype(np.float64), s[:, 5].astype(np.float64)
    m = (w[:, None] * uv).sum(0) / w.sum()
    C = ((w[:, None, None] * (uv - m)[:, :, None] * (uv - m)[:, None, :]).sum(0)) / w.sum()
    for j in range(8):
        assert np.allclose(gd.mu[0, j], uv[int(math.floor((j + 0.5) * 500 / 8))])
        assert np.allclose(gd.cov[0, j], [C[0, 0] + reg, C[0, 1], C[1, 1] + reg], rtol=1e-5)
        assert gd.pi[0, j] == 1 / 8


def test_em_moment_invariants_and_monotone_likelihood(oracle_lib):
    g = np.random.default_rng(8)
    lo, hi = [0, 0, 0], [1, 1, 1]
    s = em_samples(800, g, [[0, 0], [1, 0.5], [-0.5, 1]], 0.15, lo, hi)
    reg = 1e-5
    uv, w = s[:, 3:5].astype(np.float64), s[:, 5].astype(np.float64)
    m = (w[:, None] * uv).sum(0) / w.sum()
    M2 = (w[:, None, None] * uv[:, :, None] * uv[:, None, :]).sum(0) / w.sum()
    prev = -np.inf
    for it in range(1, 12):
        gd = O.fit_guide(s, lo, hi, res=1, iters=it, reg=reg)
        # after any M step: sum_j pi_j mu_j is the weighted sample mean and
        # sum_j pi_j (Sigma_j - reg I + mu_j mu_j^T) the weighted second moment
        pm = (gd.pi[0][:, None] * gd.mu[0]).sum(0)
        assert np.allclose(pm, m, atol=1e-10)
        S2 = np.zeros((2, 2))
        for j in range(8):
            a, b, c = gd.cov[0, j]
            S2 += gd.pi[0, j] * (np.array([[a - reg, b], [b, c - reg]]) + np.outer(gd.mu[0, j], gd.mu[0, j]))
        assert np.allclose(S2, M2, atol=1e-10)
        assert abs(gd.pi[0].sum() - 1) < 1e-12
        ll = weighted_ll(s, gd)
        assert ll >= prev - 1e-7 * abs(ll)
        prev = ll


def test_em_recovers_separated_components(oracle_lib):
    g = np.random.default_rng(9)
    lo, hi = [0, 0, 0], [1, 1, 1]
    centres = [[0, 0], [3, 0]]
    s = em_samples(4000, g, centres, 0.1, lo, hi)
    s[:, 5] = 1.0
    gd = O.fit_guide(s, lo, hi, res=1, iters=60, reg=1e-6)
    for cen in centres:
        near = np.linalg.norm(gd.mu[0] - cen, axis=1) < 0.5
        assert abs(gd.pi[0][near].sum() - 0.5) < 0.05
        mean = (gd.pi[0][near][:, None] * gd.mu[0][near]).sum(0) / gd.pi[0][near].sum()
        assert np.linalg.norm(mean - cen) < 0.02


def test_em_cells_and_min_samples(oracle_lib):
    g = np.random.default_rng(10)
    lo, hi = [0, 0, 0], [2, 2, 2]
    s = em_samples(3000, g, [[0, 0]], 0.2, lo, [1, 1, 1])   # only the (0,0,0) octant is populated
    gd = O.fit_guide(s, lo, hi, res=2, iters=5, min_samples=16)
    assert gd.valid[0] == 1 and gd.valid[1:].sum() == 0
    assert gd.count[0] == 3000


def test_newton_converges_quadratically_on_the_smooth_mirror(oracle_lib):
    # Newton's method on the constraints converges quadratically near a
    # solution of a smooth manifold (the footnote on convergence basins in
    # Sec. 5.2): for accepted full steps the residual
    # obeys |C_{k+1}| <= c |C_k|^2.  The walk is re-run with max_iter = k to
    # read the chain after k trials.  A Jacobian that is off (a dropped term,
    # a transposed block) still converges, but only linearly, which puts the
    # ratio |C_{k+1}| / |C_k|^2 above 1e3 once |C_k| < 1e-3.
    sc = W.sphere_mirror_scene()
    ep = W.sphere_mirror_endpoints(1024)
    osc = O.Scene(sc)
    cone = math.cos(math.radians(W.SEED_CONE_DEG))
    prim, pos, st = O.sample_seeds(osc, ep, prm=O.params(sc.scale, cone_cos=cone))
    pos = pos.astype(np.float32)
    K = 12
    res = np.full((K + 1, ep.n), np.nan)
    for k in range(1, K + 1):
        r = O.walk(osc, ep, prim, pos, st, polish=False, prm=O.params(sc.scale, cone_cos=cone, max_iter=k))
        for c in np.nonzero((r["status"] == O.CONVERGED) | (r["status"] == O.MAX_ITER))[0]:
            Cv, _, _ = O.constraint(osc, 1, int(ep.types[c]), ep.xD[:, c].astype(np.float64),
                                    ep.xL[:, c].astype(np.float64), r["prim"][:1, c], r["pos"][:, :1, c].T)
            res[k, c] = np.abs(Cv).max()
    a, b = res[:-1], res[1:]
    near = np.isfinite(a) & np.isfinite(b) & (b > 1e-12) & (b < a) & (a < 1e-3)
    ratio = b[near] / a[near] ** 2
    assert ratio.size > 100
    assert np.median(ratio) < 50 and np.percentile(ratio, 90) < 200
