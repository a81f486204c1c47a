"""Pins of the oracle's glossy chains (Sec. 5.7): offset normals drawn from
the GGX distribution against its closed-form law, chains walked against an
offset normal against a direct root solve of the half-vector condition, and
zero offsets against the specular walk."""
import math
import types

import numpy as np
import pytest
from scipy.optimize import fsolve

import oracle as O
import workloads as W
from tests import scenes as S


def ep64(xD, xL, n=1, types_=0, nD=(0, 0, 1), obj1=0):
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


@pytest.mark.parametrize("rough", [0.05, 0.3])
def test_ggx_offsets_follow_the_microfacet_law(oracle_lib, rough):
    # D(m) cos(theta_m) of GGX: P(tan^2 theta_m <= x) = x / (a^2 + x), phi uniform
    N = 20000
    off = O.sample_offsets(N, seed=3, trial=1, roughness=rough)
    for i in (0, 5):
        o = off[:, i, :]
        s2 = (o ** 2).sum(0)
        assert s2.max() < 1.0
        t2 = s2 / (1.0 - s2)
        assert ks(t2, lambda x: x / (rough ** 2 + x)) < 1.95 / math.sqrt(N)
        phi = (np.arctan2(o[1], o[0]) + np.pi) / (2 * np.pi)
        assert ks(phi, lambda x: x) < 1.95 / math.sqrt(N)
    # vertices and trials draw independent offsets
    assert abs(np.corrcoef(off[0, 0], off[0, 1])[0, 1]) < 0.03


def offset_root(xD, xL, m, eta_D=1.0, eta_L=1.0):
    """Point x on the plane z = 0 where the generalized half vector
    eta_D w_i + eta_L w_o (turned to +z) is parallel to the unit vector m."""
    def f(uv):
        x = np.array([uv[0], uv[1], 0.0])
        wi = (xD - x) / np.linalg.norm(xD - x)
        wo = (xL - x) / np.linalg.norm(xL - x)
        h = eta_D * wi + eta_L * wo
        h = h / np.linalg.norm(h)
        if h[2] < 0:
            h = -h
        return [h[0] - m[0], h[1] - m[1]]
    guess = xD[:2] + (xL[:2] - xD[:2]) * abs(xD[2]) / (abs(xD[2]) + abs(xL[2]))
    uv, info, ier, msg = fsolve(f, guess, full_output=True, xtol=1e-13)
    assert np.abs(f(uv)).max() < 1e-12, msg
    return np.array([uv[0], uv[1], 0.0])


@pytest.mark.parametrize("material,eta", [(W.MAT_MIRROR, 1.0), (W.MAT_DIELECTRIC, 1.5)])
def test_glossy_chain_matches_the_offset_root(oracle_lib, material, eta):
    # On a plane the offset frame is the world frame (s = x, t = y), so the
    # offset normal is the constant m = (o_s, o_t, sqrt(1 - |o|^2)).
    sc = S.plane_scene(material, ior=eta, half=6.0)
    osc = O.Scene(sc)
    g = np.random.default_rng(21)
    N = 200
    refl = material == W.MAT_MIRROR
    zD = g.uniform(0.5, 2.0, N) if refl else -g.uniform(0.5, 2.0, N)
    xD = np.stack([g.uniform(-1.5, 1.5, N), g.uniform(-1.5, 1.5, N), zD], 1)
    xL = np.stack([g.uniform(-1.5, 1.5, N), g.uniform(-1.5, 1.5, N), g.uniform(0.5, 2.0, N)], 1)
    ep = ep64(xD, xL, types_=0 if refl else 1, obj1=0)
    off = O.sample_offsets(N, seed=5, roughness=0.15)
    prim, pos, st = O.sample_seeds(osc, ep, offsets=off)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st, offsets=off)
    conv = r["status"] == O.CONVERGED
    assert conv.mean() > 0.3       # seeds uniform over a 12 x 12 plane
    for c in np.nonzero(conv)[0][:80]:
        o = off[:, 0, c]
        m = np.array([o[0], o[1], math.sqrt(1 - o @ o)])
        want = offset_root(xD[c], xL[c], m, *((1.0, 1.0) if refl else (eta, 1.0)))
        assert np.linalg.norm(r["pos"][:, 0, c] - want) < 1e-9, c
    # the walk really used the offsets: the specular point differs
    r0 = O.walk(osc, ep, prim, pos.astype(np.float32), st)
    both = conv & (r0["status"] == O.CONVERGED)
    d = np.linalg.norm(r["pos"][:, 0, both] - r0["pos"][:, 0, both], axis=0)
    assert np.median(d) > 1e-3


def test_zero_offsets_reproduce_the_specular_walk(oracle_lib):
    # (slab interfaces: the offset frame is defined away from n_s = +-x)
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    ep = W.slab_adjoint_endpoints(2048, seed=4)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)))
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    zero = np.zeros((2, 8, ep.n))
    prim2, pos2, st2 = O.sample_seeds(osc, ep, prm=prm, offsets=zero)
    assert np.array_equal(st, st2) and np.array_equal(prim, prim2)
    assert np.abs(pos - pos2).max() < 1e-12
    # the glossy constraint measures h in a frame turning with the position
    # differently from the specular one, so the Newton paths differ while
    # converging to the same admissible chains
    a = O.walk(osc, ep, prim, pos.astype(np.float32), st, prm=prm)
    b = O.walk(osc, ep, prim, pos.astype(np.float32), st, prm=prm, offsets=zero)
    assert (a["status"] == b["status"]).mean() > 0.97
    conv = (a["status"] == O.CONVERGED) & (b["status"] == O.CONVERGED) & (a["sol"] == b["sol"])
    assert conv.sum() > 0.95 * (a["status"] == O.CONVERGED).sum()
    assert np.abs(a["pos"][:, :, conv] - b["pos"][:, :, conv]).max() < 1e-10
    assert np.allclose(a["G"][conv], b["G"][conv], rtol=1e-9)
    assert np.allclose(a["kappa"][conv], b["kappa"][conv], rtol=1e-12)


def test_glossy_slab_chains_are_admissible_about_their_offsets(oracle_lib):
    # multi-vertex glossy chains through the slab stack converge and keep
    # their residual (with offsets) below 1e-10
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    ep = W.slab_adjoint_endpoints(1024, seed=6)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)))
    off = O.sample_offsets(ep.n, seed=8, roughness=0.05)
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm, offsets=off)
    r = O.walk(osc, ep, prim, pos.astype(np.float32), st, prm=prm, offsets=off)
    conv = r["status"] == O.CONVERGED
    assert conv.mean() > 0.3
    assert r["residual"][conv].max() < 1e-10


def test_glossy_jacobian_matches_central_differences(oracle_lib):
    # the offset-normal constraint's Jacobian (sign turn and world-axis frame
    # included) against central differences of the constraint itself
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    ep = W.slab_adjoint_endpoints(512, seed=12)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)))
    off = O.sample_offsets(ep.n, seed=12, roughness=0.05)
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm, offsets=off)
    checked = 0
    for c in np.nonzero(st == 0)[0][:30]:
        n = int(ep.length[c])
        pr, p = prim[:n, c], pos[:, :n, c].T.copy()
        o = off[:, :n, c].T.copy()
        xD, xL = ep.xD[:, c].astype(np.float64), ep.xL[:, c].astype(np.float64)
        C0, J, _ = O.constraint(osc, n, int(ep.types[c]), xD, xL, pr, p, offsets=o)
        h = 1e-6
        Jfd = np.zeros_like(J)
        for k in range(2 * n):
            y = np.zeros(2 * n)
            y[k] = h
            Cp, _, _ = O.constraint(osc, n, int(ep.types[c]), xD, xL, pr, O.offset_positions(osc, pr, p, y),
                                    offsets=o)
            y[k] = -h
            Cm, _, _ = O.constraint(osc, n, int(ep.types[c]), xD, xL, pr, O.offset_positions(osc, pr, p, y),
                                    offsets=o)
            Jfd[:, k] = (Cp - Cm) / (2 * h)
        assert np.abs(J - Jfd).max() < 1e-6 * max(1.0, np.abs(J).max())
        checked += 1
    assert checked > 20
