"""Pins of the oracle's chain gradients (implicit function theorem, Sec. 5.2).

The oracle differentiates converged chains with a forward IFT in FP64 with
nested dual numbers.  These tests check it against (a) the closed-form mirror
image solution of a plane mirror, whose reflection point and generalized
geometry term are explicit functions of the endpoints, and (b) central finite
differences (h = 1e-4) of the oracle's own Newton walk, re-solved to a 1e-12
residual for every perturbed endpoint or surface parameter.
"""
import math
import types

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import scenes as S

H_FD = 1e-4


def _ep(xD, nD, xL, length, types_, obj1):
    return types.SimpleNamespace(xD=np.ascontiguousarray(xD, np.float64), nD=np.ascontiguousarray(nD, np.float64),
                                 xL=np.ascontiguousarray(xL, np.float64), length=np.asarray(length, np.uint8),
                                 types=np.asarray(types_, np.uint8), obj1=np.asarray(obj1, np.int32),
                                 n=len(length))


def _loss(r, out, g):
    """Per-chain l = sum_i r_i . x_i + g G."""
    return (r * out["pos"]).sum(axis=(0, 1)) + g * out["G"]


# ---------------------------------------------------------------------------
# plane mirror: closed form
# ---------------------------------------------------------------------------

def _plane_mirror_closed_form(xD, nD, xL):
    """Reflection point on z = 0 and G for a point light: the chain is the
    straight segment from x_D to the mirror image x_L' = (xL_x, xL_y, -xL_z);
    the generalized geometry term reduces to |n_D . w| / |x_L' - x_D|^2."""
    img = np.array([xL[0], xL[1], -xL[2]])
    t = xD[2] / (xD[2] + xL[2])
    x1 = xD + (img - xD) * t
    d = img - xD
    w = d / np.linalg.norm(d)
    G = abs(np.dot(nD, w)) / np.dot(d, d)
    return x1, G


def test_plane_mirror_gradient_matches_closed_form(oracle_lib):
    g = np.random.default_rng(3)
    n = 12
    xD = np.stack([g.uniform(-1, 1, n), g.uniform(-1, 1, n), g.uniform(0.5, 2, n)], 0)
    xL = np.stack([g.uniform(-1, 1, n), g.uniform(-1, 1, n), g.uniform(1, 3, n)], 0)
    nDv = g.normal(size=(3, n))
    nDv /= np.linalg.norm(nDv, axis=0)
    ep = _ep(xD, nDv, xL, np.ones(n), np.zeros(n), np.full(n, -1))
    osc = O.Scene(S.plane_scene())
    prm = O.params(osc.scale)
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    out = O.walk(osc, ep, prim, pos, st, prm=prm)
    assert (out["status"] == O.CONVERGED).all()
    r = np.zeros((3, O.KMAX, n))
    r[:, 0, :] = g.normal(size=(3, n))
    gG = g.normal(size=n)
    gxD, gxL, _, ok = O.adjoint(osc, ep, out["prim"], out["pos"], out["status"], r, gG, prm=prm)
    assert ok.all()
    h = 1e-6
    for c in range(n):
        def l(a, b):
            x1, G = _plane_mirror_closed_form(a, nDv[:, c], b)
            return np.dot(r[:, 0, c], x1) + gG[c] * G
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd_D = (l(xD[:, c] + e, xL[:, c]) - l(xD[:, c] - e, xL[:, c])) / (2 * h)
            fd_L = (l(xD[:, c], xL[:, c] + e) - l(xD[:, c], xL[:, c] - e)) / (2 * h)
            assert gxD[k, c] == pytest.approx(fd_D, rel=1e-6, abs=1e-8)
            assert gxL[k, c] == pytest.approx(fd_L, rel=1e-6, abs=1e-8)


def test_plane_mirror_position_jacobian_is_explicit(oracle_lib):
    """With g = 0 and r = e_z the loss is the height of the reflection
    point, identically 0 on the plane: every gradient vanishes.  With
    r = e_x it is x_1 = xD_x + (xL_x - xD_x) zD / (zD + zL), whose partial
    derivatives are written out here."""
    xD = np.array([[0.3], [-0.2], [1.1]])
    xL = np.array([[-0.7], [0.4], [2.3]])
    ep = _ep(xD, np.array([[0.0], [0.0], [1.0]]), xL, [1], [0], [-1])
    osc = O.Scene(S.plane_scene())
    prm = O.params(osc.scale)
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    out = O.walk(osc, ep, prim, pos, st, prm=prm)
    for axis, want_fn in ((2, None), (0, "x")):
        r = np.zeros((3, O.KMAX, 1))
        r[axis, 0, 0] = 1.0
        gxD, gxL, _, ok = O.adjoint(osc, ep, out["prim"], out["pos"], out["status"], r, np.zeros(1), prm=prm)
        assert ok[0] == 1
        if want_fn is None:
            assert np.abs(gxD).max() < 1e-12 and np.abs(gxL).max() < 1e-12
            continue
        zD, zL = xD[2, 0], xL[2, 0]
        s = zD / (zD + zL)
        dx = xL[0, 0] - xD[0, 0]
        want_D = [1 - s, 0.0, dx * zL / (zD + zL) ** 2]
        want_L = [s, 0.0, -dx * zD / (zD + zL) ** 2]
        np.testing.assert_allclose(gxD[:, 0], want_D, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(gxL[:, 0], want_L, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# finite differences of the walk
# ---------------------------------------------------------------------------

def _fd_walk(osc, ep, base, prm):
    """Re-solve every chain from the base solution; returns outputs."""
    return O.walk(osc, ep, base["prim"], base["pos"], None, prm=prm)


def _same(a, b, base):
    return ((a["status"] == O.CONVERGED) & (b["status"] == O.CONVERGED)
            & (a["prim"] == base["prim"]).all(0) & (b["prim"] == base["prim"]).all(0))


@pytest.fixture(scope="module")
def slab_case(oracle_lib):
    sc = W.slab_stack_scene()
    n = 96
    ep32 = W.slab_adjoint_endpoints(n, seed=5)
    ep = _ep(ep32.xD, ep32.nD, ep32.xL, ep32.length, ep32.types, ep32.obj1)
    osc = O.Scene(sc)
    prm = O.params(sc.scale, cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)))
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm)
    base = O.walk(osc, ep, prim, pos, st, prm=prm)
    conv = base["status"] == O.CONVERGED
    assert conv.sum() >= 40
    r64, g64 = W.loss_weights(n, seed=5)
    r = r64.astype(np.float64)
    g = g64.astype(np.float64)
    theta = W.slab_theta(sc)
    gxD, gxL, gth, ok = O.adjoint(osc, ep, base["prim"], base["pos"], base["status"], r, g, theta=theta, prm=prm)
    assert (ok.astype(bool) == conv).all()
    return types.SimpleNamespace(sc=sc, osc=osc, ep=ep, prm=prm, base=base, conv=conv, r=r, g=g, theta=theta,
                                 gxD=gxD, gxL=gxL, gth=gth)


def _close(adj, fd, scale):
    return np.abs(adj - fd) <= 1e-5 * scale + 1e-4 * np.abs(fd)


@pytest.mark.parametrize("which", ["xD", "xL"])
def test_endpoint_gradients_match_central_differences(slab_case, which):
    c = slab_case
    adj = c.gxD if which == "xD" else c.gxL
    ok_all = np.zeros_like(c.conv)
    checked = np.zeros_like(c.conv)
    fails = 0
    for k in range(3):
        eps = []
        for sgn in (1, -1):
            xD, xL = c.ep.xD.copy(), c.ep.xL.copy()
            (xD if which == "xD" else xL)[k] += sgn * H_FD
            eps.append(_ep(xD, c.ep.nD, xL, c.ep.length, c.ep.types, c.ep.obj1))
        a = _fd_walk(c.osc, eps[0], c.base, c.prm)
        b = _fd_walk(c.osc, eps[1], c.base, c.prm)
        use = c.conv & _same(a, b, c.base)
        fd = (_loss(c.r, a, c.g) - _loss(c.r, b, c.g)) / (2 * H_FD)
        scale = np.abs(c.r).sum((0, 1)) + np.abs(c.g * c.base["G"])
        good = _close(adj[k], fd, scale)
        fails += int((use & ~good).sum())
        checked |= use
        ok_all |= use & good
    assert checked.sum() >= 0.9 * c.conv.sum()
    assert fails == 0, f"{fails} gradient entries differ from central differences"


def test_theta_gradients_match_central_differences(slab_case):
    c = slab_case
    # chains of length <= 4 cross objects 0..3 only: slabs 0 and 1
    touched = 16
    assert np.abs(c.gth[:, touched:]).max() == 0.0
    fails = 0
    used = 0
    for k in range(touched):
        outs = []
        for sgn in (1, -1):
            th = c.theta.copy()
            th[k] += sgn * H_FD
            c.osc.set_theta(th)
            outs.append(_fd_walk(c.osc, c.ep, c.base, c.prm))
        c.osc.set_theta(c.theta)
        a, b = outs
        use = c.conv & _same(a, b, c.base)
        fd = (_loss(c.r, a, c.g) - _loss(c.r, b, c.g)) / (2 * H_FD)
        scale = np.abs(c.r).sum((0, 1)) + np.abs(c.g * c.base["G"])
        good = _close(c.gth[:, k], fd, scale)
        fails += int((use & ~good).sum())
        used += int(use.sum())
    assert used >= 0.9 * touched * c.conv.sum()
    assert fails == 0, f"{fails} theta gradient entries differ from central differences"


def test_theta_roundtrip_restores_solutions(slab_case):
    """Setting the parameters the scene was built with reproduces the walk
    (vertices rebuilt in FP64 differ from the float32 mesh by rounding)."""
    c = slab_case
    c.osc.set_theta(c.theta)
    again = _fd_walk(c.osc, c.ep, c.base, c.prm)
    m = c.conv
    assert (again["status"][m] == O.CONVERGED).all()
    assert (again["prim"][:, m] == c.base["prim"][:, m]).all()
    assert np.abs(again["pos"][:, :, m] - c.base["pos"][:, :, m]).max() < 1e-5
