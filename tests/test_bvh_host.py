"""CPU checks of the host BVH builder (binned SAH, collapsed to 4-wide nodes):
every triangle sits in exactly one leaf, every child box bounds its range,
and a near-first stack traversal of the emitted nodes -- the device
traversal's steps, written out in numpy -- finds the same first hit as brute
force, with a stack that never exceeds the depth the builder reports."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2311_12818_amd", "csrc")


@pytest.fixture(scope="module")
def bvhlib():
    out = os.path.join(tempfile.mkdtemp(prefix="mpg_bvh_"), "libbvh.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", out,
                           os.path.join(HERE, "native", "bvh_host.cpp"), os.path.join(CSRC, "mpg_scene.cpp")])
    L = C.CDLL(out)
    L.bvh_build.restype = C.c_int
    return L


def build(L, sc, pad=1e-6):
    v = np.ascontiguousarray(sc.verts, np.float32)
    t = np.ascontiguousarray(sc.tris, np.int32)
    nt = t.shape[0]
    cap = nt + 8
    nodes = np.zeros((cap, 32), np.float32)
    order = np.zeros(nt, np.int32)
    ranges = np.zeros((cap, 8), np.int32)
    depth = C.c_int(0)
    n = L.bvh_build(v.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p), nt, C.c_float(pad), cap,
                    nodes.ctypes.data_as(C.c_void_p), order.ctypes.data_as(C.c_void_p),
                    ranges.ctypes.data_as(C.c_void_p), C.byref(depth))
    assert n > 0
    return nodes[:n], order, ranges[:n], depth.value


def refs(nodes):
    return nodes[:, 24:28].copy().view(np.int32)


def tri_hit(o, d, P0, P1, P2):
    """Moller-Trumbore in float64: t or inf."""
    e1, e2 = P1 - P0, P2 - P0
    p = np.cross(d, e2)
    det = e1 @ p
    if abs(det) < 1e-14:
        return np.inf
    s = o - P0
    u = (s @ p) / det
    q = np.cross(s, e1)
    v = (d @ q) / det
    if u < -1e-9 or v < -1e-9 or u + v > 1 + 1e-9:
        return np.inf
    t = (e2 @ q) / det
    return t if t > 1e-6 else np.inf


def brute(o, d, V, T):
    """First hit over all triangles (vectorized Moller-Trumbore, float64)."""
    P0, P1, P2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    e1, e2 = P1 - P0, P2 - P0
    p = np.cross(d, e2)
    det = (e1 * p).sum(1)
    ok = np.abs(det) >= 1e-14
    det = np.where(ok, det, 1.0)
    s = o - P0
    u = (s * p).sum(1) / det
    q = np.cross(s, e1)
    v = (q @ d) / det
    t = (e2 * q).sum(1) / det
    ok &= (u >= -1e-9) & (v >= -1e-9) & (u + v <= 1 + 1e-9) & (t > 1e-6)
    t = np.where(ok, t, np.inf)
    k = int(np.argmin(t))
    return (k, t[k]) if np.isfinite(t[k]) else (-1, np.inf)


def traverse(nodes, order, V, T, o, d, depth_cap):
    """Near-first traversal of 4-wide nodes (the device's steps)."""
    inv = 1.0 / np.where(np.abs(d) > 1e-30, d, np.copysign(1e-30, d))
    R = refs(nodes)
    best_t, best_p = np.inf, -1
    stack = []
    max_sp = 0
    ref = 0
    with np.errstate(invalid="ignore", over="ignore"):
        while True:
            if ref >= 0:
                nd = nodes[ref].astype(np.float64)
                lo = nd[0:12].reshape(3, 4).T
                hi = nd[12:24].reshape(3, 4).T
                t0s = (lo - o) * inv
                t1s = (hi - o) * inv
                t0 = np.maximum(np.minimum(t0s, t1s).max(1), 0.0)
                t1 = np.minimum(np.maximum(t0s, t1s).min(1), best_t)
                tn = np.where(t0 <= t1, t0, np.inf)
                ks = np.argsort(tn, kind="stable")
                hits = [k for k in ks if np.isfinite(tn[k])]
                if hits:
                    for k in reversed(hits[1:]):
                        stack.append(int(R[ref, k]))
                    max_sp = max(max_sp, len(stack))
                    assert len(stack) <= depth_cap
                    ref = int(R[ref, hits[0]])
                    continue
            else:
                u = ref & 0xFFFFFFFF
                start, count = u & 0xFFFFFF, (u >> 24) & 0x7F
                for k in range(start, start + count):
                    tri = order[k]
                    t = tri_hit(o, d, *(V[T[tri]].astype(np.float64)))
                    if t < best_t:
                        best_t, best_p = t, tri
            if not stack:
                break
            ref = stack.pop()
    return best_p, best_t, max_sp


@pytest.mark.parametrize("scene_fn", [W.icosphere_glass_scene, lambda: W.slab_stack_scene(res=32)])
def test_bvh4_structure_and_traversal(bvhlib, scene_fn):
    sc = scene_fn()
    nodes, order, ranges, max_depth = build(bvhlib, sc)
    V, T = sc.verts.astype(np.float64), sc.tris
    nt = T.shape[0]
    # every triangle exactly once in the leaf order, leaves cover it once
    assert np.array_equal(np.sort(order), np.arange(nt))
    R = refs(nodes)
    leaf_tris = []
    for g in range(len(nodes)):
        for k in range(4):
            r = int(R[g, k])
            start, count = int(ranges[g, 2 * k]), int(ranges[g, 2 * k + 1])
            lo = nodes[g, [k, 4 + k, 8 + k]]
            hi = nodes[g, [12 + k, 16 + k, 20 + k]]
            if r < 0:
                u = r & 0xFFFFFFFF
                if (u >> 24) & 0x7F == 0:
                    assert count == 0 and np.all(np.isinf(lo)) and np.all(np.isinf(hi))
                    continue
                assert (u & 0xFFFFFF, (u >> 24) & 0x7F) == (start, count) and count <= 4
                leaf_tris += list(order[start:start + count])
            else:
                assert 0 < r < len(nodes)
            pts = V[T[order[start:start + count]]].reshape(-1, 3)
            assert np.all(lo <= pts.min(0) + 1e-7) and np.all(hi >= pts.max(0) - 1e-7)
    assert sorted(leaf_tris) == list(range(nt))
    # traversal == brute force on random rays
    g = np.random.default_rng(2)
    lo, hi = V.min(0), V.max(0)
    worst = 0
    for _ in range(200):
        o = g.uniform(lo - 1.0, hi + 1.0)
        tgt = g.uniform(lo, hi)
        d = (tgt - o) / np.linalg.norm(tgt - o)
        p, t, msp = traverse(nodes, order, V, T, o, d, max_depth + 1)
        worst = max(worst, msp)
        bp, bt = brute(o, d, V, T)
        assert (p == bp) or (np.isfinite(bt) and abs(t - bt) <= 1e-9 * max(1.0, bt)), (p, bp, t, bt)
    assert worst <= max_depth + 1
