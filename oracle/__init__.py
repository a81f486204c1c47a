"""FP64 CPU oracle for the batched manifold-walk path (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It is an independent, plain FP64 restatement of
the method (C++17 in ``mpg_oracle.cpp``, loaded with ctypes) and shares no code
with the HIP library.

Layouts match the library's: positions ``[3][K][N]``, primitive ids
``[K][N]`` with K = 8, per-chain arrays ``[N]``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

KMAX = 8
HERE = os.path.dirname(os.path.abspath(__file__))
PRIM_NONE = np.iinfo(np.int32).min

CONVERGED, MAX_ITER, SINGULAR, SIDE_INVALID, OCCLUDED, SEED_INVALID, FP64_REJECT, BAD_INPUT = range(8)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


P = C.c_void_p
I32 = C.c_int32
U64 = C.c_uint64
D = C.c_double


class orc_params(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("tol_vertex", D), ("tol_residual", D), ("scale", D),
                ("tmin_rel", D), ("match_rel", D), ("polish_tol", D), ("cone_cos", D)]


def _declare(L):
    L.orc_scene_create.restype = P
    L.orc_scene_create.argtypes = [C.c_int, P, P, C.c_int, P, P, C.c_int, P, P, C.c_int, P, P, D]
    L.orc_scene_destroy.argtypes = [P]
    L.orc_scene_set_heightfield.restype = C.c_int
    L.orc_scene_set_heightfield.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, D, D, D, D, D, C.c_int,
                                            P, P, P, P]
    L.orc_philox.argtypes = [U64, U64, U64, U64, U64, U64, P]
    L.orc_uniforms.argtypes = [U64, U64, U64, U64, P]
    L.orc_solution_id.restype = U64
    L.orc_solution_id.argtypes = [C.c_int, C.c_int, P]
    L.orc_raycast.argtypes = [P, C.c_int, P, P, P, D, C.c_int, P, P, C.c_int]
    L.orc_constraint.restype = C.c_int
    L.orc_constraint.argtypes = [P, C.c_int, C.c_int, P, P, P, P, P, P, P, P]
    L.orc_offset_positions.restype = C.c_int
    L.orc_offset_positions.argtypes = [P, C.c_int, P, P, P, P]
    L.orc_sample_seeds.argtypes = [P, P, P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, U64, U64, D, P, P,
                                   P, C.c_int, P]
    L.orc_sample_offsets.argtypes = [C.c_int, U64, U64, D, P]
    L.orc_walk.argtypes = [P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, P, P, P, C.c_int, P, P, P, P, P,
                           P, P, P, P, C.c_int, P]
    L.orc_inv_prob.argtypes = [P, P, P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, P, P, P, P, C.c_int,
                               C.c_int, U64, D, P, P, P, C.c_int, P]
    L.orc_validate.argtypes = [P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, P, P, P, P, P, P, P, C.c_int, P]
    L.orc_scene_set_theta.restype = C.c_int
    L.orc_scene_set_theta.argtypes = [P, C.c_int, P]
    L.orc_adjoint.argtypes = [P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P,
                              C.c_int]
    L.orc_fit_guide.argtypes = [C.c_int, P, C.c_int, C.c_int, C.c_int, C.c_int, P, P, D, P, P, P, P, P, C.c_int]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def params(scale: float, max_iter: int = 20, tol_vertex: float = 1e-4, tol_residual: float = 1e-5,
           tmin_rel: float = 1e-5, match_rel: float = 1e-3, polish_tol: float = 1e-12,
           cone_cos: float = 0.0) -> orc_params:
    return orc_params(max_iter, tol_vertex, tol_residual, scale, tmin_rel, match_rel, polish_tol, cone_cos)


class Scene:
    """Oracle-side scene built from a :class:`workloads.Scene`."""

    def __init__(self, sc):
        L = lib()
        self._keep = [_c(sc.verts, np.float32), _c(sc.normals, np.float32), _c(sc.tris, np.int32),
                      _c(sc.tri_obj, np.int32), _c(sc.obj_material, np.int32), _c(sc.obj_ior, np.float32),
                      _c(sc.spheres, np.float32).reshape(-1), _c(sc.sphere_obj, np.int32)]
        v, n, t, to, m, io, s, so = self._keep
        self.h = L.orc_scene_create(v.shape[0], _p(v), _p(n), t.shape[0], _p(t), _p(to), m.shape[0], _p(m),
                                    _p(io), so.shape[0], _p(s), _p(so), float(sc.scale))
        for hf in sc.heightfields:
            arr = [_c(hf.amp, np.float64), _c(hf.freq, np.float64), _c(hf.psi, np.float64),
                   _c(hf.phase, np.float64)]
            L.orc_scene_set_heightfield(self.h, hf.obj, hf.res, hf.first_vert, hf.first_tri, hf.x0, hf.x1, hf.y0,
                                        hf.y1, hf.z0, len(hf.amp), *[_p(a) for a in arr])
        self.scale = float(sc.scale)
        self.src = sc

    def n_theta(self):
        return sum(2 * len(hf.amp) for hf in self.src.heightfields)

    def set_theta(self, theta):
        """Replace the height-field parameters (amplitude, phase per sine, in
        height-field order): vertices and normals are recomputed in FP64 and
        the BVH is rebuilt."""
        th = _c(theta, np.float64)
        if lib().orc_scene_set_theta(self.h, th.shape[0], _p(th)) != 0:
            raise ValueError("theta has the wrong length")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_scene_destroy(self.h)
            self.h = None


def philox(seed, ctr, key1=0):
    out = np.zeros(4, np.uint64)
    lib().orc_philox(int(seed), int(ctr[0]), int(ctr[1]), int(ctr[2]), int(ctr[3]), int(key1), _p(out))
    return out


def uniforms(seed, chain, trial, attempt=0):
    out = np.zeros(8, np.float64)
    lib().orc_uniforms(int(seed), int(chain), int(trial), int(attempt), _p(out))
    return out


def solution_id(n, type_, prims):
    pr = _c(prims, np.int32)
    return int(lib().orc_solution_id(int(n), int(type_), _p(pr)))


def raycast(osc: Scene, o, d, exclude=None, tmin=0.0, brute=False, nthreads=0):
    o = _c(o, np.float64).reshape(-1, 3)
    d = _c(d, np.float64).reshape(-1, 3)
    n = o.shape[0]
    ex = _c(np.full(n, PRIM_NONE) if exclude is None else exclude, np.int32)
    prim = np.zeros(n, np.int32)
    t = np.zeros(n, np.float64)
    lib().orc_raycast(osc.h, n, _p(o), _p(d), _p(ex), float(tmin), int(brute), _p(prim), _p(t), nthreads)
    return prim, t


def constraint(osc: Scene, n, type_, xD, xL, prims, pos, offsets=None):
    """Residual C (2n) and dense Jacobian J (2n x 2n) w.r.t. local offsets; frames (n, 2, 3)."""
    Cv = np.zeros(2 * n)
    J = np.zeros((2 * n, 2 * n))
    fr = np.zeros((n, 2, 3))
    rc = lib().orc_constraint(osc.h, n, type_, _p(_c(xD, np.float64)), _p(_c(xL, np.float64)),
                              _p(_c(prims, np.int32)), _p(_c(pos, np.float64).reshape(-1)), _p(Cv), _p(J), _p(fr),
                              _p(None if offsets is None else _c(offsets, np.float64).reshape(-1)))
    if rc != 0:
        raise ValueError("invalid chain")
    return Cv, J, fr


def offset_positions(osc: Scene, prims, pos, y):
    n = len(prims)
    out = np.zeros((n, 3))
    lib().orc_offset_positions(osc.h, n, _p(_c(prims, np.int32)), _p(_c(pos, np.float64).reshape(-1)),
                               _p(_c(y, np.float64)), _p(out))
    return out


class Guide:
    """Guide parameters on the host: grid bounds, per-cell validity and the
    8-component mixtures (weights, means, covariances)."""

    def __init__(self, lo, hi, res, comps, target_obj, valid, pi, mu, cov, count=None):
        self.lo = np.asarray(lo, np.float64)
        self.hi = np.asarray(hi, np.float64)
        self.res, self.comps, self.target_obj = int(res), int(comps), int(target_obj)
        self.valid = _c(valid, np.int32)
        self.pi = _c(pi, np.float64)
        self.mu = _c(mu, np.float64)
        self.cov = _c(cov, np.float64)
        self.count = count

    def chol(self):
        a, b, c = self.cov[..., 0], self.cov[..., 1], self.cov[..., 2]
        l00 = np.sqrt(np.maximum(a, 0))
        l10 = np.where(l00 > 0, b / np.where(l00 > 0, l00, 1), 0)
        l11 = np.sqrt(np.maximum(c - l10 * l10, 0))
        return np.stack([l00, l10, l11], -1)

    def packed(self):
        gi = _c(np.concatenate([[self.res, self.comps, self.target_obj], self.valid.reshape(-1)]), np.int32)
        gd = _c(np.concatenate([self.lo, self.hi, self.pi.reshape(-1), self.mu.reshape(-1),
                                self.chol().reshape(-1)]), np.float64)
        return gi, gd


def _guide_args(guide):
    if guide is None:
        return None, None, None
    gi, gd = guide.packed()
    return gi, gd, (gi, gd)


def _off(offsets):
    return None if offsets is None else _c(offsets, np.float64)


def sample_offsets(N, seed=0, trial=0, roughness=0.1):
    """GGX offset normals (o_s, o_t) of glossy chains, [2][K][N] (Sec. 5.7)."""
    out = np.zeros((2, KMAX, N))
    lib().orc_sample_offsets(int(N), int(seed), int(trial), float(roughness), _p(out))
    return out


def sample_seeds(osc: Scene, ep, seed=0, trial=0, alpha=0.5, guide=None, prm=None, nthreads=0, offsets=None):
    N = ep.n
    prm = prm or params(osc.scale)
    gi, gd, keep = _guide_args(guide)
    prim = np.zeros((KMAX, N), np.int32)
    pos = np.zeros((3, KMAX, N), np.float64)
    st = np.zeros(N, np.int8)
    lib().orc_sample_seeds(osc.h, _p(gi), _p(gd), C.byref(prm), N, _p(_c(ep.xD, np.float64)),
                           _p(_c(ep.nD, np.float64)), _p(_c(ep.length, np.uint8)), _p(_c(ep.types, np.uint8)), _p(_c(ep.obj1, np.int32)),
                           int(seed), int(trial), float(alpha), _p(prim), _p(pos), _p(st), nthreads,
                           _p(_off(offsets)))
    return prim, pos, st


def walk(osc: Scene, ep, seed_prim, seed_pos, seed_status=None, polish=True, prm=None, nthreads=0, offsets=None):
    """Walk every chain from the given seeds (positions are taken as float32,
    widened to FP64).  Returns a dict of outputs."""
    N = ep.n
    prm = prm or params(osc.scale)
    sp = _c(seed_pos, np.float32)
    spr = _c(seed_prim, np.int32)
    ss = None if seed_status is None else _c(seed_status, np.int8)
    out = dict(prim=np.zeros((KMAX, N), np.int32), pos=np.zeros((3, KMAX, N)), status=np.zeros(N, np.int8),
               iters=np.zeros(N, np.int32), sol=np.zeros(N, np.uint64), G=np.zeros(N), kappa=np.zeros(N),
               residual=np.zeros(N), polished=np.zeros(N, np.int8))
    lib().orc_walk(osc.h, C.byref(prm), N, _p(_c(ep.xD, np.float64)), _p(_c(ep.nD, np.float64)),
                   _p(_c(ep.xL, np.float64)), _p(_c(ep.length, np.uint8)), _p(_c(ep.types, np.uint8)), _p(spr),
                   _p(sp), _p(ss), int(polish), _p(out["prim"]), _p(out["pos"]), _p(out["status"]),
                   _p(out["iters"]), _p(out["sol"]), _p(out["G"]), _p(out["kappa"]), _p(out["residual"]),
                   _p(out["polished"]), nthreads, _p(_off(offsets)))
    return out


def validate(osc: Scene, ep, prim, pos, prm=None, nthreads=0, offsets=None):
    """FP64 admissibility of given chains (e.g. the GPU's converged chains):
    polish from the given vertices, then side and visibility tests.  Returns
    a dict of per-chain arrays: ok, residual, moved, side, visible,
    same_prims."""
    N = ep.n
    prm = prm or params(osc.scale)
    out = dict(ok=np.zeros(N, np.int8), residual=np.zeros(N), moved=np.zeros(N), side=np.zeros(N, np.int8),
               visible=np.zeros(N, np.int8), same_prims=np.zeros(N, np.int8))
    lib().orc_validate(osc.h, C.byref(prm), N, _p(_c(ep.xD, np.float64)), _p(_c(ep.xL, np.float64)),
                       _p(_c(ep.length, np.uint8)), _p(_c(ep.types, np.uint8)), _p(_c(prim, np.int32)),
                       _p(_c(pos, np.float64)), _p(out["ok"]), _p(out["residual"]), _p(out["moved"]),
                       _p(out["side"]), _p(out["visible"]), _p(out["same_prims"]), nthreads, _p(_off(offsets)))
    return out


def inv_prob(osc: Scene, ep, tgt_prim, tgt_pos, tgt_status, max_trials=64, repeats=1, seed=0, alpha=0.5,
             guide=None, prm=None, nthreads=0, offsets=None):
    N = ep.n
    prm = prm or params(osc.scale)
    gi, gd, keep = _guide_args(guide)
    trials = np.zeros(N, np.int32)
    ip = np.zeros(N)
    tr = np.zeros(N, np.int8)
    lib().orc_inv_prob(osc.h, _p(gi), _p(gd), C.byref(prm), N, _p(_c(ep.xD, np.float64)),
                       _p(_c(ep.nD, np.float64)), _p(_c(ep.xL, np.float64)), _p(_c(ep.length, np.uint8)), _p(_c(ep.types, np.uint8)),
                       _p(_c(ep.obj1, np.int32)), _p(_c(tgt_prim, np.int32)), _p(_c(tgt_pos, np.float64)),
                       _p(_c(tgt_status, np.int8)), int(max_trials), int(repeats), int(seed), float(alpha),
                       _p(trials), _p(ip), _p(tr), nthreads, _p(_off(offsets)))
    return trials, ip, tr


def fit_guide(samples, lo, hi, res=32, comps=8, iters=30, min_samples=16, reg=None, scale=4.0, target_obj=0,
              nthreads=0):
    """Weighted EM per cell.  ``samples`` is float32 [M, 8]: x_D (3), u, v, w, 0, 0."""
    s = _c(samples, np.float32)
    M = s.shape[0]
    cells = res ** 3
    reg = 1e-6 * scale * scale if reg is None else reg
    valid = np.zeros(cells, np.int32)
    pi = np.zeros((cells, comps))
    mu = np.zeros((cells, comps, 2))
    cov = np.zeros((cells, comps, 3))
    count = np.zeros(cells, np.int32)
    lib().orc_fit_guide(M, _p(s), res, comps, iters, min_samples, _p(_c(lo, np.float64)), _p(_c(hi, np.float64)),
                        float(reg), _p(valid), _p(pi), _p(mu), _p(cov), _p(count), nthreads)
    return Guide(lo, hi, res, comps, target_obj, valid, pi, mu, cov, count)


def adjoint(osc: Scene, ep, prim, pos, status, grad_pos, grad_G, theta=None, prm=None, nthreads=0):
    """Per-chain gradients of l = sum_i grad_pos_i . x_i + grad_G * G over
    converged chains (forward implicit-function-theorem form in FP64).

    Returns (grad_xD [3, N], grad_xL [3, N], grad_theta [N, P], ok [N])."""
    N = ep.n
    prm = prm or params(osc.scale)
    P = osc.n_theta()
    th = _c(np.zeros(0) if theta is None else theta, np.float64)
    if theta is None and P:
        th = _c([v for hf in osc.src.heightfields for ap in zip(hf.amp, hf.phase) for v in ap], np.float64)
    gxD = np.zeros((3, N))
    gxL = np.zeros((3, N))
    gth = np.zeros((N, max(P, 1)))
    ok = np.zeros(N, np.int8)
    gp = None if grad_pos is None else _c(grad_pos, np.float64)
    gg = None if grad_G is None else _c(grad_G, np.float64)
    lib().orc_adjoint(osc.h, C.byref(prm), N, _p(_c(ep.xD, np.float64)), _p(_c(ep.nD, np.float64)),
                      _p(_c(ep.xL, np.float64)), _p(_c(ep.length, np.uint8)), _p(_c(ep.types, np.uint8)),
                      _p(_c(prim, np.int32)), _p(_c(pos, np.float64)), _p(_c(status, np.int8)), _p(gp), _p(gg),
                      _p(th), _p(gxD), _p(gxL), _p(gth), _p(ok), nthreads)
    return gxD, gxL, gth[:, :P], ok


# ---------------------------------------------------------------------------
# the paper's guide: 6-D tree over (x_D, x_L), per-leaf length / type
# histograms and vMF lobes (Sec. 5.5, 5.6)
# ---------------------------------------------------------------------------

def _declare_stree(L):
    L.orc_stree_build.restype = P
    L.orc_stree_build.argtypes = [C.c_int, P, P, P, D, D, C.c_int, D, D]
    L.orc_stree_destroy.argtypes = [P]
    L.orc_stree_set_prior.argtypes = [P, P, D, D]
    L.orc_stree_n_nodes.restype = C.c_int
    L.orc_stree_n_nodes.argtypes = [P]
    L.orc_stree_n_lobes.restype = C.c_int
    L.orc_stree_n_lobes.argtypes = [P]
    L.orc_stree_nodes.argtypes = [P] + [P] * 12
    L.orc_stree_node_entries.restype = C.c_int
    L.orc_stree_node_entries.argtypes = [P, C.c_int, P, P]
    L.orc_stree_lobes.argtypes = [P, P, P, P, P, P]
    L.orc_stree_lookup.argtypes = [P, C.c_int, P, P, P]
    L.orc_vmf_pdf.restype = D
    L.orc_vmf_pdf.argtypes = [P, D, P]
    L.orc_vmf_sample.argtypes = [P, D, C.c_int, P, P]
    L.orc_stree_sample_seeds.argtypes = [P, P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, U64, U64, P, P, P, P,
                                         P, P, C.c_int]
    L.orc_stree_inv_prob.argtypes = [P, P, C.POINTER(orc_params), C.c_int, P, P, P, P, P, P, P, P, P, C.c_int,
                                     C.c_int, U64, P, P, P, P, C.c_int]


def sample_records(xD, xL, wD, w, n, types):
    """Pack sub-path samples into [N, 16] float32 records:
    x_D (3), x_L (3), w_D (3), w, n, tau, 0 x 4."""
    N = len(w)
    r = np.zeros((N, 16), np.float32)
    r[:, 0:3] = xD
    r[:, 3:6] = xL
    r[:, 6:9] = wD
    r[:, 9] = w
    r[:, 10] = n
    r[:, 11] = types
    return r


class STree:
    """The paper's guide built from sample records (see sample_records)."""

    def __init__(self, records, lo, hi, eps=0.1, thr_scale=1.0, max_depth=20, sigma_min=1e-3, sigma_lone=0.1,
                 p0n=None, alpha=0.5, p_transmit=0.5):
        L = lib()
        if not hasattr(L, "_stree_declared"):
            _declare_stree(L)
            L._stree_declared = True
        self.rec = _c(records, np.float32).reshape(-1, 16)
        self.lo = _c(lo, np.float64)
        self.hi = _c(hi, np.float64)
        self.h = L.orc_stree_build(len(self.rec), _p(self.rec), _p(self.lo), _p(self.hi), float(eps),
                                   float(thr_scale), int(max_depth), float(sigma_min), float(sigma_lone))
        self.set_prior(np.full(8, 1.0 / 8) if p0n is None else p0n, alpha, p_transmit)

    def set_prior(self, p0n, alpha=0.5, p_transmit=0.5):
        self.p0n = _c(p0n, np.float64)
        self.alpha, self.p_transmit = float(alpha), float(p_transmit)
        lib().orc_stree_set_prior(self.h, _p(self.p0n), self.alpha, self.p_transmit)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_stree_destroy(self.h)
            self.h = None

    def nodes(self):
        n = lib().orc_stree_n_nodes(self.h)
        d = dict(axis=np.zeros(n, np.int32), mid=np.zeros(n), child=np.zeros(n, np.int32),
                 depth=np.zeros(n, np.int32), lo=np.zeros((n, 6)), hi=np.zeros((n, 6)),
                 n_entries=np.zeros(n, np.int32), n_own=np.zeros(n, np.int32), W=np.zeros(n),
                 Wn=np.zeros((n, 8)), n_groups=np.zeros(n, np.int32), lobe0=np.zeros(n, np.int32))
        lib().orc_stree_nodes(self.h, *[_p(d[k]) for k in ("axis", "mid", "child", "depth", "lo", "hi", "n_entries",
                                                           "n_own", "W", "Wn", "n_groups", "lobe0")])
        return d

    def node_entries(self, k, count):
        ids = np.zeros(max(1, count), np.int32)
        own = np.zeros(max(1, count), np.int8)
        m = lib().orc_stree_node_entries(self.h, int(k), _p(ids), _p(own))
        return ids[:m], own[:m]

    def lobes(self):
        m = lib().orc_stree_n_lobes(self.h)
        d = dict(mu=np.zeros((m, 3)), kappa=np.zeros(m), w=np.zeros(m), n=np.zeros(m, np.int32),
                 type=np.zeros(m, np.int32))
        lib().orc_stree_lobes(self.h, *[_p(d[k]) for k in ("mu", "kappa", "w", "n", "type")])
        return d

    def lookup(self, xD, xL):
        xD = _c(xD, np.float64)
        xL = _c(xL, np.float64)
        N = xD.shape[1]
        out = np.zeros(N, np.int32)
        lib().orc_stree_lookup(self.h, N, _p(xD), _p(xL), _p(out))
        return out


def vmf_pdf(mu, kappa, w):
    L = lib()
    if not hasattr(L, "_stree_declared"):
        _declare_stree(L)
        L._stree_declared = True
    return L.orc_vmf_pdf(_p(_c(mu, np.float64)), float(kappa), _p(_c(w, np.float64)))


def vmf_sample(mu, kappa, u):
    L = lib()
    if not hasattr(L, "_stree_declared"):
        _declare_stree(L)
        L._stree_declared = True
    u = _c(u, np.float64).reshape(-1, 2)
    out = np.zeros((len(u), 3))
    L.orc_vmf_sample(_p(_c(mu, np.float64)), float(kappa), len(u), _p(u), _p(out))
    return out


def stree_sample_seeds(osc: Scene, st: STree, ep, seed=0, trial=0, n_fixed=None, prm=None, nthreads=0):
    """Seeds from the paper's guide; returns (n, type, P(n), prim, pos, status)."""
    N = ep.n
    prm = prm or params(osc.scale)
    n_out = np.zeros(N, np.uint8)
    t_out = np.zeros(N, np.uint8)
    pn = np.zeros(N)
    prim = np.zeros((KMAX, N), np.int32)
    pos = np.zeros((3, KMAX, N))
    status = np.zeros(N, np.int8)
    nf = None if n_fixed is None else _c(n_fixed, np.uint8)
    lib().orc_stree_sample_seeds(osc.h, st.h, C.byref(prm), N, _p(_c(ep.xD, np.float64)), _p(_c(ep.nD, np.float64)),
                                 _p(_c(ep.xL, np.float64)), _p(nf), _p(_c(ep.obj1, np.int32)), int(seed), int(trial),
                                 _p(n_out), _p(t_out), _p(pn), _p(prim), _p(pos), _p(status), nthreads)
    return n_out, t_out, pn, prim, pos, status


def stree_inv_prob(osc: Scene, st: STree, ep, length, types, tgt_prim, tgt_pos, tgt_status, max_trials=64,
                   repeats=1, seed=0, prm=None, nthreads=0):
    """Reciprocal probability with the paper's guide; returns (trials, inv_prob = K / P(n), truncated, P(n))."""
    N = ep.n
    prm = prm or params(osc.scale)
    trials = np.zeros(N, np.int32)
    ip = np.zeros(N)
    tr = np.zeros(N, np.int8)
    pn = np.zeros(N)
    lib().orc_stree_inv_prob(osc.h, st.h, C.byref(prm), N, _p(_c(ep.xD, np.float64)), _p(_c(ep.nD, np.float64)),
                             _p(_c(ep.xL, np.float64)), _p(_c(length, np.uint8)), _p(_c(types, np.uint8)),
                             _p(_c(ep.obj1, np.int32)), _p(_c(tgt_prim, np.int32)), _p(_c(tgt_pos, np.float64)),
                             _p(_c(tgt_status, np.int8)), int(max_trials), int(repeats), int(seed), _p(trials), _p(ip),
                             _p(tr), _p(pn), nthreads)
    return trials, ip, tr, pn
