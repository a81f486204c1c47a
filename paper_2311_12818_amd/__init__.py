"""Python binding of libmpg (MI355X batched manifold walks).

Thin ctypes marshalling over the C ABI in ``include/mpg.h``: every step of the
path runs in the HIP library; PyTorch provides device memory and the stream.
The binding refuses to run without the built library (no CPU fallback).

Names follow the C ABI: :func:`sample_seeds`, :func:`manifold_walk_batch`,
:func:`estimate_inv_prob`, :func:`fit_guide`, :func:`manifold_walk_adjoint`.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpg.so")
KMAX = 8
PRIM_NONE = -2 ** 31

CONVERGED, MAX_ITER, SINGULAR, SIDE_INVALID, OCCLUDED, SEED_INVALID, FP64_REJECT, BAD_INPUT, NEEDS_FP64 = range(9)
STATUS_NAMES = ["converged", "max_iter", "singular", "side_invalid", "occluded", "seed_invalid", "fp64_reject",
                "bad_input"]
FORM_PLAIN, FORM_PERSISTENT = 0, 1
OK, ERR_INVALID_ARG, ERR_HIP, ERR_OOM, ERR_UNSUPPORTED = 0, -1, -2, -3, -4
P0_ANY_OBJECT, P0_DIRECTION = -1, -2

_lib = None


class MPGError(RuntimeError):
    pass


P = C.c_void_p
I32 = C.c_int32
F32 = C.c_float
U32 = C.c_uint32


class mpg_heightfield(C.Structure):
    _fields_ = [("obj", I32), ("res", I32), ("first_vert", I32), ("first_tri", I32), ("n_sines", I32),
                ("x0", F32), ("x1", F32), ("y0", F32), ("y1", F32), ("z0", F32),
                ("amp", F32 * 8), ("freq", F32 * 8), ("psi", F32 * 8), ("phase", F32 * 8)]


class mpg_scene_desc(C.Structure):
    _fields_ = [("n_verts", I32), ("verts", P), ("normals", P), ("n_tris", I32), ("tris", P), ("tri_obj", P),
                ("n_objects", I32), ("obj_material", P), ("obj_ior", P), ("n_spheres", I32), ("spheres", P),
                ("sphere_obj", P), ("scale", F32), ("n_heightfields", I32), ("heightfields", P)]


class mpg_endpoints(C.Structure):
    _fields_ = [("N", I32), ("d_xD", P), ("d_nD", P), ("d_xL", P), ("d_len", P), ("d_type", P), ("d_obj1", P),
                ("d_offset", P)]


class mpg_chains(C.Structure):
    _fields_ = [("d_prim", P), ("d_pos", P)]


class mpg_walk_out(C.Structure):
    _fields_ = [("d_status", P), ("d_iters", P), ("d_solution_id", P), ("d_G", P), ("d_kappa", P),
                ("d_residual", P)]


class mpg_walk_params(C.Structure):
    _fields_ = [("max_iter", I32), ("tol_vertex", F32), ("tol_residual", F32), ("scale", F32), ("tmin_rel", F32),
                ("match_rel", F32), ("fp64_cond_threshold", F32), ("fp64_graze_cos", F32), ("cone_cos", F32), ("form", I32),
                ("bucketing", I32), ("waves_per_group", I32), ("stack_depth", I32), ("refill", I32),
                ("max_len", I32), ("defer_fp64", I32), ("length_order", U32)]


class mpg_guide_desc(C.Structure):
    _fields_ = [("lo", F32 * 3), ("hi", F32 * 3), ("res", I32), ("comps", I32), ("em_iters", I32),
                ("min_samples", I32), ("reg", F32), ("target_obj", I32)]


def lib():
    """Load libmpg.so; raise if it has not been built (there is no fallback).
    torch is imported first: with the library's HIP runtime initialised
    before torch's, the library found no device on the GPU host."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise MPGError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        L.mpg_last_error.restype = C.c_char_p
        L.mpg_version.restype = C.c_char_p
        L.mpg_scene_create.argtypes = [C.POINTER(mpg_scene_desc), C.POINTER(P)]
        L.mpg_scene_destroy.argtypes = [P]
        L.mpg_scene_set_params.argtypes = [P, P, I32, P]
        L.mpg_scene_params_error.argtypes = [P, P, P]
        L.mpg_scene_stats.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]
        L.mpg_walk_params_default.argtypes = [F32, C.POINTER(mpg_walk_params)]
        L.mpg_workspace_create.argtypes = [I32, C.POINTER(P)]
        L.mpg_workspace_destroy.argtypes = [P]
        L.mpg_guide_create.argtypes = [C.POINTER(mpg_guide_desc), C.POINTER(P)]
        L.mpg_guide_destroy.argtypes = [P]
        L.mpg_guide_upload.argtypes = [P, P, P, P, P]
        L.mpg_guide_download.argtypes = [P, P, P, P, P, P]
        L.sample_seeds.argtypes = [P, P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints), C.c_uint64,
                                   C.c_uint32, F32, C.POINTER(mpg_chains), P, P, P]
        L.manifold_walk_batch.argtypes = [P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints),
                                          C.POINTER(mpg_chains), P, C.POINTER(mpg_chains), C.POINTER(mpg_walk_out),
                                          P, P]
        L.estimate_inv_prob.argtypes = [P, P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints),
                                        C.POINTER(mpg_chains), P, I32, I32, C.c_uint64, F32, P, P, P, P, P]
        L.fit_guide.argtypes = [P, P, I32, P, P, P]
        L.make_guide_samples.argtypes = [C.POINTER(mpg_endpoints), C.POINTER(mpg_chains), P, P, P, P, P, P]
        L.manifold_walk_batch_noalloc.argtypes = [P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints),
                                                  C.POINTER(mpg_chains), P, C.POINTER(mpg_chains),
                                                  C.POINTER(mpg_walk_out), P]
        L.manifold_walk_fp64.argtypes = [P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints),
                                         C.POINTER(mpg_chains), C.POINTER(mpg_walk_out), P]
        L.mpg_walk_count.argtypes = [P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints), C.POINTER(mpg_chains),
                                     P, C.POINTER(mpg_chains), C.POINTER(mpg_walk_out), P, P]
        L.manifold_walk_adjoint.argtypes = [P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints),
                                            C.POINTER(mpg_chains), P, P, P, P, P, P, P, P]
        for name in ["mpg_scene_create", "mpg_scene_stats", "mpg_walk_params_default", "mpg_workspace_create",
                     "mpg_guide_create", "mpg_guide_upload", "mpg_guide_download", "sample_seeds",
                     "manifold_walk_batch", "estimate_inv_prob", "fit_guide", "manifold_walk_adjoint",
                     "manifold_walk_fp64", "mpg_walk_count", "make_guide_samples", "mpg_scene_set_params",
                     "mpg_scene_params_error", "manifold_walk_batch_noalloc"]:
            getattr(L, name).restype = I32
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise MPGError(f"{what} failed ({rc}): {lib().mpg_last_error().decode()}")


def version() -> str:
    return lib().mpg_version().decode()


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(a, dtype=None, device="cuda"):
    torch = _torch()
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device).contiguous()


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class Scene:
    """Device scene built from a ``workloads.Scene`` (host arrays)."""

    def __init__(self, sc):
        L = lib()
        self._keep = [np.ascontiguousarray(sc.verts, np.float32), np.ascontiguousarray(sc.normals, np.float32),
                      np.ascontiguousarray(sc.tris, np.int32), np.ascontiguousarray(sc.tri_obj, np.int32),
                      np.ascontiguousarray(sc.obj_material, np.int32), np.ascontiguousarray(sc.obj_ior, np.float32),
                      np.ascontiguousarray(sc.spheres, np.float32).reshape(-1),
                      np.ascontiguousarray(sc.sphere_obj, np.int32)]
        hfs = (mpg_heightfield * max(1, len(sc.heightfields)))()
        for k, hf in enumerate(sc.heightfields):
            h = hfs[k]
            h.obj, h.res, h.first_vert, h.first_tri, h.n_sines = hf.obj, hf.res, hf.first_vert, hf.first_tri, len(hf.amp)
            h.x0, h.x1, h.y0, h.y1, h.z0 = hf.x0, hf.x1, hf.y0, hf.y1, hf.z0
            for j in range(len(hf.amp)):
                h.amp[j], h.freq[j], h.psi[j], h.phase[j] = hf.amp[j], hf.freq[j], hf.psi[j], hf.phase[j]
        self._hfs = hfs
        v, n, t, to, m, io, s, so = self._keep
        d = mpg_scene_desc(v.shape[0], v.ctypes.data, n.ctypes.data, t.shape[0], t.ctypes.data, to.ctypes.data,
                           m.shape[0], m.ctypes.data, io.ctypes.data, so.shape[0], s.ctypes.data, so.ctypes.data,
                           float(sc.scale), len(sc.heightfields), C.cast(hfs, C.c_void_p))
        h = P()
        _check(L.mpg_scene_create(C.byref(d), C.byref(h)), "mpg_scene_create")
        self.h = h
        self.scale = float(sc.scale)
        self.n_params = 2 * sum(len(hf.amp) for hf in sc.heightfields)
        self.src = sc

    def set_params(self, theta):
        """New height-field parameters (device float tensor [n_params]); see
        mpg_scene_set_params."""
        torch = _torch()
        th = theta.detach().to(device="cuda", dtype=torch.float32).contiguous()
        _check(lib().mpg_scene_set_params(self.h, th.data_ptr(), int(th.numel()), _stream()), "mpg_scene_set_params")
        self._theta_keep = th   # stays alive until the queued update has read it

    def params_error(self):
        """The scene's device error word after the last set_params (int32
        device tensor of one element, read in stream order): 0 when theta was
        valid, MPG_ERR_INVALID_ARG when it held a non-finite value and the
        scene was left unchanged."""
        torch = _torch()
        out = torch.empty(1, dtype=torch.int32, device="cuda")
        _check(lib().mpg_scene_params_error(self.h, out.data_ptr(), _stream()), "mpg_scene_params_error")
        return out

    def stats(self):
        a, b, c = I32(), I32(), I32()
        _check(lib().mpg_scene_stats(self.h, C.byref(a), C.byref(b), C.byref(c)), "mpg_scene_stats")
        return dict(n_nodes=a.value, max_depth=b.value, n_tris=c.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mpg_scene_destroy(self.h)
            self.h = None


class Workspace:
    def __init__(self, max_chains: int):
        h = P()
        _check(lib().mpg_workspace_create(int(max_chains), C.byref(h)), "mpg_workspace_create")
        self.h = h
        self.cap = int(max_chains)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mpg_workspace_destroy(self.h)
            self.h = None


class Guide:
    def __init__(self, lo, hi, res=32, comps=8, em_iters=30, min_samples=16, reg=None, scale=4.0, target_obj=0):
        reg = 1e-6 * scale * scale if reg is None else reg
        self.desc = mpg_guide_desc((F32 * 3)(*lo), (F32 * 3)(*hi), res, comps, em_iters, min_samples, reg,
                                   target_obj)
        h = P()
        _check(lib().mpg_guide_create(C.byref(self.desc), C.byref(h)), "mpg_guide_create")
        self.h = h
        self.res, self.comps, self.cells = res, comps, res ** 3

    def upload(self, valid, pi, mu, cov):
        a = [np.ascontiguousarray(valid, np.int32), np.ascontiguousarray(pi, np.float32),
             np.ascontiguousarray(mu, np.float32), np.ascontiguousarray(cov, np.float32)]
        _check(lib().mpg_guide_upload(self.h, *[x.ctypes.data for x in a]), "mpg_guide_upload")

    def download(self):
        C_, K = self.cells, self.comps
        valid = np.zeros(C_, np.int32)
        pi = np.zeros((C_, K), np.float32)
        mu = np.zeros((C_, K, 2), np.float32)
        cov = np.zeros((C_, K, 3), np.float32)
        count = np.zeros(C_, np.int32)
        _check(lib().mpg_guide_download(self.h, valid.ctypes.data, pi.ctypes.data, mu.ctypes.data, cov.ctypes.data,
                                        count.ctypes.data), "mpg_guide_download")
        return dict(valid=valid, pi=pi, mu=mu, cov=cov, count=count)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mpg_guide_destroy(self.h)
            self.h = None


def pack_length_order(lengths) -> int:
    """The ``length_order`` word of a launch order of the lengths 1..8 (the
    first length in the lowest nibble)."""
    lengths = [int(n) for n in lengths]
    if sorted(lengths) != list(range(1, 9)):
        raise ValueError("length order must hold every length 1..8 once")
    return sum(n << (4 * k) for k, n in enumerate(lengths))


def walk_params(scale: float, **kw) -> mpg_walk_params:
    """Defaults for a scene of scale ``scale`` with fields overridden by ``kw``
    (``length_order`` may be given as a list of the lengths 1..8)."""
    p = mpg_walk_params()
    _check(lib().mpg_walk_params_default(float(scale), C.byref(p)), "mpg_walk_params_default")
    for k, v in kw.items():
        if k == "length_order" and isinstance(v, (list, tuple)):
            v = pack_length_order(v)
        setattr(p, k, v)
    return p


class Endpoints:
    """Device copy of a ``workloads.Endpoints`` batch."""

    def __init__(self, ep, device="cuda"):
        torch = _torch()
        self.N = ep.n
        self.xD = _dev(ep.xD, torch.float32, device)
        self.nD = _dev(ep.nD, torch.float32, device)
        self.xL = _dev(ep.xL, torch.float32, device)
        self.len = _dev(ep.length, torch.uint8, device)
        self.type = _dev(ep.types, torch.uint8, device)
        self.obj1 = _dev(ep.obj1, torch.int32, device)
        self.off = None   # glossy offset normals [2][K][N] (float32 device tensor), see sample_offsets

    @classmethod
    def from_tensors(cls, xD, nD, xL, length, types, obj1):
        """Wrap device tensors ([3][N] float32 points / normal, [N] uint8
        lengths and types, [N] int32 p_0 objects) without copying."""
        self = cls.__new__(cls)
        self.N = int(length.shape[0])
        self.xD, self.nD, self.xL = xD.contiguous(), nD.contiguous(), xL.contiguous()
        self.len, self.type, self.obj1 = length.contiguous(), types.contiguous(), obj1.contiguous()
        self.off = None
        for t, dt in ((self.xD, "float32"), (self.nD, "float32"), (self.xL, "float32"), (self.len, "uint8"),
                      (self.type, "uint8"), (self.obj1, "int32")):
            if str(t.dtype) != "torch." + dt or not t.is_cuda:
                raise MPGError(f"Endpoints.from_tensors: expected a device tensor of {dt}, got {t.dtype}")
        return self

    def c(self) -> mpg_endpoints:
        return mpg_endpoints(self.N, self.xD.data_ptr(), self.nD.data_ptr(), self.xL.data_ptr(),
                             self.len.data_ptr(), self.type.data_ptr(), self.obj1.data_ptr(),
                             self.off.data_ptr() if self.off is not None else None)


def empty_chains(N, device="cuda"):
    torch = _torch()
    return (torch.full((KMAX, N), PRIM_NONE, dtype=torch.int32, device=device),
            torch.zeros((3, KMAX, N), dtype=torch.float32, device=device))


# ---------------------------------------------------------------------------
# hot path
# ---------------------------------------------------------------------------

def sample_seeds(scene: Scene, ep: Endpoints, params: mpg_walk_params, seed=0, trial=0, alpha=0.5,
                 guide: Optional[Guide] = None, out=None, ws: Optional[Workspace] = None, status=None):
    """Seed chains; the persistent form (params.form) needs a workspace."""
    torch = _torch()
    prim, pos = out if out is not None else empty_chains(ep.N, ep.xD.device)
    st = torch.zeros(ep.N, dtype=torch.int8, device=ep.xD.device) if status is None else status
    ch = mpg_chains(prim.data_ptr(), pos.data_ptr())
    _check(lib().sample_seeds(scene.h, guide.h if guide else None, C.byref(params), C.byref(ep.c()), int(seed),
                              int(trial), float(alpha), C.byref(ch), st.data_ptr(), ws.h if ws else None,
                              _stream()), "sample_seeds")
    return prim, pos, st


def walk_outputs(N, device="cuda"):
    torch = _torch()
    return dict(status=torch.zeros(N, dtype=torch.int8, device=device),
                iters=torch.zeros(N, dtype=torch.uint8, device=device),
                sol=torch.zeros(N, dtype=torch.int64, device=device),
                G=torch.zeros(N, dtype=torch.float32, device=device),
                kappa=torch.zeros(N, dtype=torch.float32, device=device),
                residual=torch.zeros(N, dtype=torch.float32, device=device))


def manifold_walk_batch(scene: Scene, params: mpg_walk_params, ep: Endpoints, seed_prim, seed_pos,
                        seed_status=None, out_prim=None, out_pos=None, outs=None, ws: Optional[Workspace] = None):
    """Walks every chain.  Returns (prim, pos, outputs dict).  out_* may alias the seeds."""
    if out_prim is None:
        out_prim, out_pos = empty_chains(ep.N, ep.xD.device)
    outs = outs if outs is not None else walk_outputs(ep.N, ep.xD.device)
    seeds = mpg_chains(seed_prim.data_ptr(), seed_pos.data_ptr())
    oc = mpg_chains(out_prim.data_ptr(), out_pos.data_ptr())
    wo = mpg_walk_out(outs["status"].data_ptr(), outs["iters"].data_ptr(), outs["sol"].data_ptr(),
                      outs["G"].data_ptr(), outs["kappa"].data_ptr(), outs["residual"].data_ptr())
    _check(lib().manifold_walk_batch(scene.h, C.byref(params), C.byref(ep.c()), C.byref(seeds), _ptr(seed_status),
                                     C.byref(oc), C.byref(wo), ws.h if ws else None, _stream()),
           "manifold_walk_batch")
    return out_prim, out_pos, outs


NOALLOC_MAX_CHAINS = 1 << 20


def manifold_walk_batch_noalloc(scene: Scene, params: mpg_walk_params, ep: Endpoints, seed_prim, seed_pos,
                                seed_status=None, out_prim=None, out_pos=None, outs=None):
    """manifold_walk_batch without a workspace (allocation-free entry point;
    see manifold_walk_batch_noalloc in mpg.h).  The caller passes every
    input and output; returns (prim, pos, outputs dict)."""
    seeds = mpg_chains(seed_prim.data_ptr(), seed_pos.data_ptr())
    oc = mpg_chains(out_prim.data_ptr(), out_pos.data_ptr())
    _check(lib().manifold_walk_batch_noalloc(scene.h, C.byref(params), C.byref(ep.c()), C.byref(seeds),
                                             _ptr(seed_status), C.byref(oc), C.byref(_wout(outs)), _stream()),
           "manifold_walk_batch_noalloc")
    return out_prim, out_pos, outs


def sample_offsets(N, seed=0, trial=0, roughness=0.1, device="cuda"):
    """GGX offset normals of glossy chains: float32 device tensor [2][K][N]."""
    torch = _torch()
    out = torch.zeros((2, KMAX, N), dtype=torch.float32, device=device)
    L = lib()
    L.sample_offsets.argtypes = [I32, C.c_uint64, C.c_uint32, F32, P, P]
    L.sample_offsets.restype = I32
    _check(L.sample_offsets(int(N), int(seed), int(trial), float(roughness), out.data_ptr(), _stream()),
           "sample_offsets")
    return out


def _wout(outs):
    return mpg_walk_out(outs["status"].data_ptr(), outs["iters"].data_ptr(), outs["sol"].data_ptr(),
                        outs["G"].data_ptr(), outs["kappa"].data_ptr(), outs["residual"].data_ptr())


def manifold_walk_fp64(scene: Scene, params: mpg_walk_params, ep: Endpoints, prim, pos, outs):
    """FP64 pass over chains left as NEEDS_FP64 by a deferred walk (in place)."""
    ch = mpg_chains(prim.data_ptr(), pos.data_ptr())
    _check(lib().manifold_walk_fp64(scene.h, C.byref(params), C.byref(ep.c()), C.byref(ch), C.byref(_wout(outs)),
                                    _stream()), "manifold_walk_fp64")
    return prim, pos, outs


COUNT_NAMES = ["box_tests", "tri_tests", "sphere_tests", "rays", "vertex_residual_evals", "vertex_jacobian_evals",
               "vertex_jacobian_evals_fp64", "chains"]


def walk_count(scene: Scene, params: mpg_walk_params, ep: Endpoints, seed_prim, seed_pos, seed_status=None):
    """Untimed counting walk: returns (prim, pos, outputs, work tallies dict)."""
    torch = _torch()
    out_prim, out_pos = empty_chains(ep.N, ep.xD.device)
    outs = walk_outputs(ep.N, ep.xD.device)
    counts = torch.zeros(8, dtype=torch.int64, device=ep.xD.device)
    seeds = mpg_chains(seed_prim.data_ptr(), seed_pos.data_ptr())
    oc = mpg_chains(out_prim.data_ptr(), out_pos.data_ptr())
    _check(lib().mpg_walk_count(scene.h, C.byref(params), C.byref(ep.c()), C.byref(seeds), _ptr(seed_status),
                                C.byref(oc), C.byref(_wout(outs)), counts.data_ptr(), _stream()), "mpg_walk_count")
    torch.cuda.synchronize()
    return out_prim, out_pos, outs, dict(zip(COUNT_NAMES, [int(v) for v in counts.cpu().tolist()]))


def estimate_inv_prob(scene: Scene, params: mpg_walk_params, ep: Endpoints, tprim, tpos, tstatus, max_trials=64,
                      repeats=1, seed=0, alpha=0.5, guide: Optional[Guide] = None, ws: Optional[Workspace] = None,
                      outs=None):
    torch = _torch()
    dev = ep.xD.device
    if outs is None:
        outs = (torch.zeros(ep.N, dtype=torch.int32, device=dev), torch.zeros(ep.N, dtype=torch.float32, device=dev),
                torch.zeros(ep.N, dtype=torch.uint8, device=dev))
    trials, inv, trunc = outs
    tc = mpg_chains(tprim.data_ptr(), tpos.data_ptr())
    _check(lib().estimate_inv_prob(scene.h, guide.h if guide else None, C.byref(params), C.byref(ep.c()),
                                   C.byref(tc), tstatus.data_ptr(), int(max_trials), int(repeats), int(seed),
                                   float(alpha), trials.data_ptr(), inv.data_ptr(), trunc.data_ptr(),
                                   ws.h if ws else None, _stream()), "estimate_inv_prob")
    return trials, inv, trunc


def make_guide_samples(ep: Endpoints, pos, outs, inv_prob):
    """Sample records [N, 8] (x_D, x, y of x_1, w = kappa G <1/P>, 0, 0) on the device."""
    torch = _torch()
    out = torch.empty((ep.N, 8), dtype=torch.float32, device=ep.xD.device)
    ch = mpg_chains(0, pos.data_ptr())
    _check(lib().make_guide_samples(C.byref(ep.c()), C.byref(ch), outs["status"].data_ptr(), outs["G"].data_ptr(),
                                    outs["kappa"].data_ptr(), inv_prob.data_ptr(), out.data_ptr(), _stream()),
           "make_guide_samples")
    return out


def fit_guide(scene: Scene, samples, guide: Guide, ws: Workspace):
    """samples: float32 device tensor [M, 8] (x_D, u, v, w, 0, 0)."""
    _check(lib().fit_guide(scene.h if scene is not None else None, samples.data_ptr(), int(samples.shape[0]),
                           guide.h, ws.h, _stream()), "fit_guide")
    return guide


def manifold_walk_adjoint(scene: Scene, params: mpg_walk_params, ep: Endpoints, prim, pos, status, grad_pos=None,
                          grad_G=None, grad_xD=None, grad_xL=None, grad_theta=None, ws: Optional[Workspace] = None):
    torch = _torch()
    dev = ep.xD.device
    grad_xD = torch.zeros((3, ep.N), dtype=torch.float32, device=dev) if grad_xD is None else grad_xD
    grad_xL = torch.zeros((3, ep.N), dtype=torch.float32, device=dev) if grad_xL is None else grad_xL
    if grad_theta is None:
        grad_theta = torch.zeros(max(1, scene.n_params), dtype=torch.float32, device=dev)
    ch = mpg_chains(prim.data_ptr(), pos.data_ptr())
    _check(lib().manifold_walk_adjoint(scene.h, C.byref(params), C.byref(ep.c()), C.byref(ch), status.data_ptr(),
                                       _ptr(grad_pos), _ptr(grad_G), grad_xD.data_ptr(), grad_xL.data_ptr(),
                                       grad_theta.data_ptr(), ws.h if ws else None, _stream()),
           "manifold_walk_adjoint")
    return grad_xD, grad_xL, grad_theta


# ---------------------------------------------------------------------------
# the paper's guide: 6-D tree, length / type distributions, vMF lobes
# ---------------------------------------------------------------------------

class mpg_stree_desc(C.Structure):
    _fields_ = [("lo", F32 * 6), ("hi", F32 * 6), ("eps", F32), ("thr_scale", F32), ("max_depth", I32),
                ("sigma_min", F32), ("sigma_lone", F32), ("p0n", F32 * 8), ("alpha", F32), ("p_transmit", F32)]


def _declare_stree(L):
    L.mpg_stree_desc_default.argtypes = [C.POINTER(mpg_stree_desc)]
    L.mpg_stree_create.argtypes = [C.POINTER(mpg_stree_desc), C.POINTER(P)]
    L.mpg_stree_destroy.argtypes = [P]
    L.mpg_stree_set_prior.argtypes = [P, P, F32, F32]
    L.fit_guide_stree.argtypes = [P, P, I32, P]
    L.mpg_stree_stats.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]
    L.mpg_stree_download.argtypes = [P] * 13
    L.sample_seeds_stree.argtypes = [P, P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints), C.c_uint64,
                                     C.c_uint32, P, P, P, C.POINTER(mpg_chains), P, P, P]
    L.estimate_inv_prob_stree.argtypes = [P, P, C.POINTER(mpg_walk_params), C.POINTER(mpg_endpoints),
                                          C.POINTER(mpg_chains), P, I32, I32, C.c_uint64, P, P, P, P, P, P]
    L.make_guide_records.argtypes = [C.POINTER(mpg_endpoints), C.POINTER(mpg_chains), P, P, P, P, P, P]
    L.mpg_stree_active.argtypes = [P, C.POINTER(mpg_endpoints), P, P]
    for name in ["mpg_stree_desc_default", "mpg_stree_create", "mpg_stree_set_prior", "fit_guide_stree",
                 "mpg_stree_stats", "mpg_stree_download", "sample_seeds_stree", "estimate_inv_prob_stree",
                 "make_guide_records", "mpg_stree_active"]:
        getattr(L, name).restype = I32


def _slib():
    L = lib()
    if not getattr(L, "_stree_declared", False):
        _declare_stree(L)
        L._stree_declared = True
    return L


class STree:
    """The paper's guide on the device (see the mpg_stree_* calls)."""

    def __init__(self, lo, hi, eps=0.1, thr_scale=1.0, max_depth=20, sigma_min=1e-3, sigma_lone=0.1, p0n=None,
                 alpha=0.5, p_transmit=0.5):
        L = _slib()
        d = mpg_stree_desc()
        _check(L.mpg_stree_desc_default(C.byref(d)), "mpg_stree_desc_default")
        for a in range(6):
            d.lo[a], d.hi[a] = float(lo[a]), float(hi[a])
        d.eps, d.thr_scale, d.max_depth = float(eps), float(thr_scale), int(max_depth)
        d.sigma_min, d.sigma_lone = float(sigma_min), float(sigma_lone)
        for k in range(8):
            d.p0n[k] = 1.0 / 8 if p0n is None else float(p0n[k])
        d.alpha, d.p_transmit = float(alpha), float(p_transmit)
        h = P()
        _check(L.mpg_stree_create(C.byref(d), C.byref(h)), "mpg_stree_create")
        self.h = h.value
        self.desc = d

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mpg_stree_destroy(self.h)
            self.h = None

    def set_prior(self, p0n, alpha=0.5, p_transmit=0.5):
        arr = (F32 * 8)(*[float(v) for v in p0n])
        _check(_slib().mpg_stree_set_prior(self.h, C.cast(arr, P), float(alpha), float(p_transmit)),
               "mpg_stree_set_prior")

    def fit(self, records):
        """records: float32 device tensor [M, 16] (see make_guide_records)."""
        _check(_slib().fit_guide_stree(self.h, records.data_ptr(), int(records.shape[0]), _stream()),
               "fit_guide_stree")
        return self

    def stats(self):
        v = [I32() for _ in range(4)]
        _check(_slib().mpg_stree_stats(self.h, *[C.byref(x) for x in v]), "mpg_stree_stats")
        return dict(zip(("nodes", "leaves", "groups", "lobes"), [x.value for x in v]))

    def download(self):
        import numpy as np
        s = self.stats()
        nn, ng, nl = s["nodes"], s["groups"], s["lobes"]
        d = dict(axis=np.zeros(nn, np.int32), mid=np.zeros(nn, np.float32), child=np.zeros(nn, np.int32),
                 W=np.zeros(nn, np.float32), Wn=np.zeros((nn, 8), np.float32), own=np.zeros(nn, np.int32),
                 leaf_groups=np.zeros((nn, 2), np.int32), grp_key=np.zeros(max(ng, 1), np.int32),
                 grp_w=np.zeros(max(ng, 1), np.float32), grp_lobes=np.zeros((max(ng, 1), 2), np.int32),
                 lobe=np.zeros((max(nl, 1), 4), np.float32), lobe_cdf=np.zeros(max(nl, 1), np.float32))
        keys = ("axis", "mid", "child", "W", "Wn", "own", "leaf_groups", "grp_key", "grp_w", "grp_lobes", "lobe",
                "lobe_cdf")
        _check(_slib().mpg_stree_download(self.h, *[d[k].ctypes.data_as(P) for k in keys]), "mpg_stree_download")
        for k in ("grp_key", "grp_w", "grp_lobes"):
            d[k] = d[k][:ng]
        for k in ("lobe", "lobe_cdf"):
            d[k] = d[k][:nl]
        return d


def sample_seeds_stree(scene: Scene, tree: STree, ep: Endpoints, params: mpg_walk_params, seed=0, trial=0,
                       ws: Workspace = None):
    """Seeds from the paper's guide.  Returns (n, tau, P(n), prim, pos, status)
    as device tensors; ep.len holds the fixed lengths (0 = sampled).
    Persistent form: params.form = FORM_PERSISTENT with bucketing and a
    workspace."""
    torch = _torch()
    dev = ep.xD.device
    n = torch.zeros(ep.N, dtype=torch.uint8, device=dev)
    ty = torch.zeros(ep.N, dtype=torch.uint8, device=dev)
    pn = torch.zeros(ep.N, dtype=torch.float32, device=dev)
    prim, pos = empty_chains(ep.N, dev)
    st = torch.zeros(ep.N, dtype=torch.int8, device=dev)
    ch = mpg_chains(prim.data_ptr(), pos.data_ptr())
    _check(_slib().sample_seeds_stree(scene.h, tree.h, C.byref(params), C.byref(ep.c()), int(seed), int(trial),
                                      n.data_ptr(), ty.data_ptr(), pn.data_ptr(), C.byref(ch), st.data_ptr(),
                                      ws.h if ws is not None else None, _stream()), "sample_seeds_stree")
    return n, ty, pn, prim, pos, st


def estimate_inv_prob_stree(scene: Scene, tree: STree, params: mpg_walk_params, ep: Endpoints, tprim, tpos, tstatus,
                            max_trials=64, repeats=1, seed=0, ws: Workspace = None):
    """Returns (trials, inv_prob = K / P(n), truncated, P(n)) as device tensors
    (persistent form: params.form = FORM_PERSISTENT with bucketing and a
    workspace)."""
    torch = _torch()
    dev = ep.xD.device
    trials = torch.zeros(ep.N, dtype=torch.int32, device=dev)
    ip = torch.zeros(ep.N, dtype=torch.float32, device=dev)
    tr = torch.zeros(ep.N, dtype=torch.uint8, device=dev)
    pn = torch.zeros(ep.N, dtype=torch.float32, device=dev)
    ch = mpg_chains(tprim.data_ptr(), tpos.data_ptr())
    _check(_slib().estimate_inv_prob_stree(scene.h, tree.h, C.byref(params), C.byref(ep.c()), C.byref(ch),
                                           tstatus.data_ptr(), int(max_trials), int(repeats), int(seed),
                                           trials.data_ptr(), ip.data_ptr(), tr.data_ptr(), pn.data_ptr(),
                                           ws.h if ws is not None else None, _stream()),
           "estimate_inv_prob_stree")
    return trials, ip, tr, pn


def make_guide_records(ep: Endpoints, pos, outs, inv_prob):
    """Sample records [N, 16] for STree.fit on the device."""
    torch = _torch()
    out = torch.empty((ep.N, 16), dtype=torch.float32, device=ep.xD.device)
    ch = mpg_chains(0, pos.data_ptr())
    _check(_slib().make_guide_records(C.byref(ep.c()), C.byref(ch), outs["status"].data_ptr(), outs["G"].data_ptr(),
                                      outs["kappa"].data_ptr(), inv_prob.data_ptr(), out.data_ptr(), _stream()),
           "make_guide_records")
    return out


def stree_active(tree: STree, ep: Endpoints):
    """Selective activation flags (uint8 device tensor [N])."""
    torch = _torch()
    out = torch.zeros(ep.N, dtype=torch.uint8, device=ep.xD.device)
    _check(_slib().mpg_stree_active(tree.h, C.byref(ep.c()), out.data_ptr(), _stream()), "mpg_stree_active")
    return out


# ---------------------------------------------------------------------------
# progressive training schedule (Sec. 5.8)
# ---------------------------------------------------------------------------

TRAIN, RENDER = 0, 1


class mpg_train_plan(C.Structure):
    _fields_ = [("budget", C.c_double), ("train_fraction", C.c_double), ("base_samples", C.c_int64)]


class mpg_train_state(C.Structure):
    _fields_ = [("phase", I32), ("iteration", I32), ("target", C.c_int64), ("done", C.c_int64), ("refit", I32)]


def _tlib():
    L = lib()
    if not getattr(L, "_train_declared", False):
        L.mpg_train_init.argtypes = [C.POINTER(mpg_train_plan), C.POINTER(mpg_train_state)]
        L.mpg_train_step.argtypes = [C.POINTER(mpg_train_plan), C.POINTER(mpg_train_state), C.c_int64, C.c_double]
        L.mpg_train_init.restype = I32
        L.mpg_train_step.restype = I32
        L._train_declared = True
    return L


def train_init(plan: mpg_train_plan) -> mpg_train_state:
    st = mpg_train_state()
    _check(_tlib().mpg_train_init(C.byref(plan), C.byref(st)), "mpg_train_init")
    return st


def train_step(plan: mpg_train_plan, st: mpg_train_state, batch: int, elapsed: float) -> mpg_train_state:
    _check(_tlib().mpg_train_step(C.byref(plan), C.byref(st), int(batch), float(elapsed)), "mpg_train_step")
    return st
