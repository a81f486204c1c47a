"""GPU parity of seeds and manifold walks (HIP path through the C ABI) against
the FP64 oracle on identical seeded inputs."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import gpu_common as GC
from tests import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2311_12818_amd as M
    M.lib()
    return M


def run_gpu_walk(M, sc, ep, seeds_prim, seeds_pos, seed_status=None, **pkw):
    import torch
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), **pkw)
    sp = torch.as_tensor(seeds_prim).cuda()
    spos = torch.as_tensor(seeds_pos).cuda()
    sst = None if seed_status is None else torch.as_tensor(seed_status).cuda()
    ws = M.Workspace(ep.n) if pkw.get("form", 0) == M.FORM_PERSISTENT else None
    prim, pos, outs = M.manifold_walk_batch(scene, prm, dep, sp, spos, sst, ws=ws)
    torch.cuda.synchronize()
    g = {k: GC.to_np(v) for k, v in outs.items()}
    g["prim"] = GC.to_np(prim)
    g["pos"] = GC.to_np(pos).astype(np.float64)
    g["sol"] = g["sol"].view(np.uint64)
    return g


CASES = [
    ("sphere_mirror", 4096, 1),
    ("icosphere_tt", 8192, 2),
    ("water_caustic", 8192, 1),
    ("slab_uneven", 8192, 8),
    ("slab_adjoint", 4096, 4),
]


@pytest.mark.parametrize("name,n,max_len", CASES)
def test_walk_parity_on_oracle_seeds(mpg, name, n, max_len):
    scene_fn, ep_fn = W.WORKLOADS[name]
    sc = scene_fn()
    ep = ep_fn(n)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    o = O.walk(osc, ep, prim, pos, st, prm=O.params(sc.scale, cone_cos=GC.cone_cos()))
    g = run_gpu_walk(mpg, sc, ep, prim, pos, st, max_len=max_len)
    GC.compare_walks(ep, g, o, sc.scale, tag=name)
    both = (g["status"] == 0) & (o["status"] == 0) & (g["sol"] == o["sol"])
    # G and kappa within FP32 error of the FP64 values.  G = |n.w| |det dw/dA|
    # passes through J^-1 and a 2x2 determinant of two columns that are
    # nearly parallel for strongly anisotropic (near-caustic) chains, so its
    # FP32 error is ~ eps32 (cond(J) + column aspect): typically 1e-5,
    # at most a few 1e-3 for G values far below the batch median.
    rel = np.abs(g["G"][both] - o["G"][both]) / o["G"][both]
    assert np.median(rel) <= 1e-4 and np.quantile(rel, 0.99) <= 2e-3 and rel.max() <= 1e-2
    # kappa: Fresnel factors are Lipschitz in the cosines with constant
    # <= eta^2 / cos_min ~ 112 once chains within cos 0.02 of grazing are
    # finished in FP64; FP32 vertex errors <= 1e-5 over segments of length
    # >= ~5e-3 L move the cosines by <= ~2e-6 per vertex, so |d kappa| <= 5e-4
    dk = np.abs(g["kappa"][both] - o["kappa"][both])
    assert dk.max() <= 5e-4 and np.median(dk) <= 1e-5
    assert np.all(g["residual"][both] <= 1e-4)


@pytest.mark.parametrize("name,n", [("sphere_mirror", 4096), ("icosphere_tt", 8192), ("water_caustic", 8192),
                                    ("slab_uneven", 8192)])
def test_seed_parity(mpg, name, n):
    import torch
    scene_fn, ep_fn = W.WORKLOADS[name]
    sc = scene_fn()
    ep = ep_fn(n)
    osc = O.Scene(sc)
    oprim, opos, ost = GC.oracle_seeds(osc, ep)
    scene = mpg.Scene(sc)
    dep = mpg.Endpoints(ep)
    prm = mpg.walk_params(sc.scale, cone_cos=GC.cone_cos())
    prim, pos, st = mpg.sample_seeds(scene, dep, prm, seed=0, trial=0, alpha=0.5)
    torch.cuda.synchronize()
    gprim, gpos, gst = GC.to_np(prim), GC.to_np(pos), GC.to_np(st)
    ok = (gst == 0) & (ost == 0)
    agree = (gst == ost).mean()
    same = ok.copy()
    err = np.zeros(ep.n)
    for i in range(8):
        m = ep.length > i
        same &= np.where(m, gprim[i] == oprim[i], True)
        err = np.where(m, np.maximum(err, np.abs(gpos[:, i, :] - opos[:, i, :]).max(0)), err)
    # a seed matches when the status, every primitive and every vertex (within
    # 1e-4 L) agree; grazing first hits (position error ~ eps t / cos) and
    # edge hits spend the 0.1% budget
    close = same & (err <= 1e-4 * sc.scale)
    frac = (np.sum(gst != ost) + np.sum(ok & ~close)) / ep.n
    print(dict(name=name, status_agree=agree, mismatch=frac, med_err=float(np.median(err[same]))), flush=True)
    assert frac <= 1e-3
    assert np.median(err[same]) <= 1e-6 * sc.scale


def test_end_to_end_sphere_mirror_full_size(mpg):
    """GPU seeds + GPU walk on the whole 4096-configuration batch against the
    oracle's own seeds + walk."""
    import torch
    sc = W.sphere_mirror_scene()
    ep = W.sphere_mirror_endpoints(4096)
    osc = O.Scene(sc)
    oprim, opos, ost = GC.oracle_seeds(osc, ep)
    o = O.walk(osc, ep, oprim, opos, ost)
    scene = mpg.Scene(sc)
    dep = mpg.Endpoints(ep)
    prm = mpg.walk_params(sc.scale, max_len=1)
    prim, pos, st = mpg.sample_seeds(scene, dep, prm)
    prim, pos, outs = mpg.manifold_walk_batch(scene, prm, dep, prim, pos, st, out_prim=prim, out_pos=pos)
    torch.cuda.synchronize()
    g = {k: GC.to_np(v) for k, v in outs.items()}
    g["prim"], g["pos"] = GC.to_np(prim), GC.to_np(pos).astype(np.float64)
    g["sol"] = g["sol"].view(np.uint64)
    GC.compare_walks(ep, g, o, sc.scale, tag="sphere_mirror_e2e")


def test_edge_cases(mpg):
    import torch
    sc = W.icosphere_glass_scene()
    scene = mpg.Scene(sc)
    prm = mpg.walk_params(sc.scale, max_len=2)
    # empty batch: no launch, no error
    e0 = W.icosphere_endpoints(0)
    dep = mpg.Endpoints(e0)
    p0, q0 = mpg.empty_chains(0)
    mpg.manifold_walk_batch(scene, prm, dep, p0, q0)
    # ragged: 1 chain, 65 chains (one wave + 1), non-finite endpoint, bad length
    ep = W.icosphere_endpoints(65)
    ep.xD[0, 3] = np.nan
    ep.length[5] = 9
    ep.length[6] = 0
    dep = mpg.Endpoints(ep)
    prim, pos, st = mpg.sample_seeds(scene, dep, prm)
    prim, pos, outs = mpg.manifold_walk_batch(scene, prm, dep, prim, pos, st)
    torch.cuda.synchronize()
    s = GC.to_np(outs["status"])
    assert s[3] == mpg.BAD_INPUT and s[5] == mpg.BAD_INPUT and s[6] == mpg.BAD_INPUT
    # chains longer than max_len are rejected as bad input
    ep2 = W.icosphere_endpoints(64)
    prm1 = mpg.walk_params(sc.scale, max_len=1)
    dep2 = mpg.Endpoints(ep2)
    prim, pos, st = mpg.sample_seeds(scene, dep2, prm)
    prim, pos, outs = mpg.manifold_walk_batch(scene, prm1, dep2, prim, pos, st)
    torch.cuda.synchronize()
    assert np.all(GC.to_np(outs["status"]) == mpg.BAD_INPUT)
    # host-side argument errors
    with pytest.raises(mpg.MPGError):
        mpg.manifold_walk_batch(scene, mpg.walk_params(sc.scale, max_len=9), dep2, prim, pos)
    with pytest.raises(mpg.MPGError):
        mpg.manifold_walk_batch(scene, mpg.walk_params(sc.scale, waves_per_group=3), dep2, prim, pos)
    with pytest.raises(mpg.MPGError):
        mpg.manifold_walk_batch(scene, mpg.walk_params(sc.scale, stack_depth=1), dep2, prim, pos)


def test_plane_mirror_closed_form_on_gpu(mpg):
    """The HIP walk reproduces the image-point reflection on a plane."""
    sc = S.plane_scene(W.MAT_MIRROR)
    g = np.random.default_rng(2)
    N = 2048
    xD = np.stack([g.uniform(-2, 2, N), g.uniform(-2, 2, N), g.uniform(0.3, 2, N)], 1)
    xL = np.stack([g.uniform(-2, 2, N), g.uniform(-2, 2, N), g.uniform(0.5, 3, N)], 1)
    ep = S.endpoints(xD, xL, obj1=0)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    res = run_gpu_walk(mpg, sc, ep, prim, pos, st, max_len=1)
    conv = res["status"] == 0
    assert conv.mean() > 0.9
    xD64, xL64 = ep.xD.T.astype(np.float64), ep.xL.T.astype(np.float64)
    img = xL64 * np.array([1, 1, -1.0])
    t = xD64[:, 2] / (xD64[:, 2] - img[:, 2])
    x1 = xD64 + (img - xD64) * t[:, None]
    err = np.linalg.norm(res["pos"][:, 0, :].T - x1, axis=1)
    assert err[conv].max() < 1e-4 * sc.scale
    d = np.linalg.norm(img - xD64, axis=1)
    w = (x1 - xD64) / np.linalg.norm(x1 - xD64, axis=1, keepdims=True)
    Gt = np.abs(w[:, 2]) / d ** 2
    assert np.allclose(res["G"][conv], Gt[conv], rtol=1e-3)


def test_determinism(mpg):
    """Same inputs, same outputs, bit for bit (counter-based randomness, no
    order-dependent reductions in the walk)."""
    import torch
    sc = W.slab_stack_scene()
    ep = W.slab_uneven_endpoints(4096)
    scene = mpg.Scene(sc)
    dep = mpg.Endpoints(ep)
    prm = mpg.walk_params(sc.scale, cone_cos=GC.cone_cos())
    outs = []
    for _ in range(2):
        prim, pos, st = mpg.sample_seeds(scene, dep, prm)
        prim, pos, o = mpg.manifold_walk_batch(scene, prm, dep, prim, pos, st)
        torch.cuda.synchronize()
        outs.append((GC.to_np(prim), GC.to_np(pos), GC.to_np(o["status"]), GC.to_np(o["G"])))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("bucketing,waves,refill", [(1, 4, 0), (1, 1, 0), (0, 2, 0), (1, 4, 1), (1, 2, 1),
                                                   (2, 1, 1), (3, 4, 1), (2, 4, 0)])
def test_persistent_form_matches_plain_bit_for_bit(mpg, bucketing, waves, refill):
    """The persistent batched form computes every chain with the same code as
    the plain form, only scheduled differently: outputs are identical."""
    import torch
    sc = W.slab_stack_scene()
    ep = W.slab_uneven_endpoints(20000 + 37)   # ragged: not a multiple of 64
    ep.length[11] = 0                          # invalid length -> bad input
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    plain = run_gpu_walk(mpg, sc, ep, prim, pos, st)
    pers = run_gpu_walk(mpg, sc, ep, prim, pos, st, form=mpg.FORM_PERSISTENT, bucketing=bucketing,
                        waves_per_group=waves, refill=refill)
    for k in ("status", "iters", "sol", "G", "kappa", "residual"):
        assert np.array_equal(plain[k], pers[k]), k
    ok = plain["status"] != mpg.BAD_INPUT
    assert np.array_equal(plain["prim"][:, ok], pers["prim"][:, ok])
    assert np.array_equal(plain["pos"][:, :, ok], pers["pos"][:, :, ok])
    assert plain["status"][11] == mpg.BAD_INPUT
    o = O.walk(osc, ep, prim, pos, st, prm=O.params(sc.scale, cone_cos=GC.cone_cos()))
    GC.compare_walks(ep, pers, o, sc.scale, tag="slab_persistent")


@pytest.mark.parametrize("order,max_len", [([3, 8, 7, 6, 5, 4, 2, 1], 8), ([1, 2, 3, 4, 5, 6, 7, 8], 8),
                                           ([2, 8, 7, 6, 5, 4, 3, 1], 5)])
def test_length_order_changes_scheduling_only(mpg, order, max_len):
    """The order in which the per-length kernels are dealt to the workers
    leaves every output unchanged (also with lengths above max_len, which are
    skipped and whose chains are bad input)."""
    sc = W.slab_stack_scene()
    ep = W.slab_uneven_endpoints(12000 + 5)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    kw = dict(form=mpg.FORM_PERSISTENT, bucketing=1, refill=1, waves_per_group=1, max_len=max_len)
    ref = run_gpu_walk(mpg, sc, ep, prim, pos, st, **kw)
    got = run_gpu_walk(mpg, sc, ep, prim, pos, st, length_order=order, **kw)
    for k in ("status", "iters", "sol", "G", "kappa", "residual"):
        assert np.array_equal(ref[k], got[k]), k
    ok = ref["status"] != mpg.BAD_INPUT
    assert np.array_equal(ref["prim"][:, ok], got["prim"][:, ok])
    assert np.array_equal(ref["pos"][:, :, ok], got["pos"][:, :, ok])
    assert (ref["status"][ep.length > max_len] == mpg.BAD_INPUT).all()


def test_length_order_must_be_a_permutation(mpg):
    sc = W.slab_stack_scene()
    ep = W.slab_uneven_endpoints(256)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    with pytest.raises(mpg.MPGError, match="length_order"):
        run_gpu_walk(mpg, sc, ep, prim, pos, st, form=mpg.FORM_PERSISTENT, length_order=0x12345677)


def test_deferred_fp64_pass(mpg):
    """defer_fp64 leaves NEEDS_FP64 chains; manifold_walk_fp64 finishes them
    exactly as the one-call walk does."""
    import torch
    sc = W.sphere_mirror_scene()
    ep = W.sphere_mirror_endpoints(4096)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    one = run_gpu_walk(mpg, sc, ep, prim, pos, st, max_len=1)
    scene = mpg.Scene(sc)
    dep = mpg.Endpoints(ep)
    prm = mpg.walk_params(sc.scale, max_len=1, defer_fp64=1)
    p, q, outs = mpg.manifold_walk_batch(scene, prm, dep, torch.as_tensor(prim).cuda(), torch.as_tensor(pos).cuda(),
                                         torch.as_tensor(st).cuda())
    torch.cuda.synchronize()
    mid = GC.to_np(outs["status"])
    assert (mid == mpg.NEEDS_FP64).sum() > 0
    mpg.manifold_walk_fp64(scene, prm, dep, p, q, outs)
    torch.cuda.synchronize()
    assert np.array_equal(GC.to_np(outs["status"]), one["status"])
    assert np.array_equal(GC.to_np(q).astype(np.float64), one["pos"])


def test_counting_walk_matches_and_counts(mpg):
    """The counting launch produces the same chains as the timed walk and
    positive work tallies."""
    import torch
    sc = W.icosphere_glass_scene()
    ep = W.icosphere_endpoints(8192)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    ref = run_gpu_walk(mpg, sc, ep, prim, pos, st, max_len=2)
    scene = mpg.Scene(sc)
    dep = mpg.Endpoints(ep)
    prm = mpg.walk_params(sc.scale, max_len=2)
    p, q, outs, counts = mpg.walk_count(scene, prm, dep, torch.as_tensor(prim).cuda(), torch.as_tensor(pos).cuda(),
                                        torch.as_tensor(st).cuda())
    assert np.array_equal(GC.to_np(outs["status"]), ref["status"])
    assert counts["chains"] == ep.n
    assert counts["rays"] > ep.n and counts["box_tests"] > counts["rays"] and counts["tri_tests"] > 0
    assert counts["vertex_jacobian_evals"] > 0 and counts["vertex_residual_evals"] > 0


@pytest.mark.parametrize("bucketing,order", [(1, 0), (2, 0), (1, [3, 8, 7, 6, 5, 4, 2, 1])])
def test_persistent_seeds_match_plain_seeds(mpg, bucketing, order):
    """Seeds drawn by the persistent per-length kernels equal the plain
    launch's bit for bit (same routine, same Philox counters)."""
    import torch
    sc = W.slab_stack_scene()
    ep = W.slab_uneven_endpoints(30000 + 5, seed=4)
    ep.length[3] = 0            # invalid length -> bad input on both paths
    scene = mpg.Scene(sc)
    dep = mpg.Endpoints(ep)
    plain = mpg.walk_params(sc.scale, cone_cos=GC.cone_cos())
    pers = mpg.walk_params(sc.scale, cone_cos=GC.cone_cos(), form=mpg.FORM_PERSISTENT, bucketing=bucketing,
                           length_order=order)
    ws = mpg.Workspace(ep.n)
    a = mpg.sample_seeds(scene, dep, plain, seed=9, trial=2)
    b = mpg.sample_seeds(scene, dep, pers, seed=9, trial=2, ws=ws)
    torch.cuda.synchronize()
    sa, sb = GC.to_np(a[2]), GC.to_np(b[2])
    assert np.array_equal(sa, sb) and sa[3] == mpg.BAD_INPUT
    ok = sa == 0
    assert ok.mean() > 0.5
    used = (np.arange(8)[:, None] < ep.length[None, :]) & ok[None, :]
    assert np.array_equal(GC.to_np(a[0])[used], GC.to_np(b[0])[used])
    assert np.array_equal(GC.to_np(a[1])[:, used], GC.to_np(b[1])[:, used])

