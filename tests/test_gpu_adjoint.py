"""GPU parity of the implicit-function-theorem adjoint (HIP path through the
C ABI) against the FP64 oracle's forward-IFT gradient, plus the autograd
wrapper against central differences of the GPU walk.

Both sides walk from the same oracle seeds; gradients are compared on chains
that both sides converge to the same triangles.  Loss:
l = sum_c (sum_i r_ci . x_ci + g_c G_c) with fixed random cotangents.

Tolerance: per chain, the gradient w.r.t. (x_D, x_L) as a 6-vector is within
1e-3 relative (plus 1e-5 absolute) of the oracle's on >= 99% of matched chains
that the walk itself treats as regular: Jacobian condition number <= 1e4 and
smallest incident / outgoing cosine >= 0.02 (the walk's thresholds for its
FP64 pass).  The gradient needs second derivatives of the constraint, whose
FP32 rounding grows like eps / cos^2 at grazing angles, so grazing chains
get the bound 1e-3 + 2^-24 / cos_min^2 instead; chains above the condition
threshold are only reported.  The theta gradient (summed over chains) is
within 1e-3 of the sum of per-chain magnitudes for every parameter.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import gpu_common as GC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2311_12818_amd as M
    M.lib()
    return M


def _cond(osc, ep, prim, pos, c):
    n = int(ep.length[c])
    _, J, _ = O.constraint(osc, n, int(ep.types[c]), ep.xD[:, c].astype(np.float64), ep.xL[:, c].astype(np.float64),
                           prim[:n, c], pos[:, :n, c].T.copy())
    return np.linalg.cond(J)


def _cos_min(sc, ep, prim, pos, c):
    """Smallest |n_g . w| over the incident and outgoing directions of chain c."""
    n = int(ep.length[c])
    pts = [ep.xD[:, c].astype(np.float64)] + [pos[:, i, c] for i in range(n)] + [ep.xL[:, c].astype(np.float64)]
    best = 1.0
    for i in range(n):
        p = int(prim[i, c])
        x = pts[i + 1]
        if p < 0:
            s = sc.spheres[-1 - p]
            ng = (x - s[:3]) / np.linalg.norm(x - s[:3])
        else:
            a, b, d = (sc.verts[int(v)].astype(np.float64) for v in sc.tris[p])
            ng = np.cross(b - a, d - a)
            ng /= np.linalg.norm(ng)
        for q in (pts[i], pts[i + 2]):
            w = (q - x) / np.linalg.norm(q - x)
            best = min(best, abs(float(np.dot(ng, w))))
    return best


def _run(M, name, n, max_len, seed=0):
    import torch
    scene_fn, ep_fn = W.WORKLOADS[name]
    sc = scene_fn()
    ep = ep_fn(n, seed=seed)
    osc = O.Scene(sc)
    prm_o = O.params(sc.scale, cone_cos=GC.cone_cos())
    sprim, spos, sst = GC.oracle_seeds(osc, ep)
    o = O.walk(osc, ep, sprim, spos, sst, prm=prm_o)
    r32, g32 = W.loss_weights(n, seed=seed + 1)
    theta = W.slab_theta(sc) if sc.heightfields else None
    oxD, oxL, oth, ook = O.adjoint(osc, ep, o["prim"], o["pos"], o["status"], r32.astype(np.float64),
                                   g32.astype(np.float64), theta=theta, prm=prm_o)

    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=max_len)
    prim, pos, outs = M.manifold_walk_batch(scene, prm, dep, torch.as_tensor(sprim).cuda(),
                                            torch.as_tensor(spos).cuda(), torch.as_tensor(sst).cuda())
    g_st = GC.to_np(outs["status"])
    g_prim = GC.to_np(prim)
    match = (g_st == O.CONVERGED) & (o["status"] == O.CONVERGED) & (ook == 1)
    for i in range(max_len):
        match &= (ep.length <= i) | (g_prim[i] == o["prim"][i])
    # cotangents only on matched chains, so the summed theta gradients compare
    r = np.where(match[None, None, :], r32, 0).astype(np.float32)
    g = np.where(match, g32, 0).astype(np.float32)
    gxD, gxL, gth = M.manifold_walk_adjoint(scene, prm, dep, prim, pos, outs["status"], torch.as_tensor(r).cuda(),
                                            torch.as_tensor(g).cuda())
    torch.cuda.synchronize()
    return dict(sc=sc, ep=ep, osc=osc, o=o, match=match, oxD=oxD, oxL=oxL, oth=oth, gxD=GC.to_np(gxD),
                gxL=GC.to_np(gxL), gth=GC.to_np(gth)[:scene.n_params], g_st=g_st, g_prim=g_prim,
                g_pos=GC.to_np(pos).astype(np.float64))


def _check_endpoint_grads(R, tag, min_match):
    m = R["match"]
    assert m.sum() >= min_match, (tag, int(m.sum()))
    ref = np.concatenate([R["oxD"], R["oxL"]], 0)[:, m]
    got = np.concatenate([R["gxD"], R["gxL"]], 0)[:, m]
    nref = np.linalg.norm(ref, axis=0)
    err = np.linalg.norm(got - ref, axis=0)
    rel = err / np.maximum(nref, 1e-12)
    idx = np.nonzero(m)[0]
    cond = np.array([_cond(R["osc"], R["ep"], R["o"]["prim"], R["o"]["pos"], c) for c in idx])
    cmin = np.array([_cos_min(R["sc"], R["ep"], R["o"]["prim"], R["o"]["pos"], c) for c in idx])
    well = cond <= 1e4
    graze = well & (cmin < 0.02)
    regular = well & ~graze
    good = err <= 1e-3 * nref + 1e-5
    good_graze = err <= (1e-3 + 2.0 ** -24 / cmin ** 2) * nref + 1e-5
    stats = dict(tag=tag, matched=int(m.sum()), regular=int(regular.sum()), grazing=int(graze.sum()),
                 ill_conditioned=int((~well).sum()), rel_median=float(np.median(rel)),
                 rel_q99_regular=float(np.quantile(rel[regular], 0.99)) if regular.any() else 0.0,
                 rel_max_regular=float(rel[regular].max()) if regular.any() else 0.0,
                 rel_max_grazing=float(rel[graze].max()) if graze.any() else 0.0,
                 good_frac_regular=float(good[regular].mean()) if regular.any() else 1.0,
                 ill_rel_max=float(rel[~well].max()) if (~well).any() else 0.0)
    print(stats, flush=True)
    assert stats["good_frac_regular"] >= 0.99, stats
    assert good_graze[graze].all(), stats
    # the GPU must not produce gradients for chains it did not converge
    bad = R["g_st"] != O.CONVERGED
    assert np.all(R["gxD"][:, bad] == 0) and np.all(R["gxL"][:, bad] == 0)
    return stats


def test_adjoint_matches_oracle_slab(mpg):
    R = _run(mpg, "slab_adjoint", 1024, 4)
    _check_endpoint_grads(R, "slab_adjoint", 600)
    # theta: summed over matched chains
    m = R["match"]
    ref = R["oth"][m].sum(0)
    mag = np.abs(R["oth"][m]).sum(0)
    err = np.abs(R["gth"] - ref)
    print(dict(theta_err_over_mag_max=float((err / np.maximum(mag, 1e-12)).max()), theta_mag_max=float(mag.max())),
          flush=True)
    assert np.all(err <= 1e-3 * mag + 1e-5), (err, mag)
    # parameters of the two lowest slabs are never crossed by these chains
    assert np.all(R["gth"][16:] == 0)


def test_adjoint_matches_oracle_sphere_mirror(mpg):
    R = _run(mpg, "sphere_mirror", 4096, 1)
    _check_endpoint_grads(R, "sphere_mirror", 300)
    assert R["gth"].size == 0


def test_adjoint_matches_oracle_water(mpg):
    R = _run(mpg, "water_caustic", 2048, 1)
    _check_endpoint_grads(R, "water_caustic", 300)
    m = R["match"]
    ref = R["oth"][m].sum(0)
    mag = np.abs(R["oth"][m]).sum(0)
    assert np.all(np.abs(R["gth"] - ref) <= 1e-3 * mag + 1e-5)


def test_adjoint_ignores_missing_cotangents_and_empty_batches(mpg):
    import torch
    M = mpg
    sc = W.slab_stack_scene()
    ep = W.slab_adjoint_endpoints(256, seed=3)
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=4)
    p, q, st = M.sample_seeds(scene, dep, prm)
    prim, pos, outs = M.manifold_walk_batch(scene, prm, dep, p, q, st)
    gxD, gxL, gth = M.manifold_walk_adjoint(scene, prm, dep, prim, pos, outs["status"], None, None)
    torch.cuda.synchronize()
    assert float(gxD.abs().max()) == 0 and float(gxL.abs().max()) == 0 and float(gth.abs().max()) == 0
    # only G cotangents: equals the full loss minus the position part
    r, g = W.loss_weights(256, seed=4)
    rt, gt = torch.as_tensor(r).cuda(), torch.as_tensor(g).cuda()
    a = M.manifold_walk_adjoint(scene, prm, dep, prim, pos, outs["status"], rt, gt)
    b = M.manifold_walk_adjoint(scene, prm, dep, prim, pos, outs["status"], rt, None)
    c = M.manifold_walk_adjoint(scene, prm, dep, prim, pos, outs["status"], None, gt)
    torch.cuda.synchronize()
    for k in range(2):
        np.testing.assert_allclose(GC.to_np(a[k]), GC.to_np(b[k]) + GC.to_np(c[k]), rtol=1e-4, atol=1e-4)
    # an empty batch is a no-op
    e0 = W.slab_adjoint_endpoints(0, seed=3)
    d0 = M.Endpoints(e0)
    pr0, po0 = M.empty_chains(0)
    st0 = torch.zeros(0, dtype=torch.int8, device="cuda")
    M.manifold_walk_adjoint(scene, prm, d0, pr0, po0, st0, None, None)
    torch.cuda.synchronize()


def test_autograd_function_matches_central_differences(mpg):
    """The torch.autograd.Function's backward (the adjoint) against central
    differences of its own forward (FP32 GPU walks from fixed seeds), in
    x_D, x_L and theta, along random directions."""
    import torch
    M = mpg
    from paper_2311_12818_amd.autograd import WalkProblem, manifold_walk
    n = 64
    sc0 = W.slab_stack_scene()
    ep = W.slab_adjoint_endpoints(n, seed=7)
    osc = O.Scene(sc0)
    sprim, spos, sst = GC.oracle_seeds(osc, ep)
    # every converged chain takes the FP64 pass (graze threshold above 1), so
    # the forward's vertices are Newton-polished in FP64 and G is evaluated in
    # FP64: differences of re-solved chains then resolve h = 1e-4 (FP32
    # vertices alone carry ~1e-6 of convergence slack, and FP32 G up to 1e-3
    # relative at poorly conditioned chains)
    prm = M.walk_params(sc0.scale, cone_cos=GC.cone_cos(), max_len=4, defer_fp64=1, fp64_graze_cos=2.0)
    dev = "cuda"
    problem = WalkProblem(M.Scene(sc0), prm,
                          torch.as_tensor(ep.nD).to(dev), torch.as_tensor(ep.length).to(dev),
                          torch.as_tensor(ep.types).to(dev), torch.as_tensor(ep.obj1).to(dev),
                          torch.as_tensor(sprim).to(dev), torch.as_tensor(spos).to(dev),
                          torch.as_tensor(sst).to(dev))
    xD = torch.as_tensor(ep.xD).to(dev).requires_grad_(True)
    xL = torch.as_tensor(ep.xL).to(dev).requires_grad_(True)
    theta = torch.as_tensor(W.slab_theta(sc0), dtype=torch.float32).to(dev).requires_grad_(True)
    r, g = W.loss_weights(n, seed=8)
    rt, gt = torch.as_tensor(r).to(dev), torch.as_tensor(g).to(dev)
    pos, G, st = manifold_walk(xD, xL, theta, problem)
    base_conv = st == 0
    assert int(base_conv.sum()) >= 32
    zero = torch.zeros((), device=dev)
    # the walk's own primitive ids (not differentiable; read through the
    # C ABI binding on the same inputs)
    dep = problem.endpoints(xD, xL)
    base_prim, _, _ = M.manifold_walk_batch(problem.scene(theta), prm, dep, problem.seed_prim, problem.seed_pos,
                                            problem.seed_status)
    lens = torch.as_tensor(ep.length).to(dev).long()
    used = torch.arange(8, device=dev)[:, None] < lens[None, :]

    def per_chain(dxD, dxL, dth):
        with torch.no_grad():
            p, Gv, s = manifold_walk(xD + dxD, xL + dxL, theta + dth, problem)
            prim, _, _ = M.manifold_walk_batch(problem.scene(theta + dth), prm, problem.endpoints(xD + dxD, xL + dxL),
                                               problem.seed_prim, problem.seed_pos, problem.seed_status)
            same = ((prim == base_prim) | ~used).all(0)
            return ((p * rt).sum((0, 1)) + Gv * gt).double(), (s == 0) & same

    gen = torch.Generator(device="cpu").manual_seed(0)
    for which in ("xD", "xL", "theta"):
        for _ in range(2):
            shape = theta.shape if which == "theta" else xD.shape
            u = torch.randn(shape, generator=gen, dtype=torch.float32).to(dev)
            if which == "theta":
                u[16:] = 0
            h = 1e-4
            z3 = torch.zeros_like(xD)
            zt = torch.zeros_like(theta)
            args_p = (h * u if which == "xD" else z3, h * u if which == "xL" else z3, h * u if which == "theta" else zt)
            args_m = tuple(-a for a in args_p)
            lp, cp = per_chain(*args_p)
            lm, cm = per_chain(*args_m)
            # chains that stay converged on the same triangles on both sides:
            # with interpolated vertex normals the normal's derivative, and
            # so G, jumps across triangle edges
            keep = base_conv & cp & cm
            assert int(keep.sum()) >= 0.9 * int(base_conv.sum())
            fd = float(torch.where(keep, lp - lm, zero.double()).sum()) / (2 * h)
            # the adjoint of the same masked loss through the autograd function
            pos, G, st = manifold_walk(xD, xL, theta, problem)
            loss = torch.where(keep, (pos * rt).sum((0, 1)) + G * gt, zero).sum()
            inp = {"xD": xD, "xL": xL, "theta": theta}[which]
            (grad,) = torch.autograd.grad(loss, [inp])
            an = float((grad * u).double().sum())
            print(dict(which=which, kept=int(keep.sum()), fd=fd, adjoint=an), flush=True)
            assert an == pytest.approx(fd, rel=1e-2, abs=0.05)


def test_persistent_adjoint_matches_plain(mpg):
    """Length-bucketed persistent adjoint kernels: the same per-chain
    gradients as the plain launch (x_D, x_L bit for bit; theta up to the
    order of the atomic float additions)."""
    import torch
    M = mpg
    sc = W.slab_stack_scene()
    ep = W.slab_adjoint_endpoints(12000 + 7, seed=9)
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    plain = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=4)
    pers = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=4, form=M.FORM_PERSISTENT, bucketing=1)
    ws = M.Workspace(ep.n)
    p, q, st = M.sample_seeds(scene, dep, plain)
    prim, pos, outs = M.manifold_walk_batch(scene, plain, dep, p, q, st)
    r, g = W.loss_weights(ep.n, seed=10)
    rt, gt = torch.as_tensor(r).cuda(), torch.as_tensor(g).cuda()
    a = M.manifold_walk_adjoint(scene, plain, dep, prim, pos, outs["status"], rt, gt)
    b = M.manifold_walk_adjoint(scene, pers, dep, prim, pos, outs["status"], rt, gt, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(GC.to_np(a[0]), GC.to_np(b[0])) and np.array_equal(GC.to_np(a[1]), GC.to_np(b[1]))
    ta, tb = GC.to_np(a[2]).astype(np.float64), GC.to_np(b[2]).astype(np.float64)
    assert np.all(np.abs(ta - tb) <= 1e-4 * np.abs(ta).max() + 1e-6)
    assert (GC.to_np(outs["status"]) == M.CONVERGED).sum() > 5000

