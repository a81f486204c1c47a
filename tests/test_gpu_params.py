"""mpg_scene_set_params: a scene moved to new height-field parameters on the
GPU walks like a scene built from scratch with them, and like the oracle's
scene with the same parameters (vertices recomputed in FP64)."""
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


def _walk(M, scene, sc, ep, prim, pos, st):
    import torch
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos())
    p, q, outs = M.manifold_walk_batch(scene, prm, dep, torch.as_tensor(prim).cuda(), torch.as_tensor(pos).cuda(),
                                       torch.as_tensor(st).cuda())
    torch.cuda.synchronize()
    g = {k: GC.to_np(v) for k, v in outs.items()}
    g["prim"] = GC.to_np(p)
    g["pos"] = GC.to_np(q).astype(np.float64)
    g["sol"] = g["sol"].view(np.uint64)
    return g


def test_set_params_matches_fresh_scene_and_oracle(mpg):
    import torch
    M = mpg
    sc0 = W.slab_stack_scene()
    th0 = W.slab_theta(sc0)
    g = np.random.default_rng(5)
    th1 = th0.copy()
    th1[0::2] *= g.uniform(0.5, 1.5, th1[0::2].shape)
    th1[1::2] += g.uniform(-0.5, 0.5, th1[1::2].shape)
    sc1 = W.slab_stack_scene(theta=th1)
    moved = M.Scene(sc0)
    moved.set_params(torch.as_tensor(th1, dtype=torch.float32))
    fresh = M.Scene(sc1)
    ep = W.slab_uneven_endpoints(8192, seed=21)
    osc = O.Scene(sc1)
    osc.set_theta(th1.astype(np.float32).astype(np.float64))
    prim, pos, st = GC.oracle_seeds(osc, ep)
    a = _walk(M, moved, sc1, ep, prim, pos, st)
    b = _walk(M, fresh, sc1, ep, prim, pos, st)
    # same decisions as the freshly built scene (vertices differ by FP32 rounding)
    agree = (a["status"] == b["status"]).mean()
    both = (a["status"] == 0) & (b["status"] == 0)
    same = both & (a["sol"] == b["sol"])
    err = np.abs(a["pos"] - b["pos"]).max((0, 1))[same]
    print(dict(status_agree=float(agree), both=int(both.sum()), same_sol=int(same.sum()), max_err=float(err.max())),
          flush=True)
    assert agree >= 0.999 and same.sum() >= 0.999 * both.sum()
    assert err.max() <= 1e-5 * sc1.scale
    # parity with the oracle on the moved parameters
    o = O.walk(osc, ep, prim, pos, st, prm=O.params(sc1.scale, cone_cos=GC.cone_cos()))
    GC.compare_walks(ep, a, o, sc1.scale, tag="set_params")
    # and back: the original parameters reproduce the original scene's walks
    moved.set_params(torch.as_tensor(th0, dtype=torch.float32))
    orig = M.Scene(sc0)
    osc0 = O.Scene(sc0)
    p0, q0, s0 = GC.oracle_seeds(osc0, ep)
    c = _walk(M, moved, sc0, ep, p0, q0, s0)
    d = _walk(M, orig, sc0, ep, p0, q0, s0)
    assert (c["status"] == d["status"]).mean() >= 0.999
    # p_0 area tables: seeds drawn on the moved scene match the fresh scene's
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc0.scale, cone_cos=GC.cone_cos())
    moved.set_params(torch.as_tensor(th1, dtype=torch.float32))
    sa = M.sample_seeds(moved, dep, prm, seed=3)
    sb = M.sample_seeds(fresh, dep, prm, seed=3)
    torch.cuda.synchronize()
    ok = (GC.to_np(sa[2]) == 0) & (GC.to_np(sb[2]) == 0)
    same_prim = (GC.to_np(sa[0]) == GC.to_np(sb[0])).all(0) & ok
    assert same_prim.sum() >= 0.999 * ok.sum()


def test_set_params_rejects_bad_input(mpg):
    import torch
    M = mpg
    scene = M.Scene(W.slab_stack_scene())
    with pytest.raises(M.MPGError):
        scene.set_params(torch.zeros(31))
    sph = M.Scene(W.sphere_mirror_scene())
    sph.set_params(torch.zeros(0))   # no parameters: a no-op


def test_set_params_non_finite_theta_leaves_the_scene_unchanged(mpg):
    # a non-finite theta is found on the device (the call never reads theta
    # back): the error word is set, every later kernel of the update skips,
    # and walks on the scene are exactly those before the call
    import torch
    M = mpg
    sc = W.slab_stack_scene()
    scene = M.Scene(sc)
    assert int(scene.params_error().item()) == 0
    ep = W.slab_uneven_endpoints(4096, seed=23)
    osc = O.Scene(sc)
    prim, pos, st = GC.oracle_seeds(osc, ep)
    before = _walk(M, scene, sc, ep, prim, pos, st)
    bad = torch.as_tensor(W.slab_theta(sc), dtype=torch.float32)
    bad[5] = float("nan")
    scene.set_params(bad)
    assert int(scene.params_error().item()) == M.ERR_INVALID_ARG
    after = _walk(M, scene, sc, ep, prim, pos, st)
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    scene.set_params(torch.as_tensor(W.slab_theta(sc), dtype=torch.float32))
    assert int(scene.params_error().item()) == 0


def test_captured_set_params_walk_and_adjoint_replay_bit_exact(mpg):
    # the differentiable step (new theta -> seeds -> walk -> adjoint) is
    # stream ordered without host synchronization, so it can be captured into
    # one HIP graph; every replay (with other eager work between replays)
    # must reproduce the eager step bit for bit
    import torch
    M = mpg
    sc = W.slab_stack_scene()
    th0 = W.slab_theta(sc)
    g = np.random.default_rng(7)
    th1 = th0.copy()
    th1[0::2] *= g.uniform(0.7, 1.3, th1[0::2].shape)
    theta = torch.as_tensor(th1, dtype=torch.float32).cuda()
    n = 1 << 14
    ep = W.slab_adjoint_endpoints(n, seed=31)
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=4)
    prim, pos = M.empty_chains(n)
    outs = M.walk_outputs(n)
    r, gG = W.loss_weights(n)
    gpos = torch.as_tensor(r).cuda()
    ggG = torch.as_tensor(gG).cuda()
    gxD = torch.zeros(3, n, device="cuda")
    gxL = torch.zeros(3, n, device="cuda")
    gth = torch.zeros(32, device="cuda")

    def step():
        scene.set_params(theta)
        p, q, st = M.sample_seeds(scene, dep, prm, out=(prim, pos))
        M.manifold_walk_batch(scene, prm, dep, p, q, st, out_prim=prim, out_pos=pos, outs=outs)
        gth.zero_()
        M.manifold_walk_adjoint(scene, prm, dep, prim, pos, outs["status"], grad_pos=gpos, grad_G=ggG,
                                grad_xD=gxD, grad_xL=gxL, grad_theta=gth)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = {k: GC.to_np(v).copy() for k, v in outs.items()}
    ref_xD, ref_xL = GC.to_np(gxD).copy(), GC.to_np(gxL).copy()
    assert (ref["status"] == M.CONVERGED).mean() > 0.3
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        # move the scene elsewhere eagerly, clobber the outputs, then replay
        scene.set_params(torch.as_tensor(th0, dtype=torch.float32))
        for v in outs.values():
            v.fill_(-1) if v.dtype != torch.float32 else v.fill_(float("nan"))
        gxD.fill_(float("nan"))
        gxL.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert np.array_equal(GC.to_np(v), ref[k]), (rep, k)
        assert np.array_equal(GC.to_np(gxD), ref_xD), rep
        assert np.array_equal(GC.to_np(gxL), ref_xL), rep
