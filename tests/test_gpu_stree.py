"""GPU parity of the paper's guide (Sec. 5.5, 5.6) against the FP64 oracle:
the fitted tree and lobes, seeds with sampled length and type, the
P(n)-factored Bernoulli trials and selective activation; and the end-to-end
effect of learning: guided seeds find admissible chains more often than
the initial distribution."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import gpu_common as GC

pytestmark = pytest.mark.gpu

ROOT_LO = [0.0, 0.0, -2.5, 1.5, 1.5, 2.5]
ROOT_HI = [7.5, 4.0, 0.5, 2.5, 2.5, 3.5]


@pytest.fixture(scope="module")
def mpg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2311_12818_amd as M
    M.lib()
    return M


def geometric_prior():
    """P_0(n): min(Geometric(0.4), 8), the length law of the uneven batch."""
    p = np.array([0.4 * 0.6 ** (k - 1) for k in range(1, 8)] + [0.6 ** 7])
    return p / p.sum()


def synthetic_records(n, seed=0):
    """Sub-path samples over the slab-stack configurations: x_D, x_L of the
    uneven batch, its length and type, w_D towards the light with a spread,
    weights in [0.1, 2]."""
    g = np.random.default_rng(seed)
    ep = W.slab_uneven_endpoints(n, seed=100 + seed)
    xD, xL = ep.xD.T.astype(np.float64), ep.xL.T.astype(np.float64)
    d = xL - xD
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d += g.normal(scale=0.05, size=d.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    w = g.uniform(0.1, 2.0, n)
    return O.sample_records(xD, xL, d, w, ep.length, ep.types)


def both_trees(M, rec, **kw):
    """The oracle's and the library's guide from the same records; the
    oracle gets the parameters as the library holds them (FP32)."""
    import torch
    f32 = lambda v: float(np.float32(v))
    kw.setdefault("eps", 0.1)
    kw.setdefault("sigma_min", 1e-3)
    kw.setdefault("sigma_lone", 0.1)
    okw = {k: (f32(v) if k in ("eps", "sigma_min", "sigma_lone", "alpha", "p_transmit", "thr_scale") else v)
           for k, v in kw.items()}
    if "p0n" in okw:
        okw["p0n"] = np.asarray(okw["p0n"], np.float32).astype(np.float64)
    ot = O.STree(rec, ROOT_LO, ROOT_HI, **okw)
    gt = M.STree(ROOT_LO, ROOT_HI, **kw)
    gt.fit(torch.as_tensor(rec).cuda())
    torch.cuda.synchronize()
    return ot, gt


def test_fitted_tree_and_lobes_match_oracle(mpg):
    M = mpg
    rec = synthetic_records(1 << 16)
    rec[17, 9] = 0.0            # zero weight: not a sample
    rec[33, 6] = np.nan         # non-finite: not a sample
    ot, gt = both_trees(M, rec, p0n=geometric_prior())
    o = ot.nodes()
    g = gt.download()
    # integer structure identical (decisions in FP64 on the host for both)
    assert np.array_equal(g["axis"], o["axis"])
    assert np.array_equal(g["child"][o["axis"] >= 0], o["child"][o["axis"] >= 0])
    assert np.allclose(g["mid"], o["mid"].astype(np.float32))
    leaf = o["axis"] < 0
    assert np.array_equal(g["own"][leaf], o["n_own"][leaf])
    assert np.allclose(g["W"][leaf], o["W"][leaf], rtol=1e-6)
    assert np.allclose(g["Wn"][leaf], o["Wn"][leaf], rtol=1e-6, atol=1e-6)
    L = ot.lobes()
    assert len(g["lobe"]) == len(L["kappa"])
    assert np.allclose(g["lobe"][:, :3], L["mu"], atol=1e-6)
    # footprints: nearest-direction angle in FP32 on the GPU
    rel = np.abs(g["lobe"][:, 3] - L["kappa"]) / L["kappa"]
    print(dict(lobes=len(rel), kappa_rel_med=float(np.median(rel)), kappa_rel_max=float(rel.max())), flush=True)
    assert np.median(rel) < 1e-5 and rel.max() < 2e-2
    assert (rel > 1e-3).mean() < 1e-3


def test_stree_seeds_match_oracle(mpg):
    import torch
    M = mpg
    rec = synthetic_records(1 << 15, seed=1)
    ot, gt = both_trees(M, rec, p0n=geometric_prior(), alpha=0.5)
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    ep = W.slab_uneven_endpoints(8192, seed=41)
    ep.length[:] = 0                          # lengths drawn by the guide
    prm_o = O.params(sc.scale, cone_cos=GC.cone_cos())
    on, oty, opn, oprim, opos, ost = O.stree_sample_seeds(osc, ot, ep, seed=3, prm=prm_o)
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos())
    gn, gty, gpn, gprim, gpos, gst = M.sample_seeds_stree(scene, gt, dep, prm, seed=3)
    torch.cuda.synchronize()
    gn, gty, gpn, gst = GC.to_np(gn), GC.to_np(gty), GC.to_np(gpn), GC.to_np(gst)
    gprim, gpos = GC.to_np(gprim), GC.to_np(gpos)
    assert np.mean(gn != on) <= 1e-3
    same = gn == on
    assert np.allclose(gpn[same], opn[same], rtol=1e-5)
    ok = same & (gst == 0) & (ost == 0)
    assert np.mean(gty[ok] != oty[ok]) <= 1e-3
    err = np.zeros(ep.n)
    for i in range(8):
        m = ok & (on > i)
        err = np.where(m, np.maximum(err, np.abs(gpos[:, i, :] - opos[:, i, :]).max(0)), err)
    close = ok & (gty == oty) & (err <= 1e-4 * sc.scale)
    frac = (np.sum(gst != ost) + np.sum(ok & ~close)) / ep.n
    hist = np.bincount(on.astype(np.int64), minlength=9)[1:]
    print(dict(n_hist=hist.tolist(), seed_ok=int(ok.sum()), mismatch=float(frac)), flush=True)
    assert frac <= 2e-3
    assert ok.sum() > 2000


def test_stree_trials_match_oracle(mpg):
    import torch
    M = mpg
    rec = synthetic_records(1 << 15, seed=2)
    ot, gt = both_trees(M, rec, p0n=geometric_prior(), alpha=0.5)
    sc = W.slab_stack_scene()
    osc = O.Scene(sc)
    ep = W.slab_uneven_endpoints(3000, seed=43)
    ep.length[:] = 0
    prm_o = O.params(sc.scale, cone_cos=GC.cone_cos())
    on, oty, opn, oprim, opos, ost = O.stree_sample_seeds(osc, ot, ep, seed=5, prm=prm_o)
    ep.length[:] = on
    ep.types[:] = oty
    o = O.walk(osc, ep, oprim, opos.astype(np.float32), ost, prm=prm_o)
    t_o, ip_o, tr_o, pn_o = O.stree_inv_prob(osc, ot, ep, on, oty, o["prim"], o["pos"], o["status"], max_trials=24,
                                             seed=9, prm=prm_o)
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos())
    t_g, ip_g, tr_g, pn_g = M.estimate_inv_prob_stree(scene, gt, prm, dep, torch.as_tensor(o["prim"]).cuda(),
                                                      torch.as_tensor(o["pos"].astype(np.float32)).cuda(),
                                                      torch.as_tensor(o["status"]).cuda(), max_trials=24, seed=9)
    torch.cuda.synchronize()
    t_g, ip_g, pn_g = GC.to_np(t_g), GC.to_np(ip_g), GC.to_np(pn_g)
    conv = o["status"] == O.CONVERGED
    agree = (t_g[conv] == t_o[conv]).mean()
    print(dict(n_conv=int(conv.sum()), K_agree=float(agree), mean_g=float(t_g[conv].mean()),
               mean_o=float(t_o[conv].mean())), flush=True)
    assert conv.sum() > 500
    assert agree >= 0.98
    assert np.allclose(pn_g[conv], pn_o[conv], rtol=1e-5)
    assert np.allclose(ip_g[conv], t_g[conv] / pn_g[conv], rtol=1e-6)
    assert np.all(t_g[~conv] == 0)


def test_selective_activation_matches_oracle_leaves(mpg):
    import torch
    M = mpg
    rec = synthetic_records(1 << 14, seed=3)
    ot, gt = both_trees(M, rec)
    ep = W.slab_uneven_endpoints(4096, seed=44)
    ep.xD[0, :200] += 10.0                    # far outside the samples: no own samples there
    dep = M.Endpoints(ep)
    act = GC.to_np(M.stree_active(gt, dep))
    torch.cuda.synchronize()
    leaf = ot.lookup(ep.xD.astype(np.float64), ep.xL.astype(np.float64))
    want = (ot.nodes()["n_own"][leaf] > 0).astype(np.uint8)
    assert np.mean(act != want) <= 1e-3
    assert act.mean() > 0.5 and act[:200].mean() < act[200:].mean()


def test_learned_guide_beats_the_initial_distribution(mpg):
    """Training round (p_0 only: an empty guide) -> walks -> P(n)-factored
    trials -> records -> fit; the fitted guide's seeds then find admissible
    chains more often, with the length drawn by the guide."""
    import torch
    M = mpg
    sc = W.slab_stack_scene()
    scene = M.Scene(sc)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos())
    tree = M.STree(ROOT_LO, ROOT_HI, p0n=geometric_prior(), alpha=0.5)
    rates = []
    for it in range(2):
        ep = W.slab_uneven_endpoints(1 << 17, seed=50 + it)
        ep.length[:] = 0
        dep = M.Endpoints(ep)
        n, ty, pn, prim, pos, st = M.sample_seeds_stree(scene, tree, dep, prm, seed=7 + it)
        wep = M.Endpoints.from_tensors(dep.xD, dep.nD, dep.xL, n, ty, dep.obj1)
        prim, pos, outs = M.manifold_walk_batch(scene, prm, wep, prim, pos, st, out_prim=prim, out_pos=pos)
        conv = (outs["status"] == M.CONVERGED).float().mean().item()
        rates.append(conv)
        trials, ip, tr, pn2 = M.estimate_inv_prob_stree(scene, tree, prm, wep, prim, pos, outs["status"],
                                                        max_trials=16, seed=11 + it)
        rec = M.make_guide_records(wep, pos, outs, ip)
        tree.fit(rec)
        torch.cuda.synchronize()
    s = tree.stats()
    print(dict(rates=rates, tree=s), flush=True)
    assert s["leaves"] > 10
    assert rates[1] > rates[0] + 0.05


def test_stree_trials_persistent_form_matches_plain(mpg):
    """The lane-refill trial kernels (targets bucketed by length) give the
    plain form's trials, P(n) and 1/P bit for bit, over lengths 1..8 drawn
    by a fitted guide; targets longer than max_len get 0 in both forms."""
    import torch
    M = mpg
    rec = synthetic_records(1 << 15, seed=4)
    _, gt = both_trees(M, rec, p0n=geometric_prior(), alpha=0.5)
    sc = W.slab_stack_scene()
    scene = M.Scene(sc)
    ep = W.slab_uneven_endpoints(20000, seed=45)
    ep.length[:] = 0
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos())
    n, ty, pn, prim, pos, st = M.sample_seeds_stree(scene, gt, dep, prm, seed=13)
    wep = M.Endpoints.from_tensors(dep.xD, dep.nD, dep.xL, n, ty, dep.obj1)
    prim, pos, outs = M.manifold_walk_batch(scene, prm, wep, prim, pos, st, out_prim=prim, out_pos=pos)
    ws = M.Workspace(ep.n)
    for max_len in (8, 5):
        plain = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=max_len)
        pers = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=max_len, form=M.FORM_PERSISTENT, bucketing=1,
                             refill=1)
        a = M.estimate_inv_prob_stree(scene, gt, plain, wep, prim, pos, outs["status"], max_trials=16, seed=21)
        b = M.estimate_inv_prob_stree(scene, gt, pers, wep, prim, pos, outs["status"], max_trials=16, seed=21, ws=ws)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert np.array_equal(GC.to_np(x), GC.to_np(y))
        nn = GC.to_np(n)
        conv = GC.to_np(outs["status"]) == M.CONVERGED
        t = GC.to_np(a[0])
        assert np.all(t[nn > max_len] == 0) and np.all(t[conv & (nn <= max_len)] >= 1)
        hist = np.bincount(nn[conv].astype(np.int64), minlength=9)[1:]
        print(dict(max_len=max_len, conv_by_length=hist.tolist(), mean_trials=float(t[conv & (nn <= max_len)].mean())),
              flush=True)
        assert (hist > 0).sum() >= 6
    with pytest.raises(M.MPGError):
        M.estimate_inv_prob_stree(scene, gt, pers, wep, prim, pos, outs["status"], max_trials=16, seed=21,
                                  ws=M.Workspace(100))


def test_stree_seeds_persistent_form_matches_plain(mpg):
    """Lengths drawn first, configurations bucketed by length, one seed
    kernel per length: the same n, tau, P(n), seed chains and statuses as
    one thread per configuration, including fixed lengths and bad inputs."""
    import torch
    M = mpg
    rec = synthetic_records(1 << 15, seed=5)
    _, gt = both_trees(M, rec, p0n=geometric_prior(), alpha=0.5)
    sc = W.slab_stack_scene()
    scene = M.Scene(sc)
    ep = W.slab_uneven_endpoints(30000, seed=46)
    ep.length[: 20000] = 0                    # drawn; the rest keep their fixed lengths
    ep.xD[0, 7] = np.nan                      # bad inputs
    ep.length[9] = 11
    dep = M.Endpoints(ep)
    plain = M.walk_params(sc.scale, cone_cos=GC.cone_cos())
    pers = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), form=M.FORM_PERSISTENT, bucketing=1, refill=1)
    ws = M.Workspace(ep.n)
    a = M.sample_seeds_stree(scene, gt, dep, plain, seed=17, trial=3)
    b = M.sample_seeds_stree(scene, gt, dep, pers, seed=17, trial=3, ws=ws)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert np.array_equal(GC.to_np(x), GC.to_np(y), equal_nan=True)
    st = GC.to_np(a[5])
    assert st[7] == M.BAD_INPUT and st[9] == M.BAD_INPUT
    assert np.array_equal(GC.to_np(a[0])[20000:][st[20000:] != M.BAD_INPUT], ep.length[20000:][st[20000:] != M.BAD_INPUT])
    assert (st == 0).mean() > 0.5
    drawn = GC.to_np(a[0])[:20000]
    assert np.array_equal(np.unique(drawn[st[:20000] != M.BAD_INPUT]), np.arange(1, 9))
