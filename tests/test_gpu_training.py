"""The progressive training loop (Sec. 5.8) end to end on the GPU: the
schedule of the host state machine driving guided seeds, walks,
P(n)-factored trials, sample records and refits of the paper's guide, in
the persistent form, with a deterministic clock; the trained guide then
finds admissible chains more often than the prior alone."""
import numpy as np
import pytest

import workloads as W
from tests import gpu_common as GC
from tests.test_gpu_stree import ROOT_HI, ROOT_LO, geometric_prior

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2311_12818_amd as M
    M.lib()
    return M


def converged_fraction(M, scene, tree, prm, ws, n, seed):
    ep = W.slab_uneven_endpoints(n, seed=seed)
    ep.length[:] = 0
    dep = M.Endpoints(ep)
    ln, ty, pn, prim, pos, st = M.sample_seeds_stree(scene, tree, dep, prm, seed=seed, ws=ws)
    wep = M.Endpoints.from_tensors(dep.xD, dep.nD, dep.xL, ln, ty, dep.obj1)
    _, _, outs = M.manifold_walk_batch(scene, prm, wep, prim, pos, st, out_prim=prim, out_pos=pos, ws=ws)
    return float((outs["status"] == M.CONVERGED).float().mean())


def test_training_loop_schedule_and_effect(mpg):
    import torch
    from paper_2311_12818_amd.training import train_guide
    M = mpg
    sc = W.slab_stack_scene()
    scene = M.Scene(sc)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), form=M.FORM_PERSISTENT, bucketing=1, refill=1)
    ws = M.Workspace(1 << 16)
    tree = M.STree(ROOT_LO, ROOT_HI, p0n=geometric_prior(), alpha=0.5)
    # time advances by 1e-5 units per configuration drawn: budget 1, training
    # share 0.3 (half of it: 0.15)
    now = [0.0]

    def make_configs(i, count):
        now[0] += count * 1e-5
        ep = W.slab_uneven_endpoints(count, seed=600 + i)
        ep.length[:] = 0
        return M.Endpoints(ep)

    log = train_guide(scene, tree, prm, make_configs, budget=1.0, train_fraction=0.3, base_samples=1 << 12,
                      batch=1 << 15, max_trials=16, seed=5, clock=lambda: now[0], ws=ws)
    torch.cuda.synchronize()
    sched = [(it, n, refit) for it, n, conv, refit, _ in log]
    print(dict(log=log, tree=tree.stats()), flush=True)
    # iteration 0: 4096 samples (t = 0.04) -> refit; iteration 1: 8192 (t =
    # 0.12) -> refit; iteration 2: 16384 ends at t = 0.29, past half the
    # training budget, so it keeps gathering: 32768 more, training ends at
    # t = 0.62 with the refit from iteration 2's samples
    assert sched == [(0, 4096, True), (1, 8192, True), (2, 16384, False), (2, 32768, True)]
    s = tree.stats()
    assert s["leaves"] > 4 and s["lobes"] > 1000
    prior = M.STree(ROOT_LO, ROOT_HI, p0n=geometric_prior(), alpha=0.5)
    f0 = converged_fraction(M, scene, prior, prm, ws, 1 << 16, seed=777)
    f1 = converged_fraction(M, scene, tree, prm, ws, 1 << 16, seed=777)
    print(dict(prior=f0, trained=f1), flush=True)
    assert f1 > f0 + 0.05
