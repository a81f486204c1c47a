"""manifold_walk_batch_noalloc (the allocation-free entry point) against
manifold_walk_batch with a workspace: the same kernels, so every output must
agree bit for bit, on two calls in a row, the second with a smaller batch
(the static scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

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


def _run(M, fn, scene, prm, dep, prim0, pos0, st0, **kw):
    import torch
    n = dep.N
    prim, pos = M.empty_chains(n)
    outs = M.walk_outputs(n)
    fn(scene, prm, dep, prim0, pos0, st0, out_prim=prim, out_pos=pos, outs=outs, **kw)
    torch.cuda.synchronize()
    res = {k: GC.to_np(v).copy() for k, v in outs.items()}
    res["prim"] = GC.to_np(prim).copy()
    res["pos"] = GC.to_np(pos).copy()
    return res


@pytest.mark.parametrize("bucketing,refill", [(1, 1), (1, 0), (0, 0)])
def test_noalloc_walk_matches_workspace_walk(mpg, bucketing, refill):
    M = mpg
    sc = W.slab_stack_scene()
    scene = M.Scene(sc)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), form=M.FORM_PERSISTENT, bucketing=bucketing,
                        refill=refill, waves_per_group=1, stack_depth=32,
                        length_order=M.pack_length_order([3, 8, 7, 6, 5, 4, 2, 1]))
    for n, seed in [(1 << 18, 41), ((1 << 14) + 17, 42)]:
        print(dict(case="noalloc", n=n, seed=seed, bucketing=bucketing, refill=refill), flush=True)
        ep = W.slab_uneven_endpoints(n, seed=seed)
        dep = M.Endpoints(ep)
        ws = M.Workspace(n)
        prim0, pos0, st0 = M.sample_seeds(scene, dep, prm, ws=ws)
        a = _run(M, M.manifold_walk_batch, scene, prm, dep, prim0, pos0, st0, ws=ws)
        b = _run(M, M.manifold_walk_batch_noalloc, scene, prm, dep, prim0, pos0, st0)
        assert (a["status"] == M.CONVERGED).mean() > 0.3
        used = np.arange(8)[:, None] < ep.length[None, :]
        for k in a:
            if k == "prim":
                assert np.array_equal(a[k][used], b[k][used]), (n, k)
            elif k == "pos":
                assert np.array_equal(a[k][:, used], b[k][:, used]), (n, k)
            else:
                assert np.array_equal(a[k], b[k]), (n, k)


def test_noalloc_rejects_oversize_and_spatial_bucketing(mpg):
    import torch
    M = mpg
    sc = W.sphere_mirror_scene()
    scene = M.Scene(sc)
    L = M.lib()
    prm = M.walk_params(sc.scale, form=M.FORM_PERSISTENT, bucketing=1)
    big = M.mpg_endpoints(M.NOALLOC_MAX_CHAINS + 1, None, None, None, None, None, None)
    assert L.manifold_walk_batch_noalloc(scene.h, ctypes.byref(prm), ctypes.byref(big), None, None, None, None,
                                         None) == M.ERR_INVALID_ARG
    assert b"MPG_NOALLOC_MAX_CHAINS" in L.mpg_last_error()
    ep = W.sphere_mirror_endpoints(256)
    dep = M.Endpoints(ep)
    prim, pos = M.empty_chains(ep.n)
    outs = M.walk_outputs(ep.n)
    prm2 = M.walk_params(sc.scale, form=M.FORM_PERSISTENT, bucketing=2)
    with pytest.raises(M.MPGError):
        M.manifold_walk_batch_noalloc(scene, prm2, dep, prim, pos, None, out_prim=prim, out_pos=pos, outs=outs)
    torch.cuda.synchronize()
