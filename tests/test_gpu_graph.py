"""The hot-path step (sample_seeds -> persistent manifold_walk_batch ->
manifold_walk_fp64) captured once into a HIP graph through torch's graph API
and replayed: every replay must reproduce the eager step bit for bit, with
eager work and synchronizations between the replays."""
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


def test_captured_step_replays_match_eager(mpg):
    import torch
    M = mpg
    n = 1 << 16
    sc = W.slab_stack_scene()
    ep = W.slab_uneven_endpoints(n, seed=11)
    scene = M.Scene(sc)
    dep = M.Endpoints(ep)
    prm = M.walk_params(sc.scale, cone_cos=GC.cone_cos(), max_len=8, defer_fp64=1, form=M.FORM_PERSISTENT)
    ws = M.Workspace(n)
    prim, pos = M.empty_chains(n)
    outs = M.walk_outputs(n)
    seed_status = torch.zeros(n, dtype=torch.int8, device="cuda")

    def step():
        p, q, st = M.sample_seeds(scene, dep, prm, out=(prim, pos), ws=ws)
        seed_status.copy_(st)
        M.manifold_walk_batch(scene, prm, dep, p, q, st, out_prim=prim, out_pos=pos, outs=outs, ws=ws)
        M.manifold_walk_fp64(scene, prm, dep, prim, pos, outs)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = {k: GC.to_np(v).copy() for k, v in outs.items()}
    ref_prim, ref_pos = GC.to_np(prim).copy(), GC.to_np(pos).copy()
    assert (ref["status"] == M.CONVERGED).mean() > 0.3

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    other = W.slab_uneven_endpoints(4096, seed=12)
    dep2 = M.Endpoints(other)
    for rep in range(3):
        # clobber every output, then run unrelated eager work before the replay
        for v in outs.values():
            v.fill_(-1) if v.dtype != torch.float32 else v.fill_(float("nan"))
        prim.fill_(-7)
        pos.fill_(float("nan"))
        p2, q2, s2 = M.sample_seeds(scene, dep2, prm, ws=ws)
        M.manifold_walk_batch(scene, prm, dep2, p2, q2, s2, ws=ws)   # reuses (clobbers) the workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert np.array_equal(GC.to_np(v), ref[k]), (rep, k)
        used = np.arange(8)[:, None] < ep.length[None, :]
        assert np.array_equal(GC.to_np(prim)[used], ref_prim[used]), rep
        got_pos = GC.to_np(pos)
        assert np.array_equal(got_pos[:, used], ref_pos[:, used]), rep
