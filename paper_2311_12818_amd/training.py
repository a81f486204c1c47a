"""Progressive training of the paper's guide (Sec. 5.8) over the library's
calls.  Every decision of the schedule comes from mpg_train_step; every
computation runs in the library's kernels: seeds from the current guide
(sample_seeds_stree, lengths drawn), walks (manifold_walk_batch), the
P(n)-factored reciprocal probability (estimate_inv_prob_stree), sample
records (make_guide_records) and the refit (fit_guide_stree) from the
records of the iteration that just ended."""
from __future__ import annotations

import time

from . import (RENDER, STree, Endpoints, Scene, estimate_inv_prob_stree, make_guide_records, manifold_walk_batch,
               mpg_train_plan, sample_seeds_stree, train_init, train_step)


def train_guide(scene: Scene, tree: STree, params, make_configs, budget: float, train_fraction: float = 0.3,
                base_samples: int = 1 << 14, batch: int = 1 << 14, max_trials: int = 16, seed: int = 0,
                clock=time.perf_counter, ws=None):
    """Runs the training stage.  make_configs(i, count) returns device
    Endpoints of `count` training configurations for batch i (lengths 0:
    drawn by the guide).  Returns a log with one entry per batch:
    (iteration, samples, converged, refit, elapsed).  ws: a Workspace of at
    least `batch` chains, needed when params select the persistent form."""
    import torch
    plan = mpg_train_plan(float(budget), float(train_fraction), int(base_samples))
    st = train_init(plan)
    t0 = clock()
    records = []
    log = []
    i = 0
    while st.phase != RENDER:
        count = batch if st.done >= st.target else min(batch, st.target - st.done)
        ep = make_configs(i, count)
        n, ty, pn, prim, pos, status = sample_seeds_stree(scene, tree, ep, params, seed=seed, trial=2 * i, ws=ws)
        wep = Endpoints.from_tensors(ep.xD, ep.nD, ep.xL, n, ty, ep.obj1)
        prim, pos, outs = manifold_walk_batch(scene, params, wep, prim, pos, status, out_prim=prim, out_pos=pos,
                                              ws=ws)
        _, ip, _, _ = estimate_inv_prob_stree(scene, tree, params, wep, prim, pos, outs["status"],
                                              max_trials=max_trials, seed=seed + 1 + i, ws=ws)
        records.append(make_guide_records(wep, pos, outs, ip))
        torch.cuda.synchronize()
        it = st.iteration
        train_step(plan, st, count, clock() - t0)
        conv = int((outs["status"] == 0).sum())
        if st.refit:
            tree.fit(torch.cat(records))
            records = []
        log.append((it, count, conv, bool(st.refit), clock() - t0))
        i += 1
    return log
