"""Autotuner for the persistent batched walk.

Sweeps the knobs of the persistent form -- bucketing (none, by length, by
length and spatial cell), lane
refill on / off, waves per workgroup (1, 2, 4) and the LDS BVH stack depth
(the scene's minimum and larger) -- timing one manifold_walk_batch launch with HIP events on the
caller's batch, and returns the fastest setting.  With more lengths than
workers it then sweeps the order in which the per-length kernels are dealt to
the workers (longest first, or one length first and the rest longest first).  Every candidate produces the
same per-chain results (the knobs change scheduling only), which the tuner
checks against the first candidate's statuses.

Command line (on a GPU):

    python -m paper_2311_12818_amd.autotune --workload slab_uneven --out tuned.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

from . import (FORM_PERSISTENT, Endpoints, MPGError, Scene, Workspace, empty_chains, manifold_walk_batch,
               sample_seeds, walk_outputs, walk_params)


def candidates(min_depth: int):
    depths = sorted({min_depth, min_depth + 4, 2 * min_depth})
    for bucketing, refill, waves, depth in itertools.product((3, 2, 1, 0), (1, 0), (1, 2, 4), depths):
        if waves * depth * 64 * 4 > 64 * 1024 or (refill and not bucketing) or (bucketing == 3 and not refill):
            continue
        yield dict(bucketing=bucketing, refill=refill, waves_per_group=waves, stack_depth=depth)


def order_candidates(max_len: int):
    longest = list(range(8, 0, -1))
    yield dict(length_order=longest)
    for first in range(max_len, 0, -1):
        if first != 8:
            yield dict(length_order=[first] + [n for n in longest if n != first])


WORKERS = 4  # per-length kernels run on the caller's stream and three internal streams


def tune(scene: Scene, ep: Endpoints, base_kw: dict, reps: int = 3, log=None, fixed: dict | None = None):
    """Times every candidate on (scene, ep); returns (best knobs, table).  With
    ``fixed`` knobs only the length order is swept."""
    import torch
    N = ep.N
    min_depth = scene.stats()["max_depth"] + 1
    prm0 = walk_params(scene.scale, form=FORM_PERSISTENT, **base_kw)
    ws = Workspace(N)
    seeds = sample_seeds(scene, ep, prm0, ws=ws)
    prim, pos = empty_chains(N)
    outs = walk_outputs(N)
    stream = torch.cuda.current_stream()
    table = []
    ref_status = None

    def sweep(cands):
        nonlocal ref_status
        rows = []
        for knobs in cands:
            prm = walk_params(scene.scale, form=FORM_PERSISTENT, **base_kw, **knobs)
            try:
                manifold_walk_batch(scene, prm, ep, *seeds, out_prim=prim, out_pos=pos, outs=outs, ws=ws)
                torch.cuda.synchronize()
            except MPGError as exc:
                rows.append(dict(knobs, error=str(exc)))
                continue
            st = outs["status"].clone()
            if ref_status is None:
                ref_status = st
            same = bool(torch.equal(st, ref_status))
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                manifold_walk_batch(scene, prm, ep, *seeds, out_prim=prim, out_pos=pos, outs=outs, ws=ws)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            row = dict(knobs, ms=min(times), same_status=same)
            rows.append(row)
            if log:
                log(row)
        good = [r for r in rows if "ms" in r and r["same_status"]]
        if not good:
            raise MPGError("autotune: no candidate ran")
        return min(good, key=lambda r: r["ms"]), rows

    keys = ("bucketing", "refill", "waves_per_group", "stack_depth")
    if fixed is None:
        best, table = sweep(candidates(min_depth))
        fixed = {k: best[k] for k in keys}
    else:
        fixed = {k: fixed[k] for k in keys}
    result = dict(fixed)
    max_len = int(base_kw.get("max_len", 8))
    if fixed["bucketing"] and max_len > WORKERS:
        best, rows = sweep(dict(fixed, **o) for o in order_candidates(max_len))
        table += rows
        result["length_order"] = best["length_order"]
    return result, table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="slab_uneven")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", required=True, help="JSON file to update (one entry per workload)")
    ap.add_argument("--orders-only", action="store_true",
                    help="keep the workload's knobs in --out and sweep only the length order")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch

    import workloads as W
    scene_fn, ep_fn = W.WORKLOADS[args.workload]
    max_len = {"sphere_mirror": 1, "icosphere_tt": 2, "water_caustic": 1, "slab_uneven": 8, "slab_adjoint": 4}
    sizes = {"sphere_mirror": 4096, "icosphere_tt": 1 << 20, "water_caustic": 1 << 22, "slab_uneven": 1 << 23,
             "slab_adjoint": 1 << 20}
    N = args.n or sizes[args.workload]
    sc = scene_fn()
    scene = Scene(sc)
    ep = Endpoints(ep_fn(N))
    base = dict(cone_cos=math.cos(math.radians(W.SEED_CONE_DEG)), max_len=max_len[args.workload], defer_fp64=1)
    t0 = time.time()
    out = {}
    if os.path.exists(args.out):
        with open(args.out) as fh:
            out = json.load(fh)
    entry = out.get(args.workload, {})
    fixed = entry if args.orders_only else None
    best, table = tune(scene, ep, base, reps=args.reps, log=lambda r: print(json.dumps(r), flush=True), fixed=fixed)
    if args.orders_only:
        out[args.workload] = dict(entry, **best, order_table=table)
    else:
        out[args.workload] = dict(best, chains=N, device=torch.cuda.get_device_name(0), table=table)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({"workload": args.workload, "best": best, "seconds": time.time() - t0}), flush=True)


if __name__ == "__main__":
    main()
