"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
identical seeded inputs and compare them."""
import math

import numpy as np

import oracle as O
import workloads as W

KMAX = 8


def cone_cos():
    return math.cos(math.radians(W.SEED_CONE_DEG))


def oracle_seeds(osc, ep, **kw):
    prm = O.params(osc.scale, cone_cos=cone_cos())
    prim, pos, st = O.sample_seeds(osc, ep, prm=prm, **kw)
    return prim, pos.astype(np.float32), st


def to_np(t):
    return t.detach().cpu().numpy()


def compare_walks(ep, g, o, scale, min_conv=50, tag=""):
    """g: GPU outputs (numpy), o: oracle outputs.  Returns a stats dict and
    asserts the parity bar: same convergence decision and same solution id
    for >= 99.9% of chains, converged vertices within 1e-4 L."""
    N = ep.n
    gc = g["status"] == 0
    oc = o["status"] == 0
    agree = (gc == oc).mean()
    both = gc & oc
    same_sol = g["sol"][both].astype(np.uint64) == o["sol"][both]
    sol_agree = (np.sum(gc != oc) + np.sum(~same_sol)) / N
    err = np.zeros(N)
    for i in range(KMAX):
        m = both & (ep.length > i)
        d = np.linalg.norm(g["pos"][:, i, :] - o["pos"][:, i, :], axis=0)
        err = np.where(m, np.maximum(err, d), err)
    idx = np.nonzero(both)[0][same_sol]
    stats = dict(tag=tag, N=N, gpu_conv=float(gc.mean()), oracle_conv=float(oc.mean()), status_agree=float(agree),
                 mismatch_frac=float(sol_agree), max_vertex_err=float(err[idx].max()) if len(idx) else 0.0,
                 n_both=int(both.sum()))
    print(stats, flush=True)
    assert both.sum() >= min_conv, stats
    assert sol_agree <= 1e-3, stats
    assert err[idx].max() <= 1e-4 * scale, stats
    # integer triangle ids identical where the solution ids agree
    for i in range(KMAX):
        m = ep.length[idx] > i
        assert np.array_equal(g["prim"][i, idx][m], o["prim"][i, idx][m])
    return stats
