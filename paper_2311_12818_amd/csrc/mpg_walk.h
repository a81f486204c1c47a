// Per-chain walk and finish routines shared by the plain and persistent forms.
#pragma once
#include "mpg_internal.h"

// Seed chain c: primitive ids and positions, validity (finite, in range,
// transmissions only at dielectrics, seed status 0).
template <int N>
__device__ __forceinline__ bool load_seed(const DevScene& S, const EpView& E, const WalkIO& io, int c, int type,
                                          int* prim, f3* x) {
  const size_t NN = E.N;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    prim[i] = io.seed_prim[i * NN + c];
    x[i] = {io.seed_pos[(0 * KMAX + i) * NN + c], io.seed_pos[(1 * KMAX + i) * NN + c],
            io.seed_pos[(2 * KMAX + i) * NN + c]};
  }
  bool seed_ok = !(io.seed_status && io.seed_status[c] != 0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    bool inr = prim[i] >= 0 ? prim[i] < S.n_tris : (prim[i] != PRIM_NONE && -1 - prim[i] < S.n_spheres);
    seed_ok = seed_ok && inr && finite3(x[i]);
  }
  if (seed_ok) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (((type >> i) & 1) && prim_material(S, prim[i]) != MAT_DIELECTRIC) seed_ok = false;
  }
  return seed_ok;
}

// Walk outcome of chain c.  Converged chains are stored as ST_PENDING: the
// finish pass (FP32) and, when flagged there or stalled in the walk, the
// FP64 pass complete them.
template <int N>
__device__ __forceinline__ void store_walk(const EpView& E, const WalkIO& io, int c, int status, int iters,
                                           bool have, const int* prim, const f3* x) {
  const size_t NN = E.N;
  if (status == ST_CONVERGED) status = ST_PENDING;
  io.status[c] = (int8_t)status;
  if (io.iters) io.iters[c] = (uint8_t)iters;
  if (io.sol) io.sol[c] = 0;
  if (io.G) io.G[c] = 0.f;
  if (io.kappa) io.kappa[c] = 0.f;
  if (io.resid) io.resid[c] = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    io.prim_out[i * NN + c] = have ? prim[i] : PRIM_NONE;
    io.pos_out[(0 * KMAX + i) * NN + c] = have ? x[i].x : 0.f;
    io.pos_out[(1 * KMAX + i) * NN + c] = have ? x[i].y : 0.f;
    io.pos_out[(2 * KMAX + i) * NN + c] = have ? x[i].z : 0.f;
  }
}

template <int N, class STK>
__device__ __forceinline__ void walk_one(const DevScene& S, const WalkParams& P, const EpView& E, const WalkIO& io, int c,
                         STK& stk) {
  int prim[N];
  f3 x[N];
  const int type = E.type[c];
  const bool seed_ok = load_seed<N>(S, E, io, c, type, prim, x);
  int status = ST_SEED_INVALID, it = 0;
  if (seed_ok)
    status = walk_core<N>(S, P, ld_pt(E.xD, E.N, c), ld_pt(E.xL, E.N, c), type, prim, x, it, stk, chain_offs(E, c));
  store_walk<N>(E, io, c, status, it, seed_ok, prim, x);
}

template <int NMAX, class STK>
__device__ __forceinline__ void walk_dispatch(const DevScene& S, const WalkParams& P, const EpView& E,
                                              const WalkIO& io, int c, STK& stk) {
  int n = E.len[c];
  if (n < 1 || n > NMAX || !finite3(ld_pt(E.xD, E.N, c)) || !finite3(ld_pt(E.xL, E.N, c)) ||
      !finite3(ld_pt(E.nD, E.N, c))) {
    io.status[c] = ST_BAD_INPUT;
    if (io.iters) io.iters[c] = 0;
    if (io.sol) io.sol[c] = 0;
    if (io.G) io.G[c] = 0.f;
    if (io.kappa) io.kappa[c] = 0.f;
    if (io.resid) io.resid[c] = 0.f;
    return;
  }
  switch (n) {
    case 1: walk_one<1>(S, P, E, io, c, stk); break;
    case 2: if (NMAX >= 2) walk_one<(NMAX >= 2 ? 2 : 1)>(S, P, E, io, c, stk); break;
    case 3: if (NMAX >= 3) walk_one<(NMAX >= 3 ? 3 : 1)>(S, P, E, io, c, stk); break;
    case 4: if (NMAX >= 4) walk_one<(NMAX >= 4 ? 4 : 1)>(S, P, E, io, c, stk); break;
    case 5: if (NMAX >= 5) walk_one<(NMAX >= 5 ? 5 : 1)>(S, P, E, io, c, stk); break;
    case 6: if (NMAX >= 6) walk_one<(NMAX >= 6 ? 6 : 1)>(S, P, E, io, c, stk); break;
    case 7: if (NMAX >= 7) walk_one<(NMAX >= 7 ? 7 : 1)>(S, P, E, io, c, stk); break;
    default: if (NMAX >= 8) walk_one<(NMAX >= 8 ? 8 : 1)>(S, P, E, io, c, stk); break;
  }
}

// Finish pass over the chains the walk left as ST_PENDING (FP32 side and
// visibility tests, kappa, G; near-singular or grazing chains become
// ST_NEEDS_FP64).
template <int N, class STK>
__device__ __forceinline__ void finish_one(const DevScene& S, const WalkParams& P, const EpView& E, const WalkIO& io, int c,
                           STK& stk) {
  const size_t NN = E.N;
  int prim[N];
  f3 x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    prim[i] = io.prim_out[i * NN + c];
    x[i] = {io.pos_out[(0 * KMAX + i) * NN + c], io.pos_out[(1 * KMAX + i) * NN + c],
            io.pos_out[(2 * KMAX + i) * NN + c]};
  }
  WalkOut R;
  R.sol = 0; R.G = 0.f; R.kappa = 0.f; R.resid = 0.f;
  finish<N>(S, P, ld_pt(E.xD, E.N, c), ld_pt(E.nD, E.N, c), ld_pt(E.xL, E.N, c), E.type[c], prim, x, stk, R,
            chain_offs(E, c));
  io.status[c] = (int8_t)R.status;
  if (io.sol) io.sol[c] = R.status == ST_CONVERGED ? R.sol : 0;
  if (io.G) io.G[c] = R.status == ST_CONVERGED ? R.G : 0.f;
  if (io.kappa) io.kappa[c] = R.status == ST_CONVERGED ? R.kappa : 0.f;
  if (io.resid) io.resid[c] = R.resid;
}

template <int NMAX, class STK>
__device__ __forceinline__ void finish_dispatch(const DevScene& S, const WalkParams& P, const EpView& E,
                                                const WalkIO& io, int c, STK& stk) {
  if (io.status[c] != ST_PENDING) return;
  int n = E.len[c];
  switch (n) {
    case 1: finish_one<1>(S, P, E, io, c, stk); break;
    case 2: if (NMAX >= 2) finish_one<(NMAX >= 2 ? 2 : 1)>(S, P, E, io, c, stk); break;
    case 3: if (NMAX >= 3) finish_one<(NMAX >= 3 ? 3 : 1)>(S, P, E, io, c, stk); break;
    case 4: if (NMAX >= 4) finish_one<(NMAX >= 4 ? 4 : 1)>(S, P, E, io, c, stk); break;
    case 5: if (NMAX >= 5) finish_one<(NMAX >= 5 ? 5 : 1)>(S, P, E, io, c, stk); break;
    case 6: if (NMAX >= 6) finish_one<(NMAX >= 6 ? 6 : 1)>(S, P, E, io, c, stk); break;
    case 7: if (NMAX >= 7) finish_one<(NMAX >= 7 ? 7 : 1)>(S, P, E, io, c, stk); break;
    default: if (NMAX >= 8) finish_one<(NMAX >= 8 ? 8 : 1)>(S, P, E, io, c, stk); break;
  }
}

// FP64 pass over one chain the walk left as ST_NEEDS_FP64.
template <int N, class STK>
__device__ __forceinline__ void fp64_one(const DevScene& S, const WalkParams& P, const EpView& E, const WalkIO& io, int c,
                         STK& stk) {
  const size_t NN = E.N;
  int prim[N];
  f3 x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    prim[i] = io.prim_out[i * NN + c];
    x[i] = {io.pos_out[(0 * KMAX + i) * NN + c], io.pos_out[(1 * KMAX + i) * NN + c],
            io.pos_out[(2 * KMAX + i) * NN + c]};
  }
  WalkOut R;
  R.sol = 0; R.G = 0.f; R.kappa = 0.f; R.resid = 0.f;
  finish_fp64<N>(S, P, ld_pt(E.xD, E.N, c), ld_pt(E.nD, E.N, c), ld_pt(E.xL, E.N, c), E.type[c], prim, x, stk, R,
                 chain_offs(E, c));
  io.status[c] = (int8_t)R.status;
  if (io.sol) io.sol[c] = R.status == ST_CONVERGED ? R.sol : 0;
  if (io.G) io.G[c] = R.status == ST_CONVERGED ? R.G : 0.f;
  if (io.kappa) io.kappa[c] = R.status == ST_CONVERGED ? R.kappa : 0.f;
  if (io.resid) io.resid[c] = R.resid;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    io.pos_out[(0 * KMAX + i) * NN + c] = x[i].x;
    io.pos_out[(1 * KMAX + i) * NN + c] = x[i].y;
    io.pos_out[(2 * KMAX + i) * NN + c] = x[i].z;
  }
}

// Seed chain of configuration c (sample_seed), stored as the walk reads it.
template <int N, class STK>
__device__ __forceinline__ void seed_one(const DevScene& S, const DevGuide* G, const WalkParams& P, const EpView& E, int c,
                         uint64_t seed, uint64_t trial, float alpha, int32_t* prim_out, float* pos_out, int8_t* st,
                         STK& stk) {
  int prim[N];
  f3 pos[N];
  int r = sample_seed<N>(S, G, P, E.type[c], E.obj1[c], ld_pt(E.xD, E.N, c), ld_pt(E.nD, E.N, c), seed,
                         (uint64_t)c, trial, alpha, prim, pos, stk, chain_offs(E, c));
  st[c] = (int8_t)r;
  const size_t NN = E.N;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    prim_out[i * NN + c] = r == 0 ? prim[i] : PRIM_NONE;
    pos_out[(0 * KMAX + i) * NN + c] = r == 0 ? pos[i].x : 0.f;
    pos_out[(1 * KMAX + i) * NN + c] = r == 0 ? pos[i].y : 0.f;
    pos_out[(2 * KMAX + i) * NN + c] = r == 0 ? pos[i].z : 0.f;
  }
}

