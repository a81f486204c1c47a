// The paper's guide on the GPU (Sec. 5.5, Sec. 5.6): a binary tree over the
// 6-D configuration (x_D, x_L) whose leaves hold discrete distributions of the
// chain length n and type tau and a mixture of von Mises-Fisher lobes over
// the first direction w_D, one lobe per sub-path sample with a nearest-
// neighbour footprint.  Seeds draw n (unless given) and (w_D, tau) from the
// defensive one-sample mixtures alpha p_0 + (1 - alpha) p_e; the reciprocal
// probability keeps n across trials and divides by the analytic P(n)
// (Sec. 5.8).  The tree is built from the sample records on the GPU
// (mpg_stree_build.hip); the footprints and everything per configuration run
// here.
#include "mpg_internal.h"
#include "mpg_stree_build.h"

namespace {

struct DevSTree {
  const int* axis;            // [nodes] split axis (0..5), -1 for a leaf
  const float* mid;           // [nodes] split plane
  const int* child;           // [nodes] left child (right = left + 1)
  const float* W;             // [nodes] leaf weight
  const float* Wn;            // [nodes][8] leaf weight per length
  const int* own;             // [nodes] own samples of a leaf
  const int2* leaf_groups;    // [nodes] (first group, count)
  const int* grp_key;         // [groups] n | tau << 8
  const float* grp_w;         // [groups]
  const int2* grp_lobes;      // [groups] (first lobe, count)
  const float4* lobe;         // [lobes] mean direction, kappa
  const float* lobe_cdf;      // [lobes] inclusive prefix of lobe weights within the group
  float p0n[KMAX];            // P_0(n), n = 1..8, normalised
  float alpha, p_transmit;
};

__device__ __forceinline__ int stree_leaf(const DevSTree& T, const float* q) {
  int k = 0;
  for (int a; (a = T.axis[k]) >= 0;) k = T.child[k] + (q[a] < T.mid[k] ? 0 : 1);
  return k;
}

// inverse CDF over non-negative weights: first i whose running sum exceeds
// u total, else the last positive weight
__device__ __forceinline__ int pick8(const float* w, float total, float u) {
  float target = u * total, acc = 0.0f;
  int last = KMAX - 1;
  for (int i = 0; i < KMAX; ++i) {
    acc += w[i];
    if (target < acc) return i;
  }
  for (int i = KMAX - 1; i >= 0; --i)
    if (w[i] > 0.0f) return i;
  return last;
}

__device__ __forceinline__ float stree_pn(const DevSTree& T, int leaf, int n) {
  const float W = T.W[leaf];
  if (!(W > 0.0f)) return T.p0n[n - 1];
  return T.alpha * T.p0n[n - 1] + (1.0f - T.alpha) * T.Wn[(size_t)leaf * KMAX + n - 1] / W;
}

// The length: alpha P_0(n) + (1 - alpha) P_e(n | leaf) (P_0 alone for a leaf
// without samples).
__device__ __forceinline__ int stree_length(const DevSTree& T, int leaf, const U8& U) {
  const float W = T.W[leaf];
  const bool prior = !(W > 0.0f) || U.u[0] < T.alpha;
  if (prior) return 1 + pick8(T.p0n, 1.0f, U.u[1]);
  return 1 + pick8(T.Wn + (size_t)leaf * KMAX, W, U.u[1]);
}

// (w_D, tau) of a chain of length N and its seed chain: p_0 (x_1 by the obj1
// mode, tau decided at each vertex as it is reached) with probability alpha
// or when the leaf holds no chain of this length, else tau from P_e(tau | n),
// a lobe by weight and w_D from the lobe.
template <int N, class STK>
__device__ __forceinline__ int stree_seed(const DevScene& S, const DevSTree& T, const WalkParams& P, int leaf,
                                          int obj1, f3 xD, f3 nD, uint64_t seed, uint64_t chain, uint64_t trial,
                                          const U8& U, int* prim, f3* pos, int* type_out, STK& stk) {
  const float Wn = T.Wn[(size_t)leaf * KMAX + N - 1];
  const bool prior = !(Wn > 0.0f) || U.u[2] < T.alpha;
  if (prior) {
    U8 V = philox_uniforms(seed, chain, trial, 1);
    f3 pt;
    if (!p0_point(S, P, obj1, xD, nD, V.u[1], V.u[2], V.u[3], pt)) return ST_SEED_INVALID;
    U8 Cn = philox_uniforms(seed, chain, trial, 2);
    *type_out = 0;
    return deduce<N, true>(S, P, 0, Cn.u, T.p_transmit, xD, pt, prim, pos, stk, type_out);
  }
  const int2 gr = T.leaf_groups[leaf];
  float target = U.u[3] * Wn, acc = 0.0f;
  int g = -1, last = -1;
  for (int q = gr.x; q < gr.x + gr.y; ++q) {
    if ((T.grp_key[q] & 0xff) != N) continue;
    const float w = T.grp_w[q];
    if (w > 0.0f) last = q;
    acc += w;
    if (g < 0 && target < acc) g = q;
  }
  if (g < 0) g = last;
  if (g < 0) return ST_SEED_INVALID;
  const int type = T.grp_key[g] >> 8;
  const int2 lr = T.grp_lobes[g];
  const float t2 = U.u[4] * T.grp_w[g];
  int lo = 0, hi = lr.y;  // first lobe whose prefix exceeds t2
  while (lo < hi) {
    int m = (lo + hi) >> 1;
    if (T.lobe_cdf[lr.x + m] > t2) hi = m;
    else lo = m + 1;
  }
  if (lo >= lr.y) lo = lr.y - 1;
  const float4 L = T.lobe[lr.x + lo];
  const f3 mu = {L.x, L.y, L.z};
  const float kappa = L.w;
  // vMF (Eq. vMF) by inversion: 1 - cos theta = -log(u + (1 - u) e^{-2 kappa}) / kappa
  float v = -logf(U.u[5] + (1.0f - U.u[5]) * expf(-2.0f * kappa)) / kappa;
  v = fminf(fmaxf(v, 0.0f), 2.0f);
  const float ct = 1.0f - v, st = sqrtf(fmaxf(0.0f, v * (2.0f - v)));
  f3 b1, b2;
  onb(mu, b1, b2);
  float sn, cs;
  sincospif(2.0f * U.u[6], &sn, &cs);
  const f3 w = b1 * (st * cs) + b2 * (st * sn) + mu * ct;
  *type_out = type;
  return deduce<N, false>(S, P, type, nullptr, 0.0f, xD, xD + w, prim, pos, stk, nullptr);
}

__device__ __forceinline__ void query6(const EpView& E, int c, float* q) {
  const size_t N = E.N;
  q[0] = E.xD[c]; q[1] = E.xD[N + c]; q[2] = E.xD[2 * N + c];
  q[3] = E.xL[c]; q[4] = E.xL[N + c]; q[5] = E.xL[2 * N + c];
}

struct SeedOut {
  uint8_t* len;
  uint8_t* type;
  float* pn;
  int32_t* prim;
  float* pos;
  int8_t* status;
};

template <int N, class STK>
__device__ __forceinline__ void stree_seed_one(const DevScene& S, const DevSTree& T, const WalkParams& P,
                                               const EpView& E, int c, int leaf, uint64_t seed, uint64_t trial,
                                               const U8& U, const SeedOut& o, STK& stk) {
  const size_t NN = E.N;
  int prim[N], type = 0;
  f3 pos[N];
  int st = stree_seed<N>(S, T, P, leaf, E.obj1[c], ld_pt(E.xD, E.N, c), ld_pt(E.nD, E.N, c), seed, (uint64_t)c,
                         trial, U, prim, pos, &type, stk);
  o.status[c] = (int8_t)st;
  o.type[c] = (uint8_t)type;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    o.prim[i * NN + c] = st == 0 ? prim[i] : PRIM_NONE;
    o.pos[(0 * KMAX + i) * NN + c] = st == 0 ? pos[i].x : 0.0f;
    o.pos[(1 * KMAX + i) * NN + c] = st == 0 ? pos[i].y : 0.0f;
    o.pos[(2 * KMAX + i) * NN + c] = st == 0 ? pos[i].z : 0.0f;
  }
}

// The configuration's leaf and length: n = ep->d_len[c] when it is 1..8,
// else drawn from the leaf; false for non-finite inputs or a fixed length
// above 8.
__device__ __forceinline__ bool stree_config(const DevSTree& T, const EpView& E, int c, uint64_t seed,
                                             uint64_t trial, int* leaf, U8* U, int* n) {
  float q[6];
  query6(E, c, q);
  const int nfix = E.len[c];
  bool ok = nfix <= KMAX;
  for (int a = 0; a < 6; ++a) ok = ok && isfinite(q[a]);
  ok = ok && finite3(ld_pt(E.nD, E.N, c));
  if (!ok) return false;
  *leaf = stree_leaf(T, q);
  *U = philox_uniforms(seed, (uint64_t)c, trial, 0);
  *n = nfix >= 1 ? nfix : stree_length(T, *leaf, *U);
  return true;
}

__device__ __forceinline__ void stree_bad_input(const SeedOut& o, int c) {
  o.status[c] = ST_BAD_INPUT;
  o.len[c] = 0;
  o.type[c] = 0;
  o.pn[c] = 0.0f;
}

__global__ void __launch_bounds__(256) k_stree_seeds(DevScene S, DevSTree T, WalkParams P, EpView E, uint64_t seed,
                                                     uint64_t trial, SeedOut o) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  int leaf, n;
  U8 U;
  if (!stree_config(T, E, c, seed, trial, &leaf, &U, &n)) {
    stree_bad_input(o, c);
    return;
  }
  o.len[c] = (uint8_t)n;
  o.pn[c] = stree_pn(T, leaf, n);
  switch (n) {
    case 1: stree_seed_one<1>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    case 2: stree_seed_one<2>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    case 3: stree_seed_one<3>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    case 4: stree_seed_one<4>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    case 5: stree_seed_one<5>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    case 6: stree_seed_one<6>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    case 7: stree_seed_one<7>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
    default: stree_seed_one<8>(S, T, P, E, c, leaf, seed, trial, U, o, stk); break;
  }
}

// Persistent form of the seeds: the lengths are drawn first (class = n, 0
// for bad inputs, whose outputs are written here), the configurations
// bucketed by length, and each length's seeds drawn by a kernel of its own
// (same leaf, uniforms and length as the plain form, so the same seeds).
__global__ void __launch_bounds__(256) k_stree_draw(DevSTree T, EpView E, uint64_t seed, uint64_t trial, SeedOut o,
                                                    int8_t* cls) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  int leaf, n;
  U8 U;
  if (!stree_config(T, E, c, seed, trial, &leaf, &U, &n)) {
    stree_bad_input(o, c);
    cls[c] = 0;
    return;
  }
  o.len[c] = (uint8_t)n;
  o.pn[c] = stree_pn(T, leaf, n);
  cls[c] = (int8_t)n;
}

template <int N>
__global__ void __launch_bounds__(256) k_stree_seeds_persist(DevScene S, DevSTree T, WalkParams P, EpView E,
                                                             uint64_t seed, uint64_t trial, SeedOut o, int* ctr,
                                                             const int* perm) {
  Stack stk = lane_stack(P.depth);
  const int start = ctr[CTR_OFF + N];
  const int end = ctr[CTR_OFF + N + 1];
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int base = next_batch(&ctr[CTR_HEAD3 + N - 1]);
    if (start + base >= end) break;
    const int c = perm[start + base + lane];
    if (c >= 0) {
      int leaf, n;
      U8 U;
      stree_config(T, E, c, seed, trial, &leaf, &U, &n);
      stree_seed_one<N>(S, T, P, E, c, leaf, seed, trial, U, o, stk);
    }
  }
}

typedef void (*stree_seed_kernel_t)(DevScene, DevSTree, WalkParams, EpView, uint64_t, uint64_t, SeedOut, int*,
                                    const int*);
static stree_seed_kernel_t stree_seed_kernel(int n) {
  switch (n) {
    case 1: return k_stree_seeds_persist<1>;
    case 2: return k_stree_seeds_persist<2>;
    case 3: return k_stree_seeds_persist<3>;
    case 4: return k_stree_seeds_persist<4>;
    case 5: return k_stree_seeds_persist<5>;
    case 6: return k_stree_seeds_persist<6>;
    case 7: return k_stree_seeds_persist<7>;
    default: return k_stree_seeds_persist<8>;
  }
}

struct StreeInvIO {
  const int32_t* tprim;
  const float* tpos;
  const int8_t* tstatus;
  int32_t* trials;
  float* inv_prob;
  uint8_t* truncated;
  float* pn;
  int max_trials, repeats;
  uint64_t seed;
  int max_len;  // targets longer than this are left out (outputs 0)
};

template <int N, class STK>
__device__ __forceinline__ void stree_inv_one(const DevScene& S, const DevSTree& T, const WalkParams& P,
                                              const EpView& E, const StreeInvIO& io, int c, int leaf, STK& stk) {
  const size_t NN = E.N;
  f3 tx[N];
  int tobj[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    tx[i] = {io.tpos[(0 * KMAX + i) * NN + c], io.tpos[(1 * KMAX + i) * NN + c], io.tpos[(2 * KMAX + i) * NN + c]};
    tobj[i] = prim_obj(S, io.tprim[i * NN + c]);
  }
  const f3 xD = ld_pt(E.xD, E.N, c), nD = ld_pt(E.nD, E.N, c), xL = ld_pt(E.xL, E.N, c);
  const int ttype = E.type[c], obj1 = E.obj1[c];
  int total = 0;
  bool trunc = false;
  for (int r = 0; r < io.repeats; ++r) {
    int K = io.max_trials;
    bool found = false;
    for (int k = 1; k <= io.max_trials && !found; ++k) {
      const uint64_t trial = 1 + (uint64_t)r * io.max_trials + (uint64_t)(k - 1);
      const U8 U = philox_uniforms(io.seed, (uint64_t)c, trial, 0);
      int prim[N], type = 0;
      f3 x[N];
      if (stree_seed<N>(S, T, P, leaf, obj1, xD, nD, io.seed, (uint64_t)c, trial, U, prim, x, &type, stk) != 0)
        continue;
      if (type != ttype) continue;
      int it;
      const int ws = walk_core<N>(S, P, xD, xL, type, prim, x, it, stk);
      if (ws != ST_CONVERGED && ws != ST_NEEDS_FP64) continue;
      bool m = true;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        f3 d = x[i] - tx[i];
        m = m && prim_obj(S, prim[i]) == tobj[i] && dot(d, d) <= P.match2;
      }
      if (m) { K = k; found = true; }
    }
    if (!found) trunc = true;
    total += K;
  }
  const float pn = stree_pn(T, leaf, N);
  io.trials[c] = total;
  io.pn[c] = pn;
  io.inv_prob[c] = pn > 0.0f ? (float)total / (float)io.repeats / pn : 0.0f;
  if (io.truncated) io.truncated[c] = trunc ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_stree_inv(DevScene S, DevSTree T, WalkParams P, EpView E, StreeInvIO io) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  const int n = E.len[c];
  if (io.tstatus[c] != ST_CONVERGED || n < 1 || n > io.max_len || io.repeats < 1 || io.max_trials < 1) {
    io.trials[c] = 0;
    io.inv_prob[c] = 0.0f;
    io.pn[c] = 0.0f;
    if (io.truncated) io.truncated[c] = 0;
    return;
  }
  float q[6];
  query6(E, c, q);
  const int leaf = stree_leaf(T, q);
  switch (n) {
    case 1: stree_inv_one<1>(S, T, P, E, io, c, leaf, stk); break;
    case 2: stree_inv_one<2>(S, T, P, E, io, c, leaf, stk); break;
    case 3: stree_inv_one<3>(S, T, P, E, io, c, leaf, stk); break;
    case 4: stree_inv_one<4>(S, T, P, E, io, c, leaf, stk); break;
    case 5: stree_inv_one<5>(S, T, P, E, io, c, leaf, stk); break;
    case 6: stree_inv_one<6>(S, T, P, E, io, c, leaf, stk); break;
    case 7: stree_inv_one<7>(S, T, P, E, io, c, leaf, stk); break;
    default: stree_inv_one<8>(S, T, P, E, io, c, leaf, stk); break;
  }
}

// Persistent form of the trials: targets bucketed by length, one kernel per
// length in which every lane owns one target at a time and advances it by
// one step per turn of the loop: a new trial (guided seed; a seed that fails
// or draws another type ends the trial at once) or one walk step; a lane
// whose target is done takes the next target of the bucket in the same
// turn.  The trials of a target are the plain form's, in the same order, so
// the results are identical.  Lanes waiting for a new trial start together
// (at least half of the busy lanes, or no lane walking), so that their seed
// rays are cast together.
__global__ void __launch_bounds__(256) k_stree_classify(EpView E, StreeInvIO io, int8_t* cls) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  const int n = E.len[c];
  const bool target = io.tstatus[c] == ST_CONVERGED && n >= 1 && n <= io.max_len && io.repeats >= 1 &&
                      io.max_trials >= 1;
  cls[c] = (int8_t)(target ? n : 0);
  if (!target) {
    io.trials[c] = 0;
    io.inv_prob[c] = 0.0f;
    io.pn[c] = 0.0f;
    if (io.truncated) io.truncated[c] = 0;
  }
}

template <int N>
__global__ void __launch_bounds__(256) k_stree_inv_refill(DevScene S, DevSTree T, WalkParams P, EpView E,
                                                          StreeInvIO io, int* ctr, const int* perm) {
  Stack stk = lane_stack(P.depth);
  const size_t NN = E.N;
  const int start = ctr[CTR_OFF + N];
  const int count = ctr[CTR_HIST + N];
  int* head = &ctr[CTR_HEAD4 + N - 1];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  int c = -1;
  bool drained = false;
  // the target chain stays in memory (read back when a trial converges)
  // rather than in 4 N registers held through every walk step
  f3 xD = {0.f, 0.f, 0.f}, nD = {0.f, 0.f, 1.f}, xL = {0.f, 0.f, 0.f};
  int ttype = 0, obj1 = 0, leaf = 0;
  int r = 0, k = 0, total = 0;
  bool trunc = false, walking = false;
  WalkState<N> w;
  for (;;) {
    const unsigned long long idle = __ballot(c < 0);
    if (idle && !drained) {
      const int nidle = __popcll(idle);
      int base = 0;
      if (lane == 0) base = atomicAdd(head, nidle);
      base = __shfl(base, 0, 64);
      if (c < 0) {
        const int slot = base + __popcll(idle & below);
        if (slot < count) {
          c = perm[start + slot];
          xD = ld_pt(E.xD, E.N, c);
          nD = ld_pt(E.nD, E.N, c);
          xL = ld_pt(E.xL, E.N, c);
          ttype = E.type[c];
          obj1 = E.obj1[c];
          float q[6];
          query6(E, c, q);
          leaf = stree_leaf(T, q);
          r = 0;
          k = 0;
          total = 0;
          trunc = false;
          walking = false;
        }
      }
      if (base + nidle >= count) drained = true;
    }
    if (__ballot(c >= 0) == 0) {
      if (drained) break;
      continue;
    }
    const unsigned long long waiting = __ballot(c >= 0 && !walking);
    const unsigned long long busy = __ballot(c >= 0);
    const bool start_trials = 2 * __popcll(waiting) >= __popcll(busy);
    bool finished = false;
    if (c >= 0 && !walking && start_trials) {
      if (k == io.max_trials) {  // no match within the budget: K = max_trials, truncated
        trunc = true;
        total += io.max_trials;
        ++r;
        k = 0;
        finished = r == io.repeats;
      }
      if (!finished) {
        ++k;
        const uint64_t trial = 1 + (uint64_t)r * io.max_trials + (uint64_t)(k - 1);
        const U8 U = philox_uniforms(io.seed, (uint64_t)c, trial, 0);
        int type = 0;
        if (stree_seed<N>(S, T, P, leaf, obj1, xD, nD, io.seed, (uint64_t)c, trial, U, w.prim, w.x, &type, stk) ==
                0 &&
            type == ttype) {
          walk_begin<N>(S, w);
          walking = true;
        }
      }
    }
    if (c >= 0 && walking) {
      const int st = walk_step<N>(S, P, xD, xL, ttype, w, stk);
      if (st >= 0) {
        walking = false;
        bool m = st == ST_CONVERGED || st == ST_NEEDS_FP64;
        if (m) {
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const f3 t = {io.tpos[(0 * KMAX + i) * NN + c], io.tpos[(1 * KMAX + i) * NN + c],
                          io.tpos[(2 * KMAX + i) * NN + c]};
            const f3 d = w.x[i] - t;
            m = m && prim_obj(S, w.prim[i]) == prim_obj(S, io.tprim[i * NN + c]) && dot(d, d) <= P.match2;
          }
        }
        if (m) {
          total += k;
          ++r;
          k = 0;
          finished = r == io.repeats;
        }
      }
    }
    if (finished) {
      const float pn = stree_pn(T, leaf, N);
      io.trials[c] = total;
      io.pn[c] = pn;
      io.inv_prob[c] = pn > 0.0f ? (float)total / (float)io.repeats / pn : 0.0f;
      if (io.truncated) io.truncated[c] = trunc ? 1 : 0;
      c = -1;
    }
  }
}

typedef void (*stree_inv_kernel_t)(DevScene, DevSTree, WalkParams, EpView, StreeInvIO, int*, const int*);
static stree_inv_kernel_t stree_inv_refill_kernel(int n) {
  switch (n) {
    case 1: return k_stree_inv_refill<1>;
    case 2: return k_stree_inv_refill<2>;
    case 3: return k_stree_inv_refill<3>;
    case 4: return k_stree_inv_refill<4>;
    case 5: return k_stree_inv_refill<5>;
    case 6: return k_stree_inv_refill<6>;
    case 7: return k_stree_inv_refill<7>;
    default: return k_stree_inv_refill<8>;
  }
}

// Lobe footprints: for every lobe the angle sigma to the nearest other lobe
// direction of its group (as 2 asin(chord / 2), exact for small angles),
// floored at sigma_min, sigma_lone for a lobe alone in its group; kappa =
// sigma^-2.  One workgroup per group.
__global__ void __launch_bounds__(256) k_stree_footprint(const int2* grp_lobes, int n_groups, float4* lobe,
                                                         float sigma_min, float sigma_lone) {
  const int g = blockIdx.x;
  if (g >= n_groups) return;
  const int2 r = grp_lobes[g];
  for (int j = threadIdx.x; j < r.y; j += blockDim.x) {
    const float4 a = lobe[r.x + j];
    float best = INFINITY;
    for (int k = 0; k < r.y; ++k) {
      if (k == j) continue;
      const float4 b = lobe[r.x + k];
      const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
      best = fminf(best, dx * dx + dy * dy + dz * dz);
    }
    float sigma = r.y == 1 ? sigma_lone : fmaxf(2.0f * asinf(fminf(1.0f, 0.5f * sqrtf(best))), sigma_min);
    lobe[r.x + j].w = 1.0f / (sigma * sigma);
  }
}

// Sample records {x_D, x_L, w_D, w, n, tau, 0 x 4} of walked chains with
// w = T <1/P> (Eq. eq_weight), T = kappa G (L_o = 1); w = 0 unless converged.
__global__ void k_stree_records(EpView E, const float* pos, const int8_t* status, const float* G, const float* kap,
                                const float* inv_prob, float* rec) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  const size_t NN = E.N;
  const f3 xD = ld_pt(E.xD, E.N, c), xL = ld_pt(E.xL, E.N, c);
  const f3 x1 = {pos[c], pos[KMAX * NN + c], pos[2 * KMAX * NN + c]};
  const bool conv = status[c] == ST_CONVERGED;
  f3 w = x1 - xD;
  const float l2 = dot(w, w);
  w = conv && l2 > 0.0f ? w * rsqrtf(l2) : f3{0.0f, 0.0f, 0.0f};
  const float wt = conv ? kap[c] * G[c] * inv_prob[c] : 0.0f;
  float* r = rec + 16 * (size_t)c;
  const float v[16] = {xD.x, xD.y, xD.z, xL.x, xL.y, xL.z, w.x, w.y, w.z, (isfinite(wt) ? wt : 0.0f),
                       (float)E.len[c], (float)E.type[c], 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < 16; ++a) r[a] = v[a];
}

// Selective activation (Sec. 5.8): 1 when the configuration's leaf holds own
// samples (samples kept only for the child overlap do not count), else 0.
__global__ void k_stree_active(DevSTree T, EpView E, uint8_t* active) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  float q[6];
  query6(E, c, q);
  bool ok = true;
  for (int a = 0; a < 6; ++a) ok = ok && isfinite(q[a]);
  active[c] = ok && T.own[stree_leaf(T, q)] > 0 ? 1 : 0;
}

}  // namespace

struct mpg_stree {
  mpg_stree_desc desc;
  DevSTree dev;
  std::vector<void*> allocs;
  int n_nodes = 0, n_leaves = 0, n_groups = 0, n_lobes = 0;
  int fitted = 0;
};

static void stree_prior(mpg_stree* t) {
  float tot = 0.0f;
  for (int k = 0; k < KMAX; ++k) tot += t->desc.p0n[k];
  for (int k = 0; k < KMAX; ++k) t->dev.p0n[k] = tot > 0.0f ? t->desc.p0n[k] / tot : 0.0f;
  t->dev.alpha = t->desc.alpha;
  t->dev.p_transmit = t->desc.p_transmit;
}

static mpg_status check_desc(const mpg_stree_desc* d) {
  for (int a = 0; a < 6; ++a)
    if (!(d->hi[a] > d->lo[a])) return fail(MPG_ERR_INVALID_ARG, "mpg_stree: empty root box");
  if (!(d->eps >= 0.0f && d->eps < 1.0f) || !(d->thr_scale > 0.0f) || d->max_depth < 0 || d->max_depth > 64 ||
      !(d->sigma_min > 0.0f) || !(d->sigma_lone > 0.0f) || !(d->alpha >= 0.0f && d->alpha <= 1.0f) ||
      !(d->p_transmit >= 0.0f && d->p_transmit <= 1.0f))
    return fail(MPG_ERR_INVALID_ARG, "mpg_stree: parameter out of range");
  float tot = 0.0f;
  for (int k = 0; k < KMAX; ++k) {
    if (!(d->p0n[k] >= 0.0f)) return fail(MPG_ERR_INVALID_ARG, "mpg_stree: negative P_0(n)");
    tot += d->p0n[k];
  }
  if (!(tot > 0.0f)) return fail(MPG_ERR_INVALID_ARG, "mpg_stree: P_0(n) sums to zero");
  return MPG_OK;
}

extern "C" mpg_status mpg_stree_desc_default(mpg_stree_desc* d) {
  if (!d) return fail(MPG_ERR_INVALID_ARG, "mpg_stree_desc_default: NULL");
  std::memset(d, 0, sizeof(*d));
  for (int a = 0; a < 6; ++a) { d->lo[a] = 0.0f; d->hi[a] = 1.0f; }
  d->eps = 0.1f;
  d->thr_scale = 1.0f;
  d->max_depth = 20;
  d->sigma_min = 1e-3f;
  d->sigma_lone = 0.1f;
  for (int k = 0; k < KMAX; ++k) d->p0n[k] = 1.0f / KMAX;
  d->alpha = 0.5f;
  d->p_transmit = 0.5f;
  return MPG_OK;
}

extern "C" mpg_status mpg_stree_create(const mpg_stree_desc* d, mpg_stree** out) {
  if (!d || !out) return fail(MPG_ERR_INVALID_ARG, "mpg_stree_create: NULL argument");
  mpg_status st = check_desc(d);
  if (st != MPG_OK) return st;
  mpg_stree* t = new mpg_stree();
  t->desc = *d;
  std::memset(&t->dev, 0, sizeof(t->dev));
  stree_prior(t);
  // an empty tree: one leaf without samples (p_0 only)
  const int axis = -1, child = -1, zero_i = 0;
  const float zero_f = 0.0f;
  const float zeros8[KMAX] = {0};
  const int2 none = make_int2(0, 0);
  hipError_t e;
  if ((e = upload(t->allocs, &t->dev.axis, &axis, 1)) != hipSuccess ||
      (e = upload(t->allocs, &t->dev.mid, &zero_f, 1)) != hipSuccess ||
      (e = upload(t->allocs, &t->dev.child, &child, 1)) != hipSuccess ||
      (e = upload(t->allocs, &t->dev.W, &zero_f, 1)) != hipSuccess ||
      (e = upload(t->allocs, &t->dev.Wn, zeros8, KMAX)) != hipSuccess ||
      (e = upload(t->allocs, &t->dev.own, &zero_i, 1)) != hipSuccess ||
      (e = upload(t->allocs, &t->dev.leaf_groups, &none, 1)) != hipSuccess) {
    free_all(t->allocs);
    delete t;
    return fail(MPG_ERR_HIP, std::string("mpg_stree_create: ") + hipGetErrorString(e));
  }
  t->n_nodes = 1;
  t->n_leaves = 1;
  *out = t;
  return MPG_OK;
}

extern "C" void mpg_stree_destroy(mpg_stree* t) {
  if (!t) return;
  free_all(t->allocs);
  delete t;
}

extern "C" mpg_status mpg_stree_set_prior(mpg_stree* t, const float* p0n, float alpha, float p_transmit) {
  if (!t || !p0n) return fail(MPG_ERR_INVALID_ARG, "mpg_stree_set_prior: NULL argument");
  mpg_stree_desc d = t->desc;
  for (int k = 0; k < KMAX; ++k) d.p0n[k] = p0n[k];
  d.alpha = alpha;
  d.p_transmit = p_transmit;
  mpg_status st = check_desc(&d);
  if (st != MPG_OK) return st;
  t->desc = d;
  stree_prior(t);
  return MPG_OK;
}

extern "C" mpg_status fit_guide_stree(mpg_stree* t, const float* d_records, int32_t n_records, void* stream_) {
  if (!t || (n_records > 0 && !d_records) || n_records < 0)
    return fail(MPG_ERR_INVALID_ARG, "fit_guide_stree: bad argument");
  hipStream_t stream = (hipStream_t)stream_;
  StreeBuildParams prm;
  for (int a = 0; a < 6; ++a) { prm.lo[a] = t->desc.lo[a]; prm.hi[a] = t->desc.hi[a]; }
  prm.eps = t->desc.eps;
  prm.thr_scale = t->desc.thr_scale;
  prm.max_depth = t->desc.max_depth;
  // the new tree is built into arrays of its own; the previous one is
  // released once the build has succeeded
  std::vector<void*> fresh;
  StreeBuilt B;
  mpg_status st = stree_build_gpu(d_records, n_records, prm, fresh, &B, stream);
  if (st != MPG_OK) {
    free_all(fresh);
    return st;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) {
    free_all(fresh);
    return fail(MPG_ERR_HIP, "fit_guide_stree: stream synchronisation failed");
  }
  free_all(t->allocs);
  t->allocs.swap(fresh);
  std::memset(&t->dev, 0, sizeof(t->dev));
  stree_prior(t);
  t->dev.axis = B.axis;
  t->dev.mid = B.mid;
  t->dev.child = B.child;
  t->dev.W = B.W;
  t->dev.Wn = B.Wn;
  t->dev.own = B.own;
  t->dev.leaf_groups = B.leaf_groups;
  t->dev.grp_key = B.grp_key;
  t->dev.grp_w = B.grp_w;
  t->dev.grp_lobes = B.grp_lobes;
  t->dev.lobe = B.lobe;
  t->dev.lobe_cdf = B.lobe_cdf;
  t->n_nodes = B.n_nodes;
  t->n_leaves = B.n_leaves;
  t->n_groups = B.n_groups;
  t->n_lobes = B.n_lobes;
  if (t->n_groups > 0) {
    hipLaunchKernelGGL(k_stree_footprint, dim3(t->n_groups), dim3(256), 0, stream, t->dev.grp_lobes, t->n_groups,
                       B.lobe, t->desc.sigma_min, t->desc.sigma_lone);
    HIP_TRY(hipGetLastError());
  }
  t->fitted = 1;
  return MPG_OK;
}

extern "C" mpg_status mpg_stree_stats(const mpg_stree* t, int32_t* n_nodes, int32_t* n_leaves, int32_t* n_groups,
                                      int32_t* n_lobes) {
  if (!t) return fail(MPG_ERR_INVALID_ARG, "mpg_stree_stats: NULL tree");
  if (n_nodes) *n_nodes = t->n_nodes;
  if (n_leaves) *n_leaves = t->n_leaves;
  if (n_groups) *n_groups = t->n_groups;
  if (n_lobes) *n_lobes = t->n_lobes;
  return MPG_OK;
}

extern "C" mpg_status mpg_stree_download(const mpg_stree* t, int32_t* axis, float* mid, int32_t* child, float* W,
                                         float* Wn, int32_t* own, int32_t* leaf_groups, int32_t* grp_key,
                                         float* grp_w, int32_t* grp_lobes, float* lobe, float* lobe_cdf) {
  if (!t) return fail(MPG_ERR_INVALID_ARG, "mpg_stree_download: NULL tree");
  HIP_TRY(hipDeviceSynchronize());
  const size_t nn = t->n_nodes, ng = t->n_groups, nl = t->n_lobes;
  if (axis) HIP_TRY(hipMemcpy(axis, t->dev.axis, nn * 4, hipMemcpyDeviceToHost));
  if (mid) HIP_TRY(hipMemcpy(mid, t->dev.mid, nn * 4, hipMemcpyDeviceToHost));
  if (child) HIP_TRY(hipMemcpy(child, t->dev.child, nn * 4, hipMemcpyDeviceToHost));
  if (W) HIP_TRY(hipMemcpy(W, t->dev.W, nn * 4, hipMemcpyDeviceToHost));
  if (Wn) HIP_TRY(hipMemcpy(Wn, t->dev.Wn, nn * KMAX * 4, hipMemcpyDeviceToHost));
  if (own) HIP_TRY(hipMemcpy(own, t->dev.own, nn * 4, hipMemcpyDeviceToHost));
  if (leaf_groups) HIP_TRY(hipMemcpy(leaf_groups, t->dev.leaf_groups, nn * 8, hipMemcpyDeviceToHost));
  if (ng && grp_key) HIP_TRY(hipMemcpy(grp_key, t->dev.grp_key, ng * 4, hipMemcpyDeviceToHost));
  if (ng && grp_w) HIP_TRY(hipMemcpy(grp_w, t->dev.grp_w, ng * 4, hipMemcpyDeviceToHost));
  if (ng && grp_lobes) HIP_TRY(hipMemcpy(grp_lobes, t->dev.grp_lobes, ng * 8, hipMemcpyDeviceToHost));
  if (nl && lobe) HIP_TRY(hipMemcpy(lobe, t->dev.lobe, nl * 16, hipMemcpyDeviceToHost));
  if (nl && lobe_cdf) HIP_TRY(hipMemcpy(lobe_cdf, t->dev.lobe_cdf, nl * 4, hipMemcpyDeviceToHost));
  return MPG_OK;
}

extern "C" mpg_status sample_seeds_stree(const mpg_scene* s, const mpg_stree* t, const mpg_walk_params* p,
                                         const mpg_endpoints* ep, uint64_t philox_seed, uint32_t trial,
                                         uint8_t* d_len_out, uint8_t* d_type_out, float* d_pn, mpg_chains* out,
                                         int8_t* d_status, mpg_workspace* ws, void* stream) {
  if (!s || !t) return fail(MPG_ERR_INVALID_ARG, "sample_seeds_stree: NULL scene or guide");
  WalkParams P;
  int waves;
  EpView E;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!out || !out->d_prim || !out->d_pos || !d_status || !d_len_out || !d_type_out || !d_pn)
    return fail(MPG_ERR_INVALID_ARG, "sample_seeds_stree: NULL output");
  SeedOut o{d_len_out, d_type_out, d_pn, out->d_prim, out->d_pos, d_status};
  const int threads = 64 * waves;
  const size_t lds = (size_t)waves * P.depth * 64 * 4;
  hipStream_t st0 = (hipStream_t)stream;
  if (p->form == MPG_FORM_PERSISTENT && p->bucketing) {
    if (!ws || ws->cap < E.N) return fail(MPG_ERR_INVALID_ARG, "sample_seeds_stree: workspace too small");
    int8_t* cls = (int8_t*)ws->aux;
    hipLaunchKernelGGL(k_stree_draw, dim3((E.N + 255) / 256), dim3(256), 0, st0, t->dev, E, philox_seed,
                       (uint64_t)trial, o, cls);
    HIP_TRY(hipGetLastError());
    if ((st = bucket_classes(E.N, cls, ws, st0)) != MPG_OK) return st;
    hipStream_t wk[MPG_WORKERS];
    if ((st = workers_fork(st0, wk)) != MPG_OK) return st;
    for (int n = KMAX, q = 0; n >= 1; --n, q = (q + 1) % MPG_WORKERS) {
      stree_seed_kernel_t k = stree_seed_kernel(n);
      const int grid = resident_blocks((const void*)k, threads, lds);
      hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, wk[q], s->dev, t->dev, P, E, philox_seed,
                         (uint64_t)trial, o, ws->counters, (const int*)ws->perm);
      HIP_TRY(hipGetLastError());
    }
    return workers_join(st0);
  }
  hipLaunchKernelGGL(k_stree_seeds, dim3((E.N + threads - 1) / threads), dim3(threads), lds, st0, s->dev, t->dev, P,
                     E, philox_seed, (uint64_t)trial, o);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

extern "C" mpg_status estimate_inv_prob_stree(const mpg_scene* s, const mpg_stree* t, const mpg_walk_params* p,
                                              const mpg_endpoints* ep, const mpg_chains* target,
                                              const int8_t* d_target_status, int32_t max_trials, int32_t repeats,
                                              uint64_t philox_seed, int32_t* d_trials, float* d_inv_prob,
                                              uint8_t* d_truncated, float* d_pn, mpg_workspace* ws,
                                              void* stream) {
  if (!s || !t) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob_stree: NULL scene or guide");
  WalkParams P;
  int waves;
  EpView E;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!target || !target->d_prim || !target->d_pos || !d_target_status || !d_trials || !d_inv_prob || !d_pn)
    return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob_stree: NULL argument");
  if (max_trials < 0 || repeats < 0) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob_stree: negative count");
  StreeInvIO io{target->d_prim, target->d_pos, d_target_status, d_trials, d_inv_prob, d_truncated, d_pn,
                max_trials, repeats, philox_seed, std::min(std::max(p->max_len, 1), KMAX)};
  const int threads = 64 * waves;
  const size_t lds = (size_t)waves * P.depth * 64 * 4;
  hipStream_t st0 = (hipStream_t)stream;
  if (p->form == MPG_FORM_PERSISTENT && p->bucketing) {
    if (!ws || ws->cap < E.N) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob_stree: workspace too small");
    int8_t* cls = (int8_t*)ws->aux;
    hipLaunchKernelGGL(k_stree_classify, dim3((E.N + 255) / 256), dim3(256), 0, st0, E, io, cls);
    HIP_TRY(hipGetLastError());
    if ((st = bucket_classes(E.N, cls, ws, st0)) != MPG_OK) return st;
    hipStream_t wk[MPG_WORKERS];
    if ((st = workers_fork(st0, wk)) != MPG_OK) return st;
    // the lengths the call may hold (1..max_len), longest first
    for (int n = io.max_len, q = 0; n >= 1; --n, q = (q + 1) % MPG_WORKERS) {
      stree_inv_kernel_t k = stree_inv_refill_kernel(n);
      const int grid = resident_blocks((const void*)k, threads, lds);
      hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, wk[q], s->dev, t->dev, P, E, io, ws->counters,
                         (const int*)ws->perm);
      HIP_TRY(hipGetLastError());
    }
    return workers_join(st0);
  }
  hipLaunchKernelGGL(k_stree_inv, dim3((E.N + threads - 1) / threads), dim3(threads), lds, st0, s->dev, t->dev, P,
                     E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

extern "C" mpg_status make_guide_records(const mpg_endpoints* ep, const mpg_chains* chains, const int8_t* d_status,
                                         const float* d_G, const float* d_kappa, const float* d_inv_prob,
                                         float* d_records, void* stream) {
  EpView E;
  mpg_status st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!chains || !chains->d_pos || !d_status || !d_G || !d_kappa || !d_inv_prob || !d_records)
    return fail(MPG_ERR_INVALID_ARG, "make_guide_records: NULL argument");
  hipLaunchKernelGGL(k_stree_records, dim3((E.N + 255) / 256), dim3(256), 0, (hipStream_t)stream, E,
                     (const float*)chains->d_pos, d_status, d_G, d_kappa, d_inv_prob, d_records);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

extern "C" mpg_status mpg_stree_active(const mpg_stree* t, const mpg_endpoints* ep, uint8_t* d_active, void* stream) {
  if (!t || !d_active) return fail(MPG_ERR_INVALID_ARG, "mpg_stree_active: NULL argument");
  EpView E;
  mpg_status st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  hipLaunchKernelGGL(k_stree_active, dim3((E.N + 255) / 256), dim3(256), 0, (hipStream_t)stream, t->dev, E,
                     d_active);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}
