#include "mpg_internal.h"
#include "mpg_walk.h"

// ---------------------------------------------------------------------------
// Bernoulli trials (Sec. 5.8)
// ---------------------------------------------------------------------------
struct InvIO {
  const int32_t* tprim;
  const float* tpos;
  const int8_t* tstatus;
  int32_t* trials;
  float* inv_prob;
  uint8_t* truncated;
  int max_trials, repeats;
  int max_len;  // targets longer than this are not estimated (zero outputs)
  uint64_t seed;
  float alpha;
};

template <int N, class STK>
__device__ __forceinline__ void inv_one(const DevScene& S, const DevGuide* G, const WalkParams& P, const EpView& E,
                        const InvIO& io, int c, STK& stk) {
  const size_t NN = E.N;
  f3 tx[N];
  int tobj[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    tx[i] = {io.tpos[(0 * KMAX + i) * NN + c], io.tpos[(1 * KMAX + i) * NN + c], io.tpos[(2 * KMAX + i) * NN + c]};
    tobj[i] = prim_obj(S, io.tprim[i * NN + c]);
  }
  f3 xD = ld_pt(E.xD, E.N, c), nD = ld_pt(E.nD, E.N, c), xL = ld_pt(E.xL, E.N, c);
  int type = E.type[c], obj1 = E.obj1[c];
  int total = 0;
  bool trunc = false;
  for (int r = 0; r < io.repeats; ++r) {
    int K = io.max_trials;
    bool found = false;
    for (int k = 1; k <= io.max_trials && !found; ++k) {
      uint64_t trial = 1 + (uint64_t)r * io.max_trials + (uint64_t)(k - 1);
      int prim[N];
      f3 x[N];
      if (sample_seed<N>(S, G, P, type, obj1, xD, nD, io.seed, (uint64_t)c, trial, io.alpha, prim, x, stk,
                         chain_offs(E, c)) != 0)
        continue;
      int it;
      int ws = walk_core<N>(S, P, xD, xL, type, prim, x, it, stk, chain_offs(E, c));
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
  io.trials[c] = total;
  io.inv_prob[c] = (float)total / (float)io.repeats;
  if (io.truncated) io.truncated[c] = trunc ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_inv_prob(DevScene S, DevGuide G, WalkParams P, EpView E,
                                                  InvIO io) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  int n = E.len[c];
  if (io.tstatus[c] != ST_CONVERGED || n < 1 || n > io.max_len || io.repeats < 1 || io.max_trials < 1) {
    io.trials[c] = 0;
    io.inv_prob[c] = 0.f;
    if (io.truncated) io.truncated[c] = 0;
    return;
  }
  // always the argument's address (no guide: a zeroed DevGuide); a pointer
  // that may be null would make the compiler copy G to private memory
  const DevGuide* g = &G;
  switch (n) {
    case 1: inv_one<1>(S, g, P, E, io, c, stk); break;
    case 2: inv_one<2>(S, g, P, E, io, c, stk); break;
    case 3: inv_one<3>(S, g, P, E, io, c, stk); break;
    case 4: inv_one<4>(S, g, P, E, io, c, stk); break;
    case 5: inv_one<5>(S, g, P, E, io, c, stk); break;
    case 6: inv_one<6>(S, g, P, E, io, c, stk); break;
    case 7: inv_one<7>(S, g, P, E, io, c, stk); break;
    default: inv_one<8>(S, g, P, E, io, c, stk); break;
  }
}

// ---------------------------------------------------------------------------
// Persistent form of the trials: chains with a converged target are bucketed
// by length; each lane owns one target chain and advances its current trial
// walk by one walk_step per turn; a lane whose walk has ended takes the next
// chain at once if its target is done, and starts its next trial together
// with the other waiting lanes of its wavefront, so lanes do not idle while
// the chain with the most trials of a batch finishes.  Same seeds, walks,
// matches and counts as inv_one.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_inv_classify(EpView E, InvIO io, int8_t* cls) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  int n = E.len[c];
  bool target = io.tstatus[c] == ST_CONVERGED && n >= 1 && n <= io.max_len && io.repeats >= 1 && io.max_trials >= 1;
  cls[c] = (int8_t)(target ? n : 0);
  if (!target) {
    io.trials[c] = 0;
    io.inv_prob[c] = 0.f;
    if (io.truncated) io.truncated[c] = 0;
  }
}

template <int N>
__global__ void __launch_bounds__(256) k_inv_refill(DevScene S, DevGuide G, WalkParams P, EpView E,
                                                    InvIO io, int* ctr, const int* perm) {
  Stack stk = lane_stack(P.depth);
  // always the argument's address (no guide: a zeroed DevGuide); a pointer
  // that may be null would make the compiler copy G to private memory
  const DevGuide* g = &G;
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
  int type = 0, obj1 = 0;
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
          type = E.type[c];
          obj1 = E.obj1[c];
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
    // A new trial starts with seed sampling (a guided lift ray and the
    // deduction rays), traversals that the lanes in the middle of a walk sit
    // out.  Lanes waiting for a new trial therefore start together, once
    // they are at least half of the busy lanes (or no lane is walking); each
    // trial's seed depends on (chain, trial) only, so the results do not
    // change.  On the guided water batch: 114 against 123 ms on average over
    // five runs each (run-to-run spread about 5%).
    const unsigned long long waiting = __ballot(c >= 0 && !walking);
    const unsigned long long busy = __ballot(c >= 0);
    const bool start_trials = 2 * __popcll(waiting) >= __popcll(busy);
    if (c >= 0 && !walking && start_trials) {
      if (k == io.max_trials) {  // no match within the budget: K = max_trials, truncated
        trunc = true;
        total += io.max_trials;
        ++r;
        k = 0;
        if (r == io.repeats) {
          io.trials[c] = total;
          io.inv_prob[c] = (float)total / (float)io.repeats;
          if (io.truncated) io.truncated[c] = 1;
          c = -1;
        }
      }
      if (c >= 0) {
        ++k;
        const uint64_t trial = 1 + (uint64_t)r * io.max_trials + (uint64_t)(k - 1);
        if (sample_seed<N>(S, g, P, type, obj1, xD, nD, io.seed, (uint64_t)c, trial, io.alpha, w.prim, w.x, stk,
                           chain_offs(E, c)) == 0) {
          walk_begin<N>(S, w);
          walking = true;
        }
      }
    }
    if (c >= 0 && walking) {
      const int st = walk_step<N>(S, P, xD, xL, type, w, stk, chain_offs(E, c));
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
          if (r == io.repeats) {
            io.trials[c] = total;
            io.inv_prob[c] = (float)total / (float)io.repeats;
            if (io.truncated) io.truncated[c] = trunc ? 1 : 0;
            c = -1;
          }
        }
      }
    }
  }
}

typedef void (*inv_kernel_t)(DevScene, DevGuide, WalkParams, EpView, InvIO, int*, const int*);
static inv_kernel_t inv_refill_kernel(int n) {
  switch (n) {
    case 1: return k_inv_refill<1>;
    case 2: return k_inv_refill<2>;
    case 3: return k_inv_refill<3>;
    case 4: return k_inv_refill<4>;
    case 5: return k_inv_refill<5>;
    case 6: return k_inv_refill<6>;
    case 7: return k_inv_refill<7>;
    default: return k_inv_refill<8>;
  }
}

static mpg_status inv_persistent(const mpg_scene* s, const DevGuide& G, const WalkParams& P,
                                 int waves, const EpView& E, const InvIO& io, mpg_workspace* ws, hipStream_t stream) {
  const int threads = 64 * waves;
  const size_t lds = (size_t)waves * P.depth * 64 * 4;
  int8_t* cls = (int8_t*)ws->aux;
  hipLaunchKernelGGL(k_inv_classify, dim3((E.N + 255) / 256), dim3(256), 0, stream, E, io, cls);
  HIP_TRY(hipGetLastError());
  mpg_status st = bucket_classes(E.N, cls, ws, stream);
  if (st != MPG_OK) return st;
  hipStream_t wk[MPG_WORKERS];
  if ((st = workers_fork(stream, wk)) != MPG_OK) return st;
  // only the lengths the call may hold (1..max_len), longest first
  for (int n = io.max_len, q = 0; n >= 1; --n, q = (q + 1) % MPG_WORKERS) {
    inv_kernel_t k = inv_refill_kernel(n);
    int grid = resident_blocks((const void*)k, threads, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, wk[q], s->dev, G, P, E, io, ws->counters,
                       (const int*)ws->perm);
    HIP_TRY(hipGetLastError());
  }
  return workers_join(stream);
}

extern "C" mpg_status estimate_inv_prob(const mpg_scene* s, const mpg_guide* g, const mpg_walk_params* p,
                                        const mpg_endpoints* ep, const mpg_chains* target,
                                        const int8_t* d_target_status, int32_t max_trials, int32_t repeats,
                                        uint64_t philox_seed, float alpha, int32_t* d_trials, float* d_inv_prob,
                                        uint8_t* d_truncated, mpg_workspace* ws, void* stream) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob: NULL scene");
  WalkParams P;
  int waves;
  EpView E;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!target || !target->d_prim || !target->d_pos || !d_target_status || !d_trials || !d_inv_prob)
    return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob: NULL argument");
  if (max_trials < 0 || repeats < 0) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob: negative trial count");
  if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob: alpha outside [0, 1]");
  DevGuide G;
  std::memset(&G, 0, sizeof(G));
  if (g) G = g->dev();
  InvIO io;
  io.tprim = target->d_prim; io.tpos = target->d_pos; io.tstatus = d_target_status;
  io.trials = d_trials; io.inv_prob = d_inv_prob; io.truncated = d_truncated;
  io.max_trials = max_trials; io.repeats = repeats; io.seed = philox_seed; io.alpha = alpha;
  io.max_len = std::min(std::max(p->max_len, 1), KMAX);
  if (p->form == MPG_FORM_PERSISTENT && p->bucketing) {
    if (!ws || ws->cap < E.N) return fail(MPG_ERR_INVALID_ARG, "estimate_inv_prob: workspace too small");
    return inv_persistent(s, G, P, waves, E, io, ws, (hipStream_t)stream);
  }
  int threads = 64 * waves;
  size_t lds = (size_t)waves * P.depth * 64 * 4;
  hipLaunchKernelGGL(k_inv_prob, dim3((E.N + threads - 1) / threads), dim3(threads), lds, (hipStream_t)stream,
                     s->dev, G, P, E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

