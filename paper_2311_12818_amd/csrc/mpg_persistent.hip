#include "mpg_internal.h"
#include "mpg_walk.h"

// Persistent batched form of manifold_walk_batch.
//
// 1. k_bucket_hist: chains are classified by length n (invalid ones are
//    finished at once); per-block LDS histograms, one atomic per bin per block.
// 2. k_bucket_scan: one wave turns the histogram into bucket offsets, each
//    bucket padded to a multiple of 64 so that a wavefront's batch never
//    straddles two lengths; padding slots get -1; queue heads are zeroed.
// 3. k_bucket_scatter: block-aggregated slot reservation, perm[] = chain ids.
// 4. One persistent kernel per length N (its own register budget), sized to
//    the machine's occupancy; each wavefront pulls 64-slot batches from its
//    bucket's atomic queue until the bucket drains.
// Without bucketing a single persistent kernel pulls batches of 64
// consecutive chains of mixed length.  All launches are graph-capture safe.

enum : int { CTR_HIST = 0, CTR_OFF = 16, CTR_CUR = 32, CTR_HEAD = 48, CTR_HEAD2 = 56 };

__global__ void __launch_bounds__(256) k_bucket_hist(EpView E, WalkIO io, int max_len, int* ctr, int8_t* cls) {
  __shared__ int h[KMAX + 1];
  if (threadIdx.x <= KMAX) h[threadIdx.x] = 0;
  __syncthreads();
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < E.N) {
    int n = E.len[c];
    bool ok = n >= 1 && n <= max_len && finite3(ld_pt(E.xD, E.N, c)) && finite3(ld_pt(E.xL, E.N, c)) &&
              finite3(ld_pt(E.nD, E.N, c));
    int b = ok ? n : 0;
    cls[c] = (int8_t)b;
    if (b == 0) {
      io.status[c] = ST_BAD_INPUT;
      if (io.iters) io.iters[c] = 0;
      if (io.sol) io.sol[c] = 0;
      if (io.G) io.G[c] = 0.f;
      if (io.kappa) io.kappa[c] = 0.f;
      if (io.resid) io.resid[c] = 0.f;
    } else {
      atomicAdd(&h[b], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x >= 1 && threadIdx.x <= KMAX && h[threadIdx.x]) atomicAdd(&ctr[CTR_HIST + threadIdx.x], h[threadIdx.x]);
}

__global__ void k_bucket_zero(int* ctr) {
  if (threadIdx.x < 64) ctr[threadIdx.x] = 0;
}

__global__ void k_bucket_scan(int* ctr, int* perm) {
  // one block of 64 threads
  __shared__ int off[KMAX + 2];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 1; b <= KMAX; ++b) {
      off[b] = acc;
      ctr[CTR_OFF + b] = acc;
      acc += (ctr[CTR_HIST + b] + 63) & ~63;
    }
    off[KMAX + 1] = acc;
    ctr[CTR_OFF + KMAX + 1] = acc;
  }
  __syncthreads();
  if (threadIdx.x >= 1 && threadIdx.x <= KMAX) {
    ctr[CTR_CUR + threadIdx.x] = 0;
    ctr[CTR_HEAD + threadIdx.x - 1] = 0;
    ctr[CTR_HEAD2 + threadIdx.x - 1] = 0;
  }
  // padding slots of every bucket
  for (int b = 1; b <= KMAX; ++b) {
    int start = off[b] + ctr[CTR_HIST + b], end = off[b + 1];
    for (int i = start + (int)threadIdx.x; i < end; i += blockDim.x) perm[i] = -1;
  }
}

__global__ void __launch_bounds__(256) k_bucket_scatter(int N, const int8_t* cls, int* ctr, int* perm) {
  __shared__ int cnt[KMAX + 1], base[KMAX + 1];
  if (threadIdx.x <= KMAX) cnt[threadIdx.x] = 0;
  __syncthreads();
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  int b = c < N ? cls[c] : 0;
  int local = b > 0 ? atomicAdd(&cnt[b], 1) : 0;
  __syncthreads();
  if (threadIdx.x >= 1 && threadIdx.x <= KMAX && cnt[threadIdx.x])
    base[threadIdx.x] = atomicAdd(&ctr[CTR_CUR + threadIdx.x], cnt[threadIdx.x]);
  __syncthreads();
  if (b > 0) perm[ctr[CTR_OFF + b] + base[b] + local] = c;
}

// Pull the next 64-slot batch of a queue; wave-uniform result.
__device__ __forceinline__ int next_batch(int* head) {
  int base = 0;
  if ((threadIdx.x & 63) == 0) base = atomicAdd(head, 64);
  return __shfl(base, 0, 64);
}

template <int N>
__global__ void __launch_bounds__(256) k_walk_persist(DevScene S, WalkParams P, EpView E, WalkIO io, int* ctr,
                                                      const int* perm) {
  Stack stk = lane_stack(P.depth);
  const int start = ctr[CTR_OFF + N];
  const int end = ctr[CTR_OFF + N + 1];
  const int lane = threadIdx.x & 63;
  for (;;) {
    int base = next_batch(&ctr[CTR_HEAD + N - 1]);
    if (start + base >= end) break;
    int c = perm[start + base + lane];
    if (c >= 0) walk_one<N>(S, P, E, io, c, stk);
  }
}

// Lane-refill walk of one length bucket.  Each lane owns one chain at a time
// and advances it by one walk_step per turn of the loop (the routine the
// plain form's walk_core loops over, so results are identical); a lane whose chain has
// finished takes the next chain of the bucket in the same turn, so lanes do
// not idle while the slowest chain of a 64-chain batch finishes.  Idle lanes
// of a wavefront share one queue atomic per turn and take consecutive slots
// by their rank in the ballot.  Every lane's chain ends within max_iter
// trials and the queue is finite, so every wavefront leaves the loop.
template <int N>
__global__ void __launch_bounds__(256) k_walk_refill(DevScene S, WalkParams P, EpView E, WalkIO io, int* ctr,
                                                     const int* perm) {
  Stack stk = lane_stack(P.depth);
  const int start = ctr[CTR_OFF + N];
  const int count = ctr[CTR_HIST + N];
  int* head = &ctr[CTR_HEAD + N - 1];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  int c = -1;
  bool drained = false;  // wave-uniform: the queue has no slot left for this wavefront
  WalkState<N> w;
  f3 xD = {0.f, 0.f, 0.f}, xL = {0.f, 0.f, 0.f};
  int type = 0;
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
          type = E.type[c];
          xD = ld_pt(E.xD, E.N, c);
          xL = ld_pt(E.xL, E.N, c);
          if (load_seed<N>(S, E, io, c, type, w.prim, w.x)) {
            walk_begin<N>(S, w);
          } else {
            store_walk<N>(E, io, c, ST_SEED_INVALID, 0, false, w.prim, w.x);
            c = -1;
          }
        }
      }
      if (base + nidle >= count) drained = true;
    }
    if (__ballot(c >= 0) == 0) {
      if (drained) break;
      continue;
    }
    if (c >= 0) {
      const int st = walk_step<N>(S, P, xD, xL, type, w, stk);
      if (st >= 0) {
        store_walk<N>(E, io, c, st, w.it, true, w.prim, w.x);
        c = -1;
      }
    }
  }
}

// Finish pass of one length bucket (same queue scheme, second head).
template <int N>
__global__ void __launch_bounds__(256) k_finish_persist(DevScene S, WalkParams P, EpView E, WalkIO io, int* ctr,
                                                        const int* perm) {
  Stack stk = lane_stack(P.depth);
  const int start = ctr[CTR_OFF + N];
  const int end = ctr[CTR_OFF + N + 1];
  const int lane = threadIdx.x & 63;
  for (;;) {
    int base = next_batch(&ctr[CTR_HEAD2 + N - 1]);
    if (start + base >= end) break;
    int c = perm[start + base + lane];
    if (c >= 0 && io.status[c] == ST_PENDING) finish_one<N>(S, P, E, io, c, stk);
  }
}

template <int NMAX>
__global__ void __launch_bounds__(256) k_walk_persist_mixed(DevScene S, WalkParams P, EpView E, WalkIO io,
                                                            int* ctr) {
  Stack stk = lane_stack(P.depth);
  const int lane = threadIdx.x & 63;
  for (;;) {
    int base = next_batch(&ctr[CTR_HEAD]);
    if (base >= E.N) break;
    int c = base + lane;
    if (c < E.N) walk_dispatch<NMAX>(S, P, E, io, c, stk);
  }
}

typedef void (*persist_kernel_t)(DevScene, WalkParams, EpView, WalkIO, int*, const int*);
typedef void (*mixed_kernel_t)(DevScene, WalkParams, EpView, WalkIO, int*);

static persist_kernel_t finish_persist_kernel(int n) {
  switch (n) {
    case 1: return k_finish_persist<1>;
    case 2: return k_finish_persist<2>;
    case 3: return k_finish_persist<3>;
    case 4: return k_finish_persist<4>;
    case 5: return k_finish_persist<5>;
    case 6: return k_finish_persist<6>;
    case 7: return k_finish_persist<7>;
    default: return k_finish_persist<8>;
  }
}
static persist_kernel_t persist_kernel(int n) {
  switch (n) {
    case 1: return k_walk_persist<1>;
    case 2: return k_walk_persist<2>;
    case 3: return k_walk_persist<3>;
    case 4: return k_walk_persist<4>;
    case 5: return k_walk_persist<5>;
    case 6: return k_walk_persist<6>;
    case 7: return k_walk_persist<7>;
    default: return k_walk_persist<8>;
  }
}
static persist_kernel_t refill_kernel(int n) {
  switch (n) {
    case 1: return k_walk_refill<1>;
    case 2: return k_walk_refill<2>;
    case 3: return k_walk_refill<3>;
    case 4: return k_walk_refill<4>;
    case 5: return k_walk_refill<5>;
    case 6: return k_walk_refill<6>;
    case 7: return k_walk_refill<7>;
    default: return k_walk_refill<8>;
  }
}
static mixed_kernel_t mixed_kernel(int nmax) {
  switch (nmax) {
    case 1: return k_walk_persist_mixed<1>;
    case 2: return k_walk_persist_mixed<2>;
    case 3: return k_walk_persist_mixed<3>;
    case 4: return k_walk_persist_mixed<4>;
    case 5: return k_walk_persist_mixed<5>;
    case 6: return k_walk_persist_mixed<6>;
    case 7: return k_walk_persist_mixed<7>;
    default: return k_walk_persist_mixed<8>;
  }
}

// Resident workgroups of a kernel across the device (persistent grid size).
static int resident_blocks(const void* fn, int threads, size_t lds) {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds) != hipSuccess || per < 1) per = 1;
  return std::max(1, cus) * per;
}

// Internal streams of the current device for the per-length kernels (four:
// the runtime exposes four hardware queues per process by default).  All at
// the default priority; fork / join through events, which graph capture
// records as dependencies.
struct SideStreams {
  int device = -1;
  hipStream_t s[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[4] = {nullptr, nullptr, nullptr, nullptr};
};
static SideStreams g_side[64];
static std::mutex g_side_mu;

static mpg_status side_streams(SideStreams** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MPG_ERR_UNSUPPORTED, "device index >= 64");
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStreams& ss = g_side[dev];
  if (ss.device != dev) {
    for (int k = 0; k < 4; ++k) {
      HIP_TRY(hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
    ss.device = dev;
  }
  *out = &ss;
  return MPG_OK;
}

mpg_status walk_persistent(const mpg_scene* s, const WalkParams& P, int waves, int bucketing, int refill,
                           int max_len, const EpView& E, const WalkIO& io, mpg_workspace* ws, hipStream_t stream) {
  const int threads = 64 * waves;
  const size_t lds = (size_t)waves * P.depth * 64 * 4;
  const int blocks = (E.N + 255) / 256;
  int* ctr = ws->counters;
  hipLaunchKernelGGL(k_bucket_zero, dim3(1), dim3(64), 0, stream, ctr);
  HIP_TRY(hipGetLastError());
  if (!bucketing) {
    mixed_kernel_t k = mixed_kernel(max_len);
    int grid = resident_blocks((const void*)k, threads, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, stream, s->dev, P, E, io, ctr);
    HIP_TRY(hipGetLastError());
    return launch_finish_plain(s, P, E, io, max_len, threads, lds, stream);
  }
  int8_t* cls = (int8_t*)ws->aux;
  hipLaunchKernelGGL(k_bucket_hist, dim3(blocks), dim3(256), 0, stream, E, io, max_len, ctr, cls);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, stream, ctr, ws->perm);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scatter, dim3(blocks), dim3(256), 0, stream, E.N, (const int8_t*)cls, ctr, ws->perm);
  HIP_TRY(hipGetLastError());
  SideStreams* ss;
  mpg_status st = side_streams(&ss);
  if (st != MPG_OK) return st;
  HIP_TRY(hipEventRecord(ss->fork, stream));
  for (int k = 0; k < 4; ++k) HIP_TRY(hipStreamWaitEvent(ss->s[k], ss->fork, 0));
  // lengths round-robin over the side streams, longest first; each length's
  // finish pass follows its walk on the same stream
  for (int n = max_len, q = 0; n >= 1; --n, q = (q + 1) & 3) {
    persist_kernel_t k = refill ? refill_kernel(n) : persist_kernel(n);
    int grid = resident_blocks((const void*)k, threads, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, ss->s[q], s->dev, P, E, io, ctr, (const int*)ws->perm);
    HIP_TRY(hipGetLastError());
    persist_kernel_t f = finish_persist_kernel(n);
    int fgrid = resident_blocks((const void*)f, threads, lds);
    hipLaunchKernelGGL(f, dim3(fgrid), dim3(threads), lds, ss->s[q], s->dev, P, E, io, ctr, (const int*)ws->perm);
    HIP_TRY(hipGetLastError());
  }
  for (int k = 0; k < 4; ++k) {
    HIP_TRY(hipEventRecord(ss->join[k], ss->s[k]));
    HIP_TRY(hipStreamWaitEvent(stream, ss->join[k], 0));
  }
  return MPG_OK;
}
