#include "mpg_internal.h"
#include "mpg_walk.h"

// Persistent batched form of manifold_walk_batch.
//
// 1. k_bucket_hist: chains are classified by length n (invalid ones are
//    finished at once); per-block LDS histograms, one atomic per bin per block.
// 2. k_bucket_scan: one wave turns the histogram into bucket offsets, each
//    bucket padded to a multiple of 64 so that a wavefront's batch never
//    straddles two lengths; padding slots get -1; queue heads are zeroed.
// 3. k_bucket_scatter: workgroup-aggregated slot reservation over contiguous
//    ranges of chains, perm[] = chain ids
//    (bucketing = 2: ordered by spatial cell inside each bucket, see below).
// 4. One persistent kernel per length N (its own register budget), sized to
//    the machine's occupancy; each wavefront pulls 64-slot batches from its
//    bucket's atomic queue until the bucket drains.
// Without bucketing a single persistent kernel pulls batches of 64
// consecutive chains of mixed length.  All launches are graph-capture safe.


__global__ void __launch_bounds__(256) k_bucket_hist(EpView E, WalkIO io, int max_len, int check_xl, int* ctr,
                                                     int8_t* cls) {
  __shared__ int h[KMAX + 1];
  if (threadIdx.x <= KMAX) h[threadIdx.x] = 0;
  __syncthreads();
  // grid-stride: a capped grid keeps the global atomics on the eight bins
  // to a few per workgroup
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < E.N; c += gridDim.x * blockDim.x) {
    int n = E.len[c];
    bool ok = n >= 1 && n <= max_len && finite3(ld_pt(E.xD, E.N, c)) &&
              (!check_xl || finite3(ld_pt(E.xL, E.N, c))) && finite3(ld_pt(E.nD, E.N, c));
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
  if (threadIdx.x < MPG_WS_COUNTERS) ctr[threadIdx.x] = 0;
}

// Histogram of precomputed classes (1..8; 0 = no slot).
__global__ void __launch_bounds__(256) k_class_hist(int N, const int8_t* cls, int* ctr) {
  __shared__ int h[KMAX + 1];
  if (threadIdx.x <= KMAX) h[threadIdx.x] = 0;
  __syncthreads();
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x)
    if (cls[c] > 0) atomicAdd(&h[(int)cls[c]], 1);
  __syncthreads();
  if (threadIdx.x >= 1 && threadIdx.x <= KMAX && h[threadIdx.x]) atomicAdd(&ctr[CTR_HIST + threadIdx.x], h[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Spatial order inside each length bucket (bucketing = 2): chains are binned
// by the Morton index of x_D on a 32^3 grid over the batch's bounding box, so
// that the chains a wavefront takes together start close to each other and
// trace nearly the same BVH nodes.  Counting sort with atomic cursors (the
// order inside a cell is arbitrary; every chain's result is independent of
// it).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ordered_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ordered_value(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 5 bits -> every third bit
  v &= 31u;
  v = (v | (v << 8)) & 0x0000f00fu;
  v = (v | (v << 4)) & 0x000c30c3u;
  v = (v | (v << 2)) & 0x00249249u;
  return v;
}

__global__ void __launch_bounds__(256) k_cells_zero(int* cells, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) cells[i] = 0;
}

// bounding box of the valid shading points: per-wave reduction, then one
// atomic max per wave and bound (minima as max of the complemented keys)
__global__ void __launch_bounds__(256) k_box_reduce(EpView E, const int8_t* cls, int* ctr) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t hi[3] = {0u, 0u, 0u}, lo[3] = {0u, 0u, 0u};
  if (c < E.N && cls[c] > 0) {
    f3 x = ld_pt(E.xD, E.N, c);
    float v[3] = {x.x, x.y, x.z};
    for (int a = 0; a < 3; ++a) { hi[a] = ordered_key(v[a]); lo[a] = ~ordered_key(v[a]); }
  }
  for (int a = 0; a < 3; ++a) {
    for (int o = 32; o > 0; o >>= 1) {
      hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], o, 64));
      lo[a] = max(lo[a], (uint32_t)__shfl_xor((int)lo[a], o, 64));
    }
  }
  if ((threadIdx.x & 63) == 0) {
    for (int a = 0; a < 3; ++a) {
      if (hi[a]) atomicMax((unsigned int*)&ctr[CTR_BOX + a], hi[a]);
      if (lo[a]) atomicMax((unsigned int*)&ctr[CTR_BOX + 3 + a], lo[a]);
    }
  }
}

__device__ __forceinline__ int cell_bin(const EpView& E, const int* ctr, int c, int len) {
  f3 x = ld_pt(E.xD, E.N, c);
  float v[3] = {x.x, x.y, x.z};
  uint32_t q[3];
  for (int a = 0; a < 3; ++a) {
    float lo = ordered_value(~(uint32_t)ctr[CTR_BOX + 3 + a]), hi = ordered_value((uint32_t)ctr[CTR_BOX + a]);
    float ext = hi - lo;
    float u = ext > 0.0f ? (v[a] - lo) / ext : 0.0f;
    int k = (int)(u * (float)MPG_CELL_RES);
    q[a] = (uint32_t)min(max(k, 0), MPG_CELL_RES - 1);
  }
  int morton = (int)(spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2));
  return (len - 1) * MPG_CELLS + morton;
}

__global__ void __launch_bounds__(256) k_cell_hist(EpView E, const int8_t* cls, const int* ctr, int* hist) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N || cls[c] <= 0) return;
  atomicAdd(&hist[cell_bin(E, ctr, c, cls[c])], 1);
}

// exclusive scan of every length's cell counts, offset by the (64-padded)
// start of the length's bucket: cursors for the scatter.  One block of 1024.
__global__ void __launch_bounds__(1024) k_cell_scan(const int* ctr, const int* hist, int* cursor) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  constexpr int PER = MPG_CELLS / 1024;
  for (int len = 1; len <= KMAX; ++len) {
    const int* h = hist + (len - 1) * MPG_CELLS;
    int local = 0;
    for (int i = 0; i < PER; ++i) local += h[t * PER + i];
    part[t] = local;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int v = t >= o ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = ctr[CTR_OFF + len] + part[t] - local;
    for (int i = 0; i < PER; ++i) {
      cursor[(len - 1) * MPG_CELLS + t * PER + i] = run;
      run += h[t * PER + i];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_cell_scatter(EpView E, const int8_t* cls, const int* ctr, int* cursor,
                                                      int* perm) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N || cls[c] <= 0) return;
  int slot = atomicAdd(&cursor[cell_bin(E, ctr, c, cls[c])], 1);
  perm[slot] = c;
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

// Each workgroup takes a contiguous range of per_block chains: it counts
// their classes, reserves its slots in every bucket with one global atomic
// per bucket, then writes the chains into them (LDS cursors).
__global__ void __launch_bounds__(256) k_bucket_scatter(int N, const int8_t* cls, int* ctr, int* perm, int per_block) {
  __shared__ int cnt[KMAX + 1], base[KMAX + 1];
  if (threadIdx.x <= KMAX) cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long c0 = (long long)blockIdx.x * per_block;
  const int c1 = (int)(c0 + per_block < N ? c0 + per_block : N);
  for (int c = (int)c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const int b = cls[c];
    if (b > 0) atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  if (threadIdx.x >= 1 && threadIdx.x <= KMAX) {
    const int k = threadIdx.x;
    base[k] = cnt[k] ? ctr[CTR_OFF + k] + atomicAdd(&ctr[CTR_CUR + k], cnt[k]) : 0;
    cnt[k] = 0;  // now the cursor of the bucket
  }
  __syncthreads();
  for (int c = (int)c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const int b = cls[c];
    if (b > 0) perm[base[b] + atomicAdd(&cnt[b], 1)] = c;
  }
}

// launch shape of the bucketing passes: at most 1024 workgroups of 256
static int bucket_blocks(int N) { return std::max(1, std::min((N + 255) / 256, 1024)); }
static int bucket_per_block(int N) {
  const int g = bucket_blocks(N);
  return ((N + g - 1) / g + 255) / 256 * 256;
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
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(refill_waves(N))))
k_walk_refill(DevScene S, WalkParams P, EpView E, WalkIO io, int* ctr, const int* perm, int parts) {
  Stack stk = lane_stack(P.depth);
  const int start = ctr[CTR_OFF + N];
  const int count = ctr[CTR_HIST + N];
  int* heads = &ctr[CTR_PHEAD + (N - 1) * MPG_MAX_PARTS];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  // the bucket is split into `parts` consecutive slot ranges (spatial regions
  // when the bucket is in Morton order); a workgroup starts on the range of
  // its XCD (workgroups are dealt to the XCDs round robin) and moves on when
  // that range is empty, so each XCD's L2 holds the part of the scene its
  // region needs
  int part = blockIdx.x % parts, tried = 0;
  int c = -1;
  bool drained = false;  // wave-uniform: the queue has no slot left for this wavefront
  WalkState<N> w;
  f3 xD = {0.f, 0.f, 0.f}, xL = {0.f, 0.f, 0.f};
  int type = 0;
  for (;;) {
    const unsigned long long idle = __ballot(c < 0);
    if (idle && !drained) {
      const int nidle = __popcll(idle);
      const int lo = (int)((long long)count * part / parts), hi = (int)((long long)count * (part + 1) / parts);
      int base = 0;
      if (lane == 0) base = atomicAdd(&heads[part], nidle);
      base = lo + __shfl(base, 0, 64);
      if (c < 0) {
        const int slot = base + __popcll(idle & below);
        if (slot < hi) {
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
      if (base + nidle >= hi) {  // this range is used up: the next one
        part = part + 1 == parts ? 0 : part + 1;
        if (++tried == parts) drained = true;
      }
    }
    if (__ballot(c >= 0) == 0) {
      if (drained) break;
      continue;
    }
    if (c >= 0) {
      const int st = walk_step<N>(S, P, xD, xL, type, w, stk, chain_offs(E, c));
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

// Seed sampling of one length bucket (same queue scheme, third head): every
// chain of a bucket traces the same number of deduction rays.
template <int N>
__global__ void __launch_bounds__(256) k_seeds_persist(DevScene S, DevGuide G, WalkParams P,
                                                       EpView E, uint64_t seed, uint64_t trial, float alpha,
                                                       int32_t* prim_out, float* pos_out, int8_t* st, int* ctr,
                                                       const int* perm) {
  Stack stk = lane_stack(P.depth);
  const int start = ctr[CTR_OFF + N];
  const int end = ctr[CTR_OFF + N + 1];
  const int lane = threadIdx.x & 63;
  // always the argument's address (no guide: a zeroed DevGuide); a pointer
  // that may be null would make the compiler copy G to private memory
  const DevGuide* g = &G;
  for (;;) {
    int base = next_batch(&ctr[CTR_HEAD3 + N - 1]);
    if (start + base >= end) break;
    int c = perm[start + base + lane];
    if (c >= 0) seed_one<N>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk);
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
typedef void (*refill_kernel_t)(DevScene, WalkParams, EpView, WalkIO, int*, const int*, int);
static refill_kernel_t refill_kernel(int n) {
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
typedef void (*seeds_kernel_t)(DevScene, DevGuide, WalkParams, EpView, uint64_t, uint64_t, float, int32_t*,
                               float*, int8_t*, int*, const int*);
static seeds_kernel_t seeds_kernel(int n) {
  switch (n) {
    case 1: return k_seeds_persist<1>;
    case 2: return k_seeds_persist<2>;
    case 3: return k_seeds_persist<3>;
    case 4: return k_seeds_persist<4>;
    case 5: return k_seeds_persist<5>;
    case 6: return k_seeds_persist<6>;
    case 7: return k_seeds_persist<7>;
    default: return k_seeds_persist<8>;
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
int resident_blocks(const void* fn, int threads, size_t lds) {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds) != hipSuccess || per < 1) per = 1;
  return std::max(1, cus) * per;
}

// Workers for the per-length kernels: the caller's stream and three internal
// streams of the current device.  The runtime gives a process four hardware
// queues by default; the caller's stream holds one, so a fourth internal
// stream would share a queue (and its in-order execution) with another.  All
// at the default priority; fork / join through events, which graph capture
// records as dependencies.
struct SideStreams {
  int device = -1;
  hipStream_t s[MPG_WORKERS - 1] = {};
  hipEvent_t fork = nullptr, join[MPG_WORKERS - 1] = {};
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
    for (int k = 0; k < MPG_WORKERS - 1; ++k) {
      HIP_TRY(hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
    ss.device = dev;
  }
  *out = &ss;
  return MPG_OK;
}

mpg_status workers_fork(hipStream_t stream, hipStream_t wk[MPG_WORKERS]) {
  SideStreams* ss;
  mpg_status st = side_streams(&ss);
  if (st != MPG_OK) return st;
  HIP_TRY(hipEventRecord(ss->fork, stream));
  wk[0] = stream;
  for (int k = 0; k < MPG_WORKERS - 1; ++k) {
    HIP_TRY(hipStreamWaitEvent(ss->s[k], ss->fork, 0));
    wk[k + 1] = ss->s[k];
  }
  return MPG_OK;
}

mpg_status workers_join(hipStream_t stream) {
  SideStreams* ss;
  mpg_status st = side_streams(&ss);
  if (st != MPG_OK) return st;
  for (int k = 0; k < MPG_WORKERS - 1; ++k) {
    HIP_TRY(hipEventRecord(ss->join[k], ss->s[k]));
    HIP_TRY(hipStreamWaitEvent(stream, ss->join[k], 0));
  }
  return MPG_OK;
}

// Length buckets (and, for bucketing = 2, spatial order inside them) of a
// batch in ws->perm; chains that fail the input checks get MPG_BAD_INPUT in
// io.status and no slot.
static mpg_status bucket_chains(int bucketing, int max_len, int check_xl, const EpView& E, const WalkIO& io,
                                mpg_workspace* ws, hipStream_t stream) {
  const int blocks = (E.N + 255) / 256;
  int* ctr = ws->counters;
  int8_t* cls = (int8_t*)ws->aux;
  hipLaunchKernelGGL(k_bucket_hist, dim3(bucket_blocks(E.N)), dim3(256), 0, stream, E, io, max_len, check_xl, ctr,
                     cls);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, stream, ctr, ws->perm);
  HIP_TRY(hipGetLastError());
  if (bucketing >= 2) {
    int* hist = ws->cells;
    int* cursor = ws->cells + KMAX * MPG_CELLS;
    hipLaunchKernelGGL(k_cells_zero, dim3(256), dim3(256), 0, stream, hist, KMAX * MPG_CELLS);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_box_reduce, dim3(blocks), dim3(256), 0, stream, E, (const int8_t*)cls, ctr);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_cell_hist, dim3(blocks), dim3(256), 0, stream, E, (const int8_t*)cls, (const int*)ctr, hist);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, stream, (const int*)ctr, (const int*)hist, cursor);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_cell_scatter, dim3(blocks), dim3(256), 0, stream, E, (const int8_t*)cls, (const int*)ctr,
                       cursor, ws->perm);
  } else {
    hipLaunchKernelGGL(k_bucket_scatter, dim3(bucket_blocks(E.N)), dim3(256), 0, stream, E.N, (const int8_t*)cls, ctr,
                       ws->perm, bucket_per_block(E.N));
  }
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

// The lengths 1..max_len in launch order: the nibbles of length_order (the
// first in the lowest), else longest first.
static int launch_order(uint32_t length_order, int max_len, int order[KMAX]) {
  int n_order = 0;
  for (int k = 0; k < KMAX; ++k) {
    int n = length_order ? (int)((length_order >> (4 * k)) & 15u) : KMAX - k;
    if (n <= max_len) order[n_order++] = n;
  }
  return n_order;
}

mpg_status seeds_persistent(const mpg_scene* s, const DevGuide& G, const WalkParams& P, int waves,
                            int bucketing, uint32_t length_order, const EpView& E, uint64_t seed, uint32_t trial,
                            float alpha, int32_t* prim_out, float* pos_out, int8_t* status, mpg_workspace* ws,
                            hipStream_t stream) {
  const int threads = 64 * waves;
  const size_t lds = (size_t)waves * P.depth * 64 * 4;
  int* ctr = ws->counters;
  hipLaunchKernelGGL(k_bucket_zero, dim3(1), dim3(MPG_WS_COUNTERS), 0, stream, ctr);
  HIP_TRY(hipGetLastError());
  WalkIO io;
  std::memset(&io, 0, sizeof(io));
  io.status = status;
  mpg_status bst = bucket_chains(bucketing, KMAX, 0, E, io, ws, stream);
  if (bst != MPG_OK) return bst;
  hipStream_t wk[MPG_WORKERS];
  mpg_status st = workers_fork(stream, wk);
  if (st != MPG_OK) return st;
  // lengths dealt round robin to the workers in launch order
  int order[KMAX];
  const int n_order = launch_order(length_order, KMAX, order);
  for (int j = 0; j < n_order; ++j) {
    const int n = order[j], q = j % MPG_WORKERS;
    seeds_kernel_t k = seeds_kernel(n);
    int grid = resident_blocks((const void*)k, threads, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, wk[q], s->dev, G, P, E, seed,
                       (uint64_t)trial, alpha, prim_out, pos_out, status, ctr, (const int*)ws->perm);
    HIP_TRY(hipGetLastError());
  }
  return workers_join(stream);
}

mpg_status bucket_classes(int N, const int8_t* cls, mpg_workspace* ws, hipStream_t stream) {
  int* ctr = ws->counters;
  hipLaunchKernelGGL(k_bucket_zero, dim3(1), dim3(MPG_WS_COUNTERS), 0, stream, ctr);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_class_hist, dim3(bucket_blocks(N)), dim3(256), 0, stream, N, cls, ctr);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, stream, ctr, ws->perm);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scatter, dim3(bucket_blocks(N)), dim3(256), 0, stream, N, cls, ctr, ws->perm,
                     bucket_per_block(N));
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

mpg_status walk_persistent(const mpg_scene* s, const WalkParams& P, int waves, int bucketing, int refill,
                           int max_len, uint32_t length_order, const EpView& E, const WalkIO& io, mpg_workspace* ws,
                           hipStream_t stream) {
  const int threads = 64 * waves;
  const size_t lds = (size_t)waves * P.depth * 64 * 4;
  int* ctr = ws->counters;
  hipLaunchKernelGGL(k_bucket_zero, dim3(1), dim3(MPG_WS_COUNTERS), 0, stream, ctr);
  HIP_TRY(hipGetLastError());
  if (!bucketing) {
    mixed_kernel_t k = mixed_kernel(max_len);
    int grid = resident_blocks((const void*)k, threads, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, stream, s->dev, P, E, io, ctr);
    HIP_TRY(hipGetLastError());
    return launch_finish_plain(s, P, E, io, max_len, threads, lds, stream);
  }
  mpg_status bst = bucket_chains(bucketing, max_len, 1, E, io, ws, stream);
  if (bst != MPG_OK) return bst;
  hipStream_t wk[MPG_WORKERS];
  if (ws->single_stream) {
    for (int q = 0; q < MPG_WORKERS; ++q) wk[q] = stream;
  } else {
    mpg_status st = workers_fork(stream, wk);
    if (st != MPG_OK) return st;
  }
  // lengths dealt round robin to the workers in launch order (length_order,
  // else longest first; lengths above max_len left out); every finish pass
  // is queued after all walks, on its walk's worker.  A finish pass launched
  // while other lengths' persistent walks hold the compute units gets few
  // slots and holds up the walks queued behind it on its worker.
  int order[KMAX];
  const int n_order = launch_order(length_order, max_len, order);
  for (int j = 0; j < n_order; ++j) {
    const int n = order[j], q = j % MPG_WORKERS;
    if (refill) {
      refill_kernel_t k = refill_kernel(n);
      int grid = resident_blocks((const void*)k, threads, lds);
      hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, wk[q], s->dev, P, E, io, ctr, (const int*)ws->perm,
                         bucketing == 3 ? MPG_MAX_PARTS : 1);
    } else {
      persist_kernel_t k = persist_kernel(n);
      int grid = resident_blocks((const void*)k, threads, lds);
      hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, wk[q], s->dev, P, E, io, ctr, (const int*)ws->perm);
    }
    HIP_TRY(hipGetLastError());
  }
  for (int j = 0; j < n_order; ++j) {
    const int n = order[j], q = j % MPG_WORKERS;
    persist_kernel_t f = finish_persist_kernel(n);
    int fgrid = resident_blocks((const void*)f, threads, lds);
    hipLaunchKernelGGL(f, dim3(fgrid), dim3(threads), lds, wk[q], s->dev, P, E, io, ctr, (const int*)ws->perm);
    HIP_TRY(hipGetLastError());
  }
  return ws->single_stream ? MPG_OK : workers_join(stream);
}
