// Internal interface shared by the library's translation units: handle
// layouts, host helpers and the per-chain views the kernels take.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpg.h"
#include "mpg_device.h"
#include "mpg_scene.h"

using namespace mpg;

// errors: a thread-local message for mpg_last_error()
mpg_status fail(mpg_status code, const std::string& msg);
// On a HIP error the runtime's per-thread error state is cleared before
// returning, so that the failure is reported once, through the status code.
#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      (void)hipGetLastError();                                                               \
      return fail(MPG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    }                                                                                        \
  } while (0)

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct mpg_scene {
  DevScene dev;
  std::vector<void*> allocs;
  int n_nodes = 0, max_depth = 0, n_tris = 0, n_verts = 0, n_objects = 0;
  std::vector<mpg_heightfield> hfs;
  const DevHF* dev_hf = nullptr;
  int n_params = 0;
  float scale = 1.0f;
  int device = 0;
  // surface-parameter updates (mpg_scene_set_params): BVH leaf order, the
  // triangle ranges under every node's children, the box padding, the top of
  // the geometry that theta does not move, one word of device scratch
  const int32_t* order = nullptr;
  const int32_t* ranges = nullptr;
  float pad = 0.0f;
  float zmax_static = -INFINITY;
  uint32_t* zmax_bits = nullptr;
  int32_t* param_err = nullptr;  // MPG_OK, or MPG_ERR_INVALID_ARG after a non-finite theta
};

// Lower bound on resident wavefronts per SIMD for the lane-refill kernels of
// chain length n (amdgpu_waves_per_eu): the compiler keeps such a kernel
// within 512 / waves registers per lane and spills the rest.  A refill walk
// spends most of its time waiting on ray-traversal loads, so more wavefronts
// in flight outweigh the spill traffic: lengths 1-2 at 5 (96 registers,
// against the compiler's own 4), length 3 at 4 (128, against 3), lengths
// 4-5 at 3 (168, against 2) and lengths 6-8 at 2 (256, against 1).
constexpr int refill_waves(int n) { return n <= 2 ? 5 : n == 3 ? 4 : n <= 5 ? 3 : 2; }

// persistent form: counter words per workspace, spatial cells per length
#define MPG_WS_COUNTERS 256
#define MPG_MAX_PARTS 8
#define MPG_CELL_RES 32
#define MPG_CELLS (MPG_CELL_RES * MPG_CELL_RES * MPG_CELL_RES)

struct mpg_workspace {
  int32_t cap = 0;
  int32_t* perm = nullptr;     // [cap] chain order for the persistent form
  int32_t* counters = nullptr; // [MPG_WS_COUNTERS] histogram / offsets / queue heads / batch box
  int32_t* cells = nullptr;    // [2 * 8 * MPG_CELLS] spatial-cell counts and cursors
  int32_t* aux = nullptr;      // [cap] scratch (sample cell ids, sorted indices)
  int single_stream = 0;       // 1: every per-length kernel on the caller's stream (no internal streams)
  std::vector<void*> allocs;
};

struct mpg_guide {
  mpg_guide_desc desc;
  int cells = 0;
  int32_t* valid = nullptr;
  float* pi = nullptr;
  float* mu = nullptr;
  float* cov = nullptr;
  float* chol = nullptr;
  int32_t* count = nullptr;
  int32_t* scratch = nullptr;  // fit_guide per-cell offsets and cursors
  std::vector<void*> allocs;
  DevGuide dev() const {
    DevGuide g;
    g.valid = valid; g.pi = pi; g.mu = mu; g.chol = chol;
    for (int a = 0; a < 3; ++a) { g.lo[a] = desc.lo[a]; g.hi[a] = desc.hi[a]; }
    g.res = desc.res; g.comps = desc.comps; g.target_obj = desc.target_obj;
    return g;
  }
};

template <class T>
inline hipError_t dalloc(std::vector<void*>& list, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) { list.push_back(q); *p = (T*)q; }
  return e;
}
template <class T>
inline hipError_t upload(std::vector<void*>& list, const T** p, const T* host, size_t count) {
  T* q = nullptr;
  hipError_t e = dalloc(list, &q, count);
  if (e != hipSuccess) return e;
  if (count) e = hipMemcpy(q, host, count * sizeof(T), hipMemcpyHostToDevice);
  *p = q;
  return e;
}
inline void free_all(std::vector<void*>& list) {
  for (void* p : list) (void)hipFree(p);
  list.clear();
}

// ---------------------------------------------------------------------------
// per-batch views
// ---------------------------------------------------------------------------
struct EpView {
  const float* xD;
  const float* nD;
  const float* xL;
  const uint8_t* len;
  const uint8_t* type;
  const int32_t* obj1;
  const float* off;  // glossy offset normals [2][K][N] or null
  int N;
};
__device__ __forceinline__ Offs chain_offs(const EpView& E, int c) { return Offs{E.off, (size_t)E.N, c}; }
__device__ __forceinline__ f3 ld_pt(const float* a, int N, int i) { return {a[i], a[N + i], a[2 * (size_t)N + i]}; }
__device__ __forceinline__ bool finite3(f3 v) { return isfinite(v.x) && isfinite(v.y) && isfinite(v.z); }

__device__ __forceinline__ Stack lane_stack(int depth) {
  extern __shared__ int lds_stack[];
  int lane = threadIdx.x & 63;
  int wave = threadIdx.x >> 6;
  return Stack{lds_stack + (size_t)wave * depth * 64 + lane, depth};
}

struct WalkIO {
  const int32_t* seed_prim;
  const float* seed_pos;
  const int8_t* seed_status;
  int32_t* prim_out;
  float* pos_out;
  int8_t* status;
  uint8_t* iters;
  uint64_t* sol;
  float* G;
  float* kappa;
  float* resid;
};

// Counter words of the persistent forms (workspace counters): per-length
// histogram, 64-padded bucket offsets, scatter cursors, queue heads (walk,
// finish, seeds, trials), batch bounding box.
enum : int {
  CTR_HIST = 0, CTR_OFF = 16, CTR_CUR = 32, CTR_HEAD = 48, CTR_HEAD2 = 56, CTR_BOX = 64, CTR_HEAD3 = 72,
  CTR_HEAD4 = 80, CTR_PHEAD = 128  // + (length - 1) * MPG_MAX_PARTS + part
};

// Pull the next 64-slot batch of a queue; wave-uniform result.
__device__ __forceinline__ int next_batch(int* head) {
  int base = 0;
  if ((threadIdx.x & 63) == 0) base = atomicAdd(head, 64);
  return __shfl(base, 0, 64);
}

// persistent-form helpers (mpg_persistent.hip): resident workgroups of a
// kernel across the device, length buckets of precomputed classes (1..8, 0 =
// none) in ws->perm and ws->counters
int resident_blocks(const void* fn, int threads, size_t lds);
mpg_status bucket_classes(int N, const int8_t* cls, mpg_workspace* ws, hipStream_t stream);
// per-length kernels run on MPG_WORKERS streams: wk[0] is the caller's
// stream, the others internal streams of the device that wait for the work
// queued on it so far; workers_join makes the caller's stream wait for them
#define MPG_WORKERS 4
mpg_status workers_fork(hipStream_t stream, hipStream_t wk[MPG_WORKERS]);
mpg_status workers_join(hipStream_t stream);

// host-side checks shared by every entry point
mpg_status walk_io(const mpg_chains* chains, const mpg_walk_out* wout, WalkIO* io);
mpg_status check_params(const mpg_scene* s, const mpg_walk_params* p, WalkParams* w, int* waves);
mpg_status check_endpoints(const mpg_endpoints* e, EpView* v);

// persistent form (its own translation unit)
mpg_status walk_persistent(const mpg_scene* s, const WalkParams& P, int waves, int bucketing, int refill,
                           int max_len, uint32_t length_order, const EpView& E, const WalkIO& io, mpg_workspace* ws,
                           hipStream_t stream);
mpg_status seeds_persistent(const mpg_scene* s, const DevGuide& G, const WalkParams& P, int waves,
                            int bucketing, uint32_t length_order, const EpView& E, uint64_t seed, uint32_t trial,
                            float alpha,
                            int32_t* prim_out, float* pos_out, int8_t* status, mpg_workspace* ws,
                            hipStream_t stream);
// plain FP32 finish pass over a whole batch (used by the unbucketed persistent form)
mpg_status launch_finish_plain(const mpg_scene* s, const WalkParams& P, const EpView& E, const WalkIO& io,
                               int max_len, int threads, size_t lds, hipStream_t stream);
