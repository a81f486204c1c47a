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
#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(MPG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
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
};

struct mpg_workspace {
  int32_t cap = 0;
  int32_t* perm = nullptr;     // [cap] chain order for the persistent form
  int32_t* counters = nullptr; // [64] histogram / offsets / queue heads
  int32_t* aux = nullptr;      // [cap] scratch (sample cell ids, sorted indices)
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
  int N;
};
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

// host-side checks shared by every entry point
mpg_status check_params(const mpg_scene* s, const mpg_walk_params* p, WalkParams* w, int* waves);
mpg_status check_endpoints(const mpg_endpoints* e, EpView* v);

// persistent form (its own translation unit)
mpg_status walk_persistent(const mpg_scene* s, const WalkParams& P, int waves, int bucketing, int refill,
                           int max_len, const EpView& E, const WalkIO& io, mpg_workspace* ws, hipStream_t stream);
// plain FP32 finish pass over a whole batch (used by the unbucketed persistent form)
mpg_status launch_finish_plain(const mpg_scene* s, const WalkParams& P, const EpView& E, const WalkIO& io,
                               int max_len, int threads, size_t lds, hipStream_t stream);
