#include "mpg_adjoint.h"

// Persistent form: converged chains bucketed by length, one kernel per length
// (its own register budget, no mixing of lengths inside a wavefront); each
// workgroup adds its theta partial sums to the output once at the end.
__device__ __forceinline__ bool adjoint_target(const DevScene& S, const EpView& E, const AdjIO& io, int c) {
  int n = E.len[c];
  bool ok = io.status[c] == ST_CONVERGED && n >= 1 && n <= KMAX;
  for (int i = 0; ok && i < n; ++i) {
    int pr = io.prim[(size_t)i * E.N + c];
    ok = pr >= -S.n_spheres && pr < S.n_tris;
  }
  return ok;
}

__global__ void __launch_bounds__(256) k_adjoint_classify(DevScene S, EpView E, AdjIO io, int max_len, int8_t* cls) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  bool ok = adjoint_target(S, E, io, c) && E.len[c] <= max_len;
  cls[c] = (int8_t)(ok ? E.len[c] : 0);
  if (!ok) {
    for (int a = 0; a < 3; ++a) {
      io.grad_xD[(size_t)a * E.N + c] = 0.0f;
      io.grad_xL[(size_t)a * E.N + c] = 0.0f;
    }
  }
}

// At least two wavefronts per SIMD (the compiler's own choice is one, with
// every register used): 8.4 against 10.6 ms for 2^20 chains of length 2-4;
// three or four were slower (spills).
template <int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_adjoint_persist(DevScene S, WalkParams P, EpView E, AdjIO io, int* ctr,
                                                         const int* perm) {
  __shared__ float acc[64];
  if (threadIdx.x < 64) acc[threadIdx.x] = 0.0f;
  __syncthreads();
  const int start = ctr[CTR_OFF + N];
  const int end = ctr[CTR_OFF + N + 1];
  const int lane = threadIdx.x & 63;
  for (;;) {
    int base = next_batch(&ctr[CTR_HEAD + N - 1]);
    if (start + base >= end) break;
    int c = perm[start + base + lane];
    if (c >= 0) adjoint_one<N>(S, P, E, io, c, acc);
  }
  __syncthreads();
  if (threadIdx.x < io.n_params && threadIdx.x < 64 && acc[threadIdx.x] != 0.0f)
    atomicAdd(&io.grad_theta[threadIdx.x], acc[threadIdx.x]);
}

typedef void (*adj_persist_t)(DevScene, WalkParams, EpView, AdjIO, int*, const int*);
static adj_persist_t adjoint_persist_kernel(int n) {
  switch (n) {
    case 1: return k_adjoint_persist<1>;
    case 2: return k_adjoint_persist<2>;
    case 3: return k_adjoint_persist<3>;
    case 4: return k_adjoint_persist<4>;
    case 5: return k_adjoint_persist<5>;
    case 6: return k_adjoint_persist<6>;
    case 7: return k_adjoint_persist<7>;
    default: return k_adjoint_persist<8>;
  }
}

extern "C" mpg_status manifold_walk_adjoint(const mpg_scene* s, const mpg_walk_params* p, const mpg_endpoints* ep,
                                            const mpg_chains* converged, const int8_t* d_status,
                                            const float* d_grad_pos, const float* d_grad_G, float* d_grad_xD,
                                            float* d_grad_xL, float* d_grad_theta, mpg_workspace* ws,
                                            void* stream) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_adjoint: NULL scene");
  WalkParams P;
  int waves;
  EpView E;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!converged || !converged->d_prim || !converged->d_pos || !d_status || !d_grad_xD || !d_grad_xL)
    return fail(MPG_ERR_INVALID_ARG, "manifold_walk_adjoint: NULL argument");
  if (s->n_params > 0 && !d_grad_theta) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_adjoint: NULL grad_theta");
  AdjIO io;
  io.prim = converged->d_prim;
  io.pos = converged->d_pos;
  io.status = d_status;
  io.grad_pos = d_grad_pos;
  io.grad_G = d_grad_G;
  io.grad_xD = d_grad_xD;
  io.grad_xL = d_grad_xL;
  io.grad_theta = d_grad_theta;
  io.hf = s->dev_hf;
  io.n_hf = (int)s->hfs.size();
  io.n_params = s->n_params;
  if (p->form == MPG_FORM_PERSISTENT && p->bucketing) {
    if (!ws || ws->cap < E.N) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_adjoint: workspace too small");
    const int threads = 64 * waves;
    int8_t* cls = (int8_t*)ws->aux;
    hipLaunchKernelGGL(k_adjoint_classify, dim3((E.N + 255) / 256), dim3(256), 0, (hipStream_t)stream, s->dev, E, io,
                       p->max_len, cls);
    HIP_TRY(hipGetLastError());
    if ((st = bucket_classes(E.N, cls, ws, (hipStream_t)stream)) != MPG_OK) return st;
    hipStream_t wk[MPG_WORKERS];
    if ((st = workers_fork((hipStream_t)stream, wk)) != MPG_OK) return st;
    for (int n = p->max_len, q = 0; n >= 1; --n, q = (q + 1) % MPG_WORKERS) {
      adj_persist_t k = adjoint_persist_kernel(n);
      int grid = resident_blocks((const void*)k, threads, 0);
      hipLaunchKernelGGL(k, dim3(grid), dim3(threads), 0, wk[q], s->dev, P, E, io, ws->counters,
                         (const int*)ws->perm);
      HIP_TRY(hipGetLastError());
    }
    return workers_join((hipStream_t)stream);
  }
  return launch_adjoint_plain(s, P, E, io, p->max_len, (hipStream_t)stream);
}
