// Plain form of the adjoint (its own translation unit: every length is
// inlined into one kernel, which makes it the slowest unit to compile).
#include "mpg_adjoint.h"

template <int NMAX>
__global__ void __launch_bounds__(256) k_adjoint(DevScene S, WalkParams P, EpView E, AdjIO io) {
  __shared__ float acc[64];
  if (threadIdx.x < 64) acc[threadIdx.x] = 0.0f;
  __syncthreads();
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < E.N) {
    int n = E.len[c];
    bool ok = io.status[c] == ST_CONVERGED && n >= 1 && n <= NMAX;
    for (int i = 0; ok && i < n; ++i) {
      int pr = io.prim[(size_t)i * E.N + c];
      ok = pr >= -S.n_spheres && pr < S.n_tris;
    }
    if (!ok) {
      for (int a = 0; a < 3; ++a) {
        io.grad_xD[(size_t)a * E.N + c] = 0.0f;
        io.grad_xL[(size_t)a * E.N + c] = 0.0f;
      }
    } else {
      switch (n) {
        case 1: adjoint_one<1>(S, P, E, io, c, acc); break;
        case 2: if (NMAX >= 2) adjoint_one<(NMAX >= 2 ? 2 : 1)>(S, P, E, io, c, acc); break;
        case 3: if (NMAX >= 3) adjoint_one<(NMAX >= 3 ? 3 : 1)>(S, P, E, io, c, acc); break;
        case 4: if (NMAX >= 4) adjoint_one<(NMAX >= 4 ? 4 : 1)>(S, P, E, io, c, acc); break;
        case 5: if (NMAX >= 5) adjoint_one<(NMAX >= 5 ? 5 : 1)>(S, P, E, io, c, acc); break;
        case 6: if (NMAX >= 6) adjoint_one<(NMAX >= 6 ? 6 : 1)>(S, P, E, io, c, acc); break;
        case 7: if (NMAX >= 7) adjoint_one<(NMAX >= 7 ? 7 : 1)>(S, P, E, io, c, acc); break;
        default: if (NMAX >= 8) adjoint_one<(NMAX >= 8 ? 8 : 1)>(S, P, E, io, c, acc); break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < io.n_params && threadIdx.x < 64 && acc[threadIdx.x] != 0.0f)
    atomicAdd(&io.grad_theta[threadIdx.x], acc[threadIdx.x]);
}

typedef void (*adj_kernel_t)(DevScene, WalkParams, EpView, AdjIO);
static adj_kernel_t adjoint_kernel(int nmax) {
  switch (nmax) {
    case 1: return k_adjoint<1>;
    case 2: return k_adjoint<2>;
    case 3: return k_adjoint<3>;
    case 4: return k_adjoint<4>;
    case 5: return k_adjoint<5>;
    case 6: return k_adjoint<6>;
    case 7: return k_adjoint<7>;
    default: return k_adjoint<8>;
  }
}

mpg_status launch_adjoint_plain(const mpg_scene* s, const WalkParams& P, const EpView& E, const AdjIO& io, int max_len,
                                hipStream_t stream) {
  const int threads = 256;  // k_adjoint's launch bound
  hipLaunchKernelGGL(adjoint_kernel(max_len), dim3((E.N + threads - 1) / threads), dim3(threads), 0, stream, s->dev,
                     P, E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}
