// Plain form of the adjoint: one thread per chain, every length up to NMAX
// inlined into one kernel.  The instantiations are spread over three
// translation units (NMAX 1-5, 6-7, 8) so that they compile in parallel.
#pragma once
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
adj_kernel_t adjoint_kernel_1to5(int nmax);
adj_kernel_t adjoint_kernel_6to7(int nmax);
adj_kernel_t adjoint_kernel_8();
