// Counting walk: the plain walk with every unit of work tallied (untimed; it
// gives the algorithmic work of a launch).
#include "mpg_internal.h"
#include "mpg_walk.h"

template <int NMAX>
__global__ void __launch_bounds__(256) k_walk_count(DevScene S, WalkParams P, EpView E, WalkIO io,
                                                    unsigned long long* counts) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack base = lane_stack(P.depth);
  CountStack stk{base.base, base.depth, 0, 0, 0, 0, 0, 0, 0};
  if (c < E.N) walk_dispatch<NMAX>(S, P, E, io, c, stk);
  if (c < E.N) finish_dispatch<NMAX>(S, P, E, io, c, stk);
  if (c < E.N && io.status[c] == ST_NEEDS_FP64) {
    int n = E.len[c];
    switch (n) {
      case 1: fp64_one<1>(S, P, E, io, c, stk); break;
      case 2: if (NMAX >= 2) fp64_one<(NMAX >= 2 ? 2 : 1)>(S, P, E, io, c, stk); break;
      case 3: if (NMAX >= 3) fp64_one<(NMAX >= 3 ? 3 : 1)>(S, P, E, io, c, stk); break;
      case 4: if (NMAX >= 4) fp64_one<(NMAX >= 4 ? 4 : 1)>(S, P, E, io, c, stk); break;
      case 5: if (NMAX >= 5) fp64_one<(NMAX >= 5 ? 5 : 1)>(S, P, E, io, c, stk); break;
      case 6: if (NMAX >= 6) fp64_one<(NMAX >= 6 ? 6 : 1)>(S, P, E, io, c, stk); break;
      case 7: if (NMAX >= 7) fp64_one<(NMAX >= 7 ? 7 : 1)>(S, P, E, io, c, stk); break;
      default: if (NMAX >= 8) fp64_one<(NMAX >= 8 ? 8 : 1)>(S, P, E, io, c, stk); break;
    }
  }
  if (c < E.N) {
    atomicAdd(&counts[0], (unsigned long long)stk.nbox);
    atomicAdd(&counts[1], (unsigned long long)stk.ntri);
    atomicAdd(&counts[2], (unsigned long long)stk.nsph);
    atomicAdd(&counts[3], (unsigned long long)stk.nray);
    atomicAdd(&counts[4], (unsigned long long)stk.nvc);
    atomicAdd(&counts[5], (unsigned long long)stk.nvj);
    atomicAdd(&counts[6], (unsigned long long)stk.nvj64);
    atomicAdd(&counts[7], 1ULL);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ULL;
}

typedef void (*count_kernel_t)(DevScene, WalkParams, EpView, WalkIO, unsigned long long*);
static count_kernel_t count_kernel(int nmax) {
  switch (nmax) {
    case 1: return k_walk_count<1>;
    case 2: return k_walk_count<2>;
    case 3: return k_walk_count<3>;
    case 4: return k_walk_count<4>;
    case 5: return k_walk_count<5>;
    case 6: return k_walk_count<6>;
    case 7: return k_walk_count<7>;
    default: return k_walk_count<8>;
  }
}
extern "C" mpg_status mpg_walk_count(const mpg_scene* s, const mpg_walk_params* p, const mpg_endpoints* ep,
                                     const mpg_chains* seeds, const int8_t* d_seed_status, mpg_chains* out,
                                     const mpg_walk_out* wout, uint64_t* d_counts, void* stream) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "mpg_walk_count: NULL scene");
  WalkParams P;
  int waves;
  EpView E;
  WalkIO io;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (!d_counts) return fail(MPG_ERR_INVALID_ARG, "mpg_walk_count: NULL counts");
  if ((st = walk_io(out, wout, &io)) != MPG_OK) return st;
  if (!seeds || !seeds->d_prim || !seeds->d_pos) return fail(MPG_ERR_INVALID_ARG, "mpg_walk_count: NULL seeds");
  io.seed_prim = seeds->d_prim; io.seed_pos = seeds->d_pos; io.seed_status = d_seed_status;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, (hipStream_t)stream, (unsigned long long*)d_counts, 8);
  HIP_TRY(hipGetLastError());
  if (E.N == 0) return MPG_OK;
  int threads = 64 * waves;
  size_t lds = (size_t)waves * P.depth * 64 * 4;
  hipLaunchKernelGGL(count_kernel(p->max_len), dim3((E.N + threads - 1) / threads), dim3(threads), lds,
                     (hipStream_t)stream, s->dev, P, E, io, (unsigned long long*)d_counts);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

