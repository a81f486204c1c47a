// Counting walk: the plain walk with every unit of work tallied (untimed; it
// gives the algorithmic work of a launch).  The instantiations are spread
// over three translation units (NMAX 1-5, 6-7, 8) so that they compile in
// parallel.
#pragma once
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

typedef void (*count_kernel_t)(DevScene, WalkParams, EpView, WalkIO, unsigned long long*);
count_kernel_t count_kernel_1to5(int nmax);
count_kernel_t count_kernel_6to7(int nmax);
count_kernel_t count_kernel_8();
