// Counting walk: entry point (the kernels are instantiated in mpg_count_*.hip).
#include "mpg_count.h"

__global__ void k_zero_u64(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ULL;
}

static count_kernel_t count_kernel(int nmax) {
  if (nmax <= 5) return count_kernel_1to5(nmax);
  if (nmax <= 7) return count_kernel_6to7(nmax);
  return count_kernel_8();
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

