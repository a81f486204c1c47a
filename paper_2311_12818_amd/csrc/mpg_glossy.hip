// Offset normals of glossy chains (Sec. 5.7): sampled from the GGX
// (Trowbridge-Reitz) distribution of microfacet normals, D(m) cos theta_m
// (Walter, Marschner, Li, Torrance, EGSR 2007), before the manifold walk; the
// walk then solves the specular chain about these normals.
#include "mpg_internal.h"

namespace {

// tan^2 theta_m = a^2 u / (1 - u), phi = 2 pi v, (o_s, o_t) = sin theta_m
// (cos phi, sin phi); vertex i of chain c takes uniforms 2 (i mod 4) and
// 2 (i mod 4) + 1 of the Philox block (c, trial, 16 + i / 4).
__global__ void k_sample_offsets(int N, uint64_t seed, uint64_t trial, float rough, float* off) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const size_t NN = N;
#pragma unroll
  for (int b = 0; b < KMAX / 4; ++b) {
    const U8 U = philox_uniforms(seed, (uint64_t)c, trial, (uint64_t)(16 + b));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 4 * b + q;
      const float u = U.u[2 * q], v = U.u[2 * q + 1];
      const float t2 = rough * rough * u / (1.0f - u);
      const float st = sqrtf(t2 / (1.0f + t2));
      float sn, cs;
      sincospif(2.0f * v, &sn, &cs);
      off[(0 * KMAX + i) * NN + c] = st * cs;
      off[(1 * KMAX + i) * NN + c] = st * sn;
    }
  }
}

}  // namespace

extern "C" mpg_status sample_offsets(int32_t N, uint64_t philox_seed, uint32_t trial, float roughness,
                                     float* d_offset, void* stream) {
  if (N < 0 || (N > 0 && !d_offset) || !(roughness >= 0.0f && roughness <= 1.0f))
    return fail(MPG_ERR_INVALID_ARG, "sample_offsets: bad argument");
  if (N == 0) return MPG_OK;
  hipLaunchKernelGGL(k_sample_offsets, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, N, philox_seed,
                     (uint64_t)trial, roughness, d_offset);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}
