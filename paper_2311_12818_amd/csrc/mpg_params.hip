// Surface-parameter update: new height-field parameters theta (the surface
// parameters the adjoint differentiates, Sec. 5.2) move the height-field
// vertices and normals; the triangle copies in BVH leaf order, the BVH boxes
// (same topology, every child box recomputed from the triangles under it),
// the per-object area tables used by p_0 (Sec. 5.4) and the scene top follow.
#include <cfloat>

#include "mpg_internal.h"

namespace {

__device__ __forceinline__ uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered_bits(uint32_t u) {
  uint32_t v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(v);
}

// Validates theta and installs it: a single workgroup checks every value;
// when one is not finite the error word is set and the scene is left as it
// was (every later kernel of the update reads the word and does nothing).
// Otherwise the amplitude and phase of every sine are stored and the scene
// top accumulator is reset.
__global__ void __launch_bounds__(256) k_hf_params(DevHF* hf, int n_hf, const float* theta, int n_params,
                                                   int32_t* err, uint32_t* zmax_bits) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n_params; i += blockDim.x)
    if (!isfinite(theta[i])) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    *err = bad ? MPG_ERR_INVALID_ARG : MPG_OK;
    if (!bad) *zmax_bits = 0u;
  }
  if (bad) return;
  for (int h = 0; h < n_hf; ++h)
    for (int k = threadIdx.x; k < hf[h].n_sines; k += blockDim.x) {
      hf[h].amp[k] = theta[hf[h].param_base + 2 * k];
      hf[h].phase[k] = theta[hf[h].param_base + 2 * k + 1];
    }
}

// vertices of one height field: z = z0 + sum a sin(f (cos psi x + sin psi y) + phi),
// n = normalize(-dz/dx, -dz/dy, 1), in FP32
__global__ void k_hf_vertices(const DevHF* hf, int h, float z0, float4* vpos, float4* vnrm, uint32_t* zmax_bits,
                              const int32_t* err) {
  if (*err != MPG_OK) return;
  const DevHF& H = hf[h];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H.n_verts) return;
  int v = H.first_vert + i;
  float4 p = vpos[v];
  float z = 0.0f, hx = 0.0f, hy = 0.0f;
  for (int k = 0; k < H.n_sines; ++k) {
    float sp, cp;
    sincosf(H.psi[k], &sp, &cp);
    float arg = H.freq[k] * (cp * p.x + sp * p.y) + H.phase[k];
    float sa, ca;
    sincosf(arg, &sa, &ca);
    z += H.amp[k] * sa;
    float c = H.amp[k] * H.freq[k] * ca;
    hx += c * cp;
    hy += c * sp;
  }
  float il = rsqrtf(hx * hx + hy * hy + 1.0f);
  float nx = -hx * il, ny = -hy * il, nz = il;
  float l = sqrtf(nx * nx + ny * ny + nz * nz);
  float zf = z0 + z;
  vpos[v] = make_float4(p.x, p.y, zf, 0.f);
  vnrm[v] = make_float4(nx / l, ny / l, nz / l, 0.f);
  atomicMax(zmax_bits, ordered_bits(zf));
}

// scene top used to lift guided seeds: the static geometry's top and the
// highest height-field vertex
__global__ void k_zmax(const uint32_t* zmax_bits, float zmax_static, float* zmax, const int32_t* err) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || *err != MPG_OK) return;
  uint32_t b = *zmax_bits;
  *zmax = b == 0u ? zmax_static : fmaxf(zmax_static, from_ordered_bits(b));
}

// triangle copies in BVH leaf order (first vertex carries the primitive id)
// and the per-primitive geometry records (vertex positions keep the object,
// material and index of refraction in their w slots; normals follow)
__global__ void k_tri_copies(int n_tris, const int32_t* order, const int4* tri_idx, const float4* vpos,
                             const float4* vnrm, float4* tri_v, float4* tri_geo, const int32_t* err) {
  if (*err != MPG_OK) return;
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_tris) return;
  int t = order[k];
  int4 id = tri_idx[t];
  float4 a = vpos[id.x], b = vpos[id.y], c = vpos[id.z];
  tri_v[3 * (size_t)k + 0] = make_float4(a.x, a.y, a.z, __int_as_float(t));
  tri_v[3 * (size_t)k + 1] = make_float4(b.x, b.y, b.z, 0.f);
  tri_v[3 * (size_t)k + 2] = make_float4(c.x, c.y, c.z, 0.f);
  float4* g = tri_geo + 6 * (size_t)t;
  g[0] = make_float4(a.x, a.y, a.z, tri_geo[6 * (size_t)t].w);
  g[1] = make_float4(b.x, b.y, b.z, tri_geo[6 * (size_t)t + 1].w);
  g[2] = make_float4(c.x, c.y, c.z, tri_geo[6 * (size_t)t + 2].w);
  g[3] = vnrm[id.x];
  g[4] = vnrm[id.y];
  g[5] = vnrm[id.z];
}

__device__ __forceinline__ float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// BVH refit: one wavefront per 4-wide node; each child box is the bounding
// box of the triangles of its range, padded like the builder's (an empty
// child keeps its box at +infinity)
__global__ void __launch_bounds__(256) k_refit(int n_nodes, const int32_t* ranges, const float4* tri_v, float* nodes,
                                               float pad, const int32_t* err) {
  if (*err != MPG_OK) return;
  int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (g >= n_nodes) return;
  float* f = nodes + 32 * (size_t)g;
  for (int q = 0; q < 4; ++q) {
    int start = ranges[8 * (size_t)g + 2 * q], count = ranges[8 * (size_t)g + 2 * q + 1];
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int i = lane; i < 3 * count; i += 64) {
      float4 p = tri_v[3 * (size_t)start + i];
      lo[0] = fminf(lo[0], p.x); lo[1] = fminf(lo[1], p.y); lo[2] = fminf(lo[2], p.z);
      hi[0] = fmaxf(hi[0], p.x); hi[1] = fmaxf(hi[1], p.y); hi[2] = fmaxf(hi[2], p.z);
    }
    for (int a = 0; a < 3; ++a) {
      lo[a] = wave_min(lo[a]);
      hi[a] = wave_max(hi[a]);
      if (count > 0) {
        lo[a] -= pad;
        hi[a] += pad;
      } else {
        lo[a] = INFINITY;
        hi[a] = INFINITY;
      }
    }
    if (lane == 0) {
      for (int a = 0; a < 3; ++a) {
        f[4 * a + q] = lo[a];
        f[12 + 4 * a + q] = hi[a];
      }
    }
  }
}

// per-object area prefix sums (one thread per run, the builder's order) as
// FP32 pairs hi + lo: each area is added with Knuth's two-sum, whose rounding
// error goes into lo, and the pair is renormalized, so the prefixes carry
// about 48 significant bits
__global__ void k_area_cdf(int n_runs, const int2* range, const int* cdf_prim, const int4* tri_idx,
                           const float4* vpos, const float4* spheres, float2* cdf, const int32_t* err) {
  if (*err != MPG_OK) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_runs) return;
  int2 rg = range[r];
  float hi = 0.0f, lo = 0.0f;
  for (int i = 0; i < rg.y; ++i) {
    int p = cdf_prim[rg.x + i];
    float area;
    if (p >= 0) {
      int4 id = tri_idx[p];
      float4 a = vpos[id.x], b = vpos[id.y], c = vpos[id.z];
      float e1[3] = {b.x - a.x, b.y - a.y, b.z - a.z};
      float e2[3] = {c.x - a.x, c.y - a.y, c.z - a.z};
      float cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2];
      float cz = e1[0] * e2[1] - e1[1] * e2[0];
      area = 0.5f * sqrtf(cx * cx + cy * cy + cz * cz);
    } else {
      float rad = spheres[-1 - p].w;
      area = 4.0f * (float)M_PI * rad * rad;
    }
    float s = hi + area;
    float bb = s - hi;
    float e = (hi - (s - bb)) + (area - bb);
    lo += e;
    hi = s + lo;
    lo = lo - (hi - s);
    cdf[rg.x + i] = make_float2(hi, lo);
  }
}

}  // namespace

extern "C" mpg_status mpg_scene_set_params(mpg_scene* s, const float* d_theta, int32_t n_params, void* stream_) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_set_params: NULL scene");
  if (n_params != s->n_params)
    return fail(MPG_ERR_INVALID_ARG, "mpg_scene_set_params: n_params differs from the scene's parameter count");
  if (n_params == 0) return MPG_OK;
  if (!d_theta) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_set_params: NULL theta");
  hipStream_t stream = (hipStream_t)stream_;
  DevScene& D = s->dev;
  const int n_hf = (int)s->hfs.size();
  hipLaunchKernelGGL(k_hf_params, dim3(1), dim3(256), 0, stream, (DevHF*)s->dev_hf, n_hf, d_theta, n_params,
                     s->param_err, s->zmax_bits);
  HIP_TRY(hipGetLastError());
  for (int h = 0; h < n_hf; ++h) {
    int nv = s->hfs[h].res * s->hfs[h].res;
    hipLaunchKernelGGL(k_hf_vertices, dim3((nv + 255) / 256), dim3(256), 0, stream, s->dev_hf, h, s->hfs[h].z0,
                       (float4*)D.vpos, (float4*)D.vnrm, s->zmax_bits, (const int32_t*)s->param_err);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_zmax, dim3(1), dim3(64), 0, stream, (const uint32_t*)s->zmax_bits, s->zmax_static,
                     (float*)D.zmax, (const int32_t*)s->param_err);
  HIP_TRY(hipGetLastError());
  if (s->n_tris > 0) {
    hipLaunchKernelGGL(k_tri_copies, dim3((s->n_tris + 255) / 256), dim3(256), 0, stream, s->n_tris, s->order,
                       D.tri_idx, D.vpos, D.vnrm, (float4*)D.tri_v, (float4*)D.tri_geo,
                       (const int32_t*)s->param_err);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_refit, dim3((s->n_nodes + 3) / 4), dim3(256), 0, stream, s->n_nodes, s->ranges, D.tri_v,
                       (float*)D.nodes, s->pad, (const int32_t*)s->param_err);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_area_cdf, dim3((s->n_objects + 1 + 63) / 64), dim3(64), 0, stream, s->n_objects + 1,
                     D.cdf_range, D.cdf_prim, D.tri_idx, D.vpos, D.spheres, (float2*)D.cdf,
                     (const int32_t*)s->param_err);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

extern "C" mpg_status mpg_scene_params_error(const mpg_scene* s, int32_t* d_out, void* stream) {
  if (!s || !d_out) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_params_error: NULL scene or output");
  HIP_TRY(hipMemcpyAsync(d_out, s->param_err, sizeof(int32_t), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return MPG_OK;
}
