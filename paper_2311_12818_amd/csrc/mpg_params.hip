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
inline float from_ordered_bits(uint32_t u) {
  uint32_t v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  float f;
  std::memcpy(&f, &v, 4);
  return f;
}

__global__ void k_set_word(uint32_t* p, uint32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// amplitude and phase of every sine of every height field
__global__ void k_hf_params(DevHF* hf, int n_hf, const float* theta) {
  int h = blockIdx.x, k = threadIdx.x;
  if (h >= n_hf || k >= hf[h].n_sines) return;
  hf[h].amp[k] = theta[hf[h].param_base + 2 * k];
  hf[h].phase[k] = theta[hf[h].param_base + 2 * k + 1];
}

// vertices of one height field: z = z0 + sum a sin(f (cos psi x + sin psi y) + phi),
// n = normalize(-dz/dx, -dz/dy, 1), evaluated in FP64 and stored in FP32
__global__ void k_hf_vertices(const DevHF* hf, int h, float z0, float4* vpos, float4* vnrm, uint32_t* zmax_bits) {
  const DevHF& H = hf[h];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H.n_verts) return;
  int v = H.first_vert + i;
  float4 p = vpos[v];
  double x = p.x, y = p.y;
  double z = z0, hx = 0.0, hy = 0.0;
  for (int k = 0; k < H.n_sines; ++k) {
    double cp = cos((double)H.psi[k]), sp = sin((double)H.psi[k]);
    double arg = (double)H.freq[k] * (cp * x + sp * y) + (double)H.phase[k];
    z += (double)H.amp[k] * sin(arg);
    double c = (double)H.amp[k] * (double)H.freq[k] * cos(arg);
    hx += c * cp;
    hy += c * sp;
  }
  double il = 1.0 / sqrt(hx * hx + hy * hy + 1.0);
  float nx = (float)(-hx * il), ny = (float)(-hy * il), nz = (float)il;
  float l = sqrtf(nx * nx + ny * ny + nz * nz);
  float zf = (float)z;
  vpos[v] = make_float4(p.x, p.y, zf, 0.f);
  vnrm[v] = make_float4(nx / l, ny / l, nz / l, 0.f);
  atomicMax(zmax_bits, ordered_bits(zf));
}

// triangle copies in BVH leaf order (first vertex carries the primitive id)
__global__ void k_tri_copies(int n_tris, const int32_t* order, const int4* tri_idx, const float4* vpos, float4* tri_v) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_tris) return;
  int t = order[k];
  int4 id = tri_idx[t];
  float4 a = vpos[id.x], b = vpos[id.y], c = vpos[id.z];
  tri_v[3 * (size_t)k + 0] = make_float4(a.x, a.y, a.z, __int_as_float(t));
  tri_v[3 * (size_t)k + 1] = make_float4(b.x, b.y, b.z, 0.f);
  tri_v[3 * (size_t)k + 2] = make_float4(c.x, c.y, c.z, 0.f);
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
                                               float pad) {
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

// per-object area prefix sums (one thread per run, sequential in FP64, the
// builder's order)
__global__ void k_area_cdf(int n_runs, const int2* range, const int* cdf_prim, const int4* tri_idx,
                           const float4* vpos, const float4* spheres, double* cdf) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_runs) return;
  int2 rg = range[r];
  double acc = 0.0;
  for (int i = 0; i < rg.y; ++i) {
    int p = cdf_prim[rg.x + i];
    double area;
    if (p >= 0) {
      int4 id = tri_idx[p];
      float4 a = vpos[id.x], b = vpos[id.y], c = vpos[id.z];
      double e1[3] = {(double)b.x - a.x, (double)b.y - a.y, (double)b.z - a.z};
      double e2[3] = {(double)c.x - a.x, (double)c.y - a.y, (double)c.z - a.z};
      double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2];
      double cz = e1[0] * e2[1] - e1[1] * e2[0];
      area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    } else {
      double rad = spheres[-1 - p].w;
      area = 4.0 * M_PI * rad * rad;
    }
    acc += area;
    cdf[rg.x + i] = acc;
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
  std::vector<float> th(n_params);
  HIP_TRY(hipMemcpyAsync(th.data(), d_theta, n_params * sizeof(float), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (float v : th)
    if (!std::isfinite(v)) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_set_params: non-finite theta");
  DevScene& D = s->dev;
  const int n_hf = (int)s->hfs.size();
  hipLaunchKernelGGL(k_set_word, dim3(1), dim3(64), 0, stream, s->zmax_bits, 0u);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_hf_params, dim3(n_hf), dim3(64), 0, stream, (DevHF*)s->dev_hf, n_hf, d_theta);
  HIP_TRY(hipGetLastError());
  for (int h = 0; h < n_hf; ++h) {
    int nv = s->hfs[h].res * s->hfs[h].res;
    hipLaunchKernelGGL(k_hf_vertices, dim3((nv + 255) / 256), dim3(256), 0, stream, s->dev_hf, h, s->hfs[h].z0,
                       (float4*)D.vpos, (float4*)D.vnrm, s->zmax_bits);
    HIP_TRY(hipGetLastError());
  }
  if (s->n_tris > 0) {
    hipLaunchKernelGGL(k_tri_copies, dim3((s->n_tris + 255) / 256), dim3(256), 0, stream, s->n_tris, s->order,
                       D.tri_idx, D.vpos, (float4*)D.tri_v);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_refit, dim3((s->n_nodes + 3) / 4), dim3(256), 0, stream, s->n_nodes, s->ranges, D.tri_v,
                       (float*)D.nodes, s->pad);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_area_cdf, dim3((s->n_objects + 1 + 63) / 64), dim3(64), 0, stream, s->n_objects + 1, D.cdf_range, D.cdf_prim, D.tri_idx,
                     D.vpos, D.spheres, (double*)D.cdf);
  HIP_TRY(hipGetLastError());
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, s->zmax_bits, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  D.zmax = bits == 0 ? s->zmax_static : std::max(s->zmax_static, from_ordered_bits(bits));
  for (int h = 0; h < n_hf; ++h) {
    mpg_heightfield& H = s->hfs[h];
    int base = 0;
    for (int k = 0; k < h; ++k) base += 2 * s->hfs[k].n_sines;
    for (int k = 0; k < H.n_sines; ++k) { H.amp[k] = th[base + 2 * k]; H.phase[k] = th[base + 2 * k + 1]; }
  }
  return MPG_OK;
}
