#include "mpg_internal.h"

// Guide handles and fit_guide (weighted EM per cell).
extern "C" mpg_status mpg_guide_create(const mpg_guide_desc* d, mpg_guide** out) {
  if (!d || !out) return fail(MPG_ERR_INVALID_ARG, "mpg_guide_create: NULL argument");
  if (d->res < 1 || d->res > 128 || d->comps < 1 || d->comps > 8 || d->em_iters < 0 || d->min_samples < 1)
    return fail(MPG_ERR_INVALID_ARG, "mpg_guide_create: res 1..128, comps 1..8, em_iters >= 0, min_samples >= 1");
  for (int a = 0; a < 3; ++a)
    if (!(d->hi[a] > d->lo[a])) return fail(MPG_ERR_INVALID_ARG, "mpg_guide_create: empty bounding box");
  mpg_guide* g = new mpg_guide();
  g->desc = *d;
  g->cells = d->res * d->res * d->res;
  size_t C = g->cells, K = d->comps;
  hipError_t e;
  if ((e = dalloc(g->allocs, &g->valid, C)) != hipSuccess || (e = dalloc(g->allocs, &g->pi, C * K)) != hipSuccess ||
      (e = dalloc(g->allocs, &g->mu, C * K * 2)) != hipSuccess ||
      (e = dalloc(g->allocs, &g->cov, C * K * 3)) != hipSuccess ||
      (e = dalloc(g->allocs, &g->chol, C * K * 3)) != hipSuccess ||
      (e = dalloc(g->allocs, &g->count, C)) != hipSuccess ||
      (e = dalloc(g->allocs, &g->scratch, 2 * C + 1)) != hipSuccess ||
      (e = hipMemset(g->valid, 0, C * sizeof(int32_t))) != hipSuccess ||
      (e = hipMemset(g->count, 0, C * sizeof(int32_t))) != hipSuccess) {
    free_all(g->allocs);
    delete g;
    return fail(MPG_ERR_HIP, std::string("mpg_guide_create: ") + hipGetErrorString(e));
  }
  *out = g;
  return MPG_OK;
}

extern "C" void mpg_guide_destroy(mpg_guide* g) {
  if (!g) return;
  free_all(g->allocs);
  delete g;
}

extern "C" mpg_status mpg_guide_upload(mpg_guide* g, const int32_t* valid, const float* pi, const float* mu,
                                       const float* cov) {
  if (!g || !valid || !pi || !mu || !cov) return fail(MPG_ERR_INVALID_ARG, "mpg_guide_upload: NULL argument");
  size_t C = g->cells, K = g->desc.comps;
  std::vector<float> chol(C * K * 3);
  for (size_t i = 0; i < C * K; ++i) {
    float a = cov[3 * i], b = cov[3 * i + 1], c = cov[3 * i + 2];
    float l00 = std::sqrt(std::max(a, 0.0f));
    float l10 = l00 > 0.0f ? b / l00 : 0.0f;
    float l11 = std::sqrt(std::max(c - l10 * l10, 0.0f));
    chol[3 * i] = l00; chol[3 * i + 1] = l10; chol[3 * i + 2] = l11;
  }
  HIP_TRY(hipMemcpy(g->valid, valid, C * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(g->pi, pi, C * K * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(g->mu, mu, C * K * 2 * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(g->cov, cov, C * K * 3 * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(g->chol, chol.data(), C * K * 3 * sizeof(float), hipMemcpyHostToDevice));
  return MPG_OK;
}

extern "C" mpg_status mpg_guide_download(const mpg_guide* g, int32_t* valid, float* pi, float* mu, float* cov,
                                         int32_t* count) {
  if (!g) return fail(MPG_ERR_INVALID_ARG, "mpg_guide_download: NULL guide");
  size_t C = g->cells, K = g->desc.comps;
  HIP_TRY(hipDeviceSynchronize());
  if (valid) HIP_TRY(hipMemcpy(valid, g->valid, C * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (pi) HIP_TRY(hipMemcpy(pi, g->pi, C * K * sizeof(float), hipMemcpyDeviceToHost));
  if (mu) HIP_TRY(hipMemcpy(mu, g->mu, C * K * 2 * sizeof(float), hipMemcpyDeviceToHost));
  if (cov) HIP_TRY(hipMemcpy(cov, g->cov, C * K * 3 * sizeof(float), hipMemcpyDeviceToHost));
  if (count) HIP_TRY(hipMemcpy(count, g->count, C * sizeof(int32_t), hipMemcpyDeviceToHost));
  return MPG_OK;
}

// ---------------------------------------------------------------------------
// fit_guide: weighted EM per cell (weights w = T <1/P>, Eq. eq_weight)
// ---------------------------------------------------------------------------
struct EMDesc {
  float lo[3], hi[3];
  int res, comps, iters, min_samples;
  float reg;
};

// Cell of a sample, decided in FP32: floor((x - lo) / (hi - lo) * res) per
// axis, clamped to the grid; -1 for w <= 0 or non-finite input.
__device__ __forceinline__ int em_cell(const EMDesc& D, const float* r) {
  if (!(r[5] > 0.0f) || !isfinite(r[3]) || !isfinite(r[4]) || !isfinite(r[5])) return -1;
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float f = (r[a] - D.lo[a]) / (D.hi[a] - D.lo[a]) * (float)D.res;
    if (!(f == f)) return -1;
    int k = (int)floorf(f);
    idx[a] = min(max(k, 0), D.res - 1);
  }
  return (idx[2] * D.res + idx[1]) * D.res + idx[0];
}

__global__ void k_em_zero(int* a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ void k_em_hist(const float* samples, int M, EMDesc D, int* cell_of, int* count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int c = em_cell(D, samples + 8 * (size_t)i);
  cell_of[i] = c;
  if (c >= 0) atomicAdd(&count[c], 1);
}

// Exclusive scan of the per-cell counts by one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_em_scan(const int* count, int cells, int* offset, int* cursor) {
  __shared__ int part[1024];
  int t = threadIdx.x;
  int per = (cells + 1023) / 1024;
  int lo = t * per, hi = min(cells, lo + per);
  int acc = 0;
  for (int i = lo; i < hi; ++i) acc += count[i];
  part[t] = acc;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int base = part[t] - acc;
  for (int i = lo; i < hi; ++i) {
    offset[i] = base;
    cursor[i] = 0;
    base += count[i];
  }
  if (t == 1023) offset[cells] = part[1023];
}

__global__ void k_em_scatter(int M, const int* cell_of, const int* offset, int* cursor, int* order) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int c = cell_of[i];
  if (c >= 0) order[offset[c] + atomicAdd(&cursor[c], 1)] = i;
}

// Wavefront-scope barrier for the per-wave LDS slices of k_em_cells (waves of
// one workgroup work on different cells and may leave early).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Input order within each cell: the scatter above leaves a cell's sample
// indices in atomic order, which would make the EM sums depend on the run.
// One wavefront per cell puts each index at its rank (the number of smaller
// indices of the cell), writing the sorted order to a second array.
__global__ void __launch_bounds__(256) k_em_sort(const int* offset, const int* order, int cells, int* sorted) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cell = blockIdx.x * 4 + wave;
  if (cell >= cells) return;
  const int beg = offset[cell], m = offset[cell + 1] - beg;
  for (int k = lane; k < m; k += 64) {
    const int idx = order[beg + k];
    int rank = 0;
    for (int q = 0; q < m; ++q) rank += order[beg + q] < idx;
    sorted[beg + rank] = idx;
  }
}

// One wavefront per cell, the cell's sample indices in input order.  The
// initial means are the samples of rank floor((j + 1/2) m / K).  Then
// em_iters iterations of
//   E: r_ij = pi_j N(x_i; mu_j, S_j) / sum_k ...
//   M: N_j = sum w r, mu_j = sum w r x / N_j,
//      S_j = sum w r (x - mu_j)(x - mu_j)^T / N_j + reg I
// with the second moments accumulated about the previous means m_j and
// shifted exactly: sum w r (x - mu)(x - mu)^T = S'_j - N_j (mu - m)(mu - m)^T.
__global__ void __launch_bounds__(256) k_em_cells(const float* samples, EMDesc D, const int* offset,
                                                  const int* order, int cells, int* valid, float* pi, float* mu,
                                                  float* cov, float* chol, int* count_out) {
  __shared__ float par[4][8][6];  // per wave: pi, mux, muy, sxx, sxy, syy
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cell = blockIdx.x * 4 + wave;
  if (cell >= cells) return;
  const int K = D.comps;
  const int beg = offset[cell], m = offset[cell + 1] - beg;
  float (*P)[6] = par[wave];
  if (lane == 0) count_out[cell] = m;
  bool ok = m >= D.min_samples;
  // weighted mean and covariance of the cell (two passes)
  float W = 0.f, sx = 0.f, sy = 0.f;
  if (ok) {
    for (int k = lane; k < m; k += 64) {
      const float* r = samples + 8 * (size_t)order[beg + k];
      W += r[5]; sx += r[5] * r[3]; sy += r[5] * r[4];
    }
    W = wave_sum(W); sx = wave_sum(sx); sy = wave_sum(sy);
    ok = W > 0.0f;
  }
  if (!ok) {
    if (lane < K) {
      size_t q = (size_t)cell * K + lane;
      pi[q] = 0.f; mu[2 * q] = 0.f; mu[2 * q + 1] = 0.f;
      cov[3 * q] = 1.f; cov[3 * q + 1] = 0.f; cov[3 * q + 2] = 1.f;
      chol[3 * q] = 1.f; chol[3 * q + 1] = 0.f; chol[3 * q + 2] = 1.f;
    }
    if (lane == 0) valid[cell] = 0;
    return;
  }
  float mx = sx / W, my = sy / W;
  float cxx = 0.f, cxy = 0.f, cyy = 0.f;
  for (int k = lane; k < m; k += 64) {
    const float* r = samples + 8 * (size_t)order[beg + k];
    float dx = r[3] - mx, dy = r[4] - my;
    cxx += r[5] * dx * dx; cxy += r[5] * dx * dy; cyy += r[5] * dy * dy;
  }
  cxx = wave_sum(cxx) / W + D.reg; cxy = wave_sum(cxy) / W; cyy = wave_sum(cyy) / W + D.reg;
  // initial means by rank in input order
  if (lane < K) {
    const float* r = samples + 8 * (size_t)order[beg + (2 * lane + 1) * m / (2 * K)];
    P[lane][1] = r[3];
    P[lane][2] = r[4];
    P[lane][0] = 1.0f / K;
    P[lane][3] = cxx; P[lane][4] = cxy; P[lane][5] = cyy;
  }
  wave_sync();
  for (int it = 0; it < D.iters; ++it) {
    float acc[8][6];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[j][q] = 0.f;
    float cpi[8], cmx[8], cmy[8], ia[8], ib[8], ic[8], lnorm[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      cpi[j] = j < K ? P[j][0] : 0.f;
      cmx[j] = P[j][1]; cmy[j] = P[j][2];
      float a = P[j][3], b = P[j][4], c = P[j][5];
      float det = a * c - b * b;
      ia[j] = c / det; ib[j] = -b / det; ic[j] = a / det;
      lnorm[j] = cpi[j] > 0.f ? logf(cpi[j]) - 0.5f * logf(det) : -INFINITY;
    }
    for (int k = lane; k < m; k += 64) {
      const float* r = samples + 8 * (size_t)order[beg + k];
      float x = r[3], y = r[4], w = r[5];
      float lp[8], best = -INFINITY;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float dx = x - cmx[j], dy = y - cmy[j];
        float qd = ia[j] * dx * dx + 2.f * ib[j] * dx * dy + ic[j] * dy * dy;
        lp[j] = cpi[j] > 0.f ? lnorm[j] - 0.5f * qd : -INFINITY;
        best = fmaxf(best, lp[j]);
      }
      float z = 0.f;
#pragma unroll
      for (int j = 0; j < 8; ++j) { lp[j] = cpi[j] > 0.f ? expf(lp[j] - best) : 0.f; z += lp[j]; }
      float iz = w / z;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float rw = lp[j] * iz;
        float dx = x - cmx[j], dy = y - cmy[j];
        acc[j][0] += rw; acc[j][1] += rw * dx; acc[j][2] += rw * dy;
        acc[j][3] += rw * dx * dx; acc[j][4] += rw * dx * dy; acc[j][5] += rw * dy * dy;
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[j][q] = wave_sum(acc[j][q]);
    wave_sync();
    if (lane < K) {
      int j = lane;
      float Nj = acc[j][0];
      if (cpi[j] > 0.f && Nj > 1e-8f * W) {
        float ux = acc[j][1] / Nj, uy = acc[j][2] / Nj;  // mean shift from the previous mean
        P[j][0] = Nj / W;
        P[j][1] = cmx[j] + ux;
        P[j][2] = cmy[j] + uy;
        P[j][3] = acc[j][3] / Nj - ux * ux + D.reg;
        P[j][4] = acc[j][4] / Nj - ux * uy;
        P[j][5] = acc[j][5] / Nj - uy * uy + D.reg;
      } else {
        P[j][0] = 0.f;
      }
    }
    wave_sync();
  }
  if (lane < K) {
    size_t q = (size_t)cell * K + lane;
    pi[q] = P[lane][0];
    mu[2 * q] = P[lane][1]; mu[2 * q + 1] = P[lane][2];
    float a = P[lane][3], b = P[lane][4], c = P[lane][5];
    cov[3 * q] = a; cov[3 * q + 1] = b; cov[3 * q + 2] = c;
    float l00 = sqrtf(fmaxf(a, 0.f));
    float l10 = l00 > 0.f ? b / l00 : 0.f;
    float l11 = sqrtf(fmaxf(c - l10 * l10, 0.f));
    chol[3 * q] = l00; chol[3 * q + 1] = l10; chol[3 * q + 2] = l11;
  }
  if (lane == 0) valid[cell] = 1;
}

extern "C" mpg_status fit_guide(const mpg_scene* s, const float* d_samples, int32_t n_samples, mpg_guide* g,
                                mpg_workspace* ws, void* stream) {
  (void)s;
  if (!g) return fail(MPG_ERR_INVALID_ARG, "fit_guide: NULL guide");
  if (n_samples < 0) return fail(MPG_ERR_INVALID_ARG, "fit_guide: n_samples < 0");
  if (n_samples > 0 && !d_samples) return fail(MPG_ERR_INVALID_ARG, "fit_guide: NULL samples");
  if (!ws || ws->cap < n_samples) return fail(MPG_ERR_INVALID_ARG, "fit_guide: workspace smaller than n_samples");
  if (g->desc.comps > 8) return fail(MPG_ERR_UNSUPPORTED, "fit_guide: at most 8 components");
  hipStream_t st = (hipStream_t)stream;
  const int cells = g->cells;
  EMDesc D;
  for (int a = 0; a < 3; ++a) { D.lo[a] = g->desc.lo[a]; D.hi[a] = g->desc.hi[a]; }
  D.res = g->desc.res; D.comps = g->desc.comps; D.iters = g->desc.em_iters; D.min_samples = g->desc.min_samples;
  D.reg = g->desc.reg;
  // scratch: per-sample cell (aux, then the order sorted within each cell),
  // order (perm), per-cell count (guide count), offsets and cursors
  // (guide-owned scratch)
  int* offset = g->scratch;
  int* cursor = g->scratch + cells + 1;
  hipLaunchKernelGGL(k_em_zero, dim3((cells + 255) / 256), dim3(256), 0, st, g->count, cells);
  HIP_TRY(hipGetLastError());
  if (n_samples > 0) {
    hipLaunchKernelGGL(k_em_hist, dim3((n_samples + 255) / 256), dim3(256), 0, st, d_samples, n_samples, D,
                       ws->aux, g->count);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_em_scan, dim3(1), dim3(1024), 0, st, (const int*)g->count, cells, offset, cursor);
  HIP_TRY(hipGetLastError());
  if (n_samples > 0) {
    hipLaunchKernelGGL(k_em_scatter, dim3((n_samples + 255) / 256), dim3(256), 0, st, n_samples,
                       (const int*)ws->aux, (const int*)offset, cursor, ws->perm);
    HIP_TRY(hipGetLastError());
    // the cell ids in aux are no longer needed: aux takes the sorted order
    hipLaunchKernelGGL(k_em_sort, dim3((cells + 3) / 4), dim3(256), 0, st, (const int*)offset,
                       (const int*)ws->perm, cells, ws->aux);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_em_cells, dim3((cells + 3) / 4), dim3(256), 0, st, d_samples, D, (const int*)offset,
                     (const int*)ws->aux, cells, g->valid, g->pi, g->mu, g->cov, g->chol, g->count);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

// Sub-path samples for the guide (Eq. eq_weight: w = T <1/P> with
// T = kappa G L_o, L_o = 1): {x_D, x, y of x_1, w, 0, 0}; w = 0 unless the
// chain converged.
__global__ void k_make_samples(EpView E, const float* pos, const int8_t* status, const float* G, const float* kappa,
                               const float* inv_prob, float* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E.N) return;
  const size_t NN = E.N;
  bool ok = status[c] == ST_CONVERGED;
  float* r = out + 8 * (size_t)c;
  r[0] = E.xD[c];
  r[1] = E.xD[NN + c];
  r[2] = E.xD[2 * NN + c];
  r[3] = pos[(0 * KMAX) * NN + c];
  r[4] = pos[(1 * KMAX) * NN + c];
  r[5] = ok ? kappa[c] * G[c] * inv_prob[c] : 0.0f;
  r[6] = 0.0f;
  r[7] = 0.0f;
}

extern "C" mpg_status make_guide_samples(const mpg_endpoints* ep, const mpg_chains* chains, const int8_t* d_status,
                                         const float* d_G, const float* d_kappa, const float* d_inv_prob,
                                         float* d_samples, void* stream) {
  EpView E;
  mpg_status st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!chains || !chains->d_pos || !d_status || !d_G || !d_kappa || !d_inv_prob || !d_samples)
    return fail(MPG_ERR_INVALID_ARG, "make_guide_samples: NULL argument");
  hipLaunchKernelGGL(k_make_samples, dim3((E.N + 255) / 256), dim3(256), 0, (hipStream_t)stream, E, chains->d_pos,
                     d_status, d_G, d_kappa, d_inv_prob, d_samples);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}
