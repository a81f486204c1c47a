// Per-chain adjoint routine shared by the plain and persistent adjoint
// kernels (mpg_adjoint_plain.hip, mpg_adjoint.hip).
#pragma once
#include "mpg_internal.h"

// Implicit-function-theorem adjoint of converged chains (continuity of the
// specular manifold, Sec. 5.2): the converged local coordinates y* satisfy
// C(y*, p) = 0 for the parameters p = (x_D, x_L, theta), so for a loss
//   l = sum_i r_i . x_i + g G
// the total derivative is
//   dl/dp = dl/dp|_y - mu^T dC/dp,   J^T mu = E^T r + g dG/dy,
// with E_i = [e1 e2] of vertex i.  J^T is block tridiagonal (transposed
// blocks of the walk's Jacobian) and is solved by block Thomas.  G is built
// from J^-1 (the walk's IFT for d x_1 / d x_L), so dG/dy and dG/dp need
// second derivatives of C: they come from forward-mode dual numbers through
// the same templated sweep, one direction at a time.  Height-field
// parameters move triangle vertices and normals at fixed barycentrics.

struct AdjIO {
  const int32_t* prim;
  const float* pos;
  const int8_t* status;
  const float* grad_pos;  // [3][K][N] or NULL
  const float* grad_G;    // [N] or NULL
  float* grad_xD;         // [3][N]
  float* grad_xL;         // [3][N]
  float* grad_theta;      // [P], accumulated
  const DevHF* hf;
  int n_hf, n_params;
};

// C and G along one dual direction (positions / endpoints carry the tangent).
// Inlined at every call site (a call keeps its arrays in a stack frame in
// scratch memory): measured 37% faster in the persistent adjoint kernels.
template <int N>
__device__ __forceinline__ void dual_eval(const DevScene& S, const ThetaDir* td, vec3<dfloat> xD, f3 nDf,
                                          vec3<dfloat> xL, int type, const int* prim, const vec3<dfloat>* x,
                                          dfloat (*C)[2], dfloat& G) {
  Stack none{nullptr, 0};
  Sweep<dfloat, N> W;
  sweep<dfloat, N, true, Stack, false>(S, xD, xL, type, prim, x, W, none, td);
#pragma unroll
  for (int i = 0; i < N; ++i) { C[i][0] = W.Cv[i][0]; C[i][1] = W.Cv[i][1]; }
  vec3<dfloat> wl = normalize(x[N - 1] - xL), t1, t2;
  onb(wl, t1, t2);
  dfloat B[4] = {dot(W.gso_last, t1), dot(W.gso_last, t2), dot(W.gto_last, t1), dot(W.gto_last, t2)};
  dfloat X[4];
  mul22(W.Dinv_last, B, X);
  X[0] = -X[0]; X[1] = -X[1]; X[2] = -X[2]; X[3] = -X[3];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) {
    dfloat Y[4];
    mul22(W.G[i], X, Y);
    X[0] = -Y[0]; X[1] = -Y[1]; X[2] = -Y[2]; X[3] = -Y[3];
  }
  Geo<dfloat> g0 = load_geo<dfloat, false>(S, prim[0], x[0], td);
  vec3<dfloat> dx0 = g0.e1 * X[0] + g0.e2 * X[2];
  vec3<dfloat> dx1 = g0.e1 * X[1] + g0.e2 * X[3];
  vec3<dfloat> dd = x[0] - xD;
  dfloat il = rsq(dot(dd, dd));
  vec3<dfloat> w = dd * il;
  vec3<dfloat> dw0 = (dx0 - w * dot(w, dx0)) * il, dw1 = (dx1 - w * dot(w, dx1)) * il;
  vec3<dfloat> nD = cvt<dfloat>(nDf);
  G = fabs(dot(nD, w)) * fabs(dot(w, cross(dw0, dw1)));
}

__device__ __forceinline__ vec3<dfloat> dual3(f3 v, f3 d) { return {dfloat(v.x, d.x), dfloat(v.y, d.y), dfloat(v.z, d.z)}; }

template <int N>
__device__ __forceinline__ void adjoint_one(const DevScene& S, const WalkParams& P, const EpView& E, const AdjIO& io,
                                            int c, float* theta_acc) {
  const size_t NN = E.N;
  int prim[N];
  f3 x[N], r[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    prim[i] = io.prim[i * NN + c];
    x[i] = {io.pos[(0 * KMAX + i) * NN + c], io.pos[(1 * KMAX + i) * NN + c], io.pos[(2 * KMAX + i) * NN + c]};
    r[i] = io.grad_pos ? f3{io.grad_pos[(0 * KMAX + i) * NN + c], io.grad_pos[(1 * KMAX + i) * NN + c],
                            io.grad_pos[(2 * KMAX + i) * NN + c]}
                       : f3{0.f, 0.f, 0.f};
  }
  const float g = io.grad_G ? io.grad_G[c] : 0.0f;
  const f3 xD = ld_pt(E.xD, E.N, c), xL = ld_pt(E.xL, E.N, c), nD = ld_pt(E.nD, E.N, c);
  const int type = E.type[c];
  const f3 zero = {0.f, 0.f, 0.f};
  // primal Jacobian blocks and frames
  float Lb[N][4], Db[N][4], Ub[N][4];
  f3 e1[N], e2[N];
  {
    Geo<float> gc = load_geo<float, true>(S, prim[0], x[0]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Geo<float> gn = i + 1 < N ? load_geo<float, true>(S, prim[i + 1 < N ? i + 1 : 0], x[i + 1 < N ? i + 1 : 0]) : gc;
      f3 xp = i == 0 ? xD : x[i > 0 ? i - 1 : 0];
      f3 xq = i == N - 1 ? xL : x[i + 1 < N ? i + 1 : 0];
      float ea, eb;
      vertex_etas(gc, (type >> i) & 1, xp, ea, eb);
      VJ<float> v;
      vertex_cj<float, true>(gc, xp, xq, ea, eb, i > 0 ? e1[i > 0 ? i - 1 : 0] : gc.e1,
                             i > 0 ? e2[i > 0 ? i - 1 : 0] : gc.e2, gn.e1, gn.e2, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) { Lb[i][q] = v.L[q]; Db[i][q] = v.D[q]; Ub[i][q] = v.U[q]; }
      e1[i] = gc.e1;
      e2[i] = gc.e2;
      gc = gn;
    }
  }
  // right-hand side: E^T r + g dG/dy
  float b[N][2];
  vec3<dfloat> dD = dual3(xD, zero), dL = dual3(xL, zero);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    b[i][0] = dot(e1[i], r[i]);
    b[i][1] = dot(e2[i], r[i]);
  }
  if (g != 0.0f) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        vec3<dfloat> xd[N];
#pragma unroll
        for (int j = 0; j < N; ++j) xd[j] = dual3(x[j], j == i ? (k == 0 ? e1[i] : e2[i]) : zero);
        dfloat Cd[N][2], Gd;
        dual_eval<N>(S, nullptr, dD, nD, dL, type, prim, xd, Cd, Gd);
        b[i][k] += g * Gd.d;
      }
    }
  }
  // J^T mu = b by block Thomas on the transpose: diagonal D_i^T, super
  // (i, i+1) = L_{i+1}^T, sub (i, i-1) = U_{i-1}^T
  float Gt[N][4], gt[N][2];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    float Dt[4] = {Db[i][0], Db[i][2], Db[i][1], Db[i][3]};
    float rr0 = b[i][0], rr1 = b[i][1];
    if (i > 0) {
      float Ut[4] = {Ub[i - 1][0], Ub[i - 1][2], Ub[i - 1][1], Ub[i - 1][3]};  // U_{i-1}^T
      float M[4];
      mul22(Ut, Gt[i > 0 ? i - 1 : 0], M);
      Dt[0] -= M[0]; Dt[1] -= M[1]; Dt[2] -= M[2]; Dt[3] -= M[3];
      rr0 -= Ut[0] * gt[i - 1][0] + Ut[1] * gt[i - 1][1];
      rr1 -= Ut[2] * gt[i - 1][0] + Ut[3] * gt[i - 1][1];
    }
    float I[4];
    inv2(Dt, I);
    if (i < N - 1) {
      float Lt[4] = {Lb[i + 1 < N ? i + 1 : 0][0], Lb[i + 1 < N ? i + 1 : 0][2], Lb[i + 1 < N ? i + 1 : 0][1],
                     Lb[i + 1 < N ? i + 1 : 0][3]};  // L_{i+1}^T
      mul22(I, Lt, Gt[i]);
    }
    gt[i][0] = I[0] * rr0 + I[1] * rr1;
    gt[i][1] = I[2] * rr0 + I[3] * rr1;
  }
  float mu[N][2];
  mu[N - 1][0] = gt[N - 1][0];
  mu[N - 1][1] = gt[N - 1][1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) {
    mu[i][0] = gt[i][0] - (Gt[i][0] * mu[i + 1][0] + Gt[i][1] * mu[i + 1][1]);
    mu[i][1] = gt[i][1] - (Gt[i][2] * mu[i + 1][0] + Gt[i][3] * mu[i + 1][1]);
  }
  // parameter directions: dl/dp = sum r.dx/dp|_y + g dG/dp|_y - mu . dC/dp|_y
  auto contrib = [&](const ThetaDir* td, vec3<dfloat> xDd, vec3<dfloat> xLd, const vec3<dfloat>* xd) -> float {
    dfloat Cd[N][2], Gd;
    dual_eval<N>(S, td, xDd, nD, xLd, type, prim, xd, Cd, Gd);
    float acc = g * Gd.d;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      acc += r[i].x * xd[i].x.d + r[i].y * xd[i].y.d + r[i].z * xd[i].z.d;
      acc -= mu[i][0] * Cd[i][0].d + mu[i][1] * Cd[i][1].d;
    }
    return acc;
  };
  vec3<dfloat> xfix[N];
#pragma unroll
  for (int j = 0; j < N; ++j) xfix[j] = dual3(x[j], zero);
  float gxD[3], gxL[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    f3 u = {a == 0 ? 1.f : 0.f, a == 1 ? 1.f : 0.f, a == 2 ? 1.f : 0.f};
    gxD[a] = contrib(nullptr, dual3(xD, u), dL, xfix);
    gxL[a] = contrib(nullptr, dD, dual3(xL, u), xfix);
  }
  for (int a = 0; a < 3; ++a) {
    io.grad_xD[a * NN + c] = gxD[a];
    io.grad_xL[a * NN + c] = gxL[a];
  }
  // height-field parameters of the fields this chain touches
  for (int h = 0; h < io.n_hf; ++h) {
    const DevHF& H = io.hf[h];
    bool touched = false;
#pragma unroll
    for (int i = 0; i < N; ++i) touched = touched || (prim[i] >= H.first_tri && prim[i] < H.first_tri + H.n_tris);
    if (!touched) continue;
    for (int s = 0; s < H.n_sines; ++s) {
      for (int which = 0; which < 2; ++which) {
        ThetaDir td{&H, s, which};
        vec3<dfloat> xd[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          f3 dx = zero;
          if (prim[i] >= H.first_tri && prim[i] < H.first_tri + H.n_tris) {
            // the vertex rides on its triangle at fixed barycentrics
            int4 id = S.tri_idx[prim[i]];
            f3 P0 = ld3(S.vpos[id.x]), P1 = ld3(S.vpos[id.y]), P2 = ld3(S.vpos[id.z]);
            f3 E1 = P1 - P0, E2 = P2 - P0, q = x[i] - P0;
            float d11 = dot(E1, E1), d12 = dot(E1, E2), d22 = dot(E2, E2), q1 = dot(q, E1), q2 = dot(q, E2);
            float den = d11 * d22 - d12 * d12;
            float b1 = (d22 * q1 - d12 * q2) / den, b2 = (d11 * q2 - d12 * q1) / den, b0 = 1.0f - b1 - b2;
            int vid[3] = {id.x, id.y, id.z};
            float bw[3] = {b0, b1, b2};
            for (int k = 0; k < 3; ++k) {
              float4 pv = S.vpos[vid[k]], nv = S.vnrm[vid[k]];
              f3 dP, dN;
              hf_vertex_deriv(H, s, which, pv.x, pv.y, ld3(nv), dP, dN);
              dx = dx + dP * bw[k];
            }
          }
          xd[i] = dual3(x[i], dx);
        }
        float v = contrib(&td, dD, dL, xd);
        atomicAdd(&theta_acc[H.param_base + 2 * s + which], v);
      }
    }
  }
}

// plain form: one thread per chain, any length up to max_len
mpg_status launch_adjoint_plain(const mpg_scene* s, const WalkParams& P, const EpView& E, const AdjIO& io, int max_len,
                                hipStream_t stream);
