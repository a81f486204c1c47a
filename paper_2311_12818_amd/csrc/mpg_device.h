// Device code of the batched manifold-walk path for CDNA4 (gfx950, wave64).
//
// Layout of the work: one chain per lane.  A chain of length N (1..8) keeps
// its vertices, the Newton step and the block-tridiagonal elimination state
// in registers (every loop over vertices is unrolled for the compile-time N),
// BVH traversal stacks live in LDS (one column of `depth` ints per lane,
// lane-interleaved so the 64 lanes of a wave hit 64 distinct banks), and the
// scene (BVH nodes, triangles, vertex normals) is read through L2/MALL.
// Nothing here is a dense contraction, so there is no MFMA: the path is bound
// by FP32 VALU throughput and by the latency of dependent BVH node fetches.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

constexpr int KMAX = 8;
constexpr int PRIM_NONE = (int)0x80000000;
enum : int { ST_CONVERGED = 0, ST_MAX_ITER = 1, ST_SINGULAR = 2, ST_SIDE_INVALID = 3, ST_OCCLUDED = 4,
             ST_SEED_INVALID = 5, ST_FP64_REJECT = 6, ST_BAD_INPUT = 7,
             ST_NEEDS_FP64 = 8 /* converged, awaiting the FP64 pass */,
             ST_PENDING = 9 /* internal: converged in the walk kernel, awaiting the finish pass */ };
enum : int { MAT_MIRROR = 0, MAT_DIELECTRIC = 1 };
constexpr int P0_DIRECTION = -2;

// ---------------------------------------------------------------------------
// small vectors (float and double)
// ---------------------------------------------------------------------------
template <typename T>
struct vec3 {
  T x, y, z;
};
template <typename T> __device__ __forceinline__ vec3<T> mk(T a, T b, T c) { return vec3<T>{a, b, c}; }
template <typename T> __device__ __forceinline__ vec3<T> operator+(vec3<T> a, vec3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T> __device__ __forceinline__ vec3<T> operator-(vec3<T> a, vec3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T> __device__ __forceinline__ vec3<T> operator-(vec3<T> a) { return {-a.x, -a.y, -a.z}; }
template <typename T> __device__ __forceinline__ vec3<T> operator*(vec3<T> a, T s) { return {a.x * s, a.y * s, a.z * s}; }
template <typename T> __device__ __forceinline__ vec3<T> operator*(T s, vec3<T> a) { return {a.x * s, a.y * s, a.z * s}; }
template <typename T> __device__ __forceinline__ T dot(vec3<T> a, vec3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T> __device__ __forceinline__ vec3<T> cross(vec3<T> a, vec3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float rsq(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqr_t(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqr_t(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T norm(vec3<T> a) { return sqr_t(dot(a, a)); }
template <typename T> __device__ __forceinline__ vec3<T> normalize(vec3<T> a) { return a * rsq(dot(a, a)); }
template <typename T> __device__ __forceinline__ vec3<T> fmav(vec3<T> a, T s, vec3<T> b) {  // a*s + b
  return {fma(a.x, s, b.x), fma(a.y, s, b.y), fma(a.z, s, b.z)};
}
template <typename T, typename U> __device__ __forceinline__ vec3<T> cvt(vec3<U> a) { return {(T)a.x, (T)a.y, (T)a.z}; }
typedef vec3<float> f3;
typedef vec3<double> d3;
__device__ __forceinline__ f3 ld3(const float4& v) { return {v.x, v.y, v.z}; }

// Forward-mode dual number (value, one directional derivative) for the
// adjoint: the same templated geometry / constraint / elimination code runs
// on it to differentiate J and G along one direction at a time.
struct dfloat {
  float v, d;
  __device__ __forceinline__ dfloat() : v(0.f), d(0.f) {}
  __device__ __forceinline__ dfloat(float x) : v(x), d(0.f) {}  // NOLINT
  __device__ __forceinline__ dfloat(float x, float y) : v(x), d(y) {}
};
__device__ __forceinline__ dfloat operator+(dfloat a, dfloat b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dfloat operator-(dfloat a, dfloat b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dfloat operator-(dfloat a) { return {-a.v, -a.d}; }
__device__ __forceinline__ dfloat operator*(dfloat a, dfloat b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ dfloat operator/(dfloat a, dfloat b) {
  float q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ dfloat& operator+=(dfloat& a, dfloat b) { a = a + b; return a; }
__device__ __forceinline__ dfloat& operator-=(dfloat& a, dfloat b) { a = a - b; return a; }
__device__ __forceinline__ dfloat& operator*=(dfloat& a, dfloat b) { a = a * b; return a; }
__device__ __forceinline__ bool operator<(dfloat a, dfloat b) { return a.v < b.v; }
__device__ __forceinline__ bool operator>(dfloat a, dfloat b) { return a.v > b.v; }
__device__ __forceinline__ bool operator<=(dfloat a, dfloat b) { return a.v <= b.v; }
__device__ __forceinline__ bool operator>=(dfloat a, dfloat b) { return a.v >= b.v; }
__device__ __forceinline__ dfloat rsq(dfloat a) {
  float r = 1.0f / sqrtf(a.v);
  return {r, -0.5f * a.d * r * r * r};
}
__device__ __forceinline__ dfloat sqr_t(dfloat a) {
  float r = sqrtf(a.v);
  return {r, 0.5f * a.d / r};
}
// float / double forms (the dual overloads below would otherwise hide them)
__device__ __forceinline__ float fabs(float a) { return ::fabsf(a); }
__device__ __forceinline__ double fabs(double a) { return ::fabs(a); }
__device__ __forceinline__ float fmax(float a, float b) { return ::fmaxf(a, b); }
__device__ __forceinline__ double fmax(double a, double b) { return ::fmax(a, b); }
__device__ __forceinline__ float fmin(float a, float b) { return ::fminf(a, b); }
__device__ __forceinline__ double fmin(double a, double b) { return ::fmin(a, b); }
__device__ __forceinline__ float copysign(float a, float b) { return ::copysignf(a, b); }
__device__ __forceinline__ double copysign(double a, double b) { return ::copysign(a, b); }
__device__ __forceinline__ float fma(float a, float b, float c) { return ::fmaf(a, b, c); }
__device__ __forceinline__ double fma(double a, double b, double c) { return ::fma(a, b, c); }
__device__ __forceinline__ dfloat fabs(dfloat a) { return a.v < 0.f ? -a : a; }
__device__ __forceinline__ dfloat fmax(dfloat a, dfloat b) { return a.v >= b.v ? a : b; }
__device__ __forceinline__ dfloat fmin(dfloat a, dfloat b) { return a.v <= b.v ? a : b; }
__device__ __forceinline__ dfloat copysign(dfloat a, dfloat b) { return {copysignf(a.v, b.v), 0.f}; }
__device__ __forceinline__ dfloat fma(dfloat a, dfloat b, dfloat c) { return a * b + c; }
template <typename T> struct is_dual { static constexpr bool value = false; };
template <> struct is_dual<dfloat> { static constexpr bool value = true; };

// Orthonormal basis about a unit vector: Duff et al., "Building an
// orthonormal basis, revisited", JCGT 6(1), 2017 (branchless form).
template <typename T>
__device__ __forceinline__ void onb(vec3<T> n, vec3<T>& b1, vec3<T>& b2) {
  T sign = copysign((T)1, n.z);
  T a = (T)-1 / (sign + n.z);
  T b = n.x * n.y * a;
  b1 = {(T)1 + sign * n.x * n.x * a, sign * b, -sign * n.x};
  b2 = {b, sign + n.y * n.y * a, -n.y};
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC 2011) and splitmix64 (Steele et al. 2014)
// ---------------------------------------------------------------------------
struct U8 {
  float u[8];
};
__device__ __forceinline__ U8 philox_uniforms(uint64_t key0, uint64_t c0, uint64_t c1, uint64_t c2) {
  uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = 0, k0 = key0, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B97F4A7C15ULL;
      k1 += 0xBB67AE8584CAA73BULL;
    }
    uint64_t h0 = __umul64hi(0xD2E7470EE14C6C93ULL, x0), l0 = 0xD2E7470EE14C6C93ULL * x0;
    uint64_t h1 = __umul64hi(0xCA5A826395121157ULL, x2), l1 = 0xCA5A826395121157ULL * x2;
    uint64_t n0 = h1 ^ x1 ^ k0, n2 = h0 ^ x3 ^ k1;
    x0 = n0; x1 = l1; x2 = n2; x3 = l0;
  }
  uint64_t w[4] = {x0, x1, x2, x3};
  U8 U;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uint32_t half = (j & 1) ? (uint32_t)(w[j >> 1] & 0xffffffffULL) : (uint32_t)(w[j >> 1] >> 32);
    U.u[j] = (float)(half >> 8) * (1.0f / 16777216.0f);
  }
  return U;
}
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// device scene
// ---------------------------------------------------------------------------
struct DevScene {
  const float4* nodes;      // 8 x float4 per 4-wide node: child boxes (SoA) + int4 child references + pad
  const float4* tri_v;      // 3 x float4 per triangle in BVH order; v0.w = primitive id (int bits)
  const float4* tri_geo;    // 6 x float4 per triangle in primitive order: P0, P1, P2, N0, N1, N2 (unit);
                            // P0.w = object, P1.w = material (int bits), P2.w = index of refraction
  const int4* tri_idx;      // [n_tris] vertex ids (i0, i1, i2) and object
  const float4* vpos;       // [n_verts]
  const float4* vnrm;       // [n_verts]
  const int2* obj_info;     // [n_objects] (material, ior as float bits)
  const float4* spheres;    // [n_spheres] centre, radius
  const int* sphere_obj;    // [n_spheres]
  const float2* cdf;        // area prefix sums as unevaluated FP32 pairs (hi + lo), one run per object
                            // and one over all objects
  const int* cdf_prim;
  const int2* cdf_range;    // [n_objects + 1] (start, count)
  const float4* obj_bounds; // [n_objects] (lo_x, lo_y, hi_x, hi_y)
  const float* zmax;        // top of the geometry (device word, follows surface-parameter updates)
  int n_tris, n_spheres, n_objects, n_nodes;
};

struct DevGuide {
  const int* valid;    // [cells]
  const float* pi;     // [cells][comps]
  const float* mu;     // [cells][comps][2]
  const float* chol;   // [cells][comps][3]
  float lo[3], hi[3];
  int res, comps, target_obj;
};

// Height field of the scene (the adjoint's surface parameters): triangles
// [first_tri, first_tri + n_tris), vertices [first_vert, first_vert + n_verts),
// parameters [param_base, param_base + 2 n_sines): (amplitude, phase) per sine.
struct DevHF {
  int first_vert, n_verts, first_tri, n_tris, n_sines, param_base;
  float amp[8], freq[8], psi[8], phase[8];
};
// One parameter direction of the adjoint: sine s of height field hf, which =
// 0 for its amplitude, 1 for its phase; hf < 0 for none.
struct ThetaDir {
  const DevHF* hf;
  int s, which;
};

struct WalkParams {
  int max_iter;
  float tol_step2;     // (tol_vertex * L)^2
  float tol_residual;
  float tmin;          // tmin_rel * L
  float match2;        // (match_rel * L)^2
  float fp64_cond;
  float graze_cos;     // chains with an incident / outgoing cosine below this take the FP64 pass
  float cone_cos;
  int depth;           // LDS stack entries per lane
};

__device__ __forceinline__ int prim_obj(const DevScene& S, int prim) {
  return prim >= 0 ? __float_as_int(S.tri_geo[6 * (size_t)prim].w) : S.sphere_obj[-1 - prim];
}
__device__ __forceinline__ int prim_material(const DevScene& S, int prim) {
  return prim >= 0 ? __float_as_int(S.tri_geo[6 * (size_t)prim + 1].w) : S.obj_info[S.sphere_obj[-1 - prim]].x;
}

// ---------------------------------------------------------------------------
// ray casting: r(x, w) of Sec. 5.3 -- first hit over the specular surfaces
// ---------------------------------------------------------------------------
struct Hit {
  float t;
  int prim;
};

// Lane-private traversal stack in LDS: entry k of lane l at base[k * 64].
// The work tallies are empty here; CountStack below carries real counters
// for the untimed counting launch (every device routine that does counted
// work is templated on the stack type, so the timed kernels carry none).
struct Stack {
  int* base;
  int depth;
  __device__ __forceinline__ void box(int) {}
  __device__ __forceinline__ void tri() {}
  __device__ __forceinline__ void sph() {}
  __device__ __forceinline__ void ray() {}
  __device__ __forceinline__ void vc() {}
  __device__ __forceinline__ void vj() {}
  __device__ __forceinline__ void vj64() {}
};
struct CountStack {
  int* base;
  int depth;
  uint32_t nbox, ntri, nsph, nray, nvc, nvj, nvj64;
  __device__ __forceinline__ void box(int k) { nbox += k; }
  __device__ __forceinline__ void tri() { ++ntri; }
  __device__ __forceinline__ void sph() { ++nsph; }
  __device__ __forceinline__ void ray() { ++nray; }
  __device__ __forceinline__ void vc() { ++nvc; }
  __device__ __forceinline__ void vj() { ++nvj; }
  __device__ __forceinline__ void vj64() { ++nvj64; }
};

__device__ __forceinline__ void take(Hit& h, int prim, float t) {
  if (t < h.t || (t == h.t && prim < h.prim)) {
    h.t = t;
    h.prim = prim;
  }
}

__device__ __forceinline__ float comp(f3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// Returns false only on stack overflow (the library sizes stacks so that it
// cannot happen).  h.prim == PRIM_NONE when nothing was hit.
// Watertight ray/triangle test on the sheared frame (rx, ry, rz) of the ray:
// the hit distance, or +infinity.
__device__ __forceinline__ float tri_test(f3 rx, f3 ry, f3 rz, f3 o, float4 v0, float4 v1, float4 v2) {
  f3 A = ld3(v0) - o, B = ld3(v1) - o, C = ld3(v2) - o;
  float Ax = dot(rx, A), Ay = dot(ry, A), Bx = dot(rx, B), By = dot(ry, B), Cx = dot(rx, C), Cy = dot(ry, C);
  float U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
  if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return INFINITY;
  float det = U + V + W;
  if (det == 0.f) return INFINITY;
  float T = U * dot(rz, A) + V * dot(rz, B) + W * dot(rz, C);
  return T / det;
}

// First hit of the ray o + t d, t in (tmin, tmax), over the specular
// surfaces, skipping primitive excl.  cand (a triangle id, optional) is tested
// before the traversal: its hit, when there is one, bounds the traversal,
// which then only looks for closer hits; ties go to the smaller primitive id
// either way, so the result does not depend on cand.
template <class STK>
__device__ bool trace(const DevScene& S, f3 o, f3 d, int excl, float tmin, Hit& h, STK& stk,
                      float tmax = INFINITY, int cand = PRIM_NONE) {
  h.t = tmax;
  h.prim = PRIM_NONE;
  stk.ray();
  for (int s = 0; s < S.n_spheres; ++s) {
    stk.sph();
    float4 sp = S.spheres[s];
    int prim = -1 - s;
    f3 oc = o - ld3(sp);
    float b = dot(oc, d);
    if (prim == excl) {
      // the ray leaves this sphere: its root at the origin is skipped
      float t = -2.0f * b;
      if (t > tmin) take(h, prim, t);
      continue;
    }
    // discriminant from the closest-approach vector (no b^2 - c cancellation)
    f3 q = oc - d * b;
    float disc = sp.w * sp.w - dot(q, q);
    if (disc < 0.0f) continue;
    float sq = sqrtf(disc);
    float t0 = -b - sq, t1 = -b + sq;
    if (t0 > tmin) take(h, prim, t0);
    else if (t1 > tmin) take(h, prim, t1);
  }
  if (S.n_tris == 0) return true;
  // watertight ray/triangle set-up (Woop, Benthin, Wald, JCGT 2(1), 2013):
  // permute so that the dominant direction axis is z, shear it onto +z.
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  float dz = comp(d, kz);
  if (dz < 0.0f) { int t = kx; kx = ky; ky = t; }
  float Sx = comp(d, kx) / dz, Sy = comp(d, ky) / dz, Sz = 1.0f / dz;
  // shear rows as vectors: X' = rx . v, Y' = ry . v, Z' = rz . v
  f3 ex = {kx == 0 ? 1.f : 0.f, kx == 1 ? 1.f : 0.f, kx == 2 ? 1.f : 0.f};
  f3 ey = {ky == 0 ? 1.f : 0.f, ky == 1 ? 1.f : 0.f, ky == 2 ? 1.f : 0.f};
  f3 ez = {kz == 0 ? 1.f : 0.f, kz == 1 ? 1.f : 0.f, kz == 2 ? 1.f : 0.f};
  f3 rx = ex - ez * Sx, ry = ey - ez * Sy, rz = ez * Sz;
  f3 inv = {1.0f / (fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x)),
            1.0f / (fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y)),
            1.0f / (fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z))};
  f3 oinv = {o.x * inv.x, o.y * inv.y, o.z * inv.z};
  // Byte offsets, within a node, of the near and the far planes of the
  // child boxes along each axis (the low plane is the near one where the
  // direction is positive), fixed once per ray: the slab test then needs no
  // min / max per axis.  With lo <= hi in every box the distances are the
  // ones a min / max of both planes gives, bit for bit.
  const uint32_t onx = inv.x < 0.0f ? 48u : 0u, ony = inv.y < 0.0f ? 64u : 16u, onz = inv.z < 0.0f ? 80u : 32u;
  const uint32_t ofx = 48u - onx, ofy = 80u - ony, ofz = 112u - onz;
  const char* node_bytes = reinterpret_cast<const char*>(S.nodes);
  if (cand >= 0 && cand < S.n_tris && cand != excl) {
    stk.tri();
    const float4* tg = S.tri_geo + 6 * (size_t)cand;
    float t = tri_test(rx, ry, rz, o, tg[0], tg[1], tg[2]);
    if (t > tmin) take(h, cand, t);
  }
  // traversal stack: the top entry lives in a register, the entries below it
  // in the lane's LDS column, so a pop needs no LDS round trip (the reload of
  // the next top is only waited for at the following pop)
  int sp = 0, top = 0;
  int ref = 0;
  bool done = false;
  // Interior nodes and leaves in separate phases (Aila and Laine, HPG 2009,
  // "while-while" with speculative traversal): a lane that reaches a leaf
  // keeps it aside and goes on through interior nodes until every lane of
  // the wavefront holds a leaf, then all test their leaf's triangles
  // together.  The set of leaves tested, and so the hit, is unchanged; the
  // step budget bounds the work of a malformed tree.
  int leaf = 0;
  bool have_leaf = false;
  int budget = 8 * (S.n_nodes + S.n_tris) + 64;
  for (;;) {
    while (!done && (ref >= 0 || !have_leaf)) {
      if (--budget < 0) return false;
      if (ref < 0) {  // a leaf: set it aside, continue with the next entry
        leaf = ref;
        have_leaf = true;
        if (sp == 0) {
          done = true;
          break;
        }
        ref = top;
        if (--sp > 0) top = stk.base[(sp - 1) * 64];
        continue;
      }
      // 4-wide node: slab test of the four child boxes (SoA), then descend
      // into the nearest hit child and push the others, farthest first
      if (ref >= S.n_nodes) return false;
      stk.box(4);
      const uint32_t nb = (uint32_t)ref << 7;
      auto plane = [&](uint32_t off) { return *reinterpret_cast<const float4*>(node_bytes + (nb + off)); };
      const float4 nx = plane(onx), ny = plane(ony), nz = plane(onz), fx = plane(ofx), fy = plane(ofy), fz = plane(ofz);
      const int4 ch = *reinterpret_cast<const int4*>(node_bytes + (nb + 96u));
      float tn[4];
      int cr[4];
      {
        const float nxa[4] = {nx.x, nx.y, nx.z, nx.w}, nya[4] = {ny.x, ny.y, ny.z, ny.w};
        const float nza[4] = {nz.x, nz.y, nz.z, nz.w}, fxa[4] = {fx.x, fx.y, fx.z, fx.w};
        const float fya[4] = {fy.x, fy.y, fy.z, fy.w}, fza[4] = {fz.x, fz.y, fz.z, fz.w};
        const int cha[4] = {ch.x, ch.y, ch.z, ch.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float x0 = fmaf(nxa[k], inv.x, -oinv.x), x1 = fmaf(fxa[k], inv.x, -oinv.x);
          float y0 = fmaf(nya[k], inv.y, -oinv.y), y1 = fmaf(fya[k], inv.y, -oinv.y);
          float z0 = fmaf(nza[k], inv.z, -oinv.z), z1 = fmaf(fza[k], inv.z, -oinv.z);
          float t0 = fmaxf(fmaxf(x0, y0), fmaxf(z0, tmin));
          float t1 = fminf(fminf(x1, y1), fminf(z1, h.t));
          tn[k] = t0 <= t1 ? t0 : INFINITY;
          cr[k] = cha[k];
        }
      }
      // the child references are needed only by a push; without this use
      // (after the slab tests) the compiler issues their load inside the
      // push branch, a second memory round trip per node
      asm volatile("" : : "v"(ch.x), "v"(ch.y), "v"(ch.z), "v"(ch.w), "v"(tn[0]), "v"(tn[1]), "v"(tn[2]), "v"(tn[3]));
      // sort the four entry distances (misses at +infinity last)
#define MPG_CSWAP(a, b)                                                     \
  if (tn[b] < tn[a]) {                                                      \
    float tt = tn[a]; tn[a] = tn[b]; tn[b] = tt;                            \
    int rr = cr[a]; cr[a] = cr[b]; cr[b] = rr;                              \
  }
      MPG_CSWAP(0, 1) MPG_CSWAP(2, 3) MPG_CSWAP(0, 2) MPG_CSWAP(1, 3) MPG_CSWAP(1, 2)
#undef MPG_CSWAP
      const int nh = (tn[0] != INFINITY) + (tn[1] != INFINITY) + (tn[2] != INFINITY) + (tn[3] != INFINITY);
      if (nh == 0) {
        if (sp == 0) {
          done = true;
          break;
        }
        // pop: the entry below the top comes up from the LDS column (read
        // unconditionally; when the stack is now empty the value is unused)
        ref = top;
        --sp;
        top = stk.base[(sp > 0 ? sp - 1 : 0) * 64];
      } else {
        // descend into the nearest hit child, push the other m = nh - 1 hits
        // farthest first.  The pushes' LDS stores are made unconditional:
        // a store a push does not need goes to the first column entry above
        // the new stack (free, and inside the column by the depth check).
        const int m = nh - 1;
        if (sp + m > stk.depth) return false;
        const int spare = sp + m > 0 ? sp + m - 1 : 0;
        stk.base[(m >= 1 && sp > 0 ? sp - 1 : spare) * 64] = top;
        stk.base[(m >= 2 ? sp : spare) * 64] = nh == 4 ? cr[3] : cr[2];
        stk.base[(m >= 3 ? sp + 1 : spare) * 64] = cr[2];
        top = m >= 1 ? cr[1] : top;
        sp += m;
        ref = cr[0];
      }
      // every lane still traversing holds a leaf: test them together
      if (__ballot(!have_leaf) == 0) break;
    }
    if (have_leaf) {
      int start = leaf & 0xFFFFFF;
      int count = (leaf >> 24) & 0x7F;
      if (start + count > S.n_tris) return false;
      // the next triangle's vertices are loaded while this one is tested
      // (the last iteration reloads its own, in bounds), and the excluded
      // primitive is tested too and then dropped, so no load waits on a
      // branch
      const int end = start + count;
      float4 v0, v1, v2;
      if (count > 0) {
        v0 = S.tri_v[3 * (size_t)start];
        v1 = S.tri_v[3 * (size_t)start + 1];
        v2 = S.tri_v[3 * (size_t)start + 2];
      }
#pragma unroll 2
      for (int k = start; k < end; ++k) {
        const float4 a0 = v0, a1 = v1, a2 = v2;
        const size_t kn = 3 * (size_t)(k + 1 < end ? k + 1 : k);
        v0 = S.tri_v[kn];
        v1 = S.tri_v[kn + 1];
        v2 = S.tri_v[kn + 2];
        const int prim = __float_as_int(a0.w);
        const float t = tri_test(rx, ry, rz, o, a0, a1, a2);
        if (prim != excl) {
          stk.tri();
          if (t > tmin) take(h, prim, t);
        }
      }
      have_leaf = false;
    }
    if (done) break;
  }
  return true;
}

// ---------------------------------------------------------------------------
// local geometry of a specular vertex (two degrees of freedom y = (a, b) on
// an orthonormal tangent frame (e1, e2) of its primitive at the current point)
//   triangle: e1 = normalize(P1 - P0), n_g = normalize(E1 x E2), e2 = n_g x e1,
//             shading normal = normalized barycentric blend of vertex normals;
//   sphere:   n = normalize(x - c), (e1, e2) = onb(n), shading normal = n.
// ---------------------------------------------------------------------------
template <typename T>
struct Geo {
  vec3<T> x, e1, e2, ng, ns, dns_a, dns_b;
  T ior;
  int mat;
};

// d/dtheta of a height-field vertex position and unit normal (z = z0 +
// sum a sin(f (cos psi x + sin psi y) + phi), n = normalize(-h_x, -h_y, 1)).
__device__ __forceinline__ void hf_vertex_deriv(const DevHF& h, int s, int which, float x, float y, f3 n, f3& dP,
                                                f3& dN) {
  float hx = 0.f, hy = 0.f;
  for (int k = 0; k < h.n_sines; ++k) {
    float arg = h.freq[k] * (cosf(h.psi[k]) * x + sinf(h.psi[k]) * y) + h.phase[k];
    float c = h.amp[k] * h.freq[k] * cosf(arg);
    hx += c * cosf(h.psi[k]);
    hy += c * sinf(h.psi[k]);
  }
  float arg = h.freq[s] * (cosf(h.psi[s]) * x + sinf(h.psi[s]) * y) + h.phase[s];
  float dz, dfac;  // dz/dtheta and d(h_x, h_y)/dtheta = dfac (cos psi, sin psi)
  if (which == 0) {
    dz = sinf(arg);
    dfac = h.freq[s] * cosf(arg);
  } else {
    dz = h.amp[s] * cosf(arg);
    dfac = -h.amp[s] * h.freq[s] * sinf(arg);
  }
  dP = {0.f, 0.f, dz};
  f3 dm = {-dfac * cosf(h.psi[s]), -dfac * sinf(h.psi[s]), 0.f};
  float ilm = rsq(hx * hx + hy * hy + 1.0f);
  dN = (dm - n * dot(n, dm)) * ilm;
}

template <typename T>
__device__ __forceinline__ void theta_vertex(const DevScene& S, const ThetaDir* td, int vid, vec3<T>& P,
                                             vec3<T>& N) {
  if constexpr (is_dual<T>::value) {
    if (td && vid >= td->hf->first_vert && vid < td->hf->first_vert + td->hf->n_verts) {
      float4 p = S.vpos[vid], nn = S.vnrm[vid];
      f3 dP, dN;
      hf_vertex_deriv(*td->hf, td->s, td->which, p.x, p.y, ld3(nn), dP, dN);
      P.x.d = dP.x; P.y.d = dP.y; P.z.d = dP.z;
      N.x.d = dN.x; N.y.d = dN.y; N.z.d = dN.z;
    }
  }
}

template <typename T, bool DERIV>
__device__ __forceinline__ Geo<T> load_geo(const DevScene& S, int prim, vec3<T> x, const ThetaDir* td = nullptr) {
  Geo<T> g;
  g.x = x;
  if (prim < 0) {
    int s = -1 - prim;
    float4 sp = S.spheres[s];
    const int2 oi = S.obj_info[S.sphere_obj[s]];
    g.mat = oi.x;
    g.ior = (T)__int_as_float(oi.y);
    vec3<T> c = {(T)sp.x, (T)sp.y, (T)sp.z};
    vec3<T> d = x - c;
    T il = rsq(dot(d, d));
    g.ng = d * il;
    onb(g.ng, g.e1, g.e2);
    g.ns = g.ng;
    if (DERIV) {
      g.dns_a = g.e1 * il;
      g.dns_b = g.e2 * il;
    }
  } else {
    const float4* tg = S.tri_geo + 6 * (size_t)prim;
    const float4 q0 = tg[0], q1 = tg[1], q2 = tg[2];
    vec3<T> P0 = cvt<T>(ld3(q0)), P1 = cvt<T>(ld3(q1)), P2 = cvt<T>(ld3(q2));
    vec3<T> N0 = cvt<T>(ld3(tg[3])), N1 = cvt<T>(ld3(tg[4])), N2 = cvt<T>(ld3(tg[5]));
    g.mat = __float_as_int(q1.w);
    g.ior = (T)q2.w;
    if constexpr (is_dual<T>::value) {
      if (td) {
        const int4 id = S.tri_idx[prim];
        theta_vertex(S, td, id.x, P0, N0);
        theta_vertex(S, td, id.y, P1, N1);
        theta_vertex(S, td, id.z, P2, N2);
      }
    }
    vec3<T> E1 = P1 - P0, E2 = P2 - P0;
    T lenE1 = norm(E1);
    g.e1 = E1 * ((T)1 / lenE1);
    g.ng = normalize(cross(E1, E2));
    g.e2 = cross(g.ng, g.e1);
    T E2e1 = dot(E2, g.e1), E2e2 = dot(E2, g.e2);
    vec3<T> q = x - P0;
    T a = dot(q, g.e1), b = dot(q, g.e2);
    T b2 = b / E2e2;
    T b1 = (a - b2 * E2e1) / lenE1;
    T b0 = (T)1 - b1 - b2;
    vec3<T> nt = N0 * b0 + N1 * b1 + N2 * b2;
    T il = rsq(dot(nt, nt));
    g.ns = nt * il;
    if (DERIV) {
      T db1a = (T)1 / lenE1, db1b = -E2e1 / (lenE1 * E2e2), db2b = (T)1 / E2e2;
      vec3<T> dna = (N1 - N0) * db1a;
      vec3<T> dnb = (N1 - N0) * db1b + (N2 - N0) * db2b;
      g.dns_a = (dna - g.ns * dot(g.ns, dna)) * il;
      g.dns_b = (dnb - g.ns * dot(g.ns, dnb)) * il;
    }
  }
  return g;
}

// Tangent frame (e1, e2) of a vertex only (the back-substitution recomputes
// it instead of keeping 6 floats per vertex live across the sweep).
template <typename T>
__device__ __forceinline__ void load_frame(const DevScene& S, int prim, vec3<T> x, vec3<T>& e1, vec3<T>& e2) {
  if (prim < 0) {
    float4 sp = S.spheres[-1 - prim];
    vec3<T> c = {(T)sp.x, (T)sp.y, (T)sp.z};
    onb(normalize(x - c), e1, e2);
  } else {
    const float4* tg = S.tri_geo + 6 * (size_t)prim;
    vec3<T> P0 = cvt<T>(ld3(tg[0])), P1 = cvt<T>(ld3(tg[1])), P2 = cvt<T>(ld3(tg[2]));
    vec3<T> E1 = P1 - P0;
    e1 = normalize(E1);
    e2 = cross(normalize(cross(E1, P2 - P0)), e1);
  }
}

// Indices of refraction on the two sides of a vertex for incoming w_i.
template <typename T>
__device__ __forceinline__ void vertex_etas(const Geo<T>& g, bool transmit, vec3<T> xp, T& ea, T& eb) {
  if (!transmit) { ea = eb = (T)1; return; }
  bool outside = dot(xp - g.x, g.ng) > (T)0;
  ea = outside ? (T)1 : g.ior;
  eb = outside ? g.ior : (T)1;
}

// Per-vertex constraint and its Jacobian blocks.  The generalized half vector
// h = eta_a w_i + eta_b w_o must be parallel to the shading normal; the two
// residuals are its projections on the orthonormal shading frame
// s = normalize(e1 - (e1.n_s) n_s), t = n_s x s.
//   L = dC/dy_{i-1}, D = dC/dy_i, U = dC/dy_{i+1}; 2x2 blocks, row-major.
// With P_w = (I - w w^T)/l and Q = (I - h h^T)/|h|, the row vectors
//   gs_i = eta_a P_i Q s, gt_i = eta_a P_i Q t, gs_o = eta_b P_o Q s, gt_o = eta_b P_o Q t
// give L = [gs_i.e'; gt_i.e'] (e' of vertex i-1), U likewise with gs_o, gt_o
// and the next frame, and D = -[gs_i+gs_o; gt_i+gt_o].e + h.(ds, dt) where
// ds, dt are the shading-frame changes caused by dn_s.
template <typename T>
struct VJ {
  T C0, C1;
  T L[4], D[4], U[4];
  vec3<T> gso, gto;  // kept for dC/dx_L of the last vertex
  T cmin;            // min(|w_i.n_s|, |w_o.n_s|): grazing measure
};

//
// Glossy vertices (Sec. 5.7) carry an offset normal m = o_s s + o_t t +
// sqrt(1 - |o|^2) n_s and are specular about it: C = (sg h.s - o_s,
// sg h.t - o_t) with sg = sign(h.n_s), the frame (s, t) built from the world
// x axis instead of e1 so that it turns smoothly across triangles; the
// blocks scale by sg (the offsets are constants).
template <typename T>
__device__ __forceinline__ vec3<T> glossy_ref() { return vec3<T>{(T)1, (T)0, (T)0}; }

template <typename T, bool JAC>
__device__ __forceinline__ void vertex_cj(const Geo<T>& g, vec3<T> xp, vec3<T> xn, T ea, T eb, vec3<T> pe1,
                                          vec3<T> pe2, vec3<T> ne1, vec3<T> ne2, VJ<T>& o, bool glossy = false,
                                          T os = 0, T ot = 0) {
  vec3<T> di = xp - g.x, dq = xn - g.x;
  T ili = rsq(dot(di, di)), ilo = rsq(dot(dq, dq));
  vec3<T> wi = di * ili, wo = dq * ilo;
  vec3<T> h = wi * ea + wo * eb;
  T ilh = rsq(dot(h, h));
  vec3<T> hh = h * ilh;
  const vec3<T> ref = glossy ? glossy_ref<T>() : g.e1;
  vec3<T> st = ref - g.ns * dot(ref, g.ns);
  T ils = rsq(dot(st, st));
  vec3<T> s = st * ils;
  vec3<T> t = cross(g.ns, s);
  const T hs = dot(hh, s), ht = dot(hh, t);
  o.C0 = hs;
  o.C1 = ht;
  const T sg = glossy && dot(hh, g.ns) < (T)0 ? (T)-1 : (T)1;
  if (glossy) {
    o.C0 = sg * hs - os;
    o.C1 = sg * ht - ot;
  }
  if (!JAC) return;
  o.cmin = fmin(fabs(dot(wi, g.ns)), fabs(dot(wo, g.ns)));
  vec3<T> Qs = (s - hh * hs) * ilh, Qt = (t - hh * ht) * ilh;
  vec3<T> gsi = (Qs - wi * dot(wi, Qs)) * (ea * ili);
  vec3<T> gti = (Qt - wi * dot(wi, Qt)) * (ea * ili);
  vec3<T> gso = (Qs - wo * dot(wo, Qs)) * (eb * ilo);
  vec3<T> gto = (Qt - wo * dot(wo, Qt)) * (eb * ilo);
  o.gso = gso;
  o.gto = gto;
  o.L[0] = dot(gsi, pe1); o.L[1] = dot(gsi, pe2); o.L[2] = dot(gti, pe1); o.L[3] = dot(gti, pe2);
  o.U[0] = dot(gso, ne1); o.U[1] = dot(gso, ne2); o.U[2] = dot(gto, ne1); o.U[3] = dot(gto, ne2);
  vec3<T> gs = gsi + gso, gt = gti + gto;
  T e1n = dot(ref, g.ns);
  vec3<T> sxh = cross(s, hh), hxn = cross(hh, g.ns);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    vec3<T> ek = k == 0 ? g.e1 : g.e2;
    vec3<T> dn = k == 0 ? g.dns_a : g.dns_b;
    vec3<T> dst = g.ns * (-dot(ref, dn)) - dn * e1n;
    vec3<T> ds = (dst - s * dot(s, dst)) * ils;
    // h.dt with dt = dn x s + n x ds
    T hdt = dot(dn, sxh) + dot(ds, hxn);
    o.D[k] = -dot(gs, ek) + dot(hh, ds);
    o.D[2 + k] = -dot(gt, ek) + hdt;
  }
  if (glossy) {
#pragma unroll
    for (int k = 0; k < 4; ++k) { o.L[k] *= sg; o.D[k] *= sg; o.U[k] *= sg; }
    o.gso = o.gso * sg;
    o.gto = o.gto * sg;
  }
}

// Offset normals of a glossy chain: [2][K][N] device array (null: specular),
// chain c; (o_s, o_t) of vertex i.
struct Offs {
  const float* p;
  size_t NN;
  int c;
  __device__ __forceinline__ float s(int i) const { return p[(0 * KMAX + i) * NN + c]; }
  __device__ __forceinline__ float t(int i) const { return p[(1 * KMAX + i) * NN + c]; }
};
__device__ __forceinline__ Offs no_offs() { return Offs{nullptr, 0, 0}; }

// The offset normal of a glossy vertex from its shading normal.
template <typename T>
__device__ __forceinline__ vec3<T> offset_normal(vec3<T> ns, T os, T ot) {
  const vec3<T> ref = glossy_ref<T>();
  vec3<T> st = ref - ns * dot(ref, ns);
  vec3<T> s = st * rsq(dot(st, st));
  vec3<T> t = cross(ns, s);
  T c = sqrt(fmax((T)0, (T)1 - os * os - ot * ot));
  vec3<T> m = s * os + t * ot + ns * c;
  return m * rsq(dot(m, m));
}

template <typename T>
__device__ __forceinline__ T inv2(const T* A, T* I) {
  T det = A[0] * A[3] - A[1] * A[2];
  T id = (T)1 / det;
  I[0] = A[3] * id; I[1] = -A[1] * id; I[2] = -A[2] * id; I[3] = A[0] * id;
  return det;
}
template <typename T>
__device__ __forceinline__ void mul22(const T* A, const T* B, T* C) {
  C[0] = A[0] * B[0] + A[1] * B[2];
  C[1] = A[0] * B[1] + A[1] * B[3];
  C[2] = A[2] * B[0] + A[3] * B[2];
  C[3] = A[2] * B[1] + A[3] * B[3];
}
template <typename T> __device__ __forceinline__ T amax4(const T* A) {
  return fmax(fmax(fabs(A[0]), fabs(A[1])), fmax(fabs(A[2]), fabs(A[3])));
}

// Result of one sweep over the chain: residual norms, Newton step, and the
// elimination state needed by G and the FP64 check.
template <typename T, int N>
struct Sweep {
  vec3<T> dl[N];    // 3-D Newton displacement of each vertex
  T G[N][4];        // D~_i^-1 U_i
  T Dinv_last[4];   // D~_n^-1
  vec3<T> gso_last, gto_last;
  T Cv[N][2];       // the residual itself
  T c2, cinf;       // |C|_2^2, |C|_inf
  T cond;           // max |J| * max |D~^-1|
  T cmin;           // smallest incident / outgoing cosine along the chain
  bool singular;
};

// Forward sweep: evaluate C, J blocks vertex by vertex (a sliding window of
// three vertices) and eliminate the block-tridiagonal system J y = -C on the
// fly (block Thomas: D~_i = D_i - L_i G_{i-1}, r~_i = -C_i - L_i g_{i-1},
// G_i = D~_i^-1 U_i, g_i = D~_i^-1 r~_i), then back-substitute
// y_n = g_n, y_i = g_i - G_i y_{i+1}.  JAC = false evaluates C only.
template <typename T, int N, bool JAC, class STK, bool BACK = true>
__device__ __forceinline__ void sweep(const DevScene& S, vec3<T> xD, vec3<T> xL, int type, const int* prim,
                                      const vec3<T>* x, Sweep<T, N>& W, STK& stk,
                                      const ThetaDir* td = nullptr, Offs off = Offs{nullptr, 0, 0}) {
  T g[N][2];
  W.c2 = 0;
  W.cinf = 0;
  W.cond = 0;
  W.cmin = 1;
  W.singular = false;
  T jmax = 0, imax = 0;
  Geo<T> gc = load_geo<T, JAC>(S, prim[0], x[0], td);
  Geo<T> gn;
  if (N > 1) gn = load_geo<T, JAC>(S, prim[1], x[1], td);
  vec3<T> pe1 = gc.e1, pe2 = gc.e2;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    vec3<T> xp = i == 0 ? xD : x[i - 1];
    vec3<T> xn = i == N - 1 ? xL : x[i + 1];
    T ea, eb;
    vertex_etas(gc, (type >> i) & 1, xp, ea, eb);
    VJ<T> v;
    if (!JAC) stk.vc();
    else if (sizeof(T) == 4) stk.vj();
    else stk.vj64();
    if (off.p)
      vertex_cj<T, JAC>(gc, xp, xn, ea, eb, pe1, pe2, N > 1 && i < N - 1 ? gn.e1 : gc.e1,
                        N > 1 && i < N - 1 ? gn.e2 : gc.e2, v, true, (T)off.s(i), (T)off.t(i));
    else
      vertex_cj<T, JAC>(gc, xp, xn, ea, eb, pe1, pe2, N > 1 && i < N - 1 ? gn.e1 : gc.e1,
                        N > 1 && i < N - 1 ? gn.e2 : gc.e2, v);
    W.Cv[i][0] = v.C0;
    W.Cv[i][1] = v.C1;
    W.c2 += v.C0 * v.C0 + v.C1 * v.C1;
    W.cinf = fmax(W.cinf, fmax(fabs(v.C0), fabs(v.C1)));
    if (JAC) {
      W.cmin = fmin(W.cmin, v.cmin);
      T Dt[4] = {v.D[0], v.D[1], v.D[2], v.D[3]};
      T r0 = -v.C0, r1 = -v.C1;
      jmax = fmax(jmax, amax4(v.D));
      if (i > 0) {
        jmax = fmax(jmax, amax4(v.L));
        T LG[4];
        mul22(v.L, W.G[i - 1], LG);
        Dt[0] -= LG[0]; Dt[1] -= LG[1]; Dt[2] -= LG[2]; Dt[3] -= LG[3];
        r0 -= v.L[0] * g[i - 1][0] + v.L[1] * g[i - 1][1];
        r1 -= v.L[2] * g[i - 1][0] + v.L[3] * g[i - 1][1];
      }
      T I[4];
      T det = inv2(Dt, I);
      T sc = amax4(Dt);
      if (!(fabs(det) > (T)1e-10 * sc * sc) || !(sc > 0)) W.singular = true;
      imax = fmax(imax, amax4(I));
      g[i][0] = I[0] * r0 + I[1] * r1;
      g[i][1] = I[2] * r0 + I[3] * r1;
      if (i < N - 1) {
        jmax = fmax(jmax, amax4(v.U));
        mul22(I, v.U, W.G[i]);
      } else {
        W.Dinv_last[0] = I[0]; W.Dinv_last[1] = I[1]; W.Dinv_last[2] = I[2]; W.Dinv_last[3] = I[3];
        W.gso_last = v.gso;
        W.gto_last = v.gto;
      }
    }
    pe1 = gc.e1;
    pe2 = gc.e2;
    if (i + 1 < N) {
      gc = gn;
      if (i + 2 < N) gn = load_geo<T, JAC>(S, prim[i + 2 < N ? i + 2 : 0], x[i + 2 < N ? i + 2 : 0], td);
    }
  }
  if (!JAC) return;
  W.cond = jmax * imax;
  if (!BACK) return;
  T y0 = g[N - 1][0], y1 = g[N - 1][1];
  vec3<T> f1, f2;
  load_frame(S, prim[N - 1], x[N - 1], f1, f2);
  W.dl[N - 1] = f1 * y0 + f2 * y1;
#pragma unroll
  for (int i = N - 2; i >= 0; --i) {
    T z0 = g[i][0] - (W.G[i][0] * y0 + W.G[i][1] * y1);
    T z1 = g[i][1] - (W.G[i][2] * y0 + W.G[i][3] * y1);
    y0 = z0;
    y1 = z1;
    load_frame(S, prim[i], x[i], f1, f2);
    W.dl[i] = f1 * y0 + f2 * y1;
  }
}

// Reprojection: for i = 1..n in order, cast from the moved previous vertex
// (x_0 = x_D) toward the displaced vertex i; the first hit must lie on vertex
// i's object.
template <int N, class STK>
__device__ __forceinline__ bool reproject(const DevScene& S, f3 xD, const f3* x, const int* prim, const f3* dl,
                                          float beta, float tmin, STK& stk, f3* xn, int* pn) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    f3 o = i == 0 ? xD : xn[i > 0 ? i - 1 : 0];
    int excl = i == 0 ? PRIM_NONE : pn[i > 0 ? i - 1 : 0];
    f3 step = dl[i] * beta;
    f3 tg = x[i] + step;
    f3 d = tg - o;
    float l2 = dot(d, d);
    if (!(l2 > 0.0f)) return false;
    float il = rsq(l2);
    d = d * il;
    // The surface is expected near the target: search [tmin, bound] first;
    // the closest hit there is the closest overall.  Only a miss needs the
    // unbounded traversal.  The vertex's current triangle is tested first
    // (the moved point usually stays on it), which tightens the bound.
    float bound = 1.5f * l2 * il + 2.0f * norm(step) + 4.0f * tmin;
    Hit h;
    if (!trace(S, o, d, excl, tmin, h, stk, bound, prim[i])) return false;
    if (h.prim == PRIM_NONE && !trace(S, o, d, excl, tmin, h, stk)) return false;
    // the vertex stays on its object (looked up again rather than kept live
    // through the walk)
    if (h.prim == PRIM_NONE || prim_obj(S, h.prim) != prim_obj(S, prim[i])) return false;
    xn[i] = fmav(d, h.t, o);
    pn[i] = h.prim;
  }
  return true;
}

// Manifold walk (Newton + reprojection, Sec. 3) with the step rule:
// beta = 1; each trial counts as one iteration; the trial length is beta, or
// 1 once the full step moves every vertex by at most tol_vertex L; a failed
// reprojection halves the length; converged when the full step is that small
// and the trial's max|C| <= tol_residual; otherwise the trial is accepted iff
// |C|_2 decreases (then beta = min(1, 2 length)); a rejected full step that
// was within tol_vertex L ends the walk as ST_NEEDS_FP64 (precision floor);
// any other rejection sets beta = length / 2.
// Walk state of one chain between trial steps.
template <int N>
struct WalkState {
  int prim[N];
  f3 x[N], dl[N];
  float beta, c2, step2;
  int it;
  bool need_jac;  // the Jacobian sweep at x is due before the next trial
};

template <int N>
__device__ __forceinline__ void walk_begin(const DevScene& S, WalkState<N>& w) {
  w.beta = 1.0f;
  w.it = 0;
  w.need_jac = true;
}

// One step of a walk: the Jacobian sweep when due, then one trial.  Returns
// the final status, or -1 while the walk goes on.  walk_core loops over it;
// the lane-refill kernel interleaves it with taking new chains.
template <int N, class STK>
__device__ __forceinline__ int walk_step(const DevScene& S, const WalkParams& P, f3 xD, f3 xL, int type,
                                         WalkState<N>& w, STK& stk, Offs off = Offs{nullptr, 0, 0}) {
  if (w.need_jac) {
    Sweep<float, N> W;
    sweep<float, N, true>(S, xD, xL, type, w.prim, w.x, W, stk, nullptr, off);
    if (W.singular) return ST_SINGULAR;
    w.c2 = W.c2;
    w.step2 = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      w.dl[i] = W.dl[i];
      w.step2 = fmaxf(w.step2, dot(W.dl[i], W.dl[i]));
    }
    w.need_jac = false;
  }
  if (w.it >= P.max_iter) return ST_MAX_ITER;
  ++w.it;
  f3 xn[N];
  int pn[N];
  const bool small = w.step2 <= P.tol_step2;
  const float bt = small ? 1.0f : w.beta;
  if (!reproject<N>(S, xD, w.x, w.prim, w.dl, bt, P.tmin, stk, xn, pn)) {
    w.beta = 0.5f * bt;
    return -1;
  }
  Sweep<float, N> Wc;
  sweep<float, N, false>(S, xD, xL, type, pn, xn, Wc, stk, nullptr, off);
  const bool done = small && Wc.cinf <= P.tol_residual;
  if (done || Wc.c2 < w.c2) {
#pragma unroll
    for (int i = 0; i < N; ++i) { w.x[i] = xn[i]; w.prim[i] = pn[i]; }
    if (done) return ST_CONVERGED;
    w.need_jac = true;
    w.beta = fminf(1.0f, 2.0f * bt);
    return -1;
  }
  // the full step is within tolerance but no longer lowers the residual:
  // FP32 has reached its precision floor (e.g. near-grazing half vectors);
  // the FP64 pass decides
  if (small) return ST_NEEDS_FP64;
  w.beta = 0.5f * bt;
  return -1;
}

template <int N, class STK>
__device__ __forceinline__ int walk_core(const DevScene& S, const WalkParams& P, f3 xD, f3 xL, int type, int* prim, f3* x,
                         int& iters, STK& stk, Offs off = Offs{nullptr, 0, 0}) {
  WalkState<N> w;
#pragma unroll
  for (int i = 0; i < N; ++i) { w.prim[i] = prim[i]; w.x[i] = x[i]; }
  walk_begin<N>(S, w);
  int st;
  while ((st = walk_step<N>(S, P, xD, xL, type, w, stk, off)) < 0) {
  }
#pragma unroll
  for (int i = 0; i < N; ++i) { prim[i] = w.prim[i]; x[i] = w.x[i]; }
  iters = w.it;
  return st;
}

// Unpolarized Fresnel reflectance of a smooth dielectric (textbook form).
__device__ __forceinline__ float fresnel(float cos_i, float eta_i, float eta_t) {
  cos_i = fabsf(cos_i);
  float e = eta_i / eta_t;
  float s2 = e * e * fmaxf(0.0f, 1.0f - cos_i * cos_i);
  if (s2 >= 1.0f) return 1.0f;
  float ct = sqrtf(1.0f - s2);
  float rs = (eta_i * cos_i - eta_t * ct) / (eta_i * cos_i + eta_t * ct);
  float rp = (eta_t * cos_i - eta_i * ct) / (eta_t * cos_i + eta_i * ct);
  return 0.5f * (rs * rs + rp * rp);
}

// FP64 residual check of a near-singular converged chain: re-evaluate C in
// FP64 at the FP32 vertices and take up to two FP64 Newton steps inside the
// current primitives (planar for triangles, radial projection for spheres).
// On success xd holds the FP64 vertices and W their FP64 Jacobian sweep.
template <int N, class STK>
__device__ __forceinline__ bool fp64_check(const DevScene& S, d3 xD, d3 xL, int type, const int* prim, d3* xd,
                           Sweep<double, N>& W, float& resid, STK& stk, Offs off = Offs{nullptr, 0, 0}) {
  for (int k = 0; k < 2; ++k) {
    sweep<double, N, true>(S, xD, xL, type, prim, xd, W, stk, nullptr, off);
    if (W.cinf < 1e-12 || W.singular) break;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      d3 nx = xd[i] + W.dl[i];
      if (prim[i] < 0) {
        float4 sp = S.spheres[-1 - prim[i]];
        d3 c = {(double)sp.x, (double)sp.y, (double)sp.z};
        nx = c + normalize(nx - c) * (double)sp.w;
      }
      xd[i] = nx;
    }
  }
  sweep<double, N, true>(S, xD, xL, type, prim, xd, W, stk, nullptr, off);
  resid = (float)W.cinf;
  return W.cinf < 1e-6 && !W.singular;
}

struct WalkOut {
  int status, iters;
  uint64_t sol;
  float G, kappa, resid;
};

// Converged chain: FP64 check when near-singular, R/T side conditions,
// shadow ray to x_L, kappa, G (Eq. ThroughputEval) and the solution id.
// G = |n_D . w_D| |d w_D / d A_L| with d x_1 / d u_L from the implicit
// function theorem: only the last block row of dC/du_L is nonzero, so
// X_n = -D~_n^-1 B and X_i = -G_i X_{i+1}; u_L spans the plane
// perpendicular to x_n - x_L.
// Converged chain, after the FP64 decision: R/T side conditions, shadow ray
// to x_L, kappa, G (Eq. ThroughputEval) and the solution id, in precision T.
// G = |n_D . w_D| |d w_D / d A_L| with d x_1 / d u_L from the implicit
// function theorem: only the last block row of dC/du_L is nonzero, so
// X_n = -D~_n^-1 B and X_i = -G_i X_{i+1}; u_L spans the plane
// perpendicular to x_n - x_L.  W is the Jacobian sweep at the chain.
__device__ __forceinline__ float fresnel_t(float ci, float ei, float et) { return fresnel(ci, ei, et); }
__device__ __forceinline__ double fresnel_t(double cos_i, double eta_i, double eta_t) {
  cos_i = fabs(cos_i);
  double e = eta_i / eta_t;
  double s2 = e * e * fmax(0.0, 1.0 - cos_i * cos_i);
  if (s2 >= 1.0) return 1.0;
  double ct = sqrt(1.0 - s2);
  double rs = (eta_i * cos_i - eta_t * ct) / (eta_i * cos_i + eta_t * ct);
  double rp = (eta_t * cos_i - eta_i * ct) / (eta_t * cos_i + eta_i * ct);
  return 0.5 * (rs * rs + rp * rp);
}

template <typename T, int N, class STK>
__device__ __forceinline__ void finish_with(const DevScene& S, const WalkParams& P, vec3<T> xD, vec3<T> nD, vec3<T> xL, int type,
                            const int* prim, const vec3<T>* x, const Sweep<T, N>& W, STK& stk, WalkOut& R,
                            Offs off = Offs{nullptr, 0, 0}) {
  T kappa = 1;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    Geo<T> g = load_geo<T, false>(S, prim[i], x[i]);
    vec3<T> xp = i == 0 ? xD : x[i > 0 ? i - 1 : 0];
    vec3<T> xq = i == N - 1 ? xL : x[i < N - 1 ? i + 1 : 0];
    T a = dot(xp - x[i], g.ng), b = dot(xq - x[i], g.ng);
    bool Tr = (type >> i) & 1;
    if (Tr ? !(a * b < (T)0) : !(a * b > (T)0)) { R.status = ST_SIDE_INVALID; return; }
    if (g.mat != MAT_MIRROR) {
      vec3<T> wi = normalize(xp - x[i]);
      bool outside = a > (T)0;
      // a glossy vertex scatters at its offset normal
      vec3<T> nm = off.p ? offset_normal<T>(g.ns, (T)off.s(i), (T)off.t(i)) : g.ns;
      T F = fresnel_t(dot(wi, nm), outside ? (T)1 : g.ior, outside ? g.ior : (T)1);
      kappa *= Tr ? (T)1 - F : F;
    }
  }
  {
    f3 xl = cvt<float>(xL), xn = cvt<float>(x[N - 1]);
    f3 d = xl - xn;
    float dist = norm(d);
    Hit h;
    // only occluders strictly before the light matter
    trace(S, xn, d * (1.0f / dist), prim[N - 1], P.tmin, h, stk, dist * (1.0f - 1e-6f));
    if (h.prim != PRIM_NONE) { R.status = ST_OCCLUDED; return; }
  }
  vec3<T> wl = normalize(x[N - 1] - xL), t1, t2;
  onb(wl, t1, t2);
  T B[4] = {dot(W.gso_last, t1), dot(W.gso_last, t2), dot(W.gto_last, t1), dot(W.gto_last, t2)};
  T X[4];
  mul22(W.Dinv_last, B, X);
  X[0] = -X[0]; X[1] = -X[1]; X[2] = -X[2]; X[3] = -X[3];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) {
    T Y[4];
    mul22(W.G[i], X, Y);
    X[0] = -Y[0]; X[1] = -Y[1]; X[2] = -Y[2]; X[3] = -Y[3];
  }
  vec3<T> e1, e2;
  load_frame(S, prim[0], x[0], e1, e2);
  vec3<T> dx0 = e1 * X[0] + e2 * X[2];
  vec3<T> dx1 = e1 * X[1] + e2 * X[3];
  vec3<T> dd = x[0] - xD;
  T il = rsq(dot(dd, dd));
  vec3<T> w = dd * il;
  vec3<T> dw0 = (dx0 - w * dot(w, dx0)) * il, dw1 = (dx1 - w * dot(w, dx1)) * il;
  R.G = (float)(fabs(dot(nD, w)) * fabs(dot(w, cross(dw0, dw1))));
  R.kappa = (float)kappa;
  uint64_t hsh = splitmix64((uint64_t)N | ((uint64_t)type << 8));
#pragma unroll
  for (int i = 0; i < N; ++i) hsh = splitmix64(hsh ^ (uint64_t)(uint32_t)prim[i]);
  R.sol = hsh;
  R.status = ST_CONVERGED;
}

// First pass after convergence: chains whose final Jacobian is singular, whose
// condition estimate exceeds fp64_cond, or that scatter within graze_cos of
// grazing (where the FP32 Jacobian entries cancel) are left as ST_NEEDS_FP64
// for the FP64 pass; the others are finished in FP32.
template <int N, class STK>
__device__ __forceinline__ void finish(const DevScene& S, const WalkParams& P, f3 xD, f3 nD, f3 xL, int type, const int* prim,
                       const f3* x, STK& stk, WalkOut& R, Offs off = Offs{nullptr, 0, 0}) {
  Sweep<float, N> W;
  sweep<float, N, true>(S, xD, xL, type, prim, x, W, stk, nullptr, off);
  R.resid = W.cinf;
  if (W.singular || !(W.cond <= P.fp64_cond) || !(W.cmin >= P.graze_cos)) { R.status = ST_NEEDS_FP64; return; }
  finish_with<float, N, STK>(S, P, xD, nD, xL, type, prim, x, W, stk, R, off);
}

// FP64 pass for one flagged chain: FP64 residual check and polish, then the
// side / visibility tests, kappa and G in FP64.
template <int N, class STK>
__device__ __forceinline__ void finish_fp64(const DevScene& S, const WalkParams& P, f3 xD, f3 nD, f3 xL, int type, const int* prim,
                            f3* x, STK& stk, WalkOut& R, Offs off = Offs{nullptr, 0, 0}) {
  d3 xd[N];
#pragma unroll
  for (int i = 0; i < N; ++i) xd[i] = cvt<double>(x[i]);
  Sweep<double, N> W;
  float r64;
  bool ok = fp64_check<N>(S, cvt<double>(xD), cvt<double>(xL), type, prim, xd, W, r64, stk, off);
  R.resid = r64;
  if (!ok) { R.status = ST_FP64_REJECT; return; }
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = cvt<float>(xd[i]);
  finish_with<double, N, STK>(S, P, cvt<double>(xD), cvt<double>(nD), cvt<double>(xL), type, prim, xd, W, stk, R,
                              off);
}

// ---------------------------------------------------------------------------
// seeds: p_0 (Sec. 5.4), guided mixture and defensive MIS (Sec. 5.5),
// deduction (Eq. deduction)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int guide_cell(const DevGuide& G, f3 x) {
  float xs[3] = {x.x, x.y, x.z};
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float f = (xs[a] - G.lo[a]) / (G.hi[a] - G.lo[a]) * (float)G.res;
    if (!(f == f)) return -1;
    int k = (int)floorf(f);
    idx[a] = min(max(k, 0), G.res - 1);
  }
  return (idx[2] * G.res + idx[1]) * G.res + idx[0];
}

__device__ __forceinline__ bool p0_point(const DevScene& S, const WalkParams& P, int obj1, f3 xD, f3 nD, float u1, float u2,
                         float u3, f3& pt) {
  if (obj1 == P0_DIRECTION) {
    f3 ax = normalize(nD), b1, b2;
    onb(ax, b1, b2);
    float v = u2 * (1.0f - P.cone_cos);  // 1 - cos(theta), exact for the cap's small angles
    float ct = 1.0f - v;
    float st = sqrtf(fmaxf(0.0f, v * (2.0f - v)));
    float sn, cs;
    sincospif(2.0f * u3, &sn, &cs);
    pt = xD + b1 * (st * cs) + b2 * (st * sn) + ax * ct;
    return true;
  }
  int key = obj1 < 0 ? S.n_objects : obj1;
  if (key > S.n_objects) return false;
  int2 rg = S.cdf_range[key];
  if (rg.y <= 0) return false;
  // Inverse CDF in pair arithmetic (Dekker's exact product and Knuth's
  // two-sum, FP32 operations only): a prefix sum of ~10^5 triangle areas needs
  // about 40 significant bits to place the target between two neighbouring
  // prefixes as exactly as an FP64 evaluation would, which one FP32 value
  // cannot hold.
  const float2* cdf = S.cdf + rg.x;
  const float2 total = cdf[rg.y - 1];
  if (!(total.x > 0.0f)) return false;
  float th = u1 * total.x;
  float tl = fmaf(u1, total.x, -th) + u1 * total.y;
  {
    float s = th + tl;
    tl = tl - (s - th);
    th = s;
  }
  int lo = 0, hi = rg.y;  // first index with cdf > target
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    float2 c = cdf[mid];
    if (c.x > th || (c.x == th && c.y > tl)) hi = mid;
    else lo = mid + 1;
  }
  if (lo >= rg.y) lo = rg.y - 1;
  int prim = S.cdf_prim[rg.x + lo];
  if (prim >= 0) {
    const float4* tg = S.tri_geo + 6 * (size_t)prim;
    f3 a = ld3(tg[0]), b = ld3(tg[1]), c = ld3(tg[2]);
    float r = sqrtf(u2);
    pt = a * (1.0f - r) + b * (r * (1.0f - u3)) + c * (r * u3);
    return true;
  }
  float4 sp = S.spheres[-1 - prim];
  f3 cen = ld3(sp);
  f3 oc = xD - cen;
  float d = norm(oc);
  if (!(d > sp.w)) return false;
  f3 ax = oc * (1.0f / d), b1, b2;
  onb(ax, b1, b2);
  float cmax = sp.w / d;
  float v = u2 * (1.0f - cmax);
  float ct = 1.0f - v;
  float st = sqrtf(fmaxf(0.0f, v * (2.0f - v)));
  float sn, cs;
  sincospif(2.0f * u3, &sn, &cs);
  pt = cen + (b1 * (st * cs) + b2 * (st * sn) + ax * ct) * sp.w;
  return true;
}

template <class STK>
__device__ __forceinline__ bool guided_point(const DevScene& S, const DevGuide& G, int cell, uint64_t seed, uint64_t chain,
                             uint64_t trial, const U8& U0, STK& stk, f3& pt) {
  const int K = G.comps;
  for (int attempt = 0; attempt <= 8; ++attempt) {
    U8 U = attempt == 0 ? U0 : philox_uniforms(seed, chain, trial, (uint64_t)attempt);
    float acc = 0.0f;
    int j = K - 1;
    for (int q = 0; q < K; ++q) {
      acc += G.pi[cell * K + q];
      if (U.u[1] < acc) { j = q; break; }
    }
    float rr = sqrtf(-2.0f * logf(1.0f - U.u[2]));
    float sn, cs;
    sincospif(2.0f * U.u[3], &sn, &cs);
    float z0 = rr * cs, z1 = rr * sn;
    const float* mu = G.mu + (size_t)(cell * K + j) * 2;
    const float* L = G.chol + (size_t)(cell * K + j) * 3;
    float px = mu[0] + L[0] * z0, py = mu[1] + L[1] * z0 + L[2] * z1;
    float4 bd = S.obj_bounds[G.target_obj];
    if (px < bd.x || px > bd.z || py < bd.y || py > bd.w) continue;
    Hit h;
    const float top = *S.zmax + 1.0f;
    f3 o = {px, py, top};
    trace(S, o, f3{0.0f, 0.0f, -1.0f}, PRIM_NONE, 0.0f, h, stk);
    if (h.prim == PRIM_NONE) return false;
    pt = {px, py, top - h.t};
    return true;
  }
  return false;
}

template <int N, bool COINS, class STK>
__device__ __forceinline__ int deduce(const DevScene& S, const WalkParams& P, int type, const float* coins,
                                      float p_transmit, f3 xD, f3 pt, int* prim, f3* pos, STK& stk, int* type_out,
                                      Offs off = Offs{nullptr, 0, 0});

// One seed chain of length N.  Returns 0 or ST_SEED_INVALID.
template <int N, class STK>
__device__ __forceinline__ int sample_seed(const DevScene& S, const DevGuide* G, const WalkParams& P, int type, int obj1, f3 xD,
                           f3 nD, uint64_t seed, uint64_t chain, uint64_t trial, float alpha, int* prim, f3* pos,
                           STK& stk, Offs off = Offs{nullptr, 0, 0}) {
  U8 U = philox_uniforms(seed, chain, trial, 0);
  f3 pt;
  bool ok = false;
  // a guide without a cell table (valid == nullptr) stands for p_0 only
  int cell = G && G->valid ? guide_cell(*G, xD) : -1;
  bool guided = G && cell >= 0 && G->valid[cell] && !(U.u[0] < alpha);
  if (guided) ok = guided_point(S, *G, cell, seed, chain, trial, U, stk, pt);
  if (!ok) ok = p0_point(S, P, obj1, xD, nD, U.u[1], U.u[2], U.u[3], pt);
  if (!ok) return ST_SEED_INVALID;
  return deduce<N, false>(S, P, type, nullptr, 0.0f, xD, pt, prim, pos, stk, nullptr, off);
}

// Eq. (deduction): x_1 = r(x_D, w_D) with w_D towards pt, then x_i =
// r(x_{i-1}, s_tau(x_{i-1}, ...)).  COINS = false: the given type.  COINS =
// true: the type of each vertex is decided when the ray reaches it, as a path
// tracer would (Sec. 5.4): a mirror reflects, a dielectric transmits when its
// coin (coins[i]) is below p_transmit; the decided type goes to *type_out.
// Returns 0 or ST_SEED_INVALID.
template <int N, bool COINS, class STK>
__device__ __forceinline__ int deduce(const DevScene& S, const WalkParams& P, int type, const float* coins,
                                      float p_transmit, f3 xD, f3 pt, int* prim, f3* pos, STK& stk, int* type_out,
                                      Offs off) {
  f3 d = pt - xD;
  float l2 = dot(d, d);
  if (!(l2 > 0.0f)) return ST_SEED_INVALID;
  d = d * rsq(l2);
  f3 o = xD;
  int excl = PRIM_NONE;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i > 0) {
      int pp = prim[i > 0 ? i - 1 : 0];
      f3 xp = pos[i > 0 ? i - 1 : 0];
      Geo<float> g = load_geo<float, false>(S, pp, xp);
      // a glossy vertex scatters about its offset normal (Sec. 5.7)
      if (off.p) g.ns = offset_normal<float>(g.ns, off.s(i > 0 ? i - 1 : 0), off.t(i > 0 ? i - 1 : 0));
      if ((type >> (i - 1)) & 1) {
        if (g.mat != MAT_DIELECTRIC) return ST_SEED_INVALID;
        bool entering = dot(d, g.ng) < 0.0f;
        float eta = entering ? 1.0f / g.ior : g.ior;
        f3 nn = entering ? g.ns : -g.ns;
        float ci = -dot(d, nn);
        if (!(ci > 0.0f)) return ST_SEED_INVALID;
        float s2 = eta * eta * (1.0f - ci * ci);
        if (s2 >= 1.0f) return ST_SEED_INVALID;
        d = normalize(d * eta + nn * (eta * ci - sqrtf(1.0f - s2)));
      } else {
        d = normalize(d - g.ns * (2.0f * dot(d, g.ns)));
      }
      o = xp;
      excl = pp;
    }
    Hit h;
    if (!trace(S, o, d, excl, P.tmin, h, stk) || h.prim == PRIM_NONE) return ST_SEED_INVALID;
    prim[i] = h.prim;
    pos[i] = fmav(d, h.t, o);
    if (COINS) {
      bool transmit = prim_material(S, h.prim) == MAT_DIELECTRIC && coins[i] < p_transmit;
      type = transmit ? (type | (1 << i)) : (type & ~(1 << i));
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (((type >> i) & 1) && prim_material(S, prim[i]) != MAT_DIELECTRIC) return ST_SEED_INVALID;
  }
  if (COINS) *type_out = type;
  return 0;
}

}  // namespace mpg
