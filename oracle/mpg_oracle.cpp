// FP64 CPU oracle for the batched manifold-walk path of "Manifold Path Guiding
// for Importance Sampling Specular Chains" (Fan et al., ACM TOG 42(6), 2023).
//
// TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct reference
// that the tests, the benchmark's CPU-baseline leg and the smoke check run
// beside the HIP path.  It shares no code, header, table or constant generator
// with the HIP library; the two meet only through the seeded synthetic inputs.
// The product path must never call it.
//
// What it follows (paper sections; the constraint and Newton details the paper
// inherits by citation are restated from the geometry itself):
//   * sub-path / chain notation x_0 = x_D, x_1..x_n, x_{n+1} = x_L  -- Sec. 3, Table 1
//   * manifold walk = Newton's method + reprojection                 -- Sec. 3 "Manifold walks"
//   * admissible chains: every specular vertex satisfies the law of
//     reflection / refraction (generalized half-vector parallel to the
//     shading normal)                                               -- Sec. 3 "Specular manifolds"
//   * sub-path throughput T = kappa * G * L_o                          -- Eq. (ThroughputEval)
//   * seed deduction x_i = r(x_{i-1}, s_tau(...))                      -- Eq. (deduction), Sec. 5.3
//   * initial distribution p_0 (x_1 uniform on specular surfaces)     -- Sec. 5.4
//   * defensive one-sample MIS, alpha = 0.5                           -- Sec. 5.5 "Defensive sampling"
//   * reciprocal probability by repeated trials, P(n) factored out    -- Sec. 5.8
//   * sample weight w = T <1/P>                                       -- Eq. (eq_weight)
// Every reading where the paper is silent is listed in the design notes
// and restated at the function that implements it.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

#include "dual.hpp"

namespace oracle {

static const double kInf = std::numeric_limits<double>::infinity();
static const double kPi = 3.14159265358979323846;
static const int KMAX = 8;

enum Status : int8_t {
  ST_CONVERGED = 0,
  ST_MAX_ITER = 1,
  ST_SINGULAR = 2,
  ST_SIDE_INVALID = 3,
  ST_OCCLUDED = 4,
  ST_SEED_INVALID = 5,
  ST_FP64_REJECT = 6,
  ST_BAD_INPUT = 7,
  ST_STALLED = 8,  // internal: tiny full step that no longer lowers the residual
};
enum Material : int { MAT_MIRROR = 0, MAT_DIELECTRIC = 1 };

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  Round function:
// two 64x64->128 multiplies, xor with the other counter words and the round
// key; the key is bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}
static void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint64_t k[2] = {key_in[0], key_in[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B97F4A7C15ULL;
      k[1] += 0xBB67AE8584CAA73BULL;
    }
    uint64_t h0, l0, h1, l1;
    mulhilo64(0xD2E7470EE14C6C93ULL, c[0], &h0, &l0);
    mulhilo64(0xCA5A826395121157ULL, c[2], &h1, &l1);
    uint64_t n0 = h1 ^ c[1] ^ k[0], n2 = h0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = l1; c[2] = n2; c[3] = l0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}
// Eight uniforms in [0, 1) with 24-bit resolution from one Philox block:
// uniform j takes the high (j even) or low (j odd) 32-bit half of word j/2
// and keeps its top 24 bits.
struct Uniforms {
  double u[8];
};
static Uniforms draw(uint64_t seed, uint64_t chain, uint64_t trial, uint64_t attempt) {
  uint64_t ctr[4] = {chain, trial, attempt, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t w[4];
  philox4x64_10(ctr, key, w);
  Uniforms U;
  for (int j = 0; j < 8; ++j) {
    uint64_t word = w[j >> 1];
    uint32_t half = (j & 1) ? (uint32_t)(word & 0xffffffffULL) : (uint32_t)(word >> 32);
    U.u[j] = (double)(half >> 8) * (1.0 / 16777216.0);
  }
  return U;
}

// splitmix64 finalizer (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014) used to hash a chain's identity.
static inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static uint64_t solution_id(int n, int type, const int* prim) {
  uint64_t h = splitmix64((uint64_t)n | ((uint64_t)type << 8));
  for (int i = 0; i < n; ++i) h = splitmix64(h ^ (uint64_t)(uint32_t)prim[i]);
  return h;
}

// Orthonormal basis around a unit vector: the branchless construction of
// Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin, "Building an
// orthonormal basis, revisited", JCGT 6(1), 2017.
static void onb(const V3d& n, V3d* b1, V3d* b2) {
  double sign = std::copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  *b1 = V3d(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
  *b2 = V3d(b, sign + n.y * n.y * a, -n.y);
}

// ---------------------------------------------------------------------------
// Scene: triangles with vertex normals, analytic spheres, per-object material.
// Primitive ids: triangles >= 0 (input order), spheres -1 - s.
// ---------------------------------------------------------------------------
struct HeightField {
  int obj, res, first_vert, first_tri, n_sines;
  double x0, x1, y0, y1, z0;
  double amp[8], freq[8], psi[8], phase[8];
};

struct Node {
  V3d lo, hi;
  int left, right;   // children (interior) or -1
  int start, count;  // leaf range in `order`
};

struct Scene {
  std::vector<V3d> P, N;
  std::vector<int> tri;  // 3 per triangle
  std::vector<int> tri_obj;
  std::vector<int> mat;
  std::vector<double> ior;
  std::vector<V3d> sc;
  std::vector<double> sr;
  std::vector<int> sobj;
  double scale = 1.0;
  std::vector<HeightField> hfs;
  // median-split BVH over triangles
  std::vector<Node> nodes;
  std::vector<int> order;
  // area-proportional primitive choice per object (index n_obj = all objects)
  std::vector<std::vector<double>> cdf;
  std::vector<std::vector<int>> cdf_prim;
  // per object xy bounds (guided sampling domain)
  std::vector<double> obj_lo_x, obj_lo_y, obj_hi_x, obj_hi_y;
  double zmax = 0.0;
  int ntri() const { return (int)tri_obj.size(); }
  int nobj() const { return (int)mat.size(); }
  int prim_obj(int prim) const { return prim >= 0 ? tri_obj[prim] : sobj[-1 - prim]; }
};

static void tri_verts(const Scene& s, int t, V3d* a, V3d* b, V3d* c) {
  *a = s.P[s.tri[3 * t]];
  *b = s.P[s.tri[3 * t + 1]];
  *c = s.P[s.tri[3 * t + 2]];
}

static int build_node(Scene& s, std::vector<V3d>& cen, int start, int count) {
  Node nd;
  nd.lo = V3d(kInf, kInf, kInf);
  nd.hi = V3d(-kInf, -kInf, -kInf);
  V3d clo = nd.lo, chi = nd.hi;
  for (int i = start; i < start + count; ++i) {
    V3d v[3];
    tri_verts(s, s.order[i], &v[0], &v[1], &v[2]);
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) {
        nd.lo[a] = std::min(nd.lo[a], v[k][a]);
        nd.hi[a] = std::max(nd.hi[a], v[k][a]);
      }
    for (int a = 0; a < 3; ++a) {
      clo[a] = std::min(clo[a], cen[s.order[i]][a]);
      chi[a] = std::max(chi[a], cen[s.order[i]][a]);
    }
  }
  // pad the box so that rounding in the slab test cannot cull a true hit
  for (int a = 0; a < 3; ++a) {
    double pad = 1e-9 * (1.0 + std::fabs(nd.lo[a]) + std::fabs(nd.hi[a]));
    nd.lo[a] -= pad;
    nd.hi[a] += pad;
  }
  int idx = (int)s.nodes.size();
  s.nodes.push_back(nd);
  if (count <= 4) {
    s.nodes[idx].left = s.nodes[idx].right = -1;
    s.nodes[idx].start = start;
    s.nodes[idx].count = count;
    return idx;
  }
  int axis = 0;
  double ext = chi.x - clo.x;
  if (chi.y - clo.y > ext) { axis = 1; ext = chi.y - clo.y; }
  if (chi.z - clo.z > ext) { axis = 2; }
  int mid = start + count / 2;
  std::nth_element(s.order.begin() + start, s.order.begin() + mid, s.order.begin() + start + count,
                   [&](int a, int b) {
                     if (cen[a][axis] != cen[b][axis]) return cen[a][axis] < cen[b][axis];
                     return a < b;
                   });
  int l = build_node(s, cen, start, mid - start);
  int r = build_node(s, cen, mid, start + count - mid);
  s.nodes[idx].left = l;
  s.nodes[idx].right = r;
  s.nodes[idx].start = s.nodes[idx].count = 0;
  return idx;
}

// Moller-Trumbore ray/triangle test in FP64 (edges inclusive).
static bool hit_triangle(const V3d& o, const V3d& d, const V3d& a, const V3d& b, const V3d& c, double* t) {
  V3d e1 = b - a, e2 = c - a;
  V3d p = cross(d, e2);
  double det = dot(e1, p);
  if (det == 0.0) return false;
  double inv = 1.0 / det;
  V3d q = o - a;
  double u = dot(q, p) * inv;
  if (u < 0.0 || u > 1.0) return false;
  V3d r = cross(q, e1);
  double v = dot(d, r) * inv;
  if (v < 0.0 || u + v > 1.0) return false;
  *t = dot(e2, r) * inv;
  return true;
}

struct Hit {
  int prim = 0;
  double t = kInf;
  bool ok = false;
};

static void consider(Hit* h, int prim, double t) {
  if (!h->ok || t < h->t || (t == h->t && prim < h->prim)) {
    h->ok = true;
    h->t = t;
    h->prim = prim;
  }
}

// Sphere hit.  A ray leaving a point of the same sphere (`own`) has the root
// t = 0 at its origin; the other root t = -2 (o - c).d is the only candidate.
static void sphere_hits(const Scene& s, const V3d& o, const V3d& d, int exclude, double tmin, Hit* h) {
  for (size_t k = 0; k < s.sr.size(); ++k) {
    int prim = -1 - (int)k;
    V3d oc = o - s.sc[k];
    double b = dot(oc, d);
    if (prim == exclude) {
      double t = -2.0 * b;
      if (t > tmin) consider(h, prim, t);
      continue;
    }
    double cc = dot(oc, oc) - s.sr[k] * s.sr[k];
    double disc = b * b - cc;
    if (disc < 0.0) continue;
    double sq = std::sqrt(disc);
    double t0 = -b - sq, t1 = -b + sq;
    if (t0 > tmin) consider(h, prim, t0);
    else if (t1 > tmin) consider(h, prim, t1);
  }
}

// r(x, w): first intersection of the ray with the specular surfaces (Sec. 5.3),
// skipping the primitive the ray starts on and anything closer than tmin.
static Hit cast_ray(const Scene& s, const V3d& o, const V3d& d, int exclude, double tmin, bool brute = false) {
  Hit h;
  sphere_hits(s, o, d, exclude, tmin, &h);
  if (s.ntri() == 0) return h;
  if (brute) {
    for (int t = 0; t < s.ntri(); ++t) {
      if (t == exclude) continue;
      V3d a, b, c;
      tri_verts(s, t, &a, &b, &c);
      double th;
      if (hit_triangle(o, d, a, b, c, &th) && th > tmin) consider(&h, t, th);
    }
    return h;
  }
  V3d inv(1.0 / d.x, 1.0 / d.y, 1.0 / d.z);
  std::vector<int> stack;
  stack.reserve(64);
  stack.push_back(0);
  while (!stack.empty()) {
    const Node& nd = s.nodes[stack.back()];
    stack.pop_back();
    double t0 = -kInf, t1 = kInf;
    bool miss = false;
    for (int a = 0; a < 3; ++a) {
      if (d[a] == 0.0) {
        if (o[a] < nd.lo[a] || o[a] > nd.hi[a]) miss = true;
        continue;
      }
      double ta = (nd.lo[a] - o[a]) * inv[a], tb = (nd.hi[a] - o[a]) * inv[a];
      if (ta > tb) std::swap(ta, tb);
      t0 = std::max(t0, ta);
      t1 = std::min(t1, tb);
    }
    if (miss || t0 > t1 || t1 < tmin || (h.ok && t0 > h.t)) continue;
    if (nd.left < 0) {
      for (int i = nd.start; i < nd.start + nd.count; ++i) {
        int t = s.order[i];
        if (t == exclude) continue;
        V3d a, b, c;
        tri_verts(s, t, &a, &b, &c);
        double th;
        if (hit_triangle(o, d, a, b, c, &th) && th > tmin) consider(&h, t, th);
      }
    } else {
      stack.push_back(nd.left);
      stack.push_back(nd.right);
    }
  }
  return h;
}

// ---------------------------------------------------------------------------
// Local geometry of a specular vertex.  Each vertex has two degrees of
// freedom y = (a, b) along an orthonormal tangent frame (e1, e2) of its
// primitive at the current position:
//   triangle: e1 = normalize(P1 - P0), n_g = normalize((P1-P0) x (P2-P0)),
//             e2 = n_g x e1, x(a, b) = x_cur + a e1 + b e2 (exact, planar);
//             shading normal = normalized barycentric blend of vertex normals;
//   sphere:   n = (x_cur - c)/|x_cur - c|, (e1, e2) = onb(n),
//             x(a, b) = c + r normalize(x_cur - c + a e1 + b e2), n_s = n_g = n.
// ---------------------------------------------------------------------------
struct VGeo {
  int prim = 0, obj = 0, mat = 0;
  bool sphere = false;
  double ior = 1.0;
  V3d x, e1, e2, ng;
  V3d P0, N0, N1, N2;
  double lenE1 = 1, E2e1 = 0, E2e2 = 1;
  V3d c;
  double r = 1;
};

static VGeo make_geo(const Scene& s, int prim, const V3d& x) {
  VGeo g;
  g.prim = prim;
  g.obj = s.prim_obj(prim);
  g.mat = s.mat[g.obj];
  g.ior = s.ior[g.obj];
  g.x = x;
  if (prim < 0) {
    int k = -1 - prim;
    g.sphere = true;
    g.c = s.sc[k];
    g.r = s.sr[k];
    g.ng = normalize(x - g.c);
    onb(g.ng, &g.e1, &g.e2);
    return g;
  }
  V3d a, b, c;
  tri_verts(s, prim, &a, &b, &c);
  V3d E1 = b - a, E2 = c - a;
  g.P0 = a;
  g.N0 = s.N[s.tri[3 * prim]];
  g.N1 = s.N[s.tri[3 * prim + 1]];
  g.N2 = s.N[s.tri[3 * prim + 2]];
  g.lenE1 = norm(E1);
  g.e1 = E1 * (1.0 / g.lenE1);
  g.ng = normalize(cross(E1, E2));
  g.e2 = cross(g.ng, g.e1);
  g.E2e1 = dot(E2, g.e1);
  g.E2e2 = dot(E2, g.e2);
  return g;
}

template <class T>
static V3<T> geo_pos(const VGeo& g, const T& a, const T& b) {
  V3<T> off = lift<T>(g.e1) * a + lift<T>(g.e2) * b;
  if (g.sphere) return lift<T>(g.c) + normalize(lift<T>(g.x - g.c) + off) * T(g.r);
  return lift<T>(g.x) + off;
}

template <class T>
static V3<T> geo_shading(const VGeo& g, const V3<T>& x) {
  if (g.sphere) return normalize(x - lift<T>(g.c));
  V3<T> q = x - lift<T>(g.P0);
  T a = dot(q, lift<T>(g.e1)), b = dot(q, lift<T>(g.e2));
  T b2 = b / T(g.E2e2);
  T b1 = (a - b2 * T(g.E2e1)) / T(g.lenE1);
  T b0 = T(1) - b1 - b2;
  return normalize(lift<T>(g.N0) * b0 + lift<T>(g.N1) * b1 + lift<T>(g.N2) * b2);
}

// Per-vertex constraint: the generalized half vector
//   h = eta_a w_i + eta_b w_o,   w_i -> x_{i-1}, w_o -> x_{i+1} (unit),
// must be parallel to the shading normal n_s.  eta_a is the index of the
// medium on w_i's side of the geometric surface and eta_b that of the other
// side for a transmission; both are 1 for a reflection, where h reduces to
// the ordinary half vector.  The two residual components are the projections
// of h/|h| on the orthonormal shading tangent frame
//   s = normalize(e1 - (e1.n_s) n_s),  t = n_s x s.
//
// Glossy chains (Sec. 5.7): with a sampled offset normal m = o_s s + o_t t +
// sqrt(1 - o_s^2 - o_t^2) n_s the chain is specular about m instead of n_s,
// i.e. h/|h|, turned to the n_s side, has the tangential components (o_s,
// o_t): C = (sign(h.n_s) h.s - o_s, sign(h.n_s) h.t - o_t).  The offset is
// expressed in a frame that varies smoothly across triangles: s from the
// world x axis projected on the tangent plane (the caller passes it as e1),
// which holds wherever n_s is away from +-x (height fields, slabs).
template <class T>
static void vertex_constraint(const V3<T>& xp, const V3<T>& x, const V3<T>& xn, const V3<T>& ns, const V3d& e1,
                              double eta_a, double eta_b, const double* off, T* C) {
  V3<T> wi = normalize(xp - x), wo = normalize(xn - x);
  V3<T> h = normalize(wi * T(eta_a) + wo * T(eta_b));
  V3<T> E1 = lift<T>(e1);
  V3<T> s = normalize(E1 - ns * dot(E1, ns));
  V3<T> t = cross(ns, s);
  C[0] = dot(h, s);
  C[1] = dot(h, t);
  if (off) {
    double sg = val(dot(h, ns)) < 0.0 ? -1.0 : 1.0;
    C[0] = C[0] * T(sg) - T(off[0]);
    C[1] = C[1] * T(sg) - T(off[1]);
  }
}

static const V3d kGlossyRef(1.0, 0.0, 0.0);

// The offset normal of a glossy vertex (Sec. 5.7) in its shading frame.
static V3d offset_normal(const V3d& e1, const V3d& ns, const double* off) {
  V3d s = normalize(e1 - ns * dot(e1, ns));
  V3d t = cross(ns, s);
  double c = std::sqrt(std::max(0.0, 1.0 - off[0] * off[0] - off[1] * off[1]));
  return normalize(s * off[0] + t * off[1] + ns * c);
}

// Indices of refraction on the two sides of vertex g for incoming w_i.
static void etas(const VGeo& g, bool transmit, const V3d& wi, double* ea, double* eb) {
  if (!transmit) { *ea = *eb = 1.0; return; }
  if (dot(wi, g.ng) > 0.0) { *ea = 1.0; *eb = g.ior; }
  else { *ea = g.ior; *eb = 1.0; }
}

struct Chain {
  int n = 0, type = 0;
  VGeo v[KMAX];
  V3d xD, xL;
  double ea[KMAX], eb[KMAX];
  bool glossy = false;          // offset normals given (Sec. 5.7)
  double off[KMAX][2] = {{0}};  // per vertex (o_s, o_t)
  bool T(int i) const { return (type >> i) & 1; }
};

static void chain_etas(Chain* c) {
  for (int i = 0; i < c->n; ++i) {
    V3d xp = i == 0 ? c->xD : c->v[i - 1].x;
    etas(c->v[i], c->T(i), normalize(xp - c->v[i].x), &c->ea[i], &c->eb[i]);
  }
}

// Residual of the whole chain at offsets y (2n values) and a perturbation
// (u1, u2) of x_L in a tangent plane (t1, t2): used with dual numbers for
// the Jacobian and with doubles for the values.
template <class T>
static void chain_residual(const Chain& c, const T* y, const T& u1, const T& u2, const V3d& t1, const V3d& t2,
                           T* C) {
  V3<T> x[KMAX + 2], ns[KMAX];
  x[0] = lift<T>(c.xD);
  x[c.n + 1] = lift<T>(c.xL) + lift<T>(t1) * u1 + lift<T>(t2) * u2;
  for (int i = 0; i < c.n; ++i) {
    x[i + 1] = geo_pos(c.v[i], y[2 * i], y[2 * i + 1]);
    ns[i] = geo_shading(c.v[i], x[i + 1]);
  }
  for (int i = 0; i < c.n; ++i)
    vertex_constraint(x[i], x[i + 1], x[i + 2], ns[i], c.glossy ? kGlossyRef : c.v[i].e1, c.ea[i], c.eb[i],
                      c.glossy ? c.off[i] : nullptr, &C[2 * i]);
}

static void residual(const Chain& c, double* C) {
  double y[2 * KMAX] = {0};
  chain_residual<double>(c, y, 0.0, 0.0, V3d(), V3d(), C);
}

typedef Dual<double, 2 * KMAX + 2> DJ;

// Dense Jacobian J = dC/dy (2n x 2n) and B = dC/du_L (2n x 2) by forward-mode AD.
static void jacobian(const Chain& c, const V3d& t1, const V3d& t2, double* C, double* J, double* B) {
  const int m = 2 * c.n;
  DJ y[2 * KMAX];
  for (int k = 0; k < m; ++k) y[k] = DJ::var(0.0, k);
  DJ u1 = DJ::var(0.0, 2 * KMAX), u2 = DJ::var(0.0, 2 * KMAX + 1);
  DJ Cd[2 * KMAX];
  chain_residual<DJ>(c, y, u1, u2, t1, t2, Cd);
  for (int r = 0; r < m; ++r) {
    if (C) C[r] = Cd[r].v;
    for (int k = 0; k < m; ++k) J[r * m + k] = Cd[r].d[k];
    if (B) {
      B[r * 2] = Cd[r].d[2 * KMAX];
      B[r * 2 + 1] = Cd[r].d[2 * KMAX + 1];
    }
  }
}

// Dense Gaussian elimination with partial pivoting; X (m x k) overwrites R.
// Returns false when a pivot falls below 1e-14 of the largest entry of A.
static bool dense_solve(int m, double* A, int k, double* R) {
  double amax = 0.0;
  for (int i = 0; i < m * m; ++i) amax = std::max(amax, std::fabs(A[i]));
  if (!(amax > 0.0) || !std::isfinite(amax)) return false;
  for (int col = 0; col < m; ++col) {
    int p = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(A[r * m + col]) > std::fabs(A[p * m + col])) p = r;
    if (std::fabs(A[p * m + col]) < 1e-14 * amax) return false;
    if (p != col) {
      for (int j = 0; j < m; ++j) std::swap(A[p * m + j], A[col * m + j]);
      for (int j = 0; j < k; ++j) std::swap(R[p * k + j], R[col * k + j]);
    }
    for (int r = col + 1; r < m; ++r) {
      double f = A[r * m + col] / A[col * m + col];
      if (f == 0.0) continue;
      for (int j = col; j < m; ++j) A[r * m + j] -= f * A[col * m + j];
      for (int j = 0; j < k; ++j) R[r * k + j] -= f * R[col * k + j];
    }
  }
  for (int col = m - 1; col >= 0; --col) {
    for (int j = 0; j < k; ++j) {
      double acc = R[col * k + j];
      for (int c2 = col + 1; c2 < m; ++c2) acc -= A[col * m + c2] * R[c2 * k + j];
      R[col * k + j] = acc / A[col * m + col];
    }
  }
  return true;
}

static double inf_norm(const double* v, int m) {
  double r = 0.0;
  for (int i = 0; i < m; ++i) r = std::max(r, std::fabs(v[i]));
  return r;
}
static double two_norm(const double* v, int m) {
  double r = 0.0;
  for (int i = 0; i < m; ++i) r += v[i] * v[i];
  return std::sqrt(r);
}

struct Params {
  int max_iter;
  double tol_vertex;    // converged when the full Newton step moves every vertex <= tol_vertex * scale
  double tol_residual;  // ... and the residual's max-norm after that step is <= tol_residual
  double scale;         // scene scale L
  double tmin_rel;      // ray epsilon, relative to L
  double match_rel;     // trial-match distance, relative to L
  double polish_tol;    // FP64 polish target (oracle only)
  double cone_cos;      // direction-mode p_0: cosine of the cone half-angle about n_D
};

// Newton direction: solve J delta = -C; the 3-D displacement of vertex i is
// delta_a e1 + delta_b e2.
static bool newton_direction(const Chain& c, double* C, V3d* disp) {
  const int m = 2 * c.n;
  double J[4 * KMAX * KMAX], R[2 * KMAX];
  jacobian(c, V3d(), V3d(), C, J, nullptr);
  for (int i = 0; i < m; ++i) R[i] = -C[i];
  if (!dense_solve(m, J, 1, R)) return false;
  for (int i = 0; i < c.n; ++i) disp[i] = c.v[i].e1 * R[2 * i] + c.v[i].e2 * R[2 * i + 1];
  return true;
}

// Reprojection: for i = 1..n in order, cast a ray from the (already moved)
// previous vertex toward the displaced vertex i; the first hit over the whole
// scene must lie on vertex i's object.  x_0 = x_D.
static bool reproject(const Scene& s, const Chain& c, const V3d* target, double tmin, Chain* out) {
  *out = c;
  for (int i = 0; i < c.n; ++i) {
    V3d o = i == 0 ? c.xD : out->v[i - 1].x;
    int excl = i == 0 ? std::numeric_limits<int>::min() : out->v[i - 1].prim;
    V3d dir = target[i] - o;
    double len = norm(dir);
    if (!(len > 0.0)) return false;
    dir = dir * (1.0 / len);
    Hit h = cast_ray(s, o, dir, excl, tmin);
    if (!h.ok) return false;
    if (s.prim_obj(h.prim) != c.v[i].obj) return false;
    out->v[i] = make_geo(s, h.prim, o + dir * h.t);
  }
  chain_etas(out);
  return true;
}

struct WalkResult {
  int8_t status = ST_BAD_INPUT;
  int iters = 0;
  int polish_steps = 0;
  bool polished = false;
  double residual = 0;
  double G = 0, kappa = 0;
  uint64_t sol = 0;
  Chain chain;
};

// Manifold walk (Sec. 3): Newton's method with reprojection and the
// step-length rule below (the paper leaves the rule to its citations):
//   beta = 1; every trial step counts as one iteration;
//   the trial length is beta, or 1 when the full step max_i |delta_i| is
//   within tol_vertex L; trial x' = reproject(x + length delta);
//   a failed reprojection halves the length;
//   converged when the full step is within tol_vertex L and
//   |C(x')|_inf <= tol_residual (x' is kept);
//   otherwise accept iff |C(x')|_2 < |C(x)|_2 (then beta = min(1, 2 length));
//   a rejected full step that was within tol_vertex L stops the walk as
//   stalled (precision floor), handed to the FP64 check;
//   any other rejection sets beta = length / 2.
static void walk_core(const Scene& s, const Params& p, const Chain& start, WalkResult* res) {
  const int m = 2 * start.n;
  const double tmin = p.tmin_rel * p.scale;
  Chain c = start;
  double C[2 * KMAX];
  V3d disp[KMAX];
  if (!newton_direction(c, C, disp)) { res->status = ST_SINGULAR; res->chain = c; return; }
  double beta = 1.0;
  res->status = ST_MAX_ITER;
  for (int it = 1; it <= p.max_iter; ++it) {
    res->iters = it;
    double step = 0.0;
    for (int i = 0; i < c.n; ++i) step = std::max(step, norm(disp[i]));
    // once the full Newton step is within the vertex tolerance it is always tried whole
    bool small = step <= p.tol_vertex * p.scale;
    double bt = small ? 1.0 : beta;
    V3d target[KMAX];
    for (int i = 0; i < c.n; ++i) target[i] = c.v[i].x + disp[i] * bt;
    Chain trial;
    if (!reproject(s, c, target, tmin, &trial)) { beta = 0.5 * bt; continue; }
    double Ct[2 * KMAX];
    residual(trial, Ct);
    if (small && inf_norm(Ct, m) <= p.tol_residual) {
      c = trial;
      res->status = ST_CONVERGED;
      break;
    }
    if (two_norm(Ct, m) < two_norm(C, m)) {
      c = trial;
      if (!newton_direction(c, C, disp)) { res->status = ST_SINGULAR; break; }
      beta = std::min(1.0, 2.0 * bt);
    } else if (small) {
      // the full step is within tolerance but no longer lowers the residual:
      // the walk has reached its precision floor; the FP64 check decides
      res->status = ST_STALLED;
      break;
    } else {
      beta = 0.5 * bt;
    }
  }
  res->chain = c;
}

// Oracle-only FP64 polish: pure Newton steps (beta = 1) with reprojection.
static void polish(const Scene& s, const Params& p, WalkResult* res) {
  Chain& c = res->chain;
  const int m = 2 * c.n;
  double C[2 * KMAX];
  residual(c, C);
  for (int k = 0; k < 10 && inf_norm(C, m) >= p.polish_tol; ++k) {
    V3d disp[KMAX], target[KMAX];
    double Cn[2 * KMAX];
    if (!newton_direction(c, Cn, disp)) break;
    for (int i = 0; i < c.n; ++i) target[i] = c.v[i].x + disp[i];
    Chain t;
    if (!reproject(s, c, target, p.tmin_rel * p.scale, &t)) break;
    double Ct[2 * KMAX];
    residual(t, Ct);
    if (!(inf_norm(Ct, m) < inf_norm(C, m))) break;
    c = t;
    std::memcpy(C, Ct, sizeof(double) * m);
    res->polish_steps++;
  }
  res->residual = inf_norm(C, m);
  res->polished = res->residual < 1e-10;
}

// Unpolarized Fresnel reflectance of a smooth dielectric interface (textbook
// exact form): cos_i on the incident side, eta_i / eta_t the index ratio.
static double fresnel_dielectric(double cos_i, double eta_i, double eta_t) {
  cos_i = std::fabs(cos_i);
  double e = eta_i / eta_t;
  double sin2_t = e * e * std::max(0.0, 1.0 - cos_i * cos_i);
  if (sin2_t >= 1.0) return 1.0;
  double cos_t = std::sqrt(1.0 - sin2_t);
  double rs = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
  double rp = (eta_t * cos_i - eta_i * cos_t) / (eta_t * cos_i + eta_i * cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

// kappa of Eq. (ThroughputEval): product of the per-vertex scattering
// coefficients (ideal mirror 1, dielectric reflection F, transmission 1 - F).
static double chain_kappa(const Chain& c) {
  double k = 1.0;
  for (int i = 0; i < c.n; ++i) {
    const VGeo& g = c.v[i];
    if (g.mat == MAT_MIRROR) continue;
    V3d xp = i == 0 ? c.xD : c.v[i - 1].x;
    V3d wi = normalize(xp - g.x);
    V3d ns = geo_shading<double>(g, g.x);
    if (c.glossy) ns = offset_normal(kGlossyRef, ns, c.off[i]);
    // physical indices: incident side of w_i, transmitted side the other
    bool outside = dot(wi, g.ng) > 0.0;
    double F = fresnel_dielectric(dot(wi, ns), outside ? 1.0 : g.ior, outside ? g.ior : 1.0);
    k *= c.T(i) ? (1.0 - F) : F;
  }
  return k;
}

// Generalized geometric term (Eq. ThroughputEval; it maps the differential
// area at x_L to the projected solid angle at x_D):
//   G = |n_D . w_D| * |d w_D / d A_L|,
// with d x_1 / d x_L from the implicit function theorem on the constraint
// (dy/du_L = -J^{-1} dC/du_L, only the last block row of dC/du_L is nonzero)
// and x_L's area element taken in the plane perpendicular to x_n - x_L
// (point lights).  For n = 0 it reduces to |cos_D| |cos_L| / d^2.
static double chain_G(const Chain& c, const V3d& nD) {
  const int m = 2 * c.n;
  V3d wl = normalize(c.v[c.n - 1].x - c.xL);
  V3d t1, t2;
  onb(wl, &t1, &t2);
  double J[4 * KMAX * KMAX], B[4 * KMAX];
  jacobian(c, t1, t2, nullptr, J, B);
  for (int i = 0; i < 2 * m; ++i) B[i] = -B[i];
  if (!dense_solve(m, J, 2, B)) return 0.0;
  V3d dx[2];
  for (int k = 0; k < 2; ++k) dx[k] = c.v[0].e1 * B[0 * 2 + k] + c.v[0].e2 * B[1 * 2 + k];
  V3d d = c.v[0].x - c.xD;
  double len = norm(d);
  V3d w = d * (1.0 / len);
  V3d dw[2];
  for (int k = 0; k < 2; ++k) dw[k] = (dx[k] - w * dot(w, dx[k])) * (1.0 / len);
  double area = std::fabs(dot(w, cross(dw[0], dw[1])));
  return std::fabs(dot(nD, w)) * area;
}

static bool side_ok(const Chain& c) {
  for (int i = 0; i < c.n; ++i) {
    V3d xp = i == 0 ? c.xD : c.v[i - 1].x;
    V3d xn = i == c.n - 1 ? c.xL : c.v[i + 1].x;
    double a = dot(xp - c.v[i].x, c.v[i].ng), b = dot(xn - c.v[i].x, c.v[i].ng);
    if (c.T(i) ? !(a * b < 0.0) : !(a * b > 0.0)) return false;
  }
  return true;
}

static bool visible_to_light(const Scene& s, const Params& p, const Chain& c) {
  const VGeo& last = c.v[c.n - 1];
  V3d d = c.xL - last.x;
  double dist = norm(d);
  Hit h = cast_ray(s, last.x, d * (1.0 / dist), last.prim, p.tmin_rel * p.scale);
  return !(h.ok && h.t < dist * (1.0 - 1e-6));
}

static bool load_chain(const Scene& s, int n, int type, const V3d& xD, const V3d& xL, const int* prim,
                       const V3d* pos, Chain* c) {
  if (n < 1 || n > KMAX) return false;
  c->n = n;
  c->type = type;
  c->xD = xD;
  c->xL = xL;
  for (int i = 0; i < n; ++i) {
    if (prim[i] >= s.ntri() || (prim[i] < 0 && -1 - prim[i] >= (int)s.sr.size())) return false;
    c->v[i] = make_geo(s, prim[i], pos[i]);
    if (c->T(i) && c->v[i].mat != MAT_DIELECTRIC) return false;
  }
  chain_etas(c);
  return true;
}

static bool finite3(const V3d& v) { return std::isfinite(v.x) && std::isfinite(v.y) && std::isfinite(v.z); }

// Full walk of one chain: walk, (oracle) polish, side and visibility tests,
// then G, kappa and the solution id.
static void walk_chain(const Scene& s, const Params& p, int n, int type, const V3d& xD, const V3d& nD, const V3d& xL,
                       const int* prim, const V3d* pos, bool do_polish, WalkResult* res, const double* offs = nullptr) {
  Chain c;
  if (!finite3(xD) || !finite3(xL) || n < 1 || n > KMAX) { res->status = ST_BAD_INPUT; return; }
  if (!load_chain(s, n, type, xD, xL, prim, pos, &c)) { res->status = ST_SEED_INVALID; res->chain = c; return; }
  if (offs) {
    c.glossy = true;
    for (int i = 0; i < n; ++i) { c.off[i][0] = offs[2 * i]; c.off[i][1] = offs[2 * i + 1]; }
  }
  walk_core(s, p, c, res);
  bool stalled = res->status == ST_STALLED;
  if (res->status != ST_CONVERGED && !stalled) return;
  if (do_polish || stalled) polish(s, p, res);
  else {
    double C[2 * KMAX];
    residual(res->chain, C);
    res->residual = inf_norm(C, 2 * n);
  }
  // FP64 check of a stalled walk: accepted when the FP64 residual is < 1e-6
  if (stalled) {
    if (!(res->residual < 1e-6)) { res->status = ST_FP64_REJECT; return; }
    res->status = ST_CONVERGED;
  }
  if (!side_ok(res->chain)) { res->status = ST_SIDE_INVALID; return; }
  if (!visible_to_light(s, p, res->chain)) { res->status = ST_OCCLUDED; return; }
  res->kappa = chain_kappa(res->chain);
  res->G = chain_G(res->chain, nD);
  int prims[KMAX];
  for (int i = 0; i < n; ++i) prims[i] = res->chain.v[i].prim;
  res->sol = solution_id(n, type, prims);
}

// ---------------------------------------------------------------------------
// Seeds: p_0 (Sec. 5.4), the guided 2-D Gaussian mixture, the defensive
// one-sample mixture of the two (Sec. 5.5), and deduction (Eq. deduction).
// ---------------------------------------------------------------------------
struct Guide {
  int res = 32, comps = 8;
  double lo[3], hi[3];
  int target_obj = 0;
  std::vector<int> valid;      // [cells]
  std::vector<double> pi;      // [cells][comps]
  std::vector<double> mu;      // [cells][comps][2]
  std::vector<double> chol;    // [cells][comps][3]  L00, L10, L11
};

// Cell of a point on the regular res^3 grid over [lo, hi] (the spatial
// structure of the guide, Sec. 5.6): floor((x - lo) / (hi - lo) res) per axis
// in FP64, clamped to the grid.  Points within rounding of a cell face may
// land in the neighbouring cell on an FP32 implementation.
static int grid_cell(const double* lo, const double* hi, int res, const double* x) {
  int idx[3];
  for (int a = 0; a < 3; ++a) {
    double f = (x[a] - lo[a]) / (hi[a] - lo[a]) * (double)res;
    if (!(f == f)) return -1;
    double k = std::floor(f);
    idx[a] = (int)std::min(std::max(k, 0.0), (double)(res - 1));
  }
  return (idx[2] * res + idx[1]) * res + idx[0];
}

static int guide_cell(const Guide& g, const V3d& x) {
  double p[3] = {x.x, x.y, x.z};
  return grid_cell(g.lo, g.hi, g.res, p);
}

// p_0 (Sec. 5.4).  obj1 >= 0: x_1 uniform by area on that object;
// obj1 == -1: uniform by area over all specular objects; for an analytic
// sphere the point is uniform over the cap visible from x_D.  obj1 == -2:
// the direction-based initialization (Sec. 6.4, "Initialization": w_D uniform
// on the hemisphere about n_D, cone_cos = 0), here restricted to the cone
// with cos(half-angle) = cone_cos when that cone contains every admissible
// first direction of the workload.
static bool sample_p0_point(const Scene& s, const Params& p, int obj1, const V3d& xD, const V3d& nD, double u1,
                            double u2, double u3, V3d* pt) {
  if (obj1 == -2) {
    V3d ax = normalize(nD), b1, b2;
    onb(ax, &b1, &b2);
    double v = u2 * (1.0 - p.cone_cos);  // 1 - cos(theta)
    double ct = 1.0 - v;
    double st = std::sqrt(std::max(0.0, v * (2.0 - v)));
    double ph = 2.0 * kPi * u3;
    *pt = xD + b1 * (st * std::cos(ph)) + b2 * (st * std::sin(ph)) + ax * ct;
    return true;
  }
  (void)u1;
  int key = obj1 < 0 ? s.nobj() : obj1;
  if (key > s.nobj()) return false;
  const std::vector<double>& cdf = s.cdf[key];
  if (cdf.empty() || !(cdf.back() > 0.0)) return false;
  double target = u1 * cdf.back();
  size_t j = std::upper_bound(cdf.begin(), cdf.end(), target) - cdf.begin();
  if (j >= cdf.size()) j = cdf.size() - 1;
  int prim = s.cdf_prim[key][j];
  if (prim >= 0) {
    V3d a, b, c;
    tri_verts(s, prim, &a, &b, &c);
    double r = std::sqrt(u2);
    *pt = a * (1.0 - r) + b * (r * (1.0 - u3)) + c * (r * u3);
    return true;
  }
  // sphere: uniform over the cap visible from x_D
  int k = -1 - prim;
  V3d oc = xD - s.sc[k];
  double d = norm(oc);
  if (!(d > s.sr[k])) return false;
  V3d ax = oc * (1.0 / d), b1, b2;
  onb(ax, &b1, &b2);
  double cmax = s.sr[k] / d;
  double v = u2 * (1.0 - cmax);  // 1 - cos(theta)
  double ct = 1.0 - v;
  double st = std::sqrt(std::max(0.0, v * (2.0 - v)));
  double ph = 2.0 * kPi * u3;
  *pt = s.sc[k] + (b1 * (st * std::cos(ph)) + b2 * (st * std::sin(ph)) + ax * ct) * s.sr[k];
  return true;
}

static bool sample_guided_point(const Scene& s, const Guide& g, int cell, uint64_t seed, uint64_t chain,
                                uint64_t trial, const Uniforms& U0, V3d* pt) {
  const int K = g.comps;
  for (int attempt = 0; attempt <= 8; ++attempt) {
    Uniforms U = attempt == 0 ? U0 : draw(seed, chain, trial, attempt);
    double acc = 0.0;
    int j = K - 1;
    for (int q = 0; q < K; ++q) {
      acc += g.pi[cell * K + q];
      if (U.u[1] < acc) { j = q; break; }
    }
    double rr = std::sqrt(-2.0 * std::log(1.0 - U.u[2]));
    double z0 = rr * std::cos(2.0 * kPi * U.u[3]), z1 = rr * std::sin(2.0 * kPi * U.u[3]);
    const double* mu = &g.mu[(cell * K + j) * 2];
    const double* L = &g.chol[(cell * K + j) * 3];
    double px = mu[0] + L[0] * z0, py = mu[1] + L[1] * z0 + L[2] * z1;
    int o = g.target_obj;
    if (px < s.obj_lo_x[o] || px > s.obj_hi_x[o] || py < s.obj_lo_y[o] || py > s.obj_hi_y[o]) continue;
    // lift onto the surface with a vertical ray from above the scene
    Hit h = cast_ray(s, V3d(px, py, s.zmax + 1.0), V3d(0, 0, -1), std::numeric_limits<int>::min(), 0.0);
    if (!h.ok) return false;
    *pt = V3d(px, py, s.zmax + 1.0 - h.t);
    return true;
  }
  return false;
}

static int8_t deduce_chain(const Scene& s, const Params& p, int n, int type, const double* coins, double p_transmit,
                           const V3d& xD, const V3d& pt, int* prim, V3d* pos, int* type_out,
                           const double* offs = nullptr);

static int8_t sample_seed(const Scene& s, const Guide* g, const Params& p, int n, int type, int obj1,
                          const V3d& xD, const V3d& nD, uint64_t seed, uint64_t chain, uint64_t trial, double alpha,
                          int* prim, V3d* pos, const double* offs = nullptr) {
  if (n < 1 || n > KMAX || !finite3(xD)) return ST_BAD_INPUT;
  Uniforms U = draw(seed, chain, trial, 0);
  V3d pt;
  bool ok;
  int cell = g ? guide_cell(*g, xD) : -1;
  bool guided = g && cell >= 0 && g->valid[cell] && !(U.u[0] < alpha);
  if (guided) {
    ok = sample_guided_point(s, *g, cell, seed, chain, trial, U, &pt);
    if (!ok) ok = sample_p0_point(s, p, obj1, xD, nD, U.u[1], U.u[2], U.u[3], &pt);
  } else {
    ok = sample_p0_point(s, p, obj1, xD, nD, U.u[1], U.u[2], U.u[3], &pt);
  }
  if (!ok) return ST_SEED_INVALID;
  return deduce_chain(s, p, n, type, nullptr, 0.0, xD, pt, prim, pos, nullptr, offs);
}

// Eq. (deduction): x_1 = r(x_D, w_D) with w_D towards pt, then x_i = r(x_{i-1},
// s_tau(x_{i-1}, ...)) with the scattering type of vertex i-1.  With coins
// == nullptr the type is the given one; otherwise the type of each vertex is
// decided when the ray reaches it, as a path tracer would (Sec. 5.4): a
// mirror reflects, a dielectric transmits when its coin is below
// p_transmit and reflects otherwise; the decided type is returned in
// *type_out.  Returns 0 or ST_SEED_INVALID.
static int8_t deduce_chain(const Scene& s, const Params& p, int n, int type, const double* coins, double p_transmit,
                           const V3d& xD, const V3d& pt, int* prim, V3d* pos, int* type_out, const double* offs) {
  const double tmin = p.tmin_rel * p.scale;
  V3d o = xD, d = pt - xD;
  double len = norm(d);
  if (!(len > 0.0)) return ST_SEED_INVALID;
  d = d * (1.0 / len);
  int excl = std::numeric_limits<int>::min();
  for (int i = 0; i < n; ++i) {
    if (i > 0) {
      // scatter at vertex i-1 with its type (Eq. deduction)
      VGeo gv = make_geo(s, prim[i - 1], pos[i - 1]);
      V3d ns = geo_shading<double>(gv, gv.x);
      // a glossy vertex scatters about its offset normal (Sec. 5.7)
      if (offs) ns = offset_normal(kGlossyRef, ns, offs + 2 * (i - 1));
      if ((type >> (i - 1)) & 1) {
        if (gv.mat != MAT_DIELECTRIC) return ST_SEED_INVALID;
        bool entering = dot(d, gv.ng) < 0.0;
        double eta = entering ? 1.0 / gv.ior : gv.ior;
        V3d nn = entering ? ns : -ns;
        double ci = -dot(d, nn);
        if (!(ci > 0.0)) return ST_SEED_INVALID;
        double s2 = eta * eta * (1.0 - ci * ci);
        if (s2 >= 1.0) return ST_SEED_INVALID;
        d = normalize(d * eta + nn * (eta * ci - std::sqrt(1.0 - s2)));
      } else {
        d = normalize(d - ns * (2.0 * dot(d, ns)));
      }
      o = pos[i - 1];
      excl = prim[i - 1];
    }
    Hit h = cast_ray(s, o, d, excl, tmin);
    if (!h.ok) return ST_SEED_INVALID;
    prim[i] = h.prim;
    pos[i] = o + d * h.t;
    if (coins) {
      bool transmit = s.mat[s.prim_obj(prim[i])] == MAT_DIELECTRIC && coins[i] < p_transmit;
      type = transmit ? (type | (1 << i)) : (type & ~(1 << i));
    }
  }
  for (int i = 0; i < n; ++i)
    if (((type >> i) & 1) && s.mat[s.prim_obj(prim[i])] != MAT_DIELECTRIC) return ST_SEED_INVALID;
  if (type_out) *type_out = type;
  return ST_CONVERGED;  // 0: valid seed
}

static bool chains_match(const Scene& s, const Chain& a, const Chain& b, double tol) {
  if (a.n != b.n || a.type != b.type) return false;
  for (int i = 0; i < a.n; ++i) {
    if (s.prim_obj(a.v[i].prim) != s.prim_obj(b.v[i].prim)) return false;
    if (norm(a.v[i].x - b.v[i].x) > tol) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Weighted EM for a 2-D Gaussian mixture per spatial cell (the guide's
// directional stand-in).  Standard EM (Dempster, Laird, Rubin 1977) with
// per-sample weights w = T <1/P> (Eq. eq_weight).
// ---------------------------------------------------------------------------
struct EMParams {
  int res, comps, iters, min_samples;
  double lo[3], hi[3];
  double reg;  // added to the covariance diagonal
};

static void em_cell(const EMParams& ep, const std::vector<int>& idx, const float* samples, int* valid, double* pi,
                    double* mu, double* cov) {
  const int K = ep.comps;
  const int m = (int)idx.size();
  *valid = 0;
  for (int j = 0; j < K; ++j) {
    pi[j] = 0.0;
    mu[2 * j] = mu[2 * j + 1] = 0.0;
    cov[3 * j] = cov[3 * j + 2] = 1.0;
    cov[3 * j + 1] = 0.0;
  }
  if (m < ep.min_samples) return;
  std::vector<double> X(2 * m), W(m);
  double Wt = 0.0;
  for (int i = 0; i < m; ++i) {
    const float* r = samples + 8 * (size_t)idx[i];
    X[2 * i] = r[3];
    X[2 * i + 1] = r[4];
    W[i] = r[5];
    Wt += W[i];
  }
  if (!(Wt > 0.0)) return;
  double mx = 0, my = 0;
  for (int i = 0; i < m; ++i) { mx += W[i] * X[2 * i]; my += W[i] * X[2 * i + 1]; }
  mx /= Wt; my /= Wt;
  double sxx = 0, sxy = 0, syy = 0;
  for (int i = 0; i < m; ++i) {
    double dx = X[2 * i] - mx, dy = X[2 * i + 1] - my;
    sxx += W[i] * dx * dx; sxy += W[i] * dx * dy; syy += W[i] * dy * dy;
  }
  sxx = sxx / Wt + ep.reg; sxy /= Wt; syy = syy / Wt + ep.reg;
  for (int j = 0; j < K; ++j) {
    int s = (2 * j + 1) * m / (2 * K);  // floor((j + 1/2) m / K)
    pi[j] = 1.0 / K;
    mu[2 * j] = X[2 * s];
    mu[2 * j + 1] = X[2 * s + 1];
    cov[3 * j] = sxx; cov[3 * j + 1] = sxy; cov[3 * j + 2] = syy;
  }
  std::vector<double> R((size_t)m * K);
  for (int it = 0; it < ep.iters; ++it) {
    // E step: responsibilities under the current parameters
    for (int i = 0; i < m; ++i) {
      double lp[8], best = -kInf;
      for (int j = 0; j < K; ++j) {
        lp[j] = -kInf;
        if (!(pi[j] > 0.0)) continue;
        double a = cov[3 * j], b = cov[3 * j + 1], c = cov[3 * j + 2];
        double det = a * c - b * b;
        double dx = X[2 * i] - mu[2 * j], dy = X[2 * i + 1] - mu[2 * j + 1];
        double q = (c * dx * dx - 2.0 * b * dx * dy + a * dy * dy) / det;
        lp[j] = std::log(pi[j]) - 0.5 * q - 0.5 * std::log(det);
        best = std::max(best, lp[j]);
      }
      double z = 0.0;
      for (int j = 0; j < K; ++j) z += lp[j] == -kInf ? 0.0 : std::exp(lp[j] - best);
      for (int j = 0; j < K; ++j) R[(size_t)i * K + j] = lp[j] == -kInf ? 0.0 : std::exp(lp[j] - best) / z;
    }
    // M step: weighted counts, means, then covariances about the new means
    for (int j = 0; j < K; ++j) {
      double Nj = 0.0, sx = 0.0, sy = 0.0;
      for (int i = 0; i < m; ++i) {
        double r = W[i] * R[(size_t)i * K + j];
        Nj += r; sx += r * X[2 * i]; sy += r * X[2 * i + 1];
      }
      if (!(Nj > 1e-8 * Wt)) { pi[j] = 0.0; continue; }
      double ux = sx / Nj, uy = sy / Nj;
      double cxx = 0.0, cxy = 0.0, cyy = 0.0;
      for (int i = 0; i < m; ++i) {
        double r = W[i] * R[(size_t)i * K + j];
        double dx = X[2 * i] - ux, dy = X[2 * i + 1] - uy;
        cxx += r * dx * dx; cxy += r * dx * dy; cyy += r * dy * dy;
      }
      pi[j] = Nj / Wt;
      mu[2 * j] = ux; mu[2 * j + 1] = uy;
      cov[3 * j] = cxx / Nj + ep.reg; cov[3 * j + 1] = cxy / Nj; cov[3 * j + 2] = cyy / Nj + ep.reg;
    }
  }
  *valid = 1;
}

// Cell of a training sample: its x_D on the guide's grid (grid_cell, FP64).
static int em_cell_index(const EMParams& ep, const float* r) {
  double p[3] = {(double)r[0], (double)r[1], (double)r[2]};
  return grid_cell(ep.lo, ep.hi, ep.res, p);
}

// ---------------------------------------------------------------------------
// Gradients of converged chains (continuity of the specular manifold by the
// implicit function theorem, Sec. 5.2), forward form in FP64:
//   C(y*, p) = 0  =>  dy/dp = -J^-1 dC/dp,
//   dx_i/dp = dx_i/dp|_y + dx_i/dy dy/dp,   dG/dp = dG/dp|_y + dG/dy dy/dp,
// for p = (x_D, x_L, theta).  Triangles use a barycentric chart whose
// vertices (and normals) follow the height-field parameters theta; spheres
// use the tangent chart of the walk.  G needs J (first derivatives of C), so
// everything is evaluated with nested dual numbers: the inner duals carry
// d/dy and d/du_L (J and B), the outer duals d/d(y, x_D, x_L, theta).
// ---------------------------------------------------------------------------
static const int ADJ_P = 32;                       // height-field parameters supported
static const int ADJ_OUT = 2 * KMAX + 6 + ADJ_P;   // outer directions
static const int ADJ_IN = 2 * KMAX + 2;            // inner directions
typedef Dual<double, ADJ_OUT> DA;
typedef Dual<DA, ADJ_IN> DB;

struct AdjVertex {
  int prim = 0;
  bool sphere = false;
  int hf = -1;                  // height field of the triangle, or -1
  double b1 = 0, b2 = 0;        // base barycentrics (triangles)
  V3d base;                     // base position (spheres)
  V3d e1, e2;                   // tangent frame (spheres)
  VGeo geo;                     // walk geometry at the base (etas, material)
};

static int hf_of_vertex(const Scene& s, int v) {
  for (size_t h = 0; h < s.hfs.size(); ++h)
    if (v >= s.hfs[h].first_vert && v < s.hfs[h].first_vert + s.hfs[h].res * s.hfs[h].res) return (int)h;
  return -1;
}

static int hf_param_base(const Scene& s, int h) {
  int b = 0;
  for (int k = 0; k < h; ++k) b += 2 * s.hfs[k].n_sines;
  return b;
}

// Vertex v of the mesh as a function of theta: height-field vertices are
// recomputed from the sine sum at their (x, y); others are the stored data.
template <class T>
static void mesh_vertex(const Scene& s, int v, const T* theta, V3<T>* P, V3<T>* N) {
  int h = hf_of_vertex(s, v);
  if (h < 0) {
    *P = lift<T>(s.P[v]);
    *N = lift<T>(s.N[v]);
    return;
  }
  const HeightField& H = s.hfs[h];
  int base = hf_param_base(s, h);
  double x = s.P[v].x, y = s.P[v].y;
  T z = T(H.z0), hx = T(0), hy = T(0);
  for (int k = 0; k < H.n_sines; ++k) {
    T amp = theta[base + 2 * k], ph = theta[base + 2 * k + 1];
    T arg = T(H.freq[k] * (std::cos(H.psi[k]) * x + std::sin(H.psi[k]) * y)) + ph;
    z = z + amp * sin(arg);
    T c = amp * T(H.freq[k]) * cos(arg);
    hx = hx + c * T(std::cos(H.psi[k]));
    hy = hy + c * T(std::sin(H.psi[k]));
  }
  *P = V3<T>(T(x), T(y), z);
  *N = normalize(V3<T>(-hx, -hy, T(1)));
}

struct AdjChain {
  int n = 0, type = 0;
  AdjVertex v[KMAX];
  double ea[KMAX], eb[KMAX];
};

// Positions and shading normals at chart coordinates y (2n) and theta.
template <class T>
static void adj_geometry(const Scene& s, const AdjChain& c, const T* y, const T* theta, V3<T>* x, V3<T>* ns,
                         V3<T>* e1) {
  for (int i = 0; i < c.n; ++i) {
    const AdjVertex& a = c.v[i];
    if (a.sphere) {
      int k = -1 - a.prim;
      V3<T> cen = lift<T>(s.sc[k]);
      V3<T> d = lift<T>(a.base - s.sc[k]) + lift<T>(a.e1) * y[2 * i] + lift<T>(a.e2) * y[2 * i + 1];
      V3<T> n = normalize(d);
      x[i] = cen + n * T(s.sr[k]);
      ns[i] = n;
      e1[i] = lift<T>(a.e1);
      continue;
    }
    V3<T> P[3], N[3];
    for (int k = 0; k < 3; ++k) mesh_vertex(s, s.tri[3 * a.prim + k], theta, &P[k], &N[k]);
    T b1 = T(a.b1) + y[2 * i], b2 = T(a.b2) + y[2 * i + 1], b0 = T(1) - b1 - b2;
    x[i] = P[0] * b0 + P[1] * b1 + P[2] * b2;
    ns[i] = normalize(N[0] * b0 + N[1] * b1 + N[2] * b2);
    e1[i] = normalize(P[1] - P[0]);
  }
}

// C and G at chart coordinates y, endpoints, theta (T = DA gives outer
// derivatives of both).
static void adj_eval(const Scene& s, const AdjChain& c, const DA* yA, const V3<DA>& xD, const V3<DA>& xL,
                     const DA* thA, const V3d& nD, DA* C, DA* G, V3<DA>* xout) {
  const int n = c.n, m = 2 * n;
  DB y[2 * KMAX], th[ADJ_P];
  for (int k = 0; k < m; ++k) y[k] = DB::var(yA[k], k);
  for (int k = 0; k < ADJ_P; ++k) th[k] = DB(thA[k], 0);
  V3d wl0;  // x_L tangent plane perpendicular to x_n - x_L (from the base values)
  V3<DB> x[KMAX + 2], ns[KMAX], e1[KMAX];
  {
    V3<DB> xx[KMAX], nn[KMAX], ee[KMAX];
    adj_geometry(s, c, y, th, xx, nn, ee);
    for (int i = 0; i < n; ++i) { x[i + 1] = xx[i]; ns[i] = nn[i]; e1[i] = ee[i]; }
  }
  V3d xn_val(val(x[n].x), val(x[n].y), val(x[n].z));
  V3d xL_val(val(xL.x), val(xL.y), val(xL.z));
  wl0 = normalize(xn_val - xL_val);
  V3d t1, t2;
  onb(wl0, &t1, &t2);
  DB u1 = DB::var(DA(0.0), ADJ_IN - 2), u2 = DB::var(DA(0.0), ADJ_IN - 1);
  x[0] = V3<DB>(DB(xD.x, 0), DB(xD.y, 0), DB(xD.z, 0));
  x[n + 1] = V3<DB>(DB(xL.x, 0), DB(xL.y, 0), DB(xL.z, 0)) + lift<DB>(t1) * u1 + lift<DB>(t2) * u2;
  DB Cb[2 * KMAX];
  for (int i = 0; i < n; ++i) {
    V3<DB> wi = normalize(x[i] - x[i + 1]), wo = normalize(x[i + 2] - x[i + 1]);
    V3<DB> h = normalize(wi * DB(c.ea[i]) + wo * DB(c.eb[i]));
    V3<DB> sv = normalize(e1[i] - ns[i] * dot(e1[i], ns[i]));
    V3<DB> tv = cross(ns[i], sv);
    Cb[2 * i] = dot(h, sv);
    Cb[2 * i + 1] = dot(h, tv);
  }
  // J (m x m) and B (m x 2) as DA; solve J X = -B in DA arithmetic
  DA J[4 * KMAX * KMAX], X[4 * KMAX];
  for (int r = 0; r < m; ++r) {
    C[r] = Cb[r].v;
    for (int k = 0; k < m; ++k) J[r * m + k] = Cb[r].d[k];
    X[2 * r] = -Cb[r].d[ADJ_IN - 2];
    X[2 * r + 1] = -Cb[r].d[ADJ_IN - 1];
  }
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(val(J[r * m + col])) > std::fabs(val(J[piv * m + col]))) piv = r;
    if (piv != col) {
      for (int k = 0; k < m; ++k) std::swap(J[piv * m + k], J[col * m + k]);
      std::swap(X[2 * piv], X[2 * col]);
      std::swap(X[2 * piv + 1], X[2 * col + 1]);
    }
    for (int r = col + 1; r < m; ++r) {
      DA f = J[r * m + col] / J[col * m + col];
      for (int k = col; k < m; ++k) J[r * m + k] = J[r * m + k] - f * J[col * m + k];
      X[2 * r] = X[2 * r] - f * X[2 * col];
      X[2 * r + 1] = X[2 * r + 1] - f * X[2 * col + 1];
    }
  }
  for (int col = m - 1; col >= 0; --col)
    for (int q = 0; q < 2; ++q) {
      DA acc = X[2 * col + q];
      for (int k = col + 1; k < m; ++k) acc = acc - J[col * m + k] * X[2 * k + q];
      X[2 * col + q] = acc / J[col * m + col];
    }
  // d x_1 / d u = (d x_1 / d y_1) X_1; the position map's inner derivatives
  V3<DA> dx[2];
  for (int q = 0; q < 2; ++q) {
    V3<DA> col0(x[1].x.d[0], x[1].y.d[0], x[1].z.d[0]);
    V3<DA> col1(x[1].x.d[1], x[1].y.d[1], x[1].z.d[1]);
    dx[q] = col0 * X[q] + col1 * X[2 + q];
  }
  V3<DA> x1(x[1].x.v, x[1].y.v, x[1].z.v);
  V3<DA> dd = x1 - xD;
  DA len = norm(dd);
  V3<DA> w = dd * (DA(1.0) / len);
  V3<DA> dw0 = (dx[0] - w * dot(w, dx[0])) * (DA(1.0) / len);
  V3<DA> dw1 = (dx[1] - w * dot(w, dx[1])) * (DA(1.0) / len);
  *G = fabs(dot(lift<DA>(nD), w)) * fabs(dot(w, cross(dw0, dw1)));
  for (int i = 0; i < n; ++i) xout[i] = V3<DA>(x[i + 1].x.v, x[i + 1].y.v, x[i + 1].z.v);
}

// Loss gradient of one converged chain: l = sum_i r_i . x_i + g G.
static bool chain_gradient(const Scene& s, const Params& p, int n, int type, const V3d& xD, const V3d& nD,
                           const V3d& xL, const int* prim, const V3d* pos, const V3d* r, double g, const double* theta,
                           double* gxD, double* gxL, double* gth) {
  (void)p;
  AdjChain c;
  c.n = n;
  c.type = type;
  V3d xs[KMAX];
  for (int i = 0; i < n; ++i) {
    AdjVertex& a = c.v[i];
    a.prim = prim[i];
    a.geo = make_geo(s, prim[i], pos[i]);
    xs[i] = pos[i];
    if (prim[i] < 0) {
      a.sphere = true;
      a.base = pos[i];
      a.e1 = a.geo.e1;
      a.e2 = a.geo.e2;
    } else {
      V3d P0, P1, P2;
      tri_verts(s, prim[i], &P0, &P1, &P2);
      V3d E1 = P1 - P0, E2 = P2 - P0, q = pos[i] - P0;
      double d11 = dot(E1, E1), d12 = dot(E1, E2), d22 = dot(E2, E2), q1 = dot(q, E1), q2 = dot(q, E2);
      double den = d11 * d22 - d12 * d12;
      a.b1 = (d22 * q1 - d12 * q2) / den;
      a.b2 = (d11 * q2 - d12 * q1) / den;
      a.hf = hf_of_vertex(s, s.tri[3 * prim[i]]);
    }
  }
  for (int i = 0; i < n; ++i) {
    V3d xp = i == 0 ? xD : xs[i - 1];
    etas(c.v[i].geo, (type >> i) & 1, normalize(xp - xs[i]), &c.ea[i], &c.eb[i]);
  }
  const int m = 2 * n;
  const int oy = 0, oD = 2 * KMAX, oL = 2 * KMAX + 3, oT = 2 * KMAX + 6;
  DA yA[2 * KMAX], thA[ADJ_P];
  for (int k = 0; k < m; ++k) yA[k] = DA::var(0.0, oy + k);
  int P = 0;
  for (size_t h = 0; h < s.hfs.size(); ++h) P += 2 * s.hfs[h].n_sines;
  if (P > ADJ_P) return false;
  for (int k = 0; k < ADJ_P; ++k) thA[k] = k < P ? DA::var(theta[k], oT + k) : DA(0.0);
  V3<DA> xDA(DA::var(xD.x, oD), DA::var(xD.y, oD + 1), DA::var(xD.z, oD + 2));
  V3<DA> xLA(DA::var(xL.x, oL), DA::var(xL.y, oL + 1), DA::var(xL.z, oL + 2));
  DA C[2 * KMAX], G;
  V3<DA> x[KMAX];
  adj_eval(s, c, yA, xDA, xLA, thA, nD, C, &G, x);
  // dy/dp = -J^-1 dC/dp for every outer parameter direction
  const int np = 6 + P;
  std::vector<double> J(m * m), R((size_t)m * np);
  for (int r = 0; r < m; ++r) {
    for (int k = 0; k < m; ++k) J[r * m + k] = C[r].d[oy + k];
    for (int q = 0; q < np; ++q) R[(size_t)r * np + q] = -C[r].d[q < 6 ? oD + q : oT + (q - 6)];
  }
  if (!dense_solve(m, J.data(), np, R.data())) return false;
  for (int q = 0; q < np; ++q) {
    int od = q < 6 ? oD + q : oT + (q - 6);
    double tot = 0.0;
    for (int i = 0; i < n; ++i) {
      double dxi[3];
      for (int a = 0; a < 3; ++a) {
        const DA& xa = x[i][a];
        double v = xa.d[od];
        for (int k = 0; k < m; ++k) v += xa.d[oy + k] * R[(size_t)k * np + q];
        dxi[a] = v;
      }
      tot += r[i].x * dxi[0] + r[i].y * dxi[1] + r[i].z * dxi[2];
    }
    double dG = G.d[od];
    for (int k = 0; k < m; ++k) dG += G.d[oy + k] * R[(size_t)k * np + q];
    tot += g * dG;
    if (q < 3) gxD[q] = tot;
    else if (q < 6) gxL[q - 3] = tot;
    else gth[q - 6] = tot;
  }
  return true;
}


// ---------------------------------------------------------------------------
// The paper's guide (Sec. 5.5, Sec. 5.6): sub-path samples (x_D, x_L, n, tau,
// w_D, w) organised in a binary tree over the 6-D configuration (x_D, x_L);
// per leaf, discrete distributions of the length and of the type (Eq. eq_div2)
// and a von Mises-Fisher mixture over w_D with one lobe per sample.
//
// Tree (Sec. 5.6): a node whose sample count exceeds c sqrt(|S|) is split at
// the middle of its longest side (lowest axis on ties).  Child overlap: a
// node holds every sample of its parent that lies inside the node's box
// dilated by eps times the node's own extent along the split axis (the
// paper copies about eps k samples across the split plane each way and drops
// samples far from a node's box; a dilation by eps of the node's size does
// both for locally even sample density).  A sample is "own" in the one leaf
// whose undilated box holds it.  Nodes are numbered breadth first, children
// left (below the middle) then right.
//
// Leaf (Sec. 5.5): P_e(n) = W_n / W and P_e(tau | n) = W_{n,tau} / W_n from
// the weights w of the leaf's samples; lobe j of group (n, tau) has mean
// direction mu_j = w_D of sample j, concentration kappa_j = sigma_j^-2, where
// sigma_j is the angle to the nearest other direction of the same group
// (floored at sigma_min; sigma_lone for a sample alone in its group), and
// weight proportional to w_j.  Groups are ordered by (n, tau), lobes by
// sample index.
// ---------------------------------------------------------------------------
struct SSample {
  double p[6];  // x_D, x_L
  V3d dir;      // w_D (unit)
  double w;
  int n, type;
};

struct STNode {
  double lo[6], hi[6];
  int depth = 0, axis = -1;
  double mid = 0.0;
  int child = -1;  // left child; right = child + 1
  std::vector<int> entries;
  std::vector<char> own;
};

struct STGroup {
  int n, type;
  double weight;
  int first, count;  // lobes [first, first + count) of the leaf
};

struct STLeaf {
  double W = 0.0, Wn[KMAX + 1] = {0};
  int own = 0;
  std::vector<STGroup> groups;
  std::vector<V3d> mu;
  std::vector<double> kappa, w;
};

struct STree {
  std::vector<STNode> nodes;
  std::vector<STLeaf> leaf;  // by node id (empty for inner nodes)
  double p0n[KMAX + 1] = {0};  // P_0(n), n = 1..8
  double alpha = 0.5;
  double p_transmit = 0.5;
  double sigma_min = 1e-3, sigma_lone = 0.1;
};

static double chord_angle(const V3d& a, const V3d& b) {
  double c = norm(a - b);
  return 2.0 * std::asin(std::min(1.0, 0.5 * c));
}

static void stree_build(const std::vector<SSample>& S, const double lo[6], const double hi[6], double eps,
                        double thr_scale, int max_depth, STree* t) {
  t->nodes.clear();
  t->leaf.clear();
  STNode root;
  for (int a = 0; a < 6; ++a) { root.lo[a] = lo[a]; root.hi[a] = hi[a]; }
  int n_valid = 0;
  for (int j = 0; j < (int)S.size(); ++j) {
    const SSample& q = S[j];
    if (!(q.w > 0.0) || q.n < 1 || q.n > KMAX) continue;
    bool in = true;
    for (int a = 0; a < 6; ++a) in = in && q.p[a] >= lo[a] && q.p[a] <= hi[a];
    if (!in) continue;
    root.entries.push_back(j);
    root.own.push_back(1);
    ++n_valid;
  }
  const double thr = thr_scale * std::sqrt((double)n_valid);
  t->nodes.push_back(root);
  for (size_t k = 0; k < t->nodes.size(); ++k) {
    if (!((double)t->nodes[k].entries.size() > thr) || t->nodes[k].depth >= max_depth) continue;
    STNode nd = t->nodes[k];
    int ax = 0;
    for (int a = 1; a < 6; ++a)
      if (nd.hi[a] - nd.lo[a] > nd.hi[ax] - nd.lo[ax]) ax = a;
    double mid = 0.5 * (nd.lo[ax] + nd.hi[ax]);
    double dil = eps * (mid - nd.lo[ax]);  // eps times the child's extent along the split axis
    STNode L, R;
    for (int a = 0; a < 6; ++a) { L.lo[a] = R.lo[a] = nd.lo[a]; L.hi[a] = R.hi[a] = nd.hi[a]; }
    L.hi[ax] = mid;
    R.lo[ax] = mid;
    L.depth = R.depth = nd.depth + 1;
    for (size_t e = 0; e < nd.entries.size(); ++e) {
      double v = S[nd.entries[e]].p[ax];
      if (v >= nd.lo[ax] - dil && v < mid + dil) {
        L.entries.push_back(nd.entries[e]);
        L.own.push_back(nd.own[e] && v < mid);
      }
      if (v >= mid - dil && v < nd.hi[ax] + dil) {
        R.entries.push_back(nd.entries[e]);
        R.own.push_back(nd.own[e] && v >= mid);
      }
    }
    t->nodes[k].axis = ax;
    t->nodes[k].mid = mid;
    t->nodes[k].child = (int)t->nodes.size();
    t->nodes.push_back(L);
    t->nodes.push_back(R);
  }
  t->leaf.assign(t->nodes.size(), STLeaf());
  for (size_t k = 0; k < t->nodes.size(); ++k) {
    const STNode& nd = t->nodes[k];
    if (nd.axis >= 0) continue;
    STLeaf& lf = t->leaf[k];
    std::vector<std::pair<std::pair<int, int>, int>> order;  // ((n, type), sample)
    for (size_t e = 0; e < nd.entries.size(); ++e) {
      const SSample& q = S[nd.entries[e]];
      lf.W += q.w;
      lf.Wn[q.n] += q.w;
      lf.own += nd.own[e] ? 1 : 0;
      order.push_back({{q.n, q.type}, nd.entries[e]});
    }
    std::sort(order.begin(), order.end());
    for (size_t i = 0; i < order.size();) {
      size_t e = i;
      while (e < order.size() && order[e].first == order[i].first) ++e;
      STGroup gr;
      gr.n = order[i].first.first;
      gr.type = order[i].first.second;
      gr.weight = 0.0;
      gr.first = (int)lf.mu.size();
      gr.count = (int)(e - i);
      for (size_t a = i; a < e; ++a) {
        const SSample& q = S[order[a].second];
        double sig = kInf;
        for (size_t b = i; b < e; ++b)
          if (b != a) sig = std::min(sig, chord_angle(q.dir, S[order[b].second].dir));
        sig = gr.count == 1 ? t->sigma_lone : std::max(sig, t->sigma_min);
        lf.mu.push_back(q.dir);
        lf.kappa.push_back(1.0 / (sig * sig));
        lf.w.push_back(q.w);
        gr.weight += q.w;
      }
      lf.groups.push_back(gr);
      i = e;
    }
  }
}

// Leaf of a configuration: descend by the split planes (undilated).
static int stree_leaf(const STree& t, const double p[6]) {
  int k = 0;
  while (t.nodes[k].axis >= 0) k = t.nodes[k].child + (p[t.nodes[k].axis] < t.nodes[k].mid ? 0 : 1);
  return k;
}

// Inverse CDF of a discrete distribution given by non-negative weights.
static int pick(const double* wts, int count, double total, double u) {
  double target = u * total, acc = 0.0;
  for (int i = 0; i < count; ++i) {
    acc += wts[i];
    if (target < acc) return i;
  }
  for (int i = count - 1; i >= 0; --i)
    if (wts[i] > 0.0) return i;
  return count - 1;
}

// vMF lobe (Eq. vMF) sampling by inversion of the cosine's distribution:
// 1 - cos theta = -log(u + (1 - u) exp(-2 kappa)) / kappa, phi uniform.
static V3d sample_vmf(const V3d& mu, double kappa, double u1, double u2) {
  double v = -std::log(u1 + (1.0 - u1) * std::exp(-2.0 * kappa)) / kappa;
  v = std::max(0.0, std::min(2.0, v));
  double ct = 1.0 - v;
  double st = std::sqrt(std::max(0.0, v * (2.0 - v)));
  V3d b1, b2;
  onb(mu, &b1, &b2);
  double ph = 2.0 * kPi * u2;
  return b1 * (st * std::cos(ph)) + b2 * (st * std::sin(ph)) + mu * ct;
}

static double vmf_pdf(const V3d& mu, double kappa, const V3d& w) {
  // kappa / (4 pi sinh kappa) exp(kappa mu.w), written with exp(kappa (mu.w - 1)) for large kappa
  return kappa / (2.0 * kPi * (1.0 - std::exp(-2.0 * kappa))) * std::exp(kappa * (dot(mu, w) - 1.0));
}

// P(n | x_D, x_L) of the defensive one-sample mixture (Sec. 5.5).
static double stree_pn(const STree& t, const STLeaf& lf, int n) {
  if (!(lf.W > 0.0)) return t.p0n[n];
  return t.alpha * t.p0n[n] + (1.0 - t.alpha) * lf.Wn[n] / lf.W;
}

// One seed from the paper's guide: the length n (unless given, n_fixed > 0)
// from alpha P_0(n) + (1 - alpha) P_e(n), then (w_D, tau) from
// alpha p_0 + (1 - alpha) p_e (Sec. 5.5, defensive sampling); p_0 takes x_1
// by the obj1 mode and decides tau by ray tracing, p_e picks tau from
// P_e(tau | n), a lobe by weight and w_D from the lobe.  Random numbers: block
// (chain, trial, 0) for the choices, block 1 for p_0's point, block 2 for the
// vertex coins.  Returns the status and n, tau, P(n).
static int8_t stree_sample(const Scene& s, const STree& t, const Params& p, int n_fixed, int obj1, const V3d& xD,
                           const V3d& nD, const V3d& xL, uint64_t seed, uint64_t chain, uint64_t trial, int* n_out,
                           int* type_out, double* pn_out, int* prim, V3d* pos) {
  if (!finite3(xD) || !finite3(xL)) return ST_BAD_INPUT;
  double q[6] = {xD.x, xD.y, xD.z, xL.x, xL.y, xL.z};
  const STLeaf& lf = t.leaf[stree_leaf(t, q)];
  Uniforms U = draw(seed, chain, trial, 0);
  int n = n_fixed;
  if (n < 1) {
    double pe[KMAX];
    for (int k = 1; k <= KMAX; ++k) pe[k - 1] = lf.W > 0.0 ? lf.Wn[k] : 0.0;
    bool prior = !(lf.W > 0.0) || U.u[0] < t.alpha;
    n = 1 + (prior ? pick(t.p0n + 1, KMAX, 1.0, U.u[1]) : pick(pe, KMAX, lf.W, U.u[1]));
  }
  if (n < 1 || n > KMAX) return ST_BAD_INPUT;
  *n_out = n;
  *pn_out = stree_pn(t, lf, n);
  // groups of this length
  std::vector<double> gw;
  std::vector<int> gi;
  double Wn = 0.0;
  for (size_t g = 0; g < lf.groups.size(); ++g)
    if (lf.groups[g].n == n) { gw.push_back(lf.groups[g].weight); gi.push_back((int)g); Wn += lf.groups[g].weight; }
  bool prior = !(Wn > 0.0) || U.u[2] < t.alpha;
  if (prior) {
    Uniforms V = draw(seed, chain, trial, 1), Cn = draw(seed, chain, trial, 2);
    V3d pt;
    if (!sample_p0_point(s, p, obj1, xD, nD, V.u[1], V.u[2], V.u[3], &pt)) return ST_SEED_INVALID;
    return deduce_chain(s, p, n, 0, Cn.u, t.p_transmit, xD, pt, prim, pos, type_out);
  }
  const STGroup& gr = lf.groups[gi[pick(gw.data(), (int)gw.size(), Wn, U.u[3])]];
  int j = gr.first + pick(&lf.w[gr.first], gr.count, gr.weight, U.u[4]);
  V3d w = sample_vmf(lf.mu[j], lf.kappa[j], U.u[5], U.u[6]);
  *type_out = gr.type;
  return deduce_chain(s, p, n, gr.type, nullptr, 0.0, xD, xD + w, prim, pos, nullptr);
}

// ---------------------------------------------------------------------------
// threads
// ---------------------------------------------------------------------------
template <class F>
static void parallel_for(int n, int nthreads, F fn) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  nthreads = std::max(1, std::min(nthreads, n));
  if (nthreads == 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int i0 = next.fetch_add(16);
        if (i0 >= n) break;
        for (int i = i0; i < std::min(n, i0 + 16); ++i) fn(i);
      }
    });
  for (auto& th : pool) th.join();
}

static V3d get3d(const double* a, int n, int i) { return V3d(a[i], a[n + i], a[2 * n + i]); }

}  // namespace oracle

using namespace oracle;

// ---------------------------------------------------------------------------
// C interface (ctypes)
// ---------------------------------------------------------------------------
static void build_bvh(Scene* s) {
  int nt = s->ntri();
  s->nodes.clear();
  s->order.clear();
  if (nt == 0) return;
  std::vector<V3d> cen(nt);
  for (int t = 0; t < nt; ++t) {
    V3d a, b, c;
    tri_verts(*s, t, &a, &b, &c);
    cen[t] = (a + b + c) * (1.0 / 3.0);
  }
  s->order.resize(nt);
  for (int t = 0; t < nt; ++t) s->order[t] = t;
  build_node(*s, cen, 0, nt);
}

extern "C" {

struct orc_params {
  int32_t max_iter;
  double tol_vertex, tol_residual, scale, tmin_rel, match_rel, polish_tol, cone_cos;
};

void* orc_scene_create(int nv, const float* verts, const float* normals, int nt, const int32_t* tris,
                       const int32_t* tri_obj, int nobj, const int32_t* mat, const float* ior, int ns,
                       const float* spheres, const int32_t* sphere_obj, double scale) {
  Scene* s = new Scene();
  s->P.resize(nv);
  s->N.resize(nv);
  for (int i = 0; i < nv; ++i) {
    s->P[i] = V3d(verts[3 * i], verts[3 * i + 1], verts[3 * i + 2]);
    s->N[i] = normalize(V3d(normals[3 * i], normals[3 * i + 1], normals[3 * i + 2]));
  }
  s->tri.assign(tris, tris + 3 * nt);
  s->tri_obj.assign(tri_obj, tri_obj + nt);
  s->mat.assign(mat, mat + nobj);
  s->ior.resize(nobj);
  for (int i = 0; i < nobj; ++i) s->ior[i] = ior[i];
  for (int k = 0; k < ns; ++k) {
    s->sc.push_back(V3d(spheres[4 * k], spheres[4 * k + 1], spheres[4 * k + 2]));
    s->sr.push_back(spheres[4 * k + 3]);
    s->sobj.push_back(sphere_obj[k]);
  }
  s->scale = scale;
  build_bvh(s);
  // area CDFs per object and over all objects; xy bounds per object
  s->cdf.assign(nobj + 1, {});
  s->cdf_prim.assign(nobj + 1, {});
  s->obj_lo_x.assign(nobj, kInf); s->obj_lo_y.assign(nobj, kInf);
  s->obj_hi_x.assign(nobj, -kInf); s->obj_hi_y.assign(nobj, -kInf);
  s->zmax = -kInf;
  auto add = [&](int key, int prim, double area) {
    double prev = s->cdf[key].empty() ? 0.0 : s->cdf[key].back();
    s->cdf[key].push_back(prev + area);
    s->cdf_prim[key].push_back(prim);
  };
  for (int t = 0; t < nt; ++t) {
    V3d a, b, c;
    tri_verts(*s, t, &a, &b, &c);
    double area = 0.5 * norm(cross(b - a, c - a));
    add(s->tri_obj[t], t, area);
    add(nobj, t, area);
    int o = s->tri_obj[t];
    for (const V3d* v : {&a, &b, &c}) {
      s->obj_lo_x[o] = std::min(s->obj_lo_x[o], v->x); s->obj_hi_x[o] = std::max(s->obj_hi_x[o], v->x);
      s->obj_lo_y[o] = std::min(s->obj_lo_y[o], v->y); s->obj_hi_y[o] = std::max(s->obj_hi_y[o], v->y);
      s->zmax = std::max(s->zmax, v->z);
    }
  }
  for (int k = 0; k < ns; ++k) {
    double area = 4.0 * kPi * s->sr[k] * s->sr[k];
    add(s->sobj[k], -1 - k, area);
    add(nobj, -1 - k, area);
    int o = s->sobj[k];
    s->obj_lo_x[o] = std::min(s->obj_lo_x[o], s->sc[k].x - s->sr[k]);
    s->obj_hi_x[o] = std::max(s->obj_hi_x[o], s->sc[k].x + s->sr[k]);
    s->obj_lo_y[o] = std::min(s->obj_lo_y[o], s->sc[k].y - s->sr[k]);
    s->obj_hi_y[o] = std::max(s->obj_hi_y[o], s->sc[k].y + s->sr[k]);
    s->zmax = std::max(s->zmax, s->sc[k].z + s->sr[k]);
  }
  return s;
}

void orc_scene_destroy(void* s) { delete (Scene*)s; }

int orc_scene_set_heightfield(void* sp, int obj, int res, int first_vert, int first_tri, double x0, double x1,
                              double y0, double y1, double z0, int n_sines, const double* amp, const double* freq,
                              const double* psi, const double* phase) {
  Scene* s = (Scene*)sp;
  if (n_sines > 8) return -1;
  HeightField h;
  h.obj = obj; h.res = res; h.first_vert = first_vert; h.first_tri = first_tri; h.n_sines = n_sines;
  h.x0 = x0; h.x1 = x1; h.y0 = y0; h.y1 = y1; h.z0 = z0;
  for (int k = 0; k < n_sines; ++k) { h.amp[k] = amp[k]; h.freq[k] = freq[k]; h.psi[k] = psi[k]; h.phase[k] = phase[k]; }
  s->hfs.push_back(h);
  return 0;
}

void orc_philox(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k1, uint64_t* out) {
  uint64_t ctr[4] = {c0, c1, c2, c3};
  uint64_t key[2] = {seed, k1};
  philox4x64_10(ctr, key, out);
}

void orc_uniforms(uint64_t seed, uint64_t chain, uint64_t trial, uint64_t attempt, double* out) {
  Uniforms U = draw(seed, chain, trial, attempt);
  for (int j = 0; j < 8; ++j) out[j] = U.u[j];
}

uint64_t orc_solution_id(int n, int type, const int32_t* prim) { return solution_id(n, type, prim); }

void orc_raycast(void* sp, int n, const double* o, const double* d, const int32_t* exclude, double tmin, int brute,
                 int32_t* prim, double* t, int nthreads) {
  const Scene& s = *(Scene*)sp;
  parallel_for(n, nthreads, [&](int i) {
    Hit h = cast_ray(s, V3d(o[3 * i], o[3 * i + 1], o[3 * i + 2]), V3d(d[3 * i], d[3 * i + 1], d[3 * i + 2]),
                     exclude[i], tmin, brute != 0);
    prim[i] = h.ok ? h.prim : INT32_MIN;
    t[i] = h.ok ? h.t : kInf;
  });
}

// Residual and dense Jacobian of one chain at given primitives / positions.
int orc_constraint(void* sp, int n, int type, const double* xD, const double* xL, const int32_t* prim,
                   const double* pos, double* C, double* J, double* frames, const double* off) {
  const Scene& s = *(Scene*)sp;
  Chain c;
  V3d p[KMAX];
  for (int i = 0; i < n; ++i) p[i] = V3d(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
  if (!load_chain(s, n, type, V3d(xD[0], xD[1], xD[2]), V3d(xL[0], xL[1], xL[2]), prim, p, &c)) return -1;
  if (off) {  // glossy offsets (o_s, o_t) per vertex
    c.glossy = true;
    for (int i = 0; i < n; ++i) { c.off[i][0] = off[2 * i]; c.off[i][1] = off[2 * i + 1]; }
  }
  jacobian(c, V3d(), V3d(), C, J, nullptr);
  if (frames)
    for (int i = 0; i < n; ++i) {
      frames[6 * i + 0] = c.v[i].e1.x; frames[6 * i + 1] = c.v[i].e1.y; frames[6 * i + 2] = c.v[i].e1.z;
      frames[6 * i + 3] = c.v[i].e2.x; frames[6 * i + 4] = c.v[i].e2.y; frames[6 * i + 5] = c.v[i].e2.z;
    }
  return 0;
}

// Positions of a chain moved by local offsets y (2n) -- for finite differences.
int orc_offset_positions(void* sp, int n, const int32_t* prim, const double* pos, const double* y, double* out) {
  const Scene& s = *(Scene*)sp;
  for (int i = 0; i < n; ++i) {
    VGeo g = make_geo(s, prim[i], V3d(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]));
    V3d x = geo_pos<double>(g, y[2 * i], y[2 * i + 1]);
    out[3 * i] = x.x; out[3 * i + 1] = x.y; out[3 * i + 2] = x.z;
  }
  return 0;
}

static const Guide* make_guide_view(const int32_t* gi, const double* gd, Guide* g) {
  if (!gi) return nullptr;
  // gi: res, comps, target_obj, valid[cells];  gd: lo[3], hi[3], pi, mu, chol
  g->res = gi[0];
  g->comps = gi[1];
  g->target_obj = gi[2];
  int cells = g->res * g->res * g->res;
  g->valid.assign(gi + 3, gi + 3 + cells);
  for (int a = 0; a < 3; ++a) { g->lo[a] = gd[a]; g->hi[a] = gd[3 + a]; }
  const double* q = gd + 6;
  g->pi.assign(q, q + (size_t)cells * g->comps); q += (size_t)cells * g->comps;
  g->mu.assign(q, q + (size_t)cells * g->comps * 2); q += (size_t)cells * g->comps * 2;
  g->chol.assign(q, q + (size_t)cells * g->comps * 3);
  return g;
}

static Params to_params(const orc_params* p) {
  Params q;
  q.max_iter = p->max_iter; q.tol_vertex = p->tol_vertex; q.tol_residual = p->tol_residual;
  q.scale = p->scale; q.tmin_rel = p->tmin_rel; q.match_rel = p->match_rel; q.polish_tol = p->polish_tol;
  q.cone_cos = p->cone_cos;
  return q;
}

// offsets of glossy chains, [2][K][N] (nullable): vertex i of chain c has
// (o_s, o_t) = (off[(0 K + i) N + c], off[(1 K + i) N + c])
static void chain_offsets(const double* off, int N, int c, double* o) {
  for (int i = 0; i < KMAX; ++i) {
    o[2 * i] = off[((size_t)0 * KMAX + i) * N + c];
    o[2 * i + 1] = off[((size_t)1 * KMAX + i) * N + c];
  }
}

void orc_sample_seeds(void* sp, const int32_t* gi, const double* gd, const orc_params* pp, int N, const double* xD,
                      const double* nD, const uint8_t* len, const uint8_t* type, const int32_t* obj1, uint64_t seed, uint64_t trial,
                      double alpha, int32_t* prim_out, double* pos_out, int8_t* status, int nthreads,
                      const double* off) {
  const Scene& s = *(Scene*)sp;
  Guide gstore;
  const Guide* g = make_guide_view(gi, gd, &gstore);
  Params p = to_params(pp);
  parallel_for(N, nthreads, [&](int c) {
    int prim[KMAX];
    V3d pos[KMAX];
    for (int i = 0; i < KMAX; ++i) { prim[i] = INT32_MIN; pos[i] = V3d(); }
    double o[2 * KMAX];
    if (off) chain_offsets(off, N, c, o);
    int8_t st = sample_seed(s, g, p, len[c], type[c], obj1[c], get3d(xD, N, c), get3d(nD, N, c), seed,
                            (uint64_t)c, trial, alpha, prim, pos, off ? o : nullptr);
    status[c] = st;
    for (int i = 0; i < KMAX; ++i) {
      prim_out[(size_t)i * N + c] = st == 0 ? prim[i] : INT32_MIN;
      for (int a = 0; a < 3; ++a) pos_out[((size_t)a * KMAX + i) * N + c] = st == 0 ? pos[i][a] : 0.0;
    }
  });
}

void orc_walk(void* sp, const orc_params* pp, int N, const double* xD, const double* nD, const double* xL,
              const uint8_t* len, const uint8_t* type, const int32_t* seed_prim, const float* seed_pos,
              const int8_t* seed_status, int do_polish, int32_t* prim_out, double* pos_out, int8_t* status,
              int32_t* iters, uint64_t* sol, double* G, double* kappa, double* resid, int8_t* polished,
              int nthreads, const double* off) {
  const Scene& s = *(Scene*)sp;
  Params p = to_params(pp);
  parallel_for(N, nthreads, [&](int c) {
    int n = len[c];
    int prim[KMAX];
    V3d pos[KMAX];
    for (int i = 0; i < KMAX && i < n; ++i) {
      prim[i] = seed_prim[(size_t)i * N + c];
      pos[i] = V3d(seed_pos[((size_t)0 * KMAX + i) * N + c], seed_pos[((size_t)1 * KMAX + i) * N + c],
                   seed_pos[((size_t)2 * KMAX + i) * N + c]);
    }
    WalkResult r;
    double o[2 * KMAX];
    if (off) chain_offsets(off, N, c, o);
    if (seed_status && seed_status[c] != 0) r.status = ST_SEED_INVALID;
    else walk_chain(s, p, n, type[c], get3d(xD, N, c), get3d(nD, N, c), get3d(xL, N, c), prim, pos,
                    do_polish != 0, &r, off ? o : nullptr);
    status[c] = r.status;
    iters[c] = r.iters;
    sol[c] = r.status == ST_CONVERGED ? r.sol : 0;
    G[c] = r.G;
    kappa[c] = r.kappa;
    resid[c] = r.residual;
    polished[c] = r.polished ? 1 : 0;
    for (int i = 0; i < KMAX; ++i) {
      bool have = i < n && i < r.chain.n && r.status != ST_BAD_INPUT && r.status != ST_SEED_INVALID;
      prim_out[(size_t)i * N + c] = have ? r.chain.v[i].prim : INT32_MIN;
      for (int a = 0; a < 3; ++a) pos_out[((size_t)a * KMAX + i) * N + c] = have ? r.chain.v[i].x[a] : 0.0;
    }
  });
}

// Admissibility of externally computed chains (e.g. FP32 results): each
// given vertex is first put exactly onto its primitive (radial projection on
// a sphere, orthogonal projection on a triangle's plane: rounded coordinates
// lie slightly off the surface, and the walk's steps assume a point on it),
// then the oracle's FP64 Newton polish runs within the scene, then the side
// conditions and the shadow ray of the polished chain are tested.  Per
// chain: ok (the chain could be loaded), the residual max-norm after the
// polish, the largest vertex displacement of the polish, side, visible, and
// whether the polish kept every primitive id.
void orc_validate(void* sp, const orc_params* pp, int N, const double* xD, const double* xL, const uint8_t* len,
                  const uint8_t* type, const int32_t* prim_in, const double* pos_in, int8_t* ok, double* resid,
                  double* moved, int8_t* side, int8_t* visible, int8_t* same_prims, int nthreads,
                  const double* off) {
  const Scene& s = *(Scene*)sp;
  Params p = to_params(pp);
  parallel_for(N, nthreads, [&](int c) {
    int n = len[c];
    ok[c] = 0; resid[c] = kInf; moved[c] = kInf; side[c] = 0; visible[c] = 0; same_prims[c] = 0;
    if (n < 1 || n > KMAX) return;
    int prim[KMAX];
    V3d pos[KMAX];
    for (int i = 0; i < n; ++i) {
      prim[i] = prim_in[(size_t)i * N + c];
      pos[i] = V3d(pos_in[((size_t)0 * KMAX + i) * N + c], pos_in[((size_t)1 * KMAX + i) * N + c],
                   pos_in[((size_t)2 * KMAX + i) * N + c]);
      if (prim[i] >= s.ntri() || (prim[i] < 0 && -1 - prim[i] >= (int)s.sr.size())) return;
      if (prim[i] < 0) {
        int k = -1 - prim[i];
        pos[i] = s.sc[k] + normalize(pos[i] - s.sc[k]) * s.sr[k];
      } else {
        V3d a, b, cc;
        tri_verts(s, prim[i], &a, &b, &cc);
        V3d ng = normalize(cross(b - a, cc - a));
        pos[i] = pos[i] - ng * dot(pos[i] - a, ng);
      }
    }
    WalkResult r;
    if (!load_chain(s, n, type[c], get3d(xD, N, c), get3d(xL, N, c), prim, pos, &r.chain)) return;
    if (off) {
      double o[2 * KMAX];
      chain_offsets(off, N, c, o);
      r.chain.glossy = true;
      for (int i = 0; i < n; ++i) { r.chain.off[i][0] = o[2 * i]; r.chain.off[i][1] = o[2 * i + 1]; }
    }
    ok[c] = 1;
    polish(s, p, &r);
    resid[c] = r.residual;
    double mv = 0.0;
    bool same = true;
    for (int i = 0; i < n; ++i) {
      mv = std::max(mv, norm(r.chain.v[i].x - pos[i]));
      same = same && r.chain.v[i].prim == prim[i];
    }
    moved[c] = mv;
    same_prims[c] = same ? 1 : 0;
    side[c] = side_ok(r.chain) ? 1 : 0;
    visible[c] = visible_to_light(s, p, r.chain) ? 1 : 0;
  });
}

// Reciprocal probability by repeated independent trials (Sec. 5.8): for a
// converged target, draw seeds from the same distribution with fresh random
// numbers (trial counter 1 + r M + k - 1) and walk until the same chain is
// found again; K trials give <1/P(chain | n)> = K.  With a cap of M trials the
// estimate is K = M when no trial matched (flagged).  P(n) = 1 (n is given).
void orc_inv_prob(void* sp, const int32_t* gi, const double* gd, const orc_params* pp, int N, const double* xD,
                  const double* nD, const double* xL, const uint8_t* len, const uint8_t* type, const int32_t* obj1,
                  const int32_t* tgt_prim, const double* tgt_pos, const int8_t* tgt_status, int max_trials,
                  int repeats, uint64_t seed, double alpha, int32_t* trials, double* inv_prob, int8_t* truncated,
                  int nthreads, const double* off) {
  const Scene& s = *(Scene*)sp;
  Guide gstore;
  const Guide* g = make_guide_view(gi, gd, &gstore);
  Params p = to_params(pp);
  parallel_for(N, nthreads, [&](int c) {
    trials[c] = 0;
    inv_prob[c] = 0.0;
    truncated[c] = 0;
    if (tgt_status[c] != ST_CONVERGED || repeats < 1 || max_trials < 1) return;
    int n = len[c];
    V3d xd = get3d(xD, N, c), xl = get3d(xL, N, c), nd = get3d(nD, N, c);
    Chain target;
    target.n = n;
    target.type = type[c];
    target.xD = xd;
    target.xL = xl;
    for (int i = 0; i < n; ++i) {
      V3d x(tgt_pos[((size_t)0 * KMAX + i) * N + c], tgt_pos[((size_t)1 * KMAX + i) * N + c],
            tgt_pos[((size_t)2 * KMAX + i) * N + c]);
      target.v[i] = make_geo(s, tgt_prim[(size_t)i * N + c], x);
    }
    double o[2 * KMAX];
    if (off) chain_offsets(off, N, c, o);
    int total = 0;
    for (int r = 0; r < repeats; ++r) {
      int K = max_trials;
      bool found = false;
      for (int k = 1; k <= max_trials && !found; ++k) {
        uint64_t trial = 1 + (uint64_t)r * max_trials + (uint64_t)(k - 1);
        int prim[KMAX];
        V3d pos[KMAX];
        if (sample_seed(s, g, p, n, type[c], obj1[c], xd, nd, seed, (uint64_t)c, trial, alpha, prim, pos,
                        off ? o : nullptr) != 0)
          continue;
        Chain start;
        if (!load_chain(s, n, type[c], xd, xl, prim, pos, &start)) continue;
        if (off) {
          start.glossy = true;
          for (int i = 0; i < n; ++i) { start.off[i][0] = o[2 * i]; start.off[i][1] = o[2 * i + 1]; }
        }
        WalkResult w;
        walk_core(s, p, start, &w);
        bool conv = w.status == ST_CONVERGED || w.status == ST_STALLED;
        if (conv && chains_match(s, w.chain, target, p.match_rel * p.scale)) {
          K = k;
          found = true;
        }
      }
      if (!found) truncated[c] = 1;
      total += K;
    }
    trials[c] = total;
    inv_prob[c] = (double)total / repeats;
  });
}

void orc_fit_guide(int n_samples, const float* samples, int res, int comps, int iters, int min_samples,
                   const double* lo, const double* hi, double reg, int32_t* valid, double* pi, double* mu,
                   double* cov, int32_t* count, int nthreads) {
  EMParams ep;
  ep.res = res; ep.comps = comps; ep.iters = iters; ep.min_samples = min_samples; ep.reg = reg;
  for (int a = 0; a < 3; ++a) { ep.lo[a] = lo[a]; ep.hi[a] = hi[a]; }
  int cells = res * res * res;
  std::vector<std::vector<int>> members(cells);
  for (int i = 0; i < n_samples; ++i) {
    const float* r = samples + 8 * (size_t)i;
    if (!(r[5] > 0.0f) || !std::isfinite(r[3]) || !std::isfinite(r[4]) || !std::isfinite(r[5])) continue;
    int cidx = em_cell_index(ep, r);
    if (cidx >= 0) members[cidx].push_back(i);
  }
  parallel_for(cells, nthreads, [&](int c) {
    count[c] = (int)members[c].size();
    em_cell(ep, members[c], samples, &valid[c], pi + (size_t)c * comps, mu + (size_t)c * comps * 2,
            cov + (size_t)c * comps * 3);
  });
}

// Replace the height-field parameters theta [2 * sum n_sines] (amplitude,
// phase per sine): vertex positions and normals of every height field are
// recomputed from the sine sum in FP64 and the BVH is rebuilt.
int orc_scene_set_theta(void* sp, int n, const double* theta) {
  Scene* s = (Scene*)sp;
  int P = 0;
  for (const HeightField& h : s->hfs) P += 2 * h.n_sines;
  if (n != P || P > ADJ_P) return -1;
  for (size_t h = 0; h < s->hfs.size(); ++h) {
    HeightField& H = s->hfs[h];
    int base = hf_param_base(*s, (int)h);
    for (int k = 0; k < H.n_sines; ++k) { H.amp[k] = theta[base + 2 * k]; H.phase[k] = theta[base + 2 * k + 1]; }
    for (int v = H.first_vert; v < H.first_vert + H.res * H.res; ++v) {
      V3d P, N;
      mesh_vertex<double>(*s, v, theta, &P, &N);
      s->P[v] = P;
      s->N[v] = N;
    }
  }
  build_bvh(s);
  return 0;
}

// Per-chain loss gradients (FP64 forward IFT with nested duals).  theta is
// the scene's current height-field parameters [P]; grad_theta is [N][P].
void orc_adjoint(void* sp, const orc_params* pp, int N, const double* xD, const double* nD, const double* xL,
                 const uint8_t* len, const uint8_t* type, const int32_t* prim, const double* pos, const int8_t* status,
                 const double* grad_pos, const double* grad_G, const double* theta, double* grad_xD, double* grad_xL,
                 double* grad_theta, int8_t* ok, int nthreads) {
  const Scene& s = *(Scene*)sp;
  Params p = to_params(pp);
  int P = 0;
  for (size_t h = 0; h < s.hfs.size(); ++h) P += 2 * s.hfs[h].n_sines;
  parallel_for(N, nthreads, [&](int c) {
    for (int a = 0; a < 3; ++a) { grad_xD[(size_t)a * N + c] = 0.0; grad_xL[(size_t)a * N + c] = 0.0; }
    for (int k = 0; k < P; ++k) grad_theta[(size_t)c * P + k] = 0.0;
    ok[c] = 0;
    int n = len[c];
    if (status[c] != ST_CONVERGED || n < 1 || n > KMAX) return;
    int pr[KMAX];
    V3d x[KMAX], r[KMAX];
    for (int i = 0; i < n; ++i) {
      pr[i] = prim[(size_t)i * N + c];
      x[i] = V3d(pos[((size_t)0 * KMAX + i) * N + c], pos[((size_t)1 * KMAX + i) * N + c],
                 pos[((size_t)2 * KMAX + i) * N + c]);
      r[i] = grad_pos ? V3d(grad_pos[((size_t)0 * KMAX + i) * N + c], grad_pos[((size_t)1 * KMAX + i) * N + c],
                            grad_pos[((size_t)2 * KMAX + i) * N + c])
                      : V3d();
    }
    double gxD[3], gxL[3], gth[ADJ_P];
    bool good = chain_gradient(s, p, n, type[c], get3d(xD, N, c), get3d(nD, N, c), get3d(xL, N, c), pr, x, r,
                               grad_G ? grad_G[c] : 0.0, theta, gxD, gxL, gth);
    if (!good) return;
    ok[c] = 1;
    for (int a = 0; a < 3; ++a) { grad_xD[(size_t)a * N + c] = gxD[a]; grad_xL[(size_t)a * N + c] = gxL[a]; }
    for (int k = 0; k < P; ++k) grad_theta[(size_t)c * P + k] = gth[k];
  });
}


// Offset normals of glossy chains (Sec. 5.7) drawn from the GGX
// (Trowbridge-Reitz) distribution of microfacet normals, D(m) cos theta_m
// (Walter, Marschner, Li, Torrance, EGSR 2007): tan^2 theta_m = a^2 u / (1 -
// u), phi = 2 pi v; (o_s, o_t) = sin theta_m (cos phi, sin phi).  Vertex i of
// chain c uses uniforms 2 (i mod 4) and 2 (i mod 4) + 1 of the Philox block
// (c, trial, 16 + i / 4).  Layout [2][K][N].
void orc_sample_offsets(int N, uint64_t seed, uint64_t trial, double roughness, double* off) {
  for (int c = 0; c < N; ++c)
    for (int i = 0; i < KMAX; ++i) {
      Uniforms U = draw(seed, (uint64_t)c, trial, 16 + i / 4);
      double u = U.u[2 * (i % 4)], v = U.u[2 * (i % 4) + 1];
      double t2 = roughness * roughness * u / (1.0 - u);
      double st = std::sqrt(t2 / (1.0 + t2));
      off[((size_t)0 * KMAX + i) * N + c] = st * std::cos(2.0 * kPi * v);
      off[((size_t)1 * KMAX + i) * N + c] = st * std::sin(2.0 * kPi * v);
    }
}

// ---------------------------------------------------------------------------
// The paper's guide: tree, leaf distributions, sampling and trials.
// Sample records: float [N][16] = x_D (3), x_L (3), w_D (3), w, n, tau, 0 x 4.
// ---------------------------------------------------------------------------
void* orc_stree_build(int N, const float* rec, const double* lo, const double* hi, double eps, double thr_scale,
                      int max_depth, double sigma_min, double sigma_lone) {
  std::vector<SSample> S(N);
  for (int j = 0; j < N; ++j) {
    const float* r = rec + 16 * (size_t)j;
    for (int a = 0; a < 6; ++a) S[j].p[a] = r[a];
    S[j].dir = normalize(V3d(r[6], r[7], r[8]));
    S[j].w = std::isfinite(r[9]) ? r[9] : 0.0;
    S[j].n = (int)r[10];
    S[j].type = (int)r[11];
    for (int a = 0; a < 12; ++a)
      if (!std::isfinite(r[a])) S[j].w = 0.0;
    if ((float)S[j].n != r[10]) S[j].w = 0.0;
  }
  STree* t = new STree();
  t->sigma_min = sigma_min;
  t->sigma_lone = sigma_lone;
  stree_build(S, lo, hi, eps, thr_scale, max_depth, t);
  return t;
}

void orc_stree_destroy(void* h) { delete (STree*)h; }

void orc_stree_set_prior(void* h, const double* p0n, double alpha, double p_transmit) {
  STree* t = (STree*)h;
  double tot = 0.0;
  for (int k = 0; k < KMAX; ++k) tot += p0n[k];
  for (int k = 1; k <= KMAX; ++k) t->p0n[k] = tot > 0.0 ? p0n[k - 1] / tot : 0.0;
  t->alpha = alpha;
  t->p_transmit = p_transmit;
}

int orc_stree_n_nodes(void* h) { return (int)((STree*)h)->nodes.size(); }
int orc_stree_n_lobes(void* h) {
  int n = 0;
  for (const STLeaf& l : ((STree*)h)->leaf) n += (int)l.mu.size();
  return n;
}

// per node: axis (-1 leaf), mid, child, depth, box lo/hi [6], entries, own,
// leaf weight W and W_n [8], number of groups, first lobe (leaf-major order)
void orc_stree_nodes(void* h, int32_t* axis, double* mid, int32_t* child, int32_t* depth, double* lo, double* hi,
                     int32_t* n_entries, int32_t* n_own, double* W, double* Wn, int32_t* n_groups, int32_t* lobe0) {
  const STree& t = *(STree*)h;
  int lobes = 0;
  for (size_t k = 0; k < t.nodes.size(); ++k) {
    const STNode& nd = t.nodes[k];
    axis[k] = nd.axis; mid[k] = nd.mid; child[k] = nd.child; depth[k] = nd.depth;
    for (int a = 0; a < 6; ++a) { lo[6 * k + a] = nd.lo[a]; hi[6 * k + a] = nd.hi[a]; }
    n_entries[k] = (int)nd.entries.size();
    int own = 0;
    for (char o : nd.own) own += o;
    n_own[k] = own;
    const STLeaf& lf = t.leaf[k];
    W[k] = lf.W;
    for (int q = 0; q < KMAX; ++q) Wn[KMAX * k + q] = lf.Wn[q + 1];
    n_groups[k] = (int)lf.groups.size();
    lobe0[k] = lobes;
    lobes += (int)lf.mu.size();
  }
}

// the entries (sample ids) and own flags of one node
int orc_stree_node_entries(void* h, int k, int32_t* ids, int8_t* own) {
  const STNode& nd = ((STree*)h)->nodes[k];
  for (size_t e = 0; e < nd.entries.size(); ++e) { ids[e] = nd.entries[e]; own[e] = nd.own[e]; }
  return (int)nd.entries.size();
}

// lobes in leaf-major, group, sample order: mean direction, kappa, weight,
// and the group's (n, type)
void orc_stree_lobes(void* h, double* mu, double* kappa, double* w, int32_t* n, int32_t* type) {
  const STree& t = *(STree*)h;
  size_t q = 0;
  for (const STLeaf& lf : t.leaf)
    for (const STGroup& g : lf.groups)
      for (int j = g.first; j < g.first + g.count; ++j, ++q) {
        mu[3 * q] = lf.mu[j].x; mu[3 * q + 1] = lf.mu[j].y; mu[3 * q + 2] = lf.mu[j].z;
        kappa[q] = lf.kappa[j]; w[q] = lf.w[j]; n[q] = g.n; type[q] = g.type;
      }
}

void orc_stree_lookup(void* h, int N, const double* xD, const double* xL, int32_t* leaf) {
  const STree& t = *(STree*)h;
  for (int c = 0; c < N; ++c) {
    double q[6] = {xD[c], xD[N + c], xD[2 * N + c], xL[c], xL[N + c], xL[2 * N + c]};
    leaf[c] = stree_leaf(t, q);
  }
}

double orc_vmf_pdf(const double* mu, double kappa, const double* w) {
  return vmf_pdf(V3d(mu[0], mu[1], mu[2]), kappa, V3d(w[0], w[1], w[2]));
}
void orc_vmf_sample(const double* mu, double kappa, int N, const double* u, double* out) {
  V3d m(mu[0], mu[1], mu[2]);
  for (int i = 0; i < N; ++i) {
    V3d w = sample_vmf(m, kappa, u[2 * i], u[2 * i + 1]);
    out[3 * i] = w.x; out[3 * i + 1] = w.y; out[3 * i + 2] = w.z;
  }
}

// Seeds from the paper's guide: n_fixed[c] > 0 keeps that length, 0 samples
// it.  Outputs n, type, P(n), the seed chain and the status.
void orc_stree_sample_seeds(void* sp, void* h, const orc_params* pp, int N, const double* xD, const double* nD,
                            const double* xL, const uint8_t* n_fixed, const int32_t* obj1, uint64_t seed,
                            uint64_t trial, uint8_t* n_out, uint8_t* type_out, double* pn_out, int32_t* prim_out,
                            double* pos_out, int8_t* status, int nthreads) {
  const Scene& s = *(Scene*)sp;
  const STree& t = *(STree*)h;
  Params p = to_params(pp);
  parallel_for(N, nthreads, [&](int c) {
    int prim[KMAX], n = 0, type = 0;
    V3d pos[KMAX];
    double pn = 0.0;
    for (int i = 0; i < KMAX; ++i) { prim[i] = INT32_MIN; pos[i] = V3d(); }
    int8_t st = stree_sample(s, t, p, n_fixed ? n_fixed[c] : 0, obj1[c], get3d(xD, N, c), get3d(nD, N, c),
                             get3d(xL, N, c), seed, (uint64_t)c, trial, &n, &type, &pn, prim, pos);
    status[c] = st;
    n_out[c] = (uint8_t)n;
    type_out[c] = (uint8_t)type;
    pn_out[c] = pn;
    for (int i = 0; i < KMAX; ++i) {
      bool have = st == 0 && i < n;
      prim_out[(size_t)i * N + c] = have ? prim[i] : INT32_MIN;
      for (int a = 0; a < 3; ++a) pos_out[((size_t)a * KMAX + i) * N + c] = have ? pos[i][a] : 0.0;
    }
  });
}

// Reciprocal probability with the paper's guide (Sec. 5.8): n is the
// target's and is kept across trials; each trial draws (w_D, tau) from the
// same mixture (trial counters 1 + r M + k - 1), walks, and matches the
// target (same tau, objects, vertices within match_rel L).  inv_prob =
// mean_r K_r / P(n).
void orc_stree_inv_prob(void* sp, void* h, const orc_params* pp, int N, const double* xD, const double* nD,
                        const double* xL, const uint8_t* len, const uint8_t* type, const int32_t* obj1,
                        const int32_t* tgt_prim, const double* tgt_pos, const int8_t* tgt_status, int max_trials,
                        int repeats, uint64_t seed, int32_t* trials, double* inv_prob, int8_t* truncated,
                        double* pn_out, int nthreads) {
  const Scene& s = *(Scene*)sp;
  const STree& t = *(STree*)h;
  Params p = to_params(pp);
  parallel_for(N, nthreads, [&](int c) {
    trials[c] = 0;
    inv_prob[c] = 0.0;
    truncated[c] = 0;
    pn_out[c] = 0.0;
    int n = len[c];
    if (tgt_status[c] != ST_CONVERGED || repeats < 1 || max_trials < 1 || n < 1 || n > KMAX) return;
    V3d xd = get3d(xD, N, c), xl = get3d(xL, N, c), nd = get3d(nD, N, c);
    Chain target;
    target.n = n;
    target.type = type[c];
    target.xD = xd;
    target.xL = xl;
    for (int i = 0; i < n; ++i) {
      V3d x(tgt_pos[((size_t)0 * KMAX + i) * N + c], tgt_pos[((size_t)1 * KMAX + i) * N + c],
            tgt_pos[((size_t)2 * KMAX + i) * N + c]);
      target.v[i] = make_geo(s, tgt_prim[(size_t)i * N + c], x);
    }
    double pn = 0.0;
    int total = 0;
    for (int r = 0; r < repeats; ++r) {
      int K = max_trials;
      bool found = false;
      for (int k = 1; k <= max_trials && !found; ++k) {
        uint64_t trial = 1 + (uint64_t)r * max_trials + (uint64_t)(k - 1);
        int prim[KMAX], nn = 0, tt = 0;
        V3d pos[KMAX];
        if (stree_sample(s, t, p, n, obj1[c], xd, nd, xl, seed, (uint64_t)c, trial, &nn, &tt, &pn, prim, pos) != 0)
          continue;
        if (tt != type[c]) continue;
        Chain start;
        if (!load_chain(s, n, tt, xd, xl, prim, pos, &start)) continue;
        WalkResult w;
        walk_core(s, p, start, &w);
        bool conv = w.status == ST_CONVERGED || w.status == ST_STALLED;
        if (conv && chains_match(s, w.chain, target, p.match_rel * p.scale)) {
          K = k;
          found = true;
        }
      }
      if (!found) truncated[c] = 1;
      total += K;
    }
    double q[6] = {xd.x, xd.y, xd.z, xl.x, xl.y, xl.z};
    pn = stree_pn(t, t.leaf[stree_leaf(t, q)], n);
    pn_out[c] = pn;
    trials[c] = total;
    inv_prob[c] = pn > 0.0 ? (double)total / repeats / pn : 0.0;
  });
}

}  // extern "C"
