// Forward-mode dual numbers and small 3-vectors for the FP64 oracle.
//
// TEST INFRASTRUCTURE ONLY: the oracle is a plain, slow CPU reference used by
// the tests and the benchmark's CPU-baseline leg.  The product path never
// includes, links or calls anything under oracle/.
//
// Dual<T, D> carries a value and D partial derivatives.  Nesting
// Dual<Dual<double, A>, B> gives second derivatives, which the adjoint of the
// generalized geometric term needs.
#pragma once
#include <cmath>
#include <cstring>

namespace oracle {

template <class T, int D>
struct Dual {
  T v;
  T d[D];
  Dual() : v(0) { for (int i = 0; i < D; ++i) d[i] = T(0); }
  Dual(double c) : v(c) { for (int i = 0; i < D; ++i) d[i] = T(0); }  // NOLINT
  Dual(const T& c, int) : v(c) { for (int i = 0; i < D; ++i) d[i] = T(0); }
  static Dual var(const T& value, int slot) {
    Dual r(value, 0);
    r.d[slot] = T(1);
    return r;
  }
};

// value extraction through any nesting depth
inline double val(double x) { return x; }
template <class T, int D> double val(const Dual<T, D>& x) { return val(x.v); }

#define ORACLE_DUAL_BINOP(OP, VEXPR, DEXPR)                                        \
  template <class T, int D>                                                        \
  Dual<T, D> operator OP(const Dual<T, D>& a, const Dual<T, D>& b) {               \
    Dual<T, D> r(VEXPR, 0);                                                        \
    for (int i = 0; i < D; ++i) r.d[i] = DEXPR;                                    \
    return r;                                                                      \
  }
ORACLE_DUAL_BINOP(+, a.v + b.v, a.d[i] + b.d[i])
ORACLE_DUAL_BINOP(-, a.v - b.v, a.d[i] - b.d[i])
ORACLE_DUAL_BINOP(*, a.v * b.v, a.d[i] * b.v + a.v * b.d[i])
#undef ORACLE_DUAL_BINOP

template <class T, int D>
Dual<T, D> operator/(const Dual<T, D>& a, const Dual<T, D>& b) {
  T inv = T(1) / b.v;
  T q = a.v * inv;
  Dual<T, D> r(q, 0);
  for (int i = 0; i < D; ++i) r.d[i] = (a.d[i] - q * b.d[i]) * inv;
  return r;
}
template <class T, int D> Dual<T, D> operator-(const Dual<T, D>& a) {
  Dual<T, D> r(-a.v, 0);
  for (int i = 0; i < D; ++i) r.d[i] = -a.d[i];
  return r;
}
template <class T, int D> Dual<T, D> operator+(const Dual<T, D>& a, double b) { return a + Dual<T, D>(b); }
template <class T, int D> Dual<T, D> operator+(double a, const Dual<T, D>& b) { return Dual<T, D>(a) + b; }
template <class T, int D> Dual<T, D> operator-(const Dual<T, D>& a, double b) { return a - Dual<T, D>(b); }
template <class T, int D> Dual<T, D> operator-(double a, const Dual<T, D>& b) { return Dual<T, D>(a) - b; }
template <class T, int D> Dual<T, D> operator*(const Dual<T, D>& a, double b) { return a * Dual<T, D>(b); }
template <class T, int D> Dual<T, D> operator*(double a, const Dual<T, D>& b) { return Dual<T, D>(a) * b; }
template <class T, int D> Dual<T, D> operator/(const Dual<T, D>& a, double b) { return a / Dual<T, D>(b); }
template <class T, int D> Dual<T, D> operator/(double a, const Dual<T, D>& b) { return Dual<T, D>(a) / b; }

template <class T, int D> bool operator<(const Dual<T, D>& a, const Dual<T, D>& b) { return val(a) < val(b); }
template <class T, int D> bool operator>(const Dual<T, D>& a, const Dual<T, D>& b) { return val(a) > val(b); }

using std::cos;
using std::sin;
using std::sqrt;
using std::fabs;
template <class T, int D> Dual<T, D> sqrt(const Dual<T, D>& a) {
  T s = sqrt(a.v);
  T g = T(0.5) / s;
  Dual<T, D> r(s, 0);
  for (int i = 0; i < D; ++i) r.d[i] = g * a.d[i];
  return r;
}
template <class T, int D> Dual<T, D> sin(const Dual<T, D>& a) {
  T c = cos(a.v);
  Dual<T, D> r(sin(a.v), 0);
  for (int i = 0; i < D; ++i) r.d[i] = c * a.d[i];
  return r;
}
template <class T, int D> Dual<T, D> cos(const Dual<T, D>& a) {
  T s = -sin(a.v);
  Dual<T, D> r(cos(a.v), 0);
  for (int i = 0; i < D; ++i) r.d[i] = s * a.d[i];
  return r;
}
template <class T, int D> Dual<T, D> fabs(const Dual<T, D>& a) { return val(a) < 0 ? -a : a; }

template <class T>
struct V3 {
  T x, y, z;
  V3() : x(0), y(0), z(0) {}
  V3(const T& a, const T& b, const T& c) : x(a), y(b), z(c) {}
  template <class U> static V3 from(const V3<U>& o) { return V3(T(o.x), T(o.y), T(o.z)); }
  const T& operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
  T& operator[](int i) { return i == 0 ? x : (i == 1 ? y : z); }
};
using V3d = V3<double>;

template <class T> V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> V3<T> operator-(const V3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T, class S> V3<T> operator*(const V3<T>& a, const S& s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> T norm(const V3<T>& a) { return sqrt(dot(a, a)); }
template <class T> V3<T> normalize(const V3<T>& a) {
  T inv = T(1) / norm(a);
  return a * inv;
}
// mixed double / T products (constant geometry times a dual vector)
template <class T> V3<T> lift(const V3d& a) { return {T(a.x), T(a.y), T(a.z)}; }
inline V3d vval(const V3d& a) { return a; }
template <class T, int D> V3d vval(const V3<Dual<T, D>>& a) { return {val(a.x), val(a.y), val(a.z)}; }

}  // namespace oracle
