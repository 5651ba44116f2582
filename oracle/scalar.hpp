// Scalar types for the CPU oracle.  TEST INFRASTRUCTURE ONLY: nothing in the
// product path may include, link or call anything under oracle/.
//
//  * double                - the plain reference computation;
//  * Dual                  - forward-mode dual number (value + one tangent), used
//                            to obtain exact Jacobian-vector products J*v of the
//                            time step with the switches frozen;
//  * Counting              - a double that counts the floating point operations
//                            it performs (algorithmic flop counts per step).
//
// Branch decisions (max/min/abs/comparisons) are always taken on the value, so
// a Dual run follows exactly the branches of the plain double run.
#pragma once
#include <cmath>
#include <cstdint>

namespace ora {

inline double val(double x) { return x; }

// ------------------------------------------------------------------- Dual ---
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline double val(const Dual& x) { return x.v; }
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, const Dual& b) { a = a * b; return a; }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); return Dual(e, a.d * e); }
inline Dual fabs(const Dual& a) { return a.v < 0 ? -a : a; }

// --------------------------------------------------------------- Counting ---
struct FlopCounter {
  static inline uint64_t add = 0, mul = 0, div = 0, sqrt = 0, exp = 0;
  static void reset() { add = mul = div = sqrt = exp = 0; }
};
struct Counting {
  double v;
  Counting() : v(0) {}
  Counting(double x) : v(x) {}
};
inline double val(const Counting& x) { return x.v; }
inline Counting operator+(const Counting& a, const Counting& b) { ++FlopCounter::add; return Counting(a.v + b.v); }
inline Counting operator-(const Counting& a, const Counting& b) { ++FlopCounter::add; return Counting(a.v - b.v); }
inline Counting operator-(const Counting& a) { return Counting(-a.v); }
inline Counting operator*(const Counting& a, const Counting& b) { ++FlopCounter::mul; return Counting(a.v * b.v); }
inline Counting operator/(const Counting& a, const Counting& b) { ++FlopCounter::div; return Counting(a.v / b.v); }
inline Counting& operator+=(Counting& a, const Counting& b) { a = a + b; return a; }
inline Counting& operator-=(Counting& a, const Counting& b) { a = a - b; return a; }
inline Counting& operator*=(Counting& a, const Counting& b) { a = a * b; return a; }
inline Counting sqrt(const Counting& a) { ++FlopCounter::sqrt; return Counting(std::sqrt(a.v)); }
inline Counting exp(const Counting& a) { ++FlopCounter::exp; return Counting(std::exp(a.v)); }
inline Counting fabs(const Counting& a) { return Counting(std::fabs(a.v)); }

// value-based helpers usable for every scalar type
template <class T> inline T tmax(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }
template <class T> inline T tmin(const T& a, const T& b) { return val(a) <= val(b) ? a : b; }
using std::sqrt;
using std::exp;
using std::fabs;

}  // namespace ora
