// Equation systems u_t + sum_d [ f_d(u)_{x_d} + B_d(u) u_{x_d} ] = 0 for the
// oracle (paper §3 eq. flux.and.non.cons; §5 2-D form above eq. time.step.2d).
// TEST INFRASTRUCTURE ONLY.
//
// Each system provides, templated on the scalar type T:
//   flux(d,u,f)        f_d(u)
//   ncprod(d,u,w,o)    B_d(u) w   (the non-conservative matrix applied to w)
//   sigma(d,u,ch)      spectral radius of f_d'(u) + B_d(u)  (eq. combined.wave.speed)
//   constraint(k,u)    P_k(u) of the admissible set (eq. uad.form)
//   indicator(u)       the variable the smoothness indicator looks at
//   speeds(d,u,absv,c) |v_d| and the largest characteristic speed without GLM.
// Systems with a source term (SRC = true, §2 eq. con.law.source) also provide
//   source(u,s)        s(u)
//   implicit(r,c,u)    the solution u of u - c s(u) = r (c >= 0), the pointwise
//                      implicit stage equation of eq. crkfr.inner.
#pragma once
#include "scalar.hpp"

namespace ora {

enum { EQ_SW1D = 1, EQ_SW2D = 2, EQ_MHD2D = 3, EQ_LINADV1D = 4, EQ_VARADV1D = 5, EQ_JINXIN1D = 6 };

// ---------------------------------------------------------------------------
// Shallow water with bathymetry b carried as a state variable, as the paper
// carries the advection coefficient of eq. var.coeff.adv.non.cons: u = (h, hv, b)
// and B(u) u_x = (0, g h b_x, 0).  The bathymetry is constant in time
// (b_t = 0), hence its row of f and B is zero.
struct SW1D {
  static constexpr int M = 3, DIM = 1, K = 1;
  static constexpr bool SRC = false;
  // columns of B_d that are not identically zero (B_d(u) w reads only these w_c)
  static constexpr int NCOL = 1;
  static int ncol(int, int) { return 2; }
  double g;
  template <class T> void flux(int, const T* u, T* f, double) const {
    T v = u[1] / u[0];
    f[0] = u[1];
    f[1] = u[1] * v + T(0.5 * g) * u[0] * u[0];
    f[2] = T(0.0);
  }
  template <class T> void ncprod(int, const T* u, const T* w, T* o) const {
    o[0] = T(0.0); o[1] = T(g) * u[0] * w[2]; o[2] = T(0.0);
  }
  template <class T> T sigma(int, const T* u, double) const {
    return fabs(u[1] / u[0]) + sqrt(T(g) * u[0]);
  }
  template <class T> T constraint(int, const T* u) const { return u[0]; }
  template <class T> T indicator(const T* u) const { return u[0]; }
  template <class T> void speeds(int, const T* u, T& absv, T& c) const {
    absv = fabs(u[1] / u[0]); c = sqrt(T(g) * u[0]);
  }
};

struct SW2D {
  static constexpr int M = 4, DIM = 2, K = 1;
  static constexpr bool SRC = false;
  static constexpr int NCOL = 1;
  static int ncol(int, int) { return 3; }
  double g;
  template <class T> void flux(int d, const T* u, T* f, double) const {
    T v1 = u[1] / u[0], v2 = u[2] / u[0];
    T hp = T(0.5 * g) * u[0] * u[0];
    if (d == 0) { f[0] = u[1]; f[1] = u[1] * v1 + hp; f[2] = u[1] * v2; }
    else        { f[0] = u[2]; f[1] = u[2] * v1;      f[2] = u[2] * v2 + hp; }
    f[3] = T(0.0);
  }
  template <class T> void ncprod(int d, const T* u, const T* w, T* o) const {
    o[0] = T(0.0); o[3] = T(0.0);
    T ghb = T(g) * u[0] * w[3];
    o[1] = d == 0 ? ghb : T(0.0);
    o[2] = d == 0 ? T(0.0) : ghb;
  }
  template <class T> T sigma(int d, const T* u, double) const {
    return fabs(u[1 + d] / u[0]) + sqrt(T(g) * u[0]);
  }
  template <class T> T constraint(int, const T* u) const { return u[0]; }
  template <class T> T indicator(const T* u) const { return u[0]; }
  template <class T> void speeds(int d, const T* u, T& absv, T& c) const {
    absv = fabs(u[1 + d] / u[0]); c = sqrt(T(g) * u[0]);
  }
};

// ---------------------------------------------------------------------------
// Ideal GLM-MHD with the Godunov-Powell and GLM non-conservative terms (paper
// §5.5 eq. glm.mhd, in the complete form of its cited source: the GLM
// contributions c_h psi B_d to the energy flux and c_h psi to the normal
// induction flux are included, and the energy flux carries no psi^2/2 transport,
// which the non-conservative term psi v . grad psi supplies).
// u = (rho, rho v1, rho v2, rho v3, E, B1, B2, B3, psi),
// p = (gamma-1)(E - rho|v|^2/2 - |B|^2/2 - psi^2/2).
struct MHD2D {
  static constexpr int M = 9, DIM = 2, K = 2;
  static constexpr bool SRC = false;
  static constexpr int NCOL = 2;
  static int ncol(int d, int i) { return i == 0 ? 5 + d : 8; }
  double gamma;
  template <class T> T pressure(const T* u) const {
    T kin = T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    T mag = T(0.5) * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]);
    return T(gamma - 1.0) * (u[4] - kin - mag - T(0.5) * u[8] * u[8]);
  }
  template <class T> void flux(int d, const T* u, T* f, double ch) const {
    T rho = u[0];
    T v[3] = {u[1] / rho, u[2] / rho, u[3] / rho};
    const T* B = u + 5;
    T psi = u[8];
    T p = pressure(u);
    T B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    T vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    T v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    T ptot = p + T(0.5) * B2;
    T vd = v[d], Bd = B[d];
    T md = u[1 + d];
    f[0] = md;
    for (int i = 0; i < 3; ++i) f[1 + i] = md * v[i] - Bd * B[i];
    f[1 + d] = f[1 + d] + ptot;
    f[4] = vd * (T(0.5) * rho * v2 + T(gamma / (gamma - 1.0)) * p + B2) - Bd * vB + T(ch) * psi * Bd;
    for (int i = 0; i < 3; ++i) f[5 + i] = vd * B[i] - Bd * v[i];
    f[5 + d] = T(ch) * psi;
    f[8] = T(ch) * Bd;
  }
  // B_d(u) w = (dB_d)(0, B, v.B, v, 0) + (dpsi)(0, 0, 0, 0, v_d psi, 0, 0, 0, v_d)
  // with dB_d = w[5+d], dpsi = w[8] (eq. glm.mhd, term Upsilon_GLM).
  template <class T> void ncprod(int d, const T* u, const T* w, T* o) const {
    T rho = u[0];
    T v[3] = {u[1] / rho, u[2] / rho, u[3] / rho};
    const T* B = u + 5;
    T psi = u[8];
    T divB = w[5 + d], dpsi = w[8];
    T vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    o[0] = T(0.0);
    for (int i = 0; i < 3; ++i) o[1 + i] = divB * B[i];
    o[4] = divB * vB + dpsi * v[d] * psi;
    for (int i = 0; i < 3; ++i) o[5 + i] = divB * v[i];
    o[8] = dpsi * v[d];
  }
  // fast magnetosonic speed in direction d
  template <class T> T cfast(int d, const T* u) const {
    T rho = u[0];
    T p = pressure(u);
    T a2 = T(gamma) * p / rho;
    T b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) / rho;
    T bd2 = u[5 + d] * u[5 + d] / rho;
    T s = a2 + b2;
    return sqrt(T(0.5) * (s + sqrt(s * s - T(4.0) * a2 * bd2)));
  }
  // The x_d-block of f'+B splits into the ideal-MHD waves v_d, v_d±c_a, v_d±c_s,
  // v_d±c_f and the GLM pair v_d±c_h (Powell term puts v_d on the diagonal of
  // the (B_d, psi) rows), so the spectral radius is |v_d| + max(c_f, c_h).
  template <class T> T sigma(int d, const T* u, double ch) const {
    T cf = cfast(d, u);
    T c = val(cf) >= ch ? cf : T(ch);
    return fabs(u[1 + d] / u[0]) + c;
  }
  template <class T> T constraint(int k, const T* u) const { return k == 0 ? u[0] : pressure(u); }
  template <class T> T indicator(const T* u) const { return u[0] * pressure(u); }
  template <class T> void speeds(int d, const T* u, T& absv, T& c) const {
    absv = fabs(u[1 + d] / u[0]); c = cfast<T>(d, u);
  }
};

// ---------------------------------------------------------------------------
// Test systems.  Linear advection u_t + a u_x = 0 with a = 1 (scalar law of
// eq. scalar.cons.law with f = u).
struct LinAdv1D {
  static constexpr int M = 1, DIM = 1, K = 0;
  static constexpr bool SRC = false;
  static constexpr int NCOL = 0;
  static int ncol(int, int) { return 0; }
  template <class T> void flux(int, const T* u, T* f, double) const { f[0] = u[0]; }
  template <class T> void ncprod(int, const T*, const T*, T* o) const { o[0] = T(0.0); }
  template <class T> T sigma(int, const T*, double) const { return T(1.0); }
  template <class T> T constraint(int, const T* u) const { return u[0]; }
  template <class T> T indicator(const T* u) const { return u[0]; }
  template <class T> void speeds(int, const T*, T& absv, T& c) const { absv = T(0.0); c = T(1.0); }
};

// Variable-coefficient advection cast as a non-conservative system (paper §5.1
// eq. var.coeff.adv.non.cons): u = (v, a), f = 0, B(u) w = (u_2 w_1, 0).
struct VarAdv1D {
  static constexpr int M = 2, DIM = 1, K = 0;
  static constexpr bool SRC = false;
  static constexpr int NCOL = 1;
  static int ncol(int, int) { return 0; }
  template <class T> void flux(int, const T*, T* f, double) const { f[0] = T(0.0); f[1] = T(0.0); }
  template <class T> void ncprod(int, const T* u, const T* w, T* o) const { o[0] = u[1] * w[0]; o[1] = T(0.0); }
  template <class T> T sigma(int, const T* u, double) const { return fabs(u[1]); }
  template <class T> T constraint(int, const T* u) const { return u[0]; }
  template <class T> T indicator(const T* u) const { return u[0]; }
  template <class T> void speeds(int, const T* u, T& absv, T& c) const { absv = T(0.0); c = fabs(u[1]); }
};

// Jin-Xin relaxation system (§5.1 eqs. jinxin1, jinxin2): u = (u, v), flux
// (v, a^2 u), no non-conservative product, source (0, -(v - f(u))/eps) with
// f(u) = l u + q u^2/2 (the paper's case is Burgers, l = 0, q = 1; q = 0 gives
// the linear system with exact Fourier solutions).  Eigenvalues of the flux
// Jacobian: +-a.  No admissibility constraint; the indicator looks at u.
struct JinXin1D {
  static constexpr int M = 2, DIM = 1, K = 0;
  static constexpr bool SRC = true;
  static constexpr int NCOL = 0;
  static int ncol(int, int) { return 0; }
  double a, eps, l, q;
  template <class T> T f(const T& u) const { return T(l) * u + T(0.5 * q) * u * u; }
  template <class T> void flux(int, const T* u, T* fo, double) const { fo[0] = u[1]; fo[1] = T(a * a) * u[0]; }
  template <class T> void ncprod(int, const T*, const T*, T* o) const { o[0] = T(0.0); o[1] = T(0.0); }
  template <class T> T sigma(int, const T*, double) const { return T(a); }
  template <class T> T constraint(int, const T* u) const { return u[0]; }
  template <class T> T indicator(const T* u) const { return u[0]; }
  template <class T> void speeds(int, const T*, T& absv, T& c) const { absv = T(0.0); c = T(a); }
  template <class T> void source(const T* u, T* s) const {
    s[0] = T(0.0);
    s[1] = -(u[1] - f(u[0])) / T(eps);
  }
  // u - c s(u) = r: the first component has no source, so u = r_1, and the
  // second is linear in v: v + (c/eps)(v - f(u)) = r_2
  template <class T> void implicit(const T* r, double c, T* u) const {
    u[0] = r[0];
    u[1] = (r[1] + T(c / eps) * f(r[0])) / T(1.0 + c / eps);
  }
};

}  // namespace ora
