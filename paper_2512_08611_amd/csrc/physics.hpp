// Device equation systems for u_t + sum_d [ f_d(u)_{x_d} + B_d(u) u_{x_d} ] = 0
// (paper §3 eq. flux.and.non.cons; §5 2-D form above eq. time.step.2d).
//
// Every system is a struct with compile-time sizes and static device functions:
//   M, DIM, K         variables, space dimensions, admissibility constraints
//   NCD, nc_comp(d,i) the components of u_{x_d} that B_d(u) u_{x_d} reads
//   flux<d>(u, f)     f_d(u)
//   ncprod<d>(u,w,o)  B_d(u) w   (only the nc_comp components of w are read)
//   sigma<d>(u)       spectral radius of f_d' + B_d (eq. combined.wave.speed)
//   constraint(k,u)   P_k(u) of the admissible set (eq. uad.form)
//   indicator(u)      variable seen by the smoothness indicator
//   speeds<d>(u,|v|,c) ideal wave speeds used for the time step
//   SRC               true for a system with a source term s(u); it then has
//   source(u,s)       s(u)
//   implicit(r,c,x)   the solution x of x - c s(x) = r, c >= 0 (the pointwise
//                     implicit stage equation of §2 eq. crkfr.inner)
#pragma once
#include <hip/hip_runtime.h>

namespace lwfr {

struct PhysParams {
  double g;       // gravity
  double gamma;   // ratio of specific heats
  double ch;      // GLM cleaning speed (device value for the current step)
  double ra, reps, rl, rq;  // relaxation: speed a, time eps, f(u) = rl u + rq u^2/2
};

// Shallow water with the bed b carried as a variable: B u_x = (0, g h b_x, 0).
struct SW1D {
  static constexpr int M = 3, DIM = 1, K = 1, NCD = 1;
  static constexpr bool SRC = false;
  __host__ __device__ static constexpr int nc_comp(int, int) { return 2; }
  template <int d>
  __device__ static void flux(const double* u, double* f, const PhysParams& pp) {
    const double v = u[1] / u[0];
    f[0] = u[1];
    f[1] = u[1] * v + 0.5 * pp.g * u[0] * u[0];
    f[2] = 0.0;
  }
  template <int d>
  __device__ static void ncprod(const double* u, const double* w, double* o, const PhysParams& pp) {
    o[0] = 0.0; o[1] = pp.g * u[0] * w[2]; o[2] = 0.0;
  }
  template <int d>
  __device__ static double sigma(const double* u, const PhysParams& pp) {
    return fabs(u[1] / u[0]) + sqrt(pp.g * u[0]);
  }
  __device__ static double constraint(int, const double* u, const PhysParams&) { return u[0]; }
  __device__ static double indicator(const double* u, const PhysParams&) { return u[0]; }
  template <int d>
  __device__ static void speeds(const double* u, double& av, double& c, const PhysParams& pp) {
    av = fabs(u[1] / u[0]); c = sqrt(pp.g * u[0]);
  }
  // reverse mode: ub += (d f/d u)^T fb
  template <int d>
  __device__ static void flux_vjp(const double* u, const double* fb, double* ub, const PhysParams& pp) {
    const double v = u[1] / u[0];
    ub[0] += fb[1] * (-v * v + pp.g * u[0]);
    ub[1] += fb[0] + fb[1] * 2.0 * v;
  }
  // ub += (d(B(u)w)/du)^T ob, wb += B(u)^T ob
  template <int d>
  __device__ static void ncprod_vjp(const double* u, const double* w, const double* ob, double* ub, double* wb,
                                    const PhysParams& pp) {
    ub[0] += ob[1] * pp.g * w[2];
    wb[2] += ob[1] * pp.g * u[0];
  }
  template <int d>
  __device__ static void sigma_vjp(const double* u, double sb, double* ub, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double v = u[1] * ir;
    const double sg = v < 0.0 ? -1.0 : 1.0;
    ub[0] += sb * (-sg * v * ir + 0.5 * pp.g / sqrt(pp.g * u[0]));
    ub[1] += sb * sg * ir;
  }
};

struct SW2D {
  static constexpr int M = 4, DIM = 2, K = 1, NCD = 1;
  static constexpr bool SRC = false;
  __host__ __device__ static constexpr int flux_nc_alias(int) { return -1; }
  __host__ __device__ static constexpr int nc_comp(int, int) { return 3; }
  template <int d>
  __device__ static void flux(const double* u, double* f, const PhysParams& pp) {
    const double hu = u[1 + d];
    const double vel = hu / u[0];
    f[0] = hu;
    f[1] = u[1] * vel;
    f[2] = u[2] * vel;
    f[1 + d] += 0.5 * pp.g * u[0] * u[0];
    f[3] = 0.0;
  }
  template <int d>
  __device__ static void ncprod(const double* u, const double* w, double* o, const PhysParams& pp) {
    o[0] = 0.0; o[1] = 0.0; o[2] = 0.0; o[3] = 0.0;
    o[1 + d] = pp.g * u[0] * w[3];
  }
  template <int d>
  __device__ static double sigma(const double* u, const PhysParams& pp) {
    return fabs(u[1 + d] / u[0]) + sqrt(pp.g * u[0]);
  }
  // flux and B_d(u) w with the direction d a run-time value (selects, no
  // branches: lanes of one wave may take different directions); wc holds the
  // d-derivative of the non-conservative column (b)
  __device__ static void flux_rd(const double* u, int d, double* f, const PhysParams& pp) {
    const double hu = d ? u[2] : u[1];
    const double vel = hu / u[0];
    const double ph = 0.5 * pp.g * u[0] * u[0];
    f[0] = hu;
    f[1] = d ? u[1] * vel : u[1] * vel + ph;
    f[2] = d ? u[2] * vel + ph : u[2] * vel;
    f[3] = 0.0;
  }
  __device__ static void ncprod_rd(const double* u, const double* wc, int d, double* o, const PhysParams& pp) {
    const double t = pp.g * u[0] * wc[0];
    o[0] = 0.0;
    o[1] = d ? 0.0 : t;
    o[2] = d ? t : 0.0;
    o[3] = 0.0;
  }
  __device__ static double constraint(int, const double* u, const PhysParams&) { return u[0]; }
  __device__ static double indicator(const double* u, const PhysParams&) { return u[0]; }
  template <int d>
  __device__ static void speeds(const double* u, double& av, double& c, const PhysParams& pp) {
    av = fabs(u[1 + d] / u[0]); c = sqrt(pp.g * u[0]);
  }
  // speeds<d> with the direction a run-time value (the same operations)
  __device__ static void speeds_rd(const double* u, int d, double& av, double& c, const PhysParams& pp) {
    av = fabs((d ? u[2] : u[1]) / u[0]); c = sqrt(pp.g * u[0]);
  }
  template <int d>
  __device__ static void flux_vjp(const double* u, const double* fb, double* ub, const PhysParams& pp) {
    const double vel = u[1 + d] / u[0];
    double velb = 0.0;
    ub[1 + d] += fb[0];
    ub[1] += fb[1] * vel; velb += fb[1] * u[1];
    ub[2] += fb[2] * vel; velb += fb[2] * u[2];
    ub[0] += fb[1 + d] * pp.g * u[0];
    ub[1 + d] += velb / u[0];
    ub[0] -= velb * vel / u[0];
  }
  template <int d>
  __device__ static void ncprod_vjp(const double* u, const double* w, const double* ob, double* ub, double* wb,
                                    const PhysParams& pp) {
    ub[0] += ob[1 + d] * pp.g * w[3];
    wb[3] += ob[1 + d] * pp.g * u[0];
  }
  template <int d>
  __device__ static void sigma_vjp(const double* u, double sb, double* ub, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double v = u[1 + d] * ir;
    const double sg = v < 0.0 ? -1.0 : 1.0;
    ub[0] += sb * (-sg * v * ir + 0.5 * pp.g / sqrt(pp.g * u[0]));
    ub[1 + d] += sb * sg * ir;
  }
};

// Ideal GLM-MHD with the Godunov-Powell and GLM non-conservative terms (§5.5
// eq. glm.mhd) in the complete form of the source the paper cites: the energy
// flux is v_d(rho|v|^2/2 + gamma p/(gamma-1) + |B|^2) - B_d (v.B) + c_h psi B_d,
// the normal induction flux is c_h psi and the psi flux is c_h B_d.
// u = (rho, m1, m2, m3, E, B1, B2, B3, psi).
struct MHD2D {
  static constexpr int M = 9, DIM = 2, K = 2, NCD = 2;
  static constexpr bool SRC = false;
  __host__ __device__ static constexpr int nc_comp(int d, int i) { return i == 0 ? 5 + d : 8; }
  // flux components equal to c_h times a non-conservative column in every
  // direction (f_d[8] = c_h B_d): index of that column, else -1
  __host__ __device__ static constexpr int flux_nc_alias(int v) { return v == 8 ? 0 : -1; }
  // of the pair (5, 6), component 5+d of f_d is c_h times the psi column (f_d[5+d]
  // = c_h psi); a lane of direction d that forms D_d f_d needs the other one only
  static constexpr int flux_pair_nc_alias = 5;
  __device__ static double pressure(const double* u, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double mm = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const double bb = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    return (pp.gamma - 1.0) * (u[4] - 0.5 * mm * ir - 0.5 * bb - 0.5 * u[8] * u[8]);
  }
  template <int d>
  __device__ static void flux(const double* u, double* f, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
    const double B1 = u[5], B2 = u[6], B3 = u[7], psi = u[8];
    const double bb = B1 * B1 + B2 * B2 + B3 * B3;
    const double vv = v1 * v1 + v2 * v2 + v3 * v3;
    const double p = (pp.gamma - 1.0) * (u[4] - 0.5 * u[0] * vv - 0.5 * bb - 0.5 * psi * psi);
    const double vB = v1 * B1 + v2 * B2 + v3 * B3;
    const double vd = d == 0 ? v1 : v2;
    const double Bd = d == 0 ? B1 : B2;
    const double md = u[1 + d];
    f[0] = md;
    f[1] = md * v1 - Bd * B1;
    f[2] = md * v2 - Bd * B2;
    f[3] = md * v3 - Bd * B3;
    f[1 + d] += p + 0.5 * bb;
    f[4] = vd * (0.5 * u[0] * vv + pp.gamma / (pp.gamma - 1.0) * p + bb) - Bd * vB + pp.ch * psi * Bd;
    f[5] = vd * B1 - Bd * v1;
    f[6] = vd * B2 - Bd * v2;
    f[7] = vd * B3 - Bd * v3;
    f[5 + d] = pp.ch * psi;
    f[8] = pp.ch * Bd;
  }
  // B_d(u) w = w_{B_d} (0, B, v.B, v, 0) + w_psi (0, 0, 0, 0, v_d psi, 0, 0, 0, v_d)
  template <int d>
  __device__ static void ncprod(const double* u, const double* w, double* o, const PhysParams&) {
    const double ir = 1.0 / u[0];
    const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
    const double vd = d == 0 ? v1 : v2;
    const double dB = w[5 + d], dpsi = w[8];
    const double vB = v1 * u[5] + v2 * u[6] + v3 * u[7];
    o[0] = 0.0;
    o[1] = dB * u[5];
    o[2] = dB * u[6];
    o[3] = dB * u[7];
    o[4] = dB * vB + dpsi * vd * u[8];
    o[5] = dB * v1;
    o[6] = dB * v2;
    o[7] = dB * v3;
    o[8] = dpsi * vd;
  }
  // flux and B_d(u) w with the direction d a run-time value (selects, no
  // branches); wc = (d-derivative of B_d, d-derivative of psi)
  __device__ static void flux_rd(const double* u, int d, double* f, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
    const double B1 = u[5], B2 = u[6], B3 = u[7], psi = u[8];
    const double bb = B1 * B1 + B2 * B2 + B3 * B3;
    const double vv = v1 * v1 + v2 * v2 + v3 * v3;
    const double p = (pp.gamma - 1.0) * (u[4] - 0.5 * u[0] * vv - 0.5 * bb - 0.5 * psi * psi);
    const double vB = v1 * B1 + v2 * B2 + v3 * B3;
    const double vd = d ? v2 : v1;
    const double Bd = d ? B2 : B1;
    const double md = d ? u[2] : u[1];
    const double pt = p + 0.5 * bb;
    const double f1 = md * v1 - Bd * B1, f2 = md * v2 - Bd * B2;
    f[0] = md;
    f[1] = d ? f1 : f1 + pt;
    f[2] = d ? f2 + pt : f2;
    f[3] = md * v3 - Bd * B3;
    f[4] = vd * (0.5 * u[0] * vv + pp.gamma / (pp.gamma - 1.0) * p + bb) - Bd * vB + pp.ch * psi * Bd;
    const double cp = pp.ch * psi;
    const double f5 = vd * B1 - Bd * v1, f6 = vd * B2 - Bd * v2;
    f[5] = d ? f5 : cp;
    f[6] = d ? cp : f6;
    f[7] = vd * B3 - Bd * v3;
    f[8] = pp.ch * Bd;
  }
  __device__ static void ncprod_rd(const double* u, const double* wc, int d, double* o, const PhysParams&) {
    const double ir = 1.0 / u[0];
    const double v1 = u[1] * ir, v2 = u[2] * ir, v3 = u[3] * ir;
    const double vd = d ? v2 : v1;
    const double dB = wc[0], dpsi = wc[1];
    const double vB = v1 * u[5] + v2 * u[6] + v3 * u[7];
    o[0] = 0.0;
    o[1] = dB * u[5];
    o[2] = dB * u[6];
    o[3] = dB * u[7];
    o[4] = dB * vB + dpsi * vd * u[8];
    o[5] = dB * v1;
    o[6] = dB * v2;
    o[7] = dB * v3;
    o[8] = dpsi * vd;
  }
  template <int d>
  __device__ static double cfast(const double* u, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double p = pressure(u, pp);
    const double a2 = pp.gamma * p * ir;
    const double b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * ir;
    const double bd2 = u[5 + d] * u[5 + d] * ir;
    const double s = a2 + b2;
    return sqrt(0.5 * (s + sqrt(s * s - 4.0 * a2 * bd2)));
  }
  // waves v_d, v_d ± c_a, v_d ± c_s, v_d ± c_f and the GLM pair v_d ± c_h
  template <int d>
  __device__ static double sigma(const double* u, const PhysParams& pp) {
    const double cf = cfast<d>(u, pp);
    return fabs(u[1 + d] / u[0]) + (cf >= pp.ch ? cf : pp.ch);
  }
  __device__ static double constraint(int k, const double* u, const PhysParams& pp) {
    return k == 0 ? u[0] : pressure(u, pp);
  }
  __device__ static double indicator(const double* u, const PhysParams& pp) { return u[0] * pressure(u, pp); }
  template <int d>
  __device__ static void speeds(const double* u, double& av, double& c, const PhysParams& pp) {
    av = fabs(u[1 + d] / u[0]); c = cfast<d>(u, pp);
  }
  // speeds<d> with the direction a run-time value (the same operations)
  __device__ static void speeds_rd(const double* u, int d, double& av, double& c, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double p = pressure(u, pp);
    const double a2 = pp.gamma * p * ir;
    const double b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * ir;
    const double Bd = d ? u[6] : u[5];
    const double bd2 = Bd * Bd * ir;
    const double s = a2 + b2;
    av = fabs((d ? u[2] : u[1]) / u[0]);
    c = sqrt(0.5 * (s + sqrt(s * s - 4.0 * a2 * bd2)));
  }

  // the components with x and y exchanged when d = 1 (an involution R, the
  // identity for d = 0).  The system is invariant under that exchange:
  // f_y(u) = R f_x(R u) and B_y(u) w = R B_x(R u) R w, so a lane working on
  // direction 1 can run the direction-0 code in the exchanged frame
  __device__ static void rot(int d, double* x) {
    const double a = x[1], b = x[2], c = x[5], e = x[6];
    x[1] = d ? b : a;
    x[2] = d ? a : b;
    x[5] = d ? e : c;
    x[6] = d ? c : e;
  }

  // ---- reverse mode (hand-written adjoints of flux, ncprod and sigma above)
  template <int d>
  __device__ static void flux_vjp(const double* u, const double* fb, double* ub, const PhysParams& pp) {
    const double rho = u[0], ir = 1.0 / rho;
    const double v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    const double* B = u + 5;
    const double psi = u[8];
    const double bb = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double gm1 = pp.gamma - 1.0, g1 = pp.gamma / gm1;
    const double p = gm1 * (u[4] - 0.5 * rho * vv - 0.5 * bb - 0.5 * psi * psi);
    const double vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    const double vd = v[d], Bd = B[d], md = u[1 + d];
    double vb[3] = {0.0, 0.0, 0.0}, Bb[3] = {0.0, 0.0, 0.0};
    double rhob = 0.0, mdb = 0.0, pb = 0.0, bbb = 0.0, vvb = 0.0, vBb = 0.0, psib = 0.0, Eb = 0.0;
    mdb += fb[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      mdb += fb[1 + k] * v[k];
      vb[k] += fb[1 + k] * md;
      Bb[d] -= fb[1 + k] * B[k];
      Bb[k] -= fb[1 + k] * Bd;
    }
    pb += fb[1 + d];
    bbb += 0.5 * fb[1 + d];
    const double T = 0.5 * rho * vv + g1 * p + bb;
    vb[d] += fb[4] * T;
    rhob += fb[4] * vd * 0.5 * vv;
    vvb += fb[4] * vd * 0.5 * rho;
    pb += fb[4] * vd * g1;
    bbb += fb[4] * vd;
    Bb[d] -= fb[4] * vB;
    vBb -= fb[4] * Bd;
    psib += fb[4] * pp.ch * Bd;
    Bb[d] += fb[4] * pp.ch * psi;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == d) continue;
      vb[d] += fb[5 + k] * B[k];
      Bb[k] += fb[5 + k] * vd;
      Bb[d] -= fb[5 + k] * v[k];
      vb[k] -= fb[5 + k] * Bd;
    }
    psib += fb[5 + d] * pp.ch;
    Bb[d] += fb[8] * pp.ch;
    // intermediates
#pragma unroll
    for (int k = 0; k < 3; ++k) { vb[k] += vBb * B[k]; Bb[k] += vBb * v[k]; }
    Eb += pb * gm1;
    rhob -= pb * gm1 * 0.5 * vv;
    vvb -= pb * gm1 * 0.5 * rho;
    bbb -= pb * gm1 * 0.5;
    psib -= pb * gm1 * psi;
    double irb = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      vb[k] += 2.0 * vvb * v[k];
      Bb[k] += 2.0 * bbb * B[k];
    }
    double mb[3] = {0.0, 0.0, 0.0};
    mb[d] += mdb;
#pragma unroll
    for (int k = 0; k < 3; ++k) { mb[k] += vb[k] * ir; irb += vb[k] * u[1 + k]; }
    rhob -= irb * ir * ir;
    ub[0] += rhob;
    ub[1] += mb[0]; ub[2] += mb[1]; ub[3] += mb[2];
    ub[4] += Eb;
    ub[5] += Bb[0]; ub[6] += Bb[1]; ub[7] += Bb[2];
    ub[8] += psib;
  }
  template <int d>
  __device__ static void ncprod_vjp(const double* u, const double* w, const double* ob, double* ub, double* wb,
                                    const PhysParams&) {
    const double ir = 1.0 / u[0];
    const double v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    const double vd = v[d];
    const double dB = w[5 + d], dpsi = w[8];
    const double vB = v[0] * u[5] + v[1] * u[6] + v[2] * u[7];
    double dBb = 0.0, dpsib = 0.0, vBb = 0.0;
    double vb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dBb += ob[1 + k] * u[5 + k] + ob[5 + k] * v[k];
      ub[5 + k] += ob[1 + k] * dB;
      vb[k] += ob[5 + k] * dB;
    }
    dBb += ob[4] * vB;
    vBb += ob[4] * dB;
    dpsib += ob[4] * vd * u[8] + ob[8] * vd;
    vb[d] += ob[4] * dpsi * u[8] + ob[8] * dpsi;
    ub[8] += ob[4] * dpsi * vd;
#pragma unroll
    for (int k = 0; k < 3; ++k) { vb[k] += vBb * u[5 + k]; ub[5 + k] += vBb * v[k]; }
    double irb = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) { ub[1 + k] += vb[k] * ir; irb += vb[k] * u[1 + k]; }
    ub[0] -= irb * ir * ir;
    wb[5 + d] += dBb;
    wb[8] += dpsib;
  }
  template <int d>
  __device__ static void sigma_vjp(const double* u, double sb, double* ub, const PhysParams& pp) {
    const double ir = 1.0 / u[0];
    const double vdv = u[1 + d] * ir;
    const double sg = vdv < 0.0 ? -1.0 : 1.0;
    double irb = 0.0;
    ub[1 + d] += sb * sg * ir;
    irb += sb * sg * u[1 + d];
    const double cf = cfast<d>(u, pp);
    if (cf >= pp.ch) {
      // cf = sqrt(X), X = (s + R)/2, R = sqrt(s^2 - 4 a2 bd2), s = a2 + b2
      const double mm = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
      const double bb = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
      const double gm1 = pp.gamma - 1.0;
      const double p = gm1 * (u[4] - 0.5 * mm * ir - 0.5 * bb - 0.5 * u[8] * u[8]);
      const double a2 = pp.gamma * p * ir, b2 = bb * ir, bd2 = u[5 + d] * u[5 + d] * ir;
      const double s = a2 + b2;
      const double R = sqrt(s * s - 4.0 * a2 * bd2);
      const double Xb = sb / (2.0 * cf);
      double sbar = 0.5 * Xb;
      const double Rb = 0.5 * Xb;
      const double Db = R > 0.0 ? Rb / (2.0 * R) : 0.0;
      sbar += 2.0 * s * Db;
      const double a2b = -4.0 * bd2 * Db + sbar;
      const double bd2b = -4.0 * a2 * Db;
      const double b2b = sbar;
      double pb = a2b * pp.gamma * ir;
      irb += a2b * pp.gamma * p + b2b * bb + bd2b * u[5 + d] * u[5 + d];
      double bbb = b2b * ir;
      ub[5 + d] += bd2b * 2.0 * u[5 + d] * ir;
      // p = (gamma-1)(E - mm ir/2 - bb/2 - psi^2/2)
      ub[4] += pb * gm1;
#pragma unroll
      for (int k = 0; k < 3; ++k) ub[1 + k] -= pb * gm1 * u[1 + k] * ir;
      irb -= pb * gm1 * 0.5 * mm;
      bbb -= pb * gm1 * 0.5;
      ub[8] -= pb * gm1 * u[8];
#pragma unroll
      for (int k = 0; k < 3; ++k) ub[5 + k] += 2.0 * bbb * u[5 + k];
    }
    ub[0] -= irb * ir * ir;
  }
};

// Linear advection u_t + u_x = 0.
struct LinAdv1D {
  static constexpr int M = 1, DIM = 1, K = 0, NCD = 0;
  static constexpr bool SRC = false;
  __host__ __device__ static constexpr int nc_comp(int, int) { return 0; }
  template <int d> __device__ static void flux(const double* u, double* f, const PhysParams&) { f[0] = u[0]; }
  template <int d> __device__ static void ncprod(const double*, const double*, double* o, const PhysParams&) { o[0] = 0.0; }
  template <int d> __device__ static double sigma(const double*, const PhysParams&) { return 1.0; }
  __device__ static double constraint(int, const double* u, const PhysParams&) { return u[0]; }
  __device__ static double indicator(const double* u, const PhysParams&) { return u[0]; }
  template <int d> __device__ static void speeds(const double*, double& av, double& c, const PhysParams&) { av = 0.0; c = 1.0; }
  template <int d> __device__ static void flux_vjp(const double*, const double* fb, double* ub, const PhysParams&) {
    ub[0] += fb[0];
  }
  template <int d>
  __device__ static void ncprod_vjp(const double*, const double*, const double*, double*, double*, const PhysParams&) {}
  template <int d> __device__ static void sigma_vjp(const double*, double, double*, const PhysParams&) {}
};

// Variable-coefficient advection as a non-conservative system: u = (v, a),
// f = 0, B(u) w = (u_2 w_1, 0) (§5.1 eq. var.coeff.adv.non.cons).
struct VarAdv1D {
  static constexpr int M = 2, DIM = 1, K = 0, NCD = 1;
  static constexpr bool SRC = false;
  __host__ __device__ static constexpr int nc_comp(int, int) { return 0; }
  template <int d> __device__ static void flux(const double*, double* f, const PhysParams&) { f[0] = 0.0; f[1] = 0.0; }
  template <int d> __device__ static void ncprod(const double* u, const double* w, double* o, const PhysParams&) {
    o[0] = u[1] * w[0]; o[1] = 0.0;
  }
  template <int d> __device__ static double sigma(const double* u, const PhysParams&) { return fabs(u[1]); }
  __device__ static double constraint(int, const double* u, const PhysParams&) { return u[0]; }
  __device__ static double indicator(const double* u, const PhysParams&) { return u[0]; }
  template <int d> __device__ static void speeds(const double* u, double& av, double& c, const PhysParams&) {
    av = 0.0; c = fabs(u[1]);
  }
  template <int d> __device__ static void flux_vjp(const double*, const double*, double*, const PhysParams&) {}
  template <int d>
  __device__ static void ncprod_vjp(const double* u, const double* w, const double* ob, double* ub, double* wb,
                                    const PhysParams&) {
    ub[1] += ob[0] * w[0];
    wb[0] += ob[0] * u[1];
  }
  template <int d> __device__ static void sigma_vjp(const double* u, double sb, double* ub, const PhysParams&) {
    ub[1] += sb * (u[1] < 0.0 ? -1.0 : 1.0);
  }
};

// Jin-Xin relaxation system (§5.1 eqs. jinxin1, jinxin2): u = (u, v), flux
// (v, a^2 u), no non-conservative product, source (0, -(v - f(u))/eps) with
// f(u) = l u + q u^2/2 (Burgers: l = 0, q = 1).  Flux eigenvalues +-a; no
// admissibility constraint.
struct JinXin1D {
  static constexpr int M = 2, DIM = 1, K = 0, NCD = 0;
  static constexpr bool SRC = true;
  __host__ __device__ static constexpr int nc_comp(int, int) { return 0; }
  __device__ static double feq(double u, const PhysParams& pp) { return pp.rl * u + 0.5 * pp.rq * u * u; }
  template <int d> __device__ static void flux(const double* u, double* f, const PhysParams& pp) {
    f[0] = u[1];
    f[1] = pp.ra * pp.ra * u[0];
  }
  template <int d> __device__ static void ncprod(const double*, const double*, double* o, const PhysParams&) {
    o[0] = 0.0; o[1] = 0.0;
  }
  template <int d> __device__ static double sigma(const double*, const PhysParams& pp) { return pp.ra; }
  __device__ static double constraint(int, const double* u, const PhysParams&) { return u[0]; }
  __device__ static double indicator(const double* u, const PhysParams&) { return u[0]; }
  template <int d> __device__ static void speeds(const double*, double& av, double& c, const PhysParams& pp) {
    av = 0.0; c = pp.ra;
  }
  __device__ static void source(const double* u, double* s, const PhysParams& pp) {
    s[0] = 0.0;
    s[1] = -(u[1] - feq(u[0], pp)) / pp.reps;
  }
  // x - c s(x) = r: x_1 = r_1 (no source in the first component); the second
  // equation is linear in x_2: x_2 (1 + c/eps) = r_2 + (c/eps) f(r_1)
  __device__ static void implicit(const double* r, double c, double* x, const PhysParams& pp) {
    const double k = c / pp.reps;
    x[0] = r[0];
    x[1] = (r[1] + k * feq(r[0], pp)) / (1.0 + k);
  }
};

// Components of the time-averaged flux whose face traces follow from those of
// the time-averaged solution.  Where f_d(u)[v] = c u[w] for a constant c, the
// average F_d = sum_s b_s f_d(u^(s)) equals c U[w] with U = sum_s b_s u^(s), and
// so do their face traces.  GLM-MHD: f_d[0] = u[1+d] (mass flux), f_d[5+d] =
// c_h psi and f_d[8] = c_h B_d.  src(d, v): w, or -1 where F_d[v] is stored;
// ch_scaled(v): the factor is c_h (else 1).
template <class Ph>
struct TraceAlias {
  __host__ __device__ static constexpr int src(int, int) { return -1; }
  __host__ __device__ static constexpr bool ch_scaled(int) { return false; }
};
template <>
struct TraceAlias<MHD2D> {
  __host__ __device__ static constexpr int src(int d, int v) {
    return v == 0 ? 1 + d : v == 5 + d ? 8 : v == 8 ? 5 + d : -1;
  }
  __host__ __device__ static constexpr bool ch_scaled(int v) { return v != 0; }
};

}  // namespace lwfr
