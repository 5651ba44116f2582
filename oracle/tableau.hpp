// Explicit Runge-Kutta tableaux (A~, b~) of the time-averaged compact RK step.
// TEST INFRASTRUCTURE ONLY.
//
// The paper's single-stage scheme (§2 eqs. crkfr.inner, disc.avg.flux,
// time.avg.soln; §3 eqs. crkfr.non.cons.final, local.time.avg.non.cons) uses
// only the explicit part of a tableau.  Reading adopted for degree N: a method
// of order N+1 —
//   N=0 forward Euler; N=1 Heun (explicit part of HT(1,1,2), App. C eq.
//   ht112.butcher); N=2 SSPRK(3,3) (explicit part of SSP3-IMEX(4,3,3), App. C eq.
//   ssp33.butcher, without its empty first stage); N=3 classical RK4;
//   N=4 Butcher's six-stage fifth-order method (1964).
//
// Systems with a stiff source take an IMEX pair instead (§2 eq. crkfr.inner:
// explicit A~ for the flux terms, diagonally implicit A for the source), one
// of the two pairs of App. C:
//   imex 1: HT(1,1,2) (eq. ht112.butcher), second order;
//   imex 2: SSP3-IMEX(4,3,3) of Pareschi and Russo (eq. ssp33.butcher), third
//           order, L-stable.  The printed implicit tableau is garbled: its
//           second and third rows do not sum to the printed nodes 0 and 1
//           (c_i = sum_j a_ij, §2), and its fourth row sums to 1/2, not the
//           printed 1.  The rows used, with the paper's alpha, beta, eta, are
//           (alpha), (-alpha, alpha), (0, 1 - alpha, alpha),
//           (beta, eta, 1/2 - beta - eta - alpha, alpha): nodes (alpha, 0, 1,
//           1/2), third order (the order conditions are pinned in the tests).
#pragma once
#include <vector>

namespace ora {

struct Tableau {
  int s = 1;
  std::vector<double> A;  // s*s, strictly lower triangular, A[i*s+j]
  std::vector<double> b;  // s
  int imex = 0;
  std::vector<double> Ai;  // implicit part, lower triangular with diagonal (imex only)
  std::vector<double> bi;

  explicit Tableau(int N, int imex_ = 0) : imex(imex_) {
    auto set = [&](int s_) { s = s_; A.assign(s * s, 0.0); b.assign(s, 0.0); Ai.assign(s * s, 0.0); bi.assign(s, 0.0); };
    auto a = [&](int i, int j, double v) { A[(i - 1) * s + (j - 1)] = v; };
    auto ai = [&](int i, int j, double v) { Ai[(i - 1) * s + (j - 1)] = v; };
    if (imex == 1) {
      set(2);
      a(2, 1, 1.0);
      b = {0.5, 0.5};
      ai(2, 1, 0.5); ai(2, 2, 0.5);
      bi = {0.5, 0.5};
      return;
    }
    if (imex == 2) {
      const double al = 0.241694260788, be = 0.0604235651970, et = 0.12915286960590;
      set(4);
      a(3, 2, 1.0);
      a(4, 2, 0.25); a(4, 3, 0.25);
      b = {0.0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
      ai(1, 1, al);
      ai(2, 1, -al); ai(2, 2, al);
      ai(3, 2, 1.0 - al); ai(3, 3, al);
      ai(4, 1, be); ai(4, 2, et); ai(4, 3, 0.5 - be - et - al); ai(4, 4, al);
      bi = {0.0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
      return;
    }
    switch (N) {
      case 0:
        set(1); b[0] = 1.0; break;
      case 1:
        set(2); a(2, 1, 1.0); b = {0.5, 0.5}; break;
      case 2:
        set(3); a(2, 1, 1.0); a(3, 1, 0.25); a(3, 2, 0.25);
        b = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}; break;
      case 3:
        set(4); a(2, 1, 0.5); a(3, 2, 0.5); a(4, 3, 1.0);
        b = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}; break;
      default:  // N = 4
        set(6);
        a(2, 1, 0.25);
        a(3, 1, 0.125); a(3, 2, 0.125);
        a(4, 2, -0.5); a(4, 3, 1.0);
        a(5, 1, 3.0 / 16.0); a(5, 4, 9.0 / 16.0);
        a(6, 1, -3.0 / 7.0); a(6, 2, 2.0 / 7.0); a(6, 3, 12.0 / 7.0); a(6, 4, -12.0 / 7.0); a(6, 5, 8.0 / 7.0);
        b = {7.0 / 90.0, 0.0, 32.0 / 90.0, 12.0 / 90.0, 32.0 / 90.0, 7.0 / 90.0};
        break;
    }
  }
};

}  // namespace ora
