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
#pragma once
#include <vector>

namespace ora {

struct Tableau {
  int s = 1;
  std::vector<double> A;  // s*s, strictly lower triangular, A[i*s+j]
  std::vector<double> b;  // s

  explicit Tableau(int N) {
    auto set = [&](int s_) { s = s_; A.assign(s * s, 0.0); b.assign(s, 0.0); };
    auto a = [&](int i, int j, double v) { A[(i - 1) * s + (j - 1)] = v; };
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
