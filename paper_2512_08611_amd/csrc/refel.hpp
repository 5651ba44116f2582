// Host-side reference element, tableaux and Fourier CFL number of the library.
//
// Solution points: Gauss-Legendre nodes on [0,1] (paper §2 eq. soln.points),
// found by Newton's method on P_{N+1} from Chebyshev starting points; weights
// 1/((1-z^2) P'_{N+1}(z)^2) mapped to [0,1].  Or, for the variant of App. B,
// Gauss-Lobatto-Legendre nodes: the ends and the roots of P_N' (Newton, P_N''
// from Legendre's equation), weights 1/(N(N+1) P_N(z)^2) on [0,1].  Lagrange
// data use the barycentric form: D_ij = (l_j/l_i)/(x_i - x_j),
// D_ii = -sum_{j!=i} D_ij (eq. diff.matrix); the correction slopes use App. B
// eq. correction.identities, g_R'(xi_p) = l_p(1)/w_p and g_L'(xi_p) = -l_p(0)/w_p
// (Radau correction with GL points, g_2 with GLL points).
#pragma once
#include <cmath>
#include <complex>
#include <vector>

namespace lwfr {

constexpr int kMaxN1 = 5;

struct RefData {
  int N, n1;
  double xi[kMaxN1], w[kMaxN1];
  double D[kMaxN1][kMaxN1];
  double VL[kMaxN1], VR[kMaxN1];
  double gL[kMaxN1], gR[kMaxN1];
  double Leg[kMaxN1][kMaxN1];  // Leg[k][p] = sqrt(2k+1) P_k(2 xi_p - 1)
};

inline void legendre_pair(int n, double z, double& P, double& dP) {
  // P_n(z) and P_n'(z) by the recurrence n P_n = (2n-1) z P_{n-1} - (n-1) P_{n-2}
  double pm1 = 1.0, p = z;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double pn = ((2.0 * k - 1.0) * z * p - (k - 1.0) * pm1) / k;
    pm1 = p;
    p = pn;
  }
  P = p;
  dP = n * (z * p - pm1) / (z * z - 1.0);
}

inline RefData make_refdata(int N, bool gll = false) {
  RefData r{};
  r.N = N;
  r.n1 = N + 1;
  const int n = N + 1;
  const double pi = 3.141592653589793238462643;
  if (gll && N >= 1) {
    for (int i = 0; i < n; ++i) {
      double z = i == 0 ? -1.0 : i == N ? 1.0 : -std::cos(pi * i / N);
      double P, dP;
      if (i > 0 && i < N) {
        for (int it = 0; it < 60; ++it) {
          legendre_pair(N, z, P, dP);
          const double d2P = (2.0 * z * dP - N * (N + 1.0) * P) / (1.0 - z * z);
          const double dz = dP / d2P;
          z -= dz;
          if (std::fabs(dz) < 1e-17) break;
        }
        legendre_pair(N, z, P, dP);
      } else {
        P = (i == 0 && N % 2 == 1) ? -1.0 : 1.0;  // P_N(+-1) = (+-1)^N
      }
      r.xi[i] = 0.5 * (z + 1.0);
      r.w[i] = 1.0 / (N * (N + 1.0) * P * P);
    }
  }
  for (int i = 0; i < n && !(gll && N >= 1); ++i) {
    // ascending nodes: start from -cos(pi (2i+1)/(2n))
    double z = -std::cos(pi * (2.0 * i + 1.0) / (2.0 * n));
    double P, dP;
    for (int it = 0; it < 60; ++it) {
      legendre_pair(n, z, P, dP);
      const double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    legendre_pair(n, z, P, dP);
    r.xi[i] = 0.5 * (z + 1.0);
    r.w[i] = 1.0 / ((1.0 - z * z) * dP * dP);
  }
  if (n == 1) { r.xi[0] = 0.5; r.w[0] = 1.0; }
  // barycentric weights
  double lam[kMaxN1];
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (r.xi[j] - r.xi[k]);
    lam[j] = 1.0 / prod;
  }
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      r.D[i][j] = (lam[j] / lam[i]) / (r.xi[i] - r.xi[j]);
      diag -= r.D[i][j];
    }
    r.D[i][i] = diag;
  }
  for (int end = 0; end < 2; ++end) {
    const double x = end;
    double* V = end ? r.VR : r.VL;
    int at = -1;  // an end that is itself a node (GLL): l_j(x) = delta
    for (int j = 0; j < n; ++j)
      if (x == r.xi[j]) at = j;
    if (at >= 0) {
      for (int j = 0; j < n; ++j) V[j] = j == at ? 1.0 : 0.0;
      continue;
    }
    double den = 0.0, num[kMaxN1];
    for (int j = 0; j < n; ++j) { num[j] = lam[j] / (x - r.xi[j]); den += num[j]; }
    for (int j = 0; j < n; ++j) V[j] = num[j] / den;
  }
  for (int p = 0; p < n; ++p) {
    r.gR[p] = r.VR[p] / r.w[p];
    r.gL[p] = -r.VL[p] / r.w[p];
  }
  for (int k = 0; k < n; ++k)
    for (int p = 0; p < n; ++p) {
      double P, dP;
      legendre_pair(k, 2.0 * r.xi[p] - 1.0, P, dP);
      r.Leg[k][p] = std::sqrt(2.0 * k + 1.0) * (k == 0 ? 1.0 : P);
    }
  return r;
}

// Fourier limit of the linearised step for u_t + u_x = 0 (wave speed 1,
// nu = dt/dx): the time average is T u with T = sum_{k<=N} (-nu D)^k/(k+1)!
// (the Taylor weights an order N+1 tableau reproduces), the Rusanov flux is the
// upwind trace, and the update is u_e <- u_e - nu [D T u_e + g_L (V_R.T u_{e-1}
// - V_L.T u_e)].  CFL(N) is the largest nu whose amplification matrices keep
// every eigenvalue in the unit disc for all Fourier angles.  Eigenvalues come
// from the characteristic polynomial (Faddeev-LeVerrier) and a Durand-Kerner
// iteration on its roots.
namespace detail {
using cplx = std::complex<double>;

inline double spectral_radius(int n, const cplx A[kMaxN1][kMaxN1]) {
  // characteristic polynomial z^n + c1 z^{n-1} + ... + cn by Faddeev-LeVerrier
  cplx Mk[kMaxN1][kMaxN1] = {}, AM[kMaxN1][kMaxN1];
  cplx c[kMaxN1 + 1];
  c[0] = 1.0;
  for (int i = 0; i < n; ++i) Mk[i][i] = 1.0;
  for (int k = 1; k <= n; ++k) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cplx s = 0.0;
        for (int l = 0; l < n; ++l) s += A[i][l] * Mk[l][j];
        AM[i][j] = s;
      }
    cplx tr = 0.0;
    for (int i = 0; i < n; ++i) tr += AM[i][i];
    c[k] = -tr / double(k);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Mk[i][j] = AM[i][j] + (i == j ? c[k] : cplx(0.0));
  }
  // Durand-Kerner
  cplx z[kMaxN1];
  const cplx seed(0.4, 0.9);
  for (int i = 0; i < n; ++i) z[i] = std::pow(seed, i);
  for (int it = 0; it < 500; ++it) {
    double change = 0.0;
    for (int i = 0; i < n; ++i) {
      cplx pv = 1.0;
      for (int k = 1; k <= n; ++k) pv = pv * z[i] + c[k];
      cplx den = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != i) den *= (z[i] - z[j]);
      const cplx dz = pv / den;
      z[i] -= dz;
      change = std::fmax(change, std::abs(dz));
    }
    if (change < 1e-15) break;
  }
  double rho = 0.0;
  for (int i = 0; i < n; ++i) rho = std::fmax(rho, std::abs(z[i]));
  return rho;
}

// explicit tableau (s stages, A row-major s x s, weights b) for the time average
struct ExplicitTab {
  int s = 0;
  double A[6][6] = {};
  double b[6] = {};
};

// growth factor of the linear scheme at Courant number nu: the time average is
// U = T u with T = sum_k (-nu D)^k/(k+1)! (an order N+1 tableau), or, for tab,
// T = sum_i b_i R_i with R_1 = I, R_i = I + sum_{k<i} A_ik (-nu D) R_k
inline double max_growth(const RefData& r, double nu, const ExplicitTab* tab = nullptr) {
  const int n = r.n1;
  double T[kMaxN1][kMaxN1] = {}, Pk[kMaxN1][kMaxN1] = {}, tmp[kMaxN1][kMaxN1];
  if (!tab) {
    for (int i = 0; i < n; ++i) Pk[i][i] = 1.0;
    double fact = 1.0;
    for (int k = 0; k <= r.N; ++k) {
      fact *= (k + 1);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) T[i][j] += Pk[i][j] / fact;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double s = 0.0;
          for (int l = 0; l < n; ++l) s += Pk[i][l] * (-nu * r.D[l][j]);
          tmp[i][j] = s;
        }
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Pk[i][j] = tmp[i][j];
    }
  } else {
    static thread_local double R[6][kMaxN1][kMaxN1];
    for (int st = 0; st < tab->s; ++st) {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) R[st][i][j] = i == j ? 1.0 : 0.0;
      for (int k = 0; k < st; ++k) {
        if (tab->A[st][k] == 0.0) continue;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int l = 0; l < n; ++l) acc += -nu * r.D[i][l] * R[k][l][j];
            R[st][i][j] += tab->A[st][k] * acc;
          }
      }
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) T[i][j] += tab->b[st] * R[st][i][j];
    }
  }
  double DT[kMaxN1][kMaxN1], RT[kMaxN1], LT[kMaxN1];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += r.D[i][l] * T[l][j];
      DT[i][j] = s;
    }
  for (int j = 0; j < n; ++j) {
    double sr = 0.0, sl = 0.0;
    for (int l = 0; l < n; ++l) { sr += r.VR[l] * T[l][j]; sl += r.VL[l] * T[l][j]; }
    RT[j] = sr; LT[j] = sl;
  }
  double worst = 0.0;
  const int nth = 720;
  for (int t = 1; t <= nth; ++t) {
    const double th = 3.141592653589793 * t / nth;
    const cplx ph = std::polar(1.0, -th);
    cplx G[kMaxN1][kMaxN1];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        G[i][j] = (i == j ? 1.0 : 0.0) - nu * (DT[i][j] + r.gL[i] * (ph * RT[j] - LT[j]));
    worst = std::fmax(worst, spectral_radius(n, G));
  }
  return worst;
}
}  // namespace detail

inline double fourier_cfl(int N, bool gll = false, const detail::ExplicitTab* tab = nullptr) {
  const RefData r = make_refdata(N, gll);
  // degree 4: order-5 Taylor weights give nearly undamped modes a weak growth
  // (about 5e-6 per step below the limit); the limit is the sharp loss of
  // stability of the high-frequency modes
  const double tol = N <= 3 ? 1e-11 : 1e-5;
  double lo = 0.0, hi = 1.5;
  while (hi - lo > 1e-9) {
    const double mid = 0.5 * (lo + hi);
    if (detail::max_growth(r, mid, tab) <= 1.0 + tol) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Explicit tableaux (A, b) of order N+1 used for the inner stages (paper §2
// eq. crkfr.inner, explicit part only): N=1 Heun (HT(1,1,2), App. C),
// N=2 SSPRK(3,3) (explicit part of SSP3-IMEX(4,3,3), App. C), N=3 classical
// RK4, N=4 Butcher's six-stage fifth-order method.
// Non-IMEX tableaux have no implicit part (ai, bi are zero; unused).
template <int N> struct Tableau;
template <> struct Tableau<1> {
  static constexpr int S = 2;
  static constexpr double ai(int, int) { return 0.0; }
  static constexpr double bi(int) { return 0.0; }
  static constexpr double a(int i, int j) { return (i == 1 && j == 0) ? 1.0 : 0.0; }
  static constexpr double b(int j) { return 0.5; }
};
template <> struct Tableau<2> {
  static constexpr int S = 3;
  static constexpr double ai(int, int) { return 0.0; }
  static constexpr double bi(int) { return 0.0; }
  static constexpr double a(int i, int j) {
    return (i == 1 && j == 0) ? 1.0 : (i == 2 && j < 2) ? 0.25 : 0.0;
  }
  static constexpr double b(int j) { return j == 2 ? 2.0 / 3.0 : 1.0 / 6.0; }
};
template <> struct Tableau<3> {
  static constexpr int S = 4;
  static constexpr double ai(int, int) { return 0.0; }
  static constexpr double bi(int) { return 0.0; }
  static constexpr double a(int i, int j) { return (i == j + 1) ? (i == 3 ? 1.0 : 0.5) : 0.0; }
  static constexpr double b(int j) { return (j == 0 || j == 3) ? 1.0 / 6.0 : 1.0 / 3.0; }
};
template <> struct Tableau<4> {
  static constexpr int S = 6;
  static constexpr double ai(int, int) { return 0.0; }
  static constexpr double bi(int) { return 0.0; }
  static constexpr double a(int i, int j) {
    return i == 1 ? (j == 0 ? 0.25 : 0.0)
         : i == 2 ? (j < 2 ? 0.125 : 0.0)
         : i == 3 ? (j == 1 ? -0.5 : j == 2 ? 1.0 : 0.0)
         : i == 4 ? (j == 0 ? 3.0 / 16.0 : j == 3 ? 9.0 / 16.0 : 0.0)
         : i == 5 ? (j == 0 ? -3.0 / 7.0 : j == 1 ? 2.0 / 7.0 : j == 2 ? 12.0 / 7.0 : j == 3 ? -12.0 / 7.0
                                                                              : j == 4 ? 8.0 / 7.0 : 0.0)
                  : 0.0;
  }
  static constexpr double b(int j) {
    return (j == 0 || j == 5) ? 7.0 / 90.0 : (j == 2 || j == 4) ? 32.0 / 90.0 : j == 3 ? 12.0 / 90.0 : 0.0;
  }
};

// IMEX pairs of App. C for systems with a stiff source (§2 eq. crkfr.inner):
// explicit part (a, b) on the local flux terms, diagonally implicit part
// (ai, bi) on the source.
//   ImexHT:   HT(1,1,2) (eq. ht112.butcher): Heun with the trapezoidal rule.
//   ImexSSP3: SSP3-IMEX(4,3,3) of Pareschi and Russo (eq. ssp33.butcher), with
//             the implicit rows (alpha), (-alpha, alpha), (0, 1-alpha, alpha),
//             (beta, eta, 1/2-beta-eta-alpha, alpha): the printed rows are
//             garbled, these satisfy c_i = sum_j a_ij and the order conditions.
struct ImexHT {
  static constexpr int S = 2;
  static constexpr double a(int i, int j) { return (i == 1 && j == 0) ? 1.0 : 0.0; }
  static constexpr double b(int) { return 0.5; }
  static constexpr double ai(int i, int j) { return i == 1 ? 0.5 : 0.0; }
  static constexpr double bi(int) { return 0.5; }
};
struct ImexSSP3 {
  static constexpr int S = 4;
  static constexpr double kA = 0.241694260788, kB = 0.0604235651970, kE = 0.12915286960590;
  static constexpr double a(int i, int j) { return i == 2 ? (j == 1 ? 1.0 : 0.0) : i == 3 ? (j == 1 || j == 2 ? 0.25 : 0.0) : 0.0; }
  static constexpr double b(int j) { return j == 0 ? 0.0 : j == 3 ? 2.0 / 3.0 : 1.0 / 6.0; }
  static constexpr double ai(int i, int j) {
    return i == j ? kA
         : i == 1 ? (j == 0 ? -kA : 0.0)
         : i == 2 ? (j == 1 ? 1.0 - kA : 0.0)
         : i == 3 ? (j == 0 ? kB : j == 1 ? kE : j == 2 ? 0.5 - kB - kE - kA : 0.0)
                  : 0.0;
  }
  static constexpr double bi(int j) { return b(j); }
};

// Fourier limit of degree N with the explicit part of IMEX pair Tab
template <class Tab>
inline double fourier_cfl_imex(int N, bool gll) {
  detail::ExplicitTab t;
  t.s = Tab::S;
  for (int i = 0; i < Tab::S; ++i) {
    t.b[i] = Tab::b(i);
    for (int j = 0; j < i; ++j) t.A[i][j] = Tab::a(i, j);
  }
  return fourier_cfl(N, gll, &t);
}

}  // namespace lwfr
