// Reference element of the oracle.  TEST INFRASTRUCTURE ONLY.
//
// Solution points are the Gauss-Legendre (GL) nodes mapped to [0,1] (paper §2,
// eqs. ref.map and soln.points), the nodal basis is the Lagrange basis (eq.
// defn.lagrange), D_ij = l_j'(xi_i) (eq. diff.matrix), and the FR correction
// functions are the right/left Radau polynomials g_R, g_L of degree N+1 (paper
// §2 below eq. rusanov.wave.speed; Huynh 2007).  The variant of App. B uses the
// Gauss-Lobatto-Legendre (GLL) nodes with Huynh's g_2 correction functions.
// Everything is evaluated in long double from the definitions written out,
// then rounded to double.
#pragma once
#include <cmath>
#include <vector>

namespace ora {
typedef long double ld;

// Legendre polynomial P_k and its derivative on [-1,1] (three-term recurrence;
// P'_{n+1} = P'_{n-1} + (2n+1) P_n).
inline void legendre(int k, ld x, ld& P, ld& dP) {
  if (k == 0) { P = 1; dP = 0; return; }
  ld p0 = 1, p1 = x, d0 = 0, d1 = 1;
  for (int n = 1; n < k; ++n) {
    ld p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
    ld d2 = d0 + (2 * n + 1) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  P = p1; dP = d1;
}

struct RefElem {
  int N = 0, n1 = 1;
  std::vector<double> xi, w;     // nodes / weights on [0,1]
  std::vector<double> D;         // D[i*n1+j] = l_j'(xi_i)
  std::vector<double> VL, VR;    // l_p(0), l_p(1)
  std::vector<double> gLp, gRp;  // d g_L/d xi (xi_p), d g_R/d xi (xi_p)
  std::vector<double> Leg;       // orthonormal Legendre on [0,1]: Leg[k*n1+p] = L_k(xi_p)

  bool gll = false;

  explicit RefElem(int N_, bool gll_ = false) : N(N_), n1(N_ + 1), gll(gll_) {
    std::vector<ld> x(n1), W(n1);
    const ld pi = 3.14159265358979323846264338327950288L;
    if (gll) {
      // GLL nodes: z = -1, 1 and the roots of P_N'; P_N'' from Legendre's
      // equation (1 - z^2) P'' = 2 z P' - N(N+1) P; Newton from the
      // Chebyshev-Gauss-Lobatto guess.  Weights 2/(N(N+1) P_N(z)^2) on [-1,1].
      for (int i = 0; i < n1; ++i) {
        ld z = -std::cos(pi * i / N);
        if (i > 0 && i < N) {
          for (int it = 0; it < 100; ++it) {
            ld P, dP;
            legendre(N, z, P, dP);
            const ld d2P = (2 * z * dP - N * (N + 1) * P) / (1 - z * z);
            const ld dz = dP / d2P;
            z -= dz;
            if (std::fabs(dz) < 1e-30L) break;
          }
        }
        ld P, dP;
        legendre(N, z, P, dP);
        x[i] = (1 + z) / 2;
        W[i] = 1 / ((ld)N * (N + 1) * P * P);
      }
    }
    // GL nodes = roots of P_{N+1}; Newton from the classical cosine guess.
    for (int i = 0; i < n1 && !gll; ++i) {
      ld z = std::cos(pi * (i + 0.75L) / (n1 + 0.5L));
      for (int it = 0; it < 100; ++it) {
        ld P, dP;
        legendre(n1, z, P, dP);
        ld dz = P / dP;
        z -= dz;
        if (std::fabs(dz) < 1e-30L) break;
      }
      ld P, dP;
      legendre(n1, z, P, dP);
      // descending z -> ascending xi = (1 - z)/2 ; weight 2/((1-z^2)P'^2) halved for [0,1]
      x[i] = (1 - z) / 2;
      W[i] = 1 / ((1 - z * z) * dP * dP);
    }
    xi.resize(n1); w.resize(n1);
    for (int i = 0; i < n1; ++i) { xi[i] = (double)x[i]; w[i] = (double)W[i]; }

    // Lagrange basis by its product definition
    auto lag = [&](int j, ld t) {
      ld r = 1;
      for (int k = 0; k < n1; ++k) if (k != j) r *= (t - x[k]) / (x[j] - x[k]);
      return r;
    };
    D.assign(n1 * n1, 0.0);
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j) {
        ld v;
        if (i == j) {
          v = 0;
          for (int k = 0; k < n1; ++k) if (k != j) v += 1 / (x[j] - x[k]);
        } else {
          ld num = 1, den = 1;
          for (int k = 0; k < n1; ++k) {
            if (k != j) den *= (x[j] - x[k]);
            if (k != j && k != i) num *= (x[i] - x[k]);
          }
          v = num / den;
        }
        D[i * n1 + j] = (double)v;
      }
    VL.resize(n1); VR.resize(n1);
    for (int p = 0; p < n1; ++p) { VL[p] = (double)lag(p, 0); VR[p] = (double)lag(p, 1); }

    // Correction functions on [-1,1], z = 2 xi - 1, d/dxi = 2 d/dz.  With the
    // left Radau polynomial of degree k, R_k(z) = (-1)^k (P_k(z) - P_{k-1}(z))/2
    // (R_k(-1) = 1, R_k(1) = 0):
    //   GL (g_DG):  g_L = R_{N+1};
    //   GLL (g_2):  g_L = ((N+1) R_N + N R_{N+1}) / (2N+1);
    // and g_R(z) = g_L(-z), so g_R'(z) = -g_L'(-z).
    auto dRk = [](int k, ld z) {  // dR_k/dz
      ld Pa, dPa, Pb, dPb;
      legendre(k, z, Pa, dPa);
      legendre(k - 1, z, Pb, dPb);
      const ld sgn = (k % 2 == 0) ? 1 : -1;
      return sgn * (dPa - dPb) / 2;
    };
    auto dgL = [&](ld z) {
      if (!gll) return dRk(N + 1, z);
      return ((N + 1) * dRk(N, z) + N * dRk(N + 1, z)) / (2 * N + 1);
    };
    gLp.resize(n1); gRp.resize(n1);
    for (int p = 0; p < n1; ++p) {
      const ld z = 2 * x[p] - 1;
      gLp[p] = (double)(2 * dgL(z));
      gRp[p] = (double)(-2 * dgL(-z));
    }
    // orthonormal Legendre on [0,1]: L_k(xi) = sqrt(2k+1) P_k(2 xi - 1)
    Leg.assign(n1 * n1, 0.0);
    for (int k = 0; k < n1; ++k)
      for (int p = 0; p < n1; ++p) {
        ld P, dP;
        legendre(k, 2 * x[p] - 1, P, dP);
        Leg[k * n1 + p] = (double)(std::sqrt((ld)(2 * k + 1)) * P);
      }
  }
};

}  // namespace ora
