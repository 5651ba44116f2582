// One time step of the time-averaged compact Runge-Kutta flux reconstruction
// scheme for u_t + f(u)_x + B(u) u_x = 0 with the subcell-FV blend and the
// admissibility limiters.  TEST INFRASTRUCTURE ONLY: a plain, slow, obviously
// correct CPU reference; nothing in the product path may use it.
//
// The step follows the paper in this order:
//   1. element means and time step (§5 eq. time.step.2d, Def. of admissibility
//      in means), GLM cleaning speed c_h (§5.5 below eq. glm.mhd);
//   2. smoothness indicator alpha_e (§4 eq. blended.scheme and the indicator of
//      Hennemann et al. it cites);
//   3. element-local stages (§3 eq. crkfr.non.cons.final with the inner stages
//      above it), time averages F (eq. disc.avg.flux), U (eq. time.avg.soln),
//      B^loc (eq. local.time.avg.non.cons) and the face values F^nc (§3 below
//      eq. local.time.avg.non.cons);
//   4. interface fluxes: F^num (eq. numflux.cons with the wave speed of eq.
//      combined.wave.speed), the non-conservative part B(u^{n,±}) U^num (eq.
//      good.numflux.non.cons), the lower order fluxes (eqs. combined.num.flux,
//      numflux.args), the blend of eq. Fblend and Algorithm 1;
//   5. high order update (eq. crkfr.non.cons.final), lower order subcell update
//      (eq. low.order.update), blend (eq. blended.scheme) and Algorithm 2.
// Readings of points the paper leaves open are listed in the design notes
// (time-step CFL(N), c_h, the indicator constants, the 2-D form of Alg. 1, the
// theta convention).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "physics.hpp"
#include "refel.hpp"
#include "scalar.hpp"
#include "tableau.hpp"

namespace ora {

struct Config {
  int eq, N, nx, ny;
  double lo[2], hi[2];
  double gamma, gravity;
  double cs, cfl;  // safety factor C_s and CFL(N) of eq. time.step.2d
  int blending;    // 0: pure high order; 1: indicator blend; 2: blend + Alg. 1 + Alg. 2
  double alpha_max, alpha_min;
  double alpha_force;  // >= 0: every alpha_e is set to this value (tests, residual modes)
  int gll = 0;         // 1: Gauss-Lobatto-Legendre solution points with g_2 correction (App. B)
  int imex = 0;        // IMEX pair of a system with a source (tableau.hpp): 1 HT(1,1,2), 2 SSP3-IMEX(4,3,3)
  int alw = 0;         // 1: time averages by the approximate Lax-Wendroff procedure (stages_alw)
  // threads of the element and face loops (OpenMP; 1 = serial).  Every element's
  // and face's arithmetic is the same for any count, and each writes only its
  // own entries, so results are bit for bit the same.
  int threads = 1;
  // Jin-Xin characteristic speed a, relaxation time eps, f(u) = l u + q u^2/2
  double relax_a = 3.0, relax_eps = 1e-2, relax_l = 0.0, relax_q = 1.0;
  // boundary condition of side (d, s): BC_PERIODIC, BC_OUTFLOW (the ghost copies
  // the inside face), BC_WALL (mirror with the normal momentum reversed; shallow
  // water only), BC_DIRICHLET (ghost face data given in `ghost`).  A direction is
  // periodic on both sides or on neither.
  int bc[2][2] = {{0, 0}, {0, 0}};
  // BC_DIRICHLET data: for boundary b = 2 d + s, block b of 3*M*NB_d values,
  // [quantity][v][j] with quantity 0 = u^n at the face (also the outside subcell
  // state), 1 = U (time average), 2 = F_d (time-averaged d-flux), j = position
  // along the boundary (line index * nfp + q); NB_d = lines * nfp.
  const double* ghost = nullptr;
};

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_WALL = 2, BC_DIRICHLET = 3 };

enum : uint32_t {
  FLAG_ALG2 = 1u,          // Algorithm 2 limited the element (theta < 1)
  FLAG_LOW_INADM = 2u,     // the lower order update u^L is not admissible somewhere
  FLAG_ALG1 = 4u,          // Algorithm 1 limited a flux on one of the element's faces
  FLAG_NONFINITE = 8u,     // u^{n+1} holds a non-finite value
  FLAG_ALG1_GUARD = 16u,   // Algorithm 1 met an inadmissible lower order candidate
};

// theta_{P_k}(eps, u_a, u_b) of eq. theta.adk for a concave P_k (eq.
// theta.formula), written with the weight on the candidate u_b: the limited
// state is theta u_b + (1 - theta) u_a.  Admissible candidates keep theta = 1.
inline double theta_concave(double eps, double Pa, double Pb, bool& guard) {
  if (Pa <= 0.0) { guard = true; return 0.0; }
  if (Pb >= eps) return 1.0;
  return std::min(1.0, std::fabs((eps - Pa) / (Pb - Pa)));
}

template <class Phys>
struct Scheme {
  static constexpr int M = Phys::M, DIM = Phys::DIM, K = Phys::K;
  const Phys& ph;
  Config cfg;
  RefElem re;
  Tableau tb;
  int N, n1, P, nx, ny, E, nfp;
  double dx[2];

  Scheme(const Phys& p, const Config& c)
      : ph(p), cfg(c), re(c.N, c.gll != 0), tb(c.N, c.imex), N(c.N), n1(c.N + 1) {
    P = DIM == 1 ? n1 : n1 * n1;
    nfp = DIM == 1 ? 1 : n1;
    nx = c.nx; ny = DIM == 1 ? 1 : c.ny;
    E = nx * ny;
    dx[0] = (c.hi[0] - c.lo[0]) / nx;
    dx[1] = DIM == 1 ? 1.0 : (c.hi[1] - c.lo[1]) / ny;
  }

  int nthreads() const { return cfg.threads > 0 ? cfg.threads : 1; }

  // ---------------------------------------------------------------- mesh ---
  size_t idx(int v, int e, int p) const { return ((size_t)v * E + e) * P + p; }
  // neighbour across the upper (side=1) or lower (side=0) face in direction d
  int nbr(int e, int d, int side) const {
    int ex = e % nx, ey = e / nx;
    if (d == 0) ex = side ? (ex + 1) % nx : (ex + nx - 1) % nx;
    else ey = side ? (ey + 1) % ny : (ey + ny - 1) % ny;
    return ex + nx * ey;
  }
  // element e lies on the non-periodic side (d, side) of the domain
  bool on_boundary(int e, int d, int side) const {
    if (cfg.bc[d][side] == BC_PERIODIC) return false;
    int ex = e % nx, ey = e / nx;
    int c = d == 0 ? ex : ey, n = d == 0 ? nx : ny;
    return side ? c == n - 1 : c == 0;
  }
  // position along boundary (d, side) of face point q of element e
  int bpos(int e, int d, int q) const { return (d == 0 ? e / nx : e % nx) * nfp + q; }
  int blines(int d) const { return d == 0 ? ny : nx; }
  // node with position r along direction d on line q
  int node(int d, int q, int r) const { return d == 0 ? r + n1 * q : q + n1 * r; }
  int pos(int d, int p) const { return d == 0 ? p % n1 : p / n1; }
  int line(int d, int p) const { return d == 0 ? p / n1 : p % n1; }
  double wnode(int p) const { return DIM == 1 ? re.w[p] : re.w[p % n1] * re.w[p / n1]; }
  size_t fidx(int d, int v, int e, int q) const { return (((size_t)d * M + v) * E + e) * nfp + q; }

  // ------------------------------------------------- 1. means, dt and c_h ---
  template <class T>
  void mean(const T* u, int e, T* ub) const {
    for (int v = 0; v < M; ++v) {
      T s = T(0.0);
      for (int p = 0; p < P; ++p) s = s + T(wnode(p)) * u[idx(v, e, p)];
      ub[v] = s;
    }
  }
  // Lambda = max_e sum_d (|v_d| + c_d)(ubar_e)/dx_d with the ideal (non-GLM)
  // speeds; dt = C_s CFL(N) / Lambda (eq. time.step.2d).  For GLM-MHD c_h is the
  // largest value whose waves |v_d| + max(c_f, c_h) leave Lambda unchanged.
  // (T: double, or the counting scalar for operation counts; the counting run is serial)
  template <class T>
  void dt_ch(const T* u, double& dt, double& ch) const {
    double Lam = 0;
#pragma omp parallel for num_threads(nthreads()) schedule(static) reduction(max : Lam)
    for (int e = 0; e < E; ++e) {
      T ub[M];
      mean(u, e, ub);
      T s = T(0.0);
      for (int d = 0; d < DIM; ++d) {
        T av, c;
        ph.speeds(d, ub, av, c);
        s = s + (av + c) / T(dx[d]);
      }
      Lam = std::max(Lam, val(s));
    }
    dt = val(T(cfg.cs * cfg.cfl) / T(Lam));
    ch = 0.0;
    if (cfg.eq == EQ_MHD2D) {
      double best = INFINITY;
#pragma omp parallel for num_threads(nthreads()) schedule(static) reduction(min : best)
      for (int e = 0; e < E; ++e) {
        T ub[M];
        mean(u, e, ub);
        T av[2], c[2];
        for (int d = 0; d < 2; ++d) ph.speeds(d, ub, av[d], c[d]);
        const T wx = T(1.0 / dx[0]), wy = T(1.0 / dx[1]);
        T R = T(Lam) - (av[0] * wx + av[1] * wy);
        // largest c with wx max(c_x, c) + wy max(c_y, c) <= R
        T lo = c[0], hi = c[1], wlo = wx, whi = wy;
        if (val(lo) > val(hi)) { std::swap(lo, hi); std::swap(wlo, whi); }
        T ce = val((wlo + whi) * hi) >= val(R) ? (R - whi * hi) / wlo : R / (wlo + whi);
        best = std::min(best, val(ce));
      }
      ch = best;
    }
  }

  // ---------------------------------------------------- 2. indicator -------
  // Modal energy indicator: E = max of the energy fractions of the highest and
  // second highest modes of the indicator variable in orthonormal Legendre
  // modes; alpha = logistic((s/T)(E - T)), T(N) = 0.5 10^{-1.8 (N+1)^{1/4}},
  // s = ln(9999); clip below alpha_min / above 1-alpha_min, cap alpha_max;
  // smoothing alpha_e <- max(alpha_e, alpha_nb/2) over face neighbours.
  template <class T>
  void indicator(const T* u, std::vector<double>& araw, std::vector<double>& alpha,
                 std::vector<uint8_t>& tie) const {
    araw.assign(E, 0.0); alpha.assign(E, 0.0); tie.assign(E, 0);
    if (cfg.alpha_force >= 0.0) { alpha.assign(E, cfg.alpha_force); araw = alpha; return; }
    if (cfg.blending == 0 || N == 0) return;
    const double Tn = 0.5 * std::pow(10.0, -1.8 * std::pow(N + 1.0, 0.25));
    const double s = std::log(9999.0);
#pragma omp parallel for num_threads(nthreads()) schedule(static)
    for (int e = 0; e < E; ++e) {
      std::vector<T> q(P), ue(M);
      for (int p = 0; p < P; ++p) {
        for (int v = 0; v < M; ++v) ue[v] = u[idx(v, e, p)];
        q[p] = ph.indicator(ue.data());
      }
      T tot = T(0.0), c1 = T(0.0), c2 = T(0.0);
      if (DIM == 1) {
        for (int k = 0; k < n1; ++k) {
          T m = T(0.0);
          for (int p = 0; p < n1; ++p) m = m + T(re.w[p]) * q[p] * T(re.Leg[k * n1 + p]);
          tot = tot + m * m;
          if (k <= N - 1) c1 = c1 + m * m;
          if (k <= N - 2) c2 = c2 + m * m;
        }
      } else {
        for (int l = 0; l < n1; ++l)
          for (int k = 0; k < n1; ++k) {
            T m = T(0.0);
            for (int j = 0; j < n1; ++j)
              for (int i = 0; i < n1; ++i)
                m = m + T(re.w[i]) * T(re.w[j]) * q[i + n1 * j] * T(re.Leg[k * n1 + i]) * T(re.Leg[l * n1 + j]);
            int deg = std::max(k, l);
            tot = tot + m * m;
            if (deg <= N - 1) c1 = c1 + m * m;
            if (deg <= N - 2) c2 = c2 + m * m;
          }
      }
      T En = val(tot) > 0 ? (tot - c1) / tot : T(0.0);
      if (N >= 2) {
        T E2 = val(c1) > 0 ? (c1 - c2) / c1 : T(0.0);
        if (val(E2) > val(En)) En = E2;
      }
      double a = val(T(1.0) / (T(1.0) + exp(-T(s / Tn) * (En - T(Tn)))));
      if (std::fabs(a - cfg.alpha_min) < 1e-9 || std::fabs(a - (1.0 - cfg.alpha_min)) < 1e-9) tie[e] = 1;
      if (a < cfg.alpha_min) a = 0.0;
      if (a > 1.0 - cfg.alpha_min) a = 1.0;
      a = std::min(a, cfg.alpha_max);
      araw[e] = a;
    }
    for (int e = 0; e < E; ++e) {
      double a = araw[e];
      for (int d = 0; d < DIM; ++d)
        for (int sd = 0; sd < 2; ++sd)
          if (!on_boundary(e, d, sd)) a = std::max(a, 0.5 * araw[nbr(e, d, sd)]);
      alpha[e] = a;
    }
  }

  // ------------------------------------------ 3. element-local stages -----
  template <class T>
  struct Local {
    std::vector<T> F;    // [d][v][e][p] time-averaged flux F_d
    std::vector<T> U;    // [v][e][p] time-averaged solution
    std::vector<T> Bl;   // [v][e][p] B^loc
    std::vector<T> Fnc;  // [d][side][v][e][q]
    std::vector<T> Ftr, Utr, untr;  // traces [d][side][v][e][q]
    std::vector<T> S;    // [v][e][p] time-averaged source (eq. avg.source; systems with a source)
  };
  size_t tidx(int d, int side, int v, int e, int q) const {
    return ((((size_t)d * 2 + side) * M + v) * E + e) * nfp + q;
  }

  // the arrays of the element-local phase, zero
  // (the stage loop zeroes each element's entries before it accumulates them;
  // every trace entry is written by the face traces)
  template <class T>
  void alloc_local(Local<T>& L) const {
    L.F.resize((size_t)DIM * M * E * P);
    L.U.resize((size_t)M * E * P);
    L.Bl.resize((size_t)M * E * P);
    L.Fnc.resize((size_t)DIM * 2 * M * E * nfp);
    L.Ftr.resize(L.Fnc.size());
    L.Utr.resize(L.Fnc.size());
    L.untr.resize(L.Fnc.size());
    L.S.resize(Phys::SRC ? (size_t)M * E * P : 0);
  }
  // scratch of the stage loop of one element
  template <class T>
  struct StageScratch {
    std::vector<T> Lst, uj, f, Sst, a, fo, w, o, du, nc;
    explicit StageScratch(const Scheme& S)
        : Lst((size_t)S.tb.s * M * S.P), uj((size_t)M * S.P), f((size_t)DIM * M * S.P),
          Sst(Phys::SRC ? (size_t)S.tb.s * M * S.P : 0), a(M), fo(M), w(M), o(M), du(M), nc(M) {}
  };

  template <class T>
  void stages(const T* un, double dt, double ch, Local<T>& L) const {
    alloc_local(L);
#pragma omp parallel num_threads(nthreads())
    {
      StageScratch<T> W(*this);
#pragma omp for schedule(static)
      for (int e = 0; e < E; ++e) stages_elem(un, dt, ch, L, e, W);
    }
  }

  // the stages and time averages of element e (L's entries of e accumulate from zero)
  template <class T>
  void stages_elem(const T* un, double dt, double ch, Local<T>& L, int e, StageScratch<T>& W) const {
    const int s = tb.s;
    std::vector<T>& Lst = W.Lst;
    std::vector<T>& uj = W.uj;
    std::vector<T>& f = W.f;
    std::vector<T>& Sst = W.Sst;
    std::vector<T>& a = W.a;
    std::vector<T>& fo = W.fo;
    std::vector<T>& du = W.du;
    std::vector<T>& nc = W.nc;
    for (int v = 0; v < M; ++v)
      for (int p = 0; p < P; ++p) {
        L.U[idx(v, e, p)] = T(0.0);
        L.Bl[idx(v, e, p)] = T(0.0);
        if constexpr (Phys::SRC) L.S[idx(v, e, p)] = T(0.0);
        for (int d = 0; d < DIM; ++d) L.F[(size_t)d * M * E * P + idx(v, e, p)] = T(0.0);
      }
    {
      for (int j = 0; j < s; ++j) {
        // inner stage u^(j) = u^n - dt sum_{k<j} a_jk L^(k) (sum over the tableau's non-zero a_jk)
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            T acc = T(0.0);
            bool any = false;
            for (int k = 0; k < j; ++k)
              if (tb.A[j * s + k] != 0.0) {
                T t = T(tb.A[j * s + k]) * Lst[((size_t)k * M + v) * P + p];
                acc = any ? acc + t : t;
                any = true;
              }
            uj[(size_t)v * P + p] = any ? un[idx(v, e, p)] - T(dt) * acc : un[idx(v, e, p)];
          }
        if constexpr (Phys::SRC) {
          // implicit source part of eq. crkfr.inner: + dt sum_{k<j} a_jk s(u^(k)),
          // then u^(j) solves u - dt a_jj s(u) = (explicit part) when a_jj != 0
          for (int p = 0; p < P; ++p) {
            T r[M], x[M];
            for (int v = 0; v < M; ++v) {
              T acc = T(0.0);
              bool any = false;
              for (int k = 0; k < j; ++k)
                if (tb.Ai[j * s + k] != 0.0) {
                  T t = T(tb.Ai[j * s + k]) * Sst[((size_t)k * M + v) * P + p];
                  acc = any ? acc + t : t;
                  any = true;
                }
              r[v] = any ? uj[(size_t)v * P + p] + T(dt) * acc : uj[(size_t)v * P + p];
            }
            const double ajj = tb.Ai[j * s + j];
            if (ajj != 0.0) ph.implicit(r, dt * ajj, x);
            else for (int v = 0; v < M; ++v) x[v] = r[v];
            for (int v = 0; v < M; ++v) uj[(size_t)v * P + p] = x[v];
            ph.source(x, r);
            for (int v = 0; v < M; ++v) {
              Sst[((size_t)j * M + v) * P + p] = r[v];
              if (tb.bi[j] != 0.0) L.S[idx(v, e, p)] = L.S[idx(v, e, p)] + T(tb.bi[j]) * r[v];
            }
          }
        }
        // fluxes at the solution points
        for (int p = 0; p < P; ++p) {
          for (int v = 0; v < M; ++v) a[v] = uj[(size_t)v * P + p];
          for (int d = 0; d < DIM; ++d) {
            ph.flux(d, a.data(), fo.data(), ch);
            for (int v = 0; v < M; ++v) f[((size_t)d * M + v) * P + p] = fo[v];
          }
        }
        // L^(j) = sum_d [ D_d f_d + B_d(u) D_d u ] / dx_d  (local operator, eq. dlocx.defn)
        for (int p = 0; p < P; ++p) {
          for (int v = 0; v < M; ++v) a[v] = uj[(size_t)v * P + p];
          T Lp[M], Bp[M];
          for (int v = 0; v < M; ++v) { Lp[v] = T(0.0); Bp[v] = T(0.0); }
          for (int d = 0; d < DIM; ++d) {
            int i = pos(d, p), q = line(d, p);
            for (int v = 0; v < M; ++v) {
              T df = T(0.0);
              for (int r = 0; r < n1; ++r) df = df + T(re.D[i * n1 + r]) * f[((size_t)d * M + v) * P + node(d, q, r)];
              fo[v] = df;
              du[v] = T(0.0);
            }
            // D_d u for the columns of B_d that are not identically zero
            for (int c = 0; c < Phys::NCOL; ++c) {
              const int v = Phys::ncol(d, c);
              T dv = T(0.0);
              for (int r = 0; r < n1; ++r) dv = dv + T(re.D[i * n1 + r]) * uj[(size_t)v * P + node(d, q, r)];
              du[v] = dv;
            }
            ph.ncprod(d, a.data(), du.data(), nc.data());
            for (int v = 0; v < M; ++v) {
              Lp[v] = Lp[v] + (fo[v] + nc[v]) / T(dx[d]);
              Bp[v] = Bp[v] + nc[v] / T(dx[d]);
            }
          }
          for (int v = 0; v < M; ++v) {
            Lst[((size_t)j * M + v) * P + p] = Lp[v];
            if (tb.b[j] == 0.0) continue;  // stage with zero weight adds nothing
            T bj = T(tb.b[j]);
            L.U[idx(v, e, p)] = L.U[idx(v, e, p)] + bj * a[v];
            L.Bl[idx(v, e, p)] = L.Bl[idx(v, e, p)] + bj * Bp[v];
            for (int d = 0; d < DIM; ++d)
              L.F[(size_t)d * M * E * P + idx(v, e, p)] =
                  L.F[(size_t)d * M * E * P + idx(v, e, p)] + bj * f[((size_t)d * M + v) * P + p];
          }
        }
      }
    }
  }

  // ---------------- 3'. element-local time averages, approximate Lax-Wendroff ---
  // The Lax-Wendroff form of the time averages that the cRK stages reproduce
  // (§5: cRKFR is linearly equivalent to LWFR):
  //   F_d = sum_{k=0}^{N} dt^k/(k+1)! d_t^k f_d,  U = sum_k dt^k/(k+1)! d_t^k u,
  //   B^loc = sum_k dt^k/(k+1)! d_t^k [ sum_d B_d(u) u_{x_d} ],
  // with d_t^{k+1} u = -( sum_d D_d d_t^k f_d / dx_d + d_t^k [B u_x] ) (the local
  // operator) and d_t^k f, d_t^k [B u_x] from central differences in time of
  // f(u(tau)), B(u(tau)) D u(tau) at tau = j dt along the Taylor state
  // u(tau) = sum_{m<=k} tau^m/m! d_t^m u.  Stencils (derived from Taylor series,
  // order enough for the step's order N+1): j in {-1,0,1} for N <= 2,
  // {-2..2} for N >= 3;  dt^k d_t^k g ~
  //   k=1: (g1 - g-1)/2                | (-g2 + 8g1 - 8g-1 + g-2)/12
  //   k=2: g1 - 2g0 + g-1              | (-g2 + 16g1 - 30g0 + 16g-1 - g-2)/12
  //   k=3: (g2 - 2g1 + 2g-1 - g-2)/2
  //   k=4: g2 - 4g1 + 6g0 - 4g-1 + g-2
  static double fd_weight(int N, int k, int j) {
    if (k == 0) return j == 0 ? 1.0 : 0.0;
    if (N <= 2) {
      if (j < -1 || j > 1) return 0.0;
      if (k == 1) return 0.5 * j;
      return j == 0 ? -2.0 : 1.0;  // k == 2
    }
    static const double w[5][5] = {
        {0, 0, 1, 0, 0},
        {1.0 / 12, -8.0 / 12, 0, 8.0 / 12, -1.0 / 12},
        {-1.0 / 12, 16.0 / 12, -30.0 / 12, 16.0 / 12, -1.0 / 12},
        {-0.5, 1.0, 0, -1.0, 0.5},
        {1, -4, 6, -4, 1}};
    return w[k][j + 2];
  }

  template <class T>
  void stages_alw(const T* un, double dt, double ch, Local<T>& L) const {
    L.F.assign((size_t)DIM * M * E * P, T(0.0));
    L.U.assign((size_t)M * E * P, T(0.0));
    L.Bl.assign((size_t)M * E * P, T(0.0));
    L.Fnc.assign((size_t)DIM * 2 * M * E * nfp, T(0.0));
    L.Ftr.assign(L.Fnc.size(), T(0.0));
    L.Utr.assign(L.Fnc.size(), T(0.0));
    L.untr.assign(L.Fnc.size(), T(0.0));
    const int J = N <= 2 ? 1 : 2;  // stencil half width
    // c[m][v][p]: d_t^m u at the nodes; fk[d][v][p]: dt^k d_t^k f_d; hk[v][p]: dt^k d_t^k [B u_x]
    std::vector<T> c((size_t)(N + 1) * M * P), fk((size_t)DIM * M * P), hk((size_t)M * P);
    std::vector<T> st((size_t)M * P);
    T a[M], fo[M], du[M], nc[M];
    double fact = 1.0;
    for (int e = 0; e < E; ++e) {
      for (int v = 0; v < M; ++v)
        for (int p = 0; p < P; ++p) c[(size_t)v * P + p] = un[idx(v, e, p)];
      fact = 1.0;
      for (int k = 0; k <= N; ++k) {
        fact *= (k + 1);  // (k+1)!
        for (size_t i = 0; i < fk.size(); ++i) fk[i] = T(0.0);
        for (size_t i = 0; i < hk.size(); ++i) hk[i] = T(0.0);
        for (int j = -J; j <= J; ++j) {
          const double wj = fd_weight(N, k, j);
          if (wj == 0.0) continue;
          // Taylor state at tau = j dt truncated after d_t^k u
          for (int v = 0; v < M; ++v)
            for (int p = 0; p < P; ++p) {
              T sacc = c[(size_t)v * P + p];
              double tm = 1.0;
              for (int m = 1; m <= k; ++m) {
                tm *= (j * dt) / m;
                sacc = sacc + T(tm) * c[((size_t)m * M + v) * P + p];
              }
              st[(size_t)v * P + p] = sacc;
            }
          for (int p = 0; p < P; ++p) {
            for (int v = 0; v < M; ++v) a[v] = st[(size_t)v * P + p];
            for (int d = 0; d < DIM; ++d) {
              ph.flux(d, a, fo, ch);
              for (int v = 0; v < M; ++v) fk[((size_t)d * M + v) * P + p] = fk[((size_t)d * M + v) * P + p] + T(wj) * fo[v];
            }
            // B(u(tau)) D u(tau) / dx, summed over directions
            for (int d = 0; d < DIM; ++d) {
              int i = pos(d, p), q = line(d, p);
              for (int v = 0; v < M; ++v) du[v] = T(0.0);
              for (int cc = 0; cc < Phys::NCOL; ++cc) {
                const int v = Phys::ncol(d, cc);
                T dv = T(0.0);
                for (int r = 0; r < n1; ++r) dv = dv + T(re.D[i * n1 + r]) * st[(size_t)v * P + node(d, q, r)];
                du[v] = dv;
              }
              ph.ncprod(d, a, du, nc);
              for (int v = 0; v < M; ++v) hk[(size_t)v * P + p] = hk[(size_t)v * P + p] + T(wj) * nc[v] / T(dx[d]);
            }
          }
        }
        // accumulate the time averages
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            const double tk = std::pow(dt, k) / fact;  // dt^k/(k+1)!
            L.U[idx(v, e, p)] = L.U[idx(v, e, p)] + T(tk) * c[((size_t)k * M + v) * P + p];
            L.Bl[idx(v, e, p)] = L.Bl[idx(v, e, p)] + hk[(size_t)v * P + p] / T(fact);
            for (int d = 0; d < DIM; ++d)
              L.F[(size_t)d * M * E * P + idx(v, e, p)] =
                  L.F[(size_t)d * M * E * P + idx(v, e, p)] + fk[((size_t)d * M + v) * P + p] / T(fact);
          }
        if (k == N) break;
        // d_t^{k+1} u = -(sum_d D_d d_t^k f_d / dx_d + d_t^k [B u_x]); fk, hk hold dt^k d_t^k
        const double idtk = 1.0 / std::pow(dt, k);
        for (int p = 0; p < P; ++p)
          for (int v = 0; v < M; ++v) {
            T r = hk[(size_t)v * P + p];
            for (int d = 0; d < DIM; ++d) {
              int i = pos(d, p), q = line(d, p);
              T df = T(0.0);
              for (int rr = 0; rr < n1; ++rr) df = df + T(re.D[i * n1 + rr]) * fk[((size_t)d * M + v) * P + node(d, q, rr)];
              r = r + df / T(dx[d]);
            }
            c[((size_t)(k + 1) * M + v) * P + p] = -T(idtk) * r;
          }
      }
    }
  }

  // traces of F_d, U and u^n at the faces, and F^nc
  template <class T>
  void face_traces(const T* un, Local<T>& L) const {
#pragma omp parallel for num_threads(nthreads()) schedule(static)
    for (int e = 0; e < E; ++e) face_traces_elem(un, L, e);
  }

  // the face traces and F^nc of element e
  template <class T>
  void face_traces_elem(const T* un, Local<T>& L, int e) const {
    T a[M], w[M], o[M];
    {
      for (int d = 0; d < DIM; ++d)
        for (int side = 0; side < 2; ++side) {
          const std::vector<double>& V = side ? re.VR : re.VL;
          for (int q = 0; q < nfp; ++q)
            for (int v = 0; v < M; ++v) {
              T tf = T(0.0), tu = T(0.0), tn = T(0.0);
              for (int r = 0; r < n1; ++r) {
                int p = node(d, q, r);
                tf = tf + T(V[r]) * L.F[(size_t)d * M * E * P + idx(v, e, p)];
                tu = tu + T(V[r]) * L.U[idx(v, e, p)];
                tn = tn + T(V[r]) * un[idx(v, e, p)];
              }
              size_t id = tidx(d, side, v, e, q);
              L.Ftr[id] = tf; L.Utr[id] = tu; L.untr[id] = tn;
            }
          // non-conservative extrapolation F^nc = B(u^{n,±}) U^± : the companion of
          // the interface term B(u^{n,±}) U^num of eq. good.numflux.non.cons (the
          // same replacement of the stage values u^(j)± by u^{n,±} in both terms,
          // so that their difference vanishes where the solution is continuous)
          for (int q = 0; q < nfp; ++q) {
            for (int v = 0; v < M; ++v) {
              a[v] = L.untr[tidx(d, side, v, e, q)];
              w[v] = L.Utr[tidx(d, side, v, e, q)];
            }
            ph.ncprod(d, a, w, o);
            for (int v = 0; v < M; ++v) L.Fnc[tidx(d, side, v, e, q)] = o[v];
          }
        }
    }
  }

  // ----------------------------------------------- 4. interface fluxes ----
  // lower order fluxes f^{num,-}, f^{num,+}(uL, uR) of eq. combined.num.flux
  template <class T>
  void lof(int d, const T* uL, const T* uR, double ch, T* fm, T* fp) const {
    T fL[M], fR[M], bL[M], bR[M], avg[M];
    T lam = tmax(ph.sigma(d, uL, ch), ph.sigma(d, uR, ch));
    ph.flux(d, uL, fL, ch);
    ph.flux(d, uR, fR, ch);
    for (int v = 0; v < M; ++v) avg[v] = T(0.5) * (uL[v] + uR[v]);
    ph.ncprod(d, uL, avg, bL);
    ph.ncprod(d, uR, avg, bR);
    for (int v = 0; v < M; ++v) {
      T fc = T(0.5) * (fL[v] + fR[v]) - T(0.5) * lam * (uR[v] - uL[v]);
      fm[v] = fc + bL[v];
      fp[v] = fc + bR[v];
    }
  }

  template <class T>
  bool admissible(const T* x) const {
    for (int k = 0; k < K; ++k)
      if (!(val(ph.constraint(k, x)) > 0.0)) return false;
    return true;
  }

  template <class T>
  struct Faces {
    std::vector<T> Fm, Fp;        // [d][v][e][q]: face d between e and nbr(e,d,1)
    std::vector<double> theta;    // [d][e][q] product of Alg. 1 thetas
    std::vector<uint8_t> guard;   // [d][e][q]
    // left boundary faces of non-periodic directions: F^+ for the element e on
    // that side, [d][v][e][q] (entries of other elements unused)
    std::vector<T> FpLeft;
    std::vector<double> thetaLeft;
    std::vector<uint8_t> guardLeft;
  };

  // the data of one side of a face: face values of u^n, F_d and U, and u^n at the
  // point next to the face (s) and after it (si)
  template <class T>
  struct Side {
    T a[M], F[M], U[M], s[M], si[M];
  };

  // side data of element e at its right (fs = 1) or left (fs = 0) face
  template <class T>
  void elem_side(const T* un, const Local<T>& L, int d, int e, int q, int fs, Side<T>& S) const {
    for (int v = 0; v < M; ++v) {
      S.a[v] = L.untr[tidx(d, fs, v, e, q)];
      S.F[v] = L.Ftr[tidx(d, fs, v, e, q)];
      S.U[v] = L.Utr[tidx(d, fs, v, e, q)];
      S.s[v] = un[idx(v, e, node(d, q, fs ? N : 0))];
      S.si[v] = un[idx(v, e, node(d, q, fs ? (N > 0 ? N - 1 : 0) : (N > 0 ? 1 : 0)))];
    }
  }

  // ghost side of boundary (d, side) outside the inside data `in` of element e
  template <class T>
  void ghost_side(int d, int side, int e, int q, const Side<T>& in, Side<T>& g) const {
    const int kind = cfg.bc[d][side];
    if (kind == BC_OUTFLOW) { g = in; return; }
    if (kind == BC_WALL) {
      // mirror image: the normal momentum changes sign; every component of the
      // d-flux of the mirror state is the negative of the d-flux except the
      // normal momentum flux (f_d(P u) = -P f_d(u)), and so are its time averages
      const int mn = 1 + d;
      for (int v = 0; v < M; ++v) {
        const double sgn = v == mn ? -1.0 : 1.0;
        g.a[v] = T(sgn) * in.a[v];
        g.U[v] = T(sgn) * in.U[v];
        g.s[v] = T(sgn) * in.s[v];
        g.si[v] = T(sgn) * in.si[v];
        g.F[v] = T(-sgn) * in.F[v];
      }
      return;
    }
    // Dirichlet data
    size_t off = 0;
    for (int b = 0; b < 2 * d + side; ++b) off += (size_t)3 * M * blines(b / 2) * nfp;
    const size_t NB = (size_t)blines(d) * nfp, j = bpos(e, d, q);
    for (int v = 0; v < M; ++v) {
      g.a[v] = T(cfg.ghost[off + (0 * M + v) * NB + j]);
      g.U[v] = T(cfg.ghost[off + (1 * M + v) * NB + j]);
      g.F[v] = T(cfg.ghost[off + (2 * M + v) * NB + j]);
      g.s[v] = g.a[v];
      g.si[v] = g.a[v];
    }
  }

  template <class T>
  void faces(const T* un, const Local<T>& L, const std::vector<double>& alpha, double dt, double ch,
             Faces<T>& Fc) const {
    alloc_faces(Fc);
#pragma omp parallel for num_threads(nthreads()) schedule(static)
    for (int de = 0; de < DIM * E; ++de) faces_line(un, L, alpha, dt, ch, Fc, de / E, de % E);
  }

  // (every face line writes its F^- and, inside the mesh, its F^+)
  template <class T>
  void alloc_faces(Faces<T>& Fc) const {
    Fc.Fm.resize((size_t)DIM * M * E * nfp);
    Fc.Fp.resize(Fc.Fm.size());
    Fc.FpLeft.assign(Fc.Fm.size(), T(0.0));
    Fc.theta.assign((size_t)DIM * E * nfp, 1.0);
    Fc.guard.assign((size_t)DIM * E * nfp, 0);
    Fc.thetaLeft.assign((size_t)DIM * E * nfp, 1.0);
    Fc.guardLeft.assign((size_t)DIM * E * nfp, 0);
  }

  // the face points of the face in direction d on the upper side of element e
  // (and, on a non-periodic direction's last element, the opposite boundary half face)
  template <class T>
  void faces_line(const T* un, const Local<T>& L, const std::vector<double>& alpha, double dt, double ch,
                  Faces<T>& Fc, int d, int e) const {
    Side<T> mi, pl;
    T Fm[M], Fp[M];
    {
        int en = nbr(e, d, 1);
        for (int q = 0; q < nfp; ++q) {
          size_t fi = ((size_t)d * E + e) * nfp + q;
          if (!on_boundary(e, d, 1)) {
            // interior (or periodic) face between e and en
            elem_side(un, L, d, e, q, 1, mi);
            elem_side(un, L, d, en, q, 0, pl);
            double th = 1.0;
            uint8_t gd = 0;
            face(d, mi, pl, 0.5 * (alpha[e] + alpha[en]), true, true, dt, ch, Fm, Fp, th, gd);
            for (int v = 0; v < M; ++v) {
              Fc.Fm[fidx(d, v, e, q)] = Fm[v];
              Fc.Fp[fidx(d, v, e, q)] = Fp[v];
            }
            Fc.theta[fi] = th;
            Fc.guard[fi] = gd;
            continue;
          }
          // right boundary face of e: ghost outside; the ghost carries alpha_e
          {
            elem_side(un, L, d, e, q, 1, mi);
            ghost_side(d, 1, e, q, mi, pl);
            double th = 1.0;
            uint8_t gd = 0;
            face(d, mi, pl, alpha[e], true, false, dt, ch, Fm, Fp, th, gd);
            for (int v = 0; v < M; ++v) Fc.Fm[fidx(d, v, e, q)] = Fm[v];
            Fc.theta[fi] = th;
            Fc.guard[fi] = gd;
          }
          // left boundary face of the element on the opposite side of the line
          {
            const int el = en;  // nbr wraps to the first element of the line
            elem_side(un, L, d, el, q, 0, pl);
            ghost_side(d, 0, el, q, pl, mi);
            double th = 1.0;
            uint8_t gd = 0;
            face(d, mi, pl, alpha[el], false, true, dt, ch, Fm, Fp, th, gd);
            const size_t fl = ((size_t)d * E + el) * nfp + q;
            for (int v = 0; v < M; ++v) Fc.FpLeft[fidx(d, v, el, q)] = Fp[v];
            Fc.thetaLeft[fl] = th;
            Fc.guardLeft[fl] = gd;
          }
        }
      }
  }

  // One face in direction d from its minus side mi and plus side pl: the
  // blended fluxes F^- (for the minus element) and F^+ (for the plus element).
  // Algorithm 1 limits with the candidates of the sides marked `limit_*` (a
  // ghost side has no subcell of the mesh to keep admissible).
  template <class T>
  void face(int d, const Side<T>& mi, const Side<T>& pl, double af, bool limit_minus, bool limit_plus, double dt,
            double ch, T* Fm, T* Fp, double& Theta, uint8_t& guard_out) const {
    T Fnum[M], Unum[M], Ba[M], Bb[M], fLOm[M], fLOp[M], tmp[M], finL[M], finR[M];
    T uN[M], u0[M], uNlo[M], u0lo[M];
    // high order time-averaged fluxes (eqs. numflux.cons, good.numflux.non.cons);
    // lambda from the face values of u^n (eq. rusanov.wave.speed); a face value
    // that is not admissible (an undershoot of the polynomial next to a jump)
    // gives its wave speed at the adjacent solution point instead.
    T sa = admissible(mi.a) ? ph.sigma(d, mi.a, ch) : ph.sigma(d, mi.s, ch);
    T sb = admissible(pl.a) ? ph.sigma(d, pl.a, ch) : ph.sigma(d, pl.s, ch);
    T lam = tmax(sa, sb);
    for (int v = 0; v < M; ++v) {
      Fnum[v] = T(0.5) * (mi.F[v] + pl.F[v]) - T(0.5) * lam * (pl.U[v] - mi.U[v]);
      Unum[v] = T(0.5) * (mi.U[v] + pl.U[v]);
    }
    ph.ncprod(d, mi.a, Unum, Ba);
    ph.ncprod(d, pl.a, Unum, Bb);
    // lower order flux at the face from the neighbouring subcell values
    lof(d, mi.s, pl.s, ch, fLOm, fLOp);
    // blend with alpha_{e+1/2} (eq. Fblend)
    for (int v = 0; v < M; ++v) {
      Fm[v] = T(1.0 - af) * (Fnum[v] + Ba[v]) + T(af) * fLOm[v];
      Fp[v] = T(1.0 - af) * (Fnum[v] + Bb[v]) + T(af) * fLOp[v];
    }
    Theta = 1.0;
    guard_out = 0;
    // Algorithm 1: limit F^± so that the neighbouring subcell updates stay
    // admissible; in DIM dimensions the candidate uses DIM*dt (the subcell
    // update is the mean of DIM one-directional updates with DIM*dt).
    if (cfg.blending == 2 && N >= 1) {
      lof(d, mi.si, mi.s, ch, tmp, finL);  // f^{e,+}_{N-1/2}
      lof(d, pl.s, pl.si, ch, finR, tmp);  // f^{e+1,-}_{1/2}
      T cN = T(DIM * dt / (re.w[N] * dx[d])), c0 = T(DIM * dt / (re.w[0] * dx[d]));
      auto cand = [&]() {
        for (int v = 0; v < M; ++v) {
          uN[v] = mi.s[v] - cN * (Fm[v] - finL[v]);
          u0[v] = pl.s[v] - c0 * (finR[v] - Fp[v]);
        }
      };
      for (int v = 0; v < M; ++v) {
        uNlo[v] = mi.s[v] - cN * (fLOm[v] - finL[v]);
        u0lo[v] = pl.s[v] - c0 * (finR[v] - fLOp[v]);
      }
      cand();
      bool guard = false;
      for (int k = 0; k < K; ++k) {
        double PN = val(ph.constraint(k, uNlo)), P0 = val(ph.constraint(k, u0lo));
        double th0 = limit_plus ? theta_concave(0.1 * P0, P0, val(ph.constraint(k, u0)), guard) : 1.0;
        double thN = limit_minus ? theta_concave(0.1 * PN, PN, val(ph.constraint(k, uN)), guard) : 1.0;
        double th = std::min(th0, thN);
        for (int v = 0; v < M; ++v) {
          Fm[v] = T(th) * Fm[v] + T(1.0 - th) * fLOm[v];
          Fp[v] = T(th) * Fp[v] + T(1.0 - th) * fLOp[v];
        }
        cand();
        Theta *= th;
      }
      guard_out = guard ? 1 : 0;
    }
  }

  // ------------------------------------------------ 5. element update -----
  // uL_out, ustar_out (nullable, [v][e][p]): the lower order update u^L and the
  // blend (1 - alpha_e) u^H + alpha_e u^L before Algorithm 2 (test inspection).
  template <class T>
  void update(const T* un, const Local<T>& L, const Faces<T>& Fc, const std::vector<double>& alpha,
              double dt, double ch, T* unew, uint32_t* flags, double* theta_elem, T* uL_out = nullptr,
              T* ustar_out = nullptr) const {
#pragma omp parallel num_threads(nthreads())
    {
      std::vector<T> W((size_t)3 * M * P);
#pragma omp for schedule(static)
      for (int e = 0; e < E; ++e)
        update_elem(un, L, Fc, alpha, dt, ch, unew, flags, theta_elem, uL_out, ustar_out, e, W);
    }
  }

  // the update of element e; W: scratch of 3 M P values
  template <class T>
  void update_elem(const T* un, const Local<T>& L, const Faces<T>& Fc, const std::vector<double>& alpha,
                   double dt, double ch, T* unew, uint32_t* flags, double* theta_elem, T* uL_out, T* ustar_out,
                   int e, std::vector<T>& W) const {
    T* uH = W.data();
    T* uL = W.data() + (size_t)M * P;
    T* us = W.data() + (size_t)2 * M * P;
    const size_t nMP = (size_t)M * P;
    T x0[M], x1[M], fm[M], fp[M], tmp[M];
    {
      uint32_t fl = 0;
      // faces of this element: Alg. 1 activity
      for (int d = 0; d < DIM; ++d)
        for (int q = 0; q < nfp; ++q) {
          size_t iu = ((size_t)d * E + e) * nfp + q, il = ((size_t)d * E + nbr(e, d, 0)) * nfp + q;
          const bool lb = on_boundary(e, d, 0);
          const double thl = lb ? Fc.thetaLeft[iu] : Fc.theta[il];
          const uint8_t gl = lb ? Fc.guardLeft[iu] : Fc.guard[il];
          if (Fc.theta[iu] < 1.0 || thl < 1.0) fl |= FLAG_ALG1;
          if (Fc.guard[iu] || gl) fl |= FLAG_ALG1_GUARD;
        }
      // high order update (eq. crkfr.non.cons.final), corrections along each line
      for (int p = 0; p < P; ++p)
        for (int v = 0; v < M; ++v) {
          T R = L.Bl[idx(v, e, p)];
          for (int d = 0; d < DIM; ++d) {
            int i = pos(d, p), q = line(d, p);
            T dF = T(0.0);
            for (int r = 0; r < n1; ++r)
              dF = dF + T(re.D[i * n1 + r]) * L.F[(size_t)d * M * E * P + idx(v, e, node(d, q, r))];
            int el = nbr(e, d, 0);
            const T Fleft = on_boundary(e, d, 0) ? Fc.FpLeft[fidx(d, v, e, q)] : Fc.Fp[fidx(d, v, el, q)];
            T cR = Fc.Fm[fidx(d, v, e, q)] - L.Ftr[tidx(d, 1, v, e, q)] - L.Fnc[tidx(d, 1, v, e, q)];
            T cL = Fleft - L.Ftr[tidx(d, 0, v, e, q)] - L.Fnc[tidx(d, 0, v, e, q)];
            R = R + (dF + cR * T(re.gRp[i]) + cL * T(re.gLp[i])) / T(dx[d]);
          }
          uH[(size_t)v * P + p] = un[idx(v, e, p)] - T(dt) * R;
          // + dt S (eq. crkfr with the time-averaged source of eq. avg.source)
          if constexpr (Phys::SRC) uH[(size_t)v * P + p] = uH[(size_t)v * P + p] + T(dt) * L.S[idx(v, e, p)];
        }
      if (cfg.blending == 0) {
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) unew[idx(v, e, p)] = uH[(size_t)v * P + p];
      } else {
        // lower order subcell update (eq. low.order.update); subcell p has width w_p dx
        for (int p = 0; p < P; ++p) {
          T R[M];
          for (int v = 0; v < M; ++v) R[v] = T(0.0);
          for (int d = 0; d < DIM; ++d) {
            int i = pos(d, p), q = line(d, p), el = nbr(e, d, 0);
            T right[M], left[M];
            if (i < N) {
              for (int v = 0; v < M; ++v) { x0[v] = un[idx(v, e, p)]; x1[v] = un[idx(v, e, node(d, q, i + 1))]; }
              lof(d, x0, x1, ch, fm, tmp);
              for (int v = 0; v < M; ++v) right[v] = fm[v];
            } else {
              for (int v = 0; v < M; ++v) right[v] = Fc.Fm[fidx(d, v, e, q)];
            }
            if (i > 0) {
              for (int v = 0; v < M; ++v) { x0[v] = un[idx(v, e, node(d, q, i - 1))]; x1[v] = un[idx(v, e, p)]; }
              lof(d, x0, x1, ch, tmp, fp);
              for (int v = 0; v < M; ++v) left[v] = fp[v];
            } else if (on_boundary(e, d, 0)) {
              for (int v = 0; v < M; ++v) left[v] = Fc.FpLeft[fidx(d, v, e, q)];
            } else {
              for (int v = 0; v < M; ++v) left[v] = Fc.Fp[fidx(d, v, el, q)];
            }
            for (int v = 0; v < M; ++v) R[v] = R[v] + (right[v] - left[v]) / T(re.w[i] * dx[d]);
          }
          for (int v = 0; v < M; ++v) uL[(size_t)v * P + p] = un[idx(v, e, p)] - T(dt) * R[v];
          // the source enters the subcell update implicitly (eq. low.order.update):
          // u^L = r + dt s(u^L)
          if constexpr (Phys::SRC) {
            T r[M], x[M];
            for (int v = 0; v < M; ++v) r[v] = uL[(size_t)v * P + p];
            ph.implicit(r, dt, x);
            for (int v = 0; v < M; ++v) uL[(size_t)v * P + p] = x[v];
          }
        }
        // blend (eq. blended.scheme)
        double al = alpha[e];
        for (size_t i = 0; i < nMP; ++i) us[i] = T(1.0 - al) * uH[i] + T(al) * uL[i];
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            if (uL_out) uL_out[idx(v, e, p)] = uL[(size_t)v * P + p];
            if (ustar_out) ustar_out[idx(v, e, p)] = us[(size_t)v * P + p];
          }
        // Algorithm 2
        double Theta = 1.0;
        T z[M];
        for (int k = 0; k < K; ++k) {
          double Pmin = INFINITY;
          for (int p = 0; p < P; ++p) {
            for (int v = 0; v < M; ++v) z[v] = uL[(size_t)v * P + p];
            Pmin = std::min(Pmin, val(ph.constraint(k, z)));
          }
          if (Pmin <= 0.0) fl |= FLAG_LOW_INADM;
          if (cfg.blending == 2) {
            double eps = 0.1 * Pmin, th = 1.0;
            bool guard = false;
            for (int p = 0; p < P; ++p) {
              for (int v = 0; v < M; ++v) z[v] = uL[(size_t)v * P + p];
              double Pa = val(ph.constraint(k, z));
              for (int v = 0; v < M; ++v) z[v] = us[(size_t)v * P + p];
              double Pb = val(ph.constraint(k, z));
              th = std::min(th, theta_concave(eps, Pa, Pb, guard));
            }
            for (size_t i = 0; i < nMP; ++i) us[i] = T(th) * us[i] + T(1.0 - th) * uL[i];
            Theta *= th;
          }
        }
        if (Theta < 1.0) fl |= FLAG_ALG2;
        if (theta_elem) theta_elem[e] = Theta;
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) unew[idx(v, e, p)] = us[(size_t)v * P + p];
      }
      for (int v = 0; v < M; ++v)
        for (int p = 0; p < P; ++p)
          if (!std::isfinite(val(unew[idx(v, e, p)]))) fl |= FLAG_NONFINITE;
      if (flags) flags[e] = fl;
    }
  }

  // full step for scalar type T with dt, c_h and alpha given (frozen)
  // Lp, Fcp (nullable): buffers kept by the caller over several steps
  template <class T>
  void step(const T* un, T* unew, double dt, double ch, const std::vector<double>& alpha, uint32_t* flags,
            double* theta_face, double* theta_elem, T* uL_out = nullptr, T* ustar_out = nullptr,
            Local<T>* Lp = nullptr, Faces<T>* Fcp = nullptr) const {
    Local<T> Lo;
    Faces<T> Fco;
    Local<T>& L = Lp ? *Lp : Lo;
    Faces<T>& Fc = Fcp ? *Fcp : Fco;
    if (cfg.alw) stages_alw(un, dt, ch, L);
    else stages(un, dt, ch, L);
    face_traces(un, L);
    faces(un, L, alpha, dt, ch, Fc);
    if (theta_face) std::copy(Fc.theta.begin(), Fc.theta.end(), theta_face);
    update(un, L, Fc, alpha, dt, ch, unew, flags, theta_elem, uL_out, ustar_out);
  }
};

}  // namespace ora
