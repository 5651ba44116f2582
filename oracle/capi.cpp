// C entry points of the CPU oracle for the Python test harness (ctypes).
// TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU baseline
// leg of the benchmark may load this library.
#include <cstdint>
#include <cstring>
#include <vector>

#include "reverse.hpp"
#include "scheme.hpp"

using namespace ora;

struct ora_cfg {
  int32_t eq, N, nx, ny;
  double lo[2], hi[2];
  double gamma, gravity;
  double cs, cfl;
  int32_t blending;
  double alpha_max, alpha_min, alpha_force;
  int32_t gll;
  int32_t bc[4];        // sides (x lo, x hi, y lo, y hi): 0 periodic, 1 outflow, 2 wall, 3 Dirichlet
  const double* ghost;  // Dirichlet data (see Config::ghost)
  int32_t imex;         // IMEX pair of a system with a source: 1 HT(1,1,2), 2 SSP3-IMEX(4,3,3)
  double relax_a, relax_eps, relax_l, relax_q;  // Jin-Xin a, eps and f(u) = l u + q u^2/2
  int32_t alw;          // 1: approximate Lax-Wendroff time averages
  int32_t threads;      // threads of the element and face loops (results do not depend on it)
};

static Config to_cfg(const ora_cfg* c) {
  Config k;
  k.eq = c->eq; k.N = c->N; k.nx = c->nx; k.ny = c->ny;
  for (int i = 0; i < 2; ++i) { k.lo[i] = c->lo[i]; k.hi[i] = c->hi[i]; }
  k.gamma = c->gamma; k.gravity = c->gravity; k.cs = c->cs; k.cfl = c->cfl;
  k.blending = c->blending; k.alpha_max = c->alpha_max; k.alpha_min = c->alpha_min;
  k.alpha_force = c->alpha_force;
  k.gll = c->gll;
  for (int i = 0; i < 4; ++i) k.bc[i / 2][i % 2] = c->bc[i];
  k.ghost = c->ghost;
  k.imex = c->imex;
  k.relax_a = c->relax_a;
  k.relax_eps = c->relax_eps;
  k.relax_l = c->relax_l;
  k.relax_q = c->relax_q;
  k.alw = c->alw;
  k.threads = c->threads;
  return k;
}

// Calls fn(scheme) with the scheme of the configured equation system.  Calls
// that take a step (steps_ = true) need the data of every Dirichlet side.
template <class Fn>
static int dispatch(const ora_cfg* c, Fn fn, bool steps_ = true) {
  Config k = to_cfg(c);
  if (k.N < 0 || k.N > 4 || k.nx < 1 || k.ny < 1) return 1;
  if (k.gll && k.N < 1) return 1;
  if (k.imex < 0 || k.imex > 2) return 1;
  if (k.alw && (k.imex || k.N < 1)) return 1;
  if (k.eq == EQ_JINXIN1D && (k.imex == 0 || !(k.relax_eps > 0.0) || !(k.relax_a > 0.0))) return 1;
  for (int d = 0; d < 2; ++d) {
    if ((k.bc[d][0] == BC_PERIODIC) != (k.bc[d][1] == BC_PERIODIC)) return 3;
    for (int sd = 0; sd < 2; ++sd) {
      if (k.bc[d][sd] < 0 || k.bc[d][sd] > BC_DIRICHLET) return 3;
      if (k.bc[d][sd] == BC_WALL && k.eq != EQ_SW1D && k.eq != EQ_SW2D) return 3;
      if (k.bc[d][sd] == BC_DIRICHLET && steps_ && !k.ghost) return 3;
    }
  }
  switch (k.eq) {
    case EQ_SW1D: { SW1D ph{k.gravity}; Scheme<SW1D> s(ph, k); fn(s); return 0; }
    case EQ_SW2D: { SW2D ph{k.gravity}; Scheme<SW2D> s(ph, k); fn(s); return 0; }
    case EQ_MHD2D: { MHD2D ph{k.gamma}; Scheme<MHD2D> s(ph, k); fn(s); return 0; }
    case EQ_LINADV1D: { LinAdv1D ph; Scheme<LinAdv1D> s(ph, k); fn(s); return 0; }
    case EQ_VARADV1D: { VarAdv1D ph; Scheme<VarAdv1D> s(ph, k); fn(s); return 0; }
    case EQ_JINXIN1D: { JinXin1D ph{k.relax_a, k.relax_eps, k.relax_l, k.relax_q}; Scheme<JinXin1D> s(ph, k); fn(s); return 0; }
  }
  return 2;
}

extern "C" {

int ora_refel(int N, int gll, double* xi, double* w, double* D, double* VL, double* VR, double* gLp, double* gRp,
              double* Leg) {
  if (N < 0 || N > 8 || (gll && N < 1)) return 1;
  RefElem r(N, gll != 0);
  int n1 = N + 1;
  std::memcpy(xi, r.xi.data(), n1 * sizeof(double));
  std::memcpy(w, r.w.data(), n1 * sizeof(double));
  std::memcpy(D, r.D.data(), n1 * n1 * sizeof(double));
  std::memcpy(VL, r.VL.data(), n1 * sizeof(double));
  std::memcpy(VR, r.VR.data(), n1 * sizeof(double));
  std::memcpy(gLp, r.gLp.data(), n1 * sizeof(double));
  std::memcpy(gRp, r.gRp.data(), n1 * sizeof(double));
  std::memcpy(Leg, r.Leg.data(), n1 * n1 * sizeof(double));
  return 0;
}

int ora_tableau(int N, int* s, double* A, double* b) {
  if (N < 0 || N > 4) return 1;
  Tableau t(N);
  *s = t.s;
  std::memcpy(A, t.A.data(), t.s * t.s * sizeof(double));
  std::memcpy(b, t.b.data(), t.s * sizeof(double));
  return 0;
}

// IMEX pair imex (1 HT(1,1,2), 2 SSP3-IMEX(4,3,3)): explicit (A, b) and
// implicit (Ai, bi) parts, s x s row-major (arrays of at least 36 and 6).
int ora_tableau_imex(int imex, int* s, double* A, double* b, double* Ai, double* bi) {
  if (imex < 1 || imex > 2) return 1;
  Tableau t(1, imex);
  *s = t.s;
  std::memcpy(A, t.A.data(), t.s * t.s * sizeof(double));
  std::memcpy(b, t.b.data(), t.s * sizeof(double));
  std::memcpy(Ai, t.Ai.data(), t.s * t.s * sizeof(double));
  std::memcpy(bi, t.bi.data(), t.s * sizeof(double));
  return 0;
}

// Jin-Xin pointwise parts: what = 0 flux, 1 source s(u), 2 the solution of
// u - c s(u) = r (r in u).
int ora_jinxin(int what, double a, double eps, double l, double q, double c, const double* u, double* out) {
  JinXin1D ph{a, eps, l, q};
  switch (what) {
    case 0: ph.flux<double>(0, u, out, 0.0); return 0;
    case 1: ph.source<double>(u, out); return 0;
    case 2: ph.implicit<double>(u, c, out); return 0;
  }
  return 1;
}

// Pointwise physics: what = 0 flux f_d(u), 1 B_d(u) w, 2 sigma_d(u) (out[0]),
// 3 constraints P_k(u) (out[0..K-1]), 4 indicator variable (out[0]),
// 5 ideal speeds (out[0] = |v_d|, out[1] = c).
int ora_physics(int eq, double gamma, double gravity, double ch, int what, int d, const double* u,
                const double* w, double* out) {
  auto run = [&](const auto& ph) {
    using P = std::decay_t<decltype(ph)>;
    switch (what) {
      case 0: ph.template flux<double>(d, u, out, ch); break;
      case 1: ph.template ncprod<double>(d, u, w, out); break;
      case 2: out[0] = ph.template sigma<double>(d, u, ch); break;
      case 3: for (int k = 0; k < P::K; ++k) out[k] = ph.template constraint<double>(k, u); break;
      case 4: out[0] = ph.template indicator<double>(u); break;
      case 5: ph.speeds(d, u, out[0], out[1]); break;
    }
  };
  switch (eq) {
    case EQ_SW1D: run(SW1D{gravity}); return 0;
    case EQ_SW2D: run(SW2D{gravity}); return 0;
    case EQ_MHD2D: run(MHD2D{gamma}); return 0;
    case EQ_LINADV1D: run(LinAdv1D{}); return 0;
    case EQ_VARADV1D: run(VarAdv1D{}); return 0;
  }
  return 2;
}

// Columns of B_d the oracle treats as not identically zero; returns their count.
int ora_ncols(int eq, int d, int* cols) {
  auto run = [&](const auto& ph) {
    using P = std::decay_t<decltype(ph)>;
    for (int i = 0; i < P::NCOL; ++i) cols[i] = P::ncol(d, i);
    return P::NCOL;
  };
  switch (eq) {
    case EQ_SW1D: return run(SW1D{9.81});
    case EQ_SW2D: return run(SW2D{9.81});
    case EQ_MHD2D: return run(MHD2D{5.0 / 3.0});
    case EQ_LINADV1D: return run(LinAdv1D{});
    case EQ_VARADV1D: return run(VarAdv1D{});
  }
  return -1;
}

int ora_dt_ch(const ora_cfg* c, const double* u, double* dt_ch) {
  return dispatch(c, [&](auto& s) { s.dt_ch(u, dt_ch[0], dt_ch[1]); }, false);
}

int ora_alpha(const ora_cfg* c, const double* u, double* araw, double* alpha, uint8_t* tie) {
  return dispatch(c, [&](auto& s) {
    std::vector<double> a, b;
    std::vector<uint8_t> t;
    s.indicator(u, a, b, t);
    std::memcpy(araw, a.data(), a.size() * sizeof(double));
    std::memcpy(alpha, b.data(), b.size() * sizeof(double));
    if (tie) std::memcpy(tie, t.data(), t.size());
  }, false);
}

// One step.  dt_in > 0: use it (c_h is still computed from u unless ch_in >= 0);
// otherwise dt from eq. time.step.2d.  dt_ch_out = {dt, c_h}.
// alpha_in (nullable): blending coefficients to use instead of the indicator's.
int ora_step(const ora_cfg* c, const double* u, double* unew, double dt_in, double ch_in, const double* alpha_in,
             double* dt_ch_out, double* alpha_out, uint32_t* flags, uint8_t* tie, double* theta_face,
             double* theta_elem) {
  return dispatch(c, [&](auto& s) {
    double dt, ch;
    s.dt_ch(u, dt, ch);
    if (dt_in > 0) dt = dt_in;
    if (ch_in >= 0) ch = ch_in;
    std::vector<double> araw, alpha;
    std::vector<uint8_t> t;
    s.indicator(u, araw, alpha, t);
    if (alpha_in) alpha.assign(alpha_in, alpha_in + s.E);
    s.template step<double>(u, unew, dt, ch, alpha, flags, theta_face, theta_elem);
    if (dt_ch_out) { dt_ch_out[0] = dt; dt_ch_out[1] = ch; }
    if (alpha_out) std::memcpy(alpha_out, alpha.data(), alpha.size() * sizeof(double));
    if (tie) std::memcpy(tie, t.data(), t.size());
  });
}

// The pre-Algorithm-2 parts of one step with dt, c_h and alpha as ora_step
// computes them: u^L (lower order subcell update) and u* = (1 - alpha) u^H +
// alpha u^L, plus u^{n+1} and theta_elem (product of the Algorithm 2 thetas).
int ora_step_parts(const ora_cfg* c, const double* u, double dt_in, double ch_in, double* unew, double* uL,
                   double* ustar, double* theta_elem, uint32_t* flags) {
  return dispatch(c, [&](auto& s) {
    double dt, ch;
    s.dt_ch(u, dt, ch);
    if (dt_in > 0) dt = dt_in;
    if (ch_in >= 0) ch = ch_in;
    std::vector<double> araw, alpha;
    std::vector<uint8_t> t;
    s.indicator(u, araw, alpha, t);
    s.template step<double>(u, unew, dt, ch, alpha, flags, nullptr, theta_elem, uL, ustar);
  });
}

// One face in direction d (Algorithm 1 included when cfg blending = 2) from the
// data of its two sides.  side_m, side_p: 5 M values each, [a | F | U | s | si]
// = face value of u^n, traces of F_d and U, u^n at the node next to the face
// and at the node after it.  af: alpha of the face.  Out: F^- (Fm), F^+ (Fp),
// the product of the Algorithm 1 thetas and the guard bit.
int ora_face(const ora_cfg* c, int d, const double* side_m, const double* side_p, double af, double dt, double ch,
             double* Fm, double* Fp, double* theta, uint8_t* guard) {
  return dispatch(c, [&](auto& s) {
    using S = std::decay_t<decltype(s)>;
    constexpr int M = S::M;
    typename S::template Side<double> mi, pl;
    for (int v = 0; v < M; ++v) {
      mi.a[v] = side_m[v]; mi.F[v] = side_m[M + v]; mi.U[v] = side_m[2 * M + v];
      mi.s[v] = side_m[3 * M + v]; mi.si[v] = side_m[4 * M + v];
      pl.a[v] = side_p[v]; pl.F[v] = side_p[M + v]; pl.U[v] = side_p[2 * M + v];
      pl.s[v] = side_p[3 * M + v]; pl.si[v] = side_p[4 * M + v];
    }
    double th = 1.0;
    uint8_t g = 0;
    s.face(d, mi, pl, af, true, true, dt, ch, Fm, Fp, th, g);
    *theta = th;
    *guard = g;
  }, false);
}

// nsteps steps from u0 with dt from eq. time.step.2d each step (the oracle's own
// run); the state before step k is written to saved[i] for save_at[i] == k
// (k = nsteps: the final state), and each step's {dt, c_h} to dt_ch (nsteps x 2,
// nullable).  The step buffers are kept over the run.
int ora_run(const ora_cfg* c, const double* u0, int nsteps, int nsave, const int* save_at, double* saved,
            double* dt_ch) {
  if (nsteps < 0 || nsave < 0) return 1;
  return dispatch(c, [&](auto& s) {
    using S = std::decay_t<decltype(s)>;
    const size_t n = (size_t)s.M * s.E * s.P;
    std::vector<double> a(u0, u0 + n), b(n);
    typename S::template Local<double> L;
    typename S::template Faces<double> Fc;
    auto save = [&](int k) {
      for (int i = 0; i < nsave; ++i)
        if (save_at[i] == k) std::memcpy(saved + (size_t)i * n, a.data(), n * sizeof(double));
    };
    for (int k = 0; k < nsteps; ++k) {
      save(k);
      double dt, ch;
      s.dt_ch(a.data(), dt, ch);
      std::vector<double> araw, alpha;
      std::vector<uint8_t> t;
      s.indicator(a.data(), araw, alpha, t);
      s.template step<double>(a.data(), b.data(), dt, ch, alpha, nullptr, nullptr, nullptr, nullptr, nullptr, &L,
                              &Fc);
      if (dt_ch) { dt_ch[2 * k] = dt; dt_ch[2 * k + 1] = ch; }
      std::swap(a, b);
    }
    save(nsteps);
  });
}

// Element-local time averages of one step (the stages, or the approximate LW
// procedure with cfg alw): F [d][v][e][p], U [v][e][p], B^loc [v][e][p].
int ora_time_averages(const ora_cfg* c, const double* u, double dt, double ch, double* F, double* U, double* Bl) {
  return dispatch(c, [&](auto& s) {
    using S = std::decay_t<decltype(s)>;
    typename S::template Local<double> L;
    if (s.cfg.alw) s.stages_alw(u, dt, ch, L);
    else s.stages(u, dt, ch, L);
    std::memcpy(F, L.F.data(), L.F.size() * sizeof(double));
    std::memcpy(U, L.U.data(), L.U.size() * sizeof(double));
    std::memcpy(Bl, L.Bl.data(), L.Bl.size() * sizeof(double));
  }, false);
}

// Residual R = (u^n - u^{n+1})/dt; mode 0: high order only (alpha = 0, no
// limiter), 1: lower order only (alpha = 1, no limiter), 2: as configured.
int ora_residual(const ora_cfg* c, const double* u, double dt, double ch_in, int mode, double* R) {
  ora_cfg cc = *c;
  if (mode == 0) { cc.blending = 0; cc.alpha_force = -1; }
  if (mode == 1) { cc.blending = 1; cc.alpha_force = 1.0; }
  return dispatch(&cc, [&](auto& s) {
    double dtc, ch;
    s.dt_ch(u, dtc, ch);
    if (ch_in >= 0) ch = ch_in;
    std::vector<double> araw, alpha;
    std::vector<uint8_t> t;
    s.indicator(u, araw, alpha, t);
    size_t n = (size_t)s.M * s.E * s.P;
    std::vector<double> un(n);
    s.template step<double>(u, un.data(), dt, ch, alpha, nullptr, nullptr, nullptr);
    for (size_t i = 0; i < n; ++i) R[i] = (u[i] - un[i]) / dt;
  });
}

// Forward-mode derivative of the step with dt, c_h, every alpha_e and every
// theta held at their values at u (frozen switches): Jv = d unew/du . v.
int ora_jvp(const ora_cfg* c, const double* u, const double* v, double dt, double ch, double* unew, double* Jv) {
  return dispatch(c, [&](auto& s) {
    std::vector<double> araw, alpha;
    std::vector<uint8_t> t;
    s.indicator(u, araw, alpha, t);
    size_t n = (size_t)s.M * s.E * s.P;
    std::vector<Dual> x(n), y(n);
    for (size_t i = 0; i < n; ++i) x[i] = Dual(u[i], v[i]);
    s.template step<Dual>(x.data(), y.data(), dt, ch, alpha, nullptr, nullptr, nullptr);
    for (size_t i = 0; i < n; ++i) { if (unew) unew[i] = y[i].v; Jv[i] = y[i].d; }
  });
}

// Reverse-mode derivative of the step (oracle/reverse.hpp): mu = J^T lam with
// dt, c_h, every alpha_e and every theta held at their values at u (frozen
// switches, as ora_jvp).  nthreads <= 0: the default OpenMP thread count.
// Periodic meshes, systems without a source, the cRK stages (returns 4 otherwise).
int ora_vjp(const ora_cfg* c, const double* u, const double* lam, double dt, double ch, double* mu, int nthreads) {
  if (c->alw || c->eq == EQ_JINXIN1D) return 4;
  for (int i = 0; i < 4; ++i)
    if (c->bc[i] != BC_PERIODIC) return 4;
  return dispatch(c, [&](auto& s) {
    using Phys = std::decay_t<decltype(s.ph)>;
    std::vector<double> araw, alpha;
    std::vector<uint8_t> t;
    s.indicator(u, araw, alpha, t);
    StepAdjoint<Phys> adj(s);
    adj.vjp(u, dt, ch, alpha, lam, mu, nthreads);
  });
}

// Algorithmic operation counts of one step, split into the element-local
// stages, the face traces (with F^nc), the interface fluxes, the element
// update, and the means with dt, c_h and the smoothness indicator:
// counts[phase*5 + {add, mul, div, sqrt, exp}], phase 0..4 (serial).
int ora_count_ops(const ora_cfg* c, const double* u, double dt, double ch, uint64_t* counts) {
  return dispatch(c, [&](auto& s) {
    using S = std::decay_t<decltype(s)>;
    std::vector<double> araw, alpha;
    std::vector<uint8_t> t;
    s.indicator(u, araw, alpha, t);
    size_t n = (size_t)s.M * s.E * s.P;
    std::vector<Counting> x(n), y(n);
    for (size_t i = 0; i < n; ++i) x[i] = Counting(u[i]);
    typename S::template Local<Counting> L;
    typename S::template Faces<Counting> Fc;
    auto grab = [&](int ph) {
      counts[ph * 5 + 0] = FlopCounter::add; counts[ph * 5 + 1] = FlopCounter::mul;
      counts[ph * 5 + 2] = FlopCounter::div; counts[ph * 5 + 3] = FlopCounter::sqrt;
      counts[ph * 5 + 4] = FlopCounter::exp; FlopCounter::reset();
    };
    FlopCounter::reset();
    s.template stages<Counting>(x.data(), dt, ch, L);
    grab(0);
    s.template face_traces<Counting>(x.data(), L);
    grab(1);
    s.template faces<Counting>(x.data(), L, alpha, dt, ch, Fc);
    grab(2);
    s.template update<Counting>(x.data(), L, Fc, alpha, dt, ch, y.data(), nullptr, nullptr);
    grab(3);
    double dt2, ch2;
    s.dt_ch(x.data(), dt2, ch2);
    std::vector<double> ar2, al2;
    std::vector<uint8_t> t2;
    s.indicator(x.data(), ar2, al2, t2);
    grab(4);
  });
}

}  // extern "C"
