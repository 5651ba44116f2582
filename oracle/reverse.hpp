// Reverse-mode derivative of one time step of the oracle.  TEST
// INFRASTRUCTURE ONLY.
//
// What is differentiated: the step u^n -> u^{n+1} with dt, c_h, every alpha_e
// (after clipping and smoothing), every theta of Algorithms 1 and 2 and every
// branch of a max / abs held at the values the forward step takes at u^n
// (frozen switches).  The result is mu = (d u^{n+1} / d u^n)^T lambda.
//
// How: a reverse-mode scalar `Rev` records every operation of the oracle's own
// templated arithmetic on a tape (value, parent indices, local partials); a
// sweep from the last record to the first accumulates adjoints.  Branches and
// thetas are taken on values (val), so a Rev run follows exactly the branches
// of the double run and carries no derivative through a switch, as the Dual
// forward mode does.  The step is taped one piece at a time, in the reverse
// order of the step: the update of each element, each face line (Algorithm 1
// included), the face traces of each element, the stages of each element.
// Each piece's inputs are fresh tape leaves; their adjoints are the seeds of
// the pieces before it.  A tape holds one element's or one face line's work,
// so memory stays small on meshes of any size; pieces of one phase are
// independent and run on several threads (one tape per thread), and every
// adjoint is summed in a fixed order, so the result does not depend on the
// thread count.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

#include "scalar.hpp"
#include "scheme.hpp"

#ifdef _OPENMP
#include <omp.h>
#endif

namespace ora {

// ------------------------------------------------------------------ tape ---
struct Tape {
  struct Rec {
    int32_t a, b;    // parent records (-1: none)
    double da, db;   // d(result)/d(parent)
  };
  std::vector<Rec> rec;
  std::vector<double> adj;
  void clear() { rec.clear(); }
  int32_t push(int32_t a, double da, int32_t b, double db) {
    rec.push_back(Rec{a, b, da, db});
    return (int32_t)rec.size() - 1;
  }
  int32_t leaf() { return push(-1, 0.0, -1, 0.0); }
  // adjoints of every record from the seeds already placed in adj (resized here)
  void sweep() {
    adj.resize(rec.size(), 0.0);
    for (int64_t i = (int64_t)rec.size() - 1; i >= 0; --i) {
      const double g = adj[i];
      if (g == 0.0) continue;
      const Rec& r = rec[i];
      if (r.a >= 0) adj[r.a] += r.da * g;
      if (r.b >= 0) adj[r.b] += r.db * g;
    }
  }
  void reset_adjoints() { adj.assign(rec.size(), 0.0); }
};

inline Tape*& current_tape() {
  static thread_local Tape* t = nullptr;
  return t;
}

// -------------------------------------------------------------- Rev scalar ---
// i < 0: a constant (no record); otherwise the index of its record.
struct Rev {
  double v;
  int32_t i;
  Rev() : v(0.0), i(-1) {}
  Rev(double x) : v(x), i(-1) {}
  Rev(double x, int32_t idx) : v(x), i(idx) {}
};
inline double val(const Rev& x) { return x.v; }

inline Rev rev_unary(double v, const Rev& a, double da) {
  if (a.i < 0) return Rev(v);
  return Rev(v, current_tape()->push(a.i, da, -1, 0.0));
}
inline Rev rev_binary(double v, const Rev& a, double da, const Rev& b, double db) {
  if (a.i < 0 && b.i < 0) return Rev(v);
  return Rev(v, current_tape()->push(a.i, da, b.i, db));
}
inline Rev operator+(const Rev& a, const Rev& b) { return rev_binary(a.v + b.v, a, 1.0, b, 1.0); }
inline Rev operator-(const Rev& a, const Rev& b) { return rev_binary(a.v - b.v, a, 1.0, b, -1.0); }
inline Rev operator-(const Rev& a) { return rev_unary(-a.v, a, -1.0); }
inline Rev operator*(const Rev& a, const Rev& b) { return rev_binary(a.v * b.v, a, b.v, b, a.v); }
inline Rev operator/(const Rev& a, const Rev& b) {
  const double q = a.v / b.v;
  return rev_binary(q, a, 1.0 / b.v, b, -q / b.v);
}
inline Rev& operator+=(Rev& a, const Rev& b) { a = a + b; return a; }
inline Rev& operator-=(Rev& a, const Rev& b) { a = a - b; return a; }
inline Rev& operator*=(Rev& a, const Rev& b) { a = a * b; return a; }
inline Rev sqrt(const Rev& a) {
  const double s = std::sqrt(a.v);
  return rev_unary(s, a, 0.5 / s);
}
inline Rev exp(const Rev& a) {
  const double e = std::exp(a.v);
  return rev_unary(e, a, e);
}
inline Rev fabs(const Rev& a) { return a.v < 0 ? -a : a; }

// ------------------------------------------------------- adjoint of a step ---
template <class Phys>
struct StepAdjoint {
  using S = Scheme<Phys>;
  static constexpr int M = Phys::M, DIM = Phys::DIM;
  const S& sc;
  explicit StepAdjoint(const S& s) : sc(s) {}

  // mu = J^T lam for the step from u with dt, ch and alpha frozen; nthreads <= 0:
  // the default thread count.  Periodic meshes, systems without a source,
  // the cRK stages (not the approximate Lax-Wendroff averages).
  void vjp(const double* u, double dt, double ch, const std::vector<double>& alpha, const double* lam, double* mu,
           int nthreads) const {
    const int E = sc.E, P = sc.P, nfp = sc.nfp;
    const size_t nst = (size_t)M * E * P, ntr = (size_t)DIM * 2 * M * E * nfp, nfc = (size_t)DIM * M * E * nfp;
#ifdef _OPENMP
    const int nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    const int nth = 1;
    (void)nthreads;
#endif
    // forward values in double
    typename S::template Local<double> L;
    typename S::template Faces<double> Fc;
    sc.stages(u, dt, ch, L);
    sc.face_traces(u, L);
    sc.faces(u, L, alpha, dt, ch, Fc);
    // the same values as constants of the Rev type; a piece turns its own inputs into leaves
    std::vector<Rev> uR(u, u + nst);
    typename S::template Local<Rev> LR;
    LR.F.assign(L.F.begin(), L.F.end());
    LR.U.assign(L.U.begin(), L.U.end());
    LR.Bl.assign(L.Bl.begin(), L.Bl.end());
    LR.Fnc.assign(L.Fnc.begin(), L.Fnc.end());
    LR.Ftr.assign(L.Ftr.begin(), L.Ftr.end());
    LR.Utr.assign(L.Utr.begin(), L.Utr.end());
    LR.untr.assign(L.untr.begin(), L.untr.end());
    typename S::template Faces<Rev> FcR;
    FcR.Fm.assign(Fc.Fm.begin(), Fc.Fm.end());
    FcR.Fp.assign(Fc.Fp.begin(), Fc.Fp.end());
    FcR.FpLeft.assign(Fc.FpLeft.begin(), Fc.FpLeft.end());
    FcR.theta = Fc.theta;
    FcR.guard = Fc.guard;
    FcR.thetaLeft = Fc.thetaLeft;
    FcR.guardLeft = Fc.guardLeft;
    std::vector<Rev> outR(nst);
    // adjoints of the pieces' inputs
    std::vector<double> g_un_upd(nst, 0.0), g_un_tr(nst, 0.0), g_un_st(nst, 0.0);
    std::vector<double> gF((size_t)DIM * nst, 0.0), gU(nst, 0.0), gBl(nst, 0.0);
    std::vector<double> gFtr(ntr, 0.0), gUtr(ntr, 0.0), guntr(ntr, 0.0), gFnc(ntr, 0.0);
    std::vector<double> gFm(nfc, 0.0), gFp(nfc, 0.0);
    // u^n adjoints from the face lines, per face point: [d][e][q][node slot 0..3][v]
    // (slots: minus side's node next to the face, the one after it, plus side's same)
    std::vector<double> g_sn((size_t)DIM * E * nfp * 4 * M, 0.0);

    // ---- 5. update, per element ----
#pragma omp parallel num_threads(nth)
    {
      Tape tape;
      current_tape() = &tape;
      std::vector<Rev> W((size_t)3 * M * P);
      std::vector<size_t> lu, lF, lBl, lFtr, lFnc, lFm, lFp;
#pragma omp for schedule(static)
      for (int e = 0; e < E; ++e) {
        tape.clear();
        lu.clear(); lF.clear(); lBl.clear(); lFtr.clear(); lFnc.clear(); lFm.clear(); lFp.clear();
        auto mark = [&](std::vector<Rev>& arr, size_t k, std::vector<size_t>& list) {
          arr[k].i = tape.leaf();
          list.push_back(k);
        };
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            mark(uR, sc.idx(v, e, p), lu);
            mark(LR.Bl, sc.idx(v, e, p), lBl);
            for (int d = 0; d < DIM; ++d) mark(LR.F, (size_t)d * nst + sc.idx(v, e, p), lF);
          }
        for (int d = 0; d < DIM; ++d)
          for (int v = 0; v < M; ++v)
            for (int q = 0; q < nfp; ++q) {
              for (int side = 0; side < 2; ++side) {
                mark(LR.Ftr, sc.tidx(d, side, v, e, q), lFtr);
                mark(LR.Fnc, sc.tidx(d, side, v, e, q), lFnc);
              }
              mark(FcR.Fm, sc.fidx(d, v, e, q), lFm);
              mark(FcR.Fp, sc.fidx(d, v, sc.nbr(e, d, 0), q), lFp);
            }
        sc.update_elem(uR.data(), LR, FcR, alpha, dt, ch, outR.data(), (uint32_t*)nullptr, (double*)nullptr,
                       (Rev*)nullptr, (Rev*)nullptr, e, W);
        tape.reset_adjoints();
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            const Rev& o = outR[sc.idx(v, e, p)];
            if (o.i >= 0) tape.adj[o.i] += lam[sc.idx(v, e, p)];
          }
        tape.sweep();
        auto take = [&](std::vector<Rev>& arr, const std::vector<size_t>& list, std::vector<double>& g, size_t off) {
          for (size_t k : list) {
            g[k - off] += tape.adj[arr[k].i];
            arr[k].i = -1;
          }
        };
        take(uR, lu, g_un_upd, 0);
        take(LR.Bl, lBl, gBl, 0);
        for (size_t k : lF) { gF[k] += tape.adj[LR.F[k].i]; LR.F[k].i = -1; }
        take(LR.Ftr, lFtr, gFtr, 0);
        take(LR.Fnc, lFnc, gFnc, 0);
        take(FcR.Fm, lFm, gFm, 0);
        take(FcR.Fp, lFp, gFp, 0);
      }
      current_tape() = nullptr;
    }

    // ---- 4. face lines (interior faces of the periodic mesh) ----
#pragma omp parallel num_threads(nth)
    {
      Tape tape;
      current_tape() = &tape;
      typename S::template Side<double> md, pd;
      typename S::template Side<Rev> mi, pl;
      Rev Fm[M], Fp[M];
#pragma omp for schedule(static)
      for (int de = 0; de < DIM * E; ++de) {
        const int d = de / E, e = de % E, en = sc.nbr(e, d, 1);
        const double af = 0.5 * (alpha[e] + alpha[en]);
        for (int q = 0; q < nfp; ++q) {
          tape.clear();
          sc.elem_side(u, L, d, e, q, 1, md);
          sc.elem_side(u, L, d, en, q, 0, pd);
          for (int v = 0; v < M; ++v) {
            mi.a[v] = Rev(md.a[v], tape.leaf()); mi.F[v] = Rev(md.F[v], tape.leaf());
            mi.U[v] = Rev(md.U[v], tape.leaf()); mi.s[v] = Rev(md.s[v], tape.leaf());
            mi.si[v] = Rev(md.si[v], tape.leaf());
            pl.a[v] = Rev(pd.a[v], tape.leaf()); pl.F[v] = Rev(pd.F[v], tape.leaf());
            pl.U[v] = Rev(pd.U[v], tape.leaf()); pl.s[v] = Rev(pd.s[v], tape.leaf());
            pl.si[v] = Rev(pd.si[v], tape.leaf());
          }
          double th = 1.0;
          uint8_t gd = 0;
          sc.face(d, mi, pl, af, true, true, dt, ch, Fm, Fp, th, gd);
          tape.reset_adjoints();
          for (int v = 0; v < M; ++v) {
            if (Fm[v].i >= 0) tape.adj[Fm[v].i] += gFm[sc.fidx(d, v, e, q)];
            if (Fp[v].i >= 0) tape.adj[Fp[v].i] += gFp[sc.fidx(d, v, e, q)];
          }
          tape.sweep();
          double* gs = &g_sn[(((size_t)d * E + e) * nfp + q) * 4 * M];
          for (int v = 0; v < M; ++v) {
            guntr[sc.tidx(d, 1, v, e, q)] += tape.adj[mi.a[v].i];
            gFtr[sc.tidx(d, 1, v, e, q)] += tape.adj[mi.F[v].i];
            gUtr[sc.tidx(d, 1, v, e, q)] += tape.adj[mi.U[v].i];
            guntr[sc.tidx(d, 0, v, en, q)] += tape.adj[pl.a[v].i];
            gFtr[sc.tidx(d, 0, v, en, q)] += tape.adj[pl.F[v].i];
            gUtr[sc.tidx(d, 0, v, en, q)] += tape.adj[pl.U[v].i];
            gs[0 * M + v] = tape.adj[mi.s[v].i];
            gs[1 * M + v] = tape.adj[mi.si[v].i];
            gs[2 * M + v] = tape.adj[pl.s[v].i];
            gs[3 * M + v] = tape.adj[pl.si[v].i];
          }
        }
      }
      current_tape() = nullptr;
    }

    // ---- 3b. face traces and F^nc, per element ----
#pragma omp parallel num_threads(nth)
    {
      Tape tape;
      current_tape() = &tape;
#pragma omp for schedule(static)
      for (int e = 0; e < E; ++e) {
        tape.clear();
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            uR[sc.idx(v, e, p)].i = tape.leaf();
            LR.U[sc.idx(v, e, p)].i = tape.leaf();
            for (int d = 0; d < DIM; ++d) LR.F[(size_t)d * nst + sc.idx(v, e, p)].i = tape.leaf();
          }
        sc.face_traces_elem(uR.data(), LR, e);
        tape.reset_adjoints();
        for (int d = 0; d < DIM; ++d)
          for (int side = 0; side < 2; ++side)
            for (int v = 0; v < M; ++v)
              for (int q = 0; q < nfp; ++q) {
                const size_t k = sc.tidx(d, side, v, e, q);
                if (LR.Ftr[k].i >= 0) tape.adj[LR.Ftr[k].i] += gFtr[k];
                if (LR.Utr[k].i >= 0) tape.adj[LR.Utr[k].i] += gUtr[k];
                if (LR.untr[k].i >= 0) tape.adj[LR.untr[k].i] += guntr[k];
                if (LR.Fnc[k].i >= 0) tape.adj[LR.Fnc[k].i] += gFnc[k];
              }
        tape.sweep();
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            const size_t k = sc.idx(v, e, p);
            g_un_tr[k] += tape.adj[uR[k].i];
            uR[k].i = -1;
            gU[k] += tape.adj[LR.U[k].i];
            LR.U[k].i = -1;
            for (int d = 0; d < DIM; ++d) {
              gF[(size_t)d * nst + k] += tape.adj[LR.F[(size_t)d * nst + k].i];
              LR.F[(size_t)d * nst + k].i = -1;
            }
          }
      }
      current_tape() = nullptr;
    }

    // ---- 3a. stages, per element ----
#pragma omp parallel num_threads(nth)
    {
      Tape tape;
      current_tape() = &tape;
      typename S::template StageScratch<Rev> Wst(sc);
#pragma omp for schedule(static)
      for (int e = 0; e < E; ++e) {
        tape.clear();
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            const size_t k = sc.idx(v, e, p);
            uR[k].i = tape.leaf();
            LR.U[k] = Rev(0.0);
            LR.Bl[k] = Rev(0.0);
            for (int d = 0; d < DIM; ++d) LR.F[(size_t)d * nst + k] = Rev(0.0);
          }
        sc.stages_elem(uR.data(), dt, ch, LR, e, Wst);
        tape.reset_adjoints();
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            const size_t k = sc.idx(v, e, p);
            if (LR.U[k].i >= 0) tape.adj[LR.U[k].i] += gU[k];
            if (LR.Bl[k].i >= 0) tape.adj[LR.Bl[k].i] += gBl[k];
            for (int d = 0; d < DIM; ++d)
              if (LR.F[(size_t)d * nst + k].i >= 0) tape.adj[LR.F[(size_t)d * nst + k].i] += gF[(size_t)d * nst + k];
          }
        tape.sweep();
        for (int v = 0; v < M; ++v)
          for (int p = 0; p < P; ++p) {
            const size_t k = sc.idx(v, e, p);
            g_un_st[k] += tape.adj[uR[k].i];
            uR[k].i = -1;
          }
      }
      current_tape() = nullptr;
    }

    // ---- sum: u^n adjoints of the update, the face lines, the traces and the stages ----
    for (size_t k = 0; k < nst; ++k) mu[k] = g_un_upd[k];
    for (int d = 0; d < DIM; ++d)
      for (int e = 0; e < E; ++e) {
        const int en = sc.nbr(e, d, 1);
        for (int q = 0; q < nfp; ++q) {
          const double* gs = &g_sn[(((size_t)d * E + e) * nfp + q) * 4 * M];
          const int N = sc.N;
          const int pS = sc.node(d, q, N), pSi = sc.node(d, q, N > 0 ? N - 1 : 0);
          const int qS = sc.node(d, q, 0), qSi = sc.node(d, q, N > 0 ? 1 : 0);
          for (int v = 0; v < M; ++v) {
            mu[sc.idx(v, e, pS)] += gs[0 * M + v];
            mu[sc.idx(v, e, pSi)] += gs[1 * M + v];
            mu[sc.idx(v, en, qS)] += gs[2 * M + v];
            mu[sc.idx(v, en, qSi)] += gs[3 * M + v];
          }
        }
      }
    for (size_t k = 0; k < nst; ++k) mu[k] += g_un_tr[k];
    for (size_t k = 0; k < nst; ++k) mu[k] += g_un_st[k];
  }
};

}  // namespace ora
