// Reverse-mode adjoint of one time step: lambda^n = (d u^{n+1}/d u^n)^T lambda^{n+1}
// with dt, c_h, every blending coefficient alpha_e, every Algorithm 1 and 2
// theta and every max/abs branch taken at their forward values (frozen
// switches).  The forward step from u^n runs first and leaves the face
// traces, alpha and the thetas in the workspace; the kernels below then
// sweep the step backwards:
//   k_adj_update  u^{n+1} <- (Algorithm 2, blend, correction lift, subcell FV)
//   k_adj_faces   F^±, F^± - F_tr - B U_tr <- (Algorithm 1, blend, Rusanov and
//                 non-conservative interface fluxes)
//   k_adj_stages  traces and volume residual <- stages (stage states recomputed
//                 into LDS, then swept in reverse with D^T along the lines)
#pragma once
#include "kernels.hpp"

namespace lwfr {

struct AdjParams {
  double* g_rvol;  // [M][E][P] adjoint of the volume residual
  double* g_un;    // [M][E][P] partial adjoint of u^n from the update
  double* gFm;     // [d][M][E*nfp] adjoint of F^- of face (e, e+1)
  double* gFp;     // [d][M][E*nfp] adjoint of F^+
  double* gDm;     // [d][M][E*nfp] adjoint of F^- - F_tr^- - B(u^{n,-}) U^-
  double* gDp;     // [d][M][E*nfp]
  double* gFtr;    // [d][side][M][E*nfp] adjoint of the traces
  double* gUtr;
  double* guntr;
  double* gsL;     // [d][M][E*nfp] adjoint of u^n at node N of the face's minus element
  double* gsR;     // [d][M][E*nfp] adjoint of u^n at node 0 of the face's plus element
};

// reverse of low_flux: (fmb, fpb) -> uLb, uRb (accumulated)
template <class Ph, int d>
__device__ inline void low_flux_vjp(const double* uL, const double* uR, const double* fmb, const double* fpb,
                                    double* uLb, double* uRb, const PhysParams& pp) {
  constexpr int M = Ph::M;
  double avg[M], avgb[M], fcb[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    avg[v] = 0.5 * (uL[v] + uR[v]);
    avgb[v] = 0.0;
    fcb[v] = fmb[v] + fpb[v];
  }
  Ph::template ncprod_vjp<d>(uL, avg, fmb, uLb, avgb, pp);
  Ph::template ncprod_vjp<d>(uR, avg, fpb, uRb, avgb, pp);
  const double sl = Ph::template sigma<d>(uL, pp), sr = Ph::template sigma<d>(uR, pp);
  const double lam = sl >= sr ? sl : sr;
  double lamb = 0.0, fhb[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    fhb[v] = 0.5 * fcb[v];
    lamb -= 0.5 * fcb[v] * (uR[v] - uL[v]);
    uRb[v] += -0.5 * lam * fcb[v] + 0.5 * avgb[v];
    uLb[v] += 0.5 * lam * fcb[v] + 0.5 * avgb[v];
  }
  Ph::template flux_vjp<d>(uL, fhb, uLb, pp);
  Ph::template flux_vjp<d>(uR, fhb, uRb, pp);
  if (sl >= sr) Ph::template sigma_vjp<d>(uL, lamb, uLb, pp);
  else Ph::template sigma_vjp<d>(uR, lamb, uRb, pp);
}

// ------------------------------------------------------------------------
// two waves per SIMD: GLM-MHD then spills about 8 VGPRs (36 bytes per lane),
// which costs less than the second wave gains
#ifndef ADJ_UPDATE_WAVES_PER_EU
#define ADJ_UPDATE_WAVES_PER_EU 2
#endif
template <class Ph, int N, int EPB>
__global__ void __launch_bounds__(EPB* ipow(N + 1, Ph::DIM)) __attribute__((amdgpu_waves_per_eu(ADJ_UPDATE_WAVES_PER_EU)))
    k_adj_update(const KParams kp, const AdjParams ap, const double* __restrict__ un_g,
                 const double* __restrict__ lam_g) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  __shared__ double s_u[EPB][M][P];
  __shared__ double s_a[EPB][M][P];
  __shared__ double s_b[EPB][M][P];

  const int tid = threadIdx.x;
  const int le = tid / P, p = tid - le * P;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool act = e < kp.E;
  // lanes without an element compute on element 0 and store nothing: the loads
  // stay unconditional (a load under a lane condition waits for all loads)
  const int ea = act ? e : 0;
  const int i = p % n1, j = p / n1;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  const size_t nf = (size_t)kp.E * NFP;

  double un[M], lam[M], gH[M], gL[M], gun[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    un[v] = un_g[((size_t)v * kp.E + ea) * P + p];
    lam[v] = lam_g[((size_t)v * kp.E + ea) * P + p];
    s_u[le][v][p] = un[v];
  }
  // u^{n+1} = Theta us + (1 - Theta) uL,  us = (1 - alpha) uH + alpha uL
  if (kp.blending == 0) {
#pragma unroll
    for (int v = 0; v < M; ++v) { gH[v] = lam[v]; gL[v] = 0.0; }
  } else {
    const double al = kp.alpha[ea];
    const double th = kp.blending == 2 ? kp.theta_elem[ea] : 1.0;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const double gs = th * lam[v];
      gL[v] = (1.0 - th) * lam[v] + al * gs;
      gH[v] = (1.0 - al) * gs;
    }
  }
#pragma unroll
  for (int v = 0; v < M; ++v) {
    gun[v] = gH[v] + gL[v];
    if (act) ap.g_rvol[((size_t)v * kp.E + e) * P + p] = -dt * gH[v];
  }
  int eL[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) eL[d] = nbr_elem(kp, ea, d, 0);
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int q = d == 0 ? j : i, ii = d == 0 ? i : j;
    // correction lift: uH -= dt (Dm g_R(xi_ii) + Dp g_L(xi_ii)) / dx_d along the line
#pragma unroll
    for (int v = 0; v < M; ++v) {
      s_a[le][v][p] = -dt * kp.gR[ii] * kp.inv_dx[d] * gH[v];
      s_b[le][v][p] = -dt * kp.gL[ii] * kp.inv_dx[d] * gH[v];
    }
    __syncthreads();
    if (act && ii == 0) {  // one thread per line sums it
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int r = 0; r < n1; ++r) {
          sa += s_a[le][v][node_at<n1>(d, q, r)];
          sb += s_b[le][v][node_at<n1>(d, q, r)];
        }
        ap.gDm[((size_t)d * M + v) * nf + (size_t)e * NFP + q] = sa;
        ap.gDp[((size_t)d * M + v) * nf + (size_t)eL[d] * NFP + q] = sb;
      }
    }
    __syncthreads();
    if (kp.blending != 0) {
      // subcell FV: uL -= dt (right - left) / (w_ii dx_d)
      const double cR = -dt * kp.inv_wdx[d][ii];
      // the adjoint of f^{num,+} of the subface left of this node goes to the node on the left
#pragma unroll
      for (int v = 0; v < M; ++v) s_a[le][v][p] = -cR * gL[v];
      __syncthreads();
      double ubn[M];
#pragma unroll
      for (int v = 0; v < M; ++v) ubn[v] = 0.0;
      if (ii < N) {
        const int pn = node_at<n1>(d, q, ii < N ? ii + 1 : ii);
        double fmb[M], fpb[M], u2[M];
#pragma unroll
        for (int v = 0; v < M; ++v) {
          fmb[v] = cR * gL[v];
          fpb[v] = s_a[le][v][pn];
          u2[v] = s_u[le][v][pn];
        }
        if (d == 0) low_flux_vjp<Ph, 0>(un, u2, fmb, fpb, gun, ubn, pp);
        else low_flux_vjp<Ph, (DIM > 1 ? 1 : 0)>(un, u2, fmb, fpb, gun, ubn, pp);
      } else if (act) {
#pragma unroll
        for (int v = 0; v < M; ++v) ap.gFm[((size_t)d * M + v) * nf + (size_t)e * NFP + q] = cR * gL[v];
      }
      if (ii == 0 && act) {
#pragma unroll
        for (int v = 0; v < M; ++v) ap.gFp[((size_t)d * M + v) * nf + (size_t)eL[d] * NFP + q] = -cR * gL[v];
      }
      __syncthreads();
      if (ii < N) {
        const int pn = node_at<n1>(d, q, ii < N ? ii + 1 : ii);
#pragma unroll
        for (int v = 0; v < M; ++v) s_b[le][v][pn] = ubn[v];
      }
      __syncthreads();
      if (ii > 0) {
#pragma unroll
        for (int v = 0; v < M; ++v) gun[v] += s_b[le][v][p];
      }
      __syncthreads();
    } else if (act) {
      // pure high order: the face fluxes reach the state only through the correction
      if (ii == N) {
#pragma unroll
        for (int v = 0; v < M; ++v) ap.gFm[((size_t)d * M + v) * nf + (size_t)e * NFP + q] = 0.0;
      }
      if (ii == 0) {
#pragma unroll
        for (int v = 0; v < M; ++v) ap.gFp[((size_t)d * M + v) * nf + (size_t)eL[d] * NFP + q] = 0.0;
      }
    }
  }
  if (act) {
#pragma unroll
    for (int v = 0; v < M; ++v) ap.g_un[((size_t)v * kp.E + e) * P + p] = gun[v];
  }
}

// ------------------------------------------------------------------------
template <class Ph, int N, int d>
__device__ inline void adj_face_point(const KParams& kp, const AdjParams& ap, const double* __restrict__ un_g, int e,
                                      int q, const PhysParams& pp) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  const int en = nbr_elem(kp, e, d, 1);
  const size_t nf = (size_t)kp.E * NFP;
  const size_t fiL = (size_t)e * NFP + q, fiR = (size_t)en * NFP + q;
  double a[M], b[M], UL[M], UR[M], sL[M], sR[M];
  double gFm[M], gFp[M], gDm[M], gDp[M];
  {
    // u^n at the face from each side's line of nodes, as the forward face
    // kernel forms it (the next nodes inward are not needed here)
    double inner[M];
    line_trace<Ph, N, d, 1>(kp, un_g, e, q, 1, a, sL, inner);
    line_trace<Ph, N, d, 0>(kp, un_g, en, q, 0, b, sR, inner);
  }
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const size_t oL = ((size_t)(d * 2 + 1) * M + v) * nf + fiL;
    const size_t oR = ((size_t)(d * 2 + 0) * M + v) * nf + fiR;
    UL[v] = kp.Utr[oL]; UR[v] = kp.Utr[oR];
    const size_t o = ((size_t)d * M + v) * nf + fiL;
    gFm[v] = ap.gFm[o]; gFp[v] = ap.gFp[o];
    gDm[v] = ap.gDm[o]; gDp[v] = ap.gDp[o];
  }
  double ga[M], gb[M], gUL[M], gUR[M], gFL[M], gFR[M], gsL[M], gsR[M], tmp[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    ga[v] = 0.0; gb[v] = 0.0; gUL[v] = 0.0; gUR[v] = 0.0; gsL[v] = 0.0; gsR[v] = 0.0; tmp[v] = 0.0;
    gFm[v] += gDm[v];
    gFp[v] += gDp[v];
    gFL[v] = -gDm[v];
    gFR[v] = -gDp[v];
  }
  // D^- = F^- - F_L - B(a) U_L,  D^+ = F^+ - F_R - B(b) U_R
  {
    double nb[M];
#pragma unroll
    for (int v = 0; v < M; ++v) nb[v] = -gDm[v];
    Ph::template ncprod_vjp<d>(a, UL, nb, ga, gUL, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) nb[v] = -gDp[v];
    Ph::template ncprod_vjp<d>(b, UR, nb, gb, gUR, pp);
  }
  // F^± = Theta [(1 - af) F_HO^± + af f_LO^±] + (1 - Theta) f_LO^±
  const double af = kp.blending == 0 ? 0.0 : 0.5 * (kp.alpha[e] + kp.alpha[en]);
  const double Th = kp.blending == 2 ? kp.theta_face[(size_t)d * nf + fiL] : 1.0;
  double gHm[M], gHp[M];
  const bool low = !(af == 0.0 && kp.blending != 2);
#pragma unroll
  for (int v = 0; v < M; ++v) {
    gHm[v] = low ? Th * (1.0 - af) * gFm[v] : gFm[v];
    gHp[v] = low ? Th * (1.0 - af) * gFp[v] : gFp[v];
  }
  if (low) {
    double glm[M], glp[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      glm[v] = (Th * af + (1.0 - Th)) * gFm[v];
      glp[v] = (Th * af + (1.0 - Th)) * gFp[v];
    }
    low_flux_vjp<Ph, d>(sL, sR, glm, glp, gsL, gsR, pp);
  }
  // F_HO^- = Fnum + B(a) Unum, F_HO^+ = Fnum + B(b) Unum
  double Unum[M], gUnum[M], gFnum[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    Unum[v] = 0.5 * (UL[v] + UR[v]);
    gUnum[v] = 0.0;
    gFnum[v] = gHm[v] + gHp[v];
  }
  Ph::template ncprod_vjp<d>(a, Unum, gHm, ga, gUnum, pp);
  Ph::template ncprod_vjp<d>(b, Unum, gHp, gb, gUnum, pp);
  // Fnum = (FL + FR)/2 - lam (UR - UL)/2
  const bool adma = admissible<Ph>(a, pp), admb = admissible<Ph>(b, pp);
  const double sa = adma ? Ph::template sigma<d>(a, pp) : Ph::template sigma<d>(sL, pp);
  const double sb = admb ? Ph::template sigma<d>(b, pp) : Ph::template sigma<d>(sR, pp);
  const double lam = sa >= sb ? sa : sb;
  double glam = 0.0;
#pragma unroll
  for (int v = 0; v < M; ++v) {
    gFL[v] += 0.5 * gFnum[v];
    gFR[v] += 0.5 * gFnum[v];
    gUR[v] += -0.5 * lam * gFnum[v] + 0.5 * gUnum[v];
    gUL[v] += 0.5 * lam * gFnum[v] + 0.5 * gUnum[v];
    glam -= 0.5 * gFnum[v] * (UR[v] - UL[v]);
  }
  if (sa >= sb) {
    if (adma) Ph::template sigma_vjp<d>(a, glam, ga, pp);
    else Ph::template sigma_vjp<d>(sL, glam, gsL, pp);
  } else {
    if (admb) Ph::template sigma_vjp<d>(b, glam, gb, pp);
    else Ph::template sigma_vjp<d>(sR, glam, gsR, pp);
  }
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const size_t oL = ((size_t)(d * 2 + 1) * M + v) * nf + fiL;
    const size_t oR = ((size_t)(d * 2 + 0) * M + v) * nf + fiR;
    ap.gFtr[oL] = gFL[v]; ap.gFtr[oR] = gFR[v];
    ap.gUtr[oL] = gUL[v]; ap.gUtr[oR] = gUR[v];
    ap.guntr[oL] = ga[v]; ap.guntr[oR] = gb[v];
    const size_t o = ((size_t)d * M + v) * nf + fiL;
    ap.gsL[o] = gsL[v];
    ap.gsR[o] = gsR[v];
  }
}

// a two-wave hint spills about 430 VGPRs for GLM-MHD: one wave
#ifndef ADJ_FACES_WAVES_PER_EU
#define ADJ_FACES_WAVES_PER_EU 1
#endif
template <class Ph, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ADJ_FACES_WAVES_PER_EU))) k_adj_faces(const KParams kp, const AdjParams ap, const double* __restrict__ un_g) {
  constexpr int DIM = Ph::DIM, NFP = DIM == 1 ? 1 : N + 1;
  const int nf = kp.E * NFP;
  const int gid = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (gid >= DIM * nf) return;
  const int d = gid / nf;
  const int fi = gid - d * nf;
  const int e = fi / NFP, q = fi - (fi / NFP) * NFP;
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  if (d == 0) adj_face_point<Ph, N, 0>(kp, ap, un_g, e, q, pp);
  else if constexpr (DIM == 2) adj_face_point<Ph, N, 1>(kp, ap, un_g, e, q, pp);
}

// ------------------------------------------------------------------------
// Stage adjoint.  Forward: u^(s) = u^n - dt S_s, S_s = sum_{k<s} a_sk L^(k);
// U = sum b_s u^(s); F_d = sum b_s f_d(u^(s)); R_vol = sum b_s L^(s).
// Reverse: Lb_s = b_s R_volb - dt sum_{t>s} a_ts ub_t;
// ub_s = b_s Ub + sum_d f_d'(u^(s))^T (b_s F_db + D_d^T Lb_s/dx_d)
//        + sum_d [d(B_d(u) w_d)/du]^T Lb_s/dx_d + D_d^T (B_d(u)^T Lb_s/dx_d);
// lambda^n = sum_s ub_s + (direct contributions of u^n).
template <class Ph, int N, int EPB>
__global__ void __launch_bounds__(EPB* ipow(N + 1, Ph::DIM))
    k_adj_stages(const KParams kp, const AdjParams ap, const double* __restrict__ un_g, double* __restrict__ lam_out) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  constexpr int NCD = Ph::NCD > 0 ? Ph::NCD : 1;
  using Tab = Tableau<N>;
  constexpr int S = Tab::S;
  constexpr int NX = DIM * M + DIM * NCD;
  __shared__ double s_st[EPB][S][M][P];   // stage states
  __shared__ double s_x[EPB][NX][P];      // exchange buffer

  const int tid = threadIdx.x;
  const int le = tid / P, p = tid - le * P;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool act = e < kp.E;
  const int ea = act ? e : 0;  // lanes without an element read element 0
  const int i = p % n1, j = p / n1;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  const size_t nf = (size_t)kp.E * NFP;

  double un[M];
#pragma unroll
  for (int v = 0; v < M; ++v) un[v] = un_g[((size_t)v * kp.E + ea) * P + p];
  double Drow[DIM][n1], Dcol[DIM][n1];
#pragma unroll
  for (int r = 0; r < n1; ++r) {
    Drow[0][r] = kp.D[i][r];
    Dcol[0][r] = kp.D[r][i];
    if constexpr (DIM == 2) { Drow[1][r] = kp.D[j][r]; Dcol[1][r] = kp.D[r][j]; }
  }

  // ---- forward recomputation of the stage states
  double Sp[S][M];
#pragma unroll
  for (int st = 0; st < S; ++st) {
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      u[v] = first_nz<N>(st) >= 0 ? un[v] - dt * Sp[st][v] : un[v];
      s_st[le][st][v][p] = u[v];
    }
    if (st == S - 1) break;
    double f[DIM][M];
    Ph::template flux<0>(u, f[0], pp);
    if constexpr (DIM == 2) Ph::template flux<1>(u, f[1], pp);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int v = 0; v < M; ++v) s_x[le][d * M + v][p] = f[d][v];
    if constexpr (Ph::NCD > 0) {
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) s_x[le][DIM * M + d * NCD + c][p] = u[Ph::nc_comp(d, c)];
    }
    __syncthreads();
    double Ls[M];
#pragma unroll
    for (int v = 0; v < M; ++v) Ls[v] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int q = d == 0 ? j : i;
      double df[M], w[M], nc[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < n1; ++r) sacc += Drow[d][r] * s_x[le][d * M + v][node_at<n1>(d, q, r)];
        df[v] = sacc;
        w[v] = 0.0;
      }
      if constexpr (Ph::NCD > 0) {
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) {
          double sacc = 0.0;
#pragma unroll
          for (int r = 0; r < n1; ++r) sacc += Drow[d][r] * s_x[le][DIM * M + d * NCD + c][node_at<n1>(d, q, r)];
          w[Ph::nc_comp(d, c)] = sacc;
        }
      }
      if (d == 0) Ph::template ncprod<0>(u, w, nc, pp);
      else Ph::template ncprod<(DIM > 1 ? 1 : 0)>(u, w, nc, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) Ls[v] += (df[v] + nc[v]) * kp.inv_dx[d];
    }
    __syncthreads();
#pragma unroll
    for (int t = st + 1; t < S; ++t) {
      const double a = Tab::a(t, st);
      if (a != 0.0) {
#pragma unroll
        for (int v = 0; v < M; ++v) Sp[t][v] = first_nz<N>(t) == st ? a * Ls[v] : Sp[t][v] + a * Ls[v];
      }
    }
  }

  // ---- adjoints arriving from the faces and the update
  double gF[DIM][M], gU[M], gR[M], gun[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    gR[v] = ap.g_rvol[((size_t)v * kp.E + ea) * P + p];
    gun[v] = ap.g_un[((size_t)v * kp.E + ea) * P + p];
    gU[v] = 0.0;
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int q = d == 0 ? j : i, ii = d == 0 ? i : j;
    const size_t fo = (size_t)ea * NFP + q;
    const int eLd = nbr_elem(kp, ea, d, 0);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const size_t o1 = ((size_t)(d * 2 + 1) * M + v) * nf + fo;
      const size_t o0 = ((size_t)(d * 2 + 0) * M + v) * nf + fo;
      gF[d][v] = kp.VR[ii] * ap.gFtr[o1] + kp.VL[ii] * ap.gFtr[o0];
      gU[v] += kp.VR[ii] * ap.gUtr[o1] + kp.VL[ii] * ap.gUtr[o0];
      gun[v] += kp.VR[ii] * ap.guntr[o1] + kp.VL[ii] * ap.guntr[o0];
      if (ii == N) gun[v] += ap.gsL[((size_t)d * M + v) * nf + fo];
      if (ii == 0) gun[v] += ap.gsR[((size_t)d * M + v) * nf + (size_t)eLd * NFP + q];
    }
  }

  // ---- reverse sweep over the stages
  double Q[S][M];
#pragma unroll
  for (int st = S - 1; st >= 0; --st) {
    const double bs = Tab::b(st);
    double u[M], Lb[M], ub[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      u[v] = s_st[le][st][v][p];
      bool anyq = false;
#pragma unroll
      for (int t = st + 1; t < S; ++t) anyq = anyq || (Tab::a(t, st) != 0.0);
      Lb[v] = bs * gR[v] - (anyq ? dt * Q[st][v] : 0.0);
      ub[v] = bs * gU[v];
    }
    // forward D_d u (the columns B_d reads) at this node
    double w[DIM][M];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int q = d == 0 ? j : i;
#pragma unroll
      for (int v = 0; v < M; ++v) w[d][v] = 0.0;
      if constexpr (Ph::NCD > 0) {
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) {
          const int comp = Ph::nc_comp(d, c);
          double sacc = 0.0;
#pragma unroll
          for (int r = 0; r < n1; ++r) sacc += Drow[d][r] * s_st[le][st][comp][node_at<n1>(d, q, r)];
          w[d][comp] = sacc;
        }
      }
    }
    // B_d(u)^T Lb/dx_d to LDS with Lb
#pragma unroll
    for (int v = 0; v < M; ++v) s_x[le][v][p] = Lb[v];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double Ld[M], wb[M];
#pragma unroll
      for (int v = 0; v < M; ++v) { Ld[v] = Lb[v] * kp.inv_dx[d]; wb[v] = 0.0; }
      if (d == 0) Ph::template ncprod_vjp<0>(u, w[0], Ld, ub, wb, pp);
      else Ph::template ncprod_vjp<(DIM > 1 ? 1 : 0)>(u, w[DIM > 1 ? 1 : 0], Ld, ub, wb, pp);
      if constexpr (Ph::NCD > 0) {
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) s_x[le][M + d * NCD + c][p] = wb[Ph::nc_comp(d, c)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int q = d == 0 ? j : i;
      double fb[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < n1; ++r) sacc += Dcol[d][r] * s_x[le][v][node_at<n1>(d, q, r)];
        fb[v] = bs * gF[d][v] + sacc * kp.inv_dx[d];
      }
      if (d == 0) Ph::template flux_vjp<0>(u, fb, ub, pp);
      else Ph::template flux_vjp<(DIM > 1 ? 1 : 0)>(u, fb, ub, pp);
      if constexpr (Ph::NCD > 0) {
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) {
          double sacc = 0.0;
#pragma unroll
          for (int r = 0; r < n1; ++r) sacc += Dcol[d][r] * s_x[le][M + d * NCD + c][node_at<n1>(d, q, r)];
          ub[Ph::nc_comp(d, c)] += sacc;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < M; ++v) gun[v] += ub[v];
    // fold ub_st into the sums of the earlier stages it depends on
#pragma unroll
    for (int k = 0; k < st; ++k) {
      const double a = Tab::a(st, k);
      if (a != 0.0) {
        bool first = true;
#pragma unroll
        for (int t = st + 1; t < S; ++t) first = first && (Tab::a(t, k) == 0.0);
#pragma unroll
        for (int v = 0; v < M; ++v) Q[k][v] = first ? a * ub[v] : Q[k][v] + a * ub[v];
      }
    }
  }
  if (act) {
#pragma unroll
    for (int v = 0; v < M; ++v) lam_out[((size_t)v * kp.E + e) * P + p] = gun[v];
  }
}

// ---- the same reverse sweep with two lanes per solution point (GLM-MHD).
// As in the forward two-lane stage kernel, the lanes of a point sit in the two
// halves of one wave: lane d works on direction d (its flux and
// non-conservative VJPs and D_d^T contractions, in the frame where direction d
// is x, see MHD2D::rot) and owns half of the variables' sums (stage sums, the
// adjoint sums Q_k, lambda^n).  The stage states are recomputed with the forward
// kernel's arithmetic, so they equal the forward step's bit for bit.
template <class Ph, int N, int NT>
struct AdjStages2Lds {
  static constexpr int M = Ph::M, P = ipow(N + 1, 2), EL = (NT / 2 + P - 1) / P, NCD = Ph::NCD;
  static constexpr int S = Tableau<N>::S;
  // fields of an element slot: the S stage states (st*M + v), then the
  // exchange fields at XB: forward f_x, f_y, the non-conservative columns of
  // both directions; reverse Lb (M), the column adjoints of both directions
  static constexpr int XB = S * M;
  static constexpr int NF = XB + 2 * M + 2 * NCD;
  // slot stride = P (mod 32): a half-wave's points stay consecutive in bank order
  static constexpr int ES = NF * P + (((P - NF * P) % 32) + 32) % 32;
  double s[EL][ES];
};

// elements per two-lane adjoint stage workgroup of 256 threads
constexpr int epb_adj2(int P) { return 128 / P; }

template <class Ph, int N, int EPB, int NT>
__device__ __forceinline__ void adj_stages2_body(const KParams& kp, const AdjParams& ap, AdjStages2Lds<Ph, N, NT>& L,
                                                 const double* __restrict__ un_g, double* __restrict__ lam_out,
                                                 int blk) {
  static_assert(std::is_same<Ph, MHD2D>::value, "two-lane adjoint stage body is written for GLM-MHD");
  constexpr int n1 = N + 1, M = Ph::M, P = n1 * n1, NFP = n1, NCD = Ph::NCD;
  constexpr int H0 = (M + 1) / 2, H1 = M - H0;
  using Tab = Tableau<N>;
  constexpr int S = Tab::S, XB = AdjStages2Lds<Ph, N, NT>::XB;
  static_assert(2 * EPB * P <= NT, "workgroup too small for EPB elements");
  auto& sb = L.s;

  const int tid = threadIdx.x;
  const int d = (tid >> 5) & 1, np = ((tid >> 6) << 5) | (tid & 31);
  const int le = np / P, p = np - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  const int ea = act ? e : 0;  // lanes without an element read element 0
  const int i = p % n1, j = p / n1;
  const int q = d ? i : j;            // line of the lane's direction through p
  const int ii = d ? j : i;           // position along that line
  const int sq = d ? 1 : n1, sr = d ? n1 : 1;  // node(q, r) = q*sq + r*sr
  // fields only the lane's own direction reads (the forward exchange, the
  // column adjoints) are written transposed by the direction-1 lanes and read
  // at q*n1 + r, offsets known at compile time
  const int pw = d ? i * n1 + j : p;
  const int vo = d ? H0 : 0;          // first variable of the lane's half
  const int nown = d ? H1 : H0;       // variables in the lane's half
  const double dt = kp.scal[0];
  const double idx = d ? kp.inv_dx[1] : kp.inv_dx[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  const size_t nf = (size_t)kp.E * NFP;

  double Drow[n1], Dcol[n1];
#pragma unroll
  for (int r = 0; r < n1; ++r) {
    Drow[r] = kp.D[ii][r];
    Dcol[r] = kp.D[r][ii];
  }

  // ---- forward recomputation of the stage states (the lane's half to LDS)
  {
    double uo[H0], Sp[S][H0];
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      const int v = vo + (k < nown ? k : 0);
      uo[k] = un_g[((size_t)v * kp.E + ea) * P + p];
    }
#pragma unroll
    for (int st = 0; st < S; ++st) {
      double uh[H0], u[M];
#pragma unroll
      for (int k = 0; k < H0; ++k) uh[k] = first_nz<N>(st) >= 0 ? uo[k] - dt * Sp[st][k] : uo[k];
#pragma unroll
      for (int k = 0; k < H0; ++k)
        if (k < nown) sb[le][(st * M + vo + k) * P + p] = uh[k];
      if (st == S - 1) break;
#pragma unroll
      for (int k = 0; k < H0; ++k) {
        double a = uh[k], b = uh[k];
        cross_pair(a, b);
        u[k] = a;
        if (k < H1) u[H0 + k] = b;
      }
      double f[M];
      Ph::flux_rd(u, d, f, pp);
#pragma unroll
      for (int v = 0; v < M; ++v)
        if (Ph::flux_nc_alias(v) < 0) sb[le][(XB + d * M + v) * P + pw] = f[v];
#pragma unroll
      for (int c = 0; c < NCD; ++c) {
        const double x0 = u[Ph::nc_comp(0, c)], x1 = u[Ph::nc_comp(1, c)];
        sb[le][(XB + 2 * M + d * NCD + c) * P + pw] = d ? x1 : x0;
      }
      __syncthreads();
      double Ld[M];
      {
        double wc[NCD], nc[M];
#pragma unroll
        for (int c = 0; c < NCD; ++c) {
          double sacc = 0.0;
#pragma unroll
          for (int r = 0; r < n1; ++r) sacc += Drow[r] * sb[le][(XB + 2 * M + d * NCD + c) * P + (q * n1 + r)];
          wc[c] = sacc;
        }
        Ph::ncprod_rd(u, wc, d, nc, pp);
#pragma unroll
        for (int v = 0; v < M; ++v) {
          double sacc = 0.0;
          if (Ph::flux_nc_alias(v) >= 0) {
            sacc = pp.ch * wc[Ph::flux_nc_alias(v)];
          } else {
#pragma unroll
            for (int r = 0; r < n1; ++r) sacc += Drow[r] * sb[le][(XB + d * M + v) * P + (q * n1 + r)];
          }
          Ld[v] = (sacc + nc[v]) * idx;
        }
      }
      __syncthreads();
      double Lh[H0];
#pragma unroll
      for (int k = 0; k < H0; ++k) {
        double a = Ld[k], b = k < H1 ? Ld[H0 + k] : 0.0;
        cross_pair(a, b);
        Lh[k] = a + b;
      }
#pragma unroll
      for (int t = st + 1; t < S; ++t) {
        const double a = Tab::a(t, st);
        if (a != 0.0) {
#pragma unroll
          for (int k = 0; k < H0; ++k) Sp[t][k] = first_nz<N>(t) == st ? a * Lh[k] : Sp[t][k] + a * Lh[k];
        }
      }
    }
  }
  __syncthreads();

  // ---- adjoints arriving from the faces and the update
  double gF[M], gU[H0], gR[H0], gun[H0];
  {
    // F_d traces of the lane's direction, all variables, in the lane's frame
    const size_t fo = (size_t)ea * NFP + q;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const size_t o1 = ((size_t)(d * 2 + 1) * M + v) * nf + fo;
      const size_t o0 = ((size_t)(d * 2 + 0) * M + v) * nf + fo;
      gF[v] = kp.VR[ii] * ap.gFtr[o1] + kp.VL[ii] * ap.gFtr[o0];
    }
    Ph::rot(d, gF);
  }
#pragma unroll
  for (int k = 0; k < H0; ++k) {
    const int v = vo + (k < nown ? k : 0);
    gR[k] = ap.g_rvol[((size_t)v * kp.E + ea) * P + p];
    gun[k] = ap.g_un[((size_t)v * kp.E + ea) * P + p];
    gU[k] = 0.0;
  }
  // U and u^n traces of both directions, the lane's half of the variables
#pragma unroll
  for (int dd = 0; dd < 2; ++dd) {
    const int qd = dd == 0 ? j : i, id = dd == 0 ? i : j;
    const size_t fo = (size_t)ea * NFP + qd;
    const int eLd = nbr_elem(kp, ea, dd, 0);
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      const int v = vo + (k < nown ? k : 0);
      const size_t o1 = ((size_t)(dd * 2 + 1) * M + v) * nf + fo;
      const size_t o0 = ((size_t)(dd * 2 + 0) * M + v) * nf + fo;
      gU[k] += kp.VR[id] * ap.gUtr[o1] + kp.VL[id] * ap.gUtr[o0];
      gun[k] += kp.VR[id] * ap.guntr[o1] + kp.VL[id] * ap.guntr[o0];
      if (id == N) gun[k] += ap.gsL[((size_t)dd * M + v) * nf + fo];
      if (id == 0) gun[k] += ap.gsR[((size_t)dd * M + v) * nf + (size_t)eLd * NFP + qd];
    }
  }

  // ---- reverse sweep over the stages
  double Q[S][H0];
#pragma unroll
  for (int st = S - 1; st >= 0; --st) {
    const double bs = Tab::b(st);
    bool anyq = false;
#pragma unroll
    for (int t = st + 1; t < S; ++t) anyq = anyq || (Tab::a(t, st) != 0.0);
    // Lb = b_s gR - dt Q_s on the lane's half, to LDS; the full Lb at the point
    // from the pair
    double Ld[M];
    {
      double Lbh[H0];
#pragma unroll
      for (int k = 0; k < H0; ++k) Lbh[k] = bs * gR[k] - (anyq ? dt * Q[st][k] : 0.0);
#pragma unroll
      for (int k = 0; k < H0; ++k)
        if (k < nown) sb[le][(XB + vo + k) * P + p] = Lbh[k];
#pragma unroll
      for (int k = 0; k < H0; ++k) {
        double a = Lbh[k], b = Lbh[k];
        cross_pair(a, b);
        Ld[k] = a * idx;
        if (k < H1) Ld[H0 + k] = b * idx;
      }
    }
    Ph::rot(d, Ld);
    // the stage state in the lane's frame and D_d of its non-conservative columns
    double u[M];
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = sb[le][(st * M + v) * P + p];
    Ph::rot(d, u);
    double w[M], wb[M], ubd[M];
#pragma unroll
    for (int v = 0; v < M; ++v) { w[v] = 0.0; wb[v] = 0.0; ubd[v] = 0.0; }
#pragma unroll
    for (int c = 0; c < NCD; ++c) {
      const int fld = st * M + (d ? Ph::nc_comp(1, c) : Ph::nc_comp(0, c));
      double sacc = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) sacc += Drow[r] * sb[le][fld * P + (q * sq + r * sr)];
      w[Ph::nc_comp(0, c)] = sacc;
    }
    // B_d(u)^T Lb/dx_d: its u part to ubd, its column part to LDS
    Ph::template ncprod_vjp<0>(u, w, Ld, ubd, wb, pp);
#pragma unroll
    for (int c = 0; c < NCD; ++c) sb[le][(XB + M + d * NCD + c) * P + pw] = wb[Ph::nc_comp(0, c)];
    __syncthreads();
    // f_d'(u)^T (b_s F_db + D_d^T Lb/dx_d) and D_d^T of the column adjoints
    {
      double fb[M];
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < n1; ++r) sacc += Dcol[r] * sb[le][(XB + v) * P + (q * sq + r * sr)];
        fb[v] = sacc * idx;
      }
      Ph::rot(d, fb);
#pragma unroll
      for (int v = 0; v < M; ++v) fb[v] += bs * gF[v];
      Ph::template flux_vjp<0>(u, fb, ubd, pp);
    }
#pragma unroll
    for (int c = 0; c < NCD; ++c) {
      double sacc = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) sacc += Dcol[r] * sb[le][(XB + M + d * NCD + c) * P + (q * n1 + r)];
      ubd[Ph::nc_comp(0, c)] += sacc;
    }
    __syncthreads();
    Ph::rot(d, ubd);
    // ub on the lane's half: b_s gU + the contributions of both directions
    double ubh[H0];
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      double a = ubd[k], b = k < H1 ? ubd[H0 + k] : 0.0;
      cross_pair(a, b);
      ubh[k] = bs * gU[k] + (a + b);
    }
#pragma unroll
    for (int k = 0; k < H0; ++k) gun[k] += ubh[k];
#pragma unroll
    for (int kk = 0; kk < st; ++kk) {
      const double a = Tab::a(st, kk);
      if (a != 0.0) {
        bool first = true;
#pragma unroll
        for (int t = st + 1; t < S; ++t) first = first && (Tab::a(t, kk) == 0.0);
#pragma unroll
        for (int k = 0; k < H0; ++k) Q[kk][k] = first ? a * ubh[k] : Q[kk][k] + a * ubh[k];
      }
    }
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < H0; ++k)
      if (k < nown) lam_out[((size_t)(vo + k) * kp.E + e) * P + p] = gun[k];
  }
}

template <class Ph, int N, int EPB>
__global__ void __launch_bounds__(256)
    k_adj_stages2(const KParams kp, const AdjParams ap, const double* __restrict__ un_g, double* __restrict__ lam_out) {
  __shared__ AdjStages2Lds<Ph, N, 256> L;
  adj_stages2_body<Ph, N, EPB, 256>(kp, ap, L, un_g, lam_out, xcd_block(blockIdx.x, gridDim.x));
}

}  // namespace lwfr
