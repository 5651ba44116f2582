// gfx950 kernels of one time step of the time-averaged flux reconstruction
// scheme with non-conservative products (paper §2-§4).
//
//   k_pre      element means, ideal wave speeds, smoothness indicator (raw)
//   k_dt       Lambda = max_e sum_d (|v_d|+c_d)/dx_d, dt = C_s CFL(N)/Lambda (eq. time.step.2d)
//   k_ch       GLM cleaning speed candidates per element, k_ch_fin the minimum
//   k_stages   element-local stages, time averages F, U, B^loc, volume residual and face traces
//   k_faces    interface fluxes, blend of eq. Fblend and Algorithm 1, one thread per face point
//   k_bfaces   the two half faces of each boundary face point of a non-periodic direction
//   k_update   correction update, subcell FV update, blend and Algorithm 2
//   k_residual R = (u^n - u^{n+1})/dt
//
// Layouts: state [var][elem][node]; face arrays [dir][..][var][elem*nfp + q]
// where q is the position along the face; elements and nodes x-fastest.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "physics.hpp"
#include "refel.hpp"

namespace lwfr {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// The thread's index in the workgroup, hidden from the optimiser by an empty asm
// statement (no instruction is emitted).  The batched kernels run the per-element
// bodies below once per tile in a loop; without this, everything the bodies
// derive from the thread index (node coordinates, LDS offsets) is hoisted out of
// that loop for every degree's body and held in registers throughout.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
// OT: the body runs inside a batched tile loop (single-problem kernels keep the
// plain index, whose known range gives shorter index arithmetic)
template <bool OT>
__device__ __forceinline__ int body_tid() {
  if constexpr (OT) return opaque_tid();
  else return threadIdx.x;
}

// Workgroups of a launch go to the eight XCDs in turn, and each XCD has its own
// L2.  Neighbouring workgroups share cache lines at their edges (the face data of
// adjacent elements, the node rows either side of a y face), so the block index a
// kernel works on is permuted to give each XCD one contiguous run of blocks, in
// order: XCD x takes the blocks [x*per + min(x, rem), ...) of the launch.  A
// bijection of [0, nb) for any nb.
#ifndef LWFR_XCD_REMAP
#define LWFR_XCD_REMAP 1
#endif
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  if (!LWFR_XCD_REMAP) return b;
  const int per = nb / kXcds, rem = nb - per * kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

// Algorithm 1's outcome at a face point as the update's element flags need it:
// bit 0 when the product of its thetas is below 1, bit 1 when the guard held.
__device__ __forceinline__ uint8_t face_flag(double Theta, bool guard) {
  return (uint8_t)((Theta < 1.0 ? 1u : 0u) | (guard ? 2u : 0u));
}

// Synchronisation of the lanes that share one element's LDS slot.  When no
// element straddles two waves (LANES lanes per element dividing the 64 of a
// wave), those lanes are one wave: a wave-level fence orders their LDS
// accesses, and waves no longer wait for each other at workgroup barriers.
// Otherwise a workgroup barrier.
#ifndef LWFR_WAVE_LOCAL_SYNC
#define LWFR_WAVE_LOCAL_SYNC 1
#endif
template <int LANES>
__device__ __forceinline__ void elem_sync() {
  if constexpr (LWFR_WAVE_LOCAL_SYNC && 64 % LANES == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Minimum and OR over the P lanes of one element, the result in every one of
// them, by lane exchanges: for elements whose lanes are an aligned group of a
// power of two lanes within one wave (thread t works for element t / P).  Both
// are exact, so the order of the exchanges does not change the result.
template <int P>
__host__ __device__ constexpr bool elem_lane_exchange() {
  return LWFR_WAVE_LOCAL_SYNC && P <= 64 && (P & (P - 1)) == 0;
}
template <int P>
__device__ __forceinline__ double elem_min(double x) {
#pragma unroll
  for (int o = P / 2; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, P));
  return x;
}
template <int P>
__device__ __forceinline__ uint32_t elem_or(uint32_t x) {
#pragma unroll
  for (int o = P / 2; o > 0; o >>= 1) x |= (uint32_t)__shfl_xor((int)x, o, P);
  return x;
}

#ifndef STAGES_WAVES_PER_EU
#define STAGES_WAVES_PER_EU 1
#endif
// extra doubles after each variable's node row in the stage kernel's LDS
#ifndef LWFR_STAGES_PAD
#define LWFR_STAGES_PAD 0
#endif

// everything a kernel needs besides the state pointers, passed by value
struct KParams {
  int nx, ny, E, nblk_pre, nblk_ch;
  int nblk_dt;                // blocks of k_dt's first level (GLM-MHD's c_h)
  int N;                      // degree (the batched kernels dispatch on it)
  double dx[2], inv_dx[2];
  double D[kMaxN1][kMaxN1], VL[kMaxN1], VR[kMaxN1], w[kMaxN1], gR[kMaxN1], gL[kMaxN1];
  double Leg[kMaxN1][kMaxN1];
  double inv_wdx[2][kMaxN1];  // 1/(w_p dx_d)
  double g, gamma;
  int blending;
  // 1: F^+[0] is not stored and is read from F^-[0] of the same face (GLM-MHD
  // with every side periodic: the non-conservative product has no mass
  // component, so the two sides' mass fluxes are the same F^num[0])
  int fp0_alias;
  double alpha_max, alpha_min, alpha_force;
  double ind_T, ind_s;        // indicator threshold T(N) and logistic sharpness s
  double cs_cfl;              // C_s * CFL(N)
  double dt_in;               // > 0: fixed time step
  double ch_in;               // >= 0: fixed GLM cleaning speed
  // workspace
  double* scal;               // [0] dt, [1] c_h, [2] Lambda
  double* part;               // per-block partial maxima / minima
  double* part2;
  double* part3;              // [nblk_dt] k_dt's first-level maxima
  double* speeds;             // [E][2*DIM] (|v_d|, c_d)
  double* alpha_raw;          // [E]
  double* alpha;              // [E] smoothed alpha used by the step
  double* Ftr;                // [d][side][M][E*nfp] trace of F_d
  double* Utr;                // [d][side][M][E*nfp] trace of U
  double* Fm;                 // [d][M][E*nfp] F^- of face (e, e+1)
  double* Fp;                 // [d][M][E*nfp] F^+
  double* Dm;                 // [d][M][E*nfp] F^- - F_tr^- - B(u^{n,-}) U^- (systems that do not fold it)
  double* Dp;                 // [d][M][E*nfp] F^+ - F_tr^+ - B(u^{n,+}) U^+
  double* theta_face;         // [d][E*nfp] product of Algorithm 1 thetas (a tape's; null: not kept)
  uint8_t* fflag_face;        // [d][E*nfp] bit 0: that product below 1, bit 1: the guard
  uint32_t* flag_or;          // [1] OR of every element flag since the last query
  double* theta_elem;         // [E] product of Algorithm 2 thetas
  uint32_t* eflags;           // [E] element flags of the last step with statistics
  double* stats_rows;         // per-block rows of the step statistics
  // boundaries: kind of side (d, s), 0 periodic, 1 outflow, 2 wall, 3 Dirichlet
  int bc[2][2];
  const double* ghost;        // Dirichlet face data, per side 2d+s: [3][M][lines_d*nfp]
  double* theta_left;         // [ny*nfp + nx*nfp] Algorithm 1 theta of the left boundary half faces
  uint32_t* guard_left;
  double ra, reps, rl, rq;    // relaxation systems: a, eps, f(u) = rl u + rq u^2/2
};

__device__ inline PhysParams phys_params(const KParams& kp, double ch) {
  return PhysParams{kp.g, kp.gamma, ch, kp.ra, kp.reps, kp.rl, kp.rq};
}

__device__ inline int nbr_elem(const KParams& kp, int e, int d, int side) {
  int ex = e % kp.nx, ey = e / kp.nx;
  if (d == 0) ex = side ? (ex + 1 == kp.nx ? 0 : ex + 1) : (ex == 0 ? kp.nx - 1 : ex - 1);
  else ey = side ? (ey + 1 == kp.ny ? 0 : ey + 1) : (ey == 0 ? kp.ny - 1 : ey - 1);
  return ex + kp.nx * ey;
}

// element e lies on the non-periodic side (d, side) of the mesh
__device__ inline bool on_boundary(const KParams& kp, int e, int d, int side) {
  if (kp.bc[d][side] == 0) return false;
  const int c = d == 0 ? e % kp.nx : e / kp.nx, n = d == 0 ? kp.nx : kp.ny;
  return side ? c == n - 1 : c == 0;
}
// neighbour whose raw alpha enters the smoothing of element e: across a
// non-periodic side there is none, and e itself stands in (no effect on the max)
__device__ inline int alpha_nbr(const KParams& kp, int e, int d, int side) {
  return on_boundary(kp, e, d, side) ? e : nbr_elem(kp, e, d, side);
}

template <int n1>
__device__ __host__ constexpr int node_at(int d, int q, int r) { return d == 0 ? r + n1 * q : q + n1 * r; }

// Where the element-local half of the correction terms of eq.
// crkfr.non.cons.final goes.  The nine-variable 2-D systems (two lanes per
// point in the stage and face kernels) fold C = F_tr + B_d(u^n_tr) U_tr at the
// element's own faces into the volume residual in the stage kernel, and the
// update adds F^num g'/dx: the face kernel writes only F^-, F^+.  The other
// systems, whose stage kernel is light, keep the correction jumps D^± = F^± - C^±
// that the face kernel writes beside F^±.
template <class Ph>
__host__ __device__ constexpr bool fold_correction() { return Ph::DIM == 2 && Ph::M >= 8; }

__device__ inline double theta_limit(double eps, double Pa, double Pb, bool& guard) {
  // theta_{P_k}(eps, u_a, u_b) for a concave P_k (eq. theta.formula), weight on the
  // candidate u_b; admissible candidates keep theta = 1
  if (Pa <= 0.0) { guard = true; return 0.0; }
  if (Pb >= eps) return 1.0;
  return fmin(1.0, fabs((eps - Pa) / (Pb - Pa)));
}

// ------------------------------------------------------------------------
// k_pre: one thread per solution point, EPB elements per block (coalesced
// loads); per element: mean state, ideal wave speeds, Lambda_e and the raw
// smoothness indicator; per block: the maximum of Lambda_e.
//
// The per-point kernels are written as device bodies over one block of EPB
// elements (block index blk) so that the single-problem kernels and the
// batched kernels (several problems, one launch) run the same code.  A block
// of NT threads has ceil(NT/P) element slots in LDS; slots at or beyond EPB
// hold no element (their threads only take part in the barriers).
// Rows are padded by one double: with P a multiple of 16 (2-D, N = 3) the
// threads that walk a row each (one per variable, one per element) would
// otherwise all hit the same LDS banks.
template <class Ph, int N, int NT>
struct PreLds {
  static constexpr int P = ipow(N + 1, Ph::DIM), EL = (NT + P - 1) / P;
  double s_u[EL][Ph::M][P + 1];
  double s_q[EL][P + 1];   // indicator variable at the nodes, then the squared modes
  double s_t[EL][P + 1];   // 2-D: the first pass of the modal projection
  double s_ub[EL][Ph::M];
  double s_lam[EL][2];     // (|v_d| + c_d)/dx_d of each direction
};

// The element data from the state x at the thread's node (x: every variable at
// node p of element e, the thread's): pre_body without its loads, also run by
// the update kernel on the state it has just written (chained steps).
template <class Ph, int N, int EPB, int NT>
__device__ __forceinline__ void pre_from_state(const KParams& kp, PreLds<Ph, N, NT>& L, const double (&x)[Ph::M],
                                               int blk, double* part_out) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM);
  auto& s_u = L.s_u;
  auto& s_q = L.s_q;
  auto& s_t = L.s_t;
  auto& s_ub = L.s_ub;
  auto& s_lam = L.s_lam;
  const int tid = threadIdx.x;
  const int le = tid / P, p = tid - le * P;
  const PhysParams pp = phys_params(kp, 0.0);
  const bool want_alpha = kp.blending >= 1 && kp.alpha_force < 0.0;
#pragma unroll
  for (int v = 0; v < M; ++v) s_u[le][v][p] = x[v];
  if (want_alpha) s_q[le][p] = Ph::indicator(x, pp);
  elem_sync<ipow(N + 1, Ph::DIM)>();
  // element mean of each variable, summed over the nodes in order
  for (int v = p; v < M; v += P) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const double wr = DIM == 1 ? kp.w[r] : kp.w[r % n1] * kp.w[r / n1];
      s += wr * s_u[le][v][r];
    }
    s_ub[le][v] = s;
  }
  // smoothness indicator, part 1: the modes of q in the orthonormal Legendre
  // basis, one thread per mode (1-D: m_k = sum_r w_r L_k(xi_r) q_r; 2-D in two
  // passes, t[k][jj] = sum_i w_i L_k(xi_i) q(i, jj), then
  // m[l][k] = sum_jj w_jj L_l(xi_jj) t[k][jj]); squared modes replace q in s_q
  double mode = 0.0;
  if (want_alpha) {
    if constexpr (DIM == 1) {
#pragma unroll
      for (int r = 0; r < n1; ++r) mode += kp.w[r] * s_q[le][r] * kp.Leg[p][r];
    } else {
      const int k = p % n1, jj = p / n1;
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < n1; ++i) t += kp.w[i] * kp.Leg[k][i] * s_q[le][i + n1 * jj];
      s_t[le][p] = t;
    }
  }
  elem_sync<ipow(N + 1, Ph::DIM)>();
  if (want_alpha) {
    if constexpr (DIM == 2) {
      const int k = p % n1, l = p / n1;
#pragma unroll
      for (int jj = 0; jj < n1; ++jj) mode += kp.w[jj] * kp.Leg[l][jj] * s_t[le][k + n1 * jj];
    }
    s_q[le][p] = mode * mode;
  }
  // The wave speeds and the indicator energies are short serial tasks, one per
  // (element, direction) and one per element.  They run on consecutive threads
  // of the workgroup, each group from a wave boundary where it fits, so that
  // one or two waves execute them instead of every wave with a few lanes on.
  constexpr int NS = EPB * DIM;
  constexpr int NS64 = (NS + 63) / 64 * 64;
  constexpr int E0 = NS64 + EPB <= NT ? NS64 : NS;
  __syncthreads();  // the tasks read the means and squared modes of every element
  if (tid < NS) {
    // the ideal speeds at the mean of element l in direction d
    const int l = tid / DIM, d = tid - l * DIM;
    const int el = blk * EPB + l;
    double lam = 0.0;
    if (el < kp.E) {
      double ub[M];
#pragma unroll
      for (int v = 0; v < M; ++v) ub[v] = s_ub[l][v];
      double av, c;
      if constexpr (DIM == 2) Ph::speeds_rd(ub, d, av, c, pp);
      else Ph::template speeds<0>(ub, av, c, pp);
      lam = (av + c) * (d ? kp.inv_dx[1] : kp.inv_dx[0]);
      kp.speeds[(size_t)el * 2 * DIM + 2 * d] = av;
      kp.speeds[(size_t)el * 2 * DIM + 2 * d + 1] = c;
    }
    s_lam[l][d] = lam;
  } else if (want_alpha && tid >= E0 && tid < E0 + EPB) {
    // smoothness indicator, part 2, for element l: energy fractions of the
    // highest modes, logistic map, clip and cap (mode (l, k) of degree
    // max(k, l) at slot k + n1 l)
    const int l = tid - E0;
    const int el = blk * EPB + l;
    if (el < kp.E) {
      double tot = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const double m2 = s_q[l][r];
        const int deg = DIM == 1 ? r : (r % n1 > r / n1 ? r % n1 : r / n1);
        tot += m2;
        if (deg <= N - 1) c1 += m2;
        if (deg <= N - 2) c2 += m2;
      }
      double En = tot > 0.0 ? (tot - c1) / tot : 0.0;
      if (N >= 2) {
        const double e2 = c1 > 0.0 ? (c1 - c2) / c1 : 0.0;
        En = En >= e2 ? En : e2;
      }
      double a = 1.0 / (1.0 + exp(-(kp.ind_s / kp.ind_T) * (En - kp.ind_T)));
      if (a < kp.alpha_min) a = 0.0;
      if (a > 1.0 - kp.alpha_min) a = 1.0;
      a = fmin(a, kp.alpha_max);
      kp.alpha_raw[el] = a;
    }
  }
  // Lambda_e = sum over the directions, then the largest of the block.  When
  // the speed tasks are all in the first wave, that wave alone waits for them.
  if constexpr (NS <= 64 && LWFR_WAVE_LOCAL_SYNC) {
    if (tid < 64) elem_sync<64>();
  } else {
    __syncthreads();
  }
  if (tid == 0) {
    double m = 0.0;
    for (int l = 0; l < EPB; ++l) m = fmax(m, DIM == 2 ? s_lam[l][0] + s_lam[l][1] : s_lam[l][0]);
    part_out[0] = m;
  }
}

template <class Ph, int N, int EPB, int NT>
__device__ __forceinline__ void pre_body(const KParams& kp, PreLds<Ph, N, NT>& L, const double* __restrict__ un,
                                         int blk, double* part_out) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM);
  const int tid = threadIdx.x;
  const int le = tid / P, p = tid - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  // lanes without an element read element 0 (unconditional loads pipeline;
  // a load under a lane condition waits for its data before the next one)
  const int es = act ? e : 0;
  double x[M];
#pragma unroll
  for (int v = 0; v < M; ++v) x[v] = un[((size_t)v * kp.E + es) * P + p];
  pre_from_state<Ph, N, EPB, NT>(kp, L, x, blk, part_out);
}

template <class Ph, int N, int EPB>
__global__ void __launch_bounds__(EPB* ipow(N + 1, Ph::DIM)) k_pre(const KParams kp, const double* __restrict__ un) {
  constexpr int NT = EPB * ipow(N + 1, Ph::DIM);
  __shared__ PreLds<Ph, N, NT> L;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  pre_body<Ph, N, EPB, NT>(kp, L, un, b, kp.part + b);
}

// Max / min over a workgroup of whole waves: within each wave by lane
// exchanges, then over the waves' results through LDS (one barrier).  The
// result is valid in every thread.  Max and min are exact, so the order of the
// reduction does not change the result.
__device__ inline double wave_reduce_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}
__device__ inline double wave_reduce_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o));
  return x;
}
template <bool MAX>
__device__ inline double block_reduce(double x, double* s_w /* >= blockDim.x / 64 */) {
  x = MAX ? wave_reduce_max(x) : wave_reduce_min(x);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) s_w[w] = x;
  __syncthreads();
  double r = s_w[0];
  for (int k = 1; k < nw; ++k) r = MAX ? fmax(r, s_w[k]) : fmin(r, s_w[k]);
  return r;
}

// k_dt: Lambda, the largest of the block maxima of k_pre (or of the update that
// formed this step's element data), and dt.  Without GLM-MHD's c_h one block of
// 1024 threads finishes both.  With it, k_dt is the first level of Lambda's
// reduction: block g writes the largest of partials [1024 g, 1024 g + 1024)
// to part3[g], and k_ch finishes Lambda and dt.  Max is exact, so both forms
// give the same bits.
__global__ void __launch_bounds__(1024) k_dt(const KParams kp, double* d_dt_ch, int has_ch) {
  __shared__ double s_w[16];
  const int n = kp.nblk_pre, st = blockDim.x;
  if (has_ch) {
    const int i = blockIdx.x * st + threadIdx.x;
    const double m = block_reduce<true>(i < n ? fmax(0.0, kp.part[i]) : 0.0, s_w);
    if (threadIdx.x == 0) kp.part3[blockIdx.x] = m;
    return;
  }
  // 16 loads in flight per thread (up to 16384 partials in one round trip); an
  // index past the end reads the thread's first one again, which leaves the max
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 16 * st) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int idx = i + k * st;
      v[k] = kp.part[idx < n ? idx : i];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) m = fmax(m, v[k]);
  }
  const double lam_all = block_reduce<true>(m, s_w);
  if (threadIdx.x == 0) {
    const double lam = lam_all;
    const double dt = kp.dt_in > 0.0 ? kp.dt_in : kp.cs_cfl / lam;
    kp.scal[0] = dt;
    kp.scal[2] = lam;
    const double ch = kp.ch_in >= 0.0 ? kp.ch_in : 0.0;
    kp.scal[1] = ch;
    if (d_dt_ch) { d_dt_ch[0] = dt; d_dt_ch[1] = ch; }
  }
}

// k_ch: GLM speed candidate of each element: the largest c with
// wx max(c_x, c) + wy max(c_y, c) <= Lambda - (wx |v_x| + wy |v_y|).
// Every block first forms Lambda from k_dt's first-level maxima; block 0
// stores Lambda and dt.
__global__ void __launch_bounds__(256) k_ch(const KParams kp) {
  __shared__ double s_w[4], s_l[4];
  double m = 0.0;
  for (int i = threadIdx.x; i < kp.nblk_dt; i += blockDim.x) m = fmax(m, kp.part3[i]);
  const double lam = block_reduce<true>(m, s_l);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    kp.scal[0] = kp.dt_in > 0.0 ? kp.dt_in : kp.cs_cfl / lam;
    kp.scal[2] = lam;
  }
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double ce = INFINITY;
  if (e < kp.E) {
    const double* sp = kp.speeds + (size_t)e * 4;
    const double wx = kp.inv_dx[0], wy = kp.inv_dx[1];
    const double R = lam - (sp[0] * wx + sp[2] * wy);
    double lo = sp[1], hi = sp[3], wlo = wx, whi = wy;
    if (lo > hi) { double t = lo; lo = hi; hi = t; t = wlo; wlo = whi; whi = t; }
    ce = (wlo + whi) * hi >= R ? (R - whi * hi) / wlo : R / (wlo + whi);
  }
  const double cmin = block_reduce<false>(ce, s_w);
  if (threadIdx.x == 0) kp.part2[blockIdx.x] = cmin;
}

__global__ void __launch_bounds__(1024) k_ch_fin(const KParams kp, double* d_dt_ch) {
  __shared__ double s_w[16];
  double m0 = INFINITY, m1 = INFINITY;
  const int n = kp.nblk_ch, st = blockDim.x;
  int i = threadIdx.x;
  for (; i + st < n; i += 2 * st) {
    m0 = fmin(m0, kp.part2[i]);
    m1 = fmin(m1, kp.part2[i + st]);
  }
  for (; i < n; i += st) m0 = fmin(m0, kp.part2[i]);
  const double ch = block_reduce<false>(fmin(m0, m1), s_w);
  if (threadIdx.x == 0) {
    kp.scal[1] = ch;
    if (d_dt_ch) { d_dt_ch[0] = kp.scal[0]; d_dt_ch[1] = ch; }
  }
}

// ------------------------------------------------------------------------
// k_stages: one thread per solution point, EPB elements per block.
// Inner stages u^(s) = u^n - dt sum_{k<s} a_sk L^(k) with the local operator
// L = sum_d [D_d f_d(u) + B_d(u) D_d u]/dx_d (paper §3, stages above eq.
// crkfr.non.cons.final); F_d and U accumulate with the weights b_s.  The sums
// S_t = sum_k a_tk L^(k) of later stages are carried as running partial sums
// (same order of summation), so only the partial sums still needed stay live.
// Output: the volume part of the high order residual, B^loc + sum_d D_d F_d/dx_d,
// which by linearity of D_d equals sum_s b_s L^(s) (written to the output state
// buffer), and the face traces of F_d and U.
template <class Tab>
__host__ __device__ constexpr int first_nz_t(int t) {
  for (int k = 0; k < t; ++k)
    if (Tab::a(t, k) != 0.0) return k;
  return -1;
}
template <int N>
__host__ __device__ constexpr int first_nz(int t) { return first_nz_t<Tableau<N>>(t); }
// first source term of stage t in the implicit part (k < t)
template <class Tab>
__host__ __device__ constexpr int first_nzi(int t) {
  for (int k = 0; k < t; ++k)
    if (Tab::ai(t, k) != 0.0) return k;
  return -1;
}

template <class Ph, int N, int NT>
struct StagesLds {
  static constexpr int DIM = Ph::DIM, M = Ph::M, P = ipow(N + 1, DIM), EL = (NT + P - 1) / P;
  static constexpr int NCD = Ph::NCD > 0 ? Ph::NCD : 1;
  static constexpr int NBUF = (DIM * M + DIM * NCD) > (DIM * M + M) ? (DIM * M + DIM * NCD) : (DIM * M + M);
  double s_buf[EL][NBUF][P + LWFR_STAGES_PAD];
};

// Outputs of the element-local phase, shared by the stage body and the
// approximate Lax-Wendroff body: the face traces of the time averages F_d and
// U, the volume residual and the smoothed blending coefficient.  With
// the correction folded (fold_correction) the volume residual written is
// R = Ra - sum_d (C_{d,R} g_R'(xi) + C_{d,L} g_L'(xi)) / dx_d along the lines
// through the point, with C = F_tr + B_d(u^n_tr) U_tr at the element's own
// faces, so that the update adds only F^num g'/dx; otherwise R = Ra.
// sb: the element's LDS rows (at least DIM*M + M of them); every thread of the
// workgroup calls it (it synchronises).
template <class Ph, int d>
__device__ inline void correction_offset(const double* a, const double* U, double* C, const PhysParams& pp) {
  double t[Ph::M];
  Ph::template ncprod<d>(a, U, t, pp);
#pragma unroll
  for (int v = 0; v < Ph::M; ++v) C[v] += t[v];
}

template <class Ph, int N, int NB, int PS>
__device__ __forceinline__ void stage_outputs_fold(const KParams& kp, double (&sb)[NB][PS], int p, int e, bool act,
                                              const double (&Fa)[Ph::DIM][Ph::M], const double (&Ua)[Ph::M],
                                              const double (&Ra)[Ph::M], const double* __restrict__ un_g,
                                              double* __restrict__ rvol_g, double* d_alpha_out) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  constexpr int NFT = 2 * DIM * NFP;          // face points of the element (both sides, every direction)
  constexpr int NOWN = (NFT + P - 1) / P;     // face points per thread
  static_assert(NB >= DIM * M + M && PS >= P, "LDS rows");
  static_assert(NFT * M <= NB * PS, "LDS room for the correction offsets");
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  // time-averaged flux and solution to LDS for the face traces
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int v = 0; v < M; ++v) sb[d * M + v][p] = Fa[d][v];
#pragma unroll
  for (int v = 0; v < M; ++v) sb[DIM * M + v][p] = Ua[v];
  elem_sync<ipow(N + 1, Ph::DIM)>();

  if (act) {
#pragma unroll
    for (int v = 0; v < M; ++v) rvol_g[((size_t)v * kp.E + e) * P + p] = Ra[v];
  }
  // face traces, one face point (all variables) per thread, and the correction
  // offsets C of those face points (fenced from the stage loop: its loads are
  // not to be hoisted into it)
  __builtin_amdgcn_sched_barrier(0);
  const size_t nf = (size_t)kp.E * NFP;
  double C[NOWN][M];
#pragma unroll
  for (int k = 0; k < NOWN; ++k) {
    const int w = p + k * P;
    if (!act || w >= NFT) continue;
    const int d = w / (2 * NFP);
    const int rem = w - d * 2 * NFP;
    const int side = rem / NFP;
    const int q = rem - side * NFP;
    const double* V = side ? kp.VR : kp.VL;
    const size_t fo = (size_t)e * NFP + q;
    // three passes (u^n, U, then F), each fenced from the next, so that few
    // loads are in flight at once
    double a[M], U[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) t += V[r] * un_g[((size_t)v * kp.E + e) * P + (d == 0 ? node_at<n1>(0, q, r) : node_at<n1>(1, q, r))];
      a[v] = t;
    }
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) t += V[r] * sb[DIM * M + v][d == 0 ? node_at<n1>(0, q, r) : node_at<n1>(1, q, r)];
      U[v] = t;
      kp.Utr[((size_t)(d * 2 + side) * M + v) * nf + fo] = t;
    }
#pragma unroll
    for (int v = 0; v < M; ++v) C[k][v] = 0.0;
    if (d == 0) correction_offset<Ph, 0>(a, U, C[k], pp);
    else if constexpr (DIM == 2) correction_offset<Ph, 1>(a, U, C[k], pp);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) t += V[r] * sb[d * M + v][d == 0 ? node_at<n1>(0, q, r) : node_at<n1>(1, q, r)];
      kp.Ftr[((size_t)(d * 2 + side) * M + v) * nf + fo] = t;
      C[k][v] = t + C[k][v];
    }
  }
  elem_sync<ipow(N + 1, Ph::DIM)>();  // every read of the F and U rows is done
  double* flat = &sb[0][0];
#pragma unroll
  for (int k = 0; k < NOWN; ++k) {
    const int w = p + k * P;
    if (act && w < NFT) {
#pragma unroll
      for (int v = 0; v < M; ++v) flat[w * M + v] = C[k][v];
    }
  }
  elem_sync<ipow(N + 1, Ph::DIM)>();
  if (act) {
    double R[M];
#pragma unroll
    for (int v = 0; v < M; ++v) R[v] = rvol_g[((size_t)v * kp.E + e) * P + p];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int q = DIM == 1 ? 0 : (d == 0 ? p / n1 : p % n1), ii = DIM == 1 ? p : (d == 0 ? p % n1 : p / n1);
      const int wR = d * 2 * NFP + NFP + q, wL = d * 2 * NFP + q;
#pragma unroll
      for (int v = 0; v < M; ++v)
        R[v] -= (flat[wR * M + v] * kp.gR[ii] + flat[wL * M + v] * kp.gL[ii]) * kp.inv_dx[d];
    }
#pragma unroll
    for (int v = 0; v < M; ++v) rvol_g[((size_t)v * kp.E + e) * P + p] = R[v];
    // blending coefficient of the element (smoothed over face neighbours)
    if (p == 0) {
      double a;
      if (kp.alpha_force >= 0.0) a = kp.alpha_force;
      else if (kp.blending == 0) a = 0.0;
      else {
        a = kp.alpha_raw[e];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
          for (int sd = 0; sd < 2; ++sd) a = fmax(a, 0.5 * kp.alpha_raw[alpha_nbr(kp, e, d, sd)]);
      }
      kp.alpha[e] = a;
      if (d_alpha_out) d_alpha_out[e] = a;
    }
  }
  elem_sync<ipow(N + 1, Ph::DIM)>();  // the LDS rows are free again (batched tile loops reuse them)
}

template <class Ph, int N, int NB, int PS>
__device__ __forceinline__ void stage_outputs_plain(const KParams& kp, double (&sb)[NB][PS], int p, int e, bool act,
                                              const double (&Fa)[Ph::DIM][Ph::M], const double (&Ua)[Ph::M],
                                              const double (&Ra)[Ph::M], const double* __restrict__ un_g,
                                              double* __restrict__ rvol_g, double* d_alpha_out) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  static_assert(NB >= DIM * M + M && PS >= P, "LDS rows");
  // time-averaged flux and solution to LDS for the face traces
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int v = 0; v < M; ++v) sb[d * M + v][p] = Fa[d][v];
#pragma unroll
  for (int v = 0; v < M; ++v) sb[DIM * M + v][p] = Ua[v];
  elem_sync<ipow(N + 1, Ph::DIM)>();

  if (act) {
#pragma unroll
    for (int v = 0; v < M; ++v) rvol_g[((size_t)v * kp.E + e) * P + p] = Ra[v];
    // face traces: (variable, face point) pairs of the element, variable
    // slowest, over the element's threads
    constexpr int NFT = 2 * DIM * NFP;
    for (int w = p; w < NFT * M; w += P) {
      const int v = w / NFT, t = w - v * NFT;
      const int d = t / (2 * NFP);
      const int rem = t - d * 2 * NFP;
      const int side = rem / NFP;
      const int q = rem - side * NFP;
      const double* V = side ? kp.VR : kp.VL;
      const size_t nf = (size_t)kp.E * NFP;
      const size_t fo = (size_t)e * NFP + q;
      {
        double tf = 0.0, tu = 0.0;
#pragma unroll
        for (int r = 0; r < n1; ++r) {
          const int nd = d == 0 ? node_at<n1>(0, q, r) : node_at<n1>(1, q, r);
          tf += V[r] * sb[d * M + v][nd];
          tu += V[r] * sb[DIM * M + v][nd];
        }
        const size_t o = ((size_t)(d * 2 + side) * M + v) * nf + fo;
        kp.Ftr[o] = tf;
        kp.Utr[o] = tu;
      }
    }
    // blending coefficient of the element (smoothed over face neighbours)
    if (p == 0) {
      double a;
      if (kp.alpha_force >= 0.0) a = kp.alpha_force;
      else if (kp.blending == 0) a = 0.0;
      else {
        a = kp.alpha_raw[e];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
          for (int sd = 0; sd < 2; ++sd) a = fmax(a, 0.5 * kp.alpha_raw[alpha_nbr(kp, e, d, sd)]);
      }
      kp.alpha[e] = a;
      if (d_alpha_out) d_alpha_out[e] = a;
    }
  }
}

// the outputs of the element-local phase (see fold_correction)
template <class Ph, int N, int NB, int PS>
__device__ __forceinline__ void stage_outputs(const KParams& kp, double (&sb)[NB][PS], int p, int e, bool act,
                                              const double (&Fa)[Ph::DIM][Ph::M], const double (&Ua)[Ph::M],
                                              const double (&Ra)[Ph::M], const double* __restrict__ un_g,
                                              double* __restrict__ rvol_g, double* d_alpha_out) {
  if constexpr (fold_correction<Ph>())
    stage_outputs_fold<Ph, N>(kp, sb, p, e, act, Fa, Ua, Ra, un_g, rvol_g, d_alpha_out);
  else
    stage_outputs_plain<Ph, N>(kp, sb, p, e, act, Fa, Ua, Ra, un_g, rvol_g, d_alpha_out);
}

// Tab: the explicit tableau of degree N, or for a system with a source its
// IMEX pair (the source enters each stage through the implicit part, eq.
// crkfr.inner, and its b-weighted average, eq. avg.source, is subtracted from
// the volume residual).
template <class Ph, int N, int EPB, int NT, class Tab = Tableau<N>, bool OT = false>
__device__ __forceinline__ void stages_body(const KParams& kp, StagesLds<Ph, N, NT>& L,
                                            const double* __restrict__ un_g, double* __restrict__ rvol_g,
                                            double* d_alpha_out, int blk) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  constexpr int NCD = Ph::NCD > 0 ? Ph::NCD : 1;
  constexpr int S = Tab::S;
  auto& s_buf = L.s_buf;

  const int tid = body_tid<OT>();
  const int le = tid / P, p = tid - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  const int i = p % n1, j = p / n1;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);

  double un[M];
#pragma unroll
  for (int v = 0; v < M; ++v) un[v] = un_g[((size_t)v * kp.E + (act ? e : 0)) * P + p];
  double Drow[DIM][n1];
#pragma unroll
  for (int r = 0; r < n1; ++r) {
    Drow[0][r] = kp.D[i][r];
    if constexpr (DIM == 2) Drow[1][r] = kp.D[j][r];
  }

  double Fa[DIM][M], Ua[M], Ra[M], Sp[S][M], u[M];
  double Q[Ph::SRC ? S : 1][M], Sa[M];  // implicit-part sums and the averaged source
#pragma unroll
  for (int v = 0; v < M; ++v) {
    Ua[v] = 0.0; Ra[v] = 0.0; Sa[v] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fa[d][v] = 0.0;
  }

#pragma unroll
  for (int st = 0; st < S; ++st) {
#pragma unroll
    for (int v = 0; v < M; ++v) u[v] = first_nz_t<Tab>(st) >= 0 ? un[v] - dt * Sp[st][v] : un[v];
    if constexpr (Ph::SRC) {
      // + dt sum_{k<st} a_st,k s(u^(k)), then the pointwise implicit solve
      double r[M], sv[M];
#pragma unroll
      for (int v = 0; v < M; ++v) r[v] = first_nzi<Tab>(st) >= 0 ? u[v] + dt * Q[st][v] : u[v];
      if (Tab::ai(st, st) != 0.0) Ph::implicit(r, dt * Tab::ai(st, st), u, pp);
      else {
#pragma unroll
        for (int v = 0; v < M; ++v) u[v] = r[v];
      }
      Ph::source(u, sv, pp);
      if (Tab::bi(st) != 0.0) {
#pragma unroll
        for (int v = 0; v < M; ++v) Sa[v] += Tab::bi(st) * sv[v];
      }
#pragma unroll
      for (int t = st + 1; t < S; ++t) {
        const double a = Tab::ai(t, st);
        if (a != 0.0) {
#pragma unroll
          for (int v = 0; v < M; ++v) Q[t][v] = first_nzi<Tab>(t) == st ? a * sv[v] : Q[t][v] + a * sv[v];
        }
      }
    }
    double f[DIM][M];
    Ph::template flux<0>(u, f[0], pp);
    if constexpr (DIM == 2) Ph::template flux<1>(u, f[1], pp);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int v = 0; v < M; ++v) s_buf[le][d * M + v][p] = f[d][v];
    if constexpr (Ph::NCD > 0) {
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) s_buf[le][DIM * M + d * NCD + c][p] = u[Ph::nc_comp(d, c)];
    }
    const double bs = Tab::b(st);
    if (bs != 0.0) {
#pragma unroll
      for (int v = 0; v < M; ++v) {
        Ua[v] += bs * u[v];
#pragma unroll
        for (int d = 0; d < DIM; ++d) Fa[d][v] += bs * f[d][v];
      }
    }
    elem_sync<ipow(N + 1, Ph::DIM)>();
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
        for (int r = 0; r < n1; ++r) sacc += Drow[d][r] * s_buf[le][d * M + v][node_at<n1>(d, q, r)];
        df[v] = sacc;
        w[v] = 0.0;
      }
      if constexpr (Ph::NCD > 0) {
#pragma unroll
        for (int c = 0; c < Ph::NCD; ++c) {
          double sacc = 0.0;
#pragma unroll
          for (int r = 0; r < n1; ++r) sacc += Drow[d][r] * s_buf[le][DIM * M + d * NCD + c][node_at<n1>(d, q, r)];
          w[Ph::nc_comp(d, c)] = sacc;
        }
      }
      if (d == 0) Ph::template ncprod<0>(u, w, nc, pp);
      else Ph::template ncprod<(DIM > 1 ? 1 : 0)>(u, w, nc, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) Ls[v] += (df[v] + nc[v]) * kp.inv_dx[d];
    }
    elem_sync<ipow(N + 1, Ph::DIM)>();
    if (bs != 0.0) {
#pragma unroll
      for (int v = 0; v < M; ++v) Ra[v] += bs * Ls[v];
    }
    // fold L^(st) into the running sums of the later stages that use it
#pragma unroll
    for (int t = st + 1; t < S; ++t) {
      const double a = Tab::a(t, st);
      if (a != 0.0) {
#pragma unroll
        for (int v = 0; v < M; ++v) Sp[t][v] = first_nz_t<Tab>(t) == st ? a * Ls[v] : Sp[t][v] + a * Ls[v];
      }
    }
  }
  if constexpr (Ph::SRC) {
#pragma unroll
    for (int v = 0; v < M; ++v) Ra[v] -= Sa[v];
  }

  stage_outputs<Ph, N>(kp, s_buf[le], p, e, act, Fa, Ua, Ra, un_g, rvol_g, d_alpha_out);
}

// ------------------------------------------------------------------------
// Approximate Lax-Wendroff time averages (the alternative to the cRK stages):
//   F_d = sum_{k<=N} dt^k/(k+1)! d_t^k f_d, U = sum_k dt^k/(k+1)! d_t^k u,
//   B^loc = sum_k dt^k/(k+1)! d_t^k [B u_x],
// with d_t^{k+1} u = -(sum_d D_d d_t^k f_d / dx_d + d_t^k [B u_x]) and the time
// derivatives of f_d and B(u) u_x from central differences at tau = j dt along
// the Taylor state u(tau) = sum_{m<=k} tau^m/m! d_t^m u (3 points for N <= 2,
// 5 for N >= 3).  One thread per solution point keeps the Taylor coefficients
// c[m] and the derivatives along each line of the components B reads; the
// D_d products go through LDS.

// weight of tau = j dt in dt^k d_t^k g (j in -2..2)
__host__ __device__ constexpr double alw_weight(int N, int k, int j) {
  return k == 0 ? (j == 0 ? 1.0 : 0.0)
       : N <= 2 ? ((j < -1 || j > 1) ? 0.0 : k == 1 ? 0.5 * j : (j == 0 ? -2.0 : 1.0))
       : k == 1 ? (j == -2 ? 1.0 / 12 : j == -1 ? -8.0 / 12 : j == 1 ? 8.0 / 12 : j == 2 ? -1.0 / 12 : 0.0)
       : k == 2 ? (j == 0 ? -30.0 / 12 : (j == -1 || j == 1) ? 16.0 / 12 : -1.0 / 12)
       : k == 3 ? (j == -2 ? -0.5 : j == -1 ? 1.0 : j == 1 ? -1.0 : j == 2 ? 0.5 : 0.0)
                : (j == 0 ? 6.0 : (j == -1 || j == 1) ? -4.0 : 1.0);
}

template <class Ph, int N, int EPB, int NT>
__device__ __forceinline__ void alw_body(const KParams& kp, StagesLds<Ph, N, NT>& L, const double* __restrict__ un_g,
                                         double* __restrict__ rvol_g, double* d_alpha_out, int blk) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM);
  constexpr int NCD = Ph::NCD > 0 ? Ph::NCD : 1;
  constexpr int J = N <= 2 ? 1 : 2;
  auto& s_buf = L.s_buf;
  const int tid = threadIdx.x;
  const int le = tid / P, p = tid - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  const int i = p % n1, j = p / n1;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);

  double c[N + 1][M];        // d_t^m u at this node
  double Dc[N + 1][DIM][NCD];  // D_d (d_t^m u) of the components B_d reads, / dx_d
#pragma unroll
  for (int v = 0; v < M; ++v) c[0][v] = un_g[((size_t)v * kp.E + (act ? e : 0)) * P + p];
  // derivative along direction d of LDS row `row` at this node
  auto dline = [&](int d, int row) {
    const int q = d == 0 ? j : i, ii = d == 0 ? i : j;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < n1; ++r) acc += kp.D[ii][r] * s_buf[le][row][node_at<n1>(d, q, r)];
    return acc;
  };
  // D_d of the nc components of c[m]
  auto nc_derivs = [&](int m) {
    if constexpr (Ph::NCD > 0) {
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int cc = 0; cc < Ph::NCD; ++cc) s_buf[le][d * NCD + cc][p] = c[m][Ph::nc_comp(d, cc)];
      __syncthreads();
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int cc = 0; cc < Ph::NCD; ++cc) Dc[m][d][cc] = dline(d, d * NCD + cc) * kp.inv_dx[d];
      __syncthreads();
    }
  };
  nc_derivs(0);

  double Fa[DIM][M], Ua[M], Ra[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    Ua[v] = 0.0; Ra[v] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fa[d][v] = 0.0;
  }
  double fact = 1.0, dtk = 1.0;  // (k+1)!, dt^k
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    fact *= (k + 1);
    const double ifact = 1.0 / fact;  // constants after unrolling: no division left
    double fk[DIM][M], hk[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      hk[v] = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) fk[d][v] = 0.0;
    }
#pragma unroll
    for (int jj = -J; jj <= J; ++jj) {
      const double wj = alw_weight(N, k, jj);
      if (wj == 0.0) continue;
      // Taylor state and its line derivatives at tau = jj dt
      double st[M], tm[N + 1];
      tm[0] = 1.0;
#pragma unroll
      for (int m = 1; m <= k; ++m) tm[m] = tm[m - 1] * (jj * dt) * (1.0 / m);
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double a = c[0][v];
#pragma unroll
        for (int m = 1; m <= k; ++m) a += tm[m] * c[m][v];
        st[v] = a;
      }
      double f[M];
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        if (d == 0) Ph::template flux<0>(st, f, pp);
        else Ph::template flux<(DIM > 1 ? 1 : 0)>(st, f, pp);
#pragma unroll
        for (int v = 0; v < M; ++v) fk[d][v] += wj * f[v];
        if constexpr (Ph::NCD > 0) {
          double w[M], nc[M];
#pragma unroll
          for (int v = 0; v < M; ++v) w[v] = 0.0;
#pragma unroll
          for (int cc = 0; cc < Ph::NCD; ++cc) {
            double a = Dc[0][d][cc];
#pragma unroll
            for (int m = 1; m <= k; ++m) a += tm[m] * Dc[m][d][cc];
            w[Ph::nc_comp(d, cc)] = a;
          }
          if (d == 0) Ph::template ncprod<0>(st, w, nc, pp);
          else Ph::template ncprod<(DIM > 1 ? 1 : 0)>(st, w, nc, pp);
#pragma unroll
          for (int v = 0; v < M; ++v) hk[v] += wj * nc[v];
        }
      }
    }
    // sum_d D_d fk_d / dx_d through LDS
    double r[M];
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int v = 0; v < M; ++v) s_buf[le][d * M + v][p] = fk[d][v];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double a = hk[v];
#pragma unroll
      for (int d = 0; d < DIM; ++d) a += dline(d, d * M + v) * kp.inv_dx[d];
      r[v] = a;
    }
    __syncthreads();
    const double uw = dtk * ifact;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      Ua[v] += uw * c[k][v];
      Ra[v] += r[v] * ifact;
#pragma unroll
      for (int d = 0; d < DIM; ++d) Fa[d][v] += fk[d][v] * ifact;
    }
    if (k < N) {
      const double idtk = -1.0 / dtk;
#pragma unroll
      for (int v = 0; v < M; ++v) c[k + 1][v] = r[v] * idtk;
      nc_derivs(k + 1);
      dtk *= dt;
    }
  }
  stage_outputs<Ph, N>(kp, s_buf[le], p, e, act, Fa, Ua, Ra, un_g, rvol_g, d_alpha_out);
}

template <class Ph, int N, int EPB>
__global__ void __launch_bounds__(EPB* ipow(N + 1, Ph::DIM))
    k_stages_alw(const KParams kp, const double* __restrict__ un_g, double* __restrict__ rvol_g, double* d_alpha_out) {
  constexpr int NT = EPB * ipow(N + 1, Ph::DIM);
  __shared__ StagesLds<Ph, N, NT> L;
  alw_body<Ph, N, EPB, NT>(kp, L, un_g, rvol_g, d_alpha_out, xcd_block(blockIdx.x, gridDim.x));
}

// ------------------------------------------------------------------------
// Stage kernel of the 2-D systems with two lanes per solution point.  The lane
// of direction d evaluates the d-flux f_d, its derivative D_d, the derivatives
// of the non-conservative columns along d and B_d(u) D_d u, i.e. the d-part
// L_d of the local operator; the two lanes of a point swap halves so that each
// forms L = L_x + L_y for its half of the variables (direction 0 the first
// ceil(M/2), direction 1 the rest) and keeps the running stage sums, U and R of
// that half, and both rebuild the full stage state from their halves.  Same
// arithmetic as the one-lane body, about half the registers per lane.
//
// Lane t of the workgroup takes direction (t >> 5) & 1 and point slot
// 32 (t >> 6) + (t & 31): each half-wave reads along a single direction, which
// keeps the derivative reads free of LDS bank conflicts, and partners sit in
// the two halves of one wave, where v_permlane32_swap exchanges them without
// LDS.
// v_permlane32_swap exchanges the upper half-wave of its first operand with
// the lower half-wave of its second.  Each lane passes (a, b); afterwards the
// lane holds (a of the lower-half lane, b of the upper-half lane) of its pair:
// with a the value for the first half of the variables and b for the second,
// every lane ends with the first-half value from direction 0 and the
// second-half value from direction 1, without selects.
__device__ inline void cross_pair(double& a, double& b) {
  const unsigned long long ba = (unsigned long long)__double_as_longlong(a);
  const unsigned long long bb = (unsigned long long)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned int)(ba & 0xffffffffULL),
                                                   (unsigned int)(bb & 0xffffffffULL), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned int)(ba >> 32), (unsigned int)(bb >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// threads of a two-lane stage workgroup holding EPB elements of P points: whole
// waves
constexpr int stages2_threads(int EPB, int P) { return (2 * EPB * P + 63) / 64 * 64; }

template <class Ph, int N, int NT>
struct Stages2Lds {
  static constexpr int M = Ph::M, P = ipow(N + 1, 2), EL = (NT / 2 + P - 1) / P, NCD = Ph::NCD;
  // stages: f_x, f_y, the non-conservative columns; end: F_x, F_y, U, u^n.
  // Field f of element slot le at s_buf[le][f * P + point]; the slot stride ES
  // is padded to ES = P (mod 32) so that the point slots of a half-wave, which
  // run over into the next element, stay consecutive in bank order
  static constexpr int NBUF = (2 * M + 2 * NCD) > (4 * M) ? (2 * M + 2 * NCD) : (4 * M);
  static constexpr int ES = NBUF * P + (((P - NBUF * P) % 32) + 32) % 32;
  double s_buf[EL][ES];
};

// outputs of the two-lane stage kernels: the face traces of F (lane's
// direction) and U, the volume residual (lane's half of the variables,
// with the element-local correction terms as in stage_outputs) and the
// element's blending coefficient.  Fa holds the lane's direction for all
// variables; Ua, Ra and uo the lane's half.
template <class Ph, int N, int NT>
__device__ __forceinline__ void stages2_tail(const KParams& kp, Stages2Lds<Ph, N, NT>& L, int le, int p, int d, int e,
                                             bool act, const double* Fa, const double* Ua, const double* Ra,
                                             const double* uo, double* __restrict__ rvol_g, double* d_alpha_out) {
  constexpr int n1 = N + 1, M = Ph::M, P = n1 * n1, NFP = n1, NCD = Ph::NCD;
  constexpr int H0 = (M + 1) / 2, H1 = M - H0;
  constexpr int NFT = 4 * NFP;  // face points of the element
  static_assert(NFT <= 2 * P && NFT * M <= 2 * M * P, "one face point per lane; LDS room for the offsets");
  const int vo = d ? H0 : 0;
  auto& s_buf = L.s_buf;
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  // time-averaged flux (lane's direction), solution and u^n (lane's half) to LDS
#pragma unroll
  for (int v = 0; v < M; ++v) s_buf[le][(d * M + v) * P + (p)] = Fa[v];
#pragma unroll
  for (int k = 0; k < H0; ++k)
    if (k < (d ? H1 : H0)) {
      s_buf[le][(2 * M + vo + k) * P + (p)] = Ua[k];
      s_buf[le][(3 * M + vo + k) * P + (p)] = uo[k];
    }
  elem_sync<2 * (N + 1) * (N + 1)>();

  if constexpr (NFT <= P) {
    // face traces, one face point per point slot: both lanes of the slot work
    // on it, each on its half of the variables of every trace, and swap halves
    // where the correction offset C = F_tr + B_d(u^n_tr) U_tr needs the whole
    // state.  Slots past the face points work on face point 0 and store nothing
    // (the swaps take every lane of the wave)
    const int f = p < NFT ? p : 0;
    const bool own = act && p < NFT;
    const int dd = f / (2 * NFP);
    const int rem = f - dd * 2 * NFP;
    const int side = rem / NFP;
    const int qq = rem - side * NFP;
    const double* V = side ? kp.VR : kp.VL;
    const size_t nf = (size_t)kp.E * NFP;
    const size_t fo = (size_t)e * NFP + qq;
    const int nh = d ? H1 : H0;
    auto trace = [&](int field, int v) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) {
        const int nd = dd == 0 ? node_at<n1>(0, qq, r) : node_at<n1>(1, qq, r);
        t += V[r] * s_buf[le][(field + v) * P + (nd)];
      }
      return t;
    };
    // the lane's half of each trace (the upper lane, with one variable fewer,
    // repeats its first), all reads of a field issued together
    double ah[H0], Uh[H0], Fh[H0];
#pragma unroll
    for (int k = 0; k < H0; ++k) ah[k] = trace(3 * M, vo + (k < nh ? k : 0));
#pragma unroll
    for (int k = 0; k < H0; ++k) Uh[k] = trace(2 * M, vo + (k < nh ? k : 0));
    // u^n and U from both halves: u^n whole, U in the entries the product takes
    double a[M], U[M];
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      double x = ah[k], y = ah[k];
      cross_pair(x, y);
      a[k] = x;
      if (k < H1) a[H0 + k] = y;
      U[k] = Uh[k];  // the lower lane's half; unused where the upper lane holds it
    }
#pragma unroll
    for (int k = 0; k < H1; ++k) {
      double x = Uh[k], y = Uh[k];
      cross_pair(x, y);
      U[H0 + k] = y;
    }
#pragma unroll
    for (int k = 0; k < H0; ++k) Fh[k] = trace(dd * M, vo + (k < nh ? k : 0));
    // B_dd(u^n_tr) U_tr from the columns of U that the product takes (indices
    // known at compile time, one select each)
    double wc[NCD], t[M];
#pragma unroll
    for (int c = 0; c < NCD; ++c) wc[c] = dd ? U[Ph::nc_comp(1, c)] : U[Ph::nc_comp(0, c)];
    Ph::ncprod_rd(a, wc, dd, t, pp);
    double Ch[H0];
#pragma unroll
    for (int k = 0; k < H0; ++k) Ch[k] = Fh[k] + (d ? (k < H1 ? t[H0 + k] : 0.0) : t[k]);
    if (own) {
      // F_d components that follow from U (TraceAlias) are not stored
      double* ut = kp.Utr + ((size_t)(dd * 2 + side) * M + vo) * nf + fo;
      double* ft = kp.Ftr + ((size_t)(dd * 2 + side) * M + vo) * nf + fo;
#pragma unroll
      for (int k = 0; k < H1; ++k) {
        ut[k * nf] = Uh[k];
        if (TraceAlias<Ph>::src(dd, vo + k) < 0) ft[k * nf] = Fh[k];
      }
      if (nh > H1) {
        ut[H1 * nf] = Uh[H1];
        if (TraceAlias<Ph>::src(dd, vo + H1) < 0) ft[H1 * nf] = Fh[H1];
      }
    }
    elem_sync<2 * (N + 1) * (N + 1)>();  // every read of the F, U and u^n fields is done
    if (own) {
#pragma unroll
      for (int k = 0; k < H0; ++k)
        if (k < nh) s_buf[le][f * M + vo + k] = Ch[k];
    }
    elem_sync<2 * (N + 1) * (N + 1)>();
  } else {
  // face traces, one face point (all variables) per lane, and the correction
  // offsets C = F_tr + B_d(u^n_tr) U_tr of those face points
  const int tl = 2 * p + d;
  const bool own = act && tl < NFT;
  double C[M];
  if (own) {
    const int dd = tl / (2 * NFP);
    const int rem = tl - dd * 2 * NFP;
    const int side = rem / NFP;
    const int qq = rem - side * NFP;
    const double* V = side ? kp.VR : kp.VL;
    const size_t nf = (size_t)kp.E * NFP;
    const size_t fo = (size_t)e * NFP + qq;
    // three passes (u^n, U, then F), each fenced from the next, so that few
    // LDS values are in flight at once
    auto trace = [&](int field, int v) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) {
        const int nd = dd == 0 ? node_at<n1>(0, qq, r) : node_at<n1>(1, qq, r);
        t += V[r] * s_buf[le][(field + v) * P + (nd)];
      }
      return t;
    };
    double a[M], U[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      a[v] = trace(3 * M, v);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      U[v] = trace(2 * M, v);
      kp.Utr[((size_t)(dd * 2 + side) * M + v) * nf + fo] = U[v];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < M; ++v) C[v] = 0.0;
    if (dd == 0) correction_offset<Ph, 0>(a, U, C, pp);
    else correction_offset<Ph, 1>(a, U, C, pp);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const double tf = trace(dd * M, v);
      if (TraceAlias<Ph>::src(dd, v) < 0) kp.Ftr[((size_t)(dd * 2 + side) * M + v) * nf + fo] = tf;
      C[v] = tf + C[v];
    }
  }
  elem_sync<2 * (N + 1) * (N + 1)>();  // every read of the F, U and u^n fields is done
  if (own) {
#pragma unroll
    for (int v = 0; v < M; ++v) s_buf[le][tl * M + v] = C[v];
  }
  elem_sync<2 * (N + 1) * (N + 1)>();
  }
  if (act) {
    const int i = p % n1, j = p / n1;
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      if (k >= (d ? H1 : H0)) continue;
      const int v = vo + k;
      double R = Ra[k];
#pragma unroll
      for (int dd = 0; dd < 2; ++dd) {
        const int q = dd == 0 ? j : i, ii = dd == 0 ? i : j;
        const int wR = dd * 2 * NFP + NFP + q, wL = dd * 2 * NFP + q;
        R -= (s_buf[le][wR * M + v] * kp.gR[ii] + s_buf[le][wL * M + v] * kp.gL[ii]) * kp.inv_dx[dd];
      }
      rvol_g[((size_t)v * kp.E + e) * P + p] = R;
    }
    // blending coefficient of the element (smoothed over face neighbours)
    if (p == 0 && d == 0) {
      double a;
      if (kp.alpha_force >= 0.0) a = kp.alpha_force;
      else if (kp.blending == 0) a = 0.0;
      else {
        a = kp.alpha_raw[e];
#pragma unroll
        for (int dn = 0; dn < 2; ++dn)
#pragma unroll
          for (int sd = 0; sd < 2; ++sd) a = fmax(a, 0.5 * kp.alpha_raw[alpha_nbr(kp, e, dn, sd)]);
      }
      kp.alpha[e] = a;
      if (d_alpha_out) d_alpha_out[e] = a;
    }
  }
}

template <class Ph, int N, int EPB, int NT, bool OT = false>
__device__ __forceinline__ void stages2_body(const KParams& kp, Stages2Lds<Ph, N, NT>& L,
                                             const double* __restrict__ un_g, double* __restrict__ rvol_g,
                                             double* d_alpha_out, int blk) {
  static_assert(Ph::DIM == 2 && Ph::NCD > 0, "two-lane stage body is for 2-D systems");
  constexpr int n1 = N + 1, M = Ph::M, P = n1 * n1, NFP = n1, NCD = Ph::NCD;
  constexpr int H0 = (M + 1) / 2, H1 = M - H0;
  using Tab = Tableau<N>;
  constexpr int S = Tab::S;
  auto& s_buf = L.s_buf;

  const int tid = body_tid<OT>();
  const int d = (tid >> 5) & 1, np = ((tid >> 6) << 5) | (tid & 31);
  const int le = np / P, p = np - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  const int i = p % n1, j = p / n1;
  const int q = d ? i : j;            // line of the lane's direction through p
  const int ii = d ? j : i;           // position along that line
  // exchange slots of the stage loop: the direction-1 lanes write their values
  // transposed (point (i, j) at i*n1 + j), so that every lane reads its line at
  // q*n1 + r with the offsets along the line known at compile time (paired LDS
  // reads, no per-read address arithmetic)
  const int pw = d ? i * n1 + j : p;
  constexpr int sq = n1, sr = 1;
  const int vo = d ? H0 : 0;          // first variable of the lane's half
  const double dt = kp.scal[0];
  const double idx = d ? kp.inv_dx[1] : kp.inv_dx[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);

  // u^n of the lane's half (lane 1 with H1 < H0 pads with its last variable)
  double uo[H0];
#pragma unroll
  for (int k = 0; k < H0; ++k) {
    const int v = vo + (k < (d ? H1 : H0) ? k : 0);
    uo[k] = un_g[((size_t)v * kp.E + (act ? e : 0)) * P + p];
  }
  double Drow[n1];
#pragma unroll
  for (int r = 0; r < n1; ++r) Drow[r] = kp.D[ii][r];

  double Fa[M], Ua[H0], Ra[H0], Sp[S][H0];
#pragma unroll
  for (int v = 0; v < M; ++v) Fa[v] = 0.0;
#pragma unroll
  for (int k = 0; k < H0; ++k) { Ua[k] = 0.0; Ra[k] = 0.0; }

#pragma unroll
  for (int st = 0; st < S; ++st) {
    // the lane's half of the stage state, then the full state
    double uh[H0], u[M];
#pragma unroll
    for (int k = 0; k < H0; ++k) uh[k] = first_nz<N>(st) >= 0 ? uo[k] - dt * Sp[st][k] : uo[k];
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      // direction 0 holds the first half, direction 1 the second
      double a = uh[k], b = uh[k];
      cross_pair(a, b);
      u[k] = a;
      if (k < H1) u[H0 + k] = b;
    }
    double f[M];
    Ph::flux_rd(u, d, f, pp);
    // the flux components whose derivative is c_h times that of a
    // non-conservative column are not exchanged: f_d[8] = c_h B_d, and of the
    // pair (PA, PA+1) = (5, 6) the lane's f_d[5+d] = c_h psi; slot PA holds the
    // other member of the pair (f[6] for direction 0, f[5] for direction 1)
    constexpr bool PAIR = true;
    constexpr int PA = PAIR ? Ph::flux_pair_nc_alias : -2;
#pragma unroll
    for (int v = 0; v < M; ++v)
      if (Ph::flux_nc_alias(v) < 0 && v != PA && v != PA + 1) s_buf[le][(d * M + v) * P + pw] = f[v];
    if constexpr (PAIR) s_buf[le][(d * M + PA) * P + pw] = d ? f[PA] : f[PA + 1];
#pragma unroll
    for (int c = 0; c < NCD; ++c) {
      const double x0 = u[Ph::nc_comp(0, c)], x1 = u[Ph::nc_comp(1, c)];
      s_buf[le][(2 * M + d * NCD + c) * P + pw] = d ? x1 : x0;
    }
    const double bs = Tab::b(st);
    if (bs != 0.0) {
#pragma unroll
      for (int v = 0; v < M; ++v) Fa[v] += bs * f[v];
#pragma unroll
      for (int k = 0; k < H0; ++k) Ua[k] += bs * uh[k];
    }
    elem_sync<2 * (N + 1) * (N + 1)>();
    // L_d = (D_d f_d + B_d(u) D_d u) / dx_d
    double Ld[M];
    {
      double wc[NCD], nc[M];
#pragma unroll
      for (int c = 0; c < NCD; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < n1; ++r) sacc += Drow[r] * s_buf[le][(2 * M + d * NCD + c) * P + (q * sq + r * sr)];
        wc[c] = sacc;
      }
      Ph::ncprod_rd(u, wc, d, nc, pp);
      // D_d of the stored member of the pair, and D_d (c_h psi) = c_h D_d psi
      double spair = 0.0, spsi = 0.0;
      if constexpr (PAIR) {
#pragma unroll
        for (int r = 0; r < n1; ++r) spair += Drow[r] * s_buf[le][(d * M + PA) * P + (q * sq + r * sr)];
        spsi = pp.ch * wc[1];
      }
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double sacc = 0.0;
        if (Ph::flux_nc_alias(v) >= 0) {
          sacc = pp.ch * wc[Ph::flux_nc_alias(v)];  // D_d (c_h w) = c_h D_d w
        } else if (v == PA) {
          sacc = d ? spair : spsi;
        } else if (v == PA + 1) {
          sacc = d ? spsi : spair;
        } else {
#pragma unroll
          for (int r = 0; r < n1; ++r) sacc += Drow[r] * s_buf[le][(d * M + v) * P + (q * sq + r * sr)];
        }
        Ld[v] = (sacc + nc[v]) * idx;
      }
    }
    elem_sync<2 * (N + 1) * (N + 1)>();
    // L = L_x + L_y on the lane's half
    double Lh[H0];
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      // (L_d of variable k, L_d of variable H0 + k) from both directions:
      // afterwards a = L_x and b = L_y of the lane's own variable
      double a = Ld[k], b = k < H1 ? Ld[H0 + k] : 0.0;
      cross_pair(a, b);
      Lh[k] = a + b;
    }
    if (bs != 0.0) {
#pragma unroll
      for (int k = 0; k < H0; ++k) Ra[k] += bs * Lh[k];
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

  stages2_tail<Ph, N, NT>(kp, L, le, p, d, e, act, Fa, Ua, Ra, uo, rvol_g, d_alpha_out);
}

// Approximate Lax-Wendroff time averages with two lanes per solution point
// (2-D systems with many variables).  Lane d evaluates f_d and B_d(u) D_d u at
// the Taylor points and takes the derivatives along direction d; it owns half
// of the variables' Taylor coefficients d_t^m u and sums, and the Taylor state
// at each point crosses between the two lanes of a point.
template <class Ph, int N, int EPB, int NT>
__device__ __forceinline__ void alw2_body(const KParams& kp, Stages2Lds<Ph, N, NT>& L, const double* __restrict__ un_g,
                                          double* __restrict__ rvol_g, double* d_alpha_out, int blk) {
  static_assert(Ph::DIM == 2 && Ph::NCD > 0, "two-lane body is for 2-D systems");
  constexpr int n1 = N + 1, M = Ph::M, P = n1 * n1, NCD = Ph::NCD;
  constexpr int H0 = (M + 1) / 2, H1 = M - H0;
  constexpr int J = N <= 2 ? 1 : 2;
  auto& s_buf = L.s_buf;
  const int tid = threadIdx.x;
  const int d = (tid >> 5) & 1, np = ((tid >> 6) << 5) | (tid & 31);
  const int le = np / P, p = np - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  const int i = p % n1, j = p / n1;
  const int q = d ? i : j, ii = d ? j : i;
  const int pw = d ? i * n1 + j : p;  // exchange slot, transposed for direction 1
  const int vo = d ? H0 : 0, nown = d ? H1 : H0;
  const double dt = kp.scal[0];
  const double idx = d ? kp.inv_dx[1] : kp.inv_dx[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);

  double c[N + 1][H0];  // d_t^m u at this node, the lane's half
#pragma unroll
  for (int k = 0; k < H0; ++k) {
    const int v = vo + (k < nown ? k : 0);
    c[0][k] = un_g[((size_t)v * kp.E + (act ? e : 0)) * P + p];
  }
  double Drow[n1];
#pragma unroll
  for (int r = 0; r < n1; ++r) Drow[r] = kp.D[ii][r];
  // the full state at the point from the two lanes' halves
  auto full = [&](const double* h, double* u) {
#pragma unroll
    for (int k = 0; k < H0; ++k) {
      double a = h[k], b = h[k];
      cross_pair(a, b);
      u[k] = a;
      if (k < H1) u[H0 + k] = b;
    }
  };
  double Dc[N + 1][NCD];  // D_d (d_t^m u) / dx_d of the components B_d reads
  auto nc_derivs = [&](int m) {
    double u[M];
    full(c[m], u);
#pragma unroll
    for (int cc = 0; cc < NCD; ++cc) {
      const double x0 = u[Ph::nc_comp(0, cc)], x1 = u[Ph::nc_comp(1, cc)];
      s_buf[le][(2 * M + d * NCD + cc) * P + pw] = d ? x1 : x0;
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < NCD; ++cc) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) acc += Drow[r] * s_buf[le][(2 * M + d * NCD + cc) * P + q * n1 + r];
      Dc[m][cc] = acc * idx;
    }
    __syncthreads();
  };
  nc_derivs(0);

  double Fa[M], Ua[H0], Ra[H0];
#pragma unroll
  for (int v = 0; v < M; ++v) Fa[v] = 0.0;
#pragma unroll
  for (int k = 0; k < H0; ++k) { Ua[k] = 0.0; Ra[k] = 0.0; }
  double fact = 1.0, dtk = 1.0;  // (k+1)!, dt^k
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    fact *= (k + 1);
    const double ifact = 1.0 / fact;  // constants after unrolling: no division left
    double fk[M], hk[M];  // dt^k d_t^k of f_d and of B_d(u) D_d u (lane's direction)
#pragma unroll
    for (int v = 0; v < M; ++v) { fk[v] = 0.0; hk[v] = 0.0; }
#pragma unroll
    for (int jj = -J; jj <= J; ++jj) {
      const double wj = alw_weight(N, k, jj);
      if (wj == 0.0) continue;
      double tm[N + 1];
      tm[0] = 1.0;
#pragma unroll
      for (int m = 1; m <= k; ++m) tm[m] = tm[m - 1] * (jj * dt) * (1.0 / m);
      double sh[H0], st[M];
#pragma unroll
      for (int kk = 0; kk < H0; ++kk) {
        double a = c[0][kk];
#pragma unroll
        for (int m = 1; m <= k; ++m) a += tm[m] * c[m][kk];
        sh[kk] = a;
      }
      full(sh, st);
      double f[M];
      Ph::flux_rd(st, d, f, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) fk[v] += wj * f[v];
      double wc[NCD], nc[M];
#pragma unroll
      for (int cc = 0; cc < NCD; ++cc) {
        double a = Dc[0][cc];
#pragma unroll
        for (int m = 1; m <= k; ++m) a += tm[m] * Dc[m][cc];
        wc[cc] = a;
      }
      Ph::ncprod_rd(st, wc, d, nc, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) hk[v] += wj * nc[v];
    }
    // r_d = D_d fk / dx_d + hk through LDS, then the lane's half of r_x + r_y
#pragma unroll
    for (int v = 0; v < M; ++v) s_buf[le][(d * M + v) * P + pw] = fk[v];
    __syncthreads();
    double rd[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) acc += Drow[r] * s_buf[le][(d * M + v) * P + q * n1 + r];
      rd[v] = hk[v] + acc * idx;
    }
    __syncthreads();
    double rh[H0];
#pragma unroll
    for (int kk = 0; kk < H0; ++kk) {
      double a = rd[kk], b = kk < H1 ? rd[H0 + kk] : 0.0;
      cross_pair(a, b);
      rh[kk] = a + b;
    }
    const double uw = dtk * ifact;
#pragma unroll
    for (int kk = 0; kk < H0; ++kk) {
      Ua[kk] += uw * c[k][kk];
      Ra[kk] += rh[kk] * ifact;
    }
#pragma unroll
    for (int v = 0; v < M; ++v) Fa[v] += fk[v] * ifact;
    if (k < N) {
      const double idtk = -1.0 / dtk;
#pragma unroll
      for (int kk = 0; kk < H0; ++kk) c[k + 1][kk] = rh[kk] * idtk;
      nc_derivs(k + 1);
      dtk *= dt;
    }
  }
  stages2_tail<Ph, N, NT>(kp, L, le, p, d, e, act, Fa, Ua, Ra, c[0], rvol_g, d_alpha_out);
}

// two waves per SIMD: at N = 4 GLM-MHD then spills about 30 VGPRs, and still
// runs faster than with one wave
#ifndef ALW2_WAVES_PER_EU
#define ALW2_WAVES_PER_EU 2
#endif
template <class Ph, int N, int EPB>
__global__ void __launch_bounds__(stages2_threads(EPB, ipow(N + 1, 2))) __attribute__((amdgpu_waves_per_eu(ALW2_WAVES_PER_EU)))
    k_stages_alw2(const KParams kp, const double* __restrict__ un_g, double* __restrict__ rvol_g, double* d_alpha_out) {
  constexpr int NT = stages2_threads(EPB, ipow(N + 1, 2));
  __shared__ Stages2Lds<Ph, N, NT> L;
  alw2_body<Ph, N, EPB, NT>(kp, L, un_g, rvol_g, d_alpha_out, xcd_block(blockIdx.x, gridDim.x));
}

// lanes per solution point of the stage kernel: two for the 2-D systems with
// many variables (register bound with one lane), one otherwise (the 2-D
// shallow water system already runs at high occupancy with one lane)
template <class Ph>
constexpr int stage_lanes() {
  return Ph::DIM == 2 && Ph::M >= 8 ? 2 : 1;
}
template <class Ph, int N, int NT>
using StageLdsT = typename std::conditional<stage_lanes<Ph>() == 2, Stages2Lds<Ph, N, NT>, StagesLds<Ph, N, NT>>::type;

template <class Ph, int N, int EPB, int NT, class Tab = Tableau<N>, bool OT = false>
__device__ __forceinline__ void stage_body(const KParams& kp, StageLdsT<Ph, N, NT>& L, const double* __restrict__ un_g,
                                           double* __restrict__ rvol_g, double* d_alpha_out, int blk) {
  static_assert(stage_lanes<Ph>() == 1 || std::is_same<Tab, Tableau<N>>::value, "IMEX pairs use the one-lane kernel");
  if constexpr (stage_lanes<Ph>() == 2) stages2_body<Ph, N, EPB, NT, OT>(kp, L, un_g, rvol_g, d_alpha_out, blk);
  else stages_body<Ph, N, EPB, NT, Tab, OT>(kp, L, un_g, rvol_g, d_alpha_out, blk);
}

// threads of a stage workgroup of EPB elements
template <class Ph, int N, int EPB>
constexpr int stage_threads() {
  return stage_lanes<Ph>() == 2 ? stages2_threads(EPB, ipow(N + 1, Ph::DIM)) : EPB * ipow(N + 1, Ph::DIM);
}

// at least three waves per SIMD for the two-lane stage kernels (at N = 4 the
// compiler would otherwise keep more of a stage's line reads in flight and run
// two); the one-lane kernels take no hint (under three they would spill)
template <class Ph>
constexpr int stage_waves_hint() { return stage_lanes<Ph>() == 2 ? 3 : STAGES_WAVES_PER_EU; }

template <class Ph, int N, int EPB, class Tab = Tableau<N>>
__global__ void __launch_bounds__((stage_threads<Ph, N, EPB>())) __attribute__((amdgpu_waves_per_eu(stage_waves_hint<Ph>())))
    k_stages(const KParams kp, const double* __restrict__ un_g, double* __restrict__ rvol_g, double* d_alpha_out) {
  constexpr int NT = stage_threads<Ph, N, EPB>();
  __shared__ StageLdsT<Ph, N, NT> L;
  stage_body<Ph, N, EPB, NT, Tab>(kp, L, un_g, rvol_g, d_alpha_out, xcd_block(blockIdx.x, gridDim.x));
}

// ------------------------------------------------------------------------
// lower order fluxes f^{num,-}, f^{num,+}(uL, uR) of eq. combined.num.flux
// The same with the fluxes fL = f_d(uL), fR = f_d(uR) and wave speeds sl, sr of
// the two states given (a state shared by two subfaces is evaluated once).
template <class Ph, int d>
__device__ inline void low_flux_given(const double* uL, const double* uR, const double* fL, const double* fR,
                                      double sl, double sr, double* fm, double* fp, const PhysParams& pp) {
  constexpr int M = Ph::M;
  double fc[M], t[M];
  const double lam = sl >= sr ? sl : sr;
#pragma unroll
  for (int v = 0; v < M; ++v) fc[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]);
#pragma unroll
  for (int v = 0; v < M; ++v) t[v] = 0.5 * (uL[v] + uR[v]);  // average state
  if (fm) {
    double b[M];
    Ph::template ncprod<d>(uL, t, b, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) fm[v] = fc[v] + b[v];
  }
  if (fp) {
    double b[M];
    Ph::template ncprod<d>(uR, t, b, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) fp[v] = fc[v] + b[v];
  }
}

template <class Ph, int d>
__device__ inline void low_flux(const double* uL, const double* uR, double* fm, double* fp, const PhysParams& pp) {
  // few live arrays: the central part is formed in fc, then the two
  // non-conservative parts are added one after the other
  constexpr int M = Ph::M;
  double fc[M], t[M];
  const double sl = Ph::template sigma<d>(uL, pp), sr = Ph::template sigma<d>(uR, pp);
  const double lam = sl >= sr ? sl : sr;
  Ph::template flux<d>(uL, fc, pp);
  Ph::template flux<d>(uR, t, pp);
#pragma unroll
  for (int v = 0; v < M; ++v) fc[v] = 0.5 * (fc[v] + t[v]) - 0.5 * lam * (uR[v] - uL[v]);
#pragma unroll
  for (int v = 0; v < M; ++v) t[v] = 0.5 * (uL[v] + uR[v]);  // average state
  if (fm) {
    double b[M];
    Ph::template ncprod<d>(uL, t, b, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) fm[v] = fc[v] + b[v];
  }
  if (fp) {
    double b[M];
    Ph::template ncprod<d>(uR, t, b, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) fp[v] = fc[v] + b[v];
  }
}

template <class Ph>
__device__ inline bool admissible(const double* x, const PhysParams& pp) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < Ph::K; ++k) ok = ok && (Ph::constraint(k, x, pp) > 0.0);
  return ok;
}

// u^n along the line of direction d through face point q of element el: its
// trace at the element's face fs (0 left, 1 right), the sum the stage kernel
// forms for its face traces, the node on that face (s) and the next one inward
// (si).  The line lies in the cache lines the face kernel reads for s and si,
// so the trace costs no HBM traffic of its own.
// FS: the face when every lane has the same one (0 or 1), else -1 and the
// lane's face in fs.
template <class Ph, int N, int d, int FS = -1>
__device__ __forceinline__ void line_trace(const KParams& kp, const double* __restrict__ un_g, int el, int q, int fs,
                                           double (&a)[Ph::M], double (&s)[Ph::M], double (&si)[Ph::M]) {
  constexpr int n1 = N + 1, P = ipow(n1, Ph::DIM), M = Ph::M;
  if constexpr (FS >= 0) fs = FS;
  // the line is walked from the face inward (step k at node N - k on a right
  // face, k on a left face), so that the face node and the next one are the
  // first two steps whichever face the lane has
  double w[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    if constexpr (FS >= 0) {
      w[k] = FS ? kp.VR[N - k] : kp.VL[k];
    } else {
      // both weights are loaded, then one is picked per lane (the empty asm
      // keeps the compiler from selecting between the two kernel-argument
      // addresses instead, which would copy the argument block to scratch)
      double wl = kp.VL[k], wr = kp.VR[N - k];
      asm volatile("" : "+v"(wl), "+v"(wr));
      w[k] = fs ? wr : wl;
    }
  }
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const double* x = un_g + ((size_t)v * kp.E + el) * P;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      const double y = x[node_at<n1>(d, q, fs ? N - k : k)];
      t += w[k] * y;
      if (k == 0) s[v] = y;
      if (k == 1) si[v] = y;
    }
    a[v] = t;
  }
}

// one face point of direction d between element e (minus side) and en (plus
// side).  Written so that few values are live at once: the traces die once
// F^num, U^num (and the correction offsets C^± of the systems that do not fold
// them) are formed, and the candidate states of Algorithm 1 are rebuilt for
// each constraint.
template <class Ph, int N, int d>
__device__ inline void face_point(const KParams& kp, const double* __restrict__ un_g, int e, int q, double dt,
                                  const PhysParams& pp) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  const int en = nbr_elem(kp, e, d, 1);
  const size_t nf = (size_t)kp.E * NFP;
  const size_t fiL = (size_t)e * NFP + q, fiR = (size_t)en * NFP + q;
  // trace index of side (0 left face, 1 right face)
  auto tr = [&](int side, int v, size_t fi) { return ((size_t)(d * 2 + side) * M + v) * nf + fi; };
  // u^n at the face from each side's line of nodes, the nodes on the face and
  // the next ones inward (Algorithm 1)
  double sL[M], sR[M], sLi[M], sRi[M];
  double Fm[M], Fp[M], Cm[M], Cp[M];
  {
    double a[M], b[M], UL[M], UR[M];
    line_trace<Ph, N, d, 1>(kp, un_g, e, q, 1, a, sL, sLi);
    line_trace<Ph, N, d, 0>(kp, un_g, en, q, 0, b, sR, sRi);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      UL[v] = kp.Utr[tr(1, v, fiL)];
      UR[v] = kp.Utr[tr(0, v, fiR)];
      Cm[v] = kp.Ftr[tr(1, v, fiL)];
      Cp[v] = kp.Ftr[tr(0, v, fiR)];
    }
    // wave speed from the face values of u^n; an inadmissible face value uses
    // its neighbouring solution point instead
    // (branches that admissible data never take)
    double sa = Ph::template sigma<d>(a, pp), sb = Ph::template sigma<d>(b, pp);
    if (!admissible<Ph>(a, pp)) sa = Ph::template sigma<d>(sL, pp);
    if (!admissible<Ph>(b, pp)) sb = Ph::template sigma<d>(sR, pp);
    const double lam = sa >= sb ? sa : sb;
    double Unum[M], t[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      Fm[v] = 0.5 * (Cm[v] + Cp[v]) - 0.5 * lam * (UR[v] - UL[v]);  // F^num
      Fp[v] = Fm[v];
      Unum[v] = 0.5 * (UL[v] + UR[v]);
    }
    Ph::template ncprod<d>(a, Unum, t, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) Fm[v] += t[v];
    Ph::template ncprod<d>(b, Unum, t, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) Fp[v] += t[v];
    if constexpr (!fold_correction<Ph>()) {
      // correction offsets C^- = F_tr^- + B(u^{n,-}) U^-, C^+ = F_tr^+ + B(u^{n,+}) U^+
      Ph::template ncprod<d>(a, UL, t, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) Cm[v] += t[v];
      Ph::template ncprod<d>(b, UR, t, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) Cp[v] += t[v];
    }
  }
  const double af = kp.blending == 0 ? 0.0 : 0.5 * (kp.alpha[e] + kp.alpha[en]);
  double Theta = 1.0;
  bool guard = false;
  if (!(af == 0.0 && kp.blending != 2)) {
    // the two face nodes' fluxes and wave speeds serve the face's lower order
    // flux and the inner subface fluxes of Algorithm 1
    double fL[M], fR[M];
    Ph::template flux<d>(sL, fL, pp);
    Ph::template flux<d>(sR, fR, pp);
    const double gL = Ph::template sigma<d>(sL, pp), gR = Ph::template sigma<d>(sR, pp);
    // Algorithm 1 with DIM*dt in the candidate updates of the two subcells
    // next to the face: their inner subface fluxes f^{num,+}(sLi, sL), f^{num,-}(sR, sRi)
    double finL[M], finR[M];
    if (kp.blending == 2 && N >= 1) {
      double f2[M];
      Ph::template flux<d>(sLi, f2, pp);
      low_flux_given<Ph, d>(sLi, sL, f2, fL, Ph::template sigma<d>(sLi, pp), gL, nullptr, finL, pp);
      Ph::template flux<d>(sRi, f2, pp);
      low_flux_given<Ph, d>(sR, sRi, fR, f2, gR, Ph::template sigma<d>(sRi, pp), finR, nullptr, pp);
    }
    double fLOm[M], fLOp[M];
    low_flux_given<Ph, d>(sL, sR, fL, fR, gL, gR, fLOm, fLOp, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      Fm[v] = (1.0 - af) * Fm[v] + af * fLOm[v];
      Fp[v] = (1.0 - af) * Fp[v] + af * fLOp[v];
    }
    if (kp.blending == 2 && N >= 1) {
      const double cN = DIM * dt * kp.inv_wdx[d][N], c0 = DIM * dt * kp.inv_wdx[d][0];
#pragma unroll
      for (int k = 0; k < Ph::K; ++k) {
        double x[M];
#pragma unroll
        for (int v = 0; v < M; ++v) x[v] = sL[v] - cN * (fLOm[v] - finL[v]);
        const double PN = Ph::constraint(k, x, pp);
#pragma unroll
        for (int v = 0; v < M; ++v) x[v] = sR[v] - c0 * (finR[v] - fLOp[v]);
        const double P0 = Ph::constraint(k, x, pp);
#pragma unroll
        for (int v = 0; v < M; ++v) x[v] = sR[v] - c0 * (finR[v] - Fp[v]);
        const double th0 = theta_limit(0.1 * P0, P0, Ph::constraint(k, x, pp), guard);
#pragma unroll
        for (int v = 0; v < M; ++v) x[v] = sL[v] - cN * (Fm[v] - finL[v]);
        const double thN = theta_limit(0.1 * PN, PN, Ph::constraint(k, x, pp), guard);
        const double th = th0 <= thN ? th0 : thN;
        if (th < 1.0) {
#pragma unroll
          for (int v = 0; v < M; ++v) {
            Fm[v] = th * Fm[v] + (1.0 - th) * fLOm[v];
            Fp[v] = th * Fp[v] + (1.0 - th) * fLOp[v];
          }
        }
        Theta *= th;
      }
    }
  }
  // outputs: F^- and F^+, and the correction jumps D^± = F^± - C^± (fold_correction)
  const size_t fo = (size_t)d * nf + fiL;
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const size_t o = ((size_t)d * M + v) * nf + fiL;
    kp.Fm[o] = Fm[v];
    kp.Fp[o] = Fp[v];
    if constexpr (!fold_correction<Ph>()) {
      kp.Dm[o] = Fm[v] - Cm[v];
      kp.Dp[o] = Fp[v] - Cp[v];
    }
  }
  if (kp.theta_face) kp.theta_face[fo] = Theta;
  kp.fflag_face[fo] = face_flag(Theta, guard);
}

template <class Ph, int N>
__device__ __forceinline__ void faces_body(const KParams& kp, const double* __restrict__ un_g, int gid) {
  constexpr int DIM = Ph::DIM, NFP = DIM == 1 ? 1 : N + 1;
  const int nf = kp.E * NFP;
  if (gid >= DIM * nf) return;
  const int d = gid / nf;
  const int fi = gid - d * nf;
  const int e = fi / NFP, q = fi - (fi / NFP) * NFP;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  if (d == 0) face_point<Ph, N, 0>(kp, un_g, e, q, dt, pp);
  else if constexpr (DIM == 2) face_point<Ph, N, 1>(kp, un_g, e, q, dt, pp);
}

// ------------------------------------------------------------------------
// Face kernel of the nine-variable systems with two lanes per face point: the
// lane of the minus side (lower half-wave) holds the traces of element e at its
// right face and the nodes next to it, the lane of the plus side (upper
// half-wave) those of the neighbour at its left face.  Each evaluates its own
// side's wave speed, flux, non-conservative products, lower order flux, subcell
// flux and Algorithm 1 candidate; the values the formulas combine (C, U, the
// node states and fluxes, sigma, theta) cross between the two with
// v_permlane32_swap (cross_pair).  Same arithmetic as face_point, about half
// the registers per lane.  Lane t of a workgroup: side (t >> 5) & 1, face point
// slot 32 (t >> 6) + (t & 31).
template <class Ph>
constexpr int face_lanes() { return Ph::M >= 8 ? 2 : 1; }

// (value on the minus lane, value on the plus lane) of x
__device__ inline void pair_values(double x, double& lo, double& hi) {
  lo = x; hi = x;
  cross_pair(lo, hi);
}

template <class Ph, int N, int d>
__device__ inline void face_point2(const KParams& kp, const double* __restrict__ un_g, int e, int q, int side,
                                   double dt, const PhysParams& pp) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  const int en = nbr_elem(kp, e, d, 1);
  const int eo = side ? en : e;         // the lane's element
  const int ts = side ? 0 : 1;          // its face: left (0) or right (1)
  const size_t nf = (size_t)kp.E * NFP;
  const size_t fio = (size_t)eo * NFP + q;
  auto tr = [&](int v) { return ((size_t)(d * 2 + ts) * M + v) * nf + fio; };
  // u^n at the face from the lane's line of nodes, the node on the face (s)
  // and the next one inward (si, Algorithm 1)
  double s[M], si[M];
  double F[M], C[M];
  {
    double a[M], U[M];
    line_trace<Ph, N, d>(kp, un_g, eo, q, ts, a, s, si);
#pragma unroll
    for (int v = 0; v < M; ++v) U[v] = kp.Utr[tr(v)];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      constexpr int dc = d;
      const int w = TraceAlias<Ph>::src(dc, v);
      C[v] = w < 0 ? kp.Ftr[tr(v)] : (TraceAlias<Ph>::ch_scaled(v) ? pp.ch * U[w < 0 ? 0 : w] : U[w < 0 ? 0 : w]);
    }
    // wave speed at the face value of u^n, or at the node if that is not
    // admissible (a branch that admissible data never take)
    double sg = Ph::template sigma<d>(a, pp);
    if (!admissible<Ph>(a, pp)) sg = Ph::template sigma<d>(s, pp);
    double sa, sb;
    pair_values(sg, sa, sb);
    const double lam = sa >= sb ? sa : sb;
    double Unum[M], t[M];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double cl, ch, ul, uh;
      pair_values(C[v], cl, ch);
      pair_values(U[v], ul, uh);
      F[v] = 0.5 * (cl + ch) - 0.5 * lam * (uh - ul);  // F^num
      Unum[v] = 0.5 * (ul + uh);
    }
    Ph::template ncprod<d>(a, Unum, t, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) F[v] += t[v];
  }
  const double af = kp.blending == 0 ? 0.0 : 0.5 * (kp.alpha[e] + kp.alpha[en]);
  double Theta = 1.0;
  bool guard = false;
  if (!(af == 0.0 && kp.blending != 2)) {
    // the node's flux and wave speed, for the lower order flux at the face and
    // for the inner subface flux of Algorithm 1
    double fs[M];
    Ph::template flux<d>(s, fs, pp);
    const double gs = Ph::template sigma<d>(s, pp);
    // Algorithm 1 works on the lane's subcell next to the face (DIM*dt in its
    // update).  Its inner subface flux (eq. combined.num.flux): on the plus
    // lane f^{e+1,-}_{1/2} = f^{num,-}(s, si), on the minus lane f^{e,+}_{N-1/2}
    // = f^{num,+}(si, s); both take the non-conservative product at s.  Formed
    // first, so that si and its flux die before the face's fluxes are blended
    double fin[M];
    if (kp.blending == 2 && N >= 1) {
      double fi[M], avg[M], t[M];
      Ph::template flux<d>(si, fi, pp);
      const double gi = Ph::template sigma<d>(si, pp);
      const double lam = side ? (gs >= gi ? gs : gi) : (gi >= gs ? gi : gs);
#pragma unroll
      for (int v = 0; v < M; ++v) {
        fin[v] = 0.5 * (fs[v] + fi[v]) - 0.5 * lam * (side ? si[v] - s[v] : s[v] - si[v]);
        avg[v] = 0.5 * (s[v] + si[v]);
      }
      Ph::template ncprod<d>(s, avg, t, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) fin[v] += t[v];
    }
    // lower order flux at the face from the two neighbouring node states
    double fLO[M];
    {
      double sl[M], sh[M], avg[M], t[M];
      double gl, gh;
      pair_values(gs, gl, gh);
      const double lam = gl >= gh ? gl : gh;
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double fl, fh;
        pair_values(fs[v], fl, fh);
        pair_values(s[v], sl[v], sh[v]);
        fLO[v] = 0.5 * (fl + fh) - 0.5 * lam * (sh[v] - sl[v]);
        avg[v] = 0.5 * (sl[v] + sh[v]);
      }
      Ph::template ncprod<d>(s, avg, t, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) fLO[v] += t[v];
    }
#pragma unroll
    for (int v = 0; v < M; ++v) F[v] = (1.0 - af) * F[v] + af * fLO[v];
    if (kp.blending == 2 && N >= 1) {
      const double cs = DIM * dt * kp.inv_wdx[d][side ? 0 : N];
#pragma unroll
      for (int k = 0; k < Ph::K; ++k) {
        double x[M];
#pragma unroll
        for (int v = 0; v < M; ++v) x[v] = s[v] - cs * (side ? fin[v] - fLO[v] : fLO[v] - fin[v]);
        const double Plo = Ph::constraint(k, x, pp);
#pragma unroll
        for (int v = 0; v < M; ++v) x[v] = s[v] - cs * (side ? fin[v] - F[v] : F[v] - fin[v]);
        const double thl = theta_limit(0.1 * Plo, Plo, Ph::constraint(k, x, pp), guard);
        double thN, th0;
        pair_values(thl, thN, th0);
        const double th = th0 <= thN ? th0 : thN;
        if (th < 1.0) {
#pragma unroll
          for (int v = 0; v < M; ++v) F[v] = th * F[v] + (1.0 - th) * fLO[v];
        }
        Theta *= th;
      }
      double gl, gh;
      pair_values(guard ? 1.0 : 0.0, gl, gh);
      guard = (gl != 0.0) || (gh != 0.0);
    }
  }
  // outputs: the minus lane F^-, the plus lane F^+ (slot of the face = e's)
  const size_t fiL = (size_t)e * NFP + q;
  double* Fo = side ? kp.Fp : kp.Fm;
#pragma unroll
  for (int v = 0; v < M; ++v)
    if (v > 0 || !side || !kp.fp0_alias) Fo[((size_t)d * M + v) * nf + fiL] = F[v];
  if (!side) {
    if (kp.theta_face) kp.theta_face[(size_t)d * nf + fiL] = Theta;
    kp.fflag_face[(size_t)d * nf + fiL] = face_flag(Theta, guard);
  }
}

// Face point slot `slot` (of `slots` per workgroup) of workgroup blk, as
// (direction, face point index within the direction).  In 2-D the first half of
// the slots take face points [blk*W, blk*W + W) of direction 0 and the second
// half the same points of direction 1 (W = slots/2): one workgroup reads each
// element's nodes and traces for both directions while they are in cache, and
// every wave keeps one direction.  The grid is the same as for direction-major
// slots.
template <int DIM>
__device__ __forceinline__ void face_slot(int blk, int slot, int slots, int& d, int& fi) {
  if constexpr (DIM == 2) {
    const int W = slots / 2;
    d = slot >= W ? 1 : 0;
    fi = blk * W + slot - d * W;
  } else {
    d = 0;
    fi = blk * slots + slot;
  }
}

template <class Ph, int N>
__device__ __forceinline__ void faces2_body(const KParams& kp, const double* __restrict__ un_g, int blk) {
  constexpr int DIM = Ph::DIM, NFP = DIM == 1 ? 1 : N + 1;
  const int t = threadIdx.x;
  const int side = (t >> 5) & 1;
  const int nf = kp.E * NFP;
  int d, fi;
  face_slot<DIM>(blk, ((t >> 6) << 5) | (t & 31), (int)(blockDim.x / 2), d, fi);
  if (fi >= nf) return;  // both lanes of a face point leave together
  const int e = fi / NFP, q = fi - (fi / NFP) * NFP;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  if (d == 0) face_point2<Ph, N, 0>(kp, un_g, e, q, side, dt, pp);
  else if constexpr (DIM == 2) face_point2<Ph, N, 1>(kp, un_g, e, q, side, dt, pp);
}

#ifndef FACES2_WAVES_PER_EU
#define FACES2_WAVES_PER_EU 1
#endif
template <class Ph, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FACES2_WAVES_PER_EU)))
    k_faces2(const KParams kp, const double* __restrict__ un_g) {
  faces2_body<Ph, N>(kp, un_g, xcd_block(blockIdx.x, gridDim.x));
}

#ifndef FACES_WAVES_PER_EU
#define FACES_WAVES_PER_EU 1
#endif
// at least FACES_WAVES_PER_EU waves per SIMD: the scheduler otherwise hoists
// every load of the 9-variable systems and runs at one wave per SIMD
template <class Ph, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FACES_WAVES_PER_EU)))
    k_faces(const KParams kp, const double* __restrict__ un_g) {
  constexpr int NFP = Ph::DIM == 1 ? 1 : N + 1;
  const int nf = kp.E * NFP;
  int d, fi;
  face_slot<Ph::DIM>(xcd_block(blockIdx.x, gridDim.x), threadIdx.x, (int)blockDim.x, d, fi);
  if (fi >= nf) return;
  faces_body<Ph, N>(kp, un_g, d * nf + fi);
}

// ------------------------------------------------------------------------
// Non-periodic directions.  A boundary face point is two half faces: the right
// side of the last element of a line (ghost state on the plus side) and the
// left side of the first element (ghost on the minus side).  k_faces treats
// the wrap-around face of the line as periodic; k_bfaces runs after it and
// overwrites that face's slot (the slot of the last element): F^- (and D^-),
// theta and guard from the right half face, F^+ (and D^+) from the left half face
// (k_update reads F^+ of an element's left face at the slot of its left
// neighbour, which wraps to the last element), and the left half face's theta
// and guard go to theta_left / guard_left.

// face data of one side: u^n, time-averaged U and F_d at the face, u^n at the
// solution point next to the face (s) and the one after it (si)
template <int M>
struct HalfSide {
  double a[M], U[M], F[M], s[M], si[M];
};

// ghost state outside `in` at side (d, side): outflow copies it; a wall is its
// mirror image (normal momentum reversed; f_d(P u) = -P f_d(u), so every flux
// component but the normal momentum one changes sign); Dirichlet reads u^n, U
// and F_d at boundary position j from kp.ghost.
template <class Ph, int NFP>
__device__ inline void ghost_state(const KParams& kp, int d, int side, int j, const HalfSide<Ph::M>& in,
                                   HalfSide<Ph::M>& g) {
  constexpr int M = Ph::M;
  const int kind = kp.bc[d][side];
  if (kind == 3) {
    const size_t nb0 = (size_t)kp.ny * NFP, nb1 = (size_t)kp.nx * NFP;
    const size_t nb = d == 0 ? nb0 : nb1;
    const size_t off = d == 0 ? (size_t)side * 3 * M * nb0 : 2 * 3 * M * nb0 + (size_t)side * 3 * M * nb1;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      g.a[v] = kp.ghost[off + (size_t)v * nb + j];
      g.U[v] = kp.ghost[off + (size_t)(M + v) * nb + j];
      g.F[v] = kp.ghost[off + (size_t)(2 * M + v) * nb + j];
      g.s[v] = g.a[v];
      g.si[v] = g.a[v];
    }
    return;
  }
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const double sg = (kind == 2 && v == 1 + d) ? -1.0 : 1.0;
    const double sf = kind == 2 ? -sg : 1.0;
    g.a[v] = sg * in.a[v];
    g.U[v] = sg * in.U[v];
    g.s[v] = sg * in.s[v];
    g.si[v] = sg * in.si[v];
    g.F[v] = sf * in.F[v];
  }
}

// blended, limited fluxes F^- and F^+ of one face from its two sides; Algorithm
// 1 keeps only the subcells of the sides marked lim_m / lim_p admissible (a
// ghost side has no subcell of the mesh)
template <class Ph, int d>
__device__ inline void half_face_flux(const KParams& kp, const HalfSide<Ph::M>& mi, const HalfSide<Ph::M>& pl,
                                      double af, bool lim_m, bool lim_p, double dt, int N, const PhysParams& pp,
                                      double* Fm, double* Fp, double& Theta, bool& guard) {
  constexpr int M = Ph::M, DIM = Ph::DIM;
  const double sa = admissible<Ph>(mi.a, pp) ? Ph::template sigma<d>(mi.a, pp) : Ph::template sigma<d>(mi.s, pp);
  const double sb = admissible<Ph>(pl.a, pp) ? Ph::template sigma<d>(pl.a, pp) : Ph::template sigma<d>(pl.s, pp);
  const double lam = sa >= sb ? sa : sb;
  double Unum[M], t[M];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    Fm[v] = 0.5 * (mi.F[v] + pl.F[v]) - 0.5 * lam * (pl.U[v] - mi.U[v]);
    Fp[v] = Fm[v];
    Unum[v] = 0.5 * (mi.U[v] + pl.U[v]);
  }
  Ph::template ncprod<d>(mi.a, Unum, t, pp);
#pragma unroll
  for (int v = 0; v < M; ++v) Fm[v] += t[v];
  Ph::template ncprod<d>(pl.a, Unum, t, pp);
#pragma unroll
  for (int v = 0; v < M; ++v) Fp[v] += t[v];
  double fLOm[M], fLOp[M];
  low_flux<Ph, d>(mi.s, pl.s, fLOm, fLOp, pp);
#pragma unroll
  for (int v = 0; v < M; ++v) {
    Fm[v] = (1.0 - af) * Fm[v] + af * fLOm[v];
    Fp[v] = (1.0 - af) * Fp[v] + af * fLOp[v];
  }
  Theta = 1.0;
  guard = false;
  if (kp.blending != 2) return;
  double finL[M], finR[M];
  low_flux<Ph, d>(mi.si, mi.s, nullptr, finL, pp);
  low_flux<Ph, d>(pl.s, pl.si, finR, nullptr, pp);
  const double cN = DIM * dt * kp.inv_wdx[d][N], c0 = DIM * dt * kp.inv_wdx[d][0];
#pragma unroll
  for (int k = 0; k < Ph::K; ++k) {
    double x[M];
#pragma unroll
    for (int v = 0; v < M; ++v) x[v] = mi.s[v] - cN * (fLOm[v] - finL[v]);
    const double PN = Ph::constraint(k, x, pp);
#pragma unroll
    for (int v = 0; v < M; ++v) x[v] = pl.s[v] - c0 * (finR[v] - fLOp[v]);
    const double P0 = Ph::constraint(k, x, pp);
    double th0 = 1.0, thN = 1.0;
    if (lim_p) {
#pragma unroll
      for (int v = 0; v < M; ++v) x[v] = pl.s[v] - c0 * (finR[v] - Fp[v]);
      th0 = theta_limit(0.1 * P0, P0, Ph::constraint(k, x, pp), guard);
    }
    if (lim_m) {
#pragma unroll
      for (int v = 0; v < M; ++v) x[v] = mi.s[v] - cN * (Fm[v] - finL[v]);
      thN = theta_limit(0.1 * PN, PN, Ph::constraint(k, x, pp), guard);
    }
    const double th = th0 <= thN ? th0 : thN;
    if (th < 1.0) {
#pragma unroll
      for (int v = 0; v < M; ++v) {
        Fm[v] = th * Fm[v] + (1.0 - th) * fLOm[v];
        Fp[v] = th * Fp[v] + (1.0 - th) * fLOp[v];
      }
    }
    Theta *= th;
  }
}

// one half face of direction d: half 0 is the right boundary of the last
// element of line `line`, half 1 the left boundary of its first element
template <class Ph, int N, int d>
__device__ inline void bface_point(const KParams& kp, const double* __restrict__ un_g, int half, int line, int q) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  const int eN = d == 0 ? (kp.nx - 1) + kp.nx * line : line + kp.nx * (kp.ny - 1);
  const int e0 = d == 0 ? kp.nx * line : line;
  const int j = line * NFP + q;
  const size_t nf = (size_t)kp.E * NFP;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  const int ei = half == 0 ? eN : e0;  // the inside element
  const int fs = half == 0 ? 1 : 0;    // its face: right (1) or left (0)
  HalfSide<M> in, gh;
  const size_t fi = (size_t)ei * NFP + q;
#pragma unroll
  for (int v = 0; v < M; ++v) in.U[v] = kp.Utr[((size_t)(d * 2 + fs) * M + v) * nf + fi];
#pragma unroll
  for (int v = 0; v < M; ++v) {
    const int w = TraceAlias<Ph>::src(d, v);  // F_d components that follow from U
    in.F[v] = w < 0 ? kp.Ftr[((size_t)(d * 2 + fs) * M + v) * nf + fi]
                    : (TraceAlias<Ph>::ch_scaled(v) ? pp.ch * in.U[w < 0 ? 0 : w] : in.U[w < 0 ? 0 : w]);
  }
  line_trace<Ph, N, d>(kp, un_g, ei, q, fs, in.a, in.s, in.si);
  ghost_state<Ph, NFP>(kp, d, fs, j, in, gh);
  const double af = kp.blending == 0 ? 0.0 : kp.alpha[ei];
  double Fm[M], Fp[M], Theta;
  bool guard;
  if (half == 0) half_face_flux<Ph, d>(kp, in, gh, af, true, false, dt, N, pp, Fm, Fp, Theta, guard);
  else half_face_flux<Ph, d>(kp, gh, in, af, false, true, dt, N, pp, Fm, Fp, Theta, guard);
  // correction offset of the inside side, F_tr + B(u^n) U at its face (fold_correction)
  double C[M];
  if constexpr (!fold_correction<Ph>()) Ph::template ncprod<d>(in.a, in.U, C, pp);
  const size_t slot = (size_t)eN * NFP + q;
  if (half == 0) {
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const size_t o = ((size_t)d * M + v) * nf + slot;
      kp.Fm[o] = Fm[v];
      if constexpr (!fold_correction<Ph>()) kp.Dm[o] = Fm[v] - (in.F[v] + C[v]);
    }
    if (kp.theta_face) kp.theta_face[(size_t)d * nf + slot] = Theta;
    kp.fflag_face[(size_t)d * nf + slot] = face_flag(Theta, guard);
  } else {
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const size_t o = ((size_t)d * M + v) * nf + slot;
      kp.Fp[o] = Fp[v];
      if constexpr (!fold_correction<Ph>()) kp.Dp[o] = Fp[v] - (in.F[v] + C[v]);
    }
    const size_t bl = (d == 0 ? 0 : (size_t)kp.ny * NFP) + j;
    kp.theta_left[bl] = Theta;
    kp.guard_left[bl] = guard ? 1u : 0u;
  }
}

// thread gid enumerates, per non-periodic direction d, the 2 * lines_d * nfp
// pairs (half, position along the side)
template <class Ph, int N>
__device__ inline void bfaces_body(const KParams& kp, const double* __restrict__ un_g, int gid) {
  constexpr int DIM = Ph::DIM, NFP = DIM == 1 ? 1 : N + 1;
  int d = 0;
  const int cnt0 = kp.bc[0][0] != 0 ? 2 * kp.ny * NFP : 0;
  if (gid >= cnt0) {
    if (DIM == 1 || kp.bc[1][0] == 0) return;
    gid -= cnt0;
    d = 1;
    if (gid >= 2 * kp.nx * NFP) return;
  }
  const int lines = d == 0 ? kp.ny : kp.nx;
  const int half = gid / (lines * NFP);
  const int j = gid - half * lines * NFP;
  const int line = j / NFP, q = j - line * NFP;
  if (d == 0) bface_point<Ph, N, 0>(kp, un_g, half, line, q);
  else if constexpr (DIM == 2) bface_point<Ph, N, 1>(kp, un_g, half, line, q);
}

template <class Ph, int N>
__global__ void __launch_bounds__(64) k_bfaces(const KParams kp, const double* __restrict__ un_g) {
  bfaces_body<Ph, N>(kp, un_g, blockIdx.x * blockDim.x + threadIdx.x);
}

// number of k_bfaces threads of a mesh with side kinds bc
inline int bface_threads(int DIM, int nx, int ny, int NFP, const int bc[2][2]) {
  return (bc[0][0] != 0 ? 2 * ny * NFP : 0) + (DIM == 2 && bc[1][0] != 0 ? 2 * nx * NFP : 0);
}

// ------------------------------------------------------------------------
// k_update: one thread per solution point.  High order update (eq.
// crkfr.non.cons.final: the volume residual from the stage kernel plus the
// correction terms, F^± g'/dx or D^± g'/dx, see fold_correction), subcell FV
// update (eq. low.order.update), blend (eq. blended.scheme) and Algorithm 2.
// io holds R_vol on entry and u^{n+1} on exit.
template <class Ph, int N, int NT>
struct UpdateLds {
  static constexpr int M = Ph::M, P = ipow(N + 1, Ph::DIM), EL = (NT + P - 1) / P;
  double s_u[EL][M][P];
  // f_d at the nodes (one direction at a time).  The node left of a subface is
  // the only reader of its right neighbour's slot, and overwrites it with the
  // subface flux f^{num,+} that the neighbour needs, after reading it; the
  // slots then serve Algorithm 2's reductions
  double s_f[EL][M][P];
  double s_red[EL][P];      // sigma_d at the nodes / reductions
  uint32_t s_fl[EL][P];
};

// KEEP: the final state of the thread's node also goes to us_keep (M values)
template <class Ph, int N, int EPB, int NT, bool OT = false, bool KEEP = false>
__device__ __forceinline__ void update_body(const KParams& kp, UpdateLds<Ph, N, NT>& L,
                                            const double* __restrict__ un_g, double* __restrict__ io,
                                            uint32_t* d_flags, int blk, double* us_keep = nullptr) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, P = ipow(n1, DIM), NFP = DIM == 1 ? 1 : n1;
  auto& s_u = L.s_u;
  auto& s_f = L.s_f;
  auto& s_left = L.s_f;  // f^{num,+} of the subface left of each node (see UpdateLds)
  auto& s_red = L.s_red;
  auto& s_fl = L.s_fl;

  const int tid = body_tid<OT>();
  const int le = tid / P, p = tid - le * P;
  const int e = blk * EPB + le;
  const bool act = le < EPB && e < kp.E;
  const int i = p % n1, j = p / n1;
  const double dt = kp.scal[0];
  const PhysParams pp = phys_params(kp, kp.scal[1]);
  const size_t nf = (size_t)kp.E * NFP;

  // lanes without an element read element 0 (unconditional loads pipeline)
  const int es = act ? e : 0;
  double un[M], R[M];
#pragma unroll
  for (int v = 0; v < M; ++v) un[v] = un_g[((size_t)v * kp.E + es) * P + p];
#pragma unroll
  for (int v = 0; v < M; ++v) R[v] = io[((size_t)v * kp.E + es) * P + p];
#pragma unroll
  for (int v = 0; v < M; ++v) s_u[le][v][p] = un[v];
  int eL[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) eL[d] = nbr_elem(kp, es, d, 0);
  uint32_t fl = 0;
  const double al = kp.alpha[es];
  // Algorithm 1 activity on the element's faces (a theta below 1, or the guard),
  // loaded first so that the loads' latency hides behind the update: the
  // element's threads take face points w = (side, d, q), its right faces, then
  // its left faces, whose slot is the left neighbour's, or a boundary half face
  // (a boundary half face's own values are read at the end, by its threads only)
  constexpr int NFW = 2 * DIM * NFP, NW = (NFW + P - 1) / P;
  uint32_t ffw[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int w = p + k * P < NFW ? p + k * P : 0;  // threads past the face points read point 0
    const int q = w % NFP, d = (w / NFP) % DIM, side = w / (DIM * NFP);
    const int ef = side ? (d == 0 ? eL[0] : eL[DIM - 1]) : es;
    const size_t fo = (size_t)d * nf + (size_t)ef * NFP + q;
    ffw[k] = kp.blending == 2 ? kp.fflag_face[fo] : 0u;
  }
  // high order update
  double uH[M];
  {
    // the correction terms: F^± g'/dx after a folded volume residual, else D^± g'/dx
    const double* cm = fold_correction<Ph>() ? kp.Fm : kp.Dm;
    const double* cp = fold_correction<Ph>() ? kp.Fp : kp.Dp;
    if constexpr (NFW <= P) {
      // each face value of the element is loaded once, by the thread of its
      // face point w (the layout of the flag loads above), and shared through
      // the flux slots, which the subcell update only fills after the barrier
      // that follows
      const int w = p < NFW ? p : 0;
      const int q = w % NFP, d = (w / NFP) % DIM, side = w / (DIM * NFP);
      const double* src = side ? cp : cm;
      const double* src0 = side && !kp.fp0_alias ? cp : cm;
      const size_t fo = (size_t)(side ? (d == 0 ? eL[0] : eL[DIM - 1]) : es) * NFP + q;
      double fw[M];
#pragma unroll
      for (int v = 0; v < M; ++v) fw[v] = (v == 0 ? src0 : src)[((size_t)d * M + v) * nf + fo];
      if (p < NFW) {
#pragma unroll
        for (int v = 0; v < M; ++v) s_f[le][v][p] = fw[v];
      }
      elem_sync<ipow(N + 1, Ph::DIM)>();
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int q = d == 0 ? j : i, ii = d == 0 ? i : j;
        const int wR = d * NFP + q, wL = (DIM + d) * NFP + q;
#pragma unroll
        for (int v = 0; v < M; ++v)
          R[v] += (s_f[le][v][wR] * kp.gR[ii] + s_f[le][v][wL] * kp.gL[ii]) * kp.inv_dx[d];
      }
    } else {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int q = d == 0 ? j : i, ii = d == 0 ? i : j;
        const size_t fR = (size_t)es * NFP + q, fL = (size_t)eL[d] * NFP + q;
#pragma unroll
        for (int v = 0; v < M; ++v) {
          const double fm = cm[((size_t)d * M + v) * nf + fR];
          const double fp = (v == 0 && kp.fp0_alias ? cm : cp)[((size_t)d * M + v) * nf + fL];
          R[v] += (fm * kp.gR[ii] + fp * kp.gL[ii]) * kp.inv_dx[d];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < M; ++v) uH[v] = un[v] - dt * R[v];
  }
  elem_sync<ipow(N + 1, Ph::DIM)>();
  double us[M];
  if (kp.blending == 0) {
#pragma unroll
    for (int v = 0; v < M; ++v) us[v] = uH[v];
  } else {
    // lower order subcell update: per direction, every node evaluates f_d and
    // sigma_d once; the node left of each interior subface forms its two
    // fluxes f^{num,-}, f^{num,+} (eq. combined.num.flux) and passes f^{num,+}
    // to the node on its right
    double RL[M];
#pragma unroll
    for (int v = 0; v < M; ++v) RL[v] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int q = d == 0 ? j : i, ii = d == 0 ? i : j;
      double fo[M];
      double sg;
      if (d == 0) { Ph::template flux<0>(un, fo, pp); sg = Ph::template sigma<0>(un, pp); }
      else { Ph::template flux<(DIM > 1 ? 1 : 0)>(un, fo, pp); sg = Ph::template sigma<(DIM > 1 ? 1 : 0)>(un, pp); }
#pragma unroll
      for (int v = 0; v < M; ++v) s_f[le][v][p] = fo[v];
      s_red[le][p] = sg;
      elem_sync<ipow(N + 1, Ph::DIM)>();
      double right[M];
      if (ii < N) {
        const int pn = node_at<n1>(d, q, ii < N ? ii + 1 : ii);
        double un2[M], avg[M], bL[M], bR[M];
#pragma unroll
        for (int v = 0; v < M; ++v) { un2[v] = s_u[le][v][pn]; avg[v] = 0.5 * (un[v] + un2[v]); }
        const double sr = s_red[le][pn];
        const double lam = sg >= sr ? sg : sr;
        if (d == 0) { Ph::template ncprod<0>(un, avg, bL, pp); Ph::template ncprod<0>(un2, avg, bR, pp); }
        else {
          Ph::template ncprod<(DIM > 1 ? 1 : 0)>(un, avg, bL, pp);
          Ph::template ncprod<(DIM > 1 ? 1 : 0)>(un2, avg, bR, pp);
        }
#pragma unroll
        for (int v = 0; v < M; ++v) {
          const double fc = 0.5 * (fo[v] + s_f[le][v][pn]) - 0.5 * lam * (un2[v] - un[v]);
          right[v] = fc + bL[v];
          s_left[le][v][pn] = fc + bR[v];
        }
      } else {
        const size_t fR = (size_t)es * NFP + q;
#pragma unroll
        for (int v = 0; v < M; ++v) right[v] = kp.Fm[((size_t)d * M + v) * nf + fR];
      }
      elem_sync<ipow(N + 1, Ph::DIM)>();
      double left[M];
      if (ii > 0) {
#pragma unroll
        for (int v = 0; v < M; ++v) left[v] = s_left[le][v][p];
      } else {
        const size_t fL = (size_t)eL[d] * NFP + q;
#pragma unroll
        for (int v = 0; v < M; ++v) left[v] = (v == 0 && kp.fp0_alias ? kp.Fm : kp.Fp)[((size_t)d * M + v) * nf + fL];
      }
#pragma unroll
      for (int v = 0; v < M; ++v) RL[v] += (right[v] - left[v]) * kp.inv_wdx[d][ii];
      elem_sync<ipow(N + 1, Ph::DIM)>();
    }
    double uL[M];
#pragma unroll
    for (int v = 0; v < M; ++v) uL[v] = un[v] - dt * RL[v];
    if constexpr (Ph::SRC) {
      // the source enters the subcell update implicitly (eq. low.order.update)
      double x[M];
      Ph::implicit(uL, dt, x, pp);
#pragma unroll
      for (int v = 0; v < M; ++v) uL[v] = x[v];
    }
#pragma unroll
    for (int v = 0; v < M; ++v) us[v] = (1.0 - al) * uH[v] + al * uL[v];
    // Algorithm 2.  Element minima: every point stores its value, one thread
    // per element reduces, every point reads the result.
    static_assert(2 * Ph::K <= P && Ph::K <= M, "reduction slots");
    double Theta = 1.0;
    double Pa[Ph::K > 0 ? Ph::K : 1], Pmin[Ph::K > 0 ? Ph::K : 1];
    if constexpr (elem_lane_exchange<P>()) {
#pragma unroll
      for (int k = 0; k < Ph::K; ++k) {
        Pa[k] = Ph::constraint(k, uL, pp);
        Pmin[k] = elem_min<P>(Pa[k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < Ph::K; ++k) {
        Pa[k] = Ph::constraint(k, uL, pp);
        s_f[le][k][p] = Pa[k];
      }
      elem_sync<ipow(N + 1, Ph::DIM)>();
      if (p == 0) {
#pragma unroll
        for (int k = 0; k < Ph::K; ++k) {
          double m = s_f[le][k][0];
#pragma unroll
          for (int r = 1; r < P; ++r) m = fmin(m, s_f[le][k][r]);
          s_red[le][k] = m;
        }
      }
      elem_sync<ipow(N + 1, Ph::DIM)>();
#pragma unroll
      for (int k = 0; k < Ph::K; ++k) Pmin[k] = s_red[le][k];
    }
#pragma unroll
    for (int k = 0; k < Ph::K; ++k)
      if (Pmin[k] <= 0.0) fl |= 2u;
    if (kp.blending == 2) {
#pragma unroll
      for (int k = 0; k < Ph::K; ++k) {
        bool guard = false;
        const double th_p = theta_limit(0.1 * Pmin[k], Pa[k], Ph::constraint(k, us, pp), guard);
        double th;
        if constexpr (elem_lane_exchange<P>()) {
          th = elem_min<P>(th_p);
        } else {
          elem_sync<ipow(N + 1, Ph::DIM)>();  // every point has read the previous minimum
          s_left[le][0][p] = th_p;
          elem_sync<ipow(N + 1, Ph::DIM)>();
          if (p == 0) {
            double m = s_left[le][0][0];
#pragma unroll
            for (int r = 1; r < P; ++r) m = fmin(m, s_left[le][0][r]);
            s_red[le][Ph::K + k] = m;
          }
          elem_sync<ipow(N + 1, Ph::DIM)>();
          th = s_red[le][Ph::K + k];
        }
        if (th < 1.0) {
#pragma unroll
          for (int v = 0; v < M; ++v) us[v] = th * us[v] + (1.0 - th) * uL[v];
        }
        Theta *= th;
      }
    }
    if (Theta < 1.0) fl |= 1u;
    if (act && p == 0) kp.theta_elem[e] = Theta;
  }
  bool finite = true;
#pragma unroll
  for (int v = 0; v < M; ++v) finite = finite && isfinite(us[v]);
  if (!finite) fl |= 8u;
  if (act) {
#pragma unroll
    for (int v = 0; v < M; ++v) io[((size_t)v * kp.E + e) * P + p] = us[v];
  }
  if constexpr (KEEP) {
#pragma unroll
    for (int v = 0; v < M; ++v) us_keep[v] = us[v];
  }
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int w = p + k * P;
    if (w >= NFW) continue;
    const int q = w % NFP, d = (w / NFP) % DIM, side = w / (DIM * NFP);
    if (kp.blending == 2 && side && on_boundary(kp, es, d, 0)) {  // a boundary half face
      const size_t bl = (d == 0 ? 0 : (size_t)kp.ny * NFP) + (size_t)(d == 0 ? es / kp.nx : es % kp.nx) * NFP + q;
      ffw[k] = face_flag(kp.theta_left[bl], kp.guard_left[bl] != 0u);
    }
    fl |= (ffw[k] & 1u ? 4u : 0u) | (ffw[k] & 2u ? 16u : 0u);
  }
  uint32_t f = 0;
  if constexpr (elem_lane_exchange<P>()) {
    f = elem_or<P>(fl);
  } else {
    s_fl[le][p] = fl;
    elem_sync<ipow(N + 1, Ph::DIM)>();
    if (p == 0) {
#pragma unroll
      for (int r = 0; r < P; ++r) f |= s_fl[le][r];
    }
  }
  if (act && p == 0) {
    if (d_flags) d_flags[e] = f;
    // every flag reaches the context's word; the atomic is skipped once its
    // bits are set (a stale read only costs an extra atomic)
    if (f) {
      const uint32_t seen = __hip_atomic_load(kp.flag_or, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((seen | f) != seen) atomicOr(kp.flag_or, f);
    }
  }
}

#ifndef UPDATE_WAVES_PER_EU
#define UPDATE_WAVES_PER_EU 3
#endif
// at least three waves per SIMD: GLM-MHD at N = 2 otherwise takes 170 VGPRs
// and runs at two
// NEXT: a step of a chain whose next step starts from this one's result (the
// steps of a captured graph): the kernel also forms the next step's element
// data (means, speeds, Lambda_e, raw indicator and the block maxima, exactly
// what k_pre would compute from the state it has written), so that the next
// step needs no k_pre.  Its workgroups are k_pre's.
template <class Ph, int N, int EPB, bool NEXT = false>
__global__ void __launch_bounds__(EPB* ipow(N + 1, Ph::DIM)) __attribute__((amdgpu_waves_per_eu(UPDATE_WAVES_PER_EU)))
    k_update(const KParams kp, const double* __restrict__ un_g, double* __restrict__ io, uint32_t* d_flags) {
  constexpr int NT = EPB * ipow(N + 1, Ph::DIM);
  if constexpr (!NEXT) {
    __shared__ UpdateLds<Ph, N, NT> L;
    update_body<Ph, N, EPB, NT>(kp, L, un_g, io, d_flags, xcd_block(blockIdx.x, gridDim.x));
  } else {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    union Lds {
      UpdateLds<Ph, N, NT> update;
      PreLds<Ph, N, NT> pre;
    };
    __shared__ Lds L;
    double us[Ph::M];
    update_body<Ph, N, EPB, NT, false, true>(kp, L.update, un_g, io, d_flags, b, us);
    __syncthreads();  // the update's LDS is free
    pre_from_state<Ph, N, EPB, NT>(kp, L.pre, us, b, kp.part + b);
  }
}

// ------------------------------------------------------------------------
// k_stats / k_stats_fin: statistics of one step (lwfr_stats).  One thread per
// element forms sum_p w_p |Omega_e| u_{v,e,p}, min_p P_k(u_{e,p}) and counts
// its flags and alpha_e bin; each block reduces its elements (lane exchanges
// in a fixed pattern, then the waves in order) into one row of partials; one
// block reduces the rows in a fixed order.  The bits of the result therefore
// do not depend on scheduling.
// Row layout (doubles): [0, 9) sums per variable, [9, 11) minima, [11, 16)
// counts ALG1, ALG2, LOW_INADM, NONFINITE, ALG1_GUARD, [16, 27) alpha bins.
constexpr int kStatsSums = 9, kStatsMins = 2, kStatsCounts = 5, kStatsBins = 11;
constexpr int kStatsRow = kStatsSums + kStatsMins + kStatsCounts + kStatsBins;
constexpr int kStatsMin0 = kStatsSums, kStatsCnt0 = kStatsMin0 + kStatsMins, kStatsBin0 = kStatsCnt0 + kStatsCounts;

__device__ inline double wave_reduce_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
// alpha bin: 0 for alpha = 0, k for alpha in ((k-1)/10, k/10]
__device__ inline int alpha_bin(double a) {
  if (!(a > 0.0)) return 0;
  int k = (int)ceil(a * 10.0);
  return k < 1 ? 1 : (k > 10 ? 10 : k);
}

template <class Ph, int N>
__global__ void __launch_bounds__(256) k_stats(const KParams kp, const double* __restrict__ u,
                                               const uint32_t* __restrict__ eflags, double* __restrict__ rows) {
  constexpr int n1 = N + 1, DIM = Ph::DIM, M = Ph::M, K = Ph::K, P = ipow(n1, DIM);
  static_assert(M <= kStatsSums && K <= kStatsMins, "stats row");
  __shared__ double s_w[kStatsRow][4];
  const int e = blockIdx.x * 256 + threadIdx.x;
  const bool act = e < kp.E;
  const PhysParams pp = phys_params(kp, 0.0);
  double val[kStatsRow];
#pragma unroll
  for (int i = 0; i < kStatsRow; ++i) val[i] = 0.0;
  val[kStatsMin0] = val[kStatsMin0 + 1] = INFINITY;
  if (act) {
    const double vol = kp.dx[0] * (DIM == 2 ? kp.dx[1] : 1.0);
    for (int p = 0; p < P; ++p) {
      double x[M];
#pragma unroll
      for (int v = 0; v < M; ++v) x[v] = u[((size_t)v * kp.E + e) * P + p];
      const double wp = DIM == 1 ? kp.w[p] : kp.w[p % n1] * kp.w[p / n1];
#pragma unroll
      for (int v = 0; v < M; ++v) val[v] += wp * x[v];
#pragma unroll
      for (int k = 0; k < K; ++k) val[kStatsMin0 + k] = fmin(val[kStatsMin0 + k], Ph::constraint(k, x, pp));
    }
#pragma unroll
    for (int v = 0; v < M; ++v) val[v] *= vol;
    const uint32_t f = eflags[e];
    val[kStatsCnt0 + 0] = (f & 4u) ? 1.0 : 0.0;
    val[kStatsCnt0 + 1] = (f & 1u) ? 1.0 : 0.0;
    val[kStatsCnt0 + 2] = (f & 2u) ? 1.0 : 0.0;
    val[kStatsCnt0 + 3] = (f & 8u) ? 1.0 : 0.0;
    val[kStatsCnt0 + 4] = (f & 16u) ? 1.0 : 0.0;
    val[kStatsBin0 + alpha_bin(kp.alpha[e])] = 1.0;
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kStatsRow; ++i) {
    double r;
    if (i >= kStatsMin0 && i < kStatsCnt0) r = wave_reduce_min(val[i]);
    else r = wave_reduce_sum(val[i]);
    if ((threadIdx.x & 63) == 0) s_w[i][w] = r;
  }
  __syncthreads();
  if (threadIdx.x < kStatsRow) {
    const int i = threadIdx.x;
    double r = s_w[i][0];
    for (int k = 1; k < 4; ++k) r = (i >= kStatsMin0 && i < kStatsCnt0) ? fmin(r, s_w[i][k]) : r + s_w[i][k];
    rows[(size_t)blockIdx.x * kStatsRow + i] = r;
  }
}

template <class Stats>
__global__ void __launch_bounds__(256) k_stats_fin(const KParams kp, const double* __restrict__ rows, int nrows,
                                                   Stats* __restrict__ out) {
  __shared__ double s_w[kStatsRow][4];
  const int w = threadIdx.x >> 6;
  for (int i = 0; i < kStatsRow; ++i) {
    const bool mn = i >= kStatsMin0 && i < kStatsCnt0;
    double r = mn ? INFINITY : 0.0;
    for (int b = threadIdx.x; b < nrows; b += 256) {
      const double x = rows[(size_t)b * kStatsRow + i];
      r = mn ? fmin(r, x) : r + x;
    }
    r = mn ? wave_reduce_min(r) : wave_reduce_sum(r);
    if ((threadIdx.x & 63) == 0) s_w[i][w] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kStatsRow];
    for (int i = 0; i < kStatsRow; ++i) {
      const bool mn = i >= kStatsMin0 && i < kStatsCnt0;
      double r = s_w[i][0];
      for (int k = 1; k < 4; ++k) r = mn ? fmin(r, s_w[i][k]) : r + s_w[i][k];
      t[i] = r;
    }
    Stats st;
    st.dt = kp.scal[0];
    st.ch = kp.scal[1];
    for (int v = 0; v < kStatsSums; ++v) st.mass[v] = t[v];
    for (int k = 0; k < kStatsMins; ++k) st.min_constraint[k] = t[kStatsMin0 + k];
    for (int b = 0; b < kStatsBins; ++b) st.alpha_hist[b] = (uint32_t)t[kStatsBin0 + b];
    st.n_alg1 = (uint32_t)t[kStatsCnt0 + 0];
    st.n_alg2 = (uint32_t)t[kStatsCnt0 + 1];
    st.n_low_inadm = (uint32_t)t[kStatsCnt0 + 2];
    st.n_nonfinite = (uint32_t)t[kStatsCnt0 + 3];
    st.n_alg1_guard = (uint32_t)t[kStatsCnt0 + 4];
    st.reserved = 0;
    *out = st;
  }
}

__global__ void __launch_bounds__(256) k_residual(const double* __restrict__ u, double* __restrict__ R, size_t n,
                                                  const double* __restrict__ scal) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) R[k] = (u[k] - R[k]) / scal[0];
}

}  // namespace lwfr
