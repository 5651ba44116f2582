// C ABI of the time step (declarations and contracts in include/lwfr.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lwfr.h"
#include "adjoint.hpp"
#include "kernels.hpp"

using namespace lwfr;

namespace {

thread_local std::string g_err;

lwfr_status fail(lwfr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct lwfr_ctx {
  lwfr_config cfg;
  int M = 0, DIM = 0, K = 0, N = 0, n1 = 0, P = 0, NFP = 0, E = 0;
  int nblk_pre = 0, nblk_ch = 0;
  RefData rd;
  double cfl = 0.0;
  KParams kp;
  // workspace carving (byte offsets)
  size_t off_scal, off_part, off_part2, off_speeds, off_araw, off_alpha, off_thel, off_Ftr, off_Utr, off_untr,
      off_Fm, off_Fp, off_Dm, off_Dp, off_thf, off_guard, off_flag, ws_bytes;
  // adjoint workspace (only with LWFR_CFG_ADJOINT)
  bool adjoint = false;
  size_t off_uscr, off_grvol, off_gun, off_gFm, off_gFp, off_gDm, off_gDp, off_gFtr, off_gUtr, off_guntr, off_gsL,
      off_gsR;
  AdjParams ap;
  // per-step tape: what the reverse kernels read from a forward step
  size_t tp_scal, tp_alpha, tp_thf, tp_thel, tp_untr, tp_Utr, tape_bytes;
  void* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  // optional per-kernel timing with HIP events on the bound stream
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kernel;  // kernel id of the launch between event 2i and 2i+1
  size_t ev_used = 0;
};

namespace {

struct EqInfo {
  int M, DIM, K;
};

bool eq_info(int eq, EqInfo& info) {
  switch (eq) {
    case LWFR_EQ_SW1D: info = {SW1D::M, SW1D::DIM, SW1D::K}; return true;
    case LWFR_EQ_SW2D: info = {SW2D::M, SW2D::DIM, SW2D::K}; return true;
    case LWFR_EQ_GLMMHD2D: info = {MHD2D::M, MHD2D::DIM, MHD2D::K}; return true;
    case LWFR_EQ_LINADV1D: info = {LinAdv1D::M, LinAdv1D::DIM, LinAdv1D::K}; return true;
    case LWFR_EQ_VARADV1D: info = {VarAdv1D::M, VarAdv1D::DIM, VarAdv1D::K}; return true;
  }
  return false;
}

// Elements per workgroup of the per-point kernels (k_pre, k_stages, k_update).
#ifndef LWFR_EPB_OVERRIDE
#define LWFR_EPB_OVERRIDE 0
#endif
// Default: 256 threads per workgroup; 2-D degree 4 with 9 variables uses 5
// elements (125 threads): measured fastest for the register-bound stage kernel.
template <int N>
constexpr int epb_for(int DIM, int M) {
  return LWFR_EPB_OVERRIDE > 0 ? LWFR_EPB_OVERRIDE : (DIM == 2 && N == 4 && M >= 9) ? 5 : 256 / ipow(N + 1, DIM);
}
inline int epb_runtime(int N, int DIM, int M) {
  switch (N) {
    case 1: return epb_for<1>(DIM, M);
    case 2: return epb_for<2>(DIM, M);
    case 3: return epb_for<3>(DIM, M);
    default: return epb_for<4>(DIM, M);
  }
}

#define LWFR_CHECK_LAUNCH(name)                                                   \
  do {                                                                            \
    hipError_t err_ = hipGetLastError();                                          \
    if (err_ != hipSuccess)                                                       \
      return fail(LWFR_E_HIP, std::string(name) + ": " + hipGetErrorString(err_)); \
  } while (0)

// kernel ids reported by lwfr_timing_end
enum {
  KID_PRE = 0, KID_DT, KID_CH, KID_CHFIN, KID_STAGES, KID_FACES, KID_UPDATE, KID_RESIDUAL,
  KID_ADJ_UPDATE, KID_ADJ_FACES, KID_ADJ_STAGES, KID_COUNT
};

// Records an event before (open) and after (close) a launch when timing is on.
struct TimedLaunch {
  lwfr_ctx* c;
  int kid;
  bool on;
  TimedLaunch(lwfr_ctx* c_, int kid_) : c(c_), kid(kid_), on(false) {
    if (c->timing && c->ev_used + 2 <= c->ev.size()) {
      on = true;
      (void)hipEventRecord(c->ev[c->ev_used], c->stream);
    }
  }
  void close() {
    if (on) {
      (void)hipEventRecord(c->ev[c->ev_used + 1], c->stream);
      c->ev_kernel[c->ev_used / 2] = kid;
      c->ev_used += 2;
      on = false;
    }
  }
};

#define LWFR_LAUNCH(kid, name, ...)          \
  do {                                       \
    TimedLaunch tl_(c, kid);                 \
    hipLaunchKernelGGL(__VA_ARGS__);         \
    tl_.close();                             \
    LWFR_CHECK_LAUNCH(name);                 \
  } while (0)

// The launch sequence of one step for system Ph at degree N.
template <class Ph, int N>
lwfr_status launch_step(lwfr_ctx* c, const KParams& kp, const double* u_in, double* u_out, double* d_dt_ch,
                        double* d_alpha, uint32_t* d_flags) {
  constexpr int DIM = Ph::DIM, P = ipow(N + 1, DIM), NFP = DIM == 1 ? 1 : N + 1;
  constexpr int EPB = epb_for<N>(DIM, Ph::M);
  const int E = c->E;
  hipStream_t s = c->stream;
  const bool has_ch = std::is_same<Ph, MHD2D>::value && kp.ch_in < 0.0;
  LWFR_LAUNCH(KID_PRE, "k_pre", (k_pre<Ph, N, EPB>), dim3(c->nblk_pre), dim3(EPB * P), 0, s, kp, u_in);
  LWFR_LAUNCH(KID_DT, "k_dt", k_dt, dim3(1), dim3(256), 0, s, kp, d_dt_ch, has_ch ? 1 : 0);
  if (has_ch) {
    LWFR_LAUNCH(KID_CH, "k_ch", k_ch, dim3(c->nblk_ch), dim3(256), 0, s, kp);
    LWFR_LAUNCH(KID_CHFIN, "k_ch_fin", k_ch_fin, dim3(1), dim3(256), 0, s, kp, d_dt_ch);
  }
  const int nblk_el = (E + EPB - 1) / EPB;
  LWFR_LAUNCH(KID_STAGES, "k_stages", (k_stages<Ph, N, EPB>), dim3(nblk_el), dim3(EPB * P), 0, s, kp, u_in, u_out,
              d_alpha);
  const int nfp_total = DIM * E * NFP;
  LWFR_LAUNCH(KID_FACES, "k_faces", (k_faces<Ph, N>), dim3((nfp_total + 255) / 256), dim3(256), 0, s, kp, u_in);
  LWFR_LAUNCH(KID_UPDATE, "k_update", (k_update<Ph, N, EPB>), dim3(nblk_el), dim3(EPB * P), 0, s, kp, u_in, u_out,
              d_flags);
  return LWFR_OK;
}

// elements per workgroup of the adjoint kernels: about one wave
template <int N>
constexpr int epb_adj(int DIM) {
  return DIM == 1 ? 64 / (N + 1) : (N == 1 ? 16 : N == 2 ? 7 : N == 3 ? 4 : 2);
}

template <class Ph, int N>
lwfr_status launch_adjoint(lwfr_ctx* c, const KParams& kp, const double* u_n, const double* lam1, double* lam0) {
  constexpr int DIM = Ph::DIM, P = ipow(N + 1, DIM), NFP = DIM == 1 ? 1 : N + 1;
  constexpr int EPB = epb_adj<N>(DIM);
  const int E = c->E;
  hipStream_t s = c->stream;
  const int nblk = (E + EPB - 1) / EPB;
  LWFR_LAUNCH(KID_ADJ_UPDATE, "k_adj_update", (k_adj_update<Ph, N, EPB>), dim3(nblk), dim3(EPB * P), 0, s, kp, c->ap,
              u_n, lam1);
  const int nfp_total = DIM * E * NFP;
  LWFR_LAUNCH(KID_ADJ_FACES, "k_adj_faces", (k_adj_faces<Ph, N>), dim3((nfp_total + 255) / 256), dim3(256), 0, s, kp,
              c->ap, u_n);
  LWFR_LAUNCH(KID_ADJ_STAGES, "k_adj_stages", (k_adj_stages<Ph, N, EPB>), dim3(nblk), dim3(EPB * P), 0, s, kp, c->ap,
              u_n, lam0);
  return LWFR_OK;
}

template <class Ph>
lwfr_status launch_adjoint_n(lwfr_ctx* c, const KParams& kp, const double* u_n, const double* lam1, double* lam0) {
  switch (c->N) {
    case 1: return launch_adjoint<Ph, 1>(c, kp, u_n, lam1, lam0);
    case 2: return launch_adjoint<Ph, 2>(c, kp, u_n, lam1, lam0);
    case 3: return launch_adjoint<Ph, 3>(c, kp, u_n, lam1, lam0);
    case 4: return launch_adjoint<Ph, 4>(c, kp, u_n, lam1, lam0);
  }
  return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
}

lwfr_status dispatch_adjoint(lwfr_ctx* c, const KParams& kp, const double* u_n, const double* lam1, double* lam0) {
  switch (c->cfg.equation) {
    case LWFR_EQ_SW1D: return launch_adjoint_n<SW1D>(c, kp, u_n, lam1, lam0);
    case LWFR_EQ_SW2D: return launch_adjoint_n<SW2D>(c, kp, u_n, lam1, lam0);
    case LWFR_EQ_GLMMHD2D: return launch_adjoint_n<MHD2D>(c, kp, u_n, lam1, lam0);
    case LWFR_EQ_LINADV1D: return launch_adjoint_n<LinAdv1D>(c, kp, u_n, lam1, lam0);
    case LWFR_EQ_VARADV1D: return launch_adjoint_n<VarAdv1D>(c, kp, u_n, lam1, lam0);
  }
  return fail(LWFR_E_UNSUPPORTED, "unknown equation");
}

template <class Ph>
lwfr_status launch_step_n(lwfr_ctx* c, const KParams& kp, const double* u_in, double* u_out, double* d_dt_ch,
                          double* d_alpha, uint32_t* d_flags) {
  switch (c->N) {
    case 1: return launch_step<Ph, 1>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case 2: return launch_step<Ph, 2>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case 3: return launch_step<Ph, 3>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case 4: return launch_step<Ph, 4>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
  }
  return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
}

lwfr_status dispatch_step(lwfr_ctx* c, const KParams& kp, const double* u_in, double* u_out, double* d_dt_ch,
                          double* d_alpha, uint32_t* d_flags) {
  switch (c->cfg.equation) {
    case LWFR_EQ_SW1D: return launch_step_n<SW1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case LWFR_EQ_SW2D: return launch_step_n<SW2D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case LWFR_EQ_GLMMHD2D: return launch_step_n<MHD2D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case LWFR_EQ_LINADV1D: return launch_step_n<LinAdv1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
    case LWFR_EQ_VARADV1D: return launch_step_n<VarAdv1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags);
  }
  return fail(LWFR_E_UNSUPPORTED, "unknown equation");
}

// kernel parameters whose switch and trace arrays live in a caller's tape
KParams with_tape(const lwfr_ctx* c, KParams kp, void* tape) {
  char* t = static_cast<char*>(tape);
  kp.scal = reinterpret_cast<double*>(t + c->tp_scal);
  kp.alpha = reinterpret_cast<double*>(t + c->tp_alpha);
  kp.theta_face = reinterpret_cast<double*>(t + c->tp_thf);
  kp.theta_elem = reinterpret_cast<double*>(t + c->tp_thel);
  kp.untr = reinterpret_cast<double*>(t + c->tp_untr);
  kp.Utr = reinterpret_cast<double*>(t + c->tp_Utr);
  return kp;
}

bool ranges_overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" {

const char* lwfr_last_error(void) { return g_err.c_str(); }

lwfr_status lwfr_cfl_number(int32_t degree, double* cfl) {
  if (!cfl) return fail(LWFR_E_INVALID_ARG, "cfl is null");
  if (degree < 1 || degree > 4) return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
  *cfl = fourier_cfl(degree);
  return LWFR_OK;
}

lwfr_status lwfr_init(const lwfr_config* cfg, lwfr_ctx** out) {
  if (!cfg || !out) return fail(LWFR_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (cfg->abi_version != LWFR_ABI_VERSION) return fail(LWFR_E_INVALID_ARG, "abi_version mismatch");
  EqInfo info;
  if (!eq_info(cfg->equation, info)) return fail(LWFR_E_INVALID_ARG, "unknown equation");
  if (cfg->degree < 1 || cfg->degree > 4) return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
  const int ny = info.DIM == 2 ? cfg->nelem[1] : 1;
  if (cfg->nelem[0] < 1 || ny < 1) return fail(LWFR_E_INVALID_ARG, "nelem must be positive");
  if ((long long)cfg->nelem[0] * ny > (1LL << 26)) return fail(LWFR_E_INVALID_ARG, "too many elements");
  for (int d = 0; d < info.DIM; ++d)
    if (!(cfg->hi[d] > cfg->lo[d]) || !std::isfinite(cfg->hi[d] - cfg->lo[d]))
      return fail(LWFR_E_INVALID_ARG, "domain box must have hi > lo");
  if (cfg->blending < 0 || cfg->blending > 2) return fail(LWFR_E_INVALID_ARG, "blending must be 0, 1 or 2");
  if (!(cfg->cfl_safety > 0.0)) return fail(LWFR_E_INVALID_ARG, "cfl_safety must be positive");
  if (!(cfg->alpha_max >= 0.0 && cfg->alpha_max <= 1.0)) return fail(LWFR_E_INVALID_ARG, "alpha_max in [0,1]");
  if (!(cfg->alpha_min >= 0.0 && cfg->alpha_min < 0.5)) return fail(LWFR_E_INVALID_ARG, "alpha_min in [0,0.5)");
  if (cfg->alpha_force > 1.0) return fail(LWFR_E_INVALID_ARG, "alpha_force must be <= 1");
  if (cfg->equation == LWFR_EQ_GLMMHD2D && !(cfg->gamma > 1.0)) return fail(LWFR_E_INVALID_ARG, "gamma > 1");
  if ((cfg->equation == LWFR_EQ_SW1D || cfg->equation == LWFR_EQ_SW2D) && !(cfg->gravity > 0.0))
    return fail(LWFR_E_INVALID_ARG, "gravity > 0");

  lwfr_ctx* c = new lwfr_ctx();
  c->cfg = *cfg;
  c->M = info.M; c->DIM = info.DIM; c->K = info.K;
  c->N = cfg->degree; c->n1 = c->N + 1;
  c->P = info.DIM == 1 ? c->n1 : c->n1 * c->n1;
  c->NFP = info.DIM == 1 ? 1 : c->n1;
  c->E = cfg->nelem[0] * ny;
  {
    const int epb = epb_runtime(c->N, c->DIM, c->M);
    c->nblk_pre = (c->E + epb - 1) / epb;  // k_pre: 256/P elements per block
    c->nblk_ch = (c->E + 255) / 256;       // k_ch: one thread per element
  }
  c->rd = make_refdata(c->N);
  c->cfl = cfg->cfl_number > 0.0 ? cfg->cfl_number : fourier_cfl(c->N);

  KParams& kp = c->kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.nx = cfg->nelem[0]; kp.ny = ny; kp.E = c->E; kp.nblk_pre = c->nblk_pre; kp.nblk_ch = c->nblk_ch;
  for (int d = 0; d < 2; ++d) {
    kp.dx[d] = d < info.DIM ? (cfg->hi[d] - cfg->lo[d]) / (d == 0 ? cfg->nelem[0] : ny) : 1.0;
    kp.inv_dx[d] = 1.0 / kp.dx[d];
  }
  for (int a = 0; a < c->n1; ++a) {
    for (int b = 0; b < c->n1; ++b) { kp.D[a][b] = c->rd.D[a][b]; kp.Leg[a][b] = c->rd.Leg[a][b]; }
    kp.VL[a] = c->rd.VL[a]; kp.VR[a] = c->rd.VR[a]; kp.w[a] = c->rd.w[a];
    kp.gR[a] = c->rd.gR[a]; kp.gL[a] = c->rd.gL[a];
    for (int d = 0; d < 2; ++d) kp.inv_wdx[d][a] = 1.0 / (c->rd.w[a] * kp.dx[d]);
  }
  kp.g = cfg->gravity; kp.gamma = cfg->gamma;
  kp.blending = cfg->blending;
  kp.alpha_max = cfg->alpha_max; kp.alpha_min = cfg->alpha_min; kp.alpha_force = cfg->alpha_force;
  kp.ind_T = 0.5 * std::pow(10.0, -1.8 * std::pow(c->N + 1.0, 0.25));
  kp.ind_s = std::log(9999.0);
  kp.cs_cfl = cfg->cfl_safety * c->cfl;
  kp.ch_in = -1.0;

  // workspace carving
  const size_t nfpt = (size_t)c->DIM * c->E * c->NFP;  // face points over all directions
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  c->off_scal = take(8 * sizeof(double));
  c->off_part = take((size_t)c->nblk_pre * sizeof(double));
  c->off_part2 = take((size_t)c->nblk_ch * sizeof(double));
  c->off_speeds = take((size_t)c->E * 2 * c->DIM * sizeof(double));
  c->off_araw = take((size_t)c->E * sizeof(double));
  c->off_alpha = take((size_t)c->E * sizeof(double));
  c->off_thel = take((size_t)c->E * sizeof(double));
  c->off_Ftr = take(nfpt * 2 * c->M * sizeof(double));
  c->off_Utr = take(nfpt * 2 * c->M * sizeof(double));
  c->off_untr = take(nfpt * 2 * c->M * sizeof(double));
  c->off_Fm = take(nfpt * c->M * sizeof(double));
  c->off_Fp = take(nfpt * c->M * sizeof(double));
  c->off_Dm = take(nfpt * c->M * sizeof(double));
  c->off_Dp = take(nfpt * c->M * sizeof(double));
  c->off_thf = take(nfpt * sizeof(double));
  c->off_guard = take(nfpt * sizeof(uint32_t));
  c->off_flag = take(sizeof(uint32_t));
  c->adjoint = (cfg->flags & LWFR_CFG_ADJOINT) != 0;
  if (c->adjoint) {
    const size_t nst = (size_t)c->M * c->E * c->P * sizeof(double);
    c->off_uscr = take(nst);
    c->off_grvol = take(nst);
    c->off_gun = take(nst);
    c->off_gFm = take(nfpt * c->M * sizeof(double));
    c->off_gFp = take(nfpt * c->M * sizeof(double));
    c->off_gDm = take(nfpt * c->M * sizeof(double));
    c->off_gDp = take(nfpt * c->M * sizeof(double));
    c->off_gFtr = take(nfpt * 2 * c->M * sizeof(double));
    c->off_gUtr = take(nfpt * 2 * c->M * sizeof(double));
    c->off_guntr = take(nfpt * 2 * c->M * sizeof(double));
    c->off_gsL = take(nfpt * c->M * sizeof(double));
    c->off_gsR = take(nfpt * c->M * sizeof(double));
  }
  c->ws_bytes = off;
  {
    size_t t = 0;
    auto tk = [&](size_t bytes) { size_t o = t; t += align256(bytes); return o; };
    c->tp_scal = tk(8 * sizeof(double));
    c->tp_alpha = tk((size_t)c->E * sizeof(double));
    c->tp_thf = tk(nfpt * sizeof(double));
    c->tp_thel = tk((size_t)c->E * sizeof(double));
    c->tp_untr = tk(nfpt * 2 * c->M * sizeof(double));
    c->tp_Utr = tk(nfpt * 2 * c->M * sizeof(double));
    c->tape_bytes = t;
  }
  *out = c;
  return LWFR_OK;
}

lwfr_status lwfr_workspace_bytes(const lwfr_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(LWFR_E_INVALID_ARG, "null argument");
  *bytes = c->ws_bytes;
  return LWFR_OK;
}

lwfr_status lwfr_state_size(const lwfr_ctx* c, size_t* n) {
  if (!c || !n) return fail(LWFR_E_INVALID_ARG, "null argument");
  *n = (size_t)c->M * c->E * c->P;
  return LWFR_OK;
}

lwfr_status lwfr_reference_nodes(const lwfr_ctx* c, double* xi, double* w) {
  if (!c || !xi || !w) return fail(LWFR_E_INVALID_ARG, "null argument");
  for (int p = 0; p < c->n1; ++p) { xi[p] = c->rd.xi[p]; w[p] = c->rd.w[p]; }
  return LWFR_OK;
}

lwfr_status lwfr_bind(lwfr_ctx* c, void* d_ws, size_t bytes, void* stream) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!d_ws) return fail(LWFR_E_WORKSPACE, "workspace is null");
  if (bytes < c->ws_bytes) return fail(LWFR_E_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(LWFR_E_WORKSPACE, "workspace not 256-byte aligned");
  c->ws = d_ws;
  c->stream = static_cast<hipStream_t>(stream);
  char* b = static_cast<char*>(d_ws);
  KParams& kp = c->kp;
  kp.scal = reinterpret_cast<double*>(b + c->off_scal);
  kp.part = reinterpret_cast<double*>(b + c->off_part);
  kp.part2 = reinterpret_cast<double*>(b + c->off_part2);
  kp.speeds = reinterpret_cast<double*>(b + c->off_speeds);
  kp.alpha_raw = reinterpret_cast<double*>(b + c->off_araw);
  kp.alpha = reinterpret_cast<double*>(b + c->off_alpha);
  kp.theta_elem = reinterpret_cast<double*>(b + c->off_thel);
  kp.Ftr = reinterpret_cast<double*>(b + c->off_Ftr);
  kp.Utr = reinterpret_cast<double*>(b + c->off_Utr);
  kp.untr = reinterpret_cast<double*>(b + c->off_untr);
  kp.Fm = reinterpret_cast<double*>(b + c->off_Fm);
  kp.Fp = reinterpret_cast<double*>(b + c->off_Fp);
  kp.Dm = reinterpret_cast<double*>(b + c->off_Dm);
  kp.Dp = reinterpret_cast<double*>(b + c->off_Dp);
  kp.theta_face = reinterpret_cast<double*>(b + c->off_thf);
  kp.guard_face = reinterpret_cast<uint32_t*>(b + c->off_guard);
  kp.flag_or = reinterpret_cast<uint32_t*>(b + c->off_flag);
  if (c->adjoint) {
    AdjParams& ap = c->ap;
    ap.g_rvol = reinterpret_cast<double*>(b + c->off_grvol);
    ap.g_un = reinterpret_cast<double*>(b + c->off_gun);
    ap.gFm = reinterpret_cast<double*>(b + c->off_gFm);
    ap.gFp = reinterpret_cast<double*>(b + c->off_gFp);
    ap.gDm = reinterpret_cast<double*>(b + c->off_gDm);
    ap.gDp = reinterpret_cast<double*>(b + c->off_gDp);
    ap.gFtr = reinterpret_cast<double*>(b + c->off_gFtr);
    ap.gUtr = reinterpret_cast<double*>(b + c->off_gUtr);
    ap.guntr = reinterpret_cast<double*>(b + c->off_guntr);
    ap.gsL = reinterpret_cast<double*>(b + c->off_gsL);
    ap.gsR = reinterpret_cast<double*>(b + c->off_gsR);
  }
  hipError_t err = hipMemsetAsync(kp.flag_or, 0, sizeof(uint32_t), c->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(err));
  c->bound = true;
  return LWFR_OK;
}

lwfr_status lwfr_step(lwfr_ctx* c, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                      double* d_alpha, uint32_t* d_flags) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!d_u_in || !d_u_out) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_u_in, d_u_out, bytes)) return fail(LWFR_E_INVALID_ARG, "u_out aliases u_in");
  if (!std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt is not finite");
  KParams kp = c->kp;
  kp.dt_in = dt > 0.0 ? dt : 0.0;
  kp.ch_in = -1.0;
  return dispatch_step(c, kp, d_u_in, d_u_out, d_dt_ch, d_alpha, d_flags);
}

lwfr_status lwfr_step_fixed(lwfr_ctx* c, const double* d_u_in, double* d_u_out, double dt, double ch,
                            double* d_alpha, uint32_t* d_flags) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!d_u_in || !d_u_out) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_u_in, d_u_out, bytes)) return fail(LWFR_E_INVALID_ARG, "u_out aliases u_in");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt must be positive and finite");
  if (!(ch >= 0.0) || !std::isfinite(ch)) return fail(LWFR_E_INVALID_ARG, "ch must be >= 0 and finite");
  KParams kp = c->kp;
  kp.dt_in = dt;
  kp.ch_in = ch;
  return dispatch_step(c, kp, d_u_in, d_u_out, nullptr, d_alpha, d_flags);
}

lwfr_status lwfr_residual(lwfr_ctx* c, const double* d_u, double dt, int32_t mode, double* d_R) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!d_u || !d_R) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt must be positive and finite");
  if (mode < 0 || mode > 2) return fail(LWFR_E_INVALID_ARG, "mode must be 0, 1 or 2");
  const size_t n = (size_t)c->M * c->E * c->P;
  if (ranges_overlap(d_u, d_R, n * sizeof(double))) return fail(LWFR_E_INVALID_ARG, "R aliases u");
  KParams kp = c->kp;
  kp.dt_in = dt;
  if (mode == 0) { kp.blending = 0; kp.alpha_force = -1.0; }
  if (mode == 1) { kp.blending = 1; kp.alpha_force = 1.0; }
  lwfr_status st = dispatch_step(c, kp, d_u, d_R, nullptr, nullptr, nullptr);
  if (st != LWFR_OK) return st;
  LWFR_LAUNCH(KID_RESIDUAL, "k_residual", k_residual, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
              d_u, d_R, n, (const double*)kp.scal);
  return LWFR_OK;
}

lwfr_status lwfr_tape_bytes(const lwfr_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(LWFR_E_INVALID_ARG, "null argument");
  *bytes = c->tape_bytes;
  return LWFR_OK;
}

lwfr_status lwfr_step_taped(lwfr_ctx* c, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                            void* d_tape) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!d_u_in || !d_u_out || !d_tape) return fail(LWFR_E_INVALID_ARG, "null pointer");
  if (reinterpret_cast<uintptr_t>(d_tape) % 256 != 0) return fail(LWFR_E_INVALID_ARG, "tape not 256-byte aligned");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_u_in, d_u_out, bytes)) return fail(LWFR_E_INVALID_ARG, "u_out aliases u_in");
  if (!std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt is not finite");
  KParams kp = with_tape(c, c->kp, d_tape);
  kp.dt_in = dt > 0.0 ? dt : 0.0;
  kp.ch_in = -1.0;
  return dispatch_step(c, kp, d_u_in, d_u_out, d_dt_ch, nullptr, nullptr);
}

lwfr_status lwfr_adjoint_step(lwfr_ctx* c, const double* d_u_n, double dt, const double* d_lam_np1,
                              double* d_lam_n, const void* d_tape) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!c->adjoint) return fail(LWFR_E_STATE, "context was created without LWFR_CFG_ADJOINT");
  if (!d_u_n || !d_lam_np1 || !d_lam_n) return fail(LWFR_E_INVALID_ARG, "null pointer");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt must be positive and finite");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_lam_n, d_u_n, bytes) || ranges_overlap(d_lam_n, d_lam_np1, bytes))
    return fail(LWFR_E_INVALID_ARG, "lam_n aliases an input");
  KParams kp = c->kp;
  kp.dt_in = dt;
  if (d_tape) {
    if (reinterpret_cast<uintptr_t>(d_tape) % 256 != 0) return fail(LWFR_E_INVALID_ARG, "tape not 256-byte aligned");
    kp = with_tape(c, kp, const_cast<void*>(d_tape));
  } else {
    double* uscr = reinterpret_cast<double*>(static_cast<char*>(c->ws) + c->off_uscr);
    lwfr_status st = dispatch_step(c, kp, d_u_n, uscr, nullptr, nullptr, nullptr);
    if (st != LWFR_OK) return st;
  }
  return dispatch_adjoint(c, kp, d_u_n, d_lam_np1, d_lam_n);
}

lwfr_status lwfr_query(lwfr_ctx* c, uint32_t* flags_or) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  uint32_t h = 0;
  hipError_t err = hipMemcpyAsync(&h, c->kp.flag_or, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
  if (err == hipSuccess) err = hipMemsetAsync(c->kp.flag_or, 0, sizeof(uint32_t), c->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("lwfr_query: ") + hipGetErrorString(err));
  if (flags_or) *flags_or = h;
  if (h & LWFR_FLAG_NONFINITE) return fail(LWFR_E_NONFINITE, "a step produced a non-finite value");
  if (h & LWFR_FLAG_LOW_INADM) return fail(LWFR_E_INADMISSIBLE, "a lower order update was not admissible");
  return LWFR_OK;
}

lwfr_status lwfr_timing_begin(lwfr_ctx* c, int32_t max_launches) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(LWFR_E_INVALID_ARG, "max_launches out of range");
  const size_t need = 2 * (size_t)max_launches;
  while (c->ev.size() < need) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipEventCreate: ") + hipGetErrorString(err));
    c->ev.push_back(e);
  }
  c->ev_kernel.assign(c->ev.size() / 2, -1);
  c->ev_used = 0;
  c->timing = true;
  return LWFR_OK;
}

lwfr_status lwfr_timing_end(lwfr_ctx* c, double* ms, uint32_t* launches) {
  if (!c || !ms || !launches) return fail(LWFR_E_INVALID_ARG, "null argument");
  if (!c->timing) return fail(LWFR_E_STATE, "lwfr_timing_begin has not been called");
  c->timing = false;
  hipError_t err = hipStreamSynchronize(c->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("lwfr_timing_end: ") + hipGetErrorString(err));
  for (int k = 0; k < LWFR_TIMING_KERNELS; ++k) { ms[k] = 0.0; launches[k] = 0; }
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float t = 0.0f;
    err = hipEventElapsedTime(&t, c->ev[i], c->ev[i + 1]);
    if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(err));
    const int kid = c->ev_kernel[i / 2];
    if (kid >= 0 && kid < LWFR_TIMING_KERNELS) { ms[kid] += t; launches[kid] += 1; }
  }
  return LWFR_OK;
}

lwfr_status lwfr_destroy(lwfr_ctx* c) {
  if (c)
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
  return LWFR_OK;
}

}  // extern "C"
