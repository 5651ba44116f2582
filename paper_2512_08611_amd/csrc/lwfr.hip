// C ABI of the time step (declarations and contracts in include/lwfr.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lwfr.h"
#include "adjoint.hpp"
#include "batch.hpp"
#include "kernels.hpp"

using namespace lwfr;

namespace {

thread_local std::string g_err;

lwfr_status fail(lwfr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// optional per-kernel timing with HIP events on the bound stream
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kernel;  // kernel id of the launch between event 2i and 2i+1
  size_t used = 0;
};

}  // namespace

struct lwfr_ctx {
  lwfr_config cfg;
  int M = 0, DIM = 0, K = 0, N = 0, n1 = 0, P = 0, NFP = 0, E = 0;
  int nblk_pre = 0, nblk_ch = 0, nblk_dt = 0;
  RefData rd;
  double cfl = 0.0;
  KParams kp;
  // workspace carving (byte offsets)
  size_t off_scal, off_part, off_part2, off_part3, off_speeds, off_araw, off_alpha, off_thel, off_Ftr, off_Utr,
      off_Fm, off_Fp, off_Dm, off_Dp, off_ffl, off_thf, off_thl, off_gul, off_flag, off_eflags, off_srows,
      ws_bytes;
  int nblk_stats = 0;
  size_t fwd_bytes = 0;
  // non-periodic sides: k_bfaces threads (0: periodic mesh); Dirichlet sides
  int bface_threads = 0;
  bool dirichlet = false;
  // adjoint workspace (only with LWFR_CFG_ADJOINT)
  bool adjoint = false;
  size_t off_uscr, off_grvol, off_gun, off_gFm, off_gFp, off_gDm, off_gDp, off_gFtr, off_gUtr, off_guntr, off_gsL,
      off_gsR;
  AdjParams ap;
  // per-step tape: what the reverse kernels read from a forward step
  size_t tp_scal, tp_alpha, tp_thf, tp_thel, tp_Utr, tape_bytes;
  void* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  Timing tm;
  hipGraphExec_t graph = nullptr;  // captured step sequence (lwfr_graph_capture)
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
    case LWFR_EQ_JINXIN1D: info = {JinXin1D::M, JinXin1D::DIM, JinXin1D::K}; return true;
  }
  return false;
}

// Elements per workgroup of the per-point kernels (k_pre, k_stages, k_update).
#ifndef LWFR_EPB_OVERRIDE
#define LWFR_EPB_OVERRIDE 0
#endif
// Elements per workgroup of k_pre and the update.  Default: 256 threads per
// workgroup.  2-D with 9 variables: degree 4 uses 5 elements (125 threads);
// degree 3 uses 4 elements, one wave, whose barriers then hold no other wave
// (measured fastest for the update that also forms the next step's element
// data).
template <int N>
constexpr int epb_for(int DIM, int M) {
  return LWFR_EPB_OVERRIDE > 0                 ? LWFR_EPB_OVERRIDE
         : (DIM == 2 && N == 4 && M >= 9) ? 5
         : (DIM == 2 && N == 3 && M >= 9) ? 4
                                          : 256 / ipow(N + 1, DIM);
}
// Elements per workgroup of the stage kernel (stage_lanes lanes per point):
// about 256 threads.
#ifndef LWFR_EPB_STAGES_OVERRIDE
#define LWFR_EPB_STAGES_OVERRIDE 0
#endif
template <class Ph, int N>
constexpr int epb_stages() {
  return LWFR_EPB_STAGES_OVERRIDE > 0 ? LWFR_EPB_STAGES_OVERRIDE
         : (256 / (stage_lanes<Ph>() * ipow(N + 1, Ph::DIM)) > 0 ? 256 / (stage_lanes<Ph>() * ipow(N + 1, Ph::DIM)) : 1);
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
  KID_ADJ_UPDATE, KID_ADJ_FACES, KID_ADJ_STAGES, KID_B_PRE, KID_B_DT, KID_B_STAGES, KID_B_FACES, KID_B_UPDATE,
  KID_BFACES, KID_COUNT
};
static_assert(KID_COUNT == LWFR_TIMING_KERNELS, "kernel ids and LWFR_TIMING_KERNELS disagree");

// Records an event before (open) and after (close) a launch when timing is on.
struct TimedLaunch {
  Timing& tm;
  hipStream_t s;
  int kid;
  bool on;
  TimedLaunch(Timing& tm_, hipStream_t s_, int kid_) : tm(tm_), s(s_), kid(kid_), on(false) {
    if (tm.on && tm.used + 2 <= tm.ev.size()) {
      on = true;
      (void)hipEventRecord(tm.ev[tm.used], s);
    }
  }
  void close() {
    if (on) {
      (void)hipEventRecord(tm.ev[tm.used + 1], s);
      tm.kernel[tm.used / 2] = kid;
      tm.used += 2;
      on = false;
    }
  }
};

#define LWFR_LAUNCH(kid, name, ...)          \
  do {                                       \
    TimedLaunch tl_(c->tm, c->stream, kid);  \
    hipLaunchKernelGGL(__VA_ARGS__);         \
    tl_.close();                             \
    LWFR_CHECK_LAUNCH(name);                 \
  } while (0)

// The launch sequence of one step for system Ph at degree N (Tab: the stage
// tableau, an IMEX pair for systems with a source).
// the approximate Lax-Wendroff stage kernel with two lanes per solution point
// for the systems whose cRK stage kernel has two
#ifndef LWFR_ALW2
#define LWFR_ALW2 1
#endif

// chain (steps of a captured graph, each starting from the previous one's
// result): kChainFromPrev, the previous step's update formed this step's element
// data, so k_pre is skipped; kChainToNext, this step's update forms the next
// step's.
constexpr int kChainFromPrev = 1, kChainToNext = 2;

template <class Ph, int N, class Tab = Tableau<N>>
lwfr_status launch_step(lwfr_ctx* c, const KParams& kp, const double* u_in, double* u_out, double* d_dt_ch,
                        double* d_alpha, uint32_t* d_flags, lwfr_stats* d_stats, int chain = 0) {
  constexpr int DIM = Ph::DIM, P = ipow(N + 1, DIM), NFP = DIM == 1 ? 1 : N + 1;
  constexpr int EPB = epb_for<N>(DIM, Ph::M);
  const int E = c->E;
  hipStream_t s = c->stream;
  const bool has_ch = std::is_same<Ph, MHD2D>::value && kp.ch_in < 0.0;
  if (!(chain & kChainFromPrev))
    LWFR_LAUNCH(KID_PRE, "k_pre", (k_pre<Ph, N, EPB>), dim3(c->nblk_pre), dim3(EPB * P), 0, s, kp, u_in);
  LWFR_LAUNCH(KID_DT, "k_dt", k_dt, dim3(has_ch ? c->nblk_dt : 1), dim3(1024), 0, s, kp, d_dt_ch, has_ch ? 1 : 0);
  if (has_ch) {
    LWFR_LAUNCH(KID_CH, "k_ch", k_ch, dim3(c->nblk_ch), dim3(256), 0, s, kp);
    LWFR_LAUNCH(KID_CHFIN, "k_ch_fin", k_ch_fin, dim3(1), dim3(1024), 0, s, kp, d_dt_ch);
  }
  const int nblk_el = (E + EPB - 1) / EPB;
  constexpr int EPBS = epb_stages<Ph, N>();
  if (c->cfg.flags & LWFR_CFG_ALW) {
    if constexpr (!Ph::SRC) {
      if constexpr (stage_lanes<Ph>() == 2 && LWFR_ALW2)
        LWFR_LAUNCH(KID_STAGES, "k_stages_alw", (k_stages_alw2<Ph, N, EPBS>), dim3((E + EPBS - 1) / EPBS),
                    dim3(stages2_threads(EPBS, P)), 0, s, kp, u_in, u_out, d_alpha);
      else
        LWFR_LAUNCH(KID_STAGES, "k_stages_alw", (k_stages_alw<Ph, N, EPB>), dim3(nblk_el), dim3(EPB * P), 0, s, kp,
                    u_in, u_out, d_alpha);
    }
  } else {
    LWFR_LAUNCH(KID_STAGES, "k_stages", (k_stages<Ph, N, EPBS, Tab>), dim3((E + EPBS - 1) / EPBS),
                dim3(stage_threads<Ph, N, EPBS>()), 0, s, kp, u_in, u_out, d_alpha);
  }
  const int nfp_total = DIM * E * NFP;
  if constexpr (face_lanes<Ph>() == 2)
    LWFR_LAUNCH(KID_FACES, "k_faces", (k_faces2<Ph, N>), dim3((nfp_total + 127) / 128), dim3(256), 0, s, kp, u_in);
  else
    LWFR_LAUNCH(KID_FACES, "k_faces", (k_faces<Ph, N>), dim3((nfp_total + 255) / 256), dim3(256), 0, s, kp, u_in);
  if (c->bface_threads > 0)
    LWFR_LAUNCH(KID_BFACES, "k_bfaces", (k_bfaces<Ph, N>), dim3((c->bface_threads + 63) / 64), dim3(64), 0, s, kp,
                u_in);
  // statistics need the element flags: the context's own array when the caller takes none
  uint32_t* eflags = d_stats && !d_flags ? kp.eflags : d_flags;
  if (chain & kChainToNext)
    LWFR_LAUNCH(KID_UPDATE, "k_update", (k_update<Ph, N, EPB, true>), dim3(nblk_el), dim3(EPB * P), 0, s, kp, u_in,
                u_out, eflags);
  else
    LWFR_LAUNCH(KID_UPDATE, "k_update", (k_update<Ph, N, EPB>), dim3(nblk_el), dim3(EPB * P), 0, s, kp, u_in, u_out,
                eflags);
  if (d_stats) {
    double* rows = kp.stats_rows;
    hipLaunchKernelGGL((k_stats<Ph, N>), dim3(c->nblk_stats), dim3(256), 0, s, kp, (const double*)u_out,
                       (const uint32_t*)eflags, rows);
    LWFR_CHECK_LAUNCH("k_stats");
    hipLaunchKernelGGL((k_stats_fin<lwfr_stats>), dim3(1), dim3(256), 0, s, kp, (const double*)rows, c->nblk_stats,
                       d_stats);
    LWFR_CHECK_LAUNCH("k_stats_fin");
  }
  return LWFR_OK;
}

// GLM-MHD's adjoint stage sweep with two lanes per solution point
#ifndef LWFR_ADJ_STAGES2
#define LWFR_ADJ_STAGES2 1
#endif

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
  if constexpr (std::is_same<Ph, MHD2D>::value && LWFR_ADJ_STAGES2) {
    constexpr int EPB2 = epb_adj2(P);
    LWFR_LAUNCH(KID_ADJ_STAGES, "k_adj_stages", (k_adj_stages2<Ph, N, EPB2>), dim3((E + EPB2 - 1) / EPB2), dim3(256),
                0, s, kp, c->ap, u_n, lam0);
  } else {
    LWFR_LAUNCH(KID_ADJ_STAGES, "k_adj_stages", (k_adj_stages<Ph, N, EPB>), dim3(nblk), dim3(EPB * P), 0, s, kp,
                c->ap, u_n, lam0);
  }
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
                          double* d_alpha, uint32_t* d_flags, lwfr_stats* d_stats, int chain) {
  if constexpr (Ph::SRC) {
    const bool ht = (c->cfg.flags & LWFR_CFG_IMEX_HT112) != 0;
    switch (c->N) {
      case 1: return ht ? launch_step<Ph, 1, ImexHT>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain)
                        : launch_step<Ph, 1, ImexSSP3>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
      case 2: return ht ? launch_step<Ph, 2, ImexHT>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain)
                        : launch_step<Ph, 2, ImexSSP3>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
      case 3: return ht ? launch_step<Ph, 3, ImexHT>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain)
                        : launch_step<Ph, 3, ImexSSP3>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
      case 4: return ht ? launch_step<Ph, 4, ImexHT>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain)
                        : launch_step<Ph, 4, ImexSSP3>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    }
    return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
  } else {
    switch (c->N) {
      case 1: return launch_step<Ph, 1>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
      case 2: return launch_step<Ph, 2>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
      case 3: return launch_step<Ph, 3>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
      case 4: return launch_step<Ph, 4>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    }
    return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
  }
}

lwfr_status dispatch_step(lwfr_ctx* c, const KParams& kp, const double* u_in, double* u_out, double* d_dt_ch,
                          double* d_alpha, uint32_t* d_flags, lwfr_stats* d_stats = nullptr, int chain = 0) {
  switch (c->cfg.equation) {
    case LWFR_EQ_SW1D: return launch_step_n<SW1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    case LWFR_EQ_SW2D: return launch_step_n<SW2D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    case LWFR_EQ_GLMMHD2D: return launch_step_n<MHD2D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    case LWFR_EQ_LINADV1D: return launch_step_n<LinAdv1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    case LWFR_EQ_VARADV1D: return launch_step_n<VarAdv1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
    case LWFR_EQ_JINXIN1D: return launch_step_n<JinXin1D>(c, kp, u_in, u_out, d_dt_ch, d_alpha, d_flags, d_stats, chain);
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
  kp.Utr = reinterpret_cast<double*>(t + c->tp_Utr);
  return kp;
}

// a step of a context with a Dirichlet side needs its data and a given dt
lwfr_status dirichlet_ready(const lwfr_ctx* c, double dt) {
  if (!c->dirichlet) return LWFR_OK;
  if (!c->kp.ghost) return fail(LWFR_E_STATE, "Dirichlet side without data (lwfr_set_boundary_data)");
  if (!(dt > 0.0)) return fail(LWFR_E_INVALID_ARG, "a context with a Dirichlet side needs dt > 0");
  return LWFR_OK;
}

bool ranges_overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

lwfr_status timing_begin(Timing& tm, int32_t max_launches) {
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(LWFR_E_INVALID_ARG, "max_launches out of range");
  const size_t need = 2 * (size_t)max_launches;
  while (tm.ev.size() < need) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipEventCreate: ") + hipGetErrorString(err));
    tm.ev.push_back(e);
  }
  tm.kernel.assign(tm.ev.size() / 2, -1);
  tm.used = 0;
  tm.on = true;
  return LWFR_OK;
}

lwfr_status timing_end(Timing& tm, hipStream_t s, double* ms, uint32_t* launches) {
  if (!tm.on) return fail(LWFR_E_STATE, "timing was not begun");
  tm.on = false;
  hipError_t err = hipStreamSynchronize(s);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("timing end: ") + hipGetErrorString(err));
  for (int k = 0; k < LWFR_TIMING_KERNELS; ++k) { ms[k] = 0.0; launches[k] = 0; }
  for (size_t i = 0; i + 1 < tm.used; i += 2) {
    float t = 0.0f;
    err = hipEventElapsedTime(&t, tm.ev[i], tm.ev[i + 1]);
    if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(err));
    const int kid = tm.kernel[i / 2];
    if (kid >= 0 && kid < LWFR_TIMING_KERNELS) { ms[kid] += t; launches[kid] += 1; }
  }
  return LWFR_OK;
}

// Captures nsteps calls of step(k) on stream s into an executable graph
// (replacing *exec).  Timing is suspended during the capture (events recorded
// inside a graph cannot be timed).
template <class F>
lwfr_status capture(hipStream_t s, Timing& tm, hipGraphExec_t& exec, int nsteps, F&& step) {
  if (!s) return fail(LWFR_E_STATE, "graph capture needs a non-default stream");
  const bool timing = tm.on;
  tm.on = false;
  hipError_t err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) {
    tm.on = timing;
    return fail(LWFR_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(err));
  }
  lwfr_status st = LWFR_OK;
  for (int k = 0; k < nsteps && st == LWFR_OK; ++k) st = step(k);
  hipGraph_t g = nullptr;
  err = hipStreamEndCapture(s, &g);
  tm.on = timing;
  if (st != LWFR_OK) { if (g) (void)hipGraphDestroy(g); return st; }
  if (err != hipSuccess) { if (g) (void)hipGraphDestroy(g); return fail(LWFR_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(err)); }
  hipGraphExec_t ge = nullptr;
  err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err));
  if (exec) (void)hipGraphExecDestroy(exec);
  exec = ge;
  return LWFR_OK;
}

// points the workspace arrays of kp into the buffer at b (the context's layout)
void carve_kp(const lwfr_ctx* c, char* b, KParams& kp) {
  kp.scal = reinterpret_cast<double*>(b + c->off_scal);
  kp.part = reinterpret_cast<double*>(b + c->off_part);
  kp.part2 = reinterpret_cast<double*>(b + c->off_part2);
  kp.part3 = reinterpret_cast<double*>(b + c->off_part3);
  kp.speeds = reinterpret_cast<double*>(b + c->off_speeds);
  kp.alpha_raw = reinterpret_cast<double*>(b + c->off_araw);
  kp.alpha = reinterpret_cast<double*>(b + c->off_alpha);
  kp.theta_elem = reinterpret_cast<double*>(b + c->off_thel);
  kp.Ftr = reinterpret_cast<double*>(b + c->off_Ftr);
  kp.Utr = reinterpret_cast<double*>(b + c->off_Utr);
  kp.Fm = reinterpret_cast<double*>(b + c->off_Fm);
  kp.Fp = reinterpret_cast<double*>(b + c->off_Fp);
  kp.Dm = c->off_Dm ? reinterpret_cast<double*>(b + c->off_Dm) : nullptr;
  kp.Dp = c->off_Dp ? reinterpret_cast<double*>(b + c->off_Dp) : nullptr;
  kp.theta_face = nullptr;  // kept only in a tape
  kp.fflag_face = reinterpret_cast<uint8_t*>(b + c->off_ffl);
  kp.theta_left = reinterpret_cast<double*>(b + c->off_thl);
  kp.guard_left = reinterpret_cast<uint32_t*>(b + c->off_gul);
  kp.flag_or = reinterpret_cast<uint32_t*>(b + c->off_flag);
  kp.eflags = reinterpret_cast<uint32_t*>(b + c->off_eflags);
  kp.stats_rows = reinterpret_cast<double*>(b + c->off_srows);
}

// points the context's workspace arrays into the buffer at b
void carve(lwfr_ctx* c, char* b) {
  carve_kp(c, b, c->kp);
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
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches: independent problems of one equation system advanced together, one
// launch per phase (batch.hpp).  Each problem keeps its own lwfr_ctx (for its
// parameters and workspace carving); the batch workspace holds a header (the
// problems' KParams, state offsets, tile tables, per-tile partial maxima, the
// flag word) followed by the problems' workspaces.

struct BatchTable {     // one tile table
  int tile_threads = 0;  // threads per tile (per-point phases) or 256 (faces)
  int ntiles = 0;
  std::vector<int> tinst, tblk, tile_begin;  // tile_begin: [ninst+1]
  // stage tables: tiles grouped by degree, degree N in [deg_begin[N], deg_begin[N+1])
  int deg_begin[6] = {0, 0, 0, 0, 0, 0};
  size_t off_tinst = 0, off_tblk = 0, off_tb = 0;
};

struct BatchLaunch {    // launch shape of one phase
  int tile_threads = 256;
  int grid = 0;          // workgroups; 0: one per tile
  int xcd = 1;
};

struct lwfr_batch {
  std::vector<lwfr_ctx*> inst;
  int equation = 0;
  std::vector<long long> uoff;  // [ninst+1] state offsets (doubles)
  BatchTable tab[2];            // per-point phases with 256 and 128 threads per tile
  BatchTable stab[2];           // stage phase (stage_lanes lanes per point), 256 and 128 threads
  BatchTable ftab;              // face phase
  size_t off_kps = 0, off_uoff = 0, off_part = 0, off_flag = 0, hdr_bytes = 0, ws_bytes = 0;
  std::vector<size_t> off_inst;
  std::vector<char> hdr;        // host image of the header
  BatchLaunch launch[4];        // LWFR_PHASE_*
  void* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  Timing tm;
  hipGraphExec_t graph = nullptr;
};

namespace {

const BatchTable& table_for(const lwfr_batch* b, int phase) {
  if (phase == LWFR_PHASE_FACES) return b->ftab;
  const int v = b->launch[phase].tile_threads == 128 ? 1 : 0;
  return phase == LWFR_PHASE_STAGES ? b->stab[v] : b->tab[v];
}

BatchArgs batch_args(const lwfr_batch* b, const BatchTable& t, const BatchLaunch& l) {
  char* w = static_cast<char*>(b->ws);
  BatchArgs ba;
  ba.kps = reinterpret_cast<const KParams*>(w + b->off_kps);
  ba.uoff = reinterpret_cast<const long long*>(w + b->off_uoff);
  ba.tinst = reinterpret_cast<const int*>(w + t.off_tinst);
  ba.tblk = reinterpret_cast<const int*>(w + t.off_tblk);
  ba.ntiles = t.ntiles;
  ba.xcd = l.xcd;
  ba.part = reinterpret_cast<double*>(w + b->off_part);
  return ba;
}

dim3 batch_grid(const BatchLaunch& l, int ntiles) {
  long long g = l.grid > 0 ? l.grid : ntiles;
  if (l.xcd) g = (g + 7) / 8 * 8;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

// k_bfaces of one problem of a batch (its own KParams and workspace)
template <class Ph>
lwfr_status launch_bfaces(lwfr_ctx* pc, Timing& tm, hipStream_t s, const double* u) {
  const dim3 g((pc->bface_threads + 63) / 64), blk(64);
  TimedLaunch tl(tm, s, KID_BFACES);
  switch (pc->N) {
    case 1: hipLaunchKernelGGL((k_bfaces<Ph, 1>), g, blk, 0, s, pc->kp, u); break;
    case 2: hipLaunchKernelGGL((k_bfaces<Ph, 2>), g, blk, 0, s, pc->kp, u); break;
    case 3: hipLaunchKernelGGL((k_bfaces<Ph, 3>), g, blk, 0, s, pc->kp, u); break;
    default: hipLaunchKernelGGL((k_bfaces<Ph, 4>), g, blk, 0, s, pc->kp, u); break;
  }
  tl.close();
  LWFR_CHECK_LAUNCH("k_bfaces");
  return LWFR_OK;
}

template <class Ph>
lwfr_status batch_phase(lwfr_batch* c, int phase, const double* u_in, double* u_out, double* d_dt) {
  const BatchLaunch& l = c->launch[phase];
  const BatchTable& t = table_for(c, phase);
  const BatchArgs ba = batch_args(c, t, l);
  const dim3 g = batch_grid(l, t.ntiles);
  hipStream_t s = c->stream;
  const bool big = l.tile_threads != 128;
  switch (phase) {
    case LWFR_PHASE_PRE:
      if (big) LWFR_LAUNCH(KID_B_PRE, "kb_pre", (kb_pre<Ph, 256>), g, dim3(256), 0, s, ba, u_in);
      else LWFR_LAUNCH(KID_B_PRE, "kb_pre", (kb_pre<Ph, 128>), g, dim3(128), 0, s, ba, u_in);
      {
        const int* tb = reinterpret_cast<const int*>(static_cast<char*>(c->ws) + t.off_tb);
        LWFR_LAUNCH(KID_B_DT, "kb_dt", kb_dt, dim3((unsigned)c->inst.size()), dim3(256), 0, s, ba, tb, d_dt);
      }
      break;
    case LWFR_PHASE_STAGES:
      // one launch per degree present, over that degree's contiguous tiles
      for (int deg = 1; deg <= 4; ++deg) {
        const int n = t.deg_begin[deg + 1] - t.deg_begin[deg];
        if (n == 0) continue;
        BatchArgs bd = ba;
        bd.tinst += t.deg_begin[deg];
        bd.tblk += t.deg_begin[deg];
        bd.ntiles = n;
        const dim3 gd = batch_grid(l, n);
#define LWFR_KB_STAGES(D)                                                                                   \
  do {                                                                                                      \
    if (big) LWFR_LAUNCH(KID_B_STAGES, "kb_stages", (kb_stages<Ph, D, 256>), gd, dim3(256), 0, s, bd, u_in, u_out); \
    else LWFR_LAUNCH(KID_B_STAGES, "kb_stages", (kb_stages<Ph, D, 128>), gd, dim3(128), 0, s, bd, u_in, u_out);     \
  } while (0)
        switch (deg) {
          case 1: LWFR_KB_STAGES(1); break;
          case 2: LWFR_KB_STAGES(2); break;
          case 3: LWFR_KB_STAGES(3); break;
          default: LWFR_KB_STAGES(4); break;
        }
#undef LWFR_KB_STAGES
      }
      break;
    case LWFR_PHASE_FACES:
      LWFR_LAUNCH(KID_B_FACES, "kb_faces", (kb_faces<Ph>), g, dim3(256), 0, s, ba, u_in);
      // boundary half faces of the problems with non-periodic sides, one launch each
      for (size_t i = 0; i < c->inst.size(); ++i) {
        lwfr_ctx* pc = c->inst[i];
        if (pc->bface_threads == 0) continue;
        const lwfr_status st = launch_bfaces<Ph>(pc, c->tm, s, u_in + c->uoff[i]);
        if (st != LWFR_OK) return st;
      }
      break;
    default:
      if (big) LWFR_LAUNCH(KID_B_UPDATE, "kb_update", (kb_update<Ph, 256>), g, dim3(256), 0, s, ba, u_in, u_out);
      else LWFR_LAUNCH(KID_B_UPDATE, "kb_update", (kb_update<Ph, 128>), g, dim3(128), 0, s, ba, u_in, u_out);
      break;
  }
  return LWFR_OK;
}

lwfr_status batch_phase_any(lwfr_batch* b, int phase, const double* u_in, double* u_out, double* d_dt) {
  switch (b->equation) {
    case LWFR_EQ_SW2D: return batch_phase<SW2D>(b, phase, u_in, u_out, d_dt);
  }
  return fail(LWFR_E_UNSUPPORTED, "batches support the 2-D shallow water system");
}

lwfr_status batch_step(lwfr_batch* b, const double* u_in, double* u_out, double* d_dt) {
  for (int ph = 0; ph < 4; ++ph) {
    lwfr_status st = batch_phase_any(b, ph, u_in, u_out, d_dt);
    if (st != LWFR_OK) return st;
  }
  return LWFR_OK;
}

// time of one launch of `phase` with launch shape l (ms), after `before` runs
// the untimed prerequisites; minimum over reps
template <class F>
lwfr_status time_phase(lwfr_batch* b, int phase, const BatchLaunch& l, const double* u_in, double* u_out, int reps,
                       F&& before, hipEvent_t e0, hipEvent_t e1, float& best) {
  const BatchLaunch keep = b->launch[phase];
  b->launch[phase] = l;
  best = 1e30f;
  lwfr_status st = LWFR_OK;
  for (int r = 0; r < reps && st == LWFR_OK; ++r) {
    st = before();
    if (st != LWFR_OK) break;
    (void)hipEventRecord(e0, b->stream);
    st = batch_phase_any(b, phase, u_in, u_out, nullptr);
    (void)hipEventRecord(e1, b->stream);
    hipError_t err = hipEventSynchronize(e1);
    if (err != hipSuccess) { st = fail(LWFR_E_HIP, std::string("autotune: ") + hipGetErrorString(err)); break; }
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, e0, e1);
    best = t < best ? t : best;
  }
  b->launch[phase] = keep;
  return st;
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

lwfr_status lwfr_cfl_number_for(int32_t degree, uint32_t cfg_flags, double* cfl) {
  if (!cfl) return fail(LWFR_E_INVALID_ARG, "cfl is null");
  if (degree < 1 || degree > 4) return fail(LWFR_E_UNSUPPORTED, "degree must be 1..4");
  const bool gll = (cfg_flags & LWFR_CFG_GLL) != 0;
  if (cfg_flags & LWFR_CFG_IMEX_HT112) *cfl = fourier_cfl_imex<ImexHT>(degree, gll);
  else if (cfg_flags & LWFR_CFG_IMEX_SSP3) *cfl = fourier_cfl_imex<ImexSSP3>(degree, gll);
  else *cfl = fourier_cfl(degree, gll);
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
  bool nonperiodic = false, dirichlet = false;
  for (int d = 0; d < info.DIM; ++d) {
    const int32_t* k = cfg->bc + 2 * d;
    for (int sd = 0; sd < 2; ++sd) {
      if (k[sd] < LWFR_BC_PERIODIC || k[sd] > LWFR_BC_DIRICHLET)
        return fail(LWFR_E_INVALID_ARG, "bc must be a lwfr_boundary value");
      if (k[sd] == LWFR_BC_WALL && cfg->equation != LWFR_EQ_SW1D && cfg->equation != LWFR_EQ_SW2D)
        return fail(LWFR_E_INVALID_ARG, "wall sides are defined for the shallow water systems");
      nonperiodic = nonperiodic || k[sd] != LWFR_BC_PERIODIC;
      dirichlet = dirichlet || k[sd] == LWFR_BC_DIRICHLET;
    }
    if ((k[0] == LWFR_BC_PERIODIC) != (k[1] == LWFR_BC_PERIODIC))
      return fail(LWFR_E_INVALID_ARG, "a direction is periodic on both sides or on neither");
  }
  if (nonperiodic && (cfg->flags & LWFR_CFG_ADJOINT))
    return fail(LWFR_E_UNSUPPORTED, "the adjoint step needs a periodic mesh");
  {
    const uint32_t imex = cfg->flags & (LWFR_CFG_IMEX_HT112 | LWFR_CFG_IMEX_SSP3);
    if (imex == (LWFR_CFG_IMEX_HT112 | LWFR_CFG_IMEX_SSP3))
      return fail(LWFR_E_INVALID_ARG, "at most one IMEX pair");
    if (cfg->equation == LWFR_EQ_JINXIN1D) {
      if (!imex) return fail(LWFR_E_INVALID_ARG, "a system with a source needs an IMEX pair (LWFR_CFG_IMEX_*)");
      if (!(cfg->source[0] > 0.0) || !(cfg->source[1] > 0.0) || !std::isfinite(cfg->source[2]) ||
          !std::isfinite(cfg->source[3]))
        return fail(LWFR_E_INVALID_ARG, "Jin-Xin needs a > 0, eps > 0 and finite l, q");
      if (cfg->flags & LWFR_CFG_ADJOINT) return fail(LWFR_E_UNSUPPORTED, "no adjoint for systems with a source");
    } else if (imex) {
      return fail(LWFR_E_UNSUPPORTED, "IMEX pairs are for systems with a source");
    }
    if ((cfg->flags & LWFR_CFG_ALW) && (imex || (cfg->flags & LWFR_CFG_ADJOINT)))
      return fail(LWFR_E_UNSUPPORTED, "the approximate Lax-Wendroff averages have no IMEX or adjoint form");
  }

  lwfr_ctx* c = new lwfr_ctx();
  c->cfg = *cfg;
  c->M = info.M; c->DIM = info.DIM; c->K = info.K;
  c->N = cfg->degree; c->n1 = c->N + 1;
  c->P = info.DIM == 1 ? c->n1 : c->n1 * c->n1;
  c->NFP = info.DIM == 1 ? 1 : c->n1;
  c->E = cfg->nelem[0] * ny;
  {
    const int epb = epb_runtime(c->N, c->DIM, c->M);
    c->nblk_pre = (c->E + epb - 1) / epb;  // k_pre and the update: epb elements per block
    c->nblk_ch = (c->E + 255) / 256;       // k_ch: one thread per element
    c->nblk_dt = (c->nblk_pre + 1023) / 1024;  // k_dt's first level: 1024 partials per block
  }
  const bool gll = (cfg->flags & LWFR_CFG_GLL) != 0;
  c->rd = make_refdata(c->N, gll);
  if (cfg->cfl_number > 0.0) c->cfl = cfg->cfl_number;
  else if (cfg->flags & LWFR_CFG_IMEX_HT112) c->cfl = fourier_cfl_imex<ImexHT>(c->N, gll);
  else if (cfg->flags & LWFR_CFG_IMEX_SSP3) c->cfl = fourier_cfl_imex<ImexSSP3>(c->N, gll);
  else c->cfl = fourier_cfl(c->N, gll);

  KParams& kp = c->kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.nx = cfg->nelem[0]; kp.ny = ny; kp.E = c->E; kp.nblk_pre = c->nblk_pre; kp.nblk_ch = c->nblk_ch;
  kp.nblk_dt = c->nblk_dt;
  kp.N = c->N;
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
  if (cfg->equation == LWFR_EQ_JINXIN1D) {
    kp.ra = cfg->source[0]; kp.reps = cfg->source[1]; kp.rl = cfg->source[2]; kp.rq = cfg->source[3];
  }
  kp.blending = cfg->blending;
  // F^+[0] from F^-[0]: only the two-lane GLM-MHD face kernel leaves it out, and
  // only where every face slot holds one face (all sides periodic)
  kp.fp0_alias = cfg->equation == LWFR_EQ_GLMMHD2D && cfg->bc[0] == LWFR_BC_PERIODIC &&
                         cfg->bc[1] == LWFR_BC_PERIODIC && cfg->bc[2] == LWFR_BC_PERIODIC &&
                         cfg->bc[3] == LWFR_BC_PERIODIC
                     ? 1
                     : 0;
  kp.alpha_max = cfg->alpha_max; kp.alpha_min = cfg->alpha_min; kp.alpha_force = cfg->alpha_force;
  kp.ind_T = 0.5 * std::pow(10.0, -1.8 * std::pow(c->N + 1.0, 0.25));
  kp.ind_s = std::log(9999.0);
  kp.cs_cfl = cfg->cfl_safety * c->cfl;
  kp.ch_in = -1.0;
  for (int d = 0; d < 2; ++d)
    for (int sd = 0; sd < 2; ++sd) kp.bc[d][sd] = d < info.DIM ? cfg->bc[2 * d + sd] : 0;
  kp.ghost = nullptr;
  c->bface_threads = bface_threads(info.DIM, kp.nx, kp.ny, c->NFP, kp.bc);
  c->dirichlet = dirichlet;
  (void)nonperiodic;

  // workspace carving
  const size_t nfpt = (size_t)c->DIM * c->E * c->NFP;  // face points over all directions
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  c->off_scal = take(8 * sizeof(double));
  c->off_part = take((size_t)c->nblk_pre * sizeof(double));
  c->off_part2 = take((size_t)c->nblk_ch * sizeof(double));
  c->off_part3 = take((size_t)c->nblk_dt * sizeof(double));
  c->off_speeds = take((size_t)c->E * 2 * c->DIM * sizeof(double));
  c->off_araw = take((size_t)c->E * sizeof(double));
  c->off_alpha = take((size_t)c->E * sizeof(double));
  c->off_thel = take((size_t)c->E * sizeof(double));
  c->off_Ftr = take(nfpt * 2 * c->M * sizeof(double));
  c->off_Utr = take(nfpt * 2 * c->M * sizeof(double));
  c->adjoint = (cfg->flags & LWFR_CFG_ADJOINT) != 0;
  c->off_Fm = take(nfpt * c->M * sizeof(double));
  c->off_Fp = take(nfpt * c->M * sizeof(double));
  // the correction jumps D^± of the systems that do not fold the correction
  // into the volume residual (fold_correction: 2-D with nine variables)
  const bool fold = c->DIM == 2 && c->M >= 8;
  c->off_Dm = fold ? 0 : take(nfpt * c->M * sizeof(double));
  c->off_Dp = fold ? 0 : take(nfpt * c->M * sizeof(double));
  c->off_ffl = take(nfpt * sizeof(uint8_t));
  {
    const size_t nbl = ((size_t)ny + (info.DIM == 2 ? cfg->nelem[0] : 0)) * c->NFP;  // left boundary face points
    c->off_thl = take(nbl * sizeof(double));
    c->off_gul = take(nbl * sizeof(uint32_t));
  }
  c->off_flag = take(sizeof(uint32_t));
  c->nblk_stats = (c->E + 255) / 256;
  c->off_eflags = take((size_t)c->E * sizeof(uint32_t));
  c->off_srows = take((size_t)c->nblk_stats * kStatsRow * sizeof(double));
  c->fwd_bytes = off;  // the forward step's part of the workspace (the adjoint's arrays follow)
  if (c->adjoint) {
    const size_t nst = (size_t)c->M * c->E * c->P * sizeof(double);
    c->off_uscr = take(nst);
    c->off_thf = take(nfpt * sizeof(double));  // Algorithm 1 thetas of the recomputed step (no tape)
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

lwfr_status lwfr_boundary_data_size(const lwfr_ctx* c, size_t* n) {
  if (!c || !n) return fail(LWFR_E_INVALID_ARG, "null argument");
  const size_t nb0 = (size_t)c->kp.ny * c->NFP, nb1 = c->DIM == 2 ? (size_t)c->kp.nx * c->NFP : 0;
  *n = 2 * 3 * (size_t)c->M * (nb0 + nb1);
  return LWFR_OK;
}

lwfr_status lwfr_set_boundary_data(lwfr_ctx* c, const double* d_ghost) {
  if (!c || !d_ghost) return fail(LWFR_E_INVALID_ARG, "null argument");
  if (!c->dirichlet) return fail(LWFR_E_STATE, "the context has no Dirichlet side");
  c->kp.ghost = d_ghost;
  return LWFR_OK;
}

lwfr_status lwfr_bind(lwfr_ctx* c, void* d_ws, size_t bytes, void* stream) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!d_ws) return fail(LWFR_E_WORKSPACE, "workspace is null");
  if (bytes < c->ws_bytes) return fail(LWFR_E_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(LWFR_E_WORKSPACE, "workspace not 256-byte aligned");
  c->ws = d_ws;
  c->stream = static_cast<hipStream_t>(stream);
  carve(c, static_cast<char*>(d_ws));
  const KParams& kp = c->kp;
  hipError_t err = hipMemsetAsync(kp.flag_or, 0, sizeof(uint32_t), c->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(err));
  c->bound = true;
  return LWFR_OK;
}

lwfr_status lwfr_step(lwfr_ctx* c, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                      double* d_alpha, uint32_t* d_flags, lwfr_stats* d_stats) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!d_u_in || !d_u_out) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_u_in, d_u_out, bytes)) return fail(LWFR_E_INVALID_ARG, "u_out aliases u_in");
  if (!std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt is not finite");
  if (lwfr_status st = dirichlet_ready(c, dt); st != LWFR_OK) return st;
  if (reinterpret_cast<uintptr_t>(d_stats) % 8 != 0) return fail(LWFR_E_INVALID_ARG, "d_stats not 8-byte aligned");
  KParams kp = c->kp;
  kp.dt_in = dt > 0.0 ? dt : 0.0;
  kp.ch_in = -1.0;
  return dispatch_step(c, kp, d_u_in, d_u_out, d_dt_ch, d_alpha, d_flags, d_stats);
}

}  // extern "C"

// The workspace of lwfr_step_noalloc: a static device array, one per GPU, held
// until the process ends.  Host code never passes its name to a kernel (on the
// host the name is only a stand-in); it uses the device address resolved for
// the current device by hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[LWFR_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (resolved once per device)
lwfr_status scratch_address(void** out) {
  int dev = -1;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(err));
  if (dev < 0 || dev >= kMaxDevices) return fail(LWFR_E_UNSUPPORTED, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !p)
      return fail(LWFR_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(err));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LWFR_OK;
}

}  // namespace

extern "C" {

lwfr_status lwfr_step_noalloc(lwfr_ctx* c, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                              uint32_t* d_flags, void* hip_stream) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!d_u_in || !d_u_out) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_u_in, d_u_out, bytes)) return fail(LWFR_E_INVALID_ARG, "u_out aliases u_in");
  if (!std::isfinite(dt)) return fail(LWFR_E_INVALID_ARG, "dt is not finite");
  if (c->fwd_bytes > (size_t)LWFR_STATIC_SCRATCH_BYTES)
    return fail(LWFR_E_WORKSPACE, "the step needs " + std::to_string(c->fwd_bytes) +
                                      " bytes of workspace, more than the static scratch of " +
                                      std::to_string((size_t)LWFR_STATIC_SCRATCH_BYTES) + " bytes");
  if (lwfr_status st = dirichlet_ready(c, dt); st != LWFR_OK) return st;
  void* base = nullptr;
  if (lwfr_status st = scratch_address(&base); st != LWFR_OK) return st;
  KParams kp = c->kp;
  carve_kp(c, static_cast<char*>(base), kp);
  kp.dt_in = dt > 0.0 ? dt : 0.0;
  kp.ch_in = -1.0;
  // the launches go to the caller's stream; the context's bound stream is restored after
  const hipStream_t bound = c->stream;
  c->stream = static_cast<hipStream_t>(hip_stream);
  const lwfr_status st = dispatch_step(c, kp, d_u_in, d_u_out, d_dt_ch, nullptr, d_flags);
  c->stream = bound;
  return st;
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
  if (lwfr_status st = dirichlet_ready(c, dt); st != LWFR_OK) return st;
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
  if (lwfr_status st = dirichlet_ready(c, dt); st != LWFR_OK) return st;
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
  if (lwfr_status st = dirichlet_ready(c, dt); st != LWFR_OK) return st;
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
    kp.theta_face = reinterpret_cast<double*>(static_cast<char*>(c->ws) + c->off_thf);
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
  return timing_begin(c->tm, max_launches);
}

lwfr_status lwfr_timing_end(lwfr_ctx* c, double* ms, uint32_t* launches) {
  if (!c || !ms || !launches) return fail(LWFR_E_INVALID_ARG, "null argument");
  return timing_end(c->tm, c->stream, ms, launches);
}

lwfr_status lwfr_graph_capture(lwfr_ctx* c, double* d_u_a, double* d_u_b, int32_t nsteps, double* d_dt_ch_hist) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->bound) return fail(LWFR_E_STATE, "lwfr_bind has not been called");
  if (!d_u_a || !d_u_b) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  if (nsteps < 1 || nsteps > 100000) return fail(LWFR_E_INVALID_ARG, "nsteps must be in 1..100000");
  const size_t bytes = (size_t)c->M * c->E * c->P * sizeof(double);
  if (ranges_overlap(d_u_a, d_u_b, bytes)) return fail(LWFR_E_INVALID_ARG, "u_a and u_b overlap");
  if (c->dirichlet) return fail(LWFR_E_UNSUPPORTED, "graph capture of a context with a Dirichlet side");
  KParams kp = c->kp;
  kp.dt_in = 0.0;
  kp.ch_in = -1.0;
  // each step after the first starts from the previous one's result: the
  // previous update forms its element data (the same values k_pre would)
  return capture(c->stream, c->tm, c->graph, nsteps, [&](int k) {
    const double* in = (k & 1) ? d_u_b : d_u_a;
    double* out = (k & 1) ? d_u_a : d_u_b;
    const int chain = (k > 0 ? kChainFromPrev : 0) | (k + 1 < nsteps ? kChainToNext : 0);
    return dispatch_step(c, kp, in, out, d_dt_ch_hist ? d_dt_ch_hist + 2 * (size_t)k : nullptr, nullptr, nullptr,
                         nullptr, chain);
  });
}

lwfr_status lwfr_graph_launch(lwfr_ctx* c) {
  if (!c) return fail(LWFR_E_INVALID_ARG, "null context");
  if (!c->graph) return fail(LWFR_E_STATE, "no captured graph");
  hipError_t err = hipGraphLaunch(c->graph, c->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(err));
  return LWFR_OK;
}

lwfr_status lwfr_destroy(lwfr_ctx* c) {
  if (c) {
    for (hipEvent_t e : c->tm.ev) (void)hipEventDestroy(e);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
  }
  delete c;
  return LWFR_OK;
}

// ---------------------------------------------------------------------------
// batches

lwfr_status lwfr_batch_destroy(lwfr_batch* b) {
  if (b) {
    for (lwfr_ctx* c : b->inst) lwfr_destroy(c);
    for (hipEvent_t e : b->tm.ev) (void)hipEventDestroy(e);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
  }
  delete b;
  return LWFR_OK;
}

lwfr_status lwfr_batch_init(const lwfr_config* cfgs, int32_t count, lwfr_batch** out) {
  if (!cfgs || !out) return fail(LWFR_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (count < 1 || count > 65536) return fail(LWFR_E_INVALID_ARG, "count must be in 1..65536");
  lwfr_batch* b = new lwfr_batch();
  b->equation = cfgs[0].equation;
  if (b->equation != LWFR_EQ_SW2D) {
    delete b;
    return fail(LWFR_E_UNSUPPORTED, "batches support the 2-D shallow water system");
  }
  for (int i = 0; i < count; ++i) {
    if (cfgs[i].equation != b->equation) {
      lwfr_batch_destroy(b);
      return fail(LWFR_E_INVALID_ARG, "all problems of a batch must use the same equation system");
    }
    if (cfgs[i].flags & LWFR_CFG_ADJOINT) {
      lwfr_batch_destroy(b);
      return fail(LWFR_E_UNSUPPORTED, "batches have no adjoint");
    }
    if (cfgs[i].flags & LWFR_CFG_ALW) {
      lwfr_batch_destroy(b);
      return fail(LWFR_E_UNSUPPORTED, "batches use the cRK stages");
    }
    for (int k = 0; k < 4; ++k)
      if (cfgs[i].bc[k] == LWFR_BC_DIRICHLET) {
        lwfr_batch_destroy(b);
        return fail(LWFR_E_UNSUPPORTED, "batches have no Dirichlet sides");
      }
    lwfr_ctx* c = nullptr;
    lwfr_status st = lwfr_init(&cfgs[i], &c);
    if (st != LWFR_OK) {
      const std::string msg = "problem " + std::to_string(i) + ": " + g_err;
      lwfr_batch_destroy(b);
      return fail(st, msg);
    }
    b->inst.push_back(c);
  }
  // state offsets
  b->uoff.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    const lwfr_ctx* c = b->inst[i];
    b->uoff[i + 1] = b->uoff[i] + (long long)c->M * c->E * c->P;
  }
  // tile tables
  const int tt[2] = {256, 128};
  for (int v = 0; v < 4; ++v) {
    BatchTable& t = v < 2 ? b->tab[v] : b->stab[v - 2];
    t.tile_threads = tt[v & 1];
    t.tile_begin.assign(count + 1, 0);
    // the stage tables list the tiles of each degree together (one launch per
    // degree); the other tables keep the problems in order
    for (int deg = 1; deg <= 4; ++deg) {
      t.deg_begin[deg] = (int)t.tinst.size();
      for (int i = 0; i < count; ++i) {
        const lwfr_ctx* c = b->inst[i];
        if (v >= 2 && c->N != deg) continue;
        if (v < 2 && deg != 1) continue;
        const int lanes = v < 2 ? 1 : (c->DIM == 2 && c->M >= 8 ? 2 : 1);  // stage_lanes
        const int epb = tt[v & 1] / (lanes * c->P);
        const int nb = (c->E + epb - 1) / epb;
        for (int k = 0; k < nb; ++k) { t.tinst.push_back(i); t.tblk.push_back(k); }
        t.tile_begin[i + 1] = (int)t.tinst.size();
      }
    }
    t.deg_begin[5] = (int)t.tinst.size();
    t.ntiles = (int)t.tinst.size();
  }
  {
    BatchTable& t = b->ftab;
    t.tile_threads = 256;
    t.tile_begin.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) {
      const lwfr_ctx* c = b->inst[i];
      const long long nfp = (long long)c->DIM * c->E * c->NFP;
      const int nb = (int)((nfp + 255) / 256);
      for (int k = 0; k < nb; ++k) { t.tinst.push_back(i); t.tblk.push_back(k); }
      t.tile_begin[i + 1] = (int)t.tinst.size();
    }
    t.ntiles = (int)t.tinst.size();
  }
  // workspace: header, then the problems' workspaces
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  b->off_kps = take(count * sizeof(KParams));
  b->off_uoff = take(count * sizeof(long long));
  for (BatchTable* t : {&b->tab[0], &b->tab[1], &b->stab[0], &b->stab[1], &b->ftab}) {
    t->off_tinst = take(t->ntiles * sizeof(int));
    t->off_tblk = take(t->ntiles * sizeof(int));
    t->off_tb = take((count + 1) * sizeof(int));
  }
  const int maxt = b->tab[0].ntiles > b->tab[1].ntiles ? b->tab[0].ntiles : b->tab[1].ntiles;
  b->off_part = take(maxt * sizeof(double));
  b->off_flag = take(sizeof(uint32_t));
  b->hdr_bytes = off;
  for (int i = 0; i < count; ++i) b->off_inst.push_back(take(b->inst[i]->ws_bytes));
  b->ws_bytes = off;
  for (int ph = 0; ph < 4; ++ph) b->launch[ph] = BatchLaunch();
  *out = b;
  return LWFR_OK;
}

lwfr_status lwfr_batch_workspace_bytes(const lwfr_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(LWFR_E_INVALID_ARG, "null argument");
  *bytes = b->ws_bytes;
  return LWFR_OK;
}

lwfr_status lwfr_batch_state_offsets(const lwfr_batch* b, int64_t* offsets) {
  if (!b || !offsets) return fail(LWFR_E_INVALID_ARG, "null argument");
  for (size_t i = 0; i < b->uoff.size(); ++i) offsets[i] = b->uoff[i];
  return LWFR_OK;
}

lwfr_status lwfr_batch_problem(lwfr_batch* b, int32_t i, lwfr_ctx** ctx) {
  if (!b || !ctx) return fail(LWFR_E_INVALID_ARG, "null argument");
  if (i < 0 || i >= (int)b->inst.size()) return fail(LWFR_E_INVALID_ARG, "problem index out of range");
  *ctx = b->inst[i];
  return LWFR_OK;
}

lwfr_status lwfr_batch_bind(lwfr_batch* b, void* d_ws, size_t bytes, void* stream) {
  if (!b) return fail(LWFR_E_INVALID_ARG, "null batch");
  if (!d_ws) return fail(LWFR_E_WORKSPACE, "workspace is null");
  if (bytes < b->ws_bytes) return fail(LWFR_E_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(LWFR_E_WORKSPACE, "workspace not 256-byte aligned");
  b->ws = d_ws;
  b->stream = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(d_ws);
  const int count = (int)b->inst.size();
  b->hdr.assign(b->hdr_bytes, 0);
  char* h = b->hdr.data();
  uint32_t* flag = reinterpret_cast<uint32_t*>(w + b->off_flag);
  for (int i = 0; i < count; ++i) {
    lwfr_ctx* c = b->inst[i];
    c->ws = w + b->off_inst[i];
    c->stream = b->stream;
    carve(c, static_cast<char*>(c->ws));
    c->kp.flag_or = flag;  // one flag word for the whole batch
    c->kp.dt_in = 0.0;
    c->kp.ch_in = -1.0;
    c->bound = true;
    std::memcpy(h + b->off_kps + i * sizeof(KParams), &c->kp, sizeof(KParams));
    const long long o = b->uoff[i];
    std::memcpy(h + b->off_uoff + i * sizeof(long long), &o, sizeof(long long));
  }
  for (const BatchTable* t : {&b->tab[0], &b->tab[1], &b->stab[0], &b->stab[1], &b->ftab}) {
    std::memcpy(h + t->off_tinst, t->tinst.data(), t->ntiles * sizeof(int));
    std::memcpy(h + t->off_tblk, t->tblk.data(), t->ntiles * sizeof(int));
    std::memcpy(h + t->off_tb, t->tile_begin.data(), (count + 1) * sizeof(int));
  }
  hipError_t err = hipMemcpyAsync(w, h, b->hdr_bytes, hipMemcpyHostToDevice, b->stream);
  if (err == hipSuccess) err = hipMemsetAsync(flag, 0, sizeof(uint32_t), b->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(b->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("lwfr_batch_bind: ") + hipGetErrorString(err));
  b->bound = true;
  return LWFR_OK;
}

static lwfr_status batch_check(lwfr_batch* b, const double* u_in, const double* u_out) {
  if (!b) return fail(LWFR_E_INVALID_ARG, "null batch");
  if (!b->bound) return fail(LWFR_E_STATE, "lwfr_batch_bind has not been called");
  if (!u_in || !u_out) return fail(LWFR_E_INVALID_ARG, "null state pointer");
  if (ranges_overlap(u_in, u_out, (size_t)b->uoff.back() * sizeof(double)))
    return fail(LWFR_E_INVALID_ARG, "u_out aliases u_in");
  return LWFR_OK;
}

lwfr_status lwfr_batch_step(lwfr_batch* b, const double* d_u_in, double* d_u_out, double* d_dt) {
  lwfr_status st = batch_check(b, d_u_in, d_u_out);
  if (st != LWFR_OK) return st;
  return batch_step(b, d_u_in, d_u_out, d_dt);
}

lwfr_status lwfr_batch_set_launch(lwfr_batch* b, int32_t phase, int32_t tile_threads, int32_t grid, int32_t xcd) {
  if (!b) return fail(LWFR_E_INVALID_ARG, "null batch");
  if (phase < 0 || phase > 3) return fail(LWFR_E_INVALID_ARG, "phase must be 0..3");
  if (phase == LWFR_PHASE_FACES ? tile_threads != 256 : (tile_threads != 256 && tile_threads != 128))
    return fail(LWFR_E_INVALID_ARG, "tile_threads must be 256 or 128 (faces: 256)");
  if (grid < 0 || grid > (1 << 24)) return fail(LWFR_E_INVALID_ARG, "grid out of range");
  if (xcd < 0 || xcd > 4) return fail(LWFR_E_INVALID_ARG, "xcd must be 0..4");
  b->launch[phase] = BatchLaunch{tile_threads, grid, xcd};
  return LWFR_OK;
}

lwfr_status lwfr_batch_get_launch(const lwfr_batch* b, int32_t phase, int32_t* tile_threads, int32_t* grid,
                                  int32_t* xcd) {
  if (!b || !tile_threads || !grid || !xcd) return fail(LWFR_E_INVALID_ARG, "null argument");
  if (phase < 0 || phase > 3) return fail(LWFR_E_INVALID_ARG, "phase must be 0..3");
  *tile_threads = b->launch[phase].tile_threads;
  *grid = b->launch[phase].grid;
  *xcd = b->launch[phase].xcd;
  return LWFR_OK;
}

lwfr_status lwfr_batch_autotune(lwfr_batch* b, const double* d_u_in, double* d_u_out, int32_t reps) {
  lwfr_status st = batch_check(b, d_u_in, d_u_out);
  if (st != LWFR_OK) return st;
  if (reps < 1 || reps > 100) return fail(LWFR_E_INVALID_ARG, "reps must be in 1..100");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(LWFR_E_HIP, "autotune: hipEventCreate failed");
  }
  const bool timing = b->tm.on;
  b->tm.on = false;
  st = batch_step(b, d_u_in, d_u_out, nullptr);  // every phase's inputs in place
  const int grids[5] = {0, 1024, 2048, 4096, 8192};
  auto none = [] { return LWFR_OK; };
  auto stages_first = [&] { return batch_phase_any(b, LWFR_PHASE_STAGES, d_u_in, d_u_out, nullptr); };
  for (int ph = 0; ph < 4 && st == LWFR_OK; ++ph) {
    BatchLaunch best = b->launch[ph];
    float tbest = 1e30f;
    for (int tt : {256, 128}) {
      if (ph == LWFR_PHASE_FACES && tt != 256) continue;
      for (int g : grids)
        for (int x : {0, 1, 2, 3, 4}) {
          const BatchLaunch l{tt, g, x};
          float t = 0.0f;
          if (ph == LWFR_PHASE_UPDATE) st = time_phase(b, ph, l, d_u_in, d_u_out, reps, stages_first, e0, e1, t);
          else st = time_phase(b, ph, l, d_u_in, d_u_out, reps, none, e0, e1, t);
          if (st != LWFR_OK) break;
          if (t < tbest) { tbest = t; best = l; }
        }
      if (st != LWFR_OK) break;
    }
    b->launch[ph] = best;
    // the phase's outputs with the chosen shape, for the phases after it
    if (st == LWFR_OK && ph != LWFR_PHASE_UPDATE) st = batch_phase_any(b, ph, d_u_in, d_u_out, nullptr);
  }
  if (st == LWFR_OK) st = batch_step(b, d_u_in, d_u_out, nullptr);
  hipError_t err = hipStreamSynchronize(b->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tm.on = timing;
  if (st == LWFR_OK && err != hipSuccess) st = fail(LWFR_E_HIP, std::string("autotune: ") + hipGetErrorString(err));
  return st;
}

lwfr_status lwfr_batch_graph_capture(lwfr_batch* b, double* d_u_a, double* d_u_b, int32_t nsteps,
                                     double* d_dt_hist) {
  lwfr_status st = batch_check(b, d_u_a, d_u_b);
  if (st != LWFR_OK) return st;
  if (nsteps < 1 || nsteps > 100000) return fail(LWFR_E_INVALID_ARG, "nsteps must be in 1..100000");
  const size_t count = b->inst.size();
  return capture(b->stream, b->tm, b->graph, nsteps, [&](int k) {
    const double* in = (k & 1) ? d_u_b : d_u_a;
    double* out = (k & 1) ? d_u_a : d_u_b;
    return batch_step(b, in, out, d_dt_hist ? d_dt_hist + count * (size_t)k : nullptr);
  });
}

lwfr_status lwfr_batch_graph_launch(lwfr_batch* b) {
  if (!b) return fail(LWFR_E_INVALID_ARG, "null batch");
  if (!b->graph) return fail(LWFR_E_STATE, "no captured graph");
  hipError_t err = hipGraphLaunch(b->graph, b->stream);
  if (err != hipSuccess) return fail(LWFR_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(err));
  return LWFR_OK;
}

lwfr_status lwfr_batch_query(lwfr_batch* b, uint32_t* flags_or) {
  if (!b) return fail(LWFR_E_INVALID_ARG, "null batch");
  if (!b->bound) return fail(LWFR_E_STATE, "lwfr_batch_bind has not been called");
  return lwfr_query(b->inst[0], flags_or);
}

lwfr_status lwfr_batch_timing_begin(lwfr_batch* b, int32_t max_launches) {
  if (!b) return fail(LWFR_E_INVALID_ARG, "null batch");
  if (!b->bound) return fail(LWFR_E_STATE, "lwfr_batch_bind has not been called");
  return timing_begin(b->tm, max_launches);
}

lwfr_status lwfr_batch_timing_end(lwfr_batch* b, double* ms, uint32_t* launches) {
  if (!b || !ms || !launches) return fail(LWFR_E_INVALID_ARG, "null argument");
  return timing_end(b->tm, b->stream, ms, launches);
}

}  // extern "C"
