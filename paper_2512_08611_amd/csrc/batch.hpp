// Batched kernels: many independent problems of one equation system, of any
// mix of sizes and degrees 1..4, advanced by one launch per phase of the step.
//
// The problems' states are concatenated, each in its own [var][elem][node]
// layout at an offset.  A tile table maps every tile (one block of elements of
// the per-point phases, or 256 face points of the face phase) to its problem
// and to the block index within that problem; the kernels run exactly the same
// device bodies as the single-problem kernels, selected by the problem's degree.
//
// Launches are persistent: a grid of G workgroups walks the tile table.  With
// G a multiple of 8 and an XCD option set, workgroup b (dispatched to XCD
// b mod 8) takes its tiles from the tiles of XCD b mod 8, so that the tiles one
// XCD works on are neighbours in memory and their face neighbours are mostly
// in the same L2: option 1 gives each XCD a contiguous eighth of the table;
// options 2, 3 and 4 deal the table out in chunks of 16, 64 or 256 tiles, chunk
// c to XCD c mod 8 (neighbours within a chunk, the problems of every degree
// spread over all XCDs).  The time step of each problem comes from its own
// reduction (kb_dt, one workgroup per problem).
#pragma once
#include "kernels.hpp"

namespace lwfr {

struct BatchArgs {
  const KParams* kps;     // [ninst] per-problem parameters (device memory)
  const long long* uoff;  // [ninst] offset of each problem's state, in doubles
  const int* tinst;       // [ntiles] problem of each tile
  const int* tblk;        // [ntiles] block index of the tile within its problem
  int ntiles;
  int xcd;                // 0: none; 1: XCD-contiguous eighths; 2..4: chunks of 16 << 2(xcd - 2) tiles per XCD
  double* part;           // [ntiles] per-tile maximum of Lambda_e (pre phase)
};

// The workgroup's walk over the tile table: for k = k0; k < k1; k += step, tile
// tile_at(k) (-1: the walk is over)
__device__ inline void tile_range(int ntiles, int xcd, int& k0, int& k1, int& step) {
  const int G = gridDim.x;
  if (xcd == 1 && (G & 7) == 0) {
    const int x = blockIdx.x & 7, w = blockIdx.x >> 3, per = (ntiles + 7) >> 3;
    k0 = x * per + w;
    k1 = min(ntiles, (x + 1) * per);
    step = G >> 3;
  } else if (xcd >= 2 && (G & 7) == 0) {
    k0 = blockIdx.x >> 3;
    k1 = ntiles;  // the XCD's k-th tile lies at or past k
    step = G >> 3;
  } else {
    k0 = blockIdx.x;
    k1 = ntiles;
    step = G;
  }
}
__device__ inline int tile_at(int k, int ntiles, int xcd) {
  if (xcd >= 2 && (gridDim.x & 7) == 0) {
    // the k-th tile of XCD x: chunk x + 8 (k / C), position k mod C in it
    const int lc = 4 + 2 * (xcd - 2), C = 1 << lc, x = blockIdx.x & 7;
    const int t = ((x + 8 * (k >> lc)) << lc) + (k & (C - 1));
    return t < ntiles ? t : -1;
  }
  return k;
}

// elements per tile of the batched per-point phases with NT threads
template <int N, int NT>
constexpr int batch_epb(int DIM) {
  return NT / ipow(N + 1, DIM);
}

// elements per tile of the batched stage phase (two lanes per point in 2-D)
template <class Ph, int N, int NT>
constexpr int batch_epb_stages() {
  return NT / (stage_lanes<Ph>() * ipow(N + 1, Ph::DIM));
}

template <template <class, int, int> class Lds, class Ph, int NT>
union LdsByDegree {
  Lds<Ph, 1, NT> n1;
  Lds<Ph, 2, NT> n2;
  Lds<Ph, 3, NT> n3;
  Lds<Ph, 4, NT> n4;
};

template <class Ph, int NT>
__global__ void __launch_bounds__(NT) kb_pre(const BatchArgs ba, const double* __restrict__ u) {
  constexpr int DIM = Ph::DIM;
  __shared__ LdsByDegree<PreLds, Ph, NT> L;
  int k0, k1, step;
  tile_range(ba.ntiles, ba.xcd, k0, k1, step);
  for (int k = k0; k < k1; k += step) {
    const int t = tile_at(k, ba.ntiles, ba.xcd);
    if (t < 0) break;
    const int inst = ba.tinst[t], blk = ba.tblk[t];
    const KParams& kp = ba.kps[inst];
    const double* un = u + ba.uoff[inst];
    double* po = ba.part + t;
    switch (kp.N) {
      case 1: pre_body<Ph, 1, batch_epb<1, NT>(DIM), NT>(kp, L.n1, un, blk, po); break;
      case 2: pre_body<Ph, 2, batch_epb<2, NT>(DIM), NT>(kp, L.n2, un, blk, po); break;
      case 3: pre_body<Ph, 3, batch_epb<3, NT>(DIM), NT>(kp, L.n3, un, blk, po); break;
      default: pre_body<Ph, 4, batch_epb<4, NT>(DIM), NT>(kp, L.n4, un, blk, po); break;
    }
    __syncthreads();
  }
}

// one workgroup per problem: Lambda = max over the problem's tiles, dt
// (eq. time.step.2d) unless the problem's dt is fixed
__global__ void __launch_bounds__(256) kb_dt(const BatchArgs ba, const int* __restrict__ tile_begin,
                                             double* d_dt) {
  __shared__ double s_w[4];
  const int inst = blockIdx.x;
  const KParams& kp = ba.kps[inst];
  double m = 0.0;
  for (int i = tile_begin[inst] + threadIdx.x; i < tile_begin[inst + 1]; i += blockDim.x) m = fmax(m, ba.part[i]);
  const double lam_all = block_reduce<true>(m, s_w);
  if (threadIdx.x == 0) {
    const double lam = lam_all;
    const double dt = kp.dt_in > 0.0 ? kp.dt_in : kp.cs_cfl / lam;
    kp.scal[0] = dt;
    kp.scal[1] = kp.ch_in >= 0.0 ? kp.ch_in : 0.0;
    kp.scal[2] = lam;
    if (d_dt) d_dt[inst] = dt;
  }
}

// stage phase, one launch per degree: each launch walks the tiles of the
// problems of degree N only (the tile table lists them together), so it holds
// only that degree's registers
template <class Ph, int N, int NT>
__global__ void __launch_bounds__(NT) kb_stages(const BatchArgs ba, const double* __restrict__ u_in,
                                                double* __restrict__ u_out) {
  __shared__ StageLdsT<Ph, N, NT> L;
  int k0, k1, step;
  tile_range(ba.ntiles, ba.xcd, k0, k1, step);
  for (int k = k0; k < k1; k += step) {
    const int t = tile_at(k, ba.ntiles, ba.xcd);
    if (t < 0) break;
    const int inst = ba.tinst[t], blk = ba.tblk[t];
    const KParams& kp = ba.kps[inst];
    const double* un = u_in + ba.uoff[inst];
    double* rv = u_out + ba.uoff[inst];
    stage_body<Ph, N, batch_epb_stages<Ph, N, NT>(), NT, Tableau<N>, true>(kp, L, un, rv, nullptr, blk);
    __syncthreads();
  }
}

// face phase: tiles of 128 face points in each direction
template <class Ph>
__global__ void __launch_bounds__(256) kb_faces(const BatchArgs ba, const double* __restrict__ u_in) {
  int k0, k1, step;
  tile_range(ba.ntiles, ba.xcd, k0, k1, step);
  for (int k = k0; k < k1; k += step) {
    const int t = tile_at(k, ba.ntiles, ba.xcd);
    if (t < 0) break;
    const int inst = ba.tinst[t];
    const KParams& kp = ba.kps[inst];
    const double* un = u_in + ba.uoff[inst];
    // the tile's face points in both directions (face_slot); a slot past the
    // problem's face points gets an index past them too, which the body skips
    int d, fi;
    face_slot<Ph::DIM>(ba.tblk[t], threadIdx.x, 256, d, fi);
    const int nf = kp.E * (Ph::DIM == 1 ? 1 : kp.N + 1);
    const int gid = fi < nf ? d * nf + fi : Ph::DIM * nf;
    switch (kp.N) {
      case 1: faces_body<Ph, 1>(kp, un, gid); break;
      case 2: faces_body<Ph, 2>(kp, un, gid); break;
      case 3: faces_body<Ph, 3>(kp, un, gid); break;
      default: faces_body<Ph, 4>(kp, un, gid); break;
    }
  }
}

template <class Ph, int NT>
__global__ void __launch_bounds__(NT) kb_update(const BatchArgs ba, const double* __restrict__ u_in,
                                                double* __restrict__ io) {
  constexpr int DIM = Ph::DIM;
  __shared__ LdsByDegree<UpdateLds, Ph, NT> L;
  int k0, k1, step;
  tile_range(ba.ntiles, ba.xcd, k0, k1, step);
  for (int k = k0; k < k1; k += step) {
    const int t = tile_at(k, ba.ntiles, ba.xcd);
    if (t < 0) break;
    const int inst = ba.tinst[t], blk = ba.tblk[t];
    const KParams& kp = ba.kps[inst];
    const double* un = u_in + ba.uoff[inst];
    double* o = io + ba.uoff[inst];
    switch (kp.N) {
      case 1: update_body<Ph, 1, batch_epb<1, NT>(DIM), NT, true>(kp, L.n1, un, o, nullptr, blk); break;
      case 2: update_body<Ph, 2, batch_epb<2, NT>(DIM), NT, true>(kp, L.n2, un, o, nullptr, blk); break;
      case 3: update_body<Ph, 3, batch_epb<3, NT>(DIM), NT, true>(kp, L.n3, un, o, nullptr, blk); break;
      default: update_body<Ph, 4, batch_epb<4, NT>(DIM), NT, true>(kp, L.n4, un, o, nullptr, blk); break;
    }
    __syncthreads();
  }
}

}  // namespace lwfr
