// Many independent grids advanced by one launch per RK stage.
//
// The grids of a batch are cut into tiles of one shape; their tiles are
// numbered grid after grid (tile_start[p] is the first tile of grid p).  In
// the persistent form a fixed number of workgroups -- as many as fit on the
// chip at once -- walk that tile order in rounds of gridDim.x tiles; in the
// one-tile form the launch has one workgroup per tile and the hardware
// dispatcher is the work queue (the tile loop of the persistent form makes
// the compiler keep tile-invariant values in registers across the loop,
// which can cost occupancy; the autotuner measures both).  Within a round,
// consecutive tiles go to one XCD (workgroup b runs on XCD b mod 8), so the
// halo re-reads of neighbouring tiles meet in the same L2.  Each tile runs the
// same tile function as the single-grid kernels (inviscid or viscous form,
// chosen per grid), so a grid of the batch computes what a single-grid launch
// with the same tile shape computes, up to how the compiler contracts
// multiply-adds in the two kernels.  The time step is per grid: a
// two-pass min-reduction with a fixed number of partials per grid.  Every
// workgroup leaves the tile loop after at most ceil(total / gridDim.x)
// rounds.
#pragma once
#include <type_traits>

#include "dt_kernel.hpp"
#include "stage_f32.hpp"

namespace gbr {

// One grid of the batch (host-side description; the time-step kernels read
// it on the device).
struct BatchProb {
  double* buf[3];          // the grid's three state arrays, SoA [4][ny][nx]
  int nx, ny, bcx, bcy;
  int tiles_x;             // tile columns for the batch's tile shape
  int pad_;
  double inv_dx, inv_dy, dx, dy;
  double gamma, g1inv, mu, kq, cfl;
};

// A stage launch reads the stage parameters of grid p from tab[p]: one table
// per (array roles, stage) combination, built on the host, so the tile
// function sees the same kind of read-only parameter block as a single-grid
// launch and the compiler can fetch its fields with scalar loads on demand.
struct BatchParams {
  const StageParams* __restrict__ tab;   // [nprob]
  const int* __restrict__ tile_start;    // [nprob + 1]
  int nprob, total;                      // grids, tiles
};

// Grid p with tile_start[p] <= t < tile_start[p + 1].
__device__ __forceinline__ int batch_find(const int* ts, int n, int t) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ts[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }

// MW: waves per SIMD the register budget must allow (the tile loop would
// otherwise let the compiler spend the budget of the smaller of the two forms).
template <class CI, class CV, bool F32, int MW>
struct BatchCfg {
  static_assert(CI::TX == CV::TX && CI::TY == CV::TY && CI::NT == CV::NT, "one tile shape");
  static constexpr int TX = CI::TX, TY = CI::TY, NT = CI::NT;
  static constexpr int MINW = MW;
  // the FP64 tiles take the edge form (primitive MEG7, MP test where flagged)
  using LI = typename CI::template Layout<true>;
  using LV = typename CV::template Layout<true>;
  static constexpr int U = F32 ? imax(F32Cfg<CI>::NU * CI::RS, F32Cfg<CV>::NU * CV::RS)
                                : imax(LI::NFU * CI::RS, LV::NFU * CV::RS);
  static constexpr int PH = F32 ? imax(F32Cfg<CI>::PH, F32Cfg<CV>::PH) : imax(LI::PH, LV::PH);
  static constexpr int CHI = F32 ? imax(F32Cfg<CI>::CHI, F32Cfg<CV>::CHI) : imax(CI::CHI, CV::CHI);
  static constexpr int QMAX = imax(CI::QMAX, CV::QMAX);
  using PhT = typename std::conditional<F32, float, double>::type;
  // queue entries: bytes where every slot fits (FP32 form), else 16 bits
  using QT = typename std::conditional<(F32 && QMAX <= 256), unsigned char, unsigned short>::type;
  static constexpr int LDS_BYTES = 8 * U + (int)sizeof(PhT) * PH + CHI + (int)sizeof(QT) * QMAX + 16;
};

template <class CI, class CV, bool F32, int MW, bool LOOP>
__global__ __launch_bounds__(CI::NT, MW) void meg7_batch_kernel(BatchParams B) {
  using BC = BatchCfg<CI, CV, F32, MW>;
  using PhT = typename BC::PhT;
  __shared__ double sU[BC::U];
  __shared__ PhT sPh[BC::PH];
  __shared__ unsigned char sChi[BC::CHI];
  __shared__ typename BC::QT sQueue[BC::QMAX];
  __shared__ int sQCount;
  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, per = G >> 3;   // G is a multiple of 8
  for (int base = 0; base < B.total; base += G) {
    const int t = base + xcd * per + (b >> 3);
    if (t < B.total) {
      const int p = batch_find(B.tile_start, B.nprob, t);
      const StageParams& P = B.tab[p];
      const int lt = t - B.tile_start[p];
      const int tx0 = (lt % P.tiles_x) * BC::TX, ty0 = (lt / P.tiles_x) * BC::TY;
      if constexpr (F32) {
        if (P.mu > 0.0)
          stage_tile_f32<CV, false>(P, tx0, ty0, sU, sPh, sChi, sQueue, &sQCount, nullptr);
        else
          stage_tile_f32<CI, false>(P, tx0, ty0, sU, sPh, sChi, sQueue, &sQCount, nullptr);
      } else {
        if (P.mu > 0.0)
          stage_tile<CV, false>(P, tx0, ty0, sU, sPh, sChi, sQueue, &sQCount, nullptr);
        else
          stage_tile<CI, false>(P, tx0, ty0, sU, sPh, sChi, sQueue, &sQCount, nullptr);
      }
    }
    if (!LOOP) break;   // one tile per workgroup: gridDim.x >= total
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-grid time step: kBatchDtBlocks partial minima per grid, then one thread
// per grid folds them (a min is exact: the result equals the single-grid one).
constexpr int kBatchDtBlocks = 32;

__global__ __launch_bounds__(kDtThreads) void batch_dt_reduce_kernel(const BatchProb* prob, int qn,
                                                                     double* partial,
                                                                     unsigned* status) {
  __shared__ double red[kDtThreads / 64];
  const int p = blockIdx.x / kBatchDtBlocks, k = blockIdx.x % kBatchDtBlocks;
  const BatchProb& g = prob[p];
  const double* Q = g.buf[qn];
  const size_t n = (size_t)g.nx * g.ny;
  double conv = __builtin_inf(), visc = __builtin_inf();
  bool bad = false;
  for (size_t s = (size_t)k * kDtThreads + threadIdx.x; s < n;
       s += (size_t)kBatchDtBlocks * kDtThreads)
    dt_cell(Q, n, s, g.gamma, g.mu, g.dx, g.dy, conv, visc, bad);
  if (bad) atomicOr(status, 1u);
  conv = block_min(conv, red);
  visc = block_min(visc, red);
  if (threadIdx.x == 0) {
    partial[(size_t)p * 2 * kBatchDtBlocks + k] = conv;
    partial[(size_t)p * 2 * kBatchDtBlocks + kBatchDtBlocks + k] = visc;
  }
}

__global__ __launch_bounds__(256) void batch_dt_finish_kernel(const BatchProb* prob, int nprob,
                                                              const double* partial, double* dt,
                                                              unsigned* status) {
#pragma clang fp contract(off)
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  double conv = __builtin_inf(), visc = __builtin_inf();
  for (int k = 0; k < kBatchDtBlocks; ++k) {
    conv = fmin(conv, partial[(size_t)p * 2 * kBatchDtBlocks + k]);
    visc = fmin(visc, partial[(size_t)p * 2 * kBatchDtBlocks + kBatchDtBlocks + k]);
  }
  const double d = prob[p].cfl * fmin(visc / kAlphaV, conv);
  dt[p] = d;
  if (!(d > 0.0) || !isfinite(d)) atomicOr(status, 2u);
}

}  // namespace gbr
