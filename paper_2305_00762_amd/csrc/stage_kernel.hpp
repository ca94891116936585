// Fused MEG7 residual + SSP-RK3 stage kernel for gfx950 (FP64 path).
//
// One workgroup owns a TX x TY tile of cells.  It stages the tile plus a
// 6-cell halo of primitive variables in LDS once (periodic wrap or
// transmissive clamp in the index math), then sweeps x and y:
//   pass 1 (per cell):      edge jumps of the reconstructed fields (and of
//                           T, viscous) from which the sixth-order gradients
//                           of eq. (eqn:six) are formed where read; staged
//                           gradients instead for MEG7-cons and the MP test
//                           everywhere; density detector (Sec. 2.4),
//                           cell-centre fluxes;
//   pass 2 (per interface): sigma from the 6-cell buffer; smooth interfaces
//                           take GRB states + flux reconstruction + HLLC +
//                           viscous flux at once; flagged ones are compacted
//                           with a wavefront ballot into an LDS queue;
//   pass 3 (queue):         characteristic MP (MEG7) states, F(Q), HLLC;
//   pass 4 (per cell):      flux differences accumulated in registers.
// The x sweep runs in sub-blocks of SX rows, the y sweep in sub-blocks of SY
// columns, so the per-sweep buffers stay small.  The stage update (or the
// residual store) follows in registers with one coalesced FP64 store.
#pragma once
#include "meg7_device.hpp"

namespace gbr {

enum : int { MODE_RESIDUAL = 0, MODE_STAGE1 = 1, MODE_STAGE2 = 2, MODE_STAGE3 = 3 };
enum : unsigned { STATUS_BAD_STATE = 1u };
enum : int { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECT = 2, BC_NOSLIP = 3, BC_INFLOW = 4 };

// One side of the domain (same layout as gbr_side): segment 0 where the
// tangential cell-centre coordinate is below split0 + split_speed t, segment
// 1 beyond; a kind per segment and, for BC_INFLOW, a primitive state.
struct SideDev {
  int kind[2];
  double state[2][4];
  double split0, split_speed;
};

struct StageParams {
  const double* __restrict__ Qk;  // state the residual is evaluated on
  const double* __restrict__ Qn;  // Q^n (stages 2, 3)
  double* __restrict__ out;       // Res or Q^(k+1)
  const double* __restrict__ dt;  // device scalar (stages)
  uint8_t* sigx;                  // optional flag export [ny][nx+1]
  uint8_t* sigy;                  // optional flag export [ny+1][nx]
  unsigned* status;
  int nx, ny, bcx, bcy;
  int tiles_x, ntiles;
  double inv_dx, inv_dy;
  double gamma, g1inv, mu, kq;    // kq = mu / (Pr (gamma-1))
  int mode;
  const uint8_t* chimap;          // learned-detector flags per cell [ny][nx]: bit 0 x, bit 1 y
  // boundaries by side (left, right, bottom, top); null: bcx / bcy on both sides
  const SideDev* __restrict__ sides;
  const double* tnow;             // device time of Q^n (moving boundary segments)
  double tc;                      // stage abscissa: boundary time = tnow + tc dt
  double x0, y0, dx, dy;          // cell-centre coordinates of the boundary segments
  // stage 3 only (else null): per-wave time-step extrema of the output,
  // [3][ntiles x waves per workgroup]: max(|u|+c), max(|v|+c), min rho
  double* dtx;
  // stage 3 only (else null): density and pressure of the output rounded to
  // float32, [2][ny][nx], the learned detector's inputs for the next step
  float* rp;
};

// Ghost cells by index: periodic wrap or transmissive clamp.  The offsets
// reach at most one tile plus the halo past the grid, so the wrap loops run
// at most once for any grid of 12 or more cells per tile extent.
__device__ __forceinline__ int bc_index(int k, int n, int bc) {
  if (bc == 0) {
    while (k < 0) k += n;
    while (k >= n) k -= n;
    return k;
  }
  return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

template <int TX_, int TY_, int SX_, int SY_, int NT_, bool VISC_, int MINW_ = 2>
struct TileCfg {
  static constexpr int TX = TX_, TY = TY_, SX = SX_, SY = SY_, NT = NT_;
  static constexpr int MINW = MINW_;  // waves per SIMD the register budget must allow
  static constexpr bool VISC = VISC_;
  static constexpr int H = 6;
  static constexpr int RX = TX + 2 * H, RY = TY + 2 * H, RS = RX * RY;
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  // Per-line buffers of a sweep: a first buffer of NE fields and the cell
  // fluxes (then the interface fluxes).  The first buffer holds either the
  // normal gradients of the four reconstructed fields (MEG7-cons, MP test
  // everywhere) or the edge jumps of those fields, from which every gradient
  // is formed where it is read (the edge form: the other variants); the
  // viscous edge form adds the edge jumps of T as a fifth field, and its tile
  // then holds no T.  The tangential derivatives of u_n, u_t are formed from
  // the tile where an interface needs them.
  template <int N, int NL, int NE = 4, bool EDGE = true>
  struct Phase {
    static constexpr int WD = N + 6, WF = N + 10, WFL = N + 1;
    static constexpr int WE = N + 10;   // edges j+1/2, j in [-5, N+5)
    static constexpr int D = NE * NL * (EDGE ? WE : WD);
    static constexpr int F = 4 * NL * (WF > WFL ? WF : WFL);
    static constexpr int TOT = D + F;
  };
  template <bool EDGE>
  struct Layout {
    static constexpr bool TFIELD = VISC && !EDGE;   // the tile holds T
    static constexpr int NFU = TFIELD ? 5 : 4;      // tile fields
    static constexpr int NE = VISC && EDGE ? 5 : 4;
    static constexpr int PH = cmax(Phase<TX, SX, NE, EDGE>::TOT, Phase<TY, SY, NE, EDGE>::TOT);
  };
  using PX = Phase<TX, SX>;
  using PY = Phase<TY, SY>;
  // the larger of the two layouts (the LDS bound checked at the launch sites)
  static constexpr int NF = cmax(Layout<false>::NFU, Layout<true>::NFU);
  static constexpr int PH = cmax(Layout<false>::PH, Layout<true>::PH);
  static constexpr int CHI = cmax(SX * PX::WD, SY * PY::WD);
  static constexpr int QMAX = cmax(SX * PX::WFL, SY * PY::WFL);
  static constexpr int CPT = (TX * TY + NT - 1) / NT;
  static constexpr int LDS_BYTES = 8 * (NF * RS + PH) + CHI + 2 * QMAX + 16;
};

// The edge form (per-line edge jumps instead of staged gradients) serves
// every variant but MEG7-cons and the MP test at every interface, which read
// many gradients per interface.
template <bool CONS, bool MPE>
constexpr bool edge_form() { return !CONS && !MPE; }

// Cell slot k of thread tid: tile cell (lx, ly); false for an idle slot.
// Row-major in general.  For 15 x 15 tiles on 256 threads each half-wave
// (32 lanes) takes two rows three apart, 16 lanes per row (the last idle):
// the LDS tile's row stride is 27 doubles and 3 x 27 = 17 mod 32, so the two
// rows' doubles fall on disjoint halves of the 32 eight-byte slots a
// half-wave reads at once (rows 12 and 14, two apart, share a half-wave).
template <class C>
__device__ __forceinline__ bool tile_cell(int tid, int k, int& lx, int& ly) {
  if constexpr (C::TX == 15 && C::TY == 15 && C::NT == 256) {
    const int h = tid >> 5, i = tid & 31;
    const int a = h / 3 * 6 + h % 3;   // rows a, a + 3 (h = 6: 12, 14; h = 7: 13)
    lx = i & 15;
    ly = i < 16 ? a : (h == 6 ? 14 : a + 3);
    return lx < 15 && ly < 15;
  } else {
    const int c = tid + k * C::NT;
    lx = c % C::TX;
    ly = c / C::TX;
    return c < C::TX * C::TY;
  }
}

// Shared-memory views handed to the sweep.
struct Lds {
  double* U;
  double* ph;
  unsigned char* chi;
  unsigned short* queue;
  int* qcount;
  const unsigned char* chif;   // per-cell learned-detector flags (bit 0 x, bit 1 y)
};

// Index of tile cell (lx, ly), lx in [-3, TX+3), ly in [-3, TY+3), in the
// per-cell flag array of the learned detector.
template <class C>
__device__ __forceinline__ int mlp_chi_index(int lx, int ly) {
  return (ly + 3) * (C::TX + 6) + (lx + 3);
}

// Learned-detector flags of the tile cells the sigma buffers read,
// [-3, TX+3) x [-3, TY+3), from the per-cell flag map (ghost cells take the
// flag of the cell they copy: periodic wrap or transmissive clamp).  Fetched
// into registers before the tile's loads are issued and stored to LDS after
// the tile is staged, so their latency overlaps the tile's.
template <class C>
struct ChiMap {
  static constexpr int NC = (C::TX + 6) * (C::TY + 6);
  static constexpr int R = (NC + C::NT - 1) / C::NT;
  unsigned char v[R];
};
template <class C>
__device__ __forceinline__ void fetch_chimap(const StageParams& P, ChiMap<C>& m, int tx0,
                                             int ty0) {
  constexpr int W6 = C::TX + 6;
  const bool inner = tx0 >= 3 && ty0 >= 3 && tx0 + C::TX + 3 <= P.nx && ty0 + C::TY + 3 <= P.ny;
#pragma unroll
  for (int k = 0; k < ChiMap<C>::R; ++k) {
    const int c = threadIdx.x + k * C::NT;
    if (c < ChiMap<C>::NC) {
      const int ly = c / W6 - 3, lx = c - (ly + 3) * W6 - 3;
      const int gi = inner ? ty0 + ly : bc_index(ty0 + ly, P.ny, P.bcy);
      const int gj = inner ? tx0 + lx : bc_index(tx0 + lx, P.nx, P.bcx);
      m.v[k] = P.chimap[gi * P.nx + gj];
    }
  }
}
template <class C>
__device__ __forceinline__ void put_chimap(const ChiMap<C>& m, unsigned char* chif) {
#pragma unroll
  for (int k = 0; k < ChiMap<C>::R; ++k) {
    const int c = threadIdx.x + k * C::NT;
    if (c < ChiMap<C>::NC) chif[c] = m.v[k];
  }
}

template <class C, int DIR, bool DETMLP, bool CONS, int ORD, bool LM, bool MPE>
__device__ __forceinline__ void sweep(const StageParams& P, const Lds& L, int l0, int tx0,
                                      int ty0, double (&res)[C::CPT][4]) {
  constexpr bool X = (DIR == 0);
  constexpr int N = X ? C::TX : C::TY;
  constexpr int NL = X ? C::SX : C::SY;
  constexpr int NLINES = X ? C::TY : C::TX;
  constexpr bool EDGE = edge_form<CONS, MPE>();
  constexpr bool ET = C::VISC && EDGE;   // T edges in the first buffer, no T in the tile
  using PH = typename C::template Phase<N, NL, C::template Layout<EDGE>::NE, EDGE>;
  constexpr int WD = PH::WD, WF = PH::WF, WFL = PH::WFL, WE = PH::WE;
  constexpr int RS = C::RS, RX = C::RX, H = C::H, NT = C::NT;
  constexpr int SN = X ? 1 : RX;  // normal stride in the LDS tile
  constexpr int ST = X ? RX : 1;  // tangential stride
  constexpr int FN = X ? 1 : 2;   // field holding the normal velocity
  constexpr int FT = X ? 2 : 1;   // field holding the tangential velocity
  constexpr int IPT = (NL * WFL + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int nl = (NLINES - l0) < NL ? (NLINES - l0) : NL;
  const double inv_dn = X ? P.inv_dx : P.inv_dy;
  const double inv_dt = X ? P.inv_dy : P.inv_dx;

  double* sD = L.ph;                       // [4][NL x WD]   normal gradients (rotated order), or
  double* sE = L.ph;                       // [4|5][NL x WE] edge jumps (rotated order, then T) at j + 5
  double* sF = sD + PH::D;                 // [4][NL x WF]   cell fluxes; later [4][NL x WFL] interface fluxes
  constexpr int FSTR = (WF > WFL ? WF : WFL) * NL;
  // interface values: odd row stride, so pass 4 (lanes across lines in the
  // y sweep) reads distinct banks
  constexpr int WFS = WFL | 1;
  static_assert(WFS <= WF, "interface rows fit the flux buffer");
  // buffer index and thread mapping: positions fastest in both sweeps (in the
  // y sweep consecutive lanes then step RX doubles apart in the tile, an odd
  // stride, so the FP64 tile reads fall in distinct banks)
  auto bidx = [](int line, int p, int W) { return line * W + p; };
  auto ridx = [&](int line, int pos) {
    const int lx = X ? pos : l0 + line;
    const int ly = X ? l0 + line : pos;
    return (ly + H) * RX + (lx + H);
  };
  const int rot[5] = {0, FN, FT, 3, 4};
  // MEG7-cons: the tile holds (rho, rho u, rho v, E [, T]); primitives of a
  // cell are formed on the fly, as in the tile load of MEG7-prim
  auto prim_at = [&](int r, double(&W)[4]) {
    const double* U = L.U;
    const double rho = U[r], ir = rcp_nr(rho);
    W[0] = rho;
    W[1] = U[FN * RS + r] * ir;
    W[2] = U[FT * RS + r] * ir;
    W[3] = (P.gamma - 1.0) * (U[3 * RS + r] - 0.5 * rho * (W[1] * W[1] + W[2] * W[2]));
  };
  // Sixth-order derivative of tile field f at cell r along stride d (eq. (eqn:six)).
  auto g6 = [&](int f, int r, int d) {
    const double* u = L.U + f * RS + r;
    return grad6(u[-3 * d], u[-2 * d], u[-d], u[d], u[2 * d], u[3 * d]);
  };
  // Edge form: edge jump j+1/2 of rotated field m (m < 4) on line `line`
  // (pass 1 stores j in [-5, N+5); the edge j = -6, which only gradients at
  // a line's first interface reach, is formed from the tile), and the normal
  // gradient of eq. (eqn:six) at cell k on the edges: the stencil
  // (45, -9, 1)/60 on value differences becomes (37, -8, 1)/60 on the pairs
  // of edges around k.
  auto edge = [&](int m, int line, int j) -> double {
    if (j < -5) {
      const double* u = L.U + rot[m] * RS + ridx(line, -6);
      return u[SN] - u[0];
    }
    return sE[m * NL * WE + bidx(line, j + 5, WE)];
  };
  auto g6e = [](double e0, double e1, double e2, double e3, double e4, double e5) {
    constexpr double z = 1.0 / 60.0;
    return z * (37.0 * (e2 + e3) - 8.0 * (e1 + e4) + (e0 + e5));
  };
  auto gradE = [&](int m, int line, int k) -> double {
    return g6e(edge(m, line, k - 3), edge(m, line, k - 2), edge(m, line, k - 1),
               edge(m, line, k), edge(m, line, k + 1), edge(m, line, k + 2));
  };
  // normal gradient of rotated field m at cell k of line `line`
  auto grad_at = [&](int m, int line, int k) -> double {
    if constexpr (EDGE) return gradE(m, line, k);
    else return sD[m * NL * WD + bidx(line, k + 3, WD)];
  };
  // Normal differences the viscous flux of interface (line, pos + 1/2)
  // takes, r its left cell: gv = {g(u_n), g(u_n)', g(u_t), g(u_t)', g(T),
  // g(T)', T' - T} (g at the left cell, ' at the right one; velocity entries
  // for the primitive forms only, and only with vel)
  auto visc_normal = [&](int line, int pos, int r, double* gv, bool vel) {
    if constexpr (ET) {
      // T edges pos-3 .. pos+3: stored for every interface pos in [-1, N)
      const double* e = sE + 4 * NL * WE;
      double t[7];
#pragma unroll
      for (int a = 0; a < 7; ++a) t[a] = e[bidx(line, pos + a + 2, WE)];
      gv[4] = g6e(t[0], t[1], t[2], t[3], t[4], t[5]);
      gv[5] = g6e(t[1], t[2], t[3], t[4], t[5], t[6]);
      gv[6] = t[3];
    } else {
      gv[4] = g6(4, r, SN);
      gv[5] = g6(4, r + SN, SN);
      gv[6] = L.U[4 * RS + r + SN] - L.U[4 * RS + r];
    }
    if (!CONS && vel) {
      gv[0] = grad_at(1, line, pos);
      gv[1] = grad_at(1, line, pos + 1);
      gv[2] = grad_at(2, line, pos);
      gv[3] = grad_at(2, line, pos + 1);
    }
  };
  // viscous flux of interface (line, pos + 1/2) added to F (gv as above)
  auto visc_at = [&](int line, int pos, int r, const double* gv, double* F) {
    const double* U = L.U;
    const double gT0 = gv[4], gT1 = gv[5];
    if (CONS) {
      // velocity gradients by the chain rule d u = (d(rho u) - u d rho) / rho
      const int b0 = bidx(line, pos + 3, WD), b1 = bidx(line, pos + 4, WD);
      const double* D0 = sD;
      const double* D1 = sD + 1 * NL * WD;
      const double* D2 = sD + 2 * NL * WD;
      const double ir0 = rcp_nr(U[r]), ir1 = rcp_nr(U[r + SN]);
      const double un0 = U[FN * RS + r] * ir0, un1 = U[FN * RS + r + SN] * ir1;
      const double ut0 = U[FT * RS + r] * ir0, ut1 = U[FT * RS + r + SN] * ir1;
      // tangential derivatives of un, ut at the two cells
      double dunt[2], dutt[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int rc = r + c * SN;
        const double gr = g6(0, rc, ST) * inv_dt;
        const double gn = g6(FN, rc, ST) * inv_dt;
        const double gt = g6(FT, rc, ST) * inv_dt;
        const double ir = c ? ir1 : ir0;
        dunt[c] = (gn - (U[FN * RS + rc] * ir) * gr) * ir;
        dutt[c] = (gt - (U[FT * RS + rc] * ir) * gr) * ir;
      }
      viscous_add(un0, un1, ut0, ut1, 0.0, gv[6],
                  (D1[b0] - un0 * D0[b0]) * ir0, (D1[b1] - un1 * D0[b1]) * ir1,
                  (D2[b0] - ut0 * D0[b0]) * ir0, (D2[b1] - ut1 * D0[b1]) * ir1, gT0, gT1,
                  dunt[0], dunt[1], dutt[0], dutt[1], inv_dn, P.mu, P.kq, F);
    } else {
      viscous_add(U[FN * RS + r], U[FN * RS + r + SN], U[FT * RS + r], U[FT * RS + r + SN],
                  0.0, gv[6], gv[0], gv[1], gv[2], gv[3], gT0, gT1,
                  g6(FN, r, ST) * inv_dt, g6(FN, r + SN, ST) * inv_dt,
                  g6(FT, r, ST) * inv_dt, g6(FT, r + SN, ST) * inv_dt, inv_dn, P.mu, P.kq, F);
    }
  };

  // ---- pass 1: per-cell quantities ----------------------------------------
  constexpr int P1R = (NL * WF + NT - 1) / NT;
#pragma unroll
  for (int k1 = 0; k1 < P1R; ++k1) {
    const int t = tid + k1 * NT;
    if (t >= NL * WF) break;
    const int line = t / WF;
    const int p = t % WF;
    if (line >= nl) continue;
    const int pos = p - 5;
    const int r = ridx(line, pos);
    const double* U = L.U;
    {
      double W[4];
      if (CONS) {
        prim_at(r, W);
      } else {
        W[0] = U[r]; W[1] = U[FN * RS + r]; W[2] = U[FT * RS + r]; W[3] = U[3 * RS + r];
      }
      double f[4];
      conv_flux(W, P.g1inv, f);
#pragma unroll
      for (int m = 0; m < 4; ++m) sF[m * FSTR + bidx(line, p, WF)] = f[m];
    }
    if (EDGE) {
      // edge jump pos + 1/2, pos in [-5, N+5)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double* u = U + rot[m] * RS + r;
        sE[m * NL * WE + bidx(line, pos + 5, WE)] = u[SN] - u[0];
      }
      if (ET) {
        // T = gamma p / rho on both sides (the tile holds no T)
        const double T0 = P.gamma * U[3 * RS + r] * rcp_nr(U[r]);
        const double T1 = P.gamma * U[3 * RS + r + SN] * rcp_nr(U[r + SN]);
        sE[4 * NL * WE + bidx(line, pos + 5, WE)] = T1 - T0;
      }
    }
    if (pos >= -3 && pos < N + 3) {
      const int pd = pos + 3;
      if (!EDGE) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const double* u = U + rot[m] * RS + r;
          sD[m * NL * WD + bidx(line, pd, WD)] =
              grad6(u[-3 * SN], u[-2 * SN], u[-SN], u[SN], u[2 * SN], u[3 * SN]);
        }
      }
      if (DETMLP) {
        L.chi[bidx(line, pd, WD)] =
            (L.chif[mlp_chi_index<C>(X ? pos : l0 + line, X ? l0 + line : pos)] >> DIR) & 1;
      } else {
        const double* rho = U + r;
        L.chi[bidx(line, pd, WD)] =
            detector_flag(rho[-2 * SN], rho[-SN], rho[0], rho[SN], rho[2 * SN]) ? 1 : 0;
      }
    }
  }
  if (tid == 0) *L.qcount = 0;
  __syncthreads();

  // ---- pass 2: interfaces, smooth branch; ballot-compact the flagged ------
  double fsm[IPT][4];
  bool has[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    has[k] = false;
    const int t = tid + k * NT;
    bool flagged = false;
    if (t < NL * WFL) {
      const int line = t / WFL;
      const int p = t % WFL;
      const int pos = p - 1;  // interface pos + 1/2
      if (line < nl) {
        // eq. (buffer): the six flags read at once and OR-ed (a short-circuit
        // chain would wait for each LDS read in turn)
        unsigned any = 0u;
#pragma unroll
        for (int q = 1; q <= 6; ++q) any |= L.chi[bidx(line, pos + q, WD)];
        const bool sigma = any == 0u;
        if (X) {
          const int gi = ty0 + l0 + line, gj = tx0 + pos;
          if (P.sigx && gi < P.ny && gj < P.nx) P.sigx[(size_t)gi * (P.nx + 1) + gj + 1] = sigma;
        } else {
          const int gj = tx0 + l0 + line, gi = ty0 + pos;
          if (P.sigy && gj < P.nx && gi < P.ny) P.sigy[(size_t)(gi + 1) * P.nx + gj] = sigma;
        }
        flagged = !sigma;
        if (sigma) {
          const int r = ridx(line, pos);
          double WL[4], WR[4], Fm[4], gv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const double* u = L.U + rot[m] * RS + r;
            if constexpr (EDGE) {
              // eq. (eqn:grb) (ORD 7) or its fourth-order subset with the
              // gradients of eq. (eqn:six) substituted, minus Phi_j (resp.
              // Phi_{j+1}): stencils on the edge jumps E[a] at (pos+a-4)+1/2
              double E[9];
#pragma unroll
              for (int a = 0; a < 9; ++a) E[a] = sE[m * NL * WE + bidx(line, pos + a + 1, WE)];
              double cL, cR;
              if (ORD == 4) {
                constexpr double s4 = 1.0 / 1440.0;
                cL = s4 * ((E[0] - E[7]) + 4.0 * E[1] - 60.0 * E[2] + 249.0 * E[3] + 639.0 * E[4] -
                           132.0 * E[5] + 20.0 * E[6]);
                cR = s4 * ((E[1] - E[8]) - 20.0 * E[2] + 132.0 * E[3] - 639.0 * E[4] -
                           249.0 * E[5] + 60.0 * E[6] - 4.0 * E[7]);
              } else {
                constexpr double s7 = 1.0 / 840.0;
                cL = s7 * ((E[0] - E[1] - E[7]) - 23.0 * E[2] + 123.0 * E[3] + 395.0 * E[4] -
                           89.0 * E[5] + 15.0 * E[6]);
                cR = s7 * ((E[1] - E[8] + E[7]) - 15.0 * E[2] + 89.0 * E[3] - 395.0 * E[4] -
                           123.0 * E[5] + 23.0 * E[6]);
              }
              WL[m] = u[0] + cL;
              WR[m] = u[SN] + cR;
              if (C::VISC && (m == 1 || m == 2)) {
                // velocity gradients at cells pos, pos+1 from the same edges
                gv[2 * m - 2] = g6e(E[1], E[2], E[3], E[4], E[5], E[6]);
                gv[2 * m - 1] = g6e(E[2], E[3], E[4], E[5], E[6], E[7]);
              }
            } else {
              double v[6], g[6];
#pragma unroll
              for (int q = 0; q < 6; ++q) v[q] = u[(q - 2) * SN];
#pragma unroll
              for (int q = 1; q < 5; ++q) g[q] = sD[m * NL * WD + bidx(line, pos + q + 1, WD)];
              g[0] = g[5] = 0.0;
              WL[m] = grb_l<ORD>(v, g);
              WR[m] = grb_r<ORD>(v, g);
            }
            // (F(f_L) + F(f_R))/2 on the cell fluxes f_{j-4..j+5}
            double f[10];
#pragma unroll
            for (int q = 0; q < 10; ++q) f[q] = sF[m * FSTR + bidx(line, pos + q + 1, WF)];
            Fm[m] = flux_mean<ORD>(f);
          }
          if (MPE) {
            // MP test at every interface (mp_mode everywhere): the states are
            // the characteristic MEG7 ones; the fluxes stay reconstructed
            auto Vf = [&](int q, int f) { return L.U[rot[f] * RS + r + (q - 2) * SN]; };
            auto Gf = [&](int q, int f) { return sD[f * NL * WD + bidx(line, pos + q + 1, WD)]; };
            if (CONS) {
              double QL[4], QR[4];
              meg7_char_states_cons<ORD>(Vf, Gf, P.gamma, QL, QR);
              cons_to_prim(QL, P.gamma, WL);
              cons_to_prim(QR, P.gamma, WR);
            } else {
              meg7_char_states<ORD>(Vf, Gf, P.gamma, WL, WR);
            }
          } else if (CONS) {
            // the GRB states above are conservative: to primitives
            const double QL[4] = {WL[0], WL[1], WL[2], WL[3]};
            const double QR[4] = {WR[0], WR[1], WR[2], WR[3]};
            cons_to_prim(QL, P.gamma, WL);
            cons_to_prim(QR, P.gamma, WR);
          }
          if (!(WL[0] > 0.0 && WL[3] > 0.0 && WR[0] > 0.0 && WR[3] > 0.0)) {
            // unphysical reconstruction: first-order states and fluxes
            double f0[4], f1[4];
            if (CONS) {
              prim_at(r, WL);
              prim_at(r + SN, WR);
            } else {
#pragma unroll
              for (int m = 0; m < 4; ++m) {
                WL[m] = L.U[rot[m] * RS + r];
                WR[m] = L.U[rot[m] * RS + r + SN];
              }
            }
            conv_flux(WL, P.g1inv, f0);
            conv_flux(WR, P.g1inv, f1);
#pragma unroll
            for (int m = 0; m < 4; ++m) Fm[m] = 0.5 * (f0[m] + f1[m]);
          }
          hllc<LM>(WL, WR, Fm, P.gamma, P.g1inv, fsm[k]);
          if (C::VISC) {
            // edge form: the velocity entries came with the GRB states above
            visc_normal(line, pos, r, gv, !EDGE);
            visc_at(line, pos, r, gv, fsm[k]);
          }
          has[k] = true;
        }
      }
    }
    // wavefront ballot: append the flagged interfaces of this wave to the queue
    const unsigned long long ball = __ballot(flagged);
    if (ball) {
      const int lane = __lane_id();
      int base = 0;
      if (lane == 0) base = atomicAdd(L.qcount, (int)__popcll(ball));
      base = __shfl(base, 0);
      if (flagged) {
        const int rank = (int)__popcll(ball & ((1ull << lane) - 1ull));
        L.queue[base + rank] = (unsigned short)t;
      }
    }
  }
  __syncthreads();  // every read of the cell fluxes is done: the buffer becomes the flux buffer
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (has[k]) {
      const int t = tid + k * NT;
      const int line = t / WFL;
      const int p = t % WFL;
#pragma unroll
      for (int m = 0; m < 4; ++m) sF[m * FSTR + bidx(line, p, WFS)] = fsm[k][m];
    }
  }

  // ---- pass 3: compacted shock branch (characteristic MEG7, F(Q)) --------
  const int nq = *L.qcount;
  for (int qi = tid; qi < nq; qi += NT) {
    const int t = L.queue[qi];
    const int line = t / WFL;
    const int p = t % WFL;
    const int pos = p - 1;
    const int r = ridx(line, pos);
    const double* U = L.U;
    double WL[4], WR[4];
    auto Vf = [&](int q, int f) { return U[rot[f] * RS + r + (q - 2) * SN]; };
    auto Gf = [&](int q, int f) { return grad_at(f, line, pos + q - 2); };
    // edge form: the jumps across edges (pos-5)+1/2 .. (pos+5)+1/2
    auto Ef = [&](int a, int f) { return edge(f, line, pos - 5 + a); };
    if (CONS) {
      double QL[4], QR[4];
      meg7_char_states_cons<ORD>(Vf, Gf, P.gamma, QL, QR);
      cons_to_prim(QL, P.gamma, WL);
      cons_to_prim(QR, P.gamma, WR);
    } else if constexpr (EDGE) {
      meg7_char_states_edges<ORD>(Vf, Ef, P.gamma, WL, WR);
    } else {
      meg7_char_states<ORD>(Vf, Gf, P.gamma, WL, WR);
    }
    if (!(WL[0] > 0.0 && WL[3] > 0.0 && WR[0] > 0.0 && WR[3] > 0.0)) {
      if (CONS) {
        prim_at(r, WL);
        prim_at(r + SN, WR);
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          WL[m] = U[rot[m] * RS + r];
          WR[m] = U[rot[m] * RS + r + SN];
        }
      }
    }
    double FL[4], FR[4], Fm[4], F[4];
    conv_flux(WL, P.g1inv, FL);
    conv_flux(WR, P.g1inv, FR);
#pragma unroll
    for (int m = 0; m < 4; ++m) Fm[m] = 0.5 * (FL[m] + FR[m]);
    hllc<LM>(WL, WR, Fm, P.gamma, P.g1inv, F);
    if (C::VISC) {
      double gv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      visc_normal(line, pos, r, gv, true);
      visc_at(line, pos, r, gv, F);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) sF[m * FSTR + bidx(line, p, WFS)] = F[m];
  }
  __syncthreads();

  // ---- pass 4: flux differences, eq. (deriv) -------------------------------
#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
    int lx, ly;
    if (tile_cell<C>(tid, k, lx, ly)) {
      const int line = (X ? ly : lx) - l0;
      const int pos = X ? lx : ly;
      if (line >= 0 && line < nl) {
        const int bp = bidx(line, pos + 1, WFS), bm = bidx(line, pos, WFS);
        const double d0 = sF[0 * FSTR + bp] - sF[0 * FSTR + bm];
        const double d1 = sF[1 * FSTR + bp] - sF[1 * FSTR + bm];
        const double d2 = sF[2 * FSTR + bp] - sF[2 * FSTR + bm];
        const double d3 = sF[3 * FSTR + bp] - sF[3 * FSTR + bm];
        res[k][0] -= d0 * inv_dn;
        res[k][FN] -= d1 * inv_dn;
        res[k][FT] -= d2 * inv_dn;
        res[k][3] -= d3 * inv_dn;
      }
    }
  }
  __syncthreads();
}

// Tile owned by this workgroup.  Workgroups are dealt to the 8 XCDs
// round-robin, so each XCD gets one contiguous run of tiles (halo rows shared
// in its L2).  Returns false for a workgroup past the last tile.
__device__ __forceinline__ bool tile_origin(const StageParams& P, int TX, int TY, int& tx0,
                                            int& ty0) {
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b & 7, idx = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + idx;
  if (tile >= P.ntiles) return false;
  tx0 = (tile % P.tiles_x) * TX;
  ty0 = (tile / P.tiles_x) * TY;
  return true;
}

// Stage Q^(k) of the tile plus its 6-cell halo as primitives (rho, u, v, p
// [, T = gamma p / rho]) in LDS; MEG7-cons keeps (rho, rho u, rho v, E [, T]).  All global loads are issued before any is
// consumed, so the memory latency is paid once rather than once per round.
// Boundary rules of a ghost cell at raw index k along an axis (0: x, 1: y)
// from the side table: the side's kind at the cell's segment (-1 inside the
// grid), the segment, and the source index -- wrap (periodic), mirror about
// the wall (reflecting, no-slip; clamped where a ragged tile overhangs the
// grid by more than the grid), or the nearest cell.
__device__ __forceinline__ int side_kind(const StageParams& P, int axis, int k, double tang,
                                         double tb, int& side, int& seg, int& src) {
#pragma clang fp contract(off)
  const int n = axis == 0 ? P.nx : P.ny;
  src = k;
  side = 2 * axis + (k >= n ? 1 : 0);
  seg = 0;
  if (k >= 0 && k < n) return -1;
  const SideDev& S = P.sides[side];
  seg = (tang < S.split0 + S.split_speed * tb) ? 0 : 1;
  const int kind = S.kind[seg];
  if (kind == BC_PERIODIC) {
    src = bc_index(k, n, 0);
  } else if (kind == BC_REFLECT || kind == BC_NOSLIP) {
    const int m = k < 0 ? -1 - k : 2 * n - 1 - k;
    src = m < 0 ? 0 : (m >= n ? n - 1 : m);
  } else {
    src = k < 0 ? 0 : (k >= n ? n - 1 : k);
  }
  return kind;
}

// Sign and fixed-state rules of a ghost cell, packed: bit 0 negate rho u,
// bit 1 negate rho v, bit 2 fixed state, bits 3-4 its side, bit 5 its segment.
__device__ __forceinline__ unsigned ghost_op(int kx, int ky, int sx, int gx, int sy, int gy) {
  unsigned op = 0;
  if (kx == BC_REFLECT || kx == BC_NOSLIP) op ^= 1u;
  if (kx == BC_NOSLIP) op ^= 2u;
  if (ky == BC_REFLECT || ky == BC_NOSLIP) op ^= 2u;
  if (ky == BC_NOSLIP) op ^= 1u;
  if (kx == BC_INFLOW)
    op |= 4u | ((unsigned)sx << 3) | ((unsigned)gx << 5);
  else if (ky == BC_INFLOW)
    op |= 4u | ((unsigned)sy << 3) | ((unsigned)gy << 5);
  return op;
}

// TFIELD: whether the tile holds T (the FP64 viscous kernels of MEG7-cons
// and of the MP test everywhere; the edge-form and FP32 ones form T where
// they need it).
template <class C, bool CONS = false, bool TFIELD = C::VISC>
__device__ __forceinline__ void stage_load(const StageParams& P, double* sU, int tx0, int ty0) {
  constexpr int RS = C::RS, RX = C::RX, H = C::H, NT = C::NT, TX = C::TX, TY = C::TY;
  constexpr int LR = (RS + NT - 1) / NT;
  const int tid = threadIdx.x;
  const size_t n = (size_t)P.nx * P.ny;
  bool bad = false;
  // one cell of the tile at (lx, ly): conservative values (ghost rules
  // applied) to the staged variables; op as packed by ghost_op
  auto put = [&](int lx, int ly, double r, double mx, double my, double E, unsigned op) {
    const int c = (ly + H) * RX + (lx + H);
    if (op & 1u) mx = -mx;
    if (op & 2u) my = -my;
    double ir = rcp_nr(r);
    double u = mx * ir, v = my * ir;
    double p = (P.gamma - 1.0) * (E - 0.5 * r * (u * u + v * v));
    if (op & 4u) {
      // fixed (inflow) state: primitives as given, conservative from them
      const double* st = P.sides[(op >> 3) & 3u].state[(op >> 5) & 1u];
      r = st[0]; u = st[1]; v = st[2]; p = st[3];
      ir = rcp_nr(r);
      mx = r * u; my = r * v;
      E = p * P.g1inv + 0.5 * r * (u * u + v * v);
    }
    sU[c] = r;
    sU[RS + c] = CONS ? mx : u;
    sU[2 * RS + c] = CONS ? my : v;
    sU[3 * RS + c] = CONS ? E : p;
    if (TFIELD) sU[4 * RS + c] = P.gamma * p * ir;
    // the state check covers the tile's own cells (a branch, so waves that
    // stage only halo cells skip it)
    if (lx >= 0 && lx < TX && ly >= 0 && ly < TY && tx0 + lx < P.nx && ty0 + ly < P.ny) {
      if (!(r > 0.0 && p > 0.0 && isfinite(E) && isfinite(mx) && isfinite(my) && isfinite(r)))
        bad = true;
    }
  };
  // a tile whose halo stays inside the grid needs no ghost rules
  const bool inner = tx0 >= H && ty0 >= H && tx0 + TX + H <= P.nx && ty0 + TY + H <= P.ny;
  // the side table matters only where the tile's halo reaches past the grid
  const bool walls = P.sides != nullptr && !inner;
  if (!walls) {
    // all global loads issued before any is consumed: the memory latency is
    // paid once rather than once per round.  Element offsets fit 32 bits
    // (4 nx ny <= 2^31 - 1).
    double q[LR][4];
    const double* Q0 = P.Qk;
    const double* Q1 = P.Qk + n;
    const double* Q2 = P.Qk + 2 * n;
    const double* Q3 = P.Qk + 3 * n;
#pragma unroll
    for (int k = 0; k < LR; ++k) {
      const int c = tid + k * NT;
      if (c < RS) {
        const int ly = c / RX - H, lx = c - (ly + H) * RX - H;
        const int gi = inner ? ty0 + ly : bc_index(ty0 + ly, P.ny, P.bcy);
        const int gj = inner ? tx0 + lx : bc_index(tx0 + lx, P.nx, P.bcx);
        const int o = gi * P.nx + gj;
        q[k][0] = Q0[o];
        q[k][1] = Q1[o];
        q[k][2] = Q2[o];
        q[k][3] = Q3[o];
      }
    }
#pragma unroll
    for (int k = 0; k < LR; ++k) {
      const int c = tid + k * NT;
      if (c < RS) {
        const int ly = c / RX - H, lx = c - (ly + H) * RX - H;
        put(lx, ly, q[k][0], q[k][1], q[k][2], q[k][3], 0u);
      }
    }
  } else {
    // boundary tiles with a side table: one cell at a time
    double tb;
    {
#pragma clang fp contract(off)
      tb = *P.tnow + (P.tc != 0.0 ? P.tc * *P.dt : 0.0);
    }
#pragma unroll 1
    for (int c = tid; c < RS; c += NT) {
      const int ly = c / RX - H, lx = c % RX - H;
      const int i = ty0 + ly, j = tx0 + lx;
      double xc, yc;
      {
#pragma clang fp contract(off)
        xc = P.x0 + ((double)j + 0.5) * P.dx;
        yc = P.y0 + ((double)i + 0.5) * P.dy;
      }
      int sx, gx, sy, gy, gi, gj;
      const int kx = side_kind(P, 0, j, yc, tb, sx, gx, gj);
      const int ky = side_kind(P, 1, i, xc, tb, sy, gy, gi);
      const size_t s = (size_t)gi * P.nx + gj;
      put(lx, ly, P.Qk[s], P.Qk[n + s], P.Qk[2 * n + s], P.Qk[3 * n + s],
          ghost_op(kx, ky, sx, gx, sy, gy));
    }
  }
  if (bad) atomicOr(P.status, STATUS_BAD_STATE);
}

// Velocity and pressure of a conservative state with one rounding per
// operation and IEEE division: u = (rho u)/rho, v = (rho v)/rho,
// p = (gamma-1)(E - rho (u u + v v)/2).  Inside div_rb's operand range the
// quotients share one refined reciprocal rb (the IEEE quotient bit for bit);
// fast says whether they did.  The time step and the learned detector's
// pressure are defined on exactly these values.
struct CellUVP {
  double u, v, p, rb;
  bool fast;
};
__device__ __forceinline__ CellUVP cell_uvp(const double q[4], double gamma) {
#pragma clang fp contract(off)
  CellUVP c;
  const double rho = q[0];
  c.rb = rcp_nr(rho);
  c.fast = rho != 0.0 && div_rb_ok(rho) && div_rb_ok(q[1]) && div_rb_ok(q[2]);
  if (c.fast) {
    c.u = div_rb(q[1], rho, c.rb);
    c.v = div_rb(q[2], rho, c.rb);
  } else {
    c.u = q[1] / rho;
    c.v = q[2] / rho;
  }
  c.p = (gamma - 1.0) * (q[3] - rho * (c.u * c.u + c.v * c.v) / 2.0);
  return c;
}

// Time-step extrema of one cell of the new state (Sec. 2.5): |u|+c, |v|+c
// and rho, each rounded exactly as the time-step kernel rounds them (one
// rounding per operation, IEEE division and square root), folded into
// (amax, bmax, rmin).  Since fl(d/x) is monotone in x, the minima of the
// per-cell limits follow from these extrema without loss.
__device__ __forceinline__ void dt_extrema_cell(const double q[4], const CellUVP& w, double gamma,
                                                double& amax, double& bmax, double& rmin,
                                                bool& bad) {
#pragma clang fp contract(off)
  const double rho = q[0];
  const double gp = gamma * w.p;
  const double c = sqrt((w.fast && div_rb_ok(gp)) ? div_rb(gp, rho, w.rb) : gp / rho);
  if (!(rho > 0.0) || !(w.p > 0.0) || !isfinite(c) || !isfinite(w.u) || !isfinite(w.v))
    bad = true;
  amax = fmax(amax, fabs(w.u) + c);
  bmax = fmax(bmax, fabs(w.v) + c);
  rmin = fmin(rmin, rho);
}

// A double moved across lanes by a DPP pattern (both 32-bit halves); lanes
// without a source lane, and rows the row mask leaves out, get `ident`.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v, double ident) {
  const long long b = __double_as_longlong(v), id = __double_as_longlong(ident);
  const int lo = __builtin_amdgcn_update_dpp((int)id, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(id >> 32), (int)(b >> 32), CTRL, ROWS, 0xf,
                                             false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

// Maximum (MAX) or minimum over the 64 lanes of the wave, in VALU lane moves:
// row shifts by 1, 2, 4, 8 leave each row's extremum in its lane 15, the
// broadcasts of lanes 15 and 31 carry it into rows 1 and 3 and then rows 2
// and 3, so lane 63 ends with the wave's extremum, which is read out.
template <bool MAX>
__device__ __forceinline__ double wave_extremum(double x) {
  const double id = MAX ? -__builtin_inf() : __builtin_inf();
  auto op = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
  x = op(x, dpp_f64<0x111, 0xf>(x, id));   // row_shr:1
  x = op(x, dpp_f64<0x112, 0xf>(x, id));   // row_shr:2
  x = op(x, dpp_f64<0x114, 0xf>(x, id));   // row_shr:4
  x = op(x, dpp_f64<0x118, 0xf>(x, id));   // row_shr:8
  x = op(x, dpp_f64<0x142, 0xa>(x, id));   // row_bcast:15 into rows 1, 3
  x = op(x, dpp_f64<0x143, 0xc>(x, id));   // row_bcast:31 into rows 2, 3
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

// Wave extrema written to slot `slot` of the partial arrays w[3][nslot]
// (plain stores, no barrier; the time-step kernels reduce the slots).  With
// square cells (dx = dy) min(fl(dx/a), fl(dy/b)) = fl(dx/max(a, b)), so one
// maximum serves both slots; without viscosity min rho is not needed.  Every
// lane of the wave calls it (square, visc uniform).
__device__ __forceinline__ void dt_extrema_commit(double* w, int nslot, int slot, double a,
                                                  double b, double r, bool square, bool visc) {
  if (square) a = fmax(a, b);
  a = wave_extremum<true>(a);
  if (!square) b = wave_extremum<true>(b);
  if (visc) r = wave_extremum<false>(r);
  if (__lane_id() == 0) {
    w[slot] = a;
    w[nslot + slot] = square ? a : b;
    w[2 * nslot + slot] = visc ? r : __builtin_inf();
  }
}

// Residual store or SSP-RK3 stage update, eq. (rk), for the cells this
// thread owns (c = tid + k NT, row-major in the tile); one coalesced FP64
// store per conserved variable.  Stage 3 with P.dtx set also reduces the
// time-step extrema of the new state.
template <class C>
__device__ __forceinline__ void stage_store(const StageParams& P, const double (&res)[C::CPT][4],
                                            int tx0, int ty0) {
  constexpr int NT = C::NT;
  const int tid = threadIdx.x;
  const size_t n = (size_t)P.nx * P.ny;
  const double dt = (P.mode == MODE_RESIDUAL) ? 0.0 : *P.dt;
  double qn[C::CPT][4], qk[C::CPT][4];
  bool own[C::CPT];
  size_t so[C::CPT];
#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
    int lx, ly;
    const bool in = tile_cell<C>(tid, k, lx, ly);
    const int gj = tx0 + lx, gi = ty0 + ly;
    own[k] = in && gj < P.nx && gi < P.ny;
    so[k] = (size_t)gi * P.nx + gj;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      qn[k][m] = (own[k] && P.mode != MODE_RESIDUAL) ? P.Qn[m * n + so[k]] : 0.0;
      qk[k][m] = (own[k] && P.mode >= MODE_STAGE2) ? P.Qk[m * n + so[k]] : 0.0;
    }
  }
  double v[C::CPT][4];
#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double R = res[k][m];
      if (P.mode == MODE_RESIDUAL)
        v[k][m] = R;
      else if (P.mode == MODE_STAGE1)
        v[k][m] = qn[k][m] + dt * R;
      else if (P.mode == MODE_STAGE2)
        v[k][m] = 0.75 * qn[k][m] + 0.25 * qk[k][m] + (0.25 * dt) * R;
      else
        v[k][m] = (1.0 / 3.0) * qn[k][m] + (2.0 / 3.0) * qk[k][m] + ((2.0 / 3.0) * dt) * R;
    }
  }
  float prp[C::CPT];
  if (P.dtx || P.rp) {
    // the time-step extrema of the new state, before the stores (stores
    // first would make the wave wait for them before reusing their registers)
    double amax = 0.0, bmax = 0.0, rmin = __builtin_inf();
    bool bad = false;
#pragma unroll
    for (int k = 0; k < C::CPT; ++k) {
      if (!own[k]) continue;
      const CellUVP w = cell_uvp(v[k], P.gamma);
      prp[k] = (float)w.p;
      if (P.dtx) dt_extrema_cell(v[k], w, P.gamma, amax, bmax, rmin, bad);
    }
    if (P.dtx) {
      if (bad) atomicOr(P.status, 1u);
      constexpr int NW = NT / 64;
      dt_extrema_commit(P.dtx, P.ntiles * NW, blockIdx.x * NW + (threadIdx.x >> 6), amax, bmax,
                        rmin, P.dx == P.dy, P.mu > 0.0);
    }
  }
#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
    if (!own[k]) continue;
#pragma unroll
    for (int m = 0; m < 4; ++m) P.out[m * n + so[k]] = v[k][m];
    if (P.rp) {
      P.rp[so[k]] = (float)v[k][0];
      P.rp[n + so[k]] = prp[k];
    }
  }
}

// One tile of the stage: load, both sweeps, store.  The LDS arrays are
// passed in so that a kernel can run several tile shapes from one set of
// arrays sized for the largest (the batched kernel).
template <class C, bool DETMLP, bool CONS = false, int ORD = 7, bool LM = false,
          bool MPE = false>
__device__ __forceinline__ void stage_tile(const StageParams& P, int tx0, int ty0, double* sU,
                                           double* sPh, unsigned char* sChi,
                                           unsigned short* sQueue, int* sQCount,
                                           unsigned char* sChiF) {
  ChiMap<C> cm;
  if (DETMLP) fetch_chimap<C>(P, cm, tx0, ty0);
  stage_load<C, CONS, C::template Layout<edge_form<CONS, MPE>()>::TFIELD>(P, sU, tx0, ty0);
  if (DETMLP) put_chimap<C>(cm, sChiF);
  __syncthreads();
  const Lds L{sU, sPh, sChi, sQueue, sQCount, sChiF};
  double res[C::CPT][4];
#pragma unroll
  for (int k = 0; k < C::CPT; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) res[k][m] = 0.0;
  for (int l0 = 0; l0 < C::TY; l0 += C::SX)
    sweep<C, 0, DETMLP, CONS, ORD, LM, MPE>(P, L, l0, tx0, ty0, res);
  for (int l0 = 0; l0 < C::TX; l0 += C::SY)
    sweep<C, 1, DETMLP, CONS, ORD, LM, MPE>(P, L, l0, tx0, ty0, res);
  stage_store<C>(P, res, tx0, ty0);
}

// The MP test at every interface needs more registers than any budget of
// three waves per SIMD leaves without spilling: those variants get two.
template <class C, bool DETMLP, bool CONS = false, int ORD = 7, bool LM = false, bool MPE = false>
__global__ __launch_bounds__(C::NT, (MPE && C::MINW > 2) ? 2 : C::MINW) void meg7_stage_kernel(
    StageParams P) {
  using LY = typename C::template Layout<edge_form<CONS, MPE>()>;
  __shared__ double sU[LY::NFU * C::RS];
  __shared__ double sPh[LY::PH];
  __shared__ unsigned char sChi[C::CHI];
  __shared__ unsigned short sQueue[C::QMAX];
  __shared__ unsigned char sChiF[DETMLP ? (C::TX + 6) * (C::TY + 6) : 1];
  __shared__ int sQCount;
  int tx0, ty0;
  if (!tile_origin(P, C::TX, C::TY, tx0, ty0)) return;
  stage_tile<C, DETMLP, CONS, ORD, LM, MPE>(P, tx0, ty0, sU, sPh, sChi, sQueue, &sQCount,
                                            sChiF);
}

}  // namespace gbr
