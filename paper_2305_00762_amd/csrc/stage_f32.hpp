// FP32-bulk form of the fused MEG7 residual + stage kernel.
//
// The conserved state, the LDS tile of primitives, the detector (so the flags
// are the FP64 flags), the shock branch and the flux differencing stay in
// FP64.  The smooth-interface work -- GRB reconstruction, flux reconstruction,
// the Riemann solver, the viscous flux -- runs in FP32 on small local
// quantities only, so its rounding scales with the local variation of the
// solution rather than with its magnitude:
//   * per cell edge: jumps dU = U_{k+1} - U_k and df = f_{k+1} - f_k, formed
//     in FP64 (df on the primitive jumps) and rounded to FP32;
//   * GRB states as corrections: U^L = U_j + cL, U^R = U_{j+1} + cR, with cL, cR
//     written on edge jumps alone: eq. (eqn:grb) minus U_j (its value weights
//     sum to 840) with the gradients of eq. (eqn:six) expanded into the same
//     edge jumps, an 8-tap stencil on dU_{j-7/2} .. dU_{j+7/2} (resp. one edge
//     further right); U^R - U^L = dU_{j+1/2} + cR - cL;
//   * the mean reconstructed flux minus the central flux
//     B = (f_j + f_{j+1})/2 as a stencil on edge jumps (eqs. flux-full,
//     flux-right minus B: the weights sum to zero);
//   * HLLC written on the jumps (every wave jump is proportional to
//     S* - u_L or S* - u_R, themselves formed from dp and du).
// Each interface flux is F = B + d with d in FP32; the divergence is formed in
// FP64 as (f_{j+1} - f_{j-1})/2 + (d_{j+1/2} - d_{j-1/2}).
#pragma once
#include <type_traits>

#include "stage_kernel.hpp"

namespace gbr {

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsqf(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrtf_fast(float x) { return x * __builtin_amdgcn_rsqf(x); }

// HLLC (Einfeldt bounds) dissipation |S_L|(Q*_L-Q_L) + |S*|(Q*_R-Q*_L) +
// |S_R|(Q_R-Q*_R) from the left/right primitive states and their jump
// dW = W_R - W_L, every jump evaluated as a product of small quantities.
__device__ __forceinline__ void hllc_diss_f32(const float WL[4], const float WR[4],
                                              const float dW[4], float gamma, float g1inv,
                                              float diss[4]) {
  const float rl = WL[0], ul = WL[1], vl = WL[2], pl = WL[3];
  const float rr = WR[0], ur = WR[1], vr = WR[2], pr = WR[3];
  const float dr = dW[0], du = dW[1], dv = dW[2], dp = dW[3];
  const float yl = rsqf(rl), yr = rsqf(rr);
  const float sl = rl * yl, sr = rr * yr, irl = yl * yl, irr = yr * yr;
  const float kl2 = ul * ul + vl * vl, kr2 = ur * ur + vr * vr;
  const float El = pl * g1inv + 0.5f * rl * kl2;
  const float Er = pr * g1inv + 0.5f * rr * kr2;
  const float cl = sqrtf_fast(gamma * pl * irl), cr = sqrtf_fast(gamma * pr * irr);
  const float hl = (El + pl) * irl, hr = (Er + pr) * irr;
  const float iss = rcpf(sl + sr);
  const float ut = (sl * ul + sr * ur) * iss;
  const float vt = (sl * vl + sr * vr) * iss;
  const float ht = (sl * hl + sr * hr) * iss;
  const float ct = sqrtf_fast((gamma - 1.0f) * (ht - 0.5f * (ut * ut + vt * vt)));
  const float SL = fminf(ul - cl, ut - ct);
  const float SR = fmaxf(ur + cr, ut + ct);
  const float ml = rl * (SL - ul), mr = rr * (SR - ur);
  const float iden = rcpf(ml - mr);
  const float aL = (dp - du * mr) * iden;   // S* - u_L
  const float aR = (dp - du * ml) * iden;   // S* - u_R
  const float Ss = ul + aL;
  const float iL = rcpf(SL - Ss), iR = rcpf(SR - Ss);
  // Q_R - Q_L from the primitive jumps
  const float dQ[4] = {dr, rr * du + ul * dr, rr * dv + vl * dr,
                       dp * g1inv + 0.5f * (dr * kl2 + rr * (du * (ur + ul) + dv * (vr + vl)))};
  const float aSL = fabsf(SL), aSS = fabsf(Ss), aSR = fabsf(SR);
  // |S_L| dQL + |S*| (dQ - dQR - dQL) + |S_R| dQR gathered per jump as
  // (|S_L| - |S*|) dQL + (|S_R| - |S*|) dQR + |S*| dQ, with
  //   dQL = Q*_L - Q_L = g_L (1, S_L, v_L, .),  g_L = rho_L a_L / (S_L - S*),
  //   dQR = Q_R - Q*_R = -g_R (1, S_R, v_R, .), g_R = rho_R a_R / (S_R - S*),
  // and the energy rows a_L/(S_L - S*) (E_L + p_L + m_L S*), resp. R
  const float aiL = aL * iL, aiR = aR * iR;
  const float wL = aSL - aSS, wR = aSR - aSS;
  const float GL = wL * (rl * aiL), GR = wR * (rr * aiR);
  const float HL = wL * aiL * (El + pl + ml * Ss), HR = wR * aiR * (Er + pr + mr * Ss);
  diss[0] = (GL - GR) + aSS * dQ[0];
  diss[1] = (GL * SL - GR * SR) + aSS * dQ[1];
  diss[2] = (GL * vl - GR * vr) + aSS * dQ[2];
  diss[3] = (HL - HR) + aSS * dQ[3];
}

// Per-line buffers of a sweep, for the four reconstructed fields: edge jumps
// of the primitives and of the cell fluxes.  No gradient buffer: the smooth
// branch reads gradients only through its edge-jump stencils (the viscous
// normal derivatives likewise), and the flagged branch forms its gradients
// from the same edge jumps.
//
// Bank layout.  Pass 2 gives one interface to a lane, WFL = N + 1 interfaces
// per line, so a half-wave (the 32 lanes one LDS cycle serves on 32 banks)
// covers G = 32 / WFL lines when WFL divides 32.  Row-major rows would then
// put those lines' reads at offsets W apart, which collide on the banks for
// every row width W that fits.  Instead the rows of each group of G lines are
// interleaved element by element -- element p of line g0 + i at word
// g0 W + G p + i -- so the half-wave reads G consecutive words per position:
// 32 distinct banks.  The line count is padded to whole groups (NLP), which
// keeps the stride G a constant.
template <int N, int NL, int NE = 4>
struct PhaseF32 {
  // edge jumps df at k+1/2, k in [-5, N+4), and dU, k in [-6, N+5) (pass 1,
  // one edge per item; the two outermost dU where a line end is flagged, for
  // the flagged branch's gradients); plain-detector flags at k in [-3, N+3)
  static constexpr int WU = N + 11, WG = N + 9, WFL = N + 1, WP = N + 9, WD = N + 6;
  static constexpr int G = (32 % WFL == 0) ? 32 / WFL : 1;
  static constexpr int NLP = (NL + G - 1) / G * G;
  // interface values d (pass 2/3 writes, pass 4 reads across lines in y):
  // width WFL + 2 under interleaving, else the odd width WFL | 1
  static constexpr int WFS = G > 1 ? WFL + 2 : (WFL | 1);
  // NE fields of primitive edge jumps (viscous: T = gamma p / rho as a fifth)
  static constexpr int TOT = NE * NLP * WU + 4 * NLP * (WG > WFL ? WG : WFL);
  static constexpr int CHI = NLP * WD;   // plain-detector flags
  __device__ static __forceinline__ int idx(int line, int p, int W) {
    return line / G * G * W + G * p + line % G;
  }
};

// The FP32 kernel's tile holds (rho, u, v, p) in FP64 also on viscous grids:
// T = gamma p / rho is formed where the viscous flux needs it, which keeps
// the viscous kernel at the inviscid one's LDS size (4 workgroups per CU).
// Flagged-interface queue entries are interface slots, bytes where they fit.
template <class C>
struct F32Cfg {
  using PX = PhaseF32<C::TX, C::SX, C::VISC ? 5 : 4>;
  using PY = PhaseF32<C::TY, C::SY, C::VISC ? 5 : 4>;
  static constexpr int NU = 4;                          // tile fields
  static constexpr int PH = C::cmax(PX::TOT, PY::TOT);  // floats
  static constexpr int CHI = C::cmax(PX::CHI, PY::CHI);
  static constexpr int QMAX = C::QMAX;
  using QT = typename std::conditional<(QMAX <= 256), unsigned char, unsigned short>::type;
  static constexpr int LDS_BYTES =
      8 * NU * C::RS + 4 * PH + CHI + (int)sizeof(QT) * QMAX + 16;
};

template <class QT>
struct LdsF32 {
  double* U;
  float* ph;
  unsigned char* chi;         // plain-detector flags (unused with the flag map)
  QT* queue;
  int* qcount;
  const unsigned char* chif;  // flag-map bits of the tile cells (learned detector)
};

template <class C, int DIR, bool DETMLP, class QT>
__device__ __forceinline__ void sweep_f32(const StageParams& P, const LdsF32<QT>& L, int l0,
                                          int tx0, int ty0, double (&res)[C::CPT][4]) {
  constexpr bool X = (DIR == 0);
  constexpr int N = X ? C::TX : C::TY;
  constexpr int NL = X ? C::SX : C::SY;
  constexpr int NLINES = X ? C::TY : C::TX;
  constexpr int NE = C::VISC ? 5 : 4;
  using PH = PhaseF32<N, NL, NE>;
  constexpr int WD = PH::WD, WU = PH::WU, WG = PH::WG, WFL = PH::WFL, WP = PH::WP;
  constexpr int NLP = PH::NLP;
  constexpr int RS = C::RS, RX = C::RX, H = C::H, NT = C::NT;
  constexpr int SN = X ? 1 : RX, ST = X ? RX : 1;
  constexpr int FN = X ? 1 : 2, FT = X ? 2 : 1;
  constexpr int IPT = (NL * WFL + NT - 1) / NT;
  constexpr int GSTR = (WG > WFL ? WG : WFL) * NLP;
  constexpr int WFS = PH::WFS;
  static_assert(WFS <= WG, "interface rows fit the buffer");
  const int tid = threadIdx.x;
  const int nl = (NLINES - l0) < NL ? (NLINES - l0) : NL;
  const double inv_dn = X ? P.inv_dx : P.inv_dy;
  const double inv_dt = X ? P.inv_dy : P.inv_dx;
  const float gammaf = (float)P.gamma, g1invf = (float)P.g1inv;

  float* sDU = L.ph;                 // [4][NLP x WU]   edge jumps of the primitives (rotated order)
  float* sDF = sDU + NE * NLP * WU;  // [4][NLP x WG]   edge jumps of the cell fluxes; then d
  auto bidx = [](int line, int p, int W) { return PH::idx(line, p, W); };
  auto ridx = [&](int line, int pos) {
    const int lx = X ? pos : l0 + line;
    const int ly = X ? l0 + line : pos;
    return (ly + H) * RX + (lx + H);
  };
  const int rot[5] = {0, FN, FT, 3, 4};
  const double* U = L.U;
  auto wrot = [&](int r, double W[4]) {
    W[0] = U[r]; W[1] = U[FN * RS + r]; W[2] = U[FT * RS + r]; W[3] = U[3 * RS + r];
  };
  // Sixth-order derivative of tile field f at cell r along stride d (eq. (eqn:six)).
  auto g6 = [&](int f, int r, int d) {
    const double* u = U + f * RS + r;
    return grad6(u[-3 * d], u[-2 * d], u[-d], u[d], u[2 * d], u[3 * d]);
  };
  // T = gamma p / rho at the eight cells r + (j - 3) SN, j = 0..7, that the
  // viscous flux of interface r + 1/2 reads (the arithmetic of the tile load:
  // one refined reciprocal of rho)
  auto temps = [&](int r, double (&T)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = r + (j - 3) * SN;
      T[j] = P.gamma * U[3 * RS + k] * rcp_nr(U[k]);
    }
  };

  // ---- pass 1: per edge, from the FP64 tile ----------------------------------
  // item p: edge k+1/2, k = p - 5 in [-5, N+4); plain flags at k in [-3, N+3)
  constexpr int P1R = (NL * WP + NT - 1) / NT;
  auto pass1 = [&](int t) {
    const int line = t / WP;
    const int p = t % WP;
    if (line >= nl) return;
    const int k = p - 5;
    const int r = ridx(line, k);
    double W0[4], W1[4], df[4];
    wrot(r, W0);
    wrot(r + SN, W1);
    conv_flux_jump(W0, W1, P.g1inv, df);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      sDF[m * GSTR + bidx(line, p, WG)] = (float)df[m];
      sDU[m * NLP * WU + bidx(line, p + 1, WU)] = (float)(W1[m] - W0[m]);
    }
    if (C::VISC) {
      // T = gamma p / rho with the tile load's arithmetic (one refined
      // reciprocal of rho), its edge jump as a fifth field
      const double T0 = P.gamma * W0[3] * rcp_nr(W0[0]);
      const double T1 = P.gamma * W1[3] * rcp_nr(W1[0]);
      sDU[4 * NLP * WU + bidx(line, p + 1, WU)] = (float)(T1 - T0);
    }
    if (!DETMLP && k >= -3 && k < N + 3) {
      const double* rho = U + r;
      L.chi[bidx(line, k + 3, WD)] =
          detector_flag(rho[-2 * SN], rho[-SN], rho[0], rho[SN], rho[2 * SN]) ? 1 : 0;
    }
  };
  if constexpr (DETMLP) {
#pragma unroll
    for (int k1 = 0; k1 < P1R; ++k1)
      if (tid + k1 * NT < NL * WP) pass1(tid + k1 * NT);
  } else {
    // rounds kept apart: the FP64 density detector's registers would
    // otherwise overlap the next round's loads past the 128-VGPR budget
#pragma unroll 1
    for (int k1 = 0; k1 < P1R; ++k1)
      if (tid + k1 * NT < NL * WP) pass1(tid + k1 * NT);
  }
  if (tid == 0) *L.qcount = 0;
  __syncthreads();

  // ---- pass 2: smooth interfaces in FP32; ballot-compact the flagged ----------
  float dsm[IPT][4];
  bool has[IPT];
#pragma unroll
  for (int kk = 0; kk < IPT; ++kk) {
    has[kk] = false;
    const int t = tid + kk * NT;
    bool flagged = false;
    if (t < NL * WFL) {
      const int line = t / WFL;
      const int p = t % WFL;
      const int pos = p - 1;
      if (line < nl) {
        // eq. (buffer): the six flags read at once and OR-ed (a short-circuit
        // chain would wait for each LDS read in turn)
        // (flag-map bits are read from the tile's flag map directly)
        unsigned any = 0u;
        if (DETMLP) {
#pragma unroll
          for (int q = 1; q <= 6; ++q) {
            const int k = pos + q - 3;
            any |= L.chif[mlp_chi_index<C>(X ? k : l0 + line, X ? l0 + line : k)];
          }
          any &= 1u << DIR;
        } else {
#pragma unroll
          for (int q = 1; q <= 6; ++q) any |= L.chi[bidx(line, pos + q, WD)];
        }
        const bool sigma = any == 0u;
        if (X) {
          const int gi = ty0 + l0 + line, gj = tx0 + pos;
          if (P.sigx && gi < P.ny && gj < P.nx) P.sigx[(size_t)gi * (P.nx + 1) + gj + 1] = sigma;
        } else {
          const int gj = tx0 + l0 + line, gi = ty0 + pos;
          if (P.sigy && gj < P.nx && gi < P.ny) P.sigy[(size_t)(gi + 1) * P.nx + gj] = sigma;
        }
        flagged = !sigma;
        if (flagged && (pos == -1 || pos == N - 1)) {
          // the edge past pass 1's range that the flagged branch's gradients
          // reach at a line end: (-6)+1/2 or (N+4)+1/2
          const int r = ridx(line, pos);
          const int o = pos < 0 ? -5 : 5, ix = pos < 0 ? 0 : WU - 1;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const double* u = U + rot[m] * RS + r + o * SN;
            sDU[m * NLP * WU + bidx(line, ix, WU)] = (float)(u[SN] - u[0]);
          }
        }
        if (sigma) {
          const int r = ridx(line, pos);
          float WL[4], WR[4], dW[4], dF[4];
          float gv[2][2], jv[2];   // viscous: normal derivatives of u_n, u_t at pos, pos+1; jumps
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            // edge jumps E[a] = dU at (pos+a-4)+1/2, a = 0..8
            float E[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) E[a] = sDU[m * NLP * WU + bidx(line, pos + 2 + a, WU)];
            // eq. (eqn:grb) with eq. (eqn:six) substituted, minus U_j (resp. U_{j+1});
            // integer weights over 840
            constexpr float s = 1.0f / 840.0f;
            const float cL = s * ((E[0] - E[1] - E[7]) - 23.0f * E[2] + 123.0f * E[3] +
                                  395.0f * E[4] - 89.0f * E[5] + 15.0f * E[6]);
            const float cR = s * ((E[1] - E[8] + E[7]) - 15.0f * E[2] + 89.0f * E[3] -
                                  395.0f * E[4] - 123.0f * E[5] + 23.0f * E[6]);
            const double* u = U + rot[m] * RS + r;
            WL[m] = (float)u[0] + cL;
            WR[m] = (float)u[SN] + cR;
            dW[m] = E[4] + (cR - cL);
            if (C::VISC && (m == 1 || m == 2)) {
              // eq. (eqn:six) at pos and pos+1 on the edge jumps (weights over 60)
              constexpr float z = 1.0f / 60.0f;
              gv[m - 1][0] = z * (37.0f * (E[3] + E[4]) - 8.0f * (E[2] + E[5]) + (E[1] + E[6]));
              gv[m - 1][1] = z * (37.0f * (E[4] + E[5]) - 8.0f * (E[3] + E[6]) + (E[2] + E[7]));
              jv[m - 1] = E[4];
            }
            // mean reconstructed flux minus (f_j + f_{j+1})/2 on flux edge jumps
            // h[q] at (pos-4+q)+1/2, q = 0..8
            float h[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) h[q] = sDF[m * GSTR + bidx(line, pos + 1 + q, WG)];
            constexpr float w = 1.0f / 1680.0f;
            dF[m] = w * (212.0f * (h[3] - h[5]) - 38.0f * (h[2] - h[6]) + (h[0] - h[8]));
          }
          if (!(WL[0] > 0.f && WL[3] > 0.f && WR[0] > 0.f && WR[3] > 0.f)) {
            // unphysical reconstruction: first-order states, central flux
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              WL[m] = (float)U[rot[m] * RS + r];
              WR[m] = (float)U[rot[m] * RS + r + SN];
              dW[m] = sDU[m * NLP * WU + bidx(line, pos + 6, WU)];
              dF[m] = 0.f;
            }
          }
          float diss[4];
          hllc_diss_f32(WL, WR, dW, gammaf, g1invf, diss);
#pragma unroll
          for (int m = 0; m < 4; ++m) dsm[kk][m] = dF[m] - 0.5f * diss[m];
          if (C::VISC) {
            const float gun0 = gv[0][0], gun1 = gv[0][1];
            const float gut0 = gv[1][0], gut1 = gv[1][1];
            // T's normal derivative at pos and pos+1 and its jump, on its edge
            // jumps as u_n's and u_t's (ET[a] = dT at (pos+a-4)+1/2)
            float ET[8];
#pragma unroll
            for (int a = 1; a < 8; ++a) ET[a] = sDU[4 * NLP * WU + bidx(line, pos + 2 + a, WU)];
            constexpr float z = 1.0f / 60.0f;
            const float gT0 = z * (37.0f * (ET[3] + ET[4]) - 8.0f * (ET[2] + ET[5]) + (ET[1] + ET[6]));
            const float gT1 = z * (37.0f * (ET[4] + ET[5]) - 8.0f * (ET[3] + ET[6]) + (ET[2] + ET[7]));
            const float jun = jv[0], jut = jv[1];
            const float jT = ET[4];
            const float a2 = 0.5f * (float)kAlphaV, idn = (float)inv_dn;
            const float dun = (0.5f * (gun0 + gun1) + a2 * (jun - 0.5f * (gun0 + gun1))) * idn;
            const float dut = (0.5f * (gut0 + gut1) + a2 * (jut - 0.5f * (gut0 + gut1))) * idn;
            const float dT = (0.5f * (gT0 + gT1) + a2 * (jT - 0.5f * (gT0 + gT1))) * idn;
            const float dunt = 0.5f * ((float)(g6(FN, r, ST) * inv_dt) +
                                       (float)(g6(FN, r + SN, ST) * inv_dt));
            const float dutt = 0.5f * ((float)(g6(FT, r, ST) * inv_dt) +
                                       (float)(g6(FT, r + SN, ST) * inv_dt));
            const float unf = 0.5f * ((float)U[FN * RS + r] + (float)U[FN * RS + r + SN]);
            const float utf = 0.5f * ((float)U[FT * RS + r] + (float)U[FT * RS + r + SN]);
            const float muf = (float)P.mu;
            const float tnn = (2.0f / 3.0f) * muf * (2.0f * dun - dutt);
            const float tnt = muf * (dut + dunt);
            const float qn = -(float)P.kq * dT;
            dsm[kk][1] -= tnn;
            dsm[kk][2] -= tnt;
            dsm[kk][3] += -(tnn * unf + tnt * utf) + qn;
          }
          has[kk] = true;
        }
      }
    }
    const unsigned long long ball = __ballot(flagged);
    if (ball) {
      const int lane = __lane_id();
      int base = 0;
      if (lane == 0) base = atomicAdd(L.qcount, (int)__popcll(ball));
      base = __shfl(base, 0);
      if (flagged) {
        const int rank = (int)__popcll(ball & ((1ull << lane) - 1ull));
        L.queue[base + rank] = (QT)t;
      }
    }
  }
  __syncthreads();  // edge flux jumps consumed: the buffer now holds d per interface
#pragma unroll
  for (int kk = 0; kk < IPT; ++kk) {
    if (has[kk]) {
      const int t = tid + kk * NT;
      const int line = t / WFL;
      const int p = t % WFL;
#pragma unroll
      for (int m = 0; m < 4; ++m) sDF[m * GSTR + bidx(line, p, WFS)] = dsm[kk][m];
    }
  }

  // ---- pass 3: flagged interfaces in FP64 (characteristic MEG7, F(Q)) -------
  const int nq = *L.qcount;
  for (int qi = tid; qi < nq; qi += NT) {
    const int t = L.queue[qi];
    const int line = t / WFL;
    const int p = t % WFL;
    const int pos = p - 1;
    const int r = ridx(line, pos);
    // normal gradients (eq. eqn:six) on the edge jumps, as in the smooth
    // branch: edge(f, a) = dU of rotated field f at (pos+a-5)+1/2, a = 0..10
    auto edge = [&](int f, int a) -> float {
      return sDU[f * NLP * WU + bidx(line, pos + 1 + a, WU)];
    };
    // at pos + q - 2, q = 0..5
    auto grad = [&](int q, int f) -> float {
      constexpr float z = 1.0f / 60.0f;
      return z * (37.0f * (edge(f, q + 2) + edge(f, q + 3)) -
                  8.0f * (edge(f, q + 1) + edge(f, q + 4)) + (edge(f, q) + edge(f, q + 5)));
    };
    double WL[4], WR[4];
    meg7_char_states(
        [&](int q, int f) { return U[rot[f] * RS + r + (q - 2) * SN]; },
        [&](int q, int f) { return (double)grad(q, f); },
        P.gamma, WL, WR);
    if (!(WL[0] > 0.0 && WL[3] > 0.0 && WR[0] > 0.0 && WR[3] > 0.0)) {
      wrot(r, WL);
      wrot(r + SN, WR);
    }
    double FL[4], FR[4], Fm[4], F[4], W0[4], W1[4], f0[4], f1[4];
    conv_flux(WL, P.g1inv, FL);
    conv_flux(WR, P.g1inv, FR);
#pragma unroll
    for (int m = 0; m < 4; ++m) Fm[m] = 0.5 * (FL[m] + FR[m]);
    hllc(WL, WR, Fm, P.gamma, P.g1inv, F);
    if (C::VISC) {
      double T[8];
      temps(r, T);
      viscous_add(U[FN * RS + r], U[FN * RS + r + SN], U[FT * RS + r], U[FT * RS + r + SN],
                  T[3], T[4], grad(2, 1), grad(3, 1), grad(2, 2), grad(3, 2),
                  (float)grad6(T[0], T[1], T[2], T[4], T[5], T[6]),
                  (float)grad6(T[1], T[2], T[3], T[5], T[6], T[7]), (float)(g6(FN, r, ST) * inv_dt),
                  (float)(g6(FN, r + SN, ST) * inv_dt), (float)(g6(FT, r, ST) * inv_dt),
                  (float)(g6(FT, r + SN, ST) * inv_dt), inv_dn, P.mu, P.kq, F);
    }
    wrot(r, W0);
    wrot(r + SN, W1);
    conv_flux(W0, P.g1inv, f0);
    conv_flux(W1, P.g1inv, f1);
#pragma unroll
    for (int m = 0; m < 4; ++m) sDF[m * GSTR + bidx(line, p, WFS)] = (float)(F[m] - 0.5 * (f0[m] + f1[m]));
  }
  __syncthreads();

  // ---- pass 4: divergence in FP64: (f_{j+1} - f_{j-1})/2 + d_{j+1/2} - d_{j-1/2}
#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
    int lx, ly;
    if (tile_cell<C>(tid, k, lx, ly)) {
      const int line = (X ? ly : lx) - l0;
      const int pos = X ? lx : ly;
      if (line >= 0 && line < nl) {
        const int r = ridx(line, pos);
        double Wm[4], Wp[4], dfc[4];
        wrot(r - SN, Wm);
        wrot(r + SN, Wp);
        conv_flux_jump(Wm, Wp, P.g1inv, dfc);
        const int bp = bidx(line, pos + 1, WFS), bm = bidx(line, pos, WFS);
        double d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
          d[m] = 0.5 * dfc[m] + ((double)sDF[m * GSTR + bp] - (double)sDF[m * GSTR + bm]);
        res[k][0] -= d[0] * inv_dn;
        res[k][FN] -= d[1] * inv_dn;
        res[k][FT] -= d[2] * inv_dn;
        res[k][3] -= d[3] * inv_dn;
      }
    }
  }
  __syncthreads();
}

// One tile of the FP32-bulk stage (LDS arrays passed in, as stage_tile).
template <class C, bool DETMLP, class QT>
__device__ __forceinline__ void stage_tile_f32(const StageParams& P, int tx0, int ty0, double* sU,
                                               float* sPh, unsigned char* sChi, QT* sQueue,
                                               int* sQCount, unsigned char* sChiF) {
  static_assert(C::QMAX <= (1 << (8 * sizeof(QT))), "queue entries hold every interface slot");
  ChiMap<C> cm;
  if (DETMLP) fetch_chimap<C>(P, cm, tx0, ty0);
  stage_load<C, false, false>(P, sU, tx0, ty0);
  if (DETMLP) put_chimap<C>(cm, sChiF);
  __syncthreads();
  const LdsF32<QT> L{sU, sPh, sChi, sQueue, sQCount, sChiF};
  double res[C::CPT][4];
#pragma unroll
  for (int k = 0; k < C::CPT; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) res[k][m] = 0.0;
  for (int l0 = 0; l0 < C::TY; l0 += C::SX) sweep_f32<C, 0, DETMLP>(P, L, l0, tx0, ty0, res);
  for (int l0 = 0; l0 < C::TX; l0 += C::SY) sweep_f32<C, 1, DETMLP>(P, L, l0, tx0, ty0, res);
  stage_store<C>(P, res, tx0, ty0);
}

template <class C, bool DETMLP>
__global__ __launch_bounds__(C::NT, C::MINW) void meg7_stage_kernel_f32(StageParams P) {
  using F = F32Cfg<C>;
  __shared__ double sU[F::NU * C::RS];
  __shared__ float sPh[F::PH];
  __shared__ unsigned char sChi[DETMLP ? 1 : F::CHI];
  __shared__ typename F::QT sQueue[F::QMAX];
  __shared__ unsigned char sChiF[DETMLP ? (C::TX + 6) * (C::TY + 6) : 1];
  __shared__ int sQCount;
  int tx0, ty0;
  if (!tile_origin(P, C::TX, C::TY, tx0, ty0)) return;
  stage_tile_f32<C, DETMLP>(P, tx0, ty0, sU, sPh, sChi, sQueue, &sQCount, sChiF);
}

}  // namespace gbr
