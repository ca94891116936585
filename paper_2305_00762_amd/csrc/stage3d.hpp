// MEG7 in three dimensions (the Euler equations, inviscid) for gfx950.
//
// The method is applied dimension by dimension, so each direction is one
// kernel over lines along that direction.  A workgroup owns NL lines x NP
// positions plus a 6-cell halo along the line (periodic wrap or transmissive
// clamp), stages the primitives in a frame rotated to the line,
// (rho, u_n, u_t1, u_t2, p) with the tangential components taken cyclically
// (x: v, w; y: w, u; z: u, v), and runs the passes of the 2D sweep:
//   pass 1: cell fluxes, sixth-order gradients (eq. eqn:six), the density
//           detector (Sec. 2.4);
//   pass 2: per interface, sigma from the 6-cell buffer; smooth interfaces take
//           the GRB states, the flux reconstruction and HLLC; flagged ones are
//           compacted into an LDS queue by a wavefront ballot;
//   pass 3: the queue: characteristic MEG7 states (Sec. 2.3), F(Q), HLLC;
//   pass 4: flux differences into the residual accumulator.
// The x sweep writes R = -dF/dx, the y sweep subtracts dG/dy, the z sweep
// subtracts dH/dz and stores the residual or the SSP-RK3 stage (eq. rk).
#pragma once
#include "meg7_device.hpp"
#include "stage_kernel.hpp"

namespace gbr {

struct Sweep3Params {
  const double* __restrict__ Qk;  // state the residual is evaluated on [5][nz][ny][nx]
  const double* __restrict__ Qn;  // Q^n (stages 2, 3)
  double* R;                      // residual accumulator [5][nz][ny][nx]
  double* out;                    // residual or Q^(k+1) (last sweep)
  const double* __restrict__ dt;  // device scalar (stages)
  uint8_t* sig;                   // optional interface flags of this direction
  unsigned* status;
  int nx, ny, nz;
  int bc;                         // boundary kind along this direction
  double inv_d;                   // 1 / spacing along this direction
  double gamma, g1inv;
  int first, last;                // first sweep writes R; the last one stores
  int mode;                       // MODE_RESIDUAL or MODE_STAGE1..3
  int ptiles;                     // position tiles along the direction
  // last sweep of stage 3 only (else null): per-wave time-step extrema of
  // the output, [3][gridDim.x x 4]: max(|u|+c), max(|v|+c), max(|w|+c)
  double* dtx;
};

// |u|+c, |v|+c, |w|+c of one cell of the new state, each rounded as the
// time-step kernel rounds them (IEEE division and square root, one rounding
// per operation), folded into (ea, eb, ec); since fl(d/x) is monotone in x,
// the minima of the per-cell limits follow from the maxima without loss.
__device__ __forceinline__ void dt3_extrema_cell(const double q[5], double gamma, double& ea,
                                                 double& eb, double& ec, bool& bad) {
#pragma clang fp contract(off)
  const double rho = q[0];
  const double u = q[1] / rho, v = q[2] / rho, w = q[3] / rho;
  const double p = (gamma - 1.0) * (q[4] - rho * (u * u + v * v + w * w) / 2.0);
  const double c = sqrt(gamma * p / rho);
  if (!(rho > 0.0) || !(p > 0.0) || !isfinite(c) || !isfinite(u) || !isfinite(v) ||
      !isfinite(w))
    bad = true;
  ea = fmax(ea, fabs(u) + c);
  eb = fmax(eb, fabs(v) + c);
  ec = fmax(ec, fabs(w) + c);
}

// Normal convective flux of W = (rho, u_n, u_t1, u_t2, p).
__device__ __forceinline__ void conv_flux3(const double W[5], double g1inv, double F[5]) {
  const double E = W[4] * g1inv + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  const double m = W[0] * W[1];
  F[0] = m;
  F[1] = m * W[1] + W[4];
  F[2] = m * W[2];
  F[3] = m * W[3];
  F[4] = W[1] * (E + W[4]);
}

// HLLC with Einfeldt (Roe-average) bounds in the wave-sum form, both
// tangential momenta carried by the star states (as the 2D hllc).
__device__ __forceinline__ void hllc3(const double WL[5], const double WR[5], const double Fm[5],
                                      double gamma, double g1inv, double F[5]) {
  const double rl = WL[0], ul = WL[1], vl = WL[2], wl = WL[3], pl = WL[4];
  const double rr = WR[0], ur = WR[1], vr = WR[2], wr = WR[3], pr = WR[4];
  const double yl = rsq_nr(rl), yr = rsq_nr(rr);
  const double sl = rl * yl, sr = rr * yr;
  const double irl = yl * yl, irr = yr * yr;
  const double El = pl * g1inv + 0.5 * rl * (ul * ul + vl * vl + wl * wl);
  const double Er = pr * g1inv + 0.5 * rr * (ur * ur + vr * vr + wr * wr);
  const double cl = sqrt_nr(gamma * pl * irl), cr = sqrt_nr(gamma * pr * irr);
  const double hl = (El + pl) * irl, hr = (Er + pr) * irr;
  const double iss = rcp_nr(sl + sr);
  const double ut = (sl * ul + sr * ur) * iss;
  const double vt = (sl * vl + sr * vr) * iss;
  const double wt = (sl * wl + sr * wr) * iss;
  const double ht = (sl * hl + sr * hr) * iss;
  const double ct = sqrt_nr((gamma - 1.0) * (ht - 0.5 * (ut * ut + vt * vt + wt * wt)));
  const double SL = fmin(ul - cl, ut - ct);
  const double SR = fmax(ur + cr, ut + ct);
  const double ml = rl * (SL - ul), mr = rr * (SR - ur);
  const double Ss = (pr - pl + ml * ul - mr * ur) * rcp_nr(ml - mr);
  const double kl = ml * rcp_nr(SL - Ss), kr = mr * rcp_nr(SR - Ss);
  const double QL[5] = {rl, rl * ul, rl * vl, rl * wl, El};
  const double QR[5] = {rr, rr * ur, rr * vr, rr * wr, Er};
  const double QsL[5] = {kl, kl * Ss, kl * vl, kl * wl,
                         kl * (El * irl + (Ss - ul) * (Ss + pl * rcp_nr(ml)))};
  const double QsR[5] = {kr, kr * Ss, kr * vr, kr * wr,
                         kr * (Er * irr + (Ss - ur) * (Ss + pr * rcp_nr(mr)))};
  const double aL = fabs(SL), aS = fabs(Ss), aR = fabs(SR);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const double diss = aL * (QsL[m] - QL[m]) + aS * (QsR[m] - QsL[m]) + aR * (QR[m] - QsR[m]);
    F[m] = Fm[m] - 0.5 * diss;
  }
}

// Characteristic MEG7 states in 3D: the primitive eigenvectors of the 2D
// projection at the mean density and pressure, plus the identity row and
// column of the second tangential velocity.  Wf(q, f) / Gf(q, f): rotated
// primitive field f (0..4) and its spacing-scaled normal gradient at offset
// q-2 from cell j.  Rows of L: (u_n, p), (rho, p), (u_t1), (u_t2), (u_n, p).
template <int ORD, class FW, class FG>
__device__ __forceinline__ void meg7_char_states3(FW Wf, FG Gf, double gamma, double WLo[5],
                                                  double WRo[5]) {
  const double rb = 0.5 * (Wf(2, 0) + Wf(3, 0));
  const double pb = 0.5 * (Wf(2, 4) + Wf(3, 4));
  const double irb = rcp_nr(rb);
  const double cb = sqrt_nr(gamma * pb * irb);
  const double icb = rcp_nr(cb);
  const double h2c = 0.5 * icb, ic2 = icb * icb, h2c2 = 0.5 * ic2;
  const double cor = cb * irb, c2 = cb * cb;
#pragma unroll
  for (int m = 0; m < 5; ++m) { WLo[m] = 0.0; WRo[m] = 0.0; }
#pragma unroll 1
  for (int m = 0; m < 5; ++m) {
    // row m of L as ca * field fa + cbv * field fb
    const bool tang = (m == 2 || m == 3);
    const int fa = (m == 1) ? 0 : (tang ? m : 1);
    const int fb = tang ? m : 4;
    const double ca = (m == 0) ? -rb * h2c : ((m == 4) ? rb * h2c : 1.0);
    const double cbv = (m == 1) ? -ic2 : (tang ? 0.0 : h2c2);
    double cv[6], cg[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      cv[q] = ca * Wf(q, fa) + cbv * Wf(q, fb);
      cg[q] = ca * Gf(q, fa) + cbv * Gf(q, fb);
    }
    double cl, cr;
    meg7_pair<ORD>(cv, cg, cl, cr);
    // column m of R = L^{-1}: (1,-c/rho,0,0,c^2), (1,0,0,0,0), (0,0,1,0,0), (0,0,0,1,0),
    // (1,c/rho,0,0,c^2)
    const double b0 = tang ? 0.0 : 1.0;
    const double b1 = (m == 0) ? -cor : ((m == 4) ? cor : 0.0);
    const double b2 = (m == 2) ? 1.0 : 0.0;
    const double b3 = (m == 3) ? 1.0 : 0.0;
    const double b4 = (m == 0 || m == 4) ? c2 : 0.0;
    WLo[0] += b0 * cl; WLo[1] += b1 * cl; WLo[2] += b2 * cl; WLo[3] += b3 * cl; WLo[4] += b4 * cl;
    WRo[0] += b0 * cr; WRo[1] += b1 * cr; WRo[2] += b2 * cr; WRo[3] += b3 * cr; WRo[4] += b4 * cr;
  }
}

template <int NP, int NL>
struct Sweep3Cfg {
  static constexpr int NT = 256;
  static constexpr int H = 6;
  static constexpr int WP = NP + 2 * H;   // staged positions per line
  static constexpr int WD = NP + 6;       // gradients / detector: positions -3 .. NP+2
  static constexpr int WF = NP + 10;      // cell fluxes: positions -5 .. NP+4
  static constexpr int WFL = NP + 1;      // interfaces -1/2 .. NP-1/2
};

template <int DIR, int NP, int NL, int ORD>
__global__ __launch_bounds__(256, 2) void meg7_sweep3_kernel(Sweep3Params P) {
  using C = Sweep3Cfg<NP, NL>;
  constexpr int NT = C::NT, H = C::H, WP = C::WP, WD = C::WD, WF = C::WF, WFL = C::WFL;
  constexpr bool LINEFAST = DIR != 0;     // y and z lines: consecutive lines are consecutive x
  __shared__ double sW[5][NL][WP];
  __shared__ double sD[5][NL][WD];
  __shared__ double sF[5][NL][WF];        // cell fluxes, then interface fluxes
  __shared__ unsigned char sChi[NL][WD];
  __shared__ unsigned short sQueue[NL * WFL];
  __shared__ int sQCount;
  const int tid = threadIdx.x;
  const size_t n = (size_t)P.nx * P.ny * P.nz;
  const int ndir = DIR == 0 ? P.nx : (DIR == 1 ? P.ny : P.nz);
  const size_t sdir = DIR == 0 ? 1 : (DIR == 1 ? (size_t)P.nx : (size_t)P.nx * P.ny);
  const int nlines = DIR == 0 ? P.ny * P.nz : (DIR == 1 ? P.nx * P.nz : P.nx * P.ny);
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD one
  // contiguous run of tiles, so the halo of neighbouring position tiles and
  // the 128-byte lines that neighbouring line groups share (y and z sweeps:
  // 8 consecutive x per position) meet in one L2
  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, rem = gridDim.x & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (blockIdx.x >> 3);
  const int ptile = tile % P.ptiles;
  const int group = tile / P.ptiles;
  const int p0 = ptile * NP;
  // first cell of line L (position 0)
  auto line_base = [&](int L) -> size_t {
    if (DIR == 0) return (size_t)L * P.nx;                                   // L = z ny + y
    if (DIR == 1) return (size_t)(L / P.nx) * P.nx * P.ny + (L % P.nx);      // L = z nx + x
    return (size_t)L;                                                       // L = y nx + x
  };
  // conserved index of rotated component m (cyclic tangential order)
  auto cidx = [](int m) { return (m == 0 || m == 4) ? m : 1 + (DIR + m - 1) % 3; };

  // ---- load: primitives of NL lines x (NP + 12) positions -----------------
  bool bad = false;
  for (int t = tid; t < NL * WP; t += NT) {
    const int l = LINEFAST ? t % NL : t / WP;
    const int p = LINEFAST ? t / NL : t % WP;
    int L = group * NL + l;
    const bool lv = L < nlines;
    if (!lv) L = nlines - 1;
    const int q = p0 + p - H;
    const size_t s = line_base(L) + (size_t)bc_index(q, ndir, P.bc) * sdir;
    const double r = P.Qk[s];
    const double ir = rcp_nr(r);
    double u[3];
#pragma unroll
    for (int m = 1; m <= 3; ++m) u[m - 1] = P.Qk[(size_t)cidx(m) * n + s] * ir;
    const double E = P.Qk[4 * n + s];
    const double pr = (P.gamma - 1.0) * (E - 0.5 * r * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
    sW[0][l][p] = r;
    sW[1][l][p] = u[0];
    sW[2][l][p] = u[1];
    sW[3][l][p] = u[2];
    sW[4][l][p] = pr;
    if (P.first && lv && q >= p0 && q < p0 + NP && q < ndir &&
        !(r > 0.0 && pr > 0.0 && isfinite(E) && isfinite(u[0]) && isfinite(u[1]) &&
          isfinite(u[2])))
      bad = true;
  }
  if (bad) atomicOr(P.status, STATUS_BAD_STATE);
  if (tid == 0) sQCount = 0;
  __syncthreads();

  // ---- pass 1: per cell --------------------------------------------------
  for (int t = tid; t < NL * WF; t += NT) {
    const int l = t / WF, pf = t % WF;
    const int p = pf + 1;                 // staged index of position pf - 5
    double W[5], f[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) W[m] = sW[m][l][p];
    conv_flux3(W, P.g1inv, f);
#pragma unroll
    for (int m = 0; m < 5; ++m) sF[m][l][pf] = f[m];
    const int pd = pf - 2;                // position pf - 5 = pd - 3
    if (pd >= 0 && pd < WD) {
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const double* u = &sW[m][l][p];
        sD[m][l][pd] = grad6(u[-3], u[-2], u[-1], u[1], u[2], u[3]);
      }
      const double* rho = &sW[0][l][p];
      sChi[l][pd] = detector_flag(rho[-2], rho[-1], rho[0], rho[1], rho[2]) ? 1 : 0;
    }
  }
  __syncthreads();

  // ---- pass 2: interfaces, smooth branch; ballot-compact the flagged ------
  constexpr int IPT = (NL * WFL + NT - 1) / NT;
  double fsm[IPT][5];
  bool has[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    has[k] = false;
    const int t = tid + k * NT;
    bool flagged = false;
    if (t < NL * WFL) {
      const int l = t / WFL, pi = t % WFL;   // interface between positions pi-1 and pi
      const int pos = pi - 1;                // left cell
      // eq. (buffer): the six flags read at once and OR-ed
      unsigned any = 0u;
#pragma unroll
      for (int j = 1; j <= 6; ++j) any |= sChi[l][pos + j];
      const bool sigma = any == 0u;
      const int L = group * NL + l;
      const int gi = p0 + pi;                // interface index along the line
      if (P.sig && L < nlines && gi <= ndir) {
        const size_t b = line_base(L);
        // flags array: one longer along this direction
        size_t o;
        if (DIR == 0) o = b / P.nx * (P.nx + 1) + gi;
        else if (DIR == 1) o = (b / ((size_t)P.nx * P.ny)) * (size_t)(P.ny + 1) * P.nx +
                               (size_t)gi * P.nx + (b % P.nx);
        else o = (size_t)gi * P.nx * P.ny + b;
        P.sig[o] = sigma;
      }
      flagged = !sigma;
      if (sigma) {
        const int p = pos + H;               // staged index of the left cell
        double WL[5], WR[5], Fm[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          double v[6], g[6], f[10];
#pragma unroll
          for (int q = 0; q < 6; ++q) v[q] = sW[m][l][p + q - 2];
#pragma unroll
          for (int q = 1; q < 5; ++q) g[q] = sD[m][l][pos + q + 1];
          g[0] = g[5] = 0.0;
          WL[m] = grb_l<ORD>(v, g);
          WR[m] = grb_r<ORD>(v, g);
#pragma unroll
          for (int q = 0; q < 10; ++q) f[q] = sF[m][l][pos + q + 1];
          Fm[m] = flux_mean<ORD>(f);
        }
        if (!(WL[0] > 0.0 && WL[4] > 0.0 && WR[0] > 0.0 && WR[4] > 0.0)) {
          double f0[5], f1[5];
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            WL[m] = sW[m][l][p];
            WR[m] = sW[m][l][p + 1];
          }
          conv_flux3(WL, P.g1inv, f0);
          conv_flux3(WR, P.g1inv, f1);
#pragma unroll
          for (int m = 0; m < 5; ++m) Fm[m] = 0.5 * (f0[m] + f1[m]);
        }
        hllc3(WL, WR, Fm, P.gamma, P.g1inv, fsm[k]);
        has[k] = true;
      }
    }
    const unsigned long long ball = __ballot(flagged);
    if (ball) {
      const int lane = __lane_id();
      int base = 0;
      if (lane == 0) base = atomicAdd(&sQCount, (int)__popcll(ball));
      base = __shfl(base, 0);
      if (flagged) {
        const int rank = (int)__popcll(ball & ((1ull << lane) - 1ull));
        sQueue[base + rank] = (unsigned short)t;
      }
    }
  }
  __syncthreads();  // every read of the cell fluxes is done: sF becomes the interface fluxes
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (has[k]) {
      const int t = tid + k * NT;
      const int l = t / WFL, pi = t % WFL;
#pragma unroll
      for (int m = 0; m < 5; ++m) sF[m][l][pi] = fsm[k][m];
    }
  }

  // ---- pass 3: the flagged interfaces --------------------------------------
  const int nq = sQCount;
  for (int qi = tid; qi < nq; qi += NT) {
    const int t = sQueue[qi];
    const int l = t / WFL, pi = t % WFL;
    const int pos = pi - 1;
    const int p = pos + H;
    double WL[5], WR[5];
    meg7_char_states3<ORD>([&](int q, int f) { return sW[f][l][p + q - 2]; },
                           [&](int q, int f) { return sD[f][l][pos + q + 1]; }, P.gamma, WL,
                           WR);
    if (!(WL[0] > 0.0 && WL[4] > 0.0 && WR[0] > 0.0 && WR[4] > 0.0)) {
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        WL[m] = sW[m][l][p];
        WR[m] = sW[m][l][p + 1];
      }
    }
    double FL[5], FR[5], Fm[5], F[5];
    conv_flux3(WL, P.g1inv, FL);
    conv_flux3(WR, P.g1inv, FR);
#pragma unroll
    for (int m = 0; m < 5; ++m) Fm[m] = 0.5 * (FL[m] + FR[m]);
    hllc3(WL, WR, Fm, P.gamma, P.g1inv, F);
#pragma unroll
    for (int m = 0; m < 5; ++m) sF[m][l][pi] = F[m];
  }
  __syncthreads();

  // ---- pass 4: flux differences; residual accumulation / stage update ------
  const double dtv = (P.last && P.mode != MODE_RESIDUAL) ? *P.dt : 0.0;
  double ea = 0.0, eb = 0.0, ec = 0.0;   // time-step extrema (stage 3, P.dtx)
  bool ebad = false;
  for (int t = tid; t < NL * NP; t += NT) {
    const int l = LINEFAST ? t % NL : t / NP;
    const int pc = LINEFAST ? t / NL : t % NP;
    const int L = group * NL + l;
    const int q = p0 + pc;
    if (L >= nlines || q >= ndir) continue;
    const size_t s = line_base(L) + (size_t)q * sdir;
    double nv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // the new state, conserved order (stage 3)
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const size_t o = (size_t)cidx(m) * n + s;
      const double d = (sF[m][l][pc + 1] - sF[m][l][pc]) * P.inv_d;
      double r = P.first ? -d : P.R[o] - d;
      if (!P.last) {
        P.R[o] = r;
      } else if (P.mode == MODE_RESIDUAL) {
        P.out[o] = r;
      } else if (P.mode == MODE_STAGE1) {
        P.out[o] = P.Qn[o] + dtv * r;
      } else if (P.mode == MODE_STAGE2) {
        P.out[o] = 0.75 * P.Qn[o] + 0.25 * P.Qk[o] + (0.25 * dtv) * r;
      } else {
        const double v = (1.0 / 3.0) * P.Qn[o] + (2.0 / 3.0) * P.Qk[o] + ((2.0 / 3.0) * dtv) * r;
        P.out[o] = v;
        nv[cidx(m)] = v;
      }
    }
    if (P.dtx) dt3_extrema_cell(nv, P.gamma, ea, eb, ec, ebad);
  }
  if (P.dtx) {
    // every lane of every wave reaches this point (the cell loop's bounds
    // are uniform): wave extrema into the wave's slot
    if (ebad) atomicOr(P.status, 1u);
    constexpr int NW = NT / 64;
    const int nslot = gridDim.x * NW, slot = blockIdx.x * NW + (tid >> 6);
    ea = wave_extremum<true>(ea);
    eb = wave_extremum<true>(eb);
    ec = wave_extremum<true>(ec);
    if (__lane_id() == 0) {
      P.dtx[slot] = ea;
      P.dtx[nslot + slot] = eb;
      P.dtx[2 * nslot + slot] = ec;
    }
  }
}

// ---------------------------------------------------------------------------
// The x and y sweeps fused: one workgroup per TX x TY tile of one z plane.
// The tile plus a 6-cell halo in x and y is staged once as (rho, u, v, w, p);
// the x sweep and then the y sweep run the passes above on lines of the tile
// (NL lines at a time), each thread keeping the residual of its cell in
// registers, and the sum -dF/dx - dG/dy is written to the accumulator once.
// The z line sweep then adds -dH/dz and stores the residual or the stage.
// Per cell-stage this moves Q^(k) and the accumulator once instead of three
// times.  The residual of a cell is accumulated in the order of the line
// sweeps (0 - dF/dx - dG/dy), so the fused and the line-sweep forms give the
// same residual up to the pressure of a cell, which the line sweeps form
// with the squared velocities summed in rotated order.
struct XY3Params {
  const double* __restrict__ Qk;  // [5][nz][ny][nx]
  double* R;                      // accumulator [5][nz][ny][nx] (conserved order)
  uint8_t* sigx;                  // optional flags [nz][ny][nx+1]
  uint8_t* sigy;                  // optional flags [nz][ny+1][nx]
  unsigned* status;
  int nx, ny, nz, bcx, bcy;
  int tiles_x, tiles_y, ntiles;
  double inv_dx, inv_dy, gamma, g1inv;
};

template <int TX_, int TY_, int NL_>
struct XY3Cfg {
  static constexpr int TX = TX_, TY = TY_, NL = NL_, NT = 256, H = 6;
  static constexpr int RX = TX + 2 * H, RY = TY + 2 * H, RS = RX * RY;
  static constexpr int CPT = (TX * TY + NT - 1) / NT;
  static constexpr int imax(int a, int b) { return a > b ? a : b; }
  static constexpr int WD(int N) { return N + 6; }
  static constexpr int WF(int N) { return N + 10; }
  static constexpr int WFL(int N) { return N + 1; }
  static constexpr int NMAX = imax(TX, TY);
  static constexpr int D = 5 * NL * WD(NMAX);                               // gradients
  static constexpr int F = 5 * NL * imax(WF(NMAX), WFL(NMAX) | 1);          // fluxes
  static constexpr int CHI = NL * WD(NMAX);
  static constexpr int QMAX = NL * WFL(NMAX);
  static constexpr int LDS_BYTES = 8 * (5 * RS + D + F) + CHI + 2 * QMAX + 16;
};

template <class C, int DIR, int ORD>
__device__ __forceinline__ void sweep_xy3(const XY3Params& P, const double* sU, double* sD,
                                          double* sF, unsigned char* sChi,
                                          unsigned short* sQueue, int* sQCount, int l0,
                                          int tx0, int ty0, int z, double (&res)[C::CPT][5]) {
  constexpr bool X = DIR == 0;
  constexpr int N = X ? C::TX : C::TY, NLINES = X ? C::TY : C::TX, NL = C::NL;
  constexpr int WD = C::WD(N), WF = C::WF(N), WFL = C::WFL(N), WFS = WFL | 1;
  constexpr int RS = C::RS, RX = C::RX, H = C::H, NT = C::NT;
  constexpr int SN = X ? 1 : RX;
  constexpr int FSTR = NL * (WF > WFS ? WF : WFS);   // field stride of sF
  // rotated component m -> tile field (and conserved component): the
  // tangential velocities cyclically (x: v, w; y: w, u)
  constexpr int R1 = X ? 1 : 2, R2 = X ? 2 : 3, R3 = X ? 3 : 1;
  const int rot[5] = {0, R1, R2, R3, 4};
  const int tid = threadIdx.x;
  const int nl = (NLINES - l0) < NL ? (NLINES - l0) : NL;
  const double inv_d = X ? P.inv_dx : P.inv_dy;
  auto ridx = [&](int line, int pos) {
    const int lx = X ? pos : l0 + line;
    const int ly = X ? l0 + line : pos;
    return (ly + H) * RX + (lx + H);
  };

  // ---- pass 1: cell fluxes, gradients, detector ------------------------------
  for (int t = tid; t < NL * WF; t += NT) {
    const int line = t / WF, pf = t % WF;
    if (line >= nl) continue;
    const int pos = pf - 5;
    const int r = ridx(line, pos);
    double W[5], f[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) W[m] = sU[rot[m] * RS + r];
    conv_flux3(W, P.g1inv, f);
#pragma unroll
    for (int m = 0; m < 5; ++m) sF[m * FSTR + line * WF + pf] = f[m];
    if (pos >= -3 && pos < N + 3) {
      const int pd = pos + 3;
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const double* u = sU + rot[m] * RS + r;
        sD[(m * NL + line) * WD + pd] =
            grad6(u[-3 * SN], u[-2 * SN], u[-SN], u[SN], u[2 * SN], u[3 * SN]);
      }
      const double* rho = sU + r;
      sChi[line * WD + pd] =
          detector_flag(rho[-2 * SN], rho[-SN], rho[0], rho[SN], rho[2 * SN]) ? 1 : 0;
    }
  }
  if (tid == 0) *sQCount = 0;
  __syncthreads();

  // ---- pass 2: interfaces, smooth branch; ballot-compact the flagged --------
  constexpr int IPT = (NL * WFL + NT - 1) / NT;
  double fsm[IPT][5];
  bool has[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    has[k] = false;
    const int t = tid + k * NT;
    bool flagged = false;
    if (t < NL * WFL) {
      const int line = t / WFL, pi = t % WFL;
      const int pos = pi - 1;                 // interface pos + 1/2
      if (line < nl) {
        // eq. (buffer): the six flags read at once and OR-ed
        unsigned any = 0u;
#pragma unroll
        for (int j = 1; j <= 6; ++j) any |= sChi[line * WD + pos + j];
        const bool sigma = any == 0u;
        if (X) {
          const int gy = ty0 + l0 + line, gi = tx0 + pi;
          if (P.sigx && gy < P.ny && gi <= P.nx)
            P.sigx[((size_t)z * P.ny + gy) * (P.nx + 1) + gi] = sigma;
        } else {
          const int gx = tx0 + l0 + line, gi = ty0 + pi;
          if (P.sigy && gx < P.nx && gi <= P.ny)
            P.sigy[((size_t)z * (P.ny + 1) + gi) * P.nx + gx] = sigma;
        }
        flagged = !sigma;
        if (sigma) {
          const int r = ridx(line, pos);
          double WL[5], WR[5], Fm[5];
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            const double* u = sU + rot[m] * RS + r;
            double v[6], g[6], f[10];
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] = u[(q - 2) * SN];
#pragma unroll
            for (int q = 1; q < 5; ++q) g[q] = sD[(m * NL + line) * WD + pos + q + 1];
            g[0] = g[5] = 0.0;
            WL[m] = grb_l<ORD>(v, g);
            WR[m] = grb_r<ORD>(v, g);
#pragma unroll
            for (int q = 0; q < 10; ++q) f[q] = sF[m * FSTR + line * WF + pos + q + 1];
            Fm[m] = flux_mean<ORD>(f);
          }
          if (!(WL[0] > 0.0 && WL[4] > 0.0 && WR[0] > 0.0 && WR[4] > 0.0)) {
            double f0[5], f1[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
              WL[m] = sU[rot[m] * RS + r];
              WR[m] = sU[rot[m] * RS + r + SN];
            }
            conv_flux3(WL, P.g1inv, f0);
            conv_flux3(WR, P.g1inv, f1);
#pragma unroll
            for (int m = 0; m < 5; ++m) Fm[m] = 0.5 * (f0[m] + f1[m]);
          }
          hllc3(WL, WR, Fm, P.gamma, P.g1inv, fsm[k]);
          has[k] = true;
        }
      }
    }
    const unsigned long long ball = __ballot(flagged);
    if (ball) {
      const int lane = __lane_id();
      int base = 0;
      if (lane == 0) base = atomicAdd(sQCount, (int)__popcll(ball));
      base = __shfl(base, 0);
      if (flagged) {
        const int rank = (int)__popcll(ball & ((1ull << lane) - 1ull));
        sQueue[base + rank] = (unsigned short)t;
      }
    }
  }
  __syncthreads();  // every read of the cell fluxes is done: sF becomes the interface fluxes
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (has[k]) {
      const int t = tid + k * NT;
      const int line = t / WFL, pi = t % WFL;
#pragma unroll
      for (int m = 0; m < 5; ++m) sF[m * FSTR + line * WFS + pi] = fsm[k][m];
    }
  }

  // ---- pass 3: the flagged interfaces -----------------------------------------
  const int nq = *sQCount;
  for (int qi = tid; qi < nq; qi += NT) {
    const int t = sQueue[qi];
    const int line = t / WFL, pi = t % WFL;
    const int pos = pi - 1;
    const int r = ridx(line, pos);
    double WL[5], WR[5];
    meg7_char_states3<ORD>([&](int q, int f) { return sU[rot[f] * RS + r + (q - 2) * SN]; },
                           [&](int q, int f) { return sD[(f * NL + line) * WD + pos + q + 1]; },
                           P.gamma, WL, WR);
    if (!(WL[0] > 0.0 && WL[4] > 0.0 && WR[0] > 0.0 && WR[4] > 0.0)) {
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        WL[m] = sU[rot[m] * RS + r];
        WR[m] = sU[rot[m] * RS + r + SN];
      }
    }
    double FL[5], FR[5], Fm[5], F[5];
    conv_flux3(WL, P.g1inv, FL);
    conv_flux3(WR, P.g1inv, FR);
#pragma unroll
    for (int m = 0; m < 5; ++m) Fm[m] = 0.5 * (FL[m] + FR[m]);
    hllc3(WL, WR, Fm, P.gamma, P.g1inv, F);
#pragma unroll
    for (int m = 0; m < 5; ++m) sF[m * FSTR + line * WFS + pi] = F[m];
  }
  __syncthreads();

  // ---- pass 4: flux differences into the cell residuals -----------------------
#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
    const int c = tid + k * NT;
    if (c < C::TX * C::TY) {
      const int lx = c % C::TX, ly = c / C::TX;
      const int line = (X ? ly : lx) - l0;
      const int pos = X ? lx : ly;
      if (line >= 0 && line < nl) {
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const double d = (sF[m * FSTR + line * WFS + pos + 1] - sF[m * FSTR + line * WFS + pos]) *
                           inv_d;
          res[k][rot[m]] -= d;
        }
      }
    }
  }
  __syncthreads();
}

template <class C, int ORD>
__global__ __launch_bounds__(256, 2) void meg7_xy3_kernel(XY3Params P) {
  constexpr int RS = C::RS, RX = C::RX, H = C::H, NT = C::NT, TX = C::TX, TY = C::TY;
  __shared__ double sU[5 * RS];
  __shared__ double sD[C::D];
  __shared__ double sF[C::F];
  __shared__ unsigned char sChi[C::CHI];
  __shared__ unsigned short sQueue[C::QMAX];
  __shared__ int sQCount;
  // tile of this workgroup: consecutive tiles (x fastest, then y, then z) in
  // one XCD, as in the 2D kernels
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (b >> 3);
  if (tile >= P.ntiles) return;
  const int tpp = P.tiles_x * P.tiles_y;
  const int z = tile / tpp, tp = tile - z * tpp;
  const int tx0 = (tp % P.tiles_x) * TX, ty0 = (tp / P.tiles_x) * TY;
  const size_t n = (size_t)P.nx * P.ny * P.nz;
  const size_t zb = (size_t)z * P.ny * P.nx;
  const int tid = threadIdx.x;

  // ---- load: (rho, u, v, w, p) of the tile and its halo ------------------------
  bool bad = false;
  for (int c = tid; c < RS; c += NT) {
    const int ly = c / RX - H, lx = c % RX - H;
    const int gy = bc_index(ty0 + ly, P.ny, P.bcy), gx = bc_index(tx0 + lx, P.nx, P.bcx);
    const size_t s = zb + (size_t)gy * P.nx + gx;
    const double r = P.Qk[s];
    const double ir = rcp_nr(r);
    const double u = P.Qk[n + s] * ir, v = P.Qk[2 * n + s] * ir, w = P.Qk[3 * n + s] * ir;
    const double E = P.Qk[4 * n + s];
    const double pr = (P.gamma - 1.0) * (E - 0.5 * r * (u * u + v * v + w * w));
    sU[c] = r;
    sU[RS + c] = u;
    sU[2 * RS + c] = v;
    sU[3 * RS + c] = w;
    sU[4 * RS + c] = pr;
    if (lx >= 0 && lx < TX && ly >= 0 && ly < TY && tx0 + lx < P.nx && ty0 + ly < P.ny &&
        !(r > 0.0 && pr > 0.0 && isfinite(E) && isfinite(u) && isfinite(v) && isfinite(w)))
      bad = true;
  }
  if (bad) atomicOr(P.status, STATUS_BAD_STATE);
  __syncthreads();

  double res[C::CPT][5];
#pragma unroll
  for (int k = 0; k < C::CPT; ++k)
#pragma unroll
    for (int m = 0; m < 5; ++m) res[k][m] = 0.0;
  for (int l0 = 0; l0 < TY; l0 += C::NL)
    sweep_xy3<C, 0, ORD>(P, sU, sD, sF, sChi, sQueue, &sQCount, l0, tx0, ty0, z, res);
  for (int l0 = 0; l0 < TX; l0 += C::NL)
    sweep_xy3<C, 1, ORD>(P, sU, sD, sF, sChi, sQueue, &sQCount, l0, tx0, ty0, z, res);

#pragma unroll
  for (int k = 0; k < C::CPT; ++k) {
    const int c = tid + k * NT;
    const int gx = tx0 + c % TX, gy = ty0 + c / TX;
    if (c < TX * TY && gx < P.nx && gy < P.ny) {
      const size_t s = zb + (size_t)gy * P.nx + gx;
#pragma unroll
      for (int m = 0; m < 5; ++m) P.R[m * n + s] = res[k][m];
    }
  }
}

// CFL time step in 3D (inviscid), Sec. 2.5: pass 1 of the two-pass
// reduction (pass 2 is dt_finish_kernel with no viscous limit).
struct Dt3Params {
  const double* __restrict__ Q;
  double* partial;
  unsigned* status;
  int nx, ny, nz;
  double dx, dy, dz, gamma;
};

__global__ __launch_bounds__(kDtThreads) void dt3_reduce_kernel(Dt3Params P) {
#pragma clang fp contract(off)
  __shared__ double red[kDtThreads / 64];
  const size_t n = (size_t)P.nx * P.ny * P.nz;
  double conv = __builtin_inf();
  bool bad = false;
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (size_t)gridDim.x * blockDim.x) {
    const double rho = P.Q[s];
    const double u = P.Q[n + s] / rho, v = P.Q[2 * n + s] / rho, w = P.Q[3 * n + s] / rho;
    const double p = (P.gamma - 1.0) * (P.Q[4 * n + s] - rho * (u * u + v * v + w * w) / 2.0);
    const double c = sqrt(P.gamma * p / rho);
    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(c) || !isfinite(u) || !isfinite(v) ||
        !isfinite(w))
      bad = true;
    conv = fmin(conv, fmin(P.dx / (fabs(u) + c), fmin(P.dy / (fabs(v) + c), P.dz / (fabs(w) + c))));
  }
  if (bad) atomicOr(P.status, 1u);
  conv = block_min(conv, red);
  if (threadIdx.x == 0) {
    P.partial[blockIdx.x] = conv;
    P.partial[kDtBlocks + blockIdx.x] = __builtin_inf();
  }
}

}  // namespace gbr
