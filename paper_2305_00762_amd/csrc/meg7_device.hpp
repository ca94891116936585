// Device-side building blocks of the MEG7 scheme (Chamarthi, arXiv
// 2305.00762) for gfx950, in a frame rotated to the interface normal:
// primitive vector W = (rho, un, ut, p), conservative (rho, rho un, rho ut, E).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbr {

// Constants of the scheme.
constexpr double kAlphaV = 4.0;   // alpha-damping coefficient, Sec. 2.1 eq. (eqn:alphad)
constexpr double kXiMP = 7.0;     // MP parameter xi, Sec. 2.3 eq. (eqn:alpha)
constexpr double kMPTol = 1e-40;  // MP activation threshold, eq. (eqn:hocus/mp5Condition)
constexpr double kPsiC = 0.5;     // detector threshold psi_c, Sec. 2.4 eq. (buffer)
constexpr double kXiDet = 1e-3;   // detector xi, eq. (buffer)
// eq. (buffer): eps = 0.9 psi_c / (1 - 0.9 psi_c) xi^2 (folded with IEEE rounding)
constexpr double kDetEps = (0.9 * kPsiC) / (1.0 - 0.9 * kPsiC) * (kXiDet * kXiDet);

// Reciprocal and reciprocal square root: hardware estimate refined by two
// Newton steps (full FP64 accuracy up to the last bit or two; positive,
// normal arguments only).  Used for the Riemann-solver arithmetic, never
// for the detector decision.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = rsq_nr(x);
  const double s = x * y;
  return fma(0.5 * y, fma(-s, s, x), s);
}

// fl(a / b) from rb = rcp_nr(b): the quotient a rb and one correction by the
// exact residual.  These are the steps of the hardware's IEEE division after
// its scaling step (reciprocal estimate, two Newton steps, quotient, fused
// correction), and that step leaves operands unchanged when both magnitudes
// lie in [2^-300, 2^300] or the numerator is zero (div_rb_ok): there the
// result is the IEEE quotient bit for bit, up to the sign of a zero result
// (gbr_selftest_division checks it on the device).  One reciprocal then
// serves the three quotients of a cell.
__device__ __forceinline__ double div_rb(double a, double b, double rb) {
#pragma clang fp contract(off)
  const double q = a * rb;
  return fma(fma(-b, q, a), rb, q);
}
__device__ __forceinline__ bool div_rb_ok(double a) {
  const double m = fabs(a);
  return m <= 0x1p300 && (m >= 0x1p-300 || m == 0.0);
}

// Sixth-order central first derivative, eq. (eqn:six), scaled by the
// spacing: returns dx * dPhi/dx from Phi_{-3..3} (pm3 .. p3).
__device__ __forceinline__ double grad6(double pm3, double pm2, double pm1, double p1,
                                        double p2, double p3) {
  return (45.0 * (p1 - pm1) - 9.0 * (p2 - pm2) + (p3 - pm3)) * (1.0 / 60.0);
}

// Density detector psi of Sec. 2.4 with eps in numerator and denominator.
// Evaluated with one rounding per operation in a fixed order (no FMA
// contraction) and an IEEE division, so that the decision psi < psi_c is
// reproducible bit for bit.
__device__ __forceinline__ double detector_psi(double rm2, double rm1, double r0,
                                                         double rp1, double rp2) {
#pragma clang fp contract(off)
  double a = fabs(r0 - rm1) + fabs((r0 - 2.0 * rm1) + rm2);
  double b = fabs(r0 - rp1) + fabs((r0 - 2.0 * rp1) + rp2);
  double num = (2.0 * a) * b + kDetEps;
  double den = (a * a + b * b) + kDetEps;
  return num / den;
}

// The detector's decision psi < psi_c (= 1/2) without the division: with
// num = 2ab + eps and den = a^2 + b^2 + eps as above (both positive),
// fl(num / den) < 1/2 holds exactly when num / den < 1/2 - 2^-55 (the rounding
// boundary below 1/2; a tie rounds to 1/2, whose significand is even), i.e.
// when 2 num - den < -den 2^-54.  2 num is exact, 2 num - den is exact
// wherever the two are within a factor 2 of each other (Sterbenz) and has the
// sign that decides otherwise, and den 2^-54 is exact: the comparison below
// is the division's decision bit for bit, for a fraction of its cost.
static_assert(kPsiC == 0.5, "the division-free decision assumes psi_c = 1/2");
__device__ __forceinline__ bool detector_flag(double rm2, double rm1, double r0, double rp1,
                                              double rp2) {
#pragma clang fp contract(off)
  double a = fabs(r0 - rm1) + fabs((r0 - 2.0 * rm1) + rm2);
  double b = fabs(r0 - rp1) + fabs((r0 - 2.0 * rp1) + rp2);
  double num = (2.0 * a) * b + kDetEps;
  double den = (a * a + b * b) + kDetEps;
  return (2.0 * num - den) < -(den * 0x1p-54);
}

__device__ __forceinline__ double minmod(double a, double b) {
  // (sign a + sign b)/2 * min(|a|,|b|), eq. (eqn:alpha)
  double m = fmin(fabs(a), fabs(b));
  return (a > 0.0 && b > 0.0) ? m : ((a < 0.0 && b < 0.0) ? -m : 0.0);
}

// GRB interface states, eq. (eqn:grb).  v[k] = Phi_{j+k-2} (k=0..5),
// g[k] = Phi'_{j+k-2} (Phi' = dx dPhi/dx).
__device__ __forceinline__ double grb_left(const double* v, const double* g) {
  constexpr double s = 1.0 / 840.0;
  return (3.0 * s) * (v[0] + v[4]) + (178.0 * s) * (v[1] + v[3]) + (478.0 * s) * v[2] +
         (420.0 * s) * g[2] + (60.0 * s) * (g[1] - g[3]);
}
__device__ __forceinline__ double grb_right(const double* v, const double* g) {
  constexpr double s = 1.0 / 840.0;
  return (3.0 * s) * (v[1] + v[5]) + (178.0 * s) * (v[2] + v[4]) + (478.0 * s) * v[3] -
         (420.0 * s) * g[3] + (60.0 * s) * (g[2] - g[4]);
}

// Fourth-order GRB states: the subset alpha = 4, beta = 0 of eqs.
// (good_6tth-order_scheme_flux), (alpha-beta) put into eq. (eqn:lingrb),
//   Phi^L = (4 (Phi_{j-1} + Phi_{j+1}) + 16 Phi_j + Phi'_{j-1} + 12 Phi'_j - Phi'_{j+1}) / 24
// and its mirror image for Phi^R at j+1/2.  Same v, g layout as grb_left.
__device__ __forceinline__ double grb4_left(const double* v, const double* g) {
  constexpr double s = 1.0 / 24.0;
  return (4.0 * s) * (v[1] + v[3]) + (16.0 * s) * v[2] + (12.0 * s) * g[2] + s * (g[1] - g[3]);
}
__device__ __forceinline__ double grb4_right(const double* v, const double* g) {
  constexpr double s = 1.0 / 24.0;
  return (4.0 * s) * (v[2] + v[4]) + (16.0 * s) * v[3] - (12.0 * s) * g[3] + s * (g[2] - g[4]);
}

// GRB states of the selected order: 7 (eq. eqn:grb) or 4 (the subset above).
template <int ORD>
__device__ __forceinline__ double grb_l(const double* v, const double* g) {
  return ORD == 4 ? grb4_left(v, g) : grb_left(v, g);
}
template <int ORD>
__device__ __forceinline__ double grb_r(const double* v, const double* g) {
  return ORD == 4 ? grb4_right(v, g) : grb_right(v, g);
}

// Mean of the reconstructed cell fluxes, (F(f_L) + F(f_R))/2 at j+1/2, from
// f[q] = f_{j+q-4} (q = 0..9).  The sum of a left stencil and its mirror image
// is symmetric about the interface, so pairs are added first:
//   order 7, eqs. (flux-full), (flux-right): (1052, -250, 38, 1, -1) / 1680;
//   order 4, eq. (fourth) and its mirror:    (1821, -461, 85, -4, -1) / 2880.
template <int ORD>
__device__ __forceinline__ double flux_mean(const double* f) {
  if (ORD == 4) {
    constexpr double s = 1.0 / 2880.0;
    return (1821.0 * s) * (f[4] + f[5]) - (461.0 * s) * (f[3] + f[6]) +
           (85.0 * s) * (f[2] + f[7]) - (4.0 * s) * (f[1] + f[8]) - s * (f[0] + f[9]);
  }
  constexpr double s = 1.0 / 1680.0;
  return (1052.0 * s) * (f[4] + f[5]) - (250.0 * s) * (f[3] + f[6]) +
         (38.0 * s) * (f[2] + f[7]) + s * (f[1] + f[8]) - s * (f[0] + f[9]);
}

// MP curvature d of eq. (eqn:mp-procedure) at the centre of v[-1..1], g[-1..1].
__device__ __forceinline__ double mp_curv(double vm, double v0, double vp, double gm,
                                          double gp) {
  return 2.0 * (vp - 2.0 * v0 + vm) - 0.5 * (gp - gm);
}

// MEG7 left and right values at j+1/2 of one characteristic component
// (Sec. 2.3): GRB value (of order ORD), the activation test, and the MP
// bounds.  v, g hold offsets -2..3 around cell j.  The right value is the
// mirror image.
template <int ORD = 7>
__device__ __forceinline__ void meg7_pair(const double* v, const double* g, double& outL,
                                          double& outR) {
  const double dm1 = mp_curv(v[0], v[1], v[2], g[0], g[2]);
  const double d0 = mp_curv(v[1], v[2], v[3], g[1], g[3]);
  const double dp1 = mp_curv(v[2], v[3], v[4], g[2], g[4]);
  const double dp2 = mp_curv(v[3], v[4], v[5], g[3], g[5]);
  const double md = 0.5 * (v[2] + v[3]) - 0.5 * minmod(d0, dp1);
  {
    double phi = grb_l<ORD>(v, g);
    double pmp = v[2] + minmod(v[3] - v[2], kXiMP * (v[2] - v[1]));
    if ((phi - v[2]) * (phi - pmp) > kMPTol) {
      double ul = v[2] + kXiMP * (v[2] - v[1]);
      double lc = 0.5 * (3.0 * v[2] - v[1]) + (4.0 / 3.0) * minmod(d0, dm1);
      double lo = fmax(fmin(v[2], fmin(v[3], md)), fmin(v[2], fmin(ul, lc)));
      double hi = fmin(fmax(v[2], fmax(v[3], md)), fmax(v[2], fmax(ul, lc)));
      phi = phi + minmod(lo - phi, hi - phi);
    }
    outL = phi;
  }
  {
    double phi = grb_r<ORD>(v, g);
    double pmp = v[3] + minmod(v[2] - v[3], kXiMP * (v[3] - v[4]));
    if ((phi - v[3]) * (phi - pmp) > kMPTol) {
      double ul = v[3] + kXiMP * (v[3] - v[4]);
      double lc = 0.5 * (3.0 * v[3] - v[4]) + (4.0 / 3.0) * minmod(dp1, dp2);
      double lo = fmax(fmin(v[3], fmin(v[2], md)), fmin(v[3], fmin(ul, lc)));
      double hi = fmin(fmax(v[3], fmax(v[2], md)), fmax(v[3], fmax(ul, lc)));
      phi = phi + minmod(lo - phi, hi - phi);
    }
    outR = phi;
  }
}

// Characteristic MEG7 states at an interface (Secs. 2.3, 2.4, flagged
// branch).  Wf(q, f) returns rotated primitive field f at offset q-2
// (q = 0..5) from cell j; CG(fa, fb, ca, cb, cg) writes the normal gradients
// (spacing-scaled) of the combination ca * field fa + cb * field fb at the
// same six offsets.  Eigenvectors of the primitive normal Jacobian are taken
// at the mean density and pressure of cells j, j+1.  Each characteristic
// field combines two primitive fields (rows of L: (u_n, p), (rho, p), (u_t),
// (u_n, p)); the four fields are limited one at a time in a rolled loop that
// reads only its two primitive fields, which keeps the register footprint
// small, and are projected back by accumulating the columns of R.
template <int ORD = 7, class FW, class FC>
__device__ __forceinline__ void meg7_char_states_comb(FW Wf, FC CG, double gamma, double WLo[4],
                                                      double WRo[4]) {
  const double rb = 0.5 * (Wf(2, 0) + Wf(3, 0));
  const double pb = 0.5 * (Wf(2, 3) + Wf(3, 3));
  const double irb = rcp_nr(rb);
  const double cb = sqrt_nr(gamma * pb * irb);
  const double icb = rcp_nr(cb);
  const double h2c = 0.5 * icb, ic2 = icb * icb, h2c2 = 0.5 * ic2;
  const double cor = cb * irb, c2 = cb * cb;
#pragma unroll
  for (int m = 0; m < 4; ++m) { WLo[m] = 0.0; WRo[m] = 0.0; }
#pragma unroll 1
  for (int m = 0; m < 4; ++m) {
    // row m of L as ca * field fa + cb_ * field fb
    const int fa = (m == 1) ? 0 : ((m == 2) ? 2 : 1);
    const int fb = (m == 2) ? 2 : 3;
    const double ca = (m == 0) ? -rb * h2c : ((m == 3) ? rb * h2c : 1.0);
    const double cbv = (m == 1) ? -ic2 : ((m == 2) ? 0.0 : h2c2);
    double cv[6], cg[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) cv[q] = ca * Wf(q, fa) + cbv * Wf(q, fb);
    CG(fa, fb, ca, cbv, cg);
    double cl, cr;
    meg7_pair<ORD>(cv, cg, cl, cr);
    // column m of R = L^{-1}: (1,-c/rho,0,c^2), (1,0,0,0), (0,0,1,0), (1,c/rho,0,c^2)
    const double b0 = (m == 2) ? 0.0 : 1.0;
    const double b1 = (m == 0) ? -cor : ((m == 3) ? cor : 0.0);
    const double b2 = (m == 2) ? 1.0 : 0.0;
    const double b3 = (m == 0 || m == 3) ? c2 : 0.0;
    WLo[0] += b0 * cl; WLo[1] += b1 * cl; WLo[2] += b2 * cl; WLo[3] += b3 * cl;
    WRo[0] += b0 * cr; WRo[1] += b1 * cr; WRo[2] += b2 * cr; WRo[3] += b3 * cr;
  }
}

// The same with staged gradients: Gf(q, f) is the normal gradient of rotated
// field f at offset q-2.
template <int ORD = 7, class FW, class FG>
__device__ __forceinline__ void meg7_char_states(FW Wf, FG Gf, double gamma, double WLo[4],
                                                 double WRo[4]) {
  meg7_char_states_comb<ORD>(
      Wf,
      [&](int fa, int fb, double ca, double cb, double cg[6]) {
#pragma unroll
        for (int q = 0; q < 6; ++q) cg[q] = ca * Gf(q, fa) + cb * Gf(q, fb);
      },
      gamma, WLo, WRo);
}

// The same with the gradients formed from edge jumps: Ef(a, f) is the jump of
// rotated field f across edge (j - 5 + a) + 1/2, a = 0..10.  The gradient of
// eq. (eqn:six) at cell k is (37, -8, 1)/60 on the pairs of edges around k;
// being linear, it is taken once on the combined jumps of the two fields.
template <int ORD = 7, class FW, class FE>
__device__ __forceinline__ void meg7_char_states_edges(FW Wf, FE Ef, double gamma, double WLo[4],
                                                       double WRo[4]) {
  meg7_char_states_comb<ORD>(
      Wf,
      [&](int fa, int fb, double ca, double cb, double cg[6]) {
        double ce[11];
#pragma unroll
        for (int a = 0; a < 11; ++a) ce[a] = ca * Ef(a, fa) + cb * Ef(a, fb);
        constexpr double z = 1.0 / 60.0;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          cg[q] = z * (37.0 * (ce[q + 2] + ce[q + 3]) - 8.0 * (ce[q + 1] + ce[q + 4]) +
                       (ce[q] + ce[q + 5]));
      },
      gamma, WLo, WRo);
}

// Conservative (rho, rho un, rho ut, E) to primitive (rho, un, ut, p),
// eq. (eqn:pressure).  A non-positive density gives a non-positive or NaN
// result, which the positivity test of the callers rejects.
__device__ __forceinline__ void cons_to_prim(const double Q[4], double gamma, double W[4]) {
  const double ir = rcp_nr(Q[0]);
  W[0] = Q[0];
  W[1] = Q[1] * ir;
  W[2] = Q[2] * ir;
  W[3] = (gamma - 1.0) * (Q[3] - 0.5 * (Q[1] * W[1] + Q[2] * W[2]));
}

// Characteristic MEG7 states of MEG7-cons (Sec. 2.3 on conservative
// variables).  Qf(q, f) / Gf(q, f) return rotated conservative field f and its
// normal gradient (spacing-scaled) at offset q-2 from cell j.  The
// eigenvectors are those of the conservative normal flux Jacobian at the
// arithmetic mean of the conservative states of cells j and j+1, with
// b1 = (gamma-1)/c^2, b2 = b1 (u^2+v^2)/2.  Rows of L:
//   ((b2 + u/c)/2, -(b1 u + 1/c)/2, -b1 v/2, b1/2), (1 - b2, b1 u, b1 v, -b1),
//   (-v, 0, 1, 0), ((b2 - u/c)/2, -(b1 u - 1/c)/2, -b1 v/2, b1/2);
// columns of R = L^{-1}: (1, u-c, v, H-uc), (1, u, v, (u^2+v^2)/2), (0, 0, 1, v),
//   (1, u+c, v, H+uc).  Every row reads all four fields, so the rows are
// limited one at a time in a rolled loop and projected back column by column.
template <int ORD = 7, class FQ, class FG>
__device__ __forceinline__ void meg7_char_states_cons(FQ Qf, FG Gf, double gamma,
                                                      double QLo[4], double QRo[4]) {
  const double q0 = 0.5 * (Qf(2, 0) + Qf(3, 0)), q1 = 0.5 * (Qf(2, 1) + Qf(3, 1));
  const double q2 = 0.5 * (Qf(2, 2) + Qf(3, 2)), q3 = 0.5 * (Qf(2, 3) + Qf(3, 3));
  const double iq0 = rcp_nr(q0);
  const double ub = q1 * iq0, vb = q2 * iq0;
  const double ke = 0.5 * (ub * ub + vb * vb);
  const double pb = (gamma - 1.0) * (q3 - q0 * ke);
  const double hb = (q3 + pb) * iq0;
  const double cb = sqrt_nr(gamma * pb * iq0);
  const double icb = rcp_nr(cb);
  const double b1 = (gamma - 1.0) * icb * icb, b2 = b1 * ke;
#pragma unroll
  for (int m = 0; m < 4; ++m) { QLo[m] = 0.0; QRo[m] = 0.0; }
#pragma unroll 1
  for (int m = 0; m < 4; ++m) {
    // the field reads do not depend on m: keep them inside the loop (an empty
    // asm with a memory clobber stops the compiler hoisting all 48 of them)
    __asm__ volatile("" ::: "memory");
    const double sg = (m == 0) ? 1.0 : -1.0;   // u/c and 1/c enter rows 0 and 3 with opposite signs
    double l0, l1, l2, l3;
    if (m == 1) {
      l0 = 1.0 - b2; l1 = b1 * ub; l2 = b1 * vb; l3 = -b1;
    } else if (m == 2) {
      l0 = -vb; l1 = 0.0; l2 = 1.0; l3 = 0.0;
    } else {
      l0 = 0.5 * (b2 + sg * ub * icb);
      l1 = -0.5 * (b1 * ub + sg * icb);
      l2 = -0.5 * b1 * vb;
      l3 = 0.5 * b1;
    }
    double cv[6], cg[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      cv[q] = l0 * Qf(q, 0) + l1 * Qf(q, 1) + l2 * Qf(q, 2) + l3 * Qf(q, 3);
      cg[q] = l0 * Gf(q, 0) + l1 * Gf(q, 1) + l2 * Gf(q, 2) + l3 * Gf(q, 3);
    }
    double cl, cr;
    meg7_pair<ORD>(cv, cg, cl, cr);
    double r0, r1, r2, r3;
    if (m == 1) {
      r0 = 1.0; r1 = ub; r2 = vb; r3 = ke;
    } else if (m == 2) {
      r0 = 0.0; r1 = 0.0; r2 = 1.0; r3 = vb;
    } else {
      r0 = 1.0; r1 = ub - sg * cb; r2 = vb; r3 = hb - sg * ub * cb;
    }
    QLo[0] += r0 * cl; QLo[1] += r1 * cl; QLo[2] += r2 * cl; QLo[3] += r3 * cl;
    QRo[0] += r0 * cr; QRo[1] += r1 * cr; QRo[2] += r2 * cr; QRo[3] += r3 * cr;
  }
}

// Normal convective flux of the state W (Sec. 1 flux vectors, rotated).
__device__ __forceinline__ void conv_flux(const double W[4], double g1inv, double F[4]) {
  const double E = W[3] * g1inv + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2]);
  const double m = W[0] * W[1];
  F[0] = m;
  F[1] = m * W[1] + W[3];
  F[2] = m * W[2];
  F[3] = W[1] * (E + W[3]);
}

// Jump of the normal convective flux between states Wm and Wp, F(Wp) - F(Wm),
// written on the primitive jumps so that it is exactly zero for equal states
// and carries no cancellation of the flux magnitudes.
__device__ __forceinline__ void conv_flux_jump(const double Wm[4], const double Wp[4],
                                               double g1inv, double dF[4]) {
  const double dr = Wp[0] - Wm[0], du = Wp[1] - Wm[1], dv = Wp[2] - Wm[2], dp = Wp[3] - Wm[3];
  const double mp = Wp[0] * Wp[1];
  const double dm = Wp[0] * du + Wm[1] * dr;  // jump of rho un
  const double Em = Wm[3] * g1inv + 0.5 * Wm[0] * (Wm[1] * Wm[1] + Wm[2] * Wm[2]);
  const double dE = dp * g1inv + 0.5 * (dr * (Wm[1] * Wm[1] + Wm[2] * Wm[2]) +
                                        Wp[0] * (du * (Wp[1] + Wm[1]) + dv * (Wp[2] + Wm[2])));
  dF[0] = dm;
  dF[1] = mp * du + Wm[1] * dm + dp;
  dF[2] = mp * dv + Wm[2] * dm;
  dF[3] = Wp[1] * (dE + dp) + (Em + Wm[3]) * du;
}

// sin(x) for x in [0, pi/2]: its Taylor series to x^21 (truncation below
// 3e-16 on that interval), in Horner form on x^2.  Small in registers, unlike
// the library sine, so it can sit inside the Riemann solver.
__device__ __forceinline__ double sin_quarter(double x) {
  const double z = x * x;
  double t = 1.0 / 51090942171709440000.0;          // 1/21!
  t = fma(t, -z, 1.0 / 121645100408832000.0);        // 1/19!
  t = fma(t, -z, 1.0 / 355687428096000.0);           // 1/17!
  t = fma(t, -z, 1.0 / 1307674368000.0);             // 1/15!
  t = fma(t, -z, 1.0 / 6227020800.0);                // 1/13!
  t = fma(t, -z, 1.0 / 39916800.0);                  // 1/11!
  t = fma(t, -z, 1.0 / 362880.0);                    // 1/9!
  t = fma(t, -z, 1.0 / 5040.0);                      // 1/7!
  t = fma(t, -z, 1.0 / 120.0);                       // 1/5!
  t = fma(t, -z, 1.0 / 6.0);                         // 1/3!
  t = fma(t, -z, 1.0);
  return x * t;
}

// HLLC with Einfeldt (Roe-average) bounds in the wave-sum form
//   F = (F_L + F_R)/2 - (phi |S_L|(Q*_L - Q_L) + |S*|(Q*_R - Q*_L) + phi |S_R|(Q_R - Q*_R))/2
// which is the canonical form of eq. (eqn:Riemann).  Only the mean
// Fm = (F_L + F_R)/2 of the reconstructed fluxes enters, so callers pass it.
// phi = 1 for HLLC; the shock-stable (low-Mach-limited) form takes
// phi = sin(pi/2 min(1, Ma/0.1)), Ma = max(|u_L|/c_L, |u_R|/c_R).
template <bool LOW_MACH = false>
__device__ __forceinline__ void hllc(const double WL[4], const double WR[4], const double Fm[4],
                                     double gamma, double g1inv, double F[4]) {
  const double rl = WL[0], ul = WL[1], vl = WL[2], pl = WL[3];
  const double rr = WR[0], ur = WR[1], vr = WR[2], pr = WR[3];
  const double yl = rsq_nr(rl), yr = rsq_nr(rr);
  const double sl = rl * yl, sr = rr * yr;          // sqrt(rho)
  const double irl = yl * yl, irr = yr * yr;        // 1/rho
  const double El = pl * g1inv + 0.5 * rl * (ul * ul + vl * vl);
  const double Er = pr * g1inv + 0.5 * rr * (ur * ur + vr * vr);
  const double cl = sqrt_nr(gamma * pl * irl), cr = sqrt_nr(gamma * pr * irr);
  const double hl = (El + pl) * irl, hr = (Er + pr) * irr;
  const double iss = rcp_nr(sl + sr);
  const double ut = (sl * ul + sr * ur) * iss;
  const double vt = (sl * vl + sr * vr) * iss;
  const double ht = (sl * hl + sr * hr) * iss;
  const double ct = sqrt_nr((gamma - 1.0) * (ht - 0.5 * (ut * ut + vt * vt)));
  const double SL = fmin(ul - cl, ut - ct);
  const double SR = fmax(ur + cr, ut + ct);
  const double ml = rl * (SL - ul), mr = rr * (SR - ur);
  const double Ss = (pr - pl + ml * ul - mr * ur) * rcp_nr(ml - mr);
  const double kl = ml * rcp_nr(SL - Ss), kr = mr * rcp_nr(SR - Ss);
  const double QL[4] = {rl, rl * ul, rl * vl, El};
  const double QR[4] = {rr, rr * ur, rr * vr, Er};
  const double QsL[4] = {kl, kl * Ss, kl * vl, kl * (El * irl + (Ss - ul) * (Ss + pl * rcp_nr(ml)))};
  const double QsR[4] = {kr, kr * Ss, kr * vr, kr * (Er * irr + (Ss - ur) * (Ss + pr * rcp_nr(mr)))};
  double phi = 1.0;
  if (LOW_MACH) {
    const double ma = fmax(fabs(ul) / cl, fabs(ur) / cr);
    if (ma < 0.1) phi = sin_quarter((0.5 * 3.14159265358979323846) * (ma / 0.1));
  }
  const double aL = phi * fabs(SL), aS = fabs(Ss), aR = phi * fabs(SR);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double diss = aL * (QsL[m] - QL[m]) + aS * (QsR[m] - QsL[m]) + aR * (QR[m] - QsR[m]);
    F[m] = Fm[m] - 0.5 * diss;
  }
}

// Viscous interface flux (Sec. 2.1) added to F: normal derivatives of un,
// ut, T by alpha-damping (eq. eqn:alphad, alpha_v = 4) from the shared
// gradients, tangential derivatives and velocities as two-cell means.
// g* are spacing-scaled normal gradients, d*_t true tangential derivatives.
__device__ __forceinline__ void viscous_add(double un0, double un1, double ut0, double ut1,
                                            double T0, double T1, double gun0, double gun1,
                                            double gut0, double gut1, double gT0, double gT1,
                                            double dunt0, double dunt1, double dutt0,
                                            double dutt1, double inv_dn, double mu,
                                            double kq, double F[4]) {
  // dn * dPhi/dn at j+1/2 = (g0+g1)/2 + alpha_v/2 (Phi1 - g1/2 - Phi0 - g0/2)
  const double a2 = 0.5 * kAlphaV;
  const double dun = (0.5 * (gun0 + gun1) + a2 * (un1 - 0.5 * gun1 - un0 - 0.5 * gun0)) * inv_dn;
  const double dut = (0.5 * (gut0 + gut1) + a2 * (ut1 - 0.5 * gut1 - ut0 - 0.5 * gut0)) * inv_dn;
  const double dT = (0.5 * (gT0 + gT1) + a2 * (T1 - 0.5 * gT1 - T0 - 0.5 * gT0)) * inv_dn;
  const double dunt = 0.5 * (dunt0 + dunt1), dutt = 0.5 * (dutt0 + dutt1);
  const double unf = 0.5 * (un0 + un1), utf = 0.5 * (ut0 + ut1);
  const double tnn = (2.0 / 3.0) * mu * (2.0 * dun - dutt);
  const double tnt = mu * (dut + dunt);
  const double qn = -kq * dT;  // kq = mu / (Pr (gamma - 1))
  F[1] -= tnn;
  F[2] -= tnt;
  F[3] += -(tnn * unf + tnt * utf) + qn;
}

}  // namespace gbr
