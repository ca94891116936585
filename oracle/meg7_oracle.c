/*
 * meg7_oracle.c -- plain, slow, FP64 CPU oracle for the MEG7 scheme of
 * Chamarthi, "Efficient high-order Gradient-based Reconstruction for
 * compressible flows" (arXiv 2305.00762).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or helper with the HIP path in paper_2305_00762_amd/csrc/.
 *
 * Every step follows the paper in its own order and notation:
 *   Sec. 1      eq. (CNS-base), the flux vectors, eq. (eqn:pressure),
 *               eq. (eqn:visc)                         -> physics
 *   Sec. 1      eqs. (eqn-differencing_residual), (deriv), (eqn:Riemann)
 *                                                      -> residual
 *   Sec. 2.1    eqs. (eqn:visc-interface), (eqn:alphad), (sixth-ordergrad)
 *                                                      -> viscous flux
 *   Sec. 2.2    eqs. (eqn:six), (eqn:grb)              -> GRB states
 *   Sec. 2.3    eqs. (eqn:hocus/mp5Condition), (eqn:alpha),
 *               (eqn:mp-procedure)                     -> MP limiter (MEG7)
 *   Sec. 2.4    hybrid F_L / F_R, eqs. (flux-full), (flux-right),
 *               the detector and eq. (buffer)          -> hybrid flux
 *   Sec. 2.5    eq. (rk) and the CFL time step          -> time integration
 *
 * Readings taken where the paper is silent or garbled:
 *   R-T    T := gamma p / rho, so that q = -mu/(Pr(gamma-1)) dT/dx matches
 *          kappa = Cp mu / Pr (Cp cancels).
 *   R-DET  psi = (2ab + eps) / (a^2 + b^2 + eps): the printed psi omits the
 *          eps that eq. (buffer) defines; with it the free stream (a=b=0)
 *          is defined and a=0, b=xi gives psi = 0.9 psi_c exactly.  One
 *          detector per direction, on density; psi == psi_c gives sigma=1.
 *   R-MP   The MP limiter and the characteristic projection act only on
 *          interfaces the detector flags (sigma = 0); sigma = 1 interfaces
 *          use the unlimited GRB states (mp_mode 0).  mp_mode 1 applies the
 *          MP test to the states of every interface.
 *   R-CHAR Characteristic variables: left/right eigenvectors of the
 *          primitive-variable Jacobian at the arithmetic-mean density and
 *          pressure of the two cells beside the interface.
 *   R-HLLC HLLC of Toro with Einfeldt (Roe-average) wave-speed bounds,
 *          evaluated in the wave-sum form of eq. (eqn:Riemann); with
 *          F_L = F(Q_L), F_R = F(Q_R) it is the textbook HLLC flux.
 *   R-VISC 2D viscous interface flux: normal derivatives alpha-damped,
 *          tangential derivatives and interface velocities as two-cell
 *          means; mu constant.
 *   R-BC   Ghost cells (6 layers): periodic wrap or zeroth-order copy
 *          (transmissive).
 *   R-POS  A reconstructed interface state with non-positive density or
 *          pressure (or a non-finite one) -- which characteristic MP limiting
 *          does not exclude where discontinuities interact -- is replaced by
 *          the first-order state: U_L = U_j, U_R = U_{j+1}, F_L = F(U_j),
 *          F_R = F(U_{j+1}).  The paper prescribes no positivity treatment
 *          for these cases.
 *   R-CONS MEG7-cons (recon = 1): eq. (eqn:grb) and the MP procedure act on
 *          the conservative variables and their sixth-order gradients; the
 *          velocity gradients of the viscous flux follow from the printed
 *          chain rule, du = (d(rho u) - u d rho)/rho (normal and tangential),
 *          and T' stays the sixth-order difference of T (R-T).
 *   R-CHARC The characteristic variables of MEG7-cons use the eigenvectors of
 *          the conservative-variable flux Jacobian at the arithmetic mean of
 *          the two conservative states beside the interface.
 *   R-G4   The fourth-order GRB (order = 4) is the subset alpha = 4, beta = 0
 *          of eqs. (good_6tth-order_scheme_flux), (alpha-beta) with the same
 *          sixth-order gradients.  It replaces the interface states of eq.
 *          (eqn:grb) wherever they enter (the unlimited states of the smooth
 *          branch and the value the MP procedure starts from) and the flux
 *          reconstruction by eq. (fourth); F(f_R) is the mirror image of
 *          eq. (fourth), as eq. (flux-right) mirrors eq. (flux-full).  The
 *          detector, the MP bounds, HLLC and the viscous flux are unchanged.
 *   R-WALL Boundaries beyond periodic and transmissive (the paper refers to the
 *          usual ghost-cell treatment of its test cases): a reflecting wall
 *          mirrors the cells about the wall and negates the normal velocity;
 *          an adiabatic no-slip wall mirrors and negates both velocity
 *          components; an inflow side holds a fixed state in all six ghost
 *          layers.  A side may switch kind at a point that moves with time
 *          (the double Mach reflection).  In a corner ghost cell the mirror
 *          and sign rules of both sides compose; a fixed state of the x side
 *          takes precedence over one of the y side.  Runge-Kutta stage k
 *          evaluates the boundary at t + c_k dt, c = (0, 1, 1/2).
 *   R-SSHLLC The shock-stable HLLC the paper cites for the double Mach
 *          reflection (Fleischmann et al.) is taken as its low-Mach-limited
 *          form: the two acoustic-wave terms of the wave-sum form are scaled by
 *          phi = sin(pi/2 min(1, Ma/0.1)), Ma = max(|u_L|/c_L, |u_R|/c_R) of
 *          the normal velocities; the contact term and the wave-speed bounds
 *          are those of R-HLLC.
 *   R-MPG  In eq. (eqn:mp-procedure) the hat on Phi_{j-1} and the mixed
 *          i/j subscripts are typesetting slips: plain Phi_{j-1}, index j.
 *          The MP xi (=7) and the detector xi (=1e-3) are different
 *          constants.  The right state is the mirror image of the left.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA
 * contraction anywhere, so the detector is evaluated with one rounding per
 * operation in the order written).
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NG 6 /* ghost layers: the shock branch reaches Phi_{j-5..j+6} */

enum { ORC_BC_PERIODIC = 0, ORC_BC_TRANSMISSIVE = 1, ORC_BC_REFLECT = 2, ORC_BC_NOSLIP = 3,
       ORC_BC_INFLOW = 4 };

/* One side of the domain (reading R-WALL): two segments along the side,
 * segment 0 where the tangential cell-centre coordinate is below
 * split0 + split_speed * t, segment 1 elsewhere; each with a boundary kind
 * and, for ORC_BC_INFLOW, a fixed primitive state (rho, u, v, p). */
typedef struct {
    int kind[2];
    double state[2][4];
    double split0, split_speed;
} orc_side;

typedef struct {
    int nx, ny;
    double x0, x1, y0, y1;
    int bc_x, bc_y;
    double gamma, mu, Pr;
    int mp_mode;   /* 0: MP only where sigma=0 (R-MP); 1: MP test everywhere */
    int force_sigma; /* -1: detector decides; 0 or 1: force sigma (tests)    */
    int recon;     /* 0: primitive variables (MEG7-prim); 1: conservative (MEG7-cons) */
    int order;     /* 7: the seventh-order GRB of Sec. 2.2; 4: its fourth-order subset */
    int riemann;   /* 0: HLLC (R-HLLC); 1: shock-stable HLLC (R-SSHLLC) */
    int use_sides; /* 0: bc_x / bc_y on both sides; 1: the side table below */
    double t;      /* time of the state a residual is evaluated on (moving segments) */
    orc_side side[4];  /* left (x0), right (x1), bottom (y0), top (y1) */
} orc_cfg;

/* ---------------------------------------------------------------------- */
/* Constants of the paper.                                                 */
/* ---------------------------------------------------------------------- */
static const double PI = 3.14159265358979323846;
static const double ALPHA_V = 4.0;      /* eq. (eqn:alphad): alpha_v = 4            */
static const double XI_MP = 7.0;        /* eq. (eqn:alpha): xi = 7                  */
static const double MP_TOL = 1e-40;     /* eq. (eqn:hocus/mp5Condition)             */
static const double PSI_C = 0.5;        /* eq. (buffer)                             */
static const double XI_DET = 1e-3;      /* eq. (buffer)                             */

/* Threads of the parallel loops (OpenMP; n < 1 restores the default) and the
 * number a parallel loop would use now. */
void orc_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
}

int orc_get_threads(void)
{
    return omp_get_max_threads();
}

double orc_detector_eps(void)
{
    /* eq. (buffer): eps = 0.9 psi_c / (1 - 0.9 psi_c) * xi^2 */
    return (0.9 * PSI_C) / (1.0 - 0.9 * PSI_C) * (XI_DET * XI_DET);
}

/* ---------------------------------------------------------------------- */
/* Coefficient tables exactly as printed (integer numerators over a        */
/* common denominator).  Exported so tests can check them against the      */
/* paper's derivation from (alpha, beta).                                  */
/* ---------------------------------------------------------------------- */
/* eq. (eqn:six): Phi'_j = [45(P_{j+1}-P_{j-1}) - 9(P_{j+2}-P_{j-2}) + (P_{j+3}-P_{j-3})]/60 */
static const int GRAD6[7] = {-1, 9, -45, 0, 45, -9, 1}; /* offsets -3..3, /60 */
static const int GRAD6_DEN = 60;
/* eq. (eqn:grb), left state at j+1/2: values at offsets -2..2, gradients at -1..1, /840 */
static const int GRB_L_VAL[5] = {3, 178, 478, 178, 3};
static const int GRB_L_GRD[3] = {60, 420, -60};
/* eq. (eqn:grb), right state at j+1/2: values at offsets -1..3, gradients at 0..2, /840 */
static const int GRB_R_VAL[5] = {3, 178, 478, 178, 3};
static const int GRB_R_GRD[3] = {60, -420, -60};
static const int GRB_DEN = 840;
/* eq. (flux-full): F(f_L) on offsets -4..4, /840 */
static const int FLUX_L[9] = {-1, 2, 22, -146, 568, 484, -104, 16, -1};
/* eq. (flux-right): F(f_R) on offsets -3..5, /840 */
static const int FLUX_R[9] = {-1, 16, -104, 484, 568, -146, 22, 2, -1};
static const int FLUX_DEN = 840;
/* eq. (eqn:grb-sec): Delta x^2 Phi_xx = (60 P'_{j-1} - 60 P'_{j+1} - 362 P_j
 * + 178 (P_{j-1}+P_{j+1}) + 3 (P_{j-2}+P_{j+2}))/70 -- exported for tests only. */
static const int SEC_VAL[5] = {3, 178, -362, 178, 3};
static const int SEC_GRD[3] = {60, 0, -60};
static const int SEC_DEN = 70;

/* which: 0 grad6, 1 grb_L values, 2 grb_L grads, 3 grb_R values, 4 grb_R grads,
 *        5 flux_L, 6 flux_R, 7 second-derivative values, 8 second-derivative grads.
 * Writes the numerators into num[], returns the count; *den gets the denominator. */
int orc_table(int which, int *num, int *den)
{
    const int *t; int n, d;
    switch (which) {
    case 0: t = GRAD6; n = 7; d = GRAD6_DEN; break;
    case 1: t = GRB_L_VAL; n = 5; d = GRB_DEN; break;
    case 2: t = GRB_L_GRD; n = 3; d = GRB_DEN; break;
    case 3: t = GRB_R_VAL; n = 5; d = GRB_DEN; break;
    case 4: t = GRB_R_GRD; n = 3; d = GRB_DEN; break;
    case 5: t = FLUX_L; n = 9; d = FLUX_DEN; break;
    case 6: t = FLUX_R; n = 9; d = FLUX_DEN; break;
    case 7: t = SEC_VAL; n = 5; d = SEC_DEN; break;
    case 8: t = SEC_GRD; n = 3; d = SEC_DEN; break;
    default: return -1;
    }
    for (int k = 0; k < n; ++k) num[k] = t[k];
    *den = d;
    return n;
}

/* ---------------------------------------------------------------------- */
/* Small building blocks, each an equation of the paper.                   */
/* ---------------------------------------------------------------------- */

/* eq. (eqn:six) / (sixth-ordergrad): Phi' = Delta x * dPhi/dx at the centre
 * of p[0..6] (offsets -3..3). */
double orc_grad6(const double *p)
{
    return (45.0 * (p[4] - p[2]) - 9.0 * (p[5] - p[1]) + (p[6] - p[0])) / 60.0;
}

/* The detector of Sec. 2.4 (eq. detector, reading R-DET) at cell j from
 * rho_{j-2..j+2}; evaluated with one rounding per operation in this order. */
double orc_psi(double rm2, double rm1, double r0, double rp1, double rp2)
{
    const double eps = orc_detector_eps();
    double a = fabs(r0 - rm1) + fabs((r0 - 2.0 * rm1) + rm2);
    double b = fabs(r0 - rp1) + fabs((r0 - 2.0 * rp1) + rp2);
    double num = (2.0 * a) * b + eps;
    double den = (a * a + b * b) + eps;
    return num / den;
}

/* eq. (eqn:grb): left state at j+1/2 from p[-2..2] (p points at j) and
 * gradients g[-1..1] (Phi' = Delta x dPhi/dx, g points at j). */
static double grb_left(const double *p, const double *g)
{
    return (420.0 * g[0] + 60.0 * g[-1] - 60.0 * g[1] + 478.0 * p[0] + 178.0 * p[-1]
            + 3.0 * p[-2] + 178.0 * p[1] + 3.0 * p[2]) / 840.0;
}

/* eq. (eqn:grb): right state at j+1/2 from p[-1..3] and g[0..2] (pointers at j). */
static double grb_right(const double *p, const double *g)
{
    return (60.0 * g[0] - 420.0 * g[1] - 60.0 * g[2] + 178.0 * p[0] + 3.0 * p[-1]
            + 478.0 * p[1] + 178.0 * p[2] + 3.0 * p[3]) / 840.0;
}

/* eq. (flux-full): F(f_L) at j+1/2 from f[-4..4] (pointer at j). */
static double flux_left(const double *f)
{
    return (568.0 * f[0] - 146.0 * f[-1] + 22.0 * f[-2] + 2.0 * f[-3] - f[-4]
            + 484.0 * f[1] - 104.0 * f[2] + 16.0 * f[3] - f[4]) / 840.0;
}

/* eq. (flux-right): F(f_R) at j+1/2 from f[-3..5] (pointer at j). */
static double flux_right(const double *f)
{
    return (-f[5] + 2.0 * f[4] + 22.0 * f[3] - 146.0 * f[2] + 568.0 * f[1]
            + 484.0 * f[0] - 104.0 * f[-1] + 16.0 * f[-2] - f[-3]) / 840.0;
}

/* The two-parameter family of Sec. 2.2, written out in the paper's order
 * (used for the fourth-order subset, and by tests at any alpha, beta).
 * p, g point at cell j; p[-2..2] and g[-1..1] are read.                   */

/* eq. (alpha-beta): one-sided values at interface k+1/2 (p, g at cell k). */
static void ab_face_states(const double *p, const double *g, double beta, double *PL,
                           double *PR)
{
    *PL = p[0] + 0.5 * g[0] + beta * (p[1] - 2.0 * p[0] + p[-1]);
    *PR = p[1] - 0.5 * g[1] + beta * (p[2] - 2.0 * p[1] + p[0]);
}

/* eq. (good_6tth-order_scheme_flux), times Delta x: the gradient at k+1/2. */
static double ab_face_grad(const double *p, const double *g, double alpha, double beta)
{
    double PL, PR;
    ab_face_states(p, g, beta, &PL, &PR);
    return 0.5 * (g[0] + g[1]) + 0.5 * alpha * (PR - PL);
}

/* eq. (eqn:how-second), times Delta x^2: the second derivative in cell j. */
static double ab_second(const double *p, const double *g, double alpha, double beta)
{
    return ab_face_grad(p, g, alpha, beta) - ab_face_grad(p - 1, g - 1, alpha, beta);
}

/* eq. (eqn:lingrb): left and right states at j+1/2. */
static double grb_ab_left(const double *p, const double *g, double alpha, double beta)
{
    return p[0] + 0.5 * g[0] + ab_second(p, g, alpha, beta) / 12.0;
}
static double grb_ab_right(const double *p, const double *g, double alpha, double beta)
{
    return p[1] - 0.5 * g[1] + ab_second(p + 1, g + 1, alpha, beta) / 12.0;
}

/* eq. (fourth): F(f_L) of the fourth-order GRB at j+1/2 from f[-4..4]. */
static double flux4_left(const double *f)
{
    return (1050.0 * f[0] - 309.0 * f[-1] + 64.0 * f[-2] - 3.0 * f[-3] - f[-4]
            + 771.0 * f[1] - 152.0 * f[2] + 21.0 * f[3] - f[4]) / 1440.0;
}

/* Mirror image of eq. (fourth): F(f_R) at j+1/2 from f[-3..5]. */
static double flux4_right(const double *f)
{
    return (1050.0 * f[1] - 309.0 * f[2] + 64.0 * f[3] - 3.0 * f[4] - f[5]
            + 771.0 * f[0] - 152.0 * f[-1] + 21.0 * f[-2] - f[-3]) / 1440.0;
}

/* Interface states and flux reconstruction of the selected order. */
static double grb_L(int order, const double *p, const double *g)
{
    return order == 4 ? grb_ab_left(p, g, 4.0, 0.0) : grb_left(p, g);
}
static double grb_R(int order, const double *p, const double *g)
{
    return order == 4 ? grb_ab_right(p, g, 4.0, 0.0) : grb_right(p, g);
}
static double flux_L(int order, const double *f)
{
    return order == 4 ? flux4_left(f) : flux_left(f);
}
static double flux_R(int order, const double *f)
{
    return order == 4 ? flux4_right(f) : flux_right(f);
}

/* Exported stencil applications for the polynomial / symbol tests. */
void orc_apply_interface(const double *v10, const double *g6, double out[4])
{
    /* v10: values at offsets -4..5, g6: gradients at offsets -2..3 (interface
     * j+1/2, j at index 4 of v10 and index 2 of g6).
     * out = {GRB left, GRB right, F(f_L), F(f_R)} */
    out[0] = grb_left(v10 + 4, g6 + 2);
    out[1] = grb_right(v10 + 4, g6 + 2);
    out[2] = flux_left(v10 + 4);
    out[3] = flux_right(v10 + 4);
}

/* As orc_apply_interface for the fourth-order subset (order 4). */
void orc_apply_interface4(const double *v10, const double *g6, double out[4])
{
    out[0] = grb_L(4, v10 + 4, g6 + 2);
    out[1] = grb_R(4, v10 + 4, g6 + 2);
    out[2] = flux_L(4, v10 + 4);
    out[3] = flux_R(4, v10 + 4);
}

/* GRB states of the two-parameter family at any (alpha, beta): out = {L, R}. */
void orc_apply_interface_ab(const double *v10, const double *g6, double alpha, double beta,
                            double out[2])
{
    out[0] = grb_ab_left(v10 + 4, g6 + 2, alpha, beta);
    out[1] = grb_ab_right(v10 + 4, g6 + 2, alpha, beta);
}

static double minmod(double a, double b)
{
    /* eq. (eqn:alpha): minmod(a,b) = (sign(a)+sign(b))/2 * min(|a|,|b|) */
    double sa = (a > 0.0) - (a < 0.0);
    double sb = (b > 0.0) - (b < 0.0);
    return 0.5 * (sa + sb) * fmin(fabs(a), fabs(b));
}

static double min3(double a, double b, double c) { return fmin(a, fmin(b, c)); }
static double max3(double a, double b, double c) { return fmax(a, fmax(b, c)); }

/* MP curvature of eq. (eqn:mp-procedure):
 * d_j = 2(P_{j+1} - 2P_j + P_{j-1}) - 0.5 (P'_{j+1} - P'_{j-1}) */
static double mp_curv(const double *p, const double *g)
{
    return 2.0 * (p[1] - 2.0 * p[0] + p[-1]) - 0.5 * (g[1] - g[-1]);
}

/* Sec. 2.3: MEG7 left value at j+1/2 for one scalar component, starting
 * from the GRB state of the given order.  p, g point at cell j; p[-2..3],
 * g[-2..3] are read. */
static double meg7_left_o(int order, const double *p, const double *g, int *limited)
{
    double phi = grb_L(order, p, g);
    double phi_mp = p[0] + minmod(p[1] - p[0], XI_MP * (p[0] - p[-1]));
    if ((phi - p[0]) * (phi - phi_mp) <= MP_TOL) {
        if (limited) *limited = 0;
        return phi;
    }
    double dm1 = mp_curv(p - 1, g - 1);
    double d0 = mp_curv(p, g);
    double dp1 = mp_curv(p + 1, g + 1);
    double md = 0.5 * (p[0] + p[1]) - 0.5 * minmod(d0, dp1);
    double ul = p[0] + XI_MP * (p[0] - p[-1]);
    double lc = 0.5 * (3.0 * p[0] - p[-1]) + (4.0 / 3.0) * minmod(d0, dm1);
    double pmin = fmax(min3(p[0], p[1], md), min3(p[0], ul, lc));
    double pmax = fmin(max3(p[0], p[1], md), max3(p[0], ul, lc));
    if (limited) *limited = 1;
    return phi + minmod(pmin - phi, pmax - phi);
}

/* Mirror image of meg7_left_o: right value at j+1/2 (p, g point at j). */
static double meg7_right_o(int order, const double *p, const double *g, int *limited)
{
    double phi = grb_R(order, p, g);
    double phi_mp = p[1] + minmod(p[0] - p[1], XI_MP * (p[1] - p[2]));
    if ((phi - p[1]) * (phi - phi_mp) <= MP_TOL) {
        if (limited) *limited = 0;
        return phi;
    }
    double d0 = mp_curv(p, g);
    double dp1 = mp_curv(p + 1, g + 1);
    double dp2 = mp_curv(p + 2, g + 2);
    double md = 0.5 * (p[1] + p[0]) - 0.5 * minmod(dp1, d0);
    double ul = p[1] + XI_MP * (p[1] - p[2]);
    double lc = 0.5 * (3.0 * p[1] - p[2]) + (4.0 / 3.0) * minmod(dp1, dp2);
    double pmin = fmax(min3(p[1], p[0], md), min3(p[1], ul, lc));
    double pmax = fmin(max3(p[1], p[0], md), max3(p[1], ul, lc));
    if (limited) *limited = 1;
    return phi + minmod(pmin - phi, pmax - phi);
}

/* The seventh-order MEG7 values (exported for the tests). */
double orc_meg7_left(const double *p, const double *g, int *limited)
{
    return meg7_left_o(7, p, g, limited);
}
double orc_meg7_right(const double *p, const double *g, int *limited)
{
    return meg7_right_o(7, p, g, limited);
}

/* ---------------------------------------------------------------------- */
/* Physics in a frame rotated to the interface normal: W = (rho, un, ut, p),
 * Q = (rho, rho un, rho ut, E).                                           */
/* ---------------------------------------------------------------------- */

/* eq. (eqn:pressure) inverted: conservative from primitive. */
static void prim_to_cons(const double W[4], double gamma, double Q[4])
{
    Q[0] = W[0];
    Q[1] = W[0] * W[1];
    Q[2] = W[0] * W[2];
    Q[3] = W[3] / (gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2]);
}

/* The convective flux vector of Sec. 1 along the normal. */
static void conv_flux(const double W[4], double gamma, double F[4])
{
    double Q[4];
    prim_to_cons(W, gamma, Q);
    F[0] = W[0] * W[1];
    F[1] = W[0] * W[1] * W[1] + W[3];
    F[2] = W[0] * W[1] * W[2];
    F[3] = W[1] * (Q[3] + W[3]);
}

/* HLLC (Toro 1994), reading R-HLLC, written in the wave-sum form
 * F = (F_L + F_R)/2 - (|S_L|(Q*_L - Q_L) + |S*|(Q*_R - Q*_L) + |S_R|(Q_R - Q*_R))/2
 * which is the canonical form of eq. (eqn:Riemann). */
static void hllc_impl(const double WL[4], const double WR[4], const double FL[4],
                      const double FR[4], double gamma, int riemann, double F[4])
{
    double QL[4], QR[4];
    prim_to_cons(WL, gamma, QL);
    prim_to_cons(WR, gamma, QR);
    double rl = WL[0], ul = WL[1], vl = WL[2], pl = WL[3];
    double rr = WR[0], ur = WR[1], vr = WR[2], pr = WR[3];
    double cl = sqrt(gamma * pl / rl);
    double cr = sqrt(gamma * pr / rr);
    double hl = (QL[3] + pl) / rl;
    double hr = (QR[3] + pr) / rr;
    /* Roe averages */
    double sl_ = sqrt(rl), sr_ = sqrt(rr);
    double ut = (sl_ * ul + sr_ * ur) / (sl_ + sr_);
    double vt = (sl_ * vl + sr_ * vr) / (sl_ + sr_);
    double ht = (sl_ * hl + sr_ * hr) / (sl_ + sr_);
    double ct = sqrt((gamma - 1.0) * (ht - 0.5 * (ut * ut + vt * vt)));
    /* Einfeldt bounds */
    double SL = fmin(ul - cl, ut - ct);
    double SR = fmax(ur + cr, ut + ct);
    double Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur))
              / (rl * (SL - ul) - rr * (SR - ur));
    double QsL[4], QsR[4];
    double kl = rl * (SL - ul) / (SL - Ss);
    QsL[0] = kl;
    QsL[1] = kl * Ss;
    QsL[2] = kl * vl;
    QsL[3] = kl * (QL[3] / rl + (Ss - ul) * (Ss + pl / (rl * (SL - ul))));
    double kr = rr * (SR - ur) / (SR - Ss);
    QsR[0] = kr;
    QsR[1] = kr * Ss;
    QsR[2] = kr * vr;
    QsR[3] = kr * (QR[3] / rr + (Ss - ur) * (Ss + pr / (rr * (SR - ur))));
    /* reading R-SSHLLC: the acoustic-wave terms scaled by phi at low Mach */
    double phi = 1.0;
    if (riemann == 1) {
        double ma = fmax(fabs(ul) / cl, fabs(ur) / cr);
        phi = sin(0.5 * PI * fmin(1.0, ma / 0.1));
    }
    for (int m = 0; m < 4; ++m) {
        double diss = phi * fabs(SL) * (QsL[m] - QL[m]) + fabs(Ss) * (QsR[m] - QsL[m])
                    + phi * fabs(SR) * (QR[m] - QsR[m]);
        F[m] = 0.5 * (FL[m] + FR[m]) - 0.5 * diss;
    }
}

void orc_hllc(const double WL[4], const double WR[4], const double FL[4],
              const double FR[4], double gamma, double F[4])
{
    hllc_impl(WL, WR, FL, FR, gamma, 0, F);
}

void orc_hllc_ss(const double WL[4], const double WR[4], const double FL[4],
                 const double FR[4], double gamma, double F[4])
{
    hllc_impl(WL, WR, FL, FR, gamma, 1, F);
}

/* Everything the flux at one interface j+1/2 reads, gathered along the
 * normal.  Offsets are relative to cell j.                                */
typedef struct {
    double W[4][10];   /* (rho, un, ut, p) at offsets -4..5 (index m+4)     */
    double G[4][6];    /* Delta_n * d/dn of W at offsets -2..3 (index m+2)  */
    double T[2], GT[2];        /* T and Delta_n dT/dn at offsets 0, 1       */
    double dun_t[2], dut_t[2]; /* d un/dt, d ut/dt (true derivatives) at 0,1 */
    double psi[6];     /* detector at offsets -2..3                         */
    double dn;         /* normal spacing                                    */
    /* MEG7-cons only (recon = 1): conservative variables (rho, rho un,
     * rho ut, E) at offsets -4..5, their Delta_n d/dn at -2..3, and the
     * tangential derivatives d/dt of rho, rho un, rho ut at offsets 0, 1. */
    double Qc[4][10];
    double GQ[4][6];
    double GtQ[3][2];
} orc_line;

/* Characteristic projection (reading R-CHAR) of primitive vectors for the
 * normal Jacobian at mean density rb and sound speed cb.  Rows of L:
 *   (0, -rb/2cb, 0, 1/2cb^2), (1, 0, 0, -1/cb^2), (0, 0, 1, 0), (0, rb/2cb, 0, 1/2cb^2) */
static void char_fwd(const double U[4], double rb, double cb, double Wc[4])
{
    Wc[0] = -rb / (2.0 * cb) * U[1] + U[3] / (2.0 * cb * cb);
    Wc[1] = U[0] - U[3] / (cb * cb);
    Wc[2] = U[2];
    Wc[3] = rb / (2.0 * cb) * U[1] + U[3] / (2.0 * cb * cb);
}

/* Columns of R = L^{-1}: (1, -cb/rb, 0, cb^2), (1,0,0,0), (0,0,1,0), (1, cb/rb, 0, cb^2). */
static void char_bwd(const double Wc[4], double rb, double cb, double U[4])
{
    U[0] = Wc[0] + Wc[1] + Wc[3];
    U[1] = cb / rb * (Wc[3] - Wc[0]);
    U[2] = Wc[2];
    U[3] = cb * cb * (Wc[0] + Wc[3]);
}

/* Conservative variables to primitive (eq. eqn:pressure). */
static void cons_to_prim(const double Q[4], double gamma, double W[4])
{
    W[0] = Q[0];
    W[1] = Q[1] / Q[0];
    W[2] = Q[2] / Q[0];
    W[3] = (gamma - 1.0) * (Q[3] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2]) / Q[0]);
}

/* Characteristic projection for MEG7-cons (reading R-CHARC): eigenvectors of
 * the conservative normal flux Jacobian at the state with velocity (ub, vb),
 * total enthalpy hb and sound speed cb, with b1 = (gamma-1)/cb^2 and
 * b2 = b1 (ub^2 + vb^2)/2.  Rows of L:
 *   ((b2 + ub/cb)/2, -(b1 ub + 1/cb)/2, -b1 vb/2, b1/2),
 *   (1 - b2, b1 ub, b1 vb, -b1), (-vb, 0, 1, 0),
 *   ((b2 - ub/cb)/2, -(b1 ub - 1/cb)/2, -b1 vb/2, b1/2);
 * columns of R = L^{-1}: (1, ub - cb, vb, hb - ub cb), (1, ub, vb, (ub^2+vb^2)/2),
 *   (0, 0, 1, vb), (1, ub + cb, vb, hb + ub cb). */
typedef struct { double ub, vb, hb, cb, b1, b2; } orc_cstate;

void orc_char_cons_fwd(const orc_cstate *s, const double Q[4], double Wc[4])
{
    const double u = s->ub, v = s->vb, c = s->cb, b1 = s->b1, b2 = s->b2;
    Wc[0] = 0.5 * ((b2 + u / c) * Q[0] - (b1 * u + 1.0 / c) * Q[1] - b1 * v * Q[2] + b1 * Q[3]);
    Wc[1] = (1.0 - b2) * Q[0] + b1 * u * Q[1] + b1 * v * Q[2] - b1 * Q[3];
    Wc[2] = -v * Q[0] + Q[2];
    Wc[3] = 0.5 * ((b2 - u / c) * Q[0] - (b1 * u - 1.0 / c) * Q[1] - b1 * v * Q[2] + b1 * Q[3]);
}

void orc_char_cons_bwd(const orc_cstate *s, const double Wc[4], double Q[4])
{
    const double u = s->ub, v = s->vb, c = s->cb, h = s->hb;
    Q[0] = Wc[0] + Wc[1] + Wc[3];
    Q[1] = (u - c) * Wc[0] + u * Wc[1] + (u + c) * Wc[3];
    Q[2] = v * (Wc[0] + Wc[1] + Wc[3]) + Wc[2];
    Q[3] = (h - u * c) * Wc[0] + 0.5 * (u * u + v * v) * Wc[1] + v * Wc[2] + (h + u * c) * Wc[3];
}

/* The state of R-CHARC from the arithmetic mean of two conservative states. */
void orc_char_cons_state(const double Qa[4], const double Qb[4], double gamma, orc_cstate *s)
{
    double q[4], w[4];
    for (int m = 0; m < 4; ++m) q[m] = 0.5 * (Qa[m] + Qb[m]);
    cons_to_prim(q, gamma, w);
    s->ub = w[1];
    s->vb = w[2];
    s->hb = (q[3] + w[3]) / q[0];
    s->cb = sqrt(gamma * w[3] / q[0]);
    s->b1 = (gamma - 1.0) / (s->cb * s->cb);
    s->b2 = 0.5 * s->b1 * (s->ub * s->ub + s->vb * s->vb);
}

/* Mean density and sound speed of reading R-CHAR at interface j+1/2, from
 * the primitive states (rho, un, ut, p) of cells j and j+1. */
static void char_prim_state(const double Wa[4], const double Wb[4], double gamma, double *rb,
                            double *cb)
{
    *rb = 0.5 * (Wa[0] + Wb[0]);
    double pb = 0.5 * (Wa[3] + Wb[3]);
    *cb = sqrt(gamma * pb / *rb);
}

/* Interface states (rotated primitives) at j+1/2 before the Riemann solver:
 * use_mp = 0 the unlimited GRB states (Sec. 2.2), use_mp = 1 the MEG7 states
 * in characteristic variables (Sec. 2.3; R-CHAR, or R-CHARC for MEG7-cons). */
static void interface_states(const orc_line *L, const orc_cfg *c, int use_mp, double WL[4],
                             double WR[4], int *nlimited)
{
    const double gamma = c->gamma;
    if (c->recon == 1 && !use_mp) {
        /* MEG7-cons, Sec. 2.2: unlimited GRB states on conservative variables */
        double QL[4], QR[4];
        for (int m = 0; m < 4; ++m) {
            QL[m] = grb_L(c->order, &L->Qc[m][4], &L->GQ[m][2]);
            QR[m] = grb_R(c->order, &L->Qc[m][4], &L->GQ[m][2]);
        }
        cons_to_prim(QL, gamma, WL);
        cons_to_prim(QR, gamma, WR);
    } else if (c->recon == 1) {
        /* MEG7-cons, Sec. 2.3: MEG7 in conservative characteristic variables */
        double qa[4], qb[4];
        for (int m = 0; m < 4; ++m) { qa[m] = L->Qc[m][4]; qb[m] = L->Qc[m][5]; }
        orc_cstate cs;
        orc_char_cons_state(qa, qb, gamma, &cs);
        double cw[4][6], cg[4][6];
        for (int k = 0; k < 6; ++k) {
            double q[4], w[4], g[4], wg[4];
            for (int m = 0; m < 4; ++m) { q[m] = L->Qc[m][k + 2]; g[m] = L->GQ[m][k]; }
            orc_char_cons_fwd(&cs, q, w);
            orc_char_cons_fwd(&cs, g, wg);
            for (int m = 0; m < 4; ++m) { cw[m][k] = w[m]; cg[m][k] = wg[m]; }
        }
        double wl[4], wr[4], QL[4], QR[4];
        for (int m = 0; m < 4; ++m) {
            int la = 0, lb = 0;
            wl[m] = meg7_left_o(c->order, &cw[m][2], &cg[m][2], &la);
            wr[m] = meg7_right_o(c->order, &cw[m][2], &cg[m][2], &lb);
            if (nlimited) *nlimited += la + lb;
        }
        orc_char_cons_bwd(&cs, wl, QL);
        orc_char_cons_bwd(&cs, wr, QR);
        cons_to_prim(QL, gamma, WL);
        cons_to_prim(QR, gamma, WR);
    } else if (!use_mp) {
        /* Sec. 2.2: unlimited GRB states, eq. (eqn:grb), on primitives */
        for (int m = 0; m < 4; ++m) {
            WL[m] = grb_L(c->order, &L->W[m][4], &L->G[m][2]);
            WR[m] = grb_R(c->order, &L->W[m][4], &L->G[m][2]);
        }
    } else {
        /* Sec. 2.3: MEG7 in characteristic variables (R-CHAR) */
        double wa[4], wb[4], rb, cb;
        for (int m = 0; m < 4; ++m) { wa[m] = L->W[m][4]; wb[m] = L->W[m][5]; }
        char_prim_state(wa, wb, gamma, &rb, &cb);
        double cw[4][6], cg[4][6];
        for (int k = 0; k < 6; ++k) {
            double u[4], w[4], g[4], wg[4];
            for (int m = 0; m < 4; ++m) { u[m] = L->W[m][k + 2]; g[m] = L->G[m][k]; }
            char_fwd(u, rb, cb, w);
            char_fwd(g, rb, cb, wg);
            for (int m = 0; m < 4; ++m) { cw[m][k] = w[m]; cg[m][k] = wg[m]; }
        }
        double wl[4], wr[4];
        for (int m = 0; m < 4; ++m) {
            int la = 0, lb = 0;
            wl[m] = meg7_left_o(c->order, &cw[m][2], &cg[m][2], &la);
            wr[m] = meg7_right_o(c->order, &cw[m][2], &cg[m][2], &lb);
            if (nlimited) *nlimited += la + lb;
        }
        char_bwd(wl, rb, cb, WL);
        char_bwd(wr, rb, cb, WR);
    }
}

/* Flux through one interface (rotated frame). Returns sigma in *sig_out. */
static void line_flux(const orc_line *L, const orc_cfg *c, double Fout[4], int *sig_out,
                      int *nlimited, int sig_given)
{
    const double gamma = c->gamma;
    /* eq. (buffer): psi_{j+1/2} = min(psi_{j-2..j+3}); sigma = 0 iff < psi_c */
    double pmin = L->psi[0];
    for (int k = 1; k < 6; ++k) pmin = fmin(pmin, L->psi[k]);
    int sigma = (pmin < PSI_C) ? 0 : 1;
    if (c->force_sigma == 0 || c->force_sigma == 1) sigma = c->force_sigma;
    if (sig_given == 0 || sig_given == 1) sigma = sig_given;
    *sig_out = sigma;

    double WL[4], WR[4], FL[4], FR[4];
    int use_mp = (sigma == 0) || (c->mp_mode == 1);
    interface_states(L, c, use_mp, WL, WR, nlimited);
    if (sigma == 1) {
        /* eqs. (flux-full), (flux-right) on f = F^c(U) at cell centres */
        double f[4][10];
        for (int k = 0; k < 10; ++k) {
            double w[4], ff[4];
            for (int m = 0; m < 4; ++m) w[m] = L->W[m][k];
            conv_flux(w, gamma, ff);
            for (int m = 0; m < 4; ++m) f[m][k] = ff[m];
        }
        for (int m = 0; m < 4; ++m) {
            FL[m] = flux_L(c->order, &f[m][4]);
            FR[m] = flux_R(c->order, &f[m][4]);
        }
    } else {
        conv_flux(WL, gamma, FL);   /* F(Q_L) */
        conv_flux(WR, gamma, FR);   /* F(Q_R) */
    }
    /* reading R-POS: first-order states where the reconstruction is unphysical */
    if (!(WL[0] > 0.0 && WL[3] > 0.0 && WR[0] > 0.0 && WR[3] > 0.0)) {
        for (int m = 0; m < 4; ++m) { WL[m] = L->W[m][4]; WR[m] = L->W[m][5]; }
        conv_flux(WL, gamma, FL);
        conv_flux(WR, gamma, FR);
    }
    double Fc[4];
    hllc_impl(WL, WR, FL, FR, gamma, c->riemann, Fc);

    /* Sec. 2.1 viscous flux (R-VISC). */
    double Fv[4] = {0.0, 0.0, 0.0, 0.0};
    if (c->mu > 0.0) {
        const double mu = c->mu, dn = L->dn;
        /* eq. (eqn:alphad) with Phi' = dn dPhi/dn:
         * dn*(dPhi/dn)_{j+1/2} = (Phi'_j + Phi'_{j+1})/2
         *                        + alpha_v/2 (Phi_{j+1} - Phi'_{j+1}/2 - Phi_j - Phi'_j/2) */
        double un0 = L->W[1][4], un1 = L->W[1][5];
        double ut0 = L->W[2][4], ut1 = L->W[2][5];
        double gun0 = L->G[1][2], gun1 = L->G[1][3];
        double gut0 = L->G[2][2], gut1 = L->G[2][3];
        double dunt0 = L->dun_t[0], dunt1 = L->dun_t[1];
        double dutt0 = L->dut_t[0], dutt1 = L->dut_t[1];
        if (c->recon == 1) {
            /* MEG7-cons: velocity gradients by the chain rule of Sec. 2.2,
             * d u = (d(rho u) - u d rho) / rho, from the conservative ones */
            const double r0 = L->W[0][4], r1 = L->W[0][5];
            gun0 = (L->GQ[1][2] - un0 * L->GQ[0][2]) / r0;
            gun1 = (L->GQ[1][3] - un1 * L->GQ[0][3]) / r1;
            gut0 = (L->GQ[2][2] - ut0 * L->GQ[0][2]) / r0;
            gut1 = (L->GQ[2][3] - ut1 * L->GQ[0][3]) / r1;
            dunt0 = (L->GtQ[1][0] - un0 * L->GtQ[0][0]) / r0;
            dunt1 = (L->GtQ[1][1] - un1 * L->GtQ[0][1]) / r1;
            dutt0 = (L->GtQ[2][0] - ut0 * L->GtQ[0][0]) / r0;
            dutt1 = (L->GtQ[2][1] - ut1 * L->GtQ[0][1]) / r1;
        }
        double dun_n = (0.5 * (gun0 + gun1)
                        + 0.5 * ALPHA_V * (un1 - 0.5 * gun1 - un0 - 0.5 * gun0)) / dn;
        double dut_n = (0.5 * (gut0 + gut1)
                        + 0.5 * ALPHA_V * (ut1 - 0.5 * gut1 - ut0 - 0.5 * gut0)) / dn;
        double dT_n = (0.5 * (L->GT[0] + L->GT[1])
                       + 0.5 * ALPHA_V * (L->T[1] - 0.5 * L->GT[1] - L->T[0] - 0.5 * L->GT[0])) / dn;
        double dun_t = 0.5 * (dunt0 + dunt1);
        double dut_t = 0.5 * (dutt0 + dutt1);
        double unf = 0.5 * (un0 + un1), utf = 0.5 * (ut0 + ut1);
        /* eq. (eqn:visc) in the normal frame */
        double tnn = 2.0 / 3.0 * mu * (2.0 * dun_n - dut_t);
        double tnt = mu * (dut_n + dun_t);
        double qn = -mu / (c->Pr * (gamma - 1.0)) * dT_n;
        Fv[1] = -tnn;
        Fv[2] = -tnt;
        Fv[3] = -(tnn * unf + tnt * utf) + qn;
    }
    for (int m = 0; m < 4; ++m) Fout[m] = Fc[m] + Fv[m];
}

/* ---------------------------------------------------------------------- */
/* Grid-level residual.                                                    */
/* ---------------------------------------------------------------------- */
static int bc_index(int k, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        k %= n;
        if (k < 0) k += n;
        return k;
    }
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

/* Reading R-WALL.  For raw index k along an axis (0: x, 1: y), the kind of
 * the side that governs it (-1 inside the grid), that side's fixed state,
 * and the source index: wrap (periodic), mirror about the wall (reflect,
 * no-slip; clamped into the grid where the overhang exceeds the grid), or
 * the nearest cell (transmissive, inflow).  tang is the cell-centre
 * coordinate along the side, tb the boundary time. */
static int side_rule(const orc_cfg *c, int axis, int k, double tang, double tb,
                     const double **state)
{
    const int n = axis == 0 ? c->nx : c->ny;
    *state = NULL;
    if (k >= 0 && k < n) return -1;
    int kind;
    if (!c->use_sides) {
        kind = axis == 0 ? c->bc_x : c->bc_y;
    } else {
        const orc_side *S = &c->side[2 * axis + (k >= n ? 1 : 0)];
        const int seg = (tang < S->split0 + S->split_speed * tb) ? 0 : 1;
        kind = S->kind[seg];
        *state = S->state[seg];
    }
    return kind;
}

static int source_index(int kind, int k, int n)
{
    if (kind < 0) return k;
    if (kind == ORC_BC_PERIODIC) return bc_index(k, n, ORC_BC_PERIODIC);
    if (kind == ORC_BC_REFLECT || kind == ORC_BC_NOSLIP) {
        int m = k < 0 ? -1 - k : 2 * n - 1 - k;
        return m < 0 ? 0 : (m >= n ? n - 1 : m);
    }
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

/* Primitive and conservative values of (possibly ghost) cell (i, j) at
 * boundary time tb (reading R-WALL). */
static void cell_values(const orc_cfg *c, const double *Q, int i, int j, double tb,
                        double W[4], double Cc[4])
{
    const int nx = c->nx, ny = c->ny;
    const size_t n = (size_t)nx * ny;
    const double dx = (c->x1 - c->x0) / nx, dy = (c->y1 - c->y0) / ny;
    const double xc = c->x0 + ((double)j + 0.5) * dx;
    const double yc = c->y0 + ((double)i + 0.5) * dy;
    const double *sx, *sy;
    const int kx = side_rule(c, 0, j, yc, tb, &sx);
    const int ky = side_rule(c, 1, i, xc, tb, &sy);
    const size_t s = (size_t)source_index(ky, i, ny) * nx + source_index(kx, j, nx);
    double rho = Q[s], mx = Q[n + s], my = Q[2 * n + s], E = Q[3 * n + s];
    /* mirror rules: a reflecting wall negates the normal momentum, a no-slip
     * wall both components; the rules of the two sides of a corner compose */
    if (kx == ORC_BC_REFLECT || kx == ORC_BC_NOSLIP) mx = -mx;
    if (kx == ORC_BC_NOSLIP) my = -my;
    if (ky == ORC_BC_REFLECT || ky == ORC_BC_NOSLIP) my = -my;
    if (ky == ORC_BC_NOSLIP) mx = -mx;
    double u = mx / rho, v = my / rho;
    double p = (c->gamma - 1.0) * (E - rho * (u * u + v * v) / 2.0);
    W[0] = rho; W[1] = u; W[2] = v; W[3] = p;
    Cc[0] = rho; Cc[1] = mx; Cc[2] = my; Cc[3] = E;
    const double *fixed = kx == ORC_BC_INFLOW ? sx : (ky == ORC_BC_INFLOW ? sy : NULL);
    if (fixed) {
        for (int m = 0; m < 4; ++m) W[m] = fixed[m];
        prim_to_cons(W, c->gamma, Cc);
    }
}

typedef struct {
    int NX, NY;                 /* padded sizes */
    double *W[4];               /* rho, u, v, p on the padded grid */
    double *T;
    double *Gx[5], *Gy[5];      /* Delta x d/dx, Delta y d/dy of rho,u,v,p,T */
    double *psix, *psiy;
    double *C[4];               /* rho, rho u, rho v, E (recon = 1 only) */
    double *GCx[4], *GCy[4];    /* their Delta x d/dx, Delta y d/dy       */
} orc_fields;

static void fields_free(orc_fields *F)
{
    for (int m = 0; m < 4; ++m) free(F->W[m]);
    free(F->T);
    for (int m = 0; m < 5; ++m) { free(F->Gx[m]); free(F->Gy[m]); }
    free(F->psix); free(F->psiy);
    for (int m = 0; m < 4; ++m) { free(F->C[m]); free(F->GCx[m]); free(F->GCy[m]); }
}

static int fields_build(const orc_cfg *c, const double *Q, orc_fields *F)
{
    const int nx = c->nx, ny = c->ny;
    const int NX = nx + 2 * NG, NY = ny + 2 * NG;
    const size_t np = (size_t)NX * NY;
    memset(F, 0, sizeof(*F));
    F->NX = NX; F->NY = NY;
    for (int m = 0; m < 4; ++m) F->W[m] = (double *)calloc(np, sizeof(double));
    F->T = (double *)calloc(np, sizeof(double));
    for (int m = 0; m < 5; ++m) {
        F->Gx[m] = (double *)calloc(np, sizeof(double));
        F->Gy[m] = (double *)calloc(np, sizeof(double));
    }
    F->psix = (double *)calloc(np, sizeof(double));
    F->psiy = (double *)calloc(np, sizeof(double));
    for (int m = 0; m < 4; ++m) if (!F->W[m]) return -1;
    if (!F->T || !F->psix || !F->psiy) return -1;
    for (int m = 0; m < 5; ++m) if (!F->Gx[m] || !F->Gy[m]) return -1;
    if (c->recon == 1) {
        for (int m = 0; m < 4; ++m) {
            F->C[m] = (double *)calloc(np, sizeof(double));
            F->GCx[m] = (double *)calloc(np, sizeof(double));
            F->GCy[m] = (double *)calloc(np, sizeof(double));
            if (!F->C[m] || !F->GCx[m] || !F->GCy[m]) return -1;
        }
    }

    const double gamma = c->gamma;
    /* ghost cells (R-BC) and primitives, eq. (eqn:pressure), T (R-T) */
#pragma omp parallel for schedule(static)
    for (int I = 0; I < NY; ++I) {
        for (int J = 0; J < NX; ++J) {
            double W[4], Cc[4];
            cell_values(c, Q, I - NG, J - NG, c->t, W, Cc);
            size_t P = (size_t)I * NX + J;
            for (int m = 0; m < 4; ++m) F->W[m][P] = W[m];
            F->T[P] = gamma * W[3] / W[0];
            if (c->recon == 1)
                for (int m = 0; m < 4; ++m) F->C[m][P] = Cc[m];
        }
    }
    double *src[5] = {F->W[0], F->W[1], F->W[2], F->W[3], F->T};
    /* eq. (eqn:six): gradients, computed once and shared */
#pragma omp parallel for schedule(static)
    for (int I = 0; I < NY; ++I) {
        for (int J = 0; J < NX; ++J) {
            size_t P = (size_t)I * NX + J;
            for (int m = 0; m < 5; ++m) {
                double px[7], py[7];
                int okx = (J >= 3 && J < NX - 3), oky = (I >= 3 && I < NY - 3);
                for (int k = -3; k <= 3; ++k) {
                    px[k + 3] = okx ? src[m][P + k] : 0.0;
                    py[k + 3] = oky ? src[m][P + (ptrdiff_t)k * NX] : 0.0;
                }
                F->Gx[m][P] = okx ? orc_grad6(px) : 0.0;
                F->Gy[m][P] = oky ? orc_grad6(py) : 0.0;
            }
            if (c->recon == 1) {
                int okx = (J >= 3 && J < NX - 3), oky = (I >= 3 && I < NY - 3);
                for (int m = 0; m < 4; ++m) {
                    double px[7], py[7];
                    for (int k = -3; k <= 3; ++k) {
                        px[k + 3] = okx ? F->C[m][P + k] : 0.0;
                        py[k + 3] = oky ? F->C[m][P + (ptrdiff_t)k * NX] : 0.0;
                    }
                    F->GCx[m][P] = okx ? orc_grad6(px) : 0.0;
                    F->GCy[m][P] = oky ? orc_grad6(py) : 0.0;
                }
            }
            /* detector on density, one per direction */
            const double *r = F->W[0];
            F->psix[P] = (J >= 2 && J < NX - 2)
                ? orc_psi(r[P - 2], r[P - 1], r[P], r[P + 1], r[P + 2]) : 1.0;
            F->psiy[P] = (I >= 2 && I < NY - 2)
                ? orc_psi(r[P - 2 * NX], r[P - NX], r[P], r[P + NX], r[P + 2 * NX]) : 1.0;
        }
    }
    return 0;
}

/* Gather the line for x-interface (j+1/2, i), j in [-1, nx-1]. */
static void gather_x(const orc_cfg *c, const orc_fields *F, int i, int j, orc_line *L)
{
    const int NX = F->NX;
    size_t P0 = (size_t)(i + NG) * NX + (j + NG);
    const int perm[4] = {0, 1, 2, 3}; /* (rho, u, v, p) -> (rho, un=u, ut=v, p) */
    for (int m = 0; m < 4; ++m) {
        for (int k = -4; k <= 5; ++k) L->W[m][k + 4] = F->W[perm[m]][P0 + k];
        for (int k = -2; k <= 3; ++k) L->G[m][k + 2] = F->Gx[perm[m]][P0 + k];
    }
    for (int k = 0; k < 2; ++k) {
        L->T[k] = F->T[P0 + k];
        L->GT[k] = F->Gx[4][P0 + k];
        L->dun_t[k] = F->Gy[1][P0 + k] / ((c->y1 - c->y0) / c->ny);
        L->dut_t[k] = F->Gy[2][P0 + k] / ((c->y1 - c->y0) / c->ny);
    }
    for (int k = -2; k <= 3; ++k) L->psi[k + 2] = F->psix[P0 + k];
    L->dn = (c->x1 - c->x0) / c->nx;
    if (c->recon == 1) {
        const double dt = (c->y1 - c->y0) / c->ny;
        for (int m = 0; m < 4; ++m) {
            for (int k = -4; k <= 5; ++k) L->Qc[m][k + 4] = F->C[perm[m]][P0 + k];
            for (int k = -2; k <= 3; ++k) L->GQ[m][k + 2] = F->GCx[perm[m]][P0 + k];
        }
        for (int k = 0; k < 2; ++k)
            for (int m = 0; m < 3; ++m) L->GtQ[m][k] = F->GCy[perm[m]][P0 + k] / dt;
    }
}

/* Gather the line for y-interface (j, i+1/2), i in [-1, ny-1]. */
static void gather_y(const orc_cfg *c, const orc_fields *F, int i, int j, orc_line *L)
{
    const int NX = F->NX;
    size_t P0 = (size_t)(i + NG) * NX + (j + NG);
    const int perm[4] = {0, 2, 1, 3}; /* (rho, u, v, p) -> (rho, un=v, ut=u, p) */
    for (int m = 0; m < 4; ++m) {
        for (int k = -4; k <= 5; ++k) L->W[m][k + 4] = F->W[perm[m]][P0 + (ptrdiff_t)k * NX];
        for (int k = -2; k <= 3; ++k) L->G[m][k + 2] = F->Gy[perm[m]][P0 + (ptrdiff_t)k * NX];
    }
    for (int k = 0; k < 2; ++k) {
        L->T[k] = F->T[P0 + (size_t)k * NX];
        L->GT[k] = F->Gy[4][P0 + (size_t)k * NX];
        L->dun_t[k] = F->Gx[2][P0 + (size_t)k * NX] / ((c->x1 - c->x0) / c->nx);
        L->dut_t[k] = F->Gx[1][P0 + (size_t)k * NX] / ((c->x1 - c->x0) / c->nx);
    }
    for (int k = -2; k <= 3; ++k) L->psi[k + 2] = F->psiy[P0 + (ptrdiff_t)k * NX];
    L->dn = (c->y1 - c->y0) / c->ny;
    if (c->recon == 1) {
        const double dt = (c->x1 - c->x0) / c->nx;
        for (int m = 0; m < 4; ++m) {
            for (int k = -4; k <= 5; ++k) L->Qc[m][k + 4] = F->C[perm[m]][P0 + (ptrdiff_t)k * NX];
            for (int k = -2; k <= 3; ++k) L->GQ[m][k + 2] = F->GCy[perm[m]][P0 + (ptrdiff_t)k * NX];
        }
        for (int k = 0; k < 2; ++k)
            for (int m = 0; m < 3; ++m) L->GtQ[m][k] = F->GCx[perm[m]][P0 + (size_t)k * NX] / dt;
    }
}

static int sides_ok(const orc_cfg *c)
{
    if (!c->use_sides) return 1;
    for (int a = 0; a < 2; ++a) {
        int nper = 0;
        for (int sd = 2 * a; sd < 2 * a + 2; ++sd)
            for (int g = 0; g < 2; ++g) {
                const int k = c->side[sd].kind[g];
                if (k < ORC_BC_PERIODIC || k > ORC_BC_INFLOW) return 0;
                nper += (k == ORC_BC_PERIODIC);
            }
        if (nper != 0 && nper != 4) return 0;   /* periodic: all of both sides of an axis */
    }
    return 1;
}

static int cfg_ok(const orc_cfg *c)
{
    return c && c->nx >= 2 * NG && c->ny >= 2 * NG && c->gamma > 1.0 && c->mu >= 0.0
        && c->Pr > 0.0 && c->x1 > c->x0 && c->y1 > c->y0 && (c->recon == 0 || c->recon == 1)
        && (c->order == 7 || c->order == 4) && (c->riemann == 0 || c->riemann == 1)
        && sides_ok(c);
}

/* eqs. (eqn-differencing_residual), (deriv): Res = -dF/dx - dG/dy.
 * Q, Res: SoA [4][ny][nx], x fastest.  sig_x: [ny][nx+1] (interface j+1/2 at
 * column j+1), sig_y: [ny+1][nx] (interface i+1/2 at row i+1); may be NULL.
 * Returns the number of MP-limited components (diagnostic) or -1. */
static long residual_impl(const orc_cfg *c, const double *Q, double *Res, uint8_t *sig_x,
                          uint8_t *sig_y, const uint8_t *gx, const uint8_t *gy)
{
    if (!cfg_ok(c)) return -1;
    const int nx = c->nx, ny = c->ny;
    const size_t n = (size_t)nx * ny;
    orc_fields F;
    if (fields_build(c, Q, &F) != 0) { fields_free(&F); return -1; }
    double *Fx = (double *)malloc(sizeof(double) * 4 * (size_t)ny * (nx + 1));
    double *Fy = (double *)malloc(sizeof(double) * 4 * (size_t)(ny + 1) * nx);
    if (!Fx || !Fy) { free(Fx); free(Fy); fields_free(&F); return -1; }
    const size_t nfx = (size_t)ny * (nx + 1), nfy = (size_t)(ny + 1) * nx;
    long nlim = 0;

#pragma omp parallel for schedule(static) reduction(+ : nlim)
    for (int i = 0; i < ny; ++i) {
        for (int j = -1; j < nx; ++j) {
            orc_line L; double f[4]; int sg; int nl = 0;
            gather_x(c, &F, i, j, &L);
            line_flux(&L, c, f, &sg, &nl, gx ? gx[(size_t)i * (nx + 1) + (j + 1)] : -1);
            nlim += nl;
            size_t s = (size_t)i * (nx + 1) + (j + 1);
            for (int m = 0; m < 4; ++m) Fx[m * nfx + s] = f[m];
            if (sig_x) sig_x[s] = (uint8_t)sg;
        }
    }
#pragma omp parallel for schedule(static) reduction(+ : nlim)
    for (int i = -1; i < ny; ++i) {
        for (int j = 0; j < nx; ++j) {
            orc_line L; double f[4]; int sg; int nl = 0;
            gather_y(c, &F, i, j, &L);
            line_flux(&L, c, f, &sg, &nl, gy ? gy[(size_t)(i + 1) * nx + j] : -1);
            nlim += nl;
            size_t s = (size_t)(i + 1) * nx + j;
            /* rotate back: (rho, rho v, rho u, E) -> (rho, rho u, rho v, E) */
            Fy[0 * nfy + s] = f[0];
            Fy[1 * nfy + s] = f[2];
            Fy[2 * nfy + s] = f[1];
            Fy[3 * nfy + s] = f[3];
            if (sig_y) sig_y[s] = (uint8_t)sg;
        }
    }
    const double dx = (c->x1 - c->x0) / nx, dy = (c->y1 - c->y0) / ny;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < ny; ++i) {
        for (int j = 0; j < nx; ++j) {
            size_t s = (size_t)i * nx + j;
            for (int m = 0; m < 4; ++m) {
                double dFdx = (Fx[m * nfx + (size_t)i * (nx + 1) + j + 1]
                               - Fx[m * nfx + (size_t)i * (nx + 1) + j]) / dx;
                double dGdy = (Fy[m * nfy + (size_t)(i + 1) * nx + j]
                               - Fy[m * nfy + (size_t)i * nx + j]) / dy;
                Res[m * n + s] = -dFdx - dGdy;
            }
        }
    }
    free(Fx); free(Fy);
    fields_free(&F);
    return nlim;
}

long orc_residual(const orc_cfg *c, const double *Q, double *Res, uint8_t *sig_x,
                  uint8_t *sig_y)
{
    return residual_impl(c, Q, Res, sig_x, sig_y, NULL, NULL);
}

/* The residual with the interface flags sigma given ([ny][nx+1] and
 * [ny+1][nx], layouts as above) instead of taken from the density detector:
 * the hybrid flux of Sec. 2.4 with any detector in place of eq. (buffer). */
long orc_residual_sigma(const orc_cfg *c, const double *Q, double *Res, const uint8_t *sig_x,
                        const uint8_t *sig_y)
{
    if (!sig_x || !sig_y) return -1;
    return residual_impl(c, Q, Res, NULL, NULL, sig_x, sig_y);
}

/* eq. (rk): one stage of the third-order TVD Runge-Kutta scheme.
 * stage 1: Qout = Qn + dt R(Qn)            (Qk must equal Qn)
 * stage 2: Qout = 3/4 Qn + 1/4 Qk + 1/4 dt R(Qk)
 * stage 3: Qout = 1/3 Qn + 2/3 Qk + 2/3 dt R(Qk)                          */
long orc_rk_stage(const orc_cfg *c, int stage, double dt, const double *Qn,
                  const double *Qk, double *Qout, uint8_t *sig_x, uint8_t *sig_y)
{
    if (!cfg_ok(c) || stage < 1 || stage > 3) return -1;
    const size_t N = 4 * (size_t)c->nx * c->ny;
    double *R = (double *)malloc(sizeof(double) * N);
    if (!R) return -1;
    /* reading R-WALL: the boundary of stage k at t + c_k dt, c = (0, 1, 1/2) */
    const double ck[3] = {0.0, 1.0, 0.5};
    orc_cfg cs = *c;
    cs.t = c->t + ck[stage - 1] * dt;
    long nl = orc_residual(&cs, Qk, R, sig_x, sig_y);
    if (nl < 0) { free(R); return -1; }
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < N; ++s) {
        if (stage == 1)
            Qout[s] = Qn[s] + dt * R[s];
        else if (stage == 2)
            Qout[s] = 3.0 / 4.0 * Qn[s] + 1.0 / 4.0 * Qk[s] + 1.0 / 4.0 * dt * R[s];
        else
            Qout[s] = 1.0 / 3.0 * Qn[s] + 2.0 / 3.0 * Qk[s] + 2.0 / 3.0 * dt * R[s];
    }
    free(R);
    return nl;
}

/* Sec. 2.5 time step:
 * dt = CFL min( (1/alpha_v) min(dx^2/nu, dy^2/nu), min(dx/(|u|+c), dy/(|v|+c)) ) */
double orc_dt(const orc_cfg *c, const double *Q, double cfl)
{
    if (!cfg_ok(c)) return -1.0;
    const int nx = c->nx, ny = c->ny;
    const size_t n = (size_t)nx * ny;
    const double dx = (c->x1 - c->x0) / nx, dy = (c->y1 - c->y0) / ny;
    const double gamma = c->gamma;
    double conv = INFINITY, visc = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : conv, visc)
    for (size_t s = 0; s < n; ++s) {
        double rho = Q[s], u = Q[n + s] / rho, v = Q[2 * n + s] / rho;
        double p = (gamma - 1.0) * (Q[3 * n + s] - rho * (u * u + v * v) / 2.0);
        double cs = sqrt(gamma * p / rho);
        conv = fmin(conv, fmin(dx / (fabs(u) + cs), dy / (fabs(v) + cs)));
        if (c->mu > 0.0) {
            double nu = c->mu / rho;
            visc = fmin(visc, fmin(dx * dx / nu, dy * dy / nu));
        }
    }
    return cfl * fmin(visc / ALPHA_V, conv);
}

/* One full SSP-RK3 step with dt from Qn (for trajectories in tests):
 * Q is advanced in place and c->t by dt; returns dt. */
double orc_step(orc_cfg *c, double *Q, double cfl)
{
    const size_t N = 4 * (size_t)c->nx * c->ny;
    double dt = orc_dt(c, Q, cfl);
    double *Q1 = (double *)malloc(sizeof(double) * N);
    double *Q2 = (double *)malloc(sizeof(double) * N);
    if (!Q1 || !Q2 || dt <= 0.0) { free(Q1); free(Q2); return -1.0; }
    orc_rk_stage(c, 1, dt, Q, Q, Q1, NULL, NULL);
    orc_rk_stage(c, 2, dt, Q, Q1, Q2, NULL, NULL);
    orc_rk_stage(c, 3, dt, Q, Q2, Q1, NULL, NULL);
    memcpy(Q, Q1, sizeof(double) * N);
    free(Q1); free(Q2);
    c->t += dt;
    return dt;
}

/* Per-interface flux evaluation for unit tests: W/G arrays as in orc_line. */
void orc_line_flux(const double *W40, const double *G24, const double *T2, const double *GT2,
                   const double *dun_t2, const double *dut_t2, const double *psi6,
                   double dn, const orc_cfg *c, double F[4], int *sigma)
{
    orc_line L;
    memset(&L, 0, sizeof(L));   /* primitive reconstruction only (recon = 0) */
    for (int m = 0; m < 4; ++m) {
        for (int k = 0; k < 10; ++k) L.W[m][k] = W40[m * 10 + k];
        for (int k = 0; k < 6; ++k) L.G[m][k] = G24[m * 6 + k];
    }
    for (int k = 0; k < 2; ++k) {
        L.T[k] = T2[k]; L.GT[k] = GT2[k]; L.dun_t[k] = dun_t2[k]; L.dut_t[k] = dut_t2[k];
    }
    for (int k = 0; k < 6; ++k) L.psi[k] = psi6[k];
    L.dn = dn;
    line_flux(&L, c, F, sigma, NULL, -1);
}

/* Test export: the interface states line_flux hands to the Riemann solver
 * for sigma = 0 (MEG7 characteristic states) or sigma = 1 (GRB states), from
 * W/G arrays as in orc_line (primitive reconstruction), before the
 * positivity fallback of R-POS. */
void orc_interface_states(const double *W40, const double *G24, const orc_cfg *c, int sigma,
                          double WL[4], double WR[4])
{
    orc_line L;
    memset(&L, 0, sizeof(L));
    for (int m = 0; m < 4; ++m) {
        for (int k = 0; k < 10; ++k) L.W[m][k] = W40[m * 10 + k];
        for (int k = 0; k < 6; ++k) L.G[m][k] = G24[m * 6 + k];
    }
    interface_states(&L, c, sigma == 0 || c->mp_mode == 1, WL, WR, NULL);
}

/* Test export: the characteristic projection of R-CHAR at the interface
 * between the rotated primitive states Wa, Wb, as 4x4 matrices (row-major):
 * Lm maps primitives to characteristic variables, Rm back. */
void orc_char_prim(const double Wa[4], const double Wb[4], double gamma, double Lm[16],
                   double Rm[16])
{
    double rb, cb;
    char_prim_state(Wa, Wb, gamma, &rb, &cb);
    for (int k = 0; k < 4; ++k) {
        double e[4] = {0.0, 0.0, 0.0, 0.0}, o[4];
        e[k] = 1.0;
        char_fwd(e, rb, cb, o);
        for (int m = 0; m < 4; ++m) Lm[m * 4 + k] = o[m];
        char_bwd(e, rb, cb, o);
        for (int m = 0; m < 4; ++m) Rm[m * 4 + k] = o[m];
    }
}

/* Plain detector flags chi = [psi_x < psi_c or psi_y < psi_c] per cell
 * (the per-cell label the learned detector is trained on), psi_x/psi_y
 * exported too (any pointer may be NULL). */
int orc_cell_flags(const orc_cfg *c, const double *Q, uint8_t *chi, double *psix,
                   double *psiy)
{
    if (!cfg_ok(c)) return -1;
    orc_fields F;
    if (fields_build(c, Q, &F) != 0) { fields_free(&F); return -1; }
    const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            size_t P = (size_t)(i + NG) * F.NX + (j + NG);
            size_t s = (size_t)i * nx + j;
            if (psix) psix[s] = F.psix[P];
            if (psiy) psiy[s] = F.psiy[P];
            if (chi) chi[s] = (uint8_t)((F.psix[P] < PSI_C) || (F.psiy[P] < PSI_C));
        }
    fields_free(&F);
    return 0;
}

/* ====================================================================== */
/* Three dimensions (the paper's 3D Taylor-Green comparison): the Euler     */
/* equations with conservative variables (rho, rho u, rho v, rho w, E),     */
/* discretised dimension by dimension exactly as in 2D.  Reading R-3D: the  */
/* rotated frame of direction d holds (rho, u_n, u_t1, u_t2, p) with the    */
/* tangential components taken cyclically (x: v, w; y: w, u; z: u, v); the  */
/* characteristic projection adds the identity row of the second           */
/* tangential velocity to R-CHAR; HLLC (R-HLLC) carries both tangential     */
/* momenta.  Inviscid only.                                                 */
/* ====================================================================== */

typedef struct {
    int nx, ny, nz;
    double x0, x1, y0, y1, z0, z1;
    int bc[3];
    double gamma;
    int order;
} orc3_cfg;

static int cfg3_ok(const orc3_cfg *c)
{
    return c && c->nx >= 2 * NG && c->ny >= 2 * NG && c->nz >= 2 * NG && c->gamma > 1.0
        && c->x1 > c->x0 && c->y1 > c->y0 && c->z1 > c->z0
        && (c->order == 7 || c->order == 4)
        && c->bc[0] >= 0 && c->bc[0] <= 1 && c->bc[1] >= 0 && c->bc[1] <= 1
        && c->bc[2] >= 0 && c->bc[2] <= 1;
}

/* eq. (eqn:pressure) inverted, 3D rotated frame. */
static void prim_to_cons3(const double W[5], double gamma, double Q[5])
{
    Q[0] = W[0];
    Q[1] = W[0] * W[1];
    Q[2] = W[0] * W[2];
    Q[3] = W[0] * W[3];
    Q[4] = W[4] / (gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

/* The convective flux along the normal. */
static void conv_flux3(const double W[5], double gamma, double F[5])
{
    double Q[5];
    prim_to_cons3(W, gamma, Q);
    F[0] = W[0] * W[1];
    F[1] = W[0] * W[1] * W[1] + W[4];
    F[2] = W[0] * W[1] * W[2];
    F[3] = W[0] * W[1] * W[3];
    F[4] = W[1] * (Q[4] + W[4]);
}

/* HLLC, reading R-HLLC, in 3D. */
static void hllc3(const double WL[5], const double WR[5], const double FL[5],
                  const double FR[5], double gamma, double F[5])
{
    double QL[5], QR[5];
    prim_to_cons3(WL, gamma, QL);
    prim_to_cons3(WR, gamma, QR);
    double rl = WL[0], ul = WL[1], pl = WL[4];
    double rr = WR[0], ur = WR[1], pr = WR[4];
    double cl = sqrt(gamma * pl / rl);
    double cr = sqrt(gamma * pr / rr);
    double hl = (QL[4] + pl) / rl;
    double hr = (QR[4] + pr) / rr;
    double sl_ = sqrt(rl), sr_ = sqrt(rr);
    double ut = (sl_ * ul + sr_ * ur) / (sl_ + sr_);
    double vt = (sl_ * WL[2] + sr_ * WR[2]) / (sl_ + sr_);
    double wt = (sl_ * WL[3] + sr_ * WR[3]) / (sl_ + sr_);
    double ht = (sl_ * hl + sr_ * hr) / (sl_ + sr_);
    double ct = sqrt((gamma - 1.0) * (ht - 0.5 * (ut * ut + vt * vt + wt * wt)));
    double SL = fmin(ul - cl, ut - ct);
    double SR = fmax(ur + cr, ut + ct);
    double Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur))
              / (rl * (SL - ul) - rr * (SR - ur));
    double QsL[5], QsR[5];
    double kl = rl * (SL - ul) / (SL - Ss);
    QsL[0] = kl;
    QsL[1] = kl * Ss;
    QsL[2] = kl * WL[2];
    QsL[3] = kl * WL[3];
    QsL[4] = kl * (QL[4] / rl + (Ss - ul) * (Ss + pl / (rl * (SL - ul))));
    double kr = rr * (SR - ur) / (SR - Ss);
    QsR[0] = kr;
    QsR[1] = kr * Ss;
    QsR[2] = kr * WR[2];
    QsR[3] = kr * WR[3];
    QsR[4] = kr * (QR[4] / rr + (Ss - ur) * (Ss + pr / (rr * (SR - ur))));
    for (int m = 0; m < 5; ++m) {
        double diss = fabs(SL) * (QsL[m] - QL[m]) + fabs(Ss) * (QsR[m] - QsL[m])
                    + fabs(SR) * (QR[m] - QsR[m]);
        F[m] = 0.5 * (FL[m] + FR[m]) - 0.5 * diss;
    }
}

/* R-CHAR with the second tangential velocity (row and column of identity). */
static void char_fwd3(const double U[5], double rb, double cb, double Wc[5])
{
    Wc[0] = -rb / (2.0 * cb) * U[1] + U[4] / (2.0 * cb * cb);
    Wc[1] = U[0] - U[4] / (cb * cb);
    Wc[2] = U[2];
    Wc[3] = U[3];
    Wc[4] = rb / (2.0 * cb) * U[1] + U[4] / (2.0 * cb * cb);
}

static void char_bwd3(const double Wc[5], double rb, double cb, double U[5])
{
    U[0] = Wc[0] + Wc[1] + Wc[4];
    U[1] = cb / rb * (Wc[4] - Wc[0]);
    U[2] = Wc[2];
    U[3] = Wc[3];
    U[4] = cb * cb * (Wc[0] + Wc[4]);
}

/* Everything the flux at one interface j+1/2 reads along its normal. */
typedef struct {
    double W[5][10];   /* (rho, un, ut1, ut2, p) at offsets -4..5 */
    double G[5][6];    /* their Delta_n d/dn at offsets -2..3      */
    double psi[6];     /* detector at offsets -2..3               */
} orc3_line;

static void line_flux3(const orc3_line *L, const orc3_cfg *c, double Fout[5], int *sig_out)
{
    const double gamma = c->gamma;
    double pmin = L->psi[0];
    for (int k = 1; k < 6; ++k) pmin = fmin(pmin, L->psi[k]);
    const int sigma = (pmin < PSI_C) ? 0 : 1;       /* eq. (buffer) */
    *sig_out = sigma;
    double WL[5], WR[5], FL[5], FR[5];
    if (sigma) {
        for (int m = 0; m < 5; ++m) {
            WL[m] = grb_L(c->order, &L->W[m][4], &L->G[m][2]);
            WR[m] = grb_R(c->order, &L->W[m][4], &L->G[m][2]);
        }
        double f[5][10];
        for (int k = 0; k < 10; ++k) {
            double w[5], ff[5];
            for (int m = 0; m < 5; ++m) w[m] = L->W[m][k];
            conv_flux3(w, gamma, ff);
            for (int m = 0; m < 5; ++m) f[m][k] = ff[m];
        }
        for (int m = 0; m < 5; ++m) {
            FL[m] = flux_L(c->order, &f[m][4]);
            FR[m] = flux_R(c->order, &f[m][4]);
        }
    } else {
        double rb = 0.5 * (L->W[0][4] + L->W[0][5]);
        double pb = 0.5 * (L->W[4][4] + L->W[4][5]);
        double cb = sqrt(gamma * pb / rb);
        double cw[5][6], cg[5][6];
        for (int k = 0; k < 6; ++k) {
            double u[5], w[5], g[5], wg[5];
            for (int m = 0; m < 5; ++m) { u[m] = L->W[m][k + 2]; g[m] = L->G[m][k]; }
            char_fwd3(u, rb, cb, w);
            char_fwd3(g, rb, cb, wg);
            for (int m = 0; m < 5; ++m) { cw[m][k] = w[m]; cg[m][k] = wg[m]; }
        }
        double wl[5], wr[5];
        for (int m = 0; m < 5; ++m) {
            wl[m] = meg7_left_o(c->order, &cw[m][2], &cg[m][2], NULL);
            wr[m] = meg7_right_o(c->order, &cw[m][2], &cg[m][2], NULL);
        }
        char_bwd3(wl, rb, cb, WL);
        char_bwd3(wr, rb, cb, WR);
        conv_flux3(WL, gamma, FL);
        conv_flux3(WR, gamma, FR);
    }
    /* reading R-POS */
    if (!(WL[0] > 0.0 && WL[4] > 0.0 && WR[0] > 0.0 && WR[4] > 0.0)) {
        for (int m = 0; m < 5; ++m) { WL[m] = L->W[m][4]; WR[m] = L->W[m][5]; }
        conv_flux3(WL, gamma, FL);
        conv_flux3(WR, gamma, FR);
    }
    hllc3(WL, WR, FL, FR, gamma, Fout);
}

/* Padded primitive fields, gradients and detector values (periodic wrap or
 * transmissive clamp per axis, NG ghost layers). */
typedef struct {
    int NX, NY, NZ;
    double *W[5];
    double *G[3][5];
    double *psi[3];
} orc3_fields;

static void fields3_free(orc3_fields *F)
{
    for (int m = 0; m < 5; ++m) {
        free(F->W[m]);
        for (int d = 0; d < 3; ++d) free(F->G[d][m]);
    }
    for (int d = 0; d < 3; ++d) free(F->psi[d]);
}

static int fields3_build(const orc3_cfg *c, const double *Q, orc3_fields *F)
{
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int NX = nx + 2 * NG, NY = ny + 2 * NG, NZ = nz + 2 * NG;
    const size_t np = (size_t)NX * NY * NZ, n = (size_t)nx * ny * nz;
    memset(F, 0, sizeof(*F));
    F->NX = NX; F->NY = NY; F->NZ = NZ;
    for (int m = 0; m < 5; ++m) {
        F->W[m] = (double *)calloc(np, sizeof(double));
        if (!F->W[m]) return -1;
        for (int d = 0; d < 3; ++d) {
            F->G[d][m] = (double *)calloc(np, sizeof(double));
            if (!F->G[d][m]) return -1;
        }
    }
    for (int d = 0; d < 3; ++d) {
        F->psi[d] = (double *)calloc(np, sizeof(double));
        if (!F->psi[d]) return -1;
    }
    const double gamma = c->gamma;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < NZ; ++K) {
        const int k = bc_index(K - NG, nz, c->bc[2]);
        for (int I = 0; I < NY; ++I) {
            const int i = bc_index(I - NG, ny, c->bc[1]);
            for (int J = 0; J < NX; ++J) {
                const int j = bc_index(J - NG, nx, c->bc[0]);
                const size_t s = ((size_t)k * ny + i) * nx + j;
                double rho = Q[s], mx = Q[n + s], my = Q[2 * n + s], mz = Q[3 * n + s];
                double E = Q[4 * n + s];
                double u = mx / rho, v = my / rho, w = mz / rho;
                double p = (gamma - 1.0) * (E - rho * (u * u + v * v + w * w) / 2.0);
                const size_t P = ((size_t)K * NY + I) * NX + J;
                F->W[0][P] = rho; F->W[1][P] = u; F->W[2][P] = v; F->W[3][P] = w;
                F->W[4][P] = p;
            }
        }
    }
    const ptrdiff_t stride[3] = {1, NX, (ptrdiff_t)NX * NY};
    const int ext[3] = {NX, NY, NZ};
#pragma omp parallel for schedule(static)
    for (int K = 0; K < NZ; ++K)
        for (int I = 0; I < NY; ++I)
            for (int J = 0; J < NX; ++J) {
                const size_t P = ((size_t)K * NY + I) * NX + J;
                const int idx[3] = {J, I, K};
                for (int d = 0; d < 3; ++d) {
                    const int ok6 = idx[d] >= 3 && idx[d] < ext[d] - 3;
                    for (int m = 0; m < 5; ++m) {
                        double p7[7];
                        for (int q = -3; q <= 3; ++q)
                            p7[q + 3] = ok6 ? F->W[m][P + q * stride[d]] : 0.0;
                        F->G[d][m][P] = ok6 ? orc_grad6(p7) : 0.0;
                    }
                    const double *r = F->W[0];
                    const ptrdiff_t sd = stride[d];
                    F->psi[d][P] = (idx[d] >= 2 && idx[d] < ext[d] - 2)
                        ? orc_psi(r[P - 2 * sd], r[P - sd], r[P], r[P + sd], r[P + 2 * sd]) : 1.0;
                }
            }
    return 0;
}

/* Residual in 3D: Res = -dF/dx - dG/dy - dH/dz.  Q, Res: [5][nz][ny][nx].
 * sig_d (optional): interface flags, the interface below cell index c along d
 * at position c of an array one longer along d. */
long orc3_residual(const orc3_cfg *c, const double *Q, double *Res, uint8_t *sig_x,
                   uint8_t *sig_y, uint8_t *sig_z)
{
    if (!cfg3_ok(c)) return -1;
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t n = (size_t)nx * ny * nz;
    orc3_fields F;
    if (fields3_build(c, Q, &F) != 0) { fields3_free(&F); return -1; }
    const int NX = F.NX, NY = F.NY;
    const ptrdiff_t stride[3] = {1, NX, (ptrdiff_t)NX * NY};
    const double dl[3] = {(c->x1 - c->x0) / nx, (c->y1 - c->y0) / ny, (c->z1 - c->z0) / nz};
    /* cyclic rotation: direction d -> (rho, u_d, u_{d+1}, u_{d+2}, p) */
    const int perm[3][5] = {{0, 1, 2, 3, 4}, {0, 2, 3, 1, 4}, {0, 3, 1, 2, 4}};
    uint8_t *sig[3] = {sig_x, sig_y, sig_z};
    for (size_t s = 0; s < 5 * n; ++s) Res[s] = 0.0;
    for (int d = 0; d < 3; ++d) {
        const int ext[3] = {nx, ny, nz};
        int fe[3] = {nx, ny, nz};
        fe[d] += 1;                           /* interfaces along d */
        const size_t nf = (size_t)fe[0] * fe[1] * fe[2];
        double *Fl = (double *)malloc(sizeof(double) * 5 * nf);
        if (!Fl) { fields3_free(&F); return -1; }
#pragma omp parallel for schedule(static)
        for (int k = 0; k < fe[2]; ++k)
            for (int i = 0; i < fe[1]; ++i)
                for (int j = 0; j < fe[0]; ++j) {
                    /* interface below cell (j, i, k) along d, i.e. between
                     * cell index c-1 and c: the cell left of it is c-1 */
                    int idx[3] = {j, i, k};
                    idx[d] -= 1;
                    const size_t P0 = ((size_t)(idx[2] + NG) * NY + (idx[1] + NG)) * NX
                                    + (idx[0] + NG);
                    orc3_line L;
                    for (int m = 0; m < 5; ++m) {
                        for (int q = -4; q <= 5; ++q)
                            L.W[m][q + 4] = F.W[perm[d][m]][P0 + q * stride[d]];
                        for (int q = -2; q <= 3; ++q)
                            L.G[m][q + 2] = F.G[d][perm[d][m]][P0 + q * stride[d]];
                    }
                    for (int q = -2; q <= 3; ++q) L.psi[q + 2] = F.psi[d][P0 + q * stride[d]];
                    double f[5]; int sg;
                    line_flux3(&L, c, f, &sg);
                    const size_t s = ((size_t)k * fe[1] + i) * fe[0] + j;
                    for (int m = 0; m < 5; ++m) Fl[(size_t)perm[d][m] * nf + s] = f[m];
                    if (sig[d]) sig[d][s] = (uint8_t)sg;
                }
        (void)ext;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int i = 0; i < ny; ++i)
                for (int j = 0; j < nx; ++j) {
                    int up[3] = {j, i, k};
                    up[d] += 1;
                    const size_t sm = ((size_t)k * fe[1] + i) * fe[0] + j;
                    const size_t sp = ((size_t)up[2] * fe[1] + up[1]) * fe[0] + up[0];
                    const size_t s = ((size_t)k * ny + i) * nx + j;
                    for (int m = 0; m < 5; ++m)
                        Res[m * n + s] -= (Fl[m * nf + sp] - Fl[m * nf + sm]) / dl[d];
                }
        free(Fl);
    }
    fields3_free(&F);
    return 0;
}

/* eq. (rk) in 3D (as orc_rk_stage). */
long orc3_rk_stage(const orc3_cfg *c, int stage, double dt, const double *Qn, const double *Qk,
                   double *Qout, uint8_t *sig_x, uint8_t *sig_y, uint8_t *sig_z)
{
    if (!cfg3_ok(c) || stage < 1 || stage > 3) return -1;
    const size_t N = 5 * (size_t)c->nx * c->ny * c->nz;
    double *R = (double *)malloc(sizeof(double) * N);
    if (!R) return -1;
    if (orc3_residual(c, Qk, R, sig_x, sig_y, sig_z) < 0) { free(R); return -1; }
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < N; ++s) {
        if (stage == 1)
            Qout[s] = Qn[s] + dt * R[s];
        else if (stage == 2)
            Qout[s] = 3.0 / 4.0 * Qn[s] + 1.0 / 4.0 * Qk[s] + 1.0 / 4.0 * dt * R[s];
        else
            Qout[s] = 1.0 / 3.0 * Qn[s] + 2.0 / 3.0 * Qk[s] + 2.0 / 3.0 * dt * R[s];
    }
    free(R);
    return 0;
}

/* Sec. 2.5 time step in 3D (inviscid). */
double orc3_dt(const orc3_cfg *c, const double *Q, double cfl)
{
    if (!cfg3_ok(c)) return -1.0;
    const size_t n = (size_t)c->nx * c->ny * c->nz;
    const double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
    const double dz = (c->z1 - c->z0) / c->nz;
    const double gamma = c->gamma;
    double conv = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : conv)
    for (size_t s = 0; s < n; ++s) {
        double rho = Q[s], u = Q[n + s] / rho, v = Q[2 * n + s] / rho, w = Q[3 * n + s] / rho;
        double p = (gamma - 1.0) * (Q[4 * n + s] - rho * (u * u + v * v + w * w) / 2.0);
        double cs = sqrt(gamma * p / rho);
        conv = fmin(conv, fmin(dx / (fabs(u) + cs), fmin(dy / (fabs(v) + cs), dz / (fabs(w) + cs))));
    }
    return cfl * conv;
}

double orc3_step(const orc3_cfg *c, double *Q, double cfl)
{
    const size_t N = 5 * (size_t)c->nx * c->ny * c->nz;
    double dt = orc3_dt(c, Q, cfl);
    double *Q1 = (double *)malloc(sizeof(double) * N);
    double *Q2 = (double *)malloc(sizeof(double) * N);
    if (!Q1 || !Q2 || dt <= 0.0) { free(Q1); free(Q2); return -1.0; }
    orc3_rk_stage(c, 1, dt, Q, Q, Q1, NULL, NULL, NULL);
    orc3_rk_stage(c, 2, dt, Q, Q1, Q2, NULL, NULL, NULL);
    orc3_rk_stage(c, 3, dt, Q, Q2, Q1, NULL, NULL, NULL);
    memcpy(Q, Q1, sizeof(double) * N);
    free(Q1); free(Q2);
    return dt;
}
