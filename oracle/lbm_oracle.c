/*
 * FP64 CPU oracle of the D2Q9 LBM-RANS step (Ponsin & Lozano).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference the HIP library is
 * checked against.  Nothing in the GPU library includes, links or calls it.
 *
 * Every function follows the paper's statement of the method in the paper's
 * order; where the text is silent or garbled, the reading used is stated at
 * the point of use.  Nothing here is blocked, fused or reordered for speed:
 * the collision builds the transfer matrix T(u) of eq (6) and solves with it,
 * streaming uses separate source and destination lattices, and the coarse/fine
 * transfer materialises the exploded populations in an explicit fine-level
 * band before coalescing them.
 *
 * Parity status per part (pins live in tests/):
 *   wall function, Newton, slip velocity, equilibrium, collision, SA-neg
 *   source terms and negative branch, LSQ/IDW, the Lax-Wendroff convection
 *   (quadratic fields and the bilinear cross term advected exactly), half-way
 *   and interpolated bounce-back, periodic conservation, force integral and
 *   the friction sign rule, the angle-of-attack turn of the bodies, the
 *   precomputed cut-link reader: pinned against closed forms, invariants and
 *   independently computed inputs.
 *   Coarse/fine transfer: pinned by exact mass conservation, uniform-flow
 *   preservation and a Poiseuille profile through a refined block that
 *   converges under refinement (the paper gives no formulas for it).
 *   The reference-point stencil rule, the centroid interpolation rule and the
 *   transfer's own first-order terms: parity unpinned beyond the invariants
 *   above (the paper prints no values for them).
 */
#include "oracle.h"

#include <ctype.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* errors                                                                     */
/* ------------------------------------------------------------------------- */
static char g_err[512] = "";

static int fail(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return -1;
}

const char* lbro_error(void) { return g_err; }

int lbro_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* D2Q9 lattice, Section 2.1 eq (2).  Index 0 is the rest population.  The    */
/* second row of eq (2) is read as the y component (its label repeats c_ix).  */
/* ------------------------------------------------------------------------- */
static const int CX[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int CY[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
static const double WQ[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
static const int MIRY[9] = {0, 1, 2, 4, 3, 7, 8, 5, 6}; /* reflection c_y -> -c_y */
#define CS2 (1.0 / 3.0)
/* Per-cell loops over fewer cells run on one thread: every cell's update is
   independent, so this changes the timing only, never a result. */
#define OMP_MIN_CELLS 16384

/* ------------------------------------------------------------------------- */
/* Analytic SA-consistent wall function, Section 2.2 eqs (21)-(22).           */
/* The arctangent terms of eq (22) are evaluated as atan2(b, y+ + a): the     */
/* principal-branch arctan(b/(y+ + a)) jumps by pi at y+ = -a2 and does not    */
/* integrate eq (21), the continuous branch does.                              */
/* ------------------------------------------------------------------------- */
static const double WF_B = 5.033908790505579;
static const double WF_A1 = 8.148221580024245, WF_A2 = -6.9287093849022945;
static const double WF_B1 = 7.4600876082527945, WF_B2 = 7.468145790401841;
static const double WF_C1 = 2.5496773539754747, WF_C2 = 1.3301651588535228;
static const double WF_C3 = 3.599459109332379, WF_C4 = 3.639753186868684494;

/* SA-neg constants, Section 2.2 (list after eq (17)). */
#define SA_CB1 0.1355
#define SA_CB2 0.622
#define SA_SIGMA (2.0 / 3.0)
#define SA_KAPPA 0.41
#define SA_CW2 0.3
#define SA_CW3 2.0
#define SA_CV1 7.1
#define SA_RLIM 10.0
#define SA_CV2 0.7
#define SA_CV3 0.9   /* printed as 0.3, which makes eq (14) singular; SA-neg's value */
#define SA_CT3 1.2
#define SA_CN1 16.0

static double sa_cw1(void) { return SA_CB1 / (SA_KAPPA * SA_KAPPA) + (1.0 + SA_CB2) / SA_SIGMA; }

double lbro_uplus(double y) {
    return WF_B + WF_C1 * log((y + WF_A1) * (y + WF_A1) + WF_B1 * WF_B1)
           - WF_C2 * log((y + WF_A2) * (y + WF_A2) + WF_B2 * WF_B2)
           - WF_C3 * atan2(WF_B1, y + WF_A1) - WF_C4 * atan2(WF_B2, y + WF_A2);
}

/* eq (21) */
double lbro_duplus(double y) {
    double ky = SA_KAPPA * y;
    double k3 = ky * ky * ky;
    double cv3 = SA_CV1 * SA_CV1 * SA_CV1;
    return (cv3 + k3) / (cv3 + k3 * (1.0 + ky));
}

/* Step 3 of the VN procedure (Section 2.3): solve U_t = u_tau u+(d u_tau / nu)
   for u_tau by Newton-Raphson.  phi(u) = u u+(d u / nu) is increasing and
   convex, so the iteration converges from any positive start. */
double lbro_solve_utau(double ut, double dist, double nu, double guess) {
    if (!(ut > 0.0)) return 0.0;
    double u = (guess > 0.0) ? guess : sqrt(nu * ut / dist);
    for (int it = 0; it < 100; ++it) {
        double yp = dist * u / nu;
        double up = lbro_uplus(yp);
        double F = u * up - ut;
        double dF = up + yp * lbro_duplus(yp);
        double du = F / dF;
        double un = u - du;
        if (!(un > 0.0)) un = 0.5 * u;
        u = un;
        if (fabs(du) <= 1e-14 * u) break;
    }
    if (!(u > 0.0) || !isfinite(u)) {
        /* bisection on [0, U_t * 1e3] as a safety net */
        double lo = 0.0, hi = ut * 1e3;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            double F = mid * lbro_uplus(dist * mid / nu) - ut;
            if (F > 0.0) hi = mid; else lo = mid;
        }
        u = 0.5 * (lo + hi);
    }
    return u;
}

/* eq (28) with (nu_t)_V = nu kappa y_V+ (step 5 of the VN procedure). */
double lbro_slip(double utau, double dwv, double nu) {
    double yv = dwv * utau / nu;
    double uv = utau * lbro_uplus(yv);          /* step 4: u_V = u_tau f_SA(y_V+) */
    return uv - utau * utau * dwv / (nu + nu * SA_KAPPA * yv);
}

/* ------------------------------------------------------------------------- */
/* Equilibrium, Section 2.1 eq (4).  The fourth-order coefficient is read as  */
/* 1/(4 c_s^8) (Hermite weight 1/4! times the 6 orderings of xxyy); with the  */
/* printed 1/(2 c_s^8) the central moment of order (2,2) would not be the      */
/* Maxwellian value rho c_s^4.                                                */
/* ------------------------------------------------------------------------- */
void lbro_feq(double rho, double ux, double uy, double f[9]) {
    for (int i = 0; i < 9; ++i) {
        double cx = CX[i], cy = CY[i];
        double cu = cx * ux + cy * uy;
        double h2uu = cu * cu - CS2 * (ux * ux + uy * uy);      /* H2 : uu */
        double h3xxy = (cx * cx - CS2) * cy;
        double h3xyy = cx * (cy * cy - CS2);
        double h4 = (cx * cx - CS2) * (cy * cy - CS2);
        f[i] = WQ[i] * rho *
               (1.0 + cu / CS2 + h2uu / (2.0 * CS2 * CS2) +
                (h3xxy * ux * ux * uy + h3xyy * ux * uy * uy) / (2.0 * CS2 * CS2 * CS2) +
                h4 * ux * ux * uy * uy / (4.0 * CS2 * CS2 * CS2 * CS2));
    }
}

/* Transfer matrix of eq (6) built from the shifted velocities of eq (5). */
static void tmatrix(double ux, double uy, double T[9][9]) {
    for (int i = 0; i < 9; ++i) {
        double X = CX[i] - ux, Y = CY[i] - uy;
        T[0][i] = 1.0;
        T[1][i] = X;
        T[2][i] = Y;
        T[3][i] = X * X + Y * Y;
        T[4][i] = X * X - Y * Y;
        T[5][i] = X * Y;
        T[6][i] = X * X * Y;
        T[7][i] = X * Y * Y;
        T[8][i] = X * X * Y * Y;
    }
}

/* Dense solve of A x = b (Gaussian elimination with partial pivoting). */
static int solve_dense(int n, double* A, double* b, double* x) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[r * n + k]) > fabs(A[p * n + k])) p = r;
        if (A[p * n + k] == 0.0) return -1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double m = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= m * A[k * n + c];
            b[r] -= m * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * x[c];
        x[k] = s / A[k * n + k];
    }
    return 0;
}

void lbro_central_moments(const double f[9], double ux, double uy, double k[9]) {
    double T[9][9];
    tmatrix(ux, uy, T);
    for (int a = 0; a < 9; ++a) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += T[a][i] * f[i];
        k[a] = s;
    }
}

/* Macroscopic moments, eq (3), with the half-force shift of the trapezoidal
   forcing term of eq (1): rho u = sum c f + F/2. */
static void moments(const double f[9], double fx, double fy, double* rho, double* ux, double* uy) {
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        r += f[i];
        jx += CX[i] * f[i];
        jy += CY[i] * f[i];
    }
    *rho = r;
    *ux = (jx + 0.5 * fx) / r;
    *uy = (jy + 0.5 * fy) / r;
}

/* Central-moment collision, eqs (5)-(7) and (9)-(10) with the body force of
   eq (1): k = T f, k* = (I - K) k + K k_eq + (I - K/2) k_F, f* = T^-1 k*, with
   K = diag[1,1,1,omega_b,omega_nu,omega_nu,1,1,1] and k_eq = T f_eq.  The force
   enters central-moment space as k_F = [0, F_x, F_y, 0, ..., 0]. */
void lbro_collide(const double f[9], double nu_eff, double omega_b, const double force[2],
                  double out[9]) {
    double rho, ux, uy;
    moments(f, force[0], force[1], &rho, &ux, &uy);
    double T[9][9], k[9], fe[9], keq[9], ks[9];
    tmatrix(ux, uy, T);
    lbro_feq(rho, ux, uy, fe);
    for (int a = 0; a < 9; ++a) {
        double s = 0.0, se = 0.0;
        for (int i = 0; i < 9; ++i) {
            s += T[a][i] * f[i];
            se += T[a][i] * fe[i];
        }
        k[a] = s;
        keq[a] = se;
    }
    double omega_nu = 1.0 / (nu_eff / CS2 + 0.5);  /* eq (9) with nu_eff = nu + nu_t */
    double K[9] = {1, 1, 1, omega_b, omega_nu, omega_nu, 1, 1, 1};
    double kF[9] = {0, force[0], force[1], 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 9; ++a)
        ks[a] = (1.0 - K[a]) * k[a] + K[a] * keq[a] + (1.0 - 0.5 * K[a]) * kF[a];
    double A[81];
    for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 9; ++i) A[a * 9 + i] = T[a][i];
    solve_dense(9, A, ks, out);
}

/* ------------------------------------------------------------------------- */
/* SA-neg model, Section 2.2 eqs (11)-(17).                                   */
/* ------------------------------------------------------------------------- */
static double sa_fv1(double chi) {
    double c3 = chi * chi * chi;
    return c3 / (c3 + SA_CV1 * SA_CV1 * SA_CV1);
}

/* eq (11) */
static double sa_nut(double nt, double nu) {
    double chi = nt / nu;
    return (nt > 0.0 ? nt : 0.0) * sa_fv1(chi);
}

/* Nodal diffusivity: nu + nt for nt >= 0 (eq 12), nu + nt f_n otherwise (eq 16-17). */
static double sa_mu(double nt, double nu) {
    if (nt >= 0.0) return nu + nt;
    double c3 = (nt / nu) * (nt / nu) * (nt / nu);
    return nu + nt * (SA_CN1 + c3) / (SA_CN1 - c3);
}

/* Source terms.  S-bar = nt f_v2 / (kappa^2 d^2) (the extracted text defines
   only f_v2; this is the SA-neg definition).  When S-tilde vanishes r takes
   its limit.  No trip term: fully turbulent runs. */
void lbro_sa_source(double nt, double nu, double omega, double dist, double out[7]) {
    double chi = nt / nu;
    double k2d2 = SA_KAPPA * SA_KAPPA * dist * dist;
    if (nt >= 0.0) {
        double fv1 = sa_fv1(chi);
        double fv2 = 1.0 - chi / (1.0 + chi * fv1);                   /* eq (14) */
        double sbar = nt * fv2 / k2d2;
        double st;
        if (sbar >= -SA_CV2 * omega) st = omega + sbar;               /* eq (14) */
        else st = omega + omega * (SA_CV2 * SA_CV2 * omega + SA_CV3 * sbar) /
                          ((SA_CV3 - 2.0 * SA_CV2) * omega - sbar);
        double r = (st > 1e-30) ? nt / (st * k2d2) : SA_RLIM;         /* eq (15) */
        if (r > SA_RLIM) r = SA_RLIM;
        double g = r + SA_CW2 * (pow(r, 6.0) - r);
        double cw36 = pow(SA_CW3, 6.0);
        double fw = g * pow((1.0 + cw36) / (pow(g, 6.0) + cw36), 1.0 / 6.0);
        out[0] = SA_CB1 * st * nt;                                     /* eq (13) */
        out[1] = sa_cw1() * fw * (nt / dist) * (nt / dist);
        out[4] = st;
        out[5] = r;
        out[6] = fw;
    } else {
        out[0] = SA_CB1 * (1.0 - SA_CT3) * omega * nt;                 /* eq (17) */
        out[1] = -sa_cw1() * (nt / dist) * (nt / dist);
        out[4] = 0.0;
        out[5] = 0.0;
        out[6] = 0.0;
    }
    out[2] = sa_mu(nt, nu);
    out[3] = sa_nut(nt, nu);
}

/* Unweighted least-squares gradient of a field from the 8 nearest nodes:
   minimise sum_j (v_j - v_0 - g . (x_j - x_0))^2. */
static void lsq_gradient(const double v[9], double* gx, double* gy) {
    double a11 = 0, a12 = 0, a22 = 0, b1 = 0, b2 = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            double dv = v[(dy + 1) * 3 + dx + 1] - v[4];
            a11 += dx * dx; a12 += dx * dy; a22 += dy * dy;
            b1 += dx * dv; b2 += dy * dv;
        }
    double det = a11 * a22 - a12 * a12;
    *gx = (a22 * b1 - a12 * b2) / det;
    *gy = (a11 * b2 - a12 * b1) / det;
}

/* One explicit SA-neg step at a fluid node (Section 2.2): vorticity from LSQ
   velocity gradients; convection by the unsplit 2D Lax-Wendroff scheme (or by
   first-order upwinding); diffusion by centred differences with face-averaged
   nodal diffusivity; c_b2 term outside the divergence as in eq (16).  All
   stencil values are at the old time level; dt = dx = 1. */
double lbro_sa_cell(const double nt[9], const double ux[9], const double uy[9], double nu,
                    double dist, int32_t mode, double mu_cap) {
    double dudx, dudy, dvdx, dvdy;
    lsq_gradient(ux, &dudx, &dudy);
    lsq_gradient(uy, &dvdx, &dvdy);
    double omega = fabs(dvdx - dudy);
    double src[7];
    lbro_sa_source(nt[4], nu, omega, dist, src);
    double u = ux[4], v = uy[4];
    double C = nt[4], E = nt[5], W = nt[3], N = nt[7], S = nt[1];
    double dX = 0.5 * (E - W), dY = 0.5 * (N - S);
    double conv;
    if (mode == LBRO_SA_UPWIND1) {
        double ax = (u > 0.0) ? (C - W) : (E - C);
        double ay = (v > 0.0) ? (C - S) : (N - C);
        conv = -(u * ax + v * ay);
    } else {
        double dXX = E - 2.0 * C + W, dYY = N - 2.0 * C + S;
        double dXY = 0.25 * (nt[8] - nt[6] - nt[2] + nt[0]);
        conv = -(u * dX + v * dY) + 0.5 * (u * u * dXX + 2.0 * u * v * dXY + v * v * dYY);
    }
    /* Face diffusivity: the mean of the two nodal values (eqs (12), (16)).  With
       mu_cap > 0 (an addition, off unless configured) it is limited to mu_cap:
       the explicit update is stable only while (1/sigma) sum_faces mu <= 1, which
       a large eddy viscosity on a fine level can exceed. */
    double muC = sa_mu(C, nu);
    double me = 0.5 * (muC + sa_mu(E, nu)), mw = 0.5 * (muC + sa_mu(W, nu));
    double mn = 0.5 * (muC + sa_mu(N, nu)), ms = 0.5 * (muC + sa_mu(S, nu));
    if (mu_cap > 0.0) {
        me = fmin(me, mu_cap); mw = fmin(mw, mu_cap);
        mn = fmin(mn, mu_cap); ms = fmin(ms, mu_cap);
    }
    double diff = me * (E - C) - mw * (C - W) + mn * (N - C) - ms * (C - S) +
                  SA_CB2 * (dX * dX + dY * dY);
    return C + conv + (src[0] - src[1]) + diff / SA_SIGMA;
}

/* ------------------------------------------------------------------------- */
/* Interpolation at the reference point R (step 1 of the VN procedure).       */
/* ------------------------------------------------------------------------- */
/* Linear least-squares fit v ~ a + b (x_j - x) + c (y_j - y), evaluated at (x, y). */
double lbro_lsq_point(int32_t n, const double* px, const double* py, const double* v,
                      double x, double y) {
    double A[9] = {0}, b[3] = {0}, s[3];
    for (int j = 0; j < n; ++j) {
        double r[3] = {1.0, px[j] - x, py[j] - y};
        for (int a = 0; a < 3; ++a) {
            b[a] += r[a] * v[j];
            for (int c = 0; c < 3; ++c) A[a * 3 + c] += r[a] * r[c];
        }
    }
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (n < 3 || fabs(det) < 1e-9) return NAN;
    if (solve_dense(3, A, b, s) != 0) return NAN;
    return s[0];
}

/* Inverse-distance weighting with power 2. */
double lbro_idw_point(int32_t n, const double* px, const double* py, const double* v,
                      double x, double y) {
    double sw = 0.0, sv = 0.0;
    for (int j = 0; j < n; ++j) {
        double d2 = (px[j] - x) * (px[j] - x) + (py[j] - y) * (py[j] - y);
        if (d2 < 1e-24) return v[j];
        sw += 1.0 / d2;
        sv += v[j] / d2;
    }
    return (n > 0) ? sv / sw : NAN;
}

/* ------------------------------------------------------------------------- */
/* Grid data                                                                  */
/* ------------------------------------------------------------------------- */
enum { T_INACTIVE = LBRO_T_INACTIVE, T_FLUID = LBRO_T_FLUID, T_SOLID = LBRO_T_SOLID,
       T_GHOST = LBRO_T_GHOST, T_COVERED = LBRO_T_COVERED, T_VIRT = LBRO_T_VIRT };

typedef struct {
    int cell, gi, gj, body;
    double q[9];            /* q[o] for a cut link from B in direction o, else -1 */
    double iw[2], nrm[2];   /* wall point and unit normal into the fluid (level units) */
    double dwb;
    double utau, uw[2], rhow, ut[2], chib;
} obnode;

typedef struct {
    int level;
    int nx, ny, gx0, gy0;       /* storage box, with a guard ring */
    int bx0, by0, bnx, bny;     /* I/O box: bounding box of owned and ghost cells */
    double scale;               /* 2^level */
    double nu, fx, fy;          /* lattice values at this level */
    unsigned char* type;
    unsigned char* iface;       /* owned fluid cell fed by coalescence */
    unsigned char* covb;        /* covered cell next to an owned fluid cell */
    int* bid;
    double *f, *fs, *fn, *S, *Sn;
    double *rho, *ux, *uy, *chi, *chin, *d;
    int nb;
    obnode* B;
    int64_t n_fluid, n_ghost, n_cut;
} olevel;

struct lbro_sim {
    lbro_config cfg;
    int nl;
    double u_ref, nu0;
    int64_t step;           /* coarse steps completed */
    int nbody;
    int* npts;
    double** poly;          /* level-0 lattice coordinates, 2*npts doubles each */
    double wall_lat[2];     /* channel wall y in level-0 lattice units */
    olevel lv[LBRO_MAX_LEVELS];
};

/* Start-up ramp (not part of the paper's method; ramp_steps = 0 starts the flow
   impulsively at u_ref): the initial state moves uniformly at r0 u_ref and during
   coarse step n the inlet velocity and the target of the absorbing layer are
   u_ref (r0 + (1 - r0) (1 - cos(pi min(1, n / N))) / 2). */
static double ramp(const lbro_sim* s, int64_t n) {
    double N = s->cfg.ramp_steps, r0 = s->cfg.ramp_start;
    if (!(N > 0.0) || (double)n >= N) return 1.0;
    return r0 + (1.0 - r0) * (0.5 - 0.5 * cos(3.14159265358979323846 * (double)n / N));
}

static int idx(const olevel* L, int gi, int gj) {
    int i = gi - L->gx0, j = gj - L->gy0;
    if (i < 0 || j < 0 || i >= L->nx || j >= L->ny) return -1;
    return j * L->nx + i;
}

static int floordiv2(int a) { return (a >= 0) ? a / 2 : -((-a + 1) / 2); }

static unsigned char type_at(const olevel* L, int gi, int gj) {
    int c = idx(L, gi, gj);
    return c < 0 ? T_INACTIVE : L->type[c];
}

/* Closest point on segment ab to p. */
static double seg_dist(double px, double py, double ax, double ay, double bx, double by,
                       double* cx, double* cy) {
    double ex = bx - ax, ey = by - ay;
    double l2 = ex * ex + ey * ey;
    double t = (l2 > 0.0) ? ((px - ax) * ex + (py - ay) * ey) / l2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double qx = ax + t * ex, qy = ay + t * ey;
    if (cx) { *cx = qx; *cy = qy; }
    return sqrt((px - qx) * (px - qx) + (py - qy) * (py - qy));
}

/* Distance from a point (level-l units) to the bodies; closest point, body and
   segment returned when requested. */
static double body_dist(const lbro_sim* s, double scale, double px, double py, double* qx,
                        double* qy, int* body, int* seg) {
    double best = 1e300;
    for (int b = 0; b < s->nbody; ++b) {
        const double* P = s->poly[b];
        int n = s->npts[b];
        for (int k = 0; k < n; ++k) {
            int k1 = (k + 1) % n;
            double cx, cy;
            double dd = seg_dist(px, py, P[2 * k] * scale, P[2 * k + 1] * scale,
                                 P[2 * k1] * scale, P[2 * k1 + 1] * scale, &cx, &cy);
            if (dd < best) {
                best = dd;
                if (qx) { *qx = cx; *qy = cy; }
                if (body) *body = b;
                if (seg) *seg = k;
            }
        }
    }
    return best;
}

/* Even-odd crossing test: is p inside any body polygon? */
static int inside_body(const lbro_sim* s, double scale, double px, double py) {
    if (s->cfg.body_mode == 1) return 0;   /* bodies only mark refinement */
    for (int b = 0; b < s->nbody; ++b) {
        const double* P = s->poly[b];
        int n = s->npts[b], in = 0;
        for (int k = 0; k < n; ++k) {
            int k1 = (k + 1) % n;
            double ax = P[2 * k] * scale, ay = P[2 * k + 1] * scale;
            double bx = P[2 * k1] * scale, by = P[2 * k1 + 1] * scale;
            if ((ay > py) != (by > py)) {
                double xc = ax + (py - ay) * (bx - ax) / (by - ay);
                if (px < xc) in = !in;
            }
        }
        if (in) return 1;
    }
    return 0;
}

/* Smallest parameter t in (0, 1] at which p0 + t (p1 - p0) crosses a body
   segment; returns -1 when there is none. */
static double link_cut(const lbro_sim* s, double scale, double x0, double y0, double x1,
                       double y1) {
    double best = -1.0;
    if (s->cfg.body_mode == 1) return best;
    double dx = x1 - x0, dy = y1 - y0;
    for (int b = 0; b < s->nbody; ++b) {
        const double* P = s->poly[b];
        int n = s->npts[b];
        for (int k = 0; k < n; ++k) {
            int k1 = (k + 1) % n;
            double ax = P[2 * k] * scale, ay = P[2 * k + 1] * scale;
            double ex = P[2 * k1] * scale - ax, ey = P[2 * k1 + 1] * scale - ay;
            double den = dx * ey - dy * ex;
            if (den == 0.0) continue;
            double t = ((ax - x0) * ey - (ay - y0) * ex) / den;
            double u = ((ax - x0) * dy - (ay - y0) * dx) / den;
            if (t > 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0)
                if (best < 0.0 || t < best) best = t;
        }
    }
    return best;
}

static int level_alloc(olevel* L) {
    size_t n = (size_t)L->nx * L->ny;
    L->type = calloc(n, 1);
    L->iface = calloc(n, 1);
    L->covb = calloc(n, 1);
    L->bid = malloc(n * sizeof(int));
    L->f = calloc(9 * n, sizeof(double));
    L->fs = calloc(9 * n, sizeof(double));
    L->fn = calloc(9 * n, sizeof(double));
    L->S = calloc(9 * n, sizeof(double));
    L->Sn = calloc(9 * n, sizeof(double));
    L->rho = calloc(n, sizeof(double));
    L->ux = calloc(n, sizeof(double));
    L->uy = calloc(n, sizeof(double));
    L->chi = calloc(n, sizeof(double));
    L->chin = calloc(n, sizeof(double));
    L->d = calloc(n, sizeof(double));
    if (!L->type || !L->iface || !L->covb || !L->bid || !L->f || !L->fs || !L->fn || !L->S ||
        !L->Sn || !L->rho || !L->ux || !L->uy || !L->chi || !L->chin || !L->d)
        return fail("out of host memory");
    for (size_t c = 0; c < n; ++c) L->bid[c] = -1;
    return 0;
}

static void level_free(olevel* L) {
    free(L->type); free(L->iface); free(L->covb); free(L->bid);
    free(L->f); free(L->fs); free(L->fn); free(L->S); free(L->Sn);
    free(L->rho); free(L->ux); free(L->uy); free(L->chi); free(L->chin); free(L->d);
    free(L->B);
    memset(L, 0, sizeof *L);
}

void lbro_destroy(lbro_sim* s) {
    if (!s) return;
    for (int l = 0; l < s->nl; ++l) level_free(&s->lv[l]);
    for (int b = 0; b < s->nbody; ++b) free(s->poly[b]);
    free(s->poly);
    free(s->npts);
    free(s);
}

/* Domain extent of level l in its own cell indices. */
static int dom_nx(const lbro_sim* s, int l) { return s->cfg.nx0 << l; }
static int dom_ny(const lbro_sim* s, int l) { return s->cfg.ny0 << l; }

/* Wall distance of a cell centre (level units): bodies and channel walls. */
static double wall_dist(const lbro_sim* s, const olevel* L, int gi, int gj) {
    double px = gi + 0.5, py = gj + 0.5;
    double d = (s->cfg.body_mode == 1) ? 1e300
                                       : body_dist(s, L->scale, px, py, NULL, NULL, NULL, NULL);
    if (s->cfg.bc[2] == LBRO_BC_WALL) {
        double dw = py - s->wall_lat[0] * L->scale;
        if (dw < d) d = dw;
    }
    if (s->cfg.bc[3] == LBRO_BC_WALL) {
        double dw = s->wall_lat[1] * L->scale - py;
        if (dw < d) d = dw;
    }
    return d;
}

/* Builds level l from the covered cells of level l-1 (Section 2.1: the grid is
   refined by factor 2 within a distance band of the body). */
static int build_level(lbro_sim* s, int l) {
    olevel* L = &s->lv[l];
    L->level = l;
    L->scale = (double)(1 << l);
    L->nu = s->nu0 * L->scale;        /* acoustic scaling: lattice nu doubles per level */
    L->fx = s->cfg.force[0] / L->scale;
    L->fy = s->cfg.force[1] / L->scale;
    const int G = 3;
    if (l == 0) {
        L->gx0 = -G; L->gy0 = -G;
        L->nx = s->cfg.nx0 + 2 * G; L->ny = s->cfg.ny0 + 2 * G;
        if (level_alloc(L)) return -1;
        for (int gj = 0; gj < s->cfg.ny0; ++gj)
            for (int gi = 0; gi < s->cfg.nx0; ++gi)
                L->type[idx(L, gi, gj)] =
                    inside_body(s, 1.0, gi + 0.5, gj + 0.5) ? T_SOLID : T_FLUID;
        return 0;
    }
    olevel* P = &s->lv[l - 1];
    double band = s->cfg.band[l] / s->cfg.dx0 * P->scale;
    /* covered cells of the parent level */
    int n = P->nx * P->ny;
#pragma omp parallel for schedule(dynamic, 64)
    for (int c = 0; c < n; ++c) {
        if (P->type[c] != T_FLUID && P->type[c] != T_SOLID) continue;
        int gi = c % P->nx + P->gx0, gj = c / P->nx + P->gy0;
        if (body_dist(s, P->scale, gi + 0.5, gj + 0.5, NULL, NULL, NULL, NULL) < band)
            P->type[c] = T_COVERED;
    }
    int any = 0;
    int lo_i = 1 << 30, lo_j = 1 << 30, hi_i = -(1 << 30), hi_j = -(1 << 30);
    for (int c = 0; c < n; ++c) {
        int gi = c % P->nx + P->gx0, gj = c / P->nx + P->gy0;
        if (P->type[c] == T_COVERED) {
            any = 1;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if (type_at(P, gi + dx, gj + dy) == T_FLUID) P->covb[c] = 1;
        }
        if (P->type[c] == T_FLUID) {
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if (type_at(P, gi + dx, gj + dy) == T_COVERED) P->iface[c] = 1;
        }
        if (P->type[c] == T_COVERED || P->iface[c]) {
            if (gi < lo_i) lo_i = gi;
            if (gj < lo_j) lo_j = gj;
            if (gi > hi_i) hi_i = gi;
            if (gj > hi_j) hi_j = gj;
        }
    }
    if (!any) return fail("level %d: no cells refined (band too small)", l);
    L->gx0 = 2 * lo_i - G; L->gy0 = 2 * lo_j - G;
    L->nx = 2 * (hi_i - lo_i + 1) + 2 * G; L->ny = 2 * (hi_j - lo_j + 1) + 2 * G;
    if (level_alloc(L)) return -1;
    int nn = L->nx * L->ny;
#pragma omp parallel for schedule(dynamic, 64)
    for (int c = 0; c < nn; ++c) {
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        int pc = idx(P, floordiv2(gi), floordiv2(gj));
        if (pc < 0) continue;
        if (P->type[pc] == T_COVERED)
            L->type[c] = inside_body(s, L->scale, gi + 0.5, gj + 0.5) ? T_SOLID : T_FLUID;
        else if (P->iface[pc])
            L->type[c] = T_GHOST;
    }
    /* fine cells next to the ghost band that are neither owned nor ghost carry
       the exploded populations one more cell (the outer edge of the band) */
    for (int c = 0; c < nn; ++c) {
        if (L->type[c] != T_INACTIVE) continue;
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                if (type_at(L, gi + dx, gj + dy) == T_GHOST) L->type[c] = T_VIRT;
    }
    return 0;
}

/* Checks that coarse/fine interfaces keep the clearances the transfer needs. */
static int check_nesting(const lbro_sim* s) {
    for (int l = 0; l < s->nl; ++l) {
        const olevel* L = &s->lv[l];
        for (int c = 0; c < L->nx * L->ny; ++c) {
            int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
            if (L->type[c] == T_COVERED) {
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        unsigned char t = type_at(L, gi + dx, gj + dy);
                        if (t != T_FLUID && t != T_COVERED)
                            return fail("level %d: covered cell (%d,%d) within 2 cells of a "
                                        "non-fluid cell", l, gi, gj);
                    }
                if (L->covb[c] && l + 1 < s->nl) {
                    const olevel* F = &s->lv[l + 1];
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            for (int dy = -3; dy <= 3; ++dy)
                                for (int dx = -3; dx <= 3; ++dx) {
                                    unsigned char t = type_at(F, 2 * gi + a + dx,
                                                              2 * gj + b + dy);
                                    if (t == T_SOLID || t == T_COVERED)
                                        return fail("level %d: interface too close to a "
                                                    "finer interface or a body", l + 1);
                                }
                }
            }
            if (L->type[c] == T_GHOST) {
                for (int dy = -4; dy <= 4; ++dy)
                    for (int dx = -4; dx <= 4; ++dx) {
                        unsigned char t = type_at(L, gi + dx, gj + dy);
                        if (t == T_SOLID || t == T_COVERED)
                            return fail("level %d: ghost cell (%d,%d) too close to a body "
                                        "or a finer level", l, gi, gj);
                    }
            }
        }
        if (l > 0) {
            /* refined levels must stay clear of the domain edge */
            int nxd = dom_nx(s, l), nyd = dom_ny(s, l);
            for (int c = 0; c < L->nx * L->ny; ++c) {
                if (L->type[c] == T_INACTIVE) continue;
                int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
                if (gi < 4 || gj < 4 || gi >= nxd - 4 || gj >= nyd - 4)
                    return fail("level %d reaches the domain edge", l);
            }
        }
    }
    return 0;
}

/* Link-wise wall data (Sections 2.1 and 2.3): cut links with their wall
   fractions q, and for every boundary node the wall point IW, the normal and
   the node's wall distance. */
static int build_walls(lbro_sim* s, int l) {
    olevel* L = &s->lv[l];
    int n = L->nx * L->ny;
    int nxd = dom_nx(s, l), nyd = dom_ny(s, l);
    int cap = 64, nb = 0;
    obnode* B = malloc(cap * sizeof(obnode));
    int64_t ncut = 0;
    for (int c = 0; c < n; ++c) {
        if (L->type[c] != T_FLUID) continue;
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        if (L->d[c] > 1.5) continue;   /* a link of length <= sqrt 2 cannot reach the wall */
        double px = gi + 0.5, py = gj + 0.5;
        double q[9];
        int cut = 0;
        for (int o = 0; o < 9; ++o) q[o] = -1.0;
        for (int o = 1; o < 9; ++o) {
            int ti = gi + CX[o], tj = gj + CY[o];
            int solid = 0;
            double t = -1.0;
            if (l == 0 && ((tj < 0 && s->cfg.bc[2] == LBRO_BC_WALL) ||
                           (tj >= nyd && s->cfg.bc[3] == LBRO_BC_WALL))) {
                double yw = (tj < 0 ? s->wall_lat[0] : s->wall_lat[1]) * L->scale;
                solid = 1;
                t = (yw - py) / (double)CY[o];
            } else {
                int tii = ti;
                if (s->cfg.bc[0] == LBRO_BC_PERIODIC && l == 0) tii = (ti % nxd + nxd) % nxd;
                if (type_at(L, tii, tj) == T_SOLID) solid = 1;
            }
            double tb = link_cut(s, L->scale, px, py, px + CX[o], py + CY[o]);
            if (tb >= 0.0 && (t < 0.0 || tb < t)) t = tb;
            if (solid || tb >= 0.0) {
                q[o] = (t > 0.0) ? t : 0.5;
                cut++;
            }
        }
        if (!cut) continue;
        ncut += cut;
        if (nb == cap) { cap *= 2; B = realloc(B, cap * sizeof(obnode)); }
        obnode* b = &B[nb];
        memset(b, 0, sizeof *b);
        b->cell = c; b->gi = gi; b->gj = gj;
        memcpy(b->q, q, sizeof q);
        double qx, qy;
        int body = -1, seg = -1;
        double dd = body_dist(s, L->scale, px, py, &qx, &qy, &body, &seg);
        if (s->cfg.bc[2] == LBRO_BC_WALL) {
            double yw = s->wall_lat[0] * L->scale;
            if (py - yw < dd) { dd = py - yw; qx = px; qy = yw; body = -1; seg = -1; }
        }
        if (s->cfg.bc[3] == LBRO_BC_WALL) {
            double yw = s->wall_lat[1] * L->scale;
            if (yw - py < dd) { dd = yw - py; qx = px; qy = yw; body = -2; seg = -1; }
        }
        b->iw[0] = qx; b->iw[1] = qy; b->dwb = dd; b->body = body;
        if (dd > 1e-12) {
            b->nrm[0] = (px - qx) / dd;
            b->nrm[1] = (py - qy) / dd;
        } else if (seg >= 0) {
            const double* Pp = s->poly[body];
            int k1 = (seg + 1) % s->npts[body];
            double tx = Pp[2 * k1] - Pp[2 * seg], ty = Pp[2 * k1 + 1] - Pp[2 * seg + 1];
            double tl = sqrt(tx * tx + ty * ty);
            b->nrm[0] = ty / tl; b->nrm[1] = -tx / tl;
        } else {
            b->nrm[0] = 0.0; b->nrm[1] = (body == -1) ? 1.0 : -1.0;
        }
        L->bid[c] = nb;
        nb++;
    }
    L->nb = nb;
    L->B = B;
    L->n_cut = ncut;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Precomputed cut-link lists (Section 2.1: the preprocessor hands over the    */
/* geometry and the cut-link list; Section 2.3: per boundary node the wall     */
/* point, normal, d_WB and the wall fraction q of each cut link).             */
/* File: "lbr-cut-links 1", then blocks "level l n" of n records of 16 numbers */
/* (gi gj IWx IWy nx ny d_WB body q1..q8, q = -1 where not cut); '#' starts a  */
/* comment.                                                                    */
/* ------------------------------------------------------------------------- */
#define LINK_REC 16

typedef struct {
    int64_t n[LBRO_MAX_LEVELS];
    double* rec[LBRO_MAX_LEVELS];
    int given[LBRO_MAX_LEVELS];
} olinks;

static void links_free(olinks* k) {
    for (int l = 0; l < LBRO_MAX_LEVELS; ++l) free(k->rec[l]);
}

/* Next white-space separated token, comments skipped; 0 at the end. */
static int link_token(FILE* f, char* tok, size_t cap) {
    int ch;
    for (;;) {
        ch = fgetc(f);
        if (ch == EOF) return 0;
        if (ch == '#') {
            while (ch != EOF && ch != '\n') ch = fgetc(f);
            continue;
        }
        if (!isspace(ch)) break;
    }
    size_t n = 0;
    while (ch != EOF && !isspace(ch) && ch != '#') {
        if (n + 1 < cap) tok[n++] = (char)ch;
        ch = fgetc(f);
    }
    if (ch == '#') ungetc(ch, f);
    tok[n] = 0;
    return 1;
}

static int link_number(FILE* f, double* v) {
    char tok[128], *end;
    if (!link_token(f, tok, sizeof tok)) return 0;
    *v = strtod(tok, &end);
    return *end == 0 && end != tok;
}

static int read_links(const char* path, int nl, olinks* k) {
    memset(k, 0, sizeof *k);
    FILE* f = fopen(path, "r");
    if (!f) return fail("cannot open %s", path);
    char tok[128];
    if (!link_token(f, tok, sizeof tok) || strcmp(tok, "lbr-cut-links") ||
        !link_token(f, tok, sizeof tok) || strcmp(tok, "1")) {
        fclose(f);
        return fail("%s: not a cut-link file", path);
    }
    while (link_token(f, tok, sizeof tok)) {
        double lv, cnt;
        if (strcmp(tok, "level") || !link_number(f, &lv) || !link_number(f, &cnt) || lv != floor(lv) ||
            lv < 0 || lv >= nl || cnt != floor(cnt) || cnt < 0 || k->given[(int)lv]) {
            fclose(f);
            links_free(k);
            return fail("%s: bad level block", path);
        }
        int l = (int)lv;
        k->given[l] = 1;
        k->n[l] = (int64_t)cnt;
        k->rec[l] = malloc((size_t)(k->n[l] > 0 ? k->n[l] : 1) * LINK_REC * sizeof(double));
        for (int64_t j = 0; j < k->n[l] * LINK_REC; ++j)
            if (!link_number(f, &k->rec[l][j])) {
                fclose(f);
                links_free(k);
                return fail("%s: level %d: truncated or not a number", path, l);
            }
    }
    fclose(f);
    return 0;
}

/* True where the link from (gi, gj) along c_o ends in a solid cell or crosses a
   channel wall of level 0 (the links that must be cut). */
static int link_blocked(const lbro_sim* s, const olevel* L, int l, int gi, int gj, int o) {
    int ti = gi + CX[o], tj = gj + CY[o];
    if (l == 0 && ((tj < 0 && s->cfg.bc[2] == LBRO_BC_WALL) ||
                   (tj >= dom_ny(s, l) && s->cfg.bc[3] == LBRO_BC_WALL)))
        return 1;
    if (s->cfg.bc[0] == LBRO_BC_PERIODIC && l == 0) ti = (ti % dom_nx(s, l) + dom_nx(s, l)) % dom_nx(s, l);
    return type_at(L, ti, tj) == T_SOLID;
}

/* Boundary nodes of level l taken from a precomputed list instead of the
   polyline intersections of build_walls. */
static int walls_from_links(lbro_sim* s, int l, const double* rec, int64_t n) {
    olevel* L = &s->lv[l];
    obnode* B = calloc((size_t)(n > 0 ? n : 1), sizeof(obnode));
    int64_t ncut = 0;
    for (int64_t r = 0; r < n; ++r) {
        const double* p = rec + LINK_REC * r;
        obnode* b = &B[r];
        for (int j = 0; j < LINK_REC; ++j)
            if (!isfinite(p[j])) { free(B); return fail("level %d record %lld: not finite", l, (long long)r); }
        if (p[0] != floor(p[0]) || p[1] != floor(p[1]) || p[7] != floor(p[7])) {
            free(B);
            return fail("level %d record %lld: gi, gj, body must be integers", l, (long long)r);
        }
        b->gi = (int)p[0]; b->gj = (int)p[1]; b->body = (int)p[7];
        b->cell = idx(L, b->gi, b->gj);
        if (b->cell < 0 || L->type[b->cell] != T_FLUID || L->bid[b->cell] >= 0) {
            free(B);
            return fail("level %d record %lld: (%d, %d) is not a fluid cell or is listed twice", l,
                        (long long)r, b->gi, b->gj);
        }
        int near_iface = L->iface[b->cell];
        for (int o = 1; o < 9; ++o)
            if (type_at(L, b->gi + CX[o], b->gj + CY[o]) == T_GHOST) near_iface = 1;
        if (near_iface) {
            free(B);
            return fail("level %d record %lld: (%d, %d) lies next to a level interface", l, (long long)r,
                        b->gi, b->gj);
        }
        int body_ok = (b->body >= 0) ? (s->cfg.body_mode != 1 && b->body < s->nbody)
                                     : (l == 0 && ((b->body == -1 && s->cfg.bc[2] == LBRO_BC_WALL) ||
                                                   (b->body == -2 && s->cfg.bc[3] == LBRO_BC_WALL)));
        double nn = sqrt(p[4] * p[4] + p[5] * p[5]);
        if (!body_ok || fabs(nn - 1.0) > 1e-6 || p[6] < 0.0) {
            free(B);
            return fail("level %d record %lld: bad body, normal or d_WB", l, (long long)r);
        }
        b->iw[0] = p[2]; b->iw[1] = p[3];
        b->nrm[0] = p[4]; b->nrm[1] = p[5];
        b->dwb = p[6];
        b->q[0] = -1.0;
        int cut = 0;
        for (int o = 1; o < 9; ++o) {
            double q = p[7 + o];
            if (q != -1.0 && !(q > 0.0 && q <= 1.0)) {
                free(B);
                return fail("level %d record %lld: q%d outside (0, 1]", l, (long long)r, o);
            }
            b->q[o] = q;
            if (q > 0.0) cut++;
        }
        if (!cut) { free(B); return fail("level %d record %lld: no cut link", l, (long long)r); }
        ncut += cut;
        L->bid[b->cell] = (int)r;
    }
    int n_cells = L->nx * L->ny;
    for (int c = 0; c < n_cells; ++c) {
        if (L->type[c] != T_FLUID) continue;
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        for (int o = 1; o < 9; ++o)
            if (link_blocked(s, L, l, gi, gj, o) && (L->bid[c] < 0 || B[L->bid[c]].q[o] < 0.0)) {
                free(B);
                return fail("level %d: link from (%d, %d) along c_%d reaches a wall but is not listed", l, gi,
                            gj, o);
            }
    }
    L->nb = (int)n;
    L->B = B;
    L->n_cut = ncut;
    return 0;
}

int lbro_create(const lbro_config* cfg, int32_t n_bodies, const int32_t* n_pts, const double* xy,
                lbro_sim** out) {
    return lbro_create_with_links(cfg, n_bodies, n_pts, xy, NULL, out);
}

/* Angle of attack (Section 3.1.1 gives the incidence of the free stream, which
   runs along +x here): a body point x is turned by -alpha about the pivot p,
   x' = p + R(-alpha) (x - p), R the rotation matrix. */
static void turn_point(const lbro_config* cfg, double x, double y, double* xo, double* yo) {
    const double a = -(cfg->alpha_deg * (3.14159265358979323846 / 180.0));
    const double c = cos(a), s = sin(a);
    const double dx = x - cfg->alpha_pivot[0], dy = y - cfg->alpha_pivot[1];
    *xo = (c * dx - s * dy) + cfg->alpha_pivot[0];
    *yo = (s * dx + c * dy) + cfg->alpha_pivot[1];
}

int lbro_create_with_links(const lbro_config* cfg, int32_t n_bodies, const int32_t* n_pts,
                           const double* xy, const char* links_path, lbro_sim** out) {
    *out = NULL;
    if (!cfg || cfg->n_levels < 1 || cfg->n_levels > LBRO_MAX_LEVELS || cfg->nx0 < 4 ||
        cfg->ny0 < 4 || !(cfg->dx0 > 0.0) || cfg->outlet < 0 || cfg->outlet > 2 ||
        cfg->sponge_width < 0.0 || cfg->sponge_strength < 0.0 || cfg->sponge_strength > 1.0 ||
        cfg->ramp_steps < 0.0 || cfg->ramp_start < 0.0 || cfg->ramp_start > 1.0 ||
        !(fabs(cfg->alpha_deg) <= 90.0) || !isfinite(cfg->alpha_pivot[0]) || !isfinite(cfg->alpha_pivot[1]))
        return fail("invalid configuration");
    if ((cfg->bc[0] == LBRO_BC_PERIODIC) != (cfg->bc[1] == LBRO_BC_PERIODIC) ||
        (cfg->bc[2] == LBRO_BC_PERIODIC) != (cfg->bc[3] == LBRO_BC_PERIODIC))
        return fail("periodic boundaries must come in pairs");
    if (cfg->bc[0] == LBRO_BC_WALL || cfg->bc[1] == LBRO_BC_WALL)
        return fail("wall boundaries are supported on the y sides only");
    olinks lk;
    memset(&lk, 0, sizeof lk);
    if (links_path && read_links(links_path, cfg->n_levels, &lk)) return -1;
    lbro_sim* s = calloc(1, sizeof *s);
    s->cfg = *cfg;
    s->nl = cfg->n_levels;
    /* acoustic scaling: lattice speed Mach * c_s; nu = U L / Re in level-0 cells.
       Explicit lattice values, when given, take precedence. */
    s->u_ref = (cfg->u_ref > 0.0) ? cfg->u_ref : cfg->mach * sqrt(CS2);
    s->nu0 = (cfg->nu0 > 0.0) ? cfg->nu0
                              : s->u_ref * (cfg->ref_length / cfg->dx0) / cfg->reynolds;
    if (!(s->nu0 > 0.0)) { free(s); links_free(&lk); return fail("viscosity must be positive"); }
    s->nbody = n_bodies;
    s->npts = calloc(n_bodies > 0 ? n_bodies : 1, sizeof(int));
    s->poly = calloc(n_bodies > 0 ? n_bodies : 1, sizeof(double*));
    const double* p = xy;
    for (int b = 0; b < n_bodies; ++b) {
        if (n_pts[b] < 3) { lbro_destroy(s); links_free(&lk); return fail("body %d has fewer than 3 points", b); }
        s->npts[b] = n_pts[b];
        s->poly[b] = malloc(2 * n_pts[b] * sizeof(double));
        for (int k = 0; k < n_pts[b]; ++k) {
            double x = p[2 * k], y = p[2 * k + 1];
            if (cfg->alpha_deg != 0.0) turn_point(cfg, p[2 * k], p[2 * k + 1], &x, &y);
            s->poly[b][2 * k] = (x - cfg->origin[0]) / cfg->dx0;
            s->poly[b][2 * k + 1] = (y - cfg->origin[1]) / cfg->dx0;
        }
        p += 2 * n_pts[b];
    }
    s->wall_lat[0] = (cfg->wall_y[0] - cfg->origin[1]) / cfg->dx0;
    s->wall_lat[1] = (cfg->wall_y[1] - cfg->origin[1]) / cfg->dx0;
    for (int l = 0; l < s->nl; ++l)
        if (build_level(s, l)) { lbro_destroy(s); links_free(&lk); return -1; }
    if (check_nesting(s)) { lbro_destroy(s); links_free(&lk); return -1; }
    for (int l = 0; l < s->nl; ++l) {
        olevel* L = &s->lv[l];
        int n = L->nx * L->ny;
        int lo_i = 1 << 30, lo_j = 1 << 30, hi_i = -(1 << 30), hi_j = -(1 << 30);
        for (int c = 0; c < n; ++c) {
            int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
            unsigned char t = L->type[c];
            if (t == T_FLUID) L->n_fluid++;
            if (t == T_GHOST) L->n_ghost++;
            if (t == T_FLUID || t == T_SOLID || t == T_COVERED || t == T_GHOST) {
                if (gi < lo_i) lo_i = gi;
                if (gj < lo_j) lo_j = gj;
                if (gi > hi_i) hi_i = gi;
                if (gj > hi_j) hi_j = gj;
            }
        }
        L->bx0 = lo_i; L->by0 = lo_j; L->bnx = hi_i - lo_i + 1; L->bny = hi_j - lo_j + 1;
#pragma omp parallel for schedule(dynamic, 64)
        for (int c = 0; c < n; ++c) {
            int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
            L->d[c] = (L->type[c] == T_FLUID) ? wall_dist(s, L, gi, gj) : 0.0;
        }
        int wr = (lk.given[l] && lk.n[l] > 0) ? walls_from_links(s, l, lk.rec[l], lk.n[l])
                                              : build_walls(s, l);
        if (wr) { lbro_destroy(s); links_free(&lk); return -1; }
        for (int k = 0; k < L->nb; ++k) {
            /* reference stencils must lie in owned cells of this level */
            obnode* b = &L->B[k];
            double rx = b->iw[0] + cfg->d_wr * b->nrm[0], ry = b->iw[1] + cfg->d_wr * b->nrm[1];
            int i0 = (int)floor(rx - 0.5), j0 = (int)floor(ry - 0.5);
            for (int dj = -2; dj <= 3; ++dj)
                for (int di = -2; di <= 3; ++di) {
                    int gi = i0 + di, gj = j0 + dj;
                    if (l == 0 && cfg->bc[0] == LBRO_BC_PERIODIC)
                        gi = (gi % dom_nx(s, 0) + dom_nx(s, 0)) % dom_nx(s, 0);
                    unsigned char t = type_at(L, gi, gj);
                    int outside = (l == 0) && (gj < 0 || gj >= dom_ny(s, 0));
                    if (!outside && t != T_FLUID && t != T_SOLID) {
                        lbro_destroy(s); links_free(&lk);
                        return fail("level %d: wall stencil reaches a non-owned cell", l);
                    }
                }
        }
    }
    links_free(&lk);
    /* default initial state: uniform reference flow (at rest under a start-up ramp) */
    for (int l = 0; l < s->nl; ++l) lbro_init(s, l, NULL, NULL, NULL, NULL);
    *out = s;
    return 0;
}

int lbro_level_info(const lbro_sim* s, int32_t level, int64_t info[8]) {
    if (!s || level < 0 || level >= s->nl) return fail("bad level");
    const olevel* L = &s->lv[level];
    info[0] = L->bx0; info[1] = L->by0; info[2] = L->bnx; info[3] = L->bny;
    info[4] = L->n_fluid; info[5] = L->nb; info[6] = L->n_cut; info[7] = L->n_ghost;
    return 0;
}

int64_t lbro_lups_per_coarse_step(const lbro_sim* s) {
    int64_t n = 0;
    for (int l = 0; l < s->nl; ++l) n += s->lv[l].n_fluid << l;
    return n;
}

int lbro_init(lbro_sim* s, int32_t level, const double* rho, const double* ux, const double* uy,
              const double* chi) {
    if (!s || level < 0 || level >= s->nl) return fail("bad level");
    olevel* L = &s->lv[level];
    for (int j = 0; j < L->bny; ++j)
        for (int i = 0; i < L->bnx; ++i) {
            int c = idx(L, L->bx0 + i, L->by0 + j);
            int k = j * L->bnx + i;
            double r = rho ? rho[k] : s->cfg.rho_ref;
            double u = ux ? ux[k] : s->u_ref * ramp(s, 0);
            double v = uy ? uy[k] : 0.0;
            double x = chi ? chi[k] : s->cfg.chi_init;
            lbro_feq(r, u, v, &L->f[9 * c]);
            L->chi[c] = x;
            L->chin[c] = x;
            L->rho[c] = r; L->ux[c] = u; L->uy[c] = v;
        }
    for (int k = 0; k < L->nb; ++k) L->B[k].utau = 0.0;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* One step of one level                                                      */
/* ------------------------------------------------------------------------- */
static void macros(olevel* L) {
    int n = L->nx * L->ny;
#pragma omp parallel for if (n > OMP_MIN_CELLS)
    for (int c = 0; c < n; ++c)
        if (L->type[c] == T_FLUID) moments(&L->f[9 * c], L->fx, L->fy, &L->rho[c], &L->ux[c], &L->uy[c]);
}

/* Steps 1-5 of the VN procedure (Section 2.3) for one boundary node. */
static void wall_node(const lbro_sim* s, const olevel* L, obnode* b, double* rho_out) {
    const lbro_config* cfg = &s->cfg;
    const double* rho = L->rho;
    const double* ux = L->ux;
    const double* uy = L->uy;
    int c = b->cell;
    b->ut[0] = b->ut[1] = 0.0;
    if (cfg->wall_model == LBRO_WALL_NOSLIP || cfg->wall_model == LBRO_WALL_PRESCRIBED) {
        b->utau = 0.0;
        b->rhow = rho[c];
        int up = (b->body == -2);
        b->uw[0] = (cfg->wall_model == LBRO_WALL_PRESCRIBED) ? cfg->u_wall[2 * up] : 0.0;
        b->uw[1] = (cfg->wall_model == LBRO_WALL_PRESCRIBED) ? cfg->u_wall[2 * up + 1] : 0.0;
        b->chib = 0.0;
        if (rho_out) *rho_out = b->rhow;
        return;
    }
    double dwr = (cfg->wall_model == LBRO_WALL_NISHIMURA) ? 1.75 : cfg->d_wr;
    double rx = b->iw[0] + dwr * b->nrm[0], ry = b->iw[1] + dwr * b->nrm[1];
    int i0 = (int)floor(rx - 0.5), j0 = (int)floor(ry - 0.5);
    int nxd = dom_nx(s, L->level), nyd = dom_ny(s, L->level);
    double rho_r = NAN, ux_r = NAN, uy_r = NAN;
    /* density: IDW over the enclosing 2x2 block without boundary nodes, grown to 4x4 */
    for (int grow = 0; grow <= 1 && isnan(rho_r); ++grow) {
        double px[16], py[16], v[16];
        int m = 0;
        for (int dj = -grow; dj <= 1 + grow; ++dj)
            for (int di = -grow; di <= 1 + grow; ++di) {
                int gi = i0 + di, gj = j0 + dj, gis = gi;
                if (L->level == 0 && cfg->bc[0] == LBRO_BC_PERIODIC) gis = (gi % nxd + nxd) % nxd;
                if (L->level == 0 && (gj < 0 || gj >= nyd)) continue;
                int cc = idx(L, gis, gj);
                if (cc < 0 || L->type[cc] != T_FLUID || L->bid[cc] >= 0) continue;
                px[m] = gi + 0.5; py[m] = gj + 0.5; v[m] = rho[cc]; m++;
            }
        if (m > 0) rho_r = lbro_idw_point(m, px, py, v, rx, ry);
    }
    if (isnan(rho_r)) rho_r = rho[c];
    /* velocity: linear LSQ over the enclosing 2x2 block of fluid cells, grown to 4x4 */
    for (int grow = 0; grow <= 1 && isnan(ux_r); ++grow) {
        double px[16], py[16], vx[16], vy[16];
        int m = 0;
        for (int dj = -grow; dj <= 1 + grow; ++dj)
            for (int di = -grow; di <= 1 + grow; ++di) {
                int gi = i0 + di, gj = j0 + dj, gis = gi;
                if (L->level == 0 && cfg->bc[0] == LBRO_BC_PERIODIC) gis = (gi % nxd + nxd) % nxd;
                if (L->level == 0 && (gj < 0 || gj >= nyd)) continue;
                int cc = idx(L, gis, gj);
                if (cc < 0 || L->type[cc] != T_FLUID) continue;
                px[m] = gi + 0.5; py[m] = gj + 0.5; vx[m] = ux[cc]; vy[m] = uy[cc]; m++;
            }
        ux_r = lbro_lsq_point(m, px, py, vx, rx, ry);
        uy_r = lbro_lsq_point(m, px, py, vy, rx, ry);
        if (isnan(uy_r)) ux_r = NAN;
    }
    if (isnan(ux_r)) { ux_r = ux[c]; uy_r = uy[c]; }
    /* step 2: tangential component */
    double un = ux_r * b->nrm[0] + uy_r * b->nrm[1];
    double tx = ux_r - un * b->nrm[0], ty = uy_r - un * b->nrm[1];
    double ut = sqrt(tx * tx + ty * ty);
    double nu = L->nu;
    double uw;
    if (cfg->wall_model == LBRO_WALL_NISHIMURA) {
        /* eq (31): linear extrapolation from R with d_WR = 1.75 and
           (nu_t)_R = nu kappa y_R+ */
        double utau = lbro_solve_utau(ut, dwr, nu, b->utau);
        double yr = dwr * utau / nu;
        uw = ut - utau * utau * dwr / (nu + nu * SA_KAPPA * yr);
        b->utau = utau;
    } else {
        double utau = lbro_solve_utau(ut, dwr, nu, b->utau);   /* step 3 */
        uw = lbro_slip(utau, cfg->d_wv, nu);                     /* steps 4-5 */
        b->utau = utau;
    }
    /* slip along the wall-parallel direction of the flow at R */
    b->uw[0] = (ut > 0.0) ? uw * tx / ut : 0.0;
    b->uw[1] = (ut > 0.0) ? uw * ty / ut : 0.0;
    b->ut[0] = tx; b->ut[1] = ty;
    b->rhow = rho_r;                                               /* step 6: rho_W = rho_R */
    b->chib = SA_KAPPA * b->utau * b->dwb / nu;                    /* nu-tilde_B = kappa u_tau d_WB */
    if (rho_out) *rho_out = rho_r;
}

static void wall_model_level(lbro_sim* s, olevel* L) {
#pragma omp parallel for schedule(dynamic, 16) if (L->nb > 64)
    for (int k = 0; k < L->nb; ++k) wall_node(s, L, &L->B[k], NULL);
}

static void collide_level(const lbro_sim* s, olevel* L) {
    int n = L->nx * L->ny;
    double F[2] = {L->fx, L->fy};
#pragma omp parallel for if (n > OMP_MIN_CELLS)
    for (int c = 0; c < n; ++c) {
        if (L->type[c] != T_FLUID) continue;
        double nut = sa_nut(L->chi[c] * L->nu, L->nu);
        lbro_collide(&L->f[9 * c], L->nu + nut, s->cfg.omega_b, F, &L->fs[9 * c]);
    }
}

/* Absorbing layer (an addition to the paper's method, used only when
   sponge_width > 0): level-0 post-collision populations within sponge_width
   cells of an inlet, outlet or symmetry side are relaxed towards the
   free-stream equilibrium, sigma = strength ((W - d) / W)^2. */
void lbro_sponge_cell(const double f[9], double sigma, double rho, double ux, double uy, double out[9]) {
    double t[9];
    lbro_feq(rho, ux, uy, t);
    for (int i = 0; i < 9; ++i) out[i] = f[i] - sigma * (f[i] - t[i]);
}

static void sponge_level0(const lbro_sim* s, olevel* L) {
    const lbro_config* cfg = &s->cfg;
    double W = cfg->sponge_width;
    if (L->level != 0 || !(W > 0.0) || !(cfg->sponge_strength > 0.0)) return;
    int far[4];
    for (int k = 0; k < 4; ++k)
        far[k] = cfg->bc[k] == LBRO_BC_INLET || cfg->bc[k] == LBRO_BC_OUTLET ||
                 cfg->bc[k] == LBRO_BC_SYMMETRY;
    int n = L->nx * L->ny;
    for (int c = 0; c < n; ++c) {
        if (L->type[c] != T_FLUID) continue;
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        double d = 1e300;
        if (far[0] && gi + 0.5 < d) d = gi + 0.5;
        if (far[1] && cfg->nx0 - gi - 0.5 < d) d = cfg->nx0 - gi - 0.5;
        if (far[2] && gj + 0.5 < d) d = gj + 0.5;
        if (far[3] && cfg->ny0 - gj - 0.5 < d) d = cfg->ny0 - gj - 0.5;
        if (d >= W) continue;
        double x = (W - d) / W;
        double sigma = cfg->sponge_strength * x * x;
        lbro_sponge_cell(&L->fs[9 * c], sigma, cfg->rho_ref, s->u_ref * ramp(s, s->step), 0.0,
                         &L->fs[9 * c]);
    }
}

/* Covered coarse cells next to owned cells take the mean of their four
   children's macroscopic values (used by the coarse SA stencils). */
static void restrict_level(olevel* C, const olevel* F) {
    int n = C->nx * C->ny;
    for (int c = 0; c < n; ++c) {
        if (!C->covb[c]) continue;
        int gi = c % C->nx + C->gx0, gj = c / C->nx + C->gy0;
        double r = 0, u = 0, v = 0, x = 0;
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                int fc = idx(F, 2 * gi + a, 2 * gj + b);
                r += F->rho[fc]; u += F->ux[fc]; v += F->uy[fc]; x += F->chi[fc];
            }
        C->rho[c] = 0.25 * r; C->ux[c] = 0.25 * u; C->uy[c] = 0.25 * v;
        C->chi[c] = 0.25 * x; C->chin[c] = C->chi[c];
    }
}

/* Ghost cells of the fine level get rho, u and chi from a linear least-squares
   fit over the 3x3 coarse neighbourhood of their parent (Section 2.2: LSQ
   interpolation at level interfaces). */
static void fill_ghosts(const olevel* C, olevel* F) {
    int n = F->nx * F->ny;
    for (int c = 0; c < n; ++c) {
        if (F->type[c] != T_GHOST) continue;
        int gi = c % F->nx + F->gx0, gj = c / F->nx + F->gy0;
        int pi = floordiv2(gi), pj = floordiv2(gj);
        double px[9], py[9], vr[9], vu[9], vv[9], vx[9];
        int m = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int cc = idx(C, pi + dx, pj + dy);
                px[m] = pi + dx + 0.5; py[m] = pj + dy + 0.5;
                vr[m] = C->rho[cc]; vu[m] = C->ux[cc]; vv[m] = C->uy[cc]; vx[m] = C->chi[cc];
                m++;
            }
        double x = (gi + 0.5) * 0.5, y = (gj + 0.5) * 0.5;
        F->rho[c] = lbro_lsq_point(m, px, py, vr, x, y);
        F->ux[c] = lbro_lsq_point(m, px, py, vu, x, y);
        F->uy[c] = lbro_lsq_point(m, px, py, vv, x, y);
        F->chi[c] = lbro_lsq_point(m, px, py, vx, x, y);
        F->chin[c] = F->chi[c];
    }
}

/* Homogeneous explosion (Rohde): the post-collision populations of a coarse
   cell are copied to the fine cells of the band that it covers. */
static void explode(const olevel* C, olevel* F) {
    int n = F->nx * F->ny;
    for (int c = 0; c < n; ++c) {
        if (F->type[c] != T_GHOST && F->type[c] != T_VIRT) continue;
        int gi = c % F->nx + F->gx0, gj = c / F->nx + F->gy0;
        int pc = idx(C, floordiv2(gi), floordiv2(gj));
        for (int i = 0; i < 9; ++i) F->S[9 * c + i] = C->fs[9 * pc + i];
    }
}

/* SA stencil value at a neighbour, applying the domain rules of level 0. */
static int sa_neighbour(const lbro_sim* s, const olevel* L, int gi, int gj, double* nt, double* u,
                        double* v) {
    int nxd = dom_nx(s, L->level), nyd = dom_ny(s, L->level);
    double sgn = 1.0;
    if (L->level == 0) {
        if (gi < 0 || gi >= nxd) {
            if (s->cfg.bc[0] != LBRO_BC_PERIODIC) return -1;
            gi = (gi % nxd + nxd) % nxd;
        }
        if (gj < 0 || gj >= nyd) {
            int side = (gj < 0) ? 2 : 3;
            if (s->cfg.bc[side] == LBRO_BC_PERIODIC) gj = (gj % nyd + nyd) % nyd;
            else if (s->cfg.bc[side] == LBRO_BC_SYMMETRY) { gj = (gj < 0) ? -1 - gj : 2 * nyd - 1 - gj; sgn = -1.0; }
            else return -1;
        }
    }
    int c = idx(L, gi, gj);
    if (c < 0) return -1;
    unsigned char t = L->type[c];
    if (!(t == T_FLUID || t == T_GHOST || (t == T_COVERED && L->covb[c]))) return -1;
    *nt = L->chi[c] * L->nu;
    *u = L->ux[c];
    *v = sgn * L->uy[c];
    return 0;
}

static int sa_level(const lbro_sim* s, olevel* L) {
    int n = L->nx * L->ny;
    int err = 0;
    int nxd = dom_nx(s, L->level);
#pragma omp parallel for reduction(| : err) if (n > OMP_MIN_CELLS)
    for (int c = 0; c < n; ++c) {
        L->chin[c] = L->chi[c];
        if (L->type[c] != T_FLUID || s->cfg.sa_mode == LBRO_SA_FROZEN) continue;
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        if (L->bid[c] >= 0) {                        /* wall boundary node: Dirichlet */
            L->chin[c] = L->B[L->bid[c]].chib;
            continue;
        }
        if (L->level == 0 && gi == 0 && s->cfg.bc[0] == LBRO_BC_INLET) {
            L->chin[c] = s->cfg.chi_inlet;
            continue;
        }
        if (L->level == 0 && gi == nxd - 1 && s->cfg.bc[1] == LBRO_BC_OUTLET) {
            L->chin[c] = L->chi[idx(L, gi - 1, gj)];   /* first-order extrapolation */
            continue;
        }
        double nt[9], u[9], v[9];
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int k = (dy + 1) * 3 + dx + 1;
                if (sa_neighbour(s, L, gi + dx, gj + dy, &nt[k], &u[k], &v[k])) err = 1;
            }
        if (err) continue;
        L->chin[c] = lbro_sa_cell(nt, u, v, L->nu, L->d[c], s->cfg.sa_mode, s->cfg.sa_mu_cap) / L->nu;
    }
    if (err) return fail("SA stencil reached a cell without data on level %d", L->level);
    return 0;
}

/* Post-collision source value for the pull of direction i into a cell of this
   level (interior or across a symmetry / periodic edge of level 0).  Returns
   0 when the population is unknown (inlet / outlet side). */
static int pull_value(const lbro_sim* s, const olevel* L, int gi, int gj, int i, double* val) {
    int nxd = dom_nx(s, L->level), nyd = dom_ny(s, L->level);
    int si = gi - CX[i], sj = gj - CY[i], di = i;
    if (L->level == 0) {
        if (si < 0 || si >= nxd) {
            if (s->cfg.bc[0] != LBRO_BC_PERIODIC) return 0;
            si = (si % nxd + nxd) % nxd;
        }
        if (sj < 0 || sj >= nyd) {
            int side = (sj < 0) ? 2 : 3;
            if (s->cfg.bc[side] == LBRO_BC_PERIODIC) sj = (sj % nyd + nyd) % nyd;
            else if (s->cfg.bc[side] == LBRO_BC_SYMMETRY) {
                /* specular reflection: the population left the same row with c_y mirrored */
                sj = gj;
                di = MIRY[i];
            } else return -1;
        }
    }
    int c = idx(L, si, sj);
    if (c < 0) return -1;
    unsigned char t = L->type[c];
    if (t == T_FLUID) *val = L->fs[9 * c + di];
    else if (t == T_GHOST) *val = L->S[9 * c + di];
    else return -1;
    return 1;
}

/* Bounce-back of the incoming population i at boundary node b.  Step 6 of the
   VN procedure reconstructs the missing populations with Yu's interpolated
   scheme, eq (27), read as: (A) interpolate the outgoing population to the
   wall point W, (B) reflect it there with the wall-momentum term, (C)
   interpolate between W and the next fluid node F2, whose new value is the
   population B sent towards it.  The half-way rule eq (24) is used when F2 is
   not an uncut fluid node, or everywhere when requested. */
static double bounce(const lbro_sim* s, const olevel* L, const obnode* b, int i) {
    int o = OPP[i];                 /* link from B towards the wall */
    double q = b->q[o];
    int c = b->cell;
    double fo_b = L->fs[9 * c + o];
    double fi_b = L->fs[9 * c + i];
    double mom = 2.0 * WQ[o] * b->rhow * (CX[i] * b->uw[0] + CY[i] * b->uw[1]) / CS2;
    int halfway = (s->cfg.bb_mode == LBRO_BB_HALFWAY);
    if (!halfway) {
        /* F2: next node along the link, away from the wall */
        int gi = b->gi + CX[i];
        int nxd = dom_nx(s, L->level);
        if (L->level == 0 && s->cfg.bc[0] == LBRO_BC_PERIODIC) gi = (gi % nxd + nxd) % nxd;
        int c2 = idx(L, gi, b->gj + CY[i]);
        if (c2 >= 0 && L->type[c2] == T_FLUID && b->q[i] < 0.0) {
            double fo_f2 = L->fs[9 * c2 + o];
            double fw_o = q * fo_b + (1.0 - q) * fo_f2;         /* outgoing value at W */
            double fw_i = fw_o + mom;                           /* reflected at W */
            return fw_i + (q / (1.0 + q)) * (fi_b - fw_i);      /* between W and F2 */
        }
    }
    return fo_b + mom;                                          /* eq (24) */
}

static int stream_level(lbro_sim* s, int l) {
    olevel* L = &s->lv[l];
    const olevel* Fn = (l + 1 < s->nl) ? &s->lv[l + 1] : NULL;
    const olevel* Cp = (l > 0) ? &s->lv[l - 1] : NULL;
    int n = L->nx * L->ny;
    int nxd = dom_nx(s, l);
    int err = 0;
#pragma omp parallel for reduction(| : err) if (n > OMP_MIN_CELLS)
    for (int c = 0; c < n; ++c) {
        unsigned char t = L->type[c];
        int gi = c % L->nx + L->gx0, gj = c / L->nx + L->gy0;
        if (t == T_GHOST || t == T_VIRT) {
            /* the fine band carries exploded / fine populations one cell per sub-step */
            for (int i = 0; i < 9; ++i) {
                int sc = idx(L, gi - CX[i], gj - CY[i]);
                unsigned char st = (sc >= 0) ? L->type[sc] : T_INACTIVE;
                if (st == T_FLUID) L->Sn[9 * c + i] = L->fs[9 * sc + i];
                else if (st == T_GHOST || st == T_VIRT) L->Sn[9 * c + i] = L->S[9 * sc + i];
                else {
                    int pc = idx(Cp, floordiv2(gi - CX[i]), floordiv2(gj - CY[i]));
                    L->Sn[9 * c + i] = Cp->fs[9 * pc + i];
                }
            }
            continue;
        }
        if (t != T_FLUID) continue;
        double* fo = &L->fn[9 * c];
        if (L->iface[c]) {
            /* coalescence: mean of the four children of the fine band */
            for (int i = 0; i < 9; ++i) {
                double sum = 0.0;
                for (int bb = 0; bb < 2; ++bb)
                    for (int a = 0; a < 2; ++a)
                        sum += Fn->S[9 * idx(Fn, 2 * gi + a, 2 * gj + bb) + i];
                fo[i] = 0.25 * sum;
            }
            continue;
        }
        const obnode* b = (L->bid[c] >= 0) ? &L->B[L->bid[c]] : NULL;
        for (int i = 0; i < 9; ++i) {
            if (b && b->q[OPP[i]] >= 0.0) { fo[i] = bounce(s, L, b, i); continue; }
            double v;
            int r = pull_value(s, L, gi, gj, i, &v);
            if (r < 0) { err = 1; fo[i] = NAN; }
            else if (r == 0) fo[i] = NAN;   /* unknown, set by the inlet / outlet rule */
            else fo[i] = v;
        }
        /* Zou-He velocity inlet (unknowns have c_x = +1) */
        if (l == 0 && gi == 0 && s->cfg.bc[0] == LBRO_BC_INLET) {
            double ux = s->u_ref * ramp(s, s->step), uy = 0.0;
            double rho = (fo[0] + fo[3] + fo[4] + 2.0 * (fo[2] + fo[6] + fo[8])) / (1.0 - ux);
            fo[1] = fo[2] + (2.0 / 3.0) * rho * ux;
            fo[5] = fo[6] - 0.5 * (fo[3] - fo[4]) + rho * ux / 6.0 + 0.5 * rho * uy;
            fo[7] = fo[8] + 0.5 * (fo[3] - fo[4]) + rho * ux / 6.0 - 0.5 * rho * uy;
        }
    }
    if (err) return fail("stream on level %d reached a cell without data", l);
    /* outlet: unknowns (c_x = -1) extrapolated from the upstream cells, to second
       order (two cells) or, when selected, to first order (a copy of the next
       cell); or Zou-He's rule with the density held at rho_ref and the
       tangential velocity of the upstream cell at time n */
    if (l == 0 && s->cfg.bc[1] == LBRO_BC_OUTLET) {
        for (int gj = 0; gj < dom_ny(s, 0); ++gj) {
            int c = idx(L, nxd - 1, gj);
            if (L->type[c] != T_FLUID) continue;
            int c1 = idx(L, nxd - 2, gj), c2 = idx(L, nxd - 3, gj);
            double* fo = &L->fn[9 * c];
            if (s->cfg.outlet == 2) {
                double rho = s->cfg.rho_ref, uy = L->uy[c1];
                double ux = (fo[0] + fo[3] + fo[4] + 2.0 * (fo[1] + fo[5] + fo[7])) / rho - 1.0;
                fo[2] = fo[1] - (2.0 / 3.0) * rho * ux;
                fo[6] = fo[5] + 0.5 * (fo[3] - fo[4]) - rho * ux / 6.0 - 0.5 * rho * uy;
                fo[8] = fo[7] - 0.5 * (fo[3] - fo[4]) - rho * ux / 6.0 + 0.5 * rho * uy;
                continue;
            }
            for (int i = 0; i < 9; ++i) {
                if (CX[i] != -1) continue;
                if (s->cfg.outlet == 1) fo[i] = L->fn[9 * c1 + i];
                else fo[i] = 2.0 * L->fn[9 * c1 + i] - L->fn[9 * c2 + i];
            }
        }
    }
    double* t;
    t = L->f; L->f = L->fn; L->fn = t;
    t = L->chi; L->chi = L->chin; L->chin = t;
    t = L->S; L->S = L->Sn; L->Sn = t;
    return 0;
}

/* Recursive multilevel cycle (Section 2.1): a finer level takes two sub-steps
   per step of its parent.  Order within a step of level l: macroscopic values,
   wall model, collision with the current eddy viscosity, transfer to and two
   sub-steps of the finer level, SA-neg update, streaming with bounce-back and
   coalescence, domain rules. */
static int cycle(lbro_sim* s, int l) {
    olevel* L = &s->lv[l];
    macros(L);
    wall_model_level(s, L);
    collide_level(s, L);
    sponge_level0(s, L);
    if (l + 1 < s->nl) {
        olevel* F = &s->lv[l + 1];
        macros(F);
        restrict_level(L, F);
        fill_ghosts(L, F);
        explode(L, F);
        if (cycle(s, l + 1)) return -1;
        if (cycle(s, l + 1)) return -1;
    }
    if (sa_level(s, L)) return -1;
    return stream_level(s, l);
}

int lbro_advance(lbro_sim* s, int64_t n) {
    if (!s) return fail("null simulation");
    for (int64_t k = 0; k < n; ++k) {
        if (cycle(s, 0)) return -1;
        s->step++;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Output                                                                     */
/* ------------------------------------------------------------------------- */
int lbro_get_field(const lbro_sim* s, int32_t level, int32_t field, double* out) {
    if (!s || level < 0 || level >= s->nl) return fail("bad level");
    const olevel* L = &s->lv[level];
    for (int j = 0; j < L->bny; ++j)
        for (int i = 0; i < L->bnx; ++i) {
            int c = idx(L, L->bx0 + i, L->by0 + j);
            double* o = &out[j * L->bnx + i];
            unsigned char t = L->type[c];
            if (field == LBRO_F_TYPE) { *o = t; continue; }
            if (t != T_FLUID) { *o = NAN; continue; }
            double r, u, v;
            moments(&L->f[9 * c], L->fx, L->fy, &r, &u, &v);
            switch (field) {
                case LBRO_F_RHO: *o = r; break;
                case LBRO_F_UX: *o = u; break;
                case LBRO_F_UY: *o = v; break;
                case LBRO_F_CHI: *o = L->chi[c]; break;
                case LBRO_F_NUT: *o = sa_nut(L->chi[c] * L->nu, L->nu); break;
                case LBRO_F_DIST: *o = L->d[c]; break;
                default: return fail("unknown field %d", field);
            }
        }
    return 0;
}

int lbro_wall_count(const lbro_sim* s, int32_t level) {
    if (!s || level < 0 || level >= s->nl) return fail("bad level");
    return s->lv[level].nb;
}

/* Evaluates the wall model at the current state (the value the next step
   would use) without changing the stored friction velocities. */
static void current_wall(const lbro_sim* s, int level, obnode* tmp) {
    olevel L = s->lv[level];
    size_t n = (size_t)L.nx * L.ny;
    L.rho = malloc(n * sizeof(double));
    L.ux = malloc(n * sizeof(double));
    L.uy = malloc(n * sizeof(double));
    for (size_t c = 0; c < n; ++c)
        if (L.type[c] == T_FLUID) moments(&L.f[9 * c], L.fx, L.fy, &L.rho[c], &L.ux[c], &L.uy[c]);
    for (int k = 0; k < L.nb; ++k) {
        tmp[k] = L.B[k];
        wall_node(s, &L, &tmp[k], NULL);
    }
    free(L.rho); free(L.ux); free(L.uy);
}

int lbro_get_wall(const lbro_sim* s, int32_t level, double* out) {
    if (!s || level < 0 || level >= s->nl) return fail("bad level");
    const olevel* L = &s->lv[level];
    obnode* tmp = malloc((L->nb > 0 ? L->nb : 1) * sizeof(obnode));
    current_wall(s, level, tmp);
    double U = s->u_ref, rr = s->cfg.rho_ref;
    for (int k = 0; k < L->nb; ++k) {
        const obnode* b = &tmp[k];
        double* o = &out[k * LBRO_WALL_STRIDE];
        int ncut = 0;
        for (int i = 1; i < 9; ++i) ncut += b->q[i] >= 0.0;
        o[0] = b->gi; o[1] = b->gj; o[2] = b->iw[0]; o[3] = b->iw[1];
        o[4] = b->nrm[0]; o[5] = b->nrm[1]; o[6] = b->dwb; o[7] = ncut;
        o[8] = b->utau; o[9] = b->uw[0]; o[10] = b->uw[1]; o[11] = b->rhow;
        o[12] = sqrt(b->ut[0] * b->ut[0] + b->ut[1] * b->ut[1]);
        o[13] = 2.0 * CS2 * (b->rhow - rr) / (rr * U * U);           /* Cp, eq (29) */
        o[14] = 2.0 * (b->rhow / rr) * (b->utau / U) * (b->utau / U); /* Cf, eq (29) */
        o[15] = b->body;
        o[16] = b->chib;
        o[17] = b->ut[0];
        o[18] = b->ut[1];
        for (int i = 1; i < 9; ++i) o[18 + i] = b->q[i];
        o[27] = 0.0;
    }
    free(tmp);
    return 0;
}

/* Surface coefficients at segment centroids (eq (30) and the paragraph after
   it): Cp and sign-corrected Cf interpolated by inverse-distance weighting
   from the two nearest boundary nodes of the same body (distance measured
   between the node's wall point and the centroid). */
static int surface_eval(const lbro_sim* s, int body, double* cp, double* cfs, double* fsum) {
    if (body < 0 || body >= s->nbody) return fail("bad body");
    int lf = s->nl - 1;
    for (; lf >= 0; --lf) if (s->lv[lf].nb > 0) break;
    if (lf < 0) return fail("no wall nodes");
    const olevel* L = &s->lv[lf];
    obnode* tmp = malloc(L->nb * sizeof(obnode));
    current_wall(s, lf, tmp);
    int n = s->npts[body];
    const double* P = s->poly[body];
    double U = s->u_ref, rr = s->cfg.rho_ref;
    double cf[2] = {0, 0}, cpv[2] = {0, 0};
    double dxphys = s->cfg.dx0;
    for (int k = 0; k < n; ++k) {
        int k1 = (k + 1) % n;
        double ax = P[2 * k] * L->scale, ay = P[2 * k + 1] * L->scale;
        double bx = P[2 * k1] * L->scale, by = P[2 * k1 + 1] * L->scale;
        double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by);
        double tx = bx - ax, ty = by - ay, tl = sqrt(tx * tx + ty * ty);
        tx /= tl; ty /= tl;
        double nx = ty, ny = -tx;                  /* into the fluid for a CCW polyline */
        int best[2] = {-1, -1};
        double bd[2] = {1e300, 1e300};
        for (int j = 0; j < L->nb; ++j) {
            if (tmp[j].body != body) continue;
            double dd = (tmp[j].iw[0] - mx) * (tmp[j].iw[0] - mx) + (tmp[j].iw[1] - my) * (tmp[j].iw[1] - my);
            if (dd < bd[0]) { bd[1] = bd[0]; best[1] = best[0]; bd[0] = dd; best[0] = j; }
            else if (dd < bd[1]) { bd[1] = dd; best[1] = j; }
        }
        double sw = 0, scp = 0, scf = 0;
        for (int m = 0; m < 2; ++m) {
            if (best[m] < 0) continue;
            const obnode* b = &tmp[best[m]];
            double w = (bd[m] < 1e-24) ? 1e300 : 1.0 / bd[m];
            double cpb = 2.0 * CS2 * (b->rhow - rr) / (rr * U * U);
            double cfb = 2.0 * (b->rhow / rr) * (b->utau / U) * (b->utau / U);
            double sg = (b->ut[0] * tx + b->ut[1] * ty >= 0.0) ? 1.0 : -1.0;
            sw += w; scp += w * cpb; scf += w * cfb * sg;
            if (bd[m] < 1e-24) { sw = 1.0; scp = cpb; scf = cfb * sg; break; }
        }
        double cpk = scp / sw, cfk = scf / sw;
        if (cp) cp[k] = cpk;
        if (cfs) cfs[k] = cfk;
        double ds = tl / L->scale * dxphys;        /* physical segment length */
        cf[0] += cfk * tx * ds; cf[1] += cfk * ty * ds;
        cpv[0] -= cpk * nx * ds; cpv[1] -= cpk * ny * ds;
    }
    free(tmp);
    double c = s->cfg.ref_length;
    if (fsum) {
        fsum[0] = cf[0] / c;                  /* C_Df */
        fsum[1] = cpv[0] / c;                 /* C_Dp */
        fsum[2] = (cf[0] + cpv[0]) / c;       /* C_D */
        fsum[3] = cpv[1] / c;                 /* C_L (pressure only, eq (30)) */
        fsum[4] = cf[1] / c;                  /* friction force along y */
    }
    return 0;
}

int lbro_surface(const lbro_sim* s, int32_t body, double* cp, double* cf) {
    return surface_eval(s, body, cp, cf, NULL);
}

int lbro_forces(const lbro_sim* s, int32_t body, double out[5]) {
    if (body >= 0) return surface_eval(s, body, NULL, NULL, out);
    double acc[5] = {0, 0, 0, 0, 0}, t[5];
    for (int b = 0; b < s->nbody; ++b) {
        if (surface_eval(s, b, NULL, NULL, t)) return -1;
        for (int k = 0; k < 5; ++k) acc[k] += t[k];
    }
    memcpy(out, acc, sizeof acc);
    return 0;
}
