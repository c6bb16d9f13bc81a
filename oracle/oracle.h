/*
 * FP64 CPU oracle of the D2Q9 LBM-RANS time step with the virtual-node
 * slip-velocity bounce-back (Ponsin & Lozano, "Enhanced wall boundary
 * modeling for turbulent flows using the lattice Boltzmann method with
 * adaptive Cartesian grids").
 *
 * TEST INFRASTRUCTURE.  This library is the plain, slow reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or helper with the GPU library.
 *
 * Units: the caller gives geometry in physical (chord) units together with the
 * level-0 cell size dx0 and the box origin; internally every level l works in
 * its own lattice units (cell size 1, time step 1).  Flow values in the config
 * are lattice values of level 0.
 */
#ifndef LBRO_ORACLE_H
#define LBRO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBRO_MAX_LEVELS 12

enum { LBRO_BC_PERIODIC = 0, LBRO_BC_INLET = 1, LBRO_BC_OUTLET = 2,
       LBRO_BC_SYMMETRY = 3, LBRO_BC_WALL = 4 };
enum { LBRO_WALL_VN = 0, LBRO_WALL_NISHIMURA = 1, LBRO_WALL_NOSLIP = 2,
       LBRO_WALL_PRESCRIBED = 3 };
enum { LBRO_BB_AUTO = 0, LBRO_BB_YU = 1, LBRO_BB_HALFWAY = 2 };
enum { LBRO_SA_FROZEN = 0, LBRO_SA_LW = 1, LBRO_SA_UPWIND1 = 2 };
enum { LBRO_F_RHO = 0, LBRO_F_UX = 1, LBRO_F_UY = 2, LBRO_F_CHI = 3,
       LBRO_F_NUT = 4, LBRO_F_TYPE = 5, LBRO_F_DIST = 6 };

/* Cell types reported by LBRO_F_TYPE. */
enum { LBRO_T_INACTIVE = 0, LBRO_T_FLUID = 1, LBRO_T_SOLID = 2,
       LBRO_T_GHOST = 3, LBRO_T_COVERED = 4, LBRO_T_VIRT = 5 };

typedef struct {
    int32_t nx0, ny0;             /* level-0 cells */
    int32_t n_levels;
    int32_t bc[4];                /* x-lo, x-hi, y-lo, y-hi */
    int32_t wall_model, bb_mode, sa_mode;
    int32_t body_mode;            /* 0: bodies are solid walls, 1: they only mark refinement */
    int32_t outlet;               /* 0: second-order, 1: first-order outlet extrapolation,
                                     2: Zou-He pressure outlet at rho_ref */
    double origin[2];             /* physical corner of the level-0 box */
    double dx0;                   /* physical level-0 cell size */
    double band[LBRO_MAX_LEVELS]; /* band[l], l >= 1: physical refinement distance */
    double wall_y[2];             /* physical y of channel walls (bc = WALL) */
    double mach, reynolds, ref_length;
    double u_ref, nu0;            /* level-0 lattice values; each used when > 0 */
    double rho_ref, chi_inlet, chi_init;
    double force[2];              /* level-0 lattice body force per unit volume */
    double omega_b;
    double d_wr, d_wv;            /* reference / virtual node distances, in cells */
    double u_wall[4];             /* PRESCRIBED slip velocity: lower (x,y), upper (x,y) */
    double sponge_width;          /* absorbing layer of level 0, in level-0 cells (0: none) */
    double sponge_strength;       /* its largest relaxation rate per step */
    double ramp_steps;            /* start-up: coarse steps over which the inlet velocity and
                                     the absorbing-layer target rise from ramp_start u_ref to
                                     u_ref (0: none) */
    double ramp_start;            /* initial fraction of u_ref under a start-up ramp */
    double sa_mu_cap;             /* SA face diffusivity limit in lattice units (not part of
                                     the method; <= 0: none, the scheme of eqs (12), (16)) */
    double alpha_deg;             /* angle of attack in degrees: the bodies are turned by
                                     -alpha about alpha_pivot before use (0: given at their
                                     incidence); |alpha| <= 90 */
    double alpha_pivot[2];        /* physical point they turn about */
} lbro_config;

typedef struct lbro_sim lbro_sim;

/* Number of doubles per wall-node record returned by lbro_get_wall. */
/* Record: gi, gj, IW (x, y), normal (x, y), d_WB, number of cut links,
   u_tau, u_W (x, y), rho_W, |u_Rt|, Cp, Cf, body, chi_B, u_Rt (x, y),
   q[1..8] (-1 where the link is not cut), spare. */
#define LBRO_WALL_STRIDE 28

/* Absorbing-layer rule for one cell (test access): out = f - sigma (f - f_eq(rho, ux, uy)). */
void lbro_sponge_cell(const double f[9], double sigma, double rho, double ux, double uy, double out[9]);

const char* lbro_error(void);

int  lbro_create(const lbro_config* cfg, int32_t n_bodies, const int32_t* n_pts,
                 const double* xy, lbro_sim** out);
/* The same with the boundary nodes of some levels read from a precomputed
   cut-link file (links_path; NULL: none), in place of the polyline
   intersections (Section 2.1: the preprocessor's cut-link list; Section 2.3:
   the link-wise wall data).  Format: "lbr-cut-links 1", then blocks
   "level l n" of n records gi gj IWx IWy nx ny d_WB body q1..q8 (q = -1: not
   cut); '#' starts a comment.  A block with n = 0 keeps the generated nodes. */
int  lbro_create_with_links(const lbro_config* cfg, int32_t n_bodies, const int32_t* n_pts,
                            const double* xy, const char* links_path, lbro_sim** out);
void lbro_destroy(lbro_sim* s);
/* info: gx0, gy0, nx, ny (I/O box: bounding box of owned and ghost cells, in
   global level-l cell indices), n_fluid, n_bnodes, n_cut_links, n_ghost */
int  lbro_level_info(const lbro_sim* s, int32_t level, int64_t info[8]);
/* Equilibrium initialisation of one level from dense I/O-box arrays (row-major
   ny x nx).  Any pointer may be NULL: rho_ref, (u_ref, 0) and chi_init. */
int  lbro_init(lbro_sim* s, int32_t level, const double* rho, const double* ux,
               const double* uy, const double* chi);
int  lbro_advance(lbro_sim* s, int64_t n_coarse_steps);
int  lbro_get_field(const lbro_sim* s, int32_t level, int32_t field, double* out);
int  lbro_wall_count(const lbro_sim* s, int32_t level);
int  lbro_get_wall(const lbro_sim* s, int32_t level, double* out);
int  lbro_forces(const lbro_sim* s, int32_t body, double out[5]);
int  lbro_surface(const lbro_sim* s, int32_t body, double* cp, double* cf);
int64_t lbro_lups_per_coarse_step(const lbro_sim* s);
int  lbro_threads(void);

/* Pure functions exposed for the pins. */
double lbro_uplus(double yplus);
double lbro_duplus(double yplus);
double lbro_solve_utau(double ut, double dist, double nu, double guess);
double lbro_slip(double utau, double dwv, double nu);
void   lbro_feq(double rho, double ux, double uy, double f[9]);
void   lbro_central_moments(const double f[9], double ux, double uy, double k[9]);
void   lbro_collide(const double f[9], double nu_eff, double omega_b,
                    const double force[2], double out[9]);
/* out: P, D, mu, nu_t, S_tilde, r, f_w */
void   lbro_sa_source(double nut, double nu, double omega, double dist, double out[7]);
/* stencil arrays are [3][3] row-major with index [dy+1][dx+1] */
double lbro_sa_cell(const double nt[9], const double ux[9], const double uy[9],
                    double nu, double dist, int32_t mode, double mu_cap);
double lbro_lsq_point(int32_t n, const double* px, const double* py, const double* v,
                      double x, double y);
double lbro_idw_point(int32_t n, const double* px, const double* py, const double* v,
                      double x, double y);

#ifdef __cplusplus
}
#endif
#endif
