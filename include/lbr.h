/*
 * liblbr: MI355X (gfx950) implementation of the time step of the LBM-RANS
 * method with the virtual-node slip-velocity bounce-back of Ponsin & Lozano,
 * "Enhanced wall boundary modeling for turbulent flows using the lattice
 * Boltzmann method with adaptive Cartesian grids".
 *
 * The problem is stated the way the paper states it (Sections 2.1-2.3 and
 * 3.1.1): closed wall polylines, a multilevel Cartesian grid given by the
 * level-0 resolution and the refinement bands, the flow parameters (Mach,
 * Reynolds, reference density, inlet turbulence level), a number of time
 * steps, and the outputs the paper reports (macroscopic fields, surface Cp
 * and Cf, integrated force coefficients).
 *
 * Conventions for every entry point:
 *  - Return value 0 on success, a negative LBR_ERR_* code on failure.  The
 *    message of the last failure of a context is returned by
 *    lbr_last_error(); no C++ exception crosses this interface.
 *  - Host arrays passed in are read during the call and not retained.  Host
 *    arrays passed out are written during the call (the call synchronises
 *    the context's stream first).
 *  - Device memory is owned by the library.  It is obtained from the
 *    allocator callbacks in the config (for example PyTorch's caching
 *    allocator) or, when those are NULL, from hipMalloc.
 *  - All device work of a context is enqueued on the stream given in the
 *    config (NULL: the default stream).  One context per host thread.
 *
 * Units: geometry in physical units (chord lengths); level l has cell size
 * dx0 / 2^l; lattice values (velocities, viscosity, force) refer to level 0
 * and are rescaled to finer levels with acoustic scaling (Section 2.1).
 */
#ifndef LBR_H
#define LBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBR_ABI_VERSION 6
#define LBR_MAX_LEVELS 12

enum lbr_status {
    LBR_OK = 0,
    LBR_ERR_INVALID_ARG = -1,
    LBR_ERR_OOM = -2,
    LBR_ERR_HIP = -3,
    LBR_ERR_GEOMETRY = -4,
    LBR_ERR_DIVERGED = -5,
    LBR_ERR_STATE = -6,
    LBR_ERR_IO = -7,
    LBR_ERR_NEWTON = -8,           /* a wall node's friction velocity (Section 2.3, step 3)
                                      is not finite */
    LBR_ERR_NOT_CONVERGED = -9     /* a run to steady state reached its step limit first */
};

/* Population storage.  Populations are stored shifted by their lattice
   weight (f_i - w_i); arithmetic is FP64 for LBR_STORE_F64 and FP32
   otherwise.  LBR_STORE_MIXED keeps FP32 on the two finest levels (the wall
   nodes and the boundary layer, most of the cell updates of a multilevel
   grid) and FP16 on the coarser ones.  The friction-velocity Newton solve, the
   wall-distance field and the force sums are always FP64. */
enum lbr_storage { LBR_STORE_F64 = 0, LBR_STORE_F32 = 1, LBR_STORE_F16 = 2, LBR_STORE_BF16 = 3,
                   LBR_STORE_MIXED = 4 };

/* Domain sides: x-lo, x-hi, y-lo, y-hi.  Supported per side (lbr_create
   refuses the rest): x-lo PERIODIC or INLET, x-hi PERIODIC or OUTLET, y-lo and
   y-hi PERIODIC, SYMMETRY or WALL (channel walls at wall_y); periodic sides
   come in pairs. */
enum lbr_bc { LBR_BC_PERIODIC = 0, LBR_BC_INLET = 1, LBR_BC_OUTLET = 2, LBR_BC_SYMMETRY = 3,
              LBR_BC_WALL = 4 };

/* Wall treatment: the virtual-node slip velocity (Section 2.3), Nishimura's
   linear extrapolation from R (eq. (31)), no slip, or a prescribed wall
   velocity (for laminar checks). */
enum lbr_wall_model { LBR_WALL_VN = 0, LBR_WALL_NISHIMURA = 1, LBR_WALL_NOSLIP = 2,
                      LBR_WALL_PRESCRIBED = 3 };

/* Link-wise bounce-back: Yu's interpolated scheme eq. (27) at every cut link
   (AUTO and YU), or the half-way rule eq. (24) at every cut link. */
enum lbr_bb { LBR_BB_AUTO = 0, LBR_BB_YU = 1, LBR_BB_HALFWAY = 2 };

/* SA-neg convection: frozen (no SA update), Lax-Wendroff, first-order upwind. */
enum lbr_sa { LBR_SA_FROZEN = 0, LBR_SA_LW = 1, LBR_SA_UPWIND1 = 2 };
/* Outlet (Section 3.1.1).  EXTRAP2 / EXTRAP1: the populations entering from
   outside are extrapolated from the upstream cells, to second order
   (2 f(N-1) - f(N-2), the extrapolation the paper cites) or to first order
   (f(N-1)).  PRESSURE: Zou-He's rule (the inlet's, Section 3.1.1) with the
   density held at rho_ref and the tangential velocity of the upstream cell;
   it fixes the pressure level that the two extrapolations leave free. */
enum lbr_outlet { LBR_OUTLET_EXTRAP2 = 0, LBR_OUTLET_EXTRAP1 = 1, LBR_OUTLET_PRESSURE = 2 };
/* Absorbing layer (not part of the paper's method; off unless sponge_width > 0).
   Level 0 is nearly inviscid under acoustic scaling, so pressure waves of the
   whole domain reflect between its far-field sides for thousands of steps.
   Within sponge_width cells of an INLET, OUTLET or SYMMETRY side, each level-0
   step relaxes the post-collision populations towards the free-stream
   equilibrium, f <- f - sigma (f - f_eq(rho_ref, u_ref, 0)), with
   sigma = sponge_strength ((W - d) / W)^2 at distance d (cell centre to side). */

enum lbr_body { LBR_BODY_SOLID = 0, LBR_BODY_REFINE_ONLY = 1 };

/* Fields for lbr_read_field. */
enum lbr_field { LBR_FIELD_RHO = 0, LBR_FIELD_UX = 1, LBR_FIELD_UY = 2, LBR_FIELD_CHI = 3,
                 LBR_FIELD_NUT = 4, LBR_FIELD_TYPE = 5, LBR_FIELD_DIST = 6 };

/* Cell types reported through LBR_FIELD_TYPE. */
enum lbr_cell { LBR_CELL_INACTIVE = 0, LBR_CELL_FLUID = 1, LBR_CELL_SOLID = 2,
                LBR_CELL_GHOST = 3, LBR_CELL_COVERED = 4 };

typedef void* (*lbr_alloc_fn)(size_t bytes, void* user);
typedef void (*lbr_free_fn)(void* ptr, void* user);

typedef struct lbr_config {
    int32_t version;               /* LBR_ABI_VERSION */
    int32_t storage;               /* enum lbr_storage */
    int32_t nx0, ny0;              /* level-0 cells */
    int32_t n_levels;              /* 1..LBR_MAX_LEVELS */
    int32_t bc[4];                 /* enum lbr_bc for x-lo, x-hi, y-lo, y-hi */
    int32_t wall_model;            /* enum lbr_wall_model */
    int32_t bb;                    /* enum lbr_bb */
    int32_t sa;                    /* enum lbr_sa */
    int32_t body_mode;             /* enum lbr_body */
    int32_t outlet;                /* enum lbr_outlet: rule for the unknown populations at an
                                      OUTLET edge */
    double origin[2];              /* physical position of the level-0 box corner */
    double dx0;                    /* physical size of a level-0 cell */
    double band[LBR_MAX_LEVELS];   /* band[l] (l >= 1): level l-1 cells closer than this
                                      physical distance to a body are refined */
    double wall_y[2];              /* physical y of the channel walls (bc = WALL) */
    double mach, reynolds;         /* freestream Mach and Reynolds number */
    double ref_length;             /* physical reference length (chord) */
    double u_ref;                  /* level-0 lattice reference velocity (<= 0: mach c_s) */
    double nu0;                    /* level-0 lattice viscosity (<= 0: from reynolds) */
    double rho_ref;                /* reference density (lattice units, normally 1) */
    double chi_inlet;              /* nu-tilde / nu at the inlet (paper: 3) */
    double chi_init;               /* initial nu-tilde / nu (paper: 3) */
    double force[2];               /* level-0 lattice body force per unit volume */
    double omega_b;                /* bulk relaxation frequency (paper: 1) */
    double d_wr, d_wv;             /* reference / virtual node distances in cells (2, 1) */
    double u_wall[4];              /* LBR_WALL_PRESCRIBED: (ux, uy) lower, (ux, uy) upper */
    double sponge_width;           /* absorbing layer along the INLET, OUTLET and SYMMETRY
                                      sides of level 0, in level-0 cells (0 = none) */
    double sponge_strength;        /* its largest relaxation rate per level-0 step */
    double ramp_steps;             /* start-up ramp (not part of the paper's method): coarse
                                      steps N over which the inlet velocity and the
                                      absorbing-layer target rise from ramp_start u_ref to
                                      u_ref as r0 + (1 - r0) (1 - cos(pi n / N)) / 2; the
                                      default initial state moves at ramp_start u_ref
                                      (N = 0: impulsive start at u_ref) */
    double ramp_start;             /* r0, in [0, 1] */
    int32_t shift16;               /* 16-bit population storage (FP16, BF16, the FP16 levels of
                                      LBR_STORE_MIXED): 0 stores f_i - w_i; 1 stores
                                      f_i - f_eq_i(rho_ref, u_ref e_x) (free-stream shift, exact
                                      in FP32 arithmetic on load and store); other storage
                                      formats ignore it */
    int32_t health_every;          /* health check of lbr_advance (0: none): after every
                                      health_every-th coarse step the state of every level is
                                      scanned on the device (density finite and positive,
                                      |u| <= c_s, the wall nodes' friction velocity finite);
                                      lbr_advance waits for the scans at its end and returns
                                      LBR_ERR_DIVERGED or LBR_ERR_NEWTON if one failed */
    double sa_mu_cap;              /* SA face diffusivity limit, lattice units of each level (not
                                      part of the paper's method; <= 0: none, the centred
                                      diffusion of eqs (12) and (16) as printed).  The explicit
                                      update is stable only while (1/sigma) times the sum of the
                                      four face diffusivities stays below 1; a limit of
                                      0.2 sigma keeps it there where a large eddy viscosity on a
                                      fine level would not.  Below the limit the scheme is
                                      unchanged, bit for bit. */
    double alpha_deg;              /* angle of attack in degrees (the incidence of the free
                                      stream, Section 3.1.1): lbr_set_geometry turns every body
                                      by -alpha_deg about alpha_pivot, so that the stream along
                                      +x meets it at incidence alpha (nose up for alpha > 0);
                                      C_D and C_L stay along and across +x.  0 for bodies given
                                      at their incidence.  |alpha_deg| <= 90. */
    double alpha_pivot[2];         /* physical point the bodies turn about (e.g. the
                                      quarter chord) */
    lbr_alloc_fn alloc_fn;         /* optional device allocator */
    lbr_free_fn free_fn;
    void* alloc_user;
    void* stream;                  /* hipStream_t, NULL = default stream */
} lbr_config;

typedef struct lbr_ctx lbr_ctx;

/* Level description: the I/O box is the bounding box of the level's owned and
   ghost cells, in global cell indices of the level (cell (i, j) of level l
   spans [i, i+1] x [j, j+1] * dx0 / 2^l from the origin). */
typedef struct lbr_level_desc {
    int64_t gx0, gy0, nx, ny;      /* I/O box */
    int64_t n_fluid;               /* owned fluid cells (the cells counted in MLUPS) */
    int64_t n_wall_nodes;          /* boundary nodes B */
    int64_t n_cut_links;
    int64_t n_ghost;
    int64_t n_tiles;               /* active 64 x H tiles launched per step (H: the level's tile height) */
    int64_t bytes;                 /* device bytes held by the level */
} lbr_level_desc;

/* Number of doubles per wall-node record from lbr_read_wall: gi, gj, IW (x,y),
   normal (x,y), d_WB, number of cut links, u_tau, u_W (x,y), rho_W, |u_Rt|,
   Cp, Cf, body, chi_B, u_Rt (x,y), q[1..8] (-1: not cut; directions as in
   lbr_set_cut_links), spare.  Positions
   and distances are in lattice units of the node's level. */
#define LBR_WALL_STRIDE 28

/* Creates a context and validates the config (Section 2.1 parameters:
   omega_b, d_WR = 2, d_WV = 1 unless changed).  cfg is copied; no device
   work is done.  Errors: LBR_ERR_INVALID_ARG for an inconsistent config: a
   wrong version, an enum value outside its range, periodic sides that do not
   come in pairs, a side condition the step does not implement (see enum
   lbr_bc), fewer than 4 level-0 cells per side,
   finest-level indices beyond 2^28, rho_ref, d_wr or d_wv not positive,
   omega_b outside (0, 2), a viscosity that is not positive and finite, a
   negative or non-finite band of a level in use, or any other non-finite
   parameter. */
int lbr_create(const lbr_config* cfg, lbr_ctx** out);

/* Wall geometry (Section 2.3: surface segments in 2D): n_bodies closed
   polylines, counter-clockwise (fluid on the right), given as consecutive
   (x, y) pairs without repeating the first point; n_pts[b] >= 3.  With a
   non-zero lbr_config.alpha_deg each point is first turned by -alpha_deg
   about alpha_pivot (x' = p + R(-alpha)(x - p), one rounding per product and
   per sum).  The arrays are copied.
   Must be called before lbr_build (it may be called with n_bodies = 0).
   Errors: LBR_ERR_GEOMETRY for fewer than 3 points, a non-finite point or a
   body whose signed area is not positive (clockwise); LBR_ERR_STATE after
   lbr_build. */
int lbr_set_geometry(lbr_ctx* ctx, int32_t n_bodies, const int32_t* n_pts, const double* xy);

/* Number of doubles per record of a precomputed cut-link list: gi, gj, IW
   (x, y), normal (x, y), d_WB, body, q[1..8] (-1: not cut).  The same
   quantities as the wall records of lbr_read_wall, in the same units. */
#define LBR_CUT_STRIDE 16

/* Precomputed link-wise wall data of one level (Section 2.1: the
   preprocessor's geometry and cut-link list; Section 2.3: per boundary node B
   the wall point IW, the unit normal into the fluid, the distance d_WB and the
   wall fraction q of every cut link).  rec holds n records of LBR_CUT_STRIDE
   doubles, row-major:
     gi, gj      the node's cell in level-l lattice indices (integral values);
     IW, normal  in level-l lattice units, |normal| = 1 within 1e-6;
     d_WB        >= 0, level-l lattice units;
     body        index of a body of lbr_set_geometry, or -1 / -2 for the
                 lower / upper wall side of level 0;
     q[o]        for link o = 1..8, c_1..c_8 = (1,0), (-1,0), (0,1), (0,-1),
                 (1,1), (-1,-1), (1,-1), (-1,1): the fraction of the link
                 B -> B + c_o that lies in the fluid, in (0, 1], or exactly -1
                 where the link is not cut; at least one link per record is
                 cut.
   lbr_build then takes these nodes for level l instead of intersecting the
   links with the polylines; the cell types, the wall-distance field and the
   surface segments of Cp and Cf still come from the polylines.  The records
   are in the frame of the grid: with a non-zero alpha_deg they describe the
   turned bodies.  The
   reference-point stencils are derived from IW and the normal as for
   generated nodes.  Call after lbr_create and before lbr_build; a second call
   for a level replaces its list, n = 0 withdraws it.  The records are copied.
   Errors: LBR_ERR_INVALID_ARG for a level outside the config's levels, n < 0,
   rec NULL with n > 0, or a record that breaks the ranges above (the message
   names it); LBR_ERR_STATE after lbr_build.  lbr_build returns
   LBR_ERR_GEOMETRY when a node is not an owned fluid cell of its level or
   lies next to a level interface, a cell is listed twice, a body index names
   no body, a reference-point stencil reaches a cell that the level does not
   own, or a link from an owned
   fluid cell into a solid cell (or through a wall side of level 0) is not
   listed as cut: the step would otherwise stream from a solid cell. */
int lbr_set_cut_links(lbr_ctx* ctx, int32_t level, int64_t n, const double* rec);

/* The lists of lbr_set_cut_links for any number of levels, read from a text
   file (a case file of an external preprocessor).  Format: '#' starts a
   comment to the end of its line; tokens are separated by white space; the
   first two tokens are "lbr-cut-links 1"; then blocks of "level <l> <n>"
   followed by n x LBR_CUT_STRIDE numbers (strtod syntax; 17 significant
   digits round-trip a double).  Levels not named keep generated cut links.
   Errors: LBR_ERR_IO when the file cannot be read; LBR_ERR_INVALID_ARG for a
   malformed file (wrong header, a bad token, a truncated block, a level
   listed twice) or a record out of range, with nothing set; LBR_ERR_STATE
   after lbr_build. */
int lbr_load_cut_links(lbr_ctx* ctx, const char* path);

/* Builds the multilevel grid, the cut-link list with wall fractions q, the
   wall records (IW, normal, R-stencil weights), the FP64 wall-distance field,
   and allocates device state (Sections 2.1 and 2.3).  Initialises every level
   to the uniform reference state.  Errors: LBR_ERR_GEOMETRY when a refined
   level reaches the domain edge or an interface comes too close to a body or
   to another interface; LBR_ERR_INVALID_ARG when a level's storage box (its
   cells rounded up to whole tiles) is too large for the 32-bit addressing of
   the step kernels: (9 cells + 2 pitch + 2) x 8 bytes must stay below 2 GiB,
   i.e. about 29.8M cells per level, and the box may span at most 2,097,088
   columns and 65,534 rows (15-bit tile indices); LBR_ERR_OOM; LBR_ERR_HIP. */
int lbr_build(lbr_ctx* ctx);

/* Level layout after lbr_build. */
int lbr_level_info(lbr_ctx* ctx, int32_t level, lbr_level_desc* out);

/* Equilibrium initialisation of one level from host arrays over its I/O box
   (row-major, ny x nx doubles).  NULL arrays take rho_ref, (u_ref, 0) and
   chi_init. */
int lbr_init_fields(lbr_ctx* ctx, int32_t level, const double* rho, const double* ux,
                    const double* uy, const double* chi);

/* Advances n coarse (level-0) steps: the recursive multilevel cycle of
   Section 2.1, in which level l takes 2^l sub-steps.  Asynchronous on the
   context's stream, unless the health check of the config is on: then the
   call waits for its scans at the end and returns LBR_ERR_DIVERGED (density
   not finite or not positive, or |u| > c_s, anywhere) or LBR_ERR_NEWTON (a
   non-finite friction velocity), with the first level and cell found in the
   message; the state is left as the failing steps made it. */
int lbr_advance(lbr_ctx* ctx, int64_t n_coarse_steps);

/* Waits for the context's stream. */
int lbr_synchronize(lbr_ctx* ctx);

/* Copies one field of one level into a host array over the level's I/O box
   (ny x nx doubles); cells that are not owned fluid read NaN (TYPE reads the
   cell type for every cell). */
int lbr_read_field(lbr_ctx* ctx, int32_t level, int32_t field, double* dst);

/* As lbr_read_field, into device memory: dst is a device array of at least
   capacity doubles (ny x nx of the level's I/O box, else LBR_ERR_INVALID_ARG),
   written asynchronously on the context's stream.  LBR_FIELD_DIST reads the
   distance as the step kernels hold it (FP64 in FP64 contexts, its FP32
   rounding otherwise). */
int lbr_read_field_device(lbr_ctx* ctx, int32_t level, int32_t field, double* dst, int64_t capacity);

/* Number of wall nodes on a level, and their records (LBR_WALL_STRIDE doubles
   each, in row-major cell order).  The records hold the wall model evaluated
   on the current state (steps 1-5 of the VN procedure, Section 2.3) and the
   surface coefficients Cp and Cf of eq. (29). */
int lbr_wall_count(lbr_ctx* ctx, int32_t level);
int lbr_read_wall(lbr_ctx* ctx, int32_t level, double* dst);

/* y+ of the reference point R, the boundary node B and the virtual node V of
   every wall node of a level (Section 3.1.3, Figure 6): u_tau y / nu with y
   the wall distance of each point (d_WR, d_WB, d_WV in lattice units of the
   level; d_WR = 1.75 with LBR_WALL_NISHIMURA) and u_tau from the wall model
   on the current state.  dst holds 3 doubles per wall node, in the order of
   lbr_read_wall; 0 for wall models without a wall function. */
int lbr_wall_yplus(lbr_ctx* ctx, int32_t level, double* dst);

/* Rake (Section 3.1.4, Figure 10): n points evenly spaced from (x0, y0) to
   (x1, y1) in the units of the geometry (n = 1: the first point).  Each
   point takes the values of the owned fluid cell of the finest level that
   contains it.  dst holds 5 doubles per point: level (-1 where no fluid cell
   contains the point: solid, outside, and the other four NaN), u_x / U,
   u_y / U, nu_t / nu = chi f_v1(chi) (0 for chi <= 0), rho. */
int lbr_rake(lbr_ctx* ctx, double x0, double y0, double x1, double y1, int32_t n, double* dst);

/* For callers that cannot allocate device memory (tight monitoring loops inside a
   run, harnesses that forbid hipMalloc or the allocator callbacks of the config):
   lbr_rake with no device allocation.  The gather indices and values of each
   level go through one static device scratch of 1 MiB per GPU, held until the
   process ends and shared by every context on that GPU; n may be at most
   LBR_RAKE_NOALLOC_MAX (else LBR_ERR_INVALID_ARG, nothing done).  Nothing in the
   scratch needs to start at zero (every call writes what it reads back), but
   calls that overlap on one GPU (contexts driven from different host threads)
   race on it.  dst and the results are those of lbr_rake, bit for bit; like
   lbr_rake the call waits for the context's stream. */
#define LBR_RAKE_NOALLOC_MAX 16384
int lbr_rake_noalloc(lbr_ctx* ctx, double x0, double y0, double x1, double y1, int32_t n, double* dst);

/* Surface Cp and sign-corrected Cf at the centroids of the segments of one
   body (eq. (30) and the interpolation described after it).  cp and cf hold
   n_pts[body] doubles each. */
int lbr_surface(lbr_ctx* ctx, int32_t body, double* cp, double* cf);

/* y+ of the virtual node V at the same segment centroids (the quantity of
   Section 3.1.3 and Figure 6 along the surface): u_tau d_WV / nu of each wall
   node (as in lbr_wall_yplus), interpolated to the centroids with the nodes and
   weights that lbr_surface uses for Cp and Cf.  yplus_v holds n_pts[body]
   doubles; 0 for wall models without a wall function.  Waits for the context's
   stream.  Errors: LBR_ERR_INVALID_ARG (no build, bad body, null output). */
int lbr_surface_yplus(lbr_ctx* ctx, int32_t body, double* yplus_v);

/* Integrated coefficients of eq. (30) for one body (body = -1: all bodies):
   out = {C_Df, C_Dp, C_D, C_L (pressure only, as in eq. (30)), C_F . e_y}.
   Sums are FP64 and deterministic. */
int lbr_forces(lbr_ctx* ctx, int32_t body, double out[5]);

/* Relative velocity change ||u(t) - u(t - n)||_2 / (n ||u(t)||_2) over all
   owned fluid cells weighted by cell area, since the previous call (the first
   call returns 1 and only records the state). */
int lbr_residual(lbr_ctx* ctx, double* residual);

/* Steps until lbr_residual (evaluated every check_every coarse steps) drops
   below tol or max_steps is reached; returns the steps taken and the last
   residual.  Returns LBR_ERR_NOT_CONVERGED (steps_done and residual still
   written) when max_steps is reached first, LBR_ERR_DIVERGED if the state
   becomes non-finite. */
int lbr_run_to_steady(lbr_ctx* ctx, double tol, int64_t max_steps, int64_t check_every,
                      int64_t* steps_done, double* residual);

/* Checkpoint of the whole solver state: both time levels of the populations,
   of rho, u and of chi on every level, the friction-velocity state of the wall
   nodes (the Newton start values of Section 2.3, step 3) and the coarse-step
   counter (start-up ramp), in one binary file at path, after a header that
   identifies the grid (per-level box, cell counts and a hash of the cell
   flags) and ends with a checksum of the data.  lbr_save waits for the
   context's queued work.  lbr_load needs a context built from the same case
   with the same storage (else LBR_ERR_INVALID_ARG, nothing changed); it
   verifies the whole file before touching the device state (LBR_ERR_IO for a
   missing, foreign, truncated or corrupted file) and restarts the residual
   monitor.  A run continued from a checkpoint is bit-identical to the
   uninterrupted run. */
int lbr_save(lbr_ctx* ctx, const char* path);
int lbr_load(lbr_ctx* ctx, const char* path);

/* Cell updates per coarse step: sum over levels of n_fluid * 2^l. */
int64_t lbr_lups_per_coarse_step(lbr_ctx* ctx);

/* enable != 0: after the start-up ramp, lbr_advance replays two coarse steps
   at a time from a HIP graph of the merged launch schedule; enable == 0:
   direct launches of the recursive cycle (Section 2.1), one k_step launch per
   level sub-step.  The merged schedule runs each sub-step of a level at least
   three below the finest inside the grid of the next launch of a finer level
   (the two touch disjoint state: the coarse step reads its parent, itself and
   its child, writes itself and the restriction into its parent), so a coarse
   step of an 8-level grid takes 195 launches instead of 255.  Every cell is
   computed by the same code from the same state as in the direct cycle: the
   results are bit-identical.  The default (NULL) stream cannot be captured:
   enabling the graph on a context created with stream NULL is
   LBR_ERR_INVALID_ARG. */
int lbr_use_graph(lbr_ctx* ctx, int32_t enable);

/* Tile shape of the step kernel.  A workgroup updates a tile of 64 x H cells
   (one 64-wide wavefront per row, H = 2, 4, 8 or 16 rows; 4 by default).  Every
   cell's result is a function of its stencil alone, so the fields are
   bit-identical for any choice.  lbr_tune times each height on every level
   with that level's first sub-step from the current state (trials launches
   each; the step's outputs are overwritten by the next real step and the wall
   nodes' Newton state is restored) and keeps the fastest, where a height other
   than 4 must beat 4 by 3 % (near-equal times swap from run to run); rows, if not NULL,
   receives n_levels heights.  lbr_set_tile_rows sets one level's height
   (level -1: all levels); other values of rows are LBR_ERR_INVALID_ARG. */
int lbr_tune(lbr_ctx* ctx, int32_t trials, int32_t* rows);

/* The launch schedule of two coarse steps of an n_levels grid (the table that
   lbr_use_graph replays; merge = 0: the direct recursive cycle), for
   inspection, with no device work: for every launch in order, the number m of
   level sub-steps it runs, then m pairs (level, sub-step 1 or 2; 0 on level
   0).  Writes at most cap values to out and returns the number the whole
   schedule needs (LBR_ERR_INVALID_ARG for n_levels outside 1..LBR_MAX_LEVELS). */
int32_t lbr_schedule(int32_t n_levels, int32_t merge, int32_t* out, int32_t cap);
int lbr_set_tile_rows(lbr_ctx* ctx, int32_t level, int32_t rows);

/* Average device time per launch of the step kernel over the last
   lbr_advance, in microseconds, from start / stop events attached to each
   dispatch (hipExtLaunchKernelGGL): out[0] all launches, out[1] the launches
   that step the finest level, out[2] those of level 0 alone, out[3] launches
   per coarse step.  After the start-up ramp the timed run uses the merged
   schedule of lbr_use_graph, launched directly (the graph is not replayed
   while timing).  Events go to the first 65,536 launches of a call only;
   out[3] counts every launch.  enable != 0 turns the timing on for the
   following lbr_advance calls; enable == 0 turns it off.  out may be NULL;
   it receives the figures of the last timed lbr_advance. */
int lbr_profile(lbr_ctx* ctx, int32_t enable, double out[4]);

/* Last error message of the context (never NULL). */
const char* lbr_last_error(const lbr_ctx* ctx);

/* Frees every device and host resource of the context (NULL is allowed). */
void lbr_destroy(lbr_ctx* ctx);

/* ---------------------------------------------------------------------------
   Batched sweep: several cases of one study advanced by shared launches.  The
   studies of Section 3 run one configuration at several angles of attack
   (Sections 3.1.1 and 3.2) and on several grids with different numbers of
   refinement levels (Section 3.1.3, Table 1); each case on its own fills
   only a fraction of the GPU at its coarse levels.  The cases are aligned on their finest level:
   virtual level v of the batch is level v - (lmax - L_k) of case k, so one
   super step advances case k by 2^(lmax - L_k) of its coarse steps and each
   launch of k_step covers the same virtual level of every case (one grid split
   into per-case parts).  The numbers each case computes are identical to
   advancing it alone.
   --------------------------------------------------------------------------- */
typedef struct lbr_batch lbr_batch;

/* Groups n distinct built contexts of the same storage precision on one device
   (a context listed twice, a NULL one or mixed precisions: LBR_ERR_INVALID_ARG).
   The batch launches on the first context's stream; the contexts' pending work
   is synchronised here.  Cases still inside a start-up ramp are refused
   (LBR_ERR_STATE).  The batch borrows the contexts (destroy the batch first)
   and allocates its launch tables through the first context's allocator.
   Returns 0 or a negative code; on failure *out may still hold a batch that
   carries the message (lbr_batch_last_error) and must be destroyed. */
int lbr_batch_create(int32_t n, lbr_ctx* const* cases, lbr_batch** out);

/* Enqueues n super steps on the batch stream (asynchronous).  Work already
   queued on the contexts' own streams runs first, and work queued there later
   waits for the super steps.  A case may also be advanced on its own between
   batch calls by an even number of coarse steps; after an odd number the
   batch refuses to run (LBR_ERR_STATE) because its launch tables address the
   other level-0 buffer. */
int lbr_batch_advance(lbr_batch* batch, int64_t n_super_steps);

/* Super steps until the residual of every case (lbr_residual, evaluated every
   check_every super steps) drops below tol, or max_super_steps.  A case whose
   residual is below tol leaves the launches, so the others run on without its
   cell updates; at return the batch covers every case again.  steps_done[k]
   receives the coarse steps case k took and residual[k] its last residual
   (arrays of n entries, either may be NULL).  Returns LBR_ERR_NOT_CONVERGED
   (both arrays still written) when some case has not converged after
   max_super_steps, LBR_ERR_DIVERGED if a case's state becomes non-finite. */
int lbr_batch_run_to_steady(lbr_batch* batch, double tol, int64_t max_super_steps, int64_t check_every,
                            int64_t* steps_done, double* residual);

/* Replays two super steps from one HIP graph (enable != 0) or launches
   directly (enable == 0).  As lbr_use_graph, it needs the batch's stream (its
   first case's) not to be the default stream. */
int lbr_batch_use_graph(lbr_batch* batch, int32_t enable);

/* As lbr_tune for the batch: every virtual level is timed with the parts of all
   cases in one launch and the fastest height is set on the corresponding level
   of every case (rows: lmax entries, may be NULL); the launch tables are
   rebuilt. */
int lbr_batch_tune(lbr_batch* batch, int32_t trials, int32_t* rows);

/* Persistent mode of a batch: every table of the merged schedule (one or two
   super steps) runs as a single cooperative grid of co-resident workgroups,
   which take the blocks of each launch in turn and meet at a grid-wide
   barrier where the launch boundaries were (workgroups grouped by XCD: one
   L2 writeback per XCD, then every workgroup discards its stale lines).
   Results are bit-identical to the launches (64 x 4 tiles everywhere in this
   mode).  On MI355X it is slower than the launches replayed from a graph (a
   barrier across 2,048 workgroups costs more than a launch boundary); it is
   off by default.  Every level of every case must hold one
   population format (no mixed storage).  Each advance waits for its grid and
   reports a barrier wait that ran out (LBR_ERR_HIP; only a grid that is not
   co-resident can reach it).  Profiling (lbr_batch_profile) times the
   launches of the merged schedule and is refused in this mode.  Errors:
   LBR_ERR_INVALID_ARG for mixed formats, LBR_ERR_STATE while profiling. */
int lbr_batch_use_persistent(lbr_batch* batch, int32_t enable);

/* As lbr_profile, for the batched launches: out[0] all launches, out[1] the
   launches of the finest virtual level, out[2] virtual level 0, out[3]
   launches per super step. */
int lbr_batch_profile(lbr_batch* batch, int32_t enable, double out[4]);

/* Waits for the batch stream; afterwards every per-context call (fields,
   forces, residual) sees the advanced state. */
int lbr_batch_synchronize(lbr_batch* batch);

/* Coarse steps case k takes per super step (2^(lmax - L_k), with lmax the
   most levels of any case). */
int64_t lbr_batch_steps_per_super_step(const lbr_batch* batch, int32_t k);

/* Cell updates of all cases per super step. */
int64_t lbr_batch_lups_per_super_step(lbr_batch* batch);

const char* lbr_batch_last_error(const lbr_batch* batch);
void lbr_batch_destroy(lbr_batch* batch);

#ifdef __cplusplus
}
#endif
#endif
