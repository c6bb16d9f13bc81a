// Internal declarations of liblbr: device data layout, kernel argument blocks
// and the launchers implemented in lbr_kernels.hip.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbr {

// Cell flag byte: bits 0-2 hold the cell type, the others mark cells that
// need more than the plain interior update.
enum : uint8_t {
    T_INACTIVE = 0, T_FLUID = 1, T_SOLID = 2, T_GHOST = 3, T_COVERED = 4,
    F_TYPE = 7,
    F_WALL = 8,         // boundary node B with cut links
    F_IFACE = 16,       // coarse cell fed by coalescence of the finer level
    F_NEARGHOST = 32,   // fine cell with a ghost neighbour
    F_EDGE = 64,        // level-0 cell on the domain edge
    F_COVB = 128,       // covered cell next to an owned cell (restriction target)
};

constexpr int WALL_PER_BLOCK = 16;   // wall nodes per k_step workgroup
constexpr int TILE_X = 64;   // one wavefront per tile row
// tile heights (wavefronts per workgroup) k_step is built for; the host tunes
// one per level
constexpr int NTY = 4;
constexpr int TILE_YS[NTY] = {2, 4, 8, 16};
constexpr int TILE_Y_DEFAULT = 1;   // index of 4 rows
constexpr int TILE_Y_MAX = 16;      // level boxes hold whole tiles of any height
constexpr int MAX_STENCIL = 16;
constexpr int ROWS_PER_GROUP = 4;   // wave rows per workgroup

// Geometry of a level's storage box: global cell (gx, gy) of the level lives
// at local (gx - gx0, gy - gy0), linear index ly * pitch + lx; every field is
// a set of planes of `plane` elements.
struct Box {
    int gx0, gy0, pitch, ny;
    long plane;
};

// Boundary-condition block of level 0 (all levels carry it; only level 0 has
// F_EDGE cells).
// Absorbing layer along the far-field sides of level 0 (width 0: none).
struct Absorber {
    double width, strength;          // in level-0 cells; largest relaxation rate
    int sides;                       // bit k: side k (x-lo, x-hi, y-lo, y-hi) is a far field
    double drho, ux;                 // target state: rho_ref - 1 and the free-stream velocity
};

struct Domain {
    int nxd, nyd;          // domain size in cells of this level
    int bc[4];
    int periodic_x;
    int outlet;            // LBR_OUTLET_*: rule for the unknown outlet populations
};

// Link-wise wall data of one level (Sections 2.1 and 2.3).
struct WallData {
    int nb;
    const int32_t* cell;             // storage index of each boundary node B
    const double* geo;               // [nb][6] IW (x, y), n (x, y), d_WB, body
    const int32_t* st_cell;          // [nb][MAX_STENCIL] storage index of R-stencil cells (-1 unused)
    const double* st_wr;             // [nb][MAX_STENCIL] IDW weights for rho_R
    const double* st_wu;             // [nb][MAX_STENCIL] LSQ weights for u_R
    const double* q;                 // [nb][8] wall fraction of links 1..8 (-1: not cut)
    double d_wr, d_wv, uw_lo[2], uw_hi[2];
    int model;
};

template <class ST, class CT>
struct StepArgs {
    const ST* fsrc;  ST* fdst;       // 9 population planes (shifted by w_i)
    const CT* msrc;  CT* mdst;       // 3 planes: rho, ux, uy
    const CT* csrc;  CT* cdst;       // chi = nu~ / nu
    const CT* dist;                  // wall distance (level lattice units), in CT
    const uint8_t* flag;
    const uint32_t* lmask;           // per cell: bit i, source c - c_i is owned fluid;
                                     // bit 16 + i, source is a ghost; bit 31, lower-left
                                     // child of a covered coarse cell next to coarse fluid
    const uint32_t* tiles;           // active 64 x ty tiles, (tx | ghost << 15 | ty << 16 | restriction << 31)
    int ntiles;
    const int32_t* edge;             // level-0 domain-edge cells that are not wall nodes
    int nedge;
    Box box;
    Domain dom;
    CT nu, fx, fy, omega_b, u_in, chi_in, rho_out;
    CT mu_cap;                       // SA face diffusivity limit (+inf: none)
    int sa_mode, bb_halfway, frozen;
    int substep;                     // 1 or 2 within the parent's step (0 on level 0)
    int pad;                         // spare elements before and after every field array
                                     // of the level (one row plus one cell)
    int ty;                          // tile height of the tile list (2, 4, 8 or 16 rows)
    int wall_blocks, tile_blocks;    // k_step grid: wall-node blocks of WALL_PER_BLOCK nodes
                                     // (a multiple of 8 blocks),
                                     // tile blocks (a multiple of 8), then edge-cell blocks
    Absorber sp;                     // absorbing layer (level 0 only; width 0 elsewhere)
    CT dsh[9];                       // 16-bit storage holds s_i - dsh[i] (0, or the free-stream shift)
    const void* fcoarse; Box cbox;   // parent level populations (ghost transfer), stored as
    int cst;                         // Prec cst (mixed storage: FP32 or FP16, else as ST)
    const CT* cmac;  const CT* cchi; // parent level rho, u and chi of the current parent step
    CT* rmac;        CT* rchi;       // parent level buffers of the next parent step (restriction)
    const void* ffine; Box fbox;     // child level populations (coalescence), stored as
    int fst;                         // Prec fst
    int sst;                         // Prec of this level's own populations (selects the
                                     // instantiation in a mixed launch)
    WallData wall;                   // boundary nodes of this level (k_boundary)
    double* wstate;                  // [nb][8] u_tau, u_Rt (x, y), rho_W, u_W (x, y), spare
};

// Wall model evaluated on the current state for output (does not touch the
// friction velocities the next step starts its Newton iteration from).
template <class CT>
struct WallArgs {
    WallData wall;
    const CT* mac;
    const double* guess;             // [nb][8], u_tau in column 0
    double* out;                     // [nb][8]
    long plane;
    double nu;
};

struct FillArgs {
    int n; const int32_t* list;      // ghost cells of the fine level (storage index)
    Box fbox, cbox;
    const void* cmac; const void* cchi;  // coarse current
    void* fmac0; void* fmac1; void* fchi0; void* fchi1;
};

struct RestrictArgs {
    int n; const int32_t* list;      // F_COVB cells of the coarse level
    Box fbox, cbox;
    const void* fmac; const void* fchi;  // fine current
    void* cmac; void* cchi;              // coarse current
};

struct InitArgs {
    int n; const int32_t* list;      // owned fluid cells (storage index)
    const double* rho; const double* ux; const double* uy; const double* chi;  // per listed cell
    void* f; void* mac; void* chi_a; void* chi_b;
    long plane;
    double nu, fx, fy, omega_b;
    int pitch, gx0, gy0, nxd, nyd;   // storage box origin and domain size (absorbing layer)
    Absorber sp;
    double dsh[9];                   // 16-bit storage holds s_i - dsh[i]
};

struct SurfaceArgs {
    int nseg;
    const double* seg;               // [nseg][6]: t (x, y), n (x, y), ds, unused
    const int32_t* near;             // [nseg][2] wall-node indices (-1 unused)
    const double* wgt;               // [nseg][2] IDW weights
    const double* bstate;            // wall-node state [nb][8]
    const void* bw;                  // [nb][4] (CT)
    double u_ref, rho_ref;
    double* cp; double* cf;          // per segment
    double* partial;                 // [nblocks][5]
};

// launchers (lbr_kernels.hip); `prec` selects the storage/compute pair.
// P_MIXED is never a level's storage: it tags a batched launch whose parts are
// FP32- and FP16-stored levels of mixed-storage cases.
enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3, P_MIXED = 4 };

hipError_t launch_geometry(int nx, int ny, int gx0, int gy0, double scale, int nbody,
                           const int* npts_off, const double* poly, int solid,
                           double* dist, uint8_t* inside, hipStream_t s);
// Optional events recorded by the dispatch itself at kernel start and end.
struct Timing {
    hipEvent_t start = nullptr, stop = nullptr;
};
hipError_t launch_step(Prec p, const void* args, hipStream_t s, const Timing& tm = Timing{});
// parts: device array of nparts StepArgs<ST, CT> of the precision p; start: device
// array of the first block of each part (multiples of 8); nblocks_total: grid size
hipError_t launch_step_batch(Prec p, const void* parts, const int* start, int nparts, int nblocks_total, int ty,
                             hipStream_t s, const Timing& tm = Timing{});
// Persistent batched run (lbr_batch_use_persistent): the launches of a table
// as sub-launches of one cooperative grid, separated by a grid-wide barrier.
// part: index of the launch's first StepArgs in the parts array (all of one
// format); part0: index of its first part start; nparts; nblocks.
struct PLaunch { int part, part0, nparts, nblocks; };
constexpr int PERSISTENT_TY = 4;                 // tile height of every sub-launch
// bar: BAR_WORDS device words, zero before the first grid (grid and per-XCD
// barrier counters; word 2 is a flag set when a barrier wait ran out of its spin
// limit, which only a grid that is not co-resident reaches)
constexpr int BAR_XCC = 16;                      // XCC ids are four bits
constexpr int BAR_STRIDE = 32;                   // one 128-byte line per counter group
constexpr int BAR_WORDS = BAR_STRIDE * (BAR_XCC + 1);
hipError_t launch_step_persistent(Prec p, const void* parts, const int* start, const PLaunch* launches, int nlaunches,
                                  int grid, unsigned* bar, hipStream_t s);
// largest co-resident grid of the persistent kernel of format p (a multiple of 8)
hipError_t persistent_grid(Prec p, int* grid);
hipError_t launch_wall(Prec p, const void* args, hipStream_t s);
hipError_t launch_fill(Prec p, const FillArgs& a, hipStream_t s);
hipError_t launch_restrict(Prec p, const RestrictArgs& a, hipStream_t s);
hipError_t launch_init(Prec p, const InitArgs& a, hipStream_t s);
hipError_t launch_surface(Prec p, const SurfaceArgs& a, int nblocks, hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int nblocks, double* out, hipStream_t s);
// One field over a level's I/O box into device memory (field codes of lbr.h)
struct FieldArgs {
    const void* src;                 // the rho / u_x / u_y or chi plane (CT)
    const void* dist;                // wall distance (CT)
    const uint8_t* flag;
    long pitch;
    int ox, oy, bnx, bny;            // I/O box origin in the storage box, and its size
    int field;
    double nu;
    double* out;                     // [bny][bnx]
};
hipError_t launch_field(Prec p, const FieldArgs& a, hipStream_t s);
// dst[k] = src[idx[k]] for the macroscopic / chi planes (CT of precision p)
hipError_t launch_gather(Prec p, const void* src, const int64_t* idx, int n, double* dst, hipStream_t s);
hipError_t launch_to_double(Prec p, const void* src, double* dst, long n, hipStream_t s);
// Health scans (lbr_config::health_every): out[0] |= 1 when a listed cell's density is
// not finite or not positive or |u| > c_s, |= 2 when a wall node's friction velocity
// is not finite; out[1], out[2]: level and cell (or wall node) of one failure,
// out[3]: failing cells counted.  launch_health_reset clears out[0..3].
hipError_t launch_health_reset(int* out, hipStream_t s);
hipError_t launch_health(Prec p, const void* mac, const int32_t* list, int n, long plane, int level, int* out,
                         hipStream_t s);
hipError_t launch_health_wall(const double* bstate, int nb, int level, int* out, hipStream_t s);
hipError_t launch_residual(Prec p, const void* mac, double* snap, const int32_t* list, int n,
                           long plane, double area, double* partial, int nblocks, hipStream_t s);

// Static device scratch of the allocation-free entry point (lbr_rake_noalloc):
// one array of NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.
// noalloc_scratch() returns its device address on the current device (looked up
// once per device); host code uses that address, never the array's name.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(1) << 20;
hipError_t noalloc_scratch(void** ptr);

}  // namespace lbr
