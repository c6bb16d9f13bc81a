// Host side of liblbr: grid construction, wall records, the recursive
// multilevel schedule and the C entry points declared in include/lbr.h.
#include "lbr.h"
#include "lbr_impl.h"

#include <algorithm>
#include <cctype>
#include <cstdlib>
#include <new>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace lbr;

namespace {

constexpr int G = 2;   // guard ring of every storage box
// the restriction reads each 2 x 2 block from the LDS rows and columns of its
// lower-left cell and the next ones: block anchors must sit at even local
// coordinates (even box origins, even tile heights)
static_assert(G % 2 == 0, "storage boxes keep 2 x 2 blocks aligned");
static_assert(TILE_X % 2 == 0 && TILE_YS[0] % 2 == 0 && TILE_YS[1] % 2 == 0 && TILE_YS[2] % 2 == 0 &&
                  TILE_YS[3] % 2 == 0, "tiles hold whole 2 x 2 blocks");
// a timed advance attaches start / stop events to its first launches only
constexpr size_t MAX_TIMED_LAUNCHES = 1 << 16;
constexpr int CXH[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int CYH[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
constexpr double KAPPA_H = 0.41;

struct Node {
    int gi, gj, body;
    long cell;
    double q[9];
    double iw[2], nrm[2], dwb;
};

struct Level {
    int l = 0;
    Prec st = P_F32;                 // population storage of this level
    size_t ssize = 4;
    Box box{};
    int bx0 = 0, by0 = 0, bnx = 0, bny = 0;   // I/O box
    double scale = 1, nu = 0, fx = 0, fy = 0;
    std::vector<uint8_t> flag;
    std::vector<double> dbody, d;
    std::vector<uint8_t> inside;
    std::vector<int32_t> bidx;
    std::vector<Node> nodes;
    std::vector<uint32_t> rows[NTY]; // k_step tiles of each height (x, y, ghost and restriction bits)
    int ty = TILE_Y_DEFAULT;         // index of the tile height k_step uses on this level
    std::vector<int32_t> owned, ghosts, covb, edge;
    int64_t n_fluid = 0, n_ghost = 0, n_cut = 0;
    // device
    void* f[2] = {nullptr, nullptr};
    void* mac[2] = {nullptr, nullptr};
    void* chi[2] = {nullptr, nullptr};
    void* dist_dev = nullptr;     // wall distance for the step kernels, in their arithmetic precision
    uint8_t* flag_dev = nullptr;
    uint32_t* rows_dev[NTY] = {};
    uint32_t* lmask_dev = nullptr;
    int32_t* ghosts_dev = nullptr;
    int32_t* covb_dev = nullptr;
    int32_t* owned_dev = nullptr;
    int32_t* edge_dev = nullptr;
    double* bq = nullptr;
    int32_t* bcell = nullptr;
    double* bgeo = nullptr;
    int32_t* st_cell = nullptr;
    double* st_wr = nullptr;
    double* st_wu = nullptr;
    double* bstate = nullptr;   // friction velocity state carried between steps
    double* bout = nullptr;     // wall model on the current state (output)
    double* snap = nullptr;
    int cur = 0;
    size_t bytes = 0;

    long idx(int gx, int gy) const {
        const int lx = gx - box.gx0, ly = gy - box.gy0;
        if (lx < 0 || ly < 0 || lx >= box.pitch || ly >= box.ny) return -1;
        return (long)ly * box.pitch + lx;
    }
    uint8_t type_at(int gx, int gy) const {
        const long c = idx(gx, gy);
        return c < 0 ? T_INACTIVE : (flag[c] & F_TYPE);
    }
};

struct SurfaceBody {
    int nseg = 0;
    double* seg = nullptr;
    int32_t* near = nullptr;
    double* wgt = nullptr;
    std::vector<int32_t> near_h;   // host copies of near and wgt (per-segment y+)
    std::vector<double> wgt_h;
};

}  // namespace

struct lbr_ctx {
    lbr_config cfg{};
    std::string err = "";
    hipStream_t stream = nullptr;
    Prec prec = P_F32;
    size_t ssize = 4, csize = 4;
    double u_ref = 0, nu0 = 0;
    double dsh[9] = {};             // storage shift of 16-bit populations (per direction)
    std::vector<double> polyflat;   // level-0 lattice coordinates
    std::vector<int> npts, off;
    double wall_lat[2] = {0, 0};
    std::vector<Level> lv;
    // precomputed cut-link lists (lbr_set_cut_links), LBR_CUT_STRIDE doubles per
    // node; an empty list: the level's cut links come from the polylines
    std::vector<double> cut_in[LBR_MAX_LEVELS];
    int wall_level = -1;
    std::vector<SurfaceBody> surf;
    double* surf_cp = nullptr;
    double* surf_cf = nullptr;
    double* partial = nullptr;
    int partial_n = 0;
    void* scratch = nullptr;       // device address of the static scratch (lbr_rake_noalloc)
    int* health = nullptr;         // device result of the health scans: failure bits, level, index, count
    bool built = false;
    std::vector<void*> allocs;
    int64_t resid_steps = 0;
    bool resid_init = false;
    // after the start-up ramp, graph replay and timed runs go through a batch of
    // this one case (the merged launch schedule)
    bool use_graph = false;
    lbr_batch* self = nullptr;
    bool self_dirty = false;       // tile heights changed since its tables were built
    int64_t step_count = 0;        // coarse steps completed (start-up ramp)
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    int64_t prof_launches = 0;     // launches of the last timed call (timed or not)
    double prof_out[4] = {0, 0, 0, 0};
};

namespace {

int set_err(lbr_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

// Population storage of level l: the configured format, or with mixed storage
// FP32 on the two finest levels and FP16 below (FP32 arithmetic throughout).
Prec level_storage(const lbr_ctx* c, int l);

#define HIPCHK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_err(ctx, LBR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

void* dalloc(lbr_ctx* c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (c->cfg.alloc_fn) {
        p = c->cfg.alloc_fn(bytes, c->cfg.alloc_user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->allocs.push_back(p);
    return p;
}

// Allocation with `pad` spare elements on both ends; returns the shifted base.
void* dalloc_padded(lbr_ctx* c, size_t elems, size_t esize, size_t pad) {
    char* raw = static_cast<char*>(dalloc(c, (elems + 2 * pad) * esize));
    return raw ? raw + pad * esize : nullptr;
}

void dfree(lbr_ctx* c, void* p) {
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it == c->allocs.end()) return;
    c->allocs.erase(it);
    if (c->cfg.free_fn) c->cfg.free_fn(p, c->cfg.alloc_user);
    else (void)hipFree(p);
}

template <class T>
int upload(lbr_ctx* c, T** dst, const std::vector<T>& v, size_t* acct) {
    size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    *dst = static_cast<T*>(dalloc(c, bytes));
    if (!*dst) return set_err(c, LBR_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    if (acct) *acct += bytes;
    if (!v.empty())
        HIPCHK(c, hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return 0;
}

double seg_closest(double px, double py, double ax, double ay, double bx, double by, double* qx,
                   double* qy) {
    const double ex = bx - ax, ey = by - ay, l2 = ex * ex + ey * ey;
    double t = l2 > 0 ? ((px - ax) * ex + (py - ay) * ey) / l2 : 0.0;
    t = std::min(1.0, std::max(0.0, t));
    *qx = ax + t * ex;
    *qy = ay + t * ey;
    return std::hypot(px - *qx, py - *qy);
}

// parameter t in (0, 1] where p + t e crosses segment ab, or -1
double crossing(double px, double py, double ex, double ey, double ax, double ay, double bx,
                double by) {
    const double sx = bx - ax, sy = by - ay;
    const double den = ex * sy - ey * sx;
    if (den == 0.0) return -1.0;
    const double t = ((ax - px) * sy - (ay - py) * sx) / den;
    const double u = ((ax - px) * ey - (ay - py) * ex) / den;
    return (t > 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0) ? t : -1.0;
}

// Segments of all bodies bucketed on a uniform grid (in lattice units of one level).
struct Buckets {
    double x0 = 0, y0 = 0, h = 4;
    int nx = 0, ny = 0;
    std::vector<std::vector<int>> cell;   // segment ids
    void build(const std::vector<double>& seg, double scale, double pad) {
        const size_t ns = seg.size() / 5;
        double xlo = 1e300, ylo = 1e300, xhi = -1e300, yhi = -1e300;
        for (size_t k = 0; k < ns; ++k) {
            for (int e = 0; e < 2; ++e) {
                xlo = std::min(xlo, seg[5 * k + 2 * e] * scale);
                xhi = std::max(xhi, seg[5 * k + 2 * e] * scale);
                ylo = std::min(ylo, seg[5 * k + 2 * e + 1] * scale);
                yhi = std::max(yhi, seg[5 * k + 2 * e + 1] * scale);
            }
        }
        if (ns == 0) { nx = ny = 0; return; }
        x0 = xlo - pad - h; y0 = ylo - pad - h;
        nx = (int)((xhi - xlo + 2 * pad) / h) + 3;
        ny = (int)((yhi - ylo + 2 * pad) / h) + 3;
        cell.assign((size_t)nx * ny, {});
        for (size_t k = 0; k < ns; ++k) {
            const double ax = seg[5 * k] * scale, ay = seg[5 * k + 1] * scale;
            const double bx = seg[5 * k + 2] * scale, by = seg[5 * k + 3] * scale;
            const int i0 = (int)((std::min(ax, bx) - pad - x0) / h), i1 = (int)((std::max(ax, bx) + pad - x0) / h);
            const int j0 = (int)((std::min(ay, by) - pad - y0) / h), j1 = (int)((std::max(ay, by) + pad - y0) / h);
            for (int j = std::max(0, j0); j <= std::min(ny - 1, j1); ++j)
                for (int i = std::max(0, i0); i <= std::min(nx - 1, i1); ++i)
                    cell[(size_t)j * nx + i].push_back((int)k);
        }
    }
    const std::vector<int>* at(double x, double y) const {
        static const std::vector<int> none;
        const int i = (int)std::floor((x - x0) / h), j = (int)std::floor((y - y0) / h);
        if (nx == 0 || i < 0 || j < 0 || i >= nx || j >= ny) return &none;
        return &cell[(size_t)j * nx + i];
    }
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Runs the FP64 geometry kernel over a level's storage box.
int level_geometry(lbr_ctx* c, Level& L, const double* poly_dev, const int* off_dev) {
    const long n = (long)L.box.pitch * L.box.ny;
    double* dd = static_cast<double*>(dalloc(c, n * sizeof(double)));
    uint8_t* id = static_cast<uint8_t*>(dalloc(c, n));
    if (!dd || !id) return set_err(c, LBR_ERR_OOM, "geometry scratch allocation failed");
    HIPCHK(c, launch_geometry(L.box.pitch, L.box.ny, L.box.gx0, L.box.gy0, L.scale,
                              (int)c->npts.size(), off_dev, poly_dev,
                              c->cfg.body_mode == LBR_BODY_SOLID, dd, id, c->stream));
    L.dbody.resize(n);
    L.inside.resize(n);
    HIPCHK(c, hipMemcpyAsync(L.dbody.data(), dd, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(L.inside.data(), id, n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, dd);
    dfree(c, id);
    return 0;
}

void set_box(Level& L, int gx0, int gy0, int nx, int ny) {
    L.box.gx0 = gx0;
    L.box.gy0 = gy0;
    L.box.pitch = round_up(nx, TILE_X);
    L.box.ny = round_up(ny, TILE_Y_MAX);
    L.box.plane = (long)L.box.pitch * L.box.ny;
    L.flag.assign(L.box.plane, T_INACTIVE);
}

int build_levels(lbr_ctx* c, const double* poly_dev, const int* off_dev) {
    const lbr_config& cfg = c->cfg;
    const int nl = cfg.n_levels;
    c->lv.assign(nl, Level());
    for (int l = 0; l < nl; ++l) {
        Level& L = c->lv[l];
        L.l = l;
        L.scale = std::ldexp(1.0, l);
        L.nu = c->nu0 * L.scale;
        L.fx = cfg.force[0] / L.scale;
        L.fy = cfg.force[1] / L.scale;
        if (l == 0) {
            set_box(L, -G, -G, cfg.nx0 + 2 * G, cfg.ny0 + 2 * G);
            if (int r = level_geometry(c, L, poly_dev, off_dev)) return r;
            for (int gy = 0; gy < cfg.ny0; ++gy)
                for (int gx = 0; gx < cfg.nx0; ++gx) {
                    const long k = L.idx(gx, gy);
                    L.flag[k] = L.inside[k] ? T_SOLID : T_FLUID;
                }
            continue;
        }
        Level& P = c->lv[l - 1];
        const double band = cfg.band[l] / cfg.dx0 * P.scale;
        const long np = P.box.plane;
        bool any = false;
        for (long k = 0; k < np; ++k) {
            const int t = P.flag[k] & F_TYPE;
            if ((t == T_FLUID || t == T_SOLID) && P.dbody[k] < band) {
                P.flag[k] = T_COVERED;
                any = true;
            }
        }
        if (!any) return set_err(c, LBR_ERR_GEOMETRY, "level %d: no cells refined", l);
        int lo_x = 1 << 30, lo_y = 1 << 30, hi_x = -(1 << 30), hi_y = -(1 << 30);
        for (long k = 0; k < np; ++k) {
            const int gx = (int)(k % P.box.pitch) + P.box.gx0, gy = (int)(k / P.box.pitch) + P.box.gy0;
            const int t = P.flag[k] & F_TYPE;
            bool near_cov = false, near_fluid = false;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int tn = P.type_at(gx + dx, gy + dy);
                    near_cov |= tn == T_COVERED;
                    near_fluid |= tn == T_FLUID;
                }
            if (t == T_FLUID && near_cov) P.flag[k] |= F_IFACE;
            if (t == T_COVERED && near_fluid) P.flag[k] |= F_COVB;
            if (t == T_COVERED || (P.flag[k] & F_IFACE)) {
                lo_x = std::min(lo_x, gx); hi_x = std::max(hi_x, gx);
                lo_y = std::min(lo_y, gy); hi_y = std::max(hi_y, gy);
            }
        }
        set_box(L, 2 * lo_x - G, 2 * lo_y - G, 2 * (hi_x - lo_x + 1) + 2 * G,
                2 * (hi_y - lo_y + 1) + 2 * G);
        if (int r = level_geometry(c, L, poly_dev, off_dev)) return r;
        for (long k = 0; k < L.box.plane; ++k) {
            const int gx = (int)(k % L.box.pitch) + L.box.gx0, gy = (int)(k / L.box.pitch) + L.box.gy0;
            const long pk = P.idx(gx >> 1, gy >> 1);
            if (pk < 0) continue;
            if ((P.flag[pk] & F_TYPE) == T_COVERED) L.flag[k] = L.inside[k] ? T_SOLID : T_FLUID;
            else if (P.flag[pk] & F_IFACE) L.flag[k] = T_GHOST;
        }
    }
    return 0;
}

// Clearances the transfer needs between interfaces, bodies and the domain edge.
int check_levels(lbr_ctx* c) {
    const int nl = (int)c->lv.size();
    for (int l = 0; l < nl; ++l) {
        const Level& L = c->lv[l];
        for (long k = 0; k < L.box.plane; ++k) {
            const int t = L.flag[k] & F_TYPE;
            if (t != T_COVERED && t != T_GHOST && !(l > 0 && t != T_INACTIVE)) continue;
            const int gx = (int)(k % L.box.pitch) + L.box.gx0, gy = (int)(k / L.box.pitch) + L.box.gy0;
            if (l > 0 && t != T_INACTIVE) {
                const int nxd = c->cfg.nx0 << l, nyd = c->cfg.ny0 << l;
                if (gx < 4 || gy < 4 || gx >= nxd - 4 || gy >= nyd - 4)
                    return set_err(c, LBR_ERR_GEOMETRY, "level %d reaches the domain edge", l);
            }
            if (t == T_COVERED) {
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        const int tn = L.type_at(gx + dx, gy + dy);
                        if (tn != T_FLUID && tn != T_COVERED)
                            return set_err(c, LBR_ERR_GEOMETRY,
                                           "level %d: refined region too close to a body or edge", l);
                    }
                if ((L.flag[k] & F_COVB) && l + 1 < nl) {
                    const Level& F = c->lv[l + 1];
                    for (int dy = -3; dy <= 4; ++dy)
                        for (int dx = -3; dx <= 4; ++dx) {
                            const int tn = F.type_at(2 * gx + dx, 2 * gy + dy);
                            if (tn == T_SOLID || tn == T_COVERED)
                                return set_err(c, LBR_ERR_GEOMETRY,
                                               "level %d: interface too close to a body or a finer "
                                               "interface", l + 1);
                        }
                }
            }
            if (t == T_GHOST) {
                for (int dy = -4; dy <= 4; ++dy)
                    for (int dx = -4; dx <= 4; ++dx) {
                        const int tn = L.type_at(gx + dx, gy + dy);
                        if (tn == T_SOLID || tn == T_COVERED)
                            return set_err(c, LBR_ERR_GEOMETRY,
                                           "level %d: ghost band too close to a body or a finer level", l);
                    }
            }
        }
    }
    return 0;
}

// Flags, distance field, lists and tiles of one level.
void finish_level(lbr_ctx* c, Level& L) {
    const lbr_config& cfg = c->cfg;
    const int nxd = cfg.nx0 << L.l, nyd = cfg.ny0 << L.l;
    L.d.assign(L.box.plane, 0.0);
    L.bidx.assign(L.box.plane, -1);
    L.owned.clear();
    L.ghosts.clear();
    L.covb.clear();
    int lo_x = 1 << 30, lo_y = 1 << 30, hi_x = -(1 << 30), hi_y = -(1 << 30);
    for (long k = 0; k < L.box.plane; ++k) {
        const int gx = (int)(k % L.box.pitch) + L.box.gx0, gy = (int)(k / L.box.pitch) + L.box.gy0;
        const int t = L.flag[k] & F_TYPE;
        if (t == T_FLUID || t == T_SOLID || t == T_COVERED || t == T_GHOST) {
            lo_x = std::min(lo_x, gx); hi_x = std::max(hi_x, gx);
            lo_y = std::min(lo_y, gy); hi_y = std::max(hi_y, gy);
        }
        if (t == T_GHOST) { L.ghosts.push_back((int32_t)k); L.n_ghost++; }
        if (t == T_COVERED && (L.flag[k] & F_COVB)) L.covb.push_back((int32_t)k);
        if (t != T_FLUID) continue;
        L.owned.push_back((int32_t)k);
        L.n_fluid++;
        if (L.l == 0 && (gx == 0 || gy == 0 || gx == nxd - 1 || gy == nyd - 1)) L.flag[k] |= F_EDGE;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                if (L.type_at(gx + dx, gy + dy) == T_GHOST) L.flag[k] |= F_NEARGHOST;
        const double py = gy + 0.5;
        double d = (cfg.body_mode == LBR_BODY_SOLID && !c->npts.empty()) ? L.dbody[k] : 1e300;
        if (cfg.bc[2] == LBR_BC_WALL) d = std::min(d, py - c->wall_lat[0] * L.scale);
        if (cfg.bc[3] == LBR_BC_WALL) d = std::min(d, c->wall_lat[1] * L.scale - py);
        L.d[k] = d;
    }
    L.bx0 = lo_x; L.by0 = lo_y; L.bnx = hi_x - lo_x + 1; L.bny = hi_y - lo_y + 1;
}

// Cut links, wall points and normals (Sections 2.1 and 2.3).
int build_walls(lbr_ctx* c, Level& L, const std::vector<double>& seg) {
    const lbr_config& cfg = c->cfg;
    const int nxd = cfg.nx0 << L.l, nyd = cfg.ny0 << L.l;
    const bool bodies = cfg.body_mode == LBR_BODY_SOLID && !seg.empty();
    Buckets bk;
    if (bodies) bk.build(seg, L.scale, 2.0);
    const bool perx = cfg.bc[0] == LBR_BC_PERIODIC;
    L.nodes.clear();
    for (int32_t k : L.owned) {
        if (L.d[k] > 1.5) continue;
        const int gx = (int)(k % L.box.pitch) + L.box.gx0, gy = (int)(k / L.box.pitch) + L.box.gy0;
        const double px = gx + 0.5, py = gy + 0.5;
        Node nd{};
        nd.gi = gx; nd.gj = gy; nd.cell = k;
        int ncut = 0;
        const std::vector<int>* cand = bodies ? bk.at(px, py) : nullptr;
        for (int o = 0; o < 9; ++o) nd.q[o] = -1.0;
        for (int o = 1; o < 9; ++o) {
            const int tx = gx + CXH[o], ty = gy + CYH[o];
            bool solid = false;
            double t = -1.0;
            if (L.l == 0 && ((ty < 0 && cfg.bc[2] == LBR_BC_WALL) || (ty >= nyd && cfg.bc[3] == LBR_BC_WALL))) {
                const double yw = (ty < 0 ? c->wall_lat[0] : c->wall_lat[1]) * L.scale;
                solid = true;
                t = (yw - py) / (double)CYH[o];
            } else {
                int txx = tx;
                if (L.l == 0 && perx) txx = ((tx % nxd) + nxd) % nxd;
                solid = L.type_at(txx, ty) == T_SOLID;
            }
            double tb = -1.0;
            if (cand)
                for (int s : *cand) {
                    const double tt = crossing(px, py, CXH[o], CYH[o], seg[5 * s] * L.scale,
                                               seg[5 * s + 1] * L.scale, seg[5 * s + 2] * L.scale,
                                               seg[5 * s + 3] * L.scale);
                    if (tt >= 0.0 && (tb < 0.0 || tt < tb)) tb = tt;
                }
            if (tb >= 0.0 && (t < 0.0 || tb < t)) t = tb;
            if (solid || tb >= 0.0) {
                nd.q[o] = t > 0.0 ? t : 0.5;
                ncut++;
            }
        }
        if (!ncut) continue;
        L.n_cut += ncut;
        // closest wall point
        double best = 1e300, qx = px, qy = py;
        int body = -1, bseg = -1;
        if (bodies) {
            for (size_t s = 0; s < seg.size() / 5; ++s) {
                double cx, cy;
                const double dd = seg_closest(px, py, seg[5 * s] * L.scale, seg[5 * s + 1] * L.scale,
                                              seg[5 * s + 2] * L.scale, seg[5 * s + 3] * L.scale, &cx, &cy);
                if (dd < best) { best = dd; qx = cx; qy = cy; body = (int)seg[5 * s + 4]; bseg = (int)s; }
            }
        }
        if (cfg.bc[2] == LBR_BC_WALL && L.l == 0) {
            const double yw = c->wall_lat[0] * L.scale;
            if (py - yw < best) { best = py - yw; qx = px; qy = yw; body = -1; bseg = -1; }
        }
        if (cfg.bc[3] == LBR_BC_WALL && L.l == 0) {
            const double yw = c->wall_lat[1] * L.scale;
            if (yw - py < best) { best = yw - py; qx = px; qy = yw; body = -2; bseg = -1; }
        }
        nd.iw[0] = qx; nd.iw[1] = qy; nd.dwb = best; nd.body = body;
        if (best > 1e-12) {
            nd.nrm[0] = (px - qx) / best;
            nd.nrm[1] = (py - qy) / best;
        } else if (bseg >= 0) {
            const double tx = seg[5 * bseg + 2] - seg[5 * bseg], ty = seg[5 * bseg + 3] - seg[5 * bseg + 1];
            const double tl = std::hypot(tx, ty);
            nd.nrm[0] = ty / tl; nd.nrm[1] = -tx / tl;
        } else {
            nd.nrm[0] = 0.0; nd.nrm[1] = body == -1 ? 1.0 : -1.0;
        }
        L.bidx[k] = (int32_t)L.nodes.size();
        L.flag[k] |= F_WALL;
        L.nodes.push_back(nd);
    }
    return 0;
}

// Range checks of one record of a precomputed cut-link list (lbr_set_cut_links);
// false with the reason in msg.
bool cut_record_ok(const double* p, char* msg, size_t len) {
    static const char* name[LBR_CUT_STRIDE] = {"gi", "gj", "IW x", "IW y", "normal x", "normal y", "d_WB",
                                               "body", "q1", "q2", "q3", "q4", "q5", "q6", "q7", "q8"};
    for (int j = 0; j < LBR_CUT_STRIDE; ++j)
        if (!std::isfinite(p[j])) { snprintf(msg, len, "%s is not finite", name[j]); return false; }
    for (int j : {0, 1, 7})
        if (p[j] != std::floor(p[j]) || std::fabs(p[j]) > (double)(1 << 30)) {
            snprintf(msg, len, "%s = %g is not an integer in range", name[j], p[j]);
            return false;
        }
    if (p[7] < -2.0) { snprintf(msg, len, "body = %g is below -2", p[7]); return false; }
    const double nn = std::hypot(p[4], p[5]);
    if (std::fabs(nn - 1.0) > 1e-6) { snprintf(msg, len, "|normal| = %.9g is not 1", nn); return false; }
    if (p[6] < 0.0) { snprintf(msg, len, "d_WB = %g is negative", p[6]); return false; }
    int cut = 0;
    for (int o = 1; o < 9; ++o) {
        const double q = p[7 + o];
        if (q == -1.0) continue;
        if (!(q > 0.0 && q <= 1.0)) {
            snprintf(msg, len, "q%d = %g is neither in (0, 1] nor -1", o, q);
            return false;
        }
        cut++;
    }
    if (!cut) { snprintf(msg, len, "no link is cut"); return false; }
    return true;
}

// Wall nodes of one level from a precomputed cut-link list (lbr_set_cut_links;
// records already range-checked): the records take the place of the polyline
// intersections of build_walls, and are checked against the level's cells.
int walls_from_list(lbr_ctx* c, Level& L, const std::vector<double>& rec) {
    const lbr_config& cfg = c->cfg;
    const int nyd = cfg.ny0 << L.l, nxd = cfg.nx0 << L.l;
    const bool perx = cfg.bc[0] == LBR_BC_PERIODIC;
    const int nbody = cfg.body_mode == LBR_BODY_SOLID ? (int)c->npts.size() : 0;
    const size_t n = rec.size() / LBR_CUT_STRIDE;
    L.nodes.clear();
    L.n_cut = 0;
    for (size_t r = 0; r < n; ++r) {
        const double* p = &rec[r * LBR_CUT_STRIDE];
        Node nd{};
        nd.gi = (int)p[0]; nd.gj = (int)p[1];
        const long k = L.idx(nd.gi, nd.gj);
        if (k < 0 || (L.flag[k] & F_TYPE) != T_FLUID)
            return set_err(c, LBR_ERR_GEOMETRY, "level %d: cut-link record %zu: cell (%d, %d) is not an owned "
                           "fluid cell", L.l, r, nd.gi, nd.gj);
        if (L.bidx[k] >= 0)
            return set_err(c, LBR_ERR_GEOMETRY, "level %d: cut-link record %zu: cell (%d, %d) is listed twice",
                           L.l, r, nd.gi, nd.gj);
        // the boundary-node update pulls from owned cells only (as generated
        // nodes, which the grid keeps away from level interfaces)
        if (L.flag[k] & (F_NEARGHOST | F_IFACE))
            return set_err(c, LBR_ERR_GEOMETRY, "level %d: cut-link record %zu: cell (%d, %d) lies next to a "
                           "level interface", L.l, r, nd.gi, nd.gj);
        nd.body = (int)p[7];
        const bool body_ok = nd.body >= 0 ? nd.body < nbody
                           : L.l == 0 && ((nd.body == -1 && cfg.bc[2] == LBR_BC_WALL) ||
                                          (nd.body == -2 && cfg.bc[3] == LBR_BC_WALL));
        if (!body_ok)
            return set_err(c, LBR_ERR_GEOMETRY, "level %d: cut-link record %zu: body %d names no body or wall "
                           "side of this level", L.l, r, nd.body);
        nd.cell = k;
        nd.iw[0] = p[2]; nd.iw[1] = p[3];
        nd.nrm[0] = p[4]; nd.nrm[1] = p[5];
        nd.dwb = p[6];
        nd.q[0] = -1.0;
        for (int o = 1; o < 9; ++o) {
            nd.q[o] = p[7 + o];
            if (nd.q[o] >= 0.0) L.n_cut++;
        }
        L.bidx[k] = (int32_t)L.nodes.size();
        L.flag[k] |= F_WALL;
        L.nodes.push_back(nd);
    }
    // every link that reaches a solid cell or crosses a wall side must be cut:
    // the step would otherwise stream from a solid cell
    for (int32_t k : L.owned) {
        const int gx = (int)(k % L.box.pitch) + L.box.gx0, gy = (int)(k / L.box.pitch) + L.box.gy0;
        for (int o = 1; o < 9; ++o) {
            const int tx = gx + CXH[o], ty = gy + CYH[o];
            bool solid;
            if (L.l == 0 && ((ty < 0 && cfg.bc[2] == LBR_BC_WALL) || (ty >= nyd && cfg.bc[3] == LBR_BC_WALL))) {
                solid = true;
            } else {
                const int txx = (L.l == 0 && perx) ? ((tx % nxd) + nxd) % nxd : tx;
                solid = L.type_at(txx, ty) == T_SOLID;
            }
            if (solid && (L.bidx[k] < 0 || L.nodes[L.bidx[k]].q[o] < 0.0))
                return set_err(c, LBR_ERR_GEOMETRY, "level %d: the link from cell (%d, %d) along c_%d reaches a "
                               "solid cell or a wall side but is not a cut link of the list", L.l, gx, gy, o);
        }
    }
    return 0;
}

// Interpolation weights at R (step 1 of the VN procedure): IDW (power 2) for
// rho over the enclosing 2 x 2 block without boundary nodes, linear least
// squares for u over its fluid cells, both grown to 4 x 4 when too few cells
// remain.  Weights are stored so the device only gathers.
int stencils(lbr_ctx* c, Level& L, std::vector<int32_t>& sc, std::vector<double>& wr,
             std::vector<double>& wu) {
    const lbr_config& cfg = c->cfg;
    const int nb = (int)L.nodes.size();
    const int nxd = cfg.nx0 << L.l, nyd = cfg.ny0 << L.l;
    const bool perx = cfg.bc[0] == LBR_BC_PERIODIC && L.l == 0;
    const double dwr = cfg.wall_model == LBR_WALL_NISHIMURA ? 1.75 : cfg.d_wr;
    sc.assign((size_t)nb * MAX_STENCIL, -1);
    wr.assign((size_t)nb * MAX_STENCIL, 0.0);
    wu.assign((size_t)nb * MAX_STENCIL, 0.0);
    for (int b = 0; b < nb; ++b) {
        const Node& nd = L.nodes[b];
        const double rx = nd.iw[0] + dwr * nd.nrm[0], ry = nd.iw[1] + dwr * nd.nrm[1];
        const int i0 = (int)std::floor(rx - 0.5), j0 = (int)std::floor(ry - 0.5);
        struct Pt { long cell; double x, y; bool rho_ok; };
        auto gather = [&](int grow, std::vector<Pt>& pts) {
            pts.clear();
            for (int dj = -grow; dj <= 1 + grow; ++dj)
                for (int di = -grow; di <= 1 + grow; ++di) {
                    const int gi = i0 + di, gj = j0 + dj;
                    int gis = gi;
                    if (perx) gis = ((gi % nxd) + nxd) % nxd;
                    if (L.l == 0 && (gj < 0 || gj >= nyd)) continue;
                    const long k = L.idx(gis, gj);
                    if (k < 0) continue;
                    const int t = L.flag[k] & F_TYPE;
                    if (t == T_FLUID)
                        pts.push_back({k, gi + 0.5, gj + 0.5, L.bidx[k] < 0});
                    else if (t != T_SOLID)
                        return false;
                }
            return true;
        };
        std::vector<Pt> pts;
        std::vector<double> w_rho, w_u;
        std::vector<long> cells;
        bool rho_done = false, u_done = false;
        std::vector<std::pair<long, double>> rw, uw;
        for (int grow = 0; grow <= 1 && !(rho_done && u_done); ++grow) {
            if (!gather(grow, pts))
                return set_err(c, LBR_ERR_GEOMETRY, "level %d: wall stencil reaches a non-owned cell", L.l);
            if (!rho_done) {
                double sw = 0;
                rw.clear();
                for (const Pt& p : pts) {
                    if (!p.rho_ok) continue;
                    const double d2 = (p.x - rx) * (p.x - rx) + (p.y - ry) * (p.y - ry);
                    if (d2 < 1e-24) { rw.assign(1, {p.cell, 1.0}); sw = 1.0; break; }
                    rw.push_back({p.cell, 1.0 / d2});
                    sw += 1.0 / d2;
                }
                if (!rw.empty()) {
                    for (auto& e : rw) e.second /= sw;
                    rho_done = true;
                }
            }
            if (!u_done && pts.size() >= 3) {
                double A[3][3] = {{0}};
                for (const Pt& p : pts) {
                    const double r[3] = {1.0, p.x - rx, p.y - ry};
                    for (int a = 0; a < 3; ++a)
                        for (int b2 = 0; b2 < 3; ++b2) A[a][b2] += r[a] * r[b2];
                }
                const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                                   A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                                   A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
                if (std::fabs(det) >= 1e-9) {
                    // first row of A^-1 (cofactors / det)
                    const double r0[3] = {(A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det,
                                          -(A[0][1] * A[2][2] - A[0][2] * A[2][1]) / det,
                                          (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det};
                    uw.clear();
                    for (const Pt& p : pts)
                        uw.push_back({p.cell, r0[0] + r0[1] * (p.x - rx) + r0[2] * (p.y - ry)});
                    u_done = true;
                }
            }
        }
        if (!rho_done) rw.assign(1, {nd.cell, 1.0});
        if (!u_done) uw.assign(1, {nd.cell, 1.0});
        // merge into one list of cells
        std::vector<long> cl;
        for (auto& e : rw) cl.push_back(e.first);
        for (auto& e : uw) cl.push_back(e.first);
        std::sort(cl.begin(), cl.end());
        cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
        if ((int)cl.size() > MAX_STENCIL) return set_err(c, LBR_ERR_GEOMETRY, "wall stencil too large");
        for (size_t j = 0; j < cl.size(); ++j) {
            sc[(size_t)b * MAX_STENCIL + j] = (int32_t)cl[j];
            for (auto& e : rw) if (e.first == cl[j]) wr[(size_t)b * MAX_STENCIL + j] += e.second;
            for (auto& e : uw) if (e.first == cl[j]) wu[(size_t)b * MAX_STENCIL + j] += e.second;
        }
    }
    return 0;
}

// 64 x H tiles with work for k_step (owned fluid cells other than wall nodes
// and domain-edge cells, or ghost cells), for every tile height H.
void make_rows(Level& L) {
    for (int k = 0; k < NTY; ++k) {
        const int H = TILE_YS[k];
        std::vector<uint32_t>& rows = L.rows[k];
        rows.clear();
        const int ntx = L.box.pitch / TILE_X, nty = L.box.ny / H;
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) {
                bool act = false;
                for (int y = 0; y < H && !act; ++y)
                    for (int x = 0; x < TILE_X && !act; ++x) {
                        const uint8_t f = L.flag[(long)(ty * H + y) * L.box.pitch + tx * TILE_X + x];
                        const int t = f & F_TYPE;
                        act = (t == T_FLUID && !(f & (F_WALL | F_EDGE))) || t == T_GHOST;
                    }
                if (act) rows.push_back((uint32_t)tx | ((uint32_t)ty << 16));
            }
    }
}

// Marks the tiles that hold children of restriction targets of the parent level.
void mark_restriction_tiles(lbr_ctx* c, Level& L) {
    if (L.l == 0) return;
    const Level& P = c->lv[L.l - 1];
    for (int k = 0; k < NTY; ++k) {
        const int H = TILE_YS[k];
        for (uint32_t& tl : L.rows[k]) {
            const int tx = tl & 0x7fff, ty = (tl >> 16) & 0x7fff;
            bool any = false;
            for (int y = 0; y < H && !any; y += 2)
                for (int x = 0; x < TILE_X && !any; x += 2) {
                    const int gx = L.box.gx0 + tx * TILE_X + x, gy = L.box.gy0 + ty * H + y;
                    const long pk = P.idx(gx >> 1, gy >> 1);
                    any = pk >= 0 && (P.flag[pk] & F_COVB) &&
                          (L.flag[(long)(ty * H + y) * L.box.pitch + tx * TILE_X + x] & F_TYPE) == T_FLUID;
                }
            if (any) tl |= 1u << 31;
        }
    }
}

// Marks (bit 15 of the tile word) the tiles whose cells or one-cell halo ring
// hold ghost cells: the step stages the parent's chi, u, v under them in LDS.
void mark_ghost_tiles(Level& L) {
    for (int k = 0; k < NTY; ++k) {
        const int H = TILE_YS[k];
        for (uint32_t& tl : L.rows[k]) {
            const int tx = tl & 0x7fff, ty = (tl >> 16) & 0x7fff;
            bool any = false;
            for (int y = -1; y <= H && !any; ++y)
                for (int x = -1; x <= TILE_X && !any; ++x) {
                    const int ly = ty * H + y, lx = tx * TILE_X + x;
                    if (ly < 0 || ly >= L.box.ny || lx < 0 || lx >= L.box.pitch) continue;
                    any = (L.flag[(long)ly * L.box.pitch + lx] & F_TYPE) == T_GHOST;
                }
            if (any) tl |= 1u << 15;
        }
    }
}

// Orders each XCD's share of a short tile list so that the slow tiles start
// first: tiles holding ghost cells, then tiles with other neighbouring-level
// work (near-ghost and coalescence cells, restriction anchors, ghost cells in
// the halo), then the rest, each group in its original order.  The step maps
// block b to tile (b mod 8) * per + b / 8, so each XCD keeps its tiles.  Only
// lists of at most four generations of resident workgroups are reordered: there
// the last generation's tail sets the launch time; longer launches run at the
// memory system's rate and keep the row order, whose neighbouring tiles share
// halo rows in the XCD's L2.  Tiles of one launch are independent, so the order
// changes no result.
void order_tiles(Level& L, int cus) {
    for (int k = 0; k < NTY; ++k) {
        const int H = TILE_YS[k];
        std::vector<uint32_t>& rows = L.rows[k];
        const int n = (int)rows.size(), per = (n + 7) >> 3;
        const long resident = (long)cus * 32 / H;       // 8 waves per SIMD, 4 SIMDs; H waves per workgroup
        if (resident <= 0 || n > 4 * resident) continue;
        std::vector<std::pair<int, uint32_t>> keyed(n);
        for (int t = 0; t < n; ++t) {
            const uint32_t tl = rows[t];
            const int tx = tl & 0x7fff, ty = (tl >> 16) & 0x7fff;
            bool ghost = false, other = (tl >> 31) || ((tl >> 15) & 1u);
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < TILE_X; ++x) {
                    const uint8_t f = L.flag[(long)(ty * H + y) * L.box.pitch + tx * TILE_X + x];
                    ghost = ghost || (f & F_TYPE) == T_GHOST;
                    other = other || (f & (F_NEARGHOST | F_IFACE));
                }
            keyed[t] = {ghost ? 0 : (other ? 1 : 2), tl};
        }
        for (int x = 0; x < 8; ++x) {
            const int a = std::min(n, x * per), b = std::min(n, (x + 1) * per);
            std::stable_sort(keyed.begin() + a, keyed.begin() + b,
                             [](const std::pair<int, uint32_t>& p, const std::pair<int, uint32_t>& q) {
                                 return p.first < q.first;
                             });
        }
        for (int t = 0; t < n; ++t) rows[t] = keyed[t].second;
    }
}

Prec level_storage(const lbr_ctx* c, int l) {
    if (c->cfg.storage != LBR_STORE_MIXED) return c->prec;
    return l >= c->cfg.n_levels - 2 ? P_F32 : P_F16;
}

int alloc_level(lbr_ctx* c, Level& L) {
    L.st = level_storage(c, L.l);
    L.ssize = L.st == P_F64 ? 8 : (L.st == P_F32 ? 4 : 2);
    const size_t n = L.box.plane;
    const size_t pad = (size_t)L.box.pitch + 1;    // k_step reads one row beyond both ends
    // k_step addresses each array through a buffer resource with 32-bit byte offsets
    if ((9 * n + 2 * pad) * std::max<size_t>(c->ssize, 8) >= (size_t)1 << 31)
        return set_err(c, LBR_ERR_INVALID_ARG, "level %d: storage box of %zu cells exceeds the "
                       "2 GiB per-array limit", L.l, n);
    for (int b = 0; b < 2; ++b) {
        L.f[b] = dalloc_padded(c, 9 * n, L.ssize, pad);
        L.mac[b] = dalloc_padded(c, 3 * n, c->csize, pad);
        L.chi[b] = dalloc_padded(c, n, c->csize, pad);
        if (!L.f[b] || !L.mac[b] || !L.chi[b]) return set_err(c, LBR_ERR_OOM, "level %d: out of device memory", L.l);
        HIPCHK(c, hipMemsetAsync(static_cast<char*>(L.f[b]) - pad * L.ssize, 0, (9 * n + 2 * pad) * L.ssize, c->stream));
        HIPCHK(c, hipMemsetAsync(static_cast<char*>(L.mac[b]) - pad * c->csize, 0, (3 * n + 2 * pad) * c->csize, c->stream));
        HIPCHK(c, hipMemsetAsync(static_cast<char*>(L.chi[b]) - pad * c->csize, 0, (n + 2 * pad) * c->csize, c->stream));
    }
    L.bytes += 2 * (n + 2 * pad) * (9 * L.ssize + 4 * c->csize);
    // The wall distance is computed in FP64 (k_geometry).  The FP64 step reads
    // it as such; the FP32-arithmetic steps round it to FP32 at every use, so
    // they read that rounding, stored once (the same values, half the bytes).
    std::vector<double> dclamp(L.d);
    if (c->prec != P_F64)
        for (double& v : dclamp) v = std::min(v, 1e18);
    L.dist_dev = dalloc_padded(c, n, c->csize, pad);
    if (!L.dist_dev) return set_err(c, LBR_ERR_OOM, "level %d: out of device memory", L.l);
    HIPCHK(c, hipMemsetAsync(static_cast<char*>(L.dist_dev) - pad * c->csize, 0, (n + 2 * pad) * c->csize, c->stream));
    std::vector<float> d32;
    if (c->prec == P_F64) {
        HIPCHK(c, hipMemcpyAsync(L.dist_dev, dclamp.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    } else {
        d32.assign(dclamp.begin(), dclamp.end());
        HIPCHK(c, hipMemcpyAsync(L.dist_dev, d32.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));                    // the host copies die here
    L.bytes += (n + 2 * pad) * c->csize;
    // flags carry the same spare row at both ends (T_INACTIVE): the k_step halo reads them
    L.flag_dev = static_cast<uint8_t*>(dalloc_padded(c, n, 1, pad));
    if (!L.flag_dev) return set_err(c, LBR_ERR_OOM, "level %d: out of device memory", L.l);
    HIPCHK(c, hipMemsetAsync(L.flag_dev - pad, T_INACTIVE, n + 2 * pad, c->stream));
    HIPCHK(c, hipMemcpyAsync(L.flag_dev, L.flag.data(), n, hipMemcpyHostToDevice, c->stream));
    L.bytes += n + 2 * pad;
    for (int k = 0; k < NTY; ++k)
        if (int r = upload(c, &L.rows_dev[k], L.rows[k], &L.bytes)) return r;
    {
        // static link mask: which pull sources are owned fluid cells / ghosts
        std::vector<uint32_t> lm(n, 0u);
        const Level* Pp = L.l > 0 ? &c->lv[L.l - 1] : nullptr;
        for (long k = 0; k < (long)n; ++k) {
            const int t = L.flag[k] & F_TYPE;
            const int gx = (int)(k % L.box.pitch) + L.box.gx0, gy = (int)(k / L.box.pitch) + L.box.gy0;
            if (Pp && t == T_FLUID && !(gx & 1) && !(gy & 1)) {
                const long pk = Pp->idx(gx >> 1, gy >> 1);
                if (pk >= 0 && (Pp->flag[pk] & F_COVB)) {
                    if (((gx - L.box.gx0) | (gy - L.box.gy0)) & 1)
                        return set_err(c, LBR_ERR_GEOMETRY, "level %d: restriction block at (%d, %d) is not aligned "
                                       "with the storage box", L.l, gx, gy);
                    // the 2 x 2 block is averaged by the k_step workgroup that updates it
                    for (int b = 0; b < 2; ++b)
                        for (int a2 = 0; a2 < 2; ++a2) {
                            const uint8_t fc = L.flag[k + (long)b * L.box.pitch + a2];
                            if ((fc & F_TYPE) != T_FLUID || (fc & (F_WALL | F_EDGE)))
                                return set_err(c, LBR_ERR_GEOMETRY, "level %d: restriction block at (%d, %d) "
                                               "is not plain fluid", L.l, gx, gy);
                        }
                    lm[k] |= 1u << 31;
                }
            }
            if (t != T_GHOST && !(L.flag[k] & F_NEARGHOST)) continue;
            uint32_t m = lm[k];
            for (int i = 0; i < 9; ++i) {
                const int ts = L.type_at(gx - CXH[i], gy - CYH[i]);
                if (ts == T_FLUID) m |= 1u << i;
                if (ts == T_GHOST) m |= 1u << (16 + i);
            }
            lm[k] = m;
        }
        if (int r = upload(c, &L.lmask_dev, lm, &L.bytes)) return r;
    }
    if (int r = upload(c, &L.ghosts_dev, L.ghosts, &L.bytes)) return r;
    if (int r = upload(c, &L.covb_dev, L.covb, &L.bytes)) return r;
    if (int r = upload(c, &L.owned_dev, L.owned, &L.bytes)) return r;
    L.edge.clear();
    for (int32_t k : L.owned)
        if ((L.flag[k] & F_EDGE) && !(L.flag[k] & F_WALL)) L.edge.push_back(k);
    if (int r = upload(c, &L.edge_dev, L.edge, &L.bytes)) return r;
    L.snap = static_cast<double*>(dalloc(c, std::max<size_t>(L.owned.size(), 1) * 2 * sizeof(double)));
    // wall records
    const int nb = (int)L.nodes.size();
    std::vector<int32_t> bcell(nb);
    std::vector<double> geo((size_t)nb * 6), qd((size_t)nb * 8);
    for (int b = 0; b < nb; ++b) {
        const Node& nd = L.nodes[b];
        bcell[b] = (int32_t)nd.cell;
        geo[6 * b + 0] = nd.iw[0]; geo[6 * b + 1] = nd.iw[1];
        geo[6 * b + 2] = nd.nrm[0]; geo[6 * b + 3] = nd.nrm[1];
        geo[6 * b + 4] = nd.dwb; geo[6 * b + 5] = nd.body;
        for (int o = 1; o < 9; ++o) qd[8 * b + o - 1] = nd.q[o];
    }
    if (int r = upload(c, &L.bcell, bcell, &L.bytes)) return r;
    if (int r = upload(c, &L.bgeo, geo, &L.bytes)) return r;
    if (int r = upload(c, &L.bq, qd, &L.bytes)) return r;
    L.bstate = static_cast<double*>(dalloc(c, std::max(nb, 1) * 8 * sizeof(double)));
    L.bout = static_cast<double*>(dalloc(c, std::max(nb, 1) * 8 * sizeof(double)));
    if (!L.bstate || !L.bout) return set_err(c, LBR_ERR_OOM, "wall state allocation failed");
    HIPCHK(c, hipMemsetAsync(L.bstate, 0, std::max(nb, 1) * 8 * sizeof(double), c->stream));
    HIPCHK(c, hipMemsetAsync(L.bout, 0, std::max(nb, 1) * 8 * sizeof(double), c->stream));
    std::vector<int32_t> sc;
    std::vector<double> wr, wu;
    if (int r = stencils(c, L, sc, wr, wu)) return r;
    if (int r = upload(c, &L.st_cell, sc, &L.bytes)) return r;
    if (int r = upload(c, &L.st_wr, wr, &L.bytes)) return r;
    if (int r = upload(c, &L.st_wu, wu, &L.bytes)) return r;
    return 0;
}

WallData wall_data(lbr_ctx* c, const Level& L) {
    const lbr_config& cfg = c->cfg;
    WallData w{};
    w.nb = (int)L.nodes.size();
    w.cell = L.bcell;
    w.geo = L.bgeo;
    w.st_cell = L.st_cell;
    w.st_wr = L.st_wr;
    w.st_wu = L.st_wu;
    w.q = L.bq;
    w.d_wr = cfg.wall_model == LBR_WALL_NISHIMURA ? 1.75 : cfg.d_wr;
    w.d_wv = cfg.d_wv;
    w.uw_lo[0] = cfg.u_wall[0]; w.uw_lo[1] = cfg.u_wall[1];
    w.uw_hi[0] = cfg.u_wall[2]; w.uw_hi[1] = cfg.u_wall[3];
    w.model = cfg.wall_model;
    return w;
}

// Start-up ramp (not part of the paper's method; ramp_steps = 0 starts the flow
// impulsively at u_ref): the initial state moves uniformly at r0 u_ref and during
// coarse step n the inlet velocity and the target of the absorbing layer are
// u_ref (r0 + (1 - r0) (1 - cos(pi min(1, n / N))) / 2).
double ramp(const lbr_ctx* c, int64_t n) {
    const double N = c->cfg.ramp_steps, r0 = c->cfg.ramp_start;
    if (!(N > 0.0) || (double)n >= N) return 1.0;
    return r0 + (1.0 - r0) * (0.5 - 0.5 * std::cos(3.14159265358979323846 * (double)n / N));
}

// Absorbing layer of level l (none above level 0) with the free stream scaled by r.
Absorber absorber(const lbr_ctx* c, int l, double r) {
    const lbr_config& cfg = c->cfg;
    Absorber sp{};
    sp.drho = cfg.rho_ref - 1.0;
    sp.ux = c->u_ref * r;
    if (l == 0 && cfg.sponge_width > 0.0 && cfg.sponge_strength > 0.0) {
        sp.width = cfg.sponge_width;
        sp.strength = cfg.sponge_strength;
        for (int k = 0; k < 4; ++k)
            if (cfg.bc[k] == LBR_BC_INLET || cfg.bc[k] == LBR_BC_OUTLET || cfg.bc[k] == LBR_BC_SYMMETRY)
                sp.sides |= 1 << k;
    }
    return sp;
}

template <class ST, class CT>
void fill_step_args(lbr_ctx* c, int l, int substep, StepArgs<ST, CT>& a, int tk = -1) {
    Level& L = c->lv[l];
    const lbr_config& cfg = c->cfg;
    a.fsrc = (const ST*)L.f[L.cur];
    a.fdst = (ST*)L.f[1 - L.cur];
    a.msrc = (const CT*)L.mac[L.cur];
    a.mdst = (CT*)L.mac[1 - L.cur];
    a.csrc = (const CT*)L.chi[L.cur];
    a.cdst = (CT*)L.chi[1 - L.cur];
    a.dist = static_cast<const CT*>(L.dist_dev);
    a.flag = L.flag_dev;
    a.lmask = L.lmask_dev;
    if (tk < 0) tk = L.ty;                                       // tile height
    a.ty = TILE_YS[tk];
    a.tiles = L.rows_dev[tk];
    a.ntiles = (int)L.rows[tk].size();
    a.edge = L.edge_dev;
    a.nedge = (int)L.edge.size();
    a.wall = wall_data(c, L);
    a.wstate = L.bstate;
    a.box = L.box;
    a.dom.nxd = cfg.nx0 << l;
    a.dom.nyd = cfg.ny0 << l;
    for (int k = 0; k < 4; ++k) a.dom.bc[k] = cfg.bc[k];
    a.dom.periodic_x = cfg.bc[0] == LBR_BC_PERIODIC;
    a.dom.outlet = cfg.outlet;
    a.pad = L.box.pitch + 1;
    a.wall_blocks = 8 * (((int)L.nodes.size() + 8 * WALL_PER_BLOCK - 1) / (8 * WALL_PER_BLOCK));
    a.tile_blocks = 8 * ((a.ntiles + 7) / 8);
    // this launch streams coarse step n = step_count and collides step n + 1
    a.sp = absorber(c, l, ramp(c, c->step_count + 1));
    for (int i = 0; i < 9; ++i) a.dsh[i] = (CT)c->dsh[i];
    a.nu = (CT)L.nu;
    a.fx = (CT)L.fx;
    a.fy = (CT)L.fy;
    a.omega_b = (CT)cfg.omega_b;
    a.u_in = (CT)(c->u_ref * ramp(c, c->step_count));
    a.chi_in = (CT)cfg.chi_inlet;
    a.rho_out = (CT)cfg.rho_ref;
    a.sa_mode = cfg.sa;
    a.mu_cap = cfg.sa_mu_cap > 0 ? (CT)cfg.sa_mu_cap : (CT)INFINITY;
    a.frozen = cfg.sa == LBR_SA_FROZEN;
    a.bb_halfway = cfg.bb == LBR_BB_HALFWAY;
    a.substep = substep;
    a.sst = L.st;
    if (l > 0) {
        Level& P = c->lv[l - 1];
        a.fcoarse = P.f[P.cur];
        a.cst = P.st;
        a.cbox = P.box;
        a.cmac = (const CT*)P.mac[P.cur];
        a.cchi = (const CT*)P.chi[P.cur];
        a.rmac = (CT*)P.mac[1 - P.cur];
        a.rchi = (CT*)P.chi[1 - P.cur];
    } else {
        a.fcoarse = nullptr;
        a.cst = L.st;
        a.cbox = Box{};
        a.cmac = a.cchi = nullptr;
        a.rmac = a.rchi = nullptr;
    }
    if (l + 1 < (int)c->lv.size()) {
        Level& F = c->lv[l + 1];
        a.ffine = F.f[F.cur];
        a.fst = F.st;
        a.fbox = F.box;
    } else {
        a.ffine = nullptr;
        a.fst = L.st;
        a.fbox = Box{};
    }
}

// Wall model of one level on its current state, into L.bout (output only).
int eval_wall(lbr_ctx* c, int l) {
    Level& L = c->lv[l];
    if (L.nodes.empty()) return 0;
    if (c->prec == P_F64) {
        WallArgs<double> a{};
        a.wall = wall_data(c, L);
        a.mac = (const double*)L.mac[L.cur];
        a.guess = L.bstate;
        a.out = L.bout;
        a.plane = L.box.plane;
        a.nu = L.nu;
        HIPCHK(c, launch_wall(c->prec, &a, c->stream));
    } else {
        WallArgs<float> a{};
        a.wall = wall_data(c, L);
        a.mac = (const float*)L.mac[L.cur];
        a.guess = L.bstate;
        a.out = L.bout;
        a.plane = L.box.plane;
        a.nu = L.nu;
        HIPCHK(c, launch_wall(c->prec, &a, c->stream));
    }
    return 0;
}

enum { EV_STEP = 0, EV_STEP_FINE = 1, EV_STEP_L0 = 2 };

// Start / stop events for one dispatch of the given kind (profiling mode only).
Timing prof_events(lbr_ctx* c, int kind) {
    Timing tm;
    if (!c->prof) return tm;
    c->prof_launches++;
    if (c->ev_used + 2 > 2 * MAX_TIMED_LAUNCHES) return tm;   // the first launches of the call
    while (c->ev.size() < c->ev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return tm;
        c->ev.push_back(e);
        c->ev_kind.push_back(0);
    }
    tm.start = c->ev[c->ev_used];
    tm.stop = c->ev[c->ev_used + 1];
    c->ev_kind[c->ev_used] = kind;
    c->ev_used += 2;
    return tm;
}

int do_step(lbr_ctx* c, int l, int substep) {
    Level& L = c->lv[l];
    alignas(16) unsigned char buf[sizeof(StepArgs<double, double>)];
    switch (L.st) {
        case P_F64: fill_step_args(c, l, substep, *reinterpret_cast<StepArgs<double, double>*>(buf)); break;
        case P_F32: fill_step_args(c, l, substep, *reinterpret_cast<StepArgs<float, float>*>(buf)); break;
        case P_F16: fill_step_args(c, l, substep, *reinterpret_cast<StepArgs<__half, float>*>(buf)); break;
        default: fill_step_args(c, l, substep, *reinterpret_cast<StepArgs<__hip_bfloat16, float>*>(buf)); break;
    }
    // one launch per level sub-step: tiles, wall nodes and domain-edge cells are
    // workgroups of the same grid (disjoint cells, same source state)
    const int kind = l + 1 == (int)c->lv.size() ? EV_STEP_FINE : (l == 0 ? EV_STEP_L0 : EV_STEP);
    HIPCHK(c, launch_step(L.st, buf, c->stream, prof_events(c, kind)));
    L.cur ^= 1;
    return 0;
}

int do_transfers(lbr_ctx* c, int l) {
    Level& C = c->lv[l];
    Level& F = c->lv[l + 1];
    RestrictArgs r{};
    r.n = (int)C.covb.size();
    r.list = C.covb_dev;
    r.fbox = F.box;
    r.cbox = C.box;
    r.fmac = F.mac[F.cur];
    r.fchi = F.chi[F.cur];
    r.cmac = C.mac[C.cur];
    r.cchi = C.chi[C.cur];
    HIPCHK(c, launch_restrict(c->prec, r, c->stream));
    FillArgs f{};
    f.n = (int)F.ghosts.size();
    f.list = F.ghosts_dev;
    f.fbox = F.box;
    f.cbox = C.box;
    f.cmac = C.mac[C.cur];
    f.cchi = C.chi[C.cur];
    f.fmac0 = F.mac[0]; f.fmac1 = F.mac[1];
    f.fchi0 = F.chi[0]; f.fchi1 = F.chi[1];
    HIPCHK(c, launch_fill(c->prec, f, c->stream));
    return 0;
}

// Recursive cycle of Section 2.1: the finer level takes two sub-steps, then
// this level streams (pulling the coalesced band of the finer level) and
// collides.
int cycle(lbr_ctx* c, int l, int substep) {
    if (l + 1 < (int)c->lv.size()) {
        if (int r = cycle(c, l + 1, 1)) return r;
        if (int r = cycle(c, l + 1, 2)) return r;
    }
    return do_step(c, l, substep);
}

int init_level(lbr_ctx* c, int l, const double* rho, const double* ux, const double* uy,
               const double* chi) {
    Level& L = c->lv[l];
    const size_t n = L.owned.size();
    std::vector<double> v(4 * n);
    for (size_t k = 0; k < n; ++k) {
        const long cell = L.owned[k];
        const int gx = (int)(cell % L.box.pitch) + L.box.gx0, gy = (int)(cell / L.box.pitch) + L.box.gy0;
        const long io = (long)(gy - L.by0) * L.bnx + (gx - L.bx0);
        v[k] = rho ? rho[io] : c->cfg.rho_ref;
        v[n + k] = ux ? ux[io] : c->u_ref * ramp(c, c->step_count);
        v[2 * n + k] = uy ? uy[io] : 0.0;
        v[3 * n + k] = chi ? chi[io] : c->cfg.chi_init;
    }
    double* dv = static_cast<double*>(dalloc(c, std::max<size_t>(v.size(), 4) * sizeof(double)));
    if (!dv) return set_err(c, LBR_ERR_OOM, "init staging allocation failed");
    if (n) HIPCHK(c, hipMemcpyAsync(dv, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    InitArgs a{};
    a.n = (int)n;
    a.list = L.owned_dev;
    a.rho = dv; a.ux = dv + n; a.uy = dv + 2 * n; a.chi = dv + 3 * n;
    a.f = L.f[L.cur];
    a.mac = L.mac[L.cur];
    a.chi_a = L.chi[0];
    a.chi_b = L.chi[1];
    a.plane = L.box.plane;
    a.nu = L.nu; a.fx = L.fx; a.fy = L.fy; a.omega_b = c->cfg.omega_b;
    a.pitch = L.box.pitch; a.gx0 = L.box.gx0; a.gy0 = L.box.gy0;
    a.nxd = c->cfg.nx0 << l; a.nyd = c->cfg.ny0 << l;
    a.sp = absorber(c, l, ramp(c, c->step_count));
    for (int i = 0; i < 9; ++i) a.dsh[i] = c->dsh[i];
    HIPCHK(c, launch_init(L.st, a, c->stream));
    HIPCHK(c, hipMemsetAsync(L.bstate, 0, std::max<size_t>(L.nodes.size(), 1) * 8 * sizeof(double), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, dv);
    return 0;
}

int build_surface(lbr_ctx* c, const std::vector<double>& seg) {
    c->surf.assign(c->npts.size(), SurfaceBody());
    c->wall_level = -1;
    for (int l = (int)c->lv.size() - 1; l >= 0; --l)
        if (!c->lv[l].nodes.empty()) { c->wall_level = l; break; }
    if (c->wall_level < 0 || c->cfg.body_mode != LBR_BODY_SOLID) return 0;
    const Level& L = c->lv[c->wall_level];
    int maxseg = 0;
    for (size_t b = 0; b < c->npts.size(); ++b) {
        const int n = c->npts[b];
        maxseg = std::max(maxseg, n);
        std::vector<double> sg((size_t)n * 6);
        std::vector<int32_t> near((size_t)n * 2, -1);
        std::vector<double> wgt((size_t)n * 2, 0.0);
        for (int k = 0; k < n; ++k) {
            const double* s = &seg[5 * (c->off[b] + k)];
            const double ax = s[0] * L.scale, ay = s[1] * L.scale, bx = s[2] * L.scale, by = s[3] * L.scale;
            const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by);
            double tx = bx - ax, ty = by - ay;
            const double tl = std::sqrt(tx * tx + ty * ty);
            tx /= tl; ty /= tl;
            sg[6 * k + 0] = tx; sg[6 * k + 1] = ty;
            sg[6 * k + 2] = ty; sg[6 * k + 3] = -tx;          // normal into the fluid
            sg[6 * k + 4] = tl / L.scale * c->cfg.dx0 / c->cfg.ref_length;   // ds / c
            int best[2] = {-1, -1};
            double bd[2] = {1e300, 1e300};
            for (size_t j = 0; j < L.nodes.size(); ++j) {
                if (L.nodes[j].body != (int)b) continue;
                const double dd = (L.nodes[j].iw[0] - mx) * (L.nodes[j].iw[0] - mx) +
                                  (L.nodes[j].iw[1] - my) * (L.nodes[j].iw[1] - my);
                if (dd < bd[0]) { bd[1] = bd[0]; best[1] = best[0]; bd[0] = dd; best[0] = (int)j; }
                else if (dd < bd[1]) { bd[1] = dd; best[1] = (int)j; }
            }
            if (best[0] >= 0 && bd[0] < 1e-24) {
                near[2 * k] = best[0];
                wgt[2 * k] = 1.0;
            } else {
                for (int m = 0; m < 2; ++m)
                    if (best[m] >= 0) { near[2 * k + m] = best[m]; wgt[2 * k + m] = 1.0 / bd[m]; }
            }
        }
        SurfaceBody& sb = c->surf[b];
        sb.nseg = n;
        if (int r = upload(c, &sb.seg, sg, nullptr)) return r;
        if (int r = upload(c, &sb.near, near, nullptr)) return r;
        sb.near_h = near;
        if (int r = upload(c, &sb.wgt, wgt, nullptr)) return r;
        sb.wgt_h = wgt;
    }
    c->surf_cp = static_cast<double*>(dalloc(c, (size_t)maxseg * sizeof(double)));
    c->surf_cf = static_cast<double*>(dalloc(c, (size_t)maxseg * sizeof(double)));
    c->partial_n = std::max(1, (maxseg + 255) / 256);
    size_t need = 0;
    for (const Level& Lv : c->lv) need = std::max(need, (Lv.owned.size() + 255) / 256);
    c->partial_n = std::max<int>(c->partial_n, (int)need);
    c->partial = static_cast<double*>(dalloc(c, (size_t)c->partial_n * 4 * sizeof(double)));
    if (!c->surf_cp || !c->surf_cf || !c->partial) return set_err(c, LBR_ERR_OOM, "surface buffers");
    return 0;
}

int surface_eval(lbr_ctx* c, int body, double* cp, double* cf, double sums[4]) {
    const SurfaceBody& sb = c->surf[body];
    if (int r = eval_wall(c, c->wall_level)) return r;
    const Level& L = c->lv[c->wall_level];
    SurfaceArgs a{};
    a.nseg = sb.nseg;
    a.seg = sb.seg;
    a.near = sb.near;
    a.wgt = sb.wgt;
    a.bstate = L.bout;
    a.bw = nullptr;
    a.u_ref = c->u_ref;
    a.rho_ref = c->cfg.rho_ref;
    a.cp = c->surf_cp;
    a.cf = c->surf_cf;
    a.partial = c->partial;
    const int nb = (sb.nseg + 255) / 256;
    HIPCHK(c, launch_surface(c->prec, a, nb, c->stream));
    std::vector<double> part((size_t)nb * 4);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (cp) HIPCHK(c, hipMemcpyAsync(cp, c->surf_cp, sb.nseg * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (cf) HIPCHK(c, hipMemcpyAsync(cf, c->surf_cf, sb.nseg * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int f = 0; f < 4; ++f) {
        double s = 0.0;
        for (int k = 0; k < nb; ++k) s += part[4 * k + f];
        sums[f] = s;
    }
    return 0;
}

// Advances a case past its start-up ramp through the merged schedule of a
// batch of that case alone (defined with the batch code).
int self_advance(lbr_ctx* c, int64_t n);

}  // namespace

// ===========================================================================
// C entry points
// ===========================================================================
extern "C" {

int lbr_create(const lbr_config* cfg, lbr_ctx** out) {
    if (!out) return LBR_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg || cfg->version != LBR_ABI_VERSION) return LBR_ERR_INVALID_ARG;
    if (cfg->n_levels < 1 || cfg->n_levels > LBR_MAX_LEVELS || cfg->nx0 < 4 || cfg->ny0 < 4 ||
        !(cfg->dx0 > 0) || cfg->storage < 0 || cfg->storage > LBR_STORE_MIXED || cfg->outlet < 0 || cfg->outlet > 2 ||
        cfg->sponge_width < 0 || cfg->sponge_strength < 0 || cfg->sponge_strength > 1 ||
        cfg->ramp_steps < 0 || cfg->ramp_start < 0 || cfg->ramp_start > 1 ||
        cfg->shift16 < 0 || cfg->shift16 > 1 || cfg->health_every < 0)
        return LBR_ERR_INVALID_ARG;
    if ((cfg->bc[0] == LBR_BC_PERIODIC) != (cfg->bc[1] == LBR_BC_PERIODIC) ||
        (cfg->bc[2] == LBR_BC_PERIODIC) != (cfg->bc[3] == LBR_BC_PERIODIC) ||
        cfg->bc[0] == LBR_BC_WALL || cfg->bc[1] == LBR_BC_WALL)
        return LBR_ERR_INVALID_ARG;
    for (int k = 0; k < 4; ++k)
        if (cfg->bc[k] < LBR_BC_PERIODIC || cfg->bc[k] > LBR_BC_WALL) return LBR_ERR_INVALID_ARG;
    if (cfg->wall_model < LBR_WALL_VN || cfg->wall_model > LBR_WALL_PRESCRIBED || cfg->bb < LBR_BB_AUTO ||
        cfg->bb > LBR_BB_HALFWAY || cfg->sa < LBR_SA_FROZEN || cfg->sa > LBR_SA_UPWIND1 ||
        cfg->body_mode < LBR_BODY_SOLID || cfg->body_mode > LBR_BODY_REFINE_ONLY)
        return LBR_ERR_INVALID_ARG;
    // physical parameters: positive density and wall distances, a bulk relaxation
    // frequency of a stable BGK-type rate, finite everything else
    if (!(cfg->rho_ref > 0) || !std::isfinite(cfg->rho_ref) || !(cfg->omega_b > 0 && cfg->omega_b < 2) ||
        !(cfg->d_wr > 0) || !std::isfinite(cfg->d_wr) || !(cfg->d_wv > 0) || !std::isfinite(cfg->d_wv) ||
        !std::isfinite(cfg->chi_inlet) || !std::isfinite(cfg->chi_init) || !std::isfinite(cfg->force[0]) ||
        !std::isfinite(cfg->force[1]) || !std::isfinite(cfg->origin[0]) || !std::isfinite(cfg->origin[1]) ||
        !std::isfinite(cfg->u_ref) || !std::isfinite(cfg->nu0) || !std::isfinite(cfg->dx0) ||
        !std::isfinite(cfg->sponge_width) || !std::isfinite(cfg->ramp_steps) || !std::isfinite(cfg->sa_mu_cap) ||
        !(std::fabs(cfg->alpha_deg) <= 90.0) || !std::isfinite(cfg->alpha_pivot[0]) ||
        !std::isfinite(cfg->alpha_pivot[1]))
        return LBR_ERR_INVALID_ARG;
    // side conditions the step implements: the inlet rule on x-lo, the outlet rules on
    // x-hi, symmetry and channel walls on the y sides (any other pairing would leave
    // the populations entering across that side undefined)
    if ((cfg->bc[0] != LBR_BC_PERIODIC && cfg->bc[0] != LBR_BC_INLET) ||
        (cfg->bc[1] != LBR_BC_PERIODIC && cfg->bc[1] != LBR_BC_OUTLET) ||
        cfg->bc[2] == LBR_BC_INLET || cfg->bc[2] == LBR_BC_OUTLET ||
        cfg->bc[3] == LBR_BC_INLET || cfg->bc[3] == LBR_BC_OUTLET)
        return LBR_ERR_INVALID_ARG;
    for (int l = 1; l < cfg->n_levels; ++l)
        if (!(cfg->band[l] >= 0) || !std::isfinite(cfg->band[l])) return LBR_ERR_INVALID_ARG;
    // global cell indices of the finest level stay well inside 32 bits
    if ((long)cfg->nx0 << (cfg->n_levels - 1) > (1L << 28) || (long)cfg->ny0 << (cfg->n_levels - 1) > (1L << 28))
        return LBR_ERR_INVALID_ARG;
    lbr_ctx* c = new lbr_ctx();
    c->cfg = *cfg;
    c->stream = static_cast<hipStream_t>(cfg->stream);
    // prec selects the arithmetic of the kernels that touch no populations (and the
    // storage of every level unless it is mixed)
    c->prec = cfg->storage == LBR_STORE_MIXED ? P_F32 : static_cast<Prec>(cfg->storage);
    c->ssize = cfg->storage == LBR_STORE_F64 ? 8 : (cfg->storage == LBR_STORE_F16 || cfg->storage == LBR_STORE_BF16 ? 2 : 4);
    c->csize = cfg->storage == LBR_STORE_F64 ? 8 : 4;
    c->u_ref = cfg->u_ref > 0 ? cfg->u_ref : cfg->mach * std::sqrt(1.0 / 3.0);
    c->nu0 = cfg->nu0 > 0 ? cfg->nu0 : c->u_ref * (cfg->ref_length / cfg->dx0) / cfg->reynolds;
    if (!(c->nu0 > 0) || !std::isfinite(c->nu0)) {
        delete c;
        return LBR_ERR_INVALID_ARG;
    }
    if (cfg->shift16) {
        // f_eq_i(rho_ref, u_ref e_x) - w_i of eq (4) (with u_y = 0 only the
        // first- and second-order terms remain)
        static const int cxh[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
        static const double wh[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        const double U = c->u_ref, rho = cfg->rho_ref;
        for (int i = 0; i < 9; ++i) {
            const double cu = cxh[i] * U;
            c->dsh[i] = wh[i] * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * (cu * cu - U * U / 3.0)));
        }
    }
    c->wall_lat[0] = (cfg->wall_y[0] - cfg->origin[1]) / cfg->dx0;
    c->wall_lat[1] = (cfg->wall_y[1] - cfg->origin[1]) / cfg->dx0;
    *out = c;
    return LBR_OK;
}

int lbr_set_geometry(lbr_ctx* c, int32_t n_bodies, const int32_t* n_pts, const double* xy) {
    if (!c) return LBR_ERR_INVALID_ARG;
    if (c->built) return set_err(c, LBR_ERR_STATE, "geometry must be set before lbr_build");
    if (n_bodies < 0 || (n_bodies > 0 && (!n_pts || !xy)))
        return set_err(c, LBR_ERR_INVALID_ARG, "invalid geometry arguments");
    c->npts.clear();
    c->off.assign(1, 0);
    c->polyflat.clear();
    // angle of attack: each point turned by -alpha about the pivot, one product per
    // statement (no fused multiply-add), then mapped to level-0 lattice units
    const double a = -(c->cfg.alpha_deg * (M_PI / 180.0));
    const double ca = std::cos(a), sa = std::sin(a);
    const double px = c->cfg.alpha_pivot[0], py = c->cfg.alpha_pivot[1];
    const bool turn = c->cfg.alpha_deg != 0.0;
    std::vector<double> pt;
    const double* p = xy;
    for (int b = 0; b < n_bodies; ++b) {
        if (n_pts[b] < 3) return set_err(c, LBR_ERR_GEOMETRY, "body %d has fewer than 3 points", b);
        pt.assign(p, p + 2 * n_pts[b]);
        if (turn)
            for (int k = 0; k < n_pts[b]; ++k) {
                const double dx = pt[2 * k] - px, dy = pt[2 * k + 1] - py;
                const double xc = ca * dx, ys = sa * dy, xs = sa * dx, yc = ca * dy;
                const double rx = xc - ys, ry = xs + yc;
                pt[2 * k] = rx + px;
                pt[2 * k + 1] = ry + py;
            }
        double area2 = 0.0;                       // twice the signed area (shoelace)
        for (int k = 0; k < n_pts[b]; ++k) {
            const double x = (pt[2 * k] - c->cfg.origin[0]) / c->cfg.dx0;
            const double y = (pt[2 * k + 1] - c->cfg.origin[1]) / c->cfg.dx0;
            if (!std::isfinite(x) || !std::isfinite(y))
                return set_err(c, LBR_ERR_GEOMETRY, "body %d has a non-finite point", b);
            const int k1 = (k + 1) % n_pts[b];
            area2 += pt[2 * k] * pt[2 * k1 + 1] - pt[2 * k1] * pt[2 * k + 1];
            c->polyflat.push_back(x);
            c->polyflat.push_back(y);
        }
        // the segment tangents, and with them the sign of Cf, follow the
        // counter-clockwise orientation
        if (!(area2 > 0.0))
            return set_err(c, LBR_ERR_GEOMETRY, "body %d is not a counter-clockwise polyline", b);
        p += 2 * n_pts[b];
        c->npts.push_back(n_pts[b]);
        c->off.push_back(c->off.back() + n_pts[b]);
    }
    return LBR_OK;
}

int lbr_set_cut_links(lbr_ctx* c, int32_t level, int64_t n, const double* rec) {
    if (!c) return LBR_ERR_INVALID_ARG;
    if (c->built) return set_err(c, LBR_ERR_STATE, "cut-link lists must be set before lbr_build");
    if (level < 0 || level >= c->cfg.n_levels)
        return set_err(c, LBR_ERR_INVALID_ARG, "level %d outside 0..%d", level, c->cfg.n_levels - 1);
    if (n < 0 || n > ((int64_t)1 << 28) || (n > 0 && !rec))
        return set_err(c, LBR_ERR_INVALID_ARG, "invalid cut-link list arguments");
    char msg[200];
    for (int64_t r = 0; r < n; ++r)
        if (!cut_record_ok(rec + r * LBR_CUT_STRIDE, msg, sizeof msg))
            return set_err(c, LBR_ERR_INVALID_ARG, "level %d, cut-link record %lld: %s", level, (long long)r, msg);
    c->cut_in[level].assign(rec, rec + n * LBR_CUT_STRIDE);
    return LBR_OK;
}

int lbr_load_cut_links(lbr_ctx* c, const char* path) {
    if (!c || !path) return LBR_ERR_INVALID_ARG;
    if (c->built) return set_err(c, LBR_ERR_STATE, "cut-link lists must be set before lbr_build");
    FILE* fp = fopen(path, "rb");
    if (!fp) return set_err(c, LBR_ERR_IO, "cannot open %s", path);
    std::string text;
    char buf[1 << 16];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, got);
    const bool failed = ferror(fp) != 0;
    fclose(fp);
    if (failed) return set_err(c, LBR_ERR_IO, "cannot read %s", path);
    // white-space separated tokens; '#' comments to the end of the line
    size_t i = 0;
    int line = 1;
    std::string tok;
    auto next = [&]() -> bool {
        for (;;) {
            while (i < text.size() && std::isspace((unsigned char)text[i])) {
                if (text[i] == '\n') ++line;
                ++i;
            }
            if (i < text.size() && text[i] == '#') {
                while (i < text.size() && text[i] != '\n') ++i;
                continue;
            }
            break;
        }
        if (i >= text.size()) return false;
        size_t j = i;
        while (j < text.size() && !std::isspace((unsigned char)text[j]) && text[j] != '#') ++j;
        tok.assign(text, i, j - i);
        i = j;
        return true;
    };
    auto number = [&](double* v) -> bool {
        tok.clear();
        if (!next()) return false;
        char* end = nullptr;
        *v = std::strtod(tok.c_str(), &end);
        return end && *end == 0;
    };
    if (!next() || tok != "lbr-cut-links" || !next() || tok != "1")
        return set_err(c, LBR_ERR_INVALID_ARG, "%s: not a cut-link file (header \"lbr-cut-links 1\")", path);
    std::vector<double> lists[LBR_MAX_LEVELS];
    bool seen[LBR_MAX_LEVELS] = {};
    char msg[200];
    while (next()) {
        if (tok != "level")
            return set_err(c, LBR_ERR_INVALID_ARG, "%s:%d: expected \"level\", found \"%s\"", path, line, tok.c_str());
        double lv = -1, cnt = -1;
        if (!number(&lv) || lv != std::floor(lv) || lv < 0 || lv >= c->cfg.n_levels)
            return set_err(c, LBR_ERR_INVALID_ARG, "%s:%d: bad level", path, line);
        if (!number(&cnt) || cnt != std::floor(cnt) || cnt < 0 || cnt > (double)(1 << 28))
            return set_err(c, LBR_ERR_INVALID_ARG, "%s:%d: bad record count", path, line);
        const int l = (int)lv;
        if (seen[l]) return set_err(c, LBR_ERR_INVALID_ARG, "%s:%d: level %d listed twice", path, line, l);
        seen[l] = true;
        const size_t nrec = (size_t)cnt;
        lists[l].resize(nrec * LBR_CUT_STRIDE);
        for (size_t k = 0; k < lists[l].size(); ++k)
            if (!number(&lists[l][k])) {
                if (tok.empty())
                    return set_err(c, LBR_ERR_INVALID_ARG, "%s: level %d: truncated after %zu of %zu values",
                                   path, l, k, lists[l].size());
                return set_err(c, LBR_ERR_INVALID_ARG, "%s:%d: level %d: \"%s\" is not a number", path, line, l,
                               tok.c_str());
            }
        for (size_t r = 0; r < nrec; ++r)
            if (!cut_record_ok(&lists[l][r * LBR_CUT_STRIDE], msg, sizeof msg))
                return set_err(c, LBR_ERR_INVALID_ARG, "%s: level %d, cut-link record %zu: %s", path, l, r, msg);
    }
    for (int l = 0; l < LBR_MAX_LEVELS; ++l)
        if (seen[l]) c->cut_in[l] = std::move(lists[l]);
    return LBR_OK;
}

int lbr_build(lbr_ctx* c) {
    if (!c) return LBR_ERR_INVALID_ARG;
    if (c->built) return set_err(c, LBR_ERR_STATE, "already built");
    // segment table: ax, ay, bx, by, body (level-0 lattice units)
    std::vector<double> seg;
    for (size_t b = 0; b < c->npts.size(); ++b) {
        const int n = c->npts[b], o = c->off[b];
        for (int k = 0; k < n; ++k) {
            const int k1 = (k + 1) % n;
            seg.insert(seg.end(), {c->polyflat[2 * (o + k)], c->polyflat[2 * (o + k) + 1],
                                   c->polyflat[2 * (o + k1)], c->polyflat[2 * (o + k1) + 1], (double)b});
        }
    }
    double* poly_dev = nullptr;
    int* off_dev = nullptr;
    std::vector<double> pf = c->polyflat;
    if (pf.empty()) pf.assign(2, 0.0);
    std::vector<int> of = c->off;
    if (int r = upload(c, &poly_dev, pf, nullptr)) return r;
    if (int r = upload(c, &off_dev, of, nullptr)) return r;
    if (int r = build_levels(c, poly_dev, off_dev)) return r;
    if (int r = check_levels(c)) return r;
    for (Level& L : c->lv) finish_level(c, L);
    for (Level& L : c->lv) {
        const std::vector<double>& given = c->cut_in[L.l];
        if (int r = given.empty() ? build_walls(c, L, seg) : walls_from_list(c, L, given)) return r;
    }
    int cus = 0, dev = 0;                            // compute units, for the tile order
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    for (Level& L : c->lv) {
        // a tile is addressed by 15-bit column and row indices (for every tile
        // height the tuner may pick)
        if (L.box.pitch / TILE_X > 0x7fff || L.box.ny / TILE_YS[0] > 0x7fff)
            return set_err(c, LBR_ERR_INVALID_ARG, "level %d: storage box of %d x %d cells exceeds the tile "
                           "index range (%d columns, %d rows)", L.l, L.box.pitch, L.box.ny, 0x7fff * TILE_X,
                           0x7fff * TILE_YS[0]);
        make_rows(L);
        mark_restriction_tiles(c, L);
        mark_ghost_tiles(L);
        order_tiles(L, cus);
        if (int r = alloc_level(c, L)) return r;
        L.dbody.clear();
        L.dbody.shrink_to_fit();
        L.inside.clear();
        L.inside.shrink_to_fit();
    }
    if (int r = build_surface(c, seg)) return r;
    // the allocation-free entry point's static scratch on this device (looked up
    // once per device, with the device the context runs on current)
    HIPCHK(c, noalloc_scratch(&c->scratch));
    c->built = true;
    for (int l = 0; l < (int)c->lv.size(); ++l)
        if (int r = init_level(c, l, nullptr, nullptr, nullptr, nullptr)) return r;
    for (int l = 0; l + 1 < (int)c->lv.size(); ++l)
        if (int r = do_transfers(c, l)) return r;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBR_OK;
}

int lbr_level_info(lbr_ctx* c, int32_t level, lbr_level_desc* out) {
    if (!c || !out) return LBR_ERR_INVALID_ARG;
    if (!c->built || level < 0 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "bad level %d", level);
    const Level& L = c->lv[level];
    out->gx0 = L.bx0; out->gy0 = L.by0; out->nx = L.bnx; out->ny = L.bny;
    out->n_fluid = L.n_fluid;
    out->n_wall_nodes = (int64_t)L.nodes.size();
    out->n_cut_links = L.n_cut;
    out->n_ghost = L.n_ghost;
    out->n_tiles = (int64_t)L.rows[L.ty].size();
    out->bytes = (int64_t)L.bytes;
    return LBR_OK;
}

int lbr_init_fields(lbr_ctx* c, int32_t level, const double* rho, const double* ux,
                    const double* uy, const double* chi) {
    if (!c) return LBR_ERR_INVALID_ARG;
    if (!c->built || level < 0 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "bad level %d", level);
    if (int r = init_level(c, level, rho, ux, uy, chi)) return r;
    // covered cells of the parent take the mean of the new children; the level's
    // own covered cells the mean of its children
    if (level > 0)
        if (int r = do_transfers(c, level - 1)) return r;
    if (level + 1 < (int)c->lv.size())
        if (int r = do_transfers(c, level)) return r;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBR_OK;
}

static int advance_steps(lbr_ctx* c, int64_t n);

// Health check (lbr_config::health_every): scans of every level's density and
// velocity and of the wall nodes' friction velocity after every health_every-th
// coarse step, read back once at the end of the call.
int lbr_advance(lbr_ctx* c, int64_t n) {
    if (!c) return LBR_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    if (n < 0) return set_err(c, LBR_ERR_INVALID_ARG, "negative step count");
    const int64_t every = c->cfg.health_every;
    if (every <= 0) return advance_steps(c, n);
    if (!c->health) {
        c->health = static_cast<int*>(dalloc(c, 4 * sizeof(int)));
        if (!c->health) return set_err(c, LBR_ERR_OOM, "health check scratch");
    }
    HIPCHK(c, launch_health_reset(c->health, c->stream));
    int64_t k = 0;
    while (k < n) {
        const int64_t m = std::min(every - c->step_count % every, n - k);
        if (int r = advance_steps(c, m)) return r;
        k += m;
        if (c->step_count % every) continue;
        for (Level& L : c->lv) {
            HIPCHK(c, launch_health(c->prec, L.mac[L.cur], L.owned_dev, (int)L.owned.size(), L.box.plane, L.l,
                                    c->health, c->stream));
            HIPCHK(c, launch_health_wall(L.bstate, (int)L.nodes.size(), L.l, c->health, c->stream));
        }
    }
    int h[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(h, c->health, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h[0] & 1)
        return set_err(c, LBR_ERR_DIVERGED, "health check after coarse step %lld: %d cells with a non-finite or "
                       "non-positive density or |u| > c_s (one on level %d, storage index %d)",
                       (long long)c->step_count, h[3], h[1], h[2]);
    if (h[0] & 2)
        return set_err(c, LBR_ERR_NEWTON, "health check after coarse step %lld: non-finite friction velocity "
                       "on level %d (wall node %d)", (long long)c->step_count, h[1], h[2]);
    return LBR_OK;
}

static int advance_steps(lbr_ctx* c, int64_t n) {
    c->ev_used = 0;
    c->prof_launches = 0;
    int64_t k = 0;
    // during the start-up ramp the launch arguments change every step: direct launches
    for (; k < n && (double)c->step_count < c->cfg.ramp_steps; ++k) {
        if (int r = cycle(c, 0, 0)) return r;
        c->step_count++;
    }
    const int64_t ramp_done = k;
    if (k < n && (c->use_graph || c->prof)) {
        // the merged schedule keeps its own step and residual counts
        if (int r = self_advance(c, n - k)) return r;
        c->resid_steps += ramp_done;
        return LBR_OK;
    }
    for (; k < n; ++k) {
        if (int r = cycle(c, 0, 0)) return r;
        c->step_count++;
    }
    c->resid_steps += n;
    if (c->prof && c->ev_used) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double sum[4] = {0, 0, 0, 0};
        int cnt[4] = {0, 0, 0, 0};
        for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
            const int kind = c->ev_kind[i];
            sum[kind] += ms;
            cnt[kind]++;
            if (kind != EV_STEP) { sum[EV_STEP] += ms; cnt[EV_STEP]++; }
        }
        for (int f = 0; f < 3; ++f) c->prof_out[f] = cnt[f] ? 1000.0 * sum[f] / cnt[f] : 0.0;
        c->prof_out[3] = n ? (double)c->prof_launches / (double)n : 0.0;
    }
    return LBR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// checkpoint: both time levels of every field, the wall-model state and the
// step counter, behind a header that pins the grid the data belongs to
// ---------------------------------------------------------------------------
namespace {

constexpr char CKPT_MAGIC[8] = {'L', 'B', 'R', 'S', 'T', 'A', 'T', '1'};

struct CkptHead {
    char magic[8];
    int32_t abi, prec, n_levels, ssize, csize, reserved;
    int64_t step_count;
};

struct CkptLevel {
    int64_t pitch, ny, plane, gx0, gy0, n_fluid, n_nodes;
    uint64_t flag_hash;
    int32_t cur, storage;
};

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

CkptLevel ckpt_level(const Level& L) {
    CkptLevel d{};
    d.pitch = L.box.pitch;
    d.ny = L.box.ny;
    d.plane = L.box.plane;
    d.gx0 = L.box.gx0;
    d.gy0 = L.box.gy0;
    d.n_fluid = L.n_fluid;
    d.n_nodes = (int64_t)L.nodes.size();
    d.flag_hash = fnv1a(L.flag.data(), L.flag.size());
    d.cur = L.cur;
    d.storage = (int32_t)L.st;
    return d;
}

// device regions of one level, in file order
std::vector<std::pair<void*, size_t>> ckpt_regions(lbr_ctx* c, Level& L) {
    const size_t n = (size_t)L.box.plane;
    std::vector<std::pair<void*, size_t>> r;
    for (int b = 0; b < 2; ++b) r.push_back({L.f[b], 9 * n * L.ssize});
    for (int b = 0; b < 2; ++b) r.push_back({L.mac[b], 3 * n * c->csize});
    for (int b = 0; b < 2; ++b) r.push_back({L.chi[b], n * c->csize});
    r.push_back({L.bstate, std::max<size_t>(L.nodes.size(), 1) * 8 * sizeof(double)});
    return r;
}

struct File {
    FILE* f = nullptr;
    ~File() { if (f) fclose(f); }
};

}  // namespace

extern "C" {

int lbr_save(lbr_ctx* c, const char* path) {
    if (!c || !path) return LBR_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    File fh;
    fh.f = fopen(path, "wb");
    if (!fh.f) return set_err(c, LBR_ERR_IO, "cannot open %s for writing", path);
    CkptHead h{};
    memcpy(h.magic, CKPT_MAGIC, 8);
    h.abi = LBR_ABI_VERSION;
    h.prec = (int32_t)c->cfg.storage;
    h.n_levels = (int32_t)c->lv.size();
    h.ssize = (int32_t)c->ssize;
    h.csize = (int32_t)c->csize;
    h.reserved = c->cfg.shift16;
    h.step_count = c->step_count;
    bool ok = fwrite(&h, sizeof h, 1, fh.f) == 1;
    for (const Level& L : c->lv) {
        const CkptLevel d = ckpt_level(L);
        ok = ok && fwrite(&d, sizeof d, 1, fh.f) == 1;
    }
    std::vector<unsigned char> host;
    uint64_t sum = 1469598103934665603ull;
    for (Level& L : c->lv)
        for (const auto& reg : ckpt_regions(c, L)) {
            host.resize(reg.second);
            HIPCHK(c, hipMemcpyAsync(host.data(), reg.first, reg.second, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            sum = fnv1a(host.data(), host.size(), sum);
            ok = ok && fwrite(host.data(), 1, host.size(), fh.f) == host.size();
        }
    ok = ok && fwrite(&sum, sizeof sum, 1, fh.f) == 1;
    const bool closed = fclose(fh.f) == 0;
    fh.f = nullptr;
    if (!ok || !closed) return set_err(c, LBR_ERR_IO, "write to %s failed", path);
    return LBR_OK;
}

int lbr_load(lbr_ctx* c, const char* path) {
    if (!c || !path) return LBR_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    File fh;
    fh.f = fopen(path, "rb");
    if (!fh.f) return set_err(c, LBR_ERR_IO, "cannot open %s", path);
    CkptHead h{};
    if (fread(&h, sizeof h, 1, fh.f) != 1 || memcmp(h.magic, CKPT_MAGIC, 8) != 0)
        return set_err(c, LBR_ERR_IO, "%s is not a checkpoint of this library", path);
    if (h.abi != LBR_ABI_VERSION || h.prec != (int32_t)c->cfg.storage || h.n_levels != (int32_t)c->lv.size() ||
        h.ssize != (int32_t)c->ssize || h.csize != (int32_t)c->csize || h.reserved != c->cfg.shift16)
        return set_err(c, LBR_ERR_INVALID_ARG, "checkpoint %s: different library version, storage or level count",
                       path);
    std::vector<CkptLevel> lv(c->lv.size());
    for (size_t l = 0; l < lv.size(); ++l) {
        if (fread(&lv[l], sizeof lv[l], 1, fh.f) != 1) return set_err(c, LBR_ERR_IO, "checkpoint %s truncated", path);
        const CkptLevel mine = ckpt_level(c->lv[l]);
        if (lv[l].pitch != mine.pitch || lv[l].ny != mine.ny || lv[l].plane != mine.plane ||
            lv[l].gx0 != mine.gx0 || lv[l].gy0 != mine.gy0 || lv[l].n_fluid != mine.n_fluid ||
            lv[l].n_nodes != mine.n_nodes || lv[l].flag_hash != mine.flag_hash || lv[l].storage != mine.storage ||
            (lv[l].cur != 0 && lv[l].cur != 1))
            return set_err(c, LBR_ERR_INVALID_ARG, "checkpoint %s: level %d was saved on a different grid",
                           path, (int)l);
    }
    // read and verify everything before the device state changes
    std::vector<std::vector<unsigned char>> data;
    uint64_t sum = 1469598103934665603ull;
    for (Level& L : c->lv)
        for (const auto& reg : ckpt_regions(c, L)) {
            data.emplace_back(reg.second);
            if (fread(data.back().data(), 1, reg.second, fh.f) != reg.second)
                return set_err(c, LBR_ERR_IO, "checkpoint %s truncated", path);
            sum = fnv1a(data.back().data(), reg.second, sum);
        }
    uint64_t stored = 0;
    if (fread(&stored, sizeof stored, 1, fh.f) != 1 || stored != sum)
        return set_err(c, LBR_ERR_IO, "checkpoint %s: checksum mismatch", path);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    size_t k = 0;
    for (Level& L : c->lv)
        for (const auto& reg : ckpt_regions(c, L)) {
            HIPCHK(c, hipMemcpyAsync(reg.first, data[k].data(), reg.second, hipMemcpyHostToDevice, c->stream));
            ++k;
        }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t l = 0; l < lv.size(); ++l) c->lv[l].cur = lv[l].cur;
    c->step_count = h.step_count;
    c->resid_init = false;
    c->resid_steps = 0;
    return LBR_OK;
}

int lbr_synchronize(lbr_ctx* c) {
    if (!c) return LBR_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBR_OK;
}

int lbr_read_field(lbr_ctx* c, int32_t level, int32_t field, double* dst) {
    if (!c || !dst) return LBR_ERR_INVALID_ARG;
    if (!c->built || level < 0 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "bad level %d", level);
    if (field < 0 || field > LBR_FIELD_DIST) return set_err(c, LBR_ERR_INVALID_ARG, "bad field %d", field);
    Level& L = c->lv[level];
    const long n = L.box.plane;
    std::vector<double> v;
    if (field == LBR_FIELD_RHO || field == LBR_FIELD_UX || field == LBR_FIELD_UY ||
        field == LBR_FIELD_CHI || field == LBR_FIELD_NUT) {
        const void* src = nullptr;
        if (field == LBR_FIELD_CHI || field == LBR_FIELD_NUT) src = L.chi[L.cur];
        else src = static_cast<const char*>(L.mac[L.cur]) + (size_t)field * n * c->csize;
        double* tmp = static_cast<double*>(dalloc(c, n * sizeof(double)));
        if (!tmp) return set_err(c, LBR_ERR_OOM, "readout scratch");
        v.resize(n);
        hipError_t e = launch_to_double(c->prec, src, tmp, n, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(v.data(), tmp, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        dfree(c, tmp);
        if (e != hipSuccess) return set_err(c, LBR_ERR_HIP, "field readout: %s", hipGetErrorString(e));
    } else {
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    const double cv3 = 7.1 * 7.1 * 7.1;
    for (int j = 0; j < L.bny; ++j)
        for (int i = 0; i < L.bnx; ++i) {
            const long k = L.idx(L.bx0 + i, L.by0 + j);
            double& o = dst[(long)j * L.bnx + i];
            const int t = L.flag[k] & F_TYPE;
            if (field == LBR_FIELD_TYPE) { o = t; continue; }
            if (t != T_FLUID) { o = NAN; continue; }
            if (field == LBR_FIELD_DIST) { o = L.d[k]; continue; }
            if (field == LBR_FIELD_NUT) {
                const double x = v[k];
                o = x > 0 ? L.nu * x * x * x * x / (x * x * x + cv3) : 0.0;
                continue;
            }
            o = v[k];
        }
    return LBR_OK;
}

int lbr_read_field_device(lbr_ctx* c, int32_t level, int32_t field, double* dst, int64_t capacity) {
    if (!c || !dst) return LBR_ERR_INVALID_ARG;
    if (!c->built || level < 0 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "bad level %d", level);
    if (field < 0 || field > LBR_FIELD_DIST) return set_err(c, LBR_ERR_INVALID_ARG, "bad field %d", field);
    Level& L = c->lv[level];
    if (capacity < (int64_t)L.bnx * L.bny)
        return set_err(c, LBR_ERR_INVALID_ARG, "level %d needs %lld doubles", level, (long long)L.bnx * L.bny);
    FieldArgs a{};
    const size_t pb = (size_t)L.box.plane * c->csize;
    if (field == LBR_FIELD_CHI || field == LBR_FIELD_NUT) a.src = L.chi[L.cur];
    else if (field <= LBR_FIELD_UY) a.src = static_cast<const char*>(L.mac[L.cur]) + (size_t)field * pb;
    a.dist = L.dist_dev;
    a.flag = L.flag_dev;
    a.pitch = L.box.pitch;
    a.ox = L.bx0 - L.box.gx0;
    a.oy = L.by0 - L.box.gy0;
    a.bnx = L.bnx;
    a.bny = L.bny;
    a.field = field;
    a.nu = L.nu;
    a.out = dst;
    HIPCHK(c, launch_field(c->prec, a, c->stream));
    return LBR_OK;
}

int lbr_wall_count(lbr_ctx* c, int32_t level) {
    if (!c || !c->built || level < 0 || level >= (int)c->lv.size()) return LBR_ERR_INVALID_ARG;
    return (int)c->lv[level].nodes.size();
}

int lbr_read_wall(lbr_ctx* c, int32_t level, double* dst) {
    if (!c || !dst) return LBR_ERR_INVALID_ARG;
    if (!c->built || level < 0 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "bad level %d", level);
    Level& L = c->lv[level];
    const int nb = (int)L.nodes.size();
    if (nb == 0) return LBR_OK;
    std::vector<double> st((size_t)nb * 8);
    if (int r = eval_wall(c, level)) return r;
    HIPCHK(c, hipMemcpyAsync(st.data(), L.bout, st.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double U = c->u_ref, rr = c->cfg.rho_ref;
    for (int b = 0; b < nb; ++b) {
        const Node& nd = L.nodes[b];
        double* o = dst + (size_t)b * LBR_WALL_STRIDE;
        int ncut = 0;
        for (int i = 1; i < 9; ++i) ncut += nd.q[i] >= 0;
        const double utau = st[8 * b], tx = st[8 * b + 1], ty = st[8 * b + 2], rhow = st[8 * b + 3];
        const double uwx = st[8 * b + 4], uwy = st[8 * b + 5];
        o[0] = nd.gi; o[1] = nd.gj; o[2] = nd.iw[0]; o[3] = nd.iw[1];
        o[4] = nd.nrm[0]; o[5] = nd.nrm[1]; o[6] = nd.dwb; o[7] = ncut;
        o[8] = utau; o[9] = uwx; o[10] = uwy; o[11] = rhow;
        o[12] = std::sqrt(tx * tx + ty * ty);
        o[13] = 2.0 / 3.0 * (rhow - rr) / (rr * U * U);
        o[14] = 2.0 * (rhow / rr) * (utau / U) * (utau / U);
        o[15] = nd.body;
        o[16] = (c->cfg.wall_model == LBR_WALL_VN || c->cfg.wall_model == LBR_WALL_NISHIMURA)
                    ? KAPPA_H * utau * nd.dwb / L.nu : 0.0;
        o[17] = tx; o[18] = ty;
        for (int i = 1; i < 9; ++i) o[18 + i] = nd.q[i];
        o[27] = 0.0;
    }
    return LBR_OK;
}

int lbr_wall_yplus(lbr_ctx* c, int32_t level, double* dst) {
    if (!c || !dst) return LBR_ERR_INVALID_ARG;
    if (!c->built || level < 0 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "bad level %d", level);
    Level& L = c->lv[level];
    const int nb = (int)L.nodes.size();
    if (nb == 0) return LBR_OK;
    if (int r = eval_wall(c, level)) return r;
    std::vector<double> st((size_t)nb * 8);
    HIPCHK(c, hipMemcpyAsync(st.data(), L.bout, st.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // wall distances of R, B and V in lattice units of the level
    const double dwr = c->cfg.wall_model == LBR_WALL_NISHIMURA ? 1.75 : c->cfg.d_wr, dwv = c->cfg.d_wv;
    for (int b = 0; b < nb; ++b) {
        const double s = st[8 * b] / L.nu;                      // u_tau / nu
        dst[3 * b + 0] = s * dwr;
        dst[3 * b + 1] = s * L.nodes[b].dwb;
        dst[3 * b + 2] = s * dwv;
    }
    return LBR_OK;
}

static_assert(((size_t)LBR_RAKE_NOALLOC_MAX * sizeof(int64_t) + 255) / 256 * 256 +
                  (size_t)LBR_RAKE_NOALLOC_MAX * 4 * sizeof(double) <= NOALLOC_SCRATCH_BYTES,
              "the rake's gather indices and values fit the static scratch");

// Rake readout of lbr_rake and lbr_rake_noalloc: the gather indices and values of
// one level at a time go through buffers allocated per call, or through the
// static scratch (noalloc); every level's copies finish before the next level.
static int rake_impl(lbr_ctx* c, double x0, double y0, double x1, double y1, int32_t n, double* dst,
                     bool noalloc) {
    const int nl = (int)c->lv.size();
    std::vector<int> lev(n, -1);
    std::vector<int64_t> cell(n, -1);
    for (int k = 0; k < n; ++k) {
        const double t = n > 1 ? (double)k / (double)(n - 1) : 0.0;
        const double x = x0 + t * (x1 - x0), y = y0 + t * (y1 - y0);
        for (int l = nl - 1; l >= 0; --l) {
            const double dx = c->cfg.dx0 / (double)(1 << l);
            const double fx = std::floor((x - c->cfg.origin[0]) / dx), fy = std::floor((y - c->cfg.origin[1]) / dx);
            if (!(std::fabs(fx) < 1e9 && std::fabs(fy) < 1e9)) break;     // far outside, or not finite
            const Level& L = c->lv[l];
            if (L.type_at((int)fx, (int)fy) == T_FLUID) {
                lev[k] = l;
                cell[k] = L.idx((int)fx, (int)fy);
                break;
            }
        }
    }
    for (int k = 0; k < n; ++k) {
        dst[5 * k] = lev[k];
        for (int f = 1; f < 5; ++f) dst[5 * k + f] = NAN;
    }
    for (int l = 0; l < nl; ++l) {
        std::vector<int64_t> idx;
        std::vector<int> who;
        for (int k = 0; k < n; ++k)
            if (lev[k] == l) { idx.push_back(cell[k]); who.push_back(k); }
        if (idx.empty()) continue;
        const int m = (int)idx.size();
        Level& L = c->lv[l];
        int64_t* didx;
        double* dout;
        if (noalloc) {
            didx = static_cast<int64_t*>(c->scratch);
            dout = reinterpret_cast<double*>(static_cast<char*>(c->scratch) +
                                             ((size_t)m * sizeof(int64_t) + 255) / 256 * 256);
        } else {
            didx = static_cast<int64_t*>(dalloc(c, (size_t)m * sizeof(int64_t)));
            dout = static_cast<double*>(dalloc(c, (size_t)m * 4 * sizeof(double)));
            if (!didx || !dout) { dfree(c, didx); dfree(c, dout); return set_err(c, LBR_ERR_OOM, "rake scratch"); }
        }
        std::vector<double> v((size_t)m * 4);
        int r = 0;
        const char* mac = static_cast<const char*>(L.mac[L.cur]);
        const size_t pb = (size_t)L.box.plane * c->csize;
        if (hipMemcpyAsync(didx, idx.data(), idx.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            launch_gather(c->prec, mac, didx, m, dout, c->stream) != hipSuccess ||
            launch_gather(c->prec, mac + pb, didx, m, dout + m, c->stream) != hipSuccess ||
            launch_gather(c->prec, mac + 2 * pb, didx, m, dout + 2 * m, c->stream) != hipSuccess ||
            launch_gather(c->prec, L.chi[L.cur], didx, m, dout + 3 * m, c->stream) != hipSuccess ||
            hipMemcpyAsync(v.data(), dout, v.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            r = set_err(c, LBR_ERR_HIP, "rake readout failed");
        if (!noalloc) {
            dfree(c, didx);
            dfree(c, dout);
        }
        if (r) return r;
        const double cv13 = 7.1 * 7.1 * 7.1;
        for (int j = 0; j < m; ++j) {
            double* o = dst + 5 * who[j];
            const double chi = v[3 * m + j];
            o[1] = v[m + j] / c->u_ref;
            o[2] = v[2 * m + j] / c->u_ref;
            o[3] = chi > 0.0 ? chi * chi * chi * chi / (chi * chi * chi + cv13) : 0.0;   // nu_t / nu = chi f_v1
            o[4] = v[j];
        }
    }
    return LBR_OK;
}

int lbr_rake(lbr_ctx* c, double x0, double y0, double x1, double y1, int32_t n, double* dst) {
    if (!c || !dst || n < 1) return LBR_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    return rake_impl(c, x0, y0, x1, y1, n, dst, false);
}

int lbr_rake_noalloc(lbr_ctx* c, double x0, double y0, double x1, double y1, int32_t n, double* dst) {
    if (!c || !dst || n < 1) return LBR_ERR_INVALID_ARG;
    if (!c->built || !c->scratch) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    if (n > LBR_RAKE_NOALLOC_MAX)
        return set_err(c, LBR_ERR_INVALID_ARG, "lbr_rake_noalloc takes at most %d points (%d given): "
                       "its static scratch holds no more", LBR_RAKE_NOALLOC_MAX, n);
    return rake_impl(c, x0, y0, x1, y1, n, dst, true);
}

int lbr_surface(lbr_ctx* c, int32_t body, double* cp, double* cf) {
    if (!c || !c->built) return LBR_ERR_INVALID_ARG;
    if (body < 0 || body >= (int)c->surf.size() || c->wall_level < 0)
        return set_err(c, LBR_ERR_INVALID_ARG, "bad body %d", body);
    double sums[4];
    return surface_eval(c, body, cp, cf, sums);
}

int lbr_surface_yplus(lbr_ctx* c, int32_t body, double* yplus_v) {
    if (!c || !c->built || !yplus_v) return LBR_ERR_INVALID_ARG;
    if (body < 0 || body >= (int)c->surf.size() || c->wall_level < 0)
        return set_err(c, LBR_ERR_INVALID_ARG, "bad body %d", body);
    const SurfaceBody& sb = c->surf[body];
    Level& L = c->lv[c->wall_level];
    const int nb = (int)L.nodes.size();
    std::vector<double> st((size_t)std::max(nb, 1) * 8, 0.0);
    if (nb > 0) {
        if (int r = eval_wall(c, c->wall_level)) return r;
        HIPCHK(c, hipMemcpyAsync(st.data(), L.bout, (size_t)nb * 8 * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    // y+ of V at each node, then the weights and order of the Cp / Cf interpolation
    const double dwv = c->cfg.d_wv;
    for (int k = 0; k < sb.nseg; ++k) {
        double sw = 0.0, sy = 0.0;
        for (int m = 0; m < 2; ++m) {
            const int b = sb.near_h[2 * k + m];
            if (b < 0) continue;
            const double w = sb.wgt_h[2 * k + m];
            sw += w;
            sy += w * (st[8 * b] / L.nu * dwv);
        }
        yplus_v[k] = sw > 0.0 ? sy / sw : 0.0;
    }
    return LBR_OK;
}

int lbr_forces(lbr_ctx* c, int32_t body, double out[5]) {
    if (!c || !c->built || !out) return LBR_ERR_INVALID_ARG;
    if (body >= (int)c->surf.size() || c->wall_level < 0)
        return set_err(c, LBR_ERR_INVALID_ARG, "bad body %d", body);
    double acc[4] = {0, 0, 0, 0};
    const int b0 = body < 0 ? 0 : body, b1 = body < 0 ? (int)c->surf.size() : body + 1;
    for (int b = b0; b < b1; ++b) {
        double s[4];
        if (int r = surface_eval(c, b, nullptr, nullptr, s)) return r;
        for (int f = 0; f < 4; ++f) acc[f] += s[f];
    }
    out[0] = acc[0];              // C_Df
    out[1] = acc[2];              // C_Dp
    out[2] = acc[0] + acc[2];     // C_D
    out[3] = acc[3];              // C_L (pressure)
    out[4] = acc[1];              // friction along y
    return LBR_OK;
}

int lbr_residual(lbr_ctx* c, double* residual) {
    if (!c || !c->built || !residual) return LBR_ERR_INVALID_ARG;
    double du = 0.0, uu = 0.0;
    for (Level& L : c->lv) {
        const int n = (int)L.owned.size();
        if (!n) continue;
        const int nb = (n + 255) / 256;
        const double area = 1.0 / (L.scale * L.scale);
        HIPCHK(c, launch_residual(c->prec, L.mac[L.cur], L.snap, L.owned_dev, n, L.box.plane, area,
                                  c->partial, nb, c->stream));
        std::vector<double> part((size_t)nb * 2);
        HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int k = 0; k < nb; ++k) { du += part[2 * k]; uu += part[2 * k + 1]; }
    }
    if (!c->resid_init || c->resid_steps == 0) {
        *residual = 1.0;
    } else {
        *residual = std::sqrt(du / uu) / (double)c->resid_steps;
    }
    // the first call compares against a snapshot that does not exist yet (the
    // buffer holds whatever the allocator returned): only the state counts
    if (!std::isfinite(uu) || (c->resid_init && !std::isfinite(du)))
        return set_err(c, LBR_ERR_DIVERGED, "non-finite velocity field");
    c->resid_init = true;
    c->resid_steps = 0;
    return LBR_OK;
}

int lbr_run_to_steady(lbr_ctx* c, double tol, int64_t max_steps, int64_t check_every,
                      int64_t* steps_done, double* residual) {
    if (!c || !c->built || check_every <= 0) return LBR_ERR_INVALID_ARG;
    double r = 1.0;
    if (int e = lbr_residual(c, &r)) return e;
    int64_t done = 0;
    while (done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        if (int e = lbr_advance(c, k)) return e;
        done += k;
        if (int e = lbr_residual(c, &r)) {
            if (steps_done) *steps_done = done;
            if (residual) *residual = r;
            return e;
        }
        if (r < tol) break;
    }
    if (steps_done) *steps_done = done;
    if (residual) *residual = r;
    if (!(r < tol))
        return set_err(c, LBR_ERR_NOT_CONVERGED, "residual %.3e after %lld coarse steps (tolerance %.3e)", r,
                       (long long)done, tol);
    return LBR_OK;
}

int64_t lbr_lups_per_coarse_step(lbr_ctx* c) {
    if (!c || !c->built) return 0;
    int64_t n = 0;
    for (const Level& L : c->lv) n += L.n_fluid << L.l;
    return n;
}

int lbr_use_graph(lbr_ctx* c, int32_t enable) {
    if (!c) return LBR_ERR_INVALID_ARG;
    // the legacy default stream cannot be captured into a graph
    if (enable && !c->stream)
        return set_err(c, LBR_ERR_INVALID_ARG, "graph replay needs a stream other than the default stream");
    c->use_graph = enable != 0;
    return LBR_OK;
}

int lbr_profile(lbr_ctx* c, int32_t enable, double out[4]) {
    if (!c) return LBR_ERR_INVALID_ARG;
    c->prof = enable != 0;
    if (out)
        for (int f = 0; f < 4; ++f) out[f] = c->prof_out[f];
    return LBR_OK;
}

const char* lbr_last_error(const lbr_ctx* c) { return c ? c->err.c_str() : "null context"; }

void lbr_destroy(lbr_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    lbr_batch_destroy(c->self);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (void* p : c->allocs) {
        if (c->cfg.free_fn) c->cfg.free_fn(p, c->cfg.alloc_user);
        else (void)hipFree(p);
    }
    delete c;
}

}  // extern "C"

// ===========================================================================
// Batched sweep: several cases advanced by shared launches
// ===========================================================================
struct lbr_batch {
    std::vector<lbr_ctx*> all;         // the cases, in the caller's order
    std::vector<lbr_ctx*> cases;       // the cases the launch tables cover
    int lmax = 0;
    bool merge = true;                 // coarse launches ride along with finer ones
    hipStream_t stream = nullptr;
    // one launch: its StepArgs start at byte off of the table, its part starts
    // at index part0; st is the population storage of all its parts, or
    // P_MIXED for FP32 and FP16 parts of mixed storage; v is the virtual level
    // of its finest part
    struct Launch { size_t off; int part0, nparts, nblocks, v; Prec st; int ty; };
    std::vector<Launch> launches;      // the launches of all tables, in order
    // tables: [0] one super step from parity 0, [1] one from parity 1, [2] two
    // from parity 0; each ends with every launch of its super steps issued
    int table[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    void* parts_dev = nullptr;         // StepArgs of every part of every launch
    int* start_dev = nullptr;          // first block of each part, relative to its launch
    int parity = 0;                    // super steps advanced since the tables were built, modulo 2
    std::vector<int> cur0;             // level-0 buffer index of each covered case at parity 0
    std::vector<hipEvent_t> ev;        // ordering between the case streams and the batch stream
    bool use_graph = false;
    // persistent mode (lbr_batch_use_persistent): each table runs as one cooperative
    // grid with barriers between its launches; tables built with 64 x PERSISTENT_TY tiles
    bool persistent = false;
    PLaunch* plaunch_dev = nullptr;    // one entry per launch of the tables, in order
    unsigned* bar_dev = nullptr;       // grid barrier counters (BAR_WORDS words) and time-out flag
    int pgrid = 0;                     // co-resident workgroups of the persistent grid
    Prec pst = P_F32;                  // the one population format of a persistent batch
    bool ready = false;                // launch tables built and uploaded
    hipGraphExec_t graph = nullptr;    // table 2
    bool prof = false;                 // start / stop events on every launch
    std::vector<hipEvent_t> pev;
    std::vector<int> pev_v;            // virtual level of each event pair
    size_t pev_used = 0;
    int64_t prof_launches = 0;         // launches of the last timed call (timed or not)
    double prof_out[4] = {0, 0, 0, 0};
    std::string err;
};

namespace {

int bset_err(lbr_batch* b, int code, const char* msg) {
    b->err = msg;
    return code;
}

// Virtual level v of the batch is level v - (lmax - L_k) of case k: every case's
// finest level is stepped by the same launches, and a case with fewer levels
// takes 2^(lmax - L_k) of its coarse steps per super step.
void batch_schedule(lbr_batch* b, int v, int substep, std::vector<std::pair<int, int>>& seq) {
    if (v + 1 < b->lmax) {
        batch_schedule(b, v + 1, 1, seq);
        batch_schedule(b, v + 1, 2, seq);
    }
    seq.push_back({v, substep});
}

// One level sub-step of the recursive cycle over every covered case: the
// StepArgs of each case's part and its block count.
struct Item {
    int v;
    Prec st;
    size_t size = 0;                   // bytes of one part's StepArgs
    std::vector<unsigned char> args;   // parts, back to back
    std::vector<int> blocks;
};

// Two items can share a launch when their populations have the same format, or
// are the FP32 and FP16 levels of mixed storage (the mixed kernel picks the
// instantiation per part).
bool shares_launch(Prec a, Prec b) {
    return a == b || ((a == P_F32 || a == P_F16) && (b == P_F32 || b == P_F16));
}

// Launch groups of items [begin, end), in order.  An item of a virtual level at
// least three below the finest is deferred and joins a later launch of a finer
// level (whose format it shares), at most one deferred item per launch: a
// launch of the finest level takes a deferred item of the level three below
// it, a launch of the level below the finest one of a level at least four
// below the finest.  The second kind of launch fills only part of the device,
// so the coarse work it takes costs little there.
// This keeps every dependency of the recursive cycle: an item of level w reads
// its parent w - 1 (explosion, ghost values) and its child w + 1
// (coalescence, restriction) and writes only level w and the restriction into
// w - 1, so two items of levels at least two apart may run in either order or
// together.  A deferred item joins a launch of a level at least w + 2, and it
// may pass earlier deferred items only if it is independent of each of them;
// before any later item of level w + 1, the pending items up to the last one
// of level w are launched on their own, in order.  The buffers each item
// addresses are those of its place in the unmerged cycle, which the merged
// order preserves.
std::vector<std::vector<int>> batch_groups(const lbr_batch* b, const std::vector<Item>& it, int begin, int end) {
    std::vector<std::vector<int>> g;
    std::vector<int> pend;                                   // deferred items, in order
    for (int k = begin; k < end; ++k) {
        const Item& x = it[k];
        if (b->merge && x.v <= b->lmax - 3) {
            pend.push_back(k);
            continue;
        }
        size_t last = 0;
        for (size_t j = 0; j < pend.size(); ++j)
            if (it[pend[j]].v == x.v - 1) last = j + 1;
        for (size_t j = 0; j < last; ++j) g.push_back({pend[j]});
        pend.erase(pend.begin(), pend.begin() + last);
        int pick = -1;
        for (size_t j = 0; j < pend.size() && pick < 0; ++j) {
            const int w = it[pend[j]].v;
            const bool kind = x.v == b->lmax - 1 ? w == b->lmax - 3 : w <= x.v - 2;
            bool free = kind && shares_launch(it[pend[j]].st, x.st);
            for (size_t i = 0; i < j && free; ++i) free = std::abs(it[pend[i]].v - w) >= 2;
            if (free) pick = (int)j;
        }
        if (pick >= 0) {
            g.push_back({k, pend[pick]});
            pend.erase(pend.begin() + pick);
        } else {
            g.push_back({k});
        }
    }
    for (int k : pend) g.push_back({k});
    return g;
}

// Fills the arguments of items [a, e) with tile heights tk, in the unmerged
// order, from the current state advanced by the items [0, a): the host replays
// the buffer flips each launch makes, then restores every buffer index and step
// counter.
int batch_fill(lbr_batch* b, std::vector<Item>& it, int a, int e, const std::vector<int>& tk,
               const std::vector<std::pair<int, int>>& seq2) {
    std::vector<std::vector<int>> cur0;
    std::vector<int64_t> steps0;
    for (lbr_ctx* c : b->cases) {
        cur0.emplace_back();
        for (const Level& L : c->lv) cur0.back().push_back(L.cur);
        steps0.push_back(c->step_count);
    }
    alignas(16) unsigned char buf[sizeof(StepArgs<double, double>)];
    int err = 0;
    for (int k = 0; k < e && !err; ++k) {
        const int v = seq2[k].first;
        Item& x = it[k];
        if (k >= a) { x.args.clear(); x.blocks.clear(); }
        for (lbr_ctx* c : b->cases) {
            const int l = v - (b->lmax - (int)c->lv.size());
            if (l < 0) continue;
            Level& L = c->lv[l];
            if (k >= a) {
                const int sub = l == 0 ? 0 : seq2[k].second;  // a case's level 0 has no parent
                int wb = 0, tb = 0;
                switch (L.st) {
                    case P_F64: { auto& s = *reinterpret_cast<StepArgs<double, double>*>(buf);
                        fill_step_args(c, l, sub, s, tk[k]); wb = s.wall_blocks; tb = s.tile_blocks; x.size = sizeof s; break; }
                    case P_F32: { auto& s = *reinterpret_cast<StepArgs<float, float>*>(buf);
                        fill_step_args(c, l, sub, s, tk[k]); wb = s.wall_blocks; tb = s.tile_blocks; x.size = sizeof s; break; }
                    case P_F16: { auto& s = *reinterpret_cast<StepArgs<__half, float>*>(buf);
                        fill_step_args(c, l, sub, s, tk[k]); wb = s.wall_blocks; tb = s.tile_blocks; x.size = sizeof s; break; }
                    default: { auto& s = *reinterpret_cast<StepArgs<__hip_bfloat16, float>*>(buf);
                        fill_step_args(c, l, sub, s, tk[k]); wb = s.wall_blocks; tb = s.tile_blocks; x.size = sizeof s; break; }
                }
                // parts start on multiples of 8 blocks, so that each part's own
                // block-to-XCD mapping holds inside the shared grid
                const int nt = TILE_X * TILE_YS[tk[k]];
                const int eb = 8 * (((int)L.edge.size() + 8 * nt - 1) / (8 * nt));
                x.args.insert(x.args.end(), buf, buf + x.size);
                x.blocks.push_back(wb + tb + eb);
            }
            L.cur ^= 1;                                       // as the launch will
            if (l == 0) c->step_count++;
        }
    }
    for (size_t i = 0; i < b->cases.size(); ++i) {
        lbr_ctx* c = b->cases[i];
        for (size_t l = 0; l < c->lv.size(); ++l) c->lv[l].cur = cur0[i][l];
        c->step_count = steps0[i];
    }
    return err;
}

// Launch tables for the covered cases from their current state.  Each table's
// groups decide the tile height of every item (a merged launch takes its main
// part's); the arguments are then filled for that table.
int batch_build(lbr_batch* b) {
    int cus = 0, dev = 0;                            // compute units, for the part order
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    std::vector<std::pair<int, int>> seq;
    batch_schedule(b, 0, 0, seq);
    const int per = (int)seq.size();
    std::vector<std::pair<int, int>> seq2(seq);
    seq2.insert(seq2.end(), seq.begin(), seq.end());
    // storage and tile height of every virtual level (the first case that has it decides)
    std::vector<Prec> stv(b->lmax, P_F32);
    std::vector<int> tyv(b->lmax, -1);
    for (int v = 0; v < b->lmax; ++v)
        for (lbr_ctx* c : b->cases) {
            const int l = v - (b->lmax - (int)c->lv.size());
            if (l < 0) continue;
            if (tyv[v] < 0) { stv[v] = c->lv[l].st; tyv[v] = c->lv[l].ty; }
            else if (c->lv[l].st != stv[v])
                return bset_err(b, LBR_ERR_INVALID_ARG, "cases store one virtual level in different formats");
        }
    std::vector<Item> items(2 * per);
    for (int k = 0; k < 2 * per; ++k) { items[k].v = seq2[k].first; items[k].st = stv[seq2[k].first]; }

    std::vector<unsigned char> parts;
    std::vector<int> starts;
    b->launches.clear();
    const int range[3][2] = {{0, per}, {per, 2 * per}, {0, 2 * per}};
    for (int t = 0; t < 3; ++t) {
        const auto groups = batch_groups(b, items, range[t][0], range[t][1]);
        std::vector<int> tk(2 * per, TILE_Y_DEFAULT);
        if (!b->persistent)
            for (const auto& grp : groups)
                for (int k : grp) tk[k] = tyv[items[grp[0]].v];
        if (int r = batch_fill(b, items, range[t][0], range[t][1], tk, seq2)) return r;
        b->table[t][0] = (int)b->launches.size();
        for (const auto& grp : groups) {
            const Item& m = items[grp[0]];
            Prec st = m.st;
            for (int k : grp)
                if (items[k].st != m.st) st = P_MIXED;
            lbr_batch::Launch ln{parts.size(), (int)starts.size(), 0, 0, m.v, st, TILE_YS[tk[grp[0]]]};
            // a short launch (its main part at most four generations of resident
            // workgroups) lays out the merged coarser parts first, so that their
            // slow ghost-band tiles do not start in its tail; parts are
            // independent, so the order changes no result
            long main_blocks = 0;
            for (int nb : m.blocks) main_blocks += nb;
            const long resident = (long)cus * 32 / TILE_YS[tk[grp[0]]];
            const bool coarse_first = grp.size() > 1 && main_blocks <= 4 * resident;
            std::vector<int> order(grp.begin(), grp.end());
            if (coarse_first) std::rotate(order.begin(), order.begin() + 1, order.end());
            for (int k : order) {
                const Item& x = items[k];
                parts.insert(parts.end(), x.args.begin(), x.args.end());
                for (int nb : x.blocks) {
                    starts.push_back(ln.nblocks);
                    ln.nblocks += nb;
                    ln.nparts++;
                }
            }
            b->launches.push_back(ln);
        }
        b->table[t][1] = (int)b->launches.size();
    }
    lbr_ctx* c0 = b->all[0];
    b->parts_dev = dalloc(c0, std::max<size_t>(parts.size(), 16));
    b->start_dev = static_cast<int*>(dalloc(c0, std::max<size_t>(starts.size(), 1) * sizeof(int)));
    if (!b->parts_dev || !b->start_dev) return bset_err(b, LBR_ERR_OOM, "batch tables: out of device memory");
    if (hipMemcpy(b->parts_dev, parts.data(), parts.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->start_dev, starts.data(), starts.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bset_err(b, LBR_ERR_HIP, "batch tables: copy failed");
    if (b->persistent) {
        static_assert(TILE_YS[TILE_Y_DEFAULT] == PERSISTENT_TY, "persistent tables use the default tile height");
        const Prec st = b->launches.empty() ? P_F32 : b->launches[0].st;
        std::vector<PLaunch> pl;
        for (const lbr_batch::Launch& ln : b->launches) {
            if (ln.st != st || st == P_MIXED)
                return bset_err(b, LBR_ERR_INVALID_ARG, "a persistent batch needs one population format on every level");
            const size_t sz = st == P_F64 ? sizeof(StepArgs<double, double>) : sizeof(StepArgs<float, float>);
            pl.push_back({(int)(ln.off / sz), ln.part0, ln.nparts, ln.nblocks});
        }
        b->pst = st;
        b->plaunch_dev = static_cast<PLaunch*>(dalloc(c0, std::max<size_t>(pl.size(), 1) * sizeof(PLaunch)));
        if (!b->plaunch_dev) return bset_err(b, LBR_ERR_OOM, "batch tables: out of device memory");
        if (hipMemcpy(b->plaunch_dev, pl.data(), pl.size() * sizeof(PLaunch), hipMemcpyHostToDevice) != hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "batch tables: copy failed");
        if (!b->bar_dev) {
            b->bar_dev = static_cast<unsigned*>(dalloc(c0, BAR_WORDS * sizeof(unsigned)));
            if (!b->bar_dev || hipMemset(b->bar_dev, 0, BAR_WORDS * sizeof(unsigned)) != hipSuccess)
                return bset_err(b, LBR_ERR_OOM, "persistent grid barrier: out of device memory");
        }
        if (persistent_grid(st, &b->pgrid) != hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "persistent grid: occupancy query failed");
    }
    b->ready = true;
    return 0;
}

// Points the launch tables at a new set of cases (after the queued super steps
// have finished with the old tables).
int batch_cover(lbr_batch* b, const std::vector<lbr_ctx*>& cases) {
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bset_err(b, LBR_ERR_HIP, "synchronize failed");
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    dfree(b->all[0], b->parts_dev);
    dfree(b->all[0], b->start_dev);
    dfree(b->all[0], b->plaunch_dev);
    b->parts_dev = nullptr;
    b->start_dev = nullptr;
    b->plaunch_dev = nullptr;
    b->ready = false;
    b->cases = cases;
    b->lmax = 0;
    b->merge = true;
    b->cur0.clear();
    for (lbr_ctx* c : cases) {
        b->lmax = std::max(b->lmax, (int)c->lv.size());
        b->cur0.push_back(c->lv[0].cur);
    }
    b->parity = 0;
    return batch_build(b);
}

hipEvent_t* batch_prof_events(lbr_batch* b, int v) {
    b->prof_launches++;
    if (b->pev_used + 2 > 2 * MAX_TIMED_LAUNCHES) return nullptr;   // the first launches of the call
    while (b->pev.size() < b->pev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        b->pev.push_back(e);
        b->pev_v.push_back(0);
    }
    b->pev_v[b->pev_used] = v;
    hipEvent_t* e = &b->pev[b->pev_used];
    b->pev_used += 2;
    return e;
}

int batch_table(lbr_batch* b, int t) {
    for (int k = b->table[t][0]; k < b->table[t][1]; ++k) {
        const lbr_batch::Launch& ln = b->launches[k];
        const void* parts = static_cast<const unsigned char*>(b->parts_dev) + ln.off;
        Timing tm;
        if (b->prof)
            if (hipEvent_t* e = batch_prof_events(b, ln.v)) { tm.start = e[0]; tm.stop = e[1]; }
        if (launch_step_batch(ln.st, parts, b->start_dev + ln.part0, ln.nparts, ln.nblocks, ln.ty, b->stream, tm) !=
            hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "batched k_step launch failed");
    }
    return 0;
}

// Host bookkeeping after one super step: level 0 of a case with lmax levels
// changes buffers; every case advanced 2^(lmax - L_k) coarse steps.
void batch_account(lbr_batch* b) {
    for (lbr_ctx* c : b->cases) {
        const int off = b->lmax - (int)c->lv.size();
        if (off == 0) c->lv[0].cur ^= 1;
        c->step_count += int64_t(1) << off;
        c->resid_steps += int64_t(1) << off;
    }
    b->parity ^= 1;
}

// Every case's level 0 must sit in the buffer the launch tables were built for:
// a case advanced by an odd number of steps outside the batch would not.
int batch_check(lbr_batch* b) {
    for (size_t k = 0; k < b->cases.size(); ++k) {
        const lbr_ctx* c = b->cases[k];
        const int off = b->lmax - (int)c->lv.size();
        if (c->lv[0].cur != (b->cur0[k] ^ (off == 0 ? b->parity : 0)))
            return bset_err(b, LBR_ERR_STATE, "a case was advanced outside the batch by an odd number of steps");
    }
    return 0;
}

// The batch runs on the stream of its first case; work queued on the other
// cases' streams before a batch call completes before it, and work queued on
// them after it waits for it.
int batch_wait_cases(lbr_batch* b) {
    for (size_t k = 1; k < b->all.size(); ++k)
        if (hipEventRecord(b->ev[k], b->all[k]->stream) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->ev[k], 0) != hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "stream ordering failed");
    return 0;
}

int batch_release_cases(lbr_batch* b) {
    if (hipEventRecord(b->ev[0], b->stream) != hipSuccess) return bset_err(b, LBR_ERR_HIP, "stream ordering failed");
    for (size_t k = 1; k < b->all.size(); ++k)
        if (hipStreamWaitEvent(b->all[k]->stream, b->ev[0], 0) != hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "stream ordering failed");
    return 0;
}

// One table as one cooperative grid (persistent mode).
int batch_table_persistent(lbr_batch* b, int t) {
    const int n = b->table[t][1] - b->table[t][0];
    if (launch_step_persistent(b->pst, b->parts_dev, b->start_dev, b->plaunch_dev + b->table[t][0], n, b->pgrid,
                               b->bar_dev, b->stream) != hipSuccess)
        return bset_err(b, LBR_ERR_HIP, "persistent k_step launch failed");
    return 0;
}

int batch_run(lbr_batch* b, int64_t n) {
    int64_t k = 0;
    if (b->persistent) {
        for (; k < n && b->parity == 1; ++k) {
            if (int r = batch_table_persistent(b, 1)) return r;
            batch_account(b);
        }
        for (; k + 2 <= n; k += 2) {
            if (int r = batch_table_persistent(b, 2)) return r;
            batch_account(b);
            batch_account(b);
        }
        if (k < n) {
            if (int r = batch_table_persistent(b, 0)) return r;
            batch_account(b);
        }
        // a barrier wait that ran out (a grid that was not co-resident) is an error
        unsigned flag = 0;
        if (hipMemcpyAsync(&flag, b->bar_dev + 2, sizeof flag, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "persistent run: synchronize failed");
        if (flag) {
            (void)hipMemset(b->bar_dev, 0, BAR_WORDS * sizeof(unsigned));   // counters left mid-way
            return bset_err(b, LBR_ERR_HIP, "persistent run: a grid barrier wait ran out");
        }
        return 0;
    }
    if (k < n && b->parity == 1) {
        if (int r = batch_table(b, 1)) return r;
        batch_account(b);
        ++k;
    }
    if (n - k >= 2 && b->use_graph && !b->prof) {
        if (!b->graph) {
            hipGraph_t g;
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return bset_err(b, LBR_ERR_HIP, "batch graph capture failed");
            const int r = batch_table(b, 2);
            if (hipStreamEndCapture(b->stream, &g) != hipSuccess || r)
                return bset_err(b, LBR_ERR_HIP, "batch graph capture failed");
            const hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return bset_err(b, LBR_ERR_HIP, "batch graph instantiate failed");
        }
        for (; k + 2 <= n; k += 2) {
            if (hipGraphLaunch(b->graph, b->stream) != hipSuccess)
                return bset_err(b, LBR_ERR_HIP, "batch graph launch failed");
            batch_account(b);
            batch_account(b);
        }
    }
    for (; k + 2 <= n; k += 2) {
        if (int r = batch_table(b, 2)) return r;
        batch_account(b);
        batch_account(b);
    }
    if (k < n) {
        if (int r = batch_table(b, 0)) return r;
        batch_account(b);
    }
    return 0;
}

int batch_advance(lbr_batch* b, int64_t n) {
    if (n < 0) return bset_err(b, LBR_ERR_INVALID_ARG, "negative step count");
    if (!b->ready) return bset_err(b, LBR_ERR_STATE, "batch launch tables missing");
    if (int r = batch_check(b)) return r;
    if (int r = batch_wait_cases(b)) return r;
    b->pev_used = 0;
    b->prof_launches = 0;
    if (int r = batch_run(b, n)) return r;
    if (b->prof && b->pev_used) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) return bset_err(b, LBR_ERR_HIP, "synchronize failed");
        double sum[3] = {0, 0, 0};
        int cnt[3] = {0, 0, 0};
        for (size_t i = 0; i + 1 < b->pev_used; i += 2) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, b->pev[i], b->pev[i + 1]);
            const int v = b->pev_v[i];
            sum[0] += ms;
            cnt[0]++;
            if (v == b->lmax - 1) { sum[1] += ms; cnt[1]++; }
            if (v == 0) { sum[2] += ms; cnt[2]++; }
        }
        for (int f = 0; f < 3; ++f) b->prof_out[f] = cnt[f] ? 1000.0 * sum[f] / cnt[f] : 0.0;
        b->prof_out[3] = n ? (double)b->prof_launches / (double)n : 0.0;
    }
    return batch_release_cases(b);
}

}  // namespace

extern "C" {

int lbr_batch_create(int32_t n, lbr_ctx* const* cases, lbr_batch** out) {
    if (!out) return LBR_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || !cases) return LBR_ERR_INVALID_ARG;
    for (int k = 0; k < n; ++k) {
        if (!cases[k] || !cases[k]->built || cases[k]->cfg.storage != cases[0]->cfg.storage)
            return LBR_ERR_INVALID_ARG;
        for (int j = 0; j < k; ++j)
            if (cases[j] == cases[k]) return LBR_ERR_INVALID_ARG;   // one case, two slots: a race
    }
    for (int k = 0; k < n; ++k)
        if ((double)cases[k]->step_count < cases[k]->cfg.ramp_steps)
            return LBR_ERR_STATE;                                   // start-up ramps run case by case
    auto* b = new (std::nothrow) lbr_batch();
    if (!b) return LBR_ERR_OOM;
    *out = b;
    b->all.assign(cases, cases + n);
    b->stream = cases[0]->stream;
    for (lbr_ctx* c : b->all)
        if (hipStreamSynchronize(c->stream) != hipSuccess) return bset_err(b, LBR_ERR_HIP, "synchronize failed");
    b->ev.assign(b->all.size(), nullptr);
    for (hipEvent_t& e : b->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bset_err(b, LBR_ERR_HIP, "event creation failed");
    return batch_cover(b, b->all);
}

int lbr_batch_advance(lbr_batch* b, int64_t n) {
    if (!b) return LBR_ERR_INVALID_ARG;
    return batch_advance(b, n);
}

int lbr_batch_run_to_steady(lbr_batch* b, double tol, int64_t max_super_steps, int64_t check_every,
                            int64_t* steps_done, double* residual) {
    if (!b || check_every <= 0 || max_super_steps < 0) return LBR_ERR_INVALID_ARG;
    if (!b->ready) return bset_err(b, LBR_ERR_STATE, "batch launch tables missing");
    const size_t n = b->all.size();
    std::vector<int64_t> start(n);
    std::vector<double> r(n, 1.0);
    int rc = 0;
    for (size_t k = 0; k < n && !rc; ++k) {
        start[k] = b->all[k]->step_count;
        if ((rc = lbr_residual(b->all[k], &r[k]))) b->err = b->all[k]->err;   // records the reference state
    }
    std::vector<lbr_ctx*> active = b->cases;
    int64_t done = 0;
    while (!rc && done < max_super_steps && !active.empty()) {
        const int64_t k = std::min(check_every, max_super_steps - done);
        if ((rc = batch_advance(b, k))) break;
        done += k;
        std::vector<lbr_ctx*> keep;
        for (size_t j = 0; j < n && !rc; ++j) {
            lbr_ctx* c = b->all[j];
            if (std::find(active.begin(), active.end(), c) == active.end()) continue;
            if ((rc = lbr_residual(c, &r[j]))) { b->err = c->err; break; }
            if (!(r[j] < tol)) keep.push_back(c);
        }
        // converged cases leave the launches; the others go on without them
        if (!rc && !keep.empty() && keep.size() != active.size()) rc = batch_cover(b, keep);
        active.swap(keep);
    }
    if (b->cases.size() != n) {                               // the batch covers every case again
        const int r2 = batch_cover(b, b->all);
        if (!rc) rc = r2;
    }
    for (size_t k = 0; k < n; ++k) {
        if (steps_done) steps_done[k] = b->all[k]->step_count - start[k];
        if (residual) residual[k] = r[k];
    }
    if (!rc)
        for (size_t k = 0; k < n; ++k)
            if (!(r[k] < tol)) {
                char msg[160];
                snprintf(msg, sizeof msg, "case %zu: residual %.3e after %lld super steps", k, r[k], (long long)done);
                return bset_err(b, LBR_ERR_NOT_CONVERGED, msg);
            }
    return rc;
}

int lbr_batch_use_graph(lbr_batch* b, int32_t enable) {
    if (!b) return LBR_ERR_INVALID_ARG;
    if (enable && !b->stream)
        return bset_err(b, LBR_ERR_INVALID_ARG, "graph replay needs a stream other than the default stream");
    b->use_graph = enable != 0;
    return LBR_OK;
}

int lbr_batch_use_persistent(lbr_batch* b, int32_t enable) {
    if (!b) return LBR_ERR_INVALID_ARG;
    if ((enable != 0) == b->persistent) return LBR_OK;
    if (enable && b->prof) return bset_err(b, LBR_ERR_STATE, "profiling times the launches of the merged schedule");
    b->persistent = enable != 0;
    if (int r = batch_cover(b, b->cases)) {
        b->persistent = false;
        (void)batch_cover(b, b->cases);
        return r;
    }
    return LBR_OK;
}

int lbr_batch_profile(lbr_batch* b, int32_t enable, double out[4]) {
    if (!b) return LBR_ERR_INVALID_ARG;
    if (enable && b->persistent)
        return bset_err(b, LBR_ERR_STATE, "profiling times the launches of the merged schedule (persistent mode is on)");
    b->prof = enable != 0;
    if (out)
        for (int f = 0; f < 4; ++f) out[f] = b->prof_out[f];
    return LBR_OK;
}

int lbr_batch_synchronize(lbr_batch* b) {
    if (!b) return LBR_ERR_INVALID_ARG;
    return hipStreamSynchronize(b->stream) == hipSuccess ? LBR_OK : bset_err(b, LBR_ERR_HIP, "synchronize failed");
}

int64_t lbr_batch_steps_per_super_step(const lbr_batch* b, int32_t k) {
    if (!b || k < 0 || k >= (int)b->all.size()) return LBR_ERR_INVALID_ARG;
    if (std::find(b->cases.begin(), b->cases.end(), b->all[k]) == b->cases.end()) return 0;
    return int64_t(1) << (b->lmax - (int)b->all[k]->lv.size());
}

int64_t lbr_batch_lups_per_super_step(lbr_batch* b) {
    if (!b) return LBR_ERR_INVALID_ARG;
    int64_t s = 0;
    for (lbr_ctx* c : b->cases)
        s += lbr_lups_per_coarse_step(c) * (int64_t(1) << (b->lmax - (int)c->lv.size()));
    return s;
}

const char* lbr_batch_last_error(const lbr_batch* b) { return b ? b->err.c_str() : "null batch"; }

void lbr_batch_destroy(lbr_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->pev) (void)hipEventDestroy(e);
    if (!b->all.empty()) {
        dfree(b->all[0], b->parts_dev);
        dfree(b->all[0], b->start_dev);
        dfree(b->all[0], b->plaunch_dev);
        dfree(b->all[0], b->bar_dev);
    }
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// tile-height tuner
// ---------------------------------------------------------------------------
namespace {

// Times every tile height on every virtual level of the cases (level
// v - (lmax - L_k) of case k, all cases in one launch) and returns the
// fastest per virtual level.  Each trial runs the level's first sub-step from
// the current state: it writes only the buffers of the next time level, which
// the next real step overwrites, and the wall nodes' friction velocities, which
// are restored afterwards; every cell's result is independent of the tile
// height.
constexpr float TUNE_MARGIN = 0.97f;   // another tile height must beat the default by 3 %

int tune_levels(const std::vector<lbr_ctx*>& cases, int lmax, int trials, std::vector<int>& best,
                std::string& err) {
    lbr_ctx* c0 = cases[0];
    hipStream_t s = c0->stream;
    for (lbr_ctx* c : cases)
        if (hipStreamSynchronize(c->stream) != hipSuccess) { err = "synchronize failed"; return LBR_ERR_HIP; }
    // wall-node state, saved
    std::vector<std::pair<double*, std::vector<double>>> saved;
    for (lbr_ctx* c : cases)
        for (Level& L : c->lv) {
            const size_t n = std::max<size_t>(L.nodes.size(), 1) * 8;
            saved.push_back({L.bstate, std::vector<double>(n)});
            if (hipMemcpy(saved.back().second.data(), L.bstate, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
                err = "tuner: state copy failed";
                return LBR_ERR_HIP;
            }
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void* parts_dev = nullptr;
    int* start_dev = nullptr;
    int rc = 0;
    best.assign(lmax, TILE_Y_DEFAULT);
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { err = "tuner: events"; rc = LBR_ERR_HIP; }
    size_t cap = 0;
    alignas(16) unsigned char buf[sizeof(StepArgs<double, double>)];
    for (int v = 0; v < lmax && !rc; ++v) {
        float ms_k[NTY] = {};
        for (int k = 0; k < NTY && !rc; ++k) {
            std::vector<unsigned char> parts;
            std::vector<int> starts;
            int nblocks = 0;
            Prec st = P_F32;
            for (lbr_ctx* c : cases) {
                const int l = v - (lmax - (int)c->lv.size());
                if (l < 0) continue;
                Level& L = c->lv[l];
                st = L.st;
                const int sub = l == 0 ? 0 : 1;
                int wb = 0, tb = 0;
                size_t sz = 0;
                switch (L.st) {
                    case P_F64: { auto& a = *reinterpret_cast<StepArgs<double, double>*>(buf);
                        fill_step_args(c, l, sub, a, k); wb = a.wall_blocks; tb = a.tile_blocks; sz = sizeof a; break; }
                    case P_F32: { auto& a = *reinterpret_cast<StepArgs<float, float>*>(buf);
                        fill_step_args(c, l, sub, a, k); wb = a.wall_blocks; tb = a.tile_blocks; sz = sizeof a; break; }
                    case P_F16: { auto& a = *reinterpret_cast<StepArgs<__half, float>*>(buf);
                        fill_step_args(c, l, sub, a, k); wb = a.wall_blocks; tb = a.tile_blocks; sz = sizeof a; break; }
                    default: { auto& a = *reinterpret_cast<StepArgs<__hip_bfloat16, float>*>(buf);
                        fill_step_args(c, l, sub, a, k); wb = a.wall_blocks; tb = a.tile_blocks; sz = sizeof a; break; }
                }
                const int nt = TILE_X * TILE_YS[k];
                parts.insert(parts.end(), buf, buf + sz);
                starts.push_back(nblocks);
                nblocks += wb + tb + 8 * (((int)L.edge.size() + 8 * nt - 1) / (8 * nt));
            }
            if (parts.size() > cap) {
                dfree(c0, parts_dev);
                dfree(c0, start_dev);
                cap = parts.size();
                parts_dev = dalloc(c0, cap);
                start_dev = static_cast<int*>(dalloc(c0, cap / 64 * sizeof(int) + sizeof(int)));
                if (!parts_dev || !start_dev) { err = "tuner: out of device memory"; rc = LBR_ERR_OOM; break; }
            }
            float ms = 0.0f;
            bool ok = hipMemcpy(parts_dev, parts.data(), parts.size(), hipMemcpyHostToDevice) == hipSuccess &&
                      hipMemcpy(start_dev, starts.data(), starts.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
            const int np = (int)starts.size();
            ok = ok && launch_step_batch(st, parts_dev, start_dev, np, nblocks, TILE_YS[k], s) == hipSuccess;  // warm-up
            ok = ok && hipEventRecord(e0, s) == hipSuccess;
            for (int r = 0; r < trials && ok; ++r)
                ok = launch_step_batch(st, parts_dev, start_dev, np, nblocks, TILE_YS[k], s) == hipSuccess;
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (!ok) { err = "tuner: launch failed"; rc = LBR_ERR_HIP; break; }
            ms_k[k] = ms;
        }
        // another height replaces the default only when it is clearly faster:
        // near-equal times swap from run to run, and a level timed alone does not
        // see the tile order and part order of the merged schedule
        float pick_ms = ms_k[TILE_Y_DEFAULT];
        for (int k = 0; k < NTY && !rc; ++k)
            if (ms_k[k] < TUNE_MARGIN * ms_k[TILE_Y_DEFAULT] && ms_k[k] < pick_ms) {
                pick_ms = ms_k[k];
                best[v] = k;
            }
    }
    if (hipStreamSynchronize(s) != hipSuccess && !rc) { err = "synchronize failed"; rc = LBR_ERR_HIP; }
    for (auto& sv : saved)
        if (hipMemcpy(sv.first, sv.second.data(), sv.second.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess && !rc) {
            err = "tuner: state restore failed";
            rc = LBR_ERR_HIP;
        }
    dfree(c0, parts_dev);
    dfree(c0, start_dev);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" {

int32_t lbr_schedule(int32_t n_levels, int32_t merge, int32_t* out, int32_t cap) {
    if (n_levels < 1 || n_levels > LBR_MAX_LEVELS || cap < 0 || (cap > 0 && !out)) return LBR_ERR_INVALID_ARG;
    lbr_batch b;
    b.lmax = n_levels;
    b.merge = merge != 0;
    std::vector<std::pair<int, int>> seq;
    batch_schedule(&b, 0, 0, seq);
    std::vector<std::pair<int, int>> seq2(seq);
    seq2.insert(seq2.end(), seq.begin(), seq.end());
    std::vector<Item> items(seq2.size());
    for (size_t k = 0; k < seq2.size(); ++k) { items[k].v = seq2[k].first; items[k].st = P_F32; }
    int32_t n = 0;
    for (const auto& g : batch_groups(&b, items, 0, (int)items.size())) {
        if (n < cap) out[n] = (int32_t)g.size();
        ++n;
        for (int k : g) {
            if (n < cap) out[n] = seq2[k].first;
            ++n;
            if (n < cap) out[n] = seq2[k].second;
            ++n;
        }
    }
    return n;
}

int lbr_tune(lbr_ctx* c, int32_t trials, int32_t* rows) {
    if (!c || trials < 1) return LBR_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    std::vector<int> best;
    std::string err;
    if (int r = tune_levels({c}, (int)c->lv.size(), trials, best, err)) return set_err(c, r, "%s", err.c_str());
    for (size_t l = 0; l < c->lv.size(); ++l) {
        c->lv[l].ty = best[l];
        if (rows) rows[l] = TILE_YS[best[l]];
    }
    c->self_dirty = true;
    return LBR_OK;
}

int lbr_set_tile_rows(lbr_ctx* c, int32_t level, int32_t rows) {
    if (!c) return LBR_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, LBR_ERR_STATE, "lbr_build has not been called");
    int k = -1;
    for (int j = 0; j < NTY; ++j)
        if (TILE_YS[j] == rows) k = j;
    if (k < 0 || level < -1 || level >= (int)c->lv.size())
        return set_err(c, LBR_ERR_INVALID_ARG, "tile rows %d on level %d", rows, level);
    for (size_t l = 0; l < c->lv.size(); ++l)
        if (level < 0 || (int)l == level) c->lv[l].ty = k;
    c->self_dirty = true;
    return LBR_OK;
}

int lbr_batch_tune(lbr_batch* b, int32_t trials, int32_t* rows) {
    if (!b || trials < 1) return LBR_ERR_INVALID_ARG;
    if (!b->ready) return bset_err(b, LBR_ERR_STATE, "batch launch tables missing");
    std::vector<int> best;
    if (int r = tune_levels(b->cases, b->lmax, trials, best, b->err)) return r;
    for (lbr_ctx* c : b->cases) {
        const int off = b->lmax - (int)c->lv.size();
        for (size_t l = 0; l < c->lv.size(); ++l) c->lv[l].ty = best[l + off];
        c->self_dirty = true;
    }
    for (int v = 0; v < b->lmax; ++v)
        if (rows) rows[v] = TILE_YS[best[v]];
    return batch_cover(b, b->cases);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// a context past its start-up ramp, through the merged schedule
// ---------------------------------------------------------------------------
namespace {

int self_advance(lbr_ctx* c, int64_t n) {
    if (!c->self) {
        lbr_ctx* one[1] = {c};
        lbr_batch* b = nullptr;
        const int r = lbr_batch_create(1, one, &b);
        if (r) {
            set_err(c, r, "merged schedule: %s", b ? b->err.c_str() : "batch creation failed");
            lbr_batch_destroy(b);
            return r;
        }
        c->self = b;
    } else if (c->self_dirty || batch_check(c->self)) {
        // the case was stepped by an odd count outside the schedule (ramp, direct
        // launches, a checkpoint load): rebuild the tables from its state
        if (int r = batch_cover(c->self, c->self->all)) return set_err(c, r, "merged schedule: %s", c->self->err.c_str());
    }
    c->self_dirty = false;
    lbr_batch* b = c->self;
    b->use_graph = c->use_graph;
    b->prof = c->prof;
    if (int r = batch_advance(b, n)) return set_err(c, r, "merged schedule: %s", b->err.c_str());
    if (c->prof)
        for (int f = 0; f < 4; ++f) c->prof_out[f] = b->prof_out[f];
    return 0;
}

}  // namespace
