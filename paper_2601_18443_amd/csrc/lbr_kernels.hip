// Device code of liblbr (gfx950).
//
// The hot kernel is k_step (and k_step_batch, the same work for several
// parts of one grid; k_step_batch_mixed when those parts are FP32- and
// FP16-stored levels of mixed storage): one pass per (sub-)step of a level that, for each owned
// fluid cell, advances the SA-neg variable, pulls the nine populations (with
// bounce-back at cut links, domain rules, the coarse/fine transfer), forms rho
// and u, and applies the central-moment collision.  Populations are stored
// shifted (s_i = f_i - w_i, or minus the free-stream equilibrium in the 16-bit
// formats) in planes of a level's storage box; one 64 x H tile per workgroup
// (H = 2, 4, 8 or 16), one wavefront per tile row, so every population plane is
// read and written in coalesced 64-wide rows.  The work is bandwidth-bound and
// uses no matrix cores.
#include "lbr_impl.h"
#include <hip/hip_ext.h>

#include <cmath>
#include <mutex>
#include <type_traits>

namespace lbr {
namespace {

constexpr int CX[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int CY[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
constexpr int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
constexpr int MIRY[9] = {0, 1, 2, 4, 3, 7, 8, 5, 6};

constexpr int BC_PERIODIC = 0, BC_INLET = 1, BC_OUTLET = 2, BC_SYMMETRY = 3;

// SA-neg constants (Section 2.2)
constexpr double KAPPA = 0.41, CB1 = 0.1355, CB2 = 0.622, SIGMA = 2.0 / 3.0, CW2 = 0.3,
                 CW3 = 2.0, CV1 = 7.1, RLIM = 10.0, CV2 = 0.7, CV3 = 0.9, CT3 = 1.2, CN1 = 16.0;
constexpr double CW1 = CB1 / (KAPPA * KAPPA) + (1.0 + CB2) / SIGMA;

template <class T>
__device__ __forceinline__ T wq(int i) {
    return i == 0 ? T(4.0 / 9.0) : (i < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

// storage <-> compute conversions
template <class ST, class CT> struct Cv;
template <> struct Cv<double, double> {
    static __device__ __forceinline__ double ld(const double* p) { return *p; }
    static __device__ __forceinline__ void st(double* p, double v) { *p = v; }
    static __device__ __forceinline__ double ld_val(double v) { return v; }
    static __device__ __forceinline__ double st_val(double v) { return v; }
};
template <> struct Cv<float, float> {
    static __device__ __forceinline__ float ld(const float* p) { return *p; }
    static __device__ __forceinline__ void st(float* p, float v) { *p = v; }
    static __device__ __forceinline__ float ld_val(float v) { return v; }
    static __device__ __forceinline__ float st_val(float v) { return v; }
};
template <> struct Cv<__half, float> {
    static __device__ __forceinline__ float ld(const __half* p) { return __half2float(*p); }
    static __device__ __forceinline__ void st(__half* p, float v) { *p = __float2half_rn(v); }
    static __device__ __forceinline__ float ld_val(__half v) { return __half2float(v); }
    static __device__ __forceinline__ __half st_val(float v) { return __float2half_rn(v); }
};
template <> struct Cv<__hip_bfloat16, float> {
    static __device__ __forceinline__ float ld(const __hip_bfloat16* p) { return __bfloat162float(*p); }
    static __device__ __forceinline__ void st(__hip_bfloat16* p, float v) { *p = __float2bfloat16(v); }
    static __device__ __forceinline__ float ld_val(__hip_bfloat16 v) { return __bfloat162float(v); }
    static __device__ __forceinline__ __hip_bfloat16 st_val(float v) { return __float2bfloat16(v); }
};

__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }
__device__ __forceinline__ float dmin(float a, float b) { return a < b ? a : b; }

// Reciprocal and x^(1/6): IEEE in FP64; in FP32 the hardware reciprocal and
// base-2 exp / log (about one ulp), which the FP32 tolerance absorbs.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double sixth_root(double x) { return pow(x, 1.0 / 6.0); }
__device__ __forceinline__ float sixth_root(float x) {
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 6.0f));
}

// ---------------------------------------------------------------------------
// Raw buffer access for the hot kernel: one buffer resource per array (base at
// the start of the padded allocation, size in bytes), a per-thread 32-bit byte
// offset shared by all planes, and a wave-uniform byte offset per plane in a
// scalar register -- no 64-bit address arithmetic per access.  Offsets beyond
// the resource size read 0 and drop stores instead of faulting.
// ---------------------------------------------------------------------------
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;   // raw (untyped) access on gfx9-family parts

template <class T>
__device__ __forceinline__ Rsrc make_rsrc(const T* alloc_begin, long elems) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(alloc_begin), (short)0,
                                             (int)(elems * (long)sizeof(T)), RSRC_WORD3);
}

template <class T> struct Bf;
template <> struct Bf<double> {
    static __device__ __forceinline__ double ld(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, double v) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
    }
};
template <> struct Bf<float> {
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, 0);
    }
};
template <> struct Bf<__half> {
    static __device__ __forceinline__ __half ld(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, __half v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, vo, so, 0);
    }
};
template <> struct Bf<__hip_bfloat16> {
    static __device__ __forceinline__ __hip_bfloat16 ld(Rsrc r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(__hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    static __device__ __forceinline__ void st(Rsrc r, uint32_t vo, uint32_t so, __hip_bfloat16 v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, vo, so, 0);
    }
};

// storage <-> compute conversion on top of a buffer access
template <class ST, class CT>
__device__ __forceinline__ CT bld(Rsrc r, uint32_t vo, uint32_t so) {
    return Cv<ST, CT>::ld_val(Bf<ST>::ld(r, vo, so));
}
template <class ST, class CT>
__device__ __forceinline__ void bst(Rsrc r, uint32_t vo, uint32_t so, CT v) {
    Bf<ST>::st(r, vo, so, Cv<ST, CT>::st_val(v));
}

// 16-bit population storage holds s_i - d_i, with d_i = 0 (plain shifted
// storage, f_i - w_i) or d_i = f_eq_i(rho_ref, U) - w_i (free-stream shift:
// near the free stream the stored values are small and keep their 11- or
// 8-bit relative precision); wider formats store s_i.  d is uniform per launch.
template <class ST, class CT>
__device__ __forceinline__ CT unshift(CT v, const CT* d, int i) {
    if constexpr (sizeof(ST) == 2) return v + d[i];
    else return v;
}
template <class ST, class CT>
__device__ __forceinline__ CT toshift(CT v, const CT* d, int i) {
    if constexpr (sizeof(ST) == 2) return v - d[i];
    else return v;
}

// ---------------------------------------------------------------------------
// Central-moment collision (eqs (5)-(10)) in shifted variables.  The second
// central moments are formed from the raw moments of s, the shear pair
// (k4, k5) relaxes with omega, the trace k3 with omega_b, every other central
// moment is set to its equilibrium value (K = 1), the force enters the first
// central moments as F/2 after collision, and the post-collision raw moments
// are mapped back to populations with the constant inverse of the D2Q9
// raw-moment matrix.  All moments carry the lattice-weight part removed, so
// the arithmetic never subtracts O(1) quantities.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void collide(T s[9], T drho, T ux, T uy, T omega, T omega_b, T fx,
                                        T fy) {
    const T rho = T(1) + drho;
    const T sxx = s[1] + s[2] + s[5] + s[6] + s[7] + s[8];
    const T syy = s[3] + s[4] + s[5] + s[6] + s[7] + s[8];
    const T sxy = s[5] + s[6] - s[7] - s[8];
    const T ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const T k4 = (sxx - syy) - rho * (ux2 - uy2) + (ux * fx - uy * fy);
    const T k5 = sxy - rho * uxy + T(0.5) * (ux * fy + uy * fx);
    const T K3 = (sxx + syy) - T(2.0 / 3.0) * drho - rho * (ux2 + uy2) + (ux * fx + uy * fy);
    const T k4s = (T(1) - omega) * k4;
    const T k5s = (T(1) - omega) * k5;
    const T K3s = (T(1) - omega_b) * K3;
    const T c20 = T(0.5) * (K3s + k4s);        // kappa*_20 - rho/3
    const T c02 = T(0.5) * (K3s - k4s);        // kappa*_02 - rho/3
    const T c11 = k5s;
    const T c10 = T(0.5) * fx, c01 = T(0.5) * fy;
    const T k20 = rho * T(1.0 / 3.0) + c20, k02 = rho * T(1.0 / 3.0) + c02;
    // post-collision raw moments minus those of the weights (1,0,0,1/3,1/3,0,0,0,1/9)
    const T M00 = drho;
    const T M10 = c10 + ux * rho;
    const T M01 = c01 + uy * rho;
    const T M20 = (drho * T(1.0 / 3.0) + c20) + T(2) * ux * c10 + ux2 * rho;
    const T M02 = (drho * T(1.0 / 3.0) + c02) + T(2) * uy * c01 + uy2 * rho;
    const T M11 = c11 + ux * c01 + uy * c10 + uxy * rho;
    const T M21 = T(2) * ux * c11 + uy * k20 + ux2 * c01 + T(2) * uxy * c10 + ux2 * uy * rho;
    const T M12 = T(2) * uy * c11 + ux * k02 + uy2 * c10 + T(2) * uxy * c01 + ux * uy2 * rho;
    const T M22 = drho * T(1.0 / 9.0) + uy2 * k20 + ux2 * k02 + T(4) * uxy * c11 +
                  T(2) * ux * uy2 * c10 + T(2) * ux2 * uy * c01 + ux2 * uy2 * rho;
    s[0] = M00 - M20 - M02 + M22;
    s[1] = T(0.5) * (M10 + M20 - M12 - M22);
    s[2] = T(0.5) * (-M10 + M20 + M12 - M22);
    s[3] = T(0.5) * (M01 + M02 - M21 - M22);
    s[4] = T(0.5) * (-M01 + M02 + M21 - M22);
    s[5] = T(0.25) * (M11 + M21 + M12 + M22);
    s[6] = T(0.25) * (M11 - M21 - M12 + M22);
    s[7] = T(0.25) * (-M11 - M21 + M12 + M22);
    s[8] = T(0.25) * (-M11 + M21 - M12 + M22);
}

// Equilibrium of eq (4) (fourth-order coefficient 1/(4 c_s^8)), shifted by w_i.
template <class T>
__device__ __forceinline__ void equilibrium(T s[9], T drho, T ux, T uy) {
    const T rho = T(1) + drho;
    const T u2 = ux * ux + uy * uy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T cx = T(CX[i]), cy = T(CY[i]);
        const T cu = cx * ux + cy * uy;
        const T hx = cx * cx - T(1.0 / 3.0), hy = cy * cy - T(1.0 / 3.0);
        const T e = T(3) * cu + T(4.5) * (cu * cu - u2 * T(1.0 / 3.0)) +
                    T(13.5) * (hx * cy * ux * ux * uy + cx * hy * ux * uy * uy) +
                    T(20.25) * hx * hy * ux * ux * uy * uy;
        s[i] = wq<T>(i) * (drho + rho * e);
    }
}

// ---------------------------------------------------------------------------
// SA-neg (Section 2.2): one explicit step at a fluid node from its 3 x 3
// stencil (index (dy+1)*3 + dx+1).  Vorticity from the least-squares gradient
// over the eight neighbours; Lax-Wendroff (or first-order upwind) convection;
// centred diffusion with face-averaged nodal diffusivity.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T sa_mu(T nt, T nu) {
    if (nt >= T(0)) return nu + nt;
    const T c = fdiv(nt, nu);
    const T c3 = c * c * c;
    return nu + fdiv(nt * (T(CN1) + c3), T(CN1) - c3);
}

template <class T>
__device__ T sa_update(const T nt[9], const T u[9], const T v[9], T nu, T d, int upwind, T cap) {
    const T six = T(1.0 / 6.0);
    const T dudy = ((u[7] - u[1]) + (u[8] - u[2]) + (u[6] - u[0])) * six;
    const T dvdx = ((v[5] - v[3]) + (v[8] - v[6]) + (v[2] - v[0])) * six;
    const T omega = fabs(dvdx - dudy);
    const T C = nt[4];
    const T chi = fdiv(C, nu);
    const T k2d2 = T(KAPPA * KAPPA) * d * d;
    const T Cd = fdiv(C, d);
    T P, D;
    if (C >= T(0)) {
        const T chi3 = chi * chi * chi;
        const T fv1 = fdiv(chi3, chi3 + T(CV1 * CV1 * CV1));
        const T fv2 = T(1) - fdiv(chi, T(1) + chi * fv1);
        const T sbar = fdiv(C * fv2, k2d2);
        const T st = (sbar >= -T(CV2) * omega)
                         ? omega + sbar
                         : omega + fdiv(omega * (T(CV2 * CV2) * omega + T(CV3) * sbar),
                                        T(CV3 - 2.0 * CV2) * omega - sbar);
        T r = (st > T(1e-30)) ? fdiv(C, st * k2d2) : T(RLIM);
        r = dmin(r, T(RLIM));
        const T r2 = r * r;
        const T g = r + T(CW2) * (r2 * r2 * r2 - r);
        const T g2 = g * g;
        const T c6 = T(CW3 * CW3 * CW3 * CW3 * CW3 * CW3);
        const T fw = g * sixth_root(fdiv(T(1) + c6, g2 * g2 * g2 + c6));
        P = T(CB1) * st * C;
        D = T(CW1) * fw * Cd * Cd;
    } else {
        P = T(CB1 * (1.0 - CT3)) * omega * C;
        D = -T(CW1) * Cd * Cd;
    }
    const T E = nt[5], W = nt[3], N = nt[7], S = nt[1];
    const T dX = T(0.5) * (E - W), dY = T(0.5) * (N - S);
    const T uc = u[4], vc = v[4];
    T conv;
    if (upwind) {
        conv = -(uc * (uc > T(0) ? C - W : E - C) + vc * (vc > T(0) ? C - S : N - C));
    } else {
        conv = -(uc * dX + vc * dY) +
               T(0.5) * (uc * uc * (E - T(2) * C + W) +
                         T(0.5) * uc * vc * (nt[8] - nt[6] - nt[2] + nt[0]) +
                         vc * vc * (N - T(2) * C + S));
    }
    // face diffusivity: mean of the nodal values (eqs (12), (16)), limited to cap
    // when one is configured (+inf otherwise: dmin then returns the mean itself)
    const T mC = sa_mu(C, nu);
    const T diff = dmin(T(0.5) * (mC + sa_mu(E, nu)), cap) * (E - C) -
                   dmin(T(0.5) * (mC + sa_mu(W, nu)), cap) * (C - W) +
                   dmin(T(0.5) * (mC + sa_mu(N, nu)), cap) * (N - C) -
                   dmin(T(0.5) * (mC + sa_mu(S, nu)), cap) * (C - S) +
                   T(CB2) * (dX * dX + dY * dY);
    return C + conv + (P - D) + diff * T(1.0 / SIGMA);
}

template <class T>
__device__ __forceinline__ T eddy_viscosity(T chi, T nu) {
    if (chi <= T(0)) return T(0);
    const T c3 = chi * chi * chi;
    return fdiv(nu * chi * c3, c3 + T(CV1 * CV1 * CV1));
}

// ---------------------------------------------------------------------------
// Wall function and friction velocity (eqs (21)-(22) of Section 2.2; step 3
// of the VN procedure), FP64.
// ---------------------------------------------------------------------------
constexpr double WF_B = 5.033908790505579, WF_A1 = 8.148221580024245,
                 WF_A2 = -6.9287093849022945, WF_B1 = 7.4600876082527945,
                 WF_B2 = 7.468145790401841, WF_C1 = 2.5496773539754747,
                 WF_C2 = 1.3301651588535228, WF_C3 = 3.599459109332379,
                 WF_C4 = 3.639753186868684494;

// eq (22), continuous branch of the arctangents
// (b > 0, so atan2(b, x) = pi/2 - atan(x / b): no division, no quadrant logic)
__device__ double uplus(double y) {
    const double p = y + WF_A1, m = y + WF_A2;
    constexpr double HALF_PI = 1.5707963267948966, IB1 = 1.0 / WF_B1, IB2 = 1.0 / WF_B2;
    return WF_B + WF_C1 * log(p * p + WF_B1 * WF_B1) - WF_C2 * log(m * m + WF_B2 * WF_B2) -
           WF_C3 * (HALF_PI - atan(p * IB1)) - WF_C4 * (HALF_PI - atan(m * IB2));
}

// eq (21)
__device__ double duplus(double y) {
    const double ky = KAPPA * y, k3 = ky * ky * ky, c3 = CV1 * CV1 * CV1;
    return (c3 + k3) / (c3 + k3 * (1.0 + ky));
}

__device__ double friction_velocity(double ut, double d, double nu, double guess) {
    if (!(ut > 0.0)) return 0.0;
    double u = guess > 0.0 ? guess : sqrt(nu * ut / d);
    for (int it = 0; it < 100; ++it) {
        const double yp = d * u / nu;
        const double up = uplus(yp);
        const double step = (u * up - ut) / (up + yp * duplus(yp));
        double un = u - step;
        if (!(un > 0.0)) un = 0.5 * u;
        u = un;
        // Newton converges quadratically here: after a step of at most 1e-9 u the
        // remaining error is of order 1e-18 u, below FP64 resolution, so no
        // further iteration is needed to confirm it
        if (fabs(step) <= 1e-9 * u) break;
    }
    if (!(u > 0.0) || !isfinite(u)) {
        double lo = 0.0, hi = ut * 1e3;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid * uplus(d * mid / nu) - ut > 0.0) hi = mid; else lo = mid;
        }
        u = 0.5 * (lo + hi);
    }
    return u;
}

// Steps 1-5 of the VN procedure (Section 2.3) for wall node b, from the
// macroscopic planes `mac`: rho_R and u_R with precomputed IDW / LSQ weights,
// tangential part, u_tau by Newton, u_V and the slip velocity of eq (28)
// (or eq (31)); rho_W = rho_R.  out: u_tau, u_Rt (x, y), rho_W, u_W (x, y).
template <class CT>
__device__ void wall_model(const WallData& w, int b, const CT* mac, long P, double nu,
                           double guess, double out[6]) {
    const double* g = w.geo + 6 * b;
    double uwx = 0.0, uwy = 0.0, rhow, utau = 0.0, tx = 0.0, ty = 0.0;
    if (w.model == 2 || w.model == 3) {
        rhow = (double)mac[w.cell[b]];
        if (w.model == 3) {
            const double* uw = (g[5] == -2.0) ? w.uw_hi : w.uw_lo;
            uwx = uw[0];
            uwy = uw[1];
        }
    } else {
        // gathered four slots at a time (the enclosing 2 x 2 block is the usual
        // stencil), the loads of a group issued together; unused slots of a group
        // read the node's own cell with weight 0, an exact no-op
        double rr = 0.0, ux = 0.0, uy = 0.0;
        const int own = w.cell[b];
        for (int j0 = 0; j0 < MAX_STENCIL; j0 += 4) {
            if (w.st_cell[MAX_STENCIL * b + j0] < 0) break;
#pragma unroll
            for (int j = j0; j < j0 + 4; ++j) {
                const int cj = w.st_cell[MAX_STENCIL * b + j];
                const bool use = cj >= 0;
                const int cc = use ? cj : own;
                const double wr = use ? w.st_wr[MAX_STENCIL * b + j] : 0.0;
                const double wu = use ? w.st_wu[MAX_STENCIL * b + j] : 0.0;
                rr += wr * (double)mac[cc];
                ux += wu * (double)mac[P + cc];
                uy += wu * (double)mac[2 * P + cc];
            }
        }
        const double un = ux * g[2] + uy * g[3];                 // step 2
        tx = ux - un * g[2];
        ty = uy - un * g[3];
        const double ut = sqrt(tx * tx + ty * ty);
        utau = friction_velocity(ut, w.d_wr, nu, guess);         // step 3
        double uw;
        if (w.model == 1) {                                      // eq (31)
            const double yr = w.d_wr * utau / nu;
            uw = ut - utau * utau * w.d_wr / (nu + nu * KAPPA * yr);
        } else {                                                 // steps 4-5, eq (28)
            const double yv = w.d_wv * utau / nu;
            uw = utau * uplus(yv) - utau * utau * w.d_wv / (nu + nu * KAPPA * yv);
        }
        if (ut > 0.0) {
            uwx = uw * tx / ut;
            uwy = uw * ty / ut;
        }
        rhow = rr;                                               // step 6: rho_W = rho_R
    }
    out[0] = utau; out[1] = tx; out[2] = ty; out[3] = rhow; out[4] = uwx; out[5] = uwy;
}

// ---------------------------------------------------------------------------
// Pieces of the per-cell update shared by k_step and k_boundary.
// ---------------------------------------------------------------------------
// A population of a neighbouring level.  With mixed storage (FP32 arithmetic)
// that level may hold FP32 or FP16 where this one holds the other; the kind is
// uniform over a launch, so the test is a scalar branch.
template <class ST, class CT>
__device__ __forceinline__ CT ld_pop(const void* base, long k, int kind, const CT* d, int i) {
    if constexpr (std::is_same<CT, float>::value) {
        if (kind == P_F16) return Cv<__half, float>::ld(static_cast<const __half*>(base) + k) + d[i];
        if (kind == P_F32) return Cv<float, float>::ld(static_cast<const float*>(base) + k);
    }
    return unshift<ST, CT>(Cv<ST, CT>::ld(static_cast<const ST*>(base) + k), d, i);
}

template <class ST, class CT>
__device__ __forceinline__ CT coarse_val(const StepArgs<ST, CT>& a, int i, int gx, int gy) {
    const long cc = (long)((gy >> 1) - a.cbox.gy0) * a.cbox.pitch + ((gx >> 1) - a.cbox.gx0);
    return ld_pop<ST, CT>(a.fcoarse, i * a.cbox.plane + cc, a.cst, a.dsh, i);
}

// coalescence: mean of the four children of the finer band, for each direction
template <class FT, class CT>
__device__ __forceinline__ void coalesce(const FT* f, long plane, long pitch, long f0, const CT* d, CT s[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const FT* p = f + i * plane + f0;
        s[i] = unshift<FT, CT>(CT(0.25) * ((Cv<FT, CT>::ld(p) + Cv<FT, CT>::ld(p + 1)) +
                                           (Cv<FT, CT>::ld(p + pitch) + Cv<FT, CT>::ld(p + pitch + 1))),
                               d, i);
    }
}

// Pull of direction i into (gx, gy): domain rules of level 0 (periodic wrap,
// specular reflection at symmetry edges) and the coarse band on the first
// sub-step.  Returns false for an unknown population (inlet / outlet side).
template <class ST, class CT>
__device__ bool pull_general(const StepArgs<ST, CT>& a, uint8_t fl, int i, int gx, int gy, CT& out) {
    int sx = gx - CX[i], sy = gy - CY[i], di = i;
    if (fl & F_EDGE) {
        if (sx < 0 || sx >= a.dom.nxd) {
            if (!a.dom.periodic_x) return false;
            sx = (sx + a.dom.nxd) % a.dom.nxd;
        }
        if (sy < 0 || sy >= a.dom.nyd) {
            const int side = sy < 0 ? 2 : 3;
            if (a.dom.bc[side] == BC_PERIODIC) sy = (sy + a.dom.nyd) % a.dom.nyd;
            else if (a.dom.bc[side] == BC_SYMMETRY) { sy = gy; di = MIRY[i]; }
            else return false;
        }
    }
    const long cs = (long)(sy - a.box.gy0) * a.box.pitch + (sx - a.box.gx0);
    if ((fl & F_NEARGHOST) && a.substep == 1 && (a.flag[cs] & F_TYPE) == T_GHOST)
        out = coarse_val(a, di, sx, sy);
    else
        out = unshift<ST, CT>(Cv<ST, CT>::ld(a.fsrc + di * a.box.plane + cs), a.dsh, di);
    return true;
}

// SA stencil of an edge cell: periodic wrap, mirror at symmetry edges (u_y flips).
template <class ST, class CT>
__device__ void gather_edge(const StepArgs<ST, CT>& a, int gx, int gy, CT nt[9], CT u[9], CT v[9]) {
    const long P = a.box.plane;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int k = (dy + 1) * 3 + dx + 1;
            int sx = gx + dx, sy = gy + dy;
            CT sgn = CT(1);
            if (sx < 0 || sx >= a.dom.nxd) sx = (sx + a.dom.nxd) % a.dom.nxd;
            if (sy < 0 || sy >= a.dom.nyd) {
                const int side = sy < 0 ? 2 : 3;
                if (a.dom.bc[side] == BC_PERIODIC) sy = (sy + a.dom.nyd) % a.dom.nyd;
                else { sy = (sy < 0) ? -1 - sy : 2 * a.dom.nyd - 1 - sy; sgn = CT(-1); }
            }
            const long cs = (long)(sy - a.box.gy0) * a.box.pitch + (sx - a.box.gx0);
            nt[k] = a.csrc[cs];
            u[k] = a.msrc[P + cs];
            v[k] = sgn * a.msrc[2 * P + cs];
        }
}

// Post-stream value of direction i at (gx, gy) for a cell next to the outlet
// (interior or across a symmetry / periodic y edge).
template <class ST, class CT>
__device__ __forceinline__ CT poststream(const StepArgs<ST, CT>& a, int i, int gx, int gy) {
    int sx = gx - CX[i], sy = gy - CY[i], di = i;
    if (sy < 0 || sy >= a.dom.nyd) {
        const int side = sy < 0 ? 2 : 3;
        if (a.dom.bc[side] == BC_PERIODIC) sy = (sy + a.dom.nyd) % a.dom.nyd;
        else { sy = gy; di = MIRY[i]; }
    }
    const long cs = (long)(sy - a.box.gy0) * a.box.pitch + (sx - a.box.gx0);
    return unshift<ST, CT>(Cv<ST, CT>::ld(a.fsrc + di * a.box.plane + cs), a.dsh, di);
}

// Moments (eq (3) with the half-force shift) and the collision with
// nu_eff = nu + nu_t(chi) (eqs (9), (11)), in place on s.
template <class ST, class CT>
__device__ __forceinline__ void relax_cell(const StepArgs<ST, CT>& a, CT s[9], CT chi_new, CT& rho,
                                           CT& ux, CT& uy) {
    CT drho = CT(0), jx = CT(0), jy = CT(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        drho += s[i];
        jx += CT(CX[i]) * s[i];
        jy += CT(CY[i]) * s[i];
    }
    rho = CT(1) + drho;
    // correctly rounded: the collision conserves momentum only for u = j / rho
    ux = (jx + CT(0.5) * a.fx) / rho;
    uy = (jy + CT(0.5) * a.fy) / rho;
    const CT nu_eff = a.nu + eddy_viscosity(chi_new, a.nu);
    // correctly rounded: near tau = 1/2 the viscosity amplifies an error of omega
    // by about 1 / (tau - 1/2)
    const CT omega = CT(1) / (CT(3) * nu_eff + CT(0.5));
    collide(s, drho, ux, uy, omega, a.omega_b, a.fx, a.fy);
}

// Absorbing layer of level 0 (an addition to the method; sp_width = 0 turns it
// off): within sp_width cells of a far-field side the post-collision
// populations relax towards the free-stream equilibrium with
// sigma = sp_strength ((W - d) / W)^2, d the distance of the cell centre.
template <class CT>
__device__ __forceinline__ void absorb(const Absorber& sp, int nxd, int nyd, int gx, int gy, CT s[9]) {
    if (!(sp.width > 0.0)) return;
    double d = 1e300;
    if (sp.sides & 1) d = fmin(d, gx + 0.5);
    if (sp.sides & 2) d = fmin(d, nxd - gx - 0.5);
    if (sp.sides & 4) d = fmin(d, gy + 0.5);
    if (sp.sides & 8) d = fmin(d, nyd - gy - 0.5);
    if (!(d < sp.width)) return;
    const double x = (sp.width - d) / sp.width;
    const CT sg = CT(sp.strength * x * x);
    CT t[9];
    equilibrium<CT>(t, CT(sp.drho), CT(sp.ux), CT(0));
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = s[i] - sg * (s[i] - t[i]);
}
template <class ST, class CT>
__device__ __forceinline__ void absorb(const StepArgs<ST, CT>& a, int gx, int gy, CT s[9]) {
    absorb<CT>(a.sp, a.dom.nxd, a.dom.nyd, gx, gy, s);
}

// relax_cell, the absorbing layer and plain stores of the new state (wall
// nodes and domain-edge cells).
template <class ST, class CT>
__device__ __forceinline__ void finish_cell(const StepArgs<ST, CT>& a, long c, CT s[9], CT chi_new,
                                            int gx, int gy) {
    const long P = a.box.plane;
    CT rho, ux, uy;
    relax_cell(a, s, chi_new, rho, ux, uy);
    absorb(a, gx, gy, s);
    a.mdst[c] = rho;
    a.mdst[P + c] = ux;
    a.mdst[2 * P + c] = uy;
    a.cdst[c] = chi_new;
#pragma unroll
    for (int i = 0; i < 9; ++i) Cv<ST, CT>::st(a.fdst + i * P + c, toshift<ST, CT>(s[i], a.dsh, i));
}

// ---------------------------------------------------------------------------
// k_step: all owned fluid cells of a level except the wall nodes and the
// domain edge (side-stream kernels), and the ghost band.  One workgroup per
// active 64 x H tile, one wavefront per tile row: the nine pulled populations
// are read straight from memory (coalesced rows), the 3 x 3 SA stencil of
// chi, u_x and u_y is staged in LDS with a one-cell halo (allocations carry
// one spare row at both ends, so every halo address is valid).
//
// Transfers between levels are folded in:
//  * ghost cells of the stencil take chi and u from a linear least-squares fit
//    over the 3 x 3 coarse neighbourhood of their parent (the coarse state of
//    the current parent step, Section 2.2);
//  * on the second sub-step, tiles holding children of covered coarse cells
//    next to the coarse fluid write the mean of each 2 x 2 block of new values
//    into the coarse buffer the next coarse step reads.
// ---------------------------------------------------------------------------
template <class CT>
__device__ __forceinline__ void ghost_fill(const CT* cmac, const CT* cchi, const Box& cb, int gx,
                                           int gy, CT& n, CT& u, CT& v) {
    const int px = gx >> 1, py = gy >> 1;
    const CT ox = (gx & 1) ? CT(0.25) : CT(-0.25), oy = (gy & 1) ? CT(0.25) : CT(-0.25);
    CT sn = 0, su = 0, sv = 0, xn = 0, xu = 0, xv = 0, yn = 0, yu = 0, yv = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const long q = (long)(py + dy - cb.gy0) * cb.pitch + (px + dx - cb.gx0);
            const CT a = cchi[q], b = cmac[cb.plane + q], c = cmac[2 * cb.plane + q];
            sn += a; su += b; sv += c;
            xn += CT(dx) * a; xu += CT(dx) * b; xv += CT(dx) * c;
            yn += CT(dy) * a; yu += CT(dy) * b; yv += CT(dy) * c;
        }
    const CT k9 = CT(1.0 / 9.0), k6 = CT(1.0 / 6.0);
    n = sn * k9 + (ox * xn + oy * yn) * k6;
    u = su * k9 + (ox * xu + oy * yu) * k6;
    v = sv * k9 + (ox * xv + oy * yv) * k6;
}

// ---------------------------------------------------------------------------
// k_edge: level-0 cells on the domain edge (except wall nodes), one thread
// each, beside k_step: periodic wrap, specular reflection at symmetry edges,
// Zou-He velocity inlet, extrapolation or Zou-He pressure outlet (Section
// 3.1.1), and the SA
// boundary rules (inlet chi, outlet extrapolation, mirrored stencil).
// ---------------------------------------------------------------------------
template <class ST, class CT>
__device__ __forceinline__ void edge_cell(const StepArgs<ST, CT>& a, int e) {
    const int pitch = a.box.pitch;
    const long P = a.box.plane;
    const long c = a.edge[e];
    const int gx = (int)(c % pitch) + a.box.gx0, gy = (int)(c / pitch) + a.box.gy0;
    const CT dist = a.dist[c];
    CT s[9], nt[9], u[9], v[9];
    const bool at_inlet = gx == 0 && a.dom.bc[0] == BC_INLET;
    const bool at_outlet = gx == a.dom.nxd - 1 && a.dom.bc[1] == BC_OUTLET;
    {
        gather_edge(a, gx, gy, nt, u, v);
        for (int i = 0; i < 9; ++i)
            if (!pull_general(a, (uint8_t)F_EDGE, i, gx, gy, s[i])) s[i] = CT(0);
        if (at_inlet) {
            const CT ui = a.u_in;
            const CT rho = (CT(1) + s[0] + s[3] + s[4] + CT(2) * (s[2] + s[6] + s[8])) / (CT(1) - ui);
            s[1] = s[2] + CT(2.0 / 3.0) * rho * ui;
            s[5] = s[6] - CT(0.5) * (s[3] - s[4]) + rho * ui * CT(1.0 / 6.0);
            s[7] = s[8] + CT(0.5) * (s[3] - s[4]) + rho * ui * CT(1.0 / 6.0);
        }
        if (at_outlet && a.dom.outlet == 2) {
            // Zou-He with rho = rho_ref and u_y of the upstream cell (unknowns: c_x = -1)
            const CT rho = a.rho_out, uy = v[3];
            const CT ux = (CT(1) + s[0] + s[3] + s[4] + CT(2) * (s[1] + s[5] + s[7])) / rho - CT(1);
            s[2] = s[1] - CT(2.0 / 3.0) * rho * ux;
            s[6] = s[5] + CT(0.5) * (s[3] - s[4]) - rho * ux * CT(1.0 / 6.0) - CT(0.5) * rho * uy;
            s[8] = s[7] - CT(0.5) * (s[3] - s[4]) - rho * ux * CT(1.0 / 6.0) + CT(0.5) * rho * uy;
        } else if (at_outlet) {
            for (int i = 0; i < 9; ++i)
                if (CX[i] == -1)
                    s[i] = (a.dom.outlet == 1)
                               ? poststream(a, i, gx - 1, gy)
                               : CT(2) * poststream(a, i, gx - 1, gy) - poststream(a, i, gx - 2, gy);
        }
    }
    CT chi_new;
    if (a.frozen) {
        chi_new = nt[4];
    } else if (at_inlet) {
        chi_new = a.chi_in;
    } else if (at_outlet) {
        chi_new = nt[3];                         // first-order extrapolation from upstream
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) nt[k] *= a.nu;
        chi_new = fdiv(sa_update(nt, u, v, a.nu, dist, a.sa_mode == 2, a.mu_cap), a.nu);
    }
    finish_cell(a, c, s, chi_new, gx, gy);
}

// ---------------------------------------------------------------------------
// Wall nodes B of a level, one thread each (workgroups of k_step).  Runs beside
// k_step (disjoint cells, same source state): steps 1-5 of the VN procedure
// on the macroscopic state of the previous step, the Dirichlet value
// nu~_B = kappa u_tau d_WB, Yu's interpolated bounce-back (step 6, eq (27)) or
// eq (24) for the missing populations, and the collision.  All loads are
// issued before the Newton iteration and the first store.
// ---------------------------------------------------------------------------
template <class ST, class CT>
__device__ __forceinline__ void boundary_node(const StepArgs<ST, CT>& a, int b) {
    const long P = a.box.plane;
    const int pitch = a.box.pitch;
    const int c = a.wall.cell[b];
    const int gx = c % pitch + a.box.gx0, gy = c / pitch + a.box.gy0;
    // steps 1-5 of the VN procedure on the macroscopic state of the previous step;
    // the populations are loaded afterwards so that they are not held in
    // registers through the FP64 Newton iteration
    double wm[6];
    wall_model<CT>(a.wall, b, a.msrc, P, (double)a.nu, a.wstate[8 * b], wm);
    const int pad = a.pad;
    const Rsrc rf = make_rsrc(a.fsrc - pad, 9 * P + 2 * pad);
    const Rsrc rg = make_rsrc(a.flag - pad, P + 2 * pad);
    constexpr uint32_t SS = sizeof(ST);
    const uint32_t e = (uint32_t)(c + pad);
    // one round of loads once the Newton iteration is done: link fractions,
    // pulled, own and next-node populations, next-node flags
    double q[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = a.wall.q[8 * b + k];
    CT pull[9], own[9], nxt[9];
    uint8_t f2fl[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        // pull source (periodic wrap in x on level 0) and next node F2 = B + c_i
        int sx = gx - CX[i], fx = gx + CX[i];
        if (a.dom.periodic_x) {
            sx = (sx + a.dom.nxd) % a.dom.nxd;
            fx = (fx + a.dom.nxd) % a.dom.nxd;
        }
        const uint32_t src = (uint32_t)((gy - CY[i] - a.box.gy0) * pitch + (sx - a.box.gx0) + pad);
        const uint32_t f2 = (uint32_t)((gy + CY[i] - a.box.gy0) * pitch + (fx - a.box.gx0) + pad);
        pull[i] = unshift<ST, CT>(bld<ST, CT>(rf, src * SS, (uint32_t)(i * P) * SS), a.dsh, i);
        own[i] = unshift<ST, CT>(bld<ST, CT>(rf, e * SS, (uint32_t)(i * P) * SS), a.dsh, i);
        nxt[i] = unshift<ST, CT>(bld<ST, CT>(rf, f2 * SS, (uint32_t)(OPP[i] * P) * SS), a.dsh, OPP[i]);   // f*_o at F2
        f2fl[i] = __builtin_amdgcn_raw_buffer_load_b8(rg, f2, 0, 0);
    }
    const CT rhow = CT(wm[3]), uwx = CT(wm[4]), uwy = CT(wm[5]);
    CT s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double qd = (i == 0) ? -1.0 : q[OPP[i] - 1];
        if (qd < 0.0) { s[i] = pull[i]; continue; }
        // i is the missing population; o = opp(i) is the link from B towards the wall
        const int o = OPP[i];
        const CT qo = CT(qd);
        const CT fo_b = own[o];
        const CT mom = CT(6) * wq<CT>(o) * rhow * (CT(CX[i]) * uwx + CT(CY[i]) * uwy);
        CT val = fo_b + mom;                                      // eq (24)
        if (!a.bb_halfway && q[i - 1] < 0.0 && (f2fl[i] & F_TYPE) == T_FLUID) {
            // (A) outgoing value at the wall point, (B) reflection with the wall
            // momentum, (C) interpolation between W and the next node F2
            const CT fw_o = qo * fo_b + (CT(1) - qo) * nxt[i];
            const CT fw_i = fw_o + mom;
            val = fw_i + (qo / (CT(1) + qo)) * (own[i] - fw_i);
        }
        s[i] = val;
    }
    const CT chi_new = a.frozen ? a.csrc[c]
                                : ((a.wall.model <= 1) ? CT(KAPPA * wm[0] * a.wall.geo[6 * b + 4] / (double)a.nu)
                                                       : CT(0));
    finish_cell(a, c, s, chi_new, gx, gy);
    double* st = a.wstate + 8 * b;
    for (int k = 0; k < 6; ++k) st[k] = wm[k];
}

// One workgroup of a level sub-step; blk is the block index within the level's
// part of the grid.  Tiles are 64 x TY cells (TY wavefronts, one per row); the
// tile height is a launch parameter chosen per level by the host's tuner, and
// every cell's result is the same for any TY.
// LDS of a tile workgroup: the 3 x 3 stencil values of the tile and its halo,
// and the restriction staging.  Keyed on the arithmetic type and tile height
// only, so that the storage formats of a mixed launch share one allocation.
constexpr int GC_W = TILE_X / 2 + 4;   // parent columns under a tile and its halo, with the fill stencil

template <class CT, int TY>
struct TileShared {
    CT n[TY + 2][TILE_X + 2], u[TY + 2][TILE_X + 2], v[TY + 2][TILE_X + 2];
    union {
        CT r[4][TY][TILE_X];                // restriction, after the update
        CT gc[3][TY / 2 + 4][GC_W];         // the parent's chi, u, v under a ghost tile, before it
    };
};
template <class CT, int TY>
__device__ __forceinline__ TileShared<CT, TY>& tile_shared() {
    __shared__ TileShared<CT, TY> sh;
    return sh;
}

// ghost_fill from the parent's chi, u, v staged in LDS (gc[.][0][0] holds the
// parent cell (cpx0, cpy0)): the same arithmetic in the same order, so the same
// values bit for bit
template <class CT, int TY>
__device__ __forceinline__ void ghost_fill_lds(const TileShared<CT, TY>& sh, int cpx0, int cpy0, int gx, int gy,
                                               CT& n, CT& u, CT& v) {
    const int px = gx >> 1, py = gy >> 1;
    const CT ox = (gx & 1) ? CT(0.25) : CT(-0.25), oy = (gy & 1) ? CT(0.25) : CT(-0.25);
    CT sn = 0, su = 0, sv = 0, xn = 0, xu = 0, xv = 0, yn = 0, yu = 0, yv = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int r = py + dy - cpy0, w = px + dx - cpx0;
            const CT a = sh.gc[0][r][w], b = sh.gc[1][r][w], c = sh.gc[2][r][w];
            sn += a; su += b; sv += c;
            xn += CT(dx) * a; xu += CT(dx) * b; xv += CT(dx) * c;
            yn += CT(dy) * a; yu += CT(dy) * b; yv += CT(dy) * c;
        }
    const CT k9 = CT(1.0 / 9.0), k6 = CT(1.0 / 6.0);
    n = sn * k9 + (ox * xn + oy * yn) * k6;
    u = su * k9 + (ox * xu + oy * yu) * k6;
    v = sv * k9 + (ox * xv + oy * yv) * k6;
}

// The parent populations a ghost cell (explosion: every direction whose source is
// not fluid, or not a ghost on the second sub-step, from k cells back) and a fine
// cell next to the ghost band (first sub-step: the directions whose source is a
// ghost) take, in one predicated pass for both kinds of cell, so that a wave
// holding both issues all its loads before one wait.
template <class ST, class CT>
__device__ __forceinline__ void parent_pops(const StepArgs<ST, CT>& a, int type, uint8_t fl, uint32_t lm, int gx,
                                            int gy, CT s[9]) {
    const bool ghost = type == T_GHOST;
    const bool near = type == T_FLUID && !(fl & (F_WALL | F_EDGE | F_IFACE)) && (fl & F_NEARGHOST) && a.substep == 1;
    if (!(ghost || near)) return;
    const int k = (ghost && a.substep == 2) ? 2 : 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const bool src_fluid = (lm >> i) & 1u, src_ghost = (lm >> (16 + i)) & 1u;
        const bool need = ghost ? !(src_fluid || (src_ghost && a.substep == 2)) : src_ghost;
        if (need) s[i] = coarse_val(a, i, gx - k * CX[i], gy - k * CY[i]);
    }
}

// A ghost cell stores what it carries (after parent_pops), with no collision.
template <class ST, class CT>
__device__ __forceinline__ void ghost_band_store(const StepArgs<ST, CT>& a, const CT s[9], Rsrc rfo, uint32_t e,
                                                 long P) {
    constexpr uint32_t SS = sizeof(ST);
#pragma unroll
    for (int i = 0; i < 9; ++i) bst<ST, CT>(rfo, e * SS, (uint32_t)(i * P) * SS, toshift<ST, CT>(s[i], a.dsh, i));
}

// A coarse interface cell takes the mean of its four children (coalescence).
template <class ST, class CT>
__device__ __forceinline__ void iface_cell(const StepArgs<ST, CT>& a, uint8_t fl, int gx, int gy, CT s[9]) {
    if (!(fl & F_IFACE)) return;
    const long f0 = (long)(2 * gy - a.fbox.gy0) * a.fbox.pitch + (2 * gx - a.fbox.gx0);
    if constexpr (std::is_same<CT, float>::value) {
        if (a.fst == P_F16)
            coalesce<__half, CT>(static_cast<const __half*>(a.ffine), a.fbox.plane, a.fbox.pitch, f0, a.dsh, s);
        else if (a.fst == P_F32)
            coalesce<float, CT>(static_cast<const float*>(a.ffine), a.fbox.plane, a.fbox.pitch, f0, a.dsh, s);
        else
            coalesce<ST, CT>(static_cast<const ST*>(a.ffine), a.fbox.plane, a.fbox.pitch, f0, a.dsh, s);
    } else {
        coalesce<ST, CT>(static_cast<const ST*>(a.ffine), a.fbox.plane, a.fbox.pitch, f0, a.dsh, s);
    }
}

template <class ST, class CT, int TY>
__device__ __forceinline__ void step_block(const StepArgs<ST, CT>& a, const int blk) {
    constexpr int NT = TILE_X * TY;                        // threads of the workgroup
    constexpr int NH = 2 * TILE_X + 2 * (TY + 2);          // halo cells of a tile
    constexpr int NS = (NH + NT - 1) / NT;                 // halo cells per thread (1, or 2 for TY = 2)
    TileShared<CT, TY>& lds = tile_shared<CT, TY>();
    auto& sh_n = lds.n;
    auto& sh_u = lds.u;
    auto& sh_v = lds.v;
    // grid: wall-node blocks first (their FP64 Newton iteration is the longest
    // chain), then the tiles, then the level-0 domain-edge cells; each branch is
    // uniform over a workgroup
    if (blk < a.wall_blocks) {
        // the wall nodes carry the longest dependency chain of the launch (FP64
        // Newton iteration): a few per block spreads them over many compute units
        // instead of crowding the SIMDs of a few
        if ((int)threadIdx.x >= WALL_PER_BLOCK) return;
        const int b = blk * WALL_PER_BLOCK + threadIdx.x;
        if (b < a.wall.nb) boundary_node(a, b);
        return;
    }
    const int bid = blk - a.wall_blocks;                         // a multiple of 8 shifts no XCD
    if (bid >= a.tile_blocks) {
        const int e = (bid - a.tile_blocks) * NT + threadIdx.x;
        if (e < a.nedge) edge_cell(a, e);
        return;
    }
    const int per = (a.ntiles + 7) >> 3;
    const int t = (bid & 7) * per + (bid >> 3);                  // neighbouring tiles share an XCD
    if (t >= a.ntiles) return;                                   // whole workgroup
    const uint32_t tile = a.tiles[t];
    const int pitch = a.box.pitch;
    const long P = a.box.plane;
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    const int tx0 = (int)(tile & 0x7fffu) * TILE_X, ty0 = (int)((tile >> 16) & 0x7fffu) * TY;
    const bool restrict_tile = (tile >> 31) && a.substep == 2;   // uniform over the workgroup
    // ghost tiles (cells or halo hold ghost cells) of the wider formats stage the
    // parent's chi, u, v in LDS (for 16-bit storage it measured slower)
    const bool ghost_tile = sizeof(ST) >= 4 && ((tile >> 15) & 1u);
    const int lx = tx0 + lane, ly = ty0 + wy;
    const long c = (long)ly * pitch + lx;
    const int gx = lx + a.box.gx0, gy = ly + a.box.gy0;

    // buffer resources over the padded allocations; element offset of the cell
    const int pad = a.pad;
    const Rsrc rf = make_rsrc(a.fsrc - pad, 9 * P + 2 * pad);
    const Rsrc rm = make_rsrc(a.msrc - pad, 3 * P + 2 * pad);
    const Rsrc rc = make_rsrc(a.csrc - pad, P + 2 * pad);
    const Rsrc rd = make_rsrc(a.dist - pad, P + 2 * pad);
    const Rsrc rg = make_rsrc(a.flag - pad, P + 2 * pad);
    const uint32_t e = (uint32_t)(c + pad);
    constexpr uint32_t SS = sizeof(ST), CS = sizeof(CT);

    // Every load whose address is known from the tile alone is issued first, in
    // one round: the nine pulls, the wall distance, flags, and the stencil values
    // of the cell and of its halo share (all addresses valid thanks to the spare
    // rows; ghost-band values are replaced below).
    CT s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        s[i] = unshift<ST, CT>(bld<ST, CT>(rf, e * SS, (uint32_t)(i * P - CX[i] - CY[i] * pitch) * SS), a.dsh, i);
    const CT dist = bld<CT, CT>(rd, e * CS, 0);
    const uint8_t fl = __builtin_amdgcn_raw_buffer_load_b8(rg, e, 0, 0);
    // link mask: only cells of the ghost band, next to it, or anchoring a
    // restriction block use it (most tiles have none)
    const uint32_t lm = ((fl & F_TYPE) == T_GHOST || (fl & F_NEARGHOST) || restrict_tile) ? a.lmask[c] : 0u;
    CT own_n = bld<CT, CT>(rc, e * CS, 0), own_u = bld<CT, CT>(rm, e * CS, (uint32_t)P * CS),
       own_v = bld<CT, CT>(rm, e * CS, 2u * (uint32_t)P * CS);
    // halo cells: the row below, the row above, the left and the right column
    bool halo[NS];
    int hx[NS], hy[NS];
    uint8_t hfl[NS];
    CT hn[NS], hu[NS], hv[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int h = (int)threadIdx.x + k * NT;
        halo[k] = h < NH;
        if (h < TILE_X) { hx[k] = h; hy[k] = -1; }
        else if (h < 2 * TILE_X) { hx[k] = h - TILE_X; hy[k] = TY; }
        else if (h < 2 * TILE_X + TY + 2) { hx[k] = -1; hy[k] = h - 2 * TILE_X - 1; }
        else { hx[k] = TILE_X; hy[k] = h - 2 * TILE_X - (TY + 2) - 1; }
        hfl[k] = 0;
        hn[k] = hu[k] = hv[k] = CT(0);
        if (halo[k]) {
            const uint32_t he = (uint32_t)((ty0 + hy[k]) * pitch + tx0 + hx[k] + pad);
            hfl[k] = __builtin_amdgcn_raw_buffer_load_b8(rg, he, 0, 0);
            hn[k] = bld<CT, CT>(rc, he * CS, 0);
            hu[k] = bld<CT, CT>(rm, he * CS, (uint32_t)P * CS);
            hv[k] = bld<CT, CT>(rm, he * CS, 2u * (uint32_t)P * CS);
        }
    }
    // The ghost fill of a ghost tile reads the parent's chi, u, v from LDS, staged
    // here from the first round of loads, instead of 27 scattered loads per ghost
    // cell issued once the flags have come (the tiles that end the latency-bound
    // launches).  Reads are bounds-checked: what lies outside the parent's box
    // reads 0, and no ghost cell's stencil reaches it.
    constexpr int GR = TY / 2 + 4;
    const int cpx0 = ((a.box.gx0 + tx0 - 1) >> 1) - 1, cpy0 = ((a.box.gy0 + ty0 - 1) >> 1) - 1;
    if (ghost_tile) {
        const Rsrc rcn = make_rsrc(a.cchi, a.cbox.plane);
        const Rsrc rcu = make_rsrc(a.cmac + a.cbox.plane, a.cbox.plane);
        const Rsrc rcv = make_rsrc(a.cmac + 2 * a.cbox.plane, a.cbox.plane);
        for (int k = (int)threadIdx.x; k < GR * GC_W; k += NT) {
            const int r = k / GC_W, w = k - r * GC_W;
            const long q = (long)(cpy0 + r - a.cbox.gy0) * a.cbox.pitch + (cpx0 + w - a.cbox.gx0);
            const uint32_t o = (uint32_t)q * CS;
            lds.gc[0][r][w] = bld<CT, CT>(rcn, o, 0);
            lds.gc[1][r][w] = bld<CT, CT>(rcu, o, 0);
            lds.gc[2][r][w] = bld<CT, CT>(rcv, o, 0);
        }
        __syncthreads();
    }
    const int type = fl & F_TYPE;
    // 16-bit storage issues the parent-level loads of ghost and near-ghost cells
    // before the stencil staging, so that they overlap the barrier; wider formats
    // after it (each order measured the faster for its formats; the order changes
    // no result).  The ghost cells' stores and the coalescence follow the barrier.
    constexpr bool early = sizeof(ST) == 2;
    if constexpr (early) parent_pops<ST, CT>(a, type, fl, lm, gx, gy, s);
    if (type == T_GHOST) {
        if (ghost_tile) ghost_fill_lds<CT, TY>(lds, cpx0, cpy0, gx, gy, own_n, own_u, own_v);
        else ghost_fill(a.cmac, a.cchi, a.cbox, gx, gy, own_n, own_u, own_v);
    }
    sh_n[wy + 1][lane + 1] = own_n;
    sh_u[wy + 1][lane + 1] = own_u;
    sh_v[wy + 1][lane + 1] = own_v;
#pragma unroll
    for (int k = 0; k < NS; ++k)
        if (halo[k]) {
            if ((hfl[k] & F_TYPE) == T_GHOST) {
                const int hgx = a.box.gx0 + tx0 + hx[k], hgy = a.box.gy0 + ty0 + hy[k];
                if (ghost_tile) ghost_fill_lds<CT, TY>(lds, cpx0, cpy0, hgx, hgy, hn[k], hu[k], hv[k]);
                else ghost_fill(a.cmac, a.cchi, a.cbox, hgx, hgy, hn[k], hu[k], hv[k]);
            }
            sh_n[hy[k] + 1][hx[k] + 1] = hn[k];
            sh_u[hy[k] + 1][hx[k] + 1] = hu[k];
            sh_v[hy[k] + 1][hx[k] + 1] = hv[k];
        }
    __syncthreads();

    const Rsrc rfo = make_rsrc(a.fdst - pad, 9 * P + 2 * pad);
    bool update = false;
    CT m_rho = CT(0), m_ux = CT(0), m_uy = CT(0), m_chi = CT(0);
    if constexpr (!early) parent_pops<ST, CT>(a, type, fl, lm, gx, gy, s);
    if (type == T_GHOST) {
        ghost_band_store<ST, CT>(a, s, rfo, e, P);
    } else if (type == T_FLUID && !(fl & (F_WALL | F_EDGE))) {   // others: side-stream kernels
        update = true;
        iface_cell<ST, CT>(a, fl, gx, gy, s);
        // SA-neg: chi at the new time level
        CT chi_new;
        if (a.frozen) {
            chi_new = sh_n[wy + 1][lane + 1];
        } else {
            CT nt[9], u[9], v[9];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int k = (dy + 1) * 3 + dx + 1;
                    nt[k] = sh_n[wy + 1 + dy][lane + 1 + dx] * a.nu;
                    u[k] = sh_u[wy + 1 + dy][lane + 1 + dx];
                    v[k] = sh_v[wy + 1 + dy][lane + 1 + dx];
                }
            chi_new = fdiv(sa_update(nt, u, v, a.nu, dist, a.sa_mode == 2, a.mu_cap), a.nu);
        }
        relax_cell(a, s, chi_new, m_rho, m_ux, m_uy);
        absorb(a, gx, gy, s);
        m_chi = chi_new;
        const Rsrc rmo = make_rsrc(a.mdst - pad, 3 * P + 2 * pad);
        const Rsrc rco = make_rsrc(a.cdst - pad, P + 2 * pad);
        bst<CT, CT>(rmo, e * CS, 0, m_rho);
        bst<CT, CT>(rmo, e * CS, (uint32_t)P * CS, m_ux);
        bst<CT, CT>(rmo, e * CS, 2u * (uint32_t)P * CS, m_uy);
        bst<CT, CT>(rco, e * CS, 0, chi_new);
#pragma unroll
        for (int i = 0; i < 9; ++i) bst<ST, CT>(rfo, e * SS, (uint32_t)(i * P) * SS, toshift<ST, CT>(s[i], a.dsh, i));
    }
    if (!restrict_tile) return;
    // restriction for the next parent step: the new rho, u and chi of each 2 x 2
    // block under a covered coarse cell, averaged by the block's lower-left cell
    auto& sh_r = lds.r;
    __syncthreads();
    if (update) {
        sh_r[0][wy][lane] = m_rho;
        sh_r[1][wy][lane] = m_ux;
        sh_r[2][wy][lane] = m_uy;
        sh_r[3][wy][lane] = m_chi;
    }
    __syncthreads();
    if (lm >> 31) {
        // the block's lower-left cell sits at an even local row and column (the
        // host keeps box origins and tile heights even), so wy + 1 < TY and
        // lane + 1 < TILE_X
        const long q = (long)((gy >> 1) - a.cbox.gy0) * a.cbox.pitch + ((gx >> 1) - a.cbox.gx0);
        CT m[4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
            m[f] = CT(0.25) * ((sh_r[f][wy][lane] + sh_r[f][wy][lane + 1]) +
                               (sh_r[f][wy + 1][lane] + sh_r[f][wy + 1][lane + 1]));
        a.rmac[q] = m[0];
        a.rmac[a.cbox.plane + q] = m[1];
        a.rmac[2 * a.cbox.plane + q] = m[2];
        a.rchi[q] = m[3];
    }
}


// One level sub-step of one case.
template <class ST, class CT, int TY>
__global__ __launch_bounds__(TILE_X * TY, 8) void k_step(const StepArgs<ST, CT> a) {
    step_block<ST, CT, TY>(a, (int)blockIdx.x);
}

// One launch for the same virtual level of several cases (batched sweep): the
// grid is split into parts, part p starting at block start[p] (a multiple of 8,
// so the XCD mapping of each part is kept) with its arguments in parts[p].
template <class ST, class CT, int TY>
__global__ __launch_bounds__(TILE_X * TY, 8) void k_step_batch(const StepArgs<ST, CT>* __restrict__ parts,
                                                     const int* __restrict__ start, int nparts) {
    int p = 0;
    while (p + 1 < nparts && (int)blockIdx.x >= start[p + 1]) ++p;
    step_block<ST, CT, TY>(parts[p], (int)blockIdx.x - start[p]);
}

// The same for the launches of mixed-storage cases that hold FP32- and
// FP16-stored levels (FP32 arithmetic both): each part's own format (sst)
// selects the instantiation, a branch uniform over the workgroup.  The two
// argument types differ only in the pointee type of the population pointers.
static_assert(sizeof(StepArgs<float, float>) == sizeof(StepArgs<__half, float>) &&
                  alignof(StepArgs<float, float>) == alignof(StepArgs<__half, float>),
              "mixed launch tables hold both argument types");
template <int TY>
__global__ __launch_bounds__(TILE_X * TY, 8) void k_step_batch_mixed(const StepArgs<float, float>* __restrict__ parts,
                                                           const int* __restrict__ start, int nparts) {
    int p = 0;
    while (p + 1 < nparts && (int)blockIdx.x >= start[p + 1]) ++p;
    const int blk = (int)blockIdx.x - start[p];
    if (parts[p].sst == P_F16)
        step_block<__half, float, TY>(*reinterpret_cast<const StepArgs<__half, float>*>(parts + p), blk);
    else
        step_block<float, float, TY>(parts[p], blk);
}

// Grid-wide barrier of a co-resident grid, in two levels.  A launch boundary
// writes back and invalidates each XCD's L2 once; a barrier in which every
// workgroup made its writes visible at device scope would do so once per
// workgroup, about 250 times per XCD.  So the workgroups of one XCD (grouped by
// the hardware's XCC id, read at the start of the grid) count themselves in at
// the group's counter once their stores have reached the XCD's L2; the last of
// the group writes that L2 back to memory and counts the group in at the grid
// counter; the last group opens the grid's next generation; each group's last
// workgroup then opens its group, and every workgroup discards its stale cache
// lines.  The step inside a group rests on the hardware, not on the language's
// memory model: the vector L1 writes through, a store has reached the XCD's L2
// when the wave's memory counter has drained, and one L2 serves every compute
// unit of the XCD, so the writeback of the group's last workgroup carries the
// stores of the whole group.  Between groups, release and acquire at device
// scope order everything.  The waits poll with relaxed loads (an acquire on every poll would
// invalidate the L2 under the workgroups still computing) and are bounded:
// past spin_limit polls a wait sets the flag word and gives up, which only a
// grid that is not co-resident can reach (the cooperative launch refuses such
// grids).
//
// Words of bar (zero before the first grid): [0] group arrivals at the grid
// counter, [1] grid generation, [2] time-out flag, [3] workgroups registered,
// [4] groups; group x at BAR_STRIDE * (x + 1): [0] arrivals, [1] generation,
// [2] members.
constexpr unsigned BARRIER_SPIN_LIMIT = 1u << 20;   // far beyond any sub-launch of the batch

__device__ __forceinline__ unsigned xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (BAR_XCC - 1);   // HW_REG_XCC_ID, bits 0-3
}

__device__ __forceinline__ unsigned ld_relaxed(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned add_relaxed(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls *p until it differs from old (want_equal = false) or equals old (true).
__device__ __forceinline__ void bounded_wait(unsigned* p, unsigned old, bool want_equal, unsigned* flag,
                                             unsigned spin_limit) {
    unsigned n = 0;
    while ((ld_relaxed(p) == old) != want_equal) {
        if (++n > spin_limit) {
            st_relaxed(flag, 1u);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// First thread of each workgroup: join the group of its XCD and wait until the
// whole grid has; returns the group size and sets *x to the group.
__device__ __forceinline__ unsigned grid_register(unsigned* bar, unsigned nblocks, unsigned* x, unsigned spin_limit) {
    *x = xcc_id();
    unsigned* g = bar + BAR_STRIDE * (*x + 1);
    if (add_relaxed(g + 2, 1u) == 0) add_relaxed(bar + 4, 1u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the two counts above before the registration
    add_relaxed(bar + 3, 1u);
    bounded_wait(bar + 3, nblocks, true, bar + 2, spin_limit);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every workgroup's counts after it
    return ld_relaxed(g + 2);
}

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned x, unsigned members, unsigned ngroups,
                                             unsigned spin_limit) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the XCD's L2
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* g = bar + BAR_STRIDE * (x + 1);
        const unsigned ggen = ld_relaxed(g + 1);
        if (add_relaxed(g, 1u) == members - 1) {
            st_relaxed(g, 0u);
            const unsigned gen = ld_relaxed(bar + 1);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the XCD's L2 (the whole group's writes) to memory
            if (add_relaxed(bar, 1u) == ngroups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                st_relaxed(bar, 0u);
                __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                bounded_wait(bar + 1, gen, false, bar + 2, spin_limit);
            }
            // release: the reset of the group's count before a member's next arrival
            __hip_atomic_fetch_add(g + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            bounded_wait(g + 1, ggen, false, bar + 2, spin_limit);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // drop stale L1 and L2 lines
    }
    __syncthreads();
}

// The launches of a batch table run by one cooperative grid: each workgroup
// takes the blocks b = blockIdx.x, blockIdx.x + gridDim.x, ... of every
// sub-launch (the grid is a multiple of 8 workgroups, so each block keeps the
// XCD the direct launch gives it), and a grid-wide barrier separates the
// sub-launches as the launch boundaries of the merged schedule do.  The
// registration words are cleared after the first barrier, when every
// workgroup has read its group size, for the next grid on the same words.
template <class ST, class CT>
__global__ __launch_bounds__(TILE_X * PERSISTENT_TY, 8) void k_step_persistent(
        const StepArgs<ST, CT>* __restrict__ parts, const int* __restrict__ start, const PLaunch* __restrict__ launches,
        int nlaunches, unsigned* bar) {
    unsigned x = 0, members = 0, ngroups = 0;
    if (nlaunches > 1 && threadIdx.x == 0) {
        members = grid_register(bar, gridDim.x, &x, BARRIER_SPIN_LIMIT);
        ngroups = ld_relaxed(bar + 4);
    }
    for (int L = 0; L < nlaunches; ++L) {
        const PLaunch ln = launches[L];
        for (int b = (int)blockIdx.x; b < ln.nblocks; b += (int)gridDim.x) {
            int p = 0;
            while (p + 1 < ln.nparts && b >= start[ln.part0 + p + 1]) ++p;
            step_block<ST, CT, PERSISTENT_TY>(parts[ln.part + p], b - start[ln.part0 + p]);
            __syncthreads();   // the next block reuses the LDS
        }
        if (L + 1 < nlaunches) {
            grid_barrier(bar, x, members, ngroups, BARRIER_SPIN_LIMIT);
            if (L == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
                st_relaxed(bar + 3, 0u);
                st_relaxed(bar + 4, 0u);
                for (int k = 0; k < BAR_XCC; ++k) st_relaxed(bar + BAR_STRIDE * (k + 1) + 2, 0u);
            }
        }
    }
}

// Wall model on the current state, for output.
template <class CT>
__global__ __launch_bounds__(64) void k_wall(const WallArgs<CT> a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.wall.nb) return;
    double wm[6];
    wall_model<CT>(a.wall, b, a.mac, a.plane, a.nu, a.guess[8 * b], wm);
    for (int k = 0; k < 6; ++k) a.out[8 * b + k] = wm[k];
}

// ---------------------------------------------------------------------------
// Level transfers of the macroscopic fields used by the SA stencils.
// ---------------------------------------------------------------------------
template <class CT>
__global__ void k_fill(const FillArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const long g = a.list[k];
    const int lx = (int)(g % a.fbox.pitch), ly = (int)(g / a.fbox.pitch);
    const int gx = lx + a.fbox.gx0, gy = ly + a.fbox.gy0;
    const int px = gx >> 1, py = gy >> 1;
    const CT ox = (gx & 1) ? CT(0.25) : CT(-0.25), oy = (gy & 1) ? CT(0.25) : CT(-0.25);
    const CT* cm = (const CT*)a.cmac;
    const CT* cc = (const CT*)a.cchi;
    CT sum[4] = {0, 0, 0, 0}, sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const long q = (long)(py + dy - a.cbox.gy0) * a.cbox.pitch + (px + dx - a.cbox.gx0);
            const CT v[4] = {cm[q], cm[a.cbox.plane + q], cm[2 * a.cbox.plane + q], cc[q]};
            for (int f = 0; f < 4; ++f) {
                sum[f] += v[f];
                sx[f] += CT(dx) * v[f];
                sy[f] += CT(dy) * v[f];
            }
        }
    // linear least-squares fit over the 3 x 3 coarse neighbourhood, at the child's centre
    CT out[4];
    for (int f = 0; f < 4; ++f)
        out[f] = sum[f] * CT(1.0 / 9.0) + ox * sx[f] * CT(1.0 / 6.0) + oy * sy[f] * CT(1.0 / 6.0);
    CT* m0 = (CT*)a.fmac0;
    CT* m1 = (CT*)a.fmac1;
    for (int f = 0; f < 3; ++f) {
        m0[f * a.fbox.plane + g] = out[f];
        m1[f * a.fbox.plane + g] = out[f];
    }
    ((CT*)a.fchi0)[g] = out[3];
    ((CT*)a.fchi1)[g] = out[3];
}

template <class CT>
__global__ void k_restrict(const RestrictArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const long g = a.list[k];
    const int lx = (int)(g % a.cbox.pitch), ly = (int)(g / a.cbox.pitch);
    const int gx = lx + a.cbox.gx0, gy = ly + a.cbox.gy0;
    const long f0 = (long)(2 * gy - a.fbox.gy0) * a.fbox.pitch + (2 * gx - a.fbox.gx0);
    const CT* fm = (const CT*)a.fmac;
    const CT* fc = (const CT*)a.fchi;
    CT* cm = (CT*)a.cmac;
    for (int f = 0; f < 3; ++f) {
        const CT* p = fm + f * a.fbox.plane + f0;
        cm[f * a.cbox.plane + g] = CT(0.25) * ((p[0] + p[1]) + (p[a.fbox.pitch] + p[a.fbox.pitch + 1]));
    }
    const CT* p = fc + f0;
    ((CT*)a.cchi)[g] = CT(0.25) * ((p[0] + p[1]) + (p[a.fbox.pitch] + p[a.fbox.pitch + 1]));
}

// Equilibrium initialisation followed by the first collision.
template <class ST, class CT>
__global__ void k_init(const InitArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const long c = a.list[k];
    CT s[9];
    equilibrium<CT>(s, CT(a.rho[k] - 1.0), CT(a.ux[k]), CT(a.uy[k]));
    CT drho = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
        drho += s[i];
        jx += CT(CX[i]) * s[i];
        jy += CT(CY[i]) * s[i];
    }
    const CT rho = CT(1) + drho;
    const CT ux = (jx + CT(0.5 * a.fx)) / rho, uy = (jy + CT(0.5 * a.fy)) / rho;
    CT* mac = (CT*)a.mac;
    mac[c] = rho;
    mac[a.plane + c] = ux;
    mac[2 * a.plane + c] = uy;
    const CT chi = CT(a.chi[k]);
    ((CT*)a.chi_a)[c] = chi;
    ((CT*)a.chi_b)[c] = chi;
    const CT nu = CT(a.nu);
    const CT omega = CT(1) / (CT(3) * (nu + eddy_viscosity(chi, nu)) + CT(0.5));
    collide(s, drho, ux, uy, omega, CT(a.omega_b), CT(a.fx), CT(a.fy));
    absorb<CT>(a.sp, a.nxd, a.nyd, (int)(c % a.pitch) + a.gx0, (int)(c / a.pitch) + a.gy0, s);
    ST* f = (ST*)a.f;
    CT d[9];
    for (int i = 0; i < 9; ++i) d[i] = CT(a.dsh[i]);
    for (int i = 0; i < 9; ++i) Cv<ST, CT>::st(f + i * a.plane + c, toshift<ST, CT>(s[i], d, i));
}

// ---------------------------------------------------------------------------
// Geometry: FP64 distance to the wall polylines and even-odd inside test, per
// cell centre of a level's storage box.
// ---------------------------------------------------------------------------
__global__ void k_geometry(int nx, int ny, int gx0, int gy0, double scale, int nbody,
                           const int* off, const double* poly, int solid, double* dist,
                           uint8_t* inside) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long)nx * ny) return;
    const double px = (double)(k % nx + gx0) + 0.5, py = (double)(k / nx + gy0) + 0.5;
    double best2 = 1e300;
    int in_any = 0;
    for (int b = 0; b < nbody; ++b) {
        const int s0 = off[b], n = off[b + 1] - off[b];
        int in = 0;
        for (int j = 0; j < n; ++j) {
            const int j1 = (j + 1 == n) ? 0 : j + 1;
            const double ax = poly[2 * (s0 + j)] * scale, ay = poly[2 * (s0 + j) + 1] * scale;
            const double bx = poly[2 * (s0 + j1)] * scale, by = poly[2 * (s0 + j1) + 1] * scale;
            const double ex = bx - ax, ey = by - ay;
            const double l2 = ex * ex + ey * ey;
            double t = l2 > 0.0 ? ((px - ax) * ex + (py - ay) * ey) / l2 : 0.0;
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            const double dx = px - (ax + t * ex), dy = py - (ay + t * ey);
            const double d2 = dx * dx + dy * dy;
            best2 = d2 < best2 ? d2 : best2;
            if ((ay > py) != (by > py)) {
                const double xc = ax + (py - ay) * (bx - ax) / (by - ay);
                if (px < xc) in = !in;
            }
        }
        in_any |= in;
    }
    dist[k] = nbody > 0 ? sqrt(best2) : 1e300;
    inside[k] = (uint8_t)(solid && in_any);
}

// ---------------------------------------------------------------------------
// Surface coefficients and force sums (eqs (29)-(30)), FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <class CT>
__global__ __launch_bounds__(256) void k_surface(const SurfaceArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[4] = {0, 0, 0, 0};
    if (k < a.nseg) {
        const double* sg = a.seg + 6 * k;
        double sw = 0.0, scp = 0.0, scf = 0.0;
        const double U2 = a.u_ref * a.u_ref;
        for (int m = 0; m < 2; ++m) {
            const int b = a.near[2 * k + m];
            if (b < 0) continue;
            const double w = a.wgt[2 * k + m];
            const double* st = a.bstate + 8 * b;
            const double rhow = st[3];
            const double cpb = 2.0 * (1.0 / 3.0) * (rhow - a.rho_ref) / (a.rho_ref * U2);
            const double cfb = 2.0 * (rhow / a.rho_ref) * st[0] * st[0] / U2;
            const double sg_ = (st[1] * sg[0] + st[2] * sg[1] >= 0.0) ? 1.0 : -1.0;
            sw += w;
            scp += w * cpb;
            scf += w * cfb * sg_;
        }
        const double cp = scp / sw, cf = scf / sw;
        a.cp[k] = cp;
        a.cf[k] = cf;
        acc[0] = cf * sg[0] * sg[4];
        acc[1] = cf * sg[1] * sg[4];
        acc[2] = -cp * sg[2] * sg[4];
        acc[3] = -cp * sg[3] * sg[4];
    }
    __shared__ double part[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int f = 0; f < 4; ++f) {
        const double v = wave_sum(acc[f]);
        if (lane == 0) part[wv][f] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int f = threadIdx.x;
        a.partial[4 * blockIdx.x + f] = (part[0][f] + part[1][f]) + (part[2][f] + part[3][f]);
    }
}

template <class CT>
__global__ __launch_bounds__(256) void k_residual(const CT* mac, double* snap, const int32_t* list,
                                                 int n, long plane, double area, double* partial) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double du = 0.0, uu = 0.0;
    if (k < n) {
        const long c = list[k];
        const double ux = (double)mac[plane + c], uy = (double)mac[2 * plane + c];
        const double dx = ux - snap[2 * k], dy = uy - snap[2 * k + 1];
        du = area * (dx * dx + dy * dy);
        uu = area * (ux * ux + uy * uy);
        snap[2 * k] = ux;
        snap[2 * k + 1] = uy;
    }
    __shared__ double part[4][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    du = wave_sum(du);
    uu = wave_sum(uu);
    if (lane == 0) { part[wv][0] = du; part[wv][1] = uu; }
    __syncthreads();
    if (threadIdx.x < 2)
        partial[2 * blockIdx.x + threadIdx.x] =
            (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

template <class CT>
__global__ void k_to_double(const CT* src, double* dst, long n) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = (double)src[k];
}

// One field of a level over its I/O box, into a device array (the layout of
// the host readout): the cell type for TYPE, NaN outside the owned fluid, and
// nu_t = nu chi f_v1(chi) for NUT.
template <class CT>
__global__ void k_field(const FieldArgs a) {
#pragma clang fp contract(off)   // the same roundings as the host readout (no fused multiply-add)
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long)a.bnx * a.bny) return;
    const long i = k % a.bnx, j = k / a.bnx;
    const long c = (a.oy + j) * a.pitch + (a.ox + i);
    const int t = a.flag[c] & F_TYPE;
    double o;
    if (a.field == 5) o = t;
    else if (t != T_FLUID) o = __builtin_nan("");
    else if (a.field == 6) o = (double)static_cast<const CT*>(a.dist)[c];
    else {
        const double x = (double)static_cast<const CT*>(a.src)[c];
        o = a.field == 4 ? (x > 0 ? a.nu * x * x * x * x / (x * x * x + 7.1 * 7.1 * 7.1) : 0.0) : x;
    }
    a.out[k] = o;
}

// Values of a plane at listed cells (diagnostics): dst[k] = src[idx[k]].
template <class CT>
__global__ void k_gather(const CT* src, const int64_t* idx, int n, double* dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = (double)src[idx[k]];
}

inline unsigned nblocks(long n, int b) { return (unsigned)((n + b - 1) / b); }

// Plain launch, or with start / stop events attached to the dispatch itself
// (kernel execution time without the cost of separate event records).
template <class K, class A>
inline void launch_timed(K kernel, dim3 g, dim3 b, hipStream_t s, const Timing& tm, const A& a) {
    if (tm.start) hipExtLaunchKernelGGL(kernel, g, b, 0, s, tm.start, tm.stop, 0, a);
    else hipLaunchKernelGGL(kernel, g, b, 0, s, a);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class ST, class CT, int TY>
static hipError_t step_ty(const StepArgs<ST, CT>& a, hipStream_t s, const Timing& tm) {
    const unsigned grid = (unsigned)(a.wall_blocks + a.tile_blocks) + nblocks(a.nedge, TILE_X * TY);
    if (grid == 0) return hipSuccess;
    launch_timed(k_step<ST, CT, TY>, dim3(grid), dim3(TILE_X * TY), s, tm, a);
    return hipGetLastError();
}

template <class ST, class CT>
static hipError_t step_t(const void* args, hipStream_t s, const Timing& tm) {
    const auto& a = *static_cast<const StepArgs<ST, CT>*>(args);
    switch (a.ty) {
        case 2: return step_ty<ST, CT, 2>(a, s, tm);
        case 4: return step_ty<ST, CT, 4>(a, s, tm);
        case 8: return step_ty<ST, CT, 8>(a, s, tm);
        case 16: return step_ty<ST, CT, 16>(a, s, tm);
        default: return hipErrorInvalidValue;
    }
}

template <class ST, class CT, int TY>
static hipError_t batch_ty(const StepArgs<ST, CT>* pa, const int* start, int nparts, int nblocks_total,
                           hipStream_t s, const Timing& tm) {
    if (tm.start)
        hipExtLaunchKernelGGL((k_step_batch<ST, CT, TY>), dim3(nblocks_total), dim3(TILE_X * TY), 0, s,
                              tm.start, tm.stop, 0, pa, start, nparts);
    else
        hipLaunchKernelGGL((k_step_batch<ST, CT, TY>), dim3(nblocks_total), dim3(TILE_X * TY), 0, s,
                           pa, start, nparts);
    return hipGetLastError();
}

template <class ST, class CT>
static hipError_t batch_t(const void* parts, const int* start, int nparts, int nblocks_total, int ty,
                          hipStream_t s, const Timing& tm) {
    if (nblocks_total == 0) return hipSuccess;
    const auto* pa = static_cast<const StepArgs<ST, CT>*>(parts);
    switch (ty) {
        case 2: return batch_ty<ST, CT, 2>(pa, start, nparts, nblocks_total, s, tm);
        case 4: return batch_ty<ST, CT, 4>(pa, start, nparts, nblocks_total, s, tm);
        case 8: return batch_ty<ST, CT, 8>(pa, start, nparts, nblocks_total, s, tm);
        case 16: return batch_ty<ST, CT, 16>(pa, start, nparts, nblocks_total, s, tm);
        default: return hipErrorInvalidValue;
    }
}

template <int TY>
static hipError_t batch_mixed_ty(const StepArgs<float, float>* pa, const int* start, int nparts, int nblocks_total,
                                 hipStream_t s, const Timing& tm) {
    if (tm.start)
        hipExtLaunchKernelGGL((k_step_batch_mixed<TY>), dim3(nblocks_total), dim3(TILE_X * TY), 0, s,
                              tm.start, tm.stop, 0, pa, start, nparts);
    else
        hipLaunchKernelGGL((k_step_batch_mixed<TY>), dim3(nblocks_total), dim3(TILE_X * TY), 0, s,
                           pa, start, nparts);
    return hipGetLastError();
}

static hipError_t batch_mixed(const void* parts, const int* start, int nparts, int nblocks_total, int ty,
                              hipStream_t s, const Timing& tm) {
    if (nblocks_total == 0) return hipSuccess;
    const auto* pa = static_cast<const StepArgs<float, float>*>(parts);
    switch (ty) {
        case 2: return batch_mixed_ty<2>(pa, start, nparts, nblocks_total, s, tm);
        case 4: return batch_mixed_ty<4>(pa, start, nparts, nblocks_total, s, tm);
        case 8: return batch_mixed_ty<8>(pa, start, nparts, nblocks_total, s, tm);
        case 16: return batch_mixed_ty<16>(pa, start, nparts, nblocks_total, s, tm);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_batch(Prec p, const void* parts, const int* start, int nparts, int nblocks_total, int ty,
                             hipStream_t s, const Timing& tm) {
    switch (p) {
        case P_MIXED: return batch_mixed(parts, start, nparts, nblocks_total, ty, s, tm);
        case P_F64: return batch_t<double, double>(parts, start, nparts, nblocks_total, ty, s, tm);
        case P_F32: return batch_t<float, float>(parts, start, nparts, nblocks_total, ty, s, tm);
        case P_F16: return batch_t<__half, float>(parts, start, nparts, nblocks_total, ty, s, tm);
        default: return batch_t<__hip_bfloat16, float>(parts, start, nparts, nblocks_total, ty, s, tm);
    }
}

template <class ST, class CT>
static hipError_t persistent_t(const void* parts, const int* start, const PLaunch* launches, int nlaunches, int grid,
                               unsigned* bar, hipStream_t s) {
    const StepArgs<ST, CT>* pa = static_cast<const StepArgs<ST, CT>*>(parts);
    void* args[] = {(void*)&pa, (void*)&start, (void*)&launches, (void*)&nlaunches, (void*)&bar};
    return hipLaunchCooperativeKernel((const void*)k_step_persistent<ST, CT>, dim3(grid),
                                      dim3(TILE_X * PERSISTENT_TY), args, 0, s);
}

hipError_t launch_step_persistent(Prec p, const void* parts, const int* start, const PLaunch* launches, int nlaunches,
                                  int grid, unsigned* bar, hipStream_t s) {
    if (nlaunches == 0) return hipSuccess;
    switch (p) {
        case P_F64: return persistent_t<double, double>(parts, start, launches, nlaunches, grid, bar, s);
        case P_F32: return persistent_t<float, float>(parts, start, launches, nlaunches, grid, bar, s);
        case P_F16: return persistent_t<__half, float>(parts, start, launches, nlaunches, grid, bar, s);
        case P_BF16: return persistent_t<__hip_bfloat16, float>(parts, start, launches, nlaunches, grid, bar, s);
        default: return hipErrorInvalidValue;
    }
}

template <class ST, class CT>
static hipError_t grid_t(int* grid) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_persistent<ST, CT>,
                                                                TILE_X * PERSISTENT_TY, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *grid = per_cu * cus / 8 * 8;
    return *grid > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t persistent_grid(Prec p, int* grid) {
    switch (p) {
        case P_F64: return grid_t<double, double>(grid);
        case P_F32: return grid_t<float, float>(grid);
        case P_F16: return grid_t<__half, float>(grid);
        case P_BF16: return grid_t<__hip_bfloat16, float>(grid);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(Prec p, const void* args, hipStream_t s, const Timing& tm) {
    switch (p) {
        case P_F64: return step_t<double, double>(args, s, tm);
        case P_F32: return step_t<float, float>(args, s, tm);
        case P_F16: return step_t<__half, float>(args, s, tm);
        default: return step_t<__hip_bfloat16, float>(args, s, tm);
    }
}

hipError_t launch_wall(Prec p, const void* args, hipStream_t s) {
    if (p == P_F64) {
        const auto& a = *static_cast<const WallArgs<double>*>(args);
        if (a.wall.nb == 0) return hipSuccess;
        hipLaunchKernelGGL(k_wall<double>, dim3(nblocks(a.wall.nb, 64)), dim3(64), 0, s, a);
    } else {
        const auto& a = *static_cast<const WallArgs<float>*>(args);
        if (a.wall.nb == 0) return hipSuccess;
        hipLaunchKernelGGL(k_wall<float>, dim3(nblocks(a.wall.nb, 64)), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_fill(Prec p, const FillArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (p == P_F64) hipLaunchKernelGGL(k_fill<double>, dim3(nblocks(a.n, 256)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_fill<float>, dim3(nblocks(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_restrict(Prec p, const RestrictArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (p == P_F64) hipLaunchKernelGGL(k_restrict<double>, dim3(nblocks(a.n, 256)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_restrict<float>, dim3(nblocks(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init(Prec p, const InitArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 g(nblocks(a.n, 256)), b(256);
    switch (p) {
        case P_F64: hipLaunchKernelGGL((k_init<double, double>), g, b, 0, s, a); break;
        case P_F32: hipLaunchKernelGGL((k_init<float, float>), g, b, 0, s, a); break;
        case P_F16: hipLaunchKernelGGL((k_init<__half, float>), g, b, 0, s, a); break;
        default: hipLaunchKernelGGL((k_init<__hip_bfloat16, float>), g, b, 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_geometry(int nx, int ny, int gx0, int gy0, double scale, int nbody,
                           const int* off, const double* poly, int solid, double* dist,
                           uint8_t* inside, hipStream_t s) {
    hipLaunchKernelGGL(k_geometry, dim3(nblocks((long)nx * ny, 256)), dim3(256), 0, s, nx, ny,
                       gx0, gy0, scale, nbody, off, poly, solid, dist, inside);
    return hipGetLastError();
}

hipError_t launch_surface(Prec p, const SurfaceArgs& a, int nb, hipStream_t s) {
    if (p == P_F64) hipLaunchKernelGGL(k_surface<double>, dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_surface<float>, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Health scans: a cell fails when its density is not finite or not positive or its
// speed exceeds the lattice sound speed; a wall node when its friction velocity is
// not finite.  Each failure sets its bit and one (level, index) pair (vector atomics).
template <class CT>
__global__ void k_health(const CT* mac, const int32_t* list, int n, long plane, int level, int* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const long c = list[k];
    const double rho = (double)mac[c], ux = (double)mac[plane + c], uy = (double)mac[2 * plane + c];
    const bool ok = isfinite(rho) && rho > 0.0 && isfinite(ux) && isfinite(uy) && ux * ux + uy * uy <= 1.0 / 3.0;
    if (!ok) {
        atomicOr(out, 1);
        atomicExch(out + 1, level);
        atomicExch(out + 2, (int)c);
        atomicAdd(out + 3, 1);
    }
}

__global__ void k_health_wall(const double* bstate, int nb, int level, int* out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    if (!isfinite(bstate[8 * b])) {
        atomicOr(out, 2);
        atomicExch(out + 1, level);
        atomicExch(out + 2, b);
    }
}

__global__ void k_health_reset(int* out) {
    if (threadIdx.x < 4) out[threadIdx.x] = 0;
}

hipError_t launch_health_reset(int* out, hipStream_t s) {
    hipLaunchKernelGGL(k_health_reset, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}

hipError_t launch_health(Prec p, const void* mac, const int32_t* list, int n, long plane, int level, int* out,
                         hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (p == P_F64)
        hipLaunchKernelGGL(k_health<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, (const double*)mac, list, n,
                           plane, level, out);
    else
        hipLaunchKernelGGL(k_health<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, (const float*)mac, list, n,
                           plane, level, out);
    return hipGetLastError();
}

hipError_t launch_health_wall(const double* bstate, int nb, int level, int* out, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_health_wall, dim3(nblocks(nb, 256)), dim3(256), 0, s, bstate, nb, level, out);
    return hipGetLastError();
}

hipError_t launch_residual(Prec p, const void* mac, double* snap, const int32_t* list, int n,
                           long plane, double area, double* partial, int nb, hipStream_t s) {
    if (p == P_F64)
        hipLaunchKernelGGL(k_residual<double>, dim3(nb), dim3(256), 0, s, (const double*)mac, snap,
                           list, n, plane, area, partial);
    else
        hipLaunchKernelGGL(k_residual<float>, dim3(nb), dim3(256), 0, s, (const float*)mac, snap,
                           list, n, plane, area, partial);
    return hipGetLastError();
}

hipError_t launch_field(Prec p, const FieldArgs& a, hipStream_t s) {
    const long n = (long)a.bnx * a.bny;
    if (n == 0) return hipSuccess;
    if (p == P_F64) hipLaunchKernelGGL(k_field<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_field<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(Prec p, const void* src, const int64_t* idx, int n, double* dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (p == P_F64)
        hipLaunchKernelGGL(k_gather<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, (const double*)src, idx, n, dst);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, (const float*)src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_to_double(Prec p, const void* src, double* dst, long n, hipStream_t s) {
    if (p == P_F64)
        hipLaunchKernelGGL(k_to_double<double>, dim3(nblocks(n, 256)), dim3(256), 0, s,
                           (const double*)src, dst, n);
    else
        hipLaunchKernelGGL(k_to_double<float>, dim3(nblocks(n, 256)), dim3(256), 0, s,
                           (const float*)src, dst, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free entry point.  In host code `scratch`
// names a host-side stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, once per device with that device current, and only that
// address is handed to kernels and copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** ptr) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace lbr
