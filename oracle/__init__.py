"""Python access to the FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

MAX_LEVELS = 12
WALL_STRIDE = 28
F_RHO, F_UX, F_UY, F_CHI, F_NUT, F_TYPE, F_DIST = range(7)
T_INACTIVE, T_FLUID, T_SOLID, T_GHOST, T_COVERED, T_VIRT = range(6)   # values of F_TYPE


class Config(C.Structure):
    _fields_ = [
        ("nx0", C.c_int32), ("ny0", C.c_int32), ("n_levels", C.c_int32),
        ("bc", C.c_int32 * 4),
        ("wall_model", C.c_int32), ("bb_mode", C.c_int32), ("sa_mode", C.c_int32),
        ("body_mode", C.c_int32), ("outlet", C.c_int32),
        ("origin", C.c_double * 2), ("dx0", C.c_double),
        ("band", C.c_double * MAX_LEVELS), ("wall_y", C.c_double * 2),
        ("mach", C.c_double), ("reynolds", C.c_double), ("ref_length", C.c_double),
        ("u_ref", C.c_double), ("nu0", C.c_double),
        ("rho_ref", C.c_double), ("chi_inlet", C.c_double), ("chi_init", C.c_double),
        ("force", C.c_double * 2), ("omega_b", C.c_double),
        ("d_wr", C.c_double), ("d_wv", C.c_double), ("u_wall", C.c_double * 4),
        ("sponge_width", C.c_double), ("sponge_strength", C.c_double),
        ("ramp_steps", C.c_double), ("ramp_start", C.c_double),
        ("sa_mu_cap", C.c_double),
        ("alpha_deg", C.c_double), ("alpha_pivot", C.c_double * 2),
    ]


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        dp = C.POINTER(C.c_double)
        L.lbro_error.restype = C.c_char_p
        L.lbro_create.argtypes = [C.POINTER(Config), i32, C.POINTER(C.c_int32), dp, C.POINTER(p)]
        L.lbro_create_with_links.argtypes = [C.POINTER(Config), i32, C.POINTER(C.c_int32), dp, C.c_char_p,
                                             C.POINTER(p)]
        L.lbro_destroy.argtypes = [p]
        L.lbro_destroy.restype = None
        L.lbro_level_info.argtypes = [p, i32, C.POINTER(C.c_int64)]
        L.lbro_init.argtypes = [p, i32, dp, dp, dp, dp]
        L.lbro_advance.argtypes = [p, i64]
        L.lbro_get_field.argtypes = [p, i32, i32, dp]
        L.lbro_wall_count.argtypes = [p, i32]
        L.lbro_get_wall.argtypes = [p, i32, dp]
        L.lbro_forces.argtypes = [p, i32, dp]
        L.lbro_surface.argtypes = [p, i32, dp, dp]
        L.lbro_lups_per_coarse_step.argtypes = [p]
        L.lbro_lups_per_coarse_step.restype = i64
        L.lbro_threads.restype = C.c_int
        for name in ("lbro_uplus", "lbro_duplus"):
            getattr(L, name).argtypes = [d]
            getattr(L, name).restype = d
        L.lbro_solve_utau.argtypes = [d, d, d, d]
        L.lbro_solve_utau.restype = d
        L.lbro_slip.argtypes = [d, d, d]
        L.lbro_slip.restype = d
        L.lbro_feq.argtypes = [d, d, d, dp]
        L.lbro_feq.restype = None
        L.lbro_central_moments.argtypes = [dp, d, d, dp]
        L.lbro_central_moments.restype = None
        L.lbro_collide.argtypes = [dp, d, d, dp, dp]
        L.lbro_collide.restype = None
        L.lbro_sa_source.argtypes = [d, d, d, d, dp]
        L.lbro_sa_source.restype = None
        L.lbro_sa_cell.argtypes = [dp, dp, dp, d, d, i32, d]
        L.lbro_sa_cell.restype = d
        L.lbro_lsq_point.argtypes = [i32, dp, dp, dp, d, d]
        L.lbro_lsq_point.restype = d
        L.lbro_idw_point.argtypes = [i32, dp, dp, dp, d, d]
        L.lbro_idw_point.restype = d
        L.lbro_sponge_cell.argtypes = [dp, d, d, d, d, dp]
        L.lbro_sponge_cell.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a


# ---------------------------------------------------------------- pure pins
def uplus(y):
    return lib().lbro_uplus(float(y))


def duplus(y):
    return lib().lbro_duplus(float(y))


def solve_utau(ut, dist, nu, guess=0.0):
    return lib().lbro_solve_utau(float(ut), float(dist), float(nu), float(guess))


def slip(utau, dwv, nu):
    return lib().lbro_slip(float(utau), float(dwv), float(nu))


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().lbro_feq(rho, ux, uy, _dp(out))
    return out


def sponge_cell(f, sigma, rho, ux, uy):
    f = _arr(f)
    out = np.zeros(9)
    lib().lbro_sponge_cell(_dp(f), sigma, rho, ux, uy, _dp(out))
    return out


def central_moments(f, ux, uy):
    f = _arr(f)
    out = np.zeros(9)
    lib().lbro_central_moments(_dp(f), ux, uy, _dp(out))
    return out


def collide(f, nu_eff, omega_b=1.0, force=(0.0, 0.0)):
    f = _arr(f)
    F = _arr(force)
    out = np.zeros(9)
    lib().lbro_collide(_dp(f), nu_eff, omega_b, _dp(F), _dp(out))
    return out


def sa_source(nut, nu, omega, dist):
    out = np.zeros(7)
    lib().lbro_sa_source(nut, nu, omega, dist, _dp(out))
    return dict(P=out[0], D=out[1], mu=out[2], nu_t=out[3], S_tilde=out[4], r=out[5], f_w=out[6])


def sa_cell(nt, ux, uy, nu, dist, mode=1, mu_cap=0.0):
    nt, ux, uy = _arr(nt).ravel(), _arr(ux).ravel(), _arr(uy).ravel()
    return lib().lbro_sa_cell(_dp(nt), _dp(ux), _dp(uy), nu, dist, mode, float(mu_cap))


def lsq_point(px, py, v, x, y):
    px, py, v = _arr(px), _arr(py), _arr(v)
    return lib().lbro_lsq_point(len(v), _dp(px), _dp(py), _dp(v), x, y)


def idw_point(px, py, v, x, y):
    px, py, v = _arr(px), _arr(py), _arr(v)
    return lib().lbro_idw_point(len(v), _dp(px), _dp(py), _dp(v), x, y)


def threads():
    return lib().lbro_threads()


# ---------------------------------------------------------------- simulation
def make_config(case) -> Config:
    c = Config()
    c.nx0, c.ny0, c.n_levels = case["nx0"], case["ny0"], case["n_levels"]
    for k in range(4):
        c.bc[k] = case["bc"][k]
    c.wall_model, c.bb_mode, c.sa_mode = case["wall_model"], case["bb_mode"], case["sa_mode"]
    c.body_mode = case.get("body_mode", 0)
    c.outlet = case.get("outlet", 0)
    c.origin[0], c.origin[1] = case["origin"]
    c.dx0 = case["dx0"]
    for l, b in enumerate(case.get("bands", ())):
        c.band[l] = b
    c.wall_y[0], c.wall_y[1] = case.get("wall_y", (0.0, 0.0))
    c.mach, c.reynolds, c.ref_length = case["mach"], case["reynolds"], case["ref_length"]
    c.u_ref, c.nu0 = case["u_ref"], case["nu0"]
    c.rho_ref = case.get("rho_ref", 1.0)
    c.chi_inlet, c.chi_init = case["chi_inlet"], case["chi_init"]
    c.force[0], c.force[1] = case["force"]
    c.omega_b, c.d_wr, c.d_wv = case["omega_b"], case["d_wr"], case["d_wv"]
    uw = case.get("u_wall", (0.0, 0.0, 0.0, 0.0))
    for k in range(4):
        c.u_wall[k] = uw[k]
    c.sponge_width = case.get("sponge_width", 0.0)
    c.sponge_strength = case.get("sponge_strength", 0.0)
    c.ramp_steps = case.get("ramp_steps", 0.0)
    c.ramp_start = case.get("ramp_start", 0.0)
    c.sa_mu_cap = case.get("sa_mu_cap", 0.0)
    # angle of attack turned by the oracle itself (the recipes' bodies come at
    # their incidence; their "alpha_deg" entry only records it)
    c.alpha_deg = case.get("config_alpha_deg", 0.0)
    c.alpha_pivot[0], c.alpha_pivot[1] = case.get("config_alpha_pivot", (0.0, 0.0))
    return c


class Sim:
    """One oracle simulation built from a case dictionary (see lbr_inputs);
    cut_links: path of a precomputed cut-link file whose levels replace the
    polyline intersections (None: all generated)."""

    def __init__(self, case, cut_links=None):
        L = lib()
        self.case = case
        self.cfg = make_config(case)
        bodies = case.get("bodies", [])
        npts = (C.c_int32 * max(1, len(bodies)))(*[len(b) for b in bodies])
        xy = np.ascontiguousarray(np.concatenate(bodies, axis=0) if bodies else np.zeros((1, 2)))
        self._xy = xy
        h = C.c_void_p()
        path = None if cut_links is None else os.fsencode(cut_links)
        if L.lbro_create_with_links(C.byref(self.cfg), len(bodies), npts, _dp(xy), path, C.byref(h)) != 0:
            raise RuntimeError("oracle: " + L.lbro_error().decode())
        self.h = h
        self.n_levels = case["n_levels"]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.lbro_destroy(self.h)
            self.h = None

    def level_info(self, level):
        info = (C.c_int64 * 8)()
        if lib().lbro_level_info(self.h, level, info) != 0:
            raise RuntimeError(lib().lbro_error().decode())
        keys = ("gx0", "gy0", "nx", "ny", "n_fluid", "n_bnodes", "n_cut", "n_ghost")
        return dict(zip(keys, [int(v) for v in info]))

    def init(self, level, rho=None, ux=None, uy=None, chi=None):
        keep = []

        def ptr(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            return _dp(a)
        if lib().lbro_init(self.h, level, ptr(rho), ptr(ux), ptr(uy), ptr(chi)) != 0:
            raise RuntimeError(lib().lbro_error().decode())

    def advance(self, n):
        if lib().lbro_advance(self.h, int(n)) != 0:
            raise RuntimeError("oracle: " + lib().lbro_error().decode())

    def field(self, level, which):
        inf = self.level_info(level)
        out = np.empty((inf["ny"], inf["nx"]))
        if lib().lbro_get_field(self.h, level, which, _dp(out)) != 0:
            raise RuntimeError(lib().lbro_error().decode())
        return out

    def wall(self, level):
        n = lib().lbro_wall_count(self.h, level)
        out = np.empty((max(n, 1), WALL_STRIDE))
        if n > 0 and lib().lbro_get_wall(self.h, level, _dp(out)) != 0:
            raise RuntimeError(lib().lbro_error().decode())
        return out[:n]

    def forces(self, body=-1):
        out = np.zeros(5)
        if lib().lbro_forces(self.h, body, _dp(out)) != 0:
            raise RuntimeError(lib().lbro_error().decode())
        return out

    def surface(self, body=0):
        n = len(self.case["bodies"][body])
        cp, cf = np.zeros(n), np.zeros(n)
        if lib().lbro_surface(self.h, body, _dp(cp), _dp(cf)) != 0:
            raise RuntimeError(lib().lbro_error().decode())
        return cp, cf

    def lups_per_coarse_step(self):
        return int(lib().lbro_lups_per_coarse_step(self.h))
