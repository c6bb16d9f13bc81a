"""Python binding of liblbr, the MI355X LBM-RANS library (include/lbr.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (through the allocator callbacks of the
config) and the stream.  The first call into the library (``lib()``,
``Solver``, ``Batch``, ``schedule``) loads liblbr.so and raises if it has not
been built (``python -m paper_2601_18443_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbr.so")

ABI_VERSION = 6
MAX_LEVELS = 12
WALL_STRIDE = 28
CUT_STRIDE = 16
RAKE_NOALLOC_MAX = 16384

STORE_F64, STORE_F32, STORE_F16, STORE_BF16, STORE_MIXED = 0, 1, 2, 3, 4
STORAGE = {"f64": STORE_F64, "f32": STORE_F32, "f16": STORE_F16, "bf16": STORE_BF16, "mixed": STORE_MIXED}
# the 16-bit formats with the free-stream storage shift (lbr_config.shift16 = 1)
SHIFTED = {"f16s": "f16", "bf16s": "bf16", "mixeds": "mixed"}
FIELD_RHO, FIELD_UX, FIELD_UY, FIELD_CHI, FIELD_NUT, FIELD_TYPE, FIELD_DIST = range(7)
ERR_INVALID_ARG, ERR_GEOMETRY, ERR_STATE, ERR_IO = -1, -4, -6, -7
ERR_DIVERGED, ERR_NEWTON, ERR_NOT_CONVERGED = -5, -8, -9
CELL_INACTIVE, CELL_FLUID, CELL_SOLID, CELL_GHOST, CELL_COVERED = range(5)   # values of FIELD_TYPE

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class lbr_config(C.Structure):
    _fields_ = [
        ("version", C.c_int32), ("storage", C.c_int32), ("nx0", C.c_int32), ("ny0", C.c_int32),
        ("n_levels", C.c_int32), ("bc", C.c_int32 * 4), ("wall_model", C.c_int32),
        ("bb", C.c_int32), ("sa", C.c_int32), ("body_mode", C.c_int32), ("outlet", C.c_int32),
        ("origin", C.c_double * 2), ("dx0", C.c_double), ("band", C.c_double * MAX_LEVELS),
        ("wall_y", C.c_double * 2), ("mach", C.c_double), ("reynolds", C.c_double),
        ("ref_length", C.c_double), ("u_ref", C.c_double), ("nu0", C.c_double),
        ("rho_ref", C.c_double), ("chi_inlet", C.c_double), ("chi_init", C.c_double),
        ("force", C.c_double * 2), ("omega_b", C.c_double), ("d_wr", C.c_double),
        ("d_wv", C.c_double), ("u_wall", C.c_double * 4),
        ("sponge_width", C.c_double), ("sponge_strength", C.c_double),
        ("ramp_steps", C.c_double), ("ramp_start", C.c_double), ("shift16", C.c_int32),
        ("health_every", C.c_int32), ("sa_mu_cap", C.c_double),
        ("alpha_deg", C.c_double), ("alpha_pivot", C.c_double * 2),
        ("alloc_fn", ALLOC_FN), ("free_fn", FREE_FN), ("alloc_user", C.c_void_p),
        ("stream", C.c_void_p),
    ]


class lbr_level_desc(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("gx0", "gy0", "nx", "ny", "n_fluid", "n_wall_nodes",
                                         "n_cut_links", "n_ghost", "n_tiles", "bytes")]


_lib = None


def lib():
    """The loaded liblbr.so; raises when the HIP library is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbr.so is not built: run `python -m paper_2601_18443_amd.build`")
        # PyTorch first: its HIP runtime is then the one liblbr binds to, so the
        # device memory and streams PyTorch hands over belong to the same
        # runtime (loading liblbr first would bring a second HIP runtime into
        # the process, and PyTorch's would then fail to find the GPU)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        p, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.lbr_create.argtypes = [C.POINTER(lbr_config), C.POINTER(p)]
        L.lbr_set_geometry.argtypes = [p, i32, C.POINTER(C.c_int32), dp]
        L.lbr_set_cut_links.argtypes = [p, i32, i64, dp]
        L.lbr_load_cut_links.argtypes = [p, C.c_char_p]
        L.lbr_build.argtypes = [p]
        L.lbr_level_info.argtypes = [p, i32, C.POINTER(lbr_level_desc)]
        L.lbr_init_fields.argtypes = [p, i32, dp, dp, dp, dp]
        L.lbr_advance.argtypes = [p, i64]
        L.lbr_synchronize.argtypes = [p]
        L.lbr_read_field.argtypes = [p, i32, i32, dp]
        L.lbr_wall_count.argtypes = [p, i32]
        L.lbr_read_wall.argtypes = [p, i32, dp]
        L.lbr_surface.argtypes = [p, i32, dp, dp]
        L.lbr_surface_yplus.argtypes = [p, i32, dp]
        L.lbr_forces.argtypes = [p, i32, dp]
        L.lbr_residual.argtypes = [p, dp]
        L.lbr_run_to_steady.argtypes = [p, C.c_double, i64, i64, C.POINTER(C.c_int64), dp]
        L.lbr_lups_per_coarse_step.argtypes = [p]
        L.lbr_lups_per_coarse_step.restype = i64
        L.lbr_use_graph.argtypes = [p, i32]
        L.lbr_profile.argtypes = [p, i32, dp]
        L.lbr_last_error.argtypes = [p]
        L.lbr_last_error.restype = C.c_char_p
        L.lbr_destroy.argtypes = [p]
        L.lbr_destroy.restype = None
        L.lbr_read_field_device.argtypes = [p, i32, i32, C.c_void_p, i64]
        L.lbr_wall_yplus.argtypes = [p, i32, dp]
        L.lbr_rake.argtypes = [p, C.c_double, C.c_double, C.c_double, C.c_double, i32, dp]
        L.lbr_rake_noalloc.argtypes = [p, C.c_double, C.c_double, C.c_double, C.c_double, i32, dp]
        L.lbr_schedule.argtypes = [i32, i32, C.POINTER(C.c_int32), i32]
        L.lbr_schedule.restype = i32
        L.lbr_tune.argtypes = [p, i32, C.POINTER(C.c_int32)]
        L.lbr_set_tile_rows.argtypes = [p, i32, i32]
        L.lbr_batch_tune.argtypes = [p, i32, C.POINTER(C.c_int32)]
        L.lbr_save.argtypes = [p, C.c_char_p]
        L.lbr_load.argtypes = [p, C.c_char_p]
        L.lbr_batch_create.argtypes = [i32, C.POINTER(p), C.POINTER(p)]
        L.lbr_batch_advance.argtypes = [p, i64]
        L.lbr_batch_use_graph.argtypes = [p, i32]
        L.lbr_batch_use_persistent.argtypes = [p, i32]
        L.lbr_batch_run_to_steady.argtypes = [p, C.c_double, i64, i64, C.POINTER(i64),
                                              C.POINTER(C.c_double)]
        L.lbr_batch_profile.argtypes = [p, i32, C.POINTER(C.c_double)]
        L.lbr_batch_synchronize.argtypes = [p]
        L.lbr_batch_steps_per_super_step.argtypes = [p, i32]
        L.lbr_batch_steps_per_super_step.restype = i64
        L.lbr_batch_lups_per_super_step.argtypes = [p]
        L.lbr_batch_lups_per_super_step.restype = i64
        L.lbr_batch_last_error.argtypes = [p]
        L.lbr_batch_last_error.restype = C.c_char_p
        L.lbr_batch_destroy.argtypes = [p]
        L.lbr_batch_destroy.restype = None
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


class LbrError(RuntimeError):
    pass


class _TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator.

    Blocks are taken on the library's own stream, the one every kernel of the
    context runs on: the caching allocator then hands a block freed by the
    library (a readout scratch, say) only to later work on that same stream, so
    its reuse is ordered after the kernels that still read it."""

    def __init__(self, device, stream=None, torch_module=None):
        if torch_module is None:
            import torch as torch_module
        self.torch = torch_module
        self.device = device
        self.stream = stream
        self.live = {}
        self.n_alloc = 0                # allocations requested by the library so far
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        self.n_alloc += 1
        try:
            if self.stream is not None:
                with self.torch.cuda.stream(self.stream):
                    t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
            else:
                t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


def make_config(case, storage="f32", stream=None, allocator=None) -> lbr_config:
    c = lbr_config()
    c.version = ABI_VERSION
    shift = isinstance(storage, str) and storage in SHIFTED
    if shift:
        storage = SHIFTED[storage]
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.nx0, c.ny0, c.n_levels = case["nx0"], case["ny0"], case["n_levels"]
    for k in range(4):
        c.bc[k] = case["bc"][k]
    c.wall_model, c.bb, c.sa = case["wall_model"], case["bb_mode"], case["sa_mode"]
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
    for k, v in enumerate(case.get("u_wall", (0.0, 0.0, 0.0, 0.0))):
        c.u_wall[k] = v
    c.sponge_width = case.get("sponge_width", 0.0)
    c.sponge_strength = case.get("sponge_strength", 0.0)
    c.ramp_steps = case.get("ramp_steps", 0.0)
    c.ramp_start = case.get("ramp_start", 0.0)
    c.shift16 = 1 if shift else int(case.get("shift16", 0))
    c.sa_mu_cap = float(case.get("sa_mu_cap", 0.0))
    c.health_every = int(case.get("health_every", 0))
    # angle of attack applied by the library (the recipes' bodies come at their
    # incidence already; their "alpha_deg" entry only records it)
    c.alpha_deg = float(case.get("config_alpha_deg", 0.0))
    c.alpha_pivot[0], c.alpha_pivot[1] = case.get("config_alpha_pivot", (0.0, 0.0))
    if allocator is not None:
        c.alloc_fn, c.free_fn = allocator.alloc_cb, allocator.free_cb
    c.stream = stream
    return c


class Solver:
    """One liblbr context: lbr_create + lbr_set_geometry (+ lbr_load_cut_links or
    lbr_set_cut_links) + lbr_build from a case dict.  cut_links: None (cut links
    from the polylines), the path of a cut-link file, or {level: (n, CUT_STRIDE)
    array} of precomputed records."""

    def __init__(self, case, storage="f32", device="cuda:0", use_torch_memory=True, cut_links=None):
        import torch
        L = lib()
        if not torch.cuda.is_available():
            raise LbrError("liblbr needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        # a stream of its own (default priority): the legacy default stream cannot be captured
        self.torch_stream = torch.cuda.Stream(self.device)
        self.alloc = _TorchAllocator(self.device, self.torch_stream) if use_torch_memory else None
        self.case = case
        self._batches = weakref.WeakSet()      # batches that borrow this context
        self.cfg = make_config(case, storage, C.c_void_p(self.torch_stream.cuda_stream), self.alloc)
        h = C.c_void_p()
        rc = L.lbr_create(C.byref(self.cfg), C.byref(h))
        if rc != 0:
            raise LbrError(f"lbr_create failed ({rc})")
        self.h = h
        bodies = case.get("bodies", [])
        npts = (C.c_int32 * max(1, len(bodies)))(*[len(b) for b in bodies])
        xy = np.ascontiguousarray(np.concatenate(bodies, 0) if bodies else np.zeros((1, 2)))
        self._check(L.lbr_set_geometry(self.h, len(bodies), npts, _dp(xy)))
        if isinstance(cut_links, (str, os.PathLike)):
            self._check(L.lbr_load_cut_links(self.h, os.fsencode(cut_links)))
        elif cut_links is not None:
            for level, rec in cut_links.items():
                rec = np.ascontiguousarray(rec, dtype=np.float64).reshape(-1, CUT_STRIDE)
                self._check(L.lbr_set_cut_links(self.h, int(level), rec.shape[0], _dp(rec)))
        self._check(L.lbr_build(self.h))
        self.n_levels = case["n_levels"]

    def _check(self, rc):
        if rc != 0:
            raise LbrError(f"liblbr error {rc}: {lib().lbr_last_error(self.h).decode()}")
        return rc

    def close(self):
        """Destroys the context; a batch that borrows it is closed first (its
        launch tables point into this context's memory)."""
        for b in list(getattr(self, "_batches", ())):
            b.close()
        if getattr(self, "h", None):
            lib().lbr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        d = lbr_level_desc()
        self._check(lib().lbr_level_info(self.h, level, C.byref(d)))
        return {k: int(getattr(d, k)) for k, _ in lbr_level_desc._fields_}

    def init(self, level, rho=None, ux=None, uy=None, chi=None):
        """Equilibrium initialisation of one level from (ny, nx) arrays over its I/O box."""
        inf = self.level_info(level)
        shape = (inf["ny"], inf["nx"])
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                for a in (rho, ux, uy, chi)]
        for name, a in zip(("rho", "ux", "uy", "chi"), arrs):
            if a is not None and a.shape != shape:
                raise ValueError(f"{name} has shape {a.shape}; level {level} needs {shape}")
        self._check(lib().lbr_init_fields(self.h, level, *[_dp(a) for a in arrs]))

    def advance(self, n):
        self._check(lib().lbr_advance(self.h, int(n)))

    def synchronize(self):
        self._check(lib().lbr_synchronize(self.h))

    def field(self, level, which):
        inf = self.level_info(level)
        out = np.empty((inf["ny"], inf["nx"]))
        self._check(lib().lbr_read_field(self.h, level, which, _dp(out)))
        return out

    def field_device(self, level, which, torch_module=None):
        """One field of a level as a float64 device tensor (ny, nx), written by the
        library on its stream.  The tensor comes from torch's current stream, whose
        earlier work may still use that block: the library stream waits for the
        current stream before the write, and the current stream waits for the
        library stream after it."""
        torch = torch_module
        if torch is None:
            import torch
        inf = self.level_info(level)
        cur = torch.cuda.current_stream(self.device)
        out = torch.empty((inf["ny"], inf["nx"]), dtype=torch.float64, device=self.device)
        self.torch_stream.wait_stream(cur)
        self._check(lib().lbr_read_field_device(self.h, level, which, C.c_void_p(out.data_ptr()), out.numel()))
        cur.wait_stream(self.torch_stream)
        return out

    def wall(self, level):
        n = lib().lbr_wall_count(self.h, level)
        if n < 0:
            self._check(n)
        out = np.empty((max(n, 1), WALL_STRIDE))
        if n > 0:
            self._check(lib().lbr_read_wall(self.h, level, _dp(out)))
        return out[:n]

    def forces(self, body=-1):
        out = np.zeros(5)
        self._check(lib().lbr_forces(self.h, body, _dp(out)))
        return out

    def surface(self, body=0):
        n = len(self.case["bodies"][body])
        cp, cf = np.zeros(n), np.zeros(n)
        self._check(lib().lbr_surface(self.h, body, _dp(cp), _dp(cf)))
        return cp, cf

    def surface_yplus(self, body=0):
        """y+ of the virtual node at the segment centroids of one body."""
        yv = np.zeros(len(self.case["bodies"][body]))
        self._check(lib().lbr_surface_yplus(self.h, body, _dp(yv)))
        return yv

    def residual(self):
        r = C.c_double()
        self._check(lib().lbr_residual(self.h, C.byref(r)))
        return r.value

    def run_to_steady(self, tol, max_steps, check_every=100):
        """(steps taken, last residual); converged tells whether the residual went
        below tol within max_steps (LBR_ERR_NOT_CONVERGED otherwise, not raised)."""
        done, r = C.c_int64(), C.c_double()
        rc = lib().lbr_run_to_steady(self.h, tol, max_steps, check_every, C.byref(done), C.byref(r))
        self.converged = rc == 0
        if rc != ERR_NOT_CONVERGED:
            self._check(rc)
        return done.value, r.value

    def wall_yplus(self, level):
        """(n_wall_nodes, 3) array: y+ of R, B and V of each wall node of the level."""
        n = lib().lbr_wall_count(self.h, level)
        if n < 0:
            self._check(n)
        out = np.zeros((max(n, 1), 3))
        if n > 0:
            self._check(lib().lbr_wall_yplus(self.h, level, _dp(out)))
        return out[:n]

    def rake(self, p0, p1, n, noalloc=False):
        """(n, 5) array along the segment p0 -> p1: level, u_x/U, u_y/U, nu_t/nu, rho.
        noalloc: through lbr_rake_noalloc (no device allocation, n <= RAKE_NOALLOC_MAX)."""
        out = np.zeros((int(n), 5))
        fn = lib().lbr_rake_noalloc if noalloc else lib().lbr_rake
        self._check(fn(self.h, float(p0[0]), float(p0[1]), float(p1[0]), float(p1[1]), int(n), _dp(out)))
        return out

    def tune(self, trials=5):
        """Times the tile heights on every level and keeps the fastest; returns them."""
        rows = (C.c_int32 * self.case["n_levels"])()
        self._check(lib().lbr_tune(self.h, int(trials), rows))
        return [int(r) for r in rows]

    def set_tile_rows(self, rows, level=-1):
        self._check(lib().lbr_set_tile_rows(self.h, int(level), int(rows)))

    def save(self, path):
        self._check(lib().lbr_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._check(lib().lbr_load(self.h, os.fsencode(path)))

    def lups_per_coarse_step(self):
        return int(lib().lbr_lups_per_coarse_step(self.h))

    def use_graph(self, enable=True):
        self._check(lib().lbr_use_graph(self.h, 1 if enable else 0))

    def profile(self, enable=None):
        out = np.zeros(4)
        cur = 1 if enable else 0
        self._check(lib().lbr_profile(self.h, cur, _dp(out)))
        return out


def schedule(n_levels, merge=True):
    """Launches of two coarse steps of an n_levels grid, each a list of
    (level, sub-step) pairs (the merged schedule, or the direct cycle)."""
    L = lib()
    need = L.lbr_schedule(int(n_levels), 1 if merge else 0, None, 0)
    if need < 0:
        raise LbrError(f"lbr_schedule failed ({need})")
    buf = (C.c_int32 * need)()
    L.lbr_schedule(int(n_levels), 1 if merge else 0, buf, need)
    out, k = [], 0
    while k < need:
        m = buf[k]
        out.append([(buf[k + 1 + 2 * j], buf[k + 2 + 2 * j]) for j in range(m)])
        k += 1 + 2 * m
    return out


class Batch:
    """lbr_batch over several Solver objects of the same storage precision.

    Super steps run on the first solver's stream; reads through any solver are
    ordered after them.  A solver may be advanced on its own between batch
    calls by an even number of coarse steps.  Closing one of the solvers
    closes the batch first.
    """

    def __init__(self, solvers):
        L = lib()
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = C.c_void_p()
        rc = L.lbr_batch_create(len(self.solvers), arr, C.byref(h))
        self.h = h if h.value else None
        if rc != 0:
            msg = L.lbr_batch_last_error(self.h).decode() if self.h else ""
            self.close()
            raise LbrError(f"lbr_batch_create failed ({rc}) {msg}")
        for s in self.solvers:
            s._batches.add(self)

    def _check(self, rc):
        if rc != 0:
            raise LbrError(f"liblbr batch error {rc}: {lib().lbr_batch_last_error(self.h).decode()}")

    def advance(self, n_super_steps):
        self._check(lib().lbr_batch_advance(self.h, int(n_super_steps)))

    def use_graph(self, enable=True):
        self._check(lib().lbr_batch_use_graph(self.h, 1 if enable else 0))

    def use_persistent(self, enable=True):
        """Each table of the merged schedule as one cooperative grid (lbr_batch_use_persistent)."""
        self._check(lib().lbr_batch_use_persistent(self.h, 1 if enable else 0))

    def run_to_steady(self, tol, max_super_steps, check_every=100):
        """Returns (coarse steps taken per case, last residual per case)."""
        n = len(self.solvers)
        steps, res = (C.c_int64 * n)(), (C.c_double * n)()
        rc = lib().lbr_batch_run_to_steady(self.h, float(tol), int(max_super_steps), int(check_every), steps, res)
        self.converged = rc == 0
        if rc != ERR_NOT_CONVERGED:
            self._check(rc)
        return [int(v) for v in steps], [float(v) for v in res]

    def profile(self, enable=True):
        out = (C.c_double * 4)()
        self._check(lib().lbr_batch_profile(self.h, 1 if enable else 0, out))
        return [float(v) for v in out]

    def tune(self, trials=5):
        """Tile height per virtual level, timed on the batched launches; returns them."""
        n = max(s.case["n_levels"] for s in self.solvers)
        rows = (C.c_int32 * n)()
        self._check(lib().lbr_batch_tune(self.h, int(trials), rows))
        return [int(r) for r in rows]

    def synchronize(self):
        self._check(lib().lbr_batch_synchronize(self.h))

    def steps_per_super_step(self, k):
        return int(lib().lbr_batch_steps_per_super_step(self.h, k))

    def lups_per_super_step(self):
        return int(lib().lbr_batch_lups_per_super_step(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().lbr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
