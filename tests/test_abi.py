"""The C-ABI library loads and exports every entry point declared in include/lbr.h (no GPU needed)."""
import ctypes
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbr.h")
LIB = os.path.join(ROOT, "paper_2601_18443_amd", "liblbr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(lbr_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lbr_create", "lbr_set_geometry", "lbr_build", "lbr_init_fields", "lbr_advance",
                     "lbr_read_field", "lbr_read_wall", "lbr_surface", "lbr_forces", "lbr_residual",
                     "lbr_run_to_steady", "lbr_last_error", "lbr_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_config_validation_without_gpu():
    """lbr_create only validates the config; it never touches the device."""
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    case = LI.case_channel()
    cfg = P.make_config(case, "f64")
    h = ctypes.c_void_p()
    assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    L.lbr_destroy(h)
    bad = P.make_config(case, "f64")
    bad.version = 99
    assert L.lbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = P.make_config(case, "f64")
    bad.bc[0] = LI.BC_WALL
    assert L.lbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = P.make_config(case, "f64")
    bad.bc[0] = LI.BC_INLET          # periodic sides come in pairs
    assert L.lbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    for k, v in ((2, 5), (3, -1)):   # not a boundary kind
        bad = P.make_config(case, "f64")
        bad.bc[k] = v
        assert L.lbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = P.make_config(LI.case_airfoil_small(), "f32")
    bad.band[1] = float("nan")       # refinement bands of the levels in use
    assert L.lbr_create(ctypes.byref(bad), ctypes.byref(h)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
@pytest.mark.parametrize("field,value", [
    ("n_levels", 0), ("n_levels", 13),                       # 1..LBR_MAX_LEVELS
    ("nx0", 3), ("ny0", 2),                                  # at least 4 cells
    ("nx0", 1 << 22), ("ny0", 1 << 22),                      # finest indices past 2^28 (8 levels)
    ("dx0", 0.0), ("dx0", -1.0),
    ("storage", -1), ("storage", 5),
    ("outlet", 3), ("sponge_width", -1.0), ("sponge_strength", 1.5),
    ("ramp_steps", -1.0), ("ramp_start", 1.5), ("shift16", 2),
    ("reynolds", 0.0),                                       # no finite viscosity
    ("wall_model", 4), ("bb", 3), ("sa", -1), ("sa", 3),     # enums
    ("body_mode", 2),
    ("rho_ref", 0.0), ("rho_ref", float("nan")),
    ("omega_b", 0.0), ("omega_b", 2.0),                      # bulk rate in (0, 2)
    ("d_wr", 0.0), ("d_wv", -1.0), ("chi_init", float("inf")),
    ("u_ref", float("nan")), ("sponge_width", float("inf")), ("sa_mu_cap", float("nan")), ("health_every", -1),
    ("alpha_deg", 90.5), ("alpha_deg", float("nan")),        # angle of attack within +-90 degrees
])
def test_create_refuses_out_of_range_config(field, value):
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    case = LI.case_airfoil_small()
    cfg = P.make_config(dict(case, n_levels=8) if field in ("nx0", "ny0") and value > 1000 else case, "f32")
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert not h.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
@pytest.mark.parametrize("side,kind", [
    (0, "OUTLET"), (0, "SYMMETRY"),                          # x-lo: periodic or inlet only
    (1, "INLET"), (1, "SYMMETRY"),                           # x-hi: periodic or outlet only
    (2, "INLET"), (2, "OUTLET"), (3, "INLET"), (3, "OUTLET"),  # y sides: symmetry, wall, periodic
])
def test_create_refuses_side_conditions_the_step_does_not_implement(side, kind):
    """The step applies the inlet rule on x-lo only and the outlet rules on x-hi
    only; any other pairing would leave the populations entering across that side
    undefined, so lbr_create refuses it (host check, no device work)."""
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    cfg = P.make_config(LI.case_airfoil_small(), "f32")
    cfg.bc[side] = getattr(LI, "BC_" + kind)
    h = ctypes.c_void_p()
    assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert not h.value
    ok = P.make_config(LI.case_airfoil_small(), "f32")
    ok.bc[2] = ok.bc[3] = LI.BC_WALL                         # channel walls on the y sides
    assert L.lbr_create(ctypes.byref(ok), ctypes.byref(h)) == 0
    L.lbr_destroy(h)


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16", "mixed", "f16s", "bf16s", "mixeds"])
def test_create_accepts_every_storage(storage):
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    cfg = P.make_config(LI.case_airfoil_small(), storage)
    h = ctypes.c_void_p()
    assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    L.lbr_destroy(h)


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_set_geometry_checks_the_polylines_on_the_host():
    """lbr_set_geometry is host work: it refuses short, non-finite and clockwise
    bodies, accepts the generated counter-clockwise ones, and no device call is
    needed for either answer."""
    import numpy as np
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    case = LI.case_airfoil_small()
    body = np.ascontiguousarray(case["bodies"][0], dtype=np.float64)

    def set_geo(pts):
        cfg = P.make_config(case, "f32")
        h = ctypes.c_void_p()
        assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
        n = (ctypes.c_int32 * 1)(len(pts))
        xy = np.ascontiguousarray(pts, dtype=np.float64)
        rc = L.lbr_set_geometry(h, 1, n, xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        msg = L.lbr_last_error(h).decode()
        L.lbr_destroy(h)
        return rc, msg

    assert set_geo(body) == (0, "")
    rc, msg = set_geo(body[::-1])                     # clockwise
    assert rc == -4 and "counter-clockwise" in msg
    assert set_geo(body[:2])[0] == -4                 # fewer than 3 points
    bad = body.copy()
    bad[5, 1] = np.nan
    assert set_geo(bad)[0] == -4


def _cut_record(**kw):
    """One valid cut-link record (gi, gj, IW, normal, d_WB, body, q1..q8)."""
    import numpy as np
    r = np.array([10, 3, 10.5, 2.9, 0.0, 1.0, 0.6, 0] + [-1.0] * 8)
    r[8 + 3] = 0.6                                  # q4: the link along (0, -1)
    for k, v in kw.items():
        r[int(k[1:])] = v
    return r


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_cut_link_input_checks_its_records_on_the_host(tmp_path):
    """lbr_set_cut_links and lbr_load_cut_links are host work: they range-check
    every record (finite, integral indices and body, a unit normal, d_WB >= 0,
    q in (0, 1] or -1, at least one cut link) and refuse malformed files with
    nothing set, before any device call."""
    import numpy as np
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    case = LI.case_airfoil_small()
    cfg = P.make_config(case, "f32")
    h = ctypes.c_void_p()
    assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    dp = ctypes.POINTER(ctypes.c_double)

    def put(level, rows):
        a = np.ascontiguousarray(np.atleast_2d(rows), dtype=np.float64)
        rc = L.lbr_set_cut_links(h, level, len(a), a.ctypes.data_as(dp))
        return rc, L.lbr_last_error(h).decode()

    try:
        assert put(2, _cut_record())[0] == 0
        assert put(2, np.zeros((0, 16)))[0] == 0                        # withdraws the list
        for bad, word in ((_cut_record(c0=10.5), "gi"), (_cut_record(c7=-3), "body"),
                          (_cut_record(c4=0.5), "normal"), (_cut_record(c6=-0.1), "d_WB"),
                          (_cut_record(c11=0.0), "q4"), (_cut_record(c11=1.25), "q4"),
                          (_cut_record(c11=-0.5), "q4"), (_cut_record(c11=-1.0), "no link"),
                          (_cut_record(c3=np.inf), "not finite")):
            rc, msg = put(2, bad)
            assert rc == -1 and word in msg, (rc, msg)
        assert put(3, _cut_record())[0] == -1                           # 3 levels: 0..2
        assert put(-1, _cut_record())[0] == -1
        assert L.lbr_set_cut_links(h, 2, 1, None) == -1
        # files
        good = tmp_path / "good.cut"
        LI.write_cut_links(good, {2: np.stack([_cut_record(), _cut_record(c0=11)])}, comment="two nodes")
        assert L.lbr_load_cut_links(h, str(good).encode()) == 0
        text = open(good).read()
        for name, body, code, word in (
                ("missing", None, -7, "cannot open"),
                ("header", "lbr-cut-links 2\n", -1, "header"),
                ("keyword", "lbr-cut-links 1\nlevels 2 1\n", -1, "expected"),
                ("level", "lbr-cut-links 1\nlevel 9 0\n", -1, "bad level"),
                ("twice", "lbr-cut-links 1\nlevel 2 0\nlevel 2 0\n", -1, "twice"),
                ("truncated", text[: len(text) - 12], -1, "truncated"),
                ("token", text.replace(" 0.59999999999999998", " 0.6x", 1), -1, "not a number"),
                ("range", text.replace("-1 -1 -1 -1", "-1 -1 -1 7", 1), -1, "q")):
            p = tmp_path / (name + ".cut")
            if body is not None:
                open(p, "w").write(body)
            rc = L.lbr_load_cut_links(h, str(p).encode())
            msg = L.lbr_last_error(h).decode()
            assert rc == code and word in msg, (name, rc, msg)
    finally:
        L.lbr_destroy(h)


C_CLIENT = r"""
#include "lbr.h"
#include <stdio.h>
int main(void) {
    lbr_config cfg = {0};
    lbr_ctx* ctx = NULL;
    cfg.version = LBR_ABI_VERSION;
    if (lbr_create(&cfg, &ctx) != LBR_ERR_INVALID_ARG || ctx) return 1;   /* zero grid */
    cfg.storage = LBR_STORE_F32;
    cfg.nx0 = 64; cfg.ny0 = 32; cfg.n_levels = 1;
    cfg.bc[0] = cfg.bc[1] = LBR_BC_PERIODIC; cfg.bc[2] = cfg.bc[3] = LBR_BC_WALL;
    cfg.wall_model = LBR_WALL_VN; cfg.bb = LBR_BB_AUTO; cfg.sa = LBR_SA_LW;
    cfg.dx0 = 1.0; cfg.wall_y[1] = 32.0; cfg.mach = 0.1; cfg.u_ref = 0.05; cfg.nu0 = 1e-3;
    cfg.rho_ref = 1.0; cfg.chi_inlet = 3.0; cfg.chi_init = 3.0; cfg.omega_b = 1.0;
    cfg.d_wr = 2.0; cfg.d_wv = 1.0;
    if (lbr_create(&cfg, &ctx) != LBR_OK || !ctx) return 2;
    if (lbr_set_geometry(ctx, 0, NULL, NULL) != LBR_OK) return 3;
    if (lbr_advance(ctx, 1) != LBR_ERR_STATE) return 4;      /* not built yet */
    {
        double yv[4];
        if (lbr_surface_yplus(ctx, 0, yv) != LBR_ERR_INVALID_ARG) return 5;   /* not built */
        if (lbr_surface_yplus(NULL, 0, yv) != LBR_ERR_INVALID_ARG) return 6;
        if (lbr_batch_use_persistent(NULL, 1) != LBR_ERR_INVALID_ARG) return 7;
    }
    printf("%s\n", lbr_last_error(ctx));
    lbr_destroy(ctx);
    cfg.alpha_deg = 120.0;                                    /* beyond +-90 degrees */
    if (lbr_create(&cfg, &ctx) != LBR_ERR_INVALID_ARG || ctx) return 8;
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_header_serves_a_plain_c_client(tmp_path):
    """include/lbr.h compiles as strict C99, and a C program linked against
    liblbr.so drives the host-side calls (no device work)."""
    import subprocess
    src = tmp_path / "client.c"
    src.write_text(C_CLIENT)
    exe = tmp_path / "client"
    inc = os.path.join(ROOT, "include")
    libdir = os.path.dirname(LIB)
    subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I" + inc, str(src),
                    "-L" + libdir, "-llbr", "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "lbr_build" in r.stdout


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_binding_binds_liblbr_to_pytorchs_hip_runtime():
    """lib() loads PyTorch before liblbr.so, so the process holds one HIP
    runtime (PyTorch's): the device memory and streams PyTorch hands to the
    library belong to it, and PyTorch still finds the GPU afterwards."""
    import subprocess
    code = ("import paper_2601_18443_amd as P; P.lib(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    libs = eval(r.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
    import torch
    assert os.path.dirname(libs[0]) == os.path.join(os.path.dirname(torch.__file__), "lib")


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbr.so not built")
def test_new_entry_points_refuse_missing_handles_on_the_host():
    """lbr_surface_yplus and lbr_batch_use_persistent check their arguments on
    the host: a null context or batch, or a context that was never built, is
    LBR_ERR_INVALID_ARG with no device call; the turned geometry of a non-zero
    alpha_deg is accepted by lbr_set_geometry (host work only)."""
    import numpy as np
    import paper_2601_18443_amd as P
    import lbr_inputs as LI
    L = P.lib()
    out = np.zeros(8)
    dp = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.lbr_surface_yplus(None, 0, dp) == P.ERR_INVALID_ARG
    assert L.lbr_batch_use_persistent(None, 1) == P.ERR_INVALID_ARG
    case = dict(LI.case_airfoil_small(alpha_deg=0.0), config_alpha_deg=10.0, config_alpha_pivot=(0.25, 0.0))
    cfg = P.make_config(case, "f32")
    h = ctypes.c_void_p()
    assert L.lbr_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    try:
        assert L.lbr_surface_yplus(h, 0, dp) == P.ERR_INVALID_ARG          # not built
        body = np.ascontiguousarray(case["bodies"][0], dtype=np.float64)
        n = (ctypes.c_int32 * 1)(len(body))
        assert L.lbr_set_geometry(h, 1, n, body.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    finally:
        L.lbr_destroy(h)
