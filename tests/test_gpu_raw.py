"""The C-ABI without PyTorch's memory or streams (needs an MI355X): a context
created with no allocator callbacks (device memory from hipMalloc) and the
default stream computes the same fields, bit for bit, as one on PyTorch's
allocator and stream; graph replay is refused on the default stream."""
import ctypes as C

import numpy as np
import pytest

import lbr_inputs as LI
import paper_2601_18443_amd as P
from tests import parity_util as U

pytestmark = pytest.mark.gpu


def _raw(case, storage):
    L = P.lib()
    cfg = P.make_config(case, storage, stream=None, allocator=None)
    h = C.c_void_p()
    assert L.lbr_create(C.byref(cfg), C.byref(h)) == 0
    bodies = case["bodies"]
    npts = (C.c_int32 * len(bodies))(*[len(b) for b in bodies])
    xy = np.ascontiguousarray(np.concatenate(bodies, 0), dtype=np.float64)
    assert L.lbr_set_geometry(h, len(bodies), npts, xy.ctypes.data_as(C.POINTER(C.c_double))) == 0
    assert L.lbr_build(h) == 0, L.lbr_last_error(h).decode()
    return L, h


def test_hipmalloc_and_default_stream_match_the_torch_path():
    case = LI.case_airfoil_small()
    L, h = _raw(case, "f32")
    g = U.gpu_solver(case, "f32")
    try:
        assert L.lbr_use_graph(h, 1) == -1
        assert b"default stream" in L.lbr_last_error(h)
        assert L.lbr_advance(h, 5) == 0
        assert L.lbr_synchronize(h) == 0
        g.advance(5)
        for l in range(case["n_levels"]):
            d = P.lbr_level_desc()
            assert L.lbr_level_info(h, l, C.byref(d)) == 0
            for f in range(4):
                x = np.empty((d.ny, d.nx))
                assert L.lbr_read_field(h, l, f, x.ctypes.data_as(C.POINTER(C.c_double))) == 0
                y = g.field(l, f)
                assert np.array_equal(np.isnan(x), np.isnan(y))
                m = ~np.isnan(x)
                assert np.array_equal(x[m], y[m]), (l, f)
        out = np.zeros(5)
        assert L.lbr_forces(h, -1, out.ctypes.data_as(C.POINTER(C.c_double))) == 0
        assert np.array_equal(out, g.forces())
    finally:
        L.lbr_destroy(h)
        g.close()
