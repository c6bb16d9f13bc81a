"""lbr_rake_noalloc, the allocation-free variant of lbr_rake, against lbr_rake
through the C-ABI (needs an MI355X)."""
import ctypes as C

import numpy as np
import pytest

import lbr_inputs as LI
from tests import parity_util as U

pytestmark = pytest.mark.gpu


def _noalloc(P, g, p0, p1, n, out):
    return P.lib().lbr_rake_noalloc(g.h, float(p0[0]), float(p0[1]), float(p1[0]), float(p1[1]), int(n),
                                    out.ctypes.data_as(C.POINTER(C.c_double)))


def test_rake_noalloc_matches_rake_and_allocates_nothing():
    """Two calls in a row, the second with fewer points and a changed state in
    between, each bit-identical to lbr_rake on the same state; the library asks
    its allocator for nothing during them; more points than the static scratch
    holds are refused before anything is written."""
    import paper_2601_18443_amd as P
    case = LI.case_airfoil_small()
    g = U.gpu_solver(case, "f32")
    g.advance(3)
    for p0, p1, n in (((-1.0, 0.31), (2.0, -0.27), P.RAKE_NOALLOC_MAX), ((0.2, -0.3), (0.3, 0.5), 700)):
        g.synchronize()
        expect = g.rake(p0, p1, n)
        before = g.alloc.n_alloc
        got = np.full((n, 5), -7.0)
        assert _noalloc(P, g, p0, p1, n, got) == 0
        assert g.alloc.n_alloc == before
        assert np.array_equal(np.isnan(got), np.isnan(expect))
        m = ~np.isnan(expect)
        assert np.array_equal(got[m], expect[m])
        assert len(set(got[:, 0].astype(int)) - {-1}) >= 2          # the rake crosses levels
        g.advance(1)
    big = np.full((P.RAKE_NOALLOC_MAX + 1, 5), -7.0)
    assert _noalloc(P, g, (-1.0, 0.0), (2.0, 0.0), P.RAKE_NOALLOC_MAX + 1, big) == -1
    assert np.all(big == -7.0)
    assert "at most" in P.lib().lbr_last_error(g.h).decode()
