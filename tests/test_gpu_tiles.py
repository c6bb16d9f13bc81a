"""Tile shapes of the step kernel and their tuner (needs an MI355X).

Every cell's update is a function of its stencil alone, so the fields must be
bit-identical whatever tile height (2, 4, 8 or 16 rows of 64 cells) each level
uses: under the direct cycle, the merged schedule replayed from a graph, and in
a batch; tuning only chooses among them and must not change any result.
"""
import numpy as np
import pytest

import lbr_inputs as LI

pytestmark = pytest.mark.gpu


def _deep_case():
    return LI.case_airfoil(seed=3, finest_cells_per_chord=256, n_levels=6, domain_chords=8.0,
                           band_finest=0.0625, n_side=256)


def _fields(s, n_levels):
    return [s.field(l, f) for l in range(n_levels) for f in (0, 1, 2, 3)] + [s.forces()]


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_fields_are_bit_identical_for_every_tile_height(storage):
    import paper_2601_18443_amd as P
    case = _deep_case()
    L = case["n_levels"]
    ref = None
    for rows in (4, 2, 8, 16):
        for graph in (False, True):
            s = P.Solver(case, storage=storage)
            s.set_tile_rows(rows)
            s.use_graph(graph)
            s.advance(5)
            s.advance(6)
            got = _fields(s, L)
            if ref is None:
                ref = got
            assert _same(got, ref), (rows, graph)
    # mixed heights across levels
    s = P.Solver(case, storage=storage)
    for lvl, rows in enumerate((8, 2, 16, 4, 2, 16)):
        s.set_tile_rows(rows, lvl)
    s.use_graph(True)
    s.advance(11)
    assert _same(_fields(s, L), ref)


def test_tuner_picks_valid_heights_and_changes_nothing():
    import paper_2601_18443_amd as P
    case = _deep_case()
    L = case["n_levels"]
    a, b = P.Solver(case, storage="f32"), P.Solver(case, storage="f32")
    a.advance(3)
    b.advance(3)
    rows = a.tune(trials=3)
    assert len(rows) == L and all(r in (2, 4, 8, 16) for r in rows)
    for s in (a, b):
        s.use_graph(True)
        s.advance(8)
    assert _same(_fields(a, L), _fields(b, L))
    # the wall model's state is untouched by the trials
    for lvl in range(L):
        assert np.array_equal(a.wall(lvl), b.wall(lvl), equal_nan=True)


def test_batch_tuner_keeps_batched_results_identical():
    import paper_2601_18443_amd as P
    cases = [_deep_case(), LI.case_airfoil_small()]
    batched = [P.Solver(c, storage="f32") for c in cases]
    alone = [P.Solver(c, storage="f32") for c in cases]
    batch = P.Batch(batched)
    try:
        rows = batch.tune(trials=3)
        assert len(rows) == 6 and all(r in (2, 4, 8, 16) for r in rows)
        batch.use_graph(True)
        batch.advance(4)
        batch.synchronize()
        for s, p in zip(alone, (1, 8)):
            s.advance(4 * p)
        for k, c in enumerate(cases):
            assert _same(_fields(batched[k], c["n_levels"]), _fields(alone[k], c["n_levels"])), k
    finally:
        batch.close()


def test_invalid_tile_heights_are_refused():
    import paper_2601_18443_amd as P
    s = P.Solver(LI.case_airfoil_small(), storage="f32")
    for rows, level in ((3, -1), (32, 0), (4, 7)):
        with pytest.raises(P.LbrError):
            s.set_tile_rows(rows, level)
