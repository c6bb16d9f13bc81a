"""Batched sweep against cases advanced one by one (needs an MI355X).

A batch advances several cases with shared k_step launches: the launch of
virtual level v covers level v - (lmax - L_k) of every case k, one grid split
into per-case parts.  Each case's cells are computed by the same code from the
same inputs as when it is advanced alone, in the same order, so every field,
the wall state and the forces must agree bit for bit with a twin advanced alone
by steps_per_super_step(k) coarse steps per super step.
"""
import numpy as np
import pytest

import lbr_inputs as LI

pytestmark = pytest.mark.gpu

FIELDS = (0, 1, 2, 3)          # rho, u_x, u_y, chi


def _cases():
    # different level counts (so different steps per super step), angles and bodies
    return [
        LI.case_airfoil(seed=11, finest_cells_per_chord=64, n_levels=2, domain_chords=8.0,
                        band_finest=0.5, alpha_deg=-2.0, n_side=256),
        LI.case_airfoil(seed=12, finest_cells_per_chord=64, n_levels=4, domain_chords=8.0,
                        band_finest=0.25, alpha_deg=6.0, n_side=256),
        LI.case_airfoil(seed=13, finest_cells_per_chord=64, n_levels=3, domain_chords=8.0,
                        band_finest=0.25, alpha_deg=12.0, n_side=256),
    ]


def _assert_same(a, b, n_levels, tag):
    for lvl in range(n_levels):
        for name in FIELDS:
            fa, fb = a.field(lvl, name), b.field(lvl, name)
            assert np.array_equal(fa, fb, equal_nan=True), (tag, lvl, name)
        assert np.array_equal(a.wall(lvl), b.wall(lvl), equal_nan=True), (tag, lvl, "wall")
    assert np.array_equal(a.forces(), b.forces()), tag


@pytest.mark.parametrize("storage", ["f32", "f64", "mixed", "mixeds"])
def test_batched_sweep_matches_cases_advanced_alone(storage):
    import paper_2601_18443_amd as P
    cases = _cases()
    batched = [P.Solver(c, storage=storage) for c in cases]
    alone = [P.Solver(c, storage=storage) for c in cases]
    batch = P.Batch(batched)
    try:
        per = [batch.steps_per_super_step(k) for k in range(len(cases))]
        assert per == [4, 1, 2]
        assert batch.lups_per_super_step() == sum(
            s.lups_per_coarse_step() * p for s, p in zip(alone, per))

        def advance_alone(n_super, graph):
            for s, p in zip(alone, per):
                s.use_graph(graph)
                s.advance(n_super * p)

        # direct launches, an odd count so that the graph below starts mid-pair
        batch.advance(3)
        advance_alone(3, False)
        for k, c in enumerate(cases):
            _assert_same(batched[k], alone[k], c["n_levels"], f"direct case {k}")

        # graph replay of two super steps (one direct step first to realign)
        batch.use_graph(True)
        batch.advance(5)
        advance_alone(5, True)
        for k, c in enumerate(cases):
            _assert_same(batched[k], alone[k], c["n_levels"], f"graph case {k}")

        # a case advanced alone by an even number of steps keeps the batch valid
        batched[1].advance(2)
        alone[1].advance(2)
        batch.advance(2)
        advance_alone(2, True)
        for k, c in enumerate(cases):
            _assert_same(batched[k], alone[k], c["n_levels"], f"interleaved case {k}")

        # ... an odd number does not: the batch refuses instead of computing garbage
        batched[1].advance(1)
        with pytest.raises(P.LbrError):
            batch.advance(1)
    finally:
        batch.close()


def test_batch_refuses_duplicates_and_mixed_storage():
    import paper_2601_18443_amd as P
    c = LI.case_airfoil_small()
    a, b = P.Solver(c, storage="f32"), P.Solver(c, storage="f64")
    with pytest.raises(P.LbrError):
        P.Batch([a, a])
    with pytest.raises(P.LbrError):
        P.Batch([a, b])


def test_closing_a_solver_closes_the_batch_that_borrows_it():
    """The batch's launch tables point into its cases' memory: closing a case
    first closes the batch, which then refuses work instead of launching on
    freed memory; the other case stays usable."""
    import paper_2601_18443_amd as P
    c = LI.case_airfoil_small()
    a, b = P.Solver(c, storage="f32"), P.Solver(c, storage="f32")
    batch = P.Batch([a, b])
    batch.advance(2)
    a.close()
    assert batch.h is None
    with pytest.raises(P.LbrError):
        batch.advance(1)
    b.advance(2)
    assert np.all(np.isfinite(b.forces()))


def test_batch_refuses_cases_inside_the_start_up_ramp():
    import paper_2601_18443_amd as P
    c = dict(LI.case_airfoil_small(), ramp_steps=4, ramp_start=0.5)
    s = P.Solver(c, storage="f32")
    with pytest.raises(P.LbrError):
        P.Batch([s])
    s.advance(4)
    P.Batch([s]).close()


@pytest.mark.parametrize("mode", ["graph", "persistent"])
def test_batch_run_to_steady_drops_converged_cases(mode):
    """A case whose residual falls below the tolerance leaves the launches; the
    others go on.  The threshold is placed between the residuals the cases reach
    at the first check (a deterministic quantity: the same run repeated), so the
    split is known in advance; every case must end bit-identical to a twin
    advanced alone by the coarse steps the batch reports."""
    import paper_2601_18443_amd as P
    cases = _cases()
    check, max_super = 4, 12

    probe = [P.Solver(c, storage="f32") for c in cases]
    bp = P.Batch(probe)
    per = [bp.steps_per_super_step(k) for k in range(len(cases))]
    steps0, res0 = bp.run_to_steady(0.0, check, check)
    bp.close()
    assert steps0 == [check * p for p in per]
    order = sorted(res0)
    assert order[0] < order[1], res0
    tol = 0.5 * (order[0] + order[1])                  # exactly one case converges at once

    batched = [P.Solver(c, storage="f32") for c in cases]
    batch = P.Batch(batched)
    if mode == "graph":
        batch.use_graph(True)
    else:
        batch.use_persistent(True)   # the tables are rebuilt when a case drops out
    steps, res = batch.run_to_steady(tol, max_super, check)
    assert batch.lups_per_super_step() == sum(s.lups_per_coarse_step() * p for s, p in zip(batched, per))
    batch.synchronize()
    batch.close()
    for k in range(len(cases)):
        if res0[k] < tol:
            assert steps[k] == check * per[k] and res[k] == res0[k]
        else:
            assert steps[k] == max_super * per[k] and not res[k] < tol
        twin = P.Solver(cases[k], storage="f32")
        twin.advance(steps[k])
        _assert_same(batched[k], twin, cases[k]["n_levels"], f"steady case {k}")


@pytest.mark.parametrize("storage", ["f32", "f64", "f16s"])
def test_persistent_grid_matches_the_launches(storage):
    """Persistent mode (lbr_batch_use_persistent): each table of the merged
    schedule runs as one cooperative grid whose workgroups take the blocks of
    each launch in turn and meet at a grid-wide barrier where the launch
    boundaries were.  Advanced 1 + 4 + 3 super steps (odd counts start and end
    in the middle of a two-step table) it must match the same batch run by
    launches (graph replay) bit for bit: fields, wall records and forces of
    every case."""
    import paper_2601_18443_amd as P
    cases = _cases()
    by_launch = [P.Solver(c, storage=storage) for c in cases]
    by_grid = [P.Solver(c, storage=storage) for c in cases]
    ba, bb = P.Batch(by_launch), P.Batch(by_grid)
    try:
        ba.use_graph(True)
        bb.use_persistent(True)
        for n in (1, 4, 3):
            ba.advance(n)
            bb.advance(n)
        for k, c in enumerate(cases):
            _assert_same(by_grid[k], by_launch[k], c["n_levels"], f"persistent case {k}")
        with pytest.raises(P.LbrError):
            bb.profile(True)                  # the launches it would time do not exist
        bb.use_persistent(False)
        ba.advance(2)
        bb.advance(2)
        for k, c in enumerate(cases):
            _assert_same(by_grid[k], by_launch[k], c["n_levels"], f"back to launches, case {k}")
    finally:
        ba.close()
        bb.close()


def test_persistent_mode_needs_one_population_format():
    import paper_2601_18443_amd as P
    solvers = [P.Solver(c, storage="mixeds") for c in _cases()]
    b = P.Batch(solvers)
    try:
        with pytest.raises(P.LbrError):
            b.use_persistent(True)
        b.advance(2)                          # still usable by launches
    finally:
        b.close()


def test_persistent_grid_on_full_size_sweep_cases():
    """Two cases of the 16-case sweep at full size (finest c/512, four and five
    levels): the finest virtual level alone has more tiles than the persistent
    grid has workgroups (2,048 on MI355X: 8 per CU), so workgroups take several
    blocks of one sub-launch in turn.  One plus two super steps must match the
    launches bit for bit on every level of both cases."""
    import paper_2601_18443_amd as P
    cases = [LI.case_sweep(k) for k in (1, 2)]
    by_launch = [P.Solver(c, storage="f32") for c in cases]
    by_grid = [P.Solver(c, storage="f32") for c in cases]
    finest_tiles = sum(s.level_info(c["n_levels"] - 1)["n_tiles"] for s, c in zip(by_launch, cases))
    assert finest_tiles > 2048, finest_tiles
    ba, bb = P.Batch(by_launch), P.Batch(by_grid)
    try:
        ba.use_graph(True)
        bb.use_persistent(True)
        for n in (1, 2):
            ba.advance(n)
            bb.advance(n)
        for k, c in enumerate(cases):
            _assert_same(by_grid[k], by_launch[k], c["n_levels"], f"full-size case {k}")
    finally:
        ba.close()
        bb.close()
