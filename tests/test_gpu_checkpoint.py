"""Checkpoint and restart of the HIP library (needs an MI355X).

A run saved after n steps and continued for m more in a fresh context must
end bit-identical to the uninterrupted run of n + m steps (both time levels,
the wall-model state and the step counter are restored).  Files from another
grid or storage, truncated or corrupted files are refused without changing
the context.
"""
import os

import numpy as np
import pytest

import lbr_inputs as LI

pytestmark = pytest.mark.gpu


def _state(s, n_levels):
    out = [s.field(l, k) for l in range(n_levels) for k in range(4)]
    out += [s.wall(l) for l in range(n_levels)]
    return out + [s.forces()]


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


@pytest.mark.parametrize("storage", ["f32", "f16", "mixed", "f16s"])
def test_restart_is_bit_identical_to_the_uninterrupted_run(tmp_path, storage):
    import paper_2601_18443_amd as P
    case = dict(LI.case_airfoil_small(), ramp_steps=6, ramp_start=0.5)   # restart inside the ramp
    L = case["n_levels"]
    ref = P.Solver(case, storage=storage)
    ref.advance(5)
    path = str(tmp_path / "state.lbr")
    ref.save(path)
    ref.use_graph(True)
    ref.advance(9)
    want = _state(ref, L)

    s = P.Solver(case, storage=storage)
    s.advance(1)                                   # overwritten by the load
    s.load(path)
    s.use_graph(True)
    s.advance(9)
    assert _same(_state(s, L), want)


def test_foreign_and_damaged_files_are_refused(tmp_path):
    import paper_2601_18443_amd as P
    case = LI.case_airfoil_small()
    a = P.Solver(case, storage="f32")
    a.advance(3)
    good = str(tmp_path / "a.lbr")
    a.save(good)
    before = _state(a, case["n_levels"])

    other = P.Solver(LI.case_airfoil_small(alpha_deg=4.0), storage="f32")   # another grid
    with pytest.raises(P.LbrError):
        other.load(good)
    with pytest.raises(P.LbrError):
        P.Solver(case, storage="f64").load(good)                            # another storage
    h16 = P.Solver(case, storage="f16")
    h16.advance(1)
    h16_path = str(tmp_path / "h16.lbr")
    h16.save(h16_path)
    with pytest.raises(P.LbrError):
        P.Solver(case, storage="f16s").load(h16_path)                       # another storage shift

    raw = open(good, "rb").read()
    cut = str(tmp_path / "cut.lbr")
    with open(cut, "wb") as fh:
        fh.write(raw[: len(raw) // 2])
    bad = str(tmp_path / "bad.lbr")
    flipped = bytearray(raw)
    flipped[len(raw) // 2] ^= 0x40
    with open(bad, "wb") as fh:
        fh.write(bytes(flipped))
    for path in (cut, bad, str(tmp_path / "missing.lbr")):
        with pytest.raises(P.LbrError):
            a.load(path)
    assert _same(_state(a, case["n_levels"]), before)
    a.load(good)
    assert _same(_state(a, case["n_levels"]), before)
    assert os.path.getsize(good) == len(raw)
