"""The merged launch schedule against the recursive cycle it reorders (no GPU).

The recursive cycle of Section 2.1 advances level l by two sub-steps of level
l + 1 followed by its own sub-step.  The library runs sub-steps of the coarse
levels inside the launches of finer ones.  This test rebuilds the cycle from
that definition, lists the buffers each sub-step reads and writes (the
populations, rho / u and chi of each level in its two time levels, and the
wall-node state), and requires that the library's grouping keeps every pair
of sub-steps with a common buffer, one of them writing it, in separate
launches and in the order of the cycle.  A planted mistake (a coarse
sub-step merged with its child) must be caught by the same check.
"""
import pytest

import paper_2601_18443_amd as P


def cycle(n_levels):
    """Level sub-steps of one coarse step in the order of the recursion."""
    out = []

    def rec(level, sub):
        if level + 1 < n_levels:
            rec(level + 1, 1)
            rec(level + 1, 2)
        out.append((level, sub))
    rec(0, 0)
    return out


def accesses(seq, n_levels):
    """(reads, writes) of each sub-step: a level reads its own current state, its
    child's populations (coalescence) and its parent's current state (explosion,
    ghost values); it writes its next state and, on the second sub-step, the
    restriction into its parent's next rho / u / chi."""
    cur = [0] * n_levels
    acc = []
    for lvl, sub in seq:
        c = cur[lvl]
        r = {("f", lvl, c), ("m", lvl, c), ("x", lvl, c), ("wall", lvl)}
        w = {("f", lvl, 1 - c), ("m", lvl, 1 - c), ("x", lvl, 1 - c), ("wall", lvl)}
        if lvl + 1 < n_levels:
            r.add(("f", lvl + 1, cur[lvl + 1]))
        if lvl > 0:
            p = cur[lvl - 1]
            r |= {("f", lvl - 1, p), ("m", lvl - 1, p), ("x", lvl - 1, p)}
            if sub == 2:
                w |= {("m", lvl - 1, 1 - p), ("x", lvl - 1, 1 - p)}
        acc.append((r, w))
        cur[lvl] ^= 1
    return acc


def check(groups, n_levels):
    seq = cycle(n_levels) * 2
    # each sub-step of the cycle once, matched in order per (level, sub-step)
    pos, seen = {}, {}
    for g, launch in enumerate(groups):
        for item in launch:
            k = seen.get(item, 0)
            seen[item] = k + 1
            idx = [i for i, s in enumerate(seq) if s == item][k]
            pos[idx] = g
    assert sorted(pos) == list(range(len(seq)))
    acc = accesses(seq, n_levels)
    for i in range(len(seq)):
        ri, wi = acc[i]
        for j in range(i + 1, len(seq)):
            rj, wj = acc[j]
            if (wi & rj) or (wj & ri) or (wi & wj):
                assert pos[i] < pos[j], (n_levels, seq[i], seq[j])


@pytest.mark.parametrize("n_levels", range(1, 11))
def test_merged_schedule_keeps_every_dependency_of_the_cycle(n_levels):
    groups = P.schedule(n_levels, merge=True)
    check(groups, n_levels)
    direct = P.schedule(n_levels, merge=False)
    assert [g[0] for g in direct] == cycle(n_levels) * 2 and all(len(g) == 1 for g in direct)
    assert len(groups) <= len(direct)


def test_eight_levels_take_195_launches_per_coarse_step():
    assert len(P.schedule(8, merge=True)) == 390
    assert len(P.schedule(8, merge=False)) == 510


def test_the_check_catches_a_coarse_step_merged_with_its_child():
    groups = [list(g) for g in P.schedule(6, merge=True)]
    # move the first merged coarse part (level w) into the next launch of level w + 1
    for i, g in enumerate(groups):
        if len(g) == 2:
            w = g[1][0]
            j = next(k for k in range(i + 1, len(groups)) if groups[k][0][0] == w + 1)
            groups[j].append(g.pop())
            break
    with pytest.raises(AssertionError):
        check(groups, 6)


def test_invalid_level_counts_are_refused():
    L = P.lib()
    assert L.lbr_schedule(0, 1, None, 0) < 0
    assert L.lbr_schedule(13, 1, None, 0) < 0


def test_deep_levels_ride_with_the_level_below_the_finest():
    """Eight levels: every sub-step of levels 0-4 shares a launch of level 6 (which
    fills only part of the device), level 5 shares launches of level 7, and no
    coarse sub-step runs alone except the last coarse level-0 step of the table."""
    groups = P.schedule(8, merge=True)
    pairs = {}
    for g in groups:
        if len(g) == 2:
            pairs.setdefault(g[1][0], set()).add(g[0][0])
    assert pairs == {0: {6}, 1: {6}, 2: {6}, 3: {6}, 4: {6}, 5: {7}}
    alone = [g[0] for g in groups if len(g) == 1 and g[0][0] <= 5]
    assert len(alone) <= 6
