"""The per-scene group-side policy (no GPU): probing order, choice, re-probing."""
import pytest

from paper_2605_17855_amd.adaptive import GroupChooser


def _run(ch, cost, frames):
    used = []
    for _ in range(frames):
        g = ch.next()
        used.append(g)
        ch.observe(g, cost[g])
    return used


def test_round_robin_probes_then_commits_to_fastest():
    ch = GroupChooser([1, 2, 4, 8], probes=2)
    used = _run(ch, {1: 3.0, 2: 2.0, 4: 1.5, 8: 2.5}, 12)
    assert used[:8] == [1, 2, 4, 8, 1, 2, 4, 8]
    assert used[8:] == [4, 4, 4, 4] and ch.chosen == 4


def test_best_probe_counts_and_ties_pick_the_smaller_side():
    ch = GroupChooser([1, 2], probes=2)
    for g, ms in ((1, 9.0), (2, 1.0), (1, 1.0), (2, 5.0)):   # a slow first frame of side 1
        assert ch.next() == g
        ch.observe(g, ms)
    assert ch.chosen == 1 and ch.next() == 1


def test_reprobe_after_n_frames():
    ch = GroupChooser([1, 4], probes=1, reprobe_every=3)
    cost = {1: 1.0, 4: 2.0}
    assert _run(ch, cost, 5) == [1, 4, 1, 1, 1]
    cost = {1: 2.0, 4: 1.0}                 # the scene's balance changed
    assert _run(ch, cost, 4) == [1, 4, 4, 4]


def test_no_candidates():
    with pytest.raises(ValueError):
        GroupChooser([])
