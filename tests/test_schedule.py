"""Host logic of the training policies (Sections III-C, III-D, III-E); no GPU needed."""
import collections

import numpy as np
import pytest

from paper_2411_02703_amd.schedule import DelayBuffer, KeyframeQueue, PyramidSchedule, SHSchedule


def test_new_keyframe_is_optimised_once_first():
    q = KeyframeQueue(cap=5, seed=1)
    q.add("a")
    assert q.select() == ["a"]
    q.add("b")
    assert q.select() == ["b"]  # a received keyframe is optimised once as a submap before random picks
    picks = [q.select()[0] for _ in range(2)]
    assert set(picks) <= {"a", "b"}


def test_caps_retire_keyframes_and_counts_are_exact():
    q = KeyframeQueue(cap=3, seed=2)
    for k in range(4):
        q.add(k)
    seen = collections.Counter()
    while q.active:
        for k in q.select():
            seen[k] += 1
    assert all(seen[k] == 3 for k in range(4))
    assert sorted(q.retired) == [0, 1, 2, 3]
    assert q.select() == []


def test_random_pick_is_uniform_and_seeded():
    def run(seed):
        q = KeyframeQueue(cap=10 ** 9, seed=seed)
        for k in range(5):
            q.add(k)
        for _ in range(5):
            q.select()  # the five first optimisations
        return [q.select()[0] for _ in range(20000)]

    a, b = run(7), run(7)
    assert a == b
    freq = np.bincount(a, minlength=5) / len(a)
    assert np.all(np.abs(freq - 0.2) < 0.015)


def test_batched_selection_draws_without_replacement():
    q = KeyframeQueue(cap=50, batch=3, seed=3)
    for k in range(6):
        q.add(k)
    first = q.select() + q.select()
    assert sorted(first) == list(range(6))  # fresh keyframes first, three per iteration
    for _ in range(30):
        s = q.select()
        assert len(s) == len(set(s)) == 3


def test_delay_buffer_releases_after_delay_newer_keyframes():
    d = DelayBuffer(delay=2)
    assert d.push(0) == [] and d.push(1) == []
    assert d.push(2) == [0]
    assert d.push(3) == [1]
    assert d.flush() == [2, 3]
    assert DelayBuffer(delay=0).push(5) == [5]


def test_pyramid_goes_coarse_to_fine():
    p = PyramidSchedule(levels=3, iters_per_level=4)
    levels = [p.level(k) for k in range(14)]
    assert levels == [2] * 4 + [1] * 4 + [0] * 6
    assert p.weights(0) == [0.0, 0.0, 1.0]
    assert p.weights(100, 0.5) == [0.5, 0.0, 0.0]


def test_sh_degree_ramp_is_capped_at_three():
    s = SHSchedule(every=10)
    assert [s.degree(i) for i in (0, 9, 10, 25, 30, 1000)] == [0, 0, 1, 2, 3, 3]


def test_invalid_queue_parameters():
    with pytest.raises(ValueError):
        KeyframeQueue(cap=0)
    q = KeyframeQueue()
    q.add(1)
    with pytest.raises(ValueError):
        q.add(1)
