"""Checkpoint-interval arithmetic of the rollout (host only)."""
from __future__ import annotations

import math

import pytest

from paper_1609_01479_amd.rollout import backward_bytes, default_interval, interval_for_budget


def test_backward_bytes_counts_checkpoints_and_segment_buffers():
    s = 1000
    assert backward_bytes(200, 1, s) == (200 + 2) * s            # every state kept, 2 scratch
    assert backward_bytes(200, 2, s) == (100 + 2) * s
    assert backward_bytes(200, 200, s) == (1 + 199) * s          # one checkpoint, 199 buffers
    assert backward_bytes(200, 15, s) == (14 + 14) * s
    # phi fields: one per segment, one per recomputed level
    assert backward_bytes(200, 15, s, phi_bytes=7) == 28 * s + (14 + 14) * 7
    assert backward_bytes(200, 1, s, phi_bytes=7) == 202 * s + 200 * 7
    assert backward_bytes(10, 50, s) == backward_bytes(10, 10, s)  # k is capped at T


@pytest.mark.parametrize("T", [1, 7, 200, 1000])
def test_interval_for_budget_is_the_smallest_fitting_interval(T):
    s = 336 << 20
    least = min(backward_bytes(T, k, s) for k in range(1, T + 1)) // s
    prev = None
    for states in sorted({T + 2, max(least, T // 2 + 2), max(least, 3 * math.isqrt(T)), least},
                         reverse=True):
        budget = states * s
        k = interval_for_budget(T, s, budget)
        assert backward_bytes(T, k, s) <= budget
        if k > 1:
            assert backward_bytes(T, k - 1, s) > budget
        if prev is not None:
            assert k >= prev  # less memory, more recomputation
        prev = k
    assert interval_for_budget(T, s, backward_bytes(T, 1, s)) == 1


def test_interval_for_budget_refuses_a_budget_below_the_minimum():
    s = 336 << 20
    T = 1000
    least = min(backward_bytes(T, k, s) for k in range(1, T + 1))
    assert least == backward_bytes(T, default_interval(T), s)
    with pytest.raises(ValueError):
        interval_for_budget(T, s, least - 1)
    assert backward_bytes(T, interval_for_budget(T, s, least), s) == least
