"""Pins of the oracle's selection-frequency counting: closed forms on
constructed masks and a bit-by-bit recount written independently."""
import numpy as np

import oracle as O


def test_constant_masks_closed_form():
    S, L, G = 10, 3, 2
    active = np.zeros(S * L, dtype=np.uint32)
    active[:] = 0b1011                       # features 0, 1, 3 always selected
    status = np.zeros(S * L, dtype=np.int32)
    group = np.array([0] * 4 + [1] * 6)
    freq, cnt = O.selection_frequency(active, status, group, G, L)
    assert np.all(cnt == np.array([[4] * L, [6] * L]))
    expect = np.zeros(32)
    expect[[0, 1, 3]] = 1.0
    assert np.all(freq == expect)


def test_status_filter_and_halves():
    S, L = 8, 1
    active = np.array([1 << 5] * 4 + [0] * 4, dtype=np.uint32)
    status = np.array([0, 1, 3, 0, 0, 1, 4, 0], dtype=np.int32)   # 3 and 4 are not accepted
    freq, cnt = O.selection_frequency(active, status, np.zeros(S, int), 1, L)
    assert cnt[0, 0] == 6
    assert freq[0, 0, 5] == 3 / 6 and freq[0, 0].sum() == 3 / 6


def test_random_masks_recount():
    rng = np.random.default_rng(2)
    S, L, G = 200, 4, 3
    active = rng.integers(0, 2 ** 32, size=S * L, dtype=np.uint64).astype(np.uint32)
    status = rng.integers(0, 2, size=S * L).astype(np.int32)
    group = rng.integers(0, G, size=S)
    freq, cnt = O.selection_frequency(active, status, group, G, L)
    bits = ((active.reshape(S, L)[:, :, None] >> np.arange(32)) & 1).astype(float)
    for g in range(G):
        m = group == g
        assert np.allclose(freq[g], bits[m].mean(axis=0))
        assert np.all(cnt[g] == m.sum())
