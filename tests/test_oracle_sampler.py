"""Pins of the counter-based block sampler (CPU only)."""
import os

import numpy as np

from oracle import sampler

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_values():
    vals = [int(l, 16) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert [sampler.splitmix64(0, k) for k in (1, 2, 3)] == vals


def test_epochs_are_permutations_and_differ():
    M = 90
    s = sampler.schedule(M, 5, 3001)
    assert s.shape == (450,)
    for e in range(5):
        assert sorted(s[e * M:(e + 1) * M]) == list(range(M))
    assert not np.array_equal(s[:M], s[M:2 * M])


def test_shuffle_is_roughly_uniform():
    # position of block 0 over many epochs is close to uniform on 0..M-1
    M, E = 6, 6000
    s = sampler.schedule(M, E, 17).reshape(E, M)
    pos = np.argmax(s == 0, axis=1)
    counts = np.bincount(pos, minlength=M)
    assert np.all(np.abs(counts - E / M) < 5 * np.sqrt(E / M))
