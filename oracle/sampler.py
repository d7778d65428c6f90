"""Random-cyclic block sampling from a counter-based generator (test infrastructure only).

The 2D experiment draws blocks random-cyclically (sec. 4.3): every epoch
visits each of the M blocks once, in random order.  The library draws this
order itself inside its solve loop, so both sides implement the same
published generator:

* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the k-th output (k = 1, 2,
  ...) for seed S is mix(S + k * 0x9E3779B97F4A7C15 mod 2^64), with
  mix(z) = z3 ^ (z3 >> 31), z2 = (z1 ^ (z1 >> 27)) * 0x94D049BB133111EB,
  z1 = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 (all mod 2^64);
* Fisher-Yates (Durstenfeld) shuffle of the identity 0..M-1: for i = M-1
  down to 1 draw u and swap positions i and j = floor(u * (i+1) / 2^64);
* epoch e (0-based) uses outputs k = e*(M-1) + 1 ... e*(M-1) + (M-1).

Pinned by published SplitMix64 output values and by permutation validity.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, k: int) -> int:
    z = (seed + k * GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def epoch_permutation(n_blocks: int, epoch: int, seed: int) -> np.ndarray:
    perm = list(range(n_blocks))
    k = epoch * (n_blocks - 1)
    for i in range(n_blocks - 1, 0, -1):
        k += 1
        u = splitmix64(seed, k)
        j = (u * (i + 1)) >> 64
        perm[i], perm[j] = perm[j], perm[i]
    return np.asarray(perm, dtype=np.int32)


def schedule(n_blocks: int, epochs: int, seed: int) -> np.ndarray:
    return np.concatenate([epoch_permutation(n_blocks, e, seed) for e in range(epochs)])
