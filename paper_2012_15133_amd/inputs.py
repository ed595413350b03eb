"""Seeded synthetic initial data for the square phase field crystal runs.

This module draws random numbers and nothing else: it holds none of the
scheme's arithmetic, so the CPU oracle and the GPU path can both be fed the
same bits from it.

The shape of the data follows the paper's pattern-formation experiment
(Section 5.2, initial data eqn:init2): i.i.d. uniform noise of amplitude 0.05
around a constant density, phi0 = mean + 0.05 * (2u - 1) with u ~ U[0, 1).

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Output i (i = 0, 1, ...) of the
stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15) with the published
finaliser; u = (z >> 11) * 2**-53 lies in [0, 1).  Grid point (x, y[, z]) takes
output i = x + n_x * (y + n_y * z), so x varies fastest; the returned array is
indexed [y, x] in 2-D and [z, y, x] in 3-D (C order, x contiguous).
"""

from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` SplitMix64 outputs for `seed`, as uint64."""
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """`count` doubles in [0, 1) from the top 53 bits of SplitMix64."""
    z = splitmix64(seed, count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def noise_ic(shape, mean: float, seed: int, amplitude: float = 0.05) -> np.ndarray:
    """phi0 = mean + amplitude * (2u - 1) on a grid of the given array shape.

    `shape` is (n_y, n_x) or (n_z, n_y, n_x); the result is float64, C order.
    """
    shape = tuple(int(s) for s in shape)
    count = int(np.prod(shape))
    u = uniform01(seed, count)
    return (mean + amplitude * (2.0 * u - 1.0)).reshape(shape)


def uniform_range(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    """`count` draws from U[lo, hi) (for parameter ensembles)."""
    return lo + (hi - lo) * uniform01(seed, count)


def ensemble_members(count: int = 64, sizes=(128, 256, 512), seed: int = 2024):
    """Parameter ensemble of independent 2-D runs: member k has n = sizes[k % len(sizes)]
    points per axis on a box of side n pi / 4 (h = pi / 4), epsilon ~ U[0.05, 0.5),
    mean density ~ U[-0.4, 0) and the noise initial data of `noise_ic` with seed
    seed + 1 + k.  Returns a list of dicts with keys n, L, epsilon, mean, seed."""
    eps = uniform_range(seed, count, 0.05, 0.5)
    means = uniform_range(seed + 7919, count, -0.4, 0.0)
    out = []
    for k in range(count):
        n = int(sizes[k % len(sizes)])
        side = n * np.pi / 4.0
        out.append({"n": (n, n), "L": (side, side), "epsilon": float(eps[k]), "mean": float(means[k]),
                    "seed": seed + 1 + k})
    return out
