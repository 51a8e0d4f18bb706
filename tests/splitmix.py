"""Reference of the library's counter-based normal generator (test
infrastructure): SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used
counter-wise -- value k of stream `seed` is the SplitMix64 output mix of
seed + k * 0x9E3779B97F4A7C15 -- and the Box-Muller transform of two such
values, written from the published definitions in NumPy uint64 / FP64."""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed, k):
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.asarray(k, dtype=np.uint64) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def std_normal(seed, j):
    """Normal number j of stream seed: u1 in (0, 1], u2 in [0, 1)."""
    j = np.asarray(j, dtype=np.uint64)
    u1 = ((splitmix64(seed, np.uint64(2) * j + np.uint64(1)) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (splitmix64(seed, np.uint64(2) * j + np.uint64(2)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
