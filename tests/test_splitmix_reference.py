"""The generator reference in tests/splitmix.py against SplitMix64's published
outputs (stream 0: 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
0x06c45d188009454f) and the moments of its normal numbers."""
import numpy as np

from tests import splitmix


def test_splitmix64_published_outputs():
    got = splitmix.splitmix64(0, np.arange(1, 4, dtype=np.uint64))
    assert [int(v) for v in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_normal_numbers_moments():
    z = splitmix.std_normal(12345, np.arange(400_000, dtype=np.uint64))
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(z ** 3)) < 5 * np.sqrt(15.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 5 * np.sqrt(96.0 / n)
    # consecutive numbers uncorrelated
    assert abs(np.mean(z[1:] * z[:-1])) < 5 / np.sqrt(n)
