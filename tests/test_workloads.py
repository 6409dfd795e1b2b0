"""The seeded input generators (no arithmetic of the method): pins of the
counter-based start-vector generator against its published definition."""

import numpy as np

from workloads import _splitmix64, counter_uniform_complex


def test_splitmix64_reference_outputs():
    # SplitMix64 from state 0: the first outputs of the public reference
    # implementation (state advanced by the golden-ratio increment each call)
    gamma = 0x9E3779B97F4A7C15
    states = np.array([(k * gamma) % 2 ** 64 for k in range(3)], dtype=np.uint64)
    out = [int(x) for x in _splitmix64(states)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_uniform_complex_range_and_counter_layout():
    v = counter_uniform_complex(4096, 17)
    assert v.dtype == np.complex128
    assert np.all(np.abs(v.real) <= 1) and np.all(np.abs(v.imag) <= 1)
    # uniform on [-1, 1): mean ~0, variance 1/3 per component
    assert abs(v.real.mean()) < 0.05 and abs(v.imag.mean()) < 0.05
    assert abs(v.real.var() - 1 / 3) < 0.03
    # entry i depends on (seed, i) only: a prefix is the shorter vector
    assert np.array_equal(counter_uniform_complex(100, 17), v[:100])
    assert not np.array_equal(counter_uniform_complex(100, 18), v[:100])
