"""Host-side helpers of the benchmark (no GPU)."""
import math

import numpy as np
import pytest

import bench


@pytest.mark.parametrize("n", [1, 2, 7, 100, 1001])
@pytest.mark.parametrize("p", [1, 50, 90, 99, 100])
def test_nearest_rank_definition(n, p):
    """The p-th percentile by nearest rank is the ceil(p/100 * n)-th smallest
    value: at least p% of the sample lies at or below it, and less than p%
    strictly below it."""
    rng = np.random.default_rng(n * 131 + p)
    v = rng.normal(size=n)
    q = bench.nearest_rank(v, p)
    assert q == sorted(v)[max(1, math.ceil(p / 100 * n)) - 1]
    assert np.mean(v <= q) >= p / 100 - 1e-12
    assert np.mean(v < q) < p / 100 or p == 100


def test_nearest_rank_is_a_sample_value():
    assert bench.nearest_rank([3.0, 1.0, 2.0], 50) == 2.0
    assert bench.nearest_rank([10.0], 99) == 10.0
    assert bench.nearest_rank([], 50) is None
