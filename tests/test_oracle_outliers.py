"""Pins of the force-outlier count (oracle/robustness.py).

A constructed array makes the count a closed form: m components of which k
equal a > 0 and the rest 0 have mean ka/m and population variance
a^2 (k/m)(1 - k/m). The k values a are beyond 5 sigma exactly when
(1 - k/m) > 25 k/m, i.e. k/m < 1/26, and the zeros are beyond it exactly when
k/m > 25/26. With m = 300 (100 atoms): k = 11 gives 11 outliers, k = 12 none,
k = 289 gives 289 outliers (the zeros), k = 288 none.
"""
import numpy as np
import pytest

import oracle


def _array(k, m=300, a=2.5, seed=0):
    f = np.zeros(m)
    idx = np.random.default_rng(seed).choice(m, k, replace=False)
    f[idx] = a
    return f.reshape(-1, 3), idx


@pytest.mark.parametrize("k,expected", [(1, 1), (11, 11), (12, 0), (150, 0), (288, 0), (289, 11)])
def test_two_valued_arrays(k, expected):
    F, _ = _array(k)
    assert oracle.force_outliers(F, 5.0) == expected


def test_threshold_scales_with_nsigma():
    # one component a among m - 1 zeros: |a - a/m| / sigma = sqrt(m - 1)
    F, _ = _array(1, m=300)
    s = np.sqrt(299.0)
    assert oracle.force_outliers(F, s * 0.999) == 1
    assert oracle.force_outliers(F, s * 1.001) == 0


def test_invariant_under_shift_scale_and_order():
    rng = np.random.default_rng(3)
    F = rng.normal(size=(400, 3))
    F[7, 1] = 40.0
    F[91, 0] = -35.0
    n = oracle.force_outliers(F, 5.0)
    assert n >= 2
    assert oracle.force_outliers(3.0 * F + 1.7, 5.0) == n
    assert oracle.force_outliers(F.reshape(-1)[rng.permutation(F.size)].reshape(-1, 3), 5.0) == n
