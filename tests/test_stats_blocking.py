"""Pins of the blocking error estimate (paper_1905_02521_amd.stats): the
halving by hand, independent samples (the naive standard error), and an
AR(1) series whose variance of the mean is known in closed form."""
import math

import numpy as np
from scipy.signal import lfilter

from paper_1905_02521_amd.stats import blocked_error, blocking_levels, mean_and_error


def test_levels_by_hand():
    lv = blocking_levels(np.arange(1.0, 9.0), min_blocks=2)
    assert [n for n, _, _ in lv] == [8, 4, 2]
    # 1..8: biased variance 5.25; pairs 1.5, 3.5, 5.5, 7.5: 5.0; 2.5, 6.5: 4.0
    for (n, se, d), c0 in zip(lv, (5.25, 5.0, 4.0)):
        assert abs(se - math.sqrt(c0 / (n - 1))) < 1e-15
        assert abs(d - se / math.sqrt(2 * (n - 1))) < 1e-15


def test_independent_samples_give_the_naive_error():
    x = np.random.default_rng(1).normal(2.0, 3.0, 1 << 16)
    m, se = mean_and_error(x)
    naive = x.std(ddof=1) / math.sqrt(len(x))
    assert abs(se / naive - 1.0) < 0.1
    assert abs(m - 2.0) < 4 * naive


def test_ar1_series_matches_the_exact_variance_of_the_mean():
    """x_t = phi x_{t-1} + e_t (stationary start): Var(mean) =
    s2 / N [(1 + phi) / (1 - phi) - 2 phi (1 - phi^N) / (N (1 - phi)^2)],
    s2 = 1 / (1 - phi^2) for unit innovations."""
    rng = np.random.default_rng(7)
    for phi in (0.5, 0.9, 0.98):
        N = 1 << 20
        e = rng.normal(size=N)
        x = np.empty(N)
        x[0] = e[0] / math.sqrt(1 - phi * phi)
        # x_t = phi x_{t-1} + e_t for t >= 1 as a first-order recursive filter
        x[1:] = lfilter([1.0], [1.0, -phi], e[1:], zi=[phi * x[0]])[0]
        s2 = 1.0 / (1.0 - phi * phi)
        var = s2 / N * ((1 + phi) / (1 - phi) - 2 * phi * (1 - phi ** N) / (N * (1 - phi) ** 2))
        se = blocked_error(x)
        assert abs(se / math.sqrt(var) - 1.0) < 0.1, (phi, se, math.sqrt(var))
        # the naive error underestimates it by sqrt((1 + phi) / (1 - phi))
        assert x.std() / math.sqrt(N) < 0.8 * se
