"""Error bars of time averages from correlated samples: the blocking
transformation of Flyvbjerg and Petersen (J. Chem. Phys. 91, 461 (1989)).

A series of n samples (for instance the library's observable means over
consecutive short windows) is repeatedly replaced by the means of adjacent
pairs.  At each level the naive standard error of the mean, sqrt(c0 / (n - 1))
with c0 the (biased) variance of the current series, is an estimate of the true
one that grows while the blocks are shorter than the correlation time and
stays constant once they are longer; its own relative uncertainty is
1 / sqrt(2 (n - 1)).  The error bar is taken at the first level from which the
estimate no longer rises beyond that uncertainty."""
from __future__ import annotations

import math

import numpy as np


def blocking_levels(x, min_blocks=4):
    """(blocks, standard error, its uncertainty) at every blocking level with
    at least min_blocks blocks (an odd sample is dropped at each halving)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    out = []
    while len(x) >= max(min_blocks, 2):
        n = len(x)
        c0 = float(np.mean((x - x.mean()) ** 2))
        se = math.sqrt(c0 / (n - 1))
        out.append((n, se, se / math.sqrt(2.0 * (n - 1))))
        m = n // 2
        x = 0.5 * (x[: 2 * m : 2] + x[1 : 2 * m : 2])
    return out


def blocked_error(x, min_blocks=8):
    """Standard error of the mean of the series x by blocking: the first
    level whose estimate lies within the uncertainty of every later level's
    (the plateau), else the largest estimate of the levels with at least
    min_blocks blocks (a series too short to show a plateau)."""
    lv = blocking_levels(x, min_blocks)
    if not lv:
        raise ValueError("blocking needs at least min_blocks samples")
    for k, (_, se, _) in enumerate(lv):
        if all(se + d_later >= se_later for _, se_later, d_later in lv[k + 1:]):
            return se
    return max(se for _, se, _ in lv)


def mean_and_error(x, min_blocks=8):
    """(mean, blocked standard error) of the series x."""
    x = np.asarray(x, dtype=np.float64).ravel()
    return float(x.mean()), blocked_error(x, min_blocks)
