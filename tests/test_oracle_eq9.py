"""Pins of the oracle's block generator of the random force (eq. 9: random
Fourier amplitudes on the grid omega_j = 2 pi j / (n dt), then an inverse
transform), and of the closed-form autocovariance of noise made that way.

* Per mode: the discrete Fourier transform of a generated block has mean
  |R_j|^2 / n = S_j over many dofs (statistically, every bin), for the QTB
  spectrum theta of eq. 1: the normalisation, the Hermitian completion and
  the transform's sign and scale all enter.
* White limit: with S = k_B T the block is Gaussian white noise of variance
  k_B T (Kolmogorov-Smirnov, vanishing lag correlations).
* Blocks: inside a block the covariance is the circular transform of S;
  consecutive blocks are independent; the time-averaged autocovariance over
  many blocks equals the closed form (1 - tau/n) c(tau).
"""
import math

import numpy as np
from scipy import stats

from tests.closed_forms import block_noise_autocovariance


def test_eq9_modes_carry_the_target_spectrum(orc):
    U = orc.make_units(1.0, 1.0)
    n, dt, T, n_dof = 64, 0.25, 0.3, 4096
    S = orc.noise_spectrum(1, T, 1, dt, n, U)
    # theta rises from k_B T at omega = 0 towards hbar omega / 2
    assert abs(S[0] - T) < 1e-12 and S[-1] > 5 * T
    z = orc.eq9_block(S, 7, 3, 1000, n_dof)
    assert z.shape == (n, n_dof) and np.isrealobj(z)
    F = np.fft.fft(z, axis=0)
    P = np.mean(np.abs(F[: n // 2 + 1]) ** 2, axis=1) / n
    ratio = P / S
    # (a^2 + b^2) / 2 is exponential (sd 1 per dof); a^2 at j = 0, n/2 has sd sqrt(2)
    sd = np.full(n // 2 + 1, 1.0 / math.sqrt(n_dof))
    sd[0] = sd[-1] = math.sqrt(2.0 / n_dof)
    zsc = (ratio - 1.0) / sd
    assert np.max(np.abs(zsc)) < 4.5, zsc
    assert 0.6 < np.mean(zsc ** 2) < 1.5
    # the generated amplitudes are Hermitian: the block is real to rounding
    # and the negative-frequency half mirrors the positive one
    assert np.allclose(F[n // 2 + 1:], np.conj(F[1: n // 2][::-1]), atol=1e-12 * np.max(np.abs(F)))


def test_eq9_white_limit(orc):
    U = orc.make_units(1.0, 1.0)
    n, T, n_dof = 128, 0.7, 512
    S = orc.noise_spectrum(0, T, 1, 0.1, n, U)
    assert np.allclose(S, T)
    z = orc.eq9_block(S, 11, 0, 0, n_dof)
    x = z.reshape(-1) / math.sqrt(T)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    assert abs(np.var(x) - 1.0) < 4 * math.sqrt(2.0 / x.size)
    for lag in (1, 2, 5):
        r = np.mean(z[lag:] * z[:-lag]) / T
        assert abs(r) < 4.0 / math.sqrt((n - lag) * n_dof), (lag, r)


def test_eq9_blocks_and_time_averaged_covariance(orc):
    """QTB spectrum, n = 32, 24 consecutive blocks of 2048 dofs: the empirical
    time-averaged autocovariance at lags 0..40 against the closed form, and
    zero correlation across the boundary of two blocks."""
    U = orc.make_units(1.0, 1.0)
    n, dt, T, n_dof, n_blk = 32, 0.5, 0.2, 2048, 24
    S = orc.noise_spectrum(1, T, 1, dt, n, U)
    z = np.concatenate([orc.eq9_block(S, 5, 1, b * n, n_dof) for b in range(n_blk)])
    L = 41
    emp = np.array([np.mean(z[t:] * z[: len(z) - t]) for t in range(L)])
    # positions t .. len - 1 - t: lags below n straddle a boundary for a
    # fraction tau / n of them (the closed form's weighting)
    ref = block_noise_autocovariance(S, L)
    se = np.array([np.std(z[t:] * z[: len(z) - t]) for t in range(L)]) / math.sqrt(n_dof * (n_blk - 1))
    zsc = (emp - ref) / se
    assert np.max(np.abs(zsc)) < 4.5, zsc
    # within a block the lag-1 covariance is the circular one, across the
    # boundary it vanishes
    c1 = np.fft.ifft(np.concatenate([S, S[-2:0:-1]])).real[1]
    inside = np.mean(z[1:n] * z[: n - 1])
    first, last = z[n::n], z[n - 1::n][:-1]   # first row of block b + 1, last of block b
    across = np.mean(first * last)
    assert abs(inside - c1) < 5 * np.std(z[1:n] * z[: n - 1]) / math.sqrt((n - 1) * n_dof)
    assert abs(across) < 5 * np.std(first * last) / math.sqrt((n_blk - 1) * n_dof)
    # theta rising towards the Nyquist frequency anticorrelates neighbouring steps
    assert abs(c1) > 0.2 * ref[0]
