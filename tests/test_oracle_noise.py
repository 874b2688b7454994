"""Pins of the oracle's white and coloured noise.

* Philox4x32-10: compared word for word with rocRAND's independent
  implementation (host build of its public header).
* The project-defined ln and cos(2 pi u): accuracy against libm.
* Gaussian draws: moments, Kolmogorov-Smirnov, lag correlations.
* Coloured noise: the direct FIR sum equals numpy's convolution, and the
  random-force spectrum of the O step matches 2 m gamma theta (eq. 6-7)
  within chi-square bands.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import signal, stats

from tests.closed_forms import theta_coth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    src = os.path.join(HERE, "rocrand_philox_ref.cpp")
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "ref")
    subprocess.check_call(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-o", exe, src])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(400):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        n = int(rng.integers(-(2**20), 2**32))
        d = int(rng.integers(0, 2**32))
        w = int(rng.integers(0, 2**32))
        cases.append((seed, n, d, w))
    cases += [(0, 0, 0, 0), (2**64 - 1, -(2**40), 2**32 - 1, 2**32 - 1)]
    inp = "\n".join(f"{s} {n + 2**40} {d} {w}" for s, n, d, w in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (s, n, d, w), line in zip(cases, out):
        c = n + 2**40
        ours = orc.philox([c & 0xFFFFFFFF, c >> 32, d, w], [s & 0xFFFFFFFF, s >> 32])
        assert ours == [int(x) for x in line.split()], (s, n, d, w)


def test_log_spec_accuracy(orc):
    rng = np.random.default_rng(3)
    us = list(rng.random(2000)) + [2.0**-53, 1 - 2.0**-53, 0.5, math.sqrt(0.5),
                                   math.sqrt(0.5) * (1 + 2**-52), 1e-300 * 0 + 2**-40]
    for u in us:
        ref = math.log(u)
        got = orc.log_spec(u)
        assert abs(got - ref) <= 4e-16 * max(1.0, abs(ref)), u


def test_cos2pi_spec_accuracy(orc):
    rng = np.random.default_rng(4)
    Ns = [int(x) * 2 + 1 for x in rng.integers(0, 2**52, size=3000)]
    Ns += [1, 2**53 - 1, 2**51 - 1, 2**51 + 1, 2**52 - 1, 2**52 + 1, 3 * 2**50 + 1]
    for N in Ns:
        ref = math.cos(2 * math.pi * (N / 2.0**53))
        assert abs(orc.cos2pi_spec(N) - ref) < 2e-15, N


def test_gaussian_moments_and_ks(orc):
    w = orc.gauss_fill(seed=12345, n0=-700, n_rows=1000, d0=17, n_dof=1000, stream=3, tag=0)
    x = w.ravel()
    n = x.size
    assert abs(x.mean()) < 5 / math.sqrt(n)
    assert abs(x.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(stats.skew(x)) < 5 * math.sqrt(6 / n)
    assert abs(stats.kurtosis(x)) < 5 * math.sqrt(24 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # independence along steps and along dofs
    for lag_axis in (0, 1):
        a = np.take(w, range(0, 999), axis=lag_axis).ravel()
        b = np.take(w, range(1, 1000), axis=lag_axis).ravel()
        assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


def test_gaussian_is_a_pure_function_of_counter(orc):
    a = orc.gauss(7, -5, 123, 2, 0)
    b = orc.gauss_fill(7, -5, 1, 123, 1, 2, 0)[0, 0]
    assert a == b
    assert orc.gauss(7, -5, 123, 2, 1) != a   # tag changes the stream
    assert orc.gauss(8, -5, 123, 2, 0) != a   # seed changes the stream


def test_zeta_direct_equals_convolution(orc):
    U = orc.make_units(1.0, 1.0)
    h = orc.taps(1, 1.0, 1, 0.1, 64, U)
    Nf = 32
    seed, stream, d = 99, 1, 5
    n0, n1 = -10, 40
    w = orc.gauss_fill(seed, n0 - Nf, n1 - n0 + 2 * Nf, d, 1, stream, 0)[:, 0]
    # zeta_n = sum_k h_k w_{n-k}: numpy convolution of w with taps ordered k=-Nf..Nf-1
    conv = np.convolve(w, h, mode="full")
    for n in range(n0, n1):
        # w index of step m is m - (n0 - Nf); conv[i] = sum_j h[j] w[i - j]; h[j] is k = j - Nf
        i = (n - (n0 - Nf)) + Nf
        assert abs(orc.zeta(h, seed, stream, n, d) - conv[i]) < 1e-13


def test_random_force_psd_is_2m_gamma_theta(orc):
    """Eq. (6)-(7): the O step's random force R_n = m sigma zeta_n / dt with
    sigma = sqrt((1-c1^2)/m) has PSD m (1-c1^2)/dt * |H(w dt)|^2, which equals
    2 m gamma theta(w) up to the factor (1-exp(-2 gamma dt))/(2 gamma dt)."""
    U = orc.make_units(1.0, 1.0)
    T, dt, gamma, m = 0.5, 0.1, 0.02, 1.7
    two_nf = 64
    Nf = two_nf // 2
    h = orc.taps(1, T, 1, dt, two_nf, U)
    n_steps, n_dof = 2**14, 64
    w = orc.gauss_fill(5, -Nf, n_steps + two_nf, 0, n_dof, 0, 0)
    zeta = np.stack([np.convolve(w[:, j], h, mode="valid") for j in range(n_dof)], 1)
    c1 = math.exp(-gamma * dt)
    R = m * math.sqrt((1 - c1 * c1) / m) * zeta / dt
    # Hann window: the spectrum spans a 30x range, boxcar side lobes would leak
    f, pxx = signal.welch(R, fs=1.0 / dt, nperseg=256, axis=0, return_onesided=False,
                          detrend=False, window="hann")
    pxx = pxx.mean(axis=1)
    omega = 2 * math.pi * f
    corr = (1 - c1 * c1) / (2 * gamma * dt)
    target = np.array([2 * m * gamma * theta_coth(x, T, 1.0) * corr for x in omega])
    # Welch, 256-point Hann segments: ~127 segments x 64 dofs per bin
    rel = pxx / target - 1
    sel = np.abs(omega) < 0.8 * math.pi / dt   # away from the Nyquist edge
    assert np.max(np.abs(rel[sel])) < 0.08
    assert abs(np.mean(rel[sel])) < 0.01
    # the discrete spectrum converges to eq. (7) as gamma dt -> 0
    assert abs(corr - 1) < gamma * dt
