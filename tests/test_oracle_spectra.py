"""Pins of the oracle's spectra: theta (eq. 1), kappa_P (eq. 10-11), FIR taps.

Each check is fixed by the paper or by mathematics, not by re-running the
oracle's own formula: limits of eq. (1) (Fig. 3), the coth form of theta,
eq. (10) itself at off-grid frequencies, an independent alternating-series
solution of eq. (10) for P = 2, the high-frequency asymptote, and the DFT
identity that the realised filter spectrum equals the target on the grid.
"""
import math

import numpy as np
import pytest

from tests.closed_forms import theta_coth

RED = dict(hbar=1.0, kB=1.0)


@pytest.fixture(scope="module")
def U(orc):
    return orc.make_units(1.0, 1.0)


def test_theta_limits_fig3(orc, U):
    # omega -> 0 (or T -> inf): classical kB T; T -> 0: zero-point hbar w / 2.
    assert orc.theta(0.0, 2.5, U) == 2.5
    assert abs(orc.theta(1e-7, 1.0, U) - 1.0) < 1e-12
    assert abs(orc.theta(3.0, 1e-3, U) - 1.5) < 1e-15
    # Fig. 3: normalised energy theta/(hbar w) vs kT/(hbar w) tends to kT/(hbar w) + O(1/t)
    for t in (5.0, 20.0, 100.0):
        e = orc.theta(1.0, t, U)
        assert abs(e - t) < 1.0 / (12 * t) + 1e-12
    # theta is even in omega
    assert orc.theta(-2.0, 0.7, U) == orc.theta(2.0, 0.7, U)


@pytest.mark.parametrize("w,T", [(0.2, 1.0), (2.0, 1.0), (20.0, 1.0), (0.5, 0.05), (7.0, 30.0)])
def test_theta_matches_coth_form(orc, U, w, T):
    assert abs(orc.theta(w, T, U) / theta_coth(w, T, 1.0) - 1) < 2e-15


def test_theta_metal_units(orc):
    # 1 fs^-1 angular frequency at 300 K in eV: hbar w = 0.658 eV >> kT
    u = orc.make_units(0.6582119569, 8.617333262e-5)
    x = 0.6582119569 / (8.617333262e-5 * 300.0)
    excess = orc.theta(1.0, 300.0, u) - 0.5 * 0.6582119569
    assert abs(excess / (0.6582119569 * math.exp(-x)) - 1) < 1e-6


def test_kappa_P1_is_theta(orc, U):
    for w in (0.1, 1.0, 13.0):
        assert orc.kappa(w, 1.0, 1, U) == orc.theta(w, 1.0, U)


def test_kappa_zero_frequency(orc, U):
    for P in (2, 3, 8, 32):
        assert orc.kappa(0.0, 1.7, P, U) == 1.7
        assert abs(orc.kappa(1e-6, 1.0, P, U) - 1.0) < 1e-9


@pytest.mark.parametrize("P", [2, 3, 4, 5, 8, 16, 32])
def test_kappa_satisfies_eq10(orc, U, P):
    # (1/P) sum_k kappa(w_k)/(m w_k^2) = theta(w)/(m w^2), w_k^2 = w^2/P + 4 wP^2 sin^2(k pi/P)
    T = 1.0
    wP = math.sqrt(P) * T
    for w in (0.13, 0.9, 3.7, 11.0, 41.0):
        wk2 = [w * w / P + 4 * wP * wP * math.sin(k * math.pi / P) ** 2 for k in range(P)]
        lhs = sum(orc.kappa(math.sqrt(x), T, P, U) / x for x in wk2) / P
        rhs = theta_coth(w, T, 1.0) / (w * w)
        assert abs(lhs / rhs - 1) < 1e-12, (P, w)


def _kappa2_alternating(w, kT=1.0):
    """Independent P = 2 solution: with G(x) = kappa(sqrt x)/x and s1 = 4 wP^2,
    eq. (10) is G(y) + G(y + s1) = R(y) = theta(sqrt(2y))/y, solved by the
    alternating series G(y) = sum_m (-1)^m R(y + m s1) (Euler-accelerated)."""
    s1 = 4 * 2 * kT * kT
    y = w * w

    def R(x):
        return theta_coth(math.sqrt(2 * x), kT, 1.0) / x

    terms = np.array([(-1) ** m * R(y + m * s1) for m in range(4000)])
    S = np.cumsum(terms)
    for _ in range(40):
        S = 0.5 * (S[:-1] + S[1:])
    return S[-1] * y


@pytest.mark.parametrize("w", [0.3, 1.0, 2.0, 5.0, 10.0])
def test_kappa_P2_alternating_series(orc, U, w):
    assert abs(orc.kappa(w, 1.0, 2, U) / _kappa2_alternating(w) - 1) < 1e-10


@pytest.mark.parametrize("P", [2, 4, 8])
def test_kappa_high_frequency_asymptote(orc, U, P):
    # small-t behaviour of the Laplace kernel gives kappa -> hbar w / (2 sqrt P)
    r1 = orc.kappa(200.0, 1.0, P, U) / (200.0 / (2 * math.sqrt(P)))
    r2 = orc.kappa(2000.0, 1.0, P, U) / (2000.0 / (2 * math.sqrt(P)))
    assert abs(r2 - 1) < abs(r1 - 1) + 1e-15
    assert abs(r2 - 1) < 2e-3


def test_kappa_classical_limit(orc):
    # hbar -> 0: quantum corrections vanish, kappa -> kB T
    u = orc.make_units(1e-6, 1.0)
    for P in (2, 8):
        assert abs(orc.kappa(3.0, 1.0, P, u) - 1.0) < 1e-9


def test_kappa_quadrature_converged(orc, U):
    for P in (3, 8, 32):
        for w in (0.4, 4.0, 40.0):
            a = orc.kappa(w, 1.0, P, U, 1 / 16)
            b = orc.kappa(w, 1.0, P, U, 1 / 64)
            assert abs(a / b - 1) < 1e-14


def test_kappa_regression_values(orc, U):
    # reduced units hbar = kB T = 1 (values confirmed by the two pins above)
    ref = {2: [(0.5, 1.002331), (2.0, 1.111485), (10.0, 3.606111)],
           8: [(0.5, 0.995282), (2.0, 0.984628), (10.0, 1.916355)],
           32: [(2.0, 0.984990), (10.0, 1.195919)]}
    for P, vals in ref.items():
        for w, k in vals:
            assert abs(orc.kappa(w, 1.0, P, U) - k) < 6e-7


# ----------------------------------------------------------------- FIR taps
def test_taps_classical_delta(orc, U):
    h = orc.taps(0, 2.25, 1, 0.1, 64, U)
    assert h[32] == 1.5 and np.count_nonzero(h) == 1


@pytest.mark.parametrize("kind,P", [(1, 1), (2, 2), (2, 8)])
def test_taps_realise_target_spectrum_on_grid(orc, U, kind, P):
    two_nf, dt, T = 128, 0.05, 0.8
    Nf = two_nf // 2
    h = orc.taps(kind, T, P, dt, two_nf, U)
    # H(phi_j) = sum_k h_k exp(-i k phi_j), k = -Nf..Nf-1, via numpy's FFT
    k = np.arange(-Nf, Nf)
    Hj = np.fft.fft(np.roll(h, -Nf))  # index 0 holds k = 0
    for j in range(0, Nf + 1):
        w = math.pi * j / (Nf * dt)
        S = theta_coth(w, T, 1.0) if kind == 1 else orc.kappa(w, T, P, U)
        assert abs(abs(Hj[j]) ** 2 / S - 1) < 1e-12
    # real, zero-phase: h_k = h_-k
    assert np.allclose(h[Nf + 1:], h[Nf - 1:0:-1], rtol=0, atol=1e-15)
    assert np.max(np.abs(Hj.imag)) < 1e-12
    # Parseval: sum h^2 = mean of S over the 2Nf grid
    S_full = []
    for j in range(-Nf + 1, Nf + 1):
        w = math.pi * abs(j) / (Nf * dt)
        S_full.append(theta_coth(w, T, 1.0) if kind == 1 else orc.kappa(w, T, P, U))
    assert abs(np.sum(h * h) / np.mean(S_full) - 1) < 1e-12
    del k
