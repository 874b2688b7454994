"""Pins of the oracle's velocity density of states (the time-correlation
route of Sec. 3: the spectrum of the velocity series, whose check at high
friction the paper recommends).

* Parseval: the mean of the spectrum over all frequencies is the weighted
  mean square velocity, for any series and weights.
* Pure tones: a cosine at a bin frequency puts all its weight in that bin,
  with the closed-form height; a constant goes to frequency zero.
* Linear response: QTB trajectories of the oracle on independent harmonic
  oscillators have the spectrum that linear-systems theory gives for the
  discrete BAOAB map driven by the FIR-filtered noise (transfer function of
  the map times the filter's |H|^2, smoothed by the segment's Fejer window),
  bin by bin within the statistical error.
"""
import math

import numpy as np

from tests.closed_forms import baoab_mode_map, velocity_spectrum_discrete


def _full_mean(S, seg):
    """Mean over all seg frequencies of a spectrum given for k = 0 .. seg/2."""
    return (S[0] + S[-1] + 2.0 * np.sum(S[1:-1])) / seg


def test_vdos_parseval_weights_and_segments(orc):
    rng = np.random.default_rng(4)
    seg, n_dof = 64, 5
    v = rng.normal(size=(3 * seg + 17, n_dof)) * np.array([1.0, 2.0, 0.5, 3.0, 1.5])
    w = rng.uniform(0.5, 2.0, n_dof)
    phi, S, n_seg = orc.vdos(v, seg, w)
    assert n_seg == 3 and len(S) == seg // 2 + 1
    assert np.allclose(phi, 2 * np.pi * np.arange(seg // 2 + 1) / seg)
    used = v[: 3 * seg]
    assert abs(_full_mean(S, seg) - np.sum(w * np.mean(used ** 2, axis=0))) < 1e-12 * np.sum(S)
    # each segment on its own, then the average (the trailing part is dropped)
    parts = [orc.vdos(used[q * seg:(q + 1) * seg], seg, w)[1] for q in range(3)]
    assert np.allclose(S, np.mean(parts, axis=0), rtol=1e-13, atol=0)
    # weights are linear, and unit weights are the default
    S1 = orc.vdos(v, seg)[1]
    S_each = [orc.vdos(v[:, j], seg)[1] for j in range(n_dof)]
    assert np.allclose(S1, np.sum(S_each, axis=0), rtol=1e-13, atol=0)
    assert np.allclose(S, np.array(S_each).T @ w, rtol=1e-13, atol=0)


def test_vdos_pure_tones(orc):
    seg = 128
    t = np.arange(2 * seg)
    for k0, A, ph in ((5, 1.3, 0.4), (17, 0.7, -1.1), (63, 2.0, 0.0)):
        v = A * np.cos(2 * np.pi * k0 * t / seg + ph)
        _, S, _ = orc.vdos(v, seg, [3.0])
        # V_k0 = A seg e^{i ph} / 2: |V|^2 / seg = A^2 seg / 4, times the weight
        assert abs(S[k0] - 3.0 * A * A * seg / 4) < 1e-10 * S[k0]
        assert np.max(np.delete(S, k0)) < 1e-20 * seg + 1e-12 * S[k0]
    # Nyquist tone (-1)^t and a constant
    _, S, _ = orc.vdos(np.cos(np.pi * t), seg)
    assert abs(S[-1] - seg) < 1e-10 and np.max(S[:-1]) < 1e-12
    _, S, _ = orc.vdos(np.full(2 * seg, 0.5), seg)
    assert abs(S[0] - 0.25 * seg) < 1e-12 and np.max(S[1:]) < 1e-12


def expected_periodogram(M, b, taps, seg, n_grid=1 << 15):
    """E[|V_k|^2 / seg] of a stationary series with the spectrum of the
    discrete scheme: the autocovariance c(tau) by a fine inverse DFT of the
    spectrum, then the Fejer-windowed sum over |tau| < seg."""
    phi = 2 * np.pi * np.arange(n_grid) / n_grid
    Sv = velocity_spectrum_discrete(M, b, taps, phi)
    c = np.fft.ifft(Sv).real[:seg]
    tau = np.arange(seg)
    k = np.arange(seg // 2 + 1)
    wt = (1.0 - tau / seg) * c
    return c[0], wt[0] + 2.0 * np.cos(np.outer(2 * np.pi * k / seg, tau[1:])) @ wt[1:]


def test_vdos_of_qtb_oscillators_matches_linear_response(orc):
    """256 independent oscillators, m = hbar = k_B = 1, omega = 1, k_B T = 0.25
    (hbar omega / k_B T = 4), gamma = 0.2, dt = 0.1, QTB filter 2Nf = 256:
    32 segments of 256 steps after 1000 steps of equilibration."""
    n, omega, T, gamma, dt, two_nf, seg, n_seg = 256, 1.0, 0.25, 0.2, 0.1, 256, 256, 32
    pot = orc.make_pot(1, (1.0,))
    U = orc.make_units(1.0, 1.0)
    rng = np.random.default_rng(8)
    x0 = rng.normal(0.0, 0.5, (1, 1, n))
    sim = orc.Sim(pot, U, n, 1, 1, None, np.zeros(n, np.int32), T, gamma, dt, 21, 0, 1, two_nf, x0,
                  n_threads=4, harm_omega=np.full(n, omega))
    sim.run(1000)
    v = np.empty((seg * n_seg, n))
    for t in range(seg * n_seg):
        sim.run(1)
        v[t] = sim.state()[1][0, 0]
    # per-oscillator spectra: independent samples of each bin
    per = np.array([orc.vdos(v[:, j], seg)[1] for j in range(n)])
    mean, se = per.mean(axis=0), per.std(axis=0, ddof=1) / math.sqrt(n)
    c1 = math.exp(-gamma * dt)
    M, b = baoab_mode_map(omega * omega, 0.0, c1, math.sqrt(1 - c1 * c1), dt)
    taps = orc.taps(1, T, 1, dt, two_nf, U)
    v2, Ek = expected_periodogram(M, b, taps, seg)
    z = (mean - Ek) / se
    print(f"<v^2> exact {v2:.5f}, sampled {np.mean(v ** 2):.5f}; "
          f"bins: max |z| = {np.max(np.abs(z)):.2f}, mean z^2 = {np.mean(z * z):.3f}")
    # the exact <v^2> is the QTB one, well above the classical k_B T / m
    assert v2 > 1.5 * T
    assert np.max(np.abs(z)) < 4.5
    assert 0.75 < np.mean(z * z) < 1.35
    # the peak sits at the oscillator's frequency in radians per step
    k_peak = int(np.argmax(Ek))
    assert abs(2 * np.pi * k_peak / seg - omega * dt) <= 2 * np.pi / seg
