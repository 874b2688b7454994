"""Pins of the oracle's anharmonic on-site potentials (the 1D models with the
anharmonicity parameter C of eq. 13: Morse and double well) and of the exact
quantum reference the zero-point-leakage measurements compare with.

* The finite-difference Schroedinger levels reproduce the textbook Morse
  spectrum, and the double-well levels converge under grid refinement and
  tend to the harmonic levels of the wells when C is small.
* The oracle's forces are minus the finite-difference gradient of its
  energies.
* Classical Langevin dynamics of the oracle (white noise) samples the
  classical Boltzmann distribution of each potential (quadrature).
"""
import math

import numpy as np
import pytest

from tests.closed_forms import (classical_mean, double_well_potential, morse_levels_exact,
                                morse_potential, quantum_mean_energy, schrodinger_levels)


def test_schrodinger_levels_match_morse_closed_form():
    V0, d, m = 1.0, 1.0, 1.0
    hbar = math.sqrt(2 * m * V0 * d * d * 0.02)   # C = 0.02
    x = np.linspace(-1.2, 14.0, 6001)[1:-1]
    lev = schrodinger_levels(morse_potential(x, V0, d), m, hbar, x)
    ex = morse_levels_exact(V0, d, m, hbar, 6)
    assert np.max(np.abs(lev[:6] - ex) / ex) < 2e-5
    # the canonical mean follows from the levels
    kT = 0.1
    w = np.exp(-(ex - ex[0]) / kT)
    assert abs(quantum_mean_energy(lev[:6], kT) - np.sum(ex * w) / np.sum(w)) < 1e-5


def test_double_well_levels_converge_and_approach_the_wells():
    V0, d, m = 1.0, 1.0, 1.0
    hbar = math.sqrt(2 * m * V0 * d * d * 0.002)  # C = 0.002: deep wells
    coarse = np.linspace(-2.2, 2.2, 3001)[1:-1]
    fine = np.linspace(-2.2, 2.2, 6001)[1:-1]
    lc = schrodinger_levels(double_well_potential(coarse, V0, d), m, hbar, coarse)[:4]
    lf = schrodinger_levels(double_well_potential(fine, V0, d), m, hbar, fine)[:4]
    assert np.max(np.abs(lc - lf)) < 4 * np.max(np.abs(lf)) * 1e-5
    # two nearly degenerate doublets near hw (n + 1/2) of one well, w = sqrt(8 V0 / m d^2)
    w = math.sqrt(8 * V0 / (m * d * d))
    assert abs(lf[1] - lf[0]) < 1e-6 and abs(lf[3] - lf[2]) < 1e-4
    assert abs(lf[0] / (0.5 * hbar * w) - 1) < 0.03
    assert abs((lf[2] - lf[0]) / (hbar * w) - 1) < 0.06


@pytest.mark.parametrize("kind", [2, 3])
def test_onsite_forces_are_minus_energy_gradient(orc, kind):
    V0, d = 0.8, 0.7
    pot = orc.make_pot(kind, (1.0,), V0=(V0,), d=(d,))
    U = orc.make_units(1.0, 1.0)
    h = 1e-5

    def energy_force(x):
        s = orc.Sim(pot, U, 1, 1, 1, None, np.zeros(1, np.int32), 1.0, 0.0, 0.01, 0, 0, 0, 2,
                    np.array([[[x]]]))
        _, _, f, _ = s.state()
        return s.observe()[1], f[0, 0, 0]

    for x in (-0.4, -0.1, 0.05, 0.3, 0.9, 1.6):
        e_p, _ = energy_force(x + h)
        e_m, _ = energy_force(x - h)
        _, f = energy_force(x)
        fd = -(e_p - e_m) / (2 * h)
        assert abs(f - fd) < 1e-7 * max(1.0, abs(f)), (kind, x, f, fd)
    # energies against the written-out potentials
    V = morse_potential if kind == 2 else double_well_potential
    for x in (-0.3, 0.2, 1.1):
        assert abs(energy_force(x)[0] - V(x, V0, d)) < 1e-13


@pytest.mark.parametrize("kind", [2, 3])
def test_classical_langevin_samples_boltzmann(orc, kind):
    """White-noise BAOAB on 512 independent oscillators: <V> and <x> match the
    classical canonical averages (quadrature) within four standard errors.
    (The Morse plateau makes its classical distribution unnormalisable, so it
    is sampled at k_B T = V0 / 10, where escape over the plateau is negligible.)"""
    V0, d = 1.0, 1.0
    kT = 0.1 if kind == 2 else 0.3
    pot = orc.make_pot(kind, (1.0,), V0=(V0,), d=(d,))
    U = orc.make_units(1.0, 1.0)
    n = 512
    x0 = np.zeros((1, 1, n)) + (0.0 if kind == 2 else d)
    s = orc.Sim(pot, U, n, 1, 1, None, np.zeros(n, np.int32), kT, 1.0, 0.02, 3, 0, 0, 2, x0,
                n_threads=4)
    s.run(2000)
    Vm, Xm = [], []
    for _ in range(40):
        obs = s.run(250, 25)
        Vm.append(np.mean(obs[:, 1]) / n)
        r, _, _, _ = s.state()
        Xm.append(np.mean(r))
    Vm, Xm = np.array(Vm), np.array(Xm)
    lo, hi = (-1.5, 6.0) if kind == 2 else (-3.0, 3.0)
    x = np.linspace(lo, hi, 200001)
    V = (morse_potential if kind == 2 else double_well_potential)(x, V0, d)
    # (2e-3 of the mean allows for the O(dt^2) configurational bias of BAOAB)
    ev = classical_mean(V, V, x, kT)
    se_v = Vm.std(ddof=1) / math.sqrt(len(Vm))
    assert abs(Vm.mean() - ev) < 4 * se_v + 2e-3 * ev, (Vm.mean(), ev, se_v)
    if kind == 2:  # the Morse well is asymmetric: <x> > 0
        ex = classical_mean(V, x, x, kT)
        se_x = Xm.std(ddof=1) / math.sqrt(len(Xm))
        assert ex > 0.05 and abs(Xm.mean() - ex) < 4 * se_x + 2e-3 * ex, (Xm.mean(), ex, se_x)
