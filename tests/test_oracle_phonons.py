"""Pins of the harmonic-phonon closed form used against the crystal runs.

* The vectorised stationary moments over many modes equal the one-mode
  closed forms (``ho_energy_discrete`` / ``ho_virial_discrete``) mode by mode.
* The force constants built from two displaced atoms and the lattice's
  translations equal a column computed directly for another atom; they obey
  the acoustic sum rule (a uniform translation exerts no force), which
  leaves exactly three zero modes; a mode's frequency from the eigenvalue
  equals the one from its own finite-difference curvature.
* Heat capacity limits: the quantum harmonic value tends to 3 k_B per atom
  at high temperature and vanishes at low; the integrator's closed form
  with white noise gives k_B per mode at any temperature (the classical
  equipartition the scheme keeps for harmonic modes up to O(dt^2))."""
import math

import numpy as np

from paper_1905_02521_amd import workloads as W
from tests import phonons as ph
from tests.closed_forms import (ho_energy_discrete, ho_virial_discrete, quantum_heat_capacity,
                                ring_mode_moments)
from tests.gpu_common import oracle_pair_pot, oracle_units


def test_vectorised_modes_equal_the_one_mode_closed_form(orc):
    units = orc.make_units(1.0, 1.0, 0.0, 1.0)
    for P, kind in ((1, 1), (3, 2), (4, 2)):
        taps = orc.taps(kind, 0.7, P, 0.05, 256, units)
        om = np.array([0.3, 1.0, 2.5, 7.0])
        e = ring_mode_moments(om, P, 0.7, 1.0, 0.2, 0.05, taps)
        for i, w in enumerate(om):
            E, x2, ke = ho_energy_discrete(w, 1.0, P, 0.7, 1.0, 0.2, 0.05, taps)
            Ev = ho_virial_discrete(w, 1.0, P, 0.7, 1.0, 0.2, 0.05, taps)
            assert abs(e["e_primitive"][i] - E) <= 1e-12 * abs(E)
            assert abs(e["e_virial"][i] - Ev) <= 1e-12 * abs(Ev)
            assert abs(e["kinetic"][i] - ke) <= 1e-12 * ke
            assert abs(e["potential"][i] - 0.5 * w * w * x2) <= 1e-12 * abs(E)


def test_free_mode_kinetic_energy_is_the_velocity_process():
    """omega = 0, P = 1: only the velocity map v' = c1 v + sigma zeta; with
    white noise (one tap) its variance is exactly 1 (sigma^2 = 1 - c1^2)."""
    e = ring_mode_moments(np.array([0.0]), 1, 1.0, 1.0, 0.3, 0.1, np.array([1.0]))
    assert abs(e["kinetic"][0] - 0.5) < 1e-14
    assert e["potential"][0] == 0.0


def test_force_constants_translation_symmetry_and_sum_rule(orc):
    n = 2
    Phi, e0, sp, f0 = ph.force_constants(orc, n)
    N = len(sp)
    assert np.abs(f0).max() < 1e-10            # the perfect lattice is at rest
    # sum rule: sum over the displaced atoms of a component block is zero
    assert np.abs(Phi.reshape(3, N, 3, N).sum(axis=3)).max() < 1e-7 * np.abs(Phi).max()
    # a column computed directly for atom j (an anion away from the reference)
    pos, _, box = W.rocksalt(n)
    pot, units = oracle_pair_pot(orc), oracle_units(orc, False)
    j, d = 13, 1e-3
    assert sp[j] == sp[4]
    for a in range(3):
        p = pos.copy(); p[a, j] += d
        _, fp, _ = orc.pair_bruteforce(pot, units, box, sp, p)
        p[a, j] -= 2 * d
        _, fm, _ = orc.pair_bruteforce(pot, units, box, sp, p)
        direct = (-(fp - fm) / (2 * d)).reshape(-1)
        assert np.abs(direct - Phi[:, a * N + j]).max() < 1e-6 * np.abs(Phi).max()
    om = ph.normal_mode_frequencies(Phi, sp, W.mgo_potential().mass, W.METAL_UNITS["mass_unit"])
    assert int(np.sum(om == 0.0)) == 3


def test_mode_frequency_equals_the_energy_curvature(orc):
    """Displace the perfect lattice along one eigenvector (mass-weighted
    amplitude s): V(s) - V(0) = omega^2 s^2 / 2 to second order; the central
    second difference holds it to 1e-4 (the force constants' own central
    differences and the fourth-order terms are far below that)."""
    n = 2
    Phi, e0, sp, _ = ph.force_constants(orc, n)
    N = len(sp)
    m = np.tile(np.asarray(W.mgo_potential().mass)[sp] * W.METAL_UNITS["mass_unit"], 3)
    w2, vec = np.linalg.eigh(Phi / np.sqrt(np.outer(m, m)))
    pos, _, box = W.rocksalt(n)
    pot, units = oracle_pair_pot(orc), oracle_units(orc, False)
    for q in (5, len(w2) // 2, len(w2) - 1):
        u = (vec[:, q] / np.sqrt(m)).reshape(3, N)
        s = 0.05                  # atom displacements of about 1e-3 A
        ep = orc.pair_bruteforce(pot, units, box, sp, pos + s * u)[0]
        em = orc.pair_bruteforce(pot, units, box, sp, pos - s * u)[0]
        curv = (ep + em - 2 * e0) / (s * s)
        assert abs(curv - w2[q]) <= 1e-4 * w2[q]


def test_heat_capacity_limits():
    om = np.linspace(0.02, 0.19, 600)
    assert abs(quantum_heat_capacity(om, 100.0, 1.0) / len(om) - 1.0) < 1e-5
    assert quantum_heat_capacity(om, 1e-4, 1.0) < 1e-20
    x = 0.7
    assert abs(quantum_heat_capacity(np.array([x]), 1.0, 1.0)
               - (x / 2) ** 2 / math.sinh(x / 2) ** 2) < 1e-15
    # the scheme with white noise: equipartition, no temperature dependence
    # beyond the O(dt^2) shift of the configurational part
    dt = 0.01
    e1 = ring_mode_moments(om, 1, 1.0, 1.0, 0.1, dt, np.array([1.0]))
    e2 = ring_mode_moments(om, 1, 1.1, 1.0, 0.1, dt, np.array([math.sqrt(1.1)]))
    c = (e2["e_primitive"].sum() - e1["e_primitive"].sum()) / 0.1 / len(om)
    assert abs(c - 1.0) < 1e-3
