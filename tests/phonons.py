"""Harmonic phonons of the rock-salt supercell, for the closed-form check of
the crystal's energies and heat capacity: the force constants are central
differences of the oracle's brute-force forces at the perfect lattice; the
exact stationary energies of the integrator for those harmonic modes come
from ``closed_forms.ring_mode_moments``.  Test infrastructure only."""
from __future__ import annotations

import numpy as np

from paper_1905_02521_amd import workloads as W
from tests.closed_forms import quantum_heat_capacity, ring_mode_moments
from tests.gpu_common import oracle_pair_pot, oracle_units


def force_constants(orc, n_cells, delta=1e-3):
    """Force-constant matrix Phi [3N][3N] (index = component * N + atom, eV/A^2)
    of the n_cells^3 supercell at the perfect lattice, the static energy and
    the species.  Only the first cation and the first anion are displaced
    (+-delta along x, y, z); every other column follows from the lattice
    translation that carries that reference atom onto the atom of the column
    (every translation of the fcc lattice maps the supercell onto itself)."""
    pos, sp, box = W.rocksalt(n_cells)
    pot, units = oracle_pair_pot(orc), oracle_units(orc, False)
    N = pos.shape[1]
    e0, f0, _ = orc.pair_bruteforce(pot, units, box, sp, pos)
    half = box[0] / (2 * n_cells)
    grid = np.rint(pos / half).astype(np.int64) % (2 * n_cells)
    where = {tuple(g): i for i, g in enumerate(grid.T)}
    Phi = np.zeros((3 * N, 3 * N))
    for ref in (0, 4):                      # first cation, first anion
        col = np.zeros((3, 3, N))           # [alpha][beta][k] = d^2 V / dx_ref,a dx_k,b
        for a in range(3):
            p = pos.copy()
            p[a, ref] += delta
            _, fp, _ = orc.pair_bruteforce(pot, units, box, sp, p)
            p[a, ref] -= 2 * delta
            _, fm, _ = orc.pair_bruteforce(pot, units, box, sp, p)
            col[a] = -(fp - fm) / (2 * delta)
        for j in np.nonzero(sp == sp[ref])[0]:
            shift = grid[:, j] - grid[:, ref]
            src = np.array([where[tuple((grid[:, k] - shift) % (2 * n_cells))]
                            for k in range(N)])
            for a in range(3):
                for b in range(3):
                    Phi[b * N + np.arange(N), a * N + j] = col[a, b, src]
    return 0.5 * (Phi + Phi.T), e0, sp, f0


def normal_mode_frequencies(Phi, sp, mass_amu, mass_unit, zero_tol=1e-8):
    """Angular frequencies (rad/fs) of the mass-weighted dynamical matrix;
    the uniform translations (|omega^2| below zero_tol times the largest)
    are returned as exact zeros."""
    N = len(sp)
    m = np.tile(np.asarray(mass_amu)[sp] * mass_unit, 3)
    D = Phi / np.sqrt(np.outer(m, m))
    w2 = np.linalg.eigvalsh(D)
    w2[np.abs(w2) < zero_tol * w2.max()] = 0.0
    return np.sqrt(np.clip(w2, 0.0, None))


def harmonic_energies(orc, omegas, T, P, gamma, dt, two_nf):
    """Exact stationary energies (eV, relative to the static lattice) of the
    integrator for the harmonic modes at temperature T: QTB noise (eq. 1) for
    P = 1, QTB-PIMD noise (eq. 10-11) for P > 1, the oracle's filter taps."""
    u = W.METAL_UNITS
    units = oracle_units(orc, False)
    taps = orc.taps(1 if P == 1 else 2, T, P, dt, two_nf, units)
    e = ring_mode_moments(omegas, P, u["kB"] * T, u["hbar"], gamma, dt, taps)
    return {k: float(v.sum()) for k, v in e.items()}


def quantum_cv(omegas, T):
    """Exact heat capacity of the quantum harmonic crystal, units of k_B."""
    u = W.METAL_UNITS
    return quantum_heat_capacity(omegas, u["kB"] * T, u["hbar"])
