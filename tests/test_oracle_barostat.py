"""Pins of the oracle's isotropic barostats (the isothermal-isobaric
extension of Sec. 2.1 behind the constant-pressure lattice parameters of
Fig. 6): stochastic cell rescaling and the Langevin piston, for classical
particles (P = 1) and ring polymers (P = 4, every bead coordinate scaled,
the ring-polymer pressure with its spring term).

* Ideal gas: the ring polymers' internal modes do not depend on the volume,
  so for any P the isothermal-isobaric ensemble has p(V) ~ V^N
  exp(-P0 V / k_B T): <V> = (N + 1) k_B T / P0 and Var V / <V>^2 = 1 / (N + 1).
* At T = 0 cell rescaling of a perfect lattice is the deterministic Euler map
  of ln V with the pressure from the brute-force virial tensor.
* Without friction on the particles and the piston, the piston dynamics
  conserves H + P0 V + p_e^2 / 2 W_p up to the splitting's O(dt^2) error,
  with no drift.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import oracle_units


def ideal_gas(orc, P, kind, seed=9):
    N, T = 64, 300.0
    U = oracle_units(orc, False)
    kT = U.kB * T
    V_target = 12.0 ** 3
    P0 = (N + 1) * kT / V_target
    pot = orc.make_pot(0, (1.0,), (0.0,), None, None, None, 0.0, 3.0, 0.5)
    rng = np.random.default_rng(2)
    L0 = 11.0
    x = rng.uniform(0, L0, (1, 3, N))
    pos = np.repeat(x, P, axis=0) + (rng.normal(0, 0.05, (P, 3, N)) if P > 1 else 0.0)
    sim = orc.Sim(pot, U, N, P, 3, (L0, L0, L0), np.zeros(N, np.int32), T, 0.05, 2.0, seed, 0, 0,
                  2, pos, n_threads=4)
    if kind == "rescale":
        sim.set_barostat(P0, 100.0, 1.0 / P0)
    else:
        sim.set_piston(P0, 100.0, 0.01)
    return sim, N, V_target


@pytest.mark.parametrize("P,kind", [(1, "rescale"), (4, "rescale"), (1, "piston"), (4, "piston")])
def test_ideal_gas_volume_distribution(orc, P, kind):
    sim, N, V_target = ideal_gas(orc, P, kind)
    sim.run(2000)
    vols = []
    for _ in range(400):
        sim.run(50)
        vols.append(np.prod(sim.box()))
    vols = np.array(vols)
    # samples 100 fs apart (about one relaxation time): blocks of 10 for the error
    blk = vols.reshape(40, 10).mean(axis=1)
    m, se = blk.mean(), blk.std(ddof=1) / math.sqrt(len(blk))
    print(f"P={P} {kind}: <V> = {m:.1f} +- {se:.1f} A^3 (exact {V_target:.1f}); "
          f"sd/mean {vols.std() / vols.mean():.3f} (exact {1 / math.sqrt(N + 1):.3f})")
    assert abs(m - V_target) < 4 * se
    assert abs(vols.std() / vols.mean() * math.sqrt(N + 1) - 1) < 0.25


def test_piston_conserves_extended_energy_without_friction(orc):
    """gamma = gamma_p = 0 (white-noise kind, no noise then): the particles
    and the piston exchange energy through the coupling, and
    H + P0 V + p_e^2 / (2 W_p) stays constant to a small fraction of the
    kinetic energy's fluctuation over 2000 steps (the symmetric splitting
    leaves no drift), while the volume moves."""
    N, T, P = 64, 300.0, 4
    U = oracle_units(orc, False)
    kT = U.kB * T
    P0 = (N + 1) * kT / 12.0 ** 3
    pot = orc.make_pot(0, (1.0,), (0.0,), None, None, None, 0.0, 3.0, 0.5)
    rng = np.random.default_rng(3)
    L0, tau = 11.0, 100.0
    x = rng.uniform(0, L0, (1, 3, N))
    pos = np.repeat(x, P, axis=0) + rng.normal(0, 0.05, (P, 3, N))
    vel = rng.normal(0, math.sqrt(kT / (1.0 * U.mass_unit)), (P, 3, N))
    sim = orc.Sim(pot, U, N, P, 3, (L0, L0, L0), np.zeros(N, np.int32), T, 0.0, 0.5, 4, 0, 0, 2,
                  pos, vel0=vel, n_threads=4)
    sim.set_piston(P0, tau, 0.0)
    W = (3 * N * P + 3) * kT * tau * tau

    def H():
        return sim.hamiltonian() + P0 * np.prod(sim.box()) + sim.piston_momentum() ** 2 / (2 * W)
    H0, V0 = H(), np.prod(sim.box())
    hs, vs = [], []
    for _ in range(40):
        sim.run(50)
        hs.append(H())
        vs.append(np.prod(sim.box()))
    dK = math.sqrt(1.5 * N * P) * kT   # fluctuation scale of the kinetic energy
    dev = np.abs(np.array(hs) - H0) / dK
    print(f"largest deviation {dev.max():.4f} dK, last {dev[-1]:.4f} dK")
    assert dev.max() < 0.01, dev
    assert np.max(np.abs(np.array(vs) / V0 - 1)) > 0.02   # the box did move


def test_zero_temperature_relaxation_is_the_euler_map(orc):
    """At T = 0 the noise vanishes and a perfect rock-salt lattice stays
    perfect (its forces cancel by symmetry, the velocities stay zero), so the
    box follows the deterministic map L_{n+1} = L_n exp(-(beta_T / tau_p)
    (P0 - W(L_n) / (3 L_n^3)) dt / 3), with the pair virial W taken here from
    the trace of the brute-force virial tensor of the scaled lattice.  The
    oracle's box must follow that map step by step: the sign of the drift,
    the 1/3 of the length scale and the pressure's virial term all enter."""
    from paper_1905_02521_amd import workloads as W
    from tests.gpu_common import oracle_pair_pot
    pos, sp, box = W.rocksalt(3, 4.21)
    U = oracle_units(orc, False)
    pot = oracle_pair_pot(orc)
    P0, tau, beta, dt = 0.01, 20.0, 0.5, 1.0
    sim = orc.Sim(pot, U, pos.shape[1], 1, 3, box, sp, 0.0, 1e-3, dt, 3, 0, 0, 2, pos[None],
                  n_threads=8)
    sim.set_barostat(P0, tau, beta)
    L = float(box[0])
    for _ in range(12):
        s = L / box[0]
        _, _, vir = orc.pair_bruteforce(pot, U, np.asarray(box) * s, sp, pos * s)
        p = np.trace(vir) / (3 * L ** 3)
        L *= math.exp(-(beta / tau) * (P0 - p) * dt / 3.0)
        sim.run(1)
        # between steps the box is still the one of the positions; the
        # update's factor is pending for the next step
        b = sim.box() * sim.barostat_state()[1]
        assert abs(b[0] - L) <= 1e-12 * L, (b[0], L)
    r, v, _, _ = sim.state()
    assert np.max(np.abs(v)) < 1e-9
    print(f"box after 12 steps: {L:.10f} (start {box[0]:.4f}), static pressure {p:.5f} eV/A^3")
    assert abs(L / box[0] - 1) > 1e-4   # the lattice did relax
