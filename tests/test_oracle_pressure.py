"""Pins of the oracle's pressure (pair potential): the pair virial and the
primitive ring-polymer estimator p = (2K - 2 U_spring + (1/P) sum_s W_s) / (3V).

* The pair virial W = sum over pairs of F(r) r is minus the derivative of the
  potential energy under a uniform scaling of positions and box (brute force
  over images, central differences), and equals the trace of the
  brute-force virial tensor.
* A gas of non-interacting particles has p = N k_B T / V for classical
  Langevin dynamics (P = 1) and for classical PIMD (P = 4): the ring's spring
  term must cancel the extra kinetic energy of the beads exactly.
"""
import math

import numpy as np
import pytest

from paper_1905_02521_amd import workloads as W
from tests.gpu_common import crystal, oracle_pair_pot, oracle_units


def test_pair_virial_is_minus_volume_derivative(orc):
    beads, sp, box = crystal(3, 1, seed=4)
    pos = beads[0]
    pot = oracle_pair_pot(orc)
    U = oracle_units(orc, False)
    sim = orc.Sim(pot, U, pos.shape[1], 1, 3, box, sp, 100.0, 0.0, 1.0, 1, 0, 0, 2, beads,
                  n_threads=8)
    o = sim.observe()
    Wsim = o[orc.OBS_NAMES.index("virial_pair")]
    h = 1e-5
    box = np.asarray(box, dtype=np.float64)
    up = orc.pair_bruteforce(pot, U, box * (1 + h), sp, pos * (1 + h))[0]
    um = orc.pair_bruteforce(pot, U, box * (1 - h), sp, pos * (1 - h))[0]
    W_fd = -(up - um) / (2 * h)
    _, _, vir = orc.pair_bruteforce(pot, U, box, sp, pos)
    print(f"W sim {Wsim:.8f}, -dU/ds {W_fd:.8f}, trace {np.trace(vir):.8f}")
    assert abs(Wsim - W_fd) < 1e-7 * abs(W_fd) + 1e-6
    assert abs(Wsim - np.trace(vir)) < 1e-9 * abs(Wsim)
    # the static pressure of the compressed (displaced) lattice
    p = o[orc.OBS_NAMES.index("pressure")]
    assert abs(p - Wsim / (3 * np.prod(box))) < 1e-12 * abs(p)   # K = 0 at rest


@pytest.mark.parametrize("P", [1, 4])
def test_ideal_gas_pressure(orc, P):
    """64 non-interacting particles (no charges, no Buckingham) in a 12 A box,
    k_B T = 300 K, white noise, gamma = 0.05/fs: <p> V / (N k_B T) = 1 within
    four standard errors of 40 block means."""
    N, L, T = 64, 12.0, 300.0
    pot = orc.make_pot(0, (1.0,), (0.0,), None, None, None, 0.0, 3.0, 0.5)
    U = oracle_units(orc, False)
    rng = np.random.default_rng(3)
    pos = np.broadcast_to(rng.uniform(0, L, (1, 3, N)), (P, 3, N)).copy()
    sim = orc.Sim(pot, U, N, P, 3, (L, L, L), np.zeros(N, np.int32), T, 0.05, 2.0, 5, 0, 0, 2,
                  pos, n_threads=4)
    sim.run(500)
    blocks = []
    ip = orc.OBS_NAMES.index("pressure")
    for _ in range(40):
        obs = sim.run(200, 10)
        blocks.append(np.mean(obs[:, ip]))
    blocks = np.array(blocks) * L ** 3 / (N * U.kB * T)
    m, se = blocks.mean(), blocks.std(ddof=1) / math.sqrt(len(blocks))
    print(f"P={P}: p V / N k_B T = {m:.4f} +- {se:.4f}")
    assert abs(m - 1.0) < 4 * se
    assert se < 0.03
