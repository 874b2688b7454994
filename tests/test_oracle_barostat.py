"""Pin of the oracle's isotropic stochastic cell rescaling (the barostat of
the constant-pressure runs behind Fig. 6): for an ideal gas the isothermal-
isobaric ensemble has p(V) ~ V^N exp(-P0 V / k_B T), so <V> = (N + 1) k_B T / P0
and Var V / <V>^2 = 1 / (N + 1)."""
import math

import numpy as np

from tests.gpu_common import oracle_units


def test_ideal_gas_volume_distribution(orc):
    N, T = 64, 300.0
    U = oracle_units(orc, False)
    kT = U.kB * T
    V_target = 12.0 ** 3
    P0 = (N + 1) * kT / V_target
    pot = orc.make_pot(0, (1.0,), (0.0,), None, None, None, 0.0, 3.0, 0.5)
    rng = np.random.default_rng(2)
    L0 = 11.0
    pos = rng.uniform(0, L0, (1, 3, N))
    sim = orc.Sim(pot, U, N, 1, 3, (L0, L0, L0), np.zeros(N, np.int32), T, 0.05, 2.0, 9, 0, 0, 2,
                  pos, n_threads=4)
    sim.set_barostat(P0, 100.0, 1.0 / P0)
    sim.run(2000)
    vols = []
    for _ in range(400):
        sim.run(50)
        vols.append(np.prod(sim.box()))
    vols = np.array(vols)
    # samples 100 fs apart (one relaxation time): blocks of 10 for the error
    blk = vols.reshape(40, 10).mean(axis=1)
    m, se = blk.mean(), blk.std(ddof=1) / math.sqrt(len(blk))
    print(f"<V> = {m:.1f} +- {se:.1f} A^3 (exact {V_target:.1f}); "
          f"sd/mean {vols.std() / vols.mean():.3f} (exact {1 / math.sqrt(N + 1):.3f})")
    assert abs(m - V_target) < 4 * se
    assert abs(vols.std() / vols.mean() * math.sqrt(N + 1) - 1) < 0.25
