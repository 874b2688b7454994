"""Write the oracle's thermodynamic reference for the statistical parity tests.

Runs only the FP64 oracle (and the seeded input generators) on a 3x3x3 MgO
rock-salt crystal (216 atoms, the smallest size of the batched sweep):

* QTB (eq. 6-7 noise, P = 1) at T = 50, 100, 200, 400 K;
* QTB-PIMD (eq. 10-12 noise, P = 4, normal-mode propagation) at 100 and 200 K.

Each run starts from the same displaced lattice (2 % of d_nn, seed 5) at rest,
discards an equilibration stretch, then stores block means of the eq. 5
observables (primitive energy with instantaneous momenta, kinetic, potential,
centroid-virial energy, kinetic temperature), sampled every ``EVERY`` steps.
The GPU test runs the same systems with another noise seed and compares means
and the heat capacity C = dE/dT from the temperature ladder, within two
combined standard errors of the block means.

    python tests/golden/make_thermo.py      # about fifteen minutes on 8 threads
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_1905_02521_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "thermo_mgo_3x3x3.json")

SETTINGS = dict(n_cells=3, sigma=0.0421, pos_seed=5, gamma=1e-2, dt=1.0, two_nf=512,
                noise_seed=11, every=8, block=1000, n_eq=3000)
RUNS = [dict(P=1, noise=1, T=T, n_blocks=48) for T in (50.0, 100.0, 200.0, 400.0)] + \
       [dict(P=4, noise=2, T=T, n_blocks=48) for T in (100.0, 200.0)]
FIELDS = ("kinetic", "potential", "e_primitive", "e_virial", "t_kinetic")


def oracle_run(run, n_threads=8):
    s = SETTINGS
    p = W.mgo_potential()
    pot = orc.make_pot(0, p.mass, p.charge, p.buck_A, p.buck_rho, p.buck_C, p.dsf_alpha,
                       p.r_cut, p.skin)
    units = orc.make_units(**W.METAL_UNITS)
    pos, sp, box = W.rocksalt(s["n_cells"])
    beads = W.beads_from(W.displaced(pos, s["sigma"], s["pos_seed"]), run["P"])
    sim = orc.Sim(pot, units, len(sp), run["P"], 3, box, sp, run["T"], s["gamma"], s["dt"],
                  s["noise_seed"], 0, run["noise"], s["two_nf"], beads, n_threads=n_threads)
    sim.run(s["n_eq"])
    blocks = {f: [] for f in FIELDS}
    for _ in range(run["n_blocks"]):
        obs = sim.run(s["block"], s["every"])
        for f in FIELDS:
            blocks[f].append(float(np.mean(obs[:, orc.OBS_NAMES.index(f)])))
    return blocks


def main():
    out = dict(settings=SETTINGS, fields=FIELDS, runs=[])
    for run in RUNS:
        t0 = time.time()
        blocks = oracle_run(run)
        e = np.array(blocks["e_primitive"])
        print(f"P={run['P']} T={run['T']}: <E> = {e.mean():.4f} +- "
              f"{e.std(ddof=1) / np.sqrt(len(e)):.4f} eV ({time.time() - t0:.0f} s)", flush=True)
        out["runs"].append(dict(run, blocks=blocks))
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
