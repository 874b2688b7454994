"""Write the oracle's thermodynamic reference for the ring-polymer statistical
parity test (the PIMD P = 32 reference of the QTB-PIMD comparison).

Runs only the FP64 oracle (and the seeded input generators) on a 4x4x4 MgO
rock-salt crystal (512 atoms) at 50 K:

* PIMD (white noise on every normal mode, P = 32);
* QTB-PIMD (eq. 10-12 noise, P = 8).

Each run starts from the same displaced lattice (2 % of d_nn, seed 5) with all
beads on the atom, discards an equilibration stretch, then stores block means
of the eq. 5 observables sampled every ``EVERY`` steps.  The GPU test runs the
same systems with other noise seeds and compares the means within combined
standard errors.

    python tests/golden/make_thermo_pimd32.py      # about forty minutes on 8 threads
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "thermo_mgo_4x4x4_pimd.json")

SETTINGS = dict(n_cells=4, sigma=0.0421, pos_seed=5, T=50.0, gamma=1e-2, dt=1.0, two_nf=512,
                noise_seed=11, every=8, block=400, n_eq=2000, n_blocks=40)
RUNS = [dict(P=32, noise=0), dict(P=8, noise=2)]
FIELDS = ("kinetic", "potential", "spring", "e_primitive", "e_virial", "x2_mean")


def oracle_run(run, n_threads=8):
    s = SETTINGS
    p = W.mgo_potential()
    pot = orc.make_pot(0, p.mass, p.charge, p.buck_A, p.buck_rho, p.buck_C, p.dsf_alpha,
                       p.r_cut, p.skin)
    units = orc.make_units(**W.METAL_UNITS)
    pos, sp, box = W.rocksalt(s["n_cells"])
    beads = W.beads_from(W.displaced(pos, s["sigma"], s["pos_seed"]), run["P"])
    sim = orc.Sim(pot, units, len(sp), run["P"], 3, box, sp, s["T"], s["gamma"], s["dt"],
                  s["noise_seed"], 0, run["noise"], s["two_nf"], beads, n_threads=n_threads)
    sim.run(s["n_eq"])
    blocks = {f: [] for f in FIELDS}
    for b in range(s["n_blocks"]):
        obs = sim.run(s["block"], s["every"])
        for f in FIELDS:
            blocks[f].append(float(np.mean(obs[:, orc.OBS_NAMES.index(f)])))
        if b % 8 == 7:
            print(f"  P={run['P']}: block {b + 1}/{s['n_blocks']}", flush=True)
    return blocks


def main():
    out = dict(settings=SETTINGS, fields=FIELDS, runs=[])
    for run in RUNS:
        t0 = time.time()
        blocks = oracle_run(run)
        e = np.array(blocks["e_primitive"])
        print(f"P={run['P']} noise={run['noise']}: <E_prim> = {e.mean():.4f} +- "
              f"{e.std(ddof=1) / np.sqrt(len(e)):.4f} eV ({time.time() - t0:.0f} s)", flush=True)
        out["runs"].append(dict(run, blocks=blocks))
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
