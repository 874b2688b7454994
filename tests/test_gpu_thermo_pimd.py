"""Statistical parity of the ring-polymer runs that the QTB-PIMD comparison
rests on: a 4x4x4 MgO crystal at 50 K as plain PIMD with P = 32 (white noise
on every normal mode, the converged reference) and as QTB-PIMD with P = 8
(eq. 10-12 noise), the GPU in its production precision (FP32 forces, BF16x3
FIR) against the FP64 oracle's runs stored by
``tests/golden/make_thermo_pimd32.py``.

Each GPU run uses a noise seed of its own (two seeds, both systems of a seed
in one batched context), discards the same equilibration and samples four
times as long as the oracle; standard errors by blocking
(Flyvbjerg-Petersen) on both sides.  For the eq. 5 observables (kinetic,
potential, spring, primitive and centroid-virial energy) z = (gpu - oracle) /
sqrt(se_gpu^2 + se_oracle^2); a single comparison lies within 2 sigma with
probability 0.95 only, so each seed's family of ten is bounded as a family:
every |z| below the Bonferroni bound of a 1 % family-wise error (3.29) and
at least 7 of 10 within 2 sigma; the two seeds pooled put both primitive
energies within the same bound for two comparisons (2.81)."""
import json
import math
import os

import numpy as np
import pytest

from paper_1905_02521_amd import qtb, workloads as W
from paper_1905_02521_amd.stats import mean_and_error

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "thermo_mgo_4x4x4_pimd.json")
FIELDS = ("kinetic", "potential", "spring", "e_primitive", "e_virial")
SEEDS = (12, 13)
Z_BONF = 3.29     # |z| bound: 1 % family-wise over ten comparisons
Z_BONF2 = 2.81    # the same over two


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def gpu_runs(gold):
    """Per seed, per run: the window means of every field."""
    s = gold["settings"]
    pos, sp, box = W.rocksalt(s["n_cells"])
    base = W.displaced(pos, s["sigma"], s["pos_seed"])
    out = {}
    for seed in SEEDS:
        reps = [qtb.Replica(pos=W.beads_from(base, r["P"]), species=sp, T=s["T"],
                            gamma=s["gamma"], dt=s["dt"], noise=r["noise"], box=tuple(box),
                            seed=seed, stream=k) for k, r in enumerate(gold["runs"])]
        ctx = qtb.Context(qtb.pair_potential_dict(W.mgo_potential()), reps, dict(W.METAL_UNITS),
                          prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3, obs_every=s["every"],
                          max_two_nf=s["two_nf"])
        for k, r in enumerate(gold["runs"]):
            if r["noise"]:
                ctx.build_filter(k, r["noise"], s["two_nf"])
        ctx.step(s["n_eq"])
        for k in range(len(reps)):
            ctx.observables(k)
        win = {k: {f: [] for f in FIELDS} for k in range(len(reps))}
        n_win = 4 * s["n_blocks"] * s["block"] // 128
        for _ in range(n_win):
            ctx.step(128)
            for k in range(len(reps)):
                o = ctx.observables(k)
                for f in FIELDS:
                    win[k][f].append(o[f])
        ctx.close()
        out[seed] = win
    return out


def _z(gold, gpu_runs, seed):
    zs = []
    for k, r in enumerate(gold["runs"]):
        for f in FIELDS:
            mg, sg = mean_and_error(gpu_runs[seed][k][f])
            mo, so = mean_and_error(r["blocks"][f])
            z = (mg - mo) / math.hypot(sg, so)
            print(f"seed {seed} P={r['P']} noise={r['noise']} {f}: gpu {mg:.4f} +- {sg:.4f}, "
                  f"oracle {mo:.4f} +- {so:.4f} eV, z = {z:+.2f}")
            zs.append((r["P"], f, z))
    return zs


@pytest.mark.parametrize("seed", SEEDS)
def test_ring_polymer_means_match_oracle(gold, gpu_runs, seed):
    zs = _z(gold, gpu_runs, seed)
    assert all(abs(z) < Z_BONF for _, _, z in zs), zs
    assert sum(abs(z) < 2.0 for _, _, z in zs) >= 7, zs


def test_primitive_energy_pooled_over_seeds(gold, gpu_runs):
    for k, r in enumerate(gold["runs"]):
        pooled = np.concatenate([gpu_runs[seed][k]["e_primitive"] for seed in SEEDS])
        mg = float(np.mean(pooled))
        sg = math.hypot(*[mean_and_error(gpu_runs[seed][k]["e_primitive"])[1] for seed in SEEDS]) / 2
        mo, so = mean_and_error(r["blocks"]["e_primitive"])
        z = (mg - mo) / math.hypot(sg, so)
        print(f"pooled P={r['P']}: gpu {mg:.4f} +- {sg:.4f}, oracle {mo:.4f} +- {so:.4f}, z = {z:+.2f}")
        assert abs(z) < Z_BONF2, (r["P"], z)
