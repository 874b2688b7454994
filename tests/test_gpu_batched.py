"""Batched replicas: many replicas of uneven size, bead number, temperature,
friction and noise kind step together (one launch per kernel covering all
of them, one graph per noise block).  Each replica must evolve exactly as it
does alone, and as the oracle says."""
import numpy as np
import pytest

from paper_1905_02521_amd import qtb, workloads as W
from tests.gpu_common import oracle_pair_pot, oracle_units, units_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def replica_specs():
    # (cells, P, T, gamma, noise, two_nf, stream)
    return [(2, 1, 300.0, 1e-3, 1, 128, 0), (3, 4, 50.0, 5e-3, 2, 256, 1),
            (2, 8, 80.0, 2e-2, 2, 128, 2), (3, 3, 120.0, 1e-3, 0, 2, 3),
            (2, 2, 20.0, 5e-4, 2, 256, 4)]


def make_reps(specs, seed=5):
    reps = []
    for k, (n, P, T, g, noise, two_nf, stream) in enumerate(specs):
        pos, sp, box = W.rocksalt(n)
        beads = np.stack([W.displaced(pos, 0.03, 100 * k + b) for b in range(P)])
        reps.append((qtb.Replica(pos=beads, species=sp, T=T, gamma=g, dt=1.0, noise=noise,
                                 box=tuple(box), seed=seed, stream=stream), two_nf))
    return reps


def ctx_for(reps, prec, fir, autotune=False, obs_every=0, fuse=False):
    p = W.mgo_potential(skin=0.5)
    c = qtb.Context(qtb.pair_potential_dict(p), [r for r, _ in reps], units_dict(False),
                    prec=prec, fir=fir, fir_block_K=64, obs_every=obs_every,
                    max_two_nf=max(t for _, t in reps), autotune=autotune, fuse=fuse)
    for k, (r, t) in enumerate(reps):
        if r.noise:
            c.build_filter(k, r.noise, t)
    return c


@pytest.mark.parametrize("prec,fir", [(qtb.PREC_FP64, qtb.FIR_FP64),
                                      (qtb.PREC_FP32, qtb.FIR_BF16X3)])
def test_batched_equals_each_replica_alone(prec, fir):
    reps = make_reps(replica_specs())
    batch = ctx_for(reps, prec, fir)
    batch.step(150)
    for k, rep in enumerate(reps):
        alone = ctx_for([rep], prec, fir)
        alone.step(150)
        rb, vb, sb = batch.get_state(k)
        ra, va, sa = alone.get_state(0)
        assert sb == sa == 150
        assert np.array_equal(rb, ra) and np.array_equal(vb, va), k
        alone.close()


def test_batched_matches_oracle(orc):
    reps = make_reps(replica_specs()[:4])
    batch = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, autotune=True)
    batch.step(12)
    U = oracle_units(orc, False)
    pot = oracle_pair_pot(orc, W.mgo_potential(skin=0.5))
    for k, (r, two_nf) in enumerate(reps):
        P, _, N = r.pos.shape
        s = orc.Sim(pot, U, N, P, 3, r.box, r.species, r.T, r.gamma, r.dt, r.seed, r.stream,
                    r.noise, two_nf, r.pos, n_threads=8)
        s.run(12)
        ro, _, _, _ = s.state()
        rb, _, _ = batch.get_state(k)
        assert np.sqrt(np.mean((rb - ro) ** 2)) / 0.03 < 1e-9, k


def test_autotuner_changes_only_rounding():
    reps = make_reps(replica_specs()[:3])
    a = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, autotune=True)
    b = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, autotune=False)
    a.step(20)
    b.step(20)
    for k in range(3):
        ra, _, _ = a.get_state(k)
        rb, _, _ = b.get_state(k)
        assert np.max(np.abs(ra - rb)) < 1e-10


def test_batched_observables_per_replica():
    reps = make_reps(replica_specs())
    c = ctx_for(reps, qtb.PREC_FP32, qtb.FIR_BF16X3, obs_every=8)
    c.step(64)
    for k, (r, _) in enumerate(reps):
        o = c.observables(k)
        P, _, N = r.pos.shape
        assert o["n_samples"] == 8
        assert np.isfinite(o["e_primitive"])
        # kinetic temperature of the beads is of the order of T after 64 fs
        assert 0.0 < o["t_kinetic"] < 20 * r.T


def test_mixed_decompositions_per_bead_group():
    """One launch per bead-group width, each with its own decomposition
    (what the autotuner may choose): the FP64 trajectories and the
    observables of every replica equal those of one uniform decomposition
    to the rounding of the sums' order, and the pinned mix reads back."""
    specs = [(2, 1, 300.0, 1e-3, 1, 128, 0), (3, 4, 50.0, 5e-3, 2, 256, 1),
             (2, 8, 80.0, 2e-2, 2, 128, 2), (2, 2, 20.0, 5e-4, 2, 256, 4)]
    reps = make_reps(specs)
    mix = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, obs_every=4)
    for G, W_, half in ((1, 4, False), (2, 2, True), (4, 1, True), (8, 2, False)):
        mix.set_group_decomposition(G, W_, half)
    assert [mix.group_decomposition(G) for G in (1, 2, 4, 8)] == \
        [(4, False), (2, True), (1, True), (2, False)]
    uni = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, obs_every=4)
    uni.set_decomposition(1, False)
    mix.step(40)
    uni.step(40)
    for k in range(len(reps)):
        rm, vm, _ = mix.get_state(k)
        ru, vu, _ = uni.get_state(k)
        assert np.max(np.abs(rm - ru)) < 1e-10, k
        om, ou = mix.observables(k), uni.observables(k)
        assert om["n_samples"] == ou["n_samples"] == 10
        for f in ("kinetic", "potential", "e_primitive", "e_virial"):
            assert abs(om[f] - ou[f]) <= 1e-9 * max(1.0, abs(ou[f])), (k, f)
    with pytest.raises(qtb.QtbError):
        mix.set_group_decomposition(3, 1, False)
    mix.close()
    uni.close()


def test_replica_skins_change_only_the_lists():
    """Per-replica list skins (thin ones rebuild often): the same FP64
    trajectories as the potential's skin everywhere, to the rounding of the
    sums' order; skins outside [0, the potential's skin] are rejected."""
    reps = make_reps(replica_specs()[:4])
    a = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, obs_every=4)
    b = ctx_for(reps, qtb.PREC_FP64, qtb.FIR_FP64, obs_every=4)
    for c in (a, b):
        c.set_decomposition(1, False)
    a.step(16)
    b.step(16)
    for r, sk in enumerate((0.05, 0.2, 0.5, 0.35)):   # potential skin 0.5
        a.set_replica_skin(r, sk)
    a.step(60)
    b.step(60)
    for k in range(4):
        ra, va, sa = a.get_state(k)
        rb, vb, sb = b.get_state(k)
        assert sa == sb == 76
        assert np.max(np.abs(ra - rb)) < 1e-10 and np.max(np.abs(va - vb)) < 1e-10, k
        oa, ob = a.observables(k), b.observables(k)
        for f in ("potential", "e_primitive", "e_virial"):
            assert abs(oa[f] - ob[f]) <= 1e-9 * max(1.0, abs(ob[f])), (k, f)
    a.set_replica_skin(-1, 0.5)
    for bad in (0.51, -0.1, float("nan")):
        with pytest.raises(qtb.QtbError):
            a.set_replica_skin(0, bad)
    with pytest.raises(qtb.QtbError):
        a.set_replica_skin(4, 0.2)
    a.close()
    b.close()
