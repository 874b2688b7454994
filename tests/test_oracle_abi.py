"""The oracle behind the library's call shape (oracle/qtb_oracle_abi.h): the
four calls of the method and state access with the library's argument lists
and structs, host arrays in place of device arrays, so one harness can drive
either back end (the GPU parity test of the same harness is in
tests/test_gpu_parity.py).

* Driven through that shape, the oracle gives bit for bit what its own
  simulation object gives for the same inputs (pair kind, QTB-PIMD P = 2 and
  QTB P = 1 crystals; harmonic oscillators), including the sampled means and
  the caller's state arrays, which it keeps current.
* Set state restarts the replica from the given positions, velocities and
  step, as a checkpoint restore does.
* Status codes: a step before the filter is a state error, a filter length
  that is not a power of two or exceeds the maximum and a replica out of
  range are invalid, a kind the oracle does not integrate is unsupported.
"""
import types

import numpy as np
import pytest

from paper_1905_02521_amd import workloads as W
from tests.gpu_common import oracle_pair_pot, oracle_units


def potd(p):
    return dict(kind=0, mass=p.mass, charge=p.charge, buck_A=p.buck_A, buck_rho=p.buck_rho,
                buck_C=p.buck_C, dsf_alpha=p.dsf_alpha, r_cut=p.r_cut, skin=p.skin)


def replica(pos, sp, box, T, noise, seed, stream, vel=None, omega=None, gamma=5e-3, dt=1.0):
    return types.SimpleNamespace(pos=pos, vel=vel, species=sp, T=T, gamma=gamma, dt=dt,
                                 noise=noise, box=box, seed=seed, stream=stream,
                                 harm_omega=omega)


def crystal(n, P, seed):
    pos, sp, box = W.rocksalt(n)
    base = W.displaced(pos, 0.0421, seed)
    beads = np.stack([base if P == 1 else W.displaced(base, 0.02, seed + 10 + b)
                      for b in range(P)])
    return beads, sp, box


def test_crystal_through_the_call_shape_equals_the_simulation(orc):
    pot = W.mgo_potential()
    specs = [(2, 2, 100.0, 3), (2, 1, 300.0, 1)]   # (cells, P, T, noise seed)
    reps, inputs = [], []
    for k, (n, P, T, seed) in enumerate(specs):
        beads, sp, box = crystal(n, P, 40 + k)
        inputs.append((beads, sp, box))
        reps.append(replica(beads, sp, box, T, 2 if P > 1 else 1, seed, k))
    ctx = orc.AbiContext(potd(pot), reps, dict(W.METAL_UNITS), obs_every=4, max_two_nf=256)
    for k, (_, P, _, _) in enumerate(specs):
        taps = ctx.build_filter(k, 2 if P > 1 else 1, 128)
        assert taps.shape == (128,)
    ctx.step(24)
    ctx.step(16)
    for k, ((n, P, T, seed), (beads, sp, box)) in enumerate(zip(specs, inputs)):
        sim = orc.Sim(oracle_pair_pot(orc, pot), oracle_units(orc, False), beads.shape[2], P, 3,
                      box, sp, T, 5e-3, 1.0, seed, k, 2 if P > 1 else 1, 128, beads,
                      n_threads=8)
        o1 = sim.run(24, 4)
        o2 = sim.run(16, 4)
        ro, vo, _, so = sim.state()
        r, v, st = ctx.get_state(k)
        assert st == so == 40
        assert np.array_equal(r, ro) and np.array_equal(v, vo)
        # the caller's own arrays are kept current
        assert np.array_equal(ctx.state[k][0], ro)
        g = ctx.observables(k)
        o = np.concatenate([o1, o2])
        assert g["n_samples"] == len(o) == 10
        for f in ("kinetic", "potential", "spring", "e_primitive", "e_virial", "t_kinetic",
                  "x2_mean", "pressure"):
            j = orc.OBS_NAMES.index(f)
            assert g[f] == pytest.approx(o[:, j].mean(), rel=1e-13, abs=1e-15), f
        assert g["volume"] == pytest.approx(np.prod(box), rel=1e-14)
        assert ctx.observables(k)["n_samples"] == 0   # the means were consumed
    ctx.close()


def test_oscillators_and_set_state(orc):
    n = 32
    om = 0.2 * 100.0 ** (np.arange(n) / (n - 1))
    pos = np.zeros((1, 1, n))
    units = dict(W.REDUCED_UNITS)
    rep = replica(pos, np.zeros(n, np.int32), None, 1.0, 1, 5, 0, omega=om, gamma=1.0,
                  dt=0.01)
    ctx = orc.AbiContext(dict(kind=1, mass=(1.0,)), [rep], units, obs_every=8)
    ctx.build_filter(0, 1, 256)
    ctx.step(100)
    r, v, st = ctx.get_state(0)
    sim = orc.Sim(orc.make_pot(1, (1.0,)), orc.make_units(**units), n, 1, 1, None,
                  np.zeros(n, np.int32), 1.0, 1.0, 0.01, 5, 0, 1, 256, pos, harm_omega=om,
                  n_threads=4)
    sim.run(100)
    ro, vo, _, so = sim.state()
    assert st == so == 100 and np.array_equal(r, ro) and np.array_equal(v, vo)
    # restart from a checkpoint: the same continuation as a fresh simulation from it
    ctx.set_state(0, r, v, st)
    ctx.step(50)
    r2, v2, st2 = ctx.get_state(0)
    sim2 = orc.Sim(orc.make_pot(1, (1.0,)), orc.make_units(**units), n, 1, 1, None,
                   np.zeros(n, np.int32), 1.0, 1.0, 0.01, 5, 0, 1, 256, r, vel0=v, step0=st,
                   harm_omega=om, n_threads=4)
    sim2.run(50)
    ro2, vo2, _, so2 = sim2.state()
    assert st2 == so2 == 150 and np.array_equal(r2, ro2) and np.array_equal(v2, vo2)
    ctx.close()


def test_status_codes(orc):
    pot = W.mgo_potential()
    beads, sp, box = crystal(2, 1, 7)
    ctx = orc.AbiContext(potd(pot), [replica(beads, sp, box, 100.0, 1, 1, 0)],
                         dict(W.METAL_UNITS), max_two_nf=256)
    with pytest.raises(orc.AbiError) as e:
        ctx.step(1)
    assert e.value.status == 4            # step before the filter
    for two_nf in (100, 512):
        with pytest.raises(orc.AbiError) as e:
            ctx.build_filter(0, 1, two_nf)
        assert e.value.status == 1
    with pytest.raises(orc.AbiError) as e:
        ctx.build_filter(3, 1, 128)
    assert e.value.status == 1
    ctx.close()
    with pytest.raises(orc.AbiError) as e:   # an on-site kind the oracle shape leaves out
        orc.AbiContext(dict(kind=2, mass=(1.0,)), [replica(beads, sp, box, 100.0, 1, 1, 0)],
                       dict(W.METAL_UNITS))
    assert e.value.status == 6
