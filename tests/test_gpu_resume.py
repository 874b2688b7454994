"""Checkpoint and resume through the state calls (qtb_get_state / qtb_set_state).

The white noise is a function of (seed, stream, step, dof) alone, so the
positions, velocities and step counter are the whole state of a replica: a
context created from a checkpoint continues bit for bit like the context that
took it and set it back (both rebuild the neighbour lists and open a new noise
block at the restored step).  The resumed run also follows the oracle started
from the same checkpoint (FP64 mode), and stays within rounding of a run that
was never interrupted.
"""
import numpy as np
import pytest

from paper_1905_02521_amd import qtb
from tests.gpu_common import crystal, gpu_crystal_ctx, oracle_pair_pot, oracle_units

pytestmark = pytest.mark.gpu


def _ctx(beads, sp, box, prec, fir, noise, vel=None):
    return gpu_crystal_ctx(beads, sp, box, T=100.0, gamma=5e-3, dt=1.0, noise=noise, prec=prec,
                           fir=fir, seed=17, stream=3, max_two_nf=128, obs_every=8, vel=vel,
                           autotune=False)


@pytest.mark.parametrize("prec,fir,P,noise", [(qtb.PREC_FP64, qtb.FIR_FP64, 4, 2),
                                              (qtb.PREC_FP32, qtb.FIR_BF16X3, 1, 1),
                                              (qtb.PREC_FP32, qtb.FIR_BF16X3, 16, 2)])
def test_resume_from_checkpoint_is_bit_exact(orc, prec, fir, P, noise):
    beads, sp, box = crystal(3, P, seed=31, bead_spread=0.02 if P > 1 else 0.0)
    a = _ctx(beads, sp, box, prec, fir, noise)
    a.build_filter(0, noise, 128)
    a.step(96)                      # checkpoint off the 64-step noise-block grid
    r, v, st = a.get_state(0)
    assert st == 96
    a.observables(0)                # drop the samples taken before the checkpoint
    a.set_state(0, r, v, st)
    a.step(140)                     # an eager block, a graph-replayed block, a tail
    b = _ctx(r, sp, box, prec, fir, noise, vel=v)
    b.set_state(0, r, v, st)        # the step counter of the checkpoint
    b.build_filter(0, noise, 128)
    b.step(140)
    ra, va, sa = a.get_state(0)
    rb, vb, sb = b.get_state(0)
    assert sa == sb == 236
    assert np.array_equal(ra, rb) and np.array_equal(va, vb)
    oa, ob = a.observables(0), b.observables(0)
    assert oa["n_samples"] == ob["n_samples"] == 17
    assert oa == ob
    if prec == qtb.PREC_FP64:
        # the oracle started from the checkpoint agrees to the trajectory bar
        osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), beads.shape[2], P, 3,
                       box, sp, 100.0, 5e-3, 1.0, 17, 3, noise, 128, r, vel0=v, step0=st,
                       n_threads=8)
        osim.run(140)
        ro, _, _, so = osim.state()
        assert so == 236
        assert np.sqrt(np.mean((ra - ro) ** 2)) / 0.0421 <= 1e-9
        # and so does the run that was never interrupted, to rounding
        c = _ctx(beads, sp, box, prec, fir, noise)
        c.build_filter(0, noise, 128)
        c.step(236)
        rc, _, _ = c.get_state(0)
        assert np.sqrt(np.mean((ra - rc) ** 2)) / 0.0421 <= 1e-9
