"""Positions written into a context's device arrays in place and taken with
``Context.set_positions`` (``qtb_set_state`` with null host arrays: every
list rebuilt and every force recomputed).  Two replicas of different size and
bead count; one fixed force decomposition everywhere, so that every context
sums each force in the same order.

* Against the same context history reloaded from host arrays: the same
  trajectory, bit for bit.
* Against a context created from the same positions: the same forces and
  energies at the reload, bit for bit; with the same velocities and step,
  the same trajectory bit for bit with the FP32 and the FP64 noise
  contractions.  The BF16x3 contraction sums the window in chunks aligned to
  8-row groups of each context's own step count, 100 in the reloaded context
  and 0 in the fresh one (whose replicas start at step 100): there the
  trajectories agree within 1e-5 A after 64 steps (measured 3e-7 A), and bit
  for bit when the step counts are equal modulo 8."""
import numpy as np
import pytest

from paper_1905_02521_amd import qtb, workloads as W
from tests.gpu_common import crystal

pytestmark = pytest.mark.gpu

SYSTEMS = ((3, 4, 2), (2, 1, 1))  # (cells, beads, noise)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()


def _ctx(configs, vels=None, prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3):
    reps = []
    for k, ((beads, sp, box), (_, _, noise)) in enumerate(zip(configs, SYSTEMS)):
        reps.append(qtb.Replica(pos=beads, species=sp, T=80.0, gamma=2e-3, dt=1.0, noise=noise,
                                vel=None if vels is None else vels[k], box=tuple(box), seed=5,
                                stream=k))
    ctx = qtb.Context(qtb.pair_potential_dict(W.mgo_potential()), reps, dict(W.METAL_UNITS),
                      prec=prec, fir=fir, max_two_nf=512, autotune=False)
    for k, (_, _, noise) in enumerate(SYSTEMS):
        ctx.build_filter(k, noise, 512)
    return ctx


@pytest.mark.parametrize("prec,fir", [(qtb.PREC_FP32, qtb.FIR_BF16X3), (qtb.PREC_FP32, qtb.FIR_FP32),
                                      (qtb.PREC_FP64, qtb.FIR_FP64)])
def test_positions_taken_in_place(prec, fir):
    import torch
    first = [crystal(n, P, seed=10 + k, bead_spread=0.01) for k, (n, P, _) in enumerate(SYSTEMS)]
    second = [crystal(n, P, seed=20 + k, bead_spread=0.01) for k, (n, P, _) in enumerate(SYSTEMS)]
    ctx = _ctx(first, prec=prec, fir=fir)
    ctx.step(100)
    src = torch.as_tensor(np.concatenate([b.ravel() for b, _, _ in second]), device="cuda")
    with pytest.raises(ValueError):
        ctx.set_positions(src[:-1])
    ctx.set_positions(src)
    states = [ctx.get_state(k) for k in range(len(SYSTEMS))]
    vels = [v for _, v, _ in states]
    step = states[0][2]
    fresh = _ctx(second, vels, prec=prec, fir=fir)
    for k in range(len(SYSTEMS)):
        fresh.set_state(k, None, None, step)
        assert np.array_equal(states[k][0], second[k][0]), k
    for k in range(len(SYSTEMS)):
        f1, e1 = ctx.evaluate(k)
        f2, e2 = fresh.evaluate(k)
        assert np.array_equal(f1, f2), k
        assert np.array_equal(e1, e2), k
    # the same history, then the same positions from host arrays
    host = _ctx(first, prec=prec, fir=fir)
    host.step(100)
    for k in range(len(SYSTEMS)):
        host.set_state(k, second[k][0], vels[k], step)
    for c in (ctx, fresh, host):
        c.step(64)
    for k in range(len(SYSTEMS)):
        r1, v1, n1 = ctx.get_state(k)
        r2, v2, n2 = fresh.get_state(k)
        r3, v3, n3 = host.get_state(k)
        print(f"replica {k}: max |r in place - r fresh| {np.max(np.abs(r1 - r2)):.3g}, "
              f"max |r in place - r host arrays| {np.max(np.abs(r1 - r3)):.3g}, "
              f"max |r host arrays - r fresh| {np.max(np.abs(r3 - r2)):.3g}")
        assert n1 == n2 == n3 == step + 64
    for k in range(len(SYSTEMS)):
        r1, v1, _ = ctx.get_state(k)
        r2, v2, _ = fresh.get_state(k)
        r3, v3, _ = host.get_state(k)
        assert np.array_equal(r1, r3) and np.array_equal(v1, v3), k
        if fir == qtb.FIR_BF16X3:   # step counts 100 and 0: not equal modulo 8
            assert np.max(np.abs(r1 - r2)) < 1e-5, k
        else:
            assert np.array_equal(r1, r2) and np.array_equal(v1, v2), k
    for c in (ctx, fresh, host):
        c.close()


def test_bf16x3_restore_is_bit_exact_when_step_counts_agree_modulo_8():
    """The restore condition of the BF16x3 contraction: a state restored at
    step 104 of a context's own count (104 = 0 mod 8) continues bit for bit
    like a fresh context (count 0) whose replicas start at step 104."""
    first = [crystal(n, P, seed=30 + k, bead_spread=0.01) for k, (n, P, _) in enumerate(SYSTEMS)]
    second = [crystal(n, P, seed=40 + k, bead_spread=0.01) for k, (n, P, _) in enumerate(SYSTEMS)]
    host = _ctx(first)
    host.step(104)
    vels = [host.get_state(k)[1] for k in range(len(SYSTEMS))]
    step = host.get_state(0)[2]
    assert step == 104
    for k in range(len(SYSTEMS)):
        host.set_state(k, second[k][0], vels[k], step)
    fresh = _ctx(second, vels)
    for k in range(len(SYSTEMS)):
        fresh.set_state(k, None, None, step)
    host.step(64)
    fresh.step(64)
    for k in range(len(SYSTEMS)):
        r1, v1, n1 = host.get_state(k)
        r2, v2, n2 = fresh.get_state(k)
        assert n1 == n2 == step + 64
        assert np.array_equal(r1, r2) and np.array_equal(v1, v2), k
    host.close()
    fresh.close()
