"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (from the workload contract and the arithmetic):
* white noise: bit-exact FP64;
* FIR taps (library and oracle both FP64, different quadrature / DFT): 1e-12;
* coloured noise, FP64 FIR: 1e-12 of sum_k |h_k w| (summation order only);
  FP32 MFMA: 2^-20 sum_k |h_k w| (FP32 rounding of w, h, products and sums);
  BF16x3: 3 2^-16 ... bounded by 1e-4 sum_k |h_k w| (hi/lo split drops lo*lo,
  each half-split keeps 16 bits), BF16: 1e-2;
* forces: ||F - F_oracle|| / ||F_oracle|| <= 1e-5 (FP32), 1e-12 (FP64);
* 10-step FP64 trajectories: RMS position difference / RMS displacement <= 1e-9.
"""
import math

import numpy as np
import pytest

from paper_1905_02521_amd import qtb, workloads as W
from tests.gpu_common import (crystal, gpu_crystal_ctx, gpu_ho_ctx, oracle_pair_pot,
                              oracle_units, oracle_zeta_block)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()


# ------------------------------------------------------------------ white noise
@pytest.mark.parametrize("seed,stream,tag,n0,d0", [(0, 0, 0, 0, 0), (12345, 3, 0, -700, 17),
                                                   (2**64 - 1, 2**28, 15, -(2**40) + 5, 2**32 - 300),
                                                   (0x0123456789ABCDEF, 7, 2, 2**33, 1000)])
def test_white_noise_bit_exact(orc, seed, stream, tag, n0, d0):
    rows, n_dof = 300, 256
    g = qtb.qtb_gaussian(seed, stream, tag, n0, rows, d0, n_dof).cpu().numpy()
    o = orc.gauss_fill(seed, n0, rows, d0, n_dof, stream, tag)
    assert np.array_equal(g.view(np.uint64), o.view(np.uint64)), \
        f"{np.count_nonzero(g != o)} of {g.size} differ"


def test_white_noise_bit_exact_large(orc):
    rows, n_dof = 1000, 1000
    g = qtb.qtb_gaussian(77, 1, 0, -500, rows, 0, n_dof).cpu().numpy()
    o = orc.gauss_fill(77, -500, rows, 0, n_dof, 1, 0)
    assert np.array_equal(g.view(np.uint64), o.view(np.uint64))


# ------------------------------------------------------------------ filter taps
@pytest.mark.parametrize("kind,P,T", [(1, 1, 1.0), (2, 8, 1.0), (2, 3, 0.3), (2, 32, 2.0)])
def test_taps_match_oracle(orc, kind, P, T):
    om = W.oscillator_omegas(16)
    ctx = gpu_ho_ctx(om, P, T=T, gamma=1.0, dt=0.001, noise=kind, prec=qtb.PREC_FP64,
                     fir=qtb.FIR_FP64, max_two_nf=512)
    taps = ctx.build_filter(0, kind, 512)
    ref = orc.taps(kind, T, P, 0.001, 512, oracle_units(orc, True))
    assert np.max(np.abs(taps - ref)) <= 1e-12 * np.max(np.abs(ref))


# ------------------------------------------------------------------ coloured noise
def fir_tol(fir, two_nf):
    """Per-element bound on |zeta - zeta_oracle| / sum_k |h_k w_{n-k}|.
    FP64: summation order only.  FP32: input rounding of h and w plus a
    worst-case FP32 accumulation of 2Nf terms.  BF16x3: each operand split in
    hi + lo keeps 16 bits (2^-16 each), the dropped lo*lo term adds 2^-16, plus
    the FP32 accumulation.  BF16: one 8-bit product (2 2^-8) plus accumulation."""
    acc = (two_nf + 4) * 2.0**-24
    return {qtb.FIR_FP64: 1e-12, qtb.FIR_FP32: acc, qtb.FIR_BF16X3: 3 * 2.0**-16 + acc,
            qtb.FIR_BF16: 2 * 2.0**-8 + acc}[fir]


@pytest.mark.parametrize("fir,K,two_nf,P", [(qtb.FIR_FP64, 64, 512, 1), (qtb.FIR_FP32, 64, 512, 1),
                                            (qtb.FIR_BF16X3, 64, 512, 1), (qtb.FIR_BF16, 64, 512, 1),
                                            (qtb.FIR_FP32, 128, 256, 4),
                                            (qtb.FIR_BF16X3, 256, 128, 2),
                                            (qtb.FIR_FP64, 128, 64, 3),
                                            (qtb.FIR_BF16X3, 64, 2048, 1)])
def test_colored_noise_matches_oracle(orc, fir, K, two_nf, P):
    om = W.oscillator_omegas(300)   # 300 P dofs: ragged last tile
    prec = qtb.PREC_FP64 if fir == qtb.FIR_FP64 else qtb.PREC_FP32
    kind = 1 if P == 1 else 2
    seed, stream = 11, 5
    ctx = gpu_ho_ctx(om, P, T=1.0, gamma=1.0, dt=0.01, noise=kind, prec=prec, fir=fir, seed=seed,
                     stream=stream, K=K, max_two_nf=two_nf)
    taps = ctx.build_filter(0, kind, two_nf)
    for blk in range(2):
        ctx.step(K)
        z, n0 = ctx.get_noise(0)
        assert n0 == blk * K
        ref, scale = oracle_zeta_block(orc, taps, seed, stream, n0, K, len(om) * P)
        err = np.abs(z - ref) / scale
        assert np.max(err) <= fir_tol(fir, two_nf), (fir, np.max(err))


# ------------------------------------------------------------------ forces
def _force_rel(f, ref):
    return np.linalg.norm(f - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("prec,tol", [(qtb.PREC_FP32, 1e-5), (qtb.PREC_FP64, 1e-12)])
@pytest.mark.parametrize("n_cells,P", [(4, 1), (3, 4), (2, 3), (5, 2), (3, 16), (2, 32)])
def test_forces_match_bruteforce(orc, prec, tol, n_cells, P):
    beads, sp, box = crystal(n_cells, P, seed=7, bead_spread=0.03)
    fir = qtb.FIR_FP64 if prec == qtb.PREC_FP64 else qtb.FIR_FP32
    ctx = gpu_crystal_ctx(beads, sp, box, T=100.0, gamma=1e-3, dt=1.0, noise=0, prec=prec,
                          fir=fir)
    f, e = ctx.evaluate(0)
    U = oracle_units(orc, False)
    pot = oracle_pair_pot(orc)
    for b in range(P):
        eo, fo, _ = orc.pair_bruteforce(pot, U, box, sp, beads[b])
        assert _force_rel(f[b], fo) <= tol, (b, _force_rel(f[b], fo))
        assert abs(e[b] - eo) <= (1e-6 if prec == qtb.PREC_FP32 else 1e-11) * abs(eo)


@pytest.mark.parametrize("prec,tol", [(qtb.PREC_FP32, 1e-5), (qtb.PREC_FP64, 1e-12)])
@pytest.mark.parametrize("P", [4, 8, 6])
def test_every_decomposition_matches_bruteforce(orc, prec, tol, P):
    """The autotuner's choices (1, 2 or 4 wavefronts per atom; the widest
    bead group per wavefront or half of it): each gives the brute-force
    forces, and pinning one skips the autotuning."""
    beads, sp, box = crystal(3, P, seed=8, bead_spread=0.03)
    fir = qtb.FIR_FP64 if prec == qtb.PREC_FP64 else qtb.FIR_FP32
    ctx = gpu_crystal_ctx(beads, sp, box, T=100.0, gamma=1e-3, dt=1.0, noise=0, prec=prec,
                          fir=fir)
    U = oracle_units(orc, False)
    pot = oracle_pair_pot(orc)
    ref = [orc.pair_bruteforce(pot, U, box, sp, beads[b])[1] for b in range(P)]
    for W in (1, 2, 4):
        for half in (False, True):
            ctx.set_decomposition(W, half)
            assert ctx.decomposition() == (W, half)
            f, _ = ctx.evaluate(0)
            for b in range(P):
                assert _force_rel(f[b], ref[b]) <= tol, (W, half, b)
    ctx.set_decomposition(2, True)
    ctx.step(3)   # pinned: the first step does not retune
    assert ctx.decomposition() == (2, True)
    for bad in ((3, False), (0, True)):
        with pytest.raises(qtb.QtbError):
            ctx.set_decomposition(*bad)
    ctx.close()


def test_half_groups_trajectory_fp64(orc):
    """QTB-PIMD (P = 8) with four beads per wavefront, 40 steps in FP64
    against the oracle (the bead groups of one atom sit in separate
    workgroups)."""
    P = 8
    beads, sp, box = crystal(3, P, seed=4, bead_spread=0.02)
    T, gamma, dt, seed = 100.0, 5e-3, 1.0, 12
    ctx = gpu_crystal_ctx(beads, sp, box, T=T, gamma=gamma, dt=dt, noise=2,
                          prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=seed, max_two_nf=128)
    ctx.build_filter(0, 2, 128)
    ctx.set_decomposition(1, True)
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), beads.shape[2], P, 3, box,
                   sp, T, gamma, dt, seed, 0, 2, 128, beads, n_threads=8)
    rel, dv = _traj_compare(orc, ctx, osim, 40, 0.0421)
    assert rel <= 1e-9, rel
    ctx.close()


# ------------------------------------------------------------------ trajectories
def _traj_compare(orc, ctx, osim, n_steps, scale):
    ctx.step(n_steps)
    osim.run(n_steps)
    r, v, st = ctx.get_state(0)
    ro, vo, _, sto = osim.state()
    assert st == sto == n_steps
    return np.sqrt(np.mean((r - ro) ** 2)) / scale, np.sqrt(np.mean((v - vo) ** 2))


@pytest.mark.parametrize("P,noise,two_nf", [(1, 1, 512), (4, 2, 256), (3, 2, 128), (2, 0, 2),
                                             (16, 2, 128), (32, 0, 2), (32, 2, 128)])
def test_crystal_trajectory_fp64(orc, P, noise, two_nf):
    n_cells = 3 if P > 1 else 4
    beads, sp, box = crystal(n_cells, P, seed=3, bead_spread=0.02)
    T, gamma, dt, seed = 100.0, 1e-3 * 5, 1.0, 9
    ctx = gpu_crystal_ctx(beads, sp, box, T=T, gamma=gamma, dt=dt, noise=noise,
                          prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=seed, max_two_nf=max(two_nf, 2))
    if noise:
        ctx.build_filter(0, noise, two_nf)
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), beads.shape[2], P, 3, box, sp,
                   T, gamma, dt, seed, 0, noise, two_nf, beads, n_threads=8)
    rel, _ = _traj_compare(orc, ctx, osim, 10, scale=0.0421)
    assert rel <= 1e-9, rel


@pytest.mark.parametrize("P,noise", [(1, 1), (4, 2), (16, 2)])
def test_oscillator_trajectory_fp64(orc, P, noise):
    om = W.oscillator_omegas(256)
    T, gamma, dt, two_nf = 1.0, 1.0, 0.001, 512
    ctx = gpu_ho_ctx(om, P, T=T, gamma=gamma, dt=dt, noise=noise, prec=qtb.PREC_FP64,
                     fir=qtb.FIR_FP64, seed=0, max_two_nf=two_nf)
    ctx.build_filter(0, noise, two_nf)
    osim = orc.Sim(orc.make_pot(1, (1.0,)), oracle_units(orc, True), 256, P, 1, None,
                   np.zeros(256, np.int32), T, gamma, dt, 0, 0, noise, two_nf,
                   np.zeros((P, 1, 256)), harm_omega=om, n_threads=8)
    n = 1000 if P == 1 else 200
    ctx.step(n)
    osim.run(n)
    r, v, _ = ctx.get_state(0)
    ro, vo, _, _ = osim.state()
    scale = np.sqrt(np.mean(ro**2))
    assert np.sqrt(np.mean((r - ro) ** 2)) / scale <= 1e-9


def test_crystal_trajectory_fp32_close(orc):
    """FP32 forces / BF16x3 noise: the short trajectory follows the oracle to the
    force tolerance (positions differ by ~dt^2 F err / m per step)."""
    beads, sp, box = crystal(4, 1, seed=5)
    ctx = gpu_crystal_ctx(beads, sp, box, T=100.0, gamma=1e-3, dt=1.0, noise=1,
                          prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3, seed=2)
    ctx.build_filter(0, 1, 512)
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), 512, 1, 3, box, sp, 100.0,
                   1e-3, 1.0, 2, 0, 1, 512, beads, n_threads=8)
    rel, _ = _traj_compare(orc, ctx, osim, 10, scale=0.0421)
    assert rel <= 1e-5, rel


# ------------------------------------------------------------- one harness, two back ends
def _harness(make_ctx, reps, noise_of):
    """Drive a context through the call shape both back ends export: build
    the filters, 10 + 54 eager steps and a 64-step block, a checkpoint
    restore, 30 more steps; returns the states and the observables."""
    ctx = make_ctx()
    for k in range(len(reps)):
        ctx.build_filter(k, noise_of[k], 128)
    out = []
    for n in (10, 54, 64):
        ctx.step(n)
    r, v, st = ctx.get_state(0)
    ctx.set_state(0, r, v, st)
    ctx.step(30)
    for k in range(len(reps)):
        out.append((ctx.get_state(k), ctx.observables(k)))
    ctx.close()
    return out


def test_one_harness_drives_both_back_ends(orc):
    """The same harness code on the library (FP64) and on the oracle behind
    the library's call shape: states to 1e-9, sampled means to 1e-9."""
    specs = [(2, 4, 2, 100.0, 5), (3, 1, 1, 300.0, 6)]
    reps, noise_of = [], []
    for k, (n, P, noise, T, seed) in enumerate(specs):
        beads, sp, box = crystal(n, P, seed=seed, bead_spread=0.02 if P > 1 else 0.0)
        reps.append(qtb.Replica(pos=beads, species=sp, T=T, gamma=5e-3, dt=1.0, noise=noise,
                                box=tuple(box), seed=seed, stream=k))
        noise_of.append(noise)
    potd = qtb.pair_potential_dict(W.mgo_potential())
    gpu = _harness(lambda: qtb.Context(potd, reps, dict(W.METAL_UNITS), prec=qtb.PREC_FP64,
                                       fir=qtb.FIR_FP64, max_two_nf=128, obs_every=8),
                   reps, noise_of)
    ora = _harness(lambda: orc.AbiContext(potd, reps, dict(W.METAL_UNITS), obs_every=8,
                                          max_two_nf=128), reps, noise_of)
    for ((r, v, st), og), ((ro, vo, so), oo) in zip(gpu, ora):
        assert st == so == 158
        assert np.sqrt(np.mean((r - ro) ** 2)) <= 1e-9 * 0.0421
        assert np.sqrt(np.mean((v - vo) ** 2)) <= 1e-9 * np.sqrt(np.mean(vo ** 2))
        assert og["n_samples"] == oo["n_samples"] == 19
        for f in ("kinetic", "potential", "e_primitive", "e_virial", "x2_mean", "pressure",
                  "volume"):
            assert abs(og[f] - oo[f]) <= 1e-9 * max(abs(oo[f]), 1e-12), f


# ------------------------------------------------------------------ observables
@pytest.mark.parametrize("P,noise", [(1, 1), (4, 2), (16, 2), (32, 0)])
def test_observables_match_oracle(orc, P, noise):
    beads, sp, box = crystal(3, P, seed=4, bead_spread=0.02)
    T, gamma, dt = 50.0, 5e-3, 1.0
    ctx = gpu_crystal_ctx(beads, sp, box, T=T, gamma=gamma, dt=dt, noise=noise,
                          prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=6, obs_every=5,
                          max_two_nf=256)
    ctx.build_filter(0, noise, 256)
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), beads.shape[2], P, 3, box, sp,
                   T, gamma, dt, 6, 0, noise, 256, beads, n_threads=8)
    ctx.step(40)
    obs = osim.run(40, 5)
    g = ctx.observables(0)
    assert g["n_samples"] == 8
    o = obs.mean(axis=0)
    for nm in ("kinetic", "potential", "spring", "e_primitive", "e_virial", "t_kinetic",
               "x2_mean", "virial_pair", "pressure"):
        q = orc.OBS_NAMES.index(nm)
        assert abs(g[nm] - o[q]) <= 1e-9 * max(1.0, abs(o[q])), (nm, g[nm], o[q])


# ------------------------------------------------------------------ errors
def test_step_before_filter_is_state_error():
    om = W.oscillator_omegas(8)
    ctx = gpu_ho_ctx(om, 1, T=1.0, gamma=1.0, dt=0.01, noise=1, prec=qtb.PREC_FP64,
                     fir=qtb.FIR_FP64)
    with pytest.raises(qtb.QtbError) as e:
        ctx.step(1)
    assert e.value.status == qtb.QTB_E_STATE


def test_invalid_arguments_rejected():
    om = W.oscillator_omegas(8)
    with pytest.raises(qtb.QtbError) as e:
        gpu_ho_ctx(om, 1, T=-1.0, gamma=1.0, dt=0.01, noise=1, prec=qtb.PREC_FP64,
                   fir=qtb.FIR_FP64)
    assert e.value.status == qtb.QTB_E_INVALID
    ctx = gpu_ho_ctx(om, 1, T=1.0, gamma=1.0, dt=0.01, noise=1, prec=qtb.PREC_FP64,
                     fir=qtb.FIR_FP64, max_two_nf=64)
    with pytest.raises(qtb.QtbError) as e:
        ctx.build_filter(0, 1, 128)
    assert e.value.status == qtb.QTB_E_INVALID
    with pytest.raises(qtb.QtbError) as e:  # the FIR length is a power of two
        ctx.build_filter(0, 1, 48)
    assert e.value.status == qtb.QTB_E_INVALID
    with pytest.raises(qtb.QtbError) as e:
        ctx.build_filter(0, 2, 64)
    assert e.value.status == qtb.QTB_E_STATE


def test_nonfinite_state_detected():
    om = W.oscillator_omegas(8)
    ctx = gpu_ho_ctx(om, 1, T=1.0, gamma=1.0, dt=0.01, noise=0, prec=qtb.PREC_FP64,
                     fir=qtb.FIR_FP64)
    r, v, st = ctx.get_state(0)
    v[0, 0, 3] = np.nan
    ctx.set_state(0, r, v, st)
    ctx.step(2)
    with pytest.raises(qtb.QtbError) as e:
        ctx.observables(0)
    assert e.value.status == qtb.QTB_E_NONFINITE


def test_diverged_bead_spread_is_reported():
    """A bead far from its atom's centroid (as in a diverging trajectory) asks
    the list search for more periodic images than it covers: the search is
    clamped and the next check reports the state instead of looping."""
    beads, sp, box = crystal(2, 2, seed=3)
    ctx = gpu_crystal_ctx(beads, sp, box, T=50.0, gamma=1e-3, dt=1.0, noise=0,
                          prec=qtb.PREC_FP32, fir=qtb.FIR_FP32, autotune=False)
    r, v, st = ctx.get_state(0)
    r[1, 0, 0] += 500.0
    with pytest.raises(qtb.QtbError) as e:
        ctx.set_state(0, r, v, st)
        ctx.step(1)
        ctx.observables(0)
    assert e.value.status == qtb.QTB_E_NONFINITE


# ------------------------------------------------------------------ graphs
@pytest.mark.parametrize("prec,fir", [(qtb.PREC_FP64, qtb.FIR_FP64), (qtb.PREC_FP32, qtb.FIR_BF16X3)])
def test_graph_replay_matches_eager(prec, fir):
    """Whole noise blocks replayed as captured graphs give bit-identical states
    to the eager launches, replay after replay, with host work in between."""
    beads, sp, box = crystal(3, 4, seed=8, bead_spread=0.02)
    # the same force decomposition on both sides (the autotuner times the
    # candidates, so two contexts may pick different ones and sum in another order)
    kw = dict(T=50.0, gamma=5e-3, dt=1.0, noise=2, prec=prec, fir=fir, seed=4, K=64,
              max_two_nf=256, obs_every=16, autotune=False)
    g = gpu_crystal_ctx(beads, sp, box, graphs=True, **kw)
    e = gpu_crystal_ctx(beads, sp, box, graphs=False, **kw)
    for c in (g, e):
        c.build_filter(0, 2, 256)
    for blk in range(4):
        g.step(64)
        e.step(64)
        rg, vg, sg = g.get_state(0)
        re, ve, se = e.get_state(0)
        assert sg == se == 64 * (blk + 1)
        assert np.array_equal(rg, re) and np.array_equal(vg, ve), blk
        og, oe = g.observables(0), e.observables(0)
        assert og == oe
    # a partial block, then graphs again
    g.step(10); e.step(10)
    g.step(128); e.step(128)
    rg, vg, _ = g.get_state(0)
    re, ve, _ = e.get_state(0)
    assert np.array_equal(rg, re) and np.array_equal(vg, ve)


@pytest.mark.parametrize("prec,tol,P", [(qtb.PREC_FP64, 1e-9, 4), (qtb.PREC_FP32, 1e-5, 4),
                                        (qtb.PREC_FP64, 1e-9, 16), (qtb.PREC_FP32, 1e-5, 32)])
def test_trajectory_with_frequent_rebuilds(orc, prec, tol, P):
    """A 0.02 A skin forces neighbour-list rebuilds during the run; the
    trajectory must still follow the oracle (which never misses a pair).
    P = 16 and 32 split every atom's beads over several 8-bead groups, each
    group's workgroup reading the one list the rebuild writes."""
    beads, sp, box = crystal(3, P, seed=12, bead_spread=0.03)
    p = W.mgo_potential(skin=0.02)
    fir = qtb.FIR_FP64 if prec == qtb.PREC_FP64 else qtb.FIR_FP32
    ctx = gpu_crystal_ctx(beads, sp, box, T=300.0, gamma=2e-3, dt=1.0, noise=2, prec=prec,
                          fir=fir, seed=21, max_two_nf=128, pot=p)
    ctx.build_filter(0, 2, 128)
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), beads.shape[2], P, 3, box, sp,
                   300.0, 2e-3, 1.0, 21, 0, 2, 128, beads, n_threads=8)
    rel, _ = _traj_compare(orc, ctx, osim, 30, scale=0.0421)
    assert rel <= tol, rel


@pytest.mark.parametrize("prec,tol", [(qtb.PREC_FP32, 1e-5), (qtb.PREC_FP64, 1e-9)])
def test_large_replica_list_kernel_with_rebuilds(orc, prec, tol):
    """17 576 atoms (13x13x13 cells) take the list kernel, whose scan skips
    candidate tiles by their centroid bounds; with a 0.02 A skin it rebuilds
    during the run, and the trajectory still follows the oracle."""
    beads, sp, box = crystal(13, 1, seed=14)
    assert beads.shape[2] > 16384
    p = W.mgo_potential(skin=0.02)
    fir = qtb.FIR_FP64 if prec == qtb.PREC_FP64 else qtb.FIR_FP32
    ctx = gpu_crystal_ctx(beads, sp, box, T=300.0, gamma=2e-3, dt=1.0, noise=1, prec=prec,
                          fir=fir, seed=22, max_two_nf=128, pot=p)
    ctx.build_filter(0, 1, 128)
    ctx.profile(True)
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), beads.shape[2], 1, 3, box, sp,
                   300.0, 2e-3, 1.0, 22, 0, 1, 128, beads, n_threads=8)
    rel, _ = _traj_compare(orc, ctx, osim, 30, scale=0.0421)
    prof = ctx.profile_read()
    assert prof["nlist"][1] > 0  # the list kernel ran
    assert rel <= tol, rel


@pytest.mark.parametrize("fuse", [True, False])
def test_profile_reports_every_phase(fuse):
    beads, sp, box = crystal(3, 4, seed=2)
    ctx = gpu_crystal_ctx(beads, sp, box, T=50.0, gamma=1e-3, dt=1.0, noise=2,
                          prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3, max_two_nf=128, fuse=fuse)
    ctx.build_filter(0, 2, 128)
    ctx.profile(True)
    ctx.step(128)
    prof = ctx.profile_read()
    ctx.profile(False)
    # one kernel per step: the run opens with an update and ends with a force pass
    assert prof["forces"][1] == 128 and prof["update"][1] == (1 if fuse else 128)
    assert prof["fir"][1] == 2 and prof["noise"][1] >= 2
    assert all(v[0] > 0 for k, v in prof.items() if v[1] > 0)


# ------------------------------------------------------- one kernel per step
@pytest.mark.parametrize("P", [1, 4, 8])
def test_one_kernel_steps_equal_separate_kernels(P):
    """The fused step kernel does the separate kernels' arithmetic: without
    list rebuilds the trajectories and sampled observables are bit for bit
    the same (FP64); with rebuilds every few steps (the fused kernel then
    rebuilds neighbour positions from the previous references) they agree to
    rounding."""
    beads, sp, box = crystal(3, P, seed=30, bead_spread=0.02 if P > 1 else 0.0)
    noise = 2 if P > 1 else 1
    for skin, exact in ((1.5, True), (0.02, False)):
        p = W.mgo_potential(skin=skin)
        outs = []
        for fuse in (True, False):
            ctx = gpu_crystal_ctx(beads, sp, box, T=300.0, gamma=2e-3, dt=1.0, noise=noise,
                                  prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=5, max_two_nf=128,
                                  obs_every=8, pot=p, fuse=fuse, autotune=False)
            ctx.build_filter(0, noise, 128)
            ctx.step(50)
            ctx.step(64)
            ctx.step(7)
            r, v, st = ctx.get_state(0)
            outs.append((r, v, st, ctx.observables(0)))
        (r1, v1, s1, o1), (r2, v2, s2, o2) = outs
        assert s1 == s2 == 121 and o1["n_samples"] == o2["n_samples"] == 15
        if exact:
            assert np.array_equal(r1, r2) and np.array_equal(v1, v2)
            # the centroid kinetic energy of the virial estimator is summed in
            # the kernel's own order by the one-kernel step: agreement to rounding
            assert {k: x for k, x in o1.items() if k != "e_virial"} == \
                {k: x for k, x in o2.items() if k != "e_virial"}
            assert abs(o1["e_virial"] - o2["e_virial"]) <= 1e-12 * abs(o2["e_virial"])
        else:
            assert np.max(np.abs(r1 - r2)) < 1e-10 and np.max(np.abs(v1 - v2)) < 1e-10
            assert abs(o1["e_primitive"] - o2["e_primitive"]) < 1e-9 * abs(o2["e_primitive"])
