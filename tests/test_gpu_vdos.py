"""Velocity density of states on the GPU (Sec. 3: QTB-MD gives direct access
to time-correlation functions; the DOS is the check to make at high gamma).

Parity (FP64, against the oracle's segment periodograms):
* the standalone transform on seeded series in both layouts: one dof, odd
  dof counts, a ragged trailing segment, no whole segment, the largest
  segment, a crystal's worth of dofs; every bin within 1e-12 of the largest;
* the recorder on QTB trajectories: harmonic oscillators (odd count) and the
  MgO crystal with separate and with one-kernel steps, against the spectra of
  the oracle's own trajectories; restart and set_state cut the series;
* Parseval on the GPU: the spectrum's mean over all frequencies is twice the
  mean kinetic energy the observables report over the same samples.
Statistics: the spectrum of QTB oscillators lies within the block-mean errors
of the exact spectrum of the discrete scheme (linear response, Fejer window).
"""
import math

import numpy as np
import pytest

from paper_1905_02521_amd import qtb, workloads as W
from tests.closed_forms import baoab_mode_map
from tests.gpu_common import (crystal, gpu_crystal_ctx, gpu_ho_ctx, oracle_pair_pot, units_dict,
                              oracle_units)
from tests.test_oracle_vdos import expected_periodogram

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()


def full_mean(S):
    """Mean over all seg frequencies of a spectrum given for k = 0 .. seg/2."""
    seg = 2 * (len(S) - 1)
    return (S[0] + S[-1] + 2.0 * np.sum(S[1:-1])) / seg


@pytest.mark.parametrize("dof_major", [False, True])
@pytest.mark.parametrize("n_samples,n_dof,seg", [
    (64, 1, 16), (100, 7, 16), (3 * 256 + 5, 301, 256), (2048, 3 * 4096, 1024),
    (4096, 3, 4096), (8192, 2, 4096), (10, 5, 16), (5 * 64, 4097, 64)])
def test_spectrum_matches_oracle(orc, n_samples, n_dof, seg, dof_major):
    """Both layouts: [samples][dofs] (read row by row) and [dofs][samples]
    (each dof's series contiguous, the recorder's layout)."""
    import torch
    rng = np.random.default_rng(n_samples * 7 + n_dof)
    v = rng.normal(size=(n_samples, n_dof)) * rng.uniform(0.2, 3.0, n_dof)
    w = rng.uniform(0.5, 40.0, n_dof)
    dv = torch.from_numpy(np.ascontiguousarray(v.T) if dof_major else v).cuda()
    dw = torch.from_numpy(w).cuda()
    S = qtb.vdos_spectrum(dv, dw, seg, dof_major=dof_major).cpu().numpy()
    _, So, n_seg = orc.vdos(v, seg, w)
    assert S.shape == So.shape == (seg // 2 + 1,)
    if n_seg == 0:
        assert np.all(S == 0.0)
        return
    err = np.max(np.abs(S - So)) / np.max(So)
    print(f"n_samples {n_samples} n_dof {n_dof} seg {seg}: max rel error {err:.2e}")
    assert err <= 1e-12


def test_spectrum_rejects_bad_sizes():
    import torch
    v = torch.zeros((64, 4), dtype=torch.float64, device="cuda")
    w = torch.ones(4, dtype=torch.float64, device="cuda")
    for seg in (8, 24, 8192):
        with pytest.raises(qtb.QtbError):
            qtb.vdos_spectrum(v, w, seg)


def _osc_setup(n, P=1, obs_every=2, T=0.25, gamma=0.2, dt=0.1, two_nf=256, omega=1.0, seed=4):
    om = np.full(n, omega) * (1.0 + 0.5 * np.arange(n) / max(n - 1, 1))
    ctx = gpu_ho_ctx(om, P, T=T, gamma=gamma, dt=dt, noise=1 if P == 1 else 2,
                     prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=seed, max_two_nf=two_nf,
                     obs_every=obs_every, pos=np.full((P, 1, n), 0.3))
    taps = ctx.build_filter(0, 1 if P == 1 else 2, two_nf)
    return ctx, om, taps


def test_recorder_matches_oracle_oscillators(orc):
    """257 oscillators (omega 1..1.5), QTB, FP64, a sample every 2 steps,
    segments of 32 samples: 1000 steps give 15 segments (and 20 samples of a
    16th); the oracle's trajectory sampled the same way gives the same
    spectrum."""
    n, every, seg, two_nf, T, gamma, dt = 257, 2, 32, 256, 0.25, 0.2, 0.1
    ctx, om, _ = _osc_setup(n, obs_every=every, T=T, gamma=gamma, dt=dt, two_nf=two_nf)
    ctx.vdos_attach(0, seg)
    ctx.step(1000)
    S, n_seg = ctx.vdos_read(0)
    assert n_seg == 15
    osim = orc.Sim(orc.make_pot(1, (1.0,)), oracle_units(orc, True), n, 1, 1, None,
                   np.zeros(n, np.int32), T, gamma, dt, 4, 0, 1, two_nf, np.full((1, 1, n), 0.3),
                   harm_omega=om, n_threads=8)
    v = np.empty((500, n))
    for t in range(500):
        osim.run(every)
        v[t] = osim.state()[1][0, 0]
    _, So, n_o = orc.vdos(v, seg)
    assert n_o == 15
    err = np.max(np.abs(S - So)) / np.max(So)
    print(f"oscillators: max rel error {err:.2e}")
    assert err <= 1e-8
    # restart: the next segments count afresh, from the current step
    ctx.vdos_read(0, restart=True)
    ctx.step(2 * seg * every + 3)
    S2, n2 = ctx.vdos_read(0)
    assert n2 == 2
    v2 = np.empty((2 * seg, n))
    for t in range(2 * seg):
        osim.run(every)
        v2[t] = osim.state()[1][0, 0]
    assert np.max(np.abs(S2 - orc.vdos(v2, seg)[1])) <= 1e-8 * np.max(S2)
    # set_state cuts the series
    r, vv, st = ctx.get_state(0)
    ctx.set_state(0, r, vv, st)
    assert ctx.vdos_read(0)[1] == 0
    ctx.vdos_detach(0)
    ctx.step(10)
    with pytest.raises(qtb.QtbError):
        ctx.vdos_read(0)
    ctx.close()


@pytest.mark.parametrize("fuse", [False, True])
def test_recorder_matches_oracle_crystal(orc, fuse):
    """MgO 4x4x4 (512 atoms), QTB, FP64, every step sampled, segments of 64:
    130 steps give 2 segments; weights are the masses (amu times the mass
    unit).  The one-kernel step samples a step inside the next step's kernel:
    the recorder must store the same velocities."""
    beads, sp, box = crystal(4, 1, seed=3)
    T, gamma, dt, seed, two_nf, seg = 100.0, 5e-3, 1.0, 9, 512, 64
    ctx = gpu_crystal_ctx(beads, sp, box, T=T, gamma=gamma, dt=dt, noise=1, prec=qtb.PREC_FP64,
                          fir=qtb.FIR_FP64, seed=seed, max_two_nf=two_nf, obs_every=1, fuse=fuse)
    ctx.build_filter(0, 1, two_nf)
    ctx.vdos_attach(0, seg)
    ctx.observables(0)
    ctx.step(2 * seg)
    S, n_seg = ctx.vdos_read(0)
    obs = ctx.observables(0)
    assert n_seg == 2 and obs["n_samples"] == 2 * seg
    # Parseval over exactly the same samples: mean of S = 2 <K>
    assert abs(full_mean(S) - 2 * obs["kinetic"]) <= 1e-12 * abs(full_mean(S))
    osim = orc.Sim(oracle_pair_pot(orc), oracle_units(orc, False), 512, 1, 3, box, sp, T, gamma,
                   dt, seed, 0, 1, two_nf, beads, n_threads=8)
    v = np.empty((2 * seg, 3 * 512))
    for t in range(2 * seg):
        osim.run(1)
        v[t] = osim.state()[1][0].reshape(-1)
    p = W.mgo_potential()
    w = np.tile(np.asarray(p.mass)[sp] * W.METAL_UNITS["mass_unit"], 3)
    _, So, _ = orc.vdos(v, seg, w)
    err = np.max(np.abs(S - So)) / np.max(So)
    print(f"crystal fuse={fuse}: max rel error {err:.2e}")
    assert err <= 1e-8
    ctx.close()


def test_recorder_rejects_bad_use():
    ctx, _, _ = _osc_setup(16, P=4, obs_every=2)
    with pytest.raises(qtb.QtbError):   # bead velocities: no time correlations
        ctx.vdos_attach(0, 64)
    ctx.close()
    ctx, _, _ = _osc_setup(16, obs_every=0)
    with pytest.raises(qtb.QtbError):   # nothing is sampled
        ctx.vdos_attach(0, 64)
    ctx.close()
    ctx, _, _ = _osc_setup(16, obs_every=1)
    for seg in (32, 48, 8192):           # seg * obs_every below the noise block; not 2^k; too long
        with pytest.raises(qtb.QtbError):
            ctx.vdos_attach(0, seg)
    with pytest.raises(qtb.QtbError):
        ctx.vdos_read(0)
    ctx.close()


def test_oscillator_vdos_matches_linear_response():
    """4096 oscillators, omega = 1, k_B T = 0.25, gamma = 0.2, dt = 0.1, QTB
    filter 2Nf = 256, every step sampled, segments of 256: 16 blocks of 4
    segments; each bin of the block mean within 4.5 standard errors of the
    exact expected periodogram, and the mean z^2 near 1."""
    n, seg, T, gamma, dt, two_nf = 4096, 256, 0.25, 0.2, 0.1, 256
    ctx = gpu_ho_ctx(np.full(n, 1.0), 1, T=T, gamma=gamma, dt=dt, noise=1, prec=qtb.PREC_FP64,
                     fir=qtb.FIR_FP64, seed=12, max_two_nf=two_nf, obs_every=1)
    taps = ctx.build_filter(0, 1, two_nf)
    ctx.step(2000)
    ctx.vdos_attach(0, seg)
    blocks = []
    for _ in range(16):
        ctx.step(4 * seg)
        S, nb = ctx.vdos_read(0, restart=True)
        assert nb == 4
        blocks.append(S / n)
    ctx.close()
    blocks = np.array(blocks)
    mean, se = blocks.mean(axis=0), blocks.std(axis=0, ddof=1) / math.sqrt(len(blocks))
    c1 = math.exp(-gamma * dt)
    M, b = baoab_mode_map(1.0, 0.0, c1, math.sqrt(1 - c1 * c1), dt)
    v2, Ek = expected_periodogram(M, b, taps, seg)
    z = (mean - Ek) / se
    print(f"<v^2> exact {v2:.5f}, from S {full_mean(mean):.5f}; max |z| {np.max(np.abs(z)):.2f}, "
          f"mean z^2 {np.mean(z * z):.3f}")
    assert np.max(np.abs(z)) < 4.5
    assert 0.6 < np.mean(z * z) < 1.5
    assert abs(full_mean(mean) / v2 - 1) < 0.01


def _crystal_dos(noise, gamma, T=100.0, seg=2048, n_seg=16, two_nf=1024, eq=6000):
    beads, sp, box = crystal(4, 1, seed=3)
    ctx = gpu_crystal_ctx(beads, sp, box, T=T, gamma=gamma, dt=1.0, noise=noise,
                          prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3, seed=5, max_two_nf=two_nf,
                          obs_every=1)
    taps = ctx.build_filter(0, noise, two_nf) if noise else None
    ctx.step(eq)
    ctx.vdos_attach(0, seg)
    ctx.step(seg * n_seg)
    S, n = ctx.vdos_read(0)
    ctx.close()
    assert n == n_seg
    return S, taps


def test_high_friction_dos_tail_broadening_and_zpel():
    """MgO 4x4x4 (512 atoms) at 100 K, production precision, dt = 1 fs,
    every step sampled, 16 segments of 2048 after 6000 steps, classical
    Langevin and QTB at gamma = 0.001, 0.005, 0.02, 0.05 / fs.  The claims of
    Sec. 3 on raising gamma, measured on the spectrum:
    * the spurious high-frequency tail: above four times the top of the
      phonon band the atoms answer the bath as free particles, so the tail's
      weight is the friction response of the discrete scheme to the noise
      spectrum (closed form) within a few per cent; with QTB noise it carries
      several times the classical tail's share of the kinetic energy;
    * broadening: the main peak's width grows several-fold;
    * zero-point-energy leakage at small gamma: against the harmonic share
      (classical spectrum times theta(omega) / k_B T, eq. 1) the low band of
      the QTB spectrum holds too much and the top band too little; raising
      gamma removes most of the imbalance."""
    from tests.closed_forms import theta_coth, velocity_spectrum_discrete
    gammas = (0.001, 0.005, 0.02, 0.05)
    kT, hbar, dt, seg, n_dof = W.METAL_UNITS["kB"] * 100.0, W.METAL_UNITS["hbar"], 1.0, 2048, 1536
    res = {(nz, g): _crystal_dos(nz, g) for nz in (0, 1) for g in gammas}
    w = 2 * np.pi * np.arange(seg // 2 + 1) / (seg * dt)
    S0 = res[(0, 0.001)][0]
    k_top = int(np.max(np.nonzero(S0 > 0.01 * S0.max())))   # top of the phonon band
    k0 = 4 * k_top
    tail = lambda S: (2 * np.sum(S[k0:-1]) + S[-1]) / seg
    ratio, frac, width = {}, {}, {}
    for (nz, g), (S, taps) in res.items():
        c1 = math.exp(-g * dt)
        M, b = baoab_mode_map(0.0, 0.0, c1, math.sqrt(1 - c1 * c1), dt)
        Sf = velocity_spectrum_discrete(M, b, taps if nz else [math.sqrt(kT)], w[1:] * dt)
        ratio[(nz, g)] = tail(S) / (n_dof * tail(np.concatenate([[0.0], Sf])))
        frac[(nz, g)] = tail(S) / full_mean(S)
        k = int(np.argmax(S))
        lo, hi = k, k
        while lo > 0 and S[lo] > S[k] / 2:
            lo -= 1
        while S[hi] > S[k] / 2:
            hi += 1
        width[(nz, g)] = w[hi] - w[lo]
        print(f"noise {nz} gamma {g}: tail/free-particle {ratio[(nz, g)]:.4f}, tail share of 2K "
              f"{frac[(nz, g)]:.4f}, main-peak FWHM {width[(nz, g)]:.4f} rad/fs")
    for g in gammas:
        assert 0.98 < ratio[(1, g)] < 1.06
        if g >= 0.02:
            assert 0.98 < ratio[(0, g)] < 1.06
        assert frac[(1, g)] > 5 * frac[(0, g)]
    for nz in (0, 1):
        assert all(frac[(nz, a)] < frac[(nz, b)] for a, b in zip(gammas[:-1], gammas[1:]))
    assert width[(1, 0.05)] > 4 * width[(1, 0.001)]
    # leakage: QTB band weight against classical weight x theta / k_B T
    th = np.array([theta_coth(x, kT, hbar) for x in w[1:k_top + 1]]) / kT
    edges = [0.0, 0.06, 0.09, 0.12, w[k_top]]
    share = {}
    for g in gammas:
        Sc, Sq = res[(0, g)][0][1:k_top + 1], res[(1, g)][0][1:k_top + 1]
        share[g] = [np.sum(Sq[m]) / np.sum((Sc * th)[m])
                    for m in ((w[1:k_top + 1] > a) & (w[1:k_top + 1] <= b)
                              for a, b in zip(edges[:-1], edges[1:]))]
        print(f"gamma {g}: QTB / harmonic share by band {np.round(share[g], 3)}")
    whole = np.sum(res[(1, 0.001)][0][1:k_top + 1]) / np.sum(res[(0, 0.001)][0][1:k_top + 1] * th)
    assert abs(whole - 1) < 0.02           # in-band total: the harmonic energy theta(omega)
    assert share[0.001][0] > 1.15 and share[0.001][-1] < 0.85
    assert abs(share[0.05][0] - 1) < 0.06 and abs(share[0.05][-1] - 1) < 0.03


def test_recorders_on_batched_replicas(orc):
    """Two recorded replicas and one unrecorded in one context (oscillators of
    different counts, seeds and segment lengths): each spectrum is the
    oracle's for that replica's own trajectory."""
    every, T, gamma, dt, two_nf = 1, 0.25, 0.2, 0.1, 256
    specs = [(33, 7, 64), (50, 8, None), (17, 9, 128)]   # (N, seed, seg or no recorder)
    reps, oms = [], []
    for N, seed, _ in specs:
        om = 1.0 + 0.3 * np.arange(N) / N
        oms.append(om)
        reps.append(qtb.Replica(pos=np.full((1, 1, N), 0.3), species=np.zeros(N, np.int32), T=T,
                                gamma=gamma, dt=dt, noise=1, seed=seed, stream=0, harm_omega=om))
    ctx = qtb.Context(dict(kind=qtb.POT_HARMONIC, mass=(1.0,)), reps, units_dict(True),
                      prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, obs_every=every, max_two_nf=two_nf)
    for r in range(len(specs)):
        ctx.build_filter(r, 1, two_nf)
    for r, (_, _, seg) in enumerate(specs):
        if seg:
            ctx.vdos_attach(r, seg)
    ctx.step(300)
    for r, (N, seed, seg) in enumerate(specs):
        if not seg:
            continue
        S, n_seg = ctx.vdos_read(r)
        assert n_seg == 300 // seg
        osim = orc.Sim(orc.make_pot(1, (1.0,)), oracle_units(orc, True), N, 1, 1, None,
                       np.zeros(N, np.int32), T, gamma, dt, seed, 0, 1, two_nf,
                       np.full((1, 1, N), 0.3), harm_omega=oms[r], n_threads=4)
        v = np.empty((n_seg * seg, N))
        for t in range(n_seg * seg):
            osim.run(every)
            v[t] = osim.state()[1][0, 0]
        So = orc.vdos(v, seg)[1]
        err = np.max(np.abs(S - So)) / np.max(So)
        print(f"replica {r}: {err:.2e}")
        assert err <= 1e-8
    ctx.close()
