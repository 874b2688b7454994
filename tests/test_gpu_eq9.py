"""The paper's block generator of the random force (eq. 9) on the GPU, as an
alternative to the streaming FIR (QTB_OPT_NOISE_BLOCKS).

* Parity: the coloured noise of QTB (P = 1) and QTB-PIMD (P = 4)
  oscillators, read back block by block over 320 steps that start off the
  K-step grid (so noise blocks straddle the n-step boundaries), against the
  oracle's eq. 9 blocks from the same counter-based Gaussians: 1e-12 of the
  noise's standard deviation with FP64 noise, 1e-6 with FP32.
* Statistics: the mean energy of 4096 QTB oscillators driven by block noise
  lies within two standard errors of the exact value for that noise (the
  discrete scheme's response to the time-averaged block autocovariance
  (1 - tau/n) c(tau)), which differs measurably from the exact value for the
  FIR with the same spectrum samples and from theta (eq. 1).
"""
import math

import numpy as np
import pytest

from paper_1905_02521_amd import qtb
from tests.closed_forms import (baoab_mode_map, block_noise_autocovariance, ho_energy_discrete,
                                stationary_moments_cov, theta_coth)
from tests.gpu_common import units_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()


def block_ctx(omegas, P, *, T, gamma, dt, noise, prec, n, seed, K=64, obs_every=0, pos=None):
    N = len(omegas)
    pos = np.zeros((P, 1, N)) if pos is None else pos
    rep = qtb.Replica(pos=pos, species=np.zeros(N, np.int32), T=T, gamma=gamma, dt=dt,
                      noise=noise, seed=seed, stream=2, harm_omega=np.asarray(omegas, float))
    fir = qtb.FIR_FP64 if prec == qtb.PREC_FP64 else qtb.FIR_FP32
    return qtb.Context(dict(kind=qtb.POT_HARMONIC, mass=(1.0,)), [rep], units_dict(True),
                       prec=prec, fir=fir, fir_block_K=K, obs_every=obs_every, max_two_nf=n,
                       noise_blocks=True)


@pytest.mark.parametrize("prec,tol", [(qtb.PREC_FP64, 1e-12), (qtb.PREC_FP32, 1e-6)])
@pytest.mark.parametrize("P,noise", [(1, 1), (4, 2)])
def test_block_noise_matches_oracle(orc, prec, tol, P, noise):
    n, K, T, dt, seed = 128, 64, 0.3, 0.25, 17
    N = 75
    om = np.linspace(0.5, 3.0, N)
    ctx = block_ctx(om, P, T=T, gamma=0.1, dt=dt, noise=noise, prec=prec, n=n, seed=seed, K=K,
                    pos=np.full((P, 1, N), 0.2))
    ctx.build_filter(0, noise, n)
    ctx.step(10)
    ctx.build_filter(0, noise, n)   # the next noise blocks start at step 10, off the K grid
    rows, start = [], None
    for _ in range(5):
        ctx.step(K)
        z, n0 = ctx.get_noise(0)
        start = n0 if start is None else start
        assert n0 == start + K * len(rows)
        rows.append(z)
    ctx.close()
    z = np.concatenate(rows)                       # steps 10 .. 329
    assert start == 10
    U = orc.make_units(1.0, 1.0)
    S = orc.noise_spectrum(noise, T, P, dt, n, U)
    ref = np.concatenate([orc.eq9_block(S, seed, 2, B * n, N * P) for B in range(3)])[10:330]
    err = np.max(np.abs(z - ref)) / np.std(ref)
    print(f"P={P} prec={prec}: max |zeta - oracle| / sd = {err:.2e}")
    assert err <= tol


def test_block_noise_option_errors():
    om = np.ones(8)
    for n in (96, 32, 8192):   # not a power of two; shorter than K; longer than 4096
        with pytest.raises(qtb.QtbError):
            block_ctx(om, 1, T=1.0, gamma=1.0, dt=0.1, noise=1, prec=qtb.PREC_FP64, n=n, seed=0)
    rep = qtb.Replica(pos=np.zeros((1, 1, 8)), species=np.zeros(8, np.int32), T=1.0, gamma=1.0,
                      dt=0.1, noise=1, harm_omega=om)
    with pytest.raises(qtb.QtbError):  # not with the one-kernel step
        qtb.Context(dict(kind=qtb.POT_HARMONIC, mass=(1.0,)), [rep], units_dict(True),
                    prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, max_two_nf=256, noise_blocks=True,
                    fuse=True)
    ctx = block_ctx(om, 1, T=1.0, gamma=1.0, dt=0.1, noise=1, prec=qtb.PREC_FP64, n=256, seed=0)
    with pytest.raises(qtb.QtbError):
        ctx.build_filter(0, 1, 128)   # the block length is max_two_nf
    ctx.close()


def test_block_noise_oscillator_energy_matches_exact():
    """4096 oscillators, omega = 2, k_B T = 0.4, dt = 0.05, gamma = 0.02,
    blocks of n = 1024 steps (grid spacing 0.123 rad/time; the resonance lies
    0.3 of a spacing above a grid frequency, where the blocks' spectrum takes
    in power leaked from the whole rising band): 12 blocks of 16 384 steps
    after 20 000."""
    omega, T, gamma, dt, n = 2.0, 0.4, 0.02, 0.05, 1024
    N = 4096
    ctx = block_ctx(np.full(N, omega), 1, T=T, gamma=gamma, dt=dt, noise=1, prec=qtb.PREC_FP64,
                    n=n, seed=5, obs_every=8)
    taps = ctx.build_filter(0, 1, n)
    ctx.step(20_000)
    ctx.observables(0)
    e = []
    for _ in range(12):
        ctx.step(16_384)
        e.append(ctx.observables(0)["e_primitive"] / N)
    ctx.close()
    e = np.array(e)
    m, se = e.mean(), e.std(ddof=1) / math.sqrt(len(e))
    # exact for block noise: the scheme's response to the time-averaged autocovariance
    c1 = math.exp(-gamma * dt)
    M, b = baoab_mode_map(omega * omega, 0.0, c1, math.sqrt(1 - c1 * c1), dt)
    h = n // 2
    w = 2 * math.pi * np.arange(h + 1) / (n * dt)
    S = np.array([theta_coth(x, T, 1.0) for x in w])
    R = block_noise_autocovariance(S, n)
    X = stationary_moments_cov(M, b, R)
    E_blocks = 0.5 * X[1, 1] + 0.5 * omega * omega * X[0, 0]
    E_fir = ho_energy_discrete(omega, 1.0, 1, T, 1.0, gamma, dt, taps)[0]
    th = theta_coth(omega, T, 1.0)
    print(f"block noise: gpu {m:.5f} +- {se:.5f}, exact (blocks) {E_blocks:.5f}, "
          f"exact (FIR, same grid) {E_fir:.5f}, theta {th:.5f}")
    assert abs(m - E_blocks) < 2.5 * se
    assert abs(E_blocks - E_fir) > 4 * se    # the two generators are told apart


def test_block_noise_batched_replicas(orc):
    """Three replicas in one context (QTB P = 1, QTB-PIMD P = 4, classical
    P = 2; different T, dt, seeds, streams and dof counts, so their columns
    share 256-column tiles' boundaries differently): each replica's noise is
    its own oracle eq. 9 block."""
    n, K = 256, 64
    specs = [(1, 1, 0.3, 0.25, 11, 37), (4, 2, 0.5, 0.1, 12, 21), (2, 0, 0.8, 0.2, 13, 50)]
    reps = []
    for P, noise, T, dt, seed, N in specs:
        om = np.linspace(0.5, 2.5, N)
        reps.append(qtb.Replica(pos=np.full((P, 1, N), 0.1), species=np.zeros(N, np.int32), T=T,
                                gamma=0.2, dt=dt, noise=noise, seed=seed, stream=seed % 5,
                                harm_omega=om))
    ctx = qtb.Context(dict(kind=qtb.POT_HARMONIC, mass=(1.0,)), reps, units_dict(True),
                      prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, fir_block_K=K, max_two_nf=n,
                      noise_blocks=True)
    for r, (P, noise, *_rest) in enumerate(specs):
        if noise:
            ctx.build_filter(r, noise, n)
    got = [[] for _ in specs]
    for _ in range(n // K + 2):   # into the second block
        ctx.step(K)
        for r in range(len(specs)):
            got[r].append(ctx.get_noise(r)[0])
    ctx.close()
    U = orc.make_units(1.0, 1.0)
    for r, (P, noise, T, dt, seed, N) in enumerate(specs):
        z = np.concatenate(got[r])
        S = orc.noise_spectrum(noise, T, P, dt, n, U)
        ref = np.concatenate([orc.eq9_block(S, seed, seed % 5, B * n, N * P) for B in range(2)])
        ref = ref[: len(z)]
        err = np.max(np.abs(z - ref)) / np.std(ref)
        print(f"replica {r} (P={P}, noise={noise}): {err:.2e}")
        assert err <= 1e-12
