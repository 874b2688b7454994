"""The anharmonic 1D models of Sec. 3 (Morse and double well, anharmonicity C
of eq. 13) on the GPU: trajectories against the oracle, and the zero-point
energy leakage measurement against the exact quantum mean energy.

* Parity: 64 oscillators, FP64, QTB (P = 1) and QTB-PIMD (P = 4), 400 steps:
  positions within 1e-9 of the oracle's (relative to the spread of the
  positions); FP32 forces within 1e-6 relative of the oracle's FP64 ones.
* Measurement (reduced units m = hbar = k_B = 1): 4096 oscillators per
  setting; the configurational energy <V> against the exact quantum
  canonical <V>(T) from the Schroedinger eigenpairs.
"""
import math

import numpy as np
import pytest

from paper_1905_02521_amd import qtb
from tests.closed_forms import (double_well_potential, morse_potential, quantum_mean_potential,
                                schrodinger_levels)
from tests.gpu_common import units_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()


def onsite_ctx(kind, V0, d, x0, P, *, T, gamma, dt, noise, prec, fir, seed, two_nf,
               obs_every=0, vel=None):
    N = x0.shape[-1]
    pos = np.broadcast_to(np.asarray(x0, dtype=np.float64).reshape(1, 1, N), (P, 1, N)).copy()
    rep = qtb.Replica(pos=pos, species=np.zeros(N, np.int32), T=T, gamma=gamma, dt=dt,
                      noise=noise, vel=vel, seed=seed)
    return qtb.Context(dict(kind=kind, mass=(1.0,), V0=(V0,), d=(d,)), [rep], units_dict(True),
                       prec=prec, fir=fir, max_two_nf=two_nf, obs_every=obs_every)


def start_positions(kind, d, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 0.2 * d, n)
    return x + (d * np.sign(rng.uniform(-1, 1, n)) if kind == qtb.POT_DOUBLE_WELL else 0.0)


@pytest.mark.parametrize("kind", [qtb.POT_MORSE, qtb.POT_DOUBLE_WELL])
@pytest.mark.parametrize("P,noise", [(1, 1), (4, 2)])
def test_onsite_trajectory_fp64(orc, kind, P, noise):
    V0, d, T, gamma, dt, two_nf = 1.0, 1.0, 0.2, 0.3, 0.02, 256
    x0 = start_positions(kind, d, 64, 5)
    ctx = onsite_ctx(kind, V0, d, x0, P, T=T, gamma=gamma, dt=dt, noise=noise,
                     prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=9, two_nf=two_nf)
    ctx.build_filter(0, noise, two_nf)
    pot = orc.make_pot(kind, (1.0,), V0=(V0,), d=(d,))
    pos = np.broadcast_to(x0.reshape(1, 1, -1), (P, 1, len(x0))).copy()
    osim = orc.Sim(pot, orc.make_units(1.0, 1.0), len(x0), P, 1, None,
                   np.zeros(len(x0), np.int32), T, gamma, dt, 9, 0, noise, two_nf, pos,
                   n_threads=4)
    ctx.step(400)
    osim.run(400)
    r, v, st = ctx.get_state(0)
    ro, vo, _, sto = osim.state()
    assert st == sto == 400
    scale = np.std(ro)
    assert np.sqrt(np.mean((r - ro) ** 2)) / scale <= 1e-9
    assert np.sqrt(np.mean((v - vo) ** 2)) / np.std(vo) <= 1e-9


@pytest.mark.parametrize("kind", [qtb.POT_MORSE, qtb.POT_DOUBLE_WELL])
def test_onsite_forces_fp32(orc, kind):
    V0, d = 0.8, 0.7
    x0 = start_positions(kind, d, 256, 6)
    ctx = onsite_ctx(kind, V0, d, x0, 1, T=0.2, gamma=0.1, dt=0.01, noise=0,
                     prec=qtb.PREC_FP32, fir=qtb.FIR_FP32, seed=1, two_nf=2)
    f, e = ctx.evaluate(0)
    pot = orc.make_pot(kind, (1.0,), V0=(V0,), d=(d,))
    osim = orc.Sim(pot, orc.make_units(1.0, 1.0), len(x0), 1, 1, None, np.zeros(len(x0), np.int32),
                   0.2, 0.1, 0.01, 1, 0, 0, 2, x0.reshape(1, 1, -1))
    _, _, fo, _ = osim.state()
    assert np.max(np.abs(f - fo)) <= 1e-6 * np.max(np.abs(fo))
    assert abs(e[0] - osim.observe()[1]) <= 1e-12 * abs(e[0])


def exact_means(kind, V0, d, hbar, T):
    """Exact quantum canonical (<V>, <E>) of one oscillator."""
    if kind == qtb.POT_MORSE:
        x = np.linspace(-1.0 * d, 25.0 * d, 12001)[1:-1]
        V = morse_potential(x, V0, d)
    else:
        x = np.linspace(-2.6 * d, 2.6 * d, 8001)[1:-1]
        V = double_well_potential(x, V0, d)
    # the levels that k_B T reaches (the Morse box adds states above V0 whose
    # weight is below e^{-V0 / k_B T})
    lev = schrodinger_levels(V, 1.0, hbar, x)
    n = int(np.sum(lev < lev[0] + 40.0 * T))
    return quantum_mean_potential(V, 1.0, hbar, x, T, max(n, 2))


def gpu_means(kind, V0, d, P, noise, T, gamma, dt, two_nf, n=4096, n_eq=20000, block=10000,
               n_blocks=8, seed=3):
    x0 = start_positions(kind, d, n, seed)
    ctx = onsite_ctx(kind, V0, d, x0, P, T=T, gamma=gamma, dt=dt, noise=noise,
                     prec=qtb.PREC_FP64, fir=qtb.FIR_FP64, seed=seed, two_nf=two_nf,
                     obs_every=8)
    if noise:
        ctx.build_filter(0, noise, two_nf)
    ctx.step(n_eq)
    ctx.observables(0)
    e, u = [], []
    for _ in range(n_blocks):
        ctx.step(block)
        o = ctx.observables(0)
        e.append(o["e_primitive"] / n)
        u.append(o["potential"] / n)
    ctx.close()
    e, u = np.array(e), np.array(u)
    se = lambda a: a.std(ddof=1) / math.sqrt(len(a))
    return (u.mean(), se(u)), (e.mean(), se(e))


def _dev(kind, V0, T, P, noise, g_over_w, exact_V):
    d = 1.0
    w0 = math.sqrt(2 * V0) / d if kind == qtb.POT_MORSE else math.sqrt(8 * V0) / d
    (u, su), _ = gpu_means(kind, V0, d, P, noise, T, g_over_w * w0, 0.05 / w0,
                           1024 if noise else 2)
    return (u - exact_V) / exact_V, su / exact_V


def test_zero_point_leakage_and_its_cures():
    """The claims of Sec. 3 on the exact quantum configurational energy <V>
    (the total energy with instantaneous momenta carries the friction tail of
    any Langevin scheme and is not used here):
    * Morse with C = 0.05, above the critical 0.01: QTB at small gamma leaks
      zero-point energy into the dissociative motion and misses <V> by far;
      raising gamma to omega_0 cures most of it; QTB-PIMD (P = 8) is within 3 %.
    * Double well with C = 0.3, above the critical 0.1: QTB misses by about a
      fifth whatever gamma; QTB-PIMD converges with P, and with P = 8 it is
      closer to the exact value than PIMD with the same P."""
    kind, V0, T = qtb.POT_MORSE, 10.0, 1.0                       # C = 1 / (2 V0) = 0.05
    exV, _ = exact_means(kind, V0, 1.0, 1.0, T)
    lo, _ = _dev(kind, V0, T, 1, 1, 0.05, exV)
    hi, s_hi = _dev(kind, V0, T, 1, 1, 1.0, exV)
    qp8, s_qp8 = _dev(kind, V0, T, 8, 2, 0.05, exV)
    print(f"Morse C=0.05: QTB g=0.05w {lo:+.3f}, g=w {hi:+.3f}, QTB-PIMD P=8 {qp8:+.4f}")
    assert abs(lo) > 5 * abs(hi) and abs(lo) > 0.5
    assert abs(qp8) < 0.03
    kind, V0, T = qtb.POT_DOUBLE_WELL, 5.0 / 3.0, 0.5            # C = 0.3
    exV, _ = exact_means(kind, V0, 1.0, 1.0, T)
    q, _ = _dev(kind, V0, T, 1, 1, 0.2, exV)
    qp4, _ = _dev(kind, V0, T, 4, 2, 0.05, exV)
    qp8, _ = _dev(kind, V0, T, 8, 2, 0.05, exV)
    p8, _ = _dev(kind, V0, T, 8, 0, 0.2, exV)
    print(f"double well C=0.3: QTB {q:+.3f}, QTB-PIMD P=4 {qp4:+.4f} P=8 {qp8:+.4f}, "
          f"PIMD P=8 {p8:+.4f}")
    assert abs(q) > 0.1
    assert abs(qp8) < abs(qp4) < abs(q)
    assert abs(qp8) < 0.5 * abs(p8)
