"""Pins of the oracle's integrator: QTB (eq. 7-8), PIMD (eq. 3-5), QTB-PIMD
(eq. 10-12) on harmonic oscillators, where the answer is known exactly.

For a harmonic system every normal mode obeys a linear map, so the exact
stationary moments of the discrete scheme driven by the realised FIR noise
(``closed_forms.stationary_moments``) give the target without statistics of
our own making; the continuous-time limits (theta of eq. 1 for QTB, the
closed-form P-bead energy for PIMD, theta again for QTB-PIMD through eq. 10)
are checked at settings where the discretisation error is small.  Statistical
errors come from independent oscillators (one per degree of freedom).
At gamma = 0 the step is symplectic: energy conservation and time reversal.
"""
import math

import numpy as np
import pytest

from paper_1905_02521_amd import workloads as W
from tests.closed_forms import ho_energy_discrete, pimd_ho_energy, theta_coth


def run_ho(orc, *, omega, P, noise, T, gamma, dt, two_nf, n_osc, n_eq, n_run, every,
           seed=1):
    """Integrate n_osc identical 1D oscillators; return per-oscillator time
    averages of E_prim (eq. 5 with instantaneous momenta) and bead-mean x^2."""
    U = orc.make_units(1.0, 1.0)
    pot = orc.make_pot(1, (1.0,))
    s = orc.Sim(pot, U, n_osc, P, 1, None, np.zeros(n_osc, np.int32), T, gamma, dt, seed, 0,
                noise, two_nf, np.zeros((P, 1, n_osc)), harm_omega=np.full(n_osc, omega),
                n_threads=4)
    s.run(n_eq)
    wP = math.sqrt(P) * T
    E = np.zeros(n_osc)
    X2 = np.zeros(n_osc)
    ns = 0
    for _ in range(n_run // every):
        s.run(every)
        r, v, _, _ = s.state()
        r, v = r[:, 0, :], v[:, 0, :]
        ke = 0.5 * np.sum(v * v, axis=0)
        spring = 0.5 * wP * wP * np.sum((r - np.roll(r, -1, axis=0)) ** 2, axis=0) if P > 1 else 0
        pot_e = 0.5 * omega * omega * np.sum(r * r, axis=0) / P
        E += ke - spring + pot_e
        X2 += np.mean(r * r, axis=0)
        ns += 1
    return E / ns, X2 / ns, s


def mean_se(x):
    return x.mean(), x.std(ddof=1) / math.sqrt(len(x))


@pytest.mark.parametrize("omega", [0.5, 1.0, 3.0])
def test_qtb_oscillator_exact_discrete_moments(orc, omega):
    T, gamma, dt, two_nf = 0.3, 0.25, 0.08, 128
    E, X2, s = run_ho(orc, omega=omega, P=1, noise=1, T=T, gamma=gamma, dt=dt, two_nf=two_nf,
                      n_osc=128, n_eq=600, n_run=12000, every=6)
    Ed, x2d, _ = ho_energy_discrete(omega, 1.0, 1, T, 1.0, gamma, dt, s.taps())
    m, se = mean_se(E)
    assert abs(m - Ed) < 4 * se, (m, Ed, se)
    m2, se2 = mean_se(X2)
    assert abs(m2 - x2d) < 4 * se2
    # the quantum result differs from the classical one by much more than the error bar
    assert abs(theta_coth(omega, T, 1.0) - T) > 10 * se or omega < 1.0


def test_qtb_reproduces_theta_when_resolved(orc):
    """Small gamma dt and a resolved filter: the exact discrete <E> is theta(omega)
    of eq. (1) within 1%; at gamma dt = 2.5e-3 the simulation matches it."""
    omega, T, dt = 2.0, 0.4, 0.05
    U = orc.make_units(1.0, 1.0)
    th = theta_coth(omega, T, 1.0)
    h = orc.taps(1, T, 1, dt, 2048, U)
    Ed, _, _ = ho_energy_discrete(omega, 1.0, 1, T, 1.0, 0.005, dt, h)
    assert abs(Ed / th - 1) < 0.01
    # the friction tail up to Nyquist is the residual (frictional caveat of Sec. 3): it grows with gamma
    Ed2, _, _ = ho_energy_discrete(omega, 1.0, 1, T, 1.0, 0.05, dt, h)
    assert Ed2 / th - 1 > Ed / th - 1 > 0
    E, _, s = run_ho(orc, omega=omega, P=1, noise=1, T=T, gamma=0.05, dt=dt, two_nf=512,
                     n_osc=96, n_eq=4000, n_run=24000, every=8)
    m, se = mean_se(E)
    Ed3, _, _ = ho_energy_discrete(omega, 1.0, 1, T, 1.0, 0.05, dt, s.taps())
    assert abs(m - Ed3) < 4 * se


def test_classical_baoab_configurational_exactness(orc):
    # white noise: BAOAB samples <w^2 x^2> = kT/m exactly and <v^2> = kT/m (1 - w^2 dt^2/4)
    omega, T, dt = 1.5, 0.7, 0.3
    _, X2, s = run_ho(orc, omega=omega, P=1, noise=0, T=T, gamma=0.5, dt=dt, two_nf=2,
                      n_osc=128, n_eq=200, n_run=6000, every=3)
    m, se = mean_se(X2 * omega * omega)
    assert abs(m - T) < 4 * se
    M_exact = T / omega**2
    Ed, x2d, ke = ho_energy_discrete(omega, 1.0, 1, T, 1.0, 0.5, dt, s.taps())
    assert abs(x2d - M_exact) < 1e-12
    assert abs(2 * ke - T * (1 - omega**2 * dt**2 / 4)) < 1e-12


@pytest.mark.parametrize("P", [4, 8])
def test_pimd_oscillator_energy(orc, P):
    """Classical PIMD on a harmonic oscillator: eq. (5) vs the exact discrete
    value, which itself tends to the closed-form <E>_P as dt -> 0."""
    omega, T, gamma, dt = 2.0, 0.5, 0.5, 0.02
    E, _, s = run_ho(orc, omega=omega, P=P, noise=0, T=T, gamma=gamma, dt=dt, two_nf=2,
                     n_osc=128, n_eq=400, n_run=6000, every=6)
    Ed, _, _ = ho_energy_discrete(omega, 1.0, P, T, 1.0, gamma, dt, s.taps())
    m, se = mean_se(E)
    assert abs(m - Ed) < 4 * se, (m, Ed, se)
    assert abs(Ed / pimd_ho_energy(omega, T, 1.0, P) - 1) < 0.02


def test_pimd_closed_form_limits():
    # P = 1 is classical; large P tends to theta (eq. 1)
    assert pimd_ho_energy(2.0, 1.0, 1.0, 1) == 1.0
    assert abs(pimd_ho_energy(2.0, 1.0, 1.0, 2) - 1.2) < 1e-12
    assert abs(pimd_ho_energy(2.0, 1.0, 1.0, 4096) / theta_coth(2.0, 1.0, 1.0) - 1) < 1e-6
    # equals the mode sum (kT/P) sum_k w^2 / w_k^2 with eq. (11)
    for P in (2, 8, 32):
        wP = math.sqrt(P)
        s = sum(4.0 / (4.0 / P + 4 * wP * wP * math.sin(k * math.pi / P) ** 2) for k in range(P)) / P
        assert abs(s - pimd_ho_energy(2.0, 1.0, 1.0, P)) < 1e-12


@pytest.mark.parametrize("P", [2, 4])
def test_qtb_pimd_oscillator(orc, P):
    """QTB-PIMD: noise with PSD kappa_P on the normal modes (eq. 10-12).  Eq. (5)
    matches the exact discrete value, which tends to theta for any P."""
    omega, T = 3.0, 0.4
    gamma, dt, two_nf = 0.1, 0.04, 512
    E, _, s = run_ho(orc, omega=omega, P=P, noise=2, T=T, gamma=gamma, dt=dt, two_nf=two_nf,
                     n_osc=96, n_eq=1500, n_run=9000, every=6)
    Ed, _, _ = ho_energy_discrete(omega, 1.0, P, T, 1.0, gamma, dt, s.taps())
    m, se = mean_se(E)
    assert abs(m - Ed) < 4 * se, (m, Ed, se)
    th = theta_coth(omega, T, 1.0)
    # and it is far from plain PIMD with the same P
    assert abs(th - pimd_ho_energy(omega, T, 1.0, P)) > 20 * se
    # gamma -> 0 with a resolved filter: eq. (10) makes <E_prim> = theta exactly
    U = orc.make_units(1.0, 1.0)
    h = orc.taps(2, T, P, dt, 4096, U)
    E0, _, _ = ho_energy_discrete(omega, 1.0, P, T, 1.0, 0.002, dt, h)
    assert abs(E0 / th - 1) < 3e-3
    h1 = orc.taps(2, T, P, dt, 2048, U)
    E1, _, _ = ho_energy_discrete(omega, 1.0, P, T, 1.0, 0.01, dt, h1)
    assert abs(E0 / th - 1) < abs(E1 / th - 1) < abs(Ed / th - 1)


def test_nm_matrix_orthonormal_and_diagonalises_ring(orc):
    for P in (1, 2, 3, 4, 5, 8, 32):
        C = orc.nm_matrix(P)
        assert np.allclose(C.T @ C, np.eye(P), atol=1e-14)
        K = 2 * np.eye(P) - np.roll(np.eye(P), 1, 0) - np.roll(np.eye(P), -1, 0)
        if P == 1:
            K = np.zeros((1, 1))
        lam = 4 * np.sin(np.pi * np.arange(P) / P) ** 2
        assert np.allclose(C.T @ K @ C, np.diag(lam), atol=1e-12)


def crystal_sim(orc, n, P, gamma, T=100.0, dt=1.0, noise=0, two_nf=2, seed=3):
    U = orc.make_units(**W.METAL_UNITS)
    p = W.mgo_potential()
    pot = orc.make_pot(0, p.mass, p.charge, p.buck_A, p.buck_rho, p.buck_C,
                       p.dsf_alpha, p.r_cut, p.skin)
    pos, sp, box = W.rocksalt(n)
    beads = np.stack([W.displaced(pos, 0.0421, seed + b) for b in range(P)])
    return orc.Sim(pot, U, pos.shape[1], P, 3, box, sp, T, gamma, dt, 5, 0, noise, two_nf,
                   beads, n_threads=8)


@pytest.mark.parametrize("P", [1, 4])
def test_gamma_zero_conserves_energy(orc, P):
    s = crystal_sim(orc, 2, P, gamma=0.0, dt=0.5)
    H0 = s.hamiltonian()
    Hs = []
    for _ in range(20):
        s.run(10)
        Hs.append(s.hamiltonian())
    Hs = np.array(Hs)
    ke_scale = 0.5 * 3 * 64 * P * 8.617333262e-5 * 100.0
    assert np.max(np.abs(Hs - H0)) < 5e-3 * ke_scale
    # no drift: second half fluctuates around the same value as the first
    assert abs(Hs[10:].mean() - Hs[:10].mean()) < 2e-3 * ke_scale


def test_gamma_zero_time_reversible(orc):
    s = crystal_sim(orc, 2, 4, gamma=0.0, dt=1.0)
    r0, v0, _, _ = s.state()
    s.run(50)
    r1, v1, _, _ = s.state()
    U = orc.make_units(**W.METAL_UNITS)
    p = W.mgo_potential()
    pot = orc.make_pot(0, p.mass, p.charge, p.buck_A, p.buck_rho, p.buck_C,
                       p.dsf_alpha, p.r_cut, p.skin)
    pos, sp, box = W.rocksalt(2)
    back = orc.Sim(pot, U, 64, 4, 3, box, sp, 100.0, 0.0, 1.0, 5, 0, 0, 2, r1, vel0=-v1,
                   n_threads=8)
    back.run(50)
    r2, v2, _, _ = back.state()
    assert np.max(np.abs(r2 - r0)) < 1e-9
    assert np.max(np.abs(v2 + v0)) < 1e-12
