"""Pins of the oracle's sampled observables (orc_sim_observe): the centroid
virial energy, the kinetic temperature and the mean square displacement,
beside the eq. (5) terms.

* On a set state of harmonic oscillators every field is computed by hand from
  the state (the centroid virial energy through its harmonic normal-mode form,
  which does not use the forces), so a sign or factor slip in any term fails.
* Statistically, the centroid virial energy of classical PIMD (eq. 3-5) and of
  QTB-PIMD (eq. 10-12) oscillators matches the exact stationary value of the
  discrete scheme; that value tends to the closed-form P-bead energy (PIMD) and
  to theta of eq. (1) (QTB-PIMD), where the estimator agrees with eq. (5).
"""
import math

import numpy as np
import pytest

from tests.closed_forms import (ho_energy_discrete, ho_virial_discrete, pimd_ho_energy,
                                theta_coth)

NAMES = ("kinetic", "potential", "spring", "e_primitive", "e_virial", "t_kinetic", "x2_mean")


def ho_sim(orc, *, P, noise, T, gamma, dt, two_nf, n_osc, omega, m=1.0, pos0=None, vel0=None,
           seed=1):
    U = orc.make_units(1.0, 1.0)
    pot = orc.make_pot(1, (m,))
    if pos0 is None:
        pos0 = np.zeros((P, 1, n_osc))
    return orc.Sim(pot, U, n_osc, P, 1, None, np.zeros(n_osc, np.int32), T, gamma, dt, seed, 0,
                   noise, two_nf, pos0, vel0=vel0, harm_omega=np.asarray(omega, float),
                   n_threads=4)


@pytest.mark.parametrize("P", [1, 3, 4])
def test_observables_on_a_set_state(orc, P):
    """Every field against its definition, evaluated by hand on the state the
    oracle holds after a few steps from a random start."""
    rng = np.random.default_rng(7 + P)
    n, m, T = 5, 1.7, 0.6
    omega = rng.uniform(0.5, 3.0, n)
    x0 = rng.normal(0.0, 0.7, (P, 1, n))
    v0 = rng.normal(0.0, 0.9, (P, 1, n))
    s = ho_sim(orc, P=P, noise=0, T=T, gamma=0.3, dt=0.05, two_nf=2, n_osc=n, omega=omega, m=m,
               pos0=x0, vel0=v0)
    s.run(7)
    o = dict(zip(NAMES, s.observe()))
    x, v, _, step = s.state()
    x, v = x[:, 0, :], v[:, 0, :]
    assert step == 7
    wP = math.sqrt(P) * T  # omega_P = sqrt(P) k_B T / hbar
    K = 0.5 * m * np.sum(v * v)
    Upot = np.sum(0.5 * m * omega**2 * x * x) / P
    S = 0.5 * m * wP**2 * np.sum((x - np.roll(x, -1, axis=0)) ** 2) if P > 1 else 0.0
    xc, vc = x.mean(axis=0), v.mean(axis=0)
    Kc = np.sum(0.5 * m * P * vc * vc)
    Evir = Kc + np.sum(0.5 * m * omega**2 * xc * xc) + np.sum(m * omega**2 / P * (x - xc) ** 2)
    assert o["kinetic"] == pytest.approx(K, rel=1e-13)
    assert o["potential"] == pytest.approx(Upot, rel=1e-13)
    assert o["spring"] == pytest.approx(S, rel=1e-12, abs=1e-14)
    assert o["e_primitive"] == pytest.approx(K - S + Upot, rel=1e-12)
    assert o["e_virial"] == pytest.approx(Evir, rel=1e-12)
    assert o["t_kinetic"] == pytest.approx(2 * K / (n * P), rel=1e-13)
    assert o["x2_mean"] == pytest.approx(np.mean((x - x0[:, 0, :]) ** 2), rel=1e-12)
    if P == 1:  # one bead: the centroid is the particle, both estimators coincide
        assert o["e_virial"] == pytest.approx(o["e_primitive"], rel=1e-13)


def batch_mean_se(x, n_batch=20):
    b = np.array([c.mean() for c in np.array_split(np.asarray(x), n_batch)])
    return b.mean(), b.std(ddof=1) / math.sqrt(n_batch)


def test_pimd_oscillator_virial_energy(orc):
    """Classical PIMD (white noise): <E_vir> equals the exact discrete value,
    which is within 2% of the closed-form P-bead energy, and <E_prim> agrees."""
    P, omega, T, gamma, dt, n = 4, 2.0, 0.5, 0.5, 0.02, 128
    s = ho_sim(orc, P=P, noise=0, T=T, gamma=gamma, dt=dt, two_nf=2, n_osc=n,
               omega=np.full(n, omega))
    s.run(400)
    obs = s.run(6000, obs_every=6)
    ev = obs[:, NAMES.index("e_virial")] / n
    ep = obs[:, NAMES.index("e_primitive")] / n
    Ed_vir = ho_virial_discrete(omega, 1.0, P, T, 1.0, gamma, dt, s.taps())
    Ed_prim, _, _ = ho_energy_discrete(omega, 1.0, P, T, 1.0, gamma, dt, s.taps())
    m_v, se_v = batch_mean_se(ev)
    m_p, se_p = batch_mean_se(ep)
    assert abs(m_v - Ed_vir) < 4 * se_v, (m_v, Ed_vir, se_v)
    assert abs(m_p - Ed_prim) < 4 * se_p, (m_p, Ed_prim, se_p)
    closed = pimd_ho_energy(omega, T, 1.0, P)
    assert abs(Ed_vir / closed - 1) < 0.02
    # the virial estimator has the smaller variance (it drops the internal modes' kinetic energy)
    assert ev.std() < ep.std()


@pytest.mark.parametrize("P", [2, 4])
def test_qtb_pimd_oscillator_virial_energy(orc, P):
    """QTB-PIMD: <E_vir> matches the exact discrete value; with a resolved filter
    and gamma -> 0 that value is theta of eq. (1) (eq. 10 through the centroid
    mode's own kappa_P), and it differs from the white-noise centroid term
    k_B T / 2 by far more than the error bar."""
    omega, T, gamma, dt, two_nf, n = 5.0, 0.3, 0.1, 0.04, 512, 128
    s = ho_sim(orc, P=P, noise=2, T=T, gamma=gamma, dt=dt, two_nf=two_nf, n_osc=n,
               omega=np.full(n, omega))
    s.run(1500)
    obs = s.run(12000, obs_every=6)
    ev = obs[:, NAMES.index("e_virial")] / n
    Ed = ho_virial_discrete(omega, 1.0, P, T, 1.0, gamma, dt, s.taps())
    m_v, se_v = batch_mean_se(ev)
    assert abs(m_v - Ed) < 4 * se_v, (m_v, Ed, se_v)
    th = theta_coth(omega, T, 1.0)
    U = orc.make_units(1.0, 1.0)
    h = orc.taps(2, T, P, dt, 4096, U)
    E0 = ho_virial_discrete(omega, 1.0, P, T, 1.0, 0.002, dt, h)
    assert abs(E0 / th - 1) < 3e-3
    # a centroid kinetic term of k_B T / 2 (exact only for white noise) would be off
    wrong = m_v + 0.5 * T - 0.5 * orc.kappa(omega / math.sqrt(P), T, P, U)
    assert abs(wrong - Ed) > 5 * se_v


def test_qtb_single_bead_virial_is_primitive(orc):
    """P = 1 (QTB): the centroid virial and primitive energies are the same
    number in every sample."""
    n = 32
    s = ho_sim(orc, P=1, noise=1, T=0.4, gamma=0.1, dt=0.04, two_nf=256, n_osc=n,
               omega=np.linspace(0.5, 3.0, n))
    obs = s.run(600, obs_every=20)
    assert np.allclose(obs[:, NAMES.index("e_virial")], obs[:, NAMES.index("e_primitive")],
                       rtol=1e-13, atol=0)
