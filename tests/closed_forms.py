"""Closed forms that pin the oracle (written from the mathematics, not from it).

* ``pimd_ho_energy``: exact <E_prim> of a P-bead harmonic ring polymer with the
  paper's conventions (bead mass m, V/P, omega_P = sqrt(P)/(beta hbar), eq. 3-5),
  from the product form of Z_P: sinh(a/2) = beta hbar omega / (2P),
  <E>_P = (hbar omega/2) coth(P a/2) / cosh(a/2).
* ``stationary_moments``: exact stationary covariance of the discrete linear
  scheme z_{n+1} = M z_n + b zeta_n driven by the FIR noise zeta = h * w,
  using the noise autocorrelation R(tau) = sum_k h_k h_{k+tau} and the
  discrete Lyapunov solution X0 = M X0 M^T + b b^T:
  Sigma = R(0) X0 + sum_{tau>0} R(tau) (X0 (M^tau)^T + M^tau X0).
  This is the exact answer of the integrator for harmonic systems, so it
  separates time-step / filter-resolution effects from implementation errors.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_discrete_lyapunov


def theta_coth(omega, kT, hbar):
    """theta = (hbar w/2) coth(hbar w / 2kT): eq. (1) rewritten with coth."""
    x = hbar * abs(omega) / (2 * kT)
    if x == 0:
        return kT
    return hbar * abs(omega) / 2.0 / math.tanh(x)


def pimd_ho_energy(omega, kT, hbar, P):
    if P == 1:
        return kT
    a = 2.0 * math.asinh(hbar * omega / (kT * 2.0 * P))
    return hbar * omega / 2.0 / math.tanh(P * a / 2.0) / math.cosh(a / 2.0)


def baoab_mode_map(acc2, w_free, c1, sigma, dt):
    """One B A O A B step of a single mode: B kicks with acceleration -acc2 q,
    A rotates at w_free (drift if 0) for dt/2, O applies c1 and noise sigma."""
    h = dt / 2.0
    B = np.array([[1.0, 0.0], [-h * acc2, 1.0]])
    if w_free == 0.0:
        A = np.array([[1.0, h], [0.0, 1.0]])
    else:
        c, s = math.cos(w_free * h), math.sin(w_free * h)
        A = np.array([[c, s / w_free], [-w_free * s, c]])
    Om = np.array([[1.0, 0.0], [0.0, c1]])
    M = B @ A @ Om @ A @ B
    b = B @ A @ np.array([0.0, sigma])
    return M, b


def stationary_moments(M, b, taps):
    taps = np.asarray(taps, dtype=np.float64)
    L = len(taps)
    R = np.array([np.dot(taps[: L - t], taps[t:]) for t in range(L)])
    X0 = solve_discrete_lyapunov(M, np.outer(b, b))
    S = R[0] * X0
    Mt = np.eye(len(b))
    for t in range(1, L):
        Mt = Mt @ M
        if R[t] != 0.0:
            S += R[t] * (X0 @ Mt.T + Mt @ X0)
    return S


def ho_energy_discrete(omega, m, P, kT, hbar, gamma, dt, taps):
    """Exact stationary <E_prim> (eq. 5) of the BAOAB / normal-mode scheme on a
    1D harmonic oscillator with P beads, plus <q^2> summed over modes (bead
    averaged <x^2> = sum_k <q_k^2> / P) and the kinetic part."""
    c1 = math.exp(-gamma * dt)
    sigma = math.sqrt((1 - c1 * c1) / m)
    wP = math.sqrt(P) * kT / hbar
    E = 0.0
    x2 = 0.0
    ke = 0.0
    for k in range(P):
        wf = 2 * wP * math.sin(math.pi * k / P)
        M, b = baoab_mode_map(omega * omega / P, wf, c1, sigma, dt)
        S = stationary_moments(M, b, taps)
        q2, v2 = S[0, 0], S[1, 1]
        E += 0.5 * m * v2 - 0.5 * m * wf * wf * q2 + 0.5 * m * omega * omega / P * q2
        x2 += q2
        ke += 0.5 * m * v2
    return E, x2 / P, ke


def ho_virial_discrete(omega, m, P, kT, hbar, gamma, dt, taps):
    """Exact stationary <E_vir> of the same scheme for a 1D harmonic oscillator.

    For V = m w^2 x^2 / 2 the centroid virial estimator is, state by state,
    K_c + (m w^2 / 2) x_c^2 + (m w^2 / P) sum_s (x_s - x_c)^2, with K_c the
    kinetic energy of the centroid mode.  In normal modes (q_0 = sqrt(P) x_c,
    sum_{k>0} q_k^2 = sum_s (x_s - x_c)^2) its mean is
    m <v_0^2> / 2 + (m w^2 / 2P) <q_0^2> + (m w^2 / P) sum_{k>0} <q_k^2>,
    each moment the exact stationary one of the mode's linear map."""
    c1 = math.exp(-gamma * dt)
    sigma = math.sqrt((1 - c1 * c1) / m)
    wP = math.sqrt(P) * kT / hbar
    E = 0.0
    for k in range(P):
        wf = 2 * wP * math.sin(math.pi * k / P)
        M, b = baoab_mode_map(omega * omega / P, wf, c1, sigma, dt)
        S = stationary_moments(M, b, taps)
        if k == 0:
            E += 0.5 * m * S[1, 1] + 0.5 * m * omega * omega / P * S[0, 0]
        else:
            E += m * omega * omega / P * S[0, 0]
    return E


# ------------------------------------------------------------ anharmonic 1D
def morse_potential(x, V0, d):
    return V0 * (1.0 - np.exp(-x / d)) ** 2


def double_well_potential(x, V0, d):
    return V0 * ((x / d) ** 2 - 1.0) ** 2


def schrodinger_levels(V, m, hbar, x):
    """Eigenvalues of -hbar^2/(2m) d^2/dx^2 + V(x) on the uniform grid x with
    zero boundary values (second-order finite differences, symmetric
    tridiagonal, scipy eigh_tridiagonal)."""
    from scipy.linalg import eigh_tridiagonal
    h = x[1] - x[0]
    t = hbar * hbar / (2.0 * m * h * h)
    return eigh_tridiagonal(2.0 * t + V, -t * np.ones(len(x) - 1), eigvals_only=True)


def quantum_mean_energy(levels, kT):
    """Canonical <E> = sum E_n e^{-E_n/kT} / Z over the given levels."""
    w = np.exp(-(levels - levels[0]) / kT)
    return float(np.sum(levels * w) / np.sum(w))


def morse_levels_exact(V0, d, m, hbar, n_max):
    """Textbook bound-state energies of the Morse oscillator (measured from
    the well bottom): E_n = hw (n + 1/2) - (hw)^2 (n + 1/2)^2 / (4 V0),
    w = sqrt(2 V0 / (m d^2)), for n below the dissociation limit."""
    w = math.sqrt(2.0 * V0 / (m * d * d))
    n = np.arange(n_max)
    return hbar * w * (n + 0.5) - (hbar * w) ** 2 * (n + 0.5) ** 2 / (4.0 * V0)


def classical_mean(V, f, x, kT):
    """Classical canonical <f(x)> for one dof with potential V on the grid x
    (trapezoid rule)."""
    w = np.exp(-(V - V.min()) / kT)
    return float(np.trapezoid(f * w, x) / np.trapezoid(w, x))


def quantum_mean_potential(V, m, hbar, x, kT, n_levels):
    """Canonical <V> and <E> from the lowest n_levels eigenpairs of the grid
    Hamiltonian of schrodinger_levels (<n|V|n> as the grid sum of psi_n^2 V)."""
    from scipy.linalg import eigh_tridiagonal
    h = x[1] - x[0]
    t = hbar * hbar / (2.0 * m * h * h)
    E, psi = eigh_tridiagonal(2.0 * t + V, -t * np.ones(len(x) - 1), select="i",
                              select_range=(0, n_levels - 1))
    Vn = np.sum(psi * psi * V[:, None], axis=0) / np.sum(psi * psi, axis=0)
    w = np.exp(-(E - E[0]) / kT)
    return float(np.sum(Vn * w) / np.sum(w)), float(np.sum(E * w) / np.sum(w))


# ------------------------------------------------------- velocity spectrum
def velocity_spectrum_discrete(M, b, taps, phi):
    """Exact power spectrum of v_n for the discrete linear scheme
    z_{n+1} = M z_n + b zeta_n, z = (x, v), driven by zeta = h * w (unit white
    w): S_v(phi) = |[(e^{i phi} I - M)^{-1} b]_v|^2 |sum_k h_k e^{-i k phi}|^2,
    normalised so that <v^2> = (1/2 pi) int_{-pi}^{pi} S_v d phi."""
    taps = np.asarray(taps, dtype=np.float64)
    L = len(taps)
    k = np.arange(L) - L // 2   # taps h_k for k = -Nf .. Nf - 1
    phi = np.asarray(phi, dtype=np.float64)
    Hz = np.exp(-1j * np.outer(phi, k)) @ taps
    out = np.empty(len(phi))
    I = np.eye(2)
    for q, p in enumerate(phi):
        g = np.linalg.solve(np.exp(1j * p) * I - M, b)
        out[q] = abs(g[1]) ** 2 * abs(Hz[q]) ** 2
    return out


def block_noise_autocovariance(S_half, L):
    """Time-averaged autocovariance, lags 0 .. L-1, of noise made in independent
    blocks of n steps by the inverse DFT of Hermitian random amplitudes with
    E|R_j|^2 = n S_j: within a block the covariance is circular,
    c(tau) = (1/n) sum_j S_j cos(2 pi j tau / n); a pair at lag tau shares a
    block for a fraction 1 - tau/n of the positions and is independent
    otherwise."""
    S_half = np.asarray(S_half, dtype=np.float64)
    n = 2 * (len(S_half) - 1)
    S = np.concatenate([S_half, S_half[-2:0:-1]])
    c = np.fft.ifft(S).real
    tau = np.arange(L)
    return np.where(tau < n, (1.0 - tau / n) * c[tau % n], 0.0)


def stationary_moments_cov(M, b, R):
    """Second moments of z_{n+1} = M z_n + b zeta_n for noise with the
    (time-averaged) autocovariance R[tau], tau = 0 .. len(R) - 1."""
    X0 = solve_discrete_lyapunov(M, np.outer(b, b))
    S = R[0] * X0
    Mt = np.eye(len(b))
    for t in range(1, len(R)):
        Mt = Mt @ M
        if R[t] != 0.0:
            S += R[t] * (X0 @ Mt.T + Mt @ X0)
    return S


# ------------------------------------------------ many harmonic modes at once
def ring_mode_moments(omegas, P, kT, hbar, gamma, dt, taps):
    """Exact stationary energies of the BAOAB / normal-mode scheme for many
    independent unit-mass harmonic modes (the mass-weighted normal modes of a
    crystal) at once: the same linear map and FIR-noise covariance sum as
    ``stationary_moments``, vectorised over modes and ring-polymer normal
    modes.  A mode with omega = 0 (a uniform translation) carries only its
    velocity, v_{n+1} = c1 v_n + sigma zeta_n, whose stationary variance is
    sigma^2 (R0 + 2 sum_tau c1^tau R_tau) / (1 - c1^2); its other ring modes
    are bounded by the springs.

    Returns arrays over the physical modes: kinetic, bead-averaged potential
    (omega^2 / 2P sum_k <q_k^2>), spring, E_prim (eq. 5) and the centroid
    virial energy (as in ``ho_virial_discrete``)."""
    taps = np.asarray(taps, dtype=np.float64)
    L = len(taps)
    R = np.array([np.dot(taps[: L - t], taps[t:]) for t in range(L)])
    om = np.asarray(omegas, dtype=np.float64)
    n = len(om)
    c1 = math.exp(-gamma * dt)
    sigma = math.sqrt(1.0 - c1 * c1)
    wP = math.sqrt(P) * kT / hbar
    wf = 2.0 * wP * np.sin(np.pi * np.arange(P) / P)
    acc2 = np.repeat(om * om / P, P)                       # [n*P], mode-major
    wfr = np.tile(wf, n)
    free = (acc2 == 0.0) & (wfr == 0.0)
    h = dt / 2.0
    m = n * P
    B = np.zeros((m, 2, 2)); B[:, 0, 0] = 1.0; B[:, 1, 1] = 1.0; B[:, 1, 0] = -h * acc2
    A = np.zeros((m, 2, 2))
    rot = wfr > 0.0
    c, s = np.cos(wfr * h), np.sin(wfr * h)
    A[:, 0, 0] = np.where(rot, c, 1.0)
    A[:, 0, 1] = np.where(rot, s / np.where(rot, wfr, 1.0), h)
    A[:, 1, 0] = np.where(rot, -wfr * s, 0.0)
    A[:, 1, 1] = np.where(rot, c, 1.0)
    Om = np.zeros((m, 2, 2)); Om[:, 0, 0] = 1.0; Om[:, 1, 1] = c1
    BA = B @ A
    M = BA @ Om @ A @ B
    b = BA @ np.array([0.0, sigma])
    # a free mode gets a stand-in stable map; its moments are set below
    M[free] = np.diag([0.5, 0.5])
    # discrete Lyapunov X = M X M^T + b b^T as a 4x4 linear system per mode
    K4 = np.einsum("nij,nkl->nikjl", M, M).reshape(m, 4, 4)
    rhs = np.einsum("ni,nj->nij", b, b).reshape(m, 4)
    X0 = np.linalg.solve(np.eye(4)[None] - K4, rhs[..., None])[..., 0].reshape(m, 2, 2)
    S = R[0] * X0
    Mt = np.broadcast_to(np.eye(2), (m, 2, 2)).copy()
    for t in range(1, L):
        Mt = Mt @ M
        if R[t] != 0.0:
            XM = X0 @ np.swapaxes(Mt, 1, 2)
            S += R[t] * (XM + np.swapaxes(XM, 1, 2))
    q2 = S[:, 0, 0].copy()
    v2 = S[:, 1, 1].copy()
    if free.any():
        v2[free] = sigma * sigma * (R[0] + 2.0 * np.sum(R[1:] * c1 ** np.arange(1, L))) \
            / (1.0 - c1 * c1)
        q2[free] = 0.0
    q2 = q2.reshape(n, P)
    v2 = v2.reshape(n, P)
    ke = 0.5 * v2.sum(1)
    pot = 0.5 * (om * om / P) * q2.sum(1)
    spring = 0.5 * (q2 * wf[None] ** 2).sum(1)
    e_vir = 0.5 * v2[:, 0] + 0.5 * (om * om / P) * q2[:, 0] + (om * om / P) * q2[:, 1:].sum(1)
    return {"kinetic": ke, "potential": pot, "spring": spring,
            "e_primitive": ke - spring + pot, "e_virial": e_vir}


def quantum_heat_capacity(omegas, kT, hbar):
    """Heat capacity of quantum harmonic modes in units of k_B:
    sum_m (x/2)^2 / sinh^2(x/2), x = hbar omega_m / kT (a zero mode counts
    1/2, its kinetic part)."""
    om = np.asarray(omegas, dtype=np.float64)
    x = hbar * om[om > 0] / kT
    # (x/2)^2 / sinh^2(x/2) = x^2 e^-x / (1 - e^-x)^2, without overflow
    return float(np.sum(x * x * np.exp(-x) / np.expm1(-x) ** 2) + 0.5 * np.sum(om == 0))
