"""Plain FP64 reference of the descriptor-MLP force surrogate.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library; the product path never
imports it, and this module imports nothing from the product package.

The paper has no learned component; this surrogate replaces the pair
potential V of eq. (4) and eq. (8) by a sum of atomic energies, so that the
same integrator step (and the same coloured noise) runs on it.  Definitions
(the library states the same ones in its header):

  per centre atom i and per neighbour species b, over every neighbour j
  (all periodic images) with r = |d_ij| < r_c, d_ij = r_j - r_i:
    f_c(r)      = (cos(pi r / r_c) + 1) / 2
    phi_c(r)    = exp(-eta_r (r - mu_c)^2) f_c(r),  c = 0..31,
                  mu_c = r_min + c dr, dr = (r_c - r_min)/31, eta_r = 1/(2 dr^2)
    psi_k(r)    = exp(-eta_a (r - nu_k)^2) f_c(r),  k = 0..7,
                  nu_k = r_min + k da, da = (r_c - r_min)/7, eta_a = 1/(2 da^2)
    G[b][c]      = sum_j phi_c(r_ij)
    A1[b][k]     = sum_j psi_k(r_ij) rhat_ij                (3-vector)
    A2[b][k]     = sum_j psi_k(r_ij) (rhat rhat^T - I/3)    (3x3)
    G[b][32+k]   = |A1[b][k]|^2,  G[b][40+k] = ||A2[b][k]||_F^2
  features: index 48 b + (0..47); 96 per atom for two species.
  network per centre species a:  x = (G - mu_a) * inv_sd_a,
    z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, h2 = silu(z2),
    E_i = w3 . h2 + b3 + e0_a      (96 -> 64 -> 64 -> 1)
  E = sum_i E_i,  F = -dE/dr.
  training loss over a batch of B frames of N atoms:
    L = w_E / B sum_f ((E_f - E_f^ref)/N)^2 + w_F / (3 N B) sum |F - F^ref|^2.

Everything here is written from these definitions with numpy in FP64: the
per-pair derivatives by explicit tensor formulas, the weight gradient of the
force term by forward-mode differentiation of the input gradient followed by
reverse mode (double back-propagation).
"""
from __future__ import annotations

import numpy as np

N_SPECIES = 2
N_RAD = 32
N_ANG = 8
N_FEAT_SP = N_RAD + 2 * N_ANG      # 48 per neighbour species
N_FEAT = N_SPECIES * N_FEAT_SP     # 96
HIDDEN = 64


def layer_sizes():
    """(name, shape) of one species' trainable block, in storage order."""
    return [("W1", (HIDDEN, N_FEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
            ("b2", (HIDDEN,)), ("w3", (HIDDEN,)), ("b3", (1,))]


def params_per_species():
    return sum(int(np.prod(s)) for _, s in layer_sizes())


def unpack(params):
    """Flat parameter vector [species][block] -> list of dicts per species."""
    params = np.asarray(params, dtype=np.float64)
    n = params_per_species()
    out = []
    for a in range(N_SPECIES):
        blk = params[a * n:(a + 1) * n]
        d, o = {}, 0
        for name, shape in layer_sizes():
            k = int(np.prod(shape))
            d[name] = blk[o:o + k].reshape(shape)
            o += k
        out.append(d)
    return out


def pack(blocks):
    return np.concatenate([np.concatenate([blocks[a][name].ravel() for name, _ in layer_sizes()])
                           for a in range(N_SPECIES)])


def grids(r_cut, r_min):
    dr = (r_cut - r_min) / (N_RAD - 1)
    da = (r_cut - r_min) / (N_ANG - 1)
    mu = r_min + dr * np.arange(N_RAD)
    nu = r_min + da * np.arange(N_ANG)
    return mu, 1.0 / (2 * dr * dr), nu, 1.0 / (2 * da * da)


def neighbour_pairs(pos, box, r_cut):
    """Every (i, j, image) with |r_j - r_i + n L| < r_cut, except i = j at n = 0.
    pos [3][N]; returns i, j, d [n_pairs][3] with d = r_j - r_i + n L."""
    x = np.asarray(pos, dtype=np.float64).T
    box = np.asarray(box, dtype=np.float64)
    N = x.shape[0]
    d0 = x[None, :, :] - x[:, None, :]            # [i][j] r_j - r_i
    d0 -= box * np.rint(d0 / box)
    m = [int(np.ceil(r_cut / L + 0.5)) for L in box]
    I, J, D = [], [], []
    for nx in range(-m[0], m[0] + 1):
        for ny in range(-m[1], m[1] + 1):
            for nz in range(-m[2], m[2] + 1):
                sh = np.array([nx, ny, nz]) * box
                d = d0 + sh
                r2 = np.sum(d * d, axis=-1)
                mask = r2 < r_cut * r_cut
                if nx == 0 and ny == 0 and nz == 0:
                    mask &= ~np.eye(N, dtype=bool)
                ii, jj = np.nonzero(mask)
                I.append(ii)
                J.append(jj)
                D.append(d[ii, jj])
    return np.concatenate(I), np.concatenate(J), np.concatenate(D)


def _radial(r, r_cut, r_min):
    """phi [p][32], dphi/dr, psi [p][8], dpsi/dr for pair distances r."""
    mu, eta_r, nu, eta_a = grids(r_cut, r_min)
    fc = 0.5 * (np.cos(np.pi * r / r_cut) + 1.0)
    dfc = -0.5 * np.pi / r_cut * np.sin(np.pi * r / r_cut)
    gr = np.exp(-eta_r * (r[:, None] - mu[None, :]) ** 2)
    ga = np.exp(-eta_a * (r[:, None] - nu[None, :]) ** 2)
    phi = gr * fc[:, None]
    dphi = gr * (-2.0 * eta_r * (r[:, None] - mu[None, :]) * fc[:, None] + dfc[:, None])
    psi = ga * fc[:, None]
    dpsi = ga * (-2.0 * eta_a * (r[:, None] - nu[None, :]) * fc[:, None] + dfc[:, None])
    return phi, dphi, psi, dpsi


def descriptors(pos, species, box, r_cut=6.0, r_min=0.5):
    """G [N][96], A1 [N][2][8][3], A2 [N][2][8][3][3] and the pair list."""
    species = np.asarray(species)
    N = len(species)
    i, j, d = neighbour_pairs(pos, box, r_cut)
    r = np.sqrt(np.sum(d * d, axis=1))
    rh = d / r[:, None]
    b = species[j]
    phi, _, psi, _ = _radial(r, r_cut, r_min)
    G = np.zeros((N, N_SPECIES, N_FEAT_SP))
    A1 = np.zeros((N, N_SPECIES, N_ANG, 3))
    A2 = np.zeros((N, N_SPECIES, N_ANG, 3, 3))
    M = rh[:, :, None] * rh[:, None, :] - np.eye(3)[None] / 3.0
    for p in range(len(i)):
        G[i[p], b[p], :N_RAD] += phi[p]
        A1[i[p], b[p]] += psi[p][:, None] * rh[p][None, :]
        A2[i[p], b[p]] += psi[p][:, None, None] * M[p][None]
    G[:, :, N_RAD:N_RAD + N_ANG] = np.sum(A1 * A1, axis=-1)
    G[:, :, N_RAD + N_ANG:] = np.sum(A2 * A2, axis=(-1, -2))
    return G.reshape(N, N_FEAT), A1, A2, (i, j, d, b)


def silu(z):
    """silu, its first and second derivatives."""
    s = 1.0 / (1.0 + np.exp(-z))
    return z * s, s * (1.0 + z * (1.0 - s)), s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def mlp(blocks, norm, G, species):
    """Atomic energies E_i, and dE_i/dG_i [N][96]."""
    mu, inv_sd, e0 = norm["mu"], norm["inv_sd"], norm["e0"]
    N = G.shape[0]
    E = np.zeros(N)
    dG = np.zeros((N, N_FEAT))
    for a in range(N_SPECIES):
        sel = np.nonzero(np.asarray(species) == a)[0]
        if len(sel) == 0:
            continue
        p = blocks[a]
        x = (G[sel] - mu[a]) * inv_sd[a]
        z1 = x @ p["W1"].T + p["b1"]
        h1, d1, _ = silu(z1)
        z2 = h1 @ p["W2"].T + p["b2"]
        h2, d2, _ = silu(z2)
        E[sel] = h2 @ p["w3"] + p["b3"][0] + e0[a]
        delta2 = p["w3"][None, :] * d2
        delta1 = (delta2 @ p["W2"]) * d1
        dG[sel] = (delta1 @ p["W1"]) * inv_sd[a]
    return E, dG


def _pair_jacobian(d, b, A1i, A2i, r_cut, r_min):
    """dG_i/dd for every pair: J [p][96][3] (only the neighbour-species block
    is non-zero).  A1i, A2i are the centre's A1, A2 for each pair."""
    n = len(b)
    r = np.sqrt(np.sum(d * d, axis=1))
    rh = d / r[:, None]
    _, dphi, psi, dpsi = _radial(r, r_cut, r_min)
    I3 = np.eye(3)
    # d rhat_a / d d_m = (delta_am - rhat_a rhat_m) / r
    drh = (I3[None] - rh[:, :, None] * rh[:, None, :]) / r[:, None, None]          # [p][a][m]
    # d (psi rhat_a) / d d_m
    dv = dpsi[:, :, None, None] * rh[:, None, :, None] * rh[:, None, None, :] \
        + psi[:, :, None, None] * drh[:, None, :, :]                               # [p][k][a][m]
    # d M_ab / d d_m with M = psi (rhat rhat^T - I/3)
    Mh = rh[:, :, None] * rh[:, None, :] - I3[None] / 3.0
    dRR = drh[:, :, None, :] * rh[:, None, :, None] + rh[:, :, None, None] * drh[:, None, :, :]
    dM = dpsi[:, :, None, None, None] * Mh[:, None, :, :, None] * rh[:, None, None, None, :] \
        + psi[:, :, None, None, None] * dRR[:, None]                               # [p][k][a][b][m]
    J = np.zeros((n, N_SPECIES, N_FEAT_SP, 3))
    blk = np.zeros((n, N_FEAT_SP, 3))
    blk[:, :N_RAD, :] = dphi[:, :, None] * rh[:, None, :]
    blk[:, N_RAD:N_RAD + N_ANG, :] = 2.0 * np.einsum("pka,pkam->pkm", A1i, dv)
    blk[:, N_RAD + N_ANG:, :] = 2.0 * np.einsum("pkab,pkabm->pkm", A2i, dM)
    J[np.arange(n), b] = blk
    return J.reshape(n, N_FEAT, 3)


def energy_forces(params, norm, pos, species, box, r_cut=6.0, r_min=0.5):
    """Total energy and forces F [3][N] = -dE/dr (FP64)."""
    blocks = unpack(params)
    G, A1, A2, (i, j, d, b) = descriptors(pos, species, box, r_cut, r_min)
    E_at, dG = mlp(blocks, norm, G, species)
    J = _pair_jacobian(d, b, A1[i, b], A2[i, b], r_cut, r_min)
    f = np.einsum("pf,pfm->pm", dG[i], J)        # dE_i / dd_ij
    N = len(species)
    F = np.zeros((N, 3))
    np.add.at(F, i, f)       # d_ij = r_j - r_i:  -dE/dr_i gets +f
    np.add.at(F, j, -f)      # and -dE/dr_j gets -f
    return E_at.sum(), F.T.copy(), E_at


def loss_and_grad(params, norm, frames, species, box, e_ref, f_ref, w_E, w_F,
                  r_cut=6.0, r_min=0.5):
    """Loss over a batch and its gradient with respect to the flat params.
    frames [B][3][N], e_ref [B], f_ref [B][3][N]."""
    blocks = unpack(params)
    species = np.asarray(species)
    B = len(frames)
    N = len(species)
    grad = [{k: np.zeros_like(v) for k, v in blk.items()} for blk in blocks]
    loss = 0.0
    for fidx in range(B):
        G, A1, A2, (i, j, d, b) = descriptors(frames[fidx], species, box, r_cut, r_min)
        E_at, dG = mlp(blocks, norm, G, species)
        J = _pair_jacobian(d, b, A1[i, b], A2[i, b], r_cut, r_min)
        f = np.einsum("pf,pfm->pm", dG[i], J)
        F = np.zeros((N, 3))
        np.add.at(F, i, f)
        np.add.at(F, j, -f)
        dE = E_at.sum() - e_ref[fidx]
        dF = F - np.asarray(f_ref[fidx]).T
        loss += w_E / B * (dE / N) ** 2 + w_F / (3 * N * B) * np.sum(dF * dF)
        e_bar = 2.0 * w_E / B * dE / (N * N)          # dL/dE_f
        u = 2.0 * w_F / (3 * N * B) * dF               # dL/dF [N][3]
        # dL/dtheta through F: F = -dE/dr, so it is -d/dtheta sum_i dG_i/dtheta-free
        # directional derivative: v_i = sum_j J_ij (u_j - u_i)
        v = np.zeros((N, N_FEAT))
        np.add.at(v, i, np.einsum("pfm,pm->pf", J, u[j] - u[i]))
        for a in range(N_SPECIES):
            sel = np.nonzero(species == a)[0]
            if len(sel) == 0:
                continue
            p, g = blocks[a], grad[a]
            x = (G[sel] - norm["mu"][a]) * norm["inv_sd"][a]
            xd = v[sel] * norm["inv_sd"][a]                # tangent of the input
            z1 = x @ p["W1"].T + p["b1"]
            h1, s1, t1 = silu(z1)
            z1d = xd @ p["W1"].T
            h1d = s1 * z1d
            z2 = h1 @ p["W2"].T + p["b2"]
            h2, s2, t2 = silu(z2)
            z2d = h1d @ p["W2"].T
            h2d = s2 * z2d
            # scalar per atom: e_bar * E_i - (dE_i/dx . xd); reverse mode through both
            om = -1.0
            g["w3"] += e_bar * h2.sum(axis=0) + om * h2d.sum(axis=0)
            g["b3"] += e_bar * len(sel)
            h2_bar = e_bar * np.broadcast_to(p["w3"], h2.shape)
            h2d_bar = om * np.broadcast_to(p["w3"], h2d.shape)
            z2_bar = h2_bar * s2 + h2d_bar * t2 * z2d
            z2d_bar = h2d_bar * s2
            g["W2"] += z2_bar.T @ h1 + z2d_bar.T @ h1d
            g["b2"] += z2_bar.sum(axis=0)
            h1_bar = z2_bar @ p["W2"]
            h1d_bar = z2d_bar @ p["W2"]
            z1_bar = h1_bar * s1 + h1d_bar * t1 * z1d
            z1d_bar = h1d_bar * s1
            g["W1"] += z1_bar.T @ x + z1d_bar.T @ xd
            g["b1"] += z1_bar.sum(axis=0)
    return loss, pack(grad)


def adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015); t counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
