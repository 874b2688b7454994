"""Pins of the FP64 surrogate oracle (oracle/ml_oracle.py).

The descriptors are pinned by facts that do not depend on the oracle's own
code: Gaussian-grid ratios fixed by eta = 1/(2 spacing^2), the Poisson sum of a
unit-spaced Gaussian comb, the addition theorem for the l = 1, 2 power
spectrum (trimer from dimers), rotation / translation / permutation
invariance, periodic tiling, and continuity at the cut-off.  The network and
all derivatives are pinned by central finite differences in FP64; Adam by its
closed form under a constant gradient.
"""
import math

import numpy as np
import pytest

from oracle import ml_oracle as M

RC, RMIN = 6.0, 0.5


def dimer(r, sp=(0, 1), L=40.0, direction=(1.0, 0.0, 0.0)):
    u = np.asarray(direction, dtype=float)
    u /= np.linalg.norm(u)
    p0 = np.array([10.0, 11.0, 12.0])
    pos = np.stack([p0, p0 + r * u]).T
    return pos, np.array(sp), np.array([L, L, L])


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    n = M.params_per_species() * M.N_SPECIES
    return rng.normal(0.0, scale / 3.0, n)


def random_norm(seed):
    rng = np.random.default_rng(seed)
    return {"mu": rng.normal(0.0, 0.2, (2, M.N_FEAT)),
            "inv_sd": rng.uniform(0.5, 2.0, (2, M.N_FEAT)),
            "e0": np.array([-1.5, 0.7])}


def cluster(n, seed, spread=3.0, L=60.0):
    rng = np.random.default_rng(seed)
    # random cluster with a minimum separation of 1.2 A
    pts = []
    while len(pts) < n:
        p = rng.uniform(-spread, spread, 3)
        if all(np.linalg.norm(p - q) > 1.2 for q in pts):
            pts.append(p)
    pos = np.array(pts).T + L / 2
    sp = rng.integers(0, 2, n)
    return pos, sp, np.array([L, L, L])


def test_radial_grid_ratios_and_comb_sum():
    mu, eta_r, nu, eta_a = M.grids(RC, RMIN)
    # a neighbour exactly on grid point 15: neighbours of the channel are
    # down by e^{-1/2}, two apart by e^{-2} (eta = 1 / (2 spacing^2))
    pos, sp, box = dimer(mu[15])
    G, _, _, _ = M.descriptors(pos, sp, box, RC, RMIN)
    g = G[0, 48:48 + 32]         # atom 0 sees species 1
    assert abs(g[14] / g[15] - math.exp(-0.5)) < 1e-13
    assert abs(g[16] / g[15] - math.exp(-0.5)) < 1e-13
    assert abs(g[13] / g[15] - math.exp(-2.0)) < 1e-13
    assert np.all(G[0, :48] == 0.0)     # no neighbour of species 0
    # comb sum: sum_c exp(-(r - mu_c)^2 / (2 d^2)) = sqrt(2 pi) (Poisson), and
    # the cosine cut-off is exactly 1/2 at r_c / 2
    pos, sp, box = dimer(RC / 2)
    G, _, _, _ = M.descriptors(pos, sp, box, RC, RMIN)
    assert abs(G[0, 48:80].sum() - 0.5 * math.sqrt(2 * math.pi)) < 1e-8
    # angular channel k on its grid point: l=1 ratios are squares (e^{-1})
    pos, sp, box = dimer(nu[3])
    G, _, _, _ = M.descriptors(pos, sp, box, RC, RMIN)
    l1 = G[0, 48 + 32:48 + 40]
    assert abs(l1[2] / l1[3] - math.exp(-1.0)) < 1e-13


def test_dimer_power_spectrum_ratio():
    # one neighbour: |psi rhat|^2 = psi^2, ||psi (rhat rhat^T - I/3)||^2 = 2/3 psi^2
    for r, direction in ((2.1, (1, 0, 0)), (3.7, (0.3, -0.5, 0.8))):
        pos, sp, box = dimer(r, direction=direction)
        G, _, _, _ = M.descriptors(pos, sp, box, RC, RMIN)
        for atom, blk in ((0, 1), (1, 0)):
            l1 = G[atom, 48 * blk + 32:48 * blk + 40]
            l2 = G[atom, 48 * blk + 40:48 * blk + 48]
            assert np.all(l1 > 0)
            assert np.allclose(l2, 2.0 / 3.0 * l1, rtol=1e-13, atol=0)


@pytest.mark.parametrize("alpha", [0.7, 1.9, 2.6])
def test_trimer_addition_theorem(alpha):
    """Centre with two same-species neighbours at r1, r2 and angle alpha:
    l1 = p1^2 + p2^2 + 2 p1 p2 cos(alpha),
    l2 = 2/3 (p1^2 + p2^2) + 2 p1 p2 (cos^2(alpha) - 1/3),
    with p1^2, p2^2 read from dimers (l1 of a dimer is psi^2)."""
    r1, r2 = 2.3, 3.1
    p1 = M.descriptors(*dimer(r1, (0, 1)), RC, RMIN)[0][0, 80:88]
    p2 = M.descriptors(*dimer(r2, (0, 1)), RC, RMIN)[0][0, 80:88]
    c = np.array([20.0, 20.0, 20.0])
    pos = np.stack([c, c + r1 * np.array([1.0, 0, 0]),
                    c + r2 * np.array([math.cos(alpha), math.sin(alpha), 0])]).T
    sp = np.array([0, 1, 1])
    G, _, _, _ = M.descriptors(pos, sp, np.array([40.0] * 3), RC, RMIN)
    a1, a2 = np.sqrt(p1), np.sqrt(p2)
    ca = math.cos(alpha)
    assert np.allclose(G[0, 80:88], p1 + p2 + 2 * a1 * a2 * ca, rtol=1e-12, atol=1e-15)
    assert np.allclose(G[0, 88:96], 2 / 3 * (p1 + p2) + 2 * a1 * a2 * (ca * ca - 1 / 3),
                       rtol=1e-12, atol=1e-15)


def test_invariances():
    pos, sp, box = cluster(9, 3)
    G, _, _, _ = M.descriptors(pos, sp, box, RC, RMIN)
    # rotation about the box centre
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    c = box[:, None] / 2
    Gr, _, _, _ = M.descriptors(Q @ (pos - c) + c, sp, box, RC, RMIN)
    assert np.max(np.abs(Gr - G)) < 1e-11 * np.max(np.abs(G))
    # translation
    Gt, _, _, _ = M.descriptors(pos + np.array([[1.3], [-2.2], [0.4]]), sp, box, RC, RMIN)
    assert np.max(np.abs(Gt - G)) < 1e-11 * np.max(np.abs(G))
    # permutation
    perm = rng.permutation(pos.shape[1])
    Gp, _, _, _ = M.descriptors(pos[:, perm], sp[perm], box, RC, RMIN)
    assert np.max(np.abs(Gp - G[perm])) < 1e-11 * np.max(np.abs(G))


def test_periodic_images_match_tiled_supercell():
    # 2x2x2 rock-salt cells (L = 8.42 A < 2 r_c): every image counts; the same
    # atoms tiled 2x2x2 into a 16.84 A box must see identical environments
    a, n = 4.21, 2
    cat = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    an = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0.5, 0.5, 0.5]])
    basis = np.vstack([cat, an])
    g = np.arange(n)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = ((cells[:, None, :] + basis[None]).reshape(-1, 3) * a)
    sp = np.tile([0] * 4 + [1] * 4, len(cells))
    x = x + np.random.default_rng(5).normal(0, 0.08, x.shape)
    L = n * a
    G, _, _, _ = M.descriptors(x.T, sp, np.array([L] * 3), RC, RMIN)
    t = np.arange(2)
    shifts = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3) * L
    X = (x[None] + shifts[:, None]).reshape(-1, 3)
    Gb, _, _, _ = M.descriptors(X.T, np.tile(sp, 8), np.array([2 * L] * 3), RC, RMIN)
    assert np.max(np.abs(Gb[:len(sp)] - G)) < 1e-10 * np.max(np.abs(G))


def test_cutoff_continuity():
    for sp in ((0, 1), (1, 1)):
        Gin = M.descriptors(*dimer(RC - 1e-7, sp), RC, RMIN)[0]
        Gout = M.descriptors(*dimer(RC + 1e-7, sp), RC, RMIN)[0]
        assert np.all(Gout == 0.0)
        assert np.max(np.abs(Gin)) < 1e-12


def test_mlp_input_gradient_fd():
    params, norm = random_params(1), random_norm(2)
    blocks = M.unpack(params)
    rng = np.random.default_rng(3)
    G = rng.normal(0.5, 1.0, (6, M.N_FEAT))
    sp = np.array([0, 1, 1, 0, 1, 0])
    E, dG = M.mlp(blocks, norm, G, sp)
    h = 1e-6
    for _ in range(12):
        i, f = int(rng.integers(6)), int(rng.integers(M.N_FEAT))
        Gp, Gm = G.copy(), G.copy()
        Gp[i, f] += h
        Gm[i, f] -= h
        fd = (M.mlp(blocks, norm, Gp, sp)[0][i] - M.mlp(blocks, norm, Gm, sp)[0][i]) / (2 * h)
        assert abs(fd - dG[i, f]) < 1e-7 * max(1.0, abs(dG[i, f]))


def _crystal(n_cells=2, seed=6, sigma=0.1):
    a = 4.21
    cat = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    an = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0.5, 0.5, 0.5]])
    basis = np.vstack([cat, an])
    g = np.arange(n_cells)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = ((cells[:, None, :] + basis[None]).reshape(-1, 3) * a)
    x = x + np.random.default_rng(seed).normal(0, sigma, x.shape)
    sp = np.tile([0] * 4 + [1] * 4, len(cells))
    return x.T.copy(), sp, np.array([n_cells * a] * 3)


def test_forces_are_minus_energy_gradient():
    params, norm = random_params(7), random_norm(8)
    for pos, sp, box in (_crystal(), cluster(7, 9)):
        E, F, _ = M.energy_forces(params, norm, pos, sp, box, RC, RMIN)
        assert np.max(np.abs(F.sum(axis=1))) < 1e-10 * np.max(np.abs(F))   # translation
        h = 1e-5
        rng = np.random.default_rng(10)
        for _ in range(8):
            i, d = int(rng.integers(pos.shape[1])), int(rng.integers(3))
            p1, p2 = pos.copy(), pos.copy()
            p1[d, i] += h
            p2[d, i] -= h
            fd = -(M.energy_forces(params, norm, p1, sp, box, RC, RMIN)[0] -
                   M.energy_forces(params, norm, p2, sp, box, RC, RMIN)[0]) / (2 * h)
            assert abs(fd - F[d, i]) < 1e-6 * max(1.0, np.max(np.abs(F)))


def test_isolated_cluster_is_torque_free():
    params, norm = random_params(11), random_norm(12)
    pos, sp, box = cluster(8, 13)
    _, F, _ = M.energy_forces(params, norm, pos, sp, box, RC, RMIN)
    torque = np.cross((pos - pos.mean(axis=1, keepdims=True)).T, F.T).sum(axis=0)
    assert np.max(np.abs(torque)) < 1e-10 * np.max(np.abs(F))


def test_loss_gradient_fd():
    params, norm = random_params(14), random_norm(15)
    frames, sp, box = [], None, None
    for s in range(2):
        pos, sp, box = _crystal(seed=20 + s, sigma=0.12)
        frames.append(pos)
    rng = np.random.default_rng(16)
    N = len(sp)
    e_ref = rng.normal(0.0, 3.0, 2)
    f_ref = rng.normal(0.0, 0.5, (2, 3, N))
    wE, wF = 0.7, 1.3
    L0, g = M.loss_and_grad(params, norm, frames, sp, box, e_ref, f_ref, wE, wF, RC, RMIN)
    # the loss itself from its definition through energy_forces
    Ls = 0.0
    for f in range(2):
        E, F, _ = M.energy_forces(params, norm, frames[f], sp, box, RC, RMIN)
        Ls += wE / 2 * ((E - e_ref[f]) / N) ** 2 + wF / (3 * N * 2) * np.sum((F - f_ref[f]) ** 2)
    assert abs(L0 - Ls) < 1e-12 * abs(Ls)
    n = M.params_per_species()
    # indices in every block of both species
    offs, o = [], 0
    for name, shape in M.layer_sizes():
        offs.append((o, int(np.prod(shape))))
        o += int(np.prod(shape))
    idx = []
    for a in range(2):
        for o, k in offs:
            idx += [a * n + o + int(rng.integers(k)) for _ in range(2)]
    h = 1e-6
    for k in idx:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        Lp = M.loss_and_grad(pp, norm, frames, sp, box, e_ref, f_ref, wE, wF, RC, RMIN)[0]
        Lm = M.loss_and_grad(pm, norm, frames, sp, box, e_ref, f_ref, wE, wF, RC, RMIN)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) < 2e-6 * max(abs(g[k]), 1e-3 * np.max(np.abs(g))), (k, fd, g[k])


def test_adam_closed_form_constant_gradient():
    rng = np.random.default_rng(17)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        p, m, v = M.adam(p, g, m, v, t, lr, eps=eps)
    # bias correction makes m_hat = g, v_hat = g^2 at every step
    assert np.allclose(p, p0 - 5 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
