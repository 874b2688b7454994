"""Shared builders for the GPU parity tests: the same seeded inputs go to the
HIP library (through its C ABI) and to the oracle."""
from __future__ import annotations

import numpy as np

from paper_1905_02521_amd import qtb, workloads as W


def units_dict(reduced: bool):
    return dict(W.REDUCED_UNITS if reduced else W.METAL_UNITS)


def oracle_units(orc, reduced: bool):
    return orc.make_units(**units_dict(reduced))


def oracle_pair_pot(orc, p=None):
    p = p or W.mgo_potential()
    return orc.make_pot(0, p.mass, p.charge, p.buck_A, p.buck_rho, p.buck_C, p.dsf_alpha,
                        p.r_cut, p.skin)


def crystal(n_cells, P, seed, sigma=0.0421, bead_spread=0.0):
    pos, sp, box = W.rocksalt(n_cells)
    base = W.displaced(pos, sigma, seed)
    beads = np.stack([base if bead_spread == 0 else W.displaced(base, bead_spread, seed + 100 + b)
                      for b in range(P)])
    return beads, sp, box


def gpu_crystal_ctx(beads, sp, box, *, T, gamma, dt, noise, prec, fir, seed=1, stream=0,
                    K=64, max_two_nf=512, obs_every=0, vel=None, pot=None, graphs=True,
                    fuse=False, autotune=True, list_kernel=False):
    p = pot or W.mgo_potential()
    rep = qtb.Replica(pos=beads, species=sp, T=T, gamma=gamma, dt=dt, noise=noise, vel=vel,
                      box=tuple(box), seed=seed, stream=stream)
    return qtb.Context(qtb.pair_potential_dict(p), [rep], units_dict(False), prec=prec, fir=fir,
                       fir_block_K=K, obs_every=obs_every, max_two_nf=max_two_nf, graphs=graphs,
                       fuse=fuse, autotune=autotune, list_kernel=list_kernel)


def gpu_ho_ctx(omegas, P, *, T, gamma, dt, noise, prec, fir, seed=0, stream=0, K=64,
               max_two_nf=512, obs_every=0, pos=None, vel=None):
    N = len(omegas)
    pos = np.zeros((P, 1, N)) if pos is None else pos
    rep = qtb.Replica(pos=pos, species=np.zeros(N, np.int32), T=T, gamma=gamma, dt=dt,
                      noise=noise, vel=vel, seed=seed, stream=stream, harm_omega=omegas)
    return qtb.Context(dict(kind=qtb.POT_HARMONIC, mass=(1.0,)), [rep], units_dict(True),
                       prec=prec, fir=fir, fir_block_K=K, obs_every=obs_every,
                       max_two_nf=max_two_nf)


def oracle_zeta_block(orc, taps, seed, stream, n0, K, n_dof):
    """zeta_{n,d} for n in [n0, n0+K), d in [0, n_dof), by numpy convolution of
    the oracle's white noise (oracle arithmetic only)."""
    two_nf = len(taps)
    Nf = two_nf // 2
    w = orc.gauss_fill(seed, n0 - Nf + 1, K + two_nf - 1, 0, n_dof, stream, 0)
    # zeta_n = sum_k h_k w_{n-k}; window row j holds step n0 - Nf + 1 + j
    out = np.zeros((K, n_dof))
    for k in range(-Nf, Nf):
        out += taps[k + Nf] * w[(Nf - 1 - k):(Nf - 1 - k) + K]
    abs_sum = np.zeros((K, n_dof))
    for k in range(-Nf, Nf):
        abs_sum += abs(taps[k + Nf]) * np.abs(w[(Nf - 1 - k):(Nf - 1 - k) + K])
    return out, abs_sum
