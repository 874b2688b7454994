"""Seeded synthetic inputs shared by the GPU library, the oracle and the benchmark.

This module only builds inputs: unit systems, the rock-salt crystal geometry,
Gaussian site displacements drawn with numpy's PCG64, oscillator frequency
grids and the potential parameter sets of the benchmark workloads.  It holds
none of the method's arithmetic (no spectra, noise, forces or integration),
and it imports neither the oracle nor the GPU binding.

The paper's own systems (BaTiO3 effective Hamiltonian, DFT LiH, experimental
MgO) are not available; an MgO-like rock-salt crystal with a Buckingham plus
damped-shifted-force Coulomb potential stands in for the MgO heat-capacity
application of Sec. 2.2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# CODATA 2018: eV, Angstrom, amu, fs, K.
METAL_UNITS = dict(
    hbar=0.6582119569,              # eV fs
    kB=8.617333262e-5,              # eV / K
    coulomb_k=14.3996454784,        # eV Angstrom / e^2
    mass_unit=103.64269652680505,   # eV per amu Angstrom^2 fs^-2
)
# Reduced units of the oscillator workload: m = hbar = kB = 1.
REDUCED_UNITS = dict(hbar=1.0, kB=1.0, coulomb_k=0.0, mass_unit=1.0)

MG, O = 0, 1


@dataclass
class PairPotential:
    """Species table of the pair potential: index a*n_species + b."""
    mass: tuple
    charge: tuple
    buck_A: tuple
    buck_rho: tuple
    buck_C: tuple
    dsf_alpha: float
    r_cut: float
    skin: float

    @property
    def n_species(self):
        return len(self.mass)


def mgo_potential(r_cut=9.0, skin=1.0, dsf_alpha=0.2) -> PairPotential:
    """MgO-like rock salt: charges +/-2e, masses 24.305 / 15.999 amu,
    Buckingham Mg-O A=1280 eV rho=0.300 A; O-O A=9548 eV rho=0.2192 A
    C=32 eV A^6; Mg-Mg Coulomb only; DSF alpha=0.2/A, r_c = 9 A."""
    A = (0.0, 1280.0, 1280.0, 9548.0)
    rho = (1.0, 0.300, 0.300, 0.2192)
    C = (0.0, 0.0, 0.0, 32.0)
    return PairPotential(mass=(24.305, 15.999), charge=(2.0, -2.0), buck_A=A,
                         buck_rho=rho, buck_C=C, dsf_alpha=dsf_alpha, r_cut=r_cut,
                         skin=skin)


def rocksalt(n_cells: int, a: float = 4.21):
    """Conventional rock-salt supercell n x n x n: returns (pos [3][N], species [N], box).
    Atom order: cell-major, 4 cations then 4 anions per cell."""
    cat = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    an = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0.5, 0.5, 0.5]])
    basis = np.vstack([cat, an])
    sp_basis = np.array([MG] * 4 + [O] * 4, dtype=np.int32)
    g = np.arange(n_cells)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    species = np.tile(sp_basis, len(cells))
    box = np.array([n_cells * a] * 3)
    return np.ascontiguousarray(pos.T), species, box


def displaced(pos: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Add iid N(0, sigma^2) to every Cartesian component (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def beads_from(pos: np.ndarray, P: int) -> np.ndarray:
    """All P beads start at the same positions: [P][dims][N]."""
    return np.ascontiguousarray(np.broadcast_to(pos, (P,) + pos.shape)).copy()


def oscillator_omegas(n: int = 256, lo: float = 0.2, hi: float = 20.0) -> np.ndarray:
    """Deterministic log-uniform grid omega_i = lo (hi/lo)^(i/(n-1))."""
    i = np.arange(n)
    return lo * (hi / lo) ** (i / (n - 1))


@dataclass
class Workload:
    name: str
    kind: str                    # "oscillators" or "crystal"
    n_cells: int = 0
    P: int = 1
    T: float = 1.0
    gamma: float = 1.0
    dt: float = 1.0
    two_nf: int = 512
    noise: int = 1               # 0 white, 1 QTB, 2 QTB-PIMD
    seed: int = 0
    stream: int = 0
    displacement: float = 0.02   # fraction of the nearest-neighbour distance
    n_osc: int = 256
    extra: dict = field(default_factory=dict)


def workload(name: str) -> Workload:
    """Named synthetic workloads (sizes and settings of the benchmark suite)."""
    if name == "oscillators-256":
        w_max = 20.0
        return Workload(name, "oscillators", P=1, T=1.0, gamma=0.05 * w_max,
                        dt=0.02 / w_max, two_nf=512, noise=1, seed=0, n_osc=256)
    if name == "mgo-4x4x4-qtb-100K":
        return Workload(name, "crystal", n_cells=4, P=1, T=100.0, gamma=1e-3, dt=1.0,
                        two_nf=512, noise=1, seed=1)
    if name == "mgo-8x8x8-qtbpimd-P8-50K":
        return Workload(name, "crystal", n_cells=8, P=8, T=50.0, gamma=1e-3, dt=1.0,
                        two_nf=512, noise=2, seed=2)
    if name == "mgo-4x4x4-pimd-P32-50K":
        return Workload(name, "crystal", n_cells=4, P=32, T=50.0, gamma=1e-3, dt=1.0,
                        two_nf=2, noise=0, seed=2)
    raise KeyError(name)


def batched_sweep(n_rep: int = 64):
    """Replica table of the temperature / friction / bead sweep:
    T_j = 20 * 50^(j/15) K (j = r mod 16), gamma = [0.5,1,5,20][r div 16] /ps,
    n = 3 + ((5r+3) mod 8) cells, P = [1,4,8][(r + r div 16) mod 3]."""
    reps = []
    for r in range(n_rep):
        j = r % 16
        g = [0.5, 1.0, 5.0, 20.0][(r // 16) % 4]
        n = 3 + ((5 * r + 3) % 8)
        P = [1, 4, 8][(r + r // 16) % 3]
        T = 20.0 * 50.0 ** (j / 15.0)
        reps.append(Workload(f"rep{r}", "crystal", n_cells=n, P=P, T=T, gamma=g * 1e-3,
                             dt=1.0, two_nf=2048 if T < 50.0 else 512,
                             noise=2 if P > 1 else 1, seed=3, stream=r))
    return reps


def crystal_inputs(w: Workload, a: float = 4.21):
    """Positions [P][3][N] (all beads on the displaced sites), species, box."""
    pos, sp, box = rocksalt(w.n_cells, a)
    sigma = w.displacement * a / 2.0
    pos = displaced(pos, sigma, w.seed * 1000 + w.stream)
    return beads_from(pos, w.P), sp, box
