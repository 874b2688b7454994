"""ctypes front end of the plain FP64 CPU oracle (``qtb_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU library.  The product path
never imports it, and this module imports nothing from the product package.

Paper: Dammak, Hayoun, Brieuc, Geneste, arXiv:1905.02521 (eq. numbers are
cited on each function in ``qtb_oracle.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qtb_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "qtb_oracle_abi.c")]
_HDRS = [os.path.join(_HERE, "qtb_oracle.h"), os.path.join(_HERE, "qtb_oracle_abi.h")]
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: the Gaussian transform is specified operation by operation.
CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-mavx2", "-mfma", "-std=c11"]


# AddressSanitizer and UndefinedBehaviorSanitizer build of the same source,
# loaded instead of liboracle.so when QTB_ORACLE_LIB names it (a Python
# process that preloads gcc's libasan; see tests/test_sanitizers.py).
SAN_FLAGS = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (always, when force=True)."""
    newest = max(os.path.getmtime(f) for f in _SRCS + _HDRS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out_dir: str) -> str:
    """Compile the oracle with the sanitizers into out_dir; returns the path."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle_san.so")
    subprocess.check_call(["gcc", *CFLAGS, *SAN_FLAGS, "-o", out, *_SRCS, "-lm"])
    return out


class Units(ctypes.Structure):
    _fields_ = [("hbar", ctypes.c_double), ("kB", ctypes.c_double),
                ("coulomb_k", ctypes.c_double), ("mass_unit", ctypes.c_double)]


MAX_SPECIES = 4


class Pot(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_species", ctypes.c_int),
                ("mass", ctypes.c_double * MAX_SPECIES),
                ("charge", ctypes.c_double * MAX_SPECIES),
                ("buck_A", ctypes.c_double * (MAX_SPECIES * MAX_SPECIES)),
                ("buck_rho", ctypes.c_double * (MAX_SPECIES * MAX_SPECIES)),
                ("buck_C", ctypes.c_double * (MAX_SPECIES * MAX_SPECIES)),
                ("dsf_alpha", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("skin", ctypes.c_double),
                ("os_V0", ctypes.c_double * MAX_SPECIES),
                ("os_d", ctypes.c_double * MAX_SPECIES)]


POT_PAIR, POT_HARMONIC, POT_MORSE, POT_DOUBLE_WELL = 0, 1, 2, 3


_lib = None
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PU = ctypes.POINTER(Units)
_PP = ctypes.POINTER(Pot)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("QTB_ORACLE_LIB") or build()
        _lib = ctypes.CDLL(path)
        L = _lib
        L.orc_theta.restype = _D
        L.orc_theta.argtypes = [_D, _D, _PU]
        L.orc_kappa.restype = _D
        L.orc_kappa.argtypes = [_D, _D, ctypes.c_int, _PU, _D]
        L.orc_taps.restype = ctypes.c_int
        L.orc_taps.argtypes = [ctypes.c_int, _D, ctypes.c_int, _D, ctypes.c_int, _PU, _PD]
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_gauss.restype = _D
        L.orc_gauss.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32]
        L.orc_gauss_fill.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, _PD]
        L.orc_log_spec.restype = _D
        L.orc_log_spec.argtypes = [_D]
        L.orc_cos2pi_spec.restype = _D
        L.orc_cos2pi_spec.argtypes = [ctypes.c_uint64]
        L.orc_zeta.restype = _D
        L.orc_zeta.argtypes = [_PD, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.c_int64, ctypes.c_uint32]
        L.orc_pair_bruteforce.restype = _D
        L.orc_pair_bruteforce.argtypes = [_PP, _PU, ctypes.c_int, _PD,
                                          ctypes.POINTER(ctypes.c_int32), _PD, _PD, _PD]
        L.orc_sim_new.restype = ctypes.c_void_p
        L.orc_sim_new.argtypes = [_PP, _PU, ctypes.c_int, ctypes.c_int, ctypes.c_int, _PD,
                                  ctypes.POINTER(ctypes.c_int32), _PD, _D, _D, _D,
                                  ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                  _PD, _PD, ctypes.c_int64, ctypes.c_int]
        L.orc_sim_run.restype = ctypes.c_int
        L.orc_sim_run.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, _PD]
        L.orc_sim_get.argtypes = [ctypes.c_void_p, _PD, _PD, _PD,
                                  ctypes.POINTER(ctypes.c_int64)]
        L.orc_sim_free.argtypes = [ctypes.c_void_p]
        L.orc_sim_observe.argtypes = [ctypes.c_void_p, _PD]
        L.orc_sim_hamiltonian.restype = _D
        L.orc_sim_hamiltonian.argtypes = [ctypes.c_void_p]
        L.orc_sim_taps.restype = _PD
        L.orc_sim_taps.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
        L.orc_nm_matrix.argtypes = [ctypes.c_int, _PD]
        L.orc_sim_set_barostat.restype = ctypes.c_int
        L.orc_sim_set_barostat.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_sim_set_piston.restype = ctypes.c_int
        L.orc_sim_set_piston.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.orc_sim_piston_momentum.restype = _D
        L.orc_sim_piston_momentum.argtypes = [ctypes.c_void_p]
        L.orc_sim_barostat_state.restype = None
        L.orc_sim_barostat_state.argtypes = [ctypes.c_void_p, _PD, _PD]
        L.orc_sim_box.argtypes = [ctypes.c_void_p, _PD]
    return _lib


def _pd(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def make_units(hbar, kB, coulomb_k=0.0, mass_unit=1.0) -> Units:
    return Units(hbar, kB, coulomb_k, mass_unit)


def make_pot(kind=0, mass=(1.0,), charge=(0.0,), buck_A=None, buck_rho=None, buck_C=None,
             dsf_alpha=0.0, r_cut=1.0, skin=0.0, V0=None, d=None) -> Pot:
    ns = len(mass)
    p = Pot()
    p.kind = kind
    p.n_species = ns
    for a in range(ns):
        p.mass[a] = mass[a]
        p.charge[a] = charge[a] if a < len(charge) else 0.0
    for ab in range(ns * ns):
        p.buck_A[ab] = buck_A[ab] if buck_A is not None else 0.0
        p.buck_rho[ab] = buck_rho[ab] if buck_rho is not None else 1.0
        p.buck_C[ab] = buck_C[ab] if buck_C is not None else 0.0
    p.dsf_alpha, p.r_cut, p.skin = dsf_alpha, r_cut, skin
    for a in range(ns):
        p.os_V0[a] = V0[a] if V0 is not None else 0.0
        p.os_d[a] = d[a] if d is not None else 1.0
    return p


# ---------------------------------------------------------------- spectra
def vdos(v, seg, weight=None):
    """Velocity density of states from the velocity time series, the
    time-correlation route that Sec. 3 names as QTB's advantage: by the
    Wiener-Khinchin theorem the power spectrum of v is the Fourier transform
    of its autocorrelation.  v[t, j] holds dof j at sample t; the series is
    cut into whole segments of seg samples (a trailing part is dropped), and
    each segment's periodogram |V_k|^2 / seg, V_k = sum_t v_t e^{-2 pi i k t /
    seg}, is weighted by weight[j] (masses: 1 if None), summed over dofs and
    averaged over segments.  Returns (phi_k, S_k) for k = 0 .. seg/2, phi_k =
    2 pi k / seg in radians per sample, and the number of segments; the mean
    of S over all seg frequencies (both halves) is sum_j weight_j <v_j^2>, so
    with masses as weights it is twice the mean kinetic energy."""
    v = np.asarray(v, dtype=np.float64)
    if v.ndim == 1:
        v = v[:, None]
    n_seg = v.shape[0] // seg
    w = np.ones(v.shape[1]) if weight is None else np.asarray(weight, dtype=np.float64)
    S = np.zeros(seg // 2 + 1)
    for q in range(n_seg):
        V = np.fft.rfft(v[q * seg:(q + 1) * seg], axis=0)
        S += (np.abs(V) ** 2 / seg) @ w
    if n_seg:
        S /= n_seg
    return 2.0 * np.pi * np.arange(seg // 2 + 1) / seg, S, n_seg


# ---------------------------------------------------------------- functions
def theta(omega, T, units: Units):
    return lib().orc_theta(float(omega), float(T), ctypes.byref(units))


def kappa(omega, T, P, units: Units, h_quad=0.0):
    return lib().orc_kappa(float(omega), float(T), int(P), ctypes.byref(units), float(h_quad))


def taps(kind, T, P, dt, two_nf, units: Units) -> np.ndarray:
    h = np.zeros(two_nf)
    rc = lib().orc_taps(int(kind), float(T), int(P), float(dt), int(two_nf),
                        ctypes.byref(units), _pd(h))
    if rc:
        raise ValueError("bad filter length")
    return h


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def gauss(seed, n, d, stream=0, tag=0):
    return lib().orc_gauss(seed, n, d, stream, tag)


def gauss_fill(seed, n0, n_rows, d0, n_dof, stream=0, tag=0) -> np.ndarray:
    out = np.empty((n_rows, n_dof))
    lib().orc_gauss_fill(seed, n0, n_rows, d0, n_dof, stream, tag, _pd(out))
    return out


def log_spec(u):
    return lib().orc_log_spec(float(u))


def cos2pi_spec(odd53):
    return lib().orc_cos2pi_spec(int(odd53))


def zeta(h: np.ndarray, seed, stream, n, d):
    h = np.ascontiguousarray(h, dtype=np.float64)
    return lib().orc_zeta(_pd(h), len(h), seed, stream, n, d)


def noise_spectrum(kind, T, P, dt, n, units: Units) -> np.ndarray:
    """Target spectrum of the random force on the grid omega_j = 2 pi j / (n dt),
    j = 0 .. n/2: k_B T (white), theta (eq. 1, QTB) or kappa_P (eq. 10-12)."""
    kT = units.kB * T
    out = np.empty(n // 2 + 1)
    for j in range(n // 2 + 1):
        w = 2.0 * np.pi * j / (n * dt)
        out[j] = kT if kind == 0 else (theta(w, T, units) if kind == 1 or P == 1
                                       else kappa(w, T, P, units))
    return out


def eq9_block(S, seed, stream, row0, n_dof):
    """One block of n steps of coloured noise by the paper's generator (eq. 9):
    random Fourier amplitudes (a_j + i b_j) sqrt(S_j n / 2) on the grid
    omega_j = 2 pi j / (n dt), then the inverse discrete Fourier transform.
    The paper leaves the construction of a real force implicit; here the
    amplitudes of the negative frequencies are the complex conjugates of the
    positive ones (Hermitian), and the two self-conjugate terms j = 0 and
    j = n/2 are real with amplitude a_j sqrt(S_j n), so that every mode
    carries E|R_j|^2 = n S_j and the noise has the discrete spectrum S.
    a_j, b_j are the library's counter-based unit Gaussians at step row0 + j
    (tags 1 and 2).  S: [n/2 + 1]; returns zeta [n][n_dof]."""
    S = np.asarray(S, dtype=np.float64)
    n = 2 * (len(S) - 1)
    h = n // 2
    a = gauss_fill(seed, row0, h + 1, 0, n_dof, stream, 1)
    b = gauss_fill(seed, row0, h + 1, 0, n_dof, stream, 2)
    X = np.zeros((n, n_dof), dtype=np.complex128)
    amp = np.sqrt(S * n / 2.0)
    for j in range(1, h):
        X[j] = amp[j] * (a[j] + 1j * b[j])
        X[n - j] = np.conj(X[j])
    X[0] = np.sqrt(S[0] * n) * a[0]
    X[h] = np.sqrt(S[h] * n) * a[h]
    return np.fft.ifft(X, axis=0).real


def nm_matrix(P) -> np.ndarray:
    C = np.zeros((P, P))
    lib().orc_nm_matrix(P, _pd(C))
    return C


def pair_bruteforce(pot: Pot, units: Units, box, species, pos):
    """pos: [3][N] -> (energy, forces [3][N], virial 3x3)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    N = pos.shape[1]
    sp = np.ascontiguousarray(species, dtype=np.int32)
    f = np.zeros_like(pos)
    vir = np.zeros(9)
    boxa = np.ascontiguousarray(box, dtype=np.float64)
    e = lib().orc_pair_bruteforce(ctypes.byref(pot), ctypes.byref(units), N, _pd(boxa),
                                  sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  _pd(pos), _pd(f), _pd(vir))
    return e, f, vir.reshape(3, 3)


OBS_NAMES = ("kinetic", "potential", "spring", "e_primitive", "e_virial",
             "t_kinetic", "x2_mean", "step", "pressure", "virial_pair")


class Sim:
    """One replica integrated by the oracle; state arrays are [P][dims][N]."""

    def __init__(self, pot: Pot, units: Units, N, P, dims, box, species, T, gamma, dt,
                 seed, stream, noise_kind, two_nf, pos0, vel0=None, harm_omega=None,
                 step0=0, n_threads=1):
        self.N, self.P, self.dims = N, P, dims
        self._keep = []
        sp = np.ascontiguousarray(species, dtype=np.int32)
        boxa = np.ascontiguousarray(box if box is not None else [0, 0, 0], dtype=np.float64)
        pos0 = np.ascontiguousarray(pos0, dtype=np.float64).reshape(P, dims, N)
        v0 = None if vel0 is None else np.ascontiguousarray(vel0, dtype=np.float64).reshape(P, dims, N)
        hom = None if harm_omega is None else np.ascontiguousarray(harm_omega, dtype=np.float64)
        self._keep += [sp, boxa, pos0, v0, hom]
        self.h = lib().orc_sim_new(ctypes.byref(pot), ctypes.byref(units), N, P, dims, _pd(boxa),
                                   sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   None if hom is None else _pd(hom),
                                   T, gamma, dt, seed, stream, noise_kind, two_nf,
                                   _pd(pos0), None if v0 is None else _pd(v0), step0, n_threads)
        if not self.h:
            raise ValueError("oracle rejected the replica description")

    def run(self, n_steps, obs_every=0):
        # samples fall on steps divisible by obs_every: a run that starts off
        # that grid can hold one more than n_steps // obs_every
        nmax = (n_steps // obs_every + 1) if obs_every > 0 else 0
        obs = np.zeros((max(nmax, 1), len(OBS_NAMES)))
        n = lib().orc_sim_run(self.h, n_steps, obs_every, _pd(obs))
        return obs[:n]

    def state(self):
        shape = (self.P, self.dims, self.N)
        r, v, f = np.zeros(shape), np.zeros(shape), np.zeros(shape)
        st = ctypes.c_int64()
        lib().orc_sim_get(self.h, _pd(r), _pd(v), _pd(f), ctypes.byref(st))
        return r, v, f, st.value

    def observe(self):
        o = np.zeros(len(OBS_NAMES))
        lib().orc_sim_observe(self.h, _pd(o))
        return o

    def set_barostat(self, P0, tau_p, beta_T):
        if lib().orc_sim_set_barostat(self.h, float(P0), float(tau_p), float(beta_T)):
            raise ValueError("oracle refused the barostat (the pair kind only)")

    def set_piston(self, P0, tau_p, gamma_p):
        if lib().orc_sim_set_piston(self.h, float(P0), float(tau_p), float(gamma_p)):
            raise ValueError("oracle refused the piston (the pair kind only, T > 0)")

    def piston_momentum(self):
        return lib().orc_sim_piston_momentum(self.h)

    def box(self):
        b = np.zeros(3)
        lib().orc_sim_box(self.h, _pd(b))
        return b

    def barostat_state(self):
        """(p_e, s, s_v1, s_v2): piston momentum and the pending scalings."""
        b = np.zeros(4)
        lib().orc_sim_barostat_state(self.h, _pd(b), None)
        return b

    def set_barostat_state(self, state):
        b = np.ascontiguousarray(state, dtype=np.float64)
        lib().orc_sim_barostat_state(self.h, None, _pd(b))

    def hamiltonian(self):
        return lib().orc_sim_hamiltonian(self.h)

    def taps(self):
        n = ctypes.c_int()
        p = lib().orc_sim_taps(self.h, ctypes.byref(n))
        return np.ctypeslib.as_array(p, shape=(n.value,)).copy()

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_sim_free(self.h)
            self.h = None


# ------------------------------------------------------------------------
# The oracle behind the library's call shape (qtb_oracle_abi.h): one
# harness can drive either back end.  Descriptions are duck-typed: any
# object with the replica attributes (pos, vel, species, T, gamma, dt, noise,
# box, seed, stream, harm_omega) and a potential dict with the library
# binding's keys (kind, mass, charge, buck_A, buck_rho, buck_C, dsf_alpha,
# r_cut, skin).
class AbiPotential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_species", ctypes.c_int32),
                ("mass", _PD), ("charge", _PD), ("buck_A", _PD), ("buck_rho", _PD),
                ("buck_C", _PD), ("dsf_alpha", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("skin", ctypes.c_double), ("onsite_V0", _PD), ("onsite_d", _PD)]


class AbiReplica(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_beads", ctypes.c_int32),
                ("n_dims", ctypes.c_int32), ("noise", ctypes.c_int32),
                ("box", ctypes.c_double * 3), ("T", ctypes.c_double),
                ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("species", ctypes.POINTER(ctypes.c_int32)),
                ("harm_omega", _PD), ("pos", _PD), ("vel", _PD)]


class AbiOptions(ctypes.Structure):
    _fields_ = [("hbar", ctypes.c_double), ("kB", ctypes.c_double),
                ("coulomb_k", ctypes.c_double), ("mass_unit", ctypes.c_double),
                ("prec", ctypes.c_int32), ("fir", ctypes.c_int32),
                ("fir_block_K", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("max_two_nf", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("ml_r_cut", ctypes.c_double)]


class AbiObs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("kinetic", ctypes.c_double),
                ("potential", ctypes.c_double), ("spring", ctypes.c_double),
                ("e_primitive", ctypes.c_double), ("e_virial", ctypes.c_double),
                ("t_kinetic", ctypes.c_double), ("x2_mean", ctypes.c_double),
                ("virial_pair", ctypes.c_double), ("pressure", ctypes.c_double),
                ("volume", ctypes.c_double), ("n_samples", ctypes.c_int32)]


class AbiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


def _abi_lib():
    L = lib()
    if not getattr(L, "_abi_ready", False):
        vp = ctypes.c_void_p
        L.orc_qtb_workspace_bytes.restype = ctypes.c_size_t
        L.orc_qtb_workspace_bytes.argtypes = [vp, vp, ctypes.c_int32, vp]
        L.orc_qtb_init.restype = ctypes.c_int
        L.orc_qtb_init.argtypes = [ctypes.POINTER(vp), vp, vp, ctypes.c_int32, vp, vp,
                                   ctypes.c_size_t, vp]
        L.orc_qtb_build_filter.restype = ctypes.c_int
        L.orc_qtb_build_filter.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           _PD]
        L.orc_qtb_step.restype = ctypes.c_int
        L.orc_qtb_step.argtypes = [vp, ctypes.c_int64]
        L.orc_qtb_observables.restype = ctypes.c_int
        L.orc_qtb_observables.argtypes = [vp, ctypes.c_int32, vp]
        L.orc_qtb_get_state.restype = ctypes.c_int
        L.orc_qtb_get_state.argtypes = [vp, ctypes.c_int32, _PD, _PD,
                                        ctypes.POINTER(ctypes.c_int64)]
        L.orc_qtb_set_state.restype = ctypes.c_int
        L.orc_qtb_set_state.argtypes = [vp, ctypes.c_int32, _PD, _PD, ctypes.c_int64]
        L.orc_qtb_last_error.restype = ctypes.c_char_p
        L.orc_qtb_last_error.argtypes = [vp]
        L.orc_qtb_destroy.restype = None
        L.orc_qtb_destroy.argtypes = [vp]
        L._abi_ready = True
    return L


class AbiContext:
    """The oracle driven through its ABI-shaped calls, with the methods of
    the library binding's Context that the parity harness uses
    (build_filter, step, observables, get_state, set_state, close)."""

    def __init__(self, potd, reps, units, obs_every=0, max_two_nf=512):
        L = _abi_lib()
        self._keep = []

        def arr(x, dt=np.float64):
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return a
        mass = arr(potd["mass"])
        ns = len(mass)
        pot = AbiPotential()
        pot.kind, pot.n_species = int(potd.get("kind", 0)), ns
        pot.mass = _pd(mass)
        for key in ("charge", "buck_A", "buck_rho", "buck_C"):
            if potd.get(key) is not None:
                setattr(pot, key, _pd(arr(potd[key])))
        pot.dsf_alpha = float(potd.get("dsf_alpha", 0.0))
        pot.r_cut = float(potd.get("r_cut", 1.0))
        pot.skin = float(potd.get("skin", 0.0))
        n = len(reps)
        self.reps = (AbiReplica * n)()
        self.shapes, self.state = [], []
        for k, rp in enumerate(reps):
            pos = arr(np.array(rp.pos, dtype=np.float64))
            vel = arr(np.zeros_like(pos) if rp.vel is None else np.array(rp.vel, np.float64))
            P, dims, N = pos.shape
            R = self.reps[k]
            R.n_atoms, R.n_beads, R.n_dims, R.noise = N, P, dims, int(rp.noise)
            if rp.box is not None:
                for a in range(3):
                    R.box[a] = float(rp.box[a])
            R.T, R.gamma, R.dt = float(rp.T), float(rp.gamma), float(rp.dt)
            R.seed, R.stream = int(rp.seed), int(rp.stream)
            sp = arr(rp.species, np.int32)
            R.species = sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            if getattr(rp, "harm_omega", None) is not None:
                R.harm_omega = _pd(arr(rp.harm_omega))
            R.pos, R.vel = _pd(pos), _pd(vel)
            self.shapes.append((P, dims, N))
            self.state.append((pos, vel))
        opt = AbiOptions()
        opt.hbar, opt.kB = units["hbar"], units["kB"]
        opt.coulomb_k, opt.mass_unit = units.get("coulomb_k", 0.0), units["mass_unit"]
        opt.prec, opt.fir, opt.fir_block_K = 1, 3, 64
        opt.obs_every, opt.max_two_nf = int(obs_every), int(max_two_nf)
        self.ctx = ctypes.c_void_p()
        st = L.orc_qtb_init(ctypes.byref(self.ctx), ctypes.byref(pot), self.reps, n,
                            ctypes.byref(opt), None, 0, None)
        if st:
            raise AbiError(st, "orc_qtb_init rejected the description")

    def _check(self, st):
        if st:
            raise AbiError(st, _abi_lib().orc_qtb_last_error(self.ctx).decode())

    def build_filter(self, replica, kind, two_nf):
        taps = np.zeros(max(int(two_nf), 2))
        self._check(_abi_lib().orc_qtb_build_filter(self.ctx, replica, kind, two_nf, _pd(taps)))
        return taps

    def step(self, n):
        self._check(_abi_lib().orc_qtb_step(self.ctx, int(n)))

    def observables(self, replica=0):
        o = AbiObs()
        self._check(_abi_lib().orc_qtb_observables(self.ctx, replica, ctypes.byref(o)))
        return {f: getattr(o, f) for f, _ in AbiObs._fields_}

    def get_state(self, replica=0):
        r, v = np.zeros(self.shapes[replica]), np.zeros(self.shapes[replica])
        st = ctypes.c_int64()
        self._check(_abi_lib().orc_qtb_get_state(self.ctx, replica, _pd(r), _pd(v),
                                                 ctypes.byref(st)))
        return r, v, st.value

    def set_state(self, replica, pos, vel, step):
        p = None if pos is None else np.ascontiguousarray(pos, dtype=np.float64)
        v = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
        self._check(_abi_lib().orc_qtb_set_state(self.ctx, replica,
                                                 None if p is None else _pd(p),
                                                 None if v is None else _pd(v), int(step)))

    def close(self):
        if self.ctx:
            _abi_lib().orc_qtb_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
