"""ctypes binding of libqtb.so (include/qtb.h), same names as the C ABI.

Argument marshalling only: every step of the integrator runs in the HIP
kernels of libqtb.so.  PyTorch provides device memory (state arrays and the
workspace) and the stream.  Importing this module loads nothing; the first
call loads the library and raises if it is missing (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtb.so")

QTB_OK, QTB_E_INVALID, QTB_E_NOMEM, QTB_E_DEVICE, QTB_E_STATE, QTB_E_NONFINITE, \
    QTB_E_UNSUPPORTED = range(7)
NOISE_CLASSICAL, NOISE_QTB, NOISE_QTB_PIMD = 0, 1, 2
PREC_FP32, PREC_FP64 = 0, 1
FIR_FP32, FIR_BF16X3, FIR_BF16, FIR_FP64 = 0, 1, 2, 3
POT_PAIR, POT_HARMONIC, POT_MORSE, POT_DOUBLE_WELL = 0, 1, 2, 3
OPT_NO_GRAPH = 1
OPT_NO_AUTOTUNE = 2
OPT_ML_TRAIN = 4
OPT_FUSE = 8
OPT_NOISE_BLOCKS = 16
OPT_LIST_KERNEL = 32
MAX_SPECIES = 4
ML_FEATURES = 96
ML_PARAMS_PER_SPECIES = 10433
ML_PARAMS = 2 * ML_PARAMS_PER_SPECIES
ML_NORM = 2 * 2 * ML_FEATURES + 2

_STATUS = {1: "QTB_E_INVALID", 2: "QTB_E_NOMEM", 3: "QTB_E_DEVICE", 4: "QTB_E_STATE",
           5: "QTB_E_NONFINITE", 6: "QTB_E_UNSUPPORTED"}


class QtbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_PD = ctypes.POINTER(ctypes.c_double)
_PI32 = ctypes.POINTER(ctypes.c_int32)


class qtb_potential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_species", ctypes.c_int32),
                ("mass", _PD), ("charge", _PD), ("buck_A", _PD), ("buck_rho", _PD),
                ("buck_C", _PD), ("dsf_alpha", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("skin", ctypes.c_double), ("onsite_V0", _PD), ("onsite_d", _PD)]


class qtb_replica(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_beads", ctypes.c_int32),
                ("n_dims", ctypes.c_int32), ("noise", ctypes.c_int32),
                ("box", ctypes.c_double * 3), ("T", ctypes.c_double),
                ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("species", _PI32), ("harm_omega", _PD),
                ("d_pos", ctypes.c_void_p), ("d_vel", ctypes.c_void_p)]


class qtb_options(ctypes.Structure):
    _fields_ = [("hbar", ctypes.c_double), ("kB", ctypes.c_double),
                ("coulomb_k", ctypes.c_double), ("mass_unit", ctypes.c_double),
                ("prec", ctypes.c_int32), ("fir", ctypes.c_int32),
                ("fir_block_K", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("max_two_nf", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("ml_r_cut", ctypes.c_double)]


class qtb_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("kinetic", ctypes.c_double),
                ("potential", ctypes.c_double), ("spring", ctypes.c_double),
                ("e_primitive", ctypes.c_double), ("e_virial", ctypes.c_double),
                ("t_kinetic", ctypes.c_double), ("x2_mean", ctypes.c_double),
                ("virial_pair", ctypes.c_double), ("pressure", ctypes.c_double),
                ("volume", ctypes.c_double), ("n_samples", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


EXPORTS = ("qtb_workspace_bytes", "qtb_init", "qtb_build_filter", "qtb_step",
           "qtb_observables", "qtb_get_state", "qtb_set_state", "qtb_evaluate",
           "qtb_get_noise", "qtb_gaussian", "qtb_profile", "qtb_profile_read",
           "qtb_vdos_workspace_bytes", "qtb_vdos_spectrum", "qtb_vdos_spectrum_noalloc",
           "qtb_vdos_attach", "qtb_vdos_read",
           "qtb_vdos_detach", "qtb_barostat", "qtb_barostat_piston", "qtb_get_box",
           "qtb_get_barostat_state", "qtb_set_barostat_state", "qtb_filter_taps",
           "qtb_set_decomposition", "qtb_get_decomposition",
           "qtb_set_group_decomposition", "qtb_get_group_decomposition",
           "qtb_set_replica_skin",
           "qtb_last_error", "qtb_destroy", "qtb_version",
           "qtb_ml_workspace_bytes", "qtb_ml_create", "qtb_ml_init_params", "qtb_ml_set_params",
           "qtb_ml_get_params", "qtb_ml_attach", "qtb_ml_evaluate", "qtb_ml_fit_norm",
           "qtb_ml_train_step", "qtb_ml_check", "qtb_ml_last_error", "qtb_ml_destroy")
N_PHASES = 6
PHASES = ("noise", "fir", "update", "nlist", "forces", "obs")

_lib = None


def lib():
    """Load libqtb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("QTB_LIB", LIB_PATH)  # e.g. a host-sanitizer build of the same sources
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with "
                      "`python -m paper_1905_02521_amd.build`")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.qtb_workspace_bytes.restype = ctypes.c_size_t
    L.qtb_workspace_bytes.argtypes = [ctypes.POINTER(qtb_potential), ctypes.POINTER(qtb_replica),
                                      ctypes.c_int32, ctypes.POINTER(qtb_options)]
    L.qtb_init.restype = ctypes.c_int
    L.qtb_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(qtb_potential),
                           ctypes.POINTER(qtb_replica), ctypes.c_int32,
                           ctypes.POINTER(qtb_options), vp, ctypes.c_size_t, vp]
    L.qtb_build_filter.restype = ctypes.c_int
    L.qtb_build_filter.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _PD]
    L.qtb_step.restype = ctypes.c_int
    L.qtb_step.argtypes = [vp, ctypes.c_int64]
    L.qtb_observables.restype = ctypes.c_int
    L.qtb_observables.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(qtb_obs)]
    L.qtb_get_state.restype = ctypes.c_int
    L.qtb_get_state.argtypes = [vp, ctypes.c_int32, _PD, _PD, ctypes.POINTER(ctypes.c_int64)]
    L.qtb_set_state.restype = ctypes.c_int
    L.qtb_set_state.argtypes = [vp, ctypes.c_int32, _PD, _PD, ctypes.c_int64]
    L.qtb_evaluate.restype = ctypes.c_int
    L.qtb_evaluate.argtypes = [vp, ctypes.c_int32, _PD, _PD]
    L.qtb_get_noise.restype = ctypes.c_int
    L.qtb_get_noise.argtypes = [vp, ctypes.c_int32, _PD, ctypes.POINTER(ctypes.c_int64)]
    L.qtb_gaussian.restype = ctypes.c_int
    L.qtb_gaussian.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, vp, vp]
    L.qtb_filter_taps.restype = ctypes.c_int
    L.qtb_filter_taps.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_double, ctypes.c_double, _PD]
    L.qtb_vdos_workspace_bytes.restype = ctypes.c_size_t
    L.qtb_vdos_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.qtb_vdos_spectrum.restype = ctypes.c_int
    L.qtb_vdos_spectrum.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_int64, vp, ctypes.c_int32, vp, vp, ctypes.c_size_t,
                                    vp]
    L.qtb_vdos_spectrum_noalloc.restype = ctypes.c_int
    L.qtb_vdos_spectrum_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_int64, vp, ctypes.c_int32, vp, vp]
    L.qtb_vdos_attach.restype = ctypes.c_int
    L.qtb_vdos_attach.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_size_t]
    L.qtb_vdos_read.restype = ctypes.c_int
    L.qtb_vdos_read.argtypes = [vp, ctypes.c_int32, _PD, ctypes.POINTER(ctypes.c_int64),
                                ctypes.c_int32]
    L.qtb_vdos_detach.restype = ctypes.c_int
    L.qtb_vdos_detach.argtypes = [vp, ctypes.c_int32]
    L.qtb_barostat.restype = ctypes.c_int
    L.qtb_barostat.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int32]
    L.qtb_barostat_piston.restype = ctypes.c_int
    L.qtb_barostat_piston.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int32]
    L.qtb_get_box.restype = ctypes.c_int
    L.qtb_get_box.argtypes = [vp, ctypes.c_int32, _PD]
    L.qtb_get_barostat_state.restype = ctypes.c_int
    L.qtb_get_barostat_state.argtypes = [vp, ctypes.c_int32, _PD]
    L.qtb_set_barostat_state.restype = ctypes.c_int
    L.qtb_set_barostat_state.argtypes = [vp, ctypes.c_int32, _PD]
    L.qtb_set_decomposition.restype = ctypes.c_int
    L.qtb_set_decomposition.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.qtb_set_replica_skin.restype = ctypes.c_int
    L.qtb_set_replica_skin.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    L.qtb_set_group_decomposition.restype = ctypes.c_int
    L.qtb_set_group_decomposition.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.qtb_get_group_decomposition.restype = ctypes.c_int
    L.qtb_get_group_decomposition.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]
    L.qtb_get_decomposition.restype = ctypes.c_int
    L.qtb_get_decomposition.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]
    L.qtb_profile.restype = ctypes.c_int
    L.qtb_profile.argtypes = [vp, ctypes.c_int32]
    L.qtb_profile_read.restype = ctypes.c_int
    L.qtb_profile_read.argtypes = [vp, _PD, ctypes.POINTER(ctypes.c_int64)]
    L.qtb_last_error.restype = ctypes.c_char_p
    L.qtb_last_error.argtypes = [vp]
    L.qtb_destroy.restype = None
    L.qtb_destroy.argtypes = [vp]
    L.qtb_version.restype = ctypes.c_char_p
    L.qtb_version.argtypes = []
    _PF = ctypes.POINTER(ctypes.c_float)
    L.qtb_ml_workspace_bytes.restype = ctypes.c_size_t
    L.qtb_ml_workspace_bytes.argtypes = []
    L.qtb_ml_create.restype = ctypes.c_int
    L.qtb_ml_create.argtypes = [ctypes.POINTER(vp), ctypes.c_double, ctypes.c_double, vp,
                                ctypes.c_size_t, vp]
    L.qtb_ml_init_params.restype = ctypes.c_int
    L.qtb_ml_init_params.argtypes = [vp, ctypes.c_uint64]
    L.qtb_ml_set_params.restype = ctypes.c_int
    L.qtb_ml_set_params.argtypes = [vp, _PF, _PD]
    L.qtb_ml_get_params.restype = ctypes.c_int
    L.qtb_ml_get_params.argtypes = [vp, _PF, _PF, _PD]
    L.qtb_ml_attach.restype = ctypes.c_int
    L.qtb_ml_attach.argtypes = [vp, vp, ctypes.c_int32]
    L.qtb_ml_evaluate.restype = ctypes.c_int
    L.qtb_ml_evaluate.argtypes = [vp, vp, ctypes.c_int32, _PD, _PD, _PF, _PF]
    L.qtb_ml_fit_norm.restype = ctypes.c_int
    L.qtb_ml_fit_norm.argtypes = [vp, vp, vp]
    L.qtb_ml_train_step.restype = ctypes.c_int
    L.qtb_ml_train_step.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, _PD, _PF]
    L.qtb_ml_check.restype = ctypes.c_int
    L.qtb_ml_check.argtypes = [vp, ctypes.c_int32, _PD, _PD, ctypes.POINTER(ctypes.c_int64)]
    L.qtb_ml_last_error.restype = ctypes.c_char_p
    L.qtb_ml_last_error.argtypes = [vp]
    L.qtb_ml_destroy.restype = None
    L.qtb_ml_destroy.argtypes = [vp]
    _lib = L
    return L


def _check(status, ctx=None):
    if status != QTB_OK:
        msg = lib().qtb_last_error(ctx).decode()
        raise QtbError(status, msg)


def _pd(a):
    return a.ctypes.data_as(_PD)


def _torch():
    import torch
    return torch


def current_stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- gaussian
def qtb_filter_taps(kind, T, n_beads, dt, two_nf, hbar, kB):
    """Host FIR design without a context: taps h_k, k = -Nf..Nf-1 (numpy)."""
    out = np.zeros(int(two_nf))
    st = lib().qtb_filter_taps(int(kind), float(T), int(n_beads), float(dt), int(two_nf),
                               float(hbar), float(kB), _pd(out))
    if st != QTB_OK:
        raise QtbError(st, "qtb_filter_taps rejected its arguments")
    return out


def qtb_gaussian(seed, stream, tag, n0, n_rows, d0, n_dof, out=None):
    """Device tensor [n_rows, n_dof] float64 of the library's white noise."""
    torch = _torch()
    if out is None:
        out = torch.empty((n_rows, n_dof), dtype=torch.float64, device="cuda")
    _check(lib().qtb_gaussian(seed, stream, tag, n0, n_rows, d0, n_dof,
                              ctypes.c_void_p(out.data_ptr()), current_stream_ptr()))
    return out


# ---------------------------------------------------------------- spectra
def vdos_spectrum(v, weight, seg, dof_major=False):
    """Velocity spectrum S[k], k = 0..seg/2, of a device series (float64)
    v [n_samples, n_dof] (or [n_dof, n_samples] with dof_major) with device
    weights [n_dof], over its whole segments."""
    torch = _torch()
    if dof_major:
        n_dof, n_samples = v.shape
    else:
        n_samples, n_dof = v.shape
    ts, js = v.stride() if not dof_major else v.stride()[::-1]
    nbytes = lib().qtb_vdos_workspace_bytes(n_dof, seg, 0)
    if nbytes == 0:
        raise QtbError(QTB_E_INVALID, "qtb_vdos_workspace_bytes rejected the sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=v.device)
    out = torch.empty(seg // 2 + 1, dtype=torch.float64, device=v.device)
    _check(lib().qtb_vdos_spectrum(ctypes.c_void_p(v.data_ptr()), n_samples, n_dof, ts, js,
                                   ctypes.c_void_p(weight.data_ptr()), seg,
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                   nbytes, current_stream_ptr()))
    return out


def vdos_spectrum_noalloc(v, weight, seg, dof_major=False, out=None):
    """As vdos_spectrum, through the entry point that allocates nothing (its
    scratch is the library's static per-GPU array); out: optional device
    tensor [seg/2 + 1] float64 that receives S."""
    torch = _torch()
    if dof_major:
        n_dof, n_samples = v.shape
    else:
        n_samples, n_dof = v.shape
    ts, js = v.stride() if not dof_major else v.stride()[::-1]
    if out is None:
        out = torch.empty(seg // 2 + 1, dtype=torch.float64, device=v.device)
    _check(lib().qtb_vdos_spectrum_noalloc(ctypes.c_void_p(v.data_ptr()), n_samples, n_dof, ts,
                                           js, ctypes.c_void_p(weight.data_ptr()), seg,
                                           ctypes.c_void_p(out.data_ptr()),
                                           current_stream_ptr()))
    return out


# ---------------------------------------------------------------- context
@dataclass
class Replica:
    """One replica; positions / velocities [P][dims][N] (numpy, copied to device)."""
    pos: np.ndarray
    species: np.ndarray
    T: float
    gamma: float
    dt: float
    noise: int = NOISE_QTB
    vel: np.ndarray | None = None
    box: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    stream: int = 0
    harm_omega: np.ndarray | None = None


class Context:
    """Owns the device buffers (torch) of a qtb_ctx and forwards the C calls."""

    def __init__(self, potential: dict, replicas: list[Replica], units: dict, *,
                 prec=PREC_FP32, fir=FIR_BF16X3, fir_block_K=64, obs_every=0, max_two_nf=512,
                 graphs=True, autotune=True, stream=None, ml_r_cut=0.0, ml_train=False,
                 fuse=False, noise_blocks=False, list_kernel=False):
        torch = _torch()
        L = lib()
        self._keep = []
        ns = len(potential["mass"])
        arr = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        mass = arr(potential["mass"])
        self._keep.append(mass)
        pot = qtb_potential()
        pot.kind = potential.get("kind", POT_PAIR)
        pot.n_species = ns
        pot.mass = _pd(mass)
        if pot.kind == POT_PAIR:
            tabs = [arr(potential[k]) for k in ("charge", "buck_A", "buck_rho", "buck_C")]
            self._keep += tabs
            pot.charge, pot.buck_A, pot.buck_rho, pot.buck_C = (_pd(t) for t in tabs)
            pot.dsf_alpha = potential["dsf_alpha"]
            pot.r_cut = potential["r_cut"]
            pot.skin = potential["skin"]
        elif pot.kind in (POT_MORSE, POT_DOUBLE_WELL):
            tabs = [arr(potential[k]) for k in ("V0", "d")]
            self._keep += tabs
            pot.onsite_V0, pot.onsite_d = (_pd(t) for t in tabs)
        self.pot = pot
        self.n_rep = len(replicas)
        self.reps = (qtb_replica * self.n_rep)()
        self.d_pos, self.d_vel, self.shapes = [], [], []
        for r, rp in enumerate(replicas):
            pos = arr(rp.pos)
            P, dims, N = pos.shape
            vel = np.zeros_like(pos) if rp.vel is None else arr(rp.vel).reshape(pos.shape)
            dp = torch.from_numpy(pos).to("cuda")
            dv = torch.from_numpy(vel).to("cuda")
            self.d_pos.append(dp)
            self.d_vel.append(dv)
            self.shapes.append((P, dims, N))
            sp = np.ascontiguousarray(rp.species, dtype=np.int32)
            self._keep.append(sp)
            R = self.reps[r]
            R.n_atoms, R.n_beads, R.n_dims, R.noise = N, P, dims, rp.noise
            for a in range(3):
                R.box[a] = float(rp.box[a]) if rp.box is not None else 0.0
            R.T, R.gamma, R.dt = rp.T, rp.gamma, rp.dt
            R.seed, R.stream = rp.seed, rp.stream
            R.species = sp.ctypes.data_as(_PI32)
            if rp.harm_omega is not None:
                hw = arr(rp.harm_omega)
                self._keep.append(hw)
                R.harm_omega = _pd(hw)
            R.d_pos = dp.data_ptr()
            R.d_vel = dv.data_ptr()
        opt = qtb_options()
        opt.hbar, opt.kB = units["hbar"], units["kB"]
        opt.coulomb_k, opt.mass_unit = units.get("coulomb_k", 0.0), units["mass_unit"]
        opt.prec, opt.fir, opt.fir_block_K = prec, fir, fir_block_K
        opt.obs_every, opt.max_two_nf = obs_every, max_two_nf
        opt.flags = (0 if graphs else OPT_NO_GRAPH) | (0 if autotune else OPT_NO_AUTOTUNE) | \
            (OPT_ML_TRAIN if ml_train else 0) | (OPT_FUSE if fuse else 0) | \
            (OPT_NOISE_BLOCKS if noise_blocks else 0) | (OPT_LIST_KERNEL if list_kernel else 0)
        opt.ml_r_cut = ml_r_cut
        self.opt = opt
        nbytes = L.qtb_workspace_bytes(ctypes.byref(pot), self.reps, self.n_rep, ctypes.byref(opt))
        if nbytes == 0:
            raise QtbError(QTB_E_INVALID, "qtb_workspace_bytes rejected the description")
        self.ws_bytes = nbytes
        # torch's allocator returns 512-byte aligned blocks
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        # a stream of its own (default priority): graph capture needs a
        # non-default stream; the C calls that read results synchronise it
        self.torch_stream = stream if stream is not None else torch.cuda.Stream()
        self.stream = ctypes.c_void_p(self.torch_stream.cuda_stream)
        self.ctx = ctypes.c_void_p()
        _check(L.qtb_init(ctypes.byref(self.ctx), ctypes.byref(pot), self.reps, self.n_rep,
                          ctypes.byref(opt), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                          self.stream))

    # -- the C calls ---------------------------------------------------------
    def build_filter(self, replica, kind, two_nf):
        n = two_nf
        taps = np.zeros(n)
        _check(lib().qtb_build_filter(self.ctx, replica, kind, two_nf,
                                      _pd(taps) if replica >= 0 else None), self.ctx)
        return taps

    def step(self, n):
        _check(lib().qtb_step(self.ctx, int(n)), self.ctx)

    def observables(self, replica=0):
        o = qtb_obs()
        _check(lib().qtb_observables(self.ctx, replica, ctypes.byref(o)), self.ctx)
        return o.as_dict()

    def get_state(self, replica=0):
        shape = self.shapes[replica]
        r, v = np.zeros(shape), np.zeros(shape)
        st = ctypes.c_int64()
        _check(lib().qtb_get_state(self.ctx, replica, _pd(r), _pd(v), ctypes.byref(st)), self.ctx)
        return r, v, st.value

    def set_state(self, replica, pos, vel, step):
        shape = self.shapes[replica]
        p = None if pos is None else np.ascontiguousarray(pos, dtype=np.float64).reshape(shape)
        v = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64).reshape(shape)
        _check(lib().qtb_set_state(self.ctx, replica, None if p is None else _pd(p),
                                   None if v is None else _pd(v), int(step)), self.ctx)

    def set_positions(self, d_pos):
        """New positions for every replica from a device tensor holding the
        replicas' [P][n_dims][N] arrays one after another (FP64): copied into
        the context's state arrays on its stream, then taken by the library
        (qtb_set_state with null arrays: every list rebuilt, every force
        recomputed; velocities and step unchanged)."""
        torch = _torch()
        src = d_pos.reshape(-1)
        if src.numel() != sum(dp.numel() for dp in self.d_pos):
            raise ValueError("set_positions: size does not match the replicas")
        self.torch_stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.torch_stream):
            # one fused multi-tensor copy rather than a copy per replica
            torch._foreach_copy_([dp.view(-1) for dp in self.d_pos],
                                 list(src.split([dp.numel() for dp in self.d_pos])))
        st = ctypes.c_int64()
        _check(lib().qtb_get_state(self.ctx, 0, None, None, ctypes.byref(st)), self.ctx)
        _check(lib().qtb_set_state(self.ctx, 0, None, None, st.value), self.ctx)

    def evaluate(self, replica=0):
        shape = self.shapes[replica]
        f = np.zeros(shape)
        e = np.zeros(shape[0])
        _check(lib().qtb_evaluate(self.ctx, replica, _pd(f), _pd(e)), self.ctx)
        return f, e

    def get_noise(self, replica=0):
        P, dims, N = self.shapes[replica]
        z = np.zeros((self.opt.fir_block_K, dims * N * P))
        n0 = ctypes.c_int64()
        _check(lib().qtb_get_noise(self.ctx, replica, _pd(z), ctypes.byref(n0)), self.ctx)
        return z, n0.value

    def profile(self, enable: bool):
        _check(lib().qtb_profile(self.ctx, 1 if enable else 0), self.ctx)

    def profile_read(self):
        ms = np.zeros(N_PHASES)
        n = np.zeros(N_PHASES, dtype=np.int64)
        _check(lib().qtb_profile_read(self.ctx, _pd(ms),
                                      n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), self.ctx)
        return {PHASES[q]: (float(ms[q]), int(n[q])) for q in range(N_PHASES)}

    # -- velocity spectrum ------------------------------------------------------
    def vdos_attach(self, replica, seg):
        torch = _torch()
        P, dims, N = self.shapes[replica]
        nbytes = lib().qtb_vdos_workspace_bytes(dims * N, seg, 1)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        _check(lib().qtb_vdos_attach(self.ctx, replica, seg, ctypes.c_void_p(ws.data_ptr()),
                                     nbytes), self.ctx)
        if not hasattr(self, "_vdos_ws"):
            self._vdos_ws = {}
        self._vdos_ws[replica] = (ws, seg)

    def vdos_read(self, replica=0, restart=False):
        """(S [seg/2 + 1], number of segments averaged)."""
        seg = getattr(self, "_vdos_ws", {}).get(replica, (None, 16))[1]
        S = np.zeros(seg // 2 + 1)
        n = ctypes.c_int64()
        _check(lib().qtb_vdos_read(self.ctx, replica, _pd(S), ctypes.byref(n),
                                   1 if restart else 0), self.ctx)
        return S, n.value

    def vdos_detach(self, replica=0):
        _check(lib().qtb_vdos_detach(self.ctx, replica), self.ctx)
        getattr(self, "_vdos_ws", {}).pop(replica, None)

    # -- constant pressure --------------------------------------------------------
    def barostat(self, replica, P0, tau_p, beta_T, enable=True):
        """Isotropic stochastic cell rescaling of a replica's box (P0 in
        energy / length^3, tau_p in time, beta_T in length^3 / energy)."""
        _check(lib().qtb_barostat(self.ctx, replica, float(P0), float(tau_p), float(beta_T),
                                  1 if enable else 0), self.ctx)

    def piston(self, replica, P0, tau_p, gamma_p, enable=True):
        """Isotropic Langevin piston of a replica's box (P0 in energy /
        length^3, tau_p the piston's time scale, gamma_p its friction in
        1 / time)."""
        _check(lib().qtb_barostat_piston(self.ctx, replica, float(P0), float(tau_p),
                                         float(gamma_p), 1 if enable else 0), self.ctx)

    def set_decomposition(self, waves_per_atom, half_groups=False):
        """Pin the pair-force kernel's decomposition (no autotuning)."""
        _check(lib().qtb_set_decomposition(self.ctx, int(waves_per_atom),
                                           1 if half_groups else 0), self.ctx)

    def decomposition(self):
        w, h = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qtb_get_decomposition(self.ctx, ctypes.byref(w), ctypes.byref(h)), self.ctx)
        return w.value, bool(h.value)

    def set_replica_skin(self, replica, skin):
        """Neighbour-list skin of one replica (-1: all), at most the potential's."""
        _check(lib().qtb_set_replica_skin(self.ctx, int(replica), float(skin)), self.ctx)

    def set_group_decomposition(self, group_width, waves_per_atom, half_groups=False):
        """Pin the decomposition of the force launch of one bead-group width."""
        _check(lib().qtb_set_group_decomposition(self.ctx, int(group_width), int(waves_per_atom),
                                                 1 if half_groups else 0), self.ctx)

    def group_decomposition(self, group_width):
        w, h = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qtb_get_group_decomposition(self.ctx, int(group_width), ctypes.byref(w),
                                                 ctypes.byref(h)), self.ctx)
        return w.value, bool(h.value)

    def box(self, replica=0):
        b = np.zeros(3)
        _check(lib().qtb_get_box(self.ctx, replica, _pd(b)), self.ctx)
        return b

    def barostat_state(self, replica=0):
        """(p_e, s, s_v1, s_v2): piston momentum and the pending scalings."""
        b = np.zeros(4)
        _check(lib().qtb_get_barostat_state(self.ctx, replica, _pd(b)), self.ctx)
        return b

    def set_barostat_state(self, replica, state):
        b = np.ascontiguousarray(state, dtype=np.float64)
        if b.shape != (4,):
            raise ValueError("barostat state is (p_e, s, s_v1, s_v2)")
        _check(lib().qtb_set_barostat_state(self.ctx, replica, _pd(b)), self.ctx)

    # -- surrogate --------------------------------------------------------------
    def ml_attach(self, model, check_every=0):
        self._model = model
        _check(lib().qtb_ml_attach(self.ctx, model.m if model is not None else None,
                                   int(check_every)), self.ctx)

    def ml_evaluate(self, model, replica=0):
        """Surrogate forces [P][3][N], energies [P], descriptors and dE/dG [P][N][96]."""
        P, dims, N = self.shapes[replica]
        f = np.zeros((P, dims, N))
        e = np.zeros(P)
        G = np.zeros((P, N, ML_FEATURES), dtype=np.float32)
        g = np.zeros((P, N, ML_FEATURES), dtype=np.float32)
        PF = ctypes.POINTER(ctypes.c_float)
        _check(lib().qtb_ml_evaluate(self.ctx, model.m, replica, _pd(f), _pd(e),
                                     G.ctypes.data_as(PF), g.ctypes.data_as(PF)), self.ctx)
        return f, e, G, g

    def ml_fit_norm(self, model, d_eref):
        _check(lib().qtb_ml_fit_norm(self.ctx, model.m, ctypes.c_void_p(d_eref.data_ptr())),
               self.ctx)

    def ml_train_step(self, model, d_eref, d_fref, w_E, w_F, lr, update=True, want_grad=False):
        """One loss / gradient / Adam step over the replicas (frames) of this context."""
        loss = ctypes.c_double()
        grad = np.zeros(ML_PARAMS, dtype=np.float32) if want_grad else None
        _check(lib().qtb_ml_train_step(
            self.ctx, model.m, ctypes.c_void_p(d_eref.data_ptr()),
            ctypes.c_void_p(d_fref.data_ptr()), float(w_E), float(w_F), float(lr),
            1 if update else 0, ctypes.byref(loss),
            grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None), self.ctx)
        return (loss.value, grad) if want_grad else loss.value

    def ml_check(self, replica=0):
        rmse, rel = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().qtb_ml_check(self.ctx, replica, ctypes.byref(rmse), ctypes.byref(rel),
                                  ctypes.byref(n)), self.ctx)
        return rmse.value, rel.value, n.value

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().qtb_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pair_potential_dict(p) -> dict:
    """From workloads.PairPotential to the dict Context takes."""
    return dict(kind=POT_PAIR, mass=p.mass, charge=p.charge, buck_A=p.buck_A,
                buck_rho=p.buck_rho, buck_C=p.buck_C, dsf_alpha=p.dsf_alpha, r_cut=p.r_cut,
                skin=p.skin)


class Model:
    """A surrogate model in a torch-owned device buffer (qtb_ml)."""

    def __init__(self, r_cut=6.0, r_min=0.5, stream=None):
        torch = _torch()
        L = lib()
        nbytes = L.qtb_ml_workspace_bytes()
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        self.torch_stream = stream if stream is not None else torch.cuda.Stream()
        self.m = ctypes.c_void_p()
        _check_ml(L.qtb_ml_create(ctypes.byref(self.m), r_cut, r_min,
                                  ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                  ctypes.c_void_p(self.torch_stream.cuda_stream)), None)
        self.r_cut, self.r_min = r_cut, r_min

    def init_params(self, seed):
        _check_ml(lib().qtb_ml_init_params(self.m, seed), self.m)

    def set_params(self, params=None, norm=None):
        PF = ctypes.POINTER(ctypes.c_float)
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        n = None if norm is None else np.ascontiguousarray(norm, dtype=np.float64)
        _check_ml(lib().qtb_ml_set_params(self.m, None if p is None else p.ctypes.data_as(PF),
                                          None if n is None else _pd(n)), self.m)

    def get_params(self):
        """(master FP32, values the kernels use, normalisation FP64)."""
        PF = ctypes.POINTER(ctypes.c_float)
        p = np.zeros(ML_PARAMS, dtype=np.float32)
        u = np.zeros(ML_PARAMS, dtype=np.float32)
        n = np.zeros(ML_NORM)
        _check_ml(lib().qtb_ml_get_params(self.m, p.ctypes.data_as(PF), u.ctypes.data_as(PF),
                                          _pd(n)), self.m)
        return p, u, n

    def close(self):
        if getattr(self, "m", None) and self.m.value:
            lib().qtb_ml_destroy(self.m)
            self.m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_ml(status, m):
    if status != QTB_OK:
        raise QtbError(status, lib().qtb_ml_last_error(m).decode())
