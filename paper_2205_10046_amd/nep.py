"""Thin ctypes binding of the HIP library ``libnep_hip.so`` (include/nep.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  Host-array calls take numpy arrays; the ``*_dev``
calls take torch tensors on the GPU (torch is used for device memory and the
current stream only).  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnep_hip.so")

NEP_OK = 0
NEP_E_INVALID_ARG = 1
NEP_E_BOX = 2
NEP_E_NONFINITE = 3
NEP_E_NEIGHBOR_OVERFLOW = 4
NEP_E_OOM = 5
NEP_E_HIP = 6
NEP_E_UNSUPPORTED = 7
NEP_E_BUDGET = 8
NEP_PENDING = 9
NEP_MLP_FP32 = 0
NEP_MLP_BF16 = 1

# every entry point declared in include/nep.h
EXPORTS = ["nep_num_descriptors", "nep_num_params", "nep_create", "nep_set_params",
           "nep_destroy", "nep_last_error", "nep_compute", "nep_compute_dev",
           "nep_heat_current", "nep_heat_current_dev", "nep_neighbors", "nep_descriptors",
           "nep_latent", "nep_elastic_cubic", "nep_md_run", "nep_md_run_dev", "nep_md_run_ensemble",
           "nep_compute_batch", "nep_compute_batch_dev", "nep_batch_loss", "nep_batch_loss_noalloc", "nep_snes_step",
           "nep_snes_sample", "nep_set_timing", "nep_get_timing", "nep_get_tuning", "nep_md_counters",
           "nep_server_create",
           "nep_server_submit", "nep_server_poll", "nep_server_stats", "nep_server_reset_stats",
           "nep_server_destroy"]

NEP_REQ_EVAL = 0
NEP_REQ_MD = 1


class NepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"NEP error {code}: {msg}")
        self.code = code


class nep_hparams(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("rc_radial", C.c_double),
                ("rc_angular", C.c_double), ("n_max_radial", C.c_int32),
                ("n_max_angular", C.c_int32), ("basis_radial", C.c_int32),
                ("basis_angular", C.c_int32), ("l_max_3b", C.c_int32),
                ("l_max_4b", C.c_int32), ("l_max_5b", C.c_int32),
                ("n_neurons", C.c_int32), ("nn_per_type", C.c_int32),
                ("mlp_precision", C.c_int32), ("max_nb_radial", C.c_int32),
                ("max_nb_angular", C.c_int32), ("skin", C.c_double)]


def make_hparams(h: dict, mlp_precision=NEP_MLP_FP32, max_nb_radial=0,
                 max_nb_angular=0, skin=0.0) -> nep_hparams:
    return nep_hparams(
        n_types=h["n_types"], rc_radial=h["rc_radial"], rc_angular=h["rc_angular"],
        n_max_radial=h["n_max_radial"], n_max_angular=h["n_max_angular"],
        basis_radial=h["basis_radial"], basis_angular=h["basis_angular"],
        l_max_3b=h["l_max_3b"], l_max_4b=h["l_max_4b"], l_max_5b=h["l_max_5b"],
        n_neurons=h["n_neurons"], nn_per_type=h.get("nn_per_type", 0),
        mlp_precision=h.get("mlp_precision", mlp_precision),
        max_nb_radial=h.get("max_nb_radial", max_nb_radial),
        max_nb_angular=h.get("max_nb_angular", max_nb_angular),
        skin=h.get("skin", skin))


ENSEMBLES = {"nve": 0, "nvt_berendsen": 1, "nvt_bdp": 2, "nvt_langevin": 3, "nvt_nhc": 4,
             "npt_berendsen": 5, "npt_scr": 6}


class nep_ensemble(C.Structure):
    _fields_ = [("kind", C.c_int32), ("temperature", C.c_double), ("tau_t", C.c_double),
                ("nhc_length", C.c_int32), ("pressure", C.c_double), ("tau_p", C.c_double),
                ("compressibility", C.c_double), ("seed", C.c_uint64)]


class nep_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_atoms", C.c_int64),
                ("pos", C.POINTER(C.c_double)), ("vel", C.POINTER(C.c_double)),
                ("types", C.POINTER(C.c_int32)), ("box", C.c_double * 9),
                ("pbc", C.c_int32 * 3), ("n_steps", C.c_int64), ("dt_fs", C.c_double),
                ("mass_per_type", C.POINTER(C.c_double))]


class nep_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_atoms", C.c_int64),
                ("energy", C.POINTER(C.c_double)), ("force", C.POINTER(C.c_double)),
                ("virial", C.POINTER(C.c_double)), ("pos", C.POINTER(C.c_double)),
                ("vel", C.POINTER(C.c_double)), ("totals", C.c_double * 10),
                ("latency_ms", C.c_double), ("queue_ms", C.c_double)]


class nep_server_stats_t(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "active", "queued", "ticks")] + \
               [(k, C.c_double) for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "wall_s",
                                          "busy_s", "requests_per_s", "atom_steps_per_s",
                                          "mean_batch_atoms", "mean_batch_requests")] + \
               [("bytes_in_use", C.c_size_t), ("hbm_budget", C.c_size_t)]


_lib = None


def load():
    """Load libnep_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    # torch bundles its own HIP runtime under the same soname; loading it first
    # makes the library bind to that one, so the process holds a single HIP/HSA
    # runtime shared with the torch tensors and streams passed to *_dev calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
    pd, pi32 = P(d), P(i32)
    hp = P(nep_hparams)
    L.nep_num_descriptors.argtypes = [hp]
    L.nep_num_descriptors.restype = C.c_int
    L.nep_num_params.argtypes = [hp]
    L.nep_num_params.restype = C.c_size_t
    L.nep_create.argtypes = [hp, pd, C.c_size_t, P(vp)]
    L.nep_set_params.argtypes = [vp, pd, C.c_size_t]
    L.nep_destroy.argtypes = [vp]
    L.nep_destroy.restype = None
    L.nep_last_error.argtypes = [vp]
    L.nep_last_error.restype = C.c_char_p
    L.nep_compute.argtypes = [vp, i64, pd, pi32, pd, pi32, pd, pd, pd, pd]
    L.nep_compute_dev.argtypes = [vp, i64, vp, vp, pd, pi32, vp, vp, vp, vp, vp]
    L.nep_heat_current.argtypes = [vp, i64, pd, pd, pi32, pd, pi32, pd, pd]
    L.nep_heat_current_dev.argtypes = [vp, i64, vp, vp, vp, pd, pi32, vp, vp, vp]
    L.nep_neighbors.argtypes = [vp, i64, pd, pd, pi32, i32, i32, pi32, pi32, pi32]
    L.nep_descriptors.argtypes = [vp, i64, pd, pi32, pd, pi32, pd]
    L.nep_latent.argtypes = [vp, i64, pd, pi32, pd, pi32, pd]
    L.nep_elastic_cubic.argtypes = [vp, i64, pd, pi32, pd, pi32, d, pd]
    L.nep_md_run.argtypes = [vp, i64, pd, pd, pi32, pd, pd, pi32, d, i64, i64, pd]
    L.nep_md_run_dev.argtypes = [vp, i64, vp, vp, vp, pd, pd, pi32, d, i64, i64, vp, vp]
    L.nep_md_run_ensemble.argtypes = [vp, i64, pd, pd, pi32, pd, pd, pi32, d, i64, i64, pd,
                                      P(nep_ensemble), pd]
    L.nep_compute_batch.argtypes = [vp, i32, P(i64), vp, vp, pd, pi32, i32, pd, vp, vp, vp,
                                    vp, vp]
    L.nep_compute_batch_dev.argtypes = [vp, i32, P(i64), vp, vp, pd, pi32, i32, vp, i32, vp, vp,
                                        vp, vp, vp]
    L.nep_batch_loss.argtypes = [vp, i32, P(i64), i32, vp, i64, vp, vp, vp, vp, vp, pd, vp, vp]
    L.nep_batch_loss_noalloc.argtypes = L.nep_batch_loss.argtypes
    L.nep_snes_step.argtypes = [vp, i64, i32, vp, vp, vp, vp, i64, d, d, vp]
    L.nep_snes_sample.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp]
    L.nep_server_create.argtypes = [vp, C.c_size_t, i32, P(vp)]
    L.nep_server_submit.argtypes = [vp, P(nep_request), P(C.c_uint64)]
    L.nep_server_poll.argtypes = [vp, C.c_uint64, i32, P(nep_result)]
    L.nep_server_stats.argtypes = [vp, P(nep_server_stats_t)]
    L.nep_server_reset_stats.argtypes = [vp]
    L.nep_server_destroy.argtypes = [vp]
    L.nep_server_destroy.restype = None
    L.nep_set_timing.argtypes = [vp, i32]
    L.nep_get_timing.argtypes = [vp, i32, P(C.c_char_p), pd, P(i64)]
    L.nep_get_tuning.argtypes = [vp, i32, P(i32)]
    L.nep_md_counters.argtypes = [vp, P(C.c_int64)]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or C.c_int
    _lib = L
    return L


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def nep_num_params(h: dict) -> int:
    return int(load().nep_num_params(C.byref(make_hparams(h))))


def nep_num_descriptors(h: dict) -> int:
    return int(load().nep_num_descriptors(C.byref(make_hparams(h))))


def last_error(handle=None) -> str:
    m = load().nep_last_error(handle)
    return m.decode() if m else ""


def _torch_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape, name, optional=False):
    """A tensor argument for _devs: (tensor, dtype "f64"/"i32", expected
    shape with None entries free, name, may it be None)."""
    return (t, dtype, shape, name, optional)


def _devs(*args):
    """Device pointers of torch tensors after checking what the kernels
    assume of them: dtype, C-contiguous layout and shape for every argument
    first, then GPU residence.  A mismatch raises NepError before anything
    reaches the library."""
    import torch
    kinds = {"f64": torch.float64, "i32": torch.int32}
    for t, dtype, shape, name, optional in args:
        if t is None:
            if optional:
                continue
            raise NepError(NEP_E_INVALID_ARG, f"{name} is required")
        if not isinstance(t, torch.Tensor):
            raise NepError(NEP_E_INVALID_ARG, f"{name} must be a torch tensor")
        if t.dtype != kinds[dtype]:
            raise NepError(NEP_E_INVALID_ARG, f"{name} must be {kinds[dtype]}, got {t.dtype}")
        if not t.is_contiguous():
            raise NepError(NEP_E_INVALID_ARG, f"{name} must be contiguous")
        if shape is not None and not (t.dim() == len(shape) and all(
                w is None or int(g) == int(w) for g, w in zip(t.shape, shape))):
            raise NepError(NEP_E_INVALID_ARG,
                           f"{name} has shape {tuple(t.shape)}, expected "
                           f"{tuple('*' if w is None else w for w in shape)}")
    for t, _, _, name, _ in args:
        if t is not None and not t.is_cuda:
            raise NepError(NEP_E_INVALID_ARG, f"{name} must be a CUDA tensor")
    return [None if a[0] is None else C.c_void_p(a[0].data_ptr()) for a in args]


class Handle:
    """One nep_handle: hyper-parameters + parameter vector on the current GPU."""

    def __init__(self, h: dict, params, mlp_precision=NEP_MLP_FP32,
                 max_nb_radial=0, max_nb_angular=0, skin=0.0):
        L = load()
        self.h = dict(h)
        self._hp = make_hparams(h, mlp_precision, max_nb_radial, max_nb_angular, skin)
        params = _f64(params)
        out = C.c_void_p()
        rc = L.nep_create(C.byref(self._hp), _ptr(params, C.c_double), params.shape[0],
                          C.byref(out))
        if rc != NEP_OK:
            raise NepError(rc, last_error(None))
        self._h = out
        self.n_types = h["n_types"]
        self.n_des = nep_num_descriptors(h)

    def close(self):
        if getattr(self, "_h", None):
            load().nep_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != NEP_OK:
            raise NepError(rc, last_error(self._h))

    def set_params(self, params):
        params = _f64(params)
        self._check(load().nep_set_params(self._h, _ptr(params, C.c_double), params.shape[0]))

    def compute(self, pos, types, box, pbc=None):
        """nep_compute on host arrays: dict U (N,), F (3,N), W (9,N), totals (10,)."""
        pos, types, box = _f64(pos), _i32(types), _f64(box)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        n = pos.shape[1]
        U, F, W, T = np.zeros(n), np.zeros((3, n)), np.zeros((9, n)), np.zeros(10)
        self._check(load().nep_compute(
            self._h, n, _ptr(pos, C.c_double), _ptr(types, C.c_int32), _ptr(box, C.c_double),
            _ptr(pbc, C.c_int32), _ptr(U, C.c_double), _ptr(F, C.c_double),
            _ptr(W, C.c_double), _ptr(T, C.c_double)))
        return dict(U=U, F=F, W=W, totals=T)

    def compute_dev(self, pos, types, box, pbc=None, energy=None, force=None, virial=None,
                    totals=None):
        """nep_compute_dev on torch CUDA tensors (float64 pos (3,N), int32 types)."""
        box, pbc = _f64(box), _i32(np.ones(3) if pbc is None else pbc)
        n = int(pos.shape[-1])
        args = _devs(_dev(pos, "f64", (3, n), "pos"), _dev(types, "i32", (n,), "types"),
                     _dev(energy, "f64", (n,), "energy", True), _dev(force, "f64", (3, n), "force", True),
                     _dev(virial, "f64", (9, n), "virial", True),
                     _dev(totals, "f64", (10,), "totals", True))
        self._check(load().nep_compute_dev(
            self._h, n, args[0], args[1], _ptr(box, C.c_double), _ptr(pbc, C.c_int32),
            *args[2:], _torch_stream()))

    def heat_current(self, pos, vel, types, box, pbc=None):
        """nep_heat_current on host arrays: (J_i (3,N), total J (3,))."""
        pos, vel, types, box = _f64(pos), _f64(vel), _i32(types), _f64(box)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        n = pos.shape[1]
        J, T = np.zeros((3, n)), np.zeros(3)
        self._check(load().nep_heat_current(
            self._h, n, _ptr(pos, C.c_double), _ptr(vel, C.c_double), _ptr(types, C.c_int32),
            _ptr(box, C.c_double), _ptr(pbc, C.c_int32), _ptr(J, C.c_double),
            _ptr(T, C.c_double)))
        return J, T

    def heat_current_dev(self, pos, vel, types, box, pbc=None, heat=None, total=None):
        """nep_heat_current_dev on torch CUDA tensors (float64 pos/vel (3,N))."""
        box, pbc = _f64(box), _i32(np.ones(3) if pbc is None else pbc)
        n = int(pos.shape[-1])
        a = _devs(_dev(pos, "f64", (3, n), "pos"), _dev(vel, "f64", (3, n), "vel"),
                  _dev(types, "i32", (n,), "types"), _dev(heat, "f64", (3, n), "heat", True),
                  _dev(total, "f64", (3,), "total", True))
        self._check(load().nep_heat_current_dev(
            self._h, n, *a[:3], _ptr(box, C.c_double), _ptr(pbc, C.c_int32), *a[3:],
            _torch_stream()))

    def neighbors(self, pos, box, which=0, pbc=None, cap=256):
        """Rows at the radial (0) or angular (1) cutoff: list of (j, shift (m,3))."""
        pos, box = _f64(pos), _f64(box)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        n = pos.shape[1]
        cnt = np.zeros(n, np.int32)
        nbr = np.zeros(n * cap, np.int32)
        sh = np.zeros(n * cap * 3, np.int32)
        self._check(load().nep_neighbors(
            self._h, n, _ptr(pos, C.c_double), _ptr(box, C.c_double), _ptr(pbc, C.c_int32),
            which, cap, _ptr(cnt, C.c_int32), _ptr(nbr, C.c_int32), _ptr(sh, C.c_int32)))
        nbr = nbr.reshape(n, cap)
        sh = sh.reshape(n, cap, 3)
        return [(nbr[i, :cnt[i]].copy(), sh[i, :cnt[i]].copy()) for i in range(n)]

    def descriptors(self, pos, types, box, pbc=None):
        pos, types, box = _f64(pos), _i32(types), _f64(box)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        n = pos.shape[1]
        q = np.zeros((n, self.n_des))
        self._check(load().nep_descriptors(
            self._h, n, _ptr(pos, C.c_double), _ptr(types, C.c_int32), _ptr(box, C.c_double),
            _ptr(pbc, C.c_int32), _ptr(q, C.c_double)))
        return q

    def elastic_cubic(self, pos, types, box, strain=0.01, pbc=None):
        """nep_elastic_cubic: (C11, C12, C44) in GPa by the energy-strain relation."""
        pos, types, box = _f64(pos), _i32(types), _f64(box)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        out = np.zeros(3)
        self._check(load().nep_elastic_cubic(
            self._h, pos.shape[1], _ptr(pos, C.c_double), _ptr(types, C.c_int32),
            _ptr(box, C.c_double), _ptr(pbc, C.c_int32), float(strain), _ptr(out, C.c_double)))
        return out

    def latent(self, pos, types, box, pbc=None):
        """Per-atom latent-space vectors w1_mu h_mu, (N, N_neu)."""
        pos, types, box = _f64(pos), _i32(types), _f64(box)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        n = pos.shape[1]
        lat = np.zeros((n, self.h["n_neurons"]))
        self._check(load().nep_latent(
            self._h, n, _ptr(pos, C.c_double), _ptr(types, C.c_int32), _ptr(box, C.c_double),
            _ptr(pbc, C.c_int32), _ptr(lat, C.c_double)))
        return lat

    def md_run(self, pos, vel, types, masses, box, dt, n_steps, thermo_every, pbc=None):
        """nep_md_run on host arrays; returns (pos, vel, thermo (rows, 13))."""
        pos, vel = _f64(pos).copy(), _f64(vel).copy()
        types, box, m = _i32(types), _f64(box), _f64(masses)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        rows = n_steps // thermo_every if thermo_every > 0 else 0
        th = np.zeros((max(rows, 1), 13))
        self._check(load().nep_md_run(
            self._h, pos.shape[1], _ptr(pos, C.c_double), _ptr(vel, C.c_double),
            _ptr(types, C.c_int32), _ptr(m, C.c_double), _ptr(box, C.c_double),
            _ptr(pbc, C.c_int32), float(dt), int(n_steps), int(thermo_every),
            _ptr(th, C.c_double)))
        return pos, vel, th[:rows]

    def md_run_ensemble(self, pos, vel, types, masses, box, dt, n_steps, thermo_every, ens,
                        state=None, pbc=None):
        """nep_md_run_ensemble on host arrays.  ens: dict with kind (a name of
        ENSEMBLES), temperature (K), tau_t (fs), nhc_length, pressure (GPa),
        tau_p (fs), compressibility (1/GPa), seed.  Returns (pos, vel, box,
        thermo (rows, 16), state (20,))."""
        e = nep_ensemble(kind=ENSEMBLES[ens["kind"]], temperature=ens.get("temperature", 300.0),
                         tau_t=ens.get("tau_t", 100.0), nhc_length=ens.get("nhc_length", 4),
                         pressure=ens.get("pressure", 0.0), tau_p=ens.get("tau_p", 1000.0),
                         compressibility=ens.get("compressibility", 0.01), seed=ens.get("seed", 0))
        pos, vel = _f64(pos).copy(), _f64(vel).copy()
        types, box, m = _i32(types), _f64(box).copy(), _f64(masses)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        st = np.zeros(20) if state is None else _f64(state).copy()
        rows = n_steps // thermo_every if thermo_every > 0 else 0
        th = np.zeros((max(rows, 1), 16))
        self._check(load().nep_md_run_ensemble(
            self._h, pos.shape[1], _ptr(pos, C.c_double), _ptr(vel, C.c_double),
            _ptr(types, C.c_int32), _ptr(m, C.c_double), _ptr(box, C.c_double),
            _ptr(pbc, C.c_int32), float(dt), int(n_steps), int(thermo_every),
            _ptr(th, C.c_double), C.byref(e), _ptr(st, C.c_double)))
        return pos, vel, box, th[:rows], st

    def md_run_dev(self, pos, vel, types, masses, box, dt, n_steps, thermo_every, thermo,
                   pbc=None):
        """nep_md_run_dev on torch CUDA tensors; thermo is a (rows, 13) float64 tensor."""
        box, m = _f64(box), _f64(masses)
        pbc = _i32(np.ones(3) if pbc is None else pbc)
        n = int(pos.shape[-1])
        rows = n_steps // thermo_every if thermo_every > 0 else 0
        if rows and thermo is not None and thermo.shape[0] < rows:
            raise NepError(NEP_E_INVALID_ARG, f"thermo needs {rows} rows of 13")
        a = _devs(_dev(pos, "f64", (3, n), "pos"), _dev(vel, "f64", (3, n), "vel"),
                  _dev(types, "i32", (n,), "types"),
                  _dev(thermo if rows else None, "f64", (None, 13), "thermo", rows == 0))
        self._check(load().nep_md_run_dev(
            self._h, n, *a[:3], _ptr(m, C.c_double),
            _ptr(box, C.c_double), _ptr(pbc, C.c_int32), float(dt), int(n_steps),
            int(thermo_every), a[3], _torch_stream()))

    def compute_batch(self, offsets, pos, types, boxes, params=None, energy=None, force=None,
                      virial=None, totals=None, pbc=None):
        """nep_compute_batch: pos/types and outputs are torch CUDA tensors; offsets
        (S+1), boxes (S, 9), params (P, N_par) and pbc (S, 3) are numpy arrays."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        boxes = _f64(boxes)
        S = offsets.shape[0] - 1
        P = 1 if params is None else int(np.asarray(params).shape[0])
        params = None if params is None else _f64(params)
        pbc = None if pbc is None else _i32(pbc)
        n = int(offsets[-1])
        if boxes.shape != (S, 9) or (pbc is not None and pbc.shape != (S, 3)):
            raise NepError(NEP_E_INVALID_ARG, "boxes must be (S, 9) and pbc (S, 3)")
        a = _devs(_dev(pos, "f64", (3, n), "pos"), _dev(types, "i32", (n,), "types"),
                  _dev(energy, "f64", (P, n), "energy", True),
                  _dev(force, "f64", (P, 3, n), "force", True),
                  _dev(virial, "f64", (P, 9, n), "virial", True),
                  _dev(totals, "f64", (P, S, 10), "totals", True))
        self._check(load().nep_compute_batch(
            self._h, S, _ptr(offsets, C.c_int64), *a[:2], _ptr(boxes, C.c_double),
            _ptr(pbc, C.c_int32), P, _ptr(params, C.c_double), *a[2:], _torch_stream()))

    def compute_batch_dev(self, offsets, pos, types, boxes, params, energy=None, force=None,
                          virial=None, totals=None, pbc=None, reuse_rows=False):
        """nep_compute_batch_dev: params (P, N_par) float64 on the GPU like pos,
        types and the outputs; offsets, boxes and pbc are host arrays (boxes
        may be None with reuse_rows)."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        S = offsets.shape[0] - 1
        n = int(offsets[-1])
        P = int(params.shape[0])
        boxes = None if boxes is None else _f64(boxes)
        pbc = None if pbc is None else _i32(pbc)
        if boxes is not None and boxes.shape != (S, 9):
            raise NepError(NEP_E_INVALID_ARG, "boxes must be (S, 9)")
        a = _devs(_dev(pos, "f64", (3, n), "pos"), _dev(types, "i32", (n,), "types"),
                  _dev(params, "f64", (P, None), "params"),
                  _dev(energy, "f64", (P, n), "energy", True),
                  _dev(force, "f64", (P, 3, n), "force", True),
                  _dev(virial, "f64", (P, 9, n), "virial", True),
                  _dev(totals, "f64", (P, S, 10), "totals", True))
        self._check(load().nep_compute_batch_dev(
            self._h, S, _ptr(offsets, C.c_int64), a[0], a[1], _ptr(boxes, C.c_double),
            _ptr(pbc, C.c_int32), P, a[2], 1 if reuse_rows else 0, *a[3:], _torch_stream()))

    def batch_loss(self, offsets, force, totals, energy_target, force_target, lam,
                   loss, virial_target=None, params=None, noalloc=False):
        """nep_batch_loss (nep_batch_loss_noalloc with noalloc=True): force
        (P,3,N), totals (P,S,10), targets, params (P,N_par) and loss (P,6) are
        torch CUDA float64 tensors; offsets (S+1) and lam (5) are host arrays."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        lam = _f64(lam)
        if lam.shape != (5,):
            raise NepError(NEP_E_INVALID_ARG, "lam must hold 5 weights")
        S = offsets.shape[0] - 1
        n = int(offsets[-1])
        P = int(force.shape[0])
        npar = 0 if params is None else int(params.shape[-1])
        a = _devs(_dev(params, "f64", (P, npar), "params", True),
                  _dev(force, "f64", (P, 3, n), "force"), _dev(totals, "f64", (P, S, 10), "totals"),
                  _dev(energy_target, "f64", (S,), "energy_target"),
                  _dev(force_target, "f64", (3, n), "force_target"),
                  _dev(virial_target, "f64", (S, 6), "virial_target", True),
                  _dev(loss, "f64", (P, 6), "loss"))
        fn = load().nep_batch_loss_noalloc if noalloc else load().nep_batch_loss
        self._check(fn(self._h, S, _ptr(offsets, C.c_int64), P, a[0], npar, *a[1:6],
                       _ptr(lam, C.c_double), a[6], _torch_stream()))

    def snes_step(self, mean, sigma, noise, loss, eta_mu, eta_sigma, loss_stride=1):
        """nep_snes_step on torch CUDA float64 tensors: mean, sigma (n_par,) in
        place; noise (P, n_par); loss with member k at loss[k * loss_stride]."""
        d, P = int(mean.shape[0]), int(noise.shape[0])
        if loss is not None and loss.numel() < (P - 1) * int(loss_stride) + 1:
            raise NepError(NEP_E_INVALID_ARG, "loss is shorter than n_pop * loss_stride")
        a = _devs(_dev(mean, "f64", (d,), "mean"), _dev(sigma, "f64", (d,), "sigma"),
                  _dev(noise, "f64", (P, d), "noise"), _dev(loss, "f64", None, "loss"))
        self._check(load().nep_snes_step(
            self._h, d, P, *a, int(loss_stride), float(eta_mu), float(eta_sigma), _torch_stream()))

    def snes_sample(self, mean, sigma, noise, population):
        """nep_snes_sample: population (P, n_par) = mean + sigma * noise."""
        d, P = int(mean.shape[0]), int(noise.shape[0])
        a = _devs(_dev(mean, "f64", (d,), "mean"), _dev(sigma, "f64", (d,), "sigma"),
                  _dev(noise, "f64", (P, d), "noise"), _dev(population, "f64", (P, d), "population"))
        self._check(load().nep_snes_sample(self._h, d, P, *a, _torch_stream()))

    def set_timing(self, enable=True):
        self._check(load().nep_set_timing(self._h, 1 if enable else 0))

    def timing(self):
        """{stage: (total ms, launches)} of the calls since set_timing(True)."""
        n = 32
        names = (C.c_char_p * n)()
        ms = np.zeros(n)
        calls = np.zeros(n, np.int64)
        k = load().nep_get_timing(self._h, n, names, _ptr(ms, C.c_double),
                                  _ptr(calls, C.c_int64))
        return {names[i].decode(): (float(ms[i]), int(calls[i])) for i in range(k)}


    def tuning(self, batch=False):
        """Kernel shapes fixed by the autotuner (zeros before the first evaluation)."""
        out = np.zeros(7, np.int32)
        self._check(load().nep_get_tuning(self._h, 1 if batch else 0, _ptr(out, C.c_int32)))
        keys = ("ng_desc", "block_desc", "lanes_desc", "ng_force", "block_force", "lanes_force",
                "lanes_gather")
        return dict(zip(keys, (int(x) for x in out)))

    def md_counters(self):
        """MD schedule counters (nep_md_counters): steps run in captured groups,
        chunks replayed step by step, row rebuilds and runs that continued
        from the previous run's state."""
        out = np.zeros(4, np.int64)
        self._check(load().nep_md_counters(self._h, _ptr(out, C.c_int64)))
        return {"group_steps": int(out[0]), "replayed_chunks": int(out[1]), "rebuilds": int(out[2]),
                "continued_runs": int(out[3])}


class Server:
    """A continuous-batching server (nep_server_*) on a Handle it owns."""

    def __init__(self, handle: Handle, hbm_budget_bytes: int, max_slots: int = 64):
        self.handle = handle
        out = C.c_void_p()
        rc = load().nep_server_create(handle._h, int(hbm_budget_bytes), int(max_slots),
                                      C.byref(out))
        if rc != NEP_OK:
            raise NepError(rc, last_error(handle._h))
        self._s = out
        self._keep = {}

    def submit(self, pos, types, box, kind=NEP_REQ_EVAL, vel=None, masses=None, n_steps=0,
               dt=1.0, pbc=None):
        pos, types, box = _f64(pos), _i32(types), _f64(box)
        vel = None if vel is None else _f64(vel)
        masses = None if masses is None else _f64(masses)
        r = nep_request(kind=kind, n_atoms=pos.shape[1], pos=_ptr(pos, C.c_double),
                        vel=_ptr(vel, C.c_double), types=_ptr(types, C.c_int32),
                        n_steps=int(n_steps), dt_fs=float(dt),
                        mass_per_type=_ptr(masses, C.c_double))
        r.box[:] = list(box)
        r.pbc[:] = [1, 1, 1] if pbc is None else [int(x) for x in pbc]
        t = C.c_uint64()
        rc = load().nep_server_submit(self._s, C.byref(r), C.byref(t))
        if rc != NEP_OK:
            raise NepError(rc, last_error(self.handle._h))
        self._keep[t.value] = (pos.shape[1], kind)
        return t.value

    def poll(self, ticket, wait_ms=0):
        """None while pending, else dict U, F, W, totals, latency_ms [, pos, vel]."""
        n, kind = self._keep[ticket]
        U, F, W = np.zeros(n), np.zeros((3, n)), np.zeros((9, n))
        P, V = (np.zeros((3, n)), np.zeros((3, n))) if kind == NEP_REQ_MD else (None, None)
        r = nep_result(energy=_ptr(U, C.c_double), force=_ptr(F, C.c_double),
                       virial=_ptr(W, C.c_double), pos=_ptr(P, C.c_double),
                       vel=_ptr(V, C.c_double))
        rc = load().nep_server_poll(self._s, C.c_uint64(ticket), int(wait_ms), C.byref(r))
        if rc == NEP_PENDING:
            return None
        del self._keep[ticket]
        if rc != NEP_OK:
            raise NepError(rc, last_error(self.handle._h))
        out = dict(U=U, F=F, W=W, totals=np.array(r.totals[:]), latency_ms=r.latency_ms,
                   queue_ms=r.queue_ms)
        if kind == NEP_REQ_MD:
            out.update(pos=P, vel=V)
        return out

    def stats(self):
        st = nep_server_stats_t()
        rc = load().nep_server_stats(self._s, C.byref(st))
        if rc != NEP_OK:
            raise NepError(rc, last_error(self.handle._h))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def reset_stats(self):
        load().nep_server_reset_stats(self._s)

    def close(self):
        if getattr(self, "_s", None):
            load().nep_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
