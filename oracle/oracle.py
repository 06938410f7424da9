"""ctypes wrapper of the FP64 NEP oracle (``nep_oracle.c``).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
cpu_baseline leg of ``bench.py`` may import this module.  The HIP library
never calls it and shares nothing with it.

Arrays follow the conventions of ``paper_2205_10046_amd.synth``: positions
(3, N) float64, types (N,) int32, box (9,) float64 with the cell vectors as
rows, per-atom virials (9, N) row-major per atom (W_ab at row 3a + b).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nep_oracle.c")
_LIB = os.environ.get("NEP_ORACLE_LIB",
                      os.path.join(_HERE, "libnep_oracle.so"))

GCC_CMD = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB, "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/libnep_oracle.so (plain gcc, FP64)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        subprocess.run(GCC_CMD, check=True)
    return _LIB


class _HP(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("rc_radial", C.c_double),
                ("rc_angular", C.c_double), ("n_max_radial", C.c_int32),
                ("n_max_angular", C.c_int32), ("basis_radial", C.c_int32),
                ("basis_angular", C.c_int32), ("l_max_3b", C.c_int32),
                ("l_max_4b", C.c_int32), ("l_max_5b", C.c_int32),
                ("n_neurons", C.c_int32), ("nn_per_type", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or (
                os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        pd, pi32, pi64 = P(d), P(i32), P(i64)
        hp = P(_HP)
        L.ora_num_descriptors.argtypes = [hp]
        L.ora_num_descriptors.restype = C.c_int
        L.ora_num_params.argtypes = [hp]
        L.ora_num_params.restype = i64
        L.ora_pairs.argtypes = [i64, pd, pd, pi32, d, i32, pi32, pi32, pi32,
                                pi32]
        L.ora_radial_basis.argtypes = [d, C.c_int, d, pd, pd]
        L.ora_radial_basis.restype = None
        L.ora_angular_poly.argtypes = [C.c_int, pd, pd, pd]
        L.ora_angular_poly.restype = None
        L.ora_coefficients.argtypes = [C.c_int, pd, pd, pd]
        L.ora_coefficients.restype = None
        L.ora_ann.argtypes = [hp, pd, C.c_int, pd, pd]
        L.ora_ann.restype = d
        L.ora_latent.argtypes = [hp, pd, C.c_int, pd, pd]
        L.ora_latent.restype = None
        L.ora_evaluate.argtypes = [hp, pd, i64, pd, pi32, pd, pi32, pd, pd,
                                   pd, pd]
        L.ora_heat_current.argtypes = [hp, pd, i64, pd, pd, pi32, pd, pi32,
                                       pd, pd, pd]
        L.ora_descriptors.argtypes = [hp, pd, i64, pd, pi32, pd, pi32, pd]
        L.ora_evaluate_atoms.argtypes = [hp, pd, i64, pd, pi32, pd, pi32,
                                         i64, pi64, pd, pd, pd]
        L.ora_md_nve.argtypes = [hp, pd, i64, pd, pd, pi32, pd, pd, pi32, d,
                                 i64, i64, pd]
        L.ora_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.ora_philox4x32_10.restype = None
        L.ora_normal4.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, pd]
        L.ora_normal4.restype = None
        L.ora_md_ensemble.argtypes = [hp, pd, i64, pd, pd, pi32, pd, pd, pi32, d, i64, i64, pd,
                                      C.POINTER(_Ensemble), pd]
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_set_threads.restype = None
        L.ora_get_threads.restype = C.c_int
        _lib = L
    return _lib


class _Ensemble(C.Structure):
    _fields_ = [("kind", C.c_int32), ("temperature", C.c_double), ("tau_t", C.c_double),
                ("nhc_length", C.c_int32), ("pressure", C.c_double), ("tau_p", C.c_double),
                ("compressibility", C.c_double), ("seed", C.c_uint64)]


ENSEMBLES = {"nve": 0, "nvt_berendsen": 1, "nvt_bdp": 2, "nvt_langevin": 3, "nvt_nhc": 4,
             "npt_berendsen": 5, "npt_scr": 6}


def _hp(h):
    return _HP(**{k: h[k] for k, _ in _HP._fields_})


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pbc(pbc):
    return _i32(np.ones(3) if pbc is None else pbc)


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


def num_descriptors(h) -> int:
    return int(lib().ora_num_descriptors(C.byref(_hp(h))))


def num_params(h) -> int:
    return int(lib().ora_num_params(C.byref(_hp(h))))


def radial_basis(rc, K, r):
    f = np.zeros(K)
    df = np.zeros(K)
    lib().ora_radial_basis(float(rc), int(K), float(r), _p(f, C.c_double),
                           _p(df, C.c_double))
    return f, df


def angular_poly(lmax, d):
    nb = (lmax + 1) ** 2 - 1
    d = _f64(d)
    b = np.zeros(nb)
    g = np.zeros(3 * nb)
    lib().ora_angular_poly(int(lmax), _p(d, C.c_double), _p(b, C.c_double),
                           _p(g, C.c_double))
    return b, g.reshape(nb, 3)


def coefficients(lmax):
    nb = (lmax + 1) ** 2 - 1
    c3 = np.zeros(max(nb, 48))
    c4 = np.zeros(5)
    c5 = np.zeros(3)
    lib().ora_coefficients(int(lmax), _p(c3, C.c_double), _p(c4, C.c_double),
                           _p(c5, C.c_double))
    return c3[:nb], c4, c5


def pairs(pos, box, rc, pbc=None, cap=None):
    """Neighbour rows at cutoff rc: list of (j array, shift (m,3) array)."""
    pos = _f64(pos)
    box = _f64(box)
    n = pos.shape[1]
    if cap is None:
        cap = 512
    while True:
        cnt = np.zeros(n, np.int32)
        nb = np.zeros(n * cap, np.int32)
        sh = np.zeros(n * cap * 3, np.int32)
        mx = C.c_int32(0)
        err = lib().ora_pairs(n, _p(pos, C.c_double), _p(box, C.c_double),
                              _p(_pbc(pbc), C.c_int32), float(rc), cap,
                              _p(cnt, C.c_int32), _p(nb, C.c_int32),
                              _p(sh, C.c_int32), C.byref(mx))
        if err:
            raise RuntimeError(f"ora_pairs failed ({err})")
        if mx.value <= cap:
            break
        cap = mx.value
    nb = nb.reshape(n, cap)
    sh = sh.reshape(n, cap, 3)
    return [(nb[i, :cnt[i]].copy(), sh[i, :cnt[i]].copy()) for i in range(n)]


def ann(h, params, type_, q):
    params = _f64(params)
    q = _f64(q)
    fp = np.zeros_like(q)
    u = lib().ora_ann(C.byref(_hp(h)), _p(params, C.c_double), int(type_),
                      _p(q, C.c_double), _p(fp, C.c_double))
    return u, fp


def latent(h, params, pos, types, box, pbc=None):
    """Per-atom latent-space vectors (Sec. IV), (N, N_neu): the descriptors
    of each site through the hidden layer, times the output weights."""
    q = descriptors(h, params, pos, types, box, pbc)
    params = _f64(params)
    types = _i32(types)
    out = np.zeros((q.shape[0], h["n_neurons"]))
    for i in range(q.shape[0]):
        qi = np.ascontiguousarray(q[i])
        li = np.zeros(h["n_neurons"])
        lib().ora_latent(C.byref(_hp(h)), _p(params, C.c_double), int(types[i]),
                         _p(qi, C.c_double), _p(li, C.c_double))
        out[i] = li
    return out


def evaluate(h, params, pos, types, box, pbc=None, want_q=False):
    """Full evaluation: returns dict U (N,), F (3,N), W (9,N) [, q (N,Nd)]."""
    params = _f64(params)
    pos = _f64(pos)
    types = _i32(types)
    box = _f64(box)
    n = pos.shape[1]
    U = np.zeros(n)
    F = np.zeros((3, n))
    W = np.zeros((9, n))
    q = np.zeros((n, num_descriptors(h))) if want_q else None
    err = lib().ora_evaluate(C.byref(_hp(h)), _p(params, C.c_double), n,
                             _p(pos, C.c_double), _p(types, C.c_int32),
                             _p(box, C.c_double), _p(_pbc(pbc), C.c_int32),
                             _p(U, C.c_double), _p(F, C.c_double),
                             _p(W, C.c_double),
                             _p(q, C.c_double) if want_q else None)
    if err:
        raise RuntimeError(f"ora_evaluate failed ({err})")
    out = dict(U=U, F=F, W=W)
    if want_q:
        out["q"] = q
    return out


def heat_current(h, params, pos, vel, types, box, pbc=None):
    """Heat current (Sec. II.E): J_i = W_i . v_i per atom (eq. Ji, (3,N)),
    its sum (eq. J-1) and the total by eq. J-2 (partial forces of each atom
    contracted with its neighbours' velocities).  Returns (J_atom, J1, J2)."""
    params = _f64(params)
    pos = _f64(pos)
    vel = _f64(vel)
    types = _i32(types)
    box = _f64(box)
    n = pos.shape[1]
    Ja = np.zeros((3, n))
    J1 = np.zeros(3)
    J2 = np.zeros(3)
    err = lib().ora_heat_current(C.byref(_hp(h)), _p(params, C.c_double), n,
                                 _p(pos, C.c_double), _p(vel, C.c_double),
                                 _p(types, C.c_int32), _p(box, C.c_double),
                                 _p(_pbc(pbc), C.c_int32), _p(Ja, C.c_double),
                                 _p(J1, C.c_double), _p(J2, C.c_double))
    if err:
        raise RuntimeError(f"ora_heat_current failed ({err})")
    return Ja, J1, J2


def descriptors(h, params, pos, types, box, pbc=None):
    params = _f64(params)
    pos = _f64(pos)
    types = _i32(types)
    box = _f64(box)
    n = pos.shape[1]
    q = np.zeros((n, num_descriptors(h)))
    err = lib().ora_descriptors(C.byref(_hp(h)), _p(params, C.c_double), n,
                                _p(pos, C.c_double), _p(types, C.c_int32),
                                _p(box, C.c_double), _p(_pbc(pbc), C.c_int32),
                                _p(q, C.c_double))
    if err:
        raise RuntimeError(f"ora_descriptors failed ({err})")
    return q


def evaluate_atoms(h, params, pos, types, box, idx, pbc=None):
    """U (k,), F (k,3), W (k,9) of the atoms idx only (large structures)."""
    params = _f64(params)
    pos = _f64(pos)
    types = _i32(types)
    box = _f64(box)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    k = idx.shape[0]
    U = np.zeros(k)
    F = np.zeros((k, 3))
    W = np.zeros((k, 9))
    err = lib().ora_evaluate_atoms(C.byref(_hp(h)), _p(params, C.c_double),
                                   pos.shape[1], _p(pos, C.c_double),
                                   _p(types, C.c_int32), _p(box, C.c_double),
                                   _p(_pbc(pbc), C.c_int32), k,
                                   _p(idx, C.c_int64), _p(U, C.c_double),
                                   _p(F, C.c_double), _p(W, C.c_double))
    if err:
        raise RuntimeError(f"ora_evaluate_atoms failed ({err})")
    return dict(U=U, F=F, W=W)


def md_nve(h, params, pos, vel, types, mass_per_type, box, dt, n_steps,
           thermo_every, pbc=None):
    """Run NVE; returns (pos, vel, thermo rows (n_rows, 13))."""
    params = _f64(params)
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    types = _i32(types)
    m = _f64(mass_per_type)
    box = _f64(box)
    rows = n_steps // thermo_every if thermo_every > 0 else 0
    th = np.zeros((max(rows, 1), 13))
    err = lib().ora_md_nve(C.byref(_hp(h)), _p(params, C.c_double),
                           pos.shape[1], _p(pos, C.c_double),
                           _p(vel, C.c_double), _p(types, C.c_int32),
                           _p(m, C.c_double), _p(box, C.c_double),
                           _p(_pbc(pbc), C.c_int32), float(dt), int(n_steps),
                           int(thermo_every), _p(th, C.c_double))
    if err:
        raise RuntimeError(f"ora_md_nve failed ({err})")
    return pos, vel, th[:rows]


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al. 2011) of a 4-word counter and 2-word key."""
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def normal4(seed, index, step, stream):
    """Four standard normals of counter (index, step, stream) under seed."""
    z = np.zeros(4)
    lib().ora_normal4(int(seed), int(index), int(step), int(stream), _p(z, C.c_double))
    return z


def md_ensemble(h, params, pos, vel, types, mass_per_type, box, dt, n_steps, thermo_every,
                ens, state=None, pbc=None):
    """MD in one of the ensembles (see ora_md_ensemble): ens is a dict with
    kind (a name of ENSEMBLES), temperature (K), tau_t (fs), nhc_length,
    pressure (GPa), tau_p (fs), compressibility (1/GPa), seed.  Returns
    (pos, vel, box, thermo rows (n_rows, 16), state (20,))."""
    e = _Ensemble(kind=ENSEMBLES[ens["kind"]], temperature=ens.get("temperature", 300.0),
                  tau_t=ens.get("tau_t", 100.0), nhc_length=ens.get("nhc_length", 4),
                  pressure=ens.get("pressure", 0.0), tau_p=ens.get("tau_p", 1000.0),
                  compressibility=ens.get("compressibility", 0.01), seed=ens.get("seed", 0))
    params = _f64(params)
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    box = _f64(box).copy()
    types = _i32(types)
    m = _f64(mass_per_type)
    st = np.zeros(20) if state is None else _f64(state).copy()
    rows = n_steps // thermo_every if thermo_every > 0 else 0
    th = np.zeros((max(rows, 1), 16))
    err = lib().ora_md_ensemble(C.byref(_hp(h)), _p(params, C.c_double), pos.shape[1],
                                _p(pos, C.c_double), _p(vel, C.c_double), _p(types, C.c_int32),
                                _p(m, C.c_double), _p(box, C.c_double), _p(_pbc(pbc), C.c_int32),
                                float(dt), int(n_steps), int(thermo_every),
                                _p(th, C.c_double), C.byref(e), _p(st, C.c_double))
    if err:
        raise RuntimeError(f"ora_md_ensemble failed ({err})")
    return pos, vel, box, th[:rows], st


# ---------------------------------------------------------------------------
# elastic constants of a cubic crystal by the energy-strain relation
# (Sec. V "Elastic constants": +-1 % strains)
# ---------------------------------------------------------------------------

EV_A3_GPA = 160.21766208


def strained(pos, box, eps):
    """Positions and box under the homogeneous deformation r -> (I + eps) r."""
    Fm = np.eye(3) + np.asarray(eps, float)
    return (Fm @ np.asarray(pos, float)), (np.asarray(box, float).reshape(3, 3) @ Fm.T).ravel()


def elastic_cubic(h, params, pos, types, box, delta=0.01):
    """C11, C12, C44 (GPa) from energies at +-delta strains: uniaxial xx
    (E'' = V C11), biaxial xx = yy (E'' = 2 V (C11 + C12)) and shear
    xy = yx = delta/2 (E'' = V C44), each second derivative by the central
    difference (E(+) + E(-) - 2 E(0)) / delta^2.  Atoms are not relaxed."""
    V = abs(np.linalg.det(np.asarray(box, float).reshape(3, 3)))

    def energy(eps):
        p, b = strained(pos, box, eps)
        return evaluate(h, params, p, types, b)["U"].sum()
    e0 = energy(np.zeros((3, 3)))

    def second(eps):
        e = np.asarray(eps, float) * delta
        return (energy(e) + energy(-e) - 2.0 * e0) / (delta * delta)
    c11 = second([[1, 0, 0], [0, 0, 0], [0, 0, 0]]) / V
    c11_12 = second([[1, 0, 0], [0, 1, 0], [0, 0, 0]]) / (2.0 * V)
    c44 = second([[0, 0.5, 0], [0.5, 0, 0], [0, 0, 0]]) / V
    return np.array([c11, c11_12 - c11, c44]) * EV_A3_GPA


# ---------------------------------------------------------------------------
# training loss (Sec. II.E, eq. loss)
# ---------------------------------------------------------------------------

# the six independent virial components: xx, yy, zz, xy, yz, zx (row 3a + b)
VIRIAL6 = (0, 4, 8, 1, 5, 6)


def loss_terms(e_pred, f_pred, w_pred, e_tar, f_tar, w_tar, z, lam):
    """Eq. loss written out.  e_* (S,) energy per atom of each structure,
    f_* (3, N) forces, w_* (S, 6) virial per atom in VIRIAL6 order (w_tar None:
    no virial term; a target row with a NaN: that structure has no virial, and
    the virial RMSE runs over the others), z (N_par,) parameters, lam
    (lambda_e, lambda_f, lambda_v,
    lambda_1, lambda_2).  Returns [L, L_e, L_f, L_v, L_1, L_2] where L is the
    weighted sum and the others are the unweighted terms (RMSEs and norms)."""
    e_pred, e_tar = np.asarray(e_pred, float), np.asarray(e_tar, float)
    f_pred, f_tar = np.asarray(f_pred, float), np.asarray(f_tar, float)
    z = np.asarray(z, float)
    S, N, npar = e_pred.shape[0], f_pred.shape[1], z.shape[0]
    le = math.sqrt(sum((e_pred[n] - e_tar[n]) ** 2 for n in range(S)) / S)
    lf = math.sqrt(float(((f_pred - f_tar) ** 2).sum()) / (3 * N))
    lv = 0.0
    if w_tar is not None:
        # a structure whose virial target row holds a NaN has no virial target
        w_tar = np.asarray(w_tar, float)
        have = [n for n in range(S) if not np.isnan(w_tar[n]).any()]
        if have:
            d = np.asarray(w_pred, float)[have] - w_tar[have]
            lv = math.sqrt(float((d ** 2).sum()) / (6 * len(have)))
    l1 = float(np.abs(z).sum()) / npar
    l2 = math.sqrt(float((z ** 2).sum()) / npar)
    total = lam[0] * le + lam[1] * lf + lam[2] * lv + lam[3] * l1 + lam[4] * l2
    return np.array([total, le, lf, lv, l1, l2])


def predictions(h, params, structs):
    """Per-structure energy per atom (S,), forces (3, N) and virial per atom
    (S, 6) of a list of (pos, types, box) structures."""
    e, f, w = [], [], []
    for pos, types, box in structs:
        r = evaluate(h, params, pos, types, box)
        n = pos.shape[1]
        e.append(r["U"].sum() / n)
        f.append(r["F"])
        w.append(r["W"].sum(axis=1)[list(VIRIAL6)] / n)
    return np.array(e), np.concatenate(f, axis=1), np.array(w)


# ---------------------------------------------------------------------------
# separable natural evolution strategy (SNES), the trainer of Sec. II.E
# ---------------------------------------------------------------------------
# The paper cites SNES (Schaul et al. 2011) without restating it; this follows
# that published algorithm: a Gaussian search distribution with mean mu and
# per-parameter scale sigma, population z_k = mu + sigma * s_k with standard
# normal s_k (passed in, never drawn here), fitness-shaped utilities by rank,
# and natural-gradient steps on mu and log(sigma).

def snes_rates(n_par):
    """Default learning rates of SNES: eta_mu = 1, eta_sigma = (3 + ln d)/(5 sqrt d)."""
    return 1.0, (3.0 + math.log(n_par)) / (5.0 * math.sqrt(n_par))


def snes_utilities(n_pop):
    """Utility of rank k (0 = best): max(0, ln(lambda/2 + 1) - ln(k + 1)),
    normalised to sum 1, minus 1/lambda."""
    raw = [max(0.0, math.log(n_pop / 2.0 + 1.0) - math.log(k + 1.0)) for k in range(n_pop)]
    tot = sum(raw)
    return np.array([r / tot - 1.0 / n_pop for r in raw])


def snes_ranks(losses):
    """Rank of each member, 0 for the smallest loss; ties go to the lower
    index; a non-finite loss (NaN, Inf: a diverged member) ranks after every
    finite one, non-finite ones among themselves by index."""
    L = [float(x) for x in losses]

    def key(k):
        return (0, L[k], k) if math.isfinite(L[k]) else (1, 0.0, k)
    order = sorted(range(len(L)), key=key)
    ranks = np.zeros(len(L), dtype=int)
    for r, k in enumerate(order):
        ranks[k] = r
    return ranks


def snes_step(mean, sigma, noise, losses, eta_mu, eta_sigma):
    """One SNES update from the population's standard-normal draws noise
    (P, d) and losses (P,).  Returns the new (mean, sigma)."""
    mean, sigma, noise = (np.asarray(a, dtype=np.float64) for a in (mean, sigma, noise))
    u = snes_utilities(noise.shape[0])[snes_ranks(losses)]
    g_mu = np.zeros_like(mean)
    g_sigma = np.zeros_like(mean)
    for k in range(noise.shape[0]):
        g_mu += u[k] * noise[k]
        g_sigma += u[k] * (noise[k] ** 2 - 1.0)
    return mean + eta_mu * sigma * g_mu, sigma * np.exp(0.5 * eta_sigma * g_sigma)


def snes_sample(mean, sigma, noise):
    """Population z_k = mean + sigma * s_k, (P, d)."""
    return np.asarray(mean)[None, :] + np.asarray(sigma)[None, :] * np.asarray(noise)
