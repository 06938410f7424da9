"""Seeded synthetic inputs for the NEP hot path.

This module only *makes inputs*: lattices, random periodic cells, species,
parameter vectors, Maxwell velocities and request streams.  It contains none of
the arithmetic of the NEP method (no descriptors, no network, no forces), so
both the HIP library and the FP64 oracle can consume the same arrays.

Conventions (shared by every consumer):
  * positions are SoA float64 arrays of shape (3, N): rows x, y, z in Angstrom;
  * a box is float64 (9,): the three cell vectors a, b, c as rows
    (a_x a_y a_z b_x b_y b_z c_x c_y c_z);
  * species are int32 in [0, n_types);
  * masses are in amu, velocities in Angstrom/fs, time in fs, energy in eV.

Seeds: structures 2205, weights 10046, velocities 300 unless a caller says
otherwise.  The model hyper-parameters of the five benchmark workloads are in
``WORKLOADS``; the parameter-vector length comes from the library
(``nep_num_params``) or the oracle, never from here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_STRUCT = 2205
SEED_WEIGHTS = 10046
SEED_VEL = 300

KB_EV = 8.617333262e-5           # Boltzmann constant, eV/K (CODATA 2018)
AMU_KG = 1.66053906660e-27       # atomic mass unit, kg
EV_J = 1.602176634e-19           # electron volt, J
# 1 amu * (Angstrom/fs)^2 expressed in eV
AMU_A2_FS2_EV = AMU_KG * 1e10 / EV_J


def hparams(n_types, rc_radial, rc_angular, n_max_radial, n_max_angular,
            basis_radial, basis_angular, l_max_3b, l_max_4b, l_max_5b,
            n_neurons, nn_per_type=0):
    """Plain dict of NEP hyper-parameters (names follow the paper's notation)."""
    return dict(n_types=n_types, rc_radial=float(rc_radial),
                rc_angular=float(rc_angular), n_max_radial=n_max_radial,
                n_max_angular=n_max_angular, basis_radial=basis_radial,
                basis_angular=basis_angular, l_max_3b=l_max_3b,
                l_max_4b=l_max_4b, l_max_5b=l_max_5b, n_neurons=n_neurons,
                nn_per_type=nn_per_type)


# Hyper-parameters of the benchmark workloads.  Where the workload text leaves
# a value open, the reading is recorded in DESIGN.md ("readings").
WORKLOADS = {
    # 216-atom diamond, one FP64 evaluation (parity workload)
    "diamond216": hparams(1, 5.0, 4.0, 4, 4, 7, 7, 4, 0, 0, 30, 0),
    # 131,072-atom 4-species FCC alloy, NVE MD (the throughput workload)
    "fcc131k": hparams(4, 6.0, 5.0, 8, 6, 8, 6, 4, 2, 0, 50, 1),
    # 2,000,000-atom BCC with l_max = 6, 4-body and 5-body terms
    "bcc2m": hparams(1, 6.0, 5.0, 8, 6, 8, 6, 6, 2, 1, 80, 0),
    # training-style batch of small triclinic cells, 3 species
    "train3": hparams(3, 6.0, 3.5, 12, 8, 12, 8, 4, 0, 0, 100, 1),
    # serving stream, 2 species
    "serve2": hparams(2, 6.0, 5.0, 8, 6, 8, 6, 4, 2, 0, 50, 1),
}

MASSES = {
    "diamond216": [12.011],
    "fcc131k": [26.98, 24.305, 63.546, 65.38],
    "bcc2m": [183.84],
    "train3": [26.98, 24.305, 63.546],
    "serve2": [26.98, 63.546],
}


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------

_DIAMOND_BASIS = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75],
    [0.75, 0.75, 0.25]])
_FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5],
                       [0.5, 0.5, 0.0]])
_BCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])


def _cubic_lattice(basis, n, a):
    """Replicate a cubic basis n = (nx, ny, nz) times; returns (3, N), box."""
    nx, ny, nz = n
    cells = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                                 indexing="ij"), -1).reshape(-1, 3)
    frac = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = (frac * a).T.copy()
    box = np.array([nx * a, 0, 0, 0, ny * a, 0, 0, 0, nz * a], dtype=np.float64)
    return np.ascontiguousarray(pos, dtype=np.float64), box


def _as3(n):
    return (n, n, n) if np.isscalar(n) else tuple(n)


def lattice(kind, ncell, a, sigma=0.0, n_types=1, seed=SEED_STRUCT):
    """Cubic lattice ('diamond', 'fcc', 'bcc') with Gaussian displacements.

    Every Cartesian component is displaced by N(0, sigma^2); species are drawn
    uniformly at random from [0, n_types).
    """
    basis = {"diamond": _DIAMOND_BASIS, "fcc": _FCC_BASIS,
             "bcc": _BCC_BASIS}[kind]
    pos, box = _cubic_lattice(basis, _as3(ncell), a)
    rng = np.random.default_rng(seed)
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    types = rng.integers(0, n_types, size=pos.shape[1]).astype(np.int32)
    return np.ascontiguousarray(pos), types, box


def diamond216(seed=SEED_STRUCT):
    return lattice("diamond", 3, 5.43, 0.05, 1, seed)


def fcc131k(ncell=32, seed=SEED_STRUCT):
    return lattice("fcc", ncell, 4.05, 0.0, 4, seed)


def bcc2m(ncell=100, seed=SEED_STRUCT):
    return lattice("bcc", ncell, 3.16, 0.08, 1, seed)


def bcc_subcell(seed=SEED_STRUCT):
    """8x8x8 BCC sub-cell (1,024 atoms) with the same thermal noise."""
    return lattice("bcc", 8, 3.16, 0.08, 1, seed)


# --------------------------------------------------------------------------
# random periodic cells (training-style batches)
# --------------------------------------------------------------------------

def _face_widths(box):
    h = box.reshape(3, 3)
    vol = abs(np.linalg.det(h))
    return np.array([vol / np.linalg.norm(np.cross(h[1], h[2])),
                     vol / np.linalg.norm(np.cross(h[2], h[0])),
                     vol / np.linalg.norm(np.cross(h[0], h[1]))])


def random_cell(n_atoms, rho, tilt, dmin, n_types, rng, max_tries=200000):
    """One random triclinic periodic cell with n_atoms at density rho.

    The cell is a cube of side (N/rho)^(1/3) times (I + eps) with the
    off-diagonal strains eps ~ U(-tilt, tilt).  Atoms are placed by random
    sequential addition with minimum image separation dmin (the separation is
    relaxed by 2% after many rejections so every cell can be filled).
    """
    side = (n_atoms / rho) ** (1.0 / 3.0)
    eps = rng.uniform(-tilt, tilt, size=(3, 3))
    np.fill_diagonal(eps, 0.0)
    h = side * (np.eye(3) + eps)           # rows are the cell vectors
    hinv = np.linalg.inv(h)
    fr = np.zeros((0, 3))
    d2 = dmin * dmin
    tries = 0
    while fr.shape[0] < n_atoms:
        s = rng.random(3)
        if fr.shape[0]:
            ds = fr - s
            ds -= np.rint(ds)
            dc = ds @ h
            if np.min(np.einsum("ij,ij->i", dc, dc)) < d2:
                tries += 1
                if tries > max_tries // 100 and tries % (max_tries // 100) == 0:
                    d2 *= 0.98 ** 2
                continue
        fr = np.vstack([fr, s])
    pos = (fr @ h).T.copy()
    types = rng.integers(0, n_types, size=n_atoms).astype(np.int32)
    del hinv
    return np.ascontiguousarray(pos), types, h.reshape(9).copy()


def random_structures(count=2000, nmin=8, nmax=256, rho=(0.05, 0.09),
                      tilt=0.2, dmin=1.5, n_types=3, seed=SEED_STRUCT):
    """Training-style batch: sizes uniform in [nmin, nmax], random cells."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        r = float(rng.uniform(*rho))
        out.append(random_cell(n, r, tilt, dmin, n_types, rng))
    return out


def concat_structures(structs):
    """Concatenate (pos, types, box) tuples into one batch.

    Returns pos (3, N_tot), types (N_tot,), boxes (S, 9), offsets (S+1,) int64.
    """
    offs = np.zeros(len(structs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([s[1].shape[0] for s in structs])
    pos = np.ascontiguousarray(np.concatenate([s[0] for s in structs], axis=1))
    types = np.ascontiguousarray(np.concatenate([s[1] for s in structs]))
    boxes = np.ascontiguousarray(np.stack([s[2] for s in structs]))
    return pos, types, boxes, offs


# --------------------------------------------------------------------------
# parameters and velocities
# --------------------------------------------------------------------------

def random_params(n_params, seed=SEED_WEIGHTS, sigma=0.1):
    """Every parameter i.i.d. N(0, sigma^2) (sigma is the standard deviation)."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=n_params)


def solid_params(h, n_des, n_params, seed=SEED_WEIGHTS, sigma=0.1):
    """Parameters for MD benchmarks that keep a lattice solid over a run (as a
    trained model does), where i.i.d. weights let the alloy heat up and
    cluster.  Starting from random_params, in the parameter vector (per
    network w0[N_neu][N_des], b0, w1; then b1; c^R[t_i][t_j][n][k]; c^A):
      * c^R of n = 0 is the k = 1 basis function alone (coefficient 1), a
        short-ranged positive radial function, so q_0 grows as neighbours
        come closer;
      * w0 weights on descriptor 0 are 0.02 (the network stays in its linear
        range) and all other w0 weights are scaled by 0.02;
      * w1 = 5 + |w1|, so dU_i/dq_0 > 0: a stiff repulsive term plus a small
        random many-body part.
    Every descriptor still enters the network, so the cost is that of any
    parameter vector of these hyper-parameters."""
    n_types, n_neu, per_type = h["n_types"], h["n_neurons"], h["nn_per_type"]
    n_r, k_r = h["n_max_radial"] + 1, h["basis_radial"] + 1
    p = random_params(n_params, seed, sigma)
    off = 0
    for _ in range(n_types if per_type else 1):
        w0 = p[off:off + n_neu * n_des].reshape(n_neu, n_des)
        w0[:, 1:] *= 0.02
        w0[:, 0] = 0.02
        off += n_neu * n_des + n_neu
        p[off:off + n_neu] = 5.0 + np.abs(p[off:off + n_neu])
        off += n_neu
    off += 1
    c_r = p[off:off + n_types * n_types * n_r * k_r].reshape(n_types, n_types, n_r, k_r)
    c_r[:, :, 0, :] = 0.0
    c_r[:, :, 0, 1] = 1.0
    return p


def population(mean, n_pop, seed=SEED_WEIGHTS + 1, sigma=0.1):
    """SNES-style population z_p = mean + sigma * eps_p, eps_p ~ N(0, I)."""
    rng = np.random.default_rng(seed)
    eps = rng.normal(0.0, 1.0, size=(n_pop, mean.shape[0]))
    return np.ascontiguousarray(mean[None, :] + sigma * eps)


def maxwell_velocities(masses, temperature, seed=SEED_VEL):
    """Maxwell-Boltzmann velocities (3, N) in Angstrom/fs.

    Each component ~ N(0, k_B T / m); the centre-of-mass momentum is removed
    and the velocities are rescaled so the kinetic temperature with
    3N - 3 degrees of freedom equals ``temperature`` exactly.
    """
    m = np.asarray(masses, dtype=np.float64)
    n = m.shape[0]
    rng = np.random.default_rng(seed)
    sd = np.sqrt(KB_EV * temperature / (m * AMU_A2_FS2_EV))
    v = rng.normal(0.0, 1.0, size=(3, n)) * sd[None, :]
    p = (v * m[None, :]).sum(axis=1)
    v -= (p / m.sum())[:, None]
    ek = 0.5 * np.sum(m[None, :] * v * v) * AMU_A2_FS2_EV
    t_now = 2.0 * ek / ((3 * n - 3) * KB_EV)
    if t_now > 0:
        v *= math.sqrt(temperature / t_now)
    return np.ascontiguousarray(v)


# --------------------------------------------------------------------------
# serving stream
# --------------------------------------------------------------------------

@dataclass
class Request:
    arrival_s: float
    kind: str              # "eval" or "md"
    pos: np.ndarray
    types: np.ndarray
    box: np.ndarray
    vel: np.ndarray | None = None
    n_steps: int = 0
    extra: dict = field(default_factory=dict)


def _nearest_replication(n_target, per_cell):
    """Cubic replication count whose atom count is nearest to n_target."""
    k = max(1, int(round((n_target / per_cell) ** (1.0 / 3.0))))
    return k


def serving_stream(n_requests=2000, rate_hz=100.0, nmin=64, nmax=100000,
                   n_types=2, md_steps=100, seed=SEED_STRUCT,
                   masses=(26.98, 63.546), temperature=300.0):
    """Poisson arrivals of eval / short-MD requests with log-uniform sizes.

    Each request is the cubic FCC (a = 4.05) or BCC (a = 3.16) replication
    nearest to its drawn size, species uniform at random, displacement
    sigma = 0.05 Angstrom; half are single evaluations, half are md_steps-step
    NVE runs from 300 K Maxwell velocities.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        n = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        if rng.random() < 0.5:
            kind_l, a, per = "fcc", 4.05, 4
        else:
            kind_l, a, per = "bcc", 3.16, 2
        k = _nearest_replication(n, per)
        pos, types, box = lattice(kind_l, k, a, 0.05, n_types,
                                  seed=int(rng.integers(1 << 31)))
        if rng.random() < 0.5:
            out.append(Request(t, "eval", pos, types, box))
        else:
            m = np.asarray(masses)[types]
            vel = maxwell_velocities(m, temperature,
                                     seed=int(rng.integers(1 << 31)))
            out.append(Request(t, "md", pos, types, box, vel, md_steps))
    return out
