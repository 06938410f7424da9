/*
 * nep.h -- C ABI of the MI355X (gfx950) NEP3 library.
 *
 * The library evaluates the neuroevolution potential NEP3 of Fan et al.
 * (GPUMD, Sec. II): per-atom site energies U_i (eq. Ui), forces
 * F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji) (eqs. F_ij, F_i) and per-atom virials
 * W_i = sum_j r_ij (x) dU_j/dr_ji (eq. virial), and drives velocity-Verlet NVE
 * dynamics with them.  Every step of the computation runs in hand-written HIP
 * kernels for gfx950; the host code only validates, allocates and launches.
 *
 * Conventions
 *   units        Angstrom, eV, amu, fs; velocities in Angstrom/fs
 *   positions    SoA float64 [3][N]: x[0..N), then y, then z
 *   box          float64[9]: the cell vectors a, b, c as rows
 *                (a_x a_y a_z b_x b_y b_z c_x c_y c_z), det > 0
 *   pbc          int32[3], nonzero = periodic along a, b, c
 *   types        int32[N] in [0, n_types)
 *   forces       float64 [3][N]
 *   virials      float64 [9][N]: row 3a+b holds W_ab of every atom
 *   totals       float64[10]: E = sum U_i, then W_xx, W_xy, .. W_zz summed
 *   Neighbours of i are all images (j, n) with |d|^2 < r_c^2 in float64,
 *   d = (r_j - r_i) + ((n_a a + n_b b) + n_c c), except (i, 0).  Positions need
 *   not be wrapped into the cell.
 *
 * Ownership and threading: every input and output buffer belongs to the
 * caller.  A handle owns its device workspaces (neighbour lists, descriptor
 * sums, partial forces), grown on demand by the host-synchronous calls.
 * A handle is bound to one device and is not re-entrant: calls on one handle
 * must not overlap.  Different handles are independent.
 *
 * Errors: every int-returning call returns NEP_OK (0) or a NEP_E_* code and
 * never aborts; nep_last_error() gives a message.  On error the outputs are
 * unspecified.
 */
#ifndef NEP_H
#define NEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NEP_OK 0
#define NEP_E_INVALID_ARG 1      /* bad hyper-parameter, size, type or pointer */
#define NEP_E_BOX 2              /* det(box) <= 0, non-finite, or cell too thin */
#define NEP_E_NONFINITE 3        /* NaN or Inf in positions or velocities */
#define NEP_E_NEIGHBOR_OVERFLOW 4/* a neighbour row exceeded its capacity */
#define NEP_E_OOM 5              /* device allocation failed */
#define NEP_E_HIP 6              /* a HIP runtime call failed */
#define NEP_E_UNSUPPORTED 7      /* no GPU, or a hyper-parameter beyond limits */
#define NEP_E_BUDGET 8           /* serving: request larger than the budget */
#define NEP_PENDING 9            /* serving: result not ready yet */

#define NEP_MLP_FP32 0           /* network GEMMs in FP32 on MFMA */
#define NEP_MLP_BF16 1           /* BF16 operands, FP32 accumulation, on MFMA */

/* Hyper-parameters (names follow the paper's notation, Sec. II and III.A). */
typedef struct nep_hparams {
  int32_t n_types;        /* N_typ >= 1 */
  double rc_radial;       /* r_c^R (Angstrom) */
  double rc_angular;      /* r_c^A, 0 < r_c^A <= r_c^R */
  int32_t n_max_radial;   /* n_max^R: radial functions n = 0..n_max^R (<= 15) */
  int32_t n_max_angular;  /* n_max^A (<= 15) */
  int32_t basis_radial;   /* N_bas^R: basis functions k = 0..N_bas^R (<= 15) */
  int32_t basis_angular;  /* N_bas^A (<= 15) */
  int32_t l_max_3b;       /* 1..6; 1..4 are printed in the paper, 5 and 6 use
                             real solid harmonics with the addition theorem */
  int32_t l_max_4b;       /* 0, or 2 (3 is the same): adds q_{n222} */
  int32_t l_max_5b;       /* 0, or 1: adds q_{n1111} */
  int32_t n_neurons;      /* N_neu, 1..128 */
  int32_t nn_per_type;    /* 0: one network (eq. Ui); 1: one network per species */
  int32_t mlp_precision;  /* NEP_MLP_FP32 or NEP_MLP_BF16 */
  int32_t max_nb_radial;  /* neighbour-row capacity M_R (0 = from density) */
  int32_t max_nb_angular; /* neighbour-row capacity M_A (0 = from density) */
  double skin;            /* Verlet skin for nep_md_run (Angstrom, >= 0) */
} nep_hparams;

typedef struct nep_handle nep_handle;

/* Descriptor length N_des (Sec. II.D), or -1 for invalid hyper-parameters. */
int nep_num_descriptors(const nep_hparams *hp);

/* Length of the parameter vector (Sec. II.E, N_par of NEP3; with
 * nn_per_type = 1 the network block is repeated per species), or 0 if hp is
 * invalid.  Layout, float64: for each network t (1 or n_types of them)
 * w0[N_neu][N_des] row-major, b0[N_neu], w1[N_neu]; then b1; then
 * c^R[t_i][t_j][n][k] (n <= n_max^R, k <= N_bas^R); then c^A[t_i][t_j][n][k]. */
size_t nep_num_params(const nep_hparams *hp);

/* Create a handle on the current HIP device from hyper-parameters and a
 * parameter vector of n_params = nep_num_params(hp) doubles (host memory,
 * copied).  Returns NEP_E_UNSUPPORTED when no GPU is present. */
int nep_create(const nep_hparams *hp, const double *params, size_t n_params,
               nep_handle **out);

/* Replace the parameter vector (same hyper-parameters). */
int nep_set_params(nep_handle *h, const double *params, size_t n_params);

void nep_destroy(nep_handle *h);

/* Message of the last error on this handle (or of the last nep_create on
 * this thread when h is NULL).  Valid until the next call on the handle. */
const char *nep_last_error(const nep_handle *h);

/* Energy, forces and virial of one structure (eqs. Ui, F_ij, F_i, virial).
 * Host pointers; energy (per-atom, [N]), force ([3][N]), virial ([9][N]) and
 * totals ([10]) may each be NULL.  Synchronous. */
int nep_compute(nep_handle *h, int64_t n_atoms, const double *pos,
                const int32_t *types, const double box[9], const int32_t pbc[3],
                double *energy, double *force, double *virial, double totals[10]);

/* Same as nep_compute with device pointers (pos, types, energy, force, virial,
 * totals all in device memory; outputs may be NULL) on the HIP stream
 * `stream` (hipStream_t, NULL = default).  box and pbc are host arrays.
 * Returns after the work is enqueued and the neighbour-capacity check has
 * been read back. */
int nep_compute_dev(nep_handle *h, int64_t n_atoms, const double *pos,
                    const int32_t *types, const double box[9], const int32_t pbc[3],
                    double *energy, double *force, double *virial, double *totals,
                    void *stream);

/* Heat current of one structure (Sec. II.E).  Per-atom J_i = W_i . v_i
 * (eq. Ji), J_i,a = sum_b W_i,ab v_i,b with the per-atom virial W_i of
 * eq. virial (units eV * A/fs for v in A/fs), and the total J = sum_i J_i
 * (eq. J-1).  Host pointers: vel [3][N] (required, finite), heat [3][N]
 * (may be NULL), total [3] (may be NULL).  The total is summed in float64 in
 * a fixed order: the same inputs give the same bits.  Synchronous.  Errors as
 * nep_compute, plus NEP_E_NONFINITE for non-finite velocities. */
int nep_heat_current(nep_handle *h, int64_t n_atoms, const double *pos, const double *vel,
                     const int32_t *types, const double box[9], const int32_t pbc[3],
                     double *heat, double total[3]);

/* Same as nep_heat_current with pos, vel, types, heat and total in device
 * memory on `stream` (hipStream_t, NULL = default); box and pbc are host
 * arrays.  The velocity values are not inspected (non-finite velocities give
 * non-finite currents).  Returns after the work is enqueued. */
int nep_heat_current_dev(nep_handle *h, int64_t n_atoms, const double *pos, const double *vel,
                         const int32_t *types, const double box[9], const int32_t pbc[3],
                         double *heat, double *total, void *stream);

/* Neighbour rows at the radial (which = 0) or angular (which = 1) cutoff,
 * as defined above, for diagnostics and parity.  Host pointers: count[N];
 * nbr[N][cap] neighbour indices and shift[N][cap][3] integer images n, each
 * row sorted by (j, n) lexicographically.  Rows longer than cap fail with
 * NEP_E_NEIGHBOR_OVERFLOW. */
int nep_neighbors(nep_handle *h, int64_t n_atoms, const double *pos,
                  const double box[9], const int32_t pbc[3], int32_t which,
                  int32_t cap, int32_t *count, int32_t *nbr, int32_t *shift);

/* Descriptor vectors q[N][N_des] (host, float64) in the order: radial q_n,
 * then q_{nl} (index n_R + (l-1) n_A + n), then q_{n222}, then q_{n1111}
 * (eqs. qin, S_nk and the explicit angular forms of Sec. II.D). */
int nep_descriptors(nep_handle *h, int64_t n_atoms, const double *pos,
                    const int32_t *types, const double box[9], const int32_t pbc[3],
                    double *q);

/* Zero-temperature elastic constants C11, C12, C44 (GPa) of a cubic crystal
 * by the energy-strain relation with +-strain (Sec. V "Elastic constants",
 * where strain = 0.01): the total energy is evaluated for the cell and
 * positions deformed by F = I + eps (r -> F r, cell vectors a -> F a) at
 * eps = 0 and +-strain along three paths, and
 *   C11 = E''(uniaxial xx) / V,  C11 + C12 = E''(biaxial xx = yy) / (2V),
 *   C44 = E''(shear xy = yx = strain / 2, so the engineering shear is strain) / V,
 * E'' = (E(+) + E(-) - 2 E(0)) / strain^2 and V the unstrained volume.  Atoms
 * are not relaxed inside the cell (exact for one-atom Bravais lattices).
 * Host arrays; 0 < strain < 0.2.  Seven evaluations; synchronous. */
int nep_elastic_cubic(nep_handle *h, int64_t n_atoms, const double *pos, const int32_t *types,
                      const double box[9], const int32_t pbc[3], double strain, double C[3]);

/* Latent-space vectors (Sec. IV, the active-learning scheme): for every atom
 * the N_neu products w1_mu h_mu of the hidden-layer states
 * h_mu = tanh(sum_nu w0_{mu nu} q_nu - b0_mu) and their weights to the
 * output (eq. Ui), so that sum_mu latent[i][mu] - b1 = U_i.  Host pointers:
 * latent [N][N_neu] float64, in the caller's atom order, computed with the
 * float32 or bf16 network the handle was created with.  A structure's vector
 * is the mean (or sum) of its atoms' rows.  Synchronous. */
int nep_latent(nep_handle *h, int64_t n_atoms, const double *pos, const int32_t *types,
               const double box[9], const int32_t pbc[3], double *latent);

/* Training loss of eq. loss (Sec. II.E) for each of n_param_sets parameter
 * vectors, from the outputs of nep_compute_batch on the same structures:
 *   L = l_e RMSE(energy per atom over structures)
 *     + l_f RMSE(force components over the 3N components)
 *     + l_v RMSE(virial per atom over the structures that have virial
 *                targets and the six components xx, yy, zz, xy, yz, zx)
 *     + l_1 mean|z| + l_2 sqrt(mean z^2),  lambda = {l_e, l_f, l_v, l_1, l_2}.
 * offsets (host, int64[n_struct+1], offsets[0] = 0, every structure >= 1
 * atom) and lambda (host, [5]) are host arrays; all others are device
 * pointers: force [P][3][N] and totals [P][n_struct][10] as written by
 * nep_compute_batch; energy_target [n_struct] (eV/atom); force_target
 * [3][N] (eV/A); virial_target [n_struct][6] (eV/atom) or NULL (no virial
 * term); a structure whose row holds a NaN has no virial target (training
 * sets give virials for some structures only), and the virial RMSE is
 * normalised by 6 times the number of structures that have one (0 if none);
 * params [P][n_par] or NULL (no regularisers; otherwise n_par must be
 * nep_num_params).  loss [P][6] receives [L, RMSE_e, RMSE_f, RMSE_v,
 * mean|z|, sqrt(mean z^2)]; absent terms read 0.  1 <= n_param_sets <= 65535.
 * Sums are float64 in a fixed order (same inputs, same bits).  Asynchronous
 * on `stream`, except that growing the workspace or new offsets (copied to the
 * device, then free for the caller to change) synchronise once. */
int nep_batch_loss(nep_handle *h, int32_t n_struct, const int64_t *offsets, int32_t n_param_sets,
                   const double *params, int64_t n_par, const double *force, const double *totals,
                   const double *energy_target, const double *force_target,
                   const double *virial_target, const double lambda[5], double *loss,
                   void *stream);

/* nep_batch_loss for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results (bitwise), with its
 * workspace in a fixed 1 MiB array in each GPU's memory instead of the
 * handle's growable buffers.  It allocates nothing.  The workspace holds
 * 6 n_param_sets C doubles of partial sums, C = min(256, max(1,
 * (3N + 16383) / 16384)), plus the n_struct + 1 offsets (rounded to 256
 * bytes); a larger batch fails with NEP_E_INVALID_ARG.  Every call on one GPU
 * uses the same array, and nothing in it needs to start at zero (each call
 * writes all of its partial sums before reading them): calls that overlap on
 * one GPU (different streams or threads) race.  Synchronous on `stream`. */
int nep_batch_loss_noalloc(nep_handle *h, int32_t n_struct, const int64_t *offsets,
                           int32_t n_param_sets, const double *params, int64_t n_par,
                           const double *force, const double *totals,
                           const double *energy_target, const double *force_target,
                           const double *virial_target, const double lambda[5], double *loss,
                           void *stream);

/* One step of the separable natural evolution strategy (SNES, Schaul et al.
 * 2011) that trains NEP (Sec. II.E).  The search distribution has mean
 * mean[n_par] and scales sigma[n_par]; the population that produced loss was
 * z_k = mean + sigma * noise[k] (see nep_snes_sample) with standard-normal
 * noise [n_pop][n_par] supplied by the caller.  Member k's loss is
 * loss[k * loss_stride] (so the [P][6] output of nep_batch_loss can be passed
 * with stride 6); members are ranked by loss, ties to the lower index, with
 * every non-finite loss (NaN or Inf: a diverged member) ranked after all
 * finite ones, and rank r gets the utility max(0, ln(P/2+1) - ln(r+1)) / sum
 * - 1/P.  Then
 *   mean  += eta_mu * sigma * sum_k u_k noise[k]
 *   sigma *= exp(eta_sigma / 2 * sum_k u_k (noise[k]^2 - 1))
 * in place.  The usual rates are eta_mu = 1 and
 * eta_sigma = (3 + ln n_par) / (5 sqrt n_par).  All arrays are device
 * pointers.
 * 2 <= n_pop <= 1024.  Asynchronous on `stream`; calls on one handle share a
 * small utility buffer and must not overlap. */
int nep_snes_step(nep_handle *h, int64_t n_par, int32_t n_pop, double *mean, double *sigma,
                  const double *noise, const double *loss, int64_t loss_stride, double eta_mu,
                  double eta_sigma, void *stream);

/* SNES population population[k][i] = mean[i] + sigma[i] * noise[k][i]
 * (device pointers, [n_pop][n_par]; 1 <= n_pop <= 65535), the parameter
 * vectors to pass to nep_compute_batch.  Asynchronous on `stream`. */
int nep_snes_sample(nep_handle *h, int64_t n_par, int32_t n_pop, const double *mean,
                    const double *sigma, const double *noise, double *population, void *stream);

/* Velocity-Verlet NVE for n_steps of dt_fs (the 'nve' ensemble of the paper,
 * Sec. IV): v += dt/2 F/m; r += dt v; F(r); v += dt/2 F/m.  pos and vel
 * (host, [3][N]) are updated in place.  mass_per_type: amu, [n_types].
 * Every thermo_every steps (0 = never) a row of 13 doubles
 * [step, E_pot, E_kin, T, W_xx .. W_zz] is written to thermo (host,
 * [n_steps / thermo_every][13]); T uses 3N - 3 degrees of freedom.
 * Neighbour rows are kept at r_c + skin and rebuilt when an atom has moved
 * more than skin / 2 since the last build. */
int nep_md_run(nep_handle *h, int64_t n_atoms, double *pos, double *vel,
               const int32_t *types, const double *mass_per_type,
               const double box[9], const int32_t pbc[3], double dt_fs,
               int64_t n_steps, int64_t thermo_every, double *thermo);

/* Same as nep_md_run with pos, vel, types and thermo in device memory on
 * `stream`; mass_per_type, box and pbc are host arrays.  Synchronous. */
int nep_md_run_dev(nep_handle *h, int64_t n_atoms, double *pos, double *vel,
                   const int32_t *types, const double *mass_per_type,
                   const double box[9], const int32_t pbc[3], double dt_fs,
                   int64_t n_steps, int64_t thermo_every, double *thermo,
                   void *stream);

/* ---- NVT and NPT ensembles (Sec. II.F lists them; each follows its own
 * publication) ----
 *   NEP_ENS_BERENDSEN      after each velocity-Verlet step v *= sqrt(1 + dt/tau_t (T0/T - 1))
 *                          (Berendsen et al. 1984)
 *   NEP_ENS_BDP            stochastic velocity rescaling (Bussi, Donadio, Parrinello 2007):
 *                          K' = K + (1-c)(K0 (R1^2 + S)/Nf - K) + 2 R1 sqrt(c (1-c) K0 K / Nf),
 *                          c = exp(-dt/tau_t), K0 = Nf kB T0 / 2, S = a sum of Nf - 1 squared normals
 *   NEP_ENS_LANGEVIN       Bussi-Parrinello (2007) splitting: v = c1 v + sqrt((1 - c1^2) kB T0/m) xi,
 *                          c1 = exp(-dt/(2 tau_t)), before and after each velocity-Verlet step
 *   NEP_ENS_NHC            Nose-Hoover chain of nhc_length (Martyna, Klein, Tuckerman 1992),
 *                          Q1 = Nf kB T0 tau_t^2, Qk = kB T0 tau_t^2, Trotter-split around the step
 *   NEP_ENS_NPT_BERENDSEN  Berendsen thermostat, then P = (2K + tr W)/(3V) and box and positions
 *                          scaled by mu = (1 - beta dt/tau_p (P0 - P))^(1/3)
 *   NEP_ENS_NPT_SCR        BDP thermostat, then stochastic cell rescaling (Bernetti, Bussi 2020):
 *                          d eps = -(beta/tau_p)(P0 - P - kB T0/V) dt + sqrt(2 kB T0 beta dt/(V tau_p)) R,
 *                          positions and box scaled by exp(d eps/3), velocities by exp(-d eps/3)
 * Nf = 3N - 3.  Order of one step: chain half step (NHC) or Ornstein-Uhlenbeck
 * half step (Langevin); v += dt/2 F/m; r += dt v; forces; v += dt/2 F/m;
 * thermostat; P; thermo row; barostat (the next step starts from the forces
 * of the unscaled positions).  Random numbers: Philox4x32-10 (Salmon et al.
 * 2011) of the counter (index, step, stream, 0) under the key (seed low word,
 * seed high word), each call giving four normals by the Box-Muller
 * transform of the uniform pairs (w0, w1), (w2, w3), u = (w + 1/2) 2^-32;
 * step = state[0] + the 1-based step of the call; Langevin: streams 1 and 2
 * (the two half steps), index = the caller's atom index, normals x, y, z;
 * BDP: R1 = the first normal of stream 3 index 0, S from stream 4 (the
 * normals of indices 0, 1, ... in order); SCR: stream 5 index 0. */
#define NEP_ENS_NVE 0
#define NEP_ENS_BERENDSEN 1
#define NEP_ENS_BDP 2
#define NEP_ENS_LANGEVIN 3
#define NEP_ENS_NHC 4
#define NEP_ENS_NPT_BERENDSEN 5
#define NEP_ENS_NPT_SCR 6

typedef struct nep_ensemble {
  int32_t kind;             /* NEP_ENS_* */
  double temperature;       /* T0 (K) */
  double tau_t;             /* thermostat time (fs): coupling time, 1/friction, chain period */
  int32_t nhc_length;       /* chain length, 1..8 (NEP_ENS_NHC) */
  double pressure;          /* P0 (GPa, NPT) */
  double tau_p;             /* barostat time (fs, NPT) */
  double compressibility;   /* beta (1/GPa, NPT) */
  uint64_t seed;            /* key of the random streams */
} nep_ensemble;

/* Molecular dynamics in one of the ensembles above (NEP_ENS_NVE: the steps
 * of nep_md_run with these rows).  Host arrays as in nep_md_run; box (host, inout) returns the
 * final cell for NPT; thermo rows of 16 doubles [step, E_pot, E_kin, T,
 * W_xx .. W_zz, V (A^3), P (GPa), H~] of the end-of-step state (before the
 * barostat); H~ = E_kin + E_pot + state[1] (+ P0 V for NPT), and for NHC
 * E_kin + E_pot + sum_k (Q_k v_xik^2 / 2 + (Nf if k = 0 else 1) kB T0 xi_k).
 * state (host, inout, 20 doubles, zeros to start): [0] steps done (the step
 * word of the random counters, a whole number below 2^32), [1] energy taken
 * out by thermostat and barostat, [2..9] chain positions, [10..17] chain
 * velocities (1/fs); passing it to the next call continues the run exactly.
 * NPT fails with NEP_E_BOX if the cell shrinks more than 3 % (linear) within
 * one call; a new call from the returned state continues.  Synchronous. */
int nep_md_run_ensemble(nep_handle *h, int64_t n_atoms, double *pos, double *vel,
                        const int32_t *types, const double *mass_per_type, double box[9],
                        const int32_t pbc[3], double dt_fs, int64_t n_steps,
                        int64_t thermo_every, double *thermo, const nep_ensemble *ens,
                        double state[20]);

/* Energies, forces and virials of n_struct structures for n_param_sets
 * parameter vectors in one call: the population evaluation of the SNES
 * trainer (Sec. II.E) on a training-style batch.  Structure s holds atoms
 * [offsets[s], offsets[s+1]) of pos/types (device, [3][N] and [N],
 * N = offsets[n_struct]); offsets (int64[n_struct+1]), boxes ([n_struct][9])
 * and pbc ([n_struct][3], NULL = all periodic) are host arrays.  params is a
 * host array [n_param_sets][nep_num_params] (NULL: the handle's own vector,
 * n_param_sets must then be 1).  Outputs, device, each may be NULL:
 * energy [P][N], force [P][3][N], virial [P][9][N], totals [P][n_struct][10].
 * Neighbour rows are built once for all sets; the per-set passes run as one
 * captured HIP graph.  Synchronous.  Each structure's results equal those of
 * the same structure in a batch of one (bitwise). */
int nep_compute_batch(nep_handle *h, int32_t n_struct, const int64_t *offsets,
                      const double *pos, const int32_t *types, const double *boxes,
                      const int32_t *pbc, int32_t n_param_sets, const double *params,
                      double *energy, double *force, double *virial, double *totals,
                      void *stream);

/* nep_compute_batch with the parameter vectors in device memory: params is
 * a device array [n_param_sets][nep_num_params] (float64), converted to the
 * float32 / bf16 tables by a kernel (bitwise the tables nep_compute_batch
 * builds on the host, so the results are the same bits).  With flags =
 * NEP_BATCH_REUSE_ROWS the caller declares that pos, types, offsets and boxes
 * describe the same structures as in the previous batch call on this handle,
 * whose neighbour rows are then reused (boxes may be NULL); the call fails
 * with NEP_E_INVALID_ARG if that call had other sizes.  The per-set passes
 * (with the table conversion) are captured once into a HIP graph kept in the
 * handle and replayed while the sizes and the params / output pointers are
 * unchanged.  Asynchronous on `stream` when the rows are reused (a training
 * generation of nep_snes_sample, this call, nep_batch_loss and nep_snes_step
 * then never waits on the host); building rows synchronises once. */
#define NEP_BATCH_REUSE_ROWS 1
int nep_compute_batch_dev(nep_handle *h, int32_t n_struct, const int64_t *offsets,
                          const double *pos, const int32_t *types, const double *boxes,
                          const int32_t *pbc, int32_t n_param_sets, const double *params,
                          int32_t flags, double *energy, double *force, double *virial,
                          double *totals, void *stream);

/* ---- serving: continuous batching ----
 * A server owns a handle and a worker thread.  Requests (single energy/force/
 * virial evaluations, or short NVE runs) are copied at submission and queued;
 * at every tick the worker admits queued requests while slots are free and
 * their device-memory estimate fits the budget, then advances every active
 * request by one batched evaluation (and one velocity-Verlet step for MD
 * requests past their initial evaluation) over the concatenated structures.
 * Finished requests leave the batch at the end of the tick; requests that
 * arrive meanwhile join at the next tick.  Per-request results do not depend
 * on the other requests in the batch (bitwise).  While a server exists, the
 * handle must not be used directly. */
#define NEP_REQ_EVAL 0
#define NEP_REQ_MD 1

typedef struct nep_server nep_server;

typedef struct nep_request {
  int32_t kind;                 /* NEP_REQ_EVAL or NEP_REQ_MD */
  int64_t n_atoms;
  const double *pos;            /* host [3][N], copied */
  const double *vel;            /* host [3][N] (MD), copied */
  const int32_t *types;         /* host [N], copied */
  double box[9];
  int32_t pbc[3];
  int64_t n_steps;              /* MD: velocity-Verlet steps */
  double dt_fs;                 /* MD */
  const double *mass_per_type;  /* MD: amu [n_types], copied */
} nep_request;

typedef struct nep_result {
  int32_t status;               /* NEP_OK or the request's error */
  int64_t n_atoms;
  double *energy;               /* caller buffers ([N], [3][N], [9][N], [3][N], [3][N]) or NULL; */
  double *force;                /* for MD requests: values after the last step */
  double *virial;
  double *pos;
  double *vel;
  double totals[10];            /* E, W_xx .. W_zz of the structure */
  double latency_ms;            /* completion - submission */
  double queue_ms;              /* admission - submission */
} nep_result;

typedef struct nep_server_stats_t {
  int64_t submitted, completed, active, queued, ticks;
  double p50_ms, p99_ms, mean_ms, max_ms;   /* request latency */
  double wall_s, busy_s;                    /* first submission to last completion; time in ticks */
  double requests_per_s, atom_steps_per_s;  /* over wall_s */
  double mean_batch_atoms, mean_batch_requests;
  size_t bytes_in_use, hbm_budget;
} nep_server_stats_t;

int nep_server_create(nep_handle *h, size_t hbm_budget_bytes, int32_t max_slots,
                      nep_server **out);
/* Non-blocking; fails with NEP_E_BUDGET if the request alone exceeds the budget. */
int nep_server_submit(nep_server *s, const nep_request *req, uint64_t *ticket);
/* NEP_PENDING until the request is done; wait_ms: 0 = do not wait, < 0 = wait
 * until done.  A result is returned once and then forgotten. */
int nep_server_poll(nep_server *s, uint64_t ticket, int32_t wait_ms, nep_result *out);
int nep_server_stats(nep_server *s, nep_server_stats_t *out);
int nep_server_reset_stats(nep_server *s);
/* Finishes every queued and active request, then stops the worker. */
void nep_server_destroy(nep_server *s);

/* Per-stage timing of the last nep_compute / nep_md_run call, filled when
 * timing was enabled with nep_set_timing(h, 1).  names[i] are static
 * strings; ms[i] is the summed time of that stage, calls[i] its launch
 * count.  Returns the number of stages written (<= max). */
int nep_set_timing(nep_handle *h, int32_t enable);
int nep_get_timing(const nep_handle *h, int32_t max, const char **names,
                   double *ms, int64_t *calls);

/* Kernel shapes the autotuner fixed for this handle (batch = 0: single
 * structure, 1: the batched path): out[7] = {descriptor group size, block,
 * lanes per atom; partial-force group size, block, lanes per atom; gather
 * lanes per atom}.  Zeros before the first evaluation of that kind.  Not
 * from the paper: it names the variants that profiles refer to. */
int nep_get_tuning(const nep_handle *h, int32_t batch, int32_t out[7]);

/* MD schedule counters of this handle since nep_create: out[0] = steps run
 * inside captured groups (with a skin, such a group checks for a row rebuild
 * at its first step only, with each atom's displacement extended by 1.5
 * times its speed times the group's remaining time, and verifies the skin at every
 * later step); out[1] = chunks run again step by step because an atom left
 * the skin between two checks (the chunk restarts from its saved state, so
 * results stay those of rows within the skin); out[2] = row rebuilds of MD
 * runs with a skin; out[3] = runs with a skin that continued from the state
 * the previous run left (no other call on the handle in between, the same
 * box, atom count and buffers, and positions and species equal, bit for bit,
 * to those that run returned: the atom order, rows and forces are then kept
 * instead of being set up again).  NPT runs always set up anew.  Not from the
 * paper: the paper does not describe how its rows are maintained. */
int nep_md_counters(const nep_handle *h, int64_t out[4]);

#ifdef __cplusplus
}
#endif
#endif /* NEP_H */
