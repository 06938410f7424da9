// nep_kernels.h -- argument blocks and launchers of the NEP kernels.
#pragma once
#include <vector>

#include "nep_internal.h"

namespace nep {

struct BuildArgs {
  int64_t N;
  int32_t n_cells;
  const double* pos_ext;      // caller order [3][N]
  const int32_t* types_ext;
  const int32_t* sid_ext;
  const int32_t* ext_src;     // caller index of each source atom (NULL: the source index)
  const StructInfo* structs;
  int32_t* key;               // [N]
  int32_t* cell_count;        // [n_cells]
  int32_t* cell_fill;         // [n_cells]
  int32_t* cell_start;        // [n_cells]
  int32_t* perm;              // [N] internal -> caller index
  double* pos;                // internal [3][N]
  int32_t* types;             // internal
  int32_t* sid;               // internal
  double rcR2, rcA2;
  int32_t* overflow;          // flags: [0] radial row, [1] angular row, [2] rev error,
                              // [5] candidate row overflow (max counts)
  const int32_t* gate;        // rebuild kernels run only when *gate != 0 (NULL: always)
  int32_t wide_rows = 0;      // some structure has no cells: its rows come from k_build_rows_wide
  // optional: velocities and caller indices permuted with the positions
  const double* vel_src = nullptr;
  double* vel_dst = nullptr;
  const int32_t* ext_in = nullptr;
  int32_t* ext_out = nullptr;
};

struct EvalArgs {
  const double* pos;          // internal [3][N]
  int64_t N;
  const int32_t* types;
  const int32_t* sid;
  const StructInfo* structs;
  Lists L;                    // exact rows
  DevModel M;
  float* q;                   // [N][NDp]
  float* fp;                  // [N][NDp]
  float* U;                   // [N]
  float* sums;                // [nA_pad * NB][N]
  float4* P;                  // [MR][N] dU_i/dr_ij per radial entry
  float* F;                   // [3][N] internal
  float* W;                   // [9][N] internal
  float* latent;              // [N][N_neu] w1_mu h_mu of every atom, or NULL
  // optional second half kick fused into the force gather (kick_vel != NULL):
  // v += dt/2 F / m with the float32 force just written, as a separate kick would
  double* kick_vel;
  const double* kick_inv_mass;
  double kick_dt;
  const int32_t* rows;        // network row order, [rows_len]
  int64_t rows_len;
  int32_t ngroups;            // angular radial-function groups
  int32_t NG;                 // group size
  int32_t lanes;              // lanes per atom of the pair kernels (1 or 4)
  int32_t mlp_bf16;
  int32_t block;              // threads per block of the pair kernels (0 = 256)
  int32_t batch;              // several structures: geometry from structs[sid]
  StructInfo st0;             // the geometry when batch == 0
};

// neighbor.hip
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s);
void launch_assign_struct(const int64_t* offs, int32_t n_struct, int64_t N, int32_t* sid,
                          hipStream_t s);
void launch_order_atoms(const BuildArgs& b, hipStream_t s);
// Exact rows at the cutoffs of b from candidate rows V at sqrt(b.rcR2).
void launch_build_rows(const BuildArgs& b, const StructInfo& st0, bool batch, const Lists& V,
                       const Lists& L, hipStream_t s);
void launch_reverse(int64_t N, const Lists& L, int32_t* err, const int32_t* gate, hipStream_t s);
// Sets bits of *bad when the exact rows break an invariant the evaluation
// kernels rely on for in-bounds access (see neighbor.hip).
void launch_check_rows(int64_t N, const int32_t* sid, const StructInfo* structs, const StructInfo& st0,
                       bool batch, const Lists& L, int32_t* bad, hipStream_t s);
void launch_build_verlet(const BuildArgs& b, const Lists& V, hipStream_t s);
// After a gated re-sort: pos/vel/types/ext <- their permuted copies, pos_ref <- pos
// (and *count += 1 when count is given).
void launch_commit_rebuild(int64_t N, const double* pos2, const double* vel2, const int32_t* types2,
                           const int32_t* ext2, double* pos, double* vel, int32_t* types, int32_t* ext,
                           double* pos_ref, const int32_t* gate, hipStream_t s,
                           double* mu_cum = nullptr, int32_t* count = nullptr);
void launch_filter_rows(const BuildArgs& b, const StructInfo& st0, bool batch, const Lists& V,
                        const Lists& L, hipStream_t s);
// flag = 1 if an atom moved more than allowed since the last build, or will
// have once it moves `horizon` times its current speed further (vel given);
// with mu_cum (box scaling since the build, NPT) the allowance shrinks to
// (mu (r_c + skin) - r_c) / 2 around the scaled reference positions.
void launch_check_displacement(const double* pos, const double* ref, const double* vel, int64_t N,
                               double thr2, double horizon, int32_t* flag, hipStream_t s,
                               const double* mu_cum, double rc, double rl);
void launch_copy_gated_f64(double* dst, const double* src, int64_t n, const int32_t* gate,
                           hipStream_t s);
void launch_copy_gated_i32(int32_t* dst, const int32_t* src, int64_t n, const int32_t* gate,
                           hipStream_t s);
// Species-grouped row order of the network pass; tblk and tex hold
// kMaxTypes * type_row_blocks(N) ints each.
int64_t type_row_blocks(int64_t N);
void launch_type_rows(const int32_t* types, int64_t N, int32_t T, int32_t per_type,
                      int32_t* tblk, int32_t* tex, int32_t* toff, int32_t* rows,
                      int64_t rows_len, const int32_t* gate, hipStream_t s);

// descriptor.hip / force.hip: return false if no kernel exists for (NG, L)
bool launch_descriptor(const EvalArgs& a, hipStream_t s);
bool launch_partial_forces(const EvalArgs& a, hipStream_t s);
void launch_gather_forces(const EvalArgs& a, bool virial, hipStream_t s);
size_t eval_lds_bytes(const DevModel& M, int block);
int angular_group_size(int nA, int L);
std::vector<int> angular_group_options(int nA, int L);

// mlp.hip
void launch_mlp(const EvalArgs& a, hipStream_t s);

// output.hip
void launch_scatter_outputs(const EvalArgs& a, const int32_t* perm, double* energy,
                            double* force, double* virial, hipStream_t s);
void launch_totals(const float* U, const float* W, int64_t N, double* partial, int64_t n_part,
                   double* totals, hipStream_t s);
void launch_struct_totals(const float* U, const float* W, int64_t N, const StructInfo* structs,
                          int32_t n_struct, double* totals, hipStream_t s);
void launch_descriptors_out(const float* q, int64_t N, int NDp, int ND, const int32_t* perm,
                            double* out, hipStream_t s);
void launch_neighbors_out(const Lists& L, int which, int64_t N, const int32_t* perm,
                          const int32_t* inv_perm, const double* pos, const int32_t* sid,
                          const StructInfo* structs, int32_t cap, int32_t* count, int32_t* nbr,
                          int32_t* shift, hipStream_t s);
void launch_inverse_perm(const int32_t* perm, int64_t N, int32_t* inv, hipStream_t s);

// params.hip: model tables of many parameter vectors built on the device.
// Layout of one set's tables (byte offsets) and where each part of the
// parameter vector starts.
struct TableLayout {
  int32_t nets, NN, NNp, ND, NDp32, T, nR, KR, nA, KA;
  int64_t off_b1, off_cR, off_cA;           // in the float64 parameter vector
  int32_t n_ng;                             // admissible angular group sizes
  int32_t ng_of[4], cA_pair_of[4];
  int64_t cA_off_of[4], n_cA;               // floats, per group size and in all
  int64_t at_w0, at_w0t, at_b0, at_w1, at_w0b, at_w0tb, at_cR, at_cA, set_bytes;
};
int64_t table_elements(const TableLayout& L);
void launch_model_tables(const double* params, int64_t npar, int32_t P, const TableLayout& L,
                         unsigned char* base, int64_t set_stride, hipStream_t s);

// output.hip: the fixed workspace of nep_batch_loss_noalloc (one per GPU).
constexpr int64_t kLossScratchBytes = 1 << 20;
constexpr int kMaxDevices = 64;
// Device address of the workspace on `device`, which must be current;
// looked up on the first call per device, then cached.
hipError_t loss_scratch_address(int device, void** out);

// md.hip
struct MDArgs {
  int64_t N;
  double* pos;                // internal [3][N]
  double* vel;                // internal [3][N]
  const float* F;             // internal [3][N]
  const int32_t* types;
  const double* inv_mass;     // [T] 1 / (m * amu(A/fs)^2 in eV)
  double dt;
  // optional skin guard fused into the drift (flag != NULL): *flag = 1 when
  // an atom's new position is more than sqrt(thr2) from ref (with a box
  // scaled by *mu_cum since the build: the bound of k_check_displacement)
  const double* ref = nullptr;
  int32_t* flag = nullptr;
  double thr2 = 0.0;
  const double* mu_cum = nullptr;
  double rc = 0.0, rl = 0.0;
};
void launch_kick_drift(const MDArgs& a, hipStream_t s);
void launch_kick(const MDArgs& a, hipStream_t s);
void launch_thermo(const float* U, const float* W, const double* vel, const int32_t* types,
                   const double* mass, int64_t N, double* partial, int64_t n_part,
                   double* row, double step, double kin_conv, double kB, hipStream_t s);
void launch_thermo_counted(const float* U, const float* W, const double* vel, const int32_t* types,
                           const double* mass, int64_t N, double* partial, int64_t n_part,
                           double* rows, int32_t* counter, double every, double kin_conv, double kB,
                           hipStream_t s);
// *differs = 1 unless the caller's positions and species (caller order) are
// the internal ones (internal atom k is caller atom ext[k]).
void launch_same_state(const int32_t* ext, int64_t N, const double* pos_int, const int32_t* types_int,
                       const double* pos_caller, const int32_t* types_caller, int32_t* differs, hipStream_t s);
void launch_permute_md(const int32_t* perm_old_to_new_src, int64_t N, const double* src_pos,
                       const double* src_vel, double* dst_pos, double* dst_vel, hipStream_t s);
void launch_unpermute_md(const int32_t* perm, int64_t N, const double* pos_int,
                         const double* vel_int, double* pos_ext, double* vel_ext,
                         hipStream_t s);
void launch_check_finite(const double* a, int64_t n, int32_t* flag, hipStream_t s);
void launch_check_types(const int32_t* types, int64_t n, int32_t T, int32_t* flag, hipStream_t s);
void launch_srv_kick_drift(int64_t N, double* pos, double* vel, const double* F, const double* hdm,
                           const double* dta, const uint8_t* move, hipStream_t s);
void launch_srv_kick(int64_t N, double* vel, const double* F, const double* hdm, const uint8_t* move,
                     hipStream_t s);
void launch_fill_u8(uint8_t* a, int64_t n, uint8_t v, hipStream_t s);
// The server's per-atom batch state, [3][ld] for the vectors.
struct SrvState {
  double *pos, *vel, *F, *hdm, *dta;
  int32_t* types;
  uint8_t* move;
  int64_t ld;
};
void launch_srv_place(const int64_t* tab, int32_t n_req, int64_t max_n, const SrvState& o, const SrvState& w,
                      const double* stg, int64_t ns, hipStream_t s);
void launch_srv_collect(const int64_t* tab, int32_t n_req, int64_t max_n, int64_t ld, const double* E,
                        const double* F, const double* W, const double* pos, const double* vel, double* out,
                        hipStream_t s);
void launch_gather3_gated(const int32_t* src, int64_t N, const double* in, double* out,
                          const int32_t* gate, hipStream_t s);
void launch_gather_i32_gated(const int32_t* src, int64_t N, const int32_t* in, int32_t* out,
                             const int32_t* gate, hipStream_t s);
void launch_gather_i32(const int32_t* src, int64_t N, const int32_t* in, int32_t* out, hipStream_t s);

// ensemble.hip: thermostats and barostats (kinds as NEP_ENS_* in nep.h)
constexpr int kEnsNVE = 0, kEnsBerendsen = 1, kEnsBDP = 2, kEnsLangevin = 3, kEnsNHC = 4,
              kEnsNptBerendsen = 5, kEnsNptSCR = 6;
constexpr int kMaxChain = 8;

// Scalar state of an ensemble run, in device memory.
struct EnsState {
  double K;              // kinetic energy of the current velocities (eV)
  double heat;           // energy taken out by thermostat and barostat so far (eV)
  double scale;          // velocity factor of the last thermostat or barostat kernel
  double mu;             // box factor of the last barostat step
  double mu_cum;         // box factor since the last neighbour build
  double P;              // end-of-step pressure (GPa)
  double xi[kMaxChain];  // chain positions
  double vxi[kMaxChain]; // chain velocities (1/fs)
  int64_t step;          // steps done (the step word of the random counters)
  double row[13];        // end-of-step sums: [., E_pot, E_kin, T, W_xx .. W_zz]
};

struct EnsParams {
  int32_t kind, nhc_length;
  double T0, tau_t, P0, tau_p, beta;  // K, fs, GPa, fs, 1/GPa
  double dt, kT, kB, Nf, conv;        // fs, eV, eV/K, 3N - 3, amu (A/fs)^2 in eV
  uint64_t seed;
};

int64_t ens_partials(int64_t N);
void launch_ens_kinetic(const double* vel, const int32_t* types, const double* mass, int64_t N, double conv,
                        double* partial, EnsState* st, hipStream_t s);
void launch_ens_step_begin(EnsState* st, hipStream_t s);
void launch_ens_langevin(double* vel, const int32_t* types, const double* mass, const int32_t* ext,
                         int64_t N, const EnsParams& p, uint32_t stream, EnsState* st, double* partial,
                         hipStream_t s);
// Thermostat after the second half kick (from st->K): scale the velocities.
void launch_ens_thermostat(double* vel, int64_t N, const EnsParams& p, EnsState* st, double* partial,
                           hipStream_t s);
void launch_ens_pressure_row(const EnsParams& p, EnsState* st, const StructInfo* structs, double* rows,
                             int32_t* counter, bool write_row, int64_t step_base, hipStream_t s);
void launch_ens_barostat(double* pos, double* vel, int64_t N, const EnsParams& p, EnsState* st,
                         StructInfo* structs, hipStream_t s);

}  // namespace nep
