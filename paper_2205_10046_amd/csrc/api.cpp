// api.cpp -- host implementation of the C ABI declared in include/nep.h.
//
// Validates arguments, converts the float64 parameter vector into the float32
// / bf16 device tables, owns the device workspaces of a handle, and launches
// the passes:
//   order atoms (cell sort) -> neighbour rows + reverse index -> descriptors
//   -> network (MFMA) -> partial forces -> Newton-3 gather -> outputs
// with velocity-Verlet steps around them for the MD entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "nep.h"
#include "nep_kernels.h"

using namespace nep;

namespace {

thread_local std::string g_thread_error;

constexpr double kPi = 3.14159265358979323846;
// 1 amu (Angstrom/fs)^2 in eV (CODATA 2018 amu and elementary charge)
constexpr double kAmuA2fs2 = 1.66053906660e-27 * 1e10 / 1.602176634e-19;
constexpr double kBoltzmann = 8.617333262e-5;  // eV/K
// Device flags of a handle: [0] radial overflow, [1] angular overflow, [2]
// unpaired reverse entry, [3] species out of range, [4] non-finite position,
// [5] candidate overflow, [6] row invariant broken, [7] rebuild gate, [8] an
// atom left the skin between two rebuild checks of a captured MD group; [9]
// rows rebuilt by the current MD run with a skin.
constexpr int kNumFlags = 16;
constexpr int kFlagGuard = 8;
constexpr int kFlagRebuilds = 9;
constexpr int kFlagsReset = 9;  // flags cleared at the start of an MD chunk
constexpr int kFlagsRead = 10;
constexpr size_t kPinFlags = 3072;  // pinned staging slot of the flags (64 bytes)
static_assert(kFlagsRead * sizeof(int32_t) <= 64 && kPinFlags + 64 <= 4096, "staging slot");
// A captured MD group checks for a rebuild once, at its first step, with
// every atom's displacement extended by this many times its current speed
// over the group's remaining steps; each later step only verifies the skin.
constexpr double kRebuildLookahead = 1.5;

struct Failure {
  int code;
  std::string msg;
};

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw Failure{NEP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};     \
  } while (0)

int n_descriptors(const nep_hparams& h) {
  return (h.n_max_radial + 1) +
         (h.n_max_angular + 1) * (h.l_max_3b + (h.l_max_4b >= 2 ? 1 : 0) + (h.l_max_5b >= 1 ? 1 : 0));
}

size_t n_params(const nep_hparams& h) {
  const size_t nd = n_descriptors(h);
  const size_t nets = h.nn_per_type ? h.n_types : 1;
  const size_t t2 = (size_t)h.n_types * h.n_types;
  return nets * (nd + 2) * h.n_neurons + 1 + t2 * (h.n_max_radial + 1) * (h.basis_radial + 1) +
         t2 * (h.n_max_angular + 1) * (h.basis_angular + 1);
}

bool check_hparams(const nep_hparams* hp, std::string& why) {
  if (!hp) { why = "hparams is NULL"; return false; }
  const nep_hparams& h = *hp;
  if (h.n_types < 1 || h.n_types > kMaxTypes) { why = "n_types must be in [1, 8]"; return false; }
  if (!(h.rc_radial > 0) || !(h.rc_angular > 0) || !(h.rc_angular <= h.rc_radial) ||
      !std::isfinite(h.rc_radial)) {
    why = "need 0 < rc_angular <= rc_radial (finite)";
    return false;
  }
  if (h.n_max_radial < 0 || h.n_max_radial >= kMaxBasis || h.n_max_angular < 0 ||
      h.n_max_angular >= kMaxBasis || h.basis_radial < 0 || h.basis_radial >= kMaxBasis ||
      h.basis_angular < 0 || h.basis_angular >= kMaxBasis) {
    why = "n_max and basis sizes must be in [0, 15]";
    return false;
  }
  if (h.l_max_3b < 1 || h.l_max_3b > kMaxL) { why = "l_max_3b must be in [1, 6]"; return false; }
  if (!(h.l_max_4b == 0 || h.l_max_4b == 2 || h.l_max_4b == 3)) {
    why = "l_max_4b must be 0, 2 or 3";
    return false;
  }
  if (h.l_max_4b >= 2 && h.l_max_3b < 2) { why = "4-body terms need l_max_3b >= 2"; return false; }
  if (!(h.l_max_5b == 0 || h.l_max_5b == 1)) { why = "l_max_5b must be 0 or 1"; return false; }
  if (h.n_neurons < 1 || h.n_neurons > 128) { why = "n_neurons must be in [1, 128]"; return false; }
  if (!(h.nn_per_type == 0 || h.nn_per_type == 1)) { why = "nn_per_type must be 0 or 1"; return false; }
  if (!(h.mlp_precision == NEP_MLP_FP32 || h.mlp_precision == NEP_MLP_BF16)) {
    why = "mlp_precision must be NEP_MLP_FP32 or NEP_MLP_BF16";
    return false;
  }
  if (h.max_nb_radial < 0 || h.max_nb_angular < 0) { why = "negative neighbour capacity"; return false; }
  if (!(h.skin >= 0) || !std::isfinite(h.skin)) { why = "skin must be >= 0"; return false; }
  return true;
}

// ---- angular constants (Sec. II.D) ----
// The library's polynomials for l <= 4 are the paper's b_k; each equals
// alpha_{lm} P_l^{(m)}(z) {Re, Im}(x+iy)^m on the unit sphere.  The addition
// theorem gives C = (2l+1)/(4 pi) (2 - delta_m0) (l-m)!/(l+m)! for the
// unscaled harmonics, hence C^3b = that / alpha^2; l = 5, 6 use alpha = 1.
// C^4b and C^5b are the printed S-form coefficients.
void angular_constants(int L, double* C3, double* C4, double* C5) {
  static const double alpha[5][5] = {
      {0, 0, 0, 0, 0},
      {1.0, 1.0, 0, 0, 0},
      {2.0, 1.0 / 3.0, 1.0 / 3.0, 0, 0},
      {2.0, 2.0 / 3.0, 1.0 / 15.0, 1.0 / 15.0, 0},
      {8.0, 2.0 / 5.0, 2.0 / 15.0, 1.0 / 105.0, 1.0 / 105.0}};
  auto fact = [](int n) {
    double f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  for (int l = 1; l <= L; ++l) {
    int k = l * l - 1;
    for (int m = 0; m <= l; ++m) {
      double c = (2 * l + 1) / (4 * kPi) * (m ? 2.0 : 1.0) * fact(l - m) / fact(l + m);
      if (l <= 4) c /= alpha[l][m] * alpha[l][m];
      C3[k++] = c;
      if (m) C3[k++] = c;
    }
  }
  const double y20 = 0.25 * std::sqrt(5 / kPi), y21 = 0.5 * std::sqrt(15 / (2 * kPi)),
               y22 = 0.25 * std::sqrt(15 / (2 * kPi));
  C4[0] = -std::sqrt(2.0 / 35) * y20 * y20 * y20;
  C4[1] = -6 * std::sqrt(1.0 / 70) * y20 * y21 * y21;
  C4[2] = 6 * std::sqrt(2.0 / 35) * y20 * y22 * y22;
  C4[3] = 6 * std::sqrt(3.0 / 35) * y21 * y21 * y22;
  C4[4] = -12 * std::sqrt(3.0 / 35) * y21 * y21 * y22;
  C5[0] = 21 / (80 * kPi * kPi);
  C5[1] = 21 / (40 * kPi * kPi);
  C5[2] = 21 / (80 * kPi * kPi);
}

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);                                    // round to nearest even
  return (uint16_t)(u >> 16);
}

// Bumped by every device (re)allocation: a captured HIP graph holds buffer
// addresses in its kernel arguments and is only reused while none of them
// can have moved.
std::atomic<uint64_t> g_alloc_gen{1};

template <class T>
void dev_alloc(T*& p, size_t n) {
  if (p) HIPCHK(hipFree(p));
  p = nullptr;
  g_alloc_gen.fetch_add(1);
  if (n == 0) return;
  hipError_t e = hipMalloc((void**)&p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    throw Failure{NEP_E_OOM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed"};
  }
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

struct Geometry {
  StructInfo st;
  int32_t n_cells;
  double volume;
};

// Cell inverse, face widths and the neighbour-search mode of one structure.
Geometry make_geometry(const double* box, const int32_t* pbc, int64_t n_atoms, double r_list) {
  Geometry g{};
  StructInfo& st = g.st;
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(box[k])) throw Failure{NEP_E_BOX, "box has a non-finite entry"};
    st.H[k] = box[k];
  }
  const double a = box[0], b = box[1], c = box[2], d = box[3], e = box[4], f = box[5], gg = box[6],
               hh = box[7], kk = box[8];
  const double det = a * (e * kk - f * hh) - b * (d * kk - f * gg) + c * (d * hh - e * gg);
  if (!(det > 0)) throw Failure{NEP_E_BOX, "det(box) must be positive"};
  st.Hi[0] = (e * kk - f * hh) / det;
  st.Hi[1] = (c * hh - b * kk) / det;
  st.Hi[2] = (b * f - c * e) / det;
  st.Hi[3] = (f * gg - d * kk) / det;
  st.Hi[4] = (a * kk - c * gg) / det;
  st.Hi[5] = (c * d - a * f) / det;
  st.Hi[6] = (d * hh - e * gg) / det;
  st.Hi[7] = (b * gg - a * hh) / det;
  st.Hi[8] = (a * e - b * d) / det;
  st.ortho = (box[1] == 0.0 && box[2] == 0.0 && box[3] == 0.0 && box[5] == 0.0 && box[6] == 0.0 &&
              box[7] == 0.0) ? 1 : 0;
  g.volume = det;
  // face width along cell vector k = volume / |(other two) cross product|
  double w[3];
  for (int k = 0; k < 3; ++k) {
    const double* u = box + 3 * ((k + 1) % 3);
    const double* v = box + 3 * ((k + 2) % 3);
    const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
                 cz = u[0] * v[1] - u[1] * v[0];
    w[k] = det / std::sqrt(cx * cx + cy * cy + cz * cz);
  }
  bool min_image_ok = true;
  for (int k = 0; k < 3; ++k) {
    st.pbc[k] = pbc ? (pbc[k] != 0) : 1;
    if (st.pbc[k] && !(w[k] > 2.0 * r_list * (1.0 + 1e-9))) min_image_ok = false;
  }
  st.start = 0;
  st.count = n_atoms;
  st.cell_off = 0;
  if (min_image_ok) {
    int32_t nc[3];
    int64_t total = 1;
    for (int k = 0; k < 3; ++k) {
      nc[k] = std::max(1, (int)std::floor(w[k] / (r_list * (1.0 + 1e-9))));
      nc[k] = std::min(nc[k], 1024);
      total *= nc[k];
    }
    if (n_atoms > 256 && total > 1 && total < (1 << 28)) {
      st.mode = kModeCells;
      for (int k = 0; k < 3; ++k) st.ncell[k] = nc[k];
      g.n_cells = (int32_t)total;
    } else {
      st.mode = kModeAllPairs;
      st.ncell[0] = st.ncell[1] = st.ncell[2] = 1;
      g.n_cells = 1;
    }
  } else {
    st.mode = kModeImages;
    for (int k = 0; k < 3; ++k) {
      st.reach[k] = st.pbc[k] ? (int)std::floor(r_list / w[k] + 0.5) + 1 : 0;
      if (st.reach[k] > 7)
        throw Failure{NEP_E_BOX, "cell too thin: a face width is below r_c / 6.5; replicate it"};
    }
    st.ncell[0] = st.ncell[1] = st.ncell[2] = 1;
    g.n_cells = 1;
  }
  return g;
}

struct StageTimes {
  std::vector<const char*> names;
  std::vector<double> ms;
  std::vector<int64_t> calls;
  void add(const char* n, double t) {
    for (size_t k = 0; k < names.size(); ++k)
      if (names[k] == n || std::strcmp(names[k], n) == 0) {
        ms[k] += t;
        calls[k] += 1;
        return;
      }
    names.push_back(n);
    ms.push_back(t);
    calls.push_back(1);
  }
};

// Device tables of one parameter vector (float32 / bf16 copies).
struct ModelTables {
  DevModel M{};
  float *cR = nullptr, *cA = nullptr, *w0 = nullptr, *w0t = nullptr, *b0 = nullptr, *w1 = nullptr;
  uint16_t *w0b = nullptr, *w0tb = nullptr;
  void release() {
    dev_free(cR); dev_free(cA); dev_free(w0); dev_free(w0t); dev_free(b0); dev_free(w1);
    dev_free(w0b); dev_free(w0tb);
  }
};

// Kernel shape picked for one problem shape (see autotune()).
struct Tuning {
  bool done = false;
  int NG_desc = 0, NG_force = 0, block_desc = 256, block_force = 256;
  int lanes_desc = 1, lanes_force = 1;   // lanes per atom of the pair kernels
  int lanes_gather = 1;                  // lanes per atom of the force gather
};

}  // namespace

struct nep_handle {
  nep_hparams hp{};
  int device = 0;
  std::string err;
  int nd = 0, nets = 1;
  Tuning tune[2];                   // [single structure, batch]
  ModelTables main;                 // the handle's own parameter vector
  std::vector<ModelTables> pop;     // parameter sets of the last batch call
  unsigned char* pop_tables = nullptr;  // device-built tables of a device population
  int64_t pop_tables_cap = 0;
  // the captured per-set passes of the last batch call, reused while the
  // shapes, buffers and output pointers stay the same
  hipGraph_t batch_graph = nullptr;
  hipGraphExec_t batch_exec = nullptr;
  std::vector<unsigned char> batch_key;
  // rows of the last batch call, for callers that pass the same structures
  bool batch_rows_ready = false;
  int32_t batch_S = 0;
  int64_t batch_N = 0;
  std::vector<StructInfo> batch_sts;
  int32_t batch_cells = 0;
  int64_t* offs = nullptr;          // structure offsets of a batch (device)
  int32_t cap_struct = 0;
  // training-loss workspace (grown on demand, kept until the handle ends)
  double* loss_part = nullptr;
  int64_t* loss_offs = nullptr;
  std::vector<int64_t> loss_offs_host;  // the offsets loss_offs holds
  int64_t loss_part_cap = 0, loss_offs_cap = 0;
  double* snes_util = nullptr;     // [1024] SNES utilities of the last step
  double* heat_part = nullptr;     // per-block heat-current sums
  int64_t heat_part_cap = 0;
  void* scratch = nullptr;         // this device's fixed workspace of nep_batch_loss_noalloc
  // the captured G-step MD graph, reused by later nep_md_run* calls whose
  // shapes, geometry, step and buffers (allocation generation) are the same
  hipGraph_t md_graph = nullptr;
  hipGraphExec_t md_exec = nullptr;
  std::vector<unsigned char> md_key;
  hipStream_t md_stream = nullptr;  // capture/replay stream for null-stream callers
  double* ens_state = nullptr;      // ensemble state, its chunk save and the saved cell
  double* ens_partial = nullptr;    // ensemble reduction partials
  int64_t ens_partial_cap = 0;
  DevModel& M = main.M;
  // workspace
  int64_t capN = 0, cap_part = 0, rows_cap = 0;
  int32_t MR = 0, MA = 0, cap_cells = 0;
  double *pos_ext = nullptr, *pos = nullptr, *pos2 = nullptr, *vel = nullptr, *vel2 = nullptr;
  double *vel_ext = nullptr, *out_e = nullptr, *out_f = nullptr, *out_w = nullptr;
  double *partial = nullptr, *totals = nullptr, *thermo = nullptr, *mass = nullptr, *inv_mass = nullptr;
  int64_t thermo_cap = 0;
  int32_t *types_ext = nullptr, *types = nullptr, *types2 = nullptr, *sid_ext = nullptr, *sid = nullptr;
  int32_t *key = nullptr, *perm = nullptr, *ext_id = nullptr, *ext_id2 = nullptr, *inv = nullptr;
  int32_t *cell_count = nullptr, *cell_fill = nullptr, *cell_start = nullptr;
  int32_t *rows = nullptr, *tblk = nullptr, *tex = nullptr, *toff = nullptr, *flags = nullptr;
  StructInfo* structs = nullptr;
  Lists L{};
  Lists V{};                       // candidate rows at r_c^R + skin (MD with a skin)
  double* pos_ref = nullptr;       // positions at the last candidate-row build
  int32_t* row_counter = nullptr;  // thermo row of graph-replayed MD steps
  double* ref_save = nullptr;
  float *q = nullptr, *fp = nullptr, *U = nullptr, *sums = nullptr;
  float4* P = nullptr;
  float *F = nullptr, *W = nullptr, *F_save = nullptr;
  double *pos_save = nullptr, *vel_save = nullptr;
  int32_t *types_save = nullptr, *ext_save = nullptr;
  // pinned host staging for small stream-ordered copies:
  // [0, 256) structure table, [256, 384) masses, [384, 416) flags
  unsigned char* pinned = nullptr;
  // structure tables of batch calls: pinned staging for an asynchronous
  // upload, rewritten only after the previous upload (tab_event) has read it
  unsigned char* pinned_tab = nullptr;
  size_t pinned_tab_cap = 0;
  hipEvent_t tab_event = nullptr;
  // timing
  bool timing = false;
  int64_t md_group_steps = 0;  // MD steps run in captured groups (one rebuild check each)
  int64_t md_replays = 0;      // MD chunks replayed because an atom left the skin mid-group
  int64_t md_rebuilds = 0;     // row rebuilds of MD runs with a skin
  // continuation of an MD run: after a run with a skin ends, its internal
  // state (order, rows, forces) is reused by the next run if no other call
  // came in between, the geometry and buffers are the same and the caller's
  // positions and species are those the run returned
  std::atomic<uint64_t> api_calls{0};  // also counted by a server's worker
  uint64_t md_cont_call = 0;   // api_calls at the end of the run that left the state
  std::vector<unsigned char> md_cont_key;
  int64_t md_continued = 0;    // runs that reused the previous run's state
  StageTimes times;
  std::vector<std::pair<const char*, std::pair<hipEvent_t, hipEvent_t>>> pending;

  ~nep_handle() { release(); }

  void drop_batch_graph() {
    if (batch_exec) (void)hipGraphExecDestroy(batch_exec);
    if (batch_graph) (void)hipGraphDestroy(batch_graph);
    batch_exec = nullptr;
    batch_graph = nullptr;
    batch_key.clear();
  }

  void drop_md_graph() {
    if (md_exec) (void)hipGraphExecDestroy(md_exec);
    if (md_graph) (void)hipGraphDestroy(md_graph);
    md_exec = nullptr;
    md_graph = nullptr;
    md_key.clear();
  }

  void release() {
    drop_md_graph();
    drop_batch_graph();
    dev_free(pop_tables);
    pop_tables_cap = 0;
    if (md_stream) (void)hipStreamDestroy(md_stream);
    md_stream = nullptr;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    if (tab_event) (void)hipEventSynchronize(tab_event);
    if (pinned_tab) (void)hipHostFree(pinned_tab);
    pinned_tab = nullptr;
    pinned_tab_cap = 0;
    if (tab_event) (void)hipEventDestroy(tab_event);
    tab_event = nullptr;
    dev_free(loss_part); dev_free(loss_offs); dev_free(snes_util); dev_free(heat_part);
    dev_free(ens_state); dev_free(ens_partial);
    ens_partial_cap = 0;
    heat_part_cap = 0;
    loss_part_cap = loss_offs_cap = 0;
    main.release();
    for (auto& t : pop) t.release();
    pop.clear();
    free_workspace();
    for (auto& p : pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    pending.clear();
  }

  void free_workspace() {
    dev_free(pos_ext); dev_free(pos); dev_free(pos2); dev_free(vel); dev_free(vel2);
    dev_free(vel_ext); dev_free(out_e); dev_free(out_f); dev_free(out_w);
    dev_free(partial); dev_free(totals); dev_free(thermo); dev_free(mass); dev_free(inv_mass);
    dev_free(types_ext); dev_free(types); dev_free(types2); dev_free(sid_ext); dev_free(sid);
    dev_free(key); dev_free(perm); dev_free(ext_id); dev_free(ext_id2); dev_free(inv);
    dev_free(cell_count); dev_free(cell_fill); dev_free(cell_start);
    dev_free(rows); dev_free(tblk); dev_free(tex); dev_free(toff); dev_free(flags);
    dev_free(structs); dev_free(offs);
    cap_struct = 0;
    free_lists();
    dev_free(q); dev_free(fp); dev_free(U); dev_free(sums); dev_free(F); dev_free(W);
    dev_free(F_save); dev_free(pos_save); dev_free(vel_save); dev_free(types_save);
    dev_free(ext_save); dev_free(pos_ref); dev_free(ref_save); dev_free(row_counter);
    free_verlet();
    capN = 0; cap_cells = 0; thermo_cap = 0; MR = MA = 0;
  }

  void free_verlet() {
    dev_free(V.nnR); dev_free(V.nlR); dev_free(V.cdR); dev_free(V.nnA);
    dev_free(V.revR); dev_free(V.fmap);
    V = Lists{};
  }

  void free_lists() {
    dev_free(L.nnR); dev_free(L.nlR); dev_free(L.cdR); dev_free(L.revR);
    dev_free(L.nnA);
    dev_free(P);
  }

  // ---- timing helpers ----
  void stage_begin(hipStream_t s, hipEvent_t& a) {
    a = nullptr;
    if (!timing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventRecord(a, s) != hipSuccess) a = nullptr;
  }
  void stage_end(const char* name, hipStream_t s, hipEvent_t a) noexcept {
    if (!timing || !a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    pending.push_back({name, {a, b}});
  }
  void drop_timing() noexcept {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    pending.clear();
  }
  void resolve_timing() {
    for (auto& p : pending) {
      float ms = 0;
      HIPCHK(hipEventSynchronize(p.second.second));
      HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
      times.add(p.first, ms);
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    pending.clear();
  }
};

namespace {

struct Stage {
  nep_handle* h;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Stage(nep_handle* h_, const char* n, hipStream_t s_) : h(h_), name(n), s(s_) { h->stage_begin(s, a); }
  ~Stage() { h->stage_end(name, s, a); }
};

void upload_model(nep_handle* h, const double* p, ModelTables& mt) {
  const nep_hparams& hp = h->hp;
  const int T = hp.n_types, nd = h->nd, NN = hp.n_neurons, nets = h->nets;
  const int nR = hp.n_max_radial + 1, KR = hp.basis_radial + 1;
  const int nA = hp.n_max_angular + 1, KA = hp.basis_angular + 1;
  const int NNp = (NN + 31) / 32 * 32;
  const int NDp32 = (nd + 31) / 32 * 32;
  for (size_t k = 0; k < n_params(hp); ++k)
    if (!std::isfinite(p[k])) throw Failure{NEP_E_INVALID_ARG, "parameter vector has a non-finite entry"};
  std::vector<float> w0((size_t)nets * NNp * nd, 0.f), w0t((size_t)nets * nd * NNp, 0.f);
  std::vector<float> b0((size_t)nets * NNp + 1, 0.f), w1((size_t)nets * NNp, 0.f);
  std::vector<uint16_t> w0b((size_t)nets * NNp * NDp32, 0), w0tb((size_t)nets * NDp32 * NNp, 0);
  size_t off = 0;
  for (int t = 0; t < nets; ++t) {
    for (int mu = 0; mu < NN; ++mu)
      for (int v = 0; v < nd; ++v) {
        const float x = (float)p[off + (size_t)mu * nd + v];
        w0[((size_t)t * NNp + mu) * nd + v] = x;
        w0t[((size_t)t * nd + v) * NNp + mu] = x;
        w0b[((size_t)t * NNp + mu) * NDp32 + v] = to_bf16(x);
        w0tb[((size_t)t * NDp32 + v) * NNp + mu] = to_bf16(x);
      }
    off += (size_t)NN * nd;
    for (int mu = 0; mu < NN; ++mu) b0[(size_t)t * NNp + mu] = (float)p[off + mu];
    off += NN;
    for (int mu = 0; mu < NN; ++mu) w1[(size_t)t * NNp + mu] = (float)p[off + mu];
    off += NN;
  }
  const float b1 = (float)p[off++];
  b0[(size_t)nets * NNp] = b1;  // b1 rides at the end of the b0 table
  std::vector<float> cR((size_t)T * T * nR * KR);
  for (size_t k = 0; k < cR.size(); ++k) cR[k] = (float)p[off + k];
  off += cR.size();
  // one angular table per admissible group size NG: [T][T][groups][KA][ng_pad(NG)]
  std::vector<float> cA;
  int32_t cA_off[8];
  int32_t cA_max = 0;
  for (int ng = 0; ng < 8; ++ng) cA_off[ng] = -1;
  int32_t cA_pair[8];
  for (int ng = 0; ng < 8; ++ng) cA_pair[ng] = 0;
  for (int ng : angular_group_options(nA, hp.l_max_3b)) {
    const int groups = (nA + ng - 1) / ng, w = ng_pad(ng);
    const int ps = pair_stride(groups * KA * w);
    const size_t base = cA.size();
    cA_off[ng] = (int32_t)base;
    cA_pair[ng] = ps;
    cA.resize(base + (size_t)T * T * ps, 0.f);
    for (int a = 0; a < T * T; ++a)
      for (int n = 0; n < nA; ++n)
        for (int k = 0; k < KA; ++k)
          cA[base + (size_t)a * ps + ((size_t)(n / ng) * KA + k) * w + n % ng] =
              (float)p[off + ((size_t)a * nA + n) * KA + k];
    cA_max = std::max(cA_max, (int32_t)(cA.size() - base));
  }
  off += (size_t)T * T * nA * KA;

  auto put = [](auto*& dst, const auto& v) {
    using E = std::remove_reference_t<decltype(*dst)>;
    dev_alloc(dst, v.size());
    HIPCHK(hipMemcpy(dst, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice));
  };
  put(mt.w0, w0); put(mt.w0t, w0t); put(mt.b0, b0); put(mt.w1, w1);
  put(mt.w0b, w0b); put(mt.w0tb, w0tb); put(mt.cR, cR); put(mt.cA, cA);

  DevModel& M = mt.M;
  M.T = T; M.nR = nR; M.KR = KR; M.nA = nA; M.KA = KA; M.L = hp.l_max_3b;
  M.NB = (hp.l_max_3b + 1) * (hp.l_max_3b + 1) - 1;
  M.ND = nd; M.NDp = (nd + 7) / 8 * 8; M.NN = NN; M.nets = nets;
  M.has4b = hp.l_max_4b >= 2; M.has5b = hp.l_max_5b >= 1; M.cA_max = cA_max;
  for (int ng = 0; ng < 8; ++ng) {
    M.cA_off[ng] = cA_off[ng];
    M.cA_pair[ng] = cA_pair[ng];
  }
  M.rcR = (float)hp.rc_radial; M.rcA = (float)hp.rc_angular; M.b1 = mt.b0 + (size_t)nets * NNp;
  M.cR = mt.cR; M.cA = mt.cA; M.NNp = NNp; M.NDp32 = NDp32;
  M.w0 = mt.w0; M.w0t = mt.w0t; M.b0 = mt.b0; M.w1 = mt.w1; M.w0b = mt.w0b; M.w0tb = mt.w0tb;
  double C3[kMaxNB] = {0}, C4[5], C5[3];
  angular_constants(hp.l_max_3b, C3, C4, C5);
  for (int k = 0; k < kMaxNB; ++k) M.C3[k] = (float)C3[k];
  for (int k = 0; k < 5; ++k) M.C4[k] = (float)C4[k];
  for (int k = 0; k < 3; ++k) M.C5[k] = (float)C5[k];
}

// Layout of the device-built tables of one parameter set (the same tables
// upload_model builds on the host).
TableLayout table_layout(const nep_hparams& hp, int nd) {
  TableLayout L{};
  L.nets = hp.nn_per_type ? hp.n_types : 1;
  L.NN = hp.n_neurons;
  L.NNp = (L.NN + 31) / 32 * 32;
  L.ND = nd;
  L.NDp32 = (nd + 31) / 32 * 32;
  L.T = hp.n_types;
  L.nR = hp.n_max_radial + 1;
  L.KR = hp.basis_radial + 1;
  L.nA = hp.n_max_angular + 1;
  L.KA = hp.basis_angular + 1;
  L.off_b1 = (int64_t)L.nets * (nd + 2) * L.NN;
  L.off_cR = L.off_b1 + 1;
  L.off_cA = L.off_cR + (int64_t)L.T * L.T * L.nR * L.KR;
  L.n_ng = 0;
  int64_t cA = 0;
  for (int ng : angular_group_options(L.nA, hp.l_max_3b)) {
    const int ps = pair_stride((L.nA + ng - 1) / ng * L.KA * ng_pad(ng));
    L.ng_of[L.n_ng] = ng;
    L.cA_pair_of[L.n_ng] = ps;
    L.cA_off_of[L.n_ng] = cA;
    cA += (int64_t)L.T * L.T * ps;
    ++L.n_ng;
  }
  L.n_cA = cA;
  auto take = [](int64_t& at, int64_t bytes) {
    const int64_t o = at;
    at += (bytes + 255) / 256 * 256;
    return o;
  };
  int64_t at = 0;
  L.at_w0 = take(at, (int64_t)L.nets * L.NNp * L.ND * 4);
  L.at_w0t = take(at, (int64_t)L.nets * L.ND * L.NNp * 4);
  L.at_b0 = take(at, ((int64_t)L.nets * L.NNp + 1) * 4);
  L.at_w1 = take(at, (int64_t)L.nets * L.NNp * 4);
  L.at_w0b = take(at, (int64_t)L.nets * L.NNp * L.NDp32 * 2);
  L.at_w0tb = take(at, (int64_t)L.nets * L.NDp32 * L.NNp * 2);
  L.at_cR = take(at, (int64_t)L.T * L.T * L.nR * L.KR * 4);
  L.at_cA = take(at, L.n_cA * 4);
  L.set_bytes = at;
  return L;
}

// The DevModel of tables at `base` laid out by L (scalars from the handle's).
DevModel model_at(const DevModel& proto, const TableLayout& L, const unsigned char* base) {
  DevModel M = proto;
  M.w0 = (const float*)(base + L.at_w0);
  M.w0t = (const float*)(base + L.at_w0t);
  M.b0 = (const float*)(base + L.at_b0);
  M.b1 = M.b0 + (size_t)L.nets * L.NNp;
  M.w1 = (const float*)(base + L.at_w1);
  M.w0b = (const uint16_t*)(base + L.at_w0b);
  M.w0tb = (const uint16_t*)(base + L.at_w0tb);
  M.cR = (const float*)(base + L.at_cR);
  M.cA = (const float*)(base + L.at_cA);
  for (int ng = 0; ng < 8; ++ng) {
    M.cA_off[ng] = -1;
    M.cA_pair[ng] = 0;
  }
  int32_t cA_max = 0;
  for (int o = 0; o < L.n_ng; ++o) {
    M.cA_off[L.ng_of[o]] = (int32_t)L.cA_off_of[o];
    M.cA_pair[L.ng_of[o]] = L.cA_pair_of[o];
    cA_max = std::max(cA_max, L.T * L.T * L.cA_pair_of[o]);
  }
  M.cA_max = cA_max;
  return M;
}

// Length of the species-grouped row order: every species segment is padded
// to whole groups of kRowGroup rows, so it never exceeds round(N) + kRowGroup T.
int64_t rows_length(int64_t N, int T) {
  return (N + kRowGroup - 1) / kRowGroup * kRowGroup + kRowGroup * (int64_t)T;
}

int64_t num_partials(int64_t N) { return std::min<int64_t>(512, std::max<int64_t>(1, (N + 1023) / 1024)); }

int32_t estimate_capacity(double rc, double density) {
  const double expect = 4.0 / 3.0 * kPi * rc * rc * rc * density;
  int32_t m = (int32_t)std::ceil(1.3 * expect + 24);
  return (m + 3) / 4 * 4;
}

void ensure_lists(nep_handle* h, int64_t N, int32_t MR, int32_t MA) {
  if (N <= h->capN && MR <= h->MR && MA <= h->MA && h->L.nlR) return;
  if (MR > kMaxRow || MA > kMaxRow)
    throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "neighbour rows longer than 65535 entries"};
  h->free_lists();
  const int64_t cap = std::max(N, h->capN);
  dev_alloc(h->L.nnR, cap); dev_alloc(h->L.nnA, cap);
  dev_alloc(h->L.nlR, (size_t)MR * cap); dev_alloc(h->L.cdR, (size_t)MR * cap);
  dev_alloc(h->L.revR, (size_t)MR * cap);
  dev_alloc(h->P, (size_t)MR * cap);
  h->MR = MR;
  h->MA = MA;
  h->L.MR = MR;
  // the angular row lives in the radial row; its length is only capped when
  // the caller fixed max_nb_angular
  h->L.MA = h->hp.max_nb_angular ? MA : kMaxRow;
}

// Candidate rows V of MV slots per atom (contents are not preserved).
void ensure_verlet(nep_handle* h, int64_t N, int32_t MV) {
  if (h->V.nlR && MV <= h->V.MR && N <= h->capN) return;
  if (MV > kMaxRow) throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "candidate rows longer than 65535 entries"};
  h->free_verlet();
  const int64_t cap = h->capN;
  dev_alloc(h->V.nnR, cap);
  dev_alloc(h->V.nnA, cap);
  dev_alloc(h->V.nlR, (size_t)MV * cap);
  dev_alloc(h->V.cdR, (size_t)MV * cap);
  dev_alloc(h->V.revR, (size_t)MV * cap);
  dev_alloc(h->V.fmap, (size_t)MV * cap);
  h->V.MR = MV;
  h->V.MA = 0;
  if (!h->pos_ref) {
    dev_alloc(h->pos_ref, 3 * cap);
    dev_alloc(h->ref_save, 3 * cap);
  }
}

// Per-atom buffers sized for N atoms (contents are not preserved).
void ensure_atoms(nep_handle* h, int64_t N, int32_t n_cells, bool md) {
  const DevModel& M = h->M;
  if (N > h->capN) {
    const int32_t MR = h->MR, MA = h->MA;
    h->free_workspace();
    const int64_t c = N;
    dev_alloc(h->pos_ext, 3 * c); dev_alloc(h->pos, 3 * c);
    dev_alloc(h->types_ext, c); dev_alloc(h->types, c); dev_alloc(h->sid_ext, c); dev_alloc(h->sid, c);
    dev_alloc(h->key, c); dev_alloc(h->perm, c); dev_alloc(h->inv, c);
    dev_alloc(h->out_e, c); dev_alloc(h->out_f, 3 * c); dev_alloc(h->out_w, 9 * c);
    dev_alloc(h->q, (size_t)c * M.NDp); dev_alloc(h->fp, (size_t)c * M.NDp);
    dev_alloc(h->U, c); dev_alloc(h->sums, (size_t)M.nA * M.NB * c);
    dev_alloc(h->F, 3 * c); dev_alloc(h->W, 9 * c);
    h->rows_cap = rows_length(c, M.T);
    dev_alloc(h->rows, h->rows_cap);
    dev_alloc(h->tblk, kMaxTypes * type_row_blocks(c)); dev_alloc(h->tex, kMaxTypes * type_row_blocks(c));
    dev_alloc(h->toff, kMaxTypes + 1); dev_alloc(h->flags, kNumFlags);
    HIPCHK(hipMemset(h->flags, 0, kNumFlags * sizeof(int32_t)));
    h->cap_part = num_partials(c);
    dev_alloc(h->partial, 11 * h->cap_part); dev_alloc(h->totals, 16);
    dev_alloc(h->structs, 1);
    h->capN = c;
    h->MR = MR;
    h->MA = MA;
  }
  if (n_cells > h->cap_cells) {
    dev_alloc(h->cell_count, n_cells); dev_alloc(h->cell_fill, n_cells);
    dev_alloc(h->cell_start, n_cells);
    h->cap_cells = n_cells;
  }
  if (md && !h->vel) {
    const int64_t c = h->capN;
    dev_alloc(h->pos2, 3 * c); dev_alloc(h->vel, 3 * c); dev_alloc(h->vel2, 3 * c);
    dev_alloc(h->vel_ext, 3 * c); dev_alloc(h->types2, c); dev_alloc(h->ext_id, c);
    dev_alloc(h->ext_id2, c); dev_alloc(h->F_save, 3 * c); dev_alloc(h->pos_save, 3 * c);
    dev_alloc(h->vel_save, 3 * c); dev_alloc(h->types_save, c); dev_alloc(h->ext_save, c);
    dev_alloc(h->mass, kMaxTypes); dev_alloc(h->inv_mass, kMaxTypes);
  }
}

struct Prepared {
  std::vector<StructInfo> sts;   // one per structure; start/count in internal order
  Geometry geo;                  // of structure 0 (the single-structure kernels)
  int32_t n_cells = 0;
  int64_t N = 0;
  bool batch = false;
};

BuildArgs build_args(nep_handle* h, const Prepared& pp, const double* pos_src, const int32_t* types_src,
                     double* pos_dst, int32_t* types_dst) {
  BuildArgs b{};
  b.N = pp.N;
  b.n_cells = pp.n_cells;
  b.pos_ext = pos_src;
  b.types_ext = types_src;
  b.sid_ext = h->sid_ext;
  b.structs = h->structs;
  b.key = h->key;
  b.cell_count = h->cell_count;
  b.cell_fill = h->cell_fill;
  b.cell_start = h->cell_start;
  b.perm = h->perm;
  b.pos = pos_dst;
  b.types = types_dst;
  b.sid = h->sid;
  b.rcR2 = h->hp.rc_radial * h->hp.rc_radial;
  b.rcA2 = h->hp.rc_angular * h->hp.rc_angular;
  b.overflow = h->flags;
  b.wide_rows = 0;
  for (const StructInfo& st : pp.sts)
    if (st.mode != kModeCells) b.wide_rows = 1;
  return b;
}

EvalArgs eval_args(nep_handle* h, const Prepared& pp, const DevModel& M) {
  EvalArgs a{};
  a.pos = h->pos;
  a.N = pp.N;
  a.types = h->types;
  a.sid = h->sid;
  a.structs = h->structs;
  a.L = h->L;
  a.M = M;
  a.q = h->q;
  a.fp = h->fp;
  a.U = h->U;
  a.sums = h->sums;
  a.P = h->P;
  a.F = h->F;
  a.W = h->W;
  a.rows = h->rows;
  a.rows_len = rows_length(pp.N, M.T);
  a.mlp_bf16 = h->hp.mlp_precision == NEP_MLP_BF16;
  a.batch = pp.batch ? 1 : 0;
  a.st0 = pp.geo.st;
  return a;
}

// Geometry, buffers and the structure table for structures s = 0..S-1 holding
// atoms [offs[s], offs[s+1]) (S = 1: one structure of N atoms).
Prepared prepare_batch(nep_handle* h, int32_t S, const int64_t* offs, const double* boxes,
                       const int32_t* pbcs, double r_list, bool md, bool force_batch, hipStream_t s) {
  if (S < 1) throw Failure{NEP_E_INVALID_ARG, "n_struct must be >= 1"};
  h->batch_rows_ready = false;  // the rows are about to belong to other structures
  const int64_t N = offs ? offs[S] : 0;
  if (N < 1 || N > (int64_t)1 << 30) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be in [1, 2^30]"};
  Prepared pp;
  pp.N = N;
  pp.sts.resize(S);
  double max_density = 0;
  int32_t cells = 0;
  for (int32_t k = 0; k < S; ++k) {
    const int64_t n = offs[k + 1] - offs[k];
    if (n < 1) throw Failure{NEP_E_INVALID_ARG, "every structure needs at least one atom"};
    Geometry g = make_geometry(boxes + 9 * k, pbcs ? pbcs + 3 * k : nullptr, n, r_list);
    g.st.start = offs[k];
    g.st.count = n;
    g.st.cell_off = cells;
    if ((int64_t)cells + g.n_cells > (1 << 30)) throw Failure{NEP_E_INVALID_ARG, "too many cells"};
    cells += g.n_cells;
    max_density = std::max(max_density, (double)n / g.volume);
    pp.sts[k] = g.st;
    if (k == 0) pp.geo = g;
  }
  pp.n_cells = cells;
  pp.batch = force_batch || S > 1;
  ensure_atoms(h, N, cells, md);
  int32_t MR = h->hp.max_nb_radial ? h->hp.max_nb_radial : estimate_capacity(h->hp.rc_radial, max_density);
  int32_t MA = h->hp.max_nb_angular ? h->hp.max_nb_angular : estimate_capacity(h->hp.rc_angular, max_density);
  MR = std::max(MR, h->MR);
  MA = std::max(MA, h->MA);
  ensure_lists(h, N, MR, MA);
  // candidate rows at r_list (= r_c^R, or r_c^R + skin)
  const int32_t MV = r_list > h->hp.rc_radial ? estimate_capacity(r_list, max_density) : MR;
  ensure_verlet(h, N, std::max(MV, h->V.MR));
  if (S > h->cap_struct) {
    dev_alloc(h->structs, S);
    dev_alloc(h->offs, S + 1);
    h->cap_struct = S;
  }
  if (S == 1) {
    static_assert(sizeof(StructInfo) <= 256, "staging slot");
    std::memcpy(h->pinned, &pp.sts[0], sizeof(StructInfo));
    HIPCHK(hipMemcpyAsync(h->structs, h->pinned, sizeof(StructInfo), hipMemcpyHostToDevice, s));
    launch_fill_i32(h->sid_ext, N, 0, s);
  } else {
    // the structure table and offsets go up from pinned staging in stream order
    const size_t nb = (size_t)S * sizeof(StructInfo), need = nb + (size_t)(S + 1) * sizeof(int64_t);
    if (h->tab_event) HIPCHK(hipEventSynchronize(h->tab_event));  // the last upload has read it
    if (need > h->pinned_tab_cap) {
      if (h->pinned_tab) HIPCHK(hipHostFree(h->pinned_tab));
      h->pinned_tab = nullptr;
      h->pinned_tab_cap = 0;
      const size_t cap = std::max<size_t>(need + need / 2, 1 << 14);
      HIPCHK(hipHostMalloc((void**)&h->pinned_tab, cap, hipHostMallocDefault));
      h->pinned_tab_cap = cap;
    }
    std::memcpy(h->pinned_tab, pp.sts.data(), nb);
    std::memcpy(h->pinned_tab + nb, offs, (size_t)(S + 1) * sizeof(int64_t));
    HIPCHK(hipMemcpyAsync(h->structs, h->pinned_tab, nb, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->offs, h->pinned_tab + nb, (size_t)(S + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
    if (!h->tab_event) HIPCHK(hipEventCreateWithFlags(&h->tab_event, hipEventDisableTiming));
    HIPCHK(hipEventRecord(h->tab_event, s));
    launch_assign_struct(h->offs, S, N, h->sid_ext, s);
  }
  return pp;
}

Prepared prepare(nep_handle* h, int64_t N, const double* box, const int32_t* pbc, double r_list,
                 bool md, hipStream_t s) {
  if (N < 1 || N > (int64_t)1 << 30) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be in [1, 2^30]"};
  const int64_t offs[2] = {0, N};
  return prepare_batch(h, 1, offs, box, pbc, r_list, md, false, s);
}

// The evaluation kernels index their buffers through the rows; a row that
// breaks one of the invariants k_check_rows tests would send them out of
// bounds, so it stops the call before any of them runs.
void check_row_flag(int32_t bits) {
  if (bits)
    throw Failure{NEP_E_HIP, "internal error: neighbour rows break an indexing invariant (bits " +
                                 std::to_string(bits) + ")"};
}

// Rows for the current internal positions; grows the capacities (auto mode)
// or fails (fixed capacities) when a row overflows.  Synchronises once.
void build_rows_checked(nep_handle* h, const Prepared& pp, const BuildArgs& b, hipStream_t s,
                        bool check_types) {
  for (int attempt = 0; attempt < 3; ++attempt) {
    launch_fill_i32(h->flags, 8, 0, s);
    if (check_types) {
      // flags[3]: species out of range, flags[4]: non-finite position
      launch_check_types(h->types, pp.N, h->M.T, h->flags + 3, s);
      launch_check_finite(h->pos, 3 * pp.N, h->flags + 4, s);
    }
    {
      Stage st(h, "neighbor_rows", s);
      launch_build_rows(b, pp.geo.st, pp.batch, h->V, h->L, s);
    }
    launch_check_rows(pp.N, h->sid, h->structs, pp.geo.st, pp.batch, h->L, h->flags + 6, s);
    int32_t* fl = (int32_t*)(h->pinned + kPinFlags);
    HIPCHK(hipMemcpyAsync(fl, h->flags, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (fl[3]) throw Failure{NEP_E_INVALID_ARG, "an atom type is out of range"};
    if (fl[4]) throw Failure{NEP_E_NONFINITE, "positions contain NaN or Inf"};
    // the candidate rows are at r_c^R here: their overflow count is the radial one
    fl[0] = std::max(fl[0], fl[5]);
    if (fl[0] == 0 && fl[1] == 0) {
      // without truncated rows every entry has its reverse entry
      if (fl[2]) throw Failure{NEP_E_HIP, "internal error: neighbour rows are not symmetric"};
      check_row_flag(fl[6]);
      return;
    }
    const bool fixed = h->hp.max_nb_radial || h->hp.max_nb_angular;
    if (fixed) {
      char msg[160];
      std::snprintf(msg, sizeof msg,
                    "neighbour row overflow: need max_nb_radial >= %d and max_nb_angular >= %d",
                    std::max(fl[0], h->MR), std::max(fl[1], h->MA));
      throw Failure{NEP_E_NEIGHBOR_OVERFLOW, msg};
    }
    const int32_t MR = std::max(h->MR, (int32_t)((fl[0] * 1.2 + 8) / 4 * 4 + 4));
    const int32_t MA = std::max(h->MA, (int32_t)((fl[1] * 1.2 + 8) / 4 * 4 + 4));
    ensure_lists(h, pp.N, MR, MA);
    ensure_verlet(h, pp.N, std::max(h->V.MR, MR));
  }
  throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "neighbour rows kept overflowing"};
}

void order_and_build(nep_handle* h, const Prepared& pp, const double* pos_src, const int32_t* types_src,
                     hipStream_t s, bool check) {
  BuildArgs b = build_args(h, pp, pos_src, types_src, h->pos, h->types);
  {
    Stage st(h, "order_atoms", s);
    launch_order_atoms(b, s);
    launch_type_rows(h->types, pp.N, h->M.T, h->hp.nn_per_type, h->tblk, h->tex, h->toff, h->rows,
                     rows_length(pp.N, h->M.T), nullptr, s);
  }
  build_rows_checked(h, pp, b, s, check);
}

void set_groups(EvalArgs& a, int NG, int block, int nA, int lanes) {
  a.NG = NG;
  a.ngroups = (nA + NG - 1) / NG;
  a.block = block;
  a.lanes = lanes;
}

bool autotune_enabled() {
  const char* e = std::getenv("NEP_AUTOTUNE");
  return !(e && e[0] == '0');
}

// Project autotuner: on the first evaluation of a shape, time every admissible
// (angular group size, block size, lanes per atom) of the descriptor and
// partial-force kernels on the actual rows (one warm-up and two timed
// launches each, HIP events on the work stream) and keep the fastest.  The
// choice is fixed per handle afterwards, so repeated calls stay bitwise
// reproducible.
void autotune(nep_handle* h, const Prepared& pp, hipStream_t s) {
  Tuning& t = h->tune[pp.batch ? 1 : 0];
  if (t.done) return;
  const int nA = h->M.nA, L = h->M.L;
  t.NG_desc = t.NG_force = angular_group_size(nA, L);
  t.block_desc = t.block_force = kBlock;
  t.lanes_desc = t.lanes_force = 4;
  t.done = true;
  if (!autotune_enabled()) return;
  EvalArgs a = eval_args(h, pp, h->M);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto time_it = [&](bool force, int ng, int block, int lanes) {
    set_groups(a, ng, block, nA, lanes);
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(hipEventRecord(e0, s));
      bool ok = force ? launch_partial_forces(a, s) : launch_descriptor(a, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      if (!ok) return 1e30f;
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) best = std::min(best, ms);
    }
    return best;
  };
  const int blocks[] = {128, 256};
  const int lane_opts[] = {1, 4};
  auto search = [&](bool force, int& ng_out, int& block_out, int& lanes_out) {
    float best = 1e30f;
    for (int ng : angular_group_options(nA, L))
      for (int bl : blocks)
        for (int ln : lane_opts) {
          if (eval_lds_bytes(h->M, bl) > 64 * 1024) continue;
          float ms = time_it(force, ng, bl, ln);
          if (ms < best) {
            best = ms;
            ng_out = ng;
            block_out = bl;
            lanes_out = ln;
          }
        }
  };
  search(false, t.NG_desc, t.block_desc, t.lanes_desc);
  // the partial-force kernel reads dU/dq: run the chosen descriptor pass and the network once
  set_groups(a, t.NG_desc, t.block_desc, nA, t.lanes_desc);
  launch_descriptor(a, s);
  launch_mlp(a, s);
  search(true, t.NG_force, t.block_force, t.lanes_force);
  // the gather reads the partial forces: run the chosen force pass once, then time lanes 1 and 4
  set_groups(a, t.NG_force, t.block_force, nA, t.lanes_force);
  launch_partial_forces(a, s);
  {
    float best = 1e30f;
    for (int ln : lane_opts) {
      a.lanes = ln;
      float ms_best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(hipEventRecord(e0, s));
        launch_gather_forces(a, false, s);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) ms_best = std::min(ms_best, ms);
      }
      if (ms_best < best) {
        best = ms_best;
        t.lanes_gather = ln;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Descriptors, network, partial forces and the force gather; the per-atom
// virial only when `virial` (MD steps without a thermo row skip it).
void forces(nep_handle* h, const Prepared& pp, hipStream_t s, const DevModel* model = nullptr,
            bool virial = true, const MDArgs* kick = nullptr) {
  autotune(h, pp, s);
  const Tuning& t = h->tune[pp.batch ? 1 : 0];
  EvalArgs a = eval_args(h, pp, model ? *model : h->M);
  set_groups(a, t.NG_desc, t.block_desc, h->M.nA, t.lanes_desc);
  {
    Stage st(h, "descriptor", s);
    if (!launch_descriptor(a, s)) throw Failure{NEP_E_UNSUPPORTED, "no descriptor kernel for this shape"};
  }
  {
    Stage st(h, "mlp", s);
    launch_mlp(a, s);
  }
  set_groups(a, t.NG_force, t.block_force, h->M.nA, t.lanes_force);
  {
    Stage st(h, "partial_forces", s);
    if (!launch_partial_forces(a, s)) throw Failure{NEP_E_UNSUPPORTED, "no force kernel for this shape"};
  }
  {
    Stage st(h, "gather", s);
    a.lanes = t.lanes_gather;
    if (kick) {  // the second half kick of a velocity-Verlet step
      a.kick_vel = kick->vel;
      a.kick_inv_mass = kick->inv_mass;
      a.kick_dt = kick->dt;
    }
    launch_gather_forces(a, virial, s);
  }
}

int fail(nep_handle* h, const Failure& f) {
  if (h) {
    h->err = f.msg;
    h->drop_timing();
  } else {
    g_thread_error = f.msg;
  }
  return f.code;
}

// Every entry point starts here; the count tells an MD run whether any other
// call has used the handle's buffers since the previous run ended.
void set_device(nep_handle* h) {
  HIPCHK(hipSetDevice(h->device));
  ++h->api_calls;
}

void check_host_types(const nep_handle* h, int64_t N, const int32_t* types) {
  for (int64_t i = 0; i < N; ++i)
    if (types[i] < 0 || types[i] >= h->hp.n_types)
      throw Failure{NEP_E_INVALID_ARG, "type of atom " + std::to_string(i) + " out of range"};
}

void check_host_finite(int64_t n, const double* a, const char* what) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) throw Failure{NEP_E_NONFINITE, std::string(what) + " contain NaN or Inf"};
}

int compute_impl(nep_handle* h, int64_t N, const double* d_pos, const int32_t* d_types, const double* box,
                 const int32_t* pbc, double* d_energy, double* d_force, double* d_virial, double* d_totals,
                 hipStream_t s) {
  Prepared pp = prepare(h, N, box, pbc, h->hp.rc_radial, false, s);
  order_and_build(h, pp, d_pos, d_types, s, true);
  forces(h, pp, s);
  EvalArgs a = eval_args(h, pp, h->M);
  {
    Stage st(h, "outputs", s);
    launch_scatter_outputs(a, h->perm, d_energy, d_force, d_virial, s);
    if (d_totals) launch_totals(h->U, h->W, N, h->partial, num_partials(N), d_totals, s);
  }
  return NEP_OK;
}

// Batch of structures x parameter sets (device pointers).  Rows are built once
// and shared by every parameter set (or reused from the previous batch call
// when the caller says the structures are the same); the per-set passes are
// captured into a HIP graph, kept in the handle and replayed by later calls
// with the same shapes, buffers and output pointers.  Parameter vectors come
// from the host (tables built there, one upload per set) or from device
// memory (tables built by a kernel inside the graph, so a training
// generation never goes through the host).
int batch_impl(nep_handle* h, int32_t S, const int64_t* offs, const double* d_pos, const int32_t* d_types,
               const double* boxes, const int32_t* pbcs, int32_t P, const double* params,
               const double* d_params, int32_t flags, double* d_energy, double* d_force, double* d_virial,
               double* d_totals, hipStream_t s) {
  if (!offs) throw Failure{NEP_E_INVALID_ARG, "offsets are required"};
  if (P < 1) throw Failure{NEP_E_INVALID_ARG, "n_param_sets must be >= 1"};
  if (params && d_params) throw Failure{NEP_E_INVALID_ARG, "pass host or device parameters, not both"};
  const bool reuse = (flags & NEP_BATCH_REUSE_ROWS) != 0;
  Prepared pp;
  if (reuse) {
    if (!h->batch_rows_ready || h->batch_S != S || S < 1 || h->batch_N != offs[S])
      throw Failure{NEP_E_INVALID_ARG, "no rows of the same structures to reuse: call once without "
                                       "NEP_BATCH_REUSE_ROWS first"};
    pp.sts = h->batch_sts;
    pp.geo.st = pp.sts[0];
    pp.n_cells = h->batch_cells;
    pp.N = h->batch_N;
    pp.batch = true;
  } else {
    if (!boxes) throw Failure{NEP_E_INVALID_ARG, "boxes are required"};
    h->batch_rows_ready = false;
    pp = prepare_batch(h, S, offs, boxes, pbcs, h->hp.rc_radial, false, true, s);
  }
  const int64_t N = pp.N;
  std::vector<DevModel> models;
  TableLayout TL{};
  if (params) {
    if ((int32_t)h->pop.size() < P) h->pop.resize(P);
    for (int32_t p = 0; p < P; ++p) {
      upload_model(h, params + (size_t)p * n_params(h->hp), h->pop[p]);
      models.push_back(h->pop[p].M);
    }
  } else if (d_params) {
    TL = table_layout(h->hp, h->nd);
    const int64_t need = (int64_t)P * TL.set_bytes;
    if (need > h->pop_tables_cap) {
      HIPCHK(hipStreamSynchronize(s));
      dev_alloc(h->pop_tables, (size_t)need);
      h->pop_tables_cap = need;
    }
    for (int32_t p = 0; p < P; ++p) models.push_back(model_at(h->M, TL, h->pop_tables + p * TL.set_bytes));
  } else {
    if (P != 1) throw Failure{NEP_E_INVALID_ARG, "no parameters given: use n_param_sets = 1"};
    models.push_back(h->M);
  }
  if (!reuse) {
    order_and_build(h, pp, d_pos, d_types, s, true);
    h->batch_rows_ready = true;
    h->batch_S = S;
    h->batch_N = N;
    h->batch_sts = pp.sts;
    h->batch_cells = pp.n_cells;
  }
  autotune(h, pp, s);
  // everything the captured kernels hold by value or by address
  std::vector<unsigned char> key;
  auto put = [&](const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    key.insert(key.end(), c, c + n);
  };
  const uint64_t gen = g_alloc_gen.load();
  put(&gen, sizeof gen);
  put(&S, sizeof S);
  put(&N, sizeof N);
  put(&P, sizeof P);
  const void* ptrs[6] = {d_params, d_energy, d_force, d_virial, d_totals, params};
  put(ptrs, sizeof ptrs);
  const bool timing = h->timing;
  hipStream_t cs = s;
  if (!cs) {  // the legacy null stream cannot be captured: use the handle's own stream
    if (!h->md_stream) HIPCHK(hipStreamCreateWithFlags(&h->md_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamSynchronize(s));
    cs = h->md_stream;
  }
  if (!h->batch_exec || h->batch_key != key) {
    h->drop_batch_graph();
    h->timing = false;
    try {
      HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      if (d_params) launch_model_tables(d_params, (int64_t)n_params(h->hp), P, TL, h->pop_tables, TL.set_bytes, cs);
      for (int32_t p = 0; p < P; ++p) {
        forces(h, pp, cs, &models[p]);
        EvalArgs a = eval_args(h, pp, models[p]);
        launch_scatter_outputs(a, h->perm, d_energy ? d_energy + (size_t)p * N : nullptr,
                               d_force ? d_force + (size_t)p * 3 * N : nullptr,
                               d_virial ? d_virial + (size_t)p * 9 * N : nullptr, cs);
        if (d_totals) launch_struct_totals(h->U, h->W, N, h->structs, S, d_totals + (size_t)p * S * 10, cs);
      }
      HIPCHK(hipStreamEndCapture(cs, &h->batch_graph));
      HIPCHK(hipGraphInstantiate(&h->batch_exec, h->batch_graph, nullptr, nullptr, 0));
      h->batch_key = key;
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(cs, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      h->drop_batch_graph();
      h->timing = timing;
      throw;
    }
    h->timing = timing;
  }
  {
    Stage st(h, "batch_graph", cs);
    HIPCHK(hipGraphLaunch(h->batch_exec, cs));
  }
  // host parameters (and the null stream) keep the call synchronous
  if (params || cs != s) HIPCHK(hipStreamSynchronize(cs));
  return NEP_OK;
}


// ===========================================================================
// serving: continuous batching of evaluation and short-MD requests
// ===========================================================================

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServerReq {
  uint64_t ticket = 0;
  int32_t kind = NEP_REQ_EVAL;
  int64_t n = 0;
  std::vector<double> pos, vel, mass;
  std::vector<int32_t> types;
  double box[9];
  int32_t pbc[3];
  int64_t n_steps = 0;
  double dt = 1.0;
  size_t bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t steps_done = -1;  // -1: initial forces not yet evaluated
  int64_t off = 0;          // offset in the batch state while active
  int32_t status = NEP_OK;
  std::string error;
  std::vector<double> energy, force, virial, out_pos, out_vel;
  double totals[10] = {0};
};

// Device state of the active requests, concatenated in admission order.
struct BatchState {
  int64_t cap = 0;
  int64_t ld = 0;  // current atom count: arrays are [3][ld], [9][ld]
  double *pos = nullptr, *vel = nullptr, *F = nullptr, *E = nullptr, *W = nullptr;
  double *hdm = nullptr, *dta = nullptr, *totals = nullptr, *inv_mass = nullptr;
  int32_t* types = nullptr;
  uint8_t* move = nullptr;
  int32_t cap_req = 0;
  void ensure(int64_t n, int32_t nreq) {
    if (n > cap) {
      release_atoms();
      cap = std::max<int64_t>(n, 1024);
      dev_alloc(pos, 3 * cap); dev_alloc(vel, 3 * cap); dev_alloc(F, 3 * cap); dev_alloc(E, cap);
      dev_alloc(W, 9 * cap); dev_alloc(hdm, cap); dev_alloc(dta, cap); dev_alloc(types, cap);
      dev_alloc(move, cap);
    }
    if (nreq > cap_req) {
      dev_free(totals); dev_free(inv_mass);
      cap_req = std::max(nreq, 16);
      dev_alloc(totals, 10 * (size_t)cap_req);
      dev_alloc(inv_mass, (size_t)kMaxTypes * cap_req);
    }
  }
  void release_atoms() {
    dev_free(pos); dev_free(vel); dev_free(F); dev_free(E); dev_free(W); dev_free(hdm); dev_free(dta);
    dev_free(types); dev_free(move);
    cap = 0;
  }
  void release() {
    release_atoms();
    dev_free(totals); dev_free(inv_mass);
    cap_req = 0;
  }
};

}  // namespace

struct nep_server {
  nep_handle* h = nullptr;
  size_t budget = 0;
  int32_t max_slots = 0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  std::deque<std::shared_ptr<ServerReq>> queue;
  std::vector<std::shared_ptr<ServerReq>> active;
  std::unordered_map<uint64_t, std::shared_ptr<ServerReq>> done;
  uint64_t next_ticket = 1;
  hipStream_t stream = nullptr;
  BatchState st, st2;
  // a tick's uploads (placement table + admitted requests' data) and the
  // finished requests' results: pinned host and device staging, one copy
  // each way per tick
  unsigned char* up_host = nullptr;
  unsigned char* up_dev = nullptr;
  size_t up_cap = 0;
  double* out_host = nullptr;
  double* out_dev = nullptr;
  size_t out_cap = 0;  // doubles
  void release_staging() {
    if (up_host) (void)hipHostFree(up_host);
    if (out_host) (void)hipHostFree(out_host);
    dev_free(up_dev);
    dev_free(out_dev);
    up_host = nullptr;
    out_host = nullptr;
    up_cap = out_cap = 0;
  }
  size_t bytes_active = 0;
  // statistics
  std::vector<double> latencies;
  int64_t submitted = 0, completed = 0, ticks = 0, atom_steps = 0, batch_atoms = 0, batch_reqs = 0;
  double t_first = -1, t_last = 0, busy = 0;
  std::string fatal;
};

namespace {

// Bytes one request of n atoms needs on the device while active: its share of
// the handle's workspace (rows at the density of its box, descriptor and
// partial-force buffers) plus its state in the batch.
size_t request_bytes(const nep_handle* h, int64_t n, double density) {
  const double rc = h->hp.rc_radial, ra = h->hp.rc_angular;
  const size_t MR = estimate_capacity(rc, density), MA = estimate_capacity(ra, density);
  const DevModel& M = h->M;
  const size_t per_atom = (MR + MA) * (4 + 2 + 4 + 12) + 8 + (size_t)M.NDp * 8 +
                          (size_t)M.nA * M.NB * 4 + 48 + 40 + 64 + 24 * 2 + 24 + 8 + 72 + 16 + 8 + 1;
  return per_atom * (size_t)n + 4096;
}

// One tick: every active request advances by one evaluation (and, for MD
// requests past their initial evaluation, one velocity-Verlet step).
}  // namespace

namespace nep {
// output.hip (declared here so that the force kernel's headers stay as profiled):
// per-structure totals of structures of any size, in chunks of a few thousand
// atoms (work: at least 10 doubles per structure)
void launch_struct_totals_chunked(const float* U, const float* W, int64_t N, const StructInfo* structs,
                                  int32_t n_struct, int64_t max_count, double* work, int64_t work_cap,
                                  double* totals, hipStream_t s);
}  // namespace nep

namespace {

void server_tick(nep_server* sv) {
  nep_handle* h = sv->h;
  hipStream_t s = sv->stream;
  ++h->api_calls;  // the tick uses the handle's buffers
  auto& act = sv->active;
  const int32_t S = (int32_t)act.size();
  int64_t N = 0;
  for (auto& r : act) N += r->n;
  BatchState& st = sv->st;
  // layout: keep the order of admission; re-pack when the set changed
  bool repack = false;
  {
    int64_t o = 0;
    for (auto& r : act) {
      if (r->off != o || r->t_admit == 0) repack = true;
      o += r->n;
    }
  }
  if (st.ld != N) repack = true;
  if (repack) {
    BatchState& nx = sv->st2;
    nx.ensure(N, S);
    nx.ld = N;
    // one upload: the placement table {dst, n, src, stg} per request, then the
    // admitted requests' pos [3][ns], vel [3][ns], hdm [ns], dta [ns], types [ns]
    int64_t ns = 0, max_n = 0;
    for (auto& r : act) {
      if (r->t_admit == 0) ns += r->n;
      max_n = std::max(max_n, r->n);
    }
    const size_t tab_bytes = 4 * (size_t)S * sizeof(int64_t);
    const size_t need = tab_bytes + (size_t)ns * (8 * sizeof(double) + sizeof(int32_t));
    if (need > sv->up_cap) {  // the previous tick ended with a synchronisation
      if (sv->up_host) HIPCHK(hipHostFree(sv->up_host));
      sv->up_host = nullptr;
      dev_free(sv->up_dev);
      const size_t cap = std::max<size_t>(need + need / 2, 1 << 16);
      HIPCHK(hipHostMalloc((void**)&sv->up_host, cap, hipHostMallocDefault));
      dev_alloc(sv->up_dev, cap);
      sv->up_cap = cap;
    }
    int64_t* tab = reinterpret_cast<int64_t*>(sv->up_host);
    double* stg = reinterpret_cast<double*>(sv->up_host + tab_bytes);
    int32_t* stg_types = reinterpret_cast<int32_t*>(stg + 8 * ns);
    int64_t o = 0, so = 0;
    int k = 0;
    for (auto& r : act) {
      const int64_t n = r->n;
      tab[4 * k] = o;
      tab[4 * k + 1] = n;
      if (r->t_admit == 0) {  // newly admitted: its state comes from the upload
        tab[4 * k + 2] = -1;
        tab[4 * k + 3] = so;
        const bool md = r->kind == NEP_REQ_MD;
        for (int c = 0; c < 3; ++c) {
          std::memcpy(stg + c * ns + so, r->pos.data() + c * n, n * sizeof(double));
          if (md) std::memcpy(stg + (3 + c) * ns + so, r->vel.data() + c * n, n * sizeof(double));
          else std::fill(stg + (3 + c) * ns + so, stg + (3 + c) * ns + so + n, 0.0);
        }
        // the half-step factor 0.5 dt / (m c) per atom (zero for evaluations)
        double im[kMaxTypes] = {0};
        if (md)
          for (int t = 0; t < h->hp.n_types; ++t) im[t] = 1.0 / (r->mass[t] * kAmuA2fs2);
        const double half_dt = 0.5 * r->dt;
        for (int64_t e = 0; e < n; ++e) {
          stg[6 * ns + so + e] = half_dt * im[r->types[e]];
          stg[7 * ns + so + e] = r->dt;
        }
        std::memcpy(stg_types + so, r->types.data(), n * sizeof(int32_t));
        so += n;
        r->t_admit = now_s();
      } else {  // carried over: its device state moves to the new offset
        tab[4 * k + 2] = r->off;
        tab[4 * k + 3] = 0;
      }
      r->off = o;
      o += n;
      ++k;
    }
    HIPCHK(hipMemcpyAsync(sv->up_dev, sv->up_host, need, hipMemcpyHostToDevice, s));
    const BatchState& od = sv->st;
    const SrvState from{od.pos, od.vel, od.F, od.hdm, od.dta, od.types, od.move, od.ld};
    const SrvState to{nx.pos, nx.vel, nx.F, nx.hdm, nx.dta, nx.types, nx.move, nx.ld};
    launch_srv_place(reinterpret_cast<const int64_t*>(sv->up_dev), S, max_n, from, to,
                     reinterpret_cast<const double*>(sv->up_dev + tab_bytes), ns, s);
    std::swap(sv->st, sv->st2);
  }
  BatchState& b = sv->st;
  std::vector<int64_t> offs(S + 1, 0);
  std::vector<double> boxes(9 * (size_t)S);
  std::vector<int32_t> pbcs(3 * (size_t)S);
  for (int32_t k = 0; k < S; ++k) {
    offs[k + 1] = offs[k] + act[k]->n;
    std::memcpy(&boxes[9 * k], act[k]->box, sizeof act[k]->box);
    std::memcpy(&pbcs[3 * k], act[k]->pbc, sizeof act[k]->pbc);
  }
  launch_srv_kick_drift(N, b.pos, b.vel, b.F, b.hdm, b.dta, b.move, s);
  Prepared pp = prepare_batch(h, S, offs.data(), boxes.data(), pbcs.data(), h->hp.rc_radial, false, true, s);
  order_and_build(h, pp, b.pos, b.types, s, true);
  forces(h, pp, s);
  EvalArgs a = eval_args(h, pp, h->M);
  launch_scatter_outputs(a, h->perm, b.E, b.F, b.W, s);
  {
    int64_t max_n = 0;
    for (auto& r : act) max_n = std::max(max_n, r->n);
    launch_struct_totals_chunked(h->U, h->W, N, h->structs, S, max_n, h->partial, 11 * h->cap_part, b.totals, s);
  }
  launch_srv_kick(N, b.vel, b.F, b.hdm, b.move, s);
  // bookkeeping: the finished requests' results go out in one packed copy
  std::vector<std::shared_ptr<ServerReq>> finished;
  std::vector<int64_t> fin_out;  // offset of each finished request's block in the staging
  std::vector<double> tot(10 * (size_t)S);
  HIPCHK(hipMemcpyAsync(tot.data(), b.totals, tot.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  std::vector<int64_t> ctab;
  int64_t out_n = 0, max_fin = 0;
  for (int32_t k = 0; k < S; ++k) {
    auto& r = act[k];
    bool fin = false;
    if (r->kind == NEP_REQ_EVAL) {
      fin = true;
    } else if (r->steps_done < 0) {
      r->steps_done = 0;
      launch_fill_u8(b.move + r->off, r->n, 1, s);
      fin = r->n_steps == 0;
    } else {
      r->steps_done += 1;
      fin = r->steps_done >= r->n_steps;
    }
    sv->atom_steps += r->n;
    if (fin) {
      const int64_t md = r->kind == NEP_REQ_MD ? 1 : 0;
      ctab.insert(ctab.end(), {r->off, r->n, out_n, md});
      fin_out.push_back(out_n);
      out_n += r->n * (13 + 6 * md);
      max_fin = std::max(max_fin, r->n);
      finished.push_back(r);
    }
  }
  if (!finished.empty()) {
    const size_t need = (size_t)out_n + ctab.size();  // results, then the table
    if (need > sv->out_cap) {
      if (sv->out_host) HIPCHK(hipHostFree(sv->out_host));
      sv->out_host = nullptr;
      dev_free(sv->out_dev);
      const size_t cap = std::max<size_t>(need + need / 2, 1 << 16);
      HIPCHK(hipHostMalloc((void**)&sv->out_host, cap * sizeof(double), hipHostMallocDefault));
      dev_alloc(sv->out_dev, cap);
      sv->out_cap = cap;
    }
    // the table rides in the tail of the staging (8-byte words both ways)
    std::memcpy(sv->out_host + out_n, ctab.data(), ctab.size() * sizeof(int64_t));
    HIPCHK(hipMemcpyAsync(sv->out_dev + out_n, sv->out_host + out_n, ctab.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
    launch_srv_collect(reinterpret_cast<const int64_t*>(sv->out_dev + out_n), (int32_t)finished.size(), max_fin,
                       N, b.E, b.F, b.W, b.pos, b.vel, sv->out_dev, s);
    HIPCHK(hipMemcpyAsync(sv->out_host, sv->out_dev, out_n * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  for (size_t f = 0; f < finished.size(); ++f) {
    auto& r = finished[f];
    const size_t n = r->n;
    const double* blk = sv->out_host + fin_out[f];
    r->energy.assign(blk, blk + n);
    r->force.assign(blk + n, blk + 4 * n);
    r->virial.assign(blk + 4 * n, blk + 13 * n);
    if (r->kind == NEP_REQ_MD) {
      r->out_pos.assign(blk + 13 * n, blk + 16 * n);
      r->out_vel.assign(blk + 16 * n, blk + 19 * n);
    }
  }
  const double t = now_s();
  sv->ticks += 1;
  sv->batch_atoms += N;
  sv->batch_reqs += S;
  for (int32_t k = 0; k < S; ++k) std::memcpy(act[k]->totals, &tot[10 * k], 10 * sizeof(double));
  std::lock_guard<std::mutex> lk(sv->mu);
  for (auto& r : finished) {
    r->t_done = t;
    sv->bytes_active -= r->bytes;
    sv->latencies.push_back(r->t_done - r->t_submit);
    sv->completed += 1;
    sv->t_last = t;
    sv->done[r->ticket] = r;
  }
  act.erase(std::remove_if(act.begin(), act.end(), [](const std::shared_ptr<ServerReq>& r) { return r->t_done > 0; }),
            act.end());
  // the remaining requests are re-packed next tick if their offsets moved
  sv->done_cv.notify_all();
}

void server_loop(nep_server* sv) {
  try {
    HIPCHK(hipSetDevice(sv->h->device));
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty() || !sv->active.empty(); });
        if (sv->stop && sv->queue.empty() && sv->active.empty()) return;
        // admission: free slots and HBM budget, first come first served
        while (!sv->queue.empty() && (int32_t)sv->active.size() < sv->max_slots &&
               sv->bytes_active + sv->queue.front()->bytes <= sv->budget) {
          sv->bytes_active += sv->queue.front()->bytes;
          sv->active.push_back(sv->queue.front());
          sv->queue.pop_front();
        }
      }
      if (sv->active.empty()) continue;
      const double t0 = now_s();
      server_tick(sv);
      sv->busy += now_s() - t0;
    }
  } catch (const Failure& f) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->fatal = f.msg;
    for (auto& r : sv->active) {
      r->status = f.code;
      r->error = f.msg;
      r->t_done = now_s();
      sv->done[r->ticket] = r;
    }
    for (auto& r : sv->queue) {
      r->status = f.code;
      r->error = f.msg;
      r->t_done = now_s();
      sv->done[r->ticket] = r;
    }
    sv->active.clear();
    sv->queue.clear();
    sv->done_cv.notify_all();
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

namespace nep {
// output.hip (declared here so that the force kernel's headers stay as profiled)
void launch_heat_current(const float* W, int64_t N, const int32_t* perm, const double* vel,
                         double* heat, double* total, double* partial, int64_t n_part,
                         hipStream_t s);
int64_t loss_chunks(int64_t N);
void launch_loss(const double* force, const double* totals, const int64_t* offs, int32_t S, int64_t N,
                 int32_t P, const double* e_tar, const double* f_tar, const double* w_tar,
                 const double* params, int64_t npar, const double lam[5], double* partial, double* loss,
                 hipStream_t s);
void launch_snes_step(const double* loss, int64_t stride, int32_t P, const double* noise, int64_t n_par,
                      double eta_mu, double eta_sigma, double* util, double* mean, double* sigma,
                      hipStream_t s);
void launch_snes_sample(const double* mean, const double* sigma, const double* noise, int64_t n_par,
                        int32_t P, double* pop, hipStream_t s);
}  // namespace nep

namespace {
// Heat current of eq. Ji from the per-atom virial left by compute_impl.
void heat_current_impl(nep_handle* h, int64_t N, const double* d_pos, const double* d_vel,
                       const int32_t* d_types, const double* box, const int32_t* pbc,
                       double* d_heat, double* d_total, hipStream_t s) {
  if (!d_vel) throw Failure{NEP_E_INVALID_ARG, "velocities are required"};
  compute_impl(h, N, d_pos, d_types, box, pbc, nullptr, nullptr, nullptr, nullptr, s);
  // one block of 256 threads per 256 atoms, each with its own partial row
  const int64_t n_part = (N + 255) / 256;
  if (3 * n_part > h->heat_part_cap) {
    HIPCHK(hipStreamSynchronize(s));
    dev_alloc(h->heat_part, (size_t)(3 * n_part));
    h->heat_part_cap = 3 * n_part;
  }
  Stage st(h, "heat_current", s);
  launch_heat_current(h->W, N, h->perm, d_vel, d_heat, d_total, h->heat_part, n_part, s);
}
}  // namespace

extern "C" {

int nep_num_descriptors(const nep_hparams* hp) {
  std::string why;
  if (!check_hparams(hp, why)) return -1;
  return n_descriptors(*hp);
}

size_t nep_num_params(const nep_hparams* hp) {
  std::string why;
  if (!check_hparams(hp, why)) return 0;
  return n_params(*hp);
}

const char* nep_last_error(const nep_handle* h) {
  return h ? h->err.c_str() : g_thread_error.c_str();
}

int nep_create(const nep_hparams* hp, const double* params, size_t n, nep_handle** out) {
  if (!out) return fail(nullptr, {NEP_E_INVALID_ARG, "out is NULL"});
  *out = nullptr;
  std::string why;
  if (!check_hparams(hp, why)) return fail(nullptr, {NEP_E_INVALID_ARG, why});
  if (!params || n != n_params(*hp))
    return fail(nullptr, {NEP_E_INVALID_ARG, "params must hold nep_num_params(hp) = " +
                                                 std::to_string(n_params(*hp)) + " doubles"});
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(nullptr, {NEP_E_UNSUPPORTED, "no HIP device available"});
  }
  nep_handle* h = new nep_handle();
  try {
    h->hp = *hp;
    HIPCHK(hipGetDevice(&h->device));
    HIPCHK(hipHostMalloc((void**)&h->pinned, 4096, hipHostMallocDefault));
    h->nd = n_descriptors(*hp);
    h->nets = hp->nn_per_type ? hp->n_types : 1;
    upload_model(h, params, h->main);
    HIPCHK(loss_scratch_address(h->device, &h->scratch));
    // LDS budget of the pair kernels: coefficient tables + per-thread slots
    if (eval_lds_bytes(h->M, kBlock) > 64 * 1024)
      throw Failure{NEP_E_UNSUPPORTED, "n_types x basis sizes too large for the LDS budget"};
  } catch (const Failure& f) {
    delete h;
    return fail(nullptr, f);
  }
  *out = h;
  return NEP_OK;
}

int nep_set_params(nep_handle* h, const double* params, size_t n) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!params || n != n_params(h->hp)) return fail(h, {NEP_E_INVALID_ARG, "wrong parameter count"});
  try {
    set_device(h);
    upload_model(h, params, h->main);
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

void nep_destroy(nep_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  delete h;
}

int nep_compute(nep_handle* h, int64_t N, const double* pos, const int32_t* types, const double box[9],
                const int32_t pbc[3], double* energy, double* force, double* virial, double totals[10]) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types || !box) return fail(h, {NEP_E_INVALID_ARG, "pos, types and box are required"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    hipStream_t s = nullptr;
    Prepared pp = prepare(h, N, box, pbc, h->hp.rc_radial, false, s);
    (void)pp;
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    compute_impl(h, N, h->pos_ext, h->types_ext, box, pbc, energy ? h->out_e : nullptr,
                 force ? h->out_f : nullptr, virial ? h->out_w : nullptr, totals ? h->totals : nullptr, s);
    if (energy) HIPCHK(hipMemcpyAsync(energy, h->out_e, N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (force) HIPCHK(hipMemcpyAsync(force, h->out_f, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (virial) HIPCHK(hipMemcpyAsync(virial, h->out_w, 9 * N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (totals) HIPCHK(hipMemcpyAsync(totals, h->totals, 10 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_compute_dev(nep_handle* h, int64_t N, const double* pos, const int32_t* types, const double box[9],
                    const int32_t pbc[3], double* energy, double* force, double* virial, double* totals,
                    void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types || !box) return fail(h, {NEP_E_INVALID_ARG, "pos, types and box are required"});
  try {
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    compute_impl(h, N, pos, types, box, pbc, energy, force, virial, totals, s);
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_heat_current(nep_handle* h, int64_t N, const double* pos, const double* vel,
                     const int32_t* types, const double box[9], const int32_t pbc[3], double* heat,
                     double total[3]) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !vel || !types || !box)
    return fail(h, {NEP_E_INVALID_ARG, "pos, vel, types and box are required"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    check_host_finite(3 * N, vel, "velocities");
    hipStream_t s = nullptr;
    Prepared pp = prepare(h, N, box, pbc, h->hp.rc_radial, false, s);
    (void)pp;
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // the velocities travel in the force buffer (3N doubles), unused by this call
    HIPCHK(hipMemcpyAsync(h->out_f, vel, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    heat_current_impl(h, N, h->pos_ext, h->out_f, h->types_ext, box, pbc, heat ? h->out_w : nullptr,
                      total ? h->totals : nullptr, s);
    if (heat) HIPCHK(hipMemcpyAsync(heat, h->out_w, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (total) HIPCHK(hipMemcpyAsync(total, h->totals, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_heat_current_dev(nep_handle* h, int64_t N, const double* pos, const double* vel,
                         const int32_t* types, const double box[9], const int32_t pbc[3],
                         double* heat, double* total, void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !vel || !types || !box)
    return fail(h, {NEP_E_INVALID_ARG, "pos, vel, types and box are required"});
  try {
    set_device(h);
    heat_current_impl(h, N, pos, vel, types, box, pbc, heat, total, (hipStream_t)stream);
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

}  // extern "C"

namespace {
void check_loss_args(const nep_handle* h, int32_t n_struct, const int64_t* offsets, int32_t n_param_sets,
                     const double* params, int64_t n_par, const double* force, const double* totals,
                     const double* energy_target, const double* force_target, const double* lambda,
                     const double* loss) {
  if (n_struct < 1 || n_param_sets < 1 || n_param_sets > 65535)
    throw Failure{NEP_E_INVALID_ARG, "need n_struct >= 1 and 1 <= n_param_sets <= 65535"};
  if (!offsets || !force || !totals || !energy_target || !force_target || !lambda || !loss)
    throw Failure{NEP_E_INVALID_ARG,
                  "offsets, force, totals, energy_target, force_target, lambda and loss are required"};
  if (offsets[0] != 0) throw Failure{NEP_E_INVALID_ARG, "offsets[0] must be 0"};
  for (int32_t s = 0; s < n_struct; ++s)
    if (offsets[s + 1] <= offsets[s])
      throw Failure{NEP_E_INVALID_ARG, "structure " + std::to_string(s) + " has no atoms"};
  if (params && n_par != (int64_t)n_params(h->hp))
    throw Failure{NEP_E_INVALID_ARG, "n_params does not match the model"};
  for (int v = 0; v < 5; ++v)
    if (!std::isfinite(lambda[v])) throw Failure{NEP_E_NONFINITE, "lambda contains NaN or Inf"};
}
}  // namespace

extern "C" {

int nep_batch_loss(nep_handle* h, int32_t n_struct, const int64_t* offsets, int32_t n_param_sets,
                   const double* params, int64_t n_par, const double* force, const double* totals,
                   const double* energy_target, const double* force_target, const double* virial_target,
                   const double lambda[5], double* loss, void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  try {
    check_loss_args(h, n_struct, offsets, n_param_sets, params, n_par, force, totals, energy_target,
                    force_target, lambda, loss);
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = offsets[n_struct];
    const int64_t need_part = (int64_t)n_param_sets * loss_chunks(N) * 6;  // six sums per chunk
    if (need_part > h->loss_part_cap) {
      HIPCHK(hipStreamSynchronize(s));
      dev_alloc(h->loss_part, (size_t)need_part);
      h->loss_part_cap = need_part;
    }
    if (n_struct + 1 > h->loss_offs_cap) {
      HIPCHK(hipStreamSynchronize(s));
      dev_alloc(h->loss_offs, (size_t)n_struct + 1);
      h->loss_offs_cap = n_struct + 1;
      h->loss_offs_host.clear();
    }
    // the offsets are uploaded only when they differ from the last call's
    if (h->loss_offs_host.size() != (size_t)n_struct + 1 ||
        !std::equal(offsets, offsets + n_struct + 1, h->loss_offs_host.begin())) {
      HIPCHK(hipMemcpyAsync(h->loss_offs, offsets, ((size_t)n_struct + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));  // the host array may change after the call
      h->loss_offs_host.assign(offsets, offsets + n_struct + 1);
    }
    {
      Stage st(h, "batch_loss", s);
      launch_loss(force, totals, h->loss_offs, n_struct, N, n_param_sets, energy_target, force_target,
                  virial_target, params, params ? n_par : 0, lambda, h->loss_part, loss, s);
    }
    HIPCHK(hipGetLastError());
    if (h->timing) h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_batch_loss_noalloc(nep_handle* h, int32_t n_struct, const int64_t* offsets, int32_t n_param_sets,
                           const double* params, int64_t n_par, const double* force, const double* totals,
                           const double* energy_target, const double* force_target,
                           const double* virial_target, const double lambda[5], double* loss,
                           void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  try {
    check_loss_args(h, n_struct, offsets, n_param_sets, params, n_par, force, totals, energy_target,
                    force_target, lambda, loss);
    // the workspace: per-chunk partial sums, then the structure offsets
    const int64_t N = offsets[n_struct];
    const size_t part_bytes = (size_t)n_param_sets * loss_chunks(N) * 6 * sizeof(double);
    const size_t offs_at = (part_bytes + 255) / 256 * 256;
    const size_t need = offs_at + ((size_t)n_struct + 1) * sizeof(int64_t);
    if (need > (size_t)kLossScratchBytes)
      throw Failure{NEP_E_INVALID_ARG, "batch too large for the fixed loss workspace: needs " +
                                           std::to_string(need) + " bytes, the limit is " +
                                           std::to_string(kLossScratchBytes)};
    if (!h->scratch) throw Failure{NEP_E_HIP, "the loss workspace has no device address"};
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    unsigned char* base = (unsigned char*)h->scratch;
    double* part = (double*)base;
    int64_t* d_offs = (int64_t*)(base + offs_at);
    HIPCHK(hipMemcpyAsync(d_offs, offsets, ((size_t)n_struct + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    launch_loss(force, totals, d_offs, n_struct, N, n_param_sets, energy_target, force_target, virial_target,
                params, params ? n_par : 0, lambda, part, loss, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_snes_step(nep_handle* h, int64_t n_par, int32_t n_pop, double* mean, double* sigma,
                  const double* noise, const double* loss, int64_t loss_stride, double eta_mu,
                  double eta_sigma, void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  try {
    if (n_par < 1 || n_pop < 2 || n_pop > 1024)
      throw Failure{NEP_E_INVALID_ARG, "need n_par >= 1 and 2 <= n_pop <= 1024"};
    if (!mean || !sigma || !noise || !loss || loss_stride < 1)
      throw Failure{NEP_E_INVALID_ARG, "mean, sigma, noise and loss are required, loss_stride >= 1"};
    if (!std::isfinite(eta_mu) || !std::isfinite(eta_sigma))
      throw Failure{NEP_E_NONFINITE, "learning rates must be finite"};
    set_device(h);
    hipStream_t s = (hipStream_t)stream;
    if (!h->snes_util) dev_alloc(h->snes_util, 1024);
    launch_snes_step(loss, loss_stride, n_pop, noise, n_par, eta_mu, eta_sigma, h->snes_util, mean, sigma, s);
    HIPCHK(hipGetLastError());
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_snes_sample(nep_handle* h, int64_t n_par, int32_t n_pop, const double* mean, const double* sigma,
                    const double* noise, double* population, void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  try {
    if (n_par < 1 || n_pop < 1 || n_pop > 65535)
      throw Failure{NEP_E_INVALID_ARG, "need n_par >= 1 and 1 <= n_pop <= 65535"};
    if (!mean || !sigma || !noise || !population)
      throw Failure{NEP_E_INVALID_ARG, "mean, sigma, noise and population are required"};
    set_device(h);
    launch_snes_sample(mean, sigma, noise, n_par, n_pop, population, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_neighbors(nep_handle* h, int64_t N, const double* pos, const double box[9], const int32_t pbc[3],
                  int32_t which, int32_t cap, int32_t* count, int32_t* nbr, int32_t* shift) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !box || !count || !nbr || !shift || cap < 1 || (which != 0 && which != 1))
    return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_finite(3 * N, pos, "positions");
    hipStream_t s = nullptr;
    Prepared pp = prepare(h, N, box, pbc, h->hp.rc_radial, false, s);
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    launch_fill_i32(h->types_ext, N, 0, s);
    order_and_build(h, pp, h->pos_ext, h->types_ext, s, true);
    int32_t *d_count = nullptr, *d_nbr = nullptr, *d_shift = nullptr;
    dev_alloc(d_count, N);
    dev_alloc(d_nbr, (size_t)N * cap);
    dev_alloc(d_shift, (size_t)N * cap * 3);
    launch_inverse_perm(h->perm, N, h->inv, s);
    launch_neighbors_out(h->L, which, N, h->perm, h->inv, h->pos, h->sid, h->structs, cap, d_count, d_nbr,
                         d_shift, s);
    HIPCHK(hipMemcpyAsync(count, d_count, N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(nbr, d_nbr, (size_t)N * cap * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(shift, d_shift, (size_t)N * cap * 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dev_free(d_count);
    dev_free(d_nbr);
    dev_free(d_shift);
    int32_t need = 0;
    for (int64_t i = 0; i < N; ++i) need = std::max(need, count[i]);
    if (need > cap)
      throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "a row has " + std::to_string(need) + " entries > cap"};
    std::vector<std::array<int32_t, 4>> row;
    for (int64_t i = 0; i < N; ++i) {
      row.resize(count[i]);
      for (int m = 0; m < count[i]; ++m)
        row[m] = {nbr[i * cap + m], shift[(i * cap + m) * 3], shift[(i * cap + m) * 3 + 1],
                  shift[(i * cap + m) * 3 + 2]};
      std::sort(row.begin(), row.end());
      for (int m = 0; m < count[i]; ++m) {
        nbr[i * cap + m] = row[m][0];
        for (int c = 0; c < 3; ++c) shift[(i * cap + m) * 3 + c] = row[m][1 + c];
      }
    }
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_elastic_cubic(nep_handle* h, int64_t N, const double* pos, const int32_t* types, const double box[9],
                      const int32_t pbc[3], double strain, double C[3]) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types || !box || !C) return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    if (!(strain > 0) || !(strain < 0.2)) throw Failure{NEP_E_INVALID_ARG, "strain must be in (0, 0.2)"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    const double V = std::fabs(box[0] * (box[4] * box[8] - box[5] * box[7]) -
                               box[1] * (box[3] * box[8] - box[5] * box[6]) +
                               box[2] * (box[3] * box[7] - box[4] * box[6]));
    hipStream_t s = nullptr;
    std::vector<double> p(3 * N);
    // total energy of the cell deformed by F = I + eps (positions r -> F r,
    // cell vectors a -> F a), from the device totals
    auto energy = [&](const double eps[9]) {
      double F[9], b[9];
      for (int k = 0; k < 9; ++k) F[k] = eps[k] + ((k % 4) == 0 ? 1.0 : 0.0);
      for (int64_t i = 0; i < N; ++i)
        for (int r = 0; r < 3; ++r)
          p[r * N + i] = F[3 * r] * pos[i] + F[3 * r + 1] * pos[N + i] + F[3 * r + 2] * pos[2 * N + i];
      for (int v = 0; v < 3; ++v)
        for (int r = 0; r < 3; ++r)
          b[3 * v + r] = F[3 * r] * box[3 * v] + F[3 * r + 1] * box[3 * v + 1] + F[3 * r + 2] * box[3 * v + 2];
      prepare(h, N, b, pbc, h->hp.rc_radial, false, s);
      HIPCHK(hipMemcpyAsync(h->pos_ext, p.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
      compute_impl(h, N, h->pos_ext, h->types_ext, b, pbc, nullptr, nullptr, nullptr, h->totals, s);
      double t = 0;
      HIPCHK(hipMemcpyAsync(h->pinned + 2048, h->totals, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::memcpy(&t, h->pinned + 2048, sizeof t);
      return t;
    };
    const double zero[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double e0 = energy(zero);
    // second difference (E(+d) + E(-d) - 2 E(0)) / d^2 along eps = d A
    auto curvature = [&](const double A[9]) {
      double ep[9], em[9];
      for (int k = 0; k < 9; ++k) {
        ep[k] = strain * A[k];
        em[k] = -strain * A[k];
      }
      return (energy(ep) + energy(em) - 2.0 * e0) / (strain * strain);
    };
    const double uni[9] = {1, 0, 0, 0, 0, 0, 0, 0, 0};
    const double bi[9] = {1, 0, 0, 0, 1, 0, 0, 0, 0};
    const double shear[9] = {0, 0.5, 0, 0.5, 0, 0, 0, 0, 0};
    const double c11 = curvature(uni) / V, c1112 = curvature(bi) / (2.0 * V), c44 = curvature(shear) / V;
    const double gpa = 160.21766208;  // eV/A^3 in GPa
    C[0] = c11 * gpa;
    C[1] = (c1112 - c11) * gpa;
    C[2] = c44 * gpa;
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_descriptors(nep_handle* h, int64_t N, const double* pos, const int32_t* types, const double box[9],
                    const int32_t pbc[3], double* q) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types || !box || !q) return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    hipStream_t s = nullptr;
    Prepared pp = prepare(h, N, box, pbc, h->hp.rc_radial, false, s);
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    order_and_build(h, pp, h->pos_ext, h->types_ext, s, true);
    autotune(h, pp, s);
    EvalArgs a = eval_args(h, pp, h->M);
    set_groups(a, h->tune[0].NG_desc, h->tune[0].block_desc, h->M.nA, h->tune[0].lanes_desc);
    if (!launch_descriptor(a, s)) throw Failure{NEP_E_UNSUPPORTED, "no descriptor kernel for this shape"};
    double* d_q = nullptr;
    dev_alloc(d_q, (size_t)N * h->nd);
    launch_descriptors_out(h->q, N, h->M.NDp, h->nd, h->perm, d_q, s);
    HIPCHK(hipMemcpyAsync(q, d_q, (size_t)N * h->nd * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dev_free(d_q);
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_latent(nep_handle* h, int64_t N, const double* pos, const int32_t* types, const double box[9],
               const int32_t pbc[3], double* latent) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types || !box || !latent) return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  float* d_lat = nullptr;
  double* d_out = nullptr;
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    hipStream_t s = nullptr;
    Prepared pp = prepare(h, N, box, pbc, h->hp.rc_radial, false, s);
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    order_and_build(h, pp, h->pos_ext, h->types_ext, s, true);
    autotune(h, pp, s);
    const int NN = h->hp.n_neurons;
    dev_alloc(d_lat, (size_t)N * NN);
    dev_alloc(d_out, (size_t)N * NN);
    EvalArgs a = eval_args(h, pp, h->M);
    set_groups(a, h->tune[0].NG_desc, h->tune[0].block_desc, h->M.nA, h->tune[0].lanes_desc);
    if (!launch_descriptor(a, s)) throw Failure{NEP_E_UNSUPPORTED, "no descriptor kernel for this shape"};
    a.latent = d_lat;
    launch_mlp(a, s);
    launch_descriptors_out(d_lat, N, NN, NN, h->perm, d_out, s);
    HIPCHK(hipMemcpyAsync(latent, d_out, (size_t)N * NN * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dev_free(d_lat);
    dev_free(d_out);
  } catch (const Failure& f) {
    dev_free(d_lat);
    dev_free(d_out);
    return fail(h, f);
  }
  return NEP_OK;
}

namespace {

// Rebuild now from the current internal state: re-sort into cell order
// (velocities and caller indices follow), remember the positions, and build
// the candidate rows.  gate = NULL runs unconditionally.
void skin_rebuild(nep_handle* h, const Prepared& pp, double rl, const int32_t* gate, hipStream_t s,
                  double* mu_cum = nullptr) {
  const int64_t N = pp.N;
  BuildArgs br = build_args(h, pp, h->pos, h->types, h->pos2, h->types2);
  br.ext_src = h->ext_id;
  br.gate = gate;
  br.vel_src = h->vel;
  br.vel_dst = h->vel2;
  br.ext_in = h->ext_id;
  br.ext_out = h->ext_id2;
  launch_order_atoms(br, s);
  launch_commit_rebuild(N, h->pos2, h->vel2, h->types2, h->ext_id2, h->pos, h->vel, h->types,
                        h->ext_id, h->pos_ref, gate, s, mu_cum, h->flags + kFlagRebuilds);
  BuildArgs bv = build_args(h, pp, nullptr, nullptr, h->pos, h->types);
  bv.rcR2 = rl * rl;
  bv.gate = gate;
  launch_build_verlet(bv, h->V, s);
  launch_type_rows(h->types, N, h->M.T, h->hp.nn_per_type, h->tblk, h->tex, h->toff, h->rows,
                   rows_length(N, h->M.T), gate, s);
}

void skin_filter(nep_handle* h, const Prepared& pp, hipStream_t s) {
  BuildArgs bf = build_args(h, pp, nullptr, nullptr, h->pos, h->types);
  launch_filter_rows(bf, pp.geo.st, pp.batch, h->V, h->L, s);
}

// Grow whichever rows overflowed (flags [0] radial, [1] angular, [5]
// candidate); returns false if nothing overflowed.
bool grow_rows(nep_handle* h, int64_t N, const int32_t* fl) {
  if (!fl[0] && !fl[1] && !fl[5]) return false;
  if ((fl[0] || fl[1]) && (h->hp.max_nb_radial || h->hp.max_nb_angular))
    throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "neighbour row overflow during the run"};
  if (fl[0] || fl[1])
    ensure_lists(h, N, std::max(h->MR, (int32_t)((fl[0] * 1.2 + 8) / 4 * 4 + 4)),
                 std::max(h->MA, (int32_t)((fl[1] * 1.2 + 8) / 4 * 4 + 4)));
  if (fl[5]) ensure_verlet(h, N, std::max(h->V.MR, (int32_t)((fl[5] * 1.2 + 8) / 4 * 4 + 4)));
  return true;
}

int32_t* read_flags(nep_handle* h, hipStream_t s) {
  int32_t* fl = (int32_t*)(h->pinned + kPinFlags);
  HIPCHK(hipMemcpyAsync(fl, h->flags, kFlagsRead * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return fl;
}

// NPT: the cell grid and the minimum-image rule were set up for the box at
// the start of the call (with headroom); fail clearly once the box has
// shrunk past them (a new call sets them up for the current box).
void check_npt_cell(const StructInfo& now, const StructInfo& start, double rl) {
  for (int k = 0; k < 3; ++k) {
    if (!now.pbc[k]) continue;
    const double* u = now.H + 3 * ((k + 1) % 3);
    const double* v = now.H + 3 * ((k + 2) % 3);
    const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
    const double* a = now.H + 3 * k;
    const double w = std::fabs(a[0] * cx + a[1] * cy + a[2] * cz) / std::sqrt(cx * cx + cy * cy + cz * cz);
    const bool cells_ok = start.mode != kModeCells || w / start.ncell[k] >= rl;
    const bool image_ok = start.mode == kModeImages || w > 2.0 * rl;
    if (!cells_ok || !image_ok)
      throw Failure{NEP_E_BOX, "the box shrank past the cell grid set up at the start of the call; "
                               "continue with a new call from the returned state"};
  }
}

// Velocity Verlet with candidate rows at r_c^R + skin, rebuilt on the device
// when an atom has moved more than skin / 2 since the last build; the exact
// rows are filtered from them every step.
int md_skin(nep_handle* h, const Prepared& pp, double* d_pos, double* d_vel, const int32_t* d_types,
            double dt, int64_t n_steps, int64_t thermo_every, double* thermo_out, bool thermo_on_host,
            int64_t n_rows, hipStream_t s, const EnsParams* ep = nullptr, double* ens_state = nullptr,
            double* box_out = nullptr) {
  const int64_t N = pp.N;
  const double skin = h->hp.skin, rl = h->hp.rc_radial + skin;
  const double thr2 = 0.25 * skin * skin;
  int32_t* gate = h->flags + 7;
  ensure_verlet(h, N, std::max(h->V.MR, estimate_capacity(rl, (double)N / pp.geo.volume)));
  const int64_t rebuilds0 = h->md_rebuilds;  // the device counts this call's rebuilds from 0
  launch_fill_i32(h->flags + kFlagRebuilds, 1, 0, s);
  // ensemble state on the device (thermostats and barostats)
  const bool ens = ep != nullptr;
  const bool npt = ens && ep->kind >= kEnsNptBerendsen;
  const int64_t step_base = ens ? (int64_t)ens_state[0] : 0;
  const int row_len = ens ? 16 : 13;
  EnsState* est = nullptr;
  double* mu_cum = nullptr;
  if (ens) {
    // [state][saved state][saved structure 0], 256-byte aligned parts
    if (!h->ens_state) dev_alloc(h->ens_state, 3 * 512 / sizeof(double));
    static_assert(sizeof(StructInfo) <= 512, "staging slot");
    const int64_t need = std::max<int64_t>(ens_partials(N), div_up(N, 256) + 1) + 1;
    if (need > h->ens_partial_cap) {
      dev_alloc(h->ens_partial, (size_t)need);
      h->ens_partial_cap = need;
    }
    est = (EnsState*)h->ens_state;
    EnsState init{};
    init.heat = ens_state[1];
    for (int k = 0; k < kMaxChain; ++k) {
      init.xi[k] = ens_state[2 + k];
      init.vxi[k] = ens_state[10 + k];
    }
    init.step = step_base;
    init.mu = init.mu_cum = init.scale = 1.0;
    static_assert(sizeof(EnsState) <= 512, "staging slot");
    std::memcpy(h->pinned + 1024, &init, sizeof init);
    HIPCHK(hipMemcpyAsync(est, h->pinned + 1024, sizeof init, hipMemcpyHostToDevice, s));
    if (npt) mu_cum = &est->mu_cum;
  }
  // what the internal state depends on besides the caller's arrays
  auto state_key = [&]() {
    std::vector<unsigned char> k;
    auto put = [&](const void* p, size_t n) {
      const unsigned char* c = (const unsigned char*)p;
      k.insert(k.end(), c, c + n);
    };
    const uint64_t gen = g_alloc_gen.load();
    put(&gen, sizeof gen);
    put(&N, sizeof N);
    put(&rl, sizeof rl);
    put(&pp.geo.st, sizeof pp.geo.st);
    put(&pp.n_cells, sizeof pp.n_cells);
    put(&pp.batch, sizeof pp.batch);
    return k;
  };
  // continue from the previous run's state when nothing else used the handle
  // since, the geometry and buffers are unchanged and the caller's positions
  // and species are the ones that run returned (checked on the device)
  bool cont = false;
  if (!npt && h->md_cont_call + 1 == h->api_calls && h->md_cont_key == state_key()) {
    int32_t* differs = h->flags + kFlagGuard;  // free until the chunks start
    launch_fill_i32(differs, 1, 0, s);
    launch_same_state(h->ext_id, N, h->pos, h->types, d_pos, d_types, differs, s);
    const int32_t* fl = read_flags(h, s);
    cont = fl[kFlagGuard] == 0;
  }
  h->md_cont_key.clear();
  if (cont) {
    // velocities into the internal order; order, rows and forces are kept
    launch_permute_md(h->ext_id, N, d_pos, d_vel, h->pos2, h->vel, s);  // pos2 is scratch here
    ++h->md_continued;
  }
  // initial order from the caller arrays
  if (!cont) {
    BuildArgs b0 = build_args(h, pp, d_pos, d_types, h->pos, h->types);
    launch_order_atoms(b0, s);
    launch_permute_md(h->perm, N, d_pos, d_vel, h->pos2, h->vel, s);
    HIPCHK(hipMemcpyAsync(h->ext_id, h->perm, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    launch_fill_i32(h->flags, 8, 0, s);
    launch_check_types(h->types, N, h->M.T, h->flags + 3, s);
    launch_check_finite(h->pos, 3 * N, h->flags + 4, s);
  }
  for (int attempt = 0; !cont; ++attempt) {
    launch_fill_i32(h->flags, 3, 0, s);
    launch_fill_i32(h->flags + 5, 1, 0, s);
    skin_rebuild(h, pp, rl, nullptr, s, mu_cum);
    skin_filter(h, pp, s);
    launch_fill_i32(h->flags + 6, 1, 0, s);
    launch_check_rows(N, h->sid, h->structs, pp.geo.st, pp.batch, h->L, h->flags + 6, s);
    const int32_t* fl = read_flags(h, s);
    if (fl[3]) throw Failure{NEP_E_INVALID_ARG, "an atom type is out of range"};
    if (fl[4]) throw Failure{NEP_E_NONFINITE, "positions contain NaN or Inf"};
    if (!grow_rows(h, N, fl)) {
      if (fl[2]) throw Failure{NEP_E_HIP, "internal error: neighbour rows are not symmetric"};
      check_row_flag(fl[6]);
      break;
    }
    if (attempt == 3) throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "neighbour rows kept overflowing"};
  }
  if (!cont) forces(h, pp, s);
  MDArgs md{};
  md.N = N;
  md.F = h->F;
  md.inv_mass = h->inv_mass;
  md.dt = dt;
  md.pos = h->pos;
  md.vel = h->vel;
  md.types = h->types;
  // one MD step with a device-decided rebuild (a fixed kernel sequence); in
  // an ensemble run the thermostat and barostat kernels around it follow the
  // order of the ensembles' publications (see nep.h), and `row` writes the
  // step's thermo row before the barostat acts
  // chain: this step checks for a rebuild (looking `ahead` fs further ahead)
  // and rebuilds the rows when needed; otherwise it only verifies that every
  // atom is still within half the skin of its reference position (a sticky
  // flag read at the end of the chunk, which is then replayed step by step)
  auto step_body = [&](hipStream_t cs, bool virial, bool row, bool chain, double ahead) {
    if (ens) {
      Stage st(h, "ensemble", cs);
      launch_ens_step_begin(est, cs);
      if (ep->kind == kEnsNHC) {
        launch_ens_kinetic(h->vel, h->types, h->mass, N, kAmuA2fs2, h->ens_partial, est, cs);
        launch_ens_thermostat(h->vel, N, *ep, est, h->ens_partial, cs);
      } else if (ep->kind == kEnsLangevin) {
        launch_ens_langevin(h->vel, h->types, h->mass, h->ext_id, N, *ep, 1u, est, h->ens_partial, cs);
      }
    }
    {
      Stage st(h, "integrate", cs);
      MDArgs drift = md;
      if (!chain) {  // the skin guard, on the new positions
        drift.ref = h->pos_ref;
        drift.flag = h->flags + kFlagGuard;
        drift.thr2 = thr2;
        drift.mu_cum = mu_cum;
        drift.rc = h->hp.rc_radial;
        drift.rl = rl;
      }
      launch_kick_drift(drift, cs);
    }
    if (chain) {
      Stage st(h, "order_atoms", cs);
      launch_fill_i32(gate, 1, 0, cs);
      launch_check_displacement(h->pos, h->pos_ref, h->vel, N, thr2, ahead, gate, cs, mu_cum,
                                h->hp.rc_radial, rl);
      skin_rebuild(h, pp, rl, gate, cs, mu_cum);
    }
    {
      Stage st(h, "neighbor_rows", cs);
      skin_filter(h, pp, cs);
    }
    forces(h, pp, cs, nullptr, virial || npt, &md);  // the gather applies the second half kick
    if (ens) {
      Stage st(h, "ensemble", cs);
      launch_ens_kinetic(h->vel, h->types, h->mass, N, kAmuA2fs2, h->ens_partial, est, cs);
      if (ep->kind == kEnsLangevin)
        launch_ens_langevin(h->vel, h->types, h->mass, h->ext_id, N, *ep, 2u, est, h->ens_partial, cs);
      else
        launch_ens_thermostat(h->vel, N, *ep, est, h->ens_partial, cs);
      if (row || npt) {
        launch_thermo(h->U, h->W, h->vel, h->types, h->mass, N, h->partial, num_partials(N), est->row, 0.0,
                      kAmuA2fs2, kBoltzmann, cs);
        launch_ens_pressure_row(*ep, est, h->structs, h->thermo, h->row_counter, row, step_base, cs);
      }
      if (npt) launch_ens_barostat(h->pos, h->vel, N, *ep, est, h->structs, cs);
    }
  };
  // Replay groups of G steps (+ their thermo row) from a captured HIP graph;
  // per-stage event timing (nep_set_timing) uses direct launches instead.
  const int64_t G = thermo_every > 0 ? thermo_every : 10;
  const char* genv = std::getenv("NEP_MD_GRAPH");
  // (captured even for a call shorter than G steps, so that a warm-up call
  // leaves the graph ready for the calls after it)
  const bool use_graph = !h->timing && !(genv && genv[0] == '0') && G <= 1000;
  // look-ahead of a group's rebuild check, in units of the group's remaining
  // time (NEP_MD_LOOKAHEAD overrides it; 0 checks the displacement alone)
  double lookahead = kRebuildLookahead;
  if (const char* e = std::getenv("NEP_MD_LOOKAHEAD")) lookahead = std::max(0.0, std::atof(e));
  if (!h->row_counter) dev_alloc(h->row_counter, 1);
  hipStream_t gs = s;
  // What the captured kernels' arguments depend on besides the handle's
  // fixed model and kernel shapes: sizes, geometry, step, skin and the
  // addresses of every buffer (the allocation generation).
  auto graph_key = [&]() {
    std::vector<unsigned char> k;
    auto put = [&](const void* p, size_t n) {
      const unsigned char* c = (const unsigned char*)p;
      k.insert(k.end(), c, c + n);
    };
    const uint64_t gen = g_alloc_gen.load();
    put(&gen, sizeof gen);
    put(&N, sizeof N);
    put(&G, sizeof G);
    put(&thermo_every, sizeof thermo_every);
    put(&dt, sizeof dt);
    put(&rl, sizeof rl);
    put(&thr2, sizeof thr2);
    put(&lookahead, sizeof lookahead);
    put(&pp.geo.st, sizeof pp.geo.st);
    put(&pp.n_cells, sizeof pp.n_cells);
    put(&pp.batch, sizeof pp.batch);
    const int32_t kind = ens ? ep->kind : -1;
    put(&kind, sizeof kind);
    if (ens) put(ep, sizeof *ep);
    return k;
  };
  // (Re)capture the G-step group; kept in the handle for later calls.
  auto capture = [&]() {
    h->drop_md_graph();
    HIPCHK(hipStreamSynchronize(gs));
    try {
      HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      for (int64_t k = 0; k < G; ++k) {
        const bool last_row = thermo_every > 0 && k == G - 1;
        step_body(gs, last_row, last_row, k == 0, lookahead * (double)(G - 1) * dt);
      }
      if (thermo_every > 0 && !ens)
        launch_thermo_counted(h->U, h->W, h->vel, h->types, h->mass, N, h->partial, num_partials(N),
                              h->thermo, h->row_counter, (double)thermo_every, kAmuA2fs2, kBoltzmann, gs);
      HIPCHK(hipStreamEndCapture(gs, &h->md_graph));
      HIPCHK(hipGraphInstantiate(&h->md_exec, h->md_graph, nullptr, nullptr, 0));
      h->md_key = graph_key();
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(gs, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      h->drop_md_graph();
      throw;
    }
  };
  if (use_graph) {
    if (!gs) {
      if (!h->md_stream) HIPCHK(hipStreamCreateWithFlags(&h->md_stream, hipStreamNonBlocking));
      gs = h->md_stream;
      HIPCHK(hipStreamSynchronize(s));
    }
    if (!h->md_exec || h->md_key != graph_key()) capture();
  }
  hipStream_t ws = use_graph ? gs : s;   // the stream every step runs on
  const int64_t chunk = use_graph ? G * std::max<int64_t>(1, 50 / G) : 50;
  int64_t row = 0;
  bool redo = false, replay = false;
  for (int64_t c0 = 0; c0 < n_steps;) {
    const int64_t c1 = std::min(n_steps, c0 + chunk);
    s = ws;
    HIPCHK(hipMemcpyAsync(h->pos_save, h->pos, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->vel_save, h->vel, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->ref_save, h->pos_ref, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_save, h->types, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->ext_save, h->ext_id, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->F_save, h->F, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, s));
    unsigned char* ens_base = (unsigned char*)h->ens_state;
    if (ens) {
      HIPCHK(hipMemcpyAsync(ens_base + 512, est, sizeof(EnsState), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(ens_base + 1024, h->structs, sizeof(StructInfo), hipMemcpyDeviceToDevice, s));
    }
    const int64_t row0 = row;
    launch_fill_i32(h->flags, kFlagsReset, 0, s);
    if (redo) {
      // rows were grown or the chunk is replayed: rebuild them for the
      // restored state, which re-sorts the atoms, so the forces the first
      // half kick uses are evaluated again in the new order
      skin_rebuild(h, pp, rl, nullptr, s, mu_cum);
      skin_filter(h, pp, s);
      forces(h, pp, s);
      redo = false;
    }
    if (use_graph || ens) {
      int32_t* rc = (int32_t*)(h->pinned + 416);
      *rc = (int32_t)row;
      HIPCHK(hipMemcpyAsync(h->row_counter, rc, sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    int64_t group_steps = 0;
    for (int64_t step = c0 + 1; step <= c1; ++step) {
      if (use_graph && !replay && (step - 1) % G == 0 && step - 1 + G <= c1) {
        HIPCHK(hipGraphLaunch(h->md_exec, s));
        if (thermo_every > 0) ++row;
        step += G - 1;
        group_steps += G;
        continue;
      }
      const bool row_due = thermo_every > 0 && step % thermo_every == 0;
      step_body(s, row_due, row_due, true, 0.0);
      if (ens && row_due) {
        ++row;
      } else if (row_due) {
        Stage st(h, "thermo", s);
        launch_thermo(h->U, h->W, h->vel, h->types, h->mass, N, h->partial, num_partials(N),
                      h->thermo + 13 * row, (double)step, kAmuA2fs2, kBoltzmann, s);
        ++row;
      }
    }
    launch_check_finite(h->pos, 3 * N, h->flags + 4, s);
    launch_check_rows(N, h->sid, h->structs, pp.geo.st, pp.batch, h->L, h->flags + 6, s);
    if (npt)  // the current cell, read with the flags
      HIPCHK(hipMemcpyAsync(h->pinned + 1536, h->structs, sizeof(StructInfo), hipMemcpyDeviceToHost, s));
    const int32_t* fl = read_flags(h, s);
    if (fl[4]) throw Failure{NEP_E_NONFINITE, "positions became non-finite during the run"};
    if (npt) check_npt_cell(*(const StructInfo*)(h->pinned + 1536), pp.geo.st, rl);
    const bool grown = grow_rows(h, N, fl);
    if (grown || fl[kFlagGuard]) {
      // rows overflowed, or an atom left the skin between two rebuild checks
      // of a captured group: restore the chunk's start and run it again
      // (with grown rows; a replay checks for a rebuild at every step)
      if (!grown) {
        replay = true;
        ++h->md_replays;
      }
      if (ens) {
        HIPCHK(hipMemcpyAsync(est, ens_base + 512, sizeof(EnsState), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(h->structs, ens_base + 1024, sizeof(StructInfo), hipMemcpyDeviceToDevice, s));
      }
      HIPCHK(hipMemcpyAsync(h->pos, h->pos_save, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->vel, h->vel_save, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->pos_ref, h->ref_save, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->types, h->types_save, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->ext_id, h->ext_save, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->F, h->F_save, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, s));
      row = row0;
      redo = true;
      if (use_graph && grown) capture();  // the grown rows live at new addresses
      continue;
    }
    if (fl[2]) throw Failure{NEP_E_HIP, "internal error: neighbour rows are not symmetric"};
    check_row_flag(fl[6]);
    h->md_group_steps += group_steps;
    h->md_rebuilds = rebuilds0 + fl[kFlagRebuilds];
    replay = false;
    c0 = c1;
  }
  launch_unpermute_md(h->ext_id, N, h->pos, h->vel, d_pos, d_vel, s);
  if (n_rows > 0)
    HIPCHK(hipMemcpyAsync(thermo_out, h->thermo, row_len * n_rows * sizeof(double),
                          thermo_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  if (ens) {
    HIPCHK(hipMemcpyAsync(h->pinned + 1024, est, sizeof(EnsState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h->pinned + 1536, h->structs, sizeof(StructInfo), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (ens) {
    const EnsState& e = *(const EnsState*)(h->pinned + 1024);
    ens_state[0] = (double)e.step;
    ens_state[1] = e.heat;
    for (int k = 0; k < kMaxChain; ++k) {
      ens_state[2 + k] = e.xi[k];
      ens_state[10 + k] = e.vxi[k];
    }
    if (box_out) std::memcpy(box_out, ((const StructInfo*)(h->pinned + 1536))->H, 9 * sizeof(double));
  }
  if (!npt) {
    h->md_cont_key = state_key();
    h->md_cont_call = h->api_calls.load();
  }
  return NEP_OK;
}

}  // namespace

static int md_impl(nep_handle* h, int64_t N, double* d_pos, double* d_vel, const int32_t* d_types,
                   const double* mass_per_type, const double* box, const int32_t* pbc, double dt,
                   int64_t n_steps, int64_t thermo_every, double* thermo_out, bool thermo_on_host,
                   hipStream_t s, const nep_ensemble* ens = nullptr, double* ens_state = nullptr,
                   double* box_out = nullptr) {
  if (!mass_per_type) throw Failure{NEP_E_INVALID_ARG, "mass_per_type is required"};
  for (int t = 0; t < h->hp.n_types; ++t)
    if (!(mass_per_type[t] > 0) || !std::isfinite(mass_per_type[t]))
      throw Failure{NEP_E_INVALID_ARG, "masses must be positive"};
  if (!(dt > 0) || !std::isfinite(dt)) throw Failure{NEP_E_INVALID_ARG, "dt must be positive"};
  if (n_steps < 0 || thermo_every < 0) throw Failure{NEP_E_INVALID_ARG, "negative step counts"};
  const int64_t n_rows = thermo_every > 0 ? n_steps / thermo_every : 0;
  if (n_rows > 0 && !thermo_out) throw Failure{NEP_E_INVALID_ARG, "thermo buffer is required"};
  const bool use_ens = ens != nullptr;  // NEP_ENS_NVE here: plain steps with the 16-column rows
  EnsParams ep{};
  if (use_ens) {
    if (ens->kind < 0 || ens->kind > NEP_ENS_NPT_SCR) throw Failure{NEP_E_INVALID_ARG, "unknown ensemble"};
    if (N < 2) throw Failure{NEP_E_INVALID_ARG, "an ensemble run needs at least 2 atoms"};
    if (ens->kind != NEP_ENS_NVE &&
        (!(ens->temperature > 0) || !(ens->tau_t > 0) || !std::isfinite(ens->temperature) ||
         !std::isfinite(ens->tau_t)))
      throw Failure{NEP_E_INVALID_ARG, "temperature and tau_t must be positive"};
    if (ens->kind == NEP_ENS_NHC && (ens->nhc_length < 1 || ens->nhc_length > kMaxChain))
      throw Failure{NEP_E_INVALID_ARG, "nhc_length must be in [1, 8]"};
    if (ens->kind >= NEP_ENS_NPT_BERENDSEN &&
        (!(ens->tau_p > 0) || !(ens->compressibility > 0) || !std::isfinite(ens->pressure) ||
         !std::isfinite(ens->tau_p) || !std::isfinite(ens->compressibility)))
      throw Failure{NEP_E_INVALID_ARG, "NPT needs a finite pressure and positive tau_p and compressibility"};
    if (!ens_state) throw Failure{NEP_E_INVALID_ARG, "state is required"};
    ep.kind = ens->kind;
    ep.nhc_length = ens->nhc_length;
    ep.T0 = ens->temperature;
    ep.tau_t = ens->tau_t;
    ep.P0 = ens->pressure;
    ep.tau_p = ens->tau_p;
    ep.beta = ens->compressibility;
    ep.dt = dt;
    ep.kB = kBoltzmann;
    ep.kT = kBoltzmann * ens->temperature;
    ep.Nf = 3.0 * (double)N - 3.0;
    ep.conv = kAmuA2fs2;
    ep.seed = ens->seed;
  }
  const bool npt = use_ens && ens->kind >= NEP_ENS_NPT_BERENDSEN;
  const bool with_skin = h->hp.skin > 0 || use_ens;
  // NPT: the box lives on the device (batch-mode kernels read it there), and
  // the cell grid gets 3 % headroom for a box that shrinks during the call
  Prepared pp;
  if (npt) {
    const int64_t offs[2] = {0, N};
    pp = prepare_batch(h, 1, offs, box, pbc, (h->hp.rc_radial + h->hp.skin) * 1.03, true, true, s);
  } else {
    pp = prepare(h, N, box, pbc, h->hp.rc_radial + h->hp.skin, true, s);
  }
  // rows for 4096 reports at least, allocated by the first call even when it
  // reports none: a later call of a few more rows then keeps the buffer (and
  // with it the captured step group and the state it may continue from)
  if (n_rows > h->thermo_cap || !h->thermo) {
    const int64_t cap = std::max<int64_t>(n_rows, 4096);
    dev_alloc(h->thermo, 16 * cap);
    h->thermo_cap = cap;
  }
  double m[kMaxTypes] = {0}, im[kMaxTypes] = {0};
  for (int t = 0; t < h->hp.n_types; ++t) {
    m[t] = mass_per_type[t];
    im[t] = 1.0 / (mass_per_type[t] * kAmuA2fs2);
  }
  std::memcpy(h->pinned + 256, m, sizeof m);
  std::memcpy(h->pinned + 320, im, sizeof im);
  HIPCHK(hipMemcpyAsync(h->mass, h->pinned + 256, sizeof m, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->inv_mass, h->pinned + 320, sizeof im, hipMemcpyHostToDevice, s));
  if (with_skin)
    return md_skin(h, pp, d_pos, d_vel, d_types, dt, n_steps, thermo_every, thermo_out, thermo_on_host,
                   n_rows, s, use_ens ? &ep : nullptr, ens_state, box_out);
  // initial order: internal <- caller, velocities follow
  order_and_build(h, pp, d_pos, d_types, s, true);
  launch_permute_md(h->perm, N, d_pos, d_vel, h->pos2, h->vel, s);  // pos2 is scratch here
  HIPCHK(hipMemcpyAsync(h->ext_id, h->perm, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  forces(h, pp, s);

  MDArgs md{};
  md.N = N;
  md.F = h->F;
  md.inv_mass = h->inv_mass;
  md.dt = dt;
  const int64_t chunk = 50;
  int64_t row = 0;
  for (int64_t c0 = 0; c0 < n_steps;) {
    const int64_t c1 = std::min(n_steps, c0 + chunk);
    // state at the chunk start, restored if a row overflows inside the chunk
    HIPCHK(hipMemcpyAsync(h->pos_save, h->pos, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->vel_save, h->vel, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_save, h->types, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->ext_save, h->ext_id, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(h->F_save, h->F, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, s));
    const int64_t row0 = row;
    launch_fill_i32(h->flags, 8, 0, s);
    for (int64_t step = c0 + 1; step <= c1; ++step) {
      md.pos = h->pos;
      md.vel = h->vel;
      md.types = h->types;
      {
        Stage st(h, "integrate", s);
        launch_kick_drift(md, s);
      }
      // re-sort into cell order and rebuild the rows at the new positions
      BuildArgs b = build_args(h, pp, h->pos, h->types, h->pos2, h->types2);
      b.ext_src = h->ext_id;
      {
        Stage st(h, "order_atoms", s);
        launch_order_atoms(b, s);
        launch_permute_md(h->perm, N, h->pos, h->vel, h->pos2, h->vel2, s);
        launch_type_rows(h->types2, N, h->M.T, h->hp.nn_per_type, h->tblk, h->tex, h->toff, h->rows,
                         rows_length(N, h->M.T), nullptr, s);
      }
      std::swap(h->pos, h->pos2);
      std::swap(h->vel, h->vel2);
      std::swap(h->types, h->types2);
      // caller index of every atom in the new order: ext_id2[k] = ext_id[perm[k]]
      {
        Stage st(h, "order_atoms", s);
        launch_gather_i32(h->perm, N, h->ext_id, h->ext_id2, s);
      }
      std::swap(h->ext_id, h->ext_id2);
      {
        Stage st(h, "neighbor_rows", s);
        BuildArgs b2 = build_args(h, pp, nullptr, nullptr, h->pos, h->types);
        launch_build_rows(b2, pp.geo.st, pp.batch, h->V, h->L, s);
      }
      forces(h, pp, s, nullptr, thermo_every > 0 && step % thermo_every == 0);
      md.pos = h->pos;
      md.vel = h->vel;
      md.types = h->types;
      {
        Stage st(h, "integrate", s);
        launch_kick(md, s);
      }
      if (thermo_every > 0 && step % thermo_every == 0) {
        Stage st(h, "thermo", s);
        launch_thermo(h->U, h->W, h->vel, h->types, h->mass, N, h->partial, num_partials(N),
                      h->thermo + 13 * row, (double)step, kAmuA2fs2, kBoltzmann, s);
        ++row;
      }
    }
    launch_check_finite(h->pos, 3 * N, h->flags + 4, s);
    launch_check_rows(N, h->sid, h->structs, pp.geo.st, pp.batch, h->L, h->flags + 6, s);
    int32_t* fl = (int32_t*)(h->pinned + kPinFlags);
    HIPCHK(hipMemcpyAsync(fl, h->flags, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (fl[4]) throw Failure{NEP_E_NONFINITE, "positions became non-finite during the run"};
    fl[0] = std::max(fl[0], fl[5]);  // candidate rows at r_c^R: the same count
    if (fl[2] && !(fl[0] || fl[1]))
      throw Failure{NEP_E_HIP, "internal error: neighbour rows are not symmetric"};
    if (!(fl[0] || fl[1])) check_row_flag(fl[6]);
    if (fl[0] || fl[1]) {
      if (h->hp.max_nb_radial || h->hp.max_nb_angular)
        throw Failure{NEP_E_NEIGHBOR_OVERFLOW, "neighbour row overflow during the run"};
      const int32_t MR = std::max(h->MR, (int32_t)((fl[0] * 1.2 + 8) / 4 * 4 + 4));
      const int32_t MA = std::max(h->MA, (int32_t)((fl[1] * 1.2 + 8) / 4 * 4 + 4));
      ensure_lists(h, N, MR, MA);
      ensure_verlet(h, N, std::max(h->V.MR, MR));
      HIPCHK(hipMemcpyAsync(h->pos, h->pos_save, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->vel, h->vel_save, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->types, h->types_save, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->ext_id, h->ext_save, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(h->F, h->F_save, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, s));
      row = row0;
      continue;  // redo the chunk with larger rows
    }
    c0 = c1;
  }
  launch_unpermute_md(h->ext_id, N, h->pos, h->vel, d_pos, d_vel, s);
  if (n_rows > 0)
    HIPCHK(hipMemcpyAsync(thermo_out, h->thermo, 13 * n_rows * sizeof(double),
                          thermo_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return NEP_OK;
}

int nep_md_run(nep_handle* h, int64_t N, double* pos, double* vel, const int32_t* types,
               const double* mass_per_type, const double box[9], const int32_t pbc[3], double dt_fs,
               int64_t n_steps, int64_t thermo_every, double* thermo) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !vel || !types || !box) return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    check_host_finite(3 * N, vel, "velocities");
    hipStream_t s = nullptr;
    prepare(h, N, box, pbc, h->hp.rc_radial, true, s);
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->vel_ext, vel, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    md_impl(h, N, h->pos_ext, h->vel_ext, h->types_ext, mass_per_type, box, pbc, dt_fs, n_steps, thermo_every,
            thermo, true, s);
    HIPCHK(hipMemcpy(pos, h->pos_ext, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(vel, h->vel_ext, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_md_run_dev(nep_handle* h, int64_t N, double* pos, double* vel, const int32_t* types,
                   const double* mass_per_type, const double box[9], const int32_t pbc[3], double dt_fs,
                   int64_t n_steps, int64_t thermo_every, double* thermo, void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !vel || !types || !box) return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  try {
    set_device(h);
    md_impl(h, N, pos, vel, types, mass_per_type, box, pbc, dt_fs, n_steps, thermo_every, thermo, false,
            (hipStream_t)stream);
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_md_run_ensemble(nep_handle* h, int64_t N, double* pos, double* vel, const int32_t* types,
                        const double* mass_per_type, double box[9], const int32_t pbc[3], double dt_fs,
                        int64_t n_steps, int64_t thermo_every, double* thermo, const nep_ensemble* ens,
                        double state[20]) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !vel || !types || !box || !ens || !state) return fail(h, {NEP_E_INVALID_ARG, "bad arguments"});
  try {
    set_device(h);
    if (N < 1) throw Failure{NEP_E_INVALID_ARG, "n_atoms must be >= 1"};
    check_host_types(h, N, types);
    check_host_finite(3 * N, pos, "positions");
    check_host_finite(3 * N, vel, "velocities");
    if (!(state[0] >= 0) || state[0] > 4294967295.0 || state[0] != std::floor(state[0]))
      throw Failure{NEP_E_INVALID_ARG, "state[0] (steps done) must be a whole number in [0, 2^32)"};
    hipStream_t s = nullptr;
    prepare(h, N, box, pbc, h->hp.rc_radial, true, s);
    HIPCHK(hipMemcpyAsync(h->pos_ext, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->vel_ext, vel, 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->types_ext, types, N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    double box_new[9];
    std::memcpy(box_new, box, sizeof box_new);
    md_impl(h, N, h->pos_ext, h->vel_ext, h->types_ext, mass_per_type, box, pbc, dt_fs, n_steps, thermo_every,
            thermo, true, s, ens, state, box_new);
    HIPCHK(hipMemcpy(pos, h->pos_ext, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(vel, h->vel_ext, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
    std::memcpy(box, box_new, sizeof box_new);
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_compute_batch(nep_handle* h, int32_t n_struct, const int64_t* offsets, const double* pos,
                      const int32_t* types, const double* boxes, const int32_t* pbc, int32_t n_param_sets,
                      const double* params, double* energy, double* force, double* virial, double* totals,
                      void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types) return fail(h, {NEP_E_INVALID_ARG, "pos and types are required"});
  try {
    set_device(h);
    batch_impl(h, n_struct, offsets, pos, types, boxes, pbc, n_param_sets, params, nullptr, 0, energy, force,
               virial, totals, (hipStream_t)stream);
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_compute_batch_dev(nep_handle* h, int32_t n_struct, const int64_t* offsets, const double* pos,
                          const int32_t* types, const double* boxes, const int32_t* pbc, int32_t n_param_sets,
                          const double* params, int32_t flags, double* energy, double* force, double* virial,
                          double* totals, void* stream) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  if (!pos || !types || !params) return fail(h, {NEP_E_INVALID_ARG, "pos, types and params are required"});
  if (flags & ~NEP_BATCH_REUSE_ROWS) return fail(h, {NEP_E_INVALID_ARG, "unknown flags"});
  try {
    set_device(h);
    batch_impl(h, n_struct, offsets, pos, types, boxes, pbc, n_param_sets, nullptr, params, flags, energy, force,
               virial, totals, (hipStream_t)stream);
    if (h->timing) h->resolve_timing();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_set_timing(nep_handle* h, int32_t enable) {
  if (!h) return fail(nullptr, {NEP_E_INVALID_ARG, "handle is NULL"});
  h->timing = enable != 0;
  h->times = StageTimes{};
  return NEP_OK;
}

int nep_get_timing(const nep_handle* h, int32_t max, const char** names, double* ms, int64_t* calls) {
  if (!h || max < 0) return 0;
  const int n = std::min<int>(max, (int)h->times.names.size());
  for (int k = 0; k < n; ++k) {
    if (names) names[k] = h->times.names[k];
    if (ms) ms[k] = h->times.ms[k];
    if (calls) calls[k] = h->times.calls[k];
  }
  return n;
}

int nep_get_tuning(const nep_handle* h, int32_t batch, int32_t out[7]) {
  if (!h || !out || (batch != 0 && batch != 1))
    return fail(nullptr, {NEP_E_INVALID_ARG, "handle, batch in {0, 1} and out[7] are required"});
  const Tuning& t = h->tune[batch];
  const int32_t v[7] = {t.NG_desc, t.block_desc, t.lanes_desc, t.NG_force, t.block_force,
                        t.lanes_force, t.lanes_gather};
  for (int k = 0; k < 7; ++k) out[k] = t.done ? v[k] : 0;
  return NEP_OK;
}

int nep_md_counters(const nep_handle* h, int64_t out[4]) {
  if (!h || !out) return fail(nullptr, {NEP_E_INVALID_ARG, "handle and out[4] are required"});
  out[0] = h->md_group_steps;
  out[1] = h->md_replays;
  out[2] = h->md_rebuilds;
  out[3] = h->md_continued;
  return NEP_OK;
}

int nep_server_create(nep_handle* h, size_t hbm_budget_bytes, int32_t max_slots, nep_server** out) {
  if (!h || !out) return fail(h, {NEP_E_INVALID_ARG, "handle and out are required"});
  if (max_slots < 1 || hbm_budget_bytes == 0) return fail(h, {NEP_E_INVALID_ARG, "need max_slots >= 1 and a budget"});
  *out = nullptr;
  nep_server* sv = new nep_server();
  try {
    set_device(h);
    sv->h = h;
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    HIPCHK(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
    sv->worker = std::thread(server_loop, sv);
  } catch (const Failure& f) {
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
    return fail(h, f);
  }
  *out = sv;
  return NEP_OK;
}

int nep_server_submit(nep_server* sv, const nep_request* rq, uint64_t* ticket) {
  if (!sv || !rq || !ticket) return fail(nullptr, {NEP_E_INVALID_ARG, "server, request and ticket are required"});
  nep_handle* h = sv->h;
  try {
    if (rq->kind != NEP_REQ_EVAL && rq->kind != NEP_REQ_MD) throw Failure{NEP_E_INVALID_ARG, "unknown request kind"};
    if (rq->n_atoms < 1 || !rq->pos || !rq->types) throw Failure{NEP_E_INVALID_ARG, "bad request arrays"};
    if (rq->kind == NEP_REQ_MD && (!rq->vel || !rq->mass_per_type || rq->n_steps < 0 || !(rq->dt_fs > 0)))
      throw Failure{NEP_E_INVALID_ARG, "an MD request needs vel, masses, n_steps >= 0 and dt > 0"};
    const int64_t n = rq->n_atoms;
    check_host_types(h, n, rq->types);
    check_host_finite(3 * n, rq->pos, "positions");
    Geometry g = make_geometry(rq->box, rq->pbc, n, h->hp.rc_radial);
    auto r = std::make_shared<ServerReq>();
    r->kind = rq->kind;
    r->n = n;
    r->pos.assign(rq->pos, rq->pos + 3 * n);
    r->types.assign(rq->types, rq->types + n);
    if (rq->kind == NEP_REQ_MD) {
      check_host_finite(3 * n, rq->vel, "velocities");
      r->vel.assign(rq->vel, rq->vel + 3 * n);
      r->mass.assign(rq->mass_per_type, rq->mass_per_type + h->hp.n_types);
      for (double m : r->mass)
        if (!(m > 0)) throw Failure{NEP_E_INVALID_ARG, "masses must be positive"};
      r->n_steps = rq->n_steps;
      r->dt = rq->dt_fs;
    }
    std::memcpy(r->box, rq->box, sizeof r->box);
    for (int k = 0; k < 3; ++k) r->pbc[k] = g.st.pbc[k];
    r->bytes = request_bytes(h, n, (double)n / g.volume);
    if (r->bytes > sv->budget) throw Failure{NEP_E_BUDGET, "request needs more device memory than the budget"};
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->fatal.empty()) throw Failure{NEP_E_HIP, "server stopped: " + sv->fatal};
    r->ticket = sv->next_ticket++;
    r->t_submit = now_s();
    if (sv->t_first < 0) sv->t_first = r->t_submit;
    sv->submitted += 1;
    sv->queue.push_back(r);
    *ticket = r->ticket;
    sv->cv.notify_one();
  } catch (const Failure& f) {
    return fail(h, f);
  }
  return NEP_OK;
}

int nep_server_poll(nep_server* sv, uint64_t ticket, int32_t wait_ms, nep_result* out) {
  if (!sv || !out) return fail(nullptr, {NEP_E_INVALID_ARG, "server and out are required"});
  std::shared_ptr<ServerReq> r;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return sv->done.count(ticket) > 0; };
    if (!ready() && wait_ms != 0) {
      if (wait_ms < 0) sv->done_cv.wait(lk, ready);
      else sv->done_cv.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    }
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) return NEP_PENDING;
    r = it->second;
    sv->done.erase(it);
  }
  out->status = r->status;
  out->n_atoms = r->n;
  out->latency_ms = (r->t_done - r->t_submit) * 1e3;
  out->queue_ms = r->t_admit > 0 ? (r->t_admit - r->t_submit) * 1e3 : out->latency_ms;
  std::memcpy(out->totals, r->totals, sizeof r->totals);
  if (r->status != NEP_OK) return fail(sv->h, {r->status, r->error});
  const size_t n = r->n;
  if (out->energy) std::memcpy(out->energy, r->energy.data(), n * sizeof(double));
  if (out->force) std::memcpy(out->force, r->force.data(), 3 * n * sizeof(double));
  if (out->virial) std::memcpy(out->virial, r->virial.data(), 9 * n * sizeof(double));
  if (out->pos && !r->out_pos.empty()) std::memcpy(out->pos, r->out_pos.data(), 3 * n * sizeof(double));
  if (out->vel && !r->out_vel.empty()) std::memcpy(out->vel, r->out_vel.data(), 3 * n * sizeof(double));
  return NEP_OK;
}

int nep_server_stats(nep_server* sv, nep_server_stats_t* out) {
  if (!sv || !out) return fail(nullptr, {NEP_E_INVALID_ARG, "server and out are required"});
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = sv->submitted;
  out->completed = sv->completed;
  out->active = (int64_t)sv->active.size();
  out->queued = (int64_t)sv->queue.size();
  out->ticks = sv->ticks;
  std::vector<double> l = sv->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    const double x = q * (l.size() - 1);
    const size_t a = (size_t)std::floor(x), b = std::min(l.size() - 1, a + 1);
    return (l[a] + (x - a) * (l[b] - l[a])) * 1e3;
  };
  out->p50_ms = pct(0.5);
  out->p99_ms = pct(0.99);
  out->max_ms = l.empty() ? 0 : l.back() * 1e3;
  double sum = 0;
  for (double v : l) sum += v;
  out->mean_ms = l.empty() ? 0 : sum / l.size() * 1e3;
  const double span = sv->t_first >= 0 ? sv->t_last - sv->t_first : 0;
  out->wall_s = span;
  out->busy_s = sv->busy;
  out->requests_per_s = span > 0 ? sv->completed / span : 0;
  out->atom_steps_per_s = span > 0 ? sv->atom_steps / span : 0;
  out->mean_batch_atoms = sv->ticks ? (double)sv->batch_atoms / sv->ticks : 0;
  out->mean_batch_requests = sv->ticks ? (double)sv->batch_reqs / sv->ticks : 0;
  out->bytes_in_use = sv->bytes_active;
  out->hbm_budget = sv->budget;
  return NEP_OK;
}

int nep_server_reset_stats(nep_server* sv) {
  if (!sv) return fail(nullptr, {NEP_E_INVALID_ARG, "server is NULL"});
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->latencies.clear();
  sv->completed = sv->submitted = sv->ticks = sv->atom_steps = sv->batch_atoms = sv->batch_reqs = 0;
  sv->t_first = -1;
  sv->t_last = 0;
  sv->busy = 0;
  return NEP_OK;
}

void nep_server_destroy(nep_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->h->device);
  sv->st.release();
  sv->st2.release();
  sv->release_staging();
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  delete sv;
}

}  // extern "C"
