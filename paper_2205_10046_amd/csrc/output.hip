// output.hip -- results back in the caller's atom order, and the float64
// totals E = sum_i U_i, W = sum_i W_i (a fixed two-level tree: the same
// inputs always give the same bits).
#include <algorithm>
#include <mutex>

#include "nep_kernels.h"

namespace nep {

__global__ void k_scatter_outputs(const float* __restrict__ U, const float* __restrict__ F,
                                  const float* __restrict__ W, int64_t N,
                                  const int32_t* __restrict__ perm, double* __restrict__ energy,
                                  double* __restrict__ force, double* __restrict__ virial) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int64_t e = perm[k];
  if (energy) energy[e] = (double)U[k];
  if (force)
    for (int c = 0; c < 3; ++c) force[(int64_t)c * N + e] = (double)F[(int64_t)c * N + k];
  if (virial)
    for (int v = 0; v < 9; ++v) virial[(int64_t)v * N + e] = (double)W[(int64_t)v * N + k];
}

void launch_scatter_outputs(const EvalArgs& a, const int32_t* perm, double* energy,
                            double* force, double* virial, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_outputs, dim3(div_up(a.N, kBlock)), dim3(kBlock), 0, s, a.U, a.F,
                     a.W, a.N, perm, energy, force, virial);
}

constexpr int kRedBlock = 256;
constexpr int64_t kTotalsChunk = 8192;  // atoms per block of the chunked structure totals

// Block b sums items [b*chunk, (b+1)*chunk) of the 10 quantities (U, W_0..8)
// in a fixed tree; partial[b][10].
__global__ void __launch_bounds__(kRedBlock) k_totals_partial(const float* __restrict__ U,
                                                              const float* __restrict__ W,
                                                              int64_t N, int64_t chunk,
                                                              double* __restrict__ partial) {
  __shared__ double sh[10][kRedBlock];
  const int t = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(N, lo + chunk);
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = lo + t; k < hi; k += kRedBlock) {
    acc[0] += (double)U[k];
    for (int v = 0; v < 9; ++v) acc[1 + v] += (double)W[(int64_t)v * N + k];
  }
  for (int v = 0; v < 10; ++v) sh[v][t] = acc[v];
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int v = 0; v < 10; ++v) sh[v][t] += sh[v][t + off];
    __syncthreads();
  }
  if (t < 10) partial[blockIdx.x * 10 + t] = sh[t][0];
}

__global__ void k_totals_final(const double* __restrict__ partial, int64_t n_part,
                               double* __restrict__ totals) {
  const int v = threadIdx.x;
  if (v >= 10) return;
  double s = 0.0;
  for (int64_t b = 0; b < n_part; ++b) s += partial[b * 10 + v];
  totals[v] = s;
}

void launch_totals(const float* U, const float* W, int64_t N, double* partial, int64_t n_part,
                   double* totals, hipStream_t s) {
  const int64_t chunk = (N + n_part - 1) / n_part;
  hipLaunchKernelGGL(k_totals_partial, dim3((unsigned)n_part), dim3(kRedBlock), 0, s, U, W, N,
                     chunk, partial);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, s, partial, n_part, totals);
}

// totals[s][10] of every structure s: one block per structure, fixed tree
__global__ void __launch_bounds__(kRedBlock) k_struct_totals(const float* __restrict__ U,
                                                             const float* __restrict__ W, int64_t N,
                                                             const StructInfo* __restrict__ structs,
                                                             double* __restrict__ totals) {
  __shared__ double sh[10][kRedBlock];
  const int t = threadIdx.x;
  const StructInfo& st = structs[blockIdx.x];
  const int64_t lo = st.start, hi = st.start + st.count;
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = lo + t; k < hi; k += kRedBlock) {
    acc[0] += (double)U[k];
    for (int v = 0; v < 9; ++v) acc[1 + v] += (double)W[(int64_t)v * N + k];
  }
  for (int v = 0; v < 10; ++v) sh[v][t] = acc[v];
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int v = 0; v < 10; ++v) sh[v][t] += sh[v][t + off];
    __syncthreads();
  }
  if (t < 10) totals[(int64_t)blockIdx.x * 10 + t] = sh[t][0];
}

void launch_struct_totals(const float* U, const float* W, int64_t N, const StructInfo* structs,
                          int32_t n_struct, double* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_struct_totals, dim3((unsigned)n_struct), dim3(kRedBlock), 0, s, U, W, N,
                     structs, totals);
}

// The same totals for structures of any size, in two fixed-order levels:
// block (c, s) reduces chunk c of structure s (C atoms from its start) with
// the block tree into partial[s][c][10] (zeros past the structure's end),
// then the chunk sums of a structure are added in chunk order.
__global__ void __launch_bounds__(kRedBlock) k_struct_totals_chunks(const float* __restrict__ U,
                                                                    const float* __restrict__ W, int64_t N,
                                                                    const StructInfo* __restrict__ structs,
                                                                    int64_t C, int32_t n_chunk,
                                                                    double* __restrict__ partial) {
  __shared__ double sh[10][kRedBlock];
  const int t = threadIdx.x;
  const StructInfo& st = structs[blockIdx.y];
  const int64_t end = st.start + st.count;
  const int64_t lo = st.start + (int64_t)blockIdx.x * C, hi = min(end, lo + C);
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = lo + t; k < hi; k += kRedBlock) {
    acc[0] += (double)U[k];
    for (int v = 0; v < 9; ++v) acc[1 + v] += (double)W[(int64_t)v * N + k];
  }
  for (int v = 0; v < 10; ++v) sh[v][t] = acc[v];
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int v = 0; v < 10; ++v) sh[v][t] += sh[v][t + off];
    __syncthreads();
  }
  if (t < 10) partial[((int64_t)blockIdx.y * n_chunk + blockIdx.x) * 10 + t] = sh[t][0];
}

__global__ void k_struct_totals_final(const double* __restrict__ partial, int32_t n_struct, int32_t n_chunk,
                                      double* __restrict__ totals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // structure k / 10, column k % 10
  if (k >= (int64_t)n_struct * 10) return;
  const int64_t s = k / 10, v = k % 10;
  double acc = 0.0;
  for (int c = 0; c < n_chunk; ++c) acc += partial[(s * n_chunk + c) * 10 + v];
  totals[k] = acc;
}

void launch_struct_totals_chunked(const float* U, const float* W, int64_t N, const StructInfo* structs,
                                  int32_t n_struct, int64_t max_count, double* work, int64_t work_cap,
                                  double* totals, hipStream_t s) {
  int64_t n_chunk = std::max<int64_t>(1, (max_count + kTotalsChunk - 1) / kTotalsChunk);
  n_chunk = std::min<int64_t>(n_chunk, work_cap / (10 * (int64_t)n_struct));
  if (n_chunk <= 1) {
    launch_struct_totals(U, W, N, structs, n_struct, totals, s);
    return;
  }
  const int64_t C = (max_count + n_chunk - 1) / n_chunk;
  hipLaunchKernelGGL(k_struct_totals_chunks, dim3((unsigned)n_chunk, (unsigned)n_struct), dim3(kRedBlock), 0, s,
                     U, W, N, structs, C, (int32_t)n_chunk, work);
  hipLaunchKernelGGL(k_struct_totals_final, dim3(div_up(10 * (int64_t)n_struct, kBlock)), dim3(kBlock), 0, s,
                     work, n_struct, (int32_t)n_chunk, totals);
}

__global__ void k_descriptors_out(const float* __restrict__ q, int64_t N, int NDp, int ND,
                                  const int32_t* __restrict__ perm, double* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int64_t e = perm[k];
  for (int d = 0; d < ND; ++d) out[e * ND + d] = (double)q[k * NDp + d];
}

void launch_descriptors_out(const float* q, int64_t N, int NDp, int ND, const int32_t* perm,
                            double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_descriptors_out, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, q, N, NDp,
                     ND, perm, out);
}

__global__ void k_inverse_perm(const int32_t* __restrict__ perm, int64_t N,
                               int32_t* __restrict__ inv) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) inv[perm[k]] = (int32_t)k;
}

void launch_inverse_perm(const int32_t* perm, int64_t N, int32_t* inv, hipStream_t s) {
  hipLaunchKernelGGL(k_inverse_perm, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, perm, N, inv);
}

// Neighbour rows in caller indices with absolute integer images n.  Output
// rows follow the internal order; the host sorts them by caller index.
__global__ void k_neighbors_out(Lists L, int which, int64_t N, const int32_t* __restrict__ perm,
                                const int32_t* __restrict__ inv, const double* __restrict__ pos,
                                const int32_t* __restrict__ sid,
                                const StructInfo* __restrict__ structs, int32_t cap,
                                int32_t* __restrict__ count, int32_t* __restrict__ nbr,
                                int32_t* __restrict__ shift) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const int64_t i = inv[e];
  const StructInfo& st = structs[sid[i]];
  // the angular row is the first nnA entries of the radial row
  const int32_t* nl = L.nlR;
  const uint16_t* cd = L.cdR;
  const int nn = min(which ? L.nnA[i] : L.nnR[i], L.MR);
  count[e] = nn;
  for (int m = 0; m < nn && m < cap; ++m) {
    const int64_t j = nl[(int64_t)m * N + i];
    int n0, n1, n2, a, b, c;
    min_image(st, pos[j] - pos[i], pos[N + j] - pos[N + i], pos[2 * N + j] - pos[2 * N + i], n0,
              n1, n2);
    // image codes are stored only for structures that need several images
    split_code(st.mode == kModeImages ? cd[(int64_t)m * N + i] : kCodeCenter, a, b, c);
    nbr[e * cap + m] = perm[j];
    shift[(e * cap + m) * 3 + 0] = n0 + a;
    shift[(e * cap + m) * 3 + 1] = n1 + b;
    shift[(e * cap + m) * 3 + 2] = n2 + c;
  }
}

void launch_neighbors_out(const Lists& L, int which, int64_t N, const int32_t* perm,
                          const int32_t* inv_perm, const double* pos, const int32_t* sid,
                          const StructInfo* structs, int32_t cap, int32_t* count, int32_t* nbr,
                          int32_t* shift, hipStream_t s) {
  hipLaunchKernelGGL(k_neighbors_out, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, L, which, N,
                     perm, inv_perm, pos, sid, structs, cap, count, nbr, shift);
}

}  // namespace nep

namespace nep {

// Heat current of Sec. II.E: J_i = W_i . v_i (eq. Ji), J_i,a = sum_b W_i,ab v_i,b,
// in float64 from the float32 per-atom virial (sorted order) and the caller's
// float64 velocities [3][N] (caller order).  J_i goes to heat[3][N] in caller
// order when heat is not NULL; block b sums the J_i of its chunk in a fixed
// tree into partial[b][3] for the total of eq. J-1.
__global__ void __launch_bounds__(kRedBlock) k_heat_current_partial(
    const float* __restrict__ W, int64_t N, const int32_t* __restrict__ perm,
    const double* __restrict__ vel, int64_t chunk, double* __restrict__ heat,
    double* __restrict__ partial) {
  __shared__ double sh[3][kRedBlock];
  const int t = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(N, lo + chunk);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t k = lo + t; k < hi; k += kRedBlock) {
    const int64_t e = perm[k];
    const double v[3] = {vel[e], vel[N + e], vel[2 * N + e]};
    for (int a = 0; a < 3; ++a) {
      double j = 0.0;
      for (int b = 0; b < 3; ++b) j = fma((double)W[(int64_t)(3 * a + b) * N + k], v[b], j);
      if (heat) heat[(int64_t)a * N + e] = j;
      acc[a] += j;
    }
  }
  for (int a = 0; a < 3; ++a) sh[a][t] = acc[a];
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int a = 0; a < 3; ++a) sh[a][t] += sh[a][t + off];
    __syncthreads();
  }
  if (t < 3) partial[blockIdx.x * 3 + t] = sh[t][0];
}

// total[a] = sum_b partial[b][a]: thread t adds blocks t, t + kRedBlock, ...
// in order, then a fixed tree over the threads (the same bits every call).
__global__ void __launch_bounds__(kRedBlock) k_heat_current_final(const double* __restrict__ partial,
                                                                  int64_t n_part,
                                                                  double* __restrict__ total) {
  __shared__ double sh[3][kRedBlock];
  const int t = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t b = t; b < n_part; b += kRedBlock)
    for (int a = 0; a < 3; ++a) acc[a] += partial[b * 3 + a];
  for (int a = 0; a < 3; ++a) sh[a][t] = acc[a];
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int a = 0; a < 3; ++a) sh[a][t] += sh[a][t + off];
    __syncthreads();
  }
  if (t < 3) total[t] = sh[t][0];
}

void launch_heat_current(const float* W, int64_t N, const int32_t* perm, const double* vel,
                         double* heat, double* total, double* partial, int64_t n_part,
                         hipStream_t s) {
  const int64_t chunk = (N + n_part - 1) / n_part;
  hipLaunchKernelGGL(k_heat_current_partial, dim3((unsigned)n_part), dim3(kRedBlock), 0, s, W, N,
                     perm, vel, chunk, heat, partial);
  if (total) hipLaunchKernelGGL(k_heat_current_final, dim3(1), dim3(kRedBlock), 0, s, partial, n_part, total);
}

}  // namespace nep

namespace nep {

// Training loss of Sec. II.E (eq. loss) for P parameter sets from the batch
// outputs.  Block (c, p) takes chunk c of the structures (energy per atom and
// the six virial components per atom), of the 3N force components and of the
// parameters of set p, and writes its six fixed-tree sums
// [sum de^2, sum df^2, sum dw^2, sum |z|, sum z^2, structures with a virial]
// to partial[p][c][6].  A structure whose six virial targets include a NaN
// has no virial target: it adds nothing to sum dw^2 and is not counted.
constexpr int kLossSums = 6;

struct LossArgs {
  const double* force;    // [P][3][N]
  const double* totals;   // [P][S][10]
  const int64_t* offs;    // [S + 1]
  const double* e_tar;    // [S] eV/atom
  const double* f_tar;    // [3][N]
  const double* w_tar;    // [S][6] eV/atom (xx, yy, zz, xy, yz, zx) or NULL; NaN rows absent
  const double* params;   // [P][npar] or NULL
  int64_t N, npar;
  int32_t S;
  double lam[5];
};

__global__ void __launch_bounds__(kRedBlock) k_loss_partial(LossArgs a, double* __restrict__ partial) {
  __shared__ double sh[kLossSums][kRedBlock];
  const int t = threadIdx.x;
  const int64_t p = blockIdx.y, c = blockIdx.x, C = gridDim.x;
  double acc[kLossSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  {
    const int64_t chunk = (a.S + C - 1) / C, lo = c * chunk, hi = min((int64_t)a.S, lo + chunk);
    const int comp[6] = {0, 4, 8, 1, 5, 6};
    for (int64_t n = lo + t; n < hi; n += kRedBlock) {
      const double cnt = (double)(a.offs[n + 1] - a.offs[n]);
      const double* T = a.totals + ((int64_t)p * a.S + n) * 10;
      const double de = T[0] / cnt - a.e_tar[n];
      acc[0] += de * de;
      if (a.w_tar) {
        double sw = 0.0;
        bool has = true;
        for (int v = 0; v < 6; ++v) {
          const double target = a.w_tar[n * 6 + v];
          has = has && !isnan(target);
          const double dw = T[1 + comp[v]] / cnt - target;
          sw += dw * dw;
        }
        if (has) {
          acc[2] += sw;
          acc[5] += 1.0;
        }
      }
    }
  }
  {
    const int64_t n3 = 3 * a.N, chunk = (n3 + C - 1) / C, lo = c * chunk, hi = min(n3, lo + chunk);
    const double* f = a.force + p * n3;
    for (int64_t k = lo + t; k < hi; k += kRedBlock) {
      const double df = f[k] - a.f_tar[k];
      acc[1] += df * df;
    }
  }
  if (a.params) {
    const int64_t chunk = (a.npar + C - 1) / C, lo = c * chunk, hi = min(a.npar, lo + chunk);
    const double* z = a.params + p * a.npar;
    for (int64_t k = lo + t; k < hi; k += kRedBlock) {
      acc[3] += fabs(z[k]);
      acc[4] += z[k] * z[k];
    }
  }
  for (int v = 0; v < kLossSums; ++v) sh[v][t] = acc[v];
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int v = 0; v < kLossSums; ++v) sh[v][t] += sh[v][t + off];
    __syncthreads();
  }
  if (t < kLossSums) partial[(p * C + c) * kLossSums + t] = sh[t][0];
}

// loss[p][6] = [L, L_e, L_f, L_v, L_1, L_2]: the chunk sums added in chunk
// order, the RMSEs and norms formed, and L their lambda-weighted sum.
__global__ void k_loss_final(LossArgs a, const double* __restrict__ partial, int64_t C, int32_t P,
                             double* __restrict__ loss) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s[kLossSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t c = 0; c < C; ++c)
    for (int v = 0; v < kLossSums; ++v) s[v] += partial[(p * C + c) * kLossSums + v];
  const double le = sqrt(s[0] / a.S), lf = sqrt(s[1] / (3.0 * a.N));
  // the virial RMSE runs over the structures that have virial targets
  const double lv = (a.w_tar && s[5] > 0) ? sqrt(s[2] / (6.0 * s[5])) : 0.0;
  const double l1 = a.params ? s[3] / a.npar : 0.0, l2 = a.params ? sqrt(s[4] / a.npar) : 0.0;
  double* o = loss + p * 6;
  o[0] = a.lam[0] * le + a.lam[1] * lf + a.lam[2] * lv + a.lam[3] * l1 + a.lam[4] * l2;
  o[1] = le;
  o[2] = lf;
  o[3] = lv;
  o[4] = l1;
  o[5] = l2;
}

// Workspace of the allocation-free loss entry point: a fixed 1 MiB array in
// every GPU's memory, held until the process ends.  Host code never passes
// the array's name to a kernel or a copy (on the host it is only a stand-in
// symbol): it uses the device address hipGetSymbolAddress gives for the
// current device, looked up once per device and kept here.
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t loss_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

int64_t loss_chunks(int64_t N) { return std::min<int64_t>(256, std::max<int64_t>(1, (3 * N + 16383) / 16384)); }

void launch_loss(const double* force, const double* totals, const int64_t* offs, int32_t S, int64_t N,
                 int32_t P, const double* e_tar, const double* f_tar, const double* w_tar,
                 const double* params, int64_t npar, const double lam[5], double* partial, double* loss,
                 hipStream_t s) {
  LossArgs a{force, totals, offs, e_tar, f_tar, w_tar, params, N, npar, S, {0, 0, 0, 0, 0}};
  for (int v = 0; v < 5; ++v) a.lam[v] = lam[v];
  const int64_t C = loss_chunks(N);
  hipLaunchKernelGGL(k_loss_partial, dim3((unsigned)C, (unsigned)P), dim3(kRedBlock), 0, s, a, partial);
  hipLaunchKernelGGL(k_loss_final, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, s, a, partial, C, P, loss);
}

}  // namespace nep

namespace nep {

// SNES (the trainer of Sec. II.E; Schaul et al. 2011).  One block ranks the
// population by loss (ties to the lower index, non-finite losses last) and gives member k the
// utility of its rank r: max(0, ln(P/2 + 1) - ln(r + 1)) / sum - 1/P.  Every
// thread forms the normaliser in the same order, so all agree bitwise.
constexpr int kSnesMaxPop = 1024;

__global__ void __launch_bounds__(kSnesMaxPop) k_snes_utilities(const double* __restrict__ loss,
                                                                int64_t stride, int32_t P,
                                                                double* __restrict__ util) {
  const int k = threadIdx.x;
  if (k >= P) return;
  const double top = log(0.5 * P + 1.0);
  double tot = 0.0;
  for (int r = 0; r < P; ++r) tot += fmax(0.0, top - log(r + 1.0));
  const double lk = loss[(int64_t)k * stride];
  const bool fk = isfinite(lk);
  int rank = 0;
  for (int j = 0; j < P; ++j) {
    const double lj = loss[(int64_t)j * stride];
    const bool fj = isfinite(lj);
    // finite losses first, in increasing order; non-finite ones (a diverged
    // member) after them; ties by index, so the ranks are a permutation
    const bool before = (fj && !fk) || (fj == fk && (fj ? (lj < lk || (lj == lk && j < k)) : j < k));
    rank += before ? 1 : 0;
  }
  util[k] = fmax(0.0, top - log(rank + 1.0)) / tot - 1.0 / P;
}

// Natural-gradient steps per parameter i: g_mu = sum_k u_k s_ki,
// g_sigma = sum_k u_k (s_ki^2 - 1) in member order; mu += eta_mu sigma g_mu,
// sigma *= exp(eta_sigma g_sigma / 2).  noise is [P][n_par] (coalesced in i).
__global__ void k_snes_update(const double* __restrict__ util, const double* __restrict__ noise,
                              int64_t n_par, int32_t P, double eta_mu, double eta_sigma,
                              double* __restrict__ mean, double* __restrict__ sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_par) return;
  double gm = 0.0, gs = 0.0;
  for (int k = 0; k < P; ++k) {
    const double s = noise[(int64_t)k * n_par + i], u = util[k];
    gm += u * s;
    gs += u * (s * s - 1.0);
  }
  const double sg = sigma[i];
  mean[i] += eta_mu * sg * gm;
  sigma[i] = sg * exp(0.5 * eta_sigma * gs);
}

// population[k][i] = mean[i] + sigma[i] * noise[k][i]
__global__ void k_snes_sample(const double* __restrict__ mean, const double* __restrict__ sigma,
                              const double* __restrict__ noise, int64_t n_par,
                              double* __restrict__ pop) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_par) return;
  const int64_t o = (int64_t)blockIdx.y * n_par + i;
  pop[o] = mean[i] + sigma[i] * noise[o];
}

void launch_snes_step(const double* loss, int64_t stride, int32_t P, const double* noise, int64_t n_par,
                      double eta_mu, double eta_sigma, double* util, double* mean, double* sigma,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_snes_utilities, dim3(1), dim3(kSnesMaxPop), 0, s, loss, stride, P, util);
  hipLaunchKernelGGL(k_snes_update, dim3((unsigned)div_up(n_par, kBlock)), dim3(kBlock), 0, s, util,
                     noise, n_par, P, eta_mu, eta_sigma, mean, sigma);
}

void launch_snes_sample(const double* mean, const double* sigma, const double* noise, int64_t n_par,
                        int32_t P, double* pop, hipStream_t s) {
  hipLaunchKernelGGL(k_snes_sample, dim3((unsigned)div_up(n_par, kBlock), (unsigned)P), dim3(kBlock), 0,
                     s, mean, sigma, noise, n_par, pop);
}

}  // namespace nep
