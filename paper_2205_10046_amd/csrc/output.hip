// output.hip -- results back in the caller's atom order, and the float64
// totals E = sum_i U_i, W = sum_i W_i (a fixed two-level tree: the same
// inputs always give the same bits).
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

__global__ void k_heat_current_final(const double* __restrict__ partial, int64_t n_part,
                                     double* __restrict__ total) {
  const int a = threadIdx.x;
  if (a >= 3) return;
  double s = 0.0;
  for (int64_t b = 0; b < n_part; ++b) s += partial[b * 3 + a];
  total[a] = s;
}

void launch_heat_current(const float* W, int64_t N, const int32_t* perm, const double* vel,
                         double* heat, double* total, double* partial, int64_t n_part,
                         hipStream_t s) {
  const int64_t chunk = (N + n_part - 1) / n_part;
  hipLaunchKernelGGL(k_heat_current_partial, dim3((unsigned)n_part), dim3(kRedBlock), 0, s, W, N,
                     perm, vel, chunk, heat, partial);
  if (total) hipLaunchKernelGGL(k_heat_current_final, dim3(1), dim3(64), 0, s, partial, n_part, total);
}

}  // namespace nep
