// mlp.hip -- the per-atom network of eq. (Ui) as two batched GEMMs on MFMA.
//
// For a tile of 16 atoms of one species (rows of q in the species-grouped
// order built with the neighbour lists):
//   GEMM 1   H^T = w0 q^T            [N_neu x N_des] x [N_des x 16]
//            h = tanh(H - b0),  U = sum_mu w1_mu h_mu - b1
//   GEMM 2   dU/dq = G w0,  G = w1 (1 - h^2)     [16 x N_neu] x [N_neu x N_des]
// (the derivative is the back-propagation of the printed apply_ann routine,
// App. B).  GEMM 1 is laid out so that its accumulator tile, lane l holding
// neurons 4(l/16)+r of atom l%16, is directly the A operand of GEMM 2 once
// the reduction index is read as "neuron 16 nb + 4 (l/16) + r": the B operand
// of GEMM 2 loads w0 rows in that same order, so no transpose through LDS is
// needed.  Every output element is accumulated in a fixed order that does not
// depend on the other rows of the tile, so results do not depend on how
// atoms are grouped into tiles.
//
// FP32: v_mfma_f32_16x16x4_f32.  BF16: v_mfma_f32_16x16x32_bf16 with bf16
// operands (q, w0, G) and float32 accumulation; b0, tanh and the w1 products
// stay float32.
#include "nep_kernels.h"

namespace nep {

namespace {
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8bf bf16x8_from_bits(uint4 u) {
  v8bf r;
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r[2 * k] = __builtin_bit_cast(__bf16, (uint16_t)(w[k] & 0xffffu));
    r[2 * k + 1] = __builtin_bit_cast(__bf16, (uint16_t)(w[k] >> 16));
  }
  return r;
}

__device__ __forceinline__ void bf16x4_from_bits(uint2 u, v8bf& r, int off) {
  r[off + 0] = __builtin_bit_cast(__bf16, (uint16_t)(u.x & 0xffffu));
  r[off + 1] = __builtin_bit_cast(__bf16, (uint16_t)(u.x >> 16));
  r[off + 2] = __builtin_bit_cast(__bf16, (uint16_t)(u.y & 0xffffu));
  r[off + 3] = __builtin_bit_cast(__bf16, (uint16_t)(u.y >> 16));
}
}  // namespace

template <int NNB, bool BF16>
__global__ void __launch_bounds__(256) k_mlp(EvalArgs a) {
  const DevModel& M = a.M;
  const int lane = threadIdx.x & 63;
  const int64_t base = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (base >= a.rows_len) return;
  const int first = a.rows[base];
  if (first < 0) return;  // tiles never mix species; a tile starting with padding is all padding
  const int net = M.nets > 1 ? a.types[first] : 0;
  const int col = lane & 15, grp = lane >> 4;
  const int atom = a.rows[base + col];
  const int ND = M.ND, NNp = M.NNp;
  const float* __restrict__ qrow = a.q + (int64_t)(atom < 0 ? 0 : atom) * M.NDp;
  const float* __restrict__ b0 = M.b0 + net * NNp;
  const float* __restrict__ w1 = M.w1 + net * NNp;

  // ---- GEMM 1: acc[nb][r] = sum_d w0[16 nb + 4 grp + r][d] q[atom col][d] ----
  v4f acc[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
  if constexpr (!BF16) {
    const float* __restrict__ w0t = M.w0t + (int64_t)net * ND * NNp;
    const int steps = (ND + 3) / 4;
    // the operands of step s + 1 are loaded while step s is multiplied; every
    // load is in bounds (index clamped) and the tail is selected to zero after
    float qn, wn[NNB];
    {
      const int dc = min(grp, ND - 1);
      qn = qrow[dc];
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) wn[nb] = w0t[(int64_t)dc * NNp + 16 * nb + col];
    }
    for (int s = 0; s < steps; ++s) {
      const int d = 4 * s + grp;
      const float qv = qn;
      float wv[NNB];
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) wv[nb] = wn[nb];
      const int dn = min(d + 4, ND - 1);
      qn = qrow[dn];
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) wn[nb] = w0t[(int64_t)dn * NNp + 16 * nb + col];
      const float bq = (atom >= 0 && d < ND) ? qv : 0.f;
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        const float aw = d < ND ? wv[nb] : 0.f;
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw, bq, acc[nb], 0, 0, 0);
      }
    }
  } else {
    const uint16_t* __restrict__ w0b = M.w0b + (int64_t)net * NNp * M.NDp32;
    const int steps = M.NDp32 / 32;
    for (int s = 0; s < steps; ++s) {
      const int d0 = 32 * s + 8 * grp;
      const int dq = min(d0, M.NDp - 8);  // NDp is a multiple of 8: the load stays in the row
      const bool live = atom >= 0 && d0 < M.NDp;
      const float4 x0 = *reinterpret_cast<const float4*>(qrow + dq);
      const float4 x1 = *reinterpret_cast<const float4*>(qrow + dq + 4);
      const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
      v8bf bq;
#pragma unroll
      for (int k = 0; k < 8; ++k) bq[k] = (__bf16)(live ? xs[k] : 0.f);
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        const uint4 u = *reinterpret_cast<const uint4*>(w0b + (int64_t)(16 * nb + col) * M.NDp32 + d0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf16x8_from_bits(u), bq, acc[nb], 0, 0, 0);
      }
    }
  }

  // ---- activation, site energy and G = w1 (1 - h^2) ----
  float u = 0.f;
  float g[NNB][4], b0v[NNB][4], w1v[NNB][4];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // all loads issued before the first tanh
      const int mu = 16 * nb + 4 * grp + r;
      b0v[nb][r] = b0[mu];
      w1v[nb][r] = w1[mu];
    }
  // the latent-space vector of Sec. IV is the products w1_mu h_mu, one per
  // neuron, written when asked for
  float* __restrict__ lat = (a.latent && atom >= 0) ? a.latent + (int64_t)atom * M.NN : nullptr;
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float h = tanhf(acc[nb][r] - b0v[nb][r]);
      const float wh = w1v[nb][r] * h;
      u += wh;
      g[nb][r] = w1v[nb][r] * (1.f - h * h);
      const int mu = 16 * nb + 4 * grp + r;
      if (lat && mu < M.NN) lat[mu] = wh;
    }
  u += __shfl_xor(u, 16);
  u += __shfl_xor(u, 32);
  if (grp == 0 && atom >= 0) a.U[atom] = u - *M.b1;


  // ---- GEMM 2: dU/dq[atom][d] = sum_mu G[atom][mu] w0[mu][d] ----
  int out_atom[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) out_atom[r] = a.rows[base + 4 * grp + r];
  const int dblocks = (ND + 15) / 16;
  for (int db = 0; db < dblocks; ++db) {
    const int d = 16 * db + col;
    v4f c = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF16) {
      const float* __restrict__ w0 = M.w0 + (int64_t)net * NNp * ND;
      const int dc = min(d, ND - 1);
      float wv[NNB][4];
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) wv[nb][r] = w0[(int64_t)(16 * nb + 4 * grp + r) * ND + dc];
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float bw = d < ND ? wv[nb][r] : 0.f;
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][r], bw, c, 0, 0, 0);
        }
    } else {
      const uint16_t* __restrict__ w0tb = M.w0tb + (int64_t)net * M.NDp32 * NNp;
      const uint16_t* wrow = w0tb + (int64_t)(d < M.NDp32 ? d : 0) * NNp;
#pragma unroll
      for (int p = 0; p < NNB / 2; ++p) {
        v8bf av, bv;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          av[r] = (__bf16)g[2 * p][r];
          av[4 + r] = (__bf16)g[2 * p + 1][r];
        }
        const uint2 lo = *reinterpret_cast<const uint2*>(wrow + 32 * p + 4 * grp);
        const uint2 hi = *reinterpret_cast<const uint2*>(wrow + 32 * p + 16 + 4 * grp);
        bf16x4_from_bits(lo, bv, 0);
        bf16x4_from_bits(hi, bv, 4);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int at = out_atom[r];
      if (at >= 0 && d < ND) a.fp[(int64_t)at * M.NDp + d] = c[r];
    }
  }
}

// The same two GEMMs with their operands staged in LDS: a block takes one
// group of kRowGroup = 64 species-grouped rows (four 16-row tiles, one per
// wave, never mixing species), stages that species' w0 and the 64 descriptor
// rows once with coalesced loads, and feeds every MFMA from LDS, so a wave's
// chain of dependent global loads is gone.  The MFMA operands and their order
// are those of k_mlp, so the results are the same bits.
//   FP32 LDS: w0 [NNp][ND + 1], q [64][NDp + 1] (odd strides: lanes reading
//             16 rows at one column hit 16 banks)
//   BF16 LDS: w0 [NNp][NDp32 + 8], w0^T [NDp32][NNp + 8], q [64][NDp32 + 8]
//             (bf16; rows of 16-byte multiples for the 8-wide loads)
size_t mlp_lds_bytes(const DevModel& M, bool bf16) {
  if (!bf16)
    return ((size_t)M.NNp * (M.ND + 1) + (size_t)kRowGroup * (M.NDp + 1)) * sizeof(float);
  return ((size_t)M.NNp * (M.NDp32 + 8) + (size_t)M.NDp32 * (M.NNp + 8) + (size_t)kRowGroup * (M.NDp32 + 8)) *
         sizeof(uint16_t);
}

template <int NNB, bool BF16>
__global__ void __launch_bounds__(256) k_mlp_lds(EvalArgs a) {
  extern __shared__ float4 mlp_lds[];
  const DevModel& M = a.M;
  const int64_t base = (int64_t)blockIdx.x * kRowGroup;
  if (base >= a.rows_len) return;
  const int first = a.rows[base];
  if (first < 0) return;  // a group starting with padding is all padding (the whole block leaves)
  const int net = M.nets > 1 ? a.types[first] : 0;
  const int tid = threadIdx.x, lane = tid & 63, r0 = (tid >> 6) * 16;
  const int col = lane & 15, grp = lane >> 4;
  const int ND = M.ND, NNp = M.NNp, NDp = M.NDp, NDp32 = M.NDp32;
  const int atom = a.rows[base + r0 + col];
  const float* __restrict__ b0 = M.b0 + net * NNp;
  const float* __restrict__ w1 = M.w1 + net * NNp;
  int out_atom[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) out_atom[r] = a.rows[base + r0 + 4 * grp + r];

  v4f acc[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
  float* sw = reinterpret_cast<float*>(mlp_lds);
  uint16_t* hw = reinterpret_cast<uint16_t*>(mlp_lds);
  const int SW = ND + 1, SQ = NDp + 1;
  const int SWB = NDp32 + 8, STB = NNp + 8, SQB = NDp32 + 8;
  uint16_t* swb = hw;
  uint16_t* swtb = swb + NNp * SWB;
  uint16_t* sqb = swtb + NDp32 * STB;
  float* sq = sw + NNp * SW;
  // ---- stage w0 of this species and the 64 descriptor rows ----
  if constexpr (!BF16) {
    const float* __restrict__ w0 = M.w0 + (int64_t)net * NNp * ND;
    for (int k = tid; k < NNp * ND; k += 256) sw[(k / ND) * SW + k % ND] = w0[k];
    for (int k = tid; k < kRowGroup * NDp; k += 256) {
      const int r = k / NDp, d = k % NDp, at = a.rows[base + r];
      sq[r * SQ + d] = at >= 0 ? a.q[(int64_t)at * NDp + d] : 0.f;
    }
  } else {
    const uint16_t* __restrict__ w0b = M.w0b + (int64_t)net * NNp * NDp32;
    const uint16_t* __restrict__ w0tb = M.w0tb + (int64_t)net * NDp32 * NNp;
    for (int k = tid; k < NNp * NDp32; k += 256) swb[(k / NDp32) * SWB + k % NDp32] = w0b[k];
    for (int k = tid; k < NDp32 * NNp; k += 256) swtb[(k / NNp) * STB + k % NNp] = w0tb[k];
    for (int k = tid; k < kRowGroup * NDp32; k += 256) {
      const int r = k / NDp32, d = k % NDp32, at = a.rows[base + r];
      const float x = (at >= 0 && d < NDp) ? a.q[(int64_t)at * NDp + d] : 0.f;
      sqb[r * SQB + d] = __builtin_bit_cast(uint16_t, (__bf16)x);
    }
  }
  __syncthreads();

  // ---- GEMM 1: acc[nb][r] = sum_d w0[16 nb + 4 grp + r][d] q[atom col][d] ----
  if constexpr (!BF16) {
    const int steps = (ND + 3) / 4;
    for (int st = 0; st < steps; ++st) {
      const int d = 4 * st + grp;
      const float bq = (atom >= 0 && d < ND) ? sq[(r0 + col) * SQ + d] : 0.f;
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        const float aw = d < ND ? sw[(16 * nb + col) * SW + d] : 0.f;
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw, bq, acc[nb], 0, 0, 0);
      }
    }
  } else {
    const int steps = NDp32 / 32;
    for (int st = 0; st < steps; ++st) {
      const int d0 = 32 * st + 8 * grp;
      v8bf bq = bf16x8_from_bits(*reinterpret_cast<const uint4*>(sqb + (r0 + col) * SQB + d0));
      if (atom < 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) bq[k] = (__bf16)0.f;
      }
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        const uint4 u = *reinterpret_cast<const uint4*>(swb + (16 * nb + col) * SWB + d0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf16x8_from_bits(u), bq, acc[nb], 0, 0, 0);
      }
    }
  }

  // ---- activation, site energy, latent vector and G = w1 (1 - h^2) ----
  float u = 0.f;
  float g[NNB][4];
  float* __restrict__ lat = (a.latent && atom >= 0) ? a.latent + (int64_t)atom * M.NN : nullptr;
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = 16 * nb + 4 * grp + r;
      const float h = tanhf(acc[nb][r] - b0[mu]);
      const float wh = w1[mu] * h;
      u += wh;
      g[nb][r] = w1[mu] * (1.f - h * h);
      if (lat && mu < M.NN) lat[mu] = wh;
    }
  u += __shfl_xor(u, 16);
  u += __shfl_xor(u, 32);
  if (grp == 0 && atom >= 0) a.U[atom] = u - *M.b1;

  // ---- GEMM 2: dU/dq[atom][d] = sum_mu G[atom][mu] w0[mu][d] ----
  const int dblocks = (ND + 15) / 16;
  for (int db = 0; db < dblocks; ++db) {
    const int d = 16 * db + col;
    v4f c = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF16) {
      const int dc = min(d, ND - 1);
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float bw = d < ND ? sw[(16 * nb + 4 * grp + r) * SW + dc] : 0.f;
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][r], bw, c, 0, 0, 0);
        }
    } else {
      const uint16_t* wrow = swtb + (d < NDp32 ? d : 0) * STB;
#pragma unroll
      for (int p = 0; p < NNB / 2; ++p) {
        v8bf av, bv;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          av[r] = (__bf16)g[2 * p][r];
          av[4 + r] = (__bf16)g[2 * p + 1][r];
        }
        const uint2 lo = *reinterpret_cast<const uint2*>(wrow + 32 * p + 4 * grp);
        const uint2 hi = *reinterpret_cast<const uint2*>(wrow + 32 * p + 16 + 4 * grp);
        bf16x4_from_bits(lo, bv, 0);
        bf16x4_from_bits(hi, bv, 4);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int at = out_atom[r];
      if (at >= 0 && d < ND) a.fp[(int64_t)at * M.NDp + d] = c[r];
    }
  }
}

void launch_mlp(const EvalArgs& a, hipStream_t s) {
  const int nnb = a.M.NNp / 16;
  const size_t lds = mlp_lds_bytes(a.M, a.mlp_bf16 != 0);
  if (lds <= 64 * 1024) {
    dim3 grid((unsigned)div_up(a.rows_len, kRowGroup)), block(256);
#define NEP_MLP(n)                                                                        \
  if (nnb == n) {                                                                         \
    if (a.mlp_bf16) hipLaunchKernelGGL((k_mlp_lds<n, true>), grid, block, lds, s, a);     \
    else hipLaunchKernelGGL((k_mlp_lds<n, false>), grid, block, lds, s, a);               \
    return;                                                                               \
  }
    NEP_MLP(2) NEP_MLP(4) NEP_MLP(6) NEP_MLP(8)
#undef NEP_MLP
  }
  // operands too large for LDS: one 16-row tile per wave from global memory
  const int64_t tiles = a.rows_len / 16;
  dim3 grid((unsigned)div_up(tiles, 4)), block(256);
#define NEP_MLP(n)                                                              \
  if (nnb == n) {                                                               \
    if (a.mlp_bf16) hipLaunchKernelGGL((k_mlp<n, true>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((k_mlp<n, false>), grid, block, 0, s, a);           \
    return;                                                                     \
  }
  NEP_MLP(2) NEP_MLP(4) NEP_MLP(6) NEP_MLP(8)
#undef NEP_MLP
}

}  // namespace nep
