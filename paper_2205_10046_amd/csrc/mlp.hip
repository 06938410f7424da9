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

// tanh from its definition, branch-free: the odd Taylor series through x^9
// for |x| < 1/4 (the first dropped term is below 1e-8 relative there) and
// 1 - 2 / (1 + e^{2|x|}) with the sign of x elsewhere (e^{2|x|} = inf gives
// 1).  Both forms are evaluated and one is selected, so the lanes of a wave
// never diverge.  Absolute error <= ~2e-7.
__device__ __forceinline__ float tanh_net(float x) {
  const float ax = fabsf(x), x2 = x * x;
  float p = fmaf(x2, 62.f / 2835.f, -17.f / 315.f);
  p = fmaf(x2, p, 2.f / 15.f);
  p = fmaf(x2, p, -1.f / 3.f);
  const float small = fmaf(x * x2, p, x);
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * ax);  // 2^(2 |x| log2 e)
  const float big = copysignf(fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + e), 1.f), x);
  return ax < 0.25f ? small : big;
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
      const float h = tanh_net(acc[nb][r] - b0v[nb][r]);
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

// The same two GEMMs with the species' weights staged in LDS.  The rows are
// cut into groups of kRowGroup = 64 species-grouped rows (each species padded
// to whole groups, so a group never mixes species); a block takes a run of
// consecutive groups, one 16-row tile per wave per group, and stages w0 and
// w0^T of a species once for all of its groups of that species (L2-resident
// weights, 16-byte loads, kStageBatch per lane at a time).  A lane holds its
// share of its atom's descriptor row in registers, and loads the next
// group's share while the current group is computed; the MFMA weight
// operands are 16-byte LDS reads.
//   FP32: the reduction index of GEMM 1 runs over N_des padded to a multiple
//         of 16 (zero weights past N_des), split into four contiguous
//         quarters of KS = NDp16 / 4: step s of the 16x16x4 MFMA takes k =
//         KS g + s from lane group g, so a lane's q values and w0 values are
//         contiguous.  LDS: w0 [NNp][NDp16 + 4], w0^T [NDp16][NNp + 4].
//   BF16: k = 32 s + 8 g + 0..7 as in k_mlp.  LDS: w0 [NNp][NDp32 + 8],
//         w0^T [NDp32][NNp + 8] (bf16 bits).
// Each output is accumulated in a fixed order that does not depend on the
// other rows of the tile (results do not depend on how atoms are grouped);
// the float32 order of GEMM 1 differs from k_mlp's.
constexpr int kStageBatch = 8;
constexpr int kMlpMaxKS = 24;  // LDS kernel: N_des padded to 16 at most 96
constexpr int kMlpQ = 24;      // q values per lane (float32: KS <= 24; bf16: NDp32 <= 96)
constexpr int kMlpBlocks = 1024;  // LDS kernel: target grid size
constexpr size_t kMlpMaxLds = 160 * 1024;  // LDS a gfx950 block may hold

__host__ __device__ inline int nd_pad16(int nd) { return (nd + 15) / 16 * 16; }

// Bytes of the staged weights w0 and w0^T (b0 and w1 follow, 2 N_neu floats).
__host__ __device__ inline size_t mlp_weight_bytes(const DevModel& M, bool bf16) {
  if (!bf16) {
    const size_t K = (size_t)nd_pad16(M.ND);
    return ((size_t)M.NNp * (K + 4) + K * (M.NNp + 4)) * sizeof(float);
  }
  const size_t b = ((size_t)M.NNp * (M.NDp32 + 8) + (size_t)M.NDp32 * (M.NNp + 8)) * sizeof(uint16_t);
  return (b + 15) / 16 * 16;
}

size_t mlp_lds_bytes(const DevModel& M, bool bf16) {
  return mlp_weight_bytes(M, bf16) + 2 * (size_t)M.NNp * sizeof(float);
}

namespace {

// This lane's q values of atom `atom` (zero for padding rows and past the row).
template <bool BF16>
__device__ __forceinline__ void load_q(const EvalArgs& a, int atom, int grp, int KS, float (&qv)[kMlpQ]) {
  const int NDp = a.M.NDp;
  const float* __restrict__ qrow = a.q + (int64_t)(atom < 0 ? 0 : atom) * NDp;
  if constexpr (!BF16) {
#pragma unroll
    for (int v = 0; v < kMlpQ / 4; ++v) {
      const int c = KS * grp + 4 * v;  // NDp is a multiple of 8: a word is all in or all out
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (4 * v < KS && atom >= 0 && c < NDp) x = *reinterpret_cast<const float4*>(qrow + c);
      qv[4 * v] = x.x;
      qv[4 * v + 1] = x.y;
      qv[4 * v + 2] = x.z;
      qv[4 * v + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int st = 0; st < kMlpQ / 8; ++st) {
      const int d0 = 32 * st + 8 * grp;
      float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0;
      if (32 * st < a.M.NDp32 && atom >= 0 && d0 < NDp) {
        x0 = *reinterpret_cast<const float4*>(qrow + d0);
        x1 = *reinterpret_cast<const float4*>(qrow + d0 + 4);
      }
      const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) qv[8 * st + k] = xs[k];
    }
  }
}

// w0 and w0^T of species net into LDS (the caller synchronises the block).
template <bool BF16>
__device__ __forceinline__ void stage_weights(const DevModel& M, int net, int tid, float4* lds) {
  const int ND = M.ND, NNp = M.NNp, NDp32 = M.NDp32, K16 = nd_pad16(ND);
  {  // b0 and w1 of the species after the weights
    float* bw = reinterpret_cast<float*>(reinterpret_cast<char*>(lds) + mlp_weight_bytes(M, BF16));
    for (int k = tid; k < 2 * NNp; k += 256) bw[k] = k < NNp ? M.b0[net * NNp + k] : M.w1[net * NNp + k - NNp];
  }
  if constexpr (!BF16) {
    float* sw = reinterpret_cast<float*>(lds);
    const int SW = K16 + 4, ST = NNp + 4;
    float* st = sw + NNp * SW;
    const float4* __restrict__ w04 = reinterpret_cast<const float4*>(M.w0 + (int64_t)net * NNp * ND);
    const float4* __restrict__ wt4 = reinterpret_cast<const float4*>(M.w0t + (int64_t)net * ND * NNp);
    const int nw = NNp * ND / 4, t4 = NNp / 4, total = 2 * nw;  // NNp is a multiple of 32
    for (int k0 = tid; k0 < total; k0 += kStageBatch * 256) {
      float4 v[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int k = k0 + u * 256;
        v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < nw) v[u] = w04[k];
        else if (k < total) v[u] = wt4[k - nw];
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int k = k0 + u * 256;
        if (k < nw) {
          int row = 4 * k / ND, c = 4 * k - row * ND;
          const float x[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            sw[row * SW + c] = x[j];
            if (++c == ND) {
              c = 0;
              ++row;
            }
          }
        } else if (k < total) {
          const int r = (k - nw) / t4, c = k - nw - r * t4;
          *reinterpret_cast<float4*>(st + r * ST + 4 * c) = v[u];
        }
      }
    }
    // zero weights past N_des: columns ND..K16-1 of w0, rows ND..K16-1 of w0^T
    const int pad = K16 - ND;
    for (int k = tid; k < NNp * pad; k += 256) sw[(k / pad) * SW + ND + k % pad] = 0.f;
    for (int k = tid; k < pad * NNp; k += 256) st[(ND + k / NNp) * ST + k % NNp] = 0.f;
  } else {
    uint16_t* swb = reinterpret_cast<uint16_t*>(lds);
    const int SWB = NDp32 + 8, STB = NNp + 8;
    uint16_t* swtb = swb + NNp * SWB;
    const uint4* __restrict__ wb = reinterpret_cast<const uint4*>(M.w0b + (int64_t)net * NNp * NDp32);
    const uint4* __restrict__ wtb = reinterpret_cast<const uint4*>(M.w0tb + (int64_t)net * NDp32 * NNp);
    const int c8 = NDp32 / 8, t8 = NNp / 8;
    const int n1 = NNp * c8, total = n1 + NDp32 * t8;
    for (int k0 = tid; k0 < total; k0 += kStageBatch * 256) {
      uint4 v[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int k = k0 + u * 256;
        v[u] = make_uint4(0u, 0u, 0u, 0u);
        if (k < n1) v[u] = wb[k];
        else if (k < total) v[u] = wtb[k - n1];
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int k = k0 + u * 256;
        if (k < n1) {
          const int r = k / c8, c = k - r * c8;
          *reinterpret_cast<uint4*>(swb + r * SWB + 8 * c) = v[u];
        } else if (k < total) {
          const int r = (k - n1) / t8, c = k - n1 - r * t8;
          *reinterpret_cast<uint4*>(swtb + r * STB + 8 * c) = v[u];
        }
      }
    }
  }
}

}  // namespace

template <int NNB, bool BF16>
__global__ void __launch_bounds__(256, NNB <= 4 ? 4 : 1) k_mlp_lds(EvalArgs a, int32_t groups_per_block) {
  extern __shared__ float4 mlp_lds[];
  const DevModel& M = a.M;
  const int64_t n_groups = a.rows_len / kRowGroup;
  const int64_t g_begin = (int64_t)blockIdx.x * groups_per_block;
  const int64_t g_end = min(g_begin + groups_per_block, n_groups);
  const int tid = threadIdx.x, lane = tid & 63, r0 = (tid >> 6) * 16;
  const int col = lane & 15, grp = lane >> 4;
  const int ND = M.ND, NNp = M.NNp, NDp = M.NDp, NDp32 = M.NDp32;
  const int K16 = nd_pad16(ND), KS = K16 / 4;
  const float* sw = reinterpret_cast<const float*>(mlp_lds);
  const uint16_t* hw = reinterpret_cast<const uint16_t*>(mlp_lds);
  const int SW = K16 + 4, ST = NNp + 4;
  const int SWB = NDp32 + 8, STB = NNp + 8;
  const float* st = sw + NNp * SW;
  const float* sbw = reinterpret_cast<const float*>(reinterpret_cast<const char*>(mlp_lds) +
                                                    mlp_weight_bytes(M, BF16));
  const uint16_t* swb = hw;
  const uint16_t* swtb = swb + NNp * SWB;
  // the bf16 kernel loads the next group's q while the current group is
  // computed; the float32 one loads each group's q when it starts (the
  // prefetch's 24 registers cost it a wave per SIMD)
  constexpr bool kPrefetch = BF16;
  float qn[kMlpQ];
  if (kPrefetch && g_begin < g_end) load_q<BF16>(a, a.rows[g_begin * kRowGroup + r0 + col], grp, KS, qn);
  int cur_net = -1;
  for (int64_t gi = g_begin; gi < g_end; ++gi) {
    const int64_t base = gi * kRowGroup;
    const int first = a.rows[base];
    if (first < 0) break;  // padding groups come after every species' rows
    const int net = M.nets > 1 ? a.types[first] : 0;
    if (net != cur_net) {  // the same for the whole block
      __syncthreads();     // every wave is done with the previous species
      stage_weights<BF16>(M, net, tid, mlp_lds);
      __syncthreads();
      cur_net = net;
    }
    const int atom = a.rows[base + r0 + col];
    float qv[kMlpQ];
    if constexpr (kPrefetch) {
#pragma unroll
      for (int k = 0; k < kMlpQ; ++k) qv[k] = qn[k];
      if (gi + 1 < g_end) load_q<BF16>(a, a.rows[base + kRowGroup + r0 + col], grp, KS, qn);
    } else {
      load_q<BF16>(a, atom, grp, KS, qv);
    }
    int out_atom[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) out_atom[r] = a.rows[base + r0 + 4 * grp + r];

    // ---- GEMM 1: acc[nb][r] = sum_k w0[16 nb + 4 grp + r][k] q[atom col][k] ----
    v4f acc[NNB];
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF16) {
#pragma unroll
      for (int v = 0; v < kMlpQ / 4; ++v) {
        if (4 * v >= KS) break;
        float4 w[NNB];
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb)
          w[nb] = *reinterpret_cast<const float4*>(sw + (16 * nb + col) * SW + KS * grp + 4 * v);
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[nb].x, qv[4 * v], acc[nb], 0, 0, 0);
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[nb].y, qv[4 * v + 1], acc[nb], 0, 0, 0);
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[nb].z, qv[4 * v + 2], acc[nb], 0, 0, 0);
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[nb].w, qv[4 * v + 3], acc[nb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < kMlpQ / 8; ++s) {
        if (32 * s >= NDp32) break;
        v8bf bq;
#pragma unroll
        for (int k = 0; k < 8; ++k) bq[k] = (__bf16)qv[8 * s + k];
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
          const uint4 u = *reinterpret_cast<const uint4*>(swb + (16 * nb + col) * SWB + 32 * s + 8 * grp);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf16x8_from_bits(u), bq, acc[nb], 0, 0, 0);
        }
      }
    }

    // ---- activation, site energy, latent vector and G = w1 (1 - h^2) ----
    float u = 0.f;
    float g[NNB][4];
    float* __restrict__ lat = (a.latent && atom >= 0) ? a.latent + (int64_t)atom * M.NN : nullptr;
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) {
      const float4 b4 = *reinterpret_cast<const float4*>(sbw + 16 * nb + 4 * grp);
      const float4 w4 = *reinterpret_cast<const float4*>(sbw + NNp + 16 * nb + 4 * grp);
      const float b0v[4] = {b4.x, b4.y, b4.z, b4.w}, w1v[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = 16 * nb + 4 * grp + r;
        const float h = tanh_net(acc[nb][r] - b0v[r]);
        const float wh = w1v[r] * h;
        u += wh;
        g[nb][r] = w1v[r] * (1.f - h * h);
        if (lat && mu < M.NN) lat[mu] = wh;
      }
    }
    u += __shfl_xor(u, 16);
    u += __shfl_xor(u, 32);
    if (grp == 0 && atom >= 0) a.U[atom] = u - *M.b1;

    // ---- GEMM 2: dU/dq[atom][d] = sum_mu G[atom][mu] w0[mu][d], two 16-column blocks at a time ----
    const int dblocks = (ND + 15) / 16;
    for (int db = 0; db < dblocks; db += 2) {
      const bool two = db + 1 < dblocks;
      v4f c0 = v4f{0.f, 0.f, 0.f, 0.f}, c1 = c0;
      const int d0 = 16 * db + col, d1 = d0 + 16;
      if constexpr (!BF16) {
        const float* row0 = st + d0 * ST;
        if (two) {
          const float* row1 = st + d1 * ST;
#pragma unroll
          for (int nb = 0; nb < NNB; ++nb) {
            const float4 x = *reinterpret_cast<const float4*>(row0 + 16 * nb + 4 * grp);
            const float4 y = *reinterpret_cast<const float4*>(row1 + 16 * nb + 4 * grp);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][0], x.x, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][0], y.x, c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][1], x.y, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][1], y.y, c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][2], x.z, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][2], y.z, c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][3], x.w, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][3], y.w, c1, 0, 0, 0);
          }
        } else {  // the last, unpaired column block
#pragma unroll
          for (int nb = 0; nb < NNB; ++nb) {
            const float4 x = *reinterpret_cast<const float4*>(row0 + 16 * nb + 4 * grp);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][0], x.x, c0, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][1], x.y, c0, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][2], x.z, c0, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(g[nb][3], x.w, c0, 0, 0, 0);
          }
        }
      } else {
        const uint16_t* row0 = swtb + (d0 < NDp32 ? d0 : 0) * STB;
        const uint16_t* row1 = swtb + (two && d1 < NDp32 ? d1 : 0) * STB;
#pragma unroll
        for (int p = 0; p < NNB / 2; ++p) {
          v8bf av, bv0, bv1;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            av[r] = (__bf16)g[2 * p][r];
            av[4 + r] = (__bf16)g[2 * p + 1][r];
          }
          bf16x4_from_bits(*reinterpret_cast<const uint2*>(row0 + 32 * p + 4 * grp), bv0, 0);
          bf16x4_from_bits(*reinterpret_cast<const uint2*>(row0 + 32 * p + 16 + 4 * grp), bv0, 4);
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv0, c0, 0, 0, 0);
          if (two) {
            bf16x4_from_bits(*reinterpret_cast<const uint2*>(row1 + 32 * p + 4 * grp), bv1, 0);
            bf16x4_from_bits(*reinterpret_cast<const uint2*>(row1 + 32 * p + 16 + 4 * grp), bv1, 4);
            c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv1, c1, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int at = out_atom[r];
        if (at < 0) continue;
        float* out = a.fp + (int64_t)at * NDp;
        if (d0 < ND) out[d0] = c0[r];
        if (two && d1 < ND) out[d1] = c1[r];
      }
    }
  }
}

void launch_mlp(const EvalArgs& a, hipStream_t s) {
  const int nnb = a.M.NNp / 16;
  const size_t lds = mlp_lds_bytes(a.M, a.mlp_bf16 != 0);
  const bool fits = a.mlp_bf16 ? a.M.NDp32 <= kMlpQ / 8 * 32 : nd_pad16(a.M.ND) <= 4 * kMlpMaxKS;
  if (lds <= kMlpMaxLds && fits) {
    // runs of consecutive row groups, about kMlpBlocks blocks in all
    const int64_t n_groups = a.rows_len / kRowGroup;
    const int32_t per = (int32_t)std::max<int64_t>(1, (n_groups + kMlpBlocks - 1) / kMlpBlocks);
    dim3 grid((unsigned)div_up(n_groups, per)), block(256);
    // (a block may take more than 64 KB of LDS on this chip when it asks for
    // it; if the request is refused, the global-memory kernel below runs)
#define NEP_MLP(n)                                                                                       \
  if (nnb == n) {                                                                                        \
    const void* k = a.mlp_bf16 ? (const void*)k_mlp_lds<n, true> : (const void*)k_mlp_lds<n, false>;    \
    if (lds <= 64 * 1024 ||                                                                              \
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess) {    \
      if (a.mlp_bf16) hipLaunchKernelGGL((k_mlp_lds<n, true>), grid, block, lds, s, a, per);             \
      else hipLaunchKernelGGL((k_mlp_lds<n, false>), grid, block, lds, s, a, per);                       \
      return;                                                                                            \
    }                                                                                                    \
    (void)hipGetLastError();                                                                             \
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
