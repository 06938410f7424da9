// descriptor.hip -- descriptor pass, partial-force pass and force/virial
// gather of NEP3 (Sec. II.B-II.F), one thread per atom.
//
// Both pair kernels run G lanes per atom (G = 1 or 4, adjacent lanes): lane
// s of an atom takes the row entries m = s, s + G, ...; the angular row is
// the first nnA entries of the radial row, so a lane owns the same entries
// in both loops.  More lanes per atom give more waves to hide the latency of
// the neighbour loads when N is small against the 1024 SIMDs; the per-lane
// partial sums are combined with DPP quad permutations.
//
// Descriptor pass (eqs. qin, g_n, f_n, S_nk and the explicit q_{nl},
// q_{n222}, q_{n1111}):
//   * radial: q_n = sum_j sum_k c^{t_i t_j}_{nk} f_k(r_ij) is regrouped as
//     sum_t sum_k c^{t_i t}_{nk} F_{t,k} with F_{t,k} = sum_{j of species t}
//     f_k(r_ij), accumulated in a per-thread LDS slot: K adds per bond instead
//     of n_R K multiply-adds;
//   * angular: g_n(r) for a group of NG radial functions and S_{n,k} += g_n b_k
//     held in registers (NG x NB accumulators), then q_{nl}, q_{n222},
//     q_{n1111} from S; S is kept (SoA) for the force pass.
// Partial-force pass (eq. partial_force): dU_i/dr_ij for every radial entry;
//   the radial part uses per-atom tables A_{t,k} = sum_n dU/dq_n c^{t_i t}_{nk},
//   and the angular part of a pair within r_c^A is added into the same slot
//   (the angular row maps into the radial row).
// Gather (eqs. F_ij, F_i, virial): F_i = sum_j dU_i/dr_ij - dU_j/dr_ji and
//   W_i = sum_j r_ij (x) dU_j/dr_ji over the radial row, reading dU_j/dr_ji
//   through the reverse index: no atomics, so results are bitwise
//   reproducible.
#include <type_traits>
#include <vector>

#include "angular.h"
#include "nep_kernels.h"

namespace nep {

namespace {

// Cutoff function and Chebyshev basis state for one bond.
struct Basis {
  float fc, dfc, x, dxdr;
};

__device__ __forceinline__ Basis make_basis(float r, float rc) {
  Basis b;
  const float rr = r * (1.0f / rc);
  // cos(pi r / rc) with the hardware cosine (argument in revolutions)
  b.fc = 0.5f + 0.5f * __builtin_amdgcn_cosf(0.5f * rr);
  b.dfc = -0.5f * (3.14159265358979f / rc) * __builtin_amdgcn_sinf(0.5f * rr);
  const float t = rr - 1.0f;
  b.x = 2.0f * t * t - 1.0f;
  b.dxdr = 4.0f * t * (1.0f / rc);
  return b;
}

// Sum of v over the G adjacent lanes of one atom (G in {1, 2, 4}); every
// lane of the group gets the same bits (the pairwise adds commute).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  if constexpr (G >= 4)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  return v;
}

// Visit row entries m = first, first + step, ... < nn of atom i with the
// neighbour loads software-pipelined: the index j of entry m + 2 step and the
// position and species of entry m + step are in flight while entry m is
// computed.  body(m, e, j, tj, dx, dy, dz) gets the float32 displacement
// rounded from the float64 one.  Entries past the row load atom 0 (always
// in bounds) and are never visited.
template <class Body>
__device__ __forceinline__ void for_entries(const EvalArgs& a, const StructInfo& st, int64_t i,
                                            int first, int nn, int step, Body&& body) {
  const int64_t N = a.N;
  const double* __restrict__ pos = a.pos;
  const int32_t* __restrict__ nl = a.L.nlR;
  const uint16_t* __restrict__ cd = a.L.cdR;
  const bool images = st.mode == kModeImages;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  auto index_of = [&](int m, uint16_t& code) -> int32_t {
    if (m >= nn) {
      code = kCodeCenter;
      return 0;
    }
    const int64_t e = (int64_t)m * N + i;
    code = images ? cd[e] : kCodeCenter;
    return nl[e];
  };
  uint16_t c0, c1;
  int32_t j0 = index_of(first, c0);
  int32_t j1 = index_of(first + step, c1);
  double px = pos[j0], py = pos[N + j0], pz = pos[2 * N + j0];
  int32_t t0 = a.types[j0];
  for (int m = first; m < nn; m += step) {
    const int32_t jc = j0, tc = t0;
    const uint16_t cc = c0;
    double Dx, Dy, Dz;
    {
#pragma clang fp contract(off)
      Dx = px - xi;
      Dy = py - yi;
      Dz = pz - zi;
    }
    j0 = j1;
    c0 = c1;
    px = pos[j0];
    py = pos[N + j0];
    pz = pos[2 * N + j0];
    t0 = a.types[j0];
    j1 = index_of(m + 2 * step, c1);
    int n0, n1, n2;
    min_image(st, Dx, Dy, Dz, n0, n1, n2);
    if (cc != kCodeCenter) {
      int oa, ob, oc;
      split_code(cc, oa, ob, oc);
      n0 += oa;
      n1 += ob;
      n2 += oc;
    }
    double dx, dy, dz;
    image_disp(st, Dx, Dy, Dz, n0, n1, n2, dx, dy, dz);
    body(m, (int64_t)m * N + i, jc, tc, (float)dx, (float)dy, (float)dz);
  }
}

template <bool BATCH>
__device__ __forceinline__ const StructInfo& struct_of(const EvalArgs& a, const StructInfo& st0,
                                                       int64_t i) {
  if constexpr (BATCH) return a.structs[a.sid[i]];
  else return st0;
}

// LDS: radial table [T][T][nR][KR] (rounded to 16 bytes), the angular table
// of group size NG, then per-lane slots.
__device__ __forceinline__ int radial_table_floats(const DevModel& M) {
  return round4(M.T * M.T * M.nR * M.KR);
}

template <int NG>
__device__ __forceinline__ void load_tables(const DevModel& M, int ngroups, float* sR, float* sA) {
  const int nRt = M.T * M.T * M.nR * M.KR;
  const int nAt = M.T * M.T * M.cA_pair[NG];
  const float* cA = M.cA + M.cA_off[NG];
  for (int k = threadIdx.x; k < nRt; k += blockDim.x) sR[k] = M.cR[k];
  for (int k = threadIdx.x; k < nAt; k += blockDim.x) sA[k] = cA[k];
}

// The NG coefficients of one group at one basis index (16-byte aligned rows).
template <int NG>
__device__ __forceinline__ void load_group(const float* p, float (&c)[NG]) {
  constexpr int W = ng_pad(NG);
  if constexpr (W % 4 == 0) {
#pragma unroll
    for (int v = 0; v < W / 4; ++v) {
      const float4 x = reinterpret_cast<const float4*>(p)[v];
      const float e[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * v + u < NG) c[4 * v + u] = e[u];
    }
  } else if constexpr (W == 2) {
    const float2 x = *reinterpret_cast<const float2*>(p);
    c[0] = x.x;
    c[1] = x.y;
  } else {
#pragma unroll
    for (int q = 0; q < NG; ++q) c[q] = p[q];
  }
}

}  // namespace

size_t eval_lds_bytes(const DevModel& M, int block) {
  size_t t = (size_t)round4(M.T * M.T * M.nR * M.KR) + (size_t)round4(M.cA_max);
  return (t + (size_t)M.T * M.KR * block) * sizeof(float);
}

// ---------------------------------------------------------------------------
// descriptor pass
// ---------------------------------------------------------------------------

// Basis sizes the descriptor and force kernels can take as constants: shape 1 is n_R = K_R =
// 9 and n_A = K_A = 7 (n_max 8/6 with N_bas 8/6); with them the basis loops
// have fixed trip counts (no per-iteration exit test) and the same arithmetic
// in the same order, so the results are the same bits as with shape 0, which
// reads the sizes from the model.
template <int S> struct BasisShape {
  static constexpr int nR = 0, KR = 0, nA = 0, KA = 0;
};
template <> struct BasisShape<1> {
  static constexpr int nR = 9, KR = 9, nA = 7, KA = 7;
};


// species whose radial sums the descriptor kernel can keep in registers
constexpr int kRegTypes = 4;

template <int NG, int L, bool BATCH, int G, int SH = 0>
__global__ void __launch_bounds__(kBlock, 2) k_descriptor(EvalArgs a, StructInfo st0) {
  constexpr int NB = num_poly(L);
  extern __shared__ float4 lds_v4[];  // 16-byte aligned base
  float* lds = reinterpret_cast<float*>(lds_v4);
  const DevModel& M = a.M;
  using Sh = BasisShape<SH>;
  const int T = M.T;
  const int KR = SH ? Sh::KR : M.KR, KA = SH ? Sh::KA : M.KA, nR = SH ? Sh::nR : M.nR, nA = SH ? Sh::nA : M.nA;
  const int ngroups = SH ? (Sh::nA + NG - 1) / NG : a.ngroups;
  constexpr int W = ng_pad(NG);
  float* sR = lds;
  float* sA = sR + radial_table_floats(M);
  float* acc = sA + round4(T * T * M.cA_pair[NG]);
  load_tables<NG>(M, a.ngroups, sR, sA);
  const int tid = threadIdx.x, B = blockDim.x;
  for (int k = 0; k < T * KR; ++k) acc[k * B + tid] = 0.f;
  __syncthreads();
  const int64_t N = a.N;
  const int sub = tid & (G - 1);
  const int64_t i = (xcd_block() * B + tid) / G;
  if (i >= N) return;  // the G lanes of an atom leave together
  const StructInfo& st = struct_of<BATCH>(a, st0, i);
  const int ti = a.types[i];
  const double* __restrict__ pos = a.pos;
  const int32_t* __restrict__ nl = a.L.nlR;
  const uint16_t* __restrict__ cd = a.L.cdR;
  float* __restrict__ qrow = a.q + i * M.NDp;

  // ---- radial: F_{t,k} = sum_{j of species t} f_k(r_ij) ----
  const float rcR = M.rcR;
  const int nnR = min(a.L.nnR[i], a.L.MR);
  // q_n = sum_t sum_k c^{t_i t}_{nk} F_{t,k}: each F read once, all n in registers
  float qr[kMaxBasis];
#pragma unroll
  for (int n = 0; n < kMaxBasis; ++n) qr[n] = 0.f;
  auto contract = [&](int t, int k, float F) __attribute__((always_inline)) {
    const float* c = sR + (ti * T + t) * nR * KR + k;
#pragma unroll
    for (int n = 0; n < kMaxBasis; ++n) {
      if (n >= nR) break;
      qr[n] += c[n * KR] * F;
    }
  };
  if (SH != 0 && T <= kRegTypes) {
    // fixed basis size and at most four species: the sums F_{t,k} in
    // registers (an entry adds to its species' row and zero to the others,
    // the same sums in the same order as the LDS slots)
    constexpr int KRc = SH ? Sh::KR : 1;
    float ar[kRegTypes][KRc];
#pragma unroll
    for (int t = 0; t < kRegTypes; ++t)
#pragma unroll
      for (int k = 0; k < KRc; ++k) ar[t][k] = 0.f;
    for_entries(a, st, i, sub, nnR, G,
                [&](int m, int64_t e, int32_t j, int32_t tj, float fx, float fy, float fz)
                    __attribute__((always_inline)) {
      const float r = sqrtf(fx * fx + fy * fy + fz * fz);
      const Basis bs = make_basis(r, rcR);
      float v[KRc];
      v[0] = bs.fc;
      float Tm1 = 1.f, Tk = bs.x;
#pragma unroll
      for (int k = 1; k < KRc; ++k) {
        v[k] = 0.5f * (Tk + 1.f) * bs.fc;
        const float Tn = 2.f * bs.x * Tk - Tm1;
        Tm1 = Tk;
        Tk = Tn;
      }
#pragma unroll
      for (int t = 0; t < kRegTypes; ++t)
#pragma unroll
        for (int k = 0; k < KRc; ++k) ar[t][k] += tj == t ? v[k] : 0.f;
    });
#pragma unroll
    for (int t = 0; t < kRegTypes; ++t) {
      if (t >= T) break;
#pragma unroll
      for (int k = 0; k < KRc; ++k) contract(t, k, group_sum<G>(ar[t][k]));
    }
  } else {
    for_entries(a, st, i, sub, nnR, G,
                [&](int m, int64_t e, int32_t j, int32_t tj, float fx, float fy, float fz)
                    __attribute__((always_inline)) {
      const float r = sqrtf(fx * fx + fy * fy + fz * fz);
      const Basis bs = make_basis(r, rcR);
      float* slot = acc + (tj * KR) * B + tid;
      slot[0] += bs.fc;
      float Tm1 = 1.f, Tk = bs.x;
#pragma unroll
      for (int k = 1; k < kMaxBasis; ++k) {
        if (k >= KR) break;
        slot[k * B] += 0.5f * (Tk + 1.f) * bs.fc;
        const float Tn = 2.f * bs.x * Tk - Tm1;
        Tm1 = Tk;
        Tk = Tn;
      }
    });
    if constexpr (G > 1)
      for (int k = 0; k < T * KR; ++k) acc[k * B + tid] = group_sum<G>(acc[k * B + tid]);
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < KR; ++k) contract(t, k, acc[(t * KR + k) * B + tid]);
  }
#pragma unroll
  for (int n = 0; n < kMaxBasis; ++n)
    if (n < nR && n % G == sub) qrow[n] = qr[n];

  // ---- angular: S_{n,k} = sum_j g_n(r_ij) b_k(u_ij), NG radial functions at a time ----
  const float rcA = M.rcA;
  const int nnA = min(a.L.nnA[i], a.L.MR);
  for (int g = 0; g < ngroups; ++g) {
    float S[NG][NB];
#pragma unroll
    for (int q = 0; q < NG; ++q)
#pragma unroll
      for (int k = 0; k < NB; ++k) S[q][k] = 0.f;
    for_entries(a, st, i, sub, nnA, G,
                [&](int m, int64_t e, int32_t j, int32_t tj, float fx, float fy, float fz)
                    __attribute__((always_inline)) {
      const float r = sqrtf(fx * fx + fy * fy + fz * fz);
      const float rinv = 1.0f / r;
      const Basis bs = make_basis(r, rcA);
      const float* c = sA + (ti * T + tj) * M.cA_pair[NG] + g * KA * W;
      float gq[NG];
      {
        float cv[NG];
        load_group<NG>(c, cv);
#pragma unroll
        for (int q = 0; q < NG; ++q) gq[q] = cv[q] * bs.fc;
      }
      float Tm1 = 1.f, Tk = bs.x;
#pragma unroll
      for (int k = 1; k < kMaxBasis; ++k) {
        if (k >= KA) break;
        float cv[NG];
        load_group<NG>(c + k * W, cv);
        const float f = 0.5f * (Tk + 1.f) * bs.fc;
#pragma unroll
        for (int q = 0; q < NG; ++q) gq[q] += cv[q] * f;
        const float Tn = 2.f * bs.x * Tk - Tm1;
        Tm1 = Tk;
        Tk = Tn;
      }
      angular_values<L>(fx * rinv, fy * rinv, fz * rinv,
                        [&](int k, float b) __attribute__((always_inline)) {
#pragma unroll
                          for (int q = 0; q < NG; ++q) S[q][k] += gq[q] * b;
                        });
    });
    if constexpr (G > 1) {
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int k = 0; k < NB; ++k) S[q][k] = group_sum<G>(S[q][k]);
    }
    // q_{nl} = sum_{k in l} C3_k S_{nk}^2 ; q_{n222} ; q_{n1111}
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int n = g * NG + q;
      if (n >= nA) break;
      float* sums = a.sums + (int64_t)(n * NB) * N + i;
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k % G == sub) sums[(int64_t)k * N] = S[q][k];
      if (q % G != sub) continue;
      float v[L];
#pragma unroll
      for (int l = 0; l < L; ++l) v[l] = 0.f;
#pragma unroll
      for (int k = 0; k < NB; ++k) v[degree_of(k) - 1] += M.C3[k] * S[q][k] * S[q][k];
#pragma unroll
      for (int l = 1; l <= L; ++l) qrow[nR + (l - 1) * nA + n] = v[l - 1];
      if constexpr (L >= 2) {
        if (M.has4b) {
          const float* s = S[q];
          const float v = M.C4[0] * s[3] * s[3] * s[3] + M.C4[1] * s[3] * (s[4] * s[4] + s[5] * s[5]) +
                          M.C4[2] * s[3] * (s[6] * s[6] + s[7] * s[7]) +
                          M.C4[3] * s[6] * (s[5] * s[5] - s[4] * s[4]) + M.C4[4] * s[4] * s[5] * s[7];
          qrow[nR + L * nA + n] = v;
        }
      }
      if (M.has5b) {
        const float* s = S[q];
        const float s12 = s[1] * s[1] + s[2] * s[2];
        const float v = M.C5[0] * s[0] * s[0] * s[0] * s[0] + M.C5[1] * s[0] * s[0] * s12 +
                        M.C5[2] * s12 * s12;
        qrow[nR + (L + M.has4b) * nA + n] = v;
      }
    }
  }
  if (sub == 0)
    for (int c = M.ND; c < M.NDp; ++c) qrow[c] = 0.f;
}

// ---------------------------------------------------------------------------
// partial forces dU_i/dr_ij (eq. partial_force)
// ---------------------------------------------------------------------------

// Large accumulator blocks (NG x NB > 120 floats) run at one wave per SIMD so
// the compiler can keep the D block in registers instead of spilling.
template <int NG, int L, bool BATCH, int G, int S = 0>
__global__ void __launch_bounds__(kBlock, (NG * num_poly(L) > 120) ? 1 : 2)
    k_partial_forces(EvalArgs a, StructInfo st0) {
  constexpr int NB = num_poly(L);
  extern __shared__ float4 lds_v4[];  // 16-byte aligned base
  float* lds = reinterpret_cast<float*>(lds_v4);
  const DevModel& M = a.M;
  using Sh = BasisShape<S>;
  const int T = M.T;
  const int KR = S ? Sh::KR : M.KR, KA = S ? Sh::KA : M.KA;
  const int nR = S ? Sh::nR : M.nR, nA = S ? Sh::nA : M.nA;
  constexpr int W = ng_pad(NG);
  float* sR = lds;
  float* sA = sR + radial_table_floats(M);
  float* At = sA + round4(T * T * M.cA_pair[NG]);
  load_tables<NG>(M, a.ngroups, sR, sA);
  __syncthreads();
  const int tid = threadIdx.x, B = blockDim.x;
  const int64_t N = a.N;
  const int sub = tid & (G - 1);
  const int64_t i = (xcd_block() * B + tid) / G;
  if (i >= N) return;
  const StructInfo& st = struct_of<BATCH>(a, st0, i);
  const int ti = a.types[i];
  const double* __restrict__ pos = a.pos;
  const int32_t* __restrict__ nl = a.L.nlR;
  const uint16_t* __restrict__ cd = a.L.cdR;
  const float* __restrict__ fprow = a.fp + i * M.NDp;

  // ---- radial: A_{t,k} = sum_n dU/dq_n c^{t_i t}_{nk}; dU_i/dr_ij = (sum_k A f'_k) u ----
  float fpr[kMaxBasis];  // dU/dq_n of the radial descriptors, loaded once
#pragma unroll
  for (int n = 0; n < kMaxBasis; ++n) fpr[n] = n < nR ? fprow[n] : 0.f;
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < KR; ++k) {
      const float* c = sR + (ti * T + t) * nR * KR + k;
      float s = 0.f;
#pragma unroll
      for (int n = 0; n < kMaxBasis; ++n) {
        if (n >= nR) break;
        s += fpr[n] * c[n * KR];
      }
      At[(t * KR + k) * B + tid] = s;
    }
  const float rcR = M.rcR;
  const int nnR = min(a.L.nnR[i], a.L.MR);
  const int nnA = min(a.L.nnA[i], a.L.MR);
  // radial scalar s with dU_i/dr_ij (radial part) = s * r_ij
  auto radial_scalar = [&](int32_t tj, float r, float rinv) __attribute__((always_inline)) {
    const Basis bs = make_basis(r, rcR);
    const float* At_j = At + (tj * KR) * B + tid;
    // f'_k = 1/2 T'_k x' f_c + 1/2 (T_k + 1) f_c'
    float s = At_j[0] * bs.dfc;
    float Tm1 = 1.f, Tk = bs.x, dTm1 = 0.f, dTk = 1.f;
#pragma unroll
    for (int k = 1; k < kMaxBasis; ++k) {
      if (k >= KR) break;
      const float df = 0.5f * dTk * bs.dxdr * bs.fc + 0.5f * (Tk + 1.f) * bs.dfc;
      s += At_j[k * B] * df;
      const float Tn = 2.f * bs.x * Tk - Tm1;
      const float dTn = 2.f * Tk + 2.f * bs.x * dTk - dTm1;
      Tm1 = Tk;
      Tk = Tn;
      dTm1 = dTk;
      dTk = dTn;
    }
    return s * rinv;
  };
  // entries past the angular prefix: radial part only (the prefix gets its
  // radial part in the first angular pass below); first such m of this lane
  const int m_outer = sub + (nnA > sub ? (nnA - sub + G - 1) / G * G : 0);
  for_entries(a, st, i, m_outer, nnR, G,
              [&](int m, int64_t e, int32_t j, int32_t tj, float fx, float fy, float fz)
                  __attribute__((always_inline)) {
    const float r = sqrtf(fx * fx + fy * fy + fz * fz);
    const float s = radial_scalar(tj, r, 1.0f / r);
    a.P[e] = make_float4(s * fx, s * fy, s * fz, 0.f);
  });

  // ---- angular: sum_{n,k} D_{nk} [g'_n u b_k + g_n d b_k / d r_ij] ----
  const float rcA = M.rcA;
  // one pass over the angular bonds per group of radial functions; NQ of
  // the group's NG are live (fewer in the last group when NG does not divide
  // n_A and the basis sizes are constants; for l_max <= 4 only: with the larger
  // polynomial sets the second body costs more registers than it saves)
  auto angular_group = [&](auto nq, int g) __attribute__((always_inline)) {
    constexpr int NQ = decltype(nq)::value;
    // D_{nk} = dU/dS_{nk} through q_{nl}, q_{n222}, q_{n1111}
    float D[NQ][NB];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int n = min(g * NG + q, nA - 1);
      const bool live = g * NG + q < nA;
      const float* sums = a.sums + (int64_t)(n * NB) * N + i;
      float s[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) s[k] = sums[(int64_t)k * N];
      float f3[L];
#pragma unroll
      for (int l = 1; l <= L; ++l) f3[l - 1] = live ? fprow[nR + (l - 1) * nA + n] : 0.f;
#pragma unroll
      for (int k = 0; k < NB; ++k) D[q][k] = 2.f * M.C3[k] * f3[degree_of(k) - 1] * s[k];
      if constexpr (L >= 2) {
        if (M.has4b) {
          const float f = live ? fprow[nR + L * nA + n] : 0.f;
          const float* C = M.C4;
          D[q][3] += f * (3.f * C[0] * s[3] * s[3] + C[1] * (s[4] * s[4] + s[5] * s[5]) +
                          C[2] * (s[6] * s[6] + s[7] * s[7]));
          D[q][4] += f * (2.f * C[1] * s[3] * s[4] - 2.f * C[3] * s[6] * s[4] + C[4] * s[5] * s[7]);
          D[q][5] += f * (2.f * C[1] * s[3] * s[5] + 2.f * C[3] * s[6] * s[5] + C[4] * s[4] * s[7]);
          D[q][6] += f * (2.f * C[2] * s[3] * s[6] + C[3] * (s[5] * s[5] - s[4] * s[4]));
          D[q][7] += f * (2.f * C[2] * s[3] * s[7] + C[4] * s[4] * s[5]);
        }
      }
      if (M.has5b) {
        const float f = live ? fprow[nR + (L + M.has4b) * nA + n] : 0.f;
        const float* C = M.C5;
        const float s12 = s[1] * s[1] + s[2] * s[2];
        D[q][0] += f * (4.f * C[0] * s[0] * s[0] * s[0] + 2.f * C[1] * s[0] * s12);
        D[q][1] += f * (2.f * C[1] * s[0] * s[0] * s[1] + 4.f * C[2] * s12 * s[1]);
        D[q][2] += f * (2.f * C[1] * s[0] * s[0] * s[2] + 4.f * C[2] * s12 * s[2]);
      }
    }
    for_entries(a, st, i, sub, nnA, G,
                [&](int m, int64_t e, int32_t j, int32_t tj, float fx, float fy, float fz)
                    __attribute__((always_inline)) {
      const float r = sqrtf(fx * fx + fy * fy + fz * fz);
      const float rinv = 1.0f / r;
      const float ux = fx * rinv, uy = fy * rinv, uz = fz * rinv;
      const Basis bs = make_basis(r, rcA);
      const float* c = sA + (ti * T + tj) * M.cA_pair[NG] + g * KA * W;
      float gq[NQ], dgq[NQ];
      {
        float cv[NQ];
        load_group<NQ>(c, cv);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          gq[q] = cv[q] * bs.fc;
          dgq[q] = cv[q] * bs.dfc;
        }
      }
      float Tm1 = 1.f, Tk = bs.x, dTm1 = 0.f, dTk = 1.f;
#pragma unroll
      for (int k = 1; k < kMaxBasis; ++k) {
        if (k >= KA) break;
        float cv[NQ];
        load_group<NQ>(c + k * W, cv);
        const float f = 0.5f * (Tk + 1.f) * bs.fc;
        const float df = 0.5f * dTk * bs.dxdr * bs.fc + 0.5f * (Tk + 1.f) * bs.dfc;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          gq[q] += cv[q] * f;
          dgq[q] += cv[q] * df;
        }
        const float Tn = 2.f * bs.x * Tk - Tm1;
        const float dTn = 2.f * Tk + 2.f * bs.x * dTk - dTm1;
        Tm1 = Tk;
        Tk = Tn;
        dTm1 = dTk;
        dTk = dTn;
      }
      float E[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) E[q] = 0.f;
      float Vx = 0.f, Vy = 0.f, Vz = 0.f;
      angular_terms<L>(ux, uy, uz,
                       [&](int k, float b, float gx, float gy, float gz)
                           __attribute__((always_inline)) {
                             float w = 0.f;
#pragma unroll
                             for (int q = 0; q < NQ; ++q) {
                               w += gq[q] * D[q][k];
                               E[q] += D[q][k] * b;
                             }
                             Vx += w * gx;
                             Vy += w * gy;
                             Vz += w * gz;
                           });
      float s = 0.f;
#pragma unroll
      for (int q = 0; q < NQ; ++q) s += dgq[q] * E[q];
      const float uV = ux * Vx + uy * Vy + uz * Vz;
      const float px = s * ux + (Vx - uV * ux) * rinv;
      const float py = s * uy + (Vy - uV * uy) * rinv;
      const float pz = s * uz + (Vz - uV * uz) * rinv;
      // the first pass adds the radial part of the pair (same rounding order
      // as radial first, then each angular group); later passes update it
      float4 v;
      if (g == 0) {
        const float sr = radial_scalar(tj, r, rinv);
        v = make_float4(sr * fx, sr * fy, sr * fz, 0.f);
      } else {
        v = a.P[e];
      }
      v.x += px;
      v.y += py;
      v.z += pz;
      a.P[e] = v;
    });
  };
  if constexpr (S != 0 && L <= 4) {
    constexpr int NGR = (Sh::nA + NG - 1) / NG, NL = Sh::nA - (NGR - 1) * NG;
    for (int g = 0; g < NGR - 1; ++g) angular_group(std::integral_constant<int, NG>{}, g);
    angular_group(std::integral_constant<int, NL>{}, NGR - 1);
  } else {
    for (int g = 0; g < a.ngroups; ++g) angular_group(std::integral_constant<int, NG>{}, g);
  }
}

// ---------------------------------------------------------------------------
// force and virial gather (eqs. F_ij, F_i, virial)
// ---------------------------------------------------------------------------

// G lanes per atom (1 or 4) walk its radial row (lane s takes entries
// s, s + G, ...); dU_j/dr_ji sits at position rev[m][i] of row j.  The index
// words of a lane's entry after next and the partial forces (and neighbour
// position, for the virial) of its next entry are loaded while the current
// one is accumulated; the lane sums are combined with DPP quad sums.
// VIRIAL = false leaves W untouched (MD steps without a thermo row).
template <bool BATCH, bool VIRIAL, int G>
__global__ void __launch_bounds__(kBlock) k_gather(EvalArgs a, StructInfo st0) {
  const int64_t N = a.N;
  const int sub = threadIdx.x & (G - 1);
  const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / G;
  if (i >= N) return;  // the lanes of an atom leave together
  const StructInfo& st = struct_of<BATCH>(a, st0, i);
  const int nn = min(a.L.nnR[i], a.L.MR);
  const double* __restrict__ pos = a.pos;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  struct Words {
    int32_t j, r;
    uint16_t code;
  };
  auto words = [&](int m) -> Words {
    Words w{0, 0, kCodeCenter};
    if (m < nn) {
      const int64_t e = (int64_t)m * N + i;
      w.j = a.L.nlR[e];
      w.r = a.L.revR[e];
      if (VIRIAL && st.mode == kModeImages) w.code = a.L.cdR[e];
    }
    return w;
  };
  Words w0 = words(sub), w1 = words(sub + G);
  float4 pij = a.P[(int64_t)min(sub, max(nn - 1, 0)) * N + i];
  float4 pji = a.P[(int64_t)w0.r * N + w0.j];
  double px = 0.0, py = 0.0, pz = 0.0;
  if (VIRIAL) {
    px = pos[w0.j];
    py = pos[N + w0.j];
    pz = pos[2 * N + w0.j];
  }
  float F[3] = {0.f, 0.f, 0.f}, W[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int m = sub; m < nn; m += G) {
    const Words c = w0;
    const float4 cij = pij, cji = pji;
    const double cx = px, cy = py, cz = pz;
    w0 = w1;
    w1 = words(m + 2 * G);
    pij = a.P[(int64_t)min(m + G, nn - 1) * N + i];
    pji = a.P[(int64_t)w0.r * N + w0.j];
    if (VIRIAL) {
      px = pos[w0.j];
      py = pos[N + w0.j];
      pz = pos[2 * N + w0.j];
    }
    F[0] += cij.x - cji.x;
    F[1] += cij.y - cji.y;
    F[2] += cij.z - cji.z;
    if constexpr (VIRIAL) {
      double Dx, Dy, Dz;
      {
#pragma clang fp contract(off)
        Dx = cx - xi;
        Dy = cy - yi;
        Dz = cz - zi;
      }
      int n0, n1, n2;
      min_image(st, Dx, Dy, Dz, n0, n1, n2);
      if (c.code != kCodeCenter) {
        int oa, ob, oc;
        split_code(c.code, oa, ob, oc);
        n0 += oa;
        n1 += ob;
        n2 += oc;
      }
      double dx, dy, dz;
      image_disp(st, Dx, Dy, Dz, n0, n1, n2, dx, dy, dz);
      const float d[3] = {(float)dx, (float)dy, (float)dz};
      const float q[3] = {cji.x, cji.y, cji.z};
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) W[x * 3 + y] += d[x] * q[y];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float v = group_sum<G>(F[c]);
    if (c % G == sub) {
      a.F[(int64_t)c * N + i] = v;
      if (a.kick_vel) a.kick_vel[(int64_t)c * N + i] += 0.5 * a.kick_dt * a.kick_inv_mass[a.types[i]] * (double)v;
    }
  }
  if constexpr (VIRIAL) {
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      const float x = group_sum<G>(W[v]);
      if (v % G == sub) a.W[(int64_t)v * N + i] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

// Admissible group sizes NG for n_A radial functions at a given l_max: the
// accumulator block NG x NB must fit the register budget.  The default is the
// one with the least padded work, then the fewest passes over the bonds; the
// autotuner in api.cpp may pick another one by timing.
std::vector<int> angular_group_options(int nA, int L) {
  const int cap = L <= 4 ? 7 : (L == 5 ? 5 : 4);
  static const int allowed[] = {2, 4, 5, 7};
  std::vector<int> out;
  for (int ng : allowed)
    if (ng <= cap && (ng <= nA || ng == 2)) out.push_back(ng);
  if (out.empty()) out.push_back(2);
  return out;
}

int angular_group_size(int nA, int L) {
  int best = -1, best_cost = 1 << 30;
  for (int ng : angular_group_options(nA, L)) {
    int groups = (nA + ng - 1) / ng;
    int cost = groups * ng * 4 + groups;  // padded work, then fewer passes
    if (cost < best_cost) {
      best_cost = cost;
      best = ng;
    }
  }
  return best;
}

template <int NG, int L, bool BATCH, int G, int S>
static bool launch_pair_g(const EvalArgs& a, const StructInfo& st0, bool force, hipStream_t s) {
  const int block = a.block > 0 ? a.block : kBlock;
  const size_t lds = eval_lds_bytes(a.M, block);
  // the kernels' LDS layout: radial table, the angular table of this group
  // size, then T K_R per-lane slots; refuse a shape it does not fit
  const DevModel& M = a.M;
  if (M.cA_off[NG] < 0 || block % 64 != 0 || block > kBlock) return false;
  const size_t need = ((size_t)round4(M.T * M.T * M.nR * M.KR) + (size_t)round4(M.T * M.T * M.cA_pair[NG]) +
                       (size_t)M.T * M.KR * block) * sizeof(float);
  if (need > lds || lds > 64 * 1024) return false;
  dim3 grid((unsigned)div_up(a.N * G, block));
  if (force)
    hipLaunchKernelGGL((k_partial_forces<NG, L, BATCH, G, S>), grid, dim3(block), lds, s, a, st0);
  else
    hipLaunchKernelGGL((k_descriptor<NG, L, BATCH, G, S>), grid, dim3(block), lds, s, a, st0);
  return true;
}

template <int NG, int L, bool BATCH>
static bool launch_pair(const EvalArgs& a, const StructInfo& st0, bool force, hipStream_t s) {
  const DevModel& M = a.M;
  const bool shape1 = M.nR == BasisShape<1>::nR && M.KR == BasisShape<1>::KR &&
                      M.nA == BasisShape<1>::nA && M.KA == BasisShape<1>::KA;
  if (shape1) {
    if (a.lanes == 4) return launch_pair_g<NG, L, BATCH, 4, 1>(a, st0, force, s);
    return launch_pair_g<NG, L, BATCH, 1, 1>(a, st0, force, s);
  }
  if (a.lanes == 4) return launch_pair_g<NG, L, BATCH, 4, 0>(a, st0, force, s);
  return launch_pair_g<NG, L, BATCH, 1, 0>(a, st0, force, s);
}

template <bool BATCH>
static bool dispatch(const EvalArgs& a, const StructInfo& st0, bool force, hipStream_t s) {
  const int L = a.M.L, NG = a.NG;
  if (a.lanes != 1 && a.lanes != 4) return false;
#define NEP_CASE(ng, l) \
  if (NG == ng && L == l) return launch_pair<ng, l, BATCH>(a, st0, force, s);
  NEP_CASE(2, 1) NEP_CASE(4, 1) NEP_CASE(5, 1) NEP_CASE(7, 1)
  NEP_CASE(2, 2) NEP_CASE(4, 2) NEP_CASE(5, 2) NEP_CASE(7, 2)
  NEP_CASE(2, 3) NEP_CASE(4, 3) NEP_CASE(5, 3) NEP_CASE(7, 3)
  NEP_CASE(2, 4) NEP_CASE(4, 4) NEP_CASE(5, 4) NEP_CASE(7, 4)
  NEP_CASE(2, 5) NEP_CASE(4, 5) NEP_CASE(5, 5)
  NEP_CASE(2, 6) NEP_CASE(4, 6)
#undef NEP_CASE
  return false;
}

bool launch_descriptor(const EvalArgs& a, hipStream_t s) {
  return a.batch ? dispatch<true>(a, a.st0, false, s) : dispatch<false>(a, a.st0, false, s);
}

bool launch_partial_forces(const EvalArgs& a, hipStream_t s) {
  return a.batch ? dispatch<true>(a, a.st0, true, s) : dispatch<false>(a, a.st0, true, s);
}

template <int G>
static void launch_gather_g(const EvalArgs& a, bool virial, hipStream_t s) {
  dim3 grid((unsigned)div_up(a.N * G, kBlock));
  if (a.batch) {
    if (virial) hipLaunchKernelGGL((k_gather<true, true, G>), grid, dim3(kBlock), 0, s, a, a.st0);
    else hipLaunchKernelGGL((k_gather<true, false, G>), grid, dim3(kBlock), 0, s, a, a.st0);
  } else {
    if (virial) hipLaunchKernelGGL((k_gather<false, true, G>), grid, dim3(kBlock), 0, s, a, a.st0);
    else hipLaunchKernelGGL((k_gather<false, false, G>), grid, dim3(kBlock), 0, s, a, a.st0);
  }
}

void launch_gather_forces(const EvalArgs& a, bool virial, hipStream_t s) {
  if (a.lanes == 4) launch_gather_g<4>(a, virial, s);
  else launch_gather_g<1>(a, virial, s);
}

}  // namespace nep
