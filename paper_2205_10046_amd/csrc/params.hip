// params.hip -- the float32 / bf16 model tables of many parameter vectors
// built on the device from their float64 vectors (the SNES population of
// Sec. II.E never leaves the GPU).  The tables are the same, bit for bit, as
// the ones the host builds for a single vector (api.cpp upload_model): the
// same layout, float64 -> float32 by round to nearest, bf16 by round to
// nearest even of the float32 value.
#include "nep_kernels.h"

namespace nep {

namespace {

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Value of network weight w0[t][mu][v] of the parameter vector (0 outside
// the N_neu x N_des block: padding neurons and padding descriptor slots).
__device__ __forceinline__ double w0_of(const double* p, const TableLayout& L, int t, int mu, int v) {
  if (mu >= L.NN || v >= L.ND) return 0.0;
  return p[(int64_t)t * (L.ND + 2) * L.NN + (int64_t)mu * L.ND + v];
}

}  // namespace

// One thread per table element of one parameter set (blockIdx.y = set).
__global__ void k_model_tables(const double* __restrict__ params, int64_t npar, TableLayout L,
                               unsigned char* __restrict__ base, int64_t set_stride) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double* p = params + (int64_t)blockIdx.y * npar;
  unsigned char* out = base + (int64_t)blockIdx.y * set_stride;
  int64_t k = g;
  // w0 [nets][NNp][ND] and w0t [nets][ND][NNp]
  const int64_t n_w0 = (int64_t)L.nets * L.NNp * L.ND;
  if (k < n_w0) {
    const int t = (int)(k / ((int64_t)L.NNp * L.ND)), r = (int)(k % ((int64_t)L.NNp * L.ND));
    const int mu = r / L.ND, v = r % L.ND;
    const float x = (float)w0_of(p, L, t, mu, v);
    ((float*)(out + L.at_w0))[k] = x;
    ((float*)(out + L.at_w0t))[((int64_t)t * L.ND + v) * L.NNp + mu] = x;
    return;
  }
  k -= n_w0;
  // b0 [nets][NNp] then b1; w1 [nets][NNp]
  const int64_t n_b = (int64_t)L.nets * L.NNp;
  if (k < n_b) {
    const int t = (int)(k / L.NNp), mu = (int)(k % L.NNp);
    const int64_t o = (int64_t)t * (L.ND + 2) * L.NN + (int64_t)L.NN * L.ND;
    ((float*)(out + L.at_b0))[k] = mu < L.NN ? (float)p[o + mu] : 0.f;
    ((float*)(out + L.at_w1))[k] = mu < L.NN ? (float)p[o + L.NN + mu] : 0.f;
    if (k == 0) ((float*)(out + L.at_b0))[n_b] = (float)p[L.off_b1];
    return;
  }
  k -= n_b;
  // bf16 w0b [nets][NNp][NDp32] and w0tb [nets][NDp32][NNp]
  const int64_t n_wb = (int64_t)L.nets * L.NNp * L.NDp32;
  if (k < n_wb) {
    const int t = (int)(k / ((int64_t)L.NNp * L.NDp32)), r = (int)(k % ((int64_t)L.NNp * L.NDp32));
    const int mu = r / L.NDp32, v = r % L.NDp32;
    const uint16_t b = bf16_bits((float)w0_of(p, L, t, mu, v));
    ((uint16_t*)(out + L.at_w0b))[k] = b;
    ((uint16_t*)(out + L.at_w0tb))[((int64_t)t * L.NDp32 + v) * L.NNp + mu] = b;
    return;
  }
  k -= n_wb;
  // radial coefficients c^R [T][T][nR][KR]
  const int64_t n_cR = (int64_t)L.T * L.T * L.nR * L.KR;
  if (k < n_cR) {
    ((float*)(out + L.at_cR))[k] = (float)p[L.off_cR + k];
    return;
  }
  k -= n_cR;
  // angular coefficients, one table per group size NG:
  // [T x T pairs, pair stride apart][groups][KA][ng_pad(NG)]
  if (k < L.n_cA) {
    int o = 0;
    while (o + 1 < L.n_ng && k >= L.cA_off_of[o + 1]) ++o;
    const int ng = L.ng_of[o], w = ng_pad(ng), ps = L.cA_pair_of[o];
    const int64_t r = k - L.cA_off_of[o];
    const int a = (int)(r / ps), q = (int)(r % ps);
    float x = 0.f;
    if (q < ((L.nA + ng - 1) / ng) * L.KA * w) {
      const int grp = q / (L.KA * w), rem = q % (L.KA * w), kk = rem / w, lane = rem % w;
      const int n = grp * ng + lane;
      if (lane < ng && n < L.nA) x = (float)p[L.off_cA + ((int64_t)a * L.nA + n) * L.KA + kk];
    }
    ((float*)(out + L.at_cA))[k] = x;
  }
}

int64_t table_elements(const TableLayout& L) {
  return (int64_t)L.nets * L.NNp * L.ND + (int64_t)L.nets * L.NNp + (int64_t)L.nets * L.NNp * L.NDp32 +
         (int64_t)L.T * L.T * L.nR * L.KR + L.n_cA;
}

void launch_model_tables(const double* params, int64_t npar, int32_t P, const TableLayout& L,
                         unsigned char* base, int64_t set_stride, hipStream_t s) {
  const int64_t n = table_elements(L);
  dim3 grid((unsigned)div_up(n, kBlock), (unsigned)P);
  hipLaunchKernelGGL(k_model_tables, grid, dim3(kBlock), 0, s, params, npar, L, base, set_stride);
}

}  // namespace nep
