// ensemble.hip -- thermostats and barostats for the NVT and NPT ensembles the
// paper lists for its MD driver (Sec. II.F), each after its publication:
//   Berendsen thermostat and barostat (Berendsen et al. 1984);
//   stochastic velocity rescaling (Bussi, Donadio, Parrinello 2007);
//   Langevin dynamics in the Bussi-Parrinello (2007) splitting;
//   Nose-Hoover chain (Martyna, Klein, Tuckerman 1992), Trotter-split;
//   stochastic cell rescaling (Bernetti, Bussi 2020), isotropic.
// All scalar state (kinetic energy, chain, heat, box scale, step counter)
// lives in one device block, so a step is a fixed kernel sequence that a
// HIP graph can replay; every reduction is a fixed-order float64 tree.
// Random numbers are Philox4x32-10 (Salmon et al. 2011) of the counter
// (index, step, stream, 0) under the 64-bit seed, turned into normals by
// Box-Muller; the index of a per-atom draw is the caller's atom index, so
// the draws do not depend on the internal atom order.
#include "nep_kernels.h"

namespace nep {

namespace {

constexpr int kEnsRed = 256;
constexpr double kGPa = 160.21766208;  // 1 eV/A^3 in GPa

// ---- Philox4x32-10 ----
struct U4 {
  uint32_t w[4];
};

__device__ __forceinline__ U4 philox(uint32_t index, uint32_t step, uint32_t stream, uint64_t seed) {
  uint32_t x0 = index, x1 = step, x2 = stream, x3 = 0u;
  uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo_a = 0xD2511F53u * x0, hi_a = __umulhi(0xD2511F53u, x0);
    const uint32_t lo_b = 0xCD9E8D57u * x2, hi_b = __umulhi(0xCD9E8D57u, x2);
    const uint32_t y0 = hi_b ^ x1 ^ k0, y2 = hi_a ^ x3 ^ k1;
    x0 = y0;
    x1 = lo_b;
    x2 = y2;
    x3 = lo_a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{{x0, x1, x2, x3}};
}

// Normals z[0..3] from one Philox call: words (0, 1) and (2, 3) are each a
// pair of uniforms (w + 1/2) 2^-32 for one Box-Muller transform.
__device__ __forceinline__ void normals4(uint32_t index, uint32_t step, uint32_t stream, uint64_t seed,
                                         double z[4]) {
  const U4 u = philox(index, step, stream, seed);
  const double inv = 1.0 / 4294967296.0;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double a = ((double)u.w[2 * p] + 0.5) * inv, b = ((double)u.w[2 * p + 1] + 0.5) * inv;
    const double r = sqrt(-2.0 * log(a));
    double sn, cs;
    sincos(2.0 * 3.14159265358979323846 * b, &sn, &cs);
    z[2 * p] = r * cs;
    z[2 * p + 1] = r * sn;
  }
}

// Sum of one double per thread over a block (fixed tree), thread 0 gets it.
__device__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = kEnsRed / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  return sh[0];
}

}  // namespace

// partial[b] = sum over atoms of chunk b of m v^2
__global__ void __launch_bounds__(kEnsRed) k_ens_kinetic_partial(const double* __restrict__ vel,
                                                                 const int32_t* __restrict__ types,
                                                                 const double* __restrict__ mass,
                                                                 int64_t N, int64_t chunk,
                                                                 double* __restrict__ partial) {
  __shared__ double sh[kEnsRed];
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(N, lo + chunk);
  double acc = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += kEnsRed) {
    const double vx = vel[k], vy = vel[N + k], vz = vel[2 * N + k];
    acc += mass[types[k]] * (vx * vx + vy * vy + vz * vz);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_ens_kinetic_final(const double* __restrict__ partial, int64_t n_part, double conv,
                                    EnsState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t b = 0; b < n_part; ++b) s += partial[b];
  st->K = 0.5 * s * conv;
}

__global__ void k_ens_step_begin(EnsState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->step += 1;
}

// Ornstein-Uhlenbeck half step v = c1 v + sqrt((1 - c1^2) kT / m) xi of every
// velocity component, xi from the atom's caller index; partial[b] collects
// the change of m v^2 (for the heat exchanged with the bath).
__global__ void __launch_bounds__(kEnsRed) k_ens_langevin(double* __restrict__ vel,
                                                          const int32_t* __restrict__ types,
                                                          const double* __restrict__ mass,
                                                          const int32_t* __restrict__ ext, int64_t N,
                                                          EnsParams p, uint32_t stream,
                                                          const EnsState* st,
                                                          double* __restrict__ partial) {
  __shared__ double sh[kEnsRed];
  const int64_t k = (int64_t)blockIdx.x * kEnsRed + threadIdx.x;
  double d = 0.0;
  if (k < N) {
    const double m = mass[types[k]];
    const double c1 = exp(-0.5 * p.dt / p.tau_t);
    const double amp = sqrt((1.0 - c1 * c1) * p.kT / (m * p.conv));
    double z[4];
    normals4((uint32_t)ext[k], (uint32_t)st->step, stream, p.seed, z);
    for (int c = 0; c < 3; ++c) {
      const double v0 = vel[(int64_t)c * N + k];
      const double v1 = c1 * v0 + amp * z[c];
      vel[(int64_t)c * N + k] = v1;
      d += m * (v1 * v1 - v0 * v0);
    }
  }
  const double s = block_sum(d, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// heat += -(1/2) conv sum of the changes of m v^2, K follows them
__global__ void k_ens_heat_final(const double* __restrict__ partial, int64_t n_part, double conv,
                                 EnsState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t b = 0; b < n_part; ++b) s += partial[b];
  const double dK = 0.5 * s * conv;
  st->heat -= dK;
  st->K += dK;
}

// Nose-Hoover chain half step of dt/2 from the kinetic energy st->K: chain
// forces, velocity updates with the exp(-dt/8 v_{k+1}) factors around them,
// then the particle scale exp(-dt/2 v_xi1) and the chain positions, then the
// mirrored sweep; st->scale = the velocity factor.
__global__ void k_ens_nhc(EnsParams p, EnsState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int M = p.nhc_length;
  const double h = 0.5 * p.dt, kT = p.kT;
  double Q[kMaxChain];
  for (int k = 0; k < M; ++k) Q[k] = (k == 0 ? p.Nf : 1.0) * kT * p.tau_t * p.tau_t;
  double K = st->K;
  double* v = st->vxi;
  auto force = [&](int k) {
    return k == 0 ? (2.0 * K - p.Nf * kT) / Q[0] : (Q[k - 1] * v[k - 1] * v[k - 1] - kT) / Q[k];
  };
  v[M - 1] += 0.5 * h * force(M - 1);
  for (int k = M - 2; k >= 0; --k) {
    const double a = exp(-0.25 * h * v[k + 1]);
    v[k] *= a;
    v[k] += 0.5 * h * force(k);
    v[k] *= a;
  }
  const double s = exp(-h * v[0]);
  K *= s * s;
  for (int k = 0; k < M; ++k) st->xi[k] += h * v[k];
  for (int k = 0; k < M - 1; ++k) {
    const double a = exp(-0.25 * h * v[k + 1]);
    v[k] *= a;
    v[k] += 0.5 * h * force(k);
    v[k] *= a;
  }
  v[M - 1] += 0.5 * h * force(M - 1);
  st->K = K;
  st->scale = s;
}

// Berendsen: v *= sqrt(1 + dt/tau (T0/T - 1)) (clamped at 0)
__global__ void k_ens_berendsen(EnsParams p, EnsState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double K = st->K;
  const double T = 2.0 * K / (p.Nf * p.kB);
  const double l2 = fmax(0.0, 1.0 + p.dt / p.tau_t * (p.T0 / T - 1.0));
  st->scale = sqrt(l2);
  st->heat += K * (1.0 - l2);
  st->K = K * l2;
}

// BDP: partial[b] = sum of the squares of the normals of stream 4 with
// flat index in [0, Nf - 1) that block b's counters cover (four per counter)
__global__ void __launch_bounds__(kEnsRed) k_ens_bdp_partial(EnsParams p, int64_t n_sq, const EnsState* st,
                                                             double* __restrict__ partial) {
  __shared__ double sh[kEnsRed];
  const int64_t q = (int64_t)blockIdx.x * kEnsRed + threadIdx.x;  // counter index
  double acc = 0.0;
  if (4 * q < n_sq) {
    double z[4];
    normals4((uint32_t)q, (uint32_t)st->step, 4u, p.seed, z);
    for (int c = 0; c < 4; ++c)
      if (4 * q + c < n_sq) acc += z[c] * z[c];
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_ens_bdp_final(EnsParams p, const double* __restrict__ partial, int64_t n_part,
                                EnsState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double S = 0.0;
  for (int64_t b = 0; b < n_part; ++b) S += partial[b];
  double z[4];
  normals4(0u, (uint32_t)st->step, 3u, p.seed, z);
  const double R1 = z[0], K = st->K, K0 = 0.5 * p.Nf * p.kT;
  const double c = exp(-p.dt / p.tau_t);
  double Kn = K + (1.0 - c) * (K0 * (R1 * R1 + S) / p.Nf - K) + 2.0 * R1 * sqrt(c * (1.0 - c) * K0 * K / p.Nf);
  Kn = fmax(Kn, 0.0);
  st->scale = sqrt(Kn / K);
  st->heat += K - Kn;
  st->K = Kn;
}

__global__ void k_ens_scale_vel(double* __restrict__ vel, int64_t n3, const EnsState* st) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n3) vel[k] *= st->scale;
}

__global__ void k_ens_scale_pos(double* __restrict__ pos, int64_t n3, const EnsState* st) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n3) pos[k] *= st->mu;
}

__device__ double cell_volume(const double* H) {
  return H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
         H[2] * (H[3] * H[7] - H[4] * H[6]);
}

// The end-of-step pressure P = (2K + tr W)/(3V) from the thermo sums in
// st->row (Ep, W) and the thermostat's K; with write_row, the thermo row
// [step, E_pot, E_kin, T, W (9), V, P, H~] at rows[*counter] (counter
// incremented).
__global__ void k_ens_pressure_row(EnsParams p, EnsState* st, const StructInfo* structs, double* rows,
                                   int32_t* counter, int32_t write_row, int64_t step_base) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double V = cell_volume(structs[0].H);
  const double* r = st->row;
  const double K = st->K;
  const double P = (2.0 * K + r[4] + r[8] + r[12]) / (3.0 * V) * kGPa;
  st->P = P;
  if (!write_row) return;
  const int32_t n = *counter;
  *counter = n + 1;
  double* o = rows + 16 * (int64_t)n;
  o[0] = (double)(st->step - step_base);
  o[1] = r[1];
  o[2] = K;
  o[3] = 2.0 * K / (p.Nf * p.kB);
  for (int v = 0; v < 9; ++v) o[4 + v] = r[4 + v];
  o[13] = V;
  o[14] = P;
  double H = K + r[1] + st->heat;
  if (p.kind == kEnsNHC) {
    H = K + r[1];
    for (int k = 0; k < p.nhc_length; ++k) {
      const double w = k == 0 ? p.Nf : 1.0;
      const double Q = w * p.kT * p.tau_t * p.tau_t;
      H += 0.5 * Q * st->vxi[k] * st->vxi[k] + w * p.kT * st->xi[k];
    }
  }
  if (p.kind >= kEnsNptBerendsen) H += p.P0 / kGPa * V;
  o[15] = H;
}

// Barostat step: mu from the end-of-step pressure (Berendsen) or the
// stochastic cell-rescaling equation for eps = ln V (SCR, which also scales
// the velocities by 1/mu); the cell vectors scale by mu (H^-1 by 1/mu).
__global__ void k_ens_barostat(EnsParams p, EnsState* st, StructInfo* structs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double V = cell_volume(structs[0].H);
  double mu;
  st->scale = 1.0;
  if (p.kind == kEnsNptBerendsen) {
    mu = cbrt(1.0 - p.beta * p.dt / p.tau_p * (p.P0 - st->P));
  } else {
    double z[4];
    normals4(0u, (uint32_t)st->step, 5u, p.seed, z);
    const double kTV = p.kT / V * kGPa;
    const double deps = -p.beta / p.tau_p * (p.P0 - st->P - kTV) * p.dt +
                        sqrt(2.0 * kTV * p.beta * p.dt / p.tau_p) * z[0];
    mu = exp(deps / 3.0);
    st->scale = 1.0 / mu;
    const double K = st->K, Kn = K / (mu * mu);
    st->heat += K - Kn;
    st->K = Kn;
  }
  for (int k = 0; k < 9; ++k) {
    structs[0].H[k] *= mu;
    structs[0].Hi[k] /= mu;
  }
  st->mu = mu;
  st->mu_cum *= mu;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int64_t ens_partials(int64_t N) { return std::min<int64_t>(512, std::max<int64_t>(1, (N + 1023) / 1024)); }

void launch_ens_kinetic(const double* vel, const int32_t* types, const double* mass, int64_t N, double conv,
                        double* partial, EnsState* st, hipStream_t s) {
  const int64_t np = ens_partials(N), chunk = (N + np - 1) / np;
  hipLaunchKernelGGL(k_ens_kinetic_partial, dim3((unsigned)np), dim3(kEnsRed), 0, s, vel, types, mass, N,
                     chunk, partial);
  hipLaunchKernelGGL(k_ens_kinetic_final, dim3(1), dim3(64), 0, s, partial, np, conv, st);
}

void launch_ens_step_begin(EnsState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_step_begin, dim3(1), dim3(64), 0, s, st);
}

void launch_ens_langevin(double* vel, const int32_t* types, const double* mass, const int32_t* ext,
                         int64_t N, const EnsParams& p, uint32_t stream, EnsState* st, double* partial,
                         hipStream_t s) {
  const int64_t nb = div_up(N, kEnsRed);
  hipLaunchKernelGGL(k_ens_langevin, dim3((unsigned)nb), dim3(kEnsRed), 0, s, vel, types, mass, ext, N, p,
                     stream, st, partial);
  hipLaunchKernelGGL(k_ens_heat_final, dim3(1), dim3(64), 0, s, partial, nb, p.conv, st);
}

void launch_ens_thermostat(double* vel, int64_t N, const EnsParams& p, EnsState* st, double* partial,
                           hipStream_t s) {
  if (p.kind == kEnsNHC) {
    hipLaunchKernelGGL(k_ens_nhc, dim3(1), dim3(64), 0, s, p, st);
  } else if (p.kind == kEnsBerendsen || p.kind == kEnsNptBerendsen) {
    hipLaunchKernelGGL(k_ens_berendsen, dim3(1), dim3(64), 0, s, p, st);
  } else if (p.kind == kEnsBDP || p.kind == kEnsNptSCR) {
    const int64_t n_sq = (int64_t)p.Nf - 1;
    const int64_t nb = std::max<int64_t>(1, div_up(div_up(n_sq, 4), kEnsRed));
    hipLaunchKernelGGL(k_ens_bdp_partial, dim3((unsigned)nb), dim3(kEnsRed), 0, s, p, n_sq, st, partial);
    hipLaunchKernelGGL(k_ens_bdp_final, dim3(1), dim3(64), 0, s, p, partial, nb, st);
  } else {
    return;
  }
  hipLaunchKernelGGL(k_ens_scale_vel, dim3(div_up(3 * N, kBlock)), dim3(kBlock), 0, s, vel, 3 * N, st);
}

void launch_ens_pressure_row(const EnsParams& p, EnsState* st, const StructInfo* structs, double* rows,
                             int32_t* counter, bool write_row, int64_t step_base, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_pressure_row, dim3(1), dim3(64), 0, s, p, st, structs, rows, counter,
                     (int32_t)(write_row ? 1 : 0), step_base);
}

void launch_ens_barostat(double* pos, double* vel, int64_t N, const EnsParams& p, EnsState* st,
                         StructInfo* structs, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_barostat, dim3(1), dim3(64), 0, s, p, st, structs);
  hipLaunchKernelGGL(k_ens_scale_pos, dim3(div_up(3 * N, kBlock)), dim3(kBlock), 0, s, pos, 3 * N, st);
  if (p.kind == kEnsNptSCR)
    hipLaunchKernelGGL(k_ens_scale_vel, dim3(div_up(3 * N, kBlock)), dim3(kBlock), 0, s, vel, 3 * N, st);
}

}  // namespace nep
