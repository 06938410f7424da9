// md.hip -- velocity-Verlet NVE (the 'nve' ensemble of the paper) in float64:
//   v += dt/2 F/m;  r += dt v;  (rebuild, forces);  v += dt/2 F/m
// plus the thermo row [step, E_pot, E_kin, T, W_xx..W_zz] as a fixed-order
// float64 reduction.  State is kept in the internal atom order.
#include "nep_kernels.h"

namespace nep {

__global__ void k_kick_drift(MDArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const double s = 0.5 * a.dt * a.inv_mass[a.types[i]];
  double r[3];
  for (int c = 0; c < 3; ++c) {
    const int64_t k = (int64_t)c * a.N + i;
    const double v = a.vel[k] + s * (double)a.F[k];
    a.vel[k] = v;
    r[c] = a.pos[k] + a.dt * v;
    a.pos[k] = r[c];
  }
  if (a.flag) {
    // the skin guard on the new position (the test of k_check_displacement
    // without look-ahead)
    double m = 1.0, t2 = a.thr2;
    if (a.mu_cum) {
      m = *a.mu_cum;
      const double h = fmax(0.0, 0.5 * (m * a.rl - a.rc));
      t2 = h * h;
    }
    const int64_t N = a.N;
    const double dx = r[0] - m * a.ref[i], dy = r[1] - m * a.ref[N + i], dz = r[2] - m * a.ref[2 * N + i];
    if (dx * dx + dy * dy + dz * dz > t2) atomicExch(a.flag, 1);
  }
}

__global__ void k_kick(MDArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const double s = 0.5 * a.dt * a.inv_mass[a.types[i]];
  for (int c = 0; c < 3; ++c) {
    const int64_t k = (int64_t)c * a.N + i;
    a.vel[k] += s * (double)a.F[k];
  }
}

void launch_kick_drift(const MDArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift, dim3(div_up(a.N, kBlock)), dim3(kBlock), 0, s, a);
}

void launch_kick(const MDArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_kick, dim3(div_up(a.N, kBlock)), dim3(kBlock), 0, s, a);
}

constexpr int kRed = 256;

// partial[b][11]: U, m v^2, W_0..8 over a fixed slice, fixed tree.
__global__ void __launch_bounds__(kRed) k_thermo_partial(const float* __restrict__ U,
                                                         const float* __restrict__ W,
                                                         const double* __restrict__ vel,
                                                         const int32_t* __restrict__ types,
                                                         const double* __restrict__ mass,
                                                         int64_t N, int64_t chunk,
                                                         double* __restrict__ partial) {
  __shared__ double sh[11][kRed];
  const int t = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(N, lo + chunk);
  double acc[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = lo + t; k < hi; k += kRed) {
    acc[0] += (double)U[k];
    const double vx = vel[k], vy = vel[N + k], vz = vel[2 * N + k];
    acc[1] += mass[types[k]] * (vx * vx + vy * vy + vz * vz);
    for (int v = 0; v < 9; ++v) acc[2 + v] += (double)W[(int64_t)v * N + k];
  }
  for (int v = 0; v < 11; ++v) sh[v][t] = acc[v];
  __syncthreads();
  for (int off = kRed / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int v = 0; v < 11; ++v) sh[v][t] += sh[v][t + off];
    __syncthreads();
  }
  if (t < 11) partial[blockIdx.x * 11 + t] = sh[t][0];
}

// Thread v < 11 sums column v of the partial rows in block order (the
// fixed order of the totals); thread 0 then writes the row.
__global__ void k_thermo_final(const double* __restrict__ partial, int64_t n_part, int64_t N,
                               double step, double kin_conv, double kB, double* __restrict__ row,
                               int32_t* __restrict__ counter, double every) {
  __shared__ double s[11];
  const int t = threadIdx.x;
  if (t < 11) {
    double acc = 0.0;
#pragma unroll 8
    for (int64_t b = 0; b < n_part; ++b) acc += partial[b * 11 + t];
    s[t] = acc;
  }
  __syncthreads();
  if (t != 0) return;
  if (counter) {  // row and step number from a device counter (graph replays)
    const int32_t r = *counter;
    *counter = r + 1;
    row += 13 * (int64_t)r;
    step = (double)(r + 1) * every;
  }
  const double ek = 0.5 * s[1] * kin_conv;
  row[0] = step;
  row[1] = s[0];
  row[2] = ek;
  row[3] = N > 1 ? 2.0 * ek / ((3.0 * (double)N - 3.0) * kB) : 0.0;
  for (int v = 0; v < 9; ++v) row[4 + v] = s[2 + v];
}

void launch_thermo(const float* U, const float* W, const double* vel, const int32_t* types,
                   const double* mass, int64_t N, double* partial, int64_t n_part, double* row,
                   double step, double kin_conv, double kB, hipStream_t s) {
  const int64_t chunk = (N + n_part - 1) / n_part;
  hipLaunchKernelGGL(k_thermo_partial, dim3((unsigned)n_part), dim3(kRed), 0, s, U, W, vel, types,
                     mass, N, chunk, partial);
  hipLaunchKernelGGL(k_thermo_final, dim3(1), dim3(64), 0, s, partial, n_part, N, step, kin_conv,
                     kB, row, (int32_t*)nullptr, 0.0);
}

void launch_thermo_counted(const float* U, const float* W, const double* vel, const int32_t* types,
                           const double* mass, int64_t N, double* partial, int64_t n_part,
                           double* rows, int32_t* counter, double every, double kin_conv, double kB,
                           hipStream_t s) {
  const int64_t chunk = (N + n_part - 1) / n_part;
  hipLaunchKernelGGL(k_thermo_partial, dim3((unsigned)n_part), dim3(kRed), 0, s, U, W, vel, types,
                     mass, N, chunk, partial);
  hipLaunchKernelGGL(k_thermo_final, dim3(1), dim3(64), 0, s, partial, n_part, N, 0.0, kin_conv, kB,
                     rows, counter, every);
}

// new[k] = old[src[k]] for positions and velocities ([3][N] each)
__global__ void k_permute_md(const int32_t* __restrict__ src, int64_t N,
                             const double* __restrict__ pos_old, const double* __restrict__ vel_old,
                             double* __restrict__ pos_new, double* __restrict__ vel_new) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int64_t o = src[k];
  for (int c = 0; c < 3; ++c) {
    pos_new[(int64_t)c * N + k] = pos_old[(int64_t)c * N + o];
    vel_new[(int64_t)c * N + k] = vel_old[(int64_t)c * N + o];
  }
}

void launch_permute_md(const int32_t* src, int64_t N, const double* src_pos,
                       const double* src_vel, double* dst_pos, double* dst_vel, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_md, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, src, N, src_pos,
                     src_vel, dst_pos, dst_vel);
}

// *differs = 1 unless, for every internal atom k, the caller's position and
// species of atom ext[k] are those held internally (bit for bit).
__global__ void k_same_state(const int32_t* __restrict__ ext, int64_t N, const double* __restrict__ pos_int,
                             const int32_t* __restrict__ types_int, const double* __restrict__ pos_caller,
                             const int32_t* __restrict__ types_caller, int32_t* __restrict__ differs) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int64_t e = ext[k];
  bool same = types_int[k] == types_caller[e];
  for (int c = 0; c < 3; ++c) same = same && pos_int[(int64_t)c * N + k] == pos_caller[(int64_t)c * N + e];
  if (!same) atomicExch(differs, 1);
}

void launch_same_state(const int32_t* ext, int64_t N, const double* pos_int, const int32_t* types_int,
                       const double* pos_caller, const int32_t* types_caller, int32_t* differs, hipStream_t s) {
  hipLaunchKernelGGL(k_same_state, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, ext, N, pos_int, types_int,
                     pos_caller, types_caller, differs);
}

// gated gathers used by a device-decided rebuild: out[k] = in[src[k]]
__global__ void k_gather3_gated(const int32_t* __restrict__ src, int64_t N, const double* __restrict__ in,
                                double* __restrict__ out, const int32_t* gate) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N || (gate && *gate == 0)) return;
  const int64_t o = src[k];
  for (int c = 0; c < 3; ++c) out[(int64_t)c * N + k] = in[(int64_t)c * N + o];
}

__global__ void k_gather_i32_gated(const int32_t* __restrict__ src, int64_t N, const int32_t* __restrict__ in,
                                   int32_t* __restrict__ out, const int32_t* gate) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N && !(gate && *gate == 0)) out[k] = in[src[k]];
}

void launch_gather3_gated(const int32_t* src, int64_t N, const double* in, double* out,
                          const int32_t* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_gather3_gated, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, src, N, in, out, gate);
}

void launch_gather_i32_gated(const int32_t* src, int64_t N, const int32_t* in, int32_t* out,
                             const int32_t* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_i32_gated, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, src, N, in, out,
                     gate);
}

// caller order out: ext[perm[k]] = int[k]
__global__ void k_unpermute_md(const int32_t* __restrict__ perm, int64_t N,
                               const double* __restrict__ pos_int, const double* __restrict__ vel_int,
                               double* __restrict__ pos_ext, double* __restrict__ vel_ext) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int64_t e = perm[k];
  for (int c = 0; c < 3; ++c) {
    pos_ext[(int64_t)c * N + e] = pos_int[(int64_t)c * N + k];
    vel_ext[(int64_t)c * N + e] = vel_int[(int64_t)c * N + k];
  }
}

void launch_unpermute_md(const int32_t* perm, int64_t N, const double* pos_int,
                         const double* vel_int, double* pos_ext, double* vel_ext, hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute_md, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, perm, N, pos_int,
                     vel_int, pos_ext, vel_ext);
}

__global__ void k_check_finite(const double* __restrict__ a, int64_t n, int32_t* __restrict__ flag) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && !isfinite(a[k])) atomicExch(flag, 1);
}

void launch_check_finite(const double* a, int64_t n, int32_t* flag, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_check_finite, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, a, n, flag);
}

__global__ void k_check_types(const int32_t* __restrict__ t, int64_t n, int32_t T,
                              int32_t* __restrict__ flag) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && (t[k] < 0 || t[k] >= T)) atomicExch(flag, 1);
}

void launch_check_types(const int32_t* types, int64_t n, int32_t T, int32_t* flag, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_check_types, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, types, n, T, flag);
}

// out[k] = in[src[k]]
__global__ void k_gather_i32(const int32_t* __restrict__ src, int64_t N, const int32_t* __restrict__ in,
                             int32_t* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) out[k] = in[src[k]];
}

void launch_gather_i32(const int32_t* src, int64_t N, const int32_t* in, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_i32, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, src, N, in, out);
}

// ---- serving: velocity Verlet on the concatenated request state (request
// order, caller order inside each request), forces in float64 ----

// v += hdm F; r += dt v   for atoms with move != 0
__global__ void k_srv_kick_drift(int64_t N, double* __restrict__ pos, double* __restrict__ vel,
                                 const double* __restrict__ F, const double* __restrict__ hdm,
                                 const double* __restrict__ dta, const uint8_t* __restrict__ move) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || !move[i]) return;
  for (int c = 0; c < 3; ++c) {
    const int64_t k = (int64_t)c * N + i;
    const double v = vel[k] + hdm[i] * F[k];
    vel[k] = v;
    pos[k] += dta[i] * v;
  }
}

__global__ void k_srv_kick(int64_t N, double* __restrict__ vel, const double* __restrict__ F,
                           const double* __restrict__ hdm, const uint8_t* __restrict__ move) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || !move[i]) return;
  for (int c = 0; c < 3; ++c) {
    const int64_t k = (int64_t)c * N + i;
    vel[k] += hdm[i] * F[k];
  }
}

void launch_srv_kick_drift(int64_t N, double* pos, double* vel, const double* F, const double* hdm,
                           const double* dta, const uint8_t* move, hipStream_t s) {
  hipLaunchKernelGGL(k_srv_kick_drift, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, N, pos, vel, F, hdm,
                     dta, move);
}

void launch_srv_kick(int64_t N, double* vel, const double* F, const double* hdm, const uint8_t* move,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_srv_kick, dim3(div_up(N, kBlock)), dim3(kBlock), 0, s, N, vel, F, hdm, move);
}

__global__ void k_fill_u8(uint8_t* __restrict__ a, int64_t n, uint8_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

void launch_fill_u8(uint8_t* a, int64_t n, uint8_t v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u8, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, a, n, v);
}

// New layout of the server's batch state, one launch for every request:
// blockIdx.y = request k, tab[4k..4k+3] = {dst, n, src, stg}: its n atoms go
// to dst in the new layout, from src in the old one, or (src < 0: admitted
// this tick) from offset stg of the uploaded staging, whose parts are
// pos [3][ns], vel [3][ns], hdm [ns], dta [ns] (doubles) then types [ns].
__global__ void k_srv_place(const int64_t* __restrict__ tab, SrvState o, SrvState w,
                            const double* __restrict__ stg, int64_t ns) {
  const int k = blockIdx.y;
  const int64_t dst = tab[4 * k], n = tab[4 * k + 1], src = tab[4 * k + 2], so = tab[4 * k + 3];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t i = dst + e;
  if (src >= 0) {
    const int64_t j = src + e;
    w.types[i] = o.types[j];
    w.hdm[i] = o.hdm[j];
    w.dta[i] = o.dta[j];
    w.move[i] = o.move[j];
    for (int c = 0; c < 3; ++c) {
      w.pos[c * w.ld + i] = o.pos[c * o.ld + j];
      w.vel[c * w.ld + i] = o.vel[c * o.ld + j];
      w.F[c * w.ld + i] = o.F[c * o.ld + j];
    }
  } else {
    const int64_t j = so + e;
    for (int c = 0; c < 3; ++c) {
      w.pos[c * w.ld + i] = stg[c * ns + j];
      w.vel[c * w.ld + i] = stg[(3 + c) * ns + j];
    }
    w.hdm[i] = stg[6 * ns + j];
    w.dta[i] = stg[7 * ns + j];
    w.types[i] = reinterpret_cast<const int32_t*>(stg + 8 * ns)[j];
    w.move[i] = 0;  // no step before the request's first evaluation
  }
}

void launch_srv_place(const int64_t* tab, int32_t n_req, int64_t max_n, const SrvState& o, const SrvState& w,
                      const double* stg, int64_t ns, hipStream_t s) {
  if (n_req > 0 && max_n > 0)
    hipLaunchKernelGGL(k_srv_place, dim3(div_up(max_n, kBlock), n_req), dim3(kBlock), 0, s, tab, o, w, stg, ns);
}

// Results of the requests that finished this tick, packed for one copy to
// the host: blockIdx.y = request k, tab[4k..4k+3] = {off, n, out, md}; its
// block at out holds E [n], F [3][n], W [9][n] and, for MD, pos [3][n] and
// vel [3][n].
__global__ void k_srv_collect(const int64_t* __restrict__ tab, int64_t ld, const double* __restrict__ E,
                              const double* __restrict__ F, const double* __restrict__ W,
                              const double* __restrict__ pos, const double* __restrict__ vel,
                              double* __restrict__ out) {
  const int k = blockIdx.y;
  const int64_t off = tab[4 * k], n = tab[4 * k + 1], o = tab[4 * k + 2], md = tab[4 * k + 3];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t i = off + e;
  double* b = out + o;
  b[e] = E[i];
  for (int c = 0; c < 3; ++c) b[(1 + c) * n + e] = F[c * ld + i];
  for (int v = 0; v < 9; ++v) b[(4 + v) * n + e] = W[v * ld + i];
  if (md) {
    for (int c = 0; c < 3; ++c) {
      b[(13 + c) * n + e] = pos[c * ld + i];
      b[(16 + c) * n + e] = vel[c * ld + i];
    }
  }
}

void launch_srv_collect(const int64_t* tab, int32_t n_req, int64_t max_n, int64_t ld, const double* E,
                        const double* F, const double* W, const double* pos, const double* vel, double* out,
                        hipStream_t s) {
  if (n_req > 0 && max_n > 0)
    hipLaunchKernelGGL(k_srv_collect, dim3(div_up(max_n, kBlock), n_req), dim3(kBlock), 0, s, tab, ld, E, F,
                       W, pos, vel, out);
}


}  // namespace nep
