// neighbor.hip -- neighbour rows for the sums over j != i of Sec. II.B/II.C.
//
// The paper assumes neighbour counts NN_i and rows NL_im are given and uses
// the minimum image; it does not say how they are built.  Here:
//   1. atoms are binned into cells at least r_c wide along every cell vector
//      (fractional coordinates, float64), one cell per small structure;
//   2. a deterministic counting sort gives the internal atom order
//      (structure, cell, caller index): the atoms of a cell are contiguous;
//   3. one thread per atom scans the stencil cells in increasing cell index,
//      so candidate j arrive in increasing internal index and every candidate
//      row (radius r_c^R, or r_c^R + skin in MD with a skin) comes out sorted
//      by (j, image) without a sort;
//   4. membership is the strict float64 test |d|^2 < r_c^2 on the canonical
//      displacement (no fused multiply-add), the same test for both cutoffs;
//   5. the exact radial row is filtered from the candidates with the
//      angular-range entries (|d|^2 < (r_c^A)^2) first and the rest after,
//      each part in candidate order: the angular row of the sums is the
//      first nnA entries of the radial row;
//   6. rev[m][i] locates i in the radial row of its m-th neighbour: a binary
//      search on the sorted candidate rows (once per candidate build) and the
//      candidate -> exact position map of every filter, so the force pass
//      can gather dU_j/dr_ji without atomics.
#include "nep_kernels.h"

namespace nep {

// Kernels of a rebuild take an optional gate: when it points to 0 they do
// nothing, so an MD step can issue a fixed kernel sequence and let the device
// decide whether the rows are rebuilt.
__device__ __forceinline__ bool gated_off(const int32_t* gate) { return gate && *gate == 0; }

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_i32_gated(int32_t* a, int64_t n, int32_t v, const int32_t* gate) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !gated_off(gate)) a[i] = v;
}

// Structure id of every caller-order atom from the offsets array.
__global__ void k_assign_struct(const int64_t* __restrict__ offs, int32_t n_struct, int64_t N,
                                int32_t* __restrict__ sid) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int lo = 0, hi = n_struct - 1;
  while (lo < hi) {  // last s with offs[s] <= i
    int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= i) lo = mid; else hi = mid - 1;
  }
  sid[i] = lo;
}

// Cell coordinates of a position inside structure st (fractional, wrapped
// along periodic directions, clamped along open ones).
__device__ inline void cell_coords(const StructInfo& st, double x, double y, double z,
                                   int& cx, int& cy, int& cz) {
  double s[3];
  s[0] = x * st.Hi[0] + y * st.Hi[3] + z * st.Hi[6];
  s[1] = x * st.Hi[1] + y * st.Hi[4] + z * st.Hi[7];
  s[2] = x * st.Hi[2] + y * st.Hi[5] + z * st.Hi[8];
  int c[3];
  for (int k = 0; k < 3; ++k) {
    double f = s[k];
    if (st.pbc[k]) f -= floor(f);
    f = fmin(fmax(f, 0.0), 1.0);
    int v = (int)(f * st.ncell[k]);
    c[k] = v < 0 ? 0 : (v >= st.ncell[k] ? st.ncell[k] - 1 : v);
  }
  cx = c[0];
  cy = c[1];
  cz = c[2];
}

__global__ void k_cell_key(const double* __restrict__ pos, int64_t N,
                           const int32_t* __restrict__ sid, const StructInfo* __restrict__ structs,
                           int32_t* __restrict__ key, int32_t* __restrict__ cell_count,
                           const int32_t* gate) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N || gated_off(gate)) return;
  const StructInfo& st = structs[sid[e]];
  int k = st.cell_off;
  if (st.mode == kModeCells) {
    int cx, cy, cz;
    cell_coords(st, pos[e], pos[N + e], pos[2 * N + e], cx, cy, cz);
    k += (cz * st.ncell[1] + cy) * st.ncell[0] + cx;
  }
  key[e] = k;
  atomicAdd(&cell_count[k], 1);
}

// Exclusive scan of n int32 counts by one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan_1block(const int32_t* __restrict__ in,
                                                      int32_t* __restrict__ out, int32_t n,
                                                      const int32_t* gate) {
  __shared__ int32_t part[1024];
  if (gated_off(gate)) return;
  int t = threadIdx.x;
  int chunk = (n + 1023) / 1024;
  int lo = t * chunk, hi = min(n, lo + chunk);
  int32_t s = 0;
  for (int i = lo; i < hi; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    int32_t c = in[i];
    out[i] = run;
    run += c;
  }
}

__global__ void k_cell_scatter(const int32_t* __restrict__ key, int64_t N,
                               const int32_t* __restrict__ cell_start,
                               int32_t* __restrict__ cell_fill, int32_t* __restrict__ perm,
                               const int32_t* gate) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N || gated_off(gate)) return;
  int k = key[e];
  int slot = atomicAdd(&cell_fill[k], 1);
  perm[cell_start[k] + slot] = (int32_t)e;
}

// Order the atoms of each cell by caller index (ext[source index], or the
// source index itself when ext is NULL).  The internal order is then a
// function of the positions and caller indices only: independent of the
// atomic slot assignment above and of the order the atoms came in.  One wave
// per cell: every lane holds up to kSortPerLane of the cell's atoms and
// counts, for each, the keys below its own (keys are distinct, so the counts
// are the sorted positions); the wave reads the cell's keys 64 at a time and
// passes them around with lane shuffles.  Cells above 64 kSortPerLane atoms
// (possible only for a structure that is one cell) are sorted by one lane.
constexpr int kSortPerLane = 16;

__global__ void __launch_bounds__(kBlock) k_cell_sort(const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ cell_count,
                                                      int32_t n_cells, const int32_t* __restrict__ ext,
                                                      int32_t* __restrict__ perm, const int32_t* gate) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (c >= n_cells || gated_off(gate)) return;  // the lanes of a wave leave together
  int32_t* p = perm + cell_start[c];
  const int n = cell_count[c];
  if (n <= 1) return;
  if (n > 64 * kSortPerLane) {
    if (lane != 0) return;
    for (int a = 1; a < n; ++a) {
      const int32_t v = p[a];
      const int32_t kv = ext ? ext[v] : v;
      int b = a - 1;
      while (b >= 0 && (ext ? ext[p[b]] : p[b]) > kv) {
        p[b + 1] = p[b];
        --b;
      }
      p[b + 1] = v;
    }
    return;
  }
  int32_t v[kSortPerLane], key[kSortPerLane], rank[kSortPerLane];
#pragma unroll
  for (int a = 0; a < kSortPerLane; ++a) {
    const int idx = lane + 64 * a;
    v[a] = idx < n ? p[idx] : 0;
    key[a] = idx < n ? (ext ? ext[v[a]] : v[a]) : INT32_MAX;
    rank[a] = 0;
  }
  for (int b0 = 0; b0 < n; b0 += 64) {
    const int idx = b0 + lane;
    int32_t kb = INT32_MAX;
    if (idx < n) {
      const int32_t u = p[idx];
      kb = ext ? ext[u] : u;
    }
    const int m = min(64, n - b0);
    for (int l = 0; l < m; ++l) {
      const int32_t k = __shfl(kb, l);
#pragma unroll
      for (int a = 0; a < kSortPerLane; ++a) rank[a] += k < key[a] ? 1 : 0;
    }
  }
  // every read of the cell's entries above has been consumed by the shuffles
#pragma unroll
  for (int a = 0; a < kSortPerLane; ++a)
    if (lane + 64 * a < n) p[rank[a]] = v[a];
}

__global__ void k_gather_atoms(BuildArgs b) {
  const int64_t N = b.N;
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N || gated_off(b.gate)) return;
  int64_t e = b.perm[k];
  for (int c = 0; c < 3; ++c) b.pos[c * N + k] = b.pos_ext[c * N + e];
  b.types[k] = b.types_ext[e];
  b.sid[k] = b.sid_ext[e];
  if (b.vel_src)
    for (int c = 0; c < 3; ++c) b.vel_dst[c * N + k] = b.vel_src[c * N + e];
  if (b.ext_in) b.ext_out[k] = b.ext_in[e];
}

__global__ void k_fill_cells(int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t n,
                             const int32_t* gate) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !gated_off(gate)) {
    a[i] = 0;
    b[i] = 0;
  }
}

__global__ void k_commit_rebuild(int64_t N, const double* __restrict__ pos2,
                                 const double* __restrict__ vel2, const int32_t* __restrict__ types2,
                                 const int32_t* __restrict__ ext2, double* __restrict__ pos,
                                 double* __restrict__ vel, int32_t* __restrict__ types,
                                 int32_t* __restrict__ ext, double* __restrict__ pos_ref,
                                 const int32_t* gate, double* mu_cum, int32_t* count) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N || gated_off(gate)) return;
  if (k == 0 && mu_cum) *mu_cum = 1.0;  // the reference positions are the current ones
  if (k == 0 && count) atomicAdd(count, 1);  // rebuilds done
  for (int c = 0; c < 3; ++c) {
    const double x = pos2[c * N + k];
    pos[c * N + k] = x;
    pos_ref[c * N + k] = x;
    vel[c * N + k] = vel2[c * N + k];
  }
  types[k] = types2[k];
  ext[k] = ext2[k];
}

// The up-to-3 stencil cells along one cell vector in increasing order.
__device__ inline int stencil_1d(int c, int n, int periodic, int* out) {
  if (periodic) {
    if (n < 3) {
      for (int v = 0; v < n; ++v) out[v] = v;
      return n;
    }
    if (c == 0) {
      out[0] = 0; out[1] = 1; out[2] = n - 1;
    } else if (c == n - 1) {
      out[0] = 0; out[1] = n - 2; out[2] = n - 1;
    } else {
      out[0] = c - 1; out[1] = c; out[2] = c + 1;
    }
    return 3;
  }
  int k = 0;
  for (int v = c - 1; v <= c + 1; ++v)
    if (v >= 0 && v < n) out[k++] = v;
  return k;
}

// Candidate rows of the atoms of cell-mode structures, kCellLanes lanes per
// atom: the 27 stencil cells in order, each cell's atoms taken kCellLanes at
// a time (lane s the (k0 + s)-th), each accepted one placed by a count over
// the atom's lanes' ballot bits, so the row is the one a single lane's scan
// writes (cells in stencil order, atoms in cell order).  Atoms of structures
// without cells take their rows from k_build_rows_wide.
constexpr int kCellLanes = 4;

__global__ void __launch_bounds__(kBlock) k_build_rows(
    const double* __restrict__ pos, int64_t N, const int32_t* __restrict__ sid,
    const StructInfo* __restrict__ structs, const int32_t* __restrict__ cell_start,
    const int32_t* __restrict__ cell_count, double rc2, Lists V, int32_t* __restrict__ overflow,
    const int32_t* gate) {
  constexpr int G = kCellLanes;
  const int sub = threadIdx.x & (G - 1);
  const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / G;
  if (i >= N || gated_off(gate)) return;  // the lanes of an atom leave together
  const StructInfo st = structs[sid[i]];
  if (st.mode != kModeCells) return;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  const int lane = threadIdx.x & 63;
  const uint64_t gmask = ((1ull << G) - 1) << (lane & ~(G - 1));
  const uint64_t below = (1ull << lane) - 1;
  const uint16_t code0 = make_code(0, 0, 0);
  int32_t count = 0;
  int cx, cy, cz;
  cell_coords(st, xi, yi, zi, cx, cy, cz);
  int sx[3], sy[3], sz[3];
  const int nx = stencil_1d(cx, st.ncell[0], st.pbc[0], sx);
  const int ny = stencil_1d(cy, st.ncell[1], st.pbc[1], sy);
  const int nz = stencil_1d(cz, st.ncell[2], st.pbc[2], sz);
  for (int a = 0; a < nz; ++a)
    for (int b = 0; b < ny; ++b)
      for (int c = 0; c < nx; ++c) {
        const int cell = st.cell_off + (sz[a] * st.ncell[1] + sy[b]) * st.ncell[0] + sx[c];
        const int s0 = cell_start[cell], cnt = cell_count[cell];
        for (int k0 = 0; k0 < cnt; k0 += G) {
          const int k = k0 + sub;
          const int64_t j = s0 + min(k, cnt - 1);
          bool take = false;
          if (k < cnt) {
            double Dx, Dy, Dz;
            {
#pragma clang fp contract(off)
              Dx = pos[j] - xi;
              Dy = pos[N + j] - yi;
              Dz = pos[2 * N + j] - zi;
            }
            int n0, n1, n2;
            min_image(st, Dx, Dy, Dz, n0, n1, n2);
            if (!(j == i && n0 == 0 && n1 == 0 && n2 == 0)) {
              double dx, dy, dz;
              image_disp(st, Dx, Dy, Dz, n0, n1, n2, dx, dy, dz);
              take = norm2_exact(dx, dy, dz) < rc2;
            }
          }
          const uint64_t mt = __ballot(take) & gmask;
          if (take) {
            const int32_t p = count + __popcll(mt & below);
            if (p < V.MR) {
              V.nlR[(int64_t)p * N + i] = (int32_t)j;
              V.cdR[(int64_t)p * N + i] = code0;
            }
          }
          count += __popcll(mt);
        }
      }
  if (sub == 0) {
    V.nnR[i] = count;
    if (count > V.MR) atomicMax(overflow, count);
  }
}

// Candidate rows of the atoms of structures without cells (all-pairs and
// image modes: small cells, whose rows scan every atom of the structure, or
// every (atom, image) pair), kBuildLanes lanes per atom.  The candidates of
// atom i form one sequence in row order -- the atoms of the structure, or
// the (atom, image) pairs with the image offsets innermost -- taken
// kBuildLanes at a time (lane s the s-th of each step); each member is placed
// by a count over the atom's lanes' ballot bits, so the row is the one a
// sequential scan of the sequence writes: sorted by (j, image).
constexpr int kBuildLanes = 16;

__global__ void __launch_bounds__(kBlock) k_build_rows_wide(
    const double* __restrict__ pos, int64_t N, const int32_t* __restrict__ sid,
    const StructInfo* __restrict__ structs, double rc2, Lists V, int32_t* __restrict__ overflow,
    const int32_t* gate) {
  constexpr int G = kBuildLanes;
  const int sub = threadIdx.x & (G - 1);
  const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / G;
  if (i >= N || gated_off(gate)) return;  // the lanes of an atom leave together
  if (structs[sid[i]].mode == kModeCells) return;  // k_build_rows' atoms
  const StructInfo st = structs[sid[i]];
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  const int64_t total = st.mode == kModeAllPairs
                            ? st.count
                            : st.count * (int64_t)((2 * st.reach[0] + 1) * (2 * st.reach[1] + 1) *
                                                   (2 * st.reach[2] + 1));
  // member test of candidate (j, image offset o)
  auto member = [&](int64_t j, int o0, int o1, int o2, uint16_t& code) -> bool {
    double Dx, Dy, Dz;
    {
#pragma clang fp contract(off)
      Dx = pos[j] - xi;
      Dy = pos[N + j] - yi;
      Dz = pos[2 * N + j] - zi;
    }
    int n0, n1, n2;
    min_image(st, Dx, Dy, Dz, n0, n1, n2);
    n0 += o0;
    n1 += o1;
    n2 += o2;
    if (j == i && n0 == 0 && n1 == 0 && n2 == 0) return false;
    double dx, dy, dz;
    image_disp(st, Dx, Dy, Dz, n0, n1, n2, dx, dy, dz);
    code = make_code(o0, o1, o2);
    return norm2_exact(dx, dy, dz) < rc2;
  };
  // candidates c = G t + s of the sequence (the atoms of the structure, or the
  // (atom, image) pairs with the image offsets innermost), G at a time; an
  // accepted one's slot is the count so far plus the accepted lanes below it
  const int R0 = st.reach[0], R1 = st.reach[1], R2 = st.reach[2];
  const int w1 = 2 * R1 + 1, w2 = 2 * R2 + 1, nimg = (2 * R0 + 1) * w1 * w2;
  const bool all_pairs = st.mode == kModeAllPairs;
  const int lane = threadIdx.x & 63;
  const uint64_t gmask = ((1ull << G) - 1) << (lane & ~(G - 1));
  const uint64_t below = (1ull << lane) - 1;
  int32_t count = 0;
  for (int64_t c0 = 0; c0 < total; c0 += G) {
    const int64_t c = c0 + sub;
    bool take = false;
    uint16_t code = kCodeCenter;
    int64_t j = 0;
    if (c < total) {
      int o0 = 0, o1 = 0, o2 = 0;
      if (all_pairs) {
        j = st.start + c;
      } else {
        const int64_t jl = c / nimg;
        const int img = (int)(c - jl * nimg);
        j = st.start + jl;
        o0 = img / (w1 * w2) - R0;
        o1 = (img / w2) % w1 - R1;
        o2 = img % w2 - R2;
      }
      take = member(j, o0, o1, o2, code);
    }
    const uint64_t mt = __ballot(take) & gmask;
    if (take) {
      const int32_t p = count + __popcll(mt & below);
      if (p < V.MR) {
        V.nlR[(int64_t)p * N + i] = (int32_t)j;
        V.cdR[(int64_t)p * N + i] = code;
      }
    }
    count += __popcll(mt);
  }
  if (sub == 0) {
    V.nnR[i] = count;
    if (count > V.MR) atomicMax(overflow, count);
  }
}

// rev[m][i] = position of (i, -offset) in the row of j = nl[m][i] (rows
// sorted by (j, image)).
constexpr int kReverseLanes = 4;  // lanes per atom of k_reverse: lane s searches for entries s, s + 4, ...
constexpr int kReverseChunk = 4;  // entries whose searches a lane of k_reverse runs together

__global__ void k_reverse(int64_t N, const int32_t* __restrict__ nn, const int32_t* __restrict__ nl,
                          const uint16_t* __restrict__ cd, int32_t cap, int32_t* __restrict__ rev,
                          int32_t* __restrict__ err, const int32_t* gate) {
  const int sub = threadIdx.x & (kReverseLanes - 1);
  const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / kReverseLanes;
  if (i >= N || gated_off(gate)) return;
  const int cnt = min(nn[i], cap);
  bool bad = false;
  // kReverseChunk entries of the lane at a time: their binary searches advance
  // together, so each step has that many independent loads in flight
  constexpr int U = kReverseChunk;
  for (int m0 = sub; m0 < cnt; m0 += U * kReverseLanes) {
    int32_t j[U];
    uint32_t key[U];
    int lo[U], hi[U], found[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = m0 + u * kReverseLanes;
      j[u] = 0;
      key[u] = 0;
      lo[u] = 0;
      hi[u] = -1;  // an empty search for entries past the row
      found[u] = -1;
      if (m < cnt) {
        j[u] = nl[(int64_t)m * N + i];
        int a, b, c;
        split_code(cd[(int64_t)m * N + i], a, b, c);
        key[u] = (uint32_t)make_code(-a, -b, -c);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (m0 + u * kReverseLanes < cnt) hi[u] = min(nn[j[u]], cap) - 1;
    for (;;) {
      bool any = false;
      int mid[U];
      int32_t jj[U];
      uint32_t kk[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = found[u] < 0 && lo[u] <= hi[u];
        any |= live;
        mid[u] = live ? (lo[u] + hi[u]) >> 1 : -1;
        jj[u] = 0;
        kk[u] = 0;
        if (live) {
          jj[u] = nl[(int64_t)mid[u] * N + j[u]];
          kk[u] = cd[(int64_t)mid[u] * N + j[u]];
        }
      }
      if (!any) break;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (mid[u] < 0) continue;
        if (jj[u] == (int32_t)i && kk[u] == key[u]) found[u] = mid[u];
        else if (jj[u] < (int32_t)i || (jj[u] == (int32_t)i && kk[u] < key[u])) lo[u] = mid[u] + 1;
        else hi[u] = mid[u] - 1;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = m0 + u * kReverseLanes;
      if (m >= cnt) continue;
      if (found[u] < 0) {
        bad = true;
        found[u] = 0;
      }
      rev[(int64_t)m * N + i] = found[u];
    }
  }
  if (bad) atomicExch(err, 1);
}

// ---- row order for the network pass: atoms grouped by species in
// increasing internal index, each group padded to whole kRowGroup-row groups
// (padding rows hold -1).  Counting sort by blocks of kBlock atoms:
// per-block species counts, one exclusive scan over [species][block], then
// every atom takes its rank inside the block from wave ballots. ----

// Species of atom i for the row order, clamped into [0, Tn): a type out of
// range is reported by its own check, and the rows stay in bounds meanwhile.
__device__ __forceinline__ int row_species(const int32_t* types, int64_t i, int32_t Tn,
                                           int32_t per_type) {
  return per_type ? min(max(types[i], 0), Tn - 1) : 0;
}

__global__ void __launch_bounds__(kBlock) k_type_block_count(const int32_t* __restrict__ types,
                                                             int64_t N, int32_t Tn, int32_t per_type,
                                                             int32_t nb, int32_t* __restrict__ tblk,
                                                             int32_t* __restrict__ rows,
                                                             int64_t rows_len, const int32_t* gate) {
  __shared__ int32_t hist[kMaxTypes];
  if (gated_off(gate)) return;
  const int t = threadIdx.x;
  // every row slot starts as padding (-1); the scatter kernel fills the atoms
  for (int64_t r = (int64_t)blockIdx.x * kBlock + t; r < rows_len; r += (int64_t)nb * kBlock) rows[r] = -1;
  if (t < kMaxTypes) hist[t] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + t;
  if (i < N) atomicAdd(&hist[row_species(types, i, Tn, per_type)], 1);
  __syncthreads();
  if (t < Tn) tblk[(int64_t)t * nb + blockIdx.x] = hist[t];
}

// shift[t] = (padded start of species t) - (exclusive count before species t)
__global__ void k_type_shift(const int32_t* __restrict__ tex, int64_t N, int32_t Tn, int32_t nb,
                             int32_t* __restrict__ shift, const int32_t* gate) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || gated_off(gate)) return;
  int32_t o = 0;
  for (int t = 0; t < Tn; ++t) {
    const int32_t first = tex[(int64_t)t * nb];
    const int32_t next = t + 1 < Tn ? tex[(int64_t)(t + 1) * nb] : (int32_t)N;
    shift[t] = o - first;
    o += (next - first + kRowGroup - 1) / kRowGroup * kRowGroup;
  }
}

__global__ void __launch_bounds__(kBlock) k_type_block_scatter(
    const int32_t* __restrict__ types, int64_t N, int32_t Tn, int32_t per_type, int32_t nb,
    const int32_t* __restrict__ tex, const int32_t* __restrict__ shift, int32_t* __restrict__ rows,
    const int32_t* gate) {
  constexpr int kWaves = kBlock / 64;
  __shared__ int32_t wcount[kWaves][kMaxTypes];
  if (gated_off(gate)) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * kBlock + t;
  const bool live = i < N;
  const int sp = live ? row_species(types, i, Tn, per_type) : -1;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int rank = 0;
  for (int q = 0; q < Tn; ++q) {
    const uint64_t m = __ballot(sp == q);
    if (sp == q) rank = __popcll(m & below);
    if (lane == 0) wcount[w][q] = __popcll(m);
  }
  __syncthreads();
  if (!live) return;
  for (int v = 0; v < w; ++v) rank += wcount[v][sp];
  rows[tex[(int64_t)sp * nb + blockIdx.x] + shift[sp] + rank] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static inline dim3 grid_for(int64_t n, int b = kBlock) { return dim3((unsigned)div_up(n, b)); }

void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, grid_for(n), dim3(kBlock), 0, s, a, n, v);
}

void launch_assign_struct(const int64_t* offs, int32_t n_struct, int64_t N, int32_t* sid,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_assign_struct, grid_for(N), dim3(kBlock), 0, s, offs, n_struct, N, sid);
}

void launch_order_atoms(const BuildArgs& b, hipStream_t s) {
  const int32_t* g = b.gate;
  hipLaunchKernelGGL(k_fill_cells, grid_for(b.n_cells), dim3(kBlock), 0, s, b.cell_count,
                     b.cell_fill, (int64_t)b.n_cells, g);
  hipLaunchKernelGGL(k_cell_key, grid_for(b.N), dim3(kBlock), 0, s, b.pos_ext, b.N, b.sid_ext,
                     b.structs, b.key, b.cell_count, g);
  hipLaunchKernelGGL(k_scan_1block, dim3(1), dim3(1024), 0, s, b.cell_count, b.cell_start,
                     b.n_cells, g);
  hipLaunchKernelGGL(k_cell_scatter, grid_for(b.N), dim3(kBlock), 0, s, b.key, b.N,
                     b.cell_start, b.cell_fill, b.perm, g);
  hipLaunchKernelGGL(k_cell_sort, dim3(div_up(b.n_cells, kBlock / 64)), dim3(kBlock), 0, s, b.cell_start,
                     b.cell_count, b.n_cells, b.ext_src, b.perm, g);
  hipLaunchKernelGGL(k_gather_atoms, grid_for(b.N), dim3(kBlock), 0, s, b);
}

void launch_commit_rebuild(int64_t N, const double* pos2, const double* vel2, const int32_t* types2,
                           const int32_t* ext2, double* pos, double* vel, int32_t* types, int32_t* ext,
                           double* pos_ref, const int32_t* gate, hipStream_t s, double* mu_cum,
                           int32_t* count) {
  hipLaunchKernelGGL(k_commit_rebuild, grid_for(N), dim3(kBlock), 0, s, N, pos2, vel2, types2, ext2,
                     pos, vel, types, ext, pos_ref, gate, mu_cum, count);
}

void launch_build_rows(const BuildArgs& b, const StructInfo& st0, bool batch, const Lists& V,
                       const Lists& L, hipStream_t s) {
  BuildArgs bv = b;
  bv.gate = nullptr;
  launch_build_verlet(bv, V, s);
  launch_filter_rows(b, st0, batch, V, L, s);
}

void launch_reverse(int64_t N, const Lists& L, int32_t* err, const int32_t* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_reverse, grid_for(N * kReverseLanes), dim3(kBlock), 0, s, N, L.nnR, L.nlR, L.cdR, L.MR,
                     L.revR, err, gate);
}

// Candidate rows at sqrt(b.rcR2) and their reverse index, rebuilt when the
// gate is set.
void launch_build_verlet(const BuildArgs& b, const Lists& V, hipStream_t s) {
  // structures without cells take their rows from the wide kernel
  hipLaunchKernelGGL(k_build_rows, grid_for(b.N * kCellLanes), dim3(kBlock), 0, s, b.pos, b.N, b.sid,
                     b.structs, b.cell_start, b.cell_count, b.rcR2, V, b.overflow + 5, b.gate);
  if (b.wide_rows)
    hipLaunchKernelGGL(k_build_rows_wide, grid_for(b.N * kBuildLanes), dim3(kBlock), 0, s, b.pos, b.N,
                       b.sid, b.structs, b.rcR2, V, b.overflow + 5, b.gate);
  launch_reverse(b.N, V, b.overflow + 2, b.gate, s);
}

// Exact radial row from the candidate row with the same float64 membership
// test: the entries with |d|^2 < (r_c^A)^2 first, then the others, each part
// in candidate order; nnA = size of the first part.  V.fmap[m][i] = exact
// position of candidate m (or -1).  kFilterLanes lanes per atom take the
// candidates m = s, s + 4, ..., so the 16 atoms of a wave read and write
// whole 64-byte runs of a row.  Both passes walk a lane's candidates in
// chunks of kFilterChunk: the index words of a chunk are loaded together,
// then the positions (pass 1) or the row words (pass 2), so a lane has a
// chunk's loads in flight at once instead of one dependent chain per
// candidate.  Pass 1 classifies, counts the members and keeps the classes in
// register bit masks; pass 2 goes through the candidates in order, and
// counts over wave ballots of the class flags give each member its exact position.
// The rows are the same as those of a single sequential pass.
constexpr int kFilterLanes = 4;
constexpr int kFilterChunk = 4;

template <bool BATCH>
__global__ void __launch_bounds__(kBlock) k_filter_rows(const double* __restrict__ pos, int64_t N,
                                                        const int32_t* __restrict__ sid,
                                                        const StructInfo* __restrict__ structs,
                                                        StructInfo st0, Lists V, double rcR2,
                                                        double rcA2, Lists L,
                                                        int32_t* __restrict__ overflow) {
  constexpr int G = kFilterLanes, U = kFilterChunk;
  constexpr int32_t kOuter = -2, kAngular = -3;
  const int sub = threadIdx.x & (G - 1);
  const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / G;
  if (i >= N) return;  // the lanes of an atom leave together
  const StructInfo& st = BATCH ? structs[sid[i]] : st0;
  const int32_t* __restrict__ vnl = V.nlR;
  const uint16_t* __restrict__ vcd = V.cdR;
  const int32_t* __restrict__ vrev = V.revR;
  int32_t* __restrict__ fmap = V.fmap;
  int32_t* __restrict__ lnl = L.nlR;
  int32_t* __restrict__ lrev = L.revR;
  uint16_t* __restrict__ lcd = L.cdR;
  const int nv = min(V.nnR[i], V.MR);
  const int steps = (nv + G - 1) / G;  // the same for the four lanes of an atom
  const bool images = st.mode == kModeImages;
  const double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
  int32_t na = 0, no = 0;
  // classes of the lane's first 64 candidates (t = local index) as bit masks;
  // later ones (rows over 256 candidates) go through V.fmap
  uint64_t mask_a = 0, mask_o = 0;
  // the index words of chunk t0 + U are loaded while chunk t0's positions
  // are in flight
  int32_t jn[U];
  uint16_t cn[U];
  auto load_words = [&](int t0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = (t0 + u) * G + sub;
      jn[u] = (int32_t)i;  // past the row: the atom itself, in bounds and never classified
      cn[u] = kCodeCenter;
      if (m < nv) {
        jn[u] = vnl[(int64_t)m * N + i];
        if (images) cn[u] = vcd[(int64_t)m * N + i];
      }
    }
  };
  load_words(0);
  for (int t0 = 0; t0 < steps; t0 += U) {
    int32_t j[U];
    uint16_t code[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      j[u] = jn[u];
      code[u] = cn[u];
    }
    double px[U], py[U], pz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      px[u] = pos[j[u]];
      py[u] = pos[N + j[u]];
      pz[u] = pos[2 * N + j[u]];
    }
    if (t0 + U < steps) load_words(t0 + U);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u, m = t * G + sub;
      if (m >= nv) continue;
      double Dx, Dy, Dz;
      {
#pragma clang fp contract(off)
        Dx = px[u] - xi;
        Dy = py[u] - yi;
        Dz = pz[u] - zi;
      }
      int n0, n1, n2;
      min_image(st, Dx, Dy, Dz, n0, n1, n2);
      if (code[u] != kCodeCenter) {
        int oa, ob, oc;
        split_code(code[u], oa, ob, oc);
        n0 += oa;
        n1 += ob;
        n2 += oc;
      }
      double dx, dy, dz;
      image_disp(st, Dx, Dy, Dz, n0, n1, n2, dx, dy, dz);
      const double r2 = norm2_exact(dx, dy, dz);
      int32_t f = -1;
      if (r2 < rcA2) {
        f = kAngular;
        ++na;
      } else if (r2 < rcR2) {
        f = kOuter;
        ++no;
      }
      if (t < 64) {
        if (f == kAngular) mask_a |= 1ull << t;
        if (f == kOuter) mask_o |= 1ull << t;
      } else {
        fmap[(int64_t)m * N + i] = f;
      }
    }
  }
  int32_t a_all = na, o_all = no;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    a_all += __shfl_xor(a_all, off);
    o_all += __shfl_xor(o_all, off);
  }
  // pass 2: candidate m = G t + s is lane s's t-th; every lane of the atom's
  // group runs every step, so the group's ballot bits are whole at each step
  const int lane = threadIdx.x & 63;
  const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1)) << (lane & ~(G - 1));
  const uint64_t below = (1ull << lane) - 1;
  int32_t pa = 0, po = a_all;  // next angular / outer position
  // the members' words of chunk t0 + U are loaded while chunk t0 is placed
  int32_t cq[U], jq[U], rq[U];
  uint16_t kq[U];
  auto load_members = [&](int t0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u, m = t * G + sub;
      const int64_t e = (int64_t)m * N + i;
      cq[u] = -1;
      if (m < nv) {
        if (t < 64) cq[u] = ((mask_a >> t) & 1) ? kAngular : (((mask_o >> t) & 1) ? kOuter : -1);
        else cq[u] = fmap[e];
      }
      jq[u] = 0;
      rq[u] = 0;
      kq[u] = kCodeCenter;
      if (cq[u] != -1) {
        jq[u] = vnl[e];
        rq[u] = vrev[e];
        if (images) kq[u] = vcd[e];
      }
    }
  };
  load_members(0);
  for (int t0 = 0; t0 < steps; t0 += U) {
    int32_t c[U], jn[U], rn[U];
    uint16_t cn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = cq[u];
      jn[u] = jq[u];
      rn[u] = rq[u];
      cn[u] = kq[u];
    }
    if (t0 + U < steps) load_members(t0 + U);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = (t0 + u) * G + sub;
      const int64_t e = (int64_t)m * N + i;
      const int32_t fa = c[u] == kAngular, fo = c[u] == kOuter;
      const uint64_t ma = __ballot(fa) & gmask, mo = __ballot(fo) & gmask;
      const int32_t ta = __popcll(ma), to = __popcll(mo);
      const int32_t ba = __popcll(ma & below), bo = __popcll(mo & below);
      if (m < nv && !(fa | fo)) fmap[e] = -1;
      if (fa | fo) {
        const int32_t p = fa ? pa + ba : po + bo;
        fmap[e] = p;
        if (p < L.MR) {
          lnl[(int64_t)p * N + i] = jn[u];
          lrev[(int64_t)p * N + i] = rn[u];  // candidate position, resolved by the next kernel
          if (images) lcd[(int64_t)p * N + i] = cn[u];
        }
      }
      pa += ta;
      po += to;
    }
  }
  if (sub == 0) {
    const int32_t total = a_all + o_all;
    L.nnR[i] = total;
    L.nnA[i] = a_all;
    if (total > L.MR) atomicMax(&overflow[0], total);
    if (a_all > L.MA) atomicMax(&overflow[1], a_all);
  }
}

// rev of the exact rows: the filter left in L.revR[p][i] the candidate
// position of i in the row of j = L.nlR[p][i]; the exact position there is
// V.fmap of that candidate entry, written in place.  kRevLanes lanes per atom
// take exact entries p = s, s + 4, ..., so a wave writes whole 64-byte runs of
// a row; a lane loads the words of kFilterChunk entries, then their map
// entries, then writes them.
constexpr int kRevLanes = 4;

__global__ void __launch_bounds__(kBlock) k_reverse_from_candidates(int64_t N, Lists V, Lists L,
                                                                    int32_t* __restrict__ err) {
  constexpr int G = kRevLanes, U = kFilterChunk;
  const int sub = threadIdx.x & (G - 1);
  const int64_t i = (xcd_block() * blockDim.x + threadIdx.x) / G;
  if (i >= N) return;
  const int32_t* __restrict__ fmap = V.fmap;
  const int32_t* __restrict__ lnl = L.nlR;
  int32_t* __restrict__ lrev = L.revR;
  const int nn = min(L.nnR[i], L.MR);
  bool broken = false;
  // the words of chunk p0 + U G are loaded while chunk p0's map entries are in flight
  int32_t jq[U], rq[U];
  auto load_words = [&](int p0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * G;
      jq[u] = 0;
      rq[u] = 0;
      if (p < nn) {
        jq[u] = lnl[(int64_t)p * N + i];
        rq[u] = lrev[(int64_t)p * N + i];
      }
    }
  };
  load_words(sub);
  for (int p0 = sub; p0 < nn; p0 += U * G) {
    int32_t j[U], r[U], g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      j[u] = jq[u];
      r[u] = rq[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = p0 + u * G < nn ? fmap[(int64_t)r[u] * N + j[u]] : 0;
    if (p0 + U * G < nn) load_words(p0 + U * G);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * G;
      if (p >= nn) continue;
      if (g[u] < 0) {
        broken = true;
        g[u] = 0;
      }
      lrev[(int64_t)p * N + i] = min(g[u], L.MR - 1);
    }
  }
  if (broken) atomicExch(err, 1);
}

// Checks, for every atom i of the exact rows, the invariants under which the
// evaluation kernels only touch memory inside their buffers: nnA <= nnR <= MR;
// every neighbour j lies in i's structure; its reverse position r lies in
// j's row (r < nnR[j]) and that entry points back to i with the opposite
// image code; image codes stay within the structure's image reach.  Any
// violation sets a bit of *bad (1: counts, 2: neighbour index, 4: reverse
// position, 8: reverse entry, 16: image code); rows that overflowed their
// capacity are reported by the overflow flags instead.
constexpr int kCheckLanes = 4;  // lanes per atom of k_check_rows (entries s, s + 4, ...)
constexpr int kCheckChunk = 4;  // entries a lane checks together

__global__ void __launch_bounds__(kBlock) k_check_rows(int64_t N, const int32_t* __restrict__ sid,
                                                       const StructInfo* __restrict__ structs,
                                                       StructInfo st0, int32_t batch, Lists L,
                                                       int32_t* __restrict__ bad) {
  constexpr int G = kCheckLanes, U = kCheckChunk;
  const int sub = threadIdx.x & (G - 1);
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (i >= N) return;
  const StructInfo& st = batch ? structs[sid[i]] : st0;
  const int nn = L.nnR[i], na = L.nnA[i];
  if (nn > L.MR) return;  // overflow: reported and handled by the caller
  int32_t b = 0;
  if (sub == 0 && (na < 0 || nn < 0 || na > nn)) b |= 1;
  const bool images = st.mode == kModeImages;
  const int64_t lo = st.start, hi = st.start + st.count;
  // a chunk's index words first, then the partners' row lengths and reverse
  // entries (each read only when the words before it are in bounds)
  for (int m0 = sub; m0 < max(nn, 0); m0 += U * G) {
    int32_t j[U], r[U];
    bool jok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = m0 + u * G;
      j[u] = 0;
      r[u] = 0;
      if (m < nn) {
        j[u] = L.nlR[(int64_t)m * N + i];
        r[u] = L.revR[(int64_t)m * N + i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      jok[u] = m0 + u * G < nn && j[u] >= lo && j[u] < hi;
      if (m0 + u * G < nn && !jok[u]) b |= 2;
    }
    int nj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) nj[u] = jok[u] ? L.nnR[j[u]] : 0;
    int32_t back[U];
    bool rok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rok[u] = jok[u] && r[u] >= 0 && r[u] < min(nj[u], L.MR);
      if (jok[u] && !rok[u]) b |= 4;
      back[u] = rok[u] ? L.nlR[(int64_t)r[u] * N + j[u]] : (int32_t)i;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!rok[u]) continue;
      if (back[u] != (int32_t)i) b |= 8;
      if (images) {
        const int64_t e = (int64_t)(m0 + u * G) * N + i, er = (int64_t)r[u] * N + j[u];
        int oa, ob, oc, ra, rb, rc;
        split_code(L.cdR[e], oa, ob, oc);
        split_code(L.cdR[er], ra, rb, rc);
        if (oa != -ra || ob != -rb || oc != -rc) b |= 8;
        if (abs(oa) > st.reach[0] || abs(ob) > st.reach[1] || abs(oc) > st.reach[2]) b |= 16;
      }
    }
  }
  if (b) atomicOr(bad, b);
}

void launch_check_rows(int64_t N, const int32_t* sid, const StructInfo* structs, const StructInfo& st0,
                       bool batch, const Lists& L, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_check_rows, grid_for(N * kCheckLanes), dim3(kBlock), 0, s, N, sid, structs, st0,
                     (int32_t)(batch ? 1 : 0), L, bad);
}

void launch_filter_rows(const BuildArgs& b, const StructInfo& st0, bool batch, const Lists& V,
                        const Lists& L, hipStream_t s) {
  const dim3 grid = grid_for(b.N * kFilterLanes);
  if (batch)
    hipLaunchKernelGGL(k_filter_rows<true>, grid, dim3(kBlock), 0, s, b.pos, b.N, b.sid, b.structs,
                       st0, V, b.rcR2, b.rcA2, L, b.overflow);
  else
    hipLaunchKernelGGL(k_filter_rows<false>, grid, dim3(kBlock), 0, s, b.pos, b.N, b.sid, b.structs,
                       st0, V, b.rcR2, b.rcA2, L, b.overflow);
  hipLaunchKernelGGL(k_reverse_from_candidates, grid_for(b.N * kRevLanes), dim3(kBlock), 0, s,
                     b.N, V, L, b.overflow + 2);
}

// flag = any atom whose displacement since the last build, plus horizon
// times its speed when vel is given, exceeds half the skin: |r_i - r_i(build)|
// + horizon |v_i| > sqrt(thr2) (the plain test |r_i - r_i(build)|^2 > thr2
// when horizon is 0).  With a box scaled by mu since the build (NPT), a pair
// within r_c now was within r_c + skin then as long as every
// |r_i - mu r_i(build)| <= (mu (r_c + skin) - r_c) / 2.
__global__ void k_check_displacement(const double* __restrict__ pos, const double* __restrict__ ref,
                                     const double* __restrict__ vel, int64_t N, double thr2,
                                     double horizon, int32_t* __restrict__ flag,
                                     const double* __restrict__ mu_cum, double rc, double rl) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double m = 1.0, t2 = thr2;
  if (mu_cum) {
    m = *mu_cum;
    const double a = fmax(0.0, 0.5 * (m * rl - rc));
    t2 = a * a;
  }
  const double dx = pos[i] - m * ref[i], dy = pos[N + i] - m * ref[N + i],
               dz = pos[2 * N + i] - m * ref[2 * N + i];
  const double d2 = dx * dx + dy * dy + dz * dz;
  bool out = d2 > t2;
  if (vel && horizon > 0.0) {
    const double vx = vel[i], vy = vel[N + i], vz = vel[2 * N + i];
    out = sqrt(d2) + horizon * sqrt(vx * vx + vy * vy + vz * vz) > sqrt(t2);
  }
  if (out) atomicExch(flag, 1);
}

void launch_check_displacement(const double* pos, const double* ref, const double* vel, int64_t N,
                               double thr2, double horizon, int32_t* flag, hipStream_t s,
                               const double* mu_cum, double rc, double rl) {
  hipLaunchKernelGGL(k_check_displacement, grid_for(N), dim3(kBlock), 0, s, pos, ref, vel, N, thr2, horizon,
                     flag, mu_cum, rc, rl);
}

template <class T>
__global__ void k_copy_gated(T* __restrict__ dst, const T* __restrict__ src, int64_t n,
                             const int32_t* gate) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !gated_off(gate)) dst[i] = src[i];
}

void launch_copy_gated_f64(double* dst, const double* src, int64_t n, const int32_t* gate,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_copy_gated<double>, grid_for(n), dim3(kBlock), 0, s, dst, src, n, gate);
}

void launch_copy_gated_i32(int32_t* dst, const int32_t* src, int64_t n, const int32_t* gate,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_copy_gated<int32_t>, grid_for(n), dim3(kBlock), 0, s, dst, src, n, gate);
}

int64_t type_row_blocks(int64_t N) { return div_up(N, kBlock); }

void launch_type_rows(const int32_t* types, int64_t N, int32_t T, int32_t per_type,
                      int32_t* tblk, int32_t* tex, int32_t* toff, int32_t* rows,
                      int64_t rows_len, const int32_t* gate, hipStream_t s) {
  const int32_t Tn = per_type ? T : 1;
  const int32_t nb = (int32_t)type_row_blocks(N);
  hipLaunchKernelGGL(k_type_block_count, dim3(nb), dim3(kBlock), 0, s, types, N, Tn, per_type, nb,
                     tblk, rows, rows_len, gate);
  hipLaunchKernelGGL(k_scan_1block, dim3(1), dim3(1024), 0, s, tblk, tex, Tn * nb, gate);
  hipLaunchKernelGGL(k_type_shift, dim3(1), dim3(64), 0, s, tex, N, Tn, nb, toff, gate);
  hipLaunchKernelGGL(k_type_block_scatter, dim3(nb), dim3(kBlock), 0, s, types, N, Tn, per_type,
                     nb, tex, toff, rows, gate);
}

}  // namespace nep
