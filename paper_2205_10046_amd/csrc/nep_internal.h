// nep_internal.h -- data layouts and device helpers shared by the HIP kernels
// of the NEP library (never seen by callers of nep.h).
//
// Layout in device memory (N = atom capacity of the workspace, "internal"
// atom order = structure-major, then cell-major, then caller index):
//   pos      float64 [3][N]           SoA, internal order
//   nl_*     int32   [M][N]           neighbour m of atom i at nl[m*N + i]
//   cd_*     uint16  [M][N]           image offset code of that entry (exact rows:
//                                     stored only for kModeImages structures)
//   revR     int32   [MR][N]          position of i in the radial row of that j
//   nnA                               the angular row is the first nnA[i] entries
//                                     of the radial row
//   V.*      int32/uint16 [MV][N]     candidate rows (radius r_c^R + skin), their
//                                     reverse index and candidate -> exact map
//   q, fp    float32 [N][ND_pad]      descriptor / dU/dq rows (network input)
//   sums     float32 [NA*NB][N]       angular sums S_{n,k}, SoA
//   P        float32x4 [MR][N]        dU_i/dr_ij per radial entry, radial and
//                                     angular parts summed (w unused)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nep {

constexpr int kBlock = 256;
// The network pass takes the species-grouped rows four 16-row tiles at a
// time; every species segment is padded to this many rows, so such a group
// never mixes species.
constexpr int kRowGroup = 64;
constexpr int kMaxL = 6;
constexpr int kMaxNB = (kMaxL + 1) * (kMaxL + 1) - 1;
constexpr int kMaxBasis = 16;    // N_bas + 1 and n_max + 1 limits
constexpr int kMaxTypes = 8;
constexpr uint16_t kCodeCenter = 0x888;  // image offset (0, 0, 0)

// How the neighbour images of one structure are found.
enum StructMode : int32_t {
  kModeCells = 0,      // minimum image, cell list
  kModeAllPairs = 1,   // minimum image, every atom of the structure
  kModeImages = 2,     // several images: every atom x offsets in [-R, R]^3
};

// Per-structure geometry (float64, device).  H rows are the cell vectors;
// Hi is H^{-1} so the fractional offset of a displacement d is d * Hi.
struct StructInfo {
  double H[9];
  double Hi[9];
  int64_t start;       // first internal atom
  int64_t count;       // atoms in the structure
  int32_t pbc[3];
  int32_t mode;
  int32_t ncell[3];    // cells per cell vector (kModeCells), else 1
  int32_t cell_off;    // first global cell id
  int32_t reach[3];    // image offset range R (kModeImages)
  int32_t ortho;       // 1: H is diagonal (every off-diagonal entry exactly 0)
};

__host__ __device__ inline uint16_t make_code(int a, int b, int c) {
  return (uint16_t)(((a + 8) << 8) | ((b + 8) << 4) | (c + 8));
}
__host__ __device__ inline void split_code(uint16_t code, int& a, int& b, int& c) {
  a = ((code >> 8) & 15) - 8;
  b = ((code >> 4) & 15) - 8;
  c = (code & 15) - 8;
}

// Minimum-image offset n0 = -rint(s) of the fractional bond offset s along
// each periodic cell vector (0 along open directions).
// For a diagonal H the off-diagonal products are exact zeros, so the
// diagonal-only forms below give the same bits as the general ones.
__device__ inline void min_image(const StructInfo& st, double Dx, double Dy, double Dz,
                                 int& n0, int& n1, int& n2) {
  n0 = n1 = n2 = 0;
  if (st.ortho) {
    if (st.pbc[0]) n0 = -(int)rint(Dx * st.Hi[0]);
    if (st.pbc[1]) n1 = -(int)rint(Dy * st.Hi[4]);
    if (st.pbc[2]) n2 = -(int)rint(Dz * st.Hi[8]);
    return;
  }
  if (st.pbc[0]) n0 = -(int)rint(Dx * st.Hi[0] + Dy * st.Hi[3] + Dz * st.Hi[6]);
  if (st.pbc[1]) n1 = -(int)rint(Dx * st.Hi[1] + Dy * st.Hi[4] + Dz * st.Hi[7]);
  if (st.pbc[2]) n2 = -(int)rint(Dx * st.Hi[2] + Dy * st.Hi[5] + Dz * st.Hi[8]);
}

// d = (r_j - r_i) + ((n0 a + n1 b) + n2 c) with every product and sum rounded
// separately (no fused multiply-add), so that neighbour membership decided
// from |d|^2 is reproducible bit for bit.
__device__ inline void image_disp(const StructInfo& st, double Dx, double Dy, double Dz,
                                  int n0, int n1, int n2, double& dx, double& dy,
                                  double& dz) {
#pragma clang fp contract(off)
  const double a = (double)n0, b = (double)n1, c = (double)n2;
  if (st.ortho) {
    dx = Dx + a * st.H[0];
    dy = Dy + b * st.H[4];
    dz = Dz + c * st.H[8];
    return;
  }
  double tx = (a * st.H[0] + b * st.H[3]) + c * st.H[6];
  double ty = (a * st.H[1] + b * st.H[4]) + c * st.H[7];
  double tz = (a * st.H[2] + b * st.H[5]) + c * st.H[8];
  dx = Dx + tx;
  dy = Dy + ty;
  dz = Dz + tz;
}

__device__ inline double norm2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// Displacement of list entry (i -> j, code) from internal positions.
__device__ inline void entry_disp(const double* __restrict__ pos, int64_t N, int64_t i,
                                  int64_t j, const StructInfo& st, uint16_t code,
                                  double& dx, double& dy, double& dz) {
#pragma clang fp contract(off)
  double Dx = pos[j] - pos[i];
  double Dy = pos[N + j] - pos[N + i];
  double Dz = pos[2 * N + j] - pos[2 * N + i];
  int n0, n1, n2;
  min_image(st, Dx, Dy, Dz, n0, n1, n2);
  if (code != kCodeCenter) {
    int a, b, c;
    split_code(code, a, b, c);
    n0 += a;
    n1 += b;
    n2 += c;
  }
  image_disp(st, Dx, Dy, Dz, n0, n1, n2, dx, dy, dz);
}

// Row length of a group of NG radial functions in the angular table.
__host__ __device__ constexpr int ng_pad(int ng) { return ng <= 2 ? ng : (ng + 3) / 4 * 4; }
__host__ __device__ constexpr int round4(int n) { return (n + 3) / 4 * 4; }
// Smallest stride >= n floats that is 4 mod 64 (bank-spread species pairs).
__host__ __device__ constexpr int pair_stride(int n) { return n + ((4 - n % 64) + 64) % 64; }

// Model tables in device memory, float32 (converted once from the float64
// parameter vector).  c tables are zero-padded to whole groups of radial
// functions so kernels never test n < n_max + 1.
struct DevModel {
  int32_t T, nR, KR, nA, KA, L, NB, ND, NDp, NN, nets, has4b, has5b;
  int32_t cA_max;           // largest angular table (floats) over the group sizes
  float rcR, rcA;
  const float* b1;          // the output bias b1, one float in device memory
  const float* cR;          // [T][T][nR][KR]
  // angular coefficients for group size NG at cA + cA_off[NG] (-1: none):
  // [T x T species pairs, cA_pair[NG] floats apart][groups][KA][ng_pad(NG)],
  // the NG functions of a group contiguous (zero beyond n_A), so one aligned
  // vector read serves a whole group; the pair stride is 4 mod 64 floats so
  // lanes reading different species pairs fall into different LDS banks
  const float* cA;
  int32_t cA_off[8];
  int32_t cA_pair[8];
  int32_t NNp;              // N_neu rounded up to 32 (zero-padded neurons)
  int32_t NDp32;            // N_des rounded up to 32
  const float* w0;          // [nets][NNp][ND]   network weights w0, row = neuron
  const float* w0t;         // [nets][ND][NNp]   the same, transposed
  const float* b0;          // [nets][NNp], then b1
  const float* w1;          // [nets][NNp]
  const uint16_t* w0b;      // [nets][NNp][NDp32] w0 as bf16 bits
  const uint16_t* w0tb;     // [nets][NDp32][NNp] transposed, bf16 bits
  float C3[kMaxNB];
  float C4[5];
  float C5[3];
};

// Internal neighbour lists of one build.  Row capacities stay below 65535
// so positions inside a row fit the uint16 maps.
struct Lists {
  int32_t MR, MA;           // row capacities
  int32_t* nnR;
  int32_t* nlR;
  uint16_t* cdR;
  int32_t* revR;
  int32_t* nnA;
  int32_t* nlA;
  uint16_t* cdA;
  int32_t* fmap;            // candidate rows only: candidate -> exact position, or -1
};

constexpr int32_t kMaxRow = 65535;

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// The chip deals the blocks of a grid to its 8 XCDs round-robin (block b
// runs on XCD b mod 8), each XCD with its own L2.  Numbering the work so that
// the blocks of one XCD take one contiguous range of atoms keeps the
// neighbours that its concurrent blocks share in that L2.  A bijection on
// [0, gridDim.x) for any grid size.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + k;
}

}  // namespace nep
