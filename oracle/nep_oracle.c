/*
 * nep_oracle.c -- plain FP64 reference implementation of the NEP3 potential
 * (site energy, forces, per-atom virial) and of velocity-Verlet NVE dynamics.
 *
 * TEST INFRASTRUCTURE.  This is the checker the HIP library is compared with.
 * Only the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header, table, constant generator or
 * pre/post-processing with the HIP library, and never calls it.
 *
 * Written for reading, not speed: every quantity is evaluated straight from
 * its definition in the paper (Fan et al., "GPUMD: a package for constructing
 * accurate machine-learned potentials and performing highly efficient
 * atomistic simulations", Sec. II), in double precision, with no blocking or
 * fusion.  Build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Readings adopted where the paper is silent or garbled:
 *   - S_{n,k} divides b_k by r^l with l the degree of b_k (the printed power
 *     r^n clashes with the radial index n); the b_k/r^l are then functions of
 *     the bond direction only, which is what the spherical harmonics are.
 *   - the weight in the addition-theorem form is (2 - delta_{0m}).
 *   - l = 5, 6 (not printed) use the real solid harmonics
 *     r^{l-m} P_l^{(m)}(z/r) * {Re, Im}(x + i y)^m with the addition-theorem
 *     weights (2l+1)/(4 pi) (2 - delta_{m0}) (l-m)!/(l+m)!.
 *   - descriptor order: radial q_n, then q_{nl} (l-major), then q_{n222},
 *     then q_{n1111}.
 *   - parameter blob order: per network [w0 (N_neu x N_des, row major), b0,
 *     w1], then the shared b1, then c^R[ti][tj][n][k], then c^A[ti][tj][n][k].
 *   - neighbour membership is the strict FP64 test |d|^2 < r_c^2 with
 *     d = (r_j - r_i) + ((n_a a + n_b b) + n_c c) evaluated in exactly that
 *     order and |d|^2 = (d_x d_x + d_y d_y) + d_z d_z.
 *   - "4-body" is q_{n222} and "5-body" is q_{n1111}, whatever l_max^3b is.
 *
 * Every function is pinned by tests against an independent definition: the
 * Legendre double sum, complex spherical harmonics with Wigner 3j couplings,
 * finite differences of the energy, invariances, the virial-strain relation
 * and NVE energy conservation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ===================================================================== */
/* hyper-parameters and sizes                                             */
/* ===================================================================== */

typedef struct {
  int32_t n_types;
  double rc_radial, rc_angular;
  int32_t n_max_radial, n_max_angular;
  int32_t basis_radial, basis_angular;
  int32_t l_max_3b, l_max_4b, l_max_5b;
  int32_t n_neurons;
  int32_t nn_per_type;
} ora_hparams;

enum { ORA_OK = 0, ORA_EARG = 1, ORA_EMEM = 3 };

#define ORA_LMAX 6
#define ORA_NB_MAX ((ORA_LMAX + 1) * (ORA_LMAX + 1) - 1)

static int n_rad(const ora_hparams *h) { return h->n_max_radial + 1; }
static int n_ang(const ora_hparams *h) { return h->n_max_angular + 1; }
static int k_rad(const ora_hparams *h) { return h->basis_radial + 1; }
static int k_ang(const ora_hparams *h) { return h->basis_angular + 1; }
static int use4b(const ora_hparams *h) { return h->l_max_4b >= 2; }
static int use5b(const ora_hparams *h) { return h->l_max_5b >= 1; }
static int n_poly(int lmax) { return (lmax + 1) * (lmax + 1) - 1; }

/* Sec. II.D: N_des = (n_max^R + 1) + (n_max^A + 1)(l_max^3b + [4b] + [5b]). */
int ora_num_descriptors(const ora_hparams *h) {
  return n_rad(h) + n_ang(h) * (h->l_max_3b + use4b(h) + use5b(h));
}

/* Sec. II.E, NEP3 parameter count.  With one network per species the network
 * block (N_des + 2) N_neu is repeated per species; b1 stays one number. */
int64_t ora_num_params(const ora_hparams *h) {
  int64_t nd = ora_num_descriptors(h);
  int64_t nets = h->nn_per_type ? h->n_types : 1;
  int64_t t2 = (int64_t)h->n_types * h->n_types;
  return nets * (nd + 2) * h->n_neurons + 1 + t2 * n_rad(h) * k_rad(h) +
         t2 * n_ang(h) * k_ang(h);
}

static int check_hp(const ora_hparams *h) {
  if (h->n_types < 1 || h->n_neurons < 1) return ORA_EARG;
  if (!(h->rc_radial > 0) || !(h->rc_angular > 0) ||
      h->rc_angular > h->rc_radial)
    return ORA_EARG;
  if (h->n_max_radial < 0 || h->n_max_angular < 0 || h->basis_radial < 0 ||
      h->basis_angular < 0)
    return ORA_EARG;
  if (h->l_max_3b < 1 || h->l_max_3b > ORA_LMAX) return ORA_EARG;
  if (h->l_max_4b < 0 || h->l_max_4b > 3 || h->l_max_5b < 0 || h->l_max_5b > 1)
    return ORA_EARG;
  if (use4b(h) && h->l_max_3b < 2) return ORA_EARG;
  return ORA_OK;
}

/* ===================================================================== */
/* cell geometry                                                          */
/* ===================================================================== */

/* box rows are the cell vectors a, b, c; a position is r = s_a a + s_b b + s_c c,
 * i.e. the row vector r = s H, so s = r H^{-1}. */
static void box_inverse(const double *H, double *Hi) {
  double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6],
         hh = H[7], k = H[8];
  double det = a * (e * k - f * hh) - b * (d * k - f * g) + c * (d * hh - e * g);
  Hi[0] = (e * k - f * hh) / det;
  Hi[1] = (c * hh - b * k) / det;
  Hi[2] = (b * f - c * e) / det;
  Hi[3] = (f * g - d * k) / det;
  Hi[4] = (a * k - c * g) / det;
  Hi[5] = (c * d - a * f) / det;
  Hi[6] = (d * hh - e * g) / det;
  Hi[7] = (b * g - a * hh) / det;
  Hi[8] = (a * e - b * d) / det;
}

static void cross3(const double *u, const double *v, double *w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

/* distance between opposite faces of the cell, per cell vector */
static void face_widths(const double *H, double *w) {
  double bc[3], ca[3], ab[3];
  cross3(H + 3, H + 6, bc);
  cross3(H + 6, H + 0, ca);
  cross3(H + 0, H + 3, ab);
  double vol = fabs(H[0] * bc[0] + H[1] * bc[1] + H[2] * bc[2]);
  w[0] = vol / sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  w[1] = vol / sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
  w[2] = vol / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
}

/* d = (r_j - r_i) + ((n_a a + n_b b) + n_c c); returns |d|^2 */
static double displacement(const double *pos, int64_t N, int64_t i, int64_t j,
                           const int32_t *n, const double *H, double *d) {
  for (int c = 0; c < 3; ++c) {
    double delta = pos[c * N + j] - pos[c * N + i];
    double t = ((double)n[0] * H[0 + c] + (double)n[1] * H[3 + c]) +
               (double)n[2] * H[6 + c];
    d[c] = delta + t;
  }
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* ===================================================================== */
/* neighbour environments (the sums over j != i of Sec. II.B, II.C)       */
/* ===================================================================== */

typedef struct {
  int32_t j;
  int32_t n[3];
  double d[3];
  double r;
} ora_pair;

typedef struct {
  int count, cap;
  ora_pair *p;
} ora_list;

static int list_push(ora_list *L, int32_t j, const int32_t *n, const double *d,
                     double r2) {
  if (L->count == L->cap) {
    int nc = L->cap ? 2 * L->cap : 64;
    ora_pair *np = (ora_pair *)realloc(L->p, (size_t)nc * sizeof(ora_pair));
    if (!np) return ORA_EMEM;
    L->p = np;
    L->cap = nc;
  }
  ora_pair *q = &L->p[L->count++];
  q->j = j;
  q->n[0] = n[0];
  q->n[1] = n[1];
  q->n[2] = n[2];
  q->d[0] = d[0];
  q->d[1] = d[1];
  q->d[2] = d[2];
  q->r = sqrt(r2);
  return ORA_OK;
}

static void list_free(ora_list *L) {
  free(L->p);
  L->p = NULL;
  L->count = L->cap = 0;
}

/* Integer image range that contains every image n with |d| < rc along each
 * periodic direction: the fractional offset of the bond along cell vector k
 * lies within rc / w_k of zero. */
static void image_range(const double *pos, int64_t N, int64_t i, int64_t j,
                        const double *Hi, const double *w, const int32_t *pbc,
                        double rc, int32_t *lo, int32_t *hi) {
  double delta[3];
  for (int c = 0; c < 3; ++c) delta[c] = pos[c * N + j] - pos[c * N + i];
  for (int k = 0; k < 3; ++k) {
    if (!pbc[k]) {
      lo[k] = hi[k] = 0;
      continue;
    }
    double s = delta[0] * Hi[0 * 3 + k] + delta[1] * Hi[1 * 3 + k] +
               delta[2] * Hi[2 * 3 + k];
    double reach = rc / w[k];
    lo[k] = (int32_t)floor(-s - reach) - 1;
    hi[k] = (int32_t)ceil(-s + reach) + 1;
  }
}

/* All (j, n) with |d|^2 < rc^2 except (i, 0): j ascending, then n in
 * lexicographic order.  Brute force over every atom and image. */
static int environment(const double *pos, int64_t N, int64_t i, const double *H,
                       const double *Hi, const double *w, const int32_t *pbc,
                       double rc, ora_list *out) {
  out->count = 0;
  double rc2 = rc * rc;
  for (int64_t j = 0; j < N; ++j) {
    int32_t lo[3], hi[3], n[3];
    image_range(pos, N, i, j, Hi, w, pbc, rc, lo, hi);
    for (n[0] = lo[0]; n[0] <= hi[0]; ++n[0])
      for (n[1] = lo[1]; n[1] <= hi[1]; ++n[1])
        for (n[2] = lo[2]; n[2] <= hi[2]; ++n[2]) {
          if (j == i && n[0] == 0 && n[1] == 0 && n[2] == 0) continue;
          double d[3];
          double r2 = displacement(pos, N, i, j, n, H, d);
          if (r2 < rc2) {
            if (list_push(out, (int32_t)j, n, d, r2)) return ORA_EMEM;
          }
        }
  }
  return ORA_OK;
}

/* Public: neighbour lists at one cutoff for every atom.  Rows are written in
 * the environment's order (j ascending, then image).  Returns the largest row
 * length in *max_count; rows beyond cap are counted but not stored. */
int ora_pairs(int64_t N, const double *pos, const double *box,
              const int32_t *pbc, double rc, int32_t cap, int32_t *count,
              int32_t *nbr, int32_t *shift, int32_t *max_count) {
  double Hi[9], w[3];
  box_inverse(box, Hi);
  face_widths(box, w);
  int err = ORA_OK, mx = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(max : mx)
  for (int64_t i = 0; i < N; ++i) {
    ora_list L = {0, 0, NULL};
    if (environment(pos, N, i, box, Hi, w, pbc, rc, &L)) {
      err = ORA_EMEM;
    } else {
      count[i] = L.count;
      if (L.count > mx) mx = L.count;
      for (int m = 0; m < L.count && m < cap; ++m) {
        nbr[i * cap + m] = L.p[m].j;
        for (int c = 0; c < 3; ++c) shift[(i * cap + m) * 3 + c] = L.p[m].n[c];
      }
    }
    list_free(&L);
  }
  *max_count = mx;
  return err;
}

/* ===================================================================== */
/* radial functions: eqs. (g_n), (f_n) and the cutoff function, Sec. II.B  */
/* ===================================================================== */

/* f_k(r) = 1/2 [T_k(2 (r/rc - 1)^2 - 1) + 1] f_c(r), k = 0..K-1, and df_k/dr.
 * f_c = 1/2 [1 + cos(pi r / rc)] for r <= rc, else 0. */
void ora_radial_basis(double rc, int K, double r, double *f, double *df) {
  double fc = 0.0, dfc = 0.0;
  if (r <= rc) {
    fc = 0.5 * (1.0 + cos(M_PI * r / rc));
    dfc = -0.5 * (M_PI / rc) * sin(M_PI * r / rc);
  }
  double t = r / rc - 1.0;
  double x = 2.0 * t * t - 1.0;
  double dxdr = 4.0 * t / rc;
  double T[64], dT[64];
  T[0] = 1.0;
  dT[0] = 0.0;
  if (K > 1) {
    T[1] = x;
    dT[1] = 1.0;
  }
  for (int k = 1; k + 1 < K; ++k) {
    /* Chebyshev recurrence T_{k+1} = 2 x T_k - T_{k-1}, differentiated */
    T[k + 1] = 2.0 * x * T[k] - T[k - 1];
    dT[k + 1] = 2.0 * T[k] + 2.0 * x * dT[k] - dT[k - 1];
  }
  for (int k = 0; k < K; ++k) {
    f[k] = 0.5 * (T[k] + 1.0) * fc;
    df[k] = 0.5 * dT[k] * dxdr * fc + 0.5 * (T[k] + 1.0) * dfc;
  }
}

/* g_n(r) = sum_k c^{t_i t_j}_{nk} f_k(r) for n = 0..nn-1, and dg_n/dr */
static void radial_functions(const double *c, int nn, int K, double rc, double r,
                             double *g, double *dg) {
  double f[64], df[64];
  ora_radial_basis(rc, K, r, f, df);
  for (int n = 0; n < nn; ++n) {
    double s = 0.0, ds = 0.0;
    for (int k = 0; k < K; ++k) {
      s += c[n * K + k] * f[k];
      ds += c[n * K + k] * df[k];
    }
    g[n] = s;
    dg[n] = ds;
  }
}

/* ===================================================================== */
/* angular polynomials b_k and their coefficients, Sec. II.C, II.D         */
/* ===================================================================== */

/* The 24 polynomials listed with eq. (S_nk), l = 1..4, and their gradients. */
static void poly_l4(const double *d, double *b, double *g) {
  double x = d[0], y = d[1], z = d[2];
  double x2 = x * x, y2 = y * y, z2 = z * z, r2 = x2 + y2 + z2;
#define SETB(k, v, gx, gy, gz) \
  do {                         \
    b[k] = (v);                \
    g[3 * (k) + 0] = (gx);     \
    g[3 * (k) + 1] = (gy);     \
    g[3 * (k) + 2] = (gz);     \
  } while (0)
  /* l = 1 */
  SETB(0, z, 0.0, 0.0, 1.0);
  SETB(1, x, 1.0, 0.0, 0.0);
  SETB(2, y, 0.0, 1.0, 0.0);
  /* l = 2 */
  SETB(3, 3.0 * z2 - r2, -2.0 * x, -2.0 * y, 4.0 * z);
  SETB(4, x * z, z, 0.0, x);
  SETB(5, y * z, 0.0, z, y);
  SETB(6, x2 - y2, 2.0 * x, -2.0 * y, 0.0);
  SETB(7, 2.0 * x * y, 2.0 * y, 2.0 * x, 0.0);
  /* l = 3 */
  SETB(8, (5.0 * z2 - 3.0 * r2) * z, -6.0 * x * z, -6.0 * y * z,
       6.0 * z2 - 3.0 * x2 - 3.0 * y2);
  SETB(9, (5.0 * z2 - r2) * x, 4.0 * z2 - 3.0 * x2 - y2, -2.0 * x * y,
       8.0 * x * z);
  SETB(10, (5.0 * z2 - r2) * y, -2.0 * x * y, 4.0 * z2 - x2 - 3.0 * y2,
       8.0 * y * z);
  SETB(11, (x2 - y2) * z, 2.0 * x * z, -2.0 * y * z, x2 - y2);
  SETB(12, 2.0 * x * y * z, 2.0 * y * z, 2.0 * x * z, 2.0 * x * y);
  SETB(13, (x2 - 3.0 * y2) * x, 3.0 * x2 - 3.0 * y2, -6.0 * x * y, 0.0);
  SETB(14, (3.0 * x2 - y2) * y, 6.0 * x * y, 3.0 * x2 - 3.0 * y2, 0.0);
  /* l = 4 */
  {
    double A = 7.0 * z2 - 3.0 * r2; /* for k = 16, 17 */
    double B = 7.0 * z2 - r2;       /* for k = 18, 19 */
    double D = x2 - y2, E = 2.0 * x * y;
    SETB(15, (35.0 * z2 - 30.0 * r2) * z2 + 3.0 * r2 * r2,
         x * (12.0 * r2 - 60.0 * z2), y * (12.0 * r2 - 60.0 * z2),
         80.0 * z2 * z - 48.0 * r2 * z);
    SETB(16, A * x * z, z * (A - 6.0 * x2), -6.0 * x * y * z,
         x * (15.0 * z2 - 3.0 * r2));
    SETB(17, A * y * z, -6.0 * x * y * z, z * (A - 6.0 * y2),
         y * (15.0 * z2 - 3.0 * r2));
    SETB(18, B * D, 2.0 * x * (B - D), -2.0 * y * (B + D), 12.0 * z * D);
    SETB(19, B * E, -2.0 * x * E + 2.0 * y * B, -2.0 * y * E + 2.0 * x * B,
         12.0 * z * E);
    SETB(20, (x2 - 3.0 * y2) * x * z, z * (3.0 * x2 - 3.0 * y2), -6.0 * x * y * z,
         (x2 - 3.0 * y2) * x);
    SETB(21, (3.0 * x2 - y2) * y * z, 6.0 * x * y * z, z * (3.0 * x2 - 3.0 * y2),
         (3.0 * x2 - y2) * y);
    SETB(22, D * D - 4.0 * x2 * y2, 4.0 * x * (x2 - 3.0 * y2),
         -4.0 * y * (3.0 * x2 - y2), 0.0);
    SETB(23, 4.0 * D * x * y, 4.0 * y * (3.0 * x2 - y2), 4.0 * x * (x2 - 3.0 * y2),
         0.0);
  }
#undef SETB
}

static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

static double binom(int n, int k) {
  return factorial(n) / (factorial(k) * factorial(n - k));
}

/* Coefficients p_t of the m-th derivative of the Legendre polynomial P_l:
 * P_l^{(m)}(u) = sum_t p[t] u^t, t = 0..l-m. */
static void legendre_derivative(int l, int m, double *p) {
  double c[16] = {0};
  for (int j = 0; 2 * j <= l; ++j)
    c[l - 2 * j] = pow(-1.0, j) * binom(l, j) * binom(2 * l - 2 * j, l) / pow(2.0, l);
  for (int t = 0; t <= l - m; ++t) p[t] = c[t + m] * factorial(t + m) / factorial(t);
}

/* Real solid harmonic of degree l, order m >= 0, cosine (sc = 0) or sine
 * (sc = 1) part: r^{l-m} P_l^{(m)}(z/r) {Re,Im}(x+iy)^m, as a polynomial in
 * x, y, z, with its gradient. */
static void solid_harmonic(int l, int m, int sc, const double *d, double *val,
                           double *grad) {
  double x = d[0], y = d[1], z = d[2];
  double rho = x * x + y * y + z * z;
  double p[16];
  legendre_derivative(l, m, p);
  /* A(z, rho) = sum_t p_t z^t rho^{(l-m-t)/2}, t of the parity of l - m */
  double A = 0.0, Ax = 0.0, Ay = 0.0, Az = 0.0;
  for (int t = 0; t <= l - m; ++t) {
    if ((l - m - t) % 2) continue;
    int e = (l - m - t) / 2;
    double zt = pow(z, t), re = pow(rho, e);
    A += p[t] * zt * re;
    if (e > 0) {
      double dre = e * pow(rho, e - 1);
      Ax += p[t] * zt * dre * 2.0 * x;
      Ay += p[t] * zt * dre * 2.0 * y;
      Az += p[t] * zt * dre * 2.0 * z;
    }
    if (t > 0) Az += p[t] * t * pow(z, t - 1) * re;
  }
  /* C_m + i S_m = (x + i y)^m by repeated multiplication */
  double C = 1.0, S = 0.0, Cm1 = 0.0, Sm1 = 0.0;
  for (int q = 0; q < m; ++q) {
    Cm1 = C;
    Sm1 = S;
    double nc = C * x - S * y, ns = C * y + S * x;
    C = nc;
    S = ns;
  }
  double P, Px, Py;
  if (sc == 0) {
    P = C;
    Px = m * Cm1;
    Py = -m * Sm1;
  } else {
    P = S;
    Px = m * Sm1;
    Py = m * Cm1;
  }
  *val = A * P;
  grad[0] = Ax * P + A * Px;
  grad[1] = Ay * P + A * Py;
  grad[2] = Az * P;
}

/* degree l of polynomial index k: k in [l^2 - 1, (l+1)^2 - 2] */
static int degree_of(int k) {
  int l = 1;
  while ((l + 1) * (l + 1) - 2 < k) ++l;
  return l;
}

/* b_k(d) / r^l and its gradient with respect to d, for k < nb(lmax).
 * For l <= 4 the polynomials are those printed with eq. (S_nk); higher l
 * use the solid harmonics above, ordered m = 0, then (cos, sin) for m = 1..l. */
void ora_angular_poly(int lmax, const double *d, double *bh, double *gbh) {
  double b[ORA_NB_MAX], g[3 * ORA_NB_MAX];
  poly_l4(d, b, g);
  for (int l = 5; l <= lmax; ++l) {
    int k = l * l - 1;
    solid_harmonic(l, 0, 0, d, &b[k], &g[3 * k]);
    ++k;
    for (int m = 1; m <= l; ++m) {
      solid_harmonic(l, m, 0, d, &b[k], &g[3 * k]);
      ++k;
      solid_harmonic(l, m, 1, d, &b[k], &g[3 * k]);
      ++k;
    }
  }
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double r = sqrt(r2);
  int nb = n_poly(lmax);
  for (int k = 0; k < nb; ++k) {
    int l = degree_of(k);
    double rl = pow(r, l);
    bh[k] = b[k] / rl;
    for (int c = 0; c < 3; ++c)
      gbh[3 * k + c] = g[3 * k + c] / rl - l * b[k] * d[c] / (rl * r2);
  }
}

/* C^3b (printed with the explicit q_{n1}..q_{n4}), extended to l = 5, 6 by the
 * addition theorem; C^4b and C^5b as printed with q_{n222} and q_{n1111}. */
void ora_coefficients(int lmax, double *C3, double *C4, double *C5) {
  const double pi = M_PI;
  double c3[24] = {
      0.25 * 3.0 / pi,          2 * 0.25 * 3.0 / (2 * pi),   2 * 0.25 * 3.0 / (2 * pi),
      5.0 / (16 * pi),          2 * 0.25 * 15.0 / (2 * pi),  2 * 0.25 * 15.0 / (2 * pi),
      2 * 15.0 / (16 * 2 * pi), 2 * 15.0 / (16 * 2 * pi),    7.0 / (16 * pi),
      2 * 21.0 / (64 * pi),     2 * 21.0 / (64 * pi),        2 * 105.0 / (16 * 2 * pi),
      2 * 105.0 / (16 * 2 * pi), 2 * 35.0 / (64 * pi),       2 * 35.0 / (64 * pi),
      9.0 / (256 * pi),         2 * 9.0 * 5.0 / (64 * pi),   2 * 9.0 * 5.0 / (64 * pi),
      2 * 9.0 * 5.0 / (64 * 2 * pi), 2 * 9.0 * 5.0 / (64 * 2 * pi), 2 * 9.0 * 35.0 / (64 * pi),
      2 * 9.0 * 35.0 / (64 * pi), 2 * 9.0 * 35.0 / (256 * 2 * pi), 2 * 9.0 * 35.0 / (256 * 2 * pi)};
  int nb = n_poly(lmax);
  for (int k = 0; k < nb && k < 24; ++k) C3[k] = c3[k];
  for (int l = 5; l <= lmax; ++l) {
    int k = l * l - 1;
    C3[k++] = (2 * l + 1) / (4 * pi);
    for (int m = 1; m <= l; ++m) {
      double c = (2 * l + 1) / (4 * pi) * 2.0 * factorial(l - m) / factorial(l + m);
      C3[k++] = c;
      C3[k++] = c;
    }
  }
  double y20 = 0.25 * sqrt(5.0 / pi);
  double y21 = 0.5 * sqrt(15.0 / (2 * pi));
  double y22 = 0.25 * sqrt(15.0 / (2 * pi));
  C4[0] = -sqrt(2.0 / 35.0) * y20 * y20 * y20;
  C4[1] = -6.0 * sqrt(1.0 / 70.0) * y20 * y21 * y21;
  C4[2] = 6.0 * sqrt(2.0 / 35.0) * y20 * y22 * y22;
  C4[3] = 6.0 * sqrt(3.0 / 35.0) * y21 * y21 * y22;
  C4[4] = -12.0 * sqrt(3.0 / 35.0) * y21 * y21 * y22;
  C5[0] = 21.0 / (80.0 * pi * pi);
  C5[1] = 21.0 / (40.0 * pi * pi);
  C5[2] = 21.0 / (80.0 * pi * pi);
}

/* ===================================================================== */
/* parameter blob                                                         */
/* ===================================================================== */

typedef struct {
  int nd, nR, nA, KR, KA, L, nb, T, nneu;
  const double *p;
  int64_t cR, cA, b1;
  double C3[ORA_NB_MAX], C4[5], C5[3];
} ora_model;

static void model_init(ora_model *M, const ora_hparams *h, const double *p) {
  M->nd = ora_num_descriptors(h);
  M->nR = n_rad(h);
  M->nA = n_ang(h);
  M->KR = k_rad(h);
  M->KA = k_ang(h);
  M->L = h->l_max_3b;
  M->nb = n_poly(h->l_max_3b);
  M->T = h->n_types;
  M->nneu = h->n_neurons;
  M->p = p;
  int64_t nets = h->nn_per_type ? h->n_types : 1;
  M->b1 = nets * (int64_t)(M->nd + 2) * M->nneu;
  M->cR = M->b1 + 1;
  M->cA = M->cR + (int64_t)M->T * M->T * M->nR * M->KR;
  ora_coefficients(M->L, M->C3, M->C4, M->C5);
}

static const double *coef_R(const ora_model *M, int ti, int tj) {
  return M->p + M->cR + (int64_t)(ti * M->T + tj) * M->nR * M->KR;
}
static const double *coef_A(const ora_model *M, int ti, int tj) {
  return M->p + M->cA + (int64_t)(ti * M->T + tj) * M->nA * M->KA;
}

/* descriptor slots (reading Z4) */
static int slot3(const ora_model *M, int n, int l) { return M->nR + (l - 1) * M->nA + n; }
static int slot4(const ora_model *M, int n) { return M->nR + M->L * M->nA + n; }
static int slot5(const ora_model *M, const ora_hparams *h, int n) {
  return M->nR + (M->L + use4b(h)) * M->nA + n;
}

/* ===================================================================== */
/* site quantities of one atom                                            */
/* ===================================================================== */

/* Descriptor q^i (eqs. qin, S_nk and the explicit q_{nl}, q_{n222}, q_{n1111})
 * and the sums S_{n,k} it is built from. */
static void site_descriptor(const ora_hparams *h, const ora_model *M, int ti,
                            const int32_t *types, const ora_list *R,
                            const ora_list *A, double *q, double *S) {
  double g[64], dg[64];
  for (int v = 0; v < M->nd; ++v) q[v] = 0.0;
  for (int m = 0; m < R->count; ++m) {
    const ora_pair *pr = &R->p[m];
    radial_functions(coef_R(M, ti, types[pr->j]), M->nR, M->KR, h->rc_radial, pr->r, g, dg);
    for (int n = 0; n < M->nR; ++n) q[n] += g[n];
  }
  for (int v = 0; v < M->nA * M->nb; ++v) S[v] = 0.0;
  for (int m = 0; m < A->count; ++m) {
    const ora_pair *pr = &A->p[m];
    double bh[ORA_NB_MAX], gbh[3 * ORA_NB_MAX];
    radial_functions(coef_A(M, ti, types[pr->j]), M->nA, M->KA, h->rc_angular, pr->r, g, dg);
    ora_angular_poly(M->L, pr->d, bh, gbh);
    for (int n = 0; n < M->nA; ++n)
      for (int k = 0; k < M->nb; ++k) S[n * M->nb + k] += g[n] * bh[k];
  }
  for (int n = 0; n < M->nA; ++n) {
    const double *s = S + n * M->nb;
    for (int l = 1; l <= M->L; ++l) {
      double acc = 0.0;
      for (int k = l * l - 1; k <= (l + 1) * (l + 1) - 2; ++k) acc += M->C3[k] * s[k] * s[k];
      q[slot3(M, n, l)] = acc;
    }
    if (use4b(h)) {
      const double *C = M->C4;
      q[slot4(M, n)] = C[0] * s[3] * s[3] * s[3] + C[1] * s[3] * (s[4] * s[4] + s[5] * s[5]) +
                       C[2] * s[3] * (s[6] * s[6] + s[7] * s[7]) +
                       C[3] * s[6] * (s[5] * s[5] - s[4] * s[4]) + C[4] * s[4] * s[5] * s[7];
    }
    if (use5b(h)) {
      const double *C = M->C5;
      double s12 = s[1] * s[1] + s[2] * s[2];
      q[slot5(M, h, n)] = C[0] * s[0] * s[0] * s[0] * s[0] + C[1] * s[0] * s[0] * s12 + C[2] * s12 * s12;
    }
  }
}

/* Eq. (Ui): U = sum_mu w1_mu tanh(sum_nu w0_{mu nu} q_nu - b0_mu) - b1, and
 * dU/dq_nu = sum_mu w1_mu (1 - h_mu^2) w0_{mu nu}. */
double ora_ann(const ora_hparams *h, const double *params, int type, const double *q,
               double *Fp) {
  ora_model M;
  model_init(&M, h, params);
  int net = h->nn_per_type ? type : 0;
  const double *w0 = params + (int64_t)net * (M.nd + 2) * M.nneu;
  const double *b0 = w0 + (int64_t)M.nneu * M.nd;
  const double *w1 = b0 + M.nneu;
  double U = 0.0;
  for (int v = 0; v < M.nd; ++v) Fp[v] = 0.0;
  for (int mu = 0; mu < M.nneu; ++mu) {
    double a = 0.0;
    for (int v = 0; v < M.nd; ++v) a += w0[mu * M.nd + v] * q[v];
    double hmu = tanh(a - b0[mu]);
    U += w1[mu] * hmu;
    for (int v = 0; v < M.nd; ++v) Fp[v] += w1[mu] * (1.0 - hmu * hmu) * w0[mu * M.nd + v];
  }
  return U - params[M.b1];
}

/* Latent-space vector of one site (Sec. IV): the N_neu products of the
 * hidden-layer states h_mu of eq. (Ui) and their output weights w1_mu, so
 * that sum_mu lat_mu - b1 = U. */
void ora_latent(const ora_hparams *h, const double *params, int type, const double *q,
                double *lat) {
  ora_model M;
  model_init(&M, h, params);
  int net = h->nn_per_type ? type : 0;
  const double *w0 = params + (int64_t)net * (M.nd + 2) * M.nneu;
  const double *b0 = w0 + (int64_t)M.nneu * M.nd;
  const double *w1 = b0 + M.nneu;
  for (int mu = 0; mu < M.nneu; ++mu) {
    double a = 0.0;
    for (int v = 0; v < M.nd; ++v) a += w0[mu * M.nd + v] * q[v];
    lat[mu] = w1[mu] * tanh(a - b0[mu]);
  }
}

/* D_{n,k} = dU/dS_{n,k} through q_{nl}, q_{n222} and q_{n1111}. */
static void site_dUdS(const ora_hparams *h, const ora_model *M, const double *S,
                      const double *Fp, double *D) {
  for (int n = 0; n < M->nA; ++n) {
    const double *s = S + n * M->nb;
    double *dd = D + n * M->nb;
    for (int k = 0; k < M->nb; ++k) {
      int l = degree_of(k);
      dd[k] = Fp[slot3(M, n, l)] * 2.0 * M->C3[k] * s[k];
    }
    if (use4b(h)) {
      const double *C = M->C4;
      double f = Fp[slot4(M, n)];
      dd[3] += f * (3.0 * C[0] * s[3] * s[3] + C[1] * (s[4] * s[4] + s[5] * s[5]) +
                    C[2] * (s[6] * s[6] + s[7] * s[7]));
      dd[4] += f * (2.0 * C[1] * s[3] * s[4] - 2.0 * C[3] * s[6] * s[4] + C[4] * s[5] * s[7]);
      dd[5] += f * (2.0 * C[1] * s[3] * s[5] + 2.0 * C[3] * s[6] * s[5] + C[4] * s[4] * s[7]);
      dd[6] += f * (2.0 * C[2] * s[3] * s[6] + C[3] * (s[5] * s[5] - s[4] * s[4]));
      dd[7] += f * (2.0 * C[2] * s[3] * s[7] + C[4] * s[4] * s[5]);
    }
    if (use5b(h)) {
      const double *C = M->C5;
      double f = Fp[slot5(M, h, n)];
      double s12 = s[1] * s[1] + s[2] * s[2];
      dd[0] += f * (4.0 * C[0] * s[0] * s[0] * s[0] + 2.0 * C[1] * s[0] * s12);
      dd[1] += f * (2.0 * C[1] * s[0] * s[0] * s[1] + 4.0 * C[2] * s12 * s[1]);
      dd[2] += f * (2.0 * C[1] * s[0] * s[0] * s[2] + 4.0 * C[2] * s12 * s[2]);
    }
  }
}

/* Partial forces dU_i/dr_ij (eq. partial_force) for every pair of atom i. */
static void site_partial_forces(const ora_hparams *h, const ora_model *M, int ti,
                                const int32_t *types, const ora_list *R,
                                const ora_list *A, const double *Fp,
                                const double *D, double *PR, double *PA) {
  double g[64], dg[64];
  for (int m = 0; m < R->count; ++m) {
    const ora_pair *pr = &R->p[m];
    radial_functions(coef_R(M, ti, types[pr->j]), M->nR, M->KR, h->rc_radial, pr->r, g, dg);
    double s = 0.0;
    for (int n = 0; n < M->nR; ++n) s += Fp[n] * dg[n];
    for (int c = 0; c < 3; ++c) PR[3 * m + c] = s * pr->d[c] / pr->r;
  }
  for (int m = 0; m < A->count; ++m) {
    const ora_pair *pr = &A->p[m];
    double bh[ORA_NB_MAX], gbh[3 * ORA_NB_MAX];
    radial_functions(coef_A(M, ti, types[pr->j]), M->nA, M->KA, h->rc_angular, pr->r, g, dg);
    ora_angular_poly(M->L, pr->d, bh, gbh);
    double P[3] = {0.0, 0.0, 0.0};
    for (int n = 0; n < M->nA; ++n)
      for (int k = 0; k < M->nb; ++k) {
        double Dnk = D[n * M->nb + k];
        for (int c = 0; c < 3; ++c)
          P[c] += Dnk * (dg[n] * (pr->d[c] / pr->r) * bh[k] + g[n] * gbh[3 * k + c]);
      }
    for (int c = 0; c < 3; ++c) PA[3 * m + c] = P[c];
  }
}

/* ===================================================================== */
/* whole-system evaluation (eqs. F_ij, F_i, virial)                       */
/* ===================================================================== */

typedef struct {
  ora_list R, A;
  double *PR, *PA;
  double U;
} ora_site;

static int geometry(const double *box, double *Hi, double *w) {
  double det = box[0] * (box[4] * box[8] - box[5] * box[7]) -
               box[1] * (box[3] * box[8] - box[5] * box[6]) +
               box[2] * (box[3] * box[7] - box[4] * box[6]);
  if (!(det > 0.0) || !isfinite(det)) return ORA_EARG;
  box_inverse(box, Hi);
  face_widths(box, w);
  return ORA_OK;
}

/* Energy U[N], forces F[3][N] and per-atom virials W[9][N] (row-major 3x3 per
 * atom, W_i = sum_j r_ij (x) dU_j/dr_ji) of one periodic (or partly periodic)
 * structure.  Any output pointer may be NULL; q[N][N_des] is optional too.
 * Phase 1 computes every atom's descriptor, network and partial forces
 * (parallel over atoms); phase 2 adds the partial forces into F and W in a
 * fixed serial order. */
static int evaluate_core(const ora_hparams *h, const double *params, int64_t N,
                         const double *pos, const int32_t *types, const double *box,
                         const int32_t *pbc, double *U, double *F, double *W, double *q_out,
                         const double *vel, double *J2) {
  if (check_hp(h) || N < 1) return ORA_EARG;
  for (int64_t i = 0; i < N; ++i)
    if (types[i] < 0 || types[i] >= h->n_types) return ORA_EARG;
  double Hi[9], w[3];
  if (geometry(box, Hi, w)) return ORA_EARG;
  ora_model M;
  model_init(&M, h, params);
  ora_site *sites = (ora_site *)calloc((size_t)N, sizeof(ora_site));
  if (!sites) return ORA_EMEM;
  int err = ORA_OK;
#pragma omp parallel
  {
    double *q = (double *)malloc(sizeof(double) * M.nd);
    double *Fp = (double *)malloc(sizeof(double) * M.nd);
    double *S = (double *)malloc(sizeof(double) * M.nA * M.nb);
    double *D = (double *)malloc(sizeof(double) * M.nA * M.nb);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < N; ++i) {
      ora_site *st = &sites[i];
      if (environment(pos, N, i, box, Hi, w, pbc, h->rc_radial, &st->R) ||
          environment(pos, N, i, box, Hi, w, pbc, h->rc_angular, &st->A)) {
        err = ORA_EMEM;
        continue;
      }
      site_descriptor(h, &M, types[i], types, &st->R, &st->A, q, S);
      if (q_out)
        for (int v = 0; v < M.nd; ++v) q_out[i * M.nd + v] = q[v];
      st->U = ora_ann(h, params, types[i], q, Fp);
      site_dUdS(h, &M, S, Fp, D);
      st->PR = (double *)malloc(sizeof(double) * 3 * (st->R.count + 1));
      st->PA = (double *)malloc(sizeof(double) * 3 * (st->A.count + 1));
      site_partial_forces(h, &M, types[i], types, &st->R, &st->A, Fp, D, st->PR, st->PA);
    }
    free(q);
    free(Fp);
    free(S);
    free(D);
  }
  if (err == ORA_OK) {
    if (F) memset(F, 0, sizeof(double) * 3 * N);
    if (W) memset(W, 0, sizeof(double) * 9 * N);
    if (J2) J2[0] = J2[1] = J2[2] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      ora_site *st = &sites[i];
      if (U) U[i] = st->U;
      for (int pass = 0; pass < 2; ++pass) {
        const ora_list *L = pass ? &st->A : &st->R;
        const double *P = pass ? st->PA : st->PR;
        for (int m = 0; m < L->count; ++m) {
          int64_t j = L->p[m].j;
          const double *d = L->p[m].d;
          for (int c = 0; c < 3; ++c) {
            if (F) {
              F[c * N + i] += P[3 * m + c];
              F[c * N + j] -= P[3 * m + c];
            }
          }
          if (W)
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) W[(a * 3 + b) * N + j] += (-d[a]) * P[3 * m + b];
          if (J2) {
            /* eq. J-2: J = -sum_i sum_j r_ij (dU_i/dr_ij . v_j) */
            double pv = 0.0;
            for (int b = 0; b < 3; ++b) pv += P[3 * m + b] * vel[b * N + j];
            for (int a = 0; a < 3; ++a) J2[a] -= d[a] * pv;
          }
        }
      }
    }
  }
  for (int64_t i = 0; i < N; ++i) {
    list_free(&sites[i].R);
    list_free(&sites[i].A);
    free(sites[i].PR);
    free(sites[i].PA);
  }
  free(sites);
  return err;
}

int ora_evaluate(const ora_hparams *h, const double *params, int64_t N, const double *pos,
                 const int32_t *types, const double *box, const int32_t *pbc, double *U,
                 double *F, double *W, double *q_out) {
  return evaluate_core(h, params, N, pos, types, box, pbc, U, F, W, q_out, NULL, NULL);
}

/* Heat current (Sec. II.E).  Per-atom J_i = W_i . v_i (eq. Ji), i.e.
 * J_i,a = sum_b W_i,ab v_i,b with the per-atom virial of eq. virial, written
 * to Jatom[3][N]; J1[3] = sum_i J_i (eq. J-1).  J2[3] is the same total taken
 * the other way, from each atom's own partial forces and its neighbours'
 * velocities (eq. J-2).  vel is [3][N]; any output may be NULL. */
int ora_heat_current(const ora_hparams *h, const double *params, int64_t N, const double *pos,
                     const double *vel, const int32_t *types, const double *box,
                     const int32_t *pbc, double *Jatom, double *J1, double *J2) {
  if (N < 1 || !vel) return ORA_EARG;
  double *W = (double *)malloc(sizeof(double) * 9 * N);
  if (!W) return ORA_EMEM;
  int err = evaluate_core(h, params, N, pos, types, box, pbc, NULL, NULL, W, NULL, vel, J2);
  if (err == ORA_OK) {
    if (J1) J1[0] = J1[1] = J1[2] = 0.0;
    for (int64_t i = 0; i < N; ++i)
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += W[(a * 3 + b) * N + i] * vel[b * N + i];
        if (Jatom) Jatom[a * N + i] = s;
        if (J1) J1[a] += s;
      }
  }
  free(W);
  return err;
}

/* Descriptors only, q[N][N_des]. */
int ora_descriptors(const ora_hparams *h, const double *params, int64_t N,
                    const double *pos, const int32_t *types, const double *box,
                    const int32_t *pbc, double *q_out) {
  if (check_hp(h) || N < 1) return ORA_EARG;
  double Hi[9], w[3];
  if (geometry(box, Hi, w)) return ORA_EARG;
  ora_model M;
  model_init(&M, h, params);
  int err = ORA_OK;
#pragma omp parallel
  {
    double *S = (double *)malloc(sizeof(double) * M.nA * M.nb);
    ora_list R = {0, 0, NULL}, A = {0, 0, NULL};
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < N; ++i) {
      if (environment(pos, N, i, box, Hi, w, pbc, h->rc_radial, &R) ||
          environment(pos, N, i, box, Hi, w, pbc, h->rc_angular, &A)) {
        err = ORA_EMEM;
        continue;
      }
      site_descriptor(h, &M, types[i], types, &R, &A, q_out + i * M.nd, S);
    }
    list_free(&R);
    list_free(&A);
    free(S);
  }
  return err;
}

/* ===================================================================== */
/* sampled evaluation for very large structures                           */
/* ===================================================================== */

/* Candidates around atom i within radius: (k, image) with canonical d. */
static int halo(const double *pos, int64_t N, int64_t i, const double *H, const double *Hi,
                const double *w, const int32_t *pbc, double radius, ora_list *out) {
  return environment(pos, N, i, H, Hi, w, pbc, radius, out);
}

/* Environment of image (j, nj) of a neighbour of i, taken from i's halo: every
 * (k, m) of the halo with |d|^2 < rc^2 where d is the canonical displacement
 * from j to k with image m - nj.  Rows come out j-then-image sorted as in
 * environment() after sorting; order does not matter for the sums. */
static int env_from_halo(const double *pos, int64_t N, int64_t i, int64_t j,
                         const int32_t *nj, const ora_list *HL, const double *H,
                         double rc, ora_list *out) {
  out->count = 0;
  double rc2 = rc * rc;
  /* the halo holds every image except (i, 0) itself; add it back */
  for (int e = -1; e < HL->count; ++e) {
    int32_t k, m[3];
    if (e < 0) {
      k = (int32_t)i;
      m[0] = m[1] = m[2] = 0;
    } else {
      k = HL->p[e].j;
      m[0] = HL->p[e].n[0];
      m[1] = HL->p[e].n[1];
      m[2] = HL->p[e].n[2];
    }
    int32_t rel[3] = {m[0] - nj[0], m[1] - nj[1], m[2] - nj[2]};
    if (k == j && rel[0] == 0 && rel[1] == 0 && rel[2] == 0) continue;
    double d[3];
    double r2 = displacement(pos, N, j, k, rel, H, d);
    if (r2 < rc2)
      if (list_push(out, k, rel, d, r2)) return ORA_EMEM;
  }
  return ORA_OK;
}

/* U, F, W of the atoms idx[0..n_idx-1] only, computed from their own and their
 * neighbours' environments (found within a halo of 2 r_c^R + 0.5 A). */
int ora_evaluate_atoms(const ora_hparams *h, const double *params, int64_t N,
                       const double *pos, const int32_t *types, const double *box,
                       const int32_t *pbc, int64_t n_idx, const int64_t *idx, double *U,
                       double *F, double *W) {
  if (check_hp(h) || N < 1) return ORA_EARG;
  double Hi[9], w[3];
  if (geometry(box, Hi, w)) return ORA_EARG;
  ora_model M;
  model_init(&M, h, params);
  int err = ORA_OK;
  for (int64_t s = 0; s < n_idx && err == ORA_OK; ++s) {
    int64_t i = idx[s];
    ora_list HL = {0, 0, NULL}, Ri = {0, 0, NULL}, Ai = {0, 0, NULL};
    if (halo(pos, N, i, box, Hi, w, pbc, 2.0 * h->rc_radial + 0.5, &HL)) {
      err = ORA_EMEM;
      break;
    }
    int32_t zero[3] = {0, 0, 0};
    env_from_halo(pos, N, i, i, zero, &HL, box, h->rc_radial, &Ri);
    env_from_halo(pos, N, i, i, zero, &HL, box, h->rc_angular, &Ai);
    double *q = (double *)malloc(sizeof(double) * M.nd);
    double *Fp = (double *)malloc(sizeof(double) * M.nd);
    double *S = (double *)malloc(sizeof(double) * M.nA * M.nb);
    double *D = (double *)malloc(sizeof(double) * M.nA * M.nb);
    double *PRi = (double *)malloc(sizeof(double) * 3 * (Ri.count + 1));
    double *PAi = (double *)malloc(sizeof(double) * 3 * (Ai.count + 1));
    site_descriptor(h, &M, types[i], types, &Ri, &Ai, q, S);
    double Ui = ora_ann(h, params, types[i], q, Fp);
    site_dUdS(h, &M, S, Fp, D);
    site_partial_forces(h, &M, types[i], types, &Ri, &Ai, Fp, D, PRi, PAi);
    double Fi[3] = {0, 0, 0}, Wi[9] = {0};
    for (int c = 0; c < 3; ++c) {
      for (int m = 0; m < Ri.count; ++m) Fi[c] += PRi[3 * m + c];
      for (int m = 0; m < Ai.count; ++m) Fi[c] += PAi[3 * m + c];
    }
    /* reverse partial forces dU_j/dr_ji from each neighbour image (j, n) */
    int nR = Ri.count;
    double *acc = (double *)calloc((size_t)nR * 12, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < nR; ++m) {
      const ora_pair *pj = &Ri.p[m];
      ora_list Rj = {0, 0, NULL}, Aj = {0, 0, NULL};
      env_from_halo(pos, N, i, pj->j, pj->n, &HL, box, h->rc_radial, &Rj);
      env_from_halo(pos, N, i, pj->j, pj->n, &HL, box, h->rc_angular, &Aj);
      double *qj = (double *)malloc(sizeof(double) * M.nd);
      double *Fpj = (double *)malloc(sizeof(double) * M.nd);
      double *Sj = (double *)malloc(sizeof(double) * M.nA * M.nb);
      double *Dj = (double *)malloc(sizeof(double) * M.nA * M.nb);
      double *PRj = (double *)malloc(sizeof(double) * 3 * (Rj.count + 1));
      double *PAj = (double *)malloc(sizeof(double) * 3 * (Aj.count + 1));
      int tj = types[pj->j];
      site_descriptor(h, &M, tj, types, &Rj, &Aj, qj, Sj);
      ora_ann(h, params, tj, qj, Fpj);
      site_dUdS(h, &M, Sj, Fpj, Dj);
      site_partial_forces(h, &M, tj, types, &Rj, &Aj, Fpj, Dj, PRj, PAj);
      double P[3] = {0, 0, 0};
      int32_t back[3] = {-pj->n[0], -pj->n[1], -pj->n[2]};
      for (int pass = 0; pass < 2; ++pass) {
        const ora_list *L = pass ? &Aj : &Rj;
        const double *PP = pass ? PAj : PRj;
        for (int e = 0; e < L->count; ++e)
          if (L->p[e].j == i && L->p[e].n[0] == back[0] && L->p[e].n[1] == back[1] &&
              L->p[e].n[2] == back[2])
            for (int c = 0; c < 3; ++c) P[c] += PP[3 * e + c];
      }
      for (int c = 0; c < 3; ++c) acc[12 * m + c] = P[c];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[12 * m + 3 + a * 3 + b] = pj->d[a] * P[b];
      list_free(&Rj);
      list_free(&Aj);
      free(qj);
      free(Fpj);
      free(Sj);
      free(Dj);
      free(PRj);
      free(PAj);
    }
    for (int m = 0; m < nR; ++m) {
      for (int c = 0; c < 3; ++c) Fi[c] -= acc[12 * m + c];
      for (int v = 0; v < 9; ++v) Wi[v] += acc[12 * m + 3 + v];
    }
    if (U) U[s] = Ui;
    if (F)
      for (int c = 0; c < 3; ++c) F[3 * s + c] = Fi[c];
    if (W)
      for (int v = 0; v < 9; ++v) W[9 * s + v] = Wi[v];
    free(acc);
    free(q);
    free(Fp);
    free(S);
    free(D);
    free(PRi);
    free(PAi);
    list_free(&HL);
    list_free(&Ri);
    list_free(&Ai);
  }
  return err;
}

/* ===================================================================== */
/* velocity-Verlet NVE                                                    */
/* ===================================================================== */

/* 1 amu (A/fs)^2 in eV, from the CODATA 2018 amu and elementary charge */
static double amu_a2_fs2_ev(void) { return 1.66053906660e-27 * 1e10 / 1.602176634e-19; }
static const double ORA_KB = 8.617333262e-5; /* eV/K */

/* NVE velocity Verlet: v += dt/2 F/m; r += dt v; F(r); v += dt/2 F/m.
 * Every thermo_every steps a row [step, E_pot, E_kin, T, W_xx .. W_zz]
 * (13 numbers, totals in eV, T with 3N - 3 degrees of freedom) is written.
 * Positions are never wrapped: the pair search enumerates images. */
int ora_md_nve(const ora_hparams *h, const double *params, int64_t N, double *pos,
               double *vel, const int32_t *types, const double *mass_per_type,
               const double *box, const int32_t *pbc, double dt, int64_t n_steps,
               int64_t thermo_every, double *thermo) {
  double conv = amu_a2_fs2_ev();
  double *F = (double *)malloc(sizeof(double) * 3 * N);
  double *U = (double *)malloc(sizeof(double) * N);
  double *W = (double *)malloc(sizeof(double) * 9 * N);
  if (!F || !U || !W) return ORA_EMEM;
  int err = ora_evaluate(h, params, N, pos, types, box, pbc, U, F, W, NULL);
  int64_t row = 0;
  for (int64_t step = 1; step <= n_steps && err == ORA_OK; ++step) {
    for (int64_t i = 0; i < N; ++i) {
      double a = 1.0 / (mass_per_type[types[i]] * conv);
      for (int c = 0; c < 3; ++c) {
        vel[c * N + i] += 0.5 * dt * F[c * N + i] * a;
        pos[c * N + i] += dt * vel[c * N + i];
      }
    }
    err = ora_evaluate(h, params, N, pos, types, box, pbc, U, F, W, NULL);
    if (err) break;
    double ek = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      double a = 1.0 / (mass_per_type[types[i]] * conv);
      for (int c = 0; c < 3; ++c) vel[c * N + i] += 0.5 * dt * F[c * N + i] * a;
    }
    if (thermo_every > 0 && step % thermo_every == 0) {
      double ep = 0.0, wt[9] = {0};
      for (int64_t i = 0; i < N; ++i) {
        ep += U[i];
        double m = mass_per_type[types[i]];
        for (int c = 0; c < 3; ++c) ek += 0.5 * m * vel[c * N + i] * vel[c * N + i];
        for (int v = 0; v < 9; ++v) wt[v] += W[v * N + i];
      }
      ek *= conv;
      double *t = thermo + 13 * row++;
      t[0] = (double)step;
      t[1] = ep;
      t[2] = ek;
      t[3] = N > 1 ? 2.0 * ek / ((3.0 * N - 3.0) * ORA_KB) : 0.0;
      for (int v = 0; v < 9; ++v) t[4 + v] = wt[v];
    }
  }
  free(F);
  free(U);
  free(W);
  return err;
}

/* ===================================================================== */
/* counter-based random numbers: Philox4x32-10                            */
/* ===================================================================== */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): each round multiplies counter words
 * 0 and 2 by the two round constants, takes high and low halves and mixes
 * them with words 1 and 3 and the key; the key is bumped by the two Weyl
 * constants between rounds. */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Four standard normal numbers from counter (index, step, stream, 0) under
 * the 64-bit seed: the four Philox words as uniforms (x + 1/2) 2^-32 in
 * (0, 1), turned into normals pairwise by the Box-Muller transform. */
void ora_normal4(uint64_t seed, uint32_t index, uint32_t step, uint32_t stream, double z[4]) {
  const uint32_t ctr[4] = {index, step, stream, 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  ora_philox4x32_10(ctr, key, w);
  for (int p = 0; p < 2; ++p) {
    double u1 = ((double)w[2 * p] + 0.5) * (1.0 / 4294967296.0);
    double u2 = ((double)w[2 * p + 1] + 0.5) * (1.0 / 4294967296.0);
    double rad = sqrt(-2.0 * log(u1));
    z[2 * p] = rad * cos(2.0 * M_PI * u2);
    z[2 * p + 1] = rad * sin(2.0 * M_PI * u2);
  }
}

/* ===================================================================== */
/* thermostats and barostats (the NVT and NPT ensembles of Sec. II.F)     */
/* ===================================================================== */

/* The paper lists the ensembles GPUMD offers and cites their methods without
 * restating them; each follows its publication:
 *   1 Berendsen thermostat (Berendsen et al. 1984): after a velocity-Verlet
 *     step, v *= sqrt(1 + dt/tau (T0/T - 1)).
 *   2 Bussi-Donadio-Parrinello stochastic velocity rescaling (2007): the
 *     kinetic energy K is replaced by
 *     K + (1-c)(K0 (R1^2 + S)/Nf - K) + 2 R1 sqrt(c (1-c) K0 K / Nf),
 *     c = exp(-dt/tau), K0 = Nf kB T0 / 2, R1 normal, S a sum of Nf - 1
 *     squared normals; v *= sqrt(K'/K).
 *   3 Langevin dynamics in the Bussi-Parrinello (2007) splitting: a half-step
 *     Ornstein-Uhlenbeck update v = c1 v + sqrt((1 - c1^2) kB T0 / m) xi,
 *     c1 = exp(-dt / (2 tau)), before and after the velocity-Verlet step.
 *   4 Nose-Hoover chain (Martyna, Klein, Tuckerman 1992) of length M with
 *     masses Q1 = Nf kB T0 tau^2, Qk = kB T0 tau^2, integrated by the Trotter
 *     splitting chain(dt/2), velocity Verlet, chain(dt/2) (Martyna et al.
 *     1996, one sub-step).
 *   5 Berendsen barostat (isotropic) with the Berendsen thermostat: after
 *     the thermostat, P = (2K + tr W)/(3V); box and positions scale by
 *     mu = (1 - beta dt/tau_p (P0 - P))^(1/3).
 *   6 Stochastic cell rescaling (Bernetti, Bussi 2020, isotropic) with the
 *     BDP thermostat: d eps = -(beta/tau_p)(P0 - P - kB T0/V) dt
 *     + sqrt(2 kB T0 beta dt / (V tau_p)) R, eps = ln V; positions and box
 *     scale by exp(d eps / 3), velocities by exp(-d eps / 3).
 * Nf = 3N - 3.  Random numbers come from ora_normal4 with counter
 * (index, step, stream): Langevin streams 1 and 2 (the two half steps,
 * index = atom), BDP stream 3 (R1 = the first normal of index 0) and 4 (the
 * Nf - 1 normals of S, four per index in order), SCR stream 5 (index 0).
 * The step in the counter is state[0] + the step number (1-based) of this
 * call, so consecutive calls continue one stream.
 *
 * state (in/out, 20 doubles): [0] steps done before this call; [1] energy
 * taken out of the system by thermostat and barostat so far (so that
 * K + U (+ P0 V for NPT) + state[1] is the effective energy H~; for the
 * Nose-Hoover chain H~ adds the chain's own energy instead); [2..9] chain
 * positions xi_k; [10..17] chain velocities v_xi_k.
 * Thermo rows of 16: step, E_pot, E_kin, T, W (9), V, P (GPa), H~. */

#define ORA_GPA (160.21766208)  /* 1 eV/A^3 in GPa */

typedef struct {
  int32_t kind;
  double temperature, tau_t;
  int32_t nhc_length;
  double pressure, tau_p, compressibility;
  uint64_t seed;
} ora_ensemble;

static double kinetic(int64_t N, const double *vel, const int32_t *types, const double *mass,
                      double conv) {
  double k = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    double m = mass[types[i]];
    for (int c = 0; c < 3; ++c) k += 0.5 * m * vel[c * N + i] * vel[c * N + i];
  }
  return k * conv;
}

static void scale_vel(int64_t N, double *vel, double s) {
  for (int64_t i = 0; i < 3 * N; ++i) vel[i] *= s;
}

/* Chain half step of length dt/2 (MKT 1992 / Martyna et al. 1996): returns
 * the velocity scale and updates xi, v_xi; K is the current kinetic energy. */
static double nhc_half(int M, double dt, double K, double Nf, double kT, double tau, double *xi,
                       double *vx) {
  double Q[8];
  for (int k = 0; k < M; ++k) Q[k] = (k == 0 ? Nf : 1.0) * kT * tau * tau;
  const double h = 0.5 * dt;
  double G;
#define ORA_G(k) ((k) == 0 ? (2.0 * K - Nf * kT) / Q[0] : (Q[(k)-1] * vx[(k)-1] * vx[(k)-1] - kT) / Q[k])
  G = ORA_G(M - 1);
  vx[M - 1] += 0.5 * h * G;
  for (int k = M - 2; k >= 0; --k) {
    double a = exp(-0.25 * h * vx[k + 1]);
    vx[k] *= a;
    G = ORA_G(k);
    vx[k] += 0.5 * h * G;
    vx[k] *= a;
  }
  double s = exp(-h * vx[0]);
  K *= s * s;
  for (int k = 0; k < M; ++k) xi[k] += h * vx[k];
  for (int k = 0; k < M - 1; ++k) {
    double a = exp(-0.25 * h * vx[k + 1]);
    vx[k] *= a;
    G = ORA_G(k);
    vx[k] += 0.5 * h * G;
    vx[k] *= a;
  }
  G = ORA_G(M - 1);
  vx[M - 1] += 0.5 * h * G;
#undef ORA_G
  return s;
}

/* Box volume from the rows of H. */
static double volume(const double *H) {
  return H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
         H[2] * (H[3] * H[7] - H[4] * H[6]);
}

/* BDP kinetic-energy resampling; returns the new kinetic energy. */
static double bdp_target(double K, double K0, double Nf, double c, uint64_t seed, uint32_t step) {
  double z[4];
  ora_normal4(seed, 0u, step, 3u, z);
  const double R1 = z[0];
  double S = 0.0;
  const int64_t nS = (int64_t)Nf - 1;
  for (int64_t k = 0; k < nS; k += 4) {
    ora_normal4(seed, (uint32_t)(k / 4), step, 4u, z);
    for (int q = 0; q < 4 && k + q < nS; ++q) S += z[q] * z[q];
  }
  return K + (1.0 - c) * (K0 * (R1 * R1 + S) / Nf - K) + 2.0 * R1 * sqrt(c * (1.0 - c) * K0 * K / Nf);
}

int ora_md_ensemble(const ora_hparams *h, const double *params, int64_t N, double *pos,
                    double *vel, const int32_t *types, const double *mass, double *box,
                    const int32_t *pbc, double dt, int64_t n_steps, int64_t thermo_every,
                    double *thermo, const ora_ensemble *ens, double *state) {
  if (ens->kind < 0 || ens->kind > 6 || N < 2) return ORA_EARG;
  const int M = ens->nhc_length;
  if (ens->kind == 4 && (M < 1 || M > 8)) return ORA_EARG;
  double conv = amu_a2_fs2_ev();
  const double Nf = 3.0 * N - 3.0, kT = ORA_KB * ens->temperature;
  const double K0 = 0.5 * Nf * kT;
  double *F = (double *)malloc(sizeof(double) * 3 * N);
  double *U = (double *)malloc(sizeof(double) * N);
  double *W = (double *)malloc(sizeof(double) * 9 * N);
  if (!F || !U || !W) return ORA_EMEM;
  int err = ora_evaluate(h, params, N, pos, types, box, pbc, U, F, W, NULL);
  int64_t row = 0;
  double *xi = state + 2, *vx = state + 10;
  for (int64_t step = 1; step <= n_steps && err == ORA_OK; ++step) {
    const uint32_t rstep = (uint32_t)((int64_t)state[0] + step);
    if (ens->kind == 4) {
      double s = nhc_half(M, dt, kinetic(N, vel, types, mass, conv), Nf, kT, ens->tau_t, xi, vx);
      scale_vel(N, vel, s);
    }
    if (ens->kind == 3) {  /* first Ornstein-Uhlenbeck half step */
      double c1 = exp(-0.5 * dt / ens->tau_t), k_before = kinetic(N, vel, types, mass, conv);
      for (int64_t i = 0; i < N; ++i) {
        double z[4], m = mass[types[i]] * conv;
        ora_normal4(ens->seed, (uint32_t)i, rstep, 1u, z);
        for (int c = 0; c < 3; ++c)
          vel[c * N + i] = c1 * vel[c * N + i] + sqrt((1.0 - c1 * c1) * kT / m) * z[c];
      }
      state[1] += k_before - kinetic(N, vel, types, mass, conv);
    }
    for (int64_t i = 0; i < N; ++i) {
      double a = 1.0 / (mass[types[i]] * conv);
      for (int c = 0; c < 3; ++c) {
        vel[c * N + i] += 0.5 * dt * F[c * N + i] * a;
        pos[c * N + i] += dt * vel[c * N + i];
      }
    }
    err = ora_evaluate(h, params, N, pos, types, box, pbc, U, F, W, NULL);
    if (err) break;
    for (int64_t i = 0; i < N; ++i) {
      double a = 1.0 / (mass[types[i]] * conv);
      for (int c = 0; c < 3; ++c) vel[c * N + i] += 0.5 * dt * F[c * N + i] * a;
    }
    double K = kinetic(N, vel, types, mass, conv);
    if (ens->kind == 3) {  /* second Ornstein-Uhlenbeck half step */
      double c1 = exp(-0.5 * dt / ens->tau_t);
      for (int64_t i = 0; i < N; ++i) {
        double z[4], m = mass[types[i]] * conv;
        ora_normal4(ens->seed, (uint32_t)i, rstep, 2u, z);
        for (int c = 0; c < 3; ++c)
          vel[c * N + i] = c1 * vel[c * N + i] + sqrt((1.0 - c1 * c1) * kT / m) * z[c];
      }
      double Kn = kinetic(N, vel, types, mass, conv);
      state[1] += K - Kn;
      K = Kn;
    } else if (ens->kind == 1 || ens->kind == 5) {  /* Berendsen */
      double T = 2.0 * K / (Nf * ORA_KB);
      double l2 = 1.0 + dt / ens->tau_t * (ens->temperature / T - 1.0);
      if (l2 < 0.0) l2 = 0.0;
      scale_vel(N, vel, sqrt(l2));
      state[1] += K * (1.0 - l2);
      K *= l2;
    } else if (ens->kind == 2 || ens->kind == 6) {  /* BDP */
      double Kn = bdp_target(K, K0, Nf, exp(-dt / ens->tau_t), ens->seed, rstep);
      if (Kn < 0.0) Kn = 0.0;
      scale_vel(N, vel, sqrt(Kn / K));
      state[1] += K - Kn;
      K = Kn;
    } else if (ens->kind == 4) {
      double s = nhc_half(M, dt, K, Nf, kT, ens->tau_t, xi, vx);
      scale_vel(N, vel, s);
      K *= s * s;
    }
    /* pressure of the state at the end of the step (before any box change) */
    double V = volume(box);
    double wtr = 0.0;
    for (int64_t i = 0; i < N; ++i) wtr += W[0 * N + i] + W[4 * N + i] + W[8 * N + i];
    const double P = (2.0 * K + wtr) / (3.0 * V) * ORA_GPA;
    if (thermo_every > 0 && step % thermo_every == 0) {
      double ep = 0.0, wt[9] = {0};
      for (int64_t i = 0; i < N; ++i) {
        ep += U[i];
        for (int v = 0; v < 9; ++v) wt[v] += W[v * N + i];
      }
      double *t = thermo + 16 * row++;
      t[0] = (double)step;
      t[1] = ep;
      t[2] = K;
      t[3] = 2.0 * K / (Nf * ORA_KB);
      for (int v = 0; v < 9; ++v) t[4 + v] = wt[v];
      t[13] = V;
      t[14] = P;
      double Hx = K + ep + state[1];
      if (ens->kind == 4) {
        Hx = K + ep;
        for (int k = 0; k < M; ++k) {
          double Q = (k == 0 ? Nf : 1.0) * kT * ens->tau_t * ens->tau_t;
          Hx += 0.5 * Q * vx[k] * vx[k] + (k == 0 ? Nf : 1.0) * kT * xi[k];
        }
      }
      if (ens->kind >= 5) Hx += ens->pressure / ORA_GPA * V;
      t[15] = Hx;
    }
    /* barostat: scale the box and the positions (and for SCR the velocities);
     * the next step starts from the forces of the unscaled positions */
    if (ens->kind == 5 || ens->kind == 6) {
      double mu;
      if (ens->kind == 5) {
        mu = cbrt(1.0 - ens->compressibility * dt / ens->tau_p * (ens->pressure - P));
      } else {
        double z[4];
        ora_normal4(ens->seed, 0u, rstep, 5u, z);
        double kTV = kT / V * ORA_GPA;
        double deps = -ens->compressibility / ens->tau_p * (ens->pressure - P - kTV) * dt +
                      sqrt(2.0 * kTV * ens->compressibility * dt / ens->tau_p) * z[0];
        mu = exp(deps / 3.0);
        scale_vel(N, vel, 1.0 / mu);
        state[1] += K - K / (mu * mu);
      }
      for (int64_t i = 0; i < 3 * N; ++i) pos[i] *= mu;
      for (int k = 0; k < 9; ++k) box[k] *= mu;
    }
  }
  state[0] += (double)n_steps;
  free(F);
  free(U);
  free(W);
  return err;
}

/* ===================================================================== */
/* threads                                                                */
/* ===================================================================== */

void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int ora_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
