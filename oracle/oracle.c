/*
 * CPU reference for noisy density-matrix circuit simulation.  TEST INFRASTRUCTURE ONLY:
 * it is used by the test-suite, by the smoke check and by the timed CPU baseline, and
 * nothing on the product path links, loads or calls it.  It shares no code with the
 * HIP library.
 *
 * What it computes is the problem statement of Sec. 2.1 (Eq. eq:dmsim, with each
 * transformation generalised to a Kraus channel as in Sec. 3.1):
 *
 *     rho_out = E_m( ... E_1(rho_in) ... ),   E(rho) = sum_i K_i rho K_i^dagger,
 *
 * applied operation by operation, unfused, in IEEE double precision.  K_i acts on the
 * listed target qubits and as the identity elsewhere (Kronecker product with I,
 * Sec. 2.1).  rho is held as an ordinary row-major 2^n x 2^n matrix of interleaved
 * (re, im) doubles: element (r, c) is at rho[2 * (r * 2^n + c)].  This is deliberately
 * NOT the column-stacked vector used by the superoperator method.
 *
 * Basis convention: qubit q is bit q of a row (or column) index.  A j-qubit matrix on
 * qubits (q_0 .. q_{j-1}) is indexed by sum_t b_{q_t} 2^t and stored row-major as
 * M[out * 2^j + in] (interleaved complex).
 *
 * Each Kraus term is applied as the two matrix products it is made of:
 *   T = K rho     (K mixes the 2^j rows that differ only in the target bits),
 *   T = T K^dag   (K^dag mixes the 2^j columns that differ only in the target bits),
 *   acc += T.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXJ 6 /* up to 6-qubit operators: 64 x 64 */

/* Scatter the low bits of a (bit t) to bit position q[t]. */
static uint64_t deposit(uint64_t a, const int* q, int j) {
  uint64_t r = 0;
  for (int t = 0; t < j; ++t)
    if ((a >> t) & 1u) r |= (uint64_t)1 << q[t];
  return r;
}

static int check_targets(int n, int j, const int* q) {
  if (j < 1 || j > MAXJ || j > n) return -1;
  for (int t = 0; t < j; ++t) {
    if (q[t] < 0 || q[t] >= n) return -1;
    for (int u = 0; u < t; ++u)
      if (q[u] == q[t]) return -1;
  }
  return 0;
}

/* T = K * rho restricted to the target row bits; rho and T are dim x dim, interleaved. */
static void left_multiply(int n, const double* rho, double* T, int j, const int* q, const double* K) {
  const uint64_t dim = (uint64_t)1 << n;
  const int D = 1 << j;
  uint64_t tmask = 0;
  for (int t = 0; t < j; ++t) tmask |= (uint64_t)1 << q[t];
  uint64_t off[1 << MAXJ];
  for (int a = 0; a < D; ++a) off[a] = deposit((uint64_t)a, q, j);

#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < (int64_t)dim; ++c) {
    for (uint64_t rbase = 0; rbase < dim; ++rbase) {
      if (rbase & tmask) continue; /* visit each group of rows once, via its base row */
      for (int b = 0; b < D; ++b) {
        double sr = 0.0, si = 0.0;
        for (int a = 0; a < D; ++a) {
          const double kr = K[2 * (b * D + a)], ki = K[2 * (b * D + a) + 1];
          const uint64_t e = ((rbase | off[a]) * dim + (uint64_t)c) * 2;
          const double xr = rho[e], xi = rho[e + 1];
          sr += kr * xr - ki * xi;
          si += kr * xi + ki * xr;
        }
        const uint64_t o = ((rbase | off[b]) * dim + (uint64_t)c) * 2;
        T[o] = sr;
        T[o + 1] = si;
      }
    }
  }
}

/* T = T * K^dagger restricted to the target column bits, in place. */
static void right_multiply_adjoint(int n, double* T, int j, const int* q, const double* K) {
  const uint64_t dim = (uint64_t)1 << n;
  const int D = 1 << j;
  uint64_t tmask = 0;
  for (int t = 0; t < j; ++t) tmask |= (uint64_t)1 << q[t];
  uint64_t off[1 << MAXJ];
  for (int a = 0; a < D; ++a) off[a] = deposit((uint64_t)a, q, j);

#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < (int64_t)dim; ++r) {
    double vr[1 << MAXJ], vi[1 << MAXJ];
    for (uint64_t cbase = 0; cbase < dim; ++cbase) {
      if (cbase & tmask) continue;
      for (int a = 0; a < D; ++a) {
        const uint64_t e = ((uint64_t)r * dim + (cbase | off[a])) * 2;
        vr[a] = T[e];
        vi[a] = T[e + 1];
      }
      /* (T K^dag)[r][c'] = sum_c T[r][c] * conj(K[c'][c]) */
      for (int b = 0; b < D; ++b) {
        double sr = 0.0, si = 0.0;
        for (int a = 0; a < D; ++a) {
          const double kr = K[2 * (b * D + a)], ki = -K[2 * (b * D + a) + 1];
          sr += vr[a] * kr - vi[a] * ki;
          si += vr[a] * ki + vi[a] * kr;
        }
        const uint64_t o = ((uint64_t)r * dim + (cbase | off[b])) * 2;
        T[o] = sr;
        T[o + 1] = si;
      }
    }
  }
}

/*
 * rho <- sum_i K_i rho K_i^dagger for the m Kraus matrices K (each 2^j x 2^j).
 * T and acc are caller-provided scratch of the same size as rho (acc unused when m == 1).
 * Returns 0, or -1 on bad arguments.
 */
int oracle_apply_kraus(int n, double* rho, double* T, double* acc, int j, const int* qubits, int m,
                       const double* K) {
  if (n < 1 || n > 20 || !rho || !T || !K || m < 1) return -1;
  if (check_targets(n, j, qubits)) return -1;
  const uint64_t dim = (uint64_t)1 << n;
  const uint64_t nd = dim * dim * 2;
  const int D = 1 << j;
  const size_t kstride = (size_t)D * D * 2;
  if (m == 1) {
    left_multiply(n, rho, T, j, qubits, K);
    right_multiply_adjoint(n, T, j, qubits, K);
    memcpy(rho, T, nd * sizeof(double));
    return 0;
  }
  if (!acc) return -1;
  memset(acc, 0, nd * sizeof(double));
  for (int i = 0; i < m; ++i) {
    left_multiply(n, rho, T, j, qubits, K + i * kstride);
    right_multiply_adjoint(n, T, j, qubits, K + i * kstride);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)nd; ++e) acc[e] += T[e];
  }
  memcpy(rho, acc, nd * sizeof(double));
  return 0;
}

/* rho <- |0..0><0..0| */
int oracle_init_zero(int n, double* rho) {
  if (n < 1 || n > 20 || !rho) return -1;
  const uint64_t dim = (uint64_t)1 << n;
  memset(rho, 0, dim * dim * 2 * sizeof(double));
  rho[0] = 1.0;
  return 0;
}

/* diag_out[x] = Re rho[x][x]; returns the trace through *trace. */
int oracle_diagonal(int n, const double* rho, double* diag_out, double* trace) {
  if (n < 1 || n > 20 || !rho || !diag_out) return -1;
  const uint64_t dim = (uint64_t)1 << n;
  double t = 0.0;
  for (uint64_t x = 0; x < dim; ++x) {
    diag_out[x] = rho[2 * (x * dim + x)];
    t += diag_out[x];
  }
  if (trace) *trace = t;
  return 0;
}

/*
 * Tr(P rho) for the Pauli string P = (x)_t sigma_{pauli[t]}, where character t acts on
 * qubit t.  Uses the definition Tr(P rho) = sum_{a,b} P[a][b] rho[b][a] with
 * P[a][b] = prod_t sigma_t[a_t][b_t]; for each b exactly one a (b with the X/Y bits
 * flipped) has a non-zero product, so the double sum is evaluated over that a only.
 */
int oracle_expect_pauli(int n, const double* rho, const char* pauli, double* re, double* im) {
  if (n < 1 || n > 20 || !rho || !pauli || !re || !im) return -1;
  /* sigma[s][out][in] as (re, im) */
  static const double SIG[4][2][2][2] = {
      {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}},   /* I */
      {{{0, 0}, {1, 0}}, {{1, 0}, {0, 0}}},   /* X */
      {{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},  /* Y = [[0,-i],[i,0]] */
      {{{1, 0}, {0, 0}}, {{0, 0}, {-1, 0}}},  /* Z */
  };
  int code[64];
  uint64_t flip = 0;
  for (int t = 0; t < n; ++t) {
    switch (pauli[t]) {
      case 'I': code[t] = 0; break;
      case 'X': code[t] = 1; flip |= (uint64_t)1 << t; break;
      case 'Y': code[t] = 2; flip |= (uint64_t)1 << t; break;
      case 'Z': code[t] = 3; break;
      default: return -1;
    }
  }
  if (pauli[n] != '\0') return -1;
  const uint64_t dim = (uint64_t)1 << n;
  double sr = 0.0, si = 0.0;
  for (uint64_t b = 0; b < dim; ++b) {
    const uint64_t a = b ^ flip;
    double pr = 1.0, pi = 0.0; /* P[a][b] */
    for (int t = 0; t < n; ++t) {
      const int at = (int)((a >> t) & 1u), bt = (int)((b >> t) & 1u);
      const double zr = SIG[code[t]][at][bt][0], zi = SIG[code[t]][at][bt][1];
      const double nr = pr * zr - pi * zi, ni = pr * zi + pi * zr;
      pr = nr;
      pi = ni;
    }
    const uint64_t e = 2 * (b * dim + a); /* rho[b][a] */
    sr += pr * rho[e] - pi * rho[e + 1];
    si += pr * rho[e + 1] + pi * rho[e];
  }
  *re = sr;
  *im = si;
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
