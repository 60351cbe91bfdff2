/*
 * Seeded synthetic input fields for the lattice Dirac-operator workloads.
 *
 * This is input preparation only. It holds none of the method's arithmetic
 * (no Dirac operator, no clover term, no long link, no solver): it turns
 * Gaussian draws made by the Python side into
 *   - SU(3) link matrices U = exp(i eps H), H = sum_a h_a lambda_a / 2;
 *   - the synthetic "fat" links used by the improved-staggered workload,
 *     fat_mu(x) = U_mu(x) + w * sum_{nu != mu} [ S_munu(x) + sigma G_munu(x) ],
 *     S_munu(x) = U_nu(x) U_mu(x+nu) U_nu(x+mu)^dagger (forward staple).
 * Both the CPU oracle and the GPU path receive the same bytes.
 *
 * Natural layout: site index i = x + Lx*(y + Ly*(z + Lz*t)); a gauge field is
 * [site][mu][row][col] complex double.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

static void mat_mul(const cplx a[9], const cplx b[9], cplx c[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      c[3 * i + j] = s;
    }
}

/* Gell-Mann matrices lambda_1..lambda_8, row-major. */
static void gell_mann_combination(const double h[8], cplx H[9]) {
  const double r3 = 1.0 / sqrt(3.0);
  memset(H, 0, 9 * sizeof(cplx));
  /* lambda1 */ H[1] += h[0]; H[3] += h[0];
  /* lambda2 */ H[1] += -I * h[1]; H[3] += I * h[1];
  /* lambda3 */ H[0] += h[2]; H[4] -= h[2];
  /* lambda4 */ H[2] += h[3]; H[6] += h[3];
  /* lambda5 */ H[2] += -I * h[4]; H[6] += I * h[4];
  /* lambda6 */ H[5] += h[5]; H[7] += h[5];
  /* lambda7 */ H[5] += -I * h[6]; H[7] += I * h[6];
  /* lambda8 */ H[0] += r3 * h[7]; H[4] += r3 * h[7]; H[8] += -2.0 * r3 * h[7];
  for (int k = 0; k < 9; ++k) H[k] *= 0.5;
}

/* exp(i A) for a Hermitian 3x3 A: scaling and squaring with a Taylor core. */
static void exp_i_hermitian(const cplx A[9], cplx out[9]) {
  double nrm = 0;
  for (int k = 0; k < 9; ++k) nrm += creal(A[k] * conj(A[k]));
  nrm = sqrt(nrm);
  int s = 0;
  while (nrm > 0.125 && s < 60) { nrm *= 0.5; ++s; }
  const double scale = ldexp(1.0, -s);
  cplx X[9], T[9], tmp[9];
  for (int k = 0; k < 9; ++k) X[k] = I * scale * A[k];
  /* sum_{n=0}^{14} X^n / n! ; ||X|| <= 1/8 so the remainder is < 1e-30 */
  memset(out, 0, sizeof(cplx) * 9);
  memset(T, 0, sizeof(cplx) * 9);
  out[0] = out[4] = out[8] = 1.0;
  T[0] = T[4] = T[8] = 1.0;
  for (int n = 1; n <= 14; ++n) {
    mat_mul(T, X, tmp);
    for (int k = 0; k < 9; ++k) { T[k] = tmp[k] / (double)n; out[k] += T[k]; }
  }
  for (int q = 0; q < s; ++q) {
    mat_mul(out, out, tmp);
    memcpy(out, tmp, sizeof(tmp));
  }
}

/* Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): exactly SU(3) up to rounding. */
static void reunitarize(cplx U[9]) {
  double n0 = 0;
  for (int j = 0; j < 3; ++j) n0 += creal(U[j] * conj(U[j]));
  n0 = 1.0 / sqrt(n0);
  for (int j = 0; j < 3; ++j) U[j] *= n0;
  cplx d = 0;
  for (int j = 0; j < 3; ++j) d += conj(U[j]) * U[3 + j];
  for (int j = 0; j < 3; ++j) U[3 + j] -= d * U[j];
  double n1 = 0;
  for (int j = 0; j < 3; ++j) n1 += creal(U[3 + j] * conj(U[3 + j]));
  n1 = 1.0 / sqrt(n1);
  for (int j = 0; j < 3; ++j) U[3 + j] *= n1;
  U[6] = conj(U[1] * U[5] - U[2] * U[4]);
  U[7] = conj(U[2] * U[3] - U[0] * U[5]);
  U[8] = conj(U[0] * U[4] - U[1] * U[3]);
}

/* n links: h is [n][8] Gaussian draws, U is [n][9] complex output. */
void synth_su3_exp(int64_t n, const double *h, double eps, cplx *U) {
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < n; ++l) {
    cplx H[9];
    gell_mann_combination(h + 8 * l, H);
    for (int k = 0; k < 9; ++k) H[k] *= eps;
    exp_i_hermitian(H, U + 9 * l);
    reunitarize(U + 9 * l);
  }
}

static int64_t site_shift(const int L[4], int64_t i, int mu, int step) {
  int c[4];
  int64_t r = i;
  for (int d = 0; d < 4; ++d) { c[d] = (int)(r % L[d]); r /= L[d]; }
  c[mu] = ((c[mu] + step) % L[mu] + L[mu]) % L[mu];
  return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

/*
 * Fat links for the sites [site_begin, site_end). G holds, for those sites in
 * order, [site][mu][k][3][3] complex Gaussians, k = 0..2 enumerating nu != mu
 * in increasing nu.
 */
void synth_fat_links(const int L[4], const cplx *U, int64_t site_begin, int64_t site_end,
                     const cplx *G, double w, double sigma, cplx *fat) {
#pragma omp parallel for schedule(static)
  for (int64_t i = site_begin; i < site_end; ++i) {
    for (int mu = 0; mu < 4; ++mu) {
      const cplx *Umu = U + 9 * (4 * i + mu);
      cplx acc[9];
      for (int k = 0; k < 9; ++k) acc[k] = Umu[k];
      int kk = 0;
      for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const int64_t xn = site_shift(L, i, nu, +1);
        const int64_t xm = site_shift(L, i, mu, +1);
        const cplx *a = U + 9 * (4 * i + nu);
        const cplx *b = U + 9 * (4 * xn + mu);
        const cplx *c = U + 9 * (4 * xm + nu);
        cplx ab[9], cd[9], st[9];
        mat_mul(a, b, ab);
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) cd[3 * r + q] = conj(c[3 * q + r]);
        mat_mul(ab, cd, st);
        const cplx *g = G + 9 * (3 * (4 * (i - site_begin) + mu) + kk);
        for (int k = 0; k < 9; ++k) acc[k] += w * (st[k] + sigma * g[k]);
        ++kk;
      }
      cplx *out = fat + 9 * (4 * (i - site_begin) + mu);
      for (int k = 0; k < 9; ++k) out[k] = acc[k];
    }
  }
}
