/*
 * CPU oracle for the lattice Dirac operators: plain, slow, FP64.
 *
 * TEST INFRASTRUCTURE ONLY. This file is used by the test suite, by the smoke
 * check and by the CPU-baseline timing in the benchmark; the GPU library never
 * links, loads or calls it, and it shares no code with the GPU kernels.
 *
 * Everything here is written out from the definitions in the paper
 * (Babich et al., "Scaling Lattice QCD beyond 100 GPUs", SC11):
 *   - the Wilson hopping term D of the Wilson-clover matrix, Section II-B, eq. (2);
 *   - the clover field A_x of eq. (2) (footnote: 72 reals per site);
 *   - the improved-staggered hopping term with fat and 3-hop long links,
 *     Section II-C, eq. (3), long link = product of three thin links.
 * Conventions that the paper leaves open are fixed as follows (each is listed
 * with its reason in the design notes of the repository):
 *   - chiral gamma basis, gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]];
 *   - the spin factors of eq. (2) are read as (1 -/+ gamma_mu);
 *   - kappa normalisation: M = A - kappa D, A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu,
 *     F_munu = (Q_munu - Q_numu)/8 from the four clover leaves, sigma = (i/2)[g_mu,g_nu];
 *   - staggered backward hops carry a minus sign (the operator is anti-Hermitian,
 *     Section III-A), Kogut-Susskind phases eta_mu(x);
 *   - a hop that crosses the t boundary k times is multiplied by bc_t^k;
 *   - Dirichlet block cut: a hop is dropped when its two end sites lie in
 *     different blocks of size B (blocks tile from the origin); along an axis
 *     with a single block the periodic hop is kept.
 *
 * Natural layout: site i = x + Lx*(y + Ly*(z + Lz*t)).
 *   gauge  [site][mu][3][3]      Wilson spinor [site][spin][colour]
 *   clover [site][12][12] with row/column index spin*3 + colour
 *   staggered spinor [site][colour]
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                            */

static void site_coords(const int L[4], int64_t i, int c[4]) {
  for (int d = 0; d < 4; ++d) {
    c[d] = (int)(i % L[d]);
    i /= L[d];
  }
}

static int64_t site_index(const int L[4], const int c[4]) {
  return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

static int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

/* Site reached from c by `step` hops along mu; *wraps = boundary crossings. */
static int64_t hop_site(const int L[4], const int c[4], int mu, int step, int *wraps) {
  int d[4] = {c[0], c[1], c[2], c[3]};
  int raw = c[mu] + step;
  int w = floor_div(raw, L[mu]);
  d[mu] = raw - w * L[mu];
  *wraps = w < 0 ? -w : w;
  return site_index(L, d);
}

/* Phase of a hop: bc_t per crossing of the t boundary. */
static double hop_phase(int mu, int wraps, int bc_t) {
  if (mu != 3) return 1.0;
  return (wraps % 2) ? (double)bc_t : 1.0;
}

/* Dirichlet cut: is the hop from coordinate a to a+step along mu inside one block? */
static int hop_kept(const int L[4], const int *block, const int c[4], int mu, int step) {
  if (!block) return 1;
  const int B = block[mu];
  if (B >= L[mu]) return 1;
  const int raw = c[mu] + step;
  if (raw < 0 || raw >= L[mu]) return 0; /* leaves the lattice: necessarily another block */
  return (c[mu] / B) == (raw / B);
}

static int site_parity(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* ------------------------------------------------------------------ */
/* small complex linear algebra                                        */

static void mat3_vec(const cplx *U, const cplx *v, cplx *out) {
  for (int a = 0; a < 3; ++a) out[a] = U[3 * a] * v[0] + U[3 * a + 1] * v[1] + U[3 * a + 2] * v[2];
}

static void mat3_dag_vec(const cplx *U, const cplx *v, cplx *out) {
  for (int a = 0; a < 3; ++a)
    out[a] = conj(U[a]) * v[0] + conj(U[3 + a]) * v[1] + conj(U[6 + a]) * v[2];
}

static void mat3_mul(const cplx *a, const cplx *b, cplx *c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      c[3 * i + j] = s;
    }
}

static void mat3_dag(const cplx *a, cplx *c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c[3 * i + j] = conj(a[3 * j + i]);
}

/* ------------------------------------------------------------------ */
/* gamma matrices, chiral basis                                        */

static cplx GAMMA[5][4][4];
static cplx SIGMA[4][4][4][4]; /* sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] */

__attribute__((constructor)) static void init_gammas(void) {
  const cplx pauli[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  memset(GAMMA, 0, sizeof(GAMMA));
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        GAMMA[k][a][2 + b] = -I * pauli[k][a][b];
        GAMMA[k][2 + a][b] = I * pauli[k][a][b];
      }
  for (int a = 0; a < 2; ++a) {
    GAMMA[3][a][2 + a] = 1;
    GAMMA[3][2 + a][a] = 1;
  }
  /* gamma5 = gamma_1 gamma_2 gamma_3 gamma_4 */
  cplx t1[4][4], t2[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += GAMMA[0][i][k] * GAMMA[1][k][j];
      t1[i][j] = s;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += t1[i][k] * GAMMA[2][k][j];
      t2[i][j] = s;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += t2[i][k] * GAMMA[3][k][j];
      GAMMA[4][i][j] = s;
    }
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          cplx c = 0;
          for (int k = 0; k < 4; ++k) c += GAMMA[m][i][k] * GAMMA[n][k][j] - GAMMA[n][i][k] * GAMMA[m][k][j];
          SIGMA[m][n][i][j] = 0.5 * I * c;
        }
}

/* Copy of a gamma matrix (0..3: x,y,z,t; 4: gamma5) for the tests. */
void ora_gamma(int mu, cplx *out16) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out16[4 * i + j] = GAMMA[mu][i][j];
}

/* ------------------------------------------------------------------ */
/* Wilson hopping term, eq. (2)                                        */

/*
 * (D psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ].
 * dagger != 0 applies D^+, whose matrix elements are the conjugate transposes
 * of D's: the same hops with the spin factors (1 + gamma_mu) forward and
 * (1 - gamma_mu) backward.
 */
static void wilson_site(const int L[4], int bc_t, const cplx *U, const cplx *in, int64_t x,
                        int dagger, const int *block, cplx *out12) {
  int c[4];
  site_coords(L, x, c);
  for (int k = 0; k < 12; ++k) out12[k] = 0;
  const double sgn = dagger ? -1.0 : 1.0;
  for (int mu = 0; mu < 4; ++mu) {
    for (int dir = -1; dir <= 1; dir += 2) {
      if (!hop_kept(L, block, c, mu, dir)) continue;
      int wraps;
      const int64_t y = hop_site(L, c, mu, dir, &wraps);
      const double phase = hop_phase(mu, wraps, bc_t);
      /* colour part: U_mu(x) psi(y) forward, U_mu(y)^+ psi(y) backward */
      cplx v[4][3];
      for (int s = 0; s < 4; ++s) {
        if (dir > 0)
          mat3_vec(U + 9 * (4 * x + mu), in + 12 * y + 3 * s, v[s]);
        else
          mat3_dag_vec(U + 9 * (4 * y + mu), in + 12 * y + 3 * s, v[s]);
      }
      /* spin part: (1 - dir*sgn*gamma_mu) */
      const double g = -(double)dir * sgn;
      for (int s = 0; s < 4; ++s)
        for (int s2 = 0; s2 < 4; ++s2) {
          const cplx P = (s == s2 ? 1.0 : 0.0) + g * GAMMA[mu][s][s2];
          if (P == 0) continue;
          for (int a = 0; a < 3; ++a) out12[3 * s + a] += phase * P * v[s2][a];
        }
    }
  }
}

/*
 * out = D in (or D^+ in).
 * sites == NULL: compute every site of parity out_parity (-1: all sites);
 *   out is a full natural field with zeros on the other parity.
 * sites != NULL: compute only those nsites sites; out is [nsites][12].
 * block: NULL or the Dirichlet block size per axis.
 */
void ora_wilson_dslash(const int L[4], int bc_t, const cplx *U, const cplx *in, cplx *out,
                       int out_parity, int dagger, const int *block, const int64_t *sites,
                       int64_t nsites) {
  if (sites) {
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < nsites; ++n) wilson_site(L, bc_t, U, in, sites[n], dagger, block, out + 12 * n);
    return;
  }
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x) {
    int c[4];
    site_coords(L, x, c);
    if (out_parity >= 0 && site_parity(c) != out_parity) {
      for (int k = 0; k < 12; ++k) out[12 * x + k] = 0;
      continue;
    }
    wilson_site(L, bc_t, U, in, x, dagger, block, out + 12 * x);
  }
}

/* ------------------------------------------------------------------ */
/* clover term                                                         */

static const cplx *link(const cplx *U, int64_t x, int mu) { return U + 9 * (4 * x + mu); }

static int64_t shifted(const int L[4], int64_t x, int mu, int step) {
  int c[4], w;
  site_coords(L, x, c);
  return hop_site(L, c, mu, step, &w);
}

/* Product of four 3x3 matrices, each optionally daggered. */
static void prod4(const cplx *a, int da, const cplx *b, int db, const cplx *c, int dc, const cplx *d,
                  int dd, cplx *out) {
  cplx A[9], B[9], C[9], D[9], t1[9], t2[9];
  if (da) mat3_dag(a, A); else memcpy(A, a, sizeof(A));
  if (db) mat3_dag(b, B); else memcpy(B, b, sizeof(B));
  if (dc) mat3_dag(c, C); else memcpy(C, c, sizeof(C));
  if (dd) mat3_dag(d, D); else memcpy(D, d, sizeof(D));
  mat3_mul(A, B, t1);
  mat3_mul(t1, C, t2);
  mat3_mul(t2, D, out);
}

/* Sum of the four clover leaves Q_{mu nu}(x) in the (mu, nu) plane. */
static void clover_leaves(const int L[4], const cplx *U, int64_t x, int mu, int nu, cplx Q[9]) {
  const int64_t xpm = shifted(L, x, mu, +1), xpn = shifted(L, x, nu, +1);
  const int64_t xmm = shifted(L, x, mu, -1), xmn = shifted(L, x, nu, -1);
  const int64_t xmm_pn = shifted(L, xmm, nu, +1), xmm_mn = shifted(L, xmm, nu, -1);
  const int64_t xpm_mn = shifted(L, xpm, nu, -1);
  cplx leaf[9];
  for (int k = 0; k < 9; ++k) Q[k] = 0;
  /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
  prod4(link(U, x, mu), 0, link(U, xpm, nu), 0, link(U, xpn, mu), 1, link(U, x, nu), 1, leaf);
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  /* U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
  prod4(link(U, x, nu), 0, link(U, xmm_pn, mu), 1, link(U, xmm, nu), 1, link(U, xmm, mu), 0, leaf);
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  /* U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
  prod4(link(U, xmm, mu), 1, link(U, xmm_mn, nu), 1, link(U, xmm_mn, mu), 0, link(U, xmn, nu), 0, leaf);
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  /* U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+ */
  prod4(link(U, xmn, nu), 1, link(U, xmn, mu), 0, link(U, xpm_mn, nu), 0, link(U, x, mu), 1, leaf);
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
}

/*
 * A_x = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x),
 * F_{mu nu} = (Q_{mu nu} - Q_{nu mu}) / 8; A is [V][12][12].
 */
void ora_clover_build(const int L[4], const cplx *U, double kappa, double csw, cplx *A) {
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x) {
    cplx *Ax = A + 144 * x;
    for (int k = 0; k < 144; ++k) Ax[k] = 0;
    for (int k = 0; k < 12; ++k) Ax[13 * k] = 1;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        cplx Qmn[9], Qnm[9], F[9];
        clover_leaves(L, U, x, mu, nu, Qmn);
        clover_leaves(L, U, x, nu, mu, Qnm);
        for (int k = 0; k < 9; ++k) F[k] = (Qmn[k] - Qnm[k]) / 8.0;
        for (int s = 0; s < 4; ++s)
          for (int s2 = 0; s2 < 4; ++s2) {
            const cplx sg = SIGMA[mu][nu][s][s2];
            if (sg == 0) continue;
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) Ax[12 * (3 * s + a) + 3 * s2 + b] += I * kappa * csw * sg * F[3 * a + b];
          }
      }
  }
}

/* out(x) = A(x) in(x) on the sites of `parity` (-1: all); zeros elsewhere. */
void ora_clover_apply(const int L[4], const cplx *A, const cplx *in, cplx *out, int parity) {
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x) {
    int c[4];
    site_coords(L, x, c);
    if (parity >= 0 && site_parity(c) != parity) {
      for (int k = 0; k < 12; ++k) out[12 * x + k] = 0;
      continue;
    }
    for (int i = 0; i < 12; ++i) {
      cplx s = 0;
      for (int j = 0; j < 12; ++j) s += A[144 * x + 12 * i + j] * in[12 * x + j];
      out[12 * x + i] = s;
    }
  }
}

/* Per-site 12x12 inverse by Gauss-Jordan elimination with partial pivoting.
 * Returns the number of sites whose matrix was numerically singular. */
int64_t ora_clover_invert(const int L[4], const cplx *A, cplx *Ainv) {
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
  int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t x = 0; x < V; ++x) {
    cplx M[12][24];
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) {
        M[i][j] = A[144 * x + 12 * i + j];
        M[i][12 + j] = (i == j) ? 1.0 : 0.0;
      }
    for (int col = 0; col < 12; ++col) {
      int piv = col;
      for (int r = col + 1; r < 12; ++r)
        if (cabs(M[r][col]) > cabs(M[piv][col])) piv = r;
      if (cabs(M[piv][col]) < 1e-300) { bad++; break; }
      if (piv != col)
        for (int j = 0; j < 24; ++j) { cplx t = M[col][j]; M[col][j] = M[piv][j]; M[piv][j] = t; }
      const cplx inv = 1.0 / M[col][col];
      for (int j = 0; j < 24; ++j) M[col][j] *= inv;
      for (int r = 0; r < 12; ++r) {
        if (r == col) continue;
        const cplx f = M[r][col];
        if (f == 0) continue;
        for (int j = 0; j < 24; ++j) M[r][j] -= f * M[col][j];
      }
    }
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) Ainv[144 * x + 12 * i + j] = M[i][12 + j];
  }
  return bad;
}

/* ------------------------------------------------------------------ */
/* improved staggered, eq. (3)                                         */

/* Long link: U_mu(x) U_mu(x+mu) U_mu(x+2mu) (thin links, no boundary phase). */
void ora_long_links(const int L[4], const cplx *U, cplx *lng) {
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x)
    for (int mu = 0; mu < 4; ++mu) {
      const int64_t x1 = shifted(L, x, mu, 1), x2 = shifted(L, x, mu, 2);
      cplx t[9];
      mat3_mul(link(U, x, mu), link(U, x1, mu), t);
      mat3_mul(t, link(U, x2, mu), lng + 9 * (4 * x + mu));
    }
}

/* Kogut-Susskind phases: eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z). */
static double ks_eta(const int c[4], int mu) {
  int s = 0;
  for (int d = 0; d < mu; ++d) s += c[d];
  return (s & 1) ? -1.0 : 1.0;
}

/*
 * (D chi)(x) = sum_mu eta_mu(x) [ F_mu(x) chi(x+mu) - F_mu(x-mu)^+ chi(x-mu)
 *                                + c_long ( L_mu(x) chi(x+3mu) - L_mu(x-3mu)^+ chi(x-3mu) ) ].
 * D is anti-Hermitian, so its adjoint is -D (the caller negates).
 */
static void stag_site(const int L[4], int bc_t, const cplx *fat, const cplx *lng, double c_long,
                      const cplx *in, int64_t x, cplx *out3) {
  int c[4];
  site_coords(L, x, c);
  for (int a = 0; a < 3; ++a) out3[a] = 0;
  for (int mu = 0; mu < 4; ++mu) {
    const double eta = ks_eta(c, mu);
    const int steps[2] = {1, 3};
    for (int h = 0; h < 2; ++h) {
      const int k = steps[h];
      const cplx *G = (k == 1) ? fat : lng;
      const double coef = (k == 1) ? 1.0 : c_long;
      if (coef == 0.0) continue;
      int wf, wb;
      const int64_t yf = hop_site(L, c, mu, +k, &wf);
      const int64_t yb = hop_site(L, c, mu, -k, &wb);
      cplx v[3];
      mat3_vec(G + 9 * (4 * x + mu), in + 3 * yf, v);
      const double pf = hop_phase(mu, wf, bc_t);
      for (int a = 0; a < 3; ++a) out3[a] += eta * coef * pf * v[a];
      mat3_dag_vec(G + 9 * (4 * yb + mu), in + 3 * yb, v);
      const double pb = hop_phase(mu, wb, bc_t);
      for (int a = 0; a < 3; ++a) out3[a] -= eta * coef * pb * v[a];
    }
  }
}

void ora_stag_dslash(const int L[4], int bc_t, const cplx *fat, const cplx *lng, double c_long,
                     const cplx *in, cplx *out, int out_parity, const int64_t *sites, int64_t nsites) {
  if (sites) {
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < nsites; ++n) stag_site(L, bc_t, fat, lng, c_long, in, sites[n], out + 3 * n);
    return;
  }
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x) {
    int c[4];
    site_coords(L, x, c);
    if (out_parity >= 0 && site_parity(c) != out_parity) {
      for (int a = 0; a < 3; ++a) out[3 * x + a] = 0;
      continue;
    }
    stag_site(L, bc_t, fat, lng, c_long, in, x, out + 3 * x);
  }
}

/* ------------------------------------------------------------------ */
/* parallel-transport shift used by the learned preconditioner          */

/*
 * T_p psi for one path p: p = 0 identity; p = 1+2*mu: forward,
 * (T psi)(x) = U_mu(x) psi(x+mu); p = 2+2*mu: backward, (T psi)(x) = U_mu(x-mu)^+ psi(x-mu).
 * Boundary phases as for the Dirac operator. psi holds nfield fields of
 * [site][4][3]; the same transport is applied to each. adjoint != 0 applies
 * the adjoint map T_p^+ instead.
 */
void ora_transport(const int L[4], int bc_t, const cplx *U, int path, int adjoint, int64_t nfield,
                   const cplx *in, cplx *out) {
  const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
  int mu = -1, dir = 0;
  if (path > 0) { mu = (path - 1) / 2; dir = ((path - 1) % 2 == 0) ? +1 : -1; }
  if (adjoint) dir = -dir; /* T_{+mu}^+ = T_{-mu} and vice versa */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x) {
    if (mu < 0) {
      for (int64_t f = 0; f < nfield; ++f) memcpy(out + 12 * (f * V + x), in + 12 * (f * V + x), 12 * sizeof(cplx));
      continue;
    }
    int c[4], w;
    site_coords(L, x, c);
    const int64_t y = hop_site(L, c, mu, dir, &w);
    const double ph = hop_phase(mu, w, bc_t);
    for (int64_t f = 0; f < nfield; ++f)
      for (int s = 0; s < 4; ++s) {
        cplx v[3];
        if (dir > 0) mat3_vec(link(U, x, mu), in + 12 * (f * V + y) + 3 * s, v);
        else mat3_dag_vec(link(U, y, mu), in + 12 * (f * V + y) + 3 * s, v);
        for (int a = 0; a < 3; ++a) out[12 * (f * V + x) + 3 * s + a] = ph * v[a];
      }
  }
}
