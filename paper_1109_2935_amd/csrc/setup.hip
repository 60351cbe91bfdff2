// Setup kernels: packing between the natural FP64 exchange format and the
// packed tiled layout, SU(3) link compression, the long links of eq. (3) and
// the clover field of eq. (2) with its per-site inverse.
#include "lqcd_internal.h"

namespace lqcd {

__device__ __forceinline__ int64_t natural_index(const Geom &g, const int X[4]) {
  return X[0] + (int64_t)g.L[0] * (X[1] + (int64_t)g.L[1] * (X[2] + (int64_t)g.L[2] * X[3]));
}

__device__ __forceinline__ void site_global(const Geom &g, const Site &x, int X[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) X[m] = x.t[m] * g.B[m] + x.l[m];
}

// ---------------------------------------------------------------------------
// spinors

// nrhs natural fields (consecutive, V sites each) <-> one packed field in the
// multi-source layout (rhs_index: blocks of rhs_group(nrhs) sources).
template <typename S, int NSP>
__global__ void __launch_bounds__(256) spinor_import_kernel(Geom g, S *packed, const double *nat, int parity,
                                                            int nrhs) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= g.Vh * nrhs) return;
  const int R = rhs_group(nrhs), q = pidx / R, blk = q / g.Vh, s = q - blk * g.Vh, r = blk * R + pidx % R;
  const Site x = decode_site(g, s, parity);
  int X[4];
  site_global(g, x, X);
  const int64_t V = 2 * (int64_t)g.Vh;
  const double *src = nat + NSP * (r * V + natural_index(g, X));
  double v[NSP];
#pragma unroll
  for (int k = 0; k < NSP; ++k) v[k] = src[k];
  store_spinor_reals<S, NSP, double>(packed, (int64_t)g.Vh * nrhs, pidx, v);
}

template <typename S, int NSP>
__global__ void __launch_bounds__(256) spinor_export_kernel(Geom g, double *nat, const S *packed, int parity,
                                                            int nrhs) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= g.Vh * nrhs) return;
  const int R = rhs_group(nrhs), q = pidx / R, blk = q / g.Vh, s = q - blk * g.Vh, r = blk * R + pidx % R;
  const Site x = decode_site(g, s, parity);
  int X[4];
  site_global(g, x, X);
  double v[NSP];
  load_spinor_reals<S, NSP, double>(packed, (int64_t)g.Vh * nrhs, pidx, v);
  const int64_t V = 2 * (int64_t)g.Vh;
  double *dst = nat + NSP * (r * V + natural_index(g, X));
#pragma unroll
  for (int k = 0; k < NSP; ++k) dst[k] = v[k];
}

// out = scale * in between two tiled layouts of the same lattice (one parity
// block each, nrhs sources in the multi-source layout), any precisions: one
// thread per output (site, source), which finds its site in the input layout.
template <typename So, typename Si, int NSP>
__global__ void __launch_bounds__(256) spinor_relayout_kernel(Geom go, So *out, Geom gi, const Si *in, int parity,
                                                              int nrhs, double scale) {
  const int64_t pidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vh = go.Vh;
  if (pidx >= vh * nrhs) return;
  const int R = rhs_group(nrhs);
  const int64_t q = pidx / R, blk = q / vh;
  const int s = (int)(q - blk * vh), r = (int)(blk * R + pidx % R);
  int X[4], t[4], l[4];
  site_global(go, decode_site(go, s, parity), X);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    t[m] = X[m] / gi.B[m];
    l[m] = X[m] - t[m] * gi.B[m];
  }
  const int si = encode_site(gi, t, l);
  double v[NSP];
  load_spinor_reals<Si, NSP, double>(in, vh * nrhs, rhs_index(r, si, vh, R), v);
#pragma unroll
  for (int k = 0; k < NSP; ++k) v[k] *= scale;
  store_spinor_reals<So, NSP, double>(out, vh * nrhs, pidx, v);
}

template <typename So, int NSP>
static hipError_t relayout_in(const Geom &go, So *out, const Geom &gi, int pin, const void *in, int parity, int nrhs,
                              double scale, hipStream_t st) {
  const int bt = 256;
  const int nwg = (int)(((int64_t)go.Vh * nrhs + bt - 1) / bt);
  switch (pin) {
#define CASE(P)                                                                                                     \
  case P:                                                                                                           \
    hipLaunchKernelGGL((spinor_relayout_kernel<So, Prec<P>::S, NSP>), dim3(nwg), dim3(bt), 0, st, go, out, gi,      \
                       (const Prec<P>::S *)in, parity, nrhs, scale);                                                \
    return hipGetLastError();
    CASE(LQCD_F64)
    CASE(LQCD_F32)
    CASE(LQCD_F16)
    CASE(LQCD_BF16)
    CASE(LQCD_HALF)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spinor_relayout(const Geom &go, int pout, void *out, const Geom &gi, int pin, const void *in, int nsp,
                                  int parity, int nrhs, double scale, hipStream_t st) {
  if (go.Vh == 0) return hipSuccess;
  switch (pout) {
#define CASE(P)                                                                                                     \
  case P:                                                                                                           \
    return nsp == 24 ? relayout_in<Prec<P>::S, 24>(go, (Prec<P>::S *)out, gi, pin, in, parity, nrhs, scale, st)    \
                     : relayout_in<Prec<P>::S, 6>(go, (Prec<P>::S *)out, gi, pin, in, parity, nrhs, scale, st);
    CASE(LQCD_F64)
    CASE(LQCD_F32)
    CASE(LQCD_F16)
    CASE(LQCD_BF16)
    CASE(LQCD_HALF)
#undef CASE
  }
  return hipErrorInvalidValue;
}

template <int NSP>
static hipError_t spinor_io(const Geom &g, int prec, void *packed, double *natural, int parity, int nrhs, bool imp,
                            hipStream_t st) {
  const int bt = 256, nwg = (int)(((int64_t)g.Vh * nrhs + bt - 1) / bt);
  switch (prec) {
#define CASE(P)                                                                                               \
  case P:                                                                                                     \
    if (imp)                                                                                                  \
      hipLaunchKernelGGL((spinor_import_kernel<Prec<P>::S, NSP>), dim3(nwg), dim3(bt), 0, st, g,              \
                         (Prec<P>::S *)packed, (const double *)natural, parity, nrhs);                         \
    else                                                                                                      \
      hipLaunchKernelGGL((spinor_export_kernel<Prec<P>::S, NSP>), dim3(nwg), dim3(bt), 0, st, g, natural,     \
                         (const Prec<P>::S *)packed, parity, nrhs);                                           \
    return hipGetLastError();
    CASE(LQCD_F64)
    CASE(LQCD_F32)
    CASE(LQCD_F16)
    CASE(LQCD_BF16)
    CASE(LQCD_HALF)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spinor_import(const Geom &g, int prec, int nsp, void *packed, const double *natural, int parity,
                                int nrhs, hipStream_t st) {
  if (g.Vh == 0) return hipSuccess;
  return nsp == 24 ? spinor_io<24>(g, prec, packed, (double *)natural, parity, nrhs, true, st)
                   : spinor_io<6>(g, prec, packed, (double *)natural, parity, nrhs, true, st);
}

hipError_t launch_spinor_export(const Geom &g, int prec, int nsp, double *natural, const void *packed, int parity,
                                int nrhs, hipStream_t st) {
  if (g.Vh == 0) return hipSuccess;
  return nsp == 24 ? spinor_io<24>(g, prec, (void *)packed, natural, parity, nrhs, false, st)
                   : spinor_io<6>(g, prec, (void *)packed, natural, parity, nrhs, false, st);
}

// ---------------------------------------------------------------------------
// links

struct DLink {
  double re[3][3], im[3][3];
};

__device__ __forceinline__ DLink nat_link(const Geom &g, const double *nat, const int X[4], int mu) {
  const double *p = nat + 18 * (4 * natural_index(g, X) + mu);
  DLink u;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u.re[i][j] = p[6 * i + 2 * j];
      u.im[i][j] = p[6 * i + 2 * j + 1];
    }
  return u;
}

// c = a * b, each optionally conjugate-transposed
__device__ __forceinline__ DLink dmul(const DLink &a, bool da, const DLink &b, bool db) {
  DLink c;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double sr = 0, si = 0;
      for (int k = 0; k < 3; ++k) {
        const double ar = da ? a.re[k][i] : a.re[i][k], ai = da ? -a.im[k][i] : a.im[i][k];
        const double br = db ? b.re[j][k] : b.re[k][j], bi = db ? -b.im[j][k] : b.im[k][j];
        sr += ar * br - ai * bi;
        si += ar * bi + ai * br;
      }
      c.re[i][j] = sr;
      c.im[i][j] = si;
    }
  return c;
}

__device__ __forceinline__ void shift(const Geom &g, const int X[4], int mu, int step, int Y[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) Y[m] = X[m];
  Y[mu] = ((X[mu] + step) % g.L[mu] + g.L[mu]) % g.L[mu];
}

template <typename S, int RECON>
__device__ __forceinline__ void pack_link(S *base, int64_t vh, int s, const DLink &u) {
  double v[RECON];
  if constexpr (RECON == 8) {
    v[0] = u.re[0][1]; v[1] = u.im[0][1];
    v[2] = u.re[0][2]; v[3] = u.im[0][2];
    v[4] = u.re[1][0]; v[5] = u.im[1][0];
    v[6] = atan2(u.im[0][0], u.re[0][0]);
    v[7] = atan2(u.im[2][0], u.re[2][0]);
  } else {
#pragma unroll
    for (int k = 0; k < RECON / 2; ++k) {
      v[2 * k] = u.re[k / 3][k % 3];
      v[2 * k + 1] = u.im[k / 3][k % 3];
    }
  }
  store_site<S, RECON, double>(base, vh, s, v);
}

// One thread per (site of one parity); loops over the 4 directions.
// form_long: pack the 3-hop product U_mu(x) U_mu(x+mu) U_mu(x+2mu).
template <typename S, int RECON>
__global__ void __launch_bounds__(128) gauge_import_kernel(Geom g, S *packed, const double *nat, int form_long) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * g.Vh) return;
  const int parity = idx >= g.Vh ? 1 : 0;
  const int s = idx - parity * g.Vh;
  const Site x = decode_site(g, s, parity);
  int X[4];
  site_global(g, x, X);
  for (int mu = 0; mu < 4; ++mu) {
    DLink u = nat_link(g, nat, X, mu);
    if (form_long) {
      int Y[4], Z[4];
      shift(g, X, mu, 1, Y);
      shift(g, X, mu, 2, Z);
      u = dmul(dmul(u, false, nat_link(g, nat, Y, mu), false), false, nat_link(g, nat, Z, mu), false);
    }
    pack_link<S, RECON>(packed + (int64_t)(2 * mu + parity) * g.Vh * RECON, g.Vh, s, u);
  }
}

template <int RECON>
static hipError_t gauge_io(const Geom &g, int prec, void *packed, const double *nat, int form_long, hipStream_t st) {
  const int bt = 128, nwg = (2 * g.Vh + bt - 1) / bt;
  switch (prec) {
#define CASE(P)                                                                                                   \
  case P:                                                                                                         \
    hipLaunchKernelGGL((gauge_import_kernel<Prec<P>::S, RECON>), dim3(nwg), dim3(bt), 0, st, g,                  \
                       (Prec<P>::S *)packed, nat, form_long);                                                     \
    return hipGetLastError();
    CASE(LQCD_F64)
    CASE(LQCD_F32)
    CASE(LQCD_F16)
    CASE(LQCD_BF16)
    CASE(LQCD_HALF)
#undef CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gauge_import(const Geom &g, int prec, int recon, void *packed, const double *natural, int form_long,
                               hipStream_t st) {
  if (g.Vh == 0) return hipSuccess;
  switch (recon) {
    case 18: return gauge_io<18>(g, prec, packed, natural, form_long, st);
    case 12: return gauge_io<12>(g, prec, packed, natural, form_long, st);
    case 8: return gauge_io<8>(g, prec, packed, natural, form_long, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// clover term
//
// F_munu = (Q_munu - Q_munu^+)/8 from the four clover leaves (Q_numu is the
// adjoint of Q_munu). In the chiral basis sigma_munu is block diagonal:
// sigma_jk = -eps_jkl diag(s_l, s_l) for spatial j,k and
// sigma_k4 = diag(s_k, -s_k), so per chirality block
//   sum_{mu<nu} sigma F = s_1 (+-F_14 - F_23) + s_2 (F_13 +- F_24) + s_3 (+-F_34 - F_12)
// (upper signs for spins 0,1). Each block, 1 + i kappa c_sw (...), is a
// Hermitian 6x6 stored as 6 real diagonal entries plus the lower triangle.

__device__ DLink clover_leaf_sum(const Geom &g, const double *nat, const int X[4], int mu, int nu) {
  int Xpm[4], Xpn[4], Xmm[4], Xmn[4], Xmm_pn[4], Xmm_mn[4], Xpm_mn[4];
  shift(g, X, mu, 1, Xpm);
  shift(g, X, nu, 1, Xpn);
  shift(g, X, mu, -1, Xmm);
  shift(g, X, nu, -1, Xmn);
  shift(g, Xmm, nu, 1, Xmm_pn);
  shift(g, Xmm, nu, -1, Xmm_mn);
  shift(g, Xpm, nu, -1, Xpm_mn);
  DLink q, t;
  // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
  t = dmul(dmul(nat_link(g, nat, X, mu), false, nat_link(g, nat, Xpm, nu), false), false,
           dmul(nat_link(g, nat, X, nu), false, nat_link(g, nat, Xpn, mu), false), true);
  q = t;
  // U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
  t = dmul(dmul(nat_link(g, nat, X, nu), false, nat_link(g, nat, Xmm_pn, mu), true), false,
           dmul(nat_link(g, nat, Xmm, mu), true, nat_link(g, nat, Xmm, nu), false), true);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { q.re[i][j] += t.re[i][j]; q.im[i][j] += t.im[i][j]; }
  // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
  t = dmul(dmul(nat_link(g, nat, Xmm_mn, nu), false, nat_link(g, nat, Xmm, mu), false), true,
           dmul(nat_link(g, nat, Xmm_mn, mu), false, nat_link(g, nat, Xmn, nu), false), false);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { q.re[i][j] += t.re[i][j]; q.im[i][j] += t.im[i][j]; }
  // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
  t = dmul(dmul(nat_link(g, nat, Xmn, nu), true, nat_link(g, nat, Xmn, mu), false), false,
           dmul(nat_link(g, nat, X, mu), false, nat_link(g, nat, Xpm_mn, nu), true), true);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { q.re[i][j] += t.re[i][j]; q.im[i][j] += t.im[i][j]; }
  return q;
}

// Cholesky-based inverse of a Hermitian positive-definite 6x6 (full storage).
__device__ bool herm6_inverse(const double (&ar)[6][6], const double (&ai)[6][6], double (&br)[6][6],
                              double (&bi)[6][6]) {
  double lr[6][6], li[6][6];
  for (int j = 0; j < 6; ++j) {
    double d = ar[j][j];
    for (int k = 0; k < j; ++k) d -= lr[j][k] * lr[j][k] + li[j][k] * li[j][k];
    if (!(d > 0)) return false;
    const double ljj = sqrt(d);
    lr[j][j] = ljj;
    li[j][j] = 0;
    for (int i = j + 1; i < 6; ++i) {
      double sr = ar[i][j], si = ai[i][j];
      for (int k = 0; k < j; ++k) {  // - L_ik conj(L_jk)
        sr -= lr[i][k] * lr[j][k] + li[i][k] * li[j][k];
        si -= li[i][k] * lr[j][k] - lr[i][k] * li[j][k];
      }
      lr[i][j] = sr / ljj;
      li[i][j] = si / ljj;
    }
  }
  // W = L^-1 (lower triangular)
  double wr[6][6], wi[6][6];
  for (int j = 0; j < 6; ++j) {
    for (int i = 0; i < 6; ++i) { wr[i][j] = 0; wi[i][j] = 0; }
    wr[j][j] = 1.0 / lr[j][j];
    for (int i = j + 1; i < 6; ++i) {
      double sr = 0, si = 0;
      for (int k = j; k < i; ++k) {
        sr += lr[i][k] * wr[k][j] - li[i][k] * wi[k][j];
        si += lr[i][k] * wi[k][j] + li[i][k] * wr[k][j];
      }
      wr[i][j] = -sr / lr[i][i];
      wi[i][j] = -si / lr[i][i];
    }
  }
  // A^-1 = W^+ W
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double sr = 0, si = 0;
      for (int k = (i > j ? i : j); k < 6; ++k) {
        sr += wr[k][i] * wr[k][j] + wi[k][i] * wi[k][j];
        si += wr[k][i] * wi[k][j] - wi[k][i] * wr[k][j];
      }
      br[i][j] = sr;
      bi[i][j] = si;
    }
  return true;
}

__device__ __forceinline__ void pack_herm6(const double (&ar)[6][6], const double (&ai)[6][6], double *dst) {
  for (int i = 0; i < 6; ++i) dst[i] = ar[i][i];
  int off = 6;
  for (int i = 1; i < 6; ++i)
    for (int j = 0; j < i; ++j) {
      dst[off++] = ar[i][j];
      dst[off++] = ai[i][j];
    }
}

// A parity block of the clover field: 72 reals per site, and for fixed-point
// storage the FP32 site norms after them (two code slots per norm).
template <typename S> __host__ __device__ constexpr int64_t clover_block_elems(int64_t vh) {
  return vh * 72 + (is_fixed<S>() ? 2 * vh : 0);
}

template <typename S>
__device__ __forceinline__ void store_clover_site(S *base, int64_t vh, int s, const double *v) {
  if constexpr (is_fixed<S>()) {
    const float m = fixed_norm<72, double>(v), inv = m > 0 ? 1.0f / m : 0.0f;
    float w[72];
    for (int k = 0; k < 72; ++k) w[k] = (float)v[k] * inv;
    store_site<S, 72, float>(base, vh, s, w);
    site_norms<S, 72>(base, vh)[s] = m;
  } else {
    store_site<S, 72, double>(base, vh, s, v);
  }
}

template <typename S>
__global__ void __launch_bounds__(64) clover_build_kernel(Geom g, double kc, S *clov, S *clov_inv, const double *nat,
                                                          int *fail) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * g.Vh) return;
  const int parity = idx >= g.Vh ? 1 : 0;
  const int s = idx - parity * g.Vh;
  const Site x = decode_site(g, s, parity);
  int X[4];
  site_global(g, x, X);
  // F[mu][nu] for mu < nu, anti-Hermitian: F = (Q - Q^+)/8
  double Fr[6][3][3], Fi[6][3][3];
  const int pm[6] = {0, 0, 0, 1, 1, 2}, pn[6] = {1, 2, 3, 2, 3, 3};
  for (int p = 0; p < 6; ++p) {
    const DLink q = clover_leaf_sum(g, nat, X, pm[p], pn[p]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        Fr[p][i][j] = (q.re[i][j] - q.re[j][i]) * 0.125;
        Fi[p][i][j] = (q.im[i][j] + q.im[j][i]) * 0.125;
      }
  }
  // plane order: 0:(x,y)=F12 1:(x,z)=F13 2:(x,t)=F14 3:(y,z)=F23 4:(y,t)=F24 5:(z,t)=F34
  double packed_a[72], packed_i[72];
  bool ok = true;
  for (int b = 0; b < 2; ++b) {
    const double c = (b == 0) ? 1.0 : -1.0;
    double B1r[3][3], B1i[3][3], B2r[3][3], B2i[3][3], B3r[3][3], B3i[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        B1r[i][j] = c * Fr[2][i][j] - Fr[3][i][j];
        B1i[i][j] = c * Fi[2][i][j] - Fi[3][i][j];
        B2r[i][j] = Fr[1][i][j] + c * Fr[4][i][j];
        B2i[i][j] = Fi[1][i][j] + c * Fi[4][i][j];
        B3r[i][j] = c * Fr[5][i][j] - Fr[0][i][j];
        B3i[i][j] = c * Fi[5][i][j] - Fi[0][i][j];
      }
    // A = 1 + i kc [ s1 B1 + s2 B2 + s3 B3 ] on (spin-in-block, colour)
    double ar[6][6], ai[6][6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        // (0,0): i kc B3 ; (1,1): -i kc B3 ; (0,1): i kc (B1 - i B2) ; (1,0): i kc (B1 + i B2)
        ar[i][j] = -kc * B3i[i][j];
        ai[i][j] = kc * B3r[i][j];
        ar[3 + i][3 + j] = kc * B3i[i][j];
        ai[3 + i][3 + j] = -kc * B3r[i][j];
        // i kc (B1 - i B2) = i kc B1 + kc B2
        ar[i][3 + j] = -kc * B1i[i][j] + kc * B2r[i][j];
        ai[i][3 + j] = kc * B1r[i][j] + kc * B2i[i][j];
        // i kc (B1 + i B2) = i kc B1 - kc B2
        ar[3 + i][j] = -kc * B1i[i][j] - kc * B2r[i][j];
        ai[3 + i][j] = kc * B1r[i][j] - kc * B2i[i][j];
      }
    for (int i = 0; i < 6; ++i) ar[i][i] += 1.0;
    double br[6][6], bi[6][6];
    ok = ok && herm6_inverse(ar, ai, br, bi);
    pack_herm6(ar, ai, packed_a + 36 * b);
    pack_herm6(br, bi, packed_i + 36 * b);
  }
  if (!ok) fail[0] = 1;
  store_clover_site<S>(clov + (int64_t)parity * clover_block_elems<S>(g.Vh), g.Vh, s, packed_a);
  store_clover_site<S>(clov_inv + (int64_t)parity * clover_block_elems<S>(g.Vh), g.Vh, s, packed_i);
}

hipError_t launch_clover_build(const Geom &g, int prec, double kappa, double csw, void *clov, void *clov_inv,
                               const double *natural_gauge, int *d_fail, hipStream_t st) {
  if (g.Vh == 0) return hipSuccess;
  const int bt = 64, nwg = (2 * g.Vh + bt - 1) / bt;
  const double kc = kappa * csw;
  switch (prec) {
#define CASE(P)                                                                                              \
  case P:                                                                                                    \
    hipLaunchKernelGGL((clover_build_kernel<Prec<P>::S>), dim3(nwg), dim3(bt), 0, st, g, kc,                 \
                       (Prec<P>::S *)clov, (Prec<P>::S *)clov_inv, natural_gauge, d_fail);                  \
    return hipGetLastError();
    CASE(LQCD_F64)
    CASE(LQCD_F32)
    CASE(LQCD_F16)
    CASE(LQCD_BF16)
    CASE(LQCD_HALF)
#undef CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace lqcd
