// Device-side building blocks shared by the gfx950 kernels: storage
// precisions, chunked structure-of-arrays loads and stores, complex
// arithmetic, magic-number division and the tiled even-odd site geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lqcd.h"

namespace lqcd {

// ---------------------------------------------------------------------------
// storage types

struct bf16 {
  uint16_t bits;
};

// 16-bit fixed point (the "half" format of Section V): a signed integer code
// q in [-32767, 32767] standing for q / 32767. SU(3) link entries lie in
// [-1, 1] and are stored so directly; spinors and the clover term carry one
// FP32 norm per site (the largest magnitude among the site's reals), stored
// after the codes of their parity block, and the codes hold value / norm.
struct fx16 {
  int16_t q;
};
constexpr float kFxScale = 32767.0f;

template <int P> struct Prec;
template <> struct Prec<LQCD_F64> { using S = double; using R = double; };
template <> struct Prec<LQCD_F32> { using S = float; using R = float; };
template <> struct Prec<LQCD_F16> { using S = _Float16; using R = float; };
template <> struct Prec<LQCD_BF16> { using S = bf16; using R = float; };
template <> struct Prec<LQCD_HALF> { using S = fx16; using R = float; };

template <typename S> constexpr bool is_fixed() { return sizeof(S) == 2 && !__is_same(S, _Float16) && !__is_same(S, bf16); }
// IEEE-style 16-bit storage (FP16, BF16): the matrix-core and mixed-precision paths
template <typename S> constexpr bool is_float16() { return __is_same(S, _Float16) || __is_same(S, bf16); }

template <typename R> __device__ __forceinline__ R to_real(double v) { return (R)v; }
template <typename R> __device__ __forceinline__ R to_real(float v) { return (R)v; }
template <typename R> __device__ __forceinline__ R to_real(_Float16 v) { return (R)(float)v; }
template <typename R> __device__ __forceinline__ R to_real(bf16 v) {
  return (R)__uint_as_float(((uint32_t)v.bits) << 16);
}
// the code's unit-scale value (times the site norm where there is one)
template <typename R> __device__ __forceinline__ R to_real(fx16 v) { return (R)((float)v.q * (1.0f / kFxScale)); }

template <typename S> struct Store;
template <> struct Store<double> {
  template <typename R> __device__ __forceinline__ static double from(R v) { return (double)v; }
};
template <> struct Store<float> {
  template <typename R> __device__ __forceinline__ static float from(R v) { return (float)v; }
};
template <> struct Store<_Float16> {
  template <typename R> __device__ __forceinline__ static _Float16 from(R v) { return (_Float16)(float)v; }
};
template <> struct Store<bf16> {
  template <typename R> __device__ __forceinline__ static bf16 from(R v) {
    // round to nearest even; NaN stays NaN
    uint32_t u = __float_as_uint((float)v);
    bf16 r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      r.bits = 0x7fc0;
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      r.bits = (uint16_t)(u >> 16);
    }
    return r;
  }
};

template <> struct Store<fx16> {
  // round to nearest (even) in FP32, saturating at +-1
  template <typename R> __device__ __forceinline__ static fx16 from(R v) {
    float f = (float)v * kFxScale;
    f = fminf(fmaxf(f, -kFxScale), kFxScale);
    return fx16{(int16_t)__float2int_rn(f)};
  }
};

// Reals per 16-byte chunk that also divide N: the unit of a coalesced load.
template <typename S, int N> constexpr int chunk_reals() {
  int c = 16 / (int)sizeof(S);
  while (c > 1 && (N % c) != 0) c /= 2;
  return c;
}

template <typename S, int CH> struct alignas(sizeof(S) * CH) Chunk {
  S v[CH];
};

// A packed per-parity field of N reals per site is stored chunk-major: chunk
// c (CH reals) of site s starts at real (c * stride + s) * CH, stride = sites
// in the parity block, so consecutive threads (sites) touch consecutive
// chunks. Each chunk is moved with accesses of at most 16 bytes.
// Raw integer vectors of 2..16 bytes, for non-temporal accesses of any chunk type.
template <int BYTES> struct RawVec;
template <> struct RawVec<16> { typedef unsigned T __attribute__((ext_vector_type(4))); };
template <> struct RawVec<8> { typedef unsigned T __attribute__((ext_vector_type(2))); };
template <> struct RawVec<4> { typedef unsigned T; };
template <> struct RawVec<2> { typedef unsigned short T; };

// Streaming (non-temporal) load / store: data touched once per kernel (links,
// outputs) is marked so that it does not displace reusable lines (neighbour
// spinors) from the L2.
template <typename C> __device__ __forceinline__ C nt_load(const C *p) {
  using R = typename RawVec<sizeof(C)>::T;
  return __builtin_bit_cast(C, __builtin_nontemporal_load(reinterpret_cast<const R *>(p)));
}
template <typename C> __device__ __forceinline__ void nt_store(C *p, const C &v) {
  using R = typename RawVec<sizeof(C)>::T;
  __builtin_nontemporal_store(__builtin_bit_cast(R, v), reinterpret_cast<R *>(p));
}

template <typename S, int N, int CH, typename R, bool NT = false>
__device__ __forceinline__ void load_chunks(const S *__restrict__ base, int64_t stride, int64_t s, R *out) {
  constexpr int W = (CH * (int)sizeof(S) > 16) ? 16 / (int)sizeof(S) : CH;
#pragma unroll
  for (int c = 0; c < N / CH; ++c) {
    const S *p = base + (c * stride + s) * CH;
#pragma unroll
    for (int w = 0; w < CH / W; ++w) {
      const Chunk<S, W> *q = reinterpret_cast<const Chunk<S, W> *>(p + w * W);
      Chunk<S, W> v = NT ? nt_load(q) : *q;
#pragma unroll
      for (int k = 0; k < W; ++k) out[c * CH + w * W + k] = to_real<R>(v.v[k]);
    }
  }
}

// The same loads without conversion: out holds the stored values.
template <typename S, int N, int CH, bool NT = false>
__device__ __forceinline__ void load_chunks_raw(const S *__restrict__ base, int64_t stride, int64_t s, S *out) {
  constexpr int W = (CH * (int)sizeof(S) > 16) ? 16 / (int)sizeof(S) : CH;
#pragma unroll
  for (int c = 0; c < N / CH; ++c) {
    const S *p = base + (c * stride + s) * CH;
#pragma unroll
    for (int w = 0; w < CH / W; ++w) {
      const Chunk<S, W> *q = reinterpret_cast<const Chunk<S, W> *>(p + w * W);
      Chunk<S, W> v = NT ? nt_load(q) : *q;
#pragma unroll
      for (int k = 0; k < W; ++k) out[c * CH + w * W + k] = v.v[k];
    }
  }
}

template <typename S, int N, int CH, typename R, bool NT = false>
__device__ __forceinline__ void store_chunks(S *__restrict__ base, int64_t stride, int64_t s, const R *in) {
  constexpr int W = (CH * (int)sizeof(S) > 16) ? 16 / (int)sizeof(S) : CH;
#pragma unroll
  for (int c = 0; c < N / CH; ++c) {
    S *p = base + (c * stride + s) * CH;
#pragma unroll
    for (int w = 0; w < CH / W; ++w) {
      Chunk<S, W> v;
#pragma unroll
      for (int k = 0; k < W; ++k) v.v[k] = Store<S>::from(in[c * CH + w * W + k]);
      Chunk<S, W> *q = reinterpret_cast<Chunk<S, W> *>(p + w * W);
      if (NT)
        nt_store(q, v);
      else
        *q = v;
    }
  }
}

// Links and clover: the chunk is the widest 16-byte-or-smaller unit that
// divides N, so the layout of these fields depends on the precision.
template <typename S, int N, typename R, bool NT = false>
__device__ __forceinline__ void load_site(const S *__restrict__ base, int64_t stride, int64_t s, R *out) {
  load_chunks<S, N, chunk_reals<S, N>(), R, NT>(base, stride, s, out);
}
template <typename S, int N, typename R>
__device__ __forceinline__ void store_site(S *__restrict__ base, int64_t stride, int64_t s, const R *in) {
  store_chunks<S, N, chunk_reals<S, N>(), R>(base, stride, s, in);
}

// Per-site field that is read once per launch when stream is true (one
// right-hand side: non-temporal loads keep it from displacing reused data in
// the caches) and by several workgroups otherwise (cached loads).
template <typename S, int N, typename R>
__device__ __forceinline__ void load_site_once(const S *__restrict__ base, int64_t stride, int64_t s, R *out,
                                               bool stream) {
  if (stream)
    load_site<S, N, R, true>(base, stride, s, out);
  else
    load_site<S, N, R, false>(base, stride, s, out);
}

// Spinors: the chunk is 4 reals (Wilson, 24 reals per site) or 2 reals
// (staggered, 6) in every precision, so the k-th real of a packed spinor is
// the same spin-colour component at the same site whatever the precision and
// the level-1 kernels can convert and combine fields of different precision
// element by element.
template <int N> constexpr int spinor_chunk() { return N % 4 == 0 ? 4 : 2; }

// Fixed-point fields with a per-site norm: the FP32 norms of a block of
// `stride` sites follow its N * stride codes.
template <typename S, int N>
__device__ __forceinline__ const float *site_norms(const S *__restrict__ base, int64_t stride) {
  return reinterpret_cast<const float *>(base + N * stride);
}
template <typename S, int N> __device__ __forceinline__ float *site_norms(S *__restrict__ base, int64_t stride) {
  return reinterpret_cast<float *>(base + N * stride);
}
// The norm of a site and the codes' scale, in FP32: m = max_k |v_k|, then
// each value is stored as the code of (float)v_k * (1 / m).
template <int N, typename R> __device__ __forceinline__ float fixed_norm(const R *v) {
  R m = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) m = v[k] < 0 ? (-v[k] > m ? -v[k] : m) : (v[k] > m ? v[k] : m);
  return (float)m;
}
// The values a fixed-point store of v returns when read back.
template <int N, typename R> __device__ __forceinline__ void fixed_round(R *v) {
  const float m = fixed_norm<N, R>(v), inv = m > 0 ? 1.0f / m : 0.0f;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = (R)to_real<float>(Store<fx16>::from((float)v[k] * inv)) * (R)m;
}

template <typename S, int N, typename R>
__device__ __forceinline__ void load_spinor_reals(const S *__restrict__ base, int64_t stride, int64_t s, R *out) {
  load_chunks<S, N, spinor_chunk<N>(), R>(base, stride, s, out);
  if constexpr (is_fixed<S>()) {
    const R m = (R)site_norms<S, N>(base, stride)[s];
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] *= m;
  }
}
template <typename S, int N, typename R, bool NT = false>
__device__ __forceinline__ void store_spinor_reals(S *__restrict__ base, int64_t stride, int64_t s, const R *in) {
  if constexpr (is_fixed<S>()) {
    const float m = fixed_norm<N, R>(in), inv = m > 0 ? 1.0f / m : 0.0f;
    float w[N];
#pragma unroll
    for (int k = 0; k < N; ++k) w[k] = (float)in[k] * inv;
    store_chunks<S, N, spinor_chunk<N>(), float, NT>(base, stride, s, w);
    site_norms<S, N>(base, stride)[s] = m;
  } else {
    store_chunks<S, N, spinor_chunk<N>(), R, NT>(base, stride, s, in);
  }
}

// ---------------------------------------------------------------------------
// complex arithmetic

template <typename R> struct cpx {
  R re, im;
};
template <typename R> __device__ __forceinline__ cpx<R> mk(R a, R b) { return cpx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cpx<R> conj(cpx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R> __device__ __forceinline__ cpx<R> cmul_conj(cpx<R> a, cpx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename R> __device__ __forceinline__ cpx<R> times_i(cpx<R> a) { return {-a.im, a.re}; }
// acc += a * b
template <typename R> __device__ __forceinline__ void cmac(cpx<R> &acc, cpx<R> a, cpx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R> __device__ __forceinline__ void cmac_conj(cpx<R> &acc, cpx<R> a, cpx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}

// ---------------------------------------------------------------------------
// SU(3) link storage: 18 reals (row-major complex), 12 (first two rows; the
// third is conj(row0 x row1)) or 8 (U01, U02, U10, arg U00, arg U20; the rest
// follows from unitarity and det = 1).

template <typename R> struct Link {
  cpx<R> m[3][3];
};

template <typename R> __device__ __forceinline__ void third_row(Link<R> &u) {
  u.m[2][0] = conj(u.m[0][1] * u.m[1][2] - u.m[0][2] * u.m[1][1]);
  u.m[2][1] = conj(u.m[0][2] * u.m[1][0] - u.m[0][0] * u.m[1][2]);
  u.m[2][2] = conj(u.m[0][0] * u.m[1][1] - u.m[0][1] * u.m[1][0]);
}

__device__ __forceinline__ void sincos_r(double a, double *s, double *c) { sincos(a, s, c); }
// FP32: the hardware sine and cosine, which take the angle in revolutions (the
// stored angles lie in (-pi, pi], inside their domain); about 1e-6 absolute,
// below the FP32 storage rounding of the other link reals' products.
__device__ __forceinline__ void sincos_r(float a, float *s, float *c) {
  const float t = a * 0.159154943091895336f;  // 1 / (2 pi)
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}

template <int RECON, typename R> __device__ __forceinline__ Link<R> unpack_link(const R *v) {
  Link<R> u;
  if constexpr (RECON == 18) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) u.m[i][j] = mk<R>(v[6 * i + 2 * j], v[6 * i + 2 * j + 1]);
  } else if constexpr (RECON == 12) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) u.m[i][j] = mk<R>(v[6 * i + 2 * j], v[6 * i + 2 * j + 1]);
    third_row(u);
  } else {
    const cpx<R> a2 = mk<R>(v[0], v[1]), a3 = mk<R>(v[2], v[3]), b1 = mk<R>(v[4], v[5]);
    const R N = a2.re * a2.re + a2.im * a2.im + a3.re * a3.re + a3.im * a3.im;
    const R b1n = b1.re * b1.re + b1.im * b1.im;
    const R ra1 = sqrt(fmax(R(1) - N, R(0)));
    const R rc1 = sqrt(fmax(N - b1n, R(0)));
    R s0, c0, s2, c2;
    sincos_r(v[6], &s0, &c0);
    sincos_r(v[7], &s2, &c2);
    const cpx<R> a1 = mk<R>(ra1 * c0, ra1 * s0), c1 = mk<R>(rc1 * c2, rc1 * s2);
    const R inv = R(1) / N;
    const cpx<R> ca1 = conj(a1), ca2 = conj(a2), ca3 = conj(a3), cb1 = conj(b1), cc1 = conj(c1);
    u.m[0][0] = a1; u.m[0][1] = a2; u.m[0][2] = a3;
    u.m[1][0] = b1;
    u.m[2][0] = c1;
    u.m[1][1] = (-inv) * (ca3 * cc1 + ca1 * a2 * b1);
    u.m[1][2] = inv * (ca2 * cc1 - ca1 * a3 * b1);
    u.m[2][1] = inv * (cb1 * ca3 - ca1 * a2 * c1);
    u.m[2][2] = (-inv) * (ca2 * cb1 + ca1 * a3 * c1);
  }
  return u;
}

// out = U v  and  out = U^+ v
template <typename R> __device__ __forceinline__ void su3_mv(const Link<R> &u, const cpx<R> *v, cpx<R> *out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cpx<R> a = u.m[i][0] * v[0];
    cmac(a, u.m[i][1], v[1]);
    cmac(a, u.m[i][2], v[2]);
    out[i] = a;
  }
}
template <typename R> __device__ __forceinline__ void su3_adj_mv(const Link<R> &u, const cpx<R> *v, cpx<R> *out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cpx<R> a = cmul_conj(u.m[0][i], v[0]);
    cmac_conj(a, u.m[1][i], v[1]);
    cmac_conj(a, u.m[2][i], v[2]);
    out[i] = a;
  }
}

// ---------------------------------------------------------------------------
// magic-number division for 0 <= n < 2^31

struct FastDiv {
  uint32_t d;
  uint64_t m;
  uint32_t shift;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.shift = 31 + s;
  f.m = ((1ull << f.shift) + d - 1) / d;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
  return (uint32_t)(((uint64_t)n * f.m) >> f.shift);
}

// ---------------------------------------------------------------------------
// tiled even-odd geometry
//
// Sites of parity p are numbered s = tile * Vt2 + k, where tiles are taken in
// lexicographic order of their coordinates and k is the checkerboard index
// inside the tile: k = (lx >> 1) + (Bx/2) * (ly + By * (lz + Bz * lt)). With
// every tile extent even, a tile's origin is an even site, so the parity of a
// local coordinate equals the global parity.

struct Geom {
  int L[4];     // lattice extents
  int B[4];     // tile extents
  int NT[4];    // tiles per axis
  int Vh;       // sites per parity
  int Vt2;      // sites per parity in one tile
  int bc_t;     // +1 / -1
  int cut[4];   // Dirichlet block extents (== L[mu]: no cut along mu)
  int has_cut;  // any cut active
  int colour;   // -1: every tile; 0 / 1: only the tiles whose coordinates sum to
                // that parity (NT[0] even; the cut Schur pieces and the MR update)
  FastDiv dVt2, dBxh, dBy, dBz, dNTx, dNTy, dNTz, dNTxh;
  FastDiv dcut[4];
};

// Sites one launch covers: all of one parity, or those of one tile colour.
__host__ __device__ __forceinline__ int launch_sites(const Geom &g) { return g.colour < 0 ? g.Vh : g.Vh / 2; }

// Site of a colour-restricted launch. Launch index s < Vh/2 runs over the
// tiles of colour g.colour in order, Vt2 sites each. Along x the tiles
// alternate in colour (NT[0] even), so the j-th tile of the colour lies in
// x-row j / (NT[0]/2), at tile x coordinate 2 (j mod NT[0]/2) plus the parity
// that completes the row's coordinate sum to the colour.
__device__ __forceinline__ int colour_site(const Geom &g, int s) {
  const uint32_t j = fdiv((uint32_t)s, g.dVt2);
  const uint32_t k = (uint32_t)s - j * (uint32_t)g.Vt2;
  const uint32_t row = fdiv(j, g.dNTxh);
  const uint32_t jx = j - row * (uint32_t)(g.NT[0] >> 1);
  const uint32_t u = fdiv(row, g.dNTy);
  const uint32_t ty = row - u * (uint32_t)g.NT[1];
  const uint32_t tt = fdiv(u, g.dNTz);
  const uint32_t tz = u - tt * (uint32_t)g.NT[2];
  const uint32_t tx = 2 * jx + ((ty + tz + tt + (uint32_t)g.colour) & 1u);
  return (int)((tx + (uint32_t)g.NT[0] * row) * (uint32_t)g.Vt2 + k);
}

struct Site {
  int t[4];  // tile coordinate
  int l[4];  // coordinate inside the tile
  int p;     // parity
};

__device__ __forceinline__ Site decode_site(const Geom &g, int s, int parity) {
  Site r;
  r.p = parity;
  uint32_t tile = fdiv((uint32_t)s, g.dVt2);
  uint32_t k = (uint32_t)s - tile * (uint32_t)g.Vt2;
  uint32_t q = fdiv(k, g.dBxh);
  const int lxh = (int)(k - q * (uint32_t)(g.B[0] >> 1));
  uint32_t q2 = fdiv(q, g.dBy);
  r.l[1] = (int)(q - q2 * (uint32_t)g.B[1]);
  uint32_t q3 = fdiv(q2, g.dBz);
  r.l[2] = (int)(q2 - q3 * (uint32_t)g.B[2]);
  r.l[3] = (int)q3;
  r.l[0] = 2 * lxh + ((r.l[1] + r.l[2] + r.l[3] + parity) & 1);
  uint32_t u = fdiv(tile, g.dNTx);
  r.t[0] = (int)(tile - u * (uint32_t)g.NT[0]);
  uint32_t u2 = fdiv(u, g.dNTy);
  r.t[1] = (int)(u - u2 * (uint32_t)g.NT[1]);
  uint32_t u3 = fdiv(u2, g.dNTz);
  r.t[2] = (int)(u2 - u3 * (uint32_t)g.NT[2]);
  r.t[3] = (int)u3;
  return r;
}

__device__ __forceinline__ int encode_site(const Geom &g, const int t[4], const int l[4]) {
  const int tile = t[0] + g.NT[0] * (t[1] + g.NT[1] * (t[2] + g.NT[2] * t[3]));
  const int k = (l[0] >> 1) + (g.B[0] >> 1) * (l[1] + g.B[1] * (l[2] + g.B[2] * l[3]));
  return tile * g.Vt2 + k;
}

__device__ __forceinline__ int global_coord(const Geom &g, const Site &x, int mu) { return x.t[mu] * g.B[mu] + x.l[mu]; }

// Neighbour `step` hops along MU (|step| <= 3). Returns its site index;
// *wraps = number of times the hop crossed the lattice boundary along MU.
template <int MU>
__device__ __forceinline__ int hop(const Geom &g, const Site &x, int step, int *wraps) {
  int t[4] = {x.t[0], x.t[1], x.t[2], x.t[3]};
  int l[4] = {x.l[0], x.l[1], x.l[2], x.l[3]};
  int w = 0;
  l[MU] += step;
  while (l[MU] >= g.B[MU]) {
    l[MU] -= g.B[MU];
    if (++t[MU] == g.NT[MU]) { t[MU] = 0; ++w; }
  }
  while (l[MU] < 0) {
    l[MU] += g.B[MU];
    if (--t[MU] < 0) { t[MU] = g.NT[MU] - 1; ++w; }
  }
  *wraps = w;
  return encode_site(g, t, l);
}

// Neighbour one hop along MU (STEP = +1 or -1) without loops or branches: the
// hop crosses at most one tile face (tile extents are at least 2).
template <int MU, int STEP>
__device__ __forceinline__ int hop1(const Geom &g, const Site &x, int *wraps) {
  int t[4] = {x.t[0], x.t[1], x.t[2], x.t[3]};
  int l[4] = {x.l[0], x.l[1], x.l[2], x.l[3]};
  int lm = l[MU] + STEP, tm = t[MU];
  bool wrap;
  if constexpr (STEP > 0) {
    const bool cross = lm >= g.B[MU];
    lm = cross ? 0 : lm;
    tm = cross ? tm + 1 : tm;
    wrap = tm == g.NT[MU];
    tm = wrap ? 0 : tm;
  } else {
    const bool cross = lm < 0;
    lm = cross ? g.B[MU] - 1 : lm;
    tm = cross ? tm - 1 : tm;
    wrap = tm < 0;
    tm = wrap ? g.NT[MU] - 1 : tm;
  }
  l[MU] = lm;
  t[MU] = tm;
  *wraps = wrap ? 1 : 0;
  return encode_site(g, t, l);
}

// Neighbour STEP hops along MU (|STEP| <= 3) without loops or branches: with
// tile extents of at least 2 a hop crosses at most two tile faces, and it
// wraps the lattice at most twice (on a lattice of extent 2).
template <int MU, int STEP>
__device__ __forceinline__ int hopk(const Geom &g, const Site &x, int *wraps) {
  static_assert(STEP != 0 && STEP >= -3 && STEP <= 3, "hops of 1 to 3 sites");
  int t[4] = {x.t[0], x.t[1], x.t[2], x.t[3]};
  int l[4] = {x.l[0], x.l[1], x.l[2], x.l[3]};
  const int B = g.B[MU], NT = g.NT[MU];
  int lm = l[MU] + STEP, tm = t[MU], w;
  if constexpr (STEP > 0) {
    const int c = (lm >= B) + (lm >= 2 * B);  // tile faces crossed
    lm -= c * B;
    tm += c;
    w = (tm >= NT) + (tm >= 2 * NT);
    tm -= w * NT;
  } else {
    const int c = (lm < 0) + (lm < -B);
    lm += c * B;
    tm -= c;
    w = (tm < 0) + (tm < -NT);
    tm += w * NT;
  }
  l[MU] = lm;
  t[MU] = tm;
  *wraps = w;
  return encode_site(g, t, l);
}

// Dirichlet cut: is the hop of `step` (+1 or -1) along MU inside one block?
template <int MU>
__device__ __forceinline__ bool hop_kept(const Geom &g, const Site &x, int step) {
  if (!g.has_cut || g.cut[MU] >= g.L[MU]) return true;
  const int c = global_coord(g, x, MU);
  const uint32_t q = fdiv((uint32_t)c, g.dcut[MU]);
  const int r = c - (int)q * g.cut[MU];
  return step > 0 ? (r != g.cut[MU] - 1) : (r != 0);
}

// Map the hardware workgroup id to a logical one so that each XCD (the
// dispatcher deals workgroups round-robin over 8 XCDs) owns a contiguous range
// of sites and their neighbours stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
  constexpr int NXCD = 8;
  if (nwg % NXCD) return wg;
  return (wg % NXCD) * (nwg / NXCD) + wg / NXCD;
}

// Fields of several right-hand sides are stored in blocks of R sources
// (R = 4, 2 or 1: the largest of these dividing nrhs): within a parity block
// the packed index of (site s, source r) is ((r / R) Vh + s) R + r % R, so the
// R sources of a site are adjacent (the lanes of a wave that share a site
// share its link loads) and each group of R sources is one contiguous field
// (neighbour accesses keep the locality of a single field). R = 1 for one
// source is the plain layout.
__host__ __device__ __forceinline__ int rhs_group(int nrhs) { return (nrhs & 3) == 0 ? 4 : ((nrhs & 1) == 0 ? 2 : 1); }
__device__ __forceinline__ int64_t rhs_index(int rhs, int64_t s, int64_t vh, int R) {
  return ((int64_t)(rhs / R) * vh + s) * R + (rhs & (R - 1));
}

// A launch covers ceil(Vh / (blockDim / R)) site blocks x (nrhs / R) source
// groups, source group fastest after the XCD remap: the workgroups of one site
// block run together on one XCD and read its links and clover terms from that
// XCD's L2 rather than from memory. Lane l takes site s0 + l / R and source
// R * group + l % R.
struct RhsBlock {
  int rhs;  // source of this lane
  int s;    // site of this lane
};
__device__ __forceinline__ RhsBlock rhs_block_at(int w, int nrhs, int R) {
  const int ng = nrhs / R, spb = blockDim.x / R;
  return RhsBlock{R * (w % ng) + (int)(threadIdx.x & (R - 1)), (w / ng) * spb + (int)(threadIdx.x / R)};
}
__device__ __forceinline__ RhsBlock rhs_block(int nrhs, int R) {
  return rhs_block_at(xcd_remap(blockIdx.x, gridDim.x), nrhs, R);
}
inline int rhs_grid(int vh, int nrhs, int block_threads) {
  const int R = rhs_group(nrhs), spb = block_threads / R;
  return ((vh + spb - 1) / spb) * (nrhs / R);
}

// v_mfma_f32_4x4x4_16b_{f16,bf16}: 16 independent 4x4x4 products per
// instruction, FP32 accumulation. Block b is lanes 4b .. 4b+3; lane j of a
// block supplies row j of its A (4 K values), column j of its B (4 K values)
// and receives column j of D (4 rows). A complex 3x3 matrix U times a colour
// vector v runs in real form on two M blocks x two K steps: rows and K both
// run (c0 re, c0 im, c1 re, c1 im | c2 re, c2 im, 0, 0), the A rows being
// (Re u, -Im u) for a real row and (Im u, Re u) for an imaginary row.
typedef _Float16 mf_h4 __attribute__((ext_vector_type(4)));
typedef short mf_s4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename S> struct Mf4;
template <> struct Mf4<_Float16> {
  typedef mf_h4 T;
  __device__ __forceinline__ static T pack(float a, float b, float c, float d) {
    return T{(_Float16)a, (_Float16)b, (_Float16)c, (_Float16)d};
  }
  __device__ __forceinline__ static mf_f4 mma(T a, T b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mf4<bf16> {
  typedef mf_s4 T;
  // hardware round-to-nearest-even (v_cvt_pk_bf16_f32): for finite values
  // the same result as Store<bf16>::from
  __device__ __forceinline__ static T pack(float a, float b, float c, float d) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef __bf16 b4 __attribute__((ext_vector_type(4)));
    return __builtin_bit_cast(T, __builtin_convertvector(f4{a, b, c, d}, b4));
  }
  __device__ __forceinline__ static mf_f4 mma(T a, T b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
  }
};

// A operands [M block][K step] of row j (0..3) of U (ADJ: of U^+).
template <typename S, bool ADJ>
__device__ __forceinline__ void mf_link_rows(const Link<float> &U, int j, typename Mf4<S>::T (&a)[2][2]) {
  using M = Mf4<S>;
  cpx<float> r0[3], r2[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cpx<float> e0 = ADJ ? conj(U.m[c][0]) : U.m[0][c];
    const cpx<float> e1 = ADJ ? conj(U.m[c][1]) : U.m[1][c];
    r0[c] = (j >> 1) ? e1 : e0;  // M block 0: colour j / 2
    r2[c] = ADJ ? conj(U.m[c][2]) : U.m[2][c];
  }
  // row (colour, re) = (Re e_c, -Im e_c)_c; row (colour, im) = (Im e_c, Re e_c)_c
  const bool im0 = j & 1;
  a[0][0] = im0 ? M::pack(r0[0].im, r0[0].re, r0[1].im, r0[1].re) : M::pack(r0[0].re, -r0[0].im, r0[1].re, -r0[1].im);
  a[0][1] = im0 ? M::pack(r0[2].im, r0[2].re, 0.f, 0.f) : M::pack(r0[2].re, -r0[2].im, 0.f, 0.f);
  // M block 1: rows (c2 re, c2 im, 0, 0)
  const float z = j < 2 ? 1.f : 0.f;
  a[1][0] = (j == 1) ? M::pack(r2[0].im, r2[0].re, r2[1].im, r2[1].re)
                     : M::pack(z * r2[0].re, -z * r2[0].im, z * r2[1].re, -z * r2[1].im);
  a[1][1] = (j == 1) ? M::pack(r2[2].im, r2[2].re, 0.f, 0.f) : M::pack(z * r2[2].re, -z * r2[2].im, 0.f, 0.f);
}

}  // namespace lqcd
