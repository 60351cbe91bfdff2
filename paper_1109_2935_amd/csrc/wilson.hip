// Wilson-clover operator kernels for gfx950 (eq. (2) of the paper, kappa
// normalisation M = A - kappa D).
//
// One thread per output site of one parity. For each of the 8 hops the
// neighbour spinor is spin-projected to a half spinor (2 colour vectors) with
// (1 -/+ gamma_mu) before the SU(3) multiply, and the product is expanded back
// to 4 spins; the boundary phase and the Dirichlet cut are applied in-kernel.
// Epilogues fuse the clover term (A or A^-1), an xpay and, for the Schwarz
// block solver, per-workgroup partial inner products.
#include <type_traits>

#include "lqcd_internal.h"

namespace lqcd {

// ---------------------------------------------------------------------------
// spin projection in the chiral basis.
// For P = 1 + g gamma_mu (g = +-1) the result has rows 2,3 proportional to
// rows 0,1, so only h0 = row 0 and h1 = row 1 are formed:
//   x: h0 = s0 - g i s3, h1 = s1 - g i s2;  rows 2,3 = ( g i h1,  g i h0)
//   y: h0 = s0 - g s3,   h1 = s1 + g s2;    rows 2,3 = ( g h1,   -g h0)
//   z: h0 = s0 - g i s2, h1 = s1 + g i s3;  rows 2,3 = ( g i h0, -g i h1)
//   t: h0 = s0 + g s2,   h1 = s1 + g s3;    rows 2,3 = ( g h0,    g h1)

template <int MU, typename R>
__device__ __forceinline__ void project(const cpx<R> (&s)[4][3], R g, cpx<R> (&h)[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (MU == 0) {
      h[0][c] = s[0][c] - g * times_i(s[3][c]);
      h[1][c] = s[1][c] - g * times_i(s[2][c]);
    } else if constexpr (MU == 1) {
      h[0][c] = s[0][c] - g * s[3][c];
      h[1][c] = s[1][c] + g * s[2][c];
    } else if constexpr (MU == 2) {
      h[0][c] = s[0][c] - g * times_i(s[2][c]);
      h[1][c] = s[1][c] + g * times_i(s[3][c]);
    } else {
      h[0][c] = s[0][c] + g * s[2][c];
      h[1][c] = s[1][c] + g * s[3][c];
    }
  }
}

template <int MU, typename R>
__device__ __forceinline__ void expand_acc(cpx<R> (&acc)[4][3], const cpx<R> (&u)[2][3], R g) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] = acc[0][c] + u[0][c];
    acc[1][c] = acc[1][c] + u[1][c];
    if constexpr (MU == 0) {
      acc[2][c] = acc[2][c] + g * times_i(u[1][c]);
      acc[3][c] = acc[3][c] + g * times_i(u[0][c]);
    } else if constexpr (MU == 1) {
      acc[2][c] = acc[2][c] + g * u[1][c];
      acc[3][c] = acc[3][c] - g * u[0][c];
    } else if constexpr (MU == 2) {
      acc[2][c] = acc[2][c] + g * times_i(u[0][c]);
      acc[3][c] = acc[3][c] - g * times_i(u[1][c]);
    } else {
      acc[2][c] = acc[2][c] + g * u[0][c];
      acc[3][c] = acc[3][c] + g * u[1][c];
    }
  }
}

// ---------------------------------------------------------------------------
// FP16 storage: a hop in packed half arithmetic. The spin projection runs on
// packed FP16 pairs (each component of h rounded once to FP16; the sign flips
// and factors i are exact) and the colour products U h on v_dot2_f32_f16
// (products of two FP16 values are exact in FP32, sums in FP32). With 12
// stored link reals the third row is rebuilt in FP32 from the same dot2 sums
// and multiplied in FP32. Against the FP32-arithmetic hop this removes the 36
// half-to-float conversions of a hop and halves its colour-product
// instructions; the one new rounding (of h) is a quarter of the storage
// rounding already in the input.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2v h2_times_i(h2v a) { return h2v{-a.y, a.x}; }
__device__ __forceinline__ float dot2(h2v a, h2v b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }

template <int MU>
__device__ __forceinline__ void project_h2(const h2v (&s)[4][3], h2v g, h2v (&h)[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (MU == 0) {
      h[0][c] = s[0][c] - g * h2_times_i(s[3][c]);
      h[1][c] = s[1][c] - g * h2_times_i(s[2][c]);
    } else if constexpr (MU == 1) {
      h[0][c] = s[0][c] - g * s[3][c];
      h[1][c] = s[1][c] + g * s[2][c];
    } else if constexpr (MU == 2) {
      h[0][c] = s[0][c] - g * h2_times_i(s[2][c]);
      h[1][c] = s[1][c] + g * h2_times_i(s[3][c]);
    } else {
      h[0][c] = s[0][c] + g * s[2][c];
      h[1][c] = s[1][c] + g * s[3][c];
    }
  }
}

// u_k = U h_k (FWD) or U^+ h_k for both half-spinor rows k; U as stored: rows
// 0 and 1 (and 2 with 18 reals) as packed (re, im) pairs, row-major.
template <int RECON, bool FWD>
__device__ __forceinline__ void su3_h2(const h2v (&U)[RECON / 2], const h2v (&h)[2][3], cpx<float> (&u)[2][3]) {
  static_assert(RECON == 12 || RECON == 18, "16-bit links hold 12 or 18 reals");
  // conj-swapped forms of h: Re(a b) = dot2(a, hc), Im(a b) = dot2(a, hs);
  // Re(conj(a) b) = dot2(a, b), Im(conj(a) b) = dot2(a, ha)
  h2v hx[2][3], hy[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      hx[k][c] = FWD ? h2v{h[k][c].x, -h[k][c].y} : h[k][c];
      hy[k][c] = FWD ? h2v{h[k][c].y, h[k][c].x} : h2v{h[k][c].y, -h[k][c].x};
    }
  constexpr int NR = RECON == 18 ? 3 : 2;  // rows taken from storage
  // forward: output rows i < NR over all columns j; adjoint: all outputs i
  // over the stored rows j < NR
  constexpr int NI = FWD ? NR : 3, NJ = FWD ? 3 : NR;
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        // forward: row i of U, column j of h; adjoint: column i of U (row j)
        const h2v a = FWD ? U[3 * i + j] : U[3 * j + i];
        re = dot2(a, hx[k][j], re);
        im = dot2(a, hy[k][j], im);
      }
      u[k][i] = mk<float>(re, im);
    }
  if constexpr (RECON == 12) {
    // third row conj(row0 x row1) in FP32: U2j = conj(U0k U1l - U0l U1k)
    cpx<float> r2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int k = (j + 1) % 3, l = (j + 2) % 3;
      const h2v a = U[k], b = U[3 + l], c = U[l], d = U[3 + k];
      const float re = dot2(a, h2v{b.x, -b.y}, dot2(-c, h2v{d.x, -d.y}, 0.f));
      const float im = dot2(c, h2v{d.y, d.x}, dot2(-a, h2v{b.y, b.x}, 0.f));
      r2[j] = mk<float>(re, im);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cpx<float> hf[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) hf[j] = mk<float>((float)h[k][j].x, (float)h[k][j].y);
      if constexpr (FWD) {
        cpx<float> a = r2[0] * hf[0];
        cmac(a, r2[1], hf[1]);
        cmac(a, r2[2], hf[2]);
        u[k][2] = a;
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) cmac_conj(u[k][i], r2[i], hf[2]);
      }
    }
  }
}

// One FP16 hop from stored values: psi the neighbour's 24 halves, link its
// RECON halves, ps the projection sign (+-1); u as su3_h2.
template <int MU, int DIR, int RECON>
__device__ __forceinline__ void hop_h2(const uint32_t (&psi)[12], const uint32_t (&link)[RECON / 2], float ps,
                                       cpx<float> (&u)[2][3]) {
  h2v s[4][3], hh[2][3], U[RECON / 2];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[sp][c] = __builtin_bit_cast(h2v, psi[3 * sp + c]);
#pragma unroll
  for (int k = 0; k < RECON / 2; ++k) U[k] = __builtin_bit_cast(h2v, link[k]);
  const _Float16 g16 = (_Float16)ps;
  project_h2<MU>(s, h2v{g16, g16}, hh);
  su3_h2<RECON, (DIR > 0)>(U, hh, u);
}

template <typename S, typename R>
__device__ __forceinline__ void load_spinor(const S *__restrict__ f, int64_t vh, int s, cpx<R> (&v)[4][3]) {
  R r[24];
  load_spinor_reals<S, 24, R>(f, vh, s, r);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[sp][c] = mk<R>(r[6 * sp + 2 * c], r[6 * sp + 2 * c + 1]);
}

template <typename S, typename R, bool NT = false>
__device__ __forceinline__ void store_spinor(S *__restrict__ f, int64_t vh, int s, const cpx<R> (&v)[4][3]) {
  R r[24];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[6 * sp + 2 * c] = v[sp][c].re;
      r[6 * sp + 2 * c + 1] = v[sp][c].im;
    }
  store_spinor_reals<S, 24, R, NT>(f, vh, s, r);
}

// Round to the storage precision and back (what a store followed by a load returns).
template <typename S, typename R> __device__ __forceinline__ R quantize(R v) { return to_real<R>(Store<S>::from(v)); }

// stream: the link is read once per launch (one right-hand side)
template <typename S, typename R, int RECON>
__device__ __forceinline__ Link<R> load_link(const S *__restrict__ gauge, int64_t vh, int mu, int parity, int s,
                                             bool stream) {
  R v[RECON];
  load_site_once<S, RECON, R>(gauge + (int64_t)(2 * mu + parity) * vh * RECON, vh, s, v, stream);
  return unpack_link<RECON, R>(v);
}

// Clover: per site and chirality block a Hermitian 6x6 (index = spin-in-block*3
// + colour): 6 real diagonal entries, then the strictly lower triangle in row
// order as (re, im); block 0 = spins 0,1, block 1 = spins 2,3 (72 reals).
template <typename S, typename R>
__device__ __forceinline__ void clover_mul(const S *__restrict__ clov, int64_t vh, int s, const cpx<R> (&in)[4][3],
                                           cpx<R> (&out)[4][3], bool stream) {
  R a[72];
  load_site_once<S, 72, R>(clov, vh, s, a, stream);
  if constexpr (is_fixed<S>()) {
    const R m = (R)site_norms<S, 72>(clov, vh)[s];
#pragma unroll
    for (int k = 0; k < 72; ++k) a[k] *= m;
  }
  if constexpr (is_float16<S>()) {
    // converted here, as in the hops: kept from folding into mixed-precision FMAs
#pragma unroll
    for (int k = 0; k < 72; ++k) __asm__ volatile("" : "+v"(a[k]));
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const R *A = a + 36 * b;
    cpx<R> x[6], y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] = in[2 * b + i / 3][i % 3];
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] = A[i] * x[i];
    int off = 6;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) {
        const cpx<R> aij = mk<R>(A[off], A[off + 1]);
        off += 2;
        cmac(y[i], aij, x[j]);
        cmac_conj(y[j], aij, x[i]);
      }
#pragma unroll
    for (int i = 0; i < 6; ++i) out[2 * b + i / 3][i % 3] = y[i];
  }
}

template <typename S> struct WArgs {
  Geom g;
  S *out;
  const S *in;
  const S *gauge;
  const S *clov;
  const S *xin;
  double *partials;
  double coef;
  int parity;
  int dagger;
  int nrhs;  // right-hand sides
  int rg;    // sources per block of the multi-source layout (rhs_group(nrhs))
};

// Software-pipelined hops for launches without a cut (FP32 and 16-bit
// storage): the raw inputs of a hop (neighbour spinor, link as stored, wrap
// count) go to one of two buffers, refilled alternately, so each wave keeps
// the loads of the next hop in flight while it multiplies the current one.
// Scheduling barriers hold that order
// (without them the compiler issues the loads of all eight hops first and
// spills).
// The raw values stay in the storage type until they are used, so that no
// conversion forces an early wait for the loads.
template <typename S, int RECON> struct HopIn {
  S psi[24];
  S link[RECON];
  int w;
};

template <int MU, int DIR, bool STREAM, typename S, int RECON>
__device__ __forceinline__ void hop_fetch(const WArgs<S> &a, const Site &x, int s, int rhs, HopIn<S, RECON> &h) {
  const int64_t vh = a.g.Vh, vs = vh * a.nrhs;
  const int n = hop1<MU, DIR>(a.g, x, &h.w);
  load_chunks_raw<S, 24, spinor_chunk<24>()>(a.in, vs, rhs_index(rhs, n, vh, a.rg), h.psi);
  // forward hop: U_mu(x) of x's parity; backward: U_mu(x - mu) of the other
  const int lp = DIR > 0 ? x.p : 1 - x.p, ls = DIR > 0 ? s : n;
  load_chunks_raw<S, RECON, chunk_reals<S, RECON>(), STREAM>(a.gauge + (int64_t)(2 * MU + lp) * vh * RECON, vh, ls,
                                                           h.link);
}

// FP16 storage takes the packed-half hop (hop_h2) with 12 or 18 link reals.
template <typename S, int RECON> constexpr bool half_hop() {
  return std::is_same<S, _Float16>::value && (RECON == 12 || RECON == 18);
}

template <int MU, int DIR, typename S, typename R, int RECON>
__device__ __forceinline__ void hop_apply(const HopIn<S, RECON> &h, R sgn, int bc_t, cpx<R> (&acc)[4][3]) {
  const R ps = DIR > 0 ? -sgn : sgn;
  cpx<R> u[2][3];
  if constexpr (half_hop<S, RECON>()) {
    uint32_t pw[12], lw[RECON / 2];
#pragma unroll
    for (int j = 0; j < 12; ++j) pw[j] = __builtin_bit_cast(uint32_t, h2v{h.psi[2 * j], h.psi[2 * j + 1]});
#pragma unroll
    for (int j = 0; j < RECON / 2; ++j) lw[j] = __builtin_bit_cast(uint32_t, h2v{h.link[2 * j], h.link[2 * j + 1]});
    hop_h2<MU, DIR, RECON>(pw, lw, ps, u);
  } else {
    cpx<R> psi[4][3], hh[2][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R re = to_real<R>(h.psi[6 * sp + 2 * c]), im = to_real<R>(h.psi[6 * sp + 2 * c + 1]);
        if constexpr (is_float16<S>()) {
          // convert here: the empty asm keeps the compiler from folding the
          // stored halves into mixed-precision FMAs, which keeps them live
          // across the hop (170-230 VGPRs instead of about 110)
          __asm__ volatile("" : "+v"(re));
          __asm__ volatile("" : "+v"(im));
        }
        psi[sp][c] = mk<R>(re, im);
      }
    project<MU, R>(psi, ps, hh);
    R lv[RECON];
#pragma unroll
    for (int k = 0; k < RECON; ++k) {
      lv[k] = to_real<R>(h.link[k]);
      if constexpr (is_float16<S>()) __asm__ volatile("" : "+v"(lv[k]));
    }
    const Link<R> U = unpack_link<RECON, R>(lv);
    if constexpr (DIR > 0) {
      su3_mv(U, hh[0], u[0]);
      su3_mv(U, hh[1], u[1]);
    } else {
      su3_adj_mv(U, hh[0], u[0]);
      su3_adj_mv(U, hh[1], u[1]);
    }
  }
  if constexpr (MU == 3) {
    const R ph = ((h.w & 1) && bc_t < 0) ? R(-1) : R(1);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) u[k][c] = ph * u[k][c];
  }
  expand_acc<MU, R>(acc, u, ps);
}

// One direction of the hopping term, each hop checked against the cut.
template <int MU, typename S, typename R, int RECON>
__device__ __forceinline__ void wilson_dir(const WArgs<S> &a, const Site &x, int s, int rhs, R sgn,
                                           cpx<R> (&acc)[4][3]) {
  if constexpr (half_hop<S, RECON>()) {
    // raw loads and the packed-half hop, as in the pipelined form
    HopIn<S, RECON> h;
    if (hop_kept<MU>(a.g, x, +1)) {
      if (a.nrhs == 1)
        hop_fetch<MU, +1, true, S, RECON>(a, x, s, rhs, h);
      else
        hop_fetch<MU, +1, false, S, RECON>(a, x, s, rhs, h);
      hop_apply<MU, +1, S, R, RECON>(h, sgn, a.g.bc_t, acc);
    }
    if (hop_kept<MU>(a.g, x, -1)) {
      if (a.nrhs == 1)
        hop_fetch<MU, -1, true, S, RECON>(a, x, s, rhs, h);
      else
        hop_fetch<MU, -1, false, S, RECON>(a, x, s, rhs, h);
      hop_apply<MU, -1, S, R, RECON>(h, sgn, a.g.bc_t, acc);
    }
    return;
  }
  const int64_t vh = a.g.Vh, vs = vh * a.nrhs;
  // forward: (1 - sgn gamma_mu) U_mu(x) psi(x+mu)
  if (hop_kept<MU>(a.g, x, +1)) {
    int w;
    const int n = hop1<MU, +1>(a.g, x, &w);
    cpx<R> psi[4][3], h[2][3], u[2][3];
    load_spinor<S, R>(a.in, vs, rhs_index(rhs, n, vh, a.rg), psi);
    project<MU, R>(psi, -sgn, h);
    const Link<R> U = load_link<S, R, RECON>(a.gauge, vh, MU, x.p, s, a.nrhs == 1);
    su3_mv(U, h[0], u[0]);
    su3_mv(U, h[1], u[1]);
    if constexpr (MU == 3) {
      const R ph = ((w & 1) && a.g.bc_t < 0) ? R(-1) : R(1);
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) u[k][c] = ph * u[k][c];
    }
    expand_acc<MU, R>(acc, u, -sgn);
  }
  // backward: (1 + sgn gamma_mu) U_mu(x-mu)^+ psi(x-mu)
  if (hop_kept<MU>(a.g, x, -1)) {
    int w;
    const int n = hop1<MU, -1>(a.g, x, &w);
    cpx<R> psi[4][3], h[2][3], u[2][3];
    load_spinor<S, R>(a.in, vs, rhs_index(rhs, n, vh, a.rg), psi);
    project<MU, R>(psi, sgn, h);
    const Link<R> U = load_link<S, R, RECON>(a.gauge, vh, MU, 1 - x.p, n, a.nrhs == 1);
    su3_adj_mv(U, h[0], u[0]);
    su3_adj_mv(U, h[1], u[1]);
    if constexpr (MU == 3) {
      const R ph = ((w & 1) && a.g.bc_t < 0) ? R(-1) : R(1);
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) u[k][c] = ph * u[k][c];
    }
    expand_acc<MU, R>(acc, u, sgn);
  }
}

// Where the pipelined hops pay (measured at 32^3x64): FP32 storage with 18,
// 12 or 8 link reals (8: since the rebuild takes the hardware sine and cosine,
// 110.5 -> 105.8 us), 16-bit storage with 12 or 18, and the FP64 hopping term
// with 12 (257 -> 222 us). FP64 Schur kernels and the FP64 recon-18 hop spill
// with them, and the 16-bit xpay-only kernel (W_XPAY) spills.
template <typename S, int RECON, int MODE> constexpr bool pipelined_hops() {
  if constexpr (std::is_same<S, double>::value) return MODE == W_HOP && RECON == 12;
  if constexpr (is_fixed<S>()) return false;  // the neighbour's norm is read with its codes
  if constexpr (sizeof(S) == 4) return true;
  return RECON != 8 && MODE != W_XPAY;
}

// Apply the hop held in HA, then refill HA with the hop two ahead; the other
// buffer's loads stay in flight meanwhile.
#define HOP_STEP(MUa, DIRa, HA, MUn, DIRn)                      \
  __builtin_amdgcn_sched_barrier(0);                           \
  hop_apply<MUa, DIRa, S, R, RECON>(HA, sgn, a.g.bc_t, acc);   \
  __builtin_amdgcn_sched_barrier(0);                           \
  hop_fetch<MUn, DIRn, STREAM, S, RECON>(a, x, s, rhs, HA);

template <bool STREAM, typename S, typename R, int RECON>
__device__ __forceinline__ void wilson_hops_pipelined(const WArgs<S> &a, const Site &x, int s, int rhs, R sgn,
                                                      cpx<R> (&acc)[4][3]) {
  HopIn<S, RECON> A, B;
  hop_fetch<0, +1, STREAM, S, RECON>(a, x, s, rhs, A);
  hop_fetch<0, -1, STREAM, S, RECON>(a, x, s, rhs, B);
  HOP_STEP(0, +1, A, 1, +1)
  HOP_STEP(0, -1, B, 1, -1)
  HOP_STEP(1, +1, A, 2, +1)
  HOP_STEP(1, -1, B, 2, -1)
  HOP_STEP(2, +1, A, 3, +1)
  HOP_STEP(2, -1, B, 3, -1)
  __builtin_amdgcn_sched_barrier(0);
  hop_apply<3, +1, S, R, RECON>(A, sgn, a.g.bc_t, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_apply<3, -1, S, R, RECON>(B, sgn, a.g.bc_t, acc);
  __builtin_amdgcn_sched_barrier(0);
}
#undef HOP_STEP

// ---------------------------------------------------------------------------
// Link products of several right-hand sides on the matrix cores (16-bit
// storage). With N sources per site the products of one hop are
// U [3 x 2N] (3 colours x (2 half-spinor rows x N sources)), in real form
// [[Ur, -Ui], [Ui, Ur]] (6 x 6) times (h_re; h_im) (6 x 2N). They run on
// v_mfma_f32_4x4x4_16b_{f16,bf16}: 16 independent 4x4x4 products per
// instruction, FP32 accumulation. A block is one site and 4 of its sources
// (lanes 4b .. 4b+3): lane j supplies row j of the link (A operand) and the
// half spinor of its own source (B column j), and receives U h for its own
// source (D column j). Rows and K both run (c0 re, c0 im, c1 re, c1 im | c2 re,
// c2 im, 0, 0): 2 M blocks x 2 K steps x 2 half-spinor rows = 8 instructions
// per hop. Link and half-spinor entries are rounded to the storage format
// (a reconstructed third row and the projection sums are the only new
// roundings), products are exact and sums are FP32.

template <typename S>
__device__ __forceinline__ void mf_mul(const typename Mf4<S>::T (&a)[2][2], const cpx<float> (&h)[2][3],
                                       cpx<float> (&u)[2][3]) {
  using M = Mf4<S>;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const typename M::T b0 = M::pack(h[k][0].re, h[k][0].im, h[k][1].re, h[k][1].im);
    const typename M::T b1 = M::pack(h[k][2].re, h[k][2].im, 0.f, 0.f);
    mf_f4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
    d0 = M::mma(a[0][0], b0, d0);
    d0 = M::mma(a[0][1], b1, d0);
    d1 = M::mma(a[1][0], b0, d1);
    d1 = M::mma(a[1][1], b1, d1);
    u[k][0] = mk<float>(d0[0], d0[1]);
    u[k][1] = mk<float>(d0[2], d0[3]);
    u[k][2] = mk<float>(d1[0], d1[1]);
  }
}

// Both hops of direction MU for (site s, source rhs) with the link products on
// the matrix cores. Every lane takes part in the products (a lane without a
// contribution supplies zeros), so there is no divergence around them.
template <int MU, typename S, int RECON>
__device__ __forceinline__ void wilson_dir_mf(const WArgs<S> &a, const Site &x, int s, int rhs, bool valid, float sgn,
                                              cpx<float> (&acc)[4][3]) {
  const int64_t vh = a.g.Vh, vs = vh * a.nrhs;
  const int j = threadIdx.x & 3;
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const int step = dir == 0 ? 1 : -1;
    const float g = dir == 0 ? -sgn : sgn;
    const bool kept = valid && hop_kept<MU>(a.g, x, step);
    int w = 0;
    cpx<float> h[2][3];
    Link<float> U;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) U.m[r][c] = mk<float>(0, 0);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) h[k][c] = mk<float>(0, 0);
    if (kept) {
      const int n = hop<MU>(a.g, x, step, &w);
      cpx<float> psi[4][3];
      load_spinor<S, float>(a.in, vs, rhs_index(rhs, n, vh, a.rg), psi);
      project<MU, float>(psi, g, h);
      U = dir == 0 ? load_link<S, float, RECON>(a.gauge, vh, MU, x.p, s, false)
                   : load_link<S, float, RECON>(a.gauge, vh, MU, 1 - x.p, n, false);
    }
    typename Mf4<S>::T A[2][2];
    if (dir == 0)
      mf_link_rows<S, false>(U, j, A);
    else
      mf_link_rows<S, true>(U, j, A);
    cpx<float> u[2][3];
    mf_mul<S>(A, h, u);
    if (MU == 3 && (w & 1) && a.g.bc_t < 0) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) u[k][c] = -1.f * u[k][c];
    }
    if (dir == 0)
      expand_acc<MU, float>(acc, u, -sgn);
    else
      expand_acc<MU, float>(acc, u, sgn);
  }
}

// Per-segment sums of 3 values for the Schwarz block solver. A segment is
// seg = min(sites per tile and parity, 64) consecutive sites (a power of two:
// the tile's site count divides 64 or is a multiple of it), so a segment never
// spans two waves and the layout of the partials does not depend on the
// workgroup size. Segment j covers sites [j*seg, (j+1)*seg); its sums go to
// dst[3*j .. 3*j+2].
__device__ __forceinline__ void segment_reduce_store(double (&v)[3], int seg, int site, int vh, double *dst) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (int off = seg >> 1; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  if ((site & (seg - 1)) == 0 && site < vh)
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[3 * (site / seg) + k] = v[k];
}

// How a launch takes its hops: checked one by one at run time (any cut), or
// pipelined (no cut). A pipelined form for cuts at the tile faces (the dropped
// hop loaded like any other and zeroed by a select) measured 2.5% slower in
// the Schwarz preconditioner than the checked form, which skips the dropped
// hops' loads, and is not kept.
enum HopForm { kHopsChecked = 0, kHopsPipe = 1 };

// One output (site s, right-hand side rhs) of the hopping term and its epilogue.
// MF: link products on the matrix cores (16-bit storage, sources in groups of
// 4 lanes); then every lane of the wave calls this, `valid` marks real work.
template <typename S, typename R, int RECON, int MODE, bool REDUCE, bool MF = false, int HOPS = kHopsChecked>
__device__ __forceinline__ void wilson_point(const WArgs<S> &a, int s, int rhs, double (&red)[3], bool valid = true) {
  const Site x = decode_site(a.g, s, a.parity);
  const R sgn = a.dagger ? R(-1) : R(1);
  cpx<R> acc[4][3];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[i][c] = mk<R>(0, 0);
  if constexpr (MF) {
    wilson_dir_mf<0, S, RECON>(a, x, s, rhs, valid, sgn, acc);
    wilson_dir_mf<1, S, RECON>(a, x, s, rhs, valid, sgn, acc);
    wilson_dir_mf<2, S, RECON>(a, x, s, rhs, valid, sgn, acc);
    wilson_dir_mf<3, S, RECON>(a, x, s, rhs, valid, sgn, acc);
    if (!valid) return;
  } else {
    if constexpr (HOPS != kHopsChecked) {
      // One instantiation for every source count (streamed link loads), so a
      // site's arithmetic, and its rounding, does not depend on nrhs. The
      // branch between two calls of it is deliberate: as one basic block with
      // the epilogue, the clover kernels spill (measured: 700-900 bytes per
      // lane); split like this they need 137-158 VGPRs and no scratch.
      if (a.nrhs == 1)
        wilson_hops_pipelined<true, S, R, RECON>(a, x, s, rhs, sgn, acc);
      else
        wilson_hops_pipelined<true, S, R, RECON>(a, x, s, rhs, sgn, acc);
    } else {
      wilson_dir<0, S, R, RECON>(a, x, s, rhs, sgn, acc);
      wilson_dir<1, S, R, RECON>(a, x, s, rhs, sgn, acc);
      wilson_dir<2, S, R, RECON>(a, x, s, rhs, sgn, acc);
      wilson_dir<3, S, R, RECON>(a, x, s, rhs, sgn, acc);
    }
  }
  // the epilogue's loads (xin, clover) are not hoisted into the hop pipeline,
  // where they would hold registers through all eight hops
  if constexpr (HOPS != kHopsChecked) __builtin_amdgcn_sched_barrier(0);
  const R coef = (R)a.coef;
  const int64_t vh = a.g.Vh, vs = vh * a.nrhs, v = rhs_index(rhs, s, vh, a.rg);
  cpx<R> res[4][3];
  if constexpr (MODE == W_HOP) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) res[i][c] = coef * acc[i][c];
  } else if constexpr (MODE == W_HOP_CLOV) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[i][c] = coef * acc[i][c];
    clover_mul<S, R>(a.clov, vh, s, acc, res, a.nrhs == 1);
  } else {
    cpx<R> xv[4][3];
    load_spinor<S, R>(a.xin, vs, v, xv);
    if constexpr (is_float16<S>()) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          __asm__ volatile("" : "+v"(xv[i][c].re));
          __asm__ volatile("" : "+v"(xv[i][c].im));
        }
    }
    if constexpr (MODE == W_XPAY_CLOV) {
      clover_mul<S, R>(a.clov, vh, s, xv, res, a.nrhs == 1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) res[i][c] = res[i][c] + coef * acc[i][c];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) res[i][c] = xv[i][c] + coef * acc[i][c];
    }
    if constexpr (REDUCE) {
      // inner products of the values as stored
      R fx[24];
      if constexpr (is_fixed<S>()) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            fx[6 * i + 2 * c] = res[i][c].re;
            fx[6 * i + 2 * c + 1] = res[i][c].im;
          }
        fixed_round<24, R>(fx);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double qr, qi;
          if constexpr (is_fixed<S>()) {
            qr = fx[6 * i + 2 * c];
            qi = fx[6 * i + 2 * c + 1];
          } else {
            qr = quantize<S, R>(res[i][c].re);
            qi = quantize<S, R>(res[i][c].im);
          }
          const double rr = xv[i][c].re, ri = xv[i][c].im;
          red[0] += qr * rr + qi * ri;
          red[1] += qr * ri - qi * rr;
          red[2] += qr * qr + qi * qi;
        }
    }
  }
  store_spinor<S, R, true>(a.out, vs, v, res);
}

// One thread per (site, rhs): the lanes of a site block's source group are
// adjacent in the workgroup and the workgroups of its groups are adjacent in
// the launch (rhs_block), so link and clover loads are shared.
template <typename S, typename R, int RECON, int MODE, bool REDUCE, int HOPS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) wilson_kernel(WArgs<S> a) {
  const RhsBlock rb = rhs_block(a.nrhs, a.rg);
  double red[3] = {0, 0, 0};
  int s = rb.s;
  if constexpr (MODE == W_HOP_CLOV || MODE == W_XPAY_CLOV) {
    // one colour of tiles (single right-hand side; the host checks)
    if (a.g.colour >= 0) s = rb.s < (a.g.Vh >> 1) ? colour_site(a.g, rb.s) : a.g.Vh;
  }
  if (s < a.g.Vh) wilson_point<S, R, RECON, MODE, REDUCE, false, HOPS>(a, s, rb.rhs, red);
  if constexpr (REDUCE) {  // single right-hand side only
    segment_reduce_store(red, a.g.Vt2 < 64 ? a.g.Vt2 : 64, s, a.g.Vh, a.partials);
  }
}

// Matrix-core variant for 16-bit storage and a multiple of 4 right-hand sides:
// lanes 4b .. 4b+3 (one 4x4x4 block) are one site and its 4 sources of one
// group (the lane mapping of wilson_kernel with 4 sources per group). All
// lanes stay active through the products.
template <typename S, int RECON, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) wilson_mf_kernel(WArgs<S> a) {
  const RhsBlock rb = rhs_block(a.nrhs, 4);  // rg == 4 here
  const bool valid = rb.s < a.g.Vh;
  double red[3];
  wilson_point<S, float, RECON, MODE, false, true>(a, valid ? rb.s : 0, rb.rhs, red, valid);
}

// Persistent launch over several operators (uneven lattices, several
// right-hand sides each): a fixed grid of workgroups takes work items from a
// global counter until every item of every job is done. An item is one
// workgroup's worth of (site, rhs) pairs, numbered job after job and, within a
// job, in the order of the non-persistent launch (source fastest).
constexpr int kMaxBatchJobs = 8;
constexpr int kBatchQueues = 8;  // one work queue per XCD
template <typename S> struct BatchArgs {
  WArgs<S> job[kMaxBatchJobs];
  int begin[kMaxBatchJobs + 1];  // first work item of each job (prefix sums)
  int njobs;
  int chunk;
  int mfma;           // 16-bit jobs with a multiple of 4 sources: link products on the matrix cores
  unsigned *counter;  // kBatchQueues counters, zero at launch
};

// Items are split into kBatchQueues contiguous ranges; workgroup b serves queue
// b % kBatchQueues, i.e. the XCD it runs on, so the items of one site block
// (its source groups, adjacent in the numbering) share that XCD's L2. The grid
// is a multiple of kBatchQueues, so every queue is drained.
template <typename S, typename R, int RECON>
__device__ __forceinline__ void batch_item(const BatchArgs<S> &b, int it) {
  int j = 0;
  while (j + 1 < b.njobs && it >= b.begin[j + 1]) ++j;
  const WArgs<S> &a = b.job[j];
  const RhsBlock rb = rhs_block_at(it - b.begin[j], a.nrhs, a.rg);
  const bool valid = rb.s < a.g.Vh;
  double red[3];
  if constexpr (is_float16<S>()) {
    if (b.mfma && a.nrhs % 4 == 0) {  // uniform over the workgroup
      wilson_point<S, R, RECON, W_HOP, false, true>(a, valid ? rb.s : 0, rb.rhs, red, valid);
      return;
    }
  }
  // jobs carry no cut: the same hop code as the per-operator launch
  if (valid)
    wilson_point<S, R, RECON, W_HOP, false, false, pipelined_hops<S, RECON, W_HOP>() ? kHopsPipe : kHopsChecked>(
        a, rb.s, rb.rhs, red);
}

// Single launch with one workgroup per item (items remapped per XCD like the
// single-operator launch): the alternative the autotuner weighs against the
// persistent queue.
template <typename S, typename R, int RECON>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) wilson_batch_flat_kernel(BatchArgs<S> b) {
  batch_item<S, R, RECON>(b, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename S, typename R, int RECON>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) wilson_batch_kernel(BatchArgs<S> b) {
  __shared__ int next;
  const int total = b.begin[b.njobs];
  const int q = blockIdx.x % kBatchQueues;
  const int lo = (int)((int64_t)q * total / kBatchQueues), hi = (int)((int64_t)(q + 1) * total / kBatchQueues);
  // the index of the following item is fetched while the current one runs
  if (threadIdx.x == 0) next = lo + (int)atomicAdd(b.counter + q, 1u);
  __syncthreads();
  int it = next;
  while (it < hi) {
    __syncthreads();  // every thread has read `next`
    if (threadIdx.x == 0) next = lo + (int)atomicAdd(b.counter + q, 1u);
    batch_item<S, R, RECON>(b, it);
    __syncthreads();  // `next` is written
    it = next;
  }
}

__global__ void zero_counter_kernel(unsigned *c) { c[threadIdx.x] = 0u; }  // one workgroup, one thread per counter

template <typename S, typename R>
__global__ void __launch_bounds__(256) clover_apply_kernel(Geom g, S *out, const S *in, const S *clov, int nrhs) {
  const RhsBlock rb = rhs_block(nrhs, rhs_group(nrhs));
  const int s = rb.s;
  if (s >= g.Vh) return;
  const int64_t pidx = rhs_index(rb.rhs, s, g.Vh, rhs_group(nrhs));
  const int64_t vs = (int64_t)g.Vh * nrhs;
  cpx<R> x[4][3], y[4][3];
  load_spinor<S, R>(in, vs, pidx, x);
  clover_mul<S, R>(clov, g.Vh, s, x, y, nrhs == 1);
  store_spinor<S, R, true>(out, vs, pidx, y);
}

// ---------------------------------------------------------------------------
// Additive Schwarz with each block resident in LDS (Section 4's block solver,
// with blocks equal to the tiles and 16-bit storage: FP16, BF16, or fixed
// point with a per-site norm): one workgroup runs every
// MR step of one block. The block's spinor of the current half step (r on the
// even sites, then t on the odd sites) lives in LDS, so neighbours are read
// from there; links and clover stream from memory in each half step; the
// workgroup keeps its sites' r and q (and x, where registers allow) as stored
// 16-bit values. Per step and even site this moves the links twice and both
// clover blocks (672 bytes at 12 link reals, 768 with x in memory) instead of
// the 1152 bytes of two cut Schur launches and an update. The arithmetic is
// the launches' (same operations, same roundings to the storage format, the
// same order of the FP64 sums of <q,r> and <q,q>: per 64-site segment by the
// wave butterfly, then the block's segments in order), so both forms give the
// same result.
constexpr int kSapMaxSites = 2048;  // sites per parity of one block (96 KiB of 16-bit spinor)

template <typename S> struct SapArgs {
  S *x;           // out: x (even sites)
  const S *r0;    // in: residual (even sites)
  const S *gauge;
  const S *clov_inv_odd;  // A_oo^-1
  const S *clov_even;     // A_ee
  Geom g;                 // for the tile of a colour-restricted launch
  int64_t vh;
  int vt2;
  int b[4];   // block (tile) extents
  int wrap;   // bit mu: the block spans the lattice along mu, its hops wrap inside it
  int bc_t;
  float coef;  // -kappa^2
  double omega;
  int steps;
  int first;  // x starts at zero (not read)
};

// two stored 16-bit values in one register
template <typename S> __device__ __forceinline__ uint32_t pack16(S lo, S hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}
template <typename S> __device__ __forceinline__ float lo16(uint32_t u) {
  return to_real<float>(__builtin_bit_cast(S, (uint16_t)(u & 0xffffu)));
}
template <typename S> __device__ __forceinline__ float hi16(uint32_t u) {
  return to_real<float>(__builtin_bit_cast(S, (uint16_t)(u >> 16)));
}

// A site's stored spinor: its 24 16-bit values as 12 registers (register j =
// reals 2j, 2j+1; in LDS and in memory the spinor is chunk-major, chunk c =
// registers 2c, 2c+1) and, with fixed-point storage, the site norm.
template <typename S, bool FIXED = is_fixed<S>()> struct SapSite {
  uint32_t p[12];
};
template <typename S> struct SapSite<S, true> {
  uint32_t p[12];
  float m;
};

// stored -> FP32, as the other kernels load (fixed point: the code's value,
// then times the site norm)
template <typename S> __device__ __forceinline__ void sap_reals(const SapSite<S> &s, float (&v)[24]) {
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    v[2 * j] = lo16<S>(s.p[j]);
    v[2 * j + 1] = hi16<S>(s.p[j]);
  }
  if constexpr (is_fixed<S>()) {
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] *= s.m;
  }
}
// FP32 -> stored, as the other kernels store (fixed point: the norm is the
// largest |v_k|, the codes those of v_k times its reciprocal)
template <typename S> __device__ __forceinline__ void sap_store(const float (&v)[24], SapSite<S> &s) {
  if constexpr (is_fixed<S>()) {
    const float m = fixed_norm<24, float>(v), inv = m > 0 ? 1.0f / m : 0.0f;
    s.m = m;
#pragma unroll
    for (int j = 0; j < 12; ++j)
      s.p[j] = pack16<S>(Store<S>::from((float)v[2 * j] * inv), Store<S>::from((float)v[2 * j + 1] * inv));
  } else {
#pragma unroll
    for (int j = 0; j < 12; ++j) s.p[j] = pack16<S>(Store<S>::from(v[2 * j]), Store<S>::from(v[2 * j + 1]));
  }
}
__device__ __forceinline__ void sap_flat(const cpx<float> (&v)[4][3], float (&f)[24]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      f[6 * sp + 2 * c] = v[sp][c].re;
      f[6 * sp + 2 * c + 1] = v[sp][c].im;
    }
}
__device__ __forceinline__ void sap_cpx(const float (&f)[24], cpx<float> (&v)[4][3]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[sp][c] = mk<float>(f[6 * sp + 2 * c], f[6 * sp + 2 * c + 1]);
}
// The site's registers become opaque to the compiler here: values derived
// from them (unpacked FP32 copies) are not kept alive across the point.
template <typename S> __device__ __forceinline__ void sap_opaque(SapSite<S> &s) {
#pragma unroll
  for (int j = 0; j < 12; ++j) __asm__ volatile("" : "+v"(s.p[j]));
  if constexpr (is_fixed<S>()) __asm__ volatile("" : "+v"(s.m));
}
// LDS: 6 chunk arrays of vt2 sites (8 bytes each), then (fixed point) the
// vt2 site norms
template <typename S> __device__ __forceinline__ void sap_lds_put(uint2 *lds, int vt2, int k, const SapSite<S> &s) {
#pragma unroll
  for (int c = 0; c < 6; ++c) lds[c * vt2 + k] = make_uint2(s.p[2 * c], s.p[2 * c + 1]);
  if constexpr (is_fixed<S>()) reinterpret_cast<float *>(lds + 6 * vt2)[k] = s.m;
}
template <typename S> __device__ __forceinline__ void sap_lds_get(const uint2 *lds, int vt2, int k, SapSite<S> &s) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const uint2 v = lds[c * vt2 + k];
    s.p[2 * c] = v.x;
    s.p[2 * c + 1] = v.y;
  }
  if constexpr (is_fixed<S>()) s.m = reinterpret_cast<const float *>(lds + 6 * vt2)[k];
}
template <typename S> __device__ __forceinline__ void sap_mem_get(const S *f, int64_t vh, int64_t s, SapSite<S> &o) {
  const uint2 *q = reinterpret_cast<const uint2 *>(f);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const uint2 v = q[c * vh + s];
    o.p[2 * c] = v.x;
    o.p[2 * c + 1] = v.y;
  }
  if constexpr (is_fixed<S>()) o.m = site_norms<S, 24>(f, vh)[s];
}
template <typename S> __device__ __forceinline__ void sap_mem_put(S *f, int64_t vh, int64_t s, const SapSite<S> &o) {
  uint2 *q = reinterpret_cast<uint2 *>(f);
#pragma unroll
  for (int c = 0; c < 6; ++c) nt_store(q + c * vh + s, make_uint2(o.p[2 * c], o.p[2 * c + 1]));
  if constexpr (is_fixed<S>()) site_norms<S, 24>(f, vh)[s] = o.m;
}
// bytes of dynamic LDS: the spinor (and norms) of a block, then the segment sums
__host__ __device__ constexpr size_t sap_lds_bytes(int vt2, bool fixed) {
  return (size_t)vt2 * (48 + (fixed ? 4 : 0)) + (size_t)(vt2 / 64) * 3 * sizeof(double);
}

// Hop of STEP along MU from block coordinates l: false if the cut drops it;
// else the neighbour's block-local index and whether the hop wrapped the
// lattice along t with antiperiodic boundary (a sign flip).
template <int MU, int STEP, typename S>
__device__ __forceinline__ bool sap_hop(const SapArgs<S> &a, const int (&l)[4], int *kn, bool *flip) {
  int c[4] = {l[0], l[1], l[2], l[3]};
  c[MU] += STEP;
  const bool out = STEP > 0 ? c[MU] >= a.b[MU] : c[MU] < 0;
  if (out && !((a.wrap >> MU) & 1)) return false;
  c[MU] = out ? (STEP > 0 ? 0 : a.b[MU] - 1) : c[MU];
  *flip = MU == 3 && out && a.bc_t < 0;
  *kn = (c[0] >> 1) + (a.b[0] >> 1) * (c[1] + a.b[1] * (c[2] + a.b[2] * c[3]));
  return true;
}

template <int MU, int STEP, typename S, int RECON>
__device__ __forceinline__ void sap_hop_acc(const SapArgs<S> &a, const uint2 *lds, int base, const int (&l)[4], int k,
                                            int par, cpx<float> (&acc)[4][3]) {
  int kn;
  bool flip;
  if (!sap_hop<MU, STEP>(a, l, &kn, &flip)) return;
  SapSite<S> nb;
  cpx<float> u[2][3];
  sap_lds_get<S>(lds, a.vt2, kn, nb);
  // forward: (1 - gamma_mu) U_mu(x) psi(x+mu); backward: (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)
  const float g = STEP > 0 ? -1.f : 1.f;
  if constexpr (half_hop<S, RECON>()) {
    // the packed-half hop of the launch kernels, on the stored values
    S raw[RECON];
    uint32_t lw[RECON / 2];
    const int lpar = STEP > 0 ? par : 1 - par, ls = base + (STEP > 0 ? k : kn);
    load_chunks_raw<S, RECON, chunk_reals<S, RECON>(), true>(a.gauge + (int64_t)(2 * MU + lpar) * a.vh * RECON, a.vh,
                                                             ls, raw);
#pragma unroll
    for (int j = 0; j < RECON / 2; ++j) lw[j] = __builtin_bit_cast(uint32_t, h2v{raw[2 * j], raw[2 * j + 1]});
    hop_h2<MU, STEP, RECON>(nb.p, lw, g, u);
  } else {
    float pf[24];
    cpx<float> psi[4][3], h[2][3];
    sap_reals<S>(nb, pf);
    sap_cpx(pf, psi);
    project<MU, float>(psi, g, h);
    const Link<float> U = STEP > 0 ? load_link<S, float, RECON>(a.gauge, a.vh, MU, par, base + k, true)
                                   : load_link<S, float, RECON>(a.gauge, a.vh, MU, 1 - par, base + kn, true);
    if constexpr (STEP > 0) {
      su3_mv(U, h[0], u[0]);
      su3_mv(U, h[1], u[1]);
    } else {
      su3_adj_mv(U, h[0], u[0]);
      su3_adj_mv(U, h[1], u[1]);
    }
  }
  if constexpr (MU == 3) {
    const float ph = flip ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) u[i][c] = ph * u[i][c];
  }
  expand_acc<MU, float>(acc, u, g);
}

// D restricted to the block at block-local site k of parity par (coordinates
// packed 8 bits each: x/2, y, z, t), neighbours from LDS
template <typename S, int RECON>
__device__ __forceinline__ void sap_hops(const SapArgs<S> &a, const uint2 *lds, int base, int k, uint32_t coords,
                                         int par, cpx<float> (&acc)[4][3]) {
  int l[4];
  l[1] = (coords >> 8) & 255;
  l[2] = (coords >> 16) & 255;
  l[3] = coords >> 24;
  l[0] = 2 * (int)(coords & 255) + ((l[1] + l[2] + l[3] + par) & 1);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[i][c] = mk<float>(0, 0);
  sap_hop_acc<0, +1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<0, -1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<1, +1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<1, -1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<2, +1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<2, -1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<3, +1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
  sap_hop_acc<3, -1, S, RECON>(a, lds, base, l, k, par, acc);
  __builtin_amdgcn_sched_barrier(0);
}

// Clover product for the block kernel: the same operations as clover_mul, one
// chirality block at a time (36 values in registers instead of 72).
template <typename S>
__device__ __forceinline__ void sap_clover(const S *__restrict__ clov, int64_t vh, int s, const cpx<float> (&in)[4][3],
                                           cpx<float> (&out)[4][3]) {
  constexpr int CH = chunk_reals<S, 72>();  // reals per chunk (8 for 16-bit storage)
  static_assert(CH == 8, "16-bit clover chunks of 8 reals");
  float a[72];
  float m = 1.f;  // fixed point: the site norm of the clover term
  if constexpr (is_fixed<S>()) m = site_norms<S, 72>(clov, vh)[s];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    // chunks 0..4 hold block 0 (reals 0..35), chunks 4..8 block 1 (36..71)
#pragma unroll
    for (int c = 5 * b - b; c < 5 * b - b + 5; ++c) {
      if (b == 1 && c == 4) continue;  // loaded with block 0
      const Chunk<S, 8> v = nt_load(reinterpret_cast<const Chunk<S, 8> *>(clov + (c * vh + s) * 8));
#pragma unroll
      for (int j = 0; j < 8; ++j) a[8 * c + j] = to_real<float>(v.v[j]);
    }
#pragma unroll
    for (int k = 36 * b; k < 36 * b + 36; ++k) {
      if constexpr (is_fixed<S>())
        a[k] *= m;
      else
        __asm__ volatile("" : "+v"(a[k]));
    }
    const float *A = a + 36 * b;
    cpx<float> x[6], y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] = in[2 * b + i / 3][i % 3];
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] = A[i] * x[i];
    int off = 6;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) {
        const cpx<float> aij = mk<float>(A[off], A[off + 1]);
        off += 2;
        cmac(y[i], aij, x[j]);
        cmac_conj(y[j], aij, x[i]);
      }
#pragma unroll
    for (int i = 0; i < 6; ++i) out[2 * b + i / 3][i % 3] = y[i];
  }
}

// One workgroup per block (blockIdx.x: the block's tile, or the j-th tile of
// one colour); SPT sites per thread and parity, site k = p * blockDim.x + tid.
// XREG: x stays in registers (else it is read and written in memory each step).
// NT: the most threads per workgroup (512, or 1024 for the wide launches).
template <typename S, int RECON, int SPT, bool XREG, int NT>
__global__ void __launch_bounds__(NT) sap_block_kernel(SapArgs<S> a) {
  extern __shared__ uint2 sap_lds[];  // the block's spinor (and norms), then the segment sums
  const int vt2 = a.vt2, nt = blockDim.x, tid = threadIdx.x;
  double *seg = reinterpret_cast<double *>(reinterpret_cast<char *>(sap_lds) + sap_lds_bytes(vt2, is_fixed<S>()) -
                                           (size_t)(vt2 / 64) * 3 * sizeof(double));  // [Vt2 / 64][3]
  const int tile = a.g.colour >= 0 ? colour_site(a.g, blockIdx.x * vt2) / vt2 : (int)blockIdx.x;
  const int base = tile * vt2;
  SapSite<S> r[SPT], w[SPT];  // w: t (odd sites) or q (even sites)
  SapSite<S> x[XREG ? SPT : 1];
  uint32_t coords[SPT];
#pragma unroll
  for (int p = 0; p < SPT; ++p) {
    const int k = p * nt + tid;
    const int bxh = a.b[0] >> 1;
    const int q1 = k / bxh, q2 = q1 / a.b[1];
    coords[p] = (uint32_t)(k - q1 * bxh) | ((uint32_t)(q1 - q2 * a.b[1]) << 8) |
                ((uint32_t)(q2 % a.b[2]) << 16) | ((uint32_t)(q2 / a.b[2]) << 24);
    sap_mem_get<S>(a.r0, a.vh, base + k, r[p]);
    sap_lds_put<S>(sap_lds, vt2, k, r[p]);
    if constexpr (XREG)
      if (a.first)
        x[p] = SapSite<S>{};
      else
        sap_mem_get<S>(a.x, a.vh, base + k, x[p]);
  }
  __syncthreads();
  // In each phase the thread's site index and coordinates pass through an
  // empty asm, so that the addresses derived from them are recomputed there
  // rather than held in registers across the step loop.
  for (int step = 0; step < a.steps; ++step) {
    // t_o = A_oo^-1 D_oe r on the block's odd sites
#pragma unroll
    for (int p = 0; p < SPT; ++p) {
      int k = p * nt + tid;
      __asm__ volatile("" : "+v"(k));
      cpx<float> acc[4][3], res[4][3];
      float f[24];
      uint32_t cp = coords[p];
      __asm__ volatile("" : "+v"(cp));
      sap_hops<S, RECON>(a, sap_lds, base, k, cp, 1, acc);
      sap_clover<S>(a.clov_inv_odd, a.vh, base + k, acc, res);
      sap_flat(res, f);
      sap_store<S>(f, w[p]);
      sap_opaque<S>(w[p]);
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every read of r is done
#pragma unroll
    for (int p = 0; p < SPT; ++p) {
      int k = p * nt + tid;
      __asm__ volatile("" : "+v"(k));
      sap_lds_put<S>(sap_lds, vt2, k, w[p]);
    }
    __syncthreads();
    // q_e = A_ee r + coef D_eo t, and the segment sums of <q,r>, <q,q> over
    // the values as stored
#pragma unroll
    for (int p = 0; p < SPT; ++p) {
      int k = p * nt + tid;
      __asm__ volatile("" : "+v"(k));
      cpx<float> acc[4][3], res[4][3], xv[4][3];
      float rf[24], qf[24];
      uint32_t cp = coords[p];
      __asm__ volatile("" : "+v"(cp));
      sap_hops<S, RECON>(a, sap_lds, base, k, cp, 0, acc);
      __builtin_amdgcn_sched_barrier(0);
      sap_reals<S>(r[p], rf);
      sap_cpx(rf, xv);
      sap_clover<S>(a.clov_even, a.vh, base + k, xv, res);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) res[i][c] = res[i][c] + a.coef * acc[i][c];
      sap_flat(res, qf);
      sap_store<S>(qf, w[p]);
      if constexpr (is_fixed<S>()) {
        sap_reals<S>(w[p], qf);  // the values as stored
      } else {
#pragma unroll
        for (int j = 0; j < 24; ++j) qf[j] = quantize<S, float>(qf[j]);
      }
      double red[3] = {0, 0, 0};
#pragma unroll
      for (int j = 0; j < 12; ++j) {
        const double qr = qf[2 * j], qi = qf[2 * j + 1], rr = rf[2 * j], ri = rf[2 * j + 1];
        red[0] += qr * rr + qi * ri;
        red[1] += qr * ri - qi * rr;
        red[2] += qr * qr + qi * qi;
      }
      sap_opaque<S>(w[p]);
      sap_opaque<S>(r[p]);
#pragma unroll
      for (int j = 0; j < 3; ++j)
        for (int off = 32; off > 0; off >>= 1) red[j] += __shfl_xor(red[j], off, 64);
      if ((k & 63) == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) seg[3 * (k >> 6) + j] = red[j];
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every read of t and every segment sum is done
    double qr = 0, qi = 0, qq = 0;
    for (int j = 0; j < (vt2 >> 6); ++j) {
      qr += seg[3 * j];
      qi += seg[3 * j + 1];
      qq += seg[3 * j + 2];
    }
    const float ar = qq > 0 ? (float)(a.omega * qr / qq) : 0.f, ai = qq > 0 ? (float)(a.omega * qi / qq) : 0.f;
    const bool last = step == a.steps - 1, zero_x = a.first && step == 0;
    // x += alpha r, r -= alpha q (the last step needs no new r)
#pragma unroll
    for (int p = 0; p < SPT; ++p) {
      int k = p * nt + tid;
      __asm__ volatile("" : "+v"(k));
      SapSite<S> xo{};
      if constexpr (XREG) {
        xo = x[p];
      } else {
        if (!zero_x) sap_mem_get<S>(a.x, a.vh, base + k, xo);
      }
      float rv[24], qv[24], xv[24];
      sap_reals<S>(r[p], rv);
      sap_reals<S>(w[p], qv);
      sap_reals<S>(xo, xv);
#pragma unroll
      for (int j = 0; j < 24; ++j) xv[j] = zero_x ? 0.f : xv[j];
#pragma unroll
      for (int j = 0; j < 12; ++j) {
        const float re = rv[2 * j], im = rv[2 * j + 1];
        xv[2 * j] += ar * re - ai * im;
        xv[2 * j + 1] += ar * im + ai * re;
        rv[2 * j] = re - (ar * qv[2 * j] - ai * qv[2 * j + 1]);
        rv[2 * j + 1] = im - (ar * qv[2 * j + 1] + ai * qv[2 * j]);
      }
      sap_store<S>(xv, xo);
      if (!last) sap_store<S>(rv, r[p]);
      sap_opaque<S>(r[p]);
      if constexpr (XREG) {
        x[p] = xo;
      } else {
        sap_mem_put<S>(a.x, a.vh, base + k, xo);
      }
      if (!last) sap_lds_put<S>(sap_lds, vt2, k, r[p]);
    }
    __syncthreads();  // the new r is in LDS; the segment sums are read
  }
  if constexpr (XREG) {
#pragma unroll
    for (int p = 0; p < SPT; ++p) sap_mem_put<S>(a.x, a.vh, base + p * nt + tid, x[p]);
  }
}

// Sites per thread of the block-resident form for blocks of vt2 sites per
// parity (0: the form does not apply).
int sap_block_spt(int vt2) {
  if (vt2 % 64 || vt2 > kSapMaxSites) return 0;
  for (int spt : {1, 2, 4})
    if (vt2 / spt <= 512 && vt2 % (64 * spt) == 0) return spt;
  return 0;
}

// The wide launch: twice the threads (up to 1024) with half the sites each,
// where a block has at least two sites per thread of the 512-thread launch.
bool sap_block_wide_fits(int vt2) { return sap_block_spt(vt2) >= 2; }

template <typename S, int RECON, int SPT, bool XREG, int NT>
static hipError_t launch_sap4(const SapLaunch &l, hipStream_t st) {
  SapArgs<S> a;
  a.x = (S *)l.x;
  a.r0 = (const S *)l.r0;
  a.gauge = (const S *)l.gauge;
  a.clov_inv_odd = (const S *)l.clov_inv_odd;
  a.clov_even = (const S *)l.clov_even;
  a.g = l.g;
  a.vh = l.g.Vh;
  a.vt2 = l.g.Vt2;
  a.wrap = 0;
  for (int m = 0; m < 4; ++m) {
    a.b[m] = l.g.B[m];
    if (l.g.B[m] == l.g.L[m]) a.wrap |= 1 << m;
  }
  a.bc_t = l.g.bc_t;
  a.coef = (float)l.coef;
  a.omega = l.omega;
  a.steps = l.steps;
  a.first = l.first;
  const size_t lds = sap_lds_bytes(l.g.Vt2, is_fixed<S>());
  static bool attr_set = false;  // per instantiation
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sap_block_kernel<S, RECON, SPT, XREG, NT>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)sap_lds_bytes(kSapMaxSites, is_fixed<S>()));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int nblocks = launch_sites(l.g) / l.g.Vt2;
  hipLaunchKernelGGL((sap_block_kernel<S, RECON, SPT, XREG, NT>), dim3(nblocks), dim3(l.g.Vt2 / SPT), lds, st, a);
  return hipGetLastError();
}

template <typename S, int RECON, int SPT, int NT>
static hipError_t launch_sap3(const SapLaunch &l, hipStream_t st) {
  return l.xreg ? launch_sap4<S, RECON, SPT, true, NT>(l, st) : launch_sap4<S, RECON, SPT, false, NT>(l, st);
}

template <typename S, int RECON>
static hipError_t launch_sap2(const SapLaunch &l, hipStream_t st) {
  const int spt = sap_block_spt(l.g.Vt2);
  if (l.wide) {
    switch (spt) {
      case 2: return launch_sap3<S, RECON, 1, 1024>(l, st);
      case 4: return launch_sap3<S, RECON, 2, 1024>(l, st);
    }
    return hipErrorInvalidValue;
  }
  switch (spt) {
    case 1: return launch_sap3<S, RECON, 1, 512>(l, st);
    case 2: return launch_sap3<S, RECON, 2, 512>(l, st);
    case 4: return launch_sap3<S, RECON, 4, 512>(l, st);
  }
  return hipErrorInvalidValue;
}

template <typename S>
static hipError_t launch_sap1(const SapLaunch &l, hipStream_t st) {
  switch (l.recon) {
    case 18: return launch_sap2<S, 18>(l, st);
    case 12: return launch_sap2<S, 12>(l, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sap_block(const SapLaunch &l, hipStream_t st) {
  for (int m = 0; m < 4; ++m)  // blocks are the tiles; coordinates fit 8 bits
    if (l.g.cut[m] != l.g.B[m] || l.g.B[m] > 256) return hipErrorInvalidValue;
  if (l.steps < 1 || !sap_block_spt(l.g.Vt2)) return hipErrorInvalidValue;
  if (l.g.colour >= 0 && (l.g.NT[0] & 1)) return hipErrorInvalidValue;
  if (l.g.Vh == 0) return hipSuccess;
  switch (l.prec) {
    case LQCD_F16: return launch_sap1<_Float16>(l, st);
    case LQCD_BF16: return launch_sap1<bf16>(l, st);
    case LQCD_HALF: return launch_sap1<fx16>(l, st);
  }
  return hipErrorInvalidValue;
}

// Schwarz MR step on every block at once, after q = Mhat_B r and the
// per-segment partials of <q,r> and <q,q>: alpha_B = <q,r>_B / <q,q>_B,
// x += alpha_B r (x = alpha_B r on the first step), r -= alpha_B q.
template <typename S, typename R>
__global__ void __launch_bounds__(256) mr_update_kernel(Geom g, S *x, S *r, const S *q, const double *part, int nps,
                                                        int first, double omega) {
  int s = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (s >= launch_sites(g)) return;
  if (g.colour >= 0) s = colour_site(g, s);
  const int b = (int)fdiv((uint32_t)s, g.dVt2);
  double qr = 0, qi = 0, qq = 0;
  for (int j = 0; j < nps; ++j) {
    const double *p = part + 3 * (b * nps + j);
    qr += p[0];
    qi += p[1];
    qq += p[2];
  }
  const R ar = qq > 0 ? (R)(omega * qr / qq) : R(0), ai = qq > 0 ? (R)(omega * qi / qq) : R(0);
  R rv[24], qv[24], xv[24];
  load_spinor_reals<S, 24, R>(r, g.Vh, s, rv);
  load_spinor_reals<S, 24, R>(q, g.Vh, s, qv);
  if (first) {
#pragma unroll
    for (int k = 0; k < 24; ++k) xv[k] = R(0);
  } else {
    load_spinor_reals<S, 24, R>(x, g.Vh, s, xv);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const R re = rv[2 * k], im = rv[2 * k + 1];
    xv[2 * k] += ar * re - ai * im;
    xv[2 * k + 1] += ar * im + ai * re;
    rv[2 * k] = re - (ar * qv[2 * k] - ai * qv[2 * k + 1]);
    rv[2 * k + 1] = im - (ar * qv[2 * k + 1] + ai * qv[2 * k]);
  }
  store_spinor_reals<S, 24, R>(x, g.Vh, s, xv);
  store_spinor_reals<S, 24, R>(r, g.Vh, s, rv);
}

hipError_t launch_mr_update(const Geom &g, int prec, void *x, void *r, const void *q, const double *partials, int nps,
                            bool first, double omega, hipStream_t st) {
  const int bt = 256, nwg = (launch_sites(g) + bt - 1) / bt;
  if (g.Vh == 0) return hipSuccess;
  switch (prec) {
#define CASE(P)                                                                                              \
  case P:                                                                                                    \
    hipLaunchKernelGGL((mr_update_kernel<Prec<P>::S, Prec<P>::R>), dim3(nwg), dim3(bt), 0, st, g,            \
                       (Prec<P>::S *)x, (Prec<P>::S *)r, (const Prec<P>::S *)q, partials, nps, (int)first, omega);  \
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


template <int P, int RECON, int MODE, bool RED>
static hipError_t launch_w3(const WilsonLaunch &w, hipStream_t st) {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  WArgs<S> a;
  a.g = w.g;
  a.out = (S *)w.out;
  a.in = (const S *)w.in;
  a.gauge = (const S *)w.gauge;
  a.clov = (const S *)w.clov;
  a.xin = (const S *)w.xin;
  a.partials = w.partials;
  a.coef = w.coef;
  a.parity = w.parity;
  a.dagger = w.dagger;
  a.nrhs = w.nrhs;
  a.rg = rhs_group(w.nrhs);
  // colour-restricted launches: the cut Schur pieces, one source, tiles
  // alternating in colour along x, and a cut (blocks of one colour are
  // independent only through it)
  if (w.g.colour >= 0 && ((MODE != W_HOP_CLOV && MODE != W_XPAY_CLOV) || w.nrhs != 1 || w.mfma || (w.g.NT[0] & 1) ||
                          !w.g.has_cut))
    return hipErrorInvalidValue;
  const int nwg = rhs_grid(launch_sites(w.g), w.nrhs, w.block_threads);
  if constexpr ((P == LQCD_F16 || P == LQCD_BF16) && !RED) {
    if (w.mfma) {
      if (w.nrhs % 4 || w.block_threads % 64) return hipErrorInvalidValue;
      hipLaunchKernelGGL((wilson_mf_kernel<S, RECON, MODE>), dim3(nwg), dim3(w.block_threads), 0, st, a);
      return hipGetLastError();
    }
  }
  if (w.mfma) return hipErrorInvalidValue;
  // launches without a cut take the pipelined hops where they pay (measured);
  // the others keep the runtime-checked hops
  if constexpr (pipelined_hops<S, RECON, MODE>()) {
    if (!w.g.has_cut) {
      hipLaunchKernelGGL((wilson_kernel<S, R, RECON, MODE, RED, kHopsPipe>), dim3(nwg), dim3(w.block_threads), 0, st,
                         a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((wilson_kernel<S, R, RECON, MODE, RED, kHopsChecked>), dim3(nwg), dim3(w.block_threads), 0, st,
                     a);
  return hipGetLastError();
}

template <int P, int RECON>
static hipError_t launch_w2(const WilsonLaunch &w, hipStream_t st) {
  switch (w.mode) {
    case W_HOP: return launch_w3<P, RECON, W_HOP, false>(w, st);
    case W_HOP_CLOV: return launch_w3<P, RECON, W_HOP_CLOV, false>(w, st);
    case W_XPAY_CLOV:
      return w.partials ? launch_w3<P, RECON, W_XPAY_CLOV, true>(w, st) : launch_w3<P, RECON, W_XPAY_CLOV, false>(w, st);
    case W_XPAY:
      return w.partials ? launch_w3<P, RECON, W_XPAY, true>(w, st) : launch_w3<P, RECON, W_XPAY, false>(w, st);
  }
  return hipErrorInvalidValue;
}

template <int P>
static hipError_t launch_w1(const WilsonLaunch &w, hipStream_t st) {
  switch (w.recon) {
    case 18: return launch_w2<P, 18>(w, st);
    case 12: return launch_w2<P, 12>(w, st);
    case 8:
      if constexpr (P == LQCD_F64 || P == LQCD_F32) return launch_w2<P, 8>(w, st);
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_wilson(const WilsonLaunch &w, hipStream_t st) {
  if (w.g.Vh == 0) return hipSuccess;
  switch (w.prec) {
    case LQCD_F64: return launch_w1<LQCD_F64>(w, st);
    case LQCD_F32: return launch_w1<LQCD_F32>(w, st);
    case LQCD_F16: return launch_w1<LQCD_F16>(w, st);
    case LQCD_BF16: return launch_w1<LQCD_BF16>(w, st);
    case LQCD_HALF: return launch_w1<LQCD_HALF>(w, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_clover_apply(const Geom &g, int prec, void *out, const void *in, const void *clov, int nrhs,
                               hipStream_t st) {
  const int bt = 256, nwg = rhs_grid(g.Vh, nrhs, bt);
  if (g.Vh == 0) return hipSuccess;
  switch (prec) {
#define CASE(P)                                                                                           \
  case P:                                                                                                 \
    hipLaunchKernelGGL((clover_apply_kernel<Prec<P>::S, Prec<P>::R>), dim3(nwg), dim3(bt), 0, st, g,      \
                       (Prec<P>::S *)out, (const Prec<P>::S *)in, (const Prec<P>::S *)clov, nrhs);        \
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

template <int P, int RECON>
static hipError_t launch_b2(const BatchJob *jobs, int njobs, int dagger, const BatchTune &t, int mfma,
                            unsigned *counter, hipStream_t st) {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  BatchArgs<S> b;
  b.njobs = njobs;
  b.chunk = t.chunk;
  b.mfma = mfma;
  if (t.chunk != t.block_threads || t.block_threads % 64) return hipErrorInvalidValue;
  b.counter = counter;
  b.begin[0] = 0;
  for (int j = 0; j < njobs; ++j) {
    WArgs<S> &a = b.job[j];
    a.g = jobs[j].g;
    a.out = (S *)jobs[j].out;
    a.in = (const S *)jobs[j].in;
    a.gauge = (const S *)jobs[j].gauge;
    a.clov = nullptr;
    a.xin = nullptr;
    a.partials = nullptr;
    a.coef = 1.0;
    a.parity = jobs[j].parity;
    a.dagger = dagger;
    a.nrhs = jobs[j].nrhs;
    a.rg = rhs_group(jobs[j].nrhs);
    // items of this job: one per workgroup of the non-persistent launch
    b.begin[j + 1] = b.begin[j] + rhs_grid(jobs[j].g.Vh, jobs[j].nrhs, t.block_threads);
  }
  if (t.grid == 0) {  // one workgroup per item
    hipLaunchKernelGGL((wilson_batch_flat_kernel<S, R, RECON>), dim3(b.begin[njobs]), dim3(t.block_threads), 0, st, b);
    return hipGetLastError();
  }
  if (t.grid % kBatchQueues) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(kBatchQueues), 0, st, counter);
  hipLaunchKernelGGL((wilson_batch_kernel<S, R, RECON>), dim3(t.grid), dim3(t.block_threads), 0, st, b);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_b1(int recon, const BatchJob *jobs, int njobs, int dagger, const BatchTune &t, int mf,
                            unsigned *c, hipStream_t st) {
  switch (recon) {
    case 18: return launch_b2<P, 18>(jobs, njobs, dagger, t, mf, c, st);
    case 12: return launch_b2<P, 12>(jobs, njobs, dagger, t, mf, c, st);
    case 8:
      if constexpr (P == LQCD_F64 || P == LQCD_F32) return launch_b2<P, 8>(jobs, njobs, dagger, t, mf, c, st);
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_wilson_batch(int prec, int recon, const BatchJob *jobs, int njobs, int dagger, const BatchTune &t,
                               int mfma, unsigned *counter, hipStream_t st) {
  if (njobs < 1 || njobs > kMaxBatchJobs) return hipErrorInvalidValue;
  if (mfma && prec != LQCD_F16 && prec != LQCD_BF16) return hipErrorInvalidValue;
  switch (prec) {
    case LQCD_F64: return launch_b1<LQCD_F64>(recon, jobs, njobs, dagger, t, mfma, counter, st);
    case LQCD_F32: return launch_b1<LQCD_F32>(recon, jobs, njobs, dagger, t, mfma, counter, st);
    case LQCD_F16: return launch_b1<LQCD_F16>(recon, jobs, njobs, dagger, t, mfma, counter, st);
    case LQCD_BF16: return launch_b1<LQCD_BF16>(recon, jobs, njobs, dagger, t, mfma, counter, st);
    case LQCD_HALF: return launch_b1<LQCD_HALF>(recon, jobs, njobs, dagger, t, mfma, counter, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lqcd
