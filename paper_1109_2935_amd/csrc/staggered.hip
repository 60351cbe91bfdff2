// Improved-staggered hopping term for gfx950 (eq. (3) of the paper):
//   (D chi)(x) = sum_mu eta_mu(x) [ F_mu(x) chi(x+mu) - F_mu(x-mu)^+ chi(x-mu)
//                                  + c_long ( L_mu(x) chi(x+3mu) - L_mu(x-3mu)^+ chi(x-3mu) ) ]
// with Kogut-Susskind phases eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y),
// eta_t = (-1)^(x+y+z), fat links F (general complex, 18 reals) and long links
// L (SU(3), 18/12/8 reals). One thread per output site; the kernel can fuse
// out = coef * D in + xcoef * xin.
#include <type_traits>

#include "lqcd_internal.h"

namespace lqcd {

template <typename S> struct SArgs {
  Geom g;
  S *out;
  const S *in;
  const S *fat;
  const S *lng;
  const S *xin;
  int parity;
  double coef, xcoef, c_long;
  int nrhs;  // sources
  int rg;    // sources per block of the multi-source layout (rhs_group(nrhs))
};

template <typename S, typename R>
__device__ __forceinline__ void load_cvec(const S *__restrict__ f, int64_t vh, int s, cpx<R> (&v)[3]) {
  R r[6];
  load_spinor_reals<S, 6, R>(f, vh, s, r);
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = mk<R>(r[2 * c], r[2 * c + 1]);
}

// Hops along MU: h = 0 the fat (one-site) hops, h = 1 the long (three-site)
// hops; H0 .. H1 selects which.
template <int MU, int H0, int H1, typename S, typename R, int RECON>
__device__ __forceinline__ void stag_dir(const SArgs<S> &a, const Site &x, int s, int rhs, R eta, R cl,
                                         cpx<R> (&acc)[3]) {
  const int64_t vh = a.g.Vh, vs = vh * a.nrhs;
  const int neg = a.g.bc_t < 0;
#pragma unroll
  for (int h = H0; h <= H1; ++h) {
    const int k = h == 0 ? 1 : 3;
    const R wgt = h == 0 ? eta : eta * cl;
    {
      int w;
      const int n = hop<MU>(a.g, x, +k, &w);
      cpx<R> v[3], u[3];
      load_cvec<S, R>(a.in, vs, rhs_index(rhs, n, vh, a.rg), v);
      Link<R> U;
      if (h == 0) {
        R r[18];
        load_site_once<S, 18, R>(a.fat + (int64_t)(2 * MU + x.p) * vh * 18, vh, s, r, a.nrhs == 1);
        U = unpack_link<18, R>(r);
      } else {
        R r[RECON];
        load_site_once<S, RECON, R>(a.lng + (int64_t)(2 * MU + x.p) * vh * RECON, vh, s, r, a.nrhs == 1);
        U = unpack_link<RECON, R>(r);
      }
      su3_mv(U, v, u);
      const R f = (MU == 3 && (w & 1) && neg) ? -wgt : wgt;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = acc[c] + f * u[c];
    }
    {
      int w;
      const int n = hop<MU>(a.g, x, -k, &w);
      cpx<R> v[3], u[3];
      load_cvec<S, R>(a.in, vs, rhs_index(rhs, n, vh, a.rg), v);
      Link<R> U;
      if (h == 0) {
        R r[18];
        load_site_once<S, 18, R>(a.fat + (int64_t)(2 * MU + 1 - x.p) * vh * 18, vh, n, r, a.nrhs == 1);
        U = unpack_link<18, R>(r);
      } else {
        R r[RECON];
        load_site_once<S, RECON, R>(a.lng + (int64_t)(2 * MU + 1 - x.p) * vh * RECON, vh, n, r, a.nrhs == 1);
        U = unpack_link<RECON, R>(r);
      }
      su3_adj_mv(U, v, u);
      const R f = (MU == 3 && (w & 1) && neg) ? wgt : -wgt;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = acc[c] + f * u[c];
    }
  }
}

// Software-pipelined hops (as for the Wilson operator): the raw inputs of a
// hop (neighbour colour vector, link as stored, wrap count) go to one of two
// buffers, refilled alternately, so each wave has the next hop's loads in
// flight while it multiplies the current one; scheduling barriers hold the
// order. The hops of a pass are numbered I = 0 .. N-1 in the order of
// stag_dir (direction, then fat / long, then forward / backward), so the sums
// run in the same order.
template <typename S> struct StagIn {
  S v[6];
  S l[18];  // fat link, or the first RECON reals of a long link
  int w;
};

template <int I, int H0, int H1, int M0> struct StagHop {
  static constexpr int NH = H1 - H0 + 1;
  static constexpr int MU = M0 + I / (2 * NH);
  static constexpr int H = H0 + (I % (2 * NH)) / 2;  // 0 fat, 1 long
  static constexpr int DIR = (I % 2 == 0) ? 1 : -1;
  static constexpr int K = H == 0 ? 1 : 3;
};

template <int I, int H0, int H1, int M0, typename S, int RECON>
__device__ __forceinline__ void stag_fetch(const SArgs<S> &a, const Site &x, int s, int rhs, StagIn<S> &b) {
  using Hp = StagHop<I, H0, H1, M0>;
  constexpr int MU = Hp::MU, DIR = Hp::DIR;
  const int64_t vh = a.g.Vh, vs = vh * a.nrhs;
  const int n = hopk<MU, DIR * Hp::K>(a.g, x, &b.w);
  load_chunks_raw<S, 6, spinor_chunk<6>()>(a.in, vs, rhs_index(rhs, n, vh, a.rg), b.v);
  // forward: the link at x (x's parity); backward: at x - k mu (the other)
  const int lp = DIR > 0 ? x.p : 1 - x.p, ls = DIR > 0 ? s : n;
  if constexpr (Hp::H == 0)
    load_chunks_raw<S, 18, chunk_reals<S, 18>(), true>(a.fat + (int64_t)(2 * MU + lp) * vh * 18, vh, ls, b.l);
  else
    load_chunks_raw<S, RECON, chunk_reals<S, RECON>(), true>(a.lng + (int64_t)(2 * MU + lp) * vh * RECON, vh, ls,
                                                             b.l);
}

template <int I, int H0, int H1, int M0, typename S, typename R, int RECON>
__device__ __forceinline__ void stag_apply(const StagIn<S> &b, const R (&eta)[4], R cl, int neg, cpx<R> (&acc)[3]) {
  using Hp = StagHop<I, H0, H1, M0>;
  constexpr int MU = Hp::MU, NL = Hp::H == 0 ? 18 : RECON;
  cpx<R> v[3], u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = mk<R>(to_real<R>(b.v[2 * c]), to_real<R>(b.v[2 * c + 1]));
  R lv[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) lv[k] = to_real<R>(b.l[k]);
  const Link<R> U = unpack_link<NL, R>(lv);
  if constexpr (Hp::DIR > 0)
    su3_mv(U, v, u);
  else
    su3_adj_mv(U, v, u);
  const R wgt = Hp::H == 0 ? eta[MU] : eta[MU] * cl;
  const bool flip = MU == 3 && (b.w & 1) && neg;
  const R f = Hp::DIR > 0 ? (flip ? -wgt : wgt) : (flip ? wgt : -wgt);
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = acc[c] + f * u[c];
}

template <int I, int N, int H0, int H1, int M0, typename S, typename R, int RECON>
__device__ __forceinline__ void stag_pipe(const SArgs<S> &a, const Site &x, int s, int rhs, const R (&eta)[4], R cl,
                                          int neg, StagIn<S> (&b)[2], cpx<R> (&acc)[3]) {
  if constexpr (I < N) {
    __builtin_amdgcn_sched_barrier(0);
    stag_apply<I, H0, H1, M0, S, R, RECON>(b[I & 1], eta, cl, neg, acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (I + 2 < N) stag_fetch<I + 2, H0, H1, M0, S, RECON>(a, x, s, rhs, b[I & 1]);
    stag_pipe<I + 1, N, H0, H1, M0, S, R, RECON>(a, x, s, rhs, eta, cl, neg, b, acc);
  }
}

// Where the pipelined form pays (measured at 48^3x96): BF16 storage (18%
// faster) and FP32 (10% with recon 8, even with 12 and 18, where the compiler
// already issued each pass's loads early). FP16 runs 1% slower with it and
// FP64 the same, so both keep the per-hop form.
template <typename S> constexpr bool stag_pipelined() {
  return std::is_same<S, float>::value || std::is_same<S, bf16>::value;
}

// One pass computes the hops of types H0 .. H1 (0 fat, 1 long) along the
// directions M0 .. M1. 16-bit storage runs all 16 hops in one pass; FP32 runs
// two passes (fat, long) and FP64 four (fat and long, x/y and z/t), so that the
// loads of one pass fit in registers (16 hops in one pass spill). The FIRST
// pass writes coef * its hops (plus the xpay term); the others add theirs to
// the output in place.
template <typename S, typename R, int RECON, bool XPAY, int H0, int H1, int M0, int M1, bool FIRST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) stag_kernel(SArgs<S> a) {
  const RhsBlock rb = rhs_block(a.nrhs, a.rg);
  const int s = rb.s, rhs = rb.rhs;
  if (s >= a.g.Vh) return;
  const int64_t vs = (int64_t)a.g.Vh * a.nrhs;
  const int pidx = (int)rhs_index(rhs, s, a.g.Vh, a.rg);  // below 2^31 (checked on the host)
  const Site x = decode_site(a.g, s, a.parity);
  const int X0 = x.t[0] * a.g.B[0] + x.l[0], X1 = x.t[1] * a.g.B[1] + x.l[1], X2 = x.t[2] * a.g.B[2] + x.l[2];
  const R e1 = (X0 & 1) ? R(-1) : R(1);
  const R e2 = ((X0 + X1) & 1) ? R(-1) : R(1);
  const R e3 = ((X0 + X1 + X2) & 1) ? R(-1) : R(1);
  const R cl = (R)a.c_long;
  cpx<R> acc[3] = {mk<R>(0, 0), mk<R>(0, 0), mk<R>(0, 0)};
  if constexpr (stag_pipelined<S>()) {
    constexpr int N = 2 * (H1 - H0 + 1) * (M1 - M0 + 1);
    const R eta[4] = {R(1), e1, e2, e3};
    const int neg = a.g.bc_t < 0;
    StagIn<S> b[2];
    stag_fetch<0, H0, H1, M0, S, RECON>(a, x, s, rhs, b[0]);
    stag_fetch<1, H0, H1, M0, S, RECON>(a, x, s, rhs, b[1]);
    stag_pipe<0, N, H0, H1, M0, S, R, RECON>(a, x, s, rhs, eta, cl, neg, b, acc);
    __builtin_amdgcn_sched_barrier(0);
  } else {
    if constexpr (M0 <= 0 && 0 <= M1) stag_dir<0, H0, H1, S, R, RECON>(a, x, s, rhs, R(1), cl, acc);
    if constexpr (M0 <= 1 && 1 <= M1) stag_dir<1, H0, H1, S, R, RECON>(a, x, s, rhs, e1, cl, acc);
    if constexpr (M0 <= 2 && 2 <= M1) stag_dir<2, H0, H1, S, R, RECON>(a, x, s, rhs, e2, cl, acc);
    if constexpr (M0 <= 3 && 3 <= M1) stag_dir<3, H0, H1, S, R, RECON>(a, x, s, rhs, e3, cl, acc);
  }
  const R coef = (R)a.coef;
  R out[6];
  if constexpr (!FIRST) {
    cpx<R> prev[3];
    load_cvec<S, R>(a.out, vs, pidx, prev);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[2 * c] = fma(coef, acc[c].re, prev[c].re);
      out[2 * c + 1] = fma(coef, acc[c].im, prev[c].im);
    }
  } else if constexpr (XPAY) {
    cpx<R> xv[3];
    load_cvec<S, R>(a.xin, vs, pidx, xv);
    const R xc = (R)a.xcoef;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[2 * c] = fma(coef, acc[c].re, xc * xv[c].re);
      out[2 * c + 1] = fma(coef, acc[c].im, xc * xv[c].im);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[2 * c] = coef * acc[c].re;
      out[2 * c + 1] = coef * acc[c].im;
    }
  }
  store_spinor_reals<S, 6, R, true>(a.out, vs, pidx, out);
}

template <int P, int RECON>
static hipError_t launch_s2(const StagLaunch &l, hipStream_t st) {
  using S = typename Prec<P>::S;
  using R = typename Prec<P>::R;
  SArgs<S> a;
  a.g = l.g;
  a.out = (S *)l.out;
  a.in = (const S *)l.in;
  a.fat = (const S *)l.fat;
  a.lng = (const S *)l.lng;
  a.xin = (const S *)l.xin;
  a.parity = l.parity;
  a.coef = l.coef;
  a.xcoef = l.xcoef;
  a.c_long = l.c_long;
  a.nrhs = l.nrhs;
  a.rg = rhs_group(l.nrhs);
  const int bt = l.block_threads, nwg = rhs_grid(l.g.Vh, l.nrhs, bt);
  if constexpr (sizeof(S) == 2) {
    if (l.xin)
      hipLaunchKernelGGL((stag_kernel<S, R, RECON, true, 0, 1, 0, 3, true>), dim3(nwg), dim3(bt), 0, st, a);
    else
      hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 0, 1, 0, 3, true>), dim3(nwg), dim3(bt), 0, st, a);
  } else if constexpr (sizeof(S) == 4) {
    if (l.xin)
      hipLaunchKernelGGL((stag_kernel<S, R, RECON, true, 0, 0, 0, 3, true>), dim3(nwg), dim3(bt), 0, st, a);
    else
      hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 0, 0, 0, 3, true>), dim3(nwg), dim3(bt), 0, st, a);
    hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 1, 1, 0, 3, false>), dim3(nwg), dim3(bt), 0, st, a);
  } else {
    if (l.xin)
      hipLaunchKernelGGL((stag_kernel<S, R, RECON, true, 0, 0, 0, 1, true>), dim3(nwg), dim3(bt), 0, st, a);
    else
      hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 0, 0, 0, 1, true>), dim3(nwg), dim3(bt), 0, st, a);
    hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 0, 0, 2, 3, false>), dim3(nwg), dim3(bt), 0, st, a);
    hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 1, 1, 0, 1, false>), dim3(nwg), dim3(bt), 0, st, a);
    hipLaunchKernelGGL((stag_kernel<S, R, RECON, false, 1, 1, 2, 3, false>), dim3(nwg), dim3(bt), 0, st, a);
  }
  return hipGetLastError();
}

template <int P>
static hipError_t launch_s1(const StagLaunch &l, hipStream_t st) {
  switch (l.recon) {
    case 18: return launch_s2<P, 18>(l, st);
    case 12: return launch_s2<P, 12>(l, st);
    case 8:
      if constexpr (P == LQCD_F64 || P == LQCD_F32) return launch_s2<P, 8>(l, st);
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_staggered(const StagLaunch &l, hipStream_t st) {
  if (l.g.Vh == 0) return hipSuccess;
  switch (l.prec) {
    case LQCD_F64: return launch_s1<LQCD_F64>(l, st);
    case LQCD_F32: return launch_s1<LQCD_F32>(l, st);
    case LQCD_F16: return launch_s1<LQCD_F16>(l, st);
    case LQCD_BF16: return launch_s1<LQCD_BF16>(l, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lqcd
