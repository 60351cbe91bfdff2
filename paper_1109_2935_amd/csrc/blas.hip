// Level-1 linear algebra and global reductions for the solvers.
//
// Vectors are flat arrays of n complex numbers (2n reals) in any storage
// precision; the packed spinor layouts keep each (re, im) pair adjacent, so a
// field of any layout is such a vector. Arithmetic is done in FP32 (FP64 for
// FP64 vectors) and every reduction accumulates in FP64: per-thread sums, a
// wave64 butterfly, the waves of a workgroup through LDS into one partial per
// workgroup, then a one-workgroup launch that follows in stream order sums the
// partials in a fixed order. Results are therefore deterministic for a given
// n. (A last-workgroup-to-finish sum inside the launch needs a device-scope
// fence and an atomic ticket per workgroup; on gfx950 that cost about 35 us
// per 1024 workgroups, as much as streaming two 100 MB vectors.)
#include <type_traits>

#include "lqcd_internal.h"

namespace lqcd {

constexpr int kBT = 256;
constexpr int kMaxVec = 32;
constexpr int kMaxShiftVec = 17;  // 16 shifted systems and the base direction
constexpr int kMaxRhs = LQCD_MAX_CG_RHS;  // sources of one multi-source kernel

// 4 consecutive reals (2 complex numbers) of storage type S.
template <typename S> struct Quad;
template <> struct Quad<double> {
  __device__ static void load(const double *p, size_t i, double (&v)[4]) {
    const Chunk<double, 2> *q = reinterpret_cast<const Chunk<double, 2> *>(p + 4 * i);
    Chunk<double, 2> a = q[0], b = q[1];
    v[0] = a.v[0]; v[1] = a.v[1]; v[2] = b.v[0]; v[3] = b.v[1];
  }
  __device__ static void store(double *p, size_t i, const double (&v)[4]) {
    Chunk<double, 2> *q = reinterpret_cast<Chunk<double, 2> *>(p + 4 * i);
    Chunk<double, 2> a, b;
    a.v[0] = v[0]; a.v[1] = v[1]; b.v[0] = v[2]; b.v[1] = v[3];
    q[0] = a;
    q[1] = b;
  }
};
template <typename S> struct Quad {
  template <typename R> __device__ static void load(const S *p, size_t i, R (&v)[4]) {
    Chunk<S, 4> a = reinterpret_cast<const Chunk<S, 4> *>(p)[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = to_real<R>(a.v[k]);
  }
  template <typename R> __device__ static void store(S *p, size_t i, const R (&v)[4]) {
    Chunk<S, 4> a;
#pragma unroll
    for (int k = 0; k < 4; ++k) a.v[k] = Store<S>::from(v[k]);
    reinterpret_cast<Chunk<S, 4> *>(p)[i] = a;
  }
};

template <typename S> __device__ __forceinline__ void ld4(const S *p, size_t i, double (&v)[4]) {
  if constexpr (sizeof(S) == 8) {
    Quad<double>::load((const double *)p, i, v);
  } else {
    float f[4];
    Quad<S>::load(p, i, f);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = f[k];
  }
}
template <typename S> __device__ __forceinline__ void st4(S *p, size_t i, const double (&v)[4]) {
  if constexpr (sizeof(S) == 8) {
    Quad<double>::store((double *)p, i, v);
  } else {
    float f[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) f[k] = (float)v[k];
    Quad<S>::store(p, i, f);
  }
}

// The workgroup's partial sums of NR values: partials[blockIdx.x * NR + k].
template <int NR>
__device__ void grid_reduce(double (&v)[NR], RedScratch r) {
  __shared__ double lds[kBT / 64][NR];
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NR; ++k) lds[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < NR; ++k) {
      double t = 0;
      for (int w = 0; w < kBT / 64; ++w) t += lds[w][k];
      r.partials[(size_t)blockIdx.x * NR + k] = t;
    }
}

// One workgroup: result[j * NR + k] = the sum over the nblocks workgroups of
// partials[(w * nrows + j) * NR + k], thread t taking workgroups t, t + kBT,
// ... in order, then the wave butterfly and the waves in order.
template <int NR>
__global__ void __launch_bounds__(kBT) reduce_finish_kernel(const double *partials, int nblocks, int nrows,
                                                           double *result) {
  __shared__ double lds[kBT / 64][NR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < nrows; ++j) {
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0;
    for (int w = threadIdx.x; w < nblocks; w += kBT)
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] += partials[((size_t)w * nrows + j) * NR + k];
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < NR; ++k) lds[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = 0; k < NR; ++k) {
        double t = 0;
        for (int w = 0; w < kBT / 64; ++w) t += lds[w][k];
        result[j * NR + k] = t;
      }
  }
}

static int grid_for(size_t nquad, int max_wg) {
  size_t g = (nquad + kBT - 1) / kBT;
  if (g > (size_t)max_wg) g = max_wg;
  if (g < 1) g = 1;
  return (int)g;
}

// ---------------------------------------------------------------------------

template <typename SX, typename SY, bool RED>
__global__ void __launch_bounds__(kBT) axpby_kernel(const SX *x, SY *y, size_t nq, double ar, double ai, double br,
                                                   double bi, RedScratch r) {
  double acc[1] = {0};
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double xv[4], yv[4], o[4];
    ld4(x, i, xv);
    ld4(y, i, yv);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      o[2 * c] = ar * xv[2 * c] - ai * xv[2 * c + 1] + br * yv[2 * c] - bi * yv[2 * c + 1];
      o[2 * c + 1] = ar * xv[2 * c + 1] + ai * xv[2 * c] + br * yv[2 * c + 1] + bi * yv[2 * c];
    }
    st4(y, i, o);
    if (RED) {
      ld4(y, i, o);
      acc[0] += o[0] * o[0] + o[1] * o[1] + o[2] * o[2] + o[3] * o[3];
    }
  }
  if (RED) grid_reduce<1>(acc, r);
}

template <typename SX, typename SY>
__global__ void __launch_bounds__(kBT) convert_kernel(const SX *x, SY *y, size_t nq, double s) {
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double v[4];
    ld4(x, i, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] *= s;
    st4(y, i, v);
  }
}

template <typename S>
__global__ void __launch_bounds__(kBT) norm2_kernel(const S *x, size_t nq, RedScratch r) {
  double acc[1] = {0};
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double v[4];
    ld4(x, i, v);
    acc[0] += v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
  }
  grid_reduce<1>(acc, r);
}

struct VecPack {
  const void *p[kMaxVec];
  double c[2 * kMaxVec];
  int k;
};

// <z_i, w> for i < k (k <= 8 per launch)
// K is a template argument so that the loads of all K vectors are issued
// together, ahead of their products (with a run-time count each vector's
// load waited behind a branch).
template <typename S, int K>
__global__ void __launch_bounds__(kBT) multi_cdot_kernel(VecPack z, const S *w, size_t nq, RedScratch r) {
  double acc[2 * K];
#pragma unroll
  for (int k = 0; k < 2 * K; ++k) acc[k] = 0;
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double wv[4], zv[K][4];
    ld4(w, i, wv);
#pragma unroll
    for (int j = 0; j < K; ++j) ld4((const S *)z.p[j], i, zv[j]);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      acc[2 * j] += zv[j][0] * wv[0] + zv[j][1] * wv[1] + zv[j][2] * wv[2] + zv[j][3] * wv[3];
      acc[2 * j + 1] += zv[j][0] * wv[1] - zv[j][1] * wv[0] + zv[j][2] * wv[3] - zv[j][3] * wv[2];
    }
  }
  grid_reduce<2 * K>(acc, r);
}

// w -= sum_i beta_i z_i ; reduce ||w||^2, <w, rr>. K >= 0: that many vectors,
// their loads issued together (as in multi_cdot_kernel); K < 0: any count
// z.k, one vector after another.
template <typename S, int K>
__global__ void __launch_bounds__(kBT) multi_caxpy_dots_kernel(VecPack z, S *w, const S *rr, size_t nq, RedScratch r) {
  double acc[3] = {0, 0, 0};
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double wv[4];
    ld4(w, i, wv);
    auto sub = [&](int j, const double (&zv)[4]) {
      const double br = z.c[2 * j], bi = z.c[2 * j + 1];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        wv[2 * c] -= br * zv[2 * c] - bi * zv[2 * c + 1];
        wv[2 * c + 1] -= br * zv[2 * c + 1] + bi * zv[2 * c];
      }
    };
    if constexpr (K >= 0) {
      double zv[K > 0 ? K : 1][4];
#pragma unroll
      for (int j = 0; j < K; ++j) ld4((const S *)z.p[j], i, zv[j]);
#pragma unroll
      for (int j = 0; j < K; ++j) sub(j, zv[j]);
    } else {
      for (int j = 0; j < z.k; ++j) {
        double zv[4];
        ld4((const S *)z.p[j], i, zv);
        sub(j, zv);
      }
    }
    st4(w, i, wv);
    ld4(w, i, wv);
    double rv[4];
    ld4(rr, i, rv);
    acc[0] += wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2] + wv[3] * wv[3];
    acc[1] += wv[0] * rv[0] + wv[1] * rv[1] + wv[2] * rv[2] + wv[3] * rv[3];
    acc[2] += wv[0] * rv[1] - wv[1] * rv[0] + wv[2] * rv[3] - wv[3] * rv[2];
  }
  grid_reduce<3>(acc, r);
}

// z *= inv_gamma ; r -= alpha z ; reduce ||r||^2
template <typename S>
__global__ void __launch_bounds__(kBT) gcr_update_kernel(S *z, S *rv, size_t nq, double ig, double ar, double ai,
                                                        RedScratch r) {
  double acc[1] = {0};
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double zv[4], x[4];
    ld4(z, i, zv);
#pragma unroll
    for (int k = 0; k < 4; ++k) zv[k] *= ig;
    st4(z, i, zv);
    ld4(z, i, zv);
    ld4(rv, i, x);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      x[2 * c] -= ar * zv[2 * c] - ai * zv[2 * c + 1];
      x[2 * c + 1] -= ar * zv[2 * c + 1] + ai * zv[2 * c];
    }
    st4(rv, i, x);
    ld4(rv, i, x);
    acc[0] += x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
  }
  grid_reduce<1>(acc, r);
}

// x += sum_i chi_i p_i
template <typename SX, typename SP>
__global__ void __launch_bounds__(kBT) multi_axpy_acc_kernel(SX *x, VecPack p, size_t nq) {
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double xv[4];
    ld4(x, i, xv);
    for (int j = 0; j < p.k; ++j) {
      double pv[4];
      ld4((const SP *)p.p[j], i, pv);
      const double cr = p.c[2 * j], ci = p.c[2 * j + 1];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        xv[2 * c] += cr * pv[2 * c] - ci * pv[2 * c + 1];
        xv[2 * c + 1] += cr * pv[2 * c + 1] + ci * pv[2 * c];
      }
    }
    st4(x, i, xv);
  }
}

// BiCGstab search direction: p = r + beta (p - omega v), i.e.
// p = r + beta p + c v with c = -beta omega (complex coefficients).
template <typename S>
__global__ void __launch_bounds__(kBT) bicgstab_dir_kernel(const S *r, S *p, const S *v, size_t nq, double br,
                                                          double bi, double cr, double ci) {
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double rv[4], pv[4], vv[4], o[4];
    ld4(r, i, rv);
    ld4(p, i, pv);
    ld4(v, i, vv);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      o[2 * c] = rv[2 * c] + br * pv[2 * c] - bi * pv[2 * c + 1] + cr * vv[2 * c] - ci * vv[2 * c + 1];
      o[2 * c + 1] = rv[2 * c + 1] + br * pv[2 * c + 1] + bi * pv[2 * c] + cr * vv[2 * c + 1] + ci * vv[2 * c];
    }
    st4(p, i, o);
  }
}

// Multi-shift CG update (eq. (4)): for every shifted system j,
//   x_j += a_j p_j (skipped where x_j is NULL), then p_j = z_j r + b_j p_j,
// all from one read of r. Real coefficients (Hermitian positive-definite
// systems).
struct ShiftPack {
  void *x[kMaxShiftVec];
  void *p[kMaxShiftVec];
  double a[kMaxShiftVec], z[kMaxShiftVec], b[kMaxShiftVec];
  int k;
};

template <typename S>
__global__ void __launch_bounds__(kBT) multishift_update_kernel(ShiftPack sp, const S *r, size_t nq) {
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double rv[4];
    ld4(r, i, rv);
    for (int j = 0; j < sp.k; ++j) {
      double pv[4];
      ld4((const S *)sp.p[j], i, pv);
      if (sp.x[j]) {
        double xv[4];
        ld4((const S *)sp.x[j], i, xv);
#pragma unroll
        for (int c = 0; c < 4; ++c) xv[c] += sp.a[j] * pv[c];
        st4((S *)sp.x[j], i, xv);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) pv[c] = sp.z[j] * rv[c] + sp.b[j] * pv[c];
      st4((S *)sp.p[j], i, pv);
    }
  }
}

// x += a p ; r -= a q ; reduce ||r||^2
template <typename SX, typename SR>
__global__ void __launch_bounds__(kBT) cg_update_kernel(SX *x, const SX *p, SR *rv, const SR *q, size_t nq, double a,
                                                       RedScratch r) {
  double acc[1] = {0};
  for (size_t i = (size_t)blockIdx.x * kBT + threadIdx.x; i < nq; i += (size_t)gridDim.x * kBT) {
    double xv[4], pv[4], rr[4], qv[4];
    ld4(x, i, xv);
    ld4(p, i, pv);
#pragma unroll
    for (int k = 0; k < 4; ++k) xv[k] += a * pv[k];
    st4(x, i, xv);
    ld4(rv, i, rr);
    ld4(q, i, qv);
#pragma unroll
    for (int k = 0; k < 4; ++k) rr[k] -= a * qv[k];
    st4(rv, i, rr);
    ld4(rv, i, rr);
    acc[0] += rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2] + rr[3] * rr[3];
  }
  grid_reduce<1>(acc, r);
}

// ---------------------------------------------------------------------------
// dispatch

template <typename F> static hipError_t dispatch1(int p, F &&f) {
  switch (p) {
    case LQCD_F64: return f((double *)nullptr);
    case LQCD_F32: return f((float *)nullptr);
    case LQCD_F16: return f((_Float16 *)nullptr);
    case LQCD_BF16: return f((bf16 *)nullptr);
  }
  return hipErrorInvalidValue;
}

template <typename F> static hipError_t dispatch2(int p1, int p2, F &&f) {
  return dispatch1(p1, [&](auto t1) { return dispatch1(p2, [&](auto t2) { return f(t1, t2); }); });
}

// f(std::integral_constant<int, k>) for LO <= k <= HI (the caller checks the range)
template <int LO, int HI, typename F> static hipError_t with_count(int k, F &&f) {
  if constexpr (LO > HI) {
    return hipErrorInvalidValue;
  } else {
    if (k == LO) return f(std::integral_constant<int, LO>{});
    return with_count<LO + 1, HI>(k, f);
  }
}

// The one-workgroup sum over the nblocks partials of a reducing launch (nr
// values per row, nrows rows) into red.result, in stream order after it.
static hipError_t finish_sums(int nr, int nblocks, int nrows, const RedScratch &red, hipStream_t st) {
  return with_count<1, 16>(nr, [&](auto c) -> hipError_t {
    hipLaunchKernelGGL((reduce_finish_kernel<decltype(c)::value>), dim3(1), dim3(kBT), 0, st,
                       (const double *)red.partials, nblocks, nrows, red.result);
    return hipGetLastError();
  });
}

#define T1 std::remove_pointer_t<decltype(t1)>
#define T2 std::remove_pointer_t<decltype(t2)>

static const RedScratch kNoRed = {nullptr, nullptr, 1024};

hipError_t blas_axpby(int px, const void *x, int py, void *y, size_t n, double ar, double ai, double br, double bi,
                      const RedScratch *red, hipStream_t st) {
  const size_t nq = n / 2;
  const int g = grid_for(nq, red ? red->max_wg : 1024);
  const RedScratch r = red ? *red : kNoRed;
  const hipError_t e = dispatch2(px, py, [&](auto t1, auto t2) -> hipError_t {
    if (red)
      hipLaunchKernelGGL((axpby_kernel<T1, T2, true>), dim3(g), dim3(kBT), 0, st, (const T1 *)x, (T2 *)y, nq, ar, ai, br,
                         bi, r);
    else
      hipLaunchKernelGGL((axpby_kernel<T1, T2, false>), dim3(g), dim3(kBT), 0, st, (const T1 *)x, (T2 *)y, nq, ar, ai,
                         br, bi, r);
    return hipGetLastError();});
  if (e != hipSuccess || !red) return e;
  return finish_sums(1, g, 1, *red, st);
}

hipError_t blas_convert(int px, const void *x, int py, void *y, size_t n, double s, hipStream_t st) {
  const size_t nq = n / 2;
  const int g = grid_for(nq, 4096);
  return dispatch2(px, py, [&](auto t1, auto t2) -> hipError_t {
    hipLaunchKernelGGL((convert_kernel<T1, T2>), dim3(g), dim3(kBT), 0, st, (const T1 *)x, (T2 *)y, nq, s);
    return hipGetLastError();});
}

hipError_t blas_norm2(int px, const void *x, size_t n, const RedScratch &red, hipStream_t st) {
  const size_t nq = n / 2;
  const int g = grid_for(nq, red.max_wg);
  const hipError_t e = dispatch1(px, [&](auto t1) -> hipError_t {
    hipLaunchKernelGGL((norm2_kernel<T1>), dim3(g), dim3(kBT), 0, st, (const T1 *)x, nq, red);
    return hipGetLastError();});
  return e != hipSuccess ? e : finish_sums(1, g, 1, red, st);
}

hipError_t blas_cdot(int p, const void *x, const void *y, size_t n, const RedScratch &red, hipStream_t st) {
  const void *z[1] = {x};
  return blas_multi_cdot(p, z, 1, y, n, red, st);
}

hipError_t blas_multi_cdot(int p, const void *const *z, int k, const void *w, size_t n, const RedScratch &red,
                           hipStream_t st) {
  if (k < 1 || k > 8) return hipErrorInvalidValue;
  VecPack pk;
  pk.k = k;
  for (int j = 0; j < k; ++j) pk.p[j] = z[j];
  const size_t nq = n / 2;
  const int g = grid_for(nq, red.max_wg);
  const hipError_t e = dispatch1(p, [&](auto t1) -> hipError_t {
    return with_count<1, 8>(k, [&](auto kc) {
      hipLaunchKernelGGL((multi_cdot_kernel<T1, decltype(kc)::value>), dim3(g), dim3(kBT), 0, st, pk, (const T1 *)w,
                         nq, red);
      return hipGetLastError();
    });});
  return e != hipSuccess ? e : finish_sums(2 * k, g, 1, red, st);
}

hipError_t blas_multi_caxpy_dots(int p, const void *const *z, const double *beta, int k, void *w, const void *r,
                                 size_t n, const RedScratch &red, hipStream_t st) {
  if (k < 0 || k > kMaxVec) return hipErrorInvalidValue;
  VecPack pk;
  pk.k = k;
  for (int j = 0; j < k; ++j) {
    pk.p[j] = z[j];
    pk.c[2 * j] = beta[2 * j];
    pk.c[2 * j + 1] = beta[2 * j + 1];
  }
  const size_t nq = n / 2;
  const int g = grid_for(nq, red.max_wg);
  const hipError_t e = dispatch1(p, [&](auto t1) -> hipError_t {
    if (k > 16) {
      hipLaunchKernelGGL((multi_caxpy_dots_kernel<T1, -1>), dim3(g), dim3(kBT), 0, st, pk, (T1 *)w, (const T1 *)r, nq,
                         red);
      return hipGetLastError();
    }
    return with_count<0, 16>(k, [&](auto kc) {
      hipLaunchKernelGGL((multi_caxpy_dots_kernel<T1, decltype(kc)::value>), dim3(g), dim3(kBT), 0, st, pk, (T1 *)w,
                         (const T1 *)r, nq, red);
      return hipGetLastError();
    });});
  return e != hipSuccess ? e : finish_sums(3, g, 1, red, st);
}

hipError_t blas_gcr_update(int p, void *z, void *r, size_t n, double inv_gamma, double ar, double ai,
                           const RedScratch &red, hipStream_t st) {
  const size_t nq = n / 2;
  const int g = grid_for(nq, red.max_wg);
  const hipError_t e = dispatch1(p, [&](auto t1) -> hipError_t {
    hipLaunchKernelGGL((gcr_update_kernel<T1>), dim3(g), dim3(kBT), 0, st, (T1 *)z, (T1 *)r, nq, inv_gamma, ar, ai,
                       red);
    return hipGetLastError();});
  return e != hipSuccess ? e : finish_sums(1, g, 1, red, st);
}

hipError_t blas_multi_axpy_acc(int px, void *x, int pp, const void *const *p, const double *chi, int k, size_t n,
                               hipStream_t st) {
  if (k < 1 || k > kMaxVec) return hipErrorInvalidValue;
  VecPack pk;
  pk.k = k;
  for (int j = 0; j < k; ++j) {
    pk.p[j] = p[j];
    pk.c[2 * j] = chi[2 * j];
    pk.c[2 * j + 1] = chi[2 * j + 1];
  }
  const size_t nq = n / 2;
  const int g = grid_for(nq, 4096);
  return dispatch2(px, pp, [&](auto t1, auto t2) -> hipError_t {
    hipLaunchKernelGGL((multi_axpy_acc_kernel<T1, T2>), dim3(g), dim3(kBT), 0, st, (T1 *)x, pk, nq);
    return hipGetLastError();});
}

hipError_t blas_bicgstab_dir(int prec, const void *r, void *p, const void *v, size_t n, double br, double bi,
                             double cr, double ci, hipStream_t st) {
  const size_t nq = n / 2;
  const int g = grid_for(nq, 4096);
  return dispatch1(prec, [&](auto t1) -> hipError_t {
    hipLaunchKernelGGL((bicgstab_dir_kernel<T1>), dim3(g), dim3(kBT), 0, st, (const T1 *)r, (T1 *)p, (const T1 *)v,
                       nq, br, bi, cr, ci);
    return hipGetLastError();});
}

hipError_t blas_multishift_update(int prec, void *const *x, void *const *p, const double *a, const double *z,
                                  const double *b, int k, const void *r, size_t n, hipStream_t st) {
  if (k < 1 || k > kMaxShiftVec) return hipErrorInvalidValue;
  ShiftPack sp;
  sp.k = k;
  for (int j = 0; j < k; ++j) {
    sp.x[j] = x[j];
    sp.p[j] = p[j];
    sp.a[j] = a[j];
    sp.z[j] = z[j];
    sp.b[j] = b[j];
  }
  const size_t nq = n / 2;
  const int g = grid_for(nq, 4096);
  return dispatch1(prec, [&](auto t1) -> hipError_t {
    hipLaunchKernelGGL((multishift_update_kernel<T1>), dim3(g), dim3(kBT), 0, st, sp, (const T1 *)r, nq);
    return hipGetLastError();});
}

hipError_t blas_cg_update(int px, void *x, const void *p, int pr, void *r, const void *q, size_t n, double a,
                          const RedScratch &red, hipStream_t st) {
  const size_t nq = n / 2;
  const int g = grid_for(nq, red.max_wg);
  const hipError_t e = dispatch2(px, pr, [&](auto t1, auto t2) -> hipError_t {
    hipLaunchKernelGGL((cg_update_kernel<T1, T2>), dim3(g), dim3(kBT), 0, st, (T1 *)x, (const T1 *)p, (T2 *)r,
                       (const T2 *)q, nq, a, red);
    return hipGetLastError();});
  return e != hipSuccess ? e : finish_sums(1, g, 1, red, st);
}


// ---------------------------------------------------------------------------
// Several right-hand sides, in the multi-source layout (blocks of R sources,
// lqcd_device.h): packed index p of a parity block holds site (p / R) mod vh
// of source R ((p / R) / vh) + p mod R. Threads walk p in order, one source
// group (R vh consecutive indices) after the other, each thread with all the
// reals of its index, so every access is coalesced; the grid stride is a
// multiple of R, so a thread's source within its group never changes and
// per-source sums need no per-thread arrays. Each source has its own
// coefficients and its own reductions, in a fixed order: per-thread sums, a
// wave butterfly over the lanes of one source, the waves through LDS, then the
// last workgroup of the launch sums each source's per-workgroup partials in
// workgroup order.

struct RhsCoef {
  double a[kMaxRhs], b[kMaxRhs];
};

// After a source group: partials[(blockIdx.x * nrhs + src0 + j) * NR + k] for
// the R sources src0 + j of the group (v is reset).
template <int NR>
__device__ __forceinline__ void group_partials(double (&v)[NR], int R, int src0, int nrhs, double *partials) {
  __shared__ double lds[kBT / 64][4][NR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NR; ++k)
    for (int off = 32; off >= R; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  if (lane < R)
#pragma unroll
    for (int k = 0; k < NR; ++k) lds[wave][lane][k] = v[k];
  __syncthreads();
  if ((int)threadIdx.x < R)
    for (int k = 0; k < NR; ++k) {
      double t = 0;
      for (int w = 0; w < kBT / 64; ++w) t += lds[w][threadIdx.x][k];
      partials[((size_t)blockIdx.x * nrhs + src0 + threadIdx.x) * NR + k] = t;
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0;
}

// y_j = a_j x_j + b_j y_j (y not read where b_j = 0); RED: ||y_j||^2 of the stored y.
template <typename SX, typename SY, int NSP, bool RED>
__global__ void __launch_bounds__(kBT) mrhs_axpby_kernel(const SX *x, SY *y, int64_t vh, int nrhs, RhsCoef c,
                                                        RedScratch r) {
  const int R = rhs_group(nrhs);
  const int64_t stride = vh * nrhs, gsize = (int64_t)R * vh, step = (int64_t)gridDim.x * kBT;
  double acc[1] = {0};
  for (int g = 0; g < nrhs / R; ++g) {
    const int j = g * R + (int)(threadIdx.x % R);
    const double a = c.a[j], b = c.b[j];
    for (int64_t p = g * gsize + (int64_t)blockIdx.x * kBT + threadIdx.x; p < (g + 1) * gsize; p += step) {
      double xv[NSP], yv[NSP];
      load_spinor_reals<SX, NSP, double>(x, stride, p, xv);
      if (b != 0) {
        load_spinor_reals<SY, NSP, double>(y, stride, p, yv);
#pragma unroll
        for (int k = 0; k < NSP; ++k) yv[k] = a * xv[k] + b * yv[k];
      } else {
#pragma unroll
        for (int k = 0; k < NSP; ++k) yv[k] = a * xv[k];
      }
      store_spinor_reals<SY, NSP, double>(y, stride, p, yv);
      if (RED) {
        load_spinor_reals<SY, NSP, double>(y, stride, p, yv);
#pragma unroll
        for (int k = 0; k < NSP; ++k) acc[0] += yv[k] * yv[k];
      }
    }
    if (RED) group_partials<1>(acc, R, g * R, nrhs, r.partials);
  }
}

// <x_j, y_j> (re, im) per source
template <typename S, int NSP>
__global__ void __launch_bounds__(kBT) mrhs_cdot_kernel(const S *x, const S *y, int64_t vh, int nrhs, RedScratch r) {
  const int R = rhs_group(nrhs);
  const int64_t stride = vh * nrhs, gsize = (int64_t)R * vh, step = (int64_t)gridDim.x * kBT;
  double acc[2] = {0, 0};
  for (int g = 0; g < nrhs / R; ++g) {
    for (int64_t p = g * gsize + (int64_t)blockIdx.x * kBT + threadIdx.x; p < (g + 1) * gsize; p += step) {
      double xv[NSP], yv[NSP];
      load_spinor_reals<S, NSP, double>(x, stride, p, xv);
      load_spinor_reals<S, NSP, double>(y, stride, p, yv);
#pragma unroll
      for (int k = 0; k < NSP / 2; ++k) {
        acc[0] += xv[2 * k] * yv[2 * k] + xv[2 * k + 1] * yv[2 * k + 1];
        acc[1] += xv[2 * k] * yv[2 * k + 1] - xv[2 * k + 1] * yv[2 * k];
      }
    }
    group_partials<2>(acc, R, g * R, nrhs, r.partials);
  }
}

// x_j += a_j p_j ; r_j -= a_j q_j ; ||r_j||^2 of the stored r (sources with
// a_j = 0 are only read)
template <typename SX, typename SR, int NSP>
__global__ void __launch_bounds__(kBT) mrhs_cg_update_kernel(SX *x, const SX *p, SR *rv, const SR *q, int64_t vh,
                                                            int nrhs, RhsCoef c, RedScratch r) {
  const int R = rhs_group(nrhs);
  const int64_t stride = vh * nrhs, gsize = (int64_t)R * vh, step = (int64_t)gridDim.x * kBT;
  double acc[1] = {0};
  for (int g = 0; g < nrhs / R; ++g) {
    const double a = c.a[g * R + (int)(threadIdx.x % R)];
    for (int64_t i = g * gsize + (int64_t)blockIdx.x * kBT + threadIdx.x; i < (g + 1) * gsize; i += step) {
      double u[NSP], w[NSP];
      if (a != 0) {
        load_spinor_reals<SX, NSP, double>(x, stride, i, u);
        load_spinor_reals<SX, NSP, double>(p, stride, i, w);
#pragma unroll
        for (int k = 0; k < NSP; ++k) u[k] += a * w[k];
        store_spinor_reals<SX, NSP, double>(x, stride, i, u);
        load_spinor_reals<SR, NSP, double>(rv, stride, i, u);
        load_spinor_reals<SR, NSP, double>(q, stride, i, w);
#pragma unroll
        for (int k = 0; k < NSP; ++k) u[k] -= a * w[k];
        store_spinor_reals<SR, NSP, double>(rv, stride, i, u);
      }
      load_spinor_reals<SR, NSP, double>(rv, stride, i, u);
#pragma unroll
      for (int k = 0; k < NSP; ++k) acc[0] += u[k] * u[k];
    }
    group_partials<1>(acc, R, g * R, nrhs, r.partials);
  }
}

static int mrhs_grid(int64_t vh, int nrhs, int nr, const RedScratch *red) {
  int64_t g = (vh * rhs_group(nrhs) + kBT - 1) / kBT;
  const int64_t cap = red ? (int64_t)red->max_wg * kMaxRed / ((int64_t)nrhs * nr) : 4096;
  if (g > cap) g = cap;
  if (g > 4096) g = 4096;
  return g < 1 ? 1 : (int)g;
}

// The per-site kernels also take 16-bit fixed point (each thread owns a
// site's reals, so it can form the site norm); the element-wise kernels above
// do not.
template <typename F> static hipError_t dispatch1h(int p, F &&f) {
  if (p == LQCD_HALF) return f((fx16 *)nullptr);
  return dispatch1(p, f);
}
template <typename F> static hipError_t dispatch2h(int p1, int p2, F &&f) {
  return dispatch1h(p1, [&](auto t1) { return dispatch1h(p2, [&](auto t2) { return f(t1, t2); }); });
}

template <typename F> static hipError_t dispatch_nsp(int nsp, F &&f) {
  if (nsp == 24) return f(std::integral_constant<int, 24>());
  if (nsp == 6) return f(std::integral_constant<int, 6>());
  return hipErrorInvalidValue;
}

hipError_t blas_mrhs_axpby(int px, const void *x, int py, void *y, int64_t vh, int nsp, int nrhs, const double *a,
                           const double *b, const RedScratch *red, hipStream_t st) {
  if (nrhs < 1 || nrhs > kMaxRhs || (red && nrhs > kMaxRed)) return hipErrorInvalidValue;
  RhsCoef c;
  for (int j = 0; j < nrhs; ++j) {
    c.a[j] = a[j];
    c.b[j] = b[j];
  }
  const dim3 grid(mrhs_grid(vh, nrhs, 1, red));
  const RedScratch r = red ? *red : kNoRed;
  const hipError_t e = dispatch2h(px, py, [&](auto t1, auto t2) -> hipError_t {
    return dispatch_nsp(nsp, [&](auto ns) -> hipError_t {
      constexpr int NS = decltype(ns)::value;
      if (red)
        hipLaunchKernelGGL((mrhs_axpby_kernel<T1, T2, NS, true>), grid, dim3(kBT), 0, st, (const T1 *)x, (T2 *)y, vh,
                           nrhs, c, r);
      else
        hipLaunchKernelGGL((mrhs_axpby_kernel<T1, T2, NS, false>), grid, dim3(kBT), 0, st, (const T1 *)x, (T2 *)y, vh,
                           nrhs, c, r);
      return hipGetLastError();
    });
  });
  if (e != hipSuccess || !red) return e;
  return finish_sums(1, (int)grid.x, nrhs, *red, st);
}

hipError_t blas_mrhs_cdot(int p, const void *x, const void *y, int64_t vh, int nsp, int nrhs, const RedScratch &red,
                          hipStream_t st) {
  if (nrhs < 1 || 2 * nrhs > kMaxRed) return hipErrorInvalidValue;
  const dim3 grid(mrhs_grid(vh, nrhs, 2, &red));
  const hipError_t e = dispatch1h(p, [&](auto t1) -> hipError_t {
    return dispatch_nsp(nsp, [&](auto ns) -> hipError_t {
      constexpr int NS = decltype(ns)::value;
      hipLaunchKernelGGL((mrhs_cdot_kernel<T1, NS>), grid, dim3(kBT), 0, st, (const T1 *)x, (const T1 *)y, vh, nrhs,
                         red);
      return hipGetLastError();
    });
  });
  return e != hipSuccess ? e : finish_sums(2, (int)grid.x, nrhs, red, st);
}

hipError_t blas_mrhs_cg_update(int px, void *x, const void *p, int pr, void *r, const void *q, int64_t vh, int nsp,
                               int nrhs, const double *a, const RedScratch &red, hipStream_t st) {
  if (nrhs < 1 || nrhs > kMaxRhs || nrhs > kMaxRed) return hipErrorInvalidValue;
  RhsCoef c;
  for (int j = 0; j < nrhs; ++j) {
    c.a[j] = a[j];
    c.b[j] = 0;
  }
  const dim3 grid(mrhs_grid(vh, nrhs, 1, &red));
  const hipError_t e = dispatch2h(px, pr, [&](auto t1, auto t2) -> hipError_t {
    return dispatch_nsp(nsp, [&](auto ns) -> hipError_t {
      constexpr int NS = decltype(ns)::value;
      hipLaunchKernelGGL((mrhs_cg_update_kernel<T1, T2, NS>), grid, dim3(kBT), 0, st, (T1 *)x, (const T1 *)p, (T2 *)r,
                         (const T2 *)q, vh, nrhs, c, red);
      return hipGetLastError();
    });
  });
  return e != hipSuccess ? e : finish_sums(1, (int)grid.x, nrhs, red, st);
}

// ---------------------------------------------------------------------------
// Streaming copy: 16-byte non-temporal loads and stores, grid-stride, four
// loads in flight per thread before their stores (the fastest of the forms
// measured on gfx950: 5.8 TB/s for 2 GiB with 16384 workgroups). The measured
// ceiling of a read-once/write-once kernel, and the known-size kernel that
// calibrates the profiler's byte counters.
typedef RawVec<16>::T u32x4;
__global__ void __launch_bounds__(kBT) stream_copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                         size_t n16) {
  constexpr int U = 4;
  const size_t step = (size_t)gridDim.x * kBT * U;
  for (size_t i = (size_t)blockIdx.x * kBT * U + threadIdx.x; i < n16; i += step) {
    u32x4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (i + k * kBT < n16) v[k] = __builtin_nontemporal_load(src + i + k * kBT);
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (i + k * kBT < n16) __builtin_nontemporal_store(v[k], dst + i + k * kBT);
  }
}

hipError_t blas_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t st) {
  if (bytes % 16) return hipErrorInvalidValue;
  const size_t n16 = bytes / 16;
  if (!n16) return hipSuccess;
  size_t g = (n16 + 4 * kBT - 1) / (4 * kBT);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)g), dim3(kBT), 0, st, (const u32x4 *)src, (u32x4 *)dst, n16);
  return hipGetLastError();
}

}  // namespace lqcd
