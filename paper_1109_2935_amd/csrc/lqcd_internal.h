// Host-side internals shared by the library's translation units: the context,
// validated operator descriptions and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "lqcd.h"
#include "lqcd_device.h"

struct lqcd_context {
  int device = 0;
  std::string last_error;
  // reduction scratch: per-workgroup partials, and the result in pinned host
  // memory (red_host; red_host_dev is its device address)
  double *red_partials = nullptr;
  size_t red_partials_count = 0;
  double *red_host = nullptr;
  double *red_host_dev = nullptr;
  // general scratch vectors, grown on demand and reused between calls
  std::vector<void *> scratch;
  std::vector<size_t> scratch_bytes;
  std::vector<void *> retired;  // outgrown scratch buffers, freed with the context
  // autotuner results: launch parameter per kernel/shape key
  std::map<std::string, int> tuned;
  std::string tune_file;
  bool tune_enabled = true;
  bool tune_frozen = false;  // no timing runs: tuned or default launch parameters only
};

namespace lqcd {

constexpr int kMaxRed = 64;  // max values one reduction kernel returns

// Spin-colour reals per site of the action's spinor.
inline int spinor_reals(int action) { return action == LQCD_WILSON_CLOVER ? 24 : 6; }
inline size_t prec_bytes(int prec) { return prec == LQCD_F64 ? 8 : (prec == LQCD_F32 ? 4 : 2); }
// Bytes of one parity block of a per-site field of n reals (fixed-point
// storage adds an FP32 norm per site for spinors and the clover term).
inline size_t site_block_bytes(int prec, int n, size_t sites, bool normed) {
  return sites * n * prec_bytes(prec) + (prec == LQCD_HALF && normed ? sites * 4 : 0);
}

struct OpInfo {
  const lqcd_operator *op;
  Geom g;             // no cut
  int prec;
  int recon;
  int nsp;            // reals per site of the spinor
  size_t vh;          // sites per parity
  size_t spinor_bytes;  // one parity
};

// Validation helpers (return a status and set ctx->last_error).
lqcd_status set_error(lqcd_context *ctx, lqcd_status st, const std::string &msg);
lqcd_status check_op(lqcd_context *ctx, const lqcd_operator *op, OpInfo *info);
lqcd_status apply_cut(lqcd_context *ctx, const OpInfo &info, const int32_t *block, Geom *g);
lqcd_status hip_check(lqcd_context *ctx, hipError_t e, const char *what);
Geom make_geom(const int32_t dims[4], const int32_t tile[4], int bc_t);

// Scratch memory owned by the context (slot-indexed, grown on demand).
lqcd_status scratch(lqcd_context *ctx, int slot, size_t bytes, void **ptr);

// ---------------------------------------------------------------------------
// Wilson-clover kernels (wilson.hip)

enum WilsonMode {
  W_HOP = 0,        // out = coef * D in
  W_HOP_CLOV = 1,   // out = C (coef * D in)
  W_XPAY_CLOV = 2,  // out = C xin + coef * D in
  W_XPAY = 3        // out = xin + coef * D in
};

struct WilsonLaunch {
  Geom g;
  int prec, recon;
  void *out;
  const void *in;
  const void *gauge;
  const void *clov;  // clover block of the output parity (or nullptr)
  const void *xin;   // second input (modes 2, 3)
  int parity;        // output parity
  double coef;
  int dagger;
  int mode;
  double *partials;  // if non-null: per-segment <out,xin> (re, im) and <out,out> (nrhs = 1)
  int block_threads;
  int nrhs;          // right-hand sides (source-major)
  int mfma;          // link products on the matrix cores (16-bit, nrhs % 4 == 0, no partials)
};
hipError_t launch_wilson(const WilsonLaunch &w, hipStream_t st);

// Persistent multi-operator hopping term (mode W_HOP, coef 1).
struct BatchJob {
  Geom g;
  void *out;
  const void *in;
  const void *gauge;
  int parity;
  int nrhs;
};
struct BatchTune {
  int block_threads;  // 64..256
  int chunk;          // (site, rhs) pairs per work item: equal to block_threads
  int grid;           // workgroups of the persistent launch; 0: one workgroup per item, no queue
};
// mfma: 16-bit jobs whose source count is a multiple of 4 use the matrix-core link products
hipError_t launch_wilson_batch(int prec, int recon, const BatchJob *jobs, int njobs, int dagger, const BatchTune &t,
                               int mfma, unsigned *counter, hipStream_t st);

// Schwarz MR with each block resident in LDS: `steps` MR steps of the cut
// Schur operator on every block, or on the blocks of one colour (blocks equal
// to the tiles; 16-bit storage; 12 or 18 link reals) in one launch: x += K r0
// (x starts at zero, unread, if first).
struct SapLaunch {
  Geom g;  // cut equal to the tiles; colour -1 or 0 / 1
  int prec, recon;
  void *x;
  const void *r0;
  const void *gauge;
  const void *clov_inv_odd;
  const void *clov_even;
  double coef;  // -kappa^2
  double omega;
  int steps;
  int first;
  int xreg;  // x kept in registers (else read and written in memory each step)
  int wide;  // twice the threads, half the sites per thread (sap_block_wide_fits)
};
hipError_t launch_sap_block(const SapLaunch &l, hipStream_t st);
int sap_block_spt(int vt2);  // sites per thread of that launch; 0: blocks of vt2 sites do not fit
bool sap_block_wide_fits(int vt2);

hipError_t launch_clover_apply(const Geom &g, int prec, void *out, const void *in, const void *clov, int nrhs,
                               hipStream_t st);

// setup kernels
hipError_t launch_spinor_import(const Geom &g, int prec, int nsp, void *packed, const double *natural,
                                int parity, int nrhs, hipStream_t st);
hipError_t launch_spinor_export(const Geom &g, int prec, int nsp, double *natural, const void *packed,
                                int parity, int nrhs, hipStream_t st);
// out (layout go, precision pout) = scale * in (layout gi, precision pin): one
// parity block of the same lattice in two tilings
hipError_t launch_spinor_relayout(const Geom &go, int pout, void *out, const Geom &gi, int pin, const void *in, int nsp,
                                  int parity, int nrhs, double scale, hipStream_t st);
hipError_t launch_gauge_import(const Geom &g, int prec, int recon, void *packed, const double *natural,
                               int form_long, hipStream_t st);
hipError_t launch_clover_build(const Geom &g, int prec, double kappa, double csw, void *clov, void *clov_inv,
                               const double *natural_gauge, int *d_fail, hipStream_t st);

// ---------------------------------------------------------------------------
// staggered kernels (staggered.hip)

struct StagLaunch {
  Geom g;
  int prec, recon;
  void *out;
  const void *in;
  const void *fat;
  const void *lng;
  const void *xin;  // xpay input or nullptr
  int parity;
  double coef;      // multiplies D in
  double xcoef;     // multiplies xin
  double c_long;
  int block_threads;
  int nrhs;
};
hipError_t launch_staggered(const StagLaunch &s, hipStream_t st);

// ---------------------------------------------------------------------------
// BLAS and reductions (blas.hip). Vectors are flat arrays of n complex numbers
// stored as 2n reals in precision `prec`.

struct RedScratch {
  double *partials;  // one set of values per workgroup of the reducing launch
  double *result;    // their sum, written by a one-workgroup launch that follows it
  int max_wg;
};

// y = a*x + b*y  (a, b complex; x, y may differ in precision). If red: ||y||^2.
hipError_t blas_axpby(int px, const void *x, int py, void *y, size_t n, double ar, double ai, double br, double bi,
                      const RedScratch *red, hipStream_t st);
// y = s * x (conversion between precisions)
hipError_t blas_convert(int px, const void *x, int py, void *y, size_t n, double s, hipStream_t st);
// result[0] = ||x||^2
hipError_t blas_norm2(int px, const void *x, size_t n, const RedScratch &red, hipStream_t st);
// result[0..1] = <x, y>
hipError_t blas_cdot(int p, const void *x, const void *y, size_t n, const RedScratch &red, hipStream_t st);
// result[2i..2i+1] = <z_i, w>, i < k (all of precision p)
hipError_t blas_multi_cdot(int p, const void *const *z, int k, const void *w, size_t n, const RedScratch &red,
                           hipStream_t st);
// w -= sum_i beta_i z_i; result: ||w||^2, <w, r> (re, im)
hipError_t blas_multi_caxpy_dots(int p, const void *const *z, const double *beta, int k, void *w, const void *r,
                                 size_t n, const RedScratch &red, hipStream_t st);
// z *= 1/gamma; r -= alpha z (after scaling); result: ||r||^2
hipError_t blas_gcr_update(int p, void *z, void *r, size_t n, double inv_gamma, double ar, double ai,
                           const RedScratch &red, hipStream_t st);
// x (precision px) += sum_i chi_i p_i (precision pp)
hipError_t blas_multi_axpy_acc(int px, void *x, int pp, const void *const *p, const double *chi, int k, size_t n,
                               hipStream_t st);
// multi-shift CG: x_j += a_j p_j (x_j may be NULL), p_j = z_j r + b_j p_j, k <= 17
hipError_t blas_multishift_update(int prec, void *const *x, void *const *p, const double *a, const double *z,
                                  const double *b, int k, const void *r, size_t n, hipStream_t st);
// BiCGstab: p = r + b p + c v (b, c complex), all of precision prec
hipError_t blas_bicgstab_dir(int prec, const void *r, void *p, const void *v, size_t n, double br, double bi,
                             double cr, double ci, hipStream_t st);
// CG: x += a p; r -= a q; result ||r||^2 (x, p in px; r, q in pr)
hipError_t blas_cg_update(int px, void *x, const void *p, int pr, void *r, const void *q, size_t n, double a,
                          const RedScratch &red, hipStream_t st);

// Several right-hand sides (nrhs <= LQCD_MAX_CG_RHS) of vh sites and nsp
// reals per site each, in the multi-source layout; per-source coefficients
// a[j], b[j] and per-source results (result[j], or result[2j..2j+1]).
// y_j = a_j x_j + b_j y_j (y_j not read where b_j = 0); red: ||y_j||^2.
hipError_t blas_mrhs_axpby(int px, const void *x, int py, void *y, int64_t vh, int nsp, int nrhs, const double *a,
                           const double *b, const RedScratch *red, hipStream_t st);
// <x_j, y_j>
hipError_t blas_mrhs_cdot(int p, const void *x, const void *y, int64_t vh, int nsp, int nrhs, const RedScratch &red,
                          hipStream_t st);
// x_j += a_j p_j; r_j -= a_j q_j; ||r_j||^2 (sources with a_j = 0 are left as they are)
hipError_t blas_mrhs_cg_update(int px, void *x, const void *p, int pr, void *r, const void *q, int64_t vh, int nsp,
                               int nrhs, const double *a, const RedScratch &red, hipStream_t st);
// dst = src (bytes a multiple of 16), streaming
hipError_t blas_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t st);

}  // namespace lqcd
