// Solvers: mixed-precision GCR-DD (Algorithm 1, Section VIII-A) and CG with
// reliable updates (Section III-A), as host loops over the device kernels.
// Reductions come back to the host once per step; all scalars of the
// recurrences are kept in FP64 on the host.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <vector>

#include "lqcd_internal.h"
#include "lqcd_ops.h"

using namespace lqcd;
using cd = std::complex<double>;

#define TRY(expr)                    \
  do {                               \
    lqcd_status _s = (expr);         \
    if (_s != LQCD_OK) return _s;    \
  } while (0)

namespace {

// The same physical system; `any_tile`: the memory tiles may differ.
bool same_system(const lqcd_operator *a, const lqcd_operator *b, bool any_tile = false) {
  if (a->action != b->action || a->bc_t != b->bc_t) return false;
  for (int m = 0; m < 4; ++m)
    if (a->dims[m] != b->dims[m] || (!any_tile && a->tile[m] != b->tile[m])) return false;
  if (a->action == LQCD_WILSON_CLOVER) return a->kappa == b->kappa && a->csw == b->csw;
  return a->mass == b->mass && a->c_long == b->c_long;
}

bool same_tile(const OpInfo &a, const OpInfo &b) {
  for (int m = 0; m < 4; ++m)
    if (a.op->tile[m] != b.op->tile[m]) return false;
  return true;
}

struct Solver {
  lqcd_context *ctx;
  hipStream_t st;
  int slot;  // next free scratch slot
  // Every work vector is given at least this many bytes (the size of the
  // system's FP64 vectors), so that solves of other precisions that follow
  // find their slots large enough and never reallocate.
  size_t min_bytes = 0;
  lqcd_status vec(size_t bytes, void **p) { return scratch(ctx, slot++, std::max(bytes, min_bytes), p); }
  lqcd_status result(int n, double *out) { return read_result(ctx, st, n, out); }
  RedScratch red() { return red_scratch(ctx); }
  lqcd_status hip(hipError_t e, const char *what) { return hip_check(ctx, e, what); }
};

// number of complex entries of one parity spinor
size_t ncomplex(const OpInfo &i) { return i.vh * i.nsp / 2; }

// y = b - y, returns ||y||^2 (same precision p)
lqcd_status residual_from(Solver &S, int p, const void *b, void *y, size_t n, double *rr) {
  RedScratch r = S.red();
  TRY(S.hip(blas_axpby(p, b, p, y, n, 1.0, 0.0, -1.0, 0.0, &r, S.st), "axpby"));
  return S.result(1, rr);
}

// Wilson even-odd source bhat = b_e + kappa D_eo A_oo^-1 b_o.
// nrhs sources: b_full holds the even blocks of all sources, then the odd ones.
lqcd_status wilson_schur_source(Solver &S, const OpInfo &hi, void *bhat, const void *b_full, void *tmp, int nrhs = 1) {
  const char *be = (const char *)b_full, *bo = be + hi.spinor_bytes * nrhs;
  TRY(S.hip(launch_clover_apply(hi.g, hi.prec, tmp, bo, clover_block(hi, hi.op->clover_inv, 1), nrhs, S.st),
            "clover"));
  return wilson_hop(S.ctx, hi, hi.g, W_XPAY, bhat, tmp, be, nullptr, 0, hi.op->kappa, 0, nullptr, S.st, nrhs);
}

// x_o = A_oo^-1 (b_o + kappa D_oe x_e), then the true full residual ||b - M x|| / ||b||.
lqcd_status wilson_finish(Solver &S, const OpInfo &hi, void *x_full, const void *b_full, void *tmp, void *y,
                          double bnorm, double *true_res) {
  char *xe = (char *)x_full, *xo = xe + hi.spinor_bytes;
  const char *be = (const char *)b_full, *bo = be + hi.spinor_bytes;
  const lqcd_operator *op = hi.op;
  TRY(wilson_hop(S.ctx, hi, hi.g, W_XPAY, tmp, xe, bo, nullptr, 1, op->kappa, 0, nullptr, S.st));
  TRY(S.hip(launch_clover_apply(hi.g, hi.prec, xo, tmp, clover_block(hi, op->clover_inv, 1), 1, S.st), "clover"));
  double tot = 0, rr;
  // even: A_ee x_e - kappa D_eo x_o - b_e
  TRY(wilson_hop(S.ctx, hi, hi.g, W_XPAY_CLOV, y, xo, xe, clover_block(hi, op->clover, 0), 0, -op->kappa, 0, nullptr,
                 S.st));
  TRY(residual_from(S, hi.prec, be, y, ncomplex(hi), &rr));
  tot += rr;
  TRY(wilson_hop(S.ctx, hi, hi.g, W_XPAY_CLOV, y, xe, xo, clover_block(hi, op->clover, 1), 1, -op->kappa, 0, nullptr,
                 S.st));
  TRY(residual_from(S, hi.prec, bo, y, ncomplex(hi), &rr));
  tot += rr;
  *true_res = bnorm > 0 ? std::sqrt(tot) / bnorm : 0.0;
  return LQCD_OK;
}

// x_o = A_oo^-1 (b_o + kappa D_oe x_e) for nrhs sources, then each source's
// true full residual ||b_j - M x_j|| / ||b_j|| (res[j]; 0 for a zero source).
lqcd_status wilson_finish_mrhs(Solver &S, const OpInfo &hi, void *x_full, const void *b_full, void *tmp, void *y,
                               const double *bn2, int nrhs, double *res) {
  const size_t blk = hi.spinor_bytes * nrhs;
  char *xe = (char *)x_full, *xo = xe + blk;
  const char *be = (const char *)b_full, *bo = be + blk;
  const lqcd_operator *op = hi.op;
  TRY(wilson_hop(S.ctx, hi, hi.g, W_XPAY, tmp, xe, bo, nullptr, 1, op->kappa, 0, nullptr, S.st, nrhs));
  TRY(S.hip(launch_clover_apply(hi.g, hi.prec, xo, tmp, clover_block(hi, op->clover_inv, 1), nrhs, S.st), "clover"));
  std::vector<double> one(nrhs, 1.0), mone(nrhs, -1.0), rr(nrhs), tot(nrhs, 0.0);
  RedScratch red = S.red();
  for (int par = 0; par < 2; ++par) {
    // y = A_pp x_p - kappa D_p,1-p x_1-p, then y = b_p - y
    TRY(wilson_hop(S.ctx, hi, hi.g, W_XPAY_CLOV, y, par ? xe : xo, par ? xo : xe, clover_block(hi, op->clover, par),
                   par, -op->kappa, 0, nullptr, S.st, nrhs));
    TRY(S.hip(blas_mrhs_axpby(hi.prec, par ? bo : be, hi.prec, y, (int64_t)hi.vh, hi.nsp, nrhs, one.data(),
                              mone.data(), &red, S.st),
              "residual"));
    TRY(S.result(nrhs, rr.data()));
    for (int j = 0; j < nrhs; ++j) tot[j] += rr[j];
  }
  for (int j = 0; j < nrhs; ++j) res[j] = bn2[j] > 0 ? std::sqrt(tot[j] / bn2[j]) : 0.0;
  return LQCD_OK;
}

// Per-iteration log on stderr when the environment variable LQCD_VERBOSE is set.
bool verbose() {
  static const bool v = std::getenv("LQCD_VERBOSE") != nullptr;
  return v;
}

double elapsed(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Scale that brings a vector of norm `nrm` with `nreal` reals to unit RMS per
// real (used before 16-bit storage; K and the Krylov recurrences are
// positively homogeneous, so the scaling is exact).
double unit_rms_scale(double nrm, size_t nreal) { return nrm > 0 ? std::sqrt((double)nreal) / nrm : 1.0; }

}  // namespace

extern "C" lqcd_status lqcd_gcr_solve(lqcd_context *ctx, const lqcd_operator *op_hi, const lqcd_operator *op_krylov,
                                      const lqcd_operator *op_precond, const lqcd_gcr_params *prm, void *x_full,
                                      const void *b_full, lqcd_solve_info *info, lqcd_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  OpInfo hi, kr, pc;
  TRY(check_op(ctx, op_hi, &hi));
  TRY(check_op(ctx, op_krylov, &kr));
  if (op_hi->action != LQCD_WILSON_CLOVER) return set_error(ctx, LQCD_ERR_INVALID_ARG, "GCR solves Wilson-clover systems");
  if (op_hi->prec != LQCD_F64) return set_error(ctx, LQCD_ERR_UNSUPPORTED, "op_hi must be FP64");
  if (!same_system(op_hi, op_krylov)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "op_krylov describes another system");
  if (op_krylov->prec == LQCD_HALF)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "the Krylov space is kept in FP64, FP32, FP16 or BF16");
  TRY(check_fields_internal(ctx, op_hi));
  TRY(check_fields_internal(ctx, op_krylov));
  if (!prm) return set_error(ctx, LQCD_ERR_INVALID_ARG, "params are NULL");
  if (!(prm->tol > 0) || prm->k_max < 1 || prm->k_max > 32 || !(prm->delta > 0) || prm->max_iter < 1)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "need tol > 0, 1 <= k_max <= 32, delta > 0, max_iter >= 1");
  if (prm->orth_passes < 0 || prm->orth_passes > 2)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "orth_passes must be 0, 1 or 2");
  if (prm->res_history_max < 0 || (prm->res_history_max > 0 && !prm->res_history))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "res_history_max > 0 needs a res_history array");
  const int pk = prm->precond;
  if (pk == LQCD_PRECOND_SCHWARZ) {
    TRY(check_op(ctx, op_precond, &pc));
    if (!same_system(op_hi, op_precond, true))
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "op_precond describes another system");
    TRY(check_schwarz(ctx, pc, &prm->schwarz));
  } else if (pk == LQCD_PRECOND_LEARNED) {
    TRY(check_op(ctx, op_precond, &pc));
    if (!same_system(op_hi, op_precond, true))
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "op_precond describes another system");
    if (op_precond->prec != LQCD_F32 || op_krylov->prec != LQCD_F32)
      return set_error(ctx, LQCD_ERR_UNSUPPORTED, "the learned preconditioner runs with FP32 op_krylov and op_precond");
    if (!prm->learned) return set_error(ctx, LQCD_ERR_INVALID_ARG, "learned network is NULL");
    TRY(check_fields_internal(ctx, op_precond));
    if (prm->schwarz.mr_steps > 0) TRY(check_schwarz(ctx, pc, &prm->schwarz));
  } else if (pk != LQCD_PRECOND_NONE) {
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "unknown preconditioner kind");
  }
  if (!x_full || !b_full || ((uintptr_t)x_full & 15) || ((uintptr_t)b_full & 15))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");

  Solver S{ctx, (hipStream_t)stream, kSlotSolver};
  S.min_bytes = hi.spinor_bytes;
  const size_t n = ncomplex(hi);
  const int kmax = prm->k_max;
  void *bhat, *r, *y, *tmp, *rhat, *ktmp, *pin = nullptr, *pout = nullptr;
  TRY(S.vec(hi.spinor_bytes, &bhat));
  TRY(S.vec(hi.spinor_bytes, &r));
  TRY(S.vec(hi.spinor_bytes, &y));
  TRY(S.vec(hi.spinor_bytes, &tmp));
  TRY(S.vec(kr.spinor_bytes, &rhat));
  TRY(S.vec(kr.spinor_bytes, &ktmp));
  std::vector<void *> P(kmax), Z(kmax);
  for (int i = 0; i < kmax; ++i) TRY(S.vec(kr.spinor_bytes, &P[i]));
  for (int i = 0; i < kmax; ++i) TRY(S.vec(kr.spinor_bytes, &Z[i]));
  // K works in op_precond's precision and tile; its input and output are
  // converted (and re-laid out when the tiles differ)
  const bool k_relayout = pk != LQCD_PRECOND_NONE && !same_tile(kr, pc);
  if (pk == LQCD_PRECOND_SCHWARZ || (pk == LQCD_PRECOND_LEARNED && (prm->schwarz.mr_steps > 0 || k_relayout))) {
    TRY(S.vec(pc.spinor_bytes, &pin));
    TRY(S.vec(pc.spinor_bytes, &pout));
  }
  auto to_layout = [&](const OpInfo &a, const void *in, const OpInfo &b, void *out, double scale) -> lqcd_status {
    // element-wise when only the precision changes (fixed point needs the
    // per-site kernel, which forms each site's norm)
    if (same_tile(a, b) && a.prec != LQCD_HALF && b.prec != LQCD_HALF)
      return S.hip(blas_convert(a.prec, in, b.prec, out, ncomplex(a), scale, S.st), "convert");
    return S.hip(launch_spinor_relayout(b.g, b.prec, out, a.g, a.prec, in, a.nsp, 0, 1, scale, S.st), "relayout");
  };
  // LEARNED: a step whose residual reduction stalls (or whose network output
  // is not finite) makes the next step use the Schwarz preconditioner.
  bool use_fallback = false;
  double rhn_prev = 0;
  RedScratch red = S.red();
  void *xe = x_full;

  double bn2;
  TRY(S.hip(blas_norm2(hi.prec, b_full, 2 * n, red, S.st), "norm"));
  TRY(S.result(1, &bn2));
  if (!std::isfinite(bn2)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "source contains non-finite values");
  lqcd_solve_info inf{};
  if (bn2 == 0) {
    TRY(S.hip(hipMemsetAsync(x_full, 0, 2 * hi.spinor_bytes, S.st), "memset"));
    TRY(S.hip(hipStreamSynchronize(S.st), "sync"));
    inf.seconds = elapsed(t0);
    if (info) *info = inf;
    return LQCD_OK;
  }
  const double bn = std::sqrt(bn2);
  TRY(wilson_schur_source(S, hi, bhat, b_full, tmp));
  // r = bhat - Mhat x_e
  TRY(schur_apply(ctx, hi, hi.g, y, xe, tmp, 0, nullptr, S.st));
  double rr;
  TRY(S.hip(hipMemcpyAsync(r, bhat, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
  TRY(S.hip(blas_axpby(hi.prec, y, hi.prec, r, n, -1.0, 0.0, 1.0, 0.0, &red, S.st), "axpby"));
  TRY(S.result(1, &rr));
  double r0n = std::sqrt(rr);
  TRY(S.hip(blas_convert(hi.prec, r, kr.prec, rhat, n, 1.0, S.st), "convert"));
  double rhn = r0n;

  std::vector<cd> alpha(kmax), beta((size_t)kmax * kmax), chi(kmax);
  std::vector<double> gamma(kmax);
  int k = 0, iters = 0, restarts = 0;
  bool converged = r0n <= prm->tol * bn;
  lqcd_status status = LQCD_OK;
  while (!converged) {
    // p_k = K rhat_k
    const bool schwarz_now = pk == LQCD_PRECOND_SCHWARZ || (pk == LQCD_PRECOND_LEARNED && use_fallback);
    if (schwarz_now) {
      const double sc = unit_rms_scale(rhn, 2 * n);
      TRY(to_layout(kr, rhat, pc, pin, sc));
      TRY(schwarz_apply(ctx, pc, &prm->schwarz, pout, pin, kSlotSchwarz, S.st));
      TRY(to_layout(pc, pout, kr, P[k], 1.0 / sc));
      inf.precond_applies++;
      if (pk == LQCD_PRECOND_LEARNED) inf.fallback_applies++;
      use_fallback = false;
    } else if (pk == LQCD_PRECOND_LEARNED) {
      if (k_relayout) {
        TRY(to_layout(kr, rhat, pc, pin, 1.0));
        TRY(ptc_apply(ctx, op_precond, prm->learned, pout, pin, S.st));
        TRY(to_layout(pc, pout, kr, P[k], 1.0));
      } else {
        TRY(ptc_apply(ctx, op_precond, prm->learned, P[k], rhat, S.st));
      }
      inf.precond_applies++;
    } else {
      TRY(S.hip(hipMemcpyAsync(P[k], rhat, kr.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
    }
    // z_k = Mhat p_k
    TRY(schur_apply(ctx, kr, kr.g, Z[k], P[k], ktmp, 0, nullptr, S.st));
    inf.matvecs++;
    // orthogonalise against z_0..z_{k-1}: classical Gram-Schmidt (all
    // beta_{i,k} from one pass, then one multi-axpy), once, or twice (CGS2:
    // the second pass removes what rounding left of the first, and its
    // coefficients add to beta_{i,k})
    const int passes = prm->orth_passes == 2 ? 2 : 1;
    double zd[3] = {0, 0, 0};
    std::vector<double> bc(2 * std::max(k, 1));
    for (int pass = 0; pass < passes && (k > 0 || pass == 0); ++pass) {
      for (int i0 = 0; i0 < k; i0 += 8) {
        const int m = std::min(8, k - i0);
        double d[16];
        TRY(S.hip(blas_multi_cdot(kr.prec, (const void *const *)&Z[i0], m, Z[k], n, red, S.st), "multi dot"));
        TRY(S.result(2 * m, d));
        for (int j = 0; j < m; ++j) {
          bc[2 * (i0 + j)] = d[2 * j];
          bc[2 * (i0 + j) + 1] = d[2 * j + 1];
          cd &b = beta[(size_t)(i0 + j) * kmax + k];
          b = pass == 0 ? cd(d[2 * j], d[2 * j + 1]) : b + cd(d[2 * j], d[2 * j + 1]);
        }
      }
      TRY(S.hip(blas_multi_caxpy_dots(kr.prec, (const void *const *)Z.data(), bc.data(), k, Z[k], rhat, n, red, S.st),
                "multi caxpy"));
      TRY(S.result(3, zd));
    }
    const double g = std::sqrt(zd[0]);
    if (!(g > 0) || !std::isfinite(g)) {
      if (pk == LQCD_PRECOND_LEARNED && !schwarz_now && prm->schwarz.mr_steps > 0) {
        // the network's direction is unusable (zero, or not finite): take
        // this step again with the Schwarz preconditioner (rhat is unchanged)
        use_fallback = true;
        continue;
      }
      status = set_error(ctx, LQCD_ERR_BREAKDOWN, "GCR breakdown: orthogonalised direction has zero norm");
      break;
    }
    gamma[k] = g;
    alpha[k] = cd(zd[1], zd[2]) / g;
    TRY(S.hip(blas_gcr_update(kr.prec, Z[k], rhat, n, 1.0 / g, alpha[k].real(), alpha[k].imag(), red, S.st),
              "gcr update"));
    TRY(S.result(1, &rr));
    rhn_prev = rhn;
    rhn = std::sqrt(rr);
    if (prm->res_history && inf.history_len < prm->res_history_max) prm->res_history[inf.history_len++] = rhn;
    if (pk == LQCD_PRECOND_LEARNED && prm->schwarz.mr_steps > 0 && !schwarz_now &&
        (!(rhn < 0.95 * rhn_prev) || !std::isfinite(rhn)))
      use_fallback = true;
    if (verbose())
      fprintf(stderr, "gcr it %d k %d |rhat|/|b| %.3e gamma %.3e |alpha| %.3e\n", iters, k, rhn / bn, g,
              std::abs(alpha[k]));
    ++k;
    ++iters;
    if (k == kmax || rhn / r0n < prm->delta || rhn < prm->tol * bn || iters >= prm->max_iter) {
      // back substitution: gamma_l chi_l + sum_{i>l} beta_{l,i} chi_i = alpha_l
      for (int l = k - 1; l >= 0; --l) {
        cd sacc = alpha[l];
        for (int i = l + 1; i < k; ++i) sacc -= beta[(size_t)l * kmax + i] * chi[i];
        chi[l] = sacc / gamma[l];
      }
      std::vector<double> cc(2 * k);
      for (int i = 0; i < k; ++i) {
        cc[2 * i] = chi[i].real();
        cc[2 * i + 1] = chi[i].imag();
      }
      TRY(S.hip(blas_multi_axpy_acc(hi.prec, xe, kr.prec, (const void *const *)P.data(), cc.data(), k, n, S.st),
                "solution update"));
      // high-precision restart: r = bhat - Mhat x
      TRY(schur_apply(ctx, hi, hi.g, y, xe, tmp, 0, nullptr, S.st));
      TRY(S.hip(hipMemcpyAsync(r, bhat, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
      TRY(S.hip(blas_axpby(hi.prec, y, hi.prec, r, n, -1.0, 0.0, 1.0, 0.0, &red, S.st), "axpby"));
      TRY(S.result(1, &rr));
      r0n = std::sqrt(rr);
      rhn = r0n;
      ++restarts;
      if (verbose()) fprintf(stderr, "gcr restart %d true |r|/|b| %.3e\n", restarts, r0n / bn);
      k = 0;
      if (r0n <= prm->tol * bn) {
        converged = true;
        break;
      }
      if (iters >= prm->max_iter) break;
      TRY(S.hip(blas_convert(hi.prec, r, kr.prec, rhat, n, 1.0, S.st), "convert"));
    }
  }
  double tres = 0;
  TRY(wilson_finish(S, hi, x_full, b_full, tmp, y, bn, &tres));
  inf.iters = iters;
  inf.restarts = restarts;
  inf.true_residual = tres;
  inf.seconds = elapsed(t0);
  if (info) *info = inf;
  if (status != LQCD_OK) return status;
  if (!converged) return set_error(ctx, LQCD_ERR_NOT_CONVERGED, "GCR reached max_iter");
  return LQCD_OK;
}

// ---------------------------------------------------------------------------
// CG with reliable updates

namespace {

struct CgOps {
  Solver *S;
  const OpInfo *hi, *lo;
  int kind;
  void *tmp_hi, *tmp_lo;
  // A applied in the given precision. For CGNE: A = Mhat (dag = 0) or Mhat^+ (dag = 1).
  lqcd_status apply(const OpInfo &o, void *out, const void *in, int dag, void *tmp, int nrhs = 1) {
    return schur_apply(S->ctx, o, o.g, out, in, tmp, dag, nullptr, S->st, nrhs);
  }
};

// CG or CGNE (the same recurrences as lqcd_cg_solve) on nrhs systems at once:
// every operator application is one launch over all sources, while each
// system keeps its own scalars, its own reliable-update scale and its own stop
// test. A system that has converged takes no further steps (its coefficients
// are zero); a reliable update, triggered by any system, refreshes all of them.
lqcd_status cg_solve_mrhs(Solver &S, const OpInfo &hi, const OpInfo &lo, const lqcd_cg_params *prm, int nrhs, void *x,
                          const void *b, lqcd_solve_info *inf) {
  lqcd_context *ctx = S.ctx;
  const bool cgne = prm->kind == LQCD_CG_CGNE_SCHUR;
  const bool mixed = lo.prec != hi.prec;
  const bool half = lo.prec == LQCD_F16 || lo.prec == LQCD_BF16;
  const double delta = prm->delta_reliable;
  const int64_t vh = (int64_t)hi.vh;
  const int nsp = hi.nsp;
  const size_t nreal = (size_t)vh * nsp;  // reals of one source on one parity
  void *bhat, *r, *y, *tmp_hi, *rs, *xs, *p, *q, *t, *tmp_lo;
  TRY(S.vec(hi.spinor_bytes * nrhs, &bhat));
  TRY(S.vec(hi.spinor_bytes * nrhs, &r));
  TRY(S.vec(hi.spinor_bytes * nrhs, &y));
  TRY(S.vec(hi.spinor_bytes * nrhs, &tmp_hi));
  TRY(S.vec(lo.spinor_bytes * nrhs, &rs));
  TRY(S.vec(lo.spinor_bytes * nrhs, &xs));
  TRY(S.vec(lo.spinor_bytes * nrhs, &p));
  TRY(S.vec(lo.spinor_bytes * nrhs, &q));
  TRY(S.vec(lo.spinor_bytes * nrhs, &t));
  TRY(S.vec(lo.spinor_bytes * nrhs, &tmp_lo));
  RedScratch red = S.red();
  CgOps A{&S, &hi, &lo, prm->kind, tmp_hi, tmp_lo};
  std::vector<double> bn2(nrhs), part(2 * nrhs), coef(nrhs), coef2(nrhs), one(nrhs, 1.0), mone(nrhs, -1.0),
      zero(nrhs, 0.0);
  // source norms: both parities (CGNE_SCHUR) or the even sites
  for (int j = 0; j < nrhs; ++j) bn2[j] = 0;
  for (int par = 0; par < (cgne ? 2 : 1); ++par) {
    const char *bp = (const char *)b + par * hi.spinor_bytes * nrhs;
    TRY(S.hip(blas_mrhs_cdot(hi.prec, bp, bp, vh, nsp, nrhs, red, S.st), "norms"));
    TRY(S.result(2 * nrhs, part.data()));
    for (int j = 0; j < nrhs; ++j) bn2[j] += part[2 * j];
  }
  for (int j = 0; j < nrhs; ++j)
    if (!std::isfinite(bn2[j])) return set_error(ctx, LQCD_ERR_INVALID_ARG, "source contains non-finite values");
  // a zero source has the solution zero
  for (int j = 0; j < nrhs; ++j) coef[j] = bn2[j] > 0 ? 1.0 : 0.0;
  for (int par = 0; par < (cgne ? 2 : 1); ++par) {
    char *xp = (char *)x + par * hi.spinor_bytes * nrhs;
    TRY(S.hip(blas_mrhs_axpby(hi.prec, xp, hi.prec, xp, vh, nsp, nrhs, coef.data(), zero.data(), nullptr, S.st),
              "zero sources"));
  }
  if (cgne)
    TRY(wilson_schur_source(S, hi, bhat, b, tmp_hi, nrhs));
  else
    TRY(S.hip(hipMemcpyAsync(bhat, b, hi.spinor_bytes * nrhs, hipMemcpyDeviceToDevice, S.st), "copy"));
  void *xe = x;
  std::vector<double> rr_true(nrhs);
  auto true_residual = [&]() -> lqcd_status {
    TRY(A.apply(hi, y, xe, 0, tmp_hi, nrhs));
    TRY(S.hip(hipMemcpyAsync(r, bhat, hi.spinor_bytes * nrhs, hipMemcpyDeviceToDevice, S.st), "copy"));
    TRY(S.hip(blas_mrhs_axpby(hi.prec, y, hi.prec, r, vh, nsp, nrhs, mone.data(), one.data(), &red, S.st), "axpby"));
    return S.result(nrhs, rr_true.data());
  };
  TRY(true_residual());
  std::vector<double> sc(nrhs), rr(nrhs), rr_new(nrhs), pp(nrhs, 0.0), maxrr(nrhs), stop(nrhs), a(nrhs), bta(nrhs);
  std::vector<char> conv(nrhs);
  for (int j = 0; j < nrhs; ++j) {
    sc[j] = half ? unit_rms_scale(std::sqrt(rr_true[j]), nreal) : 1.0;
    rr[j] = rr_true[j] * sc[j] * sc[j];
    maxrr[j] = rr_true[j];
    stop[j] = prm->tol * prm->tol * bn2[j];
    conv[j] = rr_true[j] <= stop[j];
  }
  TRY(S.hip(blas_mrhs_axpby(hi.prec, r, lo.prec, rs, vh, nsp, nrhs, sc.data(), zero.data(), nullptr, S.st),
            "convert"));
  TRY(S.hip(hipMemsetAsync(xs, 0, lo.spinor_bytes * nrhs, S.st), "memset"));
  if (cgne) {
    TRY(A.apply(lo, p, rs, 1, tmp_lo, nrhs));
    TRY(S.hip(blas_mrhs_cdot(lo.prec, p, p, vh, nsp, nrhs, red, S.st), "norms"));
    TRY(S.result(2 * nrhs, part.data()));
    for (int j = 0; j < nrhs; ++j) pp[j] = part[2 * j];
    inf->matvecs += nrhs;
  } else {
    TRY(S.hip(hipMemcpyAsync(p, rs, lo.spinor_bytes * nrhs, hipMemcpyDeviceToDevice, S.st), "copy"));
  }
  auto all_converged = [&]() {
    for (int j = 0; j < nrhs; ++j)
      if (!conv[j]) return false;
    return true;
  };
  lqcd_status status = LQCD_OK;
  int it = 0;
  while (!all_converged() && it < prm->max_iter) {
    TRY(A.apply(lo, q, p, 0, tmp_lo, nrhs));
    inf->matvecs += nrhs;
    if (!cgne) {
      TRY(S.hip(blas_mrhs_cdot(lo.prec, p, q, vh, nsp, nrhs, red, S.st), "dots"));
      TRY(S.result(2 * nrhs, part.data()));
    }
    bool broke = false;
    for (int j = 0; j < nrhs; ++j) {
      a[j] = 0;
      if (conv[j]) continue;
      const double den = cgne ? pp[j] : part[2 * j];
      if (!(den > 0)) broke = true;
      else a[j] = rr[j] / den;
    }
    if (broke) {
      status = set_error(ctx, LQCD_ERR_BREAKDOWN, cgne ? "CGNE breakdown: |p| = 0" : "CG breakdown: <p, A p> <= 0");
      break;
    }
    TRY(S.hip(blas_mrhs_cg_update(lo.prec, xs, p, lo.prec, rs, q, vh, nsp, nrhs, a.data(), red, S.st), "cg update"));
    TRY(S.result(nrhs, rr_new.data()));
    ++it;
    bool trigger = false;
    for (int j = 0; j < nrhs; ++j) {
      if (conv[j]) continue;
      const double rt = rr_new[j] / (sc[j] * sc[j]);
      if (rt <= stop[j] || (mixed && rt < delta * delta * maxrr[j])) trigger = true;
    }
    if (trigger) {
      // x += xs / sc ; r = bhat - A x ; every sloppy residual restarts from it
      for (int j = 0; j < nrhs; ++j) coef[j] = 1.0 / sc[j];
      TRY(S.hip(blas_mrhs_axpby(lo.prec, xs, hi.prec, xe, vh, nsp, nrhs, coef.data(), one.data(), nullptr, S.st),
                "x update"));
      TRY(true_residual());
      inf->restarts++;
      for (int j = 0; j < nrhs; ++j) {
        const double sn = half ? unit_rms_scale(std::sqrt(rr_true[j]), nreal) : 1.0;
        coef[j] = sn;
        coef2[j] = sn / sc[j];
        rr[j] *= coef2[j] * coef2[j];
        sc[j] = sn;
        rr_new[j] = rr_true[j] * sn * sn;
        maxrr[j] = rr_true[j];
        if (rr_true[j] <= stop[j]) conv[j] = 1;
      }
      TRY(S.hip(blas_mrhs_axpby(hi.prec, r, lo.prec, rs, vh, nsp, nrhs, coef.data(), zero.data(), nullptr, S.st),
                "convert"));
      TRY(S.hip(hipMemsetAsync(xs, 0, lo.spinor_bytes * nrhs, S.st), "memset"));
      if (half)
        TRY(S.hip(blas_mrhs_axpby(lo.prec, p, lo.prec, p, vh, nsp, nrhs, coef2.data(), zero.data(), nullptr, S.st),
                  "rescale"));
      if (all_converged()) break;
    }
    for (int j = 0; j < nrhs; ++j) bta[j] = conv[j] ? 0.0 : rr_new[j] / rr[j];
    if (cgne) {
      TRY(A.apply(lo, t, rs, 1, tmp_lo, nrhs));
      inf->matvecs += nrhs;
      TRY(S.hip(blas_mrhs_axpby(lo.prec, t, lo.prec, p, vh, nsp, nrhs, one.data(), bta.data(), &red, S.st), "xpay"));
      TRY(S.result(nrhs, pp.data()));
    } else {
      TRY(S.hip(blas_mrhs_axpby(lo.prec, rs, lo.prec, p, vh, nsp, nrhs, one.data(), bta.data(), nullptr, S.st),
                "xpay"));
    }
    for (int j = 0; j < nrhs; ++j) {
      rr[j] = rr_new[j];
      maxrr[j] = std::max(maxrr[j], rr_new[j] / (sc[j] * sc[j]));
    }
  }
  if (!all_converged()) {
    for (int j = 0; j < nrhs; ++j) coef[j] = 1.0 / sc[j];
    TRY(S.hip(blas_mrhs_axpby(lo.prec, xs, hi.prec, xe, vh, nsp, nrhs, coef.data(), one.data(), nullptr, S.st),
              "x update"));
  }
  std::vector<double> res(nrhs);
  if (cgne) {
    TRY(wilson_finish_mrhs(S, hi, x, b, tmp_hi, y, bn2.data(), nrhs, res.data()));
  } else {
    TRY(true_residual());
    for (int j = 0; j < nrhs; ++j) res[j] = bn2[j] > 0 ? std::sqrt(rr_true[j] / bn2[j]) : 0.0;
  }
  inf->iters = it;
  inf->true_residual = 0;
  for (int j = 0; j < nrhs; ++j) {
    inf->true_residual = std::max(inf->true_residual, res[j]);
    if (prm->rhs_residuals) prm->rhs_residuals[j] = res[j];
  }
  if (status != LQCD_OK) return status;
  if (!all_converged()) return set_error(ctx, LQCD_ERR_NOT_CONVERGED, "CG reached max_iter");
  return LQCD_OK;
}

}  // namespace

extern "C" lqcd_status lqcd_cg_solve(lqcd_context *ctx, const lqcd_operator *op_hi, const lqcd_operator *op_sloppy,
                                     const lqcd_cg_params *prm, void *x, const void *b, lqcd_solve_info *info,
                                     lqcd_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if (!prm) return set_error(ctx, LQCD_ERR_INVALID_ARG, "params are NULL");
  OpInfo hi, lo;
  TRY(check_op(ctx, op_hi, &hi));
  if (op_sloppy) {
    TRY(check_op(ctx, op_sloppy, &lo));
    if (!same_system(op_hi, op_sloppy)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "op_sloppy describes another system");
    TRY(check_fields_internal(ctx, op_sloppy));
  } else {
    lo = hi;
  }
  TRY(check_fields_internal(ctx, op_hi));
  const int kind = prm->kind;
  if (kind == LQCD_CG_CGNE_SCHUR && op_hi->action != LQCD_WILSON_CLOVER)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "CGNE_SCHUR needs a Wilson-clover operator");
  if (kind == LQCD_CG_STAG_NORMAL && op_hi->action != LQCD_STAGGERED)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "STAG_NORMAL needs a staggered operator");
  if (kind != LQCD_CG_CGNE_SCHUR && kind != LQCD_CG_STAG_NORMAL)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "unknown CG kind");
  if (!(prm->tol > 0) || prm->max_iter < 1 || prm->delta_reliable < 0 || prm->delta_reliable >= 1)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "need tol > 0, max_iter >= 1, 0 <= delta_reliable < 1");
  if (!x || !b || ((uintptr_t)x & 15) || ((uintptr_t)b & 15))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  if (hi.prec != LQCD_F64) return set_error(ctx, LQCD_ERR_UNSUPPORTED, "op_hi must be FP64");
  const int nrhs = prm->nrhs <= 0 ? 1 : prm->nrhs;
  if (nrhs > LQCD_MAX_CG_RHS) return set_error(ctx, LQCD_ERR_INVALID_ARG, "nrhs exceeds LQCD_MAX_CG_RHS");
  TRY(check_nrhs(ctx, hi, nrhs));
  if (prm->res_history_max < 0 || (prm->res_history_max > 0 && !prm->res_history))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "res_history_max > 0 needs a res_history array");

  Solver S{ctx, (hipStream_t)stream, kSlotSolver};
  S.min_bytes = hi.spinor_bytes * nrhs;
  // several sources, or 16-bit fixed-point sloppy vectors (whose kernels
  // work site by site): the multi-source iteration
  if (nrhs > 1 || lo.prec == LQCD_HALF) {
    if (prm->record_max > 0 || prm->res_history_max > 0)
      return set_error(ctx, LQCD_ERR_INVALID_ARG,
                       "recording and residual histories need nrhs = 1 and op_sloppy not in fixed point");
    lqcd_solve_info inf{};
    const lqcd_status st = cg_solve_mrhs(S, hi, lo, prm, nrhs, x, b, &inf);
    inf.seconds = elapsed(t0);
    if (info) *info = inf;
    return st;
  }
  const bool cgne = kind == LQCD_CG_CGNE_SCHUR;
  const size_t n = ncomplex(hi);
  const bool mixed = lo.prec != hi.prec;
  const bool recording = prm->record_max > 0;
  if (recording) {
    if (!cgne || op_sloppy || prm->record_every < 1 || !prm->record_r || !prm->record_e || !prm->record_xstar ||
        !prm->record_count)
      return set_error(ctx, LQCD_ERR_INVALID_ARG,
                       "recording needs CGNE_SCHUR in pure op_hi precision, record_every >= 1 and all record buffers");
    *prm->record_count = 0;
  }
  const bool half = lo.prec == LQCD_F16 || lo.prec == LQCD_BF16;
  // 16-bit sloppy operator in the plain CG: the iteration's vectors (xs, rs,
  // p, q) stay in FP32, and only the operator's input and output are 16-bit
  const bool mid = half && !cgne;
  const int vp = mid ? (int)LQCD_F32 : lo.prec;
  const size_t vb = mid ? site_block_bytes(LQCD_F32, lo.nsp, lo.vh, true) : lo.spinor_bytes;
  const double delta = prm->delta_reliable;
  void *bhat, *r, *y, *tmp_hi, *rs, *xs, *p, *q, *t, *tmp_lo, *p16 = nullptr, *q16 = nullptr;
  TRY(S.vec(hi.spinor_bytes, &bhat));
  TRY(S.vec(hi.spinor_bytes, &r));
  TRY(S.vec(hi.spinor_bytes, &y));
  TRY(S.vec(hi.spinor_bytes, &tmp_hi));
  TRY(S.vec(vb, &rs));
  TRY(S.vec(vb, &xs));
  TRY(S.vec(vb, &p));
  TRY(S.vec(vb, &q));
  TRY(S.vec(lo.spinor_bytes, &t));
  TRY(S.vec(lo.spinor_bytes, &tmp_lo));
  if (mid) {
    TRY(S.vec(lo.spinor_bytes, &p16));
    TRY(S.vec(lo.spinor_bytes, &q16));
  }
  RedScratch red = S.red();
  CgOps A{&S, &hi, &lo, kind, tmp_hi, tmp_lo};
  lqcd_solve_info inf{};

  // source norm (full lattice for CGNE, even sites for the staggered system)
  double bn2;
  TRY(S.hip(blas_norm2(hi.prec, b, cgne ? 2 * n : n, red, S.st), "norm"));
  TRY(S.result(1, &bn2));
  if (!std::isfinite(bn2)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "source contains non-finite values");
  if (bn2 == 0) {
    TRY(S.hip(hipMemsetAsync(x, 0, (cgne ? 2 : 1) * hi.spinor_bytes, S.st), "memset"));
    TRY(S.hip(hipStreamSynchronize(S.st), "sync"));
    inf.seconds = elapsed(t0);
    if (info) *info = inf;
    return LQCD_OK;
  }
  const double bn = std::sqrt(bn2);
  if (cgne)
    TRY(wilson_schur_source(S, hi, bhat, b, tmp_hi));
  else
    TRY(S.hip(hipMemcpyAsync(bhat, b, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
  void *xe = x;

  // true residual r = bhat - A x (A = Mhat or N_e), returns ||r||^2
  auto true_residual = [&](double *rr) -> lqcd_status {
    TRY(A.apply(hi, y, xe, 0, tmp_hi));
    TRY(S.hip(hipMemcpyAsync(r, bhat, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
    TRY(S.hip(blas_axpby(hi.prec, y, hi.prec, r, n, -1.0, 0.0, 1.0, 0.0, &red, S.st), "axpby"));
    return S.result(1, rr);
  };

  double rr_true;
  TRY(true_residual(&rr_true));
  double sc = half ? unit_rms_scale(std::sqrt(rr_true), 2 * n) : 1.0;
  TRY(S.hip(blas_convert(hi.prec, r, vp, rs, n, sc, S.st), "convert"));
  TRY(S.hip(hipMemsetAsync(xs, 0, vb, S.st), "memset"));
  double rr = rr_true * sc * sc;  // in scaled units
  double pp = 0;
  if (cgne) {
    TRY(A.apply(lo, p, rs, 1, tmp_lo));
    TRY(S.hip(blas_norm2(lo.prec, p, n, red, S.st), "norm"));
    TRY(S.result(1, &pp));
    inf.matvecs++;
  } else {
    TRY(S.hip(hipMemcpyAsync(p, rs, vb, hipMemcpyDeviceToDevice, S.st), "copy"));
  }
  double maxrr = rr_true;
  const double stop = prm->tol * prm->tol * bn2;
  bool converged = rr_true <= stop;
  lqcd_status status = LQCD_OK;
  int it = 0;
  while (!converged && it < prm->max_iter) {
    double a;
    if (mid) {
      TRY(S.hip(blas_convert(vp, p, lo.prec, p16, n, 1.0, S.st), "convert"));
      TRY(A.apply(lo, q16, p16, 0, tmp_lo));
      TRY(S.hip(blas_convert(lo.prec, q16, vp, q, n, 1.0, S.st), "convert"));
    } else {
      TRY(A.apply(lo, q, p, 0, tmp_lo));
    }
    inf.matvecs++;
    if (cgne) {
      if (!(pp > 0)) { status = set_error(ctx, LQCD_ERR_BREAKDOWN, "CGNE breakdown: |p| = 0"); break; }
      a = rr / pp;
    } else {
      double d[2];
      TRY(S.hip(blas_cdot(vp, p, q, n, red, S.st), "dot"));
      TRY(S.result(2, d));
      if (!(d[0] > 0)) { status = set_error(ctx, LQCD_ERR_BREAKDOWN, "CG breakdown: <p, A p> <= 0"); break; }
      a = rr / d[0];
    }
    double rr_new;
    TRY(S.hip(blas_cg_update(vp, xs, p, vp, rs, q, n, a, red, S.st), "cg update"));
    TRY(S.result(1, &rr_new));
    ++it;
    double rr_new_true = rr_new / (sc * sc);
    if (inf.history_len < prm->res_history_max) prm->res_history[inf.history_len++] = std::sqrt(rr_new_true);
    if (verbose()) fprintf(stderr, "cg it %d |r|/|b| %.3e alpha %.3e\n", it, std::sqrt(rr_new_true) / bn, a);
    if (recording && it % prm->record_every == 0 && *prm->record_count < prm->record_max) {
      // pure precision: x_k = x_e + xs, r_k = rs; e_k = x* - x_k
      const int j = *prm->record_count;
      char *rdst = (char *)prm->record_r + (size_t)j * hi.spinor_bytes;
      char *edst = (char *)prm->record_e + (size_t)j * hi.spinor_bytes;
      TRY(S.hip(hipMemcpyAsync(rdst, rs, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "record"));
      TRY(S.hip(hipMemcpyAsync(edst, prm->record_xstar, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "record"));
      TRY(S.hip(blas_axpby(hi.prec, xe, hi.prec, edst, n, -1.0, 0.0, 1.0, 0.0, nullptr, S.st), "record"));
      TRY(S.hip(blas_axpby(lo.prec, xs, hi.prec, edst, n, -1.0, 0.0, 1.0, 0.0, nullptr, S.st), "record"));
      *prm->record_count = j + 1;
    }
    // reliable update when the iterated residual dropped by delta since the
    // last one (mixed precision), and always before declaring convergence
    const bool trigger = rr_new_true <= stop || (mixed && rr_new_true < delta * delta * maxrr);
    if (trigger) {
      // x += xs / sc ; r = bhat - A x ; restart the sloppy residual from it
      TRY(S.hip(blas_axpby(vp, xs, hi.prec, xe, n, 1.0 / sc, 0.0, 1.0, 0.0, nullptr, S.st), "x update"));
      TRY(true_residual(&rr_new_true));
      inf.restarts++;
      if (verbose()) fprintf(stderr, "cg reliable update %d true |r|/|b| %.3e\n", inf.restarts, std::sqrt(rr_new_true) / bn);
      const double sc_new = half ? unit_rms_scale(std::sqrt(rr_new_true), 2 * n) : 1.0;
      TRY(S.hip(blas_convert(hi.prec, r, vp, rs, n, sc_new, S.st), "convert"));
      TRY(S.hip(hipMemsetAsync(xs, 0, vb, S.st), "memset"));
      if (sc_new != sc) TRY(S.hip(blas_convert(vp, p, vp, p, n, sc_new / sc, S.st), "rescale"));
      rr *= (sc_new / sc) * (sc_new / sc);
      sc = sc_new;
      rr_new = rr_new_true * sc * sc;
      maxrr = rr_new_true;
      if (rr_new_true <= stop) {
        converged = true;
        break;
      }
    }
    const double bta = rr_new / rr;
    if (cgne) {
      TRY(A.apply(lo, t, rs, 1, tmp_lo));
      inf.matvecs++;
      TRY(S.hip(blas_axpby(lo.prec, t, lo.prec, p, n, 1.0, 0.0, bta, 0.0, &red, S.st), "xpay"));
      TRY(S.result(1, &pp));
    } else {
      TRY(S.hip(blas_axpby(vp, rs, vp, p, n, 1.0, 0.0, bta, 0.0, nullptr, S.st), "xpay"));
    }
    rr = rr_new;
    maxrr = std::max(maxrr, rr_new / (sc * sc));
  }
  if (!converged) {
    // fold in the last sloppy correction
    TRY(S.hip(blas_axpby(vp, xs, hi.prec, xe, n, 1.0 / sc, 0.0, 1.0, 0.0, nullptr, S.st), "x update"));
  }
  double tres;
  if (cgne) {
    TRY(wilson_finish(S, hi, x, b, tmp_hi, y, bn, &tres));
  } else {
    double rrt;
    TRY(true_residual(&rrt));
    tres = std::sqrt(rrt) / bn;
  }
  inf.iters = it;
  inf.true_residual = tres;
  inf.seconds = elapsed(t0);
  if (info) *info = inf;
  if (status != LQCD_OK) return status;
  if (!converged) return set_error(ctx, LQCD_ERR_NOT_CONVERGED, "CG reached max_iter");
  return LQCD_OK;
}

extern "C" lqcd_status lqcd_multishift_cg_solve(lqcd_context *ctx, const lqcd_operator *op_hi,
                                                const lqcd_operator *op_sloppy, const lqcd_multishift_params *prm,
                                                void *const *x, const void *b, lqcd_multishift_info *info,
                                                lqcd_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if (!prm) return set_error(ctx, LQCD_ERR_INVALID_ARG, "params are NULL");
  OpInfo hi, lo;
  TRY(check_op(ctx, op_hi, &hi));
  if (op_hi->action != LQCD_STAGGERED) return set_error(ctx, LQCD_ERR_INVALID_ARG, "multi-shift CG needs a staggered operator");
  if (hi.prec != LQCD_F64) return set_error(ctx, LQCD_ERR_UNSUPPORTED, "op_hi must be FP64");
  TRY(check_fields_internal(ctx, op_hi));
  if (op_sloppy) {
    TRY(check_op(ctx, op_sloppy, &lo));
    if (!same_system(op_hi, op_sloppy)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "op_sloppy describes another system");
    TRY(check_fields_internal(ctx, op_sloppy));
    if (lo.prec != LQCD_F32 && lo.prec != LQCD_F64)
      return set_error(ctx, LQCD_ERR_UNSUPPORTED, "the multi-shift stage runs in FP32 or FP64, not in 16-bit precision");
  } else {
    lo = hi;
  }
  const int ns = prm->nshift;
  if (ns < 1 || ns > LQCD_MAX_SHIFTS) return set_error(ctx, LQCD_ERR_INVALID_ARG, "nshift must be 1 .. LQCD_MAX_SHIFTS");
  if (!(prm->tol > 0) || !(prm->tol_sloppy > 0) || prm->max_iter < 1 || prm->delta_reliable < 0 ||
      prm->delta_reliable >= 1)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "need tol > 0, tol_sloppy > 0, max_iter >= 1, 0 <= delta_reliable < 1");
  const double m2 = op_hi->mass * op_hi->mass;
  double smin = prm->shifts[0];
  for (int i = 0; i < ns; ++i) {
    if (!std::isfinite(prm->shifts[i]) || !(m2 + prm->shifts[i] > 0))
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "every shift needs m^2 + sigma > 0");
    smin = std::min(smin, prm->shifts[i]);
  }
  if (!x || !b || ((uintptr_t)b & 15)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  for (int i = 0; i < ns; ++i) {
    if (!x[i] || ((uintptr_t)x[i] & 15) || x[i] == b) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad solution pointer");
    for (int j = 0; j < i; ++j)
      if (x[j] == x[i]) return set_error(ctx, LQCD_ERR_INVALID_ARG, "solution pointers must be distinct");
  }

  Solver S{ctx, (hipStream_t)stream, kSlotSolver};
  S.min_bytes = hi.spinor_bytes;
  const size_t n = ncomplex(hi);  // complex entries of one even field
  RedScratch red = S.red();
  lqcd_multishift_info inf{};

  double bn2;
  TRY(S.hip(blas_norm2(hi.prec, b, n, red, S.st), "norm"));
  TRY(S.result(1, &bn2));
  if (!std::isfinite(bn2)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "source contains non-finite values");
  if (bn2 == 0) {
    for (int i = 0; i < ns; ++i) TRY(S.hip(hipMemsetAsync(x[i], 0, hi.spinor_bytes, S.st), "memset"));
    TRY(S.hip(hipStreamSynchronize(S.st), "sync"));
    inf.seconds = elapsed(t0);
    if (info) *info = inf;
    return LQCD_OK;
  }
  const double bn = std::sqrt(bn2);

  // Multi-shift stage in the sloppy precision: CG on A = N_e + smin (the
  // normal operator at mass sqrt(m^2 + smin)); the systems A + s_i with
  // s_i = sigma_i - smin >= 0 follow from the collinear residuals r_i = z_i r.
  lqcd_operator base_op = op_sloppy ? *op_sloppy : *op_hi;
  base_op.mass = std::sqrt(m2 + smin);
  OpInfo lb = lo;
  lb.op = &base_op;
  void *r, *q, *tmp, *p, *xs[LQCD_MAX_SHIFTS], *ps[LQCD_MAX_SHIFTS];
  TRY(S.vec(lo.spinor_bytes, &r));
  TRY(S.vec(lo.spinor_bytes, &q));
  TRY(S.vec(lo.spinor_bytes, &tmp));
  TRY(S.vec(lo.spinor_bytes, &p));
  for (int i = 0; i < ns; ++i) {
    TRY(S.vec(lo.spinor_bytes, &xs[i]));
    TRY(S.vec(lo.spinor_bytes, &ps[i]));
  }
  TRY(S.hip(blas_convert(hi.prec, b, lo.prec, r, n, 1.0, S.st), "convert"));
  TRY(S.hip(hipMemcpyAsync(p, r, lo.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
  for (int i = 0; i < ns; ++i) {
    TRY(S.hip(hipMemcpyAsync(ps[i], r, lo.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
    TRY(S.hip(hipMemsetAsync(xs[i], 0, lo.spinor_bytes, S.st), "memset"));
  }
  double rr;
  TRY(S.hip(blas_norm2(lo.prec, r, n, red, S.st), "norm"));
  TRY(S.result(1, &rr));
  double z[LQCD_MAX_SHIFTS], zp[LQCD_MAX_SHIFTS], res[LQCD_MAX_SHIFTS];
  bool active[LQCD_MAX_SHIFTS];
  for (int i = 0; i < ns; ++i) {
    z[i] = zp[i] = 1.0;
    res[i] = 1.0;
    active[i] = true;
  }
  double a_prev = 1.0, b_prev = 0.0;
  int it = 0;
  auto any_active = [&] {
    for (int i = 0; i < ns; ++i)
      if (active[i]) return true;
    return false;
  };
  while (any_active() && it < prm->max_iter) {
    TRY(schur_apply(ctx, lb, lb.g, q, p, tmp, 0, nullptr, S.st));
    inf.ms_matvecs++;
    double d[2];
    TRY(S.hip(blas_cdot(lo.prec, p, q, n, red, S.st), "dot"));
    TRY(S.result(2, d));
    if (!(d[0] > 0)) return set_error(ctx, LQCD_ERR_BREAKDOWN, "multi-shift CG breakdown: <p, A p> <= 0");
    const double a = rr / d[0];
    double rr_new;
    TRY(S.hip(blas_axpby(lo.prec, q, lo.prec, r, n, -a, 0.0, 1.0, 0.0, &red, S.st), "axpby"));
    TRY(S.result(1, &rr_new));
    const double bk = rr_new / rr;
    void *ux[LQCD_MAX_SHIFTS + 1], *up[LQCD_MAX_SHIFTS + 1];
    double ua[LQCD_MAX_SHIFTS + 1], uz[LQCD_MAX_SHIFTS + 1], ub[LQCD_MAX_SHIFTS + 1];
    int k = 0;
    for (int i = 0; i < ns; ++i) {
      if (!active[i]) continue;
      const double s = prm->shifts[i] - smin;
      const double den = a * b_prev * (zp[i] - z[i]) + zp[i] * a_prev * (1.0 + s * a);
      const double zn = z[i] * zp[i] * a_prev / den;
      if (!std::isfinite(zn) || zn == 0 || !(den != 0))
        return set_error(ctx, LQCD_ERR_BREAKDOWN, "multi-shift CG breakdown in the shift recurrence");
      ux[k] = xs[i];
      up[k] = ps[i];
      ua[k] = a * zn / z[i];
      uz[k] = zn;
      ub[k] = bk * (zn / z[i]) * (zn / z[i]);
      ++k;
      zp[i] = z[i];
      z[i] = zn;
    }
    // the base direction p = r + bk p
    ux[k] = nullptr;
    up[k] = p;
    ua[k] = 0.0;
    uz[k] = 1.0;
    ub[k] = bk;
    ++k;
    TRY(S.hip(blas_multishift_update(lo.prec, ux, up, ua, uz, ub, k, r, n, S.st), "multi-shift update"));
    a_prev = a;
    b_prev = bk;
    rr = rr_new;
    ++it;
    for (int i = 0; i < ns; ++i) {
      if (!active[i]) continue;
      res[i] = std::fabs(z[i]) * std::sqrt(rr) / bn;
      if (res[i] <= prm->tol_sloppy) active[i] = false;
    }
    if (verbose()) fprintf(stderr, "multi-shift it %d |r|/|b| %.3e (base shift)\n", it, std::sqrt(rr) / bn);
  }
  inf.ms_iters = it;
  // hand the solutions over in FP64 (before the refinements reuse the scratch)
  for (int i = 0; i < ns; ++i) TRY(S.hip(blas_convert(lo.prec, xs[i], hi.prec, x[i], n, 1.0, S.st), "convert"));
  TRY(S.hip(hipStreamSynchronize(S.st), "sync"));
  inf.ms_seconds = elapsed(t0);

  // Refinement of each x_i: reliable-update CG on the normal operator at mass
  // sqrt(m^2 + sigma_i), starting from the multi-shift solution.
  lqcd_status status = LQCD_OK;
  for (int i = 0; i < ns && status == LQCD_OK; ++i) {
    lqcd_operator oh = *op_hi, ol{};
    oh.mass = std::sqrt(m2 + prm->shifts[i]);
    if (op_sloppy) {
      ol = *op_sloppy;
      ol.mass = oh.mass;
    }
    lqcd_cg_params cg{};
    cg.tol = prm->tol;
    cg.max_iter = prm->max_iter;
    cg.delta_reliable = prm->delta_reliable;
    cg.kind = LQCD_CG_STAG_NORMAL;
    status = lqcd_cg_solve(ctx, &oh, op_sloppy ? &ol : nullptr, &cg, x[i], b, &inf.shift[i], stream);
  }
  inf.seconds = elapsed(t0);
  if (info) *info = inf;
  return status;
}

// ---------------------------------------------------------------------------
// Mixed-precision BiCGstab with reliable updates (Section III-A; the baseline
// of the GCR-DD comparison in Section IX)

extern "C" lqcd_status lqcd_bicgstab_solve(lqcd_context *ctx, const lqcd_operator *op_hi,
                                           const lqcd_operator *op_sloppy, const lqcd_bicgstab_params *prm,
                                           void *x_full, const void *b_full, lqcd_solve_info *info,
                                           lqcd_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if (!prm) return set_error(ctx, LQCD_ERR_INVALID_ARG, "params are NULL");
  OpInfo hi, lo;
  TRY(check_op(ctx, op_hi, &hi));
  if (op_hi->action != LQCD_WILSON_CLOVER)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "BiCGstab solves Wilson-clover systems");
  if (hi.prec != LQCD_F64) return set_error(ctx, LQCD_ERR_UNSUPPORTED, "op_hi must be FP64");
  TRY(check_fields_internal(ctx, op_hi));
  if (op_sloppy) {
    TRY(check_op(ctx, op_sloppy, &lo));
    if (!same_system(op_hi, op_sloppy)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "op_sloppy describes another system");
    if (op_sloppy->prec == LQCD_HALF)
      return set_error(ctx, LQCD_ERR_UNSUPPORTED, "BiCGstab's sloppy iteration runs in FP32, FP16 or BF16");
    TRY(check_fields_internal(ctx, op_sloppy));
  } else {
    lo = hi;
  }
  if (!(prm->tol > 0) || prm->max_iter < 1 || prm->delta_reliable < 0 || prm->delta_reliable >= 1)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "need tol > 0, max_iter >= 1, 0 <= delta_reliable < 1");
  if (!x_full || !b_full || ((uintptr_t)x_full & 15) || ((uintptr_t)b_full & 15))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");

  Solver S{ctx, (hipStream_t)stream, kSlotSolver};
  S.min_bytes = hi.spinor_bytes;
  const size_t n = ncomplex(hi);
  const bool mixed = lo.prec != hi.prec;
  const bool half = lo.prec == LQCD_F16 || lo.prec == LQCD_BF16;
  const double delta = prm->delta_reliable;
  void *bhat, *r, *y, *tmp_hi, *rs, *rh, *xs, *p, *v, *t, *tmp_lo;
  TRY(S.vec(hi.spinor_bytes, &bhat));
  TRY(S.vec(hi.spinor_bytes, &r));
  TRY(S.vec(hi.spinor_bytes, &y));
  TRY(S.vec(hi.spinor_bytes, &tmp_hi));
  TRY(S.vec(lo.spinor_bytes, &rs));  // iterated residual; holds s after the half step
  TRY(S.vec(lo.spinor_bytes, &rh));  // shadow residual
  TRY(S.vec(lo.spinor_bytes, &xs));  // sloppy solution since the last reliable update
  TRY(S.vec(lo.spinor_bytes, &p));
  TRY(S.vec(lo.spinor_bytes, &v));
  TRY(S.vec(lo.spinor_bytes, &t));
  TRY(S.vec(lo.spinor_bytes, &tmp_lo));
  RedScratch red = S.red();
  lqcd_solve_info inf{};
  void *xe = x_full;

  double bn2;
  TRY(S.hip(blas_norm2(hi.prec, b_full, 2 * n, red, S.st), "norm"));
  TRY(S.result(1, &bn2));
  if (!std::isfinite(bn2)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "source contains non-finite values");
  if (bn2 == 0) {
    TRY(S.hip(hipMemsetAsync(x_full, 0, 2 * hi.spinor_bytes, S.st), "memset"));
    TRY(S.hip(hipStreamSynchronize(S.st), "sync"));
    inf.seconds = elapsed(t0);
    if (info) *info = inf;
    return LQCD_OK;
  }
  const double bn = std::sqrt(bn2);
  const double stop = prm->tol * prm->tol * bn2;
  TRY(wilson_schur_source(S, hi, bhat, b_full, tmp_hi));

  // r = bhat - Mhat x_e in FP64; returns ||r||^2
  auto true_residual = [&](double *rr) -> lqcd_status {
    TRY(schur_apply(ctx, hi, hi.g, y, xe, tmp_hi, 0, nullptr, S.st));
    TRY(S.hip(hipMemcpyAsync(r, bhat, hi.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
    TRY(S.hip(blas_axpby(hi.prec, y, hi.prec, r, n, -1.0, 0.0, 1.0, 0.0, &red, S.st), "axpby"));
    return S.result(1, rr);
  };
  auto cdot = [&](const void *a, const void *b, cd *out) -> lqcd_status {
    double d[2];
    TRY(S.hip(blas_cdot(lo.prec, a, b, n, red, S.st), "dot"));
    TRY(S.result(2, d));
    *out = cd(d[0], d[1]);
    return LQCD_OK;
  };

  // The sloppy vectors live in units of sc times the FP64 ones (sc != 1 only
  // for 16-bit storage, which needs O(1) entries); every recurrence of
  // BiCGstab is homogeneous in that scale except rho, which carries it.
  double rr_true;
  TRY(true_residual(&rr_true));
  double sc = half ? unit_rms_scale(std::sqrt(rr_true), 2 * n) : 1.0;
  TRY(S.hip(blas_convert(hi.prec, r, lo.prec, rs, n, sc, S.st), "convert"));
  TRY(S.hip(hipMemsetAsync(xs, 0, lo.spinor_bytes, S.st), "memset"));

  // (re)start: shadow residual = current residual, p = r
  cd rho_new, rho(1, 0), alpha(1, 0), omega(1, 0);
  bool fresh = true;
  auto restart_shadow = [&]() -> lqcd_status {
    TRY(S.hip(hipMemcpyAsync(rh, rs, lo.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
    TRY(cdot(rh, rs, &rho_new));
    fresh = true;
    return LQCD_OK;
  };
  TRY(restart_shadow());
  double maxrr = rr_true;
  bool converged = rr_true <= stop;
  bool progress_since_restart = true;
  int shadow_restarts = 0;
  lqcd_status status = LQCD_OK;

  // fold the sloppy solution into x_e, recompute r in FP64 and replace the
  // iterated residual with it (rescaling p, v and rho to the new units)
  auto reliable_update = [&](double *rr_out) -> lqcd_status {
    TRY(S.hip(blas_axpby(lo.prec, xs, hi.prec, xe, n, 1.0 / sc, 0.0, 1.0, 0.0, nullptr, S.st), "x update"));
    TRY(true_residual(rr_out));
    inf.restarts++;
    const double sc_new = half ? unit_rms_scale(std::sqrt(*rr_out), 2 * n) : 1.0;
    TRY(S.hip(blas_convert(hi.prec, r, lo.prec, rs, n, sc_new, S.st), "convert"));
    TRY(S.hip(hipMemsetAsync(xs, 0, lo.spinor_bytes, S.st), "memset"));
    if (sc_new != sc) {
      const double f = sc_new / sc;
      TRY(S.hip(blas_convert(lo.prec, p, lo.prec, p, n, f, S.st), "rescale"));
      TRY(S.hip(blas_convert(lo.prec, v, lo.prec, v, n, f, S.st), "rescale"));
      rho *= f;
    }
    sc = sc_new;
    TRY(cdot(rh, rs, &rho_new));
    maxrr = *rr_out;
    if (verbose())
      fprintf(stderr, "bicgstab reliable update %d true |r|/|b| %.3e\n", inf.restarts, std::sqrt(*rr_out) / bn);
    return LQCD_OK;
  };

  int it = 0;
  while (!converged && it < prm->max_iter) {
    if (fresh) {
      TRY(S.hip(hipMemcpyAsync(p, rs, lo.spinor_bytes, hipMemcpyDeviceToDevice, S.st), "copy"));
      fresh = false;
    } else {
      const cd beta = (rho_new / rho) * (alpha / omega);
      const cd c = -beta * omega;
      TRY(S.hip(blas_bicgstab_dir(lo.prec, rs, p, v, n, beta.real(), beta.imag(), c.real(), c.imag(), S.st), "dir"));
    }
    rho = rho_new;
    TRY(schur_apply(ctx, lo, lo.g, v, p, tmp_lo, 0, nullptr, S.st));
    inf.matvecs++;
    cd rhv;
    TRY(cdot(rh, v, &rhv));
    ++it;
    if (!(std::abs(rhv) > 0) || !std::isfinite(std::abs(rhv)) || !(std::abs(rho) > 0)) {
      // <rhat, v> = 0 (or rho = 0): fold in what we have and take a new shadow
      if (!progress_since_restart) {
        status = set_error(ctx, LQCD_ERR_BREAKDOWN, "BiCGstab breakdown: <rhat, A p> = 0 after a restart");
        break;
      }
      double rrt;
      TRY(reliable_update(&rrt));
      if (rrt <= stop) { converged = true; break; }
      TRY(restart_shadow());
      ++shadow_restarts;
      progress_since_restart = false;
      continue;
    }
    alpha = rho / rhv;
    // s = r - alpha v (in place of r)
    double ss;
    TRY(S.hip(blas_axpby(lo.prec, v, lo.prec, rs, n, -alpha.real(), -alpha.imag(), 1.0, 0.0, &red, S.st), "axpby"));
    TRY(S.result(1, &ss));
    if (ss / (sc * sc) <= stop) {
      // converged at the half step: x += alpha p, then check in FP64
      const double chi[2] = {alpha.real(), alpha.imag()};
      const void *pp[1] = {p};
      TRY(S.hip(blas_multi_axpy_acc(lo.prec, xs, lo.prec, pp, chi, 1, n, S.st), "x update"));
      double rrt;
      TRY(reliable_update(&rrt));
      if (rrt <= stop) { converged = true; break; }
      TRY(restart_shadow());
      ++shadow_restarts;
      continue;
    }
    TRY(schur_apply(ctx, lo, lo.g, t, rs, tmp_lo, 0, nullptr, S.st));
    inf.matvecs++;
    double d[4];  // <t, t>, <s, t>
    {
      const void *z[2] = {t, rs};
      TRY(S.hip(blas_multi_cdot(lo.prec, z, 2, t, n, red, S.st), "dots"));
      TRY(S.result(4, d));
    }
    if (!(d[0] > 0) || !std::isfinite(d[0])) {
      status = set_error(ctx, LQCD_ERR_BREAKDOWN, "BiCGstab breakdown: A s = 0 with s != 0");
      break;
    }
    omega = std::conj(cd(d[2], d[3])) / d[0];
    {
      const double chi[4] = {alpha.real(), alpha.imag(), omega.real(), omega.imag()};
      const void *pp[2] = {p, rs};
      TRY(S.hip(blas_multi_axpy_acc(lo.prec, xs, lo.prec, pp, chi, 2, n, S.st), "x update"));
    }
    // r = s - omega t; ||r||^2 and <r, rhat>
    double e[3];
    {
      const void *z[1] = {t};
      const double w[2] = {omega.real(), omega.imag()};
      TRY(S.hip(blas_multi_caxpy_dots(lo.prec, z, w, 1, rs, rh, n, red, S.st), "r update"));
      TRY(S.result(3, e));
    }
    rho_new = std::conj(cd(e[1], e[2]));
    const double rr_now = e[0] / (sc * sc);
    progress_since_restart = true;
    if (verbose()) fprintf(stderr, "bicgstab it %d |r|/|b| %.3e\n", it, std::sqrt(rr_now) / bn);
    if (!std::isfinite(rr_now)) {
      status = set_error(ctx, LQCD_ERR_BREAKDOWN, "BiCGstab: the iterated residual is not finite");
      break;
    }
    if (rr_now <= stop || (mixed && rr_now < delta * delta * maxrr)) {
      double rrt;
      TRY(reliable_update(&rrt));
      if (rrt <= stop) { converged = true; break; }
    } else {
      maxrr = std::max(maxrr, rr_now);
    }
  }
  if (!converged) {
    // fold in the last sloppy correction (also after a breakdown: xs is valid)
    TRY(S.hip(blas_axpby(lo.prec, xs, hi.prec, xe, n, 1.0 / sc, 0.0, 1.0, 0.0, nullptr, S.st), "x update"));
  }
  if (verbose()) fprintf(stderr, "bicgstab: %d steps, %d shadow restarts\n", it, shadow_restarts);
  double tres;
  TRY(wilson_finish(S, hi, x_full, b_full, tmp_hi, y, bn, &tres));
  inf.iters = it;
  inf.true_residual = tres;
  inf.seconds = elapsed(t0);
  if (info) *info = inf;
  if (status != LQCD_OK) return status;
  if (!converged) return set_error(ctx, LQCD_ERR_NOT_CONVERGED, "BiCGstab reached max_iter");
  return LQCD_OK;
}
