// C ABI entry points: validation, context and scratch management, packing
// calls and the operator compositions (Schur complement, staggered normal
// operator, additive Schwarz). Solvers live in solvers.cpp.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <string>

#include "lqcd_internal.h"
#include "lqcd_ops.h"

using namespace lqcd;

static std::string g_last_error;  // errors of calls made without a context

namespace lqcd {

lqcd_status set_error(lqcd_context *ctx, lqcd_status st, const std::string &msg) {
  if (ctx)
    ctx->last_error = msg;
  else
    g_last_error = msg;
  return st;
}

lqcd_status hip_check(lqcd_context *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return LQCD_OK;
  return set_error(ctx, LQCD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

Geom make_geom(const int32_t dims[4], const int32_t tile[4], int bc_t) {
  Geom g;
  memset(&g, 0, sizeof(g));
  for (int m = 0; m < 4; ++m) {
    g.L[m] = dims[m];
    g.B[m] = tile[m];
    g.NT[m] = dims[m] / tile[m];
    g.cut[m] = dims[m];
  }
  const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
  g.Vh = (int)(V / 2);
  g.Vt2 = tile[0] * tile[1] * tile[2] * tile[3] / 2;
  g.bc_t = bc_t;
  g.has_cut = 0;
  g.colour = -1;
  g.dVt2 = make_fastdiv(g.Vt2);
  g.dBxh = make_fastdiv(tile[0] / 2);
  g.dBy = make_fastdiv(tile[1]);
  g.dBz = make_fastdiv(tile[2]);
  g.dNTx = make_fastdiv(g.NT[0]);
  g.dNTy = make_fastdiv(g.NT[1]);
  g.dNTz = make_fastdiv(g.NT[2]);
  g.dNTxh = make_fastdiv(g.NT[0] >= 2 ? g.NT[0] / 2 : 1);
  for (int m = 0; m < 4; ++m) g.dcut[m] = make_fastdiv(dims[m]);
  return g;
}

lqcd_status check_op(lqcd_context *ctx, const lqcd_operator *op, OpInfo *info) {
  if (!op) return set_error(ctx, LQCD_ERR_INVALID_ARG, "operator is NULL");
  if (op->action != LQCD_WILSON_CLOVER && op->action != LQCD_STAGGERED)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "unknown action");
  int64_t V = 1;
  for (int m = 0; m < 4; ++m) {
    if (op->dims[m] < 2 || (op->dims[m] & 1))
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "lattice extents must be even and >= 2");
    if (op->tile[m] < 2 || (op->tile[m] & 1) || op->dims[m] % op->tile[m])
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "tile extents must be even and divide the lattice");
    V *= op->dims[m];
  }
  if (V / 2 >= (int64_t)1 << 30) return set_error(ctx, LQCD_ERR_UNSUPPORTED, "lattice too large");
  if (op->bc_t != 1 && op->bc_t != -1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bc_t must be +1 or -1");
  if (op->prec < LQCD_F64 || op->prec > LQCD_HALF) return set_error(ctx, LQCD_ERR_INVALID_ARG, "unknown precision");
  if (op->recon != 18 && op->recon != 12 && op->recon != 8)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "recon must be 18, 12 or 8");
  if (op->recon == 8 && (op->prec == LQCD_F16 || op->prec == LQCD_BF16 || op->prec == LQCD_HALF))
    return set_error(ctx, LQCD_ERR_UNSUPPORTED,
                     "8-real link compression divides by |U01|^2+|U02|^2 and is not supported in 16-bit storage");
  if (op->prec == LQCD_HALF && op->action != LQCD_WILSON_CLOVER)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "16-bit fixed-point storage is implemented for Wilson-clover");
  if (info) {
    info->op = op;
    info->g = make_geom(op->dims, op->tile, op->bc_t);
    info->prec = op->prec;
    info->recon = op->recon;
    info->nsp = spinor_reals(op->action);
    info->vh = (size_t)(V / 2);
    info->spinor_bytes = site_block_bytes(op->prec, info->nsp, info->vh, true);
  }
  return LQCD_OK;
}

lqcd_status apply_cut(lqcd_context *ctx, const OpInfo &info, const int32_t *block, Geom *g) {
  *g = info.g;
  if (!block) return LQCD_OK;
  for (int m = 0; m < 4; ++m) {
    if (block[m] < 2 || (block[m] & 1) || info.g.L[m] % block[m])
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "Dirichlet block extents must be even and divide the lattice");
    g->cut[m] = block[m];
    g->dcut[m] = make_fastdiv(block[m]);
    if (block[m] < info.g.L[m]) g->has_cut = 1;
  }
  return LQCD_OK;
}

lqcd_status check_nrhs(lqcd_context *ctx, const OpInfo &info, int nrhs) {
  if (nrhs < 1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "nrhs must be >= 1");
  if ((int64_t)info.vh * nrhs >= ((int64_t)1 << 31))
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "sites x right-hand sides must stay below 2^31");
  return LQCD_OK;
}

lqcd_status scratch(lqcd_context *ctx, int slot, size_t bytes, void **ptr) {
  if (slot >= (int)ctx->scratch.size()) {
    ctx->scratch.resize(slot + 1, nullptr);
    ctx->scratch_bytes.resize(slot + 1, 0);
  }
  if (ctx->scratch_bytes[slot] < bytes) {
    // A slot that must grow keeps its old buffer until the context is
    // destroyed: work already enqueued may still use it, and freeing it here
    // would stall every stream of the device in the middle of a call.
    if (ctx->scratch[slot]) {
      ctx->retired.push_back(ctx->scratch[slot]);
      ctx->scratch[slot] = nullptr;
      ctx->scratch_bytes[slot] = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_error(ctx, LQCD_ERR_OUT_OF_MEMORY, "scratch allocation of " + std::to_string(bytes) + " bytes failed");
    }
    ctx->scratch[slot] = p;
    ctx->scratch_bytes[slot] = bytes;
  }
  *ptr = ctx->scratch[slot];
  return LQCD_OK;
}

RedScratch red_scratch(lqcd_context *ctx) {
  RedScratch r;
  r.partials = ctx->red_partials;
  r.result = ctx->red_host_dev;
  r.max_wg = 1024;
  return r;
}

// The finishing launch of a reduction writes its result straight into pinned
// host memory, so reading it back is one stream synchronisation (no copy).
lqcd_status read_result(lqcd_context *ctx, hipStream_t st, int n, double *out) {
  const lqcd_status s = hip_check(ctx, hipStreamSynchronize(st), "stream synchronize");
  if (s) return s;
  for (int i = 0; i < n; ++i) out[i] = ctx->red_host[i];
  return LQCD_OK;
}

const void *clover_block(const OpInfo &info, const void *clov, int parity) {
  return (const char *)clov + (size_t)parity * site_block_bytes(info.prec, 72, info.vh, true);
}

// ---------------------------------------------------------------------------
// operator compositions used by the entry points and the solvers

// With LQCD_MRHS_MFMA=1 the link products of 16-bit operators with a multiple
// of 4 right-hand sides run on the matrix cores. The hopping term is bound by
// memory traffic, and on gfx950 the vector-ALU form measures faster, so it is
// the default. Read on every call.
static bool use_mfma(int prec, int nrhs, const double *partials) {
  const char *e = std::getenv("LQCD_MRHS_MFMA");
  return e && e[0] == '1' && (prec == LQCD_F16 || prec == LQCD_BF16) && nrhs % 4 == 0 && !partials;
}

lqcd_status wilson_hop(lqcd_context *ctx, const OpInfo &info, const Geom &g, int mode, void *out, const void *in,
                       const void *xin, const void *clov, int parity, double coef, int dagger, double *partials,
                       hipStream_t st, int nrhs) {
  WilsonLaunch w;
  w.g = g;
  w.prec = info.prec;
  w.recon = info.recon;
  w.out = out;
  w.in = in;
  w.gauge = info.op->gauge;
  w.clov = clov;
  w.xin = xin;
  w.parity = parity;
  w.coef = coef;
  w.dagger = dagger;
  w.mode = mode;
  w.partials = partials;
  w.nrhs = nrhs;
  w.mfma = use_mfma(info.prec, nrhs, partials) ? 1 : 0;
  w.block_threads = 256;
  // Workgroup size picked by the autotuner per (kernel, precision, links,
  // geometry, rhs). Calls that overwrite one of their inputs are not re-run
  // for timing; they use the tuned value if there is one, else 128.
  const bool rerunnable = out != in && out != xin;
  const std::string key = "wilson m" + std::to_string(mode) + (partials ? "r" : "") + " p" + std::to_string(info.prec) +
                          " r" + std::to_string(info.recon) + " " + geom_key(g) + " n" + std::to_string(nrhs) +
                          (w.mfma ? " mf" : "");
  w.block_threads = tune_pick(ctx, key, {64, 128, 256}, 128, rerunnable, st, [&](int bt) {
    WilsonLaunch v = w;
    v.block_threads = bt;
    return launch_wilson(v, st);
  });
  return hip_check(ctx, launch_wilson(w, st), "wilson dslash launch");
}

lqcd_status stag_hop(lqcd_context *ctx, const OpInfo &info, void *out, const void *in, const void *xin, int parity,
                     double coef, double xcoef, hipStream_t st, int nrhs) {
  StagLaunch l;
  l.g = info.g;
  l.prec = info.prec;
  l.recon = info.recon;
  l.out = out;
  l.in = in;
  l.fat = info.op->gauge;
  l.lng = info.op->long_links;
  l.xin = xin;
  l.parity = parity;
  l.coef = coef;
  l.xcoef = xcoef;
  l.c_long = info.op->c_long;
  l.nrhs = nrhs;
  l.block_threads = 256;
  const bool rerunnable = out != in && out != xin;
  const std::string key = "stag x" + std::to_string(xin != nullptr) + " p" + std::to_string(info.prec) + " r" +
                          std::to_string(info.recon) + " " + geom_key(info.g) + " n" + std::to_string(nrhs);
  l.block_threads = tune_pick(ctx, key, {64, 128, 256}, 128, rerunnable, st, [&](int bt) {
    StagLaunch v = l;
    v.block_threads = bt;
    return launch_staggered(v, st);
  });
  return hip_check(ctx, launch_staggered(l, st), "staggered dslash launch");
}

// Wilson: Mhat in = A_ee in - kappa^2 D_eo A_oo^-1 D_oe in (optionally cut, daggered,
// with per-workgroup partials <out,in>, <out,out>). Staggered: N_e in.
// tmp: one single-parity spinor of this operator.
lqcd_status schur_apply(lqcd_context *ctx, const OpInfo &info, const Geom &g, void *out, const void *in, void *tmp,
                        int dagger, double *partials, hipStream_t st, int nrhs) {
  const lqcd_operator *op = info.op;
  if (op->action == LQCD_WILSON_CLOVER) {
    lqcd_status s = wilson_hop(ctx, info, g, W_HOP_CLOV, tmp, in, nullptr, clover_block(info, op->clover_inv, 1), 1,
                               1.0, dagger, nullptr, st, nrhs);
    if (s) return s;
    return wilson_hop(ctx, info, g, W_XPAY_CLOV, out, tmp, in, clover_block(info, op->clover, 0), 0,
                      -op->kappa * op->kappa, dagger, partials, st, nrhs);
  }
  lqcd_status s = stag_hop(ctx, info, tmp, in, nullptr, 1, 1.0, 0.0, st, nrhs);
  if (s) return s;
  return stag_hop(ctx, info, out, tmp, in, 0, -0.25, op->mass * op->mass, st, nrhs);
}

// The Schwarz preconditioner on the blocks (additive: every block at once;
// multiplicative: the blocks of one colour after the other): out = K in, both
// packed even spinors of op_precond. Form 0 runs each MR step as two cut Schur
// launches and an update, with work vectors from scratch slots
// [slot0, slot0+4); forms 1 and 2 run every MR step of a block in one
// workgroup with the block in LDS (blocks equal to the tiles, 16-bit
// storage), x in memory (1) or in registers (2); forms 3 and 4 are 1 and 2
// with twice the threads and half the sites per thread (blocks with at least
// two sites per thread of 512; elsewhere they run as 1 and 2).
static lqcd_status schwarz_form(lqcd_context *ctx, const OpInfo &info, const Geom &g, const lqcd_schwarz_params *prm,
                                void *out, const void *in, int slot0, hipStream_t st, int form) {
  const lqcd_operator *op = info.op;
  const size_t sb = info.spinor_bytes;
  const double omega = prm->omega == 0 ? 1.0 : prm->omega;
  lqcd_status s;
  SapLaunch bl;
  bl.prec = info.prec;
  bl.recon = info.recon;
  bl.gauge = op->gauge;
  bl.clov_inv_odd = clover_block(info, op->clover_inv, 1);
  bl.clov_even = clover_block(info, op->clover, 0);
  bl.coef = -op->kappa * op->kappa;
  bl.omega = omega;
  bl.steps = prm->mr_steps;
  bl.x = out;
  bl.xreg = form == 2 || form == 4;
  bl.wide = form >= 3 && sap_block_wide_fits(g.Vt2);
  void *r = nullptr, *q = nullptr, *t = nullptr, *part = nullptr;
  if (form == 0 || prm->cycles > 0) {
    if ((s = scratch(ctx, slot0, sb, &r)) || (s = scratch(ctx, slot0 + 1, sb, &q)) ||
        (s = scratch(ctx, slot0 + 2, sb, &t)))
      return s;
  }
  // one (<q,r>, <q,q>) triple per reduction segment of min(tile sites, 64) sites
  const int seg = info.g.Vt2 < 64 ? info.g.Vt2 : 64;
  const size_t nseg = (info.vh + seg - 1) / seg;
  if (form == 0 && (s = scratch(ctx, slot0 + 3, nseg * 3 * sizeof(double), &part))) return s;
  const int nps = info.g.Vt2 > 64 ? info.g.Vt2 / 64 : 1;  // reduction segments per block
  if (prm->cycles == 0) {
    // additive: MR on every block at once
    if (form != 0) {
      bl.g = g;
      bl.r0 = in;
      bl.first = 1;
      return hip_check(ctx, launch_sap_block(bl, st), "schwarz block launch");
    }
    s = hip_check(ctx, hipMemcpyAsync(r, in, sb, hipMemcpyDeviceToDevice, st), "schwarz copy");
    if (s) return s;
    for (int it = 0; it < prm->mr_steps; ++it) {
      if ((s = schur_apply(ctx, info, g, q, r, t, 0, (double *)part, st))) return s;
      if ((s = hip_check(ctx, launch_mr_update(info.g, info.prec, out, r, q, (const double *)part, nps, it == 0, omega, st),
                         "schwarz MR update")))
        return s;
    }
    return LQCD_OK;
  }
  // multiplicative: the blocks of colour 0, then those of colour 1, `cycles`
  // times; each visit runs MR in the current residual r of the whole system on
  // its blocks only, and r = in - Mhat out is recomputed (uncut) for the next.
  // out starts at zero, since the residual reads it on every block.
  if ((s = hip_check(ctx, hipMemsetAsync(out, 0, sb, st), "schwarz clear"))) return s;
  const void *rc = in;  // the current residual
  Geom gc[2] = {g, g};
  gc[0].colour = 0;
  gc[1].colour = 1;
  const size_t n = info.vh * info.nsp / 2;
  for (int cyc = 0; cyc < prm->cycles; ++cyc) {
    for (int c = 0; c < 2; ++c) {
      if (form != 0) {
        bl.g = gc[c];
        bl.r0 = rc;
        bl.first = 0;
        if ((s = hip_check(ctx, launch_sap_block(bl, st), "schwarz block launch"))) return s;
      } else {
        if (rc != r && (s = hip_check(ctx, hipMemcpyAsync(r, rc, sb, hipMemcpyDeviceToDevice, st), "schwarz copy")))
          return s;
        for (int it = 0; it < prm->mr_steps; ++it) {
          if ((s = schur_apply(ctx, info, gc[c], q, r, t, 0, (double *)part, st))) return s;
          if ((s = hip_check(ctx, launch_mr_update(gc[c], info.prec, out, r, q, (const double *)part, nps,
                                                   cyc == 0 && it == 0, omega, st),
                             "schwarz MR update")))
            return s;
        }
      }
      if (cyc == prm->cycles - 1 && c == 1) break;
      if ((s = schur_apply(ctx, info, info.g, q, out, t, 0, nullptr, st))) return s;
      const double one = 1.0, mone = -1.0;
      const hipError_t e = info.prec == LQCD_HALF
                               ? blas_mrhs_axpby(info.prec, in, info.prec, q, (int64_t)info.vh, info.nsp, 1, &one,
                                                 &mone, nullptr, st)
                               : blas_axpby(info.prec, in, info.prec, q, n, 1.0, 0.0, -1.0, 0.0, nullptr, st);
      if ((s = hip_check(ctx, e, "schwarz residual"))) return s;
      std::swap(r, q);
      rc = r;
    }
  }
  return LQCD_OK;
}

// Does the block-resident form apply (blocks equal to the tiles, 16-bit
// storage, 12 or 18 link reals, a block in LDS)?
static bool schwarz_block_form_fits(const OpInfo &info, const Geom &g) {
  if ((info.prec != LQCD_F16 && info.prec != LQCD_BF16 && info.prec != LQCD_HALF) || info.recon == 8) return false;
  for (int m = 0; m < 4; ++m)
    if (g.cut[m] != info.g.B[m] || info.g.B[m] > 256) return false;
  return sap_block_spt(info.g.Vt2) != 0;
}

lqcd_status schwarz_apply(lqcd_context *ctx, const OpInfo &info, const lqcd_schwarz_params *prm, void *out,
                          const void *in, int slot0, hipStream_t st) {
  Geom g;
  lqcd_status s = apply_cut(ctx, info, prm->block, &g);
  if (s) return s;
  int form = 0;
  if (schwarz_block_form_fits(info, g)) {
    // the forms give the same result; the autotuner keeps the fastest, and
    // LQCD_SCHWARZ_FORM=0 .. 4 fixes the choice
    const char *f = std::getenv("LQCD_SCHWARZ_FORM");
    if (f && f[0] >= '0' && f[0] <= '4' && f[1] == 0) {
      form = f[0] - '0';
    } else {
      const std::string key = "schwarz p" + std::to_string(info.prec) + " r" + std::to_string(info.recon) + " " +
                              geom_key(g) + " m" + std::to_string(prm->mr_steps) + " c" + std::to_string(prm->cycles);
      std::vector<int> cands = {2, 1, 0};
      if (sap_block_wide_fits(info.g.Vt2)) cands = {4, 3, 2, 1, 0};
      form = tune_pick(ctx, key, cands, 2, out != in, st, [&](int c) {
        return schwarz_form(ctx, info, g, prm, out, in, slot0, st, c) == LQCD_OK ? hipSuccess : hipErrorUnknown;
      });
    }
  }
  return schwarz_form(ctx, info, g, prm, out, in, slot0, st, form);
}

lqcd_status check_schwarz(lqcd_context *ctx, const OpInfo &info, const lqcd_schwarz_params *prm) {
  if (!prm) return set_error(ctx, LQCD_ERR_INVALID_ARG, "schwarz params are NULL");
  if (info.op->action != LQCD_WILSON_CLOVER)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "the Schwarz preconditioner is implemented for Wilson-clover");
  lqcd_status s = check_fields_internal(ctx, info.op);
  if (s) return s;
  if (prm->mr_steps < 1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "mr_steps must be >= 1");
  if (prm->cycles < 0 || prm->cycles > 64) return set_error(ctx, LQCD_ERR_INVALID_ARG, "cycles must be in 0 .. 64");
  if (!(prm->omega >= 0 && prm->omega < 2))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "omega must be in (0, 2) (0 selects 1)");
  if (prm->cycles > 0 && (info.g.NT[0] & 1))
    return set_error(ctx, LQCD_ERR_UNSUPPORTED,
                     "multiplicative Schwarz needs an even number of blocks along x (the colours alternate there)");
  for (int m = 0; m < 4; ++m)
    if (prm->block[m] != info.op->tile[m])
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "Schwarz blocks must equal the operator's layout tile");
  const int v = info.g.Vt2;
  if (!((v <= 64 && 64 % v == 0) || (v > 64 && v % 64 == 0)))
    return set_error(ctx, LQCD_ERR_UNSUPPORTED,
                     "Schwarz block sites per parity must divide 64 or be a multiple of 64");
  return LQCD_OK;
}

lqcd_status check_fields_internal(lqcd_context *ctx, const lqcd_operator *op) {
  auto ok = [](const void *p) { return p && ((uintptr_t)p & 15) == 0; };
  if (!ok(op->gauge)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "operator gauge field missing or misaligned");
  if (op->action == LQCD_STAGGERED && !ok(op->long_links))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "staggered operator needs long links");
  if (op->action == LQCD_WILSON_CLOVER && (!ok(op->clover) || !ok(op->clover_inv)))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "Wilson-clover operator needs clover and clover_inv");
  return LQCD_OK;
}

}  // namespace lqcd

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

static bool aligned16(const void *p);

lqcd_status lqcd_context_create(lqcd_context **out) {
  if (!out) return set_error(nullptr, LQCD_ERR_INVALID_ARG, "ctx pointer is NULL");
  lqcd_context *ctx = new lqcd_context();
  hipGetDevice(&ctx->device);
  noalloc_init_device(ctx->device);
  lqcd_status s = LQCD_OK;
  if (hipMalloc(&ctx->red_partials, 1024 * kMaxRed * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&ctx->red_host, kMaxRed * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess)
    s = LQCD_ERR_OUT_OF_MEMORY;
  if (!s && hipHostGetDevicePointer((void **)&ctx->red_host_dev, ctx->red_host, 0) != hipSuccess)
    s = LQCD_ERR_DEVICE;
  if (s) {
    (void)hipGetLastError();
    lqcd_context_destroy(ctx);
    return set_error(nullptr, s, "context allocation failed");
  }
  ctx->red_partials_count = 1024 * kMaxRed;
  *out = ctx;
  return LQCD_OK;
}

lqcd_status lqcd_context_destroy(lqcd_context *ctx) {
  if (!ctx) return LQCD_OK;
  hipDeviceSynchronize();
  for (void *p : ctx->scratch)
    if (p) hipFree(p);
  for (void *p : ctx->retired) hipFree(p);
  if (ctx->red_partials) hipFree(ctx->red_partials);
  if (ctx->red_host) hipHostFree(ctx->red_host);
  delete ctx;
  return LQCD_OK;
}

lqcd_status lqcd_stream_copy(lqcd_context *ctx, void *dst, const void *src, size_t bytes, lqcd_stream stream) {
  if (!aligned16(dst) || !aligned16(src) || bytes % 16)
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
  const char *d = (const char *)dst, *s = (const char *)src;
  if (d < s + bytes && s < d + bytes) return set_error(ctx, LQCD_ERR_INVALID_ARG, "copy source and destination overlap");
  return hip_check(ctx, blas_stream_copy(dst, src, bytes, (hipStream_t)stream), "stream copy");
}

const char *lqcd_last_error(const lqcd_context *ctx) { return ctx ? ctx->last_error.c_str() : g_last_error.c_str(); }

lqcd_status lqcd_field_bytes(const lqcd_operator *op, int32_t kind, int32_t nrhs, size_t *bytes) {
  OpInfo info;
  lqcd_status s = check_op(nullptr, op, &info);
  if (s) return s;
  if (!bytes || nrhs < 1) return set_error(nullptr, LQCD_ERR_INVALID_ARG, "bad bytes pointer or nrhs");
  const size_t pb = prec_bytes(op->prec), vh = info.vh;
  size_t n = 0;
  switch (kind) {
    case LQCD_FIELD_SPINOR: n = site_block_bytes(op->prec, info.nsp, vh, true); break;
    case LQCD_FIELD_SPINOR_FULL: n = 2 * site_block_bytes(op->prec, info.nsp, vh, true); break;
    case LQCD_FIELD_GAUGE: n = 8 * vh * (op->action == LQCD_STAGGERED ? 18 : op->recon) * pb; break;
    case LQCD_FIELD_LONG:
      if (op->action != LQCD_STAGGERED) return set_error(nullptr, LQCD_ERR_INVALID_ARG, "long links are staggered only");
      n = 8 * vh * op->recon * pb;
      break;
    case LQCD_FIELD_CLOVER:
      if (op->action != LQCD_WILSON_CLOVER) return set_error(nullptr, LQCD_ERR_INVALID_ARG, "clover is Wilson only");
      n = 2 * site_block_bytes(op->prec, 72, vh, true);
      break;
    default: return set_error(nullptr, LQCD_ERR_INVALID_ARG, "unknown field kind");
  }
  *bytes = n * (size_t)nrhs;
  return LQCD_OK;
}

static bool aligned16(const void *p) { return p && ((uintptr_t)p & 15) == 0; }

lqcd_status lqcd_gauge_import(lqcd_context *ctx, const lqcd_operator *op, void *packed, const void *natural,
                              int32_t which, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (!aligned16(packed) || !aligned16(natural))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "field pointers must be non-NULL and 16-byte aligned");
  int recon;
  if (which == LQCD_FIELD_GAUGE)
    recon = op->action == LQCD_STAGGERED ? 18 : op->recon;
  else if (which == LQCD_FIELD_LONG && op->action == LQCD_STAGGERED)
    recon = op->recon;
  else
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "which must be LQCD_FIELD_GAUGE or (staggered) LQCD_FIELD_LONG");
  return hip_check(ctx, launch_gauge_import(info.g, op->prec, recon, packed, (const double *)natural, 0,
                                            (hipStream_t)stream),
                   "gauge import");
}

lqcd_status lqcd_long_link_build(lqcd_context *ctx, const lqcd_operator *op, void *packed_long,
                                 const void *natural_thin, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (op->action != LQCD_STAGGERED) return set_error(ctx, LQCD_ERR_INVALID_ARG, "long links need a staggered operator");
  if (!aligned16(packed_long) || !aligned16(natural_thin))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "field pointers must be non-NULL and 16-byte aligned");
  return hip_check(ctx, launch_gauge_import(info.g, op->prec, op->recon, packed_long, (const double *)natural_thin, 1,
                                            (hipStream_t)stream),
                   "long link build");
}

lqcd_status lqcd_clover_build(lqcd_context *ctx, const lqcd_operator *op, void *clover, void *clover_inv,
                              const void *natural_gauge, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if (op->action != LQCD_WILSON_CLOVER) return set_error(ctx, LQCD_ERR_INVALID_ARG, "clover needs a Wilson-clover operator");
  if (!aligned16(clover) || !aligned16(clover_inv) || !aligned16(natural_gauge))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "field pointers must be non-NULL and 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  void *flag;
  if ((s = scratch(ctx, kSlotFlag, 16, &flag))) return s;
  if ((s = hip_check(ctx, hipMemsetAsync(flag, 0, 16, st), "flag clear"))) return s;
  if ((s = hip_check(ctx, launch_clover_build(info.g, op->prec, op->kappa, op->csw, clover, clover_inv,
                                              (const double *)natural_gauge, (int *)flag, st),
                     "clover build")))
    return s;
  int h = 0;
  if ((s = hip_check(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "flag copy"))) return s;
  if ((s = hip_check(ctx, hipStreamSynchronize(st), "stream synchronize"))) return s;
  if (h) return set_error(ctx, LQCD_ERR_BREAKDOWN, "clover block not positive definite (Cholesky failed)");
  return LQCD_OK;
}

static lqcd_status spinor_io(lqcd_context *ctx, const lqcd_operator *op, void *packed, const void *natural,
                             int parity, int nrhs, lqcd_stream stream, bool imp) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (parity < -1 || parity > 1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "parity must be 0, 1 or -1");
  if ((s = check_nrhs(ctx, info, nrhs))) return s;
  if (!aligned16(packed) || !aligned16(natural))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "field pointers must be non-NULL and 16-byte aligned");
  for (int p = 0; p < 2; ++p) {
    if (parity >= 0 && p != parity) continue;
    char *blk = (char *)packed + (parity < 0 ? p * info.spinor_bytes * nrhs : 0);
    hipError_t e = imp ? launch_spinor_import(info.g, op->prec, info.nsp, blk, (const double *)natural, p, nrhs,
                                              (hipStream_t)stream)
                       : launch_spinor_export(info.g, op->prec, info.nsp, (double *)natural, blk, p, nrhs,
                                              (hipStream_t)stream);
    if ((s = hip_check(ctx, e, imp ? "spinor import" : "spinor export"))) return s;
  }
  return LQCD_OK;
}

lqcd_status lqcd_spinor_import(lqcd_context *ctx, const lqcd_operator *op, void *packed, const void *natural,
                               int32_t parity, int32_t nrhs, lqcd_stream stream) {
  return spinor_io(ctx, op, packed, natural, parity, nrhs, stream, true);
}

lqcd_status lqcd_spinor_export(lqcd_context *ctx, const lqcd_operator *op, void *natural, const void *packed,
                               int32_t parity, int32_t nrhs, lqcd_stream stream) {
  return spinor_io(ctx, op, (void *)packed, natural, parity, nrhs, stream, false);
}

lqcd_status lqcd_spinor_convert(lqcd_context *ctx, const lqcd_operator *op_out, void *out, const lqcd_operator *op_in,
                                const void *in, int32_t parity, int32_t nrhs, double scale, lqcd_stream stream) {
  OpInfo io, ii;
  lqcd_status s = check_op(ctx, op_out, &io);
  if (s) return s;
  if ((s = check_op(ctx, op_in, &ii))) return s;
  if (op_out->action != op_in->action) return set_error(ctx, LQCD_ERR_INVALID_ARG, "actions differ");
  bool same_tile = true;
  for (int m = 0; m < 4; ++m) {
    if (op_out->dims[m] != op_in->dims[m]) return set_error(ctx, LQCD_ERR_INVALID_ARG, "lattices differ");
    same_tile = same_tile && op_out->tile[m] == op_in->tile[m];
  }
  if (parity < -1 || parity > 1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "parity must be 0, 1 or -1");
  if ((s = check_nrhs(ctx, io, nrhs))) return s;
  if (!aligned16(out) || !aligned16(in)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  if (out == in && (op_out->prec != op_in->prec || !same_tile))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "in-place conversion needs equal precisions and tiles");
  hipStream_t st = (hipStream_t)stream;
  if (same_tile && op_out->prec != LQCD_HALF && op_in->prec != LQCD_HALF) {
    // the packed spinor layout does not depend on the precision: element-wise
    const size_t n = io.vh * io.nsp / 2 * (parity < 0 ? 2 : 1) * (size_t)nrhs;
    return hip_check(ctx, blas_convert(op_in->prec, in, op_out->prec, out, n, scale, st), "convert");
  }
  for (int p = 0; p < 2; ++p) {
    if (parity >= 0 && p != parity) continue;
    const size_t off_o = parity < 0 ? p * io.spinor_bytes * nrhs : 0, off_i = parity < 0 ? p * ii.spinor_bytes * nrhs : 0;
    if ((s = hip_check(ctx, launch_spinor_relayout(io.g, op_out->prec, (char *)out + off_o, ii.g, op_in->prec,
                                                   (const char *)in + off_i, io.nsp, p, nrhs, scale, st),
                       "relayout")))
      return s;
  }
  return LQCD_OK;
}

static lqcd_status check_fields(lqcd_context *ctx, const lqcd_operator *op, bool need_clover) {
  if (!aligned16(op->gauge)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "operator gauge field missing or misaligned");
  if (op->action == LQCD_STAGGERED && !aligned16(op->long_links))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "staggered operator needs long links");
  if (need_clover && op->action == LQCD_WILSON_CLOVER && (!aligned16(op->clover) || !aligned16(op->clover_inv)))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "Wilson-clover operator needs clover and clover_inv");
  return LQCD_OK;
}

lqcd_status lqcd_dslash(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in, int32_t out_parity,
                        int32_t dagger, const int32_t *block, int32_t nrhs, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if ((s = check_fields(ctx, op, false))) return s;
  if (out_parity != 0 && out_parity != 1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "out_parity must be 0 or 1");
  if ((s = check_nrhs(ctx, info, nrhs))) return s;
  if (!aligned16(out) || !aligned16(in))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "field pointers must be non-NULL and 16-byte aligned");
  if (out == in) return set_error(ctx, LQCD_ERR_INVALID_ARG, "out and in must not alias");
  Geom g;
  if ((s = apply_cut(ctx, info, block, &g))) return s;
  if (op->action == LQCD_STAGGERED && g.has_cut)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "Dirichlet cut is implemented for the Wilson operator");
  if (op->action == LQCD_WILSON_CLOVER)
    return wilson_hop(ctx, info, g, W_HOP, out, in, nullptr, nullptr, out_parity, 1.0, dagger, nullptr,
                      (hipStream_t)stream, nrhs);
  return stag_hop(ctx, info, out, in, nullptr, out_parity, dagger ? -1.0 : 1.0, 0.0, (hipStream_t)stream, nrhs);
}

lqcd_status lqcd_clover_apply(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in, int32_t parity,
                              int32_t inverse, int32_t nrhs, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (op->action != LQCD_WILSON_CLOVER) return set_error(ctx, LQCD_ERR_INVALID_ARG, "clover needs a Wilson-clover operator");
  if (!aligned16(op->clover) || !aligned16(op->clover_inv))
    return set_error(ctx, LQCD_ERR_INVALID_ARG, "operator clover fields missing or misaligned");
  if (parity != 0 && parity != 1) return set_error(ctx, LQCD_ERR_INVALID_ARG, "parity must be 0 or 1");
  if ((s = check_nrhs(ctx, info, nrhs))) return s;
  if (!aligned16(out) || !aligned16(in)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  const void *c = clover_block(info, inverse ? op->clover_inv : op->clover, parity);
  return hip_check(ctx, launch_clover_apply(info.g, op->prec, out, in, c, nrhs, (hipStream_t)stream), "clover apply");
}

lqcd_status lqcd_schur_apply(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in, int32_t dagger,
                             const int32_t *block, int32_t nrhs, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if ((s = check_fields(ctx, op, true))) return s;
  if ((s = check_nrhs(ctx, info, nrhs))) return s;
  if (!aligned16(out) || !aligned16(in)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  if (out == in) return set_error(ctx, LQCD_ERR_INVALID_ARG, "out and in must not alias");
  Geom g;
  if ((s = apply_cut(ctx, info, block, &g))) return s;
  if (op->action == LQCD_STAGGERED && g.has_cut)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "Dirichlet cut is implemented for the Wilson operator");
  void *tmp;
  if ((s = scratch(ctx, kSlotSchurTmp, info.spinor_bytes * nrhs, &tmp))) return s;
  return schur_apply(ctx, info, g, out, in, tmp, dagger, nullptr, (hipStream_t)stream, nrhs);
}

lqcd_status lqcd_dslash_batch(lqcd_context *ctx, const lqcd_dslash_job *jobs, int32_t njobs, int32_t dagger,
                              lqcd_stream stream) {
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if (!jobs || njobs < 1 || njobs > 8) return set_error(ctx, LQCD_ERR_INVALID_ARG, "need 1 to 8 jobs");
  BatchJob bj[8];
  int prec = -1, recon = -1;
  std::string key = "batch d" + std::to_string(dagger != 0);
  for (int j = 0; j < njobs; ++j) {
    OpInfo info;
    lqcd_status s = check_op(ctx, jobs[j].op, &info);
    if (s) return s;
    if (jobs[j].op->action != LQCD_WILSON_CLOVER)
      return set_error(ctx, LQCD_ERR_UNSUPPORTED, "batched dslash is implemented for Wilson-clover operators");
    if ((s = check_nrhs(ctx, info, jobs[j].nrhs))) return s;
    if (!aligned16(jobs[j].op->gauge)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "job gauge field missing");
    if (!aligned16(jobs[j].out) || !aligned16(jobs[j].in) || jobs[j].out == jobs[j].in)
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "job fields must be aligned, non-NULL and distinct");
    if (jobs[j].out_parity != 0 && jobs[j].out_parity != 1)
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "out_parity must be 0 or 1");
    if (j == 0) {
      prec = info.prec;
      recon = info.recon;
    } else if (info.prec != prec || info.recon != recon) {
      return set_error(ctx, LQCD_ERR_INVALID_ARG, "all jobs of a batch share precision and link format");
    }
    bj[j].g = info.g;
    bj[j].out = jobs[j].out;
    bj[j].in = jobs[j].in;
    bj[j].gauge = jobs[j].op->gauge;
    bj[j].parity = jobs[j].out_parity;
    bj[j].nrhs = jobs[j].nrhs;
    key += " " + geom_key(info.g) + "n" + std::to_string(jobs[j].nrhs);
  }
  key += " p" + std::to_string(prec) + " r" + std::to_string(recon);
  void *counter;
  lqcd_status s = scratch(ctx, kSlotBatchCounter, 256, &counter);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  // candidates: workgroup size (= pairs per work item) x persistent grid (0: one workgroup per item)
  static const BatchTune cands[] = {{128, 128, 2048}, {128, 128, 4096}, {256, 256, 1024}, {256, 256, 2048},
                                    {64, 64, 4096},   {128, 128, 8192}, {128, 128, 0},    {256, 256, 0},
                                    {64, 64, 0}};
  const int ncand = sizeof(cands) / sizeof(cands[0]);
  std::vector<int> idx(ncand);
  for (int i = 0; i < ncand; ++i) idx[i] = i;
  bool distinct = true;
  for (int a = 0; a < njobs; ++a)
    for (int b = 0; b < njobs; ++b)
      if (bj[a].out == bj[b].in || (a != b && bj[a].out == bj[b].out)) distinct = false;
  // the same link-product path as lqcd_dslash for each job
  const int mf = use_mfma(prec, 4, nullptr) ? 1 : 0;
  if (mf) key += " mf";
  const int pick = tune_pick(ctx, key, idx, 2, distinct, st, [&](int i) {
    return launch_wilson_batch(prec, recon, bj, njobs, dagger, cands[i], mf, (unsigned *)counter, st);
  });
  return hip_check(ctx, launch_wilson_batch(prec, recon, bj, njobs, dagger, cands[pick], mf, (unsigned *)counter, st),
                   "batched dslash launch");
}

lqcd_status lqcd_schwarz_precond(lqcd_context *ctx, const lqcd_operator *op_precond, const lqcd_schwarz_params *params,
                                 void *out_even, const void *in_even, lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op_precond, &info);
  if (s) return s;
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if ((s = check_schwarz(ctx, info, params))) return s;
  if (!aligned16(out_even) || !aligned16(in_even)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  if (out_even == in_even) return set_error(ctx, LQCD_ERR_INVALID_ARG, "out and in must not alias");
  return schwarz_apply(ctx, info, params, out_even, in_even, kSlotSchwarz, (hipStream_t)stream);
}

}  // extern "C"
