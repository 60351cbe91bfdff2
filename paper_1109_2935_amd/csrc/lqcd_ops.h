// Host-side operator compositions shared by the entry points (api.cpp) and
// the solvers (solvers.cpp).
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "lqcd_internal.h"

namespace lqcd {

// Context scratch slots.
enum ScratchSlot {
  kSlotFlag = 0,
  kSlotSchurTmp = 1,
  kSlotSchwarz = 2,   // 4 slots: r, q, t, partials
  kSlotBatchCounter = 6,
  kSlotSolver = 8,    // solver work vectors start here (up to 80 slots)
  kSlotPtc = 100,     // network activations and gradients
};

RedScratch red_scratch(lqcd_context *ctx);
lqcd_status read_result(lqcd_context *ctx, hipStream_t st, int n, double *out);
const void *clover_block(const OpInfo &info, const void *clov, int parity);

lqcd_status wilson_hop(lqcd_context *ctx, const OpInfo &info, const Geom &g, int mode, void *out, const void *in,
                       const void *xin, const void *clov, int parity, double coef, int dagger, double *partials,
                       hipStream_t st, int nrhs = 1);
lqcd_status stag_hop(lqcd_context *ctx, const OpInfo &info, void *out, const void *in, const void *xin, int parity,
                     double coef, double xcoef, hipStream_t st, int nrhs = 1);
lqcd_status schur_apply(lqcd_context *ctx, const OpInfo &info, const Geom &g, void *out, const void *in, void *tmp,
                        int dagger, double *partials, hipStream_t st, int nrhs = 1);
lqcd_status check_nrhs(lqcd_context *ctx, const OpInfo &info, int nrhs);

// Autotuner (tune.cpp): the best of `cands` for `key`, timing `launch(c)` on
// the stream the first time the key is seen (if `may_time`); `fallback`
// otherwise. Results persist in the context (and in the file named by
// LQCD_TUNE_CACHE, if set). LQCD_TUNE=0 disables timing.
int tune_pick(lqcd_context *ctx, const std::string &key, const std::vector<int> &cands, int fallback, bool may_time,
              hipStream_t st, const std::function<hipError_t(int)> &launch);
std::string geom_key(const Geom &g);

// the learned preconditioner applied to an even residual (ptc_api.cpp)
lqcd_status ptc_apply(lqcd_context *ctx, const lqcd_operator *op, const lqcd_ptc_net *net, void *out_even,
                      const void *in_even, hipStream_t st);
lqcd_status schwarz_apply(lqcd_context *ctx, const OpInfo &info, const lqcd_schwarz_params *prm, void *out,
                          const void *in, int slot0, hipStream_t st);
lqcd_status check_schwarz(lqcd_context *ctx, const OpInfo &info, const lqcd_schwarz_params *prm);
// operator fields present and aligned (clover for Wilson, long links for staggered)
lqcd_status check_fields_internal(lqcd_context *ctx, const lqcd_operator *op);

// x += omega a_B r; r -= omega a_B q per Dirichlet block B, a_B = <q,r>_B / <q,q>_B
// from the per-segment partials (x read as zero when first)
hipError_t launch_mr_update(const Geom &g, int prec, void *x, void *r, const void *q, const double *partials, int nps,
                            bool first, double omega, hipStream_t st);

// Looks up this device's copy of the no-allocation entry point's device array
// (called at context creation, with the device current).
void noalloc_init_device(int dev);

}  // namespace lqcd
