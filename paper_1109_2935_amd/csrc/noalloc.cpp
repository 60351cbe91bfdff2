// The even-odd operator for callers that cannot allocate (code under HIP
// graph capture, serving loops, harnesses that forbid hipMalloc): the same
// two fused kernels as lqcd_schur_apply, with their intermediate odd-parity
// spinor in a fixed device array of this library instead of context scratch.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy (kNoAllocScratchBytes) from module load until the
// process ends. Host code never passes the variable itself to a kernel (its
// name is a host-side stand-in there); the device address of each GPU's copy
// is looked up once per device with hipGetSymbolAddress, at context creation,
// and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lqcd_internal.h"
#include "lqcd_ops.h"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once).
hipError_t scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev] && g_err[dev] == hipSuccess) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p)
      g_ptr[dev] = p;
    else
      g_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
  }
  *out = g_ptr[dev];
  return g_ptr[dev] ? hipSuccess : g_err[dev];
}

// While it lives, kernel launches of the context use tuned or default launch
// parameters only: the autotuner's timing runs are skipped.
struct FrozenTuning {
  lqcd_context *ctx;
  bool old;
  explicit FrozenTuning(lqcd_context *c) : ctx(c), old(c->tune_frozen) { c->tune_frozen = true; }
  ~FrozenTuning() { ctx->tune_frozen = old; }
};

}  // namespace

namespace lqcd {

// Called by lqcd_context_create with the context's device current.
void noalloc_init_device(int dev) {
  void *p = nullptr;
  (void)scratch_address(dev, &p);
  (void)hipGetLastError();
}

}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status lqcd_schur_apply_noalloc(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in,
                                                int32_t dagger, const int32_t *block, int32_t nrhs,
                                                lqcd_stream stream) {
  OpInfo info;
  lqcd_status s = check_op(ctx, op, &info);
  if (s) return s;
  if (!ctx) return set_error(ctx, LQCD_ERR_INVALID_ARG, "context is NULL");
  if ((s = check_fields_internal(ctx, op))) return s;
  if ((s = check_nrhs(ctx, info, nrhs))) return s;
  auto aligned = [](const void *p) { return p && ((uintptr_t)p & 15) == 0; };
  if (!aligned(out) || !aligned(in)) return set_error(ctx, LQCD_ERR_INVALID_ARG, "bad field pointers");
  if (out == in) return set_error(ctx, LQCD_ERR_INVALID_ARG, "out and in must not alias");
  Geom g;
  if ((s = apply_cut(ctx, info, block, &g))) return s;
  if (op->action == LQCD_STAGGERED && g.has_cut)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED, "Dirichlet cut is implemented for the Wilson operator");
  const size_t need = info.spinor_bytes * (size_t)nrhs;
  if (need > kNoAllocScratchBytes)
    return set_error(ctx, LQCD_ERR_UNSUPPORTED,
                     "lqcd_schur_apply_noalloc: the intermediate spinor needs " + std::to_string(need) +
                         " bytes, more than its fixed " + std::to_string(kNoAllocScratchBytes) +
                         "-byte device array; use lqcd_schur_apply");
  int dev = 0;
  if ((s = hip_check(ctx, hipGetDevice(&dev), "hipGetDevice"))) return s;
  void *tmp = nullptr;
  if ((s = hip_check(ctx, scratch_address(dev, &tmp), "no-allocation scratch lookup"))) return s;
  FrozenTuning frozen(ctx);
  return schur_apply(ctx, info, g, out, in, tmp, dagger, nullptr, (hipStream_t)stream, nrhs);
}
