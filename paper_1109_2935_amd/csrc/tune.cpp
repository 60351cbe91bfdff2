// Autotuner for launch parameters (workgroup size of the stencil kernels,
// work-item size and grid of the persistent batched launch).
//
// The first time a key (kernel, precision, link format, geometry, number of
// right-hand sides) is seen, every candidate is timed with HIP events on the
// caller's stream (one warm-up and three timed launches each) and the fastest
// is kept in the context. With LQCD_TUNE_CACHE=<file> results are also read
// from and appended to a text file ("key<TAB>value" lines) tagged with the
// device architecture; LQCD_TUNE=0 disables timing (fallback values).
// The candidates of the stencil and batch kernels compute the same result
// (each output element is written by one thread with a fixed summation
// order). The network's forward forms differ in the order of their FP32 sums
// (dot2 or matrix-core colour products), so there the choice can change an
// output by BF16 roundings; LQCD_PTC_VARIANT or a cache file fixes it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <algorithm>
#include <fstream>
#include <sstream>

#include "lqcd_internal.h"
#include "lqcd_ops.h"

namespace lqcd {

std::string geom_key(const Geom &g) {
  std::ostringstream o;
  o << g.L[0] << "x" << g.L[1] << "x" << g.L[2] << "x" << g.L[3] << "/" << g.B[0] << "x" << g.B[1] << "x" << g.B[2]
    << "x" << g.B[3] << (g.has_cut ? "c" : "") << (g.colour >= 0 ? "h" : "");
  return o.str();
}

static std::string arch_tag() {
  static std::string tag;
  if (tag.empty()) {
    hipDeviceProp_t p;
    int dev = 0;
    hipGetDevice(&dev);
    tag = (hipGetDeviceProperties(&p, dev) == hipSuccess) ? std::string(p.gcnArchName) : std::string("unknown");
    const size_t colon = tag.find(':');
    if (colon != std::string::npos) tag = tag.substr(0, colon);
  }
  return tag;
}

static void load_file(lqcd_context *ctx) {
  const char *t = std::getenv("LQCD_TUNE");
  ctx->tune_enabled = !(t && t[0] == '0');
  const char *f = std::getenv("LQCD_TUNE_CACHE");
  if (!f || ctx->tune_file == f) return;
  ctx->tune_file = f;
  std::ifstream in(f);
  std::string line;
  const std::string pre = arch_tag() + " ";
  while (std::getline(in, line)) {
    const size_t tab = line.rfind('\t');
    if (tab == std::string::npos || line.compare(0, pre.size(), pre) != 0) continue;
    ctx->tuned[line.substr(pre.size(), tab - pre.size())] = std::atoi(line.c_str() + tab + 1);
  }
}

int tune_pick(lqcd_context *ctx, const std::string &key, const std::vector<int> &cands, int fallback, bool may_time,
              hipStream_t st, const std::function<hipError_t(int)> &launch) {
  if (!ctx) return fallback;
  load_file(ctx);
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) return it->second;
  if (!may_time || !ctx->tune_enabled || ctx->tune_frozen) return fallback;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fallback;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fallback;
  }
  // two interleaved rounds over the candidates, each candidate scored by its
  // faster round, so that clock ramp-up or a cold cache in the first
  // measurements does not decide the choice
  int best = fallback;
  float best_ms = 1e30f;
  std::vector<float> score(cands.size(), 1e30f);
  for (int round = 0; round < 2; ++round) {
    for (size_t i = 0; i < cands.size(); ++i) {
      const int c = cands[i];
      if (launch(c) != hipSuccess) continue;
      hipEventRecord(e0, st);
      bool ok = true;
      for (int r = 0; r < 3 && ok; ++r) ok = launch(c) == hipSuccess;
      hipEventRecord(e1, st);
      if (!ok || hipEventSynchronize(e1) != hipSuccess) continue;
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      score[i] = std::min(score[i], ms);
    }
  }
  for (size_t i = 0; i < cands.size(); ++i)
    if (score[i] < best_ms) {
      best_ms = score[i];
      best = cands[i];
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  (void)hipGetLastError();
  ctx->tuned[key] = best;
  if (!ctx->tune_file.empty()) {
    std::ofstream out(ctx->tune_file, std::ios::app);
    out << arch_tag() << " " << key << "\t" << best << "\n";
  }
  return best;
}

}  // namespace lqcd

extern "C" lqcd_status lqcd_tuned_choices(lqcd_context *ctx, char *buf, size_t cap, size_t *len) {
  if (!ctx || !len) return lqcd::set_error(ctx, LQCD_ERR_INVALID_ARG, "context and len must not be NULL");
  std::string text;
  for (const auto &kv : ctx->tuned) text += kv.first + "\t" + std::to_string(kv.second) + "\n";
  *len = text.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, text.size());
    memcpy(buf, text.data(), n);
    buf[n] = 0;
  }
  return LQCD_OK;
}
