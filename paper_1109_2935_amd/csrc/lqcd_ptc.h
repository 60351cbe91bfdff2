// Device-side descriptions of the parallel-transport convolution network.
#pragma once

#include "lqcd_internal.h"

namespace lqcd {

constexpr int kPtcMaxLayers = 8;

struct PtcGeo {
  Geom g;
  const float *gauge;  // FP32 links of a Wilson operator instance (recon 18 or 12)
  int recon;
};

// One layer Cin -> Cout and the MFMA tiling of its three GEMMs.
//
// Forward K index: k = 8 q + 2 s' + r' over items q = p * Cin + i (path-major,
// so the items of one chunk share their path when Cin is a multiple of 4),
// padded to a multiple of 4 items (one 32-deep MFMA step); chunks of fw_ipc
// items are staged in LDS one at a time.
struct PtcLayerDev {
  int cin, cout;
  int chunk_ch;    // input channels per weight-gradient chunk
  int nchunk;      // weight-gradient chunks
  int kchunk;      // real K per weight-gradient chunk (72 * chunk_ch padded to 32)
  int fw_items;    // forward items 9 * Cin
  int fw_ks;       // forward 32-deep K steps (fw_items padded to 4, / 4)
  int fw_ipc;      // forward items per LDS chunk (multiple of 4, at most 16)
  int mtiles;      // forward M tiles (8 * cout real rows / 16, rounded up)
  int kadj;        // adjoint real K (8 * cout padded to 32)
  int madj_tiles;  // adjoint M tiles (72 * cin / 16, rounded up)
  int mw_tiles;    // weight-gradient M tiles (8 * cout / 16, rounded up)
  const void *A;     // packed forward fragments
  const void *Aadj;  // packed adjoint fragments
};

inline PtcLayerDev ptc_layer_desc(int cin, int cout) {
  PtcLayerDev L{};
  L.cin = cin;
  L.cout = cout;
  L.chunk_ch = cin < 4 ? cin : 4;
  L.nchunk = (cin + L.chunk_ch - 1) / L.chunk_ch;
  L.kchunk = ((72 * L.chunk_ch + 31) / 32) * 32;
  L.fw_items = 9 * cin;
  L.fw_ks = (L.fw_items + 3) / 4;
  L.fw_ipc = 4 * L.fw_ks < 16 ? 4 * L.fw_ks : 16;
  L.mtiles = (8 * cout + 15) / 16;
  L.kadj = ((8 * cout + 31) / 32) * 32;
  L.madj_tiles = (72 * cin + 15) / 16;
  L.mw_tiles = (8 * cout + 15) / 16;
  return L;
}

// bytes of the packed fragments of one layer (forward, then adjoint)
inline size_t ptc_fwd_frag_bytes(const PtcLayerDev &L) { return (size_t)L.mtiles * L.fw_ks * 64 * 16; }
inline size_t ptc_adj_frag_bytes(const PtcLayerDev &L) { return (size_t)L.madj_tiles * (L.kadj / 32) * 64 * 16; }

// neighbour table of the 8 hop paths, 2 * 8 * Vh ints (see ptc_nbr_kernel)
hipError_t launch_ptc_nbr(const Geom &g, int *tab, hipStream_t st);
// variant: 10 x sites per workgroup + waves per SIMD hint: 642 or 322
// in: BF16 activations; out: BF16 activations, or (out_f32, one channel) an FP32 packed spinor
// par: output parity, or -1 for both in one launch (workgroups of the two
// parities interleaved); zero_par: parity on which the input is known to
// vanish (-1: none)
hipError_t launch_ptc_forward(const PtcGeo &q, const PtcLayerDev &L, const int *nbr, const void *in, void *out,
                              int out_f32, int par, int variant, int zero_par, hipStream_t st);
// layer-0 activations from an FP32 packed even field
hipError_t launch_ptc_input(int64_t vh, const void *in_even, void *act, hipStream_t st);
hipError_t launch_ptc_bwd_data(const PtcGeo &q, const PtcLayerDev &L, const float *delta, float *gy, int par,
                               hipStream_t st);
hipError_t launch_ptc_adjoint_gather(const PtcGeo &q, int cin, const float *gy, float *gpsi, int par, hipStream_t st);
hipError_t launch_ptc_bwd_weight(const PtcGeo &q, const PtcLayerDev &L, const void *in, const float *delta,
                                 float *partial, int par, int groups, hipStream_t st);
hipError_t launch_ptc_weight_reduce(const PtcLayerDev &L, const float *partial, int groups, float *gw, int accumulate,
                                    hipStream_t st);
hipError_t launch_ptc_pack(const PtcLayerDev &L, const float *W, hipStream_t st);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, size_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, float gscale, hipStream_t st);

}  // namespace lqcd
