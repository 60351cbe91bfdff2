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
struct PtcLayerDev {
  int cin, cout;
  int chunk_ch;    // input channels per forward K chunk
  int nchunk;      // forward K chunks
  int kchunk;      // real K per chunk (72 * chunk_ch padded to 32)
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
  L.mtiles = (8 * cout + 15) / 16;
  L.kadj = ((8 * cout + 31) / 32) * 32;
  L.madj_tiles = (72 * cin + 15) / 16;
  L.mw_tiles = (8 * cout + 15) / 16;
  return L;
}

// bytes of the packed fragments of one layer (forward, then adjoint)
inline size_t ptc_fwd_frag_bytes(const PtcLayerDev &L) { return (size_t)L.nchunk * L.mtiles * (L.kchunk / 32) * 64 * 16; }
inline size_t ptc_adj_frag_bytes(const PtcLayerDev &L) { return (size_t)L.madj_tiles * (L.kadj / 32) * 64 * 16; }

hipError_t launch_ptc_forward(const PtcGeo &q, const PtcLayerDev &L, const float *in, float *out, int par,
                              hipStream_t st);
hipError_t launch_ptc_bwd_data(const PtcGeo &q, const PtcLayerDev &L, const float *delta, float *gy, int par,
                               hipStream_t st);
hipError_t launch_ptc_adjoint_gather(const PtcGeo &q, int cin, const float *gy, float *gpsi, int par, hipStream_t st);
hipError_t launch_ptc_bwd_weight(const PtcGeo &q, const PtcLayerDev &L, const float *in, const float *delta,
                                 float *partial, int par, int groups, hipStream_t st);
hipError_t launch_ptc_weight_reduce(const PtcLayerDev &L, const float *partial, int groups, float *gw, int accumulate,
                                    hipStream_t st);
hipError_t launch_ptc_pack(const PtcLayerDev &L, const float *W, hipStream_t st);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, size_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, float gscale, hipStream_t st);

}  // namespace lqcd
