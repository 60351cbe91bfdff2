// Gauge-equivariant parallel-transport convolution (PTC) network kernels.
//
// One layer maps Cin channels of colour-spinor fields to Cout channels:
//   psi'_o(x) = sum_i sum_p W[o,i,p] (T_p psi_i)(x),
// p = 0 identity, 1+2mu forward hop (U_mu(x) psi(x+mu)), 2+2mu backward hop
// (U_mu(x-mu)^+ psi(x-mu)), W[o,i,p] a complex 4x4 spin matrix. The paper has
// no such network; it is used as a learned preconditioner of flexible GCR
// (Section III-B: the outer solver must be flexible).
//
// Activations between layers are BF16, channel-interleaved per site (packed
// index site * C + channel) in 16-byte chunks of 8 reals, chunk-major within
// each parity block (act_load / act_store); the network output is an FP32
// packed spinor. The channel mixing is a complex GEMM
//   O[(o,s)][(c,x)] = sum_{(i,p,s')} W[(o,s)][(i,p,s')] Y[(i,p,s')][(c,x)],
// Y = T_p psi_i, run on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) in real form with interleaved real/imaginary rows:
//   A[2m+r][2k+r'] = [[Wr, -Wi],[Wi, Wr]][r][r'],  B[2k+r'][n] = (Yr, Yi)[r'].
// A workgroup owns a tile of 16 sites of one parity: it builds Y for a chunk of
// input channels in LDS (parallel transport, converted to BF16), then each of
// its 4 waves runs the MFMA tiles it owns; weights come pre-packed in the
// per-lane A-operand order, so each A fragment is one coalesced 16-byte load.
#include <type_traits>

#include "lqcd_internal.h"
#include "lqcd_ptc.h"

namespace lqcd {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

// (x, y) rounded to nearest-even BF16, x in the low half
__device__ __forceinline__ bf16x2_t pack_bf16x2(float x, float y) {
  return __builtin_convertvector(f32x2_t{x, y}, bf16x2_t);
}

constexpr int kTile = 16;      // sites per workgroup tile
constexpr int kPtcThreads = 256;
constexpr int kLdsPad = 8;     // bf16 padding per LDS row (bank spread)

// activation access: 24 reals of packed index idx in a parity block of vs entries
__device__ __forceinline__ void act_load(const bf16 *__restrict__ blk, int64_t vs, int64_t idx, float *r) {
  load_chunks<bf16, 24, 8, float>(blk, vs, idx, r);
}

__device__ __forceinline__ f32x4_t mfma_bf16(const bf16x8_t &a, const bf16x8_t &b, const f32x4_t &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// (T_p psi)(x) for one channel of a channel-interleaved activation field.
// x: site index of parity `par`; the identity path reads parity par, the hops
// read parity 1 - par. Boundary phases as in the Dirac operator.
template <int RECON>
__device__ __forceinline__ void transport_one(const PtcGeo &q, const bf16 *__restrict__ act, int C, int ch, int p,
                                              const Site &x, int s, cpx<float> (&out)[4][3]) {
  const int par = x.p;
  const int64_t vh = q.g.Vh, vs = vh * C;
  const bf16 *blk_same = act + (int64_t)par * vs * 24;
  const bf16 *blk_other = act + (int64_t)(1 - par) * vs * 24;
  float r[24];
  if (p == 0) {
    act_load(blk_same, vs, (int64_t)s * C + ch, r);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) out[sp][c] = mk<float>(r[6 * sp + 2 * c], r[6 * sp + 2 * c + 1]);
    return;
  }
  const int mu = (p - 1) >> 1;
  const bool fwd = ((p - 1) & 1) == 0;
  int w = 0, n = 0;
  switch (mu) {
    case 0: n = hop<0>(q.g, x, fwd ? 1 : -1, &w); break;
    case 1: n = hop<1>(q.g, x, fwd ? 1 : -1, &w); break;
    case 2: n = hop<2>(q.g, x, fwd ? 1 : -1, &w); break;
    default: n = hop<3>(q.g, x, fwd ? 1 : -1, &w); break;
  }
  act_load(blk_other, vs, (int64_t)n * C + ch, r);
  float lv[RECON];
  if (fwd)
    load_site<float, RECON, float>(q.gauge + (int64_t)(2 * mu + par) * vh * RECON, vh, s, lv);
  else
    load_site<float, RECON, float>(q.gauge + (int64_t)(2 * mu + 1 - par) * vh * RECON, vh, n, lv);
  const Link<float> U0 = unpack_link<RECON, float>(lv);
  const float ph = (mu == 3 && (w & 1) && q.g.bc_t < 0) ? -1.f : 1.f;
  Link<float> U;  // U or U^+, times the boundary sign
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) U.m[a][b] = ph * (fwd ? U0.m[a][b] : conj(U0.m[b][a]));
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    cpx<float> v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = mk<float>(r[6 * sp + 2 * c], r[6 * sp + 2 * c + 1]);
    su3_mv(U, v, out[sp]);
  }
}

__device__ __forceinline__ void transport_any(const PtcGeo &q, const bf16 *act, int C, int ch, int p, const Site &x,
                                              int s, cpx<float> (&out)[4][3]) {
  if (q.recon == 12)
    transport_one<12>(q, act, C, ch, p, x, s, out);
  else
    transport_one<18>(q, act, C, ch, p, x, s, out);
}

// Neighbour table of the transport paths: entry [par][p-1][s] (p = 1..8) is
// the index of the site reached by path p from site s of parity par, with
// bit 31 set where the hop crosses the antiperiodic time boundary.
__global__ void ptc_nbr_kernel(Geom g, int *tab) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int par = blockIdx.y;
  if (s >= g.Vh) return;
  const Site x = decode_site(g, s, par);
  int *t = tab + (int64_t)par * 8 * g.Vh + s;
  int w, n;
#define PTC_NBR(MU)                                                              \
  n = hop<MU>(g, x, 1, &w);                                                      \
  t[(2 * MU) * (int64_t)g.Vh] = n | ((MU == 3 && (w & 1) && g.bc_t < 0) << 31);  \
  n = hop<MU>(g, x, -1, &w);                                                     \
  t[(2 * MU + 1) * (int64_t)g.Vh] = n | ((MU == 3 && (w & 1) && g.bc_t < 0) << 31);
  PTC_NBR(0)
  PTC_NBR(1)
  PTC_NBR(2)
  PTC_NBR(3)
#undef PTC_NBR
}

// Transport of NCH channels i0, i0 + kstep, ... of one path p at site s of
// parity par, written to LDS as BF16 (row stride `cstride` between colours, 8
// K values per channel: spin-major, re/im interleaved; channel i0 + k kstep at
// column 8 k kstep). The link and the neighbour are read once; the NCH
// channel loads are issued together.
template <int RECON, int NCH>
__device__ __forceinline__ void transportn_lds(const PtcGeo &q, const int *__restrict__ nbr, const bf16 *__restrict__ act,
                                               int C, int i0, int kstep, int p, int par, int s, __bf16 *dst,
                                               int cstride) {
  const int64_t vh = q.g.Vh, vs = vh * C;
  int n = s;
  float ph = 1.f;
  if (p != 0) {
    const int e = nbr[((int64_t)par * 8 + p - 1) * vh + s];
    n = e & 0x7fffffff;
    ph = e < 0 ? -1.f : 1.f;
  }
  const bf16 *blk = act + (int64_t)(p == 0 ? par : 1 - par) * vs * 24;
  float r[NCH][24];
#pragma unroll
  for (int k = 0; k < NCH; ++k) act_load(blk, vs, (int64_t)n * C + i0 + k * kstep, r[k]);
  if (p != 0) {
    const int mu = (p - 1) >> 1;
    const bool fwd = ((p - 1) & 1) == 0;
    float lv[RECON];
    // forward: U_mu(x) at x; backward: U_mu(x - mu)^+ at the neighbour
    load_site<float, RECON, float>(q.gauge + (int64_t)(2 * mu + (fwd ? par : 1 - par)) * vh * RECON, vh, fwd ? s : n,
                                   lv);
    const Link<float> U0 = unpack_link<RECON, float>(lv);
    // the matrix applied: U, or U^+ for a backward hop (selected once), times the boundary sign
    Link<float> U;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const cpx<float> e = fwd ? U0.m[a][b] : conj(U0.m[b][a]);
        U.m[a][b] = ph * e;
      }
#pragma unroll
    for (int k = 0; k < NCH; ++k)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        cpx<float> v[3], u[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = mk<float>(r[k][6 * sp + 2 * c], r[k][6 * sp + 2 * c + 1]);
        su3_mv(U, v, u);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          r[k][6 * sp + 2 * c] = u[c].re;
          r[k][6 * sp + 2 * c + 1] = u[c].im;
        }
      }
  }
#pragma unroll
  for (int k = 0; k < NCH; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bf16x8_t v;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        v[2 * sp] = (__bf16)r[k][6 * sp + 2 * c];
        v[2 * sp + 1] = (__bf16)r[k][6 * sp + 2 * c + 1];
      }
      *reinterpret_cast<bf16x8_t *>(dst + c * cstride + 8 * k * kstep) = v;
    }
}

__device__ __forceinline__ bf16x8_t lds_frag(const __bf16 *row) {
  return *reinterpret_cast<const bf16x8_t *>(row);
}

// ---------------------------------------------------------------------------
// forward: out (Cout channels, parity par) = sum W (T psi_in)
//
// A workgroup owns NS sites, i.e. N = 3 * NS GEMM columns
// (n = colour * NS + site). Per K chunk its 256 threads transport
// kFwSites x fw_ipc items into LDS (BF16, row n holds the chunk's K values),
// then each wave multiplies its block of 16x16 output tiles: m-tiles
// {mbase + 4j} by n-tiles [nbase, nbase + nn), so each B fragment read from
// LDS feeds up to two MFMAs and each A fragment (pre-packed, one 16-byte load
// per lane) up to 3 NS / 16. NS = 64 halves the weight traffic per site of
// NS = 32 but needs twice the accumulators; the launch picks one by timing
// (both give identical results: the K order of every output is the same).

constexpr int kFwRow = 16 * 8 + kLdsPad;  // bf16 per LDS row: 16 items x 8 K values + padding

// PIPE: 0 generic; 1 and 2 the pipelined 16-channel form with the colour
// products on BF16 dot2 (1) or on 4x4x4 matrix-core blocks (2); 3 and 4 the
// same split between waves: the first half of the waves transport path p + 1
// into one LDS buffer while the second half multiply path p from the other
// (one barrier per path, so the vector and matrix work of a workgroup overlap).
// NTH threads (NTH / 64 waves) per workgroup; RC the link format (12 or 18
// reals) of the pipelined forms.
template <int NS, int WPE, int PIPE, int NTH = kPtcThreads, int RC = 18>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(WPE)))
ptc_forward_kernel(PtcGeo q, PtcLayerDev L, const int *nbr, const bf16 *in, void *out, int out_f32, int par_arg,
                   int zero_par) {
  constexpr int kFwSites = NS, NT = 3 * NS / 16;
  constexpr bool SPLIT = PIPE >= 3;
  constexpr int TRANS = (PIPE == 2 || PIPE == 4) ? 2 : 1;  // colour products: 1 dot2, 2 matrix cores
  constexpr int NW = NTH / 64;                // waves
  constexpr int NWC = SPLIT ? NW / 2 : NW;    // waves doing the matrix products
  constexpr int JM = (8 + NWC - 1) / NWC;     // m-tiles per wave at most (8 m-tiles for 16 output channels)
  constexpr int kBuf = 3 * NS * kFwRow;       // bf16 per LDS buffer of transported inputs
  __shared__ __align__(16) __bf16 Bt[(SPLIT ? 2 : 1) * kBuf];
  // each XCD takes a contiguous range of site tiles, so that the neighbours'
  // activations are read from its own L2; with par_arg < 0 both output
  // parities are computed, workgroups 2t and 2t + 1 taking tile t of the even
  // and the odd sites, so that an input site's reads as a hop input (by one
  // parity) and as its own identity input (by the other) come close in time
  int wl = xcd_remap(blockIdx.x, gridDim.x);
  const int par = par_arg < 0 ? (wl & 1) : par_arg;
  if (par_arg < 0) wl >>= 1;
  const int s0 = wl * kFwSites;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool producer = SPLIT && wave < NW / 2;  // (split forms) transports only
  const int cw = SPLIT ? wave - NW / 2 : wave;   // index among the waves doing products
  // this wave's output tiles
  int mbase = 0, nm = 0, nbase = 0, nn = 0;
  if (producer) {
  } else if (L.mtiles >= NWC) {
    mbase = cw;
    nm = (L.mtiles - cw + NWC - 1) / NWC;
    nbase = 0;
    nn = NT;
  } else {
    const int split = NWC / L.mtiles;  // waves per m-tile
    mbase = cw % L.mtiles;
    nm = 1;
    nn = (NT + split - 1) / split;
    nbase = (cw / L.mtiles) * nn;
    nn = max(0, min(nn, NT - nbase));
  }
  f32x4_t acc[JM][NT];
#pragma unroll
  for (int j = 0; j < JM; ++j)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[j][t] = f32x4_t{0, 0, 0, 0};
  const bf16x8_t *A = (const bf16x8_t *)L.A;
  // one K chunk (items q0 .. q0+ipc-1) from LDS into the accumulators
  auto mma_chunk = [&](auto &ac, const __bf16 *Bb, int q0, int ipc) {
    for (int kl = 0; kl < ipc / 4; ++kl) {
      const int ks = q0 / 4 + kl;
      bf16x8_t a[JM];
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (j < nm) a[j] = A[((size_t)(mbase + NWC * j) * L.fw_ks + ks) * 64 + lane];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t < nn) {
          const bf16x8_t b = lds_frag(Bb + ((nbase + t) * 16 + (lane & 15)) * kFwRow + kl * 32 + 8 * (lane >> 4));
#pragma unroll
          for (int j = 0; j < JM; ++j)
            if (j < nm) ac[j][t] = mfma_bf16(a[j], b, ac[j][t]);
        }
      }
    }
  };
  // the same product with compile-time tile counts (all loads of a K step
  // issued before its MFMAs, no per-tile branches): SM m-tiles x SN n-tiles
  auto mma_static = [&](auto smc, auto snc, auto &ac, const __bf16 *Bb, int q0) {
    constexpr int SM = decltype(smc)::value, SN = decltype(snc)::value;
#pragma unroll
    for (int kl = 0; kl < 4; ++kl) {
      const int ks = q0 / 4 + kl;
      bf16x8_t a[SM], b[SN];
#pragma unroll
      for (int j = 0; j < SM; ++j) a[j] = A[((size_t)(mbase + NWC * j) * L.fw_ks + ks) * 64 + lane];
#pragma unroll
      for (int t = 0; t < SN; ++t)
        b[t] = lds_frag(Bb + ((nbase + t) * 16 + (lane & 15)) * kFwRow + kl * 32 + 8 * (lane >> 4));
#pragma unroll
      for (int t = 0; t < SN; ++t)
#pragma unroll
        for (int j = 0; j < SM; ++j) ac[j][t] = mfma_bf16(a[j], b[t], ac[j][t]);
    }
  };
  // Output. Row m = 16 mt + 4 g + jj (g = lane / 16) of a tile is channel
  // o = 2 mt + g / 2, spin 2 (g % 2) + jj / 2, real/imaginary part jj % 2;
  // column n = 16 nt + lane % 16. The tile is staged in LDS as
  // [site][channel][24 reals] (rows padded against bank conflicts) by stage(),
  // then stored in whole 16-byte chunks by store_out() (after a barrier).
  const int g = lane >> 4;
  const int64_t vs = (int64_t)q.g.Vh * L.cout;
  const int srow = L.cout * 24 + (out_f32 ? 4 : 8);  // staging row, in elements of the output type
  auto stage = [&](const f32x4_t (&ac)[JM][NT]) {
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      if (j >= nm) continue;
      const int o = 2 * (mbase + NWC * j) + (g >> 1);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t >= nn) continue;
        const int n = (nbase + t) * 16 + (lane & 15);
        const int c = n / kFwSites, sl = n % kFwSites;
        if (o < L.cout) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = (2 * (g & 1) + h) * 6 + 2 * c;
            if (!out_f32) {
              Bt[sl * srow + o * 24 + r] = (__bf16)ac[j][t][2 * h];
              Bt[sl * srow + o * 24 + r + 1] = (__bf16)ac[j][t][2 * h + 1];
            } else {
              *reinterpret_cast<float2 *>(reinterpret_cast<float *>(Bt) + sl * srow + o * 24 + r) =
                  make_float2(ac[j][t][2 * h], ac[j][t][2 * h + 1]);
            }
          }
        }
      }
    }
  };
  auto store_out = [&]() {
    const int per_chunk = kFwSites * L.cout;
    if (!out_f32) {
      bf16 *blk = (bf16 *)out + (int64_t)par * vs * 24;
      for (int w = threadIdx.x; w < 3 * per_chunk; w += NTH) {
        const int k = w / per_chunk, rem = w - k * per_chunk;
        const int sl = rem / L.cout, o = rem - sl * L.cout;
        const int s = s0 + sl;
        if (s < q.g.Vh)
          *reinterpret_cast<uint4 *>(blk + ((int64_t)k * vs + (int64_t)s * L.cout + o) * 8) =
              *reinterpret_cast<const uint4 *>(Bt + sl * srow + o * 24 + 8 * k);
      }
    } else {
      // FP32 packed spinor (chunks of 4 reals); the network's last layer (one channel)
      const float *Sf = reinterpret_cast<const float *>(Bt);
      float *blk = (float *)out + (int64_t)par * vs * 24;
      for (int w = threadIdx.x; w < 6 * per_chunk; w += NTH) {
        const int k = w / per_chunk, rem = w - k * per_chunk;
        const int sl = rem / L.cout, o = rem - sl * L.cout;
        const int s = s0 + sl;
        if (s < q.g.Vh)
          *reinterpret_cast<float4 *>(blk + ((int64_t)k * vs + (int64_t)s * L.cout + o) * 4) =
              *reinterpret_cast<const float4 *>(Sf + sl * srow + o * 24 + 4 * k);
      }
    }
  };
  if constexpr (PIPE != 0) {
    // 16 input channels: TPS threads per site, thread un taking channels
    // un + TPS k (k < KC); one path per chunk; the loads of path p + 1 are
    // issued before the matrix products of path p, so their latency overlaps them.
    constexpr int TPS = (SPLIT ? NTH / 2 : NTH) / kFwSites, KC = 16 / TPS;
    static_assert(TPS * KC == 16 && (TPS == 8 || TPS == 16), "pipelined path: 8 or 16 threads per site");
    __shared__ int nbL[kFwSites][8];
    // (in the split forms the transporting threads are 0 .. NTH / 2 - 1)
    const int un = threadIdx.x % TPS, sl = (threadIdx.x / TPS) % kFwSites, s = s0 + sl;
    const bool valid = s < q.g.Vh;
    const int64_t vh = q.g.Vh, vs = vh * 16;
    if (un < 8 && (!SPLIT || producer)) nbL[sl][un] = valid ? nbr[((int64_t)par * 8 + un) * vh + s] : 0;
    __syncthreads();
    // activation words and link reals of the path in flight
    static_assert(RC == 12 || RC == 18, "link format");
    uint4 rawA[KC][3];
    float lvA[RC] = {};
    // (always inlined: the register sets are passed by reference and must not
    // go to memory)
    auto issue = [&](uint4 (&raw)[KC][3], float (&lv)[RC], int p) __attribute__((always_inline)) {
      if (!valid) return;
      const int n = p == 0 ? s : (nbL[sl][p - 1] & 0x7fffffff);
      const bf16 *blk = in + (int64_t)(p == 0 ? par : 1 - par) * vs * 24;
#pragma unroll
      for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          raw[k][c] = *reinterpret_cast<const uint4 *>(blk + ((int64_t)c * vs + (int64_t)n * 16 + un + TPS * k) * 8);
      if (p != 0) {
        const int mu = (p - 1) >> 1;
        const bool fwd = ((p - 1) & 1) == 0;
        const int lsite = fwd ? s : n, lpar = fwd ? par : 1 - par;
        load_site<float, RC, float>(q.gauge + (int64_t)(2 * mu + lpar) * vh * RC, vh, lsite, lv);
      }
    };
    auto compute = [&](__bf16 *Bb, const uint4 (&raw)[KC][3], const float (&lv)[RC], int p)
                       __attribute__((always_inline)) {
      __bf16 *dst = Bb + sl * kFwRow + 8 * un;
      // (the matrix-core form keeps every lane in its products: a lane of a
      // site beyond Vh multiplies zeros and stores zeros)
      if (TRANS != 2 && !valid) {
        const bf16x8_t zero = {};
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            *reinterpret_cast<bf16x8_t *>(dst + c * kFwSites * kFwRow + 8 * TPS * k) = zero;
        return;
      }
      // word 3 sp + col of a channel: the (re, im) BF16 pair of spin sp, colour col
      uint32_t w[KC][12];
#pragma unroll
      for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[k][4 * c + 0] = valid ? raw[k][c].x : 0u;
          w[k][4 * c + 1] = valid ? raw[k][c].y : 0u;
          w[k][4 * c + 2] = valid ? raw[k][c].z : 0u;
          w[k][4 * c + 3] = valid ? raw[k][c].w : 0u;
        }
      if (p != 0) {
        const bool fwd = ((p - 1) & 1) == 0;
        const float ph = nbL[sl][p - 1] < 0 ? -1.f : 1.f;
        const Link<float> U0 = unpack_link<RC, float>(lv);
        if constexpr (TRANS == 2) {
          // matrix cores: lanes 4b .. 4b+3 are one site (8 lanes per site), so
          // a 4x4x4 block is one site's link times 4 of its (channel, spin)
          // vectors; a vector's 3 words are its own B operand (K = c0 re, c0 im,
          // c1 re, c1 im | c2 re, c2 im, 0, 0) and its D column is U v in FP32
          Link<float> U;  // U, or U^+ for a backward hop, times the boundary sign
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const cpx<float> e = fwd ? U0.m[a][b] : conj(U0.m[b][a]);
              U.m[a][b] = ph * e;
            }
          mf_s4 A4[2][2];
          mf_link_rows<bf16, false>(U, lane & 3, A4);
          const mf_f4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
              const mf_s4 b0 = __builtin_bit_cast(mf_s4, u32x2_t{w[k][3 * sp], w[k][3 * sp + 1]});
              const mf_s4 b1 = __builtin_bit_cast(mf_s4, u32x2_t{w[k][3 * sp + 2], 0u});
              mf_f4 d0 = Mf4<bf16>::mma(A4[0][0], b0, zero4);
              d0 = Mf4<bf16>::mma(A4[0][1], b1, d0);
              mf_f4 d1 = Mf4<bf16>::mma(A4[1][0], b0, zero4);
              d1 = Mf4<bf16>::mma(A4[1][1], b1, d1);
              w[k][3 * sp + 0] = __builtin_bit_cast(uint32_t, pack_bf16x2(d0[0], d0[1]));
              w[k][3 * sp + 1] = __builtin_bit_cast(uint32_t, pack_bf16x2(d0[2], d0[3]));
              w[k][3 * sp + 2] = __builtin_bit_cast(uint32_t, pack_bf16x2(d1[0], d1[1]));
            }
        } else {
          // the applied matrix (U, or U^+ for a backward hop, times the boundary
          // sign) as BF16 pairs: re(u v) = dot((Ur, -Ui), (vr, vi)),
          // im(u v) = dot((Ui, Ur), (vr, vi)), products exact, FP32 sums
          bf16x2_t Pr[3][3], Pi[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const cpx<float> e = fwd ? U0.m[a][b] : conj(U0.m[b][a]);
              Pr[a][b] = pack_bf16x2(ph * e.re, -ph * e.im);
              Pi[a][b] = pack_bf16x2(ph * e.im, ph * e.re);
            }
#pragma unroll
          for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
              bf16x2_t v[3];
#pragma unroll
              for (int b = 0; b < 3; ++b) v[b] = __builtin_bit_cast(bf16x2_t, w[k][3 * sp + b]);
              uint32_t o[3];
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                  re = __builtin_amdgcn_fdot2_f32_bf16(Pr[a][b], v[b], re, false);
                  im = __builtin_amdgcn_fdot2_f32_bf16(Pi[a][b], v[b], im, false);
                }
                o[a] = __builtin_bit_cast(uint32_t, pack_bf16x2(re, im));
              }
#pragma unroll
              for (int a = 0; a < 3; ++a) w[k][3 * sp + a] = o[a];
            }
        }
      }
      // colour c: the four spins' (re, im) words
#pragma unroll
      for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          *reinterpret_cast<uint4 *>(dst + c * kFwSites * kFwRow + 8 * TPS * k) =
              make_uint4(w[k][c], w[k][3 + c], w[k][6 + c], w[k][9 + c]);
    };
    // per path: transport into LDS, issue the next path's loads, then the
    // matrix products (their latency overlaps the products)
    constexpr int kSplitN = (NT + NWC - 1) / NWC;  // n-tiles per wave when one m-tile is split over all waves
    const int form = (nm == JM && nn == NT) ? 2 : (nm == 1 && nn == kSplitN) ? 1 : (nn > 0 ? 0 : -1);
    auto products = [&](auto &ac, const __bf16 *Bb, int p) {
      if (form == 2)
        mma_static(std::integral_constant<int, JM>(), std::integral_constant<int, NT>(), ac, Bb, 16 * p);
      else if (form == 1)
        mma_static(std::integral_constant<int, 1>(), std::integral_constant<int, kSplitN>(), ac, Bb, 16 * p);
      else if (form == 0)
        mma_chunk(ac, Bb, 16 * p, 16);
    };
    if constexpr (SPLIT) {
      // iteration i: the transporting waves fill buffer i % 2 with path i while
      // the others multiply path i - 1 from buffer (i - 1) % 2; the barrier
      // ending iteration i publishes path i and frees buffer (i - 1) % 2. The
      // accumulators live in the multiplying waves' branch only (they are not
      // held while transporting), which also stages the output tile.
      if (producer) {
        issue(rawA, lvA, 0);
#pragma unroll 1
        for (int i = 0; i < 10; ++i) {
          if (i < 9) {
            compute(Bt + (i & 1) * kBuf, rawA, lvA, i);
            if (i + 1 < 9) issue(rawA, lvA, i + 1);
          }
          __syncthreads();
        }
      } else {
        f32x4_t cacc[JM][NT];
#pragma unroll
        for (int j = 0; j < JM; ++j)
#pragma unroll
          for (int t = 0; t < NT; ++t) cacc[j][t] = f32x4_t{0, 0, 0, 0};
#pragma unroll 1
        for (int i = 0; i < 10; ++i) {
          if (i > 0) products(cacc, Bt + ((i - 1) & 1) * kBuf, i - 1);
          __syncthreads();
        }
        stage(cacc);
      }
      __syncthreads();
      store_out();
      return;
    } else {
      issue(rawA, lvA, 0);
#pragma unroll 1
      for (int p = 0; p < 9; ++p) {
        __syncthreads();
        compute(Bt, rawA, lvA, p);
        if (p + 1 < 9) issue(rawA, lvA, p + 1);
        __syncthreads();
        products(acc, Bt, p);
      }
    }
  } else {
  // input known to vanish on parity zero_par (the network input lives on even
  // sites): the items reading that parity are zero, and when every hop is
  // zero only the identity items' K steps are multiplied
  const int hop_par = 1 - par;
  const int q_end = zero_par == hop_par ? 4 * ((L.cin + 3) / 4) : 4 * L.fw_ks;
  for (int q0 = 0; q0 < q_end; q0 += L.fw_ipc) {
    const int ipc = min(L.fw_ipc, q_end - q0);
    __syncthreads();
    if (L.cin % 4 == 0) {
      // kNch items (one site and path) per thread: channels un and un + gn of
      // the chunk when it is one path (lanes of a site then read whole cache
      // lines), else kNch consecutive channels
      constexpr int kNch = 2;
      const int gn = ipc / kNch;
      const bool one_path = ipc == L.cin;
#pragma unroll 1
      for (int w = threadIdx.x; w < kFwSites * gn; w += kPtcThreads) {
        const int un = w % gn, sl = w / gn;
        const int u0 = one_path ? un : kNch * un, kstep = one_path ? gn : 1;
        const int qi = q0 + u0, s = s0 + sl;
        __bf16 *dst = Bt + sl * kFwRow + 8 * u0;
        const int pq = qi / L.cin;
        if (s < q.g.Vh && qi < L.fw_items && (pq == 0 ? par : hop_par) != zero_par) {
          const int p = pq, i0 = qi - p * L.cin;
          if (q.recon == 12)
            transportn_lds<12, kNch>(q, nbr, in, L.cin, i0, kstep, p, par, s, dst, kFwSites * kFwRow);
          else
            transportn_lds<18, kNch>(q, nbr, in, L.cin, i0, kstep, p, par, s, dst, kFwSites * kFwRow);
        } else {
          const bf16x8_t zero = {};
#pragma unroll
          for (int k = 0; k < kNch; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              *reinterpret_cast<bf16x8_t *>(dst + c * kFwSites * kFwRow + 8 * k * kstep) = zero;
        }
      }
    } else {
      // one item per thread, sites fastest (narrow activations)
#pragma unroll 1
      for (int w = threadIdx.x; w < kFwSites * ipc; w += kPtcThreads) {
        const int sl = w % kFwSites, u = w / kFwSites;
        const int qi = q0 + u, s = s0 + sl;
        __bf16 *dst = Bt + sl * kFwRow + 8 * u;
        const int pq = qi / L.cin;
        if (s < q.g.Vh && qi < L.fw_items && (pq == 0 ? par : hop_par) != zero_par) {
          const int p = pq, i = qi - p * L.cin;
          if (q.recon == 12)
            transportn_lds<12, 1>(q, nbr, in, L.cin, i, 1, p, par, s, dst, kFwSites * kFwRow);
          else
            transportn_lds<18, 1>(q, nbr, in, L.cin, i, 1, p, par, s, dst, kFwSites * kFwRow);
        } else {
          const bf16x8_t zero = {};
#pragma unroll
          for (int c = 0; c < 3; ++c) *reinterpret_cast<bf16x8_t *>(dst + c * kFwSites * kFwRow) = zero;
        }
      }
    }
    __syncthreads();
    mma_chunk(acc, Bt, q0, ipc);
  }
  }
  __syncthreads();
  stage(acc);
  __syncthreads();
  store_out();
}

// ---------------------------------------------------------------------------
// backward, data: gY[(i,p)](x) = sum_o W[o,i,p]^+ delta_o(x), on parity par.
// Output channel-interleaved with Cin*9 channels.

__global__ void __launch_bounds__(kPtcThreads) ptc_bwd_data_kernel(PtcGeo q, PtcLayerDev L, const float *delta,
                                                                    float *gy, int par) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int krow = L.kadj + kLdsPad;
  __bf16 *Bt = reinterpret_cast<__bf16 *>(smem);  // [48][krow]: delta, k = 2*(o*4+s) + r
  const int s0 = xcd_remap(blockIdx.x, gridDim.x) * kTile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < 48 * krow; e += kPtcThreads) Bt[e] = (__bf16)0.f;
  __syncthreads();
  const int64_t vsd = (int64_t)q.g.Vh * L.cout;
  const float *dblk = delta + (int64_t)par * vsd * 24;
  for (int it = threadIdx.x; it < kTile * L.cout; it += kPtcThreads) {
    const int sl = it / L.cout, o = it % L.cout;
    const int s = s0 + sl;
    float r[24];
    if (s < q.g.Vh)
      load_spinor_reals<float, 24, float>(dblk, vsd, (int64_t)s * L.cout + o, r);
    else
      for (int k = 0; k < 24; ++k) r[k] = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bf16x8_t v;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        v[2 * sp] = (__bf16)r[6 * sp + 2 * c];
        v[2 * sp + 1] = (__bf16)r[6 * sp + 2 * c + 1];
      }
      *reinterpret_cast<bf16x8_t *>(Bt + (c * kTile + sl) * krow + 8 * o) = v;
    }
  }
  __syncthreads();
  const int C9 = L.cin * 9;
  const int64_t vsg = (int64_t)q.g.Vh * C9;
  float *gblk = gy + (int64_t)par * vsg * 24;
  const int ks_n = L.kadj / 32;
  const int ntile_total = L.madj_tiles * 3;
  for (int tid = wave; tid < ntile_total; tid += 4) {
    const int mt = tid / 3, nt = tid % 3;
    f32x4_t acc = {0, 0, 0, 0};
    for (int ks = 0; ks < ks_n; ++ks) {
      const bf16x8_t a = ((const bf16x8_t *)L.Aadj)[((size_t)mt * ks_n + ks) * 64 + lane];
      const bf16x8_t b = lds_frag(Bt + (nt * kTile + (lane & 15)) * krow + ks * 32 + 8 * (lane >> 4));
      acc = mfma_bf16(a, b, acc);
    }
    const int sl = lane & 15, s = s0 + sl;
    if (s >= q.g.Vh) continue;
    // rows 4*(lane>>4)+j: two complex entries (k', k'+1) of the same (i,p) group
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
      const int m = mt * 16 + 4 * (lane >> 4) + j;
      const int kp = m >> 1;  // (i*9 + p)*4 + s'
      const int ip = kp >> 2, sp = kp & 3;
      if (ip < C9) {
        float *dst = gblk + ((int64_t)(sp * 6 + nt * 2) / 4 * vsg + (int64_t)s * C9 + ip) * 4 + ((sp * 6 + nt * 2) & 3);
        dst[0] = acc[j];
        dst[1] = acc[j + 1];
      }
    }
  }
}

// gpsi_i(x) = sum_p (T_p^+ gY[i,p])(x); T_{+mu}^+ = T_{-mu}. One thread per
// (site, channel) of parity par.
__global__ void __launch_bounds__(256) ptc_adjoint_gather_kernel(PtcGeo q, int cin, const float *gy, float *gpsi,
                                                                  int par) {
  const int pidx = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (pidx >= q.g.Vh * cin) return;
  const int s = pidx / cin, i = pidx - s * cin;
  const Site x = decode_site(q.g, s, par);
  const int C9 = cin * 9;
  const int64_t vh = q.g.Vh, vsg = vh * C9;
  const float *same = gy + (int64_t)par * vsg * 24;
  const float *other = gy + (int64_t)(1 - par) * vsg * 24;
  float acc[24], r[24];
  load_spinor_reals<float, 24, float>(same, vsg, (int64_t)s * C9 + i * 9 + 0, acc);
  for (int mu = 0; mu < 4; ++mu) {
    for (int f = 0; f < 2; ++f) {
      // f = 0: term T_{-mu} gY[i,+mu] = U_mu(x-mu)^+ g(x-mu); f = 1: T_{+mu} gY[i,-mu] = U_mu(x) g(x+mu)
      const int p = f == 0 ? 1 + 2 * mu : 2 + 2 * mu;
      int w = 0, n = 0;
      const int step = f == 0 ? -1 : 1;
      switch (mu) {
        case 0: n = hop<0>(q.g, x, step, &w); break;
        case 1: n = hop<1>(q.g, x, step, &w); break;
        case 2: n = hop<2>(q.g, x, step, &w); break;
        default: n = hop<3>(q.g, x, step, &w); break;
      }
      load_spinor_reals<float, 24, float>(other, vsg, (int64_t)n * C9 + i * 9 + p, r);
      float lv[18];
      Link<float> U;
      if (q.recon == 12) {
        if (f == 0)
          load_site<float, 12, float>(q.gauge + (int64_t)(2 * mu + 1 - par) * vh * 12, vh, n, lv);
        else
          load_site<float, 12, float>(q.gauge + (int64_t)(2 * mu + par) * vh * 12, vh, s, lv);
        U = unpack_link<12, float>(lv);
      } else {
        if (f == 0)
          load_site<float, 18, float>(q.gauge + (int64_t)(2 * mu + 1 - par) * vh * 18, vh, n, lv);
        else
          load_site<float, 18, float>(q.gauge + (int64_t)(2 * mu + par) * vh * 18, vh, s, lv);
        U = unpack_link<18, float>(lv);
      }
      const float ph = (mu == 3 && (w & 1) && q.g.bc_t < 0) ? -1.f : 1.f;
      for (int sp = 0; sp < 4; ++sp) {
        cpx<float> v[3], u[3];
        for (int c = 0; c < 3; ++c) v[c] = mk<float>(r[6 * sp + 2 * c], r[6 * sp + 2 * c + 1]);
        if (f == 0)
          su3_adj_mv(U, v, u);
        else
          su3_mv(U, v, u);
        for (int c = 0; c < 3; ++c) {
          acc[6 * sp + 2 * c] += ph * u[c].re;
          acc[6 * sp + 2 * c + 1] += ph * u[c].im;
        }
      }
    }
  }
  store_spinor_reals<float, 24, float>(gpsi + (int64_t)par * vh * cin * 24, vh * cin, pidx, acc);
}

// ---------------------------------------------------------------------------
// backward, weights: partial sums over site tiles of
//   G[(m', r)][k'] = sum_{(n, r')} D[(m', r)][(n, r')] Y'[(n, r')][k'],
//   D = [[dr, di],[di, -dr]],  Y' = (Yr, Yi),
// i.e. G = (Re, Im) of sum_x delta (T psi)^+. A workgroup owns one input
// channel chunk and a strided set of site tiles of parity par.

__global__ void __launch_bounds__(kPtcThreads) ptc_bwd_weight_kernel(PtcGeo q, PtcLayerDev L, const bf16 *in,
                                                                      const float *delta, float *partial, int par,
                                                                      int groups) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int KROW = 2 * 48 + kLdsPad;  // k = 2*n + r', n = colour*16 + site
  __bf16 *At = reinterpret_cast<__bf16 *>(smem);             // [Mpad][KROW]  (delta embedding)
  const int mrows = L.mw_tiles * 16;
  __bf16 *Bt = At + mrows * KROW;                             // [chunk_ch*36][KROW]  (Y' transposed)
  const int ck = blockIdx.y;
  const int grp = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ncol = L.chunk_ch * 36;        // k' in this chunk
  const int ntiles_n = (ncol + 15) / 16;
  const int ntile_total = L.mw_tiles * ntiles_n;
  f32x4_t acc[24];
#pragma unroll
  for (int t = 0; t < 24; ++t) acc[t] = f32x4_t{0, 0, 0, 0};
  const int ntile_sites = (q.g.Vh + kTile - 1) / kTile;
  const int64_t vsd = (int64_t)q.g.Vh * L.cout;
  const float *dblk = delta + (int64_t)par * vsd * 24;
  for (int tile = grp; tile < ntile_sites; tile += groups) {
    const int s0 = tile * kTile;
    __syncthreads();
    for (int e = threadIdx.x; e < (mrows + ntiles_n * 16) * KROW; e += kPtcThreads) At[e] = (__bf16)0.f;
    __syncthreads();
    // delta -> A: row 2*(o*4+s)+r, col 2*(c*16+sl)+r'
    for (int it = threadIdx.x; it < kTile * L.cout; it += kPtcThreads) {
      const int sl = it / L.cout, o = it % L.cout;
      const int s = s0 + sl;
      if (s >= q.g.Vh) continue;
      float r[24];
      load_spinor_reals<float, 24, float>(dblk, vsd, (int64_t)s * L.cout + o, r);
      for (int sp = 0; sp < 4; ++sp)
        for (int c = 0; c < 3; ++c) {
          const float dr = r[6 * sp + 2 * c], di = r[6 * sp + 2 * c + 1];
          const int row = 2 * (o * 4 + sp), col = 2 * (c * kTile + sl);
          At[row * KROW + col] = (__bf16)dr;
          At[row * KROW + col + 1] = (__bf16)di;
          At[(row + 1) * KROW + col] = (__bf16)di;
          At[(row + 1) * KROW + col + 1] = (__bf16)(-dr);
        }
    }
    // Y' -> B (stored [k'][k]): transported inputs of this channel chunk
    const int nitem = kTile * L.chunk_ch * 9;
    for (int it = threadIdx.x; it < nitem; it += kPtcThreads) {
      const int sl = it % kTile, rem = it / kTile, p = rem % 9, il = rem / 9;
      const int i = ck * L.chunk_ch + il;
      const int s = s0 + sl;
      if (s >= q.g.Vh || i >= L.cin) continue;
      const Site x = decode_site(q.g, s, par);
      cpx<float> y[4][3];
      transport_any(q, in, L.cin, i, p, x, s, y);
      for (int sp = 0; sp < 4; ++sp) {
        const int kp = (il * 9 + p) * 4 + sp;
        for (int c = 0; c < 3; ++c) {
          const int col = 2 * (c * kTile + sl);
          Bt[kp * KROW + col] = (__bf16)y[sp][c].re;
          Bt[kp * KROW + col + 1] = (__bf16)y[sp][c].im;
        }
      }
    }
    __syncthreads();
    for (int ks = 0; ks < 3; ++ks) {
#pragma unroll
      for (int t = 0; t < 24; ++t) {
        const int tid = wave + 4 * t;
        if (tid < ntile_total) {
          const int mt = tid / ntiles_n, nt = tid % ntiles_n;
          const bf16x8_t a = lds_frag(At + (mt * 16 + (lane & 15)) * KROW + ks * 32 + 8 * (lane >> 4));
          const bf16x8_t b = lds_frag(Bt + (nt * 16 + (lane & 15)) * KROW + ks * 32 + 8 * (lane >> 4));
          acc[t] = mfma_bf16(a, b, acc[t]);
        }
      }
    }
  }
  // partial[ck][grp][row][col]
  float *dst = partial + ((size_t)ck * groups + grp) * (size_t)mrows * (ntiles_n * 16);
#pragma unroll
  for (int t = 0; t < 24; ++t) {
    const int tid = wave + 4 * t;
    if (tid < ntile_total) {
      const int mt = tid / ntiles_n, nt = tid % ntiles_n;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = mt * 16 + 4 * (lane >> 4) + j, col = nt * 16 + (lane & 15);
        dst[(size_t)row * (ntiles_n * 16) + col] = acc[t][j];
      }
    }
  }
}

// gW[o][i][p][s][s'] (complex, FP32) += sum over groups of the partials, in a
// fixed order (deterministic).
__global__ void ptc_weight_reduce_kernel(PtcLayerDev L, const float *partial, int groups, float *gw, int accumulate) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // complex entry index
  const int total = L.cout * L.cin * 9 * 16;
  if (idx >= total) return;
  const int sp2 = idx % 4, sp = (idx / 4) % 4, p = (idx / 16) % 9, i = (idx / 144) % L.cin, o = idx / (144 * L.cin);
  const int ck = i / L.chunk_ch, il = i - ck * L.chunk_ch;
  const int ncol = L.chunk_ch * 36, ldc = ((ncol + 15) / 16) * 16;
  const int mrows = L.mw_tiles * 16;
  const int col = (il * 9 + p) * 4 + sp2;
  const int row = 2 * (o * 4 + sp);
  double re = 0, im = 0;
  for (int g = 0; g < groups; ++g) {
    const float *base = partial + ((size_t)ck * groups + g) * (size_t)mrows * ldc;
    re += base[(size_t)row * ldc + col];
    im += base[(size_t)(row + 1) * ldc + col];
  }
  if (accumulate) {
    gw[2 * idx] += (float)re;
    gw[2 * idx + 1] += (float)im;
  } else {
    gw[2 * idx] = (float)re;
    gw[2 * idx + 1] = (float)im;
  }
}

// ---------------------------------------------------------------------------
// weight packing: master FP32 complex W[o][i][p][s][s'] -> MFMA A fragments.

__device__ __forceinline__ float wval(const float *W, int cin, int o, int i, int p, int s, int s2, int im) {
  return W[2 * ((((o * cin + i) * 9 + p) * 4 + s) * 4 + s2) + im];
}

// forward A: row m = 2*(o*4+s) + r, col k = 2*(q*4+s') + r' with q = p*Cin + i.
__global__ void ptc_pack_forward_kernel(PtcLayerDev L, const float *W, bf16x8_t *A) {
  const int total = L.mtiles * L.fw_ks * 64;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = idx % 64, ks = (idx / 64) % L.fw_ks, mt = idx / (64 * L.fw_ks);
  const int m = mt * 16 + (lane & 15);
  const int mp = m >> 1, r = m & 1, o = mp >> 2, s = mp & 3;
  bf16x8_t v;
  for (int j = 0; j < 8; ++j) {
    const int k = ks * 32 + 8 * (lane >> 4) + j;
    const int kp = k >> 1, r2 = k & 1;
    const int qi = kp >> 2, s2 = kp & 3;
    const int p = qi / L.cin, i = qi % L.cin;
    float val = 0.f;
    if (o < L.cout && qi < L.fw_items) {
      const float wr = wval(W, L.cin, o, i, p, s, s2, 0), wi = wval(W, L.cin, o, i, p, s, s2, 1);
      val = (r == 0) ? (r2 == 0 ? wr : -wi) : (r2 == 0 ? wi : wr);
    }
    v[j] = (__bf16)val;
  }
  A[idx] = v;
}

// adjoint A: row m = 2*((i*9+p)*4+s') + r, col k = 2*(o*4+s) + r'; conj(W)^T embedded.
__global__ void ptc_pack_adjoint_kernel(PtcLayerDev L, const float *W, bf16x8_t *A) {
  const int ks_n = L.kadj / 32;
  const int total = L.madj_tiles * ks_n * 64;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = idx % 64, ks = (idx / 64) % ks_n, mt = idx / (64 * ks_n);
  const int m = mt * 16 + (lane & 15);
  const int kp = m >> 1, r = m & 1;
  const int i = kp / 36, p = (kp / 4) % 9, s2 = kp & 3;
  bf16x8_t v;
  for (int j = 0; j < 8; ++j) {
    const int k = ks * 32 + 8 * (lane >> 4) + j;
    const int mp = k >> 1, r2 = k & 1, o = mp >> 2, s = mp & 3;
    float val = 0.f;
    if (i < L.cin && o < L.cout) {
      const float wr = wval(W, L.cin, o, i, p, s, s2, 0), wi = wval(W, L.cin, o, i, p, s, s2, 1);
      // conj(W)^T: [[Wr, Wi], [-Wi, Wr]]
      val = (r == 0) ? (r2 == 0 ? wr : wi) : (r2 == 0 ? -wi : wr);
    }
    v[j] = (__bf16)val;
  }
  A[idx] = v;
}

// ---------------------------------------------------------------------------
// host launchers

size_t ptc_bwd_data_lds(const PtcLayerDev &L) { return 48 * (L.kadj + kLdsPad) * 2; }
size_t ptc_bwd_weight_lds(const PtcLayerDev &L) {
  const int ncol = L.chunk_ch * 36, ntn = (ncol + 15) / 16;
  return (size_t)(L.mw_tiles * 16 + ntn * 16) * (2 * 48 + kLdsPad) * 2;
}

hipError_t launch_ptc_nbr(const Geom &g, int *tab, hipStream_t st) {
  if (g.Vh == 0) return hipSuccess;
  hipLaunchKernelGGL(ptc_nbr_kernel, dim3((g.Vh + 255) / 256, 2), dim3(256), 0, st, g, tab);
  return hipGetLastError();
}

hipError_t launch_ptc_forward(const PtcGeo &q, const PtcLayerDev &L, const int *nbr, const void *in, void *out,
                              int out_f32, int par, int variant, int zero_par, hipStream_t st) {
  // LDS staging of the output tile: BF16 up to 16 channels; FP32 one channel
  if (out_f32 && L.cout != 1) return hipErrorInvalidValue;
  if (par < -1 || par > 1) return hipErrorInvalidValue;
  const int npar = par < 0 ? 2 : 1;  // par -1: both parities in one launch
  switch (variant) {
#define PTC_FWD_RC(NS, WPE, PIPE, NTH, RC)                                                                   \
  hipLaunchKernelGGL((ptc_forward_kernel<NS, WPE, PIPE, NTH, RC>), dim3(npar * ((q.g.Vh + NS - 1) / NS)),         \
                     dim3(NTH), 0, st, q, L, nbr, (const bf16 *)in, out, out_f32, par, zero_par)
#define PTC_FWD(NS, WPE, PIPE, NTH)              \
  if constexpr (PIPE == 0) {                     \
    PTC_FWD_RC(NS, WPE, PIPE, NTH, 18);          \
  } else if (q.recon == 18) {                    \
    PTC_FWD_RC(NS, WPE, PIPE, NTH, 18);          \
  } else {                                       \
    PTC_FWD_RC(NS, WPE, PIPE, NTH, 12);          \
  }                                              \
  break;
    case 642: PTC_FWD(64, 2, 0, 256)
    case 322: PTC_FWD(32, 2, 0, 256)
    // the pipelined 16-channel path: 256 threads (8 per site) at 2 or 3 waves
    // per SIMD, or 512 threads (16 per site) at 3 or 4; colour products on
    // dot2 (..1) or on the matrix cores (..2). It reads every path, so no
    // input parity may be known zero.
    case 3221: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 2, 1, 256)
    case 3231: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 3, 1, 256)
    case 3222: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 2, 2, 256)
    case 3232: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 3, 2, 256)
    case 5031: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 3, 1, 512)
    case 5041: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 4, 1, 512)
    case 5032: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 3, 2, 512)
    case 5042: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 4, 2, 512)
    // split forms (512 threads: 4 waves transport, 4 multiply), at 3 or 4 waves per SIMD
    case 5033: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 3, 3, 512)
    case 5043: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 4, 3, 512)
    case 5034: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 3, 4, 512)
    case 5044: if (L.cin != 16 || zero_par >= 0) return hipErrorInvalidValue; PTC_FWD(32, 4, 4, 512)
    default: return hipErrorInvalidValue;
#undef PTC_FWD
#undef PTC_FWD_RC
  }
  return hipGetLastError();
}

// Layer-0 input: the even field (FP32 packed spinor) as BF16 activations
// with one channel, zero on odd sites.
__global__ void ptc_input_kernel(int64_t vh, const float *in_even, bf16 *act) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= vh) return;
  float r[24];
  load_spinor_reals<float, 24, float>(in_even, vh, s, r);
  store_chunks<bf16, 24, 8, float>(act, vh, s, r);
  float z[24] = {};
  store_chunks<bf16, 24, 8, float>(act + vh * 24, vh, s, z);
}

hipError_t launch_ptc_input(int64_t vh, const void *in_even, void *act, hipStream_t st) {
  if (vh == 0) return hipSuccess;
  hipLaunchKernelGGL(ptc_input_kernel, dim3((unsigned)((vh + 255) / 256)), dim3(256), 0, st, vh, (const float *)in_even,
                     (bf16 *)act);
  return hipGetLastError();
}

hipError_t launch_ptc_bwd_data(const PtcGeo &q, const PtcLayerDev &L, const float *delta, float *gy, int par,
                               hipStream_t st) {
  const int nt = (q.g.Vh + kTile - 1) / kTile;
  hipLaunchKernelGGL(ptc_bwd_data_kernel, dim3(nt), dim3(kPtcThreads), ptc_bwd_data_lds(L), st, q, L, delta, gy, par);
  return hipGetLastError();
}

hipError_t launch_ptc_adjoint_gather(const PtcGeo &q, int cin, const float *gy, float *gpsi, int par,
                                     hipStream_t st) {
  const int n = q.g.Vh * cin, bt = 256;
  hipLaunchKernelGGL(ptc_adjoint_gather_kernel, dim3((n + bt - 1) / bt), dim3(bt), 0, st, q, cin, gy, gpsi, par);
  return hipGetLastError();
}

hipError_t launch_ptc_bwd_weight(const PtcGeo &q, const PtcLayerDev &L, const void *in, const float *delta,
                                 float *partial, int par, int groups, hipStream_t st) {
  hipLaunchKernelGGL(ptc_bwd_weight_kernel, dim3(groups, L.nchunk), dim3(kPtcThreads), ptc_bwd_weight_lds(L), st, q,
                     L, (const bf16 *)in, delta, partial, par, groups);
  return hipGetLastError();
}

hipError_t launch_ptc_weight_reduce(const PtcLayerDev &L, const float *partial, int groups, float *gw, int accumulate,
                                    hipStream_t st) {
  const int total = L.cout * L.cin * 9 * 16, bt = 256;
  hipLaunchKernelGGL(ptc_weight_reduce_kernel, dim3((total + bt - 1) / bt), dim3(bt), 0, st, L, partial, groups, gw,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_ptc_pack(const PtcLayerDev &L, const float *W, hipStream_t st) {
  const int bt = 256;
  const int nf = L.mtiles * L.fw_ks * 64;
  hipLaunchKernelGGL(ptc_pack_forward_kernel, dim3((nf + bt - 1) / bt), dim3(bt), 0, st, L, W, (bf16x8_t *)L.A);
  const int na = L.madj_tiles * (L.kadj / 32) * 64;
  hipLaunchKernelGGL(ptc_pack_adjoint_kernel, dim3((na + bt - 1) / bt), dim3(bt), 0, st, L, W, (bf16x8_t *)L.Aadj);
  return hipGetLastError();
}

__global__ void adam_kernel(float *w, float *m, float *v, const float *g, size_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2, float gscale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = gscale * g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, size_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, float gscale, hipStream_t st) {
  const int bt = 256;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + bt - 1) / bt)), dim3(bt), 0, st, w, m, v, g, n, lr, b1, b2, eps,
                     bc1, bc2, gscale);
  return hipGetLastError();
}

}  // namespace lqcd
