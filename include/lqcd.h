/*
 * lqcd.h - C ABI of the MI355X (gfx950) lattice-QCD linear-solver library.
 *
 * The library applies the even-odd preconditioned Wilson-clover operator of
 * eq. (2) and the improved-staggered operator of eq. (3) of Babich et al.,
 * "Scaling Lattice QCD beyond 100 GPUs" (SC11), and solves M x = b (eq. (1))
 * with the mixed-precision, Schwarz-preconditioned GCR of Algorithm 1
 * (Section VIII-A) or with CG (Section III-A), on one GPU.
 *
 * Conventions (fixed here because the paper leaves them open):
 *   - lattice dims (Lx, Ly, Lz, Lt), all even; site parity (x+y+z+t) mod 2,
 *     0 = even; every direction periodic, and a hop that crosses the t
 *     boundary is multiplied by bc_t (+1 periodic, -1 antiperiodic);
 *   - chiral gamma basis gamma_k = [[0,-i s_k],[i s_k,0]] (k = x,y,z),
 *     gamma_t = [[0,1],[1,0]]; spin factors of eq. (2) read as (1 -/+ gamma_mu);
 *   - Wilson-clover in kappa normalisation: M = A - kappa D, with
 *     A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu (clover leaves,
 *     F = (Q_munu - Q_numu)/8); this is 2 kappa times the matrix of eq. (2);
 *   - even-odd Schur complement on even sites (Section III-A):
 *     Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe;
 *   - improved staggered: M = m - D/2 with Kogut-Susskind phases, backward
 *     hops with a minus sign (D is anti-Hermitian), long link weight c_long;
 *     the even normal operator N_e = m^2 - D_eo D_oe / 4.
 *
 * Memory. Every field pointer is DEVICE memory owned by the caller; the
 * library neither frees nor retains caller pointers after a call returns.
 * Packed fields use the library's layout; their sizes come from
 * lqcd_field_bytes and must be 16-byte aligned. "Natural" fields are the
 * exchange format: complex double (re, im interleaved), site index
 * i = x + Lx*(y + Ly*(z + Lz*t)), gauge [i][mu][row][col], Wilson spinor
 * [i][spin][colour], staggered spinor [i][colour].
 * The context owns all scratch memory (allocated on first use, freed by
 * lqcd_context_destroy).
 *
 * Streams. Work is enqueued on the given HIP stream (0 = null stream).
 * Operator and import/export calls return once the work is enqueued.
 * Solver calls block the host (they read reduction results).
 *
 * Errors. Every call returns lqcd_status. Arguments are validated before any
 * launch and nothing is written when validation fails. LQCD_ERR_DEVICE wraps
 * HIP failures; lqcd_last_error() returns the text of the most recent error
 * of the context (or of the library, for calls without a context).
 *
 * Environment. LQCD_TUNE=0 disables the autotuner's timing (fixed fallback
 * launch parameters); LQCD_TUNE_CACHE=<file> keeps its choices across
 * processes; LQCD_MRHS_MFMA=1 selects the matrix-core form of the multi-source
 * link products; LQCD_PTC_VARIANT=<form> forces the form of the network's
 * 16-input-channel layers (for testing every form); LQCD_VERBOSE prints the
 * solvers' residual history to stderr. The tuned launch parameters of the
 * stencil and batch kernels never change a result; the network's forms differ
 * in the order of their FP32 sums (dot2 or matrix-core colour products), so
 * the form timed fastest can change its output by BF16 roundings (fix it with
 * LQCD_PTC_VARIANT or a tuning cache for bit-reproducible runs).
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lqcd_context lqcd_context;
typedef void *lqcd_stream; /* a hipStream_t */

typedef enum {
  LQCD_OK = 0,
  LQCD_ERR_INVALID_ARG = 1,
  LQCD_ERR_UNSUPPORTED = 2,
  LQCD_ERR_OUT_OF_MEMORY = 3,
  LQCD_ERR_DEVICE = 4,
  LQCD_ERR_NOT_CONVERGED = 5,
  LQCD_ERR_BREAKDOWN = 6
} lqcd_status;

/*
 * Storage precisions. Arithmetic is FP64 for LQCD_F64 and FP32 otherwise,
 * except that the Wilson hops of LQCD_F16 operators (12 or 18 link reals)
 * form the spin projection in packed FP16 (one rounding of each half-spinor
 * component) and the colour products as FP16 x FP16 products with FP32 sums.
 * LQCD_HALF is 16-bit fixed point (the paper's "half" format, Section V):
 * integer codes q in [-32767, 32767] standing for q / 32767; link entries are
 * stored so directly (recon 18 or 12), while spinors and the clover term
 * carry one FP32 norm per site (its largest magnitude; codes hold value /
 * norm), stored after the codes of each parity block (lqcd_field_bytes counts
 * them). HALF operators are Wilson-clover; they serve the Schwarz
 * preconditioner and sloppy CG iterations.
 */
typedef enum { LQCD_F64 = 0, LQCD_F32 = 1, LQCD_F16 = 2, LQCD_BF16 = 3, LQCD_HALF = 4 } lqcd_precision;

typedef enum { LQCD_WILSON_CLOVER = 0, LQCD_STAGGERED = 1 } lqcd_action;

typedef enum {
  LQCD_FIELD_SPINOR = 0,      /* one parity of a colour-spinor field (Vh sites) */
  LQCD_FIELD_SPINOR_FULL = 1, /* both parities: [parity 0 block][parity 1 block] */
  LQCD_FIELD_GAUGE = 2,       /* Wilson links or staggered fat links, 4 directions x 2 parities */
  LQCD_FIELD_LONG = 3,        /* staggered long links */
  LQCD_FIELD_CLOVER = 4       /* clover A (or A^-1), both parities, 72 reals per site */
} lqcd_field_kind;

/*
 * One operator instance: the action, geometry, precision and storage of its
 * fields. The same physical operator is usually described by several
 * instances of different precision (FP64 for restarts, FP32 Krylov, FP16/BF16
 * preconditioner); each owns its own packed copies of the links and clover.
 *
 * tile: the site-ordering tile of every packed field of this operator. Sites
 * of one parity are stored tile by tile (tiles in lexicographic order, sites
 * lexicographic inside a tile), so a tile's sites are contiguous. Each entry
 * must be even and divide dims. tile = dims gives plain lexicographic
 * even-odd order. The Schwarz blocks of lqcd_schwarz_precond must equal the
 * tile.
 */
typedef struct {
  int32_t action;       /* lqcd_action */
  int32_t dims[4];      /* Lx, Ly, Lz, Lt: all even, >= 2 */
  int32_t tile[4];      /* layout tile (see above) */
  int32_t bc_t;         /* +1 or -1 */
  int32_t prec;         /* lqcd_precision of every packed field of this instance */
  int32_t recon;        /* 18, 12 or 8 reals per stored SU(3) link (Wilson U, staggered long) */
  double kappa, csw;    /* Wilson-clover */
  double mass, c_long;  /* staggered */
  const void *gauge;      /* packed LQCD_FIELD_GAUGE (staggered fat links are always 18 reals) */
  const void *long_links; /* packed LQCD_FIELD_LONG (staggered only) */
  const void *clover;     /* packed A, both parities (Wilson-clover only) */
  const void *clover_inv; /* packed A^-1, both parities (Wilson-clover only) */
} lqcd_operator;

typedef struct {
  int32_t iters;             /* Krylov steps (GCR) or CG iterations */
  int32_t restarts;          /* high-precision restarts / reliable updates */
  int32_t matvecs;           /* operator applications in the Krylov precision */
  int32_t precond_applies;   /* applications of K */
  int32_t fallback_applies;  /* of those, Schwarz steps taken in place of the learned K */
  int32_t history_len;       /* entries written to the params' res_history (0 without one) */
  double true_residual;      /* ||b - M x|| / ||b||, recomputed in FP64 at the end */
  double seconds;            /* wall time of the call */
} lqcd_solve_info;

typedef enum { LQCD_PRECOND_NONE = 0, LQCD_PRECOND_SCHWARZ = 1, LQCD_PRECOND_LEARNED = 2 } lqcd_precond_kind;

/*
 * Parallel-transport convolution network (the learned preconditioner; the
 * paper has none: it only requires the outer solver to be flexible,
 * Section III-B). Layer l maps channels[l] -> channels[l+1] colour-spinor
 * fields: psi'_o(x) = sum_i sum_p W[o,i,p] (T_p psi_i)(x) over 9 paths
 * (identity and the 8 one-hop parallel transports), W[o,i,p] a complex 4x4
 * spin matrix; the network is linear, channels[0] = channels[nlayers] = 1.
 * Master weights: FP32 complex (re, im), [layer][o][i][p][s][s'];
 * lqcd_ptc_pack converts them to the BF16 matrix-core layout.
 */
typedef struct {
  int32_t nlayers;      /* 1..8 */
  int32_t channels[9];  /* 1..4 or multiples of 4 up to 16 */
} lqcd_ptc_shape;

typedef struct {
  lqcd_ptc_shape shape;
  const void *packed;   /* device, lqcd_ptc_sizes(...)->packed_bytes */
} lqcd_ptc_net;

typedef struct {
  int32_t block[4]; /* Dirichlet block; must equal the tile of op_precond */
  int32_t mr_steps; /* MR steps per block and visit (the paper uses 10) */
  int32_t cycles;   /* 0: additive (the paper's); n >= 1: multiplicative, n sweeps over the two block colours */
  double omega;     /* MR over-relaxation, 0 < omega < 2: x += omega a r, r -= omega a q; 0 is read as 1,
                       the plain MR of Section VIII-A (the paper gives no relaxation factor) */
} lqcd_schwarz_params;

typedef struct {
  double tol;        /* stop when ||b - M x|| <= tol ||b|| (FP64) */
  int32_t k_max;     /* Krylov space size before a restart */
  double delta;      /* early restart when ||rhat|| / ||r0|| < delta */
  int32_t max_iter;  /* total Krylov steps */
  int32_t precond;   /* lqcd_precond_kind */
  lqcd_schwarz_params schwarz; /* SCHWARZ; with LEARNED, the fallback (mr_steps 0: none) */
  const lqcd_ptc_net *learned; /* LEARNED: the network (op_precond: FP32 instance for its transports) */
  /* Optional residual history (host memory, may be NULL): entry k receives
   * ||rhat|| after Krylov step k+1 (the iterated residual of Algorithm 1, in
   * the Krylov precision, not divided by ||b||), while k < res_history_max;
   * info->history_len is the number written. */
  double *res_history;
  int32_t res_history_max;
  /* Gram-Schmidt passes of the orthogonalisation (Algorithm 1's MGS loop
   * over z_0..z_{k-1}): 0 or 1 one classical pass (all coefficients from one
   * set of dot products, then one multi-axpy), 2 classical Gram-Schmidt with
   * re-orthogonalisation (CGS2: a second pass whose coefficients add to the
   * first's). Both equal MGS in exact arithmetic; other values are refused. */
  int32_t orth_passes;
} lqcd_gcr_params;

typedef enum { LQCD_CG_CGNE_SCHUR = 0, LQCD_CG_STAG_NORMAL = 1 } lqcd_cg_kind;

typedef struct {
  double tol;            /* stop when ||b - A x|| <= tol ||b|| (FP64) */
  int32_t max_iter;
  double delta_reliable; /* reliable update when ||r|| < delta * max ||r|| since the last one */
  int32_t kind;          /* lqcd_cg_kind */
  /* Optional iterate recording (kind CGNE_SCHUR, op_sloppy NULL): after every
   * record_every-th iteration, while fewer than record_max are stored, the
   * even-site residual r_k = bhat - Mhat x_k goes to record_r[j] and the error
   * e_k = record_xstar - x_k to record_e[j] (packed even spinors of op_hi, j
   * consecutive fields); *record_count (host) receives the number stored.
   * These are the residual -> error pairs the learned preconditioner trains on. */
  void *record_r;
  void *record_e;
  const void *record_xstar;
  int32_t record_every;
  int32_t record_max;
  int32_t *record_count;
  /* Right-hand sides solved together (0 is read as 1), at most LQCD_MAX_CG_RHS.
   * x and b then hold nrhs fields in the multi-source layout of
   * lqcd_spinor_import; every system runs its own CG recurrences and stops on
   * its own ||b_j - A x_j|| <= tol ||b_j||, while the operator is applied to
   * all sources in one launch (each link is read once for all of them). */
  int32_t nrhs;
  /* Optional (host, may be NULL): nrhs entries, the final FP64 true residual
   * ||b_j - M x_j|| / ||b_j|| of each system (info->true_residual is their
   * maximum). */
  double *rhs_residuals;
  /* Optional residual history (host, may be NULL; nrhs = 1): entry k receives
   * ||r|| after iteration k+1 (the iterated residual, in absolute units:
   * ||bhat - Mhat x|| for CGNE_SCHUR), while k < res_history_max. */
  double *res_history;
  int32_t res_history_max;
} lqcd_cg_params;

#define LQCD_MAX_CG_RHS 32

/* ---------------------------------------------------------------------- */
/* context and sizes                                                       */

/* Create a context on the current HIP device. */
lqcd_status lqcd_context_create(lqcd_context **ctx);
lqcd_status lqcd_context_destroy(lqcd_context *ctx);
/* Text of the last error (never NULL; "" if none). ctx may be NULL. */
const char *lqcd_last_error(const lqcd_context *ctx);

/* Bytes of one packed field of `kind` for operator `op` with nrhs right-hand sides. */
lqcd_status lqcd_field_bytes(const lqcd_operator *op, int32_t kind, int32_t nrhs, size_t *bytes);

/*
 * dst = src on the device, `bytes` a multiple of 16 (both pointers 16-byte
 * aligned, not overlapping): one streaming pass of 16-byte loads and stores.
 * Not part of the paper's method: it measures the bandwidth a
 * read-once/write-once kernel reaches on this GPU (the practical ceiling next
 * to the stencil kernels) and calibrates hardware byte counters with a kernel
 * of known traffic.
 */
lqcd_status lqcd_stream_copy(lqcd_context *ctx, void *dst, const void *src, size_t bytes, lqcd_stream stream);

/*
 * The autotuner's choices so far in this context, as text: one
 * "key<TAB>value" line per tuned kernel shape (kernel, precision, link format,
 * lattice/tile and source count in the key; workgroup size, batch form or
 * network form as the value). Writes at most cap bytes including the
 * terminating NUL (buf may be NULL to query); *len receives the full size
 * needed, NUL included.
 */
lqcd_status lqcd_tuned_choices(lqcd_context *ctx, char *buf, size_t cap, size_t *len);

/* ---------------------------------------------------------------------- */
/* setup: packing and derived fields                                       */

/*
 * Pack natural FP64 links (device, [V][4][3][3] complex) into op's layout,
 * precision and compression. which = LQCD_FIELD_GAUGE packs Wilson links
 * (recon op->recon) or staggered fat links (always 18 reals);
 * which = LQCD_FIELD_LONG packs staggered long links already formed.
 * Compression 12/8 assumes SU(3) links.
 */
lqcd_status lqcd_gauge_import(lqcd_context *ctx, const lqcd_operator *op, void *packed,
                              const void *natural, int32_t which, lqcd_stream stream);

/*
 * Long links of eq. (3): L_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu), formed in
 * FP64 from natural thin links (device) and packed with op->recon.
 */
lqcd_status lqcd_long_link_build(lqcd_context *ctx, const lqcd_operator *op, void *packed_long,
                                 const void *natural_thin, lqcd_stream stream);

/*
 * Clover field of eq. (2) (its footnote: 72 reals per site) in kappa
 * normalisation, A = 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu, built
 * in FP64 from natural links (device) and inverted per site (two Hermitian
 * 6x6 chiral blocks, Cholesky); both packed in op's layout and precision for
 * both parities. Returns LQCD_ERR_BREAKDOWN if a block is not positive definite.
 */
lqcd_status lqcd_clover_build(lqcd_context *ctx, const lqcd_operator *op, void *clover,
                              void *clover_inv, const void *natural_gauge, lqcd_stream stream);

/*
 * Pack / unpack a spinor between natural FP64 (device) and op's layout.
 * parity 0 or 1: only that parity (packed = one LQCD_FIELD_SPINOR block);
 * parity -1: both (packed = LQCD_FIELD_SPINOR_FULL). Export writes only the
 * natural sites of the parities it covers.
 * nrhs > 1: `natural` holds nrhs consecutive natural fields, and the packed
 * field stores them source-major (packed index rhs * (sites per parity) +
 * site, i.e. nrhs single-source blocks one after another, within each parity
 * block), the layout every nrhs > 1 call below expects; its size is
 * lqcd_field_bytes(op, kind, nrhs).
 */
lqcd_status lqcd_spinor_import(lqcd_context *ctx, const lqcd_operator *op, void *packed,
                               const void *natural, int32_t parity, int32_t nrhs, lqcd_stream stream);
lqcd_status lqcd_spinor_export(lqcd_context *ctx, const lqcd_operator *op, void *natural,
                               const void *packed, int32_t parity, int32_t nrhs, lqcd_stream stream);

/*
 * out = scale * in between two instances of the same action and lattice
 * (any precisions and tiles; fields are re-laid out when the tiles differ):
 * parity 0 or 1 (single-parity fields) or -1 (full fields), nrhs right-hand
 * sides. out and in may be the same buffer only if precisions and tiles are
 * equal.
 */
lqcd_status lqcd_spinor_convert(lqcd_context *ctx, const lqcd_operator *op_out, void *out,
                                const lqcd_operator *op_in, const void *in, int32_t parity, int32_t nrhs,
                                double scale, lqcd_stream stream);

/* ---------------------------------------------------------------------- */
/* operators                                                               */

/*
 * Hopping term between parities: out_p = D_{p,1-p} in_{1-p}.
 * Wilson (eq. (2)): D = sum_mu (1-gamma_mu) U_mu(x) delta_{x+mu} + (1+gamma_mu) U^+_mu(x-mu) delta_{x-mu};
 * dagger = 1 applies D^+ = gamma5 D gamma5.
 * Staggered (eq. (3)): fat and long hops with Kogut-Susskind phases; dagger = 1 applies D^+ = -D.
 * block: NULL, or the Dirichlet block size per axis (each divides dims):
 * every hop whose two sites lie in different blocks is dropped (Section III-B,
 * Section VIII-A); an axis with one block keeps its periodic hop.
 * out and in are packed single-parity spinors with nrhs right-hand sides
 * (source-major; one launch whose workgroups for the sources of a site block
 * run together, so a link is fetched from memory once for all of them).
 * With LQCD_MRHS_MFMA=1, 16-bit operators with a multiple of 4 sources take
 * the link products on the matrix cores (the default vector form measures
 * faster on gfx950). out must not alias in.
 */
lqcd_status lqcd_dslash(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in,
                        int32_t out_parity, int32_t dagger, const int32_t *block, int32_t nrhs,
                        lqcd_stream stream);

/*
 * Clover term of eq. (2): out_p = A_p in_p (inverse = 0) or A_p^-1 in_p
 * (inverse = 1), single-parity packed spinors, nrhs right-hand sides (source-major).
 */
lqcd_status lqcd_clover_apply(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in,
                              int32_t parity, int32_t inverse, int32_t nrhs, lqcd_stream stream);

/*
 * Even-odd operator on even sites (Section III-A):
 * Wilson-clover: out = Mhat in = A_ee in - kappa^2 D_eo A_oo^-1 D_oe in (dagger: Mhat^+);
 * staggered: out = N_e in = m^2 in - D_eo D_oe in / 4.
 * block as in lqcd_dslash (Dirichlet-cut operator Mhat_B).
 */
lqcd_status lqcd_schur_apply(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in,
                             int32_t dagger, const int32_t *block, int32_t nrhs, lqcd_stream stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): exactly
 * lqcd_schur_apply (the same kernels and result, bit for bit), but its
 * intermediate odd-parity spinor lives in a fixed 64 MiB device array of the
 * library (one per GPU, held from library load until the process ends)
 * instead of context scratch, and the autotuner does not run timing launches
 * (tuned launch parameters if the shape was tuned in this context, else
 * defaults). Nothing is allocated: no hipMalloc, hipFree or event creation.
 * The caller passes the inputs and outputs as for lqcd_schur_apply.
 * Errors: LQCD_ERR_UNSUPPORTED when one parity of nrhs spinors of op
 * (lqcd_field_bytes(op, LQCD_FIELD_SPINOR, nrhs)) exceeds 64 MiB, with
 * nothing launched; otherwise the checks of lqcd_schur_apply.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other host threads, other contexts) race and must be
 * ordered by the caller. The array needs no clearing (each call writes the
 * part it reads first).
 */
lqcd_status lqcd_schur_apply_noalloc(lqcd_context *ctx, const lqcd_operator *op, void *out, const void *in,
                                     int32_t dagger, const int32_t *block, int32_t nrhs, lqcd_stream stream);

/*
 * Batched Wilson hopping term over several operators in one persistent
 * launch (the lattices may differ in size): for every job,
 * out = D_{p,1-p} in (dagger: D^+) with nrhs right-hand sides (source-major).
 * All jobs share precision and link compression; at most 8 jobs. Work items
 * are one workgroup's worth of site x source pairs; either a fixed grid of
 * workgroups takes them from per-XCD queues until every job is done, or one
 * workgroup runs per item. The form, workgroup size and grid come from the
 * autotuner (timed on first use of a batch shape, see LQCD_TUNE /
 * LQCD_TUNE_CACHE). The paper is silent on batching; each job computes
 * exactly lqcd_dslash (the same arithmetic, bit for bit).
 */
typedef struct {
  const lqcd_operator *op;
  void *out;
  const void *in;
  int32_t out_parity;
  int32_t nrhs;
} lqcd_dslash_job;
lqcd_status lqcd_dslash_batch(lqcd_context *ctx, const lqcd_dslash_job *jobs, int32_t njobs, int32_t dagger,
                              lqcd_stream stream);

/*
 * Schwarz preconditioner on the Dirichlet blocks of params->block (Section
 * III-B; Section VIII-A). out_even = K in_even, packed even spinors in
 * op_precond's precision (out_even is overwritten, in_even is not).
 * cycles = 0, additive (the paper's): on every block B, mr_steps
 *   minimal-residual steps on the cut operator Mhat_B, started from zero, with
 *   inner products over B only; the blocks are independent (block Jacobi).
 * cycles = n >= 1, multiplicative (the alternating procedure; Section X names
 *   it as the next step): blocks are coloured by the parity of the sum of
 *   their coordinates, so blocks of one colour never touch. Starting from
 *   out = 0, each of n cycles visits colour 0 then colour 1; a visit runs the
 *   same block MR on that colour's blocks only, on the current residual
 *   in - Mhat out of the whole system, and adds the result to out. One
 *   uncut application of Mhat per visit but the last. Needs an even number of
 *   blocks along x (else LQCD_ERR_UNSUPPORTED).
 * Either K is positively homogeneous, K(c r) = c K(r), and depends on
 * in_even nonlinearly (MR), so the outer solver must be flexible (GCR).
 */
lqcd_status lqcd_schwarz_precond(lqcd_context *ctx, const lqcd_operator *op_precond,
                                 const lqcd_schwarz_params *params, void *out_even,
                                 const void *in_even, lqcd_stream stream);

/* ---------------------------------------------------------------------- */
/* solvers                                                                 */

/*
 * Mixed-precision GCR-DD, Algorithm 1: solves M x = b for the full
 * Wilson-clover lattice through the even-odd system (source
 * bhat = b_e + kappa D_eo A_oo^-1 b_o, solve Mhat x_e = bhat, then
 * x_o = A_oo^-1 (b_o + kappa D_oe x_e)). The Krylov space (p, z) is built
 * in op_krylov's precision, K in op_precond's, and every restart recomputes
 * r = bhat - Mhat x with op_hi (FP64), where the solution accumulates.
 * op_hi and op_krylov share one tile; op_precond may use another (the Schwarz
 * blocks equal its tile), and K's input and output are then re-laid out.
 * x_full (in: initial guess, out: solution) and b_full are packed
 * LQCD_FIELD_SPINOR_FULL fields of op_hi. Returns LQCD_ERR_NOT_CONVERGED
 * (best iterate in x_full, info filled) when max_iter is reached.
 * precond = LQCD_PRECOND_LEARNED with params->schwarz.mr_steps > 0: a step
 * whose residual drops by less than 5%, or whose network output is zero or
 * not finite, hands the next step (or, for an unusable output, the same step)
 * to the Schwarz preconditioner; info->fallback_applies counts those steps.
 * Without the fallback an unusable direction returns LQCD_ERR_BREAKDOWN.
 */
lqcd_status lqcd_gcr_solve(lqcd_context *ctx, const lqcd_operator *op_hi,
                           const lqcd_operator *op_krylov, const lqcd_operator *op_precond,
                           const lqcd_gcr_params *params, void *x_full, const void *b_full,
                           lqcd_solve_info *info, lqcd_stream stream);

/*
 * CG (Section III-A) with reliable updates when op_sloppy is less precise
 * than op_hi (x and the true residual kept in op_hi's precision).
 * params->nrhs > 1 solves that many systems with the same operator at once
 * (x and b in the multi-source layout; see lqcd_cg_params).
 * kind = LQCD_CG_CGNE_SCHUR: solves M x = b for the full Wilson-clover
 *   lattice through CG on the normal equations of Mhat (x, b packed FULL);
 * kind = LQCD_CG_STAG_NORMAL: solves N_e x_e = b_e on even sites (eq. (4)
 *   with one shift sigma = 0; x, b packed single-parity even).
 * op_sloppy may be NULL (pure op_hi). With an FP16 or BF16 op_sloppy and
 * kind STAG_NORMAL (one source), the iteration's vectors are kept in FP32 and
 * only the operator's input and output are 16-bit. x holds the starting guess
 * on entry (zero for a cold start) and the solution on return.
 */
lqcd_status lqcd_cg_solve(lqcd_context *ctx, const lqcd_operator *op_hi,
                          const lqcd_operator *op_sloppy, const lqcd_cg_params *params, void *x,
                          const void *b, lqcd_solve_info *info, lqcd_stream stream);

/*
 * Multi-shift CG for the shifted staggered systems of eq. (4),
 *   (N_e + sigma_i) x_i = b,  i = 0 .. nshift - 1,  on even sites,
 * N_e = m^2 - D_eo D_oe / 4 (so N_e + sigma is the same normal operator at mass
 * sqrt(m^2 + sigma)). The strategy of Section VIII-B: one multi-shift CG in the
 * precision of op_sloppy produces every x_i from the Krylov space of the
 * smallest shift (Section III-A: the residuals of all shifted systems stay
 * collinear), each shift stopping once its residual estimate is below
 * tol_sloppy; then each x_i is refined to tol by the reliable-update CG of
 * lqcd_cg_solve (op_hi FP64, op_sloppy) starting from it, its residual
 * recomputed in FP64. op_sloppy: FP32, or NULL (multi-shift stage in FP64);
 * 16-bit is refused (the multi-shift solutions would be too inaccurate to
 * refine, as the paper notes). x: host array of nshift device pointers, each a
 * packed even spinor of op_hi (written, not read); b: packed even spinor of
 * op_hi. Both operators staggered, same system except precision and links.
 */
#define LQCD_MAX_SHIFTS 16

typedef struct {
  int32_t nshift;                 /* 1 .. LQCD_MAX_SHIFTS */
  double shifts[LQCD_MAX_SHIFTS]; /* sigma_i, with m^2 + sigma_i > 0 */
  double tol;                     /* final ||b - (N_e + sigma_i) x_i|| <= tol ||b||, recomputed in FP64 */
  double tol_sloppy;              /* multi-shift stage, per shift (in FP32, 1e-8: about where the
                                     refinements stop getting shorter) */
  int32_t max_iter;               /* per stage and per refinement */
  double delta_reliable;          /* of the refinements (see lqcd_cg_params) */
} lqcd_multishift_params;

typedef struct {
  int32_t ms_iters;                       /* iterations of the multi-shift stage */
  int32_t ms_matvecs;                     /* its applications of N_e */
  double ms_seconds;                      /* its wall time */
  lqcd_solve_info shift[LQCD_MAX_SHIFTS]; /* refinement of each x_i: iters, reliable updates, matvecs,
                                             final FP64 true residual, seconds */
  double seconds;                         /* wall time of the call */
} lqcd_multishift_info;

lqcd_status lqcd_multishift_cg_solve(lqcd_context *ctx, const lqcd_operator *op_hi, const lqcd_operator *op_sloppy,
                                     const lqcd_multishift_params *params, void *const *x, const void *b,
                                     lqcd_multishift_info *info, lqcd_stream stream);

/*
 * Mixed-precision BiCGstab (van der Vorst; Section III-A names it as the usual
 * non-Hermitian method for Wilson-clover, and Section IX compares GCR-DD with
 * its mixed-precision form): solves M x = b for the full Wilson-clover lattice
 * through the even-odd system Mhat x_e = bhat (the same reduction and
 * reconstruction as lqcd_gcr_solve). The iteration runs in op_sloppy's
 * precision (FP32, FP16 or BF16; NULL: FP64), its shadow residual the first
 * residual. Reliable updates (residual replacement): when ||r|| falls below
 * delta_reliable times its largest value since the previous update, or the
 * iterated residual claims convergence, the sloppy solution is added to the
 * FP64 x_e and r = bhat - Mhat x_e is recomputed with op_hi; the search
 * directions and the shadow residual are kept. If the half-step residual s
 * meets tol but the recomputed one does not, or <rhat, v> vanishes, the
 * iteration restarts with the current residual as the new shadow residual.
 * x_full (in: initial guess, out: solution) and b_full are packed
 * LQCD_FIELD_SPINOR_FULL fields of op_hi (FP64); op_sloppy: same system and
 * tile. info: iters (BiCGstab steps, two applications of Mhat each),
 * restarts (reliable updates), matvecs, true_residual (FP64, full lattice),
 * seconds; the other fields zero. Returns LQCD_ERR_NOT_CONVERGED (best
 * iterate in x_full, info filled) at max_iter, LQCD_ERR_BREAKDOWN if a
 * restart breaks down again before any progress.
 */
typedef struct {
  double tol;            /* stop when ||b - M x|| <= tol ||b|| (FP64) */
  int32_t max_iter;      /* BiCGstab steps */
  double delta_reliable; /* 0 <= delta < 1 (0: updates only at apparent convergence) */
} lqcd_bicgstab_params;

lqcd_status lqcd_bicgstab_solve(lqcd_context *ctx, const lqcd_operator *op_hi, const lqcd_operator *op_sloppy,
                                const lqcd_bicgstab_params *params, void *x_full, const void *b_full,
                                lqcd_solve_info *info, lqcd_stream stream);

/* ---------------------------------------------------------------------- */
/* learned preconditioner                                                  */

/* Number of complex master weights and bytes of the packed weights. */
lqcd_status lqcd_ptc_sizes(const lqcd_ptc_shape *shape, size_t *n_weights, size_t *packed_bytes);

/* Convert FP32 master weights (device) to the packed BF16 layout (device). */
lqcd_status lqcd_ptc_pack(lqcd_context *ctx, const lqcd_ptc_shape *shape, const void *weights, void *packed,
                          lqcd_stream stream);

/*
 * out_even = N(in_even): the network applied to a residual on even sites
 * (zero on odd sites), output read on even sites. op: FP32 Wilson-clover
 * instance (links for the transports, its layout for the fields).
 */
lqcd_status lqcd_ptc_apply(lqcd_context *ctx, const lqcd_operator *op, const lqcd_ptc_net *net, void *out_even,
                           const void *in_even, lqcd_stream stream);

/*
 * Loss L = |N(r) - e|^2 / |e|^2 over even sites and its gradient
 * grad = dL/d conj(W) (FP32 complex, master layout; dL = 2 Re <grad, dW>).
 * r_even, e_even: FP32 packed even spinors of op. *loss (host) is set.
 */
lqcd_status lqcd_ptc_gradient(lqcd_context *ctx, const lqcd_operator *op, const lqcd_ptc_net *net,
                              const void *r_even, const void *e_even, void *grad, double *loss, lqcd_stream stream);

/*
 * Residual loss L = |Mhat N(r) - r|^2 / |r|^2 over even sites (Mhat the even-odd
 * Schur operator of op, which must carry its clover fields) and its gradient
 * grad = dL/d conj(W); *loss (host) is set. The network then approximates
 * Mhat^-1 on the directions r it is shown, weighted as GCR weights them: the
 * residual left after a preconditioned step.
 */
lqcd_status lqcd_ptc_residual_gradient(lqcd_context *ctx, const lqcd_operator *op, const lqcd_ptc_net *net,
                                       const void *r_even, void *grad, double *loss, lqcd_stream stream);

/*
 * Vector-Jacobian product: grad = dL/d conj(W) for any real loss L whose
 * derivative with respect to the network output y = N(r_even) is
 * dy_even = dL/d conj(y) (FP32 packed even spinor of op; dL = 2 Re <dy, dy'>
 * to first order). The forward pass on r_even is recomputed. Used to train on
 * losses that involve the Dirac operator, e.g. |Mhat N(r) - r|^2 / |r|^2 with
 * dy = Mhat^+ (Mhat N(r) - r) / |r|^2.
 */
lqcd_status lqcd_ptc_vjp(lqcd_context *ctx, const lqcd_operator *op, const lqcd_ptc_net *net, const void *r_even,
                         const void *dy_even, void *grad, lqcd_stream stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the FP32 master weights. */
lqcd_status lqcd_ptc_adam(lqcd_context *ctx, const lqcd_ptc_shape *shape, void *weights, void *m, void *v,
                          const void *grad, int32_t step, double lr, lqcd_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* LQCD_H */
