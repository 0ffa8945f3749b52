/*
 * lbmz.h -- DWT-compressed stencil simulation on one AMD Instinct GPU (gfx950).
 *
 * C99 ABI of the library liblbmz.so.  The library keeps a regular-grid
 * finite-volume or lattice-Boltzmann state in compressed form and advances it
 * patch by patch: every patch is rebuilt from its thresholded wavelet
 * coefficients by the inverse transform, completed with a one-node ghost ring
 * taken from its neighbours, advanced by the stencil update, transformed
 * forward, hard-thresholded, and its surviving coefficients are compacted back
 * into the store.  This is the patch-at-a-time residency the paper proposes in
 * its Introduction (Flint & Helluy, arXiv 2302.09883) and leaves as future
 * work in its Conclusions; its compression pipeline is Section 2 (wavelet
 * transform 2.1, thresholding 2.2, lossless stage 2.3) and its subgrid
 * structure is Section 3.1.1.
 *
 * Conventions shared by every call:
 *   - Every call returns an lbmz_status; on failure lbmz_last_error() gives a
 *     per-context message.  No call throws or aborts.
 *   - Ownership: the library owns every device allocation it makes (pools,
 *     offset tables, halo strips, scratch).  Buffers passed in belong to the
 *     caller and are only read or written during the call.
 *   - Host buffers are used synchronously: the call returns after the copy on
 *     the context's stream has completed.  Device buffers (flag *_on_device)
 *     must live on the context's device and are used in stream order.
 *   - Dense fields are n[0] x n[1] elements, x fastest (element (x, y) at
 *     x + n[0] * y), unique cells only, in the scheme's dtype.
 *   - A context is not thread-safe; separate contexts are independent.
 */
#ifndef LBMZ_H
#define LBMZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmz_ctx lbmz_ctx;

typedef enum {
  LBMZ_OK = 0,
  LBMZ_EINVAL = -1,    /* invalid argument or geometry */
  LBMZ_ENOMEM = -2,    /* device or host allocation failed */
  LBMZ_EDEVICE = -3,   /* HIP runtime error */
  LBMZ_EOVERFLOW = -4, /* pool could not be grown to hold the store */
  LBMZ_ENAN = -5,      /* a non-finite coefficient appeared; state kept at the last good step */
  LBMZ_ESTATE = -6     /* call not valid in the context's current state */
} lbmz_status;

typedef enum { LBMZ_F32 = 0, LBMZ_F64 = 1 } lbmz_dtype;

/* Periodic regular grid of n[0] x n[1] (x n[2]) cells of size h (Section 1,
 * the periodicity condition).  dim is 2 (n[2] ignored) or 3 (the D3Q19
 * scheme only, n[0] = n[1] = n[2]); periodic must be 1.  Dense fields are
 * arrays [n[2]][n[1]][n[0]] (x fastest). */
typedef struct {
  int dim;
  int64_t n[3];
  int periodic;
  double h;
} lbmz_grid;

typedef enum {
  /* Finite-volume scheme of equation "vf_scheme" with the upwind transport
   * flux of equation "upwind_trans": one scalar field, velocity vel[0..1],
   * time step dt = cfl * h / max(|vel[0]|, |vel[1]|). */
  LBMZ_FV_UPWIND = 0,
  /* D2Q9 lattice-Boltzmann BGK (the paper names LBM and cites the textbook
   * scheme): 9 populations with velocities (0,0) (1,0) (0,1) (-1,0) (0,-1)
   * (1,1) (-1,1) (-1,-1) (1,-1), weights 4/9, 1/9, 1/36; pull streaming then
   * collision with relaxation time tau; the stored state is post-collision. */
  LBMZ_LBM_D2Q9_BGK = 1,
  /* Compressible Euler equations, four conserved fields (rho, rho u, rho v,
   * E), scheme of equation "vf_scheme" with the Rusanov flux
   * Q(W_L, W_R, N) = (F(W_L).N + F(W_R).N) / 2 - lambda (W_R - W_L) / 2,
   * lambda = max(|u.N| + c) over both states, c = sqrt(gamma p / rho),
   * p = (gamma - 1)(E - rho |u|^2 / 2); time step dt = cfl * h / vel[0] with
   * vel[0] a bound of |u| + c given by the caller.  float32 only. */
  LBMZ_EULER_RUSANOV = 2,
  /* D3Q19 lattice-Boltzmann BGK on 3-D grids (the textbook scheme; the
   * paper's subgrids of Section 3.1.1 are 3-D): 19 populations with
   * velocities (0,0,0), (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1),
   * (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
   * (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1), weights 1/3, 1/18, 1/36; pull
   * streaming then collision with relaxation time tau; float32, folded BL5/3
   * patches of 16^3 or 32^3 cells, float32 records only. */
  LBMZ_LBM_D3Q19_BGK = 3
} lbmz_scheme_kind;

typedef struct {
  lbmz_scheme_kind kind;
  lbmz_dtype dtype;   /* arithmetic and storage type of the state */
  double vel[3];      /* FV: transport velocity (alpha, beta); Euler: vel[0] bounds |u| + c */
  double cfl;         /* FV, Euler: Courant number */
  double tau;         /* LBM: relaxation time (> 1/2) */
  double gamma;       /* Euler: ratio of specific heats (> 1) */
} lbmz_scheme;

typedef enum {
  /* Haar lifting on 2^J nodes per patch (d = b - a, s = a + d/2); patches
   * partition the grid.  Not in the paper; used by the transport workload. */
  LBMZ_HAAR = 0,
  /* Folded BL5/3 lifting on 2^J + 1 nodes per patch (Section 2.1.2): the
   * bordering node is shared with the neighbour (Section 3.1.1), which keeps
   * the trapezoid mass of the grid exactly conserved. */
  LBMZ_BL53 = 1
} lbmz_wavelet;

/* Section 2.2.  A detail of level lev (1 = finest) in an L-level transform
 * has rank r = L - lev per dimension (0 = coarsest detail, a sample dimension
 * counts 0).  Threshold: constant eps; capped eps * 2^max(r); accumulation
 * eps * 2^sum(r).  A detail with |c| < threshold is set to zero; samples are
 * never thresholded. */
typedef enum { LBMZ_THR_CAPPED = 0, LBMZ_THR_CONSTANT = 1, LBMZ_THR_ACCUM = 2 } lbmz_thr_rule;

/* How the surviving coefficients of a record are stored (the record layouts
 * are given with the store access calls below).  The narrow formats need a
 * float32 state: the coarse samples stay float32 -- by equation
 * "conservation" they alone carry the tile's mass, so the stored mass is
 * exact -- and the details are stored as IEEE binary16 or OCP E4M3 codes
 * with one power-of-two float32 scale per subband and record. */
typedef enum {
  LBMZ_VALUES_F32 = 0,   /* every kept coefficient in the state's dtype */
  LBMZ_VALUES_F16 = 1,   /* float32 samples, binary16 details */
  LBMZ_VALUES_E4M3 = 2,  /* float32 samples, E4M3 details */
  /* float32 samples; per record, E4M3 details when E4M3's rounding bound
   * max(2^-4 m_b, 2^(k_b - 10)) at the largest kept magnitude m_b of every
   * occupied subband b (E4M3 scale 2^k_b) is at most half of that subband's
   * threshold (Section 2.2), binary16 details otherwise: the quantisation
   * then adds at most half of the error the threshold already allows per
   * coefficient.  At eps = 0 every record with a detail is binary16. */
  LBMZ_VALUES_E4M3_BOUNDED = 3
} lbmz_values;

/* Patch decomposition: p[0] = p[1] = cells per patch side, a power of two
 * in {8, 16, 32, 64} dividing n (32 or 64 for the narrow value formats);
 * p[2] is ignored in 2-D and equals p[0] (16 or 32) in 3-D. */
typedef struct {
  int p[3];
  lbmz_wavelet wavelet;
  lbmz_thr_rule rule;
  lbmz_values values;
} lbmz_patch;

typedef struct {
  int64_t steps;          /* steps taken since the state was last set */
  int64_t nnz_total;      /* sum of the offset-table counts (kept coefficients; kept
                             details for the narrow value formats) */
  int64_t store_bytes;    /* record bytes + offset-table bytes of the current store */
  int64_t capacity_bytes; /* bytes allocated for one pool buffer */
  int64_t dense_bytes;    /* n[0] * n[1] * fields * sizeof(dtype) */
  double ratio;           /* dense_bytes / store_bytes */
  int32_t nfields;        /* 1 (FV), 9 (LBM) or 4 (Euler) */
  int32_t npatch;         /* patches in the grid */
  double totals[16];      /* FP64 per-field sums of the decompressed state: trapezoid
                             weights 1/2 on shared bordering nodes (bl53), else 1;
                             the first 16 fields (all of them: lbmz_get_totals) */
  int64_t regrows;        /* pool regrowths absorbed since creation */
  int64_t mask_records;   /* records stored as a bitmask */
  int64_t list_records;   /* records stored as an index list */
  double ms_last_call;    /* GPU time of the last lbmz_step call (HIP events) */
} lbmz_stats_t;

/* Create a compressed context (the method).  levels: wavelet levels L per
 * dimension, 0 <= L <= J - 1 (bl53) or J (Haar) for patches of 2^J cells
 * (one more bl53 level would have no update step and would not conserve
 * mass).  eps >= 0 is the threshold constant c of Section 2.2.  The state is
 * zero until lbmz_set_field / lbmz_set_macroscopic.  On success *out owns a
 * new context.  Errors: LBMZ_EINVAL (geometry, levels, dtype/patch size
 * without a compiled kernel, LDS limit), LBMZ_EDEVICE, LBMZ_ENOMEM. */
int lbmz_create(const lbmz_grid* grid, const lbmz_scheme* scheme, const lbmz_patch* patch,
                int levels, double eps, lbmz_ctx** out);

/* Create an uncompressed context for the same grid and scheme: the plain
 * two-buffer time loop of Section 1 on dense fields.  The same calls apply;
 * lbmz_stats reports store_bytes = dense_bytes. */
int lbmz_create_reference(const lbmz_grid* grid, const lbmz_scheme* scheme, lbmz_ctx** out);

/* Route the context's device allocations through a caller allocator (e.g. a
 * PyTorch caching allocator).  Must be called before the first allocation
 * (right after create).  alloc returns NULL on failure. */
int lbmz_set_allocator(lbmz_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                       void (*free_)(void* ptr, void* user), void* user);

/* Run all work of the context on the given hipStream_t (NULL = default stream). */
int lbmz_set_stream(lbmz_ctx* ctx, void* hip_stream);

/* Bytes of one pool buffer (two are kept: step input and step output).  The
 * pool grows by itself when a step needs more (counted in regrows).  Default:
 * one quarter of the worst-case store. */
int lbmz_set_pool_capacity(lbmz_ctx* ctx, int64_t bytes);

/* Set field `field` (0 <= field < nfields) of the state W^0 (Section 1: the
 * initial condition of the time loop) from a dense array of `bytes` =
 * n[0] * n[1] * sizeof(dtype) bytes, host or device (src_on_device).  Other
 * fields keep their values.  The state is compressed -- forward transform of
 * Section 2.1, hard threshold of Section 2.2, records of Section 2.3.1 -- before
 * the next step, exactly as the compression stage of Section 3.1.3 does after
 * every step.  Errors: LBMZ_EINVAL (field out of range, bytes != field size),
 * LBMZ_EDEVICE, LBMZ_ENOMEM (pool growth). */
int lbmz_set_field(lbmz_ctx* ctx, int field, const void* src, size_t bytes, int src_on_device);

/* LBM only: set all populations to the equilibrium of the given density and
 * velocity fields (each a dense n[0] x n[1] array of the dtype). */
int lbmz_set_macroscopic(lbmz_ctx* ctx, const void* rho, const void* ux, const void* uy,
                         size_t bytes_each, int on_device);

/* Advance n >= 0 steps of the time loop of Section 1 (W^{n+1} from W^n by the
 * scheme, two buffers swapped after every step), each step being the
 * decompress -> step -> compress cycle of Section 3.1.3 carried out patch by
 * patch: inverse transform of the patch's records, ghost ring from the
 * neighbours' lossy values (Section 3.1.1, Fig. 3), stencil update, forward
 * transform, hard threshold (Section 2.2) and compaction (Section 2.3.1).
 * One device-to-host read of the control block per call; n = 0 returns
 * LBMZ_OK at once.  A pool overflow is absorbed by regrowing and replaying the
 * remaining steps from the last good state; LBMZ_ENAN leaves the state at
 * the last step whose coefficients were all finite.  LBMZ_EOVERFLOW only when
 * the regrowth itself fails. */
int lbmz_step(lbmz_ctx* ctx, int n);

/* Decompress field `field` of the current state into a dense array of
 * n[0] * n[1] (n^3 in 3-D) elements of the dtype, host or device
 * (dst_on_device): the decompression of Section 3.1.3 (records expanded, the
 * inverse transform of Section 2.1.2 applied), keeping the owned nodes of
 * every patch (a shared bordering node is written once, by the patch that
 * owns it; Section 3.1.1).  The state is not changed.  Errors: LBMZ_EINVAL
 * (field out of range, bytes != field size), LBMZ_EDEVICE. */
int lbmz_decompress_field(lbmz_ctx* ctx, int field, void* dst, size_t bytes, int dst_on_device);

/* Statistics of the current state (Section 3.1.4, methodology): the
 * compression ratio as dense bytes / store bytes (the x-factors of Section
 * 3.2), the kept-coefficient count, the record encodings, and the FP64 totals
 * that equation "conservation" keeps constant.  Error norms against an
 * uncompressed run (equation "L2_error") are computed by the caller from
 * lbmz_decompress_field of both contexts.  Errors: LBMZ_EINVAL (null out). */
int lbmz_stats(lbmz_ctx* ctx, lbmz_stats_t* out);

/* The per-field totals of lbmz_stats for all `count` = nfields fields. */
int lbmz_get_totals(lbmz_ctx* ctx, double* out, int count);

/* D3Q19 only: set all populations to the equilibrium of the given density
 * and velocity fields (each a dense n^3 float32 array [z][y][x]). */
int lbmz_set_macroscopic3(lbmz_ctx* ctx, const void* rho, const void* ux, const void* uy, const void* uz,
                          size_t bytes_each, int on_device);

/* ---- compressed store access (checkpoint, parity tests) -------------------
 * Record order of the s x s coefficients of one (patch, field) tile, s = p + 1
 * (bl53) or p (Haar), in-place interleaved wavelet layout: the owned p x p
 * block row by row (x fastest), then for bl53 the shared column x = p
 * (y = 0..p-1), the shared row y = p (x = 0..p-1) and the corner (p, p).  The
 * record index k of a coefficient is its position in this order; W =
 * ceil(s*s/64) mask words cover all k.
 * LBMZ_VALUES_F32 record: the kept (non-zero) coefficients in ascending k
 *   (dtype, little endian), zero padding to a multiple of 8 bytes, then
 *   either their u16 indices k (when 2 nnz < 8 W) or W u64 mask words (bit
 *   k%64 of word k/64), zero padding to a multiple of 16 bytes.  The offset
 *   table count is nnz.
 * Narrow records (LBMZ_VALUES_F16 / E4M3 / E4M3_BOUNDED): u64 OCC with bit b
 *   set when subband b = cy (L + 1) + cx holds a kept detail (cx, cy: 0 for a
 *   sample index, else the detail level, 1 = finest), and for E4M3_BOUNDED
 *   bit 63 set when the record's codes are E4M3 (else binary16, scales and
 *   codes of that format); one float32 scale 2^k per set
 *   bit, in increasing b, where 2^k is the smallest power of two with
 *   max |detail| <= 65504 (F16) or 448 (E4M3) times 2^k; zero pad to 8;
 *   float32 samples of all SC x SC sample positions (SC = (s-1)/2^L + 1),
 *   slot (y >> L) SC + (x >> L), zero or not; zero pad to 8; the kept
 *   details' codes code(c / 2^k) in ascending k (2 or 1 bytes each, round to
 *   nearest even); zero pad to 8; then the u16 indices k of the kept details
 *   (when 2 ndet < 8 W) or W mask words over them; zero pad to 16.  The
 *   offset-table count is ndet, the number of kept details.
 * 3-D tiles (D3Q19): s = p + 1 nodes per side; the record index of node
 *   (x, y, z) is k = x + s y + s^2 z; W = ceil(s^3/64); float32 records
 *   with the layout above.
 * Offset table: npatch * nfields entries of two u32, patch-major
 *   (patch index px + (n/p) py (+ (n/p)^2 pz)), field-minor: record offset
 *   in 16-byte units and the count | (1u << 31 when the record is a bitmask).
 * Record placement in the pool is not canonical (any non-overlapping layout
 * is valid); the records themselves are. */

/* ---- execution of the step --------------------------------------------------
 * persistent = 1: every step runs as one launch of a fixed set of resident
 * workgroups (as many as the device holds at once) that take patches from a
 * work queue, instead of one workgroup per patch.  graph = 1: lbmz_step issues
 * its steps in chunks of six as one HIP graph launch (kernel nodes only; the
 * arguments of every node are updated before each launch).  Every mode
 * computes the same records; only their placement in the pool may differ. */
int lbmz_set_execution(lbmz_ctx* ctx, int persistent, int graph);
int lbmz_get_execution(lbmz_ctx* ctx, int* persistent, int* graph);

/* Autotuner: runs 2 * steps_per_variant steps in each of the four modes
 * (advancing the simulation by 8 * steps_per_variant steps; the modes give
 * identical results), times the second half of each with HIP events, and
 * keeps the fastest.  ms_out (may be null) receives the four per-step times,
 * index 2 * persistent + graph. */
int lbmz_autotune(lbmz_ctx* ctx, int steps_per_variant, float* ms_out);

/* ---- per-patch thresholds and the learned predictor's inputs ------------ */

/* Per-patch threshold constants: eps[q] replaces the context's eps for patch
 * q (patch index px + (n/p) py) in every following step and set-up call;
 * count = npatch (host values must be finite and >= 0; device values are the
 * caller's responsibility), or count = 0 to return to the single eps.  The
 * threshold rule stays that of the context (Section 2.2 gives one constant
 * per run; a constant per patch is the learned part's control); shared
 * bordering lines take the smaller threshold of their tiles (see
 * lbmz_set_patch_levels).  2-D contexts with float32 records only. */
int lbmz_set_patch_eps(lbmz_ctx* ctx, const double* eps, size_t count, int on_device);

/* Per-patch threshold level counts: levels[q] (0 <= levels[q] <= L) takes
 * the place of L in the thresholds of patch q (patch index px + (n/p) py) in
 * every following step and set-up call: the levels[q] finest detail levels
 * may be zeroed, with ranks counted from the coarsest of them, and the
 * coefficients of coarser levels are kept like samples (levels[q] = 0 keeps
 * every coefficient).  The transform keeps its L levels.  count = npatch, or
 * count = 0 to return to L.  Section 2.2 gives one threshold and one level
 * count per run; per patch they are the learned part's controls.  With
 * per-patch thresholds or level counts, a bordering line of BL5/3 tiles
 * (stored by both tiles that share it, Section 3.1.1) takes, entry by entry,
 * the smaller threshold of the two tiles, so that both keep the same
 * coefficients of it and the shared values, and the conservation of the
 * totals, hold.  2-D contexts with float32 records only (LBMZ_EINVAL). */
int lbmz_set_patch_levels(lbmz_ctx* ctx, const int* levels, size_t count);

/* With on != 0, every step also writes each patch's network input: the
 * stored coefficients of every field at the owned positions (8 i, 8 j),
 * i, j < 8, as float [npatch][nfields][8][8] (y major).  64 x 64 patches
 * only (LBMZ_EINVAL otherwise). */
int lbmz_enable_features(lbmz_ctx* ctx, int on);

/* Copy the inputs written by the last completed lbmz_step; LBMZ_ESTATE when
 * they are not enabled or no step has completed since.  Layout, float32
 * [npatch][4 nfields][8][8]: channel f < nfields holds field f's stored
 * coefficients at the owned positions (8 i, 8 j) (index j * 8 + i);
 * channel nfields + 3 f + l - 1 the energy (sum of squares, before the
 * threshold) of field f's coefficients of level l = 1, 2, 3 in the 8 x 8
 * block of owned positions [8 i, 8 i + 8) x [8 j, 8 j + 8) (a coefficient's
 * level is the finer of its two per-dimension levels, Section 2.2's classes;
 * every coefficient of a block but its stride-8 corner has a level <= 3).
 * 2-D float32 records and 64 x 64 patches only. */
int lbmz_get_features(lbmz_ctx* ctx, float* dst, size_t bytes, int dst_on_device);

/* ---- the learned threshold predictor ---------------------------------------
 * A small convolutional network (bfloat16 weights, float32 accumulation) that
 * maps a patch's features (lbmz_get_features, 36 channels for the 9 D2Q9
 * populations) to K outputs (the caller's targets, e.g. predicted log10
 * window errors and record bytes of K candidate controls):
 *   input map [12][8][8]: asinh(c / 1e-4) of the 9 coefficient channels and
 *   asinh(sqrt(sum over fields of the level-l energy) / 1e-4), l = 1, 2, 3
 *   -> conv 3x3 12->32, ReLU -> conv 3x3 32->32, ReLU
 *   -> conv 3x3 stride 2 32->32, ReLU -> mean over 4 x 4 -> linear 32->K.
 * Parameters, float32, in this order: w1[32][12][3][3], b1[32],
 * w2[32][32][3][3], b2[32], w3[32][32][3][3], b3[32], wh[K][32], bh[K]
 * (21984 + 33 K values).  The float32 master copy is what set/get exchange;
 * every pass uses its round-to-nearest-even bfloat16 copy.  Loss of a batch:
 * the mean of its B x K squared differences to the targets; training is Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on the master copy.  x: [B][36][8][8],
 * targets and outputs: [B][K], float32, host or device (on_device). */
typedef struct lbmz_net lbmz_net;
int lbmz_net_create(int k, lbmz_net** out);          /* 1 <= k <= 32; parameters start at 0 */
int lbmz_net_param_count(const lbmz_net* net);
int lbmz_net_set_stream(lbmz_net* net, void* hip_stream);
int lbmz_net_set_params(lbmz_net* net, const float* params, size_t count);   /* host; resets Adam */
int lbmz_net_get_params(lbmz_net* net, float* params, size_t count);         /* host */
int lbmz_net_forward(lbmz_net* net, const float* x, int batch, float* y, int on_device);
/* Gradients of the batch loss with respect to the parameters (host buffer of
 * count parameters) and the loss; for checks against a reference. */
int lbmz_net_gradients(lbmz_net* net, const float* x, const float* t, int batch, float* grad_host, float* loss,
                       int on_device);
/* One Adam step on the batch; *loss (may be null) is the loss before the step. */
int lbmz_net_train_step(lbmz_net* net, const float* x, const float* t, int batch, float lr, float* loss,
                        int on_device);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc.  The same
 * gradients and loss as lbmz_net_gradients, computed by the same kernels, but
 * the per-workgroup partial sums (the workspace lbmz_net_gradients allocates
 * and grows with the batch) live in one fixed device array of
 * LBMZ_NET_SCRATCH_BYTES per GPU, set up by lbmz_net_create and held until
 * the process ends; this call allocates nothing and frees nothing.
 * x [batch][36][8][8], t [batch][K], grad [param_count] and loss [1] are
 * float32 device pointers on the network's device; grad and *loss are
 * written.  The call is asynchronous on the network's stream.  The workspace
 * needs ceil(batch / 16) * (4 * param_count) bytes, rounded up to 256, plus
 * 4 * ceil(batch / 16): a batch above that (2992 samples at K = 12) returns
 * LBMZ_EINVAL with the limit in lbmz_net_last_error.  Every call on one GPU
 * shares its array (each call fully rewrites the part it reads), so calls
 * that overlap in time on one GPU -- from any network or stream -- race. */
#define LBMZ_NET_SCRATCH_BYTES (16 * 1024 * 1024)
int lbmz_net_gradients_noalloc(lbmz_net* net, const float* x, const float* t, int batch, float* grad,
                               float* loss);
const char* lbmz_net_last_error(const lbmz_net* net);
void lbmz_net_destroy(lbmz_net* net);

/* Sizes of the current store: pool bytes in use and offset-table entries. */
int lbmz_store_size(lbmz_ctx* ctx, int64_t* pool_bytes, int64_t* table_entries);

/* Copy the current store to host buffers (table: 2 * table_entries u32). */
int lbmz_get_store(lbmz_ctx* ctx, uint32_t* table_host, void* pool_host, size_t pool_bytes);

/* Replace the state by a store given on the host; every record is validated
 * on the host first (LBMZ_EINVAL on any inconsistency).  Halo strips and
 * totals are rebuilt on the device. */
int lbmz_put_store(lbmz_ctx* ctx, const uint32_t* table_host, const void* pool_host,
                   size_t pool_bytes);

/* Replace the state by given wavelet coefficient tiles [npatch][nfields][s][s]
 * ([npatch][19][s][s][s] in 3-D) (dtype): the library thresholds and
 * compacts them (the store's write path fed with known coefficients). */
int lbmz_set_coefficients(lbmz_ctx* ctx, const void* coef, size_t bytes, int on_device);

const char* lbmz_last_error(const lbmz_ctx* ctx);

void lbmz_destroy(lbmz_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBMZ_H */
