/*
 * skmmse.h — C ABI of the MI355X (gfx950) scalable K-MMSE spatial error
 * concealment library (libskmmse.so).
 *
 * Method: Koloda, Seiler, Peinado, Kaup, "Scalable Kernel-Based Minimum Mean
 * Square Error Estimator for Accelerated Image Error Concealment" (arXiv
 * 2205.11226).  Problem statement: Sec. "Reconstruction framework" — a frame
 * region R splits into received pixels S and lost pixels L; every lost vector
 * x0 is estimated from its received context y0 and from all vectors of S with
 * the same spatial configuration, and each estimate is transferred into S
 * once made.  Estimators: Sec. "K-MMSE overview" (eqs. kmmse, weights,
 * bandwidthScaled, epsy, epsx) and Sec. "Scalable K-MMSE estimator" (HQL,
 * IDL eq. slpe, BRL eq. mean).  Gate: Sec. "Layer switching and profile
 * selection" (flatness phi, normalisation factor nu of eq. factor, Table
 * "Profile definitions").
 *
 * Geometry (block mode): a B x B cell of the block grid that holds any lost
 * pixel is a block x0 (loss of any shape, Sec. "Reconstruction framework").
 * Its context is the ring of width `ring` around it plus the cell's own
 * received pixels; candidates are the displacements in [-window, window]^2
 * whose B x B prototype does not overlap the cell and is received.  Distances
 * run over the context pixels known on both sides (a candidate's own positions
 * are its prototype) and are normalised by their count.
 *
 * Conventions shared by every entry point
 *  - All pixel planes are 8-bit, row-major, `stride` bytes between rows
 *    (stride >= width).  `loss_mask` has one byte per pixel, nonzero = lost.
 *  - Lost pixels must lie in B x B cells of the block grid that are fully
 *    inside the frame (not in a partial last row or column of cells);
 *    anything else returns SKM_EUNSUPPORTED.  Values at lost pixels are never
 *    read.  Received pixels are copied unchanged, also inside a block.
 *  - The caller owns every buffer; the library keeps no pointer after return.
 *    `out` may alias `frame` (in place).
 *  - Lost blocks are concealed in rounds: a round takes every pending block
 *    whose known context holds at least ring*block pixels (or, if none does,
 *    the pending blocks with the most known context pixels), estimates them
 *    all from the state at the start of the round and only then marks them
 *    received.
 *  - Output is bitwise deterministic for identical inputs and parameters.
 *  - Errors are status codes; a thread-local message is kept for
 *    skm_last_error().  Nothing throws across the ABI.
 *  - A context is used by one host thread (and one stream) at a time.
 */
#ifndef SKMMSE_H
#define SKMMSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum skm_status {
  SKM_OK = 0,
  SKM_EINVAL = -1,        /* bad argument, or a frame with no received pixel */
  SKM_ENOMEM = -2,        /* device or host allocation failed */
  SKM_EDEVICE = -3,       /* HIP runtime error */
  SKM_EUNSUPPORTED = -4   /* lost pixels outside the in-frame B x B cells     */
} skm_status;

/* Estimation modes (skm_params.mode). */
enum {
  SKM_MODE_PROFILE = 0, /* paper's layered scheme: BRL / IDL with support-area
                           expansion / HQL chosen by (t_phi, t_nu)            */
  SKM_MODE_CNN = 1,     /* BRL where the known context is flat (phi <= t_phi,
                           the profile rule's test), elsewhere the layer
                           chosen by the learned gate; profile rule when no
                           network is loaded                                  */
  SKM_MODE_BRL = 2,     /* context mean for every block (eq. mean)            */
  SKM_MODE_IDL = 3,     /* IDL with expansion, never HQL                      */
  SKM_MODE_FULL = 4,    /* full K-MMSE (HQL) where >= min_hql_cands complete
                           candidates exist, else IDL over the whole window   */
  SKM_MODE_PLAIN = 5    /* fixed-bandwidth kernel regression over the whole
                           window (SLP-E, eq. slpe with M' = M), no gating    */
};

/* Layer codes reported in skm_block_info.layer. */
enum { SKM_LAYER_FILL = -1, SKM_LAYER_BRL = 0, SKM_LAYER_IDL = 1, SKM_LAYER_HQL = 2 };

/* skm_block_info.flags bits. */
enum {
  SKM_FLAG_CTX_RELAXED = 1, /* concealed with fewer than ring*block context px */
  SKM_FLAG_NO_HQL = 2,      /* HQL wanted, too few complete (with hql_partial:
                               admissible) candidates: IDL                    */
  SKM_FLAG_NO_CAND = 4,     /* no admissible candidate: BRL                   */
  SKM_FLAG_EMPTY_CTX = 8,   /* forced fill without context: frame mean        */
  SKM_FLAG_HQL_SINGULAR = 16 /* HQL: C_YY + lambda I met a Cholesky pivot <= 0
                                in FP64 (no covariance model): context mean,
                                layer reported as SKM_LAYER_BRL               */
};

typedef struct skm_params {
  int32_t block;           /* B: 2, 4, 8 or 16 (2: no SKM_MODE_CNN)           */
  int32_t ring;            /* context ring width r, 1..8                      */
  int32_t window;          /* search window half-size W, 1..32                */
  int32_t expand_step;     /* IDL support-area growth step (Chebyshev px);
                              radii step, 2 step, ..., window (at most 16)    */
  int32_t min_overlap_pct; /* candidate needs >= ceil(pct*|m0|/100) common
                              known context pixels (and >= 1), 0..100         */
  int32_t min_hql_cands;   /* HQL needs this many complete candidates (>= 2) */
  int32_t mode;            /* SKM_MODE_*                                       */
  int32_t max_rounds;      /* 0 = until every block is concealed; otherwise
                              remaining blocks get a context-mean fill        */
  double sigma2;           /* IDL kernel decay factor (paper: 10)             */
  double t_phi;            /* flatness threshold T_phi (BRL iff phi <= T_phi) */
  double t_nu;             /* normalisation threshold T_nu (IDL iff nu >= T_nu)*/
  double ridge_rel;        /* HQL ridge: lambda = ridge_rel tr(C_YY)/N_y + 1e-12,
                              ridge_rel >= -1.  C_YY + lambda I is positive
                              definite for ridge_rel >= 0 (up to rounding); a
                              negative value makes it indefinite for any
                              non-isotropic C_YY, which sends HQL blocks to
                              the SKM_FLAG_HQL_SINGULAR fallback (for tests) */
  int32_t hql_partial;     /* 0: HQL over the candidates whose context covers
                              all of m0 (the paper's candidates); 1: over every
                              admissible candidate, partly known contexts
                              completed -- pairwise-complete covariance (each
                              pair of coordinates over the candidates knowing
                              both), lambda x10 up to 6 times until C_YY +
                              lambda I factorises, unknown context pixels set
                              to their coordinate's rounded mean over the
                              candidates knowing it, I0 by d_j / n_j.  Makes
                              full K-MMSE available under lattice and slice
                              loss (a reading: the paper is silent)           */
  int32_t reserved;        /* must be 0                                       */
} skm_params;

/* Per lost block result, in the raster order (by, then bx) of the lost cells. */
typedef struct skm_block_info {
  int32_t bx, by;          /* cell coordinates                                 */
  int32_t layer;           /* SKM_LAYER_*                                      */
  int32_t round;           /* 1-based round that concealed the block           */
  int32_t n_cand;          /* admissible candidates (-1: not evaluated)       */
  int32_t n_complete;      /* candidates whose ring covers all of m0 (-1: n/a)*/
  int32_t radius;          /* accepted IDL radius, or window; 0 for BRL       */
  int32_t flags;           /* SKM_FLAG_*                                       */
  int32_t phi;             /* flatness max(y0) - min(y0) of the known ring    */
  int32_t n_ctx;           /* |m0|: known context pixels (ring and own)        */
  double log_nu;           /* log of the sum of raw IDL weights at `radius`
                              (NaN when not evaluated)                        */
} skm_block_info;

typedef struct skm_ctx skm_ctx;

/* Fill `p` with the paper's defaults: B 16, ring 4, window 24, step 4,
 * overlap 50 %, HQL from 64 complete candidates, sigma^2 10, the "efficient"
 * profile (T_phi 20, T_nu 0.1), ridge 1e-3, SKM_MODE_PROFILE, no round limit. */
void skm_default_params(skm_params* p);

/* Fill `p` with the paper's own patch geometry (Sec. "Reconstruction
 * framework"): the missing vector x0 is a 2 x 2 patch and its context the
 * available pixels of the 6 x 6 neighbourhood centred on it, so B 2 and
 * ring 2; everything else as skm_default_params.  The window of +-24 pixels
 * around a patch at the centre of a lost 16 x 16 block spans the 8
 * neighbouring blocks, the support area of the paper's experiments.
 * Patches whose ring holds fewer than ring*block = 4 known pixels wait for
 * the next round, so the rounds fill a lost region layer by layer from its
 * border towards its centre (the sequential order of the same section and
 * its filling-order figure).  SKM_MODE_CNN is not available. */
void skm_patch_params(skm_params* p);

/* Create a context bound to HIP device `hip_device`.  The context owns its
 * device workspace (grown on demand) and, once loaded, the CNN gate weights.
 * Returns SKM_EINVAL for a bad device or NULL `out`. */
skm_status skm_create(int32_t hip_device, skm_ctx** out);

/* Release the context and all device memory it owns.  NULL is ignored. */
void skm_destroy(skm_ctx* ctx);

/* Host-memory entry point (Sec. "Reconstruction framework" problem
 * statement: conceal(frame, loss_mask, params) -> frame).
 *   frame, loss_mask, out : host planes of height x stride bytes.
 *   info      : optional host array of `info_cap` records (may be NULL).
 *   n_lost    : optional; receives the number of lost blocks.
 * Copies in, runs the rounds on the context's stream, copies out, and
 * returns when the frame is complete.  If info is given and info_cap is
 * smaller than the number of lost blocks, SKM_EINVAL is returned and `out`
 * is left untouched. */
skm_status skm_conceal(skm_ctx* ctx, const uint8_t* frame, const uint8_t* loss_mask,
                       int32_t width, int32_t height, int32_t stride,
                       const skm_params* params, uint8_t* out,
                       skm_block_info* info, int32_t info_cap, int32_t* n_lost);

/* Device-memory entry point; all pointers are device pointers owned by the
 * caller (e.g. PyTorch tensors).  Work is enqueued on `hip_stream` (NULL =
 * the null stream); the call returns once the stream has finished the frame
 * (the round loop reads back one counter per batch of rounds).
 *   d_info : optional device array of cap records (lost-cell raster order).
 *   d_xhat : optional device float array of cap * B * B pre-rounding
 *            estimates, block i at offset i*B*B, row-major in the block.
 *   cap    : capacity of d_info / d_xhat in blocks; SKM_EINVAL if too small.
 *   n_lost : optional host pointer receiving the number of lost blocks. */
skm_status skm_conceal_device(skm_ctx* ctx, const uint8_t* d_frame, const uint8_t* d_mask,
                              int32_t width, int32_t height, int32_t stride,
                              const skm_params* params, uint8_t* d_out,
                              skm_block_info* d_info, float* d_xhat, int32_t cap,
                              int32_t* n_lost, void* hip_stream);

/* Allocation-free variant of skm_conceal_device, for callers that cannot
 * allocate device memory while concealing (tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and return behaviour as
 * skm_conceal_device, bitwise; the caller still owns frame, mask, out, info
 * and xhat.  The call makes no hipMalloc, hipFree or other allocation: the
 * frame's workspace (value plane, block tables, round state, gate and HQL
 * scratch) is carved from a 64 MiB device array of the library, one per GPU,
 * held from skm_create until the process ends.  Frames whose workspace does
 * not fit return SKM_EINVAL with the size they need: without HQL scratch
 * this is about 2 bytes per pixel plus 33 bytes per B x B cell (a 1920 x 1080
 * frame takes 4.4 MB, a 3840 x 2160 frame at B = 16 17.7 MB); modes that may run HQL
 * (SKM_MODE_PROFILE, SKM_MODE_CNN, SKM_MODE_FULL) also need one HQL slot,
 * 12.9 MB at B = 16 (ring 4, window 24), and use as many HQL workgroups
 * as the rest of the array holds (fewer than skm_conceal_device: slower HQL,
 * same results).  Frames are launched eagerly (no graph) and without kernel
 * timing.  Every call on one GPU, from any context, shares that GPU's array,
 * which keeps the last call's contents: calls that overlap in time on one GPU
 * race and must be serialised by the caller. */
skm_status skm_conceal_device_noalloc(skm_ctx* ctx, const uint8_t* d_frame,
                                      const uint8_t* d_mask, int32_t width, int32_t height,
                                      int32_t stride, const skm_params* params, uint8_t* d_out,
                                      skm_block_info* d_info, float* d_xhat, int32_t cap,
                                      int32_t* n_lost, void* hip_stream);

/* Distance table of the kernel-regression core (eq. weights / eq. slpe):
 * for each lost block i (lost-cell raster order) and each displacement
 * (dx, dy) in [-W, W]^2 (index (dy+W)*(2W+1) + (dx+W)), the exact integer
 * d = sum over context pixels known on both sides of (y0 - y_j)^2 and their
 * count n, evaluated on the received frame before any concealment.
 * d = -1 (and n = 0) where the displacement is not an admissible candidate.
 *   d_dist, d_cnt : device int32 arrays of cap * (2W+1)^2 entries.
 * Mode and thresholds in `params` are ignored.  Same argument rules and
 * return behaviour as skm_conceal_device. */
skm_status skm_distances_device(skm_ctx* ctx, const uint8_t* d_frame, const uint8_t* d_mask,
                                int32_t width, int32_t height, int32_t stride,
                                const skm_params* params, int32_t* d_dist, int32_t* d_cnt,
                                int32_t cap, int32_t* n_lost, void* hip_stream);

/* ---------------------------------------------------------- learned gate
 * A small CNN can replace the profile rule of the layer switching (Sec.
 * "Layer switching and profile selection"): from a 48 x 48 window centred on
 * a lost block (channels: (u - 128)/128 at known pixels and 0 elsewhere; 1 at
 * unknown pixels) it predicts g1 = dB gain of IDL over BRL and g2 = dB gain
 * of HQL over IDL.  In SKM_MODE_CNN a block takes BRL if g1 <= tau1, else HQL
 * if g2 > tau2 (full-window IDL when HQL is unavailable), else IDL with the
 * support-area expansion of t_nu.  Without a loaded network SKM_MODE_CNN
 * applies the profile rule.  Network: the (2, 48, 48) window rearranged
 * without loss into (8, 24, 24) (channel 4 c + 2 dy + dx at (Y, X) holds
 * channel c at pixel (2 Y + dy, 2 X + dx)); three 3x3 convolutions (stride
 * 2, zero padding 1, 32 channels, ReLU: 24 -> 12 -> 6 -> 3), global average
 * pool, linear 32 -> 2; bfloat16 weights and convolution inputs, FP32
 * accumulation; 20898 FP32 master parameters in the order w1[32][8][3][3],
 * b1[32], w2[32][32][3][3], b2[32], w3[32][32][3][3], b3[32], wh[2][32],
 * bh[2].  Training inputs are bfloat16 bit patterns in the rearranged layout,
 * [n][8][24][24]; targets FP32 [n][2].  All device pointers belong to the
 * caller.  The gate is not in the paper. */

/* He-uniform initialisation from `seed` (zero biases, Adam state reset). */
skm_status skm_cnn_init(skm_ctx* ctx, uint64_t seed);
/* Copy the 20898 master parameters in (resets Adam) or out (host arrays). */
skm_status skm_cnn_set_weights(skm_ctx* ctx, const float* host_weights, int32_t n);
skm_status skm_cnn_get_weights(skm_ctx* ctx, float* host_weights, int32_t n);
/* Decision thresholds in dB (see above). */
skm_status skm_cnn_set_thresholds(skm_ctx* ctx, double tau1, double tau2);
/* Weight file: "SKMGATE1", uint32 version 2, uint32 20898, 2 x uint32 0,
 * float32 tau1, tau2, 20898 float32 weights; little endian. */
skm_status skm_save_cnn(skm_ctx* ctx, const char* path);
skm_status skm_load_cnn(skm_ctx* ctx, const char* path);
/* Network inputs of every lost block of a frame (received pixels only),
 * [n][8][24][24] bfloat16 bits in lost-cell raster order; SKM_EINVAL if
 * cap < number of lost blocks. */
skm_status skm_cnn_inputs(skm_ctx* ctx, const uint8_t* d_frame, const uint8_t* d_mask,
                          int32_t width, int32_t height, int32_t stride, const skm_params* params,
                          uint16_t* d_inputs, int32_t cap, int32_t* n_lost, void* hip_stream);
/* Predictions d_out[n][2] for n inputs (training-path forward). */
skm_status skm_cnn_forward(skm_ctx* ctx, const uint16_t* d_inputs, int32_t n, float* d_out,
                           void* hip_stream);
/* Mean squared error over the batch and both outputs and its gradient with
 * respect to the master parameters (copied to host_grad[20898]). */
skm_status skm_cnn_gradients(skm_ctx* ctx, const uint16_t* d_inputs, const float* d_targets,
                             int32_t n, float* host_grad, float* loss, void* hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr on a
 * batch; `loss` (host, optional) receives the batch loss before the step. */
skm_status skm_cnn_train_step(skm_ctx* ctx, const uint16_t* d_inputs, const float* d_targets,
                              int32_t n, float lr, float* loss, void* hip_stream);
/* Gate predictions (g1, g2) of the last SKM_MODE_CNN frame, per lost block in
 * lost-cell raster order (entries of blocks the gate did not see are stale). */
skm_status skm_cnn_last_predictions(skm_ctx* ctx, float* host, int32_t cap);

/* Batch: conceal n independent frames (device buffers), each with its own
 * geometry and parameters (block sizes may differ).  Work starts after the
 * work already enqueued on hip_stream and is complete (every frame) when the
 * call returns.  Per frame: `n_lost`, `rounds` and `status` are written; the
 * call returns the first non-OK status, after finishing every frame it could.
 * Two launch modes (SKM_OPT_BATCH_MODE):
 *  1 (default), batched kernels: frames of equal size and parameters form a
 *    group whose pipeline is one launch per stage over the (frame, lost
 *    block) items of all its frames -- loss geometry, then per round the
 *    context statistics or the learned gate (persistent workgroups), the
 *    estimation kernel (one workgroup per item), HQL and the end-of-round
 *    bookkeeping -- with every frame's rounds and results as if it were
 *    concealed alone.  A group's launches are replayed from a captured
 *    hipGraph while the launch shapes repeat.  Up to SKM_OPT_BATCH_STREAMS
 *    groups run at once on their own streams.  The estimation variant and
 *    gate grid of a group come from the tile table (skm_autotune), else from
 *    SKM_OPT_EST_VARIANT and SKM_OPT_GATE_GRID.
 *  0, frame pipelines: frames are spread over up to SKM_OPT_BATCH_STREAMS
 *    frame slots, each with its own workspace, stream and captured graph of
 *    one frame's pipeline.
 * Results are bitwise those of skm_conceal_device in both modes.
 * Not in the paper: batching is an implementation layer around the
 * per-frame method (Sec. "Reconstruction framework"). */
typedef struct skm_frame_desc {
  const uint8_t* frame;        /* device, stride-pitched uint8 plane          */
  const uint8_t* mask;         /* device, same pitch, nonzero = lost          */
  uint8_t* out;                /* device, same pitch; may alias frame         */
  int32_t width, height, stride;
  const skm_params* params;    /* host pointer, read during the call          */
  skm_block_info* info;        /* device, optional                            */
  float* xhat;                 /* device, optional                            */
  int32_t cap;                 /* capacity of info / xhat in blocks           */
  int32_t n_lost;              /* out */
  int32_t rounds;              /* out */
  int32_t status;              /* out: skm_status of this frame               */
  int32_t reserved;
} skm_frame_desc;
skm_status skm_conceal_batch(skm_ctx* ctx, skm_frame_desc* frames, int32_t n, void* hip_stream);

/* Launch configuration (library-level, not the method's parameters). */
enum {
  SKM_OPT_GRAPHS = 1,         /* 1 (default): replay captured hipGraphs; 0: eager */
  SKM_OPT_BATCH_STREAMS = 2,  /* frames in flight in skm_conceal_batch, 1..8 (4)  */
  SKM_OPT_GATE_GRID = 3,      /* workgroups of the CNN gate kernel, multiple of 8
                                 in 8..4096 (1280: five per CU are resident)      */
  SKM_OPT_HQL_GRID = 4,       /* most workgroups of the HQL kernel, 1..1024; 0
                                 (default): as many as 1 GiB of scratch per frame
                                 slot holds, 128..1024 by geometry                */
  SKM_OPT_BATCH_MODE = 5,     /* skm_conceal_batch: 1 (default) batched kernels per
                                 group of equal frames, 0 frame pipelines         */
  SKM_OPT_EST_VARIANT = 6,    /* batched estimation kernel variant: -1 (default)
                                 the geometry's first; 0: compile-time unit offsets
                                 of B 16 / ring 4 / window 24 (6 candidates per
                                 thread); 1, 2, 3: 6, 9, 17 candidates per thread
                                 (variants too small for the geometry are replaced
                                 by its first).  Setting it, or SKM_OPT_GATE_GRID,
                                 clears the tile table                           */
  SKM_OPT_GROUP_SPLIT = 7     /* batched mode: a group's frames are split into this
                                 many sub-groups of contiguous frames, each on its
                                 own stream, so that their stages overlap, 1..8 (1) */
};
skm_status skm_set_option(skm_ctx* ctx, int32_t option, int64_t value);
skm_status skm_get_option(skm_ctx* ctx, int32_t option, int64_t* value);

/* Autotuner: times skm_conceal_batch on these frames under each launch
 * configuration -- batched mode with every estimation variant of the first
 * frame's geometry, gate grids 640, 1280, 2560 and 3840 (CNN mode) and group
 * splits 1, 2 and 4, and
 * frame pipelines on 1, 2, 4 and 8 streams with gate grids 640, 1280 and 2560
 * (CNN mode); graphs on and off -- keeping the best of `reps` runs each.  The
 * winner's batch mode, streams and graph use are set on the context; in
 * batched mode its estimation variant and gate grid are kept in the tile
 * table under the first frame's (block, ring, window).  The frames are
 * concealed several times.  best_ms (optional) receives the best batch time. */
skm_status skm_autotune(skm_ctx* ctx, skm_frame_desc* frames, int32_t n, int32_t reps,
                        double* best_ms);

/* Tuning cache as JSON: {"version": 1, "batch_mode", "batch_streams",
 * "group_split", "graphs", "gate_grid", "tiles": [{"block", "ring", "window", "est_variant",
 * "gate_grid", "batch_ms"}, ...]}.  Save writes the context's options and
 * tile table; load validates every field (SKM_EINVAL on a missing or
 * out-of-range one, the context unchanged) and replaces them. */
skm_status skm_autotune_save(skm_ctx* ctx, const char* path);
skm_status skm_autotune_load(skm_ctx* ctx, const char* path);

/* Kernel timing for measurement tools (not needed for concealment).  While
 * enabled, the context brackets every launch of its per-block estimation
 * kernel (the kernel that stages the search window, computes the distances,
 * weights and weighted averages) with a HIP event pair on the stream that
 * launch uses; while enabled, frames are launched eagerly (no graph
 * replay).  Each frame's pairs are read when the frame completes;
 * skm_profile_read returns the summed elapsed time in milliseconds and the
 * number of launches since the last read, and resets both.  Either pointer
 * may be NULL. */
skm_status skm_profile_enable(skm_ctx* ctx, int32_t enable);
skm_status skm_profile_read(skm_ctx* ctx, double* total_ms, int32_t* launches);

/* Message of the last error on the calling thread ("" if none). */
const char* skm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SKMMSE_H */
