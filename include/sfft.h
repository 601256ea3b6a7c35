/*
 * sfft.h -- C ABI of the MI355X (gfx950) multiscale sparse FFT hot path.
 *
 * The method is sFFT4.0 as analysed in B. Li, Z. Jiang, J. Chen, "On
 * Performance of Multiscale Sparse Fast Fourier Transform Algorithm"
 * (arXiv 2011.05698).  Given a length-N signal whose spectrum is (close to)
 * K-sparse, an execute recovers the K largest coefficients of
 *     xhat_f = (1/N) sum_j x_j exp(-2 pi i f j / N)        (Sec. 2.1, Eq. 2)
 * from a sublinear number of samples.
 *
 * Conventions that hold for every call:
 *   - Every call returns sfft_status; nothing throws across the ABI.
 *   - Pointers named d_* are device (HIP) pointers owned by the caller;
 *     h_* are host pointers owned by the caller.  The library never frees a
 *     caller's buffer.  Plans and batches own their workspace and free it in
 *     sfft_destroy / sfft_batch_destroy.  A plan's read-only tables (window,
 *     window spectrum, twiddles) are shared with the other live plans of the
 *     same N, B, w, loops, delta and dtype on the same device, and freed with
 *     the last of them.
 *   - Execute calls are asynchronous and stream-ordered on `stream` (a
 *     hipStream_t; NULL is the default stream).  Outputs are valid once the
 *     stream has been synchronised.  At most one execute may be in flight
 *     per plan (and per batch): the workspace is per object.
 *   - Parameter and state errors are reported synchronously, before
 *     anything is enqueued.  Kernel launch failures return SFFT_ERR_LAUNCH.
 *     sfft_last_error() returns a thread-local description of the most
 *     recent failure on the calling thread.
 *   - SFFT_ERR_ALLOC: sfft_plan and the batch constructors release whatever
 *     they had allocated and leave *out NULL.  For tests of this path, the
 *     environment variable SFFT_FAIL_ALLOC=n makes the n-th host or device
 *     allocation of such a call (counted from the call's start, on the
 *     calling thread) fail as if memory were exhausted.
 *   - Complex values are interleaved (re, im): float2 for SFFT_C64 and
 *     SFFT_F16X2_SCALED outputs, double2 for SFFT_C128.
 */
#ifndef SFFT_H
#define SFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SFFT_OK = 0,
  SFFT_ERR_PARAM = 1,        /* an argument violates the rules stated at sfft_plan */
  SFFT_ERR_UNSUPPORTED = 2,  /* valid per the paper, but beyond this library's limits */
  SFFT_ERR_ALLOC = 3,        /* device or host allocation failed */
  SFFT_ERR_LAUNCH = 4,       /* a HIP call or kernel launch failed */
  SFFT_ERR_CAPACITY = 5,     /* a workspace exceeds a fixed capacity (sfft_execute_noalloc)  */
  SFFT_ERR_STATE = 6         /* object used in a state that does not allow the call */
} sfft_status;

/* Storage type of the input samples (and, for C128, of all arithmetic). */
typedef enum {
  SFFT_C64 = 0,           /* float2 samples; FP32 window, fold, FFT and recovery        */
  SFFT_C128 = 1,          /* double2 samples; everything in FP64                        */
  SFFT_F16X2_SCALED = 2   /* __half2 samples x_j ~= scale * (re, im); FP32 arithmetic   */
} sfft_dtype;

typedef struct sfft_plan_s* sfft_plan_t;
typedef struct sfft_batch_s* sfft_batch_t;

/* Plan flags. */
#define SFFT_PLAN_HOST_ONLY 1u   /* build host tables only; no device memory, no execute */

/* Optional plan settings; pass NULL to sfft_plan for the defaults below. */
/* How an iteration locates the lone coefficient of a bucket:
 *   SFFT_LOCATE_MULTISCALE -- sFFT4.0 (Sec. 3.2): block by block over R
 *       rounds with multipliers tau_j = floor(N / len_j), a final enumeration;
 *   SFFT_LOCATE_DIRECT -- the two-round location of sFFT3.0 that the paper
 *       sets sFFT4.0 against (Sec. 1, Sec. 3.1: R_m = 2 rounds): offsets tau0
 *       and tau0 + 1, u = round(theta N / 2 pi) mod N (Eq. 16 with tau = 1);
 *       theta in FP64 at N >= 2^24.  Faster, and less robust to collisions
 *       and noise.  Verification and estimation are the same for both. */
typedef enum { SFFT_LOCATE_MULTISCALE = 0, SFFT_LOCATE_DIRECT = 1 } sfft_location;

/* How the loops' findings are combined:
 *   SFFT_COMBINE_SUM -- the iterative framework of sFFT4.0 (Sec. 3.1): B_m
 *       halves per iteration, each iteration first subtracts what earlier ones
 *       recovered, and rec[f] += v;
 *   SFFT_COMBINE_VOTE -- the one-shot framework that Sec. 1 and the opening
 *       of Sec. 3 set against it (several random bucketizations and a vote):
 *       every loop keeps B and w, no loop subtracts, a frequency is kept when
 *       at least half of the loops located it (2 n >= loops), and its value is
 *       the median of its n loop estimates, real and imaginary parts
 *       separately (mean of the two middle values for an even n).  The
 *       workspace grows by (sum of B_m) x loops complex values. */
typedef enum { SFFT_COMBINE_SUM = 0, SFFT_COMBINE_VOTE = 1 } sfft_combine;

typedef struct {
  double delta;     /* window leakage / truncation level, 0 < delta < 0.1 (default 1e-6)   */
  uint64_t seed;    /* SplitMix64 seed of the per-iteration sigma, tau0 draws (default 0)  */
  int32_t dtype;    /* sfft_dtype (default SFFT_C64)                                        */
  int32_t kahan;    /* 1: compensated (Kahan) summation in the fold (default 0)             */
  int32_t b_min;    /* smallest bucket count of late iterations, power of two (default 16) */
  int32_t combine;  /* sfft_combine (default SFFT_COMBINE_SUM)                               */
  double eta;       /* detection floor relative to the strongest bucket (default 1e-4)     */
  double rho;       /* round-to-round magnitude tolerance of a lone bucket (default 0.25)  */
  uint32_t flags;   /* SFFT_PLAN_* bits                                                     */
  uint32_t location; /* sfft_location (default SFFT_LOCATE_MULTISCALE)                      */
} sfft_options;

/* Fills *opt with the defaults. */
void sfft_default_options(sfft_options* opt);

/*
 * sfft_plan -- validate parameters and build a reusable plan.
 *
 * Parameters (the method of Sec. 3; readings of unstated details follow):
 *   N      signal length, a power of two, 2^4 <= N <= 2^30.
 *   K      number of coefficients returned, 1 <= K <= B.
 *   B      buckets of the first iteration, a power of two, 16 <= B <= N/4
 *          (Sec. 2.3: bucket width L = N/B).  Iteration m uses
 *          B_m = max(B >> (m-1), b_min) buckets (Sec. 3.3: B halves);
 *          B_m = B under SFFT_COMBINE_VOTE.
 *   w      window support of the first iteration, B <= w <= N-1; an even w
 *          is rounded up to odd.  Iteration m uses w_m = floor(w B_m / B) | 1.
 *   loops  number of iterations M (Sec. 3.1), 1 <= loops <= 64.
 *   multiscale  the multiscale parameter l: number of blocks per location
 *          step (Sec. 3.2), a power of two, 2 <= l <= 1024.
 *   extension   the extension parameter q (Sec. 3.2): a dyadic rational
 *          (q * 2^16 an integer), q > 0 and l > q + 1 (regions must shrink).
 *   opt    NULL for defaults.
 * Window (Sec. 2.3, Eq. 9-10): width-L boxcar with half-weight edges times a
 * Gaussian that falls to delta at the support edge; its spectrum Ghat is
 * tabulated exactly (FP64) out to L/2 + e, e = ceil of the transition
 * half-width.  The location schedule (Sec. 3.2) and the per-iteration
 * sigma_m (odd) and tau0_m come from SplitMix64(seed).
 * Limits (SFFT_ERR_UNSUPPORTED): B <= 16384 for SFFT_C64/SFFT_F16X2_SCALED,
 * B <= 8192 for SFFT_C128 (the bucket DFT keeps B values in 128 KiB of LDS);
 * at most 47 location steps per iteration.
 * On success *out holds a plan owning its workspace and holding its tables
 * (shared with the live plans that need the same ones).
 */
sfft_status sfft_plan(sfft_plan_t* out, int64_t N, int64_t K, int64_t B, int64_t w, int32_t loops,
                      int32_t multiscale, double extension, const sfft_options* opt);

/*
 * sfft_execute -- the whole method on one signal (Sec. 3.1): for every
 * iteration, HashToBins over its R_m+1 rounds (Lemma 1: permuted gather,
 * window, fold, B-point DFT with the 1/N factor), subtraction of the
 * coefficients recovered so far, singleton detection, multiscale location
 * (Eq. 15-19), verification, median estimation (Eq. 14), dedupe and
 * accumulation; finally the K largest coefficients.
 *   d_x     N samples: float2 (C64), double2 (C128) or __half2 (F16X2_SCALED).
 *   scale   F16X2_SCALED only: the sample value is scale * d_x[j]; ignored otherwise.
 *   d_idx   K int64: recovered frequencies, ascending.
 *   d_val   K complex (float2, or double2 for C128): their values.
 *   d_count 1 int64: number of valid outputs (<= K).
 * Entries of d_idx/d_val beyond *d_count are left untouched.
 */
sfft_status sfft_execute(sfft_plan_t p, const void* d_x, float scale, int64_t* d_idx, void* d_val,
                         int64_t* d_count, void* stream);

/*
 * sfft_execute_noalloc -- sfft_execute for callers that cannot allocate
 * device memory while they run (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results as sfft_execute (bit for bit); the only difference is where the
 * per-signal workspace lives: instead of the plan's own workspace, a static
 * device array of 16 MiB that the library holds on every device it runs on
 * until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); its first call on a device looks
 * up that device's array address once.
 *   SFFT_ERR_CAPACITY  the plan's workspace (sfft_plan_info.workspace_bytes)
 *                      exceeds 16 MiB; nothing is enqueued.
 * Every call on one device shares that device's array, and the array keeps
 * the last call's contents: two calls that overlap in time on one device
 * (different streams, or different host threads without ordering) race and
 * give undefined results.  Calls on one stream are ordered and safe.
 */
sfft_status sfft_execute_noalloc(sfft_plan_t p, const void* d_x, float scale, int64_t* d_idx, void* d_val,
                                 int64_t* d_count, void* stream);

/*
 * sfft_hash_to_bins -- HashToBins alone (Sec. 2.4, Lemma 1, Eq. 13) for all
 * iterations and rounds of the plan, without subtraction:
 *   d_yhat[off_m + j*B_m + i] = (1/N) sum_b y_{m,j}[b] exp(-2 pi i i b / B_m),
 *   y_{m,j}[b] = sum_{|t| <= h_m, t = b mod B_m} G_t x[sigma_m (t - T_{m,j}) mod N].
 * off_m is the prefix sum of (R_k+1) B_k over k < m (sfft_iter_info.y_offset);
 * d_yhat holds sfft_plan_info.yhat_elems complex values (float2, double2 for C128).
 */
sfft_status sfft_hash_to_bins(sfft_plan_t p, const void* d_x, float scale, void* d_yhat, void* stream);

/*
 * sfft_recover -- the reconstruction half of sfft_execute (subtraction,
 * detection, location, estimation, accumulation, top-K) run on
 * caller-supplied bucket values in the sfft_hash_to_bins layout.  d_yhat is
 * read only (the plan copies it into its workspace first).
 */
sfft_status sfft_recover(sfft_plan_t p, const void* d_yhat, int64_t* d_idx, void* d_val, int64_t* d_count,
                         void* stream);

/* Plan-wide facts. */
typedef struct {
  int64_t N, K, B, w;
  int32_t loops, multiscale;
  double extension, delta;
  int32_t dtype, kahan;
  int64_t samples;      /* samples one execute reads: sum_m (R_m+1) w_m (Sec. 2.4 / 3.1 cost) */
  int64_t yhat_elems;   /* complex elements of the sfft_hash_to_bins output                    */
  int64_t rec_capacity; /* capacity of the recovered-coefficient store                        */
  int64_t workspace_bytes; /* device workspace owned by the plan                              */
  uint64_t seed;
} sfft_plan_info;
sfft_status sfft_get_plan_info(sfft_plan_t p, sfft_plan_info* info);

/* Per-iteration facts (m counts from 0).  Arrays are indexed by location
 * step j = 1..R; index 0 holds the reference round (tau = 0, len = 0). */
typedef struct {
  int64_t B, L, w, h, e, R;
  double d_delta;        /* transition half-width in bins (Ghat falls to delta past L/2 + d_delta) */
  uint64_t sigma, sigma_inv, tau0;
  int64_t y_offset;      /* complex-element offset of this iteration in the yhat layout */
  int64_t T[48], tau[48], len[48];
  int32_t last_kind;     /* 1: the last step enumerates positions (multiscale),
                            2: direct phase-to-position conversion (two-round)  */
  int32_t pad;
} sfft_iter_info;
sfft_status sfft_get_iter_info(sfft_plan_t p, int32_t m, sfft_iter_info* info);

/* Copies iteration m's FP64 window G_0..G_h (h+1 values) and spectrum
 * Ghat_0..Ghat_{L/2+e} (L/2+e+1 values) into host buffers (either may be NULL). */
sfft_status sfft_plan_dump_tables(sfft_plan_t p, int32_t m, double* h_window, double* h_ghat);

sfft_status sfft_destroy(sfft_plan_t p);

/*
 * Batches: many signals, each with its own plan (uneven N, K, B, loops are
 * allowed), executed together: one launch per kernel stage for the whole
 * batch, replayed from a HIP graph.  Plans must outlive the batch; a plan
 * may appear several times.  The batch owns the workspace of its signals.
 */
sfft_status sfft_batch_create(sfft_batch_t* out, const sfft_plan_t* h_plans, int32_t n);

/*
 * sfft_execute_batch -- sfft_execute for every signal s of the batch:
 *   h_x[s]    device pointer to signal s (dtype of its plan);
 *   h_scale   per-signal scales (F16X2_SCALED plans) or NULL;
 *   h_idx[s], h_val[s]  device output buffers of K_s entries;
 *   d_count   device array of n int64 counts.
 * The h_* arrays are host arrays of device pointers.  When they differ from
 * the previous call's, the batch re-uploads its descriptor table with a
 * blocking copy before enqueueing; repeated calls with the same buffers only
 * replay the batch's graph on `stream`.  In the stage launches each signal's
 * results equal, bit for bit, what sfft_execute gives for it alone: the
 * launch shapes the library picks by batch size (the recovery's workgroup
 * size among them) split every sum the same way.
 */
sfft_status sfft_execute_batch(sfft_batch_t b, const void* const* h_x, const float* h_scale,
                               int64_t* const* h_idx, void* const* h_val, int64_t* d_count, void* stream);

/*
 * Position-major batches: nsig signals that share one plan (one draw of the
 * permutations sigma_m and offsets tau0_m, Sec. 2.4 and 3.1, applied to
 * every signal) and are stored sample-interleaved, as a multichannel stream
 * is: sample c of signal s is element c * ld + s of d_x (ld >= nsig; an
 * element is one sample of the plan's dtype).  Since every signal gathers
 * the same positions, each tap reads a contiguous run of the row instead of
 * one sample per cache line.  Results are those sfft_execute gives for each
 * signal on its own with the same plan.
 *
 * sfft_batch_create_interleaved -- the plan must outlive the batch.
 * sfft_execute_interleaved --
 *   d_x      device array of N rows of ld elements;
 *   h_scale  host array of nsig scales (F16X2_SCALED plans) or NULL;
 *   d_idx    device int64 array [nsig][K], d_val device array [nsig][K] of
 *            the output value type, d_count device int64 array [nsig].
 * Binding, graph replay and stream ordering are those of sfft_execute_batch
 * (a changed d_x, ld, scale or output pointer re-uploads the descriptor
 * table with a blocking copy; a d_x alignment or ld that changes how many
 * signals a fold lane takes, see fold_lanes, captures the graph again).
 * The fold reads two (complex64) or four (FP16 pairs) adjacent signals per
 * load when d_x is aligned to that many elements and ld, nsig and the number
 * of 64-signal groups are multiples of it; results are the same bits either
 * way.  SFFT_ERR_PARAM for ld < nsig or ld >= 2^32;
 * SFFT_ERR_STATE when a batch of the other kind is passed to either execute
 * call.  sfft_batch_launch_stage, sfft_batch_set_fold_config (unroll only;
 * wg_per_cu is ignored), sfft_batch_autotune and sfft_batch_destroy apply.
 */
sfft_status sfft_batch_create_interleaved(sfft_batch_t* out, sfft_plan_t plan, int32_t nsig);
sfft_status sfft_execute_interleaved(sfft_batch_t b, const void* d_x, int64_t ld, const float* h_scale,
                                     int64_t* d_idx, void* d_val, int64_t* d_count, void* stream);

/*
 * sfft_batch_launch_stage -- enqueue one stage of the batch on `stream`, for
 * timing the stages separately (the sequence fold, bucket DFT, recover is
 * exactly what sfft_execute_batch replays in SFFT_BATCH_STAGES mode):
 *   stage 0: permuted gather + window + fold (HashToBins, Eq. 7, 10, 11)
 *   stage 1: B-point DFT of every round (Eq. 12 with the 1/N factor)
 *   stage 2: recovery (subtraction .. top-K)
 *   stage 3: the whole step as one persistent launch (SFFT_BATCH_FUSED, see
 *            sfft_batch_tuning); SFFT_ERR_UNSUPPORTED when the batch cannot
 *            run it.
 * Uses the buffers bound by the last execute of the batch (SFFT_ERR_STATE if
 * none).
 */
sfft_status sfft_batch_launch_stage(sfft_batch_t b, int32_t stage, void* stream);

/*
 * Launch shape of the fold stage (the permuted gather): taps fetched per
 * thread before use (unroll: 8, 16 or 24), and a cap on resident workgroups
 * per compute unit (wg_per_cu: 0 for none, else 2..8) that bounds how many
 * signals are gathered at once.  Shapes never change results.
 */
typedef struct {
  int32_t unroll;
  int32_t wg_per_cu;
  double fold_ms;   /* filled by sfft_batch_autotune: mean fold time of the winner */
} sfft_fold_config;

/* SFFT_ERR_PARAM for a shape outside the list above (fold_ms is ignored).
 * The batch form, when the batch already holds a captured graph, waits for
 * that batch's last replay to finish (an event recorded after it on the
 * caller's stream; other work on the device is not waited for), drops the
 * graph, and captures again on the next sfft_execute_batch; bound buffers
 * stay bound. */
sfft_status sfft_plan_set_fold_config(sfft_plan_t p, const sfft_fold_config* cfg);
sfft_status sfft_batch_set_fold_config(sfft_batch_t b, const sfft_fold_config* cfg);

/*
 * How a batch runs (sfft_batch_get_tuning / sfft_batch_set_tuning):
 *   SFFT_BATCH_STAGES  three launches replayed from a graph: the fold stage
 *                      (taps in flight fold_unroll = 8, 16 or 24; residency
 *                      cap fold_wg_per_cu = 0 or 2..8, per-signal layout
 *                      only), the bucket DFTs (fft_group_points = 1024, 2048
 *                      or 4096 points per workgroup when B is smaller), and
 *                      the recovery;
 *   SFFT_BATCH_FUSED   one persistent launch (after a small kernel that
 *                      clears its counters), also replayed from a graph: the
 *                      workgroups take fold tiles and per-signal finish items
 *                      (bucket DFTs, then recovery) from a queue ordered in
 *                      chunks of fused_chunk signals (per-signal layout) or
 *                      groups of 64 signals (position-major); a signal's
 *                      finish item waits for its fold tiles, so the recovery
 *                      of early signals overlaps the gather of later ones.
 *                      Available when every round of every plan (B_m complex
 *                      values) fits in 78,848 bytes: B <= 8192 for complex64
 *                      and FP16 storage, B <= 4096 for complex128.  A wait
 *                      that has not ended after a bounded number of polls
 *                      (seconds) gives up: that signal's count reads -2.
 * Every STAGES setting gives bit-identical results; FUSED runs the bucket
 * DFT as the LDS radix-2^2 pass for every B, so its results agree with
 * them to rounding.  Setting a tuning waits for the batch's last replay and
 * drops its graph, like sfft_batch_set_fold_config.
 * SFFT_ERR_PARAM for a value outside the lists, or (FUSED) fused_chunk
 * outside 1 .. the number of signals (or groups); SFFT_ERR_UNSUPPORTED for
 * FUSED where it is not available.
 */
typedef enum { SFFT_BATCH_STAGES = 0, SFFT_BATCH_FUSED = 1 } sfft_batch_mode;
typedef struct {
  int32_t mode;             /* sfft_batch_mode */
  int32_t fused_chunk;      /* FUSED: signals (per-signal layout) or groups of 64 signals per chunk */
  int32_t fold_unroll;      /* STAGES: fold taps in flight */
  int32_t fold_wg_per_cu;   /* STAGES: fold residency cap */
  int32_t fft_group_points; /* STAGES: bucket-DFT points per workgroup */
  int32_t fused_available;  /* read only: 1 if the batch can run FUSED */
  double step_ms;           /* read only: one step of this configuration, as sfft_batch_autotune timed it */
  int32_t fold_lanes;       /* STAGES, position-major: adjacent signals per fold lane, 1, 2 (complex64,
                               FP16 pairs) or 4 (FP16 pairs), or 0 for as many as the bound input allows
                               (the default).  L > 1 needs the input aligned to L elements and ld, the
                               signal count and the number of 64-signal groups multiples of L; otherwise
                               the fold takes the largest allowed count below L.  Read back: the count the
                               bound input runs with (1 for a per-signal batch; before the first
                               execute, the setting) */
} sfft_batch_tuning;
sfft_status sfft_batch_get_tuning(sfft_batch_t b, sfft_batch_tuning* t);
sfft_status sfft_batch_set_tuning(sfft_batch_t b, const sfft_batch_tuning* t);

/*
 * sfft_batch_autotune -- choose how the bound batch (buffers bound by a prior
 * execute) runs, by timing launches on `stream`: first the fold stage for
 * every unroll x wg_per_cu candidate, then the bucket DFT for every
 * fft_group_points candidate, then one whole step of the three stages
 * against the fused launch at four chunk sizes; the fastest step wins.
 * *best receives the fold choice (fold_ms: its mean fold time, as timed when
 * the choice was made);
 * sfft_batch_get_tuning gives the whole choice.  The choice is kept for the
 * life of the process per batch shape (dtype, Kahan, layout, number of
 * signals and every plan's N, B, w, loops, l and combine): a later call on a
 * batch of the same shape applies it without timing.  Blocks until the
 * timing launches finish; they rewrite the batch's workspace and outputs
 * with the values an execute gives.  The graph is captured again by the
 * next execute.  SFFT_ERR_STATE when no buffers are bound.
 */
sfft_status sfft_batch_autotune(sfft_batch_t b, void* stream, sfft_fold_config* best);

sfft_status sfft_batch_destroy(sfft_batch_t b);

const char* sfft_status_string(sfft_status s);
const char* sfft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_H */
