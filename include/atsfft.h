/*
 * atsfft.h - C ABI of an MI355X (gfx950) implementation of ATSFFT, the
 * adaptive-tuning sparse FFT with sparsity detection of Shi, Yang, Zhang and
 * You (arXiv:1908.02461).
 *
 * The library takes a signal (1D, length n) or an image (2D, N x N) whose
 * spectrum is sparse, probes the unknown sparsity k with the paper's
 * adaptive bucket-count iteration (Sec. III-A, Algorithm 2), locates the
 * significant frequencies by voting over randomly permuted, windowed and
 * folded copies of the input (Sec. II-A and II-B, Algorithm 1), and
 * estimates their coefficients as the median over several estimation loops
 * (the estimator display of Sec. II-B).  The output is the k-sparse
 * approximation x' of the unnormalised DFT, x_hat_f = sum_u x_u omega^{f u},
 * omega = e^{-2 pi i / n} (the DFT display of Sec. II): ascending frequency
 * indices (1D: f; 2D: f1 * N + f2) and their complex values.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device pointers (HIP global memory); all other
 *     pointers are host pointers.
 *   - Complex arrays are interleaved (re, im) in the plan's precision:
 *     ATSFFT_C64 = two floats, ATSFFT_C128 = two doubles.
 *   - 2D images are row-major, x[u * N + v].
 *   - The caller owns every buffer it passes in; the plan owns its window
 *     tables (device memory it allocates and atsfft_destroy frees).
 *   - Execution entry points only enqueue work on `stream` and return; their
 *     return code reports argument and launch errors.  Per-signal outcomes
 *     are the ATSFFT_SIG_* bits written to sig_status_dev.
 *   - No entry point aborts, exits or throws.  A plan may be used by one
 *     stream at a time.
 */
#ifndef ATSFFT_H
#define ATSFFT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum atsfft_status {
  ATSFFT_SUCCESS = 0,
  ATSFFT_EINVAL = 1,        /* invalid descriptor, plan or argument */
  ATSFFT_ENODEVICE = 2,     /* no usable gfx950 device */
  ATSFFT_ENOMEM = 3,        /* device allocation failed */
  ATSFFT_ELAUNCH = 4,       /* a kernel launch or HIP call failed */
  ATSFFT_ENOTSUPPORTED = 5  /* a valid request the library does not provide */
} atsfft_status;

enum { ATSFFT_C64 = 0, ATSFFT_C128 = 1 };

/* Per-signal outcome bits (sig_status_dev). */
enum {
  ATSFFT_SIG_OK = 0,
  ATSFFT_SIG_TRUNCATED = 1,           /* |S| > max_out: count holds |S|, locs/vals unwritten */
  ATSFFT_SIG_PROBE_NOT_CONVERGED = 2, /* the probe hit its iteration limit */
  ATSFFT_SIG_PROBE_SATURATED = 4,     /* the probe wanted a bucket count above B_max */
  ATSFFT_SIG_EMPTY = 8,               /* the probed sparsity is 0: nothing located */
  ATSFFT_SIG_RETRIED = 16,            /* the residual test re-ran location at a larger B */
  ATSFFT_SIG_PROBE_TIMEOUT = 32,      /* a probe level's count never reached the probe control
                                         within its bounded wait: the probe stopped at the last
                                         level it acted on (B_star, khat as that level left them;
                                         EMPTY if none), so B_star and khat are not the method's */
  ATSFFT_SIG_BAD_LENGTH = 64          /* atsfft_execute_uneven_dev: the signal's length is not a
                                         power of two in [n_min, n]; nothing ran (also EMPTY) */
};

/* Descriptor flags. */
enum {
  ATSFFT_FLAG_FIXED_B = 1, /* skip the probe: bucket count fixed_B, khat = fixed_k (Algorithm 1) */
  ATSFFT_FLAG_PROFILE = 2, /* record stage timing events on every execute (atsfft_profile_read) */
  ATSFFT_FLAG_COMPENSATED = 4, /* C64: Neumaier-compensated FP32 fold sums (the product's rounding
                                  error from an fma), slab partials added in FP64; no effect for C128 */
  ATSFFT_FLAG_GRAPH = 8        /* atsfft_execute_batched/atsfft_execute capture their launches into a
                                  HIP graph once per call shape (batch and the seven buffer pointers;
                                  the last 64 shapes are kept) and replay it on the caller's stream;
                                  the buffers' contents may change between calls.  Not with
                                  ATSFFT_FLAG_PROFILE (EINVAL).  The plan's first call of a shape
                                  captures on a stream of its own, so that call must not come from a
                                  thread that is capturing another stream. */
};

/* Stages timed under ATSFFT_FLAG_PROFILE, in order. */
enum {
  ATSFFT_STAGE_PROBE = 0,       /* control init and the adaptive probe iterations */
  ATSFFT_STAGE_HASH_MAIN = 1,   /* permute/window/fold of the location and estimation loops */
  ATSFFT_STAGE_BUCKET_MAIN = 2, /* their bucket DFTs and the location-loop cutoffs */
  ATSFFT_STAGE_VOTE = 3,        /* reverse hash and vote */
  ATSFFT_STAGE_ESTIMATE = 4,    /* estimation and medians */
  ATSFFT_NUM_STAGES = 5
};

/*
 * Plan descriptor.  atsfft_default_desc fills every knob; fields set to the
 * defaults reproduce the readings documented with the library.
 *
 *   ndim, n      1 (length n) or 2 (N x N image, n = N); n a power of two,
 *                1D: 2^6 <= n <= 2^30; 2D: 2^4 <= N <= 2^15.
 *   dtype        ATSFFT_C64 or ATSFFT_C128 (input, values and arithmetic).
 *   max_out      capacity of locs/vals per signal, 1 <= max_out <= 16384.
 *   seed         key of the counter-based SplitMix64 draws of (sigma, tau)
 *                (Definition 1's random spectral permutation): the loop of
 *                phase p (0 probe, 1 location, 2 estimation), iteration i
 *                (probe level, or loop index within its phase) and axis a of
 *                signal s (its index in the call) takes r = the SplitMix64
 *                output at index ((s * 4 + p) * 256 + i) * 2 + a, i.e. the
 *                variant-13 finaliser of seed + (index + 1) * 0x9E3779B97F4A7C15
 *                (mod 2^64); sigma = (r mod n) | 1, tau = (r >> 32) mod n.
 *                The loop samples x[(sigma * t + tau) mod n] for the taps
 *                t in [-w/2, w/2).
 *   B0, B_max    first and largest bucket count per axis (powers of two);
 *                B_max^ndim complex values must fit the device's LDS twice.
 *   alpha_probe, alpha   window length factors (w = alpha * B, capped at n),
 *                even, >= 2.
 *   L_loc, L_est location and estimation loop counts (L_est odd, <= 31;
 *                L_loc <= 31); T_vote in [1, L_loc] is the vote threshold.
 *   P_max        probe iteration limit (<= 32).
 *   d            cutoff multiplier: each location loop keeps the d * khat
 *                strongest significant buckets.
 *   gamma        occupancy guard of the probe: a local-maximum count k is
 *                acted on only once B^ndim >= gamma * k (0 disables it).
 *   delta        window leakage (the Gaussian's value at the window edge).
 *   q, noise_rate, rho   significance threshold: noise floor from the
 *                q-quantile of |y_hat|^2, c_noise = ln(B^ndim / noise_rate),
 *                and a relative floor rho * max |y_hat|^2.
 *   fixed_B, fixed_k     used with ATSFFT_FLAG_FIXED_B.
 *   max_batch    largest batch passed to atsfft_execute_batched.
 *   n_min        0, or the shortest length (power of two) atsfft_execute_uneven
 *                accepts; the plan then also holds tables for every power of
 *                two in [n_min, n), with B0 and B_max clipped to each length.
 *   res_tol, res_retries   residual test (an addition to the method; the
 *                paper has none).  res_tol = 0 (the default) disables it.
 *                Otherwise, after estimation, each estimation loop's bucket
 *                DFT y_hat is compared with the buckets the located values
 *                predict by Lemma 1 and the fold (each located f adds
 *                X_f omega^{-tau f} G'(q), q = b n/B - sigma f, to its own
 *                bucket and the R = ceil(2 ln(1/delta) / (pi alpha)) buckets
 *                to each side, R <= (B-1)/2); when E_res / E_tot, summed in
 *                FP64 over loops and buckets, exceeds res_tol (a truncated
 *                pass counts as infinite), location and estimation re-run at
 *                2 B_star with fresh draws (iterations offset by 32 per pass),
 *                at most res_retries times (<= 7), while 2 B_star <= B_max.
 *                Re-run signals carry ATSFFT_SIG_RETRIED.  With FIXED_B the
 *                re-runs may grow past fixed_B up to B_max.
 */
typedef struct atsfft_desc {
  int32_t ndim;
  int32_t dtype;
  int64_t n;
  int64_t max_out;
  uint64_t seed;
  uint32_t flags;
  int32_t max_batch;
  int64_t B0;
  int64_t B_max;
  int32_t alpha_probe;
  int32_t alpha;
  int32_t L_loc;
  int32_t L_est;
  int32_t T_vote;
  int32_t P_max;
  int32_t d;
  int32_t gamma;
  double delta;
  double q;
  double noise_rate;
  double rho;
  int64_t fixed_B;
  int64_t fixed_k;
  int64_t n_min;
  double res_tol;
  int32_t res_retries;
  int32_t pad0;
} atsfft_desc;

typedef struct atsfft_plan_s *atsfft_plan_t;

/* Fill *d with the defaults for (ndim, n, dtype).  Host only, no device use. */
atsfft_status atsfft_default_desc(atsfft_desc *d, int32_t ndim, int64_t n, int32_t dtype);

/*
 * Create a plan on the current HIP device: validates *d synchronously,
 * builds the window tables of every bucket count the probe may visit (the
 * flat window of Sec. II-A-2 generated in FP64, stored in the plan's
 * precision) and keeps them until atsfft_destroy.  On error *out is NULL.
 * Errors: ATSFFT_EINVAL, ATSFFT_ENODEVICE, ATSFFT_ENOMEM, ATSFFT_ELAUNCH.
 *
 * Launch-shape settings, read from the environment when a plan is created
 * (for measurement; the defaults are the measured best on gfx950, and none of
 * them changes a result beyond the order of floating-point sums):
 *   ATSFFT_HASH_LOOPS    1D main loops per hash workgroup, 1..3 (3)
 *   ATSFFT_MAIN_SLOTS    main-loop hash workgroups per address slab and loop
 *                        group, 1..64 (64 for batches up to 64 signals, else 32)
 *   ATSFFT_TILE_SLOTS    probe hash workgroups per slab and level, at most,
 *                        1..64 (32; at least 4 per compute unit over the batch)
 *   ATSFFT_PROBE_SLABS   1D probe levels: address slabs, 1 or 8 (1)
 *   ATSFFT_ONE_SLAB_MAX_N  1D main-loop hash: lengths up to this power of two
 *                        hashed as one address slab instead of 8 (2^21 when
 *                        alpha <= 8, else none; 0: none)
 *   ATSFFT_VOTE_BLOCKS   vote workgroups per candidate loop (128 / batch, >= 32;
 *                        2D: 256 / batch, >= 64)
 *   ATSFFT_PROBE_FIRST   the first probe launch covers B up to this (2048)
 *   ATSFFT_PROBE_STEP    probe levels per later launch, 1..32 (2)
 *   ATSFFT_ROWS2D        2D main-loop hash: 0 slab gather, 1 per bucket row,
 *                        2 rows streamed once; only lowers the plan's form (2)
 *   ATSFFT_STREAM_ROWS   rows per workgroup of the streamed 2D hash, 1..64 (2)
 *   ATSFFT_GATHER_LDS    0: the adjoint gather reads bucket adjoints from
 *                        device memory instead of staging them in LDS
 *   ATSFFT_GATHER_BLOCKS adjoint gather workgroups per signal, 1..1024
 *                        (1024); the rest of a signal by grid stride
 *   ATSFFT_PROBE_SPIN    sleeps (s_sleep 2 each) the probe control waits for
 *                        a level's count still in flight before it gives up
 *                        with ATSFFT_SIG_PROBE_TIMEOUT, 0..2^24 (2^20)
 *   ATSFFT_PROBE_DROP_LEVEL  test hook: the probe level whose count is never
 *                        recorded, so that the wait gives up (unset: none)
 *   ATSFFT_CUTOFF_TIES   test hook, 1: the location loops' top-num cutoff
 *                        always takes its path for buckets tied at the cut
 *                        (taken in index order), which otherwise runs only
 *                        when more buckets equal the cut value than it takes
 */
atsfft_status atsfft_plan(atsfft_plan_t *out, const atsfft_desc *d);

/* Bytes of device workspace atsfft_execute_batched needs for `batch` signals. */
atsfft_status atsfft_workspace_size(atsfft_plan_t plan, int32_t batch, size_t *bytes);

/*
 * Algorithm 2 on `batch` signals of the plan's size, stored back to back in
 * x_dev ([batch][n] or [batch][N][N]).  Outputs, all device memory:
 *   locs_dev       int64 [batch][max_out], ascending located frequencies;
 *   vals_dev       complex [batch][max_out], their estimated coefficients;
 *   count_dev      int32 [batch], |S| (may exceed max_out: TRUNCATED);
 *   khat_dev       int32 [batch], the probed sparsity;
 *   sig_status_dev uint32 [batch], ATSFFT_SIG_* bits.
 * Entries past count are left unwritten.  ws_dev must hold
 * atsfft_workspace_size(plan, batch) bytes; its contents on entry do not
 * matter and on return hold the trace read by atsfft_trace_read.
 * Errors: ATSFFT_EINVAL (null pointer, batch outside [1, max_batch], ws too
 * small), ATSFFT_ELAUNCH.
 */
atsfft_status atsfft_execute_batched(atsfft_plan_t plan, int32_t batch, const void *x_dev,
                                     int64_t *locs_dev, void *vals_dev, int32_t *count_dev,
                                     int32_t *khat_dev, uint32_t *sig_status_dev, void *ws_dev,
                                     size_t ws_bytes, hipStream_t stream);

/*
 * Algorithm 2 on `batch` signals of different lengths (powers of two in
 * [n_min, n] of the plan; 2D: sides) packed in x_dev.  offsets and ns are
 * HOST arrays [batch]: signal i starts at complex element offsets[i] of x_dev
 * and has length ns[i] (2D: ns[i] x ns[i] elements).  Outputs are indexed by
 * i exactly as for atsfft_execute_batched, and signal i draws its
 * permutations with signal key i, so a signal gets the same result whatever
 * else the batch holds.  Signals of one length run as one group (one launch
 * sequence per distinct length).  The per-signal tables are staged through a
 * plan-owned pinned buffer; a call waits for the previous call's upload.
 * ws_dev must hold atsfft_workspace_size_uneven(plan, batch, ns) bytes.
 * The adjoint and the trace read do not apply to uneven calls.
 * Errors: ATSFFT_EINVAL (a length the plan does not cover, null pointers,
 * workspace too small), ATSFFT_ENOMEM, ATSFFT_ELAUNCH.
 */
atsfft_status atsfft_execute_uneven(atsfft_plan_t plan, int32_t batch, const void *x_dev, const int64_t *offsets,
                                    const int64_t *ns, int64_t *locs_dev, void *vals_dev, int32_t *count_dev,
                                    int32_t *khat_dev, uint32_t *sig_status_dev, void *ws_dev, size_t ws_bytes,
                                    hipStream_t stream);

/*
 * Algorithm 2 on an uneven 1D batch whose lengths and offsets are DEVICE
 * arrays (int64 [batch]): signal i starts at complex element offsets_dev[i]
 * of x_dev and has length ns_dev[i].  The host reads neither array, so the
 * call is a fixed sequence of kernel launches whatever the lengths (no
 * grouping on the host, no host-to-device copy) and can be captured into a
 * HIP graph (ATSFFT_FLAG_GRAPH replays it; a caller may also capture it into
 * its own graph); the arrays' contents may change between replays.  Every
 * signal runs with the knobs and window tables of its own length, as in
 * atsfft_execute_uneven, and draws with signal key i, so each signal's result
 * equals that call's.  A length that is not a power of two in [n_min, n]
 * gives ATSFFT_SIG_BAD_LENGTH | ATSFFT_SIG_EMPTY for that signal; offsets are
 * the caller's to keep inside x_dev.  Needs a 1D plan with n_min > 0 and
 * res_tol = 0; ws_dev must hold atsfft_workspace_size_uneven_dev(plan, batch)
 * bytes.  The adjoint and the trace read do not apply.
 * Errors: ATSFFT_EINVAL (a plan without this form, ATSFFT_FLAG_PROFILE, batch
 * outside [1, max_batch], null pointers, workspace too small), ATSFFT_ELAUNCH.
 */
atsfft_status atsfft_execute_uneven_dev(atsfft_plan_t plan, int32_t batch, const void *x_dev,
                                        const int64_t *offsets_dev, const int64_t *ns_dev, int64_t *locs_dev,
                                        void *vals_dev, int32_t *count_dev, int32_t *khat_dev,
                                        uint32_t *sig_status_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of atsfft_execute_uneven_dev for `batch` signals: a slice of
   the plan's longest length per signal, whatever the lengths. */
atsfft_status atsfft_workspace_size_uneven_dev(atsfft_plan_t plan, int32_t batch, size_t *bytes);

/* Workspace bytes of atsfft_execute_uneven for the lengths ns (host, [batch]). */
atsfft_status atsfft_workspace_size_uneven(atsfft_plan_t plan, int32_t batch, const int64_t *ns, size_t *bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * atsfft_execute_batched with its workspace in a fixed device array that the
 * library holds on each device it runs on, ATSFFT_NOALLOC_WORKSPACE_BYTES
 * (64 MiB) per device, kept until the process ends.  The call allocates
 * nothing (no hipMalloc, pinned memory, event or graph); the caller passes
 * the input and the outputs exactly as for atsfft_execute_batched and gets
 * the same results.  Every call on one device shares that device's array:
 * calls that overlap on one device (other streams, other threads, other
 * plans) race and give undefined results, and atsfft_trace_read and
 * atsfft_backward do not apply (the workspace is not the caller's).  The
 * array keeps the previous call's contents; the call needs no particular
 * contents on entry.
 * Errors: ATSFFT_EINVAL (a plan with ATSFFT_FLAG_GRAPH or ATSFFT_FLAG_PROFILE,
 * which allocate; batch outside [1, max_batch]; a null pointer; a batch whose
 * atsfft_workspace_size exceeds ATSFFT_NOALLOC_WORKSPACE_BYTES, with the
 * sizes in atsfft_last_error), ATSFFT_ELAUNCH.
 */
#define ATSFFT_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
atsfft_status atsfft_execute_batched_noalloc(atsfft_plan_t plan, int32_t batch, const void *x_dev,
                                             int64_t *locs_dev, void *vals_dev, int32_t *count_dev,
                                             int32_t *khat_dev, uint32_t *sig_status_dev, hipStream_t stream);

/* atsfft_execute_batched with batch = 1. */
atsfft_status atsfft_execute(atsfft_plan_t plan, const void *x_dev, int64_t *locs_dev,
                             void *vals_dev, int32_t *count_dev, int32_t *khat_dev,
                             uint32_t *sig_status_dev, void *ws_dev, size_t ws_bytes,
                             hipStream_t stream);

/*
 * Gradient of a real loss L through the values of the last execute that used
 * ws_dev, at its located frequencies and median choices held fixed (the
 * located set and the medians are piecewise constant in x; on each piece the
 * values are real-linear in x).  Each value is the coordinate-wise median of
 * the estimator display (Sec. II-B): its real part comes from one estimation
 * loop and its imaginary part from one (recorded by the execute).  Inputs:
 *   grad_vals_dev  complex [batch][max_out]: dL/dRe v + i dL/dIm v for each
 *                  value (entries at or past a signal's count are ignored);
 *   ws_dev         the execute's workspace, unchanged since.
 * Output grad_x_dev, complex, the layout of x: dL/dRe x + i dL/dIm x, written
 * in full (zero where no estimation loop samples).  Signals that were EMPTY
 * or TRUNCATED get a zero gradient; after a residual-test re-run the
 * gradient is that of the last pass.  Every address of grad_x is written
 * once, its loops added in order; located frequencies that share a bucket add
 * their bucket cotangents with atomics, so the last bits may vary between
 * calls.  Errors: ATSFFT_EINVAL, ATSFFT_ELAUNCH.
 */
atsfft_status atsfft_backward(atsfft_plan_t plan, int32_t batch, const void *grad_vals_dev,
                              const void *ws_dev, void *grad_x_dev, hipStream_t stream);

/*
 * Debug trace of one signal of the last execute that used ws_dev, copied to
 * host memory after synchronising `stream`.  Fills the scalar fields and,
 * when non-NULL, the arrays (sizes from the plan: Bc = Bm^ndim with Bm the
 * largest bucket count of the location and estimation loops: B_max, or with
 * ATSFFT_FLAG_FIXED_B fixed_B, max(fixed_B, B_max) when res_tol > 0):
 *   probe_B/probe_k/probe_dec  int32 [P_max], probe_T double [P_max];
 *   T_loc double [L_loc], J_count int32 [L_loc];
 *   yhat   complex (plan precision) [L_loc + L_est][Bc] (bucket DFTs at B_star);
 *   J_bits uint32 [L_loc][Bc / 32] (bit b of loop l: bucket b selected).
 */
typedef struct atsfft_trace {
  int32_t B_star, khat, n_probe, count;
  uint32_t status;
  int32_t *probe_B, *probe_k, *probe_dec;
  double *probe_T;
  double *T_loc;
  int32_t *J_count;
  void *yhat;
  uint32_t *J_bits;
  double res_ratio; /* residual test: E_res / E_tot of the last pass (0 when off) */
  int32_t retries;  /* passes re-run at a larger B */
  int32_t pad0;
} atsfft_trace;

atsfft_status atsfft_trace_read(atsfft_plan_t plan, const void *ws_dev, int32_t signal,
                                atsfft_trace *out, hipStream_t stream);

/*
 * Stage durations (milliseconds, HIP events on the execute's stream) summed
 * over every execute since the previous call, and the number of executes.
 * Waits for those executes to finish.  stage_ms has ATSFFT_NUM_STAGES
 * entries.  Without ATSFFT_FLAG_PROFILE it reports zero executes.
 */
atsfft_status atsfft_profile_read(atsfft_plan_t plan, double *stage_ms, int32_t *executes);

/* Release the plan's device tables.  Null is accepted. */
atsfft_status atsfft_destroy(atsfft_plan_t plan);

/* Static description of a status code. */
const char *atsfft_status_string(atsfft_status s);

/* Library version string. */
const char *atsfft_version(void);

/* Last error message recorded on this thread (static storage, never null). */
const char *atsfft_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
