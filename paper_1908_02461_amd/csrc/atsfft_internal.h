// Internal types shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace atsfft {

constexpr int kMaxLoops = 32;        // L_loc, L_est <= 31
constexpr int kMaxProbe = 32;        // P_max <= 32
constexpr int kBucketThreads = 1024; // one workgroup per bucket array
constexpr int kBucketMaxPer = 16;    // bucket values per thread: B^ndim <= 16384
constexpr int kSmallBucketThreads = 256;  // k_bucket workgroups for arrays of at most kSmallBuckets
constexpr uint32_t kSmallBuckets = 4096;
constexpr int kHashThreads = 256;    // hash workgroup: 64 buckets x 4 wrap groups
constexpr int kSlabs = 8;            // address slabs of a signal, one per XCD
constexpr int kVoteThreads = 256;
constexpr int kEstThreads = 256;
constexpr int kEstGroups = 8;          // estimate workgroups per signal (more for small batches)
constexpr uint32_t kEstRankMax = 1024; // located sets up to this size are sorted by rank
constexpr int kGatherThreads = 1024;  // adjoint gather: threads per block
constexpr int kGatherPer = 16;        // addresses per thread and pass
constexpr size_t kGatherLdsBytes = 65536;  // adjoint gather: most LDS for a staged bucket adjoint
constexpr int kRowTaps = 8;                // 2D row hash: column wraps per thread, at most
constexpr uint32_t kRowBytes = 64u << 10;  // 2D row hash: largest row staged in LDS
constexpr int kMaxOut = 16384;
constexpr uint32_t kBigMax = 1024;  // 2D bucket arrays in device memory: largest B per axis
// fixed device workspace of atsfft_execute_batched_noalloc (bytes per device)
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

enum : uint32_t {
  kSigTruncated = 1,
  kSigNotConverged = 2,
  kSigSaturated = 4,
  kSigEmpty = 8,
  kSigRetried = 16,
  kSigProbeTimeout = 32,
  kSigBadLength = 64,
};

enum : int { kPhaseProbe = 0, kPhaseLoc = 1, kPhaseEst = 2 };
constexpr int kPassIter = 32;  // draw iterations of residual-test pass p start at 32 p

// Per-signal control block of the adaptive probe and the vote (device memory).
struct SigState {
  int32_t B;        // bucket count (per axis) of the next probe iteration
  int32_t k_prev;   // previous local-maximum count
  int32_t done;     // probe finished
  int32_t B_star;   // bucket count of the location and estimation loops
  int32_t khat;     // probed sparsity
  uint32_t status;  // ATSFFT_SIG_* bits
  uint32_t visited; // bit log2(B) set once B was probed
  int32_t n_probe;  // probe iterations run
  uint32_t count;   // |S|, appended by the vote
  int32_t pass;     // location/estimation pass of the residual test (draw iterations + 32 pass)
  double res_ratio; // E_res / E_tot of the last pass (residual test)
  uint32_t round_blocks;  // probe workgroups of the current round that have recorded their count
  uint32_t loc_loaded;    // location-loop k_bucket workgroups that have read their partials (all passes)
  int32_t pad[2];
};
static_assert(sizeof(SigState) == 64, "SigState layout");

struct ProbeRec {
  int32_t B, k, dec, pad;
  double T;
  double pad2;
};
static_assert(sizeof(ProbeRec) == 32, "ProbeRec layout");

// Workspace layout: one slice of `slice` bytes per signal; the fields are
// byte offsets inside a slice (and strides between loops).
struct Layout {
  size_t slice;
  size_t state, hist, yprobe, ymain, ymain_loop, tloc, jcount;
  size_t jbits, jbits_loop, jlist, jlist_loop, S, Ssort, tape, bflag, resid;
  size_t total;
};

// Everything a kernel needs, passed by value.
struct KParams {
  uint64_t seed;
  uint32_t n, logn, ndim, Bc_max;
  uint32_t B0, B_max, alpha_probe, alpha;
  uint32_t L_loc, L_est, T_vote, P_max, d, gamma, max_out, fixed;
  uint32_t fixed_B, fixed_k;
  uint32_t tile_slots;  // probe hash: most tile slots per slab and level
  uint32_t hash_loops;  // main-pass loops per hash workgroup (1D: 1..3)
  uint32_t vote_blocks;  // vote workgroups per (loop, signal)
  uint32_t rows2d_ok;    // 2D main-loop hash by rows allowed: 0 no, 1 per bucket row, 2 streamed (plan)
  uint32_t rows2d;       // the form this launch sequence uses (0, 1 or 2)
  uint32_t stream_rows;  // streamed form: rows per workgroup
  uint32_t gather_lds;   // adjoint gather: most LDS bytes for a staged bucket adjoint (0: none)
  uint32_t gather_blocks;  // adjoint gather: most workgroups per signal (the rest by grid stride)
  uint32_t probe_first;  // first probe round: every level with B (per axis) up to this
  uint32_t probe_step;   // probe levels per later round
  uint32_t probe_slabs;  // 1D probe levels: address slabs (1 or kSlabs), each a partial per bucket
  uint32_t probe_levels;               // bucket counts B0 * 2^i, i < probe_levels
  uint32_t probe_spin;   // sleeps before the probe control stops waiting for a level's count
  int32_t probe_drop;    // test hook: probe level whose count is never recorded (-1: none)
  uint64_t probe_off[kMaxProbe];       // complex offset of level i's bucket arrays in the probe area
  double q, neg_log1mq, noise_rate, rho;
  double res_tol;        // residual test: re-run at 2 B_star above this E_res / E_tot (0: off)
  uint32_t res_retries;  // most re-runs
  uint32_t res_reach;    // model reach in buckets to each side of a frequency's own
  uint32_t pass;         // the pass this launch runs (signals of other passes skip)
  uint32_t comp;         // FP32 fold sums compensated (Neumaier), slab partials added in FP64
  uint32_t big;          // 2D bucket arrays above the LDS-resident size: DFTs and cutoffs in device memory
  uint32_t lds_cap;      // largest bucket array (B^ndim) k_bucket holds in LDS
  uint32_t n_cu;         // compute units of the device
  uint32_t est_wait;     // main k_bucket: estimation loops read their partials after the signal's
                         // location loops have (set for launches whose whole grid is resident)
  uint32_t cut_ties;     // test hook: location loops always take the tie-aware cutoff path
  uint32_t one_slab_logn;  // 1D main-pass hash: signals of length at most 2^this as one address slab (0: none)
  uint32_t pad_kp;
  uint32_t main_slots;   // main-pass hash: tile slots (workgroups) per slab and loop group (0: by batch)
  const void *G;       // window taps, plan precision
  const void *Ghat;    // G'(o) tables, plan precision
  int64_t tab[128];    // [4][32] element offsets by log2 B: probe taps, main taps, main G'(o),
                       // main G'(q) for |q| <= (reach + 1) n/B (residual test); in the
                       // kernel arguments, one scalar load from the offset
  uint8_t *ws;
  Layout lay;
  const void *x;
  int64_t x_sig;       // complex elements per signal
  const int64_t *x_off;    // per-signal element offsets into x (device), or null: sig * x_sig
  const int32_t *sig_map;  // per-signal index in the caller's batch (device), or null: sig
  int64_t *locs;
  void *vals;
  int32_t *count;
  int32_t *khat;
  uint32_t *status;
  // uneven batches with device-side lengths: ns[sig] is signal sig's length
  // and devP[log2 ns[sig]] the parameters of that length (written into the
  // workspace by k_dev_setup), for log2 lengths dev_lg_lo..dev_lg_hi; null
  // otherwise
  const struct KParams *devP;
  const int64_t *ns;
  uint32_t dev_lg_lo, dev_lg_hi;
};
static_assert(sizeof(KParams) % 8 == 0, "KParams is copied in 8-byte words");

// Host-side launchers (atsfft_kernels.hip).
// mark(ctx, i) is called after stage i's launches are enqueued (i = 0 before
// the first launch; 1 probe, 2 main hash, 3 main bucket DFTs, 4 vote,
// 5 estimate); it may record an event on the stream.  May be null.
typedef void (*StageMark)(void *ctx, int stage);
hipError_t launch_execute(const KParams &P, int dtype, int batch, hipStream_t s, StageMark mark, void *ctx);
// One launch sequence over an uneven 1D batch whose lengths are on the device
// (P.ns, P.devP set; tmpl: the plan's per-length parameters, device memory,
// one per log2 length from P.dev_lg_lo).
hipError_t launch_execute_dev(const KParams &P, const KParams *tmpl, int dtype, int batch, hipStream_t s);
hipError_t launch_window_hat(const double *taps, int64_t w, int64_t n, int64_t c, double *out,
                             hipStream_t s);
hipError_t prepare_kernels(int dtype, int ndim, size_t bucket_smem, size_t est_smem, size_t bwd_smem);
hipError_t launch_backward(const KParams &P, int dtype, int batch, const void *grad_vals, void *grad_x,
                           hipStream_t s);
size_t bwd_smem_bytes(int dtype, uint32_t Bc_max, uint32_t max_out);
size_t bucket_smem_bytes(int dtype, uint32_t Bc_max);
size_t estimate_smem_bytes(uint32_t max_out);
size_t residual_smem_bytes(int dtype, uint32_t Bc_max);
size_t vote_smem_bytes(uint32_t L_loc, uint32_t Bc_max);
size_t big_rows_smem(int dtype, uint32_t B);
size_t big_cols_smem(int dtype, uint32_t B);
// Device address of `device`'s fixed workspace (kScratchBytes), looked up once
// per device; `device` must be the current device on the first call for it.
hipError_t scratch_address(int device, void **ptr);

}  // namespace atsfft
