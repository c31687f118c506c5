// gfx950 kernels of ATSFFT (arXiv:1908.02461): the permute/window/fold hash,
// the LDS-resident bucket DFT with significance threshold, local-maximum count
// and adaptive-B control, the top-num cutoff, the vote over inverse-permuted
// buckets, and median value estimation.
//
// One batch runs as a fixed sequence of launches on one stream:
//   k_init                      per-signal control blocks
//   rounds of { k_hash(probe), k_bucket(probe) }
//                               adaptive probe (Sec. III-A), several bucket
//                               counts per round; the last bucket workgroup
//                               of a signal's round applies the B-update rule
//   k_hash(main)                L_loc + L_est loops at the probed B
//   k_bucket(main)              bucket DFTs; location loops also select J
//   k_vote                      located set S (reverse hash, threshold)
//   k_estimate                  sort S, estimate and take medians
//   [k_residual, k_retry_control and re-run passes, with the residual test]
// Data-dependent sizes (B, |S|) stay on the device: grids are sized for the
// largest case and workgroups past a signal's actual extent exit at once.
// The adjoint adds k_bwd_bucket and k_bwd_gather.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "atsfft_internal.h"

namespace atsfft {

// ---------------------------------------------------------------- types ----

template <typename R> struct CT;
template <> struct CT<float> {
  using C = float2;
  using K = uint32_t;
};
template <> struct CT<double> {
  using C = double2;
  using K = unsigned long long;
};

__device__ __forceinline__ uint32_t key_of(float v) { return __float_as_uint(v); }
__device__ __forceinline__ unsigned long long key_of(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ float val_of(uint32_t k) { return __uint_as_float(k); }
__device__ __forceinline__ double val_of(unsigned long long k) { return __longlong_as_double((long long)k); }

__device__ __forceinline__ void sincos_pi(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincos_pi(double x, double *s, double *c) { sincospi(x, s, c); }

// ---------------------------------------------------------------- draws ----

// SplitMix64 (Steele, Lea, Flood 2014): output `index` of the stream seeded
// with `seed` is the variant-13 finaliser of seed + (index + 1) * gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Draw {
  uint32_t sigma, tau;
};

// One loop's permutation (Definition 1) for the key (signal, phase, iteration,
// axis): sigma odd from the low word, tau from the high word, both mod n.
// The signal key is the signal's index in the caller's batch (sig_map when a
// call is split into groups of equal length).
__device__ __forceinline__ Draw draw(const KParams &P, uint32_t sig, int phase, int iter, int axis) {
  const uint64_t key = P.sig_map ? (uint64_t)P.sig_map[sig] : (uint64_t)sig;  // the signal's index in the call
  const uint64_t index =
      ((((uint64_t)key * 4ull + (uint64_t)phase) * 256ull + (uint64_t)iter) * 2ull) + (uint64_t)axis;
  const uint64_t r = splitmix64_at(P.seed, index);
  const uint32_t mask = P.n - 1u;
  Draw d;
  d.sigma = ((uint32_t)r & mask) | 1u;
  d.tau = (uint32_t)(r >> 32) & mask;
  return d;
}

// Inverse of an odd a modulo 2^32 by Newton's iteration x <- x (2 - a x): the
// start x = a is right to 3 bits and every step doubles the correct bits.
__device__ __forceinline__ uint32_t inv_odd(uint32_t a) {
  uint32_t x = a;
#pragma unroll
  for (int i = 0; i < 5; ++i) x *= 2u - a * x;
  return x;
}

// ------------------------------------------------------------ workspace ----

__device__ __forceinline__ uint8_t *slice_of(const KParams &P, uint32_t sig) {
  return P.ws + (size_t)sig * P.lay.slice;
}
// element offset of a signal in the caller's input, and its output slot
__device__ __forceinline__ int64_t x_offset(const KParams &P, uint32_t sig) {
  return P.x_off ? P.x_off[sig] : (int64_t)sig * P.x_sig;
}
__device__ __forceinline__ int64_t out_slot(const KParams &P, uint32_t sig) {
  return P.sig_map ? (int64_t)P.sig_map[sig] : (int64_t)sig;
}
__device__ __forceinline__ SigState *state_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<SigState *>(slice_of(P, sig) + P.lay.state);
}
__device__ __forceinline__ ProbeRec *hist_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<ProbeRec *>(slice_of(P, sig) + P.lay.hist);
}
template <typename C> __device__ __forceinline__ C *yprobe_of(const KParams &P, uint32_t sig, uint32_t level) {
  return reinterpret_cast<C *>(slice_of(P, sig) + P.lay.yprobe) + P.probe_off[level];
}
template <typename C> __device__ __forceinline__ C *ymain_of(const KParams &P, uint32_t sig, uint32_t loop) {
  return reinterpret_cast<C *>(slice_of(P, sig) + P.lay.ymain + loop * P.lay.ymain_loop);
}
__device__ __forceinline__ double *tloc_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<double *>(slice_of(P, sig) + P.lay.tloc);
}
__device__ __forceinline__ int32_t *jcount_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<int32_t *>(slice_of(P, sig) + P.lay.jcount);
}
__device__ __forceinline__ uint32_t *jbits_of(const KParams &P, uint32_t sig, uint32_t loop) {
  return reinterpret_cast<uint32_t *>(slice_of(P, sig) + P.lay.jbits + loop * P.lay.jbits_loop);
}
__device__ __forceinline__ int32_t *jlist_of(const KParams &P, uint32_t sig, uint32_t loop) {
  return reinterpret_cast<int32_t *>(slice_of(P, sig) + P.lay.jlist + loop * P.lay.jlist_loop);
}
__device__ __forceinline__ uint32_t *S_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<uint32_t *>(slice_of(P, sig) + P.lay.S);
}
__device__ __forceinline__ uint32_t *Ssort_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<uint32_t *>(slice_of(P, sig) + P.lay.Ssort);
}
__device__ __forceinline__ double *resid_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<double *>(slice_of(P, sig) + P.lay.resid);
}
__device__ __forceinline__ int32_t *bflag_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<int32_t *>(slice_of(P, sig) + P.lay.bflag);
}
__device__ __forceinline__ uint16_t *tape_of(const KParams &P, uint32_t sig) {
  return reinterpret_cast<uint16_t *>(slice_of(P, sig) + P.lay.tape);
}
template <typename R>
__device__ __forceinline__ const R *taps_of(const KParams &P, int which, uint32_t logB) {
  return reinterpret_cast<const R *>(P.G) + P.tab[which * 32 + logB];
}
// G'(q) for |q| <= (reach + 1) n/B, centred (residual test)
template <typename R> __device__ __forceinline__ const R *ghat_wide_of(const KParams &P, uint32_t logB) {
  return reinterpret_cast<const R *>(P.Ghat) + P.tab[96 + logB];
}
template <typename R> __device__ __forceinline__ const R *ghat_of(const KParams &P, uint32_t logB) {
  return reinterpret_cast<const R *>(P.Ghat) + P.tab[64 + logB];
}

__device__ __forceinline__ uint32_t ilog2(uint32_t v) { return 31u - __clz(v); }

// log2 of a signal's length (DEV: clamped to the covered lengths, as
// params_of picks them), without the per-length table.
template <bool DEV> __device__ __forceinline__ uint32_t sig_logn(const KParams &P, uint32_t sig) {
  if constexpr (DEV) {
    const int64_t n = P.ns[sig];
    const uint32_t lg = n > 0 ? 63u - (uint32_t)__clzll((unsigned long long)n) : 0u;
    return min(max(lg, P.dev_lg_lo), P.dev_lg_hi);
  } else {
    return P.logn;
  }
}

// Address slabs of a signal's 1D main-pass hash: one for lengths up to
// 2^one_slab_logn (plans whose lanes have few wraps each), else kSlabs.
template <bool DEV, int NDIM> __device__ __forceinline__ uint32_t main_slabs(const KParams &P, uint32_t sig) {
  if (NDIM != 1 || P.one_slab_logn == 0u) return (uint32_t)kSlabs;
  return sig_logn<DEV>(P, sig) <= P.one_slab_logn ? 1u : (uint32_t)kSlabs;
}

// The parameters signal `sig` runs with: the launch's own, or (DEV, an uneven
// batch whose lengths are on the device) those of the signal's length, which
// k_dev_setup wrote into the workspace.  A length outside the plan's range
// reads the nearest covered one; k_init marks such a signal and every kernel
// skips it.
template <bool DEV> __device__ __forceinline__ const KParams &params_of(const KParams &P, uint32_t sig) {
  if constexpr (DEV)
    return P.devP[sig_logn<DEV>(P, sig)];
  else
    return P;
}
__device__ __forceinline__ uint32_t bitrev(uint32_t v, uint32_t bits) {
  return bits ? (__brev(v) >> (32u - bits)) : 0u;
}

// ------------------------------------------------------- block helpers ----

// Wave-level primitives on the DPP crossbar (every lane of the wave active):
// shifts within rows of 16 lanes, then the row totals broadcast into the rows
// above, a handful of VALU operations instead of LDS permutes.  `old` is the
// value a lane without a source lane takes (the identity of the operation).
template <int CTRL, int ROWS = 0xF> __device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += dpp<0x111>(0u, v);  // row_shr:1
  v += dpp<0x112>(0u, v);  // row_shr:2
  v += dpp<0x114>(0u, v);  // row_shr:4
  v += dpp<0x118>(0u, v);  // row_shr:8
  v += dpp<0x142, 0xA>(0u, v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xC>(0u, v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum over the wave, uniform.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return lane_value(wave_incl_scan(v), 63); }

// 64-bit values: both halves moved alike
template <int CTRL, int ROWS = 0xF> __device__ __forceinline__ unsigned long long dpp(uint32_t old, unsigned long long v) {
  return ((unsigned long long)dpp<CTRL, ROWS>(old, (uint32_t)(v >> 32)) << 32) | dpp<CTRL, ROWS>(old, (uint32_t)v);
}
__device__ __forceinline__ unsigned long long lane_value(unsigned long long v, uint32_t lane) {
  return ((unsigned long long)lane_value((uint32_t)(v >> 32), lane) << 32) | lane_value((uint32_t)v, lane);
}

// Largest (MAX) or smallest key over the wave, uniform.
template <bool MAX, typename K> __device__ __forceinline__ K wave_extreme(K v) {
  const uint32_t id = MAX ? 0u : ~0u;  // per 32-bit half
  auto op = [](K a, K b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
  v = op(v, dpp<0x111>(id, v));
  v = op(v, dpp<0x112>(id, v));
  v = op(v, dpp<0x114>(id, v));
  v = op(v, dpp<0x118>(id, v));
  v = op(v, dpp<0x142, 0xA>(id, v));
  v = op(v, dpp<0x143, 0xC>(id, v));
  return lane_value(v, 63);
}

// Set bits of a wave mask in the lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Sum over the block; `sh` holds one LDS word per wave.  Every thread gets
// the total.
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *sh) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  const uint32_t r = wave_sum(lane < nw ? sh[lane] : 0u);
  __syncthreads();
  return r;
}

// Exclusive prefix sum over the block in thread order, and the block total;
// `sh` holds one word per wave, from word 8 on (words 0..7 are left to the
// callers' other uses).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total = nullptr) {
  const uint32_t lane = threadIdx.x & 63u, nw = (blockDim.x + 63) >> 6;
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) sh[8 + wave] = incl;
  __syncthreads();
  const uint32_t waves = wave_incl_scan(lane < nw ? sh[8 + lane] : 0u);
  const uint32_t before = wave ? lane_value(waves, wave - 1) : 0u;
  if (total) *total = lane_value(waves, nw - 1);
  __syncthreads();
  return before + incl - v;
}

// The k-th smallest (0-based) of a block's values that exceed `above`
// (default: all non-negative ones), by most-significant-digit radix selection
// on the bit patterns (the values are non-negative, so their patterns order
// like the values; negative ones mark empty slots).  `for_each(f)` calls f on
// each of the calling thread's values.
// When the keys' range [lo, hi] is known, the digits are taken of key - lo
// from the top bit of hi - lo, so that the first pass spreads the keys over
// all 256 bins instead of the few that the exponent's top bits give.  `hist`
// has 2 x 256 words, used in turn so that each pass clears the next pass's
// histogram while it counts; `sh` has 4 words (the chosen digit and rank,
// also in turn).
__device__ __forceinline__ int bit_length(uint32_t v) { return v ? 32 - __clz((int)v) : 0; }
__device__ __forceinline__ int bit_length(unsigned long long v) { return v ? 64 - __clzll((long long)v) : 0; }

// A thread's run of equal digits in a digit pass, added with one atomic
// (leading digits are shared by many values, and same-address atomics
// serialise)
struct DigitRun {
  uint32_t bin, run;
};
__device__ __forceinline__ void digit_add(DigitRun &r, uint32_t *h, uint32_t bin, bool take) {
  // selects rather than branches: only the atomic is predicated
  const bool flush = take && r.run != 0u && bin != r.bin;
  if (flush) atomicAdd(&h[r.bin], r.run);
  r.run = take ? (flush ? 1u : r.run + 1u) : r.run;
  r.bin = take ? bin : r.bin;
}
__device__ __forceinline__ void digit_flush(const DigitRun &r, uint32_t *h) {
  if (r.run) atomicAdd(&h[r.bin], r.run);
}

// After a pass's histogram h is complete: one wave finds the digit whose bin
// holds rank k and writes it and the rank within the bin to out[0], out[1].
__device__ __forceinline__ void digit_pick(const uint32_t *h, uint32_t k, uint32_t *out) {
  const uint32_t l = threadIdx.x & 63u;
  const uint4 c = *reinterpret_cast<const uint4 *>(h + 4 * l);  // h 16-byte aligned
  const uint32_t c0 = c.x, c1 = c.y, c2 = c.z, c3 = c.w;
  const uint32_t s = c0 + c1 + c2 + c3;
  const uint32_t incl = wave_incl_scan(s);
  const uint32_t excl = incl - s;
  if (excl <= k && k < incl) {
    uint32_t digit, run;
    if (k < excl + c0) {
      digit = 4 * l;
      run = excl;
    } else if (k < excl + c0 + c1) {
      digit = 4 * l + 1;
      run = excl + c0;
    } else if (k < excl + c0 + c1 + c2) {
      digit = 4 * l + 2;
      run = excl + c0 + c1;
    } else {
      digit = 4 * l + 3;
      run = excl + c0 + c1 + c2;
    }
    out[0] = digit;
    out[1] = k - run;
  }
}

// The values a select reads: thread t's v[j], j < per (REGS; uniform over
// the block, negative where the thread has no value), or m[t + i blockDim.x]
// below cnt.
template <typename R, int NPER, bool REGS> struct SelSrc {
  const R (&v)[NPER];
  uint32_t per;
  const R *m;
  uint32_t cnt;
};

template <typename R, int NPER, bool REGS>
__device__ __forceinline__ R radix_select(const SelSrc<R, NPER, REGS> &src, uint32_t k, uint32_t *hist,
                                          uint32_t *sh, R above, typename CT<R>::K lo, typename CT<R>::K hi) {
  using K = typename CT<R>::K;
  const int nbits = hi > lo ? bit_length(hi - lo) : 1;
  K prefix = 0, mask = 0;
  for (uint32_t i = threadIdx.x; i < 512; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  int pass = 0;
  for (int top = nbits; top > 0; ++pass) {
    const int width = top < 8 ? top : 8;
    const int shift = top - width;
    top = shift;
    const uint32_t dmask = (1u << width) - 1u;
    uint32_t *h = hist + 256 * (pass & 1);
    uint32_t *hn = hist + 256 * ((pass + 1) & 1);
    uint32_t *out = sh + 2 * (pass & 1);
    DigitRun r = {0, 0};
    if constexpr (REGS) {
#pragma unroll
      for (int j = 0; j < NPER; ++j) {
        if ((uint32_t)j < src.per) {
          const R mb = src.v[j];
          const K key = key_of(mb) - lo;
          digit_add(r, h, (uint32_t)(key >> shift) & dmask,
                    (key & mask) == prefix && (above < (R)0 ? mb >= (R)0 : mb > above));
        }
      }
    } else {
      for (uint32_t b = threadIdx.x; b < src.cnt; b += blockDim.x) {
        const R mb = src.m[b];
        const K key = key_of(mb) - lo;
        digit_add(r, h, (uint32_t)(key >> shift) & dmask,
                  (key & mask) == prefix && (above < (R)0 ? mb >= (R)0 : mb > above));
      }
    }
    digit_flush(r, h);
    if (top > 0)
      for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) hn[i] = 0;
    __syncthreads();
    if (threadIdx.x < 64) digit_pick(h, k, out);
    __syncthreads();
    const uint32_t digit = out[0];
    k = out[1];
    prefix |= (K)digit << shift;
    mask |= (K)dmask << shift;
  }
  __syncthreads();
  return val_of(prefix + lo);
}

// ... of the values m[0..cnt) (in LDS or device memory)
template <typename R>
__device__ __forceinline__ R block_kth_smallest(const R *m, uint32_t cnt, uint32_t k, uint32_t *hist,
                                                uint32_t *sh, R above = (R)-1,
                                                typename CT<R>::K lo = 0,
                                                typename CT<R>::K hi = ~(typename CT<R>::K)0) {
  const R none[1] = {(R)-1};
  return radix_select<R, 1, false>(SelSrc<R, 1, false>{none, 0u, m, cnt}, k, hist, sh, above, lo, hi);
}

// The ka-th (and with TWO also the kb-th) smallest (0-based) of the block's
// non-negative float values held in registers: thread t holds v[j], j < per
// (uniform), negative where it has no value.  Radix selection on key - lo as
// in radix_select, trimmed for registers: the keys are formed once, with bit
// 31 set for empty slots so that one mask-and-compare per pass also excludes
// them (a real key - lo is below 2^31); the count adds one per matching key
// (no runs); a value slot none of whose wave's keys match skips its atomic;
// waves 0 and 1 pick the two digits.  `hist` has 3 x 512 words (histogram
// pairs in turn), `sh` 8 words.
template <bool TWO, int NPER>
__device__ __forceinline__ void select_regs(const float (&v)[NPER], uint32_t per, uint32_t ka, uint32_t kb,
                                            uint32_t *hist, uint32_t *sh, uint32_t lo, uint32_t hi, float &va,
                                            float &vb) {
  const int nbits = hi > lo ? bit_length(hi - lo) : 1;
  uint32_t key[NPER];
#pragma unroll
  for (int j = 0; j < NPER; ++j) key[j] = (uint32_t)j < per && v[j] >= 0.f ? key_of(v[j]) - lo : 0xFFFFFFFFu;
  for (uint32_t i = threadIdx.x; i < 1024; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  uint32_t pa = 0, pb = 0, mask = 0x80000000u;
  int pass = 0;
  for (int top = nbits; top > 0; ++pass) {
    const int width = top < 8 ? top : 8;
    const int shift = top - width;
    top = shift;
    const uint32_t dmask = (1u << width) - 1u;
    uint32_t *ha = hist + 512 * (pass % 3), *hb = ha + 256;
    uint32_t *hn = hist + 512 * ((pass + 1) % 3);
#pragma unroll
    for (int j = 0; j < NPER; ++j) {
      const uint32_t kp = key[j] & mask;
      const bool ma = kp == pa, mb = TWO && kp == pb;
      // slots past per (the same for the whole block) are skipped whole
      if ((uint32_t)j >= per || __ballot(ma || mb) == 0) continue;
      const uint32_t bin = (key[j] >> shift) & dmask;
      if (ma)
        atomicAdd(&ha[bin], 1u);
      else if (mb)
        atomicAdd(&hb[bin], 1u);
    }
    if (top > 0)
      for (uint32_t i = threadIdx.x; i < 512; i += blockDim.x) hn[i] = 0;
    __syncthreads();
    uint32_t *out = sh + 4 * (pass & 1);
    if (threadIdx.x < 64)
      digit_pick(ha, ka, out);
    else if (TWO && threadIdx.x < 128)
      digit_pick(pa == pb ? ha : hb, kb, out + 2);
    __syncthreads();
    pa |= out[0] << shift;
    ka = out[1];
    if (TWO) {
      pb |= out[2] << shift;
      kb = out[3];
    }
    mask |= dmask << shift;
  }
  va = val_of(pa + lo);
  vb = val_of(pb + lo);
}

// The ka-th and kb-th smallest (0-based) of a block's non-negative values in
// one series of digit passes: both searches share each pass's scan over the
// values; while their prefixes agree they share its histogram, after that
// each counts the values of its own prefix.  `hist` has 4 x 256 words (a pair
// per pass, in turn), `sh` 8 words; digits and range as in radix_select.
template <typename R, int NPER, bool REGS>
__device__ __forceinline__ void radix_select2(const SelSrc<R, NPER, REGS> &src, uint32_t ka, uint32_t kb,
                                              uint32_t *hist, uint32_t *sh, typename CT<R>::K lo,
                                              typename CT<R>::K hi, R &va, R &vb) {
  using K = typename CT<R>::K;
  const int nbits = hi > lo ? bit_length(hi - lo) : 1;
  K pa = 0, pb = 0, mask = 0;
  for (uint32_t i = threadIdx.x; i < 1024; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  int pass = 0;
  for (int top = nbits; top > 0; ++pass) {
    const int width = top < 8 ? top : 8;
    const int shift = top - width;
    top = shift;
    const uint32_t dmask = (1u << width) - 1u;
    uint32_t *ha = hist + 512 * (pass & 1), *hb = ha + 256;
    uint32_t *hn = hist + 512 * ((pass + 1) & 1);
    uint32_t *out = sh + 4 * (pass & 1);
    const bool apart = pa != pb;  // otherwise every value counts in ha
    DigitRun ra = {0, 0}, rb = {0, 0};
    if constexpr (REGS) {
#pragma unroll
      for (int j = 0; j < NPER; ++j) {
        if ((uint32_t)j < src.per) {
          const R mb = src.v[j];
          const K key = key_of(mb) - lo, kp = key & mask;
          const uint32_t bin = (uint32_t)(key >> shift) & dmask;
          const bool ok = mb >= (R)0;
          digit_add(ra, ha, bin, ok && kp == pa);
          digit_add(rb, hb, bin, ok && kp == pb && kp != pa);
        }
      }
    } else {
      for (uint32_t b = threadIdx.x; b < src.cnt; b += blockDim.x) {
        const R mb = src.m[b];
        const K key = key_of(mb) - lo, kp = key & mask;
        const uint32_t bin = (uint32_t)(key >> shift) & dmask;
        const bool ok = mb >= (R)0;
        digit_add(ra, ha, bin, ok && kp == pa);
        digit_add(rb, hb, bin, ok && kp == pb && kp != pa);
      }
    }
    digit_flush(ra, ha);
    digit_flush(rb, hb);
    if (top > 0)
      for (uint32_t i = threadIdx.x; i < 512; i += blockDim.x) hn[i] = 0;
    __syncthreads();
    // wave 0 searches for ka, wave 1 for kb (in the shared histogram while
    // the prefixes agree)
    if (threadIdx.x < 64)
      digit_pick(ha, ka, out);
    else if (threadIdx.x < 128)
      digit_pick(apart ? hb : ha, kb, out + 2);
    __syncthreads();
    pa |= (K)out[0] << shift;
    ka = out[1];
    pb |= (K)out[2] << shift;
    kb = out[3];
    mask |= (K)dmask << shift;
  }
  __syncthreads();
  va = val_of(pa + lo);
  vb = val_of(pb + lo);
}

// ------------------------------------------------------------- k_init ----

template <bool DEV>
__global__ void k_init(KParams P0, int batch) {
  const int sig = blockIdx.x * blockDim.x + threadIdx.x;
  if (sig >= batch) return;
  const KParams &P = params_of<DEV>(P0, (uint32_t)sig);
  SigState s;
  s.B = (int32_t)P.B0;
  s.k_prev = 0;
  s.done = 0;
  s.B_star = (int32_t)P.B0;
  s.khat = 0;
  s.status = 0;
  s.visited = 0;
  s.n_probe = 0;
  s.count = 0;
  s.pass = 0;
  s.res_ratio = 0.0;
  s.round_blocks = 0;
  s.loc_loaded = 0;
  for (int i = 0; i < 3; ++i) s.pad[i] = 0;
  if (P.fixed) {
    s.done = 1;
    s.B_star = (int32_t)P.fixed_B;
    s.khat = (int32_t)P.fixed_k;
    if (s.khat <= 0) s.status |= kSigEmpty;
  }
  if constexpr (DEV) {
    // a length that is not a power of two the plan covers: nothing runs
    const int64_t n = P0.ns[sig];
    if (n != (int64_t)P.n) {
      s.done = 1;
      s.khat = 0;
      s.status |= kSigBadLength | kSigEmpty;
    }
  }
  *state_of(P, sig) = s;
  // a probe level's count is -1 until its k_bucket workgroup stores it
  ProbeRec *h = hist_of(P, sig);
  for (uint32_t i = 0; i < P.probe_levels; ++i) h[i].k = -1;
}

// ------------------------------------------------------------- k_hash ----

// Permute, window and fold (Definition 1, the window paragraph, Lemma 2):
// for every loop, y_b = sum over taps t = b mod B, -w/2 <= t < w/2, of
// x[(sigma t + tau) mod n] G_t.
//
// The gathers are random 8- or 16-byte loads, and what they cost depends on
// where the line comes from: random loads that hit L2 run about four times
// faster than loads served by HBM or the Infinity Cache.  A loop touches a
// random slice of the signal, so most lines are touched by several loops and
// those touches should hit L2.  The signal is cut into kSlabs address slabs
// (2D: bands of rows); a workgroup gathers only the samples of one slab, and
// its slab is its index modulo kSlabs, which under the hardware's round-robin
// dispatch is its XCD, so each XCD's L2 serves one slab.  The grid is
// (kSlabs x kTileSlots, loops, signals) and is dispatched signal by signal,
// so the resident workgroups cover about one signal at a time.
//
// A workgroup owns 64-bucket tiles (slot, slot + kTileSlots, ...) of up to
// three loops (1D main pass); its four 64-lane groups split each bucket's w/B
// wraps and issue their in-slab loads eight wraps at a time; a wrap's window
// tap depends only on the bucket and the wrap, so every lane loads it once
// (coalesced) for all the workgroup's loops; a fixed-order LDS sum combines
// the groups into the slab's partial y_b.  k_bucket adds the kSlabs partials
// in slab order.
constexpr int kTile = 64;        // buckets per tile
constexpr int kVoteIlp = 4;      // vote candidates tested together
constexpr int kTileSlots = 64;   // most tile slots per slab (grid x = kSlabs * slots)
constexpr int kHashU = 8;        // wraps whose loads are issued together

// s + c += a b with Neumaier's compensated sum: the product's rounding error
// comes exactly from an fma and the addition's from the larger operand; the
// explicitly rounded operations keep the compiler from contracting them.
__device__ __forceinline__ void neumaier_fma(float &s, float &c, float a, float b) {
  const float p = __fmul_rn(a, b);
  const float e = fmaf(a, b, -p);
  const float t = __fadd_rn(s, p);
  const float d = fabsf(s) >= fabsf(p) ? __fadd_rn(__fsub_rn(s, t), p) : __fadd_rn(__fsub_rn(p, t), s);
  c = __fadd_rn(c, __fadd_rn(d, e));
  s = t;
}
__device__ __forceinline__ void neumaier_add(float &s, float &c, float v) {
  const float t = __fadd_rn(s, v);
  const float d = fabsf(s) >= fabsf(v) ? __fadd_rn(__fsub_rn(s, t), v) : __fadd_rn(__fsub_rn(v, t), s);
  c = __fadd_rn(c, d);
  s = t;
}

// COMP (FP32 only): every accumulation carries a Neumaier compensation term
// through the wraps and the LDS reduction, and the partial is s + c.
template <typename R, int NDIM, int LG, bool COMP = false, bool MAIN = true, bool DEV = false>
__global__ __launch_bounds__(kHashThreads) void k_hash(KParams P0, int iter, int iter_hi) {
  using C = typename CT<R>::C;
  const uint32_t sig = blockIdx.z;
  // the control block's address needs no per-length parameters (every
  // length of a device-length launch shares the slice layout): it is read
  // first, and a main-pass workgroup with no tile of its signal's B leaves
  // before the per-length parameters are read
  const SigState st = *state_of(P0, sig);  // one 64-byte read
  const uint32_t NSm = MAIN ? main_slabs<DEV, NDIM>(P0, sig) : 1u;
  if constexpr (MAIN) {
    if ((st.status & kSigEmpty) || st.pass != (int32_t)P0.pass) return;
    const uint32_t Bs = (uint32_t)st.B_star;
    if ((blockIdx.x / NSm) * kTile >= (NDIM == 1 ? Bs : Bs * Bs)) return;
  }
  constexpr bool main_phase = MAIN;
  static_assert(NDIM == 1 || LG == 1, "2D hashes one loop per workgroup");
  // 2D probe levels read few rows more than once: one slab, no row filter;
  // 1D probe levels as the plan says (their lines are cold and rarely
  // touched twice, so one slab spares the other workgroups' address scans)
  const uint32_t NS = MAIN ? NSm : NDIM == 1 ? P0.probe_slabs : 1u;
  const uint32_t slab = blockIdx.x % NS;
  uint32_t slot = blockIdx.x / NS;
  uint32_t nslots = gridDim.x / NS;
  // a probe round's grid lists (level, slot) pairs, each level with as many
  // slots as it has 64-bucket tiles (at most tile_slots), counted with the
  // launch's B0 (a shorter signal of an uneven batch has no more tiles)
  uint32_t level = (uint32_t)iter;
  if (!main_phase) {
    for (;;) {
      const uint32_t Bl = P0.B0 << level;
      const uint32_t tl = ((NDIM == 1 ? Bl : Bl * Bl) + kTile - 1) / kTile;
      nslots = max(1u, min(P0.tile_slots, tl));
      if (slot < nslots || level + 1u >= (uint32_t)iter_hi) break;
      slot -= nslots;
      ++level;
    }
    if (slot >= nslots || st.done) return;
  }
  const KParams &P = params_of<DEV>(P0, sig);
  uint32_t B, alpha, nl = 1;
  Draw d0[LG], d1[LG];
  C *y[LG];
  size_t sstride;
  if (!main_phase) {
    if (slot >= nslots || st.done || level >= P.probe_levels) return;
    B = P.B0 << level;
    alpha = P.alpha_probe;
    d0[0] = draw(P, sig, kPhaseProbe, (int)level, 0);
    d1[0] = NDIM == 2 ? draw(P, sig, kPhaseProbe, (int)level, 1) : d0[0];
    y[0] = yprobe_of<C>(P, sig, level);
    sstride = NDIM == 1 ? B : (size_t)B * B;
  } else {
    if ((st.status & kSigEmpty) || st.pass != (int32_t)P.pass) return;
    B = (uint32_t)st.B_star;
    alpha = P.alpha;
    const uint32_t loops = P.L_loc + P.L_est;
    const uint32_t l0 = blockIdx.y * LG;
    nl = min((uint32_t)LG, loops - l0);
#pragma unroll
    for (int q = 0; q < LG; ++q) {
      const uint32_t loop = min(l0 + q, loops - 1);
      const int phase = loop < P.L_loc ? kPhaseLoc : kPhaseEst;
      const int it = (loop < P.L_loc ? (int)loop : (int)(loop - P.L_loc)) + kPassIter * st.pass;
      d0[q] = draw(P, sig, phase, it, 0);
      d1[q] = NDIM == 2 ? draw(P, sig, phase, it, 1) : d0[q];
      y[q] = ymain_of<C>(P, sig, loop);
    }
    sstride = P.Bc_max;
  }
  const uint32_t logB = ilog2(B);
  const uint32_t Bc = NDIM == 1 ? B : B * B;
  if (slot * kTile >= Bc) return;
  const uint32_t n = P.n, mask = n - 1u;
  const uint32_t slab_shift = P.logn - 3;  // kSlabs = 8 slabs of n/8 addresses (2D: rows)
  const uint32_t w = min(alpha * B, n);
  const uint32_t half = w >> 1;
  const uint32_t wraps = w >> logB;
  const R *G = taps_of<R>(P, main_phase ? 1 : 0, logB);
  const C *x = reinterpret_cast<const C *>(P.x) + x_offset(P, sig);
  const uint32_t bi = threadIdx.x & (kTile - 1), g = threadIdx.x >> 6;
  __shared__ R red_x[LG][4][kTile], red_y[LG][4][kTile];
  __shared__ R red_cx[COMP ? LG : 1][COMP ? 4 : 1][COMP ? kTile : 1];
  __shared__ R red_cy[COMP ? LG : 1][COMP ? 4 : 1][COMP ? kTile : 1];

  for (uint32_t tile = slot; tile * kTile < Bc; tile += nslots) {
    const uint32_t b = tile * kTile + bi;
    R ax[LG], ay[LG], cx[LG], cy[LG];
#pragma unroll
    for (int q = 0; q < LG; ++q) ax[q] = ay[q] = cx[q] = cy[q] = 0;
    if (b < Bc) {
      if (NDIM == 1) {
        // the group's wraps r = g, g + 4, ...: addresses advance by sigma * 4B;
        // the in-slab loads of all the workgroup's loops go out together
        uint32_t a[LG], step[LG];
#pragma unroll
        for (int q = 0; q < LG; ++q) {
          a[q] = (d0[q].sigma * (b + (g << logB) - half) + d0[q].tau) & mask;
          step[q] = (d0[q].sigma << (logB + 2)) & mask;
        }
        for (uint32_t r0 = g; r0 < wraps; r0 += 4 * kHashU) {
          C v[LG][kHashU];
          R gt[kHashU];
          // a wrap's tap is the same for every loop: one load by every lane
          // (64 consecutive taps, two lines), shared by the workgroup's loops
#pragma unroll
          for (int u = 0; u < kHashU; ++u) gt[u] = r0 + 4u * u < wraps ? G[b + ((r0 + 4u * u) << logB)] : (R)0;
#pragma unroll
          for (int q = 0; q < LG; ++q) {
#pragma unroll
            for (int u = 0; u < kHashU; ++u) {
              const uint32_t aq = a[q];
              const bool pp = (uint32_t)q < nl && r0 + 4u * u < wraps && (NS == 1u || (aq >> slab_shift) == slab);
              a[q] = (aq + step[q]) & mask;
              v[q][u].x = 0;
              v[q][u].y = 0;
              if (pp) v[q][u] = x[aq];
            }
          }
#pragma unroll
          for (int q = 0; q < LG; ++q) {
#pragma unroll
            for (int u = 0; u < kHashU; ++u) {
              if constexpr (COMP) {
                neumaier_fma(ax[q], cx[q], v[q][u].x, gt[u]);
                neumaier_fma(ay[q], cy[q], v[q][u].y, gt[u]);
              } else {
                ax[q] += v[q][u].x * gt[u];
                ay[q] += v[q][u].y * gt[u];
              }
            }
          }
        }
      } else {
        const uint32_t b1 = b >> logB, b2 = b & (B - 1u);
        for (uint32_t r1 = g; r1 < wraps; r1 += 4) {
          const uint32_t i1 = b1 + (r1 << logB);
          const uint32_t a1 = (d0[0].sigma * (i1 - half) + d0[0].tau) & mask;
          if (NS > 1u && (a1 >> slab_shift) != slab) continue;
          const R g1 = G[i1];
          const C *row = x + (size_t)a1 * n;
          for (uint32_t r0 = 0; r0 < wraps; r0 += kHashU) {
            C v[kHashU];
            R gt[kHashU];
#pragma unroll
            for (int u = 0; u < kHashU; ++u) {
              v[u].x = 0;
              v[u].y = 0;
              gt[u] = 0;
              if (r0 + u < wraps) {
                const uint32_t i2 = b2 + ((r0 + u) << logB);
                v[u] = row[(d1[0].sigma * (i2 - half) + d1[0].tau) & mask];
                gt[u] = g1 * G[i2];
              }
            }
#pragma unroll
            for (int u = 0; u < kHashU; ++u) {
              if constexpr (COMP) {
                neumaier_fma(ax[0], cx[0], v[u].x, gt[u]);
                neumaier_fma(ay[0], cy[0], v[u].y, gt[u]);
              } else {
                ax[0] += v[u].x * gt[u];
                ay[0] += v[u].y * gt[u];
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < LG; ++q) {
      red_x[q][g][bi] = ax[q];
      red_y[q][g][bi] = ay[q];
      if constexpr (COMP) {
        red_cx[q][g][bi] = cx[q];
        red_cy[q][g][bi] = cy[q];
      }
    }
    __syncthreads();
    if (g == 0 && b < Bc) {
#pragma unroll
      for (int q = 0; q < LG; ++q) {
        if ((uint32_t)q < nl) {
          C s;
          if constexpr (COMP) {
            R sx = red_x[q][0][bi], sy = red_y[q][0][bi], ex = red_cx[q][0][bi], ey = red_cy[q][0][bi];
            for (int gg = 1; gg < 4; ++gg) {
              neumaier_add(sx, ex, red_x[q][gg][bi]);
              neumaier_add(sy, ey, red_y[q][gg][bi]);
              ex = __fadd_rn(ex, red_cx[q][gg][bi]);
              ey = __fadd_rn(ey, red_cy[q][gg][bi]);
            }
            s.x = __fadd_rn(sx, ex);
            s.y = __fadd_rn(sy, ey);
          } else {
            s.x = ((red_x[q][0][bi] + red_x[q][1][bi]) + red_x[q][2][bi]) + red_x[q][3][bi];
            s.y = ((red_y[q][0][bi] + red_y[q][1][bi]) + red_y[q][2][bi]) + red_y[q][3][bi];
          }
          y[q][(size_t)slab * sstride + b] = s;
        }
      }
    }
    __syncthreads();
  }
}

// --------------------------------------------------------- LDS FFT ----

// In-register DFTs of 2, 4 and 8 points, natural order in and out,
// omega = e^{-2 pi i / RAD}.
template <typename C> __device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C> __device__ __forceinline__ C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C> __device__ __forceinline__ C mul_mi(C a) {  // a * (-i)
  C r;
  r.x = a.y;
  r.y = -a.x;
  return r;
}

template <typename C> __device__ __forceinline__ void dft4(C &x0, C &x1, C &x2, C &x3) {
  const C a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = mul_mi(csub(x1, x3));
  x0 = cadd(a0, a2);
  x2 = csub(a0, a2);
  x1 = cadd(a1, a3);
  x3 = csub(a1, a3);
}

// 16-point DFT, natural order in and out, as 4 x 4: DFTs of the four
// stride-4 subsequences, twiddles omega_16^{n2 k1}, DFTs across them
template <typename R> __device__ __forceinline__ void dft16(typename CT<R>::C *x) {
  using C = typename CT<R>::C;
  const R c1 = (R)0.92387953251128675612818318939678828;  // cos(pi / 8)
  const R s1 = (R)0.38268343236508977172845998403039887;  // sin(pi / 8)
  const R h = (R)0.70710678118654752440084436210484904;   // cos(pi / 4)
  C y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = x[n2];
    y[n2][1] = x[4 + n2];
    y[n2][2] = x[8 + n2];
    y[n2][3] = x[12 + n2];
    dft4(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
  }
  auto tw = [](C a, R wr, R wi) {
    C r;
    r.x = a.x * wr - a.y * wi;
    r.y = a.x * wi + a.y * wr;
    return r;
  };
  // omega_16^m = cos(2 pi m / 16) - i sin(2 pi m / 16) for m = n2 k1
  y[1][1] = tw(y[1][1], c1, -s1);  // m = 1
  y[1][2] = tw(y[1][2], h, -h);    // m = 2
  y[1][3] = tw(y[1][3], s1, -c1);  // m = 3
  y[2][1] = tw(y[2][1], h, -h);    // m = 2
  y[2][2] = mul_mi(y[2][2]);       // m = 4
  y[2][3] = tw(y[2][3], -h, -h);   // m = 6
  y[3][1] = tw(y[3][1], s1, -c1);  // m = 3
  y[3][2] = tw(y[3][2], -h, -h);   // m = 6
  y[3][3] = tw(y[3][3], -c1, s1);  // m = 9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
    dft4(a0, a1, a2, a3);
    x[k1] = a0;
    x[k1 + 4] = a1;
    x[k1 + 8] = a2;
    x[k1 + 12] = a3;
  }
}

template <typename R, int RB> __device__ __forceinline__ void dft_reg(typename CT<R>::C *x) {
  using C = typename CT<R>::C;
  if (RB == 4) {
    dft16<R>(x);
  } else if (RB == 1) {
    const C a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
  } else if (RB == 2) {
    dft4(x[0], x[1], x[2], x[3]);
  } else {
    // split into even and odd halves, then X_m = E_m + w8^m O_m and
    // X_{m+4} = E_m - w8^m O_m with w8 = e^{-i pi / 4}
    C e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6], o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const R h = (R)0.70710678118654752440084436210484904;
    C t1, t3;
    t1.x = h * (o1.x + o1.y);
    t1.y = h * (o1.y - o1.x);
    const C t2 = mul_mi(o2);
    t3.x = h * (o3.y - o3.x);
    t3.y = -h * (o3.x + o3.y);
    x[0] = cadd(e0, o0);
    x[4] = csub(e0, o0);
    x[1] = cadd(e1, t1);
    x[5] = csub(e1, t1);
    x[2] = cadd(e2, t2);
    x[6] = csub(e2, t2);
    x[3] = cadd(e3, t3);
    x[7] = csub(e3, t3);
  }
}

// One pass of the in-place decimation-in-time DFT on bit-reversed input (count
// a power of two): the
// completed sub-transforms of length L = 2^logL are combined RAD = 2^RB at a
// time into length RAD L.  For offset p < L the RAD inputs are taken from
// sub-transforms in bit-reversed order (which is how the radix-2 stages this
// pass replaces would have paired them), scaled by omega_{RAD L}^{j p}, and
// transformed in registers; output m goes to position p + m L.
// LDS index of element e when the buffer holds one pad element after every
// 32 (PAD): strided passes and the bit-reversed load then spread over the banks
template <bool PAD> __device__ __forceinline__ uint32_t lds_at(uint32_t e) { return PAD ? e + (e >> 5) : e; }

template <typename R, int RB, bool PAD = false>
__device__ __forceinline__ void fft_pass(typename CT<R>::C *buf, uint32_t logB, uint32_t logL, uint32_t count,
                                         uint32_t fstride, uint32_t estride) {
  using C = typename CT<R>::C;
  constexpr int RAD = 1 << RB;
  const uint32_t gl = logB - RB;  // log2 of the groups per transform
  const uint32_t total = count << gl;
  const uint32_t L = 1u << logL;
  const R inv_n2 = (R)1 / (R)(L << RB);
  // transforms along a strided axis (2D columns) put neighbouring threads on
  // neighbouring transforms, so that their LDS accesses are contiguous
  const bool ffast = fstride < estride;
  const uint32_t lc = ffast ? 31u - __clz(count) : 0u;
  for (uint32_t kk = threadIdx.x; kk < total; kk += blockDim.x) {
    const uint32_t f = ffast ? (kk & (count - 1u)) : (kk >> gl);
    const uint32_t q = ffast ? (kk >> lc) : (kk & ((1u << gl) - 1u));
    const uint32_t p = q & (L - 1u), g = q >> logL;
    const uint32_t base = f * fstride + (((g << (logL + RB)) + p) * estride);
    const uint32_t step = L * estride;
    C x[RAD];
#pragma unroll
    for (int j = 0; j < RAD; ++j) {
      const int jr = RB == 1   ? j
                     : RB == 2 ? ((j & 1) << 1 | (j >> 1))
                     : RB == 3 ? ((j & 1) << 2 | (j & 2) | (j >> 2))
                               : ((j & 1) << 3 | (j & 2) << 1 | (j & 4) >> 1 | (j >> 3));
      x[j] = buf[lds_at<PAD>(base + (uint32_t)jr * step)];
    }
    if (logL > 0) {
      C w1;  // omega_{RAD L}^p, the angle an exact multiple of pi
      sincos_pi((R)(-2) * (R)p * inv_n2, &w1.y, &w1.x);
      if (RB == 4) {
        // omega^{jp} from omega^p, omega^{2p}, omega^{4p}, omega^{8p}: at
        // most three products per twiddle instead of up to fifteen
        C w[4];
        w[0] = w1;
#pragma unroll
        for (int e = 1; e < 4; ++e) sincos_pi((R)(-2) * (R)(p << e) * inv_n2, &w[e].y, &w[e].x);
#pragma unroll
        for (int j = 1; j < RAD; ++j) {
          C wj;
          bool first = true;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (j & (1 << e)) {
              wj = first ? w[e] : cmul(wj, w[e]);
              first = false;
            }
          x[j] = cmul(x[j], wj);
        }
      } else {
        C wj = w1;
#pragma unroll
        for (int j = 1; j < RAD; ++j) {
          x[j] = cmul(x[j], wj);
          if (j + 1 < RAD) wj = cmul(wj, w1);
        }
      }
    }
    dft_reg<R, RB>(x);
#pragma unroll
    for (int m = 0; m < RAD; ++m) buf[lds_at<PAD>(base + (uint32_t)m * step)] = x[m];
  }
  __syncthreads();
}

// Unnormalised DFT with omega = e^{-2 pi i / B} (the DFT display) along one
// axis of `count` independent length-2^logB transforms held in LDS in
// bit-reversed order; element j of transform f sits at
// buf[f * fstride + j * estride].  Radix-8 passes, led by one radix-2 or
// radix-4 pass when log2 B is not a multiple of 3.
template <typename R, bool PAD = false, bool R16 = false>
__device__ __forceinline__ void fft_axis(typename CT<R>::C *buf, uint32_t logB, uint32_t count, uint32_t fstride,
                                         uint32_t estride) {
  uint32_t logL = 0;
  if (R16) {
    // radix-16 passes led by one radix-2, -4 or -8 pass (for arrays with
    // enough groups per pass to occupy the workgroup)
    const uint32_t lead = logB % 4;
    if (lead == 1) {
      fft_pass<R, 1, PAD>(buf, logB, 0, count, fstride, estride);
    } else if (lead == 2) {
      fft_pass<R, 2, PAD>(buf, logB, 0, count, fstride, estride);
    } else if (lead == 3) {
      fft_pass<R, 3, PAD>(buf, logB, 0, count, fstride, estride);
    }
    for (logL = lead; logL < logB; logL += 4) fft_pass<R, 4, PAD>(buf, logB, logL, count, fstride, estride);
    return;
  }
  const uint32_t lead = logB % 3;
  if (lead == 1) {
    fft_pass<R, 1, PAD>(buf, logB, 0, count, fstride, estride);
    logL = 1;
  } else if (lead == 2) {
    fft_pass<R, 2, PAD>(buf, logB, 0, count, fstride, estride);
    logL = 2;
  }
  for (; logL < logB; logL += 3) fft_pass<R, 3, PAD>(buf, logB, logL, count, fstride, estride);
}

// key order of the local-maximum and cutoff steps: larger m first, equal m
// broken by the smaller bucket index
template <typename R>
__device__ __forceinline__ bool key_gt(const R *m, uint32_t a, uint32_t b) {
  const R ma = m[a], mb = m[b];
  return ma > mb || (ma == mb && a < b);
}

// B-update rule with the paper's constants (Sec. III-A) in exact integers,
// D = |k - k_prev|: 100 D < 2 k_prev halves, 100 D < 5 k_prev keeps, else
// doubles; k_prev = 0 doubles.
__device__ __forceinline__ int brule(int k_prev, int k) {
  if (k_prev <= 0) return 1;
  const long long D = k > k_prev ? k - k_prev : k_prev - k;
  if (100 * D < 2 * (long long)k_prev) return -1;
  if (100 * D < 5 * (long long)k_prev) return 0;
  return 1;
}

// ---------------------------------------------------------- 2D row hash ----

// 2D main-loop hash by rows: one workgroup per (bucket row b1, loop, signal).
// The row wraps r1 of b1 pick the rows a1 = sigma1 (b1 + r1 B - w/2) + tau1;
// each row is staged whole in LDS with coalesced 16-byte loads.  A thread
// owns bucket b2 = tid mod B and a share of its column wraps; the column
// addresses and taps are the same in every row, so they stay in registers,
// and the samples come from LDS.  The workgroup completes y[b1][.] itself
// (rows added in order, then the column shares in group order), so there are
// no slab partials.  Used for rows of at most kRowBytes.
template <typename R>
__global__ __launch_bounds__(kHashThreads) void k_hash2d_rows(KParams P) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  C *row = reinterpret_cast<C *>(smem);
  const uint32_t b1 = blockIdx.x, loop = blockIdx.y, sig = blockIdx.z;
  const SigState st = *state_of(P, sig);
  if ((st.status & kSigEmpty) || st.pass != (int32_t)P.pass) return;
  const uint32_t B = (uint32_t)st.B_star;
  if (b1 >= B) return;
  const uint32_t logB = ilog2(B);
  const uint32_t n = P.n, mask = n - 1u;
  const uint32_t w = min(P.alpha * B, n), half = w >> 1, wraps = w >> logB;
  const int phase = loop < P.L_loc ? kPhaseLoc : kPhaseEst;
  const int it = (loop < P.L_loc ? (int)loop : (int)(loop - P.L_loc)) + kPassIter * st.pass;
  const Draw d0 = draw(P, sig, phase, it, 0), d1 = draw(P, sig, phase, it, 1);
  const R *G = taps_of<R>(P, 1, logB);
  const C *x = reinterpret_cast<const C *>(P.x) + x_offset(P, sig);
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  const uint32_t b2 = tid & (B - 1u), grp = tid >> logB, ngrp = T >> logB;
  uint32_t col[kRowTaps];
  R gc[kRowTaps];
#pragma unroll
  for (int k = 0; k < kRowTaps; ++k) {
    const uint32_t r2 = grp + (uint32_t)k * ngrp;
    const uint32_t i2 = b2 + (min(r2, wraps - 1u) << logB);
    col[k] = (d1.sigma * (i2 - half) + d1.tau) & mask;
    gc[k] = r2 < wraps ? G[i2] : (R)0;
  }
  const uint32_t units = n * (uint32_t)sizeof(C) / 16u;  // 16-byte units per row
  R ax = 0, ay = 0;
  for (uint32_t r1 = 0; r1 < wraps; ++r1) {
    const uint32_t i1 = b1 + (r1 << logB);
    const uint32_t a1 = (d0.sigma * (i1 - half) + d0.tau) & mask;
    const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)a1 * n);
    float4 *dst = reinterpret_cast<float4 *>(row);
    __syncthreads();  // the previous row has been read
    for (uint32_t q = tid; q < units; q += T) dst[q] = src[q];
    __syncthreads();
    R rx = 0, ry = 0;
#pragma unroll
    for (int k = 0; k < kRowTaps; ++k) {
      const C v = row[col[k]];
      rx += gc[k] * v.x;
      ry += gc[k] * v.y;
    }
    const R g1 = G[i1];
    ax += g1 * rx;
    ay += g1 * ry;
  }
  // combine the column shares of each bucket in group order
  __syncthreads();
  R *red = reinterpret_cast<R *>(smem);
  red[2 * tid] = ax;
  red[2 * tid + 1] = ay;
  __syncthreads();
  if (grp == 0) {
    R sx = red[2 * tid], sy = red[2 * tid + 1];
    for (uint32_t gq = 1; gq < ngrp; ++gq) {
      sx += red[2 * (tid + (gq << logB))];
      sy += red[2 * (tid + (gq << logB)) + 1];
    }
    C out;
    out.x = sx;
    out.y = sy;
    ymain_of<C>(P, sig, loop)[(b1 << logB) | b2] = out;
  }
}

// 2D main-loop hash streamed by rows: every input row is read once per
// signal.  A workgroup takes P.stream_rows consecutive rows a1 of one image.
// Loop l uses row a1 iff its row wrap index i1 = sigma1^-1 (a1 - tau1) + w/2
// (mod N) is below w; the row is staged in LDS only if some loop uses it.
// For each such loop a group of B threads forms the row's column sums of all
// B buckets b2 (a thread holds bucket b2's taps for every column wrap, which
// are the same in every loop), scales them by G[i1] and writes them as
// partial r1 = i1 / B of bucket row b1 = i1 mod B.  Every partial slot is
// written by exactly one row and k_bucket adds a bucket's partials in r1
// order, so the result does not depend on scheduling.  Needs w / B <= 8
// partials and B <= the workgroup size.
// rows are read once: non-temporal loads, so that they do not push the
// partials (read back by k_bucket) out of the caches
typedef float nt4 __attribute__((ext_vector_type(4)));
template <typename R, int U, int NT = kHashThreads>
__global__ __launch_bounds__(NT) void k_hash2d_stream(KParams P) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_inv0[2 * kMaxLoops], s_tau0[2 * kMaxLoops], s_sig1[2 * kMaxLoops], s_tau1[2 * kMaxLoops];
  C *row = reinterpret_cast<C *>(smem);
  const uint32_t sig = blockIdx.y;
  const SigState st = *state_of(P, sig);
  if ((st.status & kSigEmpty) || st.pass != (int32_t)P.pass) return;
  const uint32_t B = (uint32_t)st.B_star, logB = ilog2(B);
  // arrays above the LDS size are hashed by the 1024-thread instantiation
  if (P.big && ((size_t)B * B > (size_t)P.lds_cap) != (NT == kBucketThreads)) return;
  const uint32_t n = P.n, mask = n - 1u;
  const uint32_t w = min(P.alpha * B, n), half = w >> 1, wraps = w >> logB;
  const uint32_t nloops = P.L_loc + P.L_est;
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  if (tid < nloops) {
    const int phase = tid < P.L_loc ? kPhaseLoc : kPhaseEst;
    const int it = (tid < P.L_loc ? (int)tid : (int)(tid - P.L_loc)) + kPassIter * st.pass;
    const Draw d0 = draw(P, sig, phase, it, 0), d1 = draw(P, sig, phase, it, 1);
    s_inv0[tid] = inv_odd(d0.sigma);
    s_tau0[tid] = d0.tau;
    s_sig1[tid] = d1.sigma;
    s_tau1[tid] = d1.tau;
  }
  const R *G = taps_of<R>(P, 1, logB);
  const uint32_t b2 = tid & (B - 1u), grp = tid >> logB, ngrp = T >> logB;
  R gc[kSlabs];
#pragma unroll
  for (int k = 0; k < kSlabs; ++k) gc[k] = (uint32_t)k < wraps ? G[b2 + ((uint32_t)k << logB)] : (R)0;
  const float4 *xs = reinterpret_cast<const float4 *>(reinterpret_cast<const C *>(P.x) + x_offset(P, sig));
  const uint32_t units = n * (uint32_t)sizeof(C) / 16u;  // 16-byte units per row
  float4 *dst = reinterpret_cast<float4 *>(row);
  __syncthreads();
  // the loops that use row a1 (the same in every thread)
  auto uses = [&](uint32_t a1) {
    uint64_t m = 0;
    if (a1 < n)
      for (uint32_t l = 0; l < nloops; ++l) {
        const uint32_t i1 = (s_inv0[l] * (a1 - s_tau0[l]) + half) & mask;
        if (i1 < w) m |= 1ull << l;
      }
    return m;
  };
  // the next used row is loaded into registers while the current one is hashed
  float4 pf[U];  // U >= the row's 16-byte units per thread
#define ATSFFT_STREAM_FETCH(A1)                                      \
  {                                                                  \
    const float4 *src_ = xs + (size_t)(A1) * units;                  \
    _Pragma("unroll") for (int k = 0; k < U; ++k) {                  \
      const uint32_t q = tid + (uint32_t)k * T;                      \
      pf[k] = make_float4(0.f, 0.f, 0.f, 0.f);                       \
      if (q < units) {                                               \
        const nt4 t_ = __builtin_nontemporal_load(reinterpret_cast<const nt4 *>(src_) + q); \
        pf[k] = make_float4(t_.x, t_.y, t_.z, t_.w);                 \
      }                                                              \
    }                                                                \
  }
  const uint32_t nrows = P.stream_rows, a_lo = blockIdx.x * nrows;
  uint32_t rr = 0;
  uint64_t use = 0;
  for (; rr < nrows && !(use = uses(a_lo + rr)); ++rr) {
  }
  if (rr < nrows) ATSFFT_STREAM_FETCH(a_lo + rr);
  while (rr < nrows) {
    const uint32_t a1 = a_lo + rr;
    __syncthreads();  // the previous row has been read
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t q = tid + (uint32_t)k * T;
      if (q < units) dst[q] = pf[k];
    }
    __syncthreads();
    const uint64_t cur = use;
    use = 0;
    for (++rr; rr < nrows && !(use = uses(a_lo + rr)); ++rr) {
    }
    if (rr < nrows) ATSFFT_STREAM_FETCH(a_lo + rr);
    // the j-th loop of the row goes to group j mod ngrp
    uint32_t j = 0;
    for (uint64_t u = cur; u; u &= u - 1ull, ++j) {
      if (j % ngrp != grp) continue;
      const uint32_t l = (uint32_t)__ffsll((unsigned long long)u) - 1u;
      const uint32_t i1 = (s_inv0[l] * (a1 - s_tau0[l]) + half) & mask;
      const uint32_t sg = s_sig1[l], tu = s_tau1[l];
      R rx = 0, ry = 0;
#pragma unroll
      for (int k = 0; k < kSlabs; ++k) {
        if ((uint32_t)k < wraps) {
          const uint32_t i2 = b2 + ((uint32_t)k << logB);
          const C v = row[(sg * (i2 - half) + tu) & mask];
          rx += gc[k] * v.x;
          ry += gc[k] * v.y;
        }
      }
      const R g1 = G[i1];
      C out;
      out.x = g1 * rx;
      out.y = g1 * ry;
      ymain_of<C>(P, sig, l)[(size_t)(i1 >> logB) * P.Bc_max + (((i1 & (B - 1u)) << logB) | b2)] = out;
    }
  }
}
#undef ATSFFT_STREAM_FETCH

// ------------------------------------------------------- probe control ----

// A probe level's local-maximum count.  Every workgroup of a round stores its
// count before it counts itself in, so a count that still reads -1 (k_init's
// value) is on its way; the wait is bounded, and -1 comes back if it gives up.
__device__ __forceinline__ int32_t probe_count(const KParams &P, ProbeRec *h) {
  int32_t k = __hip_atomic_load(&h->k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (uint32_t spin = 0; k < 0 && spin < P.probe_spin; ++spin) {
    __builtin_amdgcn_s_sleep(2);
    k = __hip_atomic_load(&h->k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return k;
}

// The adaptive-B iteration (Sec. III-A, Algorithm 2) for probe levels
// [lo, hi) of one signal, on the counts its k_bucket workgroups recorded,
// kv[i - lo] (-1: a count that never arrived), run by one thread of the last
// of them to finish.  The
// probe starts at B0 and only doubles until it stops: a halving always lands
// on a bucket count already probed (or below the occupancy guard, or below
// B0) and ends the probe there, so iteration i always hashes at B0 * 2^i and
// the counts of a round can be computed before its decisions are taken.
// Decisions: the B-update rule in exact integers (D = |k_i - k_{i-1}|: 100 D
// < 2 k_{i-1} halves, 100 D < 5 k_{i-1} keeps, else doubles; k_{i-1} = 0 and
// the first iteration double); a count is acted on only once B^ndim >=
// gamma * k_i; keep stops at B; halve stops at B/2 (k-hat from B); doubling
// past B_max stops (saturated); P_max iterations stop (not converged).
// s0: the signal's state as the round found it (written only by this routine
// and k_init, in earlier launches, so a copy read when the round's workgroup
// started is current).
template <int NDIM>
__device__ void probe_control(const KParams &P, uint32_t sig, int lo, int hi, const int32_t *kv,
                              const SigState &s0) {
  SigState *st = state_of(P, sig);
  SigState s = s0;
  ProbeRec *hist = hist_of(P, sig);
  for (int i = lo; i < hi && !s.done; ++i) {
    ProbeRec *h = hist + i;
    const uint32_t B = (uint32_t)s.B;
    const uint32_t logB = ilog2(B);
    const long long Bc = NDIM == 1 ? (long long)B : (long long)B * B;
    const int k = kv[i - lo];
    if (k < 0) {
      // the count never arrived: the probe stops at the last level it acted
      // on (B_star and khat as that level left them; before level 0, B0 and
      // khat = 0, so EMPTY) and the signal carries PROBE_TIMEOUT
      s.status |= kSigProbeTimeout;
      s.done = 1;
      if (s.khat <= 0) s.status |= kSigEmpty;
      break;
    }
    int dec = i == 0 ? 1 : brule(s.k_prev, k);
    if (P.gamma > 0 && Bc < (long long)P.gamma * (long long)k) dec = 1;
    s.visited |= 1u << logB;
    h->dec = dec;
    s.n_probe = i + 1;
    bool stop = false;
    if (dec == 0) {
      s.B_star = (int32_t)B;
      s.khat = k;
      stop = true;
    } else if (dec < 0) {
      const uint32_t Bh = B >> 1;
      const long long Bhc = NDIM == 1 ? (long long)Bh : (long long)Bh * Bh;
      s.khat = k;
      if (Bh < P.B0 || (P.gamma > 0 && Bhc < (long long)P.gamma * (long long)k) || !(s.visited & (1u << (logB - 1))))
        s.B_star = (int32_t)B;  // the last case cannot occur on the doubling chain
      else
        s.B_star = (int32_t)Bh;
      stop = true;
    } else {
      if (2 * B > P.B_max) {
        s.B_star = (int32_t)B;
        s.khat = k;
        s.status |= kSigSaturated;
        stop = true;
      } else {
        s.B = (int32_t)(2 * B);
      }
    }
    if (!stop) {
      s.k_prev = k;
      s.B_star = (int32_t)B;
      s.khat = k;
      if ((uint32_t)i + 1 >= P.P_max) {
        s.status |= kSigNotConverged;
        stop = true;
      }
    }
    if (stop) {
      s.done = 1;
      if (s.khat <= 0) s.status |= kSigEmpty;
    }
  }
  // field by field: round_blocks, in the same line, is only ever updated
  // atomically
  st->B = s.B;
  st->k_prev = s.k_prev;
  st->done = s.done;
  st->B_star = s.B_star;
  st->khat = s.khat;
  st->status = s.status;
  st->visited = s.visited;
  st->n_probe = s.n_probe;
}

// ------------------------------------------------------------ k_bucket ----

// One workgroup per bucket array: bucket DFT (B or B x B points) in LDS,
// then for probe and location loops m_b = |y_hat_b|^2, the noise-floor
// threshold T, and either the local-maximum count with the adaptive-B
// control (probe) or the top-num cutoff J (location loops).
template <typename R, int NDIM, bool DEV = false>
__global__ __launch_bounds__(kBucketThreads) void k_bucket(KParams P0, int main_phase, int iter) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t sig = blockIdx.y, loop = blockIdx.x;
  if (main_phase >= 2) {
    // one linear grid, every signal's location loops first: their chain is
    // the longer, and when the grid takes several rounds of the chip the
    // short estimation loops then fill the last one
    const uint32_t batch = gridDim.x / (P0.L_loc + P0.L_est), nloc = P0.L_loc * batch;
    const uint32_t i = blockIdx.x;
    loop = i < nloc ? i / batch : P0.L_loc + (i - nloc) / batch;
    sig = (i < nloc ? i : i - nloc) % batch;
  }
  const uint32_t level = (uint32_t)iter + blockIdx.x;
  SigState *st = state_of(P0, sig);  // the slice layout is every length's (see k_hash)
  if (main_phase) {
    if ((st->status & kSigEmpty) || st->pass != (int32_t)P0.pass) return;
    const uint32_t Bs = (uint32_t)st->B_star, Bcs = NDIM == 1 ? Bs : Bs * Bs;
    if ((main_phase == 3 && Bcs > kSmallBuckets) || (main_phase == 4 && Bcs <= kSmallBuckets)) return;
  }
  SigState st0;  // probe role: the state as this round found it
  if (!main_phase) {
    st0 = *st;
    if (st0.done) return;
  }
  const KParams &P = params_of<DEV>(P0, sig);
  uint32_t B;
  C *yg;
  if (!main_phase) {
    if (level >= P.probe_levels) return;
    B = P.B0 << level;
    yg = yprobe_of<C>(P, sig, level);
  } else {
    if ((st->status & kSigEmpty) || st->pass != (int32_t)P.pass) return;
    B = (uint32_t)st->B_star;
    yg = ymain_of<C>(P, sig, loop);
  }
  const uint32_t logB = ilog2(B);
  const uint32_t Bc = NDIM == 1 ? B : B * B;
  if (Bc > P.lds_cap) return;  // a large array: k_big_rows, k_big_cols, the k_bs_* steps
  // a main pass whose grid exceeds the chip runs arrays of at most
  // kSmallBuckets in 256- or 512-thread workgroups, several to a CU, and the
  // larger ones in a launch of their own (phase 3: the small class, 4: the
  // large); the same test as at the top, where it is made on the control block
  if ((main_phase == 3 && Bc > kSmallBuckets) || (main_phase == 4 && Bc <= kSmallBuckets)) return;
  const size_t sstride = main_phase ? (size_t)P.Bc_max : (size_t)Bc;  // between slab partials
  // what the statistics read from device memory, read before the bucket
  // stores below: a vector load after them would wait for every one of them
  const int32_t khat_in = st->khat;
  const double q_in = P.q, noise_rate_in = P.noise_rate, neg_log1mq_in = P.neg_log1mq, rho_in = P.rho;
  const uint32_t d_in = P.d;
  const bool cut_ties_in = P.cut_ties != 0u;
  // With the whole grid resident, an estimation loop leaves the memory system
  // to its signal's location loops until they have read their partials: the
  // location loops go on to the threshold and cutoff, the longer chain.  The
  // location loops have lower workgroup indices, so they were dispatched
  // first; the wait is bounded all the same.
  const bool est_wait = main_phase && P.est_wait;
  if (est_wait && loop >= P.L_loc) {
    if (threadIdx.x == 0) {
      const uint32_t target = P.L_loc * (uint32_t)(st->pass + 1);
      for (uint32_t spin = 0; spin < 4096u; ++spin) {
        if (__hip_atomic_load(&st->loc_loaded, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
        __builtin_amdgcn_s_sleep(8);
      }
    }
    __syncthreads();
  }
  const uint32_t tid = threadIdx.x, T = blockDim.x;

  // bucket DFT
  C *buf = reinterpret_cast<C *>(smem);
  auto dst_of = [&](uint32_t b) -> uint32_t {
    if (NDIM == 1) return bitrev(b, logB);
    return (bitrev(b >> logB, logB) << logB) | bitrev(b & (B - 1u), logB);
  };
  // the partials are added in slab (or row-wrap) order: the streamed 2D row
  // hash leaves one per row wrap, the row hash one in all, k_hash kSlabs; the
  // compensated FP32 fold adds them in FP64.  A thread's buckets have their
  // loads issued together.
  const uint32_t nsl = !main_phase ? (NDIM == 1 ? P.probe_slabs : 1u)
                       : P.rows2d == 1 ? 1u
                       : P.rows2d == 2 ? (min(P.alpha * B, P.n) >> logB)
                                       : main_slabs<DEV, NDIM>(P0, sig);
  if constexpr (sizeof(R) == 4) {
    // c64: two neighbouring buckets per 16-byte load (bucket counts and slab
    // strides are even), two pairs per thread in flight; the same order of
    // addition
    const bool comp = P.comp && !(main_phase && P.rows2d);
    for (uint32_t p0 = tid; 2u * p0 < Bc; p0 += 2u * T) {
      float4 u[2][kSlabs];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t p = p0 + (uint32_t)k * T;
#pragma unroll
        for (int sl = 0; sl < kSlabs; ++sl) {
          u[k][sl] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (2u * p < Bc && (uint32_t)sl < nsl)
            u[k][sl] = *reinterpret_cast<const float4 *>(yg + (size_t)sl * sstride + 2u * p);
        }
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t p = p0 + (uint32_t)k * T;
        float4 v = u[k][0];
        if (comp) {
          double a = v.x, b = v.y, c = v.z, d = v.w;
#pragma unroll
          for (int sl = 1; sl < kSlabs; ++sl) {
            a += (double)u[k][sl].x;
            b += (double)u[k][sl].y;
            c += (double)u[k][sl].z;
            d += (double)u[k][sl].w;
          }
          v = make_float4((float)a, (float)b, (float)c, (float)d);
        } else {
#pragma unroll
          for (int sl = 1; sl < kSlabs; ++sl) {
            const bool on = (uint32_t)sl < nsl;
            v.x += on ? u[k][sl].x : 0.f;
            v.y += on ? u[k][sl].y : 0.f;
            v.z += on ? u[k][sl].z : 0.f;
            v.w += on ? u[k][sl].w : 0.f;
          }
        }
        if (2u * p < Bc) {
          buf[lds_at<true>(dst_of(2u * p))] = make_float2(v.x, v.y);
          buf[lds_at<true>(dst_of(2u * p + 1u))] = make_float2(v.z, v.w);
        }
      }
    }
  } else {
    constexpr int kSumU = sizeof(R) == 4 ? 4 : 2;
    for (uint32_t b0 = tid; b0 < Bc; b0 += kSumU * T) {
      C u[kSumU][kSlabs];
#pragma unroll
      for (int k = 0; k < kSumU; ++k) {
        const uint32_t b = b0 + (uint32_t)k * T;
#pragma unroll
        for (int sl = 0; sl < kSlabs; ++sl) {
          u[k][sl].x = 0;
          u[k][sl].y = 0;
          if (b < Bc && (uint32_t)sl < nsl) u[k][sl] = yg[(size_t)sl * sstride + b];
        }
      }
#pragma unroll
      for (int k = 0; k < kSumU; ++k) {
        const uint32_t b = b0 + (uint32_t)k * T;
        C v = u[k][0];
        if (P.comp && !(main_phase && P.rows2d)) {
          double vx = v.x, vy = v.y;
#pragma unroll
          for (int sl = 1; sl < kSlabs; ++sl) {
            vx += (double)u[k][sl].x;
            vy += (double)u[k][sl].y;
          }
          v.x = (R)vx;
          v.y = (R)vy;
        } else {
#pragma unroll
          for (int sl = 1; sl < kSlabs; ++sl) {
            v.x += (uint32_t)sl < nsl ? u[k][sl].x : (R)0;
            v.y += (uint32_t)sl < nsl ? u[k][sl].y : (R)0;
          }
        }
        if (b < Bc) buf[lds_at<true>(dst_of(b))] = v;
      }
    }
  }
  __syncthreads();
  if (est_wait && loop < P.L_loc && threadIdx.x == 0)
    __hip_atomic_fetch_add(&st->loc_loaded, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (NDIM == 1) {
    // radix-16 passes once a pass has groups for half the workgroup
    if (logB >= 13)
      fft_axis<R, true, true>(buf, logB, 1, 0, 1);
    else
      fft_axis<R, true>(buf, logB, 1, 0, 1);
  } else {
    fft_axis<R, true, true>(buf, logB, B, B, 1);
    fft_axis<R, true, true>(buf, logB, B, 1, B);
  }
  // y_hat back to the workspace; for probe and location loops also
  // m_b = |y_hat_b|^2 and the largest key, kept in registers while the DFT
  // buffer is still being read, then m written over the buffer's front
  using K = typename CT<R>::K;
  const uint32_t per = (Bc + T - 1) / T;
  const bool stats = !(main_phase && loop >= P.L_loc);
  R mv[kBucketMaxPer];
  K kmax = 0, kmin = ~(K)0;
#pragma unroll
  for (int j = 0; j < kBucketMaxPer; ++j) {
    const uint32_t b = tid + (uint32_t)j * T;
    mv[j] = (R)-1;  // no bucket: below every threshold and select
    if ((uint32_t)j < per && b < Bc) {
      const C v = buf[lds_at<true>(b)];
      yg[b] = v;
      mv[j] = v.x * v.x + v.y * v.y;
      kmax = max(kmax, key_of(mv[j]));
      kmin = min(kmin, key_of(mv[j]));
    }
  }
  if (!stats) return;
  kmax = wave_extreme<true>(kmax);
  kmin = wave_extreme<false>(kmin);
  R *ms = reinterpret_cast<R *>(smem);
  // LDS after the DFT: m (probe levels; c128 also for the selects), then the
  // selects' histograms and scratch
  uint32_t *hist = reinterpret_cast<uint32_t *>(smem + (((size_t)Bc * sizeof(R) + 15) & ~(size_t)15));
  uint32_t *sh = hist + 1536;              // 32 words of scratch
  K *wmax = reinterpret_cast<K *>(sh + 32);  // one key per wave
  K *wmin = wmax + kBucketThreads / 64;
  __syncthreads();
  // m in LDS for the probe's neighbour tests, and in c128 for the selects
  // (c64 selects read the registers; c128's sixteen values would not fit)
  constexpr bool kRegSel = sizeof(R) == 4;
  if (!main_phase || !kRegSel) {
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      const uint32_t b = tid + (uint32_t)j * T;
      if ((uint32_t)j < per && b < Bc) ms[b] = mv[j];
    }
  }
  if ((tid & 63) == 0) {
    wmax[tid >> 6] = kmax;
    wmin[tid >> 6] = kmin;
  }
  __syncthreads();

  // threshold: noise floor from the floor(q (Bc-1))-th order statistic,
  // c_noise = ln(Bc / noise_rate), and the relative floor rho * max m
  {
    const uint32_t ln = tid & 63u, nw = (T + 63) / 64;
    kmax = wave_extreme<true>(ln < nw ? wmax[ln] : (K)0);
    kmin = wave_extreme<false>(ln < nw ? wmin[ln] : ~(K)0);
  }
  const R mmax = val_of(kmax);
  const uint32_t qi = (uint32_t)floor(q_in * (double)(Bc - 1));
  // location loops: the cutoff value v (the num-th largest above T, when
  // more than num values exceed T) is the overall order statistic of rank
  // Bc - num, so it is selected in the same passes as the noise floor
  uint32_t num = 0;
  R floor_m, vcut = 0;
  if (main_phase) {
    num = d_in * (uint32_t)max(khat_in, 0);
    if (num > Bc) num = Bc;
    const uint32_t kb = num > 0 ? Bc - num : 0u;
    if constexpr (kRegSel)
      select_regs<true>(mv, per, qi, kb, hist, sh + 24, kmin, kmax, floor_m, vcut);
    else
      radix_select2<R, kBucketMaxPer, false>(SelSrc<R, kBucketMaxPer, false>{mv, 0u, ms, Bc}, qi, kb, hist, sh + 24,
                                             kmin, kmax, floor_m, vcut);
  } else if constexpr (kRegSel) {
    R unused;
    select_regs<false>(mv, per, qi, 0u, hist, sh + 24, kmin, kmax, floor_m, unused);
  } else {
    floor_m = block_kth_smallest<R>(ms, Bc, qi, hist, sh, (R)-1, kmin, kmax);
  }
  const double c_noise = log((double)Bc / noise_rate_in);
  const double t1 = c_noise * ((double)floor_m / neg_log1mq_in);
  const double t2 = rho_in * (double)mmax;
  const double Td = t1 > t2 ? t1 : t2;
  const R Tr = (R)Td;

  if (!main_phase) {
    // local maxima among significant buckets (1D ring / 2D torus neighbours)
    uint32_t c = 0;
    if (NDIM == 1) {
      for (uint32_t b = tid; b < Bc; b += T) {
        if (!(ms[b] > Tr)) continue;
        c += key_gt(ms, b, (b - 1u) & (B - 1u)) && key_gt(ms, b, (b + 1u) & (B - 1u)) ? 1u : 0u;
      }
    } else {
      // four buckets of a row per step: the three rows' six columns around
      // them (wrapping on the torus) are read once and every bucket is
      // compared with its eight neighbours without branches (B >= 4)
      for (uint32_t b0 = 4u * tid; b0 < Bc; b0 += 4u * T) {
        const uint32_t b1 = b0 >> logB, c0 = b0 & (B - 1u);
        uint32_t ridx[3];
        R v[3][6];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          ridx[i] = ((b1 + (uint32_t)i - 1u) & (B - 1u)) << logB;
          const R *rowp = ms + ridx[i];
          v[i][0] = rowp[(c0 - 1u) & (B - 1u)];
#pragma unroll
          for (int j = 0; j < 4; ++j) v[i][1 + j] = rowp[c0 + (uint32_t)j];
          v[i][5] = rowp[(c0 + 4u) & (B - 1u)];
        }
        if constexpr (sizeof(R) == 4) {
          // (m, -index) as one 64-bit key: m_b > m_n, or m_b = m_n with b < n,
          // is key_b > key_n (m >= 0, so its bit pattern orders like m)
          unsigned long long kk[3][6];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 6; ++j) {
              const uint32_t idx = ridx[i] | ((c0 + (uint32_t)j - 1u) & (B - 1u));
              kk[i][j] = ((unsigned long long)key_of(v[i][j]) << 32) | (0xFFFFFFFFu - idx);
            }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const unsigned long long kb = kk[1][1 + j];
            bool is_max = v[1][1 + j] > Tr;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int dj = -1; dj <= 1; ++dj) {
                if (i == 1 && dj == 0) continue;
                is_max = is_max & (kb > kk[i][1 + j + dj]);
              }
            c += is_max ? 1u : 0u;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const R mb = v[1][1 + j];
            const uint32_t b = ridx[1] | (c0 + (uint32_t)j);
            bool is_max = mb > Tr;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int dj = -1; dj <= 1; ++dj) {
                if (i == 1 && dj == 0) continue;
                const R mn = v[i][1 + j + dj];
                const uint32_t nb = ridx[i] | ((c0 + (uint32_t)(j + dj)) & (B - 1u));
                is_max = is_max & (mb > mn || (mb == mn && b < nb));
              }
            c += is_max ? 1u : 0u;
          }
        }
      }
    }
    const uint32_t k = block_sum(c, &sh[4]);
    if (tid >= 64) return;
    // the last of the round's workgroups of this signal applies the rule;
    // it reads only the counts, themselves atomics, so no fence (an
    // agent-scope fence writes back and invalidates the L2).  A signal has
    // as many workgroups in the round as it has levels in it (a shorter
    // signal of an uneven batch may have fewer levels than the launch).
    const uint32_t in_round = min((uint32_t)iter + gridDim.x, P.probe_levels) - (uint32_t)iter;
    uint32_t last = 0;
    if (tid == 0) {
      ProbeRec *h = hist_of(P, sig) + level;
      h->B = (int32_t)B;
      h->dec = 0;
      h->T = Td;
      if ((int32_t)level != P.probe_drop)
        __hip_atomic_store(&h->k, (int32_t)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t prior = __hip_atomic_fetch_add(&st->round_blocks, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
      last = prior + 1u == in_round ? 1u : 0u;
      if (last) __hip_atomic_store(&st->round_blocks, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (__builtin_amdgcn_readfirstlane(last)) {
      // wave 0 reads the round's counts together, a lane per level, into
      // LDS words the selects no longer use; lane 0 then applies the rule
      int32_t *kv = reinterpret_cast<int32_t *>(hist);
      if (tid < in_round) kv[tid] = probe_count(P, hist_of(P, sig) + iter + tid);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (tid == 0) probe_control<NDIM>(P, sig, iter, iter + (int)in_round, kv, st0);
    }
    return;
  }

  // location loop: J = the min(num, #{m > T}) largest keys above T.  Taken
  // are the buckets above v, and of those equal to v the first `need` in
  // index order (v = T and need = 0 when all above T fit).  A thread's keys
  // are still in mv; the list is built in index order from 64-bucket chunks,
  // one wave ballot each, so no LDS pass runs over a thread's own chunk.
  // #{m > T} and #{m >= vcut} in one block sum (each at most 16384)
  uint32_t cnt2 = 0;
#pragma unroll
  for (int j = 0; j < kBucketMaxPer; ++j) {
    if ((uint32_t)j < per) cnt2 += (mv[j] > Tr ? 65536u : 0u) + (mv[j] >= vcut ? 1u : 0u);
  }
  cnt2 = block_sum(cnt2, &sh[4]);
  const uint32_t n_above = cnt2 >> 16, n_ge = cnt2 & 0xFFFFu;
  const uint32_t lane = tid & 63u;
  uint32_t *cg = hist, *ce = hist + 256;
  int32_t *jl = jlist_of(P, sig, loop);
  uint32_t *jb = jbits_of(P, sig, loop);
  // J is {m > T} when every bucket above T fits, else {m >= vcut} when no
  // more buckets equal vcut than the cutoff takes (the usual case: one);
  // otherwise the buckets above vcut and, of those equal to it, the first
  // `need` in index order
  const bool fits = n_above <= num;
  const R v = fits ? Tr : vcut;
  uint32_t total;
  if ((fits || n_ge == num) && !cut_ties_in) {
    // per chunk (a wave's 64 buckets of one j; Bc / 64 <= 256 of them): the
    // taken buckets' count and bitmap words, then one wave scans the counts
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      if ((uint32_t)j < per) {  // uniform over the block
        const uint32_t b0 = (tid & ~63u) + (uint32_t)j * T;
        const unsigned long long fm = __ballot(fits ? mv[j] > v : mv[j] >= v);
        if (lane == 0 && b0 < Bc) {
          cg[b0 >> 6] = (uint32_t)__popcll(fm);
          jb[b0 >> 5] = (uint32_t)fm;
          if (b0 + 32u < Bc) jb[(b0 >> 5) + 1] = (uint32_t)(fm >> 32);
        }
      }
    }
    __syncthreads();
    if (tid < 64) {
      const uint32_t nch = (Bc + 63u) >> 6;
      uint32_t g4[4], ss = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = 4u * tid + (uint32_t)i;
        g4[i] = c < nch ? cg[c] : 0u;
        ss += g4[i];
      }
      const uint32_t incl = wave_incl_scan(ss);
      uint32_t run = incl - ss;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = 4u * tid + (uint32_t)i;
        if (c < nch) cg[c] = run;
        run += g4[i];
      }
      if (tid == 63) sh[6] = incl;
    }
    __syncthreads();
    total = sh[6];
    // the list in index order
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      if ((uint32_t)j < per) {
        const uint32_t b0 = (tid & ~63u) + (uint32_t)j * T;
        const bool f = fits ? mv[j] > v : mv[j] >= v;
        const unsigned long long fm = __ballot(f);
        if (f) jl[cg[b0 >> 6] + lanes_below(fm)] = (int32_t)(b0 + lane);
      }
    }
  } else {
    uint32_t gt = 0;
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      if ((uint32_t)j < per) gt += mv[j] > vcut ? 1u : 0u;
    }
    const uint32_t need = num - block_sum(gt, &sh[4]);
    // per chunk (Bc / 64 <= 256 of them): buckets above v, buckets equal to v
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      if ((uint32_t)j < per) {  // uniform over the block
        const uint32_t b0 = (tid & ~63u) + (uint32_t)j * T, b = b0 + lane;
        const unsigned long long g = __ballot(b < Bc && mv[j] > v);
        const unsigned long long e = __ballot(b < Bc && need > 0u && mv[j] == v);
        if (lane == 0 && b0 < Bc) {
          cg[b0 >> 6] = (uint32_t)__popcll(g);
          ce[b0 >> 6] = (uint32_t)__popcll(e);
        }
      }
    }
    __syncthreads();
    if (tid < 64) {
      // one wave scans the chunks, four per lane: ties before each chunk, then
      // list positions (the chunk's taken ties are the first `need` overall)
      const uint32_t nch = (Bc + 63u) >> 6;
      uint32_t g4[4], e4[4], te[4], sel[4], es = 0, ss = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = 4u * tid + (uint32_t)i;
        g4[i] = c < nch ? cg[c] : 0u;
        e4[i] = c < nch ? ce[c] : 0u;
        es += e4[i];
      }
      uint32_t run = wave_incl_scan(es) - es;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        te[i] = run;
        run += e4[i];
        sel[i] = g4[i] + min(e4[i], need > te[i] ? need - te[i] : 0u);
        ss += sel[i];
      }
      const uint32_t incl = wave_incl_scan(ss);
      run = incl - ss;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = 4u * tid + (uint32_t)i;
        if (c < nch) {
          cg[c] = run;
          ce[c] = te[i];
        }
        run += sel[i];
      }
      if (tid == 63) sh[6] = incl;
    }
    __syncthreads();
    total = sh[6];
    // the list in index order and the cutoff bitmap, one ballot per chunk
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      if ((uint32_t)j < per) {  // uniform over the block
        const uint32_t b0 = (tid & ~63u) + (uint32_t)j * T, b = b0 + lane;
        const bool ok = b < Bc;
        const bool eq = ok && need > 0u && mv[j] == v;
        const unsigned long long e = __ballot(eq);
        const uint32_t c = b0 >> 6;
        const bool f = (ok && mv[j] > v) || (eq && ce[c] + lanes_below(e) < need);
        const unsigned long long fm = __ballot(f);
        if (f) jl[cg[c] + lanes_below(fm)] = (int32_t)b;
        if (lane == 0 && b0 < Bc) {
          jb[b0 >> 5] = (uint32_t)fm;
          if (b0 + 32u < Bc) jb[(b0 >> 5) + 1] = (uint32_t)(fm >> 32);
        }
      }
    }
  }
  if (tid == 0) {
    jcount_of(P, sig)[loop] = (int32_t)total;
    tloc_of(P, sig)[loop] = Td;
  }
}

// ------------------------------------------------ large 2D bucket arrays ----

// 2D bucket arrays above the LDS-resident size (B x B > lds_cap, up to
// 1024 x 1024: the known-k form at the sparse FFT's bucket count, B =
// sqrt(N k) per axis, and probe levels and main loops of plans whose B_max
// goes beyond the LDS) are transformed and cut in device memory: k_big_rows
// adds a bucket row's row-wrap partials and takes its B-point DFT along b2,
// k_big_cols takes the B-point DFTs along b1 of a block of big_cols()
// columns, and k_big_stats computes m = |y|^2, the noise floor and T, then
// either the top-num cutoff J (location loops) or the local-maximum count
// and the B-update rule (probe levels), with the selects over device
// memory.  The results sit where k_bucket leaves them (y_hat in the first
// partial slot, m in a spare one, J as bitmap and list).  The in-LDS kernels
// skip such arrays and these kernels skip the others, so a batch may mix them.

// The array a large-array kernel works on: role 0 main loop `idx` (its
// row-wrap partials at stride Bc_max, m written into the second), role 1
// probe level `idx` (one partial; m written after it).  `ok` is false when
// the signal does not run it here (finished, beyond its levels, or an array
// that k_bucket holds in LDS).
template <typename C> struct BigArr {
  C *y;
  uint32_t B, parts;
  size_t pstride;
  bool ok;
};
template <typename C>
__device__ __forceinline__ BigArr<C> big_arr(const KParams &P, uint32_t sig, int role, uint32_t idx) {
  BigArr<C> a;
  a.ok = false;
  a.y = nullptr;
  a.B = 0;
  a.parts = 0;
  a.pstride = 0;
  const SigState *st = state_of(P, sig);
  if (role == 0) {
    if ((st->status & kSigEmpty) || st->pass != (int32_t)P.pass) return a;
    a.B = (uint32_t)st->B_star;
    a.y = ymain_of<C>(P, sig, idx);
    a.parts = min(P.alpha * a.B, P.n) >> ilog2(a.B);
    a.pstride = P.Bc_max;
  } else {
    if (st->done || idx >= P.probe_levels) return a;
    a.B = P.B0 << idx;
    a.y = yprobe_of<C>(P, sig, idx);
    a.parts = 1;
    a.pstride = (size_t)a.B * a.B;
  }
  a.ok = (size_t)a.B * a.B > (size_t)P.lds_cap;
  return a;
}

constexpr uint32_t kBigChunk = 4096;
constexpr uint32_t kBigThreads = 256;
constexpr uint32_t kBigChunks = kBigMax * kBigMax / kBigChunk;
struct BigStat {
  unsigned long long kmin, kmax;      // extreme keys of m
  unsigned long long pa, pb, mask;    // prefixes (of key - kmin) of the two searches, settled digits
  uint32_t ka, kb;                    // their ranks within the prefixes
  uint32_t n_above, n_ge, n_gt, nmax; // #{m > T}, #{m >= v}, #{m > v}; local maxima (probe)
  uint32_t num, need, mode, pad;      // mode 1: J = {m > T}; 2: {m >= v}; 3: above v, then ties in order
  double T, vcut;
  uint32_t hist[2][256];
  uint32_t ctake[kBigChunks], ctie[kBigChunks];  // per chunk: counts, then list positions and ties before
};
template <typename C> __device__ __forceinline__ BigStat *big_stat(const BigArr<C> &a) {
  return reinterpret_cast<BigStat *>(a.y + 2 * a.pstride);
}
template <typename R> __device__ __forceinline__ R *big_m(const BigArr<typename CT<R>::C> &a) {
  return reinterpret_cast<R *>(a.y + a.pstride);
}

// one workgroup per (bucket row b1, loop or level, signal)
template <typename R>
__global__ __launch_bounds__(256) void k_big_rows(KParams P, int role, int iter) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  C *buf = reinterpret_cast<C *>(smem);
  const uint32_t b1 = blockIdx.x, sig = blockIdx.z;
  const BigArr<C> ar = big_arr<C>(P, sig, role, (uint32_t)iter + blockIdx.y);
  if (!ar.ok || b1 >= ar.B) return;
  const uint32_t B = ar.B, logB = ilog2(B);
  C *y = ar.y;
  const size_t row = (size_t)b1 << logB;
  for (uint32_t b2 = threadIdx.x; b2 < B; b2 += blockDim.x) {
    C v = y[row + b2];
    for (uint32_t r = 1; r < ar.parts; ++r) {
      const C u = y[(size_t)r * ar.pstride + row + b2];
      v.x += u.x;
      v.y += u.y;
    }
    buf[lds_at<true>(bitrev(b2, logB))] = v;
  }
  __syncthreads();
  fft_axis<R, true>(buf, logB, 1, 0, 1);
  for (uint32_t b2 = threadIdx.x; b2 < B; b2 += blockDim.x) y[row + b2] = buf[lds_at<true>(b2)];
}

template <typename R> constexpr uint32_t big_cols() { return sizeof(R) == 4 ? 16u : 8u; }

// one workgroup per (block of big_cols() columns, loop or level, signal)
template <typename R>
__global__ __launch_bounds__(1024) void k_big_cols(KParams P, int role, int iter) {
  using C = typename CT<R>::C;
  constexpr uint32_t CB = big_cols<R>();
  extern __shared__ __align__(16) unsigned char smem[];
  C *buf = reinterpret_cast<C *>(smem);
  const uint32_t sig = blockIdx.z;
  const BigArr<C> ar = big_arr<C>(P, sig, role, (uint32_t)iter + blockIdx.y);
  const uint32_t c0 = blockIdx.x * CB;
  if (!ar.ok || c0 >= ar.B) return;
  const uint32_t B = ar.B, logB = ilog2(B);
  C *y = ar.y;
  if (blockIdx.x == 0) {
    // the array's statistics record, in a partial slot the row pass has
    // consumed: zero, with the smallest key at its largest value
    uint32_t *w = reinterpret_cast<uint32_t *>(y + 2 * ar.pstride);
    for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(BigStat) / 4); i += blockDim.x) w[i] = i < 2 ? ~0u : 0u;
  }
  for (uint32_t i = threadIdx.x; i < B * CB; i += blockDim.x) {
    const uint32_t b1 = i / CB, c = i % CB;
    buf[lds_at<true>(bitrev(b1, logB) * CB + c)] = y[((size_t)b1 << logB) + c0 + c];
  }
  __syncthreads();
  fft_axis<R, true>(buf, logB, CB, 1, CB);
  for (uint32_t i = threadIdx.x; i < B * CB; i += blockDim.x) {
    const uint32_t b1 = i / CB, c = i % CB;
    y[((size_t)b1 << logB) + c0 + c] = buf[lds_at<true>(b1 * CB + c)];
  }
}

// The statistics of a large array are spread over many workgroups, a launch
// per step: a 256-thread workgroup per (4096-bucket chunk, array, signal), or
// per (array, signal) for the picks and the end step.  An array's running
// state is a BigStat record in a spare partial slot (slot 2; k_big_cols zeroes
// it).  The steps: m = |y|^2 and its key range; per 8-bit digit a histogram
// and a pick, for the noise floor's rank and, in location loops, the cutoff
// value's rank Bc - num at once (as in k_bucket); the counts above T and at
// or above the cutoff value (location) or the local maxima (probe); the
// B-update rule (probe) or the cutoff's mode (location); then per chunk the
// taken buckets' count, a scan over the chunks, and the list and bitmap.
// The digit of rank k in a 256-bin histogram (LDS or device memory), uniform
// over the calling wave; k becomes the rank within the digit's bin.
__device__ __forceinline__ uint32_t wave_pick_digit(const uint32_t *h, uint32_t &k) {
  const uint32_t l = threadIdx.x & 63u;
  const uint32_t c0 = h[4 * l], c1 = h[4 * l + 1], c2 = h[4 * l + 2], c3 = h[4 * l + 3];
  const uint32_t s = c0 + c1 + c2 + c3;
  const uint32_t incl = wave_incl_scan(s), excl = incl - s;
  const unsigned long long m = __ballot(excl <= k && k < incl);
  const uint32_t src = m ? (uint32_t)__builtin_ctzll(m) : 0u;
  uint32_t digit, run;
  if (k < excl + c0) {
    digit = 4 * l;
    run = excl;
  } else if (k < excl + c0 + c1) {
    digit = 4 * l + 1;
    run = excl + c0;
  } else if (k < excl + c0 + c1 + c2) {
    digit = 4 * l + 2;
    run = excl + c0 + c1;
  } else {
    digit = 4 * l + 3;
    run = excl + c0 + c1 + c2;
  }
  k = lane_value(k - run, src);
  return lane_value(digit, src);
}

// the chunk of a (chunk, array, signal) workgroup, or false when it has none
template <typename C>
__device__ __forceinline__ bool big_chunk(const KParams &P, int role, int iter, BigArr<C> &ar, uint32_t &b0) {
  ar = big_arr<C>(P, blockIdx.z, role, (uint32_t)iter + blockIdx.y);
  b0 = blockIdx.x * kBigChunk;
  return ar.ok && b0 < ar.B * ar.B;
}

template <typename R>
__global__ __launch_bounds__(kBigThreads) void k_bs_m(KParams P, int role, int iter) {
  using C = typename CT<R>::C;
  using K = typename CT<R>::K;
  __shared__ K wk[2 * (kBigThreads / 64)];
  BigArr<C> ar;
  uint32_t b0;
  if (!big_chunk(P, role, iter, ar, b0)) return;
  R *m = big_m<R>(ar);
  K kmax = 0, kmin = ~(K)0;
  for (uint32_t b = b0 + threadIdx.x; b < b0 + kBigChunk; b += kBigThreads) {
    const C v = ar.y[b];
    const R mb = v.x * v.x + v.y * v.y;
    m[b] = mb;
    kmax = max(kmax, key_of(mb));
    kmin = min(kmin, key_of(mb));
  }
  kmax = wave_extreme<true>(kmax);
  kmin = wave_extreme<false>(kmin);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  if (lane == 0) {
    wk[2 * wave] = kmax;
    wk[2 * wave + 1] = kmin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < kBigThreads / 64; ++w) {
      kmax = max(kmax, wk[2 * w]);
      kmin = min(kmin, wk[2 * w + 1]);
    }
    BigStat *bs = big_stat(ar);
    atomicMax(&bs->kmax, (unsigned long long)kmax);
    atomicMin(&bs->kmin, (unsigned long long)kmin);
  }
}

// the digit pass `pass` of an array: its top bit, width and shift (width 0:
// the selection is complete)
template <typename K>
__device__ __forceinline__ int big_pass(const BigStat *bs, int pass, int &shift) {
  const K lo = (K)bs->kmin, hi = (K)bs->kmax;
  const int nbits = hi > lo ? bit_length(hi - lo) : 1;
  const int top = nbits - 8 * pass;
  const int width = top <= 0 ? 0 : (top < 8 ? top : 8);
  shift = top - width;
  return width;
}

template <typename R>
__global__ __launch_bounds__(kBigThreads) void k_bs_hist(KParams P, int role, int iter, int pass) {
  using C = typename CT<R>::C;
  using K = typename CT<R>::K;
  __shared__ uint32_t h[512];
  BigArr<C> ar;
  uint32_t b0;
  if (!big_chunk(P, role, iter, ar, b0)) return;
  BigStat *bs = big_stat(ar);
  int shift;
  const int width = big_pass<K>(bs, pass, shift);
  if (width == 0) return;
  const uint32_t dmask = (1u << width) - 1u;
  const K lo = (K)bs->kmin, pa = (K)bs->pa, pb = (K)bs->pb, mask = (K)bs->mask;
  const bool two = role == 0;
  for (uint32_t i = threadIdx.x; i < 512; i += kBigThreads) h[i] = 0;
  __syncthreads();
  const R *m = big_m<R>(ar);
  for (uint32_t b = b0 + threadIdx.x; b < b0 + kBigChunk; b += kBigThreads) {
    const K key = key_of(m[b]) - lo, kp = key & mask;
    const uint32_t bin = (uint32_t)(key >> shift) & dmask;
    if (kp == pa)
      atomicAdd(&h[bin], 1u);
    else if (two && kp == pb)
      atomicAdd(&h[256 + bin], 1u);
  }
  __syncthreads();
  uint32_t *g = &bs->hist[0][0];
  for (uint32_t i = threadIdx.x; i < 512; i += kBigThreads)
    if (h[i]) atomicAdd(&g[i], h[i]);
}

// one workgroup of two waves per (array, signal): wave 0 picks the noise
// floor's digit, wave 1 (location loops) the cutoff value's; after the last
// digit the threshold T and the cutoff value
template <typename R>
__global__ __launch_bounds__(128) void k_bs_pick(KParams P, int role, int iter, int pass) {
  using C = typename CT<R>::C;
  using K = typename CT<R>::K;
  const uint32_t sig = blockIdx.y, idx = (uint32_t)iter + blockIdx.x;
  const BigArr<C> ar = big_arr<C>(P, sig, role, idx);
  if (!ar.ok) return;
  BigStat *bs = big_stat(ar);
  int shift;
  const int width = big_pass<K>(bs, pass, shift);
  if (width == 0) return;
  const uint32_t dmask = (1u << width) - 1u;
  const uint32_t Bc = ar.B * ar.B;
  uint32_t ka = bs->ka, kb = bs->kb, num = bs->num;
  if (pass == 0) {
    ka = (uint32_t)floor(P.q * (double)(Bc - 1));
    num = 0;
    if (role == 0) {
      num = (uint32_t)P.d * (uint32_t)max(state_of(P, sig)->khat, 0);
      if (num > Bc) num = Bc;
    }
    kb = num > 0 ? Bc - num : 0u;
  }
  const K lo = (K)bs->kmin, pa = (K)bs->pa, pb = (K)bs->pb;
  const bool second = threadIdx.x >= 64;
  uint32_t digit = 0, k = second ? kb : ka;
  if (!second || role == 0) digit = wave_pick_digit(second && pa != pb ? bs->hist[1] : bs->hist[0], k);
  __syncthreads();  // both waves have read the histograms
  uint32_t *g = &bs->hist[0][0];
  for (uint32_t i = threadIdx.x; i < 512; i += blockDim.x) g[i] = 0;
  if ((threadIdx.x & 63u) == 0) {
    if (!second) {
      const K p = pa | ((K)digit << shift);
      bs->pa = p;
      bs->ka = k;
      bs->mask = bs->mask | ((unsigned long long)dmask << shift);
      bs->num = num;
      if (shift == 0) {
        // threshold as in k_bucket
        const double floor_m = (double)val_of((K)(p + lo));
        const double c_noise = log((double)Bc / P.noise_rate);
        const double t1 = c_noise * (floor_m / P.neg_log1mq);
        const double t2 = P.rho * (double)val_of((K)bs->kmax);
        bs->T = t1 > t2 ? t1 : t2;
      }
    } else if (role == 0) {
      const K p = pb | ((K)digit << shift);
      bs->pb = p;
      bs->kb = k;
      if (shift == 0) bs->vcut = (double)val_of((K)(p + lo));
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kBigThreads) void k_bs_count(KParams P, int role, int iter) {
  using C = typename CT<R>::C;
  __shared__ uint32_t sh[16];
  BigArr<C> ar;
  uint32_t b0;
  if (!big_chunk(P, role, iter, ar, b0)) return;
  BigStat *bs = big_stat(ar);
  const R *m = big_m<R>(ar);
  const R Tr = (R)bs->T;
  if (role == 0) {
    const R v = (R)bs->vcut;
    uint32_t a = 0, g = 0, t = 0;
    for (uint32_t b = b0 + threadIdx.x; b < b0 + kBigChunk; b += kBigThreads) {
      const R mb = m[b];
      a += mb > Tr ? 1u : 0u;
      g += mb >= v ? 1u : 0u;
      t += mb > v ? 1u : 0u;
    }
    const uint32_t ag = block_sum(a | (g << 16), sh), tt = block_sum(t, sh);
    if (threadIdx.x == 0) {
      atomicAdd(&bs->n_above, ag & 0xFFFFu);
      atomicAdd(&bs->n_ge, ag >> 16);
      atomicAdd(&bs->n_gt, tt);
    }
  } else {
    // local maxima among significant buckets, the 8-neighbourhood on the
    // torus, strict on the key (m, -index)
    const uint32_t B = ar.B, logB = ilog2(B);
    uint32_t c = 0;
    for (uint32_t b = b0 + threadIdx.x; b < b0 + kBigChunk; b += kBigThreads) {
      if (!(m[b] > Tr)) continue;
      const uint32_t r = b >> logB, q = b & (B - 1u);
      bool is_max = true;
      for (int dr = -1; dr <= 1; ++dr)
        for (int dq = -1; dq <= 1; ++dq) {
          if (dr == 0 && dq == 0) continue;
          const uint32_t nb = (((r + (uint32_t)dr) & (B - 1u)) << logB) | ((q + (uint32_t)dq) & (B - 1u));
          is_max = is_max && key_gt(m, b, nb);
        }
      c += is_max ? 1u : 0u;
    }
    c = block_sum(c, sh);
    if (threadIdx.x == 0) atomicAdd(&bs->nmax, c);
  }
}

// one thread per (array, signal): the probe level's count and its B-update
// rule (a large level is a round of its own), or the location loop's T and
// cutoff mode
template <typename R>
__global__ __launch_bounds__(64) void k_bs_end(KParams P, int role, int iter) {
  using C = typename CT<R>::C;
  if (threadIdx.x != 0) return;
  const uint32_t sig = blockIdx.y, idx = (uint32_t)iter + blockIdx.x;
  const BigArr<C> ar = big_arr<C>(P, sig, role, idx);
  if (!ar.ok) return;
  BigStat *bs = big_stat(ar);
  if (role == 1) {
    ProbeRec *h = hist_of(P, sig) + idx;
    h->B = (int32_t)ar.B;
    h->dec = 0;
    h->T = bs->T;
    if ((int32_t)idx != P.probe_drop)
      __hip_atomic_store(&h->k, (int32_t)bs->nmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t kv = probe_count(P, h);
    probe_control<2>(P, sig, (int)idx, (int)idx + 1, &kv, *state_of(P, sig));
    return;
  }
  tloc_of(P, sig)[idx] = bs->T;
  const uint32_t num = bs->num;
  const bool fits = bs->n_above <= num;
  bs->mode = fits ? 1u : (bs->n_ge == num && !P.cut_ties ? 2u : 3u);
  bs->need = fits ? 0u : num - bs->n_gt;
}

// location loops: the buckets of a chunk the cutoff takes (J) and, in mode 3,
// those equal to the cutoff value v (of which the first `need` are taken)
template <typename R>
__device__ __forceinline__ void big_take(const BigStat *bs, R mb, bool &f0, bool &eq) {
  const uint32_t mode = bs->mode;
  const R v = mode == 1 ? (R)bs->T : (R)bs->vcut;
  f0 = mode == 2 ? mb >= v : mb > v;
  eq = mode == 3 && mb == v;
}

template <typename R>
__global__ __launch_bounds__(kBigThreads) void k_bs_chunks(KParams P, int iter) {
  using C = typename CT<R>::C;
  __shared__ uint32_t sh[16];
  BigArr<C> ar;
  uint32_t b0;
  if (!big_chunk(P, 0, iter, ar, b0)) return;
  BigStat *bs = big_stat(ar);
  const R *m = big_m<R>(ar);
  uint32_t g = 0, e = 0;
  for (uint32_t b = b0 + threadIdx.x; b < b0 + kBigChunk; b += kBigThreads) {
    bool f0, eq;
    big_take<R>(bs, m[b], f0, eq);
    g += f0 ? 1u : 0u;
    e += eq ? 1u : 0u;
  }
  const uint32_t ge = block_sum(g | (e << 16), sh);
  if (threadIdx.x == 0) {
    bs->ctake[blockIdx.x] = ge & 0xFFFFu;
    bs->ctie[blockIdx.x] = ge >> 16;
  }
}

// one workgroup per (array, signal), a thread per chunk: ties before each
// chunk, then its first list position (the first `need` ties are taken)
template <typename R>
__global__ __launch_bounds__(kBigChunks) void k_bs_scan(KParams P, int iter) {
  using C = typename CT<R>::C;
  __shared__ uint32_t sh[32];
  const uint32_t sig = blockIdx.y, idx = (uint32_t)iter + blockIdx.x;
  const BigArr<C> ar = big_arr<C>(P, sig, 0, idx);
  if (!ar.ok) return;
  BigStat *bs = big_stat(ar);
  const uint32_t nch = ar.B * ar.B / kBigChunk, t = threadIdx.x, need = bs->need;
  const uint32_t take = t < nch ? bs->ctake[t] : 0u, tie = t < nch ? bs->ctie[t] : 0u;
  const uint32_t te = block_excl_scan(tie, sh);
  const uint32_t sel = take + min(tie, need > te ? need - te : 0u);
  uint32_t total;
  const uint32_t pos = block_excl_scan(sel, sh, &total);
  if (t < nch) {
    bs->ctake[t] = pos;
    bs->ctie[t] = te;
  }
  if (t == 0) jcount_of(P, sig)[idx] = (int32_t)total;
}

// per chunk: the list in index order and the bitmap, a 64-bucket run per
// ballot (a wave takes 16 consecutive runs)
template <typename R>
__global__ __launch_bounds__(kBigThreads) void k_bs_list(KParams P, int iter) {
  using C = typename CT<R>::C;
  __shared__ uint32_t sg[64], se[64];
  BigArr<C> ar;
  uint32_t b0;
  if (!big_chunk(P, 0, iter, ar, b0)) return;
  const BigStat *bs = big_stat(ar);
  const R *m = big_m<R>(ar);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, need = bs->need;
  for (uint32_t r = wave; r < 64; r += kBigThreads / 64) {
    const uint32_t b = b0 + 64 * r + lane;
    bool f0, eq;
    big_take<R>(bs, m[b], f0, eq);
    const unsigned long long g = __ballot(f0), e = __ballot(eq);
    if (lane == 0) {
      sg[r] = (uint32_t)__popcll(g);
      se[r] = (uint32_t)__popcll(e);
    }
  }
  __syncthreads();
  if (wave == 0) {
    // the runs' ties before them and list positions, from the chunk's
    const uint32_t tie0 = bs->ctie[blockIdx.x], pos0 = bs->ctake[blockIdx.x];
    const uint32_t e = se[lane], g = sg[lane];
    const uint32_t te = tie0 + wave_incl_scan(e) - e;
    const uint32_t sel = g + min(e, need > te ? need - te : 0u);
    const uint32_t pos = pos0 + wave_incl_scan(sel) - sel;
    sg[lane] = pos;
    se[lane] = te;
  }
  __syncthreads();
  int32_t *jl = jlist_of(P, blockIdx.z, (uint32_t)iter + blockIdx.y);
  uint32_t *jb = jbits_of(P, blockIdx.z, (uint32_t)iter + blockIdx.y);
  for (uint32_t r = wave; r < 64; r += kBigThreads / 64) {
    const uint32_t b = b0 + 64 * r + lane;
    bool f0, eq;
    big_take<R>(bs, m[b], f0, eq);
    const unsigned long long e = __ballot(eq);
    const bool f = f0 || (eq && se[r] + lanes_below(e) < need);
    const unsigned long long fm = __ballot(f);
    if (f) jl[sg[r] + lanes_below(fm)] = (int32_t)b;
    if (lane == 0) {
      jb[(b0 >> 5) + 2 * r] = (uint32_t)fm;
      jb[(b0 >> 5) + 2 * r + 1] = (uint32_t)(fm >> 32);
    }
  }
}

// -------------------------------------------------------------- k_vote ----

constexpr uint32_t kVoteBlock2d = 4;  // 2D vote: a thread's block of row x column preimages

// Reverse hash and vote (Algorithm 1/2): votes(f) = #{l : h_l(f) in J_l},
// S = {f : votes >= T_vote}.  Any f in S is in J_l for at least one of the
// first E = L_loc - T_vote + 1 loops, so the candidates are the preimages of
// those loops' selected buckets; a candidate is emitted only by the first of
// those loops that holds it, which makes S duplicate-free with no sort and
// no n-sized histogram.  The cutoff bitmaps sit in LDS.
//
// A candidate of loop e has one vote; it is tested against the other loops in
// index order, and after m tests with v hits it can still reach T_vote only
// if v >= m - (L_loc - T_vote).  No candidate can fail before the first
// L_loc - T_vote + 1 tests, so those run for every candidate without
// branches, kVoteIlp candidates per thread (2, 4 and 8 measured at n = 2^22,
// batch 32: 76, 64 and 70 us); the few candidates still alive
// then go through an LDS queue, so that the remaining tests, which stop at
// the first hopeless miss, run only on them.  In 2D a loop's bucket of (f1, f2)
// is the pair of its bucket of f1 along rows and of f2 along columns, so a
// thread tests a block of row x column preimages with one axis hash per row
// and per column instead of two per pair.  SMALL: every hash product fits
// 24-bit operands (1D n <= 2^24, and 2D), so the full-rate 24-bit multiply
// gives the product modulo n.
// GB: the cutoff bitmaps are read from device memory (the L2) where they do
// not fit in LDS (the large 2D bucket arrays).
template <int NDIM, bool SMALL, bool DEV = false, bool GB = false>
__global__ __launch_bounds__(kVoteThreads) void k_vote(KParams P0) {
  extern __shared__ uint32_t s_bits[];  // [L_loc][words]
  constexpr int K = kVoteIlp;
  constexpr uint32_t KB = kVoteBlock2d;
  // survivors of one round of first tests: K per thread, 2D KB x KB
  constexpr uint32_t QCAP = kVoteThreads * (NDIM == 2 ? KB * KB : (uint32_t)K);
  __shared__ uint32_t s_qf[QCAP];
  __shared__ uint8_t s_qv[QCAP];
  __shared__ uint32_t s_qn;
  const uint32_t e = blockIdx.y, sig = blockIdx.z;
  // the control block and the cutoff counts have every length's slice layout,
  // and the signal's length is its own: a workgroup with no work items leaves
  // before the per-length parameters are read (see k_hash)
  SigState *st = state_of(P0, sig);
  if ((st->status & kSigEmpty) || st->pass != (int32_t)P0.pass) return;
  const int it0 = kPassIter * st->pass;
  const uint32_t ncand = (uint32_t)jcount_of(P0, sig)[e];
  const uint32_t B = (uint32_t)st->B_star, logB = ilog2(B);
  const uint32_t Bc = NDIM == 1 ? B : B * B;
  const uint32_t logn = sig_logn<DEV>(P0, sig);
  const uint32_t logW = logn - logB, W = 1u << logW, c = W >> 1;
  // workgroup work items: selected buckets, or in 2D rounds of KB x KB blocks
  const bool blocks2 = NDIM == 2 && logW >= 2u;
  // otherwise (bucket, preimage) pairs, K per thread
  const uint32_t logPer = NDIM == 1 ? logW : 2u * logW;
  const uint32_t items = blocks2 ? ((ncand << (2u * (logW - 2u))) + blockDim.x - 1u) / blockDim.x
                                 : ((ncand << logPer) + (uint32_t)K * blockDim.x - 1u) / ((uint32_t)K * blockDim.x);
  if (blockIdx.x >= items) return;
  const KParams &P = params_of<DEV>(P0, sig);
  if ((Bc > P.lds_cap) != GB) return;  // bitmaps in LDS, or (GB) of the large arrays in device memory
  const uint32_t n = P.n, mask = n - 1u;
  const uint32_t L = P.L_loc, Tv = P.T_vote;
  const uint32_t words = (Bc + 31) >> 5;
  // tests before a candidate can fail; the slack of misses it may take
  const uint32_t slack = L - Tv, nA = min(slack + 1u, L - 1u);
  __shared__ uint32_t s_sig[kMaxLoops][2];
  if (threadIdx.x < L) {
    s_sig[threadIdx.x][0] = draw(P, sig, kPhaseLoc, it0 + (int)threadIdx.x, 0).sigma;
    s_sig[threadIdx.x][1] = NDIM == 2 ? draw(P, sig, kPhaseLoc, it0 + (int)threadIdx.x, 1).sigma : 0u;
  }
  if (threadIdx.x == 0) s_qn = 0;
  // the bitmaps: loop l's word i at bsrc[l * bstride + i]
  const uint32_t *bsrc = GB ? jbits_of(P, sig, 0) : s_bits;
  const uint32_t bstride = GB ? (uint32_t)(P.lay.jbits_loop / 4) : words;
  if (!GB)
    for (uint32_t i = threadIdx.x; i < L * words; i += blockDim.x) {
      const uint32_t l = i / words, wi = i - l * words;
      s_bits[i] = jbits_of(P, sig, l)[wi];
    }
  __syncthreads();
  const int32_t *jl = jlist_of(P, sig, e);
  const uint32_t inv0 = inv_odd(s_sig[e][0]) & mask;
  const uint32_t inv1 = NDIM == 2 ? (inv_odd(s_sig[e][1]) & mask) : 0u;
  uint32_t *S = S_of(P, sig);

  auto mulmod = [&](uint32_t a, uint32_t b) -> uint32_t { return (SMALL ? __umul24(a, b) : a * b) & mask; };
  // bucket of f along one axis: bits logW .. logn - 1 of sigma f + c, the
  // product taken modulo 2^32
  auto axis = [&](uint32_t sg, uint32_t f) -> uint32_t {
    return __builtin_amdgcn_ubfe((SMALL ? __umul24(sg, f) : sg * f) + c, logW, logB);
  };
  auto bucket = [&](uint32_t l, uint32_t f) -> uint32_t {
    if (NDIM == 1) return axis(s_sig[l][0], f);
    return (axis(s_sig[l][0], f >> logn) << logB) | axis(s_sig[l][1], f & mask);
  };
  // the bit extract takes the bit index modulo 32 by itself
  auto in_J = [&](uint32_t l, uint32_t h) -> uint32_t {
    return __builtin_amdgcn_ubfe(bsrc[l * bstride + (h >> 5)], h, 1u);
  };
  // the m-th loop other than e
  auto other = [&](uint32_t m) -> uint32_t { return m < e ? m : m + 1u; };
  // a candidate with all its votes counted: emitted unless an earlier
  // candidate loop also holds it
  auto emit = [&](uint32_t f) {
    for (uint32_t e2 = 0; e2 < e; ++e2)
      if (in_J(e2, bucket(e2, f))) return;
    const uint32_t pos = atomicAdd(&st->count, 1u);
    if (pos < P.max_out) S[pos] = f;
  };

  const uint32_t T = blockDim.x;
  // a candidate after its first nA tests: emitted, queued for the rest of its
  // tests, or dropped
  auto keep = [&](uint32_t f, uint32_t v) {
    if (v + slack >= nA && v < 0x80000000u) {
      if (nA == L - 1u) {
        if (1u + v >= Tv) emit(f);
      } else {
        const uint32_t q = atomicAdd(&s_qn, 1u);
        s_qf[q] = f;
        s_qv[q] = (uint8_t)v;
      }
    }
  };
  // the queued candidates' remaining tests, which stop at the first hopeless
  // miss; every thread of the block calls this the same number of times
  auto drain = [&]() {
    __syncthreads();
    const uint32_t qn = s_qn;
    for (uint32_t q = threadIdx.x; q < qn; q += T) {
      const uint32_t fq = s_qf[q];
      uint32_t vq = s_qv[q];
      uint32_t m = nA;
      for (; m < L - 1u && vq + slack >= m; ++m) vq += in_J(other(m), bucket(other(m), fq));
      if (vq + slack >= m && 1u + vq >= Tv) emit(fq);
    }
    __syncthreads();
    if (threadIdx.x == 0) s_qn = 0;
    // the next round's pushes come after this barrier
    __syncthreads();
  };

  if (blocks2) {
    // The W x W preimages of a selected bucket (b1, b2) are the pairs of its W
    // row preimages f1 and W column preimages f2, and a loop hashes (f1, f2)
    // to the pair of its axis buckets.  A thread takes a KB x KB block of one
    // bucket's preimages: per loop it hashes KB row and KB column values and
    // makes KB^2 bitmap tests.  The block's threads cover consecutive blocks
    // of the selected buckets in list order.
    const uint32_t lq = logW - 2u;  // block index bits per axis
    const uint32_t logQ = 2u * lq;
    const uint32_t units = ncand << logQ;
    for (uint32_t u0 = blockIdx.x * T; u0 < units; u0 += gridDim.x * T) {
      const uint32_t u = u0 + threadIdx.x;
      const bool real = u < units;
      const uint32_t j = (uint32_t)jl[real ? (u >> logQ) : 0u];
      const uint32_t qi = u & ((1u << logQ) - 1u);
      const uint32_t p1 = ((j >> logB) << logW) - c + ((qi >> lq) << 2);
      const uint32_t p2 = ((j & (B - 1u)) << logW) - c + ((qi & ((1u << lq) - 1u)) << 2);
      uint32_t f1[KB], f2[KB], v[KB * KB];
#pragma unroll
      for (uint32_t a = 0; a < KB; ++a) {
        f1[a] = mulmod(inv0, (p1 + a) & mask);
        f2[a] = mulmod(inv1, (p2 + a) & mask);
      }
#pragma unroll
      for (uint32_t k = 0; k < KB * KB; ++k) v[k] = real ? 0u : 0x80000000u;
      if (logB >= 5u) {
        // a bitmap row is whole words: byte offsets of row h1's words and of
        // h2's word within a row, and h2's bit
        const char *bits = reinterpret_cast<const char *>(bsrc);
        for (uint32_t m = 0; m < nA; ++m) {
          const uint32_t l = other(m);
          const uint32_t s1 = s_sig[l][0], s2 = s_sig[l][1];
          uint32_t r[KB], w2[KB], t2[KB];
#pragma unroll
          for (uint32_t a = 0; a < KB; ++a) {
            r[a] = (l * bstride + (axis(s1, f1[a]) << (logB - 5u))) << 2;
            t2[a] = axis(s2, f2[a]);
            w2[a] = (t2[a] >> 5) << 2;
          }
#pragma unroll
          for (uint32_t a = 0; a < KB; ++a) {
#pragma unroll
            for (uint32_t bb = 0; bb < KB; ++bb) {
              const uint32_t word = *reinterpret_cast<const uint32_t *>(bits + r[a] + w2[bb]);
              v[a * KB + bb] += __builtin_amdgcn_ubfe(word, t2[bb], 1u);
            }
          }
        }
      } else {
        for (uint32_t m = 0; m < nA; ++m) {
          const uint32_t l = other(m);
          const uint32_t s1 = s_sig[l][0], s2 = s_sig[l][1];
          // bit offsets: loop l's bitmap, then row h1 of it
          uint32_t r[KB], h2[KB];
#pragma unroll
          for (uint32_t a = 0; a < KB; ++a) {
            r[a] = ((l * bstride) << 5) + (axis(s1, f1[a]) << logB);
            h2[a] = axis(s2, f2[a]);
          }
#pragma unroll
          for (uint32_t a = 0; a < KB; ++a) {
#pragma unroll
            for (uint32_t bb = 0; bb < KB; ++bb) {
              const uint32_t hb = r[a] + h2[bb];
              v[a * KB + bb] += __builtin_amdgcn_ubfe(bsrc[hb >> 5], hb, 1u);
            }
          }
        }
      }
#pragma unroll
      for (uint32_t a = 0; a < KB; ++a) {
#pragma unroll
        for (uint32_t bb = 0; bb < KB; ++bb) keep((f1[a] << logn) | f2[bb], v[a * KB + bb]);
      }
      drain();
    }
    return;
  }

  // every (selected bucket, preimage) pair, the buckets in list order: a
  // block's K x T consecutive pairs may span several buckets (W may be as
  // small as 2 per axis)
  const uint32_t units = ncand << logPer;
  for (uint32_t u0 = blockIdx.x * (uint32_t)K * T; u0 < units; u0 += gridDim.x * (uint32_t)K * T) {
    // the block's candidates and their first nA tests
    uint32_t f[K], v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t u = u0 + threadIdx.x + (uint32_t)k * T;
      const bool real = u < units;
      v[k] = real ? 0u : 0x80000000u;  // the high bit marks no candidate
      const uint32_t j = (uint32_t)jl[real ? (u >> logPer) : 0u];
      const uint32_t idx = u & ((1u << logPer) - 1u);
      const uint32_t p01 = ((NDIM == 1 ? j : (j >> logB)) << logW) - c;
      if (NDIM == 1) {
        f[k] = mulmod(inv0, (p01 + idx) & mask);
      } else {
        const uint32_t p02 = ((j & (B - 1u)) << logW) - c;
        const uint32_t p1 = (p01 + (idx >> logW)) & mask;
        const uint32_t p2 = (p02 + (idx & (W - 1u))) & mask;
        f[k] = (mulmod(inv0, p1) << logn) | mulmod(inv1, p2);
      }
    }
    for (uint32_t m = 0; m < nA; ++m) {
      const uint32_t l = other(m);
      uint32_t h[K];
#pragma unroll
      for (int k = 0; k < K; ++k) h[k] = bucket(l, f[k]);
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] += in_J(l, h[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) keep(f[k], v[k]);
    drain();
  }
}

// ---------------------------------------------------------- k_estimate ----

// Bucket, phase and window factor of the estimator display for frequency f
// in one estimation loop (draw words es[] = sigma1, tau1, sigma2, tau2):
// e_l(f) = y_hat_l[h] omega^{phase} / g with omega = e^{-2 pi i / n}.
template <typename R> struct EstTerm {
  uint32_t h, phase;
  R g;
};

template <typename R, int NDIM>
__device__ __forceinline__ EstTerm<R> est_term(const uint32_t *es, uint32_t f, uint32_t n, uint32_t logn,
                                               uint32_t logB, uint32_t logW, uint32_t c, const R *gh) {
  const uint32_t mask = n - 1u;
  EstTerm<R> t;
  if (NDIM == 1) {
    const uint32_t p = (es[0] * f) & mask;
    t.h = ((p + c) & mask) >> logW;
    const uint32_t dd = ((t.h << logW) - p) & mask;
    const int o = dd > (n >> 1) ? (int)dd - (int)n : (int)dd;
    t.g = gh[o + (int)c];
    t.phase = (es[1] * f) & mask;
  } else {
    const uint32_t f1 = f >> logn, f2 = f & mask;
    const uint32_t p1 = (es[0] * f1) & mask, p2 = (es[2] * f2) & mask;
    const uint32_t h1 = ((p1 + c) & mask) >> logW, h2 = ((p2 + c) & mask) >> logW;
    const uint32_t dd1 = ((h1 << logW) - p1) & mask, dd2 = ((h2 << logW) - p2) & mask;
    const int o1 = dd1 > (n >> 1) ? (int)dd1 - (int)n : (int)dd1;
    const int o2 = dd2 > (n >> 1) ? (int)dd2 - (int)n : (int)dd2;
    t.g = gh[o1 + (int)c] * gh[o2 + (int)c];
    t.h = (h1 << logB) | h2;
    t.phase = ((es[1] * f1) + (es[3] * f2)) & mask;
  }
  return t;
}

// Sort S ascending, then for each located f and estimation loop l the
// estimator display: e_l(f) = y_hat_l[h_l(f)] omega^{tau_l f} / G'(o_l(f)),
// and the coordinate-wise median over the L_est loops.  The workgroups of a
// signal (kEstGroups, more for small batches) each sort S (by rank when
// |S| <= kEstRankMax: the entries are distinct, so each lands at the count of
// smaller ones).  ML
// lanes (a power of two >= L_est) take one located frequency, one loop each,
// so that the loops' loads and arithmetic run side by side; the median of
// the real parts is the value whose rank among the lanes' (ties by loop
// order, unused lanes +inf) is L_est / 2, and likewise for the imaginary
// parts.
template <typename R, int NDIM, int ML, bool DEV = false>
__global__ __launch_bounds__(kEstThreads) void k_estimate(KParams P0) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t sig = blockIdx.y, grp = blockIdx.x;
  const KParams &P = params_of<DEV>(P0, sig);
  SigState *st = state_of(P, sig);
  const SigState s = *st;
  __syncthreads();
  if (s.pass != (int32_t)P.pass) return;
  uint32_t status = s.status;
  const bool empty = (s.status & kSigEmpty) != 0;
  const uint32_t count = empty ? 0u : s.count;
  if (!empty && count > P.max_out) status |= kSigTruncated;
  if (threadIdx.x == 0 && grp == 0) {
    const int64_t slot = out_slot(P, sig);
    P.khat[slot] = s.khat;
    P.count[slot] = (int32_t)count;
    P.status[slot] = status;
    st->status = status;
  }
  if (empty || count > P.max_out || count == 0) return;

  uint32_t *sS = reinterpret_cast<uint32_t *>(smem);
  const uint32_t *S = S_of(P, sig);
  __shared__ uint32_t sIn[kEstRankMax];
  uint32_t P2 = 1;
  if (count <= kEstRankMax) {
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) sIn[i] = S[i];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
      const uint32_t v = sIn[i];
      uint32_t r = 0;
      for (uint32_t j = 0; j < count; ++j) r += sIn[j] < v ? 1u : 0u;
      sS[r] = v;
    }
    __syncthreads();
  } else {
    while (P2 < count) P2 <<= 1;
    for (uint32_t i = threadIdx.x; i < P2; i += blockDim.x) sS[i] = i < count ? S[i] : 0xFFFFFFFFu;
    __syncthreads();
  }
  for (uint32_t k = 2; k <= P2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < P2; i += blockDim.x) {
        const uint32_t l = i ^ j;
        if (l > i) {
          const uint32_t a = sS[i], b = sS[l];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            sS[i] = b;
            sS[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }

  __shared__ uint32_t es[kMaxLoops][4];
  if (threadIdx.x < P.L_est) {
    const Draw d0 = draw(P, sig, kPhaseEst, kPassIter * s.pass + (int)threadIdx.x, 0);
    es[threadIdx.x][0] = d0.sigma;
    es[threadIdx.x][1] = d0.tau;
    if (NDIM == 2) {
      const Draw d1 = draw(P, sig, kPhaseEst, kPassIter * s.pass + (int)threadIdx.x, 1);
      es[threadIdx.x][2] = d1.sigma;
      es[threadIdx.x][3] = d1.tau;
    }
  }
  __syncthreads();

  const uint32_t B = (uint32_t)s.B_star, logB = ilog2(B);
  const uint32_t n = P.n, mask = n - 1u, logn = P.logn;
  const uint32_t logW = logn - logB, c = (1u << logW) >> 1;
  const R *gh = ghat_of<R>(P, logB);
  const R two_over_n = (R)2 / (R)n;
  int64_t *locs = P.locs + out_slot(P, sig) * P.max_out;
  C *vals = reinterpret_cast<C *>(P.vals) + out_slot(P, sig) * P.max_out;
  const uint32_t Le = P.L_est;

  // the sorted set goes to its own array: every workgroup reads S above
  uint32_t *Sg = Ssort_of(P, sig);
  uint16_t *tape = tape_of(P, sig);
  const uint32_t l = threadIdx.x & (uint32_t)(ML - 1);  // this lane's loop
  const uint32_t per = (gridDim.x * blockDim.x) / (uint32_t)ML;
  // a group's lanes share i, so each group leaves the loop as one
  for (uint32_t i = (grp * blockDim.x + threadIdx.x) / (uint32_t)ML; i < count; i += per) {
    const uint32_t f = sS[i];
    R re = (R)INFINITY, im = (R)INFINITY;
    if (l < Le) {
      const EstTerm<R> t = est_term<R, NDIM>(es[l], f, n, logn, logB, logW, c, gh);
      const C yv = ymain_of<C>(P, sig, P.L_loc + l)[t.h];
      R sn, cs;
      sincos_pi(-(R)t.phase * two_over_n, &sn, &cs);
      const R zr = yv.x * cs - yv.y * sn;
      const R zi = yv.x * sn + yv.y * cs;
      re = zr / t.g;
      im = zi / t.g;
    }
    // ranks among the group's lanes, ties broken by loop index
    uint32_t rre = 0, rim = 0;
#pragma unroll
    for (int j = 0; j < ML; ++j) {
      const R oj = __shfl(re, j, ML), pj = __shfl(im, j, ML);
      rre += (oj < re || (oj == re && (uint32_t)j < l)) ? 1u : 0u;
      rim += (pj < im || (pj == im && (uint32_t)j < l)) ? 1u : 0u;
    }
    // the medians, and the first loop holding each (the adjoint's tape)
    const uint32_t gbase = threadIdx.x & 63u & ~(uint32_t)(ML - 1);
    const unsigned long long gmask = (ML == 64 ? ~0ull : ((1ull << ML) - 1ull)) << gbase;
    const uint32_t src_re = (uint32_t)__ffsll((long long)(__ballot(rre == Le / 2u) & gmask)) - 1u - gbase;
    const uint32_t src_im = (uint32_t)__ffsll((long long)(__ballot(rim == Le / 2u) & gmask)) - 1u - gbase;
    C v;
    v.x = __shfl(re, (int)src_re, ML);
    v.y = __shfl(im, (int)src_im, ML);
    const uint32_t lre = (uint32_t)__ffsll((long long)(__ballot(re == v.x) & gmask)) - 1u - gbase;
    const uint32_t lim = (uint32_t)__ffsll((long long)(__ballot(im == v.y) & gmask)) - 1u - gbase;
    if (l == 0) {
      locs[i] = (int64_t)f;
      vals[i] = v;
      Sg[i] = f;
      tape[i] = (uint16_t)(lre | (lim << 8));
    }
  }
}

// ------------------------------------------------------ residual test ----

// A check added to the method (the paper has none): one workgroup per
// (estimation loop, signal) of the launch's pass.  The loop's bucket DFT is
// modelled from the located values by Lemma 1 and the fold: each f adds
// X_f omega^{-tau f} G'(q) to the buckets h + j (|j| <= R per axis, R at most
// (B-1)/2) around its own bucket h, with q = o + j n/B and o its offset.  The
// model is accumulated in LDS (located frequencies sharing a bucket add with
// atomics); E_res = sum |y_hat - M|^2 and E_tot = sum |y_hat|^2 are summed in
// FP64 and stored per loop.
template <typename R, int NDIM>
__global__ __launch_bounds__(kBucketThreads) void k_residual(KParams P) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t l = blockIdx.x, sig = blockIdx.y;
  const SigState s = *state_of(P, sig);
  if ((s.status & kSigEmpty) || s.pass != (int32_t)P.pass) return;
  double *res = resid_of(P, sig);
  if (s.status & kSigTruncated) {  // no values to model: the control counts it as infinite
    if (threadIdx.x == 0) {
      res[l] = 0.0;
      res[kMaxLoops + l] = 0.0;
    }
    return;
  }
  const uint32_t B = (uint32_t)s.B_star, logB = ilog2(B);
  const uint32_t Bc = NDIM == 1 ? B : B * B;
  const uint32_t n = P.n, mask = n - 1u, logn = P.logn;
  const uint32_t logW = logn - logB, c = (1u << logW) >> 1;
  const int reach = (int)min(P.res_reach, (B - 1u) / 2u);
  const int cw = (int)((P.res_reach + 1u) << logW);
  const R *gw = ghat_wide_of<R>(P, logB) + cw;
  const R two_over_n = (R)2 / (R)n;
  const uint32_t tid = threadIdx.x, T = blockDim.x;
  R *M = reinterpret_cast<R *>(smem);  // [Bc] complex, interleaved
  double *red = reinterpret_cast<double *>(smem + (size_t)P.Bc_max * sizeof(C));
  for (uint32_t b = tid; b < 2 * Bc; b += T) M[b] = 0;
  __syncthreads();
  uint32_t es[4];
  {
    const int it = kPassIter * s.pass + (int)l;
    const Draw d0 = draw(P, sig, kPhaseEst, it, 0);
    es[0] = d0.sigma;
    es[1] = d0.tau;
    if (NDIM == 2) {
      const Draw d1 = draw(P, sig, kPhaseEst, it, 1);
      es[2] = d1.sigma;
      es[3] = d1.tau;
    } else {
      es[2] = es[3] = 0;
    }
  }
  const int64_t *locs = P.locs + out_slot(P, sig) * P.max_out;
  const C *vals = reinterpret_cast<const C *>(P.vals) + out_slot(P, sig) * P.max_out;
  for (uint32_t i = tid; i < s.count; i += T) {
    const uint32_t f = (uint32_t)locs[i];
    const C X = vals[i];
    const uint32_t fa[2] = {NDIM == 1 ? f : f >> logn, NDIM == 1 ? 0u : f & mask};
    uint32_t h[2] = {0, 0};
    int o[2] = {0, 0};
    uint32_t phase = 0;
#pragma unroll
    for (int a = 0; a < NDIM; ++a) {
      const uint32_t pa = (es[2 * a] * fa[a]) & mask;
      h[a] = ((pa + c) & mask) >> logW;
      const uint32_t dd = ((h[a] << logW) - pa) & mask;
      o[a] = dd > (n >> 1) ? (int)dd - (int)n : (int)dd;
      phase += es[2 * a + 1] * fa[a];
    }
    phase &= mask;
    // X_f omega^{-tau f}, omega^{-m} = e^{+2 pi i m / n}
    R sn, cs;
    sincos_pi((R)phase * two_over_n, &sn, &cs);
    const R cr = X.x * cs - X.y * sn, ci = X.x * sn + X.y * cs;
    for (int j1 = -reach; j1 <= reach; ++j1) {
      const R g1 = gw[o[0] + (j1 << logW)];
      const uint32_t b1 = (h[0] + (uint32_t)j1) & (B - 1u);
      if (NDIM == 1) {
        atomicAdd(&M[2 * b1], cr * g1);
        atomicAdd(&M[2 * b1 + 1], ci * g1);
      } else {
        for (int j2 = -reach; j2 <= reach; ++j2) {
          const R g = g1 * gw[o[1] + (j2 << logW)];
          const uint32_t b = (b1 << logB) | ((h[1] + (uint32_t)j2) & (B - 1u));
          atomicAdd(&M[2 * b], cr * g);
          atomicAdd(&M[2 * b + 1], ci * g);
        }
      }
    }
  }
  __syncthreads();
  const C *y = ymain_of<C>(P, sig, P.L_loc + l);
  double er = 0.0, et = 0.0;
  for (uint32_t b = tid; b < Bc; b += T) {
    const C v = y[b];
    const double dr = (double)v.x - (double)M[2 * b], di = (double)v.y - (double)M[2 * b + 1];
    er += dr * dr + di * di;
    et += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    er += __shfl_xor(er, off);
    et += __shfl_xor(et, off);
  }
  if ((tid & 63u) == 0) {
    red[2 * (tid >> 6)] = er;
    red[2 * (tid >> 6) + 1] = et;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (uint32_t wv = 0; wv < (T + 63) / 64; ++wv) {
      a += red[2 * wv];
      b += red[2 * wv + 1];
    }
    res[l] = a;
    res[kMaxLoops + l] = b;
  }
}

// One thread per signal of the launch's pass: E_res / E_tot over the
// estimation loops in loop order (infinite for a truncated pass); above
// res_tol, while re-runs remain and 2 B_star <= B_max, the next pass runs
// location and estimation at 2 B_star.
__global__ void k_retry_control(KParams P, int batch) {
  const int sig = blockIdx.x * blockDim.x + threadIdx.x;
  if (sig >= batch) return;
  SigState *st = state_of(P, (uint32_t)sig);
  const SigState s = *st;
  if ((s.status & kSigEmpty) || s.pass != (int32_t)P.pass) return;
  const double *res = resid_of(P, (uint32_t)sig);
  double er = 0.0, et = 0.0;
  for (uint32_t l = 0; l < P.L_est; ++l) {
    er += res[l];
    et += res[kMaxLoops + l];
  }
  const double ratio = (s.status & kSigTruncated) ? (double)INFINITY : (et > 0.0 ? er / et : 0.0);
  st->res_ratio = ratio;
  const uint32_t B2 = 2u * (uint32_t)s.B_star;
  if (ratio > P.res_tol && P.pass < P.res_retries && B2 <= P.B_max && B2 <= P.n / 2u) {
    st->B_star = (int32_t)B2;
    st->pass = s.pass + 1;
    st->status = (s.status | kSigRetried) & ~(uint32_t)kSigTruncated;
    st->count = 0;
  }
}

// ------------------------------------------------------------ adjoint ----

// Gradient of a real loss through the values at fixed located frequencies
// and fixed median choices.  Given the decisions, each value is real-linear
// in x: its real part is Re(e_{l_re}(f)) and its imaginary part Im(e_{l_im}(f))
// with e_l(f) = sum_t K_t x[sigma_l t + tau_l], K_t = c_l(f) G_t omega_B^{h t},
// c_l(f) = omega^{tau_l f} / G'(o).  With g_f = dL/dRe v_f + i dL/dIm v_f the
// gradient (same convention) is, per estimation loop l,
//   ytil_l[j] = sum over f with h_l(f) = j of conj(c_l(f)) (g_re [l = l_re(f)]
//                                                         + i g_im [l = l_im(f)]),
//   u_l = the unnormalised inverse B-point DFT of ytil_l,
//   grad_x[sigma_l t + tau_l] += G_t u_l[t mod B],
// and zero at addresses no estimation loop samples.

// One workgroup per (estimation loop, signal): the bucket cotangent, then
// its inverse DFT in LDS.
template <typename R, int NDIM>
__global__ __launch_bounds__(kBucketThreads) void k_bwd_bucket(KParams P, const void *grad_vals) {
  using C = typename CT<R>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t l = blockIdx.x, sig = blockIdx.y;
  const SigState s = *state_of(P, sig);
  int32_t *flag = bflag_of(P, sig);
  const bool usable = !(s.status & (kSigEmpty | kSigTruncated)) && s.count > 0 && s.count <= P.max_out;
  if (!usable) {
    if (threadIdx.x == 0) flag[l] = 0;
    return;
  }
  const uint32_t count = s.count;
  const uint32_t B = (uint32_t)s.B_star, logB = ilog2(B);
  const uint32_t Bc = NDIM == 1 ? B : B * B;
  const uint32_t n = P.n, logn = P.logn;
  const uint32_t logW = logn - logB, c = (1u << logW) >> 1;
  const R *gh = ghat_of<R>(P, logB);
  const R two_over_n = (R)2 / (R)n;
  uint32_t es[4];
  {
    const Draw d0 = draw(P, sig, kPhaseEst, kPassIter * s.pass + (int)l, 0);
    es[0] = d0.sigma;
    es[1] = d0.tau;
    if (NDIM == 2) {
      const Draw d1 = draw(P, sig, kPhaseEst, kPassIter * s.pass + (int)l, 1);
      es[2] = d1.sigma;
      es[3] = d1.tau;
    } else {
      es[2] = es[3] = 0;
    }
  }
  // ytil accumulated in LDS in natural order (collisions of located
  // frequencies in one bucket add atomically), then conjugated into
  // bit-reversed order so that a forward DFT gives the conjugate of the
  // inverse one
  C *buf = reinterpret_cast<C *>(smem);
  R *bufr = reinterpret_cast<R *>(smem);
  __shared__ uint32_t any;
  if (threadIdx.x == 0) any = 0;
  for (uint32_t b = threadIdx.x; b < Bc; b += blockDim.x) {
    C z;
    z.x = 0;
    z.y = 0;
    buf[b] = z;
  }
  __syncthreads();
  const uint32_t *S = Ssort_of(P, sig);
  const uint16_t *tape = tape_of(P, sig);
  const C *gv = reinterpret_cast<const C *>(grad_vals) + (int64_t)sig * P.max_out;
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
    const uint32_t tp = tape[i];
    const bool on_re = (tp & 0xFFu) == l, on_im = (tp >> 8) == l;
    if (!(on_re || on_im)) continue;
    const EstTerm<R> t = est_term<R, NDIM>(es, S[i], n, logn, logB, logW, c, gh);
    R sn, cs;
    sincos_pi(-(R)t.phase * two_over_n, &sn, &cs);  // c_l(f) = (cs + i sn) / g
    const C g = gv[i];
    const R cr = on_re ? g.x : (R)0, ci = on_im ? g.y : (R)0;  // coefficient cr + i ci
    // conj(c) (cr + i ci) = (cs - i sn)(cr + i ci) / g
    atomicAdd(&bufr[2 * t.h], (cs * cr + sn * ci) / t.g);
    atomicAdd(&bufr[2 * t.h + 1], (cs * ci - sn * cr) / t.g);
    any = 1u;
  }
  __syncthreads();
  if (threadIdx.x == 0) flag[l] = any ? 1 : 0;
  if (!any) return;
  {
    C v[kBucketMaxPer];
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      const uint32_t b = threadIdx.x + (uint32_t)j * blockDim.x;
      if (b < Bc) v[j] = buf[b];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBucketMaxPer; ++j) {
      const uint32_t b = threadIdx.x + (uint32_t)j * blockDim.x;
      if (b < Bc) {
        uint32_t dst;
        if (NDIM == 1)
          dst = bitrev(b, logB);
        else
          dst = (bitrev(b >> logB, logB) << logB) | bitrev(b & (B - 1u), logB);
        C w = v[j];
        w.y = -w.y;
        buf[dst] = w;
      }
    }
  }
  __syncthreads();
  if (NDIM == 1) {
    fft_axis<R>(buf, logB, 1, 0, 1);
  } else {
    fft_axis<R>(buf, logB, B, B, 1);
    fft_axis<R>(buf, logB, B, 1, B);
  }
  C *u = ymain_of<C>(P, sig, P.L_loc + l) + P.Bc_max;  // slab-1 area: free after the forward
  for (uint32_t b = threadIdx.x; b < Bc; b += blockDim.x) {
    C v = buf[b];
    v.y = -v.y;
    u[b] = v;
  }
}

// The scatter grad_x[sigma_l t + tau_l] += G_t u_l[t mod B], done as a gather:
// within one loop t -> sigma_l t + tau_l is a bijection of Z_n (sigma_l odd),
// so address a is reached by the single tap t = sigma_l^{-1} (a - tau_l) at
// most, and only when t lies in the window.  Each thread owns gather_per
// addresses, sums its loops in index order and writes every address once,
// zero included: no atomics, no separate clearing pass, and the same result
// on every run.  For 2D the tap test splits per axis (row, then column).
// A hit costs two random loads, the tap and the bucket adjoint; when a loop's
// bucket adjoint fits the workgroup's LDS (`lds` bytes) it is staged there
// with coalesced loads first, which leaves one random load per hit.
// addresses per thread (measured for the 1D FP32 gather at n = 2^20, B = 4096:
// 8, 16 and 32 addresses 791, 632 and 673 us); FP64 takes half as many to stay
// within the registers
template <typename R, int NDIM> constexpr int gather_per() { return sizeof(R) == 4 ? kGatherPer : kGatherPer / 2; }

template <typename R, int NDIM>
__global__ __launch_bounds__(kGatherThreads) void k_bwd_gather(KParams P, void *grad_x, uint32_t lds) {
  using C = typename CT<R>::C;
  constexpr int PER = gather_per<R, NDIM>();
  extern __shared__ __align__(16) unsigned char smem[];
  C *su = reinterpret_cast<C *>(smem);
  const uint32_t sig = blockIdx.y;
  __shared__ uint32_t s_inv[kMaxLoops][2], s_tau[kMaxLoops][2];
  __shared__ const C *s_u[kMaxLoops];
  __shared__ uint32_t s_nl;
  const int32_t *flag = bflag_of(P, sig);
  if (threadIdx.x == 0) {
    const int it0 = kPassIter * state_of(P, sig)->pass;
    uint32_t nl = 0;
    for (uint32_t l = 0; l < P.L_est; ++l) {
      if (!flag[l]) continue;
      for (int ax = 0; ax < NDIM; ++ax) {
        const Draw d = draw(P, sig, kPhaseEst, it0 + (int)l, ax);
        s_inv[nl][ax] = inv_odd(d.sigma);
        s_tau[nl][ax] = d.tau;
      }
      s_u[nl] = ymain_of<C>(P, sig, P.L_loc + l) + P.Bc_max;
      ++nl;
    }
    s_nl = nl;
  }
  __syncthreads();
  const uint32_t nl = s_nl;
  const uint32_t B = (uint32_t)state_of(P, sig)->B_star;
  const uint32_t logB = ilog2(B);
  const uint32_t Bc = NDIM == 1 ? B : B * B;
  const bool staged = (size_t)Bc * sizeof(C) <= (size_t)lds;  // uniform over the workgroup
  const uint32_t n = P.n, mask = n - 1u;
  const uint32_t w = min(P.alpha * B, n), half = w >> 1;
  const R *G = nl ? taps_of<R>(P, 1, logB) : nullptr;
  C *gx = reinterpret_cast<C *>(grad_x) + (int64_t)sig * P.x_sig;
  const uint32_t total = (uint32_t)P.x_sig;
  const uint32_t span = kGatherThreads * PER;
  for (uint32_t base = blockIdx.x * span; base < total; base += gridDim.x * span) {
    R acc_re[PER], acc_im[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc_re[j] = acc_im[j] = (R)0;
    for (uint32_t q = 0; q < nl; ++q) {
      const C *u = s_u[q];
      if (staged) {
        __syncthreads();  // the previous loop's reads are done
        for (uint32_t b = threadIdx.x; b < Bc; b += kGatherThreads) su[b] = u[b];
        __syncthreads();
        u = su;
      }
      if (NDIM == 1) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const uint32_t a = base + (uint32_t)j * kGatherThreads + threadIdx.x;
          const uint32_t i = (s_inv[q][0] * (a - s_tau[q][0]) + half) & mask;
          if (i < w) {
            const R g = G[i];
            const C v = u[i & (B - 1u)];
            acc_re[j] += g * v.x;
            acc_im[j] += g * v.y;
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const uint32_t a = base + (uint32_t)j * kGatherThreads + threadIdx.x;
          const uint32_t a1 = a >> P.logn, a2 = a & mask;
          const uint32_t i1 = (s_inv[q][0] * (a1 - s_tau[q][0]) + half) & mask;
          if (i1 >= w) continue;
          const uint32_t i2 = (s_inv[q][1] * (a2 - s_tau[q][1]) + half) & mask;
          if (i2 >= w) continue;
          const R g = G[i1] * G[i2];
          const C v = u[((i1 & (B - 1u)) << logB) | (i2 & (B - 1u))];
          acc_re[j] += g * v.x;
          acc_im[j] += g * v.y;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t a = base + (uint32_t)j * kGatherThreads + threadIdx.x;
      if (a < total) {
        C o;
        o.x = acc_re[j];
        o.y = acc_im[j];
        gx[a] = o;
      }
    }
  }
}

template <typename R, int NDIM>
static hipError_t run_backward(const KParams &P, int batch, const void *grad_vals, void *grad_x, hipStream_t s) {
  const size_t smem = bwd_smem_bytes(sizeof(R) == 4 ? 0 : 1, P.Bc_max, P.max_out);
  hipLaunchKernelGGL((k_bwd_bucket<R, NDIM>), dim3(P.L_est, batch), dim3(kBucketThreads), smem, s, P, grad_vals);
  const uint32_t span = kGatherThreads * gather_per<R, NDIM>();
  const uint32_t blocks = (uint32_t)std::min<int64_t>((P.x_sig + span - 1) / span, (int64_t)P.gather_blocks);
  const size_t lds = std::min<size_t>((size_t)P.Bc_max * 2 * sizeof(R), P.gather_lds);
  hipLaunchKernelGGL((k_bwd_gather<R, NDIM>), dim3(blocks, batch), dim3(kGatherThreads), lds, s, P, grad_x,
                     (uint32_t)lds);
  return hipGetLastError();
}

hipError_t launch_backward(const KParams &P, int dtype, int batch, const void *grad_vals, void *grad_x, hipStream_t s) {
  if (dtype == 0)
    return P.ndim == 1 ? run_backward<float, 1>(P, batch, grad_vals, grad_x, s)
                       : run_backward<float, 2>(P, batch, grad_vals, grad_x, s);
  return P.ndim == 1 ? run_backward<double, 1>(P, batch, grad_vals, grad_x, s)
                     : run_backward<double, 2>(P, batch, grad_vals, grad_x, s);
}

size_t bwd_smem_bytes(int dtype, uint32_t Bc_max, uint32_t max_out) {
  (void)max_out;
  return (dtype == 0 ? 8 : 16) * (size_t)Bc_max;
}

// ------------------------------------------------------- window tables ----

// G'(q) = (1/n) sum_t G_t omega^{q t} for the symmetric taps of one window,
// q in [0, c], written to out[c + q] and out[c - q]; FP64.  cos(2 pi q t / n)
// is evaluated exactly (integer reduction of q t mod n, then cospi) at every
// 32nd tap and advanced by a rotation through the angle 2 pi q / n in
// between, which keeps the error of each term within a few 1e-16.
__global__ void k_window_hat(const double *taps, int64_t w, int64_t n, int64_t c, double *out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q > c) return;
  const int64_t half = w / 2;
  double rs, rc;
  sincospi(2.0 * (double)q / (double)n, &rs, &rc);
  double acc = taps[half];
  for (int64_t t0 = 1; t0 < half; t0 += 32) {
    double sn, cs;
    sincospi(2.0 * (double)((q * t0) & (n - 1)) / (double)n, &sn, &cs);
    const int64_t t1 = t0 + 32 < half ? t0 + 32 : half;
    for (int64_t t = t0; t < t1; ++t) {
      acc += 2.0 * taps[half + t] * cs;
      const double c2 = cs * rc - sn * rs;
      sn = sn * rc + cs * rs;
      cs = c2;
    }
  }
  const double v = acc / (double)n;
  out[c + q] = v;
  out[c - q] = v;
}

hipError_t launch_window_hat(const double *taps, int64_t w, int64_t n, int64_t c, double *out,
                             hipStream_t s) {
  const int threads = 256;
  const int64_t blocks = (c + 1 + threads - 1) / threads;
  hipLaunchKernelGGL(k_window_hat, dim3((uint32_t)blocks), dim3(threads), 0, s, taps, w, n, c, out);
  return hipGetLastError();
}

// ------------------------------------------------------ fixed workspace ----

// The workspace of atsfft_execute_batched_noalloc, for callers that cannot
// allocate device memory.  Each device the library runs on holds its own copy
// until the process ends.  In host code the array's name is only a host-side
// stand-in, never a device address: scratch_address looks the address up once
// per device with hipGetSymbolAddress, and host code uses that address alone.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

hipError_t scratch_address(int device, void **ptr) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  if (!ptr || device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ------------------------------------------------------------ launches ----

size_t bucket_smem_bytes(int dtype, uint32_t Bc_max) {
  const size_t rs = dtype == 0 ? sizeof(float) : sizeof(double);
  const size_t fft = 2 * rs * (Bc_max + Bc_max / 32);  // one pad element per 32
  const size_t sel = ((rs * Bc_max + 15) & ~(size_t)15) + 4 * (1536 + 32) + 2 * 8 * (kBucketThreads / 64);
  return fft > sel ? fft : sel;
}

size_t residual_smem_bytes(int dtype, uint32_t Bc_max) {
  const size_t cs = dtype == 0 ? 2 * sizeof(float) : 2 * sizeof(double);
  return cs * Bc_max + 2 * sizeof(double) * (kBucketThreads / 64);
}

size_t vote_smem_bytes(uint32_t L_loc, uint32_t Bc_max) { return 4 * (size_t)L_loc * ((Bc_max + 31) / 32); }

// LDS of the large-array kernels for B per axis (padded DFT buffers; the
// cutoff's histograms, wave keys and two words per 64-bucket chunk)
size_t big_rows_smem(int dtype, uint32_t B) {
  const size_t cs = dtype == 0 ? 8 : 16;
  return cs * (B + B / 32);
}
size_t big_cols_smem(int dtype, uint32_t B) {
  const size_t cs = dtype == 0 ? 8 : 16, e = (size_t)B * (dtype == 0 ? 16 : 8);
  return cs * (e + e / 32);
}

size_t estimate_smem_bytes(uint32_t max_out) {
  uint32_t p2 = 1;
  while (p2 < max_out) p2 <<= 1;
  return 4 * (size_t)p2;
}

template <typename R, int NDIM> static hipError_t set_smem(size_t bucket, size_t est, size_t bwd) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bucket<R, NDIM>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bucket);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd_bucket<R, NDIM>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwd);
  if (e != hipSuccess) return e;
  // the residual model: B^ndim complex plus the FP64 reduction scratch, at
  // most the bucket kernel's LDS plus 256 bytes
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_residual<R, NDIM>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bucket + 256));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd_gather<R, NDIM>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGatherLdsBytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hash2d_rows<R>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRowBytes);
  if (e != hipSuccess) return e;
  for (const void *f : {reinterpret_cast<const void *>(&k_hash2d_stream<R, 4>),
                        reinterpret_cast<const void *>(&k_hash2d_stream<R, 8>),
                        reinterpret_cast<const void *>(&k_hash2d_stream<R, 16>),
                        reinterpret_cast<const void *>(&k_hash2d_stream<R, 4, kBucketThreads>)}) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRowBytes);
    if (e != hipSuccess) return e;
  }
  if (NDIM == 2) {
    const int dt = sizeof(R) == 4 ? 0 : 1;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_big_rows<R>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)big_rows_smem(dt, kBigMax));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_big_cols<R>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)big_cols_smem(dt, kBigMax));
    if (e != hipSuccess) return e;
  }
  for (const void *f : {reinterpret_cast<const void *>(&k_vote<NDIM, true>),
                        reinterpret_cast<const void *>(&k_vote<NDIM, false>)}) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(4 * (kMaxLoops - 1) * (kBucketThreads * kBucketMaxPer / 32)));
    if (e != hipSuccess) return e;
  }
  const void *ks[3] = {reinterpret_cast<const void *>(&k_estimate<R, NDIM, 8>),
                       reinterpret_cast<const void *>(&k_estimate<R, NDIM, 16>),
                       reinterpret_cast<const void *>(&k_estimate<R, NDIM, 32>)};
  for (const void *k : ks) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)est);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t prepare_kernels(int dtype, int ndim, size_t bucket_smem, size_t est_smem, size_t bwd_smem) {
  if (dtype == 0)
    return ndim == 1 ? set_smem<float, 1>(bucket_smem, est_smem, bwd_smem)
                     : set_smem<float, 2>(bucket_smem, est_smem, bwd_smem);
  return ndim == 1 ? set_smem<double, 1>(bucket_smem, est_smem, bwd_smem)
                   : set_smem<double, 2>(bucket_smem, est_smem, bwd_smem);
}

static uint32_t ilog2_host_u32(uint32_t v) {
  uint32_t r = 0;
  while (v >>= 1) ++r;
  return r;
}

// The statistics steps of the large arrays of a launch: `arrays` of them per
// signal from index `iter` (role 0: the location loops; role 1: one probe
// level) with at most `chunks` 4096-bucket chunks each.
template <typename R>
static void big_stats(const KParams &P, int role, int iter, uint32_t arrays, uint32_t chunks, int batch,
                      hipStream_t s) {
  const dim3 cg(chunks, arrays, batch), ag(arrays, batch);
  hipLaunchKernelGGL((k_bs_m<R>), cg, dim3(kBigThreads), 0, s, P, role, iter);
  const int passes = sizeof(R) == 4 ? 4 : 8;  // 8-bit digits of the key range
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_bs_hist<R>), cg, dim3(kBigThreads), 0, s, P, role, iter, p);
    hipLaunchKernelGGL((k_bs_pick<R>), ag, dim3(128), 0, s, P, role, iter, p);
  }
  hipLaunchKernelGGL((k_bs_count<R>), cg, dim3(kBigThreads), 0, s, P, role, iter);
  hipLaunchKernelGGL((k_bs_end<R>), ag, dim3(64), 0, s, P, role, iter);
  if (role == 0) {
    hipLaunchKernelGGL((k_bs_chunks<R>), cg, dim3(kBigThreads), 0, s, P, iter);
    hipLaunchKernelGGL((k_bs_scan<R>), ag, dim3(kBigChunks), 0, s, P, iter);
    hipLaunchKernelGGL((k_bs_list<R>), cg, dim3(kBigThreads), 0, s, P, iter);
  }
}

template <typename R, int NDIM, bool DEV = false>
static hipError_t run(const KParams &P, int batch, hipStream_t s, StageMark mark, void *ctx) {
  const size_t bsmem = bucket_smem_bytes(sizeof(R) == 4 ? 0 : 1, min(P.Bc_max, P.lds_cap));
  const size_t bsmem_small = bucket_smem_bytes(sizeof(R) == 4 ? 0 : 1, min(min(P.Bc_max, P.lds_cap), kSmallBuckets));
  // the main k_bucket launches, one per class of array that can occur
  const uint64_t bc_min = NDIM == 1 ? (uint64_t)P.B0 : (uint64_t)P.B0 * P.B0;
  const size_t esmem = estimate_smem_bytes(P.max_out);
  const uint32_t main_slots = P.main_slots ? P.main_slots : batch <= 64 ? 64u : 32u;
  const uint32_t hash_blocks = kSlabs * max(1u, min(main_slots, (P.Bc_max + kTile - 1) / kTile));
  if (mark) mark(ctx, 0);
  hipLaunchKernelGGL(k_init<DEV>, dim3((batch + 255) / 256), dim3(256), 0, s, P, batch);
  if (!P.fixed) {
    // rounds of probe levels: every level up to B = probe_first at once, then
    // probe_step levels per round
    uint32_t lo = 0;
    // probe levels have few tiles per signal: about four workgroups per CU
    // over the batch (levels with fewer tiles take one slot per tile)
    KParams Qp = P;
    Qp.tile_slots = max(P.tile_slots, 4u * P.n_cu / (uint32_t)batch);
    auto level_bc = [&](uint32_t l) -> uint64_t {
      const uint64_t Bl = (uint64_t)P.B0 << l;
      return NDIM == 1 ? Bl : Bl * Bl;
    };
    while (lo < P.probe_levels) {
      if (NDIM == 2 && level_bc(lo) > P.lds_cap) {
        // a level above the LDS size is a round of its own: hashed, then its
        // DFT, threshold, local maxima and B-update rule in device memory
        const uint32_t Bl = P.B0 << lo;
        const int dt = sizeof(R) == 4 ? 0 : 1;
        const uint32_t slots = max(1u, min(Qp.tile_slots, (Bl * Bl + kTile - 1) / kTile));
        hipLaunchKernelGGL((k_hash<R, NDIM, 1, false, false, DEV>), dim3(slots, 1, batch), dim3(kHashThreads), 0, s,
                           Qp, (int)lo, (int)lo + 1);
        hipLaunchKernelGGL((k_big_rows<R>), dim3(Bl, 1, batch), dim3(256), big_rows_smem(dt, Bl), s, P, 1, (int)lo);
        hipLaunchKernelGGL((k_big_cols<R>), dim3(max(1u, Bl / big_cols<R>()), 1, batch), dim3(1024),
                           big_cols_smem(dt, Bl), s, P, 1, (int)lo);
        big_stats<R>(P, 1, (int)lo, 1, max(1u, Bl * Bl / kBigChunk), batch, s);
        ++lo;
        continue;
      }
      uint32_t hi = lo == 0 ? 1 : lo + P.probe_step;
      if (lo == 0)
        while (hi < P.probe_levels && (P.B0 << hi) <= P.probe_first) ++hi;
      hi = min(hi, P.probe_levels);
      while (hi > lo + 1 && level_bc(hi - 1) > P.lds_cap) --hi;  // k_bucket rounds hold LDS-sized levels only
      // (level, slot) pairs: each level as many slots as it has tiles, at
      // most Qp.tile_slots (so that small levels launch no idle workgroups)
      uint32_t slots = 0;
      for (uint32_t l = lo; l < hi; ++l) {
        const uint32_t Bl = P.B0 << l;
        slots += max(1u, min(Qp.tile_slots, ((NDIM == 1 ? Bl : Bl * Bl) + kTile - 1) / kTile));
      }
      const uint32_t kProbeSlabs = NDIM == 1 ? P.probe_slabs : 1u;
      if (sizeof(R) == 4 && P.comp)
        hipLaunchKernelGGL((k_hash<R, NDIM, 1, sizeof(R) == 4, false, DEV>), dim3(kProbeSlabs * slots, 1, batch),
                           dim3(kHashThreads), 0, s, Qp, (int)lo, (int)hi);
      else
        hipLaunchKernelGGL((k_hash<R, NDIM, 1, false, false, DEV>), dim3(kProbeSlabs * slots, 1, batch),
                           dim3(kHashThreads), 0, s, Qp, (int)lo, (int)hi);
      // a round whose grid is more than two workgroups per CU runs in
      // 256-thread workgroups, several to a CU, when its levels allow (the
      // workgroups of a small batch are latency chains, kept at 1024 threads)
      const bool small_wg = (uint64_t)(hi - lo) * (uint64_t)batch > 2ull * P.n_cu && level_bc(hi - 1) <= kSmallBuckets;
      hipLaunchKernelGGL((k_bucket<R, NDIM, DEV>), dim3(hi - lo, batch),
                         dim3(small_wg ? kSmallBucketThreads : kBucketThreads), small_wg ? bsmem_small : bsmem, s, P, 0,
                         (int)lo);
      lo = hi;
    }
  }
  if (mark) mark(ctx, 1);
  // location and estimation of one pass; Q.pass selects the signals
  const uint32_t loops = P.L_loc + P.L_est;
  const uint32_t LG = NDIM == 1 ? P.hash_loops : 1u;
  const dim3 hgrid(hash_blocks, (loops + LG - 1) / LG, batch);
  const dim3 hgrid1(hash_blocks, loops, batch);
  const uint32_t E = P.L_loc - P.T_vote + 1;
  // vote workgroups per (loop, signal): more for small batches, where the
  // launch is latency-bound, and twice as many in 2D, whose blocks of
  // preimages give a workgroup more candidates (measured at 4096^2, batch 8:
  // 16, 32, 64, 128 workgroups 67, 63, 60, 68 us; a plan knob overrides)
  const uint32_t vote_blocks = P.vote_blocks ? P.vote_blocks
                               : NDIM == 2 ? (uint32_t)max(64, 256 / batch)
                                           : (uint32_t)max(32, 128 / batch);
  const size_t vsmem = vote_smem_bytes(P.L_loc, P.Bc_max);
  // 2D rows staged in LDS when the row fits and the input is 16-byte aligned
  const size_t rows_smem = std::max<size_t>((size_t)P.n * sizeof(typename CT<R>::C), 2 * kHashThreads * sizeof(R));
  const bool rows = !DEV && NDIM == 2 && P.rows2d_ok && !P.x_off && (reinterpret_cast<uintptr_t>(P.x) & 15u) == 0 && !P.comp;
  const uint32_t row_mode = rows ? P.rows2d_ok : 0u;  // 1: per bucket row, 2: streamed
  // when the grid exceeds the chip (one 1024-thread workgroup per CU) the
  // small arrays take 256-thread workgroups, several to a CU, or 512-thread
  // ones while there are at most four arrays per CU (n = 2^22, batch 32: 48 ->
  // 44 us; 512 signals of 2^16..2^22: 4.88 -> 4.96 ms per call with 512
  // threads throughout); otherwise every array a 1024-thread one (a chain of
  // four waves is the longer)
  const bool split = (uint64_t)loops * (uint64_t)batch > (uint64_t)P.n_cu;
  const uint32_t small_threads =
      (uint64_t)loops * (uint64_t)batch <= 4ull * P.n_cu ? 2u * (uint32_t)kSmallBucketThreads : (uint32_t)kSmallBucketThreads;
  const bool small_main = (P.fixed ? (uint64_t)P.Bc_max : bc_min) <= kSmallBuckets;
  const bool large_main = min(P.Bc_max, P.lds_cap) > kSmallBuckets;
  auto launch_main_bucket = [&](const KParams &Q) {
    if (!split) {
      hipLaunchKernelGGL((k_bucket<R, NDIM, DEV>), dim3(loops * batch), dim3(kBucketThreads), bsmem, s, Q, 2, 0);
      return;
    }
    if (small_main)
      hipLaunchKernelGGL((k_bucket<R, NDIM, DEV>), dim3(loops * batch), dim3(small_threads), bsmem_small, s, Q, 3, 0);
    if (large_main)
      hipLaunchKernelGGL((k_bucket<R, NDIM, DEV>), dim3(loops * batch), dim3(kBucketThreads), bsmem, s, Q, 4, 0);
  };
  auto main_pass = [&](const KParams &Q0, bool marks) {
    KParams Q = Q0;
    Q.est_wait = !DEV && (uint64_t)loops * (uint64_t)batch <= (uint64_t)P.n_cu ? 1u : 0u;
    if (NDIM == 2 && Q.big) {
      // arrays above the LDS size (this branch) and the others (the usual
      // launches below) each skip the other kind, so a batch may hold both:
      // rows streamed once, by 1024-thread workgroups for the large arrays,
      // then their DFTs and cutoffs in device memory
      const uint32_t Bb = 1u << (ilog2_host_u32(P.Bc_max) / 2);
      const int dt = sizeof(R) == 4 ? 0 : 1;
      Q.rows2d = 2;
      const dim3 sgrid((P.n + P.stream_rows - 1) / P.stream_rows, batch);
      const size_t rb = (size_t)P.n * sizeof(typename CT<R>::C);
      hipLaunchKernelGGL((k_hash2d_stream<R, 4, kBucketThreads>), sgrid, dim3(kBucketThreads), rb, s, Q);
      if (rb <= 16u * 4u * kHashThreads)
        hipLaunchKernelGGL((k_hash2d_stream<R, 4>), sgrid, dim3(kHashThreads), rb, s, Q);
      else if (rb <= 16u * 8u * kHashThreads)
        hipLaunchKernelGGL((k_hash2d_stream<R, 8>), sgrid, dim3(kHashThreads), rb, s, Q);
      else
        hipLaunchKernelGGL((k_hash2d_stream<R, 16>), sgrid, dim3(kHashThreads), rb, s, Q);
      if (marks && mark) mark(ctx, 2);
      hipLaunchKernelGGL((k_big_rows<R>), dim3(Bb, loops, batch), dim3(256), big_rows_smem(dt, Bb), s, Q, 0, 0);
      hipLaunchKernelGGL((k_big_cols<R>), dim3(max(1u, Bb / big_cols<R>()), loops, batch), dim3(1024),
                         big_cols_smem(dt, Bb), s, Q, 0, 0);
      big_stats<R>(Q, 0, 0, P.L_loc, max(1u, Bb * Bb / kBigChunk), batch, s);
      launch_main_bucket(Q);
      if (marks && mark) mark(ctx, 3);
      hipLaunchKernelGGL((k_vote<NDIM, true, DEV, true>), dim3(vote_blocks, E, batch), dim3(kVoteThreads), 0, s, Q);
      hipLaunchKernelGGL((k_vote<NDIM, true, DEV>), dim3(vote_blocks, E, batch), dim3(kVoteThreads),
                         vote_smem_bytes(P.L_loc, P.lds_cap), s, Q);
      if (marks && mark) mark(ctx, 4);
    } else {
      Q.rows2d = row_mode;
      if (row_mode == 2) {
        const dim3 sgrid((P.n + P.stream_rows - 1) / P.stream_rows, batch);
        const size_t rb = (size_t)P.n * sizeof(typename CT<R>::C);
        if (rb <= 16u * 4u * kHashThreads)
          hipLaunchKernelGGL((k_hash2d_stream<R, 4>), sgrid, dim3(kHashThreads), rb, s, Q);
        else if (rb <= 16u * 8u * kHashThreads)
          hipLaunchKernelGGL((k_hash2d_stream<R, 8>), sgrid, dim3(kHashThreads), rb, s, Q);
        else
          hipLaunchKernelGGL((k_hash2d_stream<R, 16>), sgrid, dim3(kHashThreads), rb, s, Q);
      }
      else if (row_mode == 1)
        hipLaunchKernelGGL((k_hash2d_rows<R>), dim3(1u << (ilog2_host_u32(P.Bc_max) / 2), loops, batch),
                           dim3(kHashThreads), rows_smem, s, Q);
      else if (sizeof(R) == 4 && Q.comp)
        hipLaunchKernelGGL((k_hash<R, NDIM, 1, sizeof(R) == 4, true, DEV>), hgrid1, dim3(kHashThreads), 0, s, Q, 0, 0);
      else if (NDIM == 2 || LG == 1)
        hipLaunchKernelGGL((k_hash<R, NDIM, 1, false, true, DEV>), hgrid, dim3(kHashThreads), 0, s, Q, 0, 0);
      else if (LG == 2)
        hipLaunchKernelGGL((k_hash<R, NDIM == 1 ? 1 : 1, 2, false, true, DEV>), hgrid, dim3(kHashThreads), 0, s, Q, 0, 0);
      else
        hipLaunchKernelGGL((k_hash<R, NDIM == 1 ? 1 : 1, 3, false, true, DEV>), hgrid, dim3(kHashThreads), 0, s, Q, 0, 0);
      if (marks && mark) mark(ctx, 2);
      launch_main_bucket(Q);
      if (marks && mark) mark(ctx, 3);
      if (NDIM == 2 || P.logn <= 24)
        hipLaunchKernelGGL((k_vote<NDIM, true, DEV>), dim3(vote_blocks, E, batch), dim3(kVoteThreads), vsmem, s, Q);
      else
        hipLaunchKernelGGL((k_vote<NDIM, false, DEV>), dim3(vote_blocks, E, batch), dim3(kVoteThreads), vsmem, s, Q);
      if (marks && mark) mark(ctx, 4);
    }
    // estimate workgroups per signal: more for small batches, up to 32
    const uint32_t est_groups = std::min<uint32_t>(32u, std::max<uint32_t>((uint32_t)kEstGroups, 128u / (uint32_t)batch));
    if (Q.L_est <= 8)
      hipLaunchKernelGGL((k_estimate<R, NDIM, 8, DEV>), dim3(est_groups, batch), dim3(kEstThreads), esmem, s, Q);
    else if (Q.L_est <= 16)
      hipLaunchKernelGGL((k_estimate<R, NDIM, 16, DEV>), dim3(est_groups, batch), dim3(kEstThreads), esmem, s, Q);
    else
      hipLaunchKernelGGL((k_estimate<R, NDIM, 32, DEV>), dim3(est_groups, batch), dim3(kEstThreads), esmem, s, Q);
  };
  main_pass(P, true);
  if (!DEV && P.res_tol > 0.0) {
    // residual test after every pass; a pass r > 0 runs only the signals the
    // test sent back at 2 B_star
    const size_t rsmem = residual_smem_bytes(sizeof(R) == 4 ? 0 : 1, P.Bc_max);
    KParams Q = P;
    for (uint32_t r = 0;; ++r) {
      Q.pass = r;
      if (r > 0) main_pass(Q, false);
      hipLaunchKernelGGL((k_residual<R, NDIM>), dim3(P.L_est, batch), dim3(kBucketThreads), rsmem, s, Q);
      hipLaunchKernelGGL(k_retry_control, dim3((batch + 255) / 256), dim3(256), 0, s, Q, batch);
      if (r >= P.res_retries) break;
    }
  }
  if (mark) mark(ctx, 5);
  return hipGetLastError();
}

hipError_t launch_execute(const KParams &P, int dtype, int batch, hipStream_t s, StageMark mark, void *ctx) {
  if (dtype == 0) return P.ndim == 1 ? run<float, 1>(P, batch, s, mark, ctx) : run<float, 2>(P, batch, s, mark, ctx);
  return P.ndim == 1 ? run<double, 1>(P, batch, s, mark, ctx) : run<double, 2>(P, batch, s, mark, ctx);
}

// The per-length parameters of a device-driven uneven call: block i copies
// the plan's template for log2 length dev_lg_lo + i into the workspace table
// and completes it with the call's buffers.
__global__ void k_dev_setup(KParams P, const KParams *tmpl) {
  const uint32_t lg = P.dev_lg_lo + blockIdx.x;
  KParams *q = const_cast<KParams *>(P.devP) + lg;
  const uint64_t *src = reinterpret_cast<const uint64_t *>(tmpl + blockIdx.x);
  uint64_t *dst = reinterpret_cast<uint64_t *>(q);
  for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(KParams) / 8); i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    q->ws = P.ws;
    q->x = P.x;
    q->x_off = P.x_off;
    q->sig_map = nullptr;
    q->locs = P.locs;
    q->vals = P.vals;
    q->count = P.count;
    q->khat = P.khat;
    q->status = P.status;
    q->pass = 0;
    q->devP = nullptr;
    q->ns = P.ns;
  }
}

hipError_t launch_execute_dev(const KParams &P, const KParams *tmpl, int dtype, int batch, hipStream_t s) {
  if (P.ndim != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dev_setup, dim3(P.dev_lg_hi - P.dev_lg_lo + 1), dim3(256), 0, s, P, tmpl);
  return dtype == 0 ? run<float, 1, true>(P, batch, s, nullptr, nullptr) : run<double, 1, true>(P, batch, s, nullptr, nullptr);
}

}  // namespace atsfft
