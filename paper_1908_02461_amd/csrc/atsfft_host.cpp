// Host side of the ATSFFT C ABI: descriptor defaults and validation, the
// plan's window tables, workspace layout and the execute entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <array>
#include <new>
#include <string>
#include <vector>

#include "atsfft.h"
#include "atsfft_internal.h"

using namespace atsfft;

struct atsfft_plan_s {
  atsfft_desc d;
  int device;
  uint32_t logn;
  uint32_t Bc_max;   // largest bucket array (B^ndim) any loop can use
  uint32_t big;      // 2D arrays above the LDS-resident size: DFTs and cutoffs in device memory
  uint32_t lds_cap;  // largest bucket array (B^ndim) k_bucket holds in LDS
  uint32_t n_cu;     // compute units of the device
  void *G_dev;       // taps, plan precision
  void *Ghat_dev;    // G'(o) tables, plan precision
  int64_t tab_host[128];  // element offsets by log2 B (passed in the kernel arguments)
  size_t bucket_smem, est_smem, bwd_smem;
  uint32_t tile_slots;  // probe hash workgroups per slab and level, at most
  uint32_t main_slots;  // main-pass hash workgroups per slab and loop group
  uint32_t one_slab_logn;  // 1D main pass: lengths up to 2^this hashed as one address slab
  uint32_t hash_loops;  // main-pass loops per hash workgroup
  uint32_t vote_blocks; // vote workgroups per (loop, signal)
  uint32_t rows2d_ok;   // 2D main loops may be hashed by rows staged in LDS
  uint32_t stream_rows; // 2D streamed row hash: rows per workgroup
  uint32_t gather_lds;  // adjoint gather: most LDS bytes for a staged bucket adjoint (0: none)
  uint32_t gather_blocks;  // adjoint gather: most workgroups per signal
  uint32_t probe_first; // first probe round covers B up to this
  uint32_t probe_step;  // probe levels per later round
  uint32_t probe_slabs; // 1D probe levels: address slabs
  uint32_t probe_spin;  // sleeps before the probe control gives up waiting for a count
  int32_t probe_drop;   // test hook: probe level whose count is never recorded (-1: none)
  uint32_t cut_ties;    // test hook: the location loops' tie-aware cutoff path always
  // stage timing (ATSFFT_FLAG_PROFILE): six events per execute
  std::vector<std::array<hipEvent_t, 6>> prof_used, prof_free;
  // uneven batches: one plan per power-of-two length below n (index log2 n'),
  // and a pinned staging buffer for the per-signal tables
  atsfft_plan_s *sub[32];
  void *stage_host;
  size_t stage_bytes;
  hipEvent_t stage_done;
  // ATSFFT_FLAG_GRAPH: the execute's launches captured once per call shape
  // (batch and buffers) on a plan-owned stream, replayed on the caller's
  struct GraphEntry {
    int32_t kind;  // 0 batched execute, 1 uneven execute with device lengths
    int32_t batch;
    const void *ptrs[9];
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream;
  // the device's fixed workspace (atsfft_execute_batched_noalloc), or null
  // when its address lookup failed (scratch_err)
  void *scratch;
  hipError_t scratch_err;
  // uneven batches with device-side lengths (1D, n_min > 0): the parameters
  // of every covered length, log2 lengths dev_lg_lo..dev_lg_hi (device)
  KParams *dev_tmpl;
  uint32_t dev_lg_lo, dev_lg_hi;
};

static_assert(kScratchBytes == ATSFFT_NOALLOC_WORKSPACE_BYTES, "fixed workspace size and its header constant");

namespace {

thread_local std::string g_err = "";
constexpr size_t kMaxGraphs = 64;  // call shapes kept per plan under ATSFFT_FLAG_GRAPH

atsfft_status fail(atsfft_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

uint32_t ilog2_host(uint64_t v) {
  uint32_t r = 0;
  while ((uint64_t)1 << (r + 1) <= v) ++r;
  return r;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The flat window of Sec. II-A-2, read as a Gaussian in time multiplied by
// the time image of a one-bucket box car (a Dirichlet kernel over the n/B+1
// bins |o| <= n/(2B)).  The Gaussian falls to delta at |t| = w/2; the tap at
// t = -w/2 is zero so that the taps are symmetric.  out[t + w/2].
void window_taps(int64_t n, int64_t B, int64_t w, double delta, std::vector<double> &out) {
  out.assign((size_t)w, 0.0);
  const int64_t half = w / 2;
  const double ln_delta = std::log(delta);
  const int64_t width = n / B + 1;
  for (int64_t t = 0; t < half; ++t) {
    const double u = (double)t / (double)half;
    const double gauss = std::exp(ln_delta * u * u);
    double dir;
    if (t == 0) {
      dir = (double)width;
    } else {
      const int64_t num = (width * t) % (2 * n);  // exact reduction of width * t modulo 2n
      dir = std::sin(M_PI * (double)num / (double)n) / std::sin(M_PI * (double)t / (double)n);
    }
    const double v = gauss * dir;
    out[(size_t)(half + t)] = v;
    if (t > 0) out[(size_t)(half - t)] = v;
  }
}

// Largest bucket count per axis of the location and estimation loops: B_max,
// or fixed_B in the Algorithm 1 form (which residual-test re-runs may grow up
// to B_max).
int64_t main_bmax(const atsfft_desc *d) {
  if (!(d->flags & ATSFFT_FLAG_FIXED_B)) return d->B_max;
  return d->res_tol > 0.0 ? std::max(d->fixed_B, d->B_max) : d->fixed_B;
}

// Model reach of the residual test in buckets to each side of a frequency's
// own: ceil(2 ln(1/delta) / (pi alpha)), the Gaussian's transition half-width
// in bucket widths, at least 1.
uint32_t residual_reach(const atsfft_desc *d) {
  const double r = 2.0 * std::log(1.0 / d->delta) / (M_PI * (double)d->alpha);
  const int v = (int)std::ceil(r);
  return v < 1 ? 1u : (uint32_t)v;
}

atsfft_status validate(const atsfft_desc *d) {
  if (!d) return fail(ATSFFT_EINVAL, "null descriptor");
  if (d->ndim != 1 && d->ndim != 2) return fail(ATSFFT_EINVAL, "ndim must be 1 or 2");
  if (d->dtype != ATSFFT_C64 && d->dtype != ATSFFT_C128) return fail(ATSFFT_EINVAL, "bad dtype");
  if (!is_pow2(d->n)) return fail(ATSFFT_EINVAL, "n must be a power of two");
  if (d->ndim == 1 && (d->n < 64 || d->n > ((int64_t)1 << 30)))
    return fail(ATSFFT_EINVAL, "1D n must be in [2^6, 2^30]");
  if (d->ndim == 2 && (d->n < 16 || d->n > ((int64_t)1 << 15)))
    return fail(ATSFFT_EINVAL, "2D N must be in [2^4, 2^15]");
  if (d->max_out < 1 || d->max_out > kMaxOut) return fail(ATSFFT_EINVAL, "max_out must be in [1, 16384]");
  if (d->max_batch < 1 || d->max_batch > 65535) return fail(ATSFFT_EINVAL, "max_batch must be in [1, 65535]");
  if (d->n_min != 0 && (!is_pow2(d->n_min) || d->n_min > d->n || d->n_min < (d->ndim == 1 ? 64 : 16)))
    return fail(ATSFFT_EINVAL, "n_min must be 0 or a power of two in [2^6 (2D: 2^4), n]");
  const int64_t Bmin = d->ndim == 1 ? 2 : 4;
  const bool fixed = (d->flags & ATSFFT_FLAG_FIXED_B) != 0;
  if (fixed) {
    if (!is_pow2(d->fixed_B) || d->fixed_B < Bmin || d->fixed_B > d->n / 2)
      return fail(ATSFFT_EINVAL, "fixed_B must be a power of two in [2, n/2] (2D: [4, N/2])");
    if (d->fixed_k < 0) return fail(ATSFFT_EINVAL, "fixed_k must be >= 0");
  } else {
    if (!is_pow2(d->B0) || !is_pow2(d->B_max) || d->B0 < Bmin || d->B0 > d->B_max || d->B_max > d->n / 2)
      return fail(ATSFFT_EINVAL, "need B0 <= B_max, powers of two in [2, n/2] (2D: [4, N/2])");
    if (d->alpha_probe < 2 || d->alpha_probe > 1024 || (d->alpha_probe & 1))
      return fail(ATSFFT_EINVAL, "alpha_probe must be even in [2, 1024]");
    if (d->P_max < 1 || d->P_max > kMaxProbe) return fail(ATSFFT_EINVAL, "P_max must be in [1, 32]");
    if (d->gamma < 0) return fail(ATSFFT_EINVAL, "gamma must be >= 0");
  }
  if ((d->flags & ATSFFT_FLAG_GRAPH) && (d->flags & ATSFFT_FLAG_PROFILE))
    return fail(ATSFFT_EINVAL, "ATSFFT_FLAG_GRAPH and ATSFFT_FLAG_PROFILE exclude each other");
  if (!(d->res_tol >= 0.0) || d->res_retries < 0 || d->res_retries > 7)
    return fail(ATSFFT_EINVAL, "res_tol must be >= 0 and res_retries in [0, 7]");
  if (fixed && d->res_tol > 0.0 && (!is_pow2(d->B_max) || d->B_max < Bmin || d->B_max > d->n / 2))
    return fail(ATSFFT_EINVAL, "the residual test needs B_max a power of two in [2, n/2] (2D: [4, N/2])");
  const int64_t Bbig = main_bmax(d);
  const int64_t Bc = d->ndim == 1 ? Bbig : Bbig * Bbig;
  if (Bc > (int64_t)kBucketThreads * kBucketMaxPer && !(d->ndim == 2 && Bbig <= (int64_t)kBigMax))
    return fail(ATSFFT_EINVAL, "largest bucket array B^ndim must be <= 16384 (2D: B <= 1024)");
  if (d->alpha < 2 || d->alpha > 1024 || (d->alpha & 1)) return fail(ATSFFT_EINVAL, "alpha must be even in [2, 1024]");
  if (d->L_loc < 1 || d->L_loc > kMaxLoops - 1) return fail(ATSFFT_EINVAL, "L_loc must be in [1, 31]");
  if (d->L_est < 1 || d->L_est > kMaxLoops - 1 || (d->L_est % 2) == 0)
    return fail(ATSFFT_EINVAL, "L_est must be odd in [1, 31]");
  if (d->T_vote < 1 || d->T_vote > d->L_loc) return fail(ATSFFT_EINVAL, "T_vote must be in [1, L_loc]");
  if (d->d < 1 || d->d > 64) return fail(ATSFFT_EINVAL, "d must be in [1, 64]");
  if (!(d->delta > 0.0 && d->delta < 1.0)) return fail(ATSFFT_EINVAL, "delta must be in (0, 1)");
  if (!(d->q > 0.0 && d->q < 1.0)) return fail(ATSFFT_EINVAL, "q must be in (0, 1)");
  if (!(d->noise_rate > 0.0)) return fail(ATSFFT_EINVAL, "noise_rate must be > 0");
  if (!(d->rho >= 0.0)) return fail(ATSFFT_EINVAL, "rho must be >= 0");
  return ATSFFT_SUCCESS;
}

uint32_t probe_levels(const atsfft_plan_s *p) {
  const atsfft_desc &d = p->d;
  if (d.flags & ATSFFT_FLAG_FIXED_B) return 0;
  uint32_t lv = ilog2_host((uint64_t)(d.B_max / d.B0)) + 1;
  return lv < (uint32_t)d.P_max ? lv : (uint32_t)d.P_max;
}

// bucket values (per slab) of probe levels below `level`
uint64_t probe_offset(const atsfft_plan_s *p, uint32_t level) {
  uint64_t off = 0;
  for (uint32_t i = 0; i < level; ++i) {
    const uint64_t B = (uint64_t)p->d.B0 << i;
    off += p->d.ndim == 1 ? B : B * B;
  }
  return off;
}

uint64_t probe_elems(const atsfft_plan_s *p) { return probe_offset(p, probe_levels(p)); }

Layout make_layout(const atsfft_plan_s *p, int32_t batch) {
  const atsfft_desc &d = p->d;
  const size_t A = 256;
  const size_t cs = d.dtype == ATSFFT_C64 ? 8 : 16;
  const size_t Bc = p->Bc_max;
  const size_t L = (size_t)(d.L_loc + d.L_est);
  Layout l;
  std::memset(&l, 0, sizeof(l));
  size_t off = 0;
  l.state = off;
  off = align_up(off + sizeof(SigState), A);
  l.hist = off;
  off = align_up(off + (size_t)kMaxProbe * sizeof(ProbeRec), A);
  l.tloc = off;
  off = align_up(off + (size_t)kMaxLoops * 8, A);
  l.jcount = off;
  off = align_up(off + (size_t)kMaxLoops * 4, A);
  // bucket arrays hold kSlabs partials each (k_hash); the DFT lands in slab 0
  // probe area: the kSlabs partials of every probe level B0 * 2^i
  l.yprobe = off;
  off = align_up(off + (size_t)kSlabs * probe_elems(p) * cs, A);
  l.ymain_loop = align_up((size_t)kSlabs * Bc * cs, A);
  l.ymain = off;
  off = align_up(off + L * l.ymain_loop, A);
  l.jbits_loop = align_up(((Bc + 31) / 32) * 4, 16);
  l.jbits = off;
  off = align_up(off + (size_t)d.L_loc * l.jbits_loop, A);
  l.jlist_loop = align_up(Bc * 4, 16);
  l.jlist = off;
  off = align_up(off + (size_t)d.L_loc * l.jlist_loop, A);
  l.S = off;  // located set in vote order
  off = align_up(off + (size_t)d.max_out * 4, A);
  l.Ssort = off;  // the same, ascending (aligned with the tape)
  off = align_up(off + (size_t)d.max_out * 4, A);
  l.tape = off;  // median loops of each located frequency (adjoint)
  off = align_up(off + (size_t)d.max_out * 2, A);
  l.bflag = off;
  off = align_up(off + (size_t)kMaxLoops * 4, A);
  l.resid = off;  // residual test: E_res and E_tot of each estimation loop
  off = align_up(off + (size_t)2 * kMaxLoops * 8, A);
  l.slice = off;
  l.total = off * (size_t)batch;
  return l;
}

template <typename T> std::vector<T> convert(const std::vector<double> &v) {
  std::vector<T> out(v.size());
  for (size_t i = 0; i < v.size(); ++i) out[i] = (T)v[i];
  return out;
}

void free_plan(atsfft_plan_s *p) {
  if (!p) return;
  for (atsfft_plan_s *q : p->sub)
    if (q && q != p) free_plan(q);
  if (p->stage_host) (void)hipHostFree(p->stage_host);
  if (p->stage_done) (void)hipEventDestroy(p->stage_done);
  for (auto *pool : {&p->prof_used, &p->prof_free})
    for (auto &rec : *pool)
      for (hipEvent_t e : rec) (void)hipEventDestroy(e);
  if (p->G_dev) (void)hipFree(p->G_dev);
  if (p->Ghat_dev) (void)hipFree(p->Ghat_dev);
  if (p->dev_tmpl) (void)hipFree(p->dev_tmpl);
  for (auto &g : p->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

KParams make_params(const atsfft_plan_s *plan, const Layout &lay, const void *x_dev, int64_t *locs_dev,
                    void *vals_dev, int32_t *count_dev, int32_t *khat_dev, uint32_t *sig_status_dev, void *ws_dev) {
  const atsfft_desc &d = plan->d;
  KParams P;
  std::memset(&P, 0, sizeof(P));
  P.seed = d.seed;
  P.n = (uint32_t)d.n;
  P.logn = plan->logn;
  P.ndim = (uint32_t)d.ndim;
  P.Bc_max = plan->Bc_max;
  P.B0 = (uint32_t)d.B0;
  P.B_max = (uint32_t)d.B_max;
  P.alpha_probe = (uint32_t)d.alpha_probe;
  P.alpha = (uint32_t)d.alpha;
  P.L_loc = (uint32_t)d.L_loc;
  P.L_est = (uint32_t)d.L_est;
  P.T_vote = (uint32_t)d.T_vote;
  P.P_max = (uint32_t)d.P_max;
  P.d = (uint32_t)d.d;
  P.gamma = (uint32_t)d.gamma;
  P.max_out = (uint32_t)d.max_out;
  P.fixed = (d.flags & ATSFFT_FLAG_FIXED_B) ? 1u : 0u;
  P.fixed_B = (uint32_t)d.fixed_B;
  P.fixed_k = (uint32_t)d.fixed_k;
  P.vote_blocks = plan->vote_blocks;
  P.rows2d_ok = plan->rows2d_ok;
  P.stream_rows = plan->stream_rows;
  P.gather_lds = plan->gather_lds;
  P.gather_blocks = plan->gather_blocks;
  P.probe_first = plan->probe_first;
  P.probe_step = plan->probe_step;
  P.probe_slabs = plan->probe_slabs;
  P.probe_spin = plan->probe_spin;
  P.probe_drop = plan->probe_drop;
  P.cut_ties = plan->cut_ties;
  P.tile_slots = plan->tile_slots;
  P.main_slots = plan->main_slots;
  P.one_slab_logn = plan->one_slab_logn;
  P.pad_kp = 0;
  P.hash_loops = plan->hash_loops;
  P.probe_levels = probe_levels(plan);
  for (uint32_t i = 0; i < (uint32_t)kMaxProbe; ++i)
    P.probe_off[i] = i < P.probe_levels ? (uint64_t)kSlabs * probe_offset(plan, i) : 0;
  P.res_tol = d.res_tol;
  P.res_retries = (uint32_t)d.res_retries;
  P.res_reach = residual_reach(&d);
  P.pass = 0;
  P.comp = (d.flags & ATSFFT_FLAG_COMPENSATED) && d.dtype == ATSFFT_C64 ? 1u : 0u;
  P.big = plan->big;
  P.lds_cap = plan->lds_cap;
  P.n_cu = plan->n_cu;
  P.est_wait = 0;
  P.q = d.q;
  P.neg_log1mq = -std::log(1.0 - d.q);
  P.noise_rate = d.noise_rate;
  P.rho = d.rho;
  P.G = plan->G_dev;
  P.Ghat = plan->Ghat_dev;
  std::memcpy(P.tab, plan->tab_host, sizeof(P.tab));
  P.ws = static_cast<uint8_t *>(ws_dev);
  P.lay = lay;
  P.x = x_dev;
  P.x_sig = d.ndim == 1 ? d.n : d.n * d.n;
  P.locs = locs_dev;
  P.vals = vals_dev;
  P.count = count_dev;
  P.khat = khat_dev;
  P.status = sig_status_dev;
  return P;
}

// ATSFFT_FLAG_GRAPH: replay the launches `enqueue` makes for this call shape
// (kind, batch and buffers), capturing them on the plan's own stream the
// first time; the last kMaxGraphs shapes are kept.
template <typename F>
atsfft_status graph_launch(atsfft_plan_s *plan, int32_t kind, int32_t batch, const void *const key[9],
                           hipStream_t stream, F enqueue) {
  atsfft_plan_s::GraphEntry *hit = nullptr;
  for (auto &g : plan->graphs)
    if (g.kind == kind && g.batch == batch && std::memcmp(g.ptrs, key, sizeof(g.ptrs)) == 0) hit = &g;
  if (!hit) {
    if (plan->graphs.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(plan->graphs.front().exec);
      (void)hipGraphDestroy(plan->graphs.front().graph);
      plan->graphs.erase(plan->graphs.begin());
    }
    if (!plan->cap_stream && hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(ATSFFT_ELAUNCH, "hipStreamCreateWithFlags failed");
    atsfft_plan_s::GraphEntry e;
    e.kind = kind;
    e.batch = batch;
    std::memcpy(e.ptrs, key, sizeof(e.ptrs));
    e.graph = nullptr;
    e.exec = nullptr;
    if (hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(ATSFFT_ELAUNCH, "hipStreamBeginCapture failed");
    const hipError_t le = enqueue(plan->cap_stream);
    const hipError_t ce = hipStreamEndCapture(plan->cap_stream, &e.graph);
    if (le != hipSuccess || ce != hipSuccess || hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
      if (e.graph) (void)hipGraphDestroy(e.graph);
      (void)hipGetLastError();
      return fail(ATSFFT_ELAUNCH, "graph capture of the execute failed");
    }
    plan->graphs.push_back(e);
    hit = &plan->graphs.back();
  }
  if (hipGraphLaunch(hit->exec, stream) != hipSuccess) {
    hipError_t e = hipGetLastError();
    return fail(ATSFFT_ELAUNCH, std::string("graph launch failed: ") + hipGetErrorString(e));
  }
  return ATSFFT_SUCCESS;
}

}  // namespace

extern "C" {

const char *atsfft_version(void) { return "atsfft-mi355x 0.1.0 (gfx950)"; }

const char *atsfft_last_error(void) { return g_err.c_str(); }

const char *atsfft_status_string(atsfft_status s) {
  switch (s) {
    case ATSFFT_SUCCESS: return "success";
    case ATSFFT_EINVAL: return "invalid argument";
    case ATSFFT_ENODEVICE: return "no usable gfx950 device";
    case ATSFFT_ENOMEM: return "device allocation failed";
    case ATSFFT_ELAUNCH: return "kernel launch or HIP call failed";
    case ATSFFT_ENOTSUPPORTED: return "not supported by the library";
  }
  return "unknown status";
}

atsfft_status atsfft_default_desc(atsfft_desc *d, int32_t ndim, int64_t n, int32_t dtype) {
  if (!d) return fail(ATSFFT_EINVAL, "null descriptor");
  std::memset(d, 0, sizeof(*d));
  d->ndim = ndim;
  d->dtype = dtype;
  d->n = n;
  d->max_out = 4096;
  d->seed = 0;
  d->flags = 0;
  d->max_batch = 1;
  const bool c64 = dtype == ATSFFT_C64;
  if (ndim == 2) {
    d->alpha_probe = 4;
    d->alpha = 8;
    d->B0 = 8;
    const int64_t cap = c64 ? 128 : 64;
    d->B_max = n / d->alpha < cap ? n / d->alpha : cap;
  } else {
    d->alpha_probe = 16;
    d->alpha = 32;
    d->B0 = 32;
    const int64_t cap = c64 ? 16384 : 8192;
    d->B_max = n / d->alpha < cap ? n / d->alpha : cap;
  }
  if (d->B_max < d->B0) d->B_max = d->B0;
  d->L_loc = 9;
  d->L_est = 9;
  d->T_vote = 5;
  d->P_max = 12;
  d->d = 2;
  d->gamma = 32;
  d->delta = c64 ? 1e-6 : 1e-8;
  d->q = 0.1;
  d->noise_rate = 0.01;
  d->rho = 1e-6;
  d->fixed_B = 0;
  d->fixed_k = 0;
  d->res_tol = 0.0;
  d->res_retries = 1;
  return ATSFFT_SUCCESS;
}

static atsfft_status create_plan(atsfft_plan_t *out, const atsfft_desc *d) {
  if (!out) return fail(ATSFFT_EINVAL, "null plan pointer");
  *out = nullptr;
  atsfft_status st = validate(d);
  if (st != ATSFFT_SUCCESS) return st;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(ATSFFT_ENODEVICE, "no HIP device");
  }
  atsfft_plan_s *p = new (std::nothrow) atsfft_plan_s();
  if (!p) return fail(ATSFFT_ENOMEM, "host allocation failed");
  p->d = *d;
  if (hipGetDevice(&p->device) != hipSuccess) {
    free_plan(p);
    return fail(ATSFFT_ENODEVICE, "hipGetDevice failed");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) {
    free_plan(p);
    return fail(ATSFFT_ENODEVICE, "hipGetDeviceProperties failed");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    free_plan(p);
    return fail(ATSFFT_ENODEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  }

  const bool fixed = (d->flags & ATSFFT_FLAG_FIXED_B) != 0;
  const int64_t n = d->n;
  p->logn = ilog2_host((uint64_t)n);
  const int64_t Bbig = main_bmax(d);
  p->Bc_max = (uint32_t)(d->ndim == 1 ? Bbig : Bbig * Bbig);
  p->bucket_smem = bucket_smem_bytes(d->dtype, p->Bc_max);
  p->hash_loops = 3;  // measured at n = 2^22, batch 32: 1, 2, 3 loops 442, 429, 418 us
  if (const char *env = std::getenv("ATSFFT_HASH_LOOPS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 3) p->hash_loops = (uint32_t)v;
  }
  p->tile_slots = 32;
  if (const char *env = std::getenv("ATSFFT_TILE_SLOTS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 64) p->tile_slots = (uint32_t)v;
  }
  // 0: by batch, 64 slots up to 64 signals, else 32 (measured at n = 2^22, batch
  // 32, B* 2048 and 4096: 32, 48, 64 slots 420, 416, 413 us; batch 64: 822 and
  // 807 us for 32 and 64; n = 2^20, batch 64 forward + adjoint: 2.381 and 2.331
  // ms per step; on the uneven batch of 512 signals, most with few 64-bucket
  // tiles, the idle slots cost more: 6.87 ms per call with 32, 7.33 with 64)
  p->main_slots = 0;
  // 1D main pass in one address slab where a lane has few wraps: at alpha = 8
  // (two wraps per lane and loop) eight slabs leave most of its loads masked
  // off.  Measured, batch 32, k = 64, hash us for 8 / 1 slabs: n = 2^18 alpha 8
  // 174 / 98, alpha 32 210 / 258; n = 2^20 alpha 8 185 / 177, alpha 32 251 / 599;
  // n = 2^21 alpha 8 177 / 195 (whole call 587 / 577: one partial per bucket
  // for k_bucket); the uneven batch at alpha 8 is fastest with one slab up to
  // 2^21 (5.01 ms per call, 6.46 with none, 5.14 up to 2^22).
  p->one_slab_logn = d->ndim == 1 && d->alpha <= 8 ? 21u : 0u;
  if (const char *env = std::getenv("ATSFFT_ONE_SLAB_MAX_N")) {
    const long long v = std::strtoll(env, nullptr, 10);
    if (v == 0) p->one_slab_logn = 0;
    if (v >= 2 && (v & (v - 1)) == 0 && v <= (1LL << 30)) p->one_slab_logn = ilog2_host((uint64_t)v);
  }
  if (const char *env = std::getenv("ATSFFT_MAIN_SLOTS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 64) p->main_slots = (uint32_t)v;
  }
  p->vote_blocks = 0;  // by batch
  {
    const uint64_t row_bytes = (uint64_t)n * (d->dtype == ATSFFT_C64 ? 8 : 16);
    const int64_t Bm = main_bmax(d);
    // per bucket row: a thread owns one bucket column and at most kRowTaps
    // of its wraps; streamed: at most kSlabs row wraps (one partial each)
    p->rows2d_ok = 0;
    if (d->ndim == 2 && row_bytes <= kRowBytes && Bm <= kHashThreads &&
        (int64_t)d->alpha * Bm <= (int64_t)kHashThreads * kRowTaps)
      p->rows2d_ok = d->alpha <= kSlabs ? 2u : 1u;
    if (const char *env = std::getenv("ATSFFT_ROWS2D")) {
      const long v = std::strtol(env, nullptr, 10);
      if (v >= 0 && v < (long)p->rows2d_ok) p->rows2d_ok = (uint32_t)v;
    }
  }
  p->stream_rows = 2;  // measured at 4096^2 c64: 2 rows 249 us, 8 rows 265, 32 rows 271
  if (const char *env = std::getenv("ATSFFT_STREAM_ROWS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 64) p->stream_rows = (uint32_t)v;
  }
  p->gather_blocks = 1024;
  if (const char *env = std::getenv("ATSFFT_GATHER_BLOCKS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 1024) p->gather_blocks = (uint32_t)v;
  }
  p->gather_lds = (uint32_t)kGatherLdsBytes;
  if (const char *env = std::getenv("ATSFFT_GATHER_LDS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v == 0) p->gather_lds = 0;
  }
  if (const char *env = std::getenv("ATSFFT_VOTE_BLOCKS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 1024) p->vote_blocks = (uint32_t)v;
  }
  p->probe_first = 2048;
  if (const char *env = std::getenv("ATSFFT_PROBE_FIRST")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= (1 << 20)) p->probe_first = (uint32_t)v;
  }
  p->probe_step = 2;
  if (const char *env = std::getenv("ATSFFT_PROBE_STEP")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1 && v <= 32) p->probe_step = (uint32_t)v;
  }
  // 1D probe levels gather cold lines that few other gathers touch again: one
  // slab (measured at n = 2^22, batch 32: probe 160 us against 168 with kSlabs)
  p->probe_slabs = 1;
  if (const char *env = std::getenv("ATSFFT_PROBE_SLABS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v == 1 || v == kSlabs) p->probe_slabs = (uint32_t)v;
  }
  p->probe_spin = 1u << 20;
  if (const char *env = std::getenv("ATSFFT_PROBE_SPIN")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 0 && v <= (1L << 24)) p->probe_spin = (uint32_t)v;
  }
  p->probe_drop = -1;
  if (const char *env = std::getenv("ATSFFT_PROBE_DROP_LEVEL")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 0 && v < kMaxProbe) p->probe_drop = (int32_t)v;
  }
  p->cut_ties = 0;
  if (const char *env = std::getenv("ATSFFT_CUTOFF_TIES")) p->cut_ties = std::strtol(env, nullptr, 10) == 1 ? 1u : 0u;
  p->est_smem = estimate_smem_bytes((uint32_t)d->max_out);
  p->big = 0;
  p->lds_cap = p->Bc_max;
  p->n_cu = (uint32_t)prop.multiProcessorCount;
  if (p->bucket_smem > prop.sharedMemPerBlock) {
    // 2D arrays above the LDS size (the known-k form at the sparse FFT's
    // bucket count, or a B_max beyond it): those arrays live in device
    // memory; needs rows streamed once (a row fits the row buffer, w / B <=
    // kSlabs partials) and no residual test, compensated fold, uneven
    // lengths or adjoint
    const uint64_t row_bytes = (uint64_t)n * (d->dtype == ATSFFT_C64 ? 8 : 16);
    const bool big_ok = d->ndim == 2 && d->res_tol == 0.0 && d->n_min == 0 &&
                        !(d->flags & ATSFFT_FLAG_COMPENSATED) && Bbig <= (int64_t)kBigMax &&
                        d->alpha <= kSlabs && row_bytes <= kRowBytes &&
                        big_cols_smem(d->dtype, (uint32_t)Bbig) <= prop.sharedMemPerBlock;
    if (!big_ok) {
      char msg[200];
      std::snprintf(msg, sizeof(msg),
                    "B_max^ndim = %u needs %zu bytes of LDS, device has %zu (larger arrays: 2D, "
                    "B <= %u, alpha <= 8, no residual test, compensation or uneven lengths)",
                    p->Bc_max, p->bucket_smem, (size_t)prop.sharedMemPerBlock, kBigMax);
      free_plan(p);
      return fail(ATSFFT_EINVAL, msg);
    }
    p->big = 1;
    // the largest B x B array k_bucket still holds in LDS takes the smaller
    // ones (probe levels, signals whose B_star is small); the adjoint does
    // not run on such a plan
    while (p->lds_cap > 16 && (p->lds_cap > kBucketThreads * kBucketMaxPer ||
                               bucket_smem_bytes(d->dtype, p->lds_cap) > prop.sharedMemPerBlock))
      p->lds_cap /= 4;
    p->bucket_smem = bucket_smem_bytes(d->dtype, p->lds_cap);
    // the 2D main-loop hash streams rows (one partial per row wrap)
    p->rows2d_ok = 2;
  }
  p->bwd_smem = bwd_smem_bytes(d->dtype, p->big ? p->lds_cap : p->Bc_max, (uint32_t)d->max_out);

  // window tables for every bucket count a loop may use
  std::vector<double> taps_all, ghat_all;
  std::vector<int64_t> tab(128, 0);
  std::vector<double> taps;
  const int64_t Blo = fixed ? d->fixed_B : d->B0;
  const int64_t Bhi = Bbig;
  const bool resid = d->res_tol > 0.0;
  const int64_t reach = (int64_t)residual_reach(d);
  std::vector<int64_t> main_taps_off;
  double *taps_dev64 = nullptr, *ghat_dev64 = nullptr;
  for (int64_t B = Blo; B <= Bhi; B *= 2) {
    const uint32_t lb = ilog2_host((uint64_t)B);
    if (!fixed) {
      const int64_t wp = std::min<int64_t>((int64_t)d->alpha_probe * B, n);
      window_taps(n, B, wp, d->delta, taps);
      tab[lb] = (int64_t)taps_all.size();
      taps_all.insert(taps_all.end(), taps.begin(), taps.end());
    }
    const int64_t w = std::min<int64_t>((int64_t)d->alpha * B, n);
    window_taps(n, B, w, d->delta, taps);
    tab[32 + lb] = (int64_t)taps_all.size();
    taps_all.insert(taps_all.end(), taps.begin(), taps.end());
    tab[64 + lb] = (int64_t)ghat_all.size();
    ghat_all.resize(ghat_all.size() + (size_t)(n / B + 1), 0.0);
    if (resid) {  // G'(q), |q| <= (reach + 1) n/B, for the residual model
      tab[96 + lb] = (int64_t)ghat_all.size();
      ghat_all.resize(ghat_all.size() + (size_t)(2 * (reach + 1) * (n / B) + 1), 0.0);
    }
  }
  // G'(o) from the FP64 taps, on the device
  if (hipMalloc(&taps_dev64, taps_all.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&ghat_dev64, ghat_all.size() * sizeof(double)) != hipSuccess) {
    (void)hipFree(taps_dev64);
    (void)hipFree(ghat_dev64);
    free_plan(p);
    return fail(ATSFFT_ENOMEM, "window table allocation failed");
  }
  bool ok = hipMemcpy(taps_dev64, taps_all.data(), taps_all.size() * sizeof(double), hipMemcpyHostToDevice) ==
            hipSuccess;
  for (int64_t B = Blo; ok && B <= Bhi; B *= 2) {
    const uint32_t lb = ilog2_host((uint64_t)B);
    const int64_t w = std::min<int64_t>((int64_t)d->alpha * B, n);
    ok = launch_window_hat(taps_dev64 + tab[32 + lb], w, n, n / (2 * B), ghat_dev64 + tab[64 + lb], nullptr) ==
         hipSuccess;
    if (ok && resid)
      ok = launch_window_hat(taps_dev64 + tab[32 + lb], w, n, (reach + 1) * (n / B), ghat_dev64 + tab[96 + lb],
                             nullptr) == hipSuccess;
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  ok = ok && hipMemcpy(ghat_all.data(), ghat_dev64, ghat_all.size() * sizeof(double), hipMemcpyDeviceToHost) ==
                 hipSuccess;
  (void)hipFree(taps_dev64);
  (void)hipFree(ghat_dev64);
  if (!ok) {
    (void)hipGetLastError();
    free_plan(p);
    return fail(ATSFFT_ELAUNCH, "window table generation failed");
  }
  const size_t rs = d->dtype == ATSFFT_C64 ? sizeof(float) : sizeof(double);
  if (hipMalloc(&p->G_dev, taps_all.size() * rs) != hipSuccess ||
      hipMalloc(&p->Ghat_dev, ghat_all.size() * rs) != hipSuccess) {
    free_plan(p);
    return fail(ATSFFT_ENOMEM, "window table allocation failed");
  }
  if (d->dtype == ATSFFT_C64) {
    std::vector<float> g = convert<float>(taps_all), gh = convert<float>(ghat_all);
    ok = hipMemcpy(p->G_dev, g.data(), g.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(p->Ghat_dev, gh.data(), gh.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
  } else {
    ok = hipMemcpy(p->G_dev, taps_all.data(), taps_all.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(p->Ghat_dev, ghat_all.data(), ghat_all.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
  }
  std::memcpy(p->tab_host, tab.data(), 128 * sizeof(int64_t));
  ok = ok && prepare_kernels(d->dtype, d->ndim, p->bucket_smem, p->est_smem, p->bwd_smem) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_plan(p);
    return fail(ATSFFT_ELAUNCH, "window table upload or kernel setup failed");
  }
  // the fixed workspace's device address, looked up once per device (the
  // plan's device is current here); only atsfft_execute_batched_noalloc uses it
  p->scratch = nullptr;
  p->scratch_err = scratch_address(p->device, &p->scratch);
  if (p->scratch_err != hipSuccess) {
    p->scratch = nullptr;
    (void)hipGetLastError();
  }
  *out = p;
  return ATSFFT_SUCCESS;
}

// The parameters of every length an uneven plan covers, for the execute with
// device-side lengths: each length's own knobs and window tables, with the
// workspace layout, bucket stride and probe-area offsets of the longest
// (every signal's slice is the longest one's, so that a signal's slice is
// found from its index alone).  1D plans without the residual test only.
static atsfft_status build_dev_templates(atsfft_plan_s *p) {
  if (p->d.ndim != 1 || p->d.res_tol > 0.0) return ATSFFT_SUCCESS;
  const KParams top = make_params(p, make_layout(p, 1), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  std::vector<KParams> t;
  uint32_t lo = p->logn;
  while (lo > 0 && p->sub[lo - 1]) --lo;
  for (uint32_t lg = lo; lg <= p->logn; ++lg) {
    KParams q = make_params(p->sub[lg], top.lay, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    q.Bc_max = top.Bc_max;
    std::memcpy(q.probe_off, top.probe_off, sizeof(q.probe_off));
    if (q.probe_levels > top.probe_levels) return fail(ATSFFT_EINVAL, "a shorter length probes more levels");
    t.push_back(q);
  }
  if (hipMalloc(&p->dev_tmpl, t.size() * sizeof(KParams)) != hipSuccess) {
    p->dev_tmpl = nullptr;
    return fail(ATSFFT_ENOMEM, "parameter table allocation failed");
  }
  if (hipMemcpy(p->dev_tmpl, t.data(), t.size() * sizeof(KParams), hipMemcpyHostToDevice) != hipSuccess)
    return fail(ATSFFT_ELAUNCH, "parameter table upload failed");
  p->dev_lg_lo = lo;
  p->dev_lg_hi = p->logn;
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_plan(atsfft_plan_t *out, const atsfft_desc *d) {
  atsfft_status st = create_plan(out, d);
  if (st != ATSFFT_SUCCESS) return st;
  atsfft_plan_s *p = *out;
  p->sub[p->logn] = p;
  if (d->n_min > 0 && d->n_min < d->n) {
    // a plan for every shorter power-of-two length, with the same knobs
    // clipped to that length
    for (int64_t m = d->n_min; m < d->n; m *= 2) {
      atsfft_desc e = *d;
      e.n = m;
      e.n_min = 0;
      if (!(e.flags & ATSFFT_FLAG_FIXED_B)) {
        const int64_t cap = m / e.alpha > 0 ? m / e.alpha : 1;
        if (e.B_max > cap) e.B_max = cap;
        const int64_t Bmin = e.ndim == 1 ? 2 : 4;
        if (e.B_max < Bmin) e.B_max = Bmin;
        if (e.B0 > e.B_max) e.B0 = e.B_max;
      } else {
        if (e.fixed_B > m / 2) e.fixed_B = m / 2;
        if (e.res_tol > 0.0 && e.B_max > m / 2) e.B_max = m / 2;
      }
      atsfft_plan_t q = nullptr;
      st = create_plan(&q, &e);
      if (st != ATSFFT_SUCCESS) {
        free_plan(p);
        *out = nullptr;
        return st;
      }
      p->sub[q->logn] = q;
    }
    st = build_dev_templates(p);
    if (st != ATSFFT_SUCCESS) {
      free_plan(p);
      *out = nullptr;
      return st;
    }
  }
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_workspace_size(atsfft_plan_t plan, int32_t batch, size_t *bytes) {
  if (!plan || !bytes) return fail(ATSFFT_EINVAL, "null argument");
  if (batch < 1 || batch > plan->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  *bytes = make_layout(plan, batch).total;
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_execute_batched(atsfft_plan_t plan, int32_t batch, const void *x_dev, int64_t *locs_dev,
                                     void *vals_dev, int32_t *count_dev, int32_t *khat_dev,
                                     uint32_t *sig_status_dev, void *ws_dev, size_t ws_bytes,
                                     hipStream_t stream) {
  if (!plan) return fail(ATSFFT_EINVAL, "null plan");
  if (batch < 1 || batch > plan->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  if (!x_dev || !locs_dev || !vals_dev || !count_dev || !khat_dev || !sig_status_dev || !ws_dev)
    return fail(ATSFFT_EINVAL, "null device pointer");
  const Layout lay = make_layout(plan, batch);
  if (ws_bytes < lay.total) return fail(ATSFFT_EINVAL, "workspace too small");
  if (plan->big && (reinterpret_cast<uintptr_t>(x_dev) & 15u))
    return fail(ATSFFT_EINVAL, "x must be 16-byte aligned for bucket arrays above the LDS-resident size");
  KParams P = make_params(plan, lay, x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev, ws_dev);
  const atsfft_desc &d = plan->d;
  if (d.flags & ATSFFT_FLAG_GRAPH) {
    const void *key[9] = {x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev, ws_dev, nullptr, nullptr};
    return graph_launch(plan, 0, batch, key, stream, [&](hipStream_t cs) {
      return launch_execute(P, d.dtype, batch, cs, nullptr, nullptr);
    });
  }
  std::array<hipEvent_t, 6> *rec = nullptr;
  if (d.flags & ATSFFT_FLAG_PROFILE) {
    if (plan->prof_free.empty()) {
      std::array<hipEvent_t, 6> r;
      for (auto &e : r)
        if (hipEventCreate(&e) != hipSuccess) return fail(ATSFFT_ELAUNCH, "hipEventCreate failed");
      plan->prof_free.push_back(r);
    }
    plan->prof_used.push_back(plan->prof_free.back());
    plan->prof_free.pop_back();
    rec = &plan->prof_used.back();
  }
  struct MarkCtx {
    std::array<hipEvent_t, 6> *rec;
    hipStream_t s;
  } mctx{rec, stream};
  StageMark mark = nullptr;
  if (rec)
    mark = [](void *c, int stage) {
      MarkCtx *m = static_cast<MarkCtx *>(c);
      (void)hipEventRecord((*m->rec)[(size_t)stage], m->s);
    };
  if (launch_execute(P, d.dtype, batch, stream, mark, &mctx) != hipSuccess) {
    hipError_t e = hipGetLastError();
    return fail(ATSFFT_ELAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  }
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_execute_batched_noalloc(atsfft_plan_t plan, int32_t batch, const void *x_dev,
                                             int64_t *locs_dev, void *vals_dev, int32_t *count_dev,
                                             int32_t *khat_dev, uint32_t *sig_status_dev, hipStream_t stream) {
  if (!plan) return fail(ATSFFT_EINVAL, "null plan");
  if (plan->d.flags & (ATSFFT_FLAG_GRAPH | ATSFFT_FLAG_PROFILE))
    return fail(ATSFFT_EINVAL, "the fixed-workspace execute takes no GRAPH or PROFILE plan (both allocate)");
  if (batch < 1 || batch > plan->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  if (!x_dev || !locs_dev || !vals_dev || !count_dev || !khat_dev || !sig_status_dev)
    return fail(ATSFFT_EINVAL, "null device pointer");
  const Layout lay = make_layout(plan, batch);
  if (lay.total > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "batch %d needs %zu bytes of workspace, above the fixed workspace of %zu bytes "
                  "(ATSFFT_NOALLOC_WORKSPACE_BYTES)",
                  (int)batch, lay.total, kScratchBytes);
    return fail(ATSFFT_EINVAL, msg);
  }
  if (plan->big && (reinterpret_cast<uintptr_t>(x_dev) & 15u))
    return fail(ATSFFT_EINVAL, "x must be 16-byte aligned for bucket arrays above the LDS-resident size");
  if (!plan->scratch)
    return fail(ATSFFT_ELAUNCH, std::string("fixed workspace address lookup failed: ") +
                                    hipGetErrorString(plan->scratch_err));
  KParams P = make_params(plan, lay, x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev, plan->scratch);
  if (launch_execute(P, plan->d.dtype, batch, stream, nullptr, nullptr) != hipSuccess) {
    hipError_t e = hipGetLastError();
    return fail(ATSFFT_ELAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  }
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_execute(atsfft_plan_t plan, const void *x_dev, int64_t *locs_dev, void *vals_dev,
                             int32_t *count_dev, int32_t *khat_dev, uint32_t *sig_status_dev, void *ws_dev,
                             size_t ws_bytes, hipStream_t stream) {
  return atsfft_execute_batched(plan, 1, x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev,
                                ws_dev, ws_bytes, stream);
}

atsfft_status atsfft_backward(atsfft_plan_t plan, int32_t batch, const void *grad_vals_dev, const void *ws_dev,
                              void *grad_x_dev, hipStream_t stream) {
  if (!plan) return fail(ATSFFT_EINVAL, "null plan");
  if (batch < 1 || batch > plan->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  if (!grad_vals_dev || !ws_dev || !grad_x_dev) return fail(ATSFFT_EINVAL, "null device pointer");
  if (plan->big) return fail(ATSFFT_ENOTSUPPORTED, "no adjoint for bucket arrays above the LDS-resident size");
  const Layout lay = make_layout(plan, batch);
  KParams P = make_params(plan, lay, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, const_cast<void *>(ws_dev));
  if (launch_backward(P, plan->d.dtype, batch, grad_vals_dev, grad_x_dev, stream) != hipSuccess) {
    hipError_t e = hipGetLastError();
    return fail(ATSFFT_ELAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  }
  return ATSFFT_SUCCESS;
}

namespace {

// Grouping of an uneven batch: signals of each length, in call order.
struct Groups {
  std::vector<std::vector<int32_t>> members;  // by log2 length
  size_t header;                              // bytes of the per-signal tables
  std::vector<size_t> base;                   // workspace offset of each group's slices
  size_t total;
};

atsfft_status make_groups(const atsfft_plan_s *p, int32_t batch, const int64_t *ns, Groups &g) {
  if (!ns) return fail(ATSFFT_EINVAL, "null ns");
  if (batch < 1 || batch > p->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  g.members.assign(32, {});
  for (int32_t i = 0; i < batch; ++i) {
    const int64_t m = ns[i];
    if (!is_pow2(m) || m > p->d.n) return fail(ATSFFT_EINVAL, "ns[i] must be a power of two the plan covers");
    const uint32_t lg = ilog2_host((uint64_t)m);
    if (!p->sub[lg]) return fail(ATSFFT_EINVAL, "ns[i] below the plan's n_min");
    g.members[lg].push_back(i);
  }
  g.header = align_up((size_t)batch * 8, 256) + align_up((size_t)batch * 4, 256);
  g.base.assign(32, 0);
  size_t off = g.header;
  for (uint32_t lg = 0; lg < 32; ++lg) {
    if (g.members[lg].empty()) continue;
    g.base[lg] = off;
    off += make_layout(p->sub[lg], (int32_t)g.members[lg].size()).total;
  }
  g.total = off;
  return ATSFFT_SUCCESS;
}

}  // namespace

atsfft_status atsfft_workspace_size_uneven(atsfft_plan_t plan, int32_t batch, const int64_t *ns, size_t *bytes) {
  if (!plan || !bytes) return fail(ATSFFT_EINVAL, "null argument");
  Groups g;
  atsfft_status st = make_groups(plan, batch, ns, g);
  if (st != ATSFFT_SUCCESS) return st;
  *bytes = g.total;
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_execute_uneven(atsfft_plan_t plan, int32_t batch, const void *x_dev, const int64_t *offsets,
                                    const int64_t *ns, int64_t *locs_dev, void *vals_dev, int32_t *count_dev,
                                    int32_t *khat_dev, uint32_t *sig_status_dev, void *ws_dev, size_t ws_bytes,
                                    hipStream_t stream) {
  if (!plan) return fail(ATSFFT_EINVAL, "null plan");
  if (!x_dev || !offsets || !locs_dev || !vals_dev || !count_dev || !khat_dev || !sig_status_dev || !ws_dev)
    return fail(ATSFFT_EINVAL, "null pointer");
  Groups g;
  atsfft_status st = make_groups(plan, batch, ns, g);
  if (st != ATSFFT_SUCCESS) return st;
  if (ws_bytes < g.total) return fail(ATSFFT_EINVAL, "workspace too small");
  for (int32_t i = 0; i < batch; ++i)
    if (offsets[i] < 0) return fail(ATSFFT_EINVAL, "negative offset");
  // per-signal tables, group by group: input offsets, then call indices
  if (!plan->stage_host || plan->stage_bytes < g.header) {
    if (plan->stage_host) {
      (void)hipEventSynchronize(plan->stage_done);
      (void)hipHostFree(plan->stage_host);
      plan->stage_host = nullptr;
    }
    if (hipHostMalloc(&plan->stage_host, g.header) != hipSuccess) return fail(ATSFFT_ENOMEM, "pinned staging allocation failed");
    plan->stage_bytes = g.header;
    if (!plan->stage_done && hipEventCreateWithFlags(&plan->stage_done, hipEventDisableTiming) != hipSuccess)
      return fail(ATSFFT_ELAUNCH, "hipEventCreate failed");
  } else if (plan->stage_done) {
    (void)hipEventSynchronize(plan->stage_done);  // the previous upload has read the buffer
  }
  int64_t *h_off = static_cast<int64_t *>(plan->stage_host);
  int32_t *h_map = reinterpret_cast<int32_t *>(static_cast<uint8_t *>(plan->stage_host) + align_up((size_t)batch * 8, 256));
  std::vector<int32_t> start(32, 0);
  int32_t k = 0;
  for (uint32_t lg = 0; lg < 32; ++lg) {
    start[lg] = k;
    for (int32_t i : g.members[lg]) {
      h_off[k] = offsets[i];
      h_map[k] = i;
      ++k;
    }
  }
  uint8_t *ws = static_cast<uint8_t *>(ws_dev);
  if (hipMemcpyAsync(ws, plan->stage_host, g.header, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipEventRecord(plan->stage_done, stream) != hipSuccess)
    return fail(ATSFFT_ELAUNCH, "table upload failed");
  const int64_t *d_off = reinterpret_cast<const int64_t *>(ws);
  const int32_t *d_map = reinterpret_cast<const int32_t *>(ws + align_up((size_t)batch * 8, 256));
  for (uint32_t lg = 0; lg < 32; ++lg) {
    const int32_t cnt = (int32_t)g.members[lg].size();
    if (!cnt) continue;
    const atsfft_plan_s *q = plan->sub[lg];
    const Layout lay = make_layout(q, cnt);
    KParams P = make_params(q, lay, x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev, ws + g.base[lg]);
    P.x_off = d_off + start[lg];
    P.sig_map = d_map + start[lg];
    if (launch_execute(P, q->d.dtype, cnt, stream, nullptr, nullptr) != hipSuccess) {
      hipError_t e = hipGetLastError();
      return fail(ATSFFT_ELAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
    }
  }
  return ATSFFT_SUCCESS;
}

// Workspace of atsfft_execute_uneven_dev: the per-length parameter table,
// then one slice of the plan's longest length per signal.
static size_t dev_table_bytes() { return align_up((size_t)32 * sizeof(KParams), 256); }

atsfft_status atsfft_workspace_size_uneven_dev(atsfft_plan_t plan, int32_t batch, size_t *bytes) {
  if (!plan || !bytes) return fail(ATSFFT_EINVAL, "null argument");
  if (!plan->dev_tmpl) return fail(ATSFFT_EINVAL, "plan has no device-length uneven form (1D, n_min > 0, res_tol = 0)");
  if (batch < 1 || batch > plan->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  *bytes = dev_table_bytes() + make_layout(plan, batch).total;
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_execute_uneven_dev(atsfft_plan_t plan, int32_t batch, const void *x_dev,
                                        const int64_t *offsets_dev, const int64_t *ns_dev, int64_t *locs_dev,
                                        void *vals_dev, int32_t *count_dev, int32_t *khat_dev,
                                        uint32_t *sig_status_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
  if (!plan) return fail(ATSFFT_EINVAL, "null plan");
  if (!plan->dev_tmpl) return fail(ATSFFT_EINVAL, "plan has no device-length uneven form (1D, n_min > 0, res_tol = 0)");
  if (plan->d.flags & ATSFFT_FLAG_PROFILE) return fail(ATSFFT_EINVAL, "no stage profile for the device-length uneven form");
  if (batch < 1 || batch > plan->d.max_batch) return fail(ATSFFT_EINVAL, "batch outside [1, max_batch]");
  if (!x_dev || !offsets_dev || !ns_dev || !locs_dev || !vals_dev || !count_dev || !khat_dev || !sig_status_dev ||
      !ws_dev)
    return fail(ATSFFT_EINVAL, "null device pointer");
  const size_t tb = dev_table_bytes();
  const Layout lay = make_layout(plan, batch);
  if (ws_bytes < tb + lay.total) return fail(ATSFFT_EINVAL, "workspace too small");
  uint8_t *ws = static_cast<uint8_t *>(ws_dev);
  KParams P = make_params(plan, lay, x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev, ws + tb);
  P.x_off = offsets_dev;
  P.ns = ns_dev;
  P.devP = reinterpret_cast<const KParams *>(ws);
  P.dev_lg_lo = plan->dev_lg_lo;
  P.dev_lg_hi = plan->dev_lg_hi;
  const KParams *tmpl = plan->dev_tmpl;
  const int dtype = plan->d.dtype;
  if (plan->d.flags & ATSFFT_FLAG_GRAPH) {
    const void *key[9] = {x_dev, locs_dev, vals_dev, count_dev, khat_dev, sig_status_dev, ws_dev, offsets_dev, ns_dev};
    return graph_launch(plan, 1, batch, key, stream, [&](hipStream_t cs) {
      return launch_execute_dev(P, tmpl, dtype, batch, cs);
    });
  }
  if (launch_execute_dev(P, tmpl, dtype, batch, stream) != hipSuccess) {
    hipError_t e = hipGetLastError();
    return fail(ATSFFT_ELAUNCH, std::string("launch failed: ") + hipGetErrorString(e));
  }
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_trace_read(atsfft_plan_t plan, const void *ws_dev, int32_t signal, atsfft_trace *out,
                                hipStream_t stream) {
  if (!plan || !ws_dev || !out) return fail(ATSFFT_EINVAL, "null argument");
  if (signal < 0 || signal >= plan->d.max_batch) return fail(ATSFFT_EINVAL, "signal outside [0, max_batch)");
  const atsfft_desc &d = plan->d;
  const Layout lay = make_layout(plan, 1);
  const uint8_t *ws = static_cast<const uint8_t *>(ws_dev) + (size_t)signal * lay.slice;
  const size_t cs = d.dtype == ATSFFT_C64 ? 8 : 16;
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(ATSFFT_ELAUNCH, "stream synchronisation failed");
  SigState s;
  bool ok = hipMemcpy(&s, ws + lay.state, sizeof(s), hipMemcpyDeviceToHost) ==
            hipSuccess;
  if (!ok) return fail(ATSFFT_ELAUNCH, "trace copy failed");
  out->B_star = s.B_star;
  out->khat = s.khat;
  out->n_probe = s.n_probe;
  out->count = (int32_t)s.count;
  out->status = s.status;
  out->res_ratio = s.res_ratio;
  out->retries = s.pass;
  if (out->probe_B || out->probe_k || out->probe_dec || out->probe_T) {
    std::vector<ProbeRec> h((size_t)kMaxProbe);
    ok = hipMemcpy(h.data(), ws + lay.hist, kMaxProbe * sizeof(ProbeRec),
                   hipMemcpyDeviceToHost) == hipSuccess;
    for (int i = 0; ok && i < d.P_max; ++i) {
      if (out->probe_B) out->probe_B[i] = h[(size_t)i].B;
      if (out->probe_k) out->probe_k[i] = h[(size_t)i].k;
      if (out->probe_dec) out->probe_dec[i] = h[(size_t)i].dec;
      if (out->probe_T) out->probe_T[i] = h[(size_t)i].T;
    }
  }
  if (ok && out->T_loc)
    ok = hipMemcpy(out->T_loc, ws + lay.tloc, (size_t)d.L_loc * 8,
                   hipMemcpyDeviceToHost) == hipSuccess;
  if (ok && out->J_count)
    ok = hipMemcpy(out->J_count, ws + lay.jcount, (size_t)d.L_loc * 4,
                   hipMemcpyDeviceToHost) == hipSuccess;
  if (ok && out->yhat) {
    const size_t L = (size_t)(d.L_loc + d.L_est);
    for (size_t l = 0; ok && l < L; ++l)
      ok = hipMemcpy(static_cast<uint8_t *>(out->yhat) + l * plan->Bc_max * cs,
                     ws + lay.ymain + l * lay.ymain_loop, plan->Bc_max * cs,
                     hipMemcpyDeviceToHost) == hipSuccess;
  }
  if (ok && out->J_bits) {
    const size_t words = (plan->Bc_max + 31) / 32;
    for (int l = 0; ok && l < d.L_loc; ++l)
      ok = hipMemcpy(out->J_bits + (size_t)l * words, ws + lay.jbits + l * lay.jbits_loop,
                     words * 4, hipMemcpyDeviceToHost) == hipSuccess;
  }
  if (!ok) return fail(ATSFFT_ELAUNCH, "trace copy failed");
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_profile_read(atsfft_plan_t plan, double *stage_ms, int32_t *executes) {
  if (!plan || !stage_ms || !executes) return fail(ATSFFT_EINVAL, "null argument");
  for (int i = 0; i < ATSFFT_NUM_STAGES; ++i) stage_ms[i] = 0.0;
  *executes = (int32_t)plan->prof_used.size();
  for (auto &rec : plan->prof_used) {
    if (hipEventSynchronize(rec[5]) != hipSuccess) return fail(ATSFFT_ELAUNCH, "hipEventSynchronize failed");
    for (int i = 0; i < ATSFFT_NUM_STAGES; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, rec[(size_t)i], rec[(size_t)i + 1]) != hipSuccess)
        return fail(ATSFFT_ELAUNCH, "hipEventElapsedTime failed");
      stage_ms[i] += (double)ms;
    }
  }
  for (auto &rec : plan->prof_used) plan->prof_free.push_back(rec);
  plan->prof_used.clear();
  return ATSFFT_SUCCESS;
}

atsfft_status atsfft_destroy(atsfft_plan_t plan) {
  free_plan(plan);
  return ATSFFT_SUCCESS;
}

}  // extern "C"
