/*
 * FP64 CPU oracle of ATSFFT, the adaptive-tuning sparse FFT with sparsity
 * detection of Shi, Yang, Zhang and You (arXiv:1908.02461).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, literal reading of the paper.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * Conventions (paper Sec. II, first paragraphs):
 *   - complex arrays are interleaved (re, im) doubles;
 *   - 1D signals have length n, 2D images are N x N stored row-major, x[u*N+v];
 *   - n, N and B are powers of two, B divides n;
 *   - the DFT is unnormalised with omega = exp(-2 pi i / n) (the DFT display).
 */
#ifndef ATSFFT_ORACLE_H
#define ATSFFT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* draw phases: the probe iterations, the location loops, the estimation loops */
enum { OR_PHASE_PROBE = 0, OR_PHASE_LOC = 1, OR_PHASE_EST = 2 };

/* per-signal status bits */
enum {
  OR_OK = 0,
  OR_TRUNCATED = 1,
  OR_PROBE_NOT_CONVERGED = 2,
  OR_PROBE_SATURATED = 4,
  OR_EMPTY = 8,
  OR_RETRIED = 16 /* the residual test re-ran location and estimation at a larger B */
};

typedef struct {
  int ndim;          /* 1 or 2 */
  int64_t n;         /* 1D length, or 2D side N */
  int64_t B0;        /* first probe bucket count (per axis) */
  int64_t B_max;     /* largest bucket count the probe may reach (per axis) */
  int alpha_probe;   /* window length factor during the probe, w = alpha_probe*B */
  int alpha;         /* window length factor of location/estimation loops */
  int L_loc, L_est;  /* loop counts */
  int T_vote;        /* vote threshold */
  int P_max;         /* probe iteration limit */
  int d;             /* cutoff multiplier, num = d * khat */
  int gamma;         /* occupancy guard: a count k is trusted once B^ndim >= gamma*k (0: off) */
  double delta;      /* window leakage tolerance */
  double q;          /* noise-floor quantile */
  double noise_rate; /* false-bucket rate: c_noise = ln(Bcount / noise_rate) */
  double rho;        /* relative floor: T >= rho * max m */
  uint64_t seed;
  uint32_t signal;   /* signal index inside a batch (a draw key) */
  int64_t fixed_B;   /* > 0: skip the probe (Algorithm 1 form) */
  int64_t fixed_k;   /* khat used when fixed_B > 0 */
  int64_t max_out;   /* capacity of locs / vals */
  double res_tol;    /* residual test (an addition to the method): > 0 re-runs location and
                        estimation at 2 B_star while E_res / E_tot exceeds it; 0 disables */
  int res_retries;   /* at most this many re-runs (<= 7) */
} or_params;

#define OR_TRACE_MAX_PROBE 64
#define OR_TRACE_MAX_LOOPS 64

typedef struct {
  /* results */
  int status;
  int64_t khat, B_star, count;
  /* probe trace */
  int n_probe;
  int64_t probe_B[OR_TRACE_MAX_PROBE];
  int64_t probe_k[OR_TRACE_MAX_PROBE];
  double probe_T[OR_TRACE_MAX_PROBE];
  int probe_decision[OR_TRACE_MAX_PROBE]; /* -1 halve, 0 keep, +1 double */
  /* main-loop trace */
  double T_loc[OR_TRACE_MAX_LOOPS];
  int64_t J_count[OR_TRACE_MAX_LOOPS];
  /* caller-owned arrays, each may be NULL */
  double *yhat;   /* [(L_loc+L_est)][Bcount_max] complex, Bcount = B^ndim at B_star */
  int64_t yhat_stride; /* complex elements per loop in yhat (>= B_star^ndim) */
  uint8_t *J;     /* [L_loc][yhat_stride] membership flags */
  int64_t *locs;  /* [max_out] ascending */
  double *vals;   /* [max_out] complex */
  double *est;    /* [max_out][L_est] complex, per-loop estimates */
  /* residual test */
  double res_ratio; /* E_res / E_tot of the last pass (0 when the test is off) */
  int retries;      /* passes re-run at a larger B */
} or_result;

/* ---- building blocks, each exported so tests can pin it on its own ---- */
int or_residual_reach(int alpha, double delta);
void or_residual(int ndim, int64_t n, int64_t B, int64_t w, const double *G, int R, int L,
                 const int64_t *sigma, const int64_t *tau, const double *yhat, int64_t S, const int64_t *locs,
                 const double *vals, double *E_res, double *E_tot);
uint64_t or_splitmix64_at(uint64_t seed, uint64_t index);
uint64_t or_draw_word(uint64_t seed, uint32_t signal, int phase, int iter, int axis);
void or_draw(uint64_t seed, uint32_t signal, int phase, int iter, int axis, int64_t n,
             int64_t *sigma, int64_t *tau, int64_t *sigma_inv);
int64_t or_inverse_mod(int64_t a, int64_t n);

void or_dft_naive(int64_t n, const double *x, double *X);
void or_fft(int64_t n, const double *x, double *X);
void or_fft2(int64_t N, const double *x, double *X);
void or_idft_naive(int64_t n, const double *X, double *x);

int64_t or_window_len(int64_t n, int64_t B, int alpha);
void or_window_taps(int64_t n, int64_t B, int64_t w, double delta, double *G);
double or_window_hat(int64_t n, int64_t w, const double *G, int64_t q, double *im_out);

int64_t or_hash_bucket(int64_t n, int64_t B, int64_t sigma, int64_t f);
int64_t or_hash_offset(int64_t n, int64_t B, int64_t sigma, int64_t f);

void or_hash_1d(int64_t n, const double *x, int64_t sigma, int64_t tau, int64_t B, int64_t w,
                const double *G, double *yhat);
void or_hash_2d(int64_t N, const double *x, const int64_t *sigma, const int64_t *tau, int64_t B,
                int64_t w, const double *G, double *yhat);

double or_threshold(const double *m, int64_t count, double q, double noise_rate, double rho);
int64_t or_local_max_1d(const double *m, int64_t B, double T);
int64_t or_local_max_2d(const double *m, int64_t B, double T);
int or_rule(int64_t k_prev, int64_t k_cur);
int64_t or_topnum(const double *m, int64_t count, double T, int64_t num, uint8_t *J);
void or_vote_hist(int ndim, int64_t n, int64_t B, int L, const int64_t *sigma_inv,
                  const uint8_t *J, int32_t *votes);
double or_median(const double *v, int L);

double or_l1_error(int64_t total, const double *Xtrue, int64_t count, const int64_t *locs,
                   const double *vals, int64_t k);

/* State of the adaptive-B probe (Sec. III-A, Algorithm 2) between its
   iterations.  or_probe_init starts it at B0; or_probe_step takes the
   local-maximum count k of the iteration just hashed at s->B and applies the
   B-update rule, the occupancy guard and the stop rules, returning the
   decision (-1 halve, 0 keep, +1 double).  Once s->done is set, B_star, khat
   and status (OR_PROBE_SATURATED, OR_PROBE_NOT_CONVERGED, OR_EMPTY) hold the
   probe's outcome. */
typedef struct {
  int64_t B;        /* bucket count (per axis) of the next iteration */
  int64_t k_prev;   /* the previous iteration's count */
  uint64_t visited; /* bit log2(B) set once B was hashed */
  int iter;         /* iterations run */
  int done;
  int status;
  int64_t B_star, khat;
} or_probe_state;

void or_probe_init(const or_params *p, or_probe_state *s);
int or_probe_step(const or_params *p, or_probe_state *s, int64_t k);

void or_default_params(or_params *p, int ndim, int64_t n);
int or_atsfft(const or_params *p, const double *x, or_result *r);

#ifdef __cplusplus
}
#endif
#endif
