/*
 * FP64 CPU oracle of ATSFFT (arXiv:1908.02461).  TEST INFRASTRUCTURE ONLY:
 * loaded by the test suite, the smoke check and the benchmark's CPU-baseline
 * leg, never by the GPU library, with which it shares no code.
 *
 * Every function is a plain, sequential, literal statement of one step of the
 * paper's method, with no blocking, fusion or reordering.  Where the paper is
 * silent or garbled the reading taken is stated next to the code.
 *
 * Pins (tests/test_oracle_*.py): naive DFT vs radix-2 FFT vs numpy; Parseval;
 * impulse and tone closed forms; Lemma 1 and Lemma 2 by brute force; window
 * symmetry, flatness and stop band against the analytic Gaussian-times-box
 * form; the hash partition; exact estimation of 1-sparse inputs; median vs a
 * full sort; vote histogram vs direct evaluation of every hash; the B-update
 * rule table at its exact boundaries; the error metric on hand cases; the
 * paper's two-spike example; exact recovery of planted noiseless spectra;
 * published SplitMix64 outputs.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Random draws                                                              */
/* ------------------------------------------------------------------------ */

/*
 * SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the state advances by the golden-ratio gamma and
 * each output is the state passed through the variant-13 finaliser.  The
 * index-th output of a stream seeded with `seed` is the finaliser applied to
 * seed + (index + 1) * gamma, which makes the generator counter-based.
 */
uint64_t or_splitmix64_at(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* The draw counter packs (signal, phase, iteration, axis). */
uint64_t or_draw_word(uint64_t seed, uint32_t signal, int phase, int iter, int axis) {
  uint64_t index = ((((uint64_t)signal * 4u + (uint64_t)phase) * 256u + (uint64_t)iter) * 2u) +
                   (uint64_t)axis;
  return or_splitmix64_at(seed, index);
}

/* Multiplicative inverse modulo n by the extended Euclidean algorithm. */
int64_t or_inverse_mod(int64_t a, int64_t n) {
  int64_t t = 0, newt = 1, r = n, newr = a % n;
  while (newr != 0) {
    int64_t qq = r / newr;
    int64_t tmp = t - qq * newt;
    t = newt;
    newt = tmp;
    tmp = r - qq * newr;
    r = newr;
    newr = tmp;
  }
  if (r != 1) return -1; /* not invertible */
  if (t < 0) t += n;
  return t;
}

/*
 * One loop's permutation (Definition 1): sigma odd, hence invertible modulo
 * the power of two n; tau uniform in [n].  sigma comes from the low word of
 * the draw, tau from the high word.
 */
void or_draw(uint64_t seed, uint32_t signal, int phase, int iter, int axis, int64_t n,
             int64_t *sigma, int64_t *tau, int64_t *sigma_inv) {
  uint64_t r = or_draw_word(seed, signal, phase, iter, axis);
  int64_t s = (int64_t)((r & 0xFFFFFFFFull) % (uint64_t)n) | 1;
  int64_t t = (int64_t)((r >> 32) % (uint64_t)n);
  *sigma = s;
  *tau = t;
  *sigma_inv = or_inverse_mod(s, n);
}

/* ------------------------------------------------------------------------ */
/* DFT (Sec. II, the DFT display: unnormalised, omega = e^{-2 pi i / n})      */
/* ------------------------------------------------------------------------ */

/* omega^m for an exact integer exponent m reduced modulo n */
static void omega_pow(int64_t n, int64_t m, double *re, double *im) {
  m %= n;
  if (m < 0) m += n;
  double ang = -2.0 * OR_PI * (double)m / (double)n;
  *re = cos(ang);
  *im = sin(ang);
}

void or_dft_naive(int64_t n, const double *x, double *X) {
  for (int64_t f = 0; f < n; f++) {
    double sr = 0.0, si = 0.0;
    for (int64_t u = 0; u < n; u++) {
      double wr, wi;
      omega_pow(n, (f * u) % n, &wr, &wi);
      sr += x[2 * u] * wr - x[2 * u + 1] * wi;
      si += x[2 * u] * wi + x[2 * u + 1] * wr;
    }
    X[2 * f] = sr;
    X[2 * f + 1] = si;
  }
}

/* x_u = (1/n) sum_f X_f omega^{-f u}: the inverse of the DFT display */
void or_idft_naive(int64_t n, const double *X, double *x) {
  for (int64_t u = 0; u < n; u++) {
    double sr = 0.0, si = 0.0;
    for (int64_t f = 0; f < n; f++) {
      double wr, wi;
      omega_pow(n, -((f * u) % n), &wr, &wi);
      sr += X[2 * f] * wr - X[2 * f + 1] * wi;
      si += X[2 * f] * wi + X[2 * f + 1] * wr;
    }
    x[2 * u] = sr / (double)n;
    x[2 * u + 1] = si / (double)n;
  }
}

/* Radix-2 decimation-in-time FFT computing the same sum as or_dft_naive. */
void or_fft(int64_t n, const double *x, double *X) {
  int lg = 0;
  while (((int64_t)1 << lg) < n) lg++;
  for (int64_t i = 0; i < n; i++) {
    int64_t j = 0;
    for (int b = 0; b < lg; b++)
      if (i & ((int64_t)1 << b)) j |= (int64_t)1 << (lg - 1 - b);
    X[2 * j] = x[2 * i];
    X[2 * j + 1] = x[2 * i + 1];
  }
  double *tw = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n : 2));
  for (int64_t m = 0; m < n / 2; m++) omega_pow(n, m, &tw[2 * m], &tw[2 * m + 1]);
  for (int64_t len = 2; len <= n; len <<= 1) {
    int64_t half = len / 2, step = n / len;
    for (int64_t s = 0; s < n; s += len) {
      for (int64_t k = 0; k < half; k++) {
        double wr = tw[2 * (k * step)], wi = tw[2 * (k * step) + 1];
        double *u = &X[2 * (s + k)], *v = &X[2 * (s + k + half)];
        double vr = v[0] * wr - v[1] * wi, vi = v[0] * wi + v[1] * wr;
        double ur = u[0], ui = u[1];
        u[0] = ur + vr;
        u[1] = ui + vi;
        v[0] = ur - vr;
        v[1] = ui - vi;
      }
    }
  }
  free(tw);
}

/* 2D DFT of an N x N row-major image: rows, then columns. */
void or_fft2(int64_t N, const double *x, double *X) {
  double *a = (double *)malloc(sizeof(double) * 2 * (size_t)N);
  double *b = (double *)malloc(sizeof(double) * 2 * (size_t)N);
  for (int64_t r = 0; r < N; r++) or_fft(N, x + 2 * r * N, X + 2 * r * N);
  for (int64_t c = 0; c < N; c++) {
    for (int64_t r = 0; r < N; r++) {
      a[2 * r] = X[2 * (r * N + c)];
      a[2 * r + 1] = X[2 * (r * N + c) + 1];
    }
    or_fft(N, a, b);
    for (int64_t r = 0; r < N; r++) {
      X[2 * (r * N + c)] = b[2 * r];
      X[2 * (r * N + c) + 1] = b[2 * r + 1];
    }
  }
  free(a);
  free(b);
}

/* ------------------------------------------------------------------------ */
/* Flat window (Sec. II-A-2, the box-car and Gaussian displays)               */
/* ------------------------------------------------------------------------ */

/*
 * Reading of the window paragraph: the flat window is the Gaussian convolved
 * with a box car in the frequency domain, so in time it is the Gaussian
 * multiplied by the box car's time image, the Dirichlet kernel
 * D_c(t) = sum_{|o|<=c} omega^{-o t} = sin(pi (2c+1) t / n) / sin(pi t / n),
 * with box half-width c = n/(2B) (one bucket).  The Gaussian's width s puts
 * it at delta at the window edge t = w/2, and the taps are t in [-w/2, w/2)
 * with G_{-w/2} = 0 so that the window is symmetric.
 */
int64_t or_window_len(int64_t n, int64_t B, int alpha) {
  int64_t w = (int64_t)alpha * B;
  return w > n ? n : w;
}

void or_window_taps(int64_t n, int64_t B, int64_t w, double delta, double *G) {
  double c = (double)(n / (2 * B));
  double s = ((double)w / 2.0) / sqrt(2.0 * log(1.0 / delta));
  for (int64_t i = 0; i < w; i++) {
    int64_t t = i - w / 2;
    if (t == -w / 2) {
      G[i] = 0.0;
      continue;
    }
    double gauss = exp(-((double)t * (double)t) / (2.0 * s * s));
    double dir;
    if (t == 0)
      dir = 2.0 * c + 1.0;
    else
      dir = sin(OR_PI * (2.0 * c + 1.0) * (double)t / (double)n) / sin(OR_PI * (double)t / (double)n);
    G[i] = gauss * dir;
  }
}

/* G'(q) = (1/n) sum_t G_t omega^{q t}, summed literally over the taps. */
double or_window_hat(int64_t n, int64_t w, const double *G, int64_t q, double *im_out) {
  double sr = 0.0, si = 0.0;
  for (int64_t i = 0; i < w; i++) {
    int64_t t = i - w / 2;
    double wr, wi;
    omega_pow(n, (q % n) * (t % n) % n, &wr, &wi);
    sr += G[i] * wr;
    si += G[i] * wi;
  }
  if (im_out) *im_out = si / (double)n;
  return sr / (double)n;
}

/* ------------------------------------------------------------------------ */
/* Hash function (Sec. II-A-3, the hash display; 2D read per axis)           */
/* ------------------------------------------------------------------------ */

/*
 * h(f) = round(sigma f B / n) with round half up, taken in integers:
 * p = sigma f mod n, h = ((p + n/(2B)) mod n) / (n/B).
 */
int64_t or_hash_bucket(int64_t n, int64_t B, int64_t sigma, int64_t f) {
  int64_t p = (sigma % n) * (f % n) % n;
  int64_t c = n / (2 * B);
  return ((p + c) % n) / (n / B);
}

/* o(f) = h(f) n/B - sigma f, taken modulo n in (-n/(2B), n/(2B)]. */
int64_t or_hash_offset(int64_t n, int64_t B, int64_t sigma, int64_t f) {
  int64_t p = (sigma % n) * (f % n) % n;
  int64_t h = or_hash_bucket(n, B, sigma, f);
  int64_t o = (h * (n / B) - p) % n;
  if (o < 0) o += n;
  if (o > n / 2) o -= n;
  return o;
}

/*
 * Permute, filter and subsample (Definition 1, the window paragraph, Lemma 2
 * with the index ranges read as u in [n/B], i in [B]):
 *   y_b = sum_{t = b mod B, -w/2 <= t < w/2} x[(sigma t + tau) mod n] G_t,
 * summed in increasing t, followed by the B-point DFT.
 */
void or_hash_1d(int64_t n, const double *x, int64_t sigma, int64_t tau, int64_t B, int64_t w,
                const double *G, double *yhat) {
  double *y = (double *)calloc(2 * (size_t)B, sizeof(double));
  for (int64_t i = 0; i < w; i++) {
    int64_t t = i - w / 2;
    int64_t a = ((sigma * t + tau) % n + n) % n;
    int64_t b = ((t % B) + B) % B;
    y[2 * b] += x[2 * a] * G[i];
    y[2 * b + 1] += x[2 * a + 1] * G[i];
  }
  or_fft(B, y, yhat);
  free(y);
}

/* 2D form: separable window G_{t1} G_{t2}, per-axis permutation, B x B DFT. */
void or_hash_2d(int64_t N, const double *x, const int64_t *sigma, const int64_t *tau, int64_t B,
                int64_t w, const double *G, double *yhat) {
  double *y = (double *)calloc(2 * (size_t)(B * B), sizeof(double));
  for (int64_t i1 = 0; i1 < w; i1++) {
    int64_t t1 = i1 - w / 2;
    int64_t a1 = ((sigma[0] * t1 + tau[0]) % N + N) % N;
    int64_t b1 = ((t1 % B) + B) % B;
    for (int64_t i2 = 0; i2 < w; i2++) {
      int64_t t2 = i2 - w / 2;
      int64_t a2 = ((sigma[1] * t2 + tau[1]) % N + N) % N;
      int64_t b2 = ((t2 % B) + B) % B;
      double g = G[i1] * G[i2];
      const double *xa = &x[2 * (a1 * N + a2)];
      y[2 * (b1 * B + b2)] += xa[0] * g;
      y[2 * (b1 * B + b2) + 1] += xa[1] * g;
    }
  }
  or_fft2(B, y, yhat);
  free(y);
}

/* ------------------------------------------------------------------------ */
/* Significance and local maxima (Sec. III-A, "number of local maximum      */
/* points"; Algorithm 2, the local-maximum step)                             */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/*
 * Significance threshold on m_b = |yhat_b|^2.  The paper does not state one;
 * the reading: an empty bucket's energy is exponential, so its q-quantile
 * over the buckets (the floor(q (count-1))-th order statistic) divided by
 * -ln(1-q) estimates the noise level; buckets above c_noise times that, with
 * c_noise = ln(count / noise_rate), are significant, and a relative floor
 * rho * max m guards noiseless inputs.
 */
double or_threshold(const double *m, int64_t count, double q, double noise_rate, double rho) {
  double *s = (double *)malloc(sizeof(double) * (size_t)count);
  memcpy(s, m, sizeof(double) * (size_t)count);
  qsort(s, (size_t)count, sizeof(double), cmp_double);
  int64_t qi = (int64_t)floor(q * (double)(count - 1));
  double floor_est = s[qi] / (-log(1.0 - q));
  double mx = s[count - 1];
  free(s);
  double c_noise = log((double)count / noise_rate);
  double t1 = c_noise * floor_est, t2 = rho * mx;
  return t1 > t2 ? t1 : t2;
}

/* key order: larger m first, equal m broken by the smaller index */
static int key_gt(const double *m, int64_t a, int64_t b) {
  return m[a] > m[b] || (m[a] == m[b] && a < b);
}

/* Count of significant buckets whose key beats both ring neighbours. */
int64_t or_local_max_1d(const double *m, int64_t B, double T) {
  int64_t cnt = 0;
  for (int64_t b = 0; b < B; b++) {
    if (!(m[b] > T)) continue;
    int64_t l = (b - 1 + B) % B, r = (b + 1) % B;
    if (key_gt(m, b, l) && key_gt(m, b, r)) cnt++;
  }
  return cnt;
}

/* 2D: the 8-neighbourhood on the B x B torus, bucket index b1*B + b2. */
int64_t or_local_max_2d(const double *m, int64_t B, double T) {
  int64_t cnt = 0;
  for (int64_t b1 = 0; b1 < B; b1++) {
    for (int64_t b2 = 0; b2 < B; b2++) {
      int64_t b = b1 * B + b2;
      if (!(m[b] > T)) continue;
      int is_max = 1;
      for (int d1 = -1; d1 <= 1 && is_max; d1++) {
        for (int d2 = -1; d2 <= 1; d2++) {
          if (d1 == 0 && d2 == 0) continue;
          int64_t nb = ((b1 + d1 + B) % B) * B + ((b2 + d2 + B) % B);
          if (!key_gt(m, b, nb)) {
            is_max = 0;
            break;
          }
        }
      }
      cnt += is_max;
    }
  }
  return cnt;
}

/*
 * The B-update rule with the paper's constants (the display with 1/2, 1, 2
 * and 2%, 5%): r = |1 - k_i / k_{i-1}|.  Read in exact integers with
 * D = |k_i - k_{i-1}|: 100 D < 2 k_{i-1} halves, 100 D < 5 k_{i-1} keeps,
 * anything else doubles.  The ratio is undefined at k_{i-1} = 0; B doubles.
 * Returns -1 (halve), 0 (keep), +1 (double).
 */
int or_rule(int64_t k_prev, int64_t k_cur) {
  if (k_prev <= 0) return 1;
  int64_t D = k_cur > k_prev ? k_cur - k_prev : k_prev - k_cur;
  if (100 * D < 2 * k_prev) return -1;
  if (100 * D < 5 * k_prev) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Cutoff (Algorithm 1, "num largest"; Sec. III-A, "top dk")                  */
/* ------------------------------------------------------------------------ */

static const double *g_sort_m;
static int cmp_key_desc(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  if (key_gt(g_sort_m, x, y)) return -1;
  if (key_gt(g_sort_m, y, x)) return 1;
  return 0;
}

/* J = the min(num, #{m > T}) largest keys among the significant buckets. */
int64_t or_topnum(const double *m, int64_t count, double T, int64_t num, uint8_t *J) {
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
  int64_t c = 0;
  for (int64_t b = 0; b < count; b++)
    if (m[b] > T) idx[c++] = b;
  g_sort_m = m;
  qsort(idx, (size_t)c, sizeof(int64_t), cmp_key_desc);
  int64_t take = c < num ? c : num;
  memset(J, 0, (size_t)count);
  for (int64_t i = 0; i < take; i++) J[idx[i]] = 1;
  free(idx);
  return take;
}

/* ------------------------------------------------------------------------ */
/* Reverse hash and vote (Algorithm 1 / 2, reverse-hash and keep steps)      */
/* ------------------------------------------------------------------------ */

/*
 * Literal histogram: every selected bucket j of loop l votes once for each
 * frequency that hashes into it, i.e. for sigma_l^{-1} p with the permuted
 * position p in [j n/B - n/(2B), j n/B + n/(2B)).  2D: per axis.
 * votes has n (1D) or N*N (2D) counters, zeroed by the caller.
 */
void or_vote_hist(int ndim, int64_t n, int64_t B, int L, const int64_t *sigma_inv,
                  const uint8_t *J, int32_t *votes) {
  int64_t c = n / (2 * B), width = n / B;
  int64_t count = ndim == 1 ? B : B * B;
  for (int l = 0; l < L; l++) {
    const uint8_t *Jl = J + (size_t)l * (size_t)count;
    for (int64_t j = 0; j < count; j++) {
      if (!Jl[j]) continue;
      if (ndim == 1) {
        int64_t si = sigma_inv[l];
        for (int64_t k = 0; k < width; k++) {
          int64_t p = ((j * width - c + k) % n + n) % n;
          votes[(si * p) % n] += 1;
        }
      } else {
        int64_t j1 = j / B, j2 = j % B;
        int64_t s1 = sigma_inv[2 * l], s2 = sigma_inv[2 * l + 1];
        for (int64_t k1 = 0; k1 < width; k1++) {
          int64_t p1 = ((j1 * width - c + k1) % n + n) % n;
          int64_t f1 = (s1 * p1) % n;
          for (int64_t k2 = 0; k2 < width; k2++) {
            int64_t p2 = ((j2 * width - c + k2) % n + n) % n;
            int64_t f2 = (s2 * p2) % n;
            votes[f1 * n + f2] += 1;
          }
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Median (Sec. II-B: median over the estimation loops, per real/imag part) */
/* ------------------------------------------------------------------------ */

double or_median(const double *v, int L) {
  double *s = (double *)malloc(sizeof(double) * (size_t)L);
  memcpy(s, v, sizeof(double) * (size_t)L);
  qsort(s, (size_t)L, sizeof(double), cmp_double);
  double r = (L % 2) ? s[L / 2] : 0.5 * (s[L / 2 - 1] + s[L / 2]);
  free(s);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Error metric (Sec. IV-C display): (1/k) sum over all bins |x'_f - x_f|    */
/* ------------------------------------------------------------------------ */

double or_l1_error(int64_t total, const double *Xtrue, int64_t count, const int64_t *locs,
                   const double *vals, int64_t k) {
  double acc = 0.0;
  int64_t s = 0;
  for (int64_t f = 0; f < total; f++) {
    double er = 0.0, ei = 0.0;
    if (s < count && locs[s] == f) {
      er = vals[2 * s];
      ei = vals[2 * s + 1];
      s++;
    }
    acc += hypot(er - Xtrue[2 * f], ei - Xtrue[2 * f + 1]);
  }
  return acc / (double)k;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2                                                               */
/* ------------------------------------------------------------------------ */

static int64_t bcount(int ndim, int64_t B);

/*
 * The probe of Algorithm 2 as a state machine, one call per iteration.  The
 * paper runs a fixed number of iterations and gives no stop rule; the
 * readings taken here:
 *   - the first iteration hashes at B0 and always doubles (B1 = 2 B0);
 *   - later ones apply or_rule to (k_{i-1}, k_i); k_{i-1} = 0 doubles, so
 *     a run of zero counts keeps doubling;
 *   - occupancy guard: while B^ndim < gamma k_i the count is not acted on
 *     and B doubles (gamma = 0: the rule alone, as printed);
 *   - keep stops at B with khat = k_i;
 *   - halve stops at B/2 with khat = k_i when B/2 was already hashed, and at
 *     B (khat = k_i) when B/2 would fall below B0 or below the guard;
 *     otherwise B halves (on the doubling chain B/2 has always been hashed);
 *   - doubling past B_max stops at B, PROBE_SATURATED;
 *   - after P_max iterations without a stop: B and khat of the last one,
 *     PROBE_NOT_CONVERGED;
 *   - a probe that ends with khat = 0 is EMPTY.
 */
void or_probe_init(const or_params *p, or_probe_state *s) {
  memset(s, 0, sizeof(*s));
  s->B = p->B0;
}

int or_probe_step(const or_params *p, or_probe_state *s, int64_t k) {
  int64_t B = s->B;
  int64_t cnt = bcount(p->ndim, B);
  int lgB = 0;
  while (((int64_t)1 << lgB) < B) lgB++;
  s->visited |= (uint64_t)1 << lgB;
  int dec = (s->iter == 0) ? 1 : or_rule(s->k_prev, k);
  /* occupancy guard: while fewer than gamma buckets per counted maximum
     exist, merged neighbours bias the count and the ratio means nothing */
  if (p->gamma > 0 && cnt < (int64_t)p->gamma * k) dec = 1;
  s->iter++;
  int stopped = 0;
  if (dec == 0) {
    s->B_star = B;
    s->khat = k;
    stopped = 1;
  } else if (dec < 0) {
    if (B / 2 < p->B0 || (p->gamma > 0 && bcount(p->ndim, B / 2) < (int64_t)p->gamma * k)) {
      s->B_star = B;
      s->khat = k;
      stopped = 1;
    } else if (s->visited & ((uint64_t)1 << (lgB - 1))) {
      s->B_star = B / 2;
      s->khat = k;
      stopped = 1;
    } else {
      s->B = B / 2;
    }
  } else {
    if (2 * B > p->B_max) {
      s->B_star = B;
      s->khat = k;
      s->status |= OR_PROBE_SATURATED;
      stopped = 1;
    } else {
      s->B = 2 * B;
    }
  }
  if (!stopped) {
    s->k_prev = k;
    s->B_star = B;
    s->khat = k;
    if (s->iter >= p->P_max) {
      s->status |= OR_PROBE_NOT_CONVERGED;
      stopped = 1;
    }
  }
  if (stopped) {
    s->done = 1;
    if (s->khat <= 0) s->status |= OR_EMPTY;
  }
  return dec;
}

void or_default_params(or_params *p, int ndim, int64_t n) {
  memset(p, 0, sizeof(*p));
  p->ndim = ndim;
  p->n = n;
  p->alpha_probe = 16;
  p->alpha = 32;
  if (ndim == 1) {
    p->B0 = 32;
    p->B_max = n / p->alpha < 16384 ? n / p->alpha : 16384;
  } else {
    p->B0 = 8;
    p->B_max = n / p->alpha < 128 ? n / p->alpha : 128;
  }
  p->L_loc = 9;
  p->L_est = 9;
  p->T_vote = 5;
  p->P_max = 12;
  p->d = 2;
  p->gamma = 32;
  p->delta = 1e-8;
  p->q = 0.1;
  p->noise_rate = 0.01;
  p->rho = 1e-6;
  p->seed = 0;
  p->signal = 0;
  p->fixed_B = 0;
  p->fixed_k = 0;
  p->max_out = 4096;
  p->res_tol = 0.0;
  p->res_retries = 1;
}

static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

/* hash one loop at bucket count B (per axis) with window factor alpha */
static void hash_loop(const or_params *p, const double *x, int phase, int iter, int64_t B,
                      int alpha, double *yhat, int64_t *sig, int64_t *tau, int64_t *sinv) {
  int64_t n = p->n;
  int64_t w = or_window_len(n, B, alpha);
  double *G = (double *)malloc(sizeof(double) * (size_t)w);
  or_window_taps(n, B, w, p->delta, G);
  for (int a = 0; a < p->ndim; a++)
    or_draw(p->seed, p->signal, phase, iter, a, n, &sig[a], &tau[a], &sinv[a]);
  if (p->ndim == 1)
    or_hash_1d(n, x, sig[0], tau[0], B, w, G, yhat);
  else
    or_hash_2d(n, x, sig, tau, B, w, G, yhat);
  free(G);
}

static int64_t bcount(int ndim, int64_t B) { return ndim == 1 ? B : B * B; }

/* Reach of the residual model in buckets on each side of a frequency's own
   bucket: the window's response falls to delta by n/(2B) + D, with the
   transition half-width D = (n/B) 2 ln(1/delta) / (pi alpha) of the Gaussian
   (the window paragraph of Sec. II-A-2 read as Gaussian times Dirichlet), and
   bucket h + j covers offsets up to (j + 1/2) n/B, so R = ceil(D B / n)
   buckets reach every response above delta. */
int or_residual_reach(int alpha, double delta) {
  double d = 2.0 * log(1.0 / delta) / (OR_PI * (double)alpha);
  int R = (int)ceil(d);
  return R < 1 ? 1 : R;
}

/* Residual energy of the estimation loops against the bucket values the
   located set predicts (a check added to the method, not in the paper).  By
   Lemma 1 and the fold, a coefficient X_f puts X_f omega^{-tau f} G'(q) into
   bucket b with q = b n/B - sigma f (per axis, centred mod n); the model keeps
   every located f in the buckets h - R .. h + R around its own bucket h (per
   axis; R at most (B-1)/2 so no bucket is reached twice).  E_res = sum over
   loops and buckets of |yhat - model|^2, E_tot = sum of |yhat|^2. */
void or_residual(int ndim, int64_t n, int64_t B, int64_t w, const double *G, int R, int L,
                 const int64_t *sigma, const int64_t *tau, const double *yhat, int64_t S, const int64_t *locs,
                 const double *vals, double *E_res, double *E_tot) {
  int64_t cnt = ndim == 1 ? B : B * B;
  int64_t nb = n / B;
  if (R > (B - 1) / 2) R = (int)((B - 1) / 2);
  int span = 2 * R + 1;
  int64_t half = (int64_t)(R + 1) * nb; /* |q| <= (R + 1/2) n/B */
  double *M = (double *)malloc(sizeof(double) * 2 * (size_t)cnt);
  double *gq = (double *)malloc(sizeof(double) * (size_t)(2 * half + 1));
  uint8_t *gq_done = (uint8_t *)calloc((size_t)(2 * half + 1), 1);
  int64_t *hb = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)span);
  double *gb = (double *)malloc(sizeof(double) * 2 * (size_t)span);
  double er = 0.0, et = 0.0;
  for (int l = 0; l < L; l++) {
    const double *y = yhat + 2 * (size_t)l * (size_t)cnt;
    for (int64_t b = 0; b < 2 * cnt; b++) M[b] = 0.0;
    for (int64_t s = 0; s < S; s++) {
      int64_t f = locs[s];
      int64_t fa[2] = {ndim == 1 ? f : f / n, ndim == 1 ? 0 : f % n};
      int64_t ph = 0;
      /* per axis: buckets h + j, j in [-R, R], with q = o + j n/B */
      for (int a = 0; a < ndim; a++) {
        int64_t h = or_hash_bucket(n, B, sigma[ndim * l + a], fa[a]);
        int64_t o = or_hash_offset(n, B, sigma[ndim * l + a], fa[a]);
        for (int j = -R; j <= R; j++) {
          int64_t q = o + (int64_t)j * nb;
          if (!gq_done[q + half]) {
            gq[q + half] = or_window_hat(n, w, G, q, NULL);
            gq_done[q + half] = 1;
          }
          hb[a * span + (j + R)] = ((h + j) % B + B) % B;
          gb[a * span + (j + R)] = gq[q + half];
        }
        ph = (ph + (tau[ndim * l + a] % n) * fa[a]) % n;
      }
      /* X_f omega^{-tau f} */
      double wr, wi;
      omega_pow(n, (n - ph) % n, &wr, &wi);
      double cr = vals[2 * s] * wr - vals[2 * s + 1] * wi;
      double ci = vals[2 * s] * wi + vals[2 * s + 1] * wr;
      int s2 = ndim == 1 ? 1 : span;
      for (int i = 0; i < span; i++)
        for (int j = 0; j < s2; j++) {
          double g = gb[i] * (ndim == 1 ? 1.0 : gb[span + j]);
          int64_t b = ndim == 1 ? hb[i] : hb[i] * B + hb[span + j];
          M[2 * b] += cr * g;
          M[2 * b + 1] += ci * g;
        }
    }
    for (int64_t b = 0; b < cnt; b++) {
      double dr = y[2 * b] - M[2 * b], di = y[2 * b + 1] - M[2 * b + 1];
      er += dr * dr + di * di;
      et += y[2 * b] * y[2 * b] + y[2 * b + 1] * y[2 * b + 1];
    }
  }
  *E_res = er;
  *E_tot = et;
  free(M);
  free(gq);
  free(gq_done);
  free(hb);
  free(gb);
}

/* Location loops, vote and estimation at bucket count B_star (per axis) with
   the draws of pass `pass` (iteration index offset by 32 per pass); fills the
   located set, values and trace of r.  With the residual test enabled,
   *ratio = E_res / E_tot of the estimation loops. */
static void main_phase(const or_params *p, const double *x, int64_t B_star, int64_t khat, int pass,
                       or_result *r, double *ratio) {
  int64_t n = p->n;
  int nd = p->ndim;
  int off = 32 * pass;
  int64_t cnt = bcount(nd, B_star);
  double *yh = (double *)malloc(sizeof(double) * 2 * (size_t)cnt);
  double *m = (double *)malloc(sizeof(double) * (size_t)cnt);
  int64_t sig[2], tau[2], sinv[2];
  int keep_trace = cnt <= r->yhat_stride;
  r->status &= ~OR_TRUNCATED;

  /* ---- location loops: hash, DFT, cutoff, reverse hash (votes) ---- */
  int64_t num = (int64_t)p->d * khat;
  if (num > cnt) num = cnt;
  uint8_t *J = (uint8_t *)calloc((size_t)(p->L_loc * cnt), 1);
  int64_t *sinv_loc = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)p->L_loc);
  for (int l = 0; l < p->L_loc; l++) {
    hash_loop(p, x, OR_PHASE_LOC, off + l, B_star, p->alpha, yh, sig, tau, sinv);
    for (int64_t b = 0; b < cnt; b++) m[b] = yh[2 * b] * yh[2 * b] + yh[2 * b + 1] * yh[2 * b + 1];
    double T = or_threshold(m, cnt, p->q, p->noise_rate, p->rho);
    r->T_loc[l] = T;
    r->J_count[l] = or_topnum(m, cnt, T, num, J + (size_t)l * (size_t)cnt);
    for (int a = 0; a < nd; a++) sinv_loc[nd * l + a] = sinv[a];
    if (r->yhat && keep_trace)
      memcpy(r->yhat + 2 * (size_t)l * (size_t)r->yhat_stride, yh, sizeof(double) * 2 * (size_t)cnt);
    if (r->J && keep_trace)
      memcpy(r->J + (size_t)l * (size_t)r->yhat_stride, J + (size_t)l * (size_t)cnt, (size_t)cnt);
  }
  int64_t total = nd == 1 ? n : n * n;
  int32_t *votes = (int32_t *)calloc((size_t)total, sizeof(int32_t));
  or_vote_hist(nd, n, B_star, p->L_loc, sinv_loc, J, votes);
  int64_t S = 0;
  for (int64_t f = 0; f < total; f++)
    if (votes[f] >= p->T_vote) S++;
  r->count = S;
  if (S > p->max_out) r->status |= OR_TRUNCATED;

  /* ---- estimation loops: hash, estimate, median ---- */
  int64_t *Sl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
  int64_t si = 0;
  for (int64_t f = 0; f < total; f++)
    if (votes[f] >= p->T_vote) Sl[si++] = f;
  double *e = (double *)malloc(sizeof(double) * 2 * (size_t)(S > 0 ? S : 1) * (size_t)p->L_est);
  int64_t w = or_window_len(n, B_star, p->alpha);
  double *G = (double *)malloc(sizeof(double) * (size_t)w);
  or_window_taps(n, B_star, w, p->delta, G);
  /* the estimation loops' bucket DFTs and draws, kept for the residual */
  int want_res = p->res_tol > 0.0;
  double *yest = want_res ? (double *)malloc(sizeof(double) * 2 * (size_t)cnt * (size_t)p->L_est) : NULL;
  int64_t *sig_est = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)p->L_est);
  int64_t *tau_est = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)p->L_est);
  /* G'(o) for o in (-n/(2B), n/(2B)], each evaluated once, on first use */
  int64_t cB = n / (2 * B_star);
  double *ghat = (double *)malloc(sizeof(double) * (size_t)(2 * cB + 1));
  uint8_t *ghat_done = (uint8_t *)calloc((size_t)(2 * cB + 1), 1);
  for (int l = 0; l < p->L_est; l++) {
    hash_loop(p, x, OR_PHASE_EST, off + l, B_star, p->alpha, yh, sig, tau, sinv);
    for (int a = 0; a < nd; a++) {
      sig_est[nd * l + a] = sig[a];
      tau_est[nd * l + a] = tau[a];
    }
    if (yest) memcpy(yest + 2 * (size_t)l * (size_t)cnt, yh, sizeof(double) * 2 * (size_t)cnt);
    if (r->yhat && keep_trace)
      memcpy(r->yhat + 2 * (size_t)(p->L_loc + l) * (size_t)r->yhat_stride, yh,
             sizeof(double) * 2 * (size_t)cnt);
    for (int64_t s = 0; s < S; s++) {
      int64_t f = Sl[s];
      int64_t fa[2] = {nd == 1 ? f : f / n, nd == 1 ? 0 : f % n};
      int64_t hb = 0, phase = 0;
      double gh = 1.0;
      for (int a = 0; a < nd; a++) {
        int64_t h = or_hash_bucket(n, B_star, sig[a], fa[a]);
        int64_t o = or_hash_offset(n, B_star, sig[a], fa[a]);
        hb = hb * B_star + h;
        phase = (phase + (tau[a] * fa[a]) % n) % n;
        if (!ghat_done[o + cB]) {
          ghat[o + cB] = or_window_hat(n, w, G, o, NULL);
          ghat_done[o + cB] = 1;
        }
        gh *= ghat[o + cB];
      }
      /* the estimator display: yhat_h omega^{tau f} / G'(o) */
      double wr, wi;
      omega_pow(n, phase, &wr, &wi);
      double zr = yh[2 * hb] * wr - yh[2 * hb + 1] * wi;
      double zi = yh[2 * hb] * wi + yh[2 * hb + 1] * wr;
      e[2 * ((size_t)s * (size_t)p->L_est + (size_t)l)] = zr / gh;
      e[2 * ((size_t)s * (size_t)p->L_est + (size_t)l) + 1] = zi / gh;
    }
  }
  /* a truncated pass has no values to model: it counts as an infinite ratio */
  *ratio = want_res && (r->status & OR_TRUNCATED) ? HUGE_VAL : 0.0;
  if (!(r->status & OR_TRUNCATED)) {
    double *re = (double *)malloc(sizeof(double) * (size_t)p->L_est);
    double *im = (double *)malloc(sizeof(double) * (size_t)p->L_est);
    double *V = (double *)malloc(sizeof(double) * 2 * (size_t)(S > 0 ? S : 1));
    for (int64_t s = 0; s < S; s++) {
      for (int l = 0; l < p->L_est; l++) {
        re[l] = e[2 * ((size_t)s * (size_t)p->L_est + (size_t)l)];
        im[l] = e[2 * ((size_t)s * (size_t)p->L_est + (size_t)l) + 1];
      }
      V[2 * s] = or_median(re, p->L_est);
      V[2 * s + 1] = or_median(im, p->L_est);
      if (r->locs) r->locs[s] = Sl[s];
      if (r->vals) {
        r->vals[2 * s] = V[2 * s];
        r->vals[2 * s + 1] = V[2 * s + 1];
      }
      if (r->est)
        memcpy(r->est + 2 * (size_t)s * (size_t)p->L_est, e + 2 * (size_t)s * (size_t)p->L_est,
               sizeof(double) * 2 * (size_t)p->L_est);
    }
    if (want_res) {
      double er, et;
      or_residual(nd, n, B_star, w, G, or_residual_reach(p->alpha, p->delta), p->L_est, sig_est, tau_est,
                  yest, S, Sl, V, &er, &et);
      *ratio = et > 0.0 ? er / et : 0.0;
    }
    free(V);
    free(re);
    free(im);
  }
  free(yest);
  free(sig_est);
  free(tau_est);
  free(ghat);
  free(ghat_done);
  free(G);
  free(e);
  free(Sl);
  free(votes);
  free(sinv_loc);
  free(J);
  free(yh);
  free(m);
}

int or_atsfft(const or_params *p, const double *x, or_result *r) {
  int64_t n = p->n;
  int nd = p->ndim;
  if ((nd != 1 && nd != 2) || !is_pow2(n) || !is_pow2(p->B0) || !is_pow2(p->B_max) ||
      p->B0 > p->B_max || p->B_max > n || p->L_loc < 1 || p->L_loc > OR_TRACE_MAX_LOOPS ||
      p->L_est < 1 || p->L_est > OR_TRACE_MAX_LOOPS || (p->L_est % 2) == 0 || p->T_vote < 1 ||
      p->T_vote > p->L_loc || p->P_max < 1 || p->P_max > OR_TRACE_MAX_PROBE || p->d < 1 ||
      !(p->delta > 0.0 && p->delta < 1.0) || !(p->q > 0.0 && p->q < 1.0) ||
      (p->fixed_B > 0 && (!is_pow2(p->fixed_B) || p->fixed_B > n)) || p->res_tol < 0.0 ||
      p->res_retries < 0 || p->res_retries > 7)
    return -1;

  r->status = OR_OK;
  r->count = 0;
  r->n_probe = 0;
  r->res_ratio = 0.0;
  r->retries = 0;
  int64_t Bcap = p->fixed_B > 0 ? p->fixed_B : p->B_max;
  double *yh = (double *)malloc(sizeof(double) * 2 * (size_t)bcount(nd, Bcap));
  double *m = (double *)malloc(sizeof(double) * (size_t)bcount(nd, Bcap));
  int64_t sig[2], tau[2], sinv[2];

  /* ---- probe: the adaptive tuning iteration ---- */
  int64_t B_star = 0, khat = 0;
  if (p->fixed_B > 0) {
    B_star = p->fixed_B;
    khat = p->fixed_k;
  } else {
    or_probe_state ps;
    or_probe_init(p, &ps);
    while (!ps.done) {
      int64_t B = ps.B;
      int i = ps.iter;
      int64_t cnt = bcount(nd, B);
      hash_loop(p, x, OR_PHASE_PROBE, i, B, p->alpha_probe, yh, sig, tau, sinv);
      for (int64_t b = 0; b < cnt; b++) m[b] = yh[2 * b] * yh[2 * b] + yh[2 * b + 1] * yh[2 * b + 1];
      double T = or_threshold(m, cnt, p->q, p->noise_rate, p->rho);
      int64_t k = nd == 1 ? or_local_max_1d(m, B, T) : or_local_max_2d(m, B, T);
      r->probe_B[i] = B;
      r->probe_k[i] = k;
      r->probe_T[i] = T;
      r->probe_decision[i] = or_probe_step(p, &ps, k);
      r->n_probe = ps.iter;
    }
    B_star = ps.B_star;
    khat = ps.khat;
    r->status |= ps.status;
  }
  r->B_star = B_star;
  r->khat = khat;
  if (khat <= 0) {
    r->status |= OR_EMPTY; /* the probe's outcome, or fixed_k = 0 */
    free(yh);
    free(m);
    return 0;
  }

  /* ---- location, vote and estimation at B_star; with the residual test
     enabled, again at 2 B_star (fresh draws) while the residual is large ---- */
  free(yh);
  free(m);
  for (int pass = 0;; pass++) {
    double ratio = 0.0;
    main_phase(p, x, B_star, khat, pass, r, &ratio);
    r->res_ratio = ratio;
    r->retries = pass;
    int64_t Bcap = p->B_max;
    if (!(p->res_tol > 0.0) || !(ratio > p->res_tol) || pass >= p->res_retries || 2 * B_star > Bcap ||
        2 * B_star > n / 2)
      break;
    B_star *= 2;
    r->B_star = B_star;
    r->status |= OR_RETRIED;
  }
  return 0;
}

