/*
 * CPU oracle for brute-force incoherent dedispersion and the boxcar
 * single-pulse search.  TEST INFRASTRUCTURE ONLY: nothing in the library
 * links, includes or calls this file; only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark do.
 *
 * It is deliberately plain: loops written straight from the definitions,
 * no blocking, no vectorisation, no shared code with the GPU library.
 *
 * Paper: You et al., "A GPU single-pulse search pipeline ..." (arXiv
 * 2110.12749).  The method is the shift-and-sum of Section 2.3 (Algorithms 2
 * and 3: each dedispersed sample of a DM trial is the sum over channels of the
 * channel's sample at the time shifted by that channel's delay), applied per
 * DM trial of a DDplan-style plan (Section 2.1, Tables 2 and 3: rows of
 * low DM, DM step, number of DMs and time downsampling).  The paper prints no
 * dispersion law, no rounding rule and no single-pulse statistic; the
 * readings taken are:
 *   delay   d = floor(r + 0.5),  r = ((K * dm) * (1/f^2 - 1/fref^2)) / (tsamp * D)
 *           K = 4148.808 s MHz^2 cm^3/pc, f in MHz, fref = highest channel,
 *           evaluated in IEEE double in this order with no FMA contraction;
 *   downsampling = integer sum of D consecutive samples per channel, the
 *           remainder dropped;
 *   valid length n_out = floor(nsamp / D) - max delay over the segment;
 *   statistics = population mean and sigma from exact integer moments about
 *           the first sample;
 *   boxcar  snr(e, w) = (sum_{k=e-w+1..e} x_k - w mu) / (sigma sqrt(w)),
 *           boxes end-aligned at e, best over widths (ties -> smaller w),
 *           one candidate per maximal run of best >= threshold at the run's
 *           argmax (ties -> earlier e).
 * Parity of the delay table, the downsampled sums, the dedispersed sums, the
 * statistics and the search is pinned by the CPU tests (exact rationals,
 * brute force, closed forms, conservation, injected-pulse recovery).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_K_DISP 4148.808

/* Threads an OpenMP loop of the oracle uses (reported with CPU timings). */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Threads for later OpenMP loops (timings on fewer cores). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

typedef struct {
  double dm_lo;
  double dm_step;
  int32_t n_dm;
  int32_t downsamp;
} orc_seg;

typedef struct {
  int32_t trial;   /* DM index within the segment */
  int32_t width;   /* boxcar width of the peak, samples */
  int64_t t_peak;  /* first sample of the peak box */
  int64_t t_first; /* first box end of the run */
  int64_t t_last;  /* last box end of the run */
  double snr;
} orc_cand;

/* Highest channel frequency: the reference frequency of every delay. */
double orc_fref(const double *freqs, int32_t nchan) {
  double f = freqs[0];
  for (int32_t c = 1; c < nchan; ++c)
    if (freqs[c] > f) f = freqs[c];
  return f;
}

/* Trial DM of index i of a plan row: lo + i * step (half-open grid). */
double orc_trial_dm(orc_seg s, int32_t i) { return s.dm_lo + (double)i * s.dm_step; }

/* Delay of one channel for one trial, in samples of tsamp * D. */
int64_t orc_delay(double dm, double f, double fref, double tsamp, int32_t D) {
  double r = ((ORC_K_DISP * dm) * (1.0 / (f * f) - 1.0 / (fref * fref))) / (tsamp * (double)D);
  return (int64_t)floor(r + 0.5);
}

/* Delay table of one segment: int64 [n_dm][nchan]. */
void orc_delay_table(const double *freqs, int32_t nchan, double tsamp, orc_seg s, int64_t *d) {
  double fref = orc_fref(freqs, nchan);
  for (int32_t i = 0; i < s.n_dm; ++i)
    for (int32_t c = 0; c < nchan; ++c)
      d[(int64_t)i * nchan + c] = orc_delay(orc_trial_dm(s, i), freqs[c], fref, tsamp, s.downsamp);
}

/* Per segment: max delay and valid output length (<= 0 means too short). */
void orc_plan_shape(int64_t nsamp, const double *freqs, int32_t nchan, double tsamp,
                    const orc_seg *segs, int32_t n_seg, int64_t *max_delay, int64_t *n_out) {
  double fref = orc_fref(freqs, nchan);
  for (int32_t s = 0; s < n_seg; ++s) {
    int64_t m = 0;
    for (int32_t i = 0; i < segs[s].n_dm; ++i)
      for (int32_t c = 0; c < nchan; ++c) {
        int64_t d = orc_delay(orc_trial_dm(segs[s], i), freqs[c], fref, tsamp, segs[s].downsamp);
        if (d > m) m = d;
      }
    max_delay[s] = m;
    n_out[s] = nsamp / segs[s].downsamp - m;
  }
}

/* Y[c][j] = sum_{k<D} X[j*D + k][c]; X time-major uint8 [nsamp][nchan]. */
void orc_downsample(const uint8_t *X, int64_t nsamp, int32_t nchan, int32_t D, uint32_t *Y) {
  int64_t N = nsamp / D;
  for (int32_t c = 0; c < nchan; ++c)
    for (int64_t j = 0; j < N; ++j) {
      uint32_t acc = 0;
      for (int32_t k = 0; k < D; ++k) acc += X[(j * D + k) * nchan + c];
      Y[(int64_t)c * N + j] = acc;
    }
}

/*
 * Whole segment: out[i][t] = sum_c Y[c][t + d[i][c]], t in [0, n_out), with
 * Y[c][j] = sum_{m<D} X[j*D + m][c] evaluated on the fly from the raw
 * filterbank (no intermediate array).  Trials [i0, i1) only (the full
 * segment when i0 = 0, i1 = n_dm); rows of `out` are indexed by i - i0.
 * OpenMP over the (trial, sample) pairs, nothing else.
 */
int orc_dedisperse_segment(const uint8_t *X, int64_t nsamp, int32_t nchan, const double *freqs,
                           double tsamp, orc_seg s, int32_t i0, int32_t i1, int64_t n_out,
                           int32_t *out) {
  (void)nsamp;
  int32_t nt = i1 - i0;
  int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1) * (size_t)nchan);
  if (!d) return -1;
  double fref = orc_fref(freqs, nchan);
  for (int32_t i = i0; i < i1; ++i)
    for (int32_t c = 0; c < nchan; ++c)
      d[(int64_t)(i - i0) * nchan + c] = orc_delay(orc_trial_dm(s, i), freqs[c], fref, tsamp, s.downsamp);
  const int64_t D = s.downsamp;
#pragma omp parallel for collapse(2) schedule(static)
  for (int32_t i = 0; i < nt; ++i)
    for (int64_t t = 0; t < n_out; ++t) {
      int64_t acc = 0;
      for (int32_t c = 0; c < nchan; ++c) {
        int64_t j = t + d[(int64_t)i * nchan + c];
        for (int64_t m = 0; m < D; ++m) acc += X[(j * D + m) * nchan + c];
      }
      out[(int64_t)i * n_out + t] = (int32_t)acc;
    }
  free(d);
  return 0;
}

/*
 * Individual outputs straight from the raw filterbank, no intermediate
 * arrays: value[k] = sum_c sum_{m<D} X[(t_k + d(i_k, c)) * D + m][c].
 */
void orc_dedisperse_points(const uint8_t *X, int64_t nsamp, int32_t nchan, const double *freqs,
                           double tsamp, orc_seg s, const int32_t *trial, const int64_t *t,
                           int64_t npts, int64_t *value) {
  double fref = orc_fref(freqs, nchan);
  (void)nsamp;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npts; ++k) {
    double dm = orc_trial_dm(s, trial[k]);
    int64_t acc = 0;
    for (int32_t c = 0; c < nchan; ++c) {
      int64_t d = orc_delay(dm, freqs[c], fref, tsamp, s.downsamp);
      for (int32_t m = 0; m < s.downsamp; ++m) acc += X[((t[k] + d) * s.downsamp + m) * nchan + c];
    }
    value[k] = acc;
  }
}

/*
 * Population mean and sigma of x[0..n), from exact moments about x0 = x[0]:
 * S1 = sum (x - x0), S2 = sum (x - x0)^2 in 128-bit integers, then
 * mu = x0 + S1/n and sigma = sqrt(S2/n - (S1/n)^2) in double.
 */
void orc_stats(const int32_t *x, int64_t n, double *mu, double *sigma) {
  __int128 s1 = 0, s2 = 0;
  int64_t x0 = x[0];
  for (int64_t k = 0; k < n; ++k) {
    __int128 v = (__int128)((int64_t)x[k] - x0);
    s1 += v;
    s2 += v * v;
  }
  double m1 = (double)s1 / (double)n;
  double m2 = (double)s2 / (double)n;
  double var = m2 - m1 * m1;
  *mu = (double)x0 + m1;
  *sigma = var > 0.0 ? sqrt(var) : 0.0;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Boxcar search of the box ends e in [e0, e1) of series x[0..n), with the
 * statistics mu, sigma given.  Boxes may start anywhere >= 0 (they reach back
 * before e0 when e0 > 0).  Candidates are appended to out (capacity cap);
 * returns the number found (may exceed cap; only cap are written).
 */
int64_t orc_search_range(const int32_t *x, int64_t n, int64_t e0, int64_t e1, double mu, double sigma,
                         const int32_t *widths_in, int32_t nw, float threshold, int32_t trial,
                         orc_cand *out, int64_t cap) {
  if (e0 < 0) e0 = 0;
  if (e1 > n) e1 = n;
  if (!(sigma > 0.0) || e1 <= e0 || nw <= 0) return 0;
  /* widths as a sorted set */
  int32_t *w = (int32_t *)malloc(sizeof(int32_t) * (size_t)nw);
  memcpy(w, widths_in, sizeof(int32_t) * (size_t)nw);
  qsort(w, (size_t)nw, sizeof(int32_t), cmp_i32);
  int32_t nu = 0;
  for (int32_t k = 0; k < nw; ++k)
    if (nu == 0 || w[k] != w[nu - 1]) w[nu++] = w[k];
  /* prefix sums P[k] = x[0] + ... + x[k-1] */
  int64_t *P = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  P[0] = 0;
  for (int64_t k = 0; k < n; ++k) P[k + 1] = P[k] + (int64_t)x[k];
  double thr = (double)threshold;
  int64_t found = 0;
  int in_run = 0;
  int64_t run_first = 0, best_e = 0;
  int32_t best_w = 0;
  double best_snr = 0.0;
  for (int64_t e = e0; e <= e1; ++e) {
    int flagged = 0;
    double b = 0.0;
    int32_t bw = 0;
    if (e < e1) {
      for (int32_t k = 0; k < nu; ++k) {
        int64_t wk = w[k];
        if (wk > e + 1) break; /* box would start before sample 0 */
        double s = (double)(P[e + 1] - P[e + 1 - wk]);
        double snr = (s - (double)wk * mu) / (sigma * sqrt((double)wk));
        if (bw == 0 || snr > b) {
          b = snr;
          bw = (int32_t)wk;
        }
      }
      flagged = bw != 0 && b >= thr;
    }
    if (flagged) {
      if (!in_run) {
        in_run = 1;
        run_first = e;
        best_e = e;
        best_w = bw;
        best_snr = b;
      } else if (b > best_snr) {
        best_e = e;
        best_w = bw;
        best_snr = b;
      }
    } else if (in_run) {
      if (found < cap) {
        orc_cand *c = &out[found];
        c->trial = trial;
        c->width = best_w;
        c->t_peak = best_e - best_w + 1;
        c->t_first = run_first;
        c->t_last = e - 1;
        c->snr = best_snr;
      }
      ++found;
      in_run = 0;
    }
  }
  free(P);
  free(w);
  return found;
}

/* Whole-series search: statistics over all n samples, every box end. */
int64_t orc_search_series(const int32_t *x, int64_t n, const int32_t *widths, int32_t nw,
                          float threshold, int32_t trial, orc_cand *out, int64_t cap) {
  double mu, sigma;
  if (n <= 0) return 0;
  orc_stats(x, n, &mu, &sigma);
  return orc_search_range(x, n, 0, n, mu, sigma, widths, nw, threshold, trial, out, cap);
}

/*
 * Streaming window search: statistics over the window's own samples
 * x[w0..w1) and boxes ending in it, which may reach back before w0.
 */
int64_t orc_search_window(const int32_t *x, int64_t n, int64_t w0, int64_t w1, const int32_t *widths,
                          int32_t nw, float threshold, int32_t trial, orc_cand *out, int64_t cap) {
  double mu, sigma;
  if (w0 < 0) w0 = 0;
  if (w1 > n) w1 = n;
  if (w1 <= w0) return 0;
  orc_stats(x + w0, w1 - w0, &mu, &sigma);
  return orc_search_range(x, n, w0, w1, mu, sigma, widths, nw, threshold, trial, out, cap);
}

/*
 * Sub-band (two-stage) dedispersion, the algorithm the paper's pipeline uses
 * (Section 2.3 names it and cites Barsdell et al. 2012 for it; PRESTO's
 * prepsubband works this way).  The channels are split into n_sub
 * contiguous sub-bands, band b = channels [b*nchan/n_sub, (b+1)*nchan/n_sub),
 * with reference frequency f_b = the band's highest channel frequency.  The
 * row's trials are split into groups of `group` consecutive trials, group g
 * = trials [g*group, min((g+1)*group, n_dm)), each with a nominal DM at its
 * centre: DM_g = dm_lo + (g*group + (n_g - 1)/2) * dm_step, n_g its size.
 *   stage 1: Z[g][b][t] = sum over channels c of band b of
 *            Y[c][t + d1(g, c)],  d1(g, c) = delay of DM_g at f_c against f_b;
 *   stage 2: out[i][t] = sum over bands b of Z[g(i)][b][t + d2(i, b)],
 *            d2(i, b) = delay of DM_i at f_b against fref.
 * Both delays use the rounding rule of orc_delay with the reference
 * frequency replaced.  The valid length is n_out = floor(nsamp/D) - the
 * largest d2(i, b) + max_{c in b} d1(g(i), c) over the row.  Composite
 * delays differ from the brute-force ones by the in-band smearing of
 * |DM_i - DM_g| plus at most one sample of double rounding.
 */
int64_t orc_delay_ref(double dm, double f, double fb, double tsamp, int32_t D) {
  double r = ((ORC_K_DISP * dm) * (1.0 / (f * f) - 1.0 / (fb * fb))) / (tsamp * (double)D);
  return (int64_t)floor(r + 0.5);
}

/* Highest frequency of the channels of band b. */
static double orc_band_ref(const double *freqs, int32_t nchan, int32_t n_sub, int32_t b) {
  int32_t c0 = (int32_t)((int64_t)b * nchan / n_sub), c1 = (int32_t)((int64_t)(b + 1) * nchan / n_sub);
  double f = freqs[c0];
  for (int32_t c = c0 + 1; c < c1; ++c)
    if (freqs[c] > f) f = freqs[c];
  return f;
}

/* Nominal DM of group g of a row. */
double orc_group_dm(orc_seg s, int32_t group, int32_t g) {
  int32_t first = g * group;
  int32_t n_g = s.n_dm - first < group ? s.n_dm - first : group;
  return s.dm_lo + ((double)first + (double)(n_g - 1) / 2.0) * s.dm_step;
}

/* Composite delay table int64 [n_dm][nchan]: d2(i, b(c)) + d1(g(i), c),
 * and the row's valid length through *n_out. */
void orc_subband_delays(const double *freqs, int32_t nchan, int64_t nsamp, double tsamp, orc_seg s, int32_t n_sub,
                        int32_t group, int64_t *d, int64_t *n_out) {
  double fref = orc_fref(freqs, nchan);
  int64_t m = 0;
  for (int32_t i = 0; i < s.n_dm; ++i) {
    double dm = orc_trial_dm(s, i), dmg = orc_group_dm(s, group, i / group);
    for (int32_t b = 0; b < n_sub; ++b) {
      double fb = orc_band_ref(freqs, nchan, n_sub, b);
      int64_t d2 = orc_delay_ref(dm, fb, fref, tsamp, s.downsamp);
      int32_t c0 = (int32_t)((int64_t)b * nchan / n_sub), c1 = (int32_t)((int64_t)(b + 1) * nchan / n_sub);
      int64_t m1 = 0;
      for (int32_t c = c0; c < c1; ++c) {
        int64_t d1 = orc_delay_ref(dmg, freqs[c], fb, tsamp, s.downsamp);
        d[(int64_t)i * nchan + c] = d2 + d1;
        if (d1 > m1) m1 = d1;
      }
      if (d2 + m1 > m) m = d2 + m1;
    }
  }
  *n_out = nsamp / s.downsamp - m;
}

/*
 * The two stages as written above, trials [i0, i1) of a row: stage 1 forms
 * the sub-band series of every group the trials need over the samples
 * stage 2 reads, stage 2 sums them.  out int32 [i1 - i0][n_out].
 */
int orc_dedisperse_subband(const uint8_t *X, int64_t nsamp, int32_t nchan, const double *freqs, double tsamp,
                           orc_seg s, int32_t n_sub, int32_t group, int32_t i0, int32_t i1, int64_t n_out,
                           int32_t *out) {
  const int64_t D = s.downsamp, N = nsamp / s.downsamp;
  double fref = orc_fref(freqs, nchan);
  int32_t g0 = i0 / group, g1 = (i1 - 1) / group + 1;
  int64_t *d1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)nchan);
  int64_t *d2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_sub);
  int64_t *Z = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_sub * (size_t)N);
  if (!d1 || !d2 || !Z) {
    free(d1);
    free(d2);
    free(Z);
    return -1;
  }
  for (int32_t g = g0; g < g1; ++g) {
    /* stage 1 for group g: every band, every sample whose channels all exist */
    double dmg = orc_group_dm(s, group, g);
    for (int32_t b = 0; b < n_sub; ++b) {
      double fb = orc_band_ref(freqs, nchan, n_sub, b);
      int32_t c0 = (int32_t)((int64_t)b * nchan / n_sub), c1 = (int32_t)((int64_t)(b + 1) * nchan / n_sub);
      int64_t m1 = 0;
      for (int32_t c = c0; c < c1; ++c) {
        d1[c] = orc_delay_ref(dmg, freqs[c], fb, tsamp, s.downsamp);
        if (d1[c] > m1) m1 = d1[c];
      }
#pragma omp parallel for schedule(static)
      for (int64_t t = 0; t < N - m1; ++t) {
        int64_t acc = 0;
        for (int32_t c = c0; c < c1; ++c) {
          int64_t j = t + d1[c];
          for (int64_t k = 0; k < D; ++k) acc += X[(j * D + k) * nchan + c];
        }
        Z[(int64_t)b * N + t] = acc;
      }
    }
    /* stage 2 for the group's trials in [i0, i1) */
    int32_t ia = g * group > i0 ? g * group : i0;
    int32_t ib = (g + 1) * group < i1 ? (g + 1) * group : i1;
    for (int32_t i = ia; i < ib; ++i) {
      double dm = orc_trial_dm(s, i);
      for (int32_t b = 0; b < n_sub; ++b)
        d2[b] = orc_delay_ref(dm, orc_band_ref(freqs, nchan, n_sub, b), fref, tsamp, s.downsamp);
#pragma omp parallel for schedule(static)
      for (int64_t t = 0; t < n_out; ++t) {
        int64_t acc = 0;
        for (int32_t b = 0; b < n_sub; ++b) acc += Z[(int64_t)b * N + t + d2[b]];
        out[(int64_t)(i - i0) * n_out + t] = (int32_t)acc;
      }
    }
  }
  free(d1);
  free(d2);
  free(Z);
  return 0;
}

/*
 * RFI mitigation of a filterbank, in integers throughout (Section 2.1 lists
 * RFI mitigation among the search steps; Section 3.1 reports PRESTO's
 * 'clip' option giving the same results on CPU and GPU).  The paper does not
 * define either operation; the readings taken:
 *   clip (clip_sigma > 0): spectra in blocks of `block` (the last block may
 *     be shorter).  Per block the zero-DM series s_j = sum_c x[j][c] has
 *     population mean mu and sigma from exact integer moments about its
 *     first value (as orc_stats); spectrum j is flagged when
 *     |s_j - mu| > clip_sigma * sigma, in double.  Flagged spectra are
 *     replaced by the block's channel means over its unflagged spectra,
 *     m_c = floor((2 S_c + n_u) / (2 n_u)) (S_c the channel's sum, n_u the
 *     unflagged count: a mean rounded half up); with n_u = 0 or sigma = 0
 *     nothing is replaced.
 *   zero-DM filter (zero_dm != 0), after clipping: each spectrum's rounded
 *     mean z_j = floor((2 s'_j + nchan) / (2 nchan)) is subtracted and 128
 *     added back, clamped to 0..255: x'[j][c] = clamp(x[j][c] - z_j + 128).
 * Returns the number of flagged spectra.
 */
int64_t orc_rfi_clean(const uint8_t *X, int64_t nsamp, int32_t nchan, double clip_sigma, int64_t block,
                      int32_t zero_dm, uint8_t *out) {
  int64_t flagged_total = 0;
  memcpy(out, X, (size_t)nsamp * (size_t)nchan);
  if (clip_sigma > 0.0 && block > 0) {
    int64_t *sj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(block > 0 ? block : 1));
    uint8_t *flag = (uint8_t *)malloc((size_t)block);
    int64_t *sc = (int64_t *)malloc(sizeof(int64_t) * (size_t)nchan);
    for (int64_t j0 = 0; j0 < nsamp; j0 += block) {
      int64_t n = nsamp - j0 < block ? nsamp - j0 : block;
      for (int64_t j = 0; j < n; ++j) {
        int64_t a = 0;
        for (int32_t c = 0; c < nchan; ++c) a += X[(j0 + j) * nchan + c];
        sj[j] = a;
      }
      __int128 s1 = 0, s2 = 0;
      for (int64_t j = 0; j < n; ++j) {
        __int128 v = (__int128)(sj[j] - sj[0]);
        s1 += v;
        s2 += v * v;
      }
      double m1 = (double)s1 / (double)n, m2 = (double)s2 / (double)n;
      double var = m2 - m1 * m1;
      double mu = (double)sj[0] + m1, sigma = var > 0.0 ? sqrt(var) : 0.0;
      int64_t n_u = 0;
      for (int64_t j = 0; j < n; ++j) {
        flag[j] = sigma > 0.0 && fabs((double)sj[j] - mu) > clip_sigma * sigma;
        n_u += !flag[j];
      }
      if (n_u == 0 || n_u == n) continue;
      for (int32_t c = 0; c < nchan; ++c) sc[c] = 0;
      for (int64_t j = 0; j < n; ++j)
        if (!flag[j])
          for (int32_t c = 0; c < nchan; ++c) sc[c] += X[(j0 + j) * nchan + c];
      for (int64_t j = 0; j < n; ++j)
        if (flag[j]) {
          for (int32_t c = 0; c < nchan; ++c) out[(j0 + j) * nchan + c] = (uint8_t)((2 * sc[c] + n_u) / (2 * n_u));
          ++flagged_total;
        }
    }
    free(sj);
    free(flag);
    free(sc);
  }
  if (zero_dm) {
    for (int64_t j = 0; j < nsamp; ++j) {
      int64_t a = 0;
      for (int32_t c = 0; c < nchan; ++c) a += out[j * nchan + c];
      int64_t z = (2 * a + nchan) / (2 * (int64_t)nchan);
      for (int32_t c = 0; c < nchan; ++c) {
        int64_t v = (int64_t)out[j * nchan + c] - z + 128;
        out[j * nchan + c] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
      }
    }
  }
  return flagged_total;
}

/*
 * Friends-of-friends grouping of candidates of one segment.  Two candidates
 * are linked when their trial indices differ by at most one and their run
 * extents [t_first, t_last] overlap.  group[k] receives, for candidate k, the
 * index of its group's representative: the member of highest snr (ties ->
 * lower trial, then earlier t_peak).  Quadratic on purpose.
 */
void orc_group(const orc_cand *c, int64_t n, int64_t *group) {
  int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t k = 0; k < n; ++k) parent[k] = k;
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = a + 1; b < n; ++b) {
      int64_t dt = (int64_t)c[a].trial - (int64_t)c[b].trial;
      if (dt < -1 || dt > 1) continue;
      if (c[a].t_last < c[b].t_first || c[b].t_last < c[a].t_first) continue;
      int64_t ra = a, rb = b;
      while (parent[ra] != ra) ra = parent[ra];
      while (parent[rb] != rb) rb = parent[rb];
      if (ra != rb) parent[ra > rb ? ra : rb] = ra < rb ? ra : rb;
    }
  /* representative = best member of each root's set */
  int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t k = 0; k < n; ++k) best[k] = -1;
  for (int64_t k = 0; k < n; ++k) {
    int64_t r = k;
    while (parent[r] != r) r = parent[r];
    int64_t b = best[r];
    int better = b < 0 || c[k].snr > c[b].snr ||
                 (c[k].snr == c[b].snr &&
                  (c[k].trial < c[b].trial || (c[k].trial == c[b].trial && c[k].t_peak < c[b].t_peak)));
    if (better) best[r] = k;
  }
  for (int64_t k = 0; k < n; ++k) {
    int64_t r = k;
    while (parent[r] != r) r = parent[r];
    group[k] = best[r];
  }
  free(best);
  free(parent);
}
