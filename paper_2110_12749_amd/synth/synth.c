/*
 * Seeded synthetic filterbank generator.
 *
 * This module only makes test and benchmark inputs: it contains none of the
 * dedispersion or search arithmetic.  Both the CPU oracle and the GPU library
 * are fed from what it writes, so it shares code with neither.
 *
 * Model of one pixel (time row t, channel c), written as uint8:
 *     v = clip(rint(mean + std * n(t, c) + s(t, c)), 0, 255)
 * with rint rounding half to even, n a standard normal deviate and s the sum
 * of the injected signals:
 *   - dispersed pulses: a unit-peak Gaussian of the given FWHM, centred in
 *     channel c at t0 + 4148.808 s * DM * (f_c^-2 - f_max^-2) (f in MHz),
 *     averaged over each sample interval, times a per-channel peak amplitude;
 *   - narrowband RFI bursts: amp * (1 + sin(2 pi j / period + phase)) / 2 in
 *     one channel over a time interval;
 *   - broadband zero-DM spikes: +amp in every channel over a few rows.
 *
 * Noise: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by the
 * 64-bit seed, counter = (flat pixel index / 4, beam, 0); its four 32-bit
 * words become uniforms (w + 0.5) / 2^32 and two Box-Muller pairs give the
 * normals of four consecutive pixels.  Any block of rows of a beam therefore
 * regenerates independently and identically.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GSPS_K_DISP 4148.808 /* s MHz^2 cm^3 / pc */

typedef struct {
  double dm;     /* pc cm^-3 */
  double t0_s;   /* centre time at the highest frequency, s from row 0 */
  double fwhm_s; /* Gaussian FWHM, s */
  double amp;    /* per-channel peak amplitude, counts */
} gsps_pulse;

typedef struct {
  int32_t chan;
  int32_t pad_;
  double t_start_s, dur_s; /* active interval */
  double amp;              /* peak-to-peak amplitude, counts */
  double period_samp;      /* sinusoid period in samples */
  double phase;            /* radians */
} gsps_burst;

typedef struct {
  int64_t t_sample; /* first row */
  int32_t n_samp;   /* rows */
  int32_t pad_;
  double amp;       /* counts, added to every channel */
} gsps_spike;

static inline uint32_t mulhilo32(uint32_t a, uint32_t b, uint32_t *hi) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  return (uint32_t)p;
}

/* Philox4x32 with 10 rounds, as published (Random123). */
void gsps_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0, hi1;
    uint32_t lo0 = mulhilo32(0xD2511F53u, c0, &hi0);
    uint32_t lo1 = mulhilo32(0xCD9E8D57u, c2, &hi1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Four standard normals for pixel group g (flat pixels 4g .. 4g+3). */
static inline void normals4(uint64_t seed, uint32_t beam, uint64_t g, double n[4]) {
  uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), beam, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  gsps_philox4x32_10(ctr, key, w);
  const double two32inv = 1.0 / 4294967296.0;
  const double twopi = 6.283185307179586476925;
  for (int k = 0; k < 4; k += 2) {
    double u1 = ((double)w[k] + 0.5) * two32inv;
    double u2 = ((double)w[k + 1] + 0.5) * two32inv;
    double r = sqrt(-2.0 * log(u1));
    double a = twopi * u2;
    n[k] = r * cos(a);
    n[k + 1] = r * sin(a);
  }
}

/* Normal deviate of one flat pixel (used by tests of the noise model). */
double gsps_normal(uint64_t seed, uint32_t beam, uint64_t flat_index) {
  double n[4];
  normals4(seed, beam, flat_index >> 2, n);
  return n[flat_index & 3];
}

static inline uint8_t quantise(double v) {
  double r = rint(v); /* default rounding mode: half to even */
  if (r < 0.0) r = 0.0;
  if (r > 255.0) r = 255.0;
  return (uint8_t)r;
}

#define ROWS_PER_BLOCK 64

/* Rows [t_begin, t_begin + nrows) of a beam, time-major uint8 [nrows][nchan]. */
int gsps_filterbank(uint8_t *out, int64_t t_begin, int64_t nrows, int32_t nchan,
                    const double *freqs_mhz, double tsamp_s, uint64_t seed, uint32_t beam,
                    double mean, double std, const gsps_pulse *pulses, int32_t n_pulses,
                    const gsps_burst *bursts, int32_t n_bursts, const gsps_spike *spikes,
                    int32_t n_spikes) {
  if (!out || nrows < 0 || nchan < 1 || !freqs_mhz || !(tsamp_s > 0)) return -1;
  double fmax = freqs_mhz[0];
  for (int32_t c = 1; c < nchan; ++c)
    if (freqs_mhz[c] > fmax) fmax = freqs_mhz[c];

  /* Per pulse and channel: centre time in samples, Gaussian sigma in samples. */
  double *tc = NULL;
  double *p_lo = NULL, *p_hi = NULL; /* overall sample range of each pulse */
  if (n_pulses > 0) {
    tc = (double *)malloc(sizeof(double) * (size_t)n_pulses * (size_t)nchan);
    p_lo = (double *)malloc(sizeof(double) * (size_t)n_pulses);
    p_hi = (double *)malloc(sizeof(double) * (size_t)n_pulses);
    if (!tc || !p_lo || !p_hi) {
      free(tc);
      free(p_lo);
      free(p_hi);
      return -2;
    }
    for (int32_t p = 0; p < n_pulses; ++p) {
      double sig = pulses[p].fwhm_s / (2.0 * sqrt(2.0 * log(2.0))) / tsamp_s;
      double lo = 1e300, hi = -1e300;
      for (int32_t c = 0; c < nchan; ++c) {
        double f = freqs_mhz[c];
        double delay_s = GSPS_K_DISP * pulses[p].dm * (1.0 / (f * f) - 1.0 / (fmax * fmax));
        double t = (pulses[p].t0_s + delay_s) / tsamp_s;
        tc[(size_t)p * nchan + c] = t;
        if (t < lo) lo = t;
        if (t > hi) hi = t;
      }
      p_lo[p] = lo - 8.0 * sig - 2.0;
      p_hi[p] = hi + 8.0 * sig + 2.0;
    }
  }

  int64_t n_blocks = (nrows + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
  int fail = 0;
#pragma omp parallel
  {
    float *sig = (float *)malloc(sizeof(float) * (size_t)ROWS_PER_BLOCK * (size_t)nchan);
    if (!sig) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t b = 0; b < n_blocks; ++b) {
      if (!sig) continue;
      int64_t r0 = b * ROWS_PER_BLOCK;
      int64_t r1 = r0 + ROWS_PER_BLOCK < nrows ? r0 + ROWS_PER_BLOCK : nrows;
      int64_t ta = t_begin + r0, tb = t_begin + r1; /* absolute rows */
      int any = 0;
      /* pulses */
      for (int32_t p = 0; p < n_pulses; ++p) {
        if (p_hi[p] < (double)ta || p_lo[p] > (double)tb) continue;
        double sig_s = pulses[p].fwhm_s / (2.0 * sqrt(2.0 * log(2.0))) / tsamp_s;
        double span = 8.0 * sig_s + 2.0;
        double scale = pulses[p].amp * sig_s * sqrt(2.0 * M_PI) * 0.5;
        double inv = 1.0 / (sig_s * sqrt(2.0));
        for (int32_t c = 0; c < nchan; ++c) {
          double t = tc[(size_t)p * nchan + c];
          if (t + span < (double)ta || t - span > (double)tb) continue;
          int64_t j0 = (int64_t)floor(t - span), j1 = (int64_t)ceil(t + span);
          if (j0 < ta) j0 = ta;
          if (j1 > tb - 1) j1 = tb - 1;
          for (int64_t j = j0; j <= j1; ++j) {
            /* mean of the unit-peak Gaussian over [j, j+1) in samples */
            double v = scale * (erf(((double)j + 1.0 - t) * inv) - erf(((double)j - t) * inv));
            if (!any) {
              memset(sig, 0, sizeof(float) * (size_t)ROWS_PER_BLOCK * (size_t)nchan);
              any = 1;
            }
            sig[(size_t)(j - ta) * nchan + c] += (float)v;
          }
        }
      }
      /* narrowband bursts */
      for (int32_t k = 0; k < n_bursts; ++k) {
        int32_t c = bursts[k].chan;
        if (c < 0 || c >= nchan) continue;
        int64_t j0 = (int64_t)ceil(bursts[k].t_start_s / tsamp_s);
        int64_t j1 = (int64_t)ceil((bursts[k].t_start_s + bursts[k].dur_s) / tsamp_s);
        if (j0 < ta) j0 = ta;
        if (j1 > tb) j1 = tb;
        for (int64_t j = j0; j < j1; ++j) {
          double v = bursts[k].amp * 0.5 *
                     (1.0 + sin(2.0 * M_PI * (double)j / bursts[k].period_samp + bursts[k].phase));
          if (!any) {
            memset(sig, 0, sizeof(float) * (size_t)ROWS_PER_BLOCK * (size_t)nchan);
            any = 1;
          }
          sig[(size_t)(j - ta) * nchan + c] += (float)v;
        }
      }
      /* broadband spikes */
      for (int32_t k = 0; k < n_spikes; ++k) {
        int64_t j0 = spikes[k].t_sample, j1 = spikes[k].t_sample + spikes[k].n_samp;
        if (j0 < ta) j0 = ta;
        if (j1 > tb) j1 = tb;
        for (int64_t j = j0; j < j1; ++j) {
          if (!any) {
            memset(sig, 0, sizeof(float) * (size_t)ROWS_PER_BLOCK * (size_t)nchan);
            any = 1;
          }
          for (int32_t c = 0; c < nchan; ++c) sig[(size_t)(j - ta) * nchan + c] += (float)spikes[k].amp;
        }
      }
      /* noise + quantisation over the flat pixel range of this block */
      uint64_t q0 = (uint64_t)ta * (uint64_t)nchan, q1 = (uint64_t)tb * (uint64_t)nchan;
      uint8_t *dst = out + (size_t)r0 * (size_t)nchan;
      double n4[4];
      for (uint64_t g = q0 >> 2; (g << 2) < q1; ++g) {
        normals4(seed, beam, g, n4);
        for (int k = 0; k < 4; ++k) {
          uint64_t q = (g << 2) + (uint64_t)k;
          if (q < q0 || q >= q1) continue;
          double v = mean + std * n4[k];
          if (any) v += (double)sig[q - q0];
          dst[q - q0] = quantise(v);
        }
      }
    }
    free(sig);
  }
  free(tc);
  free(p_lo);
  free(p_hi);
  return fail ? -2 : 0;
}
