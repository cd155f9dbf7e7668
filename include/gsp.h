/*
 * gsp.h -- C ABI of the MI355X (gfx950) dedispersion + single-pulse-search
 * library.
 *
 * The operations follow You et al., "A GPU single-pulse search pipeline and
 * candidate archiving database" (arXiv 2110.12749):
 *   - dedispersion is the shift-and-sum of Section 2.3 (Algorithms 2 and 3):
 *     every output sample of a DM trial is the sum over frequency channels of
 *     that channel's sample shifted by a per-(trial, channel) delay, the delays
 *     forming a [numdm][numchan] table;
 *   - trials come from a DDplan-style plan (Section 2.1, Tables 2 and 3): rows
 *     of (low DM, DM step, number of DMs, time downsampling);
 *   - the single-pulse search (named in Section 2.1, not specified there) is a
 *     boxcar matched filter over each dedispersed series.
 * The readings the paper leaves open, fixed here:
 *   delay  d = floor(r + 0.5) with r = ((K*dm) * (1/f^2 - 1/fref^2)) / (tsamp*D),
 *          K = 4148.808 s MHz^2 cm^3 / pc, f in MHz, fref = highest channel,
 *          in IEEE double, in that order, without FMA contraction;
 *   DM of trial i of a row = dm_lo + i * dm_step, i in [0, n_dm);
 *   downsampling by D = integer sum of D consecutive samples per channel
 *          (a trailing remainder is dropped);
 *   valid output length of a row n_out = floor(nsamp / D) - max delay;
 *   output = exact int32 sums (no mean subtraction).
 *
 * Conventions.  Every function returns a status: GSP_OK (0) or a negative
 * GSP_E* code; nothing aborts and no C++ exception crosses this boundary.
 * "device" pointers are HIP device memory on the context's device; "host"
 * pointers are ordinary host memory.  The caller owns every buffer it passes;
 * the library owns only its handle objects and their internal scratch.
 * `stream` arguments are hipStream_t values passed as void* (NULL = the null
 * stream).  A context is used by one host thread at a time.
 */
#ifndef GSP_H
#define GSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GSP_OK = 0,
  GSP_EINVAL = -1,     /* invalid argument */
  GSP_ETOOSHORT = -2,  /* input shorter than a plan row's maximum delay */
  GSP_EOVERFLOW = -3,  /* sums could overflow the int32 output or internal lanes */
  GSP_ECAPACITY = -4,  /* output buffer too small (required size reported) */
  GSP_ENOMEM = -5,     /* device or host allocation failed */
  GSP_EDEVICE = -6,    /* HIP runtime error */
  GSP_EAGAIN = -7      /* streaming: not admitted now, retry later */
};

#define GSP_MAX_SEG 16

typedef struct gsp_ctx gsp_ctx;

/* One context per host thread on `device`.  Owns delay tables, staging and
 * search scratch, and the tuned launch shapes. */
int gsp_create(int device, gsp_ctx **out);
void gsp_destroy(gsp_ctx *ctx);
/* Static text of a status code. */
const char *gsp_strerror(int status);
/* Message of the last failure on this context ("" if none).  Owned by ctx. */
const char *gsp_last_error(const gsp_ctx *ctx);

/* One plan row (Section 2.1, Tables 2-3). */
typedef struct gsp_segment {
  double dm_lo;     /* first trial DM, pc cm^-3, >= 0 */
  double dm_step;   /* > 0 */
  int32_t n_dm;     /* >= 1 */
  int32_t downsamp; /* D, 1 <= D <= 257 */
} gsp_segment;

/* Shape of a DM-time output: the per-row arrays are concatenated row by row,
 * each row-block being int32 [n_dm][n_out] (trial-major, time contiguous). */
typedef struct gsp_dmt_desc {
  int64_t nsamp;   /* input samples (time rows) */
  int32_t nchan;   /* channels */
  int32_t n_seg;   /* plan rows */
  double tsamp;    /* s */
  double fref_mhz; /* highest channel frequency */
  gsp_segment seg[GSP_MAX_SEG];
  int64_t max_delay[GSP_MAX_SEG]; /* largest delay of the row, samples of D*tsamp */
  int64_t n_out[GSP_MAX_SEG];     /* valid outputs per trial of the row */
  int64_t offset[GSP_MAX_SEG];    /* element offset of the row's block */
  int32_t trial0[GSP_MAX_SEG];    /* global index of the row's first trial */
  int32_t n_trials;               /* sum of n_dm */
  int32_t pad_;
  int64_t total;                  /* int32 elements of the whole output */
} gsp_dmt_desc;

/* Host only.  Validates the plan and fills `desc`.
 * freqs_mhz: host double[nchan], any order, all > 0 and finite.
 * Errors: EINVAL (bad argument), ETOOSHORT (a row's n_out <= 0), EOVERFLOW
 * (255 * D * nchan >= 2^31, or an element count beyond int64). */
int gsp_plan_shape(int64_t nsamp, int32_t nchan, const double *freqs_mhz, double tsamp_s,
                   const gsp_segment *segs, int32_t n_seg, gsp_dmt_desc *desc);

/* Host only.  The delay table of row `seg` of a shaped plan, as the
 * dedispersion uses it: out int32 [n_dm][nchan] (host, caller-allocated). */
int gsp_delay_table(const gsp_dmt_desc *desc, const double *freqs_mhz, int32_t seg, int32_t *out);

/* Dedisperse a filterbank over a plan.  Asynchronous on `stream`.
 * fb_dev:  device uint8 [nsamp][nchan], time-major (spectrum by spectrum),
 *          as recorded (Algorithm 2's [numpts][numchan] layout).
 * freqs_mhz: host double[nchan] (the same array given to gsp_plan_shape).
 * dmt_dev: device int32 [desc->total], caller-allocated, fully overwritten:
 *          dmt[offset[s] + i*n_out[s] + t] = sum_c Y_s[c][t + d_s(i, c)] where
 *          Y_s is the D_s-downsampled input.
 * The filterbank must stay unchanged until the work on `stream` completes. */
int gsp_dedisperse(gsp_ctx *ctx, const uint8_t *fb_dev, const double *freqs_mhz, const gsp_dmt_desc *desc,
                   int32_t *dmt_dev, void *stream);

/* Population mean and sigma of every trial's series over its n_out samples,
 * from exact integer moments about the series' first sample.
 * mu_host, sigma_host: host double[desc->n_trials].  Synchronises `stream`. */
int gsp_trial_stats(gsp_ctx *ctx, const int32_t *dmt_dev, const gsp_dmt_desc *desc, double *mu_host,
                    double *sigma_host, void *stream);

/* One single-pulse candidate: the peak of a maximal run of box ends whose
 * best boxcar SNR is >= threshold. */
typedef struct gsp_candidate {
  int32_t seg;      /* plan row */
  int32_t dm_index; /* trial index within the row */
  double dm;        /* trial DM */
  int64_t t_peak;   /* first sample of the peak box (row resolution) */
  int64_t t_first;  /* first box end of the run */
  int64_t t_last;   /* last box end of the run */
  int32_t width;    /* peak box width, samples of the row */
  float snr;        /* peak SNR */
  double time_s;    /* (t_peak + width/2) * D * tsamp, s from the first sample */
} gsp_candidate;

/* Boxcar matched-filter search of a dedispersed plan.
 * For every trial: mu, sigma as in gsp_trial_stats; for every width w of the
 * set `widths` (host int32[n_widths], n_widths <= 64, each in [1, 4096],
 * duplicates ignored) and box
 * end e with w-1 <= e < n_out:  snr(e,w) = (sum_{k=e-w+1..e} x_k - w*mu) /
 * (sigma*sqrt(w)) in double; best(e) = max over w (ties -> smaller w); each
 * maximal run of e with best(e) >= threshold gives one candidate at its
 * argmax (ties -> earlier e).  Trials with sigma = 0 give none.
 * cands_host: host array of `capacity`; candidates sorted by
 * (seg, dm_index, t_peak).  *n_found = total count; if it exceeds capacity the
 * first `capacity` are written and GSP_ECAPACITY is returned.
 * Synchronises `stream` (the count is data-dependent). */
int gsp_single_pulse_search(gsp_ctx *ctx, const int32_t *dmt_dev, const gsp_dmt_desc *desc,
                            const int32_t *widths, int32_t n_widths, float threshold,
                            gsp_candidate *cands_host, int64_t capacity, int64_t *n_found, void *stream);

/* Friends-of-friends grouping of candidates (host only): two candidates are
 * linked when they share the plan row, their trial indices differ by at most
 * one and their run extents [t_first, t_last] overlap.  rep_out[k] = index of
 * the representative of k's group: the member of highest snr (ties -> lower
 * dm_index, then earlier t_peak).  Returns the number of groups via n_groups. */
int gsp_group_candidates(const gsp_candidate *cands, int64_t n, int64_t *rep_out, int64_t *n_groups);

/* Launch shape of the dedispersion kernel for one plan row: each workgroup
 * holds `waves` wavefronts of 64 lanes; a wave accumulates `tpw` DM trials
 * over 128*`groups` output samples; `chunk` channels are staged into LDS per
 * pass (the library lowers it to fit LDS and its staging registers). */
typedef struct gsp_shape {
  int32_t groups; /* 2, 4 or 8 */
  int32_t tpw;    /* 4 or 8 */
  int32_t waves;  /* 1 .. 8 */
  int32_t chunk;  /* >= 1 */
} gsp_shape;

/* Autotuner.  For every plan row of `desc`, times the dedispersion kernel
 * with each built-in candidate shape on the given input (dmt_dev is
 * overwritten; fb_dev as in gsp_dedisperse), `n_reps` timed launches each,
 * keeps the fastest and uses it for every later call on this context whose
 * row has the same signature (nchan, D, n_dm, maximum delay, length class).
 * Synchronises `stream`. */
int gsp_autotune(gsp_ctx *ctx, const uint8_t *fb_dev, const double *freqs_mhz, const gsp_dmt_desc *desc,
                 int32_t *dmt_dev, int32_t n_reps, void *stream);
/* The shape in use (or that would be used) for row `seg` of a plan. */
int gsp_row_shape(gsp_ctx *ctx, const double *freqs_mhz, const gsp_dmt_desc *desc, int32_t seg, gsp_shape *out);
/* Force a shape for rows with the signature of row `seg` (tests, tuning). */
int gsp_set_row_shape(gsp_ctx *ctx, const double *freqs_mhz, const gsp_dmt_desc *desc, int32_t seg,
                      const gsp_shape *shape);
/* Tuned shapes as text, one "signature groups tpw waves chunk" line per row
 * signature; load merges into the context's table. */
int gsp_tuning_save(const gsp_ctx *ctx, const char *path);
int gsp_tuning_load(gsp_ctx *ctx, const char *path);

/* Kernel timing (tracing).  When enabled, the library brackets each of its
 * kernel launches with a pair of HIP events on the launch's stream.
 * gsp_profile_read waits for the recorded events, then reports per kernel
 * name: launch count, summed duration and summed algorithmic work (integer
 * adds for the dedispersion kernel, bytes read + written for the streaming
 * kernels).  out: host array of `cap` entries; *n = number of kernel names.
 * reset != 0 clears the records after reading.  Disabled by default. */
typedef struct gsp_kernel_stat {
  char name[32];
  int64_t launches;
  double total_ms;
  double work;
} gsp_kernel_stat;
int gsp_profile_enable(gsp_ctx *ctx, int enable);
int gsp_profile_read(gsp_ctx *ctx, gsp_kernel_stat *out, int32_t cap, int32_t *n, int reset);

#ifdef __cplusplus
}
#endif

#endif /* GSP_H */
