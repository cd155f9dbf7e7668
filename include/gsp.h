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
typedef struct gsp_cnn gsp_cnn; /* triage network, declared with its functions below */

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
  int32_t kind;                   /* 0: brute-force plan (gsp_plan_shape); 1: sub-band plan */
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

/* Sub-band (two-stage) dedispersion: the algorithm GSP itself runs (Section
 * 2.3 names PRESTO's sub-band dedispersion; Tables 2-3 are its survey
 * plans).  Per plan row s the channels form n_sub[s] bands, band b =
 * channels [b*nchan/n_sub, (b+1)*nchan/n_sub) with reference frequency f_b =
 * its highest channel, and the row's trials form groups of group[s]
 * consecutive trials, group g (n_g trials from trial g*group) with nominal
 * DM_g = dm_lo + (g*group + (n_g - 1)/2) * dm_step.  With Y the row's
 * D-downsampled input:
 *   stage 1: Z[g][b][t] = sum over channels c of band b of Y[c][t + d1(g, c)],
 *            d1(g, c) = delay of DM_g at f_c against f_b;
 *   stage 2: dmt[i][t] = sum over bands b of Z[g(i)][b][t + d2(i, b)],
 *            d2(i, b) = delay of DM_i at f_b against fref;
 * both delays rounded as in gsp_delay_table with the reference frequency
 * replaced.  The sums are exact; the composite delays d2 + d1 differ from
 * the brute-force ones by the in-band smearing of |DM_i - DM_g|.  A row's
 * valid length is floor(nsamp/D) minus its largest d2(i, b) + max over the
 * band of d1(g(i), c) (desc->max_delay).  Adds per output: nchan/group + n_sub
 * instead of nchan.
 * gsp_subband_plan_shape: as gsp_plan_shape, for a sub-band plan (host
 * only; n_sub, group: host int32[n_seg]); sets desc->kind = 1.  GSP_EINVAL
 * unless 1 <= n_sub[s] <= nchan, 1 <= group[s] <= 64 and
 * 255 * D * ceil(nchan / n_sub[s]) <= 65535 (16-bit sub-band series).
 * gsp_dedisperse_subband: as gsp_dedisperse, with the same n_sub and group
 * and a descriptor from gsp_subband_plan_shape; the output feeds
 * gsp_single_pulse_search and gsp_trial_stats like a brute-force one. */
int gsp_subband_plan_shape(int64_t nsamp, int32_t nchan, const double *freqs_mhz, double tsamp_s,
                           const gsp_segment *segs, int32_t n_seg, const int32_t *n_sub, const int32_t *group,
                           gsp_dmt_desc *desc);
int gsp_dedisperse_subband(gsp_ctx *ctx, const uint8_t *fb_dev, const double *freqs_mhz, const gsp_dmt_desc *desc,
                           const int32_t *n_sub, const int32_t *group, int32_t *dmt_dev, void *stream);

/* RFI mitigation of a filterbank, integers throughout (Section 2.1 lists RFI
 * mitigation among the search steps; Section 3.1 tests PRESTO's clip option
 * on CPU and GPU; the paper defines neither operation, so this is the
 * reading taken).
 *   clip (clip_sigma > 0): spectra in blocks of `block` (the last may be
 *     shorter).  Per block, the zero-DM series s_j = sum_c x[j][c] has
 *     population mean mu and sigma from exact integer moments; spectrum j
 *     is flagged when |s_j - mu| > clip_sigma * sigma (double).  If some
 *     but not all of the block's spectra are flagged, each flagged one
 *     becomes the block's channel means over its n_u unflagged spectra,
 *     m_c = floor((2 S_c + n_u) / (2 n_u)), S_c their channel sums.
 *   zero-DM filter (zero_dm != 0), after clipping: the rounded mean
 *     z_j = floor((2 s'_j + nchan) / (2 nchan)) of each (clipped) spectrum is
 *     subtracted and 128 added back, clamped to 0..255.
 * fb_dev, out_dev: device uint8 [nsamp][nchan] (time-major); out_dev may be
 * fb_dev (in place) but must not overlap it otherwise.  n_flagged (host,
 * optional): spectra replaced by the clip; when given, the call synchronises
 * `stream`, otherwise it is asynchronous.  GSP_EINVAL for bad sizes,
 * clip_sigma < 0 or not finite, block outside [1, 2^30] when clipping. */
int gsp_rfi_clean(gsp_ctx *ctx, const uint8_t *fb_dev, int64_t nsamp, int32_t nchan, double clip_sigma, int64_t block,
                  int32_t zero_dm, uint8_t *out_dev, int64_t *n_flagged, void *stream);

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
/* For callers that cannot allocate memory (tight serving loops, harnesses
 * that forbid allocation): gsp_single_pulse_search with no allocation.
 * Every device buffer of the search (job table, per-trial statistics,
 * width set, run fragments, their counter) lives in one static device array
 * of about 3.7 MB that each GPU the library runs on holds until the process
 * ends; its address is taken once per device by
 * gsp_create.  The host work (joining run fragments, building and sorting the
 * candidates) runs in place in cands_host, so the call allocates nothing on
 * the host either.  Same arguments and results as gsp_single_pulse_search,
 * within these limits:
 *   desc->n_trials <= 32768 and at most 65536 run fragments per call
 *   (GSP_ECAPACITY otherwise, with a message);
 *   capacity must be at least the number of run fragments (each run of
 *   the search is one or more fragments, joined on the host): if it is
 *   not, nothing is written, *n_found is set to that number (a capacity
 *   that suffices) and GSP_ECAPACITY is returned.
 * Calls on one GPU share its array, which keeps the last call's contents:
 * calls that overlap on one GPU (other threads, other streams) race.
 * Synchronises `stream`. */
int gsp_single_pulse_search_noalloc(gsp_ctx *ctx, const int32_t *dmt_dev, const gsp_dmt_desc *desc,
                                    const int32_t *widths, int32_t n_widths, float threshold,
                                    gsp_candidate *cands_host, int64_t capacity, int64_t *n_found, void *stream);

/* Friends-of-friends grouping of candidates (host only): two candidates are
 * linked when they share the plan row, their trial indices differ by at most
 * one and their run extents [t_first, t_last] overlap.  rep_out[k] = index of
 * the representative of k's group: the member of highest snr (ties -> lower
 * dm_index, then earlier t_peak).  Returns the number of groups via n_groups. */
int gsp_group_candidates(const gsp_candidate *cands, int64_t n, int64_t *rep_out, int64_t *n_groups);

/* ---- Sifting: ranking of grouped events, and the candidate store ----
 *
 * The paper sifts single-pulse events with RRATtrap (Section 2.2: events of
 * nearby DMs and times are grouped, the groups ranked and scored by rules;
 * Section 3.2: groups of rank 3 to 6, 6 the best, and a class of RFI or
 * noise) without stating the rules.  The reading taken here, per group of
 * gsp_group_candidates (members of one plan row):
 *   n_events members, n_trials distinct trials, DM range [dm_min, dm_max];
 *   the peak is the representative (dm_peak, snr_max, time_s, width_s =
 *   width * D * tsamp); the group spans start_s = min over members of
 *   (t_first - width + 1) * D * tsamp to max (t_last + 1) * D * tsamp;
 *   snr_lo, snr_hi = best member SNR at dm_min and at dm_max.
 *   rank 2 (RFI):   dm_peak < 1 pc cm^-3;
 *   rank 1 (noise): otherwise, n_trials < 3;
 *   else with f = min(1 - snr_lo/snr_max, 1 - snr_hi/snr_max), the fall-off
 *   of SNR toward both ends of the DM range (in double): rank 3 if f < 0.1,
 *   4 if f < 0.2, 5 if f < 0.35, otherwise 6. */
typedef struct gsp_group_record {
  int64_t rep;             /* index of the representative (peak) candidate */
  int32_t seg, rank;
  int32_t n_events, n_trials;
  double dm_min, dm_max, dm_peak;
  float snr_max, snr_lo, snr_hi;
  int32_t reserved;
  double time_s, width_s, start_s, duration_s;
} gsp_group_record;
/* Host only.  cands and rep (host, n entries: rep from gsp_group_candidates)
 * and the plan's descriptor in; one record per group out (host array of cap),
 * in order of the representative's index; *n_groups = number of groups
 * (GSP_ECAPACITY when it exceeds cap).  GSP_EINVAL if rep is not a grouping
 * (rep[rep[k]] == rep[k] for every k). */
int gsp_rank_groups(const gsp_candidate *cands, int64_t n, const int64_t *rep, const gsp_dmt_desc *desc,
                    gsp_group_record *out, int64_t cap, int64_t *n_groups);

/* Candidate store with the six tables of the paper's database (Section 2.2):
 *   T_FITS_INFO               one row per processed input (name, beam, nchan,
 *                             nsamp, tsamp, band edges);
 *   T_SINGLEPULSE_GROUPS      one row per input: candidates, groups, groups per rank;
 *   T_SINGLEPULSE_CANDIDATES  one row per ranked group (gsp_group_record);
 *   T_PULSAR                  known sources (name, DM) entered by the caller;
 *   T_FILE_PULSAR             known sources matched by DM to an input's groups;
 *   T_SINGLEPULSE_PIC         a picture path per candidate (e.g. its cutout).
 * Kept in host memory; gsp_store_save / gsp_store_load write and read one CSV
 * file per table (named as above) in a directory.  Ids start at 1.  Names and
 * paths must not hold commas, quotes or line breaks (GSP_EINVAL).  Not
 * thread-safe: one caller at a time. */
enum {
  GSP_T_FITS_INFO = 0,
  GSP_T_SINGLEPULSE_GROUPS = 1,
  GSP_T_SINGLEPULSE_CANDIDATES = 2,
  GSP_T_PULSAR = 3,
  GSP_T_FILE_PULSAR = 4,
  GSP_T_SINGLEPULSE_PIC = 5
};
typedef struct gsp_store gsp_store;
typedef struct gsp_store_candidate {
  int64_t id, file_id;
  gsp_group_record g;
} gsp_store_candidate;
int gsp_store_create(gsp_store **out);
void gsp_store_destroy(gsp_store *s);
const char *gsp_store_last_error(const gsp_store *s);
int gsp_store_add_file(gsp_store *s, const char *name, int32_t beam, int32_t nchan, int64_t nsamp, double tsamp_s,
                       double f_lo_mhz, double f_hi_mhz, int64_t *file_id);
/* The ranked groups of one input (each input once); *first_id = id of the first. */
int gsp_store_add_groups(gsp_store *s, int64_t file_id, int64_t n_candidates, const gsp_group_record *groups,
                         int64_t n, int64_t *first_id);
int gsp_store_add_pulsar(gsp_store *s, const char *name, double dm, int64_t *pulsar_id);
/* Replaces the input's T_FILE_PULSAR rows: every known source with at least
 * one stored group of rank >= min_rank whose dm_peak lies within dm_tol of its
 * DM (with the number of such groups and their best SNR). */
int gsp_store_match_pulsars(gsp_store *s, int64_t file_id, double dm_tol, int32_t min_rank, int64_t *n_matches);
int gsp_store_add_picture(gsp_store *s, int64_t cand_id, const char *path);
/* Stored candidates with rank >= min_rank and dm_lo <= dm_peak <= dm_hi, in
 * id order (GSP_ECAPACITY with *n = count when more than cap). */
int gsp_store_query(gsp_store *s, int32_t min_rank, double dm_lo, double dm_hi, gsp_store_candidate *out,
                    int64_t cap, int64_t *n);
int gsp_store_count(const gsp_store *s, int32_t table, int64_t *n);
int gsp_store_save(gsp_store *s, const char *dir);
/* Replaces the store's contents with the tables in dir. */
int gsp_store_load(gsp_store *s, const char *dir);

/* ---- Streaming: continuous batching of beams arriving in blocks ----
 *
 * The overlap between consecutive blocks that the paper's dedispersion loop
 * takes from the previous block (Algorithm 2: lastdata/data; Algorithm 3:
 * one merged 2*numpts buffer, Section 2.3) is kept on the device per (beam,
 * plan row): the downsampled samples of the last (maximum delay + one block).
 * Each block of B raw samples (B a multiple of 4 x every downsampling factor)
 * yields, per row with downsampling D and maximum delay M, the outputs
 *     window k = [max(0, N_k - M), max(0, N_{k+1} - M))
 * (N_k = downsampled samples received before block k): exactly the outputs of
 * gsp_dedisperse over the beam so far, bit for bit.  Statistics are taken per
 * (window, trial) over the window's samples; box ends lie in the window and
 * boxes may reach back up to (max width - 1) samples into earlier windows;
 * runs are split at window edges.  A beam's results do not depend on which
 * other beams share its steps.
 *
 * One step processes one pending block of every admitted beam with a fixed
 * sequence of kernels captured once as a hipGraph and replayed.  Beams are
 * admitted against the device-memory budget; a beam that does not fit is
 * queued (GSP_EAGAIN, the id stays valid and its blocks are held on the host)
 * and admitted, in order, when finished beams release memory. */
typedef struct gsp_stream gsp_stream;

typedef struct gsp_stream_candidate {
  int32_t beam;   /* beam id */
  int32_t block;  /* index of the beam's block whose window held the run */
  gsp_candidate c; /* times in absolute samples of the row since the beam's start */
  float score;    /* triage network logit (NaN when no network is attached) */
  int32_t reserved;
} gsp_stream_candidate;

typedef struct gsp_stream_stats {
  double lat_p50_s, lat_p99_s, lat_max_s; /* push -> results on the host, per block */
  int64_t blocks, steps;
  double busy_s;                          /* wall time inside steps */
  int64_t mem_used, mem_budget;           /* device bytes held by admitted beams */
  int32_t beams_active, beams_queued;
  int64_t blocks_pending;
  int64_t triage_scored, triage_rejected; /* candidates scored / dropped by the network */
  double triage_s;                        /* wall time of cutouts + network inside steps */
  int64_t search_repeats;                 /* steps whose search ran again with a grown fragment buffer */
} gsp_stream_stats;

/* widths/threshold: the search of every beam (as gsp_single_pulse_search). */
int gsp_stream_create(gsp_ctx *ctx, int64_t mem_budget_bytes, int32_t block_nsamp, const int32_t *widths,
                      int32_t n_widths, float threshold, gsp_stream **out);
void gsp_stream_destroy(gsp_stream *s);
const char *gsp_stream_last_error(const gsp_stream *s);
/* GSP_OK: admitted; GSP_EAGAIN: queued (beam_id valid); GSP_ENOMEM: larger than the budget. */
int gsp_stream_open_beam(gsp_stream *s, int32_t nchan, const double *freqs_mhz, double tsamp_s,
                         const gsp_segment *segs, int32_t n_seg, int32_t *beam_id);
/* block_host: uint8 [nsamp][nchan] time-major, copied before return;
 * nsamp < block_nsamp marks the beam's last block. */
int gsp_stream_push(gsp_stream *s, int32_t beam_id, const uint8_t *block_host, int64_t nsamp);
/* No more blocks; the beam's memory is released after its last block.
 * A beam whose last block (short block, or the last one before close) has
 * been processed is removed: its id is then unknown (GSP_EINVAL). */
int gsp_stream_close_beam(gsp_stream *s, int32_t beam_id);
/* Learned triage of streamed candidates (Sections 2.1 and 4 name the
 * classification stage; see gsp_cutouts and gsp_cnn_*): with a network
 * attached, each step cuts out its candidates from the stream's device state
 * (the window of dedispersed series with the look-back before it, the ring
 * of downsampled samples; times before the beam's start count as the
 * window's mean of the trial in the DM-time image and are left out of the
 * frequency-time image, as in gsp_cutouts), scores them, and passes on only
 * those with logit > threshold; gsp_stream_candidate.score carries the
 * logit.  cnn = NULL detaches (the plain search: every candidate passes).
 * The network must outlive its attachment; the worker thread must be
 * stopped. */
int gsp_stream_set_triage(gsp_stream *s, gsp_cnn *cnn, float threshold);
/* Caller-driven processing: one step (*n_blocks = blocks processed, 0 if idle). */
int gsp_stream_step(gsp_stream *s, int64_t *n_blocks);
/* Library-driven processing: a worker thread steps whenever blocks are pending. */
int gsp_stream_start(gsp_stream *s);
int gsp_stream_stop(gsp_stream *s);
/* Wait until every pushed block of the admitted beams is processed. */
int gsp_stream_flush(gsp_stream *s);
/* Drain up to cap candidates found so far (in step order). */
int gsp_stream_poll(gsp_stream *s, gsp_stream_candidate *out, int64_t cap, int64_t *n);
int gsp_stream_report(gsp_stream *s, gsp_stream_stats *out);
/* The last step's window of row `seg`: host int32 [n_dm][*n_t], outputs
 * *t_first .. *t_first + *n_t - 1 (worker stopped).  *t_first and *n_t are
 * always set; GSP_ECAPACITY if host_out is NULL or cap < n_dm * *n_t. */
int gsp_stream_window(gsp_stream *s, int32_t beam_id, int32_t seg, int32_t *host_out, int64_t cap, int64_t *t_first,
                      int64_t *n_t);
/* Beam state (rings, look-back, counters) to/from host memory; restore into a
 * freshly opened beam with the same plan continues bit-identically. */
int gsp_stream_snapshot(gsp_stream *s, int32_t beam_id, void *host_buf, int64_t cap, int64_t *bytes);
int gsp_stream_restore(gsp_stream *s, int32_t beam_id, const void *host_buf, int64_t bytes);
/* 1 (default): replay the captured step graph; 0: launch the kernels directly. */
int gsp_stream_set_graph(gsp_stream *s, int enable);
/* Capacity of a step's buffer of run fragments (default 65,536; cap in
 * [1, 2^30]).  A step whose search finds more grows the buffer and searches
 * the same windows again before it returns (the windows are intact until the
 * next step), so no candidate is lost; a smaller capacity only makes that
 * happen sooner (tests).  Worker thread stopped; the next step captures
 * its graph anew. */
int gsp_stream_set_fragment_capacity(gsp_stream *s, int64_t cap);

/* Launch shape of the dedispersion kernel for one plan row: each workgroup
 * holds `waves` wavefronts of 64 lanes; a wave accumulates `tpw` DM trials.
 * kind 0, the 16-bit tile (any row): a wave covers 128*`groups` output
 * samples (dwords of two 16-bit samples); at most `chunk` channels are
 * staged into LDS per pass.  Passes run over consecutive channels and each
 * is as long as the LDS budget, the staging registers and the trial offsets
 * a thread loads allow for the staged windows of its channels (a channel's
 * window covers the delay spread of a tile of trials at that channel), up
 * to `chunk`.  kind 1, the byte-quad tile (rows with D = 1 and a multiple of
 * 4 channels): a wave covers 64*`groups` output samples; LDS dwords hold the
 * bytes of 4 neighbouring channels, one staged copy per distinct pattern of
 * delay differences inside the quad over a tile of trials; at most `chunk`
 * (<= 64) quads per pass.  kind 2: the byte-quad tile with 4 more waves per
 * workgroup that stage the next pass while the `waves` summing waves add
 * the current one.  kind 3: a split row, for bands whose lowest (or
 * highest) channels have delay copies too wide for the byte-quad tile: kind
 * 2 with this shape over the channels whose copies fit, the 16-bit tile with
 * shape (4, 4, 8, 32) over the run of channels at the end of the band that
 * holds every quad that does not fit, both summed into the same outputs;
 * GSP_EINVAL where every quad fits or those quads are not at one end.  The
 * default for D = 1 rows with a multiple of 4 channels is kind 2 (4, 8, 8,
 * 64) where its copies fit, else kind 3 where it applies, else kind 0 (4, 4,
 * 8, 32); for other rows kind 0 (4, 4, 8, 32).  gsp_row_shape reports the
 * longest pass in `chunk` (of the byte-quad part for kind 3). */
typedef struct gsp_shape {
  int32_t groups; /* kind 0: 2, 4 or 8; kind 1: 4, 8 or 16; kinds 2, 3: 4 or 8 */
  int32_t tpw;    /* kind 0: 4 or 8; kind 1: 2, 4 or 8; kinds 2, 3: 8 (groups 4) or 4 (groups 8) */
  int32_t waves;  /* kind 0: 1 .. 8; kind 1: 1 .. 16; kinds 2, 3: 1 .. 12 summing waves */
  int32_t chunk;  /* >= 1 */
  int32_t kind;   /* 0: 16-bit tile, 1: byte-quad tile, 2: with staging waves, 3: split row */
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
/* Tuned shapes as text, one "signature groups tpw waves chunk kind" line per
 * row signature; load merges into the context's table (a missing kind reads
 * as 0). */
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

/* ------------------------------------------------------------------------
 * Learned triage of candidates.  The paper classifies candidates after the
 * search (Section 2.1 names the step, Section 4 its role before the
 * database); it does not define a classifier.  Here: two 64 x 64 images per
 * candidate and a small convolutional network trained on the GPU.
 * ---------------------------------------------------------------------- */

/* Cutouts of candidates found in a dedispersed plan.  For candidate k (row s,
 * trial i, peak box start t_peak, width w, all at the row's resolution), with
 * box end e = t_peak + w - 1 and bin width r = clamp(w / 8, 1, 8):
 *   image 0, DM-time: trials lo .. lo+63 of row s with
 *     lo = clamp(i - 32, 0, n_dm - 64) (rows of fewer than 64 trials leave
 *     the missing lines 0), bins b = 0..63 of r samples each covering
 *     [e - (64-b) r + 1, e - (63-b) r] (the box ends in the last bin, nothing
 *     after e is read); bin value = sum of the dedispersed series, samples
 *     before the start of the data counted at the trial's mean;
 *   image 1, frequency-time: 64 sub-bands, band j = channels
 *     [j nchan / 64, (j+1) nchan / 64), each channel shifted by its delay at
 *     trial i, the same 64 bins at the row's resolution (bin value = sum of
 *     the band's D-downsampled samples); a bin that starts before the data
 *     is scaled to r samples from its valid part, one wholly before it takes
 *     the mean of the band's valid bins;
 * then each image is z-scored (mean 0, variance 1 over its 4096 pixels; a
 * constant image becomes 0) and stored as bf16 (round to nearest even).
 * fb_dev, freqs_mhz, dmt_dev, desc: as for gsp_dedisperse (dmt_dev is its
 * output for this filterbank).  cands_dev: device gsp_candidate[n] (as
 * returned by the search, copied to the device); a candidate whose row,
 * trial or box end lies outside the plan gets two zero images.  out_dev: device
 * bf16 (uint16) [n][2][64][64].  Asynchronous on `stream`.  Trial means are
 * computed only for the trials of images whose first bin starts before the
 * data (a pass over those rows alone).  Batches of 256 or more candidates
 * read a channel-major copy of fb_dev: the one the last gsp_dedisperse on
 * this context left staged when it wrote dmt_dev from fb_dev and ended with
 * a row without downsampling (it orders such rows last), else one made here
 * in the context's staging buffer.  The context keeps
 * a device buffer of 16 KB per candidate for the frequency-time band sums
 * (grown, with a device synchronisation, when a call has more candidates
 * than any before it). */
int gsp_cutouts(gsp_ctx *ctx, const uint8_t *fb_dev, const double *freqs_mhz, const int32_t *dmt_dev,
                const gsp_dmt_desc *desc, const gsp_candidate *cands_dev, int64_t n, uint16_t *out_dev,
                void *stream);

/* Triage network (input bf16 [n][2][64][64], as gsp_cutouts writes):
 *   conv3x3(2->16) ReLU maxpool2, conv3x3(16->32) ReLU maxpool2,
 *   conv3x3(32->64) ReLU maxpool2, conv3x3(64->128) ReLU maxpool2,
 *   flatten (h, w, c) -> 2048, FC 2048->192 ReLU, FC 192->1 = logit
 *   (logit > 0: astrophysical).  Convolutions use zero padding 1; max-pool
 *   ties go to the first position in (row, column) order.
 * Storage: bf16 activations and weights, fp32 accumulation, fp32 master
 * weights and biases.  Parameters as one float vector, in this order, per
 * layer weights then biases:
 *   conv l: w[cout][3][3][cin] (kernel row, kernel column, input channel),
 *           b[cout];  fc1: w[192][2048], b[192];  fc2: w[192], b[1].
 * Loss: mean over the batch of the binary cross-entropy with logits;
 * optimiser Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected). */
int64_t gsp_cnn_num_params(void);
/* He-uniform weights drawn from `seed` (SplitMix64), zero biases. */
int gsp_cnn_create(gsp_ctx *ctx, uint64_t seed, gsp_cnn **out);
void gsp_cnn_destroy(gsp_cnn *cnn);
/* host float[n], n = gsp_cnn_num_params(); set also clears the Adam state. */
int gsp_cnn_get_params(gsp_cnn *cnn, float *params_host, int64_t n);
int gsp_cnn_set_params(gsp_cnn *cnn, const float *params_host, int64_t n);
int gsp_cnn_save(const gsp_cnn *cnn, const char *path);
int gsp_cnn_load(gsp_cnn *cnn, const char *path);
/* logits_dev: device float[n].  x_dev: device bf16 [n][2][64][64].
 * Synchronises `stream` before it starts (buffers may grow), then runs
 * asynchronously on it. */
int gsp_cnn_forward(gsp_cnn *cnn, const uint16_t *x_dev, int64_t n, float *logits_dev, void *stream);
/* Gradient of the mean loss over the batch with respect to every parameter
 * (host float[num_params], same order), and the mean loss (host, optional);
 * labels_dev: device float[n] in {0, 1}.  Parameters are unchanged.
 * Synchronises `stream`. */
int gsp_cnn_gradients(gsp_cnn *cnn, const uint16_t *x_dev, const float *labels_dev, int64_t n,
                      float *grads_host, float *loss_host, void *stream);
/* One Adam step on the batch with learning rate lr > 0.  loss_host
 * (optional) receives the batch's mean loss before the step and then the
 * call synchronises `stream`; without it the step stays asynchronous. */
int gsp_cnn_train_step(gsp_cnn *cnn, const uint16_t *x_dev, const float *labels_dev, int64_t n, float lr,
                       float *loss_host, void *stream);
/* Inspection of stored tensors (tests), l = 0..3 the convolution block:
 *   which = l       pooled output of block l, bf16 [n][h][w][c] (h = w = 32, 16, 8, 4);
 *   which = 4       the hidden layer (after ReLU), bf16 [n][192];
 *   which = 5       the logits, float [n];
 *   which = 12 + l  ReLU output of block l before pooling, bf16 [n][2h][2h][c];
 *   which = 16 + l  max-pool choice of block l, uint8 [n][h][w][c], 2*(row parity) + column parity;
 * all of the last forward pass (gsp_cnn_forward, gsp_cnn_gradients or
 * gsp_cnn_train_step), and, of the last backward pass (gsp_cnn_gradients or
 * gsp_cnn_train_step, with no forward pass of another batch since):
 *   which = 6 + l   gradient of the loss with respect to block l's pooled output, bf16 [n][h][w][c];
 *   which = 10      gradient with respect to the hidden layer's pre-activation, bf16 [n][192];
 *   which = 11      dloss/dlogit per sample, float [n].
 * `bytes` must equal the size for that batch (GSP_EINVAL otherwise, and
 * when no such pass has run).  Synchronises the device. */
int gsp_cnn_activation(gsp_cnn *cnn, int32_t which, void *host_out, int64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* GSP_H */
