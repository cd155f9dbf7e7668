// Plan expansion and delay tables (host side).
//
// A plan is a list of DDplan-style rows (paper Section 2.1, Tables 2-3).  The
// per-(trial, channel) delays are the [numdm][numchan] table of Algorithms
// 2-3 (Section 2.3); the paper gives no dispersion law or rounding rule, so
// the reading documented in gsp.h is used: cold-plasma law with
// K = 4148.808 s MHz^2 cm^3/pc, referenced to the highest channel, rounded
// half up in IEEE double.  This file must be compiled without FMA
// contraction so that every host evaluates the expression the same way.
#include <cmath>
#include <cstring>
#include <limits>

#include "gsp_internal.h"

namespace gsp {

static const double kDispersion = 4148.808;

double fref_of(const double *freqs, int32_t nchan) {
  double f = freqs[0];
  for (int32_t c = 1; c < nchan; ++c) f = freqs[c] > f ? freqs[c] : f;
  return f;
}

static inline double trial_dm(const gsp_segment &s, int32_t i) { return s.dm_lo + (double)i * s.dm_step; }

int64_t delay_of(double dm, double f, double fref, double tsamp, int32_t D) {
  const double sweep = 1.0 / (f * f) - 1.0 / (fref * fref);
  const double r = ((kDispersion * dm) * sweep) / (tsamp * (double)D);
  return (int64_t)std::floor(r + 0.5);
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

void compute_delays(const gsp_dmt_desc *desc, const double *freqs, int32_t s, int32_t *out) {
  const gsp_segment &g = desc->seg[s];
  const double fref = desc->fref_mhz;
  for (int32_t i = 0; i < g.n_dm; ++i) {
    const double dm = trial_dm(g, i);
    int32_t *row = out + (int64_t)i * desc->nchan;
    for (int32_t c = 0; c < desc->nchan; ++c)
      row[c] = (int32_t)delay_of(dm, freqs[c], fref, desc->tsamp, g.downsamp);
  }
}

void validate_desc(const gsp_dmt_desc *d) {
  if (!d) fail(GSP_EINVAL, "null plan descriptor");
  if (d->nsamp < 1 || d->nchan < 1 || !finite_pos(d->tsamp) || d->n_seg < 1 || d->n_seg > GSP_MAX_SEG)
    fail(GSP_EINVAL, "plan descriptor is not shaped (call gsp_plan_shape)");
  if (d->kind != 0 && d->kind != 1) fail(GSP_EINVAL, "plan descriptor kind must be 0 or 1");
  int64_t off = 0;
  int32_t t0 = 0;
  for (int32_t s = 0; s < d->n_seg; ++s) {
    if (d->n_out[s] < 1 || d->offset[s] != off || d->trial0[s] != t0 || d->seg[s].n_dm < 1 ||
        d->seg[s].downsamp < 1 || d->seg[s].downsamp > 257)
      fail(GSP_EINVAL, "plan descriptor is inconsistent (call gsp_plan_shape)");
    off += (int64_t)d->seg[s].n_dm * d->n_out[s];
    t0 += d->seg[s].n_dm;
  }
  if (off != d->total || t0 != d->n_trials) fail(GSP_EINVAL, "plan descriptor totals are inconsistent");
}

std::string plan_key(const gsp_dmt_desc *desc, const double *freqs) {
  std::string k;
  k.append(reinterpret_cast<const char *>(desc), sizeof(gsp_dmt_desc));
  k.append(reinterpret_cast<const char *>(freqs), sizeof(double) * (size_t)desc->nchan);
  return k;
}

void plan_shape_impl(int64_t nsamp, int32_t nchan, const double *freqs, double tsamp, const gsp_segment *segs,
                     int32_t n_seg, gsp_dmt_desc *desc) {
  if (!desc || !freqs || !segs) fail(GSP_EINVAL, "null pointer argument");
  if (nsamp < 1) fail(GSP_EINVAL, "nsamp must be >= 1");
  if (nchan < 1) fail(GSP_EINVAL, "nchan must be >= 1");
  if (!finite_pos(tsamp)) fail(GSP_EINVAL, "tsamp must be finite and > 0");
  if (n_seg < 1 || n_seg > GSP_MAX_SEG) fail(GSP_EINVAL, "n_seg must be in [1, 16]");
  for (int32_t c = 0; c < nchan; ++c)
    if (!finite_pos(freqs[c])) fail(GSP_EINVAL, "channel frequencies must be finite and > 0");
  gsp_dmt_desc d;
  std::memset(&d, 0, sizeof(d));
  d.nsamp = nsamp;
  d.nchan = nchan;
  d.n_seg = n_seg;
  d.tsamp = tsamp;
  d.fref_mhz = fref_of(freqs, nchan);
  int64_t off = 0;
  int64_t trials = 0;
  for (int32_t s = 0; s < n_seg; ++s) {
    const gsp_segment &g = segs[s];
    if (g.n_dm < 1) fail(GSP_EINVAL, "n_dm must be >= 1");
    if (g.downsamp < 1 || g.downsamp > 257) fail(GSP_EINVAL, "downsamp must be in [1, 257]");
    if (!(std::isfinite(g.dm_lo) && g.dm_lo >= 0.0)) fail(GSP_EINVAL, "dm_lo must be finite and >= 0");
    if (!finite_pos(g.dm_step)) fail(GSP_EINVAL, "dm_step must be finite and > 0");
    if (255.0 * g.downsamp * (double)nchan >= 2147483648.0)
      fail(GSP_EOVERFLOW, "255 * downsamp * nchan must stay below 2^31 (int32 sums)");
    d.seg[s] = g;
    // delays grow with DM and with falling frequency: the largest is at the last trial
    int64_t m = 0;
    const double dm_last = g.dm_lo + (double)(g.n_dm - 1) * g.dm_step;
    for (int32_t c = 0; c < nchan; ++c) {
      int64_t v = delay_of(dm_last, freqs[c], d.fref_mhz, tsamp, g.downsamp);
      m = v > m ? v : m;
    }
    if (m > (int64_t)std::numeric_limits<int32_t>::max()) fail(GSP_EOVERFLOW, "delay exceeds int32");
    d.max_delay[s] = m;
    d.n_out[s] = nsamp / g.downsamp - m;
    if (d.n_out[s] < 1) fail(GSP_ETOOSHORT, "input shorter than a plan row's maximum delay");
    d.offset[s] = off;
    d.trial0[s] = (int32_t)trials;
    if ((double)g.n_dm * (double)d.n_out[s] + (double)off > 9.0e18) fail(GSP_EOVERFLOW, "output too large");
    off += (int64_t)g.n_dm * d.n_out[s];
    trials += g.n_dm;
    if (trials > std::numeric_limits<int32_t>::max()) fail(GSP_EOVERFLOW, "too many trials");
  }
  d.n_trials = (int32_t)trials;
  d.total = off;
  *desc = d;
}

}  // namespace gsp
