// Single-pulse search over a dedispersed plan: per-trial statistics and the
// boxcar matched filter with run extraction.
//
// The paper names a single-pulse search stage (Section 2.1) without giving its
// statistic.  The one computed here (documented in gsp.h): population mean and
// sigma of each trial's series from exact integer moments; for every box end
// e and width w, snr = (box sum - w mu) / (sigma sqrt(w)); best over widths;
// one candidate per maximal run of best >= threshold.
//
// Both kernels are HBM-bound streaming passes over the int32 DM-time array:
//  k_stats  one workgroup per trial, 128-bit integer moment sums, tree
//           reduction in LDS, mu and sigma finished in double on the device;
//  k_search one workgroup per (trial, tile of box ends): the tile plus a
//           look-back of (max width - 1) samples is loaded once, turned into
//           exact int64 prefix sums by a workgroup scan in LDS, every width
//           is evaluated from two LDS reads, and maximal runs inside the tile
//           are appended as fragments with one atomic each.  Fragments that
//           touch a tile edge are joined on the host.
#include "gsp_internal.h"

namespace gsp {

struct SegTable {
  int64_t offset[GSP_MAX_SEG];
  int64_t n_out[GSP_MAX_SEG];
  int32_t trial0[GSP_MAX_SEG];
  int32_t n_dm[GSP_MAX_SEG];
  int64_t block0[GSP_MAX_SEG + 1];  // search: first workgroup of each row
  int32_t n_seg;
};

static SegTable make_table(const gsp_dmt_desc *d) {
  SegTable t{};
  t.n_seg = d->n_seg;
  for (int s = 0; s < d->n_seg; ++s) {
    t.offset[s] = d->offset[s];
    t.n_out[s] = d->n_out[s];
    t.trial0[s] = d->trial0[s];
    t.n_dm[s] = d->seg[s].n_dm;
  }
  return t;
}

__device__ __forceinline__ int seg_of_trial(const SegTable &t, int g) {
  int s = 0;
  for (int k = 1; k < t.n_seg; ++k)
    if (g >= t.trial0[k]) s = k;
  return s;
}

// ---------------------------------------------------------------------------
// statistics
// ---------------------------------------------------------------------------
static constexpr int kStatsThreads = 256;

__global__ __launch_bounds__(kStatsThreads) void k_stats(const int32_t *__restrict__ dmt, SegTable tb,
                                                          double *__restrict__ musig) {
  __shared__ int64_t r1[kStatsThreads];
  __shared__ unsigned __int128 r2[kStatsThreads];
  const int g = blockIdx.x;
  const int s = seg_of_trial(tb, g);
  const int64_t n = tb.n_out[s];
  const int32_t *x = dmt + tb.offset[s] + (int64_t)(g - tb.trial0[s]) * n;
  const int64_t x0 = x[0];
  int64_t s1 = 0;
  unsigned __int128 s2 = 0;
  for (int64_t k = threadIdx.x; k < n; k += kStatsThreads) {
    const int64_t v = (int64_t)x[k] - x0;
    s1 += v;
    const uint64_t a = (uint64_t)(v < 0 ? -v : v);
    s2 += (unsigned __int128)(a * a);
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int h = kStatsThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dn = (double)n;
    const double m1 = (double)r1[0] / dn;
    const double m2 = (double)r2[0] / dn;
    const double var = m2 - m1 * m1;
    musig[2 * g] = (double)x0 + m1;
    musig[2 * g + 1] = var > 0.0 ? sqrt(var) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// boxcar search
// ---------------------------------------------------------------------------
static constexpr int kSearchThreads = 256;
static constexpr int kSearchTile = 2048;  // box ends per workgroup

__global__ void k_zero_counter(unsigned long long *c) { *c = 0ull; }

__global__ __launch_bounds__(kSearchThreads) void k_search(const int32_t *__restrict__ dmt, SegTable tb,
                                                            const double *__restrict__ musig,
                                                            const int32_t *__restrict__ widths, int32_t nw,
                                                            int32_t wmax, float thr_f, Frag *__restrict__ frags,
                                                            int64_t cap, unsigned long long *__restrict__ counter) {
  extern __shared__ int64_t sm[];
  // layout: prefix Q[kSearchTile + wmax + 1] | best[kSearchTile] (double) | bw[kSearchTile] (int32)
  int64_t *Q = sm;
  double *best = reinterpret_cast<double *>(sm + kSearchTile + wmax + 1);
  int32_t *bw = reinterpret_cast<int32_t *>(best + kSearchTile);
  __shared__ int64_t wsum[kSearchThreads / 64];

  // workgroup -> (row, trial, tile)
  const int64_t b = blockIdx.x;
  int s = 0;
  for (int k = 1; k < tb.n_seg; ++k)
    if (b >= tb.block0[k]) s = k;
  const int64_t n = tb.n_out[s];
  const int64_t n_tiles = (n + kSearchTile - 1) / kSearchTile;
  const int64_t local = b - tb.block0[s];
  const int trial = (int)(local / n_tiles);
  const int64_t tile = local - (int64_t)trial * n_tiles;
  const int g = tb.trial0[s] + trial;
  const double mu = musig[2 * g], sigma = musig[2 * g + 1];
  if (!(sigma > 0.0)) return;
  const int32_t *x = dmt + tb.offset[s] + (int64_t)trial * n;
  const int64_t e0 = tile * kSearchTile;
  const int64_t e1 = min(e0 + (int64_t)kSearchTile, n);
  const int64_t lo = max((int64_t)0, e0 - (int64_t)(wmax - 1));
  const int m = (int)(e1 - lo);  // samples loaded; Q has m + 1 entries

  // ---- exact prefix sums of x[lo .. e1) : Q[0] = 0, Q[k+1] = Q[k] + x[lo+k] ----
  // coalesced load into Q[1..m], then each thread scans a contiguous segment
  for (int k = threadIdx.x; k < m; k += kSearchThreads) Q[k + 1] = x[lo + k];
  __syncthreads();
  const int per = (m + kSearchThreads - 1) / kSearchThreads;
  const int k0 = threadIdx.x * per;
  int64_t run = 0;
  for (int k = k0; k < min(k0 + per, m); ++k) run += Q[k + 1];
  // inclusive scan of the per-thread sums: wave scan then across waves
  int64_t incl = run;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int64_t before = 0;
  for (int w = 0; w < wv; ++w) before += wsum[w];
  int64_t acc = before + incl - run;  // exclusive prefix of this thread's segment
  if (threadIdx.x == 0) Q[0] = 0;
  for (int k = k0; k < min(k0 + per, m); ++k) {
    acc += Q[k + 1];
    Q[k + 1] = acc;
  }
  __syncthreads();

  // ---- best SNR over widths for every box end ----
  const double thr = (double)thr_f;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kSearchThreads) {
    double bsnr = 0.0;
    int32_t bwid = 0;
    const int64_t qe = Q[e + 1 - lo];
    for (int k = 0; k < nw; ++k) {
      const int64_t w = widths[k];
      if (w > e + 1) break;  // box would start before sample 0
      const double sum = (double)(qe - Q[e + 1 - w - lo]);
      const double snr = (sum - (double)w * mu) / (sigma * sqrt((double)w));
      if (bwid == 0 || snr > bsnr) {
        bsnr = snr;
        bwid = (int32_t)w;
      }
    }
    const int el = (int)(e - e0);
    best[el] = bsnr;
    bw[el] = (bwid != 0 && bsnr >= thr) ? bwid : 0;  // 0 = not flagged
  }
  __syncthreads();

  // ---- maximal runs inside the tile ----
  const int len = (int)(e1 - e0);
  for (int el = threadIdx.x; el < len; el += kSearchThreads) {
    if (bw[el] == 0) continue;
    if (el > 0 && bw[el - 1] != 0) continue;  // not a run start
    int pk = el;
    double ps = best[el];
    int k = el + 1;
    for (; k < len && bw[k] != 0; ++k)
      if (best[k] > ps) {
        ps = best[k];
        pk = k;
      }
    const unsigned long long idx = atomicAdd(counter, 1ull);
    if ((int64_t)idx < cap) {
      Frag f;
      f.trial = g;
      f.width = bw[pk];
      f.t_first = e0 + el;
      f.t_last = e0 + k - 1;
      f.e_peak = e0 + pk;
      f.snr = ps;
      f.open_left = (el == 0 && e0 > 0) ? 1 : 0;
      f.open_right = (k == len && e1 < n) ? 1 : 0;
      frags[idx] = f;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void launch_stats(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, hipStream_t st) {
  ctx->stats.device = ctx->device;
  ctx->stats.reserve((size_t)desc->n_trials * 2 * sizeof(double));
  SegTable tb = make_table(desc);
  // bytes: the int32 DM-time array read once
  ProfScope prof(ctx, "stats", st, 4.0 * (double)desc->total);
  hipLaunchKernelGGL(k_stats, dim3(desc->n_trials), dim3(kStatsThreads), 0, st, dmt, tb, ctx->stats.as<double>());
  check_hip(hipGetLastError(), "launch statistics kernel");
}

const double *stats_musig(gsp_ctx *ctx, const gsp_dmt_desc *) { return ctx->stats.as<double>(); }

void launch_search(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, const int32_t *widths_dev,
                   int32_t n_widths, int32_t max_width, float thr, Frag *frags, int64_t cap,
                   unsigned long long *counter, hipStream_t st) {
  SegTable tb = make_table(desc);
  int64_t nb = 0;
  for (int s = 0; s < desc->n_seg; ++s) {
    tb.block0[s] = nb;
    nb += (int64_t)desc->seg[s].n_dm * ((desc->n_out[s] + kSearchTile - 1) / kSearchTile);
  }
  tb.block0[desc->n_seg] = nb;
  if (nb >= (1LL << 31)) fail(GSP_EOVERFLOW, "too many search workgroups");
  const size_t lds = sizeof(int64_t) * (size_t)(kSearchTile + max_width + 1) + sizeof(double) * kSearchTile +
                     sizeof(int32_t) * kSearchTile;
  check_hip(hipFuncSetAttribute((const void *)k_search, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
            "set search LDS size");
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, counter);
  // bytes: the int32 DM-time array read once (look-back overlap not counted)
  ProfScope prof(ctx, "search", st, 4.0 * (double)desc->total);
  hipLaunchKernelGGL(k_search, dim3((unsigned)nb), dim3(kSearchThreads), lds, st, dmt, tb, stats_musig(ctx, desc),
                     widths_dev, n_widths, max_width, thr, frags, cap, counter);
  check_hip(hipGetLastError(), "launch search kernel");
}

}  // namespace gsp
