// Single-pulse search over dedispersed series: per-trial statistics and the
// boxcar matched filter with run extraction.
//
// The paper names a single-pulse search stage (Section 2.1) without giving its
// statistic.  The one computed here (documented in gsp.h): population mean and
// sigma of each trial's series from exact integer moments; for every box end
// e and width w, snr = (box sum - w mu) / (sigma sqrt(w)); best over widths;
// one candidate per maximal run of best >= threshold.
//
// The kernels work on a table of series jobs.  A job is the n_dm trials of
// one plan row: either a whole dedispersed row (batch search) or one
// streaming window whose boxes may reach back into retained samples of the
// previous window (a look-back region in front of the window).  Both kernels
// stride over their work items, so the same code serves the per-call batch
// launches (one item per workgroup) and the fixed-grid launches of the
// streaming graph.
//
// Both are HBM-bound streaming passes over the int32 DM-time data:
//  k_stats  one workgroup per trial, 8 loads in flight per lane, 128-bit
//           integer moment sums, mu and sigma finished in double;
//  k_search one workgroup per (trial, tile of box ends): tile plus look-back
//           loaded once, exact int64 prefix sums in LDS, an integer prefilter
//           per width, exact double SNRs only where a box can pass, and run
//           fragments appended with one atomic each (joined on the host).
#include <algorithm>
#include <vector>

#include "gsp_internal.h"

namespace gsp {

__device__ __forceinline__ int find_job_by_trial(const SeriesTable *t, int g) {
  int lo = 0, hi = t->n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t->job[mid].trial0 <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_job_by_item(const SeriesTable *t, int64_t b) {
  int lo = 0, hi = t->n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t->job[mid].block0 <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// statistics
// ---------------------------------------------------------------------------
static constexpr int kStatsThreads = 256;

__global__ __launch_bounds__(kStatsThreads) void k_stats(const SeriesTable *__restrict__ tb,
                                                          double *__restrict__ musig) {
  __shared__ int64_t r1[kStatsThreads];
  __shared__ unsigned __int128 r2[kStatsThreads];
  const int n_trials = tb->n_trials;
  for (int g = blockIdx.x; g < n_trials; g += gridDim.x) {
    const SeriesJob &J = tb->job[find_job_by_trial(tb, g)];
    const int64_t n = J.n;
    const int32_t *x = J.x + (int64_t)(g - J.trial0) * J.pitch + J.e_begin;
    const int64_t x0 = n > 0 ? x[0] : 0;
    int64_t s1 = 0;
    unsigned __int128 s2 = 0;
    auto add = [&](int32_t xv) {
      const int64_t v = (int64_t)xv - x0;
      s1 += v;
      const uint64_t a = (uint64_t)(v < 0 ? -v : v);
      s2 += (unsigned __int128)(a * a);
    };
    constexpr int kU = 8;  // loads in flight per thread
    int64_t k = threadIdx.x;
    for (; k + (kU - 1) * kStatsThreads < n; k += kU * kStatsThreads) {
      int32_t v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = x[k + u * kStatsThreads];
#pragma unroll
      for (int u = 0; u < kU; ++u) add(v[u]);
    }
    for (; k < n; k += kStatsThreads) add(x[k]);
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
      if (n > 0) {
        const double dn = (double)n;
        const double m1 = (double)r1[0] / dn;
        const double m2 = (double)r2[0] / dn;
        const double var = m2 - m1 * m1;
        musig[2 * g] = (double)x0 + m1;
        musig[2 * g + 1] = var > 0.0 ? sqrt(var) : 0.0;
      } else {
        musig[2 * g] = 0.0;
        musig[2 * g + 1] = 0.0;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// boxcar search
// ---------------------------------------------------------------------------
static constexpr int kSearchThreads = 256;

__global__ void k_zero_counter(unsigned long long *c) { *c = 0ull; }

struct SearchArgs {
  const SeriesTable *tb;
  const double *musig;
  const int32_t *widths;  // sorted, unique
  int32_t nw, wmax;
  int32_t tile;           // box ends per workgroup (multiple of kSearchThreads)
  float thr;
  Frag *frags;
  int64_t cap;
  unsigned long long *counter;
};

// Padded LDS index of prefix entry k: one spare slot every 16 entries, so
// that a thread scanning 16 contiguous entries and its neighbours (16 apart)
// hit different banks.
__device__ __forceinline__ int qp(int k) { return k + (k >> 4); }

template <int PER>
__global__ __launch_bounds__(kSearchThreads) void k_search(SearchArgs a) {
  static_assert(PER % 16 == 0, "segments of 16 entries");
  // LDS: prefix sums Q (padded), reused for the per-box-end best SNR once the
  // sums are no longer needed; flags hold 1 + index of the best width
  extern __shared__ int64_t Q[];
  constexpr int kSpan = kSearchThreads * PER;
  uint8_t *flag = reinterpret_cast<uint8_t *>(Q + kSpan + kSpan / 16 + 2);
  double *best = reinterpret_cast<double *>(Q);
  __shared__ int64_t wsum[kSearchThreads / 64];
  __shared__ int64_t lim[64];
  __shared__ int32_t wsh[64];
  const int tid = threadIdx.x;
  const SeriesTable *tb = a.tb;
  const int64_t n_items = tb->n_items;
  const double thr = (double)a.thr;

  for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
    const SeriesJob &J = tb->job[find_job_by_item(tb, b)];
    const int64_t n = J.n;
    const int64_t local = b - J.block0;
    const int trial = (int)(local / J.tiles);
    const int64_t tile = local - (int64_t)trial * J.tiles;
    const int g = J.trial0 + trial;
    const double mu = a.musig[2 * g], sigma = a.musig[2 * g + 1];
    if (!(sigma > 0.0)) continue;  // uniform: the whole workgroup skips
    // positions relative to the window's first box end
    const int32_t *x = J.x + (int64_t)trial * J.pitch + J.e_begin;
    const int64_t e0 = tile * a.tile;
    const int64_t e1 = min(e0 + (int64_t)a.tile, n);
    const int64_t lo = max(-J.look, e0 - (int64_t)(a.wmax - 1));  // may be negative (look-back)
    const int m = (int)(e1 - lo);  // samples; Q has m + 1 entries, m <= kSpan

    // widths and the integer prefilter bounds: a box can reach the
    // threshold only if its sum is >= w mu + thr sigma sqrt(w); lim sits 2
    // below that bound (far more than its double rounding), so every box end
    // the exact test flags passes the prefilter
    if (tid < a.nw) {
      const int32_t w = a.widths[tid];
      wsh[tid] = w;
      const double wd = (double)w;
      const double bound = wd * mu + thr * sigma * sqrt(wd);
      lim[tid] = bound < -4.0e18 ? INT64_MIN : (bound > 4.0e18 ? INT64_MAX : (int64_t)floor(bound) - 2);
    }

    // ---- coalesced load: entry k+1 <- x[lo + k] ----
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = tid + i * kSearchThreads;
      if (k < m) Q[qp(k + 1)] = (int64_t)x[lo + k];
    }
    if (tid == 0) Q[0] = 0;
    __syncthreads();
    // ---- exact prefix sums: each thread scans PER contiguous entries ----
    const int k0 = tid * PER + 1;
    int64_t run = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (k0 + i <= m) run += Q[qp(k0 + i)];
    int64_t incl = run;
    const int lane = tid & 63, wv = tid >> 6;
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(incl, d, 64);
      if (lane >= d) incl += o;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int64_t acc = incl - run;
    for (int w = 0; w < wv; ++w) acc += wsum[w];
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (k0 + i <= m) {
        acc += Q[qp(k0 + i)];
        Q[qp(k0 + i)] = acc;
      }
    __syncthreads();

    // ---- prefilter (integer compares), then exact SNR where it passes ----
    // box end e (relative) uses Q[e + 1 - lo] - Q[e + 1 - w - lo]; the box
    // must start at or after -look
    const int len = (int)(e1 - e0);
    const int Jn = a.tile / kSearchThreads;  // box ends per thread (<= PER)
    const bool full = (e0 + J.look >= a.wmax - 1) && (len == a.tile);
    int64_t qe[PER];
    uint32_t maybe = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if (j < Jn) qe[j] = Q[qp((int)(min(e0 + tid + j * kSearchThreads, e1 - 1) + 1 - lo))];
    if (full) {
      for (int k = 0; k < a.nw; ++k) {
        const int w = wsh[k];
        const int64_t L = lim[k];
#pragma unroll
        for (int j = 0; j < PER; ++j)
          if (j < Jn && qe[j] - Q[qp((int)(e0 + tid + j * kSearchThreads + 1 - w - lo))] >= L) maybe |= 1u << j;
      }
    } else {
      for (int k = 0; k < a.nw; ++k) {
        const int64_t w = wsh[k];
        const int64_t L = lim[k];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const int64_t e = e0 + tid + j * kSearchThreads;
          if (j < Jn && e < e1 && w <= e + J.look + 1 && qe[j] - Q[qp((int)(e + 1 - w - lo))] >= L)
            maybe |= 1u << j;
        }
      }
    }
    // exact best over widths for the box ends that passed (rare): kept in
    // registers until the prefix sums are dead, then stored over them
    double bs[PER];
    uint32_t bk[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      bs[j] = 0.0;
      bk[j] = 0;
    }
    if (maybe) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        if (!(maybe & (1u << j))) continue;
        const int64_t e = e0 + tid + j * kSearchThreads;
        const int64_t q1 = Q[qp((int)(e + 1 - lo))];
        double bb = 0.0;
        uint32_t kb = 0;
        for (int k = 0; k < a.nw; ++k) {
          const int64_t w = wsh[k];
          if (w > e + J.look + 1) break;  // box would start before the first valid sample
          const double sum = (double)(q1 - Q[qp((int)(e + 1 - w - lo))]);
          const double snr = (sum - (double)w * mu) / (sigma * sqrt((double)w));
          if (kb == 0 || snr > bb) {
            bb = snr;
            kb = (uint32_t)k + 1;
          }
        }
        bs[j] = bb;
        bk[j] = (kb != 0 && bb >= thr) ? kb : 0;
      }
    }
    __syncthreads();  // prefix sums dead from here on
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int el = tid + j * kSearchThreads;
      if (j < Jn && el < len) {
        flag[el] = (uint8_t)bk[j];
        if (bk[j]) best[el] = bs[j];
      }
    }
    __syncthreads();

    // ---- maximal runs inside the tile (argmax ties -> earlier box end) ----
    for (int el = tid; el < len; el += kSearchThreads) {
      if (!flag[el]) continue;
      if (el > 0 && flag[el - 1]) continue;  // not a run start
      int pk = el;
      double ps = best[el];
      int kk = el + 1;
      for (; kk < len && flag[kk]; ++kk)
        if (best[kk] > ps) {
          ps = best[kk];
          pk = kk;
        }
      const unsigned long long idx = atomicAdd(a.counter, 1ull);
      if ((int64_t)idx < a.cap) {
        Frag f;
        f.trial = g;
        f.width = wsh[flag[pk] - 1];
        f.t_first = J.abs0 + e0 + el;
        f.t_last = J.abs0 + e0 + kk - 1;
        f.e_peak = J.abs0 + e0 + pk;
        f.snr = ps;
        f.open_left = (el == 0 && e0 > 0) ? 1 : 0;
        f.open_right = (kk == len && e1 < n) ? 1 : 0;
        a.frags[idx] = f;
      }
    }
    __syncthreads();  // LDS reused by the next item
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void set_search_attributes(const SearchTiling &tl) {
  const void *k = tl.per == 16 ? (const void *)k_search<16> : (const void *)k_search<32>;
  check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl.lds), "set search LDS size");
}

SearchTiling search_tiling(int32_t max_width) {
  SearchTiling t;
  t.per = max_width <= 2049 ? 16 : 32;
  const int span = kSearchThreads * t.per;
  const int look = (max_width - 1 + kSearchThreads - 1) / kSearchThreads * kSearchThreads;
  t.tile = span - look;
  if (t.tile < kSearchThreads) fail(GSP_EINVAL, "widths too large for the search tile");
  t.lds = sizeof(int64_t) * (size_t)(span + span / 16 + 2) + (size_t)span;
  return t;
}

void finalize_table(SeriesTable &t, const SearchTiling &tl) {
  int64_t nb = 0;
  int32_t trials = 0;
  for (int j = 0; j < t.n_jobs; ++j) {
    SeriesJob &J = t.job[j];
    J.tiles = (J.n + tl.tile - 1) / tl.tile;
    J.block0 = nb;
    J.trial0 = trials;
    nb += (int64_t)J.n_dm * J.tiles;
    trials += J.n_dm;
  }
  t.n_items = nb;
  t.n_trials = trials;
}

void launch_stats_table(gsp_ctx *ctx, const SeriesTable *tb_dev, int64_t grid, double *musig, double bytes,
                        hipStream_t st) {
  if (grid <= 0) return;
  ProfScope prof(ctx, "stats", st, bytes);
  hipLaunchKernelGGL(k_stats, dim3((unsigned)grid), dim3(kStatsThreads), 0, st, tb_dev, musig);
  check_hip(hipGetLastError(), "launch statistics kernel");
}

void launch_search_table(gsp_ctx *ctx, const SeriesTable *tb_dev, int64_t grid, const SearchTiling &tl,
                         const double *musig, const int32_t *widths_dev, int32_t n_widths, int32_t max_width,
                         float thr, Frag *frags, int64_t cap, unsigned long long *counter, double bytes,
                         hipStream_t st) {
  SearchArgs a;
  a.tb = tb_dev;
  a.musig = musig;
  a.widths = widths_dev;
  a.nw = n_widths;
  a.wmax = max_width;
  a.tile = tl.tile;
  a.thr = thr;
  a.frags = frags;
  a.cap = cap;
  a.counter = counter;
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, counter);
  if (grid <= 0) return;
  if (grid >= (1LL << 31)) fail(GSP_EOVERFLOW, "too many search workgroups");
  ProfScope prof(ctx, "search", st, bytes);
  if (tl.per == 16)
    hipLaunchKernelGGL(k_search<16>, dim3((unsigned)grid), dim3(kSearchThreads), tl.lds, st, a);
  else
    hipLaunchKernelGGL(k_search<32>, dim3((unsigned)grid), dim3(kSearchThreads), tl.lds, st, a);
  check_hip(hipGetLastError(), "launch search kernel");
}

// Batch: one job per plan row over the whole dedispersed output.
static void batch_table(const gsp_dmt_desc *desc, const int32_t *dmt, SeriesTable &t) {
  t.n_jobs = desc->n_seg;
  for (int s = 0; s < desc->n_seg; ++s) {
    SeriesJob &J = t.job[s];
    J.x = dmt + desc->offset[s];
    J.pitch = desc->n_out[s];
    J.e_begin = 0;
    J.n = desc->n_out[s];
    J.look = 0;
    J.abs0 = 0;
    J.n_dm = desc->seg[s].n_dm;
  }
}

static SeriesTable *upload_table(gsp_ctx *ctx, const SeriesTable &t, hipStream_t st) {
  ctx->jobs.device = ctx->device;
  ctx->jobs.reserve(sizeof(SeriesTable));
  *ctx->jobs_host = t;
  check_hip(hipMemcpyAsync(ctx->jobs.ptr, ctx->jobs_host.get(), sizeof(SeriesTable), hipMemcpyHostToDevice, st),
            "copy job table");
  return ctx->jobs.as<SeriesTable>();
}

void launch_stats(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, hipStream_t st) {
  ctx->stats.device = ctx->device;
  ctx->stats.reserve((size_t)desc->n_trials * 2 * sizeof(double));
  SeriesTable t;
  batch_table(desc, dmt, t);
  finalize_table(t, search_tiling(1));
  SeriesTable *d = upload_table(ctx, t, st);
  // bytes: the int32 DM-time array read once
  launch_stats_table(ctx, d, t.n_trials, ctx->stats.as<double>(), 4.0 * (double)desc->total, st);
}

const double *stats_musig(gsp_ctx *ctx, const gsp_dmt_desc *) { return ctx->stats.as<double>(); }

void launch_search(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, const int32_t *widths_dev,
                   int32_t n_widths, int32_t max_width, float thr, Frag *frags, int64_t cap,
                   unsigned long long *counter, hipStream_t st) {
  const SearchTiling tl = search_tiling(max_width);
  SeriesTable t;
  batch_table(desc, dmt, t);
  finalize_table(t, tl);
  SeriesTable *d = upload_table(ctx, t, st);
  set_search_attributes(tl);
  // bytes: the int32 DM-time array read once (look-back overlap not counted)
  launch_search_table(ctx, d, t.n_items, tl, stats_musig(ctx, desc), widths_dev, n_widths, max_width, thr, frags,
                      cap, counter, 4.0 * (double)desc->total, st);
}

}  // namespace gsp
