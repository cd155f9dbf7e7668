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

__global__ void k_zero_counter(unsigned long long *c) { *c = 0ull; }

struct SearchArgs {
  const int32_t *dmt;
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
__global__ __launch_bounds__(kSearchThreads) void k_search(SearchArgs a, SegTable tb) {
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

  // workgroup -> (row, trial, tile)
  const int64_t b = blockIdx.x;
  int s = 0;
  for (int k = 1; k < tb.n_seg; ++k)
    if (b >= tb.block0[k]) s = k;
  const int64_t n = tb.n_out[s];
  const int64_t n_tiles = (n + a.tile - 1) / a.tile;
  const int64_t local = b - tb.block0[s];
  const int trial = (int)(local / n_tiles);
  const int64_t tile = local - (int64_t)trial * n_tiles;
  const int g = tb.trial0[s] + trial;
  const double mu = a.musig[2 * g], sigma = a.musig[2 * g + 1];
  if (!(sigma > 0.0)) return;
  const int32_t *x = a.dmt + tb.offset[s] + (int64_t)trial * n;
  const int64_t e0 = tile * a.tile;
  const int64_t e1 = min(e0 + (int64_t)a.tile, n);
  const int64_t lo = max((int64_t)0, e0 - (int64_t)(a.wmax - 1));
  const int m = (int)(e1 - lo);  // samples; Q has m + 1 entries, m <= kSpan

  // widths and the integer prefilter bounds: a box can reach the threshold
  // only if its sum is >= w mu + thr sigma sqrt(w); lim sits 2 below that
  // bound (far more than its double rounding), so every box end the exact
  // test flags passes the prefilter
  const double thr = (double)a.thr;
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
  const int len = (int)(e1 - e0);
  const int J = a.tile / kSearchThreads;  // box ends per thread (<= PER)
  const bool full = (e0 >= a.wmax - 1) && (len == a.tile);  // every width valid at every box end
  int64_t qe[PER];
  uint32_t maybe = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (j < J) qe[j] = Q[qp((int)(min(e0 + tid + j * kSearchThreads, e1 - 1) + 1 - lo))];
  if (full) {
    for (int k = 0; k < a.nw; ++k) {
      const int w = wsh[k];
      const int64_t L = lim[k];
#pragma unroll
      for (int j = 0; j < PER; ++j)
        if (j < J && qe[j] - Q[qp((int)(e0 + tid + j * kSearchThreads + 1 - w - lo))] >= L) maybe |= 1u << j;
    }
  } else {
    for (int k = 0; k < a.nw; ++k) {
      const int64_t w = wsh[k];
      const int64_t L = lim[k];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int64_t e = e0 + tid + j * kSearchThreads;
        if (j < J && e < e1 && w <= e + 1 && qe[j] - Q[qp((int)(e + 1 - w - lo))] >= L) maybe |= 1u << j;
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
        if (w > e + 1) break;  // box would start before sample 0
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
    if (j < J && el < len) {
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
      f.t_first = e0 + el;
      f.t_last = e0 + kk - 1;
      f.e_peak = e0 + pk;
      f.snr = ps;
      f.open_left = (el == 0 && e0 > 0) ? 1 : 0;
      f.open_right = (kk == len && e1 < n) ? 1 : 0;
      a.frags[idx] = f;
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
  // samples per workgroup = 256 * PER; the look-back of (max width - 1)
  // samples is taken from that budget, the rest are box ends
  const int per = max_width <= 2049 ? 16 : 32;
  const int span = kSearchThreads * per;
  const int look = (max_width - 1 + kSearchThreads - 1) / kSearchThreads * kSearchThreads;
  const int tile = span - look;
  if (tile < kSearchThreads) fail(GSP_EINVAL, "widths too large for the search tile");
  int64_t nb = 0;
  for (int s = 0; s < desc->n_seg; ++s) {
    tb.block0[s] = nb;
    nb += (int64_t)desc->seg[s].n_dm * ((desc->n_out[s] + tile - 1) / tile);
  }
  tb.block0[desc->n_seg] = nb;
  if (nb >= (1LL << 31)) fail(GSP_EOVERFLOW, "too many search workgroups");
  SearchArgs a;
  a.dmt = dmt;
  a.musig = stats_musig(ctx, desc);
  a.widths = widths_dev;
  a.nw = n_widths;
  a.wmax = max_width;
  a.tile = tile;
  a.thr = thr;
  a.frags = frags;
  a.cap = cap;
  a.counter = counter;
  const size_t lds = sizeof(int64_t) * (size_t)(span + span / 16 + 2) + (size_t)span;
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, counter);
  // bytes: the int32 DM-time array read once (look-back overlap not counted)
  ProfScope prof(ctx, "search", st, 4.0 * (double)desc->total);
  if (per == 16) {
    check_hip(hipFuncSetAttribute((const void *)k_search<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "set search LDS size");
    hipLaunchKernelGGL(k_search<16>, dim3((unsigned)nb), dim3(kSearchThreads), lds, st, a, tb);
  } else {
    check_hip(hipFuncSetAttribute((const void *)k_search<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "set search LDS size");
    hipLaunchKernelGGL(k_search<32>, dim3((unsigned)nb), dim3(kSearchThreads), lds, st, a, tb);
  }
  check_hip(hipGetLastError(), "launch search kernel");
}

}  // namespace gsp
