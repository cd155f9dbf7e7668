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
// launches (one item per workgroup or wave) and the fixed-grid launches of the
// streaming graph.
//
// Both are HBM-bound streaming passes over the int32 DM-time data:
//  k_stats  one workgroup per trial, 8 loads in flight per lane, 128-bit
//           integer moment sums, mu and sigma finished in double;
//  k_search one wave per (trial, segment of box ends): segment plus look-back
//           read once, exact int64 prefix sums by wave scans into a per-wave
//           LDS ring, an integer prefilter per width, exact double SNRs only
//           where a box can pass, and run fragments appended with one atomic
//           each (joined on the host).
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
                                                          double *__restrict__ musig,
                                                          const uint32_t *__restrict__ need) {
  __shared__ int64_t r1[kStatsThreads];
  __shared__ unsigned __int128 r2[kStatsThreads];
  const int n_trials = tb->n_trials;
  for (int g = blockIdx.x; g < n_trials; g += gridDim.x) {
    if (need && need[g] == 0) continue;  // a trial nobody reads: left as it was
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
// One wave owns one item: a trial and a segment [s0, s1) of its box ends.  It
// walks the samples from lo = max(first valid sample, s0 - (w_max - 1)) in
// blocks of 8 x 64: each lane holds one sample per 64-sample step, a wave-wide
// scan (DPP) plus the running carry gives the exact prefix sums C of the
// samples less the trial's integer mean c, and these go into a per-wave LDS
// ring that keeps the last RING of them.  A box (e, w) sums to
// C(e) - C(e - w) + w c.  Per width an integer prefilter flags the box ends
// whose sum can reach the threshold (in 32 bits, on the ring's low halves,
// wherever no sample within a box's reach lies 2^31 / w_max or more from c,
// so that every box's C difference fits; in 64 bits elsewhere); only those
// get the exact double SNR.  Runs of flagged ends are followed across steps and blocks inside the
// wave and written as fragments (one atomic each).  Waves never wait for each
// other: there is no workgroup barrier after the widths are loaded.
static constexpr int kSearchThreads = 256;
static constexpr int kSearchBlock = 512;  // samples per block: 8 steps of 64

__global__ void k_zero_counter(unsigned long long *c) { *c = 0ull; }

struct SearchArgs {
  const SeriesTable *tb;
  const double *musig;
  const int32_t *widths;  // sorted, unique
  int32_t nw, wmax;
  int32_t tile;           // box ends per item
  float thr;
  Frag *frags;
  int64_t cap;
  unsigned long long *counter;
};

// One step of the wave scan: v plus v of the lane CTRL selects (DPP), 0 where
// the row mask or the row boundary gives no source.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int64_t add_dpp(int64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)v >> 32), CTRL, ROW_MASK, 0xf, false);
  return v + (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Inclusive scan of an int64 over the 64 lanes: shifts inside rows of 16,
// then the row totals broadcast to the following rows.
__device__ __forceinline__ int64_t wave_scan_i64(int64_t x) {
  x = add_dpp<0x111, 0xf>(x);  // row_shr:1
  x = add_dpp<0x112, 0xf>(x);  // row_shr:2
  x = add_dpp<0x114, 0xf>(x);  // row_shr:4
  x = add_dpp<0x118, 0xf>(x);  // row_shr:8
  x = add_dpp<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = add_dpp<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Inclusive scan of an int32 over the 64 lanes (same DPP pattern as the
// int64 scan below), for partial sums known to fit.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t add_dpp_i32(int32_t v) {
  return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ int32_t wave_scan_i32(int32_t x) {
  x = add_dpp_i32<0x111, 0xf>(x);
  x = add_dpp_i32<0x112, 0xf>(x);
  x = add_dpp_i32<0x114, 0xf>(x);
  x = add_dpp_i32<0x118, 0xf>(x);
  x = add_dpp_i32<0x142, 0xa>(x);
  x = add_dpp_i32<0x143, 0xc>(x);
  return x;
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t lane63(int64_t v) { return readlane_i64(v, 63); }

// Per-wave LDS: the prefix ring, the step's exact best SNR and width per
// lane, and the open run.
template <int RING>
struct SearchWaveLds {
  int32_t ring_lo[RING], ring_hi[RING];  // the centred prefix sums, low and high halves
  __device__ int64_t get(int j) const {
    return (int64_t)(((uint64_t)(uint32_t)ring_hi[j] << 32) | (uint32_t)ring_lo[j]);
  }
  __device__ void put(int j, int64_t v) {
    ring_lo[j] = (int32_t)(uint32_t)v;
    ring_hi[j] = (int32_t)(uint32_t)((uint64_t)v >> 32);
  }
  double sb[64];
  int32_t sk[64];
  int64_t o_first, o_peak;
  double o_snr;
  int32_t o_k, o_left;
};

// Four waves per SIMD (at most 128 VGPRs): occupancy hides the LDS and
// memory latency better than the registers a lower occupancy would free.
template <int RING>
__global__ __launch_bounds__(kSearchThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_search(SearchArgs a) {
  static_assert((RING & (RING - 1)) == 0, "ring length is a power of two");
  extern __shared__ int64_t lds64[];
  __shared__ int32_t wsh[64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  SearchWaveLds<RING> &W = reinterpret_cast<SearchWaveLds<RING> *>(lds64)[wave];
  const SeriesTable *tb = a.tb;
  const int64_t n_items = tb->n_items;
  const double thr = (double)a.thr;
  const int nw = a.nw;
  if ((int)threadIdx.x < nw) wsh[threadIdx.x] = a.widths[threadIdx.x];
  __syncthreads();  // the only workgroup barrier

  for (int64_t b = (int64_t)blockIdx.x * nwaves + wave; b < n_items; b += (int64_t)gridDim.x * nwaves) {
    const SeriesJob &J = tb->job[find_job_by_item(tb, b)];
    const int64_t n = J.n;
    const int64_t local = b - J.block0;
    const int trial = (int)(local / J.tiles);
    const int64_t seg = local - (int64_t)trial * J.tiles;
    const int g = J.trial0 + trial;
    const double mu = a.musig[2 * g], sigma = a.musig[2 * g + 1];
    // an integer near the mean (any value is exact; near the mean keeps the
    // centred samples small)
    const int64_t cmean = (int64_t)fmin(fmax(rint(mu), -2147483648.0), 2147483647.0);
    if (!(sigma > 0.0)) continue;  // uniform over the wave
    const int32_t *x = J.x + (int64_t)trial * J.pitch + J.e_begin;  // relative positions
    const int64_t look = J.look;
    const int64_t s0 = seg * a.tile;
    const int64_t s1 = min(s0 + (int64_t)a.tile, n);
    const int64_t lo = max(-look, s0 - (int64_t)(a.wmax - 1));
    // every box of every end in [s0, s1) starts at or after the first sample
    const bool full = s0 - (int64_t)(a.wmax - 1) >= -look;

    // prefilter bounds: a box can reach the threshold only if its sum is
    // >= w mu + thr sigma sqrt(w); lim sits 2 below that bound (far more than
    // its double rounding), so every box end the exact test flags passes
    // (lane k holds width k and its bound; the loops below read them with
    // readlane, so they cost no LDS round trip)
    // The bound is kept against the centred sums: C difference >= lim - w c,
    // in 64 bits and, clamped, in 32 (a clamp only lets more ends through).
    int lane_w = 0;
    int64_t lane_lim = INT64_MAX;
    int32_t lane_l32 = INT32_MAX;
    double lane_wmu = 0.0, lane_den = 1.0;  // w mu and sigma sqrt(w), as the exact SNR takes them
    if (lane < nw) {
      lane_w = wsh[lane];
      const double wd = (double)lane_w;
      lane_wmu = wd * mu;
      lane_den = sigma * sqrt(wd);
      const double bound = wd * mu + thr * sigma * sqrt(wd);
      lane_lim = bound < -4.0e18 ? INT64_MIN : (bound > 4.0e18 ? INT64_MAX : (int64_t)floor(bound) - 2);
      if (lane_lim != INT64_MIN && lane_lim != INT64_MAX) lane_lim -= cmean * (int64_t)lane_w;
      lane_l32 = (int32_t)max((int64_t)INT32_MIN, min((int64_t)INT32_MAX, lane_lim));
    }
    // samples this far from c or farther make the 32-bit prefilter unsafe for
    // the boxes that reach them (w_max of them sum to less than 2^31 in size)
    const int64_t big = (int64_t)(0x7FFFFFFF / (uint32_t)a.wmax);
    const int64_t reach_blocks = (a.wmax - 1 + kSearchBlock - 1) / kSearchBlock;
    int64_t last_big = -(reach_blocks + 1);  // the last block holding such a sample
    if (lane == 0) W.put(0, 0);  // C(lo - 1)
    __builtin_amdgcn_wave_barrier();

    bool open = false;
    int64_t o_first = 0, o_peak = 0, o_last = 0;
    double o_snr = 0.0;
    int o_k = 0, o_left = 0;
    auto emit = [&](int64_t t_first, int64_t t_last, int64_t e_peak, double snr, int k, int left, int right) {
      const unsigned long long idx = atomicAdd(a.counter, 1ull);
      if ((int64_t)idx < a.cap) {
        Frag f;
        f.trial = g;
        f.width = wsh[k - 1];
        f.t_first = J.abs0 + t_first;
        f.t_last = J.abs0 + t_last;
        f.e_peak = J.abs0 + e_peak;
        f.snr = snr;
        f.open_left = left;
        f.open_right = right;
        a.frags[idx] = f;
      }
    };

    const int64_t count = s1 - lo;
    const int64_t nblk = (count + kSearchBlock - 1) / kSearchBlock;
    // samples in flight: the next block's 8 per lane (indices clamped into
    // [lo, s1 - 1], so every load stays inside the series)
    int32_t vn[8];
#pragma unroll
    for (int it = 0; it < 8; ++it) vn[it] = x[min(lo + 64 * it + lane, s1 - 1)];
    int64_t carry = 0;
    for (int64_t blk = 0; blk < nblk; ++blk) {
      const int64_t eb = lo + blk * kSearchBlock;  // position of lane 0, step 0
      int32_t v[8];
#pragma unroll
      for (int it = 0; it < 8; ++it) v[it] = vn[it];
      if (blk + 1 < nblk) {
#pragma unroll
        for (int it = 0; it < 8; ++it) vn[it] = x[min(eb + kSearchBlock + 64 * it + lane, s1 - 1)];
      }
      // ---- exact centred prefix sums into the ring ----
      const int r0 = (int)(eb - lo + 1);
      int64_t P[8];  // C at the lane's box end + 1
      bool blk_big = false;
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int64_t e = eb + 64 * it + lane;
        // samples about the trial's integer mean c: when every |x - c| of the
        // step is below 2^25 their 64-lane partial sums fit an int32 scan
        // (positions past the segment count as c, i.e. add nothing)
        const int64_t y = e < s1 ? (int64_t)v[it] - cmean : 0;
        if (__ballot(y <= -(int64_t)(1 << 25) || y >= (int64_t)(1 << 25)) == 0ull)
          P[it] = carry + (int64_t)wave_scan_i32((int32_t)y);
        else
          P[it] = carry + wave_scan_i64(y);
        blk_big |= __ballot(y <= -big || y >= big) != 0ull;
        carry = lane63(P[it]);
        W.put((r0 + 64 * it + lane) & (RING - 1), P[it]);
      }
      if (blk_big) last_big = blk;
      __builtin_amdgcn_wave_barrier();
      if (eb + kSearchBlock - 1 < s0) continue;  // look-back block: sums only

      // ---- integer prefilter, widths outer: per width the 8 ring reads are
      // issued together; each compare leaves a wave mask ----
      uint64_t mk[8];
#pragma unroll
      for (int it = 0; it < 8; ++it) mk[it] = 0;
      if (full && blk - last_big > reach_blocks) {
        // every box of the block sums to less than 2^31 in size about w c:
        // the C differences are exact in 32 bits (the ring's low halves)
        uint32_t p32[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) p32[it] = (uint32_t)P[it];
        for (int k = 0; k < nw; ++k) {
          const int w = __builtin_amdgcn_readlane(lane_w, k);
          const int32_t L = __builtin_amdgcn_readlane(lane_l32, k);
          const int bw = r0 + lane - w;
          uint32_t qv[8];
#pragma unroll
          for (int it = 0; it < 8; ++it) qv[it] = (uint32_t)W.ring_lo[(bw + 64 * it) & (RING - 1)];
#pragma unroll
          for (int it = 0; it < 8; ++it) mk[it] |= __ballot((int32_t)(p32[it] - qv[it]) >= L);
        }
      } else if (full) {
        for (int k = 0; k < nw; ++k) {
          const int w = __builtin_amdgcn_readlane(lane_w, k);
          const int64_t L = readlane_i64(lane_lim, k);
          const int bw = r0 + lane - w;
          int64_t qv[8];
#pragma unroll
          for (int it = 0; it < 8; ++it) qv[it] = W.get((bw + 64 * it) & (RING - 1));
#pragma unroll
          for (int it = 0; it < 8; ++it) mk[it] |= __ballot(P[it] - qv[it] >= L);
        }
      } else {
        for (int k = 0; k < nw; ++k) {
          const int w = __builtin_amdgcn_readlane(lane_w, k);
          const int64_t L = readlane_i64(lane_lim, k);
          const int bw = r0 + lane - w;
          int64_t qv[8];
#pragma unroll
          for (int it = 0; it < 8; ++it) qv[it] = W.get((bw + 64 * it) & (RING - 1));
#pragma unroll
          for (int it = 0; it < 8; ++it)
            mk[it] |= __ballot((P[it] - qv[it] >= L) & ((int64_t)w <= eb + 64 * it + lane + look + 1));
        }
      }
      uint32_t mbits = 0;
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int64_t e = eb + 64 * it + lane;
        mbits |= (uint32_t)(((mk[it] >> lane) & 1ull) & (e >= s0) & (e < s1)) << it;
      }

      // ---- exact SNR and runs, step by step ----
#pragma unroll 1
      for (int it = 0; it < 8; ++it) {
        const int64_t e0 = eb + 64 * it;
        const int64_t e = e0 + lane;
        const bool maybe = (mbits >> it) & 1u;
        if (__ballot(maybe) == 0ull && !open) continue;
        bool fl = false;
        double bs = 0.0;
        int kb = 0;
        if (maybe) {
          const int re = (int)(e - lo + 1);
          const int64_t q1 = W.get(re & (RING - 1));
          // only widths whose integer sum passes the prefilter bound can
          // reach the threshold; when one does, the best width is among them
          // (a width below its bound has an SNR below the threshold), so the
          // others are skipped, for the whole wave when none of its lanes pass
          for (int k = 0; k < nw; ++k) {
            const int w = __builtin_amdgcn_readlane(lane_w, k);
            if ((int64_t)w > e + look + 1) break;  // box would start before the first sample
            const int64_t d = q1 - W.get((re - w) & (RING - 1));  // C difference
            const bool pass = d >= readlane_i64(lane_lim, k);
            if (__ballot(pass) == 0ull) continue;
            const double sum = (double)(d + cmean * (int64_t)w);
            const double wmu = __builtin_bit_cast(double, readlane_i64(__builtin_bit_cast(int64_t, lane_wmu), k));
            const double den = __builtin_bit_cast(double, readlane_i64(__builtin_bit_cast(int64_t, lane_den), k));
            const double snr = (sum - wmu) / den;
            if (pass && (kb == 0 || snr > bs)) {
              bs = snr;
              kb = k + 1;
            }
          }
          fl = kb != 0 && bs >= thr;
        }
        const uint64_t m = __ballot(fl);
        if (open && !(m & 1ull)) {  // the open run ended on the previous step
          if (lane == 0) emit(o_first, o_last, o_peak, o_snr, o_k, o_left, 0);
          open = false;
        }
        if (m == 0ull) continue;
        W.sb[lane] = bs;
        W.sk[lane] = kb;
        __builtin_amdgcn_wave_barrier();
        const bool last_step = e0 + 63 >= s1 - 1;  // the segment's last box end is on this step
        const bool start = fl && (lane == 0 || !((m >> (lane - 1)) & 1ull));
        if (start) {
          int l = lane, pk = lane;
          double ps = bs;
          while (l + 1 < 64 && ((m >> (l + 1)) & 1ull)) {
            ++l;
            const double s = W.sb[l];
            if (s > ps) {  // ties keep the earlier box end
              ps = s;
              pk = l;
            }
          }
          int64_t f_first = e0 + lane, f_peak = e0 + pk;
          double f_snr = ps;
          int f_k = W.sk[pk];
          int f_left = (f_first == s0 && s0 > 0) ? 1 : 0;
          if (lane == 0 && open) {  // continues the open run
            f_first = o_first;
            f_left = o_left;
            if (!(ps > o_snr)) {
              f_peak = o_peak;
              f_snr = o_snr;
              f_k = o_k;
            }
          }
          if (l == 63 && !last_step) {  // still open: hand over to the next step
            W.o_first = f_first;
            W.o_peak = f_peak;
            W.o_snr = f_snr;
            W.o_k = f_k;
            W.o_left = f_left;
          } else {
            const int64_t f_last = e0 + l;
            emit(f_first, f_last, f_peak, f_snr, f_k, f_left, (f_last == s1 - 1 && s1 < n) ? 1 : 0);
          }
        }
        __builtin_amdgcn_wave_barrier();
        open = ((m >> 63) & 1ull) && !last_step;
        if (open) {
          o_first = W.o_first;
          o_peak = W.o_peak;
          o_snr = W.o_snr;
          o_k = W.o_k;
          o_left = W.o_left;
          o_last = e0 + 63;
        }
      }
    }
    if (open && lane == 0) emit(o_first, o_last, o_peak, o_snr, o_k, o_left, (o_last == s1 - 1 && s1 < n) ? 1 : 0);
    __builtin_amdgcn_wave_barrier();  // per-wave LDS reused by the next item
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static const void *search_kernel(int ring) {
  switch (ring) {
    case 1024: return (const void *)k_search<1024>;
    case 2048: return (const void *)k_search<2048>;
    case 4096: return (const void *)k_search<4096>;
    default: return (const void *)k_search<8192>;
  }
}

void set_search_attributes(const SearchTiling &tl) {
  check_hip(hipFuncSetAttribute(search_kernel(tl.ring), hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl.lds),
            "set search LDS size");
}

SearchTiling search_tiling(int32_t max_width) {
  SearchTiling t;
  // the ring holds the sums of one block plus w_max before it
  t.ring = 1024;
  while (t.ring < max_width + kSearchBlock) t.ring *= 2;
  if (t.ring > 8192) fail(GSP_EINVAL, "widths too large for the search ring (at most 7680)");
  size_t per_wave = 0;
  switch (t.ring) {
    case 1024: per_wave = sizeof(SearchWaveLds<1024>); break;
    case 2048: per_wave = sizeof(SearchWaveLds<2048>); break;
    case 4096: per_wave = sizeof(SearchWaveLds<4096>); break;
    default: per_wave = sizeof(SearchWaveLds<8192>); break;
  }
  t.waves = (int)std::max<size_t>(1, std::min<size_t>(kSearchThreads / 64, (size_t)(128 * 1024) / per_wave));
  t.lds = per_wave * (size_t)t.waves;
  // long segments keep the look-back re-read small; at least 16 blocks
  t.tile = std::max(8192, ((max_width - 1) / kSearchBlock + 1) * kSearchBlock * 16);
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
                        hipStream_t st, const uint32_t *need) {
  if (grid <= 0) return;
  ProfScope prof(ctx, "stats", st, bytes);
  hipLaunchKernelGGL(k_stats, dim3((unsigned)grid), dim3(kStatsThreads), 0, st, tb_dev, musig, need);
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
  const dim3 blk((unsigned)(64 * tl.waves));
  switch (tl.ring) {
    case 1024: hipLaunchKernelGGL(k_search<1024>, dim3((unsigned)grid), blk, tl.lds, st, a); break;
    case 2048: hipLaunchKernelGGL(k_search<2048>, dim3((unsigned)grid), blk, tl.lds, st, a); break;
    case 4096: hipLaunchKernelGGL(k_search<4096>, dim3((unsigned)grid), blk, tl.lds, st, a); break;
    default: hipLaunchKernelGGL(k_search<8192>, dim3((unsigned)grid), blk, tl.lds, st, a); break;
  }
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

void launch_stats(gsp_ctx *ctx, const int32_t *dmt, const gsp_dmt_desc *desc, hipStream_t st,
                  const uint32_t *need) {
  ctx->stats.device = ctx->device;
  ctx->stats.reserve((size_t)desc->n_trials * 2 * sizeof(double));
  SeriesTable t;
  batch_table(desc, dmt, t);
  finalize_table(t, search_tiling(1));
  SeriesTable *d = upload_table(ctx, t, st);
  // bytes: the int32 DM-time array read once (the selected trials' rows only
  // when `need` is given; not known on the host then)
  launch_stats_table(ctx, d, t.n_trials, ctx->stats.as<double>(), need ? 0.0 : 4.0 * (double)desc->total, st,
                     need);
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
  launch_search_table(ctx, d, (t.n_items + tl.waves - 1) / tl.waves, tl, stats_musig(ctx, desc), widths_dev, n_widths, max_width, thr, frags,
                      cap, counter, 4.0 * (double)desc->total, st);
}

}  // namespace gsp
