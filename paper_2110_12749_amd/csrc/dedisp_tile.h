// Device code of the dedispersion tile, shared by the batch launch
// (dedisp.hip) and the streaming launch (stream.hip).
#pragma once

#include "gsp_internal.h"

namespace gsp {

struct DedispArgs {
  const void *Y;            // channel-major staged input (uint8 or uint16)
  int64_t pitch;            // elements per channel row of Y
  const uint32_t *addr;     // [nchan][n_dm_pad] LDS dword offsets
  const int32_t *base;      // [n_tiles_dm][nchan] staging start (delay of tile's first trial, /4*4)
  void *out;                // OutT out[i * out_pitch + (t - t_lo)] for t in [t_lo, t_hi)
  int64_t out_pitch;
  int64_t t_origin;         // absolute output index of tile 0's first sample (multiple of 4)
  int64_t t_lo, t_hi;       // outputs stored
  int64_t ring;             // staged samples per channel in a ring (0: linear copy)
  int64_t phys0;            // position of sample t_origin in the staged row (multiple of 4)
  int32_t n_dm, n_dm_pad, nchan;
  // staging passes: pass k covers channels [chunks[2k], chunks[2k+2]) with
  // chunks[2k+1] dwords per staged copy of a channel (a multiple of 8);
  // chunks[2 n_chunks] = nchan
  const int32_t *chunks;
  int32_t n_chunks;
  int32_t max_chunk;        // most channels in one pass
  int32_t data_dw;          // LDS dwords of the largest pass's staged copies
  int32_t flush;            // channels between flushes of the 16-bit lanes
  int32_t n_dm_tiles, n_t_tiles;
  // output segments (0: none): the sums of channels [s*seg_ch, (s+1)*seg_ch)
  // go to out + s*seg_stride (elements), each segment's sums starting from
  // zero; passes never straddle a segment boundary
  int32_t seg_ch;
  int64_t seg_stride;
};

__device__ __forceinline__ int xcd_remap(int b, int G) {
  // hardware dispatches workgroup b to XCD b % 8; give each XCD a contiguous
  // range of logical tiles
  const int q = G >> 3, r = G & 7;
  const int x = b & 7, k = b >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Staging unit: 16 consecutive samples of one channel, i.e. 8 dwords of each
// LDS copy.  Per pass each thread stages at most unit_max units (uint8
// sources: 3; uint16 sources, 9 registers a unit: 2, which keeps 4 waves per
// SIMD).  Longer passes mean fewer workgroup barriers per channel.  The trial
// offsets of a pass live in registers, one channel per lane, so a pass has
// at most kPassMax channels.
template <typename SrcT>
constexpr int unit_max() { return sizeof(SrcT) == 1 ? 3 : 2; }
constexpr int unit_max_for_d(int D) { return D == 1 ? 3 : 2; }
static constexpr int kPassMax = 64;

template <typename SrcT>
struct Unit {
  static constexpr int W = 16 / (4 / sizeof(SrcT));  // source dwords holding 16 samples
  uint32_t w[W];
  uint32_t tail;  // sample 16 (needed by the shifted copy)
};

// One tile: trials [dm_tile*MT, +MT) x outputs t0 + [0, 128*K) with
// t0 = t_origin + t_tile * 128*K.  Every thread of the workgroup calls it.
// OutT: int32_t, or uint16_t where every sum is known to fit 16 bits (the
// sub-band series of sub-band dedispersion).
// SEG: the sums go to output segments of a.seg_ch channels (the sub-band
// series of sub-band dedispersion); without it a.seg_ch is ignored.
template <int K, int TPW, typename SrcT, typename OutT = int32_t, bool SEG = false>
__device__ __forceinline__ void dedisp_tile(const DedispArgs &a, int dm_tile, int t_tile, uint32_t *lds) {
  static_assert(TPW % 4 == 0, "offsets are read four trials at a time");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x;
  const int nwaves = nthreads >> 6;
  constexpr int T = 128 * K;
  const int64_t t_rel = (int64_t)t_tile * T;  // tile start relative to t_origin
  const int64_t t0 = a.t_origin + t_rel;
  const int MT = TPW * nwaves;
  const int i_tile = dm_tile * MT;
  const int n_chunks = a.n_chunks;
  const int maxc = a.max_chunk;
  // LDS: samples [pass channels][2][row dwords] | staging bases [2][max_chunk]
  uint32_t *data = lds;
  int32_t *bases = reinterpret_cast<int32_t *>(lds + a.data_dw);
  const int i_wave = i_tile + wave * TPW;  // this wave's first trial
  // the pass table is read 64 passes at a time into one register per lane
  // (lane l: pass w0 + l) and taken with readlane, so no scalar load (whose
  // wait would also drain the LDS queue) sits in the pass loop
  int w0 = 0;
  int32_t win_cs = 0, win_rd = 0;
  auto fetch_window = [&](int from) {
    w0 = from;
    const int j = from + lane;
    win_cs = j <= n_chunks ? a.chunks[2 * j] : a.nchan;
    win_rd = j < n_chunks ? a.chunks[2 * j + 1] : 8;
  };
  auto ch_begin = [&](int j) { return __builtin_amdgcn_readlane(win_cs, j - w0); };
  auto row_dw_of = [&](int j) { return __builtin_amdgcn_readlane(win_rd, j - w0); };
  fetch_window(0);

  const SrcT *Y = static_cast<const SrcT *>(a.Y);
  const int32_t *base_row = a.base + (int64_t)dm_tile * a.nchan;

  // ---- staging helpers ----
  Unit<SrcT> pu[unit_max<SrcT>()];
  // trial offsets of the wave's TPW trials: lane l holds channel l of the
  // pass (roff: the pass being summed, noff: the next one, in flight); the
  // sums read them with readlane, so they cost no LDS traffic
  uint32_t roff[TPW], noff[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) noff[j] = 0;
  auto prefetch = [&](int j) {  // global -> registers for pass j (bases of j already in LDS)
    const int cs = ch_begin(j), ce = ch_begin(j + 1);
    const int U = row_dw_of(j) >> 3;  // staging units per channel
    const int nu = (ce - cs) * U;
    const int32_t *bj = bases + (j & 1) * maxc;
    // all addresses first, then all loads, so every load is issued back to back
    const SrcT *rows[unit_max<SrcT>()];
#pragma unroll
    for (int i = 0; i < unit_max<SrcT>(); ++i) {
      const int u = min(tid + i * nthreads, nu - 1);  // clamped: loads stay in bounds
      const int cl = u / U;
      const int p = u - cl * U;
      int64_t e0 = t0 + bj[cl] + 16 * (int64_t)p;  // multiple of 4
      if (a.ring)  // ring position; the 17 samples read may run into the mirrored guard
        e0 = (uint32_t)(t_rel + bj[cl] + 16 * p + a.phys0) % (uint32_t)a.ring;
      rows[i] = Y + (int64_t)(cs + cl) * a.pitch + e0;
    }
#pragma unroll
    for (int i = 0; i < unit_max<SrcT>(); ++i) {
      const uint32_t *w = reinterpret_cast<const uint32_t *>(rows[i]);
#pragma unroll
      for (int m = 0; m < Unit<SrcT>::W; ++m) pu[i].w[m] = w[m];
      pu[i].tail = rows[i][16];
    }
    {
      // offsets of the wave's trials at channel cs + lane (clamped into the pass)
      const uint32_t *src = a.addr + (int64_t)(cs + min(lane, ce - cs - 1)) * a.n_dm_pad + i_wave;
#pragma unroll
      for (int j = 0; j < TPW; j += 4) {
        const uint4 q = *reinterpret_cast<const uint4 *>(src + j);
        noff[j] = q.x;
        noff[j + 1] = q.y;
        noff[j + 2] = q.z;
        noff[j + 3] = q.w;
      }
    }
  };
  auto store = [&](int j) {  // registers -> LDS for pass j
    const int cs = ch_begin(j), ce = ch_begin(j + 1);
    const int row_dw = row_dw_of(j);
    const int U = row_dw >> 3;
    const int nu = (ce - cs) * U;
#pragma unroll
    for (int i = 0; i < unit_max<SrcT>(); ++i) {
      const int u = tid + i * nthreads;
      if (u < nu) {
        const int cl = u / U;
        const int p = u - cl * U;
        uint32_t c0[8], c1[8];
        if constexpr (sizeof(SrcT) == 1) {
          // samples y0..y15 in 4 dwords, y16 in tail; each 16-bit pair is one
          // byte permute (selector byte k < 4: byte k of the second operand,
          // 4..7: byte k-4 of the first, 0x0c: zero)
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const uint32_t w = pu[i].w[m >> 1];
            const uint32_t wn = (m >> 1) + 1 < 4 ? pu[i].w[(m >> 1) + 1] : pu[i].tail;
            if (m & 1) {
              c0[m] = __builtin_amdgcn_perm(0u, w, 0x0C030C02u);  // (y[2m], y[2m+1]) = bytes 2, 3
              c1[m] = __builtin_amdgcn_perm(wn, w, 0x0C040C03u);  // byte 3 of w, byte 0 of wn
            } else {
              c0[m] = __builtin_amdgcn_perm(0u, w, 0x0C010C00u);  // bytes 0, 1
              c1[m] = __builtin_amdgcn_perm(0u, w, 0x0C020C01u);  // bytes 1, 2
            }
          }
        } else {
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const uint32_t w = pu[i].w[m];
            const uint32_t nxt = m + 1 < 8 ? (pu[i].w[m + 1] & 0xFFFFu) : (pu[i].tail & 0xFFFFu);
            c0[m] = w;
            c1[m] = (w >> 16) | (nxt << 16);
          }
        }
        uint4 *d0 = reinterpret_cast<uint4 *>(data + (cl * 2) * row_dw + 8 * p);
        uint4 *d1 = reinterpret_cast<uint4 *>(data + (cl * 2 + 1) * row_dw + 8 * p);
        d0[0] = make_uint4(c0[0], c0[1], c0[2], c0[3]);
        d0[1] = make_uint4(c0[4], c0[5], c0[6], c0[7]);
        d1[0] = make_uint4(c1[0], c1[1], c1[2], c1[3]);
        d1[1] = make_uint4(c1[4], c1[5], c1[6], c1[7]);
      }
    }
  };

  // ---- accumulators ----
  uint32_t acc[TPW][K];
  int32_t tot[TPW][K][2];
#pragma unroll
  for (int j = 0; j < TPW; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[j][k] = 0;
      tot[j][k][0] = 0;
      tot[j][k][1] = 0;
    }
  int since_flush = 0;
  auto add_flush = [&](uint32_t (*x)[K]) {
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) acc[j][k] += x[j][k];
    if (++since_flush == a.flush) {
      since_flush = 0;
#pragma unroll
      for (int j = 0; j < TPW; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          tot[j][k][0] += (int32_t)(acc[j][k] & 0xFFFFu);
          tot[j][k][1] += (int32_t)(acc[j][k] >> 16);
          acc[j][k] = 0;
        }
    }
  };
  auto load_off = [&](int c, uint32_t *o) {  // offsets of channel c of the pass (c uniform)
#pragma unroll
    for (int j = 0; j < TPW; ++j) o[j] = (uint32_t)__builtin_amdgcn_readlane((int)roff[j], c);
  };
  auto load_v = [&](const uint32_t *o, uint32_t (*dst)[K]) {
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const uint32_t *src = data + o[j] + lane;
#pragma unroll
      for (int k = 0; k < K; ++k) dst[j][k] = src[64 * k];
    }
  };

  // fold the 16-bit lanes into the totals, store the sums of output
  // segment `seg`, and start the next segment from zero
  auto finish = [&](int seg) {
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        tot[j][k][0] += (int32_t)(acc[j][k] & 0xFFFFu);
        tot[j][k][1] += (int32_t)(acc[j][k] >> 16);
        acc[j][k] = 0;
      }
    since_flush = 0;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int i = i_wave + j;
      if (i >= a.n_dm) break;
      OutT *orow_out = static_cast<OutT *>(a.out) + (int64_t)seg * a.seg_stride + (int64_t)i * a.out_pitch - a.t_lo;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int64_t t = t0 + 2 * (int64_t)(lane + 64 * k);
        if (t >= a.t_lo && t < a.t_hi) orow_out[t] = (OutT)tot[j][k][0];
        if (t + 1 >= a.t_lo && t + 1 < a.t_hi) orow_out[t + 1] = (OutT)tot[j][k][1];
      }
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        tot[j][k][0] = 0;
        tot[j][k][1] = 0;
      }
  };

  // ---- prologue: bases of passes 0 (LDS) and 1 (register), samples of pass 0 ----
  // (a pass has at most max_chunk <= threads channels: one base per thread)
  if (tid < ch_begin(1) - ch_begin(0)) bases[tid] = base_row[ch_begin(0) + tid];
  int32_t pbase = (n_chunks > 1 && tid < ch_begin(2) - ch_begin(1)) ? base_row[ch_begin(1) + tid] : 0;
  __syncthreads();
  prefetch(0);

  for (int kc = 0; kc < n_chunks; ++kc) {
    if (kc + 3 > w0 + 63) fetch_window(kc);  // passes kc .. kc + 3 are read below
    const int cs = ch_begin(kc), ce = ch_begin(kc + 1);
    __syncthreads();  // every wave is done with pass kc-1
    store(kc);
    if (tid < maxc) bases[((kc + 1) & 1) * maxc + tid] = pbase;
    __syncthreads();
    // in flight during the accumulation below: samples of pass kc+1, bases of kc+2
    if (kc + 2 < n_chunks)
      pbase = tid < ch_begin(kc + 3) - ch_begin(kc + 2) ? base_row[ch_begin(kc + 2) + tid] : 0;
#pragma unroll
    for (int j = 0; j < TPW; ++j) roff[j] = noff[j];  // loaded with pass kc's samples
    if (kc + 1 < n_chunks) prefetch(kc + 1);

    // ---- accumulate pass kc: per channel TPW trials x K dwords per lane ----
    // two register sets: while one channel is added, the next one's samples
    // are in flight.  The loads are unconditional (channel index clamped to
    // the pass) so that no branch forces a full wait before the adds.
    const int last = ce - 1 - cs;
    uint32_t offA[TPW], offB[TPW], vA[TPW][K], vB[TPW][K];
    load_off(0, offA);
    load_v(offA, vA);
    load_off(min(1, last), offB);
    for (int c = 0; c <= last; c += 2) {
      load_v(offB, vB);
      load_off(min(c + 2, last), offA);
      add_flush(vA);
      if (c + 1 > last) break;
      load_v(offA, vA);
      load_off(min(c + 3, last), offB);
      add_flush(vB);
    }
    if constexpr (SEG) {
      if (kc + 1 < n_chunks && ce % a.seg_ch == 0) finish(ce / a.seg_ch - 1);
    }
  }
  finish(SEG ? (a.nchan - 1) / a.seg_ch : 0);
}

// Batch launch: one tile per workgroup, XCD-aware tile order.
template <int K, int TPW, typename SrcT>
__global__ __launch_bounds__(512) void k_dedisp(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  const int G = a.n_dm_tiles * a.n_t_tiles;
  const int L = xcd_remap(blockIdx.x, G);
  dedisp_tile<K, TPW, SrcT>(a, L % a.n_dm_tiles, L / a.n_dm_tiles, lds);
}


}  // namespace gsp
