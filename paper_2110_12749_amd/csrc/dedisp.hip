// Brute-force incoherent dedispersion on gfx950.
//
// What is computed (paper Section 2.3, Algorithms 2-3): for every DM trial i
// of a plan row and output sample t, out[i][t] = sum_c Y[c][t + d(i, c)],
// where Y is the row's D-downsampled input and d the delay table.  The sums
// are exact integers.
//
// How (MI355X design, not the paper's per-thread global-memory loop):
//  1. k_stage turns the recorded time-major uint8 filterbank into a
//     channel-major copy Y, summing D samples (uint8 for D = 1, uint16 for
//     D > 1), through an LDS transpose so both the reads and the writes are
//     coalesced.
//  2. k_dedisp gives every workgroup a tile of DM trials x output samples.
//     Channels are staged into LDS in chunks as uint16 pairs, in two copies
//     (one shifted by a sample), so that every trial's shifted read is an
//     aligned dword holding two consecutive samples.  Lanes accumulate those
//     dwords directly as packed 2 x uint16 sums (one VALU add per two
//     sample-adds) and flush them into int32 before a 16-bit lane can
//     overflow.  Each staged sample is reused by every trial of the tile.
//     The per-(trial, channel) LDS offsets are precomputed on the host and
//     read with scalar loads, so the inner loop is ds_read + v_add.
//  3. Workgroup ids are remapped so that each XCD walks a contiguous range of
//     tiles, DM tiles fastest: concurrent workgroups of an XCD share their
//     input window in that XCD's L2.
#include <algorithm>
#include <cstring>

#include "gsp_internal.h"

namespace gsp {

// ---------------------------------------------------------------------------
// Staging: time-major uint8 [nsamp][nchan] -> channel-major Y [nchan][pitch]
// ---------------------------------------------------------------------------
// Tile = kStageC channels x kStageT outputs.  Read phase: each lane loads a
// dword (4 channels) of a recorded spectrum and sums the D spectra of one
// output (nchan % 4 == 0), or single bytes otherwise.  Write phase: a
// channel row of the tile is written as contiguous dwords.
static constexpr int kStageT = 128;  // outputs per tile
static constexpr int kStageC = 128;  // channels per tile
static constexpr int kStagePitch = kStageT + 1;  // odd u16 pitch spreads LDS banks

template <typename OutT, bool VEC>
__global__ __launch_bounds__(256) void k_stage(const uint8_t *__restrict__ X, int64_t nsamp, int32_t nchan,
                                               int32_t D, int64_t N, OutT *__restrict__ Y, int64_t pitch) {
  __shared__ uint16_t tile[kStageC * kStagePitch];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kStageT;
  const int32_t c0 = blockIdx.y * kStageC;
  if constexpr (VEC) {
    const int q = tid & 31;  // channel quad
    const int c = c0 + 4 * q;
    for (int jl = tid >> 5; jl < kStageT; jl += 8) {
      const int64_t j = j0 + jl;
      uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      if (c < nchan && j < N) {
        const uint8_t *p = X + (j * D) * (int64_t)nchan + c;
        for (int m = 0; m < D; ++m) {
          const uint32_t w = *reinterpret_cast<const uint32_t *>(p + (int64_t)m * nchan);
          a0 += w & 0xFFu;
          a1 += (w >> 8) & 0xFFu;
          a2 += (w >> 16) & 0xFFu;
          a3 += w >> 24;
        }
      }
      tile[(4 * q + 0) * kStagePitch + jl] = (uint16_t)a0;
      tile[(4 * q + 1) * kStagePitch + jl] = (uint16_t)a1;
      tile[(4 * q + 2) * kStagePitch + jl] = (uint16_t)a2;
      tile[(4 * q + 3) * kStagePitch + jl] = (uint16_t)a3;
    }
  } else {
    for (int u = tid; u < kStageC * kStageT; u += 256) {
      const int cl = u % kStageC, jl = u / kStageC;
      const int c = c0 + cl;
      const int64_t j = j0 + jl;
      uint32_t acc = 0;
      if (c < nchan && j < N) {
        const uint8_t *p = X + (j * D) * (int64_t)nchan + c;
        for (int m = 0; m < D; ++m) acc += p[(int64_t)m * nchan];
      }
      tile[cl * kStagePitch + jl] = (uint16_t)acc;
    }
  }
  __syncthreads();
  constexpr int per_dw = 4 / sizeof(OutT);
  constexpr int row_dw = kStageT / per_dw;
  for (int idx = tid; idx < kStageC * row_dw; idx += 256) {
    const int cl = idx / row_dw;
    const int p = idx % row_dw;
    const int c = c0 + cl;
    if (c >= nchan) continue;
    const int64_t j = j0 + (int64_t)p * per_dw;
    if (j >= pitch) continue;
    const uint16_t *t = tile + cl * kStagePitch + p * per_dw;
    uint32_t v;
    if constexpr (sizeof(OutT) == 1)
      v = (uint32_t)t[0] | ((uint32_t)t[1] << 8) | ((uint32_t)t[2] << 16) | ((uint32_t)t[3] << 24);
    else
      v = (uint32_t)t[0] | ((uint32_t)t[1] << 16);
    *reinterpret_cast<uint32_t *>(Y + (int64_t)c * pitch + j) = v;
  }
}

// ---------------------------------------------------------------------------
// Dedispersion
// ---------------------------------------------------------------------------
struct DedispArgs {
  const void *Y;            // channel-major staged input (uint8 or uint16)
  int64_t pitch;            // elements per channel row of Y
  const uint32_t *addr;     // [nchan][n_dm_pad] LDS dword offsets
  const int32_t *base;      // [n_tiles_dm][nchan] staging start (delay of tile's first trial, /4*4)
  int32_t *out;             // int32 [n_dm][n_out]
  int64_t n_out;
  int32_t n_dm, n_dm_pad, nchan;
  int32_t chunk;            // channels per staging pass
  int32_t flush;            // channels between flushes of the 16-bit lanes
  int32_t row_dw;           // dwords per staged copy of a channel
  int32_t n_dm_tiles, n_t_tiles;
};

__device__ __forceinline__ int xcd_remap(int b, int G) {
  // hardware dispatches workgroup b to XCD b % 8; give each XCD a contiguous
  // range of logical tiles
  const int q = G >> 3, r = G & 7;
  const int x = b & 7, k = b >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Staging unit: 16 consecutive samples of one channel, i.e. 8 dwords of each
// LDS copy.  Each thread stages at most kUnitMax units per chunk.
static constexpr int kUnitMax = 2;

template <typename SrcT>
struct Unit {
  static constexpr int W = 16 / (4 / sizeof(SrcT));  // source dwords holding 16 samples
  uint32_t w[W];
  uint32_t tail;  // sample 16 (needed by the shifted copy)
};

template <int K, int TPW, typename SrcT>
__global__ __launch_bounds__(512) void k_dedisp(DedispArgs a) {
  static_assert(TPW % 4 == 0, "offsets are read four trials at a time");
  extern __shared__ uint32_t lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x;
  const int nwaves = nthreads >> 6;
  const int G = a.n_dm_tiles * a.n_t_tiles;
  const int L = xcd_remap(blockIdx.x, G);
  const int dm_tile = L % a.n_dm_tiles;
  const int t_tile = L / a.n_dm_tiles;
  constexpr int T = 128 * K;
  const int64_t t0 = (int64_t)t_tile * T;
  const int MT = TPW * nwaves;
  const int i_tile = dm_tile * MT;
  const int row_dw = a.row_dw;  // multiple of 8
  const int U = row_dw >> 3;    // staging units per channel
  const int chunk = a.chunk;
  const int n_chunks = (a.nchan + chunk - 1) / chunk;
  // LDS: samples [chunk][2][row_dw] | offsets [chunk][MT] | staging bases [2][chunk]
  uint32_t *data = lds;
  uint32_t *offs = lds + 2 * chunk * row_dw;
  int32_t *bases = reinterpret_cast<int32_t *>(offs + chunk * MT);

  const SrcT *Y = static_cast<const SrcT *>(a.Y);
  const int32_t *base_row = a.base + (int64_t)dm_tile * a.nchan;

  // ---- staging helpers ----
  Unit<SrcT> pu[kUnitMax];
  uint32_t poff = 0;
  auto prefetch = [&](int j) {  // global -> registers for chunk j (bases of j already in LDS)
    const int cs = j * chunk, ce = min(cs + chunk, a.nchan);
    const int nu = (ce - cs) * U;
    const int32_t *bj = bases + (j & 1) * chunk;
    // all addresses first, then all loads, so every load is issued back to back
    const SrcT *rows[kUnitMax];
#pragma unroll
    for (int i = 0; i < kUnitMax; ++i) {
      const int u = min(tid + i * nthreads, nu - 1);  // clamped: loads stay in bounds
      const int cl = u / U;
      const int p = u - cl * U;
      const int64_t e0 = t0 + bj[cl] + 16 * (int64_t)p;  // multiple of 4
      rows[i] = Y + (int64_t)(cs + cl) * a.pitch + e0;
    }
#pragma unroll
    for (int i = 0; i < kUnitMax; ++i) {
      const uint32_t *w = reinterpret_cast<const uint32_t *>(rows[i]);
#pragma unroll
      for (int m = 0; m < Unit<SrcT>::W; ++m) pu[i].w[m] = w[m];
      pu[i].tail = rows[i][16];
    }
    if (tid < (ce - cs) * MT) poff = a.addr[(int64_t)(cs + tid / MT) * a.n_dm_pad + i_tile + tid % MT];
  };
  auto store = [&](int j) {  // registers -> LDS for chunk j
    const int cs = j * chunk, ce = min(cs + chunk, a.nchan);
    const int nu = (ce - cs) * U;
#pragma unroll
    for (int i = 0; i < kUnitMax; ++i) {
      const int u = tid + i * nthreads;
      if (u < nu) {
        const int cl = u / U;
        const int p = u - cl * U;
        uint32_t c0[8], c1[8];
        if constexpr (sizeof(SrcT) == 1) {
          // samples y0..y15 in 4 dwords, y16 in tail
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const uint32_t w = pu[i].w[m >> 1];
            const uint32_t wn = (m >> 1) + 1 < 4 ? pu[i].w[(m >> 1) + 1] : pu[i].tail;
            const int b = (m & 1) * 2;  // byte of sample 2m within w
            const uint32_t ya = (w >> (8 * b)) & 0xFFu;
            const uint32_t yb = (w >> (8 * b + 8)) & 0xFFu;
            const uint32_t yc = b == 2 ? (wn & 0xFFu) : ((w >> (8 * b + 16)) & 0xFFu);
            c0[m] = ya | (yb << 16);
            c1[m] = yb | (yc << 16);
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
    if (tid < (ce - cs) * MT) offs[tid] = poff;
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
  auto load_off = [&](const uint32_t *p, uint32_t *o) {
#pragma unroll
    for (int j = 0; j < TPW; j += 4) {
      const uint4 q = *reinterpret_cast<const uint4 *>(p + j);
      o[j] = q.x;
      o[j + 1] = q.y;
      o[j + 2] = q.z;
      o[j + 3] = q.w;
    }
  };
  auto load_v = [&](const uint32_t *o, uint32_t (*dst)[K]) {
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const uint32_t *src = data + o[j] + lane;
#pragma unroll
      for (int k = 0; k < K; ++k) dst[j][k] = src[64 * k];
    }
  };

  // ---- prologue: bases of chunks 0 (LDS) and 1 (register), samples of chunk 0 ----
  if (tid < chunk) bases[tid] = tid < a.nchan ? base_row[tid] : 0;
  int32_t pbase = (tid < chunk && chunk + tid < a.nchan) ? base_row[chunk + tid] : 0;
  __syncthreads();
  prefetch(0);

  for (int kc = 0; kc < n_chunks; ++kc) {
    const int cs = kc * chunk, ce = min(cs + chunk, a.nchan);
    __syncthreads();  // every wave is done with chunk kc-1
    store(kc);
    if (tid < chunk) bases[((kc + 1) & 1) * chunk + tid] = pbase;
    __syncthreads();
    // in flight during the accumulation below: samples of chunk kc+1, bases of kc+2
    if (kc + 2 < n_chunks && tid < chunk)
      pbase = (kc + 2) * chunk + tid < a.nchan ? base_row[(kc + 2) * chunk + tid] : 0;
    if (kc + 1 < n_chunks) prefetch(kc + 1);

    // ---- accumulate chunk kc: per channel TPW trials x K dwords per lane ----
    // two register sets: while one channel is added, the next one's samples
    // and the one after's offsets are in flight (LDS returns in order).  The
    // loads are unconditional (channel index clamped to the chunk) so that no
    // branch forces a full wait before the adds.
    const uint32_t *orow = offs + wave * TPW;
    const int last = ce - 1 - cs;
    uint32_t offA[TPW], offB[TPW], vA[TPW][K], vB[TPW][K];
    load_off(orow, offA);
    load_v(offA, vA);
    load_off(orow + min(1, last) * MT, offB);
    for (int c = 0; c <= last; c += 2) {
      load_v(offB, vB);
      load_off(orow + min(c + 2, last) * MT, offA);
      add_flush(vA);
      if (c + 1 > last) break;
      load_v(offA, vA);
      load_off(orow + min(c + 3, last) * MT, offB);
      add_flush(vB);
    }
  }
#pragma unroll
  for (int j = 0; j < TPW; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      tot[j][k][0] += (int32_t)(acc[j][k] & 0xFFFFu);
      tot[j][k][1] += (int32_t)(acc[j][k] >> 16);
    }
  // ---- store ----
  const int i_wave = i_tile + wave * TPW;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int i = i_wave + j;
    if (i >= a.n_dm) break;
    int32_t *orow_out = a.out + (int64_t)i * a.n_out;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t t = t0 + 2 * (int64_t)(lane + 64 * k);
      if (t < a.n_out) orow_out[t] = tot[j][k][0];
      if (t + 1 < a.n_out) orow_out[t + 1] = tot[j][k][1];
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
DedispShape default_shape(int32_t D) {
  DedispShape s;
  s.tpw = 4;
  s.waves = 8;
  s.groups = 4;
  s.chunk = 16;
  (void)D;
  return s;
}

bool shape_supported(const DedispShape &s) {
  const int kt = s.groups * 16 + s.tpw;
  const bool inst = kt == 8 * 16 + 4 || kt == 4 * 16 + 8 || kt == 4 * 16 + 4 || kt == 2 * 16 + 8;
  return inst && s.waves >= 1 && s.waves <= 8 && s.chunk >= 1;
}

std::string row_signature(const gsp_dmt_desc *desc, int32_t s) {
  // length class: n_out rounded down to a power of two
  int lc = 0;
  while ((desc->n_out[s] >> (lc + 1)) > 0) ++lc;
  return "nc" + std::to_string(desc->nchan) + "-D" + std::to_string(desc->seg[s].downsamp) + "-ndm" +
         std::to_string(desc->seg[s].n_dm) + "-md" + std::to_string(desc->max_delay[s]) + "-L" + std::to_string(lc);
}

DedispShape shape_for_row(gsp_ctx *ctx, const gsp_dmt_desc *desc, int32_t s) {
  auto it = ctx->tuned.find(row_signature(desc, s));
  return it != ctx->tuned.end() ? it->second : default_shape(desc->seg[s].downsamp);
}

static constexpr int64_t kLdsBudget = 80 * 1024;  // two workgroups per CU
static constexpr int64_t kLdsMax = 160 * 1024;

static int flush_interval(int32_t D) {
  // a uint16 lane holds at most 65535; each add contributes <= 255 * D
  const int f = 65535 / (255 * D);
  return std::max(1, std::min(f, 256));
}

int64_t staged_pitch(const RowTables &rt) {
  // furthest element a staging pass can touch: t0 + base + 2 * row_dw + 2
  const int64_t T = rt.shape.samples_per_block();
  const int64_t n_t = (rt.n_out + T - 1) / T;
  const int64_t far = (n_t - 1) * T + rt.max_delay + 2 * (int64_t)rt.row_dwords + 8;
  int64_t p = std::max(far, rt.N);
  return (p + 255) / 256 * 256;
}

void build_row_tables(gsp_ctx *ctx, const gsp_dmt_desc *desc, const double *freqs, int32_t s,
                      const DedispShape &shape, RowTables &rt) {
  const gsp_segment &g = desc->seg[s];
  rt.n_dm = g.n_dm;
  rt.D = g.downsamp;
  rt.nchan = desc->nchan;
  rt.N = desc->nsamp / g.downsamp;
  rt.n_out = desc->n_out[s];
  rt.max_delay = desc->max_delay[s];
  rt.shape = shape;
  rt.addr.device = ctx->device;
  rt.dmin.device = ctx->device;
  const int nchan = desc->nchan;
  if (rt.delays_host.empty()) {
    rt.delays_host.resize((size_t)g.n_dm * nchan);
    compute_delays(desc, freqs, s, rt.delays_host.data());
  }
  const int MT = shape.trials_per_block();
  const int n_tiles = (g.n_dm + MT - 1) / MT;
  const int n_dm_pad = n_tiles * MT;
  const int32_t *d = rt.delays_host.data();
  auto delay = [&](int i, int c) { return d[(int64_t)std::min(i, g.n_dm - 1) * nchan + c]; };
  // staging base per (tile, channel) and the widest window
  std::vector<int32_t> base((size_t)n_tiles * nchan);
  int64_t max_e = 0;
  for (int tl = 0; tl < n_tiles; ++tl)
    for (int c = 0; c < nchan; ++c) {
      const int32_t b = delay(tl * MT, c) & ~3;
      base[(size_t)tl * nchan + c] = b;
      max_e = std::max<int64_t>(max_e, delay(tl * MT + MT - 1, c) - b);
    }
  const int K = shape.groups;
  // a multiple of 8 dwords: whole 16-sample staging units, 16-byte aligned rows
  rt.row_dwords = (int32_t)((((max_e >> 1) + 64 * K + 1) + 7) & ~7);
  // channels per staging pass: as many as fit the LDS budget (two copies of
  // row_dwords dwords + MT offsets + 2 bases per channel), as the staging
  // registers allow, and at most the requested chunk
  const int threads = 64 * shape.waves;
  const int64_t per_chan = 2 * (int64_t)rt.row_dwords * 4 + (int64_t)MT * 4 + 8;
  int64_t chunk64 = std::min<int64_t>(shape.chunk, std::max<int64_t>(1, kLdsBudget / per_chan));
  chunk64 = std::min<int64_t>(chunk64, (int64_t)kUnitMax * threads / (rt.row_dwords / 8));
  chunk64 = std::min<int64_t>(chunk64, threads / MT);
  if (chunk64 < 1 || chunk64 * per_chan > kLdsMax)
    fail(GSP_EINVAL, "dedispersion tile does not fit in LDS (delay spread too wide)");
  const int chunk = (int)chunk64;
  rt.shape.chunk = chunk;
  rt.lds_bytes = (int64_t)chunk * per_chan;
  std::vector<uint32_t> addr((size_t)nchan * n_dm_pad);
  for (int c = 0; c < nchan; ++c) {
    const int cl = c % chunk;
    for (int i = 0; i < n_dm_pad; ++i) {
      const int tl = i / MT;
      const int32_t e = delay(i, c) - base[(size_t)tl * nchan + c];
      addr[(size_t)c * n_dm_pad + i] = (uint32_t)((cl * 2 + (e & 1)) * rt.row_dwords + (e >> 1));
    }
  }
  rt.addr.reserve(addr.size() * 4);
  rt.dmin.reserve(base.size() * 4);
  check_hip(hipMemcpy(rt.addr.ptr, addr.data(), addr.size() * 4, hipMemcpyHostToDevice), "copy LDS offsets");
  check_hip(hipMemcpy(rt.dmin.ptr, base.data(), base.size() * 4, hipMemcpyHostToDevice), "copy staging bases");
}

void stage_row(gsp_ctx *ctx, const uint8_t *fb, const gsp_dmt_desc *desc, const RowTables &rt, hipStream_t st) {
  const int64_t pitch = staged_pitch(rt);
  const size_t elem = rt.D == 1 ? 1 : 2;
  ctx->staged.device = ctx->device;
  ctx->staged.reserve((size_t)pitch * rt.nchan * elem + 256);
  dim3 grid((unsigned)((pitch + kStageT - 1) / kStageT), (unsigned)((rt.nchan + kStageC - 1) / kStageC));
  // bytes: the filterbank rows read once + the staged copy written once
  ProfScope prof(ctx, "stage", st, (double)rt.N * rt.D * rt.nchan + (double)pitch * rt.nchan * elem);
  const bool vec = (rt.nchan % 4) == 0 && (reinterpret_cast<uintptr_t>(fb) % 4) == 0;
  if (rt.D == 1) {
    auto k = vec ? k_stage<uint8_t, true> : k_stage<uint8_t, false>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, st, fb, desc->nsamp, rt.nchan, rt.D, rt.N, ctx->staged.as<uint8_t>(),
                       pitch);
  } else {
    auto k = vec ? k_stage<uint16_t, true> : k_stage<uint16_t, false>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, st, fb, desc->nsamp, rt.nchan, rt.D, rt.N, ctx->staged.as<uint16_t>(),
                       pitch);
  }
  check_hip(hipGetLastError(), "launch staging kernel");
}

template <int K, int TPW>
static void launch_k(const DedispArgs &a, int waves, int64_t lds, int D, hipStream_t st) {
  const int G = a.n_dm_tiles * a.n_t_tiles;
  if (D == 1) {
    auto kern = k_dedisp<K, TPW, uint8_t>;
    check_hip(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "set LDS size");
    hipLaunchKernelGGL(kern, dim3(G), dim3(64 * waves), (size_t)lds, st, a);
  } else {
    auto kern = k_dedisp<K, TPW, uint16_t>;
    check_hip(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "set LDS size");
    hipLaunchKernelGGL(kern, dim3(G), dim3(64 * waves), (size_t)lds, st, a);
  }
}

void launch_dedisp(gsp_ctx *ctx, const RowTables &rt, int32_t *out_row, hipStream_t st) {
  const DedispShape &sh = rt.shape;
  DedispArgs a;
  a.Y = ctx->staged.ptr;
  a.pitch = staged_pitch(rt);
  a.addr = rt.addr.as<uint32_t>();
  a.base = rt.dmin.as<int32_t>();
  a.out = out_row;
  a.n_out = rt.n_out;
  a.n_dm = rt.n_dm;
  const int MT = sh.trials_per_block();
  a.n_dm_tiles = (rt.n_dm + MT - 1) / MT;
  a.n_dm_pad = a.n_dm_tiles * MT;
  a.nchan = rt.nchan;
  a.chunk = sh.chunk;
  a.flush = flush_interval(rt.D);
  a.row_dw = rt.row_dwords;
  const int64_t T = sh.samples_per_block();
  a.n_t_tiles = (int32_t)((rt.n_out + T - 1) / T);
  if ((int64_t)a.n_dm_tiles * a.n_t_tiles >= (1LL << 31)) fail(GSP_EOVERFLOW, "too many dedispersion tiles");
  // algorithmic work: one integer add per (trial, output sample, channel)
  ProfScope prof(ctx, "dedisperse", st, (double)rt.n_dm * (double)rt.n_out * (double)rt.nchan);
  switch (sh.groups * 16 + sh.tpw) {
    case 8 * 16 + 4: launch_k<8, 4>(a, sh.waves, rt.lds_bytes, rt.D, st); break;
    case 4 * 16 + 8: launch_k<4, 8>(a, sh.waves, rt.lds_bytes, rt.D, st); break;
    case 4 * 16 + 4: launch_k<4, 4>(a, sh.waves, rt.lds_bytes, rt.D, st); break;
    case 2 * 16 + 8: launch_k<2, 8>(a, sh.waves, rt.lds_bytes, rt.D, st); break;
    default: fail(GSP_EINVAL, "unsupported dedispersion shape");
  }
  check_hip(hipGetLastError(), "launch dedispersion kernel");
}

}  // namespace gsp
