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
static constexpr int kStageT = 256;  // outputs per tile
static constexpr int kStageC = 64;   // channels per tile

template <typename OutT>
__global__ __launch_bounds__(256) void k_stage(const uint8_t *__restrict__ X, int64_t nsamp, int32_t nchan,
                                               int32_t D, int64_t N, OutT *__restrict__ Y, int64_t pitch) {
  __shared__ uint16_t tile[kStageC][kStageT + 2];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kStageT;
  const int32_t c0 = blockIdx.y * kStageC;
  // read phase: lane -> channel, wave -> output sample
  {
    const int cl = tid & 63;
    const int c = c0 + cl;
    for (int jl = tid >> 6; jl < kStageT; jl += 4) {
      const int64_t j = j0 + jl;
      uint32_t acc = 0;
      if (c < nchan && j < N) {
        const uint8_t *p = X + (j * D) * (int64_t)nchan + c;
        for (int m = 0; m < D; ++m) acc += p[(int64_t)m * nchan];
      }
      tile[cl][jl] = (uint16_t)acc;
    }
  }
  __syncthreads();
  // write phase: consecutive lanes -> consecutive dwords of one channel row
  constexpr int per_dw = 4 / sizeof(OutT);
  constexpr int row_dw = kStageT / per_dw;
  for (int idx = tid; idx < kStageC * row_dw; idx += 256) {
    const int cl = idx / row_dw;
    const int q = idx % row_dw;
    const int c = c0 + cl;
    if (c >= nchan) continue;
    const int64_t j = j0 + (int64_t)q * per_dw;
    if (j >= pitch) continue;
    uint32_t v;
    if constexpr (sizeof(OutT) == 1) {
      v = (uint32_t)tile[cl][4 * q] | ((uint32_t)tile[cl][4 * q + 1] << 8) |
          ((uint32_t)tile[cl][4 * q + 2] << 16) | ((uint32_t)tile[cl][4 * q + 3] << 24);
    } else {
      v = (uint32_t)tile[cl][2 * q] | ((uint32_t)tile[cl][2 * q + 1] << 16);
    }
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

template <int K, int TPW, typename SrcT>
__global__ __launch_bounds__(512) void k_dedisp(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int G = a.n_dm_tiles * a.n_t_tiles;
  const int L = xcd_remap(blockIdx.x, G);
  const int dm_tile = L % a.n_dm_tiles;
  const int t_tile = L / a.n_dm_tiles;
  constexpr int T = 128 * K;
  const int64_t t0 = (int64_t)t_tile * T;
  const int MT = TPW * nwaves;
  const int i_wave = dm_tile * MT + wave * TPW;  // first trial of this wave

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

  const SrcT *Y = static_cast<const SrcT *>(a.Y);
  const int32_t *base_row = a.base + (int64_t)dm_tile * a.nchan;
  const int row_dw = a.row_dw;
  int since_flush = 0;

  for (int cs = 0; cs < a.nchan; cs += a.chunk) {
    const int ce = min(cs + a.chunk, a.nchan);
    __syncthreads();
    // ---- stage channels [cs, ce) as two uint16-pair rows each ----
    {
      const int n_units = (ce - cs) * row_dw;  // one unit = one dword of each copy
      for (int u = threadIdx.x; u < n_units; u += blockDim.x) {
        const int cl = u / row_dw;
        const int q = u - cl * row_dw;
        const int c = cs + cl;
        const int64_t e0 = t0 + base_row[c] + 2 * (int64_t)q;  // element of copy 0, dword q
        const SrcT *row = Y + (int64_t)c * a.pitch;
        uint32_t w0, w1;
        if constexpr (sizeof(SrcT) == 1) {
          const uint32_t y0 = row[e0], y1 = row[e0 + 1], y2 = row[e0 + 2];
          w0 = y0 | (y1 << 16);
          w1 = y1 | (y2 << 16);
        } else {
          const uint32_t lo = *reinterpret_cast<const uint32_t *>(row + e0);
          const uint32_t y2 = row[e0 + 2];
          w0 = lo;
          w1 = (lo >> 16) | (y2 << 16);
        }
        uint32_t *dst = lds + (cl * 2) * row_dw + q;
        dst[0] = w0;
        dst[row_dw] = w1;
      }
    }
    __syncthreads();
    // ---- accumulate ----
    for (int c = cs; c < ce; ++c) {
      const uint32_t *ap = a.addr + (int64_t)c * a.n_dm_pad + i_wave;
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        const uint32_t off = __builtin_amdgcn_readfirstlane(ap[j]);
        const uint32_t *src = lds + off + lane;
#pragma unroll
        for (int k = 0; k < K; ++k) acc[j][k] += src[64 * k];
      }
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
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int i = i_wave + j;
    if (i >= a.n_dm) break;
    int32_t *orow = a.out + (int64_t)i * a.n_out;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t t = t0 + 2 * (int64_t)(lane + 64 * k);
      if (t < a.n_out) orow[t] = tot[j][k][0];
      if (t + 1 < a.n_out) orow[t + 1] = tot[j][k][1];
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
  s.groups = 8;
  s.chunk = 16;
  (void)D;
  return s;
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
  rt.row_dwords = (int32_t)((max_e >> 1) + 64 * K + 1);
  // channels per staging pass: as many as fit the LDS budget (two copies of
  // row_dwords dwords per channel), at most the requested chunk
  const int64_t per_chan = 2 * (int64_t)rt.row_dwords * 4;
  int chunk = (int)std::min<int64_t>(shape.chunk, std::max<int64_t>(1, kLdsBudget / per_chan));
  if (chunk * per_chan > kLdsMax) fail(GSP_EINVAL, "dedispersion tile does not fit in LDS (delay spread too wide)");
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
  if (rt.D == 1)
    hipLaunchKernelGGL(k_stage<uint8_t>, grid, dim3(256), 0, st, fb, desc->nsamp, rt.nchan, rt.D, rt.N,
                       ctx->staged.as<uint8_t>(), pitch);
  else
    hipLaunchKernelGGL(k_stage<uint16_t>, grid, dim3(256), 0, st, fb, desc->nsamp, rt.nchan, rt.D, rt.N,
                       ctx->staged.as<uint16_t>(), pitch);
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
    case 8 * 16 + 2: launch_k<8, 2>(a, sh.waves, rt.lds_bytes, rt.D, st); break;
    default: fail(GSP_EINVAL, "unsupported dedispersion shape");
  }
  check_hip(hipGetLastError(), "launch dedispersion kernel");
}

}  // namespace gsp
