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
// Tile = kStageC channels x kStageT outputs.  Read phase: each lane loads 16
// bytes (16 channels) of a recorded spectrum (nchan % 16 == 0, 16-byte
// aligned input), a dword (nchan % 4 == 0) or single bytes otherwise, and
// sums the D spectra of one output; the 16-byte form keeps four rows of
// loads in flight per lane.  Write phase: a channel row of the tile is
// written as contiguous dwords.
static constexpr int kStageT = 128;  // outputs per tile
static constexpr int kStageC = 128;  // channels per tile
static constexpr int kStagePitch = kStageT + 1;  // odd u16 pitch spreads LDS banks

// MODE: 2 = 16-byte loads, 1 = dword loads, 0 = byte loads.
template <typename OutT, int MODE>
__global__ __launch_bounds__(256) void k_stage(const uint8_t *__restrict__ X, int64_t nsamp, int32_t nchan,
                                               int32_t D, int64_t N, OutT *__restrict__ Y, int64_t pitch) {
  __shared__ uint16_t tile[kStageC * kStagePitch];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kStageT;
  const int32_t c0 = blockIdx.y * kStageC;
  if constexpr (MODE == 2) {
    // 8 lanes per 128-channel spectrum, 32 outputs per pass, 4 passes (the
    // first spectrum of all 4 loaded together); the D spectra of an output
    // are summed as even/odd bytes in 16-bit halves (255 D <= 65535)
    const int g = tid & 7;
    const int c = c0 + 16 * g;
    const bool cin = c < nchan;
    uint4 w0[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int64_t j = j0 + (tid >> 3) + 32 * it;
      w0[it] = (cin && j < N) ? *reinterpret_cast<const uint4 *>(X + (j * D) * (int64_t)nchan + c)
                              : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int jl = (tid >> 3) + 32 * it;
      const int64_t j = j0 + jl;
      uint32_t ev[4], od[4];
      const uint32_t a[4] = {w0[it].x, w0[it].y, w0[it].z, w0[it].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ev[q] = a[q] & 0x00FF00FFu;
        od[q] = (a[q] >> 8) & 0x00FF00FFu;
      }
      if (cin && j < N) {
        const uint8_t *p = X + (j * D) * (int64_t)nchan + c;
        for (int m = 1; m < D; ++m) {
          const uint4 w = *reinterpret_cast<const uint4 *>(p + (int64_t)m * nchan);
          const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            ev[q] += wv[q] & 0x00FF00FFu;
            od[q] += (wv[q] >> 8) & 0x00FF00FFu;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        tile[(16 * g + 4 * q + 0) * kStagePitch + jl] = (uint16_t)(ev[q] & 0xFFFFu);
        tile[(16 * g + 4 * q + 1) * kStagePitch + jl] = (uint16_t)(od[q] & 0xFFFFu);
        tile[(16 * g + 4 * q + 2) * kStagePitch + jl] = (uint16_t)(ev[q] >> 16);
        tile[(16 * g + 4 * q + 3) * kStagePitch + jl] = (uint16_t)(od[q] >> 16);
      }
    }
  } else if constexpr (MODE == 1) {
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
  // 16 bytes per store: 16 (uint8) or 8 (uint16) outputs of one channel;
  // rows of Y are 256-element aligned and the tile never crosses the pitch
  constexpr int per_st = 16 / sizeof(OutT);
  constexpr int row_st = kStageT / per_st;
  for (int idx = tid; idx < kStageC * row_st; idx += 256) {
    const int cl = idx / row_st;
    const int p = idx % row_st;
    const int c = c0 + cl;
    if (c >= nchan) continue;
    const int64_t j = j0 + (int64_t)p * per_st;
    if (j >= pitch) continue;
    const uint16_t *t = tile + cl * kStagePitch + p * per_st;
    uint32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if constexpr (sizeof(OutT) == 1)
        v[q] = (uint32_t)t[4 * q] | ((uint32_t)t[4 * q + 1] << 8) | ((uint32_t)t[4 * q + 2] << 16) |
               ((uint32_t)t[4 * q + 3] << 24);
      else
        v[q] = (uint32_t)t[2 * q] | ((uint32_t)t[2 * q + 1] << 16);
    }
    *reinterpret_cast<uint4 *>(Y + (int64_t)c * pitch + j) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

}  // namespace gsp

#include "dedisp_tile.h"

namespace gsp {

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
DedispShape default_shape(int32_t D, int32_t nchan) {
  DedispShape s;
  s.tpw = 4;
  s.waves = 8;
  s.groups = 4;
  s.chunk = 32;
  if (D == 1 && nchan % 4 == 0) {  // byte-quad tile with staging waves: 12 summing waves
    s.kind = 2;
    s.groups = 4;
    s.tpw = 8;
    s.waves = 12;
    s.chunk = 64;
  }
  return s;
}

bool shape_supported(const DedispShape &s) {
  if (s.kind >= 1 && s.kind <= 3) return quad_shape_supported(s);
  if (s.kind != 0) return false;
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
  return it != ctx->tuned.end() ? it->second : default_shape(desc->seg[s].downsamp, desc->nchan);
}

static constexpr int64_t kLdsBudget = 80 * 1024;  // two workgroups per CU
static constexpr int64_t kLdsMax = 160 * 1024;

static int flush_interval(int32_t D) {
  // a uint16 lane holds at most 65535; each add contributes <= 255 * D
  const int f = 65535 / (255 * D);
  return std::max(1, std::min(f, 256));
}

int64_t staged_pitch(const RowTables &rt) {
  if (rt.pitch_override > 0) return rt.pitch_override;
  if (rt.shape.kind != 0) return rt.q_pitch;
  // furthest element a staging pass can touch: t0 + base + 2 * row_dw + 2
  const int64_t T = rt.shape.samples_per_block();
  const int64_t n_t = (rt.n_out + T - 1) / T;
  const int64_t far = (n_t - 1) * T + rt.max_delay + 2 * (int64_t)rt.row_dwords + 8;
  int64_t p = std::max(far, rt.N);
  return (p + 255) / 256 * 256;
}

void build_row_tables(gsp_ctx *ctx, const gsp_dmt_desc *desc, const double *freqs, int32_t s,
                      const DedispShape &shape, RowTables &rt, int units_per_thread) {
  if (!shape_supported(shape)) fail(GSP_EINVAL, "unsupported dedispersion shape");
  const gsp_segment &g = desc->seg[s];
  if (rt.delays_host.empty()) {
    rt.delays_host.resize((size_t)g.n_dm * desc->nchan);
    compute_delays(desc, freqs, s, rt.delays_host.data());
  }
  if (shape.kind != 0) {
    rt.n_dm = g.n_dm;
    rt.D = g.downsamp;
    rt.nchan = desc->nchan;
    rt.N = desc->nsamp / g.downsamp;
    rt.n_out = desc->n_out[s];
    rt.max_delay = desc->max_delay[s];
    rt.shape = shape;
    build_quad_tables(ctx, rt);
    return;
  }
  build_tables_from_delays(ctx, g.n_dm, desc->nchan, g.downsamp, desc->nsamp / g.downsamp, desc->n_out[s],
                           desc->max_delay[s], shape, rt, units_per_thread);
}

void build_tables_from_delays(gsp_ctx *ctx, int32_t n_dm, int32_t nchan_, int32_t D, int64_t N, int64_t n_out,
                              int64_t max_delay, const DedispShape &shape, RowTables &rt, int units_per_thread,
                              int64_t lds_budget, int32_t pass_break) {
  struct {
    int32_t n_dm, downsamp;
  } g{n_dm, D};
  rt.n_dm = n_dm;
  rt.D = D;
  rt.nchan = nchan_;
  rt.N = N;
  rt.n_out = n_out;
  rt.max_delay = max_delay;
  rt.shape = shape;
  rt.addr.device = ctx->device;
  rt.dmin.device = ctx->device;
  const int nchan = nchan_;
  if (rt.delays_host.size() != (size_t)n_dm * nchan) fail(GSP_EINVAL, "delay table size");
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
  // staged window per channel: the widest delay spread of a DM tile at that
  // channel plus the tile's samples, in dwords, a multiple of 8 (whole
  // 16-sample staging units, 16-byte aligned rows)
  std::vector<int32_t> row_dw_c(nchan);
  int32_t widest = 0;
  for (int c = 0; c < nchan; ++c) {
    int64_t e = 0;
    for (int tl = 0; tl < n_tiles; ++tl) e = std::max<int64_t>(e, delay(tl * MT + MT - 1, c) - base[(size_t)tl * nchan + c]);
    row_dw_c[c] = (int32_t)((((e >> 1) + 64 * K + 1) + 7) & ~7);
    widest = std::max(widest, row_dw_c[c]);
  }
  rt.row_dwords = widest;
  // staging passes over consecutive channels (neighbouring frequencies,
  // similar spreads): each as long as its staged copies fit the LDS budget
  // left after the staging bases of the longest allowed pass, the
  // staging registers (`units` per thread) hold it, and at most the
  // requested number of channels
  const int threads = 64 * shape.waves;
  const int units = units_per_thread > 0 ? units_per_thread : unit_max_for_d(g.downsamp);
  const int64_t kmax = std::min<int64_t>({(int64_t)shape.chunk, (int64_t)kPassMax, (int64_t)threads});
  if (kmax < 1) fail(GSP_EINVAL, "unsupported dedispersion shape");
  const int64_t side = kmax * 8;  // two staging bases per channel, bytes
  const int64_t data_budget = (lds_budget > 0 ? lds_budget : kLdsBudget) - side;
  std::vector<int32_t> passes;  // start, row dwords pairs
  int64_t data_dw = 0;
  int max_chunk = 0;
  for (int c = 0; c < nchan;) {
    int k = 0;
    int32_t rd = 0;
    while (c + k < nchan) {
      if (k > 0 && pass_break > 0 && (c + k) % pass_break == 0) break;  // output segment boundary
      const int32_t rd2 = std::max(rd, row_dw_c[c + k]);
      const int64_t k2 = k + 1;
      const bool fits = k2 <= kmax && 2 * k2 * rd2 * 4 <= data_budget && k2 * (rd2 / 8) <= (int64_t)units * threads;
      if (!fits && k > 0) break;
      if (!fits) {  // one channel alone: still allowed up to the hardware LDS if the registers hold it
        if (rd2 / 8 > (int64_t)units * threads || 2 * (int64_t)rd2 * 4 + side > kLdsMax)
          fail(GSP_EINVAL, "dedispersion tile does not fit in LDS (delay spread too wide)");
      }
      rd = rd2;
      k = (int)k2;
      if (!fits) break;
    }
    passes.push_back(c);
    passes.push_back(rd);
    data_dw = std::max<int64_t>(data_dw, 2 * (int64_t)k * rd);
    max_chunk = std::max(max_chunk, k);
    c += k;
  }
  passes.push_back(nchan);
  passes.push_back(0);
  rt.n_passes = (int32_t)(passes.size() / 2 - 1);
  rt.max_chunk = max_chunk;
  rt.data_dw = (int32_t)data_dw;
  rt.shape.chunk = max_chunk;
  rt.lds_bytes = data_dw * 4 + (int64_t)max_chunk * 8;
  if (rt.lds_bytes > kLdsMax) fail(GSP_EINVAL, "dedispersion tile does not fit in LDS (delay spread too wide)");
  std::vector<uint32_t> addr((size_t)nchan * n_dm_pad);
  for (size_t q = 0; q + 2 < passes.size(); q += 2) {
    const int cs = passes[q], ce = passes[q + 2];
    const int32_t rd = passes[q + 1];
    for (int c = cs; c < ce; ++c) {
      const int cl = c - cs;
      for (int i = 0; i < n_dm_pad; ++i) {
        const int tl = i / MT;
        const int32_t e = delay(i, c) - base[(size_t)tl * nchan + c];
        addr[(size_t)c * n_dm_pad + i] = (uint32_t)((cl * 2 + (e & 1)) * rd + (e >> 1));
      }
    }
  }
  rt.passes.device = ctx->device;
  rt.passes.reserve(passes.size() * 4);
  check_hip(hipMemcpy(rt.passes.ptr, passes.data(), passes.size() * 4, hipMemcpyHostToDevice), "copy staging passes");
  rt.addr.reserve(addr.size() * 4);
  rt.dmin.reserve(base.size() * 4);
  check_hip(hipMemcpy(rt.addr.ptr, addr.data(), addr.size() * 4, hipMemcpyHostToDevice), "copy LDS offsets");
  check_hip(hipMemcpy(rt.dmin.ptr, base.data(), base.size() * 4, hipMemcpyHostToDevice), "copy staging bases");
}

void stage_row(gsp_ctx *ctx, const uint8_t *fb, const gsp_dmt_desc *desc, const RowTables &rt, hipStream_t st,
               int64_t pitch_override) {
  const int64_t pitch = pitch_override > 0 ? pitch_override : staged_pitch(rt);
  const size_t elem = rt.D == 1 ? 1 : 2;
  ctx->staged.device = ctx->device;
  ctx->staged.reserve((size_t)pitch * rt.nchan * elem + 256);
  dim3 grid((unsigned)((pitch + kStageT - 1) / kStageT), (unsigned)((rt.nchan + kStageC - 1) / kStageC));
  // bytes: the filterbank rows read once + the staged copy written once
  ProfScope prof(ctx, "stage", st, (double)rt.N * rt.D * rt.nchan + (double)pitch * rt.nchan * elem);
  const uintptr_t fa = reinterpret_cast<uintptr_t>(fb);
  // 16-byte loads need 16 channels per load and 16-byte rows; their 16-bit
  // half sums hold D <= 257 spectra of 255
  const int mode = (rt.nchan % 16 == 0 && fa % 16 == 0 && rt.D <= 257) ? 2 : ((rt.nchan % 4 == 0 && fa % 4 == 0) ? 1 : 0);
  if (rt.D == 1) {
    auto k = mode == 2 ? k_stage<uint8_t, 2> : (mode == 1 ? k_stage<uint8_t, 1> : k_stage<uint8_t, 0>);
    hipLaunchKernelGGL(k, grid, dim3(256), 0, st, fb, desc->nsamp, rt.nchan, rt.D, rt.N, ctx->staged.as<uint8_t>(),
                       pitch);
  } else {
    auto k = mode == 2 ? k_stage<uint16_t, 2> : (mode == 1 ? k_stage<uint16_t, 1> : k_stage<uint16_t, 0>);
    hipLaunchKernelGGL(k, grid, dim3(256), 0, st, fb, desc->nsamp, rt.nchan, rt.D, rt.N, ctx->staged.as<uint16_t>(),
                       pitch);
  }
  check_hip(hipGetLastError(), "launch staging kernel");
  ctx->staged_tag = {fb, desc->nsamp, pitch, rt.nchan, rt.D, nullptr};
}

void stage_raw(gsp_ctx *ctx, const uint8_t *fb, int64_t nsamp, int32_t nchan, int64_t pitch, hipStream_t st) {
  if (pitch < nsamp || pitch % 256) fail(GSP_EINVAL, "staging pitch");
  ctx->staged.device = ctx->device;
  ctx->staged.reserve((size_t)pitch * nchan + 256);
  dim3 grid((unsigned)((pitch + kStageT - 1) / kStageT), (unsigned)((nchan + kStageC - 1) / kStageC));
  ProfScope prof(ctx, "stage", st, (double)nsamp * nchan + (double)pitch * nchan);
  const uintptr_t fa = reinterpret_cast<uintptr_t>(fb);
  const int mode = (nchan % 16 == 0 && fa % 16 == 0) ? 2 : ((nchan % 4 == 0 && fa % 4 == 0) ? 1 : 0);
  auto k = mode == 2 ? k_stage<uint8_t, 2> : (mode == 1 ? k_stage<uint8_t, 1> : k_stage<uint8_t, 0>);
  hipLaunchKernelGGL(k, grid, dim3(256), 0, st, fb, nsamp, nchan, 1, nsamp, ctx->staged.as<uint8_t>(), pitch);
  check_hip(hipGetLastError(), "launch staging kernel");
  ctx->staged_tag = {fb, nsamp, pitch, nchan, 1, nullptr};
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
  if (rt.shape.kind != 0) {
    // a split row: the 16-bit tile's channels first, the byte-quad tile adds
    if (rt.shape.kind == 3) launch_dedisp(ctx, *rt.low, out_row, st);
    launch_dedisp_quad(ctx, rt, out_row, st);
    return;
  }
  const DedispShape &sh = rt.shape;
  DedispArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pitch = staged_pitch(rt);
  a.Y = static_cast<const uint8_t *>(ctx->staged.ptr) + (int64_t)rt.y_ch0 * a.pitch * (rt.D == 1 ? 1 : 2);
  a.addr = rt.addr.as<uint32_t>();
  a.base = rt.dmin.as<int32_t>();
  a.out = out_row;
  a.out_pitch = rt.n_out;
  a.t_origin = 0;
  a.t_lo = 0;
  a.t_hi = rt.n_out;
  a.ring = 0;
  a.phys0 = 0;
  a.n_dm = rt.n_dm;
  const int MT = sh.trials_per_block();
  a.n_dm_tiles = (rt.n_dm + MT - 1) / MT;
  a.n_dm_pad = a.n_dm_tiles * MT;
  a.nchan = rt.nchan;
  a.chunks = rt.passes.as<int32_t>();
  a.n_chunks = rt.n_passes;
  a.max_chunk = rt.max_chunk;
  a.data_dw = rt.data_dw;
  a.flush = flush_interval(rt.D);
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
