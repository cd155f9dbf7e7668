// Brute-force dedispersion of rows without downsampling (uint8 samples):
// the byte-quad tile.
//
// What is computed is the same as k_dedisp (paper Section 2.3): for every DM
// trial i and output sample t, out[i][t] = sum_c Y[c][t + d(i, c)], exact
// integers.
//
// How.  The 16-bit tile spends one LDS dword per two sample-adds; its LDS
// reads bound it.  Here an LDS dword holds four bytes: the samples of four
// neighbouring channels (a quad) that one trial adds into the same output,
// and one v_sad_u8 against zero adds all four into a 32-bit sum.  The four
// channels of a quad have different delays, so the dword a trial needs is
// the quad's samples at the shifts (d(i, c1) - d(i, c0), ...), its
// "pattern".  Over a tile of neighbouring trials a quad has only a few
// distinct patterns (the delay differences inside a quad change by well
// under a sample across the tile; the rounding of each delay gives the
// rest), so the tile stages one copy of the quad per pattern, covering the
// trials' spread of d(i, c0) plus the tile's outputs, and each trial reads
// its pattern's copy at its own d(i, c0).  That is one LDS byte per
// sample-add and a quarter of a VALU instruction, against two bytes and
// half an instruction for the 16-bit tile; staging costs one extra write of
// each copy (about a tenth of the reads on the realistic band).
//
// Per DM tile the host lists the copies (quad, start sample of each of its
// four channels) and groups consecutive quads into staging passes that fit
// the LDS; the per-(quad, trial) LDS offsets are precomputed as for
// k_dedisp.  A pass's copies are built in registers from the channel-major
// uint8 rows k_stage writes, 16 bytes (4 outputs of 4 channels) per thread
// at a time: one dword load per channel from its (unaligned) start, then a
// 4x4 byte transpose by v_perm.  Consecutive threads write consecutive 16-byte chunks, so the
// staging writes are free of LDS bank conflicts.
#include <algorithm>
#include <cstring>
#include <map>

#include "dedisp_tile.h"

namespace gsp {

struct QuadArgs {
  const uint8_t *Y;          // channel-major staged rows [nchan][pitch]
  int64_t pitch;
  const uint32_t *addr;      // [nq][n_dm_pad / 2] LDS dword offsets per (quad, trial) in their pass's
                             // buffer, two trials (2m, 2m + 1) per dword in its low and high halves
  const int32_t *tile_pass;  // [n_dm_tiles + 1] first pass record of each DM tile
  const int4 *passes;        // {first quad, first copy, chunks per copy, division magic}; a sentinel ends each tile
  const int4 *copies;        // per copy and channel: source byte offset from the pass's first row, at output 0
  int32_t *out;              // out[i * out_pitch + t]
  int64_t out_pitch, n_out;
  int32_t n_dm, n_dm_pad, n_dm_tiles, n_t_tiles;
  int32_t data_dw;           // LDS dwords of one buffer of staged copies (a multiple of 4)
  int32_t rec_dw;            // LDS dwords of one buffer of copy records (a multiple of 4)
  int32_t accumulate;        // add the sums to what out holds (the other part of a split row)
};

// Staging chunks per thread and pass (registers: 4 per chunk)
__host__ __device__ constexpr int quad_chunks(int K, int TPW) { return K * TPW >= 32 ? 5 : 8; }

// A dword load from any byte address (the code object assumes unaligned
// global access, as HSA configures it)
typedef uint32_t u32_unaligned __attribute__((aligned(1)));

// Staging: a pass's copies are split into 16-byte chunks (4 output samples
// of the quad's 4 channels); consecutive threads build consecutive chunks,
// so every LDS write of a wave covers 1 KB without bank conflicts.
template <int K, int TPW>
__global__ __launch_bounds__(1024) void k_dedisp_quad(QuadArgs a) {
  static_assert(TPW % 2 == 0 && TPW <= 8, "trials are read in pairs");
  constexpr int CM = quad_chunks(K, TPW);
  extern __shared__ __align__(16) uint32_t lds[];
  uint4 *lds4 = reinterpret_cast<uint4 *>(lds);  // 16-byte view: the chunk writes are ds_write_b128
  const int G = a.n_dm_tiles * a.n_t_tiles;
  const int L = xcd_remap(blockIdx.x, G);
  const int dm_tile = L % a.n_dm_tiles, t_tile = L / a.n_dm_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x;
  constexpr int T = 64 * K;
  const int t0 = t_tile * T;
  const int i_wave = dm_tile * TPW * (nthreads >> 6) + wave * TPW;
  const int p_first = a.tile_pass[dm_tile];
  const int n_pass = a.tile_pass[dm_tile + 1] - p_first - 1;
  // LDS: two buffers of staged copies, then two buffers of copy records;
  // pass j uses buffers j & 1, so the next pass is staged while this one is summed
  auto data_buf = [&](int j) { return lds + (j & 1) * a.data_dw; };
  auto rec_buf = [&](int j) { return reinterpret_cast<int4 *>(lds4 + ((2 * a.data_dw + (j & 1) * a.rec_dw) >> 2)); };

  // pass records, 64 at a time in registers (lane l: pass w0 + l), taken by readlane
  int w0 = 0;
  int4 win = make_int4(0, 0, 0, 0);
  auto fetch_window = [&](int from) {
    w0 = from;
    win = a.passes[p_first + min(from + lane, n_pass)];
  };
  auto q_begin = [&](int j) { return __builtin_amdgcn_readlane(win.x, j - w0); };
  auto c_begin = [&](int j) { return __builtin_amdgcn_readlane(win.y, j - w0); };
  auto chunks_of = [&](int j) { return __builtin_amdgcn_readlane(win.z, j - w0); };
  auto magic_of = [&](int j) { return (uint32_t)__builtin_amdgcn_readlane(win.w, j - w0); };
  fetch_window(0);

  int4 nrec = make_int4(0, 0, 0, 0);  // this thread's copy record of a coming pass
  uint32_t pw[CM][4];                 // per chunk and channel: its 4 samples
  uint32_t roff[TPW / 2], noff[TPW / 2];  // lane l: the wave's trial offsets at quad l of the pass, in pairs
  auto load_rec = [&](int j) {
    const int nc = c_begin(j + 1) - c_begin(j);
    nrec = a.copies[c_begin(j) + min(tid, nc - 1)];
  };
  auto put_rec = [&](int j) {
    if (tid < c_begin(j + 1) - c_begin(j)) rec_buf(j)[tid] = nrec;
  };
  auto load_data = [&](int j) {  // samples of pass j (its records in LDS) and its trial offsets
    const int CU = chunks_of(j);
    const uint32_t M = magic_of(j);
    const int nchk = (c_begin(j + 1) - c_begin(j)) * CU;
    const int qb = q_begin(j), qe = q_begin(j + 1);
    const uint8_t *base = a.Y + (int64_t)(4 * qb) * a.pitch;
    const int4 *rec_lds = rec_buf(j);
#pragma unroll
    for (int i = 0; i < CM; ++i) {
      const int g = min(tid + i * nthreads, nchk - 1);  // clamped: loads stay in bounds
      const int k = (int)__umulhi((uint32_t)g, M);      // g / CU (exact for these sizes)
      const int tc = t0 + 4 * (g + __mul24(k, -CU));    // t0 + 4 c: a multiple of 4
      const int4 r = rec_lds[k];
      const int rv[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) pw[i][ch] = *reinterpret_cast<const u32_unaligned *>(base + (uint32_t)(rv[ch] + tc));
    }
    const uint32_t *o = a.addr + (int64_t)(qb + min(lane, qe - qb - 1)) * (a.n_dm_pad >> 1) + (i_wave >> 1);
    if constexpr (TPW == 8) {
      const uint4 v = *reinterpret_cast<const uint4 *>(o);
      noff[0] = v.x;
      noff[1] = v.y;
      noff[2] = v.z;
      noff[3] = v.w;
    } else if constexpr (TPW == 4) {
      const uint2 v = *reinterpret_cast<const uint2 *>(o);
      noff[0] = v.x;
      noff[1] = v.y;
    } else {
      noff[0] = o[0];
    }
  };
  // registers -> LDS: chunk i of this thread (pass chunk g = tid + i *
  // nthreads) at dwords [4g, 4g + 4) of the pass's buffer; the chunks of a
  // wave's store cover consecutive 16-byte slots (no bank conflicts)
  auto store_chunk = [&](int j, int i) {
    const int nchk = (c_begin(j + 1) - c_begin(j)) * chunks_of(j);
    const int g = tid + i * nthreads;
    if (g < nchk) {
      const uint32_t *w = pw[i];  // w[ch]: the chunk's 4 samples of channel ch
      // 4x4 byte transpose: x01 interleaves channels 0 and 1, x23 channels 2 and 3
      // (selector byte k < 4: byte k of the second operand, 4..7: byte k-4 of the first)
      const uint32_t x01l = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);
      const uint32_t x01h = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);
      const uint32_t x23l = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
      const uint32_t x23h = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
      reinterpret_cast<uint4 *>(data_buf(j))[g] = make_uint4(
          __builtin_amdgcn_perm(x23l, x01l, 0x05040100u), __builtin_amdgcn_perm(x23l, x01l, 0x07060302u),
          __builtin_amdgcn_perm(x23h, x01h, 0x05040100u), __builtin_amdgcn_perm(x23h, x01h, 0x07060302u));
    }
  };
  auto store = [&](int j) {
#pragma unroll
    for (int i = 0; i < CM; ++i) store_chunk(j, i);
  };

  uint32_t acc[TPW][K];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[t][k] = 0;

  const uint32_t *cur = lds;  // buffer of the pass being summed
  auto ld = [&](int q, int t, uint32_t *v) {  // trial t's dwords of quad q (q uniform)
    // one readlane per two trials; the halves are split on the scalar unit
    const uint32_t pair = (uint32_t)__builtin_amdgcn_readlane((int)roff[t >> 1], q);
    const uint32_t o = (t & 1) ? pair >> 16 : pair & 0xFFFFu;
    const uint32_t *src = cur + o + lane;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = src[64 * k];
  };
  auto add = [&](const uint32_t *v, int t) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[t][k] = __builtin_amdgcn_sad_u8(v[k], 0u, acc[t][k]);
  };

  // ---- prologue: pass 0 staged, records of pass 1 in LDS ----
  load_rec(0);
  put_rec(0);
  __syncthreads();
  load_data(0);
  if (n_pass > 1) load_rec(1);
  store(0);
  if (n_pass > 1) put_rec(1);
  __syncthreads();

  for (int kc = 0; kc < n_pass; ++kc) {
    if (kc + 3 > w0 + 63) fetch_window(kc);  // records kc .. kc + 3 are read below
#pragma unroll
    for (int t = 0; t < TPW / 2; ++t) roff[t] = noff[t];
    if (kc + 1 < n_pass) load_data(kc + 1);  // samples of the next pass in flight
    if (kc + 2 < n_pass) load_rec(kc + 2);

    // ---- accumulate pass kc: per quad TPW trials x K dwords per lane, the
    // next trial's dwords in flight while one is added ----
    cur = data_buf(kc);
    const int last = q_begin(kc + 1) - q_begin(kc) - 1;
    uint32_t va[K], vb[K];
    ld(0, 0, va);
    for (int q = 0; q <= last; ++q) {
      const int qn = min(q + 1, last);
#pragma unroll
      for (int t = 0; t < TPW; t += 2) {
        ld(q, t + 1, vb);
        add(va, t);
        if (t + 2 < TPW)
          ld(q, t + 2, va);
        else
          ld(qn, 0, va);
        add(vb, t + 1);
      }
    }
    // stage the next pass into the other buffers (last read in pass kc - 1)
    if (kc + 1 < n_pass) store(kc + 1);
    if (kc + 2 < n_pass) put_rec(kc + 2);
    __syncthreads();
  }

#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int i = i_wave + t;
    if (i >= a.n_dm) break;
    int32_t *orow = a.out + (int64_t)i * a.out_pitch;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t tt = (int64_t)t0 + lane + 64 * k;
      if (tt < a.n_out) orow[tt] = (int32_t)acc[t][k] + (a.accumulate ? orow[tt] : 0);
    }
  }
}

// The same tile with the work split by waves: NP staging waves fill the
// next pass's LDS buffer while the other waves sum the current one (all
// waves meet at one barrier per pass).  The summing waves never wait for a
// global load; the staging waves keep R chunks per thread in flight, their
// copy records one batch ahead.
__device__ __forceinline__ void wg_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int K, int TPW, int NP>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) void k_dedisp_quad_pc(QuadArgs a) {
  static_assert(TPW % 2 == 0 && TPW <= 8, "trials are read in pairs");
  extern __shared__ __align__(16) uint32_t lds[];
  const int G = a.n_dm_tiles * a.n_t_tiles;
  const int L = xcd_remap(blockIdx.x, G);
  const int dm_tile = L % a.n_dm_tiles, t_tile = L / a.n_dm_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int NC = (int)(blockDim.x >> 6) - NP;  // summing waves
  constexpr int T = 64 * K;
  const int t0 = t_tile * T;
  const int p_first = a.tile_pass[dm_tile];
  const int n_pass = a.tile_pass[dm_tile + 1] - p_first - 1;
  auto data_buf = [&](int j) { return lds + (j & 1) * a.data_dw; };

  int w0 = 0;
  int4 win = make_int4(0, 0, 0, 0);
  auto fetch_window = [&](int from) {
    w0 = from;
    win = a.passes[p_first + min(from + lane, n_pass)];
  };
  auto q_begin = [&](int j) { return __builtin_amdgcn_readlane(win.x, j - w0); };
  auto c_begin = [&](int j) { return __builtin_amdgcn_readlane(win.y, j - w0); };
  auto chunks_of = [&](int j) { return __builtin_amdgcn_readlane(win.z, j - w0); };
  auto magic_of = [&](int j) { return (uint32_t)__builtin_amdgcn_readlane(win.w, j - w0); };
  fetch_window(0);

  if (wave >= NC) {
    // ---- staging waves ----
    constexpr int PT = 64 * NP;
    constexpr int R = 4;  // chunks per thread in flight
    const int ptid = tid - 64 * NC;
    auto stage = [&](int j) {
      const int cb = c_begin(j), CU = chunks_of(j);
      const uint32_t M = magic_of(j);
      const int nchk = (c_begin(j + 1) - cb) * CU;
      const uint8_t *base = a.Y + (int64_t)(4 * q_begin(j)) * a.pitch;
      uint4 *dst4 = reinterpret_cast<uint4 *>(data_buf(j));
      int4 rec[R];
      int tcs[R];
      auto fetch_rec = [&](int g0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int g = min(g0 + r * PT, nchk - 1);  // clamped: loads stay in bounds
          const int k = (int)__umulhi((uint32_t)g, M);
          tcs[r] = t0 + 4 * (g + __mul24(k, -CU));
          rec[r] = a.copies[cb + k];
        }
      };
      fetch_rec(ptid);
      for (int g0 = ptid; g0 < nchk; g0 += R * PT) {
        uint32_t w[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rv[4] = {rec[r].x, rec[r].y, rec[r].z, rec[r].w};
#pragma unroll
          for (int ch = 0; ch < 4; ++ch)
            w[r][ch] = *reinterpret_cast<const u32_unaligned *>(base + (uint32_t)(rv[ch] + tcs[r]));
        }
        if (g0 + R * PT < nchk) fetch_rec(g0 + R * PT);  // the next batch's records in flight
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int g = g0 + r * PT;
          if (g < nchk) {
            const uint32_t x01l = __builtin_amdgcn_perm(w[r][1], w[r][0], 0x05010400u);
            const uint32_t x01h = __builtin_amdgcn_perm(w[r][1], w[r][0], 0x07030602u);
            const uint32_t x23l = __builtin_amdgcn_perm(w[r][3], w[r][2], 0x05010400u);
            const uint32_t x23h = __builtin_amdgcn_perm(w[r][3], w[r][2], 0x07030602u);
            dst4[g] = make_uint4(
                __builtin_amdgcn_perm(x23l, x01l, 0x05040100u), __builtin_amdgcn_perm(x23l, x01l, 0x07060302u),
                __builtin_amdgcn_perm(x23h, x01h, 0x05040100u), __builtin_amdgcn_perm(x23h, x01h, 0x07060302u));
          }
        }
      }
    };
    stage(0);
    wg_barrier();  // pass 0 staged
    for (int kc = 0; kc < n_pass; ++kc) {
      if (kc + 3 > w0 + 63) fetch_window(kc);
      if (kc + 1 < n_pass) stage(kc + 1);  // into the buffer pass kc - 1 used
      wg_barrier();                        // pass kc summed, pass kc + 1 staged
    }
    return;
  }

  // ---- summing waves: as in k_dedisp_quad ----
  const int i_wave = dm_tile * TPW * NC + wave * TPW;
  uint32_t roff[TPW / 2], noff[TPW / 2];
  auto load_off = [&](int j) {
    const int qb = q_begin(j), qe = q_begin(j + 1);
    const uint32_t *o = a.addr + (int64_t)(qb + min(lane, qe - qb - 1)) * (a.n_dm_pad >> 1) + (i_wave >> 1);
    if constexpr (TPW == 8) {
      const uint4 v = *reinterpret_cast<const uint4 *>(o);
      noff[0] = v.x;
      noff[1] = v.y;
      noff[2] = v.z;
      noff[3] = v.w;
    } else if constexpr (TPW == 4) {
      const uint2 v = *reinterpret_cast<const uint2 *>(o);
      noff[0] = v.x;
      noff[1] = v.y;
    } else {
      noff[0] = o[0];
    }
  };
  uint32_t acc[TPW][K];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[t][k] = 0;
  const uint32_t *cur = lds;
  auto ld = [&](int q, int t, uint32_t *v) {
    const uint32_t pair = (uint32_t)__builtin_amdgcn_readlane((int)roff[t >> 1], q);
    const uint32_t o = (t & 1) ? pair >> 16 : pair & 0xFFFFu;
    const uint32_t *src = cur + o + lane;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = src[64 * k];
  };
  auto add = [&](const uint32_t *v, int t) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[t][k] = __builtin_amdgcn_sad_u8(v[k], 0u, acc[t][k]);
  };
  load_off(0);
  wg_barrier();  // pass 0 staged
  for (int kc = 0; kc < n_pass; ++kc) {
    if (kc + 3 > w0 + 63) fetch_window(kc);
#pragma unroll
    for (int t = 0; t < TPW / 2; ++t) roff[t] = noff[t];
    if (kc + 1 < n_pass) load_off(kc + 1);
    cur = data_buf(kc);
    const int last = q_begin(kc + 1) - q_begin(kc) - 1;
    uint32_t va[K], vb[K];
    ld(0, 0, va);
    for (int q = 0; q <= last; ++q) {
      const int qn = min(q + 1, last);
#pragma unroll
      for (int t = 0; t < TPW; t += 2) {
        ld(q, t + 1, vb);
        add(va, t);
        if (t + 2 < TPW)
          ld(q, t + 2, va);
        else
          ld(qn, 0, va);
        add(vb, t + 1);
      }
    }
    wg_barrier();  // pass kc summed, pass kc + 1 staged
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int i = i_wave + t;
    if (i >= a.n_dm) break;
    int32_t *orow = a.out + (int64_t)i * a.out_pitch;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t tt = (int64_t)t0 + lane + 64 * k;
      if (tt < a.n_out) orow[tt] = (int32_t)acc[t][k] + (a.accumulate ? orow[tt] : 0);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static constexpr int64_t kQuadLdsBudget = 80 * 1024;  // two workgroups per CU
static constexpr int64_t kQuadLdsMax = 160 * 1024;
static constexpr int kQuadPassMax = 64;               // quads per pass: one per lane for the offsets
static constexpr int kQuadRecMax = 128;               // copies per pass (their records share the LDS)

static constexpr int kQuadStagingWaves = 4;  // kind 2: staging waves besides the summing ones
// kind 3: quads whose staged copies exceed this fraction of the dwords their
// trials read go to the 16-bit tile with those that do not fit (a pass of
// such quads keeps the summing waves waiting for its staging)
static constexpr double kQuadSplitStaged = 0.25;

bool quad_shape_supported(const DedispShape &s) {
  const int kt = s.groups * 16 + s.tpw;
  if (s.kind == 2 || s.kind == 3)
    return (kt == 8 * 16 + 4 || kt == 4 * 16 + 8) && s.waves >= 1 && s.waves + kQuadStagingWaves <= 16 &&
           s.chunk >= 1;
  const bool inst = kt == 8 * 16 + 4 || kt == 8 * 16 + 2 || kt == 4 * 16 + 8 || kt == 16 * 16 + 2 ||
                    kt == 4 * 16 + 4;
  return s.kind == 1 && inst && s.waves >= 1 && s.waves <= 16 && s.chunk >= 1;
}

// The distinct delay patterns of quad q over the trials [i0, i0 + MT) (the
// last trial repeated past n_dm): pattern k = delay differences (d1, d2, d3)
// of channels 4q+1..3 from channel 4q, with the range [lo, hi] of the first
// channel's delay over its trials; pat_of[j] = the pattern of trial i0 + j.
struct QuadPat {
  int32_t d1, d2, d3, lo, hi;
};
template <class DELAY>
static void quad_patterns(DELAY delay, int i0, int MT, int q, std::vector<QuadPat> &P, uint8_t *pat_of) {
  P.clear();
  for (int j = 0; j < MT; ++j) {
    const int i = i0 + j;
    const int32_t o0 = delay(i, 4 * q), d1 = delay(i, 4 * q + 1) - o0, d2 = delay(i, 4 * q + 2) - o0,
                  d3 = delay(i, 4 * q + 3) - o0;
    size_t k = 0;
    while (k < P.size() && !(P[k].d1 == d1 && P[k].d2 == d2 && P[k].d3 == d3)) ++k;
    if (k == P.size()) {
      if (k == 255) fail(GSP_EINVAL, "too many delay patterns in a quad");
      P.push_back({d1, d2, d3, o0, o0});
    } else {
      P[k].lo = std::min(P[k].lo, o0);
      P[k].hi = std::max(P[k].hi, o0);
    }
    pat_of[j] = (uint8_t)k;
  }
}

// LDS dwords of staged copies one pass may hold (the two buffers share the
// workgroup's LDS budget; kinds 2 and 3 keep no copy records in LDS)
static int64_t quad_pass_dwords(const DedispShape &sh) {
  const bool pc = sh.kind == 2 || sh.kind == 3;
  const int rec_cap = pc ? INT32_MAX : std::min(64 * sh.waves, kQuadRecMax);
  // two workgroups per CU: up to 8 waves in kind 1, and in kinds 2 and 3 up
  // to 12 summing waves (with the 4 staging waves two 16-wave workgroups of
  // 60 VGPRs fill a CU, 4 waves per SIMD each); kind 1 above 8: one (160 KB)
  const int64_t budget = (pc || sh.waves <= 8) ? kQuadLdsBudget : kQuadLdsMax;
  return (budget / 4 - (pc ? 0 : 2 * 4 * (int64_t)rec_cap)) / 2;
}

void quad_split(const RowTables &rt, int32_t *c0, int32_t *c1) {
  const DedispShape &sh = rt.shape;
  if (rt.D != 1 || rt.nchan % 4) fail(GSP_EINVAL, "the byte-quad tile sums uint8 rows of whole channel quads");
  const int nchan = rt.nchan, nq = nchan / 4, n_dm = rt.n_dm, MT = sh.trials_per_block();
  const int T = 64 * sh.groups;
  const int64_t dw_cap = quad_pass_dwords(sh);
  const int32_t *d = rt.delays_host.data();
  auto delay = [&](int i, int c) { return d[(int64_t)std::min(i, n_dm - 1) * nchan + c]; };
  // a quad fits if its copies of every DM tile fit one pass (chunk count
  // per copy as the table builder rounds it, every copy at the longest); it
  // suits the tile if they also stay below kQuadSplitStaged of the dwords
  // the tile's trials read from them
  std::vector<uint8_t> fits(nq, 1), suits(nq, 1);
  std::vector<QuadPat> P;
  std::vector<uint8_t> pat_of(MT);
  const double reads = (double)MT * T;
  for (int i0 = 0; i0 < n_dm; i0 += MT)
    for (int q = 0; q < nq; ++q) {
      if (!fits[q]) continue;
      quad_patterns(delay, i0, MT, q, P, pat_of.data());
      int64_t cu = 0;
      for (const QuadPat &p : P) cu = std::max<int64_t>(cu, (p.hi - p.lo + T + 3) / 4);
      const int64_t staged = (int64_t)P.size() * cu * 4;
      if (staged > dw_cap) fits[q] = suits[q] = 0;
      if ((double)staged > kQuadSplitStaged * reads) suits[q] = 0;
    }
  if (std::all_of(fits.begin(), fits.end(), [](uint8_t f) { return f != 0; }))
    fail(GSP_EINVAL, "every channel quad fits: the split tile does not apply");
  int first_bad = nq, last_bad = -1;
  for (int q = 0; q < nq; ++q)
    if (!suits[q]) {
      first_bad = std::min(first_bad, q);
      last_bad = q;
    }
  // the 16-bit tile takes the shorter end run holding every quad that does
  // not fit: [0, last_bad] or [first_bad, nq)
  if (last_bad + 1 <= nq - first_bad) {
    *c0 = 4 * (last_bad + 1);
    *c1 = nchan;
  } else {
    *c0 = 0;
    *c1 = 4 * first_bad;
  }
  if (*c1 <= *c0) fail(GSP_EINVAL, "no channel quad fits the byte-quad tile");
}

void quad_tables_host(const RowTables &rt, QuadHost &H, int64_t min_pitch) {
  const DedispShape &sh = rt.shape;
  if (rt.D != 1) fail(GSP_EINVAL, "the byte-quad tile sums uint8 rows only (D = 1)");
  if (rt.nchan % 4) fail(GSP_EINVAL, "the byte-quad tile needs a multiple of 4 channels");
  if (!quad_shape_supported(sh)) fail(GSP_EINVAL, "unsupported dedispersion shape");
  const int nchan = rt.nchan, nq = nchan / 4, n_dm = rt.n_dm;
  const int MT = sh.trials_per_block();
  const int n_tiles = (n_dm + MT - 1) / MT;
  const int n_dm_pad = n_tiles * MT;
  const int T = 64 * sh.groups;
  const bool pc = sh.kind == 2 || sh.kind == 3;  // staging waves: no register or record limit on a pass
  const int threads = 64 * sh.waves;
  const int64_t chunk_cap = pc ? INT32_MAX : (int64_t)quad_chunks(sh.groups, sh.tpw) * threads;  // chunks per pass
  const int rec_cap = pc ? INT32_MAX : std::min(threads, kQuadRecMax);
  const int64_t dw_cap = quad_pass_dwords(sh);  // LDS dwords of copies per pass
  const int64_t n_t = (rt.n_out + T - 1) / T;
  if ((n_t - 1) * T + rt.max_delay + dw_cap + 1024 >= (1LL << 30))
    fail(GSP_EINVAL, "row too long for the byte-quad tile's 32-bit offsets");
  // a pass's source offsets (from its first row) stay below 2^31
  const int64_t pitch_ub =
      (std::max<int64_t>({rt.N, (n_t - 1) * T + rt.max_delay + dw_cap + 8, min_pitch}) + 255) / 256 * 256;
  const int64_t q_fit = ((1LL << 31) - 1 - pitch_ub) / (4 * pitch_ub);
  const int max_q = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)sh.chunk, kQuadPassMax, q_fit}));
  if (q_fit < 1) fail(GSP_EINVAL, "row too long for the byte-quad tile's 32-bit offsets");
  const int32_t *d = rt.delays_host.data();
  auto delay = [&](int i, int c) { return d[(int64_t)std::min(i, n_dm - 1) * nchan + c]; };

  H.tile_pass.clear();
  H.passes.clear();
  H.copies.clear();
  H.addr.assign((size_t)nq * (n_dm_pad / 2), 0);
  std::vector<int32_t> cp_start;  // per copy: start sample of each channel (offsets need the final pitch)
  std::vector<int32_t> cp_q, cp_qb;
  int64_t max_dw = 0, max_cu = 0;
  int rec_max = 1;
  double staged = 0;

  using Pat = QuadPat;
  std::vector<std::vector<Pat>> pats(nq);
  std::vector<std::vector<uint8_t>> pat_of(nq, std::vector<uint8_t>(MT));
  for (int tl = 0; tl < n_tiles; ++tl) {
    const int i0 = tl * MT;
    for (int q = 0; q < nq; ++q) quad_patterns(delay, i0, MT, q, pats[q], pat_of[q].data());
    // passes: consecutive quads while their copies (all at the pass's
    // largest chunk count) fit the LDS budget, the staging registers and
    // the record area
    H.tile_pass.push_back((int32_t)(H.passes.size() / 4));
    int q = 0;
    while (q < nq) {
      int qe = q;
      int64_t n_cp = 0, CU = 0;
      while (qe < nq && qe - q < max_q) {
        int64_t cu2 = CU;
        for (const Pat &p : pats[qe]) cu2 = std::max<int64_t>(cu2, (p.hi - p.lo + T + 3) / 4);
        const int64_t n2 = n_cp + (int64_t)pats[qe].size();
        const bool fits = n2 * cu2 <= chunk_cap && n2 * cu2 * 4 <= dw_cap && n2 <= rec_cap;
        if (!fits) {
          if (qe == q) fail(GSP_EINVAL, "a channel quad's delay copies do not fit the byte-quad tile");
          break;
        }
        n_cp = n2;
        CU = cu2;
        ++qe;
      }
      // g / CU as the high half of g * M for every chunk index g of the pass
      const uint64_t M = ((1ULL << 32) + (uint64_t)CU - 1) / (uint64_t)CU;
      for (int64_t g = CU - 1; g < n_cp * CU; g += CU)
        if ((int64_t)((g * M) >> 32) != g / CU || (int64_t)(((g + 1) * M) >> 32) != (g + 1) / CU)
          fail(GSP_EINVAL, "byte-quad division magic");
      H.passes.push_back(q);
      H.passes.push_back((int32_t)cp_q.size());
      H.passes.push_back((int32_t)CU);
      H.passes.push_back((int32_t)(uint32_t)M);
      int32_t slot = 0;
      for (int qq = q; qq < qe; ++qq) {
        const auto &P = pats[qq];
        for (size_t k = 0; k < P.size(); ++k) {
          cp_start.push_back(P[k].lo);
          cp_start.push_back(P[k].lo + P[k].d1);
          cp_start.push_back(P[k].lo + P[k].d2);
          cp_start.push_back(P[k].lo + P[k].d3);
          cp_q.push_back(qq);
          cp_qb.push_back(q);
        }
        for (int j = 0; j < MT; ++j) {
          const Pat &p = P[pat_of[qq][j]];
          const int32_t o0 = delay(i0 + j, 4 * qq);
          const int64_t off = (int64_t)(slot + pat_of[qq][j]) * CU * 4 + (o0 - p.lo);
          if (off >= 65536) fail(GSP_EINVAL, "byte-quad LDS offset beyond 16 bits");
          H.addr[(size_t)qq * (n_dm_pad / 2) + (i0 + j) / 2] |= (uint32_t)off << (16 * ((i0 + j) & 1));
        }
        slot += (int32_t)P.size();
      }
      max_dw = std::max(max_dw, n_cp * CU * 4);
      max_cu = std::max(max_cu, CU);
      rec_max = std::max<int>(rec_max, (int)n_cp);
      staged += (double)n_cp * CU * 4;
      q = qe;
    }
    H.passes.push_back(nq);  // sentinel
    H.passes.push_back((int32_t)cp_q.size());
    H.passes.push_back(0);
    H.passes.push_back(0);
  }
  H.tile_pass.push_back((int32_t)(H.passes.size() / 4));
  if (cp_q.size() >= (size_t)INT32_MAX / 4) fail(GSP_EOVERFLOW, "byte-quad tables too large");

  // staged pitch: a chunk reads 4 bytes from sample t0 + s + 4 c with
  // s <= max_delay and c below the pass's chunk count
  const int64_t far = (n_t - 1) * T + rt.max_delay + 4 * max_cu + 8;
  H.pitch = (std::max({far, rt.N, min_pitch}) + 255) / 256 * 256;
  if (H.pitch > pitch_ub) fail(GSP_EINVAL, "byte-quad pitch bound");
  H.copies.resize(cp_start.size());
  for (size_t k = 0; k < cp_q.size(); ++k)
    for (int ch = 0; ch < 4; ++ch)
      H.copies[4 * k + ch] = (int32_t)((int64_t)(4 * (cp_q[k] - cp_qb[k]) + ch) * H.pitch + cp_start[4 * k + ch]);
  H.lds_dw = max_dw;
  H.rec_max = rec_max;
  H.staged = staged;
  H.max_q = max_q;
}

// Columns [c0, c1) of a row's delay table
static std::vector<int32_t> delay_columns(const RowTables &rt, int32_t c0, int32_t c1) {
  std::vector<int32_t> out((size_t)rt.n_dm * (c1 - c0));
  for (int32_t i = 0; i < rt.n_dm; ++i)
    std::copy(rt.delays_host.begin() + (int64_t)i * rt.nchan + c0, rt.delays_host.begin() + (int64_t)i * rt.nchan + c1,
              out.begin() + (int64_t)i * (c1 - c0));
  return out;
}

void build_quad_tables(gsp_ctx *ctx, RowTables &rt) {
  QuadHost H;
  if (rt.shape.kind == 3) {
    // split row: the byte-quad tile over [c0, c1), the 16-bit tile (default
    // shape) over the channels at the other end; one staging of the whole
    // row at a pitch both accept
    int32_t c0 = 0, c1 = 0;
    quad_split(rt, &c0, &c1);
    const int32_t l0 = c0 > 0 ? 0 : c1, l1 = c0 > 0 ? c0 : rt.nchan;
    auto low = std::make_unique<RowTables>();
    low->delays_host = delay_columns(rt, l0, l1);
    DedispShape ps;  // the 16-bit tile's default: (4, 4, 8, 32)
    ps.groups = 4;
    ps.tpw = 4;
    ps.waves = 8;
    ps.chunk = 32;
    ps.kind = 0;
    build_tables_from_delays(ctx, rt.n_dm, l1 - l0, rt.D, rt.N, rt.n_out, rt.max_delay, ps, *low);
    low->y_ch0 = l0;
    RowTables sub;  // the byte-quad part as a row of its own
    sub.n_dm = rt.n_dm;
    sub.D = rt.D;
    sub.nchan = c1 - c0;
    sub.N = rt.N;
    sub.n_out = rt.n_out;
    sub.max_delay = rt.max_delay;
    sub.shape = rt.shape;
    sub.delays_host = delay_columns(rt, c0, c1);
    quad_tables_host(sub, H, staged_pitch(*low));
    low->pitch_override = H.pitch;
    rt.y_ch0 = c0;
    rt.low = std::move(low);
  } else {
    quad_tables_host(rt, H);
  }
  rt.q_pitch = H.pitch;
  rt.data_dw = (int32_t)H.lds_dw;
  rt.q_rec_dw = (rt.shape.kind == 2 || rt.shape.kind == 3) ? 0 : 4 * H.rec_max;
  rt.lds_bytes = 2 * (H.lds_dw + rt.q_rec_dw) * 4;
  rt.q_staged_dw = H.staged;
  rt.max_chunk = H.max_q;
  rt.shape.chunk = H.max_q;
  rt.n_passes = (int32_t)(H.passes.size() / 4);
  auto upload = [&](DevBuf &b, const void *src, size_t bytes, const char *what) {
    b.device = ctx->device;
    b.reserve(std::max<size_t>(bytes, 16));
    check_hip(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice), what);
  };
  upload(rt.q_tile_pass, H.tile_pass.data(), H.tile_pass.size() * 4, "copy quad pass index");
  upload(rt.q_passes, H.passes.data(), H.passes.size() * 4, "copy quad passes");
  upload(rt.q_copies, H.copies.data(), H.copies.size() * 4, "copy quad copies");
  upload(rt.addr, H.addr.data(), H.addr.size() * 4, "copy quad LDS offsets");
}

template <int K, int TPW>
static void launch_q(const QuadArgs &a, int waves, int64_t lds, hipStream_t st) {
  auto kern = k_dedisp_quad<K, TPW>;
  check_hip(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
            "set LDS size");
  hipLaunchKernelGGL(kern, dim3(a.n_dm_tiles * a.n_t_tiles), dim3(64 * waves), (size_t)lds, st, a);
}

template <int K, int TPW>
static void launch_qpc(const QuadArgs &a, int waves, int64_t lds, hipStream_t st) {
  auto kern = k_dedisp_quad_pc<K, TPW, kQuadStagingWaves>;
  check_hip(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
            "set LDS size");
  hipLaunchKernelGGL(kern, dim3(a.n_dm_tiles * a.n_t_tiles), dim3(64 * (waves + kQuadStagingWaves)), (size_t)lds, st,
                     a);
}

void launch_dedisp_quad(gsp_ctx *ctx, const RowTables &rt, int32_t *out_row, hipStream_t st) {
  const DedispShape &sh = rt.shape;
  QuadArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Y = ctx->staged.as<uint8_t>() + (int64_t)rt.y_ch0 * rt.q_pitch;
  a.pitch = rt.q_pitch;
  a.accumulate = sh.kind == 3 ? 1 : 0;  // after the 16-bit tile's part of the row
  a.addr = rt.addr.as<uint32_t>();
  a.tile_pass = rt.q_tile_pass.as<int32_t>();
  a.passes = rt.q_passes.as<int4>();
  a.copies = rt.q_copies.as<int4>();
  a.out = out_row;
  a.out_pitch = rt.n_out;
  a.n_out = rt.n_out;
  a.n_dm = rt.n_dm;
  a.data_dw = rt.data_dw;
  a.rec_dw = rt.q_rec_dw;
  const int MT = sh.trials_per_block();
  a.n_dm_tiles = (rt.n_dm + MT - 1) / MT;
  a.n_dm_pad = a.n_dm_tiles * MT;
  const int64_t T = sh.samples_per_block();
  const int64_t n_t = (rt.n_out + T - 1) / T;
  if ((int64_t)a.n_dm_tiles * n_t >= (1LL << 31)) fail(GSP_EOVERFLOW, "too many dedispersion tiles");
  a.n_t_tiles = (int32_t)n_t;
  const int32_t qch = rt.low ? rt.nchan - rt.low->nchan : rt.nchan;  // channels of this tile
  ProfScope prof(ctx, "dedisperse_quad", st, (double)rt.n_dm * (double)rt.n_out * (double)qch);
  if (sh.kind == 2 || sh.kind == 3) {
    switch (sh.groups * 16 + sh.tpw) {
      case 8 * 16 + 4: launch_qpc<8, 4>(a, sh.waves, rt.lds_bytes, st); break;
      case 4 * 16 + 8: launch_qpc<4, 8>(a, sh.waves, rt.lds_bytes, st); break;
      default: fail(GSP_EINVAL, "unsupported dedispersion shape");
    }
    check_hip(hipGetLastError(), "launch dedispersion kernel");
    return;
  }
  switch (sh.groups * 16 + sh.tpw) {
    case 8 * 16 + 4: launch_q<8, 4>(a, sh.waves, rt.lds_bytes, st); break;
    case 8 * 16 + 2: launch_q<8, 2>(a, sh.waves, rt.lds_bytes, st); break;
    case 4 * 16 + 8: launch_q<4, 8>(a, sh.waves, rt.lds_bytes, st); break;
    case 4 * 16 + 4: launch_q<4, 4>(a, sh.waves, rt.lds_bytes, st); break;
    case 16 * 16 + 2: launch_q<16, 2>(a, sh.waves, rt.lds_bytes, st); break;
    default: fail(GSP_EINVAL, "unsupported dedispersion shape");
  }
  check_hip(hipGetLastError(), "launch dedispersion kernel");
}

}  // namespace gsp
