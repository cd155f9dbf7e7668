// RFI mitigation of a uint8 filterbank in integers (paper Section 2.1 lists
// RFI mitigation among the search steps; Section 3.1 tests PRESTO's clip
// option on CPU and GPU).  What is computed:
//   clip (clip_sigma > 0): spectra in blocks of `block` (the last may be
//     shorter).  Per block the zero-DM series s_j = sum_c x[j][c] has
//     population mean mu and sigma from exact integer moments about its
//     first value; spectrum j is flagged when |s_j - mu| > clip_sigma *
//     sigma (double).  If some but not all spectra of the block are
//     flagged, each flagged spectrum becomes the block's channel means over
//     its unflagged spectra, m_c = floor((2 S_c + n_u) / (2 n_u)).
//   zero-DM filter (zero_dm != 0), after clipping: z_j = floor((2 s'_j +
//     nchan) / (2 nchan)) of the (clipped) spectrum's sum s'_j is
//     subtracted and 128 added back, clamped to 0..255.
// Design: four HBM-bound passes.  One wave per spectrum forms s_j (16-byte
// loads, byte sums by v_sad_u8, DPP reduction); one workgroup per block
// takes the moments (int64 / 128-bit sums) and flags; channel means are
// read only for blocks that replace something; a last pass writes the
// replaced spectra and applies the filter, in place if out == in.
#include <algorithm>
#include <cmath>

#include "gsp_internal.h"

namespace gsp {
namespace {

constexpr int kRfiThreads = 256;

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t bytes_sum(uint32_t w, uint32_t acc) {
  return __builtin_amdgcn_sad_u8(w, 0u, acc);  // sum of the 4 bytes of w, plus acc
}

// s[j] = sum_c x[j][c]: one wave per spectrum (grid-stride over spectra).
__global__ __launch_bounds__(kRfiThreads) void k_rfi_rowsum(const uint8_t *__restrict__ x, int64_t nsamp,
                                                           int32_t nchan, int vec, int32_t *__restrict__ s) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kRfiThreads + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kRfiThreads) >> 6;
  for (int64_t j = w0; j < nsamp; j += nw) {
    const uint8_t *row = x + j * (int64_t)nchan;
    uint32_t acc = 0;
    if (vec) {  // nchan % 16 == 0, 16-byte aligned rows
      const uint4 *r4 = reinterpret_cast<const uint4 *>(row);
      for (int k = lane; k < nchan / 16; k += 64) {
        const uint4 q = r4[k];
        acc = bytes_sum(q.x, acc);
        acc = bytes_sum(q.y, acc);
        acc = bytes_sum(q.z, acc);
        acc = bytes_sum(q.w, acc);
      }
    } else {
      for (int c = lane; c < nchan; c += 64) acc += row[c];
    }
    const int32_t t = wave_sum_i32((int32_t)acc);
    if (lane == 0) s[j] = t;
  }
}

// One workgroup per block: moments, flags, unflagged count.  A block that
// would replace nothing (no spectrum or every spectrum flagged) clears its
// flags, so the later passes leave it alone.
__global__ __launch_bounds__(kRfiThreads) void k_rfi_flags(const int32_t *__restrict__ s, int64_t nsamp,
                                                          int64_t block, double clip, uint8_t *__restrict__ flag,
                                                          int32_t *__restrict__ n_u,
                                                          unsigned long long *__restrict__ n_flagged) {
  __shared__ int64_t r1[kRfiThreads];
  __shared__ unsigned __int128 r2[kRfiThreads];
  __shared__ int32_t rc[kRfiThreads];
  __shared__ double musig[2];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t j0 = b * block;
  const int64_t n = min(block, nsamp - j0);
  const int64_t x0 = s[j0];
  int64_t s1 = 0;
  unsigned __int128 s2 = 0;
  for (int64_t k = tid; k < n; k += kRfiThreads) {
    const int64_t v = (int64_t)s[j0 + k] - x0;
    s1 += v;
    const uint64_t a = (uint64_t)(v < 0 ? -v : v);
    s2 += (unsigned __int128)(a * a);
  }
  r1[tid] = s1;
  r2[tid] = s2;
  __syncthreads();
  for (int h = kRfiThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      r1[tid] += r1[tid + h];
      r2[tid] += r2[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double dn = (double)n;
    const double m1 = (double)r1[0] / dn, m2 = (double)r2[0] / dn;
    const double var = m2 - m1 * m1;
    musig[0] = (double)x0 + m1;
    musig[1] = var > 0.0 ? sqrt(var) : 0.0;
  }
  __syncthreads();
  const double mu = musig[0], sigma = musig[1];
  int32_t unflagged = 0;
  for (int64_t k = tid; k < n; k += kRfiThreads) {
    const bool f = sigma > 0.0 && fabs((double)s[j0 + k] - mu) > clip * sigma;
    flag[j0 + k] = f ? 1 : 0;
    unflagged += f ? 0 : 1;
  }
  rc[tid] = unflagged;
  __syncthreads();
  for (int h = kRfiThreads / 2; h > 0; h >>= 1) {
    if (tid < h) rc[tid] += rc[tid + h];
    __syncthreads();
  }
  const int32_t nu = rc[0];
  const bool replace = nu > 0 && nu < n;
  if (!replace)
    for (int64_t k = tid; k < n; k += kRfiThreads) flag[j0 + k] = 0;
  if (tid == 0) {
    n_u[b] = replace ? nu : (int32_t)n;
    if (replace) atomicAdd(n_flagged, (unsigned long long)(n - nu));
  }
}

// Channel means over the unflagged spectra of blocks that replace some:
// thread = channel, workgroup = (channel tile, blocks y, y + gridDim.y, ...).
__global__ __launch_bounds__(kRfiThreads) void k_rfi_means(const uint8_t *__restrict__ x, int64_t nsamp,
                                                          int32_t nchan, int64_t block, int64_t n_blocks,
                                                          const uint8_t *__restrict__ flag,
                                                          const int32_t *__restrict__ n_u,
                                                          uint8_t *__restrict__ mean,
                                                          unsigned long long *__restrict__ msum) {
  const int c = blockIdx.x * kRfiThreads + threadIdx.x;
  for (int64_t b = blockIdx.y; b < n_blocks; b += gridDim.y) {
    const int64_t j0 = b * block;
    const int64_t n = min(block, nsamp - j0);
    const int32_t nu = n_u[b];
    if (nu == n) continue;  // nothing replaced in this block
    uint32_t acc = 0;
    if (c < nchan)
      for (int64_t k = 0; k < n; ++k)
        if (!flag[j0 + k]) acc += x[(j0 + k) * (int64_t)nchan + c];
    const uint32_t m = c < nchan ? (uint32_t)((2 * (uint64_t)acc + (uint64_t)nu) / (2 * (uint64_t)nu)) : 0u;
    if (c < nchan) mean[b * (int64_t)nchan + c] = (uint8_t)m;
    const int32_t t = wave_sum_i32((int32_t)m);
    if ((threadIdx.x & 63) == 0) atomicAdd(&msum[b], (unsigned long long)t);
  }
}

__device__ __forceinline__ uint32_t filter_word(uint32_t w, int32_t z) {
  uint32_t o = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int32_t v = (int32_t)((w >> (8 * k)) & 0xFFu) - z + 128;
    v = v < 0 ? 0 : (v > 255 ? 255 : v);
    o |= (uint32_t)v << (8 * k);
  }
  return o;
}

// Replacement of flagged spectra and the zero-DM filter: one wave per spectrum.
__global__ __launch_bounds__(kRfiThreads) void k_rfi_apply(const uint8_t *__restrict__ x, int64_t nsamp,
                                                          int32_t nchan, int64_t block, int vec,
                                                          const int32_t *__restrict__ s,
                                                          const uint8_t *__restrict__ flag,
                                                          const uint8_t *__restrict__ mean,
                                                          const unsigned long long *__restrict__ msum, int clip,
                                                          int zero_dm, int copy, uint8_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * kRfiThreads + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kRfiThreads) >> 6;
  for (int64_t j = w0; j < nsamp; j += nw) {
    const int64_t b = block > 0 ? j / block : 0;
    const bool f = clip && flag[j];
    if (!f && !zero_dm && !copy) continue;
    const uint8_t *src = f ? mean + b * (int64_t)nchan : x + j * (int64_t)nchan;
    const int64_t sp = f ? (int64_t)msum[b] : (int64_t)s[j];
    const int32_t z = zero_dm ? (int32_t)((2 * sp + nchan) / (2 * (int64_t)nchan)) : 128;
    uint8_t *dst = out + j * (int64_t)nchan;
    if (vec) {
      const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
      uint4 *d4 = reinterpret_cast<uint4 *>(dst);
      for (int k = lane; k < nchan / 16; k += 64) {
        uint4 q = s4[k];
        if (zero_dm) q = make_uint4(filter_word(q.x, z), filter_word(q.y, z), filter_word(q.z, z), filter_word(q.w, z));
        d4[k] = q;
      }
    } else {
      for (int c = lane; c < nchan; c += 64) {
        int32_t v = (int32_t)src[c] - z + 128;
        dst[c] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
      }
    }
  }
}

__global__ void k_rfi_zero(unsigned long long *__restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0ull;
}

}  // namespace
}  // namespace gsp

using namespace gsp;

extern "C" int gsp_rfi_clean(gsp_ctx *ctx, const uint8_t *fb_dev, int64_t nsamp, int32_t nchan, double clip_sigma,
                             int64_t block, int32_t zero_dm, uint8_t *out_dev, int64_t *n_flagged, void *stream) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    if (!fb_dev || !out_dev || nsamp < 1 || nchan < 1) fail(GSP_EINVAL, "bad filterbank arguments");
    if (!std::isfinite(clip_sigma) || clip_sigma < 0) fail(GSP_EINVAL, "clip_sigma must be finite and >= 0");
    const bool clip = clip_sigma > 0;
    if (clip && (block < 1 || block > (int64_t(1) << 30))) fail(GSP_EINVAL, "block must be in [1, 2^30]");
    if (clip && (nsamp + block - 1) / block >= (int64_t(1) << 31)) fail(GSP_EINVAL, "too many blocks");
    if ((int64_t)nchan * 255 >= (int64_t(1) << 31)) fail(GSP_EOVERFLOW, "nchan too large for int32 spectrum sums");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool same = fb_dev == out_dev;
    if (!same) {
      const uint8_t *a0 = fb_dev, *a1 = fb_dev + nsamp * (int64_t)nchan;
      if (out_dev < a1 && out_dev + nsamp * (int64_t)nchan > a0) fail(GSP_EINVAL, "out overlaps the input partly");
    }
    const int vec = (nchan % 16 == 0 && reinterpret_cast<uintptr_t>(fb_dev) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(out_dev) % 16 == 0)
                        ? 1
                        : 0;
    const int64_t nb = clip ? (nsamp + block - 1) / block : 0;
    // scratch: s, flags, n_u, means, mean sums, counter
    const size_t o_s = 0;
    const size_t o_flag = (o_s + (size_t)nsamp * 4 + 255) / 256 * 256;
    const size_t o_nu = (o_flag + (size_t)nsamp + 255) / 256 * 256;
    const size_t o_mean = (o_nu + (size_t)nb * 4 + 255) / 256 * 256;
    const size_t o_msum = (o_mean + (size_t)nb * nchan + 255) / 256 * 256;
    const size_t o_cnt = (o_msum + (size_t)nb * 8 + 255) / 256 * 256;
    const size_t bytes = o_cnt + 256;
    ctx->rfi.device = ctx->device;
    ctx->rfi.reserve(bytes);
    unsigned char *base = ctx->rfi.as<unsigned char>();
    int32_t *s = reinterpret_cast<int32_t *>(base + o_s);
    uint8_t *flag = base + o_flag;
    int32_t *n_u = reinterpret_cast<int32_t *>(base + o_nu);
    uint8_t *mean = base + o_mean;
    auto *msum = reinterpret_cast<unsigned long long *>(base + o_msum);
    auto *cnt = reinterpret_cast<unsigned long long *>(base + o_cnt);
    const unsigned grid = (unsigned)std::min<int64_t>((nsamp + 3) / 4, 256 * 16);  // 4 waves per workgroup
    ProfScope prof(ctx, "rfi", st, 2.0 * (double)nsamp * nchan);
    hipLaunchKernelGGL(k_rfi_zero, dim3(1), dim3(64), 0, st, cnt, (int64_t)1);
    hipLaunchKernelGGL(k_rfi_rowsum, dim3(grid), dim3(kRfiThreads), 0, st, fb_dev, nsamp, nchan,
                       (nchan % 16 == 0 && reinterpret_cast<uintptr_t>(fb_dev) % 16 == 0) ? 1 : 0, s);
    if (clip) {
      hipLaunchKernelGGL(k_rfi_zero, dim3((unsigned)std::min<int64_t>((nb + 255) / 256, 1024)), dim3(256), 0, st,
                         msum, nb);
      hipLaunchKernelGGL(k_rfi_flags, dim3((unsigned)nb), dim3(kRfiThreads), 0, st, s, nsamp, block, clip_sigma,
                         flag, n_u, cnt);
      hipLaunchKernelGGL(k_rfi_means,
                         dim3((unsigned)((nchan + kRfiThreads - 1) / kRfiThreads), (unsigned)std::min<int64_t>(nb, 65535)),
                         dim3(kRfiThreads), 0, st, fb_dev, nsamp, nchan, block, nb, flag, n_u, mean, msum);
    }
    hipLaunchKernelGGL(k_rfi_apply, dim3(grid), dim3(kRfiThreads), 0, st, fb_dev, nsamp, nchan, clip ? block : 0,
                       vec, s, flag, mean, msum, clip ? 1 : 0, zero_dm ? 1 : 0, same ? 0 : 1, out_dev);
    check_hip(hipGetLastError(), "launch RFI kernels");
    if (n_flagged) {
      unsigned long long h = 0;
      check_hip(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, st), "copy flag count");
      check_hip(hipStreamSynchronize(st), "synchronise stream");
      *n_flagged = (int64_t)h;
    }
  });
}
