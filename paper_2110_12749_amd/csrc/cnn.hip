// Learned triage: candidate cutouts and a small CNN trained on the GPU.
//
// Network (channels-last activations, BF16 storage, FP32 accumulation):
//   input 2 x 64 x 64 (DM-time and frequency-time cutouts)
//   conv3x3(2->16)+ReLU+maxpool2 -> conv3x3(16->32)+ReLU+maxpool2
//   -> conv3x3(32->64)+ReLU+maxpool2 -> conv3x3(64->128)+ReLU+maxpool2
//   -> flatten (h, w, c) 2048 -> FC 192 + ReLU -> FC 1 -> logit
//   loss: binary cross-entropy with logits (mean over the batch); Adam.
// Every convolution and fully connected product, forward and backward
// (activation and weight gradients), runs on one hand-written GEMM kernel
// built on the gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16), fed by
// im2col / col2im gathers; the epilogue fuses bias, ReLU and gradient masks.
#include <cmath>
#include <cstring>
#include <fstream>

#include "gsp_internal.h"

namespace gsp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// --- bf16 helpers (round to nearest even) ---
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));  // inf/nan
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
// double -> bf16 rounded once, to nearest even at 8 significant bits
// (bf16 subnormals: multiples of 2^-133); finite inputs below bf16's range
__device__ inline uint16_t d2bf(double x) {
  int e;
  const double m = frexp(x, &e);  // x = m 2^e, 0.5 <= |m| < 1
  const double q = e >= -125 ? ldexp(rint(ldexp(m, 8)), e - 8) : ldexp(rint(ldexp(x, 133)), -133);
  return f2bf((float)q);  // exact: q has at most 8 significant bits
}
__host__ __device__ inline float bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  return __builtin_bit_cast(float, u);
}

// ---------------------------------------------------------------------------
// GEMM: C[m][n] = sum_k A[m][k] B[k][n] (+ bias[n]) (ReLU) (mask) with
// arbitrary element strides, BF16 inputs, FP32 accumulation.
// Workgroup tile 64 x 64, k step 32 (two 32 x 32 x 16 MFMAs per wave); 4 waves, each a 32 x 32 tile.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const uint16_t *A;
  int64_t a_m, a_k;  // strides (elements)
  const uint16_t *B;
  int64_t b_k, b_n;
  void *C;
  int64_t c_m, c_n;
  int32_t M, N, K;
  const float *bias;       // [N] or null
  const uint16_t *mask;    // optional: zero the result where mask[m*c_m + n*c_n] <= 0 (bf16)
  int32_t relu;
  int32_t out_bf16;        // 1: store bf16, 0: store fp32
  int32_t accumulate;      // fp32 output only: C += result
  int32_t k_chunk;         // split-K: workgroup z covers k in [z*k_chunk, (z+1)*k_chunk); atomic fp32 adds
  // implicit im2col (3x3, padding 1) for A when im_x is set: A[m][k] =
  // x(n, c, h + dh, w + dw) with m = (n*H + h)*H + w, k = tap*C + c,
  // tap = (dh+1)*3 + (dw+1); x addressed with strides (n, c, h, w)
  const uint16_t *im_x;
  int64_t im_sn, im_sc, im_sh, im_sw;
  int32_t im_C, im_H;
};

static constexpr int kTM = 64, kTN = 64, kTK = 32;
static constexpr int kTP = kTK + 8;  // padded LDS row: 80 bytes, 16-byte aligned

static unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 64); }

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Workgroup tile 64 x 64, k step 32.  Each thread stages 8 consecutive k of
// one A row and of one B column: one 16-byte load where the operand is
// contiguous and aligned along k (plain A with unit k stride, implicit
// im2col over channel-contiguous activations, B with unit k stride), 8
// element loads otherwise.  B is kept transposed in LDS ([n][k]) so that
// both MFMA operands are 8-byte LDS reads.  The next k step's operands are
// loaded into registers while the current one is multiplied.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kTM][kTP];
  __shared__ __align__(16) uint16_t Bt[kTN][kTP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kTM;
  const int64_t n0 = (int64_t)blockIdx.y * kTN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool split = gridDim.z > 1;
  const int k_begin = split ? (int)blockIdx.z * g.k_chunk : 0;
  const int k_end = split ? min(g.K, k_begin + g.k_chunk) : g.K;
  // this thread's A row / B column and k offset inside a step
  const int srow = tid >> 2, skc = (tid & 3) * 8;
  const int64_t am = m0 + srow, bcol = n0 + srow;
  const bool a_in = am < g.M, b_in = bcol < g.N;
  // implicit im2col: the pixel of this thread's A row
  const uint16_t *im_base = nullptr;
  int im_h = 0, im_w = 0;
  if (g.im_x) {
    const int64_t m = min(am, (int64_t)g.M - 1);
    const int HH = g.im_H * g.im_H;
    const int64_t n = m / HH;
    const int hw = (int)(m - n * HH);
    im_h = hw / g.im_H;
    im_w = hw - im_h * g.im_H;
    im_base = g.im_x + n * g.im_sn;
  }
  // vector forms, decided once per launch
  const bool a_vec = g.im_x ? (g.im_C % 8 == 0 && g.im_sc == 1 && g.im_sh % 8 == 0 && g.im_sw % 8 == 0 &&
                               g.im_sn % 8 == 0 && (reinterpret_cast<uintptr_t>(g.im_x) & 15) == 0)
                            : (g.a_k == 1 && g.a_m % 8 == 0 && (reinterpret_cast<uintptr_t>(g.A) & 15) == 0);
  const bool b_vec = g.b_k == 1 && g.b_n % 8 == 0 && (reinterpret_cast<uintptr_t>(g.B) & 15) == 0;

  auto load_a = [&](int k0) -> u16x8 {
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    const int k = k0 + skc;
    if (!a_in) return v;
    if (g.im_x) {
      if (a_vec && k + 8 <= k_end) {
        const int tap = k / g.im_C, ch = k - tap * g.im_C;
        const int hh = im_h + tap / 3 - 1, ww = im_w + tap % 3 - 1;
        if (hh >= 0 && hh < g.im_H && ww >= 0 && ww < g.im_H)
          v = *reinterpret_cast<const u16x8 *>(im_base + ch + hh * g.im_sh + ww * g.im_sw);
        return v;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = k + i;
        if (kk < k_end) {
          const int tap = kk / g.im_C, ch = kk - tap * g.im_C;
          const int hh = im_h + tap / 3 - 1, ww = im_w + tap % 3 - 1;
          if (hh >= 0 && hh < g.im_H && ww >= 0 && ww < g.im_H)
            v[i] = im_base[ch * g.im_sc + hh * g.im_sh + ww * g.im_sw];
        }
      }
      return v;
    }
    if (a_vec && k + 8 <= k_end) return *reinterpret_cast<const u16x8 *>(g.A + am * g.a_m + k);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (k + i < k_end) v[i] = g.A[am * g.a_m + (int64_t)(k + i) * g.a_k];
    return v;
  };
  auto load_b = [&](int k0) -> u16x8 {
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    const int k = k0 + skc;
    if (!b_in) return v;
    if (b_vec && k + 8 <= k_end) return *reinterpret_cast<const u16x8 *>(g.B + bcol * g.b_n + k);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (k + i < k_end) v[i] = g.B[(int64_t)(k + i) * g.b_k + bcol * g.b_n];
    return v;
  };

  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  u16x8 pa = load_a(k_begin), pb = load_b(k_begin);
  for (int k0 = k_begin; k0 < k_end; k0 += kTK) {
    __syncthreads();  // the previous step's operands are read
    *reinterpret_cast<u16x8 *>(&As[srow][skc]) = pa;
    *reinterpret_cast<u16x8 *>(&Bt[srow][skc]) = pb;
    __syncthreads();
    if (k0 + kTK < k_end) {
      pa = load_a(k0 + kTK);
      pb = load_b(k0 + kTK);
    }
#pragma unroll
    for (int ks = 0; ks < kTK; ks += 16) {
      // 32 x 32 x 16: lane l holds row l % 32, k = 8 * (l / 32) .. + 7 of each operand
      const int kk = ks + (lane >> 5) * 8;
      const u16x8 a = *reinterpret_cast<const u16x8 *>(&As[wm + (lane & 31)][kk]);
      const u16x8 b = *reinterpret_cast<const u16x8 *>(&Bt[wn + (lane & 31)][kk]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc,
                                                     0, 0, 0);
    }
  }
  // epilogue: lane holds column wn + lane%32, rows 8*(j/4) + 4*(lane/32) + j%4
  const int64_t n = n0 + wn + (lane & 31);
  if (n >= g.N) return;
  const float bn = g.bias ? g.bias[n] : 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t m = m0 + wm + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    if (m >= g.M) continue;
    float v = acc[j] + bn;
    if (g.relu) v = v > 0.f ? v : 0.f;
    const int64_t o = m * g.c_m + n * g.c_n;
    if (split) {  // partial sums over a slice of k (bias, ReLU and masks not allowed)
      atomicAdd(static_cast<float *>(g.C) + o, acc[j]);
      continue;
    }
    if (g.mask && !(bf2f(g.mask[o]) > 0.f)) v = 0.f;
    if (g.out_bf16)
      static_cast<uint16_t *>(g.C)[o] = f2bf(v);
    else if (g.accumulate)
      static_cast<float *>(g.C)[o] += v;
    else
      static_cast<float *>(g.C)[o] = v;
  }
}

// The first convolution (2 input channels, 16 outputs, 3x3, padding 1, on
// 64 x 64 images) directly: as a GEMM it is N = 16, K = 18, a quarter of a
// 64 x 64 tile with a gather of single elements, so one thread per output
// pixel instead: its 18 inputs (NCHW bf16) as floats, 16 dot products of
// exact bf16 x bf16 products summed in fp32 (the weights, [16][18] bf16 with
// k = tap * 2 + channel, are uniform and come as scalar operands), bias,
// ReLU, and the pixel's 16 outputs (NHWC bf16).
__global__ __launch_bounds__(256) void k_conv1(const uint16_t *__restrict__ x, int64_t n,
                                               const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                               uint16_t *__restrict__ act) {
  // read-only in this kernel: through the constant address space the
  // uniform weight loads become scalar loads (w is 4-byte aligned)
  typedef const __attribute__((address_space(4))) uint32_t cu32;
  cu32 *wc = (cu32 *)w;
  const int64_t total = n * 4096;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < total; m += (int64_t)gridDim.x * blockDim.x) {
    const int64_t img = m >> 12;
    const int h = (int)(m >> 6) & 63, c = (int)m & 63;
    const uint16_t *xi = x + img * 8192;
    float xin[18];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int hh = h + tap / 3 - 1, ww = c + tap % 3 - 1;
      const bool in = hh >= 0 && hh < 64 && ww >= 0 && ww < 64;
      const int hc = min(max(hh, 0), 63), wc = min(max(ww, 0), 63);  // every load in bounds, issued together
#pragma unroll
      for (int ch = 0; ch < 2; ++ch) {
        const float v = bf2f(xi[ch * 4096 + hc * 64 + wc]);
        xin[tap * 2 + ch] = in ? v : 0.f;
      }
    }
    // four outputs at a time (36 weight dwords in scalar registers), an
    // 8-byte store each
#pragma unroll 1
    for (int o0 = 0; o0 < 16; o0 += 4) {
      uint32_t pk[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = o0 + q;
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 18; k += 2) {
          const uint32_t pr = wc[(o * 18 + k) >> 1];  // weights k, k + 1 (bf16, low half first)
          acc = __builtin_fmaf(xin[k], __builtin_bit_cast(float, pr << 16), acc);
          acc = __builtin_fmaf(xin[k + 1], __builtin_bit_cast(float, pr & 0xFFFF0000u), acc);
        }
        float v = acc + bias[o];
        v = v > 0.f ? v : 0.f;
        const uint32_t b = f2bf(v);
        pk[q >> 1] = (q & 1) ? (pk[q >> 1] | (b << 16)) : b;
      }
      *reinterpret_cast<uint2 *>(act + m * 16 + o0) = make_uint2(pk[0], pk[1]);
    }
  }
}

__global__ void k_zero_f32(float *__restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0.f;
}

// Plain launch, or split-K (fp32 output zeroed first, partial sums added
// atomically) when the output is small and K long: weight gradients.
static void gemm(GemmArgs g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const int64_t tiles = (int64_t)((g.M + kTM - 1) / kTM) * ((g.N + kTN - 1) / kTN);
  int splits = 1;
  if (!g.out_bf16 && !g.bias && !g.relu && !g.mask && !g.accumulate && tiles < 256 && g.K >= 8192)
    splits = (int)std::min<int64_t>(std::max<int64_t>(1, 1024 / tiles), g.K / 4096);
  dim3 grid((unsigned)((g.M + kTM - 1) / kTM), (unsigned)((g.N + kTN - 1) / kTN), (unsigned)splits);
  if (splits > 1) {
    g.k_chunk = (g.K + splits - 1) / splits;
    g.k_chunk = (g.k_chunk + kTK - 1) / kTK * kTK;
    // zero the (strided) fp32 output: M x N with strides c_m, c_n (dense here)
    const int64_t span = (int64_t)(g.M - 1) * g.c_m + (int64_t)(g.N - 1) * g.c_n + 1;
    hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(span)), dim3(256), 0, st, static_cast<float *>(g.C), span);
  } else {
    g.k_chunk = g.K;
  }
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  check_hip(hipGetLastError(), "launch gemm");
}

// ---------------------------------------------------------------------------
// im2col / col2im (3x3, padding 1, stride 1)
// col[(n*H + h)*W + w][tap*C + c] = x(n, c, h+dh, w+dw), tap = (dh+1)*3 + (dw+1)
// x addressed with strides (n, c, h, w) so both NCHW inputs and NHWC
// activations are read in place.
// ---------------------------------------------------------------------------
__global__ void k_im2col(const uint16_t *__restrict__ x, int64_t sn, int64_t sc, int64_t sh, int64_t sw, int N,
                         int C, int H, int W, uint16_t *__restrict__ col) {
  const int64_t total = (int64_t)N * H * W * 9 * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int tap = (int)((i / C) % 9);
    const int64_t p = i / (9 * (int64_t)C);
    const int w = (int)(p % W), h = (int)((p / W) % H);
    const int n = (int)(p / ((int64_t)W * H));
    const int hh = h + tap / 3 - 1, ww = w + tap % 3 - 1;
    col[i] = (hh >= 0 && hh < H && ww >= 0 && ww < W) ? x[n * sn + c * sc + hh * sh + ww * sw] : (uint16_t)0;
  }
}

// dx(n, h, w, c) = sum over taps of dcol[pixel (h - dh, w - dw)][tap*C + c]:
// the taps are fp32 products (the dcol GEMM keeps fp32), summed in fp32 and
// rounded to bf16 once (NHWC output)
__global__ void k_col2im(const float *__restrict__ dcol, int N, int C, int H, int W, uint16_t *__restrict__ dx) {
  const int64_t total = (int64_t)N * H * W * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int64_t p = i / C;
    const int w = (int)(p % W), h = (int)((p / W) % H);
    const int n = (int)(p / ((int64_t)W * H));
    float s = 0.f;
    for (int tap = 0; tap < 9; ++tap) {
      const int hh = h - (tap / 3 - 1), ww = w - (tap % 3 - 1);
      if (hh < 0 || hh >= H || ww < 0 || ww >= W) continue;
      s += dcol[(((int64_t)n * H + hh) * W + ww) * 9 * C + tap * C + c];
    }
    dx[i] = f2bf(s);
  }
}

// 2x2 max-pool (NHWC); idx = position of the maximum (first on ties)
__global__ void k_pool_fwd(const uint16_t *__restrict__ x, int N, int C, int H, int W, uint16_t *__restrict__ y,
                           uint8_t *__restrict__ idx) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t total = (int64_t)N * Ho * Wo * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int64_t p = i / C;
    const int w = (int)(p % Wo), h = (int)((p / Wo) % Ho);
    const int n = (int)(p / ((int64_t)Wo * Ho));
    float best = -INFINITY;
    int bi = 0;
    for (int q = 0; q < 4; ++q) {
      const float v = bf2f(x[(((int64_t)n * H + 2 * h + q / 2) * W + 2 * w + q % 2) * C + c]);
      if (v > best) {
        best = v;
        bi = q;
      }
    }
    y[i] = f2bf(best);
    idx[i] = (uint8_t)bi;
  }
}

// The same pooling with 8 channels per thread (C a multiple of 8, 16-byte
// aligned rows): four 16-byte loads, per channel the same comparisons in the
// same order, one 16-byte and one 8-byte store.
__global__ void k_pool_fwd8(const uint16_t *__restrict__ x, int N, int C, int H, int W, uint16_t *__restrict__ y,
                            uint8_t *__restrict__ idx) {
  const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
  const int64_t total = (int64_t)N * Ho * Wo * C8;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C8) * 8;
    const int64_t p = i / C8;
    const int w = (int)(p % Wo), h = (int)((p / Wo) % Ho);
    const int n = (int)(p / ((int64_t)Wo * Ho));
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      v[q] = *reinterpret_cast<const uint4 *>(x + (((int64_t)n * H + 2 * h + q / 2) * W + 2 * w + q % 2) * C + c);
    uint32_t yo[4], io[2] = {0, 0};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float best = -INFINITY;
      int bi = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t wd = (&v[q].x)[e >> 1];
        const float f = bf2f((uint16_t)((e & 1) ? wd >> 16 : wd & 0xFFFFu));
        if (f > best) {
          best = f;
          bi = q;
        }
      }
      const uint32_t b = f2bf(best);
      yo[e >> 1] = (e & 1) ? (yo[e >> 1] | (b << 16)) : b;
      io[e >> 2] |= (uint32_t)bi << (8 * (e & 3));
    }
    *reinterpret_cast<uint4 *>(y + p * C + c) = make_uint4(yo[0], yo[1], yo[2], yo[3]);
    *reinterpret_cast<uint2 *>(idx + p * C + c) = make_uint2(io[0], io[1]);
  }
}

// d(pre-activation) of the conv output: route dy to the pooled position,
// times the ReLU derivative (activation > 0).  dy may be fp32 or bf16 (NHWC
// of the pooled shape); output bf16 NHWC of the full shape.
__global__ void k_pool_bwd(const uint16_t *__restrict__ dy, const uint8_t *__restrict__ idx,
                           const uint16_t *__restrict__ act, int N, int C, int H, int W, uint16_t *__restrict__ dpre) {
  const int64_t total = (int64_t)N * H * W * C;
  const int Ho = H / 2, Wo = W / 2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int64_t p = i / C;
    const int w = (int)(p % W), h = (int)((p / W) % H);
    const int n = (int)(p / ((int64_t)W * H));
    const int64_t o = (((int64_t)n * Ho + h / 2) * Wo + w / 2) * C + c;
    const int q = (h & 1) * 2 + (w & 1);
    float g = 0.f;
    if (idx[o] == q && bf2f(act[i]) > 0.f) g = bf2f(dy[o]);
    dpre[i] = f2bf(g);
  }
}

static constexpr int kHiddenUnits = 192;  // fc1 outputs

// Loss head, per (sample i, hidden unit j): BCE with logits, dz_i =
// (sigmoid(z_i) - y_i) / n kept in fp32, and the gradient of fc1's
// pre-activation dh[i][j] = dz_i * w2[j] * [h[i][j] > 0] rounded to bf16 once
// (w2 the bf16 weights the forward pass used).  Lane j = 0 also stores the
// sample's loss and dz.
__global__ void k_head_bwd(const float *__restrict__ z, const float *__restrict__ y, const uint16_t *__restrict__ h,
                           const uint16_t *__restrict__ w2, int n, float *__restrict__ loss,
                           float *__restrict__ dz, uint16_t *__restrict__ dh) {
  const int64_t total = (int64_t)n * kHiddenUnits;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(k / kHiddenUnits), j = (int)(k - (int64_t)i * kHiddenUnits);
    const float zi = z[i], yi = y[i];
    const float g = (1.f / (1.f + expf(-zi)) - yi) / (float)n;
    if (j == 0) {
      loss[i] = fmaxf(zi, 0.f) - zi * yi + log1pf(expf(-fabsf(zi)));
      dz[i] = g;
    }
    dh[k] = f2bf(bf2f(h[k]) > 0.f ? g * bf2f(w2[j]) : 0.f);
  }
}

// fc2's parameter gradients from the fp32 dz: dW2[j] = sum_i dz_i h[i][j]
// (threads j < 192), db2 = sum_i dz_i (thread 192); one workgroup.
__global__ __launch_bounds__(256) void k_head_wgrad(const float *__restrict__ dz, const uint16_t *__restrict__ h,
                                                    int n, float *__restrict__ dw2, float *__restrict__ db2) {
  const int j = threadIdx.x;
  if (j > kHiddenUnits) return;
  float s = 0.f;
  if (j < kHiddenUnits) {
    for (int i = 0; i < n; ++i) s += dz[i] * bf2f(h[(int64_t)i * kHiddenUnits + j]);
    dw2[j] = s;
  } else {
    for (int i = 0; i < n; ++i) s += dz[i];
    *db2 = s;
  }
}

// Adam on fp32 master parameters; refreshes the bf16 copy
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ pb, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] -= upd;
    pb[i] = f2bf(p[i]);
  }
}

__global__ void k_to_bf16(const float *__restrict__ a, uint16_t *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = f2bf(a[i]);
}

__global__ void k_fill_bf16(uint16_t *__restrict__ a, int64_t n, uint16_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// ---------------------------------------------------------------------------
// Cutouts (a candidate's DM-time and frequency-time images)
// ---------------------------------------------------------------------------
struct CutRow {
  const int32_t *dmt;     // row block of the plan output, [n_dm][n_out]
  const int32_t *delays;  // int32 [n_dm][nchan]
  int64_t n_out;
  int32_t n_dm, D, trial0;
};
struct CutoutArgs {
  const uint8_t *fb;  // uint8 [nsamp][nchan]
  const double *musig;
  const gsp_candidate *cand;
  int64_t n;
  int32_t nchan, n_seg, rmax;
  int32_t tiled;      // bands are 16-byte aligned row segments (nchan % 1024 == 0, fb 16-byte aligned)
  CutRow row[GSP_MAX_SEG];
  uint16_t *out;  // bf16 [n][2][64][64]
  uint32_t *ftsums;  // [n][64 bands][64 bins]: frequency-time band sums (k_cutout_ft writes, k_cutout reads)
  const uint8_t *ycm;  // channel-major copy of fb, rows of cm_pitch bytes (k_cutout_ft_cm)
  int64_t cm_pitch;
};

// Sum of a uint32 over the 64 lanes of a wave (DPP shifts inside rows of 16,
// then row totals broadcast down), returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t add_dpp_u32(uint32_t v) {
  return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  x = add_dpp_u32<0x111, 0xf>(x);  // row_shr:1
  x = add_dpp_u32<0x112, 0xf>(x);  // row_shr:2
  x = add_dpp_u32<0x114, 0xf>(x);  // row_shr:4
  x = add_dpp_u32<0x118, 0xf>(x);  // row_shr:8
  x = add_dpp_u32<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = add_dpp_u32<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// One workgroup per candidate.  Box end e = t_peak + width - 1 (row
// resolution), bin width r = clamp(width / 8, 1, rmax); bin b covers samples
// e - (64 - b) r + 1 .. e - (63 - b) r, so the box fills the last ~8 bins and
// nothing after e is used.
//  image 0 (DM-time): 64 trials centred on the candidate's (clamped to the
//    row), bin sums of the dedispersed series; samples before the start
//    count as the trial's mean;
//  image 1 (frequency-time): 64 sub-bands of nchan/64 channels, each channel
//    shifted by its delay at the candidate's DM, bin sums of the raw
//    samples; a bin partly before the start is scaled up to r samples, one
//    wholly before it takes its band's mean.
// Each image is then z-scored (zero mean, unit variance; constant -> 0).
// The two images of one candidate from a data source:
//   dm(tr, t)  the dedispersed sample of trial tr at time t >= 0;
//   mean(tr)   the value counted for times before the start;
//   ft(c, t)   channel c's downsampled sample t >= 0 shifted by its delay at
//              the candidate's trial (t + d_c);
// img: LDS [2][4096] doubles, red: LDS [3][256]; out: bf16 [2][4096].
// band(band, cb, ce, e, r, mine): an optional faster way to the band's bin
// sums (bin b on lane b, every lane of the wave calls it); returns false where
// it does not apply, and the loads below run instead.
template <class DM, class MEAN, class FT, class BAND>
__device__ void cutout_images(int64_t e, int width, int dm_index, int n_dm, int nchan, int rmax, DM dm, MEAN mean,
                              FT ft, BAND band_sums, double (*img)[4096], double (*red)[256], uint16_t *out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = max(1, min(rmax, width / 8));
  const int lo = max(0, min(dm_index - 32, n_dm - 64));
  // ---- DM-time: 16 pixels per thread, their loads issued together ----
  {
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = 0.0;
    for (int j = 0; j < r; ++j) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int u = tid + 256 * i;
        const int tr = lo + u / 64, b = u % 64;
        const int64_t t = e - (int64_t)(64 - b) * r + 1 + j;
        if (tr < n_dm) v[i] += t >= 0 ? (double)dm(tr, t) : mean(tr);
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) img[0][tid + 256 * i] = v[i];
  }
  // ---- frequency-time: one wave per band, lanes over the band's channels ----
  // Every lane sums its channels' samples of all 64 bins (exact integers,
  // all loads of one sample offset in flight together); the band's bin sums
  // are then reduced over the lanes and bin b lands on lane b.
  for (int band = wave; band < 64; band += 4) {
    const int cb = (int)((int64_t)band * nchan / 64), ce = (int)((int64_t)(band + 1) * nchan / 64);
    uint32_t mine = 0;
    if (!band_sums(band, cb, ce, e, r, mine)) {
      uint32_t acc[64];
#pragma unroll
      for (int b = 0; b < 64; ++b) acc[b] = 0;
      for (int ch = cb + lane; ch < ce; ch += 64)
        for (int j = 0; j < r; ++j) {
#pragma unroll
          for (int b = 0; b < 64; ++b) {
            const int64_t t = e - (int64_t)(64 - b) * r + 1 + j;
            if (t >= 0) acc[b] += ft(ch, t);
          }
        }
#pragma unroll
      for (int b = 0; b < 64; ++b) {
        const uint32_t tot = wave_sum_u32(acc[b]);
        if (lane == b) mine = tot;
      }
    }
    const int64_t t0 = e - (int64_t)(64 - lane) * r + 1;
    const int64_t first = max((int64_t)0, t0);
    const int cnt = (int)max((int64_t)0, t0 + r - first);
    // a bin partly before the start is scaled up to r samples; one wholly
    // before it is filled below with the mean of the band's valid bins
    img[1][band * 64 + lane] = cnt > 0 ? (double)mine * (double)r / (double)cnt : NAN;
    if (__ballot(cnt == 0) != 0ull) {
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) {
        double valid_sum = 0.0;
        int n_valid = 0;
        for (int b = 0; b < 64; ++b)
          if (!isnan(img[1][band * 64 + b])) {
            valid_sum += img[1][band * 64 + b];
            ++n_valid;
          }
        const double fill = n_valid ? valid_sum / n_valid : 0.0;
        for (int b = 0; b < 64; ++b)
          if (isnan(img[1][band * 64 + b])) img[1][band * 64 + b] = fill;
      }
    }
  }
  __syncthreads();
  // ---- z-score each image (two passes; an image of equal pixels becomes 0) ----
  for (int im = 0; im < 2; ++im) {
    double s1 = 0.0, vmin = INFINITY, vmax = -INFINITY;
    for (int u = tid; u < 4096; u += 256) {
      const double v = img[im][u];
      s1 += v;
      vmin = fmin(vmin, v);
      vmax = fmax(vmax, v);
    }
    red[0][tid] = s1;
    red[1][tid] = vmin;
    red[2][tid] = vmax;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        red[0][tid] += red[0][tid + h];
        red[1][tid] = fmin(red[1][tid], red[1][tid + h]);
        red[2][tid] = fmax(red[2][tid], red[2][tid + h]);
      }
      __syncthreads();
    }
    const double mean_px = red[0][0] / 4096.0;
    const bool flat = red[1][0] == red[2][0];
    __syncthreads();
    double s2 = 0.0;
    for (int u = tid; u < 4096; u += 256) {
      const double d = img[im][u] - mean_px;
      s2 += d * d;
    }
    red[0][tid] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[0][tid] += red[0][tid + h];
      __syncthreads();
    }
    const double inv = flat ? 0.0 : 1.0 / sqrt(red[0][0] / 4096.0);
    uint16_t *o = out + im * 4096;
    for (int u = tid; u < 4096; u += 256) o[u] = d2bf((img[im][u] - mean_px) * inv);
    __syncthreads();
  }
}

// Raw rows of one band staged per wave for the tiled band sums.
static constexpr int kTileRows = 320;
// batches of at least this many candidates read a channel-major copy of the
// input (k_cutout_ft_cm); smaller ones read the recorded rows (k_cutout_ft)
static constexpr int64_t kCutStageMin = 256;

__device__ __forceinline__ int wave_min_i32(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i32(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// Tiled band sums of one frequency-time band: the band's raw rows for a run
// of bins are read as 16-byte row segments (a few cache lines per load
// instead of one per channel) into the wave's LDS tile, then each lane sums
// its channel's shifted rows from there and bin b's total over the lanes is
// added to `mine` on lane b.  The band's channels go through in groups of
// G = 64, 32 or 16, the widest for which every group's delay spread plus one
// bin fits the tile (a narrower group has a smaller spread and its G-byte
// rows leave room for more of them; lanes G..63 add nothing).  Needs bands
// of whole 16-byte segments; false where no group width fits.
__device__ bool tiled_band_sums(const uint8_t *__restrict__ fb, int nchan, int D, const int32_t *__restrict__ dly,
                                int cb, int ce, int64_t e, int r, uint4 *tile4, uint32_t &mine) {
  const int lane = threadIdx.x & 63;
  const uint8_t *tileb = reinterpret_cast<const uint8_t *>(tile4);
  auto spread_of = [&](int g0, int G) {
    const int ch = g0 + lane;
    const bool in = lane < G && ch < ce;
    const int lo = wave_min_i32(in ? dly[ch] : INT_MAX);
    const int hi = wave_max_i32(in ? dly[ch] : INT_MIN);
    return make_int2(lo, hi);
  };
  int gmax = 64;  // no wider than the band (bands are multiples of 16 channels)
  while (gmax > 16 && gmax / 2 >= ce - cb) gmax >>= 1;
  int G = 0;
  for (int g = gmax; g >= 16 && G == 0; g >>= 1) {
    const int64_t cap = (int64_t)kTileRows * 64 / g / D;  // downsampled rows the tile holds
    bool fits = true;
    for (int g0 = cb; g0 < ce && fits; g0 += g) {
      const auto lh = spread_of(g0, g);
      fits = (cap - ((int64_t)lh.y - lh.x)) / r >= 1;
    }
    if (fits) G = g;
  }
  if (G == 0) return false;
  const int lq = G == 64 ? 2 : G == 32 ? 1 : 0;  // log2 of the 16-byte segments per row
  const int64_t cap = (int64_t)kTileRows * 64 / G / D;
  const int64_t t0 = e - 64 * (int64_t)r + 1;
  for (int g0 = cb; g0 < ce; g0 += G) {
    const int ch = g0 + lane;
    const bool valid = lane < G && ch < ce;
    const auto lh = spread_of(g0, G);
    const int dmin = lh.x, dmax = lh.y;
    const int64_t nb = (cap - ((int64_t)dmax - dmin)) / r;  // >= 1 (G was chosen so)
    const int64_t dc = valid ? dly[ch] : dmin;
    for (int b0 = 0; b0 < 64; b0 += (int)nb) {
      const int b1 = (int)min((int64_t)64, b0 + nb);
      if (t0 + (int64_t)b1 * r - 1 < 0) continue;  // these bins lie before the first sample
      const int64_t s_lo = max(t0 + (int64_t)b0 * r, (int64_t)0) + dmin;
      const int64_t s_hi = t0 + (int64_t)b1 * r - 1 + dmax;
      const int64_t R0 = s_lo * D;
      const int nrows = (int)((s_hi - s_lo + 1) * D);  // <= cap * D: nrows * G bytes fit the tile
      const int nseg = nrows << lq;
      __builtin_amdgcn_wave_barrier();  // the previous pass's reads are done
      // 8 loads in flight per lane before their LDS stores
      for (int i0 = lane; i0 < nseg; i0 += 64 * 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = min(i0 + 64 * u, nseg - 1);
          const int q = i & ((1 << lq) - 1);
          v[u] = g0 + 16 * q < ce ? *reinterpret_cast<const uint4 *>(fb + (R0 + (i >> lq)) * (int64_t)nchan + g0 + 16 * q)
                                  : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + 64 * u;
          if (i < nseg) tile4[i] = v[u];
        }
      }
      __builtin_amdgcn_wave_barrier();
      for (int b = b0; b < b1; ++b) {
        const int64_t tb = t0 + (int64_t)b * r;
        const int jlo = (int)max((int64_t)0, -tb);
        uint32_t s = 0;
        if (jlo < r && valid) {
          const uint8_t *p = tileb + ((tb + jlo + dc) * D - R0) * G + (ch - g0);
          const int nu = (r - jlo) * D;
          for (int u = 0; u < nu; ++u) s += p[u * G];
        }
        const uint32_t tot = wave_sum_u32(s);
        if (lane == b) mine += tot;
      }
    }
  }
  return true;
}

// Frequency-time band sums of batch cutouts, one wave per (event, band): the
// band's bins summed over its channels as exact integers (lane b: bin b),
// written for k_cutout, which scales partial bins and z-scores.  Apart from
// the images this kernel holds only the row tiles in LDS, so several
// workgroups share a CU.  Workgroup x runs on XCD x % 8 (the grid is a
// multiple of 8); event k's 16 workgroups (4 bands each) all run on XCD
// k % 8, whose workgroups take that XCD's events in order, so neighbouring
// bands, which share cache lines of the filterbank rows, share an L2.
__global__ __launch_bounds__(256) void k_cutout_ft(CutoutArgs a) {
  __shared__ uint4 tiles[4][kTileRows * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = blockIdx.x & 7;
  const int64_t per_xcd = gridDim.x >> 3;
  for (int64_t j = blockIdx.x >> 3;; j += per_xcd) {
    const int64_t k = (j >> 4) * 8 + x;
    if (k >= a.n) break;
    const int band = (int)(j & 15) * 4 + wave;
    const gsp_candidate c = a.cand[k];
    const bool ok = c.seg >= 0 && c.seg < a.n_seg && c.width >= 1 && c.dm_index >= 0 &&
                    c.dm_index < a.row[c.seg].n_dm && c.t_peak + c.width - 1 >= 0 &&
                    c.t_peak + c.width - 1 < a.row[c.seg].n_out;
    if (!ok) continue;  // k_cutout writes zero images and reads nothing here
    const CutRow R = a.row[c.seg];
    const int nchan = a.nchan, D = R.D;
    const int32_t *dly = R.delays + (int64_t)c.dm_index * nchan;
    const int64_t e = c.t_peak + c.width - 1;
    const int r = max(1, min(a.rmax, c.width / 8));
    const int cb = (int)((int64_t)band * nchan / 64), ce = (int)((int64_t)(band + 1) * nchan / 64);
    uint32_t mine = 0;
    if (!(a.tiled && tiled_band_sums(a.fb, nchan, D, dly, cb, ce, e, r, tiles[wave], mine))) {
      // every lane reads its channels' bytes directly
      uint32_t acc[64];
#pragma unroll
      for (int b = 0; b < 64; ++b) acc[b] = 0;
      for (int ch = cb + lane; ch < ce; ch += 64)
        for (int j = 0; j < r; ++j) {
#pragma unroll
          for (int b = 0; b < 64; ++b) {
            const int64_t t = e - (int64_t)(64 - b) * r + 1 + j;
            if (t >= 0) {
              const uint8_t *p = a.fb + ((t + dly[ch]) * D) * (int64_t)nchan + ch;
              uint32_t v = 0;
              for (int m = 0; m < D; ++m) v += p[(int64_t)m * nchan];
              acc[b] += v;
            }
          }
        }
#pragma unroll
      for (int b = 0; b < 64; ++b) {
        const uint32_t tot = wave_sum_u32(acc[b]);
        if (lane == b) mine = tot;
      }
    }
    a.ftsums[(k * 64 + band) * 64 + lane] = mine;
  }
}

// The same band sums from a channel-major copy of the filterbank, for large
// batches (the copy is one transpose of the whole input): one wave per
// (event, band), lane b sums bin b over the band's channels.  For a channel
// the bins of the lanes are consecutive byte runs of its row (r D bytes
// each), read as unaligned dwords and summed by v_sad_u8, so a wave's loads
// are contiguous whatever the delays; no cross-lane reduction.  The work is
// taken band-major (band 0 of every event, then band 1, ...; a workgroup's
// four waves take one band of four events): the copy's rows are a page or
// so each, and the waves in flight then read the pages of about a hundred
// channels rather than of the whole copy, whose address translations would
// not stay cached.
__device__ __forceinline__ uint32_t load_u32_any(const uint8_t *p) {
  typedef uint32_t u32_unaligned __attribute__((aligned(1)));
  return *reinterpret_cast<const u32_unaligned *>(p);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 load_u128_any(const uint8_t *p) {
  typedef u32x4 u32x4_unaligned __attribute__((aligned(1)));
  return *reinterpret_cast<const u32x4_unaligned *>(p);
}
__global__ __launch_bounds__(256) void k_cutout_ft_cm(CutoutArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nq = (a.n + 3) / 4;  // groups of four events
  for (int64_t j = blockIdx.x; j < nq * 64; j += gridDim.x) {
    const int band = (int)(j / nq);
    const int64_t k = (j % nq) * 4 + wave;
    if (k >= a.n) continue;  // uniform over the wave; the kernel has no barrier
    const gsp_candidate c = a.cand[k];
    const bool ok = c.seg >= 0 && c.seg < a.n_seg && c.width >= 1 && c.dm_index >= 0 &&
                    c.dm_index < a.row[c.seg].n_dm && c.t_peak + c.width - 1 >= 0 &&
                    c.t_peak + c.width - 1 < a.row[c.seg].n_out;
    if (!ok) continue;  // k_cutout writes zero images and reads nothing here
    const CutRow R = a.row[c.seg];
    const int nchan = a.nchan, D = R.D;
    const int32_t *dly = R.delays + (int64_t)c.dm_index * nchan;
    const int64_t e = c.t_peak + c.width - 1;
    const int r = max(1, min(a.rmax, c.width / 8));
    const int cb = (int)((int64_t)band * nchan / 64), ce = (int)((int64_t)(band + 1) * nchan / 64);
    const int64_t t0 = e - 64 * (int64_t)r + 1;  // first sample of bin 0
    const int m = (r * D) >> 4;                    // 16-byte chunks per bin
    if (t0 >= 0 && ((r * D) & 15) == 0 && (m == 1 || m == 2 || m == 4)) {
      // Every bin after the start and a whole number of 16-byte chunks long:
      // a channel's window (64 r D bytes from (t0 + d) D) is read as chunks,
      // lane L taking chunks L + 64 q, so each load instruction covers 1 KiB
      // of the row; the lane's chunk sums add up over the band's channels
      // (the window layout is the same for every channel), and the m lanes
      // of a bin fold theirs together once at the end.
      uint32_t acc[4] = {0, 0, 0, 0};
      auto add_chunks = [&](const uint8_t *p) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < m) {
            const u32x4 v = load_u128_any(p + 16 * (lane + 64 * q));
            acc[q] = __builtin_amdgcn_sad_u8(v.x, 0u, acc[q]);
            acc[q] = __builtin_amdgcn_sad_u8(v.y, 0u, acc[q]);
            acc[q] = __builtin_amdgcn_sad_u8(v.z, 0u, acc[q]);
            acc[q] = __builtin_amdgcn_sad_u8(v.w, 0u, acc[q]);
          }
      };
      for (int c0 = cb; c0 < ce; c0 += 64) {
        const int nc = min(64, ce - c0);
        const int dl = lane < nc ? dly[c0 + lane] : 0;
        for (int i = 0; i < nc; ++i)
          add_chunks(a.ycm + (int64_t)(c0 + i) * a.cm_pitch + (t0 + __builtin_amdgcn_readlane(dl, i)) * D);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < m) {
          uint32_t v = acc[q];
          for (int sh = 1; sh < m; sh <<= 1) v += (uint32_t)__shfl_xor((int)v, sh, 64);
          if ((lane & (m - 1)) == 0) a.ftsums[(k * 64 + band) * 64 + (lane + 64 * q) / m] = v;
        }
      continue;
    }
    // bin `lane`: downsampled samples [tb, tb + r) of each channel after its
    // delay, those before the start left out (k_cutout scales the bin)
    const int64_t tb = e - (int64_t)(64 - lane) * r + 1;
    const int64_t tlo = max(tb, (int64_t)0);
    const int nb = (int)max((int64_t)0, tb + r - tlo) * D;  // raw bytes of the bin
    // The delays of up to 64 channels are read at once (one per lane) and
    // handed round by readlane; the loads of 16 channels go out together.
    uint32_t s = 0;
    for (int c0 = cb; c0 < ce; c0 += 64) {
      const int nc = min(64, ce - c0);
      const int dl = lane < nc ? dly[c0 + lane] : 0;
      int i = 0;
      for (; i + 16 <= nc; i += 16) {
        const uint8_t *p[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          p[q] = a.ycm + (int64_t)(c0 + i + q) * a.cm_pitch + (tlo + __builtin_amdgcn_readlane(dl, i + q)) * D;
        for (int u = 0; u < nb; u += 4) {
          uint32_t w[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) w[q] = load_u32_any(p[q] + u);
          const uint32_t m = u + 4 > nb ? 0xFFFFFFFFu >> (8 * (u + 4 - nb)) : 0xFFFFFFFFu;
#pragma unroll
          for (int q = 0; q < 16; ++q) s = __builtin_amdgcn_sad_u8(w[q] & m, 0u, s);
        }
      }
      for (; i < nc; ++i) {
        const uint8_t *p = a.ycm + (int64_t)(c0 + i) * a.cm_pitch + (tlo + __builtin_amdgcn_readlane(dl, i)) * D;
        for (int u = 0; u < nb; u += 4) {
          uint32_t w = load_u32_any(p + u);
          if (u + 4 > nb) w &= 0xFFFFFFFFu >> (8 * (u + 4 - nb));
          s = __builtin_amdgcn_sad_u8(w, 0u, s);
        }
      }
    }
    a.ftsums[(k * 64 + band) * 64 + lane] = s;
  }
}

// The trials whose means a batch of cutouts reads: the 64 trials of an
// event's DM-time image when its first bin starts before the series does
// (those bins count as the trial's mean).  One thread per (event, image row).
__global__ void k_cutout_need(CutoutArgs a, uint32_t *__restrict__ need, int32_t n_trials) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n_trials) need[u] = 0;
}
__global__ void k_cutout_mark(CutoutArgs a, uint32_t *__restrict__ need) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= a.n * 64) return;
  const gsp_candidate c = a.cand[u / 64];
  const bool ok = c.seg >= 0 && c.seg < a.n_seg && c.width >= 1 && c.dm_index >= 0 &&
                  c.dm_index < a.row[c.seg].n_dm && c.t_peak + c.width - 1 >= 0 &&
                  c.t_peak + c.width - 1 < a.row[c.seg].n_out;
  if (!ok) return;
  const CutRow R = a.row[c.seg];
  const int64_t e = c.t_peak + c.width - 1;
  const int r = max(1, min(a.rmax, c.width / 8));
  if (e - 64 * (int64_t)r + 1 >= 0) return;  // every bin starts inside the series
  const int lo = max(0, min(c.dm_index - 32, R.n_dm - 64));
  const int tr = lo + (int)(u % 64);
  if (tr < R.n_dm) need[R.trial0 + tr] = 1;
}

__global__ __launch_bounds__(256) void k_cutout(CutoutArgs a) {
  __shared__ double img[2][64 * 64];
  __shared__ double red[3][256];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int64_t k = blockIdx.x; k < a.n; k += gridDim.x) {
    const gsp_candidate c = a.cand[k];
    const bool ok = c.seg >= 0 && c.seg < a.n_seg && c.width >= 1 && c.dm_index >= 0 &&
                    c.dm_index < a.row[c.seg].n_dm && c.t_peak + c.width - 1 >= 0 &&
                    c.t_peak + c.width - 1 < a.row[c.seg].n_out;
    if (!ok) {  // out of range for this plan: two zero images, nothing read
      for (int u = tid; u < 2 * 4096; u += 256) a.out[(int64_t)k * 2 * 4096 + u] = 0;
      continue;
    }
    const CutRow R = a.row[c.seg];
    const uint8_t *fb = a.fb;
    const int nchan = a.nchan;
    const int D = R.D;
    const double *musig = a.musig;
    const int32_t *dly = R.delays + (int64_t)c.dm_index * nchan;
    auto dm = [&](int tr, int64_t t) { return R.dmt[(int64_t)tr * R.n_out + t]; };
    auto mean = [&](int tr) { return musig[2 * (R.trial0 + tr)]; };
    auto ft = [&](int ch, int64_t t) {
      const uint8_t *p = fb + ((t + dly[ch]) * D) * (int64_t)nchan + ch;
      uint32_t v = 0;
      for (int m = 0; m < D; ++m) v += p[(int64_t)m * nchan];
      return v;
    };
    // the band sums come from k_cutout_ft
    auto band_sums = [&](int band, int cb, int ce, int64_t e, int r, uint32_t &mine) -> bool {
      mine = a.ftsums[((int64_t)k * 64 + band) * 64 + lane];
      return true;
    };
    cutout_images(c.t_peak + c.width - 1, c.width, c.dm_index, R.n_dm, nchan, a.rmax, dm, mean, ft, band_sums, img,
                  red, a.out + (int64_t)k * 2 * 4096);
  }
}

// Cutouts of streamed candidates from the stream's device state: the
// dedispersed series of the current window (and the look-back kept before
// it) and the ring of downsampled samples.  Times before the beam's start
// count as the window's mean (DM-time) or are left out (frequency-time), as
// for batch cutouts.
// Samples per channel row of a wave's tile in the streaming cutouts (pitch
// padded by 2 so that lanes reading different channels hit different banks).
static constexpr int kRowS = 128, kRowPitch = kRowS + 2;

__global__ __launch_bounds__(256) void k_cutout_stream(const StreamCut *__restrict__ cuts, int64_t n, int rmax,
                                                       uint16_t *__restrict__ out) {
  __shared__ double img[2][64 * 64];
  __shared__ double red[3][256];
  __shared__ uint16_t rows[4][64 * kRowPitch];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint16_t *tile = rows[wave];
  for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const StreamCut C = cuts[k];
    const int32_t *dly = C.delays + (int64_t)C.dm_index * C.nchan;
    auto dm = [&](int tr, int64_t t) { return C.win[(int64_t)tr * C.win_pitch + C.look + (t - C.a)]; };
    auto mean = [&](int tr) { return C.mu[2 * tr]; };
    auto ft = [&](int ch, int64_t t) {
      return (uint32_t)C.ring[(int64_t)ch * C.ring_pitch + (t + dly[ch]) % C.R];
    };
    // Tiled band sums: for a run of bins, each channel's stretch of its ring
    // row is copied into the wave's tile by all 64 lanes (contiguous 2-byte
    // loads, one or two cache lines per load instead of one per channel),
    // then every lane sums its own channel's bins from LDS.  Bands of at
    // most 64 channels (one per lane).
    auto band_sums = [&](int band, int cb, int ce, int64_t e, int r, uint32_t &mine) -> bool {
      const int nch = ce - cb;
      if (nch > 64) return false;
      const int64_t t0 = e - 64 * (int64_t)r + 1;
      // ring column of time t0 + q for channel cb + lane: (t0 + q + d) mod R;
      // for a window that starts before the beam (t0 + d < 0) the column is
      // t0 + q + d itself wherever the time is valid (t0 + q >= 0)
      const int64_t base_l = t0 + (lane < nch ? dly[cb + lane] : 0);
      const int64_t p_band = base_l >= 0 ? base_l % C.R : base_l;
      const int nbp = kRowS / r;  // bins per pass
      for (int b0 = 0; b0 < 64; b0 += nbp) {
        const int b1 = min(64, b0 + nbp);
        const int L = (b1 - b0) * r;  // <= kRowS < R
        const int64_t ts = t0 + (int64_t)b0 * r;
        __builtin_amdgcn_wave_barrier();  // the previous pass's reads are done
        for (int cc0 = 0; cc0 < nch; cc0 += 8) {
          uint16_t v[8][2];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int cc = min(cc0 + u, nch - 1);
            const uint16_t *rrow = C.ring + (int64_t)(cb + cc) * C.ring_pitch;
            int64_t p0 = readlane_i64(p_band, cc) + (int64_t)b0 * r;
            if (p0 >= C.R) p0 -= C.R;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int q = lane + 64 * h;
              int64_t pos = p0 + q;
              if (pos >= C.R) pos -= C.R;
              v[u][h] = (q < L && ts + q >= 0) ? rrow[pos] : (uint16_t)0;
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h)
              if (cc0 + u < nch && lane + 64 * h < L) tile[(cc0 + u) * kRowPitch + lane + 64 * h] = v[u][h];
        }
        __builtin_amdgcn_wave_barrier();
        const bool has = lane < nch;
        for (int b = b0; b < b1; ++b) {
          uint32_t s = 0;
          if (has) {
            const uint16_t *p = tile + lane * kRowPitch + (b - b0) * r;
            for (int j = 0; j < r; ++j) s += p[j];
          }
          const uint32_t tot = wave_sum_u32(s);
          if (lane == b) mine = tot;
        }
      }
      return true;
    };
    cutout_images(C.t_peak + C.width - 1, C.width, C.dm_index, C.n_dm, C.nchan, rmax, dm, mean, ft, band_sums, img,
                  red, out + k * 2 * 4096);
  }
}

void launch_cutouts_stream(const StreamCut *cuts_dev, int64_t n, uint16_t *out_dev, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cutout_stream, dim3((unsigned)std::min<int64_t>(n, 256 * 8)), dim3(256), 0, st, cuts_dev, n,
                     8, out_dev);
  check_hip(hipGetLastError(), "launch stream cutouts");
}

// ---------------------------------------------------------------------------
// the network
// ---------------------------------------------------------------------------
struct ConvSpec {
  int cin, cout, h;  // input channels, output channels, input height = width
};
static const ConvSpec kConv[4] = {{2, 16, 64}, {16, 32, 32}, {32, 64, 16}, {64, 128, 8}};
static constexpr int kFlat = 128 * 4 * 4, kHidden = kHiddenUnits;

struct ParamLayout {
  int64_t w[6], b[6];  // offsets (conv1..4, fc1, fc2)
  int64_t wn[6], bn[6];
  int64_t total;
};

static ParamLayout layout() {
  ParamLayout L;
  int64_t o = 0;
  for (int l = 0; l < 6; ++l) {
    int64_t wn, bn;
    if (l < 4) {
      wn = (int64_t)kConv[l].cout * 9 * kConv[l].cin;
      bn = kConv[l].cout;
    } else if (l == 4) {
      wn = (int64_t)kHidden * kFlat;
      bn = kHidden;
    } else {
      wn = kHidden;
      bn = 1;
    }
    L.w[l] = o;
    L.wn[l] = wn;
    o += wn;
    L.b[l] = o;
    L.bn[l] = bn;
    o += bn;
  }
  L.total = o;
  return L;
}

}  // namespace gsp

using namespace gsp;

struct gsp_cnn {
  gsp_ctx *ctx = nullptr;
  ParamLayout L;
  DevBuf p32, pbf, g32, m, v, ones;
  int64_t t = 0;  // Adam steps
  // activations and scratch for batches up to `cap`
  int64_t cap = 0;
  int64_t last_n = 0;  // batch of the last forward pass
  DevBuf col[4], act[4], pool[4], idx[4], h1, z, dz, loss, dh1, dcol, dpre;
  DevBuf dpool[4];        // gradient of each block's pooled output (bf16, NHWC)
  int64_t last_bwd_n = 0;  // batch of the last backward pass
};

namespace {

void reserve_batch(gsp_cnn *c, int64_t n) {
  if (n <= c->cap) return;
  const int dev = c->ctx->device;
  for (int l = 0; l < 4; ++l) {
    const int64_t px = n * kConv[l].h * kConv[l].h;
    c->col[l].device = dev;
    c->col[l].reserve((size_t)px * 9 * kConv[l].cin * 2);
    c->act[l].device = dev;
    c->act[l].reserve((size_t)px * kConv[l].cout * 2);
    c->pool[l].device = dev;
    c->pool[l].reserve((size_t)px / 4 * kConv[l].cout * 2);
    c->idx[l].device = dev;
    c->idx[l].reserve((size_t)px / 4 * kConv[l].cout);
  }
  int64_t big = 0;
  for (int l = 0; l < 4; ++l) big = std::max<int64_t>(big, n * kConv[l].h * kConv[l].h * 9 * kConv[l].cin);
  for (DevBuf *d : {&c->h1, &c->z, &c->dz, &c->loss, &c->dh1, &c->dcol, &c->dpre, &c->ones}) d->device = dev;
  c->h1.reserve((size_t)n * kHidden * 2);
  c->z.reserve((size_t)n * 4);
  c->dz.reserve((size_t)n * 4);
  c->loss.reserve((size_t)n * 4);
  c->dh1.reserve((size_t)n * kHidden * 2);
  c->dcol.reserve((size_t)big * 4);  // fp32 taps
  c->dpre.reserve((size_t)n * 64 * 64 * 16 * 2);
  for (int l = 0; l < 4; ++l) {
    const int h = kConv[l].h / 2;
    c->dpool[l].device = dev;
    c->dpool[l].reserve((size_t)n * h * h * kConv[l].cout * 2);
  }
  c->ones.reserve((size_t)n * 64 * 64 * 2);
  hipLaunchKernelGGL(k_fill_bf16, dim3(grid_for(n * 4096)), dim3(256), 0, 0, c->ones.as<uint16_t>(), n * 4096,
                     (uint16_t)0x3F80);
  check_hip(hipDeviceSynchronize(), "fill ones");
  c->cap = n;
}

GemmArgs ga(const uint16_t *A, int64_t am, int64_t ak, const uint16_t *B, int64_t bk, int64_t bn, void *C, int64_t cm,
            int64_t cn, int64_t M, int64_t N, int64_t K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A;
  g.a_m = am;
  g.a_k = ak;
  g.B = B;
  g.b_k = bk;
  g.b_n = bn;
  g.C = C;
  g.c_m = cm;
  g.c_n = cn;
  g.M = (int32_t)M;
  g.N = (int32_t)N;
  g.K = (int32_t)K;
  return g;
}

// Forward pass of a batch; logits (fp32) left in c->z.  With keep_col the
// im2col matrices are written out for the backward pass; without, the
// convolutions gather their inputs inside the GEMM (same values, same sums).
void forward(gsp_cnn *c, const uint16_t *x, int64_t n, hipStream_t st, bool keep_col) {
  const uint16_t *wb = c->pbf.as<uint16_t>();
  const float *p = c->p32.as<float>();
  const uint16_t *in = x;
  int64_t sn = 2 * 64 * 64, sc = 64 * 64, sh = 64, sw = 1;  // NCHW input
  for (int l = 0; l < 4; ++l) {
    const ConvSpec &cs = kConv[l];
    const int H = cs.h;
    const int64_t M = n * H * H, K = 9 * cs.cin;
    GemmArgs g = ga(c->col[l].as<uint16_t>(), K, 1, wb + c->L.w[l], 1, K, c->act[l].ptr, cs.cout, 1, M, cs.cout, K);
    if (keep_col) {
      hipLaunchKernelGGL(k_im2col, dim3(grid_for(M * K)), dim3(256), 0, st, in, sn, sc, sh, sw, (int)n, cs.cin, H, H,
                         c->col[l].as<uint16_t>());
    } else {
      g.im_x = in;
      g.im_sn = sn;
      g.im_sc = sc;
      g.im_sh = sh;
      g.im_sw = sw;
      g.im_C = cs.cin;
      g.im_H = H;
    }
    g.bias = p + c->L.b[l];
    g.relu = 1;
    g.out_bf16 = 1;
    if (l == 0 && sn == 2 * 64 * 64 && sc == 64 * 64 && sh == 64 && sw == 1 && cs.cin == 2 && cs.cout == 16 &&
        H == 64 && (reinterpret_cast<uintptr_t>(wb + c->L.w[l]) & 3) == 0)
      hipLaunchKernelGGL(k_conv1, dim3(grid_for(M)), dim3(256), 0, st, in, n, wb + c->L.w[l], p + c->L.b[l],
                         c->act[l].as<uint16_t>());
    else
      gemm(g, st);
    if (cs.cout % 8 == 0)  // the buffers are device allocations: 16-byte aligned rows
      hipLaunchKernelGGL(k_pool_fwd8, dim3(grid_for(M / 4 * cs.cout / 8)), dim3(256), 0, st,
                         c->act[l].as<uint16_t>(), (int)n, cs.cout, H, H, c->pool[l].as<uint16_t>(),
                         c->idx[l].as<uint8_t>());
    else
      hipLaunchKernelGGL(k_pool_fwd, dim3(grid_for(M / 4 * cs.cout)), dim3(256), 0, st, c->act[l].as<uint16_t>(),
                         (int)n, cs.cout, H, H, c->pool[l].as<uint16_t>(), c->idx[l].as<uint8_t>());
    in = c->pool[l].as<uint16_t>();
    const int Ho = H / 2;
    sn = (int64_t)Ho * Ho * cs.cout;
    sc = 1;
    sh = (int64_t)Ho * cs.cout;
    sw = cs.cout;
  }
  // fc1 (+ReLU) and fc2
  GemmArgs g1 = ga(c->pool[3].as<uint16_t>(), kFlat, 1, wb + c->L.w[4], 1, kFlat, c->h1.ptr, kHidden, 1, n, kHidden,
                   kFlat);
  g1.bias = p + c->L.b[4];
  g1.relu = 1;
  g1.out_bf16 = 1;
  gemm(g1, st);
  GemmArgs g2 = ga(c->h1.as<uint16_t>(), kHidden, 1, wb + c->L.w[5], 1, kHidden, c->z.ptr, 1, 1, n, 1, kHidden);
  g2.bias = p + c->L.b[5];
  gemm(g2, st);
}

// Backward pass after forward(): gradients (fp32) of the mean BCE into c->g32.
void backward(gsp_cnn *c, const float *labels, int64_t n, hipStream_t st) {
  const uint16_t *wb = c->pbf.as<uint16_t>();
  float *g = c->g32.as<float>();
  const uint16_t *ones = c->ones.as<uint16_t>();
  // loss head: fp32 dz, fc2's gradients from it, bf16 gradient of fc1's pre-activation
  hipLaunchKernelGGL(k_head_bwd, dim3(grid_for(n * kHidden)), dim3(256), 0, st, c->z.as<float>(), labels,
                     c->h1.as<uint16_t>(), wb + c->L.w[5], (int)n, c->loss.as<float>(), c->dz.as<float>(),
                     c->dh1.as<uint16_t>());
  hipLaunchKernelGGL(k_head_wgrad, dim3(1), dim3(256), 0, st, c->dz.as<float>(), c->h1.as<uint16_t>(), (int)n,
                     g + c->L.w[5], g + c->L.b[5]);
  const uint16_t *dh = c->dh1.as<uint16_t>();
  // fc1: dW = dh^T x, db = colsum dh, dx = dh W1
  gemm(ga(dh, 1, kHidden, c->pool[3].as<uint16_t>(), kFlat, 1, g + c->L.w[4], kFlat, 1, kHidden, kFlat, n), st);
  gemm(ga(ones, 0, 0, dh, kHidden, 1, g + c->L.b[4], 1, 1, 1, kHidden, n), st);
  GemmArgs gx = ga(dh, kHidden, 1, wb + c->L.w[4], kFlat, 1, c->dpool[3].ptr, kFlat, 1, n, kFlat, kHidden);
  gx.out_bf16 = 1;
  gemm(gx, st);
  const uint16_t *dy = c->dpool[3].as<uint16_t>();  // gradient of the pooled output of conv l
  for (int l = 3; l >= 0; --l) {
    const ConvSpec &cs = kConv[l];
    const int H = cs.h;
    const int64_t M = n * H * H, K = 9 * cs.cin;
    uint16_t *dpre = c->dpre.as<uint16_t>();
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid_for(M * cs.cout)), dim3(256), 0, st, dy, c->idx[l].as<uint8_t>(),
                       c->act[l].as<uint16_t>(), (int)n, cs.cout, H, H, dpre);
    // dW[o][k] = sum_p dpre[p][o] col[p][k]; db[o] = sum_p dpre[p][o]
    gemm(ga(dpre, 1, cs.cout, c->col[l].as<uint16_t>(), K, 1, g + c->L.w[l], K, 1, cs.cout, K, M), st);
    gemm(ga(ones, 0, 0, dpre, cs.cout, 1, g + c->L.b[l], 1, 1, 1, cs.cout, M), st);
    if (l == 0) break;
    // dcol = dpre W (fp32); dx = col2im(dcol) (NHWC of the previous pooled output)
    GemmArgs gc = ga(dpre, cs.cout, 1, wb + c->L.w[l], K, 1, c->dcol.ptr, K, 1, M, K, cs.cout);
    gemm(gc, st);
    hipLaunchKernelGGL(k_col2im, dim3(grid_for(M * cs.cin)), dim3(256), 0, st, c->dcol.as<float>(), (int)n, cs.cin,
                       H, H, c->dpool[l - 1].as<uint16_t>());
    dy = c->dpool[l - 1].as<uint16_t>();
  }
  c->last_bwd_n = n;
}

uint64_t splitmix64(uint64_t &s) {
  // SplitMix64 (Steele, Lea & Flood, OOPSLA 2014)
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void upload_params(gsp_cnn *c, const float *host) {
  const int64_t n = c->L.total;
  check_hip(hipMemcpy(c->p32.ptr, host, (size_t)n * 4, hipMemcpyHostToDevice), "copy parameters");
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, 0, c->p32.as<float>(), c->pbf.as<uint16_t>(), n);
  hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(n)), dim3(256), 0, 0, c->m.as<float>(), n);
  hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(n)), dim3(256), 0, 0, c->v.as<float>(), n);
  check_hip(hipDeviceSynchronize(), "initialise parameters");
  c->t = 0;
}

}  // namespace

extern "C" {

int64_t gsp_cnn_num_params(void) { return layout().total; }

int gsp_cnn_create(gsp_ctx *ctx, uint64_t seed, gsp_cnn **out) {
  if (!ctx || !out) return GSP_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&] {
    auto c = std::make_unique<gsp_cnn>();
    c->ctx = ctx;
    c->L = layout();
    const int64_t n = c->L.total;
    for (DevBuf *d : {&c->p32, &c->pbf, &c->g32, &c->m, &c->v}) d->device = ctx->device;
    c->p32.reserve((size_t)n * 4);
    c->pbf.reserve((size_t)n * 2);
    c->g32.reserve((size_t)n * 4);
    c->m.reserve((size_t)n * 4);
    c->v.reserve((size_t)n * 4);
    // He-uniform weights (fan-in), zero biases
    std::vector<float> h((size_t)n, 0.f);
    uint64_t st = seed;
    for (int l = 0; l < 6; ++l) {
      const double fan_in = l < 4 ? 9.0 * kConv[l].cin : (l == 4 ? (double)kFlat : (double)kHidden);
      const double bound = std::sqrt(6.0 / fan_in);
      for (int64_t i = 0; i < c->L.wn[l]; ++i) {
        const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
        h[(size_t)(c->L.w[l] + i)] = (float)((2.0 * u - 1.0) * bound);
      }
    }
    upload_params(c.get(), h.data());
    *out = c.release();
  });
}

void gsp_cnn_destroy(gsp_cnn *c) {
  if (!c) return;
  (void)hipSetDevice(c->ctx->device);
  (void)hipDeviceSynchronize();
  delete c;
}

int gsp_cnn_get_params(gsp_cnn *c, float *host, int64_t n) {
  if (!c || !host || n != c->L.total) return GSP_EINVAL;
  return guarded(c->ctx, [&] {
    check_hip(hipMemcpy(host, c->p32.ptr, (size_t)n * 4, hipMemcpyDeviceToHost), "copy parameters");
  });
}

int gsp_cnn_set_params(gsp_cnn *c, const float *host, int64_t n) {
  if (!c || !host || n != c->L.total) return GSP_EINVAL;
  return guarded(c->ctx, [&] { upload_params(c, host); });
}

int gsp_cnn_save(const gsp_cnn *c, const char *path) {
  if (!c || !path) return GSP_EINVAL;
  std::vector<float> h((size_t)c->L.total);
  if (hipMemcpy(h.data(), c->p32.ptr, h.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return GSP_EDEVICE;
  std::ofstream f(path, std::ios::binary);
  if (!f) return GSP_EINVAL;
  const int64_t n = c->L.total;
  f.write("GSPCNN01", 8);
  f.write(reinterpret_cast<const char *>(&n), 8);
  f.write(reinterpret_cast<const char *>(h.data()), (std::streamsize)(h.size() * 4));
  return f.good() ? GSP_OK : GSP_EINVAL;
}

int gsp_cnn_load(gsp_cnn *c, const char *path) {
  if (!c || !path) return GSP_EINVAL;
  std::ifstream f(path, std::ios::binary);
  char magic[8];
  int64_t n = 0;
  if (!f.read(magic, 8) || std::memcmp(magic, "GSPCNN01", 8) || !f.read(reinterpret_cast<char *>(&n), 8) ||
      n != c->L.total)
    return GSP_EINVAL;
  std::vector<float> h((size_t)n);
  if (!f.read(reinterpret_cast<char *>(h.data()), (std::streamsize)(n * 4))) return GSP_EINVAL;
  return gsp_cnn_set_params(c, h.data(), n);
}

int gsp_cnn_forward(gsp_cnn *c, const uint16_t *x, int64_t n, float *logits, void *stream) {
  if (!c) return GSP_EINVAL;
  return guarded(c->ctx, [&] {
    if (!x || !logits || n < 0) fail(GSP_EINVAL, "bad arguments");
    if (n == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    reserve_batch(c, n);
    forward(c, x, n, st, false);
    c->last_n = n;
    check_hip(hipMemcpyAsync(logits, c->z.ptr, (size_t)n * 4, hipMemcpyDeviceToDevice, st), "copy logits");
  });
}

int gsp_cnn_gradients(gsp_cnn *c, const uint16_t *x, const float *labels, int64_t n, float *grads_host,
                      float *loss_host, void *stream) {
  if (!c) return GSP_EINVAL;
  return guarded(c->ctx, [&] {
    if (!x || !labels || n < 1 || !grads_host) fail(GSP_EINVAL, "bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    reserve_batch(c, n);
    forward(c, x, n, st, true);
    c->last_n = n;
    backward(c, labels, n, st);
    std::vector<float> loss((size_t)n);
    check_hip(hipMemcpyAsync(loss.data(), c->loss.ptr, (size_t)n * 4, hipMemcpyDeviceToHost, st), "copy loss");
    check_hip(hipMemcpyAsync(grads_host, c->g32.ptr, (size_t)c->L.total * 4, hipMemcpyDeviceToHost, st),
              "copy gradients");
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    if (loss_host) {
      double s = 0;
      for (float v : loss) s += v;
      *loss_host = (float)(s / (double)n);
    }
  });
}

int gsp_cnn_train_step(gsp_cnn *c, const uint16_t *x, const float *labels, int64_t n, float lr, float *loss_host,
                       void *stream) {
  if (!c) return GSP_EINVAL;
  return guarded(c->ctx, [&] {
    if (!x || !labels || n < 1 || !(lr > 0)) fail(GSP_EINVAL, "bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    check_hip(hipStreamSynchronize(st), "synchronise stream");
    reserve_batch(c, n);
    forward(c, x, n, st, true);
    c->last_n = n;
    backward(c, labels, n, st);
    c->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)c->t), c2 = 1.f - std::pow(b2, (float)c->t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(c->L.total)), dim3(256), 0, st, c->p32.as<float>(), c->g32.as<float>(),
                       c->m.as<float>(), c->v.as<float>(), c->pbf.as<uint16_t>(), c->L.total, lr, b1, b2, 1e-8f, c1,
                       c2);
    check_hip(hipGetLastError(), "launch adam");
    if (loss_host) {
      std::vector<float> loss((size_t)n);
      check_hip(hipMemcpyAsync(loss.data(), c->loss.ptr, (size_t)n * 4, hipMemcpyDeviceToHost, st), "copy loss");
      check_hip(hipStreamSynchronize(st), "synchronise stream");
      double s = 0;
      for (float v : loss) s += v;
      *loss_host = (float)(s / (double)n);
    }
  });
}

int gsp_cnn_activation(gsp_cnn *c, int32_t which, void *host, int64_t bytes) {
  if (!c) return GSP_EINVAL;
  return guarded(c->ctx, [&] {
    if (!host || which < 0 || which > 19) fail(GSP_EINVAL, "bad arguments");
    const bool bwd = which >= 6 && which <= 11;
    const int64_t n = bwd ? c->last_bwd_n : c->last_n;
    if (n < 1) fail(GSP_EINVAL, bwd ? "no backward pass yet" : "no forward pass yet");
    if (bwd && c->last_n != c->last_bwd_n) fail(GSP_EINVAL, "a forward pass of another batch followed the backward pass");
    const void *src;
    int64_t want;
    if (which < 4) {  // pooled output of block which
      const int h = kConv[which].h / 2;
      want = n * h * h * kConv[which].cout * 2;
      src = c->pool[which].ptr;
    } else if (which == 4) {
      want = n * kHidden * 2;
      src = c->h1.ptr;
    } else if (which == 5) {
      want = n * 4;
      src = c->z.ptr;
    } else if (which < 10) {  // gradient of the pooled output of block which - 6
      const int l = which - 6;
      const int h = kConv[l].h / 2;
      want = n * h * h * kConv[l].cout * 2;
      src = c->dpool[l].ptr;
    } else if (which == 10) {
      want = n * kHidden * 2;
      src = c->dh1.ptr;
    } else if (which == 11) {
      want = n * 4;
      src = c->dz.ptr;
    } else if (which < 16) {  // ReLU output of block which - 12, before pooling
      const int l = which - 12;
      want = n * kConv[l].h * kConv[l].h * kConv[l].cout * 2;
      src = c->act[l].ptr;
    } else {  // max-pool choices of block which - 16
      const int l = which - 16;
      const int h = kConv[l].h / 2;
      want = n * h * h * kConv[l].cout;
      src = c->idx[l].ptr;
    }
    if (bytes != want) fail(GSP_EINVAL, "size does not match the last batch");
    check_hip(hipDeviceSynchronize(), "synchronise");
    check_hip(hipMemcpy(host, src, (size_t)want, hipMemcpyDeviceToHost), "copy activation");
  });
}

int gsp_cutouts(gsp_ctx *ctx, const uint8_t *fb, const double *freqs, const int32_t *dmt, const gsp_dmt_desc *desc,
                const gsp_candidate *cands, int64_t n, uint16_t *out, void *stream) {
  if (!ctx) return GSP_EINVAL;
  return guarded(ctx, [&] {
    validate_desc(desc);
    if (!fb || !freqs || !dmt || (n > 0 && (!cands || !out)) || n < 0) fail(GSP_EINVAL, "bad arguments");
    if (desc->kind != 0) fail(GSP_EINVAL, "cutouts take a brute-force plan's output");
    if (n == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    CutoutArgs a;
    std::memset(&a, 0, sizeof(a));
    a.fb = fb;
    a.cand = cands;
    a.n = n;
    a.nchan = desc->nchan;
    a.n_seg = desc->n_seg;
    a.rmax = 8;
    a.tiled = (desc->nchan % 1024 == 0 && reinterpret_cast<uintptr_t>(fb) % 16 == 0) ? 1 : 0;
    a.out = out;
    for (int32_t s = 0; s < desc->n_seg; ++s) {
      RowTables &rt = row_tables(ctx, desc, freqs, s);
      if (!rt.delays_dev.ptr) {
        rt.delays_dev.device = ctx->device;
        rt.delays_dev.reserve(rt.delays_host.size() * 4);
        check_hip(hipMemcpy(rt.delays_dev.ptr, rt.delays_host.data(), rt.delays_host.size() * 4,
                            hipMemcpyHostToDevice),
                  "copy delays");
      }
      a.row[s].dmt = dmt + desc->offset[s];
      a.row[s].delays = rt.delays_dev.as<int32_t>();
      a.row[s].n_out = desc->n_out[s];
      a.row[s].n_dm = desc->seg[s].n_dm;
      a.row[s].D = desc->seg[s].downsamp;
      a.row[s].trial0 = desc->trial0[s];
    }
    // per-trial means for the bins before the start, of the trials read only
    ctx->need.device = ctx->device;
    ctx->need.reserve((size_t)desc->n_trials * sizeof(uint32_t));
    hipLaunchKernelGGL(k_cutout_need, dim3((unsigned)((desc->n_trials + 255) / 256)), dim3(256), 0, st, a,
                       ctx->need.as<uint32_t>(), desc->n_trials);
    hipLaunchKernelGGL(k_cutout_mark, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, st, a,
                       ctx->need.as<uint32_t>());
    check_hip(hipGetLastError(), "launch cutout trial marks");
    launch_stats(ctx, dmt, desc, st, ctx->need.as<uint32_t>());
    a.musig = ctx->stats.as<double>();
    ctx->ftsums.device = ctx->device;
    ctx->ftsums.reserve((size_t)n * 64 * 64 * sizeof(uint32_t));
    a.ftsums = ctx->ftsums.as<uint32_t>();
    // a multiple of 8 workgroups (k_cutout_ft's XCD mapping needs it)
    const dim3 ft_grid((unsigned)std::min<int64_t>((n + 7) / 8 * 8 * 16, 256 * 64));
    if (n >= kCutStageMin) {
      // a large batch: one channel-major copy of the input (in the staging
      // buffer, which every dedispersion call restages), then contiguous reads;
      // the copy the dedispersion of this output staged last serves when it
      // is of this filterbank at full resolution (rows at least nsamp + 4 long)
      const auto &tag = ctx->staged_tag;
      int64_t pitch = tag.pitch;
      if (!(tag.fb == fb && tag.dmt == dmt && tag.D == 1 && tag.nsamp == desc->nsamp &&
            tag.nchan == desc->nchan && tag.pitch >= desc->nsamp + 4)) {
        pitch = (desc->nsamp + 4 + 255) / 256 * 256;
        stage_raw(ctx, fb, desc->nsamp, desc->nchan, pitch, st);
      }
      a.ycm = ctx->staged.as<uint8_t>();
      a.cm_pitch = pitch;
      hipLaunchKernelGGL(k_cutout_ft_cm, ft_grid, dim3(256), 0, st, a);
    } else {
      hipLaunchKernelGGL(k_cutout_ft, ft_grid, dim3(256), 0, st, a);
    }
    const unsigned grid = (unsigned)std::min<int64_t>(n, 256 * 8);
    hipLaunchKernelGGL(k_cutout, dim3(grid), dim3(256), 0, st, a);
    check_hip(hipGetLastError(), "launch cutouts");
  });
}

}  // extern "C"
