// unet.hip -- gfx950 kernels of the U-Net trained on the auto-labels
// (arXiv 2403.13135, section III-C).  Entry points and layouts: include/sil_unet.h.
//
// Convolutions are GEMMs on MFMA (v_mfma_f32_16x16x32_bf16, fp32 accumulate):
//   * k_gemm_nt: C[m][n] = sum_k A[m][k] * B[n][k], B K-contiguous (weights).
//     A is read as plain rows, as the 3x3 im2col of one or two NHWC tensors
//     (channel concatenation of the decoder's up-sampled and skip maps), or as
//     the 2x2 gather of an up-sampled gradient.  Tiles 128 x BN x 32, 4 waves
//     of 64 x BN/2, operands double-buffered in LDS (rows padded to 80 bytes).
//     Epilogues: bf16 store with per-channel sum / sum of squares for batch
//     normalisation, a channel split into two tensors, or the up-convolution
//     scatter with bias.
//   * k_gemm_tn: weight gradients C[m][n] = sum_p A[p][m] * B[p][n] over pixel
//     ranges (split-K across workgroups, fp32 atomics), both operands
//     transposed into LDS so MFMA reads stay 16-byte contiguous along p.
// Forward conv:  M = pixels, N = cout, K = 9*cin.
// Input grad:    the same kernel on dy with flipped, transposed weights.
// Weight grad:   M = cout, N = 9*cin, reduction over pixels.

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "sil_unet.h"

namespace {

typedef uint16_t u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 256;      // GEMM threads (4 waves)
constexpr int kBM = 128;      // GEMM tile rows
constexpr int kBK = 32;       // reduction step (one MFMA K)
constexpr int kLdsRow = 40;   // u16 per LDS row: 32 + 8 padding (80 bytes)

__device__ __forceinline__ float bf2f(u16 v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ u16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (u16)(u >> 16);
}

enum AMode : int { A_ROWS = 0, A_IM2COL = 1, A_UPGATHER = 2 };
enum EMode : int { E_STORE = 0, E_SPLIT = 1, E_UPSCATTER = 2 };

struct GemmNT {
  int32_t M, N, K;
  const u16* a0;   // ROWS: [M][K]; IM2COL: NHWC [n][H][W][c0]; UPGATHER: [n][2H][2W][c0]
  const u16* a1;   // IM2COL: second source [n][H][W][c1]
  int32_t c0, c1;
  int32_t H, W;    // pixel grid of the A rows (m = (img*H + h)*W + w)
  const u16* b;    // [N][K]
  u16* y0;         // STORE: [M][N]; SPLIT: [M][split]; UPSCATTER: [img][2H][2W][up_cout]
  u16* y1;         // SPLIT: [M][N - split]
  int32_t split, up_cout;
  const float* bias;  // UPSCATTER
  float* stats;       // STORE: [2][N] (nullable)
};

// 16 bytes (8 bf16) of A at row m, reduction index k (k % 8 == 0).
template <int AM>
__device__ __forceinline__ uint4 load_a(const GemmNT& g, int32_t m, int32_t img, int32_t h,
                                        int32_t w, int32_t k) {
  const uint4 zero = make_uint4(0, 0, 0, 0);
  if (m >= g.M || k >= g.K) return zero;
  if constexpr (AM == A_ROWS) {
    return *(const uint4*)(g.a0 + (int64_t)m * g.K + k);
  } else if constexpr (AM == A_IM2COL) {
    const int32_t ct = g.c0 + g.c1;
    const int32_t tap = k / ct, ci = k - tap * ct;
    const int32_t hh = h + tap / 3 - 1, ww = w + tap % 3 - 1;
    if (hh < 0 || hh >= g.H || ww < 0 || ww >= g.W) return zero;
    const int64_t pix = ((int64_t)img * g.H + hh) * g.W + ww;
    if (ci < g.c0) return *(const uint4*)(g.a0 + pix * g.c0 + ci);
    return *(const uint4*)(g.a1 + pix * g.c1 + (ci - g.c0));
  } else {
    const int32_t q = k / g.c0, co = k - q * g.c0;  // k = (i*2 + j)*cout + co
    const int64_t pix = ((int64_t)img * 2 * g.H + 2 * h + (q >> 1)) * (2 * g.W) + 2 * w + (q & 1);
    return *(const uint4*)(g.a0 + pix * g.c0 + co);
  }
}

template <int AM, int EM, int BN>
__global__ __launch_bounds__(kGT) void k_gemm_nt(GemmNT g) {
  __shared__ u16 As[2][kBM][kLdsRow];
  __shared__ u16 Bs[2][BN][kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int32_t m0 = blockIdx.x * kBM, n0 = blockIdx.y * BN;
  constexpr int NJ = BN / 32;  // 16-column MFMA blocks per wave
  constexpr int BCH = BN * 4;  // B chunks per step

  // this thread's A rows (two) and chunk column
  const int kq = tid & 3;
  int32_t am[2], aimg[2], ah[2], aw[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    am[r] = m0 + (tid >> 2) + 64 * r;
    const int32_t mm = min(am[r], g.M - 1);
    aimg[r] = mm / (g.H * g.W);
    const int32_t rem = mm - aimg[r] * g.H * g.W;
    ah[r] = rem / g.W;
    aw[r] = rem - ah[r] * g.W;
  }
  uint4 ra[2], rb[2];
  auto gload = [&](int32_t k0) {
#pragma unroll
    for (int r = 0; r < 2; ++r) ra[r] = load_a<AM>(g, am[r], aimg[r], ah[r], aw[r], k0 + 8 * kq);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int c = tid + kGT * r;
      rb[r] = make_uint4(0, 0, 0, 0);
      if (c < BCH) {
        const int32_t n = n0 + (c >> 2), k = k0 + 8 * (c & 3);
        if (n < g.N && k < g.K) rb[r] = *(const uint4*)(g.b + (int64_t)n * g.K + k);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 2; ++r) *(uint4*)&As[buf][(tid >> 2) + 64 * r][8 * kq] = ra[r];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int c = tid + kGT * r;
      if (c < BCH) *(uint4*)&Bs[buf][c >> 2][8 * (c & 3)] = rb[r];
    }
  };

  f32x4 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nk = (g.K + kBK - 1) / kBK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * kBK);
    bf16x8 a[4], b[NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = __builtin_bit_cast(bf16x8,
                                *(const uint4*)&As[buf][wm * 64 + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      b[j] = __builtin_bit_cast(
          bf16x8, *(const uint4*)&Bs[buf][wn * (BN / 2) + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (kt + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue: acc[i][j][t] is C[row][col], row = wave rows + 16i + 4*(lane/16) + t,
  // col = wave cols + 16j + lane%16
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int32_t col = n0 + wn * (BN / 2) + 16 * j + (lane & 15);
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int32_t row = m0 + wm * 64 + 16 * i + 4 * (lane >> 4) + t;
        const float v = acc[i][j][t];
        if (row >= g.M || col >= g.N) continue;
        if constexpr (EM == E_STORE) {
          g.y0[(int64_t)row * g.N + col] = f2bf(v);
          s1 += v;
          s2 += v * v;
        } else if constexpr (EM == E_SPLIT) {
          if (col < g.split)
            g.y0[(int64_t)row * g.split + col] = f2bf(v);
          else
            g.y1[(int64_t)row * (g.N - g.split) + (col - g.split)] = f2bf(v);
        } else {
          const int32_t q = col / g.up_cout, co = col - q * g.up_cout;
          const int32_t img = row / (g.H * g.W), rem = row - img * g.H * g.W;
          const int32_t h = rem / g.W, w = rem - h * g.W;
          const int64_t pix =
              ((int64_t)img * 2 * g.H + 2 * h + (q >> 1)) * (2 * g.W) + 2 * w + (q & 1);
          g.y0[pix * g.up_cout + co] = f2bf(v + g.bias[co]);
        }
      }
    if constexpr (EM == E_STORE) {
      if (g.stats) {
        s1 += __shfl_xor(s1, 16);
        s1 += __shfl_xor(s1, 32);
        s2 += __shfl_xor(s2, 16);
        s2 += __shfl_xor(s2, 32);
        if (lane < 16 && col < g.N) {
          atomicAdd(&g.stats[col], s1);
          atomicAdd(&g.stats[g.N + col], s2);
        }
      }
    }
  }
}

// ---- weight gradients ----------------------------------------------------------

enum TMode : int { T_PLAIN = 0, T_IM2COL = 1, T_UPGATHER = 2 };

struct GemmTN {
  int32_t M, N;    // C [M][N] fp32, accumulate
  int64_t P;       // pixels reduced over
  int32_t H, W;    // pixel grid
  // A[p][m]: PLAIN: a [P][M]; UPGATHER: a = dy [img][2H][2W][M/4], m = q*cout + co
  const u16* a;
  // B[p][n]: PLAIN: b0 [P][N]; IM2COL: n = tap*(c0+c1) + ci over concat(b0, b1)
  const u16* b0;
  const u16* b1;
  int32_t c0, c1;
  int64_t p_per_split;
  float* c;
};

template <int MODE>
__device__ __forceinline__ uint4 load_tn(const GemmTN& g, const u16* base, int32_t ld, int64_t p,
                                         int32_t idx, bool is_b) {
  const uint4 zero = make_uint4(0, 0, 0, 0);
  if (p >= g.P) return zero;
  if constexpr (MODE == T_PLAIN) {
    return *(const uint4*)(base + p * ld + idx);
  } else {
    const int32_t img = (int32_t)(p / ((int64_t)g.H * g.W));
    const int32_t rem = (int32_t)(p - (int64_t)img * g.H * g.W);
    const int32_t h = rem / g.W, w = rem - h * g.W;
    if constexpr (MODE == T_IM2COL) {
      const int32_t ct = g.c0 + g.c1;
      const int32_t tap = idx / ct, ci = idx - tap * ct;
      const int32_t hh = h + tap / 3 - 1, ww = w + tap % 3 - 1;
      if (hh < 0 || hh >= g.H || ww < 0 || ww >= g.W) return zero;
      const int64_t pix = ((int64_t)img * g.H + hh) * g.W + ww;
      if (ci < g.c0) return *(const uint4*)(g.b0 + pix * g.c0 + ci);
      return *(const uint4*)(g.b1 + pix * g.c1 + (ci - g.c0));
    } else {
      const int32_t cout = g.M / 4;
      const int32_t q = idx / cout, co = idx - q * cout;
      const int64_t pix = ((int64_t)img * 2 * g.H + 2 * h + (q >> 1)) * (2 * g.W) + 2 * w + (q & 1);
      return *(const uint4*)(g.a + pix * cout + co);
    }
  }
}

// AM: mode of A (T_PLAIN or T_UPGATHER); BMD: mode of B (T_PLAIN or T_IM2COL).
template <int AM, int BMD, int BM, int BN>
__global__ __launch_bounds__(kGT) void k_gemm_tn(GemmTN g) {
  __shared__ u16 As[BM][kLdsRow];
  __shared__ u16 Bs[BN][kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int32_t m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  constexpr int MI = BM / 32, NJ = BN / 32;
  constexpr int ACH = kBK * BM / 8, BCH = kBK * BN / 8;  // 16-byte chunks per step
  const int64_t p_begin = (int64_t)blockIdx.z * g.p_per_split;
  const int64_t p_end = min(g.P, p_begin + g.p_per_split);

  f32x4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t p0 = p_begin; p0 < p_end; p0 += kBK) {
    // stage A^T and B^T: chunk c covers 8 consecutive m (or n) at one pixel
    for (int c = tid; c < ACH; c += kGT) {
      const int pl = c / (BM / 8), mc = 8 * (c % (BM / 8));
      const int64_t p = p0 + pl;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (p < p_end && m0 + mc < g.M) v = load_tn<AM>(g, g.a, g.M, p, m0 + mc, false);
      const u16* e = (const u16*)&v;
#pragma unroll
      for (int t = 0; t < 8; ++t) As[mc + t][pl] = e[t];
    }
    for (int c = tid; c < BCH; c += kGT) {
      const int pl = c / (BN / 8), nc = 8 * (c % (BN / 8));
      const int64_t p = p0 + pl;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (p < p_end && n0 + nc < g.N) v = load_tn<BMD>(g, g.b0, g.N, p, n0 + nc, true);
      const u16* e = (const u16*)&v;
#pragma unroll
      for (int t = 0; t < 8; ++t) Bs[nc + t][pl] = e[t];
    }
    __syncthreads();
    bf16x8 a[MI], b[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
      a[i] = __builtin_bit_cast(
          bf16x8, *(const uint4*)&As[wm * (BM / 2) + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      b[j] = __builtin_bit_cast(
          bf16x8, *(const uint4*)&Bs[wn * (BN / 2) + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int32_t row = m0 + wm * (BM / 2) + 16 * i + 4 * (lane >> 4) + t;
        const int32_t col = n0 + wn * (BN / 2) + 16 * j + (lane & 15);
        if (row < g.M && col < g.N) atomicAdd(&g.c[(int64_t)row * g.N + col], acc[i][j][t]);
      }
}

// ---- elementwise and reduction kernels ----------------------------------------

__global__ void k_fill(float* x, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_to_bf16(const float* x, u16* y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

__global__ void k_flip3x3(const u16* w, u16* wt, int32_t cout, int32_t cin) {
  const int64_t n = (int64_t)cout * 9 * cin;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // i indexes wt[ci][r][s][co]
    const int32_t co = (int32_t)(i % cout);
    const int32_t rs = (int32_t)((i / cout) % 9);
    const int32_t ci = (int32_t)(i / ((int64_t)cout * 9));
    const int32_t r = rs / 3, s = rs % 3;
    wt[i] = w[((int64_t)co * 9 + (2 - r) * 3 + (2 - s)) * cin + ci];
  }
}

__global__ void k_up_t(const u16* w, u16* wt, int32_t cin, int32_t cout) {
  const int64_t n = (int64_t)4 * cout * cin;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // i indexes wt[ci][q][co]; w is [q][co][ci]
    const int32_t co = (int32_t)(i % cout);
    const int32_t q = (int32_t)((i / cout) % 4);
    const int32_t ci = (int32_t)(i / ((int64_t)cout * 4));
    wt[i] = w[((int64_t)q * cout + co) * cin + ci];
  }
}

// per-channel (mean, rstd) from sums, in double
__global__ void k_bn_stats(const float* stats, int32_t C, int64_t count, float eps, float* mr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const double mean = (double)stats[c] / (double)count;
  double var = (double)stats[C + c] / (double)count - mean * mean;
  if (var < 0) var = 0;
  mr[c] = (float)mean;
  mr[C + c] = (float)(1.0 / sqrt(var + (double)eps));
}

__global__ void k_bn_relu(const u16* z, const float* mr, const float* gamma, const float* beta,
                          u16* out, int64_t n, int32_t C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = (int32_t)(i % C);
    const float v = (bf2f(z[i]) - mr[c]) * mr[C + c] * gamma[c] + beta[c];
    out[i] = f2bf(v > 0.f ? v : 0.f);
  }
}

// Per-channel sums over [P][C] of f(p, c) with blocks of 256 threads; C <= 256
// and 256 % C == 0.  Each block reduces its rows in LDS, then one atomic per
// channel.
__global__ void k_bn_bwd_reduce(const u16* dout, const u16* z, const float* mr,
                                const float* gamma, const float* beta, float* red, int64_t P,
                                int32_t C) {
  __shared__ float s1[256], s2[256];
  const int t = threadIdx.x;
  const int c = t % C, r0 = t / C, rstep = 256 / C;
  float a1 = 0.f, a2 = 0.f;
  const int64_t rows_per_block = (P + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(P, rb + rows_per_block);
  for (int64_t p = rb + r0; p < re; p += rstep) {
    const int64_t i = p * C + c;
    const float zh = (bf2f(z[i]) - mr[c]) * mr[C + c];
    const float pre = zh * gamma[c] + beta[c];
    const float d = pre > 0.f ? bf2f(dout[i]) : 0.f;
    a1 += d;
    a2 += d * zh;
  }
  s1[t] = a1;
  s2[t] = a2;
  __syncthreads();
  if (t < C) {
    float b1 = 0.f, b2 = 0.f;
    for (int k = t; k < 256; k += C) {
      b1 += s1[k];
      b2 += s2[k];
    }
    atomicAdd(&red[c], b1);
    atomicAdd(&red[C + c], b2);
  }
}

__global__ void k_bn_bwd_apply(const u16* dout, const u16* z, const float* mr, const float* gamma,
                               const float* beta, const float* red, u16* dz, int64_t n, int32_t C,
                               float inv_count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = (int32_t)(i % C);
    const float zh = (bf2f(z[i]) - mr[c]) * mr[C + c];
    const float pre = zh * gamma[c] + beta[c];
    const float d = pre > 0.f ? bf2f(dout[i]) : 0.f;
    const float g = gamma[c] * mr[C + c] * (d - (red[c] + zh * red[C + c]) * inv_count);
    dz[i] = f2bf(g);
  }
}

__global__ void k_affine_relu(const u16* z, const float* scale, const float* shift, u16* out,
                              int64_t n, int32_t C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = (int32_t)(i % C);
    const float v = bf2f(z[i]) * scale[c] + shift[c];
    out[i] = f2bf(v > 0.f ? v : 0.f);
  }
}

__global__ void k_scatter_argmax(const float* logits, const int32_t* origins, int32_t n_chips,
                                 int32_t chip, uint8_t* labels, int32_t H, int32_t W,
                                 int64_t lpitch) {
  const int64_t n = (int64_t)n_chips * chip * chip;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = (int32_t)(i % chip);
    const int32_t h = (int32_t)((i / chip) % chip);
    const int32_t k = (int32_t)(i / ((int64_t)chip * chip));
    const int32_t y = origins[2 * k] + h, x = origins[2 * k + 1] + w;
    if (y < 0 || y >= H || x < 0 || x >= W) continue;
    const float a = logits[3 * i], b = logits[3 * i + 1], c = logits[3 * i + 2];
    uint8_t cls = 0;
    float m = a;
    if (b > m) {
      m = b;
      cls = 1;
    }
    if (c > m) cls = 2;
    labels[(int64_t)y * lpitch + x] = cls;
  }
}

__global__ void k_add_vec(float* dst, const float* src, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += src[i];
}

__global__ void k_maxpool(const u16* x, u16* y, uint8_t* idx, int32_t N, int32_t H, int32_t W,
                          int32_t C) {
  const int32_t Ho = H / 2, Wo = W / 2;
  const int64_t n = (int64_t)N * Ho * Wo * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = (int32_t)(i % C);
    int64_t r = i / C;
    const int32_t wo = (int32_t)(r % Wo);
    r /= Wo;
    const int32_t ho = (int32_t)(r % Ho);
    const int32_t img = (int32_t)(r / Ho);
    float best = 0.f;
    int bi = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float v = bf2f(x[(((int64_t)img * H + 2 * ho + (k >> 1)) * W + 2 * wo + (k & 1)) * C + c]);
      if (k == 0 || v > best) {
        best = v;
        bi = k;
      }
    }
    y[i] = f2bf(best);
    idx[i] = (uint8_t)bi;
  }
}

__global__ void k_maxpool_bwd(const u16* dy, const uint8_t* idx, u16* dx, int32_t N, int32_t H,
                              int32_t W, int32_t C) {
  const int64_t n = (int64_t)N * H * W * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = (int32_t)(i % C);
    int64_t r = i / C;
    const int32_t w = (int32_t)(r % W);
    r /= W;
    const int32_t h = (int32_t)(r % H);
    const int32_t img = (int32_t)(r / H);
    const int64_t o = (((int64_t)img * (H / 2) + h / 2) * (W / 2) + w / 2) * C + c;
    const int k = (h & 1) * 2 + (w & 1);
    dx[i] = idx[o] == k ? dy[o] : (u16)0;
  }
}

__global__ void k_head(const u16* x, const float* w, const float* b, float* logits, int64_t P,
                       int32_t C) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    float l0 = b[0], l1 = b[1], l2 = b[2];
    for (int32_t c = 0; c < C; ++c) {
      const float v = bf2f(x[p * C + c]);
      l0 += v * w[c];
      l1 += v * w[C + c];
      l2 += v * w[2 * C + c];
    }
    logits[3 * p] = l0;
    logits[3 * p + 1] = l1;
    logits[3 * p + 2] = l2;
  }
}

__global__ void k_softmax_xent(const float* logits, const uint8_t* labels, float* loss,
                               float* dlogits, float scale, int64_t P) {
  __shared__ float part[256];
  float acc = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float a = logits[3 * p], b = logits[3 * p + 1], c = logits[3 * p + 2];
    const float mx = fmaxf(a, fmaxf(b, c));
    const float ea = expf(a - mx), eb = expf(b - mx), ec = expf(c - mx);
    const float s = ea + eb + ec;
    const int y = labels[p];
    const float ly = y == 0 ? a : (y == 1 ? b : c);
    acc += logf(s) + mx - ly;
    if (dlogits) {
      const float inv = 1.f / s;
      dlogits[3 * p] = (ea * inv - (y == 0)) * scale;
      dlogits[3 * p + 1] = (eb * inv - (y == 1)) * scale;
      dlogits[3 * p + 2] = (ec * inv - (y == 2)) * scale;
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, part[0]);
}

// head backward, input gradient: one thread per (pixel, channel)
__global__ void k_head_dx(const float* w, const float* dl, u16* dx, int64_t P, int32_t C) {
  const int64_t n = P * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / C;
    const int32_t c = (int32_t)(i - p * C);
    dx[i] = f2bf(dl[3 * p] * w[c] + dl[3 * p + 1] * w[C + c] + dl[3 * p + 2] * w[2 * C + c]);
  }
}

// head backward, weight and bias gradients: thread t sums channel t % C over
// rows t / C + k * (256 / C) of its block's row range (256 % C == 0)
__global__ void k_head_dw(const u16* x, const float* dl, float* dw, float* db, int64_t P,
                          int32_t C) {
  __shared__ float s[3][256];
  __shared__ float sb[3][256];
  const int t = threadIdx.x, c = t % C, r0 = t / C, rstep = 256 / C;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
  const int64_t rows_per_block = (P + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(P, rb + rows_per_block);
  for (int64_t p = rb + r0; p < re; p += rstep) {
    const float v = bf2f(x[p * C + c]);
    const float d0 = dl[3 * p], d1 = dl[3 * p + 1], d2 = dl[3 * p + 2];
    a0 += d0 * v;
    a1 += d1 * v;
    a2 += d2 * v;
    if (c == 0) {
      b0 += d0;
      b1 += d1;
      b2 += d2;
    }
  }
  s[0][t] = a0;
  s[1][t] = a1;
  s[2][t] = a2;
  sb[0][t] = b0;
  sb[1][t] = b1;
  sb[2][t] = b2;
  __syncthreads();
  if (t < C) {
    float e0 = 0.f, e1 = 0.f, e2 = 0.f;
    for (int k = t; k < 256; k += C) {
      e0 += s[0][k];
      e1 += s[1][k];
      e2 += s[2][k];
    }
    atomicAdd(&dw[c], e0);
    atomicAdd(&dw[C + c], e1);
    atomicAdd(&dw[2 * C + c], e2);
  }
  if (t < 3) {
    float e = 0.f;
    for (int k = 0; k < 256; k += C) e += sb[t][k];
    atomicAdd(&db[t], e);
  }
}

__global__ void k_argmax(const float* logits, uint8_t* labels, int64_t P) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float a = logits[3 * p], b = logits[3 * p + 1], c = logits[3 * p + 2];
    uint8_t k = 0;
    float m = a;
    if (b > m) {
      m = b;
      k = 1;
    }
    if (c > m) k = 2;
    labels[p] = k;
  }
}

// column sums of dy [P][C] into db (accumulate); blocks of 256, 256 % C == 0
__global__ void k_colsum(const u16* dy, float* db, int64_t P, int32_t C) {
  __shared__ float s[256];
  const int t = threadIdx.x, c = t % C, r0 = t / C, rstep = 256 / C;
  float a = 0.f;
  const int64_t rows_per_block = (P + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(P, rb + rows_per_block);
  for (int64_t p = rb + r0; p < re; p += rstep) a += bf2f(dy[p * C + c]);
  s[t] = a;
  __syncthreads();
  if (t < C) {
    float b = 0.f;
    for (int k = t; k < 256; k += C) b += s[k];
    atomicAdd(&db[c], b);
  }
}

__global__ void k_chips_input(const u16* scene, int32_t H, int32_t W, int64_t pitch,
                              const int32_t* origins, int32_t n_chips, int32_t chip,
                              float inv_refl, u16* out) {
  const int64_t n = (int64_t)n_chips * chip * chip;
  const int64_t plane = (int64_t)H * pitch;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = (int32_t)(i % chip);
    const int32_t h = (int32_t)((i / chip) % chip);
    const int32_t k = (int32_t)(i / ((int64_t)chip * chip));
    const int32_t y = origins[2 * k] + h, x = origins[2 * k + 1] + w;
    u16 v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (y >= 0 && y < H && x >= 0 && x < W) {
      const int64_t o = (int64_t)y * pitch + x;
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = f2bf((float)scene[c * plane + o] * inv_refl);
    }
    *(uint4*)(out + i * 8) = *(const uint4*)v;
  }
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, u16* wbf, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
  }
}

// ---- host helpers ---------------------------------------------------------------

int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

int done() { return hipGetLastError() == hipSuccess ? SIL_OK : SIL_EDEVICE; }

template <int AM, int EM>
int launch_nt(const GemmNT& g, hipStream_t st) {
  (void)hipGetLastError();
  const int bn = g.N % 128 == 0 ? 128 : (g.N % 64 == 0 ? 64 : 32);
  dim3 grid((g.M + kBM - 1) / kBM, (g.N + bn - 1) / bn);
  if (bn == 128)
    hipLaunchKernelGGL((k_gemm_nt<AM, EM, 128>), grid, dim3(kGT), 0, st, g);
  else if (bn == 64)
    hipLaunchKernelGGL((k_gemm_nt<AM, EM, 64>), grid, dim3(kGT), 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm_nt<AM, EM, 32>), grid, dim3(kGT), 0, st, g);
  return done();
}

template <int AM, int BMD>
int launch_tn(GemmTN g, hipStream_t st) {
  (void)hipGetLastError();
  const int bm = g.M % 128 == 0 ? 128 : (g.M % 64 == 0 ? 64 : 32);
  const int bn = g.N % 128 == 0 ? 128 : (g.N % 64 == 0 ? 64 : 32);
  const int64_t tiles = (int64_t)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  // split the pixel reduction so that roughly 2048 workgroups run
  int64_t splits = (2048 + tiles - 1) / tiles;
  const int64_t max_splits = (g.P + 255) / 256;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  g.p_per_split = ((g.P + splits - 1) / splits + kBK - 1) / kBK * kBK;
  splits = (g.P + g.p_per_split - 1) / g.p_per_split;
  dim3 grid((g.M + bm - 1) / bm, (g.N + bn - 1) / bn, (unsigned)splits);
#define SIL_TN(BMv, BNv) \
  hipLaunchKernelGGL((k_gemm_tn<AM, BMD, BMv, BNv>), grid, dim3(kGT), 0, st, g)
  if (bm == 128 && bn == 128) SIL_TN(128, 128);
  else if (bm == 128 && bn == 64) SIL_TN(128, 64);
  else if (bm == 128) SIL_TN(128, 32);
  else if (bm == 64 && bn == 128) SIL_TN(64, 128);
  else if (bm == 64 && bn == 64) SIL_TN(64, 64);
  else if (bm == 64) SIL_TN(64, 32);
  else if (bn == 128) SIL_TN(32, 128);
  else if (bn == 64) SIL_TN(32, 64);
  else SIL_TN(32, 32);
#undef SIL_TN
  return done();
}

bool ok_dims(int32_t N, int32_t H, int32_t W) { return N > 0 && H > 0 && W > 0; }

}  // namespace

extern "C" {

int sil_unet_conv3x3(const void* x0, int32_t c0, const void* x1, int32_t c1, const void* w,
                     void* y, float* stats, int32_t N, int32_t H, int32_t W, int32_t cout,
                     void* stream) {
  if (!x0 || !w || !y || (c1 > 0 && !x1) || !ok_dims(N, H, W)) return SIL_EINVAL;
  if (c0 <= 0 || c0 % 8 || c1 < 0 || c1 % 8 || cout <= 0 || cout % 8) return SIL_EINVAL;
  GemmNT g{};
  g.M = N * H * W;
  g.N = cout;
  g.K = 9 * (c0 + c1);
  g.a0 = (const u16*)x0;
  g.a1 = (const u16*)x1;
  g.c0 = c0;
  g.c1 = c1;
  g.H = H;
  g.W = W;
  g.b = (const u16*)w;
  g.y0 = (u16*)y;
  g.stats = stats;
  return launch_nt<A_IM2COL, E_STORE>(g, (hipStream_t)stream);
}

int sil_unet_conv3x3_dgrad(const void* dy, int32_t cout, const void* wt, void* dx0, int32_t c0,
                           void* dx1, int32_t c1, int32_t N, int32_t H, int32_t W, void* stream) {
  if (!dy || !wt || !dx0 || (c1 > 0 && !dx1) || !ok_dims(N, H, W)) return SIL_EINVAL;
  if (cout <= 0 || cout % 8 || c0 <= 0 || c0 % 8 || c1 < 0 || c1 % 8) return SIL_EINVAL;
  GemmNT g{};
  g.M = N * H * W;
  g.N = c0 + c1;
  g.K = 9 * cout;
  g.a0 = (const u16*)dy;
  g.c0 = cout;
  g.c1 = 0;
  g.H = H;
  g.W = W;
  g.b = (const u16*)wt;
  g.y0 = (u16*)dx0;
  g.y1 = (u16*)dx1;
  g.split = c1 > 0 ? c0 : c0 + c1;
  if (c1 > 0) return launch_nt<A_IM2COL, E_SPLIT>(g, (hipStream_t)stream);
  return launch_nt<A_IM2COL, E_STORE>(g, (hipStream_t)stream);
}

int sil_unet_conv3x3_wgrad(const void* dy, int32_t cout, const void* x0, int32_t c0,
                           const void* x1, int32_t c1, float* dw, int32_t N, int32_t H,
                           int32_t W, void* stream) {
  if (!dy || !x0 || !dw || (c1 > 0 && !x1) || !ok_dims(N, H, W)) return SIL_EINVAL;
  if (cout <= 0 || cout % 8 || c0 <= 0 || c0 % 8 || c1 < 0 || c1 % 8) return SIL_EINVAL;
  GemmTN g{};
  g.M = cout;
  g.N = 9 * (c0 + c1);
  g.P = (int64_t)N * H * W;
  g.H = H;
  g.W = W;
  g.a = (const u16*)dy;
  g.b0 = (const u16*)x0;
  g.b1 = (const u16*)x1;
  g.c0 = c0;
  g.c1 = c1;
  g.c = dw;
  return launch_tn<T_PLAIN, T_IM2COL>(g, (hipStream_t)stream);
}

int sil_unet_flip3x3(const void* w, void* wt, int32_t cout, int32_t cin, void* stream) {
  if (!w || !wt || cout <= 0 || cin <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)cout * 9 * cin;
  hipLaunchKernelGGL(k_flip3x3, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)w, (u16*)wt, cout, cin);
  return done();
}

int sil_unet_upconv(const void* x, const void* w, const float* b, void* y, int32_t N, int32_t H,
                    int32_t W, int32_t cin, int32_t cout, void* stream) {
  if (!x || !w || !b || !y || !ok_dims(N, H, W) || cin <= 0 || cin % 8 || cout <= 0 ||
      cout % 8)
    return SIL_EINVAL;
  GemmNT g{};
  g.M = N * H * W;
  g.N = 4 * cout;
  g.K = cin;
  g.a0 = (const u16*)x;
  g.H = H;
  g.W = W;
  g.b = (const u16*)w;
  g.y0 = (u16*)y;
  g.up_cout = cout;
  g.bias = b;
  return launch_nt<A_ROWS, E_UPSCATTER>(g, (hipStream_t)stream);
}

int sil_unet_upconv_dgrad(const void* dy, const void* wt, void* dx, int32_t N, int32_t H,
                          int32_t W, int32_t cin, int32_t cout, void* stream) {
  if (!dy || !wt || !dx || !ok_dims(N, H, W) || cin <= 0 || cin % 8 || cout <= 0 || cout % 8)
    return SIL_EINVAL;
  GemmNT g{};
  g.M = N * H * W;
  g.N = cin;
  g.K = 4 * cout;
  g.a0 = (const u16*)dy;
  g.c0 = cout;
  g.H = H;
  g.W = W;
  g.b = (const u16*)wt;
  g.y0 = (u16*)dx;
  return launch_nt<A_UPGATHER, E_STORE>(g, (hipStream_t)stream);
}

int sil_unet_upconv_wgrad(const void* x, const void* dy, float* dw, float* db, int32_t N,
                          int32_t H, int32_t W, int32_t cin, int32_t cout, void* stream) {
  if (!x || !dy || !dw || !db || !ok_dims(N, H, W) || cin <= 0 || cin % 8 || cout <= 0 ||
      cout % 8)
    return SIL_EINVAL;
  GemmTN g{};
  g.M = 4 * cout;
  g.N = cin;
  g.P = (int64_t)N * H * W;
  g.H = H;
  g.W = W;
  g.a = (const u16*)dy;
  g.b0 = (const u16*)x;
  g.c = dw;
  int rc = launch_tn<T_UPGATHER, T_PLAIN>(g, (hipStream_t)stream);
  if (rc != SIL_OK) return rc;
  if (256 % cout) return SIL_EINVAL;
  const int64_t Pout = (int64_t)N * 4 * H * W;
  hipLaunchKernelGGL(k_colsum, dim3(grid_for(Pout / 64 + 1, 1)), dim3(256), 0,
                     (hipStream_t)stream, (const u16*)dy, db, Pout, cout);
  return done();
}

int sil_unet_up_t(const void* w, void* wt, int32_t cin, int32_t cout, void* stream) {
  if (!w || !wt || cin <= 0 || cout <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)4 * cout * cin;
  hipLaunchKernelGGL(k_up_t, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)w, (u16*)wt, cin, cout);
  return done();
}

int sil_unet_bn_relu(const void* z, const float* stats, const float* gamma, const float* beta,
                     float eps, int64_t count, void* out, float* mr, int64_t P, int32_t C,
                     void* stream) {
  if (!z || !stats || !gamma || !beta || !out || !mr || count <= 0 || P <= 0 || C <= 0)
    return SIL_EINVAL;
  (void)hipGetLastError();
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_bn_stats, dim3((C + 255) / 256), dim3(256), 0, st, stats, C, count, eps,
                     mr);
  const int64_t n = P * C;
  hipLaunchKernelGGL(k_bn_relu, dim3(grid_for(n)), dim3(256), 0, st, (const u16*)z, mr, gamma,
                     beta, (u16*)out, n, C);
  return done();
}

int sil_unet_affine_relu(const void* z, const float* scale, const float* shift, void* out,
                         int64_t P, int32_t C, void* stream) {
  if (!z || !scale || !shift || !out || P <= 0 || C <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = P * C;
  hipLaunchKernelGGL(k_affine_relu, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)z, scale, shift, (u16*)out, n, C);
  return done();
}

int sil_unet_scatter_argmax(const float* logits, const int32_t* origins, int32_t n_chips,
                            int32_t chip, uint8_t* labels, int32_t H, int32_t W, int64_t lpitch,
                            void* stream) {
  if (!logits || !origins || !labels || n_chips <= 0 || chip <= 0 || H <= 0 || W <= 0 ||
      lpitch < W)
    return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)n_chips * chip * chip;
  hipLaunchKernelGGL(k_scatter_argmax, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     logits, origins, n_chips, chip, labels, H, W, lpitch);
  return done();
}

int sil_unet_bn_relu_bwd(const void* dout, const void* z, const float* mr, const float* gamma,
                         const float* beta, void* dz, float* dgamma, float* dbeta, float* red,
                         int64_t P, int32_t C, void* stream) {
  if (!dout || !z || !mr || !gamma || !beta || !dz || !dgamma || !dbeta || !red || P <= 0 ||
      C <= 0 || C > 256 || 256 % C)
    return SIL_EINVAL;
  (void)hipGetLastError();
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, st, red, (int64_t)2 * C, 0.f);
  hipLaunchKernelGGL(k_bn_bwd_reduce, dim3(grid_for(P / 64 + 1, 1)), dim3(256), 0, st,
                     (const u16*)dout, (const u16*)z, mr, gamma, beta, red, P, C);
  const int64_t n = P * C;
  hipLaunchKernelGGL(k_bn_bwd_apply, dim3(grid_for(n)), dim3(256), 0, st, (const u16*)dout,
                     (const u16*)z, mr, gamma, beta, red, (u16*)dz, n, C, 1.f / (float)P);
  hipLaunchKernelGGL(k_add_vec, dim3((C + 255) / 256), dim3(256), 0, st, dbeta, red, C);
  hipLaunchKernelGGL(k_add_vec, dim3((C + 255) / 256), dim3(256), 0, st, dgamma, red + C, C);
  return done();
}

int sil_unet_maxpool(const void* x, void* y, uint8_t* idx, int32_t N, int32_t H, int32_t W,
                     int32_t C, void* stream) {
  if (!x || !y || !idx || !ok_dims(N, H, W) || H % 2 || W % 2 || C <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)N * (H / 2) * (W / 2) * C;
  hipLaunchKernelGGL(k_maxpool, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)x, (u16*)y, idx, N, H, W, C);
  return done();
}

int sil_unet_maxpool_bwd(const void* dy, const uint8_t* idx, void* dx, int32_t N, int32_t H,
                         int32_t W, int32_t C, void* stream) {
  if (!dy || !idx || !dx || !ok_dims(N, H, W) || H % 2 || W % 2 || C <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)N * H * W * C;
  hipLaunchKernelGGL(k_maxpool_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)dy, idx, (u16*)dx, N, H, W, C);
  return done();
}

int sil_unet_head(const void* x, const float* w, const float* b, float* logits, int64_t P,
                  int32_t C, void* stream) {
  if (!x || !w || !b || !logits || P <= 0 || C <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_head, dim3(grid_for(P)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)x, w, b, logits, P, C);
  return done();
}

int sil_unet_softmax_xent(const float* logits, const uint8_t* labels, float* loss,
                          float* dlogits, float scale, int64_t P, void* stream) {
  if (!logits || !labels || !loss || P <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_softmax_xent, dim3(grid_for(P)), dim3(256), 0, (hipStream_t)stream,
                     logits, labels, loss, dlogits, scale, P);
  return done();
}

int sil_unet_head_bwd(const void* x, const float* w, const float* dlogits, void* dx, float* dw,
                      float* db, int64_t P, int32_t C, void* stream) {
  if (!x || !w || !dlogits || !dx || !dw || !db || P <= 0 || C <= 0 || C > 256 || 256 % C)
    return SIL_EINVAL;
  (void)hipGetLastError();
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_head_dx, dim3(grid_for(P * C)), dim3(256), 0, st, w, dlogits, (u16*)dx,
                     P, C);
  hipLaunchKernelGGL(k_head_dw, dim3(grid_for(P / 64 + 1, 1)), dim3(256), 0, st, (const u16*)x,
                     dlogits, dw, db, P, C);
  return done();
}

int sil_unet_argmax(const float* logits, uint8_t* labels, int64_t P, void* stream) {
  if (!logits || !labels || P <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_argmax, dim3(grid_for(P)), dim3(256), 0, (hipStream_t)stream, logits,
                     labels, P);
  return done();
}

int sil_unet_chips_input(const uint16_t* scene, int32_t H, int32_t W, int64_t pitch,
                         const int32_t* origins, int32_t n_chips, int32_t chip, float inv_refl,
                         void* out, void* stream) {
  if (!scene || !origins || !out || H <= 0 || W <= 0 || pitch < W || n_chips <= 0 || chip <= 0)
    return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)n_chips * chip * chip;
  hipLaunchKernelGGL(k_chips_input, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)scene, H, W, pitch, origins, n_chips, chip, inv_refl,
                     (u16*)out);
  return done();
}

int sil_unet_adam(float* w, const float* g, float* m, float* v, void* wbf, int64_t n, float lr,
                  float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (!w || !g || !m || !v || n <= 0 || step < 1) return SIL_EINVAL;
  (void)hipGetLastError();
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                     (u16*)wbf, n, lr, beta1, beta2, eps, c1, c2);
  return done();
}

int sil_unet_to_bf16(const float* x, void* y, int64_t n, void* stream) {
  if (!x || !y || n <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x,
                     (u16*)y, n);
  return done();
}

int sil_unet_fill_f32(float* x, int64_t n, float v, void* stream) {
  if (!x || n <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, n, v);
  return done();
}

}  // extern "C"
