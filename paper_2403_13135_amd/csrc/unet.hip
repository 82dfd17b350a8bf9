// unet.hip -- gfx950 kernels of the U-Net trained on the auto-labels
// (arXiv 2403.13135, section III-C).  Entry points and layouts: include/sil_unet.h.
//
// Convolutions are GEMMs on MFMA (v_mfma_f32_16x16x32_bf16, fp32 accumulate):
//   * k_gemm_nt: C[m][n] = sum_k A[m][k] * B[n][k], B K-contiguous (weights).
//     A is read as plain rows, as the 3x3 im2col of one or two NHWC tensors
//     (channel concatenation of the decoder's up-sampled and skip maps), or as
//     the 2x2 gather of an up-sampled gradient.  Tiles of 4 waves, each wave
//     64 rows x 16*NJ columns (128 x 128, 128 x 64, or 256 x 32 for narrow
//     outputs), K steps of 32, operands double-buffered in LDS (rows padded to
//     80 bytes); a block walks several M tiles.  Epilogues: bf16 store with
//     per-channel sum / sum of squares for batch normalisation (reduced in LDS,
//     one atomic per column per block), a channel split into two tensors, or
//     the up-convolution scatter with bias.
//   * k_gemm_tn: weight gradients C[m][n] = sum_p A[p][m] * B[p][n] over pixel
//     ranges (split-K across workgroups, fp32 atomics), both operands
//     transposed into LDS (pixel pairs packed into 4-byte writes) so MFMA reads
//     stay 16-byte contiguous along p; tiles 32*MI x 32*NJ.
// Forward conv:  M = pixels, N = cout, K = 9*cin.
// Input grad:    the same kernel on dy with flipped, transposed weights.
// Weight grad:   M = cout, N = 9*cin, reduction over pixels.

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "sil_unet.h"

namespace {

typedef uint16_t u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 256;      // GEMM threads (4 waves)
constexpr int kBK = 32;       // reduction step (one MFMA K)
constexpr int kLdsRow = 40;   // u16 per LDS row: 32 + 8 padding (80 bytes)

// fp32 -> bf16, round to nearest even (gfx950's v_cvt_pk_bf16_f32)
__device__ __forceinline__ u16 f2bf(float f) { return __builtin_bit_cast(u16, (__bf16)f); }

// 8 bf16 <-> 8 floats
__device__ __forceinline__ void unpack8(uint4 v, float f[8]) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[2 * i] = __uint_as_float(w[i] << 16);
    f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}
__device__ __forceinline__ uint4 pack8(const float f[8]) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Batch-norm backward sums of one layer, formed by the kernel that produces
// that layer's output gradient dout: d = dout where the layer's ReLU passed
// (xhat * gamma + beta > 0, xhat = (z - mean) * rstd), s1[c] += sum d (the
// beta gradient), s2[c] += sum d * xhat (the gamma gradient).
struct BnGrad {
  const u16* z;  // [P][C] bf16 batch-norm input; nullptr: no sums
  const float* mr;
  const float* gamma;
  const float* beta;
  float* s1;
  float* s2;
  int32_t C;
};

// One thread's share of the sums: 8 consecutive channels
struct BnAcc8 {
  float mean[8], rstd[8], gm[8], bt[8], a1[8], a2[8];
  __device__ __forceinline__ void init(const BnGrad& b, int32_t c0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool ok = c0 + j < b.C;  // channels past C (a partial tile) never pass
      mean[j] = ok ? b.mr[c0 + j] : 0.f;
      rstd[j] = ok ? b.mr[b.C + c0 + j] : 0.f;
      gm[j] = ok ? b.gamma[c0 + j] : 0.f;
      bt[j] = ok ? b.beta[c0 + j] : 0.f;
      a1[j] = 0.f;
      a2[j] = 0.f;
    }
  }
  __device__ __forceinline__ void add(const uint4 zin, const uint4 din) {
    float fz[8], fd[8];
    unpack8(zin, fz);
    unpack8(din, fd);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float zh = (fz[j] - mean[j]) * rstd[j];
      const float d = zh * gm[j] + bt[j] > 0.f ? fd[j] : 0.f;
      a1[j] += d;
      a2[j] += d * zh;
    }
  }
  // Block-wide: threads t and t' hold the same channels iff t % G == t' % G;
  // thread t's channels are c_first + 8 * (t % G) + 0..7.  lds: 16 * 256
  // floats, free on entry.  One atomic per channel per block.  Every thread
  // of the block calls this.
  __device__ __forceinline__ void flush(const BnGrad& b, float* lds, int G, int32_t c_first) {
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      lds[j * 256 + t] = a1[j];
      lds[(8 + j) * 256 + t] = a2[j];
    }
    __syncthreads();
    for (int u = t; u < 8 * G; u += 256) {
      const int grp = u >> 3, j = u & 7;
      const int32_t c = c_first + 8 * grp + j;
      if (c >= b.C) continue;
      float e1 = 0.f, e2 = 0.f;
      for (int q = grp; q < 256; q += G) {
        e1 += lds[j * 256 + q];
        e2 += lds[(8 + j) * 256 + q];
      }
      atomicAdd(&b.s1[c], e1);
      atomicAdd(&b.s2[c], e2);
    }
  }
};

// A_IM2COL32: the im2col of A_IM2COL when c0 + c1 is a multiple of 32, so a
// 32-wide reduction step lies inside one tap: the tap and channel offset are
// block-uniform counters and each row's shifted address is one add.
enum AMode : int { A_ROWS = 0, A_IM2COL = 1, A_UPGATHER = 2, A_IM2COL32 = 3 };
// E_AFFRELU: inference epilogue, y = max(0, acc * scale[n] + shift[n]) (batch
// norm with running statistics folded into scale/shift, then ReLU)
// E_BNGRAD: bf16 store of an output gradient, with the batch-norm backward
// sums of the layer it belongs to (g.bn) formed on the way
enum EMode : int { E_STORE = 0, E_SPLIT = 1, E_UPSCATTER = 2, E_AFFRELU = 3, E_BNGRAD = 4 };

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
  const float* scale;  // AFFRELU: [N]
  const float* shift;  // AFFRELU: [N]
  BnGrad bn;           // STORE: batch-norm backward sums of y0 (bn.z nullable)
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

// Tile: WM x WN waves (4 in all), each wave 64 rows x 16*NJ columns, so
// BM = 64*WM and BN = 16*NJ*WN.  Narrow outputs (32 channels) stack the waves
// along M (4 x 1) so each im2col tile feeds twice the MFMA work.  A block
// walks M tiles blockIdx.x, blockIdx.x + gridDim.x, ... (the grid holds about
// one resident wave of blocks), so the batch-norm sums it adds up are
// reduced in LDS and reach global memory with one atomic per column per
// block instead of one per column per tile.
template <int AM, int EM, int WM, int WN, int NJ>
__global__ __launch_bounds__(kGT) void k_gemm_nt(GemmNT g) {
  constexpr int BM = 64 * WM, BN = 16 * NJ * WN;
  static_assert(WM * WN == 4, "four waves");
  // the operand buffers, and after a tile's last K step its bf16 output tile
  constexpr int AS_ELEMS = 2 * BM * kLdsRow, BS_ELEMS = 2 * BN * kLdsRow;
  constexpr int SO_ROW = BN + 8;  // u16 per staged output row (padded)
  constexpr int SM_ELEMS =
      AS_ELEMS + BS_ELEMS > BM * SO_ROW ? AS_ELEMS + BS_ELEMS : BM * SO_ROW;
  __shared__ __attribute__((aligned(16))) u16 smem[SM_ELEMS];
  u16(*As)[BM][kLdsRow] = reinterpret_cast<u16(*)[BM][kLdsRow]>(smem);
  u16(*Bs)[BN][kLdsRow] = reinterpret_cast<u16(*)[BN][kLdsRow]>(smem + AS_ELEMS);
  u16* const So = smem;
  __shared__ float red[WM][2][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int32_t n0 = blockIdx.y * BN;
  const int32_t mtiles = (g.M + BM - 1) / BM;
  constexpr int BCH = BN * 4;               // B chunks per step
  constexpr int BR = (BCH + kGT - 1) / kGT;  // B chunks per thread
  const int kq = tid & 3;
  const int nk = (g.K + kBK - 1) / kBK;

  float s1[NJ], s2[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) s1[j] = s2[j] = 0.f;
  constexpr int NQ = BM * (BN / 8) / kGT;  // 16-byte output chunks per thread per tile
  static_assert(NQ * kGT == BM * (BN / 8), "whole chunks per thread");
  BnAcc8 bacc;  // E_BNGRAD: this thread's 8 channels are n0 + 8 * (tid % (BN / 8))
  if constexpr (EM == E_BNGRAD) bacc.init(g.bn, n0 + 8 * (tid % (BN / 8)));

  for (int32_t mt = blockIdx.x; mt < mtiles; mt += gridDim.x) {
    const int32_t m0 = mt * BM;
    // this thread's A rows (WM of them) and chunk column
    int32_t am[WM], aimg[WM], ah[WM], aw[WM];
#pragma unroll
    for (int r = 0; r < WM; ++r) {
      am[r] = m0 + (tid >> 2) + 64 * r;
      const int32_t mm = min(am[r], g.M - 1);
      aimg[r] = mm / (g.H * g.W);
      const int32_t rem = mm - aimg[r] * g.H * g.W;
      ah[r] = rem / g.W;
      aw[r] = rem - ah[r] * g.W;
    }
    uint4 ra[WM], rb[BR];
    int32_t nth = 0, ntw = 0, ncc = 0;  // A_IM2COL32: tap row, column and channel of the next load
    auto gload = [&](int32_t k0) {
      if constexpr (AM == A_IM2COL32) {
        const int32_t ci = ncc + 8 * kq;
        const bool first = ci < g.c0;
        const u16* src = first ? g.a0 : g.a1;
        const int32_t ld = first ? g.c0 : g.c1, off = first ? ci : ci - g.c0;
        const int32_t dh = nth - 1, dw = ntw - 1;
#pragma unroll
        for (int r = 0; r < WM; ++r) {
          const int32_t hh = ah[r] + dh, ww = aw[r] + dw;
          ra[r] = make_uint4(0, 0, 0, 0);
          if (am[r] < g.M && (uint32_t)hh < (uint32_t)g.H && (uint32_t)ww < (uint32_t)g.W)
            ra[r] = *(const uint4*)(src + (int64_t)(am[r] + dh * g.W + dw) * ld + off);
        }
        ncc += kBK;
        if (ncc == g.c0 + g.c1) {
          ncc = 0;
          if (++ntw == 3) {
            ntw = 0;
            ++nth;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < WM; ++r)
          ra[r] = load_a<AM>(g, am[r], aimg[r], ah[r], aw[r], k0 + 8 * kq);
      }
#pragma unroll
      for (int r = 0; r < BR; ++r) {
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
      for (int r = 0; r < WM; ++r) *(uint4*)&As[buf][(tid >> 2) + 64 * r][8 * kq] = ra[r];
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        const int c = tid + kGT * r;
        if (c < BCH) *(uint4*)&Bs[buf][c >> 2][8 * (c & 3)] = rb[r];
      }
    };

    f32x4 acc[4][NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // both LDS buffers are free here: the previous tile's last step ended in a barrier
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload((kt + 1) * kBK);
      bf16x8 a[4], b[NJ];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = __builtin_bit_cast(
            bf16x8, *(const uint4*)&As[buf][wm * 64 + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        b[j] = __builtin_bit_cast(
            bf16x8, *(const uint4*)&Bs[buf][wn * 16 * NJ + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      if (kt + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }

    // epilogue: acc[i][j][t] is C[row][col], row = wave rows + 16i + 4*(lane/16) + t,
    // col = wave cols + 16j + lane%16.  The bf16 tile goes through LDS (the
    // operand buffers are free: the last K step ended in a barrier) so that
    // global stores are 16 bytes of 8 consecutive columns.
    uint4 zpre[EM == E_BNGRAD ? NQ : 1];  // E_BNGRAD: batch-norm input at the stored chunks
    if constexpr (EM == E_BNGRAD) {
#pragma unroll
      for (int r = 0; r < NQ; ++r) {
        const int q = tid + kGT * r;
        const int rl = q / (BN / 8), ch = q - rl * (BN / 8);
        const int32_t row = m0 + rl, col = n0 + 8 * ch;
        zpre[r] = make_uint4(0, 0, 0, 0);
        if (row < g.M && col < g.N) zpre[r] = *(const uint4*)(g.bn.z + (int64_t)row * g.N + col);
      }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int cl = wn * 16 * NJ + 16 * j + (lane & 15);
      const int32_t col = n0 + cl;
      const bool cok = col < g.N;
      float add = 0.f, mul = 1.f;
      if constexpr (EM == E_UPSCATTER) add = cok ? g.bias[col % g.up_cout] : 0.f;
      if constexpr (EM == E_AFFRELU) {
        mul = cok ? g.scale[col] : 0.f;
        add = cok ? g.shift[col] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rl = wm * 64 + 16 * i + 4 * (lane >> 4) + t;
          const float v = acc[i][j][t];
          float o = v;
          if constexpr (EM == E_STORE) {
            if (m0 + rl < g.M && cok) {
              s1[j] += v;
              s2[j] += v * v;
            }
          } else if constexpr (EM == E_AFFRELU) {
            const float z = v * mul + add;
            o = z > 0.f ? z : 0.f;
          } else if constexpr (EM == E_UPSCATTER) {
            o = v + add;
          }
          So[rl * SO_ROW + cl] = f2bf(o);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int q = tid + kGT * r;
      const int rl = q / (BN / 8), ch = q - rl * (BN / 8);
      const int32_t row = m0 + rl, col = n0 + 8 * ch;
      if (row >= g.M || col >= g.N) continue;
      const uint4 val = *(const uint4*)&So[rl * SO_ROW + 8 * ch];
      if constexpr (EM == E_UPSCATTER) {
        // column -> (quadrant qd, channel co); 8 columns stay in one quadrant
        const int32_t qd = col / g.up_cout, co = col - qd * g.up_cout;
        const int32_t img = row / (g.H * g.W), rem = row - img * g.H * g.W;
        const int32_t h = rem / g.W, w = rem - h * g.W;
        const int64_t pix =
            ((int64_t)img * 2 * g.H + 2 * h + (qd >> 1)) * (2 * g.W) + 2 * w + (qd & 1);
        *(uint4*)(g.y0 + pix * g.up_cout + co) = val;
      } else if constexpr (EM == E_SPLIT) {
        if (col < g.split)
          *(uint4*)(g.y0 + (int64_t)row * g.split + col) = val;
        else
          *(uint4*)(g.y1 + (int64_t)row * (g.N - g.split) + (col - g.split)) = val;
      } else {
        *(uint4*)(g.y0 + (int64_t)row * g.N + col) = val;
      }
      if constexpr (EM == E_BNGRAD) bacc.add(zpre[r], val);
    }
    __syncthreads();  // the staged tile overlaps the next tile's operand buffers
  }
  if constexpr (EM == E_BNGRAD) bacc.flush(g.bn, (float*)smem, BN / 8, n0);

  if constexpr (EM == E_STORE) {
    if (g.stats) {
      // lanes l and l ^ 16, l ^ 32 hold the same column: fold them, then the WM
      // waves that share columns meet in LDS
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        s1[j] += __shfl_xor(s1[j], 16);
        s1[j] += __shfl_xor(s1[j], 32);
        s2[j] += __shfl_xor(s2[j], 16);
        s2[j] += __shfl_xor(s2[j], 32);
        if (lane < 16) {
          red[wm][0][wn * 16 * NJ + 16 * j + lane] = s1[j];
          red[wm][1][wn * 16 * NJ + 16 * j + lane] = s2[j];
        }
      }
      __syncthreads();
      if (tid < BN && n0 + tid < g.N) {
        float t1 = 0.f, t2 = 0.f;
#pragma unroll
        for (int r = 0; r < WM; ++r) {
          t1 += red[r][0][tid];
          t2 += red[r][1][tid];
        }
        atomicAdd(&g.stats[n0 + tid], t1);
        atomicAdd(&g.stats[g.N + n0 + tid], t2);
      }
    }
  }
}

// ---- 3x3 convolution with the input tile staged in LDS --------------------------
//
// Implicit GEMM over an output tile of 8 x 32 pixels of one image (M = 256) and
// BN output channels.  For each 32-channel chunk of the input, the 10 x 34
// pixel input tile (one-pixel halo, zero outside the image) and the chunk's
// weights for all 9 taps are staged in LDS once; the 9 taps then read their
// shifted A operands straight from the staged tile, so every input value
// leaves L2 once per tile instead of once per tap.  Wave w owns output rows
// 2w, 2w+1 (four 16-pixel row blocks).  The next chunk's loads (or the next
// tile's first chunk) are in flight during the current chunk's MFMAs.  Requires c0 % 32 == 0, c1 % 32 == 0 and
// N % BN == 0; epilogues as k_gemm_nt (E_STORE with BN sums, E_SPLIT,
// E_AFFRELU).
constexpr int kCTH = 8, kCTW = 32;               // output tile rows, columns
constexpr int kCIH = kCTH + 2, kCIW = kCTW + 2;  // staged input tile
constexpr int kCPix = kCIH * kCIW;               // 340 staged pixels

template <int EM, int BN>
__global__ __launch_bounds__(kGT) void k_conv3_lds(GemmNT g) {
  constexpr int NJ = BN / 16;
  constexpr int IN_CH = kCPix * 4;               // 16-byte chunks of the input tile
  constexpr int IN_R = (IN_CH + kGT - 1) / kGT;
  constexpr int W_CH = 9 * BN * 4;               // 16-byte chunks of the weights
  constexpr int W_R = (W_CH + kGT - 1) / kGT;
  __shared__ u16 Si[kCIH][kCIW][kLdsRow];
  __shared__ u16 Sw[9][BN][kLdsRow];
  __shared__ float red[4][2][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t n0 = blockIdx.y * BN;
  const int32_t ct = g.c0 + g.c1;
  const int32_t nchunk = ct / kBK;
  const int32_t ntx = (g.W + kCTW - 1) / kCTW, nty = (g.H + kCTH - 1) / kCTH;
  const int32_t ntiles = g.M / (g.H * g.W) * nty * ntx;

  float s1[NJ], s2[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) s1[j] = s2[j] = 0.f;
  BnAcc8 bacc;  // E_BNGRAD: this thread's 8 channels are n0 + 8 * (tid % (BN / 8))
  if constexpr (EM == E_BNGRAD) bacc.init(g.bn, n0 + 8 * (tid % (BN / 8)));

  // The block's work is a sequence of (tile, chunk) items: tiles blockIdx.x,
  // blockIdx.x + gridDim.x, ..., each with nchunk input chunks.  The loads of
  // the next item (possibly the next tile's first chunk) are issued before
  // the current item's MFMAs.
  uint4 ri[IN_R], rw[W_R];
  // with a single chunk the weights are the same for every tile: staged once
  const bool w_once = nchunk == 1;
  auto gload = [&](int32_t tile, int32_t cc, bool with_w) {
    const int32_t img = tile / (nty * ntx), rem = tile - img * nty * ntx;
    const int32_t oy0 = (rem / ntx) * kCTH, ox0 = (rem % ntx) * kCTW;
    const bool first = cc < g.c0;
    const u16* src = first ? g.a0 : g.a1;
    const int32_t ld = first ? g.c0 : g.c1, off = first ? cc : cc - g.c0;
#pragma unroll
    for (int r = 0; r < IN_R; ++r) {
      const int q = tid + kGT * r;
      ri[r] = make_uint4(0, 0, 0, 0);
      if (q < IN_CH) {
        const int p = q >> 2, sub = q & 3;
        const int32_t y = oy0 - 1 + p / kCIW, x = ox0 - 1 + p % kCIW;
        if ((uint32_t)y < (uint32_t)g.H && (uint32_t)x < (uint32_t)g.W)
          ri[r] = *(const uint4*)(src + (((int64_t)img * g.H + y) * g.W + x) * ld + off +
                                  8 * sub);
      }
    }
    if (!with_w) return;
#pragma unroll
    for (int r = 0; r < W_R; ++r) {
      const int q = tid + kGT * r;
      rw[r] = make_uint4(0, 0, 0, 0);
      if (q < W_CH) {
        const int sub = q & 3, nt = q >> 2, tap = nt / BN, n = nt - tap * BN;
        rw[r] = *(const uint4*)(g.b + ((int64_t)(n0 + n) * 9 + tap) * ct + cc + 8 * sub);
      }
    }
  };
  auto lstore = [&](bool with_w) {
#pragma unroll
    for (int r = 0; r < IN_R; ++r) {
      const int q = tid + kGT * r;
      if (q < IN_CH) {
        const int p = q >> 2;
        *(uint4*)&Si[p / kCIW][p % kCIW][8 * (q & 3)] = ri[r];
      }
    }
    if (!with_w) return;
#pragma unroll
    for (int r = 0; r < W_R; ++r) {
      const int q = tid + kGT * r;
      if (q < W_CH) {
        const int nt = q >> 2, tap = nt / BN;
        *(uint4*)&Sw[tap][nt - tap * BN][8 * (q & 3)] = rw[r];
      }
    }
  };

  if (blockIdx.x < ntiles) gload(blockIdx.x, 0, true);
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int32_t img = t / (nty * ntx), rem = t - img * nty * ntx;
    const int32_t oy0 = (rem / ntx) * kCTH, ox0 = (rem % ntx) * kCTW;

    f32x4 acc[4][NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int32_t c = 0; c < nchunk; ++c) {
      const bool first_item = t == (int32_t)blockIdx.x && c == 0;
      __syncthreads();  // the previous item's LDS reads are done
      lstore(!w_once || first_item);
      __syncthreads();
      if (c + 1 < nchunk)
        gload(t, (c + 1) * kBK, true);
      else if (t + gridDim.x < ntiles)
        gload(t + gridDim.x, 0, !w_once);
      // Tap (dy, dx) multiplies output row block i (row 2*wave + i/2, column
      // half i%2) with staged row 2*wave + i/2 + dy shifted by dx.  Per column
      // shift dx, the four staged rows u = i/2 + dy = 0..3 of each column half
      // are read once and serve the taps dy = u - i/2: 8 A and 3*NJ weight
      // reads per 12*NJ MFMAs.
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        bf16x8 b[3][NJ];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            b[dy][j] = __builtin_bit_cast(
                bf16x8, *(const uint4*)&Sw[dy * 3 + dx][16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bf16x8 a = __builtin_bit_cast(
                bf16x8,
                *(const uint4*)&Si[2 * wave + u][16 * h + (lane & 15) + dx][8 * (lane >> 4)]);
#pragma unroll
            for (int ih = 0; ih < 2; ++ih) {  // output row 2*wave + ih uses tap dy = u - ih
              const int dy = u - ih;
              if (dy < 0 || dy > 2) continue;
#pragma unroll
              for (int j = 0; j < NJ; ++j)
                acc[2 * ih + h][j] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[dy][j], acc[2 * ih + h][j], 0, 0, 0);
            }
          }
      }
    }

    // epilogue: acc[i][j][t] is output pixel (oy0 + 2*wave + i/2, ox0 + 16*(i%2) +
    // 4*(lane/16) + t), channel n0 + 16j + lane%16.  The bf16 tile goes through LDS
    // (the staged input is no longer needed) so that global stores are 16 bytes.
    u16* const So = &Si[0][0][0];  // [256 pixels][kLdsRow]
    uint4 zpre[BN / 8];            // E_BNGRAD: the batch-norm input at the stored chunks
    if constexpr (EM == E_BNGRAD) {
#pragma unroll
      for (int r = 0; r < BN / 8; ++r) {
        const int q = tid + kGT * r;
        const int pl = q / (BN / 8), sub = q % (BN / 8);
        const int32_t oy = oy0 + pl / kCTW, ox = ox0 + pl % kCTW;
        zpre[r] = make_uint4(0, 0, 0, 0);
        if (oy < g.H && ox < g.W)
          zpre[r] = *(const uint4*)(g.bn.z + (((int64_t)img * g.H + oy) * g.W + ox) * g.N +
                                    n0 + 8 * sub);
      }
    }
    __syncthreads();                // every wave's MFMA reads of Si are done
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int32_t col = n0 + 16 * j + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t oy = oy0 + 2 * wave + (i >> 1);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int32_t ox = ox0 + 16 * (i & 1) + 4 * (lane >> 4) + tt;
          const int pl = 32 * (2 * wave + (i >> 1)) + 16 * (i & 1) + 4 * (lane >> 4) + tt;
          const float v = acc[i][j][tt];
          float o = v;
          if constexpr (EM == E_STORE) {
            if (oy < g.H && ox < g.W) {
              s1[j] += v;
              s2[j] += v * v;
            }
          } else if constexpr (EM == E_AFFRELU) {
            const float z = v * g.scale[col] + g.shift[col];
            o = z > 0.f ? z : 0.f;
          }
          So[pl * kLdsRow + 16 * j + (lane & 15)] = f2bf(o);
        }
      }
    }
    __syncthreads();
    // 256 pixels x BN channels as 16-byte chunks of 8 channels
#pragma unroll
    for (int r = 0; r < BN / 8; ++r) {
      const int q = tid + kGT * r;
      const int pl = q / (BN / 8), sub = q % (BN / 8);
      const int32_t oy = oy0 + pl / kCTW, ox = ox0 + pl % kCTW;
      if (oy >= g.H || ox >= g.W) continue;
      const int64_t row = ((int64_t)img * g.H + oy) * g.W + ox;
      const uint4 val = *(const uint4*)&So[pl * kLdsRow + 8 * sub];
      const int32_t col = n0 + 8 * sub;
      if constexpr (EM == E_SPLIT) {
        if (col < g.split)
          *(uint4*)(g.y0 + row * g.split + col) = val;
        else
          *(uint4*)(g.y1 + row * (g.N - g.split) + (col - g.split)) = val;
      } else {
        *(uint4*)(g.y0 + row * g.N + col) = val;
      }
      if constexpr (EM == E_BNGRAD) bacc.add(zpre[r], val);
    }
  }
  if constexpr (EM == E_BNGRAD) {
    __syncthreads();  // the last tile's reads of So are done
    bacc.flush(g.bn, (float*)&Si[0][0][0], BN / 8, n0);
  }

  if constexpr (EM == E_STORE) {
    if (g.stats) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        s1[j] += __shfl_xor(s1[j], 16);
        s1[j] += __shfl_xor(s1[j], 32);
        s2[j] += __shfl_xor(s2[j], 16);
        s2[j] += __shfl_xor(s2[j], 32);
        if (lane < 16) {
          red[wave][0][16 * j + lane] = s1[j];
          red[wave][1][16 * j + lane] = s2[j];
        }
      }
      __syncthreads();
      if (tid < BN) {
        const float t1 = red[0][0][tid] + red[1][0][tid] + red[2][0][tid] + red[3][0][tid];
        const float t2 = red[0][1][tid] + red[1][1][tid] + red[2][1][tid] + red[3][1][tid];
        atomicAdd(&g.stats[n0 + tid], t1);
        atomicAdd(&g.stats[g.N + n0 + tid], t2);
      }
    }
  }
}

// ---- 3x3 convolution of an 8-channel input ---------------------------------------
//
// The first layer (the 3 bands padded to 8 channels): K = 9 taps x 8 channels,
// so each 32-wide MFMA reduction step takes 4 taps (lane group q reads the 8
// channels of tap 4s + q, shifted in the staged tile; taps past 8 are zero).
// The 72 x BN weights stay in registers for the block's life (3 steps x NJ
// fragments); per 8 x 32 output tile only the 10 x 34 input pixels (16 bytes
// each) are staged in LDS, and the next tile's are loaded during the current
// tile's MFMAs.  Wave w owns output rows 2w, 2w+1.  Requires c0 == 8, c1 == 0
// and N % BN == 0; epilogues E_STORE (with BN sums) and E_AFFRELU.
template <int EM, int BN>
__global__ __launch_bounds__(kGT) void k_conv3_c8(GemmNT g) {
  constexpr int NJ = BN / 16;
  constexpr int IN_R = (kCPix + kGT - 1) / kGT;
  __shared__ __attribute__((aligned(16))) u16 Si[kCPix * 8];
  __shared__ __attribute__((aligned(16))) u16 So[kCTH * kCTW * kLdsRow];
  __shared__ float red[4][2][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q4 = lane >> 4;
  const int32_t n0 = blockIdx.y * BN;
  const int32_t ntx = (g.W + kCTW - 1) / kCTW, nty = (g.H + kCTH - 1) / kCTH;
  const int32_t ntiles = g.M / (g.H * g.W) * nty * ntx;

  // weights: step s, fragment j, lane (n = 16j + lane % 16, tap 4s + lane / 16)
  bf16x8 wb[3][NJ];
#pragma unroll
  for (int st = 0; st < 3; ++st)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int tap = 4 * st + q4;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (tap < 9) v = *(const uint4*)(g.b + ((int64_t)(n0 + 16 * j + (lane & 15)) * 9 + tap) * 8);
      wb[st][j] = __builtin_bit_cast(bf16x8, v);
    }
  // staged-pixel offset of this lane's tap per step (taps past 8: none)
  int toff[3];
#pragma unroll
  for (int st = 0; st < 3; ++st) {
    const int tap = 4 * st + q4;
    toff[st] = tap < 9 ? (tap / 3) * kCIW + tap % 3 : -1;
  }

  float s1[NJ], s2[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) s1[j] = s2[j] = 0.f;

  uint4 ri[IN_R];
  auto gload = [&](int32_t tile) {
    const int32_t img = tile / (nty * ntx), rem = tile - img * nty * ntx;
    const int32_t oy0 = (rem / ntx) * kCTH, ox0 = (rem % ntx) * kCTW;
#pragma unroll
    for (int r = 0; r < IN_R; ++r) {
      const int p = tid + kGT * r;
      ri[r] = make_uint4(0, 0, 0, 0);
      if (p < kCPix) {
        const int32_t y = oy0 - 1 + p / kCIW, x = ox0 - 1 + p % kCIW;
        if ((uint32_t)y < (uint32_t)g.H && (uint32_t)x < (uint32_t)g.W)
          ri[r] = *(const uint4*)(g.a0 + (((int64_t)img * g.H + y) * g.W + x) * 8);
      }
    }
  };

  if ((int32_t)blockIdx.x < ntiles) gload(blockIdx.x);
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int32_t img = t / (nty * ntx), rem = t - img * nty * ntx;
    const int32_t oy0 = (rem / ntx) * kCTH, ox0 = (rem % ntx) * kCTW;
    __syncthreads();  // the previous tile's reads of Si and So are done
#pragma unroll
    for (int r = 0; r < IN_R; ++r) {
      const int p = tid + kGT * r;
      if (p < kCPix) *(uint4*)&Si[p * 8] = ri[r];
    }
    __syncthreads();
    if (t + (int32_t)gridDim.x < ntiles) gload(t + gridDim.x);

    f32x4 acc[4][NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < 3; ++st)
#pragma unroll
      for (int i = 0; i < 4; ++i) {  // output row 2*wave + i/2, column half i%2
        uint4 v = make_uint4(0, 0, 0, 0);
        if (toff[st] >= 0)
          v = *(const uint4*)&Si[((2 * wave + (i >> 1)) * kCIW + 16 * (i & 1) + (lane & 15) +
                                  toff[st]) * 8];
        const bf16x8 a = __builtin_bit_cast(bf16x8, v);
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb[st][j], acc[i][j], 0, 0, 0);
      }

    // epilogue: acc[i][j][tt] is output pixel (oy0 + 2*wave + i/2, ox0 + 16*(i%2) +
    // 4*(lane/16) + tt), channel n0 + 16j + lane%16; staged in LDS for 16-byte stores
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int32_t col = n0 + 16 * j + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t oy = oy0 + 2 * wave + (i >> 1);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int32_t ox = ox0 + 16 * (i & 1) + 4 * (lane >> 4) + tt;
          const int pl = 32 * (2 * wave + (i >> 1)) + 16 * (i & 1) + 4 * (lane >> 4) + tt;
          const float v = acc[i][j][tt];
          float o = v;
          if constexpr (EM == E_STORE) {
            if (oy < g.H && ox < g.W) {
              s1[j] += v;
              s2[j] += v * v;
            }
          } else if constexpr (EM == E_AFFRELU) {
            const float z = v * g.scale[col] + g.shift[col];
            o = z > 0.f ? z : 0.f;
          }
          So[pl * kLdsRow + 16 * j + (lane & 15)] = f2bf(o);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < BN / 8; ++r) {
      const int q = tid + kGT * r;
      const int pl = q / (BN / 8), sub = q % (BN / 8);
      const int32_t oy = oy0 + pl / kCTW, ox = ox0 + pl % kCTW;
      if (oy >= g.H || ox >= g.W) continue;
      *(uint4*)(g.y0 + (((int64_t)img * g.H + oy) * g.W + ox) * g.N + n0 + 8 * sub) =
          *(const uint4*)&So[pl * kLdsRow + 8 * sub];
    }
  }

  if constexpr (EM == E_STORE) {
    if (g.stats) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        s1[j] += __shfl_xor(s1[j], 16);
        s1[j] += __shfl_xor(s1[j], 32);
        s2[j] += __shfl_xor(s2[j], 16);
        s2[j] += __shfl_xor(s2[j], 32);
        if (lane < 16) {
          red[wave][0][16 * j + lane] = s1[j];
          red[wave][1][16 * j + lane] = s2[j];
        }
      }
      __syncthreads();
      if (tid < BN) {
        const float t1 = red[0][0][tid] + red[1][0][tid] + red[2][0][tid] + red[3][0][tid];
        const float t2 = red[0][1][tid] + red[1][1][tid] + red[2][1][tid] + red[3][1][tid];
        atomicAdd(&g.stats[n0 + tid], t1);
        atomicAdd(&g.stats[g.N + n0 + tid], t2);
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
  float* rowsum;        // nullable: += sum_p A[p][m] at index m % rowsum_mod
  int32_t rowsum_mod;
};

// ---- 3x3 weight gradient with the input tile staged in LDS ------------------------
//
// dw[n][tap][ci] += sum_p dy[p][n] * x[p + shift(tap)][ci] over 8 x 32-pixel
// tiles.  A block owns 32 output channels (n0) and a 32-channel input chunk (cc)
// and walks pixel tiles blockIdx.x, blockIdx.x + gridDim.x, ...  Per tile, dy^T
// (32 channels x 256 pixels) and x^T of the 10 x 34 halo tile are staged in
// LDS (x^T halo rows kXHalo elements apart); the K steps are the tile's 8 rows
// of 32 pixels.  A tap shifted by dx columns needs its 8-pixel MFMA operand
// dx elements past a 16-byte boundary: it is built in registers from the
// aligned 16 bytes and the next 4 (byte-align for dx = 1, a dword shift for
// dx = 2).  Each wave owns one of the 2 x 2 output blocks of 16 x 16 for all 9
// taps.  Staging stores pixel pairs as 4-byte words.  The next tile's loads
// are in flight during the current tile's MFMAs; partial sums reach dw with one
// fp32 atomic per element per block.  Requires cout, c0 and c1 divisible by 32.
constexpr int kXHalo = 40;                    // u16 per staged x^T halo row (34 used)
constexpr int kXRow = kCIH * kXHalo + 24;     // u16 per staged x^T channel row (padded)
constexpr int kARow = kCTH * kCTW + 8;  // u16 per staged dy^T channel row (padded)

// Column of a staged channel row, swizzled: channel rows 16-31 exchange
// 64-byte halves of each 128 bytes.  The staging writes of a wave cover 64
// bytes of four channel rows 8 apart, and rows 16 apart meet in the same LDS
// banks with the padded stride; the MFMA reads (16 bytes of 16 consecutive
// rows, all on one side of row 16) are unchanged in bank spread.
__device__ __forceinline__ int swz(int row, int col) { return col ^ (((row >> 4) & 1) << 5); }

__global__ __launch_bounds__(kGT) void k_wgrad3_lds(GemmTN g) {
  constexpr int A_SLOTS = (kCTH * kCTW / 2) * 4;   // pixel pairs x 4 channel groups = 512
  constexpr int A_R = A_SLOTS / kGT;               // 2
  constexpr int X_SLOTS = kCIH * (kCIW / 2) * 4;   // 10 rows x 17 pairs x 4 groups = 680
  constexpr int X_R = (X_SLOTS + kGT - 1) / kGT;   // 3
  __shared__ u16 Sa[32][kARow];
  __shared__ u16 Sx[32][kXRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t ct = g.c0 + g.c1;
  const int32_t nblk_ci = ct / 32;
  const int32_t n0 = (blockIdx.y / nblk_ci) * 32, cc = (blockIdx.y % nblk_ci) * 32;
  const int32_t cout = g.M;
  const int32_t ntx = (g.W + kCTW - 1) / kCTW, nty = (g.H + kCTH - 1) / kCTH;
  const int32_t ntiles = (int32_t)(g.P / ((int64_t)g.H * g.W)) * nty * ntx;
  const bool first = cc < g.c0;
  const u16* xsrc = first ? g.b0 : g.b1;
  const int32_t xld = first ? g.c0 : g.c1, xoff = first ? cc : cc - g.c0;

  uint4 ra[A_R][2], rx[X_R][2];
  auto gload = [&](int32_t tile) {
    const int32_t img = tile / (nty * ntx), rem = tile - img * nty * ntx;
    const int32_t oy0 = (rem / ntx) * kCTH, ox0 = (rem % ntx) * kCTW;
#pragma unroll
    for (int r = 0; r < A_R; ++r) {
      const int q = tid + kGT * r;  // pair (q >> 2) of the tile, channel group q & 3
      const int pr = q >> 2, grp = q & 3;
      const int32_t y = oy0 + pr / (kCTW / 2), x = ox0 + 2 * (pr % (kCTW / 2));
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        ra[r][e] = make_uint4(0, 0, 0, 0);
        if (y < g.H && x + e < g.W)
          ra[r][e] = *(const uint4*)(g.a + (((int64_t)img * g.H + y) * g.W + x + e) * cout + n0 +
                                     8 * grp);
      }
    }
#pragma unroll
    for (int r = 0; r < X_R; ++r) {
      const int q = tid + kGT * r;
      const int pr = q >> 2, grp = q & 3;
      const int32_t y = oy0 - 1 + pr / (kCIW / 2), x = ox0 - 1 + 2 * (pr % (kCIW / 2));
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        rx[r][e] = make_uint4(0, 0, 0, 0);
        if (q < X_SLOTS && (uint32_t)y < (uint32_t)g.H && (uint32_t)(x + e) < (uint32_t)g.W)
          rx[r][e] = *(const uint4*)(xsrc + (((int64_t)img * g.H + y) * g.W + x + e) * xld + xoff +
                                     8 * grp);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int r = 0; r < A_R; ++r) {
      const int q = tid + kGT * r;
      const int pr = q >> 2, grp = q & 3;
      const int col = 2 * pr;  // tile pixel index (row-major, 32 per row)
      const uint32_t w0[4] = {ra[r][0].x, ra[r][0].y, ra[r][0].z, ra[r][0].w};
      const uint32_t w1[4] = {ra[r][1].x, ra[r][1].y, ra[r][1].z, ra[r][1].w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ra0 = 8 * grp + 2 * t;
        *(uint32_t*)&Sa[ra0][swz(ra0, col)] = (w0[t] & 0xffffu) | (w1[t] << 16);
        *(uint32_t*)&Sa[ra0 + 1][swz(ra0 + 1, col)] = (w0[t] >> 16) | (w1[t] & 0xffff0000u);
      }
    }
#pragma unroll
    for (int r = 0; r < X_R; ++r) {
      const int q = tid + kGT * r;
      if (q >= X_SLOTS) continue;
      const int pr = q >> 2, grp = q & 3;
      const int hr = pr / (kCIW / 2), hp = pr % (kCIW / 2);  // halo row, pair (cols 2hp, 2hp+1)
      const uint32_t w0[4] = {rx[r][0].x, rx[r][0].y, rx[r][0].z, rx[r][0].w};
      const uint32_t w1[4] = {rx[r][1].x, rx[r][1].y, rx[r][1].z, rx[r][1].w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ch0 = 8 * grp + 2 * t, c0 = hr * kXHalo + 2 * hp;
        *(uint32_t*)&Sx[ch0][c0] = (w0[t] & 0xffffu) | (w1[t] << 16);          // channel 2t
        *(uint32_t*)&Sx[ch0 + 1][c0] = (w0[t] >> 16) | (w1[t] & 0xffff0000u);  // channel 2t+1
      }
    }
  };

  // this wave's output blocks: b = wave + 4k, b = tap*4 + mi*2 + nj
  f32x4 acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (blockIdx.x < ntiles) gload(blockIdx.x);
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    __syncthreads();  // the previous tile's LDS reads are done
    lstore();
    __syncthreads();
    if (t + gridDim.x < ntiles) gload(t + gridDim.x);
    // The wave's block (mi, nj) for all 9 taps: tap (dy, dx) pairs output row
    // r of dy^T with halo row r + dy of the dx-shifted x^T.  Walking the halo
    // rows s, each x^T fragment (s, dx) serves the three taps dy = 0..2 with
    // output rows s - dy, and each dy^T row fragment stays in registers for
    // the three halo rows that use it: 18 LDS reads per 72 MFMAs.
    {
      const int mi = (wave >> 1) & 1, nj = wave & 1;
      const int ar = 16 * mi + (lane & 15), xr = 16 * nj + (lane & 15);
      bf16x8 arow[kCTH];
#pragma unroll
      for (int s = 0; s < kCIH; ++s) {
        if (s < kCTH)
          arow[s] = __builtin_bit_cast(
              bf16x8, *(const uint4*)&Sa[ar][swz(ar, kCTW * s + 8 * (lane >> 4))]);
        // halo columns 8q .. 8q+9 of halo row s (q = lane / 16): the operands of
        // the three column shifts
        const int xc = kXHalo * s + 8 * (lane >> 4);
        const uint4 c0 = *(const uint4*)&Sx[xr][xc];
        const uint32_t c1 = *(const uint32_t*)&Sx[xr][xc + 8];
        bf16x8 bx[3];
        bx[0] = __builtin_bit_cast(bf16x8, c0);
        bx[1] = __builtin_bit_cast(
            bf16x8, make_uint4(__builtin_amdgcn_alignbyte(c0.y, c0.x, 2),
                               __builtin_amdgcn_alignbyte(c0.z, c0.y, 2),
                               __builtin_amdgcn_alignbyte(c0.w, c0.z, 2),
                               __builtin_amdgcn_alignbyte(c1, c0.w, 2)));
        bx[2] = __builtin_bit_cast(bf16x8, make_uint4(c0.y, c0.z, c0.w, c1));
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int r = s - dy;
          if (r < 0 || r >= kCTH) continue;
#pragma unroll
          for (int dx = 0; dx < 3; ++dx)
            acc[dy * 3 + dx] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(arow[r], bx[dx], acc[dy * 3 + dx], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int b = wave + 4 * k, tap = b >> 2, mi = (b >> 1) & 1, nj = b & 1;
    const int32_t ci = cc + 16 * nj + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int32_t n = n0 + 16 * mi + 4 * (lane >> 4) + e;
      atomicAdd(&g.c[((int64_t)n * 9 + tap) * ct + ci], acc[k][e]);
    }
  }
}

// Pixel coordinates of a running pixel index, advanced without divisions.
struct Pix {
  int32_t img, h, w;
};

__device__ __forceinline__ Pix pix_of(int64_t p, int32_t H, int32_t W) {
  const int64_t hw = (int64_t)H * W;
  Pix r;
  r.img = (int32_t)(p / hw);
  const int32_t rem = (int32_t)(p - (int64_t)r.img * hw);
  r.h = rem / W;
  r.w = rem - r.h * W;
  return r;
}

__device__ __forceinline__ void pix_adv(Pix& q, int32_t d, int32_t H, int32_t W) {
  q.w += d;
  while (q.w >= W) {
    q.w -= W;
    if (++q.h == H) {
      q.h = 0;
      ++q.img;
    }
  }
}

// Where one staged 16-byte chunk (8 consecutive m or n at one pixel) comes
// from; fixed for the whole pixel walk of a block.
struct TnSrc {
  const u16* base;
  int32_t ld, off;  // element = base[pixel * ld + off]
  int32_t dh, dw;   // pixel shift: 3x3 tap (-1..1) or, when up, 2x2 sub-pixel (0..1)
  bool ok, up;
};

__device__ __forceinline__ TnSrc tn_src(const GemmTN& g, int mode, bool is_a, int32_t idx,
                                        bool ok) {
  TnSrc s{};
  s.ok = ok;
  s.up = mode == T_UPGATHER;
  if (mode == T_PLAIN) {
    s.base = is_a ? g.a : g.b0;
    s.ld = is_a ? g.M : g.N;
    s.off = idx;
  } else if (mode == T_IM2COL) {
    const int32_t ct = g.c0 + g.c1;
    const int32_t tap = idx / ct, ci = idx - tap * ct;
    s.dh = tap / 3 - 1;
    s.dw = tap % 3 - 1;
    if (ci < g.c0) {
      s.base = g.b0;
      s.ld = g.c0;
      s.off = ci;
    } else {
      s.base = g.b1;
      s.ld = g.c1;
      s.off = ci - g.c0;
    }
  } else {  // m = (i*2 + j)*cout + co over dy [img][2H][2W][cout]
    const int32_t cout = g.M / 4;
    const int32_t q = idx / cout;
    s.base = g.a;
    s.ld = cout;
    s.off = idx - q * cout;
    s.dh = q >> 1;
    s.dw = q & 1;
  }
  return s;
}

__device__ __forceinline__ uint4 tn_load(const TnSrc& s, const Pix& q, int32_t H, int32_t W,
                                         bool in_range) {
  const uint4 zero = make_uint4(0, 0, 0, 0);
  if (!s.ok || !in_range) return zero;
  int64_t pix;
  if (s.up) {
    pix = ((int64_t)q.img * 2 * H + 2 * q.h + s.dh) * (2 * W) + 2 * q.w + s.dw;
  } else {
    const int32_t hh = q.h + s.dh, ww = q.w + s.dw;
    if (hh < 0 || hh >= H || ww < 0 || ww >= W) return zero;
    pix = ((int64_t)q.img * H + hh) * W + ww;
  }
  return *(const uint4*)(s.base + pix * s.ld + s.off);
}

// C[m][n] += sum_p A[p][m] B[p][n] over this block's pixel range.  A^T and B^T
// are staged in one LDS array S (rows 0..BM-1 = m, BM.. = n; kTnK pixels per
// row, double-buffered), so one stage feeds two MFMA K steps.  Staging slot c
// (0 .. 4*(BM+BN)) covers LDS rows 8*(c/32) .. +7 at the pixel pair 2*(c%32),
// 2*(c%32)+1: two 16-byte loads, then eight 4-byte LDS writes of (pixel 2j,
// pixel 2j+1) pairs, consecutive across the 32 lanes of a row group.  With
// g.rowsum set, the blocks of the first N tile also add up A's rows over their
// pixels (the bias gradient of the up-convolution: rowsum[m % cout] for
// UPGATHER), one atomic per row per block.
constexpr int kTnK = 64;                  // pixels per stage
constexpr int kTnRow = kTnK + 8;          // u16 per staged row (padded)

template <int AM, int BMD, int MI, int NJ>
__global__ __launch_bounds__(kGT) void k_gemm_tn(GemmTN g) {
  constexpr int BM = 32 * MI, BN = 32 * NJ;
  constexpr int SLOTS = 4 * (BM + BN);
  constexpr int SR = (SLOTS + kGT - 1) / kGT;
  __shared__ u16 S[2][BM + BN][kTnRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int32_t m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int64_t p_begin = (int64_t)blockIdx.z * g.p_per_split;
  const int64_t p_end = min(g.P, p_begin + g.p_per_split);
  const int pj = tid & 31;
  const bool sum_rows = g.rowsum != nullptr && blockIdx.y == 0 && wn == 0;

  TnSrc src[SR];
#pragma unroll
  for (int r = 0; r < SR; ++r) {
    const int c = tid + kGT * r;
    const int row = 8 * (c >> 5);
    if (c >= SLOTS) {
      src[r] = TnSrc{};
    } else if (row < BM) {
      src[r] = tn_src(g, AM, true, m0 + row, m0 + row < g.M);
    } else {
      src[r] = tn_src(g, BMD, false, n0 + row - BM, n0 + row - BM < g.N);
    }
  }

  // Two stages of loads are in flight: while stage k is multiplied out of
  // LDS, stage k+1 waits in registers for its LDS store and stage k+2 is
  // being fetched.  qn is the pixel of the next stage to fetch.
  Pix qn = pix_of(p_begin + 2 * pj, g.H, g.W);
  uint4 ra[SR][2], rb[SR][2];
  auto gload = [&](uint4 (&rv)[SR][2], int64_t p0) {
    Pix q1 = qn;
    pix_adv(q1, 1, g.H, g.W);
    const int64_t pa = p0 + 2 * pj;
#pragma unroll
    for (int r = 0; r < SR; ++r) {
      rv[r][0] = tn_load(src[r], qn, g.H, g.W, pa < p_end);
      rv[r][1] = tn_load(src[r], q1, g.H, g.W, pa + 1 < p_end);
    }
    pix_adv(qn, kTnK, g.H, g.W);
  };
  auto lstore = [&](int buf, const uint4 (&rv)[SR][2]) {
#pragma unroll
    for (int r = 0; r < SR; ++r) {
      const int c = tid + kGT * r;
      if (c >= SLOTS) continue;
      const int row = 8 * (c >> 5);
      const uint32_t w0[4] = {rv[r][0].x, rv[r][0].y, rv[r][0].z, rv[r][0].w};
      const uint32_t w1[4] = {rv[r][1].x, rv[r][1].y, rv[r][1].z, rv[r][1].w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        *(uint32_t*)&S[buf][row + 2 * t][2 * pj] = (w0[t] & 0xffffu) | (w1[t] << 16);
        *(uint32_t*)&S[buf][row + 2 * t + 1][2 * pj] = (w0[t] >> 16) | (w1[t] & 0xffff0000u);
      }
    }
  };

  f32x4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float rsum[MI];
#pragma unroll
  for (int i = 0; i < MI; ++i) rsum[i] = 0.f;

  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < kTnK / kBK; ++kk) {
      bf16x8 a[MI], b[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        a[i] = __builtin_bit_cast(
            bf16x8, *(const uint4*)&S[buf][wm * (BM / 2) + 16 * i + (lane & 15)]
                                     [kBK * kk + 8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        b[j] = __builtin_bit_cast(
            bf16x8, *(const uint4*)&S[buf][BM + wn * (BN / 2) + 16 * j + (lane & 15)]
                                     [kBK * kk + 8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      if (sum_rows) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int e = 0; e < 8; ++e) rsum[i] += (float)a[i][e];
      }
    }
  };

  gload(ra, p_begin);
  if (p_begin + kTnK < p_end) gload(rb, p_begin + kTnK);
  lstore(0, ra);
  __syncthreads();
  // stages alternate between the register sets ra and rb: the loop body is
  // written out for two stages
  for (int64_t p0 = p_begin; p0 < p_end; p0 += 2 * kTnK) {
    // stage p0 is in LDS buffer 0, stage p0 + K in rb
    if (p0 + 2 * kTnK < p_end) gload(ra, p0 + 2 * kTnK);
    compute(0);
    if (p0 + kTnK >= p_end) break;
    lstore(1, rb);
    __syncthreads();
    // stage p0 + K is in LDS buffer 1, stage p0 + 2K in ra
    if (p0 + 3 * kTnK < p_end) gload(rb, p0 + 3 * kTnK);
    compute(1);
    if (p0 + 2 * kTnK >= p_end) break;
    lstore(0, ra);
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
  if (sum_rows) {
    // lanes l, l ^ 16, l ^ 32, l ^ 48 summed the same row over different pixels
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      float v = rsum[i];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      const int32_t row = m0 + wm * (BM / 2) + 16 * i + lane;
      if (lane < 16 && row < g.M) atomicAdd(&g.rowsum[row % g.rowsum_mod], v);
    }
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


// BN + ReLU, 8 channels per thread (C % 8 == 0).  Each block first turns the
// per-channel sums into (mean, rstd) for all C channels in LDS, in double;
// block 0 also writes them to mr for the backward pass.
// The element-wise BN kernels walk [P][C] in 16-byte groups of 8 channels
// with a grid stride of gridDim.x * 256 groups.  C divides 256, so the stride
// (a multiple of 2048 elements) is a multiple of C and each thread keeps the
// same 8 channels: their parameters are loaded once, and two groups are in
// flight per iteration.
__global__ void k_bn_relu(const u16* z, const float* stats, int64_t count, float eps,
                          const float* gamma, const float* beta, u16* out, float* mr, int64_t n,
                          int32_t C) {
  __shared__ float smean[256], srstd[256];
  const int t = threadIdx.x;
  if (t < C) {
    const double mean = (double)stats[t] / (double)count;
    double var = (double)stats[C + t] / (double)count - mean * mean;
    if (var < 0) var = 0;
    smean[t] = (float)mean;
    srstd[t] = (float)(1.0 / sqrt(var + (double)eps));
    if (blockIdx.x == 0) {
      mr[t] = smean[t];
      mr[C + t] = srstd[t];
    }
  }
  __syncthreads();
  const int64_t n8 = n / 8, i0 = (int64_t)blockIdx.x * blockDim.x + t;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t c0 = (int32_t)((i0 * 8) % C);
  float mean[8], rstd[8], gm[8], bt[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    mean[j] = smean[c0 + j];
    rstd[j] = srstd[c0 + j];
    gm[j] = gamma[c0 + j];
    bt[j] = beta[c0 + j];
  }
  auto one = [&](const uint4 zin) {
    float f[8];
    unpack8(zin, f);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = (f[j] - mean[j]) * rstd[j] * gm[j] + bt[j];
      f[j] = v > 0.f ? v : 0.f;
    }
    return pack8(f);
  };
  int64_t i = i0;
  for (; i + stride < n8; i += 2 * stride) {
    const uint4 a = ((const uint4*)z)[i], b = ((const uint4*)z)[i + stride];
    ((uint4*)out)[i] = one(a);
    ((uint4*)out)[i + stride] = one(b);
  }
  if (i < n8) ((uint4*)out)[i] = one(((const uint4*)z)[i]);
}

// Per-channel sums over [P][C] for the BN backward: thread t owns channel
// group g = t % (C/8) (8 channels, 16-byte loads) and rows t / (C/8) + k *
// (256 / (C/8)) of its block's row range, four rows (eight loads) in flight;
// C <= 256, 256 % (C/8) == 0.  Partial sums meet in LDS, then one atomic per
// channel per block into r1 (sum of the masked gradient) and r2 (its sum
// against the normalised input).
__global__ void k_bn_bwd_reduce(const u16* dout, const u16* z, const float* mr,
                                const float* gamma, const float* beta, float* r1, float* r2,
                                int64_t P, int32_t C) {
  __shared__ float s1[256 * 8], s2[256 * 8];
  const int t = threadIdx.x, G = C / 8;
  const int g = t % G, r0 = t / G, rstep = 256 / G;
  const int c0 = 8 * g;
  float a1[8], a2[8], mean[8], rstd[8], gm[8], bt[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a1[j] = 0.f;
    a2[j] = 0.f;
    mean[j] = mr[c0 + j];
    rstd[j] = mr[C + c0 + j];
    gm[j] = gamma[c0 + j];
    bt[j] = beta[c0 + j];
  }
  auto add = [&](const uint4 zin, const uint4 din) {
    float fz[8], fd[8];
    unpack8(zin, fz);
    unpack8(din, fd);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float zh = (fz[j] - mean[j]) * rstd[j];
      const float d = zh * gm[j] + bt[j] > 0.f ? fd[j] : 0.f;
      a1[j] += d;
      a2[j] += d * zh;
    }
  };
  const int64_t rows_per_block = (P + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(P, rb + rows_per_block);
  const uint4* zv = (const uint4*)z;
  const uint4* dv = (const uint4*)dout;
  int64_t p = rb + r0;
  for (; p + 3 * rstep < re; p += 4 * rstep) {
    uint4 zz[4], dd[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      zz[u] = zv[(p + u * rstep) * G + g];
      dd[u] = dv[(p + u * rstep) * G + g];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) add(zz[u], dd[u]);
  }
  for (; p < re; p += rstep) add(zv[p * G + g], dv[p * G + g]);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    s1[j * 256 + t] = a1[j];
    s2[j * 256 + t] = a2[j];
  }
  __syncthreads();
  if (t < C) {
    const int gg = t / 8, j = t % 8;
    float b1 = 0.f, b2 = 0.f;
    for (int k = gg; k < 256; k += G) {
      b1 += s1[j * 256 + k];
      b2 += s2[j * 256 + k];
    }
    atomicAdd(&r1[t], b1);
    atomicAdd(&r2[t], b2);
  }
}

__global__ void k_bn_bwd_apply(const u16* dout, const u16* z, const float* mr, const float* gamma,
                               const float* beta, const float* red1, const float* red2, u16* dz,
                               int64_t n, int32_t C, float inv_count) {
  const int64_t n8 = n / 8, i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t c0 = (int32_t)((i0 * 8) % C);  // fixed per thread (see k_bn_relu)
  float mean[8], rstd[8], gm[8], bt[8], r1[8], r2[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    mean[j] = mr[c0 + j];
    rstd[j] = mr[C + c0 + j];
    gm[j] = gamma[c0 + j];
    bt[j] = beta[c0 + j];
    r1[j] = red1[c0 + j];
    r2[j] = red2[c0 + j];
  }
  auto one = [&](const uint4 zin, const uint4 din) {
    float fz[8], fd[8], o[8];
    unpack8(zin, fz);
    unpack8(din, fd);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float zh = (fz[j] - mean[j]) * rstd[j];
      const float d = zh * gm[j] + bt[j] > 0.f ? fd[j] : 0.f;
      o[j] = gm[j] * rstd[j] * (d - (r1[j] + zh * r2[j]) * inv_count);
    }
    return pack8(o);
  };
  int64_t i = i0;
  for (; i + stride < n8; i += 2 * stride) {
    const uint4 za = ((const uint4*)z)[i], da = ((const uint4*)dout)[i];
    const uint4 zb = ((const uint4*)z)[i + stride], db = ((const uint4*)dout)[i + stride];
    ((uint4*)dz)[i] = one(za, da);
    ((uint4*)dz)[i + stride] = one(zb, db);
  }
  if (i < n8) ((uint4*)dz)[i] = one(((const uint4*)z)[i], ((const uint4*)dout)[i]);
}

__global__ void k_affine_relu(const u16* z, const float* scale, const float* shift, u16* out,
                              int64_t n, int32_t C) {
  const int64_t n8 = n / 8, i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t c0 = (int32_t)((i0 * 8) % C);  // fixed per thread (see k_bn_relu)
  float sc[8], sh[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    sc[j] = scale[c0 + j];
    sh[j] = shift[c0 + j];
  }
  for (int64_t i = i0; i < n8; i += stride) {
    float f[8];
    unpack8(((const uint4*)z)[i], f);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = f[j] * sc[j] + sh[j];
      f[j] = v > 0.f ? v : 0.f;
    }
    ((uint4*)out)[i] = pack8(f);
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

// dst0[i] += src[i], dst1[i] += src[n + i] for i < n (n <= 256)
__global__ void k_add_pair(float* dst0, float* dst1, const float* src, int32_t n) {
  const int i = threadIdx.x;
  if (i < n) {
    dst0[i] += src[i];
    dst1[i] += src[n + i];
  }
}

// 2x2 max pool, 8 channels per thread
__global__ void k_maxpool(const u16* x, u16* y, uint8_t* idx, int32_t N, int32_t H, int32_t W,
                          int32_t C) {
  const int32_t Ho = H / 2, Wo = W / 2, G = C / 8;
  const int64_t n = (int64_t)N * Ho * Wo * G;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = (int32_t)(i % G);
    int64_t r = i / G;
    const int32_t wo = (int32_t)(r % Wo);
    r /= Wo;
    const int32_t ho = (int32_t)(r % Ho);
    const int32_t img = (int32_t)(r / Ho);
    float best[8], v[8];
    uint32_t bi[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      unpack8(*(const uint4*)(x + (((int64_t)img * H + 2 * ho + (k >> 1)) * W + 2 * wo + (k & 1)) *
                                      C + 8 * g),
              v);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k == 0 || v[j] > best[j]) {
          best[j] = v[j];
          bi[j] = (uint32_t)k;
        }
    }
    ((uint4*)y)[i] = pack8(best);
    uint2 packed;
    packed.x = bi[0] | (bi[1] << 8) | (bi[2] << 16) | (bi[3] << 24);
    packed.y = bi[4] | (bi[5] << 8) | (bi[6] << 16) | (bi[7] << 24);
    ((uint2*)idx)[i] = packed;
  }
}

// dx = the pooled gradient routed to each window's winner, plus dadd (the
// gradient of the same tensor from its other consumer, nullable; may be dx)
// (with bn.z set, 256 % (C/8) == 0: each thread keeps one channel group)
__global__ void k_maxpool_bwd(const u16* dy, const uint8_t* idx, const u16* dadd, u16* dx,
                              int32_t N, int32_t H, int32_t W, int32_t C, BnGrad bn) {
  __shared__ float lds[16 * 256];
  const int32_t G = C / 8;
  const int64_t n = (int64_t)N * H * W * G;
  const bool with_bn = bn.z != nullptr;
  BnAcc8 bacc;
  if (with_bn) bacc.init(bn, 8 * (int32_t)(threadIdx.x % G));
  // two chunks per iteration, every load issued before any use
  struct In {
    uint4 d, e, z;
    uint2 ix;
    uint32_t k;
  };
  const bool small = n <= INT32_MAX;  // 32-bit index arithmetic
  auto fetch = [&](int64_t i, In& v) {
    int32_t g, w, h, img;
    if (small) {
      const uint32_t i32 = (uint32_t)i, r0 = i32 / (uint32_t)G, r1 = r0 / (uint32_t)W;
      g = (int32_t)(i32 - r0 * (uint32_t)G);
      w = (int32_t)(r0 - r1 * (uint32_t)W);
      img = (int32_t)(r1 / (uint32_t)H);
      h = (int32_t)(r1 - (uint32_t)img * (uint32_t)H);
    } else {
      g = (int32_t)(i % G);
      int64_t r = i / G;
      w = (int32_t)(r % W);
      r /= W;
      h = (int32_t)(r % H);
      img = (int32_t)(r / H);
    }
    const int64_t o = (((int64_t)img * (H / 2) + h / 2) * (W / 2) + w / 2) * G + g;
    v.k = (uint32_t)((h & 1) * 2 + (w & 1));
    v.d = ((const uint4*)dy)[o];
    v.ix = ((const uint2*)idx)[o];
    if (dadd) v.e = ((const uint4*)dadd)[i];
    if (with_bn) v.z = ((const uint4*)bn.z)[i];
  };
  auto finish = [&](int64_t i, const In& v) {
    const uint32_t dw[4] = {v.d.x, v.d.y, v.d.z, v.d.w};
    uint32_t out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t word = q < 2 ? v.ix.x : v.ix.y;
      const uint32_t lo = (word >> (16 * (q & 1))) & 0xffu, hi = (word >> (16 * (q & 1) + 8)) & 0xffu;
      out[q] = (lo == v.k ? (dw[q] & 0xffffu) : 0u) | (hi == v.k ? (dw[q] & 0xffff0000u) : 0u);
    }
    uint4 res = make_uint4(out[0], out[1], out[2], out[3]);
    if (dadd) {
      float f[8], e[8];
      unpack8(res, f);
      unpack8(v.e, e);
#pragma unroll
      for (int j = 0; j < 8; ++j) f[j] += e[j];
      res = pack8(f);
    }
    ((uint4*)dx)[i] = res;
    if (with_bn) bacc.add(v.z, res);
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 2 * stride) {
    In va, vb;
    fetch(i, va);
    const bool two = i + stride < n;
    if (two) fetch(i + stride, vb);
    finish(i, va);
    if (two) finish(i + stride, vb);
  }
  if (with_bn) bacc.flush(bn, lds, G, 0);
}

// Logits of pixel p under the 1x1 head: l_k = b_k + sum_c x[p][c] w[k][c].
__device__ __forceinline__ void head_logits(const u16* x, const float* w, const float* b,
                                            int64_t p, int32_t C, float l[3]) {
  l[0] = b[0];
  l[1] = b[1];
  l[2] = b[2];
  for (int32_t c0 = 0; c0 < C; c0 += 8) {
    float f[8];
    unpack8(*(const uint4*)(x + p * C + c0), f);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      l[0] += f[j] * w[c0 + j];
      l[1] += f[j] * w[C + c0 + j];
      l[2] += f[j] * w[2 * C + c0 + j];
    }
  }
}

// Softmax cross-entropy of one pixel with label y: returns scale * -log
// softmax(l)[y]; dl (nullable) = (softmax(l) - onehot(y)) * scale.
__device__ __forceinline__ float xent_px(const float l[3], int y, float scale, float* dl) {
  const float mx = fmaxf(l[0], fmaxf(l[1], l[2]));
  const float ea = expf(l[0] - mx), eb = expf(l[1] - mx), ec = expf(l[2] - mx);
  const float s = ea + eb + ec;
  const float ly = y == 0 ? l[0] : (y == 1 ? l[1] : l[2]);
  if (dl) {
    const float inv = 1.f / s;
    dl[0] = (ea * inv - (y == 0)) * scale;
    dl[1] = (eb * inv - (y == 1)) * scale;
    dl[2] = (ec * inv - (y == 2)) * scale;
  }
  return (logf(s) + mx - ly) * scale;
}

// Block sum of v into *out with one atomic per block (blockDim.x == 256).
__device__ __forceinline__ void block_add(float v, float* out) {
  __shared__ float part[256];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, part[0]);
}

__global__ void k_head(const u16* x, const float* w, const float* b, float* logits, int64_t P,
                       int32_t C) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    float l[3];
    head_logits(x, w, b, p, C, l);
    logits[3 * p] = l[0];
    logits[3 * p + 1] = l[1];
    logits[3 * p + 2] = l[2];
  }
}

__global__ void k_softmax_xent(const float* logits, const uint8_t* labels, float* loss,
                               float* dlogits, float scale, int64_t P) {
  float acc = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float l[3] = {logits[3 * p], logits[3 * p + 1], logits[3 * p + 2]};
    float dl[3];
    acc += xent_px(l, labels[p], scale, dlogits ? dl : nullptr);
    if (dlogits) {
      dlogits[3 * p] = dl[0];
      dlogits[3 * p + 1] = dl[1];
      dlogits[3 * p + 2] = dl[2];
    }
  }
  block_add(acc, loss);
}

// The head and the loss in one pass: the logits stay in registers (written
// out only when asked for), saving their write and re-read.
__global__ void k_head_xent(const u16* x, const float* w, const float* b, const uint8_t* labels,
                            float* loss, float* dlogits, float* logits, float scale, int64_t P,
                            int32_t C) {
  float acc = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    float l[3], dl[3];
    head_logits(x, w, b, p, C, l);
    acc += xent_px(l, labels[p], scale, dl);
    dlogits[3 * p] = dl[0];
    dlogits[3 * p + 1] = dl[1];
    dlogits[3 * p + 2] = dl[2];
    if (logits) {
      logits[3 * p] = l[0];
      logits[3 * p + 1] = l[1];
      logits[3 * p + 2] = l[2];
    }
  }
  block_add(acc, loss);
}

// Head backward in one pass over x: thread t owns channel group g = t % (C/8)
// (8 channels) and rows t / (C/8) + k * (256 / (C/8)) of its block's row range
// (256 % (C/8) == 0).  Per row it writes dx = dlogits w for its 8 channels and
// adds dlogits (x) x into 24 partial sums (and dlogits into 3 for the bias);
// partial sums meet in LDS, then one atomic per output per block.
__global__ __launch_bounds__(256) void k_head_bwd(const u16* x, const float* w, const float* dl, const float* dscale,
                           u16* dx, float* dw, float* db, int64_t P, int32_t C, BnGrad bn) {
  __shared__ float s[27][256];
  const int t = threadIdx.x, G = C / 8;
  const int g = t % G, r0 = t / G, rstep = 256 / G;
  const int c0 = 8 * g;
  float wk[3][8], a[3][8], bsum[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      wk[k][j] = w[k * C + c0 + j];
      a[k][j] = 0.f;
    }
  const float sc = dscale ? *dscale : 1.f;
  const bool with_bn = bn.z != nullptr;
  BnAcc8 bacc;
  if (with_bn) bacc.init(bn, c0);
  struct Row {
    uint4 x, z;
    float d0, d1, d2;
  };
  auto fetch = [&](int64_t p, Row& v) {
    v.x = ((const uint4*)x)[p * G + g];
    v.d0 = dl[3 * p];
    v.d1 = dl[3 * p + 1];
    v.d2 = dl[3 * p + 2];
    if (with_bn) v.z = ((const uint4*)bn.z)[p * G + g];
  };
  auto one = [&](int64_t p, const Row& v) {
    const float d0 = v.d0 * sc, d1 = v.d1 * sc, d2 = v.d2 * sc;
    float f[8], o[8];
    unpack8(v.x, f);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      o[j] = d0 * wk[0][j] + d1 * wk[1][j] + d2 * wk[2][j];
      a[0][j] += d0 * f[j];
      a[1][j] += d1 * f[j];
      a[2][j] += d2 * f[j];
    }
    bsum[0] += d0;
    bsum[1] += d1;
    bsum[2] += d2;
    const uint4 res = pack8(o);
    ((uint4*)dx)[p * G + g] = res;
    if (with_bn) bacc.add(v.z, res);
  };
  const int64_t rows_per_block = (P + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(P, rb + rows_per_block);
  int64_t p = rb + r0;
  for (; p + rstep < re; p += 2 * rstep) {
    Row a, b;
    fetch(p, a);
    fetch(p + rstep, b);
    one(p, a);
    one(p + rstep, b);
  }
  if (p < re) {
    Row a;
    fetch(p, a);
    one(p, a);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int j = 0; j < 8; ++j) s[k * 8 + j][t] = a[k][j];
    s[24 + k][t] = g == 0 ? bsum[k] : 0.f;
  }
  __syncthreads();
  for (int u = t; u < 3 * C + 3; u += 256) {
    if (u < 3 * C) {
      const int k = u / C, c = u - k * C, gg = c / 8, j = c % 8;
      float e = 0.f;
      for (int q = gg; q < 256; q += G) e += s[k * 8 + j][q];
      atomicAdd(&dw[k * C + c], e);
    } else {
      const int k = u - 3 * C;
      float e = 0.f;
      for (int q = 0; q < 256; q += G) e += s[24 + k][q];
      atomicAdd(&db[k], e);
    }
  }
  if (with_bn) {
    __syncthreads();  // the head sums' reads of s are done
    bacc.flush(bn, &s[0][0], G, 0);
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

// ---- multi-tensor kernels --------------------------------------------------------
//
// One launch covers a list of tensors passed by value in the kernel
// arguments (at most kMulti per launch).  Tensor i owns blocks blk0[i] ..
// blk0[i+1]-1, each block kPerBlock consecutive elements.
constexpr int kMulti = 64;
constexpr int kPerBlock = 4 * 256;

struct AdamList {
  sil_unet_adam_tensor t[kMulti];
  int32_t blk0[kMulti + 1];
  int32_t count;
};
struct PrepList {
  sil_unet_weight_prep t[kMulti];
  int32_t blk0[kMulti + 1];
  int32_t count;
};
constexpr int kMultiBn = 32;
struct BnList {
  sil_unet_bn_layer t[kMultiBn];
};

__device__ __forceinline__ int list_find(const int32_t* blk0, int count, int b) {
  int i = 0;
  while (i + 1 < count && blk0[i + 1] <= b) ++i;
  return i;
}

// Adam with the arithmetic of k_adam, on every tensor of the list
// The step number comes from the arguments or, when step_dev is set, from
// device memory, so that a launch recorded in a graph uses the value current
// when the graph is replayed; the bias corrections are formed on the device in
// both cases.
__global__ void k_adam_multi(AdamList L, float lr, float b1, float b2, float eps, int32_t step,
                             const int32_t* step_dev) {
  const float t = (float)(step_dev ? *step_dev : step);
  const float c1 = 1.f - powf(b1, t), c2 = 1.f - powf(b2, t);
  const int i = list_find(L.blk0, L.count, blockIdx.x);
  float* w = L.t[i].w;
  const float* g = L.t[i].g;
  float* m = L.t[i].m;
  float* v = L.t[i].v;
  const int64_t n = L.t[i].n;
  const int64_t base = (int64_t)(blockIdx.x - L.blk0[i]) * kPerBlock + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kPerBlock / 256; ++u) {
    const int64_t e = base + 256 * u;
    if (e >= n) break;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// bf16 copies of the weights, and their transposed forms for the input
// gradients.  Element e is the e-th element of both outputs: wb[e] =
// bf16(w[e]), and wt[e] gathers its source from w, so that every store is
// coalesced and the scattered reads hit the cache.
__global__ void k_counter_add(int32_t* c, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] += v;
}

__global__ void k_prep_weights(PrepList L) {
  const int i = list_find(L.blk0, L.count, blockIdx.x);
  const float* w = L.t[i].w;
  u16* wb = (u16*)L.t[i].wb;
  u16* wt = (u16*)L.t[i].wt;
  const int32_t kind = L.t[i].kind, cout = L.t[i].cout, cin = L.t[i].cin;
  const int64_t n = (int64_t)(kind == SIL_UNET_W_CONV3 ? 9 : 4) * cout * cin;
  const int64_t base = (int64_t)(blockIdx.x - L.blk0[i]) * kPerBlock + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kPerBlock / 256; ++u) {
    const int64_t e = base + 256 * u;
    if (e >= n) break;
    wb[e] = f2bf(w[e]);
    if (!wt) continue;
    // 32-bit index arithmetic: tensors hold at most 2^30 elements
    const int32_t e32 = (int32_t)e, rest = e32 / cout, co = e32 - rest * cout;
    if (kind == SIL_UNET_W_CONV3) {
      // wt[ci][r][s][co] = w[co][2-r][2-s][ci]
      const int32_t ci = rest / 9, rs = rest - ci * 9;
      wt[e] = f2bf(w[(co * 9 + (8 - rs)) * cin + ci]);
    } else {
      // wt[ci][q][co] = w[q][co][ci]
      const int32_t ci = rest >> 2, q = rest & 3;
      wt[e] = f2bf(w[(q * cout + co) * cin + ci]);
    }
  }
}

// exponential moving average of the batch statistics, one block per layer
__global__ void k_bn_ema(BnList L, float mom, float eps) {
  const sil_unet_bn_layer& T = L.t[blockIdx.x];
  for (int c = threadIdx.x; c < T.C; c += blockDim.x) {
    const float mean = T.mr[c], rstd = T.mr[T.C + c];
    const float var = 1.f / (rstd * rstd) - eps;
    T.running_mean[c] = T.running_mean[c] * (1.f - mom) + mom * mean;
    T.running_var[c] = T.running_var[c] * (1.f - mom) + mom * var;
  }
}

// inference scale and shift from the running statistics, one block per layer
__global__ void k_bn_fold(BnList L, float eps) {
  const sil_unet_bn_layer& T = L.t[blockIdx.x];
  for (int c = threadIdx.x; c < T.C; c += blockDim.x) {
    const float sc = T.gamma[c] / sqrtf(T.running_var[c] + eps);
    T.scale[c] = sc;
    T.shift[c] = T.beta[c] - T.running_mean[c] * sc;
  }
}

// ---- host helpers ---------------------------------------------------------------

// Reductions that end in global atomics run at most this many blocks: atomics
// on one address serialise, so their count, not the bytes read, would bound them.
constexpr int kRedBlocks = 1024;
// The batch-norm backward sums add 2*C atomics per block onto only 2*C
// addresses: fewer, longer blocks measured faster there.
#ifndef SIL_BNRED_BLOCKS
#define SIL_BNRED_BLOCKS 256
#endif
constexpr int kBnRedBlocks = SIL_BNRED_BLOCKS;
// Pooling and head backward with the batch-norm sums: per-pixel work plus one
// atomic per channel per block.  512 blocks measured fastest (1024 queue twice
// the same-address atomics; 256 or 384 leave too few waves for the streaming).
constexpr int kGradRedBlocks = 512;
#ifndef SIL_BNRELU_BLOCKS
#define SIL_BNRELU_BLOCKS 2048
#endif

int grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

int done() { return hipGetLastError() == hipSuccess ? SIL_OK : SIL_EDEVICE; }

// Blocks of `kernel` (256 threads) that fit on the current device at once.
int resident_blocks(const void* kernel) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(dev, kernel);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kGT, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  const int n = per_cu * cus;
  cache[key] = n;
  return n;
}

template <int AM, int EM, int WM, int WN, int NJ>
void launch_nt_tile(const GemmNT& g, hipStream_t st) {
  constexpr int BM = 64 * WM, BN = 16 * NJ * WN;
  auto kern = k_gemm_nt<AM, EM, WM, WN, NJ>;
  const int gy = (g.N + BN - 1) / BN;
  const int mtiles = (g.M + BM - 1) / BM;
  const int cap = std::max(1, resident_blocks((const void*)kern) / gy);
  dim3 grid(std::min(mtiles, cap), gy);
  hipLaunchKernelGGL(kern, grid, dim3(kGT), 0, st, g);
}

template <int AM, int EM>
int launch_nt(const GemmNT& g, hipStream_t st) {
  (void)hipGetLastError();
  // (the 128-wide tile would hold the batch-norm sums' operands in too many registers)
  if (g.N % 128 == 0 && EM != E_BNGRAD)
    launch_nt_tile<AM, EM, 2, 2, 4>(g, st);
  else if (g.N % 64 == 0)
    launch_nt_tile<AM, EM, 2, 2, 2>(g, st);
  else  // narrow outputs: 256 x 32 tiles, waves stacked along M
    launch_nt_tile<AM, EM, 4, 1, 2>(g, st);
  return done();
}

// 3x3 convolutions whose channel counts allow it go through k_conv3_lds, or
// k_conv3_c8 for an 8-channel input.
bool conv_lds_ok(const GemmNT& g) { return g.c0 % kBK == 0 && g.c1 % kBK == 0 && g.N % 32 == 0; }
bool conv_c8_ok(const GemmNT& g) { return g.c0 == 8 && g.c1 == 0 && g.N % 32 == 0; }

template <int EM>
int launch_conv_c8(const GemmNT& g, hipStream_t st) {
  (void)hipGetLastError();
  const int32_t ntiles =
      g.M / (g.H * g.W) * ((g.H + kCTH - 1) / kCTH) * ((g.W + kCTW - 1) / kCTW);
  auto kern = k_conv3_c8<EM, 32>;
  const int gy = g.N / 32;
  const int cap = std::max(1, resident_blocks((const void*)kern) / gy);
  hipLaunchKernelGGL(kern, dim3(std::min(ntiles, cap), gy), dim3(kGT), 0, st, g);
  return done();
}

template <int EM>
int launch_conv_lds(const GemmNT& g, hipStream_t st) {
  (void)hipGetLastError();
  const int32_t ntiles =
      g.M / (g.H * g.W) * ((g.H + kCTH - 1) / kCTH) * ((g.W + kCTW - 1) / kCTW);
  // 32-channel output tiles: wider ones would need more registers than two
  // blocks per CU leave
  auto kern = k_conv3_lds<EM, 32>;
  const int gy = g.N / 32;
  const int cap = std::max(1, resident_blocks((const void*)kern) / gy);
  hipLaunchKernelGGL(kern, dim3(std::min(ntiles, cap), gy), dim3(kGT), 0, st, g);
  return done();
}

#ifndef SIL_TN_BLOCKS
#define SIL_TN_BLOCKS 1024
#endif
#ifndef SIL_TN_ATOMICS
#define SIL_TN_ATOMICS (1 << 22)
#endif
constexpr int64_t kTnBlocks = SIL_TN_BLOCKS, kTnAtomics = SIL_TN_ATOMICS;

// Weight-gradient tile (32*MI x 32*NJ): the widest N tile that divides N
// (192, 128, 96, 64), else 96 for N <= 96, else 32.
template <int AM, int BMD>
int launch_tn(GemmTN g, hipStream_t st) {
  (void)hipGetLastError();
  const int mi = g.M % 128 == 0 ? 4 : (g.M % 64 == 0 ? 2 : 1);
  int nj;
  if (mi == 4 && g.N % 128 == 0) nj = 4;
  else if (g.N % 192 == 0) nj = 6;
  else if (g.N % 128 == 0) nj = 4;
  else if (g.N % 96 == 0) nj = 3;
  else if (g.N % 64 == 0) nj = 2;
  else if (g.N <= 96) nj = 3;
  else nj = 1;
  const int bm = 32 * mi, bn = 32 * nj;
  const int64_t tiles = (int64_t)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  // Split the pixel reduction across workgroups: about kTnBlocks of them, but
  // every split adds one fp32 atomic per output element, and atomics on the
  // same addresses serialise, so the splits times M*N stay near kTnAtomics.
  int64_t splits = (kTnBlocks + tiles - 1) / tiles;
  splits = std::min(splits, std::max<int64_t>(1, kTnAtomics / ((int64_t)g.M * g.N)));
  const int64_t max_splits = (g.P + 255) / 256;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  g.p_per_split = ((g.P + splits - 1) / splits + kTnK - 1) / kTnK * kTnK;
  splits = (g.P + g.p_per_split - 1) / g.p_per_split;
  dim3 grid((g.M + bm - 1) / bm, (g.N + bn - 1) / bn, (unsigned)splits);
#define SIL_TN(MIv, NJv)                                                            \
  if (mi == MIv && nj == NJv) {                                                     \
    hipLaunchKernelGGL((k_gemm_tn<AM, BMD, MIv, NJv>), grid, dim3(kGT), 0, st, g); \
    return done();                                                                  \
  }
  SIL_TN(4, 4) SIL_TN(4, 6) SIL_TN(4, 3) SIL_TN(4, 2) SIL_TN(4, 1)
  SIL_TN(2, 6) SIL_TN(2, 4) SIL_TN(2, 3) SIL_TN(2, 2) SIL_TN(2, 1)
  SIL_TN(1, 6) SIL_TN(1, 4) SIL_TN(1, 3) SIL_TN(1, 2) SIL_TN(1, 1)
#undef SIL_TN
  return SIL_EINVAL;
}

bool ok_dims(int32_t N, int32_t H, int32_t W) { return N > 0 && H > 0 && W > 0; }

// The device form of a caller's batch-norm backward request (nullptr: none).
// False when the request is malformed or its channel count is not C.
bool bn_grad_of(const sil_unet_bn_grad* p, int32_t C, BnGrad* out) {
  *out = BnGrad{};
  if (!p) return true;
  if (!p->z || !p->mr || !p->gamma || !p->beta || !p->sum_d || !p->sum_dxhat || p->C != C ||
      C < 8 || C % 8 || 256 % (C / 8))
    return false;
  *out = BnGrad{(const u16*)p->z, p->mr, p->gamma, p->beta, p->sum_d, p->sum_dxhat, p->C};
  return true;
}

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
  if (conv_c8_ok(g)) return launch_conv_c8<E_STORE>(g, (hipStream_t)stream);
  if (conv_lds_ok(g)) return launch_conv_lds<E_STORE>(g, (hipStream_t)stream);
  if ((c0 + c1) % kBK == 0) return launch_nt<A_IM2COL32, E_STORE>(g, (hipStream_t)stream);
  return launch_nt<A_IM2COL, E_STORE>(g, (hipStream_t)stream);
}

int sil_unet_conv3x3_affine_relu(const void* x0, int32_t c0, const void* x1, int32_t c1,
                                 const void* w, const float* scale, const float* shift, void* y,
                                 int32_t N, int32_t H, int32_t W, int32_t cout, void* stream) {
  if (!x0 || !w || !y || !scale || !shift || (c1 > 0 && !x1) || !ok_dims(N, H, W))
    return SIL_EINVAL;
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
  g.scale = scale;
  g.shift = shift;
  if (conv_c8_ok(g)) return launch_conv_c8<E_AFFRELU>(g, (hipStream_t)stream);
  if (conv_lds_ok(g)) return launch_conv_lds<E_AFFRELU>(g, (hipStream_t)stream);
  if ((c0 + c1) % kBK == 0) return launch_nt<A_IM2COL32, E_AFFRELU>(g, (hipStream_t)stream);
  return launch_nt<A_IM2COL, E_AFFRELU>(g, (hipStream_t)stream);
}

int sil_unet_conv3x3_dgrad(const void* dy, int32_t cout, const void* wt, void* dx0, int32_t c0,
                           void* dx1, int32_t c1, int32_t N, int32_t H, int32_t W,
                           const sil_unet_bn_grad* bn, void* stream) {
  if (!dy || !wt || !dx0 || (c1 > 0 && !dx1) || !ok_dims(N, H, W)) return SIL_EINVAL;
  if (cout <= 0 || cout % 8 || c0 <= 0 || c0 % 8 || c1 < 0 || c1 % 8) return SIL_EINVAL;
  if (bn && c1 > 0) return SIL_EINVAL;
  GemmNT g{};
  if (!bn_grad_of(bn, c0, &g.bn)) return SIL_EINVAL;
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
  hipStream_t st = (hipStream_t)stream;
  if (bn) {
    if (conv_lds_ok(g)) return launch_conv_lds<E_BNGRAD>(g, st);
    if (cout % kBK == 0) return launch_nt<A_IM2COL32, E_BNGRAD>(g, st);
    return launch_nt<A_IM2COL, E_BNGRAD>(g, st);
  }
  if (conv_lds_ok(g))
    return c1 > 0 ? launch_conv_lds<E_SPLIT>(g, st) : launch_conv_lds<E_STORE>(g, st);
  if (cout % kBK == 0)
    return c1 > 0 ? launch_nt<A_IM2COL32, E_SPLIT>(g, st) : launch_nt<A_IM2COL32, E_STORE>(g, st);
  return c1 > 0 ? launch_nt<A_IM2COL, E_SPLIT>(g, st) : launch_nt<A_IM2COL, E_STORE>(g, st);
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
  if (cout % 32 == 0 && c0 % 32 == 0 && c1 % 32 == 0) {
    (void)hipGetLastError();
    const int32_t ntiles = N * ((H + kCTH - 1) / kCTH) * ((W + kCTW - 1) / kCTW);
    const int gy = (cout / 32) * ((c0 + c1) / 32);
    const int gx = std::min(ntiles, std::max(1, resident_blocks((const void*)k_wgrad3_lds) / gy));
    hipLaunchKernelGGL(k_wgrad3_lds, dim3(gx, gy), dim3(kGT), 0, (hipStream_t)stream, g);
    return done();
  }
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
                          int32_t W, int32_t cin, int32_t cout, const sil_unet_bn_grad* bn,
                          void* stream) {
  if (!dy || !wt || !dx || !ok_dims(N, H, W) || cin <= 0 || cin % 8 || cout <= 0 || cout % 8)
    return SIL_EINVAL;
  GemmNT g{};
  if (!bn_grad_of(bn, cin, &g.bn)) return SIL_EINVAL;
  g.M = N * H * W;
  g.N = cin;
  g.K = 4 * cout;
  g.a0 = (const u16*)dy;
  g.c0 = cout;
  g.H = H;
  g.W = W;
  g.b = (const u16*)wt;
  g.y0 = (u16*)dx;
  if (bn) return launch_nt<A_UPGATHER, E_BNGRAD>(g, (hipStream_t)stream);
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
  g.rowsum = db;  // the bias gradient: the column sums of dy, formed in the same pass
  g.rowsum_mod = cout;
  return launch_tn<T_UPGATHER, T_PLAIN>(g, (hipStream_t)stream);
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
  if (!z || !stats || !gamma || !beta || !out || !mr || count <= 0 || P <= 0 || C < 8 ||
      C > 256 || 256 % C)
    return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = P * C;
  // every block derives (mean, rstd) itself: a capped grid keeps that cheap
  hipLaunchKernelGGL(k_bn_relu, dim3(std::min(grid_for(n / 8), SIL_BNRELU_BLOCKS)), dim3(256), 0,
                     (hipStream_t)stream, (const u16*)z, stats, count, eps, gamma, beta,
                     (u16*)out, mr, n, C);
  return done();
}

int sil_unet_affine_relu(const void* z, const float* scale, const float* shift, void* out,
                         int64_t P, int32_t C, void* stream) {
  if (!z || !scale || !shift || !out || P <= 0 || C < 8 || C > 256 || 256 % C) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = P * C;
  hipLaunchKernelGGL(k_affine_relu, dim3(grid_for(n / 8)), dim3(256), 0, (hipStream_t)stream,
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
  if (!dout || !z || !mr || !gamma || !beta || !dz || !dgamma || !dbeta || P <= 0 || C < 8 ||
      C > 256 || 256 % C)
    return SIL_EINVAL;
  (void)hipGetLastError();
  hipStream_t st = (hipStream_t)stream;
  // with scratch the sums are formed there and added to dbeta/dgamma at the
  // end; without it they are formed in dbeta/dgamma themselves (zero on entry)
  float* r1 = red ? red : dbeta;
  float* r2 = red ? red + C : dgamma;
  if (red) hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, st, red, (int64_t)2 * C, 0.f);
  hipLaunchKernelGGL(k_bn_bwd_reduce, dim3(std::min(grid_for(P * (C / 8) / 2048 + 1, 1), kBnRedBlocks)), dim3(256), 0, st,
                     (const u16*)dout, (const u16*)z, mr, gamma, beta, r1, r2, P, C);
  const int64_t n = P * C;
  hipLaunchKernelGGL(k_bn_bwd_apply, dim3(grid_for(n / 8)), dim3(256), 0, st, (const u16*)dout,
                     (const u16*)z, mr, gamma, beta, r1, r2, (u16*)dz, n, C, 1.f / (float)P);
  if (red)
    hipLaunchKernelGGL(k_add_pair, dim3(1), dim3(256), 0, st, dbeta, dgamma, red, C);
  return done();
}

int sil_unet_bn_relu_bwd_apply(const void* dout, const void* z, const float* mr,
                               const float* gamma, const float* beta, const float* sum_d,
                               const float* sum_dxhat, void* dz, int64_t P, int32_t C,
                               void* stream) {
  if (!dout || !z || !mr || !gamma || !beta || !sum_d || !sum_dxhat || !dz || P <= 0 || C < 8 ||
      C > 256 || 256 % C)
    return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = P * C;
  hipLaunchKernelGGL(k_bn_bwd_apply, dim3(grid_for(n / 8)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)dout, (const u16*)z, mr, gamma, beta, sum_d, sum_dxhat, (u16*)dz,
                     n, C, 1.f / (float)P);
  return done();
}

int sil_unet_maxpool(const void* x, void* y, uint8_t* idx, int32_t N, int32_t H, int32_t W,
                     int32_t C, void* stream) {
  if (!x || !y || !idx || !ok_dims(N, H, W) || H % 2 || W % 2 || C <= 0 || C % 8)
    return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)N * (H / 2) * (W / 2) * (C / 8);
  hipLaunchKernelGGL(k_maxpool, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)x, (u16*)y, idx, N, H, W, C);
  return done();
}

int sil_unet_maxpool_bwd(const void* dy, const uint8_t* idx, const void* dadd, void* dx,
                         int32_t N, int32_t H, int32_t W, int32_t C, const sil_unet_bn_grad* bn,
                         void* stream) {
  if (!dy || !idx || !dx || !ok_dims(N, H, W) || H % 2 || W % 2 || C <= 0 || C % 8)
    return SIL_EINVAL;
  BnGrad b;
  if (!bn_grad_of(bn, C, &b)) return SIL_EINVAL;
  (void)hipGetLastError();
  const int64_t n = (int64_t)N * H * W * (C / 8);
  // with the batch-norm sums: a bounded grid, so that each block's atomics cover more pixels
  const int grid = bn ? std::min(grid_for(n), kGradRedBlocks) : grid_for(n);
  hipLaunchKernelGGL(k_maxpool_bwd, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)dy, idx, (const u16*)dadd, (u16*)dx, N, H, W, C, b);
  return done();
}

int sil_unet_head(const void* x, const float* w, const float* b, float* logits, int64_t P,
                  int32_t C, void* stream) {
  if (!x || !w || !b || !logits || P <= 0 || C <= 0 || C % 8) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_head, dim3(grid_for(P)), dim3(256), 0, (hipStream_t)stream,
                     (const u16*)x, w, b, logits, P, C);
  return done();
}

int sil_unet_softmax_xent(const float* logits, const uint8_t* labels, float* loss,
                          float* dlogits, float scale, int64_t P, void* stream) {
  if (!logits || !labels || !loss || P <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_softmax_xent, dim3(std::min(grid_for(P), kRedBlocks)), dim3(256), 0, (hipStream_t)stream,
                     logits, labels, loss, dlogits, scale, P);
  return done();
}

int sil_unet_head_xent(const void* x, const float* w, const float* b, const uint8_t* labels,
                       float* loss, float* dlogits, float* logits, float scale, int64_t P,
                       int32_t C, void* stream) {
  if (!x || !w || !b || !labels || !loss || !dlogits || P <= 0 || C <= 0 || C % 8)
    return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_head_xent, dim3(std::min(grid_for(P), kRedBlocks)), dim3(256), 0,
                     (hipStream_t)stream, (const u16*)x, w, b, labels, loss, dlogits, logits, scale,
                     P, C);
  return done();
}

int sil_unet_head_bwd(const void* x, const float* w, const float* dlogits, const float* dscale,
                      void* dx, float* dw, float* db, int64_t P, int32_t C,
                      const sil_unet_bn_grad* bn, void* stream) {
  if (!x || !w || !dlogits || !dx || !dw || !db || P <= 0 || C < 8 || C > 256 || 256 % C)
    return SIL_EINVAL;
  BnGrad b;
  if (!bn_grad_of(bn, C, &b)) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_head_bwd, dim3(std::min(grid_for(P * (C / 8) / 2048 + 1, 1), kGradRedBlocks)),
                     dim3(256), 0, (hipStream_t)stream, (const u16*)x, w, dlogits, dscale,
                     (u16*)dx, dw, db, P, C, b);
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

int sil_unet_adam_multi(const sil_unet_adam_tensor* t, int32_t count, float lr, float beta1,
                        float beta2, float eps, int32_t step, const int32_t* step_dev,
                        void* stream) {
  if (!t || count <= 0 || (!step_dev && step < 1)) return SIL_EINVAL;
  int64_t blocks = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (!t[i].w || !t[i].g || !t[i].m || !t[i].v || t[i].n <= 0) return SIL_EINVAL;
    blocks += (t[i].n + kPerBlock - 1) / kPerBlock;
  }
  if (blocks > INT32_MAX) return SIL_EINVAL;
  (void)hipGetLastError();
  for (int32_t s0 = 0; s0 < count; s0 += kMulti) {
    AdamList L{};
    L.count = std::min(kMulti, count - s0);
    int32_t b = 0;
    for (int32_t i = 0; i < L.count; ++i) {
      L.t[i] = t[s0 + i];
      L.blk0[i] = b;
      b += (int32_t)((t[s0 + i].n + kPerBlock - 1) / kPerBlock);
    }
    L.blk0[L.count] = b;
    hipLaunchKernelGGL(k_adam_multi, dim3(b), dim3(256), 0, (hipStream_t)stream, L, lr, beta1,
                       beta2, eps, step, step_dev);
  }
  return done();
}

int sil_unet_counter_add(int32_t* counter, int32_t v, void* stream) {
  if (!counter) return SIL_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(64), 0, (hipStream_t)stream, counter, v);
  return done();
}

int sil_unet_prep_weights(const sil_unet_weight_prep* t, int32_t count, void* stream) {
  if (!t || count <= 0) return SIL_EINVAL;
  for (int32_t i = 0; i < count; ++i) {
    if (!t[i].w || !t[i].wb || t[i].cout <= 0 || t[i].cin <= 0) return SIL_EINVAL;
    if (t[i].kind != SIL_UNET_W_CONV3 && t[i].kind != SIL_UNET_W_UP2) return SIL_EINVAL;
    if ((int64_t)9 * t[i].cout * t[i].cin > ((int64_t)1 << 30)) return SIL_EINVAL;
  }
  (void)hipGetLastError();
  for (int32_t s0 = 0; s0 < count; s0 += kMulti) {
    PrepList L{};
    L.count = std::min(kMulti, count - s0);
    int32_t b = 0;
    for (int32_t i = 0; i < L.count; ++i) {
      const sil_unet_weight_prep& T = t[s0 + i];
      L.t[i] = T;
      L.blk0[i] = b;
      const int64_t n = (int64_t)(T.kind == SIL_UNET_W_CONV3 ? 9 : 4) * T.cout * T.cin;
      b += (int32_t)((n + kPerBlock - 1) / kPerBlock);
    }
    L.blk0[L.count] = b;
    hipLaunchKernelGGL(k_prep_weights, dim3(b), dim3(256), 0, (hipStream_t)stream, L);
  }
  return done();
}

int sil_unet_bn_ema(const sil_unet_bn_layer* l, int32_t count, float momentum, float eps,
                    void* stream) {
  if (!l || count <= 0) return SIL_EINVAL;
  for (int32_t i = 0; i < count; ++i)
    if (!l[i].mr || !l[i].running_mean || !l[i].running_var || l[i].C <= 0) return SIL_EINVAL;
  (void)hipGetLastError();
  for (int32_t s0 = 0; s0 < count; s0 += kMultiBn) {
    BnList L{};
    const int32_t k = std::min(kMultiBn, count - s0);
    for (int32_t i = 0; i < k; ++i) L.t[i] = l[s0 + i];
    hipLaunchKernelGGL(k_bn_ema, dim3(k), dim3(256), 0, (hipStream_t)stream, L, momentum, eps);
  }
  return done();
}

int sil_unet_bn_fold(const sil_unet_bn_layer* l, int32_t count, float eps, void* stream) {
  if (!l || count <= 0) return SIL_EINVAL;
  for (int32_t i = 0; i < count; ++i)
    if (!l[i].running_mean || !l[i].running_var || !l[i].gamma || !l[i].beta || !l[i].scale ||
        !l[i].shift || l[i].C <= 0)
      return SIL_EINVAL;
  (void)hipGetLastError();
  for (int32_t s0 = 0; s0 < count; s0 += kMultiBn) {
    BnList L{};
    const int32_t k = std::min(kMultiBn, count - s0);
    for (int32_t i = 0; i < k; ++i) L.t[i] = l[s0 + i];
    hipLaunchKernelGGL(k_bn_fold, dim3(k), dim3(256), 0, (hipStream_t)stream, L, eps);
  }
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
