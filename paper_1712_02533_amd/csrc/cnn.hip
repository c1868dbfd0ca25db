// Learned warm start: a 6-layer convolutional encoder-decoder (BF16 weights and activations,
// FP32 accumulation) that maps a pair of level-7 frames (2 x 128 x 128, normalised) to the
// level-7 displacement (2 x 128 x 128, in level-7 cells). Trained on this GPU by the kernels in
// this file (forward, backward, Adam) on pairs registered by the plain method.
//
// Network (3x3 convolutions, padding 1; ReLU after every layer but the last):
//   L1 2->64 stride 2 (64^2)   L2 64->128 stride 2 (32^2)   L3 128->256 stride 2 (16^2)
//   L4 [up2(L3), L2] 384->128 (32^2)   L5 [up2(L4), L1] 192->64 (64^2)
//   L6 [up2(L5), input] 66->2 (128^2, linear)
// Activations are NHWC. Weights are [Cout][Kp] with k = (dy * 3 + dx) * Cin + ci, Kp = 9 Cin
// rounded up to 32 (L1 to 64), padded with zeros. L2-L5 run as fused implicit-GEMM
// convolutions on MFMAs (v_mfma_f32_16x16x32_bf16); L1 (2 input channels) and L6 (2 output
// channels, its upsampled input folded into the weights) as direct FP32 kernels. The backward
// pass uses im2col + MFMA GEMMs for the weight gradients.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <ctype.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/pprs.h"

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

namespace {

const int kBlock = 256;

int grid1d(long long work, int cap = 16384) {
  long long g = (work + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// ------------------------------------------------------------------------------------------
// GEMM: C[m][n] = sum_k A(m,k) B(n,k), bf16 operands, fp32 result.
// A(m,k) = AK ? A[k * lda + m] : A[m * lda + k]; B(n,k) = BK ? B[k * ldb + n] : B[n * ldb + k].
// 64 x 64 tiles, 32-deep K steps, 4 wavefronts each owning a 32 x 32 quarter (2 x 2 MFMA).
// Requires M % 64 == 0, N % 64 == 0, (K range of a split) % 32 == 0, lda, ldb % 8 == 0.
// blockIdx.z selects a K split; split s writes C + s * split_stride.

template <bool AK, bool BK>
__global__ void __launch_bounds__(256) k_gemm(const bf16* __restrict__ A, int lda,
                                              const bf16* __restrict__ B, int ldb,
                                              float* __restrict__ C, int ldc, int K,
                                              int k_per_split, long long split_stride) {
  constexpr int PADK = 40;  // LDS row of 32 k plus 8 (keeps 16-byte alignment)
  __shared__ __attribute__((aligned(16))) bf16 sA[64 * PADK];
  __shared__ __attribute__((aligned(16))) bf16 sB[64 * PADK];
  int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
  int kb = blockIdx.z * k_per_split, ke = min(K, kb + k_per_split);
  int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    if (!AK) {
      int m = tid >> 2, kk = (tid & 3) * 8;
      *(uint4*)&sA[m * PADK + kk] = *(const uint4*)&A[(size_t)(m0 + m) * lda + k0 + kk];
    } else {
      int kk = tid >> 3, mm = (tid & 7) * 8;
      uint4 v = *(const uint4*)&A[(size_t)(k0 + kk) * lda + m0 + mm];
      const bf16* e = (const bf16*)&v;
#pragma unroll
      for (int i = 0; i < 8; ++i) sA[(mm + i) * PADK + kk] = e[i];
    }
    if (!BK) {
      int n = tid >> 2, kk = (tid & 3) * 8;
      *(uint4*)&sB[n * PADK + kk] = *(const uint4*)&B[(size_t)(n0 + n) * ldb + k0 + kk];
    } else {
      int kk = tid >> 3, nn = (tid & 7) * 8;
      uint4 v = *(const uint4*)&B[(size_t)(k0 + kk) * ldb + n0 + nn];
      const bf16* e = (const bf16*)&v;
#pragma unroll
      for (int i = 0; i < 8; ++i) sB[(nn + i) * PADK + kk] = e[i];
    }
    __syncthreads();
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *(const bf16x8*)&sA[(wm + i * 16 + (lane & 15)) * PADK + 8 * (lane >> 4)];
      b[i] = *(const bf16x8*)&sB[(wn + i * 16 + (lane & 15)) * PADK + 8 * (lane >> 4)];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  float* Co = C + (size_t)blockIdx.z * split_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        int col = n0 + wn + j * 16 + (lane & 15);
        Co[(size_t)row * ldc + col] = acc[i][j][r];
      }
}

// ------------------------------------------------------------------------------------------
// Fused 3x3 convolution (implicit GEMM) for layers whose input channels come in multiples of
// 64: out[m][n] = relu(bias[n] + sum_k A(m,k) W[n][k]) as bf16, with m = (b, oy, ox) and
// k = tap * Cin + c. A(m,k) is read straight from the NHWC input (no im2col copy): channels
// [0, C0) from src0 (at half resolution when UP, i.e. the nearest 2x upsampling of the decoder),
// channels [C0, C0 + C1) from src1 (the skip connection), zero outside the frame.
// Tiles: 128 pixels x BN output channels x 64-deep K chunks (one tap, one source per chunk),
// 4 wavefronts in 2 x 2, each owning 64 x BN/2 with 16x16x32 MFMAs; the next chunk is fetched
// into registers while the current one is multiplied out of LDS (double buffer).
// Requires C0 % 64 == 0, C1 % 64 == 0, BN | Cout, (B * Hout^2) % 128 == 0, Kp % 8 == 0.

constexpr int CV_BM = 128, CV_BK = 64, CV_LD = CV_BK + 8;

// DGRAD: the same product for a data gradient (input dZ, weights flipped and transposed):
// no bias or ReLU, FP32 output (`out` is then a float*).
// FOLD (with UP): the upsampled source is read at its own resolution. Output pixel
// (2Y + py, 2X + px) sees through its 3x3 taps only the 2 x 2 source pixels
// (Y - 1 + py + i, X - 1 + px + j), so the taps landing on one source pixel are summed into
// folded weights, one matrix per output parity (k_fold_weights: [4][Cout][Kp'], k' = (2i + j) C0
// + c for the upsampled part, then 4 C0 + tap C1 + c for the skip part, Kp' = 4 C0 + 9 C1).
// The pixels of a 128-row tile share one parity: m = ((parity B + b) (H/2) + Y) (H/2) + X.
template <int BN, bool UP, bool DGRAD = false, bool FOLD = false>
__global__ void __launch_bounds__(256, 2) k_conv_fwd(
    const bf16* __restrict__ src0, int C0, const bf16* __restrict__ src1, int C1, int Hin,
    int stride, const bf16* __restrict__ Wt, int Kp, const float* __restrict__ bias, int Cout,
    void* __restrict__ out_) {
  static_assert(!FOLD || (UP && !DGRAD), "folding is for the upsampling layers' forward");
  constexpr int WN = BN / 2;          // columns per wave
  constexpr int TN = WN / 16;         // 16-wide MFMA tiles per wave along n
  constexpr int B_PIECES = BN * 8 / 256;
  __shared__ __attribute__((aligned(16))) bf16 sA[2][CV_BM * CV_LD];
  __shared__ __attribute__((aligned(16))) bf16 sB[2][BN * CV_LD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int Cin = C0 + C1, Hout = Hin / stride;
  const int K = FOLD ? 4 * C0 + 9 * C1 : 9 * Cin, nchunks = K / CV_BK;
  const int n0 = blockIdx.y * BN;
  const int Hs0 = UP ? Hin / 2 : Hin;
  // FOLD: the tile's parity and its pixels' half-resolution coordinates
  const long long tiles_per_par = FOLD ? (long long)gridDim.x / 4 : 1;
  const int par = FOLD ? (int)(blockIdx.x / tiles_per_par) : 0;
  const int py = par >> 1, px = par & 1;
  const long long m0 = FOLD ? (blockIdx.x - par * tiles_per_par) * CV_BM
                            : (long long)blockIdx.x * CV_BM;
  if (FOLD) Wt += (size_t)par * Cout * Kp;
  // this thread's 4 A rows (pixels) and its 16-byte piece within a 64-wide chunk; FOLD: the
  // rows hold (b, Y, X) on the half-resolution grid
  const int a_piece = tid & 7;
  const int Hm = FOLD ? Hout / 2 : Hout;
  int a_b[4], a_oy[4], a_ox[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    long long m = m0 + (tid >> 3) + 32 * r;
    a_ox[r] = (int)(m % Hm);
    a_oy[r] = (int)((m / Hm) % Hm);
    a_b[r] = (int)(m / ((long long)Hm * Hm));
  }
  uint4 ra[4], rb[B_PIECES];
  auto fetch = [&](int chunk) {
    int k0 = chunk * CV_BK;
    bool first;
    int dy, dx, c0;
    if (FOLD) {
      first = k0 < 4 * C0;
      if (first) {
        int ij = k0 / C0;
        c0 = k0 - ij * C0;
        dy = (ij >> 1) - 1 + py;  // source row offset from Y
        dx = (ij & 1) - 1 + px;
      } else {
        int r = k0 - 4 * C0, tap = r / C1;
        c0 = C0 + (r - tap * C1);
        dy = tap / 3 - 1;
        dx = tap % 3 - 1;
      }
    } else {
      int tap = k0 / Cin;
      c0 = k0 - tap * Cin;
      dy = tap / 3 - 1;
      dx = tap % 3 - 1;
      first = c0 < C0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (FOLD && first) {
        int sy = a_oy[r] + dy, sx = a_ox[r] + dx;
        if (sy >= 0 && sy < Hs0 && sx >= 0 && sx < Hs0)
          v = *(const uint4*)(src0 + (((size_t)a_b[r] * Hs0 + sy) * Hs0 + sx) * C0 + c0 +
                              a_piece * 8);
      } else {
        int oy = FOLD ? 2 * a_oy[r] + py : a_oy[r], ox = FOLD ? 2 * a_ox[r] + px : a_ox[r];
        int iy = oy * stride + dy, ix = ox * stride + dx;
        if (iy >= 0 && iy < Hin && ix >= 0 && ix < Hin) {
          const bf16* p;
          if (first) {
            int sy = UP ? iy >> 1 : iy, sx = UP ? ix >> 1 : ix;
            p = src0 + (((size_t)a_b[r] * Hs0 + sy) * Hs0 + sx) * C0 + c0;
          } else {
            p = src1 + (((size_t)a_b[r] * Hin + iy) * Hin + ix) * C1 + (c0 - C0);
          }
          v = *(const uint4*)(p + a_piece * 8);
        }
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < B_PIECES; ++r) {
      int e = tid + 256 * r;
      int n = e >> 3, pc = e & 7;
      rb[r] = *(const uint4*)(Wt + (size_t)(n0 + n) * Kp + k0 + pc * 8);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      *(uint4*)&sA[buf][((tid >> 3) + 32 * r) * CV_LD + a_piece * 8] = ra[r];
#pragma unroll
    for (int r = 0; r < B_PIECES; ++r) {
      int e = tid + 256 * r;
      *(uint4*)&sB[buf][(e >> 3) * CV_LD + (e & 7) * 8] = rb[r];
    }
  };
  f32x4 acc[4][TN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * WN;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int chunk = 0; chunk < nchunks; ++chunk) {
    int buf = chunk & 1;
    if (chunk + 1 < nchunks) fetch(chunk + 1);
#pragma unroll
    for (int ks = 0; ks < CV_BK; ks += 32) {
      bf16x8 a[4], b[TN];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *(const bf16x8*)&sA[buf][(wm + 16 * i + (lane & 15)) * CV_LD + ks + 8 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = *(const bf16x8*)&sB[buf][(wn + 16 * j + (lane & 15)) * CV_LD + ks + 8 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (chunk + 1 < nchunks) stash(buf ^ 1);
    __syncthreads();
  }
  // epilogue: bias, ReLU, bf16 NHWC (forward) or the plain FP32 sums (data gradient)
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    int col = n0 + wn + 16 * j + (lane & 15);
    float bv = DGRAD ? 0.f : bias[col];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        long long row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (FOLD) {  // (b, Y, X) -> the output pixel (b, 2Y + py, 2X + px)
          long long X = row % Hm, t = row / Hm, Y = t % Hm, bb = t / Hm;
          row = (bb * Hout + 2 * Y + py) * Hout + 2 * X + px;
        }
        float v = acc[i][j][r] + bv;
        if (DGRAD)
          ((float*)out_)[row * Cout + col] = v;
        else
          ((bf16*)out_)[row * Cout + col] = (bf16)(v > 0.f ? v : 0.f);
      }
  }
}

// Folded weights of an upsampling layer (see k_conv_fwd's FOLD): Wf[par][co][k'] from the
// layer's W[co][k] (k = tap Cin + c): for the upsampled part the sum, over the taps landing on
// source offset (i, j) for parity par, of W[co][tap Cin + c] (FP32, taps in order, rounded to
// BF16 once); the skip part copied.
__global__ void k_fold_weights(const bf16* __restrict__ W, int Cout, int C0, int C1, int Kp,
                               bf16* __restrict__ Wf) {
  const int Cin = C0 + C1, Kf = 4 * C0 + 9 * C1;
  const long long total = 4LL * Cout * Kf;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e % Kf);
    const long long t = e / Kf;
    const int co = (int)(t % Cout), par = (int)(t / Cout);
    const bf16* w = W + (size_t)co * Kp;
    if (k < 4 * C0) {
      const int ij = k / C0, c = k - ij * C0, i = ij >> 1, j = ij & 1;
      const int py = par >> 1, px = par & 1;
      // tap rows (columns) landing on source row (column) offset i (j) for parity py (px)
      const int r0 = py == 0 ? (i == 0 ? 0 : 1) : (i == 0 ? 0 : 2);
      const int r1 = py == 0 ? (i == 0 ? 0 : 2) : (i == 0 ? 1 : 2);
      const int c0 = px == 0 ? (j == 0 ? 0 : 1) : (j == 0 ? 0 : 2);
      const int c1 = px == 0 ? (j == 0 ? 0 : 2) : (j == 0 ? 1 : 2);
      float acc = 0.f;
      for (int ty = r0; ty <= r1; ++ty)
        for (int tx = c0; tx <= c1; ++tx) acc += (float)w[(ty * 3 + tx) * Cin + c];
      Wf[e] = (bf16)acc;
    } else {
      const int r = k - 4 * C0, tap = r / C1, c = r - tap * C1;
      Wf[e] = w[tap * Cin + C0 + c];
    }
  }
}

// Weights of a stride-1 3x3 layer for its data gradient: W'[ci][tap][co] = W[co][8 - tap][ci]
// (the transposed convolution is the convolution with the taps flipped), BF16.
__global__ void k_flip_weights(const bf16* __restrict__ W, int Cout, int Cin, int Kp,
                               bf16* __restrict__ Wf) {
  long long total = (long long)Cin * 9 * Cout;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int co = (int)(i % Cout);
    int tap = (int)((i / Cout) % 9);
    int ci = (int)(i / (9LL * Cout));
    Wf[i] = W[(size_t)co * Kp + (size_t)(8 - tap) * Cin + ci];
  }
}

// Sum of `splits` partial results in split order.
__global__ void k_split_sum(const float* __restrict__ part, long long stride, int splits,
                            float* __restrict__ out, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[k * stride + i];
    out[i] = s;
  }
}

// ------------------------------------------------------------------------------------------
// Layout kernels

// col[(b, oy, ox)][(dy * 3 + dx) * C + c] = X[b][oy*s + dy - 1][ox*s + dx - 1][c] (0 outside),
// zero for k >= 9 C up to Kp.
__global__ void k_im2col(const bf16* __restrict__ X, int Bn, int H, int W, int C, int s,
                         int Kp, bf16* __restrict__ col) {
  int Ho = H / s, Wo = W / s;
  long long total = (long long)Bn * Ho * Wo * Kp;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int k = (int)(i % Kp);
    long long p = i / Kp;
    int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho), b = (int)(p / ((long long)Wo * Ho));
    bf16 v = (bf16)0.f;
    if (k < 9 * C) {
      int tap = k / C, c = k - tap * C;
      int y = oy * s + tap / 3 - 1, x = ox * s + tap % 3 - 1;
      if (y >= 0 && y < H && x >= 0 && x < W) v = X[(((size_t)b * H + y) * W + x) * C + c];
    }
    col[i] = v;
  }
}

// The same columns 8 at a time (C and Kp multiples of 8, so 8 consecutive columns share one
// tap): one 16-byte load and store per thread, 32-bit index arithmetic (Bn Ho Wo Kp / 8 < 2^31).
__global__ void k_im2col8(const bf16* __restrict__ X, int Bn, int H, int W, int C, int s,
                          int Kp, bf16* __restrict__ col) {
  const int Ho = H / s, Wo = W / s, KV = Kp / 8;
  const unsigned total = (unsigned)((long long)Bn * Ho * Wo * KV);
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += gridDim.x * blockDim.x) {
    unsigned p = i / KV;
    int k = (int)(i - p * KV) * 8;
    int ox = (int)(p % Wo);
    unsigned q = p / Wo;
    int oy = (int)(q % Ho), b = (int)(q / Ho);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (k < 9 * C) {
      int tap = k / C, c = k - tap * C;
      int y = oy * s + tap / 3 - 1, x = ox * s + tap % 3 - 1;
      if (y >= 0 && y < H && x >= 0 && x < W)
        v = *(const uint4*)(X + (((size_t)b * H + y) * W + x) * C + c);
    }
    *(uint4*)(col + (size_t)p * Kp + k) = v;
  }
}

// dX[b][y][x][c] = sum of dcol over the output positions whose patch covers (y, x).
__global__ void k_col2im(const float* __restrict__ dcol, int Bn, int H, int W, int C, int s,
                         int ldk, float* __restrict__ dX, int accumulate) {
  int Ho = H / s, Wo = W / s;
  long long total = (long long)Bn * H * W * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int c = (int)(i % C);
    long long p = i / C;
    int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
    float sum = 0.f;
    for (int dy = 0; dy < 3; ++dy) {
      int ty = y + 1 - dy;
      if (ty < 0 || ty % s) continue;
      int oy = ty / s;
      if (oy >= Ho) continue;
      for (int dx = 0; dx < 3; ++dx) {
        int tx = x + 1 - dx;
        if (tx < 0 || tx % s) continue;
        int ox = tx / s;
        if (ox >= Wo) continue;
        sum += dcol[(((size_t)b * Ho + oy) * Wo + ox) * ldk + (dy * 3 + dx) * C + c];
      }
    }
    dX[i] = accumulate ? dX[i] + sum : sum;
  }
}

// U = [up2(lo) (C1 channels), skip (C2 channels)] at H x W (lo is H/2 x W/2).
__global__ void k_upcat(const bf16* __restrict__ lo, int C1, const bf16* __restrict__ skip,
                        int C2, int Bn, int H, int W, bf16* __restrict__ U) {
  int C = C1 + C2;
  long long total = (long long)Bn * H * W * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int c = (int)(i % C);
    long long p = i / C;
    int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
    U[i] = c < C1 ? lo[(((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C1 + c]
                  : skip[(((size_t)b * H + y) * W + x) * C2 + (c - C1)];
  }
}

// Backward of k_upcat: d_lo = 2x2 sums of the first C1 channels; d_skip (+)= the rest.
__global__ void k_upcat_bwd(const float* __restrict__ dU, int C1, int C2, int Bn, int H, int W,
                            float* __restrict__ dlo, float* __restrict__ dskip,
                            int skip_accumulate) {
  int C = C1 + C2;
  long long nlo = (long long)Bn * (H / 2) * (W / 2) * C1;
  long long nsk = dskip ? (long long)Bn * H * W * C2 : 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nlo + nsk;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < nlo) {
      int c = (int)(i % C1);
      long long p = i / C1;
      int X = (int)(p % (W / 2)), Y = (int)((p / (W / 2)) % (H / 2));
      int b = (int)(p / ((long long)(W / 2) * (H / 2)));
      float s = 0.f;
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          s += dU[(((size_t)b * H + 2 * Y + dy) * W + 2 * X + dx) * C + c];
      dlo[i] = s;
    } else {
      long long j = i - nlo;
      int c = (int)(j % C2);
      long long p = j / C2;
      float v = dU[p * C + C1 + c];
      dskip[j] = skip_accumulate ? dskip[j] + v : v;
    }
  }
}

// dZ = dA * (A > 0) as bf16 (A is the layer's ReLU output).
__global__ void k_relu_bwd(const float* __restrict__ dA, const bf16* __restrict__ A,
                           long long count, bf16* __restrict__ dZ) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dZ[i] = (bf16)((float)A[i] > 0.f ? dA[i] : 0.f);
}

// Column sums of a bf16 matrix [M][N] (bias gradients): per (column, chunk) partials.
__global__ void k_colsum_part(const bf16* __restrict__ G, long long M, int N, int chunks,
                              float* __restrict__ part) {
  __shared__ float red[kBlock];
  int n = blockIdx.x, ch = blockIdx.y;
  long long rows = (M + chunks - 1) / chunks;
  long long r0 = ch * rows, r1 = r0 + rows < M ? r0 + rows : M;
  float s = 0.f;
  for (long long r = r0 + threadIdx.x; r < r1; r += blockDim.x) s += (float)G[r * N + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)ch * N + n] = red[0];
}

// Column sums of per-chunk partials [chunks][N]: one workgroup (kBlock threads) per column;
// thread j sums chunks j, j + kBlock, ... in order, then a fixed tree over the threads.
__global__ void __launch_bounds__(kBlock) k_colsum_final(const float* __restrict__ part, int N,
                                                         int chunks, float* __restrict__ out) {
  __shared__ float red[kBlock];
  int n = blockIdx.x;
  float s = 0.f;
  for (int c = threadIdx.x; c < chunks; c += kBlock) s += part[(size_t)c * N + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

__global__ void k_f32_to_bf16(const float* __restrict__ x, long long count,
                              bf16* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (bf16)x[i];
}

// ------------------------------------------------------------------------------------------
// Last layer (66 -> 2 channels, stride 1), FP32 direct kernels. W6 is [2][9][66] fp32 (from the
// bf16 copy), bias b6[2].

// Last layer read straight from its sources. Channels 0..63 are the nearest 2x upsampling of
// the L5 output a5 [B][64][64][64]: output pixel (2Y + py, 2X + px) sees through its 3x3 taps
// only the 2 x 2 source pixels (Y - 1 + py + i, X - 1 + px + j), i, j in {0, 1} (tap rows
// {0} and {1, 2} land on source rows Y - 1 and Y when py = 0, {0, 1} and {2} on Y and Y + 1
// when py = 1; columns alike), so the taps that land on one source pixel are summed into the
// folded weights W6f [parity py px][i][j][output][64] (k_w6_prep): 4 source pixels of 64
// channels instead of 9. Channels 64, 65 are the network input x0 [B][128][128][2] (9 taps,
// weights W6 [2][9][66]). Eight lanes share an output pixel, lane g taking channels 8g .. 8g + 7
// (one 16-byte piece of each source pixel, so a source pixel is one 128-byte line per 8 lanes)
// and x0 tap g (and tap 8 on lane 0); the 8 partial sums are then added across the lanes.
// One workgroup per (sample, parity, 32 source pixels of a row): a wave's parity is uniform.
__global__ void __launch_bounds__(256) k_l6_fused(const bf16* __restrict__ a5,
                                                  const bf16* __restrict__ x0,
                                                  const float* __restrict__ W6,
                                                  const float* __restrict__ W6f,
                                                  const float* __restrict__ b6, int Bn,
                                                  float* __restrict__ Y) {
  constexpr int C = 66;
  __shared__ __attribute__((aligned(16))) float wf[4 * 2 * 2 * 2 * 64];
  for (int e = threadIdx.x; e < 4 * 2 * 2 * 2 * 64; e += blockDim.x) wf[e] = W6f[e];
  __syncthreads();
  const int g = threadIdx.x & 7;  // channel group
  const int nblk = Bn * 4 * 64 * 2;  // (sample, parity, source row, half row)
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int half = blk & 1, ys = (blk >> 1) & 63, par = (blk >> 7) & 3, b = blk >> 9;
    const int py = par >> 1, px = par & 1;
    const int xs = half * 32 + (threadIdx.x >> 3);
    const int y = 2 * ys + py, x = 2 * xs + px;
    float s0 = g == 0 ? b6[0] : 0.f, s1 = g == 0 ? b6[1] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int sy = ys - 1 + py + i;
      if (sy < 0 || sy >= 64) continue;  // uniform over the workgroup (one source row)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int sx = xs - 1 + px + j;
        const bool ok = sx >= 0 && sx < 64;
        uint4 v = ok ? *(const uint4*)(a5 + (((size_t)b * 64 + sy) * 64 + sx) * 64 + 8 * g)
                     : make_uint4(0u, 0u, 0u, 0u);
        const float* w0 = wf + (((par * 2 + i) * 2 + j) * 2) * 64 + 8 * g;
        const f32x4 wa = *(const f32x4*)w0, wb = *(const f32x4*)(w0 + 4);
        const f32x4 wc = *(const f32x4*)(w0 + 64), wd = *(const f32x4*)(w0 + 68);
        const unsigned int h[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float lo = __uint_as_float(h[k] << 16), hi = __uint_as_float(h[k] & 0xffff0000u);
          const float w0lo = k < 2 ? wa[2 * k] : wb[2 * k - 4];
          const float w0hi = k < 2 ? wa[2 * k + 1] : wb[2 * k - 3];
          const float w1lo = k < 2 ? wc[2 * k] : wd[2 * k - 4];
          const float w1hi = k < 2 ? wc[2 * k + 1] : wd[2 * k - 3];
          s0 = fmaf(w0lo, lo, s0);
          s1 = fmaf(w1lo, lo, s1);
          s0 = fmaf(w0hi, hi, s0);
          s1 = fmaf(w1hi, hi, s1);
        }
      }
    }
    // x0 channels: lane g takes tap g, lane 0 also tap 8
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int tap = t == 0 ? g : 8;
      if (t == 1 && g != 0) break;
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      if (yy >= 0 && yy < 128 && xx >= 0 && xx < 128) {
        const unsigned int v = *(const unsigned int*)(x0 + (((size_t)b * 128 + yy) * 128 + xx) * 2);
        const float f0 = __uint_as_float(v << 16), f1 = __uint_as_float(v & 0xffff0000u);
        s0 = fmaf(W6[tap * C + 64], f0, s0);
        s1 = fmaf(W6[9 * C + tap * C + 64], f0, s1);
        s0 = fmaf(W6[tap * C + 65], f1, s0);
        s1 = fmaf(W6[9 * C + tap * C + 65], f1, s1);
      }
    }
    // the 8 channel groups' partial sums (lanes 8p .. 8p + 7), fixed order
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
      s0 += __shfl_xor(s0, m, 64);
      s1 += __shfl_xor(s1, m, 64);
    }
    if (g == 0) {
      const size_t o = (((size_t)b * 128 + y) * 128 + x) * 2;
      Y[o] = s0;
      Y[o + 1] = s1;
    }
  }
}

// FP32 copies of the last layer's weights from the BF16 copy: W6 [2][9][66] (the backward
// pass's) and the folded W6f of k_l6_fused, each entry the sum, in tap order, of the taps that
// land on its source pixel. One workgroup.
__global__ void __launch_bounds__(256) k_w6_prep(const bf16* __restrict__ wb6,
                                                 float* __restrict__ W6,
                                                 float* __restrict__ W6f) {
  constexpr int C = 66;
  for (int k = threadIdx.x; k < 2 * 9 * C; k += blockDim.x) W6[k] = (float)wb6[k];
  __syncthreads();
  for (int e = threadIdx.x; e < 4 * 2 * 2 * 2 * 64; e += blockDim.x) {
    const int c = e & 63, o = (e >> 6) & 1, j = (e >> 7) & 1, i = (e >> 8) & 1, par = e >> 9;
    const int py = par >> 1, px = par & 1;
    // tap rows (columns) landing on source row (column) offset i (j) for parity py (px)
    const int r0 = py == 0 ? (i == 0 ? 0 : 1) : (i == 0 ? 0 : 2);
    const int r1 = py == 0 ? (i == 0 ? 0 : 2) : (i == 0 ? 1 : 2);
    const int c0 = px == 0 ? (j == 0 ? 0 : 1) : (j == 0 ? 0 : 2);
    const int c1 = px == 0 ? (j == 0 ? 0 : 2) : (j == 0 ? 1 : 2);
    float acc = 0.f;
    for (int ty = r0; ty <= r1; ++ty)
      for (int tx = c0; tx <= c1; ++tx) acc += W6[o * 9 * C + (ty * 3 + tx) * C + c];
    W6f[e] = acc;
  }
}

// First layer (2 -> 64 channels, stride 2, 128^2 -> 64^2) straight from the input x0
// [B][128][128][2]: one thread per output pixel holds its 18 inputs (k = tap * 2 + c); the
// weights (FP32 from the BF16 copy, [k][64]) and the bias sit in LDS, read four channels at a
// time at one address per wave; FP32 sums in k order, then bias and ReLU; the 64 BF16 outputs
// leave as eight 16-byte stores (NHWC).
__global__ void __launch_bounds__(256) k_l1_direct(const bf16* __restrict__ x0,
                                                   const bf16* __restrict__ W, int Kp,
                                                   const float* __restrict__ bias, int Bn,
                                                   bf16* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) float ws[18][64];
  __shared__ __attribute__((aligned(16))) float bs[64];
  for (int e = threadIdx.x; e < 18 * 64; e += blockDim.x) {
    const int co = e / 18, k = e - co * 18;
    ws[k][co] = (float)W[co * Kp + k];
  }
  if (threadIdx.x < 64) bs[threadIdx.x] = bias[threadIdx.x];
  __syncthreads();
  const long long total = (long long)Bn * 64 * 64;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < total;
       p += (long long)gridDim.x * blockDim.x) {
    const int ox = (int)(p & 63), oy = (int)((p >> 6) & 63);
    const long long b = p >> 12;
    float in[18];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
      const bool ok = iy >= 0 && iy < 128 && ix >= 0 && ix < 128;
      unsigned int v = ok ? *(const unsigned int*)(x0 + ((b * 128 + iy) * 128 + ix) * 2) : 0u;
      in[2 * tap] = __uint_as_float(v << 16);
      in[2 * tap + 1] = __uint_as_float(v & 0xffff0000u);
    }
    uint2* dst = (uint2*)(out + p * 64);
#pragma unroll 1
    for (int g = 0; g < 16; ++g) {  // output channels 4g .. 4g + 3
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 18; ++k) {
        const f32x4 w = *(const f32x4*)&ws[k][4 * g];
        acc[0] = fmaf(w[0], in[k], acc[0]);
        acc[1] = fmaf(w[1], in[k], acc[1]);
        acc[2] = fmaf(w[2], in[k], acc[2]);
        acc[3] = fmaf(w[3], in[k], acc[3]);
      }
      const f32x4 bb = *(const f32x4*)&bs[4 * g];
      unsigned int h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = acc[r] + bb[r];
        h[r] = __builtin_bit_cast(unsigned short, (bf16)(v > 0.f ? v : 0.f));
      }
      dst[g] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
  }
}

// Data gradient of the last layer for its upsampled input, straight onto the L5 output grid
// (the adjoint of k_l6_fused's folded product, which also sums the four upsampled copies):
// source pixel (Y, X) feeds the outputs (2 Ys + py, 2 Xs + px) with Ys = Y + 1 - py - i and
// Xs = X + 1 - px - j through W6f[py px][i][j][o][c] (the output rows 2Y - 1 .. 2Y + 2 and the
// columns alike, 2 outputs each). One wave per source pixel, one lane per channel: the dY
// values of a wave are the same for every lane; the weights sit in LDS.
__global__ void __launch_bounds__(256) k_l6_bwd_a5(const float* __restrict__ dY,
                                                   const float* __restrict__ W6f, int Bn,
                                                   float* __restrict__ dA5) {
  __shared__ float w[4 * 2 * 2 * 2 * 64];
  for (int e = threadIdx.x; e < 4 * 2 * 2 * 2 * 64; e += blockDim.x) w[e] = W6f[e];
  __syncthreads();
  const int c = threadIdx.x & 63;
  const long long npix = (long long)Bn * 64 * 64;
  const long long step = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long p = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6; p < npix;
       p += step) {
    // one source pixel per wave: its index in scalar registers, so the dY reads are scalar
    const int pu = __builtin_amdgcn_readfirstlane((int)p);
    const int X = pu & 63, Y = (pu >> 6) & 63;
    const long long b = pu >> 12;
    float s = 0.f;
#pragma unroll
    for (int py = 0; py < 2; ++py)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int y = 2 * (Y + 1 - py - i) + py;
        if (y < 0 || y >= 128) continue;
#pragma unroll
        for (int px = 0; px < 2; ++px)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int x = 2 * (X + 1 - px - j) + px;
            if (x < 0 || x >= 128) continue;
            const float* g = dY + ((b * 128 + y) * 128 + x) * 2;
            const float* wp = w + ((((py * 2 + px) * 2 + i) * 2 + j) * 2) * 64 + c;
            s = fmaf(wp[0], g[0], s);
            s = fmaf(wp[64], g[1], s);
          }
      }
    dA5[p * 64 + c] = s;
  }
}

// L6 weight and bias gradients by tiles: one block per 16x16 tile of output positions of one
// 128 x 128 image. The tile's 18x18 halo of the layer input U (zero outside the image: channels
// 0..63 the 2x upsampled L5 output a5 [B][64][64][64], read through the halving of the
// position; 64, 65 the network input x0 [B][128][128][2]) and its dY are staged in LDS; each
// thread sums, over the tile's 256 positions in order, dY(p, o) U(p + tap, c) for both
// outputs o of its (tap, c) pairs, or dY(p, o) for the bias. Per-block partials
// [block][2 * 9 * C + 2] (weights o-major as in the layer, then the two biases), summed over
// blocks in a fixed order by k_colsum_final. C == L6C.
constexpr int L6T = 16, L6H = L6T + 2, L6C = 66;
__global__ void __launch_bounds__(256) k_l6_bwd_w_tile(const float* __restrict__ dY,
                                                       const bf16* __restrict__ a5,
                                                       const bf16* __restrict__ x0,
                                                       float* __restrict__ part) {
  constexpr int H = 128, Wd = 128;
  __shared__ bf16 sU[L6H * L6H * L6C];
  __shared__ float2 sY[L6T * L6T];
  const int tx_n = Wd / L6T, per_img = tx_n * (H / L6T);
  const int b = blockIdx.x / per_img, tt = blockIdx.x % per_img;
  const int ty0 = (tt / tx_n) * L6T, tx0 = (tt % tx_n) * L6T;
  for (int i = threadIdx.x; i < L6H * L6H * L6C; i += blockDim.x) {
    int c = i % L6C, pix = i / L6C;
    int y = ty0 + pix / L6H - 1, x = tx0 + pix % L6H - 1;
    bool in = y >= 0 && y < H && x >= 0 && x < Wd;
    bf16 v = (bf16)0.f;
    if (in)
      v = c < 64 ? a5[(((size_t)b * 64 + (y >> 1)) * 64 + (x >> 1)) * 64 + c]
                 : x0[(((size_t)b * H + y) * Wd + x) * 2 + (c - 64)];
    sU[i] = v;
  }
  for (int p = threadIdx.x; p < L6T * L6T; p += blockDim.x) {
    size_t q = ((size_t)b * H + ty0 + p / L6T) * Wd + tx0 + p % L6T;
    sY[p] = make_float2(dY[2 * q], dY[2 * q + 1]);
  }
  __syncthreads();
  constexpr int NP = 9 * L6C;  // (tap, c) pairs
  float* out = part + (size_t)blockIdx.x * (2 * NP + 2);
  for (int q = threadIdx.x; q <= NP; q += blockDim.x) {
    float a0 = 0.f, a1 = 0.f;
    if (q < NP) {
      const int tap = q / L6C, c = q % L6C;
      const bf16* u0 = sU + ((tap / 3) * L6H + tap % 3) * L6C + c;
      for (int py = 0; py < L6T; ++py) {
        const bf16* ur = u0 + py * L6H * L6C;
#pragma unroll
        for (int px = 0; px < L6T; ++px) {
          float u = (float)ur[px * L6C];
          float2 g = sY[py * L6T + px];
          a0 = fmaf(g.x, u, a0);
          a1 = fmaf(g.y, u, a1);
        }
      }
      out[q] = a0;
      out[NP + q] = a1;
    } else {
      for (int p = 0; p < L6T * L6T; ++p) {
        a0 += sY[p].x;
        a1 += sY[p].y;
      }
      out[2 * NP] = a0;
      out[2 * NP + 1] = a1;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Loss: mean squared error over the interior (a border of `margin` pixels is left out).
// Writes per-block partial sums of squares and dY = 2 (Y - T) / count (0 in the border).

__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int Bn, int H,
                      int Wd, int margin, float inv_count, float* __restrict__ dY,
                      double* __restrict__ part) {
  __shared__ double red[kBlock];
  long long total = (long long)Bn * H * Wd * 2;
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    long long p = i / 2;
    int x = (int)(p % Wd), y = (int)((p / Wd) % H);
    bool in = x >= margin && x < Wd - margin && y >= margin && y < H - margin;
    float d = in ? Y[i] - T[i] : 0.f;
    s += (double)d * d;
    if (dY) dY[i] = 2.f * d * inv_count;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam on FP32 master weights; refreshes the bf16 copy. Gradient g is the full fp32 gradient.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long count, float lr, float b1,
                       float b2, float eps, float c1, float c2, bf16* __restrict__ wb) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (bf16)wi;
  }
}

// Pack level-7 normalised frames of pairs into the network input [P][128][128][2] (fp32):
// channel 0 = reference, 1 = template; the 129^2 grid is cropped to 128^2.
__global__ void k_pack_pairs(const float* __restrict__ lvl, int n, const int* __restrict__ ref,
                             const int* __restrict__ tmpl, int P, float* __restrict__ out) {
  int S = n - 1;
  long long total = (long long)P * S * S;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int x = (int)(i % S), y = (int)((i / S) % S), p = (int)(i / ((long long)S * S));
    out[i * 2] = lvl[(size_t)ref[p] * n * n + (size_t)y * n + x];
    out[i * 2 + 1] = lvl[(size_t)tmpl[p] * n * n + (size_t)y * n + x];
  }
}

// Level-7 displacement planes [P][2][n][n] (domain units) -> [P][n-1][n-1][2] in cells.
__global__ void k_planes_to_nhwc(const float* __restrict__ src, int n, long long pstride, int P,
                                 float scale, float* __restrict__ out) {
  int S = n - 1;
  long long total = (long long)P * S * S;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int x = (int)(i % S), y = (int)((i / S) % S), p = (int)(i / ((long long)S * S));
    const float* s = src + p * pstride;
    out[i * 2] = scale * s[(size_t)y * n + x];
    out[i * 2 + 1] = scale * s[(size_t)n * n + (size_t)y * n + x];
  }
}

// Network output [P][S][S][2] (cells) -> slot planes [2][S+1][S+1] (domain units), replicating
// the last row and column; dst of slot p = base + p * stride.
__global__ void k_nhwc_to_planes(const float* __restrict__ y, int S, int P, float scale,
                                 float* __restrict__ base, long long stride) {
  int n = S + 1;
  long long total = (long long)P * n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int x = (int)(i % n), yy = (int)((i / n) % n), p = (int)(i / ((long long)n * n));
    int xs = min(x, S - 1), ys = min(yy, S - 1);
    const float* src = y + (((size_t)p * S + ys) * S + xs) * 2;
    float* d = base + p * stride;
    d[(size_t)yy * n + x] = scale * src[0];
    d[(size_t)n * n + (size_t)yy * n + x] = scale * src[1];
  }
}

// bad[p] = 1 when sample p of y [P][n_per] has a non-finite value or one with |v| > limit.
__global__ void k_check_pred(const float* __restrict__ y, long long n_per, float limit,
                             int* __restrict__ bad) {
  __shared__ int red[kBlock];
  const float* s = y + blockIdx.x * n_per;
  int b = 0;
  for (long long i = threadIdx.x; i < n_per; i += blockDim.x) {
    float v = s[i];
    if (!(fabsf(v) <= limit)) b = 1;
  }
  red[threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] |= red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bad[blockIdx.x] = red[0];
}

}  // namespace

// ==========================================================================================
// Model

namespace pprs_cnn_impl {

struct Layer {
  int cin, cout, stride, kp;    // kp: padded K (columns of the weight matrix)
  int hin, hout;                // spatial size of input / output (square)
  long long woff, boff;         // offsets into the flat parameter vector
};

struct Model {
  int device = 0;
  hipStream_t stream = nullptr;
  Layer L[6];
  long long n_params = 0;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // fp32 master, Adam, grad
  bf16* wb = nullptr;                                            // bf16 copy of w
  bf16* wflip = nullptr;  // flipped, transposed weights of a decoder layer (its data gradient)
  bf16* wfold[2] = {nullptr, nullptr};  // folded weights of the upsampling layers L4, L5
  long long step = 0;
  int cap_b = 0;
  // activations and workspaces (sized for cap_b)
  bf16 *x0 = nullptr, *a[5] = {nullptr}, *u4 = nullptr, *u5 = nullptr,
       *col = nullptr, *dzb = nullptr;
  float *z = nullptr, *y = nullptr, *dy = nullptr, *dcol = nullptr, *du = nullptr,
        *da[5] = {nullptr}, *part = nullptr, *w6 = nullptr, *w6f = nullptr;
  double* lpart = nullptr;
  size_t part_floats = 0;
};

}  // namespace pprs_cnn_impl

struct pprs_cnn {
  pprs_cnn_impl::Model M;
};

using pprs_cnn_impl::Layer;
using pprs_cnn_impl::Model;

static thread_local std::string g_cnn_err;

static pprs_status cfail(pprs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_cnn_err = buf;
  return s;
}

#define CHK(expr)                                                                     \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return cfail(PPRS_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                         \
  } while (0)

static pprs_status gemm(Model& M, bool ak, bool bk, const bf16* A, int lda, const bf16* B,
                        int ldb, float* C, int ldc, int Mr, int Nc, int K, int splits) {
  if (Mr % 64 || Nc % 64 || K % 32 || lda % 8 || ldb % 8)
    return cfail(PPRS_EINVAL, "gemm shape %d x %d x %d not tileable", Mr, Nc, K);
  int kps = ((K / 32 + splits - 1) / splits) * 32;
  splits = (K + kps - 1) / kps;
  float* out = C;
  long long stride = (long long)Mr * ldc;
  if (splits > 1) {
    if ((size_t)splits * stride > M.part_floats)
      return cfail(PPRS_EINVAL, "split-K workspace too small");
    out = M.part;
  }
  dim3 grid(Nc / 64, Mr / 64, splits);
  if (!ak && !bk) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, M.stream, A, lda, B, ldb, out, ldc, K, kps, stride);
  else if (!ak && bk) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, M.stream, A, lda, B, ldb, out, ldc, K, kps, stride);
  else if (ak && !bk) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, M.stream, A, lda, B, ldb, out, ldc, K, kps, stride);
  else hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, M.stream, A, lda, B, ldb, out, ldc, K, kps, stride);
  CHK(hipGetLastError());
  if (splits > 1) {
    hipLaunchKernelGGL(k_split_sum, dim3(grid1d(stride)), dim3(kBlock), 0, M.stream, M.part,
                       stride, splits, C, stride);
    CHK(hipGetLastError());
  }
  return PPRS_OK;
}

static void define_layers(Model& M) {
  const int cin[6] = {2, 64, 128, 384, 192, 66}, cout[6] = {64, 128, 256, 128, 64, 2};
  const int stride[6] = {2, 2, 2, 1, 1, 1}, hin[6] = {128, 64, 32, 32, 64, 128};
  long long off = 0;
  for (int l = 0; l < 6; ++l) {
    Layer& y = M.L[l];
    y.cin = cin[l];
    y.cout = cout[l];
    y.stride = stride[l];
    y.hin = hin[l];
    y.hout = hin[l] / stride[l];
    int k = 9 * cin[l];
    y.kp = l == 0 ? 64 : (l == 5 ? k : ((k + 31) / 32) * 32);
    y.woff = off;
    off += (long long)y.cout * y.kp;
    y.boff = off;
    off += y.cout;
  }
  M.n_params = off;
}

static pprs_status alloc_batch(Model& M, int B) {
  if (B <= M.cap_b) return PPRS_OK;
  void* ptrs[] = {M.x0, M.a[0], M.a[1], M.a[2], M.a[3], M.a[4], M.u4, M.u5, M.col, M.dzb,
                  M.z, M.y, M.dy, M.dcol, M.du, M.da[0], M.da[1], M.da[2], M.da[3], M.da[4],
                  M.part, M.lpart, M.wflip};
  for (void* p : ptrs)
    if (p) CHK(hipFree(p));
  long long P128 = (long long)B * 128 * 128, P64 = P128 / 4, P32 = P128 / 16, P16 = P128 / 64;
  long long col_max = 0, z_max = 0, dcol_max = 0;
  for (int l = 0; l < 5; ++l) {
    long long pix = (long long)B * M.L[l].hout * M.L[l].hout;
    col_max = std::max(col_max, pix * M.L[l].kp);
    z_max = std::max(z_max, pix * (long long)M.L[l].cout);
    if (l == 1 || l == 2) dcol_max = std::max(dcol_max, pix * M.L[l].kp);  // via col2im
  }
  CHK(hipMalloc(&M.x0, sizeof(bf16) * P128 * 2));
  CHK(hipMalloc(&M.a[0], sizeof(bf16) * P64 * 64));
  CHK(hipMalloc(&M.a[1], sizeof(bf16) * P32 * 128));
  CHK(hipMalloc(&M.a[2], sizeof(bf16) * P16 * 256));
  CHK(hipMalloc(&M.a[3], sizeof(bf16) * P32 * 128));
  CHK(hipMalloc(&M.a[4], sizeof(bf16) * P64 * 64));
  CHK(hipMalloc(&M.u4, sizeof(bf16) * P32 * 384));
  CHK(hipMalloc(&M.u5, sizeof(bf16) * P64 * 192));
  long long wf = 0;
  for (int l = 3; l < 5; ++l) wf = std::max(wf, (long long)M.L[l].cin * 9 * M.L[l].cout);
  CHK(hipMalloc(&M.wflip, sizeof(bf16) * wf));
  CHK(hipMalloc(&M.col, sizeof(bf16) * col_max));
  CHK(hipMalloc(&M.dzb, sizeof(bf16) * z_max));
  CHK(hipMalloc(&M.z, sizeof(float) * z_max));
  CHK(hipMalloc(&M.y, sizeof(float) * P128 * 2));
  CHK(hipMalloc(&M.dy, sizeof(float) * P128 * 2));
  CHK(hipMalloc(&M.dcol, sizeof(float) * dcol_max));
  CHK(hipMalloc(&M.du, sizeof(float) * P128 * 66));
  CHK(hipMalloc(&M.da[0], sizeof(float) * P64 * 64));
  CHK(hipMalloc(&M.da[1], sizeof(float) * P32 * 128));
  CHK(hipMalloc(&M.da[2], sizeof(float) * P16 * 256));
  CHK(hipMalloc(&M.da[3], sizeof(float) * P32 * 128));
  CHK(hipMalloc(&M.da[4], sizeof(float) * P64 * 64));
  // split-K partials: weight gradients (<= 64 splits of the largest weight) or layer outputs
  long long wmax = 0;
  for (int l = 0; l < 5; ++l) wmax = std::max(wmax, (long long)M.L[l].cout * M.L[l].kp);
  M.part_floats = (size_t)std::max(64 * wmax, (long long)B * (128 / L6T) * (128 / L6T) *
                                                  (2 * 9 * L6C + 2));
  CHK(hipMalloc(&M.part, sizeof(float) * M.part_floats));
  CHK(hipMalloc(&M.lpart, sizeof(double) * 1024));
  M.cap_b = B;
  return PPRS_OK;
}

// Fused convolution of layer l (L2..L5) into M.a[l].
static pprs_status conv_fused(Model& M, int l, int B) {
  const Layer& y = M.L[l];
  const bf16* s0 = l == 1 ? M.a[0] : l == 2 ? M.a[1] : l == 3 ? M.a[2] : M.a[3];
  const bf16* s1 = l == 3 ? M.a[1] : l == 4 ? M.a[0] : nullptr;
  int c0 = l == 1 ? 64 : l == 2 ? 128 : l == 3 ? 256 : 128;
  int c1 = y.cin - c0;
  bool up = l >= 3;
  long long pix = (long long)B * y.hout * y.hout;
  if (pix % CV_BM || c0 % 64 || c1 % 64 || y.kp != 9 * y.cin)
    return cfail(PPRS_EINVAL, "layer %d does not fit the fused convolution", l + 1);
  int bn = y.cout % 128 == 0 ? 128 : 64;
  dim3 grid((unsigned)(pix / CV_BM), y.cout / bn);
  const bf16* w = M.wb + y.woff;
  const float* b = M.w + y.boff;
  if (up) {
    // folded upsampling: per output parity, 4 C0 + 9 C1 deep (pixels of one parity per tile)
    const int kf = 4 * c0 + 9 * c1;
    if ((pix / 4) % CV_BM) return cfail(PPRS_EINVAL, "layer %d does not fit the folded convolution", l + 1);
    const bf16* wf = M.wfold[l - 3];
    if (bn == 128)
      hipLaunchKernelGGL((k_conv_fwd<128, true, false, true>), grid, dim3(256), 0, M.stream, s0, c0, s1, c1, y.hin, y.stride, wf, kf, b, y.cout, M.a[l]);
    else
      hipLaunchKernelGGL((k_conv_fwd<64, true, false, true>), grid, dim3(256), 0, M.stream, s0, c0, s1, c1, y.hin, y.stride, wf, kf, b, y.cout, M.a[l]);
  } else if (bn == 128) {
    hipLaunchKernelGGL((k_conv_fwd<128, false>), grid, dim3(256), 0, M.stream, s0, c0, s1, c1, y.hin, y.stride, w, y.kp, b, y.cout, M.a[l]);
  } else {
    hipLaunchKernelGGL((k_conv_fwd<64, false>), grid, dim3(256), 0, M.stream, s0, c0, s1, c1, y.hin, y.stride, w, y.kp, b, y.cout, M.a[l]);
  }
  CHK(hipGetLastError());
  return PPRS_OK;
}

// Forward pass for B samples; input x [B][128][128][2] fp32; output in M.y. With `train`, the
// decoder inputs (upsampled + concatenated) are also kept for the weight gradients.
static pprs_status forward(Model& M, const float* x, int B, bool train) {
  hipStream_t st = M.stream;
  long long P128 = (long long)B * 128 * 128;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid1d(P128 * 2)), dim3(kBlock), 0, st, x, P128 * 2, M.x0);
  {
    // L1 (2 input channels): a direct kernel (18 products per output channel)
    const Layer& y = M.L[0];
    long long pix = (long long)B * y.hout * y.hout;
    hipLaunchKernelGGL(k_l1_direct, dim3(grid1d(pix)), dim3(kBlock), 0, st, M.x0, M.wb + y.woff, y.kp, M.w + y.boff, B, M.a[0]);
  }
  for (int l = 1; l < 5; ++l) {
    pprs_status s = conv_fused(M, l, B);
    if (s != PPRS_OK) return s;
  }
  if (train) {
    long long p32 = (long long)B * 32 * 32, p64 = (long long)B * 64 * 64;
    hipLaunchKernelGGL(k_upcat, dim3(grid1d(p32 * 384)), dim3(kBlock), 0, st, M.a[2], 256, M.a[1], 128, B, 32, 32, M.u4);
    hipLaunchKernelGGL(k_upcat, dim3(grid1d(p64 * 192)), dim3(kBlock), 0, st, M.a[3], 128, M.a[0], 64, B, 64, 64, M.u5);
  }
  // L6
  const Layer& y6 = M.L[5];
  hipLaunchKernelGGL(k_l6_fused, dim3(std::min(B * 512, 16384)), dim3(kBlock), 0, st, M.a[4], M.x0, M.w6, M.w6f, M.w + y6.boff, B, M.y);
  CHK(hipGetLastError());
  return PPRS_OK;
}

// fp32 view of the L6 weights from the bf16 copy (so every layer computes with bf16 weights).
// Weight copies derived from the BF16 weights, remade whenever they change: L6's FP32 copies
// and the folded weights of the upsampling layers L4 and L5.
static pprs_status refresh_derived(Model& M) {
  const Layer& y6 = M.L[5];
  hipLaunchKernelGGL(k_w6_prep, dim3(1), dim3(kBlock), 0, M.stream, M.wb + y6.woff, M.w6, M.w6f);
  for (int l = 3; l < 5; ++l) {
    const Layer& y = M.L[l];
    const int c0 = l == 3 ? 256 : 128, c1 = y.cin - c0;
    hipLaunchKernelGGL(k_fold_weights, dim3(grid1d(4LL * y.cout * (4 * c0 + 9 * c1))), dim3(kBlock), 0, M.stream, M.wb + y.woff, y.cout, c0, c1, y.kp, M.wfold[l - 3]);
  }
  CHK(hipGetLastError());
  return PPRS_OK;
}

// Loss and full gradient into M.g (uses M.y from forward). Returns the mean squared error.
static pprs_status backward(Model& M, const float* target, int B, int margin, double* loss) {
  hipStream_t st = M.stream;
  long long P128 = (long long)B * 128 * 128;
  int interior = 128 - 2 * margin;
  float inv_count = 1.f / ((float)B * interior * interior * 2);
  int blocks = 1024;
  hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(kBlock), 0, st, M.y, target, B, 128, 128, margin, inv_count, M.dy, M.lpart);
  std::vector<double> hp(blocks);
  CHK(hipMemcpyAsync(hp.data(), M.lpart, sizeof(double) * blocks, hipMemcpyDeviceToHost, st));
  CHK(hipMemsetAsync(M.g, 0, sizeof(float) * M.n_params, st));
  // L6: dW6, db6, dU6
  const Layer& y6 = M.L[5];
  {
    int nw = 2 * 9 * 66 + 2, chunks = B * (128 / L6T) * (128 / L6T);
    hipLaunchKernelGGL(k_l6_bwd_w_tile, dim3(chunks), dim3(256), 0, st, M.dy, M.a[4], M.x0, M.part);
    // weights [2][9*66] then bias [2] are contiguous at woff: columns 0..nw-1 map to them
    hipLaunchKernelGGL(k_colsum_final, dim3(nw), dim3(kBlock), 0, st, M.part, nw, chunks, M.g + y6.woff);
    // d a[4] through the folded weights (the input part needs no gradient)
    hipLaunchKernelGGL(k_l6_bwd_a5, dim3(grid1d(P128 / 4 * 64)), dim3(kBlock), 0, st, M.dy, M.w6f, B, M.da[4]);
  }
  CHK(hipGetLastError());
  // L5 .. L1
  const bf16* in[5] = {M.x0, M.a[0], M.a[1], M.u4, M.u5};
  for (int l = 4; l >= 0; --l) {
    const Layer& y = M.L[l];
    long long pix = (long long)B * y.hout * y.hout;
    // dZ = dA * relu'(A)
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1d(pix * y.cout)), dim3(kBlock), 0, st, M.da[l], M.a[l], pix * y.cout, M.dzb);
    // bias gradient
    int chunks = 64;
    hipLaunchKernelGGL(k_colsum_part, dim3(y.cout, chunks), dim3(kBlock), 0, st, M.dzb, pix, y.cout, chunks, M.part);
    hipLaunchKernelGGL(k_colsum_final, dim3(y.cout), dim3(kBlock), 0, st, M.part, y.cout, chunks, M.g + y.boff);
    // weight gradient: dW[co][k] = sum_pix dZ[pix][co] col[pix][k]
    if (y.cin % 8 == 0 && y.kp % 8 == 0 && pix * (y.kp / 8) < (1LL << 31))
      hipLaunchKernelGGL(k_im2col8, dim3(grid1d(pix * y.kp / 8)), dim3(kBlock), 0, st, in[l], B, y.hin, y.hin, y.cin, y.stride, y.kp, M.col);
    else
      hipLaunchKernelGGL(k_im2col, dim3(grid1d(pix * y.kp)), dim3(kBlock), 0, st, in[l], B, y.hin, y.hin, y.cin, y.stride, y.kp, M.col);
    int splits = (int)std::min<long long>(64, pix / 256);
    if (splits < 1) splits = 1;
    pprs_status s = gemm(M, true, true, M.dzb, y.cout, M.col, y.kp, M.g + y.woff, y.kp, y.cout, y.kp, (int)pix, splits);
    if (s != PPRS_OK) return s;
    if (l == 0) break;
    if (l == 4 || l == 3) {
      // data gradient of the stride-1 decoder layers as a convolution of dZ with the flipped,
      // transposed weights (implicit GEMM, no materialised columns): dU [pix][cin] FP32
      hipLaunchKernelGGL(k_flip_weights, dim3(grid1d((long long)y.cin * 9 * y.cout)), dim3(kBlock), 0, st, M.wb + y.woff, y.cout, y.cin, y.kp, M.wflip);
      int bn = y.cin % 128 == 0 ? 128 : 64;
      dim3 grid((unsigned)(pix / CV_BM), y.cin / bn);
      if (bn == 128)
        hipLaunchKernelGGL((k_conv_fwd<128, false, true>), grid, dim3(256), 0, st, M.dzb, y.cout, (const bf16*)nullptr, 0, y.hout, 1, M.wflip, 9 * y.cout, (const float*)nullptr, y.cin, (void*)M.du);
      else
        hipLaunchKernelGGL((k_conv_fwd<64, false, true>), grid, dim3(256), 0, st, M.dzb, y.cout, (const bf16*)nullptr, 0, y.hout, 1, M.wflip, 9 * y.cout, (const float*)nullptr, y.cin, (void*)M.du);
      if (l == 4)
        // input u5 = [up2(a4) 128, a1 64] at 64^2
        hipLaunchKernelGGL(k_upcat_bwd, dim3(grid1d((long long)B * 64 * 64 * 64 + (long long)B * 32 * 32 * 128)), dim3(kBlock), 0, st, M.du, 128, 64, B, 64, 64, M.da[3], M.da[0], 0);
      else
        // input u4 = [up2(a3) 256, a2 128] at 32^2
        hipLaunchKernelGGL(k_upcat_bwd, dim3(grid1d((long long)B * 16 * 16 * 256 + (long long)B * 32 * 32 * 128)), dim3(kBlock), 0, st, M.du, 256, 128, B, 32, 32, M.da[2], M.da[1], 0);
      CHK(hipGetLastError());
      continue;
    }
    // data gradient: dcol[pix][k] = sum_co dZ[pix][co] W[co][k]; then col2im into the input
    s = gemm(M, false, true, M.dzb, y.cout, M.wb + y.woff, y.kp, M.dcol, y.kp, (int)pix, y.kp, y.cout, 1);
    if (s != PPRS_OK) return s;
    if (l == 2) {
      // input a2 (32^2 x 128), stride 2; a2 already holds the skip gradient from L4
      hipLaunchKernelGGL(k_col2im, dim3(grid1d((long long)B * 32 * 32 * 128)), dim3(kBlock), 0, st, M.dcol, B, 32, 32, 128, 2, y.kp, M.da[1], 1);
    } else if (l == 1) {
      // input a1 (64^2 x 64), stride 2; a1 already holds the skip gradient from L5
      hipLaunchKernelGGL(k_col2im, dim3(grid1d((long long)B * 64 * 64 * 64)), dim3(kBlock), 0, st, M.dcol, B, 64, 64, 64, 2, y.kp, M.da[0], 1);
    }
    CHK(hipGetLastError());
  }
  CHK(hipStreamSynchronize(st));
  double sum = 0.0;
  for (int i = 0; i < blocks; ++i) sum += hp[i];
  if (loss) *loss = sum / ((double)B * interior * interior * 2);
  return PPRS_OK;
}

// ------------------------------------------------------------------------------------------
// Weights-only blob (safetensors layout): u64 little-endian header length, a JSON object
// {"name": {"dtype": ..., "shape": [...], "data_offsets": [begin, end]}, "__metadata__": {...}},
// then the tensor bytes. A small recursive-descent reader of that JSON: it accepts objects,
// arrays, strings, numbers and literals, records each top-level tensor's fields and skips
// everything else. Nothing in the blob is interpreted beyond these fields.

namespace {

struct BlobTensor {
  std::string name, dtype;
  std::vector<long long> shape;
  long long begin = -1, end = -1;
};

struct JsonReader {
  const char* p;
  const char* e;
  int depth = 0;
  bool ok = true;
  void ws() {
    while (p < e && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool eat(char ch) {
    ws();
    if (p < e && *p == ch) {
      ++p;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (p >= e || *p != '"') return ok = false;
    ++p;
    std::string r;
    while (p < e && *p != '"') {
      if (*p == '\\') {
        if (++p >= e) return ok = false;
        char c = *p;
        if (c == 'u') {  // keep the escape's text; names here are plain ASCII
          if (e - p < 5) return ok = false;
          r.append(p - 1, 6);
          p += 5;
          continue;
        }
        r.push_back(c == 'n' ? '\n' : c == 't' ? '\t' : c == 'r' ? '\r' : c == 'b' ? '\b'
                    : c == 'f' ? '\f' : c);
        ++p;
        continue;
      }
      r.push_back(*p++);
    }
    if (p >= e) return ok = false;
    ++p;
    if (out) *out = r;
    return true;
  }
  bool integer(long long* out) {
    ws();
    const char* q = p;
    bool neg = false;
    if (q < e && *q == '-') neg = true, ++q;
    if (q >= e || *q < '0' || *q > '9') return ok = false;
    long long v = 0;
    while (q < e && *q >= '0' && *q <= '9') {
      if (v > (1LL << 50)) return ok = false;
      v = v * 10 + (*q++ - '0');
    }
    if (q < e && (*q == '.' || *q == 'e' || *q == 'E')) return ok = false;
    p = q;
    *out = neg ? -v : v;
    return true;
  }
  bool skip() {  // any value
    ws();
    if (p >= e || ++depth > 64) return ok = false;
    bool r = true;
    if (*p == '"') {
      r = str(nullptr);
    } else if (*p == '{') {
      ++p;
      if (!eat('}')) {
        do {
          r = str(nullptr) && eat(':') && skip();
        } while (r && eat(','));
        r = r && eat('}');
      }
    } else if (*p == '[') {
      ++p;
      if (!eat(']')) {
        do {
          r = skip();
        } while (r && eat(','));
        r = r && eat(']');
      }
    } else {
      const char* q = p;
      while (q < e && (isalnum((unsigned char)*q) || *q == '-' || *q == '+' || *q == '.')) ++q;
      r = q > p;
      p = q;
    }
    --depth;
    if (!r) ok = false;
    return r;
  }
  bool int_list(std::vector<long long>* out) {
    if (!eat('[')) return ok = false;
    out->clear();
    if (eat(']')) return true;
    do {
      long long v;
      if (!integer(&v)) return false;
      out->push_back(v);
    } while (eat(','));
    return eat(']') || (ok = false);
  }
  bool tensor(BlobTensor* t) {
    if (!eat('{')) return ok = false;
    if (eat('}')) return true;
    do {
      std::string key;
      if (!str(&key) || !eat(':')) return ok = false;
      if (key == "dtype") {
        if (!str(&t->dtype)) return false;
      } else if (key == "shape") {
        if (!int_list(&t->shape)) return false;
      } else if (key == "data_offsets") {
        std::vector<long long> o;
        if (!int_list(&o) || o.size() != 2) return ok = false;
        t->begin = o[0];
        t->end = o[1];
      } else if (!skip()) {
        return false;
      }
    } while (eat(','));
    return eat('}') || (ok = false);
  }
};

bool parse_blob_header(const char* h, size_t n, std::vector<BlobTensor>& out) {
  JsonReader r{h, h + n};
  if (!r.eat('{')) return false;
  if (r.eat('}')) return true;
  do {
    std::string key;
    if (!r.str(&key) || !r.eat(':')) return false;
    if (key == "__metadata__") {
      if (!r.skip()) return false;
      continue;
    }
    BlobTensor t;
    t.name = key;
    if (!r.tensor(&t)) return false;
    out.push_back(t);
  } while (r.eat(','));
  return r.eat('}') && r.ok;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// C-ABI

extern "C" {

const char* pprs_cnn_last_error(void) { return g_cnn_err.c_str(); }

pprs_status pprs_cnn_create(pprs_cnn** out, int device, void* stream, unsigned long long seed) {
  if (!out) return cfail(PPRS_EINVAL, "out is NULL");
  *out = nullptr;
  CHK(hipSetDevice(device));
  pprs_cnn* c = new pprs_cnn();
  Model& M = c->M;
  M.device = device;
  M.stream = (hipStream_t)stream;
  define_layers(M);
  // He-normal initialisation from a counter-based hash (SplitMix64) of (seed, index)
  std::vector<float> hw(M.n_params, 0.f);
  auto mix = [](unsigned long long x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
  };
  for (int l = 0; l < 6; ++l) {
    const Layer& y = M.L[l];
    int k = 9 * y.cin;
    double sd = sqrt(2.0 / k) * (l == 5 ? 0.1 : 1.0);
    for (int co = 0; co < y.cout; ++co)
      for (int j = 0; j < k; ++j) {
        long long i = y.woff + (long long)co * y.kp + j;
        unsigned long long r1 = mix(seed * 0x100000001B3ULL + 2 * (unsigned long long)i);
        unsigned long long r2 = mix(seed * 0x100000001B3ULL + 2 * (unsigned long long)i + 1);
        double u1 = ((r1 >> 11) + 0.5) / 9007199254740992.0, u2 = (r2 >> 11) / 9007199254740992.0;
        hw[i] = (float)(sd * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
      }
  }
  hipError_t e = hipSuccess;
  e = hipMalloc(&M.w, sizeof(float) * M.n_params);
  if (e == hipSuccess) e = hipMalloc(&M.m, sizeof(float) * M.n_params);
  if (e == hipSuccess) e = hipMalloc(&M.v, sizeof(float) * M.n_params);
  if (e == hipSuccess) e = hipMalloc(&M.g, sizeof(float) * M.n_params);
  if (e == hipSuccess) e = hipMalloc(&M.wb, sizeof(bf16) * M.n_params);
  if (e == hipSuccess) e = hipMalloc(&M.w6, sizeof(float) * M.L[5].cout * M.L[5].kp);
  if (e == hipSuccess) e = hipMalloc(&M.w6f, sizeof(float) * 4 * 2 * 2 * 2 * 64);
  for (int l = 3; l < 5 && e == hipSuccess; ++l) {
    const int c0 = l == 3 ? 256 : 128, c1 = M.L[l].cin - c0;
    e = hipMalloc(&M.wfold[l - 3], sizeof(bf16) * 4 * M.L[l].cout * (4 * c0 + 9 * c1));
  }
  if (e != hipSuccess) {
    delete c;
    return cfail(PPRS_ENOMEM, "cnn allocation failed");
  }
  *out = c;
  pprs_status s = pprs_cnn_set_params(c, hw.data(), (size_t)M.n_params);
  return s;
}

void pprs_cnn_destroy(pprs_cnn* c) {
  if (!c) return;
  Model& M = c->M;
  (void)hipSetDevice(M.device);
  (void)hipStreamSynchronize(M.stream);
  void* ptrs[] = {M.w, M.m, M.v, M.g, M.wb, M.w6, M.w6f, M.wfold[0], M.wfold[1], M.x0, M.a[0],
                  M.a[1], M.a[2], M.a[3],
                  M.a[4], M.u4, M.u5, M.col, M.dzb, M.z, M.y, M.dy, M.dcol, M.du, M.da[0],
                  M.da[1], M.da[2], M.da[3], M.da[4], M.part, M.lpart, M.wflip};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

size_t pprs_cnn_param_count(const pprs_cnn* c) { return c ? (size_t)c->M.n_params : 0; }

pprs_status pprs_cnn_set_params(pprs_cnn* c, const float* host, size_t count) {
  if (!c || !host) return cfail(PPRS_EINVAL, "NULL argument");
  Model& M = c->M;
  if (count != (size_t)M.n_params) return cfail(PPRS_EINVAL, "expected %lld parameters", M.n_params);
  CHK(hipSetDevice(M.device));
  CHK(hipMemcpyAsync(M.w, host, sizeof(float) * count, hipMemcpyHostToDevice, M.stream));
  CHK(hipMemsetAsync(M.m, 0, sizeof(float) * count, M.stream));
  CHK(hipMemsetAsync(M.v, 0, sizeof(float) * count, M.stream));
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid1d(count)), dim3(kBlock), 0, M.stream, M.w, (long long)count, M.wb);
  CHK(hipGetLastError());
  M.step = 0;
  return refresh_derived(M);
}

pprs_status pprs_cnn_load(pprs_cnn* c, const void* blob, size_t bytes) {
  if (!c || !blob) return cfail(PPRS_EINVAL, "NULL argument");
  const unsigned char* b = (const unsigned char*)blob;
  if (bytes < 8) return cfail(PPRS_EINVAL, "blob shorter than its 8-byte header length");
  unsigned long long hl = 0;
  for (int k = 7; k >= 0; --k) hl = (hl << 8) | b[k];
  if (hl < 2 || hl > bytes - 8) return cfail(PPRS_EINVAL, "header length %llu outside the blob", hl);
  std::vector<BlobTensor> ts;
  if (!parse_blob_header((const char*)b + 8, (size_t)hl, ts))
    return cfail(PPRS_EINVAL, "malformed blob header");
  const BlobTensor* t = nullptr;
  for (const BlobTensor& x : ts)
    if (x.name == "params") t = &x;
  if (!t && ts.size() == 1) t = &ts[0];
  if (!t) return cfail(PPRS_EINVAL, "blob holds no tensor named \"params\"");
  if (t->dtype != "F32") return cfail(PPRS_EINVAL, "tensor dtype %s, expected F32", t->dtype.c_str());
  long long count = 1;
  for (long long d : t->shape) {
    if (d < 0 || d > (1LL << 40)) return cfail(PPRS_EINVAL, "bad tensor shape");
    count *= d;
  }
  Model& M = c->M;
  if (count != M.n_params)
    return cfail(PPRS_EINVAL, "blob holds %lld parameters, the network %lld", count, M.n_params);
  size_t data = 8 + (size_t)hl, avail = bytes - data;
  if (t->begin < 0 || t->end < t->begin || (unsigned long long)t->end > avail ||
      t->end - t->begin != 4 * count)
    return cfail(PPRS_EINVAL, "tensor byte range outside the blob");
  std::vector<float> host((size_t)count);  // aligned copy: the data need not be aligned
  memcpy(host.data(), b + data + t->begin, sizeof(float) * (size_t)count);
  pprs_status s = pprs_cnn_set_params(c, host.data(), (size_t)count);
  if (s != PPRS_OK) return s;
  CHK(hipStreamSynchronize(M.stream));  // the host copy must outlive the upload
  return PPRS_OK;
}

pprs_status pprs_cnn_get_params(pprs_cnn* c, float* host, size_t count) {
  if (!c || !host) return cfail(PPRS_EINVAL, "NULL argument");
  Model& M = c->M;
  if (count != (size_t)M.n_params) return cfail(PPRS_EINVAL, "expected %lld parameters", M.n_params);
  CHK(hipSetDevice(M.device));
  CHK(hipMemcpyAsync(host, M.w, sizeof(float) * count, hipMemcpyDeviceToHost, M.stream));
  CHK(hipStreamSynchronize(M.stream));
  return PPRS_OK;
}

pprs_status pprs_cnn_forward(pprs_cnn* c, const float* x, int B, float* y) {
  if (!c || !x || !y || B < 1) return cfail(PPRS_EINVAL, "bad arguments");
  Model& M = c->M;
  CHK(hipSetDevice(M.device));
  pprs_status s = alloc_batch(M, B);
  if (s != PPRS_OK) return s;
  s = forward(M, x, B, false);
  if (s != PPRS_OK) return s;
  CHK(hipMemcpyAsync(y, M.y, sizeof(float) * (size_t)B * 128 * 128 * 2, hipMemcpyDeviceToDevice, M.stream));
  CHK(hipStreamSynchronize(M.stream));
  return PPRS_OK;
}

pprs_status pprs_cnn_gradients(pprs_cnn* c, const float* x, const float* target, int B,
                               int margin, double* loss, float* grad_host) {
  if (!c || !x || !target || B < 1 || margin < 0 || margin >= 64)
    return cfail(PPRS_EINVAL, "bad arguments");
  Model& M = c->M;
  CHK(hipSetDevice(M.device));
  pprs_status s = alloc_batch(M, B);
  if (s != PPRS_OK) return s;
  if ((s = forward(M, x, B, true)) != PPRS_OK) return s;
  if ((s = backward(M, target, B, margin, loss)) != PPRS_OK) return s;
  if (grad_host) {
    CHK(hipMemcpyAsync(grad_host, M.g, sizeof(float) * M.n_params, hipMemcpyDeviceToHost, M.stream));
    CHK(hipStreamSynchronize(M.stream));
  }
  return PPRS_OK;
}

pprs_status pprs_cnn_train_step(pprs_cnn* c, const float* x, const float* target, int B,
                                int margin, float lr, double* loss) {
  pprs_status s = pprs_cnn_gradients(c, x, target, B, margin, loss, nullptr);
  if (s != PPRS_OK) return s;
  Model& M = c->M;
  M.step++;
  const float b1 = 0.9f, b2 = 0.999f;
  float c1 = 1.f - powf(b1, (float)M.step), c2 = 1.f - powf(b2, (float)M.step);
  hipLaunchKernelGGL(k_adam, dim3(grid1d(M.n_params)), dim3(kBlock), 0, M.stream, M.w, M.m, M.v, M.g, M.n_params, lr, b1, b2, 1e-8f, c1, c2, M.wb);
  CHK(hipGetLastError());
  return refresh_derived(M);
}

}  // extern "C"

// Used by the runtime: pack pairs of level-7 frames and run the network.
namespace pprs_cnn_api {
hipError_t pack_pairs(const float* lvl, int n, const int* ref, const int* tmpl, int P,
                      float* out, hipStream_t st) {
  long long work = (long long)P * (n - 1) * (n - 1);
  hipLaunchKernelGGL(k_pack_pairs, dim3(grid1d(work)), dim3(kBlock), 0, st, lvl, n, ref, tmpl, P, out);
  return hipGetLastError();
}
pprs_status forward_into(pprs_cnn* c, const float* x, int B, float* y) {
  return pprs_cnn_forward(c, x, B, y);
}
hipError_t planes_to_nhwc(const float* src, int n, long long pstride, int P, float scale,
                          float* out, hipStream_t st) {
  long long work = (long long)P * (n - 1) * (n - 1);
  hipLaunchKernelGGL(k_planes_to_nhwc, dim3(grid1d(work)), dim3(kBlock), 0, st, src, n, pstride, P, scale, out);
  return hipGetLastError();
}
hipError_t nhwc_to_planes(const float* y, int S, int P, float scale, float* base,
                          long long stride, hipStream_t st) {
  long long work = (long long)P * (S + 1) * (S + 1);
  hipLaunchKernelGGL(k_nhwc_to_planes, dim3(grid1d(work)), dim3(kBlock), 0, st, y, S, P, scale, base, stride);
  return hipGetLastError();
}
int cnn_device(const pprs_cnn* c) { return c->M.device; }
hipError_t check_pred(const float* y, int P, long long n_per, float limit, int* bad,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_check_pred, dim3(P), dim3(kBlock), 0, st, y, n_per, limit, bad);
  return hipGetLastError();
}
}  // namespace pprs_cnn_api
