// fd_mlp.hip -- direction-proposal network on gfx950 matrix cores.
//
// 112 -> 256 -> 256 -> 256 -> 3, GELU (tanh form, Hendrycks & Gimpel 2016)
// after the hidden layers, output normalised to a unit direction.  Weights
// have a float master copy (Adam state beside it) and bfloat16 copies laid
// out for v_mfma_f32_16x16x32_bf16; activations are bfloat16, accumulation
// float.
//
// MFMA 16x16x32 operand layout used here (lane l of 64, g = l / 16):
//   A (16 x 32, row-major source): lane holds A[l % 16][8g .. 8g + 7]
//   B (32 x 16):                   lane holds B[8g .. 8g + 7][l % 16]
//   D (16 x 16 float):             lane holds D[4g + r][l % 16], r = 0..3
// A and B use the same k assignment, so the sum over k is the full product.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <utility>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_kernels.hpp"

using namespace fd;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int D0 = 112, D0P = 128, DH = 256, DO = 3, DOP = 16;
// flat parameter offsets (W[k][n] row-major, then bias)
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + D0 * DH;
constexpr int OFF_W2 = OFF_B1 + DH, OFF_B2 = OFF_W2 + DH * DH;
constexpr int OFF_W3 = OFF_B2 + DH, OFF_B3 = OFF_W3 + DH * DH;
constexpr int OFF_W4 = OFF_B3 + DH, OFF_B4 = OFF_W4 + DH * DO;
constexpr int N_PARAMS = OFF_B4 + DO;
static_assert(N_PARAMS == FD_MLP_N_PARAMS, "parameter count");

__device__ __forceinline__ uint16_t f2bf(float x) {
  return __bfloat16_as_ushort(__float2bfloat16(x));  // round to nearest even
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// two floats -> bfloat16 pair (round to nearest even), a in the low half;
// a vector conversion, which gfx950 does in one instruction
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const bf16x2_t v = __builtin_convertvector((f32x2_t){a, b}, bf16x2_t);
  return __builtin_bit_cast(uint32_t, v);
}

// tanh-form GELU: 0.5 x (1 + tanh(u)) = x / (1 + exp(-2u)),
// u = sqrt(2/pi) (x + 0.044715 x^3)
__device__ __forceinline__ float gelu(float x) {
  const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
  return x / (1.0f + __expf(-2.0f * u));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float c = 0.7978845608028654f;
  const float u = c * (x + 0.044715f * x * x * x);
  const float th = tanhf(u);
  const float du = c * (1.0f + 3.0f * 0.044715f * x * x);
  return 0.5f * (1.0f + th) + 0.5f * x * (1.0f - th * th) * du;
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---- packing: float master -> bfloat16 matrix-core layouts ------------------------
// Wt[n][k] (k contiguous) for every layer; k of layer 1 padded to 128 and n of
// layer 4 padded to 16 with zeros; biases copied to float arrays (b4 padded).
struct Packed {
  uint16_t* w1t;  // DH x D0P
  uint16_t* w2t;  // DH x DH
  uint16_t* w3t;  // DH x DH
  uint16_t* w4t;  // DOP x DH
  float* bias;    // b1 | b2 | b3 | b4(16)
};

__global__ void k_mlp_pack(const float* __restrict__ m, Packed p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < DH * D0P) {  // layer 1
    const int n = i / D0P, k = i % D0P;
    p.w1t[i] = k < D0 ? f2bf(m[OFF_W1 + k * DH + n]) : 0;
  }
  if (i < DH * DH) {
    const int n = i / DH, k = i % DH;
    p.w2t[i] = f2bf(m[OFF_W2 + k * DH + n]);
    p.w3t[i] = f2bf(m[OFF_W3 + k * DH + n]);
  }
  if (i < DOP * DH) {
    const int n = i / DH, k = i % DH;
    p.w4t[i] = n < DO ? f2bf(m[OFF_W4 + k * DO + n]) : 0;
  }
  if (i < DH) {
    p.bias[i] = m[OFF_B1 + i];
    p.bias[DH + i] = m[OFF_B2 + i];
    p.bias[2 * DH + i] = m[OFF_B3 + i];
  }
  if (i < DOP) p.bias[3 * DH + i] = i < DO ? m[OFF_B4 + i] : 0.0f;
}

// ---- inference: fused four-layer forward ----------------------------------------------
// One workgroup = 128 rows.  Activations stay in LDS (128 x 256 bfloat16,
// rows padded by 16 bytes); wave w produces output columns
// [kCols w, kCols (w + 1)) of every hidden layer for all 128 rows.  The product is
// issued as Z^T = W^T X^T (weights as the A operand, activations as B), so
// that each lane ends up holding four consecutive output columns of one row
// and writes them to LDS with one 8-byte store.  Weight fragments come
// straight from the L2-resident packed weights, one k-step ahead.
constexpr int FWD_ROWS = 128;
constexpr int ACT_LD = DH + 8;
// FD_MLP_FWD_WAVES waves per workgroup, each producing kCols output columns
// of every hidden layer (kNt 16-column MFMA tiles) for all 128 rows; the
// output layer gives each wave 128 / (16 kFwdWaves) 16-row tiles.  Eight
// waves (two column tiles each) measure faster than four (four each, half
// the LDS reads per product): 0.49 against 0.53 ms per 1M rows.  The weight
// fragment loads, not the LDS reads, set the pace: splitting the rows
// between two wave groups (half the LDS reads, twice the weight loads per
// product) measured 1.65 against 0.97 ms per 2M rows, loading the weights
// two k-steps ahead instead of one 1.16 against 1.05 ms, and 256-row
// workgroups (half the weight loads per row, one workgroup per CU) 1.19;
// the GELU epilogue costs about 0.15 ms of the 1.05.
#ifndef FD_MLP_FWD_WAVES
#define FD_MLP_FWD_WAVES 8
#endif
constexpr int kFwdWaves = FD_MLP_FWD_WAVES;
constexpr int kFwdThreads = 64 * kFwdWaves;
constexpr int kCols = DH / kFwdWaves;
constexpr int kNt = kCols / 16;
constexpr int kOutTiles = FWD_ROWS / (16 * kFwdWaves);
static_assert(FWD_ROWS % (16 * kFwdWaves) == 0, "whole output-layer row tiles per wave");

// GELU (tanh form) for the inference forward: 0.5 x (1 + tanh(u)) = x / (1 +
// e^(-2u)), u = sqrt(2/pi) (x + 0.044715 x^3), with e^(-2u) = 2^(x (A + B x^2))
// so the constants fold into one multiply-add; hardware exp2 and reciprocal
// (about 1 ulp each, below the bfloat16 rounding that follows).
__device__ __forceinline__ float gelu_fast(float x) {
  constexpr float kA = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
  constexpr float kB = kA * 0.044715f;
  const float t = x * __builtin_fmaf(kB, x * x, kA);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

__global__ __launch_bounds__(kFwdThreads, 2) void k_mlp_fwd(const uint16_t* __restrict__ x,
                                                          int64_t n, Packed p,
                                                          float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t act[FWD_ROWS * ACT_LD];
  __shared__ float yout[FWD_ROWS][4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * FWD_ROWS;

  // input rows -> act[:, 0:128) (k >= 112 and rows >= n zero)
  for (int e = t; e < FWD_ROWS * (D0P / 8); e += kFwdThreads) {
    const int r = e / (D0P / 8), kb = (e % (D0P / 8)) * 8;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (row0 + r < n && kb < D0) v = *(const uint4*)(x + (row0 + r) * D0 + kb);
    *(uint4*)(act + r * ACT_LD + kb) = v;
  }
  __syncthreads();

#pragma unroll 1
  for (int layer = 0; layer < 3; ++layer) {
    const int K = layer == 0 ? D0P : DH;
    const uint16_t* wt = layer == 0 ? p.w1t : (layer == 1 ? p.w2t : p.w3t);
    // acc[mt][nt]: rows (output columns) kCols w + 16nt + 4g + r, column
    // (batch row) 16mt + c16
    f32x4 acc[8][kNt];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
      for (int nt = 0; nt < kNt; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 wa[kNt], wn[kNt];
#pragma unroll
    for (int nt = 0; nt < kNt; ++nt)
      wa[nt] = *(const bf16x8*)(wt + (size_t)(kCols * w + 16 * nt + c16) * K + 8 * g);
#pragma unroll 1
    for (int kc = 0; kc < K; kc += 32) {
      const int kn = kc + 32 < K ? kc + 32 : kc;
#pragma unroll
      for (int nt = 0; nt < kNt; ++nt)
        wn[nt] = *(const bf16x8*)(wt + (size_t)(kCols * w + 16 * nt + c16) * K + kn + 8 * g);
#pragma unroll
      for (int mt = 0; mt < 8; ++mt) {
        const bf16x8 xb = *(const bf16x8*)(act + (16 * mt + c16) * ACT_LD + kc + 8 * g);
#pragma unroll
        for (int nt = 0; nt < kNt; ++nt) acc[mt][nt] = mfma(wa[nt], xb, acc[mt][nt]);
      }
#pragma unroll
      for (int nt = 0; nt < kNt; ++nt) wa[nt] = wn[nt];
    }
    __syncthreads();  // every wave has read this layer's input
    const float* bias = p.bias + layer * DH;
#pragma unroll
    for (int nt = 0; nt < kNt; ++nt) {
      const int col = kCols * w + 16 * nt + 4 * g;
      const float4 bb = *(const float4*)(bias + col);
#pragma unroll
      for (int mt = 0; mt < 8; ++mt) {
        const int row = 16 * mt + c16;
        const uint32_t lo = pack_bf16x2(gelu_fast(acc[mt][nt][0] + bb.x),
                                        gelu_fast(acc[mt][nt][1] + bb.y));
        const uint32_t hi = pack_bf16x2(gelu_fast(acc[mt][nt][2] + bb.z),
                                        gelu_fast(acc[mt][nt][3] + bb.w));
        *(uint2*)(act + row * ACT_LD + col) = make_uint2(lo, hi);
      }
    }
    __syncthreads();
  }
  // output layer: 256 -> 16 (3 real); wave w takes batch-row tiles
  // w, w + kFwdWaves, ...
#pragma unroll
  for (int ot = 0; ot < kOutTiles; ++ot) {
    const int rt = w + ot * kFwdWaves;
    f32x4 o = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kc = 0; kc < DH; kc += 32) {
      const bf16x8 b = *(const bf16x8*)(p.w4t + (size_t)c16 * DH + kc + 8 * g);
      const bf16x8 a = *(const bf16x8*)(act + (16 * rt + c16) * ACT_LD + kc + 8 * g);
      o = mfma(a, b, o);
    }
    if (c16 < 3) {
#pragma unroll
      for (int r = 0; r < 4; ++r) yout[16 * rt + 4 * g + r][c16] = o[r] + p.bias[3 * DH + c16];
    }
  }
  __syncthreads();
  if (t < FWD_ROWS && row0 + t < n) {
    const float y0 = yout[t][0], y1 = yout[t][1], y2 = yout[t][2];
    const float inv = 1.0f / sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
    float* o3 = out + 3 * (row0 + t);
    o3[0] = y0 * inv;
    o3[1] = y1 * inv;
    o3[2] = y2 * inv;
  }
}

// ---- training: generic bfloat16 matrix product and elementwise kernels -------------
// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = a[m * sam + k * sak],
// B(k, n) = b[k * sbk + n * sbn], each operand contiguous along k (sak = 1,
// sbk = 1) or along m / n (sam = 1, sbn = 1); N % 64 == 0, K % 32 == 0 (per
// K slice), rows m >= M read as zero.  Columns >= n_real and rows >=
// m_real are not stored.  k in ascending order per slice: deterministic.
// Epilogue:
//   EPI_STORE      c[m * ldc + n] = acc
//   EPI_BIAS_GELU  z = acc + bias[n]; zf[m*ldc+n] = z; h[m*ldh+n] = bf16(gelu(z))
//   EPI_GELU_BACK  d = acc * gelu'(zf[m*ldc+n]); dq[m*ldh+n] = bf16(d); df[tile][n] =
//                  sum of d over the tile's rows (the next bias gradient's partials)
enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_BACK = 2 };

struct GemmArgs {
  const uint16_t* a;
  int64_t sam, sak;
  const uint16_t* b;
  int64_t sbk, sbn;
  int M, N, K, m_real, n_real;
  int epi;
  float* c;  // EPI_STORE: output; EPI_BIAS_GELU: z out; EPI_GELU_BACK: z in
  int64_t ldc;
  const float* bias;
  float* df;     // EPI_GELU_BACK: per 64-row tile column sums of the gradient (tiles x N)
  uint16_t* hq;  // bf16 out
  int64_t ldh;
  int ksplit;    // > 1: K in ksplit slices, fp32 partial tiles to part (EPI_STORE only)
  float* part;   // ksplit x M x N
};

// Workgroup tile 64 x 64 (four waves; wave w takes output columns
// [16w, 16w + 16) of all 64 rows: four 16 x 16 MFMA tiles).  K is taken in
// stages of up to kGemmKS: every global load of a stage is issued first
// (16 bytes per thread and 32-k step), then stored to LDS with k contiguous
// (rows padded by 8 elements) — a k-contiguous operand as it is, an m- or
// n-contiguous one transposed with 2-byte stores — and after one barrier
// the products of the whole stage run from LDS.
constexpr int kGemmT = 64, kGemmK = 32, kGemmKS = 256, kGemmLd = kGemmKS + 8;

// Operand staging registers as a native vector type (the uint4 struct
// copied between an array and LDS made the compiler keep the array in
// private memory).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool AK, bool BK>
__device__ __forceinline__ void gemm_load_step(const GemmArgs& g, int m0, int n0, int k0, int t,
                                               u32x4& va, u32x4& vb) {
  if (AK) {  // thread t: row t / 4, k 8 (t % 4) .. + 7
    const int r = t >> 2, kq = (t & 3) * 8;
    va = m0 + r < g.M ? *(const u32x4*)(g.a + (int64_t)(m0 + r) * g.sam + k0 + kq)
                      : u32x4{0u, 0u, 0u, 0u};
  } else {   // thread t: k t / 8, rows 8 (t % 8) .. + 7 (M is a multiple of 64 here)
    const int k = t >> 3, mq = (t & 7) * 8;
    va = *(const u32x4*)(g.a + (int64_t)(k0 + k) * g.sak + m0 + mq);
  }
  if (BK) {
    const int r = t >> 2, kq = (t & 3) * 8;
    vb = *(const u32x4*)(g.b + (int64_t)(n0 + r) * g.sbn + k0 + kq);
  } else {
    const int k = t >> 3, nq = (t & 7) * 8;
    vb = *(const u32x4*)(g.b + (int64_t)(k0 + k) * g.sbk + n0 + nq);
  }
}

template <bool AK, bool BK>
__device__ __forceinline__ void gemm_store_step(uint16_t (*As)[kGemmLd], uint16_t (*Bs)[kGemmLd],
                                                int kk, int t, const u32x4& va, const u32x4& vb) {
  if (AK) {
    *(u32x4*)&As[t >> 2][kk + (t & 3) * 8] = va;
  } else {
    const int k = t >> 3, mq = (t & 7) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) As[mq + j][kk + k] = (uint16_t)(va[j >> 1] >> (16 * (j & 1)));
  }
  if (BK) {
    *(u32x4*)&Bs[t >> 2][kk + (t & 3) * 8] = vb;
  } else {
    const int k = t >> 3, nq = (t & 7) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) Bs[nq + j][kk + k] = (uint16_t)(vb[j >> 1] >> (16 * (j & 1)));
  }
}

// Column sums over the tile's 64 rows of the values v[mt][r] (row
// 16 mt + 4 gr + r, column c16 of the wave's 16): rows in order within a
// lane, then the four row groups gr in order (the same for every tile).
__device__ __forceinline__ float gemm_colsum(const float (&v)[4][4], int lane) {
  float s = 0.0f;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += v[mt][r];
  // lanes c16, c16 + 16, c16 + 32, c16 + 48 hold row groups 0..3
  const float s1 = __shfl(s, (lane & 15) + 16, 64), s2 = __shfl(s, (lane & 15) + 32, 64),
              s3 = __shfl(s, (lane & 15) + 48, 64), s0 = __shfl(s, lane & 15, 64);
  return ((s0 + s1) + s2) + s3;
}

template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGemmT][kGemmLd];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGemmT][kGemmLd];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, gr = lane >> 4, c16 = lane & 15;
  const int m0 = blockIdx.x * kGemmT, n0 = blockIdx.y * kGemmT;
  f32x4 acc[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) acc[mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int kslice = g.K / g.ksplit;
  const int kz0 = blockIdx.z * kslice, kz1 = kz0 + kslice;
  for (int ks = kz0; ks < kz1; ks += kGemmKS) {
    const int kn = min(kGemmKS, kz1 - ks);  // a multiple of 32
    u32x4 va[kGemmKS / kGemmK], vb[kGemmKS / kGemmK];
#pragma unroll
    for (int q = 0; q < kGemmKS / kGemmK; ++q)
      if (q * kGemmK < kn) gemm_load_step<AK, BK>(g, m0, n0, ks + q * kGemmK, t, va[q], vb[q]);
    if (ks > kz0) __syncthreads();  // the previous stage's products are done
#pragma unroll
    for (int q = 0; q < kGemmKS / kGemmK; ++q)
      if (q * kGemmK < kn) gemm_store_step<AK, BK>(As, Bs, q * kGemmK, t, va[q], vb[q]);
    __syncthreads();
#pragma unroll 2
    for (int kk = 0; kk < kn; kk += kGemmK) {
      const bf16x8 b = *(const bf16x8*)&Bs[16 * w + c16][kk + 8 * gr];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 a = *(const bf16x8*)&As[16 * mt + c16][kk + 8 * gr];
        acc[mt] = mfma(a, b, acc[mt]);
      }
    }
  }
  // acc[mt] holds D[4 gr + r][c16] of the tile (rows 16 mt + ..., columns 16 w + ...)
  const int n = n0 + 16 * w + c16;
  if (g.ksplit > 1) {  // partial tile of this K slice; k_gemm_reduce finishes
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * mt + 4 * gr + r;
        if (m < g.M) g.part[((size_t)blockIdx.z * g.M + m) * g.N + n] = acc[mt][r];
      }
    return;
  }
  float dsum[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + 16 * mt + 4 * gr + r;
      dsum[mt][r] = 0.0f;
      if (m >= g.m_real || m >= g.M || n >= g.n_real) continue;
      const float v = acc[mt][r];
      if (g.epi == EPI_STORE) {
        g.c[m * g.ldc + n] = v;
      } else if (g.epi == EPI_BIAS_GELU) {
        const float z = v + g.bias[n];
        g.c[m * g.ldc + n] = z;
        g.hq[m * g.ldh + n] = f2bf(gelu(z));
      } else {
        const float d = v * gelu_grad(g.c[m * g.ldc + n]);
        dsum[mt][r] = d;
        g.hq[m * g.ldh + n] = f2bf(d);
      }
    }
  }
  if (g.epi == EPI_GELU_BACK) {
    // the bias gradient's partial over this tile's rows (float d), for
    // k_col_finish to sum over the row tiles in order
    const float cs = gemm_colsum(dsum, lane);
    if (gr == 0) g.df[(size_t)blockIdx.x * g.N + n] = cs;
  }
}

// The K slices of a split GEMM summed in slice order (deterministic), stored.
__global__ void k_gemm_reduce(const float* __restrict__ part, int S, int M, int N, int m_real,
                              int n_real, float* __restrict__ c, int64_t ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  const int m = i / N, n = i % N;
  if (m >= m_real || n >= n_real) return;
  float v = 0.0f;
  for (int z = 0; z < S; ++z) v += part[((size_t)z * M + m) * N + n];
  c[m * ldc + n] = v;
}

// feats (B x 112 bf16) -> X (B x 128 bf16, zero padded)
__global__ void k_pad_input(const uint16_t* __restrict__ f, int B, uint16_t* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * D0P) return;
  const int r = i / D0P, k = i % D0P;
  x[i] = k < D0 ? f[r * D0 + k] : 0;
}

// Output layer forward + loss + its gradient, eight lanes per row (lane j
// takes k in [32 j, 32 j + 32) in order; the eight partial sums are added
// by a fixed shuffle tree):
// y = h3 W4 + b4 (float, W4 as bfloat16 values), u = y/|y|, loss_b = 1 - (u.t)^2,
// dL/dy = (g - u (u.g)) / |y| with g = -2 (u.t) t / B.
constexpr int kOutLanes = 8;
__global__ __launch_bounds__(256) void k_out_loss(const uint16_t* __restrict__ h3,
                                                  const uint16_t* __restrict__ w4t,
                                                  const float* __restrict__ bias4,
                                                  const float* __restrict__ tgt, int B,
                                                  float* __restrict__ dy,
                                                  float* __restrict__ loss_row) {
  const int b = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kOutLanes);
  const int j = (int)(threadIdx.x % kOutLanes);
  const int bb = b < B ? b : B - 1;  // every lane takes part in the shuffles
  float part[3] = {0.0f, 0.0f, 0.0f};
  const int k0 = j * (DH / kOutLanes);
#pragma unroll
  for (int q = 0; q < DH / kOutLanes; q += 8) {
    const uint4 hv = *(const uint4*)(h3 + (size_t)bb * DH + k0 + q);
    const uint32_t hw[4] = {hv.x, hv.y, hv.z, hv.w};
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const uint4 wv = *(const uint4*)(w4t + n * DH + k0 + q);
      const uint32_t ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint16_t he = (uint16_t)(hw[e >> 1] >> (16 * (e & 1)));
        const uint16_t we = (uint16_t)(ww[e >> 1] >> (16 * (e & 1)));
        part[n] += bf2f(he) * bf2f(we);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int off = 1; off < kOutLanes; off <<= 1) part[n] += __shfl_xor(part[n], off, 64);
  if (j != 0 || b >= B) return;
  float y[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) y[n] = part[n] + bias4[n];
  const float nrm = sqrtf(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
  float u[3], t[3], ut = 0.0f;
  for (int n = 0; n < 3; ++n) {
    u[n] = y[n] / nrm;
    t[n] = tgt[3 * b + n];
    ut += u[n] * t[n];
  }
  loss_row[b] = 1.0f - ut * ut;
  float gg[3], ug = 0.0f;
  for (int n = 0; n < 3; ++n) {
    gg[n] = -2.0f * ut * t[n] / (float)B;
    ug += u[n] * gg[n];
  }
  for (int n = 0; n < 3; ++n) dy[3 * b + n] = (gg[n] - u[n] * ug) / nrm;
}

// Output-layer weight gradient (float): dW4[k][n] = sum_b h3[b][k] dy[b][n],
// db4[n] = sum_b dy[b][n].  Deterministic two-pass form: thread i of chunk c
// sums the kRowChunk rows of its chunk in order (k_outw_partial), then each
// entry sums its chunk partials in a fixed order (k_col_finish).
constexpr int kRowChunk = 32;
constexpr int kMaxSplit = 16;  // K slices of a weight-gradient GEMM
constexpr int kOutGrad = DH * DO + DO;  // dW4 then db4, contiguous in the parameters

__global__ void k_outw_partial(const uint16_t* __restrict__ h3, const float* __restrict__ dy,
                               int B, float* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= kOutGrad) return;
  const int b0 = c * kRowChunk, b1 = min(B, b0 + kRowChunk);
  float s = 0.0f;
  if (i < DH * DO) {
    const int k = i / DO, n = i % DO;
    for (int b = b0; b < b1; ++b) s += bf2f(h3[b * DH + k]) * dy[3 * b + n];
  } else {
    const int n = i - DH * DO;
    for (int b = b0; b < b1; ++b) s += dy[3 * b + n];
  }
  part[(size_t)c * kOutGrad + i] = s;
}

// dz3 = (dy W4^T) * gelu'(z3) (W4 as bfloat16 values); float and bfloat16 copies.
__global__ void k_out_back(const float* __restrict__ dy, const uint16_t* __restrict__ w4t,
                           const float* __restrict__ z3, int B, float* __restrict__ dz,
                           uint16_t* __restrict__ dzq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * DH) return;
  const int b = i / DH, k = i % DH;
  float s = 0.0f;
  for (int n = 0; n < 3; ++n) s += dy[3 * b + n] * bf2f(w4t[n * DH + k]);
  const float d = s * gelu_grad(z3[i]);
  dz[i] = d;
  dzq[i] = f2bf(d);
}

// bias gradient: grad[off + n] = sum_b dz[b][n] (float), as partial sums
// over chunks of kRowChunk rows in order, then the partials in a fixed order.
__global__ void k_col_partial(const float* __restrict__ dz, int B, int N,
                              float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (n >= N) return;
  const int b0 = c * kRowChunk, b1 = min(B, b0 + kRowChunk);
  float s = 0.0f;
  for (int b = b0; b < b1; ++b) s += dz[(size_t)b * N + n];
  part[(size_t)c * N + n] = s;
}

// One wave per entry: lane l sums partials l, l + 64, ... in order, then a
// fixed shuffle tree (deterministic).
__global__ void k_col_finish(const float* __restrict__ part, int chunks, int N,
                             float* __restrict__ out) {
  const int n = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = (int)(threadIdx.x & 63u);
  if (n >= N) return;  // wave-uniform
  float s = 0.0f;
  for (int c = lane; c < chunks; c += 64) s += part[(size_t)c * N + n];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[n] = s;
}

__global__ void k_sum_rows(const float* __restrict__ v, int B, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < B; i += 256) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (float)B;
}

// Adam (Kingma & Ba 2015) on the float master weights.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_init_params(float* __restrict__ w, uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N_PARAMS) return;
  // counter-based uniform in [-1, 1): splitmix64 of (seed, i)
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const float u = (float)(z >> 40) * (1.0f / 8388608.0f) - 1.0f;
  int fan_in;
  bool bias;
  if (i < OFF_B1) { fan_in = D0; bias = false; }
  else if (i < OFF_W2) { fan_in = D0; bias = true; }
  else if (i < OFF_B2) { fan_in = DH; bias = false; }
  else if (i < OFF_W3) { fan_in = DH; bias = true; }
  else if (i < OFF_B3) { fan_in = DH; bias = false; }
  else if (i < OFF_W4) { fan_in = DH; bias = true; }
  else if (i < OFF_B4) { fan_in = DH; bias = false; }
  else { fan_in = DH; bias = true; }
  // uniform with variance 2 / fan_in (He) for weights, zero biases
  w[i] = bias ? 0.0f : u * sqrtf(6.0f / (float)fan_in);
}

}  // namespace

// ---- host object ----------------------------------------------------------------------

struct fd_mlp {
  int device = 0;
  float* master = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t step = 0;
  Packed pk{};
  float learned_step0 = 0.0f;
  float fallback_cost = INFINITY;
  // training workspace
  int cap_batch = 0;
  uint16_t* x = nullptr;                 // B x 128
  float* z[3] = {nullptr, nullptr, nullptr};  // B x 256 pre-activations
  uint16_t* h[3] = {nullptr, nullptr, nullptr};  // B x 256 bf16 activations
  float* dy = nullptr;                   // B x 3
  float* lrow = nullptr;                 // B
  float* dz = nullptr;                   // B x 256
  uint16_t* dzq = nullptr;               // B x 256
  float* part = nullptr;                 // chunk partial sums of the gradients
  float* split = nullptr;                // K-slice partial tiles of the weight gradients
  float* grad = nullptr;                 // N_PARAMS
  float* loss = nullptr;                 // 1
};

namespace {

int mlp_pack(fd_mlp* m, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((DH * DH + 255) / 256), dim3(256), 0, st, m->master, m->pk);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "mlp pack");
}

int ensure_train_ws(fd_mlp* m, int B) {
  if (m->cap_batch >= B) return FD_OK;
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  fr(m->x);
  for (int l = 0; l < 3; ++l) {
    fr(m->z[l]);
    fr(m->h[l]);
  }
  fr(m->dy);
  fr(m->lrow);
  fr(m->dz);
  fr(m->dzq);
  fr(m->part);
  fr(m->split);
  hipError_t e = hipSuccess;
  size_t Bs = (size_t)B;
  e = hipMalloc(&m->x, Bs * D0P * 2);
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    e = hipMalloc(&m->z[l], Bs * DH * 4);
    if (e == hipSuccess) e = hipMalloc(&m->h[l], Bs * DH * 2);
  }
  if (e == hipSuccess) e = hipMalloc(&m->dy, Bs * 3 * 4);
  if (e == hipSuccess) e = hipMalloc(&m->lrow, Bs * 4);
  if (e == hipSuccess) e = hipMalloc(&m->dz, Bs * DH * 4);
  if (e == hipSuccess) e = hipMalloc(&m->dzq, Bs * DH * 2);
  if (e == hipSuccess)
    e = hipMalloc(&m->part, (Bs / kRowChunk + 1) * (size_t)kOutGrad * 4);  // >= tiles x DH
  if (e == hipSuccess) e = hipMalloc(&m->split, (size_t)kMaxSplit * DH * DH * 4);
  if (e != hipSuccess) {
    m->cap_batch = 0;
    return hip_error(e, "mlp training workspace");
  }
  m->cap_batch = B;
  return FD_OK;
}

int launch_gemm(const GemmArgs& g, hipStream_t st) {
  const bool ak = g.sak == 1, bk = g.sbk == 1;
  if ((!ak && g.sam != 1) || (!bk && g.sbn != 1) || g.N % kGemmT || (!ak && g.M % kGemmT) ||
      (g.K / g.ksplit) % kGemmK)
    return set_error(FD_E_INVAL, "mlp gemm: unsupported operand layout or shape");
  dim3 grid((g.M + kGemmT - 1) / kGemmT, g.N / kGemmT, g.ksplit);
  if (ak && bk)
    hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, dim3(256), 0, st, g);
  else if (ak)
    hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, dim3(256), 0, st, g);
  else if (bk)
    hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, dim3(256), 0, st, g);
  if (g.ksplit > 1)
    hipLaunchKernelGGL(k_gemm_reduce, dim3((g.M * g.N + 255) / 256), dim3(256), 0, st, g.part,
                       g.ksplit, g.M, g.N, g.m_real, g.n_real, g.c, g.ldc);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "mlp gemm");
}

// K slices for a weight-gradient GEMM over a batch of B rows: up to
// kMaxSplit, each at least 256 rows and a whole number of 32-row steps.
int wgrad_split(int B) {
  int S = 1;
  while (S < kMaxSplit && B % (64 * S) == 0 && B / (2 * S) >= 256) S *= 2;
  return S;
}

GemmArgs gemm_args() {
  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.ksplit = 1;
  return g;
}

// forward with saved activations + loss + full gradient into m->grad
int loss_grad(fd_mlp* m, const uint16_t* feats, const float* tgt, int B, hipStream_t st) {
  int r;
  if ((r = ensure_train_ws(m, B))) return r;
  hipLaunchKernelGGL(k_pad_input, dim3((B * D0P + 255) / 256), dim3(256), 0, st, feats, B, m->x);
  const uint16_t* wts[3] = {m->pk.w1t, m->pk.w2t, m->pk.w3t};
  // hidden layers: z_l = h_{l-1} W_l + b_l, h_l = bf16(gelu(z_l))
  for (int l = 0; l < 3; ++l) {
    GemmArgs g = gemm_args();
    const int K = l == 0 ? D0P : DH;
    g.a = l == 0 ? m->x : m->h[l - 1];
    g.sam = K;
    g.sak = 1;
    g.b = wts[l];  // B(k, n) = Wt[n][k]
    g.sbk = 1;
    g.sbn = K;
    g.M = B;
    g.N = DH;
    g.K = K;
    g.m_real = B;
    g.n_real = DH;
    g.epi = EPI_BIAS_GELU;
    g.c = m->z[l];
    g.ldc = DH;
    g.bias = m->pk.bias + l * DH;
    g.hq = m->h[l];
    g.ldh = DH;
    if ((r = launch_gemm(g, st))) return r;
  }
  hipLaunchKernelGGL(k_out_loss, dim3((B * kOutLanes + 255) / 256), dim3(256), 0, st, m->h[2],
                     m->pk.w4t, m->pk.bias + 3 * DH, tgt, B, m->dy, m->lrow);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, st, m->lrow, B, m->loss);
  const int chunks = (B + kRowChunk - 1) / kRowChunk;
  hipLaunchKernelGGL(k_outw_partial, dim3((kOutGrad + 255) / 256, chunks), dim3(256), 0, st,
                     m->h[2], m->dy, B, m->part);
  hipLaunchKernelGGL(k_col_finish, dim3((kOutGrad + 3) / 4), dim3(256), 0, st, m->part, chunks,
                     kOutGrad, m->grad + OFF_W4);
  hipLaunchKernelGGL(k_out_back, dim3((B * DH + 255) / 256), dim3(256), 0, st, m->dy,
                     m->pk.w4t, m->z[2], B, m->dz, m->dzq);
  const int offW[3] = {OFF_W1, OFF_W2, OFF_W3}, offB[3] = {OFF_B1, OFF_B2, OFF_B3};
  const int tiles = (B + kGemmT - 1) / kGemmT;
  for (int l = 2; l >= 0; --l) {
    // bias gradient of layer l: sums of the float dz over the batch, as row
    // chunk partials (k_out_back's dz for the last hidden layer, the
    // previous input-gradient product's tile partials for the others)
    if (l == 2)
      hipLaunchKernelGGL(k_col_partial, dim3(1, chunks), dim3(DH), 0, st, m->dz, B, DH, m->part);
    hipLaunchKernelGGL(k_col_finish, dim3(DH / 4), dim3(256), 0, st, m->part,
                       l == 2 ? chunks : tiles, DH, m->grad + offB[l]);
    // weight gradient: dW_l[k][n] = sum_b h_{l-1}[b][k] dzq[b][n]
    {
      GemmArgs g = gemm_args();
      const int Kin = l == 0 ? D0P : DH;
      g.a = l == 0 ? m->x : m->h[l - 1];  // A(m = k_in, k = b)
      g.sam = 1;
      g.sak = Kin;
      g.b = m->dzq;  // B(k = b, n) = dzq[b][n]
      g.sbk = DH;
      g.sbn = 1;
      g.M = Kin;
      g.N = DH;
      g.K = B;
      g.m_real = l == 0 ? D0 : DH;
      g.n_real = DH;
      g.epi = EPI_STORE;
      g.c = m->grad + offW[l];
      g.ldc = DH;
      g.ksplit = wgrad_split(B);
      g.part = m->split;
      if ((r = launch_gemm(g, st))) return r;
    }
    if (l == 0) break;
    // dz_{l-1} = (dzq W_l^T) * gelu'(z_{l-1})
    {
      GemmArgs g = gemm_args();
      const int Kin = DH;  // rows of W_l for l >= 1
      g.a = m->dzq;        // A(m = b, k = out) = dzq[b][out]
      g.sam = DH;
      g.sak = 1;
      g.b = wts[l];  // B(k = out, n = in) = W_l[in][out] = Wt[out][in]
      g.sbk = Kin;
      g.sbn = 1;
      g.M = B;
      g.N = Kin;
      g.K = DH;
      g.m_real = B;
      g.n_real = Kin;
      g.epi = EPI_GELU_BACK;
      g.c = m->z[l - 1];
      g.ldc = DH;
      // the new bfloat16 gradient goes to h[l] (no longer needed: h[l]'s
      // weight gradient is done), its bias-gradient partials to part
      g.df = m->part;
      g.hq = m->h[l];
      g.ldh = DH;
      if ((r = launch_gemm(g, st))) return r;
    }
    std::swap(m->dzq, m->h[l]);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "mlp backward");
}

}  // namespace

namespace fd {
int mlp_forward_dev(const fd_mlp* m, const uint16_t* feats, int64_t n, float* out, hipStream_t st) {
  if (n <= 0) return FD_OK;
  const int64_t nb = (n + FWD_ROWS - 1) / FWD_ROWS;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)nb), dim3(kFwdThreads), 0, st, feats, n, m->pk,
                     out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "mlp forward");
}
}  // namespace fd

extern "C" int fd_mlp_create(fd_mlp** out, uint64_t seed) {
  if (!out) return set_error(FD_E_INVAL, "fd_mlp_create: out is NULL");
  int dev, r;
  if ((r = check_device(&dev))) return r;
  fd_mlp* m = new (std::nothrow) fd_mlp();
  if (!m) return set_error(FD_E_NOMEM, "fd_mlp_create: host allocation failed");
  m->device = dev;
  bump_workspace_generation();  // a captured batched graph holds weight pointers
  hipError_t e = hipMalloc(&m->master, N_PARAMS * 4);
  if (e == hipSuccess) e = hipMalloc(&m->adam_m, N_PARAMS * 4);
  if (e == hipSuccess) e = hipMalloc(&m->adam_v, N_PARAMS * 4);
  if (e == hipSuccess) e = hipMalloc(&m->grad, N_PARAMS * 4);
  if (e == hipSuccess) e = hipMalloc(&m->loss, 4);
  if (e == hipSuccess) e = hipMalloc(&m->pk.w1t, DH * D0P * 2);
  if (e == hipSuccess) e = hipMalloc(&m->pk.w2t, DH * DH * 2);
  if (e == hipSuccess) e = hipMalloc(&m->pk.w3t, DH * DH * 2);
  if (e == hipSuccess) e = hipMalloc(&m->pk.w4t, DOP * DH * 2);
  if (e == hipSuccess) e = hipMalloc(&m->pk.bias, (3 * DH + DOP) * 4);
  if (e != hipSuccess) {
    fd_mlp_destroy(m);
    return hip_error(e, "fd_mlp_create");
  }
  hipLaunchKernelGGL(k_init_params, dim3((N_PARAMS + 255) / 256), dim3(256), 0, 0, m->master,
                     seed);
  (void)hipMemset(m->adam_m, 0, N_PARAMS * 4);
  (void)hipMemset(m->adam_v, 0, N_PARAMS * 4);
  if ((r = mlp_pack(m, 0))) {
    fd_mlp_destroy(m);
    return r;
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    fd_mlp_destroy(m);
    return hip_error(e, "fd_mlp_create");
  }
  *out = m;
  return FD_OK;
}

extern "C" void fd_mlp_destroy(fd_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  void* bufs[] = {m->master, m->adam_m, m->adam_v, m->grad, m->loss, m->pk.w1t, m->pk.w2t,
                  m->pk.w3t, m->pk.w4t, m->pk.bias, m->x, m->dy, m->lrow, m->dz, m->dzq,
                  m->part, m->split, m->z[0], m->z[1], m->z[2], m->h[0], m->h[1], m->h[2]};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  delete m;
}

extern "C" int fd_mlp_set_params(fd_mlp* m, const float* host) {
  if (!m || !host) return set_error(FD_E_INVAL, "fd_mlp_set_params: null argument");
  hipError_t e = hipMemcpy(m->master, host, N_PARAMS * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_error(e, "fd_mlp_set_params");
  (void)hipMemset(m->adam_m, 0, N_PARAMS * 4);
  (void)hipMemset(m->adam_v, 0, N_PARAMS * 4);
  m->step = 0;
  int r = mlp_pack(m, 0);
  if (r) return r;
  e = hipDeviceSynchronize();
  return e == hipSuccess ? FD_OK : hip_error(e, "fd_mlp_set_params");
}

extern "C" int fd_mlp_get_params(const fd_mlp* m, float* host) {
  if (!m || !host) return set_error(FD_E_INVAL, "fd_mlp_get_params: null argument");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host, m->master, N_PARAMS * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? FD_OK : hip_error(e, "fd_mlp_get_params");
}

extern "C" int fd_mlp_set_calibration(fd_mlp* m, float step0, float tau) {
  if (!m) return set_error(FD_E_INVAL, "fd_mlp_set_calibration: mlp is NULL");
  m->learned_step0 = step0;
  m->fallback_cost = tau;
  return FD_OK;
}

extern "C" int fd_mlp_get_calibration(const fd_mlp* m, float* step0, float* tau) {
  if (!m || !step0 || !tau) return set_error(FD_E_INVAL, "fd_mlp_get_calibration: null argument");
  *step0 = m->learned_step0;
  *tau = m->fallback_cost;
  return FD_OK;
}

// Checkpoint file: "FDMLP001", int32 version, int32 dims[5], int64 step,
// float learned_step0, float fallback_cost, float master[N], m[N], v[N].
extern "C" int fd_mlp_save(const fd_mlp* m, const char* path) {
  if (!m || !path) return set_error(FD_E_INVAL, "fd_mlp_save: null argument");
  float* buf = new (std::nothrow) float[3 * (size_t)N_PARAMS];
  if (!buf) return set_error(FD_E_NOMEM, "fd_mlp_save: host allocation failed");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(buf, m->master, N_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf + N_PARAMS, m->adam_m, N_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf + 2 * N_PARAMS, m->adam_v, N_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    delete[] buf;
    return hip_error(e, "fd_mlp_save");
  }
  FILE* f = fopen(path, "wb");
  if (!f) {
    delete[] buf;
    return set_error(FD_E_INVAL, "fd_mlp_save: cannot open %s", path);
  }
  const char magic[8] = {'F', 'D', 'M', 'L', 'P', '0', '0', '1'};
  const int32_t ver = 1, dims[5] = {D0, DH, DH, DH, DO};
  bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&ver, 4, 1, f) == 1 &&
            fwrite(dims, 4, 5, f) == 5 && fwrite(&m->step, 8, 1, f) == 1 &&
            fwrite(&m->learned_step0, 4, 1, f) == 1 && fwrite(&m->fallback_cost, 4, 1, f) == 1 &&
            fwrite(buf, 4, 3 * (size_t)N_PARAMS, f) == 3 * (size_t)N_PARAMS;
  ok = (fclose(f) == 0) && ok;
  delete[] buf;
  return ok ? FD_OK : set_error(FD_E_INVAL, "fd_mlp_save: write to %s failed", path);
}

extern "C" int fd_mlp_load(fd_mlp* m, const char* path) {
  if (!m || !path) return set_error(FD_E_INVAL, "fd_mlp_load: null argument");
  FILE* f = fopen(path, "rb");
  if (!f) return set_error(FD_E_INVAL, "fd_mlp_load: cannot open %s", path);
  char magic[8];
  int32_t ver = 0, dims[5] = {0, 0, 0, 0, 0};
  int64_t step = 0;
  float s0 = 0, tau = 0;
  float* buf = new (std::nothrow) float[3 * (size_t)N_PARAMS];
  bool ok = buf && fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "FDMLP001", 8) == 0 &&
            fread(&ver, 4, 1, f) == 1 && ver == 1 && fread(dims, 4, 5, f) == 5 &&
            dims[0] == D0 && dims[1] == DH && dims[2] == DH && dims[3] == DH && dims[4] == DO &&
            fread(&step, 8, 1, f) == 1 && fread(&s0, 4, 1, f) == 1 && fread(&tau, 4, 1, f) == 1 &&
            fread(buf, 4, 3 * (size_t)N_PARAMS, f) == 3 * (size_t)N_PARAMS;
  fclose(f);
  if (!ok) {
    delete[] buf;
    return set_error(FD_E_INVAL, "fd_mlp_load: %s is not a valid checkpoint", path);
  }
  hipError_t e = hipMemcpy(m->master, buf, N_PARAMS * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->adam_m, buf + N_PARAMS, N_PARAMS * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->adam_v, buf + 2 * N_PARAMS, N_PARAMS * 4, hipMemcpyHostToDevice);
  delete[] buf;
  if (e != hipSuccess) return hip_error(e, "fd_mlp_load");
  m->step = step;
  m->learned_step0 = s0;
  m->fallback_cost = tau;
  int r = mlp_pack(m, 0);
  if (r) return r;
  e = hipDeviceSynchronize();
  return e == hipSuccess ? FD_OK : hip_error(e, "fd_mlp_load");
}

static int check_mlp_batch(const fd_mlp* m, const void* feats, int64_t batch, const char* fn) {
  if (!m) return set_error(FD_E_INVAL, "%s: mlp is NULL", fn);
  if (batch < 0) return set_error(FD_E_INVAL, "%s: batch < 0", fn);
  if (batch > 0 && !feats) return set_error(FD_E_INVAL, "%s: feats is NULL", fn);
  if (((uintptr_t)feats & 15) != 0)
    return set_error(FD_E_INVAL, "%s: feats must be 16-byte aligned", fn);
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != m->device)
    return set_error(FD_E_INVAL, "%s: network lives on device %d, current is %d", fn, m->device,
                     dev);
  return FD_OK;
}

extern "C" int fd_mlp_forward(const fd_mlp* m, const void* feats, int64_t batch, float* out,
                              void* stream) {
  int r;
  if ((r = check_mlp_batch(m, feats, batch, "fd_mlp_forward"))) return r;
  if (batch > 0 && !out) return set_error(FD_E_INVAL, "fd_mlp_forward: out is NULL");
  return mlp_forward_dev(m, (const uint16_t*)feats, batch, out, (hipStream_t)stream);
}

static int check_train(fd_mlp* m, const void* feats, const float* tgt, int32_t batch,
                       const char* fn) {
  int r;
  if ((r = check_mlp_batch(m, feats, batch, fn))) return r;
  if (batch < 16 || batch > 65536 || batch % 32 != 0)
    return set_error(FD_E_INVAL, "%s: batch must be a multiple of 32 in [32, 65536], got %d", fn,
                     batch);
  if (!tgt) return set_error(FD_E_INVAL, "%s: targets is NULL", fn);
  return FD_OK;
}

extern "C" int fd_mlp_loss_grad(fd_mlp* m, const void* feats, const float* tgt, int32_t batch,
                                float* grad, float* loss, void* stream) {
  int r;
  if ((r = check_train(m, feats, tgt, batch, "fd_mlp_loss_grad"))) return r;
  if (!grad) return set_error(FD_E_INVAL, "fd_mlp_loss_grad: grad is NULL");
  hipStream_t st = (hipStream_t)stream;
  if ((r = loss_grad(m, (const uint16_t*)feats, tgt, batch, st))) return r;
  hipError_t e = hipMemcpyAsync(grad, m->grad, N_PARAMS * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? FD_OK : hip_error(e, "fd_mlp_loss_grad");
}

extern "C" int fd_mlp_train_step(fd_mlp* m, const void* feats, const float* tgt, int32_t batch,
                                 const fd_adam* opt, float* loss, void* stream) {
  int r;
  if ((r = check_train(m, feats, tgt, batch, "fd_mlp_train_step"))) return r;
  if (!opt) return set_error(FD_E_INVAL, "fd_mlp_train_step: opt is NULL");
  hipStream_t st = (hipStream_t)stream;
  if ((r = loss_grad(m, (const uint16_t*)feats, tgt, batch, st))) return r;
  m->step += 1;
  const double bc1 = 1.0 - std::pow((double)opt->beta1, (double)m->step);
  const double bc2 = 1.0 - std::pow((double)opt->beta2, (double)m->step);
  hipLaunchKernelGGL(k_adam, dim3((N_PARAMS + 255) / 256), dim3(256), 0, st, m->master, m->adam_m,
                     m->adam_v, m->grad, N_PARAMS, opt->lr, opt->beta1, opt->beta2, opt->eps,
                     (float)bc1, (float)bc2);
  if ((r = mlp_pack(m, st))) return r;
  hipError_t e = hipSuccess;
  if (loss) e = hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "fd_mlp_train_step");
}
