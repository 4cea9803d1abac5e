// fd_gabor.hip -- orientation and confidence maps from grey-level frames on
// gfx950 (the Gabor-filter extraction the paper names at the start of Sec. 3.1;
// its reading is documented with fd_orientation_maps in fusedir.h).
//
// k_gabor_mfma: the filter bank is a dense contraction over the taps, run on
// the fp32 matrix cores.  Persistent workgroups of four waves hold the bank
// in LDS and walk 16 x 32 pixel tiles, each staged in LDS with its radius-R
// halo; the epilogue takes the argmax orientation and the raw confidence, and
// the workgroup's largest raw confidence goes to the frame maximum (an
// integer atomic on the bits of a non-negative float).  k_gabor_norm divides
// by that maximum.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_kernels.hpp"

using namespace fd;

namespace {

constexpr int kTile = 16;
constexpr int kMaxRadius = 12;
constexpr float kPi = 3.14159265358979323846f;

template <typename TO>
__device__ __forceinline__ void store_map(void* out, size_t i, float v) {
  if constexpr (sizeof(TO) == 2)
    ((__half*)out)[i] = __float2half(v);
  else
    ((float*)out)[i] = v;
}

// One frame per grid row (its maximum read once), 8 pixels per thread in
// 16-byte loads and stores where the plane and the output allow it.
template <typename TO>
__global__ __launch_bounds__(256) void k_gabor_norm(const float* __restrict__ raw,
                                                    const uint32_t* __restrict__ frame_max,
                                                    int64_t plane, int vec,
                                                    void* __restrict__ conf_out) {
  const int64_t f = blockIdx.y;
  const float m = __uint_as_float(frame_max[f]);
  const float* r = raw + plane * f;
  TO* out = (TO*)conf_out + plane * f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec) {
    const int64_t n8 = plane >> 3;
    for (int64_t i = t0; i < n8; i += stride) {
      const float4 a = ((const float4*)r)[2 * i], b = ((const float4*)r)[2 * i + 1];
      const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      float o[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = m > 0.0f ? v[k] / m : 0.0f;
      if constexpr (sizeof(TO) == 2) {
        uint32_t h[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = __half_as_ushort(__float2half(o[k]));
        ((uint4*)out)[i] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16),
                                      h[4] | (h[5] << 16), h[6] | (h[7] << 16));
      } else {
        ((float4*)out)[2 * i] = make_float4(o[0], o[1], o[2], o[3]);
        ((float4*)out)[2 * i + 1] = make_float4(o[4], o[5], o[6], o[7]);
      }
    }
  } else {
    for (int64_t i = t0; i < plane; i += stride)
      store_map<TO>(out, (size_t)i, m > 0.0f ? r[i] / m : 0.0f);
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kRowsPerWave = 8;
constexpr int kMfmaRows = 4 * kRowsPerWave;  // tile rows: four waves
constexpr int kTw = kTile + 2 * kMaxRadius;  // LDS tile row stride for every radius

// The filter bank as a matrix product on the fp32 matrix cores: for a row
// of 16 pixels, F[orientation][pixel] = sum_tap G[orientation][tap] I[pixel + tap]
// in steps of 4 taps (v_mfma_f32_16x16x4f32: A = 16 orientations x 4 bank
// taps, B = the 4 x 16 image patch gathered from the LDS tile).  Persistent
// workgroups keep the bank in LDS, zero-padded to whole 4-tap steps and
// 16-orientation tiles and laid out [tap / 4][orientation tile][tap % 4][16]
// so that a wave's A operand is 64 consecutive words; they walk pixel tiles
// 16 wide and 32 high, wave w owning rows 8w .. 8w + 7, so each bank read
// feeds 8 matrix operations.  The tile rows are kTw words apart for every
// radius: the 8 row reads of a step take immediate offsets and pair up.  The
// matrix cores only reach their peak when little else is issued beside them,
// so the per-step bookkeeping is kept small: the position of the step's first
// tap is wave-uniform (scalar registers) and a lane's tap is at most one row
// further.  In the result lane (g, c) = (lane / 16, lane % 16) holds
// orientations 16 nt + 4 g + r (r < 4) of pixel c: the argmax (first of
// equals) and the confidence sum run over those 4 NT values in the lane, then
// across the four 16-lane groups; the squared bin distances come from a
// small LDS table.
// FULL: n_orient fills the NT orientation tiles (no per-lane validity
// tests).  Three waves per SIMD is what the LDS allows (three workgroups per
// CU at radius 8); the register bound keeps the compiler to it.
template <typename TO, int NT, bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gabor_mfma(const float* __restrict__ frames, int W,
                                                    int H, int R, int NO,
                                                    const float* __restrict__ bank,
                                                    int64_t n_tiles, int tiles_x,
                                                    int64_t tiles_per_frame,
                                                    void* __restrict__ theta_out,
                                                    float* __restrict__ raw,
                                                    uint32_t* __restrict__ frame_max) {
  extern __shared__ float lds[];
  __shared__ float wmax[256 / 64];
  constexpr int NJ = 16 * NT;
  const int w2 = 2 * R + 1, taps = w2 * w2, kpad = (taps + 3) & ~3, tw = kTile + 2 * R;
  const int th = kMfmaRows + 2 * R;  // tile rows with the halo
  float* sbank = lds;              // kpad x NJ
  float* tile = lds + kpad * NJ;   // th x kTw
  for (int e = threadIdx.x; e < kpad * NJ; e += blockDim.x) {
    const int t = e / NJ, j = e - t * NJ;
    const int dst = (t >> 2) * 4 * NJ + (j >> 4) * 64 + (t & 3) * 16 + (j & 15);
    sbank[dst] = (t < taps && j < NO) ? bank[(size_t)t * NO + j] : 0.0f;
  }
  // d2tab[NO + k] = squared line distance of two bins k apart (|k| < NO)
  float* d2tab = tile + kTw * th;  // 64
  if (threadIdx.x < 64) {
    const int k = abs((int)threadIdx.x - NO);
    float v = 0.0f;
    if (k < NO) {
      const float dd = (float)min(k, NO - k) * (kPi / NO);
      v = dd * dd;
    }
    d2tab[threadIdx.x] = v;
  }
  const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
  const int g = lane >> 4, c16 = lane & 15;
  const size_t plane = (size_t)W * H;
  for (int64_t tid = blockIdx.x; tid < n_tiles; tid += gridDim.x) {
    const int64_t f = tid / tiles_per_frame;
    const int64_t rem = tid - f * tiles_per_frame;
    const int ty = (int)(rem / tiles_x), tx = (int)(rem - (int64_t)ty * tiles_x);
    const int x0 = tx * kTile, y0 = ty * kMfmaRows;
    const float* img = frames + plane * f;
    __syncthreads();  // the bank is in place; the previous tile is no longer read
    for (int e = threadIdx.x; e < kTw * th; e += blockDim.x) {
      const int yy = e / kTw, xx = e - yy * kTw;
      const int x = x0 + xx - R, y = y0 + yy - R;
      tile[e] = (xx < tw && x >= 0 && x < W && y >= 0 && y < H) ? img[(size_t)y * W + x] : 0.0f;
    }
    __syncthreads();
    f32x4 acc[kRowsPerWave][NT];
#pragma unroll
    for (int p = 0; p < kRowsPerWave; ++p)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[p][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const float* base = tile + kRowsPerWave * w * kTw + c16 + g;
    const float* bk = sbank + lane;
    // wave-uniform (row offset, column) of tap k0; a lane's tap k0 + g is at
    // most one row further (g < 4 <= w2 + 1 and the column stays < w2)
    int s_off = 0, s_dx = 0;
    for (int k0 = 0; k0 < kpad; k0 += 4) {
      const int wrap = g >= w2 - s_dx ? kTw - w2 : 0;
      const int off = k0 + g < taps ? s_off + wrap : -g;
      float a[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) a[nt] = bk[k0 * NJ + 64 * nt];
      const float* src = base + off;
#pragma unroll
      for (int p = 0; p < kRowsPerWave; ++p) {
        const float v = src[p * kTw];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[p][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[nt], v, acc[p][nt], 0, 0, 0);
      }
      // issue order: the step's LDS reads (the bank, then the row pairs),
      // then its matrix operations
      __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, kRowsPerWave * NT, 0);
      s_dx += 4;
      s_off += 4;
      if (s_dx >= w2) { s_dx -= w2; s_off += kTw - w2; }
      if (s_dx >= w2) { s_dx -= w2; s_off += kTw - w2; }
    }
    // per pixel: argmax |F_j| (first of equals), then the spread of the
    // responses around it
    float m = 0.0f;
#pragma unroll
    for (int p = 0; p < kRowsPerWave; ++p) {
      float fv[NT][4];
      float fb = -1.0f;
      int jb = 0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * nt + 4 * g + r;  // increasing in the lane
          fv[nt][r] = (FULL || j < NO) ? fabsf(acc[p][nt][r]) : -1.0f;
          if (fv[nt][r] > fb) {
            fb = fv[nt][r];
            jb = j;
          }
        }
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        const float of = __shfl_xor(fb, off, 64);
        const int oj = __shfl_xor(jb, off, 64);
        if (of > fb || (of == fb && oj < jb)) {
          fb = of;
          jb = oj;
        }
      }
      float s = 0.0f;
      const float* d2 = d2tab + (NO + 4 * g - jb);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * nt + 4 * g + r;
          if (FULL || j < NO) {
            const float e = fv[nt][r] - fb;
            s = __builtin_fmaf(d2[16 * nt + r], e * e, s);
          }
        }
      s += __shfl_xor(s, 16, 64);
      s += __shfl_xor(s, 32, 64);
      const float wv = sqrtf(s);
      const int x = x0 + c16, y = y0 + kRowsPerWave * w + p;
      if (g == 0 && x < W && y < H) {
        const size_t i = plane * f + (size_t)y * W + x;
        store_map<TO>(theta_out, i, (float)jb * (kPi / NO));
        raw[i] = wv;
        m = fmaxf(m, wv);
      }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if (lane == 0) wmax[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      float bm = wmax[0];
      for (int k = 1; k < (int)(blockDim.x >> 6); ++k) bm = fmaxf(bm, wmax[k]);
      atomicMax(&frame_max[f], __float_as_uint(bm));  // bm >= 0: bits order as values
    }
  }
}

uint64_t fnv1(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

// The bank in binary64 from its definition, rounded to binary32, tap-major.
std::vector<float> make_bank(const fd_gabor_params* p) {
  const int N = p->n_orient, R = p->radius, w = 2 * R + 1;
  std::vector<double> g((size_t)N * w * w);
  for (int i = 0; i < N; ++i) {
    const double t = 3.14159265358979323846 * i / N, ct = std::cos(t), st = std::sin(t);
    double mean = 0.0;
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const double a = dx * ct + dy * st, b = -dx * st + dy * ct;
        const double sa = p->sigma_along, sb = p->sigma_across;
        const double v = std::exp(-a * a / (2 * sa * sa) - b * b / (2 * sb * sb)) *
                         std::cos(2 * 3.14159265358979323846 * b / p->wavelength);
        g[((size_t)i * w + (dy + R)) * w + (dx + R)] = v;
        mean += v;
      }
    mean /= (double)(w * w);
    for (int k = 0; k < w * w; ++k) g[(size_t)i * w * w + k] -= mean;
  }
  std::vector<float> out((size_t)N * w * w);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < w * w; ++k) out[(size_t)k * N + i] = (float)g[(size_t)i * w * w + k];
  return out;
}

template <typename TO>
hipError_t launch_gabor(const float* frames, int n, int W, int H, int R, int N, const float* bank,
                        void* theta, float* raw, uint32_t* fmax, hipStream_t st) {
  const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kMfmaRows - 1) / kMfmaRows;
  const int64_t per_frame = (int64_t)tiles_x * tiles_y, n_tiles = per_frame * n;
  const int taps = (2 * R + 1) * (2 * R + 1), kpad = (taps + 3) & ~3;
  const int th = kMfmaRows + 2 * R;
  const int nt = N > 16 ? 2 : 1;
  const size_t lds = sizeof(float) * ((size_t)kpad * 16 * nt + (size_t)kTw * th + 64);
  // N = 16 and 32 fill their orientation tiles: no per-lane validity tests
  const auto kern = nt == 2    ? k_gabor_mfma<TO, 2, true>
                    : N == 16 ? k_gabor_mfma<TO, 1, true>
                              : k_gabor_mfma<TO, 1, false>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // persistent: each workgroup loads the bank once; several resident per CU
  const int per_cu = (int)std::max<size_t>(1, (160 * 1024) / (lds + 1024));
  const int64_t grid = std::min<int64_t>(n_tiles, (int64_t)256 * std::min(per_cu, 4));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, st, frames, W, H, R, N, bank,
                     n_tiles, tiles_x, per_frame, theta, raw, fmax);
  return hipGetLastError();
}

}  // namespace

extern "C" void fd_gabor_params_init(fd_gabor_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->n_orient = 32;
  p->radius = 8;
  p->sigma_along = 2.4f;
  p->sigma_across = 1.8f;
  p->wavelength = 4.0f;
  p->out_dtype = FD_F16;
  p->stream = nullptr;
  p->ctx = nullptr;
}

extern "C" int fd_orientation_maps(const float* frames, int32_t n_frames, int32_t width,
                                   int32_t height, const fd_gabor_params* p, void* theta_out,
                                   void* conf_out) {
  const char* fn = "fd_orientation_maps";
  int r;
  if (!p) return set_error(FD_E_INVAL, "%s: params is NULL", fn);
  if (p->n_orient != 8 && p->n_orient != 16 && p->n_orient != 32)
    return set_error(FD_E_INVAL, "%s: n_orient must be 8, 16 or 32, got %d", fn, p->n_orient);
  if (p->radius < 1 || p->radius > kMaxRadius)
    return set_error(FD_E_INVAL, "%s: radius must be in [1, %d], got %d", fn, kMaxRadius,
                     p->radius);
  if (!(p->sigma_along > 0.0f) || !(p->sigma_across > 0.0f) || !(p->wavelength > 0.0f) ||
      !std::isfinite(p->sigma_along) || !std::isfinite(p->sigma_across) ||
      !std::isfinite(p->wavelength))
    return set_error(FD_E_INVAL, "%s: sigmas and wavelength must be finite and > 0", fn);
  if (p->out_dtype != FD_F32 && p->out_dtype != FD_F16)
    return set_error(FD_E_INVAL, "%s: unknown out_dtype %d", fn, p->out_dtype);
  if (n_frames < 0 || n_frames > FD_MAX_VIEWS)
    return set_error(FD_E_INVAL, "%s: n_frames must be in [0, %d]", fn, FD_MAX_VIEWS);
  if (width < 1 || height < 1 || width > 32768 || height > 32768)
    return set_error(FD_E_INVAL, "%s: frame size out of range", fn);
  if (n_frames > 0 && (!frames || !theta_out || !conf_out))
    return set_error(FD_E_INVAL, "%s: null pointer argument", fn);
  int dev = 0;
  if ((r = check_device(&dev))) return r;
  if (n_frames == 0) return FD_OK;
  fd_context* c = p->ctx;
  if (c) {
    if (c->device != dev)
      return set_error(FD_E_INVAL, "%s: context belongs to device %d", fn, c->device);
  } else {
    c = default_context(dev, 0, &r);
    if (!c) return r;
  }
  hipStream_t st = (hipStream_t)p->stream;
  // the filter bank, rebuilt when its parameters change
  uint64_t sig = 1469598103934665603ull;
  sig = fnv1(sig, &p->n_orient, sizeof p->n_orient);
  sig = fnv1(sig, &p->radius, sizeof p->radius);
  sig = fnv1(sig, &p->sigma_along, sizeof p->sigma_along);
  sig = fnv1(sig, &p->sigma_across, sizeof p->sigma_across);
  sig = fnv1(sig, &p->wavelength, sizeof p->wavelength);
  hipError_t e;
  if (c->gabor_sig != sig || !c->gabor_bank) {
    const std::vector<float> bank = make_bank(p);
    // a previous call on this stream may still read the old bank
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_error(e, "filter bank");
    if ((r = ctx_buffer((void**)&c->gabor_bank, &c->cap_gabor_bank, bank.size() * sizeof(float),
                        "filter bank")))
      return r;
    e = hipMemcpy(c->gabor_bank, bank.data(), bank.size() * sizeof(float),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "filter bank upload");
    c->gabor_sig = sig;
  }
  const size_t plane = (size_t)width * height, total = plane * (size_t)n_frames;
  if (total > ((size_t)1 << 34))
    return set_error(FD_E_INVAL, "%s: more than 2^34 pixels in one call", fn);
  if ((r = ctx_buffer((void**)&c->gabor_raw, &c->cap_gabor_raw, total * sizeof(float),
                      "raw confidence")))
    return r;
  if ((r = ctx_buffer((void**)&c->gabor_max, &c->cap_gabor_max, n_frames * sizeof(uint32_t),
                      "frame maxima")))
    return r;
  if ((e = launch_fill_u32(c->gabor_max, n_frames, 0u, st)) != hipSuccess)
    return hip_error(e, "frame maxima reset");
  StageTimer tg(c, FD_STAGE_GABOR, st);
  e = p->out_dtype == FD_F16
          ? launch_gabor<__half>(frames, n_frames, width, height, p->radius, p->n_orient,
                                 c->gabor_bank, theta_out, c->gabor_raw, c->gabor_max, st)
          : launch_gabor<float>(frames, n_frames, width, height, p->radius, p->n_orient,
                                c->gabor_bank, theta_out, c->gabor_raw, c->gabor_max, st);
  if (e != hipSuccess) return hip_error(e, "orientation kernel");
  tg.stop();
  StageTimer tn(c, FD_STAGE_GABOR_NORM, st);
  // raw is a workspace allocation, so only the plane and the caller's output
  // decide whether whole 16-byte groups line up
  const int vec = plane % 8 == 0 && (uintptr_t)conf_out % 16 == 0;
  const int64_t work = vec ? (int64_t)plane / 8 : (int64_t)plane;
  const dim3 ng((unsigned)std::min<int64_t>((work + 255) / 256, 1 << 20), (unsigned)n_frames);
  if (p->out_dtype == FD_F16)
    hipLaunchKernelGGL(k_gabor_norm<__half>, ng, dim3(256), 0, st, c->gabor_raw, c->gabor_max,
                       (int64_t)plane, vec, conf_out);
  else
    hipLaunchKernelGGL(k_gabor_norm<float>, ng, dim3(256), 0, st, c->gabor_raw, c->gabor_max,
                       (int64_t)plane, vec, conf_out);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "confidence kernel");
  tn.stop();
  return FD_OK;
}
