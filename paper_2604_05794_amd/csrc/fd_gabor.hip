// fd_gabor.hip -- orientation and confidence maps from grey-level frames on
// gfx950 (the Gabor-filter extraction the paper names at the start of Sec. 3.1;
// its reading is documented with fd_orientation_maps in fusedir.h).
//
// k_gabor: one thread per pixel, 16 x 16 pixels per workgroup.  The frame
// tile with its radius-R halo is staged in LDS; the filter bank lives in
// device memory tap-major (all orientations of one tap together), so every
// tap's n_orient weights are wave-uniform and come through the scalar cache
// as operands of the n_orient FMAs the tap costs each pixel.  The epilogue
// takes the argmax orientation and the raw confidence, and the workgroup's
// largest raw confidence goes to the frame maximum (an integer atomic on the
// bits of a non-negative float).  k_gabor_norm divides by that maximum.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

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
constexpr int kTileW = kTile + 2 * kMaxRadius;
constexpr float kPi = 3.14159265358979323846f;

template <typename TO>
__device__ __forceinline__ void store_map(void* out, size_t i, float v) {
  if constexpr (sizeof(TO) == 2)
    ((__half*)out)[i] = __float2half(v);
  else
    ((float*)out)[i] = v;
}

template <typename TO, int NO>
__global__ __launch_bounds__(256) void k_gabor(const float* __restrict__ frames, int W, int H,
                                               int R, const float* __restrict__ bank,
                                               void* __restrict__ theta_out,
                                               float* __restrict__ raw,
                                               uint32_t* __restrict__ frame_max) {
  __shared__ float tile[kTileW * kTileW];
  __shared__ float wmax[256 / 64];
  const int f = blockIdx.z;
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const size_t plane = (size_t)W * H;
  const float* img = frames + plane * f;
  const int tw = kTile + 2 * R;
  for (int e = threadIdx.x; e < tw * tw; e += blockDim.x) {
    const int ty = e / tw, tx = e - ty * tw;
    const int x = x0 + tx - R, y = y0 + ty - R;
    tile[ty * tw + tx] = (x >= 0 && x < W && y >= 0 && y < H) ? img[(size_t)y * W + x] : 0.0f;
  }
  __syncthreads();
  const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
  const int x = x0 + lx, y = y0 + ly;
  float acc[NO];
#pragma unroll
  for (int i = 0; i < NO; ++i) acc[i] = 0.0f;
  const int w2 = 2 * R + 1;
  // taps in the oracle's order: dy outer, dx inner
  for (int dy = 0; dy < w2; ++dy) {
    const float* row = tile + (ly + dy) * tw + lx;
    const float* wrow = bank + (size_t)dy * w2 * NO;
    for (int dx = 0; dx < w2; ++dx) {
      const float v = row[dx];
      const float* w = wrow + dx * NO;
#pragma unroll
      for (int i = 0; i < NO; ++i) acc[i] = __builtin_fmaf(w[i], v, acc[i]);
    }
  }
  // argmax |F_i| (first of equals) and the spread of the responses around it
  int best = 0;
  float fb = fabsf(acc[0]);
#pragma unroll
  for (int i = 1; i < NO; ++i) {
    const float fi = fabsf(acc[i]);
    if (fi > fb) {
      fb = fi;
      best = i;
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const int di = abs(i - best);
    const float d = (float)min(di, NO - di) * (kPi / NO);
    const float e = fabsf(acc[i]) - fb;
    s = __builtin_fmaf(d * d, e * e, s);
  }
  const float w = sqrtf(s);
  const bool inside = x < W && y < H;
  if (inside) {
    const size_t i = plane * f + (size_t)y * W + x;
    store_map<TO>(theta_out, i, (float)best * (kPi / NO));
    raw[i] = w;
  }
  // workgroup maximum of the raw confidence -> frame maximum
  float m = inside ? w : 0.0f;
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = wmax[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) b = fmaxf(b, wmax[k]);
    atomicMax(&frame_max[f], __float_as_uint(b));  // b >= 0: bits order as values
  }
}

template <typename TO>
__global__ __launch_bounds__(256) void k_gabor_norm(const float* __restrict__ raw,
                                                    const uint32_t* __restrict__ frame_max,
                                                    int64_t plane, int64_t n,
                                                    void* __restrict__ conf_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float m = __uint_as_float(frame_max[i / plane]);
  store_map<TO>(conf_out, (size_t)i, m > 0.0f ? raw[i] / m : 0.0f);
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
  const dim3 grid((unsigned)((W + kTile - 1) / kTile), (unsigned)((H + kTile - 1) / kTile),
                  (unsigned)n);
  switch (N) {
    case 8:
      hipLaunchKernelGGL((k_gabor<TO, 8>), grid, dim3(256), 0, st, frames, W, H, R, bank, theta,
                         raw, fmax);
      break;
    case 16:
      hipLaunchKernelGGL((k_gabor<TO, 16>), grid, dim3(256), 0, st, frames, W, H, R, bank,
                         theta, raw, fmax);
      break;
    default:
      hipLaunchKernelGGL((k_gabor<TO, 32>), grid, dim3(256), 0, st, frames, W, H, R, bank,
                         theta, raw, fmax);
      break;
  }
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
  const int64_t nb = ((int64_t)total + 255) / 256;
  if (p->out_dtype == FD_F16)
    hipLaunchKernelGGL(k_gabor_norm<__half>, dim3((unsigned)nb), dim3(256), 0, st, c->gabor_raw,
                       c->gabor_max, (int64_t)plane, (int64_t)total, conf_out);
  else
    hipLaunchKernelGGL(k_gabor_norm<float>, dim3((unsigned)nb), dim3(256), 0, st, c->gabor_raw,
                       c->gabor_max, (int64_t)plane, (int64_t)total, conf_out);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "confidence kernel");
  tn.stop();
  return FD_OK;
}
