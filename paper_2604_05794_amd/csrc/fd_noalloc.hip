// fd_noalloc.hip -- the plain search without any allocation: its workspace
// (tiling keys and counts, permutation, view lists, search constants, the
// binary64 camera table) lives
// in one fixed device array per GPU instead of a context, for callers that
// cannot allocate (graph capture, tight serving loops).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_kernels.hpp"

using namespace fd;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr size_t kMaxPts = (size_t)FD_NOALLOC_MAX_POINTS;
constexpr size_t kCellsMax = (size_t)1 << 18;  // cells of the single-scene tiling (64^3)

// byte offsets of the workspace inside the array
constexpr size_t kOffLattice = 0;
constexpr size_t kOffConsts = align_up(kOffLattice + sizeof(float) * 3 * FD_MAX_CANDIDATES);
constexpr size_t kOffBbox = align_up(kOffConsts + sizeof(double) * kConstsDoubles);
constexpr size_t kOffCounts = align_up(kOffBbox + sizeof(int) * 8);
constexpr size_t kOffCursor = align_up(kOffCounts + sizeof(uint32_t) * kCellsMax);
constexpr size_t kOffSums = align_up(kOffCursor + sizeof(uint32_t) * kCellsMax);
constexpr size_t kOffFbCount = align_up(kOffSums + sizeof(uint32_t) * (kCellsMax / 1024));
constexpr size_t kOffKey = align_up(kOffFbCount + sizeof(uint32_t) * 8);
constexpr size_t kOffPerm = align_up(kOffKey + sizeof(uint32_t) * kMaxPts);
constexpr size_t kOffViews = align_up(kOffPerm + sizeof(uint32_t) * kMaxPts);
constexpr size_t kOffKcount = align_up(kOffViews + sizeof(uint16_t) * FD_TOPK_SLOTS * kMaxPts);
constexpr size_t kOffCams = align_up(kOffKcount + sizeof(uint8_t) * kMaxPts);
constexpr size_t kScratchBytes =
    align_up(kOffCams + sizeof(double) * kCam64 * (size_t)FD_NOALLOC_MAX_VIEWS);
static_assert(kScratchBytes <= ((size_t)16 << 20), "scratch stays within 16 MiB");

}  // namespace

// The workspace of every fd_fuse_directions_noalloc call on a device: each
// device holds its own copy of this array (for the life of the process),
// at its own address.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in); it takes the device address of this
// device's copy from hipGetSymbolAddress and uses that.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// this device's address of `scratch`, looked up once per device
unsigned char* scratch_ptr(int dev, int* err) {
  static std::mutex mu;
  static unsigned char* ptrs[256] = {};
  if (dev < 0 || dev >= 256) {
    *err = set_error(FD_E_UNSUPPORTED, "fd_fuse_directions_noalloc: device %d", dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                       "fd_fuse_directions_noalloc: hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    ptrs[dev] = (unsigned char*)p;
  }
  *err = FD_OK;
  return ptrs[dev];
}

}  // namespace

extern "C" int fd_fuse_directions_noalloc(const float* points, int64_t n_points,
                                          const fd_camera* cams, int32_t n_views,
                                          const void* orient_maps, const void* conf_maps,
                                          const fd_params* params, float* dirs, float* costs) {
  const char* fn = "fd_fuse_directions_noalloc";
  int r;
  if ((r = check_scene_call(points, n_points, cams, n_views, orient_maps, conf_maps, params,
                            dirs, costs, fn)))
    return r;
  if (params->mode != FD_MODE_PLAIN)
    return set_error(FD_E_INVAL, "%s: only the plain mode runs without a context", fn);
  if (n_points > (int64_t)kMaxPts)
    return set_error(FD_E_INVAL, "%s: %lld points exceed the fixed workspace of %lld points",
                     fn, (long long)n_points, (long long)kMaxPts);
  if (n_views > FD_NOALLOC_MAX_VIEWS)
    return set_error(FD_E_INVAL, "%s: %d views exceed the fixed workspace of %d views", fn,
                     n_views, FD_NOALLOC_MAX_VIEWS);
  if ((size_t)tile_cells() > kCellsMax)
    return set_error(FD_E_UNSUPPORTED, "%s: tiling grid larger than the fixed workspace", fn);
  if (n_points == 0) return FD_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  unsigned char* base = scratch_ptr(dev, &r);
  if (!base) return r;
  // a context whose buffers are views of this device's array; it owns
  // nothing and is never destroyed through fd_context_destroy
  fd_context c;
  c.device = dev;
  c.max_points = (int64_t)kMaxPts;
  c.lattice = (float*)(base + kOffLattice);
  c.consts64 = (double*)(base + kOffConsts);
  c.bbox = (int*)(base + kOffBbox);
  c.counts = (uint32_t*)(base + kOffCounts);
  c.cursor = (uint32_t*)(base + kOffCursor);
  c.scan_sums = (uint32_t*)(base + kOffSums);
  c.fb_count = (uint32_t*)(base + kOffFbCount);
  c.key = (uint32_t*)(base + kOffKey);
  c.perm = (uint32_t*)(base + kOffPerm);
  c.views = (uint16_t*)(base + kOffViews);
  c.kcount = (uint8_t*)(base + kOffKcount);
  c.cams64 = (double*)(base + kOffCams);
  c.cap_cams64 = (size_t)kCam64 * FD_NOALLOC_MAX_VIEWS;
  const SceneArgs sa = scene_args(points, n_points, cams, n_views, orient_maps, conf_maps,
                                  params, dirs, costs);
  return run_scene(&c, sa, params, (hipStream_t)params->stream);
}
