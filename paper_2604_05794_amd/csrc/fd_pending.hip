// fd_pending.hip -- entry points whose kernels are not in this build yet.
#include <hip/hip_runtime.h>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"

using namespace fd;

#define PENDING(fn) return set_error(FD_E_UNSUPPORTED, "%s is not available in this build", fn)

int fd::run_learned(fd_context*, const SceneDev&, const SearchDev&, const fd_params*,
                    hipStream_t) {
  PENDING("learned mode");
}
int fd::context_reserve_scenes(fd_context*, int32_t, int64_t) { return FD_OK; }
extern "C" int fd_last_fallback_count(fd_context*, void*, int64_t*) {
  PENDING("fd_last_fallback_count");
}
extern "C" int fd_fuse_directions_batched(const fd_scene*, int32_t, const fd_params*,
                                          fd_context*) {
  PENDING("fd_fuse_directions_batched");
}
extern "C" int fd_mlp_create(fd_mlp**, uint64_t) { PENDING("fd_mlp_create"); }
extern "C" int fd_mlp_set_params(fd_mlp*, const float*) { PENDING("fd_mlp_set_params"); }
extern "C" int fd_mlp_get_params(const fd_mlp*, float*) { PENDING("fd_mlp_get_params"); }
extern "C" int fd_mlp_set_calibration(fd_mlp*, float, float) { PENDING("fd_mlp_set_calibration"); }
extern "C" int fd_mlp_get_calibration(const fd_mlp*, float*, float*) {
  PENDING("fd_mlp_get_calibration");
}
extern "C" int fd_mlp_save(const fd_mlp*, const char*) { PENDING("fd_mlp_save"); }
extern "C" int fd_mlp_load(fd_mlp*, const char*) { PENDING("fd_mlp_load"); }
extern "C" int fd_mlp_forward(const fd_mlp*, const void*, int64_t, float*, void*) {
  PENDING("fd_mlp_forward");
}
extern "C" int fd_mlp_loss_grad(fd_mlp*, const void*, const float*, int32_t, float*, float*,
                                void*) {
  PENDING("fd_mlp_loss_grad");
}
extern "C" int fd_mlp_train_step(fd_mlp*, const void*, const float*, int32_t, const fd_adam*,
                                 float*, void*) {
  PENDING("fd_mlp_train_step");
}
extern "C" void fd_mlp_destroy(fd_mlp*) {}
extern "C" int fd_features(const float*, int64_t, const fd_camera*, int32_t, const void*,
                           const void*, const fd_params*, void*) {
  PENDING("fd_features");
}
extern "C" int fd_autotune(fd_context*, const fd_scene*, int32_t, const fd_params*,
                           const char*) {
  PENDING("fd_autotune");
}
