// device_stubs.cpp -- host-only stand-ins for the kernel launchers and the
// run-time compiler, so that the host side of the evaluator (rule compiler,
// net validation, read-back) links into a sanitizer build without a device.
// Every stand-in reports INET_ENOSYS; the sanitizer driver never reaches them.
#include <hip/hip_runtime.h>

#include "inet.h"
#include "inet_internal.h"
#include "runtime.h"

namespace inet {
bool shape_supported(int wg) { return wg == 64 || wg == 128 || wg == 256 || wg == 512 || wg == 1024; }
LaunchShape shape_for(int wg, int engine, int maxl) { return {wg, 4096, engine, maxl}; }
int launch_reduce(const CompiledRules &, const LaunchShape &, int, const NetDesc *, const int32_t *,
                  int, int32_t *, const int32_t *, uint32_t, int, const KParams &, hipStream_t) {
  return INET_ENOSYS;
}
int max_resident(const CompiledRules &, const LaunchShape &, int *, int *) { return INET_ENOSYS; }
int launch_reset(const NetDesc *, const int32_t *, int, int, hipStream_t) { return INET_ENOSYS; }
int launch_admit(const AdmitRec *, int, NetDesc *, int, hipStream_t) { return INET_ENOSYS; }
int launch_zero(int32_t *, int, hipStream_t) { return INET_ENOSYS; }
int launch_jump_grid(const NetDesc *, GridCtl *, uint64_t, int, hipStream_t) { return INET_ENOSYS; }
int jit_function(const CompiledRules &, int, int, hipFunction_t *) { return INET_ENOSYS; }
int jit_launch(const CompiledRules &, const LaunchShape &, int, const NetDesc *, const int32_t *, int,
               int32_t *, const int32_t *, uint32_t, int, const KParams &, hipStream_t) {
  return INET_ENOSYS;
}
int jit_occupancy(const CompiledRules &, const LaunchShape &, int *) { return INET_ENOSYS; }
int jit_grid_launch(const CompiledRules &, const LaunchShape &, int, const NetDesc *, const int32_t *,
                    uint32_t, int, const KParams &, hipStream_t) {
  return INET_ENOSYS;
}
int jit_grid_occupancy(const CompiledRules &, const LaunchShape &, int *) { return INET_ENOSYS; }
}  // namespace inet
