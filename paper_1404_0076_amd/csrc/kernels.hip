// kernels.hip -- ahead-of-time instances of the device code (device.h) and
// their host-side launchers.
#include <hip/hip_runtime.h>

#include "device.h"
#include "inet_internal.h"
#include "runtime.h"

namespace inet {

// ---------------------------------------------------------------------------
// launchers

namespace {
// kernel instance for an engine and the largest link count of the rule table
// (engine 2 is compiled for rules with at most 4 links and for the maximum)
template <int WG, int QCAP>
const void *kernel_for(int engine, int maxl) {
  if (engine == 1) return (const void *)&k_reduce<WG, QCAP, 1, MAXEQ>;
  if (maxl <= 4) return (const void *)&k_reduce<WG, QCAP, 2, 4>;
  return (const void *)&k_reduce<WG, QCAP, 2, MAXEQ>;
}

template <int WG, int QCAP>
int launch_t(int engine, int maxl, int grid, const NetDesc *d, const int32_t *ord, int n,
             int32_t *ctr, const int32_t *r, int ns, int nr, uint32_t ms, int flags,
             const KParams &kp, hipStream_t s) {
  const size_t dyn = (size_t)(ns * ns + nr * RT_WORDS + ns) * 4;
  if (engine == 1)
    hipLaunchKernelGGL((k_reduce<WG, QCAP, 1, MAXEQ>), dim3(grid), dim3(WG), dyn, s, d, ord, n, ctr,
                       r, ns, nr, ms, flags, kp);
  else if (maxl <= 4)
    hipLaunchKernelGGL((k_reduce<WG, QCAP, 2, 4>), dim3(grid), dim3(WG), dyn, s, d, ord, n, ctr, r,
                       ns, nr, ms, flags, kp);
  else
    hipLaunchKernelGGL((k_reduce<WG, QCAP, 2, MAXEQ>), dim3(grid), dim3(WG), dyn, s, d, ord, n, ctr,
                       r, ns, nr, ms, flags, kp);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

template <int WG, int QCAP>
int occ_t(int engine, int maxl, int ns, int nr, int *per_cu) {
  const size_t dyn = (size_t)(ns * ns + nr * RT_WORDS + ns) * 4;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel_for<WG, QCAP>(engine, maxl),
                                                      WG, dyn) == hipSuccess
             ? INET_OK
             : INET_EHIP;
}
}  // namespace

bool shape_supported(int wg) {
  return wg == 64 || wg == 128 || wg == 256 || wg == 512 || wg == 1024;
}

LaunchShape shape_for(int wg, int engine, int maxl) {
  const int e = (engine == 1 || engine == 3 || engine == 4) ? engine : 2;
  switch (wg) {
    case 64: return {64, 512, e, maxl};
    case 128: return {128, 1024, e, maxl};
    case 256: return {256, 1024, e, maxl};
    case 512: return {512, 2048, e, maxl};
    default: return {1024, 4096, e, maxl};
  }
}

#define INET_SHAPES(X) X(64, 512) X(128, 1024) X(256, 1024) X(512, 2048) X(1024, 4096)

int launch_reduce(const CompiledRules &R, const LaunchShape &sh, int grid, const NetDesc *d,
                  const int32_t *ord, int n, int32_t *ctr, const int32_t *r, uint32_t ms, int flags,
                  const KParams &kp, hipStream_t s) {
  if (sh.engine >= 3) return jit_launch(R, sh, grid, d, ord, n, ctr, r, ms, flags, kp, s);
  const int ns = R.ns, nr = R.nr;
#define X(W, Q) \
  if (sh.wg == W && sh.qcap == Q)    \
    return launch_t<W, Q>(sh.engine, sh.maxl, grid, d, ord, n, ctr, r, ns, nr, ms, flags, kp, s);
  INET_SHAPES(X)
#undef X
  return INET_EINVAL;
}

int max_resident(const CompiledRules &R, const LaunchShape &sh, int *per_cu, int *n_cu) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INET_EHIP;
  if (hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return INET_EHIP;
  if (sh.engine >= 3) return jit_occupancy(R, sh, per_cu);
  const int ns = R.ns, nr = R.nr;
#define X(W, Q) \
  if (sh.wg == W && sh.qcap == Q) return occ_t<W, Q>(sh.engine, sh.maxl, ns, nr, per_cu);
  INET_SHAPES(X)
#undef X
  return INET_EINVAL;
}

int launch_reset(const NetDesc *d, const int32_t *idx, int n, int nr, hipStream_t s) {
  const int grid = n < 4096 ? n : 4096;
  if (grid <= 0) return INET_OK;
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, s, d, idx, n, nr);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

int launch_admit(const AdmitRec *d_recs, int n, NetDesc *d_descs, int nr, hipStream_t s) {
  const int grid = n < 4096 ? n : 4096;
  if (grid <= 0) return INET_OK;
  hipLaunchKernelGGL(k_admit, dim3(grid), dim3(256), 0, s, d_recs, n, d_descs, nr);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

int launch_zero(int32_t *p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

int launch_jump_grid(const NetDesc *d, GridCtl *ctl, uint64_t timeout, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_jump_grid, dim3(grid), dim3(256), 0, s, d, ctl,
                     (unsigned long long)timeout);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

}  // namespace inet
