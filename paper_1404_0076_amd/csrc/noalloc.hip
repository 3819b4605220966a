// noalloc.hip -- inet_reduce_noalloc: load, reduce and read back one net
// without allocating device memory, for callers that cannot allocate.
//
// Everything the kernels work on besides the caller's inputs and outputs --
// the rule table, the net's descriptor and state, its agent heap, name cells,
// frontier queues, residual list and initial image, the net counter and the
// pointer-jumping control block -- is carved out of `scratch`, a file-scope
// device array of kScratchBytes.  Each device the library runs on holds its
// own copy until the process ends.  Host code never uses the array's name as
// an address: on the first call on a device its address there is looked up
// with hipGetSymbolAddress and kept per device.  The reduction uses the
// ahead-of-time engine (engine 2, 1024 lanes), so no code object is loaded
// either.  Calls that overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"
#include "runtime.h"

namespace inet {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // INET_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == (size_t)INET_NOALLOC_SCRATCH_BYTES, "header and library disagree");

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {nullptr};  // the array's device address, per device

// the array's address on the current device (looked up once per device)
int scratch_ptr(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INET_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return INET_ENOSYS;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return INET_EHIP;
    g_ptr[dev] = (char *)p;
  }
  *out = g_ptr[dev];
  return INET_OK;
}

}  // namespace
}  // namespace inet

using namespace inet;

extern "C" int inet_reduce_noalloc(const inet_rules *rules, const int32_t *label,
                                   const int32_t *port, int32_t n_agents, const int32_t *eq_lhs,
                                   const int32_t *eq_rhs, int32_t n_eqs, int32_t n_names,
                                   int64_t agent_cap, int64_t name_cap, uint64_t max_steps,
                                   hipStream_t stream, inet_result *out, int32_t *nf,
                                   int64_t nf_cap, int64_t *nf_len) {
  if (!out || n_agents < 0 || n_eqs < 0 || n_names < 0 || nf_cap < 0) return INET_EINVAL;
  if ((n_agents && (!label || !port)) || (n_eqs && (!eq_lhs || !eq_rhs))) return INET_EINVAL;
  char *base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  CompiledRules R;
  rc = compile_rules(rules, &R);
  if (rc) return rc;
  std::vector<int32_t> iface;
  rc = validate_net(R, label, port, n_agents, eq_lhs, eq_rhs, n_eqs, n_names, &iface);
  if (rc) return rc;
  NetPlan P;
  if (!plan_net(n_agents, n_eqs, n_names, agent_cap, name_cap, &P)) return INET_EINVAL;
  // the same layout as a loaded batch of one net, inside the array
  const size_t need = P.bytes + global_bytes(R, 1, n_agents, n_eqs) + 256;
  if (need > kScratchBytes) return INET_ENOMEM;
  char *p = base;
  auto take = [&](size_t bytes) { char *q = p; p += al(bytes); return q; };
  int32_t *d_rules = (int32_t *)take(R.blob.size() * 4);
  NetDesc *d_desc = (NetDesc *)take(sizeof(NetDesc));
  int32_t *d_order = (int32_t *)take(4);
  int32_t *d_counter = (int32_t *)take(256);
  GridCtl *d_grid = (GridCtl *)take(sizeof(GridCtl));
  NetState *d_state = (NetState *)take(sizeof(NetState));
  unsigned long long *d_per_rule = (unsigned long long *)take(8 * (size_t)R.nr + 8);
  int32_t *d_label = (int32_t *)take(4 * (size_t)n_agents + 4);
  int32_t *d_port = (int32_t *)take(8 * (size_t)n_agents + 8);
  int32_t *d_eq = (int32_t *)take(8 * (size_t)n_eqs + 8);
  NetDesc D{};
  D.agent = (int32_t *)take(16 * (size_t)P.agent_cap);
  D.bind = (int32_t *)take(4 * (size_t)P.name_cap);
  D.queue0 = (unsigned long long *)take(8 * (size_t)P.qcap);
  D.queue1 = (unsigned long long *)take(8 * (size_t)P.qcap);
  D.stuck = (unsigned long long *)take(8 * (size_t)P.scap);
  if ((size_t)(p - base) > kScratchBytes) return INET_ENOMEM;
  D.per_rule = d_per_rule;
  D.st = d_state;
  D.agent_cap = (int32_t)P.agent_cap;
  D.name_cap = (int32_t)P.name_cap;
  D.qcap = (int32_t)P.qcap;
  D.scap = (int32_t)P.scap;
  D.init_label = d_label;
  D.init_port = d_port;
  D.init_eq = d_eq;
  D.n_agents0 = n_agents;
  D.n_eqs0 = n_eqs;
  D.n_names0 = n_names;
  D.order = 0;
  std::vector<int32_t> eqs((size_t)2 * n_eqs + 2);
  for (int32_t e = 0; e < n_eqs; e++) {
    eqs[2 * e] = eq_lhs[e];
    eqs[2 * e + 1] = eq_rhs[e];
  }
  const int32_t zero = 0;
  HIPCHK(hipMemcpyAsync(d_rules, R.blob.data(), R.blob.size() * 4, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(d_desc, &D, sizeof(NetDesc), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(d_order, &zero, 4, hipMemcpyHostToDevice, stream));
  if (n_agents) {
    HIPCHK(hipMemcpyAsync(d_label, label, 4 * (size_t)n_agents, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(d_port, port, 8 * (size_t)n_agents, hipMemcpyHostToDevice, stream));
  }
  if (n_eqs)
    HIPCHK(hipMemcpyAsync(d_eq, eqs.data(), 8 * (size_t)n_eqs, hipMemcpyHostToDevice, stream));
  // the state the previous call left behind is overwritten here: reset
  // writes the initial image, the cells, the counters and the net state
  rc = launch_reset(d_desc, nullptr, 1, R.nr, stream);
  if (rc) return rc;
  inet_config cfg{};
  cfg.jump = 1;
  KParams kp;
  rc = kparams_for(cfg, nullptr, &kp);
  if (rc) return rc;
  const LaunchShape sh = shape_for(1024, 2, R.max_links);
  int n_cu = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return INET_EHIP;
  NetState st{};
  uint64_t done = 0;
  for (int launches = 0;; launches++) {
    const uint64_t left = max_steps ? max_steps - done : 0;
    const uint32_t ms = (left == 0 || left > kStepsPerLaunch) ? kStepsPerLaunch : (uint32_t)left;
    rc = launch_zero(d_counter, 1, stream);
    if (!rc) rc = launch_reduce(R, sh, 1, d_desc, d_order, 1, d_counter, d_rules, ms, 0, kp, stream);
    if (!rc) rc = launch_zero((int32_t *)d_grid, (int)(offsetof(GridCtl, ent) / 4), stream);
    if (!rc) rc = launch_jump_grid(d_desc, d_grid, kp.timeout, std::max(1, n_cu), stream);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(&st, d_state, sizeof(NetState), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    done += ms;
    if (!(st.status == ST_ELIMIT && st.phase != PHASE_DONE) || (max_steps && done >= max_steps) ||
        launches >= 63)
      break;
  }
  out->status = st.status;
  out->n_stuck = st.n_stuck;
  out->interactions = st.interactions;
  out->steps = st.steps;
  out->agents_used = st.agent_top;
  out->names_used = st.name_top;
  out->max_frontier = st.max_frontier;
  out->loops = st.loops;
  if (!nf_len) return st.status;
  *nf_len = 0;
  if (st.status < 0 || st.phase != PHASE_DONE) return st.status;
  std::vector<int32_t> stream_out;
  rc = readback_net(R, D, st, iface, &stream_out);
  if (rc) return rc;
  *nf_len = (int64_t)stream_out.size();
  if (!nf || nf_cap < *nf_len) return INET_ERANGE;
  if (!stream_out.empty()) std::memcpy(nf, stream_out.data(), 4 * stream_out.size());
  return st.status;
}
