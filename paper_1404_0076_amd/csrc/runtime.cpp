// runtime.cpp -- the C ABI (include/inet.h): loading and validation of nets
// (the configuration <t | Delta> of Section 2.2), device layout, launches,
// results and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"
#include "runtime.h"

using namespace inet;

namespace inet {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

bool plan_net(int64_t n_agents, int64_t n_eqs, int64_t n_names, int64_t agent_cap,
              int64_t name_cap, NetPlan *p) {
  if (agent_cap <= 0) agent_cap = 4 * n_agents + 1024;
  if (name_cap <= 0) name_cap = 4 * n_names + 2 * agent_cap + 1024;
  agent_cap = std::max<int64_t>(agent_cap, n_agents + 2);
  name_cap = std::max<int64_t>(name_cap, n_names + 1);
  // every active pair holds two distinct live agents: the frontier never
  // exceeds agent_cap / 2; the initial equations may be more numerous
  const int64_t qcap = std::max<int64_t>(n_eqs, agent_cap / 2 + 2);
  const int64_t scap = agent_cap / 2 + 2;
  if (agent_cap > kMaxAgentCap || name_cap > kMaxCap || qcap > kMaxCap) return false;
  p->agent_cap = agent_cap;
  p->name_cap = name_cap;
  p->qcap = qcap;
  p->scap = scap;
  p->bytes = al(16 * (size_t)agent_cap) + al(4 * (size_t)name_cap) + 2 * al(8 * (size_t)qcap) +
             al(8 * (size_t)scap);
  return true;
}

size_t global_bytes(const CompiledRules &R, int32_t n_nets, int64_t total_agents, int64_t total_eqs) {
  return al(R.blob.size() * 4) + al(sizeof(NetDesc) * (size_t)n_nets) + al(4 * (size_t)n_nets) +
         256 + al(sizeof(GridCtl)) + al(sizeof(NetState) * (size_t)n_nets) +
         al(8 * (size_t)R.nr * (size_t)n_nets + 8) +
         al(4 * (size_t)total_agents + 4) + al(8 * (size_t)total_agents + 8) +
         al(8 * (size_t)total_eqs + 8);
}

// Validation of one net (Section 2.2): refs in range, every agent attached
// exactly once and below an equation side, every name at most twice.  Fills
// the interface (names occurring once, ascending).
int validate_net(const CompiledRules &R, const int32_t *label, const int32_t *port, int64_t na,
                 const int32_t *eql, const int32_t *eqr, int64_t ne, int32_t nn,
                 std::vector<int32_t> *iface) {
  if (na < 0 || ne < 0 || nn < 0 || na > kMaxAgentCap || nn > kMaxCap) return INET_EINVAL;
  std::vector<int32_t> refs((size_t)na, 0);
  std::vector<int32_t> ncnt((size_t)nn, 0);
  auto use = [&](int32_t v) -> bool {
    if (v >= 0) {
      if (v >= na) return false;
      refs[v]++;
    } else {
      const int64_t x = -1 - (int64_t)v;
      if (x >= nn) return false;
      ncnt[x]++;
    }
    return true;
  };
  for (int64_t i = 0; i < na; i++) {
    const int32_t L = label[i];
    if (L < 0 || L >= R.ns) return INET_EINVAL;
    for (int j = 0; j < R.arity[L]; j++)
      if (!use(port[2 * i + j])) return INET_EINVAL;
  }
  for (int64_t e = 0; e < ne; e++)
    if (!use(eql[e]) || !use(eqr[e])) return INET_EINVAL;
  for (int64_t i = 0; i < na; i++)
    if (refs[i] != 1) return INET_EINVAL;
  for (int32_t x = 0; x < nn; x++)
    if (ncnt[x] > 2) return INET_EINVAL;
  // all agents reachable from the equation sides (no cyclic nesting)
  std::vector<int32_t> stk;
  int64_t reached = 0;
  for (int64_t e = 0; e < ne; e++) {
    for (int32_t root : {eql[e], eqr[e]}) {
      if (root < 0) continue;
      stk.push_back(root);
      while (!stk.empty()) {
        const int32_t a = stk.back();
        stk.pop_back();
        reached++;
        for (int j = 0; j < R.arity[label[a]]; j++) {
          const int32_t c = port[2 * a + j];
          if (c >= 0) stk.push_back(c);
        }
      }
    }
  }
  if (reached != na) return INET_EINVAL;
  iface->clear();
  for (int32_t x = 0; x < nn; x++)
    if (ncnt[x] == 1) iface->push_back(x);
  return INET_OK;
}

LaunchShape effective_shape(const inet_config &cfg, int n_nets, const CompiledRules &R) {
  int wg = cfg.wg_size;
  // 1024-lane engines: for engine 3 a hybrid that steps with wave 0 alone
  // while the frontier fits one wave and with all waves while it is wider
  if (wg <= 0) wg = 1024;
  int engine = cfg.engine;
  if (engine == 0) {
    // the rule table compiled into the kernel when hipRTC can build it
    hipFunction_t f = nullptr;
    engine = jit_function(R, wg, 3, &f) == INET_OK ? 3 : 2;
  }
  LaunchShape sh = shape_for(wg, engine, R.max_links);
  // the LDS tile is a compile-time size of the load-time compiled engines
  if (cfg.qcap > 0 && engine >= 3) sh.qcap = cfg.qcap;
  if (cfg.solo_max > 0 && engine >= 3) sh.solo = cfg.solo_max;
  return sh;
}

bool config_valid(const inet_config &c) {
  if (c.wg_size != 0 && !shape_supported(c.wg_size)) return false;
  if (c.max_resident < 0 || c.engine < 0 || c.engine > 4) return false;
  if (c.solo_max < 0 || c.grid < -1 || c.grid_lo < 0 || c.grid_hi < 0 || c.grid_ppw < 0 ||
      c.timeout_us < 0 || c.round_scale < 0)
    return false;
  if (c.qcap != 0 && (c.qcap < 64 || c.qcap > 8192 || (c.qcap & (c.qcap - 1)))) return false;
  if (c.solo_max > 4096) return false;
  return true;
}

int kparams_for(const inet_config &c, GridCtl *ctl, KParams *kp) {
  static int rate_khz[64] = {0};  // wall-clock rate per device
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INET_EHIP;
  int khz = dev < 64 ? rate_khz[dev] : 0;
  if (khz <= 0) {
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;  // the documented 100 MHz constant clock
    if (dev < 64) rate_khz[dev] = khz;
  }
  *kp = KParams{};
  kp->ctl = ctl;
  kp->grid_lo = c.grid_lo > 0 ? c.grid_lo : 1024;
  kp->grid_hi = std::max(c.grid_hi > 0 ? c.grid_hi : 2048, kp->grid_lo);
  kp->grid_ppw = c.grid_ppw;
  const uint64_t us = c.timeout_us > 0 ? (uint64_t)c.timeout_us : 2000000ull;
  kp->timeout = us * (uint64_t)khz / 1000ull;
  return INET_OK;
}

int resident_grid(const LaunchShape &sh, const CompiledRules &R, const inet_config &cfg,
                  int n_nets, int *grid) {
  *grid = 1;
  if (n_nets <= 1) return INET_OK;
  int per_cu = 0, n_cu = 0;
  int rc = max_resident(R, sh, &per_cu, &n_cu);
  if (rc) return rc;
  int resident = std::max(1, per_cu) * std::max(1, n_cu);
  if (cfg.max_resident > 0) resident = std::min(resident, cfg.max_resident);
  *grid = std::min(n_nets, resident);
  return INET_OK;
}

}  // namespace inet

namespace {
LaunchShape shape_of(const inet_net *h) {
  LaunchShape sh = inet::effective_shape(h->cfg, h->n_nets, h->rules);
  sh.trace = h->tracing ? 1 : 0;
  return sh;
}
}  // namespace

extern "C" {

const char *inet_strerror(int status) {
  switch (status) {
    case INET_OK: return "ok";
    case INET_STUCK: return "reduced; residual active pairs without a rule";
    case INET_EINVAL: return "invalid rules, net, argument or configuration";
    case INET_ENOMEM: return "capacity or workspace exhausted";
    case INET_ELIMIT: return "step limit reached before normal form";
    case INET_ERANGE: return "output buffer too small";
    case INET_EAGAIN: return "no room; retry later";
    case INET_EHIP: return "HIP runtime error";
    case INET_ENOSYS: return "not supported";
    case INET_EINTERNAL: return "internal invariant violated";
    case INET_ETIMEDOUT: return "a workgroup gave up waiting at a barrier";
    default: return "unknown status";
  }
}

int inet_workspace_bytes(const inet_rules *rules, int32_t n_nets, const int64_t *n_agents,
                         const int64_t *n_eqs, const int32_t *n_names, const int64_t *agent_cap,
                         const int64_t *name_cap, size_t *bytes) {
  if (!bytes || n_nets <= 0 || !n_agents || !n_eqs || !n_names) return INET_EINVAL;
  CompiledRules R;
  int rc = compile_rules(rules, &R);
  if (rc) return rc;
  size_t total = 0;
  int64_t ta = 0, te = 0;
  for (int32_t i = 0; i < n_nets; i++) {
    NetPlan p;
    if (!plan_net(n_agents[i], n_eqs[i], n_names[i], agent_cap ? agent_cap[i] : 0,
                  name_cap ? name_cap[i] : 0, &p))
      return INET_EINVAL;
    total += p.bytes;
    ta += n_agents[i];
    te += n_eqs[i];
  }
  *bytes = total + global_bytes(R, n_nets, ta, te) + 256;
  return INET_OK;
}

int inet_batch_load(const inet_rules *rules, int32_t n_nets, const int32_t *label,
                    const int32_t *port, const int64_t *agent_off, const int32_t *eq_lhs,
                    const int32_t *eq_rhs, const int64_t *eq_off, const int32_t *n_names,
                    const int64_t *agent_cap, const int64_t *name_cap, void *dev,
                    size_t dev_bytes, hipStream_t stream, inet_net **out) {
  if (!out || n_nets <= 0 || !agent_off || !eq_off || !n_names || !dev) return INET_EINVAL;
  *out = nullptr;
  inet_net *h = new (std::nothrow) inet_net();
  if (!h) return INET_ENOMEM;
  int rc = compile_rules(rules, &h->rules);
  if (rc) { delete h; return rc; }
  const CompiledRules &R = h->rules;
  h->n_nets = n_nets;
  h->agent_off.assign(agent_off, agent_off + n_nets + 1);
  h->eq_off.assign(eq_off, eq_off + n_nets + 1);
  h->n_names.assign(n_names, n_names + n_nets);
  h->iface.resize(n_nets);
  const int64_t A = agent_off[n_nets], E = eq_off[n_nets];
  if (agent_off[0] != 0 || eq_off[0] != 0 || A < 0 || E < 0 || (A > 0 && (!label || !port)) ||
      (E > 0 && (!eq_lhs || !eq_rhs))) {
    delete h;
    return INET_EINVAL;
  }
  std::vector<NetPlan> plans(n_nets);
  size_t total = 0;
  for (int32_t i = 0; i < n_nets; i++) {
    const int64_t a0 = agent_off[i], a1 = agent_off[i + 1], e0 = eq_off[i], e1 = eq_off[i + 1];
    if (a1 < a0 || e1 < e0) { delete h; return INET_EINVAL; }
    rc = validate_net(R, label + a0, port + 2 * a0, a1 - a0, eq_lhs + e0, eq_rhs + e0, e1 - e0,
                      n_names[i], &h->iface[i]);
    if (rc) { delete h; return rc; }
    if (!plan_net(a1 - a0, e1 - e0, n_names[i], agent_cap ? agent_cap[i] : 0,
                  name_cap ? name_cap[i] : 0, &plans[i])) {
      delete h;
      return INET_EINVAL;
    }
    total += plans[i].bytes;
  }
  const size_t need = total + global_bytes(R, n_nets, A, E) + 256;
  if (dev_bytes < need) { delete h; return INET_ENOMEM; }
  // carve the buffer
  char *base = (char *)(((uintptr_t)dev + 255) & ~uintptr_t(255));
  char *p = base;
  auto take = [&](size_t bytes) { char *q = p; p += al(bytes); return q; };
  h->dev = (char *)dev;
  h->dev_bytes = dev_bytes;
  h->d_rules = (int32_t *)take(R.blob.size() * 4);
  h->d_descs = (NetDesc *)take(sizeof(NetDesc) * (size_t)n_nets);
  h->d_order = (int32_t *)take(4 * (size_t)n_nets);
  h->d_counter = (int32_t *)take(256);
  h->d_grid = (GridCtl *)take(sizeof(GridCtl));
  h->d_states = (NetState *)take(sizeof(NetState) * (size_t)n_nets);
  h->d_per_rule = (unsigned long long *)take(8 * (size_t)R.nr * (size_t)n_nets + 8);
  h->d_init_label = (int32_t *)take(4 * (size_t)A + 4);
  h->d_init_port = (int32_t *)take(8 * (size_t)A + 8);
  h->d_init_eq = (int32_t *)take(8 * (size_t)E + 8);
  h->descs.resize(n_nets);
  for (int32_t i = 0; i < n_nets; i++) {
    const NetPlan &P = plans[i];
    NetDesc &D = h->descs[i];
    D.agent = (int32_t *)take(16 * (size_t)P.agent_cap);
    D.bind = (int32_t *)take(4 * (size_t)P.name_cap);
    D.queue0 = (unsigned long long *)take(8 * (size_t)P.qcap);
    D.queue1 = (unsigned long long *)take(8 * (size_t)P.qcap);
    D.stuck = (unsigned long long *)take(8 * (size_t)P.scap);
    D.per_rule = h->d_per_rule + (size_t)i * R.nr;
    D.st = h->d_states + i;
    D.agent_cap = (int32_t)P.agent_cap;
    D.name_cap = (int32_t)P.name_cap;
    D.qcap = (int32_t)P.qcap;
    D.scap = (int32_t)P.scap;
    D.init_label = h->d_init_label + agent_off[i];
    D.init_port = h->d_init_port + 2 * agent_off[i];
    D.init_eq = h->d_init_eq + 2 * eq_off[i];
    D.n_agents0 = (int32_t)(agent_off[i + 1] - agent_off[i]);
    D.n_eqs0 = (int32_t)(eq_off[i + 1] - eq_off[i]);
    D.n_names0 = n_names[i];
    D.order = i;
  }
  if ((size_t)(p - (char *)dev) > dev_bytes) { delete h; return INET_ENOMEM; }
  h->order.resize(n_nets);
  for (int32_t i = 0; i < n_nets; i++) h->order[i] = i;
  // the equations are uploaded interleaved (lhs, rhs)
  std::vector<int32_t> eqs((size_t)2 * E + 2);
  for (int64_t e = 0; e < E; e++) {
    eqs[2 * e] = eq_lhs[e];
    eqs[2 * e + 1] = eq_rhs[e];
  }
  hipError_t err = hipSuccess;
  err = hipMemcpyAsync(h->d_rules, R.blob.data(), R.blob.size() * 4, hipMemcpyHostToDevice, stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(h->d_descs, h->descs.data(), sizeof(NetDesc) * n_nets, hipMemcpyHostToDevice, stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(h->d_order, h->order.data(), 4 * (size_t)n_nets, hipMemcpyHostToDevice, stream);
  if (err == hipSuccess && A > 0)
    err = hipMemcpyAsync(h->d_init_label, label, 4 * (size_t)A, hipMemcpyHostToDevice, stream);
  if (err == hipSuccess && A > 0)
    err = hipMemcpyAsync(h->d_init_port, port, 8 * (size_t)A, hipMemcpyHostToDevice, stream);
  if (err == hipSuccess && E > 0)
    err = hipMemcpyAsync(h->d_init_eq, eqs.data(), 8 * (size_t)E, hipMemcpyHostToDevice, stream);
  if (err != hipSuccess) { delete h; return INET_EHIP; }
  rc = launch_reset(h->d_descs, nullptr, n_nets, R.nr, stream);
  if (rc == INET_OK && hipStreamSynchronize(stream) != hipSuccess) rc = INET_EHIP;
  if (rc) { delete h; return rc; }
  *out = h;
  return INET_OK;
}

int inet_load(const inet_rules *rules, const int32_t *label, const int32_t *port, int32_t n_agents,
              const int32_t *eq_lhs, const int32_t *eq_rhs, int32_t n_eqs, int32_t n_names,
              int64_t agent_cap, int64_t name_cap, void *dev, size_t dev_bytes, hipStream_t stream,
              inet_net **out) {
  const int64_t aoff[2] = {0, n_agents}, eoff[2] = {0, n_eqs};
  return inet_batch_load(rules, 1, label, port, aoff, eq_lhs, eq_rhs, eoff, &n_names, &agent_cap,
                         &name_cap, dev, dev_bytes, stream, out);
}

int inet_set_config(inet_net *h, const inet_config *cfg) {
  if (!h || !cfg || !config_valid(*cfg)) return INET_EINVAL;
  h->cfg = *cfg;
  return INET_OK;
}

int inet_get_config(const inet_net *h, inet_config *cfg) {
  if (!h || !cfg) return INET_EINVAL;
  *cfg = h->cfg;
  cfg->wg_size = shape_of(h).wg;
  cfg->engine = shape_of(h).engine;
  return INET_OK;
}

int inet_set_order(inet_net *h, const int32_t *order) {
  if (!h || !order) return INET_EINVAL;
  std::vector<char> seen(h->n_nets, 0);
  for (int32_t i = 0; i < h->n_nets; i++) {
    if (order[i] < 0 || order[i] >= h->n_nets || seen[order[i]]) return INET_EINVAL;
    seen[order[i]] = 1;
  }
  h->order.assign(order, order + h->n_nets);
  HIPCHK(hipMemcpy(h->d_order, h->order.data(), 4 * (size_t)h->n_nets, hipMemcpyHostToDevice));
  return INET_OK;
}

// workgroups of the multi-workgroup engine for a handle's single net (0: the
// net runs on one workgroup)
static int grid_workgroups(const inet_net *h, const LaunchShape &sh, int *G) {
  *G = 0;
  if (h->n_nets != 1 || sh.engine != 3 || h->cfg.grid < 0) return INET_OK;
  int per_cu = 0, n_cu = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INET_EHIP;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return INET_EHIP;
  int rc = jit_grid_occupancy(h->rules, sh, &per_cu);
  if (rc) return rc;
  // every workgroup must be resident at once (each posts an entry in every
  // epoch and waits for all the others'): one per compute unit, which needs
  // no more than the engine fitting on a compute unit at all
  if (per_cu < 1) return INET_OK;
  int g = std::max(1, n_cu);
  if (h->cfg.grid > 0) g = std::min(g, h->cfg.grid);
  g = std::min(g, kGridMax);
  *G = g >= 2 ? g : 0;
  return INET_OK;
}

// the reduction of every net of a handle: clear the net counter, the
// persistent launch (the multi-workgroup engine for a single net), the
// pointer-jumping pass (events around the launch if timed)
static int enqueue_reduce(inet_net *h, hipStream_t stream, uint64_t max_steps, bool timed) {
  const LaunchShape sh = shape_of(h);
  const uint32_t ms = (max_steps == 0 || max_steps > kStepsPerLaunch) ? kStepsPerLaunch : (uint32_t)max_steps;
  int grid = 1, G = 0;
  int rc = resident_grid(sh, h->rules, h->cfg, h->n_nets, &grid);
  if (!rc) rc = grid_workgroups(h, sh, &G);
  if (rc) return rc;
  KParams kp;
  rc = kparams_for(h->cfg, G ? h->d_grid : nullptr, &kp);
  if (!rc) rc = launch_zero(h->d_counter, 1, stream);
  if (!rc && G) rc = launch_zero((int32_t *)h->d_grid, (int)(sizeof(GridCtl) / 4), stream);
  if (rc) return rc;
  if (timed) HIPCHK(hipEventRecord(h->ev0, stream));
  const bool jump = h->cfg.jump != 0;
  const int flags = (jump && h->n_nets > 1) ? FLAG_JUMP : 0;
  if (G)
    rc = jit_grid_launch(h->rules, sh, G, h->d_descs, h->d_rules, ms, 0, kp, stream);
  else
    rc = launch_reduce(h->rules, sh, grid, h->d_descs, h->d_order, h->n_nets, h->d_counter,
                       h->d_rules, ms, flags, kp, stream);
  if (rc) return rc;
  if (timed) HIPCHK(hipEventRecord(h->ev1, stream));
  if (jump && h->n_nets == 1) {
    int n_cu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return INET_EHIP;
    // the pointer-jumping barrier uses the scalar words only, not the entries
    rc = launch_zero((int32_t *)h->d_grid, (int)(offsetof(GridCtl, ent) / 4), stream);
    if (!rc) rc = launch_jump_grid(h->d_descs, h->d_grid, kp.timeout, std::max(1, n_cu), stream);
    if (rc) return rc;
  }
  return INET_OK;
}

int inet_reduce_async(inet_net *h, hipStream_t stream, uint64_t max_steps) {
  if (!h) return INET_EINVAL;
  if (!h->ev0) {
    HIPCHK(hipEventCreate(&h->ev0));
    HIPCHK(hipEventCreate(&h->ev1));
  }
  h->results_valid = false;
  int rc = enqueue_reduce(h, stream, max_steps, true);
  if (rc) return rc;
  h->timed = true;
  return INET_OK;
}

int inet_graph_capture(inet_net *h, uint64_t max_steps) {
  if (!h) return INET_EINVAL;
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  int rc = INET_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = INET_EHIP;
  if (rc == INET_OK) rc = launch_reset(h->d_descs, nullptr, h->n_nets, h->rules.nr, cs);
  if (rc == INET_OK) rc = enqueue_reduce(h, cs, max_steps, false);
  if (hipStreamEndCapture(cs, &g) != hipSuccess && rc == INET_OK) rc = INET_EHIP;
  if (rc == INET_OK) {
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
    if (hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) rc = INET_EHIP;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  return rc;
}

int inet_graph_launch(inet_net *h, hipStream_t stream) {
  if (!h || !h->graph_exec) return INET_EINVAL;
  h->results_valid = false;
  h->timed = false;
  HIPCHK(hipGraphLaunch(h->graph_exec, stream));
  return INET_OK;
}

float inet_last_kernel_ms(inet_net *h) {
  if (!h || !h->timed) return -1.0f;
  float ms = -1.0f;
  if (hipEventSynchronize(h->ev1) != hipSuccess) return -1.0f;
  if (hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess) return -1.0f;
  return ms;
}

int inet_results(inet_net *h, hipStream_t stream, inet_result *out) {
  if (!h) return INET_EINVAL;
  HIPCHK(hipStreamSynchronize(stream));
  h->states.resize(h->n_nets);
  HIPCHK(hipMemcpy(h->states.data(), h->d_states, sizeof(NetState) * h->n_nets, hipMemcpyDeviceToHost));
  h->results_valid = true;
  if (out) {
    for (int32_t i = 0; i < h->n_nets; i++) {
      const NetState &s = h->states[i];
      inet_result &r = out[i];
      r.status = s.status;
      r.n_stuck = s.n_stuck;
      r.interactions = s.interactions;
      r.steps = s.steps;
      r.agents_used = s.agent_top;
      r.names_used = s.name_top;
      r.max_frontier = s.max_frontier;
      r.loops = s.loops;
    }
  }
  return INET_OK;
}

int inet_reduce(inet_net *h, hipStream_t stream, uint64_t max_steps, inet_result *out) {
  if (!h) return INET_EINVAL;
  uint64_t done = 0;
  for (int launches = 0;; launches++) {
    uint64_t budget = max_steps ? max_steps - done : 0;
    int rc = inet_reduce_async(h, stream, budget);
    if (rc) return rc;
    rc = inet_results(h, stream, out);
    if (rc) return rc;
    bool again = false;
    for (const NetState &s : h->states)
      if (s.status == ST_ELIMIT && s.phase != PHASE_DONE) again = true;
    done += kStepsPerLaunch;
    if (!again || (max_steps && done >= max_steps) || launches >= 63) break;
  }
  int first_err = INET_OK;
  for (const NetState &s : h->states)
    if (s.status < 0 && first_err == INET_OK) first_err = s.status;
  if (h->n_nets == 1) return h->states[0].status;
  return first_err;
}

int inet_reset(inet_net *h, hipStream_t stream) {
  if (!h) return INET_EINVAL;
  h->results_valid = false;
  return launch_reset(h->d_descs, nullptr, h->n_nets, h->rules.nr, stream);
}

int inet_readback(inet_net *h, int32_t net, int32_t *buf, int64_t cap, int64_t *len) {
  if (!h || net < 0 || net >= h->n_nets || !len) return INET_EINVAL;
  if (!h->results_valid) return INET_EINVAL;
  const NetState &s = h->states[net];
  if (s.status < 0 && s.status != INET_ELIMIT) return s.status;
  if (s.phase != PHASE_DONE) return INET_ELIMIT;
  std::vector<int32_t> stream;
  int rc = readback_net(h->rules, h->descs[net], s, h->iface[net], &stream);
  if (rc) return rc;
  *len = (int64_t)stream.size();
  if (!buf || cap < (int64_t)stream.size()) return INET_ERANGE;
  std::memcpy(buf, stream.data(), stream.size() * 4);
  return INET_OK;
}

int inet_per_rule(inet_net *h, int32_t net, uint64_t *counts, int32_t cap) {
  if (!h || net < 0 || net >= h->n_nets || !counts || cap < h->rules.nr) return INET_EINVAL;
  if (h->rules.nr == 0) return INET_OK;
  HIPCHK(hipMemcpy(counts, h->d_per_rule + (size_t)net * h->rules.nr, 8 * (size_t)h->rules.nr,
                   hipMemcpyDeviceToHost));
  return INET_OK;
}

int inet_set_trace(inet_net *h, int32_t net, int32_t *d_buf, int64_t cap) {
  if (!h || net < 0 || net >= h->n_nets || cap < 0 || (cap > 0 && !d_buf)) return INET_EINVAL;
  NetDesc &D = h->descs[net];
  D.trace = cap > 0 ? d_buf : nullptr;
  D.trace_cap = (int32_t)std::min<int64_t>(cap, INT32_MAX);
  HIPCHK(hipMemcpy(h->d_descs + net, &D, sizeof(NetDesc), hipMemcpyHostToDevice));
  h->tracing = false;
  for (const NetDesc &d : h->descs)
    if (d.trace) h->tracing = true;
  return INET_OK;
}

int inet_cells(inet_net *h, int32_t net, int32_t *buf, int64_t cap, int64_t *len) {
  if (!h || net < 0 || net >= h->n_nets || !len) return INET_EINVAL;
  if (!h->results_valid) return INET_EINVAL;
  const NetState &s = h->states[net];
  const int64_t n = std::max<int32_t>(0, s.name_top);
  *len = n;
  if (!buf || cap < n) return INET_ERANGE;
  if (n) HIPCHK(hipMemcpy(buf, h->descs[net].bind, 4 * (size_t)n, hipMemcpyDeviceToHost));
  return INET_OK;
}

int inet_rule_bytes(const inet_net *h, int32_t *bytes, int32_t cap) {
  if (!h || !bytes || cap < h->rules.nr) return INET_EINVAL;
  for (int i = 0; i < h->rules.nr; i++) bytes[i] = h->rules.bytes[i];
  return INET_OK;
}

int inet_rules_check(const inet_rules *rules, int32_t *n_new, int32_t *n_fresh, int32_t *n_links,
                     int32_t *bytes, int32_t cap) {
  CompiledRules R;
  int rc = compile_rules(rules, &R);
  if (rc) return rc;
  if ((n_new || n_fresh || n_links || bytes) && cap < R.nr) return INET_ERANGE;
  for (int k = 0; k < R.nr; k++) {
    const int32_t *T = &R.templ[(size_t)k * RT_WORDS];
    if (n_new) n_new[k] = T[RT_NNEW];
    if (n_fresh) n_fresh[k] = T[RT_NFRESH];
    if (n_links) n_links[k] = T[RT_NEQ];
    if (bytes) bytes[k] = R.bytes[k];
  }
  return INET_OK;
}

int32_t inet_num_nets(const inet_net *h) { return h ? h->n_nets : 0; }

void inet_free(inet_net *h) {
  if (!h) return;
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
}

}  // extern "C"
