// runtime.h -- host-side structures of the evaluator (internal).
#ifndef INET_RUNTIME_H
#define INET_RUNTIME_H

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"

namespace inet {

struct CompiledRules {
  int ns = 0, nr = 0;
  std::vector<int32_t> arity;
  std::vector<int32_t> rule_of;     // [ns*ns] 2*rule+swap or -1
  std::vector<int32_t> templ;       // [nr*RT_WORDS]
  std::vector<int32_t> blob;        // device image: rule_of | templ | arity
  std::vector<int32_t> bytes;       // algorithmic bytes per interaction of each rule
  std::vector<int32_t> rhs_agents;  // agents in each literal right-hand side
  int max_links = 0;                // largest link count of any compiled rule
};

int compile_rules(const inet_rules *r, CompiledRules *out);

// kernel launchers (kernels.hip)
struct LaunchShape {
  int wg;
  int qcap;    // LDS frontier capacity per buffer
  int engine;  // 1: per-lane template interpreter, 2: rule-uniform execution,
               // 3: rule-uniform with the rule table compiled in (load time),
               // 4: engine 3 with per-lane atomic reservations (atomic append)
  int maxl;    // largest number of link equations of any rule
  int trace = 0;  // engines 3 and 4: the kernel variant that records per-step pair counts
  int solo = 64;  // engine 3: one-wave steps while at most this many pairs are active
};
int launch_reset(const NetDesc *d_descs, const int32_t *d_idx, int n, int nr, hipStream_t s);
int launch_admit(const AdmitRec *d_recs, int n, NetDesc *d_descs, int nr, hipStream_t s);
int launch_zero(int32_t *p, int n, hipStream_t s);
int launch_reduce(const CompiledRules &R, const LaunchShape &shape, int grid,
                  const NetDesc *d_descs, const int32_t *d_order, int n_nets, int32_t *d_counter,
                  const int32_t *d_rules, uint32_t max_steps, int flags, const KParams &kp,
                  hipStream_t s);
int launch_jump_grid(const NetDesc *d_desc, GridCtl *ctl, uint64_t timeout, int grid,
                     hipStream_t s);
int max_resident(const CompiledRules &R, const LaunchShape &shape, int *per_cu, int *n_cu);
// engines 3 and 4: the rule table compiled into the kernel at load time (jit.cpp)
int jit_function(const CompiledRules &R, int wg, int engine, hipFunction_t *out);
int jit_launch(const CompiledRules &R, const LaunchShape &sh, int grid, const NetDesc *d,
               const int32_t *ord, int n, int32_t *ctr, const int32_t *r, uint32_t ms, int flags,
               const KParams &kp, hipStream_t s);
int jit_occupancy(const CompiledRules &R, const LaunchShape &sh, int *per_cu);
// the multi-workgroup engine of one net (engine 3): kernel, launch, occupancy
int jit_grid_launch(const CompiledRules &R, const LaunchShape &sh, int grid, const NetDesc *d,
                    const int32_t *r, uint32_t ms, int flags, const KParams &kp, hipStream_t s);
int jit_grid_occupancy(const CompiledRules &R, const LaunchShape &sh, int *per_cu);
// configuration checks and the kernel tunables it selects (ctl: the
// multi-workgroup control block, or null)
bool config_valid(const inet_config &c);
int kparams_for(const inet_config &c, GridCtl *ctl, KParams *kp);
bool shape_supported(int wg);
LaunchShape shape_for(int wg, int engine, int maxl);


constexpr uint32_t kStepsPerLaunch = 1u << 24;  // bound on one launch of an unbounded reduce
constexpr int64_t kMaxCap = (int64_t(1) << 29) - 16;  // byte offsets of 8-byte entries fit 32 bits
constexpr int64_t kMaxAgentCap = (int64_t(1) << 28) - 16;  // and those of 16-byte agent records

struct NetPlan {
  int64_t agent_cap, name_cap, qcap, scap;
  size_t bytes;
};
size_t al(size_t x);
// device bytes of a handle's shared arrays (rules, descriptors, states, ...)
size_t global_bytes(const CompiledRules &R, int32_t n_nets, int64_t total_agents, int64_t total_eqs);
bool plan_net(int64_t n_agents, int64_t n_eqs, int64_t n_names, int64_t agent_cap, int64_t name_cap,
              NetPlan *p);
int validate_net(const CompiledRules &R, const int32_t *label, const int32_t *port, int64_t na,
                 const int32_t *eql, const int32_t *eqr, int64_t ne, int32_t nn,
                 std::vector<int32_t> *iface);
LaunchShape effective_shape(const inet_config &cfg, int n_nets, const CompiledRules &R);
int resident_grid(const LaunchShape &sh, const CompiledRules &R, const inet_config &cfg, int n_nets,
                  int *grid);
int canonical_stream(const CompiledRules &R, const int32_t *label, const int32_t *p0,
                     const int32_t *p1, int64_t n_agents, const int32_t *bind, int64_t n_cells,
                     const std::vector<int32_t> &iface, const std::vector<int2> &stuck,
                     std::vector<int32_t> *out);
// copy one finished net's heap to the host and write its canonical stream
int readback_net(const CompiledRules &R, const NetDesc &D, const NetState &s,
                 const std::vector<int32_t> &iface, std::vector<int32_t> *out);

}  // namespace inet

#define HIPCHK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return INET_EHIP;       \
  } while (0)

struct inet_net {
  inet::CompiledRules rules;
  int32_t n_nets = 0;
  char *dev = nullptr;
  size_t dev_bytes = 0;
  // device pointers into dev
  int32_t *d_rules = nullptr;
  inet::NetDesc *d_descs = nullptr;
  int32_t *d_order = nullptr;
  int32_t *d_counter = nullptr;
  int32_t *d_init_label = nullptr;
  int32_t *d_init_port = nullptr;
  int32_t *d_init_eq = nullptr;
  std::vector<inet::NetDesc> descs;       // host copy of the descriptors
  std::vector<int32_t> order;             // launch order
  std::vector<int64_t> agent_off, eq_off;
  std::vector<int32_t> n_names;
  std::vector<std::vector<int32_t>> iface; // interface name ids per net
  inet::GridCtl *d_grid = nullptr;        // multi-workgroup control block (one net)
  inet::NetState *d_states = nullptr;     // [n_nets], contiguous
  unsigned long long *d_per_rule = nullptr; // [n_nets][nr], contiguous
  std::vector<inet::NetState> states;     // from the last inet_results
  bool results_valid = false;
  inet_config cfg{0, 1, 0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool timed = false;
  bool tracing = false;                   // some net has a per-step trace buffer
  inet::NetState *h_states = nullptr;     // pinned staging
};

#endif
