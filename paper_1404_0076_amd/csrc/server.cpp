// server.cpp -- continuous batching over the net engines.
//
// Nets are admitted into slots while others are being reduced: each admitted
// net gets a region of the caller's device buffer (first-fit over free byte
// ranges; no room -> INET_EAGAIN), its image is uploaded and reset on the
// caller's upload stream, and from the next round on it runs with every other
// resident net.  A round is one launch of the persistent reduction kernel
// over the running slots with a bounded step budget; a net that is not done
// keeps its heap and its saved frontier resident for the next round.  Finished
// nets are harvested by polling; their slot and memory return on release.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"
#include "runtime.h"

using namespace inet;

struct inet_server {
  CompiledRules rules;
  int32_t max_slots = 0;
  char *dev = nullptr;
  size_t dev_bytes = 0;
  int32_t *d_rules = nullptr;
  NetDesc *d_descs = nullptr;
  int32_t *d_order = nullptr;
  int32_t *d_counter = nullptr;
  NetState *d_states = nullptr;
  unsigned long long *d_per_rule = nullptr;
  int32_t *d_idx = nullptr;
  size_t arena_lo = 0, arena_hi = 0;     // byte offsets into dev
  std::map<size_t, size_t> free_ranges;  // offset -> length
  size_t free_bytes = 0;
  struct Slot {
    int state = 0;  // 0 free, 1 running, 2 finished
    int64_t ticket = 0;
    size_t off = 0, len = 0;
    NetDesc desc{};
    NetState st{};
    std::vector<int32_t> iface;
    std::vector<int32_t> eqs;  // interleaved equations, kept until release
  };
  std::vector<Slot> slots;
  std::vector<int32_t> free_slots;
  std::unordered_map<int64_t, int32_t> by_ticket;
  int64_t next_ticket = 1;
  std::vector<int32_t> running;
  std::vector<int32_t> order_host;
  std::vector<int32_t> finished;  // slots finished but not yet reported by poll
  std::vector<NetState> h_states;
  inet_config cfg{0, 1, 0, 0};
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  bool round_in_flight = false;
};

namespace {

bool take_range(inet_server *s, size_t len, size_t *off) {
  for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
    if (it->second >= len) {
      *off = it->first;
      const size_t rest = it->second - len;
      const size_t at = it->first + len;
      s->free_ranges.erase(it);
      if (rest) s->free_ranges[at] = rest;
      s->free_bytes -= len;
      return true;
    }
  }
  return false;
}

void give_range(inet_server *s, size_t off, size_t len) {
  auto it = s->free_ranges.emplace(off, len).first;
  s->free_bytes += len;
  auto next = std::next(it);
  if (next != s->free_ranges.end() && it->first + it->second == next->first) {
    it->second += next->second;
    s->free_ranges.erase(next);
  }
  if (it != s->free_ranges.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      s->free_ranges.erase(it);
    }
  }
}

inet_server::Slot *slot_of(inet_server *s, int64_t ticket) {
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return nullptr;
  return &s->slots[it->second];
}

// a round's step budget: `steps`, or with round_scale set, `steps` times the
// running nets per resident engine (at least 1, at most round_scale), so that
// under load, when every engine already steps several nets in a round, a long
// net needs fewer rounds
uint32_t round_budget(const inet_config &cfg, uint32_t steps, int n, int grid) {
  if (cfg.round_scale <= 1 || grid <= 0) return steps;
  uint64_t k = (uint64_t)(n / grid);
  if (k < 1) k = 1;
  if (k > (uint64_t)cfg.round_scale) k = (uint64_t)cfg.round_scale;
  const uint64_t b = (uint64_t)steps * k;
  return b > 0xffffffffull ? 0xffffffffu : (uint32_t)b;
}

}  // namespace

extern "C" {

int inet_server_create(const inet_rules *rules, int32_t max_slots, void *dev, size_t dev_bytes,
                       inet_server **out) {
  if (!out || max_slots <= 0 || !dev) return INET_EINVAL;
  *out = nullptr;
  inet_server *s = new (std::nothrow) inet_server();
  if (!s) return INET_ENOMEM;
  int rc = compile_rules(rules, &s->rules);
  if (rc) { delete s; return rc; }
  const CompiledRules &R = s->rules;
  s->max_slots = max_slots;
  s->dev = (char *)dev;
  s->dev_bytes = dev_bytes;
  char *base = (char *)(((uintptr_t)dev + 255) & ~uintptr_t(255));
  char *p = base;
  auto take = [&](size_t bytes) { char *q = p; p += al(bytes); return q; };
  s->d_rules = (int32_t *)take(R.blob.size() * 4);
  s->d_descs = (NetDesc *)take(sizeof(NetDesc) * (size_t)max_slots);
  s->d_order = (int32_t *)take(4 * (size_t)max_slots);
  s->d_counter = (int32_t *)take(256);
  s->d_states = (NetState *)take(sizeof(NetState) * (size_t)max_slots);
  s->d_per_rule = (unsigned long long *)take(8 * (size_t)R.nr * (size_t)max_slots + 8);
  s->d_idx = (int32_t *)take(4 * (size_t)max_slots);
  if ((size_t)(p - (char *)dev) + 4096 > dev_bytes) { delete s; return INET_ENOMEM; }
  s->arena_lo = (size_t)(p - (char *)dev);
  s->arena_hi = dev_bytes & ~size_t(255);
  s->free_ranges[s->arena_lo] = s->arena_hi - s->arena_lo;
  s->free_bytes = s->arena_hi - s->arena_lo;
  s->slots.resize(max_slots);
  for (int32_t i = max_slots - 1; i >= 0; i--) s->free_slots.push_back(i);
  std::vector<int32_t> idx(max_slots);
  for (int32_t i = 0; i < max_slots; i++) idx[i] = i;
  std::vector<NetState> zero(max_slots);
  hipError_t e = hipMemcpy(s->d_rules, R.blob.data(), R.blob.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->d_idx, idx.data(), 4 * (size_t)max_slots, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_states, zero.data(), sizeof(NetState) * (size_t)max_slots, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->upload_done, hipEventDisableTiming);
  if (e != hipSuccess) { delete s; return INET_EHIP; }
  *out = s;
  return INET_OK;
}

int inet_server_set_config(inet_server *s, const inet_config *cfg) {
  if (!s || !cfg || !config_valid(*cfg)) return INET_EINVAL;
  s->cfg = *cfg;
  return INET_OK;
}

int inet_server_submit(inet_server *s, const int32_t *label, const int32_t *port, int32_t n_agents,
                       const int32_t *eq_lhs, const int32_t *eq_rhs, int32_t n_eqs, int32_t n_names,
                       int64_t agent_cap, int64_t name_cap, hipStream_t stream, int64_t *ticket) {
  if (!s || !ticket || n_agents < 0 || n_eqs < 0 || n_names < 0) return INET_EINVAL;
  if ((n_agents && (!label || !port)) || (n_eqs && (!eq_lhs || !eq_rhs))) return INET_EINVAL;
  const CompiledRules &R = s->rules;
  std::vector<int32_t> iface;
  int rc = validate_net(R, label, port, n_agents, eq_lhs, eq_rhs, n_eqs, n_names, &iface);
  if (rc) return rc;
  NetPlan P;
  if (!plan_net(n_agents, n_eqs, n_names, agent_cap, name_cap, &P)) return INET_EINVAL;
  const size_t len = P.bytes + al(4 * (size_t)n_agents + 4) + al(8 * (size_t)n_agents + 8) +
                     al(8 * (size_t)n_eqs + 8);
  if (s->free_slots.empty()) return INET_EAGAIN;
  size_t off = 0;
  if (!take_range(s, len, &off)) return INET_EAGAIN;
  const int32_t si = s->free_slots.back();
  s->free_slots.pop_back();
  inet_server::Slot &S = s->slots[si];
  S = inet_server::Slot();
  S.state = 1;
  S.ticket = s->next_ticket++;
  S.off = off;
  S.len = len;
  S.iface.swap(iface);
  S.eqs.resize((size_t)2 * n_eqs + 2);
  for (int32_t e = 0; e < n_eqs; e++) {
    S.eqs[2 * e] = eq_lhs[e];
    S.eqs[2 * e + 1] = eq_rhs[e];
  }
  char *p = s->dev + off;
  auto take = [&](size_t bytes) { char *q = p; p += al(bytes); return q; };
  NetDesc &D = S.desc;
  D.agent = (int32_t *)take(16 * (size_t)P.agent_cap);
  D.bind = (int32_t *)take(4 * (size_t)P.name_cap);
  D.queue0 = (unsigned long long *)take(8 * (size_t)P.qcap);
  D.queue1 = (unsigned long long *)take(8 * (size_t)P.qcap);
  D.stuck = (unsigned long long *)take(8 * (size_t)P.scap);
  int32_t *il = (int32_t *)take(4 * (size_t)n_agents + 4);
  int32_t *ip = (int32_t *)take(8 * (size_t)n_agents + 8);
  int32_t *ie = (int32_t *)take(8 * (size_t)n_eqs + 8);
  D.init_label = il;
  D.init_port = ip;
  D.init_eq = ie;
  D.per_rule = s->d_per_rule + (size_t)si * R.nr;
  D.st = s->d_states + si;
  D.agent_cap = (int32_t)P.agent_cap;
  D.name_cap = (int32_t)P.name_cap;
  D.qcap = (int32_t)P.qcap;
  D.scap = (int32_t)P.scap;
  D.n_agents0 = n_agents;
  D.n_eqs0 = n_eqs;
  D.n_names0 = n_names;
  D.order = si;
  hipError_t e = hipSuccess;
  if (n_agents) e = hipMemcpyAsync(il, label, 4 * (size_t)n_agents, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && n_agents)
    e = hipMemcpyAsync(ip, port, 8 * (size_t)n_agents, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && n_eqs)
    e = hipMemcpyAsync(ie, S.eqs.data(), 8 * (size_t)n_eqs, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_descs + si, &S.desc, sizeof(NetDesc), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return INET_EHIP;
  rc = launch_reset(s->d_descs, s->d_idx + si, 1, R.nr, stream);
  if (rc) return rc;
  HIPCHK(hipEventRecord(s->upload_done, stream));
  s->upload_pending = true;
  s->running.push_back(si);
  s->by_ticket[S.ticket] = si;
  *ticket = S.ticket;
  return INET_OK;
}

int inet_server_step(inet_server *s, hipStream_t stream, uint32_t max_steps) {
  if (!s || max_steps == 0) return INET_EINVAL;
  if (s->round_in_flight) return INET_EINVAL;
  if (s->running.empty()) return INET_OK;
  if (s->upload_pending) {
    HIPCHK(hipStreamWaitEvent(stream, s->upload_done, 0));
    s->upload_pending = false;
  }
  const int n = (int)s->running.size();
  s->order_host = s->running;
  HIPCHK(hipMemcpyAsync(s->d_order, s->order_host.data(), 4 * (size_t)n, hipMemcpyHostToDevice, stream));
  const inet_config &cfg = s->cfg;
  const LaunchShape sh = effective_shape(cfg, n > 1 ? n : 2, s->rules);
  int grid = 1;
  int rc = resident_grid(sh, s->rules, cfg, n, &grid);
  if (rc) return rc;
  rc = launch_zero(s->d_counter, 1, stream);
  if (rc) return rc;
  KParams kp;
  rc = kparams_for(cfg, nullptr, &kp);
  if (rc) return rc;
  rc = launch_reduce(s->rules, sh, grid, s->d_descs, s->d_order, n, s->d_counter, s->d_rules,
                     round_budget(cfg, max_steps, n, grid), s->cfg.jump ? FLAG_JUMP : 0, kp,
                     stream);
  if (rc) return rc;
  s->round_in_flight = true;
  return INET_OK;
}

int inet_server_poll(inet_server *s, hipStream_t stream, int64_t *done, int32_t cap,
                     int32_t *n_done) {
  if (!s || !n_done || (cap > 0 && !done)) return INET_EINVAL;
  *n_done = 0;
  if (s->round_in_flight) {
    HIPCHK(hipStreamSynchronize(stream));
    s->round_in_flight = false;
    s->h_states.resize(s->max_slots);
    HIPCHK(hipMemcpy(s->h_states.data(), s->d_states, sizeof(NetState) * (size_t)s->max_slots,
                     hipMemcpyDeviceToHost));
    // only nets that took part in the round are judged: a net admitted on
    // another stream during the round may not have been reset yet
    std::vector<char> in_round(s->max_slots, 0);
    for (int32_t si : s->order_host) in_round[si] = 1;
    std::vector<int32_t> still;
    for (int32_t si : s->running) {
      const NetState &st = s->h_states[si];
      inet_server::Slot &S = s->slots[si];
      const bool over = in_round[si] && (st.phase == PHASE_DONE || st.status == ST_ENOMEM ||
                                         st.status == ST_EINTERNAL);
      if (over) {
        S.state = 2;
        S.st = st;
        s->finished.push_back(si);
      } else {
        still.push_back(si);
      }
    }
    s->running.swap(still);
  }
  int32_t k = 0;
  while (k < cap && !s->finished.empty()) {
    done[k++] = s->slots[s->finished.front()].ticket;
    s->finished.erase(s->finished.begin());
  }
  *n_done = k;
  return INET_OK;
}

int inet_server_result(inet_server *s, int64_t ticket, inet_result *res, int32_t *buf, int64_t cap,
                       int64_t *len) {
  inet_server::Slot *S = s ? slot_of(s, ticket) : nullptr;
  if (!S || S->state != 2) return INET_EINVAL;
  const NetState &st = S->st;
  if (res) {
    res->status = st.status;
    res->n_stuck = st.n_stuck;
    res->interactions = st.interactions;
    res->steps = st.steps;
    res->agents_used = st.agent_top;
    res->names_used = st.name_top;
    res->max_frontier = st.max_frontier;
    res->loops = st.loops;
  }
  if (!len) return st.status < 0 ? st.status : INET_OK;
  if (st.status < 0) return st.status;
  std::vector<int32_t> stream;
  int rc = readback_net(s->rules, S->desc, st, S->iface, &stream);
  if (rc) return rc;
  *len = (int64_t)stream.size();
  if (!buf || cap < *len) return INET_ERANGE;
  std::memcpy(buf, stream.data(), stream.size() * 4);
  return INET_OK;
}

int inet_server_per_rule(inet_server *s, int64_t ticket, uint64_t *counts, int32_t cap) {
  inet_server::Slot *S = s ? slot_of(s, ticket) : nullptr;
  if (!S || S->state != 2 || !counts || cap < s->rules.nr) return INET_EINVAL;
  if (s->rules.nr == 0) return INET_OK;
  HIPCHK(hipMemcpy(counts, S->desc.per_rule, 8 * (size_t)s->rules.nr, hipMemcpyDeviceToHost));
  return INET_OK;
}

int inet_server_release(inet_server *s, int64_t ticket) {
  if (!s) return INET_EINVAL;
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return INET_EINVAL;
  const int32_t si = it->second;
  inet_server::Slot &S = s->slots[si];
  if (S.state != 2) return INET_EINVAL;
  give_range(s, S.off, S.len);
  S = inet_server::Slot();
  s->free_slots.push_back(si);
  s->by_ticket.erase(it);
  return INET_OK;
}

int inet_server_stats(const inet_server *s, int64_t *free_bytes, int32_t *free_slots,
                      int32_t *running) {
  if (!s) return INET_EINVAL;
  if (free_bytes) *free_bytes = (int64_t)s->free_bytes;
  if (free_slots) *free_slots = (int32_t)s->free_slots.size();
  if (running) *running = (int32_t)s->running.size();
  return INET_OK;
}

int inet_server_net_bytes(const inet_server *s, int32_t n_agents, int32_t n_eqs, int32_t n_names,
                          int64_t agent_cap, int64_t name_cap, int64_t *bytes) {
  if (!s || !bytes) return INET_EINVAL;
  NetPlan P;
  if (!plan_net(n_agents, n_eqs, n_names, agent_cap, name_cap, &P)) return INET_EINVAL;
  *bytes = (int64_t)(P.bytes + al(4 * (size_t)n_agents + 4) + al(8 * (size_t)n_agents + 8) +
                     al(8 * (size_t)n_eqs + 8));
  return INET_OK;
}

int inet_server_run(inet_server *s, int32_t n_pool, const int32_t *label, const int32_t *port,
                    const int64_t *agent_off, const int32_t *eq_lhs, const int32_t *eq_rhs,
                    const int64_t *eq_off, const int32_t *n_names, const int64_t *agent_cap,
                    const int64_t *name_cap, int64_t n_req, const double *arrival_s,
                    const int32_t *pick, uint32_t round_steps, double time_limit_s,
                    hipStream_t stream, double *done_s, int32_t *status, uint64_t *interactions,
                    uint32_t *steps, inet_serve_stats *stats, const inet_serve_capture *capture) {
  if (!s || n_pool <= 0 || n_req < 0 || !agent_off || !eq_off || !n_names || round_steps == 0)
    return INET_EINVAL;
  if (n_req > 0 && (!arrival_s || !pick || !done_s || !status || !interactions || !steps))
    return INET_EINVAL;
  const bool want_rules = capture && capture->per_rule;
  const bool want_nf = capture && capture->want_nf;
  if (want_nf && (!capture->nf_pos || !capture->nf_len || capture->nf_cap < 0 ||
                  (capture->nf_cap > 0 && !capture->nf_buf)))
    return INET_EINVAL;
  if (!s->running.empty() || !s->finished.empty() || s->round_in_flight) return INET_EINVAL;
  const CompiledRules &R = s->rules;
  const int64_t A = agent_off[n_pool], E = eq_off[n_pool];
  if (agent_off[0] != 0 || eq_off[0] != 0 || (A && (!label || !port)) || (E && (!eq_lhs || !eq_rhs)))
    return INET_EINVAL;
  for (int64_t i = 0; i < n_req; i++) {
    if (pick[i] < 0 || pick[i] >= n_pool) return INET_EINVAL;
    if (i && arrival_s[i] < arrival_s[i - 1]) return INET_EINVAL;
  }
  // validate the pool once (the interfaces are kept when normal forms are read back)
  std::vector<std::vector<int32_t>> pool_iface(want_nf ? n_pool : 0);
  for (int32_t j = 0; j < n_pool; j++) {
    const int64_t a0 = agent_off[j], na = agent_off[j + 1] - a0;
    const int64_t e0 = eq_off[j], ne = eq_off[j + 1] - e0;
    if (na < 0 || ne < 0 || na > INT32_MAX || ne > INT32_MAX) return INET_EINVAL;
    std::vector<int32_t> iface;
    int rc = validate_net(R, label + a0, port + 2 * a0, na, eq_lhs + e0, eq_rhs + e0, ne,
                          n_names[j], &iface);
    if (rc) return rc;
    if (want_nf) pool_iface[j].swap(iface);
  }
  if (want_rules && R.nr > 0)
    std::memset(capture->per_rule, 0, sizeof(uint64_t) * (size_t)n_req * (size_t)R.nr);
  if (want_nf)
    for (int64_t i = 0; i < n_req; i++) {
      capture->nf_pos[i] = -1;
      capture->nf_len[i] = 0;
    }
  int64_t nf_used = 0;
  bool nf_short = false;
  // the pool's initial images and the admission records stay resident for the run
  const int32_t M = s->max_slots;
  const size_t img_bytes = al(4 * (size_t)A + 4) + al(8 * (size_t)A + 8) + al(8 * (size_t)E + 8) +
                           al(sizeof(AdmitRec) * (size_t)M * 2);
  size_t img_off = 0;
  if (!take_range(s, img_bytes, &img_off)) return INET_ENOMEM;
  char *p = s->dev + img_off;
  auto take = [&](size_t bytes) { char *q = p; p += al(bytes); return q; };
  int32_t *d_label = (int32_t *)take(4 * (size_t)A + 4);
  int32_t *d_port = (int32_t *)take(8 * (size_t)A + 8);
  int32_t *d_eq = (int32_t *)take(8 * (size_t)E + 8);
  AdmitRec *d_admit = (AdmitRec *)take(sizeof(AdmitRec) * (size_t)M * 2);
  AdmitRec *h_admit = nullptr;
  int32_t *h_order = nullptr;
  NetState *h_states = nullptr;
  unsigned long long *h_rules = nullptr;  // per-rule counts of every slot (capture only)
  int rc = INET_OK;
  {
    std::vector<int32_t> eqs((size_t)2 * E + 2);
    for (int64_t e = 0; e < E; e++) {
      eqs[2 * e] = eq_lhs[e];
      eqs[2 * e + 1] = eq_rhs[e];
    }
    hipError_t e = hipSuccess;
    if (A) e = hipMemcpy(d_label, label, 4 * (size_t)A, hipMemcpyHostToDevice);
    if (e == hipSuccess && A) e = hipMemcpy(d_port, port, 8 * (size_t)A, hipMemcpyHostToDevice);
    if (e == hipSuccess && E) e = hipMemcpy(d_eq, eqs.data(), 8 * (size_t)E, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h_admit, sizeof(AdmitRec) * (size_t)M * 2);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h_order, 4 * (size_t)M);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h_states, sizeof(NetState) * (size_t)M);
    if (e == hipSuccess && want_rules && R.nr > 0)
      e = hipHostMalloc((void **)&h_rules, 8 * (size_t)R.nr * (size_t)M);
    if (e != hipSuccess) rc = INET_EHIP;
  }
  std::vector<int64_t> req_of(M, -1);
  std::vector<int32_t> boost_of(M, 1);
  std::deque<std::pair<int64_t, int32_t>> retry;  // (request, capacity multiplier)
  int64_t next = 0, rounds = 0, retries = 0;
  int32_t max_res = 0, n_admit = 0, buf = 0;
  using clk = std::chrono::steady_clock;
  const clk::time_point t0 = clk::now();
  auto now = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
  // admit one request into a free slot and byte range: 1 admitted, 0 no room
  // now, -1 its capacities cannot be planned (too large)
  auto admit = [&](int64_t req, int32_t boost) -> int {
    const int32_t j = pick[req];
    const int64_t a0 = agent_off[j], na = agent_off[j + 1] - a0;
    const int64_t e0 = eq_off[j], ne = eq_off[j + 1] - e0;
    NetPlan P;
    if (!plan_net(na, ne, n_names[j], agent_cap ? agent_cap[j] : 0, name_cap ? name_cap[j] : 0, &P))
      return -1;
    if (boost > 1 &&
        !plan_net(na, ne, n_names[j], P.agent_cap * boost, P.name_cap * boost, &P))
      return -1;
    if (s->free_slots.empty()) return 0;
    size_t off = 0;
    if (!take_range(s, P.bytes, &off)) return 0;
    const int32_t si = s->free_slots.back();
    s->free_slots.pop_back();
    inet_server::Slot &S = s->slots[si];
    S = inet_server::Slot();
    S.state = 1;
    S.off = off;
    S.len = P.bytes;
    char *q = s->dev + off;
    auto tk = [&](size_t bytes) { char *r = q; q += al(bytes); return r; };
    NetDesc &D = S.desc;
    D.agent = (int32_t *)tk(16 * (size_t)P.agent_cap);
    D.bind = (int32_t *)tk(4 * (size_t)P.name_cap);
    D.queue0 = (unsigned long long *)tk(8 * (size_t)P.qcap);
    D.queue1 = (unsigned long long *)tk(8 * (size_t)P.qcap);
    D.stuck = (unsigned long long *)tk(8 * (size_t)P.scap);
    D.init_label = d_label + a0;
    D.init_port = d_port + 2 * a0;
    D.init_eq = d_eq + 2 * e0;
    D.per_rule = s->d_per_rule + (size_t)si * R.nr;
    D.st = s->d_states + si;
    D.agent_cap = (int32_t)P.agent_cap;
    D.name_cap = (int32_t)P.name_cap;
    D.qcap = (int32_t)P.qcap;
    D.scap = (int32_t)P.scap;
    D.n_agents0 = (int32_t)na;
    D.n_eqs0 = (int32_t)ne;
    D.n_names0 = n_names[j];
    D.order = si;
    AdmitRec &rec = h_admit[(size_t)buf * M + n_admit++];
    rec.desc = D;
    rec.slot = si;
    rec.pad = 0;
    req_of[si] = req;
    boost_of[si] = boost;
    s->running.push_back(si);
    return 1;
  };
  auto give_up = [&](int64_t req) {
    done_s[req] = now();
    status[req] = INET_ENOMEM;
    interactions[req] = 0;
    steps[req] = 0;
  };
  // admit requests that have arrived, retries first, in arrival order
  auto admit_arrived = [&](double t) {
    while (true) {
      if (!retry.empty()) {
        const int a = admit(retry.front().first, retry.front().second);
        if (a == 0) return;
        if (a < 0) give_up(retry.front().first);
        retry.pop_front();
      } else if (next < n_req && arrival_s[next] <= t) {
        const int a = admit(next, 1);
        if (a == 0) return;
        if (a < 0) give_up(next);
        next++;
      } else {
        return;
      }
    }
  };
  auto release = [&](int32_t si) {
    inet_server::Slot &S = s->slots[si];
    give_range(s, S.off, S.len);
    S = inet_server::Slot();
    s->free_slots.push_back(si);
    req_of[si] = -1;
  };
  const int nr = R.nr;
  while (rc == INET_OK && (next < n_req || !retry.empty() || !s->running.empty())) {
    const double t = now();
    if (t > time_limit_s) { rc = INET_ELIMIT; break; }
    admit_arrived(t);
    if (s->running.empty()) {
      if (!retry.empty() || (next < n_req && arrival_s[next] <= t)) { rc = INET_ENOMEM; break; }
      const double wait = next < n_req ? arrival_s[next] - t : 0.0;
      if (wait > 5e-4) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 2e-4));
      continue;
    }
    // install this round's admissions with one copy and one launch
    if (n_admit) {
      AdmitRec *src = h_admit + (size_t)buf * M, *dst = d_admit + (size_t)buf * M;
      if (hipMemcpyAsync(dst, src, sizeof(AdmitRec) * (size_t)n_admit, hipMemcpyHostToDevice,
                         stream) != hipSuccess) { rc = INET_EHIP; break; }
      rc = launch_admit(dst, n_admit, s->d_descs, nr, stream);
      if (rc) break;
      n_admit = 0;
      buf ^= 1;
    }
    const int n = (int)s->running.size();
    std::copy(s->running.begin(), s->running.end(), h_order);
    s->order_host = s->running;
    if (hipMemcpyAsync(s->d_order, h_order, 4 * (size_t)n, hipMemcpyHostToDevice, stream) !=
        hipSuccess) { rc = INET_EHIP; break; }
    const inet_config &cfg = s->cfg;
    const LaunchShape sh = effective_shape(cfg, n > 1 ? n : 2, R);
    int grid = 1;
    rc = resident_grid(sh, R, cfg, n, &grid);
    if (!rc) rc = launch_zero(s->d_counter, 1, stream);
    KParams kp;
    if (!rc) rc = kparams_for(cfg, nullptr, &kp);
    if (!rc) rc = launch_reduce(R, sh, grid, s->d_descs, s->d_order, n, s->d_counter, s->d_rules,
                                round_budget(cfg, round_steps, n, grid),
                                s->cfg.jump ? FLAG_JUMP : 0, kp, stream);
    if (rc) break;
    if (hipMemcpyAsync(h_states, s->d_states, sizeof(NetState) * (size_t)M, hipMemcpyDeviceToHost,
                       stream) != hipSuccess) { rc = INET_EHIP; break; }
    if (h_rules && hipMemcpyAsync(h_rules, s->d_per_rule, 8 * (size_t)nr * (size_t)M,
                                  hipMemcpyDeviceToHost, stream) != hipSuccess) {
      rc = INET_EHIP;
      break;
    }
    rounds++;
    max_res = std::max(max_res, n);
    // requests arriving during the round are admitted for the next one
    admit_arrived(now());
    if (hipStreamSynchronize(stream) != hipSuccess) { rc = INET_EHIP; break; }
    const double done = now();
    std::vector<char> in_round(M, 0);
    for (int32_t si : s->order_host) in_round[si] = 1;
    std::vector<int32_t> still;
    still.reserve(s->running.size());
    for (int32_t si : s->running) {
      const NetState &st = h_states[si];
      if (!in_round[si] || !(st.phase == PHASE_DONE || st.status == ST_ENOMEM ||
                             st.status == ST_EINTERNAL)) {
        still.push_back(si);
        continue;
      }
      const int64_t req = req_of[si];
      const int32_t boost = boost_of[si];
      if (st.status == ST_ENOMEM && boost < 4096) {
        release(si);
        retry.emplace_back(req, boost * 8);
        retries++;
        continue;
      }
      done_s[req] = done;
      status[req] = st.status;
      interactions[req] = st.interactions;
      steps[req] = st.steps;
      if (h_rules)
        std::memcpy(capture->per_rule + (size_t)req * nr, h_rules + (size_t)si * nr, 8 * (size_t)nr);
      if (want_nf && capture->want_nf[req] && st.status >= 0) {
        // the heap is still the slot's: nothing is installed there before the next round
        std::vector<int32_t> nf;
        const int brc = readback_net(R, s->slots[si].desc, st, pool_iface[pick[req]], &nf);
        if (brc) { rc = brc; break; }
        capture->nf_len[req] = (int64_t)nf.size();
        if (nf_used + (int64_t)nf.size() <= capture->nf_cap) {
          if (!nf.empty()) std::memcpy(capture->nf_buf + nf_used, nf.data(), 4 * nf.size());
          capture->nf_pos[req] = nf_used;
          nf_used += (int64_t)nf.size();
        } else {
          nf_short = true;
        }
      }
      release(si);
    }
    if (rc != INET_OK) break;
    s->running.swap(still);
  }
  if (rc != INET_OK) {
    (void)hipStreamSynchronize(stream);
    for (int32_t si : std::vector<int32_t>(s->running)) release(si);
    s->running.clear();
  }
  s->order_host.clear();
  if (h_admit) (void)hipHostFree(h_admit);
  if (h_order) (void)hipHostFree(h_order);
  if (h_states) (void)hipHostFree(h_states);
  if (h_rules) (void)hipHostFree(h_rules);
  give_range(s, img_off, img_bytes);
  if (stats) {
    stats->rounds = rounds;
    stats->max_resident = max_res;
    stats->retries = (int32_t)retries;
    stats->wall_s = now();
  }
  if (rc == INET_OK && nf_short) rc = INET_ERANGE;
  return rc;
}

void inet_server_free(inet_server *s) {
  if (!s) return;
  if (s->upload_done) (void)hipEventDestroy(s->upload_done);
  delete s;
}

}  // extern "C"
