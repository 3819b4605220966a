// pipeline.hip -- the paper's own evaluation loop (Sections 3.3-3.6), kept as
// an ablation beside the net engines.
//
// The configuration is a flat list of equations.  Each iteration
//   int  -- every equation gets a fixed number n of output slots (n = the
//           largest number of equations a rule leaves); an active pair with a
//           rule fills its slots with the equations of the rule's right-hand
//           side and dummies, any other equation keeps slot 0 and dummies;
//   filter -- the dummies are removed (stream compaction);
//   com  -- the equations with a name side are oriented name first and
//           sorted by that name; neighbours that share it, x = t and x = s,
//           are merged into s = t (a reduce by key); an equation between two
//           names is keyed by one of them only, so a chain of names needs one
//           iteration per link (the remark after the correctness proposition
//           of Section 3.6);
// and the loop repeats while an int or a com happened.  Names inside agents
// are never touched: sub and col are left to the read-back (Theorem 1 of
// Section 2.2).  Allocation of the new agents and names is a prefix sum over
// the active pairs' needs.  The steps the paper runs with Thrust (remove,
// sort, reduce_by_key) are the device primitives of primitives.h (prefix sum,
// compaction, radix sort, reduce by key); the interaction and the bookkeeping
// are kernels of this file.  When the loop ends, each
// remaining equation x = t is written into x's name cell and each remaining
// pair of agents (no rule) into the residual list, which is the state the
// read-back of the net engines expects.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"
#include "primitives.h"
#include "runtime.h"

namespace inet {
namespace {

typedef unsigned long long u64;
constexpr u64 DUMMY = ~0ull;  // an output slot that holds no equation

__device__ __forceinline__ u64 pk2(int x, int y) {
  return (u64)(unsigned)x | ((u64)(unsigned)y << 32);
}
__device__ __forceinline__ int lo(u64 w) { return (int)(unsigned)w; }
__device__ __forceinline__ int hi(u64 w) { return (int)(unsigned)(w >> 32); }

// counters of one iteration, on the device
enum { C_INT = 0, C_LOOPS = 1, C_NOMEM = 2, C_STUCK = 3, C_SELECTED = 4, C_UNIQUE = 6, C_WORDS = 8 };

// the rule code of an equation between two agents, -1 if none (agent records
// are {label, port 0, port 1, unused})
__device__ __forceinline__ int rule_code(int u, int v, const int *agent, const int *rule_of,
                                         int ns) {
  if (u < 0 || v < 0) return -1;
  return rule_of[agent[4 * (size_t)u] * ns + agent[4 * (size_t)v]];
}

// what an equation allocates if it is reduced: agents in the high half,
// names in the low half
__global__ void k_pp_need(const u64 *__restrict__ eq, int m, const int *__restrict__ agent,
                          const int *__restrict__ rules, int ns, int nr, u64 *__restrict__ need) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const u64 e = eq[i];
  const int code = rule_code(lo(e), hi(e), agent, rules, ns);
  u64 w = 0;
  if (code >= 0) {
    const int *T = rules + ns * ns + (code >> 1) * RT_WORDS;
    w = ((u64)(unsigned)T[RT_NALLOC] << 32) | (u64)(unsigned)T[RT_NFRESH];
  }
  need[i] = w;
}

__device__ __forceinline__ int operand(int op, int a, int b, int pa0, int pa1, int pb0, int pb1,
                                       int my_a, int my_n) {
  const int kind = op >> 4, idx = op & 15;
  if (kind == OP_AUX) return idx == 0 ? pa0 : (idx == 1 ? pa1 : (idx == 2 ? pb0 : pb1));
  if (kind == OP_NEW) return idx == 0 ? a : (idx == 1 ? b : my_a + idx - 2);
  return -1 - (my_n + idx);
}

// int with n output slots per equation; the allocation offset of equation i
// is the inclusive prefix sum of the needs minus its own need
__global__ void k_pp_int(const u64 *__restrict__ eq, int m, const u64 *__restrict__ need,
                         const u64 *__restrict__ incl, const int *__restrict__ rules, int ns,
                         int n_slots, NetDesc D, int agent_top, int name_top,
                         u64 *__restrict__ out, int *ctr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  u64 *o = out + (size_t)i * n_slots;
  for (int j = 0; j < n_slots; j++) o[j] = DUMMY;
  const u64 e = eq[i];
  int a = lo(e), b = hi(e);
  const int code = rule_code(a, b, D.agent, rules, ns);
  if (code < 0) {  // not an active pair with a rule: the equation stays
    o[0] = e;
    return;
  }
  if (code & 1) { const int t = a; a = b; b = t; }
  const int *T = rules + ns * ns + (code >> 1) * RT_WORDS;
  int *ag = D.agent;
  const int pa0 = ag[4 * (size_t)a + 1], pa1 = ag[4 * (size_t)a + 2];
  const int pb0 = ag[4 * (size_t)b + 1], pb1 = ag[4 * (size_t)b + 2];
  const u64 off = incl[i] - need[i];
  const int my_a = agent_top + hi(off), my_n = name_top + lo(off);
  const int nnew = T[RT_NNEW], nalloc = T[RT_NALLOC], nfresh = T[RT_NFRESH], neq = T[RT_NEQ];
  if (my_a + nalloc > D.agent_cap || my_n + nfresh > D.name_cap) {
    atomicExch(&ctr[C_NOMEM], 1);
    return;
  }
  for (int k = 0; k < nnew; k++) {
    const int slot = k == 0 ? a : (k == 1 ? b : my_a + k - 2);
    ag[4 * (size_t)slot] = T[RT_LABEL + k];
    ag[4 * (size_t)slot + 1] = operand(T[RT_PORT + 2 * k], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
    ag[4 * (size_t)slot + 2] = operand(T[RT_PORT + 2 * k + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
  }
  for (int f = 0; f < nfresh; f++) D.bind[my_n + f] = EMPTY;
  int k = 0;
  for (int j = 0; j < neq; j++) {
    const int u = operand(T[RT_EQ + 2 * j], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
    const int v = operand(T[RT_EQ + 2 * j + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
    if (u == v) atomicAdd(&ctr[C_LOOPS], 1);  // x = x: a closed loop
    else o[k++] = pk2(u, v);
  }
  atomicAdd(&D.per_rule[code >> 1], 1ull);
  atomicAdd(&ctr[C_INT], 1);
}

// orient name first; the key is the name, or a key no other equation has
__global__ void k_pp_key(u64 *__restrict__ eq, int m, unsigned *__restrict__ key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int u = lo(eq[i]), v = hi(eq[i]);
  if (u >= 0 && v < 0) { const int t = u; u = v; v = t; }
  eq[i] = pk2(u, v);
  key[i] = u < 0 ? (unsigned)~u : 0x80000000u + (unsigned)i;
}

// the end state: x = t into x's cell, pairs of agents into the residuals
__global__ void k_pp_finish(const u64 *__restrict__ eq, int m, NetDesc D, int *ctr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int u = lo(eq[i]), v = hi(eq[i]);
  if (u >= 0 && v < 0) { const int t = u; u = v; v = t; }
  if (u < 0) {
    if (u == v) atomicAdd(&ctr[C_LOOPS], 1);
    else D.bind[~u] = v;
    return;
  }
  const int s = atomicAdd(&ctr[C_STUCK], 1);
  if (s < D.scap) ((u64 *)D.stuck)[s] = pk2(u, v);
  else atomicExch(&ctr[C_NOMEM], 1);
}

// com of two equations sharing their key x: (x, t) and (x, s) give (s, t)
struct Merge {
  __device__ u64 operator()(const u64 &p, const u64 &q) const { return pk2(hi(q), hi(p)); }
};
struct Sum {
  __device__ u64 operator()(const u64 &p, const u64 &q) const { return p + q; }
};

// the loop's device arrays, each of `cap` elements (temporary memory: the
// ablation allocates with hipMalloc, unlike the net engines)
struct Buffers {
  u64 *eq = nullptr, *out = nullptr, *tmp = nullptr, *need = nullptr, *incl = nullptr;
  unsigned *key = nullptr, *key2 = nullptr;
  prim::Scratch arena;  // the primitives' temporary memory
  size_t cap = 0;
  void release() {
    for (void *p : {(void *)eq, (void *)out, (void *)tmp, (void *)need, (void *)incl, (void *)key,
                    (void *)key2, (void *)arena.base})
      if (p) (void)hipFree(p);
    *this = Buffers();
  }
};

// grow the arrays to `items` elements, keeping the equations in eq
int ensure(Buffers &B, size_t items, hipStream_t s) {
  if (items <= B.cap) return INET_OK;
  (void)hipStreamSynchronize(s);
  const size_t cap = std::max(items, B.cap * 2);
  Buffers N;
  N.cap = cap;
  bool ok = hipMalloc(&N.eq, 8 * cap) == hipSuccess && hipMalloc(&N.out, 8 * cap) == hipSuccess &&
            hipMalloc(&N.tmp, 8 * cap) == hipSuccess && hipMalloc(&N.need, 8 * cap) == hipSuccess &&
            hipMalloc(&N.incl, 8 * cap) == hipSuccess && hipMalloc(&N.key, 4 * cap) == hipSuccess &&
            hipMalloc(&N.key2, 4 * cap) == hipSuccess;
  if (!ok) { N.release(); return INET_ENOMEM; }
  // temporary storage of the primitives, sized for the largest input
  N.arena.size = prim::scratch_bytes(cap);
  if (hipMalloc((void **)&N.arena.base, N.arena.size) != hipSuccess) { N.release(); return INET_ENOMEM; }
  if (B.eq && hipMemcpyAsync(N.eq, B.eq, 8 * B.cap, hipMemcpyDeviceToDevice, s) != hipSuccess) {
    N.release();
    return INET_EHIP;
  }
  (void)hipStreamSynchronize(s);
  B.release();
  B = N;
  return INET_OK;
}

int grid_of(int m) { return (m + 255) / 256; }

// the paper's loop on one net; its state is left as after a reduction
int pipeline_net(inet_net *h, int i, hipStream_t s, uint64_t max_iter, Buffers &B, int *d_ctr,
                 int64_t *d_count) {
  const CompiledRules &R = h->rules;
  const NetDesc &D = h->descs[i];
  const int ns = R.ns, n_slots = std::max(1, R.max_links);
  int m = D.n_eqs0;
  int rc = ensure(B, (size_t)std::max(m, 1) * n_slots, s);
  if (rc) return rc;
  if (m && hipMemcpyAsync(B.eq, D.queue0, 8 * (size_t)m, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return INET_EHIP;
  int agent_top = D.n_agents0, name_top = D.n_names0;
  uint64_t iters = 0, ints = 0;
  int loops = 0, max_m = m, status = INET_OK;
  for (;;) {
    if (iters >= max_iter) { status = INET_ELIMIT; break; }
    // room for every slot of this iteration's int (the filtered list is no longer)
    rc = ensure(B, (size_t)std::max(m, 1) * n_slots, s);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(d_ctr, 0, 4 * C_WORDS, s));
    int n_int = 0;
    if (m) {
      // int: allocation by prefix sum, then n slots per equation
      hipLaunchKernelGGL(k_pp_need, dim3(grid_of(m)), dim3(256), 0, s, B.eq, m, D.agent,
                         h->d_rules, ns, R.nr, B.need);
      B.arena.reset();
      if (prim::inclusive_sum<u64>(B.need, B.incl, (size_t)m, B.arena, s)) return INET_EHIP;
      hipLaunchKernelGGL(k_pp_int, dim3(grid_of(m)), dim3(256), 0, s, B.eq, m, B.need, B.incl,
                         h->d_rules, ns, n_slots, D, agent_top, name_top, B.out, d_ctr);
      u64 total = 0;  // what this iteration allocated: agents high, names low
      HIPCHK(hipMemcpyAsync(&total, B.incl + (m - 1), 8, hipMemcpyDeviceToHost, s));
      // filter: drop the dummies
      B.arena.reset();
      if (prim::select_not(B.out, B.tmp, (size_t)m * n_slots, DUMMY, d_count, B.arena, s))
        return INET_EHIP;
      int64_t sel = 0;
      int ctr[C_WORDS];
      HIPCHK(hipMemcpyAsync(&sel, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(ctr, d_ctr, 4 * C_WORDS, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (ctr[C_NOMEM]) { status = INET_ENOMEM; break; }
      n_int = ctr[C_INT];
      loops += ctr[C_LOOPS];
      agent_top += (int)(total >> 32);
      name_top += (int)(unsigned)total;
      m = (int)sel;
      if (m && hipMemcpyAsync(B.eq, B.tmp, 8 * (size_t)m, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return INET_EHIP;
    }
    // com: sort the equations by their key, merge neighbours with equal keys
    size_t n_com = 0;
    if (m > 1) {
      hipLaunchKernelGGL(k_pp_key, dim3(grid_of(m)), dim3(256), 0, s, B.eq, m, B.key);
      B.arena.reset();
      if (prim::radix_sort_pairs<u64>(B.key, B.eq, B.key2, B.tmp, (size_t)m, B.arena, s))
        return INET_EHIP;
      B.arena.reset();
      if (prim::reduce_by_key<u64>(B.key, B.eq, (size_t)m, B.key2, B.tmp, d_count, Merge(),
                                   B.arena, s))
        return INET_EHIP;
      std::swap(B.eq, B.tmp);  // the merged equations
      int64_t uniq = 0;
      HIPCHK(hipMemcpyAsync(&uniq, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      n_com = (size_t)m - uniq;
      m = (int)uniq;
    }
    iters++;
    ints += (uint64_t)n_int;
    max_m = std::max(max_m, m);
    if (n_int == 0 && n_com == 0) break;
  }
  // the end state
  NetState st{};
  if (status == INET_OK) {
    HIPCHK(hipMemsetAsync(d_ctr, 0, 4 * C_WORDS, s));
    if (m) hipLaunchKernelGGL(k_pp_finish, dim3(grid_of(m)), dim3(256), 0, s, B.eq, m, D, d_ctr);
    int ctr[C_WORDS];
    HIPCHK(hipMemcpyAsync(ctr, d_ctr, 4 * C_WORDS, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    loops += ctr[C_LOOPS];
    st.n_stuck = ctr[C_STUCK];
    if (ctr[C_NOMEM]) status = INET_ENOMEM;
  }
  st.interactions = ints;
  st.steps = (uint32_t)std::min<uint64_t>(iters, 0xffffffffu);
  st.agent_top = agent_top;
  st.name_top = name_top;
  st.loops = loops;
  st.max_frontier = max_m;
  if (status == INET_OK) {
    st.phase = PHASE_DONE;
    st.status = st.n_stuck ? ST_STUCK : ST_OK;
  } else {
    st.phase = PHASE_RUN;
    st.status = status == INET_ENOMEM ? ST_ENOMEM : ST_ELIMIT;
  }
  HIPCHK(hipMemcpyAsync(D.st, &st, sizeof(NetState), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return INET_OK;
}

}  // namespace
}  // namespace inet

extern "C" int inet_reduce_pipeline(inet_net *h, hipStream_t stream, uint64_t max_iterations) {
  using namespace inet;
  if (!h) return INET_EINVAL;
  if (max_iterations == 0) max_iterations = ~0ull;
  Buffers B;
  int *d_ctr = nullptr;
  int64_t *d_count = nullptr;
  if (hipMalloc(&d_ctr, 4 * C_WORDS) != hipSuccess) return INET_ENOMEM;
  if (hipMalloc(&d_count, 64) != hipSuccess) { (void)hipFree(d_ctr); return INET_ENOMEM; }
  int rc = INET_OK;
  for (int i = 0; i < h->n_nets && rc == INET_OK; i++)
    rc = pipeline_net(h, i, stream, max_iterations, B, d_ctr, d_count);
  (void)hipStreamSynchronize(stream);
  B.release();
  (void)hipFree(d_ctr);
  (void)hipFree(d_count);
  h->results_valid = false;
  return rc;
}

// ---------------------------------------------------------------------------
// the primitives on caller arrays (tests)

namespace {
struct ArenaFor {
  inet::prim::Scratch S;
  explicit ArenaFor(size_t n) {
    S.size = inet::prim::scratch_bytes(n);
    if (hipMalloc((void **)&S.base, S.size) != hipSuccess) S.base = nullptr;
  }
  ~ArenaFor() {
    if (S.base) (void)hipFree(S.base);
  }
};

int count_back(int64_t *d_n, int64_t *n_out, hipStream_t s) {
  if (hipMemcpyAsync(n_out, d_n, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return INET_EHIP;
  return INET_OK;
}
}  // namespace

extern "C" int inet_prim_scan(const uint64_t *d_in, uint64_t *d_out, int64_t n, hipStream_t s) {
  if (n < 0 || (n && (!d_in || !d_out))) return INET_EINVAL;
  ArenaFor A((size_t)n);
  if (!A.S.base) return INET_ENOMEM;
  if (inet::prim::inclusive_sum<unsigned long long>((const unsigned long long *)d_in,
                                                    (unsigned long long *)d_out, (size_t)n, A.S, s))
    return INET_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? INET_OK : INET_EHIP;
}

extern "C" int inet_prim_select(const uint64_t *d_in, uint64_t *d_out, int64_t n, uint64_t drop,
                                int64_t *n_out, hipStream_t s) {
  if (n < 0 || !n_out || (n && (!d_in || !d_out))) return INET_EINVAL;
  ArenaFor A((size_t)n);
  int64_t *d_n = nullptr;
  if (!A.S.base || A.S.take(sizeof(int64_t), (void **)&d_n)) return INET_ENOMEM;
  if (inet::prim::select_not((const unsigned long long *)d_in, (unsigned long long *)d_out,
                             (size_t)n, (unsigned long long)drop, d_n, A.S, s))
    return INET_EHIP;
  return count_back(d_n, n_out, s);
}

extern "C" int inet_prim_sort_pairs(uint32_t *d_keys, uint64_t *d_vals, int64_t n, hipStream_t s) {
  if (n < 0 || (n && (!d_keys || !d_vals))) return INET_EINVAL;
  if (n <= 1) return INET_OK;
  ArenaFor A((size_t)n);
  uint32_t *k2 = nullptr;
  unsigned long long *v2 = nullptr;
  if (hipMalloc((void **)&k2, 4 * (size_t)n) != hipSuccess) return INET_ENOMEM;
  if (hipMalloc((void **)&v2, 8 * (size_t)n) != hipSuccess) {
    (void)hipFree(k2);
    return INET_ENOMEM;
  }
  int rc = A.S.base ? INET_OK : INET_ENOMEM;
  if (!rc && inet::prim::radix_sort_pairs<unsigned long long>(
                 d_keys, (unsigned long long *)d_vals, k2, v2, (size_t)n, A.S, s))
    rc = INET_EHIP;
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = INET_EHIP;
  (void)hipFree(k2);
  (void)hipFree(v2);
  return rc;
}

extern "C" int inet_prim_reduce_by_key(const uint32_t *d_keys, const uint64_t *d_vals, int64_t n,
                                       uint32_t *d_keys_out, uint64_t *d_vals_out, int32_t op,
                                       int64_t *n_out, hipStream_t s) {
  if (n < 0 || !n_out || (op != 0 && op != 1) ||
      (n && (!d_keys || !d_vals || !d_keys_out || !d_vals_out)))
    return INET_EINVAL;
  ArenaFor A((size_t)n);
  int64_t *d_n = nullptr;
  if (!A.S.base || A.S.take(sizeof(int64_t), (void **)&d_n)) return INET_ENOMEM;
  int e = op == 0 ? inet::prim::reduce_by_key<unsigned long long>(
                        d_keys, (const unsigned long long *)d_vals, (size_t)n, d_keys_out,
                        (unsigned long long *)d_vals_out, d_n, inet::Sum(), A.S, s)
                  : inet::prim::reduce_by_key<unsigned long long>(
                        d_keys, (const unsigned long long *)d_vals, (size_t)n, d_keys_out,
                        (unsigned long long *)d_vals_out, d_n, inet::Merge(), A.S, s);
  if (e) return INET_EHIP;
  return count_back(d_n, n_out, s);
}
