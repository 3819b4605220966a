// kernels.hip -- gfx950 kernels of the interaction-net evaluator.
//
// One workgroup owns one net at a time ("net engine").  The frontier of
// active pairs lives in LDS (spilling to the net's global queue when it
// outgrows the LDS capacity), and every memory operation on the net's heap is
// performed at workgroup scope: a net never leaves the compute unit that is
// reducing it, so no cross-XCD coherence traffic is ever needed.  A step is
// the loop body of evaluate() (Section 3.6):
//   int  -- every lane takes one active pair, looks its rule up in the LDS
//           rule table, allocates the right-hand side's agents and names with
//           a wave-wide prefix sum and one LDS atomic per wave (the scan-based
//           output allocation proposed in Section 4.2), writes the new agents
//           into the int32 SoA heap, reusing the two slots of the pair;
//   com  -- each equation left by the rule is linked: a name side exchanges
//           the other side into the name's cell; the lane that finds the cell
//           already filled owns the second occurrence, forms the equation
//           (parked value = other side) and carries on along the chain; an
//           equation between two agents is a new active pair;
//   compaction -- new active pairs are appended to the next frontier with a
//           wave ballot, a mask prefix count and one LDS atomic per wave.
// A single workgroup barrier separates consecutive steps.  After the loop,
// name-to-name chains left in the cells (the partial com of the remark after
// the correctness proposition of Section 3.6) are compressed by pointer
// jumping.
#include <hip/hip_runtime.h>

#include "inet_internal.h"
#include "runtime.h"

namespace inet {

__device__ __forceinline__ int count_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p ? 1 : 0); }

__device__ __forceinline__ int first_lane_value(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// exclusive prefix sum over the wave of v in [0, 15]; every lane active
__device__ __forceinline__ int wave_scan16(int v, int *total) {
  int pre = 0, tot = 0;
#pragma unroll
  for (int bit = 0; bit < 4; bit++) {
    const unsigned long long m = ballot((v >> bit) & 1);
    pre += count_below(m) << bit;
    tot += __popcll(m) << bit;
  }
  *total = tot;
  return pre;
}

// append (u, v) for every lane with prod set; one LDS atomic per wave
__device__ __forceinline__ void wave_push(bool prod, int u, int v, int2 *lds_q, int lds_cap,
                                          int2 *g_q, int qcap, int *cnt, int *status) {
  const unsigned long long m = ballot(prod);
  if (m == 0ull) return;
  int base = 0;
  if (__lane_id() == 0) base = atomicAdd(cnt, __popcll(m));
  base = first_lane_value(base);
  if (prod) {
    const int i = base + count_below(m);
    if (i < lds_cap) lds_q[i] = make_int2(u, v);
    else if (i < qcap) g_q[i] = make_int2(u, v);
    else *status = ST_ENOMEM;
  }
}

__device__ __forceinline__ int xchg(int *p, int v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// com: resolve the equation u = v.  Returns true with (ou, ov) when it ends
// as an equation between two agents (a new active pair).  Every exchange that
// finds a filled cell consumes both occurrences of that name, so a chain is
// at most as long as the number of names; the guard only turns a broken
// invariant into an error instead of a spin.
__device__ __forceinline__ bool link(int u, int v, int *__restrict__ bind, int &ou, int &ov,
                                     int &loops, int *status) {
  for (int guard = 0;; guard++) {
    if (u >= 0) {
      if (v >= 0) { ou = u; ov = v; return true; }
      const int t = u; u = v; v = t;
    }
    if (u == v) { loops++; return false; }  // x = x: closed loop
    if (guard > (1 << 24)) { *status = ST_EINTERNAL; return false; }
    const int old = xchg(&bind[~u], v);
    if (old == EMPTY) return false;         // first occurrence: parked
    u = old;                                // second: old = v
  }
}

__device__ __forceinline__ int resolve(int op, int a, int b, int pa0, int pa1, int pb0, int pb1,
                                       int my_a, int my_n) {
  const int kind = op >> 4, idx = op & 15;
  if (kind == OP_AUX) return idx == 0 ? pa0 : (idx == 1 ? pa1 : (idx == 2 ? pb0 : pb1));
  if (kind == OP_NEW) return idx == 0 ? a : (idx == 1 ? b : my_a + idx - 2);
  return -1 - (my_n + idx);
}

// pointer jumping over the cells [lo, hi) with stride: a cell whose value is
// a name whose own cell is filled takes that cell's value (a com step)
__device__ __forceinline__ void jump_cells(int *__restrict__ bind, int lo, int hi, int stride) {
  for (int x = lo; x < hi; x += stride) {
    int v = bind[x];
    int hops = 0;
    while (v < 0 && hops < 64) {
      const int y = ~v;
      if (y == x) break;
      const int w = bind[y];
      if (w == EMPTY) break;
      v = w;
      hops++;
    }
    if (hops) bind[x] = v;
  }
}

template <int WG, int QCAP>
__global__ __launch_bounds__(WG) void k_reduce(const NetDesc *__restrict__ descs,
                                               const int *__restrict__ order, int n_nets,
                                               int *counter, const int *__restrict__ g_rules,
                                               int ns, int nr, unsigned max_steps, int flags) {
  extern __shared__ int s_rules[];
  __shared__ int2 q[2][QCAP];
  __shared__ int s_cnt[3];
  __shared__ int s_net;
  __shared__ int s_agent_top, s_name_top, s_status, s_nstuck, s_loops, s_maxf;
  __shared__ unsigned long long s_rc[INET_MAX_RULES];

  const int tid = threadIdx.x;
  const int nwords = ns * ns + nr * RT_WORDS + ns;
  for (int i = tid; i < nwords; i += WG) s_rules[i] = g_rules[i];
  const int *rule_of = s_rules;
  const int *templ = s_rules + ns * ns;
  const int *arity = templ + nr * RT_WORDS;

  for (;;) {
    __syncthreads();
    if (tid == 0) s_net = atomicAdd(counter, 1);
    __syncthreads();
    const int k = s_net;
    if (k >= n_nets) break;
    const NetDesc D = descs[order[k]];
    NetState *st = D.st;
    const int phase = st->phase;
    if (phase == PHASE_DONE || st->status == ST_ENOMEM || st->status == ST_EINTERNAL) continue;
    const int nfront = st->frontier;
    int cur = st->parity;
    unsigned steps = st->steps;
    // per-launch step budget (saturating)
    const unsigned stop = (max_steps > 0xffffffffu - steps) ? 0xffffffffu : steps + max_steps;
    if (tid == 0) {
      s_agent_top = st->agent_top;
      s_name_top = st->name_top;
      s_status = 0;
      s_nstuck = st->n_stuck;
      s_loops = 0;
      s_maxf = st->max_frontier;
      s_cnt[0] = (phase == PHASE_INIT) ? 0 : nfront;
      s_cnt[1] = 0;
      s_cnt[2] = 0;
    }
    for (int r = tid; r < nr; r += WG) s_rc[r] = 0ull;
    int ci = 0;
    if (phase == PHASE_INIT) {
      // the initial equations (queue0) are linked into buffer 1 (counter 1)
      __syncthreads();
      for (int base = 0; base < nfront; base += WG) {
        const int i = base + tid;
        const bool valid = i < nfront;
        int2 e = make_int2(0, 0);
        if (valid) e = D.queue0[i];
        int ou = 0, ov = 0, loops = 0;
        const bool prod = valid && link(e.x, e.y, D.bind, ou, ov, loops, &s_status);
        wave_push(prod, ou, ov, q[1], QCAP, D.queue1, D.qcap, &s_cnt[1], &s_status);
        if (loops) atomicAdd(&s_loops, loops);
      }
      cur = 1;
      ci = 1;
    } else {
      int2 *g = cur ? D.queue1 : D.queue0;
      const int nl = nfront < QCAP ? nfront : QCAP;
      for (int i = tid; i < nl; i += WG) q[cur][i] = g[i];
    }

    for (;;) {
      __syncthreads();
      const int n = s_cnt[ci];
      if (n == 0 || s_status < 0 || steps >= stop) break;
      const int cn = ci == 2 ? 0 : ci + 1;
      const int cnn = cn == 2 ? 0 : cn + 1;
      if (tid == 0) {
        s_cnt[cnn] = 0;
        if (n > s_maxf) s_maxf = n;
      }
      const int2 *cq_l = q[cur];
      const int2 *cq_g = cur ? D.queue1 : D.queue0;
      int2 *nq_l = q[cur ^ 1];
      int2 *nq_g = cur ? D.queue0 : D.queue1;
      for (int base = 0; base < n; base += WG) {
        const int i = base + tid;
        const bool valid = i < n;
        int2 rx = make_int2(0, 0);
        if (valid) rx = (i < QCAP) ? cq_l[i] : cq_g[i];
        int a = rx.x, b = rx.y;
        int la = 0, lb = 0, pa0 = 0, pa1 = 0, pb0 = 0, pb1 = 0;
        if (valid) {
          la = D.label[a];
          lb = D.label[b];
          pa0 = D.port0[a];
          pa1 = D.port1[a];
          pb0 = D.port0[b];
          pb1 = D.port1[b];
        }
        const int code = valid ? rule_of[la * ns + lb] : -1;
        // active pairs without a rule stay as residual equations
        {
          const bool stk = valid && code < 0;
          const unsigned long long m = ballot(stk);
          if (m) {
            int sb = 0;
            if (__lane_id() == 0) sb = atomicAdd(&s_nstuck, __popcll(m));
            sb = first_lane_value(sb);
            if (stk) {
              const int si = sb + count_below(m);
              if (si < D.scap) D.stuck[si] = make_int2(a, b);
              else s_status = ST_ENOMEM;
            }
          }
        }
        bool act = valid && code >= 0;
        const int rid = act ? (code >> 1) : 0;
        if (act && (code & 1)) {
          int t = a; a = b; b = t;
          t = pa0; pa0 = pb0; pb0 = t;
          t = pa1; pa1 = pb1; pb1 = t;
        }
        const int *T = templ + rid * RT_WORDS;
        const int nnew = act ? T[RT_NNEW] : 0;
        const int nalloc = act ? T[RT_NALLOC] : 0;
        const int nfresh = act ? T[RT_NFRESH] : 0;
        int neq = act ? T[RT_NEQ] : 0;
        // bump allocation: wave prefix sums, one LDS atomic per wave
        int ta, tn;
        const int oa = wave_scan16(nalloc, &ta);
        const int on = wave_scan16(nfresh, &tn);
        int ba = 0, bn = 0;
        if (__lane_id() == 0 && (ta | tn)) {
          ba = atomicAdd(&s_agent_top, ta);
          bn = atomicAdd(&s_name_top, tn);
        }
        ba = first_lane_value(ba);
        bn = first_lane_value(bn);
        const int my_a = ba + oa, my_n = bn + on;
        if (act && (my_a + nalloc > D.agent_cap || my_n + nfresh > D.name_cap)) {
          s_status = ST_ENOMEM;
          act = false;
          neq = 0;
        }
        if (act) {
          for (int kk = 0; kk < nnew; kk++) {
            const int slot = kk == 0 ? a : (kk == 1 ? b : my_a + kk - 2);
            const int L = T[RT_LABEL + kk];
            D.label[slot] = L;
            const int ar = arity[L];
            if (ar > 0)
              D.port0[slot] = resolve(T[RT_PORT + 2 * kk], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
            if (ar > 1)
              D.port1[slot] =
                  resolve(T[RT_PORT + 2 * kk + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
          }
          for (int f = 0; f < nfresh; f++) D.bind[my_n + f] = EMPTY;
          atomicAdd(&s_rc[rid], 1ull);
        }
        // com: the first exchange of every link equation is issued before
        // any result is awaited (independent cells), then chains continue
        int loops = 0;
        int eu[MAXEQ], ev[MAXEQ], eo[MAXEQ];
#pragma unroll
        for (int j = 0; j < MAXEQ; j++) {
          eo[j] = EMPTY;
          eu[j] = 0;
          ev[j] = 0;
          if (j < neq) {
            int u = resolve(T[RT_EQ + 2 * j], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
            int v = resolve(T[RT_EQ + 2 * j + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
            if (u >= 0) { const int t = u; u = v; v = t; }
            eu[j] = u;
            ev[j] = v;
            if (u < 0 && u != v) eo[j] = xchg(&D.bind[~u], v);
          }
        }
#pragma unroll
        for (int j = 0; j < MAXEQ; j++) {
          const bool has = j < neq;
          if (ballot(has) == 0ull) break;
          bool prod = false;
          int ou = 0, ov = 0;
          if (has) {
            const int u = eu[j], v = ev[j];
            if (u >= 0) {                       // both sides agents
              prod = true; ou = u; ov = v;
            } else if (u == v) {
              loops++;                          // x = x: closed loop
            } else if (eo[j] != EMPTY) {        // second occurrence: old = v
              prod = link(eo[j], v, D.bind, ou, ov, loops, &s_status);
            }
          }
          wave_push(prod, ou, ov, nq_l, QCAP, nq_g, D.qcap, &s_cnt[cn], &s_status);
        }
        if (loops) atomicAdd(&s_loops, loops);
      }
      steps++;
      cur ^= 1;
      ci = cn;
    }

    // the loop ends right after a barrier with uniform values
    const int n_left = s_cnt[ci];
    const int status = s_status;
    if (status >= 0 && n_left > 0) {
      int2 *g = cur ? D.queue1 : D.queue0;
      const int nl = n_left < QCAP ? n_left : QCAP;
      for (int i = tid; i < nl; i += WG) g[i] = q[cur][i];
    }
    for (int r = tid; r < nr; r += WG)
      if (s_rc[r]) D.per_rule[r] += s_rc[r];
    const bool done = status >= 0 && n_left == 0;
    if (tid == 0) {
      unsigned long long tot = 0;
      for (int r = 0; r < nr; r++) tot += s_rc[r];
      st->interactions += tot;
      st->steps = steps;
      st->agent_top = s_agent_top;
      st->name_top = s_name_top;
      st->n_stuck = s_nstuck;
      st->loops += s_loops;
      st->max_frontier = s_maxf;
      if (status < 0) {
        st->status = status;
      } else if (!done) {
        st->phase = PHASE_RUN;
        st->parity = cur;
        st->frontier = n_left;
        st->status = ST_ELIMIT;
      } else {
        st->phase = PHASE_DONE;
        st->frontier = 0;
        st->status = s_nstuck ? ST_STUCK : ST_OK;
      }
    }
    if ((flags & FLAG_JUMP) && done) {
      __syncthreads();
      jump_cells(D.bind, tid, s_name_top, WG);
    }
  }
}

// pointer jumping over one net's cells with the whole grid (single big nets)
__global__ __launch_bounds__(256) void k_jump_grid(const NetDesc *__restrict__ desc) {
  const NetDesc D = desc[0];
  if (D.st->phase != PHASE_DONE || D.st->status < 0) return;
  const int nn = D.st->name_top;
  jump_cells(D.bind, blockIdx.x * 256 + threadIdx.x, nn, gridDim.x * 256);
}

// restore every net to its loaded state
__global__ __launch_bounds__(256) void k_reset(const NetDesc *__restrict__ descs, int n_nets,
                                               const int *__restrict__ init_label,
                                               const int *__restrict__ init_port,
                                               const int *__restrict__ init_eq, int nr) {
  for (int ni = blockIdx.x; ni < n_nets; ni += gridDim.x) {
    const NetDesc D = descs[ni];
    const int *il = init_label + D.init_agent_off;
    const int *ip = init_port + 2 * D.init_agent_off;
    const int *ie = init_eq + 2 * D.init_eq_off;
    for (int i = threadIdx.x; i < D.n_agents0; i += 256) {
      D.label[i] = il[i];
      D.port0[i] = ip[2 * i];
      D.port1[i] = ip[2 * i + 1];
    }
    for (int i = threadIdx.x; i < D.n_eqs0; i += 256) D.queue0[i] = make_int2(ie[2 * i], ie[2 * i + 1]);
    for (int i = threadIdx.x; i < D.n_names0; i += 256) D.bind[i] = EMPTY;
    for (int i = threadIdx.x; i < nr; i += 256) D.per_rule[i] = 0ull;
    if (threadIdx.x == 0) {
      NetState s = {};
      s.agent_top = D.n_agents0;
      s.name_top = D.n_names0;
      s.frontier = D.n_eqs0;
      s.phase = PHASE_INIT;
      *D.st = s;
    }
  }
}

__global__ void k_zero(int *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// launchers

namespace {
template <int WG, int QCAP>
int launch_t(int grid, const NetDesc *d, const int32_t *ord, int n, int32_t *ctr, const int32_t *r,
             int ns, int nr, uint32_t ms, int flags, hipStream_t s) {
  const size_t dyn = (size_t)(ns * ns + nr * RT_WORDS + ns) * 4;
  hipLaunchKernelGGL((k_reduce<WG, QCAP>), dim3(grid), dim3(WG), dyn, s, d, ord, n, ctr, r, ns, nr,
                     ms, flags);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

template <int WG, int QCAP>
int occ_t(int ns, int nr, int *per_cu) {
  const size_t dyn = (size_t)(ns * ns + nr * RT_WORDS + ns) * 4;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (k_reduce<WG, QCAP>), WG, dyn) ==
                 hipSuccess
             ? INET_OK
             : INET_EHIP;
}
}  // namespace

bool shape_supported(int wg) {
  return wg == 64 || wg == 128 || wg == 256 || wg == 512 || wg == 1024;
}

LaunchShape shape_for(int wg) {
  switch (wg) {
    case 64: return {64, 512};
    case 128: return {128, 1024};
    case 256: return {256, 1024};
    case 512: return {512, 2048};
    default: return {1024, 4096};
  }
}

#define INET_SHAPES(X) X(64, 512) X(128, 1024) X(256, 1024) X(512, 2048) X(1024, 4096)

int launch_reduce(const LaunchShape &sh, int grid, const NetDesc *d, const int32_t *ord, int n,
                  int32_t *ctr, const int32_t *r, int ns, int nr, uint32_t ms, int flags,
                  hipStream_t s) {
#define X(W, Q) \
  if (sh.wg == W && sh.qcap == Q) return launch_t<W, Q>(grid, d, ord, n, ctr, r, ns, nr, ms, flags, s);
  INET_SHAPES(X)
#undef X
  return INET_EINVAL;
}

int max_resident(const LaunchShape &sh, int ns, int nr, int *per_cu, int *n_cu) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INET_EHIP;
  if (hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return INET_EHIP;
#define X(W, Q) \
  if (sh.wg == W && sh.qcap == Q) return occ_t<W, Q>(ns, nr, per_cu);
  INET_SHAPES(X)
#undef X
  return INET_EINVAL;
}

int launch_reset(const NetDesc *d, int n, const int32_t *il, const int32_t *ip, const int32_t *ie,
                 int nr, hipStream_t s) {
  const int grid = n < 4096 ? n : 4096;
  if (grid <= 0) return INET_OK;
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, s, d, n, il, ip, ie, nr);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

int launch_zero(int32_t *p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

int launch_jump_grid(const NetDesc *d, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_jump_grid, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError() == hipSuccess ? INET_OK : INET_EHIP;
}

}  // namespace inet
