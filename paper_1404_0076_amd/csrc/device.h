// device.h -- device code of the interaction-net evaluator (gfx950): the
// net-engine kernel body, the pointer-jumping, reset and counter kernels.
// Compiled ahead of time by kernels.hip (rule templates read at run time) and
// at load time through hipRTC with the rule table as compile-time constants
// (INET_STATIC_RULES), which turns each rule into straight-line code.
//
// One workgroup owns one net at a time ("net engine").  The frontier of
// active pairs lives in LDS (spilling to the net's global queue when it
// outgrows the LDS capacity), and every memory operation on the net's heap is
// performed at workgroup scope: a net never leaves the compute unit that is
// reducing it, so no cross-XCD coherence traffic is ever needed.  A step is
// the loop body of evaluate() (Section 3.6):
//   int  -- every lane takes one active pair, looks its rule up in the LDS
//           rule table, allocates the right-hand side's agents and names with
//           a wave-level scan (mask prefix counts, or a prefix sum in the
//           per-lane interpreter) and one counter update per wave (the
//           scan-based output allocation proposed in Section 4.2), and writes
//           the new agents as 16-byte records {label, port0, port1, -},
//           reusing the two slots of the pair;
//   com  -- each equation left by the rule is linked: a name side exchanges
//           the other side into the name's cell; the lane that finds the cell
//           already filled owns the second occurrence, forms the equation
//           (parked value = other side) and carries on along the chain; an
//           equation between two agents is a new active pair;
//   compaction -- new active pairs are appended to the next frontier with a
//           wave ballot, a mask prefix count and one counter update per wave.
// Engines of several waves separate steps with workgroup barriers (two per
// step: one after the step's writes, one after every wave has read the next
// step's control words); a single wave needs none (its memory operations are
// ordered).  After the
// loop, name-to-name chains left in the cells (the partial com of the remark
// after the correctness proposition of Section 3.6) are compressed by pointer
// jumping.
#ifndef INET_DEVICE_H
#define INET_DEVICE_H

#include "inet_internal.h"

namespace inet {

// heap pointers as global-address-space pointers: loads, stores and atomics
// then compile to global_* instructions (a flat access would also hold back
// every wait on LDS results)
typedef __attribute__((address_space(1))) int gint;
typedef __attribute__((address_space(1))) char gchar;
struct Pair {  // an equation or an active pair (POD, usable in any address space)
  int x, y;
};
__device__ __forceinline__ Pair mkpair(int x, int y) {
  Pair p;
  p.x = x;
  p.y = y;
  return p;
}
// in global memory a pair is one 64-bit word, x in the low half (the same
// bytes as an int2 {x, y})
typedef __attribute__((address_space(1))) unsigned long long gint2;
__device__ __forceinline__ gint2 *at2(gint2 *base, unsigned idx) {
  return (gint2 *)((gchar *)base + (idx << 3));
}
__device__ __forceinline__ unsigned long long pk(int x, int y) {
  return (unsigned long long)(unsigned)x | ((unsigned long long)(unsigned)y << 32);
}
__device__ __forceinline__ Pair unpk(unsigned long long w) {
  return mkpair((int)(unsigned)w, (int)(unsigned)(w >> 32));
}
typedef __attribute__((address_space(1))) unsigned long long gu64;

// element idx of a heap array as base + 32-bit byte offset (capacities stay
// below 2^29 elements of 8 bytes), which selects the scalar-base addressing
// form of the global instructions
__device__ __forceinline__ gint *at(gint *base, unsigned idx) {
  return (gint *)((gchar *)base + (idx << 2));
}

// an agent is one 16-byte record {label, port 0, port 1, unused}: one load or
// store moves a whole agent, and a record never straddles a cache line
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4i gv4i;
__device__ __forceinline__ gv4i *rec(gint *agent, unsigned idx) {
  return (gv4i *)((gchar *)agent + (idx << 4));
}
__device__ __forceinline__ v4i mkrec(int label, int p0, int p1) {
  v4i r;
  r.x = label;
  r.y = p0;
  r.z = p1;
  r.w = 0;
  return r;
}

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
__device__ __forceinline__ void wave_push(bool prod, int u, int v, Pair *lds_q, int lds_cap,
                                          gint2 *g_q, int qcap, int *cnt, int *status) {
  const unsigned long long m = ballot(prod);
  if (m == 0ull) return;
  int base = 0;
  if (__lane_id() == 0) base = atomicAdd(cnt, __popcll(m));
  base = first_lane_value(base);
  if (prod) {
    const int i = base + count_below(m);
    if (i < lds_cap) lds_q[i] = mkpair(u, v);
    else if (i < qcap) *at2(g_q, (unsigned)i) = pk(u, v);
    else *status = ST_ENOMEM;
  }
}

// name-cell exchange: relaxed, at agent scope, so that it is also atomic
// against the workgroups of a multi-workgroup engine (on gfx950 a relaxed
// exchange is the same instruction at workgroup and agent scope: atomics are
// performed at the L2)
__device__ __forceinline__ int xchg(gint *p, int v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// device-scope (agent) counters of a multi-workgroup engine
__device__ __forceinline__ int gadd(int *p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int gload(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gstore(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// com: resolve the equation u = v.  Returns true with (ou, ov) when it ends
// as an equation between two agents (a new active pair).  Every exchange that
// finds a filled cell consumes both occurrences of that name, so a chain is
// at most as long as the number of names; the guards only turn a broken
// invariant (an endless chain, a name outside the net's cells) into an error
// instead of a spin or a stray access.
__device__ __forceinline__ bool link(int u, int v, gint *__restrict__ bind, unsigned name_cap,
                                     int &ou, int &ov, int &loops, int *status) {
  for (int guard = 0;; guard++) {
    if (u >= 0) {
      if (v >= 0) { ou = u; ov = v; return true; }
      const int t = u; u = v; v = t;
    }
    if (u == v) { loops++; return false; }  // x = x: closed loop
    if (guard > (1 << 24) || (unsigned)~u >= name_cap) { *status = ST_EINTERNAL; return false; }
    const int old = xchg(at(bind, (unsigned)~u), v);
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

// operand of a rule template whose code is uniform across the wave: the
// kind/index tests become scalar branches and one move is left per lane
__device__ __forceinline__ int resolve_u(int op, int a, int b, int pa0, int pa1, int pb0, int pb1,
                                         int my_a, int my_n) {
  const int kind = op >> 4, idx = op & 15;
  if (kind == OP_AUX) {
    if (idx == 0) return pa0;
    if (idx == 1) return pa1;
    if (idx == 2) return pb0;
    return pb1;
  }
  if (kind == OP_NEW) {
    if (idx == 0) return a;
    if (idx == 1) return b;
    return my_a + (idx - 2);
  }
  return -1 - (my_n + idx);
}

// one pass of the interaction phase with the rule template interpreted per
// lane (ENGINE 1)
#define INET_PASS_ARGS                                                                    \
  bool valid, int a, int b, int la, int lb, int pa0, int pa1, int pb0, int pb1, const NetDesc &D, \
      gint *agent, gint *bind, gint2 *stuck, const int *rule_of,                                 \
      const int *templ, const int *arity, const int *__restrict__ g_templ,                          \
      const int *__restrict__ g_arity, int ns, Pair *nq_l, gint2 *nq_g, int *ncnt, int *s_status,  \
      int *s_agent_top, int *s_name_top, int *s_nstuck, int *s_loops, unsigned long long *s_rc

template <int QCAP>
__device__ __forceinline__ void stuck_push(bool stk, int a, int b, const NetDesc &D, gint2 *stuck,
                                           int *s_nstuck, int *s_status) {
  const unsigned long long m = ballot(stk);
  if (m) {
    int sb = 0;
    if (__lane_id() == 0) sb = atomicAdd(s_nstuck, __popcll(m));
    sb = first_lane_value(sb);
    if (stk) {
      const int si = sb + count_below(m);
      if (si < D.scap) *at2(stuck, (unsigned)si) = pk(a, b);
      else *s_status = ST_ENOMEM;
    }
  }
}

template <int QCAP>
__device__ __forceinline__ void pass_interp(INET_PASS_ARGS) {
  const int code = valid ? rule_of[valid ? la * ns + lb : 0] : -1;
  stuck_push<QCAP>(valid && code < 0, a, b, D, stuck, s_nstuck, s_status);
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
  int ta, tn;
  const int oa = wave_scan16(nalloc, &ta);
  const int on = wave_scan16(nfresh, &tn);
  int ba = 0, bn = 0;
  if (__lane_id() == 0 && (ta | tn)) {
    ba = atomicAdd(s_agent_top, ta);
    bn = atomicAdd(s_name_top, tn);
  }
  ba = first_lane_value(ba);
  bn = first_lane_value(bn);
  const int my_a = ba + oa, my_n = bn + on;
  if (act && (my_a + nalloc > D.agent_cap || my_n + nfresh > D.name_cap)) {
    *s_status = ST_ENOMEM;
    act = false;
    neq = 0;
  }
  if (act) {
    for (int kk = 0; kk < nnew; kk++) {
      const int slot = kk == 0 ? a : (kk == 1 ? b : my_a + kk - 2);
      const int L = T[RT_LABEL + kk];
      const int ar = arity[L];
      const int q0 = ar > 0 ? resolve(T[RT_PORT + 2 * kk], a, b, pa0, pa1, pb0, pb1, my_a, my_n) : 0;
      const int q1 = ar > 1 ? resolve(T[RT_PORT + 2 * kk + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n) : 0;
      *rec(agent, (unsigned)slot) = mkrec(L, q0, q1);
    }
    for (int f = 0; f < nfresh; f++) *at(bind, (unsigned)(my_n + f)) = EMPTY;
    atomicAdd(&s_rc[rid], 1ull);
  }
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
      if (u < 0 && u != v) eo[j] = xchg(at(bind, (unsigned)~u), v);
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
      if (u >= 0) { prod = true; ou = u; ov = v; }
      else if (u == v) loops++;
      else if (eo[j] != EMPTY) prod = link(eo[j], v, bind, (unsigned)D.name_cap, ou, ov, loops, s_status);
    }
    wave_push(prod, ou, ov, nq_l, QCAP, nq_g, D.qcap, ncnt, s_status);
  }
  if (loops) atomicAdd(s_loops, loops);
}

// decide each link -- a new active pair (prod), parked, a loop, or a chain --
// and append all new pairs of the wave with one LDS atomic
template <int QCAP, int MAXL>
__device__ __forceinline__ void finish_links(int lneq, int (&eu)[MAXL], int (&ev)[MAXL],
                                             int (&eo)[MAXL], const NetDesc &D, gint *bind,
                                             Pair *nq_l, gint2 *nq_g, int *ncnt, int *s_status,
                                             int *s_loops) {
  const int lane = __lane_id();
  int loops = 0;
  bool prod[MAXL];
  int ou[MAXL], ov[MAXL];
#pragma unroll
  for (int j = 0; j < MAXL; j++) {
    prod[j] = false;
    ou[j] = 0;
    ov[j] = 0;
    const bool has = j < lneq;
    const int u = eu[j], v = ev[j], o = eo[j];
    if (has) {
      if (u >= 0) { prod[j] = true; ou[j] = u; ov[j] = v; }
      else if (u == v) loops++;
      else if (o != EMPTY && o >= 0 && v >= 0) { prod[j] = true; ou[j] = o; ov[j] = v; }
    }
    const bool chain = has && u < 0 && u != v && o != EMPTY && !(o >= 0 && v >= 0);
    if (ballot(chain)) {
      if (chain) prod[j] = link(o, v, bind, (unsigned)D.name_cap, ou[j], ov[j], loops, s_status);
    }
  }
  // append all new pairs of the wave with one LDS atomic
  unsigned long long m[MAXL];
  int tot = 0;
#pragma unroll
  for (int j = 0; j < MAXL; j++) {
    m[j] = ballot(prod[j]);
    tot += __popcll(m[j]);
  }
  if (tot) {
    int base = 0;
    if (lane == 0) base = atomicAdd(ncnt, tot);
    base = first_lane_value(base);
#pragma unroll
    for (int j = 0; j < MAXL; j++) {
      if (prod[j]) {
        const int i = base + count_below(m[j]);
        if (i < QCAP) nq_l[i] = mkpair(ou[j], ov[j]);
        else if (i < D.qcap) *at2(nq_g, (unsigned)i) = pk(ou[j], ov[j]);
        else *s_status = ST_ENOMEM;
      }
      base += __popcll(m[j]);
    }
  }
  if (loops) atomicAdd(s_loops, loops);
}

// one pass with rule-uniform execution (ENGINE 2): the wave walks the
// distinct rules present among its lanes; for each, the template is read as
// scalars (constant cache), allocation is one mask count per group, and the
// operand choices are scalar branches.  MAXL bounds the links of any rule.
// The common com outcome -- the exchange returns a parked agent and the other
// side is an agent -- is decided inline; longer chains take the slow path.
// All new active pairs of the wave are appended with one LDS atomic.
template <int QCAP, int MAXL>
__device__ __forceinline__ void pass_uniform(INET_PASS_ARGS) {
  const int code = valid ? rule_of[valid ? la * ns + lb : 0] : -1;
  if (ballot(valid && code < 0)) stuck_push<QCAP>(valid && code < 0, a, b, D, stuck, s_nstuck, s_status);
  const bool act = valid && code >= 0;
  const int rid = act ? (code >> 1) : -1;
  if (act && (code & 1)) {
    int t = a; a = b; b = t;
    t = pa0; pa0 = pb0; pb0 = t;
    t = pa1; pa1 = pb1; pb1 = t;
  }
  int lneq = 0;
  int eu[MAXL], ev[MAXL], eo[MAXL];
#pragma unroll
  for (int j = 0; j < MAXL; j++) { eu[j] = 0; ev[j] = 0; eo[j] = EMPTY; }
  unsigned long long rem = ballot(act);
  const int lane = __lane_id();
  while (rem) {
    const int lead = __builtin_ctzll(rem);
    const int r = __builtin_amdgcn_readlane(rid, lead);
    const bool mine = rid == r;
    const unsigned long long gm = ballot(mine);
    rem &= ~gm;
    const int *__restrict__ T = g_templ + r * RT_WORDS;
    const int nnew = T[RT_NNEW], nalloc = T[RT_NALLOC], nfresh = T[RT_NFRESH], neq = T[RT_NEQ];
    const int cnt = __popcll(gm);
    const int rank = count_below(gm);
    int ba = 0, bn = 0;
    if (lane == lead) {
      if (nalloc) ba = atomicAdd(s_agent_top, nalloc * cnt);
      if (nfresh) bn = atomicAdd(s_name_top, nfresh * cnt);
      atomicAdd(&s_rc[r], (unsigned long long)cnt);
    }
    if (nalloc) ba = __builtin_amdgcn_readlane(ba, lead);
    if (nfresh) bn = __builtin_amdgcn_readlane(bn, lead);
    const int my_a = ba + nalloc * rank, my_n = bn + nfresh * rank;
    bool ok = mine;
    if (mine && (my_a + nalloc > D.agent_cap || my_n + nfresh > D.name_cap)) {
      *s_status = ST_ENOMEM;
      ok = false;
    }
    if (ok) {
      for (int kk = 0; kk < nnew; kk++) {
        const int slot = kk == 0 ? a : (kk == 1 ? b : my_a + kk - 2);
        const int L = T[RT_LABEL + kk];
        const int ar = g_arity[L];
        const int q0 = ar > 0 ? resolve_u(T[RT_PORT + 2 * kk], a, b, pa0, pa1, pb0, pb1, my_a, my_n) : 0;
        const int q1 = ar > 1 ? resolve_u(T[RT_PORT + 2 * kk + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n) : 0;
        *rec(agent, (unsigned)slot) = mkrec(L, q0, q1);
      }
      for (int f = 0; f < nfresh; f++) *at(bind, (unsigned)(my_n + f)) = EMPTY;
      lneq = neq;
#pragma unroll
      for (int j = 0; j < MAXL; j++) {
        if (j < neq) {
          int u = resolve_u(T[RT_EQ + 2 * j], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
          int v = resolve_u(T[RT_EQ + 2 * j + 1], a, b, pa0, pa1, pb0, pb1, my_a, my_n);
          if (u >= 0) { const int t = u; u = v; v = t; }
          eu[j] = u;
          ev[j] = v;
          if (u < 0 && u != v) eo[j] = xchg(at(bind, (unsigned)~u), v);
        }
      }
    }
  }
  finish_links<QCAP, MAXL>(lneq, eu, ev, eo, D, bind, nq_l, nq_g, ncnt, s_status, s_loops);
}

#ifdef INET_STATIC_RULES
// ---------------------------------------------------------------------------
// Engine 3: the rule table is compile-time data (namespace rt, generated at
// load time).  Each rule's right-hand side is straight-line code: labels,
// arities, operand kinds and link counts are constants.  A pass walks the
// distinct rules among the wave's lanes twice: the first walk allocates,
// writes the new agents and issues every name-cell exchange of the wave; the
// second decides each link knowing the rule's operand kinds (by then the
// exchanges of all groups are in flight together).  A single-wave engine
// keeps its heap tops, frontier count and error flag in registers.

template <int V>
struct IC {
  static constexpr int value = V;
};

// the rule code of every rule present among the wave's lanes, in rule order:
// straight-line code (one ballot per rule), so values produced for one rule
// (exchange results in flight) are not copied around a loop, which would wait
// for them; `rest` holds the lanes not handled yet, and the walk stops when
// none is left
template <int R, class F>
__device__ __forceinline__ void for_rules(int rid, unsigned long long rest, F &&f) {
  if constexpr (R < rt::NR) {
    if (rest) {
      const unsigned long long gm = ballot(rid == R);
      if (gm) f(IC<R>{}, gm);
      for_rules<R + 1>(rid, rest & ~gm, f);
    }
  }
}

struct Lane {  // a lane's active pair as the rule is stored, and its allocations
  int a, b, pa0, pa1, pb0, pb1, my_a, my_n;
};

template <int OP>
__device__ __forceinline__ int opnd(const Lane &L) {
  constexpr int kind = OP >> 4, idx = OP & 15;
  if constexpr (kind == OP_AUX) {
    if constexpr (idx == 0) return L.pa0;
    else if constexpr (idx == 1) return L.pa1;
    else if constexpr (idx == 2) return L.pb0;
    else return L.pb1;
  } else if constexpr (kind == OP_NEW) {
    if constexpr (idx == 0) return L.a;
    else if constexpr (idx == 1) return L.b;
    else return L.my_a + (idx - 2);
  } else {
    return -1 - (L.my_n + idx);
  }
}

// an opaque copy: the compiler cannot see through it, so tests on the value
// are not hoisted out of the rule code that uses them, and code after the
// copy does not wait again on the memory operation that produced the value
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// the engine's counters: wave-uniform registers when the engine is one wave
// (CM_REG), LDS words shared by the waves of the workgroup (CM_LDS), or, in a
// step shared by several workgroups (CM_GRID), the net's heap tops, residual
// count and status in global memory at agent scope with the new active pairs
// staged in the workgroup's LDS tile
enum { CM_REG = 0, CM_LDS = 1, CM_GRID = 2 };
template <int CM>
struct Ctr;

template <>
struct Ctr<CM_REG> {
  int agent_top, name_top, next, nstuck, err;
  __device__ __forceinline__ int agents(int n, int, int) {
    const int b = agent_top;
    agent_top += n;
    return b;
  }
  __device__ __forceinline__ int names(int n, int, int) {
    const int b = name_top;
    name_top += n;
    return b;
  }
  __device__ __forceinline__ int append(int n) {
    const int b = next;
    next += n;
    return b;
  }
  __device__ __forceinline__ int stuck(int n) {
    const int b = nstuck;
    nstuck += n;
    return b;
  }
  __device__ __forceinline__ void fail_uniform(int, int) { err = ST_ENOMEM; }
  // wave-uniform call: a lane out of queue space, or a broken chain invariant
  __device__ __forceinline__ void fail(bool nomem, bool internal) {
    if (ballot(nomem || internal)) err = ballot(internal) ? ST_EINTERNAL : ST_ENOMEM;
  }
};

template <>
struct Ctr<CM_LDS> {
  int *agent_top, *name_top, *next, *nstuck, *status;
  __device__ __forceinline__ int take(int *p, int n, int lane, int lead) {
    int b = 0;
    if (lane == lead) b = atomicAdd(p, n);
    return __builtin_amdgcn_readlane(b, lead);
  }
  __device__ __forceinline__ int append(int n) { return take(next, n, __lane_id(), 0); }
  __device__ __forceinline__ int stuck(int n) { return take(nstuck, n, __lane_id(), 0); }
  // agents and names for a whole wave, both atomics in flight together
  __device__ __forceinline__ void agents_names(int na, int nn, int &ba, int &bn) {
    int a = 0, b = 0;
    if (__lane_id() == 0) {
      if (na) a = atomicAdd(agent_top, na);
      if (nn) b = atomicAdd(name_top, nn);
    }
    ba = __builtin_amdgcn_readlane(a, 0);
    bn = __builtin_amdgcn_readlane(b, 0);
  }
  __device__ __forceinline__ void fail_uniform(int lane, int lead) {
    if (lane == lead) *status = ST_ENOMEM;
  }
  __device__ __forceinline__ void fail(bool nomem, bool internal) {
    if (internal) *status = ST_EINTERNAL;
    else if (nomem) *status = ST_ENOMEM;
  }
};

template <>
struct Ctr<CM_GRID> {
  int *agent_top, *name_top, *nstuck, *status;  // global (the net's state)
  int *next;                                    // LDS: entries in the tile
  int *lerr;                                    // LDS: an error in this step
  unsigned long long *spill_next;  // global: entries of all shared steps' frontiers
  unsigned long long base;         // *spill_next when this step began
  __device__ __forceinline__ int take(int *p, int n) {
    int b = 0;
    if (__lane_id() == 0) b = gadd(p, n);
    return __builtin_amdgcn_readfirstlane(b);
  }
  __device__ __forceinline__ int append(int n) {
    int b = 0;
    if (__lane_id() == 0) b = atomicAdd(next, n);
    return __builtin_amdgcn_readfirstlane(b);
  }
  // n entries past the LDS tile, straight into the global next frontier (the
  // index returned is relative to the step's frontier)
  __device__ __forceinline__ int spill(int n) {
    unsigned long long b = 0;
    if (__lane_id() == 0)
      b = __hip_atomic_fetch_add(spill_next, (unsigned long long)n, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane((int)(b - base));
  }
  __device__ __forceinline__ int stuck(int n) { return take(nstuck, n); }
  // agents and names for a whole wave.  When many workgroups share the step
  // and most waves of this one have pairs (`collective`, the same in every
  // wave) they are reserved for
  // the whole workgroup at once: the waves' needs are summed in LDS and one
  // thread takes them from the net's heap tops (two agent-scope atomics per
  // workgroup instead of two per wave, all on the same two words; every wave
  // then calls this, across two workgroup barriers).  Otherwise each wave
  // with a need takes its own.
  int *wneed, *wbase;  // LDS: needs of the waves so far [2], the workgroup's bases [2]
  bool collective;
  __device__ __forceinline__ void agents_names(int na, int nn, int &ba, int &bn) {
    if (!collective) {
      int a = 0, b = 0;
      if (__lane_id() == 0) {
        if (na) a = gadd(agent_top, na);
        if (nn) b = gadd(name_top, nn);
      }
      ba = __builtin_amdgcn_readfirstlane(a);
      bn = __builtin_amdgcn_readfirstlane(b);
      return;
    }
    int oa = 0, on = 0;
    if (__lane_id() == 0) {
      if (na) oa = atomicAdd(&wneed[0], na);
      if (nn) on = atomicAdd(&wneed[1], nn);
    }
    oa = __builtin_amdgcn_readfirstlane(oa);
    on = __builtin_amdgcn_readfirstlane(on);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int ta = wneed[0], tn = wneed[1];
      wbase[0] = ta ? gadd(agent_top, ta) : 0;
      wbase[1] = tn ? gadd(name_top, tn) : 0;
      wneed[0] = 0;
      wneed[1] = 0;
    }
    __syncthreads();
    ba = wbase[0] + oa;
    bn = wbase[1] + on;
  }
  __device__ __forceinline__ void fail_uniform(int lane, int lead) {
    if (lane == lead) {
      gstore(status, ST_ENOMEM);
      *lerr = 1;
    }
  }
  __device__ __forceinline__ void fail(bool nomem, bool internal) {
    if (internal) gstore(status, ST_EINTERNAL);
    else if (nomem) gstore(status, ST_ENOMEM);
    if (internal || nomem) *lerr = 1;
  }
};

template <int R, int K>
__device__ __forceinline__ void st_agents(const Lane &L, gint *agent) {
  if constexpr (K < rt::T[R][RT_NNEW]) {
    constexpr int LB = rt::T[R][RT_LABEL + K];
    const unsigned slot =
        K == 0 ? (unsigned)L.a : (K == 1 ? (unsigned)L.b : (unsigned)(L.my_a + K - 2));
    int q0 = 0, q1 = 0;
    if constexpr (rt::ARITY[LB] > 0) q0 = opnd<rt::T[R][RT_PORT + 2 * K]>(L);
    if constexpr (rt::ARITY[LB] > 1) q1 = opnd<rt::T[R][RT_PORT + 2 * K + 1]>(L);
    *rec(agent, slot) = mkrec(LB, q0, q1);
    st_agents<R, K + 1>(L, agent);
  }
}

// link J of rule R as (u, v) with the name side, if there is one, in u
template <int R, int J>
__device__ __forceinline__ void link_sides(const Lane &L, int &u, int &v) {
  constexpr int OU = rt::T[R][RT_EQ + 2 * J], OV = rt::T[R][RT_EQ + 2 * J + 1];
  if constexpr ((OU >> 4) == OP_NEW) {
    u = opnd<OV>(L);
    v = opnd<OU>(L);
  } else {
    u = opnd<OU>(L);
    v = opnd<OV>(L);
    if constexpr ((OU >> 4) == OP_AUX) {  // an argument: agent or name at run time
      const bool sw = u >= 0;
      const int t = u;
      u = sw ? v : u;
      v = sw ? t : v;
    }
  }
}

template <int R, int J>
struct LinkKind {
  static constexpr int OU = rt::T[R][RT_EQ + 2 * J], OV = rt::T[R][RT_EQ + 2 * J + 1];
  static constexpr bool both_new = (OU >> 4) == OP_NEW && (OV >> 4) == OP_NEW;
  // after link_sides, a v that survives the "both agents" test is an agent
  static constexpr bool v_agent = (OU >> 4) == OP_NEW || (OV >> 4) == OP_NEW;
  // a link whose name side is one of the rule's fresh names: folding leaves
  // a bound name at the top of an equation only in x = C[x] (its other
  // occurrence is inside the new agent C), so the cell was allocated by this
  // very interaction and is empty: the link parks C there without an exchange
  static constexpr bool fresh = (OU >> 4) == OP_FRESH || (OV >> 4) == OP_FRESH;
};

// fresh name F of rule R is the name side of one of its links (the cell then
// receives the parked term instead of EMPTY)
template <int R, int F, int J = 0>
constexpr bool fresh_linked() {
  if constexpr (J >= rt::T[R][RT_NEQ] || J >= MAXEQ) {
    return false;
  } else {
    constexpr int OU = rt::T[R][RT_EQ + 2 * J], OV = rt::T[R][RT_EQ + 2 * J + 1];
    constexpr int FC = (OP_FRESH << 4) | F;
    if constexpr (OU == FC || OV == FC) return true;
    else return fresh_linked<R, F, J + 1>();
  }
}

// initialise the rule's fresh name cells: EMPTY, except a cell that a link of
// the same interaction parks its term in (issue_links writes that one)
template <int R, int F>
__device__ __forceinline__ void st_fresh(const Lane &L, gint *bind) {
  if constexpr (F < rt::T[R][RT_NFRESH]) {
    if constexpr (!fresh_linked<R, F>()) *at(bind, (unsigned)(L.my_n + F)) = EMPTY;
    st_fresh<R, F + 1>(L, bind);
  }
}

// first walk, links: issue the exchange of every link whose name side is a
// name (a fresh name's cell is written directly: it holds nothing yet)
template <int R, int J, int MAXL>
__device__ __forceinline__ void issue_links(const Lane &L, gint *bind, int (&eo)[MAXL]) {
  if constexpr (J < rt::T[R][RT_NEQ] && J < MAXL) {
    if constexpr (LinkKind<R, J>::fresh) {
      int u, v;
      link_sides<R, J>(L, u, v);
      *at(bind, (unsigned)~u) = v;
      eo[J] = EMPTY;
    } else if constexpr (!LinkKind<R, J>::both_new) {
      int u, v;
      link_sides<R, J>(L, u, v);
      int e = EMPTY;
      if (u < 0 && u != v) e = xchg(at(bind, (unsigned)~u), v);
      eo[J] = e;
    }
    issue_links<R, J + 1, MAXL>(L, bind, eo);
  }
}

// second walk, links: a new active pair (pu[J] >= 0: both sides are agents),
// a parked side, a closed loop, or a chain (the exchange met a parked name:
// com carries on along it)
template <int R, int J, int MAXL>
__device__ __forceinline__ void decide_links(const Lane &L, gint *bind, unsigned name_cap,
                                             const int (&eo)[MAXL],
                                             int (&pu)[MAXL], int (&pv)[MAXL], int &loops,
                                             bool &bad) {
  if constexpr (J < rt::T[R][RT_NEQ] && J < MAXL) {
    using K = LinkKind<R, J>;
    if constexpr (K::both_new) {
      pu[J] = opnd<K::OV>(L);
      pv[J] = opnd<K::OU>(L);
    } else {
      int u, v;
      link_sides<R, J>(L, u, v);
      const int o = opaque(eo[J]);
      // the cases as selects, not nested branches (each divergent branch
      // costs exec-mask updates): both sides agents; a closed loop; the
      // exchange met an agent (a pair) or a name (a chain); else parked
      const bool direct = u >= 0;
      const bool loop = !direct && u == v;
      const bool met = !direct && !loop && o != EMPTY;
      const bool pair = met && o >= 0 && (K::v_agent || v >= 0);
      const bool chain = met && !pair;
      pu[J] = direct ? u : (pair ? o : -1);
      pv[J] = v;
      loops += loop ? 1 : 0;
      if (ballot(chain)) {
        if (chain) {
          int ou = -1, ov = 0;
          int guard = 0;
          if (!link(o, v, bind, name_cap, ou, ov, loops, &guard)) ou = -1;
          if (guard) bad = true;
          pu[J] = ou;
          pv[J] = ov;
        }
      }
    }
    decide_links<R, J + 1, MAXL>(L, bind, name_cap, eo, pu, pv, loops, bad);
  }
}

// LANE: the atomic-append variant (the proposal of Section 4.2 to drop the
// merge of result arrays): every lane reserves its own agents, cells and
// frontier entries with one atomic each, instead of one reservation per rule
// group of a wave ranked by mask counts
// HOLD (one-wave steps): the lane keeps its first new active pair in
// registers (ha, hb; ha < 0 if none) and appends only the others
template <int QCAP, int MAXL, int CM, bool LANE, bool HOLD = false>
__device__ __forceinline__ void pass_static(bool valid, int a, int b, int la, int lb, int pa0,
                                            int pa1, int pb0, int pb1, const NetDesc &D,
                                            gint *agent, gint *bind,
                                            gint2 *stuck, const int *rule_of, Pair *nq_l,
                                            gint2 *nq_g, Ctr<CM> &C, int &loops_lane,
                                            unsigned &rc_lane, int &ha, int &hb) {
  constexpr bool SOLO = CM == CM_REG;
  const int lane = __lane_id();
  const int code = rule_of[valid ? la * rt::NS + lb : 0];
  // take the loaded ports through a copy on every path: later rule blocks then
  // never wait on these loads, a wait that would also hold for the exchanges
  // issued by earlier blocks
  pa0 = opaque(pa0);
  pa1 = opaque(pa1);
  pb0 = opaque(pb0);
  pb1 = opaque(pb1);
  bool lane_err = false;
  const bool stk = valid && code < 0;
  const unsigned long long sm = ballot(stk);
  if (sm) {  // active pairs without a rule: residuals
    const int sb = C.stuck(__popcll(sm));
    if (stk) {
      const int si = sb + count_below(sm);
      if (si < D.scap) *at2(stuck, (unsigned)si) = pk(a, b);
      else lane_err = true;
    }
  }
  const bool act = valid && code >= 0;
  // the lane's rule; -1 when it has none, or when its group could not be
  // allocated (the second walk then leaves it alone)
  int rid = act ? (code >> 1) : -1;
  // the pair in the rule's orientation (selects, not a divergent branch)
  const bool sw = act && (code & 1);
  Lane L;
  L.a = sw ? b : a;
  L.b = sw ? a : b;
  L.pa0 = sw ? pb0 : pa0;
  L.pb0 = sw ? pa0 : pb0;
  L.pa1 = sw ? pb1 : pa1;
  L.pb1 = sw ? pa1 : pb1;
  L.my_a = 0; L.my_n = 0;
  // exchange results, one register per (rule, link): exchanges of different
  // rules are then in flight together without write-after-write waits
  // (written by the first walk for every lane of the rule's group, and read
  // by the second walk only for those lanes)
  int eo[rt::NR > 0 ? rt::NR : 1][MAXL];
  int pu[MAXL], pv[MAXL];  // new active pair of link j, pu[j] < 0 if none
#pragma unroll
  for (int j = 0; j < MAXL; j++) { pu[j] = -1; pv[j] = 0; }
  // a wave of a wider engine reserves the agents and cells of all its rule
  // groups at once (one pair of LDS atomics, not one per rule group)
  int wa = 0, wn = 0;
  if constexpr (!SOLO && !LANE) {
    int need_a = 0, need_n = 0;
    for_rules<0>(rid, ballot(rid >= 0), [&](auto ic, unsigned long long gm) {
      constexpr int R = decltype(ic)::value;
      need_a += rt::T[R][RT_NALLOC] * __popcll(gm);
      need_n += rt::T[R][RT_NFRESH] * __popcll(gm);
    });
    bool call = (need_a | need_n) != 0;
    if constexpr (CM == CM_GRID) call = call || C.collective;  // then every wave
    if (call) C.agents_names(need_a, need_n, wa, wn);
  }
  // first walk: allocate, write the new agents, issue the exchanges
  for_rules<0>(rid, ballot(rid >= 0), [&](auto ic, unsigned long long gm) {
      constexpr int R = decltype(ic)::value;
      constexpr int nalloc = rt::T[R][RT_NALLOC], nfresh = rt::T[R][RT_NFRESH];
      const bool mine = rid == R;
      const int cnt = __popcll(gm);
      if constexpr (LANE) {
        rc_lane += opaque(lane) == R ? (unsigned)cnt : 0u;
        if (mine) {
          int ma = 0, mn = 0;
          if constexpr (nalloc > 0) ma = atomicAdd(C.agent_top, nalloc);
          if constexpr (nfresh > 0) mn = atomicAdd(C.name_top, nfresh);
          if ((nalloc > 0 && ma + nalloc > D.agent_cap) ||
              (nfresh > 0 && mn + nfresh > D.name_cap)) {
            *C.status = ST_ENOMEM;  // the step ends with ENOMEM; this lane issues nothing
            rid = -1;
          } else {
            Lane X = L;
            X.my_a = ma;
            X.my_n = mn;
            L.my_a = X.my_a;
            L.my_n = X.my_n;
            issue_links<R, 0, MAXL>(X, bind, eo[R]);
            st_agents<R, 0>(X, agent);
            st_fresh<R, 0>(X, bind);
          }
        }
      } else {
        const int lead = __builtin_ctzll(gm);
        int ba = 0, bn = 0;
        if constexpr (SOLO) {
          if constexpr (nalloc > 0) ba = C.agents(nalloc * cnt, lane, lead);
          if constexpr (nfresh > 0) bn = C.names(nfresh * cnt, lane, lead);
        } else {
          ba = wa;
          bn = wn;
          wa += nalloc * cnt;
          wn += nfresh * cnt;
        }
        // interactions per rule: lane R of the wave counts rule R (the lane id
        // is opaque so that the test is not hoisted, per rule, out of the loop)
        rc_lane += opaque(lane) == R ? (unsigned)cnt : 0u;
        if ((nalloc > 0 && ba + nalloc * cnt > D.agent_cap) ||
            (nfresh > 0 && bn + nfresh * cnt > D.name_cap)) {
          // out of heap: the step ends with ENOMEM; these lanes issue nothing,
          // and their exchange results are never read
          C.fail_uniform(lane, lead);
          if (mine) rid = -1;
          return;
        }
        if (mine) {
          const int rank = count_below(gm);
          Lane X = L;
          X.my_a = ba + nalloc * rank;
          X.my_n = bn + nfresh * rank;
          L.my_a = X.my_a;
          L.my_n = X.my_n;
          // the exchanges first, so that they are in flight while the new
          // agents and cells are written (a lane reads agent records only at
          // the next step; an exchange never targets a fresh cell of the same
          // interaction: a link on one parks its term with a plain store, and
          // st_fresh leaves that cell alone)
          issue_links<R, 0, MAXL>(X, bind, eo[R]);
          st_agents<R, 0>(X, agent);
          st_fresh<R, 0>(X, bind);
        }
      }
  });
  // second walk: decide every link
  int loops = 0;
  bool bad = false;
  for_rules<0>(rid, ballot(rid >= 0), [&](auto ic, unsigned long long) {
    constexpr int R = decltype(ic)::value;
    if (rid == R)
      decide_links<R, 0, MAXL>(L, bind, (unsigned)D.name_cap, eo[R], pu, pv, loops, bad);
  });
  if constexpr (HOLD) {
    int h_a = -1, h_b = 0;
#pragma unroll
    for (int j = 0; j < MAXL; j++) {
      const bool take = h_a < 0 && pu[j] >= 0;
      h_a = take ? pu[j] : h_a;
      h_b = take ? pv[j] : h_b;
      pu[j] = take ? -1 : pu[j];
    }
    ha = h_a;
    hb = h_b;
  }
  // append the wave's new active pairs
  if constexpr (LANE) {
#pragma unroll
    for (int j = 0; j < MAXL; j++) {
      if (pu[j] >= 0) {
        const int i = atomicAdd(C.next, 1);
        if (i < QCAP) nq_l[i] = mkpair(pu[j], pv[j]);
        else if (i < D.qcap) *at2(nq_g, (unsigned)i) = pk(pu[j], pv[j]);
        else lane_err = true;
      }
    }
  }
  unsigned long long m[MAXL];
  int tot = 0;
#pragma unroll
  for (int j = 0; j < MAXL; j++) {
    m[j] = LANE ? 0ull : ballot(pu[j] >= 0);
    tot += __popcll(m[j]);
  }
  if (tot) {
    int base = C.append(tot);
    if (base + tot <= QCAP) {
      // all in the LDS tile: one store per link slot and lane, without a
      // branch (a lane without a pair on the slot writes its spare slot)
#pragma unroll
      for (int j = 0; j < MAXL; j++) {
        if (m[j]) {
          const int i = pu[j] >= 0 ? base + count_below(m[j]) : QCAP + lane;
          nq_l[i] = mkpair(pu[j], pv[j]);
          base += __popcll(m[j]);
        }
      }
    } else {
      // entries past the LDS tile go to the global queue: at the same index
      // when one workgroup owns the net, else at a range of the shared next
      // frontier reserved for this wave's overflow
      int gofs = 0;
      if constexpr (CM == CM_GRID) {
        const int first = base > QCAP ? base : QCAP;
        gofs = C.spill(base + tot - first) - first;
      }
#pragma unroll
      for (int j = 0; j < MAXL; j++) {
        if (pu[j] >= 0) {
          const int i = base + count_below(m[j]);
          if (i < QCAP) nq_l[i] = mkpair(pu[j], pv[j]);
          else if (i + gofs < D.qcap) *at2(nq_g, (unsigned)(i + gofs)) = pk(pu[j], pv[j]);
          else lane_err = true;
        }
        base += __popcll(m[j]);
      }
    }
  }
  loops_lane += loops;
  C.fail(lane_err, bad);
}

// the active pair of frontier slot base + tid and its two agents; lanes
// without a pair read slot 0 (always allocated) and stay idle, so the loads
// need no branch
template <int WG, int QCAP>
__device__ __forceinline__ void fetch_pair(int base, int n, int tid, const Pair *cq_l,
                                           const gint2 *cq_g, gint *agent, bool &valid, int &a,
                                           int &b, int &la,
                                           int &lb, int &pa0, int &pa1, int &pb0, int &pb1) {
  const int i = base + tid;
  valid = i < n;
  Pair rx = mkpair(0, 0);
  if (base + WG <= QCAP) {
    rx = cq_l[valid ? i : 0];
  } else if (valid) {
    if (i < QCAP) rx = cq_l[i];
    else rx = unpk(*at2((gint2 *)cq_g, (unsigned)i));
  }
  if (!valid) rx = mkpair(0, 0);
  a = rx.x;
  b = rx.y;
  const v4i ra = *rec(agent, (unsigned)a), rb = *rec(agent, (unsigned)b);
  la = ra.x;
  pa0 = ra.y;
  pa1 = ra.z;
  lb = rb.x;
  pb0 = rb.y;
  pb1 = rb.z;
}
#endif  // INET_STATIC_RULES

// Pointer jumping (com along name chains, Section 3.6): a cell x that holds a
// name y whose own cell holds a term t takes t (x = y and y = t give x = t).
// One hop per cell and round; applied to every cell in rounds separated by
// barriers, this at least halves every chain per round, so a chain of L names
// is one hop after ceil(log2 L) rounds.  A hop that would make a cell hold its
// own name is skipped (it would only close a vicious circle, whose cells are
// reachable from no agent and no interface name).
__device__ __forceinline__ bool jump_hop(gint *__restrict__ bind, int x) {
  const int v = bind[x];
  if (v >= 0) return false;  // an agent, or EMPTY
  const int y = ~v;
  if (y == x) return false;
  const int w = bind[y];
  if (w == EMPTY || w == ~x || w == v) return false;
  bind[x] = w;
  return true;
}

// wait until the epoch counter moves past `seen`; false on give-up after
// `timeout` wall-clock ticks without progress (no new epoch and no change of
// the heartbeat word).  Polls back off from tens of nanoseconds to
// microseconds the longer the wait lasts.
__device__ __forceinline__ bool wait_epoch(GridCtl *ctl, int seen, unsigned long long timeout) {
  unsigned long long t0 = wall_clock64();
  int hb = gload(&ctl->heartbeat);
  for (int polls = 0;; polls++) {
    if (gload(&ctl->gen) != seen) return true;
    const int h = gload(&ctl->heartbeat);
    const unsigned long long t = wall_clock64();
    if (h != hb) {
      hb = h;
      t0 = t;
    } else if (t - t0 > timeout) {
      return false;
    }
    if (polls < 256) __builtin_amdgcn_s_sleep(1);
    else if (polls < 4096) __builtin_amdgcn_s_sleep(32);
    else __builtin_amdgcn_s_sleep(127);
  }
}

// barrier over all G workgroups of a launch (every workgroup arrives); thread
// 0 of each workgroup holds `seen`, the epoch it last saw.  `last` runs in the
// last arriving workgroup before the others are released.  False on give-up.
template <class F>
__device__ __forceinline__ bool grid_sync(GridCtl *ctl, int G, int &seen, unsigned long long timeout,
                                          F &&last) {
  bool ok = true;
  // every wave's stores in the L2 before the workgroup barrier (which waits
  // for LDS traffic only), then one agent-scope release by thread 0
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    if (gadd(&ctl->arrive, 1) == G - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      last();
      gstore(&ctl->arrive, 0);
      __hip_atomic_store(&ctl->gen, seen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      ok = wait_epoch(ctl, seen, timeout);
    }
    seen++;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
  }
  return ok;
}

// an epoch entry of the multi-workgroup engine
__device__ __forceinline__ unsigned long long ent_pack(int epoch, bool err, int count) {
  return ((unsigned long long)(unsigned)epoch << 32) | (err ? 0x80000000ull : 0ull) |
         (unsigned long long)(unsigned)(count & 0x7fffffff);
}

// wave 0 of a workgroup: wait until all G entries of the epoch are posted;
// their new-pair counts summed and error bits or'ed (the same values in every
// lane).  False on give-up after `timeout` wall-clock ticks without progress
// (a missing entry and no change of the heartbeat word).  Polls back off from
// tens of nanoseconds to microseconds the longer the wait lasts.
__device__ __forceinline__ bool wait_entries(GridCtl *ctl, int G, int epoch,
                                             unsigned long long timeout, int &sum, bool &err) {
  const int lane = __lane_id();
  const unsigned long long *ent = ctl->ent[epoch & 1];
  unsigned long long t0 = wall_clock64();
  int hb = gload(&ctl->heartbeat);
  for (int polls = 0;; polls++) {
    int s = 0;
    bool e = false, all = true;
    for (int w = lane; w < G; w += 64) {
      const unsigned long long v =
          __hip_atomic_load(&ent[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      all = all && (int)(v >> 32) == epoch;
      s += (int)(v & 0x7fffffffull);
      e = e || (v & 0x80000000ull) != 0;
    }
    if (!ballot(!all)) {
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      sum = s;
      err = ballot(e) != 0;
      return true;
    }
    const int h = gload(&ctl->heartbeat);
    const unsigned long long t = wall_clock64();
    if (h != hb) {
      hb = h;
      t0 = t;
    } else if (t - t0 > timeout) {
      return false;
    }
    if (polls < 256) __builtin_amdgcn_s_sleep(1);
    else if (polls < 4096) __builtin_amdgcn_s_sleep(32);
    else __builtin_amdgcn_s_sleep(127);
  }
}

// pointer jumping over one net's cells by one workgroup (`flag`: an LDS word)
template <int WG>
__device__ __forceinline__ void jump_net(gint *__restrict__ bind, int n_cells, int *flag) {
  for (int round = 0; round < 32; round++) {
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    bool moved = false;
    for (int x = threadIdx.x; x < n_cells; x += WG) moved |= jump_hop(bind, x);
    if (moved) *flag = 1;
    __syncthreads();
    const int again = *flag;
    __syncthreads();
    if (!again) break;
  }
}

// LDS state of one net engine (one workgroup)
template <int QCAP>
struct EngineLds {
  Pair q[2][QCAP + 64];  // frontier double buffer (+ a spare slot per lane, for the append)
  int cnt[3];
  int net;
  int agent_top, name_top, status, nstuck, loops, maxf;
  unsigned steps;  // hand-over from one-wave steps (engine 3)
  int cur;
  unsigned long long rc[MAXRULES];
  int bcast[8];    // values broadcast to the workgroup (multi-workgroup engine)
  int wneed[2], wbase[2];  // multi-workgroup engine: the workgroup's heap reservation
};

// The rule table in LDS: rule_of[ns*ns] | templates[nr][RT_WORDS] | arity[ns]
struct RuleView {
  const int *rule_of, *templ, *arity;            // LDS
  const int *__restrict__ g_templ, *__restrict__ g_arity;  // global (scalar reads)
  int ns, nr;
};

// One net on one workgroup, from its saved state: the initial equations are
// linked (first launch), then parallel steps run until no active pair is
// left, the absolute step budget `stop` is reached or an error occurs; the
// state is saved back into the net's NetState and queues.  NARROW: the
// narrow phase of the multi-workgroup engine, which also stops once more than
// `hi` pairs are active (the other workgroups then take the net over) and
// publishes its step count in *hb every 1024 steps (progress seen by the
// workgroups waiting on it).  TRACE: the number of active pairs of each step
// goes to the net's trace buffer, if it has one.  Both are compile-time so
// that the batch kernel carries neither.  SOLO_MAX: wider engines step with
// wave 0 alone while at most this many pairs are active (a compile-time
// bound: the one-wave loop is then specialised for it).
template <int WG, int QCAP, int ENGINE, int MAXL, bool NARROW = false, bool TRACE = false,
          int SOLO_MAX = 64>
__device__ __forceinline__ void engine_net(EngineLds<QCAP> &S, const NetDesc &D, const RuleView &RV,
                                           unsigned stop, int flags, int hi, const KParams &kp,
                                           int *hb) {
  const int tid = threadIdx.x;
  const int *rule_of = RV.rule_of;
  const int nr = RV.nr;
  NetState *st = D.st;
  gint *const agent = (gint *)D.agent;
  gint *const bind = (gint *)D.bind;
  gint2 *const queue0 = (gint2 *)D.queue0;
  gint2 *const queue1 = (gint2 *)D.queue1;
  gint2 *const stuck = (gint2 *)D.stuck;
  const int phase = st->phase;
  if (phase == PHASE_DONE || st->status == ST_ENOMEM || st->status == ST_EINTERNAL ||
      st->status == ST_ETIMEDOUT)
    return;
  const int nfront = st->frontier;
  int cur = st->parity;
  unsigned steps = st->steps;
  if (tid == 0) {
    S.agent_top = st->agent_top;
    S.name_top = st->name_top;
    S.status = 0;
    S.nstuck = st->n_stuck;
    S.loops = 0;
    S.maxf = st->max_frontier;
    S.cnt[0] = (phase == PHASE_INIT) ? 0 : nfront;
    S.cnt[1] = 0;
    S.cnt[2] = 0;
  }
  for (int r = tid; r < nr; r += WG) S.rc[r] = 0ull;
  int ci = 0;
  if (phase == PHASE_INIT) {
    // the initial equations (queue0) are linked into buffer 1 (counter 1)
    __syncthreads();
    for (int base = 0; base < nfront; base += WG) {
      const int i = base + tid;
      const bool valid = i < nfront;
      Pair e = mkpair(0, 0);
      if (valid) e = unpk(queue0[i]);
      int ou = 0, ov = 0, loops = 0;
      const bool prod = valid && link(e.x, e.y, bind, (unsigned)D.name_cap, ou, ov, loops, &S.status);
      wave_push(prod, ou, ov, S.q[1], QCAP, queue1, D.qcap, &S.cnt[1], &S.status);
      if (loops) atomicAdd(&S.loops, loops);
    }
    cur = 1;
    ci = 1;
  } else {
    gint2 *g = cur ? queue1 : queue0;
    const int nl = nfront < QCAP ? nfront : QCAP;
    for (int i = tid; i < nl; i += WG) S.q[cur][i] = unpk(g[i]);
  }

#ifdef INET_STATIC_RULES
  if constexpr (ENGINE == 3 || ENGINE == 4) {
    // engine 4 reserves heap and frontier space per lane (atomic append);
    // its counters are shared words, so it always steps as a group
    constexpr bool LANE = ENGINE == 4;
    unsigned rc_lane = 0;  // lane r of each wave: interactions of rule r in this launch
    int loops_lane = 0;    // closed loops dropped by this lane
    // Steps of wave 0 alone, while the frontier holds at most `limit` pairs:
    // the counters live in registers and no barrier separates steps (a
    // wave's own memory operations are performed in order).  The other waves
    // of a wider engine wait at the caller's barrier meanwhile.  On return
    // the state is back in LDS, with the frontier count in S.cnt[ci].
    // While the pairs of a step fit the wave, each lane keeps its first new
    // pair in registers for the next step (no LDS round trip); only the
    // others go through the LDS frontier, and lanes without a pair take
    // them by rank.  Wider steps run from the LDS frontier in chunks.
    auto solo = [&](int limit) {
      Ctr<CM_REG> C;
      C.agent_top = __builtin_amdgcn_readfirstlane(S.agent_top);
      C.name_top = __builtin_amdgcn_readfirstlane(S.name_top);
      C.nstuck = __builtin_amdgcn_readfirstlane(S.nstuck);
      C.err = __builtin_amdgcn_readfirstlane(S.status);
      C.next = 0;
      int n = __builtin_amdgcn_readfirstlane(S.cnt[ci]);  // pairs in the frontier q[cur]
      int maxf = __builtin_amdgcn_readfirstlane(S.maxf);
      // the step count and budget are wave-uniform (they come from global
      // loads, which the compiler cannot see as uniform): in scalar registers
      // the loop's exit is a scalar branch and the loop needs no exec-mask
      // bookkeeping, and every value carried round it stays scalar too
      steps = __builtin_amdgcn_readfirstlane(steps);
      const unsigned stop_w = __builtin_amdgcn_readfirstlane(stop);
      int ha = -1, hb_ = 0;  // the lane's held pair (ha < 0: none)
      int nh = 0;            // held pairs of the wave
      // the held pairs back into the frontier, after its n pairs
      auto release = [&]() {
        if (nh) {
          const unsigned long long hm = ballot(ha >= 0);
          bool over = false;
          if (ha >= 0) {
            const int i = n + count_below(hm);
            if (i < QCAP) S.q[cur][i] = mkpair(ha, hb_);
            else if (i < D.qcap) *at2(cur ? queue1 : queue0, (unsigned)i) = pk(ha, hb_);
            else over = true;
          }
          C.fail(over, false);
          n += nh;
          nh = 0;
          ha = -1;
        }
      };
      for (;;) {
        const int tot = n + nh;
        if (!(tot > 0 && tot <= limit && C.err >= 0 && steps < stop_w)) break;
        if (tot > maxf) maxf = tot;
        if constexpr (NARROW)
          if ((steps & 1023u) == 0 && __lane_id() == 0) gstore(hb, (int)steps);
        if constexpr (TRACE)
          if (D.trace && steps < (unsigned)D.trace_cap && __lane_id() == 0) D.trace[steps] = tot;
        const Pair *cq_l = S.q[cur];
        const gint2 *cq_g = cur ? queue1 : queue0;
        Pair *nq_l = S.q[cur ^ 1];
        gint2 *nq_g = cur ? queue0 : queue1;
        C.next = 0;
        int nha = -1, nhb = 0;
        if (tot <= 64) {
          // held pairs stay with their lanes; the n frontier pairs (all in
          // the LDS tile: n <= 64) go to the free lanes by rank
          const int r = count_below(ballot(ha < 0));
          const bool take = ha < 0 && r < n;
          const Pair rx = cq_l[take ? r : 0];
          const bool valid = ha >= 0 || take;
          const int a = ha >= 0 ? ha : (take ? rx.x : 0);
          const int b = ha >= 0 ? hb_ : (take ? rx.y : 0);
          const v4i ra = *rec(agent, (unsigned)a), rb = *rec(agent, (unsigned)b);
          pass_static<QCAP, MAXL, CM_REG, false, true>(valid, a, b, ra.x, rb.x, ra.y, ra.z, rb.y,
                                                       rb.z, D, agent, bind, stuck, rule_of, nq_l,
                                                       nq_g, C, loops_lane, rc_lane, nha, nhb);
        } else {
          release();
          for (int base = 0; base < n; base += 64) {
            bool valid;
            int a, b, la, lb, pa0, pa1, pb0, pb1;
            fetch_pair<64, QCAP>(base, n, tid, cq_l, cq_g, agent, valid, a, b, la, lb, pa0,
                                 pa1, pb0, pb1);
            pass_static<QCAP, MAXL, CM_REG, false>(valid, a, b, la, lb, pa0, pa1, pb0, pb1, D,
                                                   agent, bind, stuck, rule_of, nq_l, nq_g, C,
                                                   loops_lane, rc_lane, nha, nhb);
          }
        }
        // lanes of one wave need no cache action or wait to see each
        // other's writes (wavefront scope); the fence only keeps the
        // compiler from moving memory operations across steps
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        steps++;
        cur ^= 1;
        n = C.next;
        ha = nha;
        hb_ = nhb;
        nh = __popcll(ballot(ha >= 0));
      }
      release();  // the frontier whole in q[cur] again, for the caller
      if (tid == 0) {
        S.cnt[ci] = n;
        S.cnt[ci == 2 ? 0 : ci + 1] = 0;
        S.cnt[ci == 0 ? 2 : ci - 1] = 0;
        S.agent_top = C.agent_top;
        S.name_top = C.name_top;
        S.nstuck = C.nstuck;
        S.maxf = maxf;
        S.steps = steps;
        S.cur = cur;
        if (C.err < 0) S.status = C.err;
      }
    };
    // the one-wave loop specialised for a compile-time bound; a hand-over
    // threshold below it (narrow phase) takes a second, generic copy
    const int solo_max = (NARROW && hi < SOLO_MAX) ? hi : SOLO_MAX;
    if constexpr (WG == 64 && !LANE) {
      __syncthreads();
      if (!NARROW) solo(0x7fffffff);
      else solo(hi);
      if (rc_lane) atomicAdd(&S.rc[tid], (unsigned long long)rc_lane);
      if (loops_lane) atomicAdd(&S.loops, loops_lane);
      __syncthreads();
    } else {
      // a wider engine: all waves step together while the frontier is wider
      // than solo_max pairs, wave 0 alone while it is not
      Ctr<CM_LDS> C;
      C.agent_top = &S.agent_top;
      C.name_top = &S.name_top;
      C.nstuck = &S.nstuck;
      C.status = &S.status;
      for (;;) {
        __syncthreads();
        const int n = S.cnt[ci];
        const int status = S.status;
        // every wave holds the step's control words before any wave can write
        // the status again (an error found in the step), so all decide alike
        __syncthreads();
        if (n == 0 || status < 0 || steps >= stop || (NARROW && n > hi)) break;
        if (!LANE && n <= solo_max) {
          if (tid < 64) {
            if (!NARROW || hi >= SOLO_MAX) solo(SOLO_MAX);
            else solo(hi);
          }
          __syncthreads();
          steps = S.steps;
          cur = S.cur;
          continue;
        }
        const int cn = ci == 2 ? 0 : ci + 1;
        const int cnn = cn == 2 ? 0 : cn + 1;
        if (tid == 0) {
          S.cnt[cnn] = 0;
          if (n > S.maxf) S.maxf = n;
          if constexpr (NARROW)
            if ((steps & 1023u) == 0) gstore(hb, (int)steps);
          if constexpr (TRACE)
            if (D.trace && steps < (unsigned)D.trace_cap) D.trace[steps] = n;
        }
        const Pair *cq_l = S.q[cur];
        const gint2 *cq_g = cur ? queue1 : queue0;
        Pair *nq_l = S.q[cur ^ 1];
        gint2 *nq_g = cur ? queue0 : queue1;
        C.next = &S.cnt[cn];
        for (int base = 0; base < n; base += WG) {
          bool valid;
          int a, b, la, lb, pa0, pa1, pb0, pb1;
          fetch_pair<WG, QCAP>(base, n, tid, cq_l, cq_g, agent, valid, a, b, la, lb, pa0, pa1,
                               pb0, pb1);
          int nha, nhb;
          pass_static<QCAP, MAXL, CM_LDS, LANE>(valid, a, b, la, lb, pa0, pa1, pb0, pb1, D, agent,
                                                bind, stuck, rule_of, nq_l, nq_g, C,
                                                loops_lane, rc_lane, nha, nhb);
        }
        steps++;
        cur ^= 1;
        ci = cn;
      }
      if (rc_lane) atomicAdd(&S.rc[__lane_id()], (unsigned long long)rc_lane);
      if (loops_lane) atomicAdd(&S.loops, loops_lane);
      __syncthreads();
    }
  } else
#endif
  for (;;) {
    __syncthreads();
    const int n = S.cnt[ci];
    const int status = S.status;
    __syncthreads();  // as above: all waves read before any can write the status
    if (n == 0 || status < 0 || steps >= stop || (NARROW && n > hi)) break;
    const int cn = ci == 2 ? 0 : ci + 1;
    const int cnn = cn == 2 ? 0 : cn + 1;
    if (tid == 0) {
      S.cnt[cnn] = 0;
      if (n > S.maxf) S.maxf = n;
      if constexpr (TRACE)
        if (D.trace && steps < (unsigned)D.trace_cap) D.trace[steps] = n;
    }
    const Pair *cq_l = S.q[cur];
    const gint2 *cq_g = cur ? queue1 : queue0;
    Pair *nq_l = S.q[cur ^ 1];
    gint2 *nq_g = cur ? queue0 : queue1;
    for (int base = 0; base < n; base += WG) {
      const int i = base + tid;
      const bool valid = i < n;
      // lanes without a pair read slot 0 (always allocated) and stay idle:
      // the loads need no branch
      Pair rx = mkpair(0, 0);
      if (base + WG <= QCAP) {
        rx = cq_l[valid ? i : 0];
      } else if (valid) {
        if (i < QCAP) rx = cq_l[i];
        else rx = unpk(*at2((gint2 *)cq_g, (unsigned)i));
      }
      if (!valid) rx = mkpair(0, 0);
      const int a = rx.x, b = rx.y;
      const unsigned ua = (unsigned)a, ub = (unsigned)b;
      const v4i ra = *rec(agent, ua), rb = *rec(agent, ub);
      const int la = ra.x, lb = rb.x;
      const int pa0 = ra.y, pa1 = ra.z;
      const int pb0 = rb.y, pb1 = rb.z;
      if constexpr (ENGINE == 1)
        pass_interp<QCAP>(valid, a, b, la, lb, pa0, pa1, pb0, pb1, D, agent, bind,
                          stuck, rule_of, RV.templ, RV.arity, RV.g_templ, RV.g_arity, RV.ns, nq_l, nq_g,
                          &S.cnt[cn], &S.status, &S.agent_top, &S.name_top, &S.nstuck, &S.loops,
                          S.rc);
      else
        pass_uniform<QCAP, MAXL>(valid, a, b, la, lb, pa0, pa1, pb0, pb1, D, agent, bind,
                                 stuck, rule_of, RV.templ, RV.arity, RV.g_templ, RV.g_arity, RV.ns,
                                 nq_l, nq_g, &S.cnt[cn], &S.status, &S.agent_top, &S.name_top,
                                 &S.nstuck, &S.loops, S.rc);
    }
    steps++;
    cur ^= 1;
    ci = cn;
  }

  // the loop ends right after a barrier with uniform values
  const int n_left = S.cnt[ci];
  const int status = S.status;
  if (status >= 0 && n_left > 0) {
    gint2 *g = cur ? queue1 : queue0;
    const int nl = n_left < QCAP ? n_left : QCAP;
    for (int i = tid; i < nl; i += WG) g[i] = pk(S.q[cur][i].x, S.q[cur][i].y);
  }
  gu64 *per_rule = (gu64 *)D.per_rule;
  for (int r = tid; r < nr; r += WG)
    if (S.rc[r]) per_rule[r] += S.rc[r];
  const bool done = status >= 0 && n_left == 0;
  if (tid == 0) {
    unsigned long long tot = 0;
    for (int r = 0; r < nr; r++) tot += S.rc[r];
    st->interactions += tot;
    st->steps = steps;
    st->agent_top = S.agent_top;
    st->name_top = S.name_top;
    st->n_stuck = S.nstuck;
    st->loops += S.loops;
    st->max_frontier = S.maxf;
    if (status < 0) {
      st->status = status;
    } else if (!done) {
      // stopped by the step budget (resumable), or handed over while wide
      st->phase = PHASE_RUN;
      st->parity = cur;
      st->frontier = n_left;
      st->status = steps >= stop ? ST_ELIMIT : ST_OK;
    } else {
      st->phase = PHASE_DONE;
      st->frontier = 0;
      st->status = S.nstuck ? ST_STUCK : ST_OK;
    }
  }
  if ((flags & FLAG_JUMP) && done) {
    __syncthreads();
    jump_net<WG>(bind, S.name_top, &S.bcast[0]);
  }
}

template <int WG, int QCAP>
__device__ __forceinline__ RuleView load_rules(const int *__restrict__ g_rules, int ns, int nr,
                                               int *s_rules) {
  const int nwords = ns * ns + nr * RT_WORDS + ns;
  for (int i = threadIdx.x; i < nwords; i += WG) s_rules[i] = g_rules[i];
  RuleView RV;
  RV.rule_of = s_rules;
  RV.templ = s_rules + ns * ns;
  RV.arity = RV.templ + nr * RT_WORDS;
  RV.g_templ = g_rules + ns * ns;
  RV.g_arity = RV.g_templ + nr * RT_WORDS;
  RV.ns = ns;
  RV.nr = nr;
  return RV;
}

// the persistent batch kernel: each workgroup takes nets from a device
// counter in the given order and runs each to normal form (or the budget)
template <int WG, int QCAP, int ENGINE, int MAXL, bool TRACE = false, int SOLO_MAX = 64>
__device__ __forceinline__ void reduce_body(const NetDesc *__restrict__ descs,
                                            const int *__restrict__ order, int n_nets,
                                            int *counter, const int *__restrict__ g_rules,
                                            int ns, int nr, unsigned max_steps, int flags,
                                            const KParams &kp) {
  extern __shared__ int s_rules[];
  __shared__ EngineLds<QCAP> S;
  const RuleView RV = load_rules<WG, QCAP>(g_rules, ns, nr, s_rules);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) S.net = atomicAdd(counter, 1);
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(S.net);
    if (k >= n_nets) break;
    const NetDesc D = descs[order[k]];
    const unsigned steps0 = D.st->steps;
    // per-launch step budget (saturating)
    const unsigned stop = (max_steps > 0xffffffffu - steps0) ? 0xffffffffu : steps0 + max_steps;
    engine_net<WG, QCAP, ENGINE, MAXL, false, TRACE, SOLO_MAX>(S, D, RV, stop, flags, 0x7fffffff,
                                                              kp, nullptr);
  }
}

#ifdef INET_STATIC_RULES
// ---------------------------------------------------------------------------
// Multi-workgroup engine for one net (the launch's only net).  Workgroup 0
// steps the net alone (engine_net, one compute unit) while at most grid_hi
// pairs are active; once more are, the net's parallel steps are shared by the
// g workgroups of lowest logical index, g = ceil(active / grid_ppw) up to the
// whole launch, until at most grid_lo pairs are left.  In such a step each
// participating workgroup takes a contiguous share of the frontier (global
// queue), runs the same pass as the one-workgroup engine with the heap tops
// and status as agent-scope atomics in the net's state, stages its new active
// pairs in its LDS tile and appends them to the next frontier with one
// agent-scope atomic.  Epochs (a run of workgroup 0 alone, or one shared
// step) end when every workgroup of the launch has posted its entry: an
// agent-scope release before posting, acquire after all entries are seen, so
// that agent records, name cells and queue entries written in an epoch are
// seen by every workgroup in the next (the name-cell exchanges themselves are
// agent-scope atomics).  Every workgroup takes the next epoch's decision from
// the same inputs (the entries, and the state workgroup 0 left after a run
// alone), so all take the same one.  Every wait gives up after kp.timeout
// wall-clock ticks without progress (all entries posted, or workgroup 0's
// step count moving), setting ST_ETIMEDOUT, so the kernel always ends.

// logical index of block b of G: blocks are handed to the XCDs in turn
// (block b runs on XCD b % 8), so logical indices run through one XCD's
// blocks before the next one's; a small group of participants then shares
// one L2
__device__ __forceinline__ int logical_wg(int b, int G) {
  const int x = b & 7;
  int before = 0;
  for (int k = 0; k < x; k++) before += (G - k + 7) >> 3;  // blocks on XCD k
  return before + (b >> 3);
}

template <int WG, int QCAP, int MAXL, bool TRACE = false, int SOLO_MAX = 64>
__device__ __forceinline__ void grid_body(const NetDesc *__restrict__ descs,
                                          const int *__restrict__ g_rules, int ns, int nr,
                                          unsigned max_steps, int flags, const KParams &kp) {
  extern __shared__ int s_rules[];
  __shared__ EngineLds<QCAP> S;
  __shared__ unsigned long long s_base;
  const RuleView RV = load_rules<WG, QCAP>(g_rules, ns, nr, s_rules);
  const NetDesc D = descs[0];
  NetState *st = D.st;
  GridCtl *ctl = kp.ctl;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int me = logical_wg(blockIdx.x, G);
  gint *const agent = (gint *)D.agent;
  gint *const bind = (gint *)D.bind;
  gint2 *const stuck = (gint2 *)D.stuck;
  const int lo = kp.grid_lo, hi = kp.grid_hi > kp.grid_lo ? kp.grid_hi : kp.grid_lo;
  const int ppw = kp.grid_ppw > 0 ? kp.grid_ppw : WG;
  unsigned rc_lane = 0;
  int loops_lane = 0;
  // epoch 1: workgroup 0 steps the net alone (linking the initial equations
  // on the first launch) until it widens or ends
  unsigned stop = 0;  // absolute step budget (workgroup 0: every thread; others: thread 0)
  if (me == 0) {
    const unsigned steps0 = st->steps;
    stop = (max_steps > 0xffffffffu - steps0) ? 0xffffffffu : steps0 + max_steps;
    if (tid == 0) ctl->stop = stop;
    engine_net<WG, QCAP, 3, MAXL, true, TRACE, SOLO_MAX>(S, D, RV, stop, 0, hi, kp,
                                                         &ctl->heartbeat);
  }
  int epoch = 1, mode = GM_NARROW;
  int count = 0;  // new active pairs of this workgroup in a GRID epoch (its entry)
  // thread 0's view of the net, the same in every workgroup: active pairs of
  // the coming GRID step, their queue, steps done before it, ctl->next before it
  int n = 0, cur = 0;
  unsigned steps = 0;
  unsigned long long base = 0;
  int maxf = 0;  // widest frontier (workgroup 0, thread 0)
  for (;;) {
    // ---- post this workgroup's entry for the epoch, then read everyone's.
    // Every wave waits until its own stores of the epoch (records, cells,
    // queue entries, the net's state) have reached the L2 before the
    // workgroup barrier, which waits for LDS traffic only; thread 0's
    // agent-scope release then writes them all back before the entry.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __builtin_amdgcn_s_waitcnt(0);
      const bool err = mode == GM_GRID && S.status != 0;
      __hip_atomic_store(&ctl->ent[epoch & 1][me], ent_pack(epoch, err, count),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid < 64) {
      int sum = 0;
      bool err = false;
      const bool ok = wait_entries(ctl, G, epoch, kp.timeout, sum, err);
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);  // the invalidation done before any wave loads
        int next_mode = GM_DONE, g = 1;
        if (!ok) {
          gstore(&ctl->gave_up, 1);
          gstore(&st->status, ST_ETIMEDOUT);
          next_mode = -1;
        } else if (mode == GM_NARROW) {
          // workgroup 0 left the net's state as the one-workgroup engine does
          n = st->phase == PHASE_DONE ? 0 : st->frontier;
          cur = st->parity;
          steps = st->steps;
          stop = ctl->stop;
          if (me == 0) maxf = st->max_frontier;
          int status = gload(&st->status);
          // a give-up by a workgroup that waited for this run ends the launch
          // with it (workgroup 0's own bookkeeping may have written over the
          // status); a give-up in a shared step stalls the next one, whose
          // waits then give up too
          if (gload(&ctl->gave_up)) {
            status = ST_ETIMEDOUT;
            if (me == 0) gstore(&st->status, ST_ETIMEDOUT);
          }
          if (!(n == 0 || status < 0 || steps >= stop)) next_mode = n <= lo ? GM_NARROW : GM_GRID;
        } else {
          // a shared step ended: `sum` new active pairs in the other queue
          const int done_n = n;
          base += (unsigned long long)sum;
          n = sum;
          cur ^= 1;
          if (me == 0) {
            if (done_n > maxf) maxf = done_n;
            if constexpr (TRACE)
              if (D.trace && steps < (unsigned)D.trace_cap) D.trace[steps] = done_n;
          }
          steps++;
          if (n == 0 || err || steps >= stop) {
            if (me == 0) {
              // the net's state as the one-workgroup engine leaves it (an
              // error status is already there)
              st->max_frontier = maxf;
              st->steps = steps;
              if (!err) {
                if (n == 0) {
                  st->phase = PHASE_DONE;
                  st->frontier = 0;
                  gstore(&st->status, gload(&st->n_stuck) ? ST_STUCK : ST_OK);
                } else {
                  st->phase = PHASE_RUN;
                  st->parity = cur;
                  st->frontier = n;
                  gstore(&st->status, ST_ELIMIT);
                }
              }
            }
          } else if (n <= lo) {
            next_mode = GM_NARROW;
            if (me == 0) {
              st->max_frontier = maxf;
              st->phase = PHASE_RUN;
              st->parity = cur;
              st->frontier = n;
              st->steps = steps;
            }
          } else {
            next_mode = GM_GRID;
          }
        }
        if (next_mode == GM_GRID) {
          g = (n + ppw - 1) / ppw;
          if (g > G) g = G;
          if (g < 1) g = 1;
        }
        S.bcast[0] = next_mode;
        S.bcast[1] = n;
        S.bcast[2] = cur;
        S.bcast[3] = g;
        s_base = base;
      }
    }
    __syncthreads();
    mode = S.bcast[0];
    if (mode < 0 || mode == GM_DONE) break;
    epoch++;
    count = 0;
    if (mode == GM_NARROW) {
      if (me == 0)
        engine_net<WG, QCAP, 3, MAXL, true, TRACE, SOLO_MAX>(S, D, RV, stop, 0, hi, kp,
                                                             &ctl->heartbeat);
      continue;
    }
    // ---- one parallel step shared by the first g workgroups
    const int sn = S.bcast[1], scur = S.bcast[2], g = S.bcast[3];
    const unsigned long long sbase = s_base;
    if (tid == 0) {
      S.cnt[0] = 0;
      S.status = 0;
      S.wneed[0] = 0;
      S.wneed[1] = 0;
    }
    if (me >= g) continue;
    const int per = (sn + g - 1) / g;
    const int i0 = me * per;
    const int i1 = i0 + per < sn ? i0 + per : sn;
    const gint2 *cq_g = (const gint2 *)(scur ? D.queue1 : D.queue0);
    gint2 *nq_g = (gint2 *)(scur ? D.queue0 : D.queue1);
    __syncthreads();
    Ctr<CM_GRID> C;
    C.agent_top = &st->agent_top;
    C.name_top = &st->name_top;
    C.nstuck = &st->n_stuck;
    C.status = &st->status;
    C.next = &S.cnt[0];
    C.lerr = &S.status;
    C.spill_next = &ctl->next;
    C.base = sbase;
    C.wneed = S.wneed;
    C.wbase = S.wbase;
    for (int base_i = i0; base_i < i1; base_i += WG) {
      const int i = base_i + tid;
      const bool valid = i < i1;
      // one reservation per workgroup when many workgroups contend for the
      // heap tops and at least half the lanes have a pair
      C.collective = g >= 16 && 2 * (i1 - base_i) >= WG;
      const Pair rx = valid ? unpk(*at2((gint2 *)cq_g, (unsigned)i)) : mkpair(0, 0);
      const v4i ra = *rec(agent, (unsigned)rx.x), rb = *rec(agent, (unsigned)rx.y);
      int nha, nhb;
      pass_static<QCAP, MAXL, CM_GRID, false>(valid, rx.x, rx.y, ra.x, rb.x, ra.y, ra.z, rb.y,
                                              rb.z, D, agent, bind, stuck, RV.rule_of, S.q[0],
                                              nq_g, C, loops_lane, rc_lane, nha, nhb);
    }
    // the workgroup's new active pairs from its LDS tile to the next frontier
    __syncthreads();
    const int total = S.cnt[0];
    const int tile = total < QCAP ? total : QCAP;
    if (tid == 0)
      S.bcast[5] = tile ? (int)(__hip_atomic_fetch_add(&ctl->next, (unsigned long long)tile,
                                                       __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) -
                                sbase)
                        : 0;
    __syncthreads();
    const int gb = S.bcast[5];
    bool over = false;
    for (int k = tid; k < tile; k += WG) {
      if (gb + k < D.qcap) *at2(nq_g, (unsigned)(gb + k)) = pk(S.q[0][k].x, S.q[0][k].y);
      else over = true;
    }
    if (over) {
      gstore(&st->status, ST_ENOMEM);
      S.status = ST_ENOMEM;
    }
    count = total;
  }
  // this workgroup's interactions per rule and dropped loops of its shared steps
  gu64 *per_rule = (gu64 *)D.per_rule;
  const int lane = __lane_id();
  if (rc_lane && lane < nr) {
    __hip_atomic_fetch_add((unsigned long long *)&per_rule[lane], (unsigned long long)rc_lane,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&st->interactions, (unsigned long long)rc_lane, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
  if (loops_lane) gadd(&st->loops, loops_lane);
}
#endif  // INET_STATIC_RULES


#ifndef __HIPCC_RTC__
template <int WG, int QCAP, int ENGINE, int MAXL>
__global__ __launch_bounds__(WG) void k_reduce(const NetDesc *__restrict__ descs,
                                               const int *__restrict__ order, int n_nets,
                                               int *counter, const int *__restrict__ g_rules,
                                               int ns, int nr, unsigned max_steps, int flags,
                                               KParams kp) {
  // the ahead-of-time engines always carry the trace (they are not the fast path)
  reduce_body<WG, QCAP, ENGINE, MAXL, true>(descs, order, n_nets, counter, g_rules, ns, nr,
                                            max_steps, flags, kp);
}

// pointer jumping over one net's cells with the whole grid (single big nets):
// rounds over all cells separated by a barrier over the launch, until a round
// moves nothing (at most 32 rounds); a barrier wait that gives up ends the
// pass early (the cells then hold partly compressed chains, which read back
// the same)
__global__ __launch_bounds__(256) void k_jump_grid(const NetDesc *__restrict__ desc, GridCtl *ctl,
                                                   unsigned long long timeout) {
  __shared__ int s_again;
  const NetDesc D = desc[0];
  // the same decision in every block: nothing writes the state meanwhile
  if (D.st->phase != PHASE_DONE || D.st->status < 0) return;
  const int nn = D.st->name_top;
  const int G = gridDim.x;
  gint *const bind = (gint *)D.bind;
  int seen = 0;
  for (int round = 0; round < 32; round++) {
    bool moved = false;
    for (int x = blockIdx.x * 256 + threadIdx.x; x < nn; x += G * 256) moved |= jump_hop(bind, x);
    if (__syncthreads_or(moved) && threadIdx.x == 0) gstore(&ctl->moved[round & 1], 1);
    const bool ok = grid_sync(ctl, G, seen, timeout,
                              [&] { gstore(&ctl->moved[(round + 1) & 1], 0); });
    if (threadIdx.x == 0) s_again = ok ? gload(&ctl->moved[round & 1]) : 0;
    __syncthreads();
    if (!s_again) break;
  }
}

// restore one net to its loaded state with the lanes tid, tid + stride, ...
__device__ __forceinline__ void reset_net(const NetDesc &D, int nr, int tid, int stride) {
  for (int i = tid; i < D.n_agents0; i += stride)
    *rec((gint *)D.agent, (unsigned)i) = mkrec(D.init_label[i], D.init_port[2 * i], D.init_port[2 * i + 1]);
  gint2 *q0 = (gint2 *)D.queue0;
  for (int i = tid; i < D.n_eqs0; i += stride) q0[i] = pk(D.init_eq[2 * i], D.init_eq[2 * i + 1]);
  for (int i = tid; i < D.n_names0; i += stride) D.bind[i] = EMPTY;
  for (int i = tid; i < nr; i += stride) D.per_rule[i] = 0ull;
  if (tid == 0) {
    NetState s = {};
    s.agent_top = D.n_agents0;
    s.name_top = D.n_names0;
    s.frontier = D.n_eqs0;
    s.phase = PHASE_INIT;
    *D.st = s;
  }
}

// restore nets to their loaded state: all n nets, or the n listed in idx
__global__ __launch_bounds__(256) void k_reset(const NetDesc *__restrict__ descs,
                                               const int *__restrict__ idx, int n, int nr) {
  for (int k = blockIdx.x; k < n; k += gridDim.x) reset_net(descs[idx ? idx[k] : k], nr, threadIdx.x, 256);
}

// install admitted nets: each record's descriptor goes to its slot and the net
// is reset from its (already resident) initial image
__global__ __launch_bounds__(256) void k_admit(const AdmitRec *__restrict__ recs, int n,
                                               NetDesc *__restrict__ descs, int nr) {
  __shared__ NetDesc sd;
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    __syncthreads();
    if (threadIdx.x == 0) {
      sd = recs[k].desc;
      descs[recs[k].slot] = recs[k].desc;
    }
    __syncthreads();
    reset_net(sd, nr, threadIdx.x, 256);
  }
}

__global__ void k_zero(int *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

#endif  // __HIPCC_RTC__

}  // namespace inet

#endif
