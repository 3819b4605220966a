// readback.cpp -- sub* col* read-back and the canonical normal-form stream.
//
// After the reduction no active pair with a rule is left (the correctness
// proposition of Section 3.6).  What remains in the heap is the result of int
// and com only; Theorem 1 of Section 2.2 says the remaining sub and col steps
// can be applied at the end.  Here they are applied on the host while the
// terms are written out: a name met at a port or in the interface whose cell
// holds a parked value is replaced by that value (sub inside a term, col at
// the interface); a name with an empty cell is a free or bound name of the
// result and is written as a name.
#include <algorithm>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "inet_internal.h"
#include "runtime.h"

namespace inet {

namespace {

struct Heap {
  const int32_t *label, *p0, *p1, *bind;
  int64_t n_agents, n_cells;
  const int32_t *arity;
  int32_t n_symbols;
};

// Writes T(ref).  canon == nullptr: names are written as -1 (erased form).
// Returns false if the walk exceeds the heap (a cycle through the cells) or
// meets a reference or label out of range.
bool emit(const Heap &H, int32_t ref, std::vector<int32_t> *canon, int32_t *next,
          std::vector<int32_t> &out, std::vector<int32_t> &stk, int64_t budget) {
  stk.clear();
  stk.push_back(ref);
  int64_t words = 0;
  while (!stk.empty()) {
    int32_t r = stk.back();
    stk.pop_back();
    int64_t hops = 0;
    while (r < 0) {
      const int32_t x = ~r;
      if (x >= H.n_cells) return false;
      const int32_t v = H.bind[x];
      if (v == EMPTY) break;
      r = v;
      if (++hops > H.n_cells) return false;
    }
    if (++words > budget) return false;
    if (r < 0) {
      if (!canon) { out.push_back(-1); continue; }
      const int32_t x = ~r;
      int32_t &c = (*canon)[x];
      if (c < 0) c = (*next)++;
      out.push_back(-1 - c);
      continue;
    }
    if (r >= H.n_agents) return false;
    const int32_t L = H.label[r];
    if (L < 0 || L >= H.n_symbols) return false;
    out.push_back(L);
    const int ar = H.arity[L];
    if (ar > 1) stk.push_back(H.p1[r]);
    if (ar > 0) stk.push_back(H.p0[r]);
  }
  return true;
}

bool seq_less_eq(const int32_t *a, size_t na, const int32_t *b, size_t nb) {
  const size_t n = std::min(na, nb);
  for (size_t i = 0; i < n; i++)
    if (a[i] != b[i]) return a[i] < b[i];
  return na <= nb;
}

}  // namespace

int canonical_stream(const CompiledRules &R, const int32_t *label, const int32_t *p0,
                     const int32_t *p1, int64_t n_agents, const int32_t *bind, int64_t n_cells,
                     const std::vector<int32_t> &iface, const std::vector<int2> &stuck,
                     std::vector<int32_t> *out) {
  Heap H{label, p0, p1, bind, n_agents, n_cells, R.arity.data(), R.ns};
  const int64_t budget = 2 * (n_agents + n_cells) + 16;
  std::vector<int32_t> canon((size_t)std::max<int64_t>(n_cells, 1), -1);
  std::vector<int32_t> stk;
  int32_t next = 0;
  out->clear();
  out->push_back((int32_t)iface.size());
  for (int32_t x : iface)
    if (!emit(H, -1 - x, &canon, &next, *out, stk, budget)) return INET_EINVAL;
  // residual active pairs: orient and sort by the name-erased encodings
  struct Res {
    int32_t l, r;
    std::vector<int32_t> kl, kr;
  };
  std::vector<Res> res;
  res.reserve(stuck.size());
  for (const int2 &p : stuck) {
    Res e;
    std::vector<int32_t> ka, kb;
    if (!emit(H, p.x, nullptr, nullptr, ka, stk, budget)) return INET_EINVAL;
    if (!emit(H, p.y, nullptr, nullptr, kb, stk, budget)) return INET_EINVAL;
    if (seq_less_eq(ka.data(), ka.size(), kb.data(), kb.size())) {
      e.l = p.x; e.r = p.y; e.kl.swap(ka); e.kr.swap(kb);
    } else {
      e.l = p.y; e.r = p.x; e.kl.swap(kb); e.kr.swap(ka);
    }
    res.push_back(std::move(e));
  }
  std::stable_sort(res.begin(), res.end(), [](const Res &a, const Res &b) {
    if (a.kl != b.kl) return std::lexicographical_compare(a.kl.begin(), a.kl.end(), b.kl.begin(), b.kl.end());
    return std::lexicographical_compare(a.kr.begin(), a.kr.end(), b.kr.begin(), b.kr.end());
  });
  out->push_back((int32_t)res.size());
  for (const Res &e : res) {
    if (!emit(H, e.l, &canon, &next, *out, stk, budget)) return INET_EINVAL;
    if (!emit(H, e.r, &canon, &next, *out, stk, budget)) return INET_EINVAL;
  }
  return INET_OK;
}

int readback_net(const CompiledRules &R, const NetDesc &D, const NetState &s,
                 const std::vector<int32_t> &iface, std::vector<int32_t> *out) {
  const int64_t na = s.agent_top, nc = s.name_top;
  std::vector<int32_t> rec(4 * (size_t)na), label(na), p0(na), p1(na), bind(nc);
  std::vector<int2> stuck(s.n_stuck);
  if (na) {
    HIPCHK(hipMemcpy(rec.data(), D.agent, 16 * (size_t)na, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < na; i++) {
      label[i] = rec[4 * i];
      p0[i] = rec[4 * i + 1];
      p1[i] = rec[4 * i + 2];
    }
  }
  if (nc) HIPCHK(hipMemcpy(bind.data(), D.bind, 4 * nc, hipMemcpyDeviceToHost));
  if (s.n_stuck)
    HIPCHK(hipMemcpy(stuck.data(), D.stuck, 8 * (size_t)s.n_stuck, hipMemcpyDeviceToHost));
  return canonical_stream(R, label.data(), p0.data(), p1.data(), na, bind.data(), nc, iface, stuck,
                          out);
}

}  // namespace inet
