// rules.cpp -- rule-table compiler.
//
// A rule alpha(x) = beta(y) -> Theta (Section 2.2) is turned into a template
// the kernels instantiate without interpretation of terms:
//   * the com and sub steps that involve only bound names of Theta are applied
//     once, here, to Theta itself (they commute with everything else, and by
//     Theorem 1 of Section 2.2 sub never creates an active pair); what is left
//     is a set of agents whose ports hold rule arguments, other new agents or
//     wires, plus the equations that still touch a rule argument (or join two
//     new agents into an active pair);
//   * the new agents are numbered in preorder; the first two reuse the slots
//     of the interacting pair, the others come from the bump allocator;
//   * bound names left after folding are wires between two ports of new
//     agents (or a name cycle): they get fresh name cells.
// The interaction count and the normal form are those of the literal rule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"
#include "runtime.h"

namespace inet {
namespace {

struct TNode {
  int kind;  // 0 agent, 1 name, -1 dead
  int sym;   // label or rule-local name id
  int ch[2];
};

struct Theta {
  std::vector<TNode> nodes;
  std::vector<std::pair<int, int>> eqs;
  std::vector<char> eq_alive;
  const int32_t *arity;
  int ns;

  int parse(const int32_t *w, int64_t n, int64_t *pos, int depth, bool *ok) {
    if (*pos >= n || depth > 32) { *ok = false; return -1; }
    int32_t v = w[(*pos)++];
    TNode t;
    t.ch[0] = t.ch[1] = -1;
    if (v >= 0) {
      if (v >= ns) { *ok = false; return -1; }
      t.kind = 0;
      t.sym = v;
      int id = (int)nodes.size();
      nodes.push_back(t);
      for (int j = 0; j < arity[v]; j++) {
        int c = parse(w, n, pos, depth + 1, ok);
        if (!*ok) return -1;
        nodes[id].ch[j] = c;
      }
      return id;
    }
    t.kind = 1;
    t.sym = -1 - v;
    nodes.push_back(t);
    return (int)nodes.size() - 1;
  }

  // location of a node: equation side (e, s) or child slot (p, j)
  struct Loc { int eq, side, parent, slot; };

  bool find_loc(int node, Loc *L) const {
    for (size_t e = 0; e < eqs.size(); e++) {
      if (!eq_alive[e]) continue;
      if (eqs[e].first == node) { *L = {(int)e, 0, -1, -1}; return true; }
      if (eqs[e].second == node) { *L = {(int)e, 1, -1, -1}; return true; }
    }
    for (size_t p = 0; p < nodes.size(); p++) {
      if (nodes[p].kind != 0) continue;
      for (int j = 0; j < arity[nodes[p].sym]; j++)
        if (nodes[p].ch[j] == node) { *L = {-1, -1, (int)p, j}; return true; }
    }
    return false;
  }

  bool contains(int root, int node) const {
    if (root == node) return true;
    if (nodes[root].kind != 0) return false;
    for (int j = 0; j < arity[nodes[root].sym]; j++)
      if (contains(nodes[root].ch[j], node)) return true;
    return false;
  }

  void put(const Loc &L, int node) {
    if (L.eq >= 0) {
      if (L.side == 0) eqs[L.eq].first = node; else eqs[L.eq].second = node;
    } else {
      nodes[L.parent].ch[L.slot] = node;
    }
  }

  // apply com/sub to bound names (local id >= nargs) until none applies
  void fold(int nargs) {
    bool changed = true;
    while (changed) {
      changed = false;
      for (size_t e = 0; e < eqs.size() && !changed; e++) {
        if (!eq_alive[e]) continue;
        for (int side = 0; side < 2 && !changed; side++) {
          int n = side == 0 ? eqs[e].first : eqs[e].second;
          int t = side == 0 ? eqs[e].second : eqs[e].first;
          if (nodes[n].kind != 1 || nodes[n].sym < nargs) continue;
          int other = -1;
          for (size_t k = 0; k < nodes.size(); k++)
            if ((int)k != n && nodes[k].kind == 1 && nodes[k].sym == nodes[n].sym) {
              Loc L;
              if (find_loc((int)k, &L)) { other = (int)k; break; }
            }
          if (other < 0) continue;
          if (other == t) {  // x = x inside Theta: a closed loop, dropped
            eq_alive[e] = 0;
            nodes[n].kind = nodes[t].kind = -1;
            changed = true;
            break;
          }
          if (contains(t, other)) continue;  // x = C[x]: a cycle, kept
          Loc L;
          find_loc(other, &L);
          eq_alive[e] = 0;
          put(L, t);
          nodes[n].kind = nodes[other].kind = -1;
          changed = true;
        }
      }
    }
  }
};

}  // namespace

int compile_rules(const inet_rules *r, CompiledRules *out) {
  if (!r || r->n_symbols <= 0 || r->n_symbols > INET_MAX_SYMBOLS || r->n_rules < 0 ||
      r->n_rules > INET_MAX_RULES || !r->arity)
    return INET_EINVAL;
  if (r->n_rules > 0 && (!r->rule_lhs || !r->rhs_off || !r->rhs)) return INET_EINVAL;
  const int ns = r->n_symbols, nr = r->n_rules;
  out->ns = ns;
  out->nr = nr;
  out->arity.assign(r->arity, r->arity + ns);
  for (int i = 0; i < ns; i++)
    if (out->arity[i] < 0 || out->arity[i] > INET_MAX_ARITY) return INET_EINVAL;
  out->rule_of.assign((size_t)ns * ns, -1);
  out->templ.assign((size_t)nr * RT_WORDS, OP_NONE);
  out->bytes.assign(nr, 0);
  out->rhs_agents.assign(nr, 0);
  out->max_links = 0;
  for (int k = 0; k < nr; k++) {
    int32_t a = r->rule_lhs[2 * k], b = r->rule_lhs[2 * k + 1];
    if (a < 0 || b < 0 || a >= ns || b >= ns || a == b) return INET_EINVAL;
    if (out->rule_of[a * ns + b] != -1) return INET_EINVAL;
    out->rule_of[a * ns + b] = 2 * k;
    out->rule_of[b * ns + a] = 2 * k + 1;
    int64_t lo = r->rhs_off[k], hi = r->rhs_off[k + 1];
    if (lo < 0 || hi <= lo || hi - lo > 4096) return INET_EINVAL;
    const int32_t *w = r->rhs + lo;
    int64_t n = hi - lo, pos = 1;
    int neq = w[0];
    if (neq < 0 || neq > 64) return INET_EINVAL;
    Theta T;
    T.arity = r->arity;
    T.ns = ns;
    bool ok = true;
    for (int e = 0; e < neq; e++) {
      int l = T.parse(w, n, &pos, 0, &ok);
      int rr = ok ? T.parse(w, n, &pos, 0, &ok) : -1;
      if (!ok) return INET_EINVAL;
      T.eqs.push_back({l, rr});
      T.eq_alive.push_back(1);
    }
    if (pos != n) return INET_EINVAL;
    const int ara = out->arity[a], arb = out->arity[b], nargs = ara + arb;
    // occurrence counts: arguments once, bound names twice
    std::vector<int> cnt(4096, 0);
    int n_agents_raw = 0;
    for (auto &t : T.nodes) {
      if (t.kind == 1) {
        if (t.sym >= 4096) return INET_EINVAL;
        cnt[t.sym]++;
      } else {
        n_agents_raw++;
      }
    }
    for (int v = 0; v < 4096; v++) {
      if (v < nargs) { if (cnt[v] != 1) return INET_EINVAL; }
      else if (cnt[v] != 0 && cnt[v] != 2) return INET_EINVAL;
    }
    out->rhs_agents[k] = n_agents_raw;
    T.fold(nargs);
    // number the surviving agents in preorder of the surviving equations
    std::vector<int> agent_idx(T.nodes.size(), -1), agents;
    std::vector<int> stack;
    for (size_t e = 0; e < T.eqs.size(); e++) {
      if (!T.eq_alive[e]) continue;
      for (int side = 0; side < 2; side++) {
        stack.push_back(side == 0 ? T.eqs[e].first : T.eqs[e].second);
        while (!stack.empty()) {
          int x = stack.back();
          stack.pop_back();
          if (T.nodes[x].kind != 0 || agent_idx[x] >= 0) continue;
          agent_idx[x] = (int)agents.size();
          agents.push_back(x);
          for (int j = T.arity[T.nodes[x].sym] - 1; j >= 0; j--) stack.push_back(T.nodes[x].ch[j]);
        }
      }
    }
    std::vector<int> fresh_idx(4096, -1);
    int n_fresh = 0;
    auto operand = [&](int x) -> int {
      const TNode &t = T.nodes[x];
      if (t.kind == 0) return (OP_NEW << 4) | agent_idx[x];
      if (t.sym < ara) return (OP_AUX << 4) | t.sym;
      if (t.sym < nargs) return (OP_AUX << 4) | (2 + t.sym - ara);
      if (fresh_idx[t.sym] < 0) fresh_idx[t.sym] = n_fresh++;
      return (OP_FRESH << 4) | fresh_idx[t.sym];
    };
    int32_t *R = &out->templ[(size_t)k * RT_WORDS];
    const int n_new = (int)agents.size();
    if (n_new > MAXNEW) return INET_EINVAL;
    int bytes = 8 + 4 * (2 + ara + arb);
    for (int i = 0; i < n_new; i++) {
      const TNode &t = T.nodes[agents[i]];
      R[RT_LABEL + i] = t.sym;
      for (int j = 0; j < T.arity[t.sym]; j++) R[RT_PORT + 2 * i + j] = operand(t.ch[j]);
      bytes += 4 * (1 + T.arity[t.sym]);
    }
    int n_links = 0;
    for (size_t e = 0; e < T.eqs.size(); e++) {
      if (!T.eq_alive[e]) continue;
      if (n_links >= MAXEQ) return INET_EINVAL;
      R[RT_EQ + 2 * n_links] = operand(T.eqs[e].first);
      R[RT_EQ + 2 * n_links + 1] = operand(T.eqs[e].second);
      n_links++;
    }
    if (n_fresh > MAXFRESH) return INET_EINVAL;
    R[RT_NNEW] = n_new;
    R[RT_NALLOC] = n_new > 2 ? n_new - 2 : 0;
    R[RT_NFRESH] = n_fresh;
    R[RT_NEQ] = n_links;
    out->max_links = std::max(out->max_links, n_links);
    bytes += 4 * n_fresh + 8 * n_links;
    out->bytes[k] = bytes;
  }
  // device blob: rule_of[ns*ns] | templates[nr*RT_WORDS] | arity[ns]
  out->blob.clear();
  out->blob.insert(out->blob.end(), out->rule_of.begin(), out->rule_of.end());
  out->blob.insert(out->blob.end(), out->templ.begin(), out->templ.end());
  out->blob.insert(out->blob.end(), out->arity.begin(), out->arity.end());
  return INET_OK;
}

}  // namespace inet
