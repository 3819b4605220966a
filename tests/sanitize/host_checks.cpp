// host_checks.cpp -- drives the host side of the evaluator under ASan/UBSan:
// the rule compiler (folding of right-hand sides), the validation of nets and
// the canonical read-back, on cases written by tests/test_sanitize.py.
//
// Input (little-endian int32 words): a count of cases, then per case
//   n_symbols, arity[n_symbols], n_rules, rule_lhs[2 n_rules],
//   rhs_off[n_rules + 1], rhs[rhs_off[n_rules]],
//   n_agents, label[n_agents], port[2 n_agents], n_eqs, eq_lhs[n_eqs],
//   eq_rhs[n_eqs], n_names, kind
// kind 0: a net as given; kind 1: the same heap with its equations parked in
// the name cells (a finished state for the read-back); kind 2: heap words
// scrambled from a seed (cycles, references out of range) for the read-back's
// error paths.  Output: one line per case with the status of each stage.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "inet.h"
#include "runtime.h"

using namespace inet;

static std::vector<int32_t> words;
static size_t pos = 0;

static int32_t next() {
  if (pos >= words.size()) {
    std::fprintf(stderr, "input ended early\n");
    std::exit(2);
  }
  return words[pos++];
}

static std::vector<int32_t> take(int64_t n) {
  if (n < 0 || (size_t)n > words.size() - pos) {
    std::fprintf(stderr, "bad length %lld\n", (long long)n);
    std::exit(2);
  }
  std::vector<int32_t> v(words.begin() + pos, words.begin() + pos + n);
  pos += n;
  return v;
}

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t w;
  while (std::fread(&w, 4, 1, f) == 1) words.push_back(w);
  std::fclose(f);
  const int32_t n_cases = next();
  for (int32_t c = 0; c < n_cases; c++) {
    const int32_t ns = next();
    std::vector<int32_t> arity = take(ns);
    const int32_t nr = next();
    std::vector<int32_t> lhs = take(2 * (int64_t)nr);
    std::vector<int32_t> off = take((int64_t)nr + 1);
    std::vector<int32_t> rhs = take(off.empty() ? 0 : off.back());
    const int32_t na = next();
    std::vector<int32_t> label = take(na), port = take(2 * (int64_t)na);
    const int32_t ne = next();
    std::vector<int32_t> el = take(ne), er = take(ne);
    const int32_t nn = next();
    const int32_t kind = next();
    inet_rules rules{ns, arity.data(), nr, lhs.data(), off.data(), rhs.data()};
    CompiledRules R;
    const int rc_rules = compile_rules(&rules, &R);
    int rc_check = inet_rules_check(&rules, nullptr, nullptr, nullptr, nullptr, 0);
    int rc_net = -100, rc_read = -100;
    size_t out_len = 0;
    if (rc_rules == INET_OK) {
      std::vector<int32_t> iface;
      rc_net = validate_net(R, label.data(), port.data(), na, el.data(), er.data(), ne, nn, &iface);
      if (rc_net == INET_OK || kind == 2) {
        // a heap: agents as given, each equation parked in a name cell (or a
        // residual pair of agents)
        std::vector<int32_t> p0(na), p1(na), bind(nn, EMPTY);
        for (int32_t i = 0; i < na; i++) {
          p0[i] = port[2 * i];
          p1[i] = port[2 * i + 1];
        }
        std::vector<int2> stuck;
        if (kind >= 1) {
          for (int32_t e = 0; e < ne; e++) {
            int32_t u = el[e], v = er[e];
            if (u >= 0) std::swap(u, v);
            if (u < 0 && ~u < nn && bind[~u] == EMPTY) bind[~u] = v;
            else if (u >= 0 && v >= 0) stuck.push_back(make_int2(u, v));
          }
        }
        if (kind == 2) {
          // scramble: every word of the heap replaced from a seeded sequence
          uint64_t x = 0x9e3779b97f4a7c15ull ^ (uint64_t)c;
          auto rnd = [&]() {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            return (int32_t)(x >> 32);
          };
          for (int32_t i = 0; i < na; i++) {
            label[i] = (int32_t)((uint32_t)rnd() % (uint32_t)(ns + 1));
            p0[i] = rnd() % (2 * na + 3) - (na + 1);
            p1[i] = rnd() % (2 * na + 3) - (na + 1);
          }
          for (int32_t x2 = 0; x2 < nn; x2++) bind[x2] = (rnd() & 3) ? rnd() % (2 * nn + 3) - nn : EMPTY;
          for (int32_t k = 0; k < nn && k < 4; k++) iface.push_back(k);
        }
        std::vector<int32_t> out;
        rc_read = canonical_stream(R, label.data(), p0.data(), p1.data(), na, bind.data(), nn,
                                   iface, stuck, &out);
        out_len = out.size();
      }
    }
    std::printf("case %d rules %d check %d net %d read %d len %zu\n", c, rc_rules, rc_check, rc_net,
                rc_read, out_len);
  }
  return 0;
}
