/* oracle_checks.c -- runs the oracle under ASan/UBSan on the cases written by
 * tests/test_sanitize.py (same input format as host_checks.cpp, kind ignored),
 * with every schedule that suits the case's size; prints one line per case
 * and schedule with the status, the interaction count and the stream length. */
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int32_t *words;
static size_t n_words, pos;

static int32_t next(void) {
  if (pos >= n_words) { fprintf(stderr, "input ended early\n"); exit(2); }
  return words[pos++];
}

static const int32_t *take(int64_t n) {
  if (n < 0 || (size_t)n > n_words - pos) { fprintf(stderr, "bad length\n"); exit(2); }
  const int32_t *p = words + pos;
  pos += (size_t)n;
  return p;
}

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  size_t cap = 1 << 16;
  words = malloc(cap * 4);
  int32_t w;
  while (fread(&w, 4, 1, f) == 1) {
    if (n_words == cap) { cap *= 2; words = realloc(words, cap * 4); }
    words[n_words++] = w;
  }
  fclose(f);
  const int32_t n_cases = next();
  for (int32_t c = 0; c < n_cases; c++) {
    orc_input in;
    in.n_symbols = next();
    in.arity = take(in.n_symbols);
    in.n_rules = next();
    in.rule_lhs = take(2 * (int64_t)in.n_rules);
    in.rhs_off = take((int64_t)in.n_rules + 1);
    in.rhs = take(in.rhs_off[in.n_rules]);
    in.n_agents = next();
    in.label = take(in.n_agents);
    in.port = take(2 * (int64_t)in.n_agents);
    in.n_eqs = next();
    in.eq_lhs = take(in.n_eqs);
    in.eq_rhs = take(in.n_eqs);
    in.n_names = next();
    (void)next(); /* kind */
    const int schedules[] = {ORC_FIFO, ORC_LIFO, ORC_RANDOM, ORC_ROUNDS, ORC_FIFO | ORC_EAGER,
                             ORC_ENUMERATE};
    const int n_sched = in.n_agents <= 4 ? 6 : 5; /* every order: tiny nets only */
    for (int k = 0; k < n_sched; k++) {
      uint64_t per_rule[64] = {0};
      int32_t *nf = NULL;
      orc_result r;
      const int rc = orc_reduce(&in, schedules[k], 7, 2000000, per_rule, &nf, &r);
      printf("case %d sched %d rc %d ints %llu len %lld\n", c, schedules[k], rc,
             (unsigned long long)r.interactions, (long long)r.nf_len);
      orc_free(nf);
      fflush(stdout);
    }
  }
  free(words);
  return 0;
}
