/*
 * oracle.h -- sequential CPU evaluator of the lightweight interaction calculus.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, layout or helper with the GPU evaluator; both only read the same
 * flat input arrays (format described below).
 *
 * What it computes (paper, Section 2.2): the configuration <t | Delta> is
 * rewritten with the four reduction rules -- interaction (int), communication
 * (com), substitution (sub), collect (col) -- until no active pair and no
 * com-eligible pair remain (the evaluate() loop of Section 3.6 with its
 * correctness proposition); then sub and col are applied exhaustively
 * (Theorem 1 of Section 2.2: sub/col can be deferred to the end).  By uniform
 * confluence (Proposition 2.1.1) the result and the number of int steps do not
 * depend on the order; the oracle lets the caller pick the order so that this
 * can be checked.
 *
 * Input format (int32):
 *   term ref r: r >= 0 agent r, r < 0 name (-1 - r).
 *   label[n_agents], port[n_agents][2] (entries past the arity ignored),
 *   eq_lhs[n_eqs], eq_rhs[n_eqs], names in [0, n_names).
 *   rules: arity[n_symbols]; lhs[n_rules][2]; rule k's words
 *   rhs[rhs_off[k] .. rhs_off[k+1]) = n_eq, then n_eq pairs of prefix-encoded
 *   terms (label >= 0 followed by its subterms, or name -1-v); rule-local
 *   names 0..ar(a)-1 are the first LHS agent's ports, then the second's, and
 *   the rest are bound names of the right-hand side.
 *
 * Output: canonical normal-form stream
 *   [n_iface] T(iface_0) ... [n_res] T(l_0) T(r_0) ...
 *   T(agent) = label, T(child_0), ..., T(child_ar-1)
 *   T(name)  = -(1 + c), c numbered by first appearance in the stream.
 *   The interface is the names occurring once in Delta, ascending id; the
 *   residual equations are the active pairs without a rule, each oriented
 *   and all sorted by their name-erased encodings.
 */
#ifndef INET_ORACLE_H
#define INET_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_FIFO = 0,      /* oldest equation first                         */
  ORC_LIFO = 1,      /* newest equation first                         */
  ORC_RANDOM = 2,    /* uniformly random pending equation (seeded)    */
  ORC_ROUNDS = 3,    /* maximal parallel rounds: all active pairs of a
                        round are reduced, then com runs to closure     */
  ORC_ENUMERATE = 4, /* every order of the int steps (tiny nets only) */
  ORC_EAGER = 0x100  /* flag: apply sub/col as soon as possible too    */
};

enum {
  ORC_OK = 0, ORC_STUCK = 1, ORC_EINVAL = -1, ORC_ENOMEM = -2,
  ORC_ELIMIT = -3, ORC_ERANGE = -4
};

typedef struct {
  int32_t n_symbols;
  const int32_t *arity;
  int32_t n_rules;
  const int32_t *rule_lhs;
  const int32_t *rhs_off;
  const int32_t *rhs;
  int32_t n_agents;
  const int32_t *label;
  const int32_t *port;
  int32_t n_eqs;
  const int32_t *eq_lhs;
  const int32_t *eq_rhs;
  int32_t n_names;
} orc_input;

typedef struct {
  int32_t status;
  int32_t n_iface;
  int32_t n_stuck;      /* residual active pairs without a rule           */
  int32_t n_cycles;     /* residual equations x = t with x inside t        */
  int32_t n_loops;      /* closed loops x = x that were dropped            */
  int32_t n_outcomes;   /* ENUMERATE: distinct (stream, count, histogram)  */
  uint64_t interactions;
  uint64_t rounds;      /* ROUNDS schedule: number of parallel rounds      */
  uint64_t n_com, n_sub, n_col;
  uint64_t max_live_agents;
  uint64_t final_live_agents;
  uint64_t n_schedules; /* ENUMERATE: complete schedules explored          */
  int64_t nf_len;       /* words of the canonical stream                   */
} orc_result;

/* Reduce to normal form.  per_rule: caller array of n_rules counters (may be
 * NULL).  nf_out (may be NULL): receives a malloc'd canonical stream of
 * out->nf_len words, to be released with orc_free.  max_interactions: 0 =
 * unlimited (ENUMERATE: cap on explored schedules).  Returns the status (also
 * in out->status). */
int orc_reduce(const orc_input *in, int schedule, uint64_t seed,
               uint64_t max_interactions, uint64_t *per_rule, int32_t **nf_out,
               orc_result *out);
void orc_free(void *p);

const char *orc_version(void);

#ifdef __cplusplus
}
#endif
#endif
