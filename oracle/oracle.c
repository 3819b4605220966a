/*
 * oracle.c -- sequential CPU evaluator of the lightweight interaction calculus
 * (paper, Section 2.2).  TEST INFRASTRUCTURE ONLY: loaded by the test-suite,
 * the smoke check and the benchmark's CPU-baseline leg, never by the product.
 *
 * The configuration is kept literally as term trees:
 *   - a node is an agent alpha(t1..tn) or one occurrence of a name;
 *   - every node knows the slot holding it: an equation side, a child slot of
 *     an agent node, or a position of the interface list;
 *   - every name knows its (at most two) occurrence nodes.
 * The four reduction rules of Section 2.2 then act locally:
 *   int : alpha(t1) = beta(t2) is replaced by Theta', the right-hand side of
 *         the rule with every bound name renamed apart and the rule's argument
 *         names replaced by the actual subterms t1, t2;
 *   com, sub, col : an equation x = t is removed and the other occurrence of x
 *         is replaced by t.  Which of the three it is depends only on where
 *         that other occurrence sits: on top of another equation (com), inside
 *         an agent term (sub), or in the interface (col).
 * The main loop applies int and com until neither applies (the loop of the
 * evaluate() pseudo-code, Section 3.6); sub and col are deferred to the end as
 * Theorem 1 allows, or applied eagerly with ORC_EAGER to check that theorem.
 */
#include "oracle.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXAR 2
#define MAXRULEWORDS 4096

/* ORC_MUTANT plants a plausible mistake; built only by the mutation test to
 * show that the pins catch it.  0 (default) = the correct oracle. */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

enum { K_FREE = 0, K_AGENT = 1, K_NAME = 2 };
enum { P_EQ = 0, P_NODE = 1, P_IFACE = 2, P_NONE = 3 };

typedef struct {
  /* nodes */
  int32_t *kind, *sym, *ptype, *pidx, *pslot, *ch; /* ch: [node][MAXAR] */
  int64_t ncap, nused;
  int32_t *nfree;
  int64_t nfree_n, nfree_cap;
  int64_t live_agents, max_live_agents;
  /* equations (ids are never reused) */
  int32_t *el, *er;
  uint8_t *ealive, *estuck;
  int64_t ecap, eused;
  /* names: two occurrence nodes each */
  int32_t *occ;
  int64_t namecap, nnames;
  /* interface */
  int32_t *iface;
  int32_t n_iface;
  /* rules */
  int32_t ns;
  const int32_t *arity;
  int32_t nr;
  int32_t *rule_of; /* [ns*ns]: 2*rule + swapped, or -1 */
  const int32_t *rhs_off, *rhs;
  const int32_t *rule_lhs;
  /* statistics */
  uint64_t interactions, n_com, n_sub, n_col, rounds;
  int32_t n_loops;
  uint64_t *per_rule;
  int oom;
} St;

/* ------------------------------------------------------------------------ */
/* storage                                                                   */
/* ------------------------------------------------------------------------ */

static void *grow(void *p, int64_t n, size_t elem) {
  void *q = realloc(p, (size_t)n * elem);
  return q;
}

static int node_new(St *s, int32_t kind, int32_t sym) {
  int32_t id;
  if (s->nfree_n > 0) {
    id = s->nfree[--s->nfree_n];
  } else {
    if (s->nused == s->ncap) {
      int64_t nc = s->ncap ? s->ncap * 2 : 1024;
      int32_t **arrs[] = {&s->kind, &s->sym, &s->ptype, &s->pidx, &s->pslot};
      for (int i = 0; i < 5; i++) {
        void *q = grow(*arrs[i], nc, sizeof(int32_t));
        if (!q) { s->oom = 1; return -1; }
        *arrs[i] = (int32_t *)q;
      }
      void *q = grow(s->ch, nc * MAXAR, sizeof(int32_t));
      if (!q) { s->oom = 1; return -1; }
      s->ch = (int32_t *)q;
      s->ncap = nc;
    }
    id = (int32_t)s->nused++;
  }
  s->kind[id] = kind;
  s->sym[id] = sym;
  s->ptype[id] = P_NONE;
  s->pidx[id] = -1;
  s->pslot[id] = -1;
  s->ch[id * MAXAR + 0] = -1;
  s->ch[id * MAXAR + 1] = -1;
  if (kind == K_AGENT) {
    s->live_agents++;
    if (s->live_agents > s->max_live_agents) s->max_live_agents = s->live_agents;
  }
  return id;
}

static void node_free(St *s, int32_t id) {
  if (s->kind[id] == K_AGENT) s->live_agents--;
  s->kind[id] = K_FREE;
  if (s->nfree_n == s->nfree_cap) {
    int64_t nc = s->nfree_cap ? s->nfree_cap * 2 : 1024;
    void *q = grow(s->nfree, nc, sizeof(int32_t));
    if (!q) { s->oom = 1; return; }
    s->nfree = (int32_t *)q;
    s->nfree_cap = nc;
  }
  s->nfree[s->nfree_n++] = id;
}

static int64_t name_new(St *s) {
  if (s->nnames == s->namecap) {
    int64_t nc = s->namecap ? s->namecap * 2 : 1024;
    void *q = grow(s->occ, nc * 2, sizeof(int32_t));
    if (!q) { s->oom = 1; return -1; }
    s->occ = (int32_t *)q;
    s->namecap = nc;
  }
  s->occ[s->nnames * 2] = -1;
  s->occ[s->nnames * 2 + 1] = -1;
  return s->nnames++;
}

/* a new occurrence node of name x */
static int name_node(St *s, int32_t x) {
  int n = node_new(s, K_NAME, x);
  if (n < 0) return -1;
  if (s->occ[x * 2] < 0) s->occ[x * 2] = n;
  else if (s->occ[x * 2 + 1] < 0) s->occ[x * 2 + 1] = n;
  else { s->oom = 2; } /* a third occurrence: impossible after validation */
  return n;
}

static int32_t other_occ(St *s, int32_t n) {
  int32_t x = s->sym[n];
  if (s->occ[x * 2] == n) return s->occ[x * 2 + 1];
  return s->occ[x * 2];
}

static void name_drop_occ(St *s, int32_t n) {
  int32_t x = s->sym[n];
  if (s->occ[x * 2] == n) s->occ[x * 2] = -1;
  else if (s->occ[x * 2 + 1] == n) s->occ[x * 2 + 1] = -1;
}

static int64_t eq_new(St *s, int32_t l, int32_t r) {
  if (s->eused == s->ecap) {
    int64_t nc = s->ecap ? s->ecap * 2 : 1024;
    void *a = grow(s->el, nc, sizeof(int32_t));
    if (!a) { s->oom = 1; return -1; }
    s->el = (int32_t *)a;
    void *b = grow(s->er, nc, sizeof(int32_t));
    if (!b) { s->oom = 1; return -1; }
    s->er = (int32_t *)b;
    void *c = grow(s->ealive, nc, 1);
    if (!c) { s->oom = 1; return -1; }
    s->ealive = (uint8_t *)c;
    void *d = grow(s->estuck, nc, 1);
    if (!d) { s->oom = 1; return -1; }
    s->estuck = (uint8_t *)d;
    s->ecap = nc;
  }
  int64_t e = s->eused++;
  s->el[e] = l;
  s->er[e] = r;
  s->ealive[e] = 1;
  s->estuck[e] = 0;
  s->ptype[l] = P_EQ; s->pidx[l] = (int32_t)e; s->pslot[l] = 0;
  s->ptype[r] = P_EQ; s->pidx[r] = (int32_t)e; s->pslot[r] = 1;
  return e;
}

/* put node t into the slot currently held by node old */
static void put_in_slot_of(St *s, int32_t old, int32_t t) {
  int32_t pt = s->ptype[old], pi = s->pidx[old], ps = s->pslot[old];
  if (pt == P_EQ) {
    if (ps == 0) s->el[pi] = t; else s->er[pi] = t;
  } else if (pt == P_NODE) {
    s->ch[pi * MAXAR + ps] = t;
  } else if (pt == P_IFACE) {
    s->iface[pi] = t;
  }
  s->ptype[t] = pt;
  s->pidx[t] = pi;
  s->pslot[t] = ps;
}

static void st_free(St *s) {
  free(s->kind); free(s->sym); free(s->ptype); free(s->pidx); free(s->pslot);
  free(s->ch); free(s->nfree); free(s->el); free(s->er); free(s->ealive);
  free(s->estuck); free(s->occ); free(s->iface); free(s->rule_of);
  memset(s, 0, sizeof(*s));
}

static void *dup_arr(const void *p, size_t bytes, int *oom) {
  if (!p || bytes == 0) return NULL;
  void *q = malloc(bytes);
  if (!q) { *oom = 1; return NULL; }
  memcpy(q, p, bytes);
  return q;
}

static int st_clone(const St *a, St *b) {
  int oom = 0;
  *b = *a;
  b->kind = dup_arr(a->kind, a->ncap * 4, &oom);
  b->sym = dup_arr(a->sym, a->ncap * 4, &oom);
  b->ptype = dup_arr(a->ptype, a->ncap * 4, &oom);
  b->pidx = dup_arr(a->pidx, a->ncap * 4, &oom);
  b->pslot = dup_arr(a->pslot, a->ncap * 4, &oom);
  b->ch = dup_arr(a->ch, a->ncap * 4 * MAXAR, &oom);
  b->nfree = dup_arr(a->nfree, a->nfree_cap * 4, &oom);
  b->el = dup_arr(a->el, a->ecap * 4, &oom);
  b->er = dup_arr(a->er, a->ecap * 4, &oom);
  b->ealive = dup_arr(a->ealive, a->ecap, &oom);
  b->estuck = dup_arr(a->estuck, a->ecap, &oom);
  b->occ = dup_arr(a->occ, a->namecap * 8, &oom);
  b->iface = dup_arr(a->iface, (size_t)(a->n_iface > 0 ? a->n_iface : 0) * 4, &oom);
  b->rule_of = dup_arr(a->rule_of, (size_t)a->ns * a->ns * 4, &oom);
  b->per_rule = NULL;
  return oom ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* worklist (a deque of equation ids)                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t *v;
  int64_t head, tail, cap;
} Deque;

static int dq_push(Deque *d, int32_t e) {
  if (d->tail == d->cap) {
    if (d->head > 0) {
      memmove(d->v, d->v + d->head, (size_t)(d->tail - d->head) * 4);
      d->tail -= d->head;
      d->head = 0;
    }
    if (d->tail == d->cap) {
      int64_t nc = d->cap ? d->cap * 2 : 1024;
      void *q = grow(d->v, nc, sizeof(int32_t));
      if (!q) return -1;
      d->v = (int32_t *)q;
      d->cap = nc;
    }
  }
  d->v[d->tail++] = e;
  return 0;
}

static int dq_empty(const Deque *d) { return d->head == d->tail; }

static uint64_t rng_next(uint64_t *x) { /* splitmix64 (Steele, Lea, Flood) */
  uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static int32_t dq_pop(Deque *d, int schedule, uint64_t *rng) {
  if (schedule == ORC_LIFO) return d->v[--d->tail];
  if (schedule == ORC_RANDOM) {
    int64_t n = d->tail - d->head;
    int64_t k = d->head + (int64_t)(rng_next(rng) % (uint64_t)n);
    int32_t e = d->v[k];
    d->v[k] = d->v[--d->tail];
    return e;
  }
  return d->v[d->head++];
}

/* ------------------------------------------------------------------------ */
/* rules                                                                     */
/* ------------------------------------------------------------------------ */

/* walk one prefix-encoded term of rule k; counts name uses in cnt[] */
static int rule_scan_term(const St *s, const int32_t *w, int64_t n, int64_t *pos,
                          int32_t *cnt, int32_t cntcap, int depth) {
  if (*pos >= n || depth > 64) return -1;
  int32_t v = w[(*pos)++];
  if (v >= 0) {
    if (v >= s->ns) return -1;
    for (int j = 0; j < s->arity[v]; j++)
      if (rule_scan_term(s, w, n, pos, cnt, cntcap, depth + 1)) return -1;
    return 0;
  }
  int32_t k = -1 - v;
  if (k >= cntcap) return -1;
  cnt[k]++;
  return 0;
}

static int rules_prepare(St *s, const orc_input *in) {
  s->ns = in->n_symbols;
  s->arity = in->arity;
  s->nr = in->n_rules;
  s->rhs_off = in->rhs_off;
  s->rhs = in->rhs;
  s->rule_lhs = in->rule_lhs;
  if (s->ns <= 0 || s->ns > 4096 || s->nr < 0) return ORC_EINVAL;
  for (int i = 0; i < s->ns; i++)
    if (s->arity[i] < 0 || s->arity[i] > MAXAR) return ORC_EINVAL;
  s->rule_of = (int32_t *)malloc((size_t)s->ns * s->ns * 4);
  if (!s->rule_of) return ORC_ENOMEM;
  for (int64_t i = 0; i < (int64_t)s->ns * s->ns; i++) s->rule_of[i] = -1;
  int32_t cnt[MAXRULEWORDS];
  for (int k = 0; k < s->nr; k++) {
    int32_t a = s->rule_lhs[2 * k], b = s->rule_lhs[2 * k + 1];
    if (a < 0 || b < 0 || a >= s->ns || b >= s->ns || a == b) return ORC_EINVAL;
    if (s->rule_of[a * s->ns + b] != -1) return ORC_EINVAL;
    s->rule_of[a * s->ns + b] = 2 * k;
    s->rule_of[b * s->ns + a] = 2 * k + 1;
    int64_t lo = s->rhs_off[k], hi = s->rhs_off[k + 1];
    if (lo < 0 || hi <= lo || hi - lo > MAXRULEWORDS) return ORC_EINVAL;
    const int32_t *w = s->rhs + lo;
    int64_t n = hi - lo, pos = 1;
    int32_t neq = w[0];
    if (neq < 0) return ORC_EINVAL;
    memset(cnt, 0, sizeof(cnt));
    for (int e = 0; e < 2 * neq; e++)
      if (rule_scan_term(s, w, n, &pos, cnt, MAXRULEWORDS, 0)) return ORC_EINVAL;
    if (pos != n) return ORC_EINVAL;
    int32_t nargs = s->arity[a] + s->arity[b];
    for (int v = 0; v < MAXRULEWORDS; v++) {
      if (v < nargs) { if (cnt[v] != 1) return ORC_EINVAL; }
      else if (cnt[v] != 0 && cnt[v] != 2) return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

typedef struct {
  int32_t args[2 * MAXAR];
  int32_t nargs;
  int32_t fresh[MAXRULEWORDS];
} Inst;

static int32_t inst_term(St *s, const int32_t *w, int64_t *pos, Inst *I) {
  int32_t v = w[(*pos)++];
  if (v >= 0) {
    int32_t n = node_new(s, K_AGENT, v);
    if (n < 0) return -1;
    for (int j = 0; j < s->arity[v]; j++) {
      int32_t c = inst_term(s, w, pos, I);
      if (c < 0) return -1;
      s->ch[n * MAXAR + j] = c;
      s->ptype[c] = P_NODE; s->pidx[c] = n; s->pslot[c] = j;
    }
    return n;
  }
  int32_t k = -1 - v;
  if (k < I->nargs) return I->args[k]; /* the actual argument term, moved */
  if (I->fresh[k] < 0) {
    int64_t x = name_new(s);
    if (x < 0) return -1;
    I->fresh[k] = (int32_t)x;
  }
  return name_node(s, I->fresh[k]);
}

/* ------------------------------------------------------------------------ */
/* reduction                                                                 */
/* ------------------------------------------------------------------------ */

/* int on equation e (both sides agents).  New equations go to wl. */
static int do_int(St *s, int32_t e, Deque *wl) {
  int32_t l = s->el[e], r = s->er[e];
  int32_t code = s->rule_of[s->sym[l] * s->ns + s->sym[r]];
  if (code < 0) { s->estuck[e] = 1; return 0; }
  int32_t k = code >> 1;
  if ((code & 1) && ORC_MUTANT != 2) { int32_t t = l; l = r; r = t; }
  Inst I;
  int32_t aa = s->arity[s->sym[l]], ab = s->arity[s->sym[r]];
  I.nargs = aa + ab;
  for (int j = 0; j < aa; j++) I.args[j] = s->ch[l * MAXAR + j];
  for (int j = 0; j < ab; j++) I.args[aa + j] = s->ch[r * MAXAR + j];
  if (ORC_MUTANT == 1 && aa == 2) { int32_t t = I.args[0]; I.args[0] = I.args[1]; I.args[1] = t; }
  int64_t lo = s->rhs_off[k], hi = s->rhs_off[k + 1];
  for (int64_t i = 0; i < hi - lo; i++) I.fresh[i] = -1;
  s->ealive[e] = 0;
  node_free(s, l);
  node_free(s, r);
  const int32_t *w = s->rhs + lo;
  int64_t pos = 1;
  int32_t neq = w[0];
  if (ORC_MUTANT == 3 && neq > 1) neq--; /* drops the last equation */
  for (int q = 0; q < neq; q++) {
    int32_t tl = inst_term(s, w, &pos, &I);
    int32_t tr = inst_term(s, w, &pos, &I);
    if (tl < 0 || tr < 0) return -1;
    int64_t ne = eq_new(s, tl, tr);
    if (ne < 0 || dq_push(wl, (int32_t)ne)) return -1;
  }
  s->interactions++;
  if (s->per_rule) s->per_rule[k]++;
  return 1;
}

/* the top-level equation (or interface slot) whose term contains node n */
static void root_of(const St *s, int32_t n, int32_t *rt, int32_t *ri) {
  while (s->ptype[n] == P_NODE) n = s->pidx[n];
  *rt = s->ptype[n];
  *ri = s->pidx[n];
}

/* Try com (and, when eager, sub/col) on equation e through its name side n.
 * Returns 1 if e was consumed. */
static int try_name_side(St *s, int32_t e, int32_t n, int eager, Deque *wl) {
  int32_t t = (s->el[e] == n) ? s->er[e] : s->el[e];
  int32_t o = other_occ(s, n);
  if (o < 0) return 0;
  if (s->ptype[o] == P_EQ && s->pidx[o] == e) {
    /* x = x: a closed loop, dropped */
    name_drop_occ(s, n); name_drop_occ(s, o);
    node_free(s, n); node_free(s, o);
    s->ealive[e] = 0;
    s->n_loops++;
    return 1;
  }
  int kind;
  if (s->ptype[o] == P_EQ) kind = 0;              /* com */
  else if (!eager) return 0;
  else {
    int32_t rt, ri;
    root_of(s, o, &rt, &ri);
    if (rt == P_EQ && ri == e) return 0;          /* x inside t: cycle */
    kind = (rt == P_IFACE) ? 2 : 1;               /* col : sub */
  }
  int32_t e2 = s->pidx[o];
  name_drop_occ(s, n); name_drop_occ(s, o);
  put_in_slot_of(s, o, t);
  node_free(s, n); node_free(s, o);
  s->ealive[e] = 0;
  if (kind == 0) {
    s->n_com++;
    if (ORC_MUTANT == 4) s->interactions++;
    if (dq_push(wl, e2)) return -1; /* e2 now reads t = u */
  } else if (kind == 1) {
    s->n_sub++;
  } else {
    s->n_col++;
  }
  return 1;
}

/* Examine one equation.  collect != NULL: active pairs are appended there
 * instead of being reduced (round schedule / enumeration). */
static int examine(St *s, int32_t e, int eager, Deque *wl, Deque *collect) {
  if (!s->ealive[e] || s->estuck[e]) return 0;
  int32_t l = s->el[e], r = s->er[e];
  if (s->kind[l] == K_AGENT && s->kind[r] == K_AGENT) {
    if (collect) {
      if (s->rule_of[s->sym[l] * s->ns + s->sym[r]] < 0) { s->estuck[e] = 1; return 0; }
      return dq_push(collect, e);
    }
    return do_int(s, e, wl) < 0 ? -1 : 0;
  }
  if (s->kind[l] == K_NAME) {
    int rc = try_name_side(s, e, l, eager, wl);
    if (rc) return rc < 0 ? -1 : 0;
  }
  if (s->ealive[e] && s->kind[r] == K_NAME) {
    int rc = try_name_side(s, e, r, eager, wl);
    if (rc) return rc < 0 ? -1 : 0;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* loading                                                                   */
/* ------------------------------------------------------------------------ */

static int load(St *s, const orc_input *in, Deque *wl) {
  int32_t na = in->n_agents, ne = in->n_eqs, nn = in->n_names;
  if (na < 0 || ne < 0 || nn < 0) return ORC_EINVAL;
  int32_t *anode = (int32_t *)malloc((size_t)(na > 0 ? na : 1) * 4);
  int32_t *refs = (int32_t *)calloc((size_t)(na > 0 ? na : 1), 4);
  int32_t *ncount = (int32_t *)calloc((size_t)(nn > 0 ? nn : 1), 4);
  if (!anode || !refs || !ncount) { free(anode); free(refs); free(ncount); return ORC_ENOMEM; }
  int rc = ORC_OK;
  /* count references of agents and names */
  for (int32_t i = 0; i < na && rc == ORC_OK; i++) {
    int32_t lab = in->label[i];
    if (lab < 0 || lab >= s->ns) { rc = ORC_EINVAL; break; }
    for (int j = 0; j < s->arity[lab]; j++) {
      int32_t v = in->port[2 * i + j];
      if (v >= 0) { if (v >= na) { rc = ORC_EINVAL; break; } refs[v]++; }
      else { int32_t x = -1 - v; if (x >= nn) { rc = ORC_EINVAL; break; } ncount[x]++; }
    }
  }
  for (int32_t e = 0; e < ne && rc == ORC_OK; e++) {
    int32_t sides[2] = {in->eq_lhs[e], in->eq_rhs[e]};
    for (int q = 0; q < 2; q++) {
      int32_t v = sides[q];
      if (v >= 0) { if (v >= na) { rc = ORC_EINVAL; break; } refs[v]++; }
      else { int32_t x = -1 - v; if (x >= nn) { rc = ORC_EINVAL; break; } ncount[x]++; }
    }
  }
  for (int32_t i = 0; i < na && rc == ORC_OK; i++) if (refs[i] != 1) rc = ORC_EINVAL;
  for (int32_t x = 0; x < nn && rc == ORC_OK; x++) if (ncount[x] > 2) rc = ORC_EINVAL;
  if (rc != ORC_OK) { free(anode); free(refs); free(ncount); return rc; }
  /* names */
  for (int32_t x = 0; x < nn; x++) if (name_new(s) < 0) { rc = ORC_ENOMEM; break; }
  /* agent nodes */
  for (int32_t i = 0; i < na && rc == ORC_OK; i++) {
    anode[i] = node_new(s, K_AGENT, in->label[i]);
    if (anode[i] < 0) rc = ORC_ENOMEM;
  }
  /* children */
  for (int32_t i = 0; i < na && rc == ORC_OK; i++) {
    int32_t lab = in->label[i];
    for (int j = 0; j < s->arity[lab]; j++) {
      int32_t v = in->port[2 * i + j];
      int32_t c = (v >= 0) ? anode[v] : name_node(s, -1 - v);
      if (c < 0) { rc = ORC_ENOMEM; break; }
      s->ch[anode[i] * MAXAR + j] = c;
      s->ptype[c] = P_NODE; s->pidx[c] = anode[i]; s->pslot[c] = j;
    }
  }
  /* equations */
  for (int32_t e = 0; e < ne && rc == ORC_OK; e++) {
    int32_t v0 = in->eq_lhs[e], v1 = in->eq_rhs[e];
    int32_t t0 = (v0 >= 0) ? anode[v0] : name_node(s, -1 - v0);
    int32_t t1 = (v1 >= 0) ? anode[v1] : name_node(s, -1 - v1);
    if (t0 < 0 || t1 < 0) { rc = ORC_ENOMEM; break; }
    int64_t id = eq_new(s, t0, t1);
    if (id < 0 || dq_push(wl, (int32_t)id)) rc = ORC_ENOMEM;
  }
  /* every agent must hang below an equation side (no cyclic nesting):
   * count the agents reachable from the equation sides */
  if (rc == ORC_OK && na > 0) {
    int32_t *stk = (int32_t *)malloc((size_t)na * 4);
    int64_t reached = 0, sp = 0;
    if (!stk) rc = ORC_ENOMEM;
    for (int64_t e = 0; e < s->eused && rc == ORC_OK; e++) {
      int32_t tops[2] = {s->el[e], s->er[e]};
      for (int q = 0; q < 2; q++) {
        if (s->kind[tops[q]] != K_AGENT) continue;
        stk[sp++] = tops[q];
        while (sp) {
          int32_t n = stk[--sp];
          reached++;
          for (int j = 0; j < s->arity[s->sym[n]]; j++) {
            int32_t c = s->ch[n * MAXAR + j];
            if (s->kind[c] == K_AGENT) stk[sp++] = c;
          }
        }
      }
    }
    if (rc == ORC_OK && reached != na) rc = ORC_EINVAL;
    free(stk);
  }
  /* interface: names occurring once, ascending id */
  if (rc == ORC_OK) {
    int32_t ni = 0;
    for (int32_t x = 0; x < nn; x++) if (ncount[x] == 1) ni++;
    s->iface = (int32_t *)malloc((size_t)(ni > 0 ? ni : 1) * 4);
    if (!s->iface) rc = ORC_ENOMEM;
    s->n_iface = 0;
    for (int32_t x = 0; x < nn && rc == ORC_OK; x++) {
      if (ncount[x] != 1) continue;
      int32_t n = name_node(s, x);
      if (n < 0) { rc = ORC_ENOMEM; break; }
      s->ptype[n] = P_IFACE; s->pidx[n] = s->n_iface; s->pslot[n] = 0;
      s->iface[s->n_iface++] = n;
    }
  }
  free(anode); free(refs); free(ncount);
  if (s->oom) return ORC_ENOMEM;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* sub* col* and the canonical stream                                        */
/* ------------------------------------------------------------------------ */

static int32_t uf_find(int32_t *p, int32_t a) {
  while (p[a] != a) { p[a] = p[p[a]]; a = p[a]; }
  return a;
}

/* Deferred sub/col (Theorem 1).  Groups: equation e -> e, interface slot i ->
 * eused + i.  A node's group is the top of its term; a substitution merges
 * the equation's group into the group of the other occurrence. */
static int readback_subst(St *s, int32_t *n_cycles) {
  int64_t ng = s->eused + s->n_iface;
  int32_t *grp = (int32_t *)malloc((size_t)(s->nused > 0 ? s->nused : 1) * 4);
  int32_t *uf = (int32_t *)malloc((size_t)(ng > 0 ? ng : 1) * 4);
  int32_t *stk = (int32_t *)malloc((size_t)(s->nused > 0 ? s->nused : 1) * 4);
  if (!grp || !uf || !stk) { free(grp); free(uf); free(stk); return ORC_ENOMEM; }
  for (int64_t g = 0; g < ng; g++) uf[g] = (int32_t)g;
  /* label every live node with the group of its root */
  for (int64_t root = 0; root < ng; root++) {
    int32_t tops[2];
    int nt = 0;
    if (root < s->eused) {
      if (!s->ealive[root]) continue;
      tops[nt++] = s->el[root];
      tops[nt++] = s->er[root];
    } else {
      tops[nt++] = s->iface[root - s->eused];
    }
    for (int q = 0; q < nt; q++) {
      int64_t sp = 0;
      stk[sp++] = tops[q];
      while (sp) {
        int32_t n = stk[--sp];
        grp[n] = (int32_t)root;
        if (s->kind[n] == K_AGENT)
          for (int j = 0; j < s->arity[s->sym[n]]; j++) stk[sp++] = s->ch[n * MAXAR + j];
      }
    }
  }
  int32_t cycles = 0;
  for (int64_t e = 0; e < s->eused; e++) {
    if (!s->ealive[e] || s->estuck[e]) continue;
    int done = 0;
    for (int side = 0; side < 2 && !done; side++) {
      int32_t n = side == 0 ? s->el[e] : s->er[e];
      if (s->kind[n] != K_NAME) continue;
      int32_t t = side == 0 ? s->er[e] : s->el[e];
      int32_t o = other_occ(s, n);
      if (o < 0) continue;
      int32_t go = uf_find(uf, grp[o]);
      if (go == uf_find(uf, (int32_t)e)) continue; /* x occurs inside t */
      /* col when the occurrence lies in the interface (at its top or nested
       * inside an interface term), sub when it lies inside an equation */
      int kind = (s->ptype[o] == P_EQ) ? 0 : (go >= s->eused ? 2 : 1);
      name_drop_occ(s, n); name_drop_occ(s, o);
      put_in_slot_of(s, o, t);
      node_free(s, n); node_free(s, o);
      s->ealive[e] = 0;
      uf[uf_find(uf, (int32_t)e)] = go;
      if (kind == 2) s->n_col++; else if (kind == 1) s->n_sub++; else s->n_com++;
      done = 1;
    }
    if (!done && s->ealive[e] && ORC_MUTANT != 7) cycles++;
  }
  *n_cycles = cycles;
  free(grp); free(uf); free(stk);
  return ORC_OK;
}

typedef struct {
  int32_t *v;
  int64_t n, cap;
  int oom;
} Buf;

static void buf_put(Buf *b, int32_t w) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? b->cap * 2 : 256;
    void *q = grow(b->v, nc, sizeof(int32_t));
    if (!q) { b->oom = 1; return; }
    b->v = (int32_t *)q;
    b->cap = nc;
  }
  b->v[b->n++] = w;
}

/* preorder encoding of the term at node t; canon == NULL: names erased (-1) */
static void encode(const St *s, int32_t t, int32_t *canon, int32_t *next, Buf *out, Buf *stk) {
  stk->n = 0;
  buf_put(stk, t);
  while (stk->n) {
    int32_t n = stk->v[--stk->n];
    if (s->kind[n] == K_AGENT) {
      buf_put(out, s->sym[n]);
      int32_t ar = s->arity[s->sym[n]];
      for (int j = ar - 1; j >= 0; j--) buf_put(stk, s->ch[n * MAXAR + j]);
    } else {
      if (!canon) { buf_put(out, -1); continue; }
      int32_t x = s->sym[n];
      if (canon[x] < 0) canon[x] = (*next)++;
      buf_put(out, -1 - canon[x]);
    }
  }
}

typedef struct {
  int32_t e;
  int32_t l, r;          /* oriented sides */
  int64_t kl, nl, kr, nr;  /* erased encodings: offsets into a key buffer */
} Res;

static const int32_t *g_keys;

static int cmp_seq(const int32_t *a, int64_t na, const int32_t *b, int64_t nb) {
  int64_t n = na < nb ? na : nb;
  for (int64_t i = 0; i < n; i++) if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return na < nb ? -1 : (na > nb ? 1 : 0);
}

static int cmp_res(const void *pa, const void *pb) {
  const Res *a = (const Res *)pa, *b = (const Res *)pb;
  if (ORC_MUTANT == 6) { /* planted: right sides compared first */
    int c = cmp_seq(g_keys + a->kr, a->nr, g_keys + b->kr, b->nr);
    if (c) return c;
    return cmp_seq(g_keys + a->kl, a->nl, g_keys + b->kl, b->nl);
  }
  int c = cmp_seq(g_keys + a->kl, a->nl, g_keys + b->kl, b->nl);
  if (c) return c;
  return cmp_seq(g_keys + a->kr, a->nr, g_keys + b->kr, b->nr);
}

static int serialise(St *s, Buf *out, int32_t *n_stuck) {
  int32_t *canon = (int32_t *)malloc((size_t)(s->nnames > 0 ? s->nnames : 1) * 4);
  if (!canon) return ORC_ENOMEM;
  for (int64_t x = 0; x < s->nnames; x++) canon[x] = -1;
  int32_t next = 0;
  Buf stk = {0};
  buf_put(out, s->n_iface);
  for (int32_t i = 0; i < s->n_iface; i++) encode(s, s->iface[i], canon, &next, out, &stk);
  /* residual active pairs */
  int64_t nres = 0;
  for (int64_t e = 0; e < s->eused; e++) if (s->ealive[e] && s->estuck[e]) nres++;
  Res *res = (Res *)malloc((size_t)(nres > 0 ? nres : 1) * sizeof(Res));
  Buf keys = {0};
  if (!res) { free(canon); free(stk.v); return ORC_ENOMEM; }
  int64_t k = 0;
  for (int64_t e = 0; e < s->eused; e++) {
    if (!(s->ealive[e] && s->estuck[e])) continue;
    Res *R = &res[k++];
    R->e = (int32_t)e;
    int64_t a0 = keys.n;
    encode(s, s->el[e], NULL, NULL, &keys, &stk);
    int64_t a1 = keys.n;
    encode(s, s->er[e], NULL, NULL, &keys, &stk);
    int64_t a2 = keys.n;
    const int ord = cmp_seq(keys.v + a0, a1 - a0, keys.v + a1, a2 - a1);
    if (ORC_MUTANT == 5 ? ord >= 0 : ord <= 0) { /* 5: planted, larger side first */
      R->l = s->el[e]; R->r = s->er[e];
      R->kl = a0; R->nl = a1 - a0; R->kr = a1; R->nr = a2 - a1;
    } else {
      R->l = s->er[e]; R->r = s->el[e];
      R->kl = a1; R->nl = a2 - a1; R->kr = a0; R->nr = a1 - a0;
    }
  }
  g_keys = keys.v;
  if (nres > 1) qsort(res, (size_t)nres, sizeof(Res), cmp_res);
  buf_put(out, (int32_t)nres);
  for (int64_t i = 0; i < nres; i++) {
    encode(s, res[i].l, canon, &next, out, &stk);
    encode(s, res[i].r, canon, &next, out, &stk);
  }
  *n_stuck = (int32_t)nres;
  int oom = out->oom || stk.oom || keys.oom;
  free(res); free(keys.v); free(stk.v); free(canon);
  return oom ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* drivers                                                                   */
/* ------------------------------------------------------------------------ */

static int run_sequential(St *s, Deque *wl, int schedule, int eager, uint64_t seed,
                          uint64_t max_ints) {
  uint64_t rng = seed;
  while (!dq_empty(wl)) {
    int32_t e = dq_pop(wl, schedule, &rng);
    if (examine(s, e, eager, wl, NULL)) return ORC_ENOMEM;
    if (s->oom) return ORC_ENOMEM;
    if (max_ints && s->interactions > max_ints) return ORC_ELIMIT;
  }
  return ORC_OK;
}

/* Maximal parallel rounds: every active pair present after com has run to
 * closure is reduced in the same round (the loop body of evaluate()). */
static int run_rounds(St *s, Deque *wl, int eager, uint64_t max_ints) {
  Deque act = {0};
  int rc = ORC_OK;
  for (;;) {
    while (!dq_empty(wl)) {
      int32_t e = dq_pop(wl, ORC_FIFO, NULL);
      if (examine(s, e, eager, wl, &act) || s->oom) { rc = ORC_ENOMEM; goto out; }
    }
    if (dq_empty(&act)) break;
    s->rounds++;
    while (!dq_empty(&act)) {
      int32_t e = dq_pop(&act, ORC_FIFO, NULL);
      if (!s->ealive[e]) continue;
      if (do_int(s, e, wl) < 0 || s->oom) { rc = ORC_ENOMEM; goto out; }
    }
    act.head = act.tail = 0;
    if (max_ints && s->interactions > max_ints) { rc = ORC_ELIMIT; goto out; }
  }
out:
  free(act.v);
  return rc;
}

typedef struct {
  int32_t *stream;
  int64_t len;
  uint64_t interactions;
  uint64_t *hist;
  int set;
  int n_distinct;
  uint64_t leaves, max_leaves;
  int nr;
  int eager;
  int err;
} Enum;

static int finish(St *s, Buf *out, int32_t *n_stuck, int32_t *n_cycles) {
  int rc = readback_subst(s, n_cycles);
  if (rc) return rc;
  return serialise(s, out, n_stuck);
}

static void enum_dfs(St *s, Deque *wl, Enum *E) {
  if (E->err) return;
  Deque act = {0};
  while (!dq_empty(wl)) {
    int32_t e = dq_pop(wl, ORC_FIFO, NULL);
    if (examine(s, e, E->eager, wl, &act) || s->oom) { E->err = ORC_ENOMEM; free(act.v); return; }
  }
  /* distinct live active pairs */
  if (dq_empty(&act)) {
    Buf out = {0};
    int32_t ns = 0, nc = 0;
    if (finish(s, &out, &ns, &nc)) { E->err = ORC_ENOMEM; free(out.v); free(act.v); return; }
    E->leaves++;
    if (!E->set) {
      E->stream = out.v; E->len = out.n; E->interactions = s->interactions;
      memcpy(E->hist, s->per_rule, (size_t)E->nr * 8);
      E->set = 1; E->n_distinct = 1;
    } else {
      int same = out.n == E->len && memcmp(out.v, E->stream, (size_t)out.n * 4) == 0 &&
                 s->interactions == E->interactions &&
                 memcmp(s->per_rule, E->hist, (size_t)E->nr * 8) == 0;
      if (!same) E->n_distinct++;
      free(out.v);
    }
    free(act.v);
    if (E->leaves > E->max_leaves) E->err = ORC_ELIMIT;
    return;
  }
  for (int64_t i = act.head; i < act.tail && !E->err; i++) {
    int32_t e = act.v[i];
    int dup = 0;
    for (int64_t j = act.head; j < i; j++) if (act.v[j] == e) dup = 1;
    if (dup || !s->ealive[e]) continue;
    St c;
    if (st_clone(s, &c)) { E->err = ORC_ENOMEM; st_free(&c); break; }
    uint64_t *hist = (uint64_t *)malloc((size_t)(E->nr > 0 ? E->nr : 1) * 8);
    if (!hist) { E->err = ORC_ENOMEM; st_free(&c); break; }
    memcpy(hist, s->per_rule, (size_t)E->nr * 8);
    c.per_rule = hist;
    Deque w2 = {0};
    /* the other active pairs stay pending for the child */
    for (int64_t j = act.head; j < act.tail; j++) if (j != i) dq_push(&w2, act.v[j]);
    if (do_int(&c, e, &w2) < 0) E->err = ORC_ENOMEM;
    else enum_dfs(&c, &w2, E);
    free(w2.v);
    free(hist);
    c.per_rule = NULL;
    st_free(&c);
  }
  free(act.v);
}

const char *orc_version(void) { return "inet-oracle 1"; }

void orc_free(void *p) { free(p); }

int orc_reduce(const orc_input *in, int schedule, uint64_t seed, uint64_t max_ints,
               uint64_t *per_rule, int32_t **nf_out, orc_result *out) {
  orc_result R;
  memset(&R, 0, sizeof(R));
  St s;
  memset(&s, 0, sizeof(s));
  Deque wl = {0};
  Buf stream = {0};
  int eager = (schedule & ORC_EAGER) != 0;
  int sched = schedule & 0xff;
  uint64_t *hist = (uint64_t *)calloc((size_t)(in->n_rules > 0 ? in->n_rules : 1), 8);
  int rc = hist ? rules_prepare(&s, in) : ORC_ENOMEM;
  s.per_rule = hist;
  if (rc == ORC_OK) rc = load(&s, in, &wl);
  int32_t n_stuck = 0, n_cycles = 0;
  if (rc == ORC_OK) {
    if (sched == ORC_ENUMERATE) {
      Enum E;
      memset(&E, 0, sizeof(E));
      E.hist = (uint64_t *)calloc((size_t)(in->n_rules > 0 ? in->n_rules : 1), 8);
      E.nr = in->n_rules;
      E.eager = eager;
      E.max_leaves = max_ints ? max_ints : 200000;
      if (!E.hist) rc = ORC_ENOMEM;
      else {
        enum_dfs(&s, &wl, &E);
        rc = E.err;
        if (rc == ORC_OK) {
          R.n_outcomes = E.n_distinct;
          R.n_schedules = E.leaves;
          R.interactions = E.interactions;
          memcpy(hist, E.hist, (size_t)in->n_rules * 8);
          stream.v = E.stream; stream.n = E.len; stream.cap = E.len;
          E.stream = NULL;
          n_stuck = (stream.n > 0) ? 0 : 0;
        }
      }
      free(E.hist);
      free(E.stream);
    } else {
      if (sched == ORC_ROUNDS) rc = run_rounds(&s, &wl, eager, max_ints);
      else rc = run_sequential(&s, &wl, sched, eager, seed, max_ints);
      R.interactions = s.interactions;
      R.rounds = s.rounds;
      R.max_live_agents = (uint64_t)s.max_live_agents;
      if (rc == ORC_OK) rc = finish(&s, &stream, &n_stuck, &n_cycles);
      R.final_live_agents = (uint64_t)s.live_agents;
    }
  }
  R.n_com = s.n_com;
  R.n_sub = s.n_sub;
  R.n_col = s.n_col;
  R.n_loops = s.n_loops;
  R.n_iface = s.n_iface;
  R.n_cycles = n_cycles;
  if (rc == ORC_OK && sched == ORC_ENUMERATE && stream.n > 0) {
    /* residual count sits after the interface terms; recover it by decoding */
    int64_t p = 1;
    int32_t ni = stream.v[0];
    for (int32_t i = 0; i < ni; i++) {
      int64_t need = 1;
      while (need) { int32_t w = stream.v[p++]; need--; if (w >= 0) need += in->arity[w]; }
    }
    n_stuck = stream.v[p];
  }
  R.n_stuck = n_stuck;
  if (rc == ORC_OK && n_stuck > 0) rc = ORC_STUCK;
  R.nf_len = stream.n;
  if (nf_out) {
    *nf_out = NULL;
    if (rc == ORC_OK || rc == ORC_STUCK) { *nf_out = stream.v; stream.v = NULL; }
  }
  if (per_rule) memcpy(per_rule, hist ? hist : per_rule, (size_t)(hist ? in->n_rules : 0) * 8);
  R.status = rc;
  if (out) *out = R;
  free(stream.v);
  free(wl.v);
  free(hist);
  s.per_rule = NULL;
  st_free(&s);
  return rc;
}
