/*
 * inet.h -- C ABI of the MI355X evaluator for the lightweight interaction
 * calculus (Jiresch, "Towards a GPU-based implementation of interaction nets").
 *
 * The library reduces nets to normal form on one GPU.  The hot path is the
 * repeated parallel step of Section 3 (evaluate() in Section 3.6): apply the
 * rule of every active pair (int, Section 3.4), then resolve the name
 * equations that the right-hand sides produced (com, Section 3.5), until no
 * active pair remains.  sub and col are deferred to the read-back (Theorem 1,
 * Section 2.2).  All arithmetic is exact int32/uint64: results are bit-exact.
 *
 * ------------------------------------------------------------------------
 * Input format (host int32 arrays; the caller keeps ownership, every call
 * copies what it needs before returning).
 *
 *   term ref r:  r >= 0  agent r of the same net
 *                r <  0  name (-1 - r), a name id in [0, n_names)
 *   label[n_agents]       symbol of each agent, in [0, rules->n_symbols)
 *   port[n_agents][2]     refs on the auxiliary ports (entries at or past
 *                         the agent's arity are ignored).  An agent ref in a
 *                         port attaches that agent's principal port there,
 *                         i.e. the nested term alpha(.., beta(..), ..).
 *   eq_lhs[n_eqs], eq_rhs[n_eqs]   the multiset Delta of equations t = s
 *   A net is a configuration <t | Delta> (Section 2.2): every agent must be
 *   attached exactly once and below some equation side (finite terms), every
 *   name occurs at most twice in Delta; the names occurring once form the
 *   interface t, ordered by ascending id.
 *
 * Rule format (inet_rules): the rule alpha(x) = beta(y) -> Theta of Section
 * 2.2.  rule_lhs[k] = {alpha, beta}; rhs[rhs_off[k] .. rhs_off[k+1]) holds
 * n_eq followed by the n_eq equations of Theta, each side a prefix-encoded
 * term (a label >= 0 followed by its arity subterms, or a name -1-v).  Inside
 * a rule, names 0..ar(alpha)-1 are alpha's auxiliary ports, the next
 * ar(beta) names are beta's; each of these occurs exactly once in Theta, every
 * other name exactly twice (bound names, renamed apart at every use).  At most
 * one rule per unordered pair {alpha, beta}; alpha != beta; arity <= 2;
 * n_symbols <= INET_MAX_SYMBOLS; n_rules <= INET_MAX_RULES; after the library
 * folds the internal com/sub steps of Theta, a rule may create at most
 * INET_MAX_RHS_AGENTS agents, INET_MAX_RHS_EQS links and INET_MAX_RHS_FRESH
 * fresh names.
 *
 * Output: the canonical normal-form stream (inet_readback)
 *   [n_iface] T(iface_0) .. T(iface_n-1) [n_res] T(l_0) T(r_0) ..
 *   T(agent) = label followed by T of its auxiliary ports in order;
 *   T(name)  = -(1 + c), c numbered by first appearance in the stream.
 *   The residual equations are the active pairs that have no rule, each
 *   oriented so that its name-erased encoding is the smaller one first, and
 *   sorted by those encodings.  Closed loops x = x are dropped; a name cycle
 *   with no agent and no interface name (a vicious circle) is not part of the
 *   stream.
 *
 * Device memory: every handle lives in ONE caller-provided device buffer
 * (e.g. a torch uint8 tensor); size it with inet_workspace_bytes.  The
 * library never allocates device memory itself except small pinned host
 * staging areas (and the paper-pipeline ablation, inet_reduce_pipeline, which
 * allocates temporary device memory); the buffer must outlive the handle.
 *
 * Streams: the *_async entry points enqueue work on the caller's stream and
 * return at once; inet_results synchronises that stream.  A handle is not
 * thread-safe; calls on one handle must not overlap.
 *
 * Errors: every function returns an inet_status; no exception crosses the
 * ABI.  inet_strerror gives a static message.
 */
#ifndef INET_H
#define INET_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  INET_MAX_ARITY = 2,
  INET_MAX_SYMBOLS = 64,
  INET_MAX_RULES = 64,
  INET_MAX_RHS_AGENTS = 8,
  INET_MAX_RHS_EQS = 8,
  INET_MAX_RHS_FRESH = 8
};

typedef enum {
  INET_OK = 0,
  INET_STUCK = 1,    /* reduced; some active pair had no rule (a residual) */
  INET_EINVAL = -1,  /* malformed rules, net, argument or configuration     */
  INET_ENOMEM = -2,  /* agent/name/queue capacity or workspace too small;
                        the net's state is then unusable (reload it)        */
  INET_ELIMIT = -3,  /* max_steps reached before normal form; resumable     */
  INET_ERANGE = -4,  /* output buffer too small; *len holds the need        */
  INET_EAGAIN = -5,  /* server: no free slot or memory; retry later         */
  INET_EHIP = -6,    /* a HIP runtime call failed                            */
  INET_ENOSYS = -7,  /* not supported on this device / build                */
  INET_EINTERNAL = -8, /* an invariant of the evaluator was violated         */
  INET_ETIMEDOUT = -9  /* a workgroup of the multi-workgroup engine waited at
                          a barrier longer than the configured give-up without
                          progress (the net's state is then unusable)        */
} inet_status;

typedef struct {
  int32_t n_symbols;
  const int32_t *arity;     /* [n_symbols], each 0..2                       */
  int32_t n_rules;
  const int32_t *rule_lhs;  /* [n_rules][2]                                 */
  const int32_t *rhs_off;   /* [n_rules + 1]                                */
  const int32_t *rhs;       /* [rhs_off[n_rules]]                           */
} inet_rules;

typedef struct {
  int32_t status;           /* inet_status of this net                     */
  int32_t n_stuck;          /* residual active pairs without a rule        */
  uint64_t interactions;    /* int steps applied (order independent)       */
  uint64_t steps;           /* parallel steps run (schedule dependent)     */
  int64_t agents_used;      /* agent slots in use (heap top)               */
  int64_t names_used;       /* name cells in use                           */
  int32_t max_frontier;     /* largest set of active pairs in one step     */
  int32_t loops;            /* closed loops x = x dropped                   */
} inet_result;

/* Launch shape of the reduction kernel; 0 fields take the defaults. */
typedef struct {
  int32_t wg_size;          /* lanes per net engine: 64,128,256,512,1024;
                               0 takes 1024.  With engine 3 a wider engine
                               runs its first wave alone while the active
                               pairs fit one wave (no group barrier per
                               step) and all its waves once they do not   */
  int32_t jump;             /* 1: compress name chains after the loop      */
  int32_t max_resident;     /* cap on simultaneously resident net engines  */
  int32_t engine;           /* 0 default (3 when the run-time compiler can
                               build it, else 2); 1 per-lane rule-template
                               interpreter; 2 rule-uniform execution with
                               the templates read at run time; 3 the same
                               with the rule table compiled into the kernel
                               at load time (hipRTC); 4 engine 3 with the
                               atomic append of Section 4.2: each lane
                               reserves its agents, name cells and frontier
                               entries with atomics of its own (all waves
                               step together, at every frontier width)    */
  int32_t solo_max;         /* engine 3, wider engines: wave 0 steps alone
                               while at most this many pairs are active
                               (1..4096, 0: 64; a compile-time bound of the
                               load-time compiled engine, one code object
                               per value)                                  */
  int32_t grid;             /* a handle holding one net, engine 3: 0 the
                               multi-workgroup engine over one workgroup per
                               compute unit; > 0 over at most this many (and
                               at most one per compute unit); -1 one
                               workgroup only.  Workgroup 0
                               steps the net alone while at most grid_hi
                               pairs are active; above that the steps are
                               shared by ceil(active / grid_ppw) workgroups
                               until at most grid_lo are left               */
  int32_t grid_lo;          /* 0: 1024 */
  int32_t grid_hi;          /* 0: 2048 (at least grid_lo) */
  int32_t grid_ppw;         /* 0: the engine width */
  int32_t timeout_us;       /* multi-workgroup engine and pointer jumping of
                               one net: a workgroup waiting at a barrier gives
                               up after this many microseconds without
                               progress of the others (INET_ETIMEDOUT for the
                               engine; the jumping pass just ends early);
                               0: 2 s                                        */
  int32_t qcap;             /* engines 3 and 4: pairs per buffer of the LDS
                               frontier tile (a power of two, 64..8192; the
                               rest of a frontier lives in the net's global
                               queue); 0: by width, 512 for 64 lanes, 1024
                               for 128 and 256, 2048 for 512, 4096 for 1024 */
  int32_t round_scale;      /* serving loop (inet_server_step,
                               inet_server_run): a round's step budget is the
                               caller's round_steps times the number of
                               running nets per resident engine, rounded
                               down, at least 1 and at most round_scale; 0 or
                               1: round_steps.  Under load, when each engine
                               already steps several nets per round, longer
                               rounds cost few admissions but cut the rounds
                               a long net needs                             */
} inet_config;

typedef struct inet_net inet_net;

/* Workspace bytes for n_nets nets.  agent_cap[i] / name_cap[i]: capacity of
 * net i's agent heap and name cells (>= its initial size; 0 = a default of 4x
 * the initial size plus 1024; at most 2^28 - 16 agents and 2^29 - 16 names,
 * else INET_EINVAL).  n_eqs[i], n_agents[i], n_names[i]: initial sizes. */
int inet_workspace_bytes(const inet_rules *rules, int32_t n_nets, const int64_t *n_agents,
                         const int64_t *n_eqs, const int32_t *n_names, const int64_t *agent_cap,
                         const int64_t *name_cap, size_t *bytes);

/* Load one net (Section 2.2 configuration) and validate it (A1 of the hot
 * path).  dev/dev_bytes: the caller's device buffer (see above).  The upload
 * is enqueued on stream; on return the host arrays may be released. */
int inet_load(const inet_rules *rules, const int32_t *label, const int32_t *port,
              int32_t n_agents, const int32_t *eq_lhs, const int32_t *eq_rhs, int32_t n_eqs,
              int32_t n_names, int64_t agent_cap, int64_t name_cap, void *dev, size_t dev_bytes,
              hipStream_t stream, inet_net **out);

/* Load n_nets independent nets packed back to back: net i owns agents
 * [agent_off[i], agent_off[i+1]) and equations [eq_off[i], eq_off[i+1]) of the
 * packed arrays; refs inside a net are local to that net (agent r of net i is
 * packed row agent_off[i] + r).  agent_cap/name_cap as for
 * inet_workspace_bytes (may be NULL for defaults). */
int inet_batch_load(const inet_rules *rules, int32_t n_nets, const int32_t *label,
                    const int32_t *port, const int64_t *agent_off, const int32_t *eq_lhs,
                    const int32_t *eq_rhs, const int64_t *eq_off, const int32_t *n_names,
                    const int64_t *agent_cap, const int64_t *name_cap, void *dev,
                    size_t dev_bytes, hipStream_t stream, inet_net **out);

int inet_set_config(inet_net *h, const inet_config *cfg);
int inet_get_config(const inet_net *h, inet_config *cfg);

/* Order in which the persistent kernel hands nets to workgroups: a
 * permutation of [0, n_nets) (longest-running nets first balances a batch). */
int inet_set_order(inet_net *h, const int32_t *order);

/* Reduce every net of the handle to normal form (or until max_steps parallel
 * steps, 0 = no limit) with one persistent kernel launch on stream, then
 * compress name chains (pointer jumping).  Enqueue only; resumable after
 * INET_ELIMIT. */
int inet_reduce_async(inet_net *h, hipStream_t stream, uint64_t max_steps);

/* Synchronise stream and copy per-net results into out[n_nets]. */
int inet_results(inet_net *h, hipStream_t stream, inet_result *out);

/* inet_reduce_async + inet_results; returns the first net's status for a
 * single net, else INET_OK if all nets ended OK/STUCK, else the first error. */
int inet_reduce(inet_net *h, hipStream_t stream, uint64_t max_steps, inet_result *out);

/* Restore every net to its loaded state (device to device, on stream). */
int inet_reset(inet_net *h, hipStream_t stream);

/* One batched step captured as a HIP graph held by the handle: restore every
 * net (device to device), clear the net counter, the persistent reduction and
 * the pointer-jumping pass.  Capture runs on a private stream; the graph can
 * then be replayed on any stream with inet_graph_launch (results as after
 * inet_reduce_async).  Recapture after inet_set_config / inet_set_order. */
int inet_graph_capture(inet_net *h, uint64_t max_steps);
int inet_graph_launch(inet_net *h, hipStream_t stream);

/* Canonical normal-form stream of net i (the sub* col* read-back of Theorem
 * 1, Section 2.2).  Needs inet_results first.  cap too small: INET_ERANGE
 * with *len set to the required words. */
int inet_readback(inet_net *h, int32_t net, int32_t *buf, int64_t cap, int64_t *len);

/* Per-rule interaction counts of net i (cap >= n_rules words). */
int inet_per_rule(inet_net *h, int32_t net, uint64_t *counts, int32_t cap);

/* Opt-in diagnostic of the available parallelism (the active pairs per loop
 * iteration that Section 4.1 discusses): from the next reduction on, net
 * `net` writes the number of active pairs it reduces in parallel step s to
 * d_buf[s] (caller-owned device memory of cap int32, written on the device)
 * for every step s < cap; cap 0 turns it off.  A resumed reduction continues
 * at its step count.  The sum over a finished net's steps is its interaction
 * count plus its residual pairs. */
int inet_set_trace(inet_net *h, int32_t net, int32_t *d_buf, int64_t cap);

/* The raw name cells of a finished net (a diagnostic of the pointer-jumping
 * pass): cell x (0 <= x < names_used) holds EMPTY (0x7fffffff) while no
 * occurrence of name x has been extracted to the top of an equation, else
 * the term parked there (>= 0 an agent, < 0 the name -1 - value).  Needs
 * inet_results first; cap too small: INET_ERANGE with *len set. */
int inet_cells(inet_net *h, int32_t net, int32_t *buf, int64_t cap, int64_t *len);

/* Algorithmic bytes one interaction of each rule moves in the evaluator's
 * layout (cap >= n_rules words): 8 (the pair) + 4 (label + ports) of both
 * agents + 4 (label + ports) of each new agent + 4 per fresh name cell + 8 per
 * link equation (a name-cell exchange or a frontier append). */
int inet_rule_bytes(const inet_net *h, int32_t *bytes, int32_t cap);

/* Host only (no device needed): validate and compile a rule table and report,
 * per rule, the agents it creates, the fresh name cells (wires) and link
 * equations left after folding the internal com/sub steps of its right-hand
 * side, and its algorithmic bytes (as inet_rule_bytes).  Each output array
 * may be NULL; otherwise it holds cap >= n_rules words. */
int inet_rules_check(const inet_rules *rules, int32_t *n_new, int32_t *n_fresh, int32_t *n_links,
                     int32_t *bytes, int32_t cap);

/* Host only: build the engines specialised for this rule table (engines 3
 * and 4, 1024 lanes; engine 3 with its multi-workgroup engine) for the given
 * device architecture (e.g. "gfx950") with the run-time compiler, without a
 * device; *code_bytes gets the total size of the two code objects, log (may be
 * NULL) the compiler's messages.  INET_ENOSYS if the compiler fails.  On a
 * device the same code objects are built on first use, one per rule table,
 * engine and engine width. */
int inet_jit_build(const inet_rules *rules, const char *arch, size_t *code_bytes, char *log,
                   size_t log_cap);

int32_t inet_num_nets(const inet_net *h);
void inet_free(inet_net *h);
const char *inet_strerror(int status);

/* Kernel time of the last reduction launch on this handle, measured with HIP
 * events on the launch stream (ms); -1 if not available yet. */
float inet_last_kernel_ms(inet_net *h);

/* The paper's own evaluation loop (Sections 3.3-3.6), kept as an ablation to
 * compare the net engines against, on the same nets and GPU: a list of
 * equations; each iteration applies int to every active pair with a fixed
 * number of output slots per equation (dummies where the rule leaves fewer),
 * removes the dummies, then applies com by sorting the equations with a name
 * side by that name and merging neighbours that share it; it repeats while an
 * int or a com happened (host-driven, one synchronisation per iteration).
 * Runs every net of the handle in turn on `stream` and leaves the results as
 * inet_reduce does (read them with inet_results, inet_readback,
 * inet_per_rule); `steps` then counts iterations of the loop.  The nets must
 * be in their loaded state (after loading or inet_reset).  max_iterations 0
 * means no limit; a net stopped by it reports INET_ELIMIT and cannot be
 * resumed.  Unlike every other entry point it allocates temporary device
 * memory (hipMalloc) for its equation lists. */
int inet_reduce_pipeline(inet_net *h, hipStream_t stream, uint64_t max_iterations);

/* The ablation's device primitives (Sections 3.4-3.5: the scan of the
 * allocation, the removal of dummies, the sort of the equations by variable
 * and the merge of communication-eligible neighbours), on caller device
 * arrays.  Each allocates temporary device memory, runs on `stream` and
 * synchronises it before returning.
 *   inet_prim_scan: out[i] = in[0] + ... + in[i] (uint64, wrapping).
 *   inet_prim_select: the elements of in that differ from `drop`, in their
 *     order, into out; *n_out (host) gets their number.
 *   inet_prim_sort_pairs: (key, value) pairs sorted by key ascending, stably,
 *     in place.
 *   inet_prim_reduce_by_key: each run of equal adjacent keys becomes one
 *     (key, value), the run's values folded left to right with op: 0 sum
 *     (the example of Section 3.5), 1 the merge of two equations sharing a
 *     variable, (x, t) and (x, s) give (s, t), an equation packed as
 *     lhs | rhs << 32; *n_out (host) gets the number of runs.
 * n < 0, null pointers with n > 0, or an unknown op: INET_EINVAL. */
int inet_prim_scan(const uint64_t *d_in, uint64_t *d_out, int64_t n, hipStream_t stream);
int inet_prim_select(const uint64_t *d_in, uint64_t *d_out, int64_t n, uint64_t drop,
                     int64_t *n_out, hipStream_t stream);
int inet_prim_sort_pairs(uint32_t *d_keys, uint64_t *d_vals, int64_t n, hipStream_t stream);
int inet_prim_reduce_by_key(const uint32_t *d_keys, const uint64_t *d_vals, int64_t n,
                            uint32_t *d_keys_out, uint64_t *d_vals_out, int32_t op,
                            int64_t *n_out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): load,
 * reduce and read back one net like inet_load + inet_reduce + inet_readback,
 * but with every device array the kernels need (rule table, descriptor,
 * state, agent heap, name cells, queues, residuals, initial image, counters)
 * carved out of a static device array of INET_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device until the process ends; no hipMalloc,
 * hipFree or run-time compilation happens (the ahead-of-time engine 2 runs,
 * 1024 lanes, one workgroup, then the pointer-jumping pass).  Inputs are the
 * host arrays of inet_load (copied on `stream`), capacities as there; a net
 * whose workspace (inet_workspace_bytes) exceeds the array gives INET_ENOMEM
 * before anything runs.  max_steps as for inet_reduce.  Outputs: *out, and
 * when nf_len is not NULL the canonical normal-form stream into nf (nf_cap
 * int32 words; INET_ERANGE with *nf_len set if it does not fit).  Returns
 * the net's status.  The call synchronises `stream`.  Every call on a device
 * shares that device's array and overwrites what the previous call left;
 * calls that overlap on one device race (serialise them). */
#define INET_NOALLOC_SCRATCH_BYTES (64ull << 20)
int inet_reduce_noalloc(const inet_rules *rules, const int32_t *label, const int32_t *port,
                        int32_t n_agents, const int32_t *eq_lhs, const int32_t *eq_rhs,
                        int32_t n_eqs, int32_t n_names, int64_t agent_cap, int64_t name_cap,
                        uint64_t max_steps, hipStream_t stream, inet_result *out, int32_t *nf,
                        int64_t nf_cap, int64_t *nf_len);

/* ------------------------------------------------------------------------
 * Continuous batching (serving).  A server owns one caller-provided device
 * buffer and up to max_slots resident nets.  inet_server_submit admits a net
 * when a slot and a free byte range of its workspace are available (else
 * INET_EAGAIN: admission is by free device bytes), uploads it on `stream`
 * and makes it part of the next round.  inet_server_step launches one round:
 * every running net advances by at most max_steps parallel steps, keeping its
 * heap and frontier resident between rounds.  inet_server_poll waits for the
 * round on `stream` and reports the tickets of nets that finished (normal
 * form, or an error such as INET_ENOMEM); their results stay readable until
 * inet_server_release returns the slot and memory.  Calls on one server must
 * not overlap. */
typedef struct inet_server inet_server;
int inet_server_create(const inet_rules *rules, int32_t max_slots, void *dev, size_t dev_bytes,
                       inet_server **out);
int inet_server_set_config(inet_server *s, const inet_config *cfg);
/* device bytes one admitted net occupies (caps as for inet_workspace_bytes) */
int inet_server_net_bytes(const inet_server *s, int32_t n_agents, int32_t n_eqs, int32_t n_names,
                          int64_t agent_cap, int64_t name_cap, int64_t *bytes);
int inet_server_submit(inet_server *s, const int32_t *label, const int32_t *port, int32_t n_agents,
                       const int32_t *eq_lhs, const int32_t *eq_rhs, int32_t n_eqs, int32_t n_names,
                       int64_t agent_cap, int64_t name_cap, hipStream_t stream, int64_t *ticket);
int inet_server_step(inet_server *s, hipStream_t stream, uint32_t max_steps);
int inet_server_poll(inet_server *s, hipStream_t stream, int64_t *done, int32_t cap,
                     int32_t *n_done);
/* result of a finished net; buf/len as for inet_readback (len NULL: counters only) */
int inet_server_result(inet_server *s, int64_t ticket, inet_result *res, int32_t *buf, int64_t cap,
                       int64_t *len);
int inet_server_per_rule(inet_server *s, int64_t ticket, uint64_t *counts, int32_t cap);
int inet_server_release(inet_server *s, int64_t ticket);
int inet_server_stats(const inet_server *s, int64_t *free_bytes, int32_t *free_slots,
                      int32_t *running);
/* The serving loop run natively (no interpreter between rounds).  Requests
 * come from a pool packed as for inet_batch_load (net j: agents
 * [agent_off[j], agent_off[j+1]), equations [eq_off[j], eq_off[j+1]),
 * n_names[j] names, capacities agent_cap[j] / name_cap[j], either array NULL
 * for the defaults); the pool is validated and uploaded once into the
 * server's buffer for the duration of the call.  Request i is pool net
 * pick[i] arriving arrival_s[i] seconds after the call starts (non-decreasing).
 * Each round admits the requests that have arrived while a slot and device
 * bytes are free, installs all of them with one copy and one kernel launch on
 * `stream`, advances every running net by at most round_steps parallel steps
 * and harvests the nets that finished; requests arriving during a round are
 * admitted for the next one.  A request that runs out of capacity is admitted
 * again with 8x its capacities (up to 4096x).  Per request the call writes its
 * completion time (seconds since the start), status, interaction count and
 * steps.  The server must be idle (no admitted nets).  INET_ELIMIT when
 * time_limit_s passes, INET_ENOMEM when a request cannot be admitted into an
 * empty server.
 *
 * `capture` (NULL: none) asks for more per request, all caller-owned host
 * memory: per_rule[i * n_rules + r] = interactions of rule r of request i
 * (copied back with the net states every round); and, for each request with
 * want_nf[i] != 0, its canonical normal-form stream (as inet_readback writes
 * it), read back when the request finishes, before its slot is reused.  The
 * streams are written back to back into nf_buf (nf_cap int32 words) in
 * completion order: request i's occupies nf_buf[nf_pos[i] .. nf_pos[i] +
 * nf_len[i]).  Requests not flagged, or that failed, get nf_pos -1 and
 * nf_len 0.  A stream that does not fit gets nf_pos -1 and nf_len its length,
 * the run goes on, and the call returns INET_ERANGE at the end (all other
 * outputs are written).  Reading streams back costs a device-to-host copy of
 * the net's heap each, inside the loop: it is meant for checking, not for
 * timing. */
typedef struct {
  int64_t rounds;
  int32_t max_resident;
  int32_t retries;
  double wall_s;
} inet_serve_stats;
typedef struct {
  uint64_t *per_rule;     /* [n_req][n_rules], or NULL */
  const uint8_t *want_nf; /* [n_req], or NULL: no normal forms */
  int32_t *nf_buf;        /* nf_cap words */
  int64_t nf_cap;
  int64_t *nf_pos;        /* [n_req] (required with want_nf) */
  int64_t *nf_len;        /* [n_req] (required with want_nf) */
} inet_serve_capture;
int inet_server_run(inet_server *s, int32_t n_pool, const int32_t *label, const int32_t *port,
                    const int64_t *agent_off, const int32_t *eq_lhs, const int32_t *eq_rhs,
                    const int64_t *eq_off, const int32_t *n_names, const int64_t *agent_cap,
                    const int64_t *name_cap, int64_t n_req, const double *arrival_s,
                    const int32_t *pick, uint32_t round_steps, double time_limit_s,
                    hipStream_t stream, double *done_s, int32_t *status, uint64_t *interactions,
                    uint32_t *steps, inet_serve_stats *stats, const inet_serve_capture *capture);
void inet_server_free(inet_server *s);

#ifdef __cplusplus
}
#endif
#endif
