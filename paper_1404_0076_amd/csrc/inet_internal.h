// inet_internal.h -- device data layout shared by the host runtime and the
// HIP kernels of the evaluator (not part of the public ABI).
//
// A net lives in its own region of the caller's device buffer:
//   agent[agent_cap][4]   agent heap: one 16-byte record {label, port0, port1,
//                         unused} per slot, so that a pair's two agents are
//                         two 16-byte loads
//   bind[name_cap]                                        one cell per name
//   queue[2][qcap]    frontier double buffer: entries >= LDS capacity of the
//                     running engine spill here; the saved frontier lives here
//                     between launches; the initial equations start here
//   stuck[scap]       active pairs without a rule
//   per_rule[n_rules] uint64 interaction counts
// A term ref is int32: r >= 0 agent slot, r < 0 name (-1 - r) = ~r.
// A name cell holds EMPTY until one occurrence of the name has been extracted
// to the top of an equation; it then holds the term on the other side of that
// equation (the parked value); the second extraction takes the value and
// forms the equation value = other (com).
#ifndef INET_INTERNAL_H
#define INET_INTERNAL_H

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
typedef int int32_t;
typedef unsigned int uint32_t;
typedef long long int64_t;
typedef unsigned long long uint64_t;
#endif

namespace inet {

constexpr int32_t EMPTY = 0x7fffffff;
constexpr int MAXRULES = 64;  // rule table limit (INET_MAX_RULES)
enum { FLAG_JUMP = 1 };      // kernel flag: compress name chains after the loop

// compiled rule template (int32 words)
constexpr int RT_WORDS = 48;
constexpr int RT_NNEW = 0;    // agents created by the rule
constexpr int RT_NALLOC = 1;  // agents needing a fresh slot (the first two reuse the pair's slots)
constexpr int RT_NFRESH = 2;  // fresh name cells (wires between two new ports)
constexpr int RT_NEQ = 3;     // link equations
constexpr int RT_LABEL = 4;   // [8] labels of the new agents
constexpr int RT_PORT = 12;   // [8][2] operands on the new agents' ports
constexpr int RT_EQ = 28;     // [8][2] operands of the link equations
constexpr int MAXNEW = 8, MAXEQ = 8, MAXFRESH = 8;

// operand code: kind << 4 | index
constexpr int OP_AUX = 0;    // index 0,1: first agent's ports; 2,3: second agent's ports
constexpr int OP_NEW = 1;    // index k: new agent k
constexpr int OP_FRESH = 2;  // index f: fresh name f
constexpr int OP_NONE = 0xff;

// net state, written by the kernels, read by the host (64 bytes)
struct NetState {
  unsigned long long interactions;
  uint32_t steps;
  int32_t status;
  int32_t agent_top;
  int32_t name_top;
  int32_t frontier;      // entries of the saved frontier / initial equations
  int32_t phase;         // 0: initial equations pending, 1: frontier saved, 2: done
  int32_t parity;        // which queue buffer holds the saved frontier
  int32_t n_stuck;
  int32_t loops;
  int32_t max_frontier;
  int32_t pad[4];
};

enum { PHASE_INIT = 0, PHASE_RUN = 1, PHASE_DONE = 2 };

// per-net descriptor (read-only for the kernels)
struct NetDesc {
  int32_t *agent;  // [agent_cap][4]: label, port 0, port 1, unused (16-byte records)
  int32_t *bind;
  unsigned long long *queue0;  // pairs as 64-bit words, x in the low half
  unsigned long long *queue1;
  unsigned long long *stuck;
  unsigned long long *per_rule;
  NetState *st;
  // initial image (for reset): label[n], port[n][2], equations[n_eqs][2]
  const int32_t *init_label;
  const int32_t *init_port;
  const int32_t *init_eq;
  int32_t agent_cap;
  int32_t name_cap;
  int32_t qcap;
  int32_t scap;
  int32_t n_agents0;
  int32_t n_eqs0;
  int32_t n_names0;
  int32_t order;  // position in the launch order (largest nets first)
  // opt-in diagnostic: active pairs reduced in each parallel step (trace[s]
  // for steps s < trace_cap), or null
  int32_t *trace;
  int32_t trace_cap;
  int32_t pad_;
};

// a net admitted by the serving loop: its descriptor and the slot it takes
struct AdmitRec {
  NetDesc desc;
  int32_t slot;
  int32_t pad;
};

// status codes as seen by the kernels (mirror inet_status)
enum { ST_OK = 0, ST_STUCK = 1, ST_ENOMEM = -2, ST_ELIMIT = -3, ST_EINTERNAL = -8,
       ST_ETIMEDOUT = -9 };

// Control block of the multi-workgroup engine of one net (global memory,
// cleared before each launch).  The launch runs in epochs: in a NARROW epoch
// workgroup 0 steps the net alone; in a GRID epoch the g workgroups of lowest
// logical index share one parallel step.  An epoch ends when every workgroup
// has posted its entry for it (epoch number, error bit, new active pairs);
// each workgroup then reads all entries and takes the same decision about the
// next epoch, so no workgroup has to publish it.  The entries alternate
// between two arrays by epoch parity: no workgroup can be two epochs ahead of
// another, since every workgroup posts in every epoch.  Each group of scalar
// words sits on its own 128-byte line; the pointer-jumping pass uses the
// arrive / gen barrier.
enum { GM_NARROW = 0, GM_GRID = 1, GM_DONE = 2 };
constexpr int kGridMax = 2048;  // workgroups of one multi-workgroup launch, at most
struct GridCtl {
  int32_t arrive;  // pointer jumping: arrivals in the current round
  int32_t pad0[31];
  int32_t gen;        // pointer jumping: round counter
  int32_t heartbeat;  // bumped by workgroup 0 while it steps alone
  int32_t pad1[30];
  uint32_t stop;     // step budget end (absolute), written by workgroup 0
  int32_t moved[2];  // pointer jumping: a cell moved in round r (moved[r & 1])
  int32_t gave_up;   // a workgroup gave up waiting (sticky)
  int32_t pad2[28];
  unsigned long long next;  // frontier entries appended by all GRID steps so far
  int32_t pad3[30];
  // per epoch parity and workgroup: (epoch << 32) | (error << 31) | new pairs
  unsigned long long ent[2][kGridMax];
};

// tunables of the reduction kernel (by value)
struct KParams {
  GridCtl *ctl;         // multi-workgroup engine: its control block (else null)
  int32_t grid_lo;      // multi-workgroup steps while more than this many are active
  int32_t grid_hi;      // workgroup 0 hands over once more than this many are active
  int32_t grid_ppw;     // target active pairs per workgroup in a multi-workgroup step
  uint64_t timeout;     // give-up of a barrier wait without progress, wall-clock ticks
};

}  // namespace inet

#endif
