// trs_layout.h -- device data layout shared by the library's host runtime and
// its HIP kernels (not part of the public ABI).
//
// Node pool: structure of arrays indexed by slot (Section 3's arrays):
//   hss[N]      int32  head symbol of the term stored at the slot
//   args[N*A]   int32  argument slots, maxarity-strided (slot s owns
//                      args[s*A .. s*A+A)); entries past the arity of hss[s]
//                      are unspecified.  Slot 0 is never used, as in the paper.
//   state[N]    uint8  replaces the paper's nf / nf_read pair (see below)
//   rc[N]       int32  reference count (the paper's refcounts)
//   fstack[2][N] int32 two free-index stacks (the paper's free_indices); round
//                      r pops stack r&1 and pushes stack (r+1)&1
//   dead[2][N]  int32  nodes whose count reached zero in round r go to list
//                      r&1 and are collected in round r+1
//
// State byte.  A node that becomes a normal form, or is created, in round r
// must not be seen as such by other nodes until round r+1 (the paper keeps a
// read copy nf_read of nf for this, Section 3).  Instead of copying, the
// marker carries the parity of the round that set it:
//   0x00          free (or never used)
//   0x01 | m<<3   live, not in normal form           (ACTIVE); m = memo
//   0x03 | e<<2   live, created in a round of parity e (ACTIVE|PEND)
//   0x80          live, normal form                  (NF)
//   0x82 | e<<2   live, became normal form in a round of parity e (NF|PEND)
// A marker with the current parity is "not yet"; with the other parity it is
// already valid, and is rewritten to the plain state in the next round (by
// the slot's own sweep, or from the retire list when only a frontier is
// swept), so markers never outlive two rounds.  The memo m (bits 3-5) is the
// paper's "last subterm checked": 1 + the index of the argument that was not
// yet a normal form when the node was last examined, so a still-blocked node
// costs one argument read and one state read.
#pragma once
#include <stdint.h>

#define ST_FREE 0x00u
#define ST_ACTIVE 0x01u
#define ST_PEND 0x02u
#define ST_EPOCH 0x04u
#define ST_NF 0x80u
#define ST_MEMO_SHIFT 3
#define ST_MEMO_MASK 0x38u

// ---------------------------------------------------------------- tables
// Compiled rule tables (int32 words), loaded into LDS by every workgroup.
//   [0] n_sym  [1] n_rules  [2] A  [3] total words
//   [TAB_SYM + f]                       symbol word: arity | deep<<3 | nrules<<8 |
//                                       first<<16 (deep: bit j set when some
//                                       rule of f has a pattern below its
//                                       argument j)
//   [TAB_SYM + n_sym + r]               word offset of rule r's program
// Rule program at offset p:
//   p+0  npat | nnew<<4 | var_root<<8 | root_nf<<9 | root_ready<<10 | npos<<12 |
//        nneg<<16 | rootpat<<20
//   p+1  root symbol (non-variable right-hand side) or -1
//   p+2  offset of the root operand list      (ar(root) operand words)
//   p+3  offset of the new-node list          (per node: header, operands)
//   p+4  offset of the reference-count deltas (npos positive, then nneg negative)
//   p+5  rule index (textual order, for the per-rule counters)
//   p+6 .. p+5+npat   pattern nodes 1..npat in prefix order:
//                     parent | pos<<4 | is_var<<8 | sym<<16
// Operand word: k >= 0 -> the slot matched by pattern node k (k >= 1);
//               k <  0 -> the slot of new node (-1-k).
// New-node header: sym | rc_init<<16 (6 bits) | born_nf<<22 | ready<<23 | referrer<<24
// (referrer: 0 = the root, j+1 = new node j; the parent hint of the node).
// born_nf: a constructor over normal forms; ready: not born_nf and all its
// arguments are normal forms at birth (queued for the next round).
// Delta word: pattern node | (delta & 0xff)<<8 (signed 8-bit delta).
#define TAB_SYM 4
#define TAB_MAX_WORDS 4096
// Learned mode appends the predictor's decision table to the rule tables
// (both are copied into LDS together): bit ((sym*32 + c)*16 + bucket), c the
// 5-bit mask of arguments in normal form (set for positions >= arity) and
// bucket the age bucket, is 1 when the node is kept.  n_sym*16 words.
#define TAB_GATE_MAX_WORDS 4096

static inline int32_t tab_sym_word(int32_t arity, int32_t nrules, int32_t first, int32_t deep) {
  return arity | (deep << 3) | (nrules << 8) | (first << 16);
}
#define SYM_ARITY(w) ((w) & 7)
#define SYM_DEEP(w) (((w) >> 3) & 31)

// ---------------------------------------------------------------- control
#define CTL_SPREAD 64    // statistics counters are spread over this many words
#define RULE_SPREAD 16   // per-rule counters are spread over this many copies
#define TICKET_GROUPS 64
#define CTL_NSTAT 13
enum {
  STAT_ACTIVE = 0,  // live non-normal-form slots visited
  STAT_READY,       // of those, all arguments in normal form
  STAT_FIRED,       // rule applications
  STAT_NFSET,       // became normal form without a rule (no match / no rules)
  STAT_ALLOC,       // nodes created
  STAT_FREED,       // nodes collected
  STAT_VISITS,      // slots examined
  STAT_MLP,         // predictor evaluations
  STAT_RCOPS,       // reference-count atomics (rewrite and collection)
  STAT_MEMO,        // active slots found still blocked by their memo argument
  STAT_KEEP,        // predictor decisions that kept the node
  STAT_TRACE,       // trace records logged (including ones past the cap)
  STAT_WALK,        // constructors marked normal forms by a walk up the
                    // parent hints in the round their last argument did
};

// Each counter on a 128-byte line of its own: atomics to one line
// serialise, and every workgroup of a launch updates several of them.
#define RC_PAD(name) int32_t name##_pad[31]
struct RoundCnt {
  int32_t alloc;   // allocation claims in the round
  RC_PAD(alloc);
  int32_t push;    // free-stack pushes in the round
  RC_PAD(push);
  int32_t dead;    // dead-list appends in the round
  RC_PAD(dead);
  int32_t active;  // nonzero if a live non-normal-form slot was seen
  RC_PAD(active);
  int32_t err;     // nonzero: trs_status of a device-detected error
  RC_PAD(err);
  int32_t front;   // appends to the next round's frontier
  RC_PAD(front);
  int32_t ret;     // appends to the retire list
  RC_PAD(ret);
  int32_t full;    // the round examined every slot (full sweep)
  RC_PAD(full);
  int32_t prog;    // a node fired or became a normal form in the round
  RC_PAD(prog);
  int32_t scan;    // plain mode: slots the round's scan listed for examination
  RC_PAD(scan);
};

struct Ctl {
  int32_t done;        // set once the fixpoint (and collection) is reached
  int32_t done_round;  // number of rounds executed
  int32_t err;         // copied from the round counters when done
  int32_t n_final;     // slot extent at the end
  int32_t n[3];        // slot extent n at the start of round r (index r % 3)
  int32_t fs[3][2];    // free-stack sizes at the start of round r
  int32_t peak_n;
  int32_t gc_rounds;
  int32_t next_need;   // workgroups the next launch's first round uses
  int32_t r_cur;       // next round to execute (advanced by the last workgroup)
  int32_t abort;       // set when a device-wide barrier wait timed out
  int32_t stamp_base;  // frontier-notification stamps of this run start here
  int32_t full_sweeps; // rounds that swept every slot
  int32_t r_reached;   // round after the last one workgroup 0 ran alone
  int32_t fs_final[2]; // free-stack sizes when the run ended
  int32_t last_prog;   // last round in which a node fired or became a normal form
  int32_t pad2;
  alignas(128) RoundCnt cnt[3];  // counters accumulated during round r (index r % 3)
  // state of the next launch's first round, published by the last workgroup
  // of a launch (the host writes it for round 0): done, r, need, n, fs0, fs1,
  // dead, frontier, retire, flags (stop | quiescent<<1 | stall<<2 |
  // scanned<<3 | scan requested<<4 | err<<8), and (set by the host, read
  // with the rest) the run's first frontier-notification stamp
  alignas(64) int32_t pub[16];
  // statistics, spread-major: the counters of one workgroup share cache
  // lines, those of workgroups with different wg mod CTL_SPREAD do not, so
  // a launch's end-of-launch atomics contend little on any one line
  unsigned long long stat[CTL_SPREAD][CTL_NSTAT];
  unsigned long long rule_apps[RULE_SPREAD][256];
  // end-of-launch tickets in two levels (a counter per group of workgroups,
  // then one for the groups), each counter on a 128-byte line of its own:
  // same-address atomics serialise, and a single counter cost about 50 ns
  // per workgroup
  // (64-bit: workgroups in bits 0-31, and the numbers of them that met a
  // live non-normal-form slot (bits 32-47) and made progress (48-63), so
  // the last one knows the round's two flags without a store per workgroup)
  unsigned long long tickets[TICKET_GROUPS + 1][16];
  // plain-mode scan: per list (up to 16, each on a 128-byte line of its
  // own) the slots listed and whether a live non-normal-form slot was met;
  // read by the round kernel that follows, cleared by its last workgroup
  int32_t scan_cnt[16][32];
};

struct Pool {
  int32_t *hss;
  int32_t *args;
  uint8_t *state;
  int32_t *rc;
  int32_t *fstack0, *fstack1;
  int32_t *dead0, *dead1;
  // frontier modes
  int32_t *par;             // parent hint: the slot that referenced the node
                            // when it was created (0 for term roots)
  int32_t *front0, *front1; // frontier of the next round (round r appends to r&1)
  int32_t *ret0, *ret1;     // markers set in round r to retire in round r+1
  int32_t *qstamp;          // last notification stamp (deduplicates appends)
  // plain mode: wake bits, two per slot (slot s: word s / 16, bit
  // 2 (s mod 16) + p; bit p set: an argument of the node became a normal
  // form in a round of parity p since the node was last examined)
  uint32_t *wake;
  // learned mode and tracing
  int32_t *lastchg;         // round in which the node was created or last changed
  int64_t *tref;            // tracing: record index << 32 | round of the
                            // node's latest trace record
  int64_t N;
};
