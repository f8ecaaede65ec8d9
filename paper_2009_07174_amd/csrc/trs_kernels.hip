// trs_kernels.hip -- gfx950 kernels of the round-synchronous innermost rewriter.
//
// One round (Section 3, the derive and collect_free_indices kernels, merged
// into one pass and re-designed for CDNA4):
//
//   1. Collection: nodes whose reference count reached zero in the previous
//      round (the dead list) drop one reference to each argument (newly dead
//      arguments go to this round's dead list), are marked free and are
//      pushed on the free stack that the next round allocates from.  This is
//      the paper's garbage collection with free-index reuse, driven by a list
//      instead of a sweep of all reference counts.
//   2. Examination: in a full round every slot below n is examined (the
//      topology-driven sweep of Section 3): a workgroup streams a tile of
//      state bytes with vector loads, retires round markers, and compacts the
//      live non-normal-form slots into an LDS work list.  In a frontier round
//      only the slots queued by the previous round are examined.
//   3. Rewrite: a slot whose arguments are all normal forms is matched
//      against the rules of its head symbol in priority order (Section 2,
//      rewrite_f) using the compiled per-symbol tables held in LDS; the first
//      match is contracted in place (Section 3): the right-hand-side root
//      overwrites the slot, new subterms go to slots taken from the free
//      stack or past n, and reference counts are adjusted, increments before
//      decrements.  A slot with no applicable rule becomes a normal form.
//
// Frontier modes add a data-driven queue to the topology-driven sweep (the
// paper chose the sweep because thousands of threads contending on a queue
// was the bottleneck on its GPU; here every append is aggregated per
// workgroup).  A node is queued for the next round when it is created or
// rewritten with all arguments already normal forms, or when one of its
// arguments becomes a normal form (through the parent hint of that argument).
// A round with an empty queue is a full sweep, and only a full sweep that
// finds no live non-normal-form slot ends the run, so the method's own test
// stays the judge of the result.
//
// Allocation takes one atomic per workgroup pass: a wave-level prefix sum of
// the per-lane node counts, then a workgroup scan of the wave totals, then a
// single fetch-add on the round's claim counter.  Claims below the free-stack
// size map to recycled slots, the rest to fresh slots n, n+1, ... (the
// paper's get_new_index with next_free_begin / next_fresh, without per-thread
// atomics).  Dead-list, frontier and retire-list appends are buffered in LDS
// and flushed with one atomic per list per pass.
//
// Round-to-round state lives in the device control block, triple-buffered by
// round (r % 3), so consecutive rounds need no host involvement and the
// persistent form needs a single device-wide barrier per round.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "trs_kernels.h"

#define MAXPAT 8
#define MAXNEW 8

namespace {

__device__ __forceinline__ int lane() { return __lane_id(); }

// coherent read of a control word written by other workgroups or kernels
__device__ __forceinline__ int ld(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Store of a control word that another workgroup of the same launch reads
// (with ld): an agent-scope store is coherent with agent-scope loads and
// fetch-adds on every XCD, where a plain store could stay in this XCD's L2.
__device__ __forceinline__ void st(int32_t *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// End-of-launch ticket (thread 0 of each of the gt workgroups that take
// one): true for the workgroup that finishes last.  Two levels: a counter
// per group of workgroups (wg mod ng), then one for the groups, with ng about
// the square root of gt, so no counter takes more than about 2 sqrt(gt)
// same-address atomics.  Each counter is reset by the one that completes
// it.  flags (bit 0: met a live non-normal-form slot, bit 1: made progress)
// travel up with the tickets; the last workgroup gets in *flags whether any
// workgroup set each.  The caller has waited for its own memory operations
// first.
__device__ __forceinline__ bool last_ticket(Ctl *ctl, int wg, int gt, int *flags) {
  // up to 32 workgroups: one level (a second fetch-add would cost a
  // dependent round trip, more than 32 same-address ones)
  int ng = 1;
  if (gt > 32)
    while (ng * ng < gt && ng < TICKET_GROUPS) ng <<= 1;
  const int g = wg & (ng - 1);
  const int gsize = (gt - g + ng - 1) / ng;  // workgroups w < gt with w mod ng = g
  auto enc = [](int f) {
    return 1ull | ((unsigned long long)(f & 1) << 32) | ((unsigned long long)((f >> 1) & 1) << 48);
  };
  auto dec = [](unsigned long long v) {
    return (((v >> 32) & 0xffff) ? 1 : 0) | ((v >> 48) ? 2 : 0);
  };
  unsigned long long *c1 = &ctl->tickets[g][0];
  const unsigned long long a1 = enc(*flags);
  const unsigned long long v1 = atomicAdd(c1, a1) + a1;
  if ((int)(v1 & 0xffffffffu) != gsize) return false;
  __hip_atomic_store(c1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ng == 1) {
    *flags = dec(v1);
    return true;
  }
  unsigned long long *c2 = &ctl->tickets[TICKET_GROUPS][0];
  const unsigned long long a2 = enc(dec(v1));
  const unsigned long long v2 = atomicAdd(c2, a2) + a2;
  if ((int)(v2 & 0xffffffffu) != min(ng, gt)) return false;
  __hip_atomic_store(c2, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *flags = dec(v2);
  return true;
}

// Workgroup barrier for LDS traffic only: each wave waits for its own LDS
// operations, not for its global stores and atomics.  Within a round no wave
// reads what another wave of its workgroup wrote to global memory (the
// method tolerates either value there, as it must for other workgroups), so
// the barriers inside a round need not wait for write acknowledgements; the
// full barrier (__syncthreads) is kept where a round ends.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 32-bit integer hash (multiply / xor-shift), used to sample trace records
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// sum over the active lanes of a wave (device-library reduction)
__device__ __forceinline__ int wave_sum(int x) { return __ockl_wfred_add_i32(x); }

// Wave-aggregated reservation on a counter: lanes with pred get distinct
// positions (others -1) and the wave issues a single atomic, where lanes
// adding to one LDS address one by one would be serialised.  Must be called
// by all 64 lanes of the wave (the masks come from ballots of pred, never
// from the set of active lanes).
__device__ __forceinline__ int wave_reserve(bool pred, int32_t *ctr) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return -1;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane() == leader) base = atomicAdd(ctr, __popcll(m));
  base = __shfl(base, leader, 64);
  return pred ? base + __popcll(m & __lanemask_lt()) : -1;
}

// The lanes of the wave that execute this call (the active lanes) and add
// the same delta d to the same count t are combined: the first of them gets
// their number, the others 0; a lane that differs from the first gets 1.
// The firings of one rule in a round on redexes that share a variable's
// binding (a subterm shared by every node of a level, as in a tree that
// doubles every round) all update one count, and same-address atomics
// serialise at about 8 ns each: millions of them per round without this.
__device__ __forceinline__ int wave_combine(int t, int d) {
  const unsigned long long act = __ballot(1);
  // (the leader is the same for the whole wave: a lane read, not an LDS
  // permute, on the rewrite's dependent chain)
  const int leader = __builtin_amdgcn_readfirstlane(__ffsll((long long)act) - 1);
  const int tl = __builtin_amdgcn_readlane(t, leader), dl = __builtin_amdgcn_readlane(d, leader);
  const bool m = t == tl && d == dl;
  const unsigned long long same = __ballot(m);
  if (!m) return 1;
  return lane() == leader ? __popcll(same) : 0;
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ int wave_incl_scan(int x) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d, 64);
    if (lane() >= d) x += y;
  }
  return x;
}

// Small per-lane arrays live in vector registers: clang's ext_vector_type is
// indexed in registers even with a run-time index, whereas plain arrays with
// run-time indices are placed in scratch memory.
typedef int ivec4 __attribute__((ext_vector_type(4)));
typedef int ivec8 __attribute__((ext_vector_type(8)));
typedef int ivec16 __attribute__((ext_vector_type(16)));
typedef int ivec32 __attribute__((ext_vector_type(32)));

// Per-argument values of a node (A entries), and the argument entries of its
// arguments (A x A), each one register vector of the smallest fitting size
// (they are indexed at run time, so the whole vector stays in registers).
template <int A>
using VecA = typename std::conditional<(A <= 4), ivec4, ivec8>::type;
template <int A>
using GcVec = typename std::conditional<
    (A * A <= 4), ivec4,
    typename std::conditional<(A * A <= 8), ivec8,
                              typename std::conditional<(A * A <= 16), ivec16, ivec32>::type>::type>::type;

// An LDS-buffered append list: lanes append with an LDS atomic, the
// workgroup flushes the buffer to the global list with one atomic.
struct Queue {
  int32_t *buf;     // LDS
  int32_t *out;     // global list
  int32_t *gcount;  // global length
  int cap_lds;
  int slot;         // index of the LDS counter in misc[]
  int lc;           // index in misc[] of the list's length in a solo round
};

struct Lds {
  int32_t *tab;
  int32_t *work;
  // misc: [0] work count [1..3] queue counts [4..6] flush / reservation bases
  //       [8..23] wave sums [32..39] statistics [47..62] second wave sums
  //       [63] barrier flag
  int32_t *misc;
  int32_t *rcnt;  // per-rule application counts of this workgroup
  uint4 *pf;      // sweep prefetch ring: 16 state bytes per thread and buffer
  uint32_t *pfw;  // and the matching wake word (32 bits: 16 slots)
                  // ([B, 2B)) per thread for the next tile
  // statistics of this workgroup over every round it runs in the launch,
  // flushed once at the end of the launch: STAT_* then gc rounds, full
  // sweeps, peak extent
  unsigned long long *lstat;
  // phase timestamps of this workgroup's current round (per-workgroup phase
  // trace only), written to the trace buffer when the round ends
  unsigned long long *tstamp;
  // a scanned round: start offsets of the scan's lists in the round's list
  // (entry scan_lists: their total)
  int32_t *soff;
  Queue qd, qf, qr;  // dead, frontier, retire
  // same-round continuation (list rounds): two LDS buffers of ready nodes
  // this workgroup created or rewrote, examined in further passes of the
  // round (counts in misc[7] and misc[27]); cap entries each
  int32_t *cb0, *cb1;
  int ccap;
  // the workgroup runs the round alone: the round's claim and list
  // counters are kept in LDS at misc[LC_SLOT ..] (alloc, push, dead,
  // frontier, retire; Queue::lc indexes the list ones) and stored to the
  // control block at the end of the round
  bool solo;
};
#define LC_SLOT 35

#define LSTAT_GC CTL_NSTAT
#define LSTAT_FULL (CTL_NSTAT + 1)
#define LSTAT_PEAK (CTL_NSTAT + 2)
#define LSTAT_N (CTL_NSTAT + 3)

__device__ __forceinline__ void qpush(const Lds &L, const Queue &q, int32_t v, int64_t cap) {
  const int i = atomicAdd(&L.misc[q.slot], 1);
  if (i < q.cap_lds) {
    q.buf[i] = v;
  } else {  // LDS buffer full: append directly
    // (the LDS count through an LDS-typed pointer: a generic one selected
    // against the global counter is not compiled correctly)
    int g;
    if (L.solo) {
      auto *lcnt = (__attribute__((address_space(3))) int32_t *)(L.misc + q.lc);
      g = __hip_atomic_fetch_add(lcnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      g = atomicAdd(q.gcount, 1);
    }
    if (g < cap) q.out[g] = v;
  }
}

// Append a ready node to continuation buffer k (0 or 1); a full buffer
// passes it on to the next round's frontier.
__device__ __forceinline__ void qpush_cont(const Lds &L, int k, int32_t v, int64_t cap) {
  int32_t *buf = k ? L.cb1 : L.cb0;
  const int i = atomicAdd(&L.misc[k ? 27 : 7], 1);
  if (i < L.ccap)
    buf[i] = v;
  else
    qpush(L, L.qf, v, cap);
}

__device__ __forceinline__ void qreserve(const Lds &L, const Queue &q, int k) {
  const int nb = min(L.misc[q.slot], q.cap_lds);
  int b = 0;
  if (nb > 0) {
    if (L.solo) {
      b = L.misc[q.lc];
      L.misc[q.lc] = b + nb;
    } else {
      b = atomicAdd(q.gcount, nb);
    }
  }
  L.misc[4 + k] = b;
}

// Flush one LDS queue's buffered entries (whole workgroup; k = flush slot).
__device__ __forceinline__ void qcopy(const Lds &L, const Queue &q, int k, int64_t cap) {
  const int nb = min(L.misc[q.slot], q.cap_lds);
  const int gb = L.misc[4 + k];
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if ((int64_t)gb + i < cap) q.out[gb + i] = q.buf[i];
}

// Flush the three LDS queues (whole workgroup).
__device__ __forceinline__ void qflush(const Lds &L, int64_t cap) {
  lds_sync();
  // (each queue is named statically: selecting one at run time would force
  // the workgroup's LDS descriptors into scratch memory)
  if (threadIdx.x == 0)
    qreserve(L, L.qd, 0);
  else if (threadIdx.x == 1)
    qreserve(L, L.qf, 1);
  else if (threadIdx.x == 2)
    qreserve(L, L.qr, 2);
  lds_sync();
  qcopy(L, L.qd, 0, cap);
  qcopy(L, L.qf, 1, cap);
  qcopy(L, L.qr, 2, cap);
  lds_sync();
  if (threadIdx.x < 3) L.misc[1 + threadIdx.x] = 0;
  lds_sync();
}

// Workgroup-wide reservation of m1 items on counter c1 and m2 items on c2.
// Returns this lane's first index for each.  Called by every thread.
__device__ __forceinline__ int2 wg_reserve2(const Lds &L, int m1, int32_t *c1, int m2,
                                            int32_t *c2) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int i1 = wave_incl_scan(m1), i2 = wave_incl_scan(m2);
  if (lane() == 63) {
    L.misc[8 + w] = i1;
    L.misc[47 + w] = i2;
  }
  lds_sync();
  if (threadIdx.x == 0) {
    int r1 = 0, r2 = 0;
    for (int i = 0; i < nw; i++) {
      int t1 = L.misc[8 + i], t2 = L.misc[47 + i];
      L.misc[8 + i] = r1;
      L.misc[47 + i] = r2;
      r1 += t1;
      r2 += t2;
    }
    if (L.solo) {  // (alone in the round: the counts are in LDS)
      L.misc[4] = L.misc[LC_SLOT];
      L.misc[5] = L.misc[LC_SLOT + 1];
      L.misc[LC_SLOT] += r1;
      L.misc[LC_SLOT + 1] += r2;
    } else {
      L.misc[4] = r1 ? atomicAdd(c1, r1) : 0;
      L.misc[5] = r2 ? atomicAdd(c2, r2) : 0;
    }
  }
  lds_sync();
  int2 b;
  b.x = L.misc[4] + L.misc[8 + w] + i1 - m1;
  b.y = L.misc[5] + L.misc[47 + w] + i2 - m2;
  lds_sync();  // misc reused by the next call
  return b;
}

__device__ __forceinline__ int xcd_remap(int wg, int G) {
  // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so that its L2 sees neighbouring slots
  if (G & 7) return wg;
  return (wg & 7) * (G >> 3) + (wg >> 3);
}

// phase timestamp (thread 0 of workgroup 0, when tracing is on)
__device__ __forceinline__ void tmark_any(const RoundArgs &a, int r, int field,
                                          bool latest = false) {
  if (!a.trace) return;
  int row = r;
  if (a.trace_shift > 0) {
    if ((r & ((1 << a.trace_shift) - 1)) >= 2) return;
    row = 2 * (r >> a.trace_shift) + (r & 1);
  }
  if (row >= a.trace_cap) return;
  long long *w = a.trace + (size_t)row * TRACE_FIELDS + field;
  const long long now = (long long)wall_clock64();
  if (latest)
    atomicMax(reinterpret_cast<unsigned long long *>(w), (unsigned long long)now);
  else
    *w = now;
}

// Phase timestamp (100 MHz wall clock, comparable across compute units) of
// round r: workgroup 0's, or with trace_max every workgroup's, kept in LDS
// until the round ends (tflush), so that tracing adds no global write (and
// no wait for one) inside the round.
__device__ __forceinline__ void tmark(const RoundArgs &a, const Lds &L, int r, int field) {
  if (!a.trace || threadIdx.x != 0) return;
  if (a.trace_max)
    L.tstamp[field] = wall_clock64();
  else if (blockIdx.x == 0)
    tmark_any(a, r, field);
}

// End of round r (per-workgroup trace): this workgroup's timestamps go to
// row (sampled round, workgroup), for the first 64 workgroups.
__device__ __forceinline__ void tflush(const RoundArgs &a, const Lds &L, int r) {
  if (!a.trace || !a.trace_max || threadIdx.x != 0) return;
  int row = r;
  bool keep = true;
  if (a.trace_shift > 0) {
    keep = (r & ((1 << a.trace_shift) - 1)) < 2;
    row = 2 * (r >> a.trace_shift) + (r & 1);
  }
  if (keep && row < a.trace_cap && blockIdx.x < 64) {
    long long *w = a.trace + ((size_t)row * 64 + blockIdx.x) * TRACE_FIELDS;
    for (int f = 0; f < TRACE_FIELDS; f++)
      if (L.tstamp[f]) w[f] = (long long)L.tstamp[f];
  }
  for (int f = 0; f < TRACE_FIELDS; f++) L.tstamp[f] = 0;
}

struct Counters {
  int active, ready, fired, nfset, alloc, freed, rcops, memo, mlp, keep, trace, walk;
};

// Age bucket of the predictor's input: 0 for age 0, else
// min(15, floor(log2 age) + 1).
__device__ __forceinline__ int age_bucket(int age) {
  return age <= 0 ? 0 : min(15, 32 - __clz(age));
}

// The predictor's keep decision for (symbol, argument normal-form bits, age
// bucket), from the decision table held in LDS.
__device__ __forceinline__ bool gate_keep(const Lds &L, int off, int sym, int bits, int bucket) {
  const int i = ((sym * 32 + bits) << 4) | bucket;
  return (L.tab[off + (i >> 5)] >> (i & 31)) & 1;
}

// visible normal form in round parity e (markers of the current parity are
// not yet valid)
__device__ __forceinline__ bool nf_visible(unsigned st, unsigned e) {
  return (st & ST_NF) && !((st & ST_PEND) && (((st >> 2) & 1u) == e));
}

// Rewrite a marker of round parity ep into the plain state.  Retire-list
// entries are handled only in frontier rounds, where no other thread writes
// the byte in the same round (a full round's sweep retires every marker
// itself), so a plain byte store suffices.
__device__ __forceinline__ void retire_marker(uint8_t *state, int s, unsigned ep) {
  const unsigned b = state[s];
  if (!(b & ST_PEND) || ((b >> 2) & 1u) != ep) return;
  state[s] = (uint8_t)((b & ST_NF) ? ST_NF : ST_ACTIVE);
}

struct RoundCtx {
  int r, n, fsP, mode;
  int room;   // claims below this take fresh slots first (locality placement)
  bool walk;     // constructor walk (nf_walk) on in this round
  int walk_max;  // constructors one walk may mark in this round
  int cbuf;      // >= 0: ready nodes this thread creates or rewrites go to
                 // continuation buffer cbuf (examined later in this round)
  int cont;      // further passes this workgroup may run in this round
  unsigned e;
  int stamp;
  const int32_t *SP;
  RoundCnt *cnt;
};

// Notify the parent of a node that just became a normal form (frontier modes).
// Returns the parent to queue once the exchange's result is in (0: none); the
// caller consumes it after issuing its other atomics, so their latencies
// overlap.
__device__ __forceinline__ int notify_parent(const RoundArgs &a, const RoundCtx &R, int par) {
  if (par > 0 && par < a.p.N) return atomicExch(&a.p.qstamp[par], R.stamp) != R.stamp ? par : 0;
  return 0;
}


// Frontier rounds: node s has just become a normal form (with this round's
// marker).  A symbol without rules over arguments that are all normal forms
// is a normal form itself; rather than leaving each constructor above s to
// a round of its own, the thread walks up the parent hints and marks such
// ancestors normal forms in this round, at most R.walk_max of them, and
// notifies the first node on the way that it does not mark (returned, as
// notify_parent's result); a notified constructor over normal forms becomes
// one next round and walks on from there.  The bound keeps a long chain
// from holding up the round (a walk is one lane's sequence of dependent
// reads, and the round ends with its longest walk).  This changes rounds
// and visits only: no node is rewritten, so normal forms and rule
// applications stay those of innermost rewriting.  (The term graph is
// acyclic and each step checks that the parent references the node below
// it, so a walk would end by itself.)
//
// An ancestor q is marked only when
//   - q's live, without a marker and not a normal form, with a count above
//     zero, and its symbol has no rules;
//   - q was not queued for this round (its notification stamp is not the
//     previous round's): no other thread examines it in this round, so no
//     memo store can overwrite the mark (constructors reach a frontier only
//     through that stamp);
//   - the node below is one of q's arguments and every other argument is a
//     normal form visible in this round.
// q gets the plain normal-form state, without a marker: its fields were
// written in earlier rounds and never change, so a parent examined later
// in this round may read it at once.  Two walks that meet at a node both
// stop there unless each sees the other's node marked; then both go on,
// marking the same nodes with the same value.  Full rounds, where every
// live slot is examined, notify only.
// One level of the walk: a parent's fields and its own parent hint, loaded
// together (the first level is loaded where the node becomes a normal form,
// so that its latency overlaps the rewrite's reference-count atomics).
template <int A>
struct WalkLvl {
  int par;  // 0: none
  unsigned st;
  int f, rc, qs, pp;
  VecA<A> raw;
};

template <int A>
__device__ __forceinline__ void walk_load(const Pool &p, int par, WalkLvl<A> &w) {
  w.par = (par > 0 && par < p.N) ? par : 0;
  if (!w.par) return;
  w.st = p.state[par];
  w.f = p.hss[par];
  w.rc = p.rc[par];
  w.qs = p.qstamp[par];
  w.pp = p.par[par];
#pragma unroll
  for (int j = 0; j < A; j++) w.raw[j] = p.args[(int64_t)par * A + j];
}

template <int A>
__device__ __forceinline__ int nf_walk(const RoundArgs &a, const Lds &L, const RoundCtx &R, int s,
                                       WalkLvl<A> w, Counters &C) {
  const Pool &p = a.p;
  const int64_t N = p.N;
  const bool track = R.mode == 2;  // keep lastchg
  int cur = s;
  for (int k = 0; k < R.walk_max; k++) {
    if (!w.par) return 0;
    const int par = w.par;
    bool ok = (w.st & (ST_NF | ST_PEND | ST_ACTIVE)) == ST_ACTIVE && w.rc > 0 &&
              w.qs != R.stamp - 1 && (unsigned)w.f < (unsigned)a.n_sym;
    const int info = ok ? L.tab[TAB_SYM + w.f] : 0;
    ok = ok && ((info >> 8) & 0xff) == 0;
    const int ar = SYM_ARITY(info);
    bool below = false;
    if (ok) {
      // (arity above one: the other arguments' states, one more step)
      VecA<A> ost = (VecA<A>)(ST_NF);
#pragma unroll
      for (int j = 0; j < A; j++) {
        if (j < ar) {
          const int c = w.raw[j];
          if (c == cur)
            below = true;
          else if ((unsigned)c < (unsigned)N && c > 0)
            ost[j] = p.state[c];
          else
            ok = false;
        }
      }
#pragma unroll
      for (int j = 0; j < A; j++)
        if (j < ar && w.raw[j] != cur && !nf_visible((unsigned)ost[j], R.e)) ok = false;
    }
    if (!ok || !below) return notify_parent(a, R, par);
    p.state[par] = (uint8_t)ST_NF;
    if (track) p.lastchg[par] = R.r;
    C.walk++;
    cur = par;
    walk_load<A>(p, w.pp, w);
  }
  return notify_parent(a, R, w.par);
}

typedef __attribute__((address_space(3))) void lds_void;

// This wave's prefetch entries in ring buffer b (state bytes, wake words),
// from wave-uniform values only, so that the address stays in scalar
// registers (a spilled vector address would be reloaded, and the wait for
// that reload would also wait for the prefetch just issued).
__device__ __forceinline__ uint4 *pf_state(const Lds &L, int b) {
  const int w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63);
  return L.pf + b * (int)blockDim.x + w0;
}
__device__ __forceinline__ uint32_t *pf_wake(const Lds &L, int b) {
  const int w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63);
  return L.pfw + b * (int)blockDim.x + w0;
}

// Asynchronous copy of 16 (4) bytes per lane from global memory straight
// into LDS (no registers held while in flight): lane l of the wave writes
// dst_wave[l], where dst_wave is the wave's (uniform) base.
__device__ __forceinline__ void lds_fetch16(const void *src, uint4 *dst_wave) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)dst_wave, 16, 0, 0);
}
__device__ __forceinline__ void lds_fetch4(const void *src, uint32_t *dst_wave) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)dst_wave, 4, 0, 0);
}

// npt (1, 2, 4, 8 or 16) consecutive bytes, in byte order from the low end
// of a uint4 (the rest zero); one vector load for 4, 8 and 16
__device__ __forceinline__ uint4 load_bytes(const uint8_t *q, int npt) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (npt == 16) {
    v = *reinterpret_cast<const uint4 *>(q);
  } else if (npt == 8) {
    const uint2 u = *reinterpret_cast<const uint2 *>(q);
    v.x = u.x;
    v.y = u.y;
  } else if (npt == 4) {
    v.x = *reinterpret_cast<const uint32_t *>(q);
  } else {
    for (int j = 0; j < npt; j++) v.x |= (unsigned)q[j] << (8 * j);
  }
  return v;
}

// Bit j (j = 0..3) set when byte j of x has any of its low 7 bits set: the
// add carries into bit 7 of the byte exactly then, and never across bytes.
__device__ __forceinline__ int nz7x4(unsigned x);

// Bit 0 of each byte of x, packed into bits 0-3 (the four products land on
// distinct bit positions, so no carries mix them).
__device__ __forceinline__ int pack4(unsigned x) {
  return (int)((((x & 0x01010101u) * 0x01020408u) >> 24) & 0xFu);
}

__device__ __forceinline__ int nz7x4(unsigned x) {
  return pack4(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) >> 7);
}

// Plain mode: tell the parent of a node that just became a normal form to
// test itself again (from the next round on: the bit of this round's parity
// is honoured only by rounds of the other parity).  A 32-bit atomic OR on the
// word that holds the parent's wake byte.
__device__ __forceinline__ void wake_parent(const RoundArgs &a, const RoundCtx &R, int s) {
  const int par = a.p.par[s];
  if (par > 0 && par < a.p.N) atomicOr(&a.p.wake[par >> 4], 1u << (((par & 15) << 1) | R.e));
}

// Wait until at most k (0..6) of the wave's vector memory operations are
// outstanding (s_waitcnt takes the count as an immediate).
__device__ __forceinline__ void vm_wait_tiles(int k) {
  switch (k) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
    case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
  }
}

// Bits 0, 2, ..., 30 of x, packed into the low 16 bits.
__device__ __forceinline__ int even_bits(unsigned x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return (int)x;
}

// A dead-list entry whose node already dropped its references to its
// arguments (in the round it died); slot indices stay below 2^30.
#define DEAD_RELEASED 0x40000000

// Drop one reference to each argument of dead node d; arguments whose
// count reaches zero go on the dead list (their own arguments still held).
template <int A>
__device__ __forceinline__ void release_args(const RoundArgs &a, const Lds &L, RoundCnt *cnt,
                                             int d, Counters &C) {
  const Pool &p = a.p;
  const int f = p.hss[d];
  const int ar = ((unsigned)f < (unsigned)a.n_sym) ? SYM_ARITY(L.tab[TAB_SYM + f]) : 0;
#pragma unroll
  for (int j = 0; j < A; j++) {
    if (j < ar) {
      const int c = p.args[(int64_t)d * A + j];
      if ((unsigned)c >= (unsigned)p.N || c == 0) {
        st(&cnt->err, -9);
        continue;
      }
      const int old = atomicSub(&p.rc[c], 1);
      C.rcops++;
      if (old == 1) qpush(L, L.qd, c, p.N);
    }
  }
}

// Examine slot s (s <= 0: idle lane) and rewrite it if it is a redex whose
// arguments are all normal forms.  memo: the slot's memo bits.  Must be
// called by every thread of the workgroup (contains the allocation barrier);
// free_slot > 0: this lane also pushes that slot (a node collected in the
// same pass) on the free stack SQ.
// A slot's symbol, argument entries and parent hint, when the caller read
// them together with the slot's state.
template <int A>
struct Pre {
  bool have;
  int f, par;
  int lc;  // round of the slot's last change (learned mode and tracing)
  VecA<A> raw;
};

template <int A>
__device__ __forceinline__ void process_slot(const RoundArgs &a, const Lds &L, const RoundCtx &R,
                                             int s, int memo, bool memo_checked, int free_slot,
                                             int32_t *SQ, int fsQ, Counters &C, const Pre<A> &pre) {
  const Pool &p = a.p;
  const int32_t *tab = L.tab;
  const unsigned e = R.e;
  const int64_t N = p.N;
  const bool frontier = R.mode != 0;
  const bool track = R.mode == 2 || a.trace_rate != 0;  // keep lastchg
  RoundCnt *cnt = R.cnt;
  bool have = s > 0;
  int info = 0, ar = 0, f = 0;
  VecA<A> av = (VecA<A>)(0);
  VecA<A> ch = (VecA<A>)(-1);  // argument symbols (read with the argument states)
  // argument entries of the arguments at the positions where some rule of
  // the symbol has a pattern below the argument (read with the argument
  // states, so that matching such patterns needs no further read)
  GcVec<A> gc = (GcVec<A>)(0);
  int par_s = 0;  // parent hint (frontier mode), read with the slot's entries
  int lc_s = 0;   // round of the slot's last change (track), read with them too
  bool ready = false;
  int nfb = -1;  // >= 0: the slot was examined and is blocked; bit j set when
                 // argument j is a visible normal form or j >= arity
  if (have) {
    if (!memo_checked) C.active++;
    // the symbol and all A argument entries are read together (entries past
    // the arity lie within the slot's stride and are ignored), then the
    // states and symbols of the arguments together: two dependent levels
    VecA<A> raw = (VecA<A>)(0);
    if (pre.have) {
      f = pre.f;
      raw = pre.raw;
      par_s = pre.par;
      lc_s = pre.lc;
    } else {
      f = p.hss[s];
#pragma unroll
      for (int j = 0; j < A; j++) raw[j] = p.args[(int64_t)s * A + j];
      if (R.mode != 0) par_s = p.par[s];
      if (track) lc_s = p.lastchg[s];
    }
    {
      if ((unsigned)f >= (unsigned)a.n_sym) {
        st(&cnt->err, -9);
      } else {
        info = tab[TAB_SYM + f];
        ar = SYM_ARITY(info);
        bool ok = true;
#pragma unroll
        for (int j = 0; j < A; j++) {
          if (j < ar) {
            const int c = raw[j];
            if ((unsigned)c >= (unsigned)N || c == 0) ok = false;
            av[j] = c;
          }
        }
        if (!ok) {
          st(&cnt->err, -9);
        } else {
          int bits = 0;
          // (not kept for arity 5: 25 more registers would spill)
          const int deep = A <= 4 ? SYM_DEEP(info) : 0;
#pragma unroll
          for (int j = 0; j < 5; j++) {
            if (j >= ar) {
              bits |= 1 << j;
            } else if (j < A) {
              const unsigned st = p.state[av[j]];
              ch[j] = p.hss[av[j]];
              if ((deep >> j) & 1) {
#pragma unroll
                for (int i = 0; i < A; i++) gc[j * A + i] = p.args[(int64_t)av[j] * A + i];
              }
              if (nf_visible(st, e)) bits |= 1 << j;
            }
          }
          ready = bits == 31;
          if (!ready) {
            // learned mode sets the memo only for nodes the predictor drops
            if (a.use_memo && R.mode != 2) {
              const int first_blocked = __builtin_ctz(~bits) + 1;
              if (first_blocked != memo)
                p.state[s] = (uint8_t)(ST_ACTIVE | (first_blocked << ST_MEMO_SHIFT));
            }
            nfb = bits;
          }
        }
      }
    }
  }
  if (nfb >= 0 && (R.mode == 2 || a.trace_rate)) {
    // a blocked node after a full readiness test: learned mode asks the
    // predictor whether to examine it again next round; tracing samples it
    const int bk = age_bucket(R.r - lc_s);
    if (R.mode == 2) {
      // kept: examined next round (no memo, so a full sweep tests it in
      // full too); dropped: sleeps on its first blocking argument until a
      // full sweep finds that argument in normal form.  A symbol without
      // rules can only become a normal form through its arguments, which
      // notification (and the walk) report exactly, so such a node is not
      // put to the predictor: it sleeps, and stays open to the walk.
      const int fb = __builtin_ctz(~nfb) + 1;
      const bool rules = ((info >> 8) & 0xff) != 0;
      C.mlp += rules;
      if (rules && gate_keep(L, a.gate_off, f, nfb, bk)) {
        C.keep++;
        // (through the notification stamp: an argument that became a
        // normal form this round may queue the node too)
        if (notify_parent(a, R, s)) qpush(L, L.qf, s, N);
        if (memo) p.state[s] = (uint8_t)ST_ACTIVE;
      } else if (fb != memo) {
        p.state[s] = (uint8_t)(ST_ACTIVE | (fb << ST_MEMO_SHIFT));
      }
    } else if (a.trace_rate) {
      const uint32_t h = mix32((uint32_t)s * 0x9E3779B1u ^ (uint32_t)R.r * 0x85EBCA77u);
      // (appends stop once the buffer is full, so the counter cannot wrap)
      if ((h & 0xffffu) < a.trace_rate && ld(a.trace_n) < a.trace_cap_rec) {
        C.trace++;
        const int idx = atomicAdd(a.trace_n, 1);
        if (idx >= 0 && idx < a.trace_cap_rec) {
          a.trace_rec[idx] = (unsigned long long)f | ((unsigned long long)ar << 16) |
                             ((unsigned long long)nfb << 20) | ((unsigned long long)bk << 25);
          p.tref[s] = ((long long)idx << 32) | (unsigned)R.r;
        }
      }
    }
  }
  if (ready && a.trace_rate && R.r > 0) {
    // label of the node's latest record, when it was logged at most
    // label_h rounds ago: the node fires or becomes a normal form now
    const long long t = p.tref[s];
    const long long idx = t >> 32;
    const int rr = (int)(t & 0xffffffff);  // round of the record
    if (rr >= 0 && rr < R.r && R.r - rr <= a.label_h && idx >= 0 && idx < a.trace_cap_rec)
      a.trace_rec[idx] |= 1ull << 32;
  }
  tmark(a, L, R.r, 6);
  int prog = -1;
  bool nfset = false;
  // 3 bits per pattern node of the rule being matched (after matching: of the
  // matched rule): 1 + the argument position of a node directly below the
  // root, 0 for deeper nodes
  unsigned d1 = 0;
  // slot matched by pattern node k: the redex s for k = 0, else ps[k - 1]
  ivec8 ps = (ivec8)(0);
  auto pslot = [&](int k) { return k == 0 ? s : ps[k - 1]; };
  if (ready) {
    C.ready++;
    const int nr = (info >> 8) & 0xff, first = info >> 16;
    if (nr == 0) {
      nfset = true;
    } else {
      const int32_t *rtab = tab + TAB_SYM + a.n_sym + first;
      // the last node below the arguments read during matching: its slot,
      // symbol and entries, read together (the rules of a symbol often test
      // the same node, and its entries bind the variables below it)
      int cc = 0, chh = -1;
      VecA<A> cargs = (VecA<A>)(0);
      for (int i = 0; i < nr && prog < 0; i++) {
        const int pg = rtab[i];
        const int npat = tab[pg] & 15;
        bool ok = true;
        d1 = 0;
        for (int k = 1; k <= npat && ok; k++) {
          const int pe = tab[pg + 5 + k];
          const int par = pe & 15, pos = (pe >> 4) & 15;
          const bool isvar = (pe >> 8) & 1;
          int c, h = -1;
          if (par == 0) {
            c = av[pos];
            if (!isvar) h = ch[pos];
            if (A <= 4) d1 |= (unsigned)(pos + 1) << (3 * k);  // (gc is kept for A <= 4)
          } else {
            const int jp = (int)((d1 >> (3 * par)) & 7);
            const int sp = pslot(par);
            c = jp ? gc[(jp - 1) * A + pos]
                   : (sp == cc ? cargs[pos] : p.args[(int64_t)sp * A + pos]);
            if ((unsigned)c >= (unsigned)N || c == 0) {  // broken invariant: stop safely
              st(&cnt->err, -9);
              c = sp;
              ok = false;
            }
            if (!isvar && ok) {
              if (c != cc) {
                cc = c;
                chh = p.hss[c];
#pragma unroll
                for (int q = 0; q < A; q++) cargs[q] = p.args[(int64_t)c * A + q];
              }
              h = chh;
            }
          }
          ps[k - 1] = c;
          if (!isvar && h != (pe >> 16)) ok = false;
        }
        if (ok) prog = pg;
      }
      if (prog < 0) nfset = true;
    }
  }
  const int hdr = prog >= 0 ? tab[prog] : 0;
  const int m = (hdr >> 4) & 15;
  C.alloc += m;
  tmark(a, L, R.r, 7);
  const int2 base = wg_reserve2(L, m, &cnt->alloc, free_slot > 0 ? 1 : 0, &cnt->push);
  tmark(a, L, R.r, 8);
  if (free_slot > 0) {
    if ((int64_t)fsQ + base.y < N)
      SQ[fsQ + base.y] = free_slot;
    else
      st(&cnt->err, -9);
  }
  ivec8 ns = (ivec8)(0);  // slots of the new nodes
  bool okalloc = true;
#pragma unroll
  for (int j = 0; j < MAXNEW; j++) {
    if (j < m) {
      const int c = base.x + j;
      // claim c: fresh slots n, n+1, ... for the first R.room claims, then
      // the recycled slots on the free stack, then fresh slots again
      const int cr = c - R.room;
      const int64_t slot = c < R.room ? (int64_t)R.n + c
                           : cr < R.fsP ? (int64_t)R.SP[R.fsP - 1 - cr]
                                        : (int64_t)R.n + (c - R.fsP);
      if (slot >= N || slot <= 0) okalloc = false;
      ns[j] = (int)slot;
    }
  }
  if (prog >= 0 && !okalloc) {
    st(&cnt->err, -5);  // TRS_E_POOL
    prog = -1;
  }
  const uint8_t pend_nf = (uint8_t)(ST_NF | ST_PEND | (e << 2));
  int note = 0;  // parent to queue (frontier mode), once its exchange returns
  bool walking = false;  // the slot became a normal form: walk up (nf_walk)
  WalkLvl<A> wl;
  wl.par = 0;
  // The slot became a normal form in this round: its marker, then parent
  // notification (frontier modes; with the walk, the walk's first level is
  // loaded here, so that its latency overlaps the reference-count atomics)
  // or the parent's wake bit (plain mode).
  auto became_nf = [&]() {
    p.state[s] = pend_nf;
    if (track) p.lastchg[s] = R.r;
    if (R.walk) {
      walking = true;
      walk_load<A>(p, par_s, wl);
    } else if (R.mode != 0) {
      note = notify_parent(a, R, par_s);
    }
    if (R.mode == 0 && a.use_memo) wake_parent(a, R, s);
    if (frontier) qpush(L, L.qr, s, N);
  };
  if (prog >= 0) {
    C.fired++;
    const int rsym = tab[prog + 1];
    const int ro = tab[prog + 2], no = tab[prog + 3], dl = tab[prog + 4];
    const bool var_root = (hdr >> 8) & 1, root_nf = (hdr >> 9) & 1, root_ready = (hdr >> 10) & 1;
    const int npos = (hdr >> 12) & 15, nneg = (hdr >> 16) & 15, rootpat = (hdr >> 20) & 15;
    // new nodes, children before parents
    int q = no;
    for (int j = 0; j < m; j++) {
      const int h = tab[q];
      const int sym = h & 0xffff, rci = (h >> 16) & 0x3f, bnf = (h >> 22) & 1;
      const int nready = (h >> 23) & 1, refr = (h >> 24) & 15;
      const int ar2 = SYM_ARITY(tab[TAB_SYM + sym]);
      const int slot = ns[j];
#pragma unroll
      for (int o = 0; o < A; o++) {
        if (o < ar2) {
          const int v = tab[q + 1 + o];
          p.args[(int64_t)slot * A + o] = v >= 0 ? pslot(v) : ns[-1 - v];
        }
      }
      p.hss[slot] = sym;
      p.rc[slot] = rci;
      // (a round marker keeps a node created in a full round from the
      // sweep of that round; in a list round with the walk, nothing but
      // this thread's own lists reaches the new node, so it is plainly
      // live and needs no retirement)
      p.state[slot] = bnf      ? (uint8_t)ST_NF
                      : R.walk ? (uint8_t)ST_ACTIVE
                               : (uint8_t)(ST_ACTIVE | ST_PEND | (e << 2));
      if (track) p.lastchg[slot] = R.r;
      p.par[slot] = refr ? ns[refr - 1] : s;
      if (frontier && !bnf) {
        // a new node that is not ready waits on new arguments whose parent
        // hint is this node: notification reports them exactly, so it is
        // not queued (nor, in learned mode, put to the predictor)
        if (nready) {
          if (R.cbuf >= 0)
            qpush_cont(L, R.cbuf, slot, N);  // examined later in this round
          else
            qpush(L, L.qf, slot, N);  // examined next round (retires its own marker)
        } else if (!R.walk) {
          qpush(L, L.qr, slot, N);
        }
      }
      q += 1 + ar2;
    }
    // the redex root is overwritten in place
    if (var_root) {
      const int src = pslot(rootpat);
      // a variable directly below the root: its symbol and entries were read
      // with the argument states
      const int jr = (int)((d1 >> (3 * rootpat)) & 7);
      int sh = jr ? ch[jr - 1] : p.hss[src];
      if ((unsigned)sh >= (unsigned)a.n_sym) {
        st(&cnt->err, -9);
        sh = 0;
      }
      const int sar = SYM_ARITY(tab[TAB_SYM + sh]);
#pragma unroll
      for (int j = 0; j < A; j++) {
        if (j < sar) {
          const int cj = jr ? gc[(jr - 1) * A + j] : p.args[(int64_t)src * A + j];
          p.args[(int64_t)s * A + j] = cj;
          if ((unsigned)cj < (unsigned)N) {
            atomicAdd(&p.rc[cj], 1);
            C.rcops++;
          } else {
            st(&cnt->err, -9);
          }
        }
      }
      p.hss[s] = sh;
      became_nf();
    } else {
      const int rar = SYM_ARITY(tab[TAB_SYM + rsym]);
#pragma unroll
      for (int o = 0; o < A; o++) {
        if (o < rar) {
          const int v = tab[ro + o];
          p.args[(int64_t)s * A + o] = v >= 0 ? pslot(v) : ns[-1 - v];
        }
      }
      p.hss[s] = rsym;
      if (track) p.lastchg[s] = R.r;
      if (root_nf) {
        became_nf();
      } else {
        if (memo) p.state[s] = (uint8_t)ST_ACTIVE;  // the arguments changed: drop the memo
        if (frontier) {
          // a root rewritten into a term that is not ready waits on new
          // arguments whose parent hint is the root: notification reports
          // them exactly, so it is not queued (nor put to the predictor)
          if (root_ready && R.cbuf >= 0)
            qpush_cont(L, R.cbuf, s, N);  // ready again: examined later in this round
          else if (root_ready)
            qpush(L, L.qf, s, N);
        }
      }
    }
    // reference counts: increments first, then decrements (a decrement that
    // reaches zero puts the node on the dead list).  The first entry of each
    // kind is combined over the wave's lanes that update the same count by
    // the same amount (one atomic for all of them, issued by the first)
    if (npos > 0) {
      const int dw = tab[dl];
      const int d = (int)(int8_t)((dw >> 8) & 0xff);
      const int t = pslot(dw & 0xff);
      const int c = wave_combine(t, d);
      if (c) atomicAdd(&p.rc[t], c * d);
    }
    for (int i = 1; i < npos; i++) {
      const int dw = tab[dl + i];
      atomicAdd(&p.rc[pslot(dw & 0xff)], (int)(int8_t)((dw >> 8) & 0xff));
    }
    // decrements: the first NEG_BATCH are all issued before any result is
    // examined, so their latencies (and the parent exchange's) overlap; the
    // combined one reaches zero only when the last reference goes
    constexpr int NEG_BATCH = 4;
    ivec4 dold, dslot;
    if (nneg > 0) {
      const int dw = tab[dl + npos];
      const int d = (int)(int8_t)((dw >> 8) & 0xff);
      dslot[0] = pslot(dw & 0xff);
      const int c = wave_combine(dslot[0], d);
      dold[0] = c ? atomicAdd(&p.rc[dslot[0]], c * d) + c * d : 1;
    }
#pragma unroll
    for (int i = 1; i < NEG_BATCH; i++) {
      if (i < nneg) {
        const int dw = tab[dl + npos + i];
        const int d = (int)(int8_t)((dw >> 8) & 0xff);
        dslot[i] = pslot(dw & 0xff);
        dold[i] = atomicAdd(&p.rc[dslot[i]], d) + d;
      }
    }
    // A node whose count reaches zero goes on the dead list; its slot is
    // freed next round.  In rounds with further passes it drops its own
    // references at once: a chain consumed one cell per pass (the peeling
    // of a numeral) would otherwise die one cell per round after the
    // passes, each cell held by the dead one above it until that is
    // collected.  (Its slot still waits for the next round, when no list
    // of this round can name it any more.)
    auto dead = [&](int x) {
      if (R.cbuf >= 0) {
        release_args<A>(a, L, cnt, x, C);
        qpush(L, L.qd, x | DEAD_RELEASED, N);
      } else {
        qpush(L, L.qd, x, N);
      }
    };
#pragma unroll
    for (int i = 0; i < NEG_BATCH; i++)
      if (i < nneg && dold[i] == 0) dead(dslot[i]);
    for (int i = NEG_BATCH; i < nneg; i++) {
      const int dw = tab[dl + npos + i];
      const int d = (int)(int8_t)((dw >> 8) & 0xff);
      const int slot = pslot(dw & 0xff);
      const int old = atomicAdd(&p.rc[slot], d);
      if (old + d == 0) dead(slot);
    }
    C.rcops += npos + nneg;
  } else if (nfset) {
    C.nfset++;
    became_nf();
  }
  if (walking) note = nf_walk<A>(a, L, R, s, wl, C);
  if (note) qpush(L, L.qf, note, N);
  // per-rule counts: one LDS atomic per distinct rule among the wave's lanes
  // (every lane of the wave runs this loop; its trip count is uniform)
  {
    const int rid = prog >= 0 ? tab[prog + 5] : -1;
    unsigned long long pending = __ballot(rid >= 0);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int rl = __shfl(rid, leader, 64);
      const unsigned long long same = __ballot(rid == rl);
      if (lane() == leader) atomicAdd(&L.rcnt[rl], __popcll(same));
      pending &= ~same;
    }
  }
  tmark(a, L, R.r, 9);
  qflush(L, N);
  tmark(a, L, R.r, 10);
}

// Collect dead-list entry e: drop one reference to each argument of its
// node (unless it did so when it died), mark the slot free.  Returns the
// slot, to be pushed on the free stack, or 0.
template <int A>
__device__ __forceinline__ int collect(const RoundArgs &a, const Lds &L, RoundCnt *cnt, int e,
                                       Counters &C) {
  const Pool &p = a.p;
  const int d = e & ~DEAD_RELEASED;
  if ((unsigned)d >= (unsigned)p.N || d == 0) {
    st(&cnt->err, -9);
    return 0;
  }
  if (!(e & DEAD_RELEASED)) release_args<A>(a, L, cnt, d, C);
  p.state[d] = (uint8_t)ST_FREE;
  C.freed++;
  return d;
}

// Locality placement (option): while the extent n is below fresh_below,
// a round's first claims take fresh slots past n, which lie next to each
// other and to the nodes created just before, instead of recycled slots
// scattered over the pool.  Returns how many claims go fresh first.
__device__ __forceinline__ int fresh_room(const RoundArgs &a, int n) {
  return a.fresh_below > n ? a.fresh_below - n : 0;
}

// State of round r, derived from the counters of round r-1.
// published flags (pub[9], besides err << 8)
#define PUB_STOP 1
#define PUB_QUIESCENT 2
#define PUB_STALL 4
#define PUB_SCANNED 8    // the round's slots were classified by k_scan
#define PUB_SCAN_REQ 16  // the round is a plain full sweep for k_scan

struct RoundState {
  int r, n, fs0, fs1, nd, nfront, nret, nlist, ntiles, need, err;
  int stamp;  // first frontier-notification stamp of the run
  bool stop, quiescent, full, done;
  bool scan_req;  // plain mode: a full round large enough for k_scan
  bool scanned;   // k_scan classified the round's slots: a list round of the
                  // dead nodes and the listed slots
  bool stall;  // the previous round met live non-normal-form slots but made no
               // progress: this round is a full sweep that tests every slot
               // (plain mode: ignoring the wake bits)
};

// Thread 0 reads the previous round's counters and derives round r; the
// values reach the workgroup through LDS.  Writes nothing.  need: number of
// workgroups the round uses -- 1 when its lists are small (at most
// small_cap items), so that one workgroup can run consecutive small rounds.
// Derive round r from the counters of round r-1 (one thread; reads only).
// need: number of workgroups the round uses -- 1 when its lists are small
// (at most small_cap items), so that one workgroup can run consecutive small
// rounds.
__device__ __forceinline__ RoundState round_state(const RoundArgs &a, int r) {
  const Pool &p = a.p;
  Ctl *ctl = a.ctl;
  const int B = blockDim.x;
  RoundState rs;
  int n, fs0, fs1, nd = 0, nfront = 0, nret = 0, err = 0;
  bool quiescent = false, stop = false, stall = false;
  if (r == 0) {
    n = ld(&ctl->n[0]);
    fs0 = ld(&ctl->fs[0][0]);
    fs1 = ld(&ctl->fs[0][1]);
  } else {
    const int p3 = (r + 2) % 3;
    const int c_alloc = ld(&ctl->cnt[p3].alloc), c_push = ld(&ctl->cnt[p3].push);
    const int c_dead = ld(&ctl->cnt[p3].dead), c_act = ld(&ctl->cnt[p3].active);
    const int c_err = ld(&ctl->cnt[p3].err), c_full = ld(&ctl->cnt[p3].full);
    const int c_prog = ld(&ctl->cnt[p3].prog);
    nfront = ld(&ctl->cnt[p3].front);
    nret = ld(&ctl->cnt[p3].ret);
    const int pn = ld(&ctl->n[p3]), pf0 = ld(&ctl->fs[p3][0]), pf1 = ld(&ctl->fs[p3][1]);
    const int P = (r - 1) & 1;  // stack popped in round r-1
    const int fsP = P ? pf1 : pf0;
    const int used = min(max(c_alloc - fresh_room(a, pn), 0), fsP);
    const int64_t nn = (int64_t)pn + (c_alloc - used);
    n = (int)min(nn, (int64_t)p.N);
    if (P == 0) {
      fs0 = pf0 - used;
      fs1 = pf1 + c_push;
    } else {
      fs1 = pf1 - used;
      fs0 = pf0 + c_push;
    }
    nd = c_dead;
    // a full round that met no live non-normal-form slot: nothing can be
    // rewritten any more; remaining rounds only collect
    quiescent = c_full && c_act == 0;
    // a round that met live non-normal-form slots but in which nothing fired
    // or became a normal form: everything it examined waits on nodes it did
    // not examine (a frontier that keeps only blocked nodes, or wake bits
    // that missed a node with two parents); the next round is a full sweep
    // that tests every slot
    stall = c_act != 0 && c_prog == 0;
    stop = c_err != 0 || nn > p.N || (quiescent && c_dead == 0);
    err = c_err ? c_err : (nn > p.N ? -5 : 0);
  }
  // the round limit (termination is undecidable, Section 2): a run that is
  // not over by round max_rounds stops there with TRS_E_ROUNDS
  if (!stop && a.max_rounds > 0 && r >= a.max_rounds) {
    stop = true;
    err = -6;
  }
  if (quiescent) nfront = 0;
  rs.r = r;
  rs.n = n;
  rs.fs0 = fs0;
  rs.fs1 = fs1;
  rs.nd = nd;
  rs.nfront = nfront;
  rs.nret = nret;
  rs.stop = stop;
  rs.quiescent = quiescent;
  rs.stall = stall;
  rs.err = err;
  rs.done = false;
  rs.full = !quiescent && (a.mode == 0 || nfront == 0 || r == 0 || stall ||
                           (a.sweep_every > 0 && r % a.sweep_every == 0));
  // in full rounds the sweep retires every marker, so the retire list is
  // skipped
  rs.nlist = nd + (rs.full ? 0 : nret + nfront);
  rs.ntiles = rs.full ? (n + B * a.npt - 1) / (B * a.npt) : 0;
  rs.need = max((rs.nlist + B - 1) / B, rs.ntiles);
  if (rs.ntiles <= 1 && rs.nlist <= a.small_cap) rs.need = 1;
  if (stop) rs.need = 1;
  rs.scanned = false;
  rs.scan_req = a.use_scan && a.mode == 0 && rs.full && !stall && !stop && rs.ntiles >= 2;
  return rs;
}

// State of a round, shared with the workgroup via LDS.  from_pub: the
// launch's first round, taken from the line the previous launch published
// (plain loads: it was written before this launch began); otherwise thread 0
// derives round r from the counters of round r-1.
__device__ __forceinline__ RoundState round_prepare(const RoundArgs &a, const Lds &L, int r,
                                                    bool from_pub, bool load_tab = false) {
  int32_t *bc = L.misc + 40;  // [40..49]
  // the published line and (load_tab) the tables are read together: one
  // dependent read at the start of a launch instead of two
  int4 x, y, z;
  int2 sc[16];  // the scan's list counts and flags (plain mode), read with the line
  if (from_pub && threadIdx.x == 0) {
    const int4 *pp = reinterpret_cast<const int4 *>(a.ctl->pub);
    x = pp[0];
    y = pp[1];
    z = pp[2];
    // (plain loads: written by the launch before, as the published line)
    if (a.use_scan) {
#pragma unroll
      for (int j = 0; j < 16; j++)
        sc[j] = j < a.scan_lists ? *reinterpret_cast<const int2 *>(&a.ctl->scan_cnt[j][0])
                                 : make_int2(0, 0);
    }
  }
  if (load_tab)
    for (int i = threadIdx.x; i < a.tab_words; i += blockDim.x) L.tab[i] = a.tab[i];
  if (threadIdx.x == 0) {
    if (from_pub) {
      bc[0] = x.x;
      bc[1] = x.y;
      bc[2] = x.z;
      bc[3] = x.w;
      bc[4] = y.x;
      bc[5] = y.y;
      bc[6] = y.z;
      bc[7] = y.w;
      bc[8] = z.x;
      bc[9] = z.y;
      L.misc[29] = z.z;  // the run's stamp base, kept for the whole launch
      if ((z.y & PUB_SCAN_REQ) && !(z.y & PUB_STOP)) {
        // the scan launched just before classified this round: its lists'
        // counts give the list offsets and the number of listed slots
        int off = 0, act = 0;
#pragma unroll
        for (int j = 0; j < 16; j++) {
          if (j < a.scan_lists) {
            L.soff[j] = off;
            off += sc[j].x;
            act |= sc[j].y;
          }
        }
        L.soff[a.scan_lists] = off;
        bc[7] = off;
        bc[9] = (z.y & ~PUB_SCAN_REQ) | PUB_SCANNED;
        L.misc[28] = act;  // a live non-normal-form slot was met
      }
    } else {
      const RoundState t = round_state(a, r);
      bc[0] = 0;
      bc[1] = r;
      bc[2] = t.need;
      bc[3] = t.n;
      bc[4] = t.fs0;
      bc[5] = t.fs1;
      bc[6] = t.nd;
      bc[7] = t.nfront;
      bc[8] = t.nret;
      bc[9] = (t.stop ? PUB_STOP : 0) | (t.quiescent ? PUB_QUIESCENT : 0) |
              (t.stall ? PUB_STALL : 0) | (t.err << 8);
    }
  }
  lds_sync();
  RoundState rs;
  const int B = blockDim.x;
  rs.done = bc[0] != 0;
  rs.r = bc[1];
  rs.n = bc[3];
  rs.fs0 = bc[4];
  rs.fs1 = bc[5];
  rs.nd = bc[6];
  rs.nfront = bc[7];
  rs.nret = bc[8];
  rs.stop = bc[9] & PUB_STOP;
  rs.quiescent = bc[9] & PUB_QUIESCENT;
  rs.stall = bc[9] & PUB_STALL;
  rs.scanned = bc[9] & PUB_SCANNED;
  rs.scan_req = false;
  rs.err = bc[9] >> 8;
  rs.stamp = L.misc[29];
  lds_sync();
  tmark(a, L, rs.r, 0);
  // a scanned round is a list round: the scan listed the slots to examine
  // (nfront of them) and retired the markers
  rs.full = !rs.quiescent && !rs.scanned &&
            (a.mode == 0 || rs.nfront == 0 || rs.r == 0 || rs.stall ||
             (a.sweep_every > 0 && rs.r % a.sweep_every == 0));
  rs.nlist = rs.nd + (rs.full ? 0 : rs.nret + rs.nfront);
  rs.ntiles = rs.full ? (rs.n + B * a.npt - 1) / (B * a.npt) : 0;
  rs.need = max((rs.nlist + B - 1) / B, rs.ntiles);
  if (rs.ntiles <= 1 && rs.nlist <= a.small_cap) rs.need = 1;
  if (rs.stop) rs.need = 1;
  return rs;
}

// The round needs a larger grid than the launch's: more list items than
// grow_list (not for a scanned round: its scan has run), or in plain and
// learned modes a sweep (or a scan) of more than grow_full slots.  k_scan
// takes the same decision from the same published line, so a round whose
// scan was skipped is skipped too.
__device__ __forceinline__ bool grid_too_small(const RoundArgs &a, const RoundState &rs) {
  if (a.grow_list > 0 && !rs.scanned && rs.nlist > a.grow_list) return true;
  return a.grow_full > 0 && a.mode != 1 && (rs.full || rs.scanned) && rs.n > a.grow_full;
}

// Publish round nx for the next launch (one thread).
__device__ __forceinline__ void publish(Ctl *ctl, const RoundState &nx) {
  const int v[10] = {0,         nx.r,      nx.need,   nx.n,      nx.fs0,
                     nx.fs1,    nx.nd,     nx.nfront, nx.nret,
                     (nx.stop ? PUB_STOP : 0) | (nx.quiescent ? PUB_QUIESCENT : 0) |
                         (nx.stall ? PUB_STALL : 0) | (nx.scan_req ? PUB_SCAN_REQ : 0) |
                         (nx.err << 8)};
#pragma unroll
  for (int i = 0; i < 10; i++)
    __hip_atomic_store(&ctl->pub[i], v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Record the end of the run (thread 0 of workgroup 0).
__device__ __forceinline__ void round_stop(const RoundArgs &a, const RoundState &rs) {
  Ctl *ctl = a.ctl;
  ctl->done = 1;
  ctl->pub[0] = 1;
  ctl->done_round = rs.r;
  ctl->err = rs.err;
  ctl->n_final = rs.n;
  ctl->fs_final[0] = rs.fs0;
  ctl->fs_final[1] = rs.fs1;
}

// Execute round rs.r: bookkeeping by workgroup 0, then this workgroup's
// share of the lists and of the sweep.  Called only by workgroups below
// rs.need; tables must be in LDS.
template <int A>
__device__ __forceinline__ void round_execute(const RoundArgs &a, Lds &L, const RoundState &rs) {
  const Pool &p = a.p;
  Ctl *ctl = a.ctl;
  const int B = blockDim.x, tid = threadIdx.x, wg = blockIdx.x;
  const int r = rs.r, r3 = r % 3, mode = a.mode;
  const int n = rs.n, fs0 = rs.fs0, fs1 = rs.fs1, nd = rs.nd, nret = rs.nret, nfront = rs.nfront;
  const bool full = rs.full, quiescent = rs.quiescent;
  const int nlist = rs.nlist, ntiles = rs.ntiles, need = rs.need;
  const int G = gridDim.x;
  tmark(a, L, r, 1);
  if (a.wgtrace && r == a.wgtrace_round && tid == 0 && wg < 4096)
    a.wgtrace[wg * 8 + 4] = (long long)wall_clock64();
  if (wg == 0 && tid == 0) {
    st(&ctl->n[r3], n);
    st(&ctl->fs[r3][0], fs0);
    st(&ctl->fs[r3][1], fs1);
    RoundCnt *nx = &ctl->cnt[(r + 1) % 3];
    for (int32_t *w : {&nx->alloc, &nx->push, &nx->dead, &nx->active, &nx->err, &nx->front,
                       &nx->ret, &nx->full, &nx->prog, &nx->scan})
      st(w, 0);
    // (a scanned round examined every slot; the scan counted its visits)
    st(&ctl->cnt[r3].full, (full || quiescent || rs.scanned) ? 1 : 0);
    if (rs.scanned && L.misc[28]) st(&ctl->cnt[r3].active, 1);
    if ((unsigned long long)n > L.lstat[LSTAT_PEAK]) L.lstat[LSTAT_PEAK] = n;
    if (nd > 0) L.lstat[LSTAT_GC]++;
    if (full) L.lstat[LSTAT_FULL]++;
    if (!rs.scanned) L.lstat[STAT_VISITS] += (unsigned long long)(full ? n : nfront);
  }
  // the first `need` workgroups run the round; list items and tiles are
  // strided over exactly those
  const int Ga = min(G, need);
  RoundCnt *cnt = &ctl->cnt[r3];
  Counters C = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  RoundCtx R;
  R.r = r;
  R.n = n;
  R.e = (unsigned)(r & 1);
  R.mode = mode;
  // A walk or a further pass lengthens the round for every term, so rounds
  // that several workgroups run (many terms or nodes at work) take the
  // short settings, and rounds that one workgroup runs alone (a few chains
  // left) the long ones.
  const bool narrow = need == 1;
  R.walk_max = narrow ? a.nf_walk : a.nf_walk_wide;
  R.cont = narrow ? a.cont_passes : a.cont_passes_wide;
  R.walk = R.walk_max > 0 && mode != 0 && !full && !quiescent;
  R.cbuf = (R.walk && R.cont > 0) ? 0 : -1;
  R.cnt = cnt;
  R.stamp = rs.stamp + r;
  R.SP = (r & 1) ? p.fstack1 : p.fstack0;
  R.fsP = (r & 1) ? fs1 : fs0;
  R.room = fresh_room(a, n);
  int32_t *SQ = ((r + 1) & 1) ? p.fstack1 : p.fstack0;
  const int fsQ = ((r + 1) & 1) ? fs1 : fs0;
  // A workgroup that runs the round alone is the only one to claim slots
  // and append to the round's lists, so it counts them in LDS (an LDS
  // atomic instead of a global one on each pass's dependent chain) and
  // stores the totals once, at the end of the round.
  const bool solo = Ga == 1;
  int32_t *lc = L.misc + LC_SLOT;  // alloc, push, dead, front, retire
  if (solo) {
    if (tid < 5) lc[tid] = 0;
    lds_sync();
  }
  L.solo = solo;
  L.qd.out = (r & 1) ? p.dead1 : p.dead0;
  L.qd.gcount = &cnt->dead;
  L.qf.out = (r & 1) ? p.front1 : p.front0;
  L.qf.gcount = &cnt->front;
  L.qr.out = (r & 1) ? p.ret1 : p.ret0;
  L.qr.gcount = &cnt->ret;
  const int32_t *D = ((r - 1) & 1) ? p.dead1 : p.dead0;
  const int32_t *F = ((r - 1) & 1) ? p.front1 : p.front0;
  const int32_t *RT = ((r - 1) & 1) ? p.ret1 : p.ret0;
  const unsigned ep = (unsigned)((r - 1) & 1);

  tmark(a, L, r, 2);
  // ---- 1. list items: collection, marker retirement, frontier slots.  In
  // a full round the list holds only the dead nodes, and their collection
  // is deferred to the sweep's last passes, where it runs beside the
  // examination of the swept slots (one dependent chain instead of two; the
  // order of the two within a round does not matter, since dead nodes are
  // normal forms, which the sweep never examines)
  const bool defer_dead = full && ntiles > 0;
  {
    const int nr_here = full ? 0 : nret;
    for (int base = wg * B; base < (defer_dead ? 0 : nlist); base += Ga * B) {
      const int i = base + tid;
      int s = 0, memo = 0, fslot = 0;
      Pre<A> pre;
      pre.have = false;
      if (i < nd) {
        fslot = collect<A>(a, L, cnt, D[i], C);
      } else if (i < nd + nr_here) {
        const int x = RT[i - nd];
        if ((unsigned)x < (unsigned)p.N && x > 0) retire_marker(p.state, x, ep);
      } else if (i < nlist) {
        int x;
        if (rs.scanned) {
          // the scan's lists: item f of the combined list is in list j with
          // scan_off[j] <= f < scan_off[j + 1]
          const int f = i - nd - nr_here;
          int j = 0;
          for (int k = 1; k < a.scan_lists; k++) j += f >= L.soff[k] ? 1 : 0;
          const int32_t *lst = ((j < 8) ? p.front0 : p.front1) + (int64_t)(j & 7) * a.scan_rs;
          x = lst[f - L.soff[j]];
        } else {
          x = F[i - nd - nr_here];
        }
        if ((unsigned)x < (unsigned)p.N && x > 0) {
          unsigned st = p.state[x];
          // queued slots are mostly live and not normal forms: their
          // symbol, entries and parent hint are read with the state, one
          // dependent read less
          pre.have = true;
          pre.f = p.hss[x];
#pragma unroll
          for (int j = 0; j < A; j++) pre.raw[j] = p.args[(int64_t)x * A + j];
          pre.par = R.mode != 0 ? p.par[x] : 0;
          pre.lc = (R.mode == 2 || a.trace_rate) ? p.lastchg[x] : 0;
          if ((st & ST_PEND) && ((st >> 2) & 1u) != R.e) {  // retire its own marker
            st = (st & ST_NF) ? ST_NF : ST_ACTIVE;
            p.state[x] = (uint8_t)st;
          }
          if ((st & ST_ACTIVE) && !(st & ST_PEND)) {
            // a queued node gets the full readiness test at once: it is
            // mostly ready, and its memo would only add two dependent reads
            s = x;
            memo = (int)((st & ST_MEMO_MASK) >> ST_MEMO_SHIFT);
          }
        }
      }
      // (a scanned round's listed slots were counted as live by the scan)
      process_slot<A>(a, L, R, s, memo, rs.scanned, fslot, SQ, fsQ, C, pre);
    }
  }

  // ---- same-round continuation (list rounds with the walk): the ready
  // nodes this workgroup created in the passes above (their arguments are
  // normal forms visible in this round: matched nodes, or nodes born normal
  // in the same rewrite), and the roots it rewrote that are ready again,
  // are examined now instead of next round, pass after pass, while any are
  // left and at most R.cont times.  Nothing outside this workgroup
  // knows these nodes in this round (no list of the round holds them, and
  // the walk never marks a node that has rules), so no other thread
  // examines or writes them; the workgroup's own global writes of the last
  // pass are complete and visible to all its waves after the barrier.
  // Pass k examines buffer k mod 2 and appends to the other one; what is
  // left when the passes run out goes to the next round's frontier.
  if (R.cbuf >= 0) {
    for (int pass = 0;; pass++) {
      __syncthreads();
      const int k = pass & 1;
      int32_t *cb = k ? L.cb1 : L.cb0;
      const int nc = min(L.misc[k ? 27 : 7], L.ccap);
      if (nc == 0) break;
      if (pass >= R.cont) {
        // the rest: one reservation on the frontier, then the copy
        if (tid == 0) {
          if (L.solo) {
            L.misc[4] = L.misc[L.qf.lc];
            L.misc[L.qf.lc] += nc;
          } else {
            L.misc[4] = atomicAdd(L.qf.gcount, nc);
          }
        }
        __syncthreads();
        const int gb = L.misc[4];
        for (int i = tid; i < nc; i += B)
          if ((int64_t)gb + i < p.N) L.qf.out[gb + i] = cb[i];
        __syncthreads();
        if (tid == 0) L.misc[k ? 27 : 7] = 0;
        break;
      }
      R.cbuf = k ^ 1;
      if (tid == 0) L.lstat[STAT_VISITS] += (unsigned long long)nc;
      for (int b0 = 0; b0 < nc; b0 += B) {
        const int i = b0 + tid;
        int x = 0;
        Pre<A> pre;
        pre.have = false;
        if (i < nc) {
          const int v = cb[i];
          if ((unsigned)v < (unsigned)p.N && v > 0) {
            const unsigned st = p.state[v];
            pre.have = true;
            pre.f = p.hss[v];
#pragma unroll
            for (int j = 0; j < A; j++) pre.raw[j] = p.args[(int64_t)v * A + j];
            pre.par = p.par[v];
            pre.lc = (R.mode == 2 || a.trace_rate) ? p.lastchg[v] : 0;
            if ((st & (ST_ACTIVE | ST_PEND | ST_NF)) == ST_ACTIVE) x = v;
          }
        }
        process_slot<A>(a, L, R, x, 0, false, 0, SQ, fsQ, C, pre);
      }
      // (every thread read the count before the passes' barriers)
      if (tid == 0) L.misc[k ? 27 : 7] = 0;
    }
    R.cbuf = 0;
  }

  tmark(a, L, r, 3);
  const bool wgt = a.wgtrace && r == a.wgtrace_round && tid == 0 && wg < 4096;
  if (wgt) {
    a.wgtrace[wg * 8 + 0] = (long long)wall_clock64();
    a.wgtrace[wg * 8 + 6] = __smid();
  }
  int ntile_done = 0, nitems = 0;
  // ---- 2./3. full sweep of all slots below n, rewrite of the ready ones
  if (full) {
    const int npt = a.npt;
    const int TILE = B * npt;
    const unsigned e = R.e;
    const bool wake_sweep = a.mode == 0 && a.use_memo && !rs.stall;
    // with 16 slots per thread, the state (and in plain mode wake) bytes of
    // the next tile are copied into LDS while the current tile is worked
    // on (the bytes of a later tile cannot change meanwhile in a way that
    // matters: collection is over, and slots that become live this round
    // carry this round's marker)
    // tiles copied ahead into an LDS ring of pf_depth buffers (each: the
    // state bytes, then in plain mode the wake bytes)
    const int depth = a.pf_depth;
    const bool ahead = depth > 0;
    int t = xcd_remap(wg, Ga);
    auto pf_issue = [&](int tt, int b) {
      const int64_t b0 = (int64_t)tt * TILE + tid * 16;
      lds_fetch16(p.state + b0, pf_state(L, b));
      if (wake_sweep) lds_fetch4(p.wake + (b0 >> 4), pf_wake(L, b));
    };
    if (ahead) {
      for (int k = 0; k < depth; k++)
        if (t + k * Ga < ntiles) pf_issue(t + k * Ga, k);
    }
    int Wb = 0;  // work-list items carried over from earlier tiles
    // deferred dead-list items of this workgroup: dbase, dbase + Ga B, ...
    const int nd_def = defer_dead ? nd : 0;
    int dbase = wg * B;
    for (int it = 0; t < ntiles; t += Ga, it++) {
      const int b_cur = ahead ? it % depth : 0;  // ring buffer of this tile
      // (phase trace: fields 1 and 12-15 time the third tile of the sweep, in
      // steady state: its start, data in, classified, appended, examined)
      if (it == 2) tmark(a, L, r, 1);
      const int base = t * TILE + tid * npt;
      uint4 vs;
      unsigned ww = 0;  // wake bits of the thread's slots, two per slot
      if (ahead) {
        const int b = b_cur;
        // wait for this tile's copy.  The copies of the following tiles
        // issued so far (at most depth - 1) were the wave's last memory
        // operations -- each issued at the end of an iteration -- and the
        // wave's vector memory counter retires in issue order, so waiting
        // until only their one or two operations per tile remain leaves
        // them in flight.
        const int ahead_tiles = min(depth - 1, (ntiles - 1 - t) / Ga);
        vm_wait_tiles(ahead_tiles * (wake_sweep ? 2 : 1));
        vs = L.pf[b * B + tid];
        if (wake_sweep) ww = L.pfw[b * B + tid];
        // the entries are read before a later copy overwrites them
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (depth == 1 && t + Ga < ntiles) pf_issue(t + Ga, 0);  // reuses the only buffer
      } else {
        vs = load_bytes(p.state + base, npt);
        if (wake_sweep) ww = p.wake[base >> 4] >> (2 * (base & 15));
      }
      if (it == 2) tmark(a, L, r, 12);
      // state bytes of this thread's slots, kept in four registers
      ivec4 sw;
      sw[0] = (int)vs.x;
      sw[1] = (int)vs.y;
      sw[2] = (int)vs.z;
      sw[3] = (int)vs.w;
      // plain mode: the wake bits of the same slots, for the parity of the
      // previous rounds, packed into a 16-bit mask (a sleeping slot -- one
      // with a memo -- is tested again only once an argument has become a
      // normal form in an earlier round)
      int wmask = 0;
      if (wake_sweep) {
        wmask = even_bits(ww >> (1u - e));
        if (npt < 16) wmask &= (1 << npt) - 1;
      }
      // classification of the slots, four bytes at a time (SWAR), within
      // 0 < slot < n:
      //   pending  live and not in normal form: an unmarked live slot, or a
      //            marker of the previous round (retired on the way) that is
      //            not a normal form
      //   memoed   an unmarked live slot with a memo
      //   retire   a marker of the previous round (a marker of this round's
      //            parity was created this round and is left alone)
      int valid = npt < 16 ? (1 << npt) - 1 : 0xffff;
      if (base == 0) valid &= ~1;
      {
        const int lim = n - base;
        if (lim < npt) valid &= lim > 0 ? (1 << lim) - 1 : 0;
      }
      int pending = 0, memoed = 0, retire = 0;
      {
        const unsigned er = e ? 0x01010101u : 0u;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const unsigned x = (unsigned)sw[q];
          const unsigned pend = (x >> 1) & 0x01010101u;
          const unsigned prev = pend & (((x >> 2) & 0x01010101u) ^ er);
          const unsigned nf = (x >> 7) & 0x01010101u;
          const unsigned live = ((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) >> 7;  // low 7 bits not 0
          const unsigned normal = live & ~pend;
          const unsigned mem = ((x & 0x38383838u) + 0x78787878u) >> 7;   // memo bits not 0
          pending |= pack4(normal | (prev & ~nf)) << (4 * q);
          memoed |= pack4(normal & mem) << (4 * q);
          retire |= pack4(prev) << (4 * q);
        }
      }
      pending &= valid;
      retire &= valid;
      memoed = a.use_memo ? memoed & valid : 0;
      for (int m = retire; m; m &= m - 1) {
        const int j = __builtin_ctz(m);
        const unsigned st = ((unsigned)sw[j >> 2] >> ((j & 3) * 8)) & 0xffu;
        p.state[base + j] = (uint8_t)((st & ST_NF) ? ST_NF : ST_ACTIVE);
      }
      // off the wake path, the recorded arguments of the memoed slots are
      // read first, then all their states, so the loads overlap
      ivec16 cidx = (ivec16)(0);  // memo argument slot (0: none)
      if (!wake_sweep) {
        for (int m = memoed; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          const unsigned st = ((unsigned)sw[j >> 2] >> ((j & 3) * 8)) & 0xffu;
          const int memo = (int)((st & ST_MEMO_MASK) >> ST_MEMO_SHIFT);
          const int c = p.args[(int64_t)(base + j) * A + (memo - 1)];
          cidx[j] = ((unsigned)c < (unsigned)p.N) ? c : 0;
        }
      }
      if (it == 2) tmark(a, L, r, 13);
      // sleeping slots that stay asleep: no wake bit of an earlier round
      // (plain mode), or the memo argument still not a visible normal form
      int still = 0;
      if (wake_sweep) {
        still = memoed & ~wmask;
        // honour (clear) the wake bits of the previous rounds' parity that
        // wake a slot; a bit set in this round stays for the next one
        for (int m = memoed & wmask; m; m &= m - 1) {
          const int slot = base + __builtin_ctz(m);
          atomicAnd(&p.wake[slot >> 4], ~(1u << (((slot & 15) << 1) | (1u - e))));
        }
      } else if (memoed) {
        ivec16 cst = (ivec16)(0);
        for (int m = memoed; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          if (cidx[j]) cst[j] = p.state[cidx[j]];
        }
        for (int m = memoed; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          if (cidx[j] && !nf_visible((unsigned)cst[j], e)) still |= 1 << j;
        }
      }
      C.active += __popc(pending);
      C.memo += __popc(still);  // still blocked by the same argument
      // the slots of this thread to examine
      const int exam = pending & ~still;
      // append them to the LDS work list behind the Wb waiting items: a
      // wave prefix sum of the counts and one LDS atomic per wave (waves
      // with nothing to append skip both); the tile's count is kept in one
      // of three rotating LDS counters, so one barrier per tile suffices
      // (counter it+2 is cleared after this tile's barrier: every wave has
      // read it in tile it-1, and none appends to it before tile it+2)
      int32_t *tcount = L.misc + 24 + it % 3;
      if (__ballot(exam != 0)) {
        const int cnt = __popc(exam);
        const int incl = wave_incl_scan(cnt);
        const int tot = __shfl(incl, 63, 64);
        int wb = 0;
        if (lane() == 63) wb = atomicAdd(tcount, tot);
        int pos = Wb + __shfl(wb, 63, 64) + incl - cnt;
        for (int m = exam; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          const unsigned byte = ((unsigned)sw[j >> 2] >> ((j & 3) * 8)) & 0xffu;
          const int memo = ((byte & ST_PEND) || !a.use_memo)
                               ? 0
                               : (int)((byte & ST_MEMO_MASK) >> ST_MEMO_SHIFT);
          L.work[pos++] = (base + j) | (memo << 29);
        }
      }
      lds_sync();
      int W = Wb + *tcount;
      if (tid == 0) L.misc[24 + (it + 2) % 3] = 0;
      if (it == 2) tmark(a, L, r, 14);
      // examine in full passes of B slots while at least B are waiting; the
      // rest carries over to the next tile (the list holds a tile plus B),
      // and after the last tile everything is examined
      const bool last = t + Ga >= ntiles;
      while (W >= B || (last && (W > 0 || dbase < nd_def))) {
        // (process_slot's barriers order these reads before later appends
        // over the same entries)
        const int take = min(W, B);
        const int wv = tid < take ? L.work[W - take + tid] : 0;
        int fslot = 0;
        if (last && dbase < nd_def) {  // deferred collection, beside the last passes
          if (dbase + tid < nd_def) fslot = collect<A>(a, L, cnt, D[dbase + tid], C);
          dbase += Ga * B;
        }
        Pre<A> none;
        none.have = false;
        process_slot<A>(a, L, R, wv & 0x1fffffff, (int)((unsigned)wv >> 29), true, fslot, SQ,
                        fsQ, C, none);
        W -= take;
      }
      Wb = W;
      if (it == 2) tmark(a, L, r, 15);
      ntile_done++;
      nitems += exam ? __popc(exam) : 0;
      // two or more buffers: the tile depth strides ahead goes into the one
      // just read, as the iteration's last memory operation
      if (depth >= 2 && t + depth * Ga < ntiles) pf_issue(t + depth * Ga, b_cur);
    }
    // a workgroup without tiles still collects its share of the dead list
    while (dbase < nd_def) {
      int fslot = 0;
      if (dbase + tid < nd_def) fslot = collect<A>(a, L, cnt, D[dbase + tid], C);
      dbase += Ga * B;
      Pre<A> none;
      none.have = false;
      process_slot<A>(a, L, R, 0, 0, true, fslot, SQ, fsQ, C, none);
    }
  }

  tmark(a, L, r, 4);
  if (wgt) {
    a.wgtrace[wg * 8 + 1] = (long long)wall_clock64();
    a.wgtrace[wg * 8 + 2] = ntile_done;
    a.wgtrace[wg * 8 + 3] = nitems;
  }
  // ---- per-workgroup statistics: wave sums, added by one lane per wave to
  // the workgroup's LDS totals; only the liveness flag of the round goes to
  // global memory
  {
    const int sa = wave_sum(C.active), sr = wave_sum(C.ready), sf = wave_sum(C.fired);
    const int sn = wave_sum(C.nfset), sl = wave_sum(C.alloc), sd = wave_sum(C.freed);
    const int so = wave_sum(C.rcops), sm = wave_sum(C.memo);
    const int sp = wave_sum(C.mlp), sk = wave_sum(C.keep), st = wave_sum(C.trace);
    const int sw = wave_sum(C.walk);
    if (lane() == 0) {
      if (sa) {
        L.misc[32] = 1;
        atomicAdd(&L.lstat[STAT_ACTIVE], (unsigned long long)sa);
      }
      if (sf || sn || sw) L.misc[33] = 1;
      if (sr) atomicAdd(&L.lstat[STAT_READY], (unsigned long long)sr);
      if (sf) atomicAdd(&L.lstat[STAT_FIRED], (unsigned long long)sf);
      if (sn) atomicAdd(&L.lstat[STAT_NFSET], (unsigned long long)sn);
      if (sl) atomicAdd(&L.lstat[STAT_ALLOC], (unsigned long long)sl);
      if (sd) atomicAdd(&L.lstat[STAT_FREED], (unsigned long long)sd);
      if (so) atomicAdd(&L.lstat[STAT_RCOPS], (unsigned long long)so);
      if (sm) atomicAdd(&L.lstat[STAT_MEMO], (unsigned long long)sm);
      if (sp) atomicAdd(&L.lstat[STAT_MLP], (unsigned long long)sp);
      if (sk) atomicAdd(&L.lstat[STAT_KEEP], (unsigned long long)sk);
      if (st) atomicAdd(&L.lstat[STAT_TRACE], (unsigned long long)st);
      if (sw) atomicAdd(&L.lstat[STAT_WALK], (unsigned long long)sw);
    }
  }
  lds_sync();
  // the round's two flags: stored here by a workgroup running the round
  // alone (it may go on to the next round itself) and in the persistent
  // form (nrounds > 0: no tickets); otherwise they travel with the
  // end-of-launch tickets (a store per workgroup to one address would
  // serialise)
  if (tid == 0 && (Ga == 1 || a.nrounds > 0)) {
    if (L.misc[32]) st(&cnt->active, 1);
    if (L.misc[33]) {
      st(&cnt->prog, 1);
      st(&ctl->last_prog, r);
    }
    L.misc[32] = L.misc[33] = 0;
  }
  if (tid == 0) L.misc[24] = L.misc[25] = L.misc[26] = 0;  // the sweep's tile counters
  if (solo && tid == 0) {
    // (the round's counts, for the derivation of the next round)
    st(&cnt->alloc, lc[0]);
    st(&cnt->push, lc[1]);
    st(&cnt->dead, lc[2]);
    st(&cnt->front, lc[3]);
    st(&cnt->ret, lc[4]);
  }
  // end of the round: every wave's global writes complete before the
  // workgroup goes on (workgroup 0 may run the next round itself)
  __syncthreads();
  tmark(a, L, r, 5);
  if (a.wgtrace && r == a.wgtrace_round && tid == 0 && wg < 4096)
    a.wgtrace[wg * 8 + 5] = (long long)wall_clock64();
}

// Add this workgroup's statistics of the launch to the control block (once,
// at the end of the launch).
// Threads t0, t0 + 1, ... add the statistics to the control block (no
// barrier: the caller has synchronised the workgroup).
__device__ __forceinline__ void stats_out(const RoundArgs &a, const Lds &L, int t0) {
  Ctl *ctl = a.ctl;
  const int wg = blockIdx.x, tid = threadIdx.x;
  if (tid < t0) return;
  if (tid == t0) {
    const int sp = wg & (CTL_SPREAD - 1);
    for (int k = 0; k < CTL_NSTAT; k++)
      if (L.lstat[k]) atomicAdd(&ctl->stat[sp][k], L.lstat[k]);
    if (L.lstat[LSTAT_GC]) atomicAdd((unsigned *)&ctl->gc_rounds, (unsigned)L.lstat[LSTAT_GC]);
    if (L.lstat[LSTAT_FULL])
      atomicAdd((unsigned *)&ctl->full_sweeps, (unsigned)L.lstat[LSTAT_FULL]);
    if (L.lstat[LSTAT_PEAK]) atomicMax(&ctl->peak_n, (int)L.lstat[LSTAT_PEAK]);
  }
  for (int i = tid - t0; i < a.n_rules; i += blockDim.x - t0) {
    const int c = L.rcnt[i];
    if (c) atomicAdd(&ctl->rule_apps[wg & (RULE_SPREAD - 1)][i], (unsigned long long)c);
  }
}

__device__ __forceinline__ void flush_stats(const RoundArgs &a, const Lds &L) {
  lds_sync();
  stats_out(a, L, 0);
}

__device__ __forceinline__ Lds setup_lds(const RoundArgs &a, int32_t *smem, bool load_tab) {
  Lds L;
  const int B = blockDim.x;
  L.tab = smem;
  L.work = L.tab + ((a.tab_words + 3) & ~3);
  int32_t *q = L.work + B * a.npt + B;  // a tile's slots plus a carried-over pass
  const int qc = a.qbuf * B;
  L.qd.buf = q;
  L.qf.buf = q + qc;
  L.qr.buf = q + 2 * qc;
  L.qd.cap_lds = L.qf.cap_lds = L.qr.cap_lds = qc;
  L.qd.slot = 1;
  L.qf.slot = 2;
  L.qr.slot = 3;
  L.qd.lc = LC_SLOT + 2;
  L.qf.lc = LC_SLOT + 3;
  L.qr.lc = LC_SLOT + 4;
  L.solo = false;
  L.cb0 = q + 3 * qc;
  L.cb1 = q + 4 * qc;
  L.ccap = qc;
  L.pf = reinterpret_cast<uint4 *>(q + 5 * qc);
  L.pfw = reinterpret_cast<uint32_t *>(q + 5 * qc + 4 * B * a.pf_depth);
  L.misc = q + 5 * qc + 5 * B * a.pf_depth;
  L.lstat = reinterpret_cast<unsigned long long *>(L.misc + 64);
  L.tstamp = reinterpret_cast<unsigned long long *>(L.misc + 64 + 2 * 16);
  L.soff = L.misc + 64 + 2 * 16 + 2 * TRACE_FIELDS;
  L.rcnt = L.soff + 32;
  if (load_tab)
    for (int i = threadIdx.x; i < a.tab_words; i += B) L.tab[i] = a.tab[i];
  for (int i = threadIdx.x; i < 64 + 2 * 16 + 2 * TRACE_FIELDS + 32; i += B) L.misc[i] = 0;
  for (int i = threadIdx.x; i < a.n_rules; i += B) L.rcnt[i] = 0;
  lds_sync();
  return L;
}

__device__ __forceinline__ int bcast(const Lds &L, int v) {
  if (threadIdx.x == 0) L.misc[31] = v;
  lds_sync();
  const int x = L.misc[31];
  lds_sync();
  return x;
}


// One launch executes round ctl->r_cur on the whole grid.  When that round
// is small enough for one workgroup, workgroup 0 runs it alone and then keeps
// running the following rounds for as long as they stay small: every write
// of those rounds is its own, so no device-wide synchronisation is needed
// and their working set stays in its XCD's L2.  The last workgroup to finish
// advances ctl->r_cur past the last round executed.
// (compiled twice: for workgroups of up to 256 threads, which frontier and
// list rounds use, the register budget is four times that of the
// 1024-thread form, so the rewrite's values need not spill)
template <int A, int MAXB>
__global__ void __launch_bounds__(MAXB) k_round(RoundArgs a) {
  extern __shared__ int32_t smem[];
  Ctl *ctl = a.ctl;
  Lds L = setup_lds(a, smem, false);
  const int wg = blockIdx.x, tid = threadIdx.x;
  // the first round of this launch, as published by the previous launch.
  // Workgroups beyond the number it uses leave at once, without reading any
  // round counter (workgroup 0 may be running later rounds alone) and
  // without a ticket, so a launch costs as many control atomics as
  // workgroups at work, however large its grid.
  RoundState rs = round_prepare(a, L, 0, true, true);
  const int r0 = rs.r;  // the launch's first round
  const bool scanned0 = rs.scanned;
  int rr_local = r0 + 1;  // the round the next launch starts with
  int r_exec = rs.r;    // the last round this workgroup executed (phase trace)
  if (rs.done) return;
  if (!rs.stop && grid_too_small(a, rs)) return;  // (every workgroup: same line)
  const int need0 = rs.need;
  if (wg >= need0) return;
  {
    if (rs.stop) {
      if (wg == 0 && tid == 0) round_stop(a, rs);
      return;
    }
    const bool alone = rs.need == 1;
    // one call site: the first round, then (workgroup 0 alone) the
    // following small rounds
    for (int k = 0;; k++) {
      round_execute<A>(a, L, rs);
      r_exec = rs.r;
      if (!alone || k + 1 >= a.cont_rounds) break;
      tflush(a, L, r_exec);
      rs = round_prepare(a, L, rs.r + 1, false);
      if (rs.stop) {
        flush_stats(a, L);
        if (tid == 0) round_stop(a, rs);
        return;
      }
      if (rs.need != 1) {
        if (tid == 0 && a.trace_max) L.tstamp[0] = 0;  // a round left to the next launch
        break;
      }
    }
    // (workgroup 0 alone: the round after the last one it ran)
    if (alone) rr_local = max(r0 + 1, rs.stop || rs.need == 1 ? rs.r + 1 : rs.r);
  }
  // Every wave waits for its own memory operations of the launch (the round
  // counters' fetch-adds among them) to complete before the workgroup takes
  // its ticket, so the workgroup that draws the last ticket sees every
  // count.  Nothing else of this launch is read by another workgroup before
  // the launch ends, so no agent-scope fence is needed here: on gfx950 that
  // fence writes back and invalidates the whole L2 of the XCD, and taken by
  // each of thousands of workgroups per round it cost more than the sweep.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // the launch's statistics: only the host reads them, after the run, so
  // the waves after the first add them while the first takes the ticket
  // (with one wave, after the ticket)
  const int t_stats = blockDim.x > 64 ? 64 : 0;
  if (t_stats) stats_out(a, L, t_stats);
  if (tid == 0) {
    int flags = (L.misc[32] ? 1 : 0) | (L.misc[33] ? 2 : 0);  // (set only by rounds run by more
                                                               // than one workgroup)
    if (last_ticket(ctl, wg, min(need0, (int)gridDim.x), &flags)) {
      if (flags) {
        RoundCnt *c0 = &ctl->cnt[r0 % 3];
        if (flags & 1) st(&c0->active, 1);
        if (flags & 2) {
          st(&c0->prog, 1);
          st(&ctl->last_prog, r0);
        }
      }
      if (scanned0) {
        // every workgroup read the scan's counts at launch start: clear them
        // for the next scan
        for (int j = 0; j < a.scan_lists; j++) {
          st(&ctl->scan_cnt[j][0], 0);
          st(&ctl->scan_cnt[j][1], 0);
        }
      }
      // last working workgroup of the launch: every round it covered is
      // complete.  It reads only counters kept with agent-scope atomics, so
      // it needs no fence either.  (With more than one workgroup the launch
      // ran round r0 alone; with one, that workgroup is this one.)
      const int rr = rr_local;
      const RoundState nx = round_state(a, rr);
      publish(ctl, nx);
      if (a.trace_max)
        L.tstamp[11] = wall_clock64();
      else
        tmark_any(a, rr - 1, 11);
      __hip_atomic_store(&ctl->next_need, nx.need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->r_cur, rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    tflush(a, L, r_exec);
  }
  if (!t_stats) stats_out(a, L, 0);
}

// Device-wide barrier for the persistent kernel.  The host zeroes *bar
// before every launch; barrier k completes when all G workgroups have
// arrived, i.e. when *bar reaches G*(k+1).  The wait is bounded: past the
// bound the workgroup raises ctl->abort, every waiting workgroup sees it and
// the whole grid leaves the kernel (the host reports an internal error).
__device__ __forceinline__ bool grid_barrier(unsigned long long *bar, unsigned long long target,
                                             int32_t *abort_flag, int32_t *lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ab = 0;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ab = 1;
        break;
      }
      if (++spins > (1u << 21)) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ab = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    *lds_flag = ab;
  }
  __syncthreads();
  return *lds_flag == 0;
}

// Plain mode, a large full round r: the classification of every slot below n
// that k_round's sweep would make, as a kernel of its own.  Markers of the
// previous round are retired, woken sleepers' wake bits cleared, and the
// slots to examine listed: gathered in LDS per workgroup and appended at the
// end with one fetch-add on the counter of list wg mod scan_lists (each on a
// line of its own; a wave that finds the LDS buffer full appends its excess
// directly).  The last workgroup publishes the lists' offsets and turns the
// round into a list round of the dead nodes and the listed slots, which the
// following k_round launch examines.  No rewrite code, so few registers; it
// does nothing unless the round was published with a scan request.
template <int A>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan(RoundArgs a) {
  Ctl *ctl = a.ctl;
  const Pool &p = a.p;
  __shared__ int32_t sbuf[SCAN_CAP];
  __shared__ int s_cnt, s_base;
  __shared__ unsigned long long s_act, s_still;
  const int tid = threadIdx.x;
  const int4 *pp = reinterpret_cast<const int4 *>(ctl->pub);
  const int4 x = pp[0], z = pp[2];  // done r need n | (pp[1]) | nret flags
  if (x.x != 0) return;
  const int flags = z.y;
  if (!(flags & PUB_SCAN_REQ) || (flags & (PUB_SCANNED | PUB_STOP))) return;
  const int r = x.y, n = x.w;
  if (a.grow_full > 0 && n > a.grow_full) return;  // k_round skips the round too
  const unsigned e = (unsigned)(r & 1);
  const int S = a.scan_lists, lj = (int)blockIdx.x & (S - 1);
  int32_t *list = ((lj < 8) ? p.front0 : p.front1) + (int64_t)(lj & 7) * a.scan_rs;
  int32_t *lcnt = &ctl->scan_cnt[lj][0];
  if (tid == 0) {
    s_cnt = 0;
    s_act = 0;
    s_still = 0;
  }
  __syncthreads();
  constexpr int TS = SCAN_BLOCK * SCAN_NPT;
  const int ntiles = (n + TS - 1) / TS;
  int act = 0, still_n = 0;
  // one tile's classification and listing (all lanes of the workgroup)
  auto tile = [&](const int base, const uint4 vs, const unsigned ww) {
    int valid = 0xffff;
    if (base == 0) valid &= ~1;
    {
      const int lim = n - base;
      if (lim < SCAN_NPT) valid &= lim > 0 ? (1 << lim) - 1 : 0;
    }
    int pending = 0, memoed = 0, retire = 0;
    {
      const unsigned er = e ? 0x01010101u : 0u;
      const unsigned w4[4] = {vs.x, vs.y, vs.z, vs.w};
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const unsigned xw = w4[q];
        const unsigned pend = (xw >> 1) & 0x01010101u;
        const unsigned prev = pend & (((xw >> 2) & 0x01010101u) ^ er);
        const unsigned nf = (xw >> 7) & 0x01010101u;
        const unsigned live = ((xw & 0x7f7f7f7fu) + 0x7f7f7f7fu) >> 7;
        const unsigned normal = live & ~pend;
        const unsigned mem = ((xw & 0x38383838u) + 0x78787878u) >> 7;
        pending |= pack4(normal | (prev & ~nf)) << (4 * q);
        memoed |= pack4(normal & mem) << (4 * q);
        retire |= pack4(prev) << (4 * q);
      }
    }
    pending &= valid;
    memoed &= valid;
    retire &= valid;
    for (int m = retire; m; m &= m - 1) {
      const int j = __builtin_ctz(m);
      const unsigned wj = (j >> 2) == 0 ? vs.x : (j >> 2) == 1 ? vs.y : (j >> 2) == 2 ? vs.z : vs.w;
      const unsigned stb = (wj >> ((j & 3) * 8)) & 0xffu;
      p.state[base + j] = (uint8_t)((stb & ST_NF) ? ST_NF : ST_ACTIVE);
    }
    const int wmask = even_bits(ww >> (1u - e));
    const int still = memoed & ~wmask;
    for (int m = memoed & wmask; m; m &= m - 1) {
      const int slot = base + __builtin_ctz(m);
      atomicAnd(&p.wake[slot >> 4], ~(1u << (((slot & 15) << 1) | (1u - e))));
    }
    act += __popc(pending);
    still_n += __popc(still);
    const int exam = pending & ~still;
    if (__ballot(exam != 0)) {
      const int c = __popc(exam);
      const int incl = wave_incl_scan(c);
      const int tot = __shfl(incl, 63, 64);
      int wb = 0;
      if (lane() == 63) wb = atomicAdd(&s_cnt, tot);
      wb = __shfl(wb, 63, 64);
      // positions at or past the LDS capacity go straight to the list
      const int lo = max(wb, SCAN_CAP);
      const int ovf = max(0, wb + tot - lo);
      int gb = 0;
      if (ovf > 0) {
        if (lane() == 63) gb = atomicAdd(lcnt, ovf);
        gb = __shfl(gb, 63, 64);
      }
      int pos = wb + incl - c;
      for (int m = exam; m; m &= m - 1, pos++) {
        const int v = base + __builtin_ctz(m);
        if (pos < SCAN_CAP)
          sbuf[pos] = v;
        else
          list[gb + (pos - lo)] = v;
      }
    }
    };
  // four tiles per iteration: their bytes are requested before any is
  // classified, so each wave keeps four loads in flight
  constexpr int U = 4;
  const int G = gridDim.x;
  for (int t = blockIdx.x; t < ntiles; t += U * G) {
    uint4 vs[U];
    unsigned ww[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      vs[u] = make_uint4(0, 0, 0, 0);
      ww[u] = 0;
      if (t + u * G < ntiles) {
        const int b = (t + u * G) * TS + tid * SCAN_NPT;
        vs[u] = *reinterpret_cast<const uint4 *>(p.state + b);
        ww[u] = p.wake[b >> 4];
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (t + u * G < ntiles) tile((t + u * G) * TS + tid * SCAN_NPT, vs[u], ww[u]);
  }
  {
    const int sa = wave_sum(act), ss = wave_sum(still_n);
    if (lane() == 0) {
      if (sa) atomicAdd(&s_act, (unsigned long long)sa);
      if (ss) atomicAdd(&s_still, (unsigned long long)ss);
    }
  }
  __syncthreads();
  // the workgroup's gathered slots: one fetch-add on its list's counter
  const int n_lds = min(s_cnt, SCAN_CAP);
  if (tid == 0) s_base = n_lds > 0 ? atomicAdd(lcnt, n_lds) : 0;
  __syncthreads();
  for (int i = tid; i < n_lds; i += blockDim.x) list[s_base + i] = sbuf[i];
  if (tid == 0) {
    const int sp = blockIdx.x & (CTL_SPREAD - 1);
    if (s_act) atomicAdd(&ctl->stat[sp][STAT_ACTIVE], s_act);
    if (s_still) atomicAdd(&ctl->stat[sp][STAT_MEMO], s_still);
    if (blockIdx.x == 0) {
      atomicAdd(&ctl->stat[sp][STAT_VISITS], (unsigned long long)n);
      atomicAdd((unsigned *)&ctl->full_sweeps, 1u);
    }
  }
  // the flag that a live non-normal-form slot was met, on the line of the
  // workgroup's list (the round kernel that follows reads the counts and
  // flags at launch start; the kernel boundary orders them)
  if (tid == 0 && s_act) st(&ctl->scan_cnt[lj][1], 1);
}

template <int A>
__global__ void __launch_bounds__(1024) k_persistent(RoundArgs a) {
  extern __shared__ int32_t smem[];
  Ctl *ctl = a.ctl;
  if (ld(&ctl->done) || ld(&ctl->abort)) return;
  Lds L = setup_lds(a, smem, true);
  const unsigned long long G = gridDim.x;
  if (threadIdx.x == 0) L.misc[29] = ld(&ctl->stamp_base);  // (read by round_prepare)
  const int r0 = bcast(L, threadIdx.x == 0 ? ld(&ctl->r_cur) : 0);
  int r = r0;
  for (int k = 0; k < a.nrounds; k++, r++) {
    RoundState rs = round_prepare(a, L, r, false);
    if (rs.stop) {
      flush_stats(a, L);
      if (blockIdx.x == 0 && threadIdx.x == 0) round_stop(a, rs);
      return;
    }
    if ((int)blockIdx.x < rs.need) round_execute<A>(a, L, rs);
    if (!grid_barrier(a.bar, G * (unsigned long long)(k + 1), &ctl->abort, &L.misc[63])) {
      flush_stats(a, L);
      return;
    }
  }
  flush_stats(a, L);
  // every workgroup read r_cur before the first barrier
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const RoundState nx = round_state(a, r);
    publish(ctl, nx);
    __hip_atomic_store(&ctl->r_cur, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->next_need, nx.need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

size_t trs_round_lds_bytes(int block, int npt, int tab_words, int n_rules, int pf_depth,
                           int qbuf) {
  size_t words = (size_t)((tab_words + 3) & ~3) + (size_t)block * npt + block +
                 (size_t)5 * qbuf * block + (size_t)5 * block * pf_depth + 64 + 2 * 16 +
                 2 * TRACE_FIELDS + 32 + (size_t)n_rules;
  return words * sizeof(int32_t);
}

#define DISPATCH_A(A, KERNEL, ...)                                   \
  switch (A) {                                                      \
    case 1: KERNEL<1>(__VA_ARGS__); break;                          \
    case 2: KERNEL<2>(__VA_ARGS__); break;                          \
    case 3: KERNEL<3>(__VA_ARGS__); break;                          \
    case 4: KERNEL<4>(__VA_ARGS__); break;                          \
    case 5: KERNEL<5>(__VA_ARGS__); break;                          \
    default: return hipErrorInvalidValue;                           \
  }

template <int A>
static void launch_round_A(const RoundArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  if (block <= 256)
    hipLaunchKernelGGL((k_round<A, 256>), dim3(grid), dim3(block), lds, s, a);
  else
    hipLaunchKernelGGL((k_round<A, 1024>), dim3(grid), dim3(block), lds, s, a);
}

static hipError_t g_coop_status = hipSuccess;

template <int A>
static void launch_pers_A(const RoundArgs &a, int grid, int block, size_t lds, hipStream_t s) {
  void *args[] = {(void *)&a};
  g_coop_status = hipLaunchCooperativeKernel((const void *)k_persistent<A>, dim3(grid),
                                             dim3(block), args, (unsigned)lds, s);
}

template <int A>
static void occ_A(int *out, int block, size_t lds) {
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_persistent<A>, block, lds);
}

template <int A>
static void set_attr_A(size_t lds) {
  (void)hipFuncSetAttribute((const void *)k_round<A, 256>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void *)k_round<A, 1024>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void *)k_persistent<A>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t trs_prepare_kernels(int A, size_t lds) {
  if (lds > 65536) DISPATCH_A(A, set_attr_A, lds);
  return hipSuccess;
}

template <int A>
static void launch_scan_A(const RoundArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_scan<A>, dim3(grid), dim3(SCAN_BLOCK), 0, s, a);
}

hipError_t trs_launch_scan(int A, const RoundArgs &a, int grid, hipStream_t s) {
  DISPATCH_A(A, launch_scan_A, a, grid, s);
  return hipGetLastError();
}

hipError_t trs_launch_round(int A, const RoundArgs &a, int grid, int block, hipStream_t s) {
  const size_t lds = trs_round_lds_bytes(block, a.npt, a.tab_words, a.n_rules, a.pf_depth, a.qbuf);
  DISPATCH_A(A, launch_round_A, a, grid, block, lds, s);
  return hipGetLastError();
}

hipError_t trs_launch_persistent(int A, const RoundArgs &a, int grid, int block, hipStream_t s) {
  const size_t lds = trs_round_lds_bytes(block, a.npt, a.tab_words, a.n_rules, a.pf_depth, a.qbuf);
  g_coop_status = hipSuccess;
  DISPATCH_A(A, launch_pers_A, a, grid, block, lds, s);
  if (g_coop_status != hipSuccess) return g_coop_status;
  return hipGetLastError();
}

template <int A>
static void occ_round_A(int *out, int block, size_t lds) {
  if (block <= 256)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_round<A, 256>, block, lds);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_round<A, 1024>, block, lds);
}

int trs_round_resident(int A, int block, size_t lds_bytes, int device) {
  int per_cu = 0;
  auto run = [&]() -> hipError_t {
    DISPATCH_A(A, occ_round_A, &per_cu, block, lds_bytes);
    return hipSuccess;
  };
  if (run() != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}

int trs_max_resident(int A, int block, size_t lds_bytes, int device) {
  int per_cu = 0;
  auto run = [&]() -> hipError_t {
    DISPATCH_A(A, occ_A, &per_cu, block, lds_bytes);
    return hipSuccess;
  };
  if (run() != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}
