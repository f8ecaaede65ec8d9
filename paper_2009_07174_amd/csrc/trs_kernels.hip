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
//   2. Sweep: every slot below n is examined (the topology-driven sweep of
//      Section 3).  A workgroup streams a tile of state bytes with vector
//      loads, retires round markers, and compacts the live non-normal-form
//      slots of the tile into an LDS work list.
//   3. Rewrite: the workgroup processes the work list densely.  A slot whose
//      arguments are all normal forms is matched against the rules of its
//      head symbol in priority order (Section 2, rewrite_f) using the
//      compiled per-symbol tables held in LDS; the first match is contracted
//      in place (Section 3): the right-hand-side root overwrites the slot,
//      new subterms go to slots taken from the free stack or past n, and
//      reference counts are adjusted, increments before decrements.  A slot
//      with no applicable rule becomes a normal form.
//
// Allocation takes one atomic per workgroup pass: a wave-level prefix sum of
// the per-lane node counts, then a workgroup scan of the wave totals, then a
// single fetch-add on the round's claim counter.  Claims below the free-stack
// size map to recycled slots, the rest to fresh slots n, n+1, ...  (the
// paper's get_new_index with next_free_begin / next_fresh, without per-thread
// atomics).  Dead-list appends are buffered in LDS and flushed with one
// atomic per pass.
//
// Round-to-round state lives in the device control block, triple-buffered by
// round (r % 3), so consecutive rounds need no host involvement and the
// persistent form needs a single device-wide barrier per round.
#include <hip/hip_runtime.h>

#include "trs_kernels.h"

#define MAXPAT 8
#define MAXNEW 8
#define DBUF_PER_THREAD 4

namespace {

__device__ __forceinline__ int lane() { return __lane_id(); }

// coherent read of a control word written by other workgroups or kernels
__device__ __forceinline__ int ld(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

struct Lds {
  int32_t *tab;
  int32_t *work;
  int32_t *dbuf;
  int32_t *misc;  // [0] work count [1] dbuf count [2] scratch base [3..18] wave sums
  int32_t *rcnt;  // per-rule application counts of this workgroup
  int dbuf_cap;
};

// Workgroup-wide reservation of m items on a global counter.  Returns this
// lane's first index.  Must be called by every thread of the workgroup.
__device__ __forceinline__ int wg_reserve(const Lds &L, int m, int32_t *counter) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = wave_incl_scan(m);
  if (lane() == 63) L.misc[3 + w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < nw; i++) {
      int t = L.misc[3 + i];
      L.misc[3 + i] = run;
      run += t;
    }
    L.misc[2] = run ? atomicAdd(counter, run) : 0;
  }
  __syncthreads();
  int base = L.misc[2] + L.misc[3 + w] + incl - m;
  __syncthreads();  // misc[2..] reused by the next call
  return base;
}

__device__ __forceinline__ void dead_push(const Lds &L, int32_t slot, int32_t *gcount,
                                          int32_t *dout, int64_t cap) {
  int i = atomicAdd(&L.misc[1], 1);
  if (i < L.dbuf_cap) {
    L.dbuf[i] = slot;
  } else {  // overflow of the LDS buffer: append directly
    int g = atomicAdd(gcount, 1);
    if (g < cap) dout[g] = slot;
  }
}

// Flush the LDS dead buffer to the global dead list (whole workgroup).
__device__ __forceinline__ void dead_flush(const Lds &L, int32_t *gcount, int32_t *dout,
                                           int64_t cap) {
  __syncthreads();
  int nb = min(L.misc[1], L.dbuf_cap);
  if (threadIdx.x == 0 && nb > 0) L.misc[2] = atomicAdd(gcount, nb);
  __syncthreads();
  if (nb > 0) {
    int gb = L.misc[2];
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
      if (gb + i < cap) dout[gb + i] = L.dbuf[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) L.misc[1] = 0;
  __syncthreads();
}

__device__ __forceinline__ int xcd_remap(int wg, int G) {
  // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so that its L2 sees neighbouring slots
  if (G & 7) return wg;
  return (wg & 7) * (G >> 3) + (wg >> 3);
}

struct Counters {
  int active, ready, fired, nfset, alloc, freed;
};

// visible normal form in round parity e (markers of the current parity are
// not yet valid)
__device__ __forceinline__ bool nf_visible(unsigned st, unsigned e) {
  return (st & ST_NF) && !((st & ST_PEND) && (((st >> 2) & 1u) == e));
}

template <int A>
__device__ __forceinline__ void process_slot(const RoundArgs &a, const Lds &L, int s, int n,
                                             int r, const int32_t *SP, int fsP, int32_t *dout,
                                             RoundCnt *cnt, Counters &C) {
  const Pool &p = a.p;
  const int32_t *tab = L.tab;
  const unsigned e = (unsigned)(r & 1);
  const int64_t N = p.N;
  bool have = s > 0;
  int info = 0, ar = 0;
  ivec8 av = (ivec8)(0);
  bool ready = false;
  if (have) {
    int f = p.hss[s];
    if ((unsigned)f >= (unsigned)a.n_sym) {
      cnt->err = -9;
      have = false;
    } else {
      info = tab[TAB_SYM + f];
      ar = info & 0xff;
      ready = true;
#pragma unroll
      for (int j = 0; j < A; j++) {
        if (j < ar) {
          int c = p.args[(int64_t)s * A + j];
          if ((unsigned)c >= (unsigned)N || c == 0) {
            cnt->err = -9;
            ready = false;
          }
          av[j] = c;
        }
      }
      if (ready) {
#pragma unroll
        for (int j = 0; j < A; j++)
          if (j < ar) ready = ready && nf_visible(p.state[av[j]], e);
      }
    }
  }
  C.active += have;
  int prog = -1;
  bool nfset = false;
  ivec16 ps = (ivec16)(0);  // ps[k]: slot matched by pattern node k (0 = the redex)
  ps[0] = s;
  if (ready) {
    C.ready++;
    const int nr = (info >> 8) & 0xff, first = info >> 16;
    if (nr == 0) {
      nfset = true;
    } else {
      ivec8 ch = (ivec8)(-1);
#pragma unroll
      for (int j = 0; j < A; j++)
        if (j < ar) ch[j] = p.hss[av[j]];
      const int32_t *rtab = tab + TAB_SYM + a.n_sym + first;
      for (int i = 0; i < nr && prog < 0; i++) {
        const int pg = rtab[i];
        const int npat = tab[pg] & 15;
        bool ok = true;
        for (int k = 1; k <= npat && ok; k++) {
          const int pe = tab[pg + 5 + k];
          const int par = pe & 15, pos = (pe >> 4) & 15;
          const bool isvar = (pe >> 8) & 1;
          int c, h = -1;
          if (par == 0) {
            c = av[pos];
            if (!isvar) h = ch[pos];
          } else {
            c = p.args[(int64_t)ps[par] * A + pos];
            if ((unsigned)c >= (unsigned)N || c == 0) {  // broken invariant: stop safely
              cnt->err = -9;
              c = ps[par];
              ok = false;
            }
            if (!isvar && ok) h = p.hss[c];
          }
          ps[k] = c;
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
  const int claim = wg_reserve(L, m, &cnt->alloc);
  ivec8 ns = (ivec8)(0);  // slots of the new nodes
  bool okalloc = true;
#pragma unroll
  for (int j = 0; j < MAXNEW; j++) {
    if (j < m) {
      const int c = claim + j;
      int64_t slot = (c < fsP) ? (int64_t)SP[fsP - 1 - c] : (int64_t)n + (c - fsP);
      if (slot >= N || slot <= 0) okalloc = false;
      ns[j] = (int)slot;
    }
  }
  if (prog >= 0 && !okalloc) {
    cnt->err = -5;  // TRS_E_POOL
    prog = -1;
  }
  const uint8_t pend_nf = (uint8_t)(ST_NF | ST_PEND | (e << 2));
  if (prog >= 0) {
    C.fired++;
    const int rsym = tab[prog + 1];
    const int ro = tab[prog + 2], no = tab[prog + 3], dl = tab[prog + 4], rid = tab[prog + 5];
    const bool var_root = (hdr >> 8) & 1, root_nf = (hdr >> 9) & 1;
    const int npos = (hdr >> 12) & 15, nneg = (hdr >> 16) & 15, rootpat = (hdr >> 20) & 15;
    // new nodes, children before parents
    int q = no;
    for (int j = 0; j < m; j++) {
      const int h = tab[q];
      const int sym = h & 0xffff, rci = (h >> 16) & 0xff, bnf = (h >> 24) & 1;
      const int ar2 = tab[TAB_SYM + sym] & 0xff;
      const int slot = ns[j];
#pragma unroll
      for (int o = 0; o < A; o++) {
        if (o < ar2) {
          const int v = tab[q + 1 + o];
          p.args[(int64_t)slot * A + o] = v >= 0 ? ps[v] : ns[-1 - v];
        }
      }
      p.hss[slot] = sym;
      p.rc[slot] = rci;
      p.state[slot] = bnf ? (uint8_t)ST_NF : (uint8_t)(ST_ACTIVE | ST_PEND | (e << 2));
      q += 1 + ar2;
    }
    // the redex root is overwritten in place
    if (var_root) {
      const int src = ps[rootpat];
      int sh = p.hss[src];
      if ((unsigned)sh >= (unsigned)a.n_sym) {
        cnt->err = -9;
        sh = 0;
      }
      const int sar = tab[TAB_SYM + sh] & 0xff;
#pragma unroll
      for (int j = 0; j < A; j++) {
        if (j < sar) {
          const int cj = p.args[(int64_t)src * A + j];
          p.args[(int64_t)s * A + j] = cj;
          if ((unsigned)cj < (unsigned)N)
            atomicAdd(&p.rc[cj], 1);
          else
            cnt->err = -9;
        }
      }
      p.hss[s] = sh;
      p.state[s] = pend_nf;
    } else {
      const int rar = tab[TAB_SYM + rsym] & 0xff;
#pragma unroll
      for (int o = 0; o < A; o++) {
        if (o < rar) {
          const int v = tab[ro + o];
          p.args[(int64_t)s * A + o] = v >= 0 ? ps[v] : ns[-1 - v];
        }
      }
      p.hss[s] = rsym;
      if (root_nf) p.state[s] = pend_nf;
    }
    // reference counts: increments first, then decrements (a decrement that
    // reaches zero puts the node on the dead list)
    for (int i = 0; i < npos; i++) {
      const int dw = tab[dl + i];
      atomicAdd(&p.rc[ps[dw & 0xff]], (int)(int8_t)((dw >> 8) & 0xff));
    }
    for (int i = 0; i < nneg; i++) {
      const int dw = tab[dl + npos + i];
      const int d = (int)(int8_t)((dw >> 8) & 0xff);
      const int slot = ps[dw & 0xff];
      const int old = atomicAdd(&p.rc[slot], d);
      if (old + d == 0) dead_push(L, slot, &cnt->dead, dout, N);
    }
    atomicAdd(&L.rcnt[rid], 1);
  } else if (nfset) {
    C.nfset++;
    p.state[s] = pend_nf;
  }
}

// The body of round r.  Returns false when the fixpoint was detected at the
// start of the round (uniformly for all workgroups).
template <int A>
__device__ bool round_body(const RoundArgs &a, const Lds &L, int r) {
  const Pool &p = a.p;
  Ctl *ctl = a.ctl;
  const int B = blockDim.x, tid = threadIdx.x, wg = blockIdx.x, G = gridDim.x;
  const int r3 = r % 3;
  int n, fs0, fs1, nd = 0;
  if (r == 0) {
    n = ld(&ctl->n[0]);
    fs0 = ld(&ctl->fs[0][0]);
    fs1 = ld(&ctl->fs[0][1]);
  } else {
    const int p3 = (r + 2) % 3;
    const int c_alloc = ld(&ctl->cnt[p3].alloc), c_push = ld(&ctl->cnt[p3].push);
    const int c_dead = ld(&ctl->cnt[p3].dead), c_act = ld(&ctl->cnt[p3].active);
    const int c_err = ld(&ctl->cnt[p3].err);
    const int pn = ld(&ctl->n[p3]), pf0 = ld(&ctl->fs[p3][0]), pf1 = ld(&ctl->fs[p3][1]);
    const int P = (r - 1) & 1;  // stack popped in round r-1
    const int fsP = P ? pf1 : pf0;
    const int used = min(c_alloc, fsP);
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
    const bool stop = c_err != 0 || (c_act == 0 && c_dead == 0) || nn > p.N;
    if (stop) {
      if (wg == 0 && tid == 0) {
        ctl->done = 1;
        ctl->done_round = r;
        ctl->err = c_err ? c_err : (nn > p.N ? -5 : 0);
        ctl->n_final = n;
      }
      return false;
    }
  }
  if (wg == 0 && tid == 0) {
    ctl->n[r3] = n;
    ctl->fs[r3][0] = fs0;
    ctl->fs[r3][1] = fs1;
    RoundCnt *nx = &ctl->cnt[(r + 1) % 3];
    nx->alloc = nx->push = nx->dead = nx->active = nx->err = nx->front = 0;
    if (n > ctl->peak_n) ctl->peak_n = n;
    if (nd > 0) ctl->gc_rounds++;
    ctl->stat[STAT_VISITS][0] += (unsigned long long)n;
  }
  RoundCnt *cnt = &ctl->cnt[r3];
  Counters C = {0, 0, 0, 0, 0, 0};
  int32_t *dout = (r & 1) ? p.dead1 : p.dead0;

  // ---- 1. collection of the previous round's dead nodes
  if (nd > 0) {
    const int32_t *D = ((r - 1) & 1) ? p.dead1 : p.dead0;
    int32_t *SQ = ((r + 1) & 1) ? p.fstack1 : p.fstack0;
    const int fsQ = ((r + 1) & 1) ? fs1 : fs0;
    for (int base = wg * B; base < nd; base += G * B) {
      const int i = base + tid;
      const bool v = i < nd;
      int d = v ? D[i] : 0;
      if (v && ((unsigned)d >= (unsigned)p.N || d == 0)) {
        cnt->err = -9;
        d = 0;
      }
      if (v && d) {
        const int f = p.hss[d];
        const int ar = ((unsigned)f < (unsigned)a.n_sym) ? (L.tab[TAB_SYM + f] & 0xff) : 0;
#pragma unroll
        for (int j = 0; j < A; j++) {
          if (j < ar) {
            const int c = p.args[(int64_t)d * A + j];
            const int old = atomicSub(&p.rc[c], 1);
            if (old == 1) dead_push(L, c, &cnt->dead, dout, p.N);
          }
        }
        p.state[d] = (uint8_t)ST_FREE;
        C.freed++;
      }
      const int pos = wg_reserve(L, (v && d) ? 1 : 0, &cnt->push);
      if (v && d) {
        if ((int64_t)fsQ + pos < p.N)
          SQ[fsQ + pos] = d;
        else
          cnt->err = -9;
      }
      dead_flush(L, &cnt->dead, dout, p.N);
    }
  }

  // ---- 2./3. sweep of all slots below n, rewrite of the ready ones
  const int npt = a.npt;
  const int TILE = B * npt;
  const int ntiles = (n + TILE - 1) / TILE;
  const unsigned e = (unsigned)(r & 1);
  const int32_t *SP = (r & 1) ? p.fstack1 : p.fstack0;
  const int fsP = (r & 1) ? fs1 : fs0;
  for (int t = xcd_remap(wg, G); t < ntiles; t += G) {
    const int base = t * TILE + tid * npt;
    // state bytes of this thread's slots, kept in four registers
    ivec4 sw = (ivec4)(0);
    if (npt == 16) {
      const uint4 v = *reinterpret_cast<const uint4 *>(p.state + base);
      sw[0] = (int)v.x;
      sw[1] = (int)v.y;
      sw[2] = (int)v.z;
      sw[3] = (int)v.w;
    } else if (npt == 8) {
      const uint2 v = *reinterpret_cast<const uint2 *>(p.state + base);
      sw[0] = (int)v.x;
      sw[1] = (int)v.y;
    } else if (npt == 4) {
      sw[0] = (int)*reinterpret_cast<const uint32_t *>(p.state + base);
    } else {
      for (int j = 0; j < npt; j++) sw[0] |= (int)p.state[base + j] << (8 * j);
    }
    for (int j = 0; j < npt; j++) {
      const int slot = base + j;
      const unsigned byte = ((unsigned)sw[j >> 2] >> ((j & 3) * 8)) & 0xffu;
      unsigned st = (slot < n && slot > 0) ? byte : 0u;
      if ((st & 0x7fu) == 0) continue;  // free or plain normal form
      if (st & ST_PEND) {
        if (((st >> 2) & 1u) == e) continue;  // created this round
        const uint8_t nst = (st & ST_NF) ? (uint8_t)ST_NF : (uint8_t)ST_ACTIVE;
        p.state[slot] = nst;
        if (nst == ST_NF) continue;
      }
      const int w = atomicAdd(&L.misc[0], 1);
      L.work[w] = slot;
    }
    __syncthreads();
    const int W = L.misc[0];
    for (int pb = 0; pb < W; pb += B) {
      const int idx = pb + tid;
      const int s = idx < W ? L.work[idx] : 0;
      process_slot<A>(a, L, s, n, r, SP, fsP, dout, cnt, C);
      dead_flush(L, &cnt->dead, dout, p.N);
    }
    __syncthreads();
    if (tid == 0) L.misc[0] = 0;
    __syncthreads();
  }

  // ---- per-workgroup statistics
  atomicAdd(&L.misc[20], C.active);
  atomicAdd(&L.misc[21], C.ready);
  atomicAdd(&L.misc[22], C.fired);
  atomicAdd(&L.misc[23], C.nfset);
  atomicAdd(&L.misc[24], C.alloc);
  atomicAdd(&L.misc[25], C.freed);
  __syncthreads();
  if (tid == 0) {
    const int sp = wg & (CTL_SPREAD - 1);
    if (L.misc[20]) {
      cnt->active = 1;
      atomicAdd(&ctl->stat[STAT_ACTIVE][sp], (unsigned long long)L.misc[20]);
    }
    if (L.misc[21]) atomicAdd(&ctl->stat[STAT_READY][sp], (unsigned long long)L.misc[21]);
    if (L.misc[22]) atomicAdd(&ctl->stat[STAT_FIRED][sp], (unsigned long long)L.misc[22]);
    if (L.misc[23]) atomicAdd(&ctl->stat[STAT_NFSET][sp], (unsigned long long)L.misc[23]);
    if (L.misc[24]) atomicAdd(&ctl->stat[STAT_ALLOC][sp], (unsigned long long)L.misc[24]);
    if (L.misc[25]) atomicAdd(&ctl->stat[STAT_FREED][sp], (unsigned long long)L.misc[25]);
    for (int i = 0; i < 20; i++) L.misc[20 + i] = 0;
  }
  for (int i = tid; i < a.n_rules; i += B) {
    const int c = L.rcnt[i];
    if (c) {
      atomicAdd(&ctl->rule_apps[i][wg & 3], (unsigned long long)c);
      L.rcnt[i] = 0;
    }
  }
  __syncthreads();
  return true;
}

__device__ __forceinline__ Lds setup_lds(const RoundArgs &a, int32_t *smem) {
  Lds L;
  const int B = blockDim.x;
  L.tab = smem;
  L.work = L.tab + ((a.tab_words + 3) & ~3);
  L.dbuf = L.work + B * a.npt;
  L.dbuf_cap = DBUF_PER_THREAD * B;
  L.misc = L.dbuf + L.dbuf_cap;
  L.rcnt = L.misc + 64;
  for (int i = threadIdx.x; i < a.tab_words; i += B) L.tab[i] = a.tab[i];
  for (int i = threadIdx.x; i < 64; i += B) L.misc[i] = 0;
  for (int i = threadIdx.x; i < a.n_rules; i += B) L.rcnt[i] = 0;
  __syncthreads();
  return L;
}

template <int A>
__global__ void __launch_bounds__(1024) k_round(RoundArgs a) {
  extern __shared__ int32_t smem[];
  if (ld(&a.ctl->done)) return;
  Lds L = setup_lds(a, smem);
  round_body<A>(a, L, ld(&a.ctl->r_base) + a.r0);
}

// Advances the round base by the number of rounds a captured chunk holds
// (the last node of the HIP graph of a chunk).
__global__ void k_advance(Ctl *ctl, int k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->r_base += k;
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

template <int A>
__global__ void __launch_bounds__(1024) k_persistent(RoundArgs a) {
  extern __shared__ int32_t smem[];
  if (ld(&a.ctl->done) || ld(&a.ctl->abort)) return;
  Lds L = setup_lds(a, smem);
  const unsigned long long G = gridDim.x;
  const int r0 = ld(&a.ctl->r_base) + a.r0;
  for (int k = 0; k < a.nrounds; k++) {
    if (!round_body<A>(a, L, r0 + k)) return;
    if (!grid_barrier(a.bar, G * (unsigned long long)(k + 1), &a.ctl->abort, &L.misc[63]))
      return;
  }
}

}  // namespace

size_t trs_round_lds_bytes(int block, int npt, int tab_words, int n_rules) {
  size_t words = (size_t)((tab_words + 3) & ~3) + (size_t)block * npt +
                 (size_t)DBUF_PER_THREAD * block + 64 + (size_t)n_rules;
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
  hipLaunchKernelGGL(k_round<A>, dim3(grid), dim3(block), lds, s, a);
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
  (void)hipFuncSetAttribute((const void *)k_round<A>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  (void)hipFuncSetAttribute((const void *)k_persistent<A>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t trs_prepare_kernels(int A, size_t lds) {
  if (lds > 65536) DISPATCH_A(A, set_attr_A, lds);
  return hipSuccess;
}

hipError_t trs_launch_round(int A, const RoundArgs &a, int grid, int block, hipStream_t s) {
  const size_t lds = trs_round_lds_bytes(block, a.npt, a.tab_words, a.n_rules);
  DISPATCH_A(A, launch_round_A, a, grid, block, lds, s);
  return hipGetLastError();
}

hipError_t trs_launch_advance(Ctl *ctl, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctl, k);
  return hipGetLastError();
}

hipError_t trs_launch_persistent(int A, const RoundArgs &a, int grid, int block, hipStream_t s) {
  const size_t lds = trs_round_lds_bytes(block, a.npt, a.tab_words, a.n_rules);
  g_coop_status = hipSuccess;
  DISPATCH_A(A, launch_pers_A, a, grid, block, lds, s);
  if (g_coop_status != hipSuccess) return g_coop_status;
  return hipGetLastError();
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
