// trs_kernels.h -- launch interface between the host runtime and the HIP
// kernels of libtrs (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include "trs_layout.h"

struct RoundArgs {
  Pool p;
  Ctl *ctl;
  const int32_t *tab;   // compiled tables in device memory
  int32_t tab_words;
  int32_t n_sym;
  int32_t n_rules;
  int32_t npt;          // slots per thread per tile
  int32_t pf_depth;     // sweep tiles copied ahead into LDS (0: none; 1..4
                        // with 16 slots per thread)
  int32_t qbuf;         // LDS entries per thread of each list buffer
  int32_t nrounds;      // rounds a persistent launch may run
  int32_t cont_rounds;  // rounds workgroup 0 may continue alone in one launch
  int64_t max_rounds;   // > 0: the run stops with TRS_E_ROUNDS before round
                        // max_rounds would execute (rounds 0 .. max_rounds-1
                        // may run); 0: unlimited
  int32_t small_cap;    // list items one workgroup takes on alone
  // a larger grid exists (0: the launch's grid is the largest): a launch
  // whose round lists more than grow_list items, or (plain and learned
  // modes) sweeps more than grow_full slots, returns at once without
  // executing it, so that the host sizes a larger grid from the published
  // round
  int32_t grow_list;
  int32_t grow_full;
  int32_t mode;         // 0 full sweeps, 1 frontier by parent notification,
                        // 2 parent notification plus the predictor's choice
                        // among blocked nodes (full sweep when the frontier
                        // is empty)
  int32_t use_memo;     // memo shortcut on (off in learned mode and tracing)
  int32_t nf_walk;      // frontier modes: most constructors above a node
                        // that becomes a normal form that are marked in the
                        // same round, in rounds one workgroup runs (0: none)
  int32_t nf_walk_wide; // the same in rounds several workgroups run
  int32_t cont_passes;  // further passes a workgroup may run in one list
                        // round over the ready nodes it created or rewrote
                        // in that round, in rounds one workgroup runs
  int32_t cont_passes_wide;  // the same in rounds several workgroups run
  int32_t fresh_below;  // allocation takes fresh slots before recycled ones
                        // while the extent n is below this (0: never)
  int32_t use_scan;     // plain mode: large full rounds are classified by k_scan
                        // (launched before each k_round) and run as list rounds
  int32_t round_block;  // k_round's block size (for the scan's hand-over)
  int32_t scan_lists;   // lists the scan appends to (1 or 16): list j is
                        // written by the workgroups wg mod scan_lists = j
  int64_t scan_rs;      // entries per list: list j starts at entry
                        // (j mod 8) scan_rs of front0 (j < 8) or front1
  int32_t gate_off;     // learned mode: word offset of the decision table in tab
  uint32_t trace_rate;  // tracing: keep a blocked node-round when its hash
                        // (16 bits) is below this; 0 = off
  int64_t trace_cap_rec;     // records the buffer holds
  int32_t label_h;      // tracing: label horizon in rounds
  int32_t sweep_every;  // learned mode: full sweep every k rounds (0: never)
  unsigned long long *trace_rec;  // trace records
  int32_t *trace_n;     // records logged so far
  unsigned long long *bar;  // grid barrier counter (persistent kernel)
  long long *trace;     // optional phase timestamps of workgroup 0 (null: off)
  int32_t trace_cap;    // rows the trace holds (TRACE_FIELDS words each)
  int32_t trace_shift;  // 0: row r is round r; s > 0: rounds r with
                        // r mod 2^s < 2, in row 2 (r >> s) + (r & 1)
  int32_t trace_max;    // nonzero: fields from 2 on hold the latest time any
                        // workgroup passed the point (else workgroup 0's)
  long long *wgtrace;   // optional per-workgroup timing of round wgtrace_round:
                        // 8 words per workgroup (null: off)
  int32_t wgtrace_round;
};

// Phase timestamps (clock64) recorded by thread 0 of workgroup 0 per round:
// prepare start, prepare end, bookkeeping end, list phase end, sweep end,
// statistics end; inside the first list pass: readiness checked, matched,
// reserved, instantiated, flushed (11 fields); then, for the workgroup's
// first sweep tile: bytes loaded, slots classified, work list appended,
// work passes done.
#define TRACE_FIELDS 16

// Threads per workgroup of k_scan, slots per thread per tile, and the
// listed slots a workgroup gathers in LDS before appending them at once.
#define SCAN_BLOCK 1024
#define SCAN_NPT 16
#define SCAN_CAP 8192

// LDS bytes a round kernel needs for this configuration.
size_t trs_round_lds_bytes(int block, int npt, int tab_words, int n_rules, int pf_depth,
                           int qbuf);

// Launches the plain-mode scan (k_scan) on stream s; it does nothing unless
// the published round state requests a scan.
hipError_t trs_launch_scan(int A, const RoundArgs &a, int grid, hipStream_t s);

// Sets kernel attributes (dynamic LDS above 64 KiB); call before launching
// or capturing with a given LDS size.
hipError_t trs_prepare_kernels(int A, size_t lds_bytes);

// One launch: round ctl->r_cur on the grid, then, while rounds stay small,
// further rounds on workgroup 0 alone; advances ctl->r_cur.
hipError_t trs_launch_round(int A, const RoundArgs &a, int grid, int block, hipStream_t s);

// Persistent cooperative kernel: rounds ctl->r_cur .. + nrounds-1,
// separated by device-wide barriers.  *a.bar must be zero at launch.  grid
// must not exceed trs_max_resident().
hipError_t trs_launch_persistent(int A, const RoundArgs &a, int grid, int block, hipStream_t s);

// Highest number of co-resident workgroups for the persistent kernel.
int trs_max_resident(int A, int block, size_t lds_bytes, int device);

// Highest number of co-resident workgroups of the round kernel.
int trs_round_resident(int A, int block, size_t lds_bytes, int device);
