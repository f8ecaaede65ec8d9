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
  int32_t r0;           // round offset of this launch from ctl->r_base
  int32_t nrounds;      // rounds this launch may run (persistent kernel)
  unsigned long long *bar;  // grid barrier counter (persistent kernel)
};

// LDS bytes a round kernel needs for this configuration.
size_t trs_round_lds_bytes(int block, int npt, int tab_words, int n_rules);

// Sets kernel attributes (dynamic LDS above 64 KiB); call before launching
// or capturing with a given LDS size.
hipError_t trs_prepare_kernels(int A, size_t lds_bytes);

// One round per launch: round ctl->r_base + r0 (nrounds ignored).
hipError_t trs_launch_round(int A, const RoundArgs &a, int grid, int block, hipStream_t s);

// ctl->r_base += k (the closing node of a captured chunk of rounds).
hipError_t trs_launch_advance(Ctl *ctl, int k, hipStream_t s);

// Persistent cooperative kernel: rounds ctl->r_base + r0 .. + nrounds-1,
// separated by device-wide barriers.  *a.bar must be zero at launch.  grid
// must not exceed trs_max_resident().
hipError_t trs_launch_persistent(int A, const RoundArgs &a, int grid, int block, hipStream_t s);

// Highest number of co-resident workgroups for the persistent kernel.
int trs_max_resident(int A, int block, size_t lds_bytes, int device);
