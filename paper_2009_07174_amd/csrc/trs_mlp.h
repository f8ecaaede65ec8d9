// trs_mlp.h -- library-internal interface of the frontier predictor kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Evaluate the predictor (bfloat16 parameters d_params, trs.h order) on
// every input (sym, bits, bucket) of an n_sym-symbol system and write the
// keep decisions p >= threshold as a bit table: bit (sym*32 + bits)*16 +
// bucket of d_words (n_sym*16 words).  Scratch: d_probs (n_sym*512 floats),
// d_rec (n_sym*512 uint64), d_loss (1 float).  Issued on stream s.
hipError_t trs_mlp_build_table(const uint16_t *d_params, int n_sym, const int32_t *d_arity,
                               float threshold, float *d_probs, uint64_t *d_rec, float *d_loss,
                               uint32_t *d_words, hipStream_t s);
