/*
 * ht_rise_profile.h - optional per-kernel timing of the batch hierarchical
 * Tucker library.  When enabled, every kernel launch of the library is bracketed
 * by HIP events on the stream it is launched on, and its algorithmic work is
 * recorded: floating-point operations and the bytes the operation must move
 * (each operand read once, each result written once).  Off by default; when off
 * the launchers do no extra work.  Host-side state, one per process.
 *
 * Kinds: 0 sum of squares, 1 unfolding Gram (FP64 matrix cores), 2 TTM contraction
 * (FP64), 3 TTM expansion / residual, 4 eigen-decomposition and truncation, 5 basis
 * expansion, 6 layout (padding, root append, copies), 7 residual Gram on FP32 matrix
 * cores, 8 TTM contraction on FP32 matrix cores (both of the HT_FP32 form, LDS-staged
 * panels), 9 and 10 the same two on register-direct blocks (mode views whose column
 * runs come in blocks of 32 or runs of 1-4), 11 FP64 residual Gram and 12 FP64 TTM
 * contraction on register-direct blocks.
 */
#ifndef HT_RISE_PROFILE_H
#define HT_RISE_PROFILE_H

#include "ht_rise.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t launches;  /* kernel launches recorded                          */
  double ms;         /* summed device time between the bracketing events  */
  double flops;      /* summed algorithmic floating-point operations       */
  double bytes;      /* summed algorithmic HBM bytes                       */
} ht_kernel_stats;

/* on != 0 enables recording and clears every counter; on == 0 disables it. */
ht_status ht_profile_enable(int32_t on);
/* Resolves pending events (synchronising on them) and returns kind's totals. */
ht_status ht_profile_read(int32_t kind, ht_kernel_stats* out);
/* Number of kinds, and a short name of each. */
int32_t ht_profile_kind_count(void);
const char* ht_profile_kind_name(int32_t kind);

#ifdef __cplusplus
}
#endif

#endif /* HT_RISE_PROFILE_H */
