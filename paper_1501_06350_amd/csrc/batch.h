// Several right-hand sides: an n x k fluid tile (node-major) solved in one sweep loop,
// with a residual, threshold and stop per column.
#pragma once
#include "sweep.h"

namespace di {

struct BatchState;

// Z: n x k column-major (NULL = uniform 1/n); det = deterministic sweeps; range_order
// (nranges, owned by the caller) and rounds drive the block-local fast sweeps
int init_batch(BatchState *&b, const DevGraph &g, SweepParams &p, int k, int det, const double *Z,
               const int *range_order, int rounds, hipStream_t st);
// range size (log2) whose fluid and history-increment tiles fit in LDS for k columns
// (0 if none does: the fast sweep then uses global atomics)
int tile_range_log2(int k, int fp32, int weighted);
int reset_batch(BatchState *b, const DevGraph &g, const SweepParams &p, hipStream_t st);
// new right-hand sides (validated by the caller; NULL = uniform), then reset
int set_batch_z(BatchState *b, const DevGraph &g, SweepParams &p, const double *Z, hipStream_t st);
int diffuse_batch(BatchState *b, const DevGraph &g, const SweepParams &p, const di_opts &o, int spc, hipStream_t st,
                  di_stats *stats);
// per-column mass balance sum F + (1-d) sum H + d l - (1-d) sum Z of the current state
// (out: k host doubles)
int batch_mass_defects(BatchState *b, const DevGraph &g, const SweepParams &p, double *out, hipStream_t st);
int read_batch(BatchState *b, const DevGraph &g, const SweepParams &p, int what, void *dst, int on_device,
               hipStream_t st);
i64 batch_sweeps(BatchState *b, hipStream_t st);
int batch_K(const BatchState *b);
// local rounds of the tile's block-local sweeps (captured chunks are dropped)
void set_batch_rounds(BatchState *b, int rounds);
void free_batch(BatchState *b);

}  // namespace di
