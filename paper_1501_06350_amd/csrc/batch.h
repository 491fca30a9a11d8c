// Several right-hand sides (an n x k fluid tile) or a block-diagonal union of
// independent graphs, solved in one sweep loop.
#pragma once
#include "sweep.h"

namespace di {

struct BatchState;

int init_batch(BatchState *&b, const DevGraph &g, SweepParams &p, int k, const std::vector<i64> &graph_ptr,
               const double *Z, hipStream_t st);
int reset_batch(BatchState *b, const DevGraph &g, const SweepParams &p, hipStream_t st);
int diffuse_batch(BatchState *b, const DevGraph &g, const SweepParams &p, const di_opts &o, int rounds, int spc,
                  hipStream_t st, di_stats *stats);
int read_batch(BatchState *b, const DevGraph &g, const SweepParams &p, int what, void *dst, int on_device,
               hipStream_t st);
i64 batch_sweeps(BatchState *b, hipStream_t st);
int batch_K(const BatchState *b);
void free_batch(BatchState *b);

}  // namespace di
