#include "batch.h"

namespace di {

struct BatchState {
    int K = 0;
};

int init_batch(BatchState *&b, const DevGraph &, SweepParams &, int, const std::vector<i64> &, const double *,
               hipStream_t) {
    b = nullptr;
    set_error("batched solves are not available yet");
    return DI_EINVAL;
}
int reset_batch(BatchState *, const DevGraph &, const SweepParams &, hipStream_t) { return DI_EINVAL; }
int diffuse_batch(BatchState *, const DevGraph &, const SweepParams &, const di_opts &, int, int, hipStream_t,
                  di_stats *) {
    return DI_EINVAL;
}
int read_batch(BatchState *, const DevGraph &, const SweepParams &, int, void *, int, hipStream_t) { return DI_EINVAL; }
i64 batch_sweeps(BatchState *, hipStream_t) { return 0; }
int batch_K(const BatchState *b) { return b ? b->K : 0; }
void free_batch(BatchState *b) { delete b; }

}  // namespace di
