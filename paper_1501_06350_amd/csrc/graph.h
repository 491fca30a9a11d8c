// Device-resident graph of a context and the construction routines.
#pragma once
#include "common.h"

namespace di {

struct DevGraph {
    i64 n = 0, m = 0;
    bool weighted = false;
    // OUT (device copies of the input): rows = sources, targets ascending
    i64 *out_ptr = nullptr;
    int *out_idx = nullptr;
    float *w = nullptr;
    // IN: rows = targets, sources ascending (stable transpose of OUT)
    i64 *in_ptr = nullptr;
    int *in_idx = nullptr;
    float *in_w = nullptr;
    double *inv_s = nullptr;  // 1 / s_j, 0 for dangling nodes
    // block-local split, ranges of 2^rb consecutive nodes
    int rb = 0;
    i64 nranges = 0;
    i64 *loc_ptr = nullptr;            // n+1: local out-edges of each node
    unsigned short *loc_tgt = nullptr; // target - range base
    float *loc_w = nullptr;
    i64 m_loc = 0;
    double *rw = nullptr;              // out-weight (or count) of each node's cross-range edges
    i64 *rem_base = nullptr;           // nranges+1: cross-range in-edges of each range
    int *rem_src = nullptr;
    unsigned short *rem_tgt = nullptr; // target - range base
    float *rem_w = nullptr;
    i64 m_rem = 0;
    i64 *loc_base = nullptr;           // nranges+1: loc_ptr at each range start
    unsigned *deg_flags = nullptr;     // n: out-degree, bit 31 set when the node has cross-range edges
};

int scan_exclusive(const i64 *in, i64 *out, i64 count, i64 *temp, hipStream_t st);
i64 scan_temp_elems(i64 count);
// remote_by_source: order each range's cross-range entries by source (the single
// right-hand-side pull) instead of by target (the k-column delivery needs target order)
int build_graph(DevGraph &g, const i64 *d_out_ptr, const int *d_out_idx, const float *d_w, int range_log2,
                bool remote_by_source,
                hipStream_t st);
void free_graph(DevGraph &g);

}  // namespace di
