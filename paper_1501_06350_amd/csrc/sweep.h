// Single right-hand-side sweep kernels: block-local D-Iteration, the deterministic
// synchronous sweep, power iteration, and the residual / control steps.
#pragma once
#include "graph.h"

namespace di {

// Work items of the row pull (power iteration), one wavefront each:
//   short  : <= RB_ROWS consecutive rows of <= RB_SHORT entries each, <= RB_NNZ in
//            total, staged in LDS and folded one row per lane;
//   vector : one row of RB_SHORT+1 .. RB_SEG entries, strided over the wave's lanes
//            and combined by a fixed-order wave reduction;
//   long   : one row of more than RB_SEG entries, cut into segments of RB_SEG that
//            separate workgroups reduce first (k_pi_segments).
constexpr int RB_ROWS = 64;
constexpr int RB_SHORT = 64;
constexpr int RB_NNZ = 1024;
constexpr int RB_SEG = 32768;
constexpr int RB_KIND_SHORT = -1;
constexpr int RB_KIND_VECTOR = -2;

struct RowBlocks {
    i64 nrb = 0, nseg = 0;
    i64 *start = nullptr;    // nrb+1 first rows
    int *seg_first = nullptr;// nrb: first segment of a long row, RB_KIND_SHORT or RB_KIND_VECTOR
    int *seg_count = nullptr;// nrb
    i64 *seg_b = nullptr, *seg_e = nullptr;  // nseg entry ranges
    double *partial = nullptr;                // nseg partial sums
};

int build_row_blocks(RowBlocks &rb, const i64 *d_ptr, i64 n, hipStream_t st);
void free_row_blocks(RowBlocks &rb);

// Block-diagonal union of independent graphs (one solve per graph in the same sweeps).
// Every graph starts on a range boundary, so a range belongs to one graph; per graph
// the residual, threshold and stop state are kept apart.
constexpr int GS_ACTIVE = 0;  // sweeping
constexpr int GS_FINISH = 1;  // certified with fluid in flight: next sweep only delivers it
constexpr int GS_FROZEN = 2;  // certified, nothing in flight: its ranges are skipped

struct GraphInfo {  // constant per graph
    i64 rbeg, rend;  // ranges [rbeg, rend)
    double n_d;      // number of (unpadded) nodes
    double zsum;     // sum of Z over the graph
};

struct GraphCtl {  // per-graph control, cleared at reset
    u64 limbsL[4];
    double R, thr, maxF;
    u64 nodes, edges, remote;  // counters of the last step
    long long done_sweep;      // sweep count when the graph froze
    int state, guard;
};

struct SolveState {
    // all pointers device; T = float when fluid_fp32 else double
    void *F = nullptr;       // n fluid
    double *F0 = nullptr;    // n initial fluid (1-d) Z, in double for every fluid type
    double *H = nullptr;     // n history
    void *S[2] = {nullptr, nullptr};  // n fluid in flight to other ranges (parity by ctl->parity)
    u64 *Sb[2] = {nullptr, nullptr};  // bit i of word i/64: S[.][i] is nonzero (same allocation as S)
    i64 S_bytes = 0;                  // bytes of each S allocation (values, then the bitmap)
    double *snap = nullptr;  // n deterministic sweep: pushed value per source
    int *frontier = nullptr; // n deterministic sweep: active set of the last sweep
    int *range_order = nullptr;  // nranges, heaviest first
    DevCtl *ctl = nullptr;
    // power iteration
    double *X[2] = {nullptr, nullptr};
    void *XT[2] = {nullptr, nullptr};
    DevCtl *pctl = nullptr;
    double *Z = nullptr;     // n, or nullptr when uniform
    double zc = 0.0;         // (1-d) * (1/n) when Z is uniform
    // per-workgroup partial sums of the last launched step (see PSR / PSC)
    u64 *partR = nullptr, *partC = nullptr;
    i64 nR = 0, nC = 0;
    // union of graphs (nullptr for one graph)
    int *range_graph = nullptr;  // nranges: graph of each range
    int *range_cnt = nullptr;    // nranges: real nodes of each cut-aligned range (padding after them)
    GraphInfo *ginfo = nullptr;  // n_graphs
    GraphCtl *gctl = nullptr;    // n_graphs
    i64 n_graphs = 0;
    // exact sums of H and of F per graph (mass balance): limb slots, then per graph
    // the sum of H and the sum of F (2 n_graphs doubles)
    u64 *partH = nullptr;
    double *hsum = nullptr;
    int rb = 0;
};

// grid caps of the grid-stride kernels; the partial-sum buffers hold
// max(number of ranges, PART_MIN) slots
constexpr int REDUCE_GRID = 4096;
constexpr int SNAP_GRID = 8192;
constexpr int PI_GRID = 4096;
constexpr int PART_MIN = 8192;

struct SweepParams {
    double d = 0.85, theta = 1.0, tol = 1e-8;
    int K = 0;
    int fp32 = 0;
    int rounds = 8;
    int normalized = 0;
    i64 n = 0;
    double zsum = 1.0;  // normalised stop uses l / zsum
    int bld_v1 = 0;     // force the global-memory block-local kernel
    // the block-local sweep after one that delivered at least this many nonzero in-flight
    // values reads them without testing the bitmap first (0: always test)
    double dense_at = 0.0;
};

// Kernels launched by the solver driver (all on stream st).
// rounds == 0 delivers the fluid in flight (runs even after convergence)
int launch_bld_sweep(const DevGraph &g, SolveState &s, const SweepParams &p, int rounds, hipStream_t st);
int set_kernel_attributes();
int launch_finalize(DevCtl *ctl, const SweepParams &p, int mode, hipStream_t st, const u64 *partR, i64 nR,
                    const u64 *partC, i64 nC);
// skip_frozen: in a union of graphs, leave out the graphs that are frozen
int launch_reduce_F(const DevGraph &g, SolveState &s, const SweepParams &p, hipStream_t st, int skip_frozen = 0);
int launch_det_sweep(const DevGraph &g, SolveState &s, const SweepParams &p, hipStream_t st);
int launch_pi_iteration(const DevGraph &g, const RowBlocks &rb, SolveState &s, const SweepParams &p, hipStream_t st);
int launch_pi_init(const DevGraph &g, SolveState &s, const SweepParams &p, hipStream_t st);
// F = F_0 + d P H - H computed in double over the IN row blocks, stored in the fluid
// type (ht: n doubles of scratch); no residual
int launch_refine_fluid(const DevGraph &g, const RowBlocks &rb, SolveState &s, const SweepParams &p, double *ht,
                        hipStream_t st);
// out = P v (n doubles); ordered: a left fold over each IN row in source order (the
// oracle's order, bit-reproducible), else the wave-parallel row pull over the row blocks
// (ht: n doubles of scratch for v / s)
int launch_P_times(const DevGraph &g, const RowBlocks &rb, const double *v, double *ht, double *out, int ordered,
                   hipStream_t st);
int launch_fill_zero(void *p, i64 bytes, hipStream_t st);
// F = F0 rounded to the fluid type (count entries)
int launch_init_fluid(const double *F0, void *F, int fp32, i64 count, hipStream_t st);
int launch_copy_fluid_to_double(const void *F, int fp32, i64 n, double *dst, hipStream_t st);
int launch_scaled_copy(const double *H, double scale, i64 n, double *dst, hipStream_t st);
size_t bld_lds_bytes(int rb, int fp32);
int bld_threads();

// finalize modes
constexpr int FIN_DI = 0;     // residual of F (+ in flight); stop on R/(1-d) or R/(1-d-dl)
constexpr int FIN_PI = 1;     // residual |x_{k+1} - x_k|; stop on R/(1-d)
constexpr int FIN_INIT = 2;   // like FIN_DI but does not count a sweep
constexpr int FIN_ADJ = 3;    // adjoint: stop on max|F| / (1-d)
constexpr int FIN_DELIVER = 4;// after delivering fluid in flight: flip parity only
constexpr int FIN_ADJ_INIT = 5;// FIN_ADJ without counting a sweep

// per-graph control step of a union of graphs (modes FIN_DI, FIN_INIT, FIN_DELIVER)
int launch_mg_finalize(SolveState &s, DevCtl *ctl, const SweepParams &p, int mode, int det, hipStream_t st);

int launch_adj_sweep(const DevGraph &g, double *F, double *H, double *snap, DevCtl *ctl, const SweepParams &p,
                     hipStream_t st, u64 *partR, u64 *partC, i64 *nR, i64 *nC);
// Fast adjoint sweep: the same snapshot, then a wave-per-row-block pull over OUT (rb_out:
// row blocks of OUT) that also sums the residual; additions in lane order, not row order.
int launch_adj_sweep_fast(const DevGraph &g, const RowBlocks &rb_out, double *F, double *H, double *snap, DevCtl *ctl,
                          const SweepParams &p, hipStream_t st, u64 *partR, u64 *partC, i64 *nR, i64 *nC);
// exact signed sum of a node vector v (n values, float or double) per graph of a union
// (else one sum) on 2^-K into out[0 .. n_graphs); part: max(nranges, PART_MIN) * PSR words
int launch_node_sums(const DevGraph &g, SolveState &s, const void *v, int is_float, int K, u64 *part, double *out,
                     hipStream_t st);
// Fast adjoint sweep: the block-local sweep on the transposed graph gT (ranges and
// numbering of the forward graph), fluid in as.F, history in as.H, in-flight buffers in
// as.S / as.Sb, control block as.ctl; tinv = 1/s of the forward graph.  The partial slots
// carry max |F| right after the fluid in flight arrived (rounds == 0: delivery only).
int launch_adj_bld_sweep(const DevGraph &gT, const double *tinv, SolveState &as, const SweepParams &p, int rounds,
                         hipStream_t st);
int launch_reduce_double(const double *F, i64 n, int K, DevCtl *ctl, hipStream_t st, u64 *partR, i64 *nR);
// dZ = (1-d) lambda and, when dw is given, the edge gradient; with mu (n doubles of scratch)
// the edge-parallel form, else the row-order sums of the oracle
int launch_edge_grad(const DevGraph &g, const double *x, const double *lam, double d, double *dZ, double *dw,
                     double *mu, hipStream_t st);

}  // namespace di
