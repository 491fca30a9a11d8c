/*
 * di.h - D-Iteration (fluid diffusion) and power iteration for PageRank on one
 * AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or
 * framework types.  Every call returns an int status (DI_OK or a negative code)
 * and never throws or aborts across the boundary.  di_last_error() returns a
 * thread-local message for the last failure.
 *
 * Problem (Hong, Huynh & Mathieu, "D-Iteration: diffusion approach for solving
 * PageRank", Section 2.1): for a directed graph with weights w(j->i) > 0,
 *     P[i][j] = w(j->i) / s_j,   s_j = sum of j's out-weights      (equation def-p)
 * (1/out(j) when unweighted; a dangling node j has a null column), solve
 *     x = d P x + (1 - d) Z,     0 < d < 1,  Z >= 0                 (equation pagerank-pf)
 *
 * D-Iteration (Section 3.1, equation defF): fluid F_0 = (1-d) Z, history H_0 = 0;
 * diffusing node i moves its fluid f into H_i and adds d f P e_i to F.  H converges
 * to x and |x - H|_1 <= |F|_1 / (1-d) (Theorem 1, equation SL).  Power iteration
 * (Section 2.2): x_{k+1} = d P x_k + (1-d) Z.
 *
 * Thread safety: one context is used by one host thread at a time; independent
 * contexts are independent.  All device work of a context runs on its stream.
 *
 * Environment (read at each use):
 *   DI_LOG=path          append JSON lines to path: one per host synchronisation of
 *                        di_diffuse (contexts with k = 1), di_power and di_adjoint, that
 *                        is every sweeps_per_sync sweeps (1 gives one per sweep): sweep
 *                        index, the call's sweeps, node and edge updates and DI rounds so
 *                        far, residual, bounds, leak, host ms; and one at the end of each
 *                        such call (plus status, converged, mass defect, device ms,
 *                        GEUPS; non-finite values as null).  Best effort: a file that
 *                        cannot be opened is skipped, never an error.
 *   DI_FAIL_ALLOC_AT=k   for tests of the error paths: the k-th device allocation after
 *                        the variable took its current value fails as out of memory
 *                        (the call returns DI_ENOMEM and frees what it had allocated).
 */
#ifndef DI_API_H_
#define DI_API_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DI_OK 0
#define DI_EINVAL (-1)   /* invalid argument; nothing was changed */
#define DI_ENOMEM (-2)   /* device or host allocation failed */
#define DI_EHIP (-3)     /* a HIP runtime call failed */
#define DI_ENOCONV (-4)  /* sweep budget spent before the tolerance; state kept, call again to continue */
#define DI_ESTATE (-5)   /* call not valid in the context's current state */
#define DI_ENUMERIC (-6) /* non-finite or out-of-range value met in the residual */

typedef struct di_ctx di_ctx; /* opaque; owns every device buffer it allocates */

/*
 * Input graph as out-adjacency CSR (rows = sources).
 *   out_ptr : n+1 int64, out_ptr[0] = 0, non-decreasing, out_ptr[n] = m
 *   out_idx : m int32 targets in [0, n); self-loops and repeated edges are allowed
 *             and count with multiplicity (they add to P[i][j] and to s_j)
 *   w       : m float32 weights, > 0 and finite, or NULL for unweighted
 *   on_device : 0 = host arrays, 1 = device arrays; either way they are only read
 *             during di_init and the caller keeps ownership.
 */
typedef struct {
    int64_t n;
    int64_t m;
    const int64_t *out_ptr;
    const int32_t *out_idx;
    const float *w;
    int on_device;
} di_csr;

/* loop_mode values */
#define DI_LOOP_STREAM 0 /* sweeps launched on the stream, host checks every sweeps_per_sync */
#define DI_LOOP_GRAPH 1  /* chunks of sweeps captured once into a HIP graph and replayed */

/*
 * Options (pass NULL for the defaults given in brackets).
 *   fluid_fp32     : 1 = fluid F stored and pushed in float; history H, residual and
 *                    leak stay double [0]
 *   theta          : frontier scale; a node is active when |F_i| >= theta * |F|_1 / n
 *                    (the DI-argmax rule of Section 3.4 applied per sweep) [1.0]
 *   max_sweeps     : sweep (or iteration) budget per di_diffuse / di_power call [100000]
 *   deterministic  : 1 = synchronous sweeps with snapshot semantics and ordered
 *                    accumulation (bit-reproducible, slower) [0].  This is also the
 *                    scatter strategy: 0 pushes inside a block-local range with LDS
 *                    atomic adds and pulls cross-range fluid through a layout sorted by
 *                    target (no atomics in memory); 1 snapshots the active set and pulls
 *                    along IN rows in row order (no atomics at all)
 *   range_log2     : block-local range size 2^range_log2 nodes, 8..13 (0 = auto).
 *                    With k > 1: 6..8 runs the tile's block-local sweep (auto: the
 *                    largest range whose fluid tile lets two workgroups share a compute
 *                    unit), larger sizes its plain push sweep
 *   inner_rounds   : block-local diffusion rounds per sweep, 1..64 (0 = auto)
 *   k              : number of right-hand sides (columns of Z), 1..64 [1].  k > 1
 *                    diffuses an n x k fluid tile (personalized PageRank, Section 2.1):
 *                    a node is taken when any column's fluid reaches that column's
 *                    threshold, and then every column of the row is diffused; each
 *                    column has its own residual and stop.  theta and inner_rounds
 *                    apply to the tile's sweeps, range_cut does not; di_power,
 *                    di_adjoint and checkpoints are single-column only.
 *   n_graphs       : > 1 declares the graph a block-diagonal union of independent
 *                    graphs whose node ranges are given by graph_ptr [1].  Every edge
 *                    must stay inside its graph.  Each graph g is solved as its own
 *                    problem in the same sweeps: threshold theta |F_g|_1 / n_g, its own
 *                    residual, leak and stop; a graph that meets the tolerance is left
 *                    alone while the others continue.  Internally each graph starts on a
 *                    block-local range boundary (padding nodes without edges or fluid);
 *                    results are read back in the caller's numbering.  Not with k > 1;
 *                    di_power, di_adjoint and checkpoints take a single graph.
 *   graph_ptr      : host array of n_graphs+1 node offsets (0 = first, n = last),
 *                    strictly increasing
 *   loop_mode      : DI_LOOP_STREAM or DI_LOOP_GRAPH [DI_LOOP_STREAM]
 *   sweeps_per_sync: sweeps enqueued between host convergence checks (0 = auto)
 *   timing         : 1 = bracket every sweep (or iteration) kernel with HIP events and
 *                    keep the summed device time (di_info DI_INFO_KERNEL_NS) [0]
 *   normalized_stop: 1 = stop on |F|_1 / (1 - d - d l/|Z|_1) instead of |F|_1 / (1-d)
 *                    (implicit completion, Section 3.3) [0]
 *   range_cut      : one right-hand side on one graph with fast sweeps: a block-local
 *                    range may end up to range_cut nodes before its 2^range_log2 slots
 *                    are full, at the boundary crossed by the fewest edges shorter than a
 *                    range (on a host-ordered web graph, between two hosts); its unused
 *                    slots become padding nodes without edges or fluid.  The internal
 *                    numbering keeps the caller's order (edges, rows and results are
 *                    mapped back), so every call behaves as on the caller's graph.
 *                    Values above 2^range_log2 / 2 act as 2^range_log2 / 2.
 *                    0 = auto (1024), -1 = ranges at multiples of 2^range_log2 (no
 *                    padding) [0]
 *   stream         : hipStream_t to run on; NULL = the null stream
 */
typedef struct {
    int fluid_fp32;
    double theta;
    int64_t max_sweeps;
    int deterministic;
    int range_log2;
    int inner_rounds;
    int k;
    int64_t n_graphs;
    const int64_t *graph_ptr;
    int loop_mode;
    int sweeps_per_sync;
    int normalized_stop;
    int timing;
    int range_cut;
    void *stream;
} di_opts;

/* Statistics of the last di_diffuse / di_power / di_adjoint call. */
typedef struct {
    int64_t sweeps;        /* sweeps (DI) or iterations (PI) run by this call */
    int64_t edge_updates;  /* edge pushes (DI) or m * iterations (PI) */
    int64_t node_updates;  /* elementary diffusions (DI) or n * iterations (PI) */
    double residual;       /* DI: |F|_1 incl. fluid in flight; PI: |x_{k+1} - x_k|_1;
                              with k > 1 or n_graphs > 1: the largest per-column/graph value */
    double bound;          /* certified distance: residual / (1-d) (Theorem 1);
                              adjoint: max|F| / (1-d) */
    double bound_norm;     /* residual / (1 - d - d l/|Z|_1): distance of the normalised result (Section 3.3) */
    double leak;           /* l: fluid diffused at dangling nodes (Section 3.3) */
    double mass_defect;    /* di_diffuse: sum F + (1-d) sum H + d l - (1-d) sum Z, the mass
                              balance that equation HnFn implies because the columns of P sum
                              to 1 except at dangling nodes (Section 2.1); zero in exact
                              arithmetic, so it measures the rounding injected by the pushes
                              (with float fluid: the rounding of F to float).  Sums are exact
                              fixed-point sums rounded once.  With k > 1 or n_graphs > 1: the
                              per-column/graph value of largest magnitude (DI_MASS_DEFECTS
                              reads them all).  0 after di_power and di_adjoint. */
    double ms;             /* device time of the call (HIP events on the context's stream) */
    int converged;         /* 1 if every column/graph met the tolerance */
} di_stats;

/*
 * Create a context for graph g, damping d in (0,1) and default distribution Z.
 *   Z : host array, n x k column-major, every entry >= 0 and finite, each column
 *       with a positive sum; NULL = uniform 1/n per column, or 1/n_g on each graph g
 *       of a union.
 * Builds on the device: IN adjacency (stable counting sort of OUT by target), 1/s_j,
 * degree-binned row blocks and the block-local / cross-range edge split, then sets
 * F = (1-d) Z, H = 0.  Errors: DI_EINVAL (bad sizes, non-monotone out_ptr, index out
 * of range, w <= 0 or non-finite, d outside (0,1), bad Z or options), DI_ENOMEM, DI_EHIP.
 * On error *ctx is set to NULL.
 */
int di_init(di_ctx **ctx, const di_csr *g, double d, const double *Z, const di_opts *o);

/*
 * D-Iteration sweeps (Section 3.1) until the certified L1 bound |F|_1 / (1-d) of every
 * column (graph) is <= tol (Theorem 1), or max_sweeps sweeps were run (DI_ENOCONV; the
 * state is kept and a further call continues from it).  tol must be > 0.
 */
int di_diffuse(di_ctx *ctx, double tol, di_stats *st);

/*
 * Power iteration x_{k+1} = d P x_k + (1-d) Z (Section 2.2) from x_0 = 0, until
 * |x_{k+1} - x_k|_1 / (1-d) <= tol; that quantity bounds |x - x_k|_1 because
 * x - x_k = (I - dP)^{-1} (x_{k+1} - x_k) and |P|_1 <= 1.  Independent of the DI state.
 * Single right-hand side, single graph only (DI_EINVAL otherwise).
 */
int di_power(di_ctx *ctx, double tol, di_stats *st);

/*
 * Adjoint of the converged solve: with g = dL/dx, computes lambda = (I - d P^T)^{-1} g
 * by diffusing signed fluid on the transposed matrix until max|F| / (1-d) <= tol_inf
 * (|P^T|_inf <= 1 because every column of P sums to at most 1, Section 2.1), then
 *   dZ[i] = (1-d) lambda_i
 *   dw[e] = (d x_j / s_j) (lambda_i - mu_j),  e = j -> i in OUT order,
 *           mu_j = sum over j's out-edges e' of P_{e'} lambda_{target(e')}
 * with x the raw history H of the last di_diffuse.  g, dZ (n doubles) and dw (m
 * doubles, may be NULL) are host arrays (on_device = 0) or device arrays (1).
 * Each sweep snapshots the active fluid and pulls it over OUT rows; a deterministic
 * context adds in row order (bit-reproducible), any other context sums a row across a
 * wave (faster, reproducible only to rounding).
 * Requires a converged di_diffuse (DI_ESTATE otherwise); k = 1, single graph.
 */
int di_adjoint(di_ctx *ctx, const double *g, double tol_inf, double *dZ, double *dw, int on_device, di_stats *st);

/*
 * di_power without any allocation, for callers that cannot allocate device memory while
 * it runs (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same power iteration and stop rule as di_power, with the two iterates,
 * the two x/s vectors and the control block in a static device array of
 * DI_NOALLOC_SCRATCH_BYTES per device (held until the process ends) instead of
 * context buffers.  The result goes to x_out, a device array of n doubles (caller's
 * numbering); di_read(DI_X_PI) is not changed.  Needs n_int * (16 + 2 T) + 256 bytes
 * (n_int: di_info DI_INFO_N_INTERNAL; T = 4 with float fluid, else 8; each part rounded up
 * to 256 bytes): up to 1,048,544 nodes with double, 1,398,080 with float x/s.  Larger
 * graphs: DI_EINVAL.  Always runs in stream mode (no graph capture, no timing events).
 * Every call on one device shares that device's array: calls that overlap on one device
 * (several host threads, or several streams) race and must be serialised by the caller.
 * Single right-hand side, single graph only (DI_EINVAL otherwise).
 */
#define DI_NOALLOC_SCRATCH_BYTES (32u << 20)
int di_power_noalloc(di_ctx *ctx, double tol, double *x_out, di_stats *st);

/* what values for di_read (sizes in elements; k = columns) */
#define DI_X_RAW 0     /* H (double, n*k, column-major): the raw D-Iteration result */
#define DI_X_NORM 1    /* (1-d)/(1-d-d l/|Z|_1) H per column: the solution completed by Z/|Z|_1
                          at dangling nodes (Section 3.3; the paper's (1-d)/(1-d-d l) when |Z|_1 = 1) */
#define DI_F 2         /* fluid F as double, n*k column-major, fluid in flight delivered */
#define DI_H 3         /* same as DI_X_RAW */
#define DI_LAMBDA 4    /* adjoint lambda (double, n) */
#define DI_X_PI 5      /* power-iteration result (double, n) */
#define DI_IN_PTR 6    /* IN adjacency row pointers (int64, n+1) */
#define DI_IN_IDX 7    /* IN adjacency sources (int32, m) */
#define DI_INV_S 8     /* 1/s_j (double, n; 0 for dangling nodes) */
#define DI_FRONTIER 9  /* deterministic mode: ascending active set of the last sweep
                          (int64 count followed by that many int32 indices; dst holds n+2 int32) */
#define DI_RESIDUALS 10 /* per column (or graph) |F|_1 (double, k or n_graphs) */
#define DI_LEAKS 11    /* per column (or graph) l (double, k or n_graphs) */
#define DI_DONE_SWEEPS 12 /* per column (or graph): total sweep count at which it met the
                             tolerance of the last di_diffuse, -1 if it has not (int64, k or
                             n_graphs; a single-column solve gives 1 value) */
#define DI_MASS_DEFECTS 13 /* per column (or graph) mass defect of the last di_diffuse (double,
                              k or n_graphs; see di_stats.mass_defect) */
/* Copy a result into dst (host if dst_on_device = 0, device otherwise). */
int di_read(di_ctx *ctx, int what, void *dst, int dst_on_device);

/*
 * Graph update (Section 3.5, Theorem 4): replace the context's graph by g (same n, any
 * edges and weights; host or device arrays, validated as in di_init) and keep the
 * D-Iteration state, so that the next di_diffuse converges to the solution of
 * x' = d P' x' + (1-d) Z:
 *     H' = H,   F' = F + d (P' - P) H   (evaluated as P'H - PH; fluid may turn negative),
 * and the leak restarts as the history at the nodes dangling in P' (Section 3.3).  The
 * certificate |x' - H'|_1 <= |F'|_1 / (1-d) holds for signed fluid too (Theorem 1's proof
 * only uses |P'|_1 <= 1).  Deterministic contexts evaluate P H as a left fold over each IN
 * row in source order (bit-reproducible).  Z, d and the options are kept; the device graph,
 * its layout and the power-iteration and adjoint state are rebuilt (the old graph is
 * released; both are resident during the call).  Single right-hand side, single graph.
 * Errors: DI_EINVAL (bad graph, other n, several columns or graphs), DI_ENOMEM, DI_EHIP;
 * on error the context is unchanged.
 */
int di_update(di_ctx *ctx, const di_csr *g);

/*
 * Change the frontier scale theta (>= 0) and, when inner_rounds > 0, the block-local rounds
 * per sweep (1..64) of a context; the graph and the D-Iteration state are kept, so the next
 * di_diffuse continues with the new options (any schedule keeps equation HnFn).  For
 * tuning and for schedules that change theta as the residual falls.  DI_EINVAL on bad
 * values.
 */
int di_set_sweep(di_ctx *ctx, double theta, int inner_rounds);

/* Back to F = (1-d) Z, H = 0, l = 0 (graph and PI state kept). */
int di_reset(di_ctx *ctx);

/*
 * Replace Z (host array, same layout and rules as in di_init; NULL = uniform) and reset
 * to F = (1-d) Z, H = 0.  The graph and every device structure built from it stay, so a
 * stream of personalized queries on one graph pays the graph build once.  DI_EINVAL
 * on a bad Z (the context is then unchanged).
 */
int di_set_z(di_ctx *ctx, const double *Z);

/*
 * Checkpoint (H, F, l, sweep count) to a file / restore it into a context built on
 * the same graph, d and options.  Equation HnFn holds for any stopping point, so a
 * restored run continues exactly.  DI_EINVAL on a mismatching file.
 */
int di_save(di_ctx *ctx, const char *path);
int di_load(di_ctx *ctx, const char *path);

/* info keys for di_info */
#define DI_INFO_N 0
#define DI_INFO_M 1
#define DI_INFO_K 2
#define DI_INFO_M_LOCAL 3   /* edges whose source and target share a block-local range */
#define DI_INFO_RANGE_LOG2 4
#define DI_INFO_INNER_ROUNDS 5
#define DI_INFO_FIXED_K 6   /* exponent K of the fixed-point residual (sums are exact on 2^-K) */
#define DI_INFO_TOTAL_SWEEPS 7
#define DI_INFO_DEVICE_BYTES 8
#define DI_INFO_KERNEL_NS 9       /* with timing: device ns of the sweep/iteration kernels of the last call */
#define DI_INFO_KERNEL_LAUNCHES 10/* with timing: kernels timed in the last call */
#define DI_INFO_LOCAL_PUSHES 11   /* block-local edge pushes since the last reset */
#define DI_INFO_REMOTE_UPDATES 12 /* nonzero cross-range deliveries since the last reset */
#define DI_INFO_M_REMOTE 13       /* cross-range edges */
#define DI_INFO_NRANGES 14        /* block-local ranges */
#define DI_INFO_N_INTERNAL 15     /* nodes held on the device (n plus the padding of a union) */
#define DI_INFO_LIVE_ALLOCATIONS 16 /* device allocations the library holds in this process, all
                                       contexts together (ctx may be NULL for this key) */
int di_info(di_ctx *ctx, int key, int64_t *value);

/* Release everything; NULL-safe. */
int di_destroy(di_ctx *ctx);

/* Message for the last failing call on this thread ("" if none). */
const char *di_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DI_API_H_ */
