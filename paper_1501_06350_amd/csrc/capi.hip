// C ABI of the library: validation, context management and the host-side sweep loop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <new>
#include <numeric>
#include <string>

#include "batch.h"
#include "sweep.h"

namespace di {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

#define DI_FAIL(code, ...)            \
    do {                              \
        ::di::set_error(__VA_ARGS__); \
        return (code);                \
    } while (0)

// ---------------------------------------------------------------------------
// Device allocations: live count and injected failures (DI_FAIL_ALLOC_AT)
// ---------------------------------------------------------------------------
std::mutex g_alloc_mu;
long long g_alloc_live = 0;
long long g_alloc_seen = 0;  // allocations since DI_FAIL_ALLOC_AT took its current value
std::string g_alloc_env;

hipError_t dev_malloc(void **p, size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        const char *e = std::getenv("DI_FAIL_ALLOC_AT");
        const std::string v = e ? e : "";
        if (v != g_alloc_env) {
            g_alloc_env = v;
            g_alloc_seen = 0;
        }
        const long long k = v.empty() ? 0 : std::atoll(v.c_str());
        if (k > 0 && ++g_alloc_seen == k) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    const hipError_t r = hipMalloc(p, bytes);
    if (r == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        ++g_alloc_live;
    }
    return r;
}

hipError_t dev_free(void *p) {
    if (!p) return hipSuccess;
    const hipError_t r = hipFree(p);
    if (r == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        --g_alloc_live;
    }
    return r;
}

long long dev_live_allocations() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc_live;
}

}  // namespace di

using namespace di;

struct di_ctx {
    std::chrono::steady_clock::time_point call_t0;  // start of the running API call (DI_LOG)
    DevGraph g;
    RowBlocks rbin;  // row blocks of IN (power iteration, fluid recomputation)
    bool rbin_ready = false;
    RowBlocks rbout;  // row blocks of OUT (fast adjoint)
    bool rbout_ready = false;
    double *ref_ht = nullptr;  // n doubles: H / s for the fluid recomputation
    SolveState s;
    SweepParams p;
    di_opts o{};
    hipStream_t st = nullptr;
    double d = 0.85;
    int k = 1;
    i64 n_graphs = 1;
    std::vector<i64> graph_ptr;
    // union of graphs: each graph is placed at a range boundary (padding nodes have no
    // edges and no fluid); internal node gstart[g] + u is node graph_ptr[g] + u
    i64 n_user = 0;
    std::vector<i64> gstart;
    std::vector<int> h_range_graph;
    i64 *d_gp = nullptr, *d_gs = nullptr;
    double *d_gscale = nullptr;
    std::vector<GraphCtl> h_gctl;
    std::vector<GraphInfo> h_ginfo;
    // one graph with cut-aligned ranges: range r holds caller nodes [seg_start[r],
    // seg_start[r+1]) at internal nodes r 2^rb + 0, 1, ...; the rest of its slots are padding
    bool seg = false;
    int seg_rb = 0;
    std::vector<i64> seg_start;
    i64 *d_seg_start = nullptr;  // device copy of seg_start
    int rounds = 8;
    int spc = 8;  // sweeps per host check
    double zsum = 1.0;  // sum of Z (single right-hand side)
    double f0max = 0.0; // largest starting fluid value (rounded to the fluid type)
    bool forward_converged = false;
    bool pi_ready = false;  // power-iteration buffers allocated
    bool pi_done = false;   // X_PI holds the result for the current Z
    DevCtl *h_ctl = nullptr;  // pinned mirror of the control block
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    i64 device_bytes = 0;
    // adjoint
    double *lam = nullptr;
    double *aF = nullptr;
    double *asnap = nullptr;
    double *aZ = nullptr;   // dZ in the internal layout
    u64 *achk = nullptr;    // check of g: max |g| (bits), first non-finite entry
    DevCtl *actl = nullptr;
    // fast adjoint: the transposed graph on the forward graph's ranges, and its two
    // in-flight buffers (values, then the bitmap of the nonzero ones)
    DevGraph gT;
    bool gT_ready = false;
    void *aS[2] = {nullptr, nullptr};
    // batched / multi-graph solve (k > 1 or n_graphs > 1)
    BatchState *b = nullptr;
    // captured sweep chunk (loop_mode = DI_LOOP_GRAPH)
    hipGraphExec_t gexec = nullptr;
    int gexec_kind = -1;
    hipStream_t cap_st = nullptr;  // private stream the sweep chunk is captured on
    // timing: one event pair per step of a chunk
    std::vector<hipEvent_t> tev;
    double kernel_ns = 0.0;
    i64 kernel_launches = 0;
    // mass balance per column / graph after the last di_diffuse
    std::vector<double> defects;
    // this device's copy of the no-allocation scratch (see di_power_noalloc)
    unsigned char *scratch = nullptr;
};

// Scratch memory of di_power_noalloc: the power iteration's two iterates (double), its two
// x/s vectors (fluid type) and its control block, each at a 256-byte boundary.  Every
// device holds its own copy for the life of the process.  In host code the array's name is
// not a device address: host code uses the address hipGetSymbolAddress returned for the
// current device (noalloc_scratch), never the name.
static __device__ __align__(256) unsigned char scratch[DI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[MAX_DEVICES] = {};

// The current device's copy of the scratch array (looked up once per device).
int noalloc_scratch(unsigned char **out) {
    int dev = 0;
    DI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) DI_FAIL(DI_EINVAL, "device %d beyond the %d the library supports", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) DI_FAIL(DI_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return DI_OK;
}

template <typename T>
int dalloc(di_ctx *c, T **p, i64 count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    DI_HIP(dev_malloc((void **)p, (size_t)count * sizeof(T)));
    c->device_bytes += count * (i64)sizeof(T);
    return DI_OK;
}

// launch order of a block-local graph's ranges: most work (edges inside plus entries
// arriving from other ranges) first, so that the last workgroups of a sweep are short
int make_range_order(di_ctx *c, const DevGraph &g, int **out) {
    const i64 nr = g.nranges;
    std::vector<i64> rbase(nr + 1), lbase(nr + 1);
    if (hipMemcpy(rbase.data(), g.rem_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(lbase.data(), g.loc_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost) != hipSuccess)
        DI_FAIL(DI_EHIP, "range table download failed");
    std::vector<int> order(nr);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (rbase[a + 1] - rbase[a]) + (lbase[a + 1] - lbase[a]) >
               (rbase[b + 1] - rbase[b]) + (lbase[b + 1] - lbase[b]);
    });
    DI_TRY(dalloc(c, out, nr));
    DI_HIP(hipMemcpy(*out, order.data(), sizeof(int) * nr, hipMemcpyHostToDevice));
    return DI_OK;
}

// Checks of a graph held on the device, the rules of validate_host_csr: out[0] = n - i for
// the first row i that ends before it starts, out[1] = m - p for the first target out of
// range, out[2] = m - p for the first weight that is not finite and > 0, out[3] = 1 when
// some row is not sorted by target (out starts at zero).  Row bounds are clamped to
// [0, m] before any edge is read, so a broken out_ptr reads nothing out of range.
__global__ void __launch_bounds__(256) k_check_csr(const i64 *__restrict__ ptr, const int *__restrict__ idx,
                                                   const float *__restrict__ w, i64 n, i64 m, u64 *out) {
    __shared__ u64 red[3][256 / WAVE];
    __shared__ unsigned uns_any;
    if (threadIdx.x == 0) uns_any = 0;
    __syncthreads();
    u64 br = 0, bi = 0, bw = 0;
    unsigned uns = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const i64 b = ptr[i], e = ptr[i + 1];
        if (e < b) br = max(br, (u64)(n - i));
        const i64 bb = min(max(b, (i64)0), m), ee = min(max(e, (i64)0), m);
        for (i64 p = bb; p < ee; ++p) {
            const int t = idx[p];
            if (t < 0 || (i64)t >= n) bi = max(bi, (u64)(m - p));
            if (p > bb && idx[p - 1] > t) uns = 1;
            if (w) {
                const float x = w[p];
                if (!(x > 0.0f) || !__builtin_isfinite(x)) bw = max(bw, (u64)(m - p));
            }
        }
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        br = max(br, (u64)__shfl_xor((unsigned long long)br, o, WAVE));
        bi = max(bi, (u64)__shfl_xor((unsigned long long)bi, o, WAVE));
        bw = max(bw, (u64)__shfl_xor((unsigned long long)bw, o, WAVE));
    }
    const int wv = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        red[0][wv] = br;
        red[1][wv] = bi;
        red[2][wv] = bw;
    }
    if (uns) atomicOr(&uns_any, 1u);
    __syncthreads();
    if (threadIdx.x == 0) {  // one atomic per block and value
        for (int k = 1; k < 256 / WAVE; ++k) {
            br = max(br, red[0][k]);
            bi = max(bi, red[1][k]);
            bw = max(bw, red[2][k]);
        }
        if (br) atomicMax((unsigned long long *)&out[0], (unsigned long long)br);
        if (bi) atomicMax((unsigned long long *)&out[1], (unsigned long long)bi);
        if (bw) atomicMax((unsigned long long *)&out[2], (unsigned long long)bw);
        if (uns_any) atomicOr((unsigned long long *)&out[3], 1ull);
    }
}

// validate_host_csr for a graph whose arrays are on the device; nothing is copied to the
// host but the verdict (and the values an error message names)
int validate_device_csr(const di_csr *g, hipStream_t st, bool *sorted) {
    const i64 n = g->n, m = g->m;
    i64 ends[2] = {0, 0};
    DI_HIP(hipMemcpy(&ends[0], g->out_ptr, sizeof(i64), hipMemcpyDeviceToHost));
    DI_HIP(hipMemcpy(&ends[1], g->out_ptr + n, sizeof(i64), hipMemcpyDeviceToHost));
    if (ends[0] != 0) DI_FAIL(DI_EINVAL, "out_ptr[0] must be 0");
    if (ends[1] != m) DI_FAIL(DI_EINVAL, "out_ptr[n] (%lld) must equal m (%lld)", (long long)ends[1], (long long)m);
    u64 *d_out = nullptr;
    DI_HIP(dev_malloc((void **)&d_out, 4 * sizeof(u64)));
    u64 h[4] = {0, 0, 0, 0};
    hipError_t e = launch_fill_zero(d_out, 4 * sizeof(u64), st) == DI_OK ? hipSuccess : hipErrorLaunchFailure;
    if (e == hipSuccess) {
        k_check_csr<<<grid_for(n, 256, 4096), 256, 0, st>>>(g->out_ptr, g->out_idx, g->w, n, m, d_out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)dev_free(d_out);
    if (e != hipSuccess) DI_FAIL(DI_EHIP, "graph check on the device failed: %s", hipGetErrorString(e));
    if (h[0]) DI_FAIL(DI_EINVAL, "out_ptr not non-decreasing at row %lld", (long long)(n - (i64)h[0]));
    if (h[1]) {
        const i64 p = m - (i64)h[1];
        int t = 0;
        DI_HIP(hipMemcpy(&t, g->out_idx + p, sizeof(int), hipMemcpyDeviceToHost));
        DI_FAIL(DI_EINVAL, "out_idx[%lld] = %d out of range [0, %lld)", (long long)p, t, (long long)n);
    }
    if (h[2]) {
        const i64 p = m - (i64)h[2];
        float x = 0.0f;
        DI_HIP(hipMemcpy(&x, g->w + p, sizeof(float), hipMemcpyDeviceToHost));
        DI_FAIL(DI_EINVAL, "w[%lld] = %g must be > 0 and finite", (long long)p, (double)x);
    }
    *sorted = h[3] == 0;
    return DI_OK;
}

int validate_host_csr(const di_csr *g, bool *sorted) {
    const i64 n = g->n, m = g->m;
    if (g->out_ptr[0] != 0) DI_FAIL(DI_EINVAL, "out_ptr[0] must be 0");
    if (g->out_ptr[n] != m) DI_FAIL(DI_EINVAL, "out_ptr[n] (%lld) must equal m (%lld)", (long long)g->out_ptr[n], (long long)m);
    *sorted = true;
    for (i64 i = 0; i < n; ++i) {
        const i64 b = g->out_ptr[i], e = g->out_ptr[i + 1];
        if (e < b) DI_FAIL(DI_EINVAL, "out_ptr not non-decreasing at row %lld", (long long)i);
        for (i64 p = b; p < e; ++p) {
            const int t = g->out_idx[p];
            if (t < 0 || (i64)t >= n) DI_FAIL(DI_EINVAL, "out_idx[%lld] = %d out of range [0, %lld)", (long long)p, t, (long long)n);
            if (p > b && g->out_idx[p - 1] > t) *sorted = false;
        }
    }
    if (g->w) {
        for (i64 p = 0; p < m; ++p) {
            const float w = g->w[p];
            if (!(w > 0.0f) || !std::isfinite(w)) DI_FAIL(DI_EINVAL, "w[%lld] = %g must be > 0 and finite", (long long)p, (double)w);
        }
    }
    return DI_OK;
}

// Sort each row by target (weights follow) on host copies.
void sort_rows(i64 n, const i64 *ptr, std::vector<int> &idx, std::vector<float> *w) {
    std::vector<i64> perm;
    for (i64 i = 0; i < n; ++i) {
        const i64 b = ptr[i], e = ptr[i + 1];
        if (e - b < 2) continue;
        perm.resize((size_t)(e - b));
        std::iota(perm.begin(), perm.end(), b);
        std::stable_sort(perm.begin(), perm.end(), [&](i64 x, i64 y) { return idx[x] < idx[y]; });
        std::vector<int> ti((size_t)(e - b));
        std::vector<float> tw(w ? (size_t)(e - b) : 0);
        for (i64 k = 0; k < e - b; ++k) {
            ti[k] = idx[perm[k]];
            if (w) tw[k] = (*w)[perm[k]];
        }
        for (i64 k = 0; k < e - b; ++k) {
            idx[b + k] = ti[k];
            if (w) (*w)[b + k] = tw[k];
        }
    }
}

int fixed_scale(double maxabs, i64 n) {
    int e_max = 0;
    if (maxabs > 0.0) std::frexp(maxabs, &e_max);
    int e_n = 0;
    while (((i64)1 << e_n) < n) ++e_n;
    return 118 - (e_max + e_n);
}

int sync_ctl(di_ctx *c, DevCtl *dctl) {
    DI_HIP(hipMemcpyAsync(c->h_ctl, dctl, sizeof(DevCtl), hipMemcpyDeviceToHost, c->st));
    DI_HIP(hipStreamSynchronize(c->st));
    return DI_OK;
}

// the leak from its limb sums (signed: fluid may be negative after a graph update)
double host_limbs(const u64 *l, int K) { return limbs_to_double_signed(l[0], l[1], l[2], l[3], K); }

__global__ void k_ctl_begin(DevCtl *c, long long max_sweeps) {
    c->done = 0;
    c->overflow = 0;
    c->budget = c->sweep + max_sweeps;
}

int ensure_row_blocks(di_ctx *c) {
    if (!c->rbin_ready) {
        const int rc = build_row_blocks(c->rbin, c->g.in_ptr, c->g.n, c->st);
        if (rc != DI_OK) {  // nothing half-built stays behind
            free_row_blocks(c->rbin);
            return rc;
        }
        c->rbin_ready = true;
    }
    return DI_OK;
}

// Frees the device buffers of a lazily allocated group and nulls them, after one of its
// allocations failed: the next call allocates the whole group again.
template <typename... P>
void free_group(P **...ps) {
    ((*ps ? (void)dev_free((void *)*ps) : (void)0, *ps = nullptr), ...);
}

__global__ void k_ctl_reopen(DevCtl *c) { c->done = 0; }

// Control step after a forward step (per graph for a union of graphs).
int enqueue_finalize(di_ctx *c, int mode, hipStream_t st) {
    if (c->s.range_graph) return launch_mg_finalize(c->s, c->s.ctl, c->p, mode, c->o.deterministic ? 1 : 0, st);
    return launch_finalize(c->s.ctl, c->p, mode, st, c->s.partR, c->s.nR, c->s.partC, mode == FIN_INIT ? 0 : c->s.nC);
}

int reset_state(di_ctx *c) {
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    DI_TRY(launch_init_fluid(c->s.F0, c->s.F, c->p.fp32, n, c->st));
    DI_TRY(launch_fill_zero(c->s.H, n * 8, c->st));
    DI_TRY(launch_fill_zero(c->s.S[0], c->s.S_bytes, c->st));
    DI_TRY(launch_fill_zero(c->s.S[1], c->s.S_bytes, c->st));
    DI_TRY(launch_fill_zero(c->s.ctl, sizeof(DevCtl), c->st));
    if (c->s.gctl) DI_TRY(launch_fill_zero(c->s.gctl, sizeof(GraphCtl) * c->s.n_graphs, c->st));
    DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st));
    DI_TRY(enqueue_finalize(c, FIN_INIT, c->st));
    DI_HIP(hipStreamSynchronize(c->st));
    c->forward_converged = false;
    return DI_OK;
}

// Fluid recomputation (float fluid): deliver the fluid in flight, then F = F_0 + dPH - H
// in double (equation HnFn), then the residual, threshold and stop state of the result.
constexpr double REFINE_DROP = 0x1p-14;
// while the fluid is float, sweeps aim at REFINE_MARGIN * tol so that the residual of
// the recomputed fluid (the float pushes' rounding added back) still meets tol
constexpr double REFINE_MARGIN = 0.8;
// share of the cross-range entries that must carry fluid in a block-local sweep for the
// next one to read the in-flight values without testing the bitmap (on the 50M web graph
// the direct reads win at about 0.6 of the entries live, the bitmap at about 0.4)
constexpr double DENSE_DELIVERY = 0.5;

int refine_fluid(di_ctx *c, double tol) {
    const size_t T = c->p.fp32 ? 4 : 8;
    DI_TRY(ensure_row_blocks(c));
    if (!c->ref_ht) DI_TRY(dalloc(c, &c->ref_ht, c->g.n));
    DI_TRY(launch_bld_sweep(c->g, c->s, c->p, 0, c->st));
    DI_TRY(enqueue_finalize(c, FIN_DELIVER, c->st));
    DI_TRY(launch_fill_zero(c->s.S[0], c->s.S_bytes, c->st));
    DI_TRY(launch_fill_zero(c->s.S[1], c->s.S_bytes, c->st));
    DI_TRY(launch_refine_fluid(c->g, c->rbin, c->s, c->p, c->ref_ht, c->st));
    if (!c->s.range_graph) {
        k_ctl_reopen<<<1, 1, 0, c->st>>>(c->s.ctl);
        DI_LAUNCH_CHECK();
    }
    DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st, 0));
    const double sweep_tol = c->p.tol;
    c->p.tol = tol;
    const int rc = enqueue_finalize(c, FIN_INIT, c->st);
    c->p.tol = sweep_tol;
    DI_TRY(rc);
    return sync_ctl(c, c->s.ctl);
}

int enqueue_di_sweep(di_ctx *c, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (e0) DI_HIP(hipEventRecord(e0, st));
    if (c->o.deterministic) DI_TRY(launch_det_sweep(c->g, c->s, c->p, st));
    else DI_TRY(launch_bld_sweep(c->g, c->s, c->p, c->rounds, st));
    if (e1) DI_HIP(hipEventRecord(e1, st));
    return enqueue_finalize(c, FIN_DI, st);
}

// one power iteration on the iterates, x/s vectors and control block of s
int enqueue_pi_iteration_on(di_ctx *c, SolveState &s, hipStream_t st, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr) {
    if (e0) DI_HIP(hipEventRecord(e0, st));
    DI_TRY(launch_pi_iteration(c->g, c->rbin, s, c->p, st));
    if (e1) DI_HIP(hipEventRecord(e1, st));
    return launch_finalize(s.pctl, c->p, FIN_PI, st, s.partR, s.nR, s.partC, 0);
}

int enqueue_pi_iteration(di_ctx *c, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    return enqueue_pi_iteration_on(c, c->s, st, e0, e1);
}

// After a synced chunk: add the device time of the steps that really ran.
int collect_timing(di_ctx *c, i64 ran) {
    for (i64 k = 0; k < ran && k < c->spc; ++k) {
        float ms = 0.0f;
        DI_HIP(hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]));
        c->kernel_ns += 1e6 * (double)ms;
        c->kernel_launches += 1;
    }
    return DI_OK;
}

// Enqueue one chunk of `spc` steps, either directly or through a captured graph.
int enqueue_chunk(di_ctx *c, int kind /* 0 DI, 1 PI */) {
    if (c->o.loop_mode == DI_LOOP_GRAPH) {
        if (!c->gexec || c->gexec_kind != kind) {
            if (c->gexec) {
                (void)hipGraphExecDestroy(c->gexec);
                c->gexec = nullptr;
            }
            if (!c->cap_st) DI_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            DI_HIP(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
            int rc = DI_OK;
            for (int k = 0; k < c->spc && rc == DI_OK; ++k)
                rc = kind ? enqueue_pi_iteration(c, c->cap_st) : enqueue_di_sweep(c, c->cap_st);
            hipError_t e = hipStreamEndCapture(c->cap_st, &graph);
            if (rc != DI_OK) return rc;
            if (e != hipSuccess) DI_FAIL(DI_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) DI_FAIL(DI_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
            c->gexec_kind = kind;
        }
        DI_HIP(hipGraphLaunch(c->gexec, c->st));
        return DI_OK;
    }
    const bool timed = c->o.timing != 0;
    if (timed && (int)c->tev.size() < 2 * c->spc) {
        while ((int)c->tev.size() < 2 * c->spc) {
            hipEvent_t e;
            DI_HIP(hipEventCreate(&e));
            c->tev.push_back(e);
        }
    }
    for (int k = 0; k < c->spc; ++k) {
        hipEvent_t e0 = timed ? c->tev[2 * k] : nullptr, e1 = timed ? c->tev[2 * k + 1] : nullptr;
        DI_TRY(kind ? enqueue_pi_iteration(c, c->st, e0, e1) : enqueue_di_sweep(c, c->st, e0, e1));
    }
    return DI_OK;
}

void fill_stats(di_stats *st, const DevCtl &h, const DevCtl &before, double d, int K, float ms, bool pi,
                double zsum = 1.0) {
    if (!st) return;
    st->sweeps = h.sweep - before.sweep;
    st->edge_updates = (int64_t)(h.tot_edges - before.tot_edges);
    st->node_updates = (int64_t)(h.tot_nodes - before.tot_nodes);
    st->residual = h.R;
    st->bound = h.R / (1.0 - d);
    const double l = pi ? 0.0 : host_limbs(h.limbsL, K);
    st->leak = l;
    st->bound_norm = pi ? st->bound : h.R / (1.0 - d - d * l / zsum);
    st->ms = ms;
    st->mass_defect = 0.0;
    st->converged = h.done && !h.overflow;
}

// ---------------------------------------------------------------------------
// DI_LOG: when the environment names a file, every host synchronisation of a solve loop
// (every sweeps_per_sync sweeps; 1 gives a record per sweep) and the end of every
// di_diffuse, di_power and di_adjoint call append one JSON line to it: the call, the
// context, the sweep index, the call's counters so far, DI rounds (diffusions / n), the
// residual, the certified bounds, the leak and the host time since the call began.  The
// end record adds the status, the convergence flag, the mass defect, the device time and
// the GEUPS.  The variable is read at every record; unset or empty, nothing is written.
// ---------------------------------------------------------------------------
std::mutex g_log_mu;
FILE *g_log_file = nullptr;
std::string g_log_path;

bool log_on() {
    const char *p = std::getenv("DI_LOG");
    return p && *p;
}

void log_line(const char *line) {
    const char *p = std::getenv("DI_LOG");
    if (!p || !*p) return;
    std::lock_guard<std::mutex> lk(g_log_mu);
    if (!g_log_file || g_log_path != p) {
        if (g_log_file) fclose(g_log_file);
        g_log_file = fopen(p, "a");
        g_log_path = p;
        if (!g_log_file) return;  // logging is best effort: a solve never fails for it
    }
    fputs(line, g_log_file);
    fputc('\n', g_log_file);
    fflush(g_log_file);
}

// a JSON number, or null for a value that is not finite (a run that overflowed)
struct JNum {
    char b[40];
    explicit JNum(double v) {
        if (std::isfinite(v)) snprintf(b, sizeof(b), "%.17g", v);
        else snprintf(b, sizeof(b), "null");
    }
};

void log_record(const di_ctx *c, i64 n, const char *call, const char *event, long long sweep, const di_stats &s,
                const int *status) {
    if (!log_on()) return;
    const double host_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c->call_t0).count();
    char buf[1024];
    int k = snprintf(buf, sizeof(buf),
                     "{\"call\":\"%s\",\"event\":\"%s\",\"ctx\":\"%p\",\"sweep\":%lld,\"sweeps\":%lld,"
                     "\"node_updates\":%lld,\"edge_updates\":%lld,\"rounds\":%.6g,\"residual\":%s,"
                     "\"bound\":%s,\"bound_norm\":%s,\"leak\":%s,\"host_ms\":%.3f",
                     call, event, (const void *)c, sweep, (long long)s.sweeps, (long long)s.node_updates,
                     (long long)s.edge_updates, n > 0 ? (double)s.node_updates / (double)n : 0.0,
                     JNum(s.residual).b, JNum(s.bound).b, JNum(s.bound_norm).b, JNum(s.leak).b, host_ms);
    if (status && k > 0 && k < (int)sizeof(buf))
        k += snprintf(buf + k, sizeof(buf) - k,
                      ",\"status\":%d,\"converged\":%d,\"mass_defect\":%s,\"device_ms\":%.4f,\"geups\":%.6g",
                      *status, s.converged, JNum(s.mass_defect).b, s.ms,
                      s.ms > 0 ? (double)s.edge_updates / (s.ms * 1e6) : 0.0);
    if (k > 0 && k < (int)sizeof(buf) - 2) {
        buf[k] = '}';
        buf[k + 1] = 0;
        log_line(buf);
    }
}

// Internal (padded) layout of a union of graphs -> caller's numbering, times a per-graph
// scale when given.  Node i of graph g (graph_ptr[g] <= i < graph_ptr[g+1]) sits at
// gstart[g] + i - graph_ptr[g].
template <typename T>
__global__ void k_unpad(const T *__restrict__ src, i64 n_user, const i64 *__restrict__ gp,
                        const i64 *__restrict__ gs, const double *__restrict__ scale, i64 G, double *dst) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n_user; i += (i64)gridDim.x * blockDim.x) {
        i64 lo = 0, hi = G - 1;  // last graph with gp[g] <= i
        while (lo < hi) {
            const i64 mid = (lo + hi + 1) >> 1;
            if (gp[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const double v = (double)src[i - gp[lo] + gs[lo]];
        dst[i] = scale ? v * scale[lo] : v;
    }
}

// Per-graph control blocks of a union of graphs, copied to c->h_gctl.
int sync_gctl(di_ctx *c) {
    c->h_gctl.resize((size_t)c->s.n_graphs);
    DI_HIP(hipMemcpyAsync(c->h_gctl.data(), c->s.gctl, sizeof(GraphCtl) * c->s.n_graphs, hipMemcpyDeviceToHost, c->st));
    DI_HIP(hipStreamSynchronize(c->st));
    return DI_OK;
}

// Statistics of a union of graphs: the residual and bounds are the largest over the
// graphs (each graph is certified on its own), the leak is the sum.
int fill_stats_mg(di_ctx *c, di_stats *st, const DevCtl &h, const DevCtl &before, float ms) {
    if (!st) return DI_OK;
    DI_TRY(sync_gctl(c));
    fill_stats(st, h, before, c->d, c->p.K, ms, false);
    double R = 0.0, bn = 0.0, lsum = 0.0;
    for (i64 g = 0; g < c->s.n_graphs; ++g) {
        const GraphCtl &gc = c->h_gctl[g];
        const double l = host_limbs(gc.limbsL, c->p.K);
        R = std::max(R, gc.R);
        bn = std::max(bn, gc.R / (1.0 - c->d - c->d * l / c->h_ginfo[g].zsum));
        lsum += l;
    }
    st->residual = R;
    st->bound = R / (1.0 - c->d);
    st->bound_norm = bn;
    st->leak = lsum;
    return DI_OK;
}

// Mass balance of the current state per graph (one value for one graph), kept in
// c->defects: sum F + (1-d) sum H + d l - (1-d) sum Z.  Equation HnFn gives
// H + F = F_0 + d P H; summing its entries with 1^T P = 1^T - 1_D^T (the columns of P sum
// to 1 except at dangling nodes, Section 2.1) leaves this sum at zero in exact
// arithmetic.  sum F and sum H are exact signed fixed-point sums on the device (the fluid
// in flight has been delivered at the end of every call); the stats get the largest
// magnitude.
int mass_defects(di_ctx *c, di_stats *st) {
    const i64 G = c->s.range_graph ? c->n_graphs : 1;
    c->defects.assign((size_t)G, 0.0);
    if (c->b) {
        c->defects.resize((size_t)c->k);
        DI_TRY(batch_mass_defects(c->b, c->g, c->p, c->defects.data(), c->st));
    } else {
        double zmax = c->zsum;
        if (G > 1)
            for (i64 q = 0; q < G; ++q) zmax = std::max(zmax, c->h_ginfo[q].zsum);
        // history and fluid sums stay within a few times the sum of Z (|P|_1 <= 1, and the
        // fluid only falls in L1 once a call has started), so a fixed-point scale for n
        // values of size 8 zmax leaves room
        const int KH = fixed_scale(8.0 * zmax, c->g.n);
        DI_TRY(launch_node_sums(c->g, c->s, c->s.H, 0, KH, c->s.partH, c->s.hsum, c->st));
        DI_TRY(launch_node_sums(c->g, c->s, c->s.F, c->p.fp32, KH, c->s.partH, c->s.hsum + G, c->st));
        std::vector<double> hs((size_t)(2 * G));
        DI_HIP(hipMemcpyAsync(hs.data(), c->s.hsum, sizeof(double) * 2 * G, hipMemcpyDeviceToHost, c->st));
        DI_TRY(sync_ctl(c, c->s.ctl));
        if (G > 1) {
            DI_TRY(sync_gctl(c));
            for (i64 q = 0; q < G; ++q) {
                const GraphCtl &gc = c->h_gctl[q];
                c->defects[q] = hs[G + q] + (1.0 - c->d) * hs[q] + c->d * host_limbs(gc.limbsL, c->p.K) -
                                (1.0 - c->d) * c->h_ginfo[q].zsum;
            }
        } else {
            const DevCtl &h = *c->h_ctl;
            c->defects[0] = hs[1] + (1.0 - c->d) * hs[0] + c->d * host_limbs(h.limbsL, c->p.K) - (1.0 - c->d) * c->zsum;
        }
    }
    if (st) {
        double v = 0.0;
        for (double x : c->defects)
            if (std::fabs(x) > std::fabs(v)) v = x;
        st->mass_defect = v;
    }
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Cut-aligned ranges (one graph, one right-hand side, fast sweeps).  lcut(p) counts the
// edges shorter than a range that cross the boundary between nodes p-1 and p; a range that
// starts at caller node s ends at the p in (s + B - X, s + B] with the smallest lcut (the
// largest such p on ties), and its slots past p - s are padding.  The relabelling is
// monotone, so rows stay sorted, IN keeps its order, and OUT keeps its edge order.
// ---------------------------------------------------------------------------
__global__ void k_short_crossings(const i64 *__restrict__ ptr, const int *__restrict__ idx, i64 n, i64 B,
                                  unsigned long long *diff) {
    for (i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (i64)gridDim.x * blockDim.x) {
        for (i64 e = ptr[u]; e < ptr[u + 1]; ++e) {
            const i64 v = idx[e];
            const i64 lo = v < u ? v : u, hi = v < u ? u : v;
            if (hi != lo && hi - lo < B) {
                atomicAdd(&diff[lo + 1], 1ull);
                atomicAdd(&diff[hi + 1], ~0ull);  // -1 modulo 2^64
            }
        }
    }
}

// internal row pointer: slot j of range r is caller node start[r] + j, or padding (an
// empty row at the end of the range's edges)
__global__ void k_pad_rows(const i64 *__restrict__ ptr, const i64 *__restrict__ start, i64 nr, int rb, i64 n_int,
                           i64 m, i64 *pptr) {
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q <= n_int; q += (i64)gridDim.x * blockDim.x) {
        if (q == n_int) {
            pptr[q] = m;
            continue;
        }
        const i64 r = q >> rb, j = q & (((i64)1 << rb) - 1), len = start[r + 1] - start[r];
        pptr[q] = ptr[start[r] + (j < len ? j : len)];
    }
}

// targets to internal numbers; coarse[t] = the range holding caller node t << cs (every
// range holds at least 2^cs caller nodes, so the walk takes at most two steps)
__global__ void k_relabel(int *idx, i64 m, const i64 *__restrict__ start, const int *__restrict__ coarse, int cs,
                          int rb) {
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (i64)gridDim.x * blockDim.x) {
        const i64 u = idx[e];
        i64 r = coarse[u >> cs];
        while (start[r + 1] <= u) ++r;
        idx[e] = (int)((r << rb) + (u - start[r]));
    }
}

// Upload OUT in the internal numbering of cut-aligned ranges.  Sets c->seg, c->seg_start and
// c->g.n; returns DI_OK with c->seg = false when no range would end early.
int upload_segmented(di_ctx *c, const i64 *ptr, const int *idx, const float *w, i64 n, i64 m, int rb, i64 X) {
    const i64 B = (i64)1 << rb;
    i64 *d_ptr = nullptr;
    int *d_idx = nullptr;
    unsigned long long *diff = nullptr;
    i64 *excl = nullptr, *temp = nullptr;
    auto cleanup = [&]() {
        for (void *q : {(void *)d_ptr, (void *)diff, (void *)excl, (void *)temp})
            if (q) (void)dev_free(q);
    };
    hipError_t last = hipSuccess;
    auto hip_ok = [&](hipError_t e) {
        if (e == hipSuccess) return true;
        last = e;
        set_error("cut-aligned range layout: %s", hipGetErrorString(e));
        return false;
    };
    auto hip_code = [&]() { return last == hipErrorOutOfMemory ? DI_ENOMEM : DI_EHIP; };
    if (!hip_ok(dev_malloc((void **)&d_ptr, sizeof(i64) * (n + 1))) ||
        !hip_ok(dev_malloc((void **)&d_idx, sizeof(int) * std::max<i64>(m, 1))) ||
        !hip_ok(dev_malloc((void **)&diff, sizeof(i64) * (n + 2))) ||
        !hip_ok(dev_malloc((void **)&excl, sizeof(i64) * (n + 2))) ||
        !hip_ok(dev_malloc((void **)&temp, sizeof(i64) * (scan_temp_elems(n + 2) + 64))) ||
        !hip_ok(hipMemcpy(d_ptr, ptr, sizeof(i64) * (n + 1), hipMemcpyDefault)) ||
        (m && !hip_ok(hipMemcpy(d_idx, idx, sizeof(int) * m, hipMemcpyDefault)))) {
        cleanup();
        if (d_idx) (void)dev_free(d_idx);
        return hip_code();
    }
    c->g.out_idx = d_idx;  // owned by the context from here on
    int rc = launch_fill_zero(diff, sizeof(i64) * (n + 2), c->st);
    if (rc == DI_OK) {
        k_short_crossings<<<grid_for(n, 256, 16384), 256, 0, c->st>>>(d_ptr, d_idx, n, B, diff);
        if (hipGetLastError() != hipSuccess) rc = DI_EHIP;
    }
    // lcut(p) = sum of diff[0..p] = the exclusive scan at p + 1
    if (rc == DI_OK) rc = scan_exclusive(reinterpret_cast<const i64 *>(diff), excl, n + 2, temp, c->st);
    std::vector<i64> lcut((size_t)n + 2);
    if (rc == DI_OK && !hip_ok(hipMemcpyAsync(lcut.data(), excl, sizeof(i64) * (n + 2), hipMemcpyDeviceToHost, c->st)))
        rc = DI_EHIP;
    if (rc == DI_OK && !hip_ok(hipStreamSynchronize(c->st))) rc = DI_EHIP;
    if (rc != DI_OK) {
        cleanup();
        return rc;
    }
    std::vector<i64> start{0};
    for (i64 s = 0; n - s > B;) {
        i64 best = s + B;
        for (i64 p = s + B; p > s + B - X; --p)
            if (lcut[p + 1] < lcut[best + 1]) best = p;
        start.push_back(best);
        s = best;
    }
    start.push_back(n);
    const i64 nr = (i64)start.size() - 1;
    if (nr == (n + B - 1) / B) {  // every range full: the plain layout (OUT as uploaded)
        c->g.out_ptr = d_ptr;
        d_ptr = nullptr;
        cleanup();
        return DI_OK;
    }
    const i64 n_int = (nr - 1) * B + (n - start[nr - 1]);
    if (n_int >= 0x7fffffffll) {
        cleanup();
        set_error("cut-aligned ranges need more than 2^31 - 1 internal nodes; use range_cut = -1");
        return DI_EINVAL;
    }
    const int cs = rb - 1;  // every range holds more than B - X >= B / 2 caller nodes
    std::vector<int> coarse((size_t)((n - 1) >> cs) + 1);
    for (i64 r = 0, t = 0; t < (i64)coarse.size(); ++t) {
        while (start[r + 1] <= (t << cs)) ++r;
        coarse[t] = (int)r;
    }
    i64 *d_start = nullptr;
    int *d_coarse = nullptr;
    i64 *pptr = nullptr;
    if (!hip_ok(dev_malloc((void **)&d_start, sizeof(i64) * (nr + 1))) ||
        !hip_ok(dev_malloc((void **)&d_coarse, sizeof(int) * coarse.size())) ||
        !hip_ok(dev_malloc((void **)&pptr, sizeof(i64) * (n_int + 1))) ||
        !hip_ok(hipMemcpy(d_start, start.data(), sizeof(i64) * (nr + 1), hipMemcpyHostToDevice)) ||
        !hip_ok(hipMemcpy(d_coarse, coarse.data(), sizeof(int) * coarse.size(), hipMemcpyHostToDevice))) {
        for (void *q : {(void *)d_start, (void *)d_coarse, (void *)pptr})
            if (q) (void)dev_free(q);
        cleanup();
        return hip_code();
    }
    k_pad_rows<<<grid_for(n_int + 1, 256, 16384), 256, 0, c->st>>>(d_ptr, d_start, nr, rb, n_int, m, pptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && m) {
        k_relabel<<<grid_for(m, 256, 16384), 256, 0, c->st>>>(d_idx, m, d_start, d_coarse, cs, rb);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    (void)dev_free(d_coarse);
    cleanup();
    if (!hip_ok(e)) {
        (void)dev_free(pptr);
        (void)dev_free(d_start);
        return hip_code();
    }
    c->d_seg_start = d_start;
    c->g.out_ptr = pptr;
    c->g.n = n_int;
    c->seg = true;
    c->seg_rb = rb;
    c->seg_start = std::move(start);
    (void)w;
    return DI_OK;
}

// the same two mappings on the device (grid-stride over internal nodes q)
__global__ void k_seg_to_internal(const double *__restrict__ src, double *dst, const i64 *__restrict__ start, int rb,
                                  i64 n_int) {
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < n_int; q += (i64)gridDim.x * blockDim.x) {
        const i64 r = q >> rb, j = q & (((i64)1 << rb) - 1);
        dst[q] = j < start[r + 1] - start[r] ? src[start[r] + j] : 0.0;
    }
}

// max |g_i| as the bits of a nonnegative double (they order like the values) into out[0],
// and n - i for the first non-finite g_i into out[1] (0: none); out starts at zero
__global__ void __launch_bounds__(256) k_check_rhs(const double *__restrict__ g, i64 n, u64 *out) {
    __shared__ u64 red[2][256 / WAVE];
    u64 mx = 0, bad = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const double v = g[i];
        if (!__builtin_isfinite(v)) bad = max(bad, (u64)(n - i));
        else mx = max(mx, (u64)__double_as_longlong(fabs(v)));
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mx = max(mx, (u64)__shfl_xor((unsigned long long)mx, o, WAVE));
        bad = max(bad, (u64)__shfl_xor((unsigned long long)bad, o, WAVE));
    }
    const int wv = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        red[0][wv] = mx;
        red[1][wv] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // one atomic per block and value
        for (int k = 1; k < 256 / WAVE; ++k) {
            mx = max(mx, red[0][k]);
            bad = max(bad, red[1][k]);
        }
        if (mx) atomicMax((unsigned long long *)&out[0], (unsigned long long)mx);
        if (bad) atomicMax((unsigned long long *)&out[1], (unsigned long long)bad);
    }
}

__global__ void k_seg_to_caller(const double *__restrict__ src, double *dst, const i64 *__restrict__ start, int rb,
                                i64 n_int) {
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < n_int; q += (i64)gridDim.x * blockDim.x) {
        const i64 r = q >> rb, j = q & (((i64)1 << rb) - 1);
        if (j < start[r + 1] - start[r]) dst[start[r] + j] = src[q];
    }
}

// caller array (n_user values) -> internal layout of cut-aligned ranges (padding gets 0)
__global__ void k_caller_to_seg(const double *__restrict__ src, double *dst, const i64 *__restrict__ start, int rb,
                                i64 n_int) {
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < n_int; q += (i64)gridDim.x * blockDim.x) {
        const i64 r = q >> rb, j = q & (((i64)1 << rb) - 1);
        dst[q] = j < start[r + 1] - start[r] ? src[start[r] + j] : 0.0;
    }
}

// Theorem 4: F' = F + d (P'H - PH) in double, stored in the fluid type; the largest |F'|
// (bits of a nonnegative double order like the double) into *maxbits
template <typename T>
__global__ void k_update_fluid(const double *__restrict__ F, const double *__restrict__ PH_new,
                               const double *__restrict__ PH_old, double d, i64 n, T *Fout, u64 *maxbits) {
    u64 mx = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const T f = (T)(F[i] + d * (PH_new[i] - PH_old[i]));
        Fout[i] = f;
        const u64 b = (u64)__double_as_longlong(fabs((double)f));
        mx = b > mx ? b : mx;
    }
    mx = wave_max_u64(mx);
    if ((threadIdx.x & (WAVE - 1)) == 0 && mx) atomicMax(maxbits, mx);
}

// exact signed sum of H over the dangling nodes (1/s = 0) into per-workgroup limb slots
__global__ void __launch_bounds__(256) k_dangling_history(const double *__restrict__ H, const double *__restrict__ inv_s,
                                                          i64 n, int K, u64 *part) {
    __shared__ u64 red[4 * 4];
    Limbs S;
    limbs_zero(S);
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        if (inv_s[i] == 0.0) limbs_add_signed(S, H[i], K);
    u64 w[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
    block_store_partials<4>(w, red, part + (i64)blockIdx.x * PSR);
}

// the leak of the control block := the sum of the slots (normalised limbs)
__global__ void __launch_bounds__(256) k_set_leak(DevCtl *ctl, const u64 *__restrict__ part, i64 nslots) {
    __shared__ u64 red[4 * 4];
    __shared__ u64 tot[4];
    u64 v[4] = {0, 0, 0, 0};
    for (i64 q = threadIdx.x; q < nslots; q += blockDim.x)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += part[q * PSR + k];
    block_store_partials<4>(v, red, tot);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; ++k) ctl->limbsL[k] = tot[k];
        limbs_normalize(ctl->limbsL);
    }
}

// caller array (n_user values) -> internal layout (padding gets fill)
void seg_expand(const di_ctx *c, const double *src, double *dst, double fill) {
    const i64 B = (i64)1 << c->seg_rb, nr = (i64)c->seg_start.size() - 1;
    for (i64 r = 0; r < nr; ++r) {
        const i64 s = c->seg_start[r], len = c->seg_start[r + 1] - s;
        for (i64 j = 0; j < B && r * B + j < c->g.n; ++j) dst[r * B + j] = j < len ? src[s + j] : fill;
    }
}

// internal layout -> caller array
template <typename T>
void seg_compact(const di_ctx *c, const T *src, T *dst) {
    const i64 B = (i64)1 << c->seg_rb, nr = (i64)c->seg_start.size() - 1;
    for (i64 r = 0; r < nr; ++r) {
        const i64 s = c->seg_start[r], len = c->seg_start[r + 1] - s;
        for (i64 j = 0; j < len; ++j) dst[s + j] = src[r * B + j];
    }
}

// caller node of internal (real) node q
inline i64 seg_user(const di_ctx *c, i64 q) {
    return c->seg_start[q >> c->seg_rb] + (q & (((i64)1 << c->seg_rb) - 1));
}

}  // namespace

extern "C" {

const char *di_last_error(void) { return g_err; }

int di_destroy(di_ctx *c) {
    if (!c) return DI_OK;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    free_graph(c->g);
    free_graph(c->gT);
    free_row_blocks(c->rbin);
    free_row_blocks(c->rbout);
    void *ps[] = {c->s.F, c->s.F0, c->s.H, c->s.S[0], c->s.S[1], c->s.snap, c->s.frontier, c->s.range_order,
                  c->s.ctl, c->s.X[0], c->s.X[1], c->s.XT[0], c->s.XT[1], c->s.pctl, c->s.Z, c->lam,
                  c->aF, c->asnap, c->aZ, c->achk, c->actl, c->s.partR, c->s.partC, c->s.range_graph, c->s.range_cnt, c->d_seg_start, c->s.ginfo, c->s.gctl,
                  c->d_gp, c->d_gs, c->d_gscale, c->ref_ht, c->s.partH, c->s.hsum, c->aS[0], c->aS[1]};
    for (void *p : ps)
        if (p) (void)dev_free(p);
    if (c->b) free_batch(c->b);
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return DI_OK;
}

int di_init(di_ctx **out, const di_csr *g, double d, const double *Z, const di_opts *o) {
    if (!out) DI_FAIL(DI_EINVAL, "ctx pointer is NULL");
    *out = nullptr;
    if (!g) DI_FAIL(DI_EINVAL, "graph is NULL");
    if (g->n < 1 || g->m < 0) DI_FAIL(DI_EINVAL, "need n >= 1 and m >= 0 (n=%lld, m=%lld)", (long long)g->n, (long long)g->m);
    if (g->n >= 0x7fffffffll) DI_FAIL(DI_EINVAL, "n must be below 2^31 - 1");
    if (g->m >= 0xffffffffll) DI_FAIL(DI_EINVAL, "m must be below 2^32 - 1");
    if (!g->out_ptr || (g->m > 0 && !g->out_idx)) DI_FAIL(DI_EINVAL, "out_ptr / out_idx are NULL");
    if (!(d > 0.0 && d < 1.0)) DI_FAIL(DI_EINVAL, "d must lie in (0, 1), got %g", d);
    di_opts opt{};
    opt.theta = 1.0;
    opt.k = 1;
    opt.n_graphs = 1;
    if (o) opt = *o;
    if (opt.theta == 0.0 && o == nullptr) opt.theta = 1.0;
    if (!(opt.theta >= 0.0) || !std::isfinite(opt.theta)) DI_FAIL(DI_EINVAL, "theta must be finite and >= 0");
    if (opt.k == 0) opt.k = 1;
    if (opt.k < 1 || opt.k > 64) DI_FAIL(DI_EINVAL, "k must be in 1..64");
    if (opt.n_graphs == 0) opt.n_graphs = 1;
    if (opt.n_graphs < 1) DI_FAIL(DI_EINVAL, "n_graphs must be >= 1");
    if (opt.n_graphs > 1 && !opt.graph_ptr) DI_FAIL(DI_EINVAL, "graph_ptr required when n_graphs > 1");
    if (opt.n_graphs > 1 && opt.k > 1) DI_FAIL(DI_EINVAL, "k > 1 with n_graphs > 1 is not supported");
    if (opt.max_sweeps < 0) DI_FAIL(DI_EINVAL, "max_sweeps must be >= 0");
    if (opt.max_sweeps == 0) opt.max_sweeps = 100000;
    {
        const int lo = opt.k > 1 ? 6 : 8, hi = 13;
        if (opt.range_log2 != 0 && (opt.range_log2 < lo || opt.range_log2 > hi))
            DI_FAIL(DI_EINVAL, "range_log2 must be 0 or in %d..%d", lo, hi);
    }
    if (opt.inner_rounds < 0 || opt.inner_rounds > 64) DI_FAIL(DI_EINVAL, "inner_rounds must be in 0..64");
    if (opt.loop_mode != DI_LOOP_STREAM && opt.loop_mode != DI_LOOP_GRAPH) DI_FAIL(DI_EINVAL, "bad loop_mode");
    if (opt.sweeps_per_sync < 0) DI_FAIL(DI_EINVAL, "sweeps_per_sync must be >= 0");
    if (opt.range_cut < -1) DI_FAIL(DI_EINVAL, "range_cut must be -1, 0 or positive");
    i64 n = g->n;
    const i64 m = g->m;
    if (opt.n_graphs > 1) {
        if (opt.graph_ptr[0] != 0 || opt.graph_ptr[opt.n_graphs] != n) DI_FAIL(DI_EINVAL, "graph_ptr must run from 0 to n");
        for (i64 q = 0; q < opt.n_graphs; ++q)
            if (opt.graph_ptr[q + 1] <= opt.graph_ptr[q]) DI_FAIL(DI_EINVAL, "graph_ptr must be strictly increasing");
    }

    // host view of the graph (copied back when given on the device), validated
    std::vector<i64> hptr;
    std::vector<int> hidx;
    std::vector<float> hw;
    const i64 *ptr = g->out_ptr;
    const int *idx = g->out_idx;
    const float *w = g->w;
    // a graph on the device with rows sorted by target is checked there and copied device
    // to device; a union of graphs (relabelled on the host) or unsorted rows take the host path
    bool checked = false;
    if (g->on_device && opt.n_graphs <= 1) {
        bool sorted_dev = false;
        DI_TRY(validate_device_csr(g, (hipStream_t)opt.stream, &sorted_dev));
        checked = sorted_dev;
    }
    if (g->on_device && !checked) {
        hptr.resize((size_t)n + 1);
        hidx.resize((size_t)std::max<i64>(m, 1));
        DI_HIP(hipMemcpy(hptr.data(), g->out_ptr, sizeof(i64) * (n + 1), hipMemcpyDeviceToHost));
        if (m) DI_HIP(hipMemcpy(hidx.data(), g->out_idx, sizeof(int) * m, hipMemcpyDeviceToHost));
        if (g->w) {
            hw.resize((size_t)std::max<i64>(m, 1));
            if (m) DI_HIP(hipMemcpy(hw.data(), g->w, sizeof(float) * m, hipMemcpyDeviceToHost));
        }
        ptr = hptr.data();
        idx = hidx.data();
        w = g->w ? hw.data() : nullptr;
    }
    di_csr hv = *g;
    hv.out_ptr = ptr;
    hv.out_idx = idx;
    hv.w = w;
    bool sorted = true;
    if (!checked) DI_TRY(validate_host_csr(&hv, &sorted));
    if (!sorted) {
        if (hidx.empty()) hidx.assign(idx, idx + m);
        if (w && hw.empty()) hw.assign(w, w + m);
        sort_rows(n, ptr, hidx, w ? &hw : nullptr);
        idx = hidx.data();
        w = w ? hw.data() : nullptr;
    }

    // Z (n x k column-major), validated; NULL = uniform per column / per graph
    const int k = opt.k;
    std::vector<double> hz;
    if (Z) {
        for (int col = 0; col < k; ++col) {
            double s = 0.0;
            for (i64 i = 0; i < n; ++i) {
                const double v = Z[(i64)col * n + i];
                if (!(v >= 0.0) || !std::isfinite(v)) DI_FAIL(DI_EINVAL, "Z[%lld, %d] must be finite and >= 0", (long long)i, col);
                s += v;
            }
            if (!(s > 0.0)) DI_FAIL(DI_EINVAL, "column %d of Z sums to zero", col);
        }
    }

    // block-local range size: unweighted graphs use the LDS-resident kernel with 2^11-node
    // ranges; weighted graphs 2^12-node ranges (two workgroups of the weighted sweep per
    // compute unit); small graphs keep at least ~256 nodes per range so that several
    // workgroups run
    int rb = opt.range_log2;
    if (rb == 0 && opt.k > 1 && !opt.deterministic) {
        // several columns: ranges whose k-column fluid tile and local edge lists fit in
        // half of a compute unit's LDS
        rb = tile_range_log2(opt.k, opt.fluid_fp32, w != nullptr);
        if (rb == 0) rb = 8;
    } else if (rb == 0) {
        // weighted: the largest range that lets two workgroups of the weighted sweep share
        // a compute unit (2^12 nodes)
        const int cap = w ? 12 : 11;
        rb = 8;
        while (rb < cap && ((i64)1 << (rb + 1)) * 256 <= n) ++rb;
    }

    // union of graphs: every graph starts on a range boundary; edges must stay inside
    // their graph; Z (given, or uniform 1/n_g per graph) is laid out the same way
    std::vector<i64> pptr, gstart;
    std::vector<int> pidx;
    std::vector<double> pz;
    std::vector<HostSum> gzsum;
    const i64 n_user = n;
    if (opt.n_graphs > 1) {
        const i64 G = opt.n_graphs, B = (i64)1 << rb;
        const i64 *gp = opt.graph_ptr;
        gstart.resize((size_t)G + 1);
        gstart[0] = 0;
        for (i64 q = 0; q < G; ++q) gstart[q + 1] = gstart[q] + ((gp[q + 1] - gp[q] + B - 1) / B) * B;
        const i64 n2 = gstart[G];
        if (n2 >= 0x7fffffffll) DI_FAIL(DI_EINVAL, "the graphs padded to ranges of %lld nodes exceed 2^31 - 1 nodes", (long long)B);
        pptr.assign((size_t)n2 + 1, 0);
        pidx.resize((size_t)std::max<i64>(m, 1));
        pz.assign((size_t)n2, 0.0);
        gzsum.assign((size_t)G, HostSum());
        for (i64 q = 0; q < G; ++q) {
            const i64 lo = gp[q], hi = gp[q + 1], ng = hi - lo;
            for (i64 u = 0; u < gstart[q + 1] - gstart[q]; ++u) pptr[gstart[q] + u] = ptr[lo + std::min(u, ng)];
            for (i64 e = ptr[lo]; e < ptr[hi]; ++e) {
                const int t = idx[e];
                if (t < lo || t >= hi) DI_FAIL(DI_EINVAL, "edge %lld leaves graph %lld (target %d)", (long long)e, (long long)q, t);
                pidx[e] = (int)(t - lo + gstart[q]);
            }
            for (i64 u = 0; u < ng; ++u) {
                const double z = Z ? Z[lo + u] : 1.0 / (double)ng;
                pz[gstart[q] + u] = z;
                gzsum[q].add(z);
            }
            if (!(gzsum[q].value() > 0.0)) DI_FAIL(DI_EINVAL, "Z sums to zero on graph %lld", (long long)q);
        }
        pptr[n2] = m;
        n = n2;
        ptr = pptr.data();
        idx = pidx.data();
        Z = pz.data();
    }

    di_ctx *c = new (std::nothrow) di_ctx();
    if (!c) DI_FAIL(DI_ENOMEM, "host allocation failed");
    c->o = opt;
    c->d = d;
    c->k = k;
    c->n_graphs = opt.n_graphs;
    c->n_user = n_user;
    if (opt.n_graphs > 1) {
        c->graph_ptr.assign(opt.graph_ptr, opt.graph_ptr + opt.n_graphs + 1);
        c->gstart = gstart;
    }
    c->st = (hipStream_t)opt.stream;
    c->p.d = d;
    c->p.theta = opt.theta;
    c->p.fp32 = opt.fluid_fp32 ? 1 : 0;
    c->p.normalized = opt.normalized_stop ? 1 : 0;
    c->p.n = n;
    c->g.n = n;
    c->g.m = m;
    c->g.weighted = w != nullptr;
    int rc = DI_OK;
    auto fail = [&](int code) {
        di_destroy(c);
        return code;
    };
    if ((rc = set_kernel_attributes()) != DI_OK) return fail(rc);
    if ((rc = noalloc_scratch(&c->scratch)) != DI_OK) return fail(rc);
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        set_error("hipEventCreate failed");
        return fail(DI_EHIP);
    }
    if (hipHostMalloc((void **)&c->h_ctl, sizeof(DevCtl), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return fail(DI_ENOMEM);
    }

    // upload OUT (for one graph with fast sweeps, in the numbering of cut-aligned ranges)
    const i64 B = (i64)1 << rb;
    std::vector<double> segz;
    if (k == 1 && opt.n_graphs == 1 && !opt.deterministic && opt.range_cut >= 0 && n > B) {
        const i64 X = std::min<i64>(opt.range_cut == 0 ? 1024 : opt.range_cut, B / 2);
        if ((rc = upload_segmented(c, ptr, idx, w, n, m, rb, X)) != DI_OK) return fail(rc);
        if (w && (rc = dalloc(c, &c->g.w, m))) return fail(rc);
        if (w && m && hipMemcpy(c->g.w, w, sizeof(float) * m, hipMemcpyDefault) != hipSuccess) {
            set_error("upload of the weights failed");
            return fail(DI_EHIP);
        }
        if (c->seg) {  // Z in the internal layout (padding nodes get none)
            n = c->g.n;
            std::vector<double> zu;
            if (!Z) zu.assign((size_t)n_user, 1.0 / (double)n_user);
            segz.assign((size_t)n, 0.0);
            seg_expand(c, Z ? Z : zu.data(), segz.data(), 0.0);
            Z = segz.data();
        }
    } else {
        if ((rc = dalloc(c, &c->g.out_ptr, n + 1)) || (rc = dalloc(c, &c->g.out_idx, m))) return fail(rc);
        if (w && (rc = dalloc(c, &c->g.w, m))) return fail(rc);
        if (hipMemcpy(c->g.out_ptr, ptr, sizeof(i64) * (n + 1), hipMemcpyDefault) != hipSuccess ||
            (m && hipMemcpy(c->g.out_idx, idx, sizeof(int) * m, hipMemcpyDefault) != hipSuccess) ||
            (w && m && hipMemcpy(c->g.w, w, sizeof(float) * m, hipMemcpyDefault) != hipSuccess)) {
            set_error("upload of the graph failed");
            return fail(DI_EHIP);
        }
    }

    c->rounds = opt.inner_rounds ? opt.inner_rounds : 4;
    c->p.rounds = c->rounds;
    c->spc = opt.sweeps_per_sync ? opt.sweeps_per_sync : 8;
    if ((rc = build_graph(c->g, c->g.out_ptr, c->g.out_idx, c->g.w, rb, k == 1, c->st)) != DI_OK) return fail(rc);
    c->p.dense_at = DENSE_DELIVERY * (double)c->g.m_rem;
    c->device_bytes += (2 * (n + 1) + 3 * n) * 8 + m * (4 + (w ? 4 : 0)) + c->g.m_loc * (2 + (w ? 4 : 0)) +
                       c->g.m_rem * (6 + (w ? 4 : 0)) + (c->g.nranges + 1) * 16;

    if ((rc = make_range_order(c, c->g, &c->s.range_order)) != DI_OK) return fail(rc);

    // cut-aligned ranges: the block-local sweeps skip the padding at the end of each range
    if (c->seg) {
        const i64 nr = c->g.nranges;
        std::vector<int> cntv((size_t)nr);
        for (i64 r = 0; r < nr; ++r) cntv[r] = (int)(c->seg_start[r + 1] - c->seg_start[r]);
        if ((rc = dalloc(c, &c->s.range_cnt, nr))) return fail(rc);
        if (hipMemcpy(c->s.range_cnt, cntv.data(), sizeof(int) * nr, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("range table upload failed");
            return fail(DI_EHIP);
        }
    }

    // per-workgroup partial sums (see PSR / PSC)
    {
        const i64 slots = std::max<i64>(c->g.nranges, PART_MIN);
        if ((rc = dalloc(c, &c->s.partR, slots * PSR)) || (rc = dalloc(c, &c->s.partC, slots * PSC)) ||
            (rc = dalloc(c, &c->s.partH, slots * PSR)) || (rc = dalloc(c, &c->s.hsum, 2 * std::max<i64>(opt.n_graphs, 1))))
            return fail(rc);
    }

    // initial fluid F_0 = (1-d) Z, rounded to float in the float-fluid mode; fixed-point scale
    if (k > 1) {
        if ((rc = init_batch(c->b, c->g, c->p, k, opt.deterministic ? 1 : 0, Z, c->s.range_order, c->rounds, c->st)) != DI_OK)
            return fail(rc);
        c->p.K = batch_K(c->b);
        *out = c;
        return DI_OK;
    }
    const size_t T = c->p.fp32 ? 4 : 8;
    std::vector<double> f0((size_t)n);
    double mx = 0.0;
    {
        HostSum zs;
        for (i64 i = 0; i < n; ++i) zs.add(Z ? Z[i] : 1.0 / (double)n);
        c->zsum = zs.value();
    }
    c->p.zsum = c->zsum;
    // F_0 is kept in double; the fluid starts from it rounded to the fluid type
    for (i64 i = 0; i < n; ++i) {
        const double z = Z ? Z[i] : 1.0 / (double)n;
        const double v = (1.0 - d) * z;
        f0[i] = v;
        mx = std::max(mx, std::fabs(c->p.fp32 ? (double)(float)v : v));
    }
    c->p.K = fixed_scale(mx, n);
    c->f0max = mx;
    // in-flight buffers: n values, then a bitmap of the nonzero ones (n/64 words)
    const i64 s_vals = ((i64)(n * T) + 255) & ~(i64)255;
    c->s.S_bytes = s_vals + ((n + 63) / 64) * 8;
    if ((rc = dalloc(c, (char **)&c->s.F, n * T)) || (rc = dalloc(c, &c->s.F0, n)) ||
        (rc = dalloc(c, &c->s.H, n)) || (rc = dalloc(c, (char **)&c->s.S[0], c->s.S_bytes)) ||
        (rc = dalloc(c, (char **)&c->s.S[1], c->s.S_bytes)) || (rc = dalloc(c, &c->s.ctl, 1)))
        return fail(rc);
    c->s.Sb[0] = reinterpret_cast<u64 *>(static_cast<char *>(c->s.S[0]) + s_vals);
    c->s.Sb[1] = reinterpret_cast<u64 *>(static_cast<char *>(c->s.S[1]) + s_vals);
    if (hipMemcpy(c->s.F0, f0.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(DI_EHIP);
    // power iteration reads Z (one graph only), or (1-d)/n for a uniform Z
    c->s.zc = (1.0 - d) * (1.0 / (double)n);
    if (Z && c->n_graphs == 1) {
        if ((rc = dalloc(c, &c->s.Z, n))) return fail(rc);
        if (hipMemcpy(c->s.Z, Z, n * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(DI_EHIP);
    }
    if (opt.deterministic) {
        if ((rc = dalloc(c, &c->s.snap, n)) || (rc = dalloc(c, &c->s.frontier, n))) return fail(rc);
    }
    if (c->n_graphs > 1) {  // per-range graph ids, per-graph constants and control blocks
        const i64 G = c->n_graphs, nr = c->g.nranges;
        c->h_range_graph.assign((size_t)nr, 0);
        c->h_ginfo.resize((size_t)G);
        for (i64 q = 0; q < G; ++q) {
            GraphInfo &gi = c->h_ginfo[q];
            gi.rbeg = c->gstart[q] >> rb;
            gi.rend = c->gstart[q + 1] >> rb;
            gi.n_d = (double)(c->graph_ptr[q + 1] - c->graph_ptr[q]);
            gi.zsum = gzsum[q].value();
            for (i64 r = gi.rbeg; r < gi.rend; ++r) c->h_range_graph[r] = (int)q;
        }
        std::vector<double> ones((size_t)G, 1.0);
        if ((rc = dalloc(c, &c->s.range_graph, nr)) || (rc = dalloc(c, &c->s.ginfo, G)) ||
            (rc = dalloc(c, &c->s.gctl, G)) || (rc = dalloc(c, &c->d_gp, G + 1)) || (rc = dalloc(c, &c->d_gs, G)) ||
            (rc = dalloc(c, &c->d_gscale, G)))
            return fail(rc);
        if (hipMemcpy(c->s.range_graph, c->h_range_graph.data(), sizeof(int) * nr, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->s.ginfo, c->h_ginfo.data(), sizeof(GraphInfo) * G, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->d_gp, c->graph_ptr.data(), sizeof(i64) * (G + 1), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->d_gs, c->gstart.data(), sizeof(i64) * G, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("upload of the graph table failed");
            return fail(DI_EHIP);
        }
        c->s.n_graphs = G;
        c->s.rb = rb;
    }
    // one graph: the IN row blocks of power iteration (and of the float fluid's
    // recomputation) are built here, so that di_power_noalloc needs no allocation
    if (c->n_graphs == 1 && (rc = ensure_row_blocks(c)) != DI_OK) return fail(rc);
    if ((rc = reset_state(c)) != DI_OK) return fail(rc);
    *out = c;
    return DI_OK;
}

int di_set_sweep(di_ctx *c, double theta, int inner_rounds) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!(theta >= 0.0) || !std::isfinite(theta)) DI_FAIL(DI_EINVAL, "theta must be finite and >= 0");
    if (inner_rounds < 0 || inner_rounds > 64) DI_FAIL(DI_EINVAL, "inner_rounds must be in 0..64");
    c->p.theta = theta;
    c->o.theta = theta;
    if (inner_rounds > 0) {
        c->rounds = inner_rounds;
        c->p.rounds = inner_rounds;
        c->o.inner_rounds = inner_rounds;
        if (c->b) set_batch_rounds(c->b, inner_rounds);
    }
    if (c->gexec) {  // captured chunks hold the old threshold scale and rounds
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    return DI_OK;
}

int di_reset(di_ctx *c) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    c->defects.clear();
    if (c->b) return reset_batch(c->b, c->g, c->p, c->st);
    return reset_state(c);
}

int di_set_z(di_ctx *c, const double *Z) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    const i64 nu = c->n_user, n = c->g.n;
    const int k = c->k;
    if (Z) {
        for (int col = 0; col < k; ++col) {
            double s = 0.0;
            for (i64 i = 0; i < nu; ++i) {
                const double v = Z[(i64)col * nu + i];
                if (!(v >= 0.0) || !std::isfinite(v)) DI_FAIL(DI_EINVAL, "Z[%lld, %d] must be finite and >= 0", (long long)i, col);
                s += v;
            }
            if (!(s > 0.0)) DI_FAIL(DI_EINVAL, "column %d of Z sums to zero", col);
        }
    }
    c->defects.clear();
    if (c->b) return set_batch_z(c->b, c->g, c->p, Z, c->st);
    // layout of the context (padded per graph in a union), F_0 = (1-d) Z in double
    std::vector<double> f0((size_t)n, 0.0);
    std::vector<HostSum> gz((size_t)c->n_graphs);
    if (c->n_graphs > 1) {
        for (i64 q = 0; q < c->n_graphs; ++q) {
            const i64 lo = c->graph_ptr[q], ng = c->graph_ptr[q + 1] - lo;
            for (i64 u = 0; u < ng; ++u) {
                const double z = Z ? Z[lo + u] : 1.0 / (double)ng;
                f0[c->gstart[q] + u] = z;
                gz[q].add(z);
            }
            if (!(gz[q].value() > 0.0)) DI_FAIL(DI_EINVAL, "Z sums to zero on graph %lld", (long long)q);
        }
    } else if (c->seg) {  // cut-aligned ranges: padding nodes get no Z
        std::vector<double> zu;
        if (!Z) zu.assign((size_t)nu, 1.0 / (double)nu);
        seg_expand(c, Z ? Z : zu.data(), f0.data(), 0.0);
    } else {
        for (i64 i = 0; i < n; ++i) f0[i] = Z ? Z[i] : 1.0 / (double)n;
    }
    std::vector<double> zint;  // Z in the internal layout, for power iteration
    if (c->seg) zint = f0;
    double mx = 0.0;
    HostSum zacc;
    for (i64 i = 0; i < n; ++i) {
        zacc.add(f0[i]);
        f0[i] = (1.0 - c->d) * f0[i];
        mx = std::max(mx, std::fabs(c->p.fp32 ? (double)(float)f0[i] : f0[i]));
    }
    if (c->n_graphs == 1) {  // power iteration reads Z
        if (Z || c->seg) {
            if (!c->s.Z) DI_TRY(dalloc(c, &c->s.Z, n));
            DI_HIP(hipMemcpy(c->s.Z, c->seg ? zint.data() : Z, sizeof(double) * n, hipMemcpyHostToDevice));
        } else if (c->s.Z) {
            (void)dev_free(c->s.Z);
            c->s.Z = nullptr;
        }
        c->s.zc = (1.0 - c->d) * (1.0 / (double)n);  // read when s.Z is null (uniform Z)
    } else {
        for (i64 q = 0; q < c->n_graphs; ++q) c->h_ginfo[q].zsum = gz[q].value();
        DI_HIP(hipMemcpy(c->s.ginfo, c->h_ginfo.data(), sizeof(GraphInfo) * c->n_graphs, hipMemcpyHostToDevice));
    }
    DI_HIP(hipMemcpy(c->s.F0, f0.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    c->zsum = zacc.value();
    c->p.zsum = c->zsum;
    c->p.K = fixed_scale(mx, n);
    c->f0max = mx;
    c->pi_done = false;
    if (c->gexec) {  // a captured chunk holds the old fixed-point scale
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    return reset_state(c);
}

static int diffuse_call(di_ctx *c, double tol, di_stats *st);
static int power_call(di_ctx *c, double tol, di_stats *st);
static int adjoint_call(di_ctx *c, const double *g, double tol_inf, double *dZ, double *dw, int on_device,
                        di_stats *st);

// the end record of DI_LOG for a finished call (stats from the call, or zeros)
static void log_end(di_ctx *c, const char *call, const di_stats &s, int rc) {
    // the single-column control block's sweep index (-1 for the k-column tile, which keeps its own)
    if (c && log_on()) log_record(c, c->n_user, call, "end", c->h_ctl && !c->b ? c->h_ctl->sweep : -1, s, &rc);
}

static void log_adjoint_sync(di_ctx *c, const DevCtl &h, const DevCtl &before) {
    if (!log_on()) return;
    di_stats ls{};
    ls.sweeps = h.sweep - before.sweep;
    ls.edge_updates = (int64_t)(h.tot_edges - before.tot_edges);
    ls.node_updates = (int64_t)(h.tot_nodes - before.tot_nodes);
    ls.residual = h.R;
    ls.bound = ls.bound_norm = h.maxF / (1.0 - c->d);
    log_record(c, c->n_user, "adjoint", "sync", h.sweep, ls, nullptr);
}

int di_diffuse(di_ctx *c, double tol, di_stats *st) {
    if (c) c->call_t0 = std::chrono::steady_clock::now();
    di_stats loc{};
    di_stats *sp = st ? st : &loc;
    const int rc = diffuse_call(c, tol, sp);
    log_end(c, "diffuse", *sp, rc);
    return rc;
}

int di_power(di_ctx *c, double tol, di_stats *st) {
    if (c) c->call_t0 = std::chrono::steady_clock::now();
    di_stats loc{};
    di_stats *sp = st ? st : &loc;
    const int rc = power_call(c, tol, sp);
    log_end(c, "power", *sp, rc);
    return rc;
}

int di_adjoint(di_ctx *c, const double *g, double tol_inf, double *dZ, double *dw, int on_device, di_stats *st) {
    if (c) c->call_t0 = std::chrono::steady_clock::now();
    di_stats loc{};
    di_stats *sp = st ? st : &loc;
    const int rc = adjoint_call(c, g, tol_inf, dZ, dw, on_device, sp);
    log_end(c, "adjoint", *sp, rc);
    return rc;
}

static int diffuse_call(di_ctx *c, double tol, di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) DI_FAIL(DI_EINVAL, "tol must be finite and > 0");
    c->p.tol = tol;
    if (c->b) {
        int rc = diffuse_batch(c->b, c->g, c->p, c->o, c->spc, c->st, st);
        if (rc == DI_OK || rc == DI_ENOCONV) {
            const std::string msg = di_last_error();
            DI_TRY(mass_defects(c, st));
            if (rc != DI_OK) set_error("%s", msg.c_str());
        }
        if (rc == DI_OK) c->forward_converged = true;
        return rc;
    }
    if (c->gexec && c->gexec_kind == 0) {  // tolerance is baked into a captured chunk
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    DI_HIP(hipEventRecord(c->ev0, c->st));
    const bool mg = c->s.range_graph != nullptr;
    if (mg) {
        // every call starts with no fluid in flight (the last one delivered it): clear the
        // in-flight buffers, then set each graph's state under the new tolerance
        const size_t T = c->p.fp32 ? 4 : 8;
        DI_TRY(launch_fill_zero(c->s.S[0], c->s.S_bytes, c->st));
        DI_TRY(launch_fill_zero(c->s.S[1], c->s.S_bytes, c->st));
        k_ctl_begin<<<1, 1, 0, c->st>>>(c->s.ctl, (long long)c->o.max_sweeps);
        DI_LAUNCH_CHECK();
        DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st, 0));
        DI_TRY(enqueue_finalize(c, FIN_INIT, c->st));
        DI_TRY(sync_ctl(c, c->s.ctl));
    } else {
        // recompute the residual of the current state under the new tolerance
        DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st));
        DI_TRY(enqueue_finalize(c, FIN_INIT, c->st));
        k_ctl_begin<<<1, 1, 0, c->st>>>(c->s.ctl, (long long)c->o.max_sweeps);
        DI_LAUNCH_CHECK();
        DI_TRY(sync_ctl(c, c->s.ctl));
    }
    // FIN_INIT already set done when the tolerance holds; k_ctl_begin cleared it: recheck
    DevCtl before = *c->h_ctl;
    if (mg && before.done && !before.overflow) {
        DI_HIP(hipEventRecord(c->ev1, c->st));
        DI_HIP(hipEventSynchronize(c->ev1));
        DI_TRY(fill_stats_mg(c, st, before, before, 0.0f));
        DI_TRY(mass_defects(c, st));
        c->forward_converged = true;
        return DI_OK;
    }
    if (!mg) {
        const double l = host_limbs(before.limbsL, c->p.K);
        const double b = c->p.normalized ? before.R / (1.0 - c->d - c->d * l / c->zsum) : before.R / (1.0 - c->d);
        if (b <= tol) {
            DI_HIP(hipEventRecord(c->ev1, c->st));
            DI_HIP(hipEventSynchronize(c->ev1));
            fill_stats(st, before, before, c->d, c->p.K, 0.0f, false, c->zsum);
            if (st) st->converged = 1;
            DI_TRY(mass_defects(c, st));
            c->forward_converged = true;
            return DI_OK;
        }
    }
    c->kernel_ns = 0.0;
    c->kernel_launches = 0;
    // Float fluid, block-local sweeps: the fluid is recomputed in double from H whenever
    // the residual has fallen by REFINE_DROP since the last recomputation, and before the
    // solve is declared converged, so that the stop rests on the exact residual.
    const bool refine = c->p.fp32 && !c->o.deterministic;
    double R_ref = before.R;
    bool in_flight = true;
    if (refine) c->p.tol = tol * REFINE_MARGIN;
    while (true) {
        const long long s0 = c->h_ctl->sweep;
        DI_TRY(enqueue_chunk(c, 0));
        DI_TRY(sync_ctl(c, c->s.ctl));
        in_flight = true;
        const DevCtl &h = *c->h_ctl;
        if (log_on()) {
            di_stats ls{};
            fill_stats(&ls, h, before, c->d, c->p.K, 0.0f, false, c->zsum);
            log_record(c, c->n_user, "diffuse", "sync", h.sweep, ls, nullptr);
        }
        if (c->o.timing && c->o.loop_mode == DI_LOOP_STREAM) DI_TRY(collect_timing(c, h.sweep - s0));
        if (h.overflow) break;
        if (refine && (h.done || h.R <= R_ref * REFINE_DROP)) {
            DI_TRY(refine_fluid(c, tol));
            in_flight = false;
            R_ref = c->h_ctl->R;
            if (c->h_ctl->done || c->h_ctl->overflow) break;
        } else if (h.done) {
            break;
        }
        if (c->h_ctl->sweep >= c->h_ctl->budget) break;
    }
    c->p.tol = tol;
    // deliver fluid still in flight so that F is complete (in a union of graphs, frozen
    // graphs have delivered theirs already)
    if (!c->o.deterministic && in_flight && !(mg && c->h_ctl->done)) {
        DI_TRY(launch_bld_sweep(c->g, c->s, c->p, 0, c->st));
        DI_TRY(enqueue_finalize(c, FIN_DELIVER, c->st));
    }
    DI_HIP(hipEventRecord(c->ev1, c->st));
    DI_TRY(sync_ctl(c, c->s.ctl));
    float ms = 0.0f;
    DI_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    const DevCtl &h = *c->h_ctl;
    if (mg) DI_TRY(fill_stats_mg(c, st, h, before, ms));
    else fill_stats(st, h, before, c->d, c->p.K, ms, false, c->zsum);
    if (h.overflow) DI_FAIL(DI_ENUMERIC, "non-finite or out-of-range fluid in the residual");
    DI_TRY(mass_defects(c, st));
    if (!h.done) {
        if (st) st->converged = 0;
        DI_FAIL(DI_ENOCONV, "sweep budget spent (%lld sweeps) before the tolerance", (long long)(h.sweep - before.sweep));
    }
    c->forward_converged = true;
    return DI_OK;
}

static int power_call(di_ctx *c, double tol, di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) DI_FAIL(DI_EINVAL, "tol must be finite and > 0");
    if (c->k != 1 || c->n_graphs != 1) DI_FAIL(DI_EINVAL, "di_power supports one right-hand side on one graph");
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    if (!c->pi_ready) {
        int rc = ensure_row_blocks(c);
        if (rc == DI_OK) rc = dalloc(c, &c->s.X[0], n);
        if (rc == DI_OK) rc = dalloc(c, &c->s.X[1], n);
        if (rc == DI_OK) rc = dalloc(c, (char **)&c->s.XT[0], n * T);
        if (rc == DI_OK) rc = dalloc(c, (char **)&c->s.XT[1], n * T);
        if (rc == DI_OK) rc = dalloc(c, &c->s.pctl, 1);
        if (rc != DI_OK) {
            free_group(&c->s.X[0], &c->s.X[1], &c->s.XT[0], &c->s.XT[1], &c->s.pctl);
            return rc;
        }
        c->pi_ready = true;
    }
    if (c->gexec && c->gexec_kind == 1) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    c->p.tol = tol;
    DI_TRY(launch_pi_init(c->g, c->s, c->p, c->st));
    DI_TRY(launch_fill_zero(c->s.pctl, sizeof(DevCtl), c->st));
    k_ctl_begin<<<1, 1, 0, c->st>>>(c->s.pctl, (long long)c->o.max_sweeps);
    DI_LAUNCH_CHECK();
    DI_TRY(sync_ctl(c, c->s.pctl));
    DevCtl before = *c->h_ctl;
    DI_HIP(hipEventRecord(c->ev0, c->st));
    c->kernel_ns = 0.0;
    c->kernel_launches = 0;
    while (true) {
        const long long s0 = c->h_ctl->sweep;
        DI_TRY(enqueue_chunk(c, 1));
        DI_TRY(sync_ctl(c, c->s.pctl));
        const DevCtl &h = *c->h_ctl;
        if (log_on()) {
            di_stats ls{};
            fill_stats(&ls, h, before, c->d, c->p.K, 0.0f, true);
            ls.edge_updates = (int64_t)((h.sweep - before.sweep) * c->g.m);
            ls.node_updates = (int64_t)((h.sweep - before.sweep) * n);
            log_record(c, c->n_user, "power", "sync", h.sweep, ls, nullptr);
        }
        if (c->o.timing && c->o.loop_mode == DI_LOOP_STREAM) DI_TRY(collect_timing(c, h.sweep - s0));
        if (h.done || h.overflow || h.sweep >= h.budget) break;
    }
    DI_HIP(hipEventRecord(c->ev1, c->st));
    DI_TRY(sync_ctl(c, c->s.pctl));
    float ms = 0.0f;
    DI_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    DevCtl h = *c->h_ctl;
    h.tot_edges = (u64)(h.sweep * c->g.m);
    h.tot_nodes = (u64)(h.sweep * n);
    fill_stats(st, h, before, c->d, c->p.K, ms, true);
    if (h.overflow) DI_FAIL(DI_ENUMERIC, "non-finite value in the power-iteration residual");
    c->pi_done = true;  // X_PI holds the last iterate (also after DI_ENOCONV)
    if (!h.done) DI_FAIL(DI_ENOCONV, "iteration budget spent before the tolerance");
    return DI_OK;
}

int di_power_noalloc(di_ctx *c, double tol, double *x_out, di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!x_out) DI_FAIL(DI_EINVAL, "x_out is NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) DI_FAIL(DI_EINVAL, "tol must be finite and > 0");
    if (c->k != 1 || c->n_graphs != 1) DI_FAIL(DI_EINVAL, "di_power_noalloc supports one right-hand side on one graph");
    if (!c->rbin_ready || !c->scratch) DI_FAIL(DI_ESTATE, "the context has no row blocks or scratch");
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bx = up((size_t)n * 8), bt = up((size_t)n * T), need = 2 * bx + 2 * bt + up(sizeof(DevCtl));
    if (need > (size_t)DI_NOALLOC_SCRATCH_BYTES)
        DI_FAIL(DI_EINVAL, "n = %lld (internal) needs %zu bytes of scratch, more than the %zu of di_power_noalloc",
                (long long)n, need, (size_t)DI_NOALLOC_SCRATCH_BYTES);
    // the context's state with the iterates, x/s vectors and control block in the scratch
    SolveState s = c->s;
    unsigned char *p = c->scratch;
    s.X[0] = reinterpret_cast<double *>(p);
    s.X[1] = reinterpret_cast<double *>(p + bx);
    s.XT[0] = p + 2 * bx;
    s.XT[1] = p + 2 * bx + bt;
    s.pctl = reinterpret_cast<DevCtl *>(p + 2 * bx + 2 * bt);
    c->p.tol = tol;
    // every buffer starts from zero (the scratch keeps the last call's contents); fill
    // kernels, no memset nodes
    DI_TRY(launch_pi_init(c->g, s, c->p, c->st));
    DI_TRY(launch_fill_zero(s.pctl, sizeof(DevCtl), c->st));
    k_ctl_begin<<<1, 1, 0, c->st>>>(s.pctl, (long long)c->o.max_sweeps);
    DI_LAUNCH_CHECK();
    DI_TRY(sync_ctl(c, s.pctl));
    const DevCtl before = *c->h_ctl;
    DI_HIP(hipEventRecord(c->ev0, c->st));
    while (true) {  // stream mode always (a captured graph would allocate)
        for (int k = 0; k < c->spc; ++k) DI_TRY(enqueue_pi_iteration_on(c, s, c->st));
        DI_TRY(sync_ctl(c, s.pctl));
        const DevCtl &h = *c->h_ctl;
        if (h.done || h.overflow || h.sweep >= h.budget) break;
    }
    const double *xr = s.X[c->h_ctl->parity];
    if (c->seg) {
        k_seg_to_caller<<<grid_for(n, 256, 16384), 256, 0, c->st>>>(xr, x_out, c->d_seg_start, c->seg_rb, n);
        DI_LAUNCH_CHECK();
    } else {
        DI_HIP(hipMemcpyAsync(x_out, xr, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    }
    DI_HIP(hipEventRecord(c->ev1, c->st));
    DI_TRY(sync_ctl(c, s.pctl));
    float ms = 0.0f;
    DI_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    DevCtl h = *c->h_ctl;
    h.tot_edges = (u64)(h.sweep * c->g.m);
    h.tot_nodes = (u64)(h.sweep * n);
    fill_stats(st, h, before, c->d, c->p.K, ms, true);
    if (h.overflow) DI_FAIL(DI_ENUMERIC, "non-finite value in the power-iteration residual");
    if (!h.done) DI_FAIL(DI_ENOCONV, "iteration budget spent before the tolerance");
    return DI_OK;
}

namespace {
int copy_small(const void *src, size_t bytes, void *dst, int on_device) {
    if (on_device) DI_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    else std::memcpy(dst, src, bytes);
    return DI_OK;
}

// di_read for a union of graphs: vectors come back in the caller's numbering.
// Reads of node-indexed values and of IN under cut-aligned ranges: the internal array is
// brought to the host and put back in the caller's numbering.  Returns 1 when `what` is
// not one of these (the caller reads it as usual).
int read_seg(di_ctx *c, int what, void *dst, int on_device, int *rc_out) {
    const i64 n = c->g.n, nu = c->n_user, m = c->g.m;
    auto put = [&](const void *src, size_t bytes) -> int {
        if (on_device) DI_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
        else std::memcpy(dst, src, bytes);
        return DI_OK;
    };
    auto doubles = [&](const double *dsrc, double scale) -> int {
        std::vector<double> v((size_t)n), out((size_t)nu);
        DI_HIP(hipMemcpy(v.data(), dsrc, sizeof(double) * n, hipMemcpyDeviceToHost));
        seg_compact(c, v.data(), out.data());
        if (scale != 1.0)
            for (double &x : out) x *= scale;
        return put(out.data(), sizeof(double) * nu);
    };
    switch (what) {
    case DI_X_RAW:
    case DI_H:
        *rc_out = doubles(c->s.H, 1.0);
        return 0;
    case DI_X_NORM: {
        DI_TRY(sync_ctl(c, c->s.ctl));
        const double l = host_limbs(c->h_ctl->limbsL, c->p.K);
        *rc_out = doubles(c->s.H, (1.0 - c->d) / (1.0 - c->d - c->d * l / c->zsum));
        return 0;
    }
    case DI_F: {
        if (!c->p.fp32) {
            *rc_out = doubles(static_cast<const double *>(c->s.F), 1.0);
            return 0;
        }
        std::vector<float> v((size_t)n);
        std::vector<double> out((size_t)nu);
        DI_HIP(hipMemcpy(v.data(), c->s.F, sizeof(float) * n, hipMemcpyDeviceToHost));
        std::vector<float> vc((size_t)nu);
        seg_compact(c, v.data(), vc.data());
        for (i64 i = 0; i < nu; ++i) out[i] = (double)vc[i];
        *rc_out = put(out.data(), sizeof(double) * nu);
        return 0;
    }
    case DI_LAMBDA:
        if (!c->lam) DI_FAIL(DI_ESTATE, "no adjoint has been computed");
        *rc_out = doubles(c->lam, 1.0);
        return 0;
    case DI_X_PI:
        if (!c->pi_done) DI_FAIL(DI_ESTATE, "di_power has not run for the current Z");
        DI_TRY(sync_ctl(c, c->s.pctl));
        *rc_out = doubles(c->s.X[c->h_ctl->parity], 1.0);
        return 0;
    case DI_INV_S:
        *rc_out = doubles(c->g.inv_s, 1.0);
        return 0;
    case DI_IN_PTR: {
        std::vector<i64> v((size_t)n + 1), out((size_t)nu + 1);
        DI_HIP(hipMemcpy(v.data(), c->g.in_ptr, sizeof(i64) * (n + 1), hipMemcpyDeviceToHost));
        seg_compact(c, v.data(), out.data());
        out[nu] = m;
        *rc_out = put(out.data(), sizeof(i64) * (nu + 1));
        return 0;
    }
    case DI_IN_IDX: {
        if (m == 0) {
            *rc_out = DI_OK;
            return 0;
        }
        std::vector<int> v((size_t)m);
        DI_HIP(hipMemcpy(v.data(), c->g.in_idx, sizeof(int) * m, hipMemcpyDeviceToHost));
        for (int &q : v) q = (int)seg_user(c, q);
        *rc_out = put(v.data(), sizeof(int) * m);
        return 0;
    }
    default:
        return 1;
    }
}

int read_union(di_ctx *c, int what, void *dst, int on_device) {
    const i64 G = c->n_graphs, nu = c->n_user;
    switch (what) {
    case DI_X_RAW:
    case DI_H:
    case DI_X_NORM:
    case DI_F: {
        const double *scale = nullptr;
        if (what == DI_X_NORM) {  // (1-d) / (1-d-d l_g/|Z_g|_1) on graph g (Section 3.3)
            DI_TRY(sync_gctl(c));
            std::vector<double> sc((size_t)G);
            for (i64 q = 0; q < G; ++q)
                sc[q] = (1.0 - c->d) / (1.0 - c->d - c->d * host_limbs(c->h_gctl[q].limbsL, c->p.K) / c->h_ginfo[q].zsum);
            DI_HIP(hipMemcpy(c->d_gscale, sc.data(), sizeof(double) * G, hipMemcpyHostToDevice));
            scale = c->d_gscale;
        }
        double *out = (double *)dst;
        if (!on_device) DI_HIP(dev_malloc((void **)&out, sizeof(double) * nu));
        const unsigned grid = grid_for(nu, 256, 16384);
        if (what == DI_F && c->p.fp32)
            k_unpad<float><<<grid, 256, 0, c->st>>>((const float *)c->s.F, nu, c->d_gp, c->d_gs, nullptr, G, out);
        else
            k_unpad<double><<<grid, 256, 0, c->st>>>(what == DI_F ? (const double *)c->s.F : c->s.H, nu, c->d_gp,
                                                     c->d_gs, scale, G, out);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && !on_device) e = hipMemcpyAsync(dst, out, sizeof(double) * nu, hipMemcpyDeviceToHost, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        if (!on_device) (void)dev_free(out);
        if (e != hipSuccess) DI_FAIL(DI_EHIP, "read failed: %s", hipGetErrorString(e));
        return DI_OK;
    }
    case DI_RESIDUALS:
    case DI_LEAKS:
    case DI_DONE_SWEEPS: {
        DI_TRY(sync_gctl(c));
        if (what == DI_DONE_SWEEPS) {
            std::vector<int64_t> v((size_t)G);
            for (i64 q = 0; q < G; ++q) v[q] = c->h_gctl[q].state == GS_FROZEN ? c->h_gctl[q].done_sweep : -1;
            return copy_small(v.data(), sizeof(int64_t) * G, dst, on_device);
        }
        std::vector<double> v((size_t)G);
        for (i64 q = 0; q < G; ++q)
            v[q] = what == DI_RESIDUALS ? c->h_gctl[q].R : host_limbs(c->h_gctl[q].limbsL, c->p.K);
        return copy_small(v.data(), sizeof(double) * G, dst, on_device);
    }
    case DI_FRONTIER: {
        if (!c->s.frontier) DI_FAIL(DI_ESTATE, "the frontier is recorded in deterministic mode only");
        DI_TRY(sync_ctl(c, c->s.ctl));
        const i64 cnt = (i64)c->h_ctl->fcount_last;
        std::vector<int> f((size_t)cnt + 2);
        if (cnt) DI_HIP(hipMemcpy(f.data() + 2, c->s.frontier, sizeof(int) * cnt, hipMemcpyDeviceToHost));
        for (i64 q = 0; q < cnt; ++q) {
            const i64 i2 = f[2 + q];
            const int g = c->h_range_graph[i2 >> c->s.rb];
            f[2 + q] = (int)(i2 - c->gstart[g] + c->graph_ptr[g]);
        }
        std::sort(f.begin() + 2, f.end());
        std::memcpy(f.data(), &cnt, sizeof(i64));
        return copy_small(f.data(), sizeof(int) * (cnt + 2), dst, on_device);
    }
    default:
        DI_FAIL(DI_EINVAL, "read target %d is not available for a union of graphs", what);
    }
}
}  // namespace

int di_read(di_ctx *c, int what, void *dst, int on_device) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!dst) DI_FAIL(DI_EINVAL, "dst is NULL");
    if (what == DI_MASS_DEFECTS) {
        if (c->defects.empty()) DI_FAIL(DI_ESTATE, "no di_diffuse has run since the last reset");
        return copy_small(c->defects.data(), sizeof(double) * c->defects.size(), dst, on_device);
    }
    if (c->b) return read_batch(c->b, c->g, c->p, what, dst, on_device, c->st);
    if (c->s.range_graph) return read_union(c, what, dst, on_device);
    if (c->seg) {
        int rc = DI_OK;
        const int h = read_seg(c, what, dst, on_device, &rc);
        if (h != 1) return h == 0 ? rc : h;  // handled, or an error
    }
    const i64 n = c->g.n, m = c->g.m;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    auto copy_out = [&](const void *src, size_t bytes) -> int {
        DI_HIP(hipMemcpyAsync(dst, src, bytes, kind, c->st));
        DI_HIP(hipStreamSynchronize(c->st));
        return DI_OK;
    };
    auto via_temp = [&](auto fill) -> int {  // produce doubles on the device, then copy
        double *tmp = nullptr;
        if (on_device) return fill((double *)dst);
        DI_HIP(dev_malloc((void **)&tmp, sizeof(double) * std::max<i64>(n, 1)));
        int rc = fill(tmp);
        if (rc == DI_OK) {
            hipError_t e = hipMemcpyAsync(dst, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, c->st);
            if (e == hipSuccess) e = hipStreamSynchronize(c->st);
            if (e != hipSuccess) {
                set_error("copy failed: %s", hipGetErrorString(e));
                rc = DI_EHIP;
            }
        }
        (void)dev_free(tmp);
        return rc;
    };
    switch (what) {
    case DI_X_RAW:
    case DI_H:
        return copy_out(c->s.H, sizeof(double) * n);
    case DI_X_NORM: {
        DI_TRY(sync_ctl(c, c->s.ctl));
        const double l = host_limbs(c->h_ctl->limbsL, c->p.K);
        const double scale = (1.0 - c->d) / (1.0 - c->d - c->d * l / c->zsum);
        return via_temp([&](double *t) { return launch_scaled_copy(c->s.H, scale, n, t, c->st); });
    }
    case DI_F:
        return via_temp([&](double *t) { return launch_copy_fluid_to_double(c->s.F, c->p.fp32, n, t, c->st); });
    case DI_LAMBDA:
        if (!c->lam) DI_FAIL(DI_ESTATE, "no adjoint has been computed");
        return copy_out(c->lam, sizeof(double) * n);
    case DI_X_PI: {
        if (!c->pi_done) DI_FAIL(DI_ESTATE, "di_power has not run for the current Z");
        DI_TRY(sync_ctl(c, c->s.pctl));
        return copy_out(c->s.X[c->h_ctl->parity], sizeof(double) * n);
    }
    case DI_IN_PTR:
        return copy_out(c->g.in_ptr, sizeof(i64) * (n + 1));
    case DI_IN_IDX:
        if (m == 0) return DI_OK;
        return copy_out(c->g.in_idx, sizeof(int) * m);
    case DI_INV_S:
        return copy_out(c->g.inv_s, sizeof(double) * n);
    case DI_FRONTIER: {
        if (!c->s.frontier) DI_FAIL(DI_ESTATE, "the frontier is recorded in deterministic mode only");
        DI_TRY(sync_ctl(c, c->s.ctl));
        const i64 cnt = (i64)c->h_ctl->fcount_last;
        std::vector<int> f((size_t)cnt + 2);
        if (cnt) DI_HIP(hipMemcpy(f.data() + 2, c->s.frontier, sizeof(int) * cnt, hipMemcpyDeviceToHost));
        std::sort(f.begin() + 2, f.end());
        std::memcpy(f.data(), &cnt, sizeof(i64));
        if (on_device) DI_HIP(hipMemcpy(dst, f.data(), sizeof(int) * (cnt + 2), hipMemcpyHostToDevice));
        else std::memcpy(dst, f.data(), sizeof(int) * (cnt + 2));
        return DI_OK;
    }
    case DI_RESIDUALS:
    case DI_LEAKS: {
        DI_TRY(sync_ctl(c, c->s.ctl));
        const double v = what == DI_RESIDUALS ? c->h_ctl->R : host_limbs(c->h_ctl->limbsL, c->p.K);
        return copy_small(&v, sizeof(double), dst, on_device);
    }
    case DI_DONE_SWEEPS: {
        DI_TRY(sync_ctl(c, c->s.ctl));
        const int64_t v = c->forward_converged ? (int64_t)c->h_ctl->sweep : -1;
        return copy_small(&v, sizeof(int64_t), dst, on_device);
    }
    default:
        DI_FAIL(DI_EINVAL, "unknown read target %d", what);
    }
}

static int adjoint_call(di_ctx *c, const double *g, double tol_inf, double *dZ, double *dw, int on_device,
                        di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!g || !dZ) DI_FAIL(DI_EINVAL, "g and dZ must not be NULL");
    if (!(tol_inf > 0.0) || !std::isfinite(tol_inf)) DI_FAIL(DI_EINVAL, "tol_inf must be finite and > 0");
    if (c->b || c->n_graphs > 1) DI_FAIL(DI_EINVAL, "the adjoint supports one right-hand side on one graph");
    if (!c->forward_converged) DI_FAIL(DI_ESTATE, "di_adjoint needs a converged di_diffuse first");
    const i64 n = c->g.n;
    if (!c->lam) {
        int rc = dalloc(c, &c->lam, n);
        if (rc == DI_OK) rc = dalloc(c, &c->aF, n);
        if (rc == DI_OK) rc = dalloc(c, &c->asnap, n);
        if (rc == DI_OK) rc = dalloc(c, &c->aZ, n);
        if (rc == DI_OK) rc = dalloc(c, &c->achk, 2);
        if (rc == DI_OK) rc = dalloc(c, &c->actl, 1);
        if (rc != DI_OK) {
            free_group(&c->lam, &c->aF, &c->asnap, &c->aZ, &c->achk, &c->actl);
            return rc;
        }
    }
    const i64 nu = c->n_user;  // the caller's node count (n is internal)
    // g checked on the device: a host g goes to the snapshot buffer (free until the sweeps
    // start) first; nothing the caller can read changes before the check has passed
    const double *gdev = g;
    if (!on_device) {
        DI_HIP(hipMemcpyAsync(c->asnap, g, sizeof(double) * nu, hipMemcpyHostToDevice, c->st));
        gdev = c->asnap;
    }
    double mx = 0.0;
    {
        DI_TRY(launch_fill_zero(c->achk, 16, c->st));
        k_check_rhs<<<grid_for(nu, 256, 512), 256, 0, c->st>>>(gdev, nu, c->achk);
        DI_LAUNCH_CHECK();
        u64 hv[2] = {0, 0};
        DI_HIP(hipMemcpyAsync(hv, c->achk, sizeof(hv), hipMemcpyDeviceToHost, c->st));
        DI_HIP(hipStreamSynchronize(c->st));
        if (hv[1]) DI_FAIL(DI_EINVAL, "g[%lld] is not finite", (long long)(nu - (i64)hv[1]));
        std::memcpy(&mx, &hv[0], sizeof(mx));
    }
    SweepParams ap = c->p;
    ap.K = fixed_scale(mx, n);
    ap.tol = tol_inf;
    if (c->seg) {  // internal layout (padding nodes get no g), spread on the device
        k_seg_to_internal<<<grid_for(n, 256, 16384), 256, 0, c->st>>>(gdev, c->aF, c->d_seg_start, c->seg_rb, n);
        DI_LAUNCH_CHECK();
    } else {
        DI_HIP(hipMemcpyAsync(c->aF, gdev, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    }
    DI_TRY(launch_fill_zero(c->lam, n * 8, c->st));
    DI_TRY(launch_fill_zero(c->actl, sizeof(DevCtl), c->st));
    DI_HIP(hipEventRecord(c->ev0, c->st));
    i64 anR = 0, anC = 0;
    DI_TRY(launch_reduce_double(c->aF, n, ap.K, c->actl, c->st, c->s.partR, &anR));
    k_ctl_begin<<<1, 1, 0, c->st>>>(c->actl, (long long)c->o.max_sweeps);
    DI_LAUNCH_CHECK();
    // sets done when g already meets the tolerance
    DI_TRY(launch_finalize(c->actl, ap, FIN_ADJ_INIT, c->st, c->s.partR, anR, c->s.partC, 0));
    DI_TRY(sync_ctl(c, c->actl));
    DevCtl before = *c->h_ctl;
    if (c->o.deterministic) {
        // snapshot and a row-order pull over OUT: reproducible, the oracle's order
        while (!c->h_ctl->done) {
            for (int k = 0; k < c->spc; ++k) {
                DI_TRY(launch_adj_sweep(c->g, c->aF, c->lam, c->asnap, c->actl, ap, c->st, c->s.partR, c->s.partC,
                                        &anR, &anC));
                DI_TRY(launch_finalize(c->actl, ap, FIN_ADJ, c->st, c->s.partR, anR, c->s.partC, anC));
            }
            DI_TRY(sync_ctl(c, c->actl));
            const DevCtl &h = *c->h_ctl;
            log_adjoint_sync(c, h, before);
            if (h.done || h.overflow || h.sweep >= h.budget) break;
        }
    } else {
        // block-local sweeps on the transposed graph (same ranges and numbering): a node
        // pushes its fluid along its IN row, local targets in LDS, the rest in flight to the
        // next sweep.  The stop needs max |F| with nothing in flight: when a sweep's
        // partials (max |F| as the sweep began, in-flight fluid delivered) meet the
        // tolerance, a delivery-only pass measures the state the call returns.
        if (!c->gT_ready) {
            free_graph(c->gT);  // a build never starts over arrays it would not free
            c->gT.n = n;
            c->gT.m = c->g.m;
            c->gT.weighted = c->g.weighted;
            const int brc = build_graph(c->gT, c->g.in_ptr, c->g.in_idx, c->g.in_w, c->g.rb, true, c->st);
            if (brc != DI_OK) {
                free_graph(c->gT);
                return brc;
            }
            c->gT_ready = true;
        }
        // in-flight buffers of double fluid (whatever the forward fluid type): n values,
        // then the bitmap of the nonzero ones
        const i64 s_vals = ((i64)(n * 8) + 255) & ~(i64)255;
        const i64 s_bytes = s_vals + ((n + 63) / 64) * 8;
        if (!c->aS[0]) {
            int rc = dalloc(c, (char **)&c->aS[0], s_bytes);
            if (rc == DI_OK) rc = dalloc(c, (char **)&c->aS[1], s_bytes);
            if (rc != DI_OK) {
                free_group(&c->aS[0], &c->aS[1]);
                return rc;
            }
        }
        SolveState as;
        as.F = c->aF;
        as.H = c->lam;
        as.S[0] = c->aS[0];
        as.S[1] = c->aS[1];
        as.Sb[0] = reinterpret_cast<u64 *>(static_cast<char *>(c->aS[0]) + s_vals);
        as.Sb[1] = reinterpret_cast<u64 *>(static_cast<char *>(c->aS[1]) + s_vals);
        as.S_bytes = s_bytes;
        as.ctl = c->actl;
        as.range_order = c->s.range_order;
        as.range_cnt = c->s.range_cnt;
        as.partR = c->s.partR;
        as.partC = c->s.partC;
        DI_TRY(launch_fill_zero(as.S[0], as.S_bytes, c->st));
        DI_TRY(launch_fill_zero(as.S[1], as.S_bytes, c->st));
        while (!c->h_ctl->done) {
            for (int k = 0; k < c->spc; ++k) {
                DI_TRY(launch_adj_bld_sweep(c->gT, c->g.inv_s, as, ap, c->rounds, c->st));
                DI_TRY(launch_finalize(c->actl, ap, FIN_ADJ, c->st, as.partR, as.nR, as.partC, as.nC));
            }
            DI_TRY(sync_ctl(c, c->actl));
            log_adjoint_sync(c, *c->h_ctl, before);
            if (c->h_ctl->overflow) break;
            if (c->h_ctl->done) {
                DI_TRY(launch_adj_bld_sweep(c->gT, c->g.inv_s, as, ap, 0, c->st));
                DI_TRY(launch_finalize(c->actl, ap, FIN_DELIVER, c->st, as.partR, as.nR, as.partC, as.nC));
                DI_TRY(sync_ctl(c, c->actl));
                if (c->h_ctl->maxF / (1.0 - c->d) <= tol_inf) break;
                k_ctl_reopen<<<1, 1, 0, c->st>>>(c->actl);  // not yet: more sweeps
                DI_LAUNCH_CHECK();
                DI_TRY(sync_ctl(c, c->actl));
            }
            if (c->h_ctl->sweep >= c->h_ctl->budget) break;
        }
    }
    // gradients from x = H (forward history) and lambda
    // (dZ goes through an internal-layout buffer for host outputs and cut-aligned ranges;
    // dw keeps the caller's edge order in every layout)
    double *ddZ = dZ, *ddw = dw;
    double *tZ = nullptr, *tw = nullptr;
    const bool zbuf = !on_device || c->seg, wbuf = !on_device && dw;
    if (zbuf) ddZ = tZ = c->aZ;
    if (wbuf) {
        if (dev_malloc((void **)&tw, sizeof(double) * std::max<i64>(c->g.m, 1)) != hipSuccess)
            DI_FAIL(DI_ENOMEM, "device allocation for the gradients failed");
        ddw = tw;
    }
    // fast contexts: the edge-parallel gradient with mu in the snapshot buffer (free once
    // the sweeps are done); deterministic ones: the oracle's row-order sums
    int rc = launch_edge_grad(c->g, c->s.H, c->lam, c->d, ddZ, ddw, c->o.deterministic ? nullptr : c->asnap, c->st);
    if (rc == DI_OK && c->seg) {  // dZ back to the caller's numbering (device dZ, or the snapshot buffer)
        double *zc = on_device ? dZ : c->asnap;
        k_seg_to_caller<<<grid_for(n, 256, 16384), 256, 0, c->st>>>(tZ, zc, c->d_seg_start, c->seg_rb, n);
        if (hipGetLastError() != hipSuccess) rc = DI_EHIP;
    }
    DI_HIP(hipEventRecord(c->ev1, c->st));
    std::vector<double> hz;
    if (rc == DI_OK && !on_device) {
        hz.resize((size_t)nu);
        if (hipMemcpyAsync(hz.data(), c->seg ? c->asnap : tZ, sizeof(double) * nu, hipMemcpyDeviceToHost, c->st) !=
            hipSuccess)
            rc = DI_EHIP;
    }
    if (rc == DI_OK && wbuf && c->g.m &&
        hipMemcpyAsync(dw, tw, sizeof(double) * c->g.m, hipMemcpyDeviceToHost, c->st) != hipSuccess)
        rc = DI_EHIP;
    if (hipStreamSynchronize(c->st) != hipSuccess) rc = DI_EHIP;
    if (tw) (void)dev_free(tw);
    if (rc != DI_OK) DI_FAIL(rc, "adjoint gradient step failed");
    if (!on_device) std::memcpy(dZ, hz.data(), sizeof(double) * nu);
    DI_TRY(sync_ctl(c, c->actl));
    float ms = 0.0f;
    DI_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    const DevCtl &h = *c->h_ctl;
    if (st) {
        st->sweeps = h.sweep - before.sweep;
        st->edge_updates = (int64_t)(h.tot_edges - before.tot_edges);
        st->node_updates = (int64_t)(h.tot_nodes - before.tot_nodes);
        st->residual = h.R;
        st->bound = h.maxF / (1.0 - c->d);
        st->bound_norm = st->bound;
        st->leak = 0.0;
        st->mass_defect = 0.0;
        st->ms = ms;
        st->converged = h.done && !h.overflow;
    }
    if (h.overflow) DI_FAIL(DI_ENUMERIC, "non-finite or out-of-range adjoint fluid");
    if (!h.done) DI_FAIL(DI_ENOCONV, "adjoint sweep budget spent before the tolerance");
    return DI_OK;
}

namespace {
struct CkptHeader {
    char magic[8];
    int64_t n, m, sweep;
    int32_t k, fp32, K, pad;
    u64 limbsL[4];
    u64 tot_nodes, tot_edges;
    double d;
};
}  // namespace

int di_update(di_ctx *c, const di_csr *g) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!g) DI_FAIL(DI_EINVAL, "graph is NULL");
    if (c->b || c->n_graphs > 1) DI_FAIL(DI_EINVAL, "di_update supports one right-hand side on one graph");
    if (g->n != c->n_user)
        DI_FAIL(DI_EINVAL, "the new graph must keep the %lld nodes (got n = %lld)", (long long)c->n_user, (long long)g->n);
    const i64 nu = c->n_user, n = c->g.n;
    const int ordered = c->o.deterministic ? 1 : 0;
    // device temporaries: H, F and P H of the current state in the caller's numbering, and
    // two internal-layout vectors (reused for the new graph's layout)
    double *tH = nullptr, *tF = nullptr, *tP = nullptr, *w0 = nullptr, *w1 = nullptr, *w2 = nullptr;
    di_ctx *c2 = nullptr;
    u64 *maxbits = nullptr;
    auto release = [&]() {
        for (void *q : {(void *)tH, (void *)tF, (void *)tP, (void *)w0, (void *)w1, (void *)w2, (void *)maxbits})
            if (q) (void)dev_free(q);
        if (c2) di_destroy(c2);
    };
    auto body = [&]() -> int {
        DI_HIP(dev_malloc((void **)&tH, sizeof(double) * nu));
        DI_HIP(dev_malloc((void **)&tF, sizeof(double) * nu));
        DI_HIP(dev_malloc((void **)&tP, sizeof(double) * nu));
        DI_HIP(dev_malloc((void **)&w0, sizeof(double) * n));
        DI_HIP(dev_malloc((void **)&w1, sizeof(double) * n));
        DI_HIP(dev_malloc((void **)&maxbits, sizeof(u64)));
        auto to_caller = [&](const double *src, double *dst) -> int {
            if (c->seg) {
                k_seg_to_caller<<<grid_for(n, 256, 16384), 256, 0, c->st>>>(src, dst, c->d_seg_start, c->seg_rb, n);
                DI_LAUNCH_CHECK();
            } else {
                DI_HIP(hipMemcpyAsync(dst, src, sizeof(double) * nu, hipMemcpyDeviceToDevice, c->st));
            }
            return DI_OK;
        };
        // P H on the current graph, then H, F, P H in the caller's numbering
        DI_TRY(launch_P_times(c->g, c->rbin, c->s.H, w0, w1, ordered, c->st));
        DI_TRY(to_caller(w1, tP));
        DI_TRY(to_caller(c->s.H, tH));
        DI_TRY(launch_copy_fluid_to_double(c->s.F, c->p.fp32, n, w0, c->st));
        DI_TRY(to_caller(w0, tF));
        // Z in the caller's numbering for the new context (NULL: uniform)
        std::vector<double> zc;
        if (c->s.Z) {
            std::vector<double> zi((size_t)n);
            DI_HIP(hipMemcpyAsync(zi.data(), c->s.Z, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
            DI_HIP(hipStreamSynchronize(c->st));
            zc.resize((size_t)nu);
            seg_compact(c, zi.data(), zc.data());
        }
        DI_HIP(hipStreamSynchronize(c->st));
        (void)dev_free(w0);
        (void)dev_free(w1);
        w0 = w1 = nullptr;
        // the new graph, with the same d, Z and options (its own layout and row blocks)
        di_opts o = c->o;
        o.k = 1;
        o.n_graphs = 1;
        o.graph_ptr = nullptr;
        DI_TRY(di_init(&c2, g, c->d, c->s.Z ? zc.data() : nullptr, &o));
        const i64 n2 = c2->g.n;
        DI_HIP(dev_malloc((void **)&w0, sizeof(double) * n2));
        DI_HIP(dev_malloc((void **)&w1, sizeof(double) * n2));
        DI_HIP(dev_malloc((void **)&w2, sizeof(double) * n2));
        auto from_caller = [&](const double *src, double *dst) -> int {
            if (c2->seg) {
                k_caller_to_seg<<<grid_for(n2, 256, 16384), 256, 0, c2->st>>>(src, dst, c2->d_seg_start, c2->seg_rb, n2);
                DI_LAUNCH_CHECK();
            } else {
                DI_HIP(hipMemcpyAsync(dst, src, sizeof(double) * nu, hipMemcpyDeviceToDevice, c2->st));
            }
            return DI_OK;
        };
        // Theorem 4: H' = H, F' = F + d (P' - P) H, evaluated as P'H - PH
        DI_TRY(from_caller(tH, c2->s.H));
        DI_TRY(launch_P_times(c2->g, c2->rbin, c2->s.H, w2, w1, ordered, c2->st));  // w1 = P'H
        DI_TRY(from_caller(tF, w0));
        DI_TRY(from_caller(tP, w2));  // w2 = P H
        DI_TRY(launch_fill_zero(maxbits, sizeof(u64), c2->st));
        if (c2->p.fp32)
            k_update_fluid<float><<<grid_for(n2, 256, 16384), 256, 0, c2->st>>>(w0, w1, w2, c2->d, n2,
                                                                               (float *)c2->s.F, maxbits);
        else
            k_update_fluid<double><<<grid_for(n2, 256, 16384), 256, 0, c2->st>>>(w0, w1, w2, c2->d, n2,
                                                                                (double *)c2->s.F, maxbits);
        DI_LAUNCH_CHECK();
        u64 mb = 0;
        DI_HIP(hipMemcpyAsync(&mb, maxbits, sizeof(u64), hipMemcpyDeviceToHost, c2->st));
        DI_HIP(hipStreamSynchronize(c2->st));
        double mxf = 0.0;
        std::memcpy(&mxf, &mb, sizeof(double));
        // the fixed-point scale covers the new fluid and the starting fluid (which bounds the
        // leak); the leak restarts as the history at the nodes dangling in P' (the fluid
        // those diffusions lose under P', Section 3.3)
        c2->p.K = fixed_scale(std::max(c2->f0max, mxf), n2);
        DI_TRY(launch_fill_zero(c2->s.S[0], c2->s.S_bytes, c2->st));
        DI_TRY(launch_fill_zero(c2->s.S[1], c2->s.S_bytes, c2->st));
        DI_TRY(launch_fill_zero(c2->s.ctl, sizeof(DevCtl), c2->st));
        const unsigned gl = grid_for(n2, 256, REDUCE_GRID);
        k_dangling_history<<<gl, 256, 0, c2->st>>>(c2->s.H, c2->g.inv_s, n2, c2->p.K, c2->s.partH);
        DI_LAUNCH_CHECK();
        k_set_leak<<<1, 256, 0, c2->st>>>(c2->s.ctl, c2->s.partH, gl);
        DI_LAUNCH_CHECK();
        DI_TRY(launch_reduce_F(c2->g, c2->s, c2->p, c2->st));
        DI_TRY(enqueue_finalize(c2, FIN_INIT, c2->st));
        DI_TRY(sync_ctl(c2, c2->s.ctl));
        if (c2->h_ctl->overflow) DI_FAIL(DI_ENUMERIC, "non-finite fluid after the update");
        // the context takes the new graph and state; the old ones are released with c2
        std::swap(*c, *c2);
        c->forward_converged = false;
        c->defects.clear();
        return DI_OK;
    };
    const int rc = body();
    release();
    return rc;
}

int di_save(di_ctx *c, const char *path) {
    if (!c || !path) DI_FAIL(DI_EINVAL, "NULL argument");
    if (c->b || c->n_graphs > 1) DI_FAIL(DI_EINVAL, "checkpoints cover single right-hand-side solves on one graph");
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    DI_TRY(sync_ctl(c, c->s.ctl));
    CkptHeader h{};
    std::memcpy(h.magic, "DICKPT01", 8);
    h.n = n;
    h.m = c->g.m;
    h.sweep = c->h_ctl->sweep;
    h.k = c->k;
    h.fp32 = c->p.fp32;
    h.K = c->p.K;
    for (int q = 0; q < 4; ++q) h.limbsL[q] = c->h_ctl->limbsL[q];
    h.tot_nodes = c->h_ctl->tot_nodes;
    h.tot_edges = c->h_ctl->tot_edges;
    h.d = c->d;
    std::vector<double> H((size_t)n);
    std::vector<char> F((size_t)n * T);
    DI_HIP(hipMemcpy(H.data(), c->s.H, sizeof(double) * n, hipMemcpyDeviceToHost));
    DI_HIP(hipMemcpy(F.data(), c->s.F, T * n, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) DI_FAIL(DI_EINVAL, "cannot open %s for writing", path);
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(H.data(), sizeof(double), n, f) == (size_t)n &&
              std::fwrite(F.data(), T, n, f) == (size_t)n;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) DI_FAIL(DI_EINVAL, "write to %s failed", path);
    return DI_OK;
}

__global__ void k_ctl_restore(DevCtl *c, long long sweep, u64 l0, u64 l1, u64 l2, u64 l3, u64 tn, u64 te) {
    c->sweep = sweep;
    c->limbsL[0] = l0;
    c->limbsL[1] = l1;
    c->limbsL[2] = l2;
    c->limbsL[3] = l3;
    c->tot_nodes = tn;
    c->tot_edges = te;
    c->parity = 0;
}

int di_load(di_ctx *c, const char *path) {
    if (c) c->defects.clear();
    if (!c || !path) DI_FAIL(DI_EINVAL, "NULL argument");
    if (c->b || c->n_graphs > 1) DI_FAIL(DI_EINVAL, "checkpoints cover single right-hand-side solves on one graph");
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    FILE *f = std::fopen(path, "rb");
    if (!f) DI_FAIL(DI_EINVAL, "cannot open %s", path);
    CkptHeader h{};
    std::vector<double> H((size_t)n);
    std::vector<char> F((size_t)n * T);
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, "DICKPT01", 8) == 0 && h.n == n &&
              h.m == c->g.m && h.k == c->k && h.fp32 == c->p.fp32 && h.K == c->p.K && h.d == c->d;
    ok = ok && std::fread(H.data(), sizeof(double), n, f) == (size_t)n && std::fread(F.data(), T, n, f) == (size_t)n;
    std::fclose(f);
    if (!ok) DI_FAIL(DI_EINVAL, "%s is not a checkpoint of this graph, d and precision", path);
    DI_HIP(hipMemcpy(c->s.H, H.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    DI_HIP(hipMemcpy(c->s.F, F.data(), T * n, hipMemcpyHostToDevice));
    DI_TRY(launch_fill_zero(c->s.S[0], c->s.S_bytes, c->st));
    DI_TRY(launch_fill_zero(c->s.S[1], c->s.S_bytes, c->st));
    DI_TRY(launch_fill_zero(c->s.ctl, sizeof(DevCtl), c->st));
    k_ctl_restore<<<1, 1, 0, c->st>>>(c->s.ctl, (long long)h.sweep, h.limbsL[0], h.limbsL[1], h.limbsL[2],
                                      h.limbsL[3], h.tot_nodes, h.tot_edges);
    DI_LAUNCH_CHECK();
    DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st));
    DI_TRY(launch_finalize(c->s.ctl, c->p, FIN_INIT, c->st, c->s.partR, c->s.nR, c->s.partC, 0));
    DI_HIP(hipStreamSynchronize(c->st));
    c->forward_converged = false;
    return DI_OK;
}

int di_info(di_ctx *c, int key, int64_t *value) {
    if (!value) DI_FAIL(DI_EINVAL, "NULL argument");
    if (key == DI_INFO_LIVE_ALLOCATIONS) {  // process-wide: ctx may be NULL
        *value = dev_live_allocations();
        return DI_OK;
    }
    if (!c) DI_FAIL(DI_EINVAL, "NULL argument");
    switch (key) {
    case DI_INFO_N: *value = c->n_user; return DI_OK;
    case DI_INFO_N_INTERNAL: *value = c->g.n; return DI_OK;
    case DI_INFO_M: *value = c->g.m; return DI_OK;
    case DI_INFO_K: *value = c->k; return DI_OK;
    case DI_INFO_M_LOCAL: *value = c->g.m_loc; return DI_OK;
    case DI_INFO_RANGE_LOG2: *value = c->g.rb; return DI_OK;
    case DI_INFO_INNER_ROUNDS: *value = c->rounds; return DI_OK;
    case DI_INFO_FIXED_K: *value = c->p.K; return DI_OK;
    case DI_INFO_TOTAL_SWEEPS: {
        if (c->b) { *value = batch_sweeps(c->b, c->st); return DI_OK; }
        DI_TRY(sync_ctl(c, c->s.ctl));
        *value = c->h_ctl->sweep;
        return DI_OK;
    }
    case DI_INFO_DEVICE_BYTES: *value = c->device_bytes; return DI_OK;
    case DI_INFO_KERNEL_NS: *value = (int64_t)c->kernel_ns; return DI_OK;
    case DI_INFO_KERNEL_LAUNCHES: *value = c->kernel_launches; return DI_OK;
    case DI_INFO_LOCAL_PUSHES:
    case DI_INFO_REMOTE_UPDATES: {
        if (c->b) DI_FAIL(DI_EINVAL, "counters of batched solves are not kept");
        DI_TRY(sync_ctl(c, c->s.ctl));
        const DevCtl &h = *c->h_ctl;
        *value = key == DI_INFO_REMOTE_UPDATES ? (int64_t)h.tot_remote
                                               : (c->o.deterministic ? (int64_t)h.tot_edges
                                                                     : (int64_t)(h.tot_edges - h.tot_remote));
        return DI_OK;
    }
    case DI_INFO_M_REMOTE: *value = c->g.m_rem; return DI_OK;
    case DI_INFO_NRANGES: *value = c->g.nranges; return DI_OK;
    default: DI_FAIL(DI_EINVAL, "unknown info key %d", key);
    }
}

}  // extern "C"
