// C ABI of the library: validation, context management and the host-side sweep loop.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <numeric>

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

}  // namespace di

using namespace di;

struct di_ctx {
    DevGraph g;
    RowBlocks rbin;  // row blocks of IN (power iteration)
    SolveState s;
    SweepParams p;
    di_opts o{};
    hipStream_t st = nullptr;
    double d = 0.85;
    int k = 1;
    i64 n_graphs = 1;
    std::vector<i64> graph_ptr;
    int rounds = 8;
    int spc = 8;  // sweeps per host check
    double zsum = 1.0;  // sum of Z (single right-hand side)
    bool forward_converged = false;
    bool pi_ready = false;
    DevCtl *h_ctl = nullptr;  // pinned mirror of the control block
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    i64 device_bytes = 0;
    // adjoint
    double *lam = nullptr;
    double *aF = nullptr;
    double *asnap = nullptr;
    DevCtl *actl = nullptr;
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
};

namespace {

template <typename T>
int dalloc(di_ctx *c, T **p, i64 count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    DI_HIP(hipMalloc((void **)p, (size_t)count * sizeof(T)));
    c->device_bytes += count * (i64)sizeof(T);
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

double host_limbs(const u64 *l, int K) { return limbs_to_double_raw(l[0], l[1], l[2], l[3], K); }

__global__ void k_ctl_begin(DevCtl *c, long long max_sweeps) {
    c->done = 0;
    c->overflow = 0;
    c->budget = c->sweep + max_sweeps;
}

int reset_state(di_ctx *c) {
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    DI_HIP(hipMemcpyAsync(c->s.F, c->s.F0, n * T, hipMemcpyDeviceToDevice, c->st));
    DI_TRY(launch_fill_zero(c->s.H, n * 8, c->st));
    DI_TRY(launch_fill_zero(c->s.S[0], n * T, c->st));
    DI_TRY(launch_fill_zero(c->s.S[1], n * T, c->st));
    DI_TRY(launch_fill_zero(c->s.ctl, sizeof(DevCtl), c->st));
    DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st));
    DI_TRY(launch_finalize(c->s.ctl, c->p, FIN_INIT, c->st, c->s.partR, c->s.nR, c->s.partC, 0));
    DI_HIP(hipStreamSynchronize(c->st));
    c->forward_converged = false;
    return DI_OK;
}

int enqueue_di_sweep(di_ctx *c, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (e0) DI_HIP(hipEventRecord(e0, st));
    if (c->o.deterministic) DI_TRY(launch_det_sweep(c->g, c->s, c->p, st));
    else DI_TRY(launch_bld_sweep(c->g, c->s, c->p, c->rounds, st));
    if (e1) DI_HIP(hipEventRecord(e1, st));
    return launch_finalize(c->s.ctl, c->p, FIN_DI, st, c->s.partR, c->s.nR, c->s.partC, c->s.nC);
}

int enqueue_pi_iteration(di_ctx *c, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (e0) DI_HIP(hipEventRecord(e0, st));
    DI_TRY(launch_pi_iteration(c->g, c->rbin, c->s, c->p, st));
    if (e1) DI_HIP(hipEventRecord(e1, st));
    return launch_finalize(c->s.pctl, c->p, FIN_PI, st, c->s.partR, c->s.nR, c->s.partC, 0);
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
    st->converged = h.done && !h.overflow;
}

}  // namespace

extern "C" {

const char *di_last_error(void) { return g_err; }

int di_destroy(di_ctx *c) {
    if (!c) return DI_OK;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    free_graph(c->g);
    free_row_blocks(c->rbin);
    void *ps[] = {c->s.F, c->s.F0, c->s.H, c->s.S[0], c->s.S[1], c->s.snap, c->s.frontier, c->s.range_order,
                  c->s.ctl, c->s.X[0], c->s.X[1], c->s.XT[0], c->s.XT[1], c->s.pctl, c->s.Z, c->lam,
                  c->aF, c->asnap, c->actl, c->s.partR, c->s.partC};
    for (void *p : ps)
        if (p) (void)hipFree(p);
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
    if (opt.range_log2 != 0 && (opt.range_log2 < 8 || opt.range_log2 > (opt.fluid_fp32 ? 14 : 13)))
        DI_FAIL(DI_EINVAL, "range_log2 must be 0 or in 8..%d", opt.fluid_fp32 ? 14 : 13);
    if (opt.inner_rounds < 0 || opt.inner_rounds > 64) DI_FAIL(DI_EINVAL, "inner_rounds must be in 0..64");
    if (opt.loop_mode != DI_LOOP_STREAM && opt.loop_mode != DI_LOOP_GRAPH) DI_FAIL(DI_EINVAL, "bad loop_mode");
    if (opt.sweeps_per_sync < 0) DI_FAIL(DI_EINVAL, "sweeps_per_sync must be >= 0");
    const i64 n = g->n, m = g->m;
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
    if (g->on_device) {
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
    DI_TRY(validate_host_csr(&hv, &sorted));
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

    di_ctx *c = new (std::nothrow) di_ctx();
    if (!c) DI_FAIL(DI_ENOMEM, "host allocation failed");
    c->o = opt;
    c->d = d;
    c->k = k;
    c->n_graphs = opt.n_graphs;
    if (opt.n_graphs > 1) c->graph_ptr.assign(opt.graph_ptr, opt.graph_ptr + opt.n_graphs + 1);
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
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        set_error("hipEventCreate failed");
        return fail(DI_EHIP);
    }
    if (hipHostMalloc((void **)&c->h_ctl, sizeof(DevCtl), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return fail(DI_ENOMEM);
    }

    // upload OUT
    if ((rc = dalloc(c, &c->g.out_ptr, n + 1)) || (rc = dalloc(c, &c->g.out_idx, m))) return fail(rc);
    if (w && (rc = dalloc(c, &c->g.w, m))) return fail(rc);
    if (hipMemcpy(c->g.out_ptr, ptr, sizeof(i64) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        (m && hipMemcpy(c->g.out_idx, idx, sizeof(int) * m, hipMemcpyHostToDevice) != hipSuccess) ||
        (w && m && hipMemcpy(c->g.w, w, sizeof(float) * m, hipMemcpyHostToDevice) != hipSuccess)) {
        set_error("upload of the graph failed");
        return fail(DI_EHIP);
    }

    // block-local range size: unweighted graphs use the LDS-resident kernel with 2^11-node
    // ranges; weighted graphs the largest range whose fluid fits in LDS; small graphs keep
    // at least ~256 nodes per range so that several workgroups run
    int rbmax = c->p.fp32 ? 14 : 13;
    int rb = opt.range_log2;
    if (rb == 0) {
        const int cap = w ? rbmax : 11;
        rb = 8;
        while (rb < cap && ((i64)1 << (rb + 1)) * 256 <= n) ++rb;
    }
    c->rounds = opt.inner_rounds ? opt.inner_rounds : 4;
    c->p.rounds = c->rounds;
    c->spc = opt.sweeps_per_sync ? opt.sweeps_per_sync : 8;
    if ((rc = build_graph(c->g, c->g.out_ptr, c->g.out_idx, c->g.w, rb, c->st)) != DI_OK) return fail(rc);
    c->device_bytes += (2 * (n + 1) + 3 * n) * 8 + m * (4 + (w ? 4 : 0)) + c->g.m_loc * (2 + (w ? 4 : 0)) +
                       c->g.m_rem * (6 + (w ? 4 : 0)) + (c->g.nranges + 1) * 16;

    // range order: most work first
    {
        const i64 nr = c->g.nranges;
        std::vector<i64> rbase(nr + 1), lbase(nr + 1);
        if (hipMemcpy(rbase.data(), c->g.rem_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(lbase.data(), c->g.loc_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error("range table download failed");
            return fail(DI_EHIP);
        }
        std::vector<int> order(nr);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (rbase[a + 1] - rbase[a]) + (lbase[a + 1] - lbase[a]) >
                   (rbase[b + 1] - rbase[b]) + (lbase[b + 1] - lbase[b]);
        });
        if ((rc = dalloc(c, &c->s.range_order, nr))) return fail(rc);
        if (hipMemcpy(c->s.range_order, order.data(), sizeof(int) * nr, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("range order upload failed");
            return fail(DI_EHIP);
        }
    }

    // per-workgroup partial sums (see PSR / PSC)
    {
        const i64 slots = std::max<i64>(c->g.nranges, PART_MIN);
        if ((rc = dalloc(c, &c->s.partR, slots * PSR)) || (rc = dalloc(c, &c->s.partC, slots * PSC))) return fail(rc);
    }

    // initial fluid F_0 = (1-d) Z, rounded to float in the float-fluid mode; fixed-point scale
    if (k > 1 || c->n_graphs > 1) {
        if ((rc = init_batch(c->b, c->g, c->p, k, c->graph_ptr, Z, c->st)) != DI_OK) return fail(rc);
        c->p.K = batch_K(c->b);
        *out = c;
        return DI_OK;
    }
    const size_t T = c->p.fp32 ? 4 : 8;
    std::vector<double> f0((size_t)n);
    double mx = 0.0;
    c->zsum = 0.0;
    for (i64 i = 0; i < n; ++i) c->zsum += Z ? Z[i] : 1.0 / (double)n;
    c->p.zsum = c->zsum;
    for (i64 i = 0; i < n; ++i) {
        const double z = Z ? Z[i] : 1.0 / (double)n;
        double v = (1.0 - d) * z;
        if (c->p.fp32) v = (double)(float)v;
        f0[i] = v;
        mx = std::max(mx, std::fabs(v));
    }
    c->p.K = fixed_scale(mx, n);
    if ((rc = dalloc(c, (char **)&c->s.F, n * T)) || (rc = dalloc(c, (char **)&c->s.F0, n * T)) ||
        (rc = dalloc(c, &c->s.H, n)) || (rc = dalloc(c, (char **)&c->s.S[0], n * T)) ||
        (rc = dalloc(c, (char **)&c->s.S[1], n * T)) || (rc = dalloc(c, &c->s.ctl, 1)))
        return fail(rc);
    if (c->p.fp32) {
        std::vector<float> f0f(f0.begin(), f0.end());
        if (hipMemcpy(c->s.F0, f0f.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess) return fail(DI_EHIP);
    } else {
        if (hipMemcpy(c->s.F0, f0.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(DI_EHIP);
    }
    if (Z) {
        if ((rc = dalloc(c, &c->s.Z, n))) return fail(rc);
        if (hipMemcpy(c->s.Z, Z, n * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(DI_EHIP);
    } else {
        c->s.zc = (1.0 - d) * (1.0 / (double)n);
    }
    if (opt.deterministic) {
        if ((rc = dalloc(c, &c->s.snap, n)) || (rc = dalloc(c, &c->s.frontier, n))) return fail(rc);
    }
    if ((rc = reset_state(c)) != DI_OK) return fail(rc);
    *out = c;
    return DI_OK;
}

int di_reset(di_ctx *c) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (c->b) return reset_batch(c->b, c->g, c->p, c->st);
    return reset_state(c);
}

int di_diffuse(di_ctx *c, double tol, di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) DI_FAIL(DI_EINVAL, "tol must be finite and > 0");
    c->p.tol = tol;
    if (c->b) {
        int rc = diffuse_batch(c->b, c->g, c->p, c->o, c->rounds, c->spc, c->st, st);
        return rc;
    }
    if (c->gexec && c->gexec_kind == 0) {  // tolerance is baked into a captured chunk
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    DI_HIP(hipEventRecord(c->ev0, c->st));
    // recompute the residual of the current state under the new tolerance
    DI_TRY(launch_reduce_F(c->g, c->s, c->p, c->st));
    DI_TRY(launch_finalize(c->s.ctl, c->p, FIN_INIT, c->st, c->s.partR, c->s.nR, c->s.partC, 0));
    k_ctl_begin<<<1, 1, 0, c->st>>>(c->s.ctl, (long long)c->o.max_sweeps);
    DI_LAUNCH_CHECK();
    DI_TRY(sync_ctl(c, c->s.ctl));
    // FIN_INIT already set done when the tolerance holds; k_ctl_begin cleared it: recheck
    DevCtl before = *c->h_ctl;
    {
        const double l = host_limbs(before.limbsL, c->p.K);
        const double b = c->p.normalized ? before.R / (1.0 - c->d - c->d * l / c->zsum) : before.R / (1.0 - c->d);
        if (b <= tol) {
            DI_HIP(hipEventRecord(c->ev1, c->st));
            DI_HIP(hipEventSynchronize(c->ev1));
            fill_stats(st, before, before, c->d, c->p.K, 0.0f, false, c->zsum);
            if (st) st->converged = 1;
            c->forward_converged = true;
            return DI_OK;
        }
    }
    c->kernel_ns = 0.0;
    c->kernel_launches = 0;
    while (true) {
        const long long s0 = c->h_ctl->sweep;
        DI_TRY(enqueue_chunk(c, 0));
        DI_TRY(sync_ctl(c, c->s.ctl));
        const DevCtl &h = *c->h_ctl;
        if (c->o.timing && c->o.loop_mode == DI_LOOP_STREAM) DI_TRY(collect_timing(c, h.sweep - s0));
        if (h.done || h.overflow || h.sweep >= h.budget) break;
    }
    if (!c->o.deterministic) {  // deliver fluid still in flight so that F is complete
        DI_TRY(launch_bld_sweep(c->g, c->s, c->p, 0, c->st));
        DI_TRY(launch_finalize(c->s.ctl, c->p, FIN_DELIVER, c->st, c->s.partR, c->s.nR, c->s.partC, c->s.nC));
    }
    DI_HIP(hipEventRecord(c->ev1, c->st));
    DI_TRY(sync_ctl(c, c->s.ctl));
    float ms = 0.0f;
    DI_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    const DevCtl &h = *c->h_ctl;
    fill_stats(st, h, before, c->d, c->p.K, ms, false, c->zsum);
    if (h.overflow) DI_FAIL(DI_ENUMERIC, "non-finite or out-of-range fluid in the residual");
    if (!h.done) {
        if (st) st->converged = 0;
        DI_FAIL(DI_ENOCONV, "sweep budget spent (%lld sweeps) before the tolerance", (long long)(h.sweep - before.sweep));
    }
    c->forward_converged = true;
    return DI_OK;
}

int di_power(di_ctx *c, double tol, di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) DI_FAIL(DI_EINVAL, "tol must be finite and > 0");
    if (c->k != 1 || c->n_graphs != 1) DI_FAIL(DI_EINVAL, "di_power supports one right-hand side on one graph");
    const i64 n = c->g.n;
    const size_t T = c->p.fp32 ? 4 : 8;
    if (!c->pi_ready) {
        DI_TRY(build_row_blocks(c->rbin, c->g.in_ptr, n, c->st));
        DI_TRY(dalloc(c, &c->s.X[0], n));
        DI_TRY(dalloc(c, &c->s.X[1], n));
        DI_TRY(dalloc(c, (char **)&c->s.XT[0], n * T));
        DI_TRY(dalloc(c, (char **)&c->s.XT[1], n * T));
        DI_TRY(dalloc(c, &c->s.pctl, 1));
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
    if (!h.done) DI_FAIL(DI_ENOCONV, "iteration budget spent before the tolerance");
    return DI_OK;
}

int di_read(di_ctx *c, int what, void *dst, int on_device) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!dst) DI_FAIL(DI_EINVAL, "dst is NULL");
    if (c->b) return read_batch(c->b, c->g, c->p, what, dst, on_device, c->st);
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
        DI_HIP(hipMalloc((void **)&tmp, sizeof(double) * std::max<i64>(n, 1)));
        int rc = fill(tmp);
        if (rc == DI_OK) {
            hipError_t e = hipMemcpyAsync(dst, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, c->st);
            if (e == hipSuccess) e = hipStreamSynchronize(c->st);
            if (e != hipSuccess) {
                set_error("copy failed: %s", hipGetErrorString(e));
                rc = DI_EHIP;
            }
        }
        (void)hipFree(tmp);
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
        if (!c->pi_ready) DI_FAIL(DI_ESTATE, "di_power has not run");
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
        if (on_device) DI_HIP(hipMemcpy(dst, &v, sizeof(double), hipMemcpyHostToDevice));
        else std::memcpy(dst, &v, sizeof(double));
        return DI_OK;
    }
    default:
        DI_FAIL(DI_EINVAL, "unknown read target %d", what);
    }
}

int di_adjoint(di_ctx *c, const double *g, double tol_inf, double *dZ, double *dw, int on_device, di_stats *st) {
    if (!c) DI_FAIL(DI_EINVAL, "ctx is NULL");
    if (!g || !dZ) DI_FAIL(DI_EINVAL, "g and dZ must not be NULL");
    if (!(tol_inf > 0.0) || !std::isfinite(tol_inf)) DI_FAIL(DI_EINVAL, "tol_inf must be finite and > 0");
    if (c->b) DI_FAIL(DI_EINVAL, "the adjoint supports one right-hand side on one graph");
    if (!c->forward_converged) DI_FAIL(DI_ESTATE, "di_adjoint needs a converged di_diffuse first");
    const i64 n = c->g.n;
    if (!c->lam) {
        DI_TRY(dalloc(c, &c->lam, n));
        DI_TRY(dalloc(c, &c->aF, n));
        DI_TRY(dalloc(c, &c->asnap, n));
        DI_TRY(dalloc(c, &c->actl, 1));
    }
    std::vector<double> hg;
    const double *gsrc = g;
    double mx = 0.0;
    {
        if (on_device) {
            hg.resize((size_t)n);
            DI_HIP(hipMemcpy(hg.data(), g, sizeof(double) * n, hipMemcpyDeviceToHost));
            gsrc = hg.data();
        }
        for (i64 i = 0; i < n; ++i) {
            if (!std::isfinite(gsrc[i])) DI_FAIL(DI_EINVAL, "g[%lld] is not finite", (long long)i);
            mx = std::max(mx, std::fabs(gsrc[i]));
        }
    }
    SweepParams ap = c->p;
    ap.K = fixed_scale(mx, n);
    ap.tol = tol_inf;
    DI_HIP(hipMemcpyAsync(c->aF, gsrc, sizeof(double) * n, hipMemcpyHostToDevice, c->st));
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
    while (!c->h_ctl->done) {
        for (int k = 0; k < c->spc; ++k) {
            DI_TRY(launch_adj_sweep(c->g, c->aF, c->lam, c->asnap, c->actl, ap, c->st, c->s.partR, c->s.partC, &anR,
                                    &anC));
            DI_TRY(launch_finalize(c->actl, ap, FIN_ADJ, c->st, c->s.partR, anR, c->s.partC, anC));
        }
        DI_TRY(sync_ctl(c, c->actl));
        const DevCtl &h = *c->h_ctl;
        if (h.done || h.overflow || h.sweep >= h.budget) break;
    }
    // gradients from x = H (forward history) and lambda
    double *ddZ = dZ, *ddw = dw;
    double *tZ = nullptr, *tw = nullptr;
    if (!on_device) {
        DI_HIP(hipMalloc((void **)&tZ, sizeof(double) * n));
        if (dw) DI_HIP(hipMalloc((void **)&tw, sizeof(double) * std::max<i64>(c->g.m, 1)));
        ddZ = tZ;
        ddw = dw ? tw : nullptr;
    }
    int rc = launch_edge_grad(c->g, c->s.H, c->lam, c->d, ddZ, ddw, c->st);
    DI_HIP(hipEventRecord(c->ev1, c->st));
    if (rc == DI_OK && !on_device) {
        if (hipMemcpyAsync(dZ, tZ, sizeof(double) * n, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
            (dw && c->g.m && hipMemcpyAsync(dw, tw, sizeof(double) * c->g.m, hipMemcpyDeviceToHost, c->st) != hipSuccess))
            rc = DI_EHIP;
    }
    if (hipStreamSynchronize(c->st) != hipSuccess) rc = DI_EHIP;
    if (tZ) (void)hipFree(tZ);
    if (tw) (void)hipFree(tw);
    if (rc != DI_OK) DI_FAIL(rc, "adjoint gradient step failed");
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

int di_save(di_ctx *c, const char *path) {
    if (!c || !path) DI_FAIL(DI_EINVAL, "NULL argument");
    if (c->b) DI_FAIL(DI_EINVAL, "checkpoints cover single right-hand-side solves");
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
    if (!c || !path) DI_FAIL(DI_EINVAL, "NULL argument");
    if (c->b) DI_FAIL(DI_EINVAL, "checkpoints cover single right-hand-side solves");
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
    DI_TRY(launch_fill_zero(c->s.S[0], n * T, c->st));
    DI_TRY(launch_fill_zero(c->s.S[1], n * T, c->st));
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
    if (!c || !value) DI_FAIL(DI_EINVAL, "NULL argument");
    switch (key) {
    case DI_INFO_N: *value = c->g.n; return DI_OK;
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
