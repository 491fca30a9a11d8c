// Several right-hand sides: personalized PageRank for k <= 64 distributions Z_c at once
// (Section 2.1 allows any Z; one solve per Z_c).  The fluid is an n x k tile stored
// node-major (row i holds F_i1..F_ik), the history an n x k double tile.  One wavefront
// owns a row and lane c is column c, so every index or weight read of a row serves all
// k columns and every row access is one contiguous k-element vector.
//
// Fast sweep: a row is taken when some column's fluid reaches that column's threshold
// theta |F_c|_1 / n; the wave then diffuses every column of the row that is still
// running (an elementary diffusion per column, Section 3.1, equation defF): H_ic += f_c,
// the fluid f_c is subtracted from F_ic with an atomic add (pushes that arrive
// meanwhile stay), and d f_c P_ji is added to each successor row j with one coalesced
// k-lane atomic add per edge.
//
// Deterministic sweep: per column exactly the synchronous sweep of one right-hand side
// (snapshot of the active entries, then an ordered pull over IN rows), so column c
// reproduces the single-column solve with Z_c bit for bit.
//
// After either sweep the residual |F_c|_1 of every column is summed in fixed point
// (exact, order-independent), and a column whose bound |F_c|_1/(1-d) meets the
// tolerance stops: its entries are no longer touched (Theorem 1 certifies it).
//
// Float fluid in the fast sweep picks up a rounding error at every atomic push, so the
// tile's fluid is recomputed in double from the history, F = F_0 + d P H - H (the fluid
// of equation HnFn), each time the residual has dropped by REFINE_DROP and before the
// columns are declared converged.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.h"

namespace di {

constexpr int KMAX = 64;
constexpr int TILE_THREADS = 256;
constexpr int TILE_WAVES = TILE_THREADS / WAVE;
constexpr int TILE_GRID = 2048;   // push / snapshot / pull: grid-stride over rows
constexpr int REDUCE_TILE_GRID = 1024;
constexpr int ROWS_U = 8;  // rows a wave loads before it inspects them (scan and reduce)
constexpr int EDGES_U = 8; // row gathers in flight per wave in the fluid recomputation

struct TileCtl {
    long long sweep, budget;
    int all_done, overflow;
    int parity, pad;  // block-local sweeps: which in-flight buffer is read
    u64 tot_nodes, tot_edges;  // rows taken, edge x column pushes
    double R[KMAX], thr[KMAX], maxF[KMAX];
    int done[KMAX];
    long long done_sweep[KMAX];
    u64 limbsL[KMAX][4];
};

// A delivery unit: cross-range in-entries [e0, e0 + len) (len <= DL_UNIT), sorted by
// target.  Whole target rows, unless `split`: then the entries are one segment of a
// row with more than DL_UNIT entries and the sum is added with a device atomic.
struct DlUnit {
    i64 e0;
    int len, split;
};

// A range as the tile sweep visits it: first row, first local edge, rows, local edges.
struct TileRange {
    i64 base, lb;
    int cnt, ne;
};

struct BatchState {
    int k = 0, fp32 = 0, K = 0, det = 0;
    i64 n = 0;
    void *F = nullptr;
    double *F0 = nullptr;  // (1-d) Z, n x k node-major, double for every fluid type
    double *H = nullptr;
    double *snap = nullptr;  // deterministic sweep: pushed value per entry
    TileCtl *ctl = nullptr, *h_ctl = nullptr;
    u64 *partR = nullptr;  // [REDUCE_TILE_GRID][KMAX][PSR]
    u64 *partC = nullptr;  // [TILE_GRID][KMAX][4] leak limbs
    u64 *partK = nullptr;  // [TILE_GRID][2] rows taken, edge pushes
    int gridP = 0, gridR = 0;
    double zsum[KMAX];
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap_st = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gexec_spc = 0;
    double gexec_tol = -1.0, gexec_theta = -1.0;  // the sweeps' tolerance and threshold scale baked in
    // block-local sweeps
    int bld = 0, rounds = 4, gridB = 0, gridD = 0;
    void *S = nullptr;           // in-flight rows (n x k)
    unsigned *fl = nullptr;      // (n + 31) / 32 words: bit i, row i of S holds this sweep's fluid
    int *blk_ptr = nullptr;      // gridB + 1: each workgroup's share of rinfo
    TileRange *rinfo = nullptr;  // nranges: the ranges, grouped by workgroup
    DlUnit *units = nullptr;     // delivery units over the cross-range in-entries
    i64 nunits = 0;
    int *rem_tgt_abs = nullptr;  // m_rem: absolute target row of each cross-range entry
    // exact per-column sums of H (mass balance): limb slots and k doubles
    u64 *partH = nullptr;
    double *hsum = nullptr;
    // fluid recomputation: IN rows longer than REFINE_SEG entries are split into segments
    // (segment s: row seg_row[s], entries [seg_p0[s], seg_p1[s])); a row's segments are
    // consecutive and their partial sums (seg_part, nseg x KMAX) are added in order
    i64 nseg = 0, nlong = 0;
    int *seg_row = nullptr;
    i64 *seg_p0 = nullptr, *seg_p1 = nullptr;
    int *long_first = nullptr;  // nlong + 1: first segment of each long row
    double *seg_part = nullptr;
};

struct TileArgs {
    const i64 *out_ptr;
    const int *out_idx;
    const float *w;
    const i64 *in_ptr;
    const int *in_idx;
    const float *in_w;
    const double *inv_s;
    void *F;
    double *H;
    double *snap;
    TileCtl *ctl;
    u64 *partR, *partC, *partK;
    i64 n;
    int k, K;
    double d;
};

// the leak's sums are signed: the float fluid recomputed from H (F = F_0 + d P H - H) may be
// slightly negative where the pushes' rounding let a node take more than its share
__device__ __forceinline__ bool tile_leak_add(Limbs &a, double v, int K) {
    if (!(v == v) || !(ldexp(fabs(v), K) < 0x1p126)) return false;
    limbs_add_signed(a, v, K);
    return true;
}

__device__ __forceinline__ bool tile_limbs_add(Limbs &a, double v, int K) {
    if (!(v == v) || !(ldexp(v, K) < 0x1p126)) return false;
    limbs_add(a, v, K);
    return true;
}

__device__ __forceinline__ bool tile_stopped(const TileCtl *ctl) {
    return ctl->all_done || ctl->sweep >= ctl->budget;
}

// Add per-lane (per-column) values over the waves of the block and store the column
// sums: out[c * NV + q].  lds: u64[TILE_WAVES * 64 * NV].  Contains barriers.
template <int NV, unsigned MAXMASK = 0, int NW = TILE_WAVES>
__device__ __forceinline__ void block_columns_store(u64 (&v)[NV], u64 *lds, u64 *out, int k) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[(w * WAVE + lane) * NV + q] = v[q];
    __syncthreads();
    if (w == 0 && lane < k) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            u64 s = 0;
            for (int x = 0; x < NW; ++x) {
                const u64 y = lds[(x * WAVE + lane) * NV + q];
                s = ((MAXMASK >> q) & 1u) ? (y > s ? y : s) : s + y;
            }
            out[lane * NV + q] = s;
        }
    }
    __syncthreads();
}

// block_columns_store over nw waves (a runtime count); lds: u64[nw * 64 * NV]
template <int NV, unsigned MAXMASK = 0>
__device__ __forceinline__ void block_columns_store_n(u64 (&v)[NV], u64 *lds, u64 *out, int k, int nw) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[(w * WAVE + lane) * NV + q] = v[q];
    __syncthreads();
    if (w == 0 && lane < k) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            u64 s = 0;
            for (int x = 0; x < nw; ++x) {
                const u64 y = lds[(x * WAVE + lane) * NV + q];
                s = ((MAXMASK >> q) & 1u) ? (y > s ? y : s) : s + y;
            }
            out[lane * NV + q] = s;
        }
    }
    __syncthreads();
}

// Fast sweep (see the file comment).
template <typename T, bool WTD>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_push(TileArgs a) {
    __shared__ u64 lds[TILE_WAVES * WAVE * 4];
    __shared__ u64 kred[2 * TILE_WAVES];
    const TileCtl *ctl = a.ctl;
    if (tile_stopped(ctl)) return;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool col = lane < a.k && !ctl->done[lane];
    const double thr = col ? ctl->thr[lane] : 0.0;
    T *F = reinterpret_cast<T *>(a.F);
    Limbs leak;
    limbs_zero(leak);
    u64 nodes = 0, edges = 0;
    int bad = 0;
    // Each wave takes ROWS_U consecutive rows at a time.  Every stage issues its loads
    // for all rows of the batch before it uses any, so that a wave waits for memory
    // once per stage rather than once per row: (1) the fluid rows, (2) row pointers,
    // 1/s and history rows of the rows taken, (3) their first 64 out-edges, (4) pushes.
    // A workgroup owns a contiguous chunk of rows, so that the rows being pushed to at
    // any moment (mostly in the same host as their source) stay few and cache-resident.
    const i64 chunk = ((a.n + gridDim.x - 1) / gridDim.x + ROWS_U - 1) / ROWS_U * ROWS_U;
    const i64 c_end = min(a.n, ((i64)blockIdx.x + 1) * chunk);
    for (i64 i0 = (i64)blockIdx.x * chunk + (i64)w * ROWS_U; i0 < c_end; i0 += TILE_WAVES * ROWS_U) {
        T vv[ROWS_U];
#pragma unroll
        for (int u = 0; u < ROWS_U; ++u) vv[u] = col ? F[min(i0 + u, a.n - 1) * a.k + lane] : (T)0;
        unsigned act = 0;  // wave-uniform: bit u = row i0 + u is taken
#pragma unroll
        for (int u = 0; u < ROWS_U; ++u)
            if (i0 + u < a.n && __ballot(vv[u] != (T)0 && fabs((double)vv[u]) >= thr) != 0) act |= 1u << u;
        if (act == 0) continue;
        // (2) lanes 0..ROWS_U hold out_ptr[i0 + lane], lanes 0..ROWS_U-1 hold 1/s
        const i64 myptr = a.out_ptr[min(i0 + (i64)min(lane, ROWS_U), a.n)];
        const double myinv = a.inv_s[min(i0 + (i64)min(lane, ROWS_U - 1), a.n - 1)];
        double hv[ROWS_U];
#pragma unroll
        for (int u = 0; u < ROWS_U; ++u)
            hv[u] = ((act >> u) & 1u) && vv[u] != (T)0 ? a.H[(i0 + u) * a.k + lane] : 0.0;
        i64 bb[ROWS_U];
        int cnt0[ROWS_U];
#pragma unroll
        for (int u = 0; u < ROWS_U; ++u) {
            bb[u] = __shfl(myptr, u, WAVE);
            cnt0[u] = (int)min((i64)WAVE, __shfl(myptr, u + 1, WAVE) - bb[u]);
        }
        // (3) first chunk of out-edges of every row taken
        int idx0[ROWS_U];
        float w0[ROWS_U];
#pragma unroll
        for (int u = 0; u < ROWS_U; ++u) {
            const bool use = ((act >> u) & 1u) && cnt0[u] > 0;
            const i64 p = bb[u] + min(lane, max(cnt0[u], 1) - 1);
            idx0[u] = use ? a.out_idx[p] : 0;
            w0[u] = (WTD && use) ? a.w[p] : 1.0f;
        }
        // take every running column of the rows (pushes that arrived since the load stay
        // in F: the taken amount is subtracted), then push
#pragma unroll
        for (int u = 0; u < ROWS_U; ++u) {
            if (!((act >> u) & 1u)) continue;
            const i64 i = i0 + u;
            const T v = vv[u];
            const double f = (double)v;
            if (v != (T)0) {
                atomicAdd(&F[i * a.k + lane], -v);
                a.H[i * a.k + lane] = hv[u] + f;
            }
            nodes += lane == 0 ? 1 : 0;
            const i64 b = bb[u], e = __shfl(myptr, u + 1, WAVE);
            if (e == b) {
                if (v != (T)0 && !tile_leak_add(leak, f, a.K)) bad = 1;
                continue;
            }
            const double q = (a.d * f) * __shfl(myinv, u, WAVE);
            edges += lane == 0 ? (u64)(e - b) * (u64)__popcll(__ballot(v != (T)0)) : 0ull;
            for (i64 eb = b; eb < e; eb += WAVE) {
                const int cnt = (int)min((i64)WAVE, e - eb);
                const int myidx = eb == b ? idx0[u] : a.out_idx[eb + min(lane, cnt - 1)];
                const float myw = eb == b ? w0[u] : (WTD ? a.w[eb + min(lane, cnt - 1)] : 1.0f);
                for (int kk = 0; kk < cnt; ++kk) {
                    const int j = __shfl(myidx, kk, WAVE);
                    const double val = WTD ? q * (double)__shfl(myw, kk, WAVE) : q;
                    if (v != (T)0) atomicAdd(&F[(i64)j * a.k + lane], (T)val);
                }
            }
        }
    }
    u64 lv[4] = {leak.l[0], leak.l[1], leak.l[2], leak.l[3]};
    block_columns_store<4>(lv, lds, a.partC + (i64)blockIdx.x * KMAX * 4, a.k);
    u64 kv[2] = {nodes, edges};
    block_store_partials<2>(kv, kred, a.partK + (i64)blockIdx.x * 2);
    if (bad) atomicOr(&a.ctl->overflow, 1);
}

// ---------------------------------------------------------------------------
// Block-local fast sweep of the tile, in two kernels per sweep.
//
// k_tile_bld: node ids are grouped into ranges of B = 2^rb rows; a workgroup of B / 16
// waves takes its ranges one after another, wave w owning rows [16 w, 16 w + 16) of a
// range.  The range's fluid tile F[B][k] (double in LDS, whatever the fluid type in
// memory) and its local edge lists sit in LDS; lane c of a wave holds column c.  For a
// range it
//   1. stages the fluid rows (they already hold what other ranges sent last sweep) and
//      the targets (and weights) of the range's local edges;
//   2. runs up to `rounds` local rounds: each wave scans its rows, takes a row when some
//      running column reaches its threshold (every running column of the row is
//      diffused, Section 3.1), adds it to the row of H (an atomic add in this XCD's L2:
//      no other wave touches the row during the sweep), pushes d f P e_i along the
//      row's local edges with LDS atomics (one k-lane row add per edge) and, for a row
//      with cross-range edges, adds d f / s_i to the row's in-flight fluid S_i;
//   3. writes its rows of F back and flags the rows whose S_i holds this sweep's fluid
//      (one bit per row).
// k_tile_deliver: one wave per unit of cross-range in-entries (whole target rows,
//   or a segment of a long row) lists the unit's flagged entries, gathers their
//   in-flight rows, adds them up per target in registers and adds the sum to the
//   target's fluid row.
// No device-scope atomics on the common path: on this chip they are carried out past
// the per-XCD L2 caches.  The residual of every column, |F|_1 plus the fluid in
// flight, is summed at write-back; delivery moves fluid without changing it.
// ---------------------------------------------------------------------------
// The LDS tile holds the fluid in double whatever the fluid type in memory: on this chip
// a 64-lane LDS atomic add costs about 8 cycles in double and about 190 in float.  A
// range whose tiles fit TB_LDS runs two workgroups per compute unit (one stages or writes
// back a range while the other runs local rounds); larger ones one workgroup, within
// TB_LDS_ONE.  A wave owns 16 rows, so a workgroup has 2^rb / 16 waves.
constexpr int TB_RPW = 16;  // rows per wave: one bit each in a wave-uniform mask, one 16-bit word of flags
constexpr int TB_MAXW = 16; // waves per workgroup at 2^8-row ranges
constexpr int TB_MAX_THREADS = TB_MAXW * WAVE;
constexpr int TB_GRID = 1024;
constexpr size_t TB_LDS = 78 * 1024;
constexpr size_t TB_LDS_ONE = 156 * 1024;
constexpr int TB_MIN_RB = 6, TB_MAX_RB = 8;
static_assert(TB_RPW == 16 && ((1 << TB_MAX_RB) / TB_RPW) <= TB_MAXW, "waves per workgroup");
constexpr int DL_THREADS = 256;
constexpr int DL_WAVES = DL_THREADS / WAVE;
constexpr int DL_GRID = 4096;
constexpr int DL_UNIT = 64;  // cross-range entries per delivery unit

struct TileBldArgs {
    const i64 *loc_ptr;
    const unsigned short *loc_tgt;
    const float *loc_w;
    const double *rw;
    const unsigned *deg_flags;
    const double *inv_s;
    const int *blk_ptr;
    const TileRange *rinfo;  // the ranges grouped by workgroup (shares given by blk_ptr)
    i64 n;
    int rb, k, K, rounds;
    int le_max;  // local edges of a range that fit the LDS edge buffer
    void *F;
    double *H;
    void *S;
    unsigned *fl;
    TileCtl *ctl;
    double d;
    u64 *partR, *partC, *partK;
};

inline size_t tile_edge_bytes(bool weighted) { return weighted ? 6 : 2; }

// LDS of a range (the edge buffer comes on top): the fluid tile (double), degrees and
// local row offsets (u32), then per row the out-weight of its cross-range edges and 1/s_i
// (doubles, 8-byte aligned)
__host__ __device__ inline size_t tile_rowdata_offset(int rb, int k) {
    const size_t B = (size_t)1 << rb;
    return (B * k * 8 + (2 * B + 1) * 4 + 7) & ~(size_t)7;
}

__host__ __device__ inline size_t tile_bld_fixed_lds(int rb, int k, bool weighted) {
    const size_t B = (size_t)1 << rb;
    (void)weighted;
    return tile_rowdata_offset(rb, k) + B * 16 + 16;
}

// two workgroups per compute unit when the tiles and 1024 local edges fit TB_LDS
inline bool tile_two_per_cu(int rb, int k, bool weighted) {
    return tile_bld_fixed_lds(rb, k, weighted) + 1024 * tile_edge_bytes(weighted) <= TB_LDS;
}

inline size_t tile_lds_budget(int rb, int k, bool weighted) {
    return tile_two_per_cu(rb, k, weighted) ? TB_LDS : TB_LDS_ONE;
}

// the per-column reductions at the end reuse the tiles: (B / 16) waves x 64 x PSR words
inline size_t tile_red_lds(int rb) { return (size_t)(((size_t)1 << rb) / TB_RPW) * WAVE * PSR * sizeof(u64); }

// local edges per range for which the edge buffer has room (0: the range size does not fit)
inline int tile_le_max(int rb, int k, bool weighted) {
    if (rb < TB_MIN_RB || rb > TB_MAX_RB) return 0;
    const size_t fixed = tile_bld_fixed_lds(rb, k, weighted), budget = tile_lds_budget(rb, k, weighted);
    if (fixed + 256 * tile_edge_bytes(weighted) > budget) return 0;
    const size_t le = (budget - fixed) / tile_edge_bytes(weighted);
    return (int)std::min<size_t>(le & ~(size_t)3, 1 << 16);
}

inline size_t tile_bld_lds_launch(int rb, int k, bool weighted) {
    const size_t le = (size_t)tile_le_max(rb, k, weighted);
    return std::max(tile_bld_fixed_lds(rb, k, weighted) + le * tile_edge_bytes(weighted), tile_red_lds(rb));
}

// a 16-byte unit of fluid (4 floats or 2 doubles) into the double LDS tile
template <typename T>
__device__ __forceinline__ void tile_lds_unit(double *dst, const uint4 &v) {
    if constexpr (sizeof(T) == 4) {
        dst[0] = (double)__uint_as_float(v.x);
        dst[1] = (double)__uint_as_float(v.y);
        dst[2] = (double)__uint_as_float(v.z);
        dst[3] = (double)__uint_as_float(v.w);
    } else {
        dst[0] = __hiloint2double((int)v.y, (int)v.x);
        dst[1] = __hiloint2double((int)v.w, (int)v.z);
    }
}

// Workgroup barrier that orders LDS accesses only: it does not wait for the waves'
// outstanding global stores and atomics (the tile sweep's rows of H, S, F and flags are
// not read back by any wave of the launch).
__device__ __forceinline__ void block_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Take the rows of act (bit u: row i0 + u, wave-uniform) of one scan group: every
// running column's fluid f moves to the history (a workgroup-scope atomic add to the
// row of H, which no other wave touches during the sweep) and is pushed along the row's
// local edges; a row with cross-range edges also adds d f / s_i to its in-flight row S_i.
// The first take of row i0 + u in this visit of the range (bit ubase + u of `taken`)
// stores S_i, so that no earlier sweep's value survives, later takes add to it.
template <typename T, bool WTD, int RU>
__device__ __forceinline__ void tile_take_rows(const TileBldArgs &a, unsigned act, int i0, int ubase,
                                               const double (&vv)[RU], unsigned &taken, bool col, bool colk, int lane,
                                               int k, double *Fl, const unsigned *Deg, const unsigned *Off,
                                               const double *Rw, const double *Inv, const unsigned short *Et,
                                               const float *Ew, bool lds_edges, i64 base,
                                               i64 lb, double &Rd, double &Ld, u64 &nodes, u64 &edges) {
    T *S = reinterpret_cast<T *>(a.S);
    double fu[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u)
        fu[u] = ((act >> u) & 1u) && col && vv[u] != 0.0 ? atomicExch(&Fl[(i0 + u) * k + lane], 0.0) : 0.0;
    for (int u = 0; u < RU; ++u) {
        if (!((act >> u) & 1u)) continue;
        const int i = i0 + u;
        const i64 gi = base + i;
        double f = fu[0];
#pragma unroll
        for (int v = 1; v < RU; ++v) f = u == v ? fu[v] : f;
        nodes += lane == 0 ? 1 : 0;
        if (f != 0.0) __hip_atomic_fetch_add(&a.H[gi * k + lane], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const unsigned dfl = Deg[i], deg = dfl & 0x7fffffffu;
        if (deg == 0) {
            Ld += f;
            continue;
        }
        const double q = (a.d * f) * Inv[i];
        if (dfl & 0x80000000u) {
            const T sv = (T)q;
            const unsigned bit = 1u << (ubase + u);
            if (taken & bit) {
                if (sv != (T)0) __hip_atomic_fetch_add(&S[gi * k + lane], sv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                if (colk) S[gi * k + lane] = sv;
                taken |= bit;
            }
            Rd += fabs((double)sv) * Rw[i];
        }
        const int st = (int)Off[i], ln = (int)Off[i + 1] - st;
        const u64 fm = __ballot(f != 0.0);
        edges += lane == 0 ? (u64)ln * (u64)__popcll(fm) : 0ull;
        if (fm == 0) continue;
        for (int eb = 0; eb < ln; eb += WAVE) {
            const int c2 = min(WAVE, ln - eb);
            const int pe = st + eb + min(lane, c2 - 1);
            const int myt = lds_edges ? (int)Et[pe] : (int)a.loc_tgt[lb + pe];
            const float myw = WTD ? (lds_edges ? Ew[pe] : a.loc_w[lb + pe]) : 1.0f;
            for (int kk = 0; kk < c2; ++kk) {
                const int t = __builtin_amdgcn_readlane(myt, kk);
                const double val =
                    WTD ? q * (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(myw), kk)) : q;
                if (f != 0.0) atomicAdd(&Fl[t * k + lane], val);
            }
        }
    }
}

template <typename T, bool WTD>
__global__ void __launch_bounds__(TB_MAX_THREADS) k_tile_bld(TileBldArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ u64 kred[2 * TB_MAXW];
    const TileCtl *ctl = a.ctl;
    if (tile_stopped(ctl)) return;
    const int B = 1 << a.rb, k = a.k, nthr = (int)blockDim.x;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool colk = lane < k;
    const bool col = colk && !ctl->done[lane];
    const double thr = col ? ctl->thr[lane] : 0.0;
    double *Fl = reinterpret_cast<double *>(smem);
    unsigned *Deg = reinterpret_cast<unsigned *>(Fl + (size_t)B * k);
    unsigned *Off = Deg + B;
    double *Rw = reinterpret_cast<double *>(smem + tile_rowdata_offset(a.rb, k));
    double *Inv = Rw + B;
    // edge buffer: weights (4-byte aligned) first, then the 16-bit targets
    float *Ew = reinterpret_cast<float *>(Inv + B);
    unsigned short *Et = reinterpret_cast<unsigned short *>(WTD ? Ew + a.le_max : Ew);
    T *F = reinterpret_cast<T *>(a.F);

    // residual and leak: each lane (column) adds its values in double; the sums are
    // raised by 2^-30 relative (far above the rounding of up to 2^22 additions) and
    // then enter the exact fixed-point sums, so the residual never falls short.  The
    // fluid in flight enters as the sum of its parts' magnitudes.
    double Rd = 0.0, Ld = 0.0;
    u64 mx = 0, nodes = 0, edges = 0;
    int bad = 0;
    // The next range's fluid (PF 16-byte units per thread), row data (B <= threads) and
    // first PE local edges per thread are loaded into registers while the current range
    // runs its local rounds; staging then stores registers (the rest, if any, is loaded
    // at staging).
    constexpr int VE = 16 / (int)sizeof(T), PF = 4, PE = 2;
    uint4 pf[PF];
    unsigned pdv = 0;
    i64 pov = 0;
    double prv = 0.0, piv = 0.0;
    unsigned short pt[PE];
    float pw[PE];
    const int tid = threadIdx.x;
    auto prefetch = [&](const TileRange &ri) {
        const int tot = ri.cnt * k, nv = tot / VE;
        const uint4 *srcv = reinterpret_cast<const uint4 *>(F + ri.base * k);
#pragma unroll
        for (int u = 0; u < PF; ++u) pf[u] = nv > 0 ? srcv[min(tid + u * nthr, nv - 1)] : make_uint4(0, 0, 0, 0);
        const bool row = tid < ri.cnt, offrow = tid <= ri.cnt;
        pdv = row ? a.deg_flags[ri.base + tid] : 0u;
        pov = offrow ? a.loc_ptr[ri.base + tid] : 0;
        prv = row ? a.rw[ri.base + tid] : 0.0;
        piv = WTD && row ? a.inv_s[ri.base + tid] : 0.0;
        const bool le = ri.ne > 0 && ri.ne <= a.le_max;
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const i64 e = ri.lb + min(tid + u * nthr, max(ri.ne - 1, 0));
            pt[u] = le ? a.loc_tgt[e] : (unsigned short)0;
            pw[u] = WTD && le ? a.loc_w[e] : 0.0f;
        }
    };
    const int q0 = a.blk_ptr[blockIdx.x], q1 = a.blk_ptr[blockIdx.x + 1];
    if (q0 < q1) prefetch(a.rinfo[q0]);
    for (int q = q0; q < q1; ++q) {
        const TileRange ri = a.rinfo[q];
        const i64 base = ri.base, lb = ri.lb;
        const int cnt = ri.cnt, ne = ri.ne;
        const bool lds_edges = ne <= a.le_max;
        // 1. stage: the range's fluid rows are one contiguous block of cnt * k values
        // (256-byte aligned: ranges start at multiples of 64 rows) in 16-byte units, the
        // row data and the local edges, from the prefetched registers where they cover them
        {
            const int tot = cnt * k, nv = tot / VE;
            const uint4 *srcv = reinterpret_cast<const uint4 *>(F + base * k);
#pragma unroll
            for (int u = 0; u < PF; ++u)
                if (tid + u * nthr < nv) tile_lds_unit<T>(Fl + (size_t)(tid + u * nthr) * VE, pf[u]);
            for (int e = tid + PF * nthr; e < nv; e += nthr) tile_lds_unit<T>(Fl + (size_t)e * VE, srcv[e]);
            for (int e = nv * VE + tid; e < tot; e += nthr) Fl[e] = (double)F[base * k + e];
            if (tid < cnt) {
                Deg[tid] = pdv;
                Rw[tid] = prv;
                const unsigned dg = pdv & 0x7fffffffu;
                Inv[tid] = WTD ? piv : dg ? 1.0 / (double)dg : 0.0;
            }
            if (tid <= cnt) Off[tid] = (unsigned)(pov - lb);
            if (lds_edges) {
#pragma unroll
                for (int u = 0; u < PE; ++u) {
                    const int e = tid + u * nthr;
                    if (e < ne) {
                        Et[e] = pt[u];
                        if (WTD) Ew[e] = pw[u];
                    }
                }
                for (int e = tid + PE * nthr; e < ne; e += nthr) {
                    Et[e] = a.loc_tgt[lb + e];
                    if (WTD) Ew[e] = a.loc_w[lb + e];
                }
            }
        }
        block_sync_lds();
        if (q + 1 < q1) prefetch(a.rinfo[q + 1]);
        // 2. local rounds over the wave's rows [my0, my1), scanned RU at a time: their LDS
        // values are read before any is taken
        const int my0 = min(cnt, w * TB_RPW), my1 = min(cnt, my0 + TB_RPW);
        constexpr int RU = 4;
        unsigned taken = 0;
        for (int round = 0; round < a.rounds; ++round) {
            bool any = false;
            for (int i0 = my0; i0 < my1; i0 += RU) {
                double vv[RU];
#pragma unroll
                for (int u = 0; u < RU; ++u)
                    vv[u] = col && i0 + u < my1
                                ? __hip_atomic_load(&Fl[(i0 + u) * k + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                                : 0.0;
                unsigned act = 0;
#pragma unroll
                for (int u = 0; u < RU; ++u)
                    if (__ballot(vv[u] != 0.0 && fabs(vv[u]) >= thr) != 0) act |= 1u << u;
                if (act != 0) {
                    any = true;
                    tile_take_rows<T, WTD, RU>(a, act, i0, i0 - my0, vv, taken, col, colk, lane, k, Fl, Deg, Off, Rw, Inv, Et, Ew,
                                               lds_edges, base, lb, Rd, Ld, nodes, edges);
                }
            }
            if (!any) break;
        }
        block_sync_lds();  // every local push has landed
        // 3. write back the wave's rows of F and their word of flags: bit i is set when row
        // i was taken, so that its in-flight row (if it has cross-range edges) holds this
        // sweep's fluid
        for (int i = my0; i < my1; ++i) {
            const i64 gi = base + i;
            const T v = colk ? (T)Fl[i * k + lane] : (T)0;
            if (colk) F[gi * k + lane] = v;
            Rd += fabs((double)v);
            const u64 vb = (u64)__double_as_longlong(fabs((double)v));
            mx = vb > mx ? vb : mx;
        }
        // (the wave's 16 rows are one 16-bit half of a flag word: ranges start at
        // multiples of 64)
        if (lane == 0 && my0 < my1) reinterpret_cast<unsigned short *>(a.fl)[(base + my0) >> 4] = (unsigned short)taken;
        block_sync_lds();  // the next range reuses the LDS tiles
    }
    Limbs R, leak;
    limbs_zero(R);
    limbs_zero(leak);
    if (!tile_limbs_add(R, Rd * (1.0 + 0x1p-30), a.K)) bad = 1;
    if (!tile_leak_add(leak, Ld, a.K)) bad = 1;
    // the per-column reductions reuse the tile's LDS (waves * 64 * PSR words)
    const int nw = nthr / WAVE;
    u64 *red = reinterpret_cast<u64 *>(smem);
    u64 rv[PSR] = {R.l[0], R.l[1], R.l[2], R.l[3], mx};
    block_columns_store_n<PSR, 1u << 4>(rv, red, a.partR + (i64)blockIdx.x * KMAX * PSR, k, nw);
    u64 lv[4] = {leak.l[0], leak.l[1], leak.l[2], leak.l[3]};
    block_columns_store_n<4, 0>(lv, red, a.partC + (i64)blockIdx.x * KMAX * 4, k, nw);
    u64 kv[2] = {nodes, edges};
    block_store_partials<2>(kv, kred, a.partK + (i64)blockIdx.x * 2);
    if (bad) atomicOr(&a.ctl->overflow, 1);
}

struct TileDlArgs {
    const DlUnit *units;
    i64 nunits;
    const int *rem_src;
    const int *rem_tgt;  // absolute target row of each entry
    const float *rem_w;
    const void *S;
    const unsigned *fl;
    void *F;
    const TileCtl *ctl;
    int k, force;
    u64 *partK;  // per-workgroup count of rows delivered
};

// The wave first works out, lane-parallel, which entries of its unit are flagged and
// which flagged entry ends its target's run (no later flagged entry of the unit has the
// same target: entries are sorted by target), and lists the flagged entries in LDS in
// entry order; it then walks the list, gathering PB in-flight rows at a time.
struct DlSlot {
    int src, tgt, w, end;
};

__device__ __forceinline__ void dl_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, bool WTD>
__global__ void __launch_bounds__(DL_THREADS) k_tile_deliver(TileDlArgs a) {
    __shared__ u64 kred[2 * DL_WAVES];
    __shared__ DlSlot slots[DL_WAVES][WAVE];
    if (!a.force && tile_stopped(a.ctl)) return;
    constexpr int PB = 8;  // in-flight rows gathered per batch
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool colk = lane < a.k;
    const int k = a.k;
    const T *S = reinterpret_cast<const T *>(a.S);
    T *F = reinterpret_cast<T *>(a.F);
    DlSlot *sl = slots[w];
    u64 delivered = 0;
    const i64 nw = (i64)gridDim.x * DL_WAVES;
    for (i64 q = (i64)blockIdx.x * DL_WAVES + w; q < a.nunits; q += nw) {
        const DlUnit un = a.units[q];
        const bool in = lane < un.len;
        const i64 p = un.e0 + min(lane, un.len - 1);
        const int src = a.rem_src[p];
        const int tgt = a.rem_tgt[p];
        const float ew = WTD ? a.rem_w[p] : 1.0f;
        const bool flg = in && ((a.fl[src >> 5] >> (src & 31)) & 1u);
        const u64 m = __ballot(flg);
        if (m == 0) continue;
        const int nf = __popcll(m);
        delivered += lane == 0 ? (u64)nf : 0ull;
        // last entry of each target's segment, then: no flagged entry after this one up
        // to the end of its segment
        const int tnext = __shfl_down(tgt, 1);
        const u64 seg_end = __ballot(in && (lane == un.len - 1 || tnext != tgt));
        const u64 ge = seg_end & (~0ull << lane);
        const int e = ge ? __ffsll((long long)ge) - 1 : WAVE - 1;
        const u64 after = lane == WAVE - 1 ? 0ull : (~0ull << (lane + 1));
        const u64 upto = e == WAVE - 1 ? ~0ull : ((1ull << (e + 1)) - 1);
        const bool end = (m & after & upto) == 0;
        const int pos = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (flg) sl[pos] = DlSlot{src, tgt, WTD ? __float_as_int(ew) : 0, end ? 1 : 0};
        dl_wave_sync();
        T run = (T)0;
        for (int b0 = 0; b0 < nf; b0 += PB) {
            DlSlot d[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) d[u] = sl[min(b0 + u, nf - 1)];
            // the in-flight rows, and the fluid rows of the targets whose run ends in this
            // batch (no other wave writes them: a unit holds whole target rows, and the
            // split units of a long row only add atomically)
            T sv[PB], fv[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                sv[u] = colk ? S[(i64)d[u].src * k + lane] : (T)0;
                fv[u] = colk && d[u].end && !un.split ? F[(i64)d[u].tgt * k + lane] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                if (b0 + u >= nf) break;
                T val = sv[u];
                if (WTD) val = (T)((double)val * (double)__int_as_float(d[u].w));
                run += val;
                if (d[u].end) {
                    if (colk && run != (T)0) {
                        if (un.split) atomicAdd(&F[(i64)d[u].tgt * k + lane], run);
                        else F[(i64)d[u].tgt * k + lane] = fv[u] + run;
                    }
                    run = (T)0;
                }
            }
        }
        dl_wave_sync();  // the next unit reuses the list
    }
    u64 kv[2] = {0, delivered};
    block_store_partials<2>(kv, kred, a.partK + (i64)blockIdx.x * 2);
}

// Deterministic sweep, step 1: active entries of running columns move to H; snap holds
// (d f) / s_i for them (0 elsewhere); dangling ones add to the leak.
template <typename T>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_snapshot(TileArgs a) {
    __shared__ u64 lds[TILE_WAVES * WAVE * 4];
    __shared__ u64 kred[2 * TILE_WAVES];
    const TileCtl *ctl = a.ctl;
    if (tile_stopped(ctl)) return;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool col = lane < a.k && !ctl->done[lane];
    const double thr = col ? ctl->thr[lane] : 0.0;
    T *F = reinterpret_cast<T *>(a.F);
    Limbs leak;
    limbs_zero(leak);
    u64 nodes = 0, edges = 0;
    int bad = 0;
    const i64 nwaves = (i64)gridDim.x * TILE_WAVES;
    for (i64 i = (i64)blockIdx.x * TILE_WAVES + w; i < a.n; i += nwaves) {
        const i64 slot = i * a.k + lane;
        const T v = lane < a.k ? F[slot] : (T)0;
        const bool act = col && v != (T)0 && fabs((double)v) >= thr;
        double q = 0.0;
        if (act) {
            const double f = (double)v;
            a.H[slot] += f;
            F[slot] = (T)0;
            const double inv = a.inv_s[i];
            if (inv == 0.0) {
                if (!tile_leak_add(leak, f, a.K)) bad = 1;
            } else {
                q = (a.d * f) * inv;
            }
        }
        const u64 am = __ballot(act);
        if (lane == 0 && am) {
            nodes += 1;
            edges += (u64)(a.out_ptr[i + 1] - a.out_ptr[i]) * (u64)__popcll(am);
        }
        if (lane < a.k) a.snap[slot] = q;
    }
    u64 lv[4] = {leak.l[0], leak.l[1], leak.l[2], leak.l[3]};
    block_columns_store<4>(lv, lds, a.partC + (i64)blockIdx.x * KMAX * 4, a.k);
    u64 kv[2] = {nodes, edges};
    block_store_partials<2>(kv, kred, a.partK + (i64)blockIdx.x * 2);
    if (bad) atomicOr(&a.ctl->overflow, 1);
}

// Deterministic sweep, step 2: F_jc = left fold over IN row j (ascending source) of
// snap_ic (* w), starting from F_jc, in double, rounded once to the fluid type.
template <typename T, bool WTD>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_pull(TileArgs a) {
    const TileCtl *ctl = a.ctl;
    if (tile_stopped(ctl)) return;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    if (lane >= a.k) return;
    T *F = reinterpret_cast<T *>(a.F);
    const i64 nwaves = (i64)gridDim.x * TILE_WAVES;
    for (i64 j = (i64)blockIdx.x * TILE_WAVES + w; j < a.n; j += nwaves) {
        const i64 p0 = a.in_ptr[j], p1 = a.in_ptr[j + 1];
        if (p0 == p1) continue;
        double acc = (double)F[j * a.k + lane];
        for (i64 p = p0; p < p1; ++p) {
            const i64 src = a.in_idx[p];
            if (WTD) acc += a.snap[src * a.k + lane] * (double)a.in_w[p];
            else acc += a.snap[src * a.k + lane];
        }
        F[j * a.k + lane] = (T)acc;
    }
}

// Fluid recomputation: F_jc = (F0_jc + d sum over IN row j of H_ic / s_i (* w)) - H_jc,
// in double, stored in the fluid type.
constexpr int REFINE_SEG = 2048;  // IN entries per segment of a long row

// d-free part of the recomputation over IN entries [p0, p1): sum of H_ic / s_i (* w), in
// entry order.  64 entries per step: lane l loads source l's index and scale; then
// RF_U history rows are gathered at a time.
constexpr int RF_U = 8;
template <bool WTD>
__device__ __forceinline__ double tile_in_sum(const TileArgs &a, i64 p0, i64 p1, int lane, bool col) {
    double acc = 0.0;
    for (i64 pb = p0; pb < p1; pb += WAVE) {
        const int cnt = (int)min((i64)WAVE, p1 - pb);
        const int mysrc = a.in_idx[pb + min(lane, cnt - 1)];
        double mys = a.inv_s[mysrc];
        if (WTD) mys *= (double)a.in_w[pb + min(lane, cnt - 1)];
        for (int kb = 0; kb < cnt; kb += RF_U) {
            double hv[RF_U], sv[RF_U];
#pragma unroll
            for (int u = 0; u < RF_U; ++u) {
                const int kk = min(kb + u, cnt - 1);
                const i64 src = __shfl(mysrc, kk, WAVE);
                sv[u] = __shfl(mys, kk, WAVE);
                hv[u] = col ? a.H[src * a.k + lane] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < RF_U; ++u)
                if (kb + u < cnt) acc += hv[u] * sv[u];
        }
    }
    return acc;
}

// Rows up to REFINE_SEG IN entries, consecutive rows on consecutive waves (the chip works
// on a window of a few hosts at a time, whose history rows the L2 caches share; a
// contiguous block of rows per wave measured 10% slower).  Then the waves share the
// segments of the longer rows, whose partial sums go to seg_part.
template <typename T, bool WTD>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_refine(TileArgs a, const double *F0, const int *seg_row,
                                                              const i64 *seg_p0, const i64 *seg_p1, i64 nseg,
                                                              double *seg_part) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool col = lane < a.k;  // every lane takes part in the index loads and shuffles
    T *F = reinterpret_cast<T *>(a.F);
    const i64 nwaves = (i64)gridDim.x * TILE_WAVES, gw = (i64)blockIdx.x * TILE_WAVES + w;
    for (i64 j = gw; j < a.n; j += nwaves) {
        const i64 p0 = a.in_ptr[j], p1 = a.in_ptr[j + 1];
        if (p1 - p0 > REFINE_SEG) continue;
        const double acc = tile_in_sum<WTD>(a, p0, p1, lane, col);
        if (col) {
            const i64 slot = j * a.k + lane;
            F[slot] = (T)((F0[slot] + a.d * acc) - a.H[slot]);
        }
    }
    for (i64 sg = gw; sg < nseg; sg += nwaves) {
        const double acc = tile_in_sum<WTD>(a, seg_p0[sg], seg_p1[sg], lane, col);
        if (col) seg_part[sg * KMAX + lane] = acc;
    }
}

// The long rows: their segments' partial sums, added in segment order.
template <typename T>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_refine_long(TileArgs a, const double *F0, const int *seg_row,
                                                                   const int *long_first, i64 nlong,
                                                                   const double *seg_part) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool col = lane < a.k;
    T *F = reinterpret_cast<T *>(a.F);
    const i64 nwaves = (i64)gridDim.x * TILE_WAVES;
    for (i64 q = (i64)blockIdx.x * TILE_WAVES + w; q < nlong; q += nwaves) {
        const int s0 = long_first[q], s1 = long_first[q + 1];
        double acc = 0.0;
        for (int sg = s0; sg < s1; ++sg) acc += col ? seg_part[(i64)sg * KMAX + lane] : 0.0;
        if (col) {
            const i64 slot = (i64)seg_row[s0] * a.k + lane;
            F[slot] = (T)((F0[slot] + a.d * acc) - a.H[slot]);
        }
    }
}

// Per-column fixed-point residual and max |F| into per-workgroup slots.
template <typename T>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_reduce(TileArgs a, int force) {
    __shared__ u64 lds[TILE_WAVES * WAVE * PSR];
    const TileCtl *ctl = a.ctl;
    if (!force && tile_stopped(ctl)) return;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    const bool col = lane < a.k;
    const T *F = reinterpret_cast<const T *>(a.F);
    Limbs R;
    limbs_zero(R);
    u64 mx = 0;
    int bad = 0;
    if (col) {
        const i64 nwaves = (i64)gridDim.x * TILE_WAVES;
        for (i64 i0 = ((i64)blockIdx.x * TILE_WAVES + w) * ROWS_U; i0 < a.n; i0 += nwaves * ROWS_U) {
            T vv[ROWS_U];
#pragma unroll
            for (int u = 0; u < ROWS_U; ++u) vv[u] = F[min(i0 + u, a.n - 1) * a.k + lane];
#pragma unroll
            for (int u = 0; u < ROWS_U; ++u) {
                if (i0 + u >= a.n) break;
                const double v = fabs((double)vv[u]);
                if (!tile_limbs_add(R, v, a.K)) bad = 1;
                const u64 bits = (u64)__double_as_longlong(v);
                mx = bits > mx ? bits : mx;
            }
        }
    }
    u64 v[PSR] = {R.l[0], R.l[1], R.l[2], R.l[3], mx};
    block_columns_store<PSR, 1u << 4>(v, lds, a.partR + (i64)blockIdx.x * KMAX * PSR, a.k);
    if (bad) atomicOr(&a.ctl->overflow, 1);
}

struct TileFin {
    TileCtl *ctl;
    const u64 *partR, *partC;
    int nR, nC;
    int k, K, mode;  // mode: FIN_DI after a sweep, FIN_INIT for the state at the start of a call
    double d, theta, tol, n_d;
};

// One workgroup per column: add the slots, then residual, bound, stop and threshold.
__global__ void __launch_bounds__(256) k_tile_finalize(TileFin a) {
    TileCtl *ctl = a.ctl;
    const int c = blockIdx.x;  // modes FIN_DI (after a sweep), FIN_INIT, FIN_DELIVER
    if (a.mode == FIN_DI && (tile_stopped(ctl) || ctl->done[c])) return;
    u64 v[PSR + 4];
#pragma unroll
    for (int q = 0; q < PSR + 4; ++q) v[q] = 0;
    for (int b = threadIdx.x; b < a.nR; b += blockDim.x) {
        const u64 *p = a.partR + ((i64)b * KMAX + c) * PSR;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += p[q];
        v[4] = p[4] > v[4] ? p[4] : v[4];
    }
    for (int b = threadIdx.x; b < a.nC; b += blockDim.x) {
        const u64 *p = a.partC + ((i64)b * KMAX + c) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[PSR + q] += p[q];
    }
    __shared__ u64 lds[(PSR + 4) * 4];
    __shared__ u64 tot[PSR + 4];
    block_store_partials<PSR + 4, 1u << 4>(v, lds, tot);
    if (threadIdx.x != 0) return;
    const double R = limbs_to_double_raw(tot[0], tot[1], tot[2], tot[3], a.K);
    for (int q = 0; q < 4; ++q) ctl->limbsL[c][q] += tot[PSR + q];
    limbs_normalize(ctl->limbsL[c]);
    const double mx = __longlong_as_double((long long)tot[4]);
    ctl->R[c] = R;
    ctl->maxF[c] = mx;
    const double bound = R / (1.0 - a.d);
    if (!(bound == bound)) atomicOr(&ctl->overflow, 1);
    const int done = bound <= a.tol ? 1 : 0;
    if (done && !ctl->done[c]) ctl->done_sweep[c] = ctl->sweep + (a.mode == FIN_DI ? 1 : 0);
    if (!done) ctl->done_sweep[c] = -1;
    ctl->done[c] = done;
    double thr = ((a.theta * R) / a.n_d) * (1.0 - 0x1p-30);
    if (mx < thr) thr = 0.0;  // nothing reaches the threshold: take every nonzero entry
    ctl->thr[c] = thr;
}

// Whole-tile control: counters, sweep count, all-done flag.
__global__ void __launch_bounds__(256) k_tile_control(TileCtl *ctl, const u64 *partK, int nK, int k, int mode) {
    if (mode == FIN_DI && tile_stopped(ctl)) return;
    u64 v[2] = {0, 0};
    if (mode != FIN_INIT)
        for (int b = threadIdx.x; b < nK; b += blockDim.x) {
            v[0] += partK[2 * b];
            v[1] += partK[2 * b + 1];
        }
    __shared__ u64 lds[2 * 4];
    __shared__ u64 tot[2];
    block_store_partials<2>(v, lds, tot);
    if (threadIdx.x != 0) return;
    if (mode == FIN_DI) {
        ctl->tot_nodes += tot[0];
        ctl->tot_edges += tot[1];
        ctl->sweep += 1;
    }
    if (mode == FIN_DI || mode == FIN_DELIVER) ctl->parity ^= 1;
    int all = 1;
    for (int c = 0; c < k; ++c) all &= ctl->done[c];
    ctl->all_done = (all || ctl->overflow) ? 1 : 0;
}

__global__ void k_tile_begin(TileCtl *ctl, long long max_sweeps) {
    ctl->overflow = 0;
    ctl->all_done = 0;
    ctl->budget = ctl->sweep + max_sweeps;
}

// node-major tile -> column-major doubles, times an optional per-column scale
template <typename T>
__global__ void k_tile_to_colmajor(const T *__restrict__ src, i64 n, int k, const double *__restrict__ scale,
                                   double *out) {
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n * k; t += (i64)gridDim.x * blockDim.x) {
        const i64 c = t / n, i = t - c * n;
        const double v = (double)src[i * k + c];
        out[t] = scale ? v * scale[c] : v;
    }
}

static TileArgs tile_args(BatchState *b, const DevGraph &g, const SweepParams &p) {
    TileArgs a;
    a.out_ptr = g.out_ptr;
    a.out_idx = g.out_idx;
    a.w = g.w;
    a.in_ptr = g.in_ptr;
    a.in_idx = g.in_idx;
    a.in_w = g.in_w;
    a.inv_s = g.inv_s;
    a.F = b->F;
    a.H = b->H;
    a.snap = b->snap;
    a.ctl = b->ctl;
    a.partR = b->partR;
    a.partC = b->partC;
    a.partK = b->partK;
    a.n = b->n;
    a.k = b->k;
    a.K = b->K;
    a.d = p.d;
    return a;
}

static int launch_tile_reduce(BatchState *b, const TileArgs &a, int force, hipStream_t st) {
    if (b->fp32) k_tile_reduce<float><<<b->gridR, TILE_THREADS, 0, st>>>(a, force);
    else k_tile_reduce<double><<<b->gridR, TILE_THREADS, 0, st>>>(a, force);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// nR / nC / nK: residual, leak and counter slots written by the step just launched
static int launch_tile_finalize(BatchState *b, const SweepParams &p, int mode, int nR, int nC, int nK,
                                hipStream_t st) {
    TileFin f;
    f.ctl = b->ctl;
    f.partR = b->partR;
    f.partC = b->partC;
    f.nR = nR;
    f.nC = nC;
    f.k = b->k;
    f.K = b->K;
    f.mode = mode;
    f.d = p.d;
    f.theta = p.theta;
    f.tol = p.tol;
    f.n_d = (double)b->n;
    k_tile_finalize<<<b->k, 256, 0, st>>>(f);
    DI_LAUNCH_CHECK();
    k_tile_control<<<1, 256, 0, st>>>(b->ctl, b->partK, nK, b->k, mode);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

static TileBldArgs tile_bld_args(BatchState *b, const DevGraph &g, const SweepParams &p) {
    TileBldArgs a;
    a.loc_ptr = g.loc_ptr;
    a.loc_tgt = g.loc_tgt;
    a.loc_w = g.loc_w;
    a.rw = g.rw;
    a.deg_flags = g.deg_flags;
    a.inv_s = g.inv_s;
    a.blk_ptr = b->blk_ptr;
    a.rinfo = b->rinfo;
    a.n = b->n;
    a.rb = g.rb;
    a.k = b->k;
    a.K = b->K;
    a.rounds = b->rounds;
    a.F = b->F;
    a.H = b->H;
    a.S = b->S;
    a.fl = b->fl;
    a.ctl = b->ctl;
    a.d = p.d;
    a.partR = b->partR;
    a.partC = b->partC;
    a.partK = b->partK;
    return a;
}

// counters of the delivery go to partK slots gridB .. gridB + gridD - 1
static int launch_tile_deliver(BatchState *b, const DevGraph &g, hipStream_t st) {
    if (b->nunits == 0) return DI_OK;
    TileDlArgs a;
    a.units = b->units;
    a.nunits = b->nunits;
    a.rem_src = g.rem_src;
    a.rem_tgt = b->rem_tgt_abs;
    a.rem_w = g.rem_w;
    a.S = b->S;
    a.fl = b->fl;
    a.F = b->F;
    a.ctl = b->ctl;
    a.k = b->k;
    a.force = 0;
    a.partK = b->partK + (size_t)b->gridB * 2;
    if (b->fp32) {
        if (g.weighted) k_tile_deliver<float, true><<<b->gridD, DL_THREADS, 0, st>>>(a);
        else k_tile_deliver<float, false><<<b->gridD, DL_THREADS, 0, st>>>(a);
    } else {
        if (g.weighted) k_tile_deliver<double, true><<<b->gridD, DL_THREADS, 0, st>>>(a);
        else k_tile_deliver<double, false><<<b->gridD, DL_THREADS, 0, st>>>(a);
    }
    DI_LAUNCH_CHECK();
    return DI_OK;
}

static int launch_tile_bld(BatchState *b, const DevGraph &g, const SweepParams &p, hipStream_t st) {
    TileBldArgs a = tile_bld_args(b, g, p);
    const int T = b->fp32 ? 4 : 8;
    a.le_max = tile_le_max(g.rb, b->k, g.weighted);
    const size_t lds = tile_bld_lds_launch(g.rb, b->k, g.weighted);
    const int threads = ((1 << g.rb) / TB_RPW) * WAVE;
    if (b->fp32) {
        if (g.weighted) k_tile_bld<float, true><<<b->gridB, threads, lds, st>>>(a);
        else k_tile_bld<float, false><<<b->gridB, threads, lds, st>>>(a);
    } else {
        if (g.weighted) k_tile_bld<double, true><<<b->gridB, threads, lds, st>>>(a);
        else k_tile_bld<double, false><<<b->gridB, threads, lds, st>>>(a);
    }
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// the largest range size whose tiles let two workgroups share a compute unit, else the
// largest that fits one (the LDS tile is double for either fluid type)
int tile_range_log2(int k, int fp32, int weighted) {
    (void)fp32;
    for (int rb = TB_MAX_RB; rb >= TB_MIN_RB; --rb)
        if (tile_two_per_cu(rb, k, weighted != 0)) return rb;
    for (int rb = TB_MAX_RB; rb >= TB_MIN_RB; --rb)
        if (tile_le_max(rb, k, weighted != 0) >= 1024) return rb;
    return 0;
}

static int set_tile_attributes() {
    static bool done = false;
    if (done) return DI_OK;
    DI_HIP(hipFuncSetAttribute((const void *)k_tile_bld<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TB_LDS_ONE));
    DI_HIP(hipFuncSetAttribute((const void *)k_tile_bld<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TB_LDS_ONE));
    DI_HIP(hipFuncSetAttribute((const void *)k_tile_bld<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TB_LDS_ONE));
    DI_HIP(hipFuncSetAttribute((const void *)k_tile_bld<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TB_LDS_ONE));
    done = true;
    return DI_OK;
}

static int enqueue_tile_sweep(BatchState *b, const DevGraph &g, const SweepParams &p, hipStream_t st) {
    if (b->bld) {  // every sweep ends with its fluid delivered: nothing in flight between sweeps
        DI_TRY(launch_tile_bld(b, g, p, st));
        DI_TRY(launch_tile_deliver(b, g, st));
        return launch_tile_finalize(b, p, FIN_DI, b->gridB, b->gridB, b->gridB + b->gridD, st);
    }
    const TileArgs a = tile_args(b, g, p);
    if (b->det) {
        if (b->fp32) k_tile_snapshot<float><<<b->gridP, TILE_THREADS, 0, st>>>(a);
        else k_tile_snapshot<double><<<b->gridP, TILE_THREADS, 0, st>>>(a);
        DI_LAUNCH_CHECK();
        if (b->fp32) {
            if (g.weighted) k_tile_pull<float, true><<<b->gridP, TILE_THREADS, 0, st>>>(a);
            else k_tile_pull<float, false><<<b->gridP, TILE_THREADS, 0, st>>>(a);
        } else {
            if (g.weighted) k_tile_pull<double, true><<<b->gridP, TILE_THREADS, 0, st>>>(a);
            else k_tile_pull<double, false><<<b->gridP, TILE_THREADS, 0, st>>>(a);
        }
    } else {
        if (b->fp32) {
            if (g.weighted) k_tile_push<float, true><<<b->gridP, TILE_THREADS, 0, st>>>(a);
            else k_tile_push<float, false><<<b->gridP, TILE_THREADS, 0, st>>>(a);
        } else {
            if (g.weighted) k_tile_push<double, true><<<b->gridP, TILE_THREADS, 0, st>>>(a);
            else k_tile_push<double, false><<<b->gridP, TILE_THREADS, 0, st>>>(a);
        }
    }
    DI_LAUNCH_CHECK();
    DI_TRY(launch_tile_reduce(b, a, 0, st));
    return launch_tile_finalize(b, p, FIN_DI, b->gridR, b->gridP, b->gridP, st);
}

constexpr double REFINE_DROP = 0x1p-14;
// while the fluid is float, sweeps aim at REFINE_MARGIN * tol so that the residual of
// the recomputed fluid (the float pushes' rounding added back) still meets tol
constexpr double REFINE_MARGIN = 0.8;

// Recompute the fluid (see above), then every column's residual, stop and threshold
// under the tolerance in p.
static int refine_tile(BatchState *b, const DevGraph &g, const SweepParams &p, hipStream_t st) {
    const TileArgs a = tile_args(b, g, p);
    if (b->fp32) {
        if (g.weighted)
            k_tile_refine<float, true><<<b->gridP, TILE_THREADS, 0, st>>>(a, b->F0, b->seg_row, b->seg_p0, b->seg_p1,
                                                                       b->nseg, b->seg_part);
        else
            k_tile_refine<float, false><<<b->gridP, TILE_THREADS, 0, st>>>(a, b->F0, b->seg_row, b->seg_p0, b->seg_p1,
                                                                        b->nseg, b->seg_part);
    } else {
        if (g.weighted)
            k_tile_refine<double, true><<<b->gridP, TILE_THREADS, 0, st>>>(a, b->F0, b->seg_row, b->seg_p0, b->seg_p1,
                                                                        b->nseg, b->seg_part);
        else
            k_tile_refine<double, false><<<b->gridP, TILE_THREADS, 0, st>>>(a, b->F0, b->seg_row, b->seg_p0, b->seg_p1,
                                                                         b->nseg, b->seg_part);
    }
    DI_LAUNCH_CHECK();
    if (b->nlong > 0) {
        const int gl = (int)std::min<i64>(TILE_GRID, (b->nlong + TILE_WAVES - 1) / TILE_WAVES);
        if (b->fp32)
            k_tile_refine_long<float><<<gl, TILE_THREADS, 0, st>>>(a, b->F0, b->seg_row, b->long_first, b->nlong,
                                                                   b->seg_part);
        else
            k_tile_refine_long<double><<<gl, TILE_THREADS, 0, st>>>(a, b->F0, b->seg_row, b->long_first, b->nlong,
                                                                    b->seg_part);
        DI_LAUNCH_CHECK();
    }
    DI_TRY(launch_tile_reduce(b, a, 1, st));
    return launch_tile_finalize(b, p, FIN_INIT, b->gridR, 0, 0, st);
}

int batch_K(const BatchState *b) { return b ? b->K : 0; }

void set_batch_rounds(BatchState *b, int rounds) {
    b->rounds = rounds;
    if (b->gexec) {  // a captured chunk holds the old launch arguments
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
}

void free_batch(BatchState *b) {
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->cap_st) (void)hipStreamDestroy(b->cap_st);
    void *ps[] = {b->F,   b->F0,      b->H,         b->snap,  b->ctl,         b->partR,
                  b->partC, b->partK, b->S,       b->fl,        b->blk_ptr,
                  b->units, b->rem_tgt_abs, b->partH, b->hsum, b->rinfo, b->seg_row, b->seg_p0, b->seg_p1,
                  b->long_first, b->seg_part};
    for (void *q : ps)
        if (q) (void)dev_free(q);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

// F_0 = (1-d) Z_c per column, node-major, kept in double (the fluid starts from it
// rounded to the fluid type); one fixed-point scale for all columns, set by the
// largest starting entry.  Uploads F_0 and sets b->K, b->zsum.
static int load_batch_z(BatchState *b, const SweepParams &p, const double *Z) {
    const i64 n = b->n;
    const int k = b->k;
    std::vector<double> f0((size_t)(n * k));
    double mx = 0.0;
    for (int c = 0; c < k; ++c) {
        HostSum zs;
        for (i64 i = 0; i < n; ++i) {
            const double z = Z ? Z[(i64)c * n + i] : 1.0 / (double)n;
            zs.add(z);
            const double v = (1.0 - p.d) * z;
            f0[(size_t)(i * k + c)] = v;
            mx = std::max(mx, std::fabs(p.fp32 ? (double)(float)v : v));
        }
        b->zsum[c] = zs.value();
    }
    int e_max = 0;
    if (mx > 0.0) std::frexp(mx, &e_max);
    int e_n = 0;
    while (((i64)1 << e_n) < n) ++e_n;
    b->K = 118 - (e_max + e_n);
    DI_HIP(hipMemcpy(b->F0, f0.data(), n * k * 8, hipMemcpyHostToDevice));
    return DI_OK;
}

int set_batch_z(BatchState *b, const DevGraph &g, SweepParams &p, const double *Z, hipStream_t st) {
    DI_TRY(load_batch_z(b, p, Z));
    p.K = b->K;
    if (b->gexec) {  // a captured chunk holds the old scale
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return reset_batch(b, g, p, st);
}

// Longest-processing-time assignment of ranges to the block-local workgroups; a range's
// work is its cross-range entries, local edges and rows.
static int assign_ranges(BatchState *b, const DevGraph &g) {
    const i64 nr = g.nranges;
    std::vector<i64> rbase(nr + 1), lbase(nr + 1);
    DI_HIP(hipMemcpy(rbase.data(), g.rem_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost));
    DI_HIP(hipMemcpy(lbase.data(), g.loc_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost));
    std::vector<i64> work((size_t)nr);
    for (i64 r = 0; r < nr; ++r) {
        const i64 rows = std::min<i64>((i64)1 << g.rb, g.n - (r << g.rb));
        work[r] = (rbase[r + 1] - rbase[r]) + (lbase[r + 1] - lbase[r]) + 2 * rows;
    }
    std::vector<int> order((size_t)nr);
    for (i64 r = 0; r < nr; ++r) order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    const int G = b->gridB;
    std::vector<std::pair<i64, int>> heap;  // (load, block), smallest load on top
    for (int q = 0; q < G; ++q) heap.emplace_back(0, q);
    auto cmp = [](const std::pair<i64, int> &x, const std::pair<i64, int> &y) {
        return x.first != y.first ? x.first > y.first : x.second > y.second;
    };
    std::make_heap(heap.begin(), heap.end(), cmp);
    std::vector<std::vector<int>> lists((size_t)G);
    for (int r : order) {
        std::pop_heap(heap.begin(), heap.end(), cmp);
        auto &top = heap.back();
        lists[top.second].push_back(r);
        top.first += work[r];
        std::push_heap(heap.begin(), heap.end(), cmp);
    }
    std::vector<int> ptr((size_t)G + 1, 0), flat;
    flat.reserve((size_t)nr);
    for (int q = 0; q < G; ++q) {
        flat.insert(flat.end(), lists[q].begin(), lists[q].end());
        ptr[q + 1] = (int)flat.size();
    }
    DI_HIP(hipMemcpy(b->blk_ptr, ptr.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice));
    std::vector<TileRange> info((size_t)nr);
    for (i64 q = 0; q < nr; ++q) {
        const i64 r = flat[q], base = r << g.rb;
        info[q] = TileRange{base, lbase[r], (int)std::min<i64>((i64)1 << g.rb, g.n - base),
                            (int)(lbase[r + 1] - lbase[r])};
    }
    DI_HIP(hipMemcpy(b->rinfo, info.data(), sizeof(TileRange) * nr, hipMemcpyHostToDevice));
    return DI_OK;
}

// Delivery units: the cross-range in-entries (grouped by target range, sorted by target
// within it) are cut into units of at most DL_UNIT entries holding whole target rows;
// a row with more entries gets units of its own, marked split.
static int build_delivery_units(BatchState *b, const DevGraph &g) {
    const i64 nr = g.nranges, mr = g.m_rem;
    if (mr == 0) return DI_OK;
    std::vector<i64> rbase(nr + 1);
    std::vector<unsigned short> rt((size_t)mr);
    DI_HIP(hipMemcpy(rbase.data(), g.rem_base, sizeof(i64) * (nr + 1), hipMemcpyDeviceToHost));
    DI_HIP(hipMemcpy(rt.data(), g.rem_tgt, sizeof(unsigned short) * mr, hipMemcpyDeviceToHost));
    std::vector<int> tabs((size_t)mr);
    for (i64 r = 0; r < nr; ++r)
        for (i64 p = rbase[r]; p < rbase[r + 1]; ++p) tabs[p] = (int)((r << g.rb) + rt[p]);
    std::vector<DlUnit> units;
    DlUnit cur{0, 0, 0};
    for (i64 p = 0; p < mr;) {
        i64 q = p + 1;
        while (q < mr && tabs[q] == tabs[p]) ++q;
        const i64 cnt = q - p;
        if (cnt > DL_UNIT) {
            if (cur.len) units.push_back(cur);
            for (i64 e = p; e < q; e += DL_UNIT) units.push_back(DlUnit{e, (int)std::min<i64>(DL_UNIT, q - e), 1});
            cur = DlUnit{q, 0, 0};
        } else {
            if (cur.len + cnt > DL_UNIT) {
                units.push_back(cur);
                cur = DlUnit{p, 0, 0};
            }
            if (cur.len == 0) cur.e0 = p;
            cur.len += (int)cnt;
        }
        p = q;
    }
    if (cur.len) units.push_back(cur);
    b->nunits = (i64)units.size();
    b->gridD = (int)std::min<i64>(DL_GRID, (b->nunits + DL_WAVES - 1) / DL_WAVES);
    if (dev_malloc((void **)&b->units, sizeof(DlUnit) * units.size()) != hipSuccess ||
        dev_malloc((void **)&b->rem_tgt_abs, sizeof(int) * mr) != hipSuccess) {
        set_error("device allocation of the delivery units failed");
        return DI_ENOMEM;
    }
    DI_HIP(hipMemcpy(b->units, units.data(), sizeof(DlUnit) * units.size(), hipMemcpyHostToDevice));
    DI_HIP(hipMemcpy(b->rem_tgt_abs, tabs.data(), sizeof(int) * mr, hipMemcpyHostToDevice));
    return DI_OK;
}

// The recomputation's segments of the IN rows longer than REFINE_SEG entries.
static int build_refine_segments(BatchState *b, const DevGraph &g) {
    const i64 n = b->n;
    std::vector<i64> ip((size_t)n + 1);
    DI_HIP(hipMemcpy(ip.data(), g.in_ptr, sizeof(i64) * (n + 1), hipMemcpyDeviceToHost));
    std::vector<int> srow, lfirst;
    std::vector<i64> sp0, sp1;
    for (i64 j = 0; j < n; ++j) {
        if (ip[j + 1] - ip[j] <= REFINE_SEG) continue;
        lfirst.push_back((int)srow.size());
        for (i64 q = ip[j]; q < ip[j + 1]; q += REFINE_SEG) {
            srow.push_back((int)j);
            sp0.push_back(q);
            sp1.push_back(std::min<i64>(q + REFINE_SEG, ip[j + 1]));
        }
    }
    b->nseg = (i64)srow.size();
    b->nlong = (i64)lfirst.size();
    lfirst.push_back((int)srow.size());
    if (b->nseg == 0) return DI_OK;
    if (dev_malloc((void **)&b->seg_row, sizeof(int) * srow.size()) != hipSuccess ||
        dev_malloc((void **)&b->seg_p0, 8 * sp0.size()) != hipSuccess ||
        dev_malloc((void **)&b->seg_p1, 8 * sp1.size()) != hipSuccess ||
        dev_malloc((void **)&b->long_first, 4 * lfirst.size()) != hipSuccess ||
        dev_malloc((void **)&b->seg_part, 8 * (size_t)KMAX * srow.size()) != hipSuccess) {
        set_error("device allocation of the recomputation segments failed");
        return DI_ENOMEM;
    }
    DI_HIP(hipMemcpy(b->seg_row, srow.data(), sizeof(int) * srow.size(), hipMemcpyHostToDevice));
    DI_HIP(hipMemcpy(b->seg_p0, sp0.data(), 8 * sp0.size(), hipMemcpyHostToDevice));
    DI_HIP(hipMemcpy(b->seg_p1, sp1.data(), 8 * sp1.size(), hipMemcpyHostToDevice));
    DI_HIP(hipMemcpy(b->long_first, lfirst.data(), 4 * lfirst.size(), hipMemcpyHostToDevice));
    return DI_OK;
}

int init_batch(BatchState *&bout, const DevGraph &g, SweepParams &p, int k, int det, const double *Z,
               const int *range_order, int rounds, hipStream_t st) {
    bout = nullptr;
    if (k < 1 || k > KMAX) {
        set_error("k must be in 1..%d", KMAX);
        return DI_EINVAL;
    }
    BatchState *b = new (std::nothrow) BatchState();
    if (!b) {
        set_error("host allocation failed");
        return DI_ENOMEM;
    }
    const i64 n = g.n;
    b->k = k;
    b->n = n;
    b->fp32 = p.fp32;
    b->det = det;
    const size_t T = p.fp32 ? 4 : 8;
    b->gridP = (int)std::min<i64>(TILE_GRID, (n + TILE_WAVES - 1) / TILE_WAVES);
    b->gridR = (int)std::min<i64>(REDUCE_TILE_GRID, (n + TILE_WAVES - 1) / TILE_WAVES);
    // fast sweeps are block-local when a range's fluid and dH tiles fit in LDS
    b->bld = !det && tile_le_max(g.rb, k, g.weighted) > 0;
    b->rounds = rounds > 0 ? rounds : 4;
    (void)range_order;
    if (b->bld) {
        // one resident workgroup per compute unit and LDS share (two when the tiles fit
        // TB_LDS); ranges are dealt out longest first, each to the least loaded workgroup
        int cus = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        const int per_cu = tile_two_per_cu(g.rb, k, g.weighted) ? 2 : 1;
        b->gridB = (int)std::min<i64>(std::min<i64>((i64)cus * per_cu, TB_GRID), g.nranges);
    }
    const size_t slots = (size_t)std::max(std::max(b->gridR, b->gridP), b->gridB + DL_GRID);
    auto fail = [&](int code) {
        free_batch(b);
        return code;
    };
    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (dev_malloc(ptr, bytes) == hipSuccess) return true;
        set_error("device allocation of %zu bytes failed", bytes);
        return false;
    };
    if (!alloc(&b->F, n * k * T) || !alloc((void **)&b->F0, n * k * 8) || !alloc((void **)&b->H, n * k * 8) ||
        !alloc((void **)&b->ctl, sizeof(TileCtl)) || !alloc((void **)&b->partR, slots * KMAX * PSR * 8) ||
        !alloc((void **)&b->partC, slots * KMAX * 4 * 8) || !alloc((void **)&b->partK, slots * 2 * 8) ||
        !alloc((void **)&b->partH, (size_t)b->gridR * KMAX * 4 * 8) || !alloc((void **)&b->hsum, 2 * KMAX * 8) ||
        (det && !alloc((void **)&b->snap, n * k * 8)))
        return fail(DI_ENOMEM);
    if (p.fp32 && !det) {
        const int src = build_refine_segments(b, g);
        if (src != DI_OK) return fail(src);
    }
    if (b->bld) {
        if (!alloc(&b->S, n * k * T) || !alloc((void **)&b->fl, (size_t)((n + 31) / 32) * 4) ||
            !alloc((void **)&b->blk_ptr, (size_t)(b->gridB + 1) * 4) ||
            !alloc((void **)&b->rinfo, (size_t)g.nranges * sizeof(TileRange)))
            return fail(DI_ENOMEM);
        int src = assign_ranges(b, g);
        if (src == DI_OK) src = build_delivery_units(b, g);
        if (src != DI_OK) return fail(src);
        const int arc = set_tile_attributes();
        if (arc != DI_OK) return fail(arc);
    }
    if (hipHostMalloc((void **)&b->h_ctl, sizeof(TileCtl), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return fail(DI_ENOMEM);
    }
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        set_error("hipEventCreate failed");
        return fail(DI_EHIP);
    }
    const int zrc = load_batch_z(b, p, Z);
    if (zrc != DI_OK) return fail(zrc);
    p.K = b->K;
    const int rc = reset_batch(b, g, p, st);
    if (rc != DI_OK) return fail(rc);
    bout = b;
    return DI_OK;
}

int reset_batch(BatchState *b, const DevGraph &g, const SweepParams &p, hipStream_t st) {
    DI_TRY(launch_init_fluid(b->F0, b->F, b->fp32, b->n * b->k, st));
    DI_TRY(launch_fill_zero(b->H, b->n * b->k * 8, st));
    DI_TRY(launch_fill_zero(b->ctl, sizeof(TileCtl), st));
    if (b->bld) DI_TRY(launch_fill_zero(b->fl, ((b->n + 31) / 32) * 4, st));
    DI_TRY(launch_tile_reduce(b, tile_args(b, g, p), 1, st));
    DI_TRY(launch_tile_finalize(b, p, FIN_INIT, b->gridR, 0, 0, st));
    DI_HIP(hipStreamSynchronize(st));
    return DI_OK;
}

static int sync_tile(BatchState *b, hipStream_t st) {
    DI_HIP(hipMemcpyAsync(b->h_ctl, b->ctl, sizeof(TileCtl), hipMemcpyDeviceToHost, st));
    DI_HIP(hipStreamSynchronize(st));
    return DI_OK;
}

// spc sweeps, launched directly or through a captured graph (loop_mode = graph)
static int enqueue_tile_chunk(BatchState *b, const DevGraph &g, const SweepParams &p, int spc, int graph_mode,
                              hipStream_t st) {
    if (!graph_mode) {
        for (int s = 0; s < spc; ++s) DI_TRY(enqueue_tile_sweep(b, g, p, st));
        return DI_OK;
    }
    if (!b->gexec || b->gexec_spc != spc || b->gexec_tol != p.tol || b->gexec_theta != p.theta) {
        if (b->gexec) {
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
        }
        if (!b->cap_st) DI_HIP(hipStreamCreateWithFlags(&b->cap_st, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        DI_HIP(hipStreamBeginCapture(b->cap_st, hipStreamCaptureModeThreadLocal));
        int rc = DI_OK;
        for (int s = 0; s < spc && rc == DI_OK; ++s) rc = enqueue_tile_sweep(b, g, p, b->cap_st);
        const hipError_t e = hipStreamEndCapture(b->cap_st, &graph);
        if (rc != DI_OK) return rc;
        if (e != hipSuccess) {
            set_error("hipStreamEndCapture: %s", hipGetErrorString(e));
            return DI_EHIP;
        }
        const hipError_t e2 = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            set_error("hipGraphInstantiate: %s", hipGetErrorString(e2));
            return DI_EHIP;
        }
        b->gexec_spc = spc;
        b->gexec_tol = p.tol;
        b->gexec_theta = p.theta;
    }
    DI_HIP(hipGraphLaunch(b->gexec, st));
    return DI_OK;
}

int diffuse_batch(BatchState *b, const DevGraph &g, const SweepParams &p, const di_opts &o, int spc,
                  hipStream_t st, di_stats *stats) {
    DI_HIP(hipEventRecord(b->ev0, st));
    // state of every column under this call's tolerance
    k_tile_begin<<<1, 1, 0, st>>>(b->ctl, (long long)o.max_sweeps);
    DI_LAUNCH_CHECK();
    DI_TRY(launch_tile_reduce(b, tile_args(b, g, p), 1, st));
    DI_TRY(launch_tile_finalize(b, p, FIN_INIT, b->gridR, 0, 0, st));
    DI_TRY(sync_tile(b, st));
    const TileCtl before = *b->h_ctl;
    auto max_R = [&](const TileCtl &h) {
        double r = 0.0;
        for (int c = 0; c < b->k; ++c) r = std::max(r, h.R[c]);
        return r;
    };
    const bool refine = b->fp32 && !b->det;
    double R_ref = max_R(before);
    SweepParams ps = p;  // the sweeps' tolerance
    if (refine) ps.tol = p.tol * REFINE_MARGIN;
    while (!b->h_ctl->all_done) {
        DI_TRY(enqueue_tile_chunk(b, g, ps, spc, o.loop_mode == DI_LOOP_GRAPH, st));
        DI_TRY(sync_tile(b, st));
        const TileCtl &h = *b->h_ctl;
        if (h.overflow) break;
        if (refine && (h.all_done || max_R(h) <= R_ref * REFINE_DROP)) {
            DI_TRY(refine_tile(b, g, p, st));
            DI_TRY(sync_tile(b, st));
            R_ref = max_R(*b->h_ctl);
            if (b->h_ctl->all_done || b->h_ctl->overflow) break;
        } else if (h.all_done) {
            break;
        }
        if (b->h_ctl->sweep >= b->h_ctl->budget) break;
    }
    DI_HIP(hipEventRecord(b->ev1, st));
    DI_TRY(sync_tile(b, st));
    float ms = 0.0f;
    DI_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    const TileCtl &h = *b->h_ctl;
    int all = 1;
    for (int c = 0; c < b->k; ++c) all &= h.done[c];
    if (stats) {
        stats->sweeps = h.sweep - before.sweep;
        stats->edge_updates = (int64_t)(h.tot_edges - before.tot_edges);
        stats->node_updates = (int64_t)(h.tot_nodes - before.tot_nodes);
        double rmax = 0.0, lsum = 0.0, bn = 0.0;
        for (int c = 0; c < b->k; ++c) {
            rmax = std::max(rmax, h.R[c]);
            const double l = limbs_to_double_signed(h.limbsL[c][0], h.limbsL[c][1], h.limbsL[c][2], h.limbsL[c][3], b->K);
            lsum += l;
            bn = std::max(bn, h.R[c] / (1.0 - p.d - p.d * l / b->zsum[c]));
        }
        stats->residual = rmax;
        stats->bound = rmax / (1.0 - p.d);
        stats->bound_norm = bn;
        stats->leak = lsum;
        stats->ms = ms;
        stats->mass_defect = 0.0;
        stats->converged = all && !h.overflow;
    }
    if (h.overflow) {
        set_error("non-finite or out-of-range fluid in the residual");
        return DI_ENUMERIC;
    }
    if (!all) {
        set_error("sweep budget spent before every column met the tolerance");
        return DI_ENOCONV;
    }
    return DI_OK;
}

// Exact signed per-column sums of an n x k node-major double or float tile into
// per-workgroup slots part[block][column][0..3].
template <typename T>
__global__ void __launch_bounds__(TILE_THREADS) k_tile_sum_signed(const T *__restrict__ v, i64 n, int k, int K,
                                                                  u64 *part) {
    __shared__ u64 lds[TILE_WAVES * WAVE * 4];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    Limbs S;
    limbs_zero(S);
    if (lane < k) {
        const i64 nwaves = (i64)gridDim.x * TILE_WAVES;
        for (i64 i = (i64)blockIdx.x * TILE_WAVES + w; i < n; i += nwaves) limbs_add_signed(S, (double)v[i * k + lane], K);
    }
    u64 q[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
    block_columns_store<4>(q, lds, part + (i64)blockIdx.x * KMAX * 4, k);
}

// One workgroup per column: add the column's limb slots of k_tile_sum_signed.
__global__ void __launch_bounds__(256) k_tile_colsum(const u64 *__restrict__ part, int nslots, int K, double *out) {
    __shared__ u64 red[4 * 4];
    __shared__ u64 tot[4];
    const int c = blockIdx.x;
    u64 v[4] = {0, 0, 0, 0};
    for (int q = threadIdx.x; q < nslots; q += blockDim.x)
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] += part[((i64)q * KMAX + c) * 4 + t];
    block_store_partials<4>(v, red, tot);
    if (threadIdx.x == 0) out[c] = limbs_to_double_signed(tot[0], tot[1], tot[2], tot[3], K);
}

int batch_mass_defects(BatchState *b, const DevGraph &g, const SweepParams &p, double *out, hipStream_t st) {
    // the history and fluid sums of a column stay within a few times |Z_c|_1
    // (x = (1-d)(I-dP)^{-1} Z_c and |P|_1 <= 1)
    double zmax = 0.0;
    for (int c = 0; c < b->k; ++c) zmax = std::max(zmax, b->zsum[c]);
    int e_max = 0, e_n = 0;
    std::frexp(8.0 * zmax, &e_max);
    while (((i64)1 << e_n) < b->n) ++e_n;
    const int KH = 118 - (e_max + e_n);
    const unsigned grid = (unsigned)b->gridR;
    k_tile_sum_signed<double><<<grid, TILE_THREADS, 0, st>>>(b->H, b->n, b->k, KH, b->partH);
    DI_LAUNCH_CHECK();
    k_tile_colsum<<<b->k, 256, 0, st>>>(b->partH, b->gridR, KH, b->hsum);
    DI_LAUNCH_CHECK();
    if (b->fp32) k_tile_sum_signed<float><<<grid, TILE_THREADS, 0, st>>>((const float *)b->F, b->n, b->k, KH, b->partH);
    else k_tile_sum_signed<double><<<grid, TILE_THREADS, 0, st>>>((const double *)b->F, b->n, b->k, KH, b->partH);
    DI_LAUNCH_CHECK();
    k_tile_colsum<<<b->k, 256, 0, st>>>(b->partH, b->gridR, KH, b->hsum + KMAX);
    DI_LAUNCH_CHECK();
    std::vector<double> hs((size_t)(2 * KMAX));
    DI_HIP(hipMemcpyAsync(hs.data(), b->hsum, sizeof(double) * 2 * KMAX, hipMemcpyDeviceToHost, st));
    DI_TRY(sync_tile(b, st));
    const TileCtl &h = *b->h_ctl;
    for (int c = 0; c < b->k; ++c) {
        const double l = limbs_to_double_signed(h.limbsL[c][0], h.limbsL[c][1], h.limbsL[c][2], h.limbsL[c][3], b->K);
        out[c] = hs[KMAX + c] + (1.0 - p.d) * hs[c] + p.d * l - (1.0 - p.d) * b->zsum[c];
    }
    return DI_OK;
}

int read_batch(BatchState *b, const DevGraph &g, const SweepParams &p, int what, void *dst, int on_device,
               hipStream_t st) {
    (void)g;
    const i64 n = b->n;
    const int k = b->k;
    auto small = [&](const void *src, size_t bytes) -> int {
        if (on_device) DI_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
        else std::memcpy(dst, src, bytes);
        return DI_OK;
    };
    if (what == DI_RESIDUALS || what == DI_LEAKS || what == DI_DONE_SWEEPS) {
        DI_TRY(sync_tile(b, st));
        const TileCtl &h = *b->h_ctl;
        if (what == DI_DONE_SWEEPS) {
            std::vector<int64_t> v((size_t)k);
            for (int c = 0; c < k; ++c) v[c] = h.done[c] ? (int64_t)h.done_sweep[c] : -1;
            return small(v.data(), sizeof(int64_t) * k);
        }
        std::vector<double> v((size_t)k);
        for (int c = 0; c < k; ++c)
            v[c] = what == DI_RESIDUALS
                       ? h.R[c]
                       : limbs_to_double_signed(h.limbsL[c][0], h.limbsL[c][1], h.limbsL[c][2], h.limbsL[c][3], b->K);
        return small(v.data(), sizeof(double) * k);
    }
    if (what != DI_X_RAW && what != DI_H && what != DI_F && what != DI_X_NORM) {
        set_error("read target %d is not available with k > 1", what);
        return DI_EINVAL;
    }
    double *scale = nullptr, *out = (double *)dst;
    if (what == DI_X_NORM) {  // completion by Z_c / |Z_c|_1 per column (Section 3.3)
        DI_TRY(sync_tile(b, st));
        const TileCtl &h = *b->h_ctl;
        std::vector<double> sc((size_t)k);
        for (int c = 0; c < k; ++c) {
            const double l = limbs_to_double_signed(h.limbsL[c][0], h.limbsL[c][1], h.limbsL[c][2], h.limbsL[c][3], b->K);
            sc[c] = (1.0 - p.d) / (1.0 - p.d - p.d * l / b->zsum[c]);
        }
        DI_HIP(dev_malloc((void **)&scale, sizeof(double) * k));
        if (hipMemcpy(scale, sc.data(), sizeof(double) * k, hipMemcpyHostToDevice) != hipSuccess) {
            (void)dev_free(scale);
            set_error("upload of the completion scales failed");
            return DI_EHIP;
        }
    }
    hipError_t e = hipSuccess;
    if (!on_device) e = dev_malloc((void **)&out, sizeof(double) * std::max<i64>(n * k, 1));
    if (e == hipSuccess) {
        const unsigned grid = grid_for(n * k, 256, 16384);
        if (what == DI_F && b->fp32) k_tile_to_colmajor<float><<<grid, 256, 0, st>>>((const float *)b->F, n, k, nullptr, out);
        else if (what == DI_F) k_tile_to_colmajor<double><<<grid, 256, 0, st>>>((const double *)b->F, n, k, nullptr, out);
        else k_tile_to_colmajor<double><<<grid, 256, 0, st>>>(b->H, n, k, scale, out);
        e = hipGetLastError();
        if (e == hipSuccess && !on_device) e = hipMemcpyAsync(dst, out, sizeof(double) * n * k, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (!on_device) (void)dev_free(out);
    }
    if (scale) (void)dev_free(scale);
    if (e != hipSuccess) {
        set_error("batched read failed: %s", hipGetErrorString(e));
        return DI_EHIP;
    }
    return DI_OK;
}

i64 batch_sweeps(BatchState *b, hipStream_t st) {
    if (sync_tile(b, st) != DI_OK) return -1;
    return b->h_ctl->sweep;
}

}  // namespace di
