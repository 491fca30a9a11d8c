// Graph construction on the device: prefix sums, a stable LSD radix sort, the IN
// adjacency (transpose of the input OUT adjacency), 1/s_j, and the block-local /
// cross-range edge split used by the D-Iteration sweep.
#include "graph.h"

#include <algorithm>
#include <vector>

namespace di {

// ---------------------------------------------------------------------------
// Exclusive prefix sum of int64 (three-phase: tile scans, scan of tile totals,
// offset add).  In place allowed.  out[count] is NOT written; totals via tile sums.
// ---------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ i64 wave_incl_scan_i64(i64 v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        i64 t = __shfl_up(v, o, WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive prefix,
// writes the block total into *total.
__device__ __forceinline__ i64 block_excl_scan_i64(i64 v, i64 *lds /* [nwaves] */, i64 *total) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    i64 inc = wave_incl_scan_i64(v);
    if (lane == WAVE - 1) lds[w] = inc;
    __syncthreads();
    i64 before = 0, all = 0;
    for (int q = 0; q < nw; ++q) {
        i64 s = lds[q];
        if (q < w) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tiles(const i64 *__restrict__ in, i64 *out, i64 *tile_sums,
                                                             i64 count) {
    __shared__ i64 lds[SCAN_THREADS / WAVE];
    const i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    i64 v[SCAN_ITEMS];
    i64 s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        i64 idx = base + k;
        v[k] = idx < count ? in[idx] : 0;
        s += v[k];
    }
    i64 total;
    i64 run = block_excl_scan_i64(s, lds, &total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        i64 idx = base + k;
        if (idx < count) out[idx] = run;
        run += v[k];
    }
    if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(i64 *out, const i64 *__restrict__ offs, i64 count) {
    const i64 idx = (i64)blockIdx.x * SCAN_TILE + threadIdx.x;
    const i64 add = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        i64 p = idx + (i64)k * SCAN_THREADS;
        if (p < count) out[p] += add;
    }
}

i64 scan_temp_elems(i64 count) {
    i64 tot = 0;
    while (count > SCAN_TILE) {
        count = (count + SCAN_TILE - 1) / SCAN_TILE;
        tot += count + 1;
    }
    return tot + 1;
}

int scan_exclusive(const i64 *in, i64 *out, i64 count, i64 *temp, hipStream_t st) {
    if (count <= 0) return DI_OK;
    const i64 tiles = (count + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        k_scan_tiles<<<1, SCAN_THREADS, 0, st>>>(in, out, nullptr, count);
        DI_LAUNCH_CHECK();
        return DI_OK;
    }
    i64 *sums = temp;
    k_scan_tiles<<<(unsigned)tiles, SCAN_THREADS, 0, st>>>(in, out, sums, count);
    DI_LAUNCH_CHECK();
    DI_TRY(scan_exclusive(sums, sums, tiles, temp + tiles + 1, st));
    k_scan_add<<<(unsigned)tiles, SCAN_THREADS, 0, st>>>(out, sums, count);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint32 key, value) pairs, 4-bit digits.
// Each tile of RS_TILE consecutive items is ranked in a blocked arrangement
// (thread t owns items t*RS_ITEMS ..), so equal digits keep their input order.
// Per-thread digit counts are packed as sixteen 16-bit fields in eight words.
// ---------------------------------------------------------------------------
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_BITS = 4;
constexpr int RS_DIGITS = 1 << RS_BITS;

__device__ __forceinline__ unsigned packed_get(const unsigned (&c)[8], unsigned dgt) {
    return (c[dgt >> 1] >> ((dgt & 1) * 16)) & 0xffffu;
}

// Block-wide exclusive scan of packed counters (fields stay below 2^16 since a tile
// has 4096 items).  Returns per-thread exclusive prefixes and the block totals.
__device__ __forceinline__ void block_scan_packed(unsigned (&c)[8], unsigned (&excl)[8], unsigned (&tot)[8],
                                                  unsigned *lds /* [nwaves*8] */) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned inc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        unsigned v = c[q];
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            unsigned t = __shfl_up(v, o, WAVE);
            if (lane >= o) v += t;
        }
        inc[q] = v;
        if (lane == WAVE - 1) lds[w * 8 + q] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        unsigned before = 0, all = 0;
        for (int p = 0; p < nw; ++p) {
            unsigned s = lds[p * 8 + q];
            if (p < w) before += s;
            all += s;
        }
        excl[q] = before + inc[q] - c[q];
        tot[q] = all;
    }
    __syncthreads();
}

template <typename V>
__global__ void __launch_bounds__(RS_THREADS) k_radix_upsweep(const unsigned *__restrict__ keys, i64 count, int shift,
                                                              i64 *__restrict__ counts, i64 ntiles) {
    __shared__ unsigned lds[(RS_THREADS / WAVE) * 8];
    const i64 base = (i64)blockIdx.x * RS_TILE + (i64)threadIdx.x * RS_ITEMS;
    unsigned c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        i64 idx = base + k;
        if (idx < count) {
            unsigned dg = (keys[idx] >> shift) & (RS_DIGITS - 1);
            c[dg >> 1] += 1u << ((dg & 1) * 16);
        }
    }
    unsigned excl[8], tot[8];
    block_scan_packed(c, excl, tot, lds);
    if (threadIdx.x < RS_DIGITS) counts[(i64)threadIdx.x * ntiles + blockIdx.x] = packed_get(tot, threadIdx.x);
}

template <typename V>
__global__ void __launch_bounds__(RS_THREADS) k_radix_downsweep(const unsigned *__restrict__ keys_in,
                                                                const V *__restrict__ vals_in, unsigned *keys_out,
                                                                V *vals_out, i64 count, int shift,
                                                                const i64 *__restrict__ offsets, i64 ntiles) {
    __shared__ unsigned lds[(RS_THREADS / WAVE) * 8];
    const i64 base = (i64)blockIdx.x * RS_TILE + (i64)threadIdx.x * RS_ITEMS;
    unsigned key[RS_ITEMS];
    unsigned c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned loc[RS_ITEMS];
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        i64 idx = base + k;
        key[k] = idx < count ? keys_in[idx] : 0u;
        if (idx < count) {
            unsigned dg = (key[k] >> shift) & (RS_DIGITS - 1);
            loc[k] = packed_get(c, dg);
            c[dg >> 1] += 1u << ((dg & 1) * 16);
        }
    }
    unsigned excl[8], tot[8];
    block_scan_packed(c, excl, tot, lds);
    __shared__ i64 gbase[RS_DIGITS];
    if (threadIdx.x < RS_DIGITS) gbase[threadIdx.x] = offsets[(i64)threadIdx.x * ntiles + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        i64 idx = base + k;
        if (idx < count) {
            unsigned dg = (key[k] >> shift) & (RS_DIGITS - 1);
            i64 pos = gbase[dg] + packed_get(excl, dg) + loc[k];
            keys_out[pos] = key[k];
            vals_out[pos] = vals_in[idx];
        }
    }
}

template <typename V>
int radix_sort_pairs(unsigned *keys, V *vals, unsigned *keys_tmp, V *vals_tmp, i64 count, int key_bits, i64 *counts,
                     i64 *scan_temp, hipStream_t st, bool *result_in_tmp) {
    *result_in_tmp = false;
    if (count <= 1 || key_bits <= 0) return DI_OK;
    const i64 ntiles = (count + RS_TILE - 1) / RS_TILE;
    unsigned *ka = keys, *kb = keys_tmp;
    V *va = vals, *vb = vals_tmp;
    for (int shift = 0; shift < key_bits; shift += RS_BITS) {
        k_radix_upsweep<V><<<(unsigned)ntiles, RS_THREADS, 0, st>>>(ka, count, shift, counts, ntiles);
        DI_LAUNCH_CHECK();
        DI_TRY(scan_exclusive(counts, counts, ntiles * RS_DIGITS, scan_temp, st));
        k_radix_downsweep<V><<<(unsigned)ntiles, RS_THREADS, 0, st>>>(ka, va, kb, vb, count, shift, counts, ntiles);
        DI_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
        *result_in_tmp = !*result_in_tmp;
    }
    return DI_OK;
}

i64 radix_counts_elems(i64 count) { return ((count + RS_TILE - 1) / RS_TILE) * RS_DIGITS + 1; }

// ---------------------------------------------------------------------------
// IN adjacency.
// ---------------------------------------------------------------------------
__global__ void k_expand_sources(const i64 *__restrict__ out_ptr, const int *__restrict__ out_idx,
                                 const float *__restrict__ w, i64 n, unsigned *keys, u64 *vals) {
    i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (i64 e = out_ptr[j]; e < out_ptr[j + 1]; ++e) {
        keys[e] = (unsigned)out_idx[e];
        u64 wb = w ? (u64)__float_as_uint(w[e]) : 0ull;
        vals[e] = (u64)(unsigned)j | (wb << 32);
    }
}

__global__ void k_fill_i64(i64 *p, i64 v, i64 count) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// in_ptr[t] = first position p with key[p] >= t (keys sorted ascending); positions
// beyond the last key keep the prefilled value m.
__global__ void k_row_ptr_from_keys(const unsigned *__restrict__ keys, i64 m, i64 *in_ptr) {
    i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    i64 k = keys[p];
    i64 prev = p ? (i64)keys[p - 1] : -1;
    for (i64 t = prev + 1; t <= k; ++t) in_ptr[t] = p;
}

__global__ void k_unpack_in(const u64 *__restrict__ vals, i64 m, int *in_idx, float *in_w) {
    i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    u64 v = vals[p];
    in_idx[p] = (int)(unsigned)(v & 0xffffffffull);
    if (in_w) in_w[p] = __uint_as_float((unsigned)(v >> 32));
}

// 1 / s_j, s_j = out-degree or the left-to-right double sum of out-weights; 0 if dangling.
__global__ void k_inv_s(const i64 *__restrict__ out_ptr, const float *__restrict__ w, i64 n, double *inv_s) {
    i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    i64 b = out_ptr[j], e = out_ptr[j + 1];
    if (e == b) {
        inv_s[j] = 0.0;
        return;
    }
    double s = 0.0;
    if (w) {
        for (i64 p = b; p < e; ++p) s += (double)w[p];
    } else {
        s = (double)(e - b);
    }
    inv_s[j] = 1.0 / s;
}

// ---------------------------------------------------------------------------
// Block-local split.  Nodes are grouped in ranges of 2^rb consecutive ids.  An edge
// is local when source and target share a range.  OUT rows are sorted by target, so a
// row's local targets form one contiguous span.
// ---------------------------------------------------------------------------
__device__ __forceinline__ i64 lower_bound_i32(const int *a, i64 lo, i64 hi, int key) {
    while (lo < hi) {
        i64 mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_local_span(const i64 *__restrict__ out_ptr, const int *__restrict__ out_idx,
                             const float *__restrict__ w, i64 n, int rb, i64 *loc_deg, i64 *loc_first,
                             double *rw) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i64 b = out_ptr[i], e = out_ptr[i + 1];
    const i64 lo_t = (i >> rb) << rb;
    const i64 hi_t = lo_t + ((i64)1 << rb);
    i64 a = lower_bound_i32(out_idx, b, e, (int)lo_t);
    i64 z = hi_t >= (i64)0x7fffffff ? e : lower_bound_i32(out_idx, a, e, (int)hi_t);
    loc_deg[i] = z - a;
    loc_first[i] = a;
    double r = 0.0;
    if (w) {
        for (i64 p = b; p < a; ++p) r += (double)w[p];
        for (i64 p = z; p < e; ++p) r += (double)w[p];
    } else {
        r = (double)((a - b) + (e - z));
    }
    rw[i] = r;
}

__global__ void k_local_copy(const int *__restrict__ out_idx, const float *__restrict__ w,
                             const i64 *__restrict__ loc_first, const i64 *__restrict__ loc_ptr, i64 n, int rb,
                             unsigned short *loc_tgt, float *loc_w) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i64 lo_t = (i >> rb) << rb;
    const i64 a = loc_first[i], dst = loc_ptr[i], cnt = loc_ptr[i + 1] - dst;
    for (i64 k = 0; k < cnt; ++k) {
        loc_tgt[dst + k] = (unsigned short)(out_idx[a + k] - lo_t);
        if (loc_w) loc_w[dst + k] = w[a + k];
    }
}

// flag cross-range IN entries (keys = targets sorted, in_idx = sources)
__global__ void k_remote_flags(const unsigned *__restrict__ tgt, const int *__restrict__ in_idx, i64 m, int rb,
                               i64 *flag) {
    i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    flag[p] = ((i64)tgt[p] >> rb) != ((i64)in_idx[p] >> rb) ? 1 : 0;
}

__global__ void k_remote_scatter(const unsigned *__restrict__ tgt, const int *__restrict__ in_idx,
                                 const float *__restrict__ in_w, const i64 *__restrict__ pos, i64 m, int rb,
                                 int *rem_src, unsigned short *rem_tgt, float *rem_w) {
    i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    i64 t = tgt[p];
    int s = in_idx[p];
    if ((t >> rb) == ((i64)s >> rb)) return;
    i64 q = pos[p];
    rem_src[q] = s;
    rem_tgt[q] = (unsigned short)(t - ((t >> rb) << rb));
    if (rem_w) rem_w[q] = in_w[p];
}

// Re-ordering of each range's cross-range entries by source (see build_graph).
__global__ void k_iota_keys(const int *__restrict__ src, i64 m, unsigned *keys, u64 *vals) {
    i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    keys[p] = (unsigned)src[p];
    vals[p] = (u64)p;
}

// keys[i] = the range whose entries hold original position pos[i]
__global__ void k_range_of(const u64 *__restrict__ pos, i64 m, const i64 *__restrict__ rem_base, i64 nranges,
                           unsigned *keys) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const i64 q = (i64)pos[i];
    i64 lo = 0, hi = nranges - 1;  // last r with rem_base[r] <= q
    while (lo < hi) {
        const i64 mid = (lo + hi + 1) >> 1;
        if (rem_base[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    keys[i] = (unsigned)lo;
}

__global__ void k_permute_remote(const u64 *__restrict__ pos, i64 m, const int *__restrict__ src,
                                 const unsigned short *__restrict__ tgt, const float *__restrict__ w, int *src2,
                                 unsigned short *tgt2, float *w2) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const i64 q = (i64)pos[i];
    src2[i] = src[q];
    tgt2[i] = tgt[q];
    if (w) w2[i] = w[q];
}

__global__ void k_deg_flags(const i64 *__restrict__ out_ptr, const double *__restrict__ rw, i64 n, unsigned *out) {
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (unsigned)(out_ptr[i + 1] - out_ptr[i]) | (rw[i] > 0.0 ? 0x80000000u : 0u);
}

// rem_base[r] = number of cross-range IN entries before range r's first row.
__global__ void k_range_bases(const i64 *__restrict__ in_ptr, const i64 *__restrict__ pos, i64 n, i64 m,
                              i64 rem_total, int rb, i64 nranges, i64 *rem_base, const i64 *__restrict__ loc_ptr,
                              i64 *loc_base) {
    i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > nranges) return;
    i64 row = r << rb;
    if (row > n) row = n;
    i64 p = in_ptr[row];
    rem_base[r] = p >= m ? rem_total : pos[p];
    loc_base[r] = loc_ptr[row];
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
template <typename T>
static int dalloc(T **p, i64 count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    DI_HIP(dev_malloc((void **)p, (size_t)count * sizeof(T)));
    return DI_OK;
}

// device temporaries of one build, freed on every way out of it
struct DevTemps {
    std::vector<void *> p;
    DevTemps() = default;
    DevTemps(const DevTemps &) = delete;
    DevTemps &operator=(const DevTemps &) = delete;
    ~DevTemps() {
        for (void *q : p)
            if (q) (void)dev_free(q);
    }
    template <typename T>
    int alloc(T **x, i64 count) {
        DI_TRY(dalloc(x, count));
        p.push_back((void *)*x);
        return DI_OK;
    }
    void release(const void *q) {  // ownership passed on
        for (void *&e : p)
            if (e == q) e = nullptr;
    }
};

int build_graph(DevGraph &g, const i64 *d_out_ptr, const int *d_out_idx, const float *d_w, int range_log2,
                bool remote_by_source,
                hipStream_t st) {
    const i64 n = g.n, m = g.m;
    const int TB = 256;
    DevTemps tmp;
    int key_bits = 0;
    while (((i64)1 << key_bits) < n) ++key_bits;

    // IN by a stable sort of (target, source|weight) pairs in OUT order
    unsigned *keys = nullptr, *keys2 = nullptr;
    u64 *vals = nullptr, *vals2 = nullptr;
    i64 *counts = nullptr, *stemp = nullptr;
    DI_TRY(tmp.alloc(&keys, m));
    DI_TRY(tmp.alloc(&keys2, m));
    DI_TRY(tmp.alloc(&vals, m));
    DI_TRY(tmp.alloc(&vals2, m));
    const i64 ccount = radix_counts_elems(m);
    i64 scount = std::max(ccount, m + 1);
    DI_TRY(tmp.alloc(&counts, std::max(ccount, m + 1)));
    DI_TRY(tmp.alloc(&stemp, scan_temp_elems(scount) + 64));
    k_expand_sources<<<grid_for(n, TB), TB, 0, st>>>(d_out_ptr, d_out_idx, d_w, n, keys, vals);
    DI_LAUNCH_CHECK();
    bool in_tmp = false;
    DI_TRY(radix_sort_pairs<u64>(keys, vals, keys2, vals2, m, key_bits, counts, stemp, st, &in_tmp));
    unsigned *sk = in_tmp ? keys2 : keys;
    u64 *sv = in_tmp ? vals2 : vals;

    DI_TRY(dalloc(&g.in_ptr, n + 1));
    DI_TRY(dalloc(&g.in_idx, m));
    if (g.weighted) DI_TRY(dalloc(&g.in_w, m));
    k_fill_i64<<<grid_for(n + 1, TB), TB, 0, st>>>(g.in_ptr, m, n + 1);
    DI_LAUNCH_CHECK();
    if (m > 0) {
        k_row_ptr_from_keys<<<grid_for(m, TB), TB, 0, st>>>(sk, m, g.in_ptr);
        DI_LAUNCH_CHECK();
        k_unpack_in<<<grid_for(m, TB), TB, 0, st>>>(sv, m, g.in_idx, g.in_w);
        DI_LAUNCH_CHECK();
    }

    DI_TRY(dalloc(&g.inv_s, n));
    k_inv_s<<<grid_for(n, TB), TB, 0, st>>>(d_out_ptr, d_w, n, g.inv_s);
    DI_LAUNCH_CHECK();

    // block-local split
    const int rb = range_log2;
    g.rb = rb;
    g.nranges = (n + ((i64)1 << rb) - 1) >> rb;
    i64 *loc_deg = nullptr, *loc_first = nullptr;
    DI_TRY(tmp.alloc(&loc_deg, n + 1));
    DI_TRY(tmp.alloc(&loc_first, n));
    DI_TRY(dalloc(&g.rw, n));
    k_local_span<<<grid_for(n, TB), TB, 0, st>>>(d_out_ptr, d_out_idx, d_w, n, rb, loc_deg, loc_first, g.rw);
    DI_LAUNCH_CHECK();
    DI_TRY(dalloc(&g.deg_flags, n));
    k_deg_flags<<<grid_for(n, TB), TB, 0, st>>>(d_out_ptr, g.rw, n, g.deg_flags);
    DI_LAUNCH_CHECK();
    DI_TRY(dalloc(&g.loc_ptr, n + 1));
    k_fill_i64<<<1, 1, 0, st>>>(loc_deg + n, 0, 1);
    DI_TRY(scan_exclusive(loc_deg, g.loc_ptr, n + 1, stemp, st));
    DI_HIP(hipMemcpyAsync(&g.m_loc, g.loc_ptr + n, sizeof(i64), hipMemcpyDeviceToHost, st));
    DI_HIP(hipStreamSynchronize(st));
    DI_TRY(dalloc(&g.loc_tgt, g.m_loc + 8));  // padded: staged as 32-bit words
    if (g.weighted) DI_TRY(dalloc(&g.loc_w, g.m_loc));
    k_local_copy<<<grid_for(n, TB), TB, 0, st>>>(d_out_idx, d_w, loc_first, g.loc_ptr, n, rb, g.loc_tgt, g.loc_w);
    DI_LAUNCH_CHECK();

    // cross-range entries of IN, kept in IN order (target, then source ascending)
    i64 *flag = counts;  // reuse: m + 1 entries
    if (m > 0) {
        k_remote_flags<<<grid_for(m, TB), TB, 0, st>>>(sk, g.in_idx, m, rb, flag);
        DI_LAUNCH_CHECK();
    }
    k_fill_i64<<<1, 1, 0, st>>>(flag + m, 0, 1);
    DI_TRY(scan_exclusive(flag, flag, m + 1, stemp, st));
    DI_HIP(hipMemcpyAsync(&g.m_rem, flag + m, sizeof(i64), hipMemcpyDeviceToHost, st));
    DI_HIP(hipStreamSynchronize(st));
    DI_TRY(dalloc(&g.rem_src, g.m_rem));
    DI_TRY(dalloc(&g.rem_tgt, g.m_rem));
    if (g.weighted) DI_TRY(dalloc(&g.rem_w, g.m_rem));
    if (m > 0) {
        k_remote_scatter<<<grid_for(m, TB), TB, 0, st>>>(sk, g.in_idx, g.in_w, flag, m, rb, g.rem_src, g.rem_tgt,
                                                          g.rem_w);
        DI_LAUNCH_CHECK();
    }
    DI_TRY(dalloc(&g.rem_base, g.nranges + 1));
    DI_TRY(dalloc(&g.loc_base, g.nranges + 1));
    k_range_bases<<<grid_for(g.nranges + 1, TB), TB, 0, st>>>(g.in_ptr, flag, n, m, g.m_rem, rb, g.nranges,
                                                              g.rem_base, g.loc_ptr, g.loc_base);
    DI_LAUNCH_CHECK();
    // Within each range, order the cross-range entries by source instead of by target:
    // a range's pull then walks the in-flight values of each neighbouring range in
    // address order, so most gathers hit lines already in cache.  (Two stable passes:
    // by source, then by range.)
    if (remote_by_source && g.m_rem > 1) {
        const i64 mr = g.m_rem;
        int sbits = 1, rbits = 1;
        while (((i64)1 << sbits) < n) ++sbits;
        while (((i64)1 << rbits) < g.nranges) ++rbits;
        k_iota_keys<<<grid_for(mr, TB), TB, 0, st>>>(g.rem_src, mr, keys, vals);
        DI_LAUNCH_CHECK();
        bool t1 = false, t2 = false;
        DI_TRY(radix_sort_pairs<u64>(keys, vals, keys2, vals2, mr, sbits, counts, stemp, st, &t1));
        unsigned *k1 = t1 ? keys2 : keys, *k1o = t1 ? keys : keys2;
        u64 *v1 = t1 ? vals2 : vals, *v1o = t1 ? vals : vals2;
        k_range_of<<<grid_for(mr, TB), TB, 0, st>>>(v1, mr, g.rem_base, g.nranges, k1);
        DI_LAUNCH_CHECK();
        DI_TRY(radix_sort_pairs<u64>(k1, v1, k1o, v1o, mr, rbits, counts, stemp, st, &t2));
        const u64 *perm = t2 ? v1o : v1;
        int *src2 = nullptr;
        unsigned short *tgt2 = nullptr;
        float *w2 = nullptr;
        DI_TRY(tmp.alloc(&src2, mr));
        DI_TRY(tmp.alloc(&tgt2, mr));
        if (g.weighted) DI_TRY(tmp.alloc(&w2, mr));
        k_permute_remote<<<grid_for(mr, TB), TB, 0, st>>>(perm, mr, g.rem_src, g.rem_tgt, g.rem_w, src2, tgt2, w2);
        DI_LAUNCH_CHECK();
        DI_HIP(hipStreamSynchronize(st));
        (void)dev_free(g.rem_src);
        (void)dev_free(g.rem_tgt);
        if (g.rem_w) (void)dev_free(g.rem_w);
        tmp.release(src2);
        tmp.release(tgt2);
        tmp.release(w2);
        g.rem_src = src2;
        g.rem_tgt = tgt2;
        g.rem_w = w2;
    }
    DI_HIP(hipStreamSynchronize(st));
    return DI_OK;
}

void free_graph(DevGraph &g) {
    void *ps[] = {g.in_ptr, g.in_idx, g.in_w, g.inv_s, g.rw, g.loc_ptr, g.loc_tgt, g.loc_w,
                  g.rem_src, g.rem_tgt, g.rem_w, g.rem_base, g.loc_base, g.out_ptr, g.out_idx, g.w,
                  g.deg_flags};
    for (void *p : ps)
        if (p) (void)dev_free(p);
    g = DevGraph{};
}

}  // namespace di
