// Sweep kernels for one right-hand side.
//
// Block-local D-Iteration (the default sweep).  Node ids are grouped into ranges of
// 2^rb consecutive nodes; one workgroup owns a range for the whole sweep and keeps
// its fluid in LDS.  A sweep of a range:
//   1. loads F of the range and adds the fluid other ranges sent in the previous
//      sweep (a pull over the range's cross-range in-edges);
//   2. runs up to `rounds` local rounds: every wave scans its share of the range,
//      takes each node whose fluid is at least the sweep threshold (an elementary
//      diffusion, Section 3.1, equation defF: f -> H_i, F_i = 0, d f P e_i pushed),
//      pushes the local part with LDS atomics and records the cross-range part per
//      source for delivery in the next sweep;
//   3. writes F back and adds |F| plus the fluid in flight to the residual.
// The identity H + F = F_0 + d P H (equation HnFn) holds whenever the fluid in
// flight is counted as fluid, so |F|_1 (with it) still bounds |x - H|_1 (Theorem 1).
#include "sweep.h"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace di {

// 12 waves: with 2^12-node ranges the LDS of two such workgroups fits one compute unit
// (2 x 81.7 KB), so a CU runs 24 waves instead of one 16-wave workgroup
constexpr int BLD_THREADS = 768;
constexpr int BLD_WAVES = BLD_THREADS / WAVE;

int bld_threads() { return BLD_THREADS; }

// The LDS tiles of the block-local sweeps hold the fluid in double for every fluid type:
// on this chip a 64-lane LDS atomic add costs about 8 cycles in double and about 190 in
// float.  The fluid type decides only what is stored in memory.
size_t bld_lds_bytes(int rb, int fp32) {
    (void)fp32;
    const size_t B = (size_t)1 << rb;
    return 2 * B * 8 + (size_t)BLD_WAVES * WAVE * (8 + 4 + 8);
}

template <typename T>
__device__ __forceinline__ T lds_load(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// inclusive prefix sum over the 64 lanes of a wave with DPP moves (rows of 16 by shifts of
// 1, 2, 4 and 8, then lane 15 of each row into the next row, then lane 31 into rows 2 and 3)
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// 1/c for an integer count c >= 1: the hardware estimate refined by two Newton steps
// (within an ulp of the correctly rounded quotient; no scaling is needed in this range)
__device__ __forceinline__ double recip_count(unsigned c) {
    const double x = (double)c;
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// returns false if v is NaN, infinite or beyond the fixed-point range
__device__ __forceinline__ bool limbs_add_checked(Limbs &a, double v, int K) {
    if (!(v == v) || !(ldexp(v, K) < 0x1p126)) return false;
    limbs_add(a, v, K);
    return true;
}

// the same for a signed value (the leak: fluid is signed after a graph update)
__device__ __forceinline__ bool limbs_add_signed_checked(Limbs &a, double v, int K) {
    if (!(v == v) || !(ldexp(fabs(v), K) < 0x1p126)) return false;
    limbs_add_signed(a, v, K);
    return true;
}

struct BldArgs {
    const i64 *loc_ptr;
    const unsigned short *loc_tgt;
    const float *loc_w;
    const int *rem_src;
    const unsigned short *rem_tgt;
    const float *rem_w;
    const i64 *rem_base;
    const double *inv_s;
    const double *rw;
    const int *range_order;
    // adjoint sweeps on the transposed graph: 1/s_j of the forward graph at each target j
    // (the push from i to j carries P[i][j] = w(j->i) / s_j); nullptr otherwise
    const double *tinv;
    i64 n;
    int rb;
    void *F;
    double *H;
    void *S0, *S1;
    u64 *Sb0, *Sb1;  // bitmaps of the nonzero in-flight values
    DevCtl *ctl;
    double d;
    int K;
    int rounds;
    int force;  // run even when the solve is marked done (delivery of fluid in flight)
    u64 *partR, *partC;  // per-workgroup partial sums (one slot per range)
    const int *range_graph;  // union of graphs: graph of each range (else nullptr)
    const int *range_cnt;    // cut-aligned ranges: real nodes of each range (else nullptr)
    const GraphCtl *gctl;
};

// Threshold and number of local rounds of range r: the solve's own, or its graph's in a
// union of graphs.  Returns false when the range's graph is frozen (nothing to do).
__device__ __forceinline__ bool range_schedule(const int *range_graph, const GraphCtl *gctl, int r, double &thr,
                                               int &rounds) {
    if (!range_graph) return true;
    const GraphCtl &gc = gctl[range_graph[r]];
    if (gc.state == GS_FROZEN) return false;
    thr = gc.thr;
    if (gc.state == GS_FINISH) rounds = 0;
    return true;
}

// ADJ: the adjoint diffusion (lambda = (I - d P^T)^{-1} g) on the transposed graph: the
// push from i along its transposed edge to j carries d f w_e / s_j (s_j of the forward
// graph, a.tinv), so the factor is applied at the target; the fluid is signed; the
// partial slot's maximum is max |F| of the range right after the fluid in flight arrived
// (the exact state between two sweeps), which the L-infinity stop needs.
template <typename T, bool WTD, bool ADJ = false>
__global__ void __launch_bounds__(BLD_THREADS) k_bld_sweep(BldArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    DevCtl *ctl = a.ctl;
    if (!a.force && (ctl->done || ctl->sweep >= ctl->budget)) return;
    const int B = 1 << a.rb;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    double *Fl = reinterpret_cast<double *>(smem);
    double *Sl = Fl + B;
    i64 *sc_start = reinterpret_cast<i64 *>(Sl + B) + w * WAVE;
    int *sc_off = reinterpret_cast<int *>(reinterpret_cast<i64 *>(Sl + B) + BLD_WAVES * WAVE) + w * WAVE;
    double *sc_q =
        reinterpret_cast<double *>(reinterpret_cast<int *>(reinterpret_cast<i64 *>(Sl + B) + BLD_WAVES * WAVE) +
                                   BLD_WAVES * WAVE) +
        w * WAVE;
    __shared__ u64 red[PSC * BLD_WAVES];
    __shared__ int bad;

    const int par = ctl->parity;
    const T *Sprev = reinterpret_cast<const T *>(par ? a.S1 : a.S0);
    T *Snext = reinterpret_cast<T *>(par ? a.S0 : a.S1);
    const u64 *Sbprev = par ? a.Sb1 : a.Sb0;
    u64 *Sbnext = par ? a.Sb0 : a.Sb1;
    T *F = reinterpret_cast<T *>(a.F);
    double thr = ctl->thr;
    int rounds = a.rounds;
    const int r = a.range_order[blockIdx.x];
    if (!range_schedule(a.range_graph, a.gctl, r, thr, rounds)) return;
    const i64 base = (i64)r << a.rb;
    // real nodes of the range (cut-aligned ranges end early; the rest is padding)
    const int cnt = a.range_cnt ? a.range_cnt[r] : (int)min((i64)B, a.n - base);
    if (threadIdx.x == 0) bad = 0;

    // 1. fluid of the range, plus fluid sent here by other ranges last sweep
    for (int i = threadIdx.x; i < cnt; i += BLD_THREADS) {
        Fl[i] = (double)F[base + i];
        Sl[i] = 0.0;
    }
    __syncthreads();
    u64 delivered = 0;
    {
        // batches of REM_U entries per thread: all index loads, then all gathers, then
        // the LDS adds, so that each thread keeps REM_U independent loads in flight
        constexpr int REM_U = 4;  // 8 would take the registers the second workgroup needs
        const i64 p0 = a.rem_base[r], p1 = a.rem_base[r + 1];
        for (i64 pb = p0 + threadIdx.x; pb < p1; pb += (i64)BLD_THREADS * REM_U) {
            // out-of-range slots re-read the last entry (a valid address) and add nothing
            int src[REM_U];
            unsigned tg[REM_U];
            float wv[REM_U];
#pragma unroll
            for (int u = 0; u < REM_U; ++u) {
                const i64 p = min(pb + (i64)u * BLD_THREADS, p1 - 1);
                src[u] = a.rem_src[p];
                tg[u] = (unsigned)a.rem_tgt[p];
                wv[u] = WTD ? a.rem_w[p] : 1.0f;
            }
            // a value is gathered only when its bit in the in-flight bitmap is set
            u64 wd[REM_U];
#pragma unroll
            for (int u = 0; u < REM_U; ++u) wd[u] = Sbprev[src[u] >> 6];
            T v[REM_U];
#pragma unroll
            for (int u = 0; u < REM_U; ++u) v[u] = ((wd[u] >> (src[u] & 63)) & 1ull) ? Sprev[src[u]] : (T)0;
#pragma unroll
            for (int u = 0; u < REM_U; ++u) {
                if (pb + (i64)u * BLD_THREADS < p1 && v[u] != (T)0) {
                    double add = (double)v[u];
                    if (WTD) add *= (double)wv[u];
                    if (ADJ) add *= a.tinv[base + tg[u]];
                    atomicAdd(&Fl[tg[u]], add);
                    ++delivered;
                }
            }
        }
    }
    __syncthreads();
    u64 mstart = 0;  // adjoint: max |F| of the range with the fluid in flight delivered
    if (ADJ)
        for (int i = threadIdx.x; i < cnt; i += BLD_THREADS) {
            const u64 b = (u64)__double_as_longlong(fabs((double)Fl[i]));
            mstart = b > mstart ? b : mstart;
        }

    // 2. local rounds; wave w owns [my0, my1)
    const int sub = (((cnt + BLD_WAVES - 1) / BLD_WAVES) + WAVE - 1) & ~(WAVE - 1);
    const int my0 = w * sub, my1 = min(cnt, my0 + sub);
    Limbs leak;
    limbs_zero(leak);
    u64 nodes = 0, edges = 0;
    for (int round = 0; round < rounds; ++round) {
        bool any = false;
        for (int c = my0; c < my1; c += WAVE) {
            const int i = c + lane;
            double f = 0.0;
            if (i < my1) {
                const double v = lds_load(&Fl[i]);
                if (v != 0.0 && fabs(v) >= thr) f = atomicExch(&Fl[i], 0.0);
            }
            if (__ballot(f != 0.0) == 0) continue;
            any = true;
            int dg = 0;
            i64 st = 0;
            double q = 0.0;
            if (f != 0.0) {
                const i64 gi = base + i;
                a.H[gi] += f;
                const double inv = a.inv_s[gi];
                if (inv == 0.0) {
                    if (!limbs_add_signed_checked(leak, f, a.K)) bad = 1;
                } else {
                    q = ADJ ? a.d * f : (a.d * f) * inv;
                    if (a.rw[gi] > 0.0) Sl[i] += q;
                    st = a.loc_ptr[gi];
                    dg = (int)(a.loc_ptr[gi + 1] - st);
                }
                ++nodes;
            }
            const int inc = wave_incl_scan_i32(dg);
            const int total = __shfl(inc, WAVE - 1, WAVE);
            sc_start[lane] = st;
            sc_off[lane] = inc - dg;
            sc_q[lane] = q;
            wave_sync_lds();
            edges += (lane == 0) ? (u64)total : 0ull;
            // EDGE_U slots per lane per step: owners by binary search over the wave's
            // exclusive degree offsets, then all target loads, then the LDS adds
            constexpr int EDGE_U = 4;
            for (int sb = lane; sb < total; sb += WAVE * EDGE_U) {
                // slots past the end search and load for slot total-1 and add nothing
                unsigned tgt[EDGE_U];
                double val[EDGE_U];
#pragma unroll
                for (int u = 0; u < EDGE_U; ++u) {
                    const int s = min(sb + u * WAVE, total - 1);
                    int lo = 0, hi = WAVE - 1;  // last k with sc_off[k] <= s (it has a nonzero degree)
#pragma unroll
                    for (int it = 0; it < 6; ++it) {
                        const int mid = (lo + hi + 1) >> 1;
                        const bool le = sc_off[mid] <= s;
                        lo = le ? mid : lo;
                        hi = le ? hi : mid - 1;
                    }
                    const i64 p = sc_start[lo] + (s - sc_off[lo]);
                    tgt[u] = a.loc_tgt[p];
                    val[u] = WTD ? sc_q[lo] * (double)a.loc_w[p] : sc_q[lo];
                    if (ADJ) val[u] *= a.tinv[base + tgt[u]];
                }
#pragma unroll
                for (int u = 0; u < EDGE_U; ++u)
                    if (sb + u * WAVE < total) atomicAdd(&Fl[tgt[u]], val[u]);
            }
            wave_sync_lds();
        }
        if (!any) break;
    }
    __syncthreads();

    // 3. write back; residual = |F| + fluid in flight
    Limbs R;
    limbs_zero(R);
    for (int i = threadIdx.x; i < cnt; i += BLD_THREADS) {
        const T v = (T)Fl[i];
        const T s = (T)Sl[i];
        F[base + i] = v;
        // the wave's 64 lanes hold 64 consecutive nodes starting at a multiple of 64
        const u64 bits = __ballot(s != (T)0);
        if (s != (T)0) Snext[base + i] = s;
        if ((threadIdx.x & (WAVE - 1)) == 0) Sbnext[(base + i) >> 6] = bits;
        if (!limbs_add_checked(R, fabs((double)v), a.K)) bad = 1;
        if (!ADJ && s != (T)0 && !limbs_add_checked(R, fabs((double)s) * a.rw[base + i], a.K)) bad = 1;
    }
    store_residual_partial(R, mstart, red, a.partR + (i64)r * PSR);
    store_counter_partial(leak, nodes, edges + delivered, delivered, red, a.partC + (i64)r * PSC);
    if (threadIdx.x == 0 && bad) atomicOr(&ctl->overflow, 1);
}

static BldArgs make_bld_args(const DevGraph &g, SolveState &s, const SweepParams &p, int rounds) {
    BldArgs a;
    a.tinv = nullptr;
    a.loc_ptr = g.loc_ptr;
    a.loc_tgt = g.loc_tgt;
    a.loc_w = g.loc_w;
    a.rem_src = g.rem_src;
    a.rem_tgt = g.rem_tgt;
    a.rem_w = g.rem_w;
    a.rem_base = g.rem_base;
    a.inv_s = g.inv_s;
    a.rw = g.rw;
    a.range_order = s.range_order;
    a.n = g.n;
    a.rb = g.rb;
    a.F = s.F;
    a.H = s.H;
    a.S0 = s.S[0];
    a.S1 = s.S[1];
    a.Sb0 = s.Sb[0];
    a.Sb1 = s.Sb[1];
    a.ctl = s.ctl;
    a.d = p.d;
    a.K = p.K;
    a.rounds = rounds;
    a.force = rounds == 0;
    a.partR = s.partR;
    a.partC = s.partC;
    a.range_graph = s.range_graph;
    a.range_cnt = s.range_cnt;
    a.gctl = s.gctl;
    return a;
}


// ---------------------------------------------------------------------------
// Block-local sweep with the range's local adjacency resident in LDS (unweighted
// graphs).  Per range the workgroup stages, with batched coalesced loads: the fluid,
// the out-degrees (1/s_j = 1/out(j) is recomputed in double), the local row offsets
// and as many 16-bit local targets as fit (the rest are read from global memory).
// The local rounds then touch LDS only; the history increment of the sweep is kept
// per node in LDS and added to H once at write-back, where the cross-range share
// d * dH_i / out(i) of every node is also written for delivery next sweep.
// ---------------------------------------------------------------------------
struct Bld2Args {
    const i64 *loc_ptr;
    const unsigned short *loc_tgt;
    const i64 *loc_base;
    const unsigned *deg_flags;
    const int *rem_src;
    const unsigned short *rem_tgt;
    const i64 *rem_base;
    const int *range_order;
    i64 n;
    int rb;
    int tcap;  // local targets staged in LDS
    void *F;
    double *H;
    void *S0, *S1;
    u64 *Sb0, *Sb1;
    DevCtl *ctl;
    double d;
    int K;
    int rounds;
    int force;
    u64 *partR, *partC;
    const int *range_cnt;
    const int *range_graph;
    const GraphCtl *gctl;
};

// LDS layout of k_bld2_sweep (bytes): F[B] (double), dH[B] (double), deg[B], off[B+1]
// (u32), padding to 8, then per wave 64 x (q double, start u32), per wave a bitmap of
// BLD2_SLOTS bits, then the targets.
__host__ __device__ inline size_t bld2_scratch_offset(int B, int tsize) {
    (void)tsize;  // the LDS fluid is double for every fluid type
    return ((size_t)B * 8 + (size_t)8 * B + (size_t)4 * (2 * B + 1) + 7) & ~(size_t)7;
}

// edge slots one wave lists before it pushes them (a multiple of 4 x 64)
constexpr int BLD2_SLOTS = 1024;

size_t bld2_fixed_lds(int rb, int fp32, int threads) {
    return bld2_scratch_offset(1 << rb, fp32 ? 4 : 8) +
           (size_t)(threads / WAVE) * (WAVE * (8 + 4) + BLD2_SLOTS / 8);
}

// Pushes the local edges of the nodes a wave has listed: listed node k sends sc_q[k] along
// its edges, which occupy the slots [o_k, o_{k+1}) of [0, ltot); bit o_k of the wave's
// bitmap is set and sc_base[k] = (start of k's targets) - o_k.  A lane finds the node of
// its slot s from the 64-bit bitmap word holding s (the same word for the whole wave) and
// the running count of set bits before it; no search.  Slots past ltot push nothing.  The
// bitmap is cleared on return.
template <typename T>
__device__ __forceinline__ void bld2_push_list(T *Fl, const unsigned short *Tg, int tdelta, int ncap, int nloc,
                                               const unsigned short *loc_tgt, i64 lb,
                                               const int *sc_base, const double *sc_q,
                                               unsigned *sc_bits, int ltot, int lane) {
    wave_sync_lds();
    constexpr int EDGE_U = 4;
    int pre = 0;  // listed nodes that start before the current window
    for (int sb = 0; sb < ltot; sb += WAVE * EDGE_U) {
        unsigned tgt[EDGE_U];
        double val[EDGE_U];
        unsigned pp[EDGE_U];
#pragma unroll
        for (int u = 0; u < EDGE_U; ++u) {
            const int wd = (sb >> 5) + 2 * u;  // 32-bit words of the window [sb + 64u, +64)
            const unsigned lo = __builtin_amdgcn_readfirstlane(sc_bits[wd]);
            const unsigned hi = __builtin_amdgcn_readfirstlane(sc_bits[wd + 1]);
            const unsigned below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            const unsigned mine = ((lane < 32 ? lo >> lane : hi >> (lane - 32)) & 1u);
            const int k = pre + (int)(below + mine) - 1;
            pre += __builtin_popcount(lo) + __builtin_popcount(hi);
            const int sl = sb + u * WAVE + lane;
            pp[u] = sl < ltot ? (unsigned)(sc_base[k] + sl) : 0u;
            val[u] = sc_q[k];
        }
        bool staged = true;
#pragma unroll
        for (int u = 0; u < EDGE_U; ++u) staged = staged && (int)pp[u] < ncap;
        if (__ballot(!staged) == 0) {
#pragma unroll
            for (int u = 0; u < EDGE_U; ++u) tgt[u] = Tg[tdelta + pp[u]];
        } else {
#pragma unroll
            for (int u = 0; u < EDGE_U; ++u) {
                unsigned t;
                if ((int)pp[u] < ncap) {
                    t = Tg[tdelta + pp[u]];
                } else {
                    t = loc_tgt[lb + min((int)pp[u], nloc - 1)];
                    asm volatile("" : "+v"(t));
                }
                tgt[u] = t;
            }
        }
#pragma unroll
        for (int u = 0; u < EDGE_U; ++u)
            if (sb + u * WAVE + lane < ltot) atomicAdd(&Fl[tgt[u]], (T)val[u]);
    }
    wave_sync_lds();
    for (int wd = lane; wd < ((ltot + 255) >> 8) * 8; wd += WAVE) sc_bits[wd] = 0u;
    wave_sync_lds();
}

template <typename T>
__global__ void __launch_bounds__(1024) k_bld2_sweep(Bld2Args a) {
    extern __shared__ __align__(16) unsigned char smem[];
    DevCtl *ctl = a.ctl;
    if (!a.force && (ctl->done || ctl->sweep >= ctl->budget)) return;
    const int B = 1 << a.rb;
    const int nthr = blockDim.x, nw = nthr >> 6;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    double *Fl = reinterpret_cast<double *>(smem);  // double for every fluid type
    double *Dl = Fl + B;                            // history increments
    unsigned *Deg = reinterpret_cast<unsigned *>(Dl + B);
    unsigned *Off = Deg + B;  // B + 1 entries
    double *sc_q_all = reinterpret_cast<double *>(smem + bld2_scratch_offset(B, (int)sizeof(T)));
    unsigned *sc_start_all = reinterpret_cast<unsigned *>(sc_q_all + nw * WAVE);
    unsigned *sc_bits_all = sc_start_all + nw * WAVE;
    unsigned short *Tg = reinterpret_cast<unsigned short *>(sc_bits_all + nw * (BLD2_SLOTS / 32));
    double *sc_q = sc_q_all + w * WAVE;
    unsigned *sc_start = sc_start_all + w * WAVE;
    unsigned *sc_bits = sc_bits_all + w * (BLD2_SLOTS / 32);
    __shared__ u64 red[PSC * 16];
    __shared__ int bad;
    __shared__ int chunk_ctr[64];  // chunks handed out in each local round

    const int par = ctl->parity;
    const T *Sprev = reinterpret_cast<const T *>(par ? a.S1 : a.S0);
    T *Snext = reinterpret_cast<T *>(par ? a.S0 : a.S1);
    const u64 *Sbprev = par ? a.Sb1 : a.Sb0;
    u64 *Sbnext = par ? a.Sb0 : a.Sb1;
    T *F = reinterpret_cast<T *>(a.F);
    double thr = ctl->thr;
    int rounds = a.rounds;
    const int r = a.range_order[blockIdx.x];
    if (!range_schedule(a.range_graph, a.gctl, r, thr, rounds)) return;
    const i64 base = (i64)r << a.rb;
    // real nodes of the range (cut-aligned ranges end early; the rest is padding)
    const int cnt = a.range_cnt ? a.range_cnt[r] : (int)min((i64)B, a.n - base);
    const i64 lb = a.loc_base[r];
    const int nloc = (int)(a.loc_base[r + 1] - lb);
    const int ncap = min(nloc, a.tcap);
    if (threadIdx.x == 0) bad = 0;
    if (threadIdx.x < 64) chunk_ctr[threadIdx.x] = 0;
    for (int wd = threadIdx.x; wd < nw * (BLD2_SLOTS / 32); wd += nthr) sc_bits_all[wd] = 0u;

    // 1. stage the range; every loop keeps SU independent loads in flight per thread
    // (out-of-range slots load a valid clamped address and store nothing)
    constexpr int SU = 4;  // 4-deep batches: 62 VGPRs (8-deep ones took 111 and ran 1.3% slower)
    for (int i0 = threadIdx.x; i0 < cnt; i0 += nthr * SU) {
        T fv[SU];
        unsigned dv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int i = min(i0 + u * nthr, cnt - 1);
            fv[u] = F[base + i];
            dv[u] = a.deg_flags[base + i];
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int i = i0 + u * nthr;
            if (i < cnt) {
                Fl[i] = (double)fv[u];
                Dl[i] = 0.0;
                Deg[i] = dv[u];
            }
        }
    }
    for (int i0 = threadIdx.x; i0 <= cnt; i0 += nthr * SU) {
        i64 ov[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) ov[u] = a.loc_ptr[base + min(i0 + u * nthr, cnt)];
#pragma unroll
        for (int u = 0; u < SU; ++u)
            if (i0 + u * nthr <= cnt) Off[i0 + u * nthr] = (unsigned)(ov[u] - lb);
    }
    // local targets as 32-bit words from the aligned word holding target lb; target p
    // sits at Tg[tdelta + p] (the target array is padded, so the last word is readable)
    const int tdelta = (int)(lb & 1);
    {
        const unsigned *srcw = reinterpret_cast<const unsigned *>(a.loc_tgt) + (lb >> 1);
        unsigned *Tw = reinterpret_cast<unsigned *>(Tg);
        const int nwords = (tdelta + ncap + 1) >> 1;
        for (int i0 = threadIdx.x; i0 < nwords; i0 += nthr * SU) {
            unsigned tv[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) tv[u] = srcw[min(i0 + u * nthr, nwords - 1)];
#pragma unroll
            for (int u = 0; u < SU; ++u)
                if (i0 + u * nthr < nwords) Tw[i0 + u * nthr] = tv[u];
        }
    }
    __syncthreads();

    // 2. fluid sent here by other ranges last sweep.  Every source with cross-range
    // edges wrote its value (zero included) and its bit in the in-flight bitmap; when few
    // sources sent, a value is gathered only if its bit is set (a random read costs a
    // full line), else every value is read directly
    u64 delivered = 0;
    const bool dense = ctl->dense != 0;
    {
        constexpr int REM_U = 4;
        const i64 p0 = a.rem_base[r], p1 = a.rem_base[r + 1];
        for (i64 pb = p0 + threadIdx.x; pb < p1; pb += (i64)nthr * REM_U) {
            int src[REM_U];
            unsigned tg[REM_U];
#pragma unroll
            for (int u = 0; u < REM_U; ++u) {
                const i64 p = min(pb + (i64)u * nthr, p1 - 1);
                src[u] = a.rem_src[p];
                tg[u] = (unsigned)a.rem_tgt[p];
            }
            T v[REM_U];
            if (dense) {
#pragma unroll
                for (int u = 0; u < REM_U; ++u) v[u] = Sprev[src[u]];
            } else {
                u64 wd[REM_U];
#pragma unroll
                for (int u = 0; u < REM_U; ++u) wd[u] = Sbprev[src[u] >> 6];
#pragma unroll
                for (int u = 0; u < REM_U; ++u) v[u] = ((wd[u] >> (src[u] & 63)) & 1ull) ? Sprev[src[u]] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < REM_U; ++u) {
                if (pb + (i64)u * nthr < p1 && v[u] != (T)0) {
                    atomicAdd(&Fl[tg[u]], (double)v[u]);
                    ++delivered;
                }
            }
        }
    }
    __syncthreads();

    // 3. local rounds (LDS only).  The waves take the range's 64-node chunks from a
    // per-round counter (the next index is requested while a chunk runs), so waves with
    // light chunks take more of them.  Waves run their rounds independently: a wave may
    // reach a chunk that another wave still handles in an earlier round.  Takes are
    // exchanges (the second wave finds only fluid that arrived after the first take, so
    // the fluid stays nonnegative) and the history increment is an atomic add.
    const int nch = (cnt + WAVE - 1) / WAVE;
    double Ld = 0.0;  // this lane's leak, added to the exact sum once at the end
    u64 nodes = 0, edges = 0;
    for (int round = 0; round < rounds; ++round) {
        bool any = false;
        // nodes taken in this round are listed across the wave's chunks and their edges
        // pushed together once the list is full: ln nodes, ltot edge slots (wave-uniform)
        int ln = 0, ltot = 0;
        int nxt = 0;
        if (lane == 0) nxt = atomicAdd(&chunk_ctr[round], 1);
        for (;;) {
            const int ch = __builtin_amdgcn_readfirstlane(nxt);
            if (ch >= nch) break;
            if (lane == 0) nxt = atomicAdd(&chunk_ctr[round], 1);
            const int c = ch * WAVE;
            const int i = c + lane;
            const bool own = i < cnt;
            const int ii = own ? i : c;  // lanes past the range load the chunk's first node
            // the node's degree, offsets and 1/degree load and compute while its fluid
            // value is read
            const double v = lds_load(&Fl[ii]);
            const unsigned deg = Deg[ii] & 0x7fffffffu;
            const unsigned o0 = Off[ii], o1 = Off[ii + 1];
            const double rdeg = recip_count(deg ? deg : 1u);
            double f = 0.0;
            if (own && v != 0.0 && fabs(v) >= thr) f = atomicExch(&Fl[i], 0.0);
            if (__ballot(f != 0.0) == 0) continue;
            any = true;
            int dg = 0;
            unsigned st = 0;
            double q = 0.0;
            if (f != 0.0) {
                atomicAdd(&Dl[i], f);
                if (deg == 0) {
                    Ld += f;
                } else {
                    q = (a.d * f) * rdeg;
                    st = o0;
                    dg = (int)(o1 - o0);
                }
                ++nodes;
            }
            // the nodes with edges to push, in lane order: their edge lists are consecutive
            // in the slot space [0, total) of this chunk
            const u64 pm = __ballot(dg > 0);
            const int nact = __popcll(pm);
            const int inc = wave_incl_scan_dpp(dg);
            const int total = __builtin_amdgcn_readlane(inc, WAVE - 1);
            edges += (lane == 0) ? (u64)total : 0ull;
            if (total == 0) continue;
            const int rk = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(pm >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)pm, 0u));
            if (ln + nact > WAVE || ltot + total > BLD2_SLOTS) {
                bld2_push_list<double>(Fl, Tg, tdelta, ncap, nloc, a.loc_tgt, lb, reinterpret_cast<const int *>(sc_start),
                                  sc_q, sc_bits, ltot, lane);
                ln = 0;
                ltot = 0;
            }
            if (total <= BLD2_SLOTS) {
                if (dg > 0) {
                    const int pos = ltot + inc - dg;
                    sc_start[ln + rk] = (unsigned)((int)st - pos);
                    sc_q[ln + rk] = q;
                    atomicOr(&sc_bits[pos >> 5], 1u << (pos & 31));
                }
                ln += nact;
                ltot += total;
                continue;
            }
            // a chunk with more edge slots than a list holds (rare): its nodes push one at a
            // time, the whole wave striding over the node's local edges
            const long long qb = __double_as_longlong(q);
            for (u64 pend = pm; pend != 0; pend &= pend - 1) {
                const int src = __builtin_ctzll(pend);
                const unsigned st_n = (unsigned)__builtin_amdgcn_readlane((int)st, src);
                const int dg_n = __builtin_amdgcn_readlane(dg, src);
                const unsigned q_lo = (unsigned)__builtin_amdgcn_readlane((int)qb, src);
                const int q_hi = __builtin_amdgcn_readlane((int)(qb >> 32), src);
                const double val = __longlong_as_double(((long long)q_hi << 32) | (long long)q_lo);
                for (int e = lane; e < dg_n; e += WAVE) {
                    const int pp = (int)st_n + e;
                    unsigned t;
                    if (pp < ncap) {
                        t = Tg[tdelta + pp];
                    } else {
                        t = a.loc_tgt[lb + min(pp, nloc - 1)];
                        asm volatile("" : "+v"(t));
                    }
                    atomicAdd(&Fl[t], val);
                }
            }
        }
        if (ltot > 0)
            bld2_push_list<double>(Fl, Tg, tdelta, ncap, nloc, a.loc_tgt, lb, reinterpret_cast<const int *>(sc_start), sc_q,
                              sc_bits, ltot, lane);
        if (!any) break;
    }
    __syncthreads();

    // 4. write back: F, H += dH, cross-range share for the next sweep, residual.
    // Untouched nodes point their H load at the range's first node (an address every
    // thread loads), so the batch needs no branches around its loads.
    // residual: each lane sums its (at most 2 * 2^rb / blockDim) terms in double, raises
    // the sum by 2^-40 relative (far above that rounding) and adds it to the exact sum once
    Limbs R;
    limbs_zero(R);
    double Rd = 0.0;
    for (int i0 = threadIdx.x; i0 < cnt; i0 += nthr * SU) {
        double hv[SU], rwv[SU], dh[SU];
        T sv[SU];
        bool rm[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int i = min(i0 + u * nthr, cnt - 1);
            dh[u] = Dl[i];
            const unsigned df = Deg[i];
            rm[u] = (df & 0x80000000u) != 0;
            sv[u] = (dh[u] != 0.0 && (df & 0x80000000u))
                        ? (T)((a.d * dh[u]) * (1.0 / (double)(df & 0x7fffffffu)))
                        : (T)0;
            hv[u] = a.H[base + (dh[u] != 0.0 ? i : 0)];
            // cross-range out-degree (the graph is unweighted): degree minus local degree
            rwv[u] = (double)((df & 0x7fffffffu) - (Off[i + 1] - Off[i]));
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int i = i0 + u * nthr;
            // the wave's 64 lanes hold 64 consecutive nodes starting at a multiple of 64
            const u64 bits = __ballot(i < cnt && sv[u] != (T)0);
            if (i < cnt) {
                const T v = (T)Fl[i];
                F[base + i] = v;
                if (rm[u]) Snext[base + i] = sv[u];
                if ((threadIdx.x & (WAVE - 1)) == 0) Sbnext[(base + i) >> 6] = bits;
                if (dh[u] != 0.0) a.H[base + i] = hv[u] + dh[u];
                Rd += fabs((double)v);
                if (sv[u] != (T)0) Rd += fabs((double)sv[u]) * rwv[u];
            }
        }
    }
    if (!limbs_add_checked(R, Rd * (1.0 + 0x1p-40), a.K)) bad = 1;
    Limbs leak;
    limbs_zero(leak);
    if (!limbs_add_signed_checked(leak, Ld, a.K)) bad = 1;
    store_residual_partial(R, 0, red, a.partR + (i64)r * PSR);
    store_counter_partial(leak, nodes, edges + delivered, delivered, red, a.partC + (i64)r * PSC);
    if (threadIdx.x == 0 && bad) atomicOr(&ctl->overflow, 1);
}

// Block size, target capacity and LDS bytes of k_bld2_sweep for ranges of 2^rb nodes
// (0 if the fixed part does not fit).
int bld2_config(int rb, int fp32, int *threads, int *tcap, size_t *lds) {
    const int thr = rb <= 11 ? 512 : 1024;
    const size_t fixed = bld2_fixed_lds(rb, fp32, thr);
    // two workgroups per CU (each also holds about 1.3 KB of static LDS) when the fixed
    // part leaves room for a useful target buffer, else one
    const size_t budget = fixed + 2 * 8192 <= 78 * 1024 ? 78 * 1024 : 156 * 1024;
    if (fixed + 2 * 1024 > budget) return 0;
    *threads = thr;
    *tcap = (int)((budget - fixed) / 2) - 2;  // two spare entries for the word-aligned staging
    *lds = fixed + 2 * ((size_t)*tcap + 2);
    return 1;
}

int launch_bld_sweep(const DevGraph &g, SolveState &s, const SweepParams &p, int rounds, hipStream_t st) {
    int thr = 0, tcap = 0;
    size_t lds2 = 0;
    if (!g.weighted && !p.bld_v1 && bld2_config(g.rb, p.fp32, &thr, &tcap, &lds2)) {
        Bld2Args b;
        b.loc_ptr = g.loc_ptr;
        b.loc_tgt = g.loc_tgt;
        b.loc_base = g.loc_base;
        b.deg_flags = g.deg_flags;
        b.rem_src = g.rem_src;
        b.rem_tgt = g.rem_tgt;
        b.rem_base = g.rem_base;
        b.range_order = s.range_order;
        b.n = g.n;
        b.rb = g.rb;
        b.tcap = tcap;
        b.F = s.F;
        b.H = s.H;
        b.S0 = s.S[0];
        b.S1 = s.S[1];
        b.Sb0 = s.Sb[0];
        b.Sb1 = s.Sb[1];
        b.ctl = s.ctl;
        b.d = p.d;
        b.K = p.K;
        b.rounds = rounds;
        b.force = rounds == 0;
        b.partR = s.partR;
        b.partC = s.partC;
        b.range_graph = s.range_graph;
        b.range_cnt = s.range_cnt;
        b.gctl = s.gctl;
        s.nR = s.nC = g.nranges;
        if (p.fp32) k_bld2_sweep<float><<<(unsigned)g.nranges, thr, lds2, st>>>(b);
        else k_bld2_sweep<double><<<(unsigned)g.nranges, thr, lds2, st>>>(b);
        DI_LAUNCH_CHECK();
        return DI_OK;
    }
    BldArgs a = make_bld_args(g, s, p, rounds);
    s.nR = s.nC = g.nranges;
    const size_t lds = bld_lds_bytes(g.rb, p.fp32);
    const unsigned grid = (unsigned)g.nranges;
    if (p.fp32) {
        if (g.weighted) k_bld_sweep<float, true><<<grid, BLD_THREADS, lds, st>>>(a);
        else k_bld_sweep<float, false><<<grid, BLD_THREADS, lds, st>>>(a);
    } else {
        if (g.weighted) k_bld_sweep<double, true><<<grid, BLD_THREADS, lds, st>>>(a);
        else k_bld_sweep<double, false><<<grid, BLD_THREADS, lds, st>>>(a);
    }
    DI_LAUNCH_CHECK();
    return DI_OK;
}

int launch_adj_bld_sweep(const DevGraph &gT, const double *tinv, SolveState &as, const SweepParams &p, int rounds,
                         hipStream_t st) {
    BldArgs a = make_bld_args(gT, as, p, rounds);
    a.tinv = tinv;
    as.nR = as.nC = gT.nranges;
    const size_t lds = bld_lds_bytes(gT.rb, 0);
    const unsigned grid = (unsigned)gT.nranges;
    if (gT.weighted) k_bld_sweep<double, true, true><<<grid, BLD_THREADS, lds, st>>>(a);
    else k_bld_sweep<double, false, true><<<grid, BLD_THREADS, lds, st>>>(a);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Control step: one thread turns the fixed-point sums into the residual, decides
// convergence and sets the next threshold.  Flips the in-flight buffer parity.
// ---------------------------------------------------------------------------
struct FinArgs {
    DevCtl *ctl;
    const u64 *partR, *partC;
    i64 nR, nC;  // slots written by the step's kernels (0: none)
    double d, theta, tol, n_d, zsum, dense_at;
    int K, mode, normalized;
};

constexpr int FIN_THREADS = 256;

__global__ void __launch_bounds__(FIN_THREADS) k_finalize(FinArgs a) {
    DevCtl *c = a.ctl;
    const bool counts = a.mode == FIN_DI || a.mode == FIN_PI || a.mode == FIN_ADJ;
    if (counts && (c->done || c->sweep >= c->budget)) return;
    // add the per-workgroup slots
    u64 v[PSR + PSC];
#pragma unroll
    for (int k = 0; k < PSR + PSC; ++k) v[k] = 0;
    for (i64 b = threadIdx.x; b < a.nR; b += FIN_THREADS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += a.partR[b * PSR + k];
        const u64 m = a.partR[b * PSR + 4];
        v[4] = m > v[4] ? m : v[4];
    }
    for (i64 b = threadIdx.x; b < a.nC; b += FIN_THREADS) {
#pragma unroll
        for (int k = 0; k < PSC; ++k) v[PSR + k] += a.partC[b * PSC + k];
    }
    __shared__ u64 lds[(PSR + PSC) * (FIN_THREADS / WAVE)];
    __shared__ u64 tot[PSR + PSC];
    block_store_partials<PSR + PSC, 1u << 4>(v, lds, tot);
    if (threadIdx.x != 0) return;
    // tot: residual limbs 0-3, max 4, leak limbs 5-8, nodes 9, edges 10, remote 11
    const double R = limbs_to_double_raw(tot[0], tot[1], tot[2], tot[3], a.K);
    for (int k = 0; k < 4; ++k) c->limbsL[k] += tot[5 + k];
    limbs_normalize(c->limbsL);
    const double l = limbs_to_double_signed(c->limbsL[0], c->limbsL[1], c->limbsL[2], c->limbsL[3], a.K);
    const double mx = __longlong_as_double((long long)tot[4]);
    const u64 nodes = tot[9], edges = tot[10], remote = tot[11];
    c->R = R;
    c->maxF = mx;
    if (a.mode == FIN_DELIVER) {
        c->tot_edges += edges;
        c->tot_remote += remote;
        c->parity ^= 1;
        return;
    }
    if (counts) {
        c->tot_nodes += nodes;
        c->tot_edges += edges;
        c->tot_remote += remote;
        c->sweep += 1;
        c->parity ^= 1;
        c->fcount_last = c->fcount;
        // most cross-range entries carried fluid this sweep: the next one reads every
        // in-flight value directly (a bitmap test would cost a random read of its own)
        c->dense = a.mode == FIN_DI && a.dense_at > 0.0 && (double)remote >= a.dense_at;
    }
    double bound;
    if (a.mode == FIN_ADJ || a.mode == FIN_ADJ_INIT) bound = mx / (1.0 - a.d);
    else if (a.normalized && a.mode != FIN_PI) bound = R / (1.0 - a.d - a.d * l / a.zsum);
    else bound = R / (1.0 - a.d);
    if (c->overflow || !(bound == bound)) c->done = 1;
    else if (bound <= a.tol) c->done = 1;
    double thr = ((a.theta * R) / a.n_d) * (1.0 - 0x1p-30);
    // a sweep that diffused nothing (possible only when theta > 1) is followed by one
    // that takes every node with nonzero fluid
    if (a.mode == FIN_DI && nodes == 0) thr = 0.0;
    // deterministic sweeps: an empty active set falls back to all nonzero fluid
    if (a.mode != FIN_PI && mx < thr) c->guard = 1;
    else c->guard = 0;
    c->thr = thr;
}

int launch_finalize(DevCtl *ctl, const SweepParams &p, int mode, hipStream_t st, const u64 *partR, i64 nR,
                    const u64 *partC, i64 nC) {
    FinArgs a;
    a.ctl = ctl;
    a.partR = partR;
    a.partC = partC;
    a.nR = nR;
    a.nC = nC;
    a.d = p.d;
    a.theta = p.theta;
    a.tol = p.tol;
    a.n_d = (double)p.n;
    a.zsum = p.zsum;
    a.dense_at = p.dense_at;
    a.K = p.K;
    a.mode = mode;
    a.normalized = p.normalized;
    k_finalize<<<1, FIN_THREADS, 0, st>>>(a);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Control step of a union of graphs.  One workgroup per graph adds the slots of the
// graph's ranges and moves the graph's state:
//   deterministic sweeps  : certified -> frozen;
//   block-local sweeps    : certified -> finish (the next sweep of its ranges only
//                           delivers the fluid in flight), certified after finishing
//                           -> frozen, else active;
//   start of a call       : certified -> frozen, else active (nothing is in flight);
//   delivery at the end   : certified -> frozen.
// A frozen graph keeps its residual and is left out of every later step of the call.
// Then one workgroup adds the per-graph counters and sets the solve's done flag.
// ---------------------------------------------------------------------------
struct MgFinArgs {
    DevCtl *ctl;
    GraphCtl *gctl;
    const GraphInfo *ginfo;
    const u64 *partR, *partC;
    int use_partC;
    double d, theta, tol;
    int K, mode, det, normalized;
};

__global__ void __launch_bounds__(FIN_THREADS) k_mg_finalize(MgFinArgs a) {
    DevCtl *c = a.ctl;
    const bool counts = a.mode == FIN_DI;
    if (counts && (c->done || c->sweep >= c->budget)) return;
    GraphCtl &gc = a.gctl[blockIdx.x];
    const GraphInfo gi = a.ginfo[blockIdx.x];
    const int st0 = gc.state;
    if (st0 == GS_FROZEN && a.mode != FIN_INIT) {
        if (threadIdx.x == 0) gc.nodes = gc.edges = gc.remote = 0;
        return;
    }
    u64 v[PSR + PSC];
#pragma unroll
    for (int k = 0; k < PSR + PSC; ++k) v[k] = 0;
    for (i64 r = gi.rbeg + threadIdx.x; r < gi.rend; r += FIN_THREADS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += a.partR[r * PSR + k];
        const u64 m = a.partR[r * PSR + 4];
        v[4] = m > v[4] ? m : v[4];
        if (a.use_partC) {
#pragma unroll
            for (int k = 0; k < PSC; ++k) v[PSR + k] += a.partC[r * PSC + k];
        }
    }
    __shared__ u64 lds[(PSR + PSC) * (FIN_THREADS / WAVE)];
    __shared__ u64 tot[PSR + PSC];
    block_store_partials<PSR + PSC, 1u << 4>(v, lds, tot);
    if (threadIdx.x != 0) return;
    const double R = limbs_to_double_raw(tot[0], tot[1], tot[2], tot[3], a.K);
    for (int k = 0; k < 4; ++k) gc.limbsL[k] += tot[5 + k];
    limbs_normalize(gc.limbsL);
    const double l = limbs_to_double_signed(gc.limbsL[0], gc.limbsL[1], gc.limbsL[2], gc.limbsL[3], a.K);
    const double mx = __longlong_as_double((long long)tot[4]);
    const u64 nodes = tot[9];
    gc.nodes = nodes;
    gc.edges = tot[10];
    gc.remote = tot[11];
    gc.R = R;
    gc.maxF = mx;
    const double bound = a.normalized ? R / (1.0 - a.d - a.d * l / gi.zsum) : R / (1.0 - a.d);
    if (!(bound == bound)) atomicOr(&c->overflow, 1);
    const bool cert = bound <= a.tol;
    int st = st0;
    if (a.mode == FIN_DI) {
        if (a.det) st = cert ? GS_FROZEN : GS_ACTIVE;
        else st = cert ? (st0 == GS_FINISH ? GS_FROZEN : GS_FINISH) : GS_ACTIVE;
    } else if (a.mode == FIN_INIT) {
        st = cert ? GS_FROZEN : GS_ACTIVE;
    } else {  // FIN_DELIVER
        st = cert ? GS_FROZEN : GS_ACTIVE;
    }
    if (st == GS_FROZEN && st0 != GS_FROZEN) gc.done_sweep = c->sweep + (counts ? 1 : 0);
    if (a.mode == FIN_INIT && st != GS_FROZEN) gc.done_sweep = -1;
    gc.state = st;
    double thr = ((a.theta * R) / gi.n_d) * (1.0 - 0x1p-30);
    // a block-local sweep that diffused nothing in an active graph (possible only when
    // theta > 1) is followed by one that takes every node with nonzero fluid
    if (a.mode == FIN_DI && !a.det && st0 == GS_ACTIVE && nodes == 0) thr = 0.0;
    gc.guard = mx < thr ? 1 : 0;
    gc.thr = thr;
}

__global__ void __launch_bounds__(FIN_THREADS) k_mg_control(DevCtl *c, const GraphCtl *gctl, i64 G, int mode) {
    const bool counts = mode == FIN_DI;
    if (counts && (c->done || c->sweep >= c->budget)) return;
    u64 v[4] = {0, 0, 0, 0};  // nodes, edges, remote deliveries, graphs not frozen
    for (i64 g = threadIdx.x; g < G; g += FIN_THREADS) {
        const GraphCtl &gc = gctl[g];
        v[0] += gc.nodes;
        v[1] += gc.edges;
        v[2] += gc.remote;
        v[3] += gc.state != GS_FROZEN ? 1 : 0;
    }
    __shared__ u64 lds[4 * (FIN_THREADS / WAVE)];
    __shared__ u64 tot[4];
    block_store_partials<4>(v, lds, tot);
    if (threadIdx.x != 0) return;
    // the solve's residual: the largest per-graph residual (each graph has its own bound)
    double R = 0.0, M = 0.0;
    for (i64 g = 0; g < G; ++g) {
        R = gctl[g].R > R ? gctl[g].R : R;
        M = gctl[g].maxF > M ? gctl[g].maxF : M;
    }
    c->R = R;
    c->maxF = M;
    if (counts) {
        c->tot_nodes += tot[0];
        c->tot_edges += tot[1];
        c->tot_remote += tot[2];
        c->sweep += 1;
        c->parity ^= 1;
        c->fcount_last = c->fcount;
    } else if (mode == FIN_DELIVER) {
        c->tot_edges += tot[1];
        c->tot_remote += tot[2];
        c->parity ^= 1;
    }
    c->done = (tot[3] == 0 || c->overflow) ? 1 : 0;
}

int launch_mg_finalize(SolveState &s, DevCtl *ctl, const SweepParams &p, int mode, int det, hipStream_t st) {
    MgFinArgs a;
    a.ctl = ctl;
    a.gctl = s.gctl;
    a.ginfo = s.ginfo;
    a.partR = s.partR;
    a.partC = s.partC;
    a.use_partC = mode != FIN_INIT;
    a.d = p.d;
    a.theta = p.theta;
    a.tol = p.tol;
    a.K = p.K;
    a.mode = mode;
    a.det = det;
    a.normalized = p.normalized;
    k_mg_finalize<<<(unsigned)s.n_graphs, FIN_THREADS, 0, st>>>(a);
    DI_LAUNCH_CHECK();
    k_mg_control<<<1, FIN_THREADS, 0, st>>>(ctl, s.gctl, s.n_graphs, mode);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Residual of F (fixed point) and max |F|: initial state and deterministic sweeps.
// ---------------------------------------------------------------------------
// Node loop of a grid-stride kernel, or, for a union of graphs, of the range whose
// number is the workgroup's (one partial-sum slot per range).
struct NodeLoop {
    i64 i0, i1, step;
};

__device__ __forceinline__ NodeLoop node_loop(i64 n, const int *range_graph, int rb) {
    NodeLoop L;
    if (range_graph) {
        const i64 base = (i64)blockIdx.x << rb;
        L.i0 = base + threadIdx.x;
        L.i1 = min(n, base + ((i64)1 << rb));
        L.step = blockDim.x;
    } else {
        L.i0 = (i64)blockIdx.x * blockDim.x + threadIdx.x;
        L.i1 = n;
        L.step = (i64)gridDim.x * blockDim.x;
    }
    return L;
}

template <typename T>
__global__ void __launch_bounds__(256) k_reduce_F(const T *__restrict__ F, i64 n, int K, DevCtl *ctl, u64 *partR,
                                                  const int *range_graph, const GraphCtl *gctl, int rb,
                                                  int skip_frozen) {
    __shared__ u64 red[PSR * 4];
    __shared__ int bad;
    if (range_graph && skip_frozen && gctl[range_graph[blockIdx.x]].state == GS_FROZEN) return;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    Limbs R;
    limbs_zero(R);
    u64 mx = 0;
    const NodeLoop L = node_loop(n, range_graph, rb);
    for (i64 i = L.i0; i < L.i1; i += L.step) {
        const double v = fabs((double)F[i]);
        if (!limbs_add_checked(R, v, K)) bad = 1;
        const u64 b = (u64)__double_as_longlong(v);
        mx = b > mx ? b : mx;
    }
    store_residual_partial(R, mx, red, partR + (i64)blockIdx.x * PSR);
    if (threadIdx.x == 0 && bad) atomicOr(&ctl->overflow, 1);
}

int launch_reduce_F(const DevGraph &g, SolveState &s, const SweepParams &p, hipStream_t st, int skip_frozen) {
    const unsigned grid = s.range_graph ? (unsigned)g.nranges : grid_for(g.n, 256, REDUCE_GRID);
    if (p.fp32)
        k_reduce_F<float><<<grid, 256, 0, st>>>((const float *)s.F, g.n, p.K, s.ctl, s.partR, s.range_graph, s.gctl,
                                                g.rb, skip_frozen);
    else
        k_reduce_F<double><<<grid, 256, 0, st>>>((const double *)s.F, g.n, p.K, s.ctl, s.partR, s.range_graph,
                                                 s.gctl, g.rb, skip_frozen);
    DI_LAUNCH_CHECK();
    s.nR = grid;
    return DI_OK;
}

// Exact signed sums of a node vector per graph (one graph: one sum), for the mass balance
// sum F + (1-d) sum H + d l = (1-d) sum Z that equation HnFn implies (the columns of P sum
// to 1 except at dangling nodes, Section 2.1).  Per-workgroup two's-complement limb slots
// (one per range in a union of graphs), then one workgroup per graph adds its slots.
template <typename T>
__global__ void __launch_bounds__(256) k_sum_signed(const T *__restrict__ v, i64 n, int K, u64 *part,
                                                    const int *range_graph, int rb) {
    __shared__ u64 red[4 * 4];
    Limbs S;
    limbs_zero(S);
    const NodeLoop L = node_loop(n, range_graph, rb);
    for (i64 i = L.i0; i < L.i1; i += L.step) limbs_add_signed(S, (double)v[i], K);
    u64 w[4] = {S.l[0], S.l[1], S.l[2], S.l[3]};
    block_store_partials<4>(w, red, part + (i64)blockIdx.x * PSR);
}

__global__ void __launch_bounds__(256) k_sum_slots(const u64 *__restrict__ part, i64 nslots,
                                                   const GraphInfo *__restrict__ gi, int K, double *out) {
    __shared__ u64 red[4 * 4];
    __shared__ u64 tot[4];
    i64 b = 0, e = nslots;
    if (gi) {
        b = gi[blockIdx.x].rbeg;
        e = gi[blockIdx.x].rend;
    }
    u64 v[4] = {0, 0, 0, 0};
    for (i64 q = b + threadIdx.x; q < e; q += blockDim.x)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += part[q * PSR + k];
    block_store_partials<4>(v, red, tot);
    if (threadIdx.x == 0) out[blockIdx.x] = limbs_to_double_signed(tot[0], tot[1], tot[2], tot[3], K);
}

int launch_node_sums(const DevGraph &g, SolveState &s, const void *v, int is_float, int K, u64 *part, double *out,
                     hipStream_t st) {
    const unsigned grid = s.range_graph ? (unsigned)g.nranges : grid_for(g.n, 256, REDUCE_GRID);
    if (is_float) k_sum_signed<float><<<grid, 256, 0, st>>>((const float *)v, g.n, K, part, s.range_graph, g.rb);
    else k_sum_signed<double><<<grid, 256, 0, st>>>((const double *)v, g.n, K, part, s.range_graph, g.rb);
    DI_LAUNCH_CHECK();
    const unsigned G = s.range_graph ? (unsigned)s.n_graphs : 1u;
    k_sum_slots<<<G, 256, 0, st>>>(part, grid, s.range_graph ? s.ginfo : nullptr, K, out);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Deterministic synchronous sweep (snapshot semantics):
//   A = { i : F_i != 0 and |F_i| >= thr } (all nonzero when guard is set);
//   snap_i = (d f_i) inv_s_i for active non-dangling i, else 0; H_i += f_i; F_i = 0;
//   then F_j = left fold over IN row j (ascending source) of snap_src (* w), starting
//   from F_j, in double, rounded once to the fluid type.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_det_snapshot(T *F, double *H, double *snap, const double *__restrict__ inv_s,
                                                      const i64 *__restrict__ out_ptr, i64 n, double d, int K,
                                                      DevCtl *ctl, int *frontier, u64 *partC,
                                                      const int *range_graph, const GraphCtl *gctl, int rb) {
    __shared__ u64 red[PSC * 4];
    if (ctl->done || ctl->sweep >= ctl->budget) return;
    double thr = ctl->thr;
    int guard = ctl->guard;
    if (range_graph) {
        const GraphCtl &gc = gctl[range_graph[blockIdx.x]];
        if (gc.state == GS_FROZEN) return;
        thr = gc.thr;
        guard = gc.guard;
    }
    Limbs leak;
    limbs_zero(leak);
    u64 nodes = 0, edges = 0;
    const NodeLoop L = node_loop(n, range_graph, rb);
    for (i64 i = L.i0; i < L.i1; i += L.step) {
        const T v = F[i];
        const bool act = v != (T)0 && (guard || fabs((double)v) >= thr);
        double q = 0.0;
        if (act) {
            const double f = (double)v;
            H[i] += f;
            F[i] = (T)0;
            const double inv = inv_s[i];
            if (inv == 0.0) limbs_add_signed(leak, f, K);
            else q = (d * f) * inv;
            ++nodes;
            edges += (u64)(out_ptr[i + 1] - out_ptr[i]);
        }
        if (frontier) {  // one counter update per wave: base + rank among the wave's actives
            const u64 mask = __ballot(act);
            u64 wbase = 0;
            if ((threadIdx.x & 63) == 0 && mask) wbase = atomicAdd(&ctl->fcount, (u64)__popcll(mask));
            wbase = __shfl(wbase, 0, WAVE);
            if (act) frontier[wbase + __popcll(mask & ((1ull << (threadIdx.x & 63)) - 1ull))] = (int)i;
        }
        snap[i] = q;
    }
    store_counter_partial(leak, nodes, edges, 0, red, partC + (i64)blockIdx.x * PSC);
}

template <typename T, bool WTD>
__global__ void __launch_bounds__(256) k_det_pull(T *F, const double *__restrict__ snap, const i64 *__restrict__ in_ptr,
                                                  const int *__restrict__ in_idx, const float *__restrict__ in_w, i64 n,
                                                  DevCtl *ctl, const int *range_graph, const GraphCtl *gctl, int rb) {
    if (ctl->done || ctl->sweep >= ctl->budget) return;
    const i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    // rows of a frozen graph: its snapshot values are stale and its fluid stays put
    if (range_graph && gctl[range_graph[j >> rb]].state == GS_FROZEN) return;
    double acc = (double)F[j];
    const i64 p1 = in_ptr[j + 1];
    for (i64 p = in_ptr[j]; p < p1; ++p) {
        if (WTD) acc += snap[in_idx[p]] * (double)in_w[p];
        else acc += snap[in_idx[p]];
    }
    F[j] = (T)acc;
}

__global__ void k_det_begin(DevCtl *ctl) {
    if (ctl->done || ctl->sweep >= ctl->budget) return;
    ctl->fcount = 0;
}

int launch_det_sweep(const DevGraph &g, SolveState &s, const SweepParams &p, hipStream_t st) {
    const unsigned grid = s.range_graph ? (unsigned)g.nranges : grid_for(g.n, 256, SNAP_GRID);
    k_det_begin<<<1, 1, 0, st>>>(s.ctl);
    DI_LAUNCH_CHECK();
    if (p.fp32)
        k_det_snapshot<float><<<grid, 256, 0, st>>>((float *)s.F, s.H, s.snap, g.inv_s, g.out_ptr, g.n, p.d, p.K, s.ctl,
                                                    s.frontier, s.partC, s.range_graph, s.gctl, g.rb);
    else
        k_det_snapshot<double><<<grid, 256, 0, st>>>((double *)s.F, s.H, s.snap, g.inv_s, g.out_ptr, g.n, p.d, p.K,
                                                     s.ctl, s.frontier, s.partC, s.range_graph, s.gctl, g.rb);
    DI_LAUNCH_CHECK();
    const i64 nC = grid;
    const unsigned gridr = grid_for(g.n, 256);
#define DI_PULL(TT, WW)                                                                                          \
    k_det_pull<TT, WW><<<gridr, 256, 0, st>>>((TT *)s.F, s.snap, g.in_ptr, g.in_idx, g.in_w, g.n, s.ctl,          \
                                              s.range_graph, s.gctl, g.rb)
    if (p.fp32) {
        if (g.weighted) DI_PULL(float, true);
        else DI_PULL(float, false);
    } else {
        if (g.weighted) DI_PULL(double, true);
        else DI_PULL(double, false);
    }
#undef DI_PULL
    DI_LAUNCH_CHECK();
    DI_TRY(launch_reduce_F(g, s, p, st, 1));
    s.nC = nC;
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Power iteration (Section 2.2): x_{k+1} = d P x_k + (1-d) Z as a pull over IN with
// xt_j = x_j / s_j prepared by the previous iteration.  One wave per row block:
// the block's entries are gathered into LDS with coalesced index reads, then each
// lane folds one row.  Long rows are summed by segments first (k_pi_segments).
//
// The same row pull recomputes the fluid from the history, in double (PM_REF):
// F = F_0 + d P H - H, the fluid that equation HnFn assigns to H.  Float fluid gathers
// a rounding error at every push; recomputing it restores the identity, so that
// |F|_1 / (1-d) certifies |x - H|_1 again (Theorem 1).
//
// Over OUT instead of IN it is the adjoint sweep's pull (PM_ADJ): row j gathers the
// snapshot d f_i of its out-neighbours i and adds (1/s_j) * sum_e snap_i w_e to F_j (the
// transposed diffusion, see k_adj_pull; here lanes share the row and the order of the
// additions is not the row order, so it is the fast adjoint, not the reproducible one).
// ---------------------------------------------------------------------------
constexpr int PI_WAVES = 4;
constexpr int PM_PI = 0, PM_REF = 1, PM_ADJ = 2, PM_PROD = 3;

struct PiArgs {
    const i64 *rb_start;
    const int *seg_first, *seg_count;
    const i64 *seg_b, *seg_e;
    double *partial;
    const i64 *in_ptr;
    const int *in_idx;
    const float *in_w;
    const double *inv_s;
    const double *Z;
    double zc;
    double *X0, *X1;
    void *XT0, *XT1;
    DevCtl *ctl;
    double d;
    i64 n, nrb, nseg;
    int K;
    u64 *partR;
    // fluid recomputation: ht = H / s (double), F_0, H, the fluid written;
    // adjoint pull: ht = the snapshot, Fout = the adjoint fluid (read and written)
    const double *ht;
    const double *F0;
    const double *H;
    void *Fout;
};

// TX: type of the gathered values; MODE: PM_PI, PM_REF (always runs), PM_ADJ or PM_PROD
// (always runs)
template <typename TX, bool WTD, int MODE>
__global__ void __launch_bounds__(256) k_pi_segments(PiArgs a) {
    __shared__ double red[256 / WAVE];
    DevCtl *ctl = a.ctl;
    if (MODE != PM_REF && MODE != PM_PROD && (ctl->done || ctl->sweep >= ctl->budget)) return;
    const TX *xt = MODE != PM_PI ? reinterpret_cast<const TX *>(a.ht)
                                 : reinterpret_cast<const TX *>(ctl->parity ? a.XT1 : a.XT0);
    const i64 sg = blockIdx.x;
    const i64 b = a.seg_b[sg], e = a.seg_e[sg];
    double acc = 0.0;
    constexpr int SU = 8;
    for (i64 pb = b + threadIdx.x; pb < e; pb += (i64)blockDim.x * SU) {
        int src[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) src[u] = a.in_idx[min(pb + (i64)u * blockDim.x, e - 1)];
        double v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) v[u] = (double)xt[src[u]];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const i64 p = pb + (i64)u * blockDim.x;
            if (p < e) acc += WTD ? v[u] * (double)a.in_w[p] : v[u];
        }
    }
    acc = wave_sum_f64(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
        a.partial[sg] = s;
    }
}

// T: type of x / s in power iteration, of the fluid in the recomputation (PM_REF);
// the adjoint pull (PM_ADJ) and the plain product (PM_PROD: out = P v with ht = v / s)
// are double throughout
template <typename T, bool WTD, int MODE>
__global__ void __launch_bounds__(PI_WAVES * WAVE) k_pi_rows(PiArgs a) {
    constexpr bool REF = MODE == PM_REF, ADJ = MODE == PM_ADJ, PROD = MODE == PM_PROD;
    using TX = typename std::conditional<MODE != PM_PI, double, T>::type;
    __shared__ double tile[PI_WAVES][RB_NNZ];
    __shared__ u64 red[PSR * PI_WAVES];
    __shared__ int bad;
    DevCtl *ctl = a.ctl;
    if (!REF && !PROD && (ctl->done || ctl->sweep >= ctl->budget)) return;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int par = MODE != PM_PI ? 0 : ctl->parity;
    const TX *xt = MODE != PM_PI ? reinterpret_cast<const TX *>(a.ht)
                                 : reinterpret_cast<const TX *>(par ? a.XT1 : a.XT0);
    u64 mx = 0;  // adjoint: largest |F| (as bits of a nonnegative double)
    T *xtn = reinterpret_cast<T *>(par ? a.XT0 : a.XT1);
    const double *x = par ? a.X1 : a.X0;
    double *xn = par ? a.X0 : a.X1;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
    Limbs R;
    limbs_zero(R);
    // each wave walks work items with a stride of the whole grid
    for (i64 rbk = (i64)blockIdx.x * PI_WAVES + w; rbk < a.nrb; rbk += (i64)gridDim.x * PI_WAVES) {
        const i64 r0 = a.rb_start[rbk], r1 = a.rb_start[rbk + 1];
        const int sf = a.seg_first[rbk];
        double acc = 0.0;
        i64 row = -1;
        if (sf >= 0) {
            if (lane == 0) {
                row = r0;
                const int sc = a.seg_count[rbk];
                for (int k = 0; k < sc; ++k) acc += a.partial[sf + k];
            }
        } else if (sf == RB_KIND_VECTOR) {
            // one row over the wave: lane l sums entries l, l+64, ... in order, then a
            // fixed butterfly combines the lanes
            const i64 e0 = a.in_ptr[r0], e1 = a.in_ptr[r0 + 1];
            constexpr int VU = 16;
            for (i64 eb = e0 + lane; eb < e1; eb += (i64)WAVE * VU) {
                int src[VU];
#pragma unroll
                for (int u = 0; u < VU; ++u) src[u] = a.in_idx[min(eb + (i64)u * WAVE, e1 - 1)];
                double v[VU];
#pragma unroll
                for (int u = 0; u < VU; ++u) v[u] = (double)xt[src[u]];
#pragma unroll
                for (int u = 0; u < VU; ++u) {
                    const i64 p = eb + (i64)u * WAVE;
                    if (p < e1) acc += WTD ? v[u] * (double)a.in_w[p] : v[u];
                }
            }
            acc = wave_sum_f64(acc);
            if (lane == 0) row = r0;
        } else {
            const i64 e0 = a.in_ptr[r0], e1 = a.in_ptr[r1];
            const int len = (int)(e1 - e0);
            // stage the block's entries (at most RB_NNZ = 16 per lane): all index loads
            // first, then all gathers
            constexpr int PU = RB_NNZ / WAVE;
            if (len > 0) {
                // slots past the end re-read entry len-1 (a valid address) and store nothing
                int src[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) src[u] = a.in_idx[e0 + min(u * WAVE + lane, len - 1)];
                double v[PU];
#pragma unroll
                for (int u = 0; u < PU; ++u) v[u] = (double)xt[src[u]];
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    const int k = u * WAVE + lane;
                    if (k < len) tile[w][k] = WTD ? v[u] * (double)a.in_w[e0 + k] : v[u];
                }
            }
            wave_sync_lds();
            if (r0 + lane < r1) {
                row = r0 + lane;
                const int kb = (int)(a.in_ptr[row] - e0), ke = (int)(a.in_ptr[row + 1] - e0);
                for (int k = kb; k < ke; ++k) acc += tile[w][k];
            }
        }
        if (row >= 0) {
            if (PROD) {
                reinterpret_cast<double *>(a.Fout)[row] = acc;
            } else if (REF) {
                const double f = (a.F0[row] + a.d * acc) - a.H[row];
                reinterpret_cast<T *>(a.Fout)[row] = (T)f;
            } else if (ADJ) {
                double *Fa = reinterpret_cast<double *>(a.Fout);
                const double f = Fa[row] + a.inv_s[row] * acc;
                Fa[row] = f;
                if (!limbs_add_checked(R, fabs(f), a.K)) bad = 1;
                const u64 b = (u64)__double_as_longlong(fabs(f));
                mx = b > mx ? b : mx;
            } else {
                const double y = a.d * acc + (a.Z ? (1.0 - a.d) * a.Z[row] : a.zc);
                xn[row] = y;
                xtn[row] = (T)(y * a.inv_s[row]);
                if (!limbs_add_checked(R, fabs(y - x[row]), a.K)) bad = 1;
            }
        }
        wave_sync_lds();  // the next item reuses this wave's tile
    }
    if (REF || PROD) return;  // the residual of the recomputed fluid is summed by k_reduce_F
    store_residual_partial(R, mx, red, a.partR + (i64)blockIdx.x * PSR);
    if (threadIdx.x == 0 && bad) atomicOr(&ctl->overflow, 1);
}

static PiArgs make_pi_args(const DevGraph &g, const RowBlocks &rb, SolveState &s, const SweepParams &p) {
    PiArgs a;
    a.rb_start = rb.start;
    a.seg_first = rb.seg_first;
    a.seg_count = rb.seg_count;
    a.seg_b = rb.seg_b;
    a.seg_e = rb.seg_e;
    a.partial = rb.partial;
    a.in_ptr = g.in_ptr;
    a.in_idx = g.in_idx;
    a.in_w = g.in_w;
    a.inv_s = g.inv_s;
    a.Z = s.Z;
    a.zc = s.zc;
    a.X0 = s.X[0];
    a.X1 = s.X[1];
    a.XT0 = s.XT[0];
    a.XT1 = s.XT[1];
    a.ctl = s.pctl;
    a.d = p.d;
    a.n = g.n;
    a.nrb = rb.nrb;
    a.nseg = rb.nseg;
    a.K = p.K;
    a.partR = s.partR;
    a.ht = nullptr;
    a.F0 = nullptr;
    a.H = nullptr;
    a.Fout = nullptr;
    return a;
}

// weighted: whether the pulled edges carry weights (a.in_w)
template <int MODE>
static int launch_row_pull(PiArgs &a, bool weighted, const RowBlocks &rb, int fp32, hipStream_t st) {
    if (rb.nseg > 0) {
        const unsigned gs = (unsigned)rb.nseg;
        if (fp32 && MODE == PM_PI) {
            if (weighted) k_pi_segments<float, true, MODE><<<gs, 256, 0, st>>>(a);
            else k_pi_segments<float, false, MODE><<<gs, 256, 0, st>>>(a);
        } else {
            if (weighted) k_pi_segments<double, true, MODE><<<gs, 256, 0, st>>>(a);
            else k_pi_segments<double, false, MODE><<<gs, 256, 0, st>>>(a);
        }
        DI_LAUNCH_CHECK();
    }
    const unsigned grid = grid_for(rb.nrb, PI_WAVES, PI_GRID);
    if (fp32 && MODE != PM_ADJ) {
        if (weighted) k_pi_rows<float, true, MODE><<<grid, PI_WAVES * WAVE, 0, st>>>(a);
        else k_pi_rows<float, false, MODE><<<grid, PI_WAVES * WAVE, 0, st>>>(a);
    } else {
        if (weighted) k_pi_rows<double, true, MODE><<<grid, PI_WAVES * WAVE, 0, st>>>(a);
        else k_pi_rows<double, false, MODE><<<grid, PI_WAVES * WAVE, 0, st>>>(a);
    }
    DI_LAUNCH_CHECK();
    return DI_OK;
}

int launch_pi_iteration(const DevGraph &g, const RowBlocks &rb, SolveState &s, const SweepParams &p, hipStream_t st) {
    PiArgs a = make_pi_args(g, rb, s, p);
    s.nR = grid_for(rb.nrb, PI_WAVES, PI_GRID);
    return launch_row_pull<PM_PI>(a, g.weighted, rb, p.fp32, st);
}

__global__ void k_scaled_by_inv_s(const double *__restrict__ H, const double *__restrict__ inv_s, i64 n,
                                  double *ht) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        ht[i] = H[i] * inv_s[i];
}

// out_i = (P v)_i as a left fold over IN row i in ascending source order, each term
// (w_e / s_j) v_j or (1 / s_j) v_j: the order and rounding of the oracle's product
__global__ void k_fold_P(const i64 *__restrict__ in_ptr, const int *__restrict__ in_idx, const float *__restrict__ in_w,
                         const double *__restrict__ inv_s, const double *__restrict__ v, i64 n, double *out) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (i64 p = in_ptr[i]; p < in_ptr[i + 1]; ++p) {
            const int j = in_idx[p];
            acc += (in_w ? (double)in_w[p] * inv_s[j] : inv_s[j]) * v[j];
        }
        out[i] = acc;
    }
}

int launch_P_times(const DevGraph &g, const RowBlocks &rb, const double *v, double *ht, double *out, int ordered,
                   hipStream_t st) {
    if (ordered) {
        k_fold_P<<<grid_for(g.n, 256, 16384), 256, 0, st>>>(g.in_ptr, g.in_idx, g.in_w, g.inv_s, v, g.n, out);
        DI_LAUNCH_CHECK();
        return DI_OK;
    }
    k_scaled_by_inv_s<<<grid_for(g.n, 256, 16384), 256, 0, st>>>(v, g.inv_s, g.n, ht);
    DI_LAUNCH_CHECK();
    PiArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rb_start = rb.start;
    a.seg_first = rb.seg_first;
    a.seg_count = rb.seg_count;
    a.seg_b = rb.seg_b;
    a.seg_e = rb.seg_e;
    a.partial = rb.partial;
    a.in_ptr = g.in_ptr;
    a.in_idx = g.in_idx;
    a.in_w = g.in_w;
    a.inv_s = g.inv_s;
    a.n = g.n;
    a.nrb = rb.nrb;
    a.nseg = rb.nseg;
    a.ht = ht;
    a.Fout = out;
    return launch_row_pull<PM_PROD>(a, g.weighted, rb, 0, st);
}

int launch_refine_fluid(const DevGraph &g, const RowBlocks &rb, SolveState &s, const SweepParams &p, double *ht,
                        hipStream_t st) {
    k_scaled_by_inv_s<<<grid_for(g.n, 256, 16384), 256, 0, st>>>(s.H, g.inv_s, g.n, ht);
    DI_LAUNCH_CHECK();
    PiArgs a = make_pi_args(g, rb, s, p);
    a.ht = ht;
    a.F0 = s.F0;
    a.H = s.H;
    a.Fout = s.F;
    return launch_row_pull<PM_REF>(a, g.weighted, rb, p.fp32, st);
}

__global__ void k_fill_bytes_zero(unsigned *p, i64 words) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (i64)gridDim.x * blockDim.x) p[i] = 0u;
}

int launch_fill_zero(void *p, i64 bytes, hipStream_t st) {
    const i64 words = (bytes + 3) / 4;
    k_fill_bytes_zero<<<grid_for(words, 256, 8192), 256, 0, st>>>((unsigned *)p, words);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

__global__ void k_round_to_float(const double *__restrict__ src, i64 n, float *dst) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

int launch_init_fluid(const double *F0, void *F, int fp32, i64 count, hipStream_t st) {
    if (fp32) {
        k_round_to_float<<<grid_for(count, 256, 16384), 256, 0, st>>>(F0, count, (float *)F);
        DI_LAUNCH_CHECK();
    } else {
        DI_HIP(hipMemcpyAsync(F, F0, sizeof(double) * count, hipMemcpyDeviceToDevice, st));
    }
    return DI_OK;
}

int launch_pi_init(const DevGraph &g, SolveState &s, const SweepParams &p, hipStream_t st) {
    DI_TRY(launch_fill_zero(s.X[0], g.n * 8, st));
    DI_TRY(launch_fill_zero(s.X[1], g.n * 8, st));
    DI_TRY(launch_fill_zero(s.XT[0], g.n * (p.fp32 ? 4 : 8), st));
    DI_TRY(launch_fill_zero(s.XT[1], g.n * (p.fp32 ? 4 : 8), st));
    return DI_OK;
}

template <typename T>
__global__ void k_to_double(const T *__restrict__ src, i64 n, double *dst) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

int launch_copy_fluid_to_double(const void *F, int fp32, i64 n, double *dst, hipStream_t st) {
    if (fp32) k_to_double<float><<<grid_for(n, 256, 8192), 256, 0, st>>>((const float *)F, n, dst);
    else k_to_double<double><<<grid_for(n, 256, 8192), 256, 0, st>>>((const double *)F, n, dst);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

__global__ void k_scaled_copy(const double *__restrict__ src, double scale, i64 n, double *dst) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        dst[i] = scale * src[i];
}

int launch_scaled_copy(const double *H, double scale, i64 n, double *dst, hipStream_t st) {
    k_scaled_copy<<<grid_for(n, 256, 8192), 256, 0, st>>>(H, scale, n, dst);
    DI_LAUNCH_CHECK();
    return DI_OK;
}

// ---------------------------------------------------------------------------
// Row blocks (host partition of a row-pointer array copied from the device).
// ---------------------------------------------------------------------------
int build_row_blocks(RowBlocks &rb, const i64 *d_ptr, i64 n, hipStream_t st) {
    std::vector<i64> ptr((size_t)n + 1);
    DI_HIP(hipMemcpyAsync(ptr.data(), d_ptr, sizeof(i64) * (size_t)(n + 1), hipMemcpyDeviceToHost, st));
    DI_HIP(hipStreamSynchronize(st));
    std::vector<i64> start;
    std::vector<int> sf, sc;
    std::vector<i64> sb, se;
    i64 r = 0;
    while (r < n) {
        const i64 len = ptr[r + 1] - ptr[r];
        if (len > RB_SEG) {
            start.push_back(r);
            sf.push_back((int)sb.size());
            int cnt = 0;
            for (i64 b = ptr[r]; b < ptr[r + 1]; b += RB_SEG) {
                sb.push_back(b);
                se.push_back(std::min(b + RB_SEG, ptr[r + 1]));
                ++cnt;
            }
            sc.push_back(cnt);
            ++r;
            continue;
        }
        if (len > RB_SHORT) {
            start.push_back(r);
            sf.push_back(RB_KIND_VECTOR);
            sc.push_back(0);
            ++r;
            continue;
        }
        const i64 r0 = r;
        while (r < n && r - r0 < RB_ROWS && ptr[r + 1] - ptr[r] <= RB_SHORT && ptr[r + 1] - ptr[r0] <= RB_NNZ) ++r;
        start.push_back(r0);
        sf.push_back(RB_KIND_SHORT);
        sc.push_back(0);
    }
    start.push_back(n);
    rb.nrb = (i64)sf.size();
    rb.nseg = (i64)sb.size();
    DI_HIP(dev_malloc((void **)&rb.start, sizeof(i64) * start.size()));
    DI_HIP(dev_malloc((void **)&rb.seg_first, sizeof(int) * std::max<size_t>(sf.size(), 1)));
    DI_HIP(dev_malloc((void **)&rb.seg_count, sizeof(int) * std::max<size_t>(sc.size(), 1)));
    DI_HIP(dev_malloc((void **)&rb.seg_b, sizeof(i64) * std::max<size_t>(sb.size(), 1)));
    DI_HIP(dev_malloc((void **)&rb.seg_e, sizeof(i64) * std::max<size_t>(se.size(), 1)));
    DI_HIP(dev_malloc((void **)&rb.partial, sizeof(double) * std::max<size_t>(sb.size(), 1)));
    DI_HIP(hipMemcpyAsync(rb.start, start.data(), sizeof(i64) * start.size(), hipMemcpyHostToDevice, st));
    if (!sf.empty()) {
        DI_HIP(hipMemcpyAsync(rb.seg_first, sf.data(), sizeof(int) * sf.size(), hipMemcpyHostToDevice, st));
        DI_HIP(hipMemcpyAsync(rb.seg_count, sc.data(), sizeof(int) * sc.size(), hipMemcpyHostToDevice, st));
    }
    if (!sb.empty()) {
        DI_HIP(hipMemcpyAsync(rb.seg_b, sb.data(), sizeof(i64) * sb.size(), hipMemcpyHostToDevice, st));
        DI_HIP(hipMemcpyAsync(rb.seg_e, se.data(), sizeof(i64) * se.size(), hipMemcpyHostToDevice, st));
    }
    DI_HIP(hipStreamSynchronize(st));
    return DI_OK;
}

void free_row_blocks(RowBlocks &rb) {
    void *ps[] = {rb.start, rb.seg_first, rb.seg_count, rb.seg_b, rb.seg_e, rb.partial};
    for (void *p : ps)
        if (p) (void)dev_free(p);
    rb = RowBlocks{};
}

}  // namespace di

namespace di {

int set_kernel_attributes() {
    static bool done = false;
    if (done) return DI_OK;
    const int maxb = 160 * 1024 - 2048;
    DI_HIP(hipFuncSetAttribute((const void *)k_bld_sweep<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld_sweep<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld_sweep<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld_sweep<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld_sweep<double, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld_sweep<double, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld2_sweep<float>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    DI_HIP(hipFuncSetAttribute((const void *)k_bld2_sweep<double>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb));
    done = true;
    return DI_OK;
}

}  // namespace di

namespace di {

// ---------------------------------------------------------------------------
// Adjoint: diffusion of signed fluid on P^T.  Node i's diffusion sends
// d f_i P[i][j] to every j with an edge j -> i; as a pull over OUT row j:
//   F_j += sum over out-edges e of j of snap[target(e)] * P_e,  P_e = w_e / s_j,
// with snap_i = d f_i on the active set (left fold in row order, double).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adj_snapshot(double *F, double *H, double *snap, const i64 *__restrict__ in_ptr,
                                                      i64 n, double d, DevCtl *ctl, u64 *partC) {
    __shared__ u64 red[PSC * 4];
    if (ctl->done || ctl->sweep >= ctl->budget) return;
    const double thr = ctl->thr;
    const int guard = ctl->guard;
    u64 nodes = 0, edges = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const double v = F[i];
        const bool act = v != 0.0 && (guard || fabs(v) >= thr);
        double q = 0.0;
        if (act) {
            H[i] += v;
            F[i] = 0.0;
            q = d * v;
            ++nodes;
            edges += (u64)(in_ptr[i + 1] - in_ptr[i]);
        }
        snap[i] = q;
    }
    Limbs none;
    limbs_zero(none);
    store_counter_partial(none, nodes, edges, 0, red, partC + (i64)blockIdx.x * PSC);
}

template <bool WTD>
__global__ void __launch_bounds__(256) k_adj_pull(double *F, const double *__restrict__ snap, const i64 *__restrict__ out_ptr,
                                                  const int *__restrict__ out_idx, const float *__restrict__ w,
                                                  const double *__restrict__ inv_s, i64 n, DevCtl *ctl) {
    if (ctl->done || ctl->sweep >= ctl->budget) return;
    const i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double acc = F[j];
    const double inv = inv_s[j];
    const i64 e1 = out_ptr[j + 1];
    for (i64 e = out_ptr[j]; e < e1; ++e) {
        const double P = WTD ? (double)w[e] * inv : inv;
        acc += snap[out_idx[e]] * P;
    }
    F[j] = acc;
}

int launch_adj_sweep(const DevGraph &g, double *F, double *H, double *snap, DevCtl *ctl, const SweepParams &p,
                     hipStream_t st, u64 *partR, u64 *partC, i64 *nR, i64 *nC) {
    const unsigned gs = grid_for(g.n, 256, SNAP_GRID);
    k_adj_snapshot<<<gs, 256, 0, st>>>(F, H, snap, g.in_ptr, g.n, p.d, ctl, partC);
    DI_LAUNCH_CHECK();
    *nC = gs;
    if (g.weighted) k_adj_pull<true><<<grid_for(g.n, 256), 256, 0, st>>>(F, snap, g.out_ptr, g.out_idx, g.w, g.inv_s, g.n, ctl);
    else k_adj_pull<false><<<grid_for(g.n, 256), 256, 0, st>>>(F, snap, g.out_ptr, g.out_idx, g.w, g.inv_s, g.n, ctl);
    DI_LAUNCH_CHECK();
    const unsigned gr = grid_for(g.n, 256, REDUCE_GRID);
    k_reduce_F<double><<<gr, 256, 0, st>>>(F, g.n, p.K, ctl, partR, nullptr, nullptr, 0, 0);
    DI_LAUNCH_CHECK();
    *nR = gr;
    return DI_OK;
}

int launch_adj_sweep_fast(const DevGraph &g, const RowBlocks &rb_out, double *F, double *H, double *snap, DevCtl *ctl,
                          const SweepParams &p, hipStream_t st, u64 *partR, u64 *partC, i64 *nR, i64 *nC) {
    const unsigned gs = grid_for(g.n, 256, SNAP_GRID);
    k_adj_snapshot<<<gs, 256, 0, st>>>(F, H, snap, g.in_ptr, g.n, p.d, ctl, partC);
    DI_LAUNCH_CHECK();
    *nC = gs;
    PiArgs a{};
    a.rb_start = rb_out.start;
    a.seg_first = rb_out.seg_first;
    a.seg_count = rb_out.seg_count;
    a.seg_b = rb_out.seg_b;
    a.seg_e = rb_out.seg_e;
    a.partial = rb_out.partial;
    a.in_ptr = g.out_ptr;  // the pull walks OUT rows
    a.in_idx = g.out_idx;
    a.in_w = g.w;
    a.inv_s = g.inv_s;
    a.ctl = ctl;
    a.d = p.d;
    a.n = g.n;
    a.nrb = rb_out.nrb;
    a.nseg = rb_out.nseg;
    a.K = p.K;
    a.partR = partR;
    a.ht = snap;
    a.Fout = F;
    *nR = grid_for(rb_out.nrb, PI_WAVES, PI_GRID);
    return launch_row_pull<PM_ADJ>(a, g.weighted, rb_out, 0, st);
}

int launch_reduce_double(const double *F, i64 n, int K, DevCtl *ctl, hipStream_t st, u64 *partR, i64 *nR) {
    const unsigned gr = grid_for(n, 256, REDUCE_GRID);
    k_reduce_F<double><<<gr, 256, 0, st>>>(F, n, K, ctl, partR, nullptr, nullptr, 0, 0);
    DI_LAUNCH_CHECK();
    *nR = gr;
    return DI_OK;
}

// dZ_j = (1-d) lambda_j; mu_j = left fold over OUT row j of P_e lambda_target;
// dw_e = (d x_j inv_s_j) (lambda_target - mu_j).
template <bool WTD>
__global__ void __launch_bounds__(256) k_edge_grad(const i64 *__restrict__ out_ptr, const int *__restrict__ out_idx,
                                                   const float *__restrict__ w, const double *__restrict__ inv_s,
                                                   const double *__restrict__ x, const double *__restrict__ lam, i64 n,
                                                   double d, double *dZ, double *dw) {
    const i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    dZ[j] = (1.0 - d) * lam[j];
    const i64 e0 = out_ptr[j], e1 = out_ptr[j + 1];
    if (!dw) return;
    const double inv = inv_s[j];
    double mu = 0.0;
    for (i64 e = e0; e < e1; ++e) mu += (WTD ? (double)w[e] * inv : inv) * lam[out_idx[e]];
    const double a = d * x[j] * inv;
    for (i64 e = e0; e < e1; ++e) dw[e] = a * (lam[out_idx[e]] - mu);
}

// Edge-parallel form of the same gradient (fast contexts; the sums of mu run in another
// order).  Each wave takes chunks of GE_CHUNK consecutive OUT edges; a chunk's rows come
// in windows of 64 consecutive rows whose offsets sit in LDS, and a lane finds the row of
// its edge there by binary search.  Pass 1 sums mu_j per window row in LDS: a row wholly
// inside the chunk is stored, a row cut by a chunk boundary is added to mu atomically (mu
// starts at zero).  Pass 2 writes dw_e = (d x_j inv_s_j)(lambda_target - mu_j) with the
// window's per-row factors in LDS.  Every load and store of an edge is coalesced.
constexpr int GE_CHUNK = 1024;
constexpr int GE_WAVES = 4;

template <bool WTD, bool DW>
__global__ void __launch_bounds__(GE_WAVES * WAVE) k_edge_grad_fast(const i64 *__restrict__ out_ptr,
                                                                   const int *__restrict__ out_idx,
                                                                   const float *__restrict__ w,
                                                                   const double *__restrict__ inv_s,
                                                                   const double *__restrict__ x,
                                                                   const double *__restrict__ lam, i64 n, i64 m,
                                                                   double d, double *mu, double *dw) {
    __shared__ i64 offs[GE_WAVES][WAVE + 1];
    __shared__ double rowa[GE_WAVES][WAVE];  // pass 1: inv_s, pass 2: d x inv_s
    __shared__ double rowb[GE_WAVES][WAVE];  // pass 1: sums of mu, pass 2: mu
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    const i64 nch = (m + GE_CHUNK - 1) / GE_CHUNK;
    for (i64 ch = (i64)blockIdx.x * GE_WAVES + wv; ch < nch; ch += (i64)gridDim.x * GE_WAVES) {
        const i64 e0 = ch * GE_CHUNK, e1 = min(m, e0 + GE_CHUNK);
        // the row holding edge e0, the last j with out_ptr[j] <= e0: 63 probes per step
        // keep out_ptr[lo] <= e0 < out_ptr[hi]
        i64 lo = 0, hi = n;
        while (hi - lo > 1) {
            const i64 step = (hi - lo + WAVE - 1) / WAVE;
            const i64 pr = lo + (i64)(lane + 1) * step;
            const bool le = lane < WAVE - 1 && pr < hi && out_ptr[pr] <= e0;
            const int c = __popcll(__ballot(le));  // the true probes form a prefix
            lo += (i64)c * step;
            hi = min(hi, lo + step);
        }
        i64 r0 = lo, es = e0;
        while (es < e1) {
            const i64 r = r0 + lane;
            offs[wv][lane] = out_ptr[min(r, n)];
            if (lane == 0) offs[wv][WAVE] = out_ptr[min(r0 + WAVE, n)];
            if (r < n) {
                const double inv = inv_s[r];
                if (DW) {
                    rowa[wv][lane] = d * x[r] * inv;
                    rowb[wv][lane] = mu[r];
                } else {
                    rowa[wv][lane] = inv;
                    rowb[wv][lane] = 0.0;
                }
            }
            wave_sync_lds();
            const i64 ee = min(e1, offs[wv][WAVE]);
            for (i64 eb = es; eb < ee; eb += WAVE) {
                // every lane runs each step (lanes past ee read edge ee-1 and add nothing)
                const bool on = eb + lane < ee;
                const i64 e = on ? eb + lane : ee - 1;
                int l = 0;  // last l with offs[l] <= e
#pragma unroll
                for (int h = WAVE / 2; h > 0; h >>= 1)
                    if (offs[wv][l + h] <= e) l += h;
                const double lt = lam[out_idx[e]];
                if (DW) {
                    if (on) dw[e] = rowa[wv][l] * (lt - rowb[wv][l]);
                } else {
                    const double P = WTD ? (double)w[e] * rowa[wv][l] : rowa[wv][l];
                    double v = on ? P * lt : 0.0;
                    const int lf = __builtin_amdgcn_readfirstlane(l);
                    if (__ballot(on && l != lf) == 0) {
                        // one row under the whole step (long rows): a wave sum, one add
                        for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
                        if (lane == 0) atomicAdd(&rowb[wv][lf], v);
                    } else if (on) {
                        atomicAdd(&rowb[wv][l], v);
                    }
                }
            }
            wave_sync_lds();
            if (!DW && r < n) {
                const i64 b = offs[wv][lane], f = offs[wv][lane + 1];
                if (max(b, es) < min(f, ee)) {  // the row has edges in this chunk
                    if (b >= e0 && f <= e1) mu[r] = rowb[wv][lane];
                    else atomicAdd(&mu[r], rowb[wv][lane]);
                }
            }
            wave_sync_lds();
            r0 += WAVE;
            es = ee;
        }
    }
}

int launch_edge_grad(const DevGraph &g, const double *x, const double *lam, double d, double *dZ, double *dw,
                     double *mu, hipStream_t st) {
    if (!mu || !dw) {  // row order (the oracle's sums), or dZ only
        if (g.weighted) k_edge_grad<true><<<grid_for(g.n, 256), 256, 0, st>>>(g.out_ptr, g.out_idx, g.w, g.inv_s, x, lam, g.n, d, dZ, dw);
        else k_edge_grad<false><<<grid_for(g.n, 256), 256, 0, st>>>(g.out_ptr, g.out_idx, g.w, g.inv_s, x, lam, g.n, d, dZ, dw);
        DI_LAUNCH_CHECK();
        return DI_OK;
    }
    DI_TRY(launch_scaled_copy(lam, 1.0 - d, g.n, dZ, st));
    if (g.m == 0) return DI_OK;
    DI_TRY(launch_fill_zero(mu, g.n * 8, st));
    const i64 nch = (g.m + GE_CHUNK - 1) / GE_CHUNK;
    const unsigned grid = (unsigned)std::min<i64>((nch + GE_WAVES - 1) / GE_WAVES, 8192);
    if (g.weighted) {
        k_edge_grad_fast<true, false><<<grid, GE_WAVES * WAVE, 0, st>>>(g.out_ptr, g.out_idx, g.w, g.inv_s, x, lam, g.n, g.m, d, mu, dw);
        k_edge_grad_fast<true, true><<<grid, GE_WAVES * WAVE, 0, st>>>(g.out_ptr, g.out_idx, g.w, g.inv_s, x, lam, g.n, g.m, d, mu, dw);
    } else {
        k_edge_grad_fast<false, false><<<grid, GE_WAVES * WAVE, 0, st>>>(g.out_ptr, g.out_idx, g.w, g.inv_s, x, lam, g.n, g.m, d, mu, dw);
        k_edge_grad_fast<false, true><<<grid, GE_WAVES * WAVE, 0, st>>>(g.out_ptr, g.out_idx, g.w, g.inv_s, x, lam, g.n, g.m, d, mu, dw);
    }
    DI_LAUNCH_CHECK();
    return DI_OK;
}

}  // namespace di
