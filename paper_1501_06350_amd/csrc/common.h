// Shared definitions of the D-Iteration / power-iteration library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/di.h"

namespace di {

using u64 = unsigned long long;
using i64 = int64_t;

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Errors: every failing path records a message and returns a DI_E* code.
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);

#define DI_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::di::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                            __LINE__);                                                     \
            return e_ == hipErrorOutOfMemory ? DI_ENOMEM : DI_EHIP;                        \
        }                                                                                  \
    } while (0)

#define DI_TRY(expr)                 \
    do {                             \
        int s_ = (expr);             \
        if (s_ != DI_OK) return s_;  \
    } while (0)

#define DI_LAUNCH_CHECK() DI_HIP(hipGetLastError())

// Every device allocation of the library goes through these two.  They keep the
// process-wide count of live allocations, and inject a failure for tests of the error
// paths: with DI_FAIL_ALLOC_AT=k in the environment, the k-th allocation after the
// variable took its current value fails as out of memory without allocating.
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_free(void *p);
long long dev_live_allocations();

inline unsigned grid_for(i64 work, int per_block, i64 cap = (1ll << 30)) {
    i64 g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Host sum of many doubles with a running compensation (Neumaier's variant of Kahan's
// summation): the error stays at a few units in the last place of the result instead of
// growing with the count (the sum of Z over 10^8 nodes of 1/n each, for instance).
struct HostSum {
    double s = 0.0, c = 0.0;
    void add(double x) {
        const double t = s + x;
        c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};

// ---------------------------------------------------------------------------
// Fixed-point residual sums.  A non-negative double v contributes floor(v * 2^K);
// the sum is kept exactly in four 64-bit accumulators of 32-bit limbs, so it does
// not depend on the order of accumulation.  The final value is rounded once to the
// nearest double (ties to even) and scaled by 2^-K.
// ---------------------------------------------------------------------------
struct Limbs {
    u64 l[4];
};

__device__ __forceinline__ void limbs_zero(Limbs &a) { a.l[0] = a.l[1] = a.l[2] = a.l[3] = 0; }

// v >= 0 and v * 2^K < 2^127 (the scale leaves ten bits of headroom above any sum)
__device__ __forceinline__ void limbs_add(Limbs &a, double v, int K) {
    if (!(v > 0.0)) return;
    double s = ldexp(v, K);
    u64 hi = 0;
    if (s >= 0x1p64) {
        hi = (u64)(s * 0x1p-64);       // floor(s / 2^64)
        s = s - (double)hi * 0x1p64;   // exact: the bits of s below 2^64
    }
    u64 lo = (u64)s;
    a.l[0] += lo & 0xffffffffull;
    a.l[1] += lo >> 32;
    a.l[2] += hi & 0xffffffffull;
    a.l[3] += hi >> 32;
}

// Signed values: the accumulator holds its sum modulo 2^128 (two's complement); a negative
// v adds the 32-bit pieces of 2^128 - floor(|v| 2^K).  Sums stay below 2^118 in magnitude,
// so bit 127 of the carried value tells the sign (limbs_to_double_signed).
__device__ __forceinline__ void limbs_add_signed(Limbs &a, double v, int K) {
    if (v > 0.0) {
        limbs_add(a, v, K);
        return;
    }
    if (!(v < 0.0)) return;
    double s = ldexp(-v, K);
    u64 hi = 0;
    if (s >= 0x1p64) {
        hi = (u64)(s * 0x1p-64);
        s = s - (double)hi * 0x1p64;
    }
    u64 lo = (u64)s;
    if ((lo | hi) == 0) return;
    // two's complement of (hi, lo)
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0 ? 1ull : 0ull);
    a.l[0] += lo & 0xffffffffull;
    a.l[1] += lo >> 32;
    a.l[2] += hi & 0xffffffffull;
    a.l[3] += hi >> 32;
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u64 t = __shfl_xor(v, o, WAVE);
        v = t > v ? t : v;
    }
    return v;
}

// Inclusive prefix sum over the wave (Hillis-Steele with shuffles).
__device__ __forceinline__ int wave_incl_scan_i32(int v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(v, o, WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

// Per-block partial sums.  Every workgroup that contributes to the residual or to the
// counters of a sweep writes its own totals with plain stores into a slot of a partials
// array; the control step adds the slots.  (Device-scope atomics from every workgroup
// onto the same few addresses serialise and cost far more than the sweep itself.)
//   residual slot (PSR words): 4 limb sums of |F|, max |F| as ordered bits
//   counter slot  (PSC words): 4 limb sums of the leak, diffusions, edge pushes,
//                              cross-range deliveries, unused
constexpr int PSR = 5;
constexpr int PSC = 8;

// Reduce NV per-thread values over the block (bit k of MAXMASK: max instead of sum) and
// store them to out[0..NV).  lds: u64[NV * blockDim.x / 64].  Contains barriers.
template <int NV, unsigned MAXMASK = 0>
__device__ __forceinline__ void block_store_partials(u64 (&v)[NV], u64 *lds, u64 *out) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((MAXMASK >> k) & 1u) ? wave_max_u64(v[k]) : wave_sum_u64(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w * NV + k] = v[k];
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        const int k = threadIdx.x;
        u64 s = 0;
        for (int q = 0; q < nw; ++q) {
            const u64 x = lds[q * NV + k];
            s = ((MAXMASK >> k) & 1u) ? (x > s ? x : s) : s + x;
        }
        out[k] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ void store_residual_partial(Limbs &R, u64 maxbits, u64 *lds, u64 *slot) {
    u64 v[PSR] = {R.l[0], R.l[1], R.l[2], R.l[3], maxbits};
    block_store_partials<PSR, 1u << 4>(v, lds, slot);
}

__device__ __forceinline__ void store_counter_partial(Limbs &leak, u64 nodes, u64 edges, u64 remote, u64 *lds,
                                                      u64 *slot) {
    u64 v[PSC] = {leak.l[0], leak.l[1], leak.l[2], leak.l[3], nodes, edges, remote, 0};
    block_store_partials<PSC>(v, lds, slot);
}

// Carry-normalise limb sums so that each limb is below 2^32 (the top one keeps the rest).
__host__ __device__ inline void limbs_normalize(u64 *l) {
    u64 c = 0;
    for (int k = 0; k < 3; ++k) {
        const u64 t = l[k] + c;
        const u64 carry_in = (t < l[k]) ? (1ull << 32) : 0ull;  // overflow of the 64-bit add
        l[k] = t & 0xffffffffull;
        c = (t >> 32) + carry_in;
    }
    l[3] += c;
}

// carry-propagate limb sums into a 128-bit value (hi, lo), modulo 2^128
__host__ __device__ inline void limbs_to_u128(u64 l0, u64 l1, u64 l2, u64 l3, u64 *hi_out, u64 *lo_out) {
    u64 lo = l0 & 0xffffffffull, c = l0 >> 32;
    u64 t = l1 + c;
    u64 carry_hi = (t < l1) ? 1ull : 0ull;  // overflow into bit 96
    lo |= (t & 0xffffffffull) << 32;
    c = (t >> 32) | (carry_hi << 32);
    t = l2 + c;
    u64 c2 = (t < l2) ? 1ull : 0ull;
    u64 hi = t & 0xffffffffull;
    c = (t >> 32) | (c2 << 32);
    t = l3 + c;
    hi |= t << 32;
    *hi_out = hi;
    *lo_out = lo;
}

// a nonnegative 128-bit integer (hi, lo) times 2^-K, rounded once to the nearest double
__host__ __device__ inline double u128_to_double(u64 hi, u64 lo, int K) {
    if (hi == 0 && lo < (1ull << 53)) return ldexp((double)lo, -K);
    int p;  // index of the top set bit
    if (hi) p = 64 + 63 - __builtin_clzll(hi);
    else p = 63 - __builtin_clzll(lo);
    int s = p - 52;  // bits dropped, s >= 1
    u64 mant;
    if (s >= 64) mant = hi >> (s - 64);
    else mant = (lo >> s) | (hi << (64 - s));
    // round bit = bit (s-1); sticky = any bit below it
    int rb = s - 1;
    bool round_bit = rb >= 64 ? ((hi >> (rb - 64)) & 1ull) : ((lo >> rb) & 1ull);
    bool sticky;
    if (rb >= 64) {
        int b = rb - 64;
        sticky = lo != 0 || (b > 0 && (hi & ((1ull << b) - 1)) != 0);
    } else {
        sticky = rb > 0 && (lo & ((1ull << rb) - 1)) != 0;
    }
    if (round_bit && (sticky || (mant & 1ull))) mant += 1;
    return ldexp((double)mant, s - K);
}

__host__ __device__ inline double limbs_to_double_raw(u64 l0, u64 l1, u64 l2, u64 l3, int K) {
    u64 hi, lo;
    limbs_to_u128(l0, l1, l2, l3, &hi, &lo);
    return u128_to_double(hi, lo, K);
}

// the same for a two's-complement signed sum (see limbs_add_signed)
__host__ __device__ inline double limbs_to_double_signed(u64 l0, u64 l1, u64 l2, u64 l3, int K) {
    u64 hi, lo;
    limbs_to_u128(l0, l1, l2, l3, &hi, &lo);
    if (hi >> 63) {  // negative: magnitude = 2^128 - value
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0 ? 1ull : 0ull);
        return -u128_to_double(hi, lo, K);
    }
    return u128_to_double(hi, lo, K);
}

// ---------------------------------------------------------------------------
// Device control block of a single-right-hand-side solve (kept in device memory).
// ---------------------------------------------------------------------------
struct DevCtl {
    u64 limbsL[4];      // cumulative leak (fluid diffused at dangling nodes), normalised limbs
    u64 tot_nodes, tot_edges;
    u64 tot_remote;     // nonzero cross-range deliveries (block-local sweep)
    u64 fcount;         // deterministic sweep: active nodes recorded so far
    u64 fcount_last;    // active nodes of the last completed sweep
    double R;           // residual of the current state
    double thr;         // activity threshold of the next sweep
    double maxF;        // max |F| of the current state
    int done;           // tolerance met
    int guard;          // next sweep takes every node with nonzero fluid
    int overflow;       // fixed-point range exceeded
    int parity;         // slot written by the next sweep
    long long sweep;    // sweeps run since reset
    long long budget;   // sweep limit of the running call (absolute sweep index)
    int dense;          // the next block-local sweep reads in-flight values without the bitmap
};


}  // namespace di
