/*
 * Seeded synthetic input generators (graphs, weights, seed vectors).
 *
 * This module produces INPUTS only: directed graphs in out-adjacency CSR form,
 * edge weights, right-hand sides and loss vectors.  It contains none of the
 * PageRank / D-Iteration arithmetic.  Both the HIP library's tests and the CPU
 * oracle's tests consume its output; neither side's solver code lives here.
 *
 * Randomness is counter based: every draw is h(seed, stream, a, b), where h
 * chains the SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014) over the
 * four words.  A draw therefore depends only on its coordinates, so the output
 * is identical for any thread count.
 *
 *   u53(x)          = x >> 11                        (uniform on [0, 2^53))
 *   Bernoulli(p)    : u53 < floor(p * 2^53)
 *   range(R)        : (u53 * R) >> 53                (128-bit product, R < 2^64)
 *   power law [a,b] : threshold table T_k = floor(2^53 * cdf_k), cdf a left-to-right
 *                     double sum of t^-alpha over t = a..b divided by the total;
 *                     a draw is a + (first k with u53 < T_k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

static uint64_t sm64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t wl_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
    uint64_t z = sm64(seed);
    z = sm64(z ^ (stream * 0xD1B54A32D192ED03ull));
    z = sm64(z ^ a);
    z = sm64(z ^ (b * 0x8CB92BA72F3D8DD7ull));
    return z;
}

static inline uint64_t u53(uint64_t x) { return x >> 11; }
static inline uint64_t thresh53(double p) { return (uint64_t)floor(p * 9007199254740992.0); }
static inline uint64_t range53(uint64_t u, uint64_t r) { return (uint64_t)(((u128)u * r) >> 53); }

/* Power-law threshold table on [a, b]; caller frees. */
static uint64_t *powerlaw_table(int64_t a, int64_t b, double alpha) {
    int64_t cnt = b - a + 1;
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cnt);
    double *cdf = (double *)malloc(sizeof(double) * (size_t)cnt);
    if (!T || !cdf) { free(T); free(cdf); return NULL; }
    double acc = 0.0;
    for (int64_t k = 0; k < cnt; ++k) { acc += pow((double)(a + k), -alpha); cdf[k] = acc; }
    for (int64_t k = 0; k < cnt; ++k) T[k] = (uint64_t)floor(cdf[k] / acc * 9007199254740992.0);
    T[cnt - 1] = 9007199254740992ull; /* guarantees every u53 finds a bucket */
    free(cdf);
    return T;
}

static inline int64_t powerlaw_draw(const uint64_t *T, int64_t cnt, uint64_t u) {
    int64_t lo = 0, hi = cnt - 1; /* first k with u < T[k] */
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (u < T[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}
static void sort_row(int32_t *v, int64_t len) {
    if (len <= 48) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t key = v[i];
            int64_t j = i - 1;
            while (j >= 0 && v[j] > key) { v[j + 1] = v[j]; --j; }
            v[j + 1] = key;
        }
    } else {
        qsort(v, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/* ---------------------------------------------------------------------------
 * Out-degrees.  Node i is dangling with probability p_dang (stream 2); otherwise
 * its out-degree is a power law with exponent alpha on [dmin, dmax] (stream 3).
 * Fills out_ptr[0..n] and returns m = out_ptr[n], or -1 on allocation failure.
 * ------------------------------------------------------------------------- */
int64_t wl_degrees(int64_t n, uint64_t seed, double p_dang, double alpha, int64_t dmin, int64_t dmax,
                   int64_t *out_ptr) {
    uint64_t *T = powerlaw_table(dmin, dmax, alpha);
    if (!T) return -1;
    const int64_t cnt = dmax - dmin + 1;
    const uint64_t pd = thresh53(p_dang);
    out_ptr[0] = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t deg = 0;
        if (u53(wl_hash(seed, 2, (uint64_t)i, 0)) >= pd)
            deg = dmin + powerlaw_draw(T, cnt, u53(wl_hash(seed, 3, (uint64_t)i, 0)));
        out_ptr[i + 1] = deg;
    }
    for (int64_t i = 0; i < n; ++i) out_ptr[i + 1] += out_ptr[i];
    free(T);
    return out_ptr[n];
}

/* Uniform targets on [0, n) (stream 6), rows sorted ascending. */
int wl_targets_uniform(int64_t n, uint64_t seed, const int64_t *out_ptr, int32_t *out_idx) {
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; ++u) {
        int64_t b = out_ptr[u], e = out_ptr[u + 1];
        for (int64_t k = 0; k < e - b; ++k)
            out_idx[b + k] = (int32_t)range53(u53(wl_hash(seed, 6, (uint64_t)u, (uint64_t)k)), (uint64_t)n);
        sort_row(out_idx + b, e - b);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Web-like targets.
 *   hosts     : consecutive node ranges; host h has size floor(exp(ln 10 + u ln 100))
 *               (log-uniform on 10..999, stream 1), the last host truncated at n.
 *   attraction: W_i = power law (alpha_in) on [1, floor(n^w_exp)] (stream 4).
 *   edge (u,k): intra-host with probability p_intra (stream 5); the target is then
 *               drawn with probability proportional to W inside u's host, otherwise
 *               proportional to W over all nodes (stream 6), by inverse transform on
 *               the integer prefix sums S of W (global draws use a guide table of
 *               n entries to start the search).
 *   rows are sorted ascending by target; self-loops and duplicates are kept.
 * ------------------------------------------------------------------------- */
static int64_t upper_search(const uint64_t *S, int64_t lo, int64_t hi, uint64_t x) {
    /* first i in [lo, hi) with S[i+1] > x; S non-decreasing, S[hi] > x */
    while (lo < hi - 1) {
        int64_t mid = (lo + hi) >> 1;
        if (S[mid] > x) hi = mid; else lo = mid;
    }
    return lo;
}

int64_t wl_host_count(int64_t n, uint64_t seed) {
    int64_t h = 0, pos = 0;
    while (pos < n) {
        double u = (double)u53(wl_hash(seed, 1, (uint64_t)h, 0)) / 9007199254740992.0;
        int64_t sz = (int64_t)floor(exp(log(10.0) + u * log(100.0)));
        pos += sz;
        ++h;
    }
    return h;
}

/* host_ptr must hold wl_host_count(n, seed) + 1 entries */
int wl_hosts(int64_t n, uint64_t seed, int64_t *host_ptr) {
    int64_t h = 0, pos = 0;
    host_ptr[0] = 0;
    while (pos < n) {
        double u = (double)u53(wl_hash(seed, 1, (uint64_t)h, 0)) / 9007199254740992.0;
        int64_t sz = (int64_t)floor(exp(log(10.0) + u * log(100.0)));
        pos += sz;
        if (pos > n) pos = n;
        host_ptr[++h] = pos;
    }
    return 0;
}

int wl_targets_web(int64_t n, uint64_t seed, double alpha_in, double w_exp, double p_intra,
                   const int64_t *out_ptr, int32_t *out_idx) {
    int64_t wmax = (int64_t)floor(pow((double)n, w_exp));
    if (wmax < 1) wmax = 1;
    uint64_t *TW = powerlaw_table(1, wmax, alpha_in);
    int64_t nh = wl_host_count(n, seed);
    int64_t *host_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nh + 1));
    uint64_t *S = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    int64_t *guide = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!TW || !host_ptr || !S || !guide) { free(TW); free(host_ptr); free(S); free(guide); return -1; }
    wl_hosts(n, seed, host_ptr);

    S[0] = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) S[i + 1] = (uint64_t)(1 + powerlaw_draw(TW, wmax, u53(wl_hash(seed, 4, (uint64_t)i, 0))));
    for (int64_t i = 0; i < n; ++i) S[i + 1] += S[i];
    const uint64_t total = S[n];
    /* guide[g] = first i with S[i+1] > floor(g * total / n) */
    {
        int64_t i = 0;
        for (int64_t g = 0; g <= n; ++g) {
            uint64_t x = (uint64_t)(((u128)(uint64_t)g * total) / (uint64_t)n);
            if (x >= total) { guide[g] = n - 1; continue; }
            while (S[i + 1] <= x) ++i;
            guide[g] = i;
        }
    }
    const uint64_t pin = thresh53(p_intra);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t h = 0; h < nh; ++h) {
        const int64_t hs = host_ptr[h], he = host_ptr[h + 1];
        for (int64_t u = hs; u < he; ++u) {
            int64_t b = out_ptr[u], e = out_ptr[u + 1];
            for (int64_t k = 0; k < e - b; ++k) {
                int intra = u53(wl_hash(seed, 5, (uint64_t)u, (uint64_t)k)) < pin;
                uint64_t r = u53(wl_hash(seed, 6, (uint64_t)u, (uint64_t)k));
                int64_t t;
                if (intra) {
                    uint64_t x = S[hs] + range53(r, S[he] - S[hs]);
                    t = upper_search(S, hs, he, x);
                } else {
                    uint64_t x = range53(r, total);
                    int64_t g = (int64_t)(((u128)x * (uint64_t)n) / total);
                    /* S[guide[g]] <= x < S[guide[g+1] + 1], and g + 1 <= n because x < total */
                    t = upper_search(S, guide[g], guide[g + 1] + 1, x);
                }
                out_idx[b + k] = (int32_t)t;
            }
            sort_row(out_idx + b, e - b);
        }
    }
    free(TW); free(host_ptr); free(S); free(guide);
    return 0;
}

/* Standard normal from two counter uniforms (Box-Muller, cosine branch). */
static double normal_draw(uint64_t seed, uint64_t stream_a, uint64_t stream_b, uint64_t idx) {
    double u1 = ((double)u53(wl_hash(seed, stream_a, idx, 0)) + 1.0) / 9007199254740992.0; /* (0,1] */
    double u2 = (double)u53(wl_hash(seed, stream_b, idx, 0)) / 9007199254740992.0;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* w_e = exp(N(0,1)) rounded to float, per edge position e (streams 7, 8). */
int wl_lognormal_weights(uint64_t seed, int64_t m, float *w) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) w[e] = (float)exp(normal_draw(seed, 7, 8, (uint64_t)e));
    return 0;
}

/* c_i ~ N(0,1) (streams 9, 10). */
int wl_normal_vector(uint64_t seed, int64_t n, double *c) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) c[i] = normal_draw(seed, 9, 10, (uint64_t)i);
    return 0;
}

/* k columns of s distinct seed nodes each (stream 11, rejection of repeats). */
int wl_seed_nodes(uint64_t seed, int64_t n, int64_t k, int64_t s, int64_t *out) {
    if (s > n) return -1;
    for (int64_t c = 0; c < k; ++c) {
        int64_t got = 0;
        for (uint64_t r = 0; got < s; ++r) {
            int64_t v = (int64_t)range53(u53(wl_hash(seed, 11, (uint64_t)c, r)), (uint64_t)n);
            int dup = 0;
            for (int64_t q = 0; q < got; ++q) dup |= (out[c * s + q] == v);
            if (!dup) out[c * s + got++] = v;
        }
    }
    return 0;
}

/* Log-uniform sizes floor(exp(ln lo + u ln(hi/lo))) and per-item seeds (streams 12, 13). */
int wl_batch_sizes(uint64_t seed, int64_t count, double lo, double hi, int64_t *sizes, uint64_t *seeds) {
    for (int64_t g = 0; g < count; ++g) {
        double u = (double)u53(wl_hash(seed, 12, (uint64_t)g, 0)) / 9007199254740992.0;
        sizes[g] = (int64_t)floor(exp(log(lo) + u * log(hi / lo)));
        seeds[g] = wl_hash(seed, 13, (uint64_t)g, 0);
    }
    return 0;
}

uint64_t wl_stream_draw(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) { return wl_hash(seed, stream, a, b); }

int wl_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
