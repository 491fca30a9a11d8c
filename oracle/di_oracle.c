/*
 * CPU reference ("oracle") for D-Iteration and power iteration on PageRank.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  The GPU library
 * never calls it and shares no code with it.
 *
 * Everything is plain sequential IEEE binary64 (compiled without contraction or
 * fast-math), one node or one row at a time, in the order the paper states.
 *
 * Notation (Section 2.1, equation def-p): P[i][j] = w(j->i) / s_j with
 * s_j = sum of j's out-weights (out-degree when unweighted), so column j of P is
 * j's out-row.  OUT = adjacency by source (the input CSR), IN = by target.
 *
 *   x = d P x + (1-d) Z                                  (equation pagerank-pf)
 *   F_0 = (1-d) Z, H_0 = 0,
 *   F_k = F_{k-1} + d F_{k-1}(i_k) P e_{i_k} - F_{k-1}(i_k) e_{i_k},
 *   H_k = H_{k-1} + F_{k-1}(i_k) e_{i_k}                 (Section 3.1, equation defF)
 *   |x - H_k|_1 <= |F_k|_1 / (1-d)                       (Theorem 1, equation SL)
 *
 * Fixed-point residual: a sum of |v_i| is defined as the exact integer sum of
 * floor(|v_i| * 2^K) rounded once to the nearest double and scaled by 2^-K
 * (K from or_fixed_scale).  Every value of magnitude >= 2^(52-K) is an exact
 * multiple of 2^-K, so in practice this is the correctly rounded sum; it does not
 * depend on summation order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* Graph preparation                                                          */
/* ------------------------------------------------------------------------- */

/* IN adjacency by a stable counting sort of OUT's edges on their target:
 * in_idx[p] = source, in_eid[p] = OUT position of the edge; each IN row lists
 * sources in ascending order (OUT is visited source by source). */
int or_build_in(int64_t n, int64_t m, const int64_t *out_ptr, const int32_t *out_idx,
                int64_t *in_ptr, int32_t *in_idx, int64_t *in_eid) {
    int64_t *cursor = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cursor) return -1;
    for (int64_t e = 0; e < m; ++e) cursor[out_idx[e] + 1] += 1;
    in_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) in_ptr[i + 1] = in_ptr[i] + cursor[i + 1];
    for (int64_t i = 0; i < n; ++i) cursor[i] = in_ptr[i];
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t e = out_ptr[j]; e < out_ptr[j + 1]; ++e) {
            int64_t pos = cursor[out_idx[e]]++;
            in_idx[pos] = (int32_t)j;
            in_eid[pos] = e;
        }
    }
    free(cursor);
    return 0;
}

/* inv_s[j] = 1 / s_j with s_j = out-degree (w == NULL) or the left-to-right double
 * sum of j's out-weights; 0 for a dangling node (P's column is null, Section 2.1). */
void or_inv_s(int64_t n, const int64_t *out_ptr, const float *w, double *inv_s) {
    for (int64_t j = 0; j < n; ++j) {
        int64_t b = out_ptr[j], e = out_ptr[j + 1];
        if (e == b) { inv_s[j] = 0.0; continue; }
        double s = 0.0;
        if (w) { for (int64_t p = b; p < e; ++p) s += (double)w[p]; }
        else s = (double)(e - b);
        inv_s[j] = 1.0 / s;
    }
}

/* P entry carried by an edge of source j: w_e / s_j, or 1 / out(j). */
static inline double p_entry(const float *w, int64_t e, double inv_s_j) {
    return w ? (double)w[e] * inv_s_j : inv_s_j;
}

/* ------------------------------------------------------------------------- */
/* Fixed-point sums                                                           */
/* ------------------------------------------------------------------------- */

/* K = 118 - (e_max + e_n), where 2^e_max > max|v| (frexp exponent, 0 when v == 0)
 * and 2^e_n >= n, so that any sum of |v_i| scaled by 2^K stays below 2^118: ten
 * bits of headroom under 2^128 for sums that grow. */
int or_fixed_scale(int64_t n, const double *v) {
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) { double a = fabs(v[i]); if (a > mx) mx = a; }
    int e_max = 0;
    if (mx > 0.0) frexp(mx, &e_max);
    int e_n = 0;
    while (((int64_t)1 << e_n) < n) ++e_n;
    return 118 - (e_max + e_n);
}

static inline u128 fixed_of(double v, int K) {
    double s = ldexp(fabs(v), K);
    return (u128)s; /* truncation toward zero */
}

static inline double fixed_to_double(u128 acc, int K) { return ldexp((double)acc, -K); }

/* A signed fixed-point accumulator holds its value modulo 2^128 (two's complement): a
 * negative v adds 2^128 - floor(|v| 2^K).  Sums stay below 2^118 in magnitude (see
 * or_fixed_scale), so the top bit tells the sign. */
static inline u128 fixed_of_signed(double v, int K) {
    u128 q = fixed_of(v, K);
    return v < 0.0 ? (u128)0 - q : q;
}

static inline double fixed_to_double_signed(u128 acc, int K) {
    if (acc >> 127) return -ldexp((double)((u128)0 - acc), -K);
    return ldexp((double)acc, -K);
}

/* Exact signed sum of v on 2^-K as a two's-complement u128 (out[0] low, out[1] high
 * 64 bits); returns the value rounded once to double. */
double or_fixed_sum_signed(int64_t n, const double *v, int K, uint64_t *out) {
    u128 acc = 0;
    for (int64_t i = 0; i < n; ++i) acc += fixed_of_signed(v[i], K);
    if (out) {
        out[0] = (uint64_t)acc;
        out[1] = (uint64_t)(acc >> 64);
    }
    return fixed_to_double_signed(acc, K);
}

double or_fixed_sum_abs(int64_t n, const double *v, int K) {
    u128 acc = 0;
    for (int64_t i = 0; i < n; ++i) acc += fixed_of(v[i], K);
    return fixed_to_double(acc, K);
}

/* ------------------------------------------------------------------------- */
/* Sequential D-Iteration (Section 3.1) with the Section 3.4 schedulers        */
/* ------------------------------------------------------------------------- */

/*
 * Run up to max_steps elementary diffusions.
 *   sched 0 (DI-cyc, Section 3.4): round robin over 0..n-1.
 *   sched 1 (DI-argmax, Section 3.4): round robin, but skip nodes whose fluid is
 *           below the average fluid |F|_1 / n of the whole graph (compared in
 *           magnitude: after a graph update, Theorem 4, fluid may be negative).
 * |F|_1 is the fixed-point sum (K from or_fixed_scale of the F given to the call), kept
 * exact as F changes: each changed entry removes its old term and adds its new one, so
 * a step costs its out-degree, not n.  *pos is the round-robin pointer (next candidate),
 * kept across calls.  Stops early when |F|_1 / (1-d) <= tol (tol <= 0 disables).
 * Returns steps done.
 */
int64_t or_di_sequential(int64_t n, const int64_t *out_ptr, const int32_t *out_idx, const float *w,
                         const double *inv_s, double d, double *F, double *H, double *l, int sched,
                         int64_t max_steps, double tol, int64_t *pos) {
    int64_t steps = 0;
    int64_t p = *pos;
    const int K = or_fixed_scale(n, F);
    u128 Rf = 0;
    for (int64_t i = 0; i < n; ++i) Rf += fixed_of(F[i], K);
    while (steps < max_steps) {
        const double R = fixed_to_double(Rf, K);
        if (tol > 0.0 && R / (1.0 - d) <= tol) break;
        int64_t i = p;
        if (sched == 1) {
            /* first node at or after p with |F| >= average; a full cycle always finds one
             * because the largest |F_i| is at least the average */
            const double avg = R / (double)n;
            int64_t tries = 0;
            while (fabs(F[i]) < avg && tries < n) { i = (i + 1) % n; ++tries; }
        }
        /* one elementary diffusion of node i (equation defF), the residual's terms updated:
         * the local fluid moves to H and is cleared, then d f P e_i goes out (any
         * self-loop share comes back) */
        Rf -= fixed_of(F[i], K);
        const double f = F[i];
        H[i] += f;
        F[i] = 0.0;
        if (out_ptr[i + 1] == out_ptr[i]) {
            *l += f; /* fluid leaving through a dangling node (Section 3.3) */
        } else {
            for (int64_t e = out_ptr[i]; e < out_ptr[i + 1]; ++e) {
                const int32_t t = out_idx[e];
                Rf -= fixed_of(F[t], K);
                F[t] += d * f * p_entry(w, e, inv_s[i]);
                Rf += fixed_of(F[t], K);
            }
        }
        p = (i + 1) % n;
        ++steps;
    }
    *pos = p;
    return steps;
}

/* ------------------------------------------------------------------------- */
/* Synchronous-sweep D-Iteration (the GPU's deterministic sweep)              */
/* ------------------------------------------------------------------------- */

/*
 * One call runs sweeps until R_t / (1-d) <= tol or max_sweeps sweeps were done.
 * Sweep t:
 *   R_t  = fixed-point sum of |F|                       (stopping quantity, Theorem 1)
 *   thr  = ((theta * R_t) / n) * (1 - 2^-30)            (DI-argmax's "at least the average
 *                                                         fluid", Section 3.4, applied to a set)
 *   A_t  = { i : F_i != 0 and |F_i| >= thr }, or { i : F_i != 0 } if that is empty
 *   f_i  = F_i on A_t (snapshot), H_i += f_i, F_i = 0 on A_t
 *   F_j += sum over IN row j, ascending source i in A_t, of (d * f_i) * inv_s_i (* w_e)
 *          as a left fold starting from F_j, in double; with fluid_fp32 the fold's
 *          result is rounded to float once.
 *   l    : dangling sources in A_t add floor(|f_i| * 2^K), with the sign of f_i, to the
 *          integer l_fixed (two's complement; fluid is signed after a graph update).
 * trace (optional, 3 doubles per sweep): R_t, |A_t|, edges pushed.
 * frontier (optional): indices of the last sweep's A_t, ascending; *frontier_len set.
 * Returns the number of sweeps that pushed; *converged = 1 if the stop test passed.
 */
int64_t or_di_sync(int64_t n, const int64_t *out_ptr, const int64_t *in_ptr, const int32_t *in_idx,
                   const float *in_w, const double *inv_s, double d, double theta, int fluid_fp32, int K,
                   double *F, double *H, uint64_t *l_fixed /* [2]: lo, hi */, double tol, int64_t max_sweeps,
                   double *trace, int32_t *frontier, int64_t *frontier_len, int *converged) {
    char *act = (char *)malloc((size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *Fn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!act || !q || !Fn) { free(act); free(q); free(Fn); return -1; }
    u128 lacc = ((u128)l_fixed[1] << 64) | (u128)l_fixed[0];
    int64_t t = 0;
    *converged = 0;
    while (1) {
        double R = or_fixed_sum_abs(n, F, K);
        if (R / (1.0 - d) <= tol) { *converged = 1; break; }
        if (t >= max_sweeps) break;
        double thr = ((theta * R) / (double)n) * (1.0 - 0x1p-30);
        int64_t na = 0, edges = 0;
        for (int64_t i = 0; i < n; ++i) {
            act[i] = (F[i] != 0.0) && (fabs(F[i]) >= thr);
            na += act[i];
        }
        if (na == 0)
            for (int64_t i = 0; i < n; ++i) { act[i] = (F[i] != 0.0); na += act[i]; }
        for (int64_t i = 0; i < n; ++i) {
            q[i] = 0.0;
            if (!act[i]) continue;
            double f = F[i];
            H[i] += f;
            F[i] = 0.0;
            if (out_ptr[i + 1] == out_ptr[i]) lacc += fixed_of_signed(f, K);
            else q[i] = (d * f) * inv_s[i];
            edges += out_ptr[i + 1] - out_ptr[i];
        }
        for (int64_t j = 0; j < n; ++j) {
            double acc = F[j];
            for (int64_t p = in_ptr[j]; p < in_ptr[j + 1]; ++p) {
                int32_t i = in_idx[p];
                if (!act[i]) continue;
                acc += in_w ? q[i] * (double)in_w[p] : q[i];
            }
            Fn[j] = fluid_fp32 ? (double)(float)acc : acc;
        }
        memcpy(F, Fn, sizeof(double) * (size_t)n);
        if (trace) { trace[3 * t] = R; trace[3 * t + 1] = (double)na; trace[3 * t + 2] = (double)edges; }
        if (frontier) {
            int64_t c = 0;
            for (int64_t i = 0; i < n; ++i) if (act[i]) frontier[c++] = (int32_t)i;
            *frontier_len = c;
        }
        ++t;
    }
    l_fixed[0] = (uint64_t)lacc;
    l_fixed[1] = (uint64_t)(lacc >> 64);
    free(act); free(q); free(Fn);
    return t;
}

double or_fixed_value(const uint64_t *l_fixed, int K) {
    u128 a = ((u128)l_fixed[1] << 64) | (u128)l_fixed[0];
    return fixed_to_double_signed(a, K);
}

/* ------------------------------------------------------------------------- */
/* Power iteration (Section 2.2)                                               */
/* ------------------------------------------------------------------------- */

/*
 * x_{k+1} = d P x_k + (1-d) Z, row by row over IN:
 *   y_i = d * (left fold over IN row i of x_j * inv_s_j (* w_e)) + (1-d) * Z_i.
 * Stops after the first iteration with |x_{k+1} - x_k|_1 / (1-d) <= tol, returning
 * x_{k+1} in x.  Rows are independent, so OpenMP over rows changes nothing in the
 * result; the residual is summed sequentially afterwards.  Returns iterations.
 */
int64_t or_power(int64_t n, const int64_t *in_ptr, const int32_t *in_idx, const float *in_w,
                 const double *inv_s, double d, const double *Z, double *x, double tol, int64_t max_iters,
                 double *trace, int *converged) {
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *xt = (double *)malloc(sizeof(double) * (size_t)n);
    if (!y || !xt) { free(y); free(xt); return -1; }
    int64_t k = 0;
    *converged = 0;
    while (k < max_iters) {
        for (int64_t j = 0; j < n; ++j) xt[j] = x[j] * inv_s[j];
#pragma omp parallel for schedule(dynamic, 2048)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t p = in_ptr[i]; p < in_ptr[i + 1]; ++p)
                acc += in_w ? xt[in_idx[p]] * (double)in_w[p] : xt[in_idx[p]];
            y[i] = d * acc + (1.0 - d) * Z[i];
        }
        double R = 0.0;
        for (int64_t i = 0; i < n; ++i) R += fabs(y[i] - x[i]);
        memcpy(x, y, sizeof(double) * (size_t)n);
        if (trace) trace[k] = R;
        ++k;
        if (R / (1.0 - d) <= tol) { *converged = 1; break; }
    }
    free(y); free(xt);
    return k;
}

/* ------------------------------------------------------------------------- */
/* Gauss-Seidel (Section 2.3), a comparison method for the convergence curves   */
/* ------------------------------------------------------------------------- */

/*
 * `sweeps` rounds of x(i) = d (sum_{j<i} P[i][j] x_new(j) + sum_{j>=i} P[i][j] x_old(j))
 * + (1-d) Z(i) for i = 0 .. n-1: one vector updated in place in index order, so the
 * entries below i are already the new ones.  Each row is a left fold over its IN row in
 * source order.  x holds the start vector on entry.
 */
void or_gauss_seidel(int64_t n, const int64_t *in_ptr, const int32_t *in_idx, const float *in_w,
                     const double *inv_s, double d, const double *Z, double *x, int64_t sweeps) {
    for (int64_t k = 0; k < sweeps; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t p = in_ptr[i]; p < in_ptr[i + 1]; ++p) {
                int32_t j = in_idx[p];
                acc += (in_w ? (double)in_w[p] * inv_s[j] : inv_s[j]) * x[j];
            }
            x[i] = d * acc + (1.0 - d) * Z[i];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Adjoint: lambda = (I - d P^T)^{-1} g by diffusion on the transposed matrix   */
/* ------------------------------------------------------------------------- */

/*
 * The same synchronous sweep as or_di_sync, on P^T and with signed fluid:
 *   F_0 = g, H_0 = 0; node i's diffusion sends d * f_i * P[i][j] to every j with an
 *   edge j -> i, i.e. along IN row i.  Written as a fold over OUT row j (ascending
 *   target i in A_t): F_j += (d * f_i) * P_e, P_e = w_e * inv_s_j or inv_s_j.
 *   Selection uses |F_i| >= ((theta * |F|_1) / n) * (1 - 2^-30) (fixed-point L1);
 *   the stop test is max|F| / (1-d) <= tol, since the largest column sum of P is
 *   at most 1 (Section 2.1) and so |P^T|_inf <= 1.
 */
int64_t or_adjoint_sync(int64_t n, const int64_t *out_ptr, const int32_t *out_idx, const float *w,
                        const double *inv_s, double d, double theta, int K, double *F, double *H, double tol,
                        int64_t max_sweeps, int *converged) {
    char *act = (char *)malloc((size_t)n);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    double *Fn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!act || !s || !Fn) { free(act); free(s); free(Fn); return -1; }
    int64_t t = 0;
    *converged = 0;
    while (1) {
        double mx = 0.0;
        for (int64_t i = 0; i < n; ++i) if (fabs(F[i]) > mx) mx = fabs(F[i]);
        if (mx / (1.0 - d) <= tol) { *converged = 1; break; }
        if (t >= max_sweeps) break;
        double R = or_fixed_sum_abs(n, F, K);
        double thr = ((theta * R) / (double)n) * (1.0 - 0x1p-30);
        int64_t na = 0;
        for (int64_t i = 0; i < n; ++i) { act[i] = (F[i] != 0.0) && (fabs(F[i]) >= thr); na += act[i]; }
        if (na == 0) for (int64_t i = 0; i < n; ++i) act[i] = (F[i] != 0.0);
        for (int64_t i = 0; i < n; ++i) {
            s[i] = 0.0;
            if (!act[i]) continue;
            H[i] += F[i];
            s[i] = d * F[i];
            F[i] = 0.0;
        }
        for (int64_t j = 0; j < n; ++j) {
            double acc = F[j];
            for (int64_t e = out_ptr[j]; e < out_ptr[j + 1]; ++e) {
                int32_t i = out_idx[e];
                if (!act[i]) continue;
                acc += s[i] * p_entry(w, e, inv_s[j]);
            }
            Fn[j] = acc;
        }
        memcpy(F, Fn, sizeof(double) * (size_t)n);
        ++t;
    }
    free(act); free(s); free(Fn);
    return t;
}

/*
 * Gradients of L(x) with dL/dx = g, given x and lambda = (I - d P^T)^{-1} g:
 *   dL/dZ_i = (1-d) lambda_i
 *   dL/dP[i][j] = d lambda_i x_j, and P[k][j] = w(j->k) / s_j gives
 *   dL/dw_e (e = j -> i) = (d * x_j * inv_s_j) * (lambda_i - mu_j),
 *   mu_j = left fold over OUT row j of P_e * lambda_{target(e)}.
 */
void or_edge_grad(int64_t n, const int64_t *out_ptr, const int32_t *out_idx, const float *w, const double *inv_s,
                  double d, const double *x, const double *lam, double *dw, double *dZ) {
    for (int64_t j = 0; j < n; ++j) {
        dZ[j] = (1.0 - d) * lam[j];
        double mu = 0.0;
        for (int64_t e = out_ptr[j]; e < out_ptr[j + 1]; ++e) mu += p_entry(w, e, inv_s[j]) * lam[out_idx[e]];
        double a = d * x[j] * inv_s[j];
        for (int64_t e = out_ptr[j]; e < out_ptr[j + 1]; ++e) dw[e] = a * (lam[out_idx[e]] - mu);
    }
}

/* y = P v (pull over IN), used for invariant checks at sizes where a dense P is too big. */
void or_spmv_P(int64_t n, const int64_t *in_ptr, const int32_t *in_idx, const float *in_w, const double *inv_s,
               const double *v, double *y) {
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t p = in_ptr[i]; p < in_ptr[i + 1]; ++p) {
            int32_t j = in_idx[p];
            acc += (in_w ? (double)in_w[p] * inv_s[j] : inv_s[j]) * v[j];
        }
        y[i] = acc;
    }
}

/* The same for selected rows only (sampled checks on large graphs). */
void or_spmv_P_rows(int64_t nrows, const int64_t *rows, const int64_t *in_ptr, const int32_t *in_idx,
                    const float *in_w, const double *inv_s, const double *v, double *y) {
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        double acc = 0.0;
        for (int64_t p = in_ptr[i]; p < in_ptr[i + 1]; ++p) {
            int32_t j = in_idx[p];
            acc += (in_w ? (double)in_w[p] * inv_s[j] : inv_s[j]) * v[j];
        }
        y[r] = acc;
    }
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
