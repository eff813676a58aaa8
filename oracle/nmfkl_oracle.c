/*
 * nmfkl_oracle.c -- plain FP64 CPU oracle for NMF with KL divergence by the paper's
 * randomized coordinate descent (Nguyen & Ho, "Fast Parallel Randomized Algorithm for
 * Nonnegative Matrix Factorization with KL Divergence for Large Sparse Datasets").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or table with the GPU library.
 *
 * Everything is double precision with no blocking or fusion.  Sums over the nonzeros of
 * one column or row run sequentially in storage order; the objective adds the columns'
 * sums in column order.  No result depends on the thread count.  Columns (F-half) and
 * rows (W-half) are independent subproblems (the separability identity, eq. 3) and are
 * run in parallel with OpenMP, as Alg. 1 states.
 *
 * Notation (the paper's, with its W r x n and F r x m stored transposed, point-major):
 *   V   n x m sparse counts, as CSC (columns = documents) and CSR (rows = words)
 *   W   n x r  (row i = the r-vector of word i)       F   m x r (row j = document j)
 *   Alg. 2 works on one column v of V (or one row), with A = the fixed factor, x = the
 *   r-vector being updated, sumA = the column sums of A, and a coordinate order ids.
 *
 * Readings where the paper is silent or garbled (each also listed in the design notes):
 *   - eps_log is added to the model inside every log and every denominator (Alg. 2's
 *     output line smooths the log; eq. 6 is then the exact derivative of that objective);
 *   - the while-test threshold is relative: enter if g < -eps_g*P, or if g > eps_g*P and
 *     x_k > 0, where P = sumA_k + alpha*x_k + beta is the positive part of g;
 *   - the break test compares the magnitude of Alg. 2's projected Newton step dx (before
 *     any halving by the guard below): |dx| < eps_x * x_before (eps_x = 0.1, Section 3);
 *     the literal signed test is kept behind literal_break for the ablation;
 *   - a decreasing step is accepted only if g(x0) + g(x1) >= 0 (else halved up to j_max
 *     times, then abandoned).  Along one coordinate g is concave, so this guarantees that
 *     the subproblem objective does not increase; increasing steps need no guard;
 *   - at most t_max Newton steps per coordinate; h <= 0 (no curvature) moves x_k to 0 if
 *     g > 0 and leaves it otherwise;
 *   - the model Ax is kept at the nonzeros of v only and clamped at 0 after each update;
 *   - the W-half uses sumF and (alpha_1, beta_1), as the W-subproblem of eq. 2 requires;
 *   - the coordinate order is a Fisher-Yates shuffle driven by Philox-4x64-10.
 *
 * parity pins: see the test suite (finite differences, 1-D brute force, r = 1 closed
 * form, dense objective, KKT and mass preservation, exact recovery, NumPy's Philox).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double alpha_W, alpha_F, beta_W, beta_F; /* eq. 2: alpha_1, alpha_2, beta_1, beta_2 */
    double eps_log;                          /* smoothing inside the log (Alg. 2 output) */
    double eps_g;                            /* relative gradient threshold (Alg. 2 while) */
    double eps_x;                            /* step-size break ratio (Section 3: 0.1) */
    int32_t t_max;                           /* Newton steps per coordinate */
    int32_t j_max;                           /* halvings of a rejected decreasing step */
    int32_t literal_break;                   /* 1: signed break test as printed */
    int32_t guard;                           /* 1: descent guard on decreasing steps */
    uint64_t seed;                           /* Philox key word 0 */
    int32_t foldin_max_passes;
    double foldin_tol;
} orc_params;

typedef struct {
    int64_t coords;      /* coordinate visits */
    int64_t evals;       /* derivative evaluations (eq. 6 reductions) */
    int64_t steps;       /* accepted Newton steps */
    int64_t halvings;    /* guard halvings */
    int64_t rejects;     /* steps abandoned by the guard */
    int64_t tmax_hits;   /* coordinates stopped by t_max */
} orc_stats;

static void stats_add(orc_stats* a, const orc_stats* b) {
    a->coords += b->coords; a->evals += b->evals; a->steps += b->steps;
    a->halvings += b->halvings; a->rejects += b->rejects; a->tmax_hits += b->tmax_hits;
}

/* ------------------------------------------------------------------------------------
 * Philox-4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, SC'11): counter (c0..c3),
 * key (k0, k1).  One round multiplies c0 and c2 by the two published multipliers, takes
 * the 128-bit products apart and recombines them with c1, c3 and the key; the key is
 * bumped by the two published Weyl increments between rounds.
 * ---------------------------------------------------------------------------------- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        __uint128_t p0 = (__uint128_t)M0 * c0;
        __uint128_t p1 = (__uint128_t)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* "ids = a randomized ordered set of values {1..r}" (Alg. 1): one permutation per outer
 * iteration t.  Words come from Philox blocks at counter (b, t, stream, 0), b = 0, 1, ...,
 * key (seed, 0), consumed in order; Fisher-Yates from the top, j = floor(w*(i+1)/2^64). */
void orc_permutation(uint64_t seed, uint64_t t, uint64_t stream, int32_t r, int32_t* ids) {
    for (int32_t i = 0; i < r; ++i) ids[i] = i;
    uint64_t key[2] = {seed, 0}, blk[4];
    uint64_t b = 0;
    int used = 4;
    for (int32_t i = r - 1; i >= 1; --i) {
        if (used == 4) {
            uint64_t ctr[4] = {b++, t, stream, 0};
            orc_philox4x64_10(ctr, key, blk);
            used = 0;
        }
        uint64_t w = blk[used++];
        int32_t j = (int32_t)(((__uint128_t)w * (uint64_t)(i + 1)) >> 64);
        int32_t tmp = ids[i]; ids[i] = ids[j]; ids[j] = tmp;
    }
}

/* sumA = A 1 : column sums of the point-major factor (Alg. 1: sumW = W 1^n, sumF = F 1^m) */
void orc_factor_sums(int64_t P, int32_t r, const double* A, double* sumA) {
    for (int32_t k = 0; k < r; ++k) sumA[k] = 0.0;
    for (int64_t p = 0; p < P; ++p)
        for (int32_t k = 0; k < r; ++k) sumA[k] += A[p * r + k];
}

/* [Ax]_l at the nonzeros of v, skipping coordinates with x_k = 0 (Alg. 2 first step and
 * the sparsity remark of Section 2). */
static void model_at_nonzeros(int64_t L, const int32_t* idx, const double* A, int32_t r,
                              const double* x, double* Ax) {
    for (int64_t l = 0; l < L; ++l) {
        double s = 0.0;
        const double* a = A + (int64_t)idx[l] * r;
        for (int32_t k = 0; k < r; ++k)
            if (x[k] != 0.0) s += a[k] * x[k];
        Ax[l] = s;
    }
}

/* eq. 6 for coordinate k at the model Ax (with eps_log in the denominators):
 *   g = -sum v_l A_lk/(Ax_l+eps) + sumA_k + alpha x_k + beta,
 *   h =  sum v_l (A_lk/(Ax_l+eps))^2 + alpha.
 * P = sumA_k + alpha x_k + beta is returned too (the scale of the while-test). */
void orc_coordinate_derivatives(int64_t L, const int32_t* idx, const double* v,
                                const double* A, int32_t r, int32_t k, const double* Ax,
                                double sumA_k, double xk, double alpha, double beta,
                                double eps_log, double* g, double* h, double* P) {
    double S1 = 0.0, S2 = 0.0;
    for (int64_t l = 0; l < L; ++l) {
        double q = A[(int64_t)idx[l] * r + k] / (Ax[l] + eps_log);
        S1 += v[l] * q;
        S2 += v[l] * q * q;
    }
    *P = sumA_k + alpha * xk + beta;
    *g = *P - S1;
    *h = S2 + alpha;
}

/* The objective Alg. 2 minimises (its output line, without constants):
 *   f(x) = sum_l -v_l log([Ax]_l + eps) + sum_i [Ax]_i + alpha/2 |x|^2 + beta |x|_1,
 * where sum over all n points of [Ax]_i = sum_k sumA_k x_k. */
double orc_subproblem_value(int64_t L, const int32_t* idx, const double* v, const double* A,
                            int32_t r, const double* sumA, const double* x, double alpha,
                            double beta, double eps_log) {
    double f = 0.0;
    for (int64_t l = 0; l < L; ++l) {
        const double* a = A + (int64_t)idx[l] * r;
        double s = 0.0;
        for (int32_t k = 0; k < r; ++k) s += a[k] * x[k];
        f -= v[l] * log(s + eps_log);
    }
    for (int32_t k = 0; k < r; ++k) f += sumA[k] * x[k] + 0.5 * alpha * x[k] * x[k] + beta * x[k];
    return f;
}

static int enter_loop(double g, double P, double xk, double eps_g) {
    return (g < -eps_g * P) || (g > eps_g * P && xk > 0.0);
}

/* The trial model at x_k + d: max(0, Ax_l + d A_lk). */
static void trial_model(int64_t L, const int32_t* idx, const double* A, int32_t r, int32_t k,
                        const double* Ax, double d, double* Axn) {
    for (int64_t l = 0; l < L; ++l) {
        double m = Ax[l] + d * A[(int64_t)idx[l] * r + k];
        Axn[l] = m > 0.0 ? m : 0.0;
    }
}

/* The inner while-loop of Alg. 2 for one coordinate k: projected Newton steps
 * x_k <- max(0, x_k - g/h) with the model update Ax += dx A_k, the re-derivation of
 * (g, h), the descent guard and the break test.  Ax (length L) is updated in place;
 * Axn is scratch of length L. */
void orc_coordinate_update(int64_t L, const int32_t* idx, const double* v, const double* A,
                           int32_t r, const double* sumA, double* x, double alpha,
                           double beta, int32_t k, const orc_params* prm, double* Ax,
                           double* Axn, orc_stats* st) {
    double g, h, P;
    orc_coordinate_derivatives(L, idx, v, A, r, k, Ax, sumA[k], x[k], alpha, beta,
                               prm->eps_log, &g, &h, &P);
    st->coords++; st->evals++;
    int32_t steps = 0;
    while (enter_loop(g, P, x[k], prm->eps_g)) {
        double d;
        if (h <= 0.0) {
            if (g > 0.0) d = -x[k];
            else break;
        } else {
            double xn = x[k] - g / h;
            d = (xn > 0.0 ? xn : 0.0) - x[k];
        }
        const double dN = d; /* the projected Newton step of Alg. 2 (before any halving) */
        double gn, hn, Pn;
        trial_model(L, idx, A, r, k, Ax, d, Axn);
        orc_coordinate_derivatives(L, idx, v, A, r, k, Axn, sumA[k], x[k] + d, alpha, beta,
                                   prm->eps_log, &gn, &hn, &Pn);
        st->evals++;
        if (prm->guard && d < 0.0) {
            int32_t j = 0;
            while (g + gn < 0.0 && j < prm->j_max) {
                d = 0.5 * d;
                trial_model(L, idx, A, r, k, Ax, d, Axn);
                orc_coordinate_derivatives(L, idx, v, A, r, k, Axn, sumA[k], x[k] + d, alpha,
                                           beta, prm->eps_log, &gn, &hn, &Pn);
                st->evals++; st->halvings++;
                ++j;
            }
            if (g + gn < 0.0) { st->rejects++; break; }
        }
        double xs = x[k];
        x[k] = xs + d;
        memcpy(Ax, Axn, (size_t)L * sizeof(double));
        g = gn; h = hn; P = Pn;
        ++steps;
        st->steps++;
        int stop = prm->literal_break ? (dN < prm->eps_x * xs) : (fabs(dN) < prm->eps_x * xs);
        if (stop) break;
        if (steps >= prm->t_max) { st->tmax_hits++; break; }
    }
}

/* Alg. 2: compute Ax, then visit the coordinates in the order ids. */
void orc_alg2(int64_t L, const int32_t* idx, const double* v, const double* A, int32_t r,
              const double* sumA, double* x, double alpha, double beta, const int32_t* ids,
              const orc_params* prm, double* Ax, double* Axn, orc_stats* st) {
    model_at_nonzeros(L, idx, A, r, x, Ax);
    for (int32_t s = 0; s < r; ++s)
        orc_coordinate_update(L, idx, v, A, r, sumA, x, alpha, beta, ids[s], prm, Ax, Axn, st);
}

/* One half of Alg. 1's while-body: for every segment (column of V for the F-half, row of V
 * for the W-half), Alg. 2 with the fixed factor A and its sums.  X (Q x r) is updated. */
static void half_sweep(int64_t Q, const int64_t* ptr, const int32_t* idx, const double* val,
                       int64_t P, const double* A, double* X, int32_t r, double alpha,
                       double beta, const int32_t* ids, const orc_params* prm, orc_stats* st,
                       double* sumA_out) {
    double* sumA = (double*)malloc((size_t)r * sizeof(double));
    orc_factor_sums(P, r, A, sumA);
    if (sumA_out) memcpy(sumA_out, sumA, (size_t)r * sizeof(double));
    int64_t Lmax = 0;
    for (int64_t q = 0; q < Q; ++q) if (ptr[q + 1] - ptr[q] > Lmax) Lmax = ptr[q + 1] - ptr[q];
    orc_stats total = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
    {
        double* Ax = (double*)malloc((size_t)(Lmax + 1) * sizeof(double));
        double* Axn = (double*)malloc((size_t)(Lmax + 1) * sizeof(double));
        orc_stats local = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < Q; ++q) {
            int64_t b = ptr[q], L = ptr[q + 1] - ptr[q];
            orc_alg2(L, idx + b, val + b, A, r, sumA, X + q * r, alpha, beta, ids, prm, Ax, Axn,
                     &local);
        }
#pragma omp critical
        stats_add(&total, &local);
        free(Ax);
        free(Axn);
    }
    if (st) stats_add(st, &total);
    free(sumA);
}

/* Alg. 1, F-half: sumW = W 1, then every column j of V (CSC) updates F_j with (alpha_2,
 * beta_2). */
void orc_sweep_F(int32_t n, int32_t m, int32_t r, const int64_t* csc_ptr,
                 const int32_t* csc_idx, const double* csc_val, const double* W, double* F,
                 const int32_t* ids, const orc_params* prm, orc_stats* st, double* sumW_out) {
    half_sweep(m, csc_ptr, csc_idx, csc_val, n, W, F, r, prm->alpha_F, prm->beta_F, ids, prm,
               st, sumW_out);
}

/* Alg. 1, W-half: sumF = F 1, then every row i of V (CSR) updates W_i with sumF and
 * (alpha_1, beta_1). */
void orc_sweep_W(int32_t n, int32_t m, int32_t r, const int64_t* csr_ptr,
                 const int32_t* csr_idx, const double* csr_val, const double* F, double* W,
                 const int32_t* ids, const orc_params* prm, orc_stats* st, double* sumF_out) {
    half_sweep(n, csr_ptr, csr_idx, csr_val, m, F, W, r, prm->alpha_W, prm->beta_W, ids, prm,
               st, sumF_out);
}

/* eq. 1: D(V || W^T F) = sum_ij V_ij log(V_ij/M_ij) - V_ij + M_ij, M = W^T F.
 * The sum of M over all n*m cells equals sumW . sumF.  A nonzero with M = 0 gives +inf;
 * explicit zeros of V contribute only through sum M. */
double orc_objective(int32_t n, int32_t m, int32_t r, const int64_t* csc_ptr,
                     const int32_t* csc_idx, const double* csc_val, const double* W,
                     const double* F) {
    double* sw = (double*)malloc((size_t)r * sizeof(double));
    double* sf = (double*)malloc((size_t)r * sizeof(double));
    orc_factor_sums(n, r, W, sw);
    orc_factor_sums(m, r, F, sf);
    double total = 0.0;
    for (int32_t k = 0; k < r; ++k) total += sw[k] * sf[k];
    /* each column's terms in storage order, then the columns in order: the same value
     * for any number of threads */
    double* col = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        double cj = 0.0;
        for (int64_t q = csc_ptr[j]; q < csc_ptr[j + 1]; ++q) {
            double v = csc_val[q];
            if (v == 0.0) continue;
            const double* w = W + (int64_t)csc_idx[q] * r;
            double M = 0.0;
            for (int32_t k = 0; k < r; ++k) M += w[k] * F[j * r + k];
            cj += v * log(v / M) - v;
        }
        col[j] = cj;
    }
    double part = 0.0;
    for (int64_t j = 0; j < m; ++j) part += col[j];
    free(col);
    free(sw);
    free(sf);
    return part + total;
}

/* The objective restricted to one column with W fixed:
 *   KL(v || A x) = sum_l (v_l log(v_l/[Ax]_l) - v_l) + sum_k sumA_k x_k. */
double orc_column_kl(int64_t L, const int32_t* idx, const double* v, const double* A,
                     int32_t r, const double* sumA, const double* x) {
    double kl = 0.0;
    for (int64_t l = 0; l < L; ++l) {
        if (v[l] == 0.0) continue;
        const double* a = A + (int64_t)idx[l] * r;
        double M = 0.0;
        for (int32_t k = 0; k < r; ++k) M += a[k] * x[k];
        kl += v[l] * log(v[l] / M) - v[l];
    }
    for (int32_t k = 0; k < r; ++k) kl += sumA[k] * x[k];
    return kl;
}

/* Fold-in of new documents with W fixed (Alg. 1's F-half applied to new columns; the
 * columns are independent).  Start: x = (sum_l v_l / sum_k sumW_k) 1.  Pass p runs
 * Alg. 2 once with the order from counter (p, stream 1); stop after the first pass whose
 * KL decrease is <= foldin_tol * KL, or after foldin_max_passes passes. */
void orc_foldin(int32_t n, int32_t r, const double* W, int64_t ndocs, const int64_t* doc_ptr,
                const int32_t* word_idx, const double* counts, const orc_params* prm,
                double* F_out, int32_t* passes_out, double* kl_out, orc_stats* st) {
    double* sumW = (double*)malloc((size_t)r * sizeof(double));
    orc_factor_sums(n, r, W, sumW);
    double totW = 0.0;
    for (int32_t k = 0; k < r; ++k) totW += sumW[k];
    int32_t PM = prm->foldin_max_passes;
    int32_t* tab = (int32_t*)malloc((size_t)PM * r * sizeof(int32_t));
    for (int32_t p = 0; p < PM; ++p) orc_permutation(prm->seed, (uint64_t)p, 1, r, tab + (int64_t)p * r);
    int64_t Lmax = 0;
    for (int64_t d = 0; d < ndocs; ++d) if (doc_ptr[d + 1] - doc_ptr[d] > Lmax) Lmax = doc_ptr[d + 1] - doc_ptr[d];
    orc_stats total = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
    {
        double* Ax = (double*)malloc((size_t)(Lmax + 1) * sizeof(double));
        double* Axn = (double*)malloc((size_t)(Lmax + 1) * sizeof(double));
        orc_stats local = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int64_t d = 0; d < ndocs; ++d) {
            int64_t b = doc_ptr[d], L = doc_ptr[d + 1] - doc_ptr[d];
            double* x = F_out + d * r;
            double mass = 0.0;
            for (int64_t l = 0; l < L; ++l) mass += counts[b + l];
            for (int32_t k = 0; k < r; ++k) x[k] = mass / totW;
            double kl_prev = orc_column_kl(L, word_idx + b, counts + b, W, r, sumW, x);
            double kl = kl_prev;
            int32_t p = 0;
            while (p < PM) {
                orc_alg2(L, word_idx + b, counts + b, W, r, sumW, x, prm->alpha_F, prm->beta_F,
                         tab + (int64_t)p * r, prm, Ax, Axn, &local);
                ++p;
                kl = orc_column_kl(L, word_idx + b, counts + b, W, r, sumW, x);
                if (kl_prev - kl <= prm->foldin_tol * kl) break;
                kl_prev = kl;
            }
            passes_out[d] = p;
            kl_out[d] = kl;
        }
#pragma omp critical
        stats_add(&total, &local);
        free(Ax);
        free(Axn);
    }
    if (st) stats_add(st, &total);
    free(tab);
    free(sumW);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
    omp_set_num_threads(t);
#else
    (void)t;
#endif
}
