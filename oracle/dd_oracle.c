/*
 * dd_oracle.c -- plain FP64 CPU oracle for generalized min-marginal averaging.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or helper with the GPU library: it never builds a
 * binary decision diagram.  Instead every min-marginal is computed on the
 * unreduced decision diagram whose states at level l are the integer partial
 * sums s = sum_{p<l} a_p x_p of the row, which is a direct dynamic program for
 *
 *     m^beta_l = min { <lambda, x> : x in X_j, x_l = beta }     (Alg. 1, min-marginal line)
 *
 * with X_j = { x in {0,1}^{I_j} : a_j^T x (<=,=,>=) b_j } (Def. 1 and the ILP
 * to BP rewrite below it).  Prefix table P_l(s) is the shortest path from the
 * root to state s at level l, suffix table Q_l(s) the shortest path from it to
 * the accepting end, so m^beta_l = min_s P_l(s) + beta*lambda_l + Q_{l+1}(s + beta*a_l)
 * -- eq. 8 of App. B on this diagram.
 *
 * Conventions (readings of the paper, all stated in the design notes):
 *  - edges (Lagrange multipliers lambda_ij) are stored row-major with the
 *    variables of each row in ascending index order; a forward pass visits the
 *    hops of every row in that order, a backward pass in reverse (blocks B_1..B_u
 *    of Alg. 1 = hop positions);
 *  - the deferred term of Alg. 1's lambda update uses S_i = sum_{k in J_i} M_ik
 *    taken at the start of the pass (the feasibility proof of Prop. 1 needs
 *    exactly this);
 *  - lambda starts at c_i / |J_i|, M at 0;
 *  - the lower bound is (D) evaluated at the flushed multipliers
 *    lambda_bar = lambda + alpha * S, plus min(0, c_i) for every variable that
 *    appears in no row;
 *  - every row must be feasible and must not fix any of its variables
 *    (otherwise a min-marginal is infinite): such rows are rejected.
 *
 * Status codes: 0 ok, -1 bad argument, -2 infeasible row, -3 row fixes a variable.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_INFEASIBLE (-2)
#define ORC_E_FORCED (-3)

static const double INF = HUGE_VAL;

/* One constraint row seen as a subproblem. */
typedef struct {
    int L;              /* number of variables */
    const int32_t *var; /* ascending global variable ids */
    const int32_t *a;   /* integer coefficients */
    int sense;          /* -1 <=, 0 ==, +1 >= */
    int64_t rhs;
    int64_t smin;       /* smallest partial sum: sum of negative coefficients */
    int W;              /* number of partial-sum states: sum |a| + 1 */
} row_t;

static int row_init(row_t *r, int L, const int32_t *var, const int32_t *a, int sense, int64_t rhs) {
    r->L = L; r->var = var; r->a = a; r->sense = sense; r->rhs = rhs;
    int64_t lo = 0, hi = 0;
    for (int l = 0; l < L; ++l) {
        if (a[l] < 0) lo += a[l]; else hi += a[l];
        if (l > 0 && var[l] <= var[l - 1]) return ORC_E_ARG; /* unsorted or duplicate */
    }
    if (hi - lo + 1 > (int64_t)1 << 26) return ORC_E_ARG;
    r->smin = lo;
    r->W = (int)(hi - lo + 1);
    return ORC_OK;
}

static int accepts(const row_t *r, int64_t s) {
    if (r->sense < 0) return s <= r->rhs;
    if (r->sense > 0) return s >= r->rhs;
    return s == r->rhs;
}

/* Table entry (level l, partial sum s), INF outside the range of sums. */
static double at(const row_t *r, const double *T, int l, int64_t s) {
    int64_t k = s - r->smin;
    if (k < 0 || k >= r->W) return INF;
    return T[(size_t)l * r->W + k];
}

/* P_0(0) = 0; P_{l+1}(s) = min(P_l(s), P_l(s - a_l) + lambda_l). */
static void prefix_level(const row_t *r, const double *lam, double *P, int l) {
    for (int k = 0; k < r->W; ++k) {
        int64_t s = r->smin + k;
        double x0 = at(r, P, l, s);
        double x1 = at(r, P, l, s - r->a[l]) + lam[l];
        P[(size_t)(l + 1) * r->W + k] = x0 <= x1 ? x0 : x1;
    }
}
static void prefix_init(const row_t *r, double *P) {
    for (int k = 0; k < r->W; ++k) P[k] = INF;
    P[-r->smin] = 0.0;
}
static void prefix_table(const row_t *r, const double *lam, double *P) {
    prefix_init(r, P);
    for (int l = 0; l < r->L; ++l) prefix_level(r, lam, P, l);
}

/* Q_L(s) = 0 if s satisfies the row else INF; Q_l(s) = min(Q_{l+1}(s), lambda_l + Q_{l+1}(s + a_l)). */
static void suffix_level(const row_t *r, const double *lam, double *Q, int l) {
    for (int k = 0; k < r->W; ++k) {
        int64_t s = r->smin + k;
        double x0 = at(r, Q, l + 1, s);
        double x1 = lam[l] + at(r, Q, l + 1, s + r->a[l]);
        Q[(size_t)l * r->W + k] = x0 <= x1 ? x0 : x1;
    }
}
static void suffix_init(const row_t *r, double *Q) {
    for (int k = 0; k < r->W; ++k) Q[(size_t)r->L * r->W + k] = accepts(r, r->smin + k) ? 0.0 : INF;
}
static void suffix_table(const row_t *r, const double *lam, double *Q) {
    suffix_init(r, Q);
    for (int l = r->L - 1; l >= 0; --l) suffix_level(r, lam, Q, l);
}

/* eq. 8 on the partial-sum diagram: m^beta_l from P_l and Q_{l+1}. */
static void marginals(const row_t *r, const double *P, const double *Q, const double *lam, int l,
                      double *m0, double *m1) {
    double b0 = INF, b1 = INF;
    for (int k = 0; k < r->W; ++k) {
        double p = P[(size_t)l * r->W + k];
        if (p == INF) continue;
        int64_t s = r->smin + k;
        double c0 = p + at(r, Q, l + 1, s);
        double c1 = p + lam[l] + at(r, Q, l + 1, s + r->a[l]);
        if (c0 < b0) b0 = c0;
        if (c1 < b1) b1 = c1;
    }
    *m0 = b0; *m1 = b1;
}

/* E^j(lambda) = min_{x in X_j} <lambda, x>  (eq. 1). */
static double energy(const row_t *r, const double *lam, double *Q) {
    suffix_table(r, lam, Q);
    return Q[-r->smin];
}

/* Smallest gap between the two options of any decision taken so far, relative (|a - b| divided by
 * the larger of |a|, |b|) and absolute (|a - b|).  A diagnostic: where it is below the rounding
 * error of the values compared, the minimizer is not unique up to rounding, so any of the
 * candidates gives a valid subgradient. */
typedef struct {
    double rel, abs;
} gap_t;
static void note_gap(gap_t *gap, double a, double b) {
    if (!gap || a == INF || b == INF) return;
    double d = fabs(a - b), s = fmax(fmax(fabs(a), fabs(b)), 1e-300);
    if (d / s < gap->rel) gap->rel = d / s;
    if (d < gap->abs) gap->abs = d;
}

/* Minimizer of <lam, x> over X_j with x_l = beta (l = -1: unconstrained), written to x[0..L).
 * Ties: lowest partial sum, then x_p = 0 before x_p = 1.  gap (may be NULL): see note_gap. */
static void minimizer(const row_t *r, const double *lam, const double *P, const double *Q, int l, int beta,
                      int8_t *x, gap_t *gap) {
    int64_t s;
    if (l < 0) {
        s = 0;
        for (int p = 0; p < r->L; ++p) {
            double x0 = at(r, Q, p + 1, s), x1 = lam[p] + at(r, Q, p + 1, s + r->a[p]);
            note_gap(gap, x0, x1);
            x[p] = x0 <= x1 ? 0 : 1;
            if (x[p]) s += r->a[p];
        }
        return;
    }
    double best = INF, second = INF; int64_t sb = 0;
    for (int k = 0; k < r->W; ++k) {
        int64_t ss = r->smin + k;
        double v = at(r, P, l, ss) + (beta ? lam[l] : 0.0) + at(r, Q, l + 1, ss + (beta ? r->a[l] : 0));
        if (v < best) { second = best; best = v; sb = ss; }
        else if (v < second) second = v;
    }
    note_gap(gap, best, second);
    x[l] = (int8_t)beta;
    s = sb;
    for (int p = l - 1; p >= 0; --p) {           /* back through the prefix table */
        double x0 = at(r, P, p, s), x1 = at(r, P, p, s - r->a[p]) + lam[p];
        note_gap(gap, x0, x1);
        x[p] = x0 <= x1 ? 0 : 1;
        if (x[p]) s -= r->a[p];
    }
    s = sb + (beta ? r->a[l] : 0);
    for (int p = l + 1; p < r->L; ++p) {         /* forward through the suffix table */
        double x0 = at(r, Q, p + 1, s), x1 = lam[p] + at(r, Q, p + 1, s + r->a[p]);
        note_gap(gap, x0, x1);
        x[p] = x0 <= x1 ? 0 : 1;
        if (x[p]) s += r->a[p];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Near-ties: how far the adjoint can move when another engine takes other decisions.          */
/* The adjoint routes through minimizers, so it is a function of the decisions taken while     */
/* tracing them.  Another engine whose arithmetic differs (fp32 instead of fp64) may take the   */
/* other option of a decision whose two options lie within its rounding error of each other,   */
/* and both choices give valid subgradients.  The functions below bound, per output, how much  */
/* such flips can change it ("flip bound"; 0: the output is determined and must agree).  tol   */
/* is the caller's bound on how far the compared values can lie from this oracle's.  The bound */
/* is first order: decisions are flipped one at a time, and the changes they cause are carried */
/* through the adjoint recurrences with absolute values.                                        */
/* ------------------------------------------------------------------------------------------ */

/* Greedy trace back through the prefix table from state s at level p: xv[q] for q < p
 * (the rules of minimizer()). */
static void trace_back(const row_t *r, const double *lam, const double *P, int p, int64_t s, int8_t *xv) {
    for (int q = p - 1; q >= 0; --q) {
        double x0 = at(r, P, q, s), x1 = at(r, P, q, s - r->a[q]) + lam[q];
        xv[q] = x0 <= x1 ? 0 : 1;
        if (xv[q]) s -= r->a[q];
    }
}

/* Greedy trace forward through the suffix table from state s at level p: xv[q] for q >= p. */
static void trace_fwd(const row_t *r, const double *lam, const double *Q, int p, int64_t s, int8_t *xv) {
    for (int q = p; q < r->L; ++q) {
        double x0 = at(r, Q, q + 1, s), x1 = lam[q] + at(r, Q, q + 1, s + r->a[q]);
        xv[q] = x0 <= x1 ? 0 : 1;
        if (xv[q]) s += r->a[q];
    }
}

static int near(double a, double b, double tol) { return a != INF && b != INF && fabs(a - b) <= tol; }

/* amb[q] = 1 for every position q where the minimizer x traced by minimizer() for (l, beta) changes
 * when one of its decisions whose two options lie within tol goes the other way: that option is
 * traced to the end by the same rules and compared with x.  Decisions are flipped one at a time. */
static void near_ties(const row_t *r, const double *lam, const double *P, const double *Q, int l, int beta,
                      const int8_t *x, double tol, int8_t *amb, int8_t *alt) {
    const int L = r->L;
    int64_t s;
    if (l < 0) {
        s = 0;
        for (int p = 0; p < L; ++p) {
            double x0 = at(r, Q, p + 1, s), x1 = lam[p] + at(r, Q, p + 1, s + r->a[p]);
            if (near(x0, x1, tol)) {
                alt[p] = (int8_t)(1 - x[p]);
                trace_fwd(r, lam, Q, p + 1, s + (alt[p] ? r->a[p] : 0), alt);
                for (int q = p; q < L; ++q) if (alt[q] != x[q]) amb[q] = 1;
            }
            if (x[p]) s += r->a[p];
        }
        return;
    }
    const int64_t shift = beta ? r->a[l] : 0;
    double best = INF; int64_t sb = 0;
    for (int k = 0; k < r->W; ++k) {
        int64_t ss = r->smin + k;
        double v = at(r, P, l, ss) + (beta ? lam[l] : 0.0) + at(r, Q, l + 1, ss + shift);
        if (v < best) { best = v; sb = ss; }
    }
    for (int k = 0; k < r->W; ++k) {            /* another state of level l within tol */
        int64_t ss = r->smin + k;
        double v = at(r, P, l, ss) + (beta ? lam[l] : 0.0) + at(r, Q, l + 1, ss + shift);
        if (ss == sb || !near(v, best, tol)) continue;
        alt[l] = (int8_t)beta;
        trace_back(r, lam, P, l, ss, alt);
        trace_fwd(r, lam, Q, l + 1, ss + shift, alt);
        for (int q = 0; q < L; ++q) if (alt[q] != x[q]) amb[q] = 1;
    }
    s = sb;
    for (int p = l - 1; p >= 0; --p) {           /* decisions back through the prefix table */
        double x0 = at(r, P, p, s), x1 = at(r, P, p, s - r->a[p]) + lam[p];
        if (near(x0, x1, tol)) {
            alt[p] = (int8_t)(1 - x[p]);
            trace_back(r, lam, P, p, s - (alt[p] ? r->a[p] : 0), alt);
            for (int q = 0; q <= p; ++q) if (alt[q] != x[q]) amb[q] = 1;
        }
        if (x[p]) s -= r->a[p];
    }
    s = sb + shift;
    for (int p = l + 1; p < L; ++p) {            /* decisions forward through the suffix table */
        double x0 = at(r, Q, p + 1, s), x1 = lam[p] + at(r, Q, p + 1, s + r->a[p]);
        if (near(x0, x1, tol)) {
            alt[p] = (int8_t)(1 - x[p]);
            trace_fwd(r, lam, Q, p + 1, s + (alt[p] ? r->a[p] : 0), alt);
            for (int q = p; q < L; ++q) if (alt[q] != x[q]) amb[q] = 1;
        }
        if (x[p]) s += r->a[p];
    }
}

/* Flip bounds of one row's pass adjoint (all arrays indexed by the row's positions). */
typedef struct {
    double tol;                          /* decision tolerance of this row */
    const double *dlo, *dmo;             /* bounds of the adjoints of the pass outputs (NULL: 0) */
    double *dli, *gS, *dalpha, *domega;  /* outputs: dli, gS set; dalpha, domega accumulated */
    double *wscale;                      /* output, accumulated: |Mt| s_j, the size of d_omega's rounding
                                            (d_omega = Mt (m1 - m0), a difference of path costs of size
                                            s_j = sum_p |lambda_p| of the row) */
    double *ad;                          /* scratch: bound of ad_new */
    int8_t *amb0, *amb1, *alt;           /* scratch */
} taint_t;

/* ------------------------------------------------------------------------------------------ */
/* One pass of Alg. 1 on one row: BlockUpdate for each hop in pass order.                      */
/*   M_new = omega (m1 - m0);  lambda_new = lambda - M_new + alpha * S  (S: pass-start sum).    */
/* literal = 1 recomputes both tables from scratch for every hop; literal = 0 keeps the prefix */
/* (forward) or suffix (backward) table up to date hop by hop and takes the other one from the */
/* pass-start multipliers, which are still current for the hops not yet visited.              */
/* ------------------------------------------------------------------------------------------ */
static int row_pass(const row_t *r, int dir, int literal, const double *omega, const double *alpha,
                    const double *S, double *lam, double *Mout, double *P, double *Q) {
    const int L = r->L;
    if (!literal) {
        if (dir == 0) { suffix_table(r, lam, Q); prefix_init(r, P); }
        else { prefix_table(r, lam, P); suffix_init(r, Q); }
    }
    for (int h = 0; h < L; ++h) {
        int l = dir == 0 ? h : L - 1 - h;
        if (literal) { prefix_table(r, lam, P); suffix_table(r, lam, Q); }
        double m0, m1;
        marginals(r, P, Q, lam, l, &m0, &m1);
        if (m0 == INF && m1 == INF) return ORC_E_INFEASIBLE;
        if (m0 == INF || m1 == INF) return ORC_E_FORCED;
        double Mn = omega[l] * (m1 - m0);
        lam[l] = lam[l] - Mn + alpha[l] * S[l];
        Mout[l] = Mn;
        if (!literal) {
            if (dir == 0) prefix_level(r, lam, P, l);
            else suffix_level(r, lam, Q, l);
        }
    }
    return ORC_OK;
}

static int max_table(int m, const int64_t *row_ptr, const int32_t *coef, size_t *out) {
    size_t mx = 0;
    for (int j = 0; j < m; ++j) {
        int64_t w = 1;
        for (int64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) w += coef[e] < 0 ? -(int64_t)coef[e] : coef[e];
        size_t sz = (size_t)(row_ptr[j + 1] - row_ptr[j] + 1) * (size_t)w;
        if (sz > mx) mx = sz;
    }
    *out = mx;
    return ORC_OK;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* S_i = sum_{k in J_i} M_ik, summed in edge order; S_edge[e] = S_{var(e)}. */
static void deferred_sums(int n, int64_t E, const int32_t *col, const double *M, double *S_var, double *S_edge) {
    memset(S_var, 0, sizeof(double) * (size_t)n);
    for (int64_t e = 0; e < E; ++e) S_var[col[e]] += M[e];
    for (int64_t e = 0; e < E; ++e) S_edge[e] = S_var[col[e]];
}

/* Pass over the given rows with the deferred sums supplied per edge (rows are independent
 * given S, so a subset of rows can be checked against any engine's pass-start state). */
int orc_rows_pass(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                  const int64_t *rhs, const double *omega, const double *alpha, const double *S_edge, int dir,
                  int literal, double *lam, double *M, int nthreads) {
    if (m < 0 || (dir != 0 && dir != 1)) return ORC_E_ARG;
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    set_threads(nthreads);
    int status = ORC_OK;
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * tab);
        double *Q = (double *)malloc(sizeof(double) * tab);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            if (st == ORC_OK)
                st = row_pass(&r, dir, literal, omega + b, alpha + b, S_edge + b, lam + b, M + b, P, Q);
            if (st != ORC_OK) {
#pragma omp critical
                status = st;
            }
        }
        free(P); free(Q);
    }
    return status;
}

/* lambda_e = c_i / |J_i| for every edge e = (i, j). */
int orc_init_lambda(int n, const double *c, int64_t E, const int32_t *col, double *lam) {
    int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!deg) return ORC_E_ARG;
    for (int64_t e = 0; e < E; ++e) deg[col[e]]++;
    for (int64_t e = 0; e < E; ++e) lam[e] = c[col[e]] / (double)deg[col[e]];
    free(deg);
    return ORC_OK;
}

/* One pass of Alg. 1 over all rows: dir 0 = forward (B_1..B_u), 1 = backward. */
int orc_pass(int n, int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
             const int64_t *rhs, const double *omega, const double *alpha, int dir, int literal, double *lam,
             double *M, int nthreads) {
    int64_t E = row_ptr[m];
    double *Sv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *Se = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    deferred_sums(n, E, col, M, Sv, Se);
    int st = orc_rows_pass(m, row_ptr, col, coef, sense, rhs, omega, alpha, Se, dir, literal, lam, M, nthreads);
    free(Sv); free(Se);
    return st;
}

/* T iterations of Alg. 1 (each a forward then a backward pass), lambda and M in/out. */
int orc_run(int n, int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
            const int64_t *rhs, const double *omega, const double *alpha, int T, int literal, double *lam, double *M,
            int nthreads) {
    for (int t = 0; t < T; ++t)
        for (int dir = 0; dir < 2; ++dir) {
            int st = orc_pass(n, m, row_ptr, col, coef, sense, rhs, omega, alpha, dir, literal, lam, M, nthreads);
            if (st) return st;
        }
    return ORC_OK;
}

/* E^j(lam_{.j}) for every row (eq. 1). */
int orc_energies(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                 const int64_t *rhs, const double *lam, double *Ej, int nthreads) {
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    set_threads(nthreads);
    int status = ORC_OK;
#pragma omp parallel
    {
        double *Q = (double *)malloc(sizeof(double) * tab);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            if (st) {
#pragma omp critical
                status = st;
                continue;
            }
            Ej[j] = energy(&r, lam + b, Q);
            if (Ej[j] == INF) {
#pragma omp critical
                status = ORC_E_INFEASIBLE;
            }
        }
        free(Q);
    }
    return status;
}

/* Smoothed subproblem (the smoothing of the feature table of the appendix, read as a soft-min):
 * E_tau^j(lambda) = -tau log sum_{x in X_j} exp(-<lambda, x> / tau), which tends to E^j as tau -> 0.
 * Its gradient is the Gibbs marginal p_l = P(x_l = 1) under exp(-<lambda, x>/tau) on X_j.  Computed
 * with the prefix/suffix tables of the partial-sum diagram in the (soft-min, +) semiring (every x
 * is one path of that diagram). */
static double softmin2(double a, double b, double tau) {
    if (a == INF) return b;
    if (b == INF) return a;
    double m = a < b ? a : b, d = fabs(a - b);
    return m - tau * log1p(exp(-d / tau));
}

static void smoothed_row(const row_t *r, const double *lam, double tau, double *P, double *Q, double *E, double *p) {
    for (int k = 0; k < r->W; ++k) P[k] = INF;
    P[-r->smin] = 0.0;
    for (int l = 0; l < r->L; ++l)
        for (int k = 0; k < r->W; ++k) {
            int64_t s = r->smin + k;
            P[(size_t)(l + 1) * r->W + k] = softmin2(at(r, P, l, s), at(r, P, l, s - r->a[l]) + lam[l], tau);
        }
    suffix_init(r, Q);
    for (int l = r->L - 1; l >= 0; --l)
        for (int k = 0; k < r->W; ++k) {
            int64_t s = r->smin + k;
            Q[(size_t)l * r->W + k] = softmin2(at(r, Q, l + 1, s), lam[l] + at(r, Q, l + 1, s + r->a[l]), tau);
        }
    double e = Q[-r->smin];
    *E = e;
    for (int l = 0; l < r->L; ++l) {
        double acc = 0.0;
        for (int k = 0; k < r->W; ++k) {
            double pl = P[(size_t)l * r->W + k];
            if (pl == INF) continue;
            double c1 = pl + lam[l] + at(r, Q, l + 1, r->smin + k + r->a[l]);
            if (c1 != INF) acc += exp(-(c1 - e) / tau);
        }
        p[l] = acc;
    }
}

int orc_smoothed(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                 const int64_t *rhs, const double *lam, double tau, double *E_out, double *p_out, int nthreads) {
    if (!(tau > 0.0)) return ORC_E_ARG;
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    set_threads(nthreads);
    int status = ORC_OK;
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * tab);
        double *Q = (double *)malloc(sizeof(double) * tab);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            if (st) {
#pragma omp critical
                status = st;
                continue;
            }
            double E;
            smoothed_row(&r, lam + b, tau, P, Q, &E, p_out + b);
            if (E_out) E_out[j] = E;
        }
        free(P);
        free(Q);
    }
    return status;
}

/* Lower bound: lambda_bar = lambda + alpha * S(M), LB = sum_j E^j(lambda_bar) + sum_{|J_i|=0} min(0, c_i).
 * Also D_L = sum_j E^j(lambda) + sum_e min(0, M_e), the lifted-representation bound of Prop. 1's proof.
 * lam_bar_out (optional) receives lambda_bar. */
int orc_lower_bound(int n, int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef,
                    const int8_t *sense, const int64_t *rhs, const double *c, const double *alpha, const double *lam,
                    const double *M, double *lb, double *dl, double *lam_bar_out, int nthreads) {
    int64_t E = row_ptr[m];
    double *Sv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *Se = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double *lb_lam = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double *Ej = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    deferred_sums(n, E, col, M, Sv, Se);
    for (int64_t e = 0; e < E; ++e) lb_lam[e] = lam[e] + alpha[e] * Se[e];
    if (lam_bar_out) memcpy(lam_bar_out, lb_lam, sizeof(double) * (size_t)E);
    int st = orc_energies(m, row_ptr, col, coef, sense, rhs, lb_lam, Ej, nthreads);
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += Ej[j];
    for (int64_t e = 0; e < E; ++e) deg[col[e]]++;
    double unc = 0.0;
    for (int i = 0; i < n; ++i)
        if (deg[i] == 0 && c[i] < 0.0) unc += c[i];
    *lb = s + unc;
    if (st == ORC_OK) st = orc_energies(m, row_ptr, col, coef, sense, rhs, lam, Ej, nthreads);
    s = 0.0;
    for (int j = 0; j < m; ++j) s += Ej[j];
    for (int64_t e = 0; e < E; ++e) s += M[e] < 0.0 ? M[e] : 0.0;
    *dl = s + unc;
    free(Sv); free(Se); free(lb_lam); free(Ej); free(deg);
    return st;
}

/* Min-marginals m0, m1 of every edge at the given multipliers (no update). */
int orc_min_marginals(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                      const int64_t *rhs, const double *lam, double *m0, double *m1, int nthreads) {
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    set_threads(nthreads);
    int status = ORC_OK;
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * tab);
        double *Q = (double *)malloc(sizeof(double) * tab);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            if (st == ORC_OK) {
                prefix_table(&r, lam + b, P);
                suffix_table(&r, lam + b, Q);
                for (int l = 0; l < r.L; ++l) marginals(&r, P, Q, lam + b, l, m0 + b + l, m1 + b + l);
            } else {
#pragma omp critical
                status = st;
            }
        }
        free(P); free(Q);
    }
    return status;
}

/* Minimizing assignment of every row at lam (the supergradient of (D), Sec. "Loss"). */
int orc_argmin(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
               const int64_t *rhs, const double *lam, int8_t *x, double *gap, int nthreads) {
    /* gap (may be NULL): [2 m], per row the smallest relative and absolute gap (note_gap) */
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    set_threads(nthreads);
    int status = ORC_OK;
#pragma omp parallel
    {
        double *Q = (double *)malloc(sizeof(double) * tab);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            gap_t g = {INF, INF};
            if (st == ORC_OK) {
                suffix_table(&r, lam + b, Q);
                minimizer(&r, lam + b, NULL, Q, -1, 0, x + b, &g);
                if (gap) { gap[2 * j] = g.rel; gap[2 * j + 1] = g.abs; }
            } else {
#pragma omp critical
                status = st;
            }
        }
        free(Q);
    }
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* Alg. 2 (BlockUpdate backpropagation), applied block by block in reverse pass order.         */
/* Given the pass input (lam_in, M_in), its output lam_out and the adjoints of the outputs,    */
/* returns the adjoints of the inputs and accumulates d_alpha, d_omega.  For the block of hop  */
/* h the multipliers it saw are lam_out on hops visited before h and lam_in on the others.     */
/* The minimizers s^j(i, beta) are traced explicitly from the dynamic-programming tables.      */
/* ------------------------------------------------------------------------------------------ */
static int row_pass_vjp(const row_t *r, int dir, const double *omega, const double *alpha, const double *S,
                        const double *lam_in, const double *lam_out, const double *dlam_out, const double *dM_out,
                        double *dlam_in, double *gS, double *d_alpha, double *d_omega, double *P, double *Q,
                        double *lam_h, double *ad_new, int8_t *x0, int8_t *x1, gap_t *gap, taint_t *tt) {
    const int L = r->L;
    for (int p = 0; p < L; ++p) { ad_new[p] = dlam_out[p]; dlam_in[p] = 0.0; }
    if (tt)
        for (int p = 0; p < L; ++p) { tt->ad[p] = tt->dlo ? tt->dlo[p] : 0.0; tt->dli[p] = 0.0; }
    for (int h = L - 1; h >= 0; --h) {
        int l = dir == 0 ? h : L - 1 - h;
        /* position p was visited before hop h iff its pass order is < h */
        for (int p = 0; p < L; ++p) {
            int order = dir == 0 ? p : L - 1 - p;
            lam_h[p] = order < h ? lam_out[p] : lam_in[p];
        }
        double g = ad_new[l];          /* adjoint of lambda_l after its update (complete now) */
        dlam_in[l] += g;               /* lambda_new = lambda_old - M_new + ...: identity part */
        double Mt = dM_out[l] - g;     /* Alg. 2: dM_new <- dM_new - dlambda_new */
        d_alpha[l] += g * S[l];        /* Alg. 2: d_alpha += dlambda * sum_k M_ik */
        gS[l] = g * alpha[l];          /* this edge's share of d S_i = sum_k dlambda_ik alpha_ik */
        double eg = 0.0, eM = 0.0;     /* flip bounds of g and of Mt */
        if (tt) {
            eg = tt->ad[l];
            eM = eg + (tt->dmo ? tt->dmo[l] : 0.0);
            tt->dli[l] += eg;
            tt->gS[l] = eg * alpha[l];
            tt->dalpha[l] += eg * fabs(S[l]);
        }
        prefix_table(r, lam_h, P);
        suffix_table(r, lam_h, Q);
        double m0, m1;
        marginals(r, P, Q, lam_h, l, &m0, &m1);
        if (m0 == INF || m1 == INF) return ORC_E_FORCED;
        d_omega[l] += Mt * (m1 - m0);  /* dM_new * M_new / omega, written without the division */
        if (tt) {
            double sj = 0.0;
            for (int p = 0; p < L; ++p) sj += fabs(lam_h[p]);
            tt->domega[l] += eM * fabs(m1 - m0);
            tt->wscale[l] += fabs(Mt) * sj;
        }
        minimizer(r, lam_h, P, Q, l, 0, x0, gap);
        minimizer(r, lam_h, P, Q, l, 1, x1, gap);
        double k = omega[l] * Mt;
        for (int p = 0; p < L; ++p) {
            double d = k * (double)(x1[p] - x0[p]);
            if (d == 0.0) continue;
            int order = dir == 0 ? p : L - 1 - p;
            if (order < h) ad_new[p] += d;  /* the block saw the updated multiplier */
            else dlam_in[p] += d;           /* the block saw the pass input */
        }
        if (tt && (k != 0.0 || eM != 0.0)) {
            /* k = omega Mt moves by at most ek on every position it reaches; a flip of either
             * minimizer's value at p moves x1[p] - x0[p] by 1, and so the contribution by |k| + ek */
            const double ek = omega[l] * eM, ef = fabs(k) + ek;
            memset(tt->amb0, 0, (size_t)L);
            memset(tt->amb1, 0, (size_t)L);
            near_ties(r, lam_h, P, Q, l, 0, x0, tt->tol, tt->amb0, tt->alt);
            near_ties(r, lam_h, P, Q, l, 1, x1, tt->tol, tt->amb1, tt->alt);
            for (int p = 0; p < L; ++p) {
                double e = (x1[p] != x0[p] ? ek : 0.0) + (tt->amb0[p] + tt->amb1[p]) * ef;
                if (e == 0.0) continue;
                int order = dir == 0 ? p : L - 1 - p;
                if (order < h) tt->ad[p] += e;
                else tt->dli[p] += e;
            }
        }
    }
    return ORC_OK;
}

/* Alg. 2 over one pass of the given rows, with the deferred sums S supplied per edge (given S the
 * rows are independent, so a subset of rows can be differentiated on its own: the adjoints of the
 * other rows' outputs only reach these rows through dM_in).  lam_in: pass input; the pass is re-run
 * here to get lam_out.  Per edge: dlam_in (set); gS = dlambda_new * alpha, the edge's share of
 * dS_i = d M_in_ik (Alg. 2, first line), set; d_alpha, d_omega accumulated (+=).
 * row_gap (may be NULL): [2 m], per row the smallest relative and absolute gap of its decisions.
 * row_tol (may be NULL: no tracking): [m] decision tolerance per row; then t_dlo, t_dmo (may be NULL)
 * are flip bounds of the adjoints of the pass outputs per edge, and t_out [5 E] receives the flip
 * bounds of dlam_in, gS (set), d_alpha and d_omega (accumulated) -- see near_ties() -- and the
 * rounding scale of d_omega (accumulated, see taint_t). */
int orc_rows_pass_vjp(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                      const int64_t *rhs, const double *omega, const double *alpha, const double *S_edge, int dir,
                      const double *lam_in, const double *dlam_out, const double *dM_out, double *dlam_in,
                      double *gS, double *d_alpha, double *d_omega, double *row_gap, const double *row_tol,
                      const double *t_dlo, const double *t_dmo, double *t_out, int nthreads) {
    if (m < 0 || (dir != 0 && dir != 1)) return ORC_E_ARG;
    int64_t E = row_ptr[m];
    size_t nE = (size_t)(E > 0 ? E : 1);
    double *lam_out = (double *)malloc(sizeof(double) * nE);
    double *M_out = (double *)malloc(sizeof(double) * nE);
    memcpy(lam_out, lam_in, sizeof(double) * (size_t)E);
    int status = orc_rows_pass(m, row_ptr, col, coef, sense, rhs, omega, alpha, S_edge, dir, 0, lam_out, M_out,
                               nthreads);
    if (status) goto done;
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    int maxL = 0;
    for (int j = 0; j < m; ++j) if (row_ptr[j + 1] - row_ptr[j] > maxL) maxL = (int)(row_ptr[j + 1] - row_ptr[j]);
    set_threads(nthreads);
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * tab);
        double *Q = (double *)malloc(sizeof(double) * tab);
        double *lam_h = (double *)malloc(sizeof(double) * (size_t)(maxL + 1));
        double *ad_new = (double *)malloc(sizeof(double) * (size_t)(maxL + 1));
        int8_t *x0 = (int8_t *)malloc((size_t)(maxL + 1));
        int8_t *x1 = (int8_t *)malloc((size_t)(maxL + 1));
        int8_t *scr = (int8_t *)malloc(3 * (size_t)(maxL + 1));
        double *ad_t = (double *)malloc(sizeof(double) * (size_t)(maxL + 1));
#pragma omp for schedule(dynamic, 4)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            gap_t g = {INF, INF};
            taint_t tt;
            if (row_tol) {
                tt.tol = row_tol[j];
                tt.dlo = t_dlo ? t_dlo + b : NULL;
                tt.dmo = t_dmo ? t_dmo + b : NULL;
                tt.dli = t_out + b;
                tt.gS = t_out + E + b;
                tt.dalpha = t_out + 2 * E + b;
                tt.domega = t_out + 3 * E + b;
                tt.wscale = t_out + 4 * E + b;
                tt.ad = ad_t;
                tt.amb0 = scr;
                tt.amb1 = scr + maxL + 1;
                tt.alt = scr + 2 * (maxL + 1);
            }
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            if (st == ORC_OK)
                st = row_pass_vjp(&r, dir, omega + b, alpha + b, S_edge + b, lam_in + b, lam_out + b, dlam_out + b,
                                  dM_out + b, dlam_in + b, gS + b, d_alpha + b, d_omega + b, P, Q, lam_h, ad_new, x0,
                                  x1, &g, row_tol ? &tt : NULL);
            if (row_gap) { row_gap[2 * j] = g.rel; row_gap[2 * j + 1] = g.abs; }
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        free(P); free(Q); free(lam_h); free(ad_new); free(x0); free(x1); free(scr); free(ad_t);
    }
done:
    free(lam_out); free(M_out);
    return status;
}

/* VJP of one full pass: S from M_in, orc_rows_pass_vjp over every row, then
 * d M_in_ik = d S_i = sum_j dlambda_new_ij alpha_ij (Alg. 2, first line).
 * Outputs dlam_in[E], dM_in[E]; d_alpha[E], d_omega[E] are accumulated (+=); row_gap, row_tol, t_dlo,
 * t_dmo as there; t_out [5 E] receives the flip bounds of dlam_in and dM_in (set) and of d_alpha and
 * d_omega (accumulated) -- dM_in's is the sum of its variable's gS bounds -- and d_omega's rounding
 * scale (accumulated). */
int orc_pass_vjp(int n, int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                 const int64_t *rhs, const double *omega, const double *alpha, int dir, const double *lam_in,
                 const double *M_in, const double *dlam_out, const double *dM_out, double *dlam_in, double *dM_in,
                 double *d_alpha, double *d_omega, double *row_gap, const double *row_tol, const double *t_dlo,
                 const double *t_dmo, double *t_out, int nthreads) {
    int64_t E = row_ptr[m];
    size_t nE = (size_t)(E > 0 ? E : 1);
    double *Sv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *Se = (double *)malloc(sizeof(double) * nE);
    double *gS = (double *)calloc(nE, sizeof(double));
    deferred_sums(n, E, col, M_in, Sv, Se);
    int status = orc_rows_pass_vjp(m, row_ptr, col, coef, sense, rhs, omega, alpha, Se, dir, lam_in, dlam_out, dM_out,
                                   dlam_in, gS, d_alpha, d_omega, row_gap, row_tol, t_dlo, t_dmo, t_out, nthreads);
    if (status == ORC_OK) {
        memset(Sv, 0, sizeof(double) * (size_t)(n > 0 ? n : 1));
        for (int64_t e = 0; e < E; ++e) Sv[col[e]] += gS[e];
        for (int64_t e = 0; e < E; ++e) dM_in[e] = Sv[col[e]];
        if (row_tol) {  /* bound of dM_in: the bounds of the variable's shares, summed */
            memset(Sv, 0, sizeof(double) * (size_t)(n > 0 ? n : 1));
            for (int64_t e = 0; e < E; ++e) Sv[col[e]] += t_out[E + e];
            for (int64_t e = 0; e < E; ++e) t_out[E + e] = Sv[col[e]];
        }
    }
    free(Sv); free(Se); free(gS);
    return status;
}

/* Gradient of the final lower bound after T iterations with respect to omega, alpha and c (or the
 * start state): T iterations from (lam0, M0) -- or, when lam0 is NULL, from lambda = c/|J_i|, M = 0 --
 * keeping every pass's state, then the seed dLB/dlambda_bar = argmin assignment (Sec. "Loss"), the
 * flush lambda_bar = lambda + alpha S, orc_pass_vjp on every pass in reverse, and finally
 * lambda_0 = c / |J_i|.  d_c (reset start only; may be NULL) is the gradient through lambda_0 and the
 * uncovered-variable constant: variables in no row contribute min(0, c_i) to LB, so dLB/dc_i = [c_i < 0]
 * for them.  d_lam0 / d_M0 (may be NULL) are the adjoints of the start state.
 * row_gap (may be NULL): [2 m], per row the smallest relative and absolute gap (note_gap) of any
 * decision taken on the way (the seed and every pass).
 * pass_tol (may be NULL: no tracking): [(2T + 1) m], the decision tolerance of every row in pass
 * p = 0 .. 2T-1 (at p m) and in the seed (at 2T m); then taint [5 E + n] receives the flip bounds
 * (near_ties()) of d_omega, d_alpha, d_lam0 and d_M0, the rounding scale of d_omega summed over the
 * passes (taint_t), and the flip bounds of d_c. */
static int seed_taint(int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                      const int64_t *rhs, const double *lam, const int8_t *x, const double *row_tol, int8_t *amb,
                      int nthreads) {
    size_t tab;
    max_table(m, row_ptr, coef, &tab);
    int maxL = 0;
    for (int j = 0; j < m; ++j) if (row_ptr[j + 1] - row_ptr[j] > maxL) maxL = (int)(row_ptr[j + 1] - row_ptr[j]);
    set_threads(nthreads);
    int status = ORC_OK;
#pragma omp parallel
    {
        double *Q = (double *)malloc(sizeof(double) * tab);
        int8_t *alt = (int8_t *)malloc((size_t)(maxL + 1));
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < m; ++j) {
            row_t r;
            int64_t b = row_ptr[j];
            int st = row_init(&r, (int)(row_ptr[j + 1] - b), col + b, coef + b, sense[j], rhs[j]);
            if (st == ORC_OK) {
                memset(amb + b, 0, (size_t)r.L);
                suffix_table(&r, lam + b, Q);
                near_ties(&r, lam + b, NULL, Q, -1, 0, x + b, row_tol[j], amb + b, alt);
            } else {
#pragma omp critical
                status = st;
            }
        }
        free(Q); free(alt);
    }
    return status;
}

int orc_unrolled_grad(int n, int m, const int64_t *row_ptr, const int32_t *col, const int32_t *coef,
                      const int8_t *sense, const int64_t *rhs, const double *c, const double *omega,
                      const double *alpha, int T, const double *lam0, const double *M0, double *lb_out,
                      double *d_omega, double *d_alpha, double *d_c, double *d_lam0, double *d_M0,
                      double *row_gap, const double *pass_tol, double *taint, int nthreads) {
    int64_t E = row_ptr[m];
    size_t nE = (size_t)(E > 0 ? E : 1);
    int npass = 2 * T;
    double *lam = (double *)malloc(sizeof(double) * nE * (size_t)(npass + 1));
    double *M = (double *)calloc(nE * (size_t)(npass + 1), sizeof(double));
    double *lam_bar = (double *)malloc(sizeof(double) * nE);
    double *dl = (double *)malloc(sizeof(double) * nE);
    double *dM = (double *)malloc(sizeof(double) * nE);
    double *dl2 = (double *)malloc(sizeof(double) * nE);
    double *dM2 = (double *)malloc(sizeof(double) * nE);
    double *Sv = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *Se = (double *)malloc(sizeof(double) * nE);
    int8_t *x = (int8_t *)malloc(nE);
    int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    double *gaps = (double *)malloc(sizeof(double) * 2 * (size_t)(m > 0 ? m : 1));
    /* flip bounds: t_dl, t_dM, the pass outputs [4 E] (dl, dM, alpha, omega), per variable [n] */
    double *t_dl = NULL, *t_dM = NULL, *t_pass = NULL, *t_var = NULL, *t_alpha = NULL, *t_omega = NULL;
    int8_t *amb = NULL;
    if (pass_tol) {
        t_dl = (double *)calloc(nE, sizeof(double));
        t_dM = (double *)calloc(nE, sizeof(double));
        t_pass = (double *)calloc(5 * nE, sizeof(double));
        t_var = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
        amb = (int8_t *)calloc(nE, 1);
        t_alpha = taint + E;
        t_omega = taint;
        for (size_t q = 0; q < 5 * (size_t)E + (size_t)n; ++q) taint[q] = 0.0;
    }
    for (int j = 0; j < 2 * m && row_gap; ++j) row_gap[j] = INF;
    int st = ORC_OK;
    if (lam0) {
        memcpy(lam, lam0, sizeof(double) * (size_t)E);
        memcpy(M, M0, sizeof(double) * (size_t)E);
    } else {
        st = orc_init_lambda(n, c, E, col, lam);
    }
    for (int p = 0; p < npass && st == ORC_OK; ++p) {
        memcpy(lam + nE * (p + 1), lam + nE * p, sizeof(double) * (size_t)E);
        memcpy(M + nE * (p + 1), M + nE * p, sizeof(double) * (size_t)E);
        st = orc_pass(n, m, row_ptr, col, coef, sense, rhs, omega, alpha, p % 2, 0, lam + nE * (p + 1),
                      M + nE * (p + 1), nthreads);
    }
    if (st) goto done;
    double dlv;
    st = orc_lower_bound(n, m, row_ptr, col, coef, sense, rhs, c, alpha, lam + nE * npass, M + nE * npass, lb_out,
                         &dlv, lam_bar, nthreads);
    if (st) goto done;
    st = orc_argmin(m, row_ptr, col, coef, sense, rhs, lam_bar, x, gaps, nthreads);
    if (st) goto done;
    for (int j = 0; j < 2 * m && row_gap; ++j) row_gap[j] = fmin(row_gap[j], gaps[j]);
    for (int64_t e = 0; e < E; ++e) { d_alpha[e] = 0.0; d_omega[e] = 0.0; }
    /* flush adjoint: lambda_bar_e = lambda_e + alpha_e S_i */
    deferred_sums(n, E, col, M + nE * npass, Sv, Se);
    memset(Sv, 0, sizeof(double) * (size_t)n);
    for (int64_t e = 0; e < E; ++e) {
        dl[e] = (double)x[e];
        d_alpha[e] += (double)x[e] * Se[e];
        Sv[col[e]] += (double)x[e] * alpha[e];
    }
    for (int64_t e = 0; e < E; ++e) dM[e] = Sv[col[e]];
    if (pass_tol) {  /* the seed: a near-tie of the argmin can flip x_e, which moves its terms by 1 * factor */
        st = seed_taint(m, row_ptr, col, coef, sense, rhs, lam_bar, x, pass_tol + (size_t)npass * m, amb, nthreads);
        if (st) goto done;
        for (int64_t e = 0; e < E; ++e) {
            t_dl[e] = amb[e];
            t_alpha[e] += amb[e] * fabs(Se[e]);
            t_var[col[e]] += amb[e] * alpha[e];
        }
        for (int64_t e = 0; e < E; ++e) t_dM[e] = t_var[col[e]];
    }
    for (int p = npass - 1; p >= 0 && st == ORC_OK; --p) {
        if (pass_tol) memset(t_pass, 0, 5 * nE * sizeof(double));
        st = orc_pass_vjp(n, m, row_ptr, col, coef, sense, rhs, omega, alpha, p % 2, lam + nE * p, M + nE * p, dl, dM,
                          dl2, dM2, d_alpha, d_omega, gaps, pass_tol ? pass_tol + (size_t)p * m : NULL, t_dl, t_dM,
                          t_pass, nthreads);
        for (int j = 0; j < 2 * m && row_gap; ++j) row_gap[j] = fmin(row_gap[j], gaps[j]);
        if (pass_tol) {
            memcpy(t_dl, t_pass, sizeof(double) * (size_t)E);
            memcpy(t_dM, t_pass + E, sizeof(double) * (size_t)E);
            for (int64_t e = 0; e < E; ++e) {
                t_alpha[e] += t_pass[2 * E + e];
                t_omega[e] += t_pass[3 * E + e];
                taint[4 * E + e] += t_pass[4 * E + e];
            }
        }
        double *t;
        t = dl; dl = dl2; dl2 = t;
        t = dM; dM = dM2; dM2 = t;
    }
    if (st) goto done;
    if (pass_tol) {
        memcpy(taint + 2 * E, t_dl, sizeof(double) * (size_t)E);
        memcpy(taint + 3 * E, t_dM, sizeof(double) * (size_t)E);
        double *tc = taint + 5 * E;
        for (int64_t e = 0; e < E; ++e) deg[col[e]]++;
        for (int64_t e = 0; e < E; ++e) tc[col[e]] += t_dl[e] / (double)deg[col[e]];
        for (int64_t e = 0; e < E; ++e) deg[col[e]] = 0;
    }
    if (d_lam0) memcpy(d_lam0, dl, sizeof(double) * (size_t)E);
    if (d_M0) memcpy(d_M0, dM, sizeof(double) * (size_t)E);
    if (d_c) {
        for (int64_t e = 0; e < E; ++e) deg[col[e]]++;
        for (int i = 0; i < n; ++i) d_c[i] = deg[i] == 0 ? (c[i] < 0.0 ? 1.0 : 0.0) : 0.0;
        for (int64_t e = 0; e < E; ++e) d_c[col[e]] += dl[e] / (double)deg[col[e]];
    }
done:
    free(lam); free(M); free(lam_bar); free(dl); free(dM); free(dl2); free(dM2); free(Sv); free(Se); free(x);
    free(deg); free(gaps); free(t_dl); free(t_dM); free(t_pass); free(t_var); free(amb);
    return st;
}

/* Threads the parallel loops above will use. */
int orc_threads(int nthreads) {
    set_threads(nthreads);
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
