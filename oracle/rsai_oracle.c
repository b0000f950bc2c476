/*
 * CPU FP64 oracle for RSAI(tol) -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct restatement of the residual-based sparse
 * approximate inverse procedure of Jia & Kang (arXiv:1503.04500):
 *   - the column split of min ||AM - I||_F into n LS problems, eqs. (2.1)-(2.3);
 *   - the basic RSAI loop, Algorithm 1 (Section 3);
 *   - the dropping of small entries during the loops, Section 4 (fixed tol, or the
 *     adaptive tolerance of eq. (4.3));
 *   - the fixed-pattern adjoint used for gradients of losses of M w.r.t. the
 *     values of A (follows from the normal equations of (2.3));
 *   - right-preconditioned BiCGStab as used in Section 5 (textbook form).
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load this
 * library. It shares no code, header, table or helper with the GPU path.
 *
 * Conventions where the paper is silent (each stated once here):
 *   - |r(i)| ties in the dominant-index choice go to the smaller global row index;
 *     L_k = { i : r(i) != 0 } uses an exact-zero test.
 *   - R_k (the union of earlier dominant sets, eq. (3.2)) is always excluded, as
 *     Algorithm 1 does, and it is never reset.
 *   - An empty J-hat consumes a loop without a solve (Algorithm 1, step 6).
 *   - If no candidate row is left the loop stops (possible only when m_k is exact,
 *     Section 3).
 *   - Dropping runs after every LS solve (including the initial one): entries with
 *     |m_j| <= t leave J, t = tol or eps/(|J| * ||A||_1) (eq. (4.3)); if anything was
 *     dropped the LS is solved again on the kept pattern (one pass). J never
 *     becomes empty: if every entry is small, the largest (smaller index on ties)
 *     is kept. I never shrinks.
 *
 * LS solves are done from scratch every time (dense Householder QR of A(I,J)
 * with I and J sorted ascending); no incremental updating, no blocking.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_DROP_NONE 0
#define OR_DROP_FIXED 1
#define OR_DROP_ADAPTIVE 2

#define OR_OK 0
#define OR_ERR_SINGULAR 3

typedef struct {
    int64_t n;
    const int64_t *colptr;
    const int32_t *rowidx;
    const double *val;
    int64_t *rowptr; /* row pattern (transpose), built here */
    int32_t *colidx;
    double norm1; /* max column absolute sum, ||A||_1 */
} omat;

/* ---------------- small growable arrays ---------------- */
typedef struct { int32_t *a; int n, cap; } ivec;
typedef struct { double *a; int n, cap; } dvec;

static void iv_reserve(ivec *v, int cap) {
    if (cap > v->cap) {
        int c = v->cap ? v->cap : 16;
        while (c < cap) c *= 2;
        v->a = (int32_t *)realloc(v->a, sizeof(int32_t) * (size_t)c);
        v->cap = c;
    }
}
static void dv_reserve(dvec *v, int cap) {
    if (cap > v->cap) {
        int c = v->cap ? v->cap : 16;
        while (c < cap) c *= 2;
        v->a = (double *)realloc(v->a, sizeof(double) * (size_t)c);
        v->cap = c;
    }
}
static void iv_push(ivec *v, int32_t x) { iv_reserve(v, v->n + 1); v->a[v->n++] = x; }

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}
/* sort ascending and remove duplicates */
static void iv_sort_unique(ivec *v) {
    if (v->n <= 1) return;
    qsort(v->a, (size_t)v->n, sizeof(int32_t), cmp_i32);
    int w = 1;
    for (int i = 1; i < v->n; ++i)
        if (v->a[i] != v->a[w - 1]) v->a[w++] = v->a[i];
    v->n = w;
}
/* binary search in a sorted array; -1 if absent */
static int find_sorted(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (a[mid] == x) return mid;
        if (a[mid] < x) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}
static int contains_linear(const int32_t *a, int n, int32_t x) {
    for (int i = 0; i < n; ++i) if (a[i] == x) return 1;
    return 0;
}
/* out = a minus b (both sorted unique), result sorted */
static void set_minus(const ivec *a, const ivec *b, ivec *out) {
    out->n = 0;
    iv_reserve(out, a->n);
    for (int i = 0; i < a->n; ++i)
        if (find_sorted(b->a, b->n, a->a[i]) < 0) out->a[out->n++] = a->a[i];
}
/* a = a union b (both sorted unique) */
static void set_union_into(ivec *a, const ivec *b, ivec *tmp) {
    tmp->n = 0;
    iv_reserve(tmp, a->n + b->n);
    int i = 0, j = 0;
    while (i < a->n || j < b->n) {
        if (j >= b->n || (i < a->n && a->a[i] < b->a[j])) tmp->a[tmp->n++] = a->a[i++];
        else if (i >= a->n || b->a[j] < a->a[i]) tmp->a[tmp->n++] = b->a[j++];
        else { tmp->a[tmp->n++] = a->a[i]; ++i; ++j; }
    }
    iv_reserve(a, tmp->n);
    memcpy(a->a, tmp->a, sizeof(int32_t) * (size_t)tmp->n);
    a->n = tmp->n;
}

/* ---------------- matrix preprocessing ---------------- */
static int build_row_pattern(omat *A) {
    int64_t n = A->n, nnz = A->colptr[n];
    A->rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    A->colidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!A->rowptr || !A->colidx) return -1;
    for (int64_t e = 0; e < nnz; ++e) A->rowptr[A->rowidx[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) A->rowptr[i + 1] += A->rowptr[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(fill, A->rowptr, sizeof(int64_t) * (size_t)n);
    /* columns visited in ascending order, so each row's list is ascending */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t e = A->colptr[j]; e < A->colptr[j + 1]; ++e)
            A->colidx[fill[A->rowidx[e]]++] = (int32_t)j;
    free(fill);
    double best = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t e = A->colptr[j]; e < A->colptr[j + 1]; ++e) s += fabs(A->val[e]);
        if (s > best) best = s;
    }
    A->norm1 = best;
    return 0;
}

/* ---------------- per-thread workspace ---------------- */
typedef struct {
    ivec I, J, Rset, Jhat, Ihat, cand, tmp, keep;
    dvec B, B0, y, v, mt, r;
} work;

static void work_free(work *w) {
    free(w->I.a); free(w->J.a); free(w->Rset.a); free(w->Jhat.a); free(w->Ihat.a);
    free(w->cand.a); free(w->tmp.a); free(w->keep.a);
    free(w->B.a); free(w->B0.a); free(w->y.a); free(w->v.a); free(w->mt.a); free(w->r.a);
}

/*
 * LS solve of eq. (2.3): min || A(I,J) m - e_k(I) ||_2 with I, J sorted ascending.
 * Dense B = A(I,J) (column-major), Householder QR B = Q [R; 0], m = R^{-1} (Q^T e)(0:q),
 * residual r = B m - e_k(I) over I. Returns ||A m_k - e_k||_2 through *resnorm, which
 * includes r(k) = -1 when k is not in I (eq. (2.4): the residual of (2.2) equals that
 * of (2.3) on I, plus the entry at row k if row k is outside I).
 * Algorithmic flop count of the solve is added to *flops.
 */
static int ls_solve(const omat *A, int32_t k, work *w, double *resnorm, double *flops) {
    const int m = w->I.n, q = w->J.n;
    if (q == 0) return OR_ERR_SINGULAR;
    if (m < q) return OR_ERR_SINGULAR;
    dv_reserve(&w->B, m * q);
    dv_reserve(&w->B0, m * q);
    dv_reserve(&w->y, m);
    dv_reserve(&w->v, m);
    dv_reserve(&w->mt, q);
    dv_reserve(&w->r, m);
    double *B = w->B.a, *B0 = w->B0.a, *y = w->y.a, *v = w->v.a, *mt = w->mt.a, *r = w->r.a;
    memset(B, 0, sizeof(double) * (size_t)m * (size_t)q);
    int64_t nzB = 0;
    for (int jj = 0; jj < q; ++jj) {
        int32_t j = w->J.a[jj];
        for (int64_t e = A->colptr[j]; e < A->colptr[j + 1]; ++e) {
            int ii = find_sorted(w->I.a, m, A->rowidx[e]);
            if (ii >= 0) { B[ii + (size_t)m * jj] = A->val[e]; ++nzB; }
        }
    }
    memcpy(B0, B, sizeof(double) * (size_t)m * (size_t)q);
    for (int ii = 0; ii < m; ++ii) y[ii] = (w->I.a[ii] == k) ? 1.0 : 0.0;

    /* Householder QR, column by column; R overwrites the upper triangle of B */
    for (int j = 0; j < q; ++j) {
        double nx = 0.0;
        for (int i = j; i < m; ++i) nx += B[i + (size_t)m * j] * B[i + (size_t)m * j];
        nx = sqrt(nx);
        if (nx == 0.0) return OR_ERR_SINGULAR;
        double x0 = B[j + (size_t)m * j];
        double alpha = (x0 >= 0.0) ? -nx : nx;
        for (int i = j; i < m; ++i) v[i] = B[i + (size_t)m * j];
        v[j] = x0 - alpha;
        double vtv = 0.0;
        for (int i = j; i < m; ++i) vtv += v[i] * v[i];
        /* apply H = I - 2 v v^T / (v^T v) to trailing columns and to y */
        for (int c = j + 1; c < q; ++c) {
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * B[i + (size_t)m * c];
            double f = 2.0 * s / vtv;
            for (int i = j; i < m; ++i) B[i + (size_t)m * c] -= f * v[i];
        }
        double s = 0.0;
        for (int i = j; i < m; ++i) s += v[i] * y[i];
        double f = 2.0 * s / vtv;
        for (int i = j; i < m; ++i) y[i] -= f * v[i];
        B[j + (size_t)m * j] = alpha;
    }
    /* back substitution R m = (Q^T e)(0:q) */
    for (int j = q - 1; j >= 0; --j) {
        double s = y[j];
        for (int c = j + 1; c < q; ++c) s -= B[j + (size_t)m * c] * mt[c];
        double d = B[j + (size_t)m * j];
        if (d == 0.0) return OR_ERR_SINGULAR;
        mt[j] = s / d;
    }
    /* residual from the original block */
    double rr = 0.0;
    int kin = 0;
    for (int ii = 0; ii < m; ++ii) {
        double s = 0.0;
        for (int jj = 0; jj < q; ++jj) s += B0[ii + (size_t)m * jj] * mt[jj];
        s -= (w->I.a[ii] == k) ? 1.0 : 0.0;
        if (w->I.a[ii] == k) kin = 1;
        r[ii] = s;
        rr += s * s;
    }
    if (!kin) rr += 1.0;
    *resnorm = sqrt(rr);
    /* flops: full QR + Q^T e + back-solve + residual */
    double md = m, qd = q;
    *flops += 2.0 * md * qd * qd - (2.0 / 3.0) * qd * qd * qd + 4.0 * md * qd - 2.0 * qd * qd + qd * qd +
              2.0 * (double)nzB;
    return OR_OK;
}

typedef struct {
    int32_t c, lmax, drop;
    double eps, tol;
} oparams;

/*
 * Flop count of one LS solve done as a Householder QR *update* (Algorithm 1, step 7,
 * with the column/row append of (3.1)): the factor of the first qlo columns was made
 * on m0 rows and is kept; the augmented block has m rows and qn columns. The rows
 * added since (I-hat) are zero in the old columns, so each stored reflector j < qlo
 * acts on rows j..m0-1 of the qn - qlo new columns only (a dot product and an update,
 * 4 (m0 - j) flops per column). Reflectors qlo..qn-1 are then formed on rows j..m-1
 * (norm 2 (m - j)) and applied to the qn - j - 1 later columns and to Q^T e
 * (4 (m - j) each); back substitution costs qn^2 and the residual norm
 * ||(Q^T e)(qn:m)|| 2 (m - qn). qlo = 0 is a from-scratch QR (m0 unused). This is
 * the algorithmic work model of the method, not the oracle's own from-scratch
 * arithmetic.
 */
static double model_solve_flops(int m0, int m, int qlo, int qn) {
    double f = 0.0;
    for (int j = 0; j < qlo; ++j) f += 4.0 * (double)(m0 - j) * (double)(qn - qlo);
    for (int j = qlo; j < qn; ++j)
        f += 2.0 * (double)(m - j) + 4.0 * (double)(m - j) * (double)(qn - j - 1) + 4.0 * (double)(m - j);
    f += (double)qn * (double)qn + 2.0 * (double)(m - qn);
    return f;
}

/* Dropping (Section 4): entries |m_j| <= t leave J; LS solved again if anything left. */
static int drop_step(const omat *A, int32_t k, const oparams *p, work *w, double *resnorm,
                     double *flops, double *drop_margin, int *ndrop, double *mflops) {
    if (p->drop == OR_DROP_NONE) return OR_OK;
    const int q = w->J.n;
    double t = (p->drop == OR_DROP_FIXED) ? p->tol : p->eps / ((double)q * A->norm1);
    w->keep.n = 0;
    iv_reserve(&w->keep, q);
    int best = 0;
    for (int jj = 0; jj < q; ++jj) {
        double a = fabs(w->mt.a[jj]);
        double gap = fabs(a - t);
        if (gap < *drop_margin) *drop_margin = gap;
        if (a > t) w->keep.a[w->keep.n++] = w->J.a[jj];
        if (a > fabs(w->mt.a[best])) best = jj; /* J ascending: first max = smaller index */
    }
    if (w->keep.n == q) return OR_OK;
    if (w->keep.n == 0) { w->keep.a[0] = w->J.a[best]; w->keep.n = 1; }
    memcpy(w->J.a, w->keep.a, sizeof(int32_t) * (size_t)w->keep.n);
    w->J.n = w->keep.n;
    *ndrop += 1;
    *mflops += model_solve_flops(0, w->I.n, 0, w->J.n);
    return ls_solve(A, k, w, resnorm, flops);
}

typedef struct {
    int32_t loops, nI, nJ, status, nsolve, ndrop;
    int32_t nImax, nJmax; /* largest |I|, |J| of any solve of the column (before dropping) */
    double resnorm, sel_margin, drop_margin, flops, mflops;
} colstat;

/*
 * One column of Algorithm 1 with dropping. On return w->J (ascending) and w->mt hold
 * the pattern and values of m_k. hist (nullable, length 2*(lmax+1)) receives the
 * residual norm after every solve.
 */
static void rsai_column(const omat *A, int32_t k, const oparams *p, work *w, colstat *st,
                        double *hist, int hist_len) {
    double rn = 0.0, flops = 0.0, sel_margin = INFINITY, drop_margin = INFINITY, mflops = 0.0;
    int nsolve = 0, ndrop = 0;
    int status = OR_OK;
    /* step 1: J^(0) = {k}, R^(0) empty, l = 0 */
    w->J.n = 0; iv_push(&w->J, k);
    w->Rset.n = 0;
    /* step 2: I^(0) = nonzero rows of A(:, J^(0)) */
    w->I.n = 0;
    for (int64_t e = A->colptr[k]; e < A->colptr[k + 1]; ++e) iv_push(&w->I, A->rowidx[e]);
    int l = 0;
    int32_t nImax = w->I.n, nJmax = w->J.n;
    status = ls_solve(A, k, w, &rn, &flops);
    mflops += model_solve_flops(0, w->I.n, 0, 1);
    if (status == OR_OK) status = drop_step(A, k, p, w, &rn, &flops, &drop_margin, &ndrop, &mflops);
    if (hist && nsolve < hist_len) hist[nsolve] = rn;
    ++nsolve;
    /* step 3 */
    while (status == OR_OK && rn > p->eps && l < p->lmax) {
        /* step 4: candidates are rows with r(i) != 0 not in R; pick the c largest |r(i)| */
        const int m = w->I.n;
        int kin = find_sorted(w->I.a, m, k) >= 0;
        w->cand.n = 0;
        for (int ii = 0; ii < m; ++ii)
            if (w->r.a[ii] != 0.0 && !contains_linear(w->Rset.a, w->Rset.n, w->I.a[ii]))
                iv_push(&w->cand, ii);
        int kcand = (!kin && !contains_linear(w->Rset.a, w->Rset.n, k)); /* r(k) = -1 */
        int ncand = w->cand.n + kcand;
        if (ncand == 0) break;
        int take = ncand < p->c ? ncand : p->c;
        /* selection by repeated max: key (|r| desc, global index asc) */
        int32_t chosen[64];
        double chosen_abs[64];
        int nchosen = 0;
        for (int t = 0; t < take; ++t) {
            double bestv = -1.0;
            int32_t bestg = -1;
            for (int u = 0; u < w->cand.n; ++u) {
                int ii = w->cand.a[u];
                if (ii < 0) continue;
                double a = fabs(w->r.a[ii]);
                int32_t g = w->I.a[ii];
                if (a > bestv || (a == bestv && g < bestg)) { bestv = a; bestg = g; }
            }
            if (kcand) {
                if (1.0 > bestv || (1.0 == bestv && k < bestg)) { bestv = 1.0; bestg = k; }
            }
            chosen[nchosen] = bestg;
            chosen_abs[nchosen] = bestv;
            ++nchosen;
            if (kcand && bestg == k) kcand = 0;
            else
                for (int u = 0; u < w->cand.n; ++u)
                    if (w->cand.a[u] >= 0 && w->I.a[w->cand.a[u]] == bestg) { w->cand.a[u] = -1; break; }
        }
        /* decision margin: last chosen vs best rejected */
        {
            double rej = -1.0;
            for (int u = 0; u < w->cand.n; ++u)
                if (w->cand.a[u] >= 0) { double a = fabs(w->r.a[w->cand.a[u]]); if (a > rej) rej = a; }
            if (kcand && 1.0 > rej) rej = 1.0;
            if (rej >= 0.0) {
                double gap = chosen_abs[nchosen - 1] - rej;
                if (gap < sel_margin) sel_margin = gap;
            }
        }
        for (int t = 0; t < nchosen; ++t) iv_push(&w->Rset, chosen[t]);
        /* step 5: J-hat = columns of A(R-hat, :) not in J */
        w->tmp.n = 0;
        for (int t = 0; t < nchosen; ++t) {
            int32_t i = chosen[t];
            for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) iv_push(&w->tmp, A->colidx[e]);
        }
        iv_sort_unique(&w->tmp);
        set_minus(&w->tmp, &w->J, &w->Jhat);
        /* step 6 */
        ++l;
        if (w->Jhat.n == 0) continue;
        /* I-hat = rows of A(:, J-hat) not in I */
        w->tmp.n = 0;
        for (int t = 0; t < w->Jhat.n; ++t) {
            int32_t j = w->Jhat.a[t];
            for (int64_t e = A->colptr[j]; e < A->colptr[j + 1]; ++e) iv_push(&w->tmp, A->rowidx[e]);
        }
        iv_sort_unique(&w->tmp);
        set_minus(&w->tmp, &w->I, &w->Ihat);
        int qprev = w->J.n, mprev = w->I.n;
        {
            ivec scratch = {0, 0, 0};
            set_union_into(&w->J, &w->Jhat, &scratch);
            set_union_into(&w->I, &w->Ihat, &scratch);
            free(scratch.a);
        }
        if (w->I.n > nImax) nImax = w->I.n;
        if (w->J.n > nJmax) nJmax = w->J.n;
        /* step 7: new LS solution and residual on the augmented pattern */
        status = ls_solve(A, k, w, &rn, &flops);
        mflops += model_solve_flops(mprev, w->I.n, qprev, w->J.n);
        if (status == OR_OK) status = drop_step(A, k, p, w, &rn, &flops, &drop_margin, &ndrop, &mflops);
        if (hist && nsolve < hist_len) hist[nsolve] = rn;
        ++nsolve;
    }
    st->loops = l;
    st->nI = w->I.n;
    st->nJ = w->J.n;
    st->status = status;
    st->resnorm = rn;
    st->sel_margin = sel_margin;
    st->drop_margin = drop_margin;
    st->flops = flops;
    st->nsolve = nsolve;
    st->ndrop = ndrop;
    st->mflops = mflops;
    st->nImax = nImax;
    st->nJmax = nJmax;
}

/* ---------------- result handle ---------------- */
typedef struct {
    int64_t n, ncols, nnz;
    int64_t *cols; /* the columns processed, ascending */
    int64_t *colptr;
    int32_t *rowidx;
    double *val;
    colstat *st;
    double *hist;
    int hist_len;
    double seconds;
    int threads;
} oresult;

static double now_seconds(void) {
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

/*
 * Run RSAI(tol) on the columns listed in cols (NULL = all n columns).
 * Returns an opaque handle (NULL on allocation failure).
 */
void *oracle_rsai(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                  int32_t c, int32_t lmax, double eps, int32_t drop, double tol, int32_t nthreads,
                  const int64_t *cols, int64_t ncols, int32_t record_hist) {
    omat A = {n, colptr, rowidx, val, NULL, NULL, 0.0};
    if (build_row_pattern(&A) != 0) return NULL;
    oparams p = {c, lmax, drop, eps, tol};
    oresult *R = (oresult *)calloc(1, sizeof(oresult));
    R->n = n;
    R->ncols = cols ? ncols : n;
    R->cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->ncols > 0 ? R->ncols : 1));
    for (int64_t t = 0; t < R->ncols; ++t) R->cols[t] = cols ? cols[t] : t;
    R->st = (colstat *)calloc((size_t)(R->ncols > 0 ? R->ncols : 1), sizeof(colstat));
    R->hist_len = record_hist ? 2 * (lmax + 1) : 0;
    if (record_hist) {
        R->hist = (double *)malloc(sizeof(double) * (size_t)R->ncols * (size_t)R->hist_len + 8);
        for (int64_t t = 0; t < R->ncols * R->hist_len; ++t) R->hist[t] = NAN;
    }
    int32_t **Jout = (int32_t **)calloc((size_t)(R->ncols > 0 ? R->ncols : 1), sizeof(int32_t *));
    double **Vout = (double **)calloc((size_t)(R->ncols > 0 ? R->ncols : 1), sizeof(double *));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double t0 = now_seconds();
    int used_threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used_threads = omp_get_num_threads();
#endif
        work w;
        memset(&w, 0, sizeof(w));
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < R->ncols; ++t) {
            int32_t k = (int32_t)R->cols[t];
            rsai_column(&A, k, &p, &w, &R->st[t], R->hist ? R->hist + t * R->hist_len : NULL, R->hist_len);
            int q = w.J.n;
            Jout[t] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(q > 0 ? q : 1));
            Vout[t] = (double *)malloc(sizeof(double) * (size_t)(q > 0 ? q : 1));
            if (R->st[t].status == OR_OK) {
                memcpy(Jout[t], w.J.a, sizeof(int32_t) * (size_t)q); /* already ascending */
                memcpy(Vout[t], w.mt.a, sizeof(double) * (size_t)q);
            } else {
                R->st[t].nJ = 0;
            }
        }
        work_free(&w);
    }
    R->seconds = now_seconds() - t0;
    R->threads = used_threads;
    R->colptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R->ncols + 1));
    R->colptr[0] = 0;
    for (int64_t t = 0; t < R->ncols; ++t) R->colptr[t + 1] = R->colptr[t] + R->st[t].nJ;
    R->nnz = R->colptr[R->ncols];
    R->rowidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R->nnz > 0 ? R->nnz : 1));
    R->val = (double *)malloc(sizeof(double) * (size_t)(R->nnz > 0 ? R->nnz : 1));
    for (int64_t t = 0; t < R->ncols; ++t) {
        memcpy(R->rowidx + R->colptr[t], Jout[t], sizeof(int32_t) * (size_t)R->st[t].nJ);
        memcpy(R->val + R->colptr[t], Vout[t], sizeof(double) * (size_t)R->st[t].nJ);
        free(Jout[t]);
        free(Vout[t]);
    }
    free(Jout);
    free(Vout);
    free(A.rowptr);
    free(A.colidx);
    return R;
}

/* The QR-update work model of one LS solve (see model_solve_flops), for tests. */
double oracle_model_solve_flops(int32_t m0, int32_t m, int32_t qlo, int32_t qn) {
    return model_solve_flops(m0, m, qlo, qn);
}

int64_t oracle_nnz(void *h) { return ((oresult *)h)->nnz; }
double oracle_seconds(void *h) { return ((oresult *)h)->seconds; }
int32_t oracle_threads(void *h) { return ((oresult *)h)->threads; }

/* Copy results out; any pointer may be NULL. Arrays are per processed column. */
void oracle_export(void *h, int64_t *colptr, int32_t *rowidx, double *val, int32_t *loops,
                   double *resnorm, int32_t *nI, int32_t *nJ, int32_t *status, double *sel_margin,
                   double *drop_margin, double *flops, int32_t *nsolve, double *hist, int32_t *ndrop,
                   double *mflops) {
    oresult *R = (oresult *)h;
    if (colptr) memcpy(colptr, R->colptr, sizeof(int64_t) * (size_t)(R->ncols + 1));
    if (rowidx) memcpy(rowidx, R->rowidx, sizeof(int32_t) * (size_t)R->nnz);
    if (val) memcpy(val, R->val, sizeof(double) * (size_t)R->nnz);
    for (int64_t t = 0; t < R->ncols; ++t) {
        if (loops) loops[t] = R->st[t].loops;
        if (resnorm) resnorm[t] = R->st[t].resnorm;
        if (nI) nI[t] = R->st[t].nI;
        if (nJ) nJ[t] = R->st[t].nJ;
        if (status) status[t] = R->st[t].status;
        if (sel_margin) sel_margin[t] = R->st[t].sel_margin;
        if (drop_margin) drop_margin[t] = R->st[t].drop_margin;
        if (flops) flops[t] = R->st[t].flops;
        if (nsolve) nsolve[t] = R->st[t].nsolve;
        if (ndrop) ndrop[t] = R->st[t].ndrop;
        if (mflops) mflops[t] = R->st[t].mflops;
    }
    if (hist && R->hist) memcpy(hist, R->hist, sizeof(double) * (size_t)R->ncols * (size_t)R->hist_len);
}

/* Largest |I_k| and |J_k| over the solves of each column (either may be NULL). */
void oracle_export_peaks(void *h, int32_t *nImax, int32_t *nJmax) {
    oresult *R = (oresult *)h;
    for (int64_t t = 0; t < R->ncols; ++t) {
        if (nImax) nImax[t] = R->st[t].nImax;
        if (nJmax) nJmax[t] = R->st[t].nJmax;
    }
}

void oracle_free(void *h) {
    oresult *R = (oresult *)h;
    if (!R) return;
    free(R->cols); free(R->colptr); free(R->rowidx); free(R->val); free(R->st); free(R->hist);
    free(R);
}

/* ====================================================================== */
/*  Fixed-pattern solve and adjoint (gradients w.r.t. the values of A)     */
/* ====================================================================== */

/*
 * For each column k, with J_k given by M's pattern, solve (2.3) with I_k the nonzero
 * rows of A(:,J_k). Writes the values into Mval and ||A m_k - e_k|| into resnorm.
 * Returns the number of columns whose LS was singular.
 */
int64_t oracle_fixed_pattern(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                             const int64_t *Mcolptr, const int32_t *Mrowidx, double *Mval,
                             double *resnorm, int32_t nthreads) {
    omat A = {n, colptr, rowidx, val, NULL, NULL, 0.0};
    int64_t bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel reduction(+ : bad)
    {
        work w;
        memset(&w, 0, sizeof(w));
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n; ++k) {
            w.J.n = 0;
            for (int64_t e = Mcolptr[k]; e < Mcolptr[k + 1]; ++e) iv_push(&w.J, Mrowidx[e]);
            w.I.n = 0;
            for (int t = 0; t < w.J.n; ++t)
                for (int64_t e = A.colptr[w.J.a[t]]; e < A.colptr[w.J.a[t] + 1]; ++e) iv_push(&w.I, A.rowidx[e]);
            iv_sort_unique(&w.I);
            double rn = 0.0, fl = 0.0;
            if (ls_solve(&A, (int32_t)k, &w, &rn, &fl) != OR_OK) {
                ++bad;
                rn = NAN;
            } else {
                for (int t = 0; t < w.J.n; ++t) Mval[Mcolptr[k] + t] = w.mt.a[t];
            }
            if (resnorm) resnorm[k] = rn;
        }
        work_free(&w);
    }
    return bad;
}

/*
 * Adjoint of the fixed-pattern LS map A -> M (pattern of M fixed, M values from the
 * LS solves of (2.3)). From the normal equations A_k^T (A_k m - e) = 0:
 *   dm = -(A_k^T A_k)^{-1} (dA_k^T r + A_k^T dA_k m),  r = A_k m - e.
 * For an upstream g_k = dL/dm_k (on J_k) and z = (A_k^T A_k)^{-1} g_k:
 *   dL/dA_k = -(r z^T + (A_k z) m^T).
 * Adds also w_frob * d(sum_k ||A m_k - e_k||^2)/dA; the part of that term through M
 * vanishes since A_k^T r = 0, leaving 2 w_frob r m^T.
 * Every contribution is restricted to the structural nonzeros of A and accumulated
 * (+=) into dA (length nnz(A)). gM may be NULL (treated as zero).
 * The normal-equation system is solved here by forming A_k^T A_k and using a
 * Cholesky factorisation (an independent route from the QR of the forward solve).
 * dA_scale (nullable) accumulates, per entry, the magnitudes of the terms summed into
 * it, sum over contributions of |r_i z_j| + |(A_k z)_i m_j| + 2 w_frob |r_i m_j|: the
 * size of a rounding error of that entry does not depend on cancellation between them.
 */
int64_t oracle_backward(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                        const int64_t *Mcolptr, const int32_t *Mrowidx, const double *Mval,
                        const double *gM, double w_frob, double *dA, double *dA_scale) {
    omat A = {n, colptr, rowidx, val, NULL, NULL, 0.0};
    int64_t bad = 0;
    work w;
    memset(&w, 0, sizeof(w));
    dvec G = {0, 0, 0}, z = {0, 0, 0}, Az = {0, 0, 0}, rr = {0, 0, 0};
    for (int64_t k = 0; k < n; ++k) {
        const int q = (int)(Mcolptr[k + 1] - Mcolptr[k]);
        if (q == 0) continue;
        w.J.n = 0;
        for (int64_t e = Mcolptr[k]; e < Mcolptr[k + 1]; ++e) iv_push(&w.J, Mrowidx[e]);
        w.I.n = 0;
        for (int t = 0; t < q; ++t)
            for (int64_t e = A.colptr[w.J.a[t]]; e < A.colptr[w.J.a[t] + 1]; ++e) iv_push(&w.I, A.rowidx[e]);
        iv_sort_unique(&w.I);
        const int m = w.I.n;
        const double *mt = Mval + Mcolptr[k];
        /* dense A_k */
        dv_reserve(&w.B, m * q);
        memset(w.B.a, 0, sizeof(double) * (size_t)m * (size_t)q);
        for (int jj = 0; jj < q; ++jj)
            for (int64_t e = A.colptr[w.J.a[jj]]; e < A.colptr[w.J.a[jj] + 1]; ++e)
                w.B.a[find_sorted(w.I.a, m, A.rowidx[e]) + (size_t)m * jj] = A.val[e];
        double *B = w.B.a;
        /* residual r = A_k m - e_k(I) */
        dv_reserve(&rr, m);
        for (int ii = 0; ii < m; ++ii) {
            double s = 0.0;
            for (int jj = 0; jj < q; ++jj) s += B[ii + (size_t)m * jj] * mt[jj];
            rr.a[ii] = s - ((w.I.a[ii] == k) ? 1.0 : 0.0);
        }
        dv_reserve(&z, q);
        dv_reserve(&Az, m);
        int have_g = 0;
        if (gM) {
            for (int jj = 0; jj < q; ++jj) if (gM[Mcolptr[k] + jj] != 0.0) have_g = 1;
        }
        if (have_g) {
            /* G = A_k^T A_k (q x q), Cholesky G = L L^T, z = G^{-1} g */
            dv_reserve(&G, q * q);
            for (int a = 0; a < q; ++a)
                for (int b = 0; b <= a; ++b) {
                    double s = 0.0;
                    for (int ii = 0; ii < m; ++ii) s += B[ii + (size_t)m * a] * B[ii + (size_t)m * b];
                    G.a[a + (size_t)q * b] = s;
                }
            int ok = 1;
            for (int j = 0; j < q && ok; ++j) {
                double d = G.a[j + (size_t)q * j];
                for (int t = 0; t < j; ++t) d -= G.a[j + (size_t)q * t] * G.a[j + (size_t)q * t];
                if (!(d > 0.0)) { ok = 0; break; }
                d = sqrt(d);
                G.a[j + (size_t)q * j] = d;
                for (int i = j + 1; i < q; ++i) {
                    double s = G.a[i + (size_t)q * j];
                    for (int t = 0; t < j; ++t) s -= G.a[i + (size_t)q * t] * G.a[j + (size_t)q * t];
                    G.a[i + (size_t)q * j] = s / d;
                }
            }
            if (!ok) { ++bad; continue; }
            for (int i = 0; i < q; ++i) { /* L y = g */
                double s = gM[Mcolptr[k] + i];
                for (int t = 0; t < i; ++t) s -= G.a[i + (size_t)q * t] * z.a[t];
                z.a[i] = s / G.a[i + (size_t)q * i];
            }
            for (int i = q - 1; i >= 0; --i) { /* L^T z = y */
                double s = z.a[i];
                for (int t = i + 1; t < q; ++t) s -= G.a[t + (size_t)q * i] * z.a[t];
                z.a[i] = s / G.a[i + (size_t)q * i];
            }
            for (int ii = 0; ii < m; ++ii) {
                double s = 0.0;
                for (int jj = 0; jj < q; ++jj) s += B[ii + (size_t)m * jj] * z.a[jj];
                Az.a[ii] = s;
            }
        } else {
            for (int jj = 0; jj < q; ++jj) z.a[jj] = 0.0;
            for (int ii = 0; ii < m; ++ii) Az.a[ii] = 0.0;
        }
        /* scatter into the structural nonzeros of A(I_k, J_k) */
        for (int jj = 0; jj < q; ++jj) {
            int32_t j = w.J.a[jj];
            for (int64_t e = A.colptr[j]; e < A.colptr[j + 1]; ++e) {
                int ii = find_sorted(w.I.a, m, A.rowidx[e]);
                double gr = -(rr.a[ii] * z.a[jj] + Az.a[ii] * mt[jj]) + 2.0 * w_frob * rr.a[ii] * mt[jj];
                dA[e] += gr;
                if (dA_scale)
                    dA_scale[e] += fabs(rr.a[ii] * z.a[jj]) + fabs(Az.a[ii] * mt[jj]) +
                                   2.0 * fabs(w_frob * rr.a[ii] * mt[jj]);
            }
        }
    }
    work_free(&w);
    free(G.a); free(z.a); free(Az.a); free(rr.a);
    return bad;
}

/* ====================================================================== */
/*  Maximum transversal (row permutation to a zero-free diagonal)          */
/* ====================================================================== */

/*
 * Section 5 first permutes the rows of its test matrices that have zero diagonal
 * entries so that the diagonal becomes zero-free. Such a permutation is a
 * transversal: n structural nonzeros, no two in one row or one column, i.e. a
 * perfect matching of columns to rows in the bipartite graph of the pattern. A
 * matching of the largest size is found here from the definition by augmenting
 * paths (a matching is of maximum size exactly when no alternating path joins an
 * unmatched column to an unmatched row): each column in turn, in ascending order,
 * searches depth-first along alternating paths, its rows in ascending order,
 * visiting each row at most once per search, and flips the first path it finds.
 * match_col[k] receives the row matched to column k, or -1. Returns the size of
 * the matching (the structural rank of A).
 */
int64_t oracle_transversal(int64_t n, const int64_t *colptr, const int32_t *rowidx, int32_t *match_col) {
    int32_t *match_row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *visit = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *scol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)); /* columns on the path */
    int64_t *sedge = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1)); /* next entry of each */
    int32_t *srow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)); /* row taken from each */
    if (!match_row || !visit || !scol || !sedge || !srow) {
        free(match_row); free(visit); free(scol); free(sedge); free(srow);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) { match_row[i] = -1; match_col[i] = -1; visit[i] = -1; }
    int64_t size = 0;
    for (int64_t k = 0; k < n; ++k) {
        int top = 0;
        scol[0] = (int32_t)k;
        sedge[0] = colptr[k];
        int found = 0;
        while (top >= 0 && !found) {
            const int32_t c = scol[top];
            if (sedge[top] >= colptr[c + 1]) { --top; continue; }  /* dead end: back up */
            const int32_t r = rowidx[sedge[top]++];
            if (visit[r] == k) continue;
            visit[r] = k;
            srow[top] = r;
            if (match_row[r] < 0) { found = 1; break; }
            ++top; /* continue through the column matched to r */
            scol[top] = match_row[r];
            sedge[top] = colptr[match_row[r]];
        }
        if (!found) continue;
        /* flip the path: column scol[d] takes row srow[d] */
        for (int d = top; d >= 0; --d) {
            match_col[scol[d]] = srow[d];
            match_row[srow[d]] = scol[d];
        }
        ++size;
    }
    free(match_row); free(visit); free(scol); free(sedge); free(srow);
    return size;
}

/* ====================================================================== */
/*  Right-preconditioned BiCGStab (Section 5 protocol, textbook algorithm) */
/* ====================================================================== */

static void csc_matvec(int64_t n, const int64_t *cp, const int32_t *ri, const double *v, const double *x, double *y) {
    for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double xj = x[j];
        if (xj == 0.0) continue;
        for (int64_t e = cp[j]; e < cp[j + 1]; ++e) y[ri[e]] += v[e] * xj;
    }
}
static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Solve A M y = b, x = M y, x0 = 0, by BiCGStab. Stops when ||b - A x|| / ||b|| < tol
 * (true residual, checked after the half step and after the full step; a half-step
 * exit counts as that iteration) or after maxit iterations. Returns the number of
 * iterations used, or -1 on breakdown; *relres receives the final relative residual.
 * M may be NULL (no preconditioner).
 */
int32_t oracle_bicgstab(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                        const int64_t *Mcolptr, const int32_t *Mrowidx, const double *Mval,
                        const double *b, double tol, int32_t maxit, double *x, double *relres) {
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(sz), *rh = malloc(sz), *p = malloc(sz), *v = malloc(sz), *s = malloc(sz),
           *t = malloc(sz), *ph = malloc(sz), *sh = malloc(sz), *tmp = malloc(sz);
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; rh[i] = b[i]; p[i] = 0.0; v[i] = 0.0; }
    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) nb = 1.0;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    int32_t it = 0, ret = -1;
    double rel = sqrt(dot(n, r, r)) / nb;
#define APPLY_M(in, out)                                                             \
    do {                                                                             \
        if (Mcolptr) csc_matvec(n, Mcolptr, Mrowidx, Mval, in, out);                 \
        else for (int64_t i_ = 0; i_ < n; ++i_) out[i_] = in[i_];                    \
    } while (0)
    if (rel < tol) { ret = 0; goto done; }
    for (it = 1; it <= maxit; ++it) {
        double rho1 = dot(n, rh, r);
        if (rho1 == 0.0) { ret = -1; goto done; }
        if (it == 1) {
            for (int64_t i = 0; i < n; ++i) p[i] = r[i];
        } else {
            double beta = (rho1 / rho) * (alpha / omega);
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        APPLY_M(p, ph);
        csc_matvec(n, colptr, rowidx, val, ph, v);
        double rv = dot(n, rh, v);
        if (rv == 0.0) { ret = -1; goto done; }
        alpha = rho1 / rv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        /* half step: x + alpha * ph */
        for (int64_t i = 0; i < n; ++i) tmp[i] = x[i] + alpha * ph[i];
        {
            double *ax = malloc(sz);
            csc_matvec(n, colptr, rowidx, val, tmp, ax);
            double nr = 0.0;
            for (int64_t i = 0; i < n; ++i) nr += (b[i] - ax[i]) * (b[i] - ax[i]);
            free(ax);
            rel = sqrt(nr) / nb;
        }
        if (rel < tol) {
            for (int64_t i = 0; i < n; ++i) x[i] = tmp[i];
            ret = it;
            goto done;
        }
        APPLY_M(s, sh);
        csc_matvec(n, colptr, rowidx, val, sh, t);
        double tt = dot(n, t, t);
        if (tt == 0.0) { ret = -1; goto done; }
        omega = dot(n, t, s) / tt;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * ph[i] + omega * sh[i];
            r[i] = s[i] - omega * t[i];
        }
        {
            double *ax = malloc(sz);
            csc_matvec(n, colptr, rowidx, val, x, ax);
            double nr = 0.0;
            for (int64_t i = 0; i < n; ++i) nr += (b[i] - ax[i]) * (b[i] - ax[i]);
            free(ax);
            rel = sqrt(nr) / nb;
        }
        if (rel < tol) { ret = it; goto done; }
        if (omega == 0.0) { ret = -1; goto done; }
        rho = rho1;
    }
    ret = maxit + 1; /* not converged */
done:
#undef APPLY_M
    *relres = rel;
    free(r); free(rh); free(p); free(v); free(s); free(t); free(ph); free(sh); free(tmp);
    return ret;
}

/*
 * Left-preconditioned BiCGStab: the textbook iteration on M A x = M b (the left form
 * of (1.2)), x0 = 0, shadow residual r^ = r0 = M b. The stopping test is the one of
 * Section 5 on the true residual, ||b - A x|| / ||b|| < tol, after the half step
 * (x + alpha p) and after the full step. Return values as oracle_bicgstab.
 */
int32_t oracle_bicgstab_left(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                             const int64_t *Mcolptr, const int32_t *Mrowidx, const double *Mval,
                             const double *b, double tol, int32_t maxit, double *x, double *relres) {
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(sz), *rh = malloc(sz), *p = malloc(sz), *v = malloc(sz), *s = malloc(sz),
           *t = malloc(sz), *tmp = malloc(sz), *ax = malloc(sz);
    csc_matvec(n, Mcolptr, Mrowidx, Mval, b, r);
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
    double nb = sqrt(dot(n, b, b));
    double rel = (nb == 0.0) ? 0.0 : 1.0;
    if (nb == 0.0) nb = 1.0;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    int32_t it = 0, ret = -1;
    if (rel < tol) { ret = 0; goto done; }
    for (it = 1; it <= maxit; ++it) {
        double rho1 = dot(n, rh, r);
        if (rho1 == 0.0) { ret = -1; goto done; }
        if (it == 1) {
            for (int64_t i = 0; i < n; ++i) p[i] = r[i];
        } else {
            double beta = (rho1 / rho) * (alpha / omega);
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        csc_matvec(n, colptr, rowidx, val, p, tmp);            /* A p */
        csc_matvec(n, Mcolptr, Mrowidx, Mval, tmp, v);         /* v = M A p */
        double rv = dot(n, rh, v);
        if (rv == 0.0) { ret = -1; goto done; }
        alpha = rho1 / rv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        for (int64_t i = 0; i < n; ++i) tmp[i] = x[i] + alpha * p[i];
        csc_matvec(n, colptr, rowidx, val, tmp, ax);
        {
            double nr = 0.0;
            for (int64_t i = 0; i < n; ++i) nr += (b[i] - ax[i]) * (b[i] - ax[i]);
            rel = sqrt(nr) / nb;
        }
        if (rel < tol) {
            for (int64_t i = 0; i < n; ++i) x[i] = tmp[i];
            ret = it;
            goto done;
        }
        csc_matvec(n, colptr, rowidx, val, s, tmp);            /* A s */
        csc_matvec(n, Mcolptr, Mrowidx, Mval, tmp, t);         /* t = M A s */
        double tt = dot(n, t, t);
        if (tt == 0.0) { ret = -1; goto done; }
        omega = dot(n, t, s) / tt;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        csc_matvec(n, colptr, rowidx, val, x, ax);
        {
            double nr = 0.0;
            for (int64_t i = 0; i < n; ++i) nr += (b[i] - ax[i]) * (b[i] - ax[i]);
            rel = sqrt(nr) / nb;
        }
        if (rel < tol) { ret = it; goto done; }
        if (omega == 0.0) { ret = -1; goto done; }
        rho = rho1;
    }
    ret = maxit + 1;
done:
    *relres = rel;
    free(r); free(rh); free(p); free(v); free(s); free(t); free(tmp); free(ax);
    return ret;
}
