/*
 * Test driver for the oracle under host sanitizers (AddressSanitizer and
 * UndefinedBehaviorSanitizer): it reads a matrix file, runs RSAI(tol), the
 * fixed-pattern re-solve, the adjoint, and both BiCGStab forms through the oracle's
 * C entry points, and prints results the test compares with the oracle library.
 * Test infrastructure only, like the rest of this directory.
 *
 * Matrix file (little-endian): int64 n, int64 nnz, int64 colptr[n+1],
 * int32 rowidx[nnz], float64 val[nnz].
 * Usage: check_main FILE c lmax eps drop tol
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void *oracle_rsai(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val, int32_t c,
                  int32_t lmax, double eps, int32_t drop, double tol, int32_t nthreads, const int64_t *cols,
                  int64_t ncols, int32_t record_hist);
int64_t oracle_nnz(void *h);
void oracle_export(void *h, int64_t *colptr, int32_t *rowidx, double *val, int32_t *loops, double *resnorm,
                   int32_t *nI, int32_t *nJ, int32_t *status, double *sel_margin, double *drop_margin,
                   double *flops, int32_t *nsolve, double *hist, int32_t *ndrop, double *mflops);
void oracle_export_peaks(void *h, int32_t *nImax, int32_t *nJmax);
void oracle_free(void *h);
int64_t oracle_fixed_pattern(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                             const int64_t *Mcolptr, const int32_t *Mrowidx, double *Mval, double *resnorm,
                             int32_t nthreads);
int64_t oracle_backward(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                        const int64_t *Mcolptr, const int32_t *Mrowidx, const double *Mval, const double *gM,
                        double w_frob, double *dA, double *dA_scale);
int32_t oracle_bicgstab(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                        const int64_t *Mcolptr, const int32_t *Mrowidx, const double *Mval, const double *b,
                        double tol, int32_t maxit, double *x, double *relres);
int32_t oracle_bicgstab_left(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                             const int64_t *Mcolptr, const int32_t *Mrowidx, const double *Mval,
                             const double *b, double tol, int32_t maxit, double *x, double *relres);

static void *read_all(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 7) {
        fprintf(stderr, "usage: %s FILE c lmax eps drop tol\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[2];
    if (fread(hdr, sizeof(int64_t), 2, f) != 2) return 2;
    const int64_t n = hdr[0], nnz = hdr[1];
    int64_t *colptr = read_all(f, sizeof(int64_t) * (size_t)(n + 1));
    int32_t *rowidx = read_all(f, sizeof(int32_t) * (size_t)nnz);
    double *val = read_all(f, sizeof(double) * (size_t)nnz);
    fclose(f);
    const int32_t c = atoi(argv[2]), lmax = atoi(argv[3]), drop = atoi(argv[5]);
    const double eps = atof(argv[4]), tol = atof(argv[6]);

    void *h = oracle_rsai(n, colptr, rowidx, val, c, lmax, eps, drop, tol, 2, NULL, n, 1);
    if (!h) return 3;
    const int64_t nzm = oracle_nnz(h);
    int64_t *mcp = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *mri = malloc(sizeof(int32_t) * (size_t)(nzm ? nzm : 1));
    double *mv = malloc(sizeof(double) * (size_t)(nzm ? nzm : 1));
    double *rn = malloc(sizeof(double) * (size_t)n);
    int32_t *nJmax = malloc(sizeof(int32_t) * (size_t)n);
    double *hist = malloc(sizeof(double) * (size_t)n * 2 * (size_t)(lmax + 1));
    oracle_export(h, mcp, mri, mv, NULL, rn, NULL, NULL, NULL, NULL, NULL, NULL, NULL, hist, NULL, NULL);
    oracle_export_peaks(h, NULL, nJmax);
    oracle_free(h);

    double sv = 0.0, srn = 0.0;
    long long sr = 0, sj = 0;
    for (int64_t e = 0; e < nzm; ++e) { sv += mv[e]; sr += mri[e]; }
    for (int64_t k = 0; k < n; ++k) { srn += rn[k]; sj += nJmax[k]; }
    printf("rsai nnz %lld rowsum %lld valsum %.17g resnorm %.17g nJmax %lld\n", (long long)nzm, sr, sv, srn, sj);

    double *mv2 = malloc(sizeof(double) * (size_t)(nzm ? nzm : 1));
    double *rn2 = malloc(sizeof(double) * (size_t)n);
    const int64_t bad = oracle_fixed_pattern(n, colptr, rowidx, val, mcp, mri, mv2, rn2, 2);
    double dmax = 0.0;
    for (int64_t e = 0; e < nzm; ++e) {
        const double d = mv2[e] > mv[e] ? mv2[e] - mv[e] : mv[e] - mv2[e];
        if (d > dmax) dmax = d;
    }
    printf("fixed bad %lld maxdiff %.3g\n", (long long)bad, dmax);

    double *gM = malloc(sizeof(double) * (size_t)(nzm ? nzm : 1));
    double *dA = calloc((size_t)nnz, sizeof(double));
    double *dAs = calloc((size_t)nnz, sizeof(double));
    for (int64_t e = 0; e < nzm; ++e) gM[e] = 1.0 / (1.0 + (double)(e % 7));
    const int64_t badb = oracle_backward(n, colptr, rowidx, val, mcp, mri, mv, gM, 0.5, dA, dAs);
    double sd = 0.0;
    for (int64_t e = 0; e < nnz; ++e) sd += dA[e];
    printf("backward bad %lld sum %.17g\n", (long long)badb, sd);

    double *b = malloc(sizeof(double) * (size_t)n), *x = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) b[i] = 1.0 + (double)(i % 5);
    double rel = 0.0;
    const int32_t it = oracle_bicgstab(n, colptr, rowidx, val, mcp, mri, mv, b, 1e-8, 500, x, &rel);
    const int32_t it0 = oracle_bicgstab(n, colptr, rowidx, val, NULL, NULL, NULL, b, 1e-8, 500, x, &rel);
    const int32_t itl = oracle_bicgstab_left(n, colptr, rowidx, val, mcp, mri, mv, b, 1e-8, 500, x, &rel);
    printf("bicgstab right %d none %d left %d\n", it, it0, itl);

    free(colptr); free(rowidx); free(val); free(mcp); free(mri); free(mv); free(rn); free(nJmax); free(hist);
    free(mv2); free(rn2); free(gM); free(dA); free(dAs); free(b); free(x);
    return 0;
}
