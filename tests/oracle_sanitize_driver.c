/* Runs the oracle's entry points on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * compiled and run by tests/test_oracle_sanitizers.py).  Exits 0 when every
 * call returns its expected status; a sanitizer report aborts the run. */
#include "../oracle/oracle_expm.c"

#include <stdio.h>

static int check(int ok, const char *what) {
    if (!ok) fprintf(stderr, "sanitize driver: %s failed\n", what);
    return ok ? 0 : 1;
}

int main(void) {
    int bad = 0;
    /* tridiag(1, -2, 1) * 3, n = 300 */
    const int64_t n = 300;
    int64_t *rp = malloc(sizeof(int64_t) * (n + 1));
    int32_t *ci = malloc(sizeof(int32_t) * 3 * n);
    double *v = malloc(sizeof(double) * 3 * n);
    int64_t k = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        if (i > 0) { ci[k] = (int32_t)(i - 1); v[k++] = 3.0; }
        ci[k] = (int32_t)i; v[k++] = -6.0;
        if (i + 1 < n) { ci[k] = (int32_t)(i + 1); v[k++] = 3.0; }
        rp[i + 1] = k;
    }
    for (int mode = 0; mode <= 2; mode++) {
        for (int norm = 0; norm <= 1; norm++) {
            ora_opts o = {-1, mode, 0.1, 64, 1, norm, mode == 0};
            int st = -99;
            ora_run *r = ora_expm(n, rp, ci, v, 1e-12, &o, &st);
            bad += check(st == ORA_OK && r, "expm");
            int64_t nnz = ora_run_nnz(r);
            double *dE = calloc((size_t)nnz, sizeof(double));
            double *dH = calloc((size_t)k, sizeof(double));
            for (int64_t p = 0; p < nnz; p += 7) dE[p] = 1.0;
            bad += check(ora_backward(r, dE, dH) == ORA_OK, "backward");
            int64_t *erp = malloc(sizeof(int64_t) * (n + 1));
            int32_t *eci = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
            double *ev = malloc(sizeof(double) * (size_t)(nnz + 1));
            ora_run_copy(r, erp, eci, ev);
            double *X = malloc(sizeof(double) * n * 5), *Y = malloc(sizeof(double) * n * 5);
            for (int64_t j = 0; j < n * 5; j++) X[j] = (double)(j % 11) - 5.0;
            ora_spmm(n, erp, eci, ev, 5, X, Y);
            free(dE); free(dH); free(erp); free(eci); free(ev); free(X); free(Y);
            ora_free(r);
        }
    }
    /* invalid input: a row pointer that decreases */
    rp[5] = rp[4] - 1;
    ora_opts o = {-1, 0, 0.1, 64, 0, 0, 0};
    int st = 0;
    ora_run *r = ora_expm(n, rp, ci, v, 1e-12, &o, &st);
    bad += check(st == ORA_EINVAL, "invalid input");
    ora_free(r);
    double norms[12];
    rp[5] = rp[4] + 3;
    bad += check(ora_power_norms(n, rp, ci, v, 12, norms) == ORA_OK, "power norms");
    int64_t ah = 0;
    bad += check(ora_alpha_hat(1e-12, 1, 8, 244.9, NULL, 0, &ah) == ORA_OK, "alpha hat 4.8");
    bad += check(ora_alpha_hat(1e-12, 1, 8, 0.0, norms, 12, &ah) == ORA_OK ||
                 ah == -1, "alpha hat 4.9");
    free(rp); free(ci); free(v);
    return bad;
}
