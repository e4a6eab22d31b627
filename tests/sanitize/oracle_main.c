/* The FP64 oracle (test infrastructure) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: ragged and degenerate instances (links on no
 * route, streams with empty routes and a finite box, one link on every
 * route, a single link), every utility, with and without the stop rule and
 * rho balancing, on one and on several threads. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int32_t *row_ptr, *col_idx;
    const double *c, *w;
    const uint8_t *utility;
    double lo, hi;
} orc_problem;
typedef struct {
    double rho0, alpha, mu, gamma, eps_abs;
    int32_t adapt_every, check_every, max_iter, stop, threads;
} orc_params;
typedef struct {
    int64_t iterations;
    double r_norm, s_norm, eps_tol, rho;
    int32_t converged;
} orc_result;

int orc_run(const orc_problem *, const orc_params *, double *, double *, double *, double *,
            double *, double *, double *, double *, double *, double *, double *, int32_t *,
            uint64_t *, const double *, double *, orc_result *);
double orc_prox_log(double, int64_t, double, double, double, double);
double orc_prox_linear(double, int64_t, double, double, double, double);
double orc_prox_alpha2(double, int64_t, double, double, double, double);
double orc_prox_slack(double, double);

#define REQUIRE(c)                                                               \
    do {                                                                         \
        if (!(c)) {                                                              \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                             \
        }                                                                        \
    } while (0)

static uint64_t rng_state = 88172645463325252ull;
static uint32_t rnd(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 11);
}

/* m links, n streams; link l uses a random subset; link m-1 (when busy) is on
 * every stream; every 7th link is empty; stream n-1 is on no route. */
static void run_case(int m, int n, int busy, int util_mode)
{
    int32_t *row_ptr = calloc((size_t)m + 1, sizeof(int32_t));
    int32_t *col_idx = malloc(((size_t)m * (size_t)n + 1) * sizeof(int32_t));
    double *c = malloc((size_t)m * sizeof(double)), *w = malloc(((size_t)n + 1) * sizeof(double));
    uint8_t *u = malloc((size_t)n + 1);
    int64_t nnz = 0;
    for (int l = 0; l < m; ++l) {
        for (int j = 0; j < n - 1; ++j) {
            const int on = (busy && l == m - 1) || (l % 7 != 3 && rnd() % 5 == 0);
            if (on) col_idx[nnz++] = j;
        }
        row_ptr[l + 1] = (int32_t)nnz;
        c[l] = 1.0 + (rnd() % 1000) / 100.0;
    }
    for (int j = 0; j < n; ++j) {
        w[j] = 0.5 + (rnd() % 1000) / 700.0;
        u[j] = (uint8_t)(util_mode < 3 ? util_mode : rnd() % 3);
    }
    orc_problem P = {m, n, nnz, row_ptr, col_idx, c, w, u, 0.0, 10.0};
    double *x = malloc(((size_t)n + 1) * sizeof(double));
    double *lam = malloc((size_t)m * sizeof(double)), *sl = malloc((size_t)m * sizeof(double));
    const int K = 300;
    double *hr = malloc(K * sizeof(double)), *hs = malloc(K * sizeof(double));
    double *hp = malloc(K * sizeof(double)), *hn = malloc(3 * K * sizeof(double));
    for (int variant = 0; variant < 4; ++variant) {
        orc_params prm = {1.0, variant == 3 ? 1.0 : 1.6, 2.0, 1.1, 1e-4, variant & 1 ? 50 : 0, 10, K,
                          variant >= 2, variant == 0 ? 1 : 3};
        double zw = 0.0, secs = 0.0;
        uint64_t dig = 0;
        int32_t thr = 0;
        orc_result res;
        REQUIRE(orc_run(&P, &prm, x, lam, sl, hr, hs, hp, hn, hn + K, hn + 2 * K, &zw, &secs, &thr,
                        &dig, NULL, NULL, &res) == 0);
        REQUIRE(res.iterations >= 1 && res.iterations <= K);
        for (int j = 0; j < n; ++j) REQUIRE(isfinite(x[j]) && x[j] >= 0.0 && x[j] <= 10.0);
        REQUIRE(x[n - 1] == 10.0);      /* empty route: the upper bound */
        for (int l = 0; l < m; ++l) REQUIRE(isfinite(lam[l]) && isfinite(sl[l]));
        REQUIRE(zw < 1e-9);
    }
    /* warm start: the saved iterate of one run starts the next */
    {
        const long long J = (long long)P.nnz + P.m;
        double *st = malloc((size_t)(3 * J + P.m + 1) * sizeof(double));
        double *st2 = malloc((size_t)(3 * J + P.m + 1) * sizeof(double));
        orc_params prm2 = {1.0, 1.6, 2.0, 1.1, 1e-4, 50, 10, 30, 0, 2};
        orc_result res2;
        REQUIRE(orc_run(&P, &prm2, x, lam, sl, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                        NULL, NULL, st, &res2) == 0);
        REQUIRE(orc_run(&P, &prm2, x, lam, sl, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                        NULL, st, st2, &res2) == 0);
        REQUIRE(st2[3 * J + P.m] > 0.0);
        free(st); free(st2);
    }
    /* NULL outputs are allowed */
    orc_params prm = {1.0, 1.6, 2.0, 1.1, 1e-4, 50, 10, 20, 0, 0};
    orc_result res;
    REQUIRE(orc_run(&P, &prm, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, &res) == 0);
    free(row_ptr); free(col_idx); free(c); free(w); free(u); free(x); free(lam); free(sl);
    free(hr); free(hs); free(hp); free(hn);
}

int main(void)
{
    /* proximal operators at their edges */
    REQUIRE(orc_prox_log(0.0, 0, 1.0, 1.0, 0.0, 7.0) == 7.0);
    REQUIRE(orc_prox_linear(3.0, 0, 1.0, 1.0, 0.0, 7.0) == 7.0);
    REQUIRE(orc_prox_alpha2(-2.0, 0, 1.0, 1.0, 0.0, 7.0) == 7.0);
    REQUIRE(orc_prox_log(-1e300, 3, 1.0, 1.0, 0.0, INFINITY) >= 0.0);
    REQUIRE(isfinite(orc_prox_alpha2(1e12, 4, 1e-9, 1e3, 0.0, INFINITY)));
    REQUIRE(orc_prox_alpha2(-1e12, 4, 2.0, 1e-3, 0.0, INFINITY) > 0.0);
    REQUIRE(orc_prox_slack(-5.0, 2.0) == -2.0 && orc_prox_slack(1.0, 2.0) == 1.0);
    /* invalid parameters are refused */
    {
        int32_t rp[2] = {0, 0};
        double c1 = 1.0;
        orc_problem P = {1, 0, 0, rp, rp, &c1, &c1, NULL, 0.0, 1.0};
        orc_params bad = {0.0, 1.6, 2.0, 1.1, 1e-4, 0, 10, 5, 0, 1};
        orc_result res;
        REQUIRE(orc_run(&P, &bad, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, &res) == -2);
        orc_params ok = {1.0, 1.6, 2.0, 1.1, 1e-4, 0, 10, 5, 0, 1};  /* no streams at all */
        REQUIRE(orc_run(&P, &ok, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, &res) == 0);
    }
    for (int mode = 0; mode < 4; ++mode) {
        run_case(40, 60, 1, mode);
        run_case(1, 9, 0, mode);
        run_case(13, 2, 1, mode);
    }
    printf("oracle: all checks passed\n");
    return 0;
}
