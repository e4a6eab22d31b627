/*
 * FP64 CPU oracle for proximal message passing (PMP) on network utility
 * maximization.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it to check and time the HIP library; the
 * library itself never links or calls anything here, and nothing here is
 * shared with it.
 *
 * It follows the paper's literal per-terminal formulation, in the paper's
 * order and notation:
 *
 *   problem      maximize sum_j U_j(x_j) s.t. R x <= c, x >= 0 (eq. (2)),
 *                written with slacks R x + s = c, s >= 0 (eq. (3)), plus a box
 *                lo <= x_j <= hi on every rate.
 *   terminals    one terminal per nonzero of R (traffic terminal of stream j at
 *                link l) and one slack terminal per link; J = nnz(R) + m
 *                (Section III, bipartite graph).
 *   ADMM         p-, z- and u-updates of the scaled augmented Lagrangian on
 *                the consensus form p = z (eq. (8), eq. (9) and the three
 *                update equations of Section III-D), with over-relaxation
 *                p+ = alpha p + (1 - alpha) z in the z- and u-updates
 *                (Section III-G, over-relaxation).
 *   prox         log, linear and slack closed forms (Section III-E).
 *   residuals    r = pbar, s = rho((p - pbar) - (p_prev - pbar_prev)), one
 *                entry per terminal; stop when both 2-norms are below
 *                eps_abs * sqrt(J) (Section III-F, eq. (16)).
 *   rho          residual balancing every `adapt_every` iterations with the
 *                scaled dual rescaled by rho_old / rho_new (Section III-G,
 *                eqs. (17) and (18)).
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes):
 *   - The z-update is the plain projection of p+ + u onto {1^T z_l = 0}; the
 *     printed shortcut "z = u + pbar" is not used (it does not follow from
 *     the projection).
 *   - The argument of every prox is z - u, the ADMM p-update; with alpha = 1
 *     this equals p - pbar - u as in the PMP form.
 *   - The linear prox uses + w/rho (the sign that minimises
 *     -w x + rho/2 sum (x - zeta_i)^2).
 *   - Box: the 1-D prox is clipped to [lo, hi], which is exact for a strictly
 *     convex scalar problem.  A stream with no links takes x = hi.
 *   - For S < 0 the log prox is evaluated in the algebraically equal form
 *     2w / (rho (sqrt(S^2 + 4wL/rho) - S)), which avoids cancellation.
 *   - Initial state: p = z = u = 0 and rho = rho0.
 *   - The residual uses the rho of the iteration (before any balancing step
 *     at that iteration); the stop test precedes the balancing step.
 *   - Link prices are lambda = rho * u (u is the scaled dual y / rho,
 *     Section III-D).
 *
 * Parallelism: plain OpenMP loops over streams and over links; residual sums
 * are formed per link and then added in link order, so results do not depend
 * on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int32_t *row_ptr;   /* [m+1] CSR of the 0/1 link-route matrix R */
    const int32_t *col_idx;   /* [nnz] streams using each link             */
    const double *c;          /* [m] link capacities, > 0                  */
    const double *w;          /* [n] stream weights, > 0                   */
    const uint8_t *utility;   /* [n] 0 = w log x, 1 = w x, 2 = -w / x      */
    double lo, hi;            /* box on every rate                         */
} orc_problem;

typedef struct {
    double rho0, alpha, mu, gamma, eps_abs;
    int32_t adapt_every;      /* 0: keep rho fixed                         */
    int32_t check_every;      /* stop-test cadence (stop = 1 only)         */
    int32_t max_iter;
    int32_t stop;             /* 0: run exactly max_iter iterations        */
    int32_t threads;          /* 0: OpenMP default                         */
} orc_params;

typedef struct {
    int64_t iterations;
    double r_norm, s_norm, eps_tol, rho;
    int32_t converged;
} orc_result;

/* ---- Section III-E: proximal operators (scalar forms) ------------------- */

/* Log utility f(x) = -w log x on L identical terminals: argmin_x
 * -w log x + rho/2 sum_i (x - zeta_i)^2 with S = sum_i zeta_i. */
double orc_prox_log(double S, int64_t L, double w, double rho, double lo, double hi)
{
    double x;
    if (L == 0) return hi;
    double disc = sqrt(S * S + 4.0 * w * (double)L / rho);
    if (S >= 0.0) x = (S + disc) / (2.0 * (double)L);
    else          x = 2.0 * w / (rho * (disc - S));
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    return x;
}

/* Linear utility f(x) = -w x: argmin_x -w x + rho/2 sum_i (x - zeta_i)^2. */
double orc_prox_linear(double S, int64_t L, double w, double rho, double lo, double hi)
{
    double x;
    if (L == 0) return hi;
    x = (S + w / rho) / (double)L;
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    return x;
}

/* Minimum potential delay fairness (the alpha = 2 member of the alpha-fair
 * family named in Section II), f(x) = w / x for x > 0: the stationarity
 * condition -w / x^2 + rho (L x - S) = 0 is the cubic
 * g(x) = x^2 (L x - S) - w/rho = 0.  With s+ = max(S/L, 0) and
 * t = (w / (rho L))^(1/3): g < 0 on (0, s+] (there L x - S <= 0), g is
 * increasing beyond s+, and g(s+ + t) >= L t^3 - w/rho = 0, so the one
 * positive root lies in (s+, s+ + t].  Plain bisection on that bracket,
 * halved until the midpoint no longer falls strictly inside it. */
double orc_prox_alpha2(double S, int64_t L, double w, double rho, double lo, double hi)
{
    if (L == 0) return hi;
    const double dl = (double)L, c = w / rho;
    double a = S > 0.0 ? S / dl : 0.0;
    double b = a + cbrt(c / dl);
    for (;;) {
        const double mid = 0.5 * (a + b);
        if (!(mid > a && mid < b)) break;
        if (mid * mid * (dl * mid - S) - c < 0.0) a = mid;
        else b = mid;
    }
    double x = b;
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    return x;
}

/* Slack stream f(p) = indicator(p + c >= 0): projection onto p >= -c. */
double orc_prox_slack(double zeta, double c)
{
    return zeta > -c ? zeta : -c;
}

/* ---- terminal graph (Section III) --------------------------------------- */

typedef struct {
    int64_t J;
    int64_t *stream_first;   /* [n+1] terminals of traffic stream j        */
    int64_t *link_first;     /* [m+1] terminals of link l (d_l + 1 each)   */
    int64_t *link_terms;     /* [J]   terminal ids, grouped by link        */
} terminals;

static int build_terminals(const orc_problem *P, terminals *T)
{
    int64_t n = P->n, m = P->m, nnz = P->nnz;
    int64_t *fill = calloc((size_t)n + 1, sizeof(int64_t));
    T->J = nnz + m;
    T->stream_first = calloc((size_t)n + 1, sizeof(int64_t));
    T->link_first = calloc((size_t)m + 1, sizeof(int64_t));
    T->link_terms = malloc((size_t)(T->J > 0 ? T->J : 1) * sizeof(int64_t));
    if (!fill || !T->stream_first || !T->link_first || !T->link_terms) {
        free(fill);
        return -1;
    }
    /* |sigma_j| = number of links on route j */
    for (int64_t k = 0; k < nnz; ++k) T->stream_first[P->col_idx[k] + 1]++;
    for (int64_t j = 0; j < n; ++j) T->stream_first[j + 1] += T->stream_first[j];
    /* traffic terminals: stream j owns [stream_first[j], stream_first[j+1]),
     * one per link on its route, in increasing link order.
     * slack terminal of link l: id nnz + l. */
    for (int64_t l = 0; l < m; ++l) {
        int64_t base = P->row_ptr[l] + l;     /* |l| = d_l + 1 terminals */
        T->link_first[l] = base;
        for (int64_t k = P->row_ptr[l]; k < P->row_ptr[l + 1]; ++k) {
            int64_t j = P->col_idx[k];
            int64_t t = T->stream_first[j] + fill[j]++;
            T->link_terms[base + (k - P->row_ptr[l])] = t;
        }
        T->link_terms[base + (P->row_ptr[l + 1] - P->row_ptr[l])] = nnz + l;
    }
    T->link_first[m] = nnz + m;
    free(fill);
    return 0;
}

static void free_terminals(terminals *T)
{
    free(T->stream_first);
    free(T->link_first);
    free(T->link_terms);
}

/*
 * Run PMP.  Outputs (any may be NULL):
 *   x[n]       stream rates
 *   lambda[m]  link prices rho * u
 *   slack[m]   s = p_slack + c (the recovery relation stated under eq. (8))
 *   hist_r, hist_s, hist_rho [max_iter]: per-iteration ||r||, ||s||, rho used
 *   hist_pn, hist_zn, hist_un [max_iter]: per-iteration ||p||, ||z|| and
 *              ||rho u|| over all terminals (u one value per terminal), the
 *              scales of the relative form of the stopping rule in the ADMM
 *              reference the paper cites for convergence (Section III-F)
 *   loop_seconds  wall time of the iteration loop (setup excluded)
 *   threads_used  OpenMP threads of the parallel loops
 *   zsum_worst  max over iterations and links of |1^T z_l| / (1 + max|z_l|):
 *               the link flow-balance indicator g_l (Section III-C) asks
 *               1^T z_l = 0 after every z-update
 *   branch_digest  64-bit FNV-1a hash, over all iterations in order, of the
 *               branch every prox took: per stream 0 (interior), 1 (x = lo) or
 *               2 (x = hi), then per link 1 when the slack prox kept its
 *               argument (z - u > -c) and 0 when it projected.  Two runs whose
 *               digests are equal took the same branches throughout, so the
 *               map from the data to x^K is smooth between them (used to drop
 *               finite-difference pairs that straddle a kink).
 *   state_in, state_out [3J + m + 1]: the iterate z[J], u[J], p[J] (the last
 *               iteration's flows, for the next dual residual), pbar[m] and
 *               rho.  With state_in the run starts from that iterate and its
 *               rho (rho0 is ignored): a warm start, for instance after the
 *               capacities changed (Section V-D); state_out receives the
 *               final iterate in the same layout.
 * Returns 0 on success, -1 on allocation failure, -2 on invalid parameters.
 */
int orc_run(const orc_problem *P, const orc_params *prm,
            double *x, double *lambda, double *slack,
            double *hist_r, double *hist_s, double *hist_rho,
            double *hist_pn, double *hist_zn, double *hist_un,
            double *zsum_worst, double *loop_seconds, int32_t *threads_used,
            uint64_t *branch_digest, const double *state_in, double *state_out,
            orc_result *res)
{
    if (prm->max_iter < 0 || prm->rho0 <= 0.0) return -2;
    if (prm->stop && prm->check_every <= 0) return -2;
#ifdef _OPENMP
    if (prm->threads > 0) omp_set_num_threads(prm->threads);
#endif
    const int64_t n = P->n, m = P->m, nnz = P->nnz;
    terminals T;
    if (build_terminals(P, &T)) return -1;
    const int64_t J = T.J;
    size_t Jz = (size_t)(J > 0 ? J : 1);
    double *p = calloc(Jz, sizeof(double));          /* stream-side flows  */
    double *z = calloc(Jz, sizeof(double));          /* link-side copies   */
    double *u = calloc(Jz, sizeof(double));          /* scaled duals       */
    double *p_prev = calloc(Jz, sizeof(double));
    double *pbar_prev = calloc((size_t)m + 1, sizeof(double));
    double *r2_link = calloc((size_t)m + 1, sizeof(double));
    double *s2_link = calloc((size_t)m + 1, sizeof(double));
    double *zs_link = calloc((size_t)m + 1, sizeof(double));
    double *pn_link = calloc((size_t)m + 1, sizeof(double));   /* sum p^2, z^2, u^2 */
    double *zn_link = calloc((size_t)m + 1, sizeof(double));
    double *un_link = calloc((size_t)m + 1, sizeof(double));
    double *xs = calloc((size_t)n + 1, sizeof(double));
    uint8_t *branch = branch_digest ? calloc((size_t)(n + m) + 1, 1) : NULL;
    if (!p || !z || !u || !p_prev || !pbar_prev || !r2_link || !s2_link ||
        !zs_link || !xs || !pn_link || !zn_link || !un_link || (branch_digest && !branch)) {
        free(p); free(z); free(u); free(p_prev); free(pbar_prev);
        free(r2_link); free(s2_link); free(zs_link); free(xs);
        free(pn_link); free(zn_link); free(un_link); free(branch); free_terminals(&T);
        return -1;
    }
    uint64_t digest = 14695981039346656037ull;       /* FNV-1a offset basis */
    const double alpha = prm->alpha;
    const double eps_tol = prm->eps_abs * sqrt((double)J);
    double rho = prm->rho0;
    if (state_in) {
        memcpy(z, state_in, (size_t)J * sizeof(double));
        memcpy(u, state_in + J, (size_t)J * sizeof(double));
        memcpy(p_prev, state_in + 2 * J, (size_t)J * sizeof(double));
        memcpy(pbar_prev, state_in + 3 * J, (size_t)m * sizeof(double));
        rho = state_in[3 * J + m];
        if (!(rho > 0.0)) rho = prm->rho0;
    }
    double r_norm = 0.0, s_norm = 0.0, zsum_max = 0.0;
    int converged = 0;
    int64_t k;
#ifdef _OPENMP
    if (threads_used) *threads_used = omp_get_max_threads();
    double t_start = omp_get_wtime();
#else
    if (threads_used) *threads_used = 1;
#endif

    for (k = 1; k <= prm->max_iter; ++k) {
        /* 1. proximal device updates: p_sigma = prox(z_sigma - u_sigma) */
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            int64_t t0 = T.stream_first[j], t1 = T.stream_first[j + 1];
            double S = 0.0;
            for (int64_t t = t0; t < t1; ++t) S += z[t] - u[t];
            double xj = P->utility[j] == 0
                ? orc_prox_log(S, t1 - t0, P->w[j], rho, P->lo, P->hi)
                : P->utility[j] == 1
                ? orc_prox_linear(S, t1 - t0, P->w[j], rho, P->lo, P->hi)
                : orc_prox_alpha2(S, t1 - t0, P->w[j], rho, P->lo, P->hi);
            xs[j] = xj;
            for (int64_t t = t0; t < t1; ++t) p[t] = xj;   /* p_sigma = x 1 */
            if (branch) branch[j] = t1 > t0 && xj == P->lo ? 1 : t1 > t0 && xj == P->hi ? 2 : 0;
        }
        #pragma omp parallel for schedule(static)
        for (int64_t l = 0; l < m; ++l) {
            int64_t t = nnz + l;
            p[t] = orc_prox_slack(z[t] - u[t], P->c[l]);
            if (branch) branch[n + l] = z[t] - u[t] > -P->c[l];
        }
        if (branch)
            for (int64_t i = 0; i < n + m; ++i) {
                digest ^= branch[i];
                digest *= 1099511628211ull;              /* FNV-1a prime */
            }

        /* 2.-4. per link: average, over-relaxed z-projection, dual update;
         * 5. residual contributions of the link's terminals */
        #pragma omp parallel for schedule(static)
        for (int64_t l = 0; l < m; ++l) {
            int64_t a = T.link_first[l], b = T.link_first[l + 1];
            double cnt = (double)(b - a);
            double sum_p = 0.0, sum_q = 0.0;
            for (int64_t i = a; i < b; ++i) sum_p += p[T.link_terms[i]];
            double pb = sum_p / cnt;                          /* pbar_l */
            for (int64_t i = a; i < b; ++i) {
                int64_t t = T.link_terms[i];
                double pplus = alpha * p[t] + (1.0 - alpha) * z[t];
                sum_q += pplus + u[t];
            }
            double q = sum_q / cnt;
            double s2 = 0.0, zsum = 0.0, zmax = 0.0, pn = 0.0, zn = 0.0, un = 0.0;
            for (int64_t i = a; i < b; ++i) {
                int64_t t = T.link_terms[i];
                double pplus = alpha * p[t] + (1.0 - alpha) * z[t];
                double znew = pplus + u[t] - q;               /* projection */
                u[t] = u[t] + pplus - znew;                   /* dual step  */
                z[t] = znew;
                zsum += znew;
                if (fabs(znew) > zmax) zmax = fabs(znew);
                double st = rho * ((p[t] - pb) - (p_prev[t] - pbar_prev[l]));
                s2 += st * st;
                p_prev[t] = p[t];
                pn += p[t] * p[t];
                zn += znew * znew;
                un += u[t] * u[t];
            }
            r2_link[l] = cnt * pb * pb;                       /* r_t = pbar */
            s2_link[l] = s2;
            pn_link[l] = pn;
            zn_link[l] = zn;
            un_link[l] = un;
            zs_link[l] = fabs(zsum) / (1.0 + zmax);
            pbar_prev[l] = pb;
        }
        double r2 = 0.0, s2 = 0.0, pn2 = 0.0, zn2 = 0.0, un2 = 0.0;
        for (int64_t l = 0; l < m; ++l) {
            r2 += r2_link[l];
            s2 += s2_link[l];
            pn2 += pn_link[l];
            zn2 += zn_link[l];
            un2 += un_link[l];
            if (zs_link[l] > zsum_max) zsum_max = zs_link[l];
        }
        r_norm = sqrt(r2);
        s_norm = sqrt(s2);
        if (hist_r) hist_r[k - 1] = r_norm;
        if (hist_s) hist_s[k - 1] = s_norm;
        if (hist_rho) hist_rho[k - 1] = rho;
        if (hist_pn) hist_pn[k - 1] = sqrt(pn2);
        if (hist_zn) hist_zn[k - 1] = sqrt(zn2);
        if (hist_un) hist_un[k - 1] = rho * sqrt(un2);

        /* 6. stopping criterion */
        if (prm->stop && k % prm->check_every == 0 &&
            r_norm < eps_tol && s_norm < eps_tol) {
            converged = 1;
            break;
        }
        /* 7. residual balancing of rho and rescaling of u */
        if (prm->adapt_every > 0 && k % prm->adapt_every == 0) {
            double rho_new = rho;
            if (r_norm > prm->mu * s_norm) rho_new = prm->gamma * rho;
            else if (s_norm > prm->mu * r_norm) rho_new = rho / prm->gamma;
            if (rho_new != rho) {
                double ratio = rho / rho_new;
                #pragma omp parallel for schedule(static)
                for (int64_t t = 0; t < J; ++t) u[t] *= ratio;
                rho = rho_new;
            }
        }
    }
    if (k > prm->max_iter) k = prm->max_iter;
#ifdef _OPENMP
    if (loop_seconds) *loop_seconds = omp_get_wtime() - t_start;
#else
    if (loop_seconds) *loop_seconds = 0.0;
#endif

    if (x) for (int64_t j = 0; j < n; ++j) x[j] = xs[j];
    if (lambda) for (int64_t l = 0; l < m; ++l) lambda[l] = rho * u[nnz + l];
    if (slack) for (int64_t l = 0; l < m; ++l) slack[l] = p[nnz + l] + P->c[l];
    if (zsum_worst) *zsum_worst = zsum_max;
    if (branch_digest) *branch_digest = digest;
    if (state_out) {
        memcpy(state_out, z, (size_t)J * sizeof(double));
        memcpy(state_out + J, u, (size_t)J * sizeof(double));
        memcpy(state_out + 2 * J, p_prev, (size_t)J * sizeof(double));
        memcpy(state_out + 3 * J, pbar_prev, (size_t)m * sizeof(double));
        state_out[3 * J + m] = rho;
    }
    if (res) {
        res->iterations = k;
        res->r_norm = r_norm;
        res->s_norm = s_norm;
        res->eps_tol = eps_tol;
        res->rho = rho;
        res->converged = converged;
    }
    free(p); free(z); free(u); free(p_prev); free(pbar_prev);
    free(r2_link); free(s2_link); free(zs_link); free(xs);
    free(pn_link); free(zn_link); free(un_link); free(branch);
    free_terminals(&T);
    return 0;
}
