/*
 * pmp.h -- proximal message passing (PMP) for network utility maximization
 * on AMD Instinct MI355X (gfx950).  C ABI; no exceptions cross it.
 *
 * Problem (eq. (2) with the slack form of eq. (3), plus a box on every rate):
 *
 *     maximize  sum_j U_j(x_j)   subject to   R x <= c,   lo <= x_j <= hi
 *
 *   R  m x n link-route matrix with R_lj = 1 when stream j uses link l
 *      (eq. (1)); only its pattern is stored (CSR here, CSC built inside).
 *   U_j = w_j log x_j  (weighted proportional fairness),  w_j x_j
 *      (linear), Section II, or  -w_j / x_j  (alpha = 2 fairness).
 *
 * Method: the over-relaxed PMP iteration of Section III-D..G (ADMM on the
 * terminal graph), held in a compact per-stream / per-link form:
 *   stream pass  S_j = L_j a_j + sum_{l in route j} v_l;  x_j = prox(S_j)
 *                (log / linear closed forms of Section III-E, clipped to the
 *                box); a_j <- alpha x_j + (1 - alpha) a_j
 *   link pass    y_l = sum_{j on link l} x_j;  ps_l = max(zs_l - u_l, -c_l)
 *                (slack prox); pbar_l = (y_l + ps_l) / (d_l + 1);
 *                b_l <- -alpha pbar_l + (1 - alpha) b_l;
 *                zs_l <- alpha (ps_l - pbar_l) + (1 - alpha) zs_l;
 *                u_l <- u_l + alpha pbar_l;  v_l = b_l - u_l
 *   (a_j + b_l is the link-side copy z of terminal (j, l), zs_l that of the
 *   slack terminal; u is the scaled dual.)  Residuals ||r||, ||s|| and the
 *   stop rule of Section III-F; residual balancing of rho every
 *   `adapt_every` iterations with the rescale of u (Section III-G, eqs. (17),
 *   (18)).  Link prices are lambda = rho u; the slack is s = ps + c.
 *
 * Memory: every device buffer lives in one caller-owned workspace (size from
 * pmp_workspace_size).  The library allocates no device memory itself; it
 * allocates a small pinned host buffer and a private stream per handle (for
 * graph capture).  Streams are passed as `void*` holding a hipStream_t
 * (NULL = the null stream).
 *
 * Errors: every call returns a pmp_status.  PMP_ERR_INVALID / PMP_ERR_SHAPE
 * carry a detail string from pmp_last_error() (thread-local).  Asynchronous
 * HIP failures surface as PMP_ERR_HIP at the next call that synchronises.
 * A non-finite residual gives PMP_ERR_NUMERIC.
 */
#ifndef PMP_H
#define PMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMP_OK = 0,
    PMP_ERR_INVALID = 1,    /* bad problem data or parameters               */
    PMP_ERR_SHAPE = 2,      /* sizes out of range, workspace too small      */
    PMP_ERR_NOMEM = 3,      /* host allocation failed                       */
    PMP_ERR_HIP = 4,        /* a HIP runtime call failed                    */
    PMP_ERR_NUMERIC = 5,    /* non-finite residual                          */
    PMP_NOT_CONVERGED = 6,  /* max_iter reached; the result is still valid  */
    PMP_ERR_STATE = 7       /* call not valid for this handle               */
} pmp_status;

/* Utilities (Section II): w log x (proportional fairness), w x (linear) and
 * -w / x (minimum potential delay fairness, the alpha = 2 member of the
 * alpha-fair family the paper names; its prox is the positive root of a
 * cubic, found by Newton's method). */
typedef enum { PMP_UTIL_LOG = 0, PMP_UTIL_LINEAR = 1, PMP_UTIL_ALPHA2 = 2 } pmp_utility;
typedef enum { PMP_F32 = 0, PMP_F64 = 1 } pmp_dtype;
typedef enum { PMP_MEM_HOST = 0, PMP_MEM_DEVICE = 1 } pmp_memory;

/* One NUM instance (eq. (1)-(2)).  All arrays are in `memory`; the floating
 * point arrays have type `dtype`.
 *   row_ptr[m+1], col_idx[nnz]  CSR pattern of R: row_ptr[0] = 0,
 *                               row_ptr[m] = nnz, nondecreasing; col_idx in
 *                               [0, n), strictly increasing within a row.
 *   c[m]        capacities, finite and > 0 (Section II).
 *   w[n]        weights, finite and > 0 (Section III-B).
 *   utility[n]  pmp_utility per stream.
 *   lo, hi      box, 0 <= lo < hi; hi may be +inf unless some stream has an
 *               empty route (such a stream takes x = hi).
 * HOST arrays are copied into the workspace during pmp_setup; DEVICE arrays
 * are read during pmp_setup only (c, w and the pattern are copied too), so
 * they may be freed after it returns.  m >= 1, n >= 0 and nnz < 2^31. */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const void *c;
    const void *w;
    const uint8_t *utility;
    double lo, hi;
    pmp_dtype dtype;
    pmp_memory memory;
} pmp_problem;

/* Solver controls (Section III-F, III-G).
 *   rho0         initial penalty (> 0)
 *   alpha        over-relaxation in (0, 2) (the paper uses 1.6)
 *   mu, gamma    residual-balancing thresholds (> 1; the paper uses 2, 1.1)
 *   eps_abs      absolute tolerance; stop when ||r||, ||s|| < eps_abs sqrt(J),
 *                J = nnz + m terminals (Section III-F)
 *   eps_rel      relative tolerance (>= 0, default 0): with eps_rel > 0 the
 *                rule becomes ||r|| < eps_abs sqrt(J) + eps_rel max(||p||, ||z||)
 *                and ||s|| < eps_abs sqrt(J) + eps_rel ||rho u||, the
 *                relative form of the ADMM stopping rule that Section III-F
 *                builds on (norms over all J terminals); each check then
 *                adds one pass over the n- and m-vectors.  Batched solves
 *                take the absolute rule only.
 *   adapt_every  rho balancing period in iterations (0 = fixed rho); must be
 *                a multiple of check_every
 *   check_every  residual / stop-test period of pmp_solve (>= 1)
 *   max_iter     iteration cap of one pmp_solve call
 *   layout       sparse layout of the iteration: PMP_LAYOUT_AUTO picks
 *                PMP_LAYOUT_BINNED for FP32 problems with nnz >= 2^21,
 *                m, n >= 256 and tiles of 16 or more nonzeros on average,
 *                PMP_LAYOUT_GATHER otherwise; BINNED asked for with more
 *                than 2^28 tiles is refused (PMP_ERR_SHAPE).  GATHER: CSR /
 *                CSC passes with LDS-staged gathers (fastest while the
 *                gathered vectors stay in cache).  BINNED: R tiled into
 *                link-block x stream-block tiles with one message per
 *                nonzero per direction, streamed through HBM in coalesced
 *                runs (for large unstructured R, where random gathers are
 *                slow); with FP32 its sums equal the gather layout's bit for
 *                bit whenever they are exact in FP64. */
typedef enum { PMP_LAYOUT_AUTO = 0, PMP_LAYOUT_GATHER = 1, PMP_LAYOUT_BINNED = 2 } pmp_layout;
typedef struct {
    double rho0, alpha, mu, gamma, eps_abs;
    int32_t adapt_every, check_every, max_iter;
    int32_t layout;
    double eps_rel;
} pmp_params;

typedef struct {
    int64_t iterations;   /* iterations done by this pmp_solve call       */
    double r_norm;        /* ||r||_2 at the last check                     */
    double s_norm;        /* ||s||_2 at the last check                     */
    double eps_tol;       /* eps_abs sqrt(J)                               */
    double rho;           /* current penalty                               */
    pmp_status status;    /* PMP_OK (converged) or PMP_NOT_CONVERGED, ...  */
} pmp_result;

typedef struct pmp_handle pmp_handle;

/* Defaults: rho0 1, alpha 1.6, mu 2, gamma 1.1, eps_abs 1e-4, adapt_every 50,
 * check_every 10, max_iter 100000 (Section III-G's constants), layout AUTO. */
pmp_status pmp_params_default(pmp_params *params);

/* Workspace bytes needed for `problem` (reads only m, n, nnz, dtype) with
 * the layout `params` selects. */
pmp_status pmp_workspace_size(const pmp_problem *problem, const pmp_params *params,
                              size_t *bytes);

/* Validate the problem, copy it into `workspace` (device memory, >= the size
 * above, 256-byte aligned), build the CSC pattern and the block tables on the
 * device and zero the state (a = b = zs = u = 0, rho = rho0: the all-zero
 * start of the ADMM iteration).  Work is queued on `stream` and the call
 * synchronises it before returning.  On success *out owns host resources
 * until pmp_destroy. */
pmp_status pmp_setup(const pmp_problem *problem, const pmp_params *params,
                     void *workspace, size_t workspace_bytes, void *stream,
                     pmp_handle **out);

/* Queue k iterations on the handle's stream (asynchronous).  rho balancing
 * runs at multiples of adapt_every; no stop test.  The last iteration also
 * computes ||r|| and ||s||, read by pmp_residuals. */
pmp_status pmp_iterate(pmp_handle *h, int32_t k);

/* Synchronise and return the residuals of the last check and the iteration
 * count. Any pointer may be NULL. */
pmp_status pmp_residuals(pmp_handle *h, double *r_norm, double *s_norm,
                         int64_t *iteration);

/* Iterate until ||r||, ||s|| < eps_tol at a check iteration (iteration
 * counts that are multiples of check_every) or for max_iter iterations.  Replays a captured hipGraph
 * of check_every iterations; the stop decision and rho balancing stay on the
 * device.  Returns PMP_OK on convergence, PMP_NOT_CONVERGED at max_iter. */
pmp_status pmp_solve(pmp_handle *h, pmp_result *out);

/* Copy the current solution into device buffers of the problem's dtype:
 * x[n] rates, lambda[m] link prices rho u, slack[m] = ps + c.  Any pointer
 * may be NULL.  Queued on the handle's stream; synchronises before return. */
pmp_status pmp_get_solution(pmp_handle *h, void *x, void *lambda, void *slack);

/* Iterate state for warm starts (Section V-D re-solves): a[n], b[m], zs[m],
 * u[m] in the problem's dtype, packed in that order, followed by rho
 * (double) and the iteration count (int64).  Size from pmp_state_size.
 * `state` is device memory. */
pmp_status pmp_state_size(pmp_handle *h, size_t *bytes);
pmp_status pmp_get_state(pmp_handle *h, void *state);
pmp_status pmp_set_state(pmp_handle *h, const void *state);

/* Replace the capacities c[m] (device memory, problem dtype, > 0) keeping the
 * iterate: the warm-started re-solve after degradation of Section V-D. */
pmp_status pmp_update_capacity(pmp_handle *h, const void *c_new);

/* Link failure and pruning (Section V-D).  failed[m] (device, uint8,
 * nonzero = the link failed) removes those links and every stream whose
 * route uses one of them; the survivors are renumbered in their old order
 * and each surviving row keeps its surviving entries in column order.
 * Outputs are device memory sized for the current (unpruned) instance; the
 * first m', n', nnz' entries are written:
 *   row_ptr[m+1], col_idx[nnz]    CSR of the pruned R (int32)
 *   c[m]                          current capacities of the surviving links
 *   w[n], utility[n]              weights (> 0) and codes of the survivors
 *   link_map[m], stream_map[n]    old index of each surviving link / stream
 *   state[pmp_state_size bytes]   the current iterate restricted to the
 *                                 survivors, in the pmp_set_state layout of
 *                                 the pruned instance (rho carried over,
 *                                 iteration count 0): the warm start
 * c, w and state use the problem dtype.  sizes (host) receives m', n', nnz'.
 * `workspace` is device scratch of pmp_prune_workspace_size bytes.  The
 * handle itself is unchanged; the pruned instance is set up with pmp_setup
 * (same lo, hi) and warm-started with pmp_set_state.  m' or n' may be 0
 * (pmp_setup rejects m' = 0).  Synchronises the handle's stream.
 * PMP_ERR_INVALID for a NULL pointer or a short workspace. */
pmp_status pmp_prune_workspace_size(pmp_handle *h, size_t *bytes);
pmp_status pmp_prune(pmp_handle *h, const uint8_t *failed, void *workspace,
                     size_t workspace_bytes, int32_t *row_ptr, int32_t *col_idx, void *c,
                     void *w, uint8_t *utility, int32_t *link_map, int32_t *stream_map,
                     void *state, int64_t *sizes);

/* For callers that cannot allocate device memory (serving loops, code that
 * forbids hipMalloc): pmp_prune with its scratch in a fixed array of 16 MiB
 * that the library keeps on every GPU it runs on until the process ends
 * (its address on the device current at pmp_setup is looked up there).
 * Arguments and results as pmp_prune, without the workspace; it allocates
 * nothing.  PMP_ERR_SHAPE when the instance needs more scratch than the
 * fixed maximum (4 (2n + 2m + 2) bytes plus the scans' block sums: about
 * m + n <= 2e6).  Every call on one GPU uses that GPU's array, so calls that
 * overlap on one GPU (several host threads, or several streams in flight)
 * race; each call writes all of the scratch it reads. */
pmp_status pmp_prune_noalloc(pmp_handle *h, const uint8_t *failed, int32_t *row_ptr,
                             int32_t *col_idx, void *c, void *w, uint8_t *utility,
                             int32_t *link_map, int32_t *stream_map, void *state, int64_t *sizes);

/* Path prices (Section VI-B): pi[n] = sum over the links l of route j of
 * lambda_l = rho u_l, the price stream j pays per unit rate; at the optimum
 * pi_j = U_j'(x_j) for an interior x_j.  pi is device memory of the
 * problem's dtype; the sum is formed in FP64.  Synchronises the handle's
 * stream. */
pmp_status pmp_get_path_prices(pmp_handle *h, void *pi);

/* Device pointers to the internal vectors for zero-copy inspection, in the
 * problem's dtype: x[n] rates, u[m] scaled duals (prices / rho), and the
 * compact iterate a[n], b[m], zs[m], v[m] = b - u.  Valid until pmp_destroy
 * and current whenever the handle's stream has finished the work of the
 * calls made so far (any pointer may be NULL). */
pmp_status pmp_device_views(pmp_handle *h, void **x, void **u, void **a, void **b,
                            void **zs, void **v);

/* Change eps_abs, eps_rel, mu, gamma and max_iter of an existing handle (alpha,
 * check_every and adapt_every are fixed at setup: PMP_ERR_INVALID if they
 * differ).  Synchronises the handle's stream. */
pmp_status pmp_update_params(pmp_handle *h, const pmp_params *params);

/* Residual history: up to `capacity` most recent checks, oldest first, as
 * rows (iteration, ||r||, ||s||, rho) of 4 doubles in host memory `out`
 * (the device keeps the last 4096).  *count receives the rows written. */
pmp_status pmp_history(pmp_handle *h, double *out, int32_t capacity, int32_t *count);

/* Measurement: run k iterations (same schedule as pmp_iterate) launching
 * each pass on its own with HIP events around it on the handle's stream, and
 * return average milliseconds in host ms[4]: stream pass and link pass of
 * the other iterations, stream pass and link pass of check iterations (the
 * latter including the check's finalize kernel and, at balancing
 * iterations, the rescale of u); 0 when none ran. */
pmp_status pmp_time_kernels(pmp_handle *h, int32_t k, double *ms);

/* Replace the weights w[n] (device memory, problem dtype, > 0), keeping each
 * stream's utility type and the iterate. */
pmp_status pmp_update_weights(pmp_handle *h, const void *w_new);

/* ---- reverse mode: gradients of K unrolled iterations ------------------
 * J = sum_j U_j(x_j^K) for the rates x^K of the K-th iteration after the
 * handle's current state, at the current rho (no balancing inside the K
 * iterations).  As K grows its gradients approach the envelope values of
 * the optimal utility U_opt: dU_opt/dc_l = lambda_l and
 * dU_opt/dw_j = log x_j (log utilities), from the KKT relation of
 * Section VI-B.
 * The forward pass keeps the state every s iterations in `adj_workspace`
 * (caller-owned device memory of pmp_adjoint_workspace_size bytes, 256-byte
 * aligned, which must stay valid until pmp_backward); the backward pass
 * recomputes each segment of s iterations, records x and the slack-prox mask,
 * and runs the reverse iteration.  Afterwards the handle holds the state of
 * iteration K again. */
pmp_status pmp_adjoint_workspace_size(pmp_handle *h, int32_t K, int32_t s, size_t *bytes);
/* Run K iterations with checkpoints every s; J (host) receives the objective. */
pmp_status pmp_forward_ckpt(pmp_handle *h, int32_t K, int32_t s, void *adj_workspace,
                            size_t adj_bytes, double *J);
/* dJ/dc[m] and dJ/dw[n] into device buffers of the problem dtype (either may be
 * NULL).  PMP_ERR_STATE without a preceding pmp_forward_ckpt. */
pmp_status pmp_backward(pmp_handle *h, void *grad_c, void *grad_w);

/* ---- batched solves of many uneven instances --------------------------
 * The instances (host memory, one dtype, each with its own box) are
 * concatenated block-diagonally and iterated together by one persistent,
 * graph-captured kernel launch per pmp_batch_solve: every instance keeps its
 * own rho, residuals, stop flag and iteration count (Section III-F/G applied
 * per instance), and stopped instances drop out of the work.  Workgroup tiles
 * never straddle instances; their nonzero limit (tile_cap, in [64, 8192]) is
 * set per instance size class: m < class_m[0], m < class_m[1], larger.
 * With reorder_streams = 1 each instance's streams are renumbered inside the
 * library by the first link of their route (ties by index), which puts the
 * streams of one link close together when routes are local (as in
 * time-expanded transit networks) and so keeps the link gathers in cache;
 * every sum keeps its order, so results are unchanged, and solutions are
 * returned in the caller's numbering. */
typedef struct pmp_batch pmp_batch;
typedef struct {
    int32_t class_m[2];
    int32_t tile_cap[3];
    int32_t reorder_streams;
    int32_t wg_per_cu;      /* resident workgroups per CU in the persistent grid
                               (1..8, capped by occupancy; 0 = 4) */
    int32_t profile;        /* 1: time the kernel's phases (pmp_batch_profile) */
    int32_t heavy_chunk;    /* link rows of more than 4096 nonzeros (congested
                               links, Section V-C) are split into chunks of this
                               many nonzeros, one workgroup each, whose sums are
                               added in chunk order; 0 or [1024, 2^20], 0 = 8192.
                               FP32 instances with a finite box sum these rows
                               in fixed point, so there the results do not depend
                               on it; otherwise 8192 gives the sums of pmp_solve's
                               gather layout */
    int32_t wait_log2;      /* a grid barrier wait gives up after 2^wait_log2
                               polls (0 or [1, 30]; 0 = 24);
                               pmp_batch_solve then returns PMP_ERR_HIP */
} pmp_batch_options;

/* Defaults (tuned on MI355X for transit batches): classes at m = 1e4 and
 * 5e4, tile caps 8192 for every class, reorder_streams 1, wg_per_cu 4,
 * heavy_chunk 8192, wait_log2 24. */
pmp_status pmp_batch_options_default(pmp_batch_options *options);
pmp_status pmp_batch_workspace_size(int32_t count, const pmp_problem *problems,
                                    const pmp_params *params, const pmp_batch_options *options,
                                    size_t *bytes);
/* Validate (on the host) and lay out the instances in `workspace` (device
 * memory, 256-byte aligned); state zero, rho = rho0 for every instance.
 * Synchronises `stream`. */
pmp_status pmp_batch_setup(int32_t count, const pmp_problem *problems, const pmp_params *params,
                           const pmp_batch_options *options, void *workspace,
                           size_t workspace_bytes, void *stream, pmp_batch **out);
/* Run up to max_iter iterations of every instance that has not met the stop
 * rule (checks every check_every iterations and at max_iter), continuing
 * from the current state; results[count] (host) receive each instance's
 * iterations in this call, residuals, rho and status.  Returns PMP_OK when
 * every instance converged, PMP_NOT_CONVERGED otherwise, PMP_ERR_HIP if the
 * kernel's bounded barrier wait expired. */
pmp_status pmp_batch_solve(pmp_batch *b, int32_t max_iter, pmp_result *results);
/* Solution of instance `index` into device buffers x[n_i], lambda[m_i],
 * slack[m_i] (any may be NULL). */
pmp_status pmp_batch_get_solution(pmp_batch *b, int32_t index, void *x, void *lambda,
                                  void *slack);
/* Back to the all-zero start, rho = rho0, for every instance. */
pmp_status pmp_batch_reset(pmp_batch *b);
/* Time of the last pmp_batch_solve's kernel by phase, averaged over its
 * workgroups, in ms (host ms[6]): stream tiles, wait at the grid barrier
 * after them, link tiles, wait after them, check finalize with its barrier,
 * rho rescale with its barrier (device wall clock).  PMP_ERR_STATE unless
 * the batch was set up with options.profile = 1. */
pmp_status pmp_batch_profile(pmp_batch *b, double *ms);
pmp_status pmp_batch_destroy(pmp_batch *b);

/* The layout chosen at setup (PMP_LAYOUT_GATHER or PMP_LAYOUT_BINNED). */
pmp_status pmp_get_layout(pmp_handle *h, int32_t *layout);

pmp_status pmp_destroy(pmp_handle *h);

const char *pmp_status_string(pmp_status s);
const char *pmp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMP_H */
