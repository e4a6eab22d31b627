// HIP kernels of the PMP iteration for gfx950 (CDNA4, wave64).
//
// The two passes of one iteration are segmented gather-sums over the 0/1
// pattern of R with the per-stream / per-link PMP algebra fused into their
// epilogues:
//   stream pass  CSC gather of v  -> S_j -> prox (Section III-E) -> x_j, a_j
//   link pass    CSR gather of x  -> y_l -> slack prox, link average,
//                over-relaxed z / u updates (Section III-G) -> b, zs, u, v
// Workgroups own consecutive segments (<= 256 segments, <= kCap nonzeros):
// all 256 lanes stream the workgroup's index range with coalesced,
// non-temporal loads and issue the gathers together, the gathered values are
// staged in LDS, and then one lane per segment sums its run in FP64 in a
// fixed order (no atomics; results are bitwise reproducible).  A segment
// longer than kCap gets a workgroup of its own that strides over it.
#include "pmp_device.h"

#include <cmath>

namespace pmp {

namespace {

// Workgroups are dealt to the 8 XCDs in turn (block b to XCD b mod 8); block
// b takes segment block xcd_order(b), so that each XCD runs one contiguous
// range of segment blocks and neighbouring blocks gather from one L2 (medium
// shape in this layout 16,280 -> 16,480 it/s, the transit case study +1-2%).
__device__ __forceinline__ int xcd_order(int b, int nblocks)
{
    const int x = b % 8, per = nblocks / 8, rem = nblocks % 8;
    return x * per + min(x, rem) + b / 8;
}

// ---- stream pass ---------------------------------------------------------

template <typename T, bool CHECK>
__global__ __launch_bounds__(kBlock) void k_stream_pass(Dev<T> d)
{
    if (d.ctl->done) return;
    __shared__ T sv[kCap];
    __shared__ double sred[kBlock / 64];
    const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int s0 = d.sblk[blk], s1 = d.sblk[blk + 1];
    const int e0 = d.col_ptr[s0];
    const int cnt = d.col_ptr[s1] - e0;
    const double rho = d.ctl->rho;
    double part = 0.0;
    if (cnt <= kCap) {
        gather_stage<T>(d.row_idx + e0, d.v, sv, cnt);
        __syncthreads();
        const int j = s0 + (int)threadIdx.x;
        if (j < s1) {
            const int b = d.col_ptr[j] - e0, e = d.col_ptr[j + 1] - e0;
            const double acc = run_sum<T>(sv, b, e);
            part = stream_update<T, CHECK>(d, j, e - b, acc, rho);
        }
    } else {
        double acc = 0.0;
        for (int k = threadIdx.x; k < cnt; k += kBlock)
            acc += (double)d.v[ld_stream(d.row_idx + e0 + k)];
        acc = block_sum(acc, sred);
        if (threadIdx.x == 0) part = stream_update<T, CHECK>(d, s0, cnt, acc, rho);
    }
    if (CHECK) {
        part = block_sum(part, sred);
        if (threadIdx.x == 0) d.spart[blk] = part;
    }
}

// ---- link pass -------------------------------------------------------------

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_link_pass(Dev<T> d)
{
    if (d.ctl->done) return;
    __shared__ T sx[kCap];
    __shared__ double sred[kBlock / 64];
    const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
    if (blk >= d.nlb) {
        // one chunk of a long row: a partial sum in a fixed order, or the
        // exact fixed-point sum (kept as int64 bits in rpart)
        const int c = blk - d.nlb;
        if (d.fx_shift) {
            long long acc = 0;
            for (int k = d.lck_beg[c] + threadIdx.x; k < d.lck_end[c]; k += kBlock)
                acc += fx_term((double)d.x[ld_stream(d.col_idx + k)], d.fx_scale);
            acc = block_sum_ll(acc, sred);
            if (threadIdx.x == 0) ((long long *)d.rpart)[c] = acc;
            return;
        }
        double acc = 0.0;
        for (int k = d.lck_beg[c] + threadIdx.x; k < d.lck_end[c]; k += kBlock)
            acc += (double)d.x[ld_stream(d.col_idx + k)];
        acc = block_sum(acc, sred);
        if (threadIdx.x == 0) d.rpart[c] = acc;
        return;
    }
    const int l0 = d.lblk[blk], l1 = d.lblk[blk + 1];
    const int e0 = d.row_ptr[l0];
    const int cnt = d.row_ptr[l1] - e0;
    double r2 = 0.0, s2 = 0.0;
    if (cnt <= kCap) {
        gather_stage<T>(d.col_idx + e0, d.x, sx, cnt);
        __syncthreads();
        const int l = l0 + (int)threadIdx.x;
        if (l < l1) {
            const int b = d.row_ptr[l] - e0, e = d.row_ptr[l + 1] - e0;
            const double acc = run_sum<T>(sx, b, e);
            link_update<T, MODE>(d, l, e - b, acc, r2, s2);
        }
    }
    // a longer row is one of the long rows: its chunks and k_long_rows do it
    if (MODE == kCheck) {
        r2 = block_sum(r2, sred);
        s2 = block_sum(s2, sred);
        if (threadIdx.x == 0) {
            d.lpart[2 * blk] = r2;
            d.lpart[2 * blk + 1] = s2;
        }
    }
}

// Long rows: add each row's chunk sums in chunk order, then the link update.
template <typename T, int MODE>
__global__ void k_long_rows(Dev<T> d)
{
    if (d.ctl->done) return;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < d.nlr; r += gridDim.x * blockDim.x) {
        const int l = d.lr_row[r];
        double y = 0.0;
        if (d.fx_shift) {
            long long t = 0;
            for (int c = d.lr_ck[r]; c < d.lr_ck[r + 1]; ++c) t += ((const long long *)d.rpart)[c];
            y = (double)t * d.fx_inv;
        } else {
            for (int c = d.lr_ck[r]; c < d.lr_ck[r + 1]; ++c) y += d.rpart[c];
        }
        double r2 = 0.0, s2 = 0.0;
        link_update<T, MODE>(d, l, d.row_ptr[l + 1] - d.row_ptr[l], y, r2, s2);
        if (MODE == kCheck) {
            d.lpart[2 * (d.nlb + r)] = r2;
            d.lpart[2 * (d.nlb + r) + 1] = s2;
        }
    }
}

// One workgroup: add the check's partials in a fixed order (each thread a
// fixed stride, then a fixed tree), then the stop rule and rho balancing.
template <typename T>
__global__ __launch_bounds__(kFinThreads) void k_check_finalize(Dev<T> d, int nspart, int nlpart,
                                                                long long delta, int stop)
{
    if (d.ctl->done) return;
    __shared__ double sred[kFinThreads / 64];
    double sr = 0.0, ss = 0.0;
    for (int i = threadIdx.x; i < nlpart; i += kFinThreads) {
        sr += d.lpart[2 * i];
        ss += d.lpart[2 * i + 1];
    }
    for (int i = threadIdx.x; i < nspart; i += kFinThreads) ss += d.spart[i];
    sr = block_sum_n<kFinThreads>(sr, sred);
    ss = block_sum_n<kFinThreads>(ss, sred);
    // norms of p, z, u from the norm pass (relative stop rule only)
    double nrm[3] = {0.0, 0.0, 0.0};
    const bool rel = d.ctl->eps_rel > 0.0;
    if (rel) {
        double q[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            double acc = 0.0;
            for (int i = threadIdx.x; i < kNormBlocks; i += kFinThreads) acc += d.npart[5 * i + k];
            q[k] = block_sum_n<kFinThreads>(acc, sred);
        }
        nrm[0] = q[0] + q[2];   // sum_j L x^2 + sum_l ps^2
        nrm[1] = q[1] + q[3];   // sum_(l,j) (a_j + b_l)^2 + sum_l zs^2
        nrm[2] = q[4];          // sum_l (d + 1) u^2
    }
    if (threadIdx.x == 0) finalize<T>(d, delta, stop, sr, ss, rel ? nrm : nullptr);
}

// Norms of a check for the relative stop rule, per workgroup (partials in
// npart, added in a fixed order by k_check_finalize).  In the compact form a
// traffic terminal (l, j) holds p = x_j and z = a_j + b_l, a slack terminal
// p = ps_l and z = zs_l, every terminal of link l the dual u_l.  With the
// link balance (R a)_l = -(d_l b_l + zs_l) (the z-update keeps each link's
// z summing to zero),
//   sum over traffic terminals of z^2 = sum_j L_j a_j^2 - sum_l (d_l b_l^2 + 2 b_l zs_l),
// so no sum over the nonzeros is needed.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rel_norms(Dev<T> d)
{
    if (d.ctl->done || !(d.ctl->eps_rel > 0.0)) return;
    __shared__ double sred[kBlock / 64];
    double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        const double L = d.rlen ? (double)d.rlen[j] : (double)(d.col_ptr[j + 1] - d.col_ptr[j]);
        const double x = (double)d.x[j], a = (double)d.a[j];
        q[0] += L * x * x;
        q[1] += L * a * a;
    }
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride) {
        const double dg = d.dlen ? (double)d.dlen[l] : (double)(d.row_ptr[l + 1] - d.row_ptr[l]);
        const double ps = d.ps_prev[l], b = (double)d.b[l], zs = (double)d.zs[l];
        const double u = (double)d.u[l];
        q[2] += ps * ps;
        q[3] += zs * zs - dg * b * b - 2.0 * b * zs;
        q[4] += (dg + 1.0) * u * u;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double t = block_sum(q[k], sred);
        if (threadIdx.x == 0) d.npart[5 * blockIdx.x + k] = t;
    }
}

// u <- (rho_old / rho_new) u after a balancing step (eq. (18)); v = b - u.
template <typename T>
__global__ void k_rescale(Dev<T> d)
{
    const double ratio = d.ctl->ratio;
    if (ratio == 1.0) return;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += gridDim.x * blockDim.x) {
        const T ut = (T)((double)d.u[l] * ratio);
        d.u[l] = ut;
        d.v[l] = (T)((double)d.b[l] - (double)ut);
    }
}

template <typename T>
__global__ void k_refresh_v(Dev<T> d)
{
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += gridDim.x * blockDim.x)
        d.v[l] = (T)((double)d.b[l] - (double)d.u[l]);
}

// ---- setup ------------------------------------------------------------------

template <typename T>
__global__ void k_init_state(Dev<T> d, const T *c_in, const T *w_in, const uint8_t *util)
{
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        const T w = w_in[j];
        const_cast<T *>(d.wsig)[j] = util[j] == PMP_UTIL_LINEAR ? -w : w;
        d.a[j] = T(0);
        d.x[j] = T(0);
    }
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride) {
        const_cast<T *>(d.c)[l] = c_in[l];
        d.b[l] = T(0);
        d.zs[l] = T(0);
        d.u[l] = T(0);
        d.v[l] = T(0);
        d.y_prev[l] = 0.0;
        d.ps_prev[l] = 0.0;
    }
}

template <typename T>
__global__ void k_zero_state(Dev<T> d)
{
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        d.a[j] = T(0);
        d.x[j] = T(0);
    }
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride) {
        d.b[l] = T(0);
        d.zs[l] = T(0);
        d.u[l] = T(0);
        d.v[l] = T(0);
        d.y_prev[l] = 0.0;
        d.ps_prev[l] = 0.0;
    }
}

template <typename T>
__global__ void k_check_vectors(const T *c, const T *w, const uint8_t *util, int m, int n,
                                Ctl *ctl)
{
    const int stride = gridDim.x * blockDim.x;
    unsigned f = 0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < m; l += stride) {
        const double v = (double)c[l];
        if (!(v > 0.0) || !isfinite(v)) f |= kErrCap;
    }
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const double v = (double)w[j];
        if (!(v > 0.0) || !isfinite(v)) f |= kErrWeight;
        if (util[j] > 2) f |= kErrUtility;
        if (util[j] == 2) f |= kHasAlpha2;
    }
    if (f) atomicOr(&ctl->flags, f);
}

__global__ void k_validate_csr(const int *row_ptr, const int *col_idx, int m, int n,
                               long long nnz, Ctl *ctl)
{
    const int stride = gridDim.x * blockDim.x;
    unsigned f = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        if (row_ptr[0] != 0 || (long long)row_ptr[m] != nnz) f |= kErrRowPtr;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < m; l += stride) {
        const long long b = row_ptr[l], e = row_ptr[l + 1];
        if (b < 0 || e < b || e > nnz) {
            f |= kErrRowPtr;
            continue;
        }
        int prev = -1;
        for (long long k = b; k < e; ++k) {
            const int j = col_idx[k];
            if (j < 0 || j >= n) f |= kErrColRange;
            else if (j <= prev) f |= kErrColOrder;
            prev = j;
        }
    }
    if (f) atomicOr(&ctl->flags, f);
}

__global__ void k_histogram(const int *col_idx, long long nnz, int *count)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nnz; k += stride)
        atomicAdd(&count[col_idx[k]], 1);
}

constexpr int kScanPer = 8;                      // elements per thread
constexpr int kScanTile = kBlock * kScanPer;     // elements per workgroup

__device__ int block_excl_scan_int(int v, int *sh, int *total)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int incl = sh[threadIdx.x];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int *in, int n, int *bsum)
{
    __shared__ int sh[kBlock];
    const long long base = (long long)blockIdx.x * kScanTile;
    int s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        const long long k = base + i;
        if (k < n) s += in[k];
    }
    int total;
    block_excl_scan_int(s, sh, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_bsums(int *bsum, int nb)
{
    __shared__ int sh[kBlock];
    int carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int ex = block_excl_scan_int(v, sh, &total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

// out[0] = 0, out[k + 1] = in[0] + ... + in[k]
__global__ __launch_bounds__(kBlock) void k_scan_apply(const int *in, int n, const int *boff,
                                                       int *out)
{
    __shared__ int sh[kBlock];
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int v[kScanPer];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const long long k = base + i;
        v[i] = k < n ? in[k] : 0;
        s += v[i];
    }
    int total;
    int run = boff[blockIdx.x] + block_excl_scan_int(s, sh, &total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const long long k = base + i;
        run += v[i];
        if (k < n) out[k + 1] = run;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

__global__ void k_scatter(const int *row_ptr, const int *col_idx, int m, const int *col_ptr,
                          int *fill, int *row_idx)
{
    const int stride = gridDim.x * blockDim.x;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < m; l += stride) {
        for (int k = row_ptr[l]; k < row_ptr[l + 1]; ++k) {
            const int j = col_idx[k];
            row_idx[col_ptr[j] + atomicAdd(&fill[j], 1)] = l;
        }
    }
}

// Sort every column's links ascending (the scatter order is arbitrary).
__global__ void k_sort_columns(const int *col_ptr, int n, int *row_idx)
{
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const int b = col_ptr[j], e = col_ptr[j + 1];
        for (int i = b + 1; i < e; ++i) {
            const int key = row_idx[i];
            int k = i - 1;
            while (k >= b && row_idx[k] > key) {
                row_idx[k + 1] = row_idx[k];
                --k;
            }
            row_idx[k + 1] = key;
        }
    }
}

__global__ void k_check_routes(const int *col_ptr, int n, double hi, Ctl *ctl)
{
    const int stride = gridDim.x * blockDim.x;
    unsigned f = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        if (col_ptr[j + 1] == col_ptr[j] && isinf(hi)) f |= kErrEmptyRoute;
    if (f) atomicOr(&ctl->flags, f);
}

__global__ void k_fill_int(int *p, int value, size_t count)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

__global__ void k_ctl_init(Ctl *c, double rho, double eps_tol, double eps_rel, double mu,
                           double gamma, int adapt_every)
{
    c->rho = rho;
    c->ratio = 1.0;
    c->r_norm = 0.0;
    c->s_norm = 0.0;
    c->eps_tol = eps_tol;
    c->eps_rel = eps_rel;
    c->p_norm = c->z_norm = c->u_norm = 0.0;
    c->mu = mu;
    c->gamma = gamma;
    c->iter = 0;
    c->nhist = 0;
    c->adapt_every = adapt_every;
    c->done = 0;
    c->status = PMP_OK;
    c->arrive = 0u;
    c->flags = 0u;
}

__global__ void k_ctl_set_tolerances(Ctl *c, double eps_tol, double eps_rel, double mu,
                                     double gamma)
{
    c->eps_tol = eps_tol;
    c->eps_rel = eps_rel;
    c->mu = mu;
    c->gamma = gamma;
}

__global__ void k_ctl_clear_done(Ctl *c)
{
    c->done = 0;
    c->status = PMP_OK;
}

__global__ void k_ctl_advance(Ctl *c, long long k) { c->iter += k; }

template <typename T>
__global__ void k_solution(Dev<T> d, T *x, T *lambda, T *slack)
{
    const int stride = gridDim.x * blockDim.x;
    const double rho = d.ctl->rho;
    if (x)
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) x[j] = d.x[j];
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride) {
        if (lambda) lambda[l] = (T)(rho * (double)d.u[l]);
        if (slack) slack[l] = (T)(d.ps_prev[l] + (double)d.c[l]);
    }
}

// pi_j = rho sum_{l in route j} u_l (CSC walk, FP64 sum in route order).
template <typename T>
__global__ void k_path_prices(Dev<T> d, T *pi)
{
    const double rho = d.ctl->rho;
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        double s = 0.0;
        for (int k = d.col_ptr[j]; k < d.col_ptr[j + 1]; ++k) s += (double)d.u[d.row_idx[k]];
        pi[j] = (T)(rho * s);
    }
}

// An update of c or w is checked in full before any of it is applied: the
// check sets its error bit (cleared first), and the copy then returns at once
// when the bit is set, so a rejected update leaves the instance as it was.
__global__ void k_ctl_clear_flags(Ctl *c, unsigned mask) { c->flags &= ~mask; }

template <typename T>
__global__ void k_check_positive(const T *v, int count, Ctl *ctl, unsigned bit)
{
    const int stride = gridDim.x * blockDim.x;
    unsigned f = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const double x = (double)v[i];
        if (!(x > 0.0) || !isfinite(x)) f = bit;
    }
    if (f) atomicOr(&ctl->flags, f);
}

template <typename T>
__global__ void k_copy_capacity(Dev<T> d, const T *c_new)
{
    if (d.ctl->flags & kErrCap) return;
    const int stride = gridDim.x * blockDim.x;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride)
        const_cast<T *>(d.c)[l] = c_new[l];
}

inline int grid_for(long long count, int block = kBlock, int cap = 65536)
{
    long long g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

// ---- launchers -----------------------------------------------------------

template <typename T>
void launch_stream_pass(const Dev<T> &d, bool check, hipStream_t s)
{
    if (d.nsb == 0) return;
    if (check) hipLaunchKernelGGL((k_stream_pass<T, true>), dim3(d.nsb), dim3(kBlock), 0, s, d);
    else hipLaunchKernelGGL((k_stream_pass<T, false>), dim3(d.nsb), dim3(kBlock), 0, s, d);
}

template <typename T>
void launch_link_pass(const Dev<T> &d, int mode, hipStream_t s)
{
    if (d.nlb == 0) return;
    const int grid = d.nlb + d.nlc;
    const int lg = d.nlr > 0 ? (d.nlr + 63) / 64 : 0;
    switch (mode) {
    case kPlain:
        hipLaunchKernelGGL((k_link_pass<T, kPlain>), dim3(grid), dim3(kBlock), 0, s, d);
        if (lg) hipLaunchKernelGGL((k_long_rows<T, kPlain>), dim3(lg), dim3(64), 0, s, d);
        break;
    case kSave:
        hipLaunchKernelGGL((k_link_pass<T, kSave>), dim3(grid), dim3(kBlock), 0, s, d);
        if (lg) hipLaunchKernelGGL((k_long_rows<T, kSave>), dim3(lg), dim3(64), 0, s, d);
        break;
    default:
        hipLaunchKernelGGL((k_link_pass<T, kCheck>), dim3(grid), dim3(kBlock), 0, s, d);
        if (lg) hipLaunchKernelGGL((k_long_rows<T, kCheck>), dim3(lg), dim3(64), 0, s, d);
        break;
    }
}

template <typename T>
void launch_check_finalize(const Dev<T> &d, int nspart, int nlpart, long long delta, int stop,
                           hipStream_t s)
{
    // the norm pass returns at once unless the stop rule has a relative part
    hipLaunchKernelGGL((k_rel_norms<T>), dim3(kNormBlocks), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL((k_check_finalize<T>), dim3(1), dim3(kFinThreads), 0, s, d, nspart, nlpart,
                       delta, stop);
}

template <typename T>
void launch_rescale(const Dev<T> &d, hipStream_t s)
{
    hipLaunchKernelGGL((k_rescale<T>), dim3(grid_for(d.m, kBlock, 4096)), dim3(kBlock), 0, s, d);
}

template <typename T>
void launch_refresh_v(const Dev<T> &d, hipStream_t s)
{
    hipLaunchKernelGGL((k_refresh_v<T>), dim3(grid_for(d.m, kBlock, 4096)), dim3(kBlock), 0, s, d);
}

template <typename T>
void launch_init_state(const Dev<T> &d, const T *c_in, const T *w_in, const uint8_t *util,
                       hipStream_t s)
{
    hipLaunchKernelGGL((k_init_state<T>), dim3(grid_for(d.n > d.m ? d.n : d.m, kBlock, 16384)),
                       dim3(kBlock), 0, s, d, c_in, w_in, util);
}

template <typename T>
void launch_zero_state(const Dev<T> &d, hipStream_t s)
{
    hipLaunchKernelGGL((k_zero_state<T>), dim3(grid_for(d.n > d.m ? d.n : d.m, kBlock, 16384)),
                       dim3(kBlock), 0, s, d);
}

template <typename T>
void launch_check_vectors(const T *c, const T *w, const uint8_t *util, int m, int n, Ctl *ctl,
                          hipStream_t s)
{
    hipLaunchKernelGGL((k_check_vectors<T>), dim3(grid_for(n > m ? n : m, kBlock, 16384)),
                       dim3(kBlock), 0, s, c, w, util, m, n, ctl);
}

template <typename T>
void launch_solution(const Dev<T> &d, T *x, T *lambda, T *slack, hipStream_t s)
{
    hipLaunchKernelGGL((k_solution<T>), dim3(grid_for(d.n > d.m ? d.n : d.m, kBlock, 16384)),
                       dim3(kBlock), 0, s, d, x, lambda, slack);
}

template <typename T>
void launch_check_positive(const T *v, int count, Ctl *ctl, unsigned bit, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_clear_flags, dim3(1), dim3(1), 0, s, ctl, bit);
    if (count > 0)
        hipLaunchKernelGGL((k_check_positive<T>), dim3(grid_for(count, kBlock, 16384)),
                           dim3(kBlock), 0, s, v, count, ctl, bit);
}

template <typename T>
void launch_copy_capacity(const Dev<T> &d, const T *c_new, hipStream_t s)
{
    launch_check_positive<T>(c_new, d.m, d.ctl, kErrCap, s);
    hipLaunchKernelGGL((k_copy_capacity<T>), dim3(grid_for(d.m, kBlock, 16384)), dim3(kBlock), 0,
                       s, d, c_new);
}

template <typename T>
void launch_path_prices(const Dev<T> &d, T *pi, hipStream_t s)
{
    if (d.n == 0) return;
    hipLaunchKernelGGL((k_path_prices<T>), dim3(grid_for(d.n, kBlock, 16384)), dim3(kBlock), 0, s,
                       d, pi);
}

void launch_validate_csr(const int *row_ptr, const int *col_idx, int m, int n, long long nnz,
                         Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(m, kBlock, 16384)), dim3(kBlock), 0, s,
                       row_ptr, col_idx, m, n, nnz, ctl);
}

size_t transpose_scratch_ints(int n)
{
    const size_t nb = ((size_t)n + kScanTile - 1) / kScanTile;
    return (size_t)n + nb + 1;
}

size_t scan_scratch_ints(int n)
{
    return ((size_t)n + kScanTile - 1) / kScanTile + 1;
}

void launch_scan_int(const int *in, int n, int *out, int *bsum, hipStream_t s)
{
    if (n > 0) {
        const int nb = (int)(((long long)n + kScanTile - 1) / kScanTile);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, n, bsum);
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kBlock), 0, s, bsum, nb);
        hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, s, in, n, bsum, out);
    } else {
        launch_fill_int(out, 0, 1, s);
    }
}

void launch_transpose(const int *row_ptr, const int *col_idx, int m, int n, long long nnz,
                      int *col_ptr, int *row_idx, int *tmp, hipStream_t s)
{
    int *count = tmp;
    int *bsum = tmp + n;
    launch_fill_int(count, 0, (size_t)n, s);
    if (nnz > 0)
        hipLaunchKernelGGL(k_histogram, dim3(grid_for(nnz, kBlock, 65536)), dim3(kBlock), 0, s,
                           col_idx, nnz, count);
    launch_scan_int(count, n, col_ptr, bsum, s);
    launch_fill_int(count, 0, (size_t)n, s);
    if (m > 0)
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(m, kBlock, 65536)), dim3(kBlock), 0, s,
                           row_ptr, col_idx, m, col_ptr, count, row_idx);
    if (n > 0)
        hipLaunchKernelGGL(k_sort_columns, dim3(grid_for(n, kBlock, 65536)), dim3(kBlock), 0, s,
                           col_ptr, n, row_idx);
}

void launch_check_routes(const int *col_ptr, int n, double hi, Ctl *ctl, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_check_routes, dim3(grid_for(n, kBlock, 16384)), dim3(kBlock), 0, s,
                       col_ptr, n, hi, ctl);
}

void launch_ctl_init(Ctl *ctl, double rho, double eps_tol, double eps_rel, double mu,
                     double gamma, int adapt_every, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, s, ctl, rho, eps_tol, eps_rel, mu, gamma,
                       adapt_every);
}

void launch_ctl_set_tolerances(Ctl *ctl, double eps_tol, double eps_rel, double mu, double gamma,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_set_tolerances, dim3(1), dim3(1), 0, s, ctl, eps_tol, eps_rel, mu,
                       gamma);
}

void launch_ctl_clear_done(Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_clear_done, dim3(1), dim3(1), 0, s, ctl);
}

void launch_ctl_advance(Ctl *ctl, long long k, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_advance, dim3(1), dim3(1), 0, s, ctl, k);
}

void launch_fill_int(int *p, int value, size_t count, hipStream_t s)
{
    if (count == 0) return;
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for((long long)count, kBlock, 16384)), dim3(kBlock),
                       0, s, p, value, count);
}

#define PMP_INSTANTIATE(T)                                                                  \
    template void launch_stream_pass<T>(const Dev<T> &, bool, hipStream_t);                \
    template void launch_link_pass<T>(const Dev<T> &, int, hipStream_t);                   \
    template void launch_check_finalize<T>(const Dev<T> &, int, int, long long, int,       \
                                           hipStream_t);                                    \
    template void launch_rescale<T>(const Dev<T> &, hipStream_t);                           \
    template void launch_refresh_v<T>(const Dev<T> &, hipStream_t);                         \
    template void launch_zero_state<T>(const Dev<T> &, hipStream_t);                        \
    template void launch_init_state<T>(const Dev<T> &, const T *, const T *,               \
                                       const uint8_t *, hipStream_t);                       \
    template void launch_check_vectors<T>(const T *, const T *, const uint8_t *, int, int, \
                                          Ctl *, hipStream_t);                              \
    template void launch_solution<T>(const Dev<T> &, T *, T *, T *, hipStream_t);           \
    template void launch_check_positive<T>(const T *, int, Ctl *, unsigned, hipStream_t);  \
    template void launch_copy_capacity<T>(const Dev<T> &, const T *, hipStream_t);         \
    template void launch_path_prices<T>(const Dev<T> &, T *, hipStream_t);

PMP_INSTANTIATE(float)
PMP_INSTANTIATE(double)

}  // namespace pmp
