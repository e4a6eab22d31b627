// Reverse mode of K unrolled PMP iterations at fixed rho.
//
// The objective is J = sum_j U_j(x_j^K) (the utilities at the rates
// of the K-th iteration).  With A, B, Z, U the adjoints of the compact state
// (a, b, zs, u) and mu_l = [zs_l - u_l > -c_l] the slack-prox mask, one
// forward iteration t reverses as
//   link step    pbb = alpha (U - B - Z);  psb = alpha Z + pbb / (d + 1)
//                ybar = pbb / (d + 1);     cbar -= (1 - mu) psb
//                B <- (1 - alpha) B;  Z <- (1 - alpha) Z + mu psb;
//                U <- U - mu psb
//   stream step  xbar = alpha A + R^T ybar (+ dJ/dx at t = K)
//                Sbar = xbar dP/dS, wbar += xbar dP/dw when lo < x < hi
//                A <- (1 - alpha) A + L Sbar
//   link gather  vbar = R Sbar;  B <- B + vbar;  U <- U - vbar
// where P is the log or linear prox of Section III-E.  For the log prox,
// rho L x^2 - rho S x - w = 0 gives sqrt(S^2 + 4wL/rho) = L x + w/(rho x), so
// dP/dS = rho x^2 / (rho L x^2 + w) and dP/dw = x / (rho L x^2 + w) follow
// from the recorded rate alone; the linear prox has dP/dS = 1/L and
// dP/dw = 1/(rho L).  The link gather of iteration t is fused with the link
// step of iteration t - 1.  The per-stream and per-link steps
// (adj_stream_step, adj_link_step) are in pmp_device.h, shared with the
// binned layout's reverse kernels in pmp_binned.hip.
#include "pmp_device.h"

#include <cmath>

namespace pmp {

namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_stream(Dev<T> d, AdjDev a, const T *xt, int last)
{
    __shared__ double sy[kCap];
    __shared__ double sred[kBlock / 64];
    const int blk = blockIdx.x;
    const int s0 = d.sblk[blk], s1 = d.sblk[blk + 1];
    const int e0 = d.col_ptr[s0];
    const int cnt = d.col_ptr[s1] - e0;
    const double rho = d.ctl->rho;
    if (cnt <= kCap) {
        gather_stage<double>(d.row_idx + e0, a.ybar, sy, cnt);
        __syncthreads();
        const int j = s0 + (int)threadIdx.x;
        if (j < s1) {
            const int b = d.col_ptr[j] - e0, e = d.col_ptr[j + 1] - e0;
            adj_stream_step<T>(d, a, xt, j, e - b, run_sum<double>(sy, b, e), last, rho);
        }
    } else {
        double acc = 0.0;
        for (int k = threadIdx.x; k < cnt; k += kBlock)
            acc += a.ybar[__builtin_nontemporal_load(d.row_idx + e0 + k)];
        acc = block_sum(acc, sred);
        if (threadIdx.x == 0) adj_stream_step<T>(d, a, xt, s0, cnt, acc, last, rho);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_link(Dev<T> d, AdjDev a, const uint8_t *mu_prev)
{
    __shared__ double ss[kCap];
    __shared__ double sred[kBlock / 64];
    const int blk = blockIdx.x;
    const int l0 = d.lblk[blk], l1 = d.lblk[blk + 1];
    const int e0 = d.row_ptr[l0];
    const int cnt = d.row_ptr[l1] - e0;
    int l = -1, deg = 0;
    double acc = 0.0;
    if (cnt <= kCap) {
        gather_stage<double>(d.col_idx + e0, a.Sbar, ss, cnt);
        __syncthreads();
        if (l0 + (int)threadIdx.x < l1) {
            l = l0 + (int)threadIdx.x;
            const int b = d.row_ptr[l] - e0, e = d.row_ptr[l + 1] - e0;
            acc = run_sum<double>(ss, b, e);
            deg = e - b;
        }
    } else {
        for (int k = threadIdx.x; k < cnt; k += kBlock)
            acc += a.Sbar[__builtin_nontemporal_load(d.col_idx + e0 + k)];
        acc = block_sum(acc, sred);
        if (threadIdx.x == 0) {
            l = l0;
            deg = cnt;
        }
    }
    if (l >= 0) {
        a.B[l] += acc;
        a.U[l] -= acc;
        if (mu_prev) adj_link_step(a, l, deg, d.alpha, mu_prev[l]);
    }
}

template <typename T>
__global__ void k_adj_link_only(Dev<T> d, AdjDev a, const uint8_t *mu)
{
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += gridDim.x * blockDim.x)
        adj_link_step(a, l, d.row_ptr[l + 1] - d.row_ptr[l], d.alpha, mu[l]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_objective(Dev<T> d, double *part)
{
    __shared__ double sred[kBlock / 64];
    double acc = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
        const double x = (double)d.x[j], ws = (double)d.wsig[j];
        if (d.util && d.util[j] == PMP_UTIL_ALPHA2) acc += -ws / x;
        else acc += ws > 0.0 ? ws * log(x) : -ws * x;
    }
    acc = block_sum(acc, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double *part, int count, double *out)
{
    __shared__ double sred[kBlock / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) acc += part[i];
    acc = block_sum(acc, sred);
    if (threadIdx.x == 0) *out = acc;
}

template <typename T>
__global__ void k_adj_init(Dev<T> d, AdjDev a)
{
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        const double x = (double)d.x[j], ws = (double)d.wsig[j];
        // dJ/dw_j (direct) and dJ/dx_j^K
        if (d.util && d.util[j] == PMP_UTIL_ALPHA2) {
            a.wbar[j] = -1.0 / x;
            a.ext[j] = ws / (x * x);
        } else {
            a.wbar[j] = ws > 0.0 ? log(x) : x;
            a.ext[j] = ws > 0.0 ? ws / x : -ws;
        }
        a.A[j] = 0.0;
        a.Sbar[j] = 0.0;
    }
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride) {
        a.B[l] = 0.0;
        a.Z[l] = 0.0;
        a.U[l] = 0.0;
        a.ybar[l] = 0.0;
        a.cbar[l] = 0.0;
    }
}

template <typename T>
__global__ void k_adj_out(Dev<T> d, AdjDev a, T *gc, T *gw)
{
    const int stride = gridDim.x * blockDim.x;
    if (gw)
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride)
            gw[j] = (T)a.wbar[j];
    if (gc)
        for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride)
            gc[l] = (T)a.cbar[l];
}

// Applied only when launch_check_positive found every new weight valid (the
// utility type, kept in the sign of the stored weight, is preserved).
template <typename T>
__global__ void k_copy_weights(Dev<T> d, const T *w_new)
{
    if (d.ctl->flags & kErrWeight) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) {
        const T w = w_new[j];
        T *ws = const_cast<T *>(d.wsig);
        ws[j] = (double)ws[j] > 0.0 ? w : (T)(-w);
    }
}

inline int grid_of(long long count, int cap = 16384)
{
    long long g = (count + kBlock - 1) / kBlock;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

template <typename T>
void launch_adj_stream(const Dev<T> &d, const AdjDev &a, const T *xt, int last, hipStream_t s)
{
    if (d.nsb) hipLaunchKernelGGL((k_adj_stream<T>), dim3(d.nsb), dim3(kBlock), 0, s, d, a, xt, last);
}

template <typename T>
void launch_adj_link(const Dev<T> &d, const AdjDev &a, const uint8_t *mu_prev, hipStream_t s)
{
    if (d.nlb) hipLaunchKernelGGL((k_adj_link<T>), dim3(d.nlb), dim3(kBlock), 0, s, d, a, mu_prev);
}

template <typename T>
void launch_adj_link_only(const Dev<T> &d, const AdjDev &a, const uint8_t *mu, hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_link_only<T>), dim3(grid_of(d.m)), dim3(kBlock), 0, s, d, a, mu);
}


template <typename T>
void launch_objective(const Dev<T> &d, double *part, int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_objective<T>), dim3(nblocks), dim3(kBlock), 0, s, d, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, part, nblocks, out);
}

template <typename T>
void launch_adj_init(const Dev<T> &d, const AdjDev &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_init<T>), dim3(grid_of(d.n > d.m ? d.n : d.m)), dim3(kBlock), 0, s,
                       d, a);
}

template <typename T>
void launch_adj_out(const Dev<T> &d, const AdjDev &a, T *gc, T *gw, hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_out<T>), dim3(grid_of(d.n > d.m ? d.n : d.m)), dim3(kBlock), 0, s,
                       d, a, gc, gw);
}

template <typename T>
void launch_copy_weights(const Dev<T> &d, const T *w_new, hipStream_t s)
{
    launch_check_positive<T>(w_new, d.n, d.ctl, kErrWeight, s);
    hipLaunchKernelGGL((k_copy_weights<T>), dim3(grid_of(d.n)), dim3(kBlock), 0, s, d, w_new);
}

#define PMP_ADJ_INSTANTIATE(T)                                                                \
    template void launch_adj_stream<T>(const Dev<T> &, const AdjDev &, const T *, int,       \
                                       hipStream_t);                                         \
    template void launch_adj_link<T>(const Dev<T> &, const AdjDev &, const uint8_t *,        \
                                     hipStream_t);                                           \
    template void launch_adj_link_only<T>(const Dev<T> &, const AdjDev &, const uint8_t *,   \
                                          hipStream_t);                                      \
    template void launch_objective<T>(const Dev<T> &, double *, int, double *, hipStream_t); \
    template void launch_adj_init<T>(const Dev<T> &, const AdjDev &, hipStream_t);           \
    template void launch_adj_out<T>(const Dev<T> &, const AdjDev &, T *, T *, hipStream_t);  \
    template void launch_copy_weights<T>(const Dev<T> &, const T *, hipStream_t);

PMP_ADJ_INSTANTIATE(float)
PMP_ADJ_INSTANTIATE(double)

}  // namespace pmp
