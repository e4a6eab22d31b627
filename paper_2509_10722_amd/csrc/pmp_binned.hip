// Binned message exchange: the PMP iteration for large, unstructured R.
//
// On a random link-route pattern the gathers of the CSR/CSC passes hit a
// different cache line for nearly every nonzero, and random 4-byte gathers
// from an 80 MB vector run an order of magnitude below streaming bandwidth.
// This layout instead moves one message per nonzero through HBM in
// coalesced runs:
//   R is tiled into P x Q tiles (link block p of LB links, stream block q of
//   SB streams).  mx holds x_j for every nonzero, tile by tile in p-major
//   order; mv holds v_l in q-major order; both list a tile's nonzeros in the
//   same order (CSR order), so entry k of tile (p, q) is the same nonzero in
//   both.
//   stream workgroup q: add its mv entries into FP64 LDS sums by local stream
//     index (six), run the stream epilogue (prox, relaxation), then write
//     x_j into mx tile by tile (one wave per tile).
//   link workgroup p: add its mx entries into FP64 LDS sums by local link
//     index (lix), run the link epilogue (slack prox, average, dual update),
//     then write v_l into mv tile by tile.
// The LDS sums are FP64 atomic adds of FP32 messages; when the addends of one
// sum span less than 2^24 in magnitude every partial sum is exact, so the
// result does not depend on the order of the adds and equals the sequential
// FP64 sum of the CSR/CSC kernels.
#include "pmp_device.h"

#include <algorithm>
#include <vector>

namespace pmp {

BinnedPlan binned_plan(int m, int n)
{
    // A multiple of 256 workgroups (one or more per CU) of at most
    // kBinMaxBlock rows each.
    auto split = [](int count, int &blocks, int &size) {
        const long long per = 256LL * kBinMaxBlock;
        const long long k = std::max<long long>(1, (count + per - 1) / per);
        blocks = (int)(256 * k);
        size = (int)std::max<long long>(1, (count + blocks - 1) / blocks);
        blocks = (int)std::max<long long>(1, (count + size - 1) / size);
    };
    BinnedPlan bp{};
    split(m, bp.P, bp.LB);
    split(n, bp.Q, bp.SB);
    return bp;
}

void binned_build_host(const int *row_ptr, const int *col_idx, int m, int n, const BinnedPlan &bp,
                       long long *ox, long long *ov, uint16_t *lix, uint16_t *six)
{
    const long long P = bp.P, Q = bp.Q;
    std::vector<long long> cnt((size_t)(P * Q), 0);
    for (int l = 0; l < m; ++l) {
        const long long p = l / bp.LB;
        for (int k = row_ptr[l]; k < row_ptr[l + 1]; ++k) cnt[(size_t)(p * Q + col_idx[k] / bp.SB)]++;
    }
    long long acc = 0;
    for (long long p = 0; p < P; ++p)
        for (long long q = 0; q < Q; ++q) {
            ox[p * Q + q] = acc;
            acc += cnt[(size_t)(p * Q + q)];
        }
    ox[P * Q] = acc;
    acc = 0;
    for (long long q = 0; q < Q; ++q)
        for (long long p = 0; p < P; ++p) {
            ov[q * P + p] = acc;
            acc += cnt[(size_t)(p * Q + q)];
        }
    ov[Q * P] = acc;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int l = 0; l < m; ++l) {
        const long long p = l / bp.LB;
        for (int k = row_ptr[l]; k < row_ptr[l + 1]; ++k) {
            const int j = col_idx[k];
            const long long q = j / bp.SB;
            const long long r = cnt[(size_t)(p * Q + q)]++;   // rank in the tile, CSR order
            lix[ox[p * Q + q] + r] = (uint16_t)(l - p * bp.LB);
            six[ov[q * P + p] + r] = (uint16_t)(j - q * bp.SB);
        }
    }
}

namespace {

template <typename T, bool CHECK>
__global__ __launch_bounds__(kBinThreads) void k_bin_stream(Dev<T> d)
{
    if (d.ctl->done) return;
    extern __shared__ double S[];
    __shared__ double sred[kBinThreads / 64];
    const int q = blockIdx.x;
    const int j0 = q * d.SB;
    const int ns = min(d.SB, d.n - j0);
    for (int i = threadIdx.x; i < ns; i += kBinThreads) S[i] = 0.0;
    __syncthreads();
    const long long e0 = d.ov[(long long)q * d.P], e1 = d.ov[(long long)(q + 1) * d.P];
    for (long long e = e0 + threadIdx.x; e < e1; e += kBinThreads)
        unsafeAtomicAdd(&S[d.six[e]], (double)__builtin_nontemporal_load(d.mv + e));
    __syncthreads();
    const double rho = d.ctl->rho;
    double part = 0.0;
    for (int i = threadIdx.x; i < ns; i += kBinThreads) {
        const int j = j0 + i;
        const int L = d.col_ptr[j + 1] - d.col_ptr[j];
        part += stream_update<T, CHECK>(d, j, L, S[i], rho);
        S[i] = (double)d.x[j];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int p = wave; p < d.P; p += kBinThreads / 64) {
        const long long src = d.ov[(long long)q * d.P + p];
        const long long cnt = d.ov[(long long)q * d.P + p + 1] - src;
        const long long dst = d.ox[(long long)p * d.Q + q];
        for (long long k = lane; k < cnt; k += 64) d.mx[dst + k] = (T)S[d.six[src + k]];
    }
    if (CHECK) {
        part = block_sum_n<kBinThreads>(part, sred);
        if (threadIdx.x == 0) d.spart[q] = part;
    }
}

template <typename T>
__device__ __forceinline__ void emit_links(const Dev<T> &d, const double *Y, int p)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = wave; q < d.Q; q += kBinThreads / 64) {
        const long long src = d.ox[(long long)p * d.Q + q];
        const long long cnt = d.ox[(long long)p * d.Q + q + 1] - src;
        const long long dst = d.ov[(long long)q * d.P + p];
        for (long long k = lane; k < cnt; k += 64) d.mv[dst + k] = (T)Y[d.lix[src + k]];
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBinThreads) void k_bin_link(Dev<T> d)
{
    if (d.ctl->done) return;
    extern __shared__ double Y[];
    __shared__ double sred[kBinThreads / 64];
    const int p = blockIdx.x;
    const int l0 = p * d.LB;
    const int nl = min(d.LB, d.m - l0);
    for (int i = threadIdx.x; i < nl; i += kBinThreads) Y[i] = 0.0;
    __syncthreads();
    const long long e0 = d.ox[(long long)p * d.Q], e1 = d.ox[(long long)(p + 1) * d.Q];
    for (long long e = e0 + threadIdx.x; e < e1; e += kBinThreads)
        unsafeAtomicAdd(&Y[d.lix[e]], (double)__builtin_nontemporal_load(d.mx + e));
    __syncthreads();
    double r2 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < nl; i += kBinThreads) {
        const int l = l0 + i;
        link_update<T, MODE>(d, l, d.row_ptr[l + 1] - d.row_ptr[l], Y[i], r2, s2);
        Y[i] = (double)d.v[l];
    }
    if (MODE != kCheck) {
        __syncthreads();
        emit_links<T>(d, Y, p);
    } else {
        // v is emitted by k_bin_emit once the rho decision is known
        r2 = block_sum_n<kBinThreads>(r2, sred);
        s2 = block_sum_n<kBinThreads>(s2, sred);
        if (threadIdx.x == 0) {
            d.lpart[2 * p] = r2;
            d.lpart[2 * p + 1] = s2;
        }
    }
}

// After a check (apply = 1): apply a pending u rescale (eq. (7)), refresh
// v = b - u and write the link messages.  With apply = 0 only the messages
// are rewritten from v.  Runs also after the stop rule fired, so the
// messages always match v.
template <typename T>
__global__ __launch_bounds__(kBinThreads) void k_bin_emit(Dev<T> d, int apply)
{
    extern __shared__ double Y[];
    const int p = blockIdx.x;
    const int l0 = p * d.LB;
    const int nl = min(d.LB, d.m - l0);
    const double ratio = apply ? d.ctl->ratio : 1.0;
    for (int i = threadIdx.x; i < nl; i += kBinThreads) {
        const int l = l0 + i;
        T vt = d.v[l];
        if (ratio != 1.0) {
            const T ut = (T)((double)d.u[l] * ratio);
            d.u[l] = ut;
            vt = (T)((double)d.b[l] - (double)ut);
            d.v[l] = vt;
        }
        Y[i] = (double)vt;
    }
    __syncthreads();
    emit_links<T>(d, Y, p);
}

}  // namespace

void binned_configure()
{
    const int bytes = kBinMaxBlock * (int)sizeof(double);
#define PMP_BIN_ATTR(K) (void)hipFuncSetAttribute((const void *)(K), hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
    PMP_BIN_ATTR((k_bin_stream<float, false>));
    PMP_BIN_ATTR((k_bin_stream<float, true>));
    PMP_BIN_ATTR((k_bin_stream<double, false>));
    PMP_BIN_ATTR((k_bin_stream<double, true>));
    PMP_BIN_ATTR((k_bin_link<float, kPlain>));
    PMP_BIN_ATTR((k_bin_link<float, kSave>));
    PMP_BIN_ATTR((k_bin_link<float, kCheck>));
    PMP_BIN_ATTR((k_bin_link<double, kPlain>));
    PMP_BIN_ATTR((k_bin_link<double, kSave>));
    PMP_BIN_ATTR((k_bin_link<double, kCheck>));
    PMP_BIN_ATTR((k_bin_emit<float>));
    PMP_BIN_ATTR((k_bin_emit<double>));
#undef PMP_BIN_ATTR
}

template <typename T>
void launch_bin_stream(const Dev<T> &d, bool check, hipStream_t s)
{
    const size_t lds = (size_t)d.SB * sizeof(double);
    if (check) hipLaunchKernelGGL((k_bin_stream<T, true>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
    else hipLaunchKernelGGL((k_bin_stream<T, false>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
}

template <typename T>
void launch_bin_link(const Dev<T> &d, int mode, hipStream_t s)
{
    const size_t lds = (size_t)d.LB * sizeof(double);
    switch (mode) {
    case kPlain:
        hipLaunchKernelGGL((k_bin_link<T, kPlain>), dim3(d.P), dim3(kBinThreads), lds, s, d);
        break;
    case kSave:
        hipLaunchKernelGGL((k_bin_link<T, kSave>), dim3(d.P), dim3(kBinThreads), lds, s, d);
        break;
    default:
        hipLaunchKernelGGL((k_bin_link<T, kCheck>), dim3(d.P), dim3(kBinThreads), lds, s, d);
        break;
    }
}

template <typename T>
void launch_bin_emit(const Dev<T> &d, int apply, hipStream_t s)
{
    hipLaunchKernelGGL((k_bin_emit<T>), dim3(d.P), dim3(kBinThreads), (size_t)d.LB * sizeof(double),
                       s, d, apply);
}

template void launch_bin_stream<float>(const Dev<float> &, bool, hipStream_t);
template void launch_bin_stream<double>(const Dev<double> &, bool, hipStream_t);
template void launch_bin_link<float>(const Dev<float> &, int, hipStream_t);
template void launch_bin_link<double>(const Dev<double> &, int, hipStream_t);
template void launch_bin_emit<float>(const Dev<float> &, int, hipStream_t);
template void launch_bin_emit<double>(const Dev<double> &, int, hipStream_t);

}  // namespace pmp
