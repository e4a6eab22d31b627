// Link failure (Section V-D): compaction of a resident instance on the device.
//
// A failed link leaves the network together with every stream routed over it
// (its path is broken).  Survivors keep their relative order: link l' of the
// pruned instance is the l'-th surviving link, stream j' the j'-th surviving
// stream, and a surviving row keeps its surviving entries in column order
// (the renumbering of streams is monotone, so the rows stay sorted).  The
// iterate (a, b, zs, u) follows its links and streams, which gives the warm
// start of the re-solve: the old solution restricted to the survivors.
//
// Steps, all on the handle's stream:
//   1. alive[j]  = no link of route j failed            (CSC walk per stream)
//      keep[l]   = link l did not fail
//   2. snew = exclusive scan of alive, lnew = exclusive scan of keep
//      (n' = snew[n], m' = lnew[m]; read back once)
//   3. cnt[l'] = surviving entries of row l           (one wave per row)
//   4. row_ptr' = exclusive scan of cnt
//   5. col_idx' = snew of the surviving entries       (one wave per row,
//      ballot compaction keeps the column order)
//   6. c, w, utility, a, b, zs, u gathered to the new numbering.

#include <algorithm>
#include <mutex>

#include "pmp_internal.h"

// Scratch of pmp_prune_noalloc (the alive / renumbering / scan arrays of the
// steps above), for callers that cannot allocate: a fixed array in device
// memory, one per GPU, held until the process ends.  Host code never uses
// the name of the array as an address: its per-device address comes from
// hipGetSymbolAddress (prune_static_scratch below).
static __device__ __align__(256) int scratch[pmp::kPruneStaticBytes / sizeof(int)];

namespace pmp {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t prune_static_scratch(int device, int **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = (int *)g_scratch_ptr[device];
    return hipSuccess;
}

namespace {

constexpr int kWave = 64;
constexpr int kPruneBlock = 256;

int prune_grid(long long count, int per_block, int cap)
{
    long long g = (count + per_block - 1) / per_block;
    return (int)std::max(1LL, std::min<long long>(g, cap));
}

__global__ void k_alive_streams(const int *col_ptr, const int *row_idx, int n,
                                const uint8_t *failed, int *alive)
{
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        int ok = 1;
        for (int k = col_ptr[j]; k < col_ptr[j + 1]; ++k)
            if (failed[row_idx[k]]) ok = 0;
        alive[j] = ok;
    }
}

__global__ void k_alive_links(const uint8_t *failed, int m, int *keep)
{
    const int stride = gridDim.x * blockDim.x;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < m; l += stride)
        keep[l] = failed[l] ? 0 : 1;
}

__device__ int wave_sum_int(int v)
{
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;
}

// One wave per row: cnt[l'] = surviving entries of surviving row l, and the
// link map l' -> l.
__global__ __launch_bounds__(kPruneBlock) void k_row_counts(const int *row_ptr, const int *col_idx,
                                                            int m, const int *lnew,
                                                            const int *alive, int *cnt,
                                                            int *link_map)
{
    const int lane = threadIdx.x % kWave;
    const int waves = gridDim.x * (kPruneBlock / kWave);
    for (int l = blockIdx.x * (kPruneBlock / kWave) + threadIdx.x / kWave; l < m; l += waves) {
        const int ln = lnew[l];
        if (lnew[l + 1] == ln) continue;               // failed link
        int c = 0;
        for (int k = row_ptr[l] + lane; k < row_ptr[l + 1]; k += kWave) c += alive[col_idx[k]];
        c = wave_sum_int(c);
        if (lane == 0) {
            cnt[ln] = c;
            link_map[ln] = l;
        }
    }
}

// One wave per surviving row: the surviving entries, renumbered, packed in
// column order at row_ptr'[l'].
__global__ __launch_bounds__(kPruneBlock) void k_row_fill(const int *row_ptr, const int *col_idx,
                                                          int m, const int *lnew,
                                                          const int *alive, const int *snew,
                                                          const int *rp_new, int *ci_new)
{
    const int lane = threadIdx.x % kWave;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    const int waves = gridDim.x * (kPruneBlock / kWave);
    for (int l = blockIdx.x * (kPruneBlock / kWave) + threadIdx.x / kWave; l < m; l += waves) {
        const int ln = lnew[l];
        if (lnew[l + 1] == ln) continue;
        int pos = rp_new[ln];
        const int end = row_ptr[l + 1];
        for (int base = row_ptr[l]; base < end; base += kWave) {
            const int k = base + lane;
            const int j = k < end ? col_idx[k] : 0;
            const bool ok = k < end && alive[j] != 0;
            const unsigned long long mask = __ballot(ok);
            if (ok) ci_new[pos + __popcll(mask & below)] = snew[j];
            pos += __popcll(mask);
        }
    }
}

template <typename T>
__global__ void k_prune_links(Dev<T> d, const int *lnew, T *c_out, T *b_out, T *zs_out,
                              T *u_out)
{
    const int stride = gridDim.x * blockDim.x;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.m; l += stride) {
        const int ln = lnew[l];
        if (lnew[l + 1] == ln) continue;
        c_out[ln] = d.c[l];
        b_out[ln] = d.b[l];
        zs_out[ln] = d.zs[l];
        u_out[ln] = d.u[l];
    }
}

// w > 0 again from the signed weight; the utility code from the device copy
// when one is kept (alpha = 2 present), else from the sign (linear: -w).
template <typename T>
__global__ void k_prune_streams(Dev<T> d, const int *snew, T *w_out, uint8_t *util_out,
                                int *stream_map, T *a_out)
{
    const int stride = gridDim.x * blockDim.x;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        const int jn = snew[j];
        if (snew[j + 1] == jn) continue;
        const T ws = d.wsig[j];
        w_out[jn] = ws < T(0) ? -ws : ws;
        util_out[jn] = d.util ? d.util[j]
                              : (uint8_t)(ws < T(0) ? PMP_UTIL_LINEAR : PMP_UTIL_LOG);
        stream_map[jn] = j;
        a_out[jn] = d.a[j];
    }
}

}  // namespace

size_t prune_scratch_ints(int m, int n)
{
    return 2 * (size_t)n + 1 + 2 * (size_t)m + 1 +
           std::max(scan_scratch_ints(n), scan_scratch_ints(m));
}

template <typename T>
hipError_t prune_device(const Dev<T> &d, const uint8_t *failed, int *scratch, int *row_ptr,
                        int *col_idx, T *c, T *w, uint8_t *util, int *link_map, int *stream_map,
                        char *state, long long sizes[3], hipStream_t s)
{
    const int m = d.m, n = d.n;
    int *alive = scratch;                 // [n]
    int *snew = alive + n;                // [n + 1]
    int *keep = snew + n + 1;             // [m], later the row counts
    int *lnew = keep + m;                 // [m + 1]
    int *bsum = lnew + m + 1;
    hipError_t e;

    if (n > 0)
        hipLaunchKernelGGL(k_alive_streams, dim3(prune_grid(n, kPruneBlock, 16384)),
                           dim3(kPruneBlock), 0, s, d.col_ptr, d.row_idx, n, failed, alive);
    if (m > 0)
        hipLaunchKernelGGL(k_alive_links, dim3(prune_grid(m, kPruneBlock, 16384)),
                           dim3(kPruneBlock), 0, s, failed, m, keep);
    launch_scan_int(alive, n, snew, bsum, s);
    launch_scan_int(keep, m, lnew, bsum, s);
    int mn[2];
    if ((e = hipMemcpyAsync(&mn[0], lnew + m, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&mn[1], snew + n, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const int m2 = mn[0], n2 = mn[1];

    int *cnt = keep;                      // keep is no longer needed
    const int wpb = kPruneBlock / kWave;
    if (m > 0)
        hipLaunchKernelGGL(k_row_counts, dim3(prune_grid(m, wpb, 16384)), dim3(kPruneBlock), 0, s,
                           d.row_ptr, d.col_idx, m, lnew, alive, cnt, link_map);
    launch_scan_int(cnt, m2, row_ptr, bsum, s);
    if (m > 0)
        hipLaunchKernelGGL(k_row_fill, dim3(prune_grid(m, wpb, 16384)), dim3(kPruneBlock), 0, s,
                           d.row_ptr, d.col_idx, m, lnew, alive, snew, row_ptr, col_idx);

    // State of the pruned instance: a[n'] b[m'] zs[m'] u[m'] rho iter.
    const size_t sz = sizeof(T);
    T *a_out = (T *)state;
    T *b_out = (T *)(state + (size_t)n2 * sz);
    T *zs_out = (T *)(state + ((size_t)n2 + m2) * sz);
    T *u_out = (T *)(state + ((size_t)n2 + 2 * (size_t)m2) * sz);
    char *tail = state + ((size_t)n2 + 3 * (size_t)m2) * sz;
    if (m > 0)
        hipLaunchKernelGGL((k_prune_links<T>), dim3(prune_grid(m, kPruneBlock, 16384)),
                           dim3(kPruneBlock), 0, s, d, lnew, c, b_out, zs_out, u_out);
    if (n > 0)
        hipLaunchKernelGGL((k_prune_streams<T>), dim3(prune_grid(n, kPruneBlock, 16384)),
                           dim3(kPruneBlock), 0, s, d, snew, w, util, stream_map, a_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const long long zero = 0;
    int nnz2 = 0;
    if ((e = hipMemcpyAsync(tail, &d.ctl->rho, 8, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(tail + 8, &zero, 8, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&nnz2, row_ptr + m2, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    sizes[0] = m2;
    sizes[1] = n2;
    sizes[2] = nnz2;
    return hipSuccess;
}

template hipError_t prune_device<float>(const Dev<float> &, const uint8_t *, int *, int *, int *,
                                        float *, float *, uint8_t *, int *, int *, char *,
                                        long long[3], hipStream_t);
template hipError_t prune_device<double>(const Dev<double> &, const uint8_t *, int *, int *, int *,
                                         double *, double *, uint8_t *, int *, int *, char *,
                                         long long[3], hipStream_t);

}  // namespace pmp
