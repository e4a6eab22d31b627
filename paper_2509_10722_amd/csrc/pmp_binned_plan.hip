// Set-up of the binned layout: the blocking of links and streams (host) and
// the tile tables (offsets and local indices) built from the CSR pattern, on
// the device, or on the host when the stream blocks are too many for one
// workgroup's LDS counters.  The kernels that use the tables are in
// pmp_binned.hip.
#include "pmp_internal.h"

#include <algorithm>
#include <thread>
#include <vector>

namespace pmp {

namespace {

// Count-based blocking: a multiple of 256 blocks (at least `groups` x 256,
// one or more per CU) of at most kBinMaxBlock rows each.
void split_by_count(int count, int groups, int &blocks, int &size)
{
    const long long per = 256LL * kBinMaxBlock;
    const long long k = std::max<long long>(groups, (count + per - 1) / per);
    blocks = (int)(256 * k);
    size = (int)std::max<long long>(1, (count + blocks - 1) / blocks);
    blocks = (int)std::max<long long>(1, (count + size - 1) / size);
}

// Blocks of both sides.  A side with fewer than 512 blocks (one workgroup
// per CU) gets twice as many when the tiles keep at least 64 nonzeros on
// average, so that two workgroups share each CU: measured on MI355X, +9% to
// +13% at 2.5e7 to 6e7 nonzeros, while at 5e6 nonzeros the smaller tiles
// cost more than the second workgroup gains.
void count_blocks(int m, int n, long long nnz, int &p0, int &lb0, int &q0, int &sb0)
{
    split_by_count(m, 1, p0, lb0);
    split_by_count(n, 1, q0, sb0);
    if (p0 < 512 && m >= 512 && nnz >= 64LL * 2 * p0 * q0) split_by_count(m, 2, p0, lb0);
    if (q0 < 512 && n >= 512 && nnz >= 64LL * p0 * 2 * q0) split_by_count(n, 2, q0, sb0);
}

// Row cap of a balanced block: a quarter above the count-based size, within
// kBinMaxBlock.
int row_cap(int size) { return std::min(kBinMaxBlock, size + (size + 3) / 4); }

// Close a block once it holds `quota` nonzeros or `cap` rows.  Blocks closed
// by the quota number at most nnz / quota, blocks closed by the cap at most
// count / cap, so there are at most blocks0 + count / cap + 1 of them.
int cut_blocks(const int *ptr, int count, long long nnz, int blocks0, int cap, int *starts,
               int &most)
{
    const long long quota = std::max<long long>(1, (nnz + blocks0 - 1) / blocks0);
    int nb = 0, s = 0;
    most = 0;
    starts[0] = 0;
    for (int i = 1; i <= count; ++i)
        if (i == count || i - s >= cap || (long long)ptr[i] - ptr[s] >= quota) {
            starts[++nb] = i;
            most = std::max(most, i - s);
            s = i;
        }
    return nb;
}

}  // namespace

BinnedPlan binned_plan(int m, int n, long long nnz)
{
    BinnedPlan bp{};
    int p0, lb0, q0, sb0;
    count_blocks(m, n, nnz, p0, lb0, q0, sb0);
    bp.LB = row_cap(lb0);
    bp.P = p0 + (m + bp.LB - 1) / bp.LB + 1;
    bp.SB = sb0;
    bp.Q = q0;
    return bp;
}

void binned_blocks(const int *row_ptr, int m, int n, long long nnz, BinnedPlan &bp, int *lbs,
                   int *sbs)
{
    int p0, lb0, q0, sb0;
    count_blocks(m, n, nnz, p0, lb0, q0, sb0);
    // links: balanced by nonzeros (a congested link has thousands)
    bp.P = cut_blocks(row_ptr, m, nnz, p0, row_cap(lb0), lbs, bp.LB);
    // streams: by count (routes are short), so the block of stream j is j / SB
    bp.Q = q0;
    bp.SB = sb0;
    for (int q = 0; q <= q0; ++q) sbs[q] = (int)std::min<long long>((long long)q * sb0, n);
}

void binned_build_host(const int *row_ptr, const int *col_idx, int m, int n, const BinnedPlan &bp,
                       const int *lbs, const int *sbs, int *ox, int *ov, uint16_t *lix,
                       uint16_t *six, int mark_long)
{
    const long long P = bp.P, Q = bp.Q;
    (void)m;
    (void)n;
    // Link block p touches only tiles (p, *) and their slots, so the counting
    // and the placing passes split over link blocks across host threads.
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto over_blocks = [&](auto &&body) {
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t)
            pool.emplace_back([&, t] {
                for (long long p = t; p < P; p += nth) body(p);
            });
        for (auto &th : pool) th.join();
    };
    std::vector<int> cnt((size_t)(P * Q), 0);
    over_blocks([&](long long p) {
        int *c = cnt.data() + p * Q;
        for (int l = lbs[p]; l < lbs[p + 1]; ++l)
            for (int k = row_ptr[l]; k < row_ptr[l + 1]; ++k) c[col_idx[k] / bp.SB]++;
    });
    long long acc = 0;   // < nnz < 2^31
    for (long long p = 0; p < P; ++p)
        for (long long q = 0; q < Q; ++q) {
            ox[p * Q + q] = (int)acc;
            acc += cnt[(size_t)(p * Q + q)];
        }
    ox[P * Q] = (int)acc;
    acc = 0;
    for (long long q = 0; q < Q; ++q)
        for (long long p = 0; p < P; ++p) {
            ov[q * P + p] = (int)acc;
            acc += cnt[(size_t)(p * Q + q)];
        }
    ov[Q * P] = (int)acc;
    over_blocks([&](long long p) {
        int *c = cnt.data() + p * Q;
        std::fill(c, c + Q, 0);
        for (int l = lbs[p]; l < lbs[p + 1]; ++l) {
            const uint16_t tag = mark_long && row_ptr[l + 1] - row_ptr[l] > kCap ? kLongBit : 0;
            for (int k = row_ptr[l]; k < row_ptr[l + 1]; ++k) {
                const int j = col_idx[k];
                const long long q = j / bp.SB;
                const int r = c[q]++;   // rank in the tile, CSR order
                lix[ox[p * Q + q] + r] = (uint16_t)((l - lbs[p]) | tag);
                six[ov[q * P + p] + r] = (uint16_t)(j - sbs[q]);
            }
        }
    });
}

namespace {

constexpr int kBuildThreads = 1024;

// cnt[p Q + q] = nonzeros of link block p in stream block q (LDS counters).
__global__ __launch_bounds__(kBuildThreads) void k_tile_count(const int *row_ptr,
                                                              const int *col_idx,
                                                              const int *lbs, int Q, int SB,
                                                              int *cnt)
{
    extern __shared__ int c[];
    const int p = blockIdx.x;
    for (int i = threadIdx.x; i < Q; i += kBuildThreads) c[i] = 0;
    __syncthreads();
    const int e0 = row_ptr[lbs[p]], e1 = row_ptr[lbs[p + 1]];
    for (int e = e0 + threadIdx.x; e < e1; e += kBuildThreads) atomicAdd(&c[col_idx[e] / SB], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < Q; i += kBuildThreads) cnt[(long long)p * Q + i] = c[i];
}

// out[c R + r] = in[r C + c] for a table of R rows of C.
__global__ void k_transpose_int(const int *in, int R, int C, int *out)
{
    const long long n = (long long)R * C;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[(i % C) * R + i / C] = in[i];
}

// Local indices.  Link block p gives each of its links to one lane; a row's
// run of nonzeros inside stream block q reserves a contiguous slot range of
// tile (p, q) with an LDS counter and fills the same ranks of the tile in
// both orders, so entry k of a tile is one nonzero in both and the nonzeros
// of one link stay together (the link pass merges such runs).
__global__ __launch_bounds__(kBuildThreads) void k_tile_place(const int *row_ptr,
                                                              const int *col_idx,
                                                              const int *lbs, int P, int Q,
                                                              int SB, const int *ox,
                                                              const int *ov, uint16_t *lix,
                                                              uint16_t *six, int mark_long)
{
    extern __shared__ int fill[];
    const int p = blockIdx.x;
    for (int i = threadIdx.x; i < Q; i += kBuildThreads) fill[i] = 0;
    __syncthreads();
    const int l0 = lbs[p], l1 = lbs[p + 1];
    for (int l = l0 + (int)threadIdx.x; l < l1; l += kBuildThreads) {
        const int end = row_ptr[l + 1];
        int e = row_ptr[l];
        const uint16_t tag = mark_long && end - e > kCap ? kLongBit : 0;
        while (e < end) {
            const int q = col_idx[e] / SB;
            int r = e + 1;
            while (r < end && col_idx[r] / SB == q) ++r;
            const int base = atomicAdd(&fill[q], r - e);
            const int xo = ox[(long long)p * Q + q] + base;
            const int vo = ov[(long long)q * P + p] + base;
            for (int k = e; k < r; ++k) {
                lix[xo + (k - e)] = (uint16_t)((l - l0) | tag);
                six[vo + (k - e)] = (uint16_t)(col_idx[k] - q * SB);
            }
            e = r;
        }
    }
}

}  // namespace

bool binned_device_build_fits(const BinnedPlan &bp)
{
    return (size_t)bp.Q * sizeof(int) <= kBinBuildLds;
}

size_t binned_build_scratch_ints(const BinnedPlan &bp)
{
    return scan_scratch_ints(bp.P * bp.Q);
}

void binned_build_device(const int *row_ptr, const int *col_idx, const BinnedPlan &bp,
                         const int *lbs, int *ox, int *ov, int *oxq, int *ovp, uint16_t *lix,
                         uint16_t *six, int *scratch, int mark_long, hipStream_t s)
{
    const int P = bp.P, Q = bp.Q, PQ = bp.P * bp.Q;
    const size_t lds = (size_t)Q * sizeof(int);
    const int grid = (int)std::min<long long>(65536, ((long long)PQ + 255) / 256);
    // counts p-major (in oxq for now), scanned into ox; q-major (in ovp),
    // scanned into ov
    hipLaunchKernelGGL(k_tile_count, dim3(P), dim3(kBuildThreads), lds, s, row_ptr, col_idx, lbs,
                       Q, bp.SB, oxq);
    launch_scan_int(oxq, PQ, ox, scratch, s);
    hipLaunchKernelGGL(k_transpose_int, dim3(grid), dim3(256), 0, s, oxq, P, Q, ovp);
    launch_scan_int(ovp, PQ, ov, scratch, s);
    hipLaunchKernelGGL(k_tile_place, dim3(P), dim3(kBuildThreads), lds, s, row_ptr, col_idx, lbs,
                       P, Q, bp.SB, ox, ov, lix, six, mark_long);
    // each side's destination offsets in its own block order
    hipLaunchKernelGGL(k_transpose_int, dim3(grid), dim3(256), 0, s, ox, P, Q, oxq);
    hipLaunchKernelGGL(k_transpose_int, dim3(grid), dim3(256), 0, s, ov, Q, P, ovp);
}

}  // namespace pmp
