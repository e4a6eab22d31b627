// Batched PMP: many uneven NUM instances in one persistent launch.
//
// The instances are concatenated block-diagonally (links and streams of each
// instance kept together, indices global), so the stream and link passes of
// all instances are the same segmented gather-sums as for one instance.  A
// persistent kernel (grid sized to what the GPU holds at once) walks the
// iterations: in each phase the workgroups of one XCD share a contiguous
// eighth of the phase's tile list (xcd_tiles), skipping tiles of instances
// that have stopped, and a grid barrier separates the phases.  Check
// iterations add a finalize phase
// (workgroup i reduces instance i's tile partials in a fixed order and takes
// its stop and rho decisions, Section III-F/G) and, at balancing iterations,
// a rescale phase.  Tiles never straddle two instances; their size limit is
// chosen per instance size class (see pmp_batch_options).
//
// Every barrier wait is bounded: a workgroup that waits too long sets an
// abort flag and all workgroups leave the kernel, which then reports
// PMP_ERR_HIP instead of hanging.
#include "pmp_device.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace pmp {

namespace {

// A barrier wait polls at most 2^wait_log2 times (2^24 by default), then
// sets the abort flag.
constexpr int kWaitLog2Default = 24;

// Threads per workgroup of the batch kernel: 512, twice the passes' kBlock,
// so that the grid barriers have half as many participants for the same
// lanes on the GPU (64-instance transit solve 1.377 -> 1.356 s).  Long rows
// and columns are still summed by the first kBlock lanes in the stride of the
// single-instance kernels, so their sums stay the same bit for bit.
constexpr int kBT = 2 * kBlock;
// Nonzeros a tile stages in LDS (the largest tile_cap): twice the passes'
// kCap, for the twice as many lanes (16 gathers in flight per lane, as there).
// Rows and columns longer than kCap still go their own way (chunk tiles,
// strided sums), as in the single-instance kernels.  64-instance transit
// solve: 1.35 s with 4096-nonzero tiles of at most 512 streams, 1.29 s with
// 8192, 1.20 s with 8192 and 1,024 streams (2,048 streams: 1.21 s; 16384-
// nonzero tiles: 1.80 s).
constexpr int kBS = 2 * kCap;

// Grid barrier in two levels.  Blocks are dealt to the 8 XCDs in turn, so
// the blocks with one value of blockIdx.x mod 8 (one XCD) first meet on their
// group's counter; the last of each group arrives at the top counter, and the
// last of those advances the generation that the others wait on.  Every
// counter and flag sits on a 256-byte line of its own (waiting blocks poll
// the generation while others add to the counters).  Each block makes its
// writes visible with one release fence before it arrives and takes the
// others' with one acquire fence after the wait (each an L2 writeback or
// invalidate on this GPU); the last arrivals of a group and of the top pass
// the writes they have taken on with an acquire-release fence.  Measured with
// 512 workgroups: about 9.5 us a barrier, against 26 us for one counter
// shared with the generation word and sequentially consistent fences on both
// sides.
constexpr int kBarTop = 0, kBarGen = 64, kBarAbort = 128, kBarGroup = 192;
constexpr int kBarWords = kBarGroup + 64 * 8;   // unsigned words of BDev::bar

// Blocks of barrier group x (blockIdx.x mod 8 == x) in a grid of nblocks,
// and the number of groups.
__host__ __device__ __forceinline__ unsigned barrier_group_size(unsigned x, unsigned nblocks)
{
    return nblocks / 8 + (x < nblocks % 8 ? 1u : 0u);
}
__host__ __device__ __forceinline__ unsigned barrier_groups(unsigned nblocks)
{
    return nblocks < 8 ? nblocks : 8u;
}

__device__ bool grid_sync(unsigned *bar, int *abort, unsigned nblocks, unsigned long long spin_limit)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned *top = bar + kBarTop, *genp = bar + kBarGen;
        const unsigned x = blockIdx.x % 8;
        unsigned *grp = bar + kBarGroup + 64 * x;
        const unsigned gsize = barrier_group_size(x, nblocks);
        const unsigned groups = barrier_groups(nblocks);
        const unsigned gen = __hip_atomic_load(genp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool last = false;
        if (atomicAdd(grp, 1u) == gsize - 1) {
            __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            if (atomicAdd(top, 1u) == groups - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_fetch_add(genp, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (!last) {
            unsigned long long spins = 0;
            while (__hip_atomic_load(genp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > spin_limit ||
                    __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    atomicExch(abort, 1);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok && !__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return s_ok != 0;
}

template <typename T>
__device__ __forceinline__ Dev<T> instance_view(const BDev<T> &d, int inst)
{
    Dev<T> di = d.g;
    di.lo = d.lo[inst];
    di.hi = d.hi[inst];
    di.ctl = &d.ictl[inst];
    di.hist = d.hist + (size_t)inst * kHist;
    return di;
}

template <typename T, bool CHECK>
__device__ void stream_tile(const BDev<T> &d, int tile, T *sv, double *sred)
{
    const int inst = d.st_inst[tile];
    if (d.ictl[inst].done) return;
    const Dev<T> di = instance_view(d, inst);
    const int s0 = d.st_seg[tile], s1 = d.st_seg[tile + 1];
    const int e0 = di.col_ptr[s0];
    const int cnt = di.col_ptr[s1] - e0;
    const double rho = d.ictl[inst].rho;
    double part = 0.0;
    if (cnt <= kBS && !(s1 - s0 == 1 && cnt > kCap)) {
        gather_stage<T, kBT, kBS>(di.row_idx + e0, di.v, sv, cnt);
        __syncthreads();
        for (int j = s0 + (int)threadIdx.x; j < s1; j += kBT) {
            const int b = di.col_ptr[j] - e0, e = di.col_ptr[j + 1] - e0;
            const double acc = run_sum<T>(sv, b, e);
            part += stream_update<T, CHECK>(di, j, e - b, acc, rho);
        }
    } else {
        // the first kBlock lanes in the single-instance order
        double acc = 0.0;
        if (threadIdx.x < kBlock)
            for (int k = threadIdx.x; k < cnt; k += kBlock)
                acc += (double)di.v[ld_stream(di.row_idx + e0 + k)];
        acc = block_sum_n<kBT>(acc, sred);
        if (threadIdx.x == 0) part = stream_update<T, CHECK>(di, s0, cnt, acc, rho);
    }
    if (CHECK) {
        part = block_sum_n<kBT>(part, sred);
        if (threadIdx.x == 0) d.st_part[tile] = part;
    }
    __syncthreads();   // sv is reused by the next tile
}

// Chunk k of the nch chunks of a long link row (a congested link): its sum
// over heavy_chunk nonzeros (strided over the first kBlock lanes, then a
// fixed tree;
// in fixed point where the instance's long rows are), published in lt_hsum.
// The workgroup that makes the row's last arrival adds the row's chunk sums
// in chunk order and runs the link update; that order and these chunks are
// those of the single-instance gather layout, so the row comes out the same
// as there.  Returns (in thread 0) whether this workgroup updated the link.
template <typename T, int MODE>
__device__ bool link_chunk(const BDev<T> &d, const Dev<T> &di, int inst, int tile, int k, int nch,
                           double *sred, double &r2, double &s2)
{
    const int l = d.lt_seg[tile];
    const int rb = di.row_ptr[l], re = di.row_ptr[l + 1];
    const int cb = rb + k * d.heavy_chunk;
    const int ce = cb + min(re - cb, d.heavy_chunk);
    const int fx = d.ifx_shift[inst];
    long long bits;
    if (fx) {
        const double sc = d.ifx_scale[inst];
        long long acc = 0;
        if (threadIdx.x < kBlock)
            for (int e = cb + (int)threadIdx.x; e < ce; e += kBlock)
                acc += fx_term((double)di.x[ld_stream(di.col_idx + e)], sc);
        bits = block_sum_ll<kBT>(acc, sred);
    } else {
        // the first kBlock lanes in the single-instance order
        double acc = 0.0;
        if (threadIdx.x < kBlock)
            for (int e = cb + (int)threadIdx.x; e < ce; e += kBlock)
                acc += (double)di.x[ld_stream(di.col_idx + e)];
        bits = __double_as_longlong(block_sum_n<kBT>(acc, sred));
    }
    bool last = false;
    if (threadIdx.x == 0) {
        const int t0 = tile - k;
        last = true;
        if (nch > 1) {
            // release before the arrival, acquire only in the last arrival
            // (each an L2 writeback or invalidate on this GPU)
            __hip_atomic_store(&d.lt_hsum[tile], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            last = atomicAdd(&d.lt_hcnt[t0], 1u) == (unsigned)(nch - 1);
            if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (last) {
            double y = 0.0;
            if (fx) {
                long long t = 0;
                for (int q = 0; q < nch; ++q)
                    t += q == k ? bits
                                : __hip_atomic_load(&d.lt_hsum[t0 + q], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                y = (double)t * d.ifx_inv[inst];
            } else {
                for (int q = 0; q < nch; ++q)
                    y += __longlong_as_double(q == k ? bits
                                                     : __hip_atomic_load(&d.lt_hsum[t0 + q], __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT));
            }
            // the next iteration's arrivals come after two grid barriers
            if (nch > 1) __hip_atomic_store(&d.lt_hcnt[t0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            link_update<T, MODE>(di, l, re - rb, y, r2, s2);
        }
    }
    return last;
}

template <typename T, int MODE>
__device__ void link_tile(const BDev<T> &d, int tile, T *sx, double *sred)
{
    const int inst = d.lt_inst[tile];
    if (d.ictl[inst].done) return;
    const Dev<T> di = instance_view(d, inst);
    const int2 ck = d.lt_ck[tile];
    double r2 = 0.0, s2 = 0.0;
    bool last = false;
    if (ck.y > 0) {
        last = link_chunk<T, MODE>(d, di, inst, tile, ck.x, ck.y, sred, r2, s2);
    } else {
        // at most kCap nonzeros: rows longer than that are chunk tiles
        const int l0 = d.lt_seg[tile], l1 = d.lt_seg[tile + 1];
        const int e0 = di.row_ptr[l0];
        const int cnt = di.row_ptr[l1] - e0;
        gather_stage<T, kBT, kBS>(di.col_idx + e0, di.x, sx, cnt);
        __syncthreads();
        const int l = l0 + (int)threadIdx.x;
        if (l < l1) {
            const int b = di.row_ptr[l] - e0, e = di.row_ptr[l + 1] - e0;
            const double acc = run_sum<T>(sx, b, e);
            link_update<T, MODE>(di, l, e - b, acc, r2, s2);
        }
    }
    if (MODE == kCheck) {
        r2 = block_sum_n<kBT>(r2, sred);
        s2 = block_sum_n<kBT>(s2, sred);
        if (threadIdx.x == 0) {
            if (ck.y == 0) {
                d.lt_part[2 * tile] = r2;
                d.lt_part[2 * tile + 1] = s2;
            } else {
                // a long row's norms go to its first chunk tile, whichever
                // workgroup updated it, so the check adds them in a fixed
                // order; the other chunk tiles hold zeros
                if (ck.x > 0) {
                    d.lt_part[2 * tile] = 0.0;
                    d.lt_part[2 * tile + 1] = 0.0;
                }
                if (last) {
                    d.lt_part[2 * (tile - ck.x)] = r2;
                    d.lt_part[2 * (tile - ck.x) + 1] = s2;
                }
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int find_instance(const int *off, int B, int idx)
{
    int lo = 0, hi = B;   // off[lo] <= idx < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= idx) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The tiles of a phase [0, count) dealt to the grid: the blocks with one
// value of blockIdx.x mod X (X = min(G, 8); one XCD, as the hardware deals
// blocks to XCDs in turn) take one contiguous eighth of the tile list, in
// turn.  Neighbouring tiles (mostly of one instance) then share an L2:
// 1.39 s against 1.41 s for the 64-instance transit solve with the tiles dealt
// to all blocks in turn.
struct TileRange {
    int t, end, step;
};
__host__ __device__ __forceinline__ TileRange xcd_tiles_of(int count, unsigned G, unsigned b)
{
    const int X = (int)(G < 8u ? G : 8u);
    const int x = (int)b % X, i = (int)b / X;
    const int gx = (int)G / X + (x < (int)G % X ? 1 : 0);
    const int per = count / X, rem = count % X;
    const int t0 = x * per + (x < rem ? x : rem);
    return TileRange{t0 + i, t0 + per + (x < rem ? 1 : 0), gx};
}
__device__ __forceinline__ TileRange xcd_tiles(int count, unsigned G)
{
    return xcd_tiles_of(count, G, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kBT) void k_batch(BDev<T> d, int max_iter, int ce, int adapt)
{
    __shared__ T sv[kBS];
    __shared__ double sred[kBT / 64];
    const unsigned G = gridDim.x;
    // phase clocks (profile only): thread 0 adds each phase's duration
    unsigned long long ph[kBatchPhases] = {};
    unsigned long long tmark = d.prof ? wall_clock64() : 0;
    auto lap = [&](int phase) {
        if (d.prof && threadIdx.x == 0) {
            const unsigned long long now = wall_clock64();
            ph[phase] += now - tmark;
            tmark = now;
        }
    };
    // a solve call continues every instance from its current state; the
    // long rows' arrival counters start at zero (a launch that left through
    // an expired barrier wait may have left counts behind)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.B; i += G * blockDim.x)
        d.ictl[i].done = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < d.nlt; t += G * blockDim.x)
        d.lt_hcnt[t] = 0;
    if (!grid_sync(d.bar, d.abort, G, d.spin_limit)) return;
    long long last_check = 0;
    for (int it = 1; it <= max_iter; ++it) {
        const bool check = it % ce == 0 || it == max_iter;
        const bool save = !check && ((it + 1) % ce == 0 || it + 1 == max_iter);
        lap(5);
        for (TileRange r = xcd_tiles(d.nst, G); r.t < r.end; r.t += r.step) {
            if (check) stream_tile<T, true>(d, r.t, sv, sred);
            else stream_tile<T, false>(d, r.t, sv, sred);
        }
        lap(0);
        if (!grid_sync(d.bar, d.abort, G, d.spin_limit)) return;
        lap(1);
        for (TileRange r = xcd_tiles(d.nlt, G); r.t < r.end; r.t += r.step) {
            if (check) link_tile<T, kCheck>(d, r.t, sv, sred);
            else if (save) link_tile<T, kSave>(d, r.t, sv, sred);
            else link_tile<T, kPlain>(d, r.t, sv, sred);
        }
        lap(2);
        if (!grid_sync(d.bar, d.abort, G, d.spin_limit)) return;
        lap(3);
        if (!check) continue;
        // finalize: one workgroup per instance, partials in tile order
        const long long delta = it - last_check;
        last_check = it;
        for (int i = blockIdx.x; i < d.B; i += G) {
            if (d.ictl[i].done) continue;
            double ss = 0.0, sr = 0.0, sl = 0.0;
            for (int t = d.inst_st[i] + threadIdx.x; t < d.inst_st[i + 1]; t += kBT)
                ss += d.st_part[t];
            for (int t = d.inst_lt[i] + threadIdx.x; t < d.inst_lt[i + 1]; t += kBT) {
                sr += d.lt_part[2 * t];
                sl += d.lt_part[2 * t + 1];
            }
            ss = block_sum_n<kBT>(ss, sred);
            sr = block_sum_n<kBT>(sr, sred);
            sl = block_sum_n<kBT>(sl, sred);
            if (threadIdx.x == 0) finalize<T>(instance_view(d, i), delta, 1, sr, ss + sl);
            __syncthreads();
        }
        if (!grid_sync(d.bar, d.abort, G, d.spin_limit)) return;
        lap(4);
        int active = 0;
        bool rescale = false;
        for (int i = 0; i < d.B; ++i) {
            active += d.ictl[i].done ? 0 : 1;
            rescale |= d.ictl[i].ratio != 1.0;
        }
        if (active == 0) break;   // every workgroup sees the same flags
        // where this check changed rho: u <- (rho_old / rho_new) u (eq. (18));
        // finalize leaves ratio = 1 otherwise
        if (adapt > 0 && rescale) {
            for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < d.g.m; l += G * blockDim.x) {
                const double r = d.ictl[find_instance(d.link_off, d.B, l)].ratio;
                if (r != 1.0) {
                    const T ut = (T)((double)d.g.u[l] * r);
                    d.g.u[l] = ut;
                    d.g.v[l] = (T)((double)d.g.b[l] - (double)ut);
                }
            }
            if (!grid_sync(d.bar, d.abort, G, d.spin_limit)) return;
        }
    }
    lap(5);
    if (d.prof && threadIdx.x == 0)
        for (int k = 0; k < kBatchPhases; ++k) d.prof[(size_t)blockIdx.x * kBatchPhases + k] = ph[k];
}

}  // namespace

namespace {
template <typename T>
__global__ void k_gather_x(const T *x, const int *pos, int n, T *out)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        out[j] = x[pos[j]];
}
}  // namespace

template <typename T>
void launch_batch_gather_x(const T *x, const int *pos, int n, T *out, hipStream_t s)
{
    if (n <= 0) return;
    const int g = std::min(16384, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_gather_x<T>), dim3(g), dim3(kBlock), 0, s, x, pos, n, out);
}

template <typename T>
void launch_batch(const BDev<T> &d, int grid, int max_iter, int check_every, int adapt_every,
                  hipStream_t s)
{
    hipLaunchKernelGGL((k_batch<T>), dim3(grid), dim3(kBT), 0, s, d, max_iter, check_every,
                       adapt_every);
}

template <typename T>
int batch_grid_size(int device, int want_per_cu)
{
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch<T>, kBT, 0) !=
        hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    // a few resident workgroups per CU: enough to cover latency, few enough to
    // keep the grid barriers short (tunable)
    return std::min(per_cu, want_per_cu > 0 ? want_per_cu : 4) * cus;
}

template void launch_batch_gather_x<float>(const float *, const int *, int, float *, hipStream_t);
template void launch_batch_gather_x<double>(const double *, const int *, int, double *, hipStream_t);
template void launch_batch<float>(const BDev<float> &, int, int, int, int, hipStream_t);
template void launch_batch<double>(const BDev<double> &, int, int, int, int, hipStream_t);
template int batch_grid_size<float>(int, int);
template int batch_grid_size<double>(int, int);


// ---- host side ----------------------------------------------------------------

namespace {

#define BATCH_TRY(expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_error(PMP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlignB = 256;
size_t align_b(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

struct BatchSizes {
    long long M = 0, N = 0, NNZ = 0;
    int B = 0;
};

struct BatchLayout {
    size_t row_ptr, col_idx, col_ptr, row_idx, c, wsig, a, x, b, zs, u, v, y_prev, ps_prev;
    size_t link_off, stream_off, lo, hi, ictl, hist, st_seg, st_inst, lt_seg, lt_inst;
    size_t inst_st, inst_lt, st_part, lt_part, lt_ck, lt_hsum, lt_hcnt, ifx_shift, ifx_scale;
    size_t ifx_inv, bar, util, sperm, prof, total;
    long long nst_max, nlt_max;
};

BatchLayout batch_plan(const BatchSizes &z, size_t sz, int min_cap, int heavy_chunk)
{
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_b(off + std::max<size_t>(bytes, 1));
        return o;
    };
    L.nst_max = z.N / kBlock + 2 * z.NNZ / min_cap + 2LL * z.B + 2;
    // chunk tiles of long rows: at most nnz / heavy_chunk + (long rows) more
    L.nlt_max = z.M / kBlock + 2 * z.NNZ / min_cap + 2LL * z.B + 2 + z.NNZ / heavy_chunk +
                z.NNZ / kCap + 1;
    const size_t M = (size_t)z.M, N = (size_t)z.N, E = (size_t)z.NNZ, B = (size_t)z.B;
    L.row_ptr = take((M + 1) * 4);
    L.col_idx = take(E * 4);
    L.col_ptr = take((N + 1) * 4);
    L.row_idx = take(E * 4);
    L.c = take(M * sz);
    L.wsig = take(N * sz);
    L.a = take(std::max(N * sz, transpose_scratch_ints((int)N) * 4));
    L.x = take(N * sz);
    L.b = take(M * sz);
    L.zs = take(M * sz);
    L.u = take(M * sz);
    L.v = take(M * sz);
    L.y_prev = take(M * 8);
    L.ps_prev = take(M * 8);
    L.link_off = take((B + 1) * 4);
    L.stream_off = take((B + 1) * 4);
    L.lo = take(B * 8);
    L.hi = take(B * 8);
    L.ictl = take(B * sizeof(Ctl));
    L.hist = take(B * kHist * sizeof(HistEntry));
    L.st_seg = take(((size_t)L.nst_max + 1) * 4);
    L.st_inst = take((size_t)L.nst_max * 4);
    L.lt_seg = take(((size_t)L.nlt_max + 1) * 4);
    L.lt_inst = take((size_t)L.nlt_max * 4);
    L.inst_st = take((B + 1) * 4);
    L.inst_lt = take((B + 1) * 4);
    L.st_part = take((size_t)L.nst_max * 8);
    L.lt_part = take((size_t)L.nlt_max * 16);
    L.lt_ck = take((size_t)L.nlt_max * sizeof(int2));
    L.lt_hsum = take((size_t)L.nlt_max * 8);
    L.lt_hcnt = take((size_t)L.nlt_max * 4);
    L.ifx_shift = take(B * 4);
    L.ifx_scale = take(B * 8);
    L.ifx_inv = take(B * 8);
    L.bar = take((size_t)kBarWords * 4);
    L.util = take(N);
    L.sperm = take(N * 4);
    L.prof = take((size_t)kBatchMaxGrid * kBatchPhases * 8);
    L.total = off;
    return L;
}

bool sizes_of(int count, const pmp_problem *pr, BatchSizes &z)
{
    z = BatchSizes{};
    z.B = count;
    for (int i = 0; i < count; ++i) {
        if (pr[i].m < 1 || pr[i].n < 0 || pr[i].nnz < 0) return false;
        z.M += pr[i].m;
        z.N += pr[i].n;
        z.NNZ += pr[i].nnz;
    }
    return z.M < (1LL << 31) && z.N < (1LL << 31) && z.NNZ < (1LL << 31);
}

// Streams per stream tile: up to 1,024, two per lane of the 512.  Short
// routes (transit trips of 2-12 links) fill a tile of 256 streams to only
// about 1,800 nonzeros (with 256-lane workgroups and 4096-nonzero tiles, 512
// streams per tile took the solve from 1.50 to 1.41 s).
constexpr int kStreamSegs = 4 * kBlock;

int heavy_chunk_of(const pmp_batch_options *o) { return o->heavy_chunk > 0 ? o->heavy_chunk : kLongChunk; }

int class_cap(const pmp_batch_options *o, int m)
{
    const int c = m < o->class_m[0] ? 0 : (m < o->class_m[1] ? 1 : 2);
    return o->tile_cap[c];
}

// Greedy tiles over segments [first, last) of one instance: at most seg_cap
// segments and `cap` nonzeros each (a longer segment, or one of more than
// kCap nonzeros, alone).  With `ck`
// (link rows), a row longer than kCap becomes ceil(len / chunk) chunk tiles
// that all start at that row.
void tiles_for(const std::vector<int> &ptr, int first, int last, int cap, int inst,
               std::vector<int> &seg, std::vector<int> &owner, int chunk = 0,
               std::vector<int2> *ck = nullptr, int seg_cap = kBlock)
{
    int s = first;
    while (s < last) {
        const long long len = ptr[s + 1] - ptr[s];
        if (ck && len > kCap) {
            const int nch = (int)((len + chunk - 1) / chunk);
            for (int k = 0; k < nch; ++k) {
                seg.push_back(k + 1 < nch ? s : s + 1);
                owner.push_back(inst);
                ck->push_back(make_int2(k, nch));
            }
            ++s;
            continue;
        }
        if (ck) ck->push_back(make_int2(0, 0));
        int e = s;
        long long cnt = 0;
        while (e < last && e - s < seg_cap && ptr[e + 1] - ptr[e] <= kCap &&
               cnt + (ptr[e + 1] - ptr[e]) <= cap) {
            cnt += ptr[e + 1] - ptr[e];
            ++e;
        }
        if (e == s) e = s + 1;
        seg.push_back(e);
        owner.push_back(inst);
        s = e;
    }
}

pmp_status validate_host(const pmp_problem &p, int i)
{
    if (p.memory != PMP_MEM_HOST) return set_error(PMP_ERR_INVALID, "batch instance %d: host memory required", i);
    if (!(p.lo >= 0.0) || !std::isfinite(p.lo) || !(p.hi > p.lo))
        return set_error(PMP_ERR_INVALID, "batch instance %d: box must satisfy 0 <= lo < hi", i);
    if (p.row_ptr[0] != 0 || p.row_ptr[p.m] != p.nnz)
        return set_error(PMP_ERR_INVALID, "batch instance %d: row_ptr must run from 0 to nnz", i);
    std::vector<int> deg((size_t)p.n, 0);
    for (int l = 0; l < p.m; ++l) {
        if (p.row_ptr[l + 1] < p.row_ptr[l]) return set_error(PMP_ERR_INVALID, "batch instance %d: row_ptr decreases", i);
        int prev = -1;
        for (int k = p.row_ptr[l]; k < p.row_ptr[l + 1]; ++k) {
            const int j = p.col_idx[k];
            if (j < 0 || j >= p.n) return set_error(PMP_ERR_INVALID, "batch instance %d: col_idx out of range", i);
            if (j <= prev) return set_error(PMP_ERR_INVALID, "batch instance %d: col_idx not strictly increasing in a row", i);
            prev = j;
            deg[(size_t)j]++;
        }
    }
    const size_t sz = p.dtype == PMP_F64 ? 8 : 4;
    for (int l = 0; l < p.m; ++l) {
        const double c = sz == 8 ? ((const double *)p.c)[l] : ((const float *)p.c)[l];
        if (!(c > 0.0) || !std::isfinite(c)) return set_error(PMP_ERR_INVALID, "batch instance %d: capacities must be finite and > 0", i);
    }
    for (int j = 0; j < p.n; ++j) {
        const double w = sz == 8 ? ((const double *)p.w)[j] : ((const float *)p.w)[j];
        if (!(w > 0.0) || !std::isfinite(w)) return set_error(PMP_ERR_INVALID, "batch instance %d: weights must be finite and > 0", i);
        if (p.utility[j] > 2) return set_error(PMP_ERR_INVALID, "batch instance %d: utility must be 0, 1 or 2", i);
        if (deg[(size_t)j] == 0 && std::isinf(p.hi))
            return set_error(PMP_ERR_INVALID, "batch instance %d: a stream with an empty route needs a finite hi", i);
    }
    return PMP_OK;
}

}  // namespace

}  // namespace pmp

using namespace pmp;

struct pmp_batch {
    int B = 0;
    pmp_dtype dtype = PMP_F32;
    pmp_params prm{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    BDev<float> bf{};
    BDev<double> bd{};
    std::vector<int> m, n, link_off, stream_off;
    std::vector<long long> nnz, iter_base;
    std::vector<double> eps_tol;
    int grid = 0;
    int *sperm = nullptr;   // device: internal position of each caller stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_iters = -1;
    bool profile = false;
};

namespace {

template <typename T>
BDev<T> &bdev_of(pmp_batch *b);
template <>
BDev<float> &bdev_of<float>(pmp_batch *b) { return b->bf; }
template <>
BDev<double> &bdev_of<double>(pmp_batch *b) { return b->bd; }

template <typename T>
pmp_status batch_init_ctl(pmp_batch *b)
{
    BDev<T> &d = bdev_of<T>(b);
    std::vector<Ctl> h((size_t)b->B);
    for (int i = 0; i < b->B; ++i) {
        Ctl &c = h[(size_t)i];
        std::memset(&c, 0, sizeof c);
        c.rho = b->prm.rho0;
        c.ratio = 1.0;
        c.eps_tol = b->eps_tol[(size_t)i];
        c.mu = b->prm.mu;
        c.gamma = b->prm.gamma;
        c.adapt_every = b->prm.adapt_every;
        c.status = PMP_OK;
    }
    BATCH_TRY(hipMemcpyAsync(d.ictl, h.data(), sizeof(Ctl) * h.size(), hipMemcpyHostToDevice, b->stream));
    std::fill(b->iter_base.begin(), b->iter_base.end(), 0);
    return PMP_OK;
}

template <typename T>
pmp_status batch_setup_impl(pmp_batch *b, const pmp_problem *pr, const pmp_batch_options *opt,
                            char *ws, const BatchSizes &z)
{
    const int min_cap = std::min(opt->tile_cap[0], std::min(opt->tile_cap[1], opt->tile_cap[2]));
    const int chunk = heavy_chunk_of(opt);
    const BatchLayout L = batch_plan(z, sizeof(T), min_cap, chunk);
    hipStream_t s = b->stream;
    BDev<T> &d = bdev_of<T>(b);
    Dev<T> &g = d.g;
    const int M = (int)z.M, N = (int)z.N, B = z.B;
    const long long E = z.NNZ;
    // concatenated host arrays (global indices)
    std::vector<int> row_ptr((size_t)M + 1), col_idx((size_t)E);
    std::vector<T> c((size_t)M), w((size_t)N);
    std::vector<uint8_t> util((size_t)N);
    std::vector<double> lo((size_t)B), hi((size_t)B);
    b->link_off.assign((size_t)B + 1, 0);
    b->stream_off.assign((size_t)B + 1, 0);
    std::vector<int> sperm((size_t)N);   // internal position of each caller stream
    long long eo = 0;
    for (int i = 0; i < B; ++i) {
        const pmp_problem &p = pr[i];
        const int lo_l = b->link_off[(size_t)i], lo_s = b->stream_off[(size_t)i];
        // stream order: by the first link of the route, then by index
        std::vector<int> newpos((size_t)p.n);
        if (opt->reorder_streams) {
            std::vector<int> first((size_t)p.n, p.m);
            for (int l = p.m - 1; l >= 0; --l)
                for (int k = p.row_ptr[l]; k < p.row_ptr[l + 1]; ++k) first[(size_t)p.col_idx[k]] = l;
            std::vector<int> order((size_t)p.n);
            for (int j = 0; j < p.n; ++j) order[(size_t)j] = j;
            std::stable_sort(order.begin(), order.end(),
                             [&](int x, int y) { return first[(size_t)x] < first[(size_t)y]; });
            for (int r = 0; r < p.n; ++r) newpos[(size_t)order[(size_t)r]] = r;
        } else {
            for (int j = 0; j < p.n; ++j) newpos[(size_t)j] = j;
        }
        for (int l = 0; l < p.m; ++l) {
            row_ptr[(size_t)lo_l + l] = (int)(eo + p.row_ptr[l]);
            c[(size_t)lo_l + l] = ((const T *)p.c)[l];
        }
        // entries keep their order inside each row, so every sum is unchanged
        for (long long k = 0; k < p.nnz; ++k)
            col_idx[(size_t)(eo + k)] = newpos[(size_t)p.col_idx[k]] + lo_s;
        for (int j = 0; j < p.n; ++j) {
            const size_t t = (size_t)lo_s + newpos[(size_t)j];
            w[t] = ((const T *)p.w)[j];
            util[t] = p.utility[j];
            sperm[(size_t)lo_s + j] = newpos[(size_t)j];
        }
        lo[(size_t)i] = p.lo;
        hi[(size_t)i] = p.hi;
        eo += p.nnz;
        b->link_off[(size_t)i + 1] = lo_l + p.m;
        b->stream_off[(size_t)i + 1] = lo_s + p.n;
    }
    row_ptr[(size_t)M] = (int)E;
    // device views
    g = Dev<T>{};
    g.m = M;
    g.n = N;
    g.nnz = E;
    g.row_ptr = (int *)(ws + L.row_ptr);
    g.col_idx = (int *)(ws + L.col_idx);
    g.col_ptr = (int *)(ws + L.col_ptr);
    g.row_idx = (int *)(ws + L.row_idx);
    g.c = (T *)(ws + L.c);
    g.wsig = (T *)(ws + L.wsig);
    g.a = (T *)(ws + L.a);
    g.x = (T *)(ws + L.x);
    g.b = (T *)(ws + L.b);
    g.zs = (T *)(ws + L.zs);
    g.u = (T *)(ws + L.u);
    g.v = (T *)(ws + L.v);
    g.y_prev = (double *)(ws + L.y_prev);
    g.ps_prev = (double *)(ws + L.ps_prev);
    g.alpha = b->prm.alpha;
    d.B = B;
    d.link_off = (int *)(ws + L.link_off);
    d.stream_off = (int *)(ws + L.stream_off);
    d.lo = (double *)(ws + L.lo);
    d.hi = (double *)(ws + L.hi);
    d.ictl = (Ctl *)(ws + L.ictl);
    d.hist = (HistEntry *)(ws + L.hist);
    d.st_seg = (int *)(ws + L.st_seg);
    d.st_inst = (int *)(ws + L.st_inst);
    d.lt_seg = (int *)(ws + L.lt_seg);
    d.lt_inst = (int *)(ws + L.lt_inst);
    d.inst_st = (int *)(ws + L.inst_st);
    d.inst_lt = (int *)(ws + L.inst_lt);
    d.st_part = (double *)(ws + L.st_part);
    d.lt_part = (double *)(ws + L.lt_part);
    d.lt_ck = (const int2 *)(ws + L.lt_ck);
    d.lt_hsum = (long long *)(ws + L.lt_hsum);
    d.lt_hcnt = (unsigned *)(ws + L.lt_hcnt);
    d.heavy_chunk = chunk;
    d.spin_limit = 1ull << (opt->wait_log2 > 0 ? opt->wait_log2 : kWaitLog2Default);
    d.ifx_shift = (const int *)(ws + L.ifx_shift);
    d.ifx_scale = (const double *)(ws + L.ifx_scale);
    d.ifx_inv = (const double *)(ws + L.ifx_inv);
    d.bar = (unsigned *)(ws + L.bar);
    d.abort = (int *)(d.bar + kBarAbort);
    d.prof = opt->profile ? (unsigned long long *)(ws + L.prof) : nullptr;
    BATCH_TRY(hipMemcpyAsync((void *)g.row_ptr, row_ptr.data(), row_ptr.size() * 4, hipMemcpyHostToDevice, s));
    if (E) BATCH_TRY(hipMemcpyAsync((void *)g.col_idx, col_idx.data(), (size_t)E * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)g.c, c.data(), c.size() * sizeof(T), hipMemcpyHostToDevice, s));
    if (N) BATCH_TRY(hipMemcpyAsync((void *)g.wsig, w.data(), w.size() * sizeof(T), hipMemcpyHostToDevice, s));
    if (N) BATCH_TRY(hipMemcpyAsync(ws + L.util, util.data(), util.size(), hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.link_off, b->link_off.data(), ((size_t)B + 1) * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.stream_off, b->stream_off.data(), ((size_t)B + 1) * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.lo, lo.data(), (size_t)B * 8, hipMemcpyHostToDevice, s));
    b->sperm = (int *)(ws + L.sperm);
    if (N) BATCH_TRY(hipMemcpyAsync(b->sperm, sperm.data(), (size_t)N * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.hi, hi.data(), (size_t)B * 8, hipMemcpyHostToDevice, s));
    launch_transpose(g.row_ptr, g.col_idx, M, N, E, (int *)g.col_ptr, (int *)g.row_idx, (int *)(ws + L.a), s);
    launch_init_state<T>(g, g.c, g.wsig, (const uint8_t *)(ws + L.util), s);
    g.util = std::any_of(util.begin(), util.end(), [](uint8_t u) { return u == PMP_UTIL_ALPHA2; })
                 ? (const uint8_t *)(ws + L.util)
                 : nullptr;
    launch_fill_int((int *)d.bar, 0, kBarWords, s);
    BATCH_TRY(hipGetLastError());
    std::vector<int> col_ptr((size_t)N + 1);
    BATCH_TRY(hipMemcpyAsync(col_ptr.data(), g.col_ptr, col_ptr.size() * 4, hipMemcpyDeviceToHost, s));
    BATCH_TRY(hipStreamSynchronize(s));
    // tiles per instance, sized by the instance's class; long link rows in
    // chunk tiles, summed in fixed point as in the single-instance layouts
    std::vector<int> st_seg{0}, st_inst, lt_seg{0}, lt_inst, inst_st{0}, inst_lt{0};
    std::vector<int2> lt_ck;
    std::vector<int> fx_shift((size_t)B);
    std::vector<double> fx_scale((size_t)B), fx_inv((size_t)B);
    for (int i = 0; i < B; ++i) {
        const int cap = class_cap(opt, b->m[(size_t)i]);
        tiles_for(col_ptr, b->stream_off[(size_t)i], b->stream_off[(size_t)i + 1], cap, i, st_seg, st_inst,
                  0, nullptr, kStreamSegs);
        tiles_for(row_ptr, b->link_off[(size_t)i], b->link_off[(size_t)i + 1], cap, i, lt_seg, lt_inst,
                  chunk, &lt_ck);
        inst_st.push_back((int)st_inst.size());
        inst_lt.push_back((int)lt_inst.size());
        long long maxlong = 0;
        for (int l = b->link_off[(size_t)i]; l < b->link_off[(size_t)i + 1]; ++l) {
            const long long len = row_ptr[(size_t)l + 1] - row_ptr[(size_t)l];
            if (len > kCap) maxlong = std::max(maxlong, len);
        }
        fx_shift[(size_t)i] = long_row_shift(sizeof(T), maxlong, hi[(size_t)i]);
        fx_scale[(size_t)i] = std::ldexp(1.0, fx_shift[(size_t)i]);
        fx_inv[(size_t)i] = std::ldexp(1.0, -fx_shift[(size_t)i]);
    }
    d.nst = (int)st_inst.size();
    d.nlt = (int)lt_inst.size();
    if (d.nst > L.nst_max || d.nlt > L.nlt_max)
        return set_error(PMP_ERR_SHAPE, "internal: batch tile tables exceed their bound");
    BATCH_TRY(hipMemcpyAsync((void *)d.st_seg, st_seg.data(), st_seg.size() * 4, hipMemcpyHostToDevice, s));
    if (d.nst) BATCH_TRY(hipMemcpyAsync((void *)d.st_inst, st_inst.data(), st_inst.size() * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.lt_seg, lt_seg.data(), lt_seg.size() * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.lt_inst, lt_inst.data(), lt_inst.size() * 4, hipMemcpyHostToDevice, s));
    if (d.nlt) {
        BATCH_TRY(hipMemcpyAsync((void *)d.lt_ck, lt_ck.data(), lt_ck.size() * sizeof(int2), hipMemcpyHostToDevice, s));
        launch_fill_int((int *)d.lt_hcnt, 0, d.nlt, s);
    }
    BATCH_TRY(hipMemcpyAsync((void *)d.ifx_shift, fx_shift.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.ifx_scale, fx_scale.data(), (size_t)B * 8, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.ifx_inv, fx_inv.data(), (size_t)B * 8, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.inst_st, inst_st.data(), inst_st.size() * 4, hipMemcpyHostToDevice, s));
    BATCH_TRY(hipMemcpyAsync((void *)d.inst_lt, inst_lt.data(), inst_lt.size() * 4, hipMemcpyHostToDevice, s));

    pmp_status st = batch_init_ctl<T>(b);
    if (st != PMP_OK) return st;
    int dev = 0;
    BATCH_TRY(hipGetDevice(&dev));
    b->grid = batch_grid_size<T>(dev, opt->wg_per_cu);
    if (b->grid < 1) return set_error(PMP_ERR_HIP, "occupancy query for the batch kernel failed");
    if (b->grid > kBatchMaxGrid) b->grid = kBatchMaxGrid;
    b->profile = opt->profile != 0;
    BATCH_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

template <typename T>
pmp_status batch_solve_impl(pmp_batch *b, int max_iter, pmp_result *res)
{
    BDev<T> &d = bdev_of<T>(b);
    if (max_iter > 0) {
        if (b->graph_iters != max_iter) {
            if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->graph_exec = nullptr;
            b->graph = nullptr;
            BATCH_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            // barrier counters and abort flag start at zero in every launch
            launch_fill_int((int *)d.bar, 0, kBarWords, b->cap_stream);
            launch_batch<T>(d, b->grid, max_iter, b->prm.check_every, b->prm.adapt_every, b->cap_stream);
            BATCH_TRY(hipStreamEndCapture(b->cap_stream, &b->graph));
            BATCH_TRY(hipGraphInstantiateWithFlags(&b->graph_exec, b->graph, 0));
            b->graph_iters = max_iter;
        }
        BATCH_TRY(hipGraphLaunch(b->graph_exec, b->stream));
    }
    std::vector<Ctl> h((size_t)b->B);
    int abort_flag = 0;
    BATCH_TRY(hipMemcpyAsync(h.data(), d.ictl, sizeof(Ctl) * h.size(), hipMemcpyDeviceToHost, b->stream));
    BATCH_TRY(hipMemcpyAsync(&abort_flag, d.abort, 4, hipMemcpyDeviceToHost, b->stream));
    BATCH_TRY(hipStreamSynchronize(b->stream));
    if (abort_flag) return set_error(PMP_ERR_HIP, "batch kernel: a grid barrier wait exceeded its bound");
    bool all = true;
    for (int i = 0; i < b->B; ++i) {
        const Ctl &c = h[(size_t)i];
        const pmp_status st = c.done ? (pmp_status)c.status : PMP_NOT_CONVERGED;
        if (res) {
            res[i].iterations = c.iter - b->iter_base[(size_t)i];
            res[i].r_norm = c.r_norm;
            res[i].s_norm = c.s_norm;
            res[i].eps_tol = c.eps_tol;
            res[i].rho = c.rho;
            res[i].status = st;
        }
        b->iter_base[(size_t)i] = c.iter;
        if (st != PMP_OK) all = false;
    }
    return all ? PMP_OK : PMP_NOT_CONVERGED;
}

template <typename T>
pmp_status batch_solution_impl(pmp_batch *b, int i, T *x, T *lambda, T *slack)
{
    BDev<T> &d = bdev_of<T>(b);
    Dev<T> di = d.g;
    const int l0 = b->link_off[(size_t)i], s0 = b->stream_off[(size_t)i];
    di.m = b->m[(size_t)i];
    di.n = b->n[(size_t)i];
    di.x += s0;
    di.u += l0;
    di.c += l0;
    di.ps_prev += l0;
    di.ctl = d.ictl + i;
    launch_solution<T>(di, nullptr, lambda, slack, b->stream);
    if (x) launch_batch_gather_x<T>(d.g.x + s0, b->sperm + s0, b->n[(size_t)i], x, b->stream);
    BATCH_TRY(hipGetLastError());
    BATCH_TRY(hipStreamSynchronize(b->stream));
    return PMP_OK;
}

}  // namespace

extern "C" {

pmp_status pmp_batch_options_default(pmp_batch_options *o)
{
    if (!o) return set_error(PMP_ERR_INVALID, "options is NULL");
    o->class_m[0] = 10000;
    o->class_m[1] = 50000;
    // the autotuner's choice on MI355X for the transit batch of Section VI
    o->tile_cap[0] = kBS;
    o->tile_cap[1] = kBS;
    o->tile_cap[2] = kBS;
    o->reorder_streams = 1;
    o->wg_per_cu = 4;
    o->profile = 0;
    o->heavy_chunk = kLongChunk;
    o->wait_log2 = kWaitLog2Default;
    return PMP_OK;
}

static pmp_status check_batch_args(int32_t count, const pmp_problem *pr, const pmp_params *prm,
                                   const pmp_batch_options *opt, BatchSizes &z)
{
    if (count < 1 || !pr || !prm || !opt) return set_error(PMP_ERR_INVALID, "bad batch arguments");
    for (int c = 0; c < 3; ++c)
        if (opt->tile_cap[c] < 64 || opt->tile_cap[c] > kBS)
            return set_error(PMP_ERR_INVALID, "tile_cap must be in [64, %d]", kBS);
    if (opt->wg_per_cu < 0 || opt->wg_per_cu > 8)
        return set_error(PMP_ERR_INVALID, "wg_per_cu must be in [0, 8]");
    if (opt->heavy_chunk != 0 && (opt->heavy_chunk < 1024 || opt->heavy_chunk > (1 << 20)))
        return set_error(PMP_ERR_INVALID, "heavy_chunk must be 0 or in [1024, 2^20]");
    if (opt->wait_log2 < 0 || opt->wait_log2 > 30)
        return set_error(PMP_ERR_INVALID, "wait_log2 must be in [0, 30]");
    for (int i = 1; i < count; ++i)
        if (pr[i].dtype != pr[0].dtype) return set_error(PMP_ERR_INVALID, "batch instances must share the dtype");
    if (!sizes_of(count, pr, z)) return set_error(PMP_ERR_SHAPE, "batch sizes out of range (m >= 1; totals < 2^31)");
    if (prm->check_every < 1 || prm->adapt_every < 0 ||
        (prm->adapt_every > 0 && prm->adapt_every % prm->check_every))
        return set_error(PMP_ERR_INVALID, "adapt_every must be 0 or a multiple of check_every");
    if (!(prm->rho0 > 0.0) || !(prm->alpha > 0.0 && prm->alpha < 2.0) || !(prm->mu > 1.0) || !(prm->gamma > 1.0))
        return set_error(PMP_ERR_INVALID, "rho0 > 0, alpha in (0, 2), mu > 1 and gamma > 1 required");
    if (prm->eps_rel != 0.0)
        return set_error(PMP_ERR_INVALID, "batched solves take the absolute stop rule (eps_rel = 0)");
    return PMP_OK;
}

pmp_status pmp_batch_workspace_size(int32_t count, const pmp_problem *problems,
                                    const pmp_params *params, const pmp_batch_options *options,
                                    size_t *bytes)
{
    BatchSizes z;
    pmp_status st = check_batch_args(count, problems, params, options, z);
    if (st != PMP_OK) return st;
    if (!bytes) return set_error(PMP_ERR_INVALID, "bytes is NULL");
    const int min_cap = std::min(options->tile_cap[0], std::min(options->tile_cap[1], options->tile_cap[2]));
    *bytes = batch_plan(z, problems[0].dtype == PMP_F64 ? 8 : 4, min_cap, heavy_chunk_of(options)).total;
    return PMP_OK;
}

pmp_status pmp_batch_setup(int32_t count, const pmp_problem *problems, const pmp_params *params,
                           const pmp_batch_options *options, void *workspace,
                           size_t workspace_bytes, void *stream, pmp_batch **out)
{
    if (!out) return set_error(PMP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    BatchSizes z;
    pmp_status st = check_batch_args(count, problems, params, options, z);
    if (st != PMP_OK) return st;
    for (int i = 0; i < count; ++i)
        if ((st = validate_host(problems[i], i)) != PMP_OK) return st;
    const size_t sz = problems[0].dtype == PMP_F64 ? 8 : 4;
    const int min_cap = std::min(options->tile_cap[0], std::min(options->tile_cap[1], options->tile_cap[2]));
    const size_t need = batch_plan(z, sz, min_cap, heavy_chunk_of(options)).total;
    if (!workspace || workspace_bytes < need)
        return set_error(PMP_ERR_SHAPE, "batch workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if ((uintptr_t)workspace % kAlignB) return set_error(PMP_ERR_INVALID, "workspace must be 256-byte aligned");
    pmp_batch *b = new (std::nothrow) pmp_batch();
    if (!b) return set_error(PMP_ERR_NOMEM, "batch handle allocation failed");
    b->B = count;
    b->dtype = problems[0].dtype;
    b->prm = *params;
    b->stream = (hipStream_t)stream;
    b->iter_base.assign((size_t)count, 0);
    for (int i = 0; i < count; ++i) {
        b->m.push_back(problems[i].m);
        b->n.push_back(problems[i].n);
        b->nnz.push_back(problems[i].nnz);
        b->eps_tol.push_back(params->eps_abs * std::sqrt((double)problems[i].nnz + problems[i].m));
    }
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return set_error(PMP_ERR_HIP, "hipStreamCreateWithFlags failed");
    }
    st = b->dtype == PMP_F32 ? batch_setup_impl<float>(b, problems, options, (char *)workspace, z)
                             : batch_setup_impl<double>(b, problems, options, (char *)workspace, z);
    if (st != PMP_OK) {
        pmp_batch_destroy(b);
        return st;
    }
    *out = b;
    return PMP_OK;
}

pmp_status pmp_batch_solve(pmp_batch *b, int32_t max_iter, pmp_result *results)
{
    if (!b || max_iter < 0) return set_error(PMP_ERR_INVALID, "bad argument");
    return b->dtype == PMP_F32 ? batch_solve_impl<float>(b, max_iter, results)
                               : batch_solve_impl<double>(b, max_iter, results);
}

pmp_status pmp_batch_get_solution(pmp_batch *b, int32_t index, void *x, void *lambda, void *slack)
{
    if (!b || index < 0 || index >= b->B) return set_error(PMP_ERR_INVALID, "bad argument");
    return b->dtype == PMP_F32
               ? batch_solution_impl<float>(b, index, (float *)x, (float *)lambda, (float *)slack)
               : batch_solution_impl<double>(b, index, (double *)x, (double *)lambda, (double *)slack);
}

pmp_status pmp_batch_reset(pmp_batch *b)
{
    if (!b) return set_error(PMP_ERR_INVALID, "batch is NULL");
    pmp_status st;
    if (b->dtype == PMP_F32) {
        launch_zero_state<float>(b->bf.g, b->stream);
        st = batch_init_ctl<float>(b);
    } else {
        launch_zero_state<double>(b->bd.g, b->stream);
        st = batch_init_ctl<double>(b);
    }
    if (st != PMP_OK) return st;
    BATCH_TRY(hipGetLastError());
    BATCH_TRY(hipStreamSynchronize(b->stream));
    return PMP_OK;
}

pmp_status pmp_batch_profile(pmp_batch *b, double *ms)
{
    if (!b || !ms) return set_error(PMP_ERR_INVALID, "NULL argument");
    if (!b->profile) return set_error(PMP_ERR_STATE, "the batch was set up without profile = 1");
    const unsigned long long *dp = b->dtype == PMP_F32 ? b->bf.prof : b->bd.prof;
    std::vector<unsigned long long> h((size_t)b->grid * kBatchPhases);
    BATCH_TRY(hipMemcpy(h.data(), dp, h.size() * 8, hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    BATCH_TRY(hipGetDevice(&dev));
    BATCH_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return set_error(PMP_ERR_HIP, "wall clock rate unknown");
    for (int k = 0; k < kBatchPhases; ++k) {
        double sum = 0.0;
        for (int g = 0; g < b->grid; ++g) sum += (double)h[(size_t)g * kBatchPhases + k];
        ms[k] = sum / b->grid / khz;   // ticks / kHz = ms
    }
    return PMP_OK;
}

pmp_status pmp_batch_destroy(pmp_batch *b)
{
    if (!b) return PMP_OK;
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return PMP_OK;
}

}  // extern "C"
