// Binned message exchange: the PMP iteration for large, unstructured R.
//
// On a random link-route pattern the gathers of the CSR/CSC passes hit a
// different cache line for nearly every nonzero, and random 4-byte gathers
// from an 80 MB vector run an order of magnitude below streaming bandwidth.
// This layout instead moves one message per nonzero through HBM in
// coalesced runs:
//   R is tiled into P x Q tiles (link block p: consecutive links holding
//   about nnz / P nonzeros, at most LB links; stream block q: SB consecutive
//   streams).  mx holds x_j for every nonzero, tile by tile in p-major
//   order; mv holds v_l in q-major order; both list a tile's nonzeros in the
//   same order (grouped by link), so entry k of tile (p, q) is the same
//   nonzero in both.
//   stream workgroup q: add its mv entries into FP64 LDS sums by local stream
//     index (six), run the stream epilogue (prox, relaxation), then write
//     x_j into mx tile by tile (one wave per tile).
//   link workgroup p: add its mx entries into FP64 LDS sums by local link
//     index (lix), run the link epilogue (slack prox, average, dual update),
//     then write v_l into mv tile by tile.
// The LDS sums are FP64 atomic adds of FP32 messages.  Every addend is a
// multiple of the smallest addend's FP32 ulp u, so while a sum stays below
// 2^53 u every partial sum is exact (for example up to 32 addends spanning
// less than 2^24 in magnitude, or 1000 spanning less than 2^19): the result
// then does not depend on the order of the adds and equals the sequential
// FP64 sum of the CSR/CSC kernels.  Beyond that the order of the adds moves
// the last bits only.
#include "pmp_device.h"

#include <algorithm>

namespace pmp {

namespace {

typedef double acc_t;   // LDS sums

// Tuning knobs (defaults measured on MI355X at the large size and on a
// congested instance):
//   PMP_BIN_RUNS    merge runs of one link index before the LDS adds
//   PMP_BIN_EMIT_U  tiles a wave emits per step
//   PMP_BIN_EPI     rows per lane whose epilogue inputs are loaded before
//                   any of them is updated
#ifndef PMP_BIN_RUNS
#define PMP_BIN_RUNS true
#endif
#ifndef PMP_BIN_EMIT_U
#define PMP_BIN_EMIT_U 4
#endif
#ifndef PMP_BIN_EPI
#define PMP_BIN_EPI 2
#endif

// Workgroups are handed to the 8 XCDs of the chip in turn (block b to XCD
// b mod 8).  Renumbered so that every XCD runs one contiguous range of
// blocks, neighbouring blocks write neighbouring tiles from the same L2, where
// the partly written cache lines at tile boundaries merge before write-back.
#ifndef PMP_BIN_XCD
#define PMP_BIN_XCD 1
#endif
__device__ __forceinline__ int xcd_block(int b, int nblocks)
{
    if (!PMP_BIN_XCD) return b;
    constexpr int X = 8;
    const int x = b % X, per = nblocks / X, rem = nblocks % X;
    return x * per + min(x, rem) + b / X;
}

// Stream blocks in descending rounds: dispatch round r (blocks [R r, R r + R),
// R = Dev::SR: one block per CU, or all of them when the GPU holds them all
// at once) takes the r-th range of R stream blocks from the top, and inside a round every XCD takes a run of
// consecutive blocks (so the tiles that neighbouring workgroups write are
// neighbours, as with xcd_block).  The link pass writes the v-message tiles in
// ascending stream-block order, so the first stream blocks read the tiles
// written last, which the 256 MB memory-side cache may still hold; likewise
// the last stream blocks write the x-message tiles that every link block
// reads first.  Measured on the large workload: stream pass 0.385 -> 0.368 ms,
// link pass 0.352 -> 0.336 ms, against xcd_block numbering (rounds of two
// blocks per CU; one per CU gains another 1%).
__device__ __forceinline__ int stream_block(int b, int nblocks, int R)
{
    constexpr int X = 8;
    const int r = b / R, i = b % R;
    const int top = nblocks - R * r;
    const int lo = max(0, top - R);
    const int cnt = top - lo;
    const int x = i % X, pos = i / X, per = cnt / X, rem = cnt % X;
    return lo + x * per + min(x, rem) + pos;
}

// Add messages msg[e0..e1) into acc[idx[e]] (FP64 LDS atomics).  FP32
// messages are read four at a time (16-byte message and 8-byte index loads,
// aligned; the arrays carry 4 entries of padding), entries outside
// [e0, e1) being masked.  Messages are loaded non-temporally; indices too,
// unless TIDX.
//
// RUNS (link side): inside a tile the x messages are grouped by link, so a
// link with many streams in the tile (a congested link) makes a long run of one
// local index, and its LDS adds would all hit one address.  When some lane's
// four entries share one index, the wave merges runs first: such a lane
// contributes the sum of its four entries, a segmented sum over the lanes
// (segments = maximal runs of equal indices) totals each run, and the last
// lane of a run adds it once.  The sums are FP64 sums of FP32 messages, exact
// under the same condition as the LDS adds, so the result does not change.
//
// FX (link side, FP32): an index carrying kLongBit belongs to a long row,
// whose slot holds an int64 fixed-point sum instead (Dev::fx_shift): the
// entry adds fx_term(x, fxs) with an integer atomic, and merged runs of such
// a row add the integer sum of their terms, so the row's total does not
// depend on the order of the adds.
template <typename T, bool RUNS, bool FX = false, bool TIDX = false>
__device__ __forceinline__ void accumulate(const T *__restrict__ msg,
                                           const uint16_t *__restrict__ idx, int e0, int e1,
                                           acc_t *acc, double fxs = 0.0)
{
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        typedef unsigned short u4 __attribute__((ext_vector_type(4)));
        const f4 *m4 = (const f4 *)msg;
        const u4 *i4 = (const u4 *)idx;
        const int lane = threadIdx.x & 63;
        auto add1 = [&](float v, unsigned key) {
            if (FX && (key & kLongBit))
                atomicAdd((unsigned long long *)&acc[key & kLocalMask],
                          (unsigned long long)fx_term((double)v, fxs));
            else
                unsafeAtomicAdd(&acc[key & kLocalMask], (acc_t)v);
        };
        auto add4 = [&](const f4 &v, const u4 &k, int e) {
            if (e >= e0 && e < e1) add1(v.x, k.x);
            if (e + 1 >= e0 && e + 1 < e1) add1(v.y, k.y);
            if (e + 2 >= e0 && e + 2 < e1) add1(v.z, k.z);
            if (e + 3 >= e0 && e + 3 < e1) add1(v.w, k.w);
        };
        // every lane of a wave takes the same trips (the run merge below is
        // wave-wide); a lane past the end loads nothing
        const int b1 = (e1 + 3) >> 2;
        for (int bw = (e0 >> 2) + (threadIdx.x & ~63); bw < b1; bw += kBinThreads) {
            const int b = bw + lane;
            const bool in = b < b1;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            u4 k = {0, 0, 0, 0};
            if (in) {
                v = __builtin_nontemporal_load(m4 + b);
                if (TIDX) k = i4[b];
                else k = __builtin_nontemporal_load(i4 + b);
            }
            const int e = b << 2;
            if constexpr (RUNS) {
                const bool uni = in && e >= e0 && e + 3 < e1 && k.x == k.y && k.y == k.z &&
                                 k.z == k.w;
                if (__ballot(uni) != 0) {
                    int key = uni ? (int)k.x : -1 - lane;   // others: segments of their own
                    const bool lng = FX && uni && (k.x & kLongBit);
                    double sum = uni && !lng
                                     ? ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w)
                                     : 0.0;
                    long long isum = 0;
                    if (lng)
                        isum = (fx_term((double)v.x, fxs) + fx_term((double)v.y, fxs)) +
                               (fx_term((double)v.z, fxs) + fx_term((double)v.w, fxs));
                    if (in && !uni) add4(v, k, e);
                    const int prev = __shfl_up(key, 1, 64);
                    int head = lane == 0 || prev != key;
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const double so = __shfl_up(sum, off, 64);
                        long long io = 0;
                        if (FX) io = __shfl_up(isum, off, 64);
                        const int ho = __shfl_up(head, off, 64);
                        if (lane >= off) {
                            if (!head) {
                                sum += so;
                                isum += io;
                            }
                            head |= ho;
                        }
                    }
                    const int next = __shfl_down(key, 1, 64);
                    if (uni && (lane == 63 || next != key)) {
                        if (lng)
                            atomicAdd((unsigned long long *)&acc[key & kLocalMask],
                                      (unsigned long long)isum);
                        else
                            unsafeAtomicAdd(&acc[key & kLocalMask], (acc_t)sum);
                    }
                    continue;
                }
            }
            if (in) add4(v, k, e);
        }
    } else {
        for (int e = e0 + threadIdx.x; e < e1; e += kBinThreads)
            unsafeAtomicAdd(&acc[idx[e] & kLocalMask], (acc_t)__builtin_nontemporal_load(msg + e));
    }
}

// Write the messages of one workgroup's tiles.  Wave w takes tiles
// w, w + W, w + 2W, ... (W waves).  Lane i first loads the offsets of the
// wave's i-th tile of the next 64.  The wave then writes its tiles four at a
// time: every lane loads the local indices of its entries in all four tiles
// (up to two entries per tile) before any value is looked up and stored, so
// eight index loads per lane are in flight; entries of longer tiles follow in
// rounds of four 64-entry chunks, again with the loads issued first.
//   src_off[t], src_off[t + 1]   tile t in the read layout (index array idx)
//   dst_off[t]                   tile t in the written layout
// LONG: the local indices may carry kLongBit (link side of a problem with
// fixed-point long rows), which is masked off where the LDS value is read.
// (Masked right at the load, the compiler waits for each index load before
// issuing the next: 17% slower passes on the large workload.)
template <typename T, bool LONG = false>
__device__ __forceinline__ void emit_tiles(const int *__restrict__ src_off,
                                           const int *__restrict__ dst_off, int ntiles,
                                           const uint16_t *__restrict__ idx, const acc_t *vals,
                                           T *__restrict__ out)
{
    constexpr int W = kBinThreads / 64;
    constexpr int U = PMP_BIN_EMIT_U;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mine = ntiles > wave ? (ntiles - wave + W - 1) / W : 0;   // tiles of this wave
    for (int base = 0; base < mine; base += 64) {
        const int t = wave + (base + lane) * W;
        int src = 0, cnt = 0, dst = 0;
        if (base + lane < mine) {
            src = src_off[t];
            cnt = src_off[t + 1] - src;
            dst = dst_off[t];
        }
        const int nt = min(64, mine - base);
        for (int i0 = 0; i0 < nt; i0 += U) {
            int s_u[U], c_u[U], d_u[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = min(i0 + u, nt - 1);
                s_u[u] = __shfl(src, i, 64);
                c_u[u] = i0 + u < nt ? __shfl(cnt, i, 64) : 0;
                d_u[u] = __shfl(dst, i, 64);
            }
            int id[U][2];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int k = lane + 64 * r;
                    id[u][r] = k < c_u[u] ? (int)idx[s_u[u] + k] : -1;
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < 2; ++r)
                    if (id[u][r] >= 0) out[d_u[u] + lane + 64 * r] = (T)vals[LONG ? id[u][r] & kLocalMask : id[u][r]];
            // long tiles: four chunks of 64 entries per round, loads first
#pragma unroll
            for (int u = 0; u < U; ++u)
                for (int k0 = lane + 128; k0 - lane < c_u[u]; k0 += 256) {
                    int it[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int k = k0 + 64 * r;
                        it[r] = k < c_u[u] ? (int)idx[s_u[u] + k] : -1;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (it[r] >= 0) out[d_u[u] + k0 + 64 * r] = (T)vals[LONG ? it[r] & kLocalMask : it[r]];
                }
        }
    }
}

// Two workgroups of kBinThreads share a CU (the LDS sums fit twice): ask for
// the register budget of 8 waves per SIMD.
#ifndef PMP_BIN_WAVES
#define PMP_BIN_WAVES 8
#endif
#if PMP_BIN_WAVES > 0
#define PMP_BIN_KERNEL \
    __global__ __launch_bounds__(kBinThreads) __attribute__((amdgpu_waves_per_eu(PMP_BIN_WAVES)))
#else
#define PMP_BIN_KERNEL __global__ __launch_bounds__(kBinThreads)
#endif

template <typename T, int MODE, bool TIDX>
PMP_BIN_KERNEL void k_bin_stream(Dev<T> d)
{
    if (d.ctl->done) return;
    extern __shared__ acc_t S[];
    __shared__ double sred[kBinThreads / 64];
    const int q = stream_block(blockIdx.x, gridDim.x, d.SR);
    const int j0 = d.sbs[q];
    const int ns = d.sbs[q + 1] - j0;
    for (int i = threadIdx.x; i < ns; i += kBinThreads) S[i] = 0.0;
    __syncthreads();
    // TIDX (chosen at launch when the stream blocks take several dispatch
    // rounds): the local stream indices are loaded as ordinary (temporal)
    // data, since the emission below reads them again; on the large workload
    // that read then hits more often (stream pass 0.367 -> 0.359 ms).  With
    // every stream block resident at once (the paper shape) the same hint
    // costs 6%, and on the link side it slows the link pass: there the
    // indices stay non-temporal.
    accumulate<T, false, false, TIDX>(d.mv, d.six, d.ov[(long long)q * d.P], d.ov[(long long)(q + 1) * d.P], S);
    __syncthreads();
    const double rho = d.ctl->rho;
    double part = 0.0;
    constexpr int G = PMP_BIN_EPI;
    // The per-stream vectors (route length, weight, a) go through
    // non-temporally: the next read of a comes a whole iteration later, far
    // beyond what the memory-side cache keeps, and leaving them out of it
    // keeps more of the message tiles and indices there (large workload:
    // stream pass 0.357 -> 0.348 ms; the link side's vectors, tried the same
    // way, slowed the link pass by 3%).
    for (int i0 = threadIdx.x; i0 < ns; i0 += G * kBinThreads) {
        int L[G];
        double a[G], w[G], xo[G];
        bool a2[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = i0 + g * kBinThreads;
            if (i < ns) {
                const int j = j0 + i;
                L[g] = d.rlen ? (int)__builtin_nontemporal_load(d.rlen + j)
                              : d.col_ptr[j + 1] - d.col_ptr[j];
                a[g] = (double)__builtin_nontemporal_load(d.a + j);
                w[g] = (double)__builtin_nontemporal_load(d.wsig + j);
                a2[g] = is_alpha2(d, j);
                xo[g] = MODE == kCheck ? (double)d.x[j] : 0.0;
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = i0 + g * kBinThreads;
            if (i < ns) {
                const int j = j0 + i;
                const T xt = (T)prox_stream((double)L[g] * a[g] + (double)S[i], L[g], w[g], rho,
                                            d.lo, d.hi, a2[g]);
                const double xn = (double)xt;
                const T at = (T)(d.alpha * xn + (1.0 - d.alpha) * a[g]);
                if (MODE == kCheck) {          // dual residual: sum_j L_j (dx_j)^2
                    const double dx = xn - xo[g];
                    part += screen((double)L[g] * dx * dx, (double)at);
                }
                if (MODE != kPlain) d.x[j] = xt;   // otherwise x travels only in the messages
                __builtin_nontemporal_store(at, d.a + j);
                S[i] = (acc_t)xn;
            }
        }
    }
    __syncthreads();
    // tile (q, p) of the v messages and tile (p, q) of the x messages list the
    // same nonzeros in the same order
    emit_tiles<T>(d.ov + (long long)q * d.P, d.oxq + (long long)q * d.P, d.P, d.six, S, d.mx);
    if (MODE == kCheck) {
        part = block_sum_n<kBinThreads>(part, sred);
        if (threadIdx.x == 0) d.spart[q] = part;
    }
}

template <typename T, int MODE>
PMP_BIN_KERNEL void k_bin_link(Dev<T> d)
{
    if (d.ctl->done) return;
    extern __shared__ acc_t Y[];
    __shared__ double sred[kBinThreads / 64];
    const int p = xcd_block(blockIdx.x, gridDim.x);
    const int l0 = d.lbs[p];
    const int nl = d.lbs[p + 1] - l0;
    for (int i = threadIdx.x; i < nl; i += kBinThreads) Y[i] = 0.0;
    __syncthreads();
    const int e0 = d.ox[(long long)p * d.Q], e1 = d.ox[(long long)(p + 1) * d.Q];
    if (sizeof(T) == 4 && d.fx_shift) accumulate<T, PMP_BIN_RUNS, true>(d.mx, d.lix, e0, e1, Y, d.fx_scale);
    else accumulate<T, PMP_BIN_RUNS>(d.mx, d.lix, e0, e1, Y);
    __syncthreads();
    double r2 = 0.0, s2 = 0.0;
    constexpr int G = MODE == kCheck ? 1 : PMP_BIN_EPI;   // a check carries more inputs
    for (int i0 = threadIdx.x; i0 < nl; i0 += G * kBinThreads) {
        int deg[G];
        LinkIn in[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = i0 + g * kBinThreads;
            if (i < nl) {
                const int l = l0 + i;
                deg[g] = d.dlen ? (int)d.dlen[l] : d.row_ptr[l + 1] - d.row_ptr[l];
                in[g] = link_load<T, MODE>(d, l);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = i0 + g * kBinThreads;
            if (i < nl) {
                const int l = l0 + i;
                // v goes out in the messages; a check also stores it
                double y = (double)Y[i];
                if (d.fx_shift && deg[g] > kCap) y = (double)__double_as_longlong(Y[i]) * d.fx_inv;
                Y[i] = (acc_t)(MODE == kCheck
                                   ? link_update_in<T, MODE, true>(d, l, deg[g], y, in[g], r2, s2)
                                   : link_update_in<T, MODE, false>(d, l, deg[g], y, in[g], r2, s2));
            }
        }
    }
    if (MODE == kCheck) {
        r2 = block_sum_n<kBinThreads>(r2, sred);
        s2 = block_sum_n<kBinThreads>(s2, sred);
        if (threadIdx.x == 0) {
            d.lpart[2 * p] = r2;
            d.lpart[2 * p + 1] = s2;
        }
    }
    __syncthreads();
    if (d.fx_shift) emit_tiles<T, true>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, d.mv);
    else emit_tiles<T>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, d.mv);
}

// After a check (apply = 1): apply a pending u rescale (eq. (18)), refresh
// v = b - u and rewrite the link messages; without a pending rescale the
// check's link pass has written them already and nothing is done.  With
// apply = 0 the messages are rewritten from v.
template <typename T>
PMP_BIN_KERNEL void k_bin_emit(Dev<T> d, int apply)
{
    if (apply && d.ctl->ratio == 1.0) return;
    extern __shared__ acc_t Y[];
    const int p = xcd_block(blockIdx.x, gridDim.x);
    const int l0 = d.lbs[p];
    const int nl = d.lbs[p + 1] - l0;
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
        Y[i] = (acc_t)vt;
    }
    __syncthreads();
    if (d.fx_shift) emit_tiles<T, true>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, d.mv);
    else emit_tiles<T>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, d.mv);
}

// Reverse mode in the binned layout: the two sums of a reversed iteration,
// R^T ybar (per stream) and R Sbar (per link), move as messages in the
// problem's precision through the same tiles as the forward messages (ybar in
// the v layout, Sbar in the x layout) and are summed in FP64 as there.  The
// FP64 values of ybar and Sbar are rounded to the message precision, so in
// FP32 these sums match the gather layout's FP64 gathers to FP32 rounding
// (a gradient of the adjoint workload: 0.0857 s, against 0.0928 s with FP64
// messages).
template <typename T>
PMP_BIN_KERNEL void k_bin_adj_stream(Dev<T> d, AdjDev a, const T *xt, int last,
                                     const T *my, T *ms)
{
    extern __shared__ acc_t S[];
    const int q = xcd_block(blockIdx.x, gridDim.x);
    const int j0 = d.sbs[q];
    const int ns = d.sbs[q + 1] - j0;
    for (int i = threadIdx.x; i < ns; i += kBinThreads) S[i] = 0.0;
    __syncthreads();
    accumulate<T, false>(my, d.six, d.ov[(long long)q * d.P], d.ov[(long long)(q + 1) * d.P], S);
    __syncthreads();
    const double rho = d.ctl->rho;
    for (int i = threadIdx.x; i < ns; i += kBinThreads) {
        const int j = j0 + i;
        const int L = d.rlen ? (int)d.rlen[j] : d.col_ptr[j + 1] - d.col_ptr[j];
        adj_stream_step<T>(d, a, xt, j, L, (double)S[i], last, rho);
        S[i] = a.Sbar[j];
    }
    __syncthreads();
    emit_tiles<T>(d.ov + (long long)q * d.P, d.oxq + (long long)q * d.P, d.P, d.six, S, ms);
}

// R Sbar per link, then (mu_prev given) the link step of the iteration
// before, whose ybar goes out as messages for the next stream step.
template <typename T>
PMP_BIN_KERNEL void k_bin_adj_link(Dev<T> d, AdjDev a, const uint8_t *mu_prev, const T *ms,
                                   T *my)
{
    extern __shared__ acc_t Y[];
    const int p = xcd_block(blockIdx.x, gridDim.x);
    const int l0 = d.lbs[p];
    const int nl = d.lbs[p + 1] - l0;
    for (int i = threadIdx.x; i < nl; i += kBinThreads) Y[i] = 0.0;
    __syncthreads();
    accumulate<T, false>(ms, d.lix, d.ox[(long long)p * d.Q], d.ox[(long long)(p + 1) * d.Q], Y);
    __syncthreads();
    for (int i = threadIdx.x; i < nl; i += kBinThreads) {
        const int l = l0 + i;
        const double vbar = (double)Y[i];
        a.B[l] += vbar;
        a.U[l] -= vbar;
        if (mu_prev) {
            const int deg = d.dlen ? (int)d.dlen[l] : d.row_ptr[l + 1] - d.row_ptr[l];
            adj_link_step(a, l, deg, d.alpha, mu_prev[l]);
            Y[i] = a.ybar[l];
        }
    }
    if (!mu_prev) return;   // ybar unchanged: its messages still hold
    __syncthreads();
    if (d.fx_shift) emit_tiles<T, true>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, my);
    else emit_tiles<T>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, my);
}

// ybar messages from a.ybar (after it changed outside k_bin_adj_link).
template <typename T>
PMP_BIN_KERNEL void k_bin_adj_emit(Dev<T> d, AdjDev a, T *my)
{
    extern __shared__ acc_t Y[];
    const int p = xcd_block(blockIdx.x, gridDim.x);
    const int l0 = d.lbs[p];
    const int nl = d.lbs[p + 1] - l0;
    for (int i = threadIdx.x; i < nl; i += kBinThreads) Y[i] = a.ybar[l0 + i];
    __syncthreads();
    if (d.fx_shift) emit_tiles<T, true>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, my);
    else emit_tiles<T>(d.ox + (long long)p * d.Q, d.ovp + (long long)p * d.Q, d.Q, d.lix, Y, my);
}

}  // namespace

void binned_configure()
{
    const int bytes = kBinMaxBlock * (int)sizeof(acc_t);
#define PMP_BIN_ATTR(K) (void)hipFuncSetAttribute((const void *)(K), hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
    PMP_BIN_ATTR((k_bin_stream<float, kPlain, false>));
    PMP_BIN_ATTR((k_bin_stream<float, kSave, false>));
    PMP_BIN_ATTR((k_bin_stream<float, kCheck, false>));
    PMP_BIN_ATTR((k_bin_stream<double, kPlain, false>));
    PMP_BIN_ATTR((k_bin_stream<double, kSave, false>));
    PMP_BIN_ATTR((k_bin_stream<double, kCheck, false>));
    PMP_BIN_ATTR((k_bin_stream<float, kPlain, true>));
    PMP_BIN_ATTR((k_bin_stream<float, kSave, true>));
    PMP_BIN_ATTR((k_bin_stream<float, kCheck, true>));
    PMP_BIN_ATTR((k_bin_stream<double, kPlain, true>));
    PMP_BIN_ATTR((k_bin_stream<double, kSave, true>));
    PMP_BIN_ATTR((k_bin_stream<double, kCheck, true>));
    PMP_BIN_ATTR((k_bin_link<float, kPlain>));
    PMP_BIN_ATTR((k_bin_link<float, kSave>));
    PMP_BIN_ATTR((k_bin_link<float, kCheck>));
    PMP_BIN_ATTR((k_bin_link<double, kPlain>));
    PMP_BIN_ATTR((k_bin_link<double, kSave>));
    PMP_BIN_ATTR((k_bin_link<double, kCheck>));
    PMP_BIN_ATTR((k_bin_emit<float>));
    PMP_BIN_ATTR((k_bin_emit<double>));
    PMP_BIN_ATTR((k_bin_adj_stream<float>));
    PMP_BIN_ATTR((k_bin_adj_stream<double>));
    PMP_BIN_ATTR((k_bin_adj_link<float>));
    PMP_BIN_ATTR((k_bin_adj_link<double>));
    PMP_BIN_ATTR((k_bin_adj_emit<float>));
    PMP_BIN_ATTR((k_bin_adj_emit<double>));
#undef PMP_BIN_ATTR
}

template <typename T>
void launch_bin_stream(const Dev<T> &d, int mode, hipStream_t s)
{
    const size_t lds = (size_t)d.SB * sizeof(acc_t);
    const bool rounds = d.SR < d.Q;   // several dispatch rounds: temporal index loads
    switch (mode) {
    case kPlain:
        if (rounds) hipLaunchKernelGGL((k_bin_stream<T, kPlain, true>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
        else hipLaunchKernelGGL((k_bin_stream<T, kPlain, false>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
        break;
    case kSave:
        if (rounds) hipLaunchKernelGGL((k_bin_stream<T, kSave, true>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
        else hipLaunchKernelGGL((k_bin_stream<T, kSave, false>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
        break;
    default:
        if (rounds) hipLaunchKernelGGL((k_bin_stream<T, kCheck, true>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
        else hipLaunchKernelGGL((k_bin_stream<T, kCheck, false>), dim3(d.Q), dim3(kBinThreads), lds, s, d);
        break;
    }
}

template <typename T>
void launch_bin_link(const Dev<T> &d, int mode, hipStream_t s)
{
    const size_t lds = (size_t)d.LB * sizeof(acc_t);
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
    hipLaunchKernelGGL((k_bin_emit<T>), dim3(d.P), dim3(kBinThreads), (size_t)d.LB * sizeof(acc_t),
                       s, d, apply);
}

template <typename T>
void launch_bin_adj_stream(const Dev<T> &d, const AdjDev &a, const T *xt, int last,
                           const T *my, T *ms, hipStream_t s)
{
    hipLaunchKernelGGL((k_bin_adj_stream<T>), dim3(d.Q), dim3(kBinThreads),
                       ((size_t)d.SB) * sizeof(acc_t), s, d, a, xt, last, my, ms);
}

template <typename T>
void launch_bin_adj_link(const Dev<T> &d, const AdjDev &a, const uint8_t *mu_prev,
                         const T *ms, T *my, hipStream_t s)
{
    hipLaunchKernelGGL((k_bin_adj_link<T>), dim3(d.P), dim3(kBinThreads),
                       ((size_t)d.LB) * sizeof(acc_t), s, d, a, mu_prev, ms, my);
}

template <typename T>
void launch_bin_adj_emit(const Dev<T> &d, const AdjDev &a, T *my, hipStream_t s)
{
    hipLaunchKernelGGL((k_bin_adj_emit<T>), dim3(d.P), dim3(kBinThreads),
                       ((size_t)d.LB) * sizeof(acc_t), s, d, a, my);
}

template void launch_bin_stream<float>(const Dev<float> &, int, hipStream_t);
template void launch_bin_stream<double>(const Dev<double> &, int, hipStream_t);
template void launch_bin_link<float>(const Dev<float> &, int, hipStream_t);
template void launch_bin_link<double>(const Dev<double> &, int, hipStream_t);
template void launch_bin_emit<float>(const Dev<float> &, int, hipStream_t);
template void launch_bin_emit<double>(const Dev<double> &, int, hipStream_t);
template void launch_bin_adj_stream<float>(const Dev<float> &, const AdjDev &, const float *, int,
                                           const float *, float *, hipStream_t);
template void launch_bin_adj_stream<double>(const Dev<double> &, const AdjDev &, const double *,
                                            int, const double *, double *, hipStream_t);
template void launch_bin_adj_link<float>(const Dev<float> &, const AdjDev &, const uint8_t *,
                                         const float *, float *, hipStream_t);
template void launch_bin_adj_link<double>(const Dev<double> &, const AdjDev &, const uint8_t *,
                                          const double *, double *, hipStream_t);
template void launch_bin_adj_emit<float>(const Dev<float> &, const AdjDev &, float *, hipStream_t);
template void launch_bin_adj_emit<double>(const Dev<double> &, const AdjDev &, double *, hipStream_t);

}  // namespace pmp
