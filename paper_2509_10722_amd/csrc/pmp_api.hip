// C ABI of the PMP library (include/pmp.h): validation, workspace layout,
// setup, the asynchronous iteration queue, the graph-replayed solve loop,
// solution / state access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pmp_internal.h"

using namespace pmp;

namespace {

thread_local std::string g_last_error;

// Record the detail text of an error for pmp_last_error and return s.
template <typename... A>
pmp_status fail(pmp_status s, const char *fmt, A... args)
{
    return pmp::set_error(s, fmt, args...);
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(PMP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kSlots = 4;   // pipelined chunks in flight in pmp_solve

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t mx, mv, lix, six, ox, ov, oxq, ovp, lbs, sbs, rlen, dlen;
    bool binned;
    BinnedPlan bp;
    size_t row_ptr, col_idx, col_ptr, row_idx, c, wsig, a, x, b, zs, u, v, y_prev, ps_prev;
    size_t sblk, lblk, spart, lpart, ctl, hist, util, lck_beg, lck_end, lr_row, lr_ck, rpart, npart,
        total;
    int nsb_max, nlb_max, nlc_max, nlr_max;
};

// Tiles of the binned layout for these sizes (bound of the plan).
long long binned_tiles(int m, int n, long long nnz)
{
    const BinnedPlan bp = binned_plan(m, n, nnz);
    return (long long)bp.P * bp.Q;
}

// The binned tables hold a few ints per tile; beyond this many tiles the
// layout is refused (int offsets, and the tables would outweigh the messages).
constexpr long long kBinMaxTiles = 1LL << 28;

bool use_binned(int m, int n, long long nnz, size_t sz, int layout)
{
    if (layout == PMP_LAYOUT_BINNED) return m > 0 && n > 0;
    if (layout == PMP_LAYOUT_GATHER) return false;
    // measured crossover on MI355X: below about 2e6 nonzeros the vectors sit
    // in L2 and the gathers win; above, the binned passes do (1.5x at 5e6);
    // tiles must keep 16 or more nonzeros on average to pay for themselves
    return sz == 4 && nnz >= (1LL << 21) && m >= 256 && n >= 256 &&
           16 * binned_tiles(m, n, nnz) <= nnz;
}

pmp_status check_binned_size(const pmp_problem *pr, const pmp_params *prm)
{
    if (prm && prm->layout == PMP_LAYOUT_BINNED && pr->m > 0 && pr->n > 0 &&
        binned_tiles(pr->m, pr->n, pr->nnz) > kBinMaxTiles)
        return fail(PMP_ERR_SHAPE, "binned layout: more than 2^28 tiles for these sizes");
    return PMP_OK;
}

Layout plan(int m, int n, long long nnz, size_t sz, int layout)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    // Greedy blocks: each has kBlock segments or is closed by kCap, so two
    // consecutive blocks hold more than kCap nonzeros.
    L.nsb_max = (int)std::min<long long>((long long)n, n / kBlock + 2 * nnz / kCap + 2);
    L.nlb_max = (int)std::min<long long>((long long)m, m / kBlock + 2 * nnz / kCap + 2);
    L.binned = use_binned(m, n, nnz, sz, layout);
    if (L.binned) {
        L.bp = binned_plan(m, n, nnz);   // bounds; the blocks are cut at setup
        L.nsb_max = std::max(L.nsb_max, L.bp.Q);
        L.nlb_max = std::max(L.nlb_max, L.bp.P);
    }
    L.row_ptr = take(((size_t)m + 1) * 4);
    L.col_idx = take((size_t)nnz * 4);
    L.col_ptr = take(((size_t)n + 1) * 4);
    L.row_idx = take((size_t)nnz * 4);
    L.c = take((size_t)m * sz);
    L.wsig = take((size_t)n * sz);
    // a and x are contiguous: the transpose scratch (n + n/2048 + 1 ints)
    // lives there during setup.
    L.a = take(std::max((size_t)n * sz, transpose_scratch_ints(n) * 4));
    L.x = take((size_t)n * sz);
    L.b = take((size_t)m * sz);
    L.zs = take((size_t)m * sz);
    L.u = take((size_t)m * sz);
    L.v = take((size_t)m * sz);
    L.y_prev = take((size_t)m * 8);
    L.ps_prev = take((size_t)m * 8);
    L.sblk = take(((size_t)L.nsb_max + 1) * 4);
    L.lblk = take(((size_t)L.nlb_max + 1) * 4);
    L.spart = take((size_t)L.nsb_max * 8);
    L.nlr_max = (int)std::min<long long>((long long)m, nnz / (kCap + 1) + 1);
    L.nlc_max = (int)(nnz / kLongChunk + L.nlr_max + 1);
    L.lpart = take(((size_t)L.nlb_max + L.nlr_max) * 16);
    L.lck_beg = take((size_t)L.nlc_max * 4);
    L.lck_end = take((size_t)L.nlc_max * 4);
    L.lr_row = take((size_t)L.nlr_max * 4);
    L.lr_ck = take(((size_t)L.nlr_max + 1) * 4);
    L.rpart = take((size_t)L.nlc_max * 8);
    L.npart = take((size_t)kNormBlocks * 5 * 8);
    L.ctl = take(sizeof(Ctl));
    L.hist = take(sizeof(HistEntry) * kHist);
    L.util = take((size_t)n);
    if (L.binned) {
        const size_t tiles = (size_t)L.bp.P * (size_t)L.bp.Q + 1;
        // 4 entries of padding: the accumulation reads aligned groups of 4
        L.mx = take((size_t)(nnz + 4) * sz);
        L.mv = take((size_t)(nnz + 4) * sz);
        L.lix = take((size_t)(nnz + 4) * 2);
        L.six = take((size_t)(nnz + 4) * 2);
        L.ox = take(tiles * 4);
        L.ov = take(tiles * 4);
        L.oxq = take(tiles * 4);
        L.ovp = take(tiles * 4);
        L.lbs = take(((size_t)L.bp.P + 1) * 4);
        L.sbs = take(((size_t)L.bp.Q + 1) * 4);
        L.rlen = take((size_t)n);
        L.dlen = take((size_t)m);
    }
    L.total = off;
    return L;
}

std::vector<int> make_blocks(const std::vector<int> &ptr, int count)
{
    std::vector<int> blk;
    blk.reserve(count / 64 + 2);
    blk.push_back(0);
    int s = 0;
    while (s < count) {
        int e = s;
        long long cnt = 0;
        while (e < count && e - s < kBlock && cnt + (ptr[e + 1] - ptr[e]) <= kCap) {
            cnt += ptr[e + 1] - ptr[e];
            ++e;
        }
        if (e == s) e = s + 1;   // a segment longer than kCap on its own
        blk.push_back(e);
        s = e;
    }
    return blk;
}

std::string flag_text(unsigned f)
{
    std::string s;
    if (f & kErrRowPtr) s += "row_ptr must start at 0, end at nnz and be nondecreasing; ";
    if (f & kErrColRange) s += "col_idx out of range [0, n); ";
    if (f & kErrColOrder)
        s += "col_idx not strictly increasing within a row (duplicate link on a route "
             "would make R non-0/1); ";
    if (f & kErrCap) s += "capacities must be finite and > 0; ";
    if (f & kErrWeight) s += "weights must be finite and > 0; ";
    if (f & kErrUtility) s += "utility must be 0 (log), 1 (linear) or 2 (alpha = 2); ";
    if (f & kErrEmptyRoute) s += "a stream with an empty route needs a finite hi; ";
    return s;
}

}  // namespace

pmp_status pmp::set_error(pmp_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

struct pmp_handle {
    int m = 0, n = 0;
    long long nnz = 0;
    pmp_dtype dtype = PMP_F32;
    pmp_params prm{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = 0;                // device current at pmp_setup
    int *prune_scratch = nullptr;  // that device's fixed pruning scratch
    Dev<float> df{};
    Dev<double> dd{};
    Ctl *ctl = nullptr;            // device
    Ctl *ctl_host = nullptr;       // pinned, kSlots entries
    hipEvent_t ev[kSlots] = {};
    long long iter_enq = 0;        // iterations queued
    long long iter_fin = 0;        // iteration of the last queued check
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // reverse mode (pmp_forward_ckpt / pmp_backward)
    char *adj_ws = nullptr;
    size_t adj_bytes = 0;
    int adj_K = 0, adj_s = 0;
    bool adj_ready = false;
};

namespace {

template <typename T>
Dev<T> &dev_of(pmp_handle *h);
template <>
Dev<float> &dev_of<float>(pmp_handle *h) { return h->df; }
template <>
Dev<double> &dev_of<double>(pmp_handle *h) { return h->dd; }

pmp_status check_params(const pmp_params *p)
{
    if (!p) return fail(PMP_ERR_INVALID, "params is NULL");
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(PMP_ERR_INVALID, "rho0 must be > 0");
    if (!(p->alpha > 0.0 && p->alpha < 2.0)) return fail(PMP_ERR_INVALID, "alpha must be in (0, 2)");
    if (!(p->mu > 1.0) || !(p->gamma > 1.0)) return fail(PMP_ERR_INVALID, "mu and gamma must be > 1");
    if (!(p->eps_abs >= 0.0)) return fail(PMP_ERR_INVALID, "eps_abs must be >= 0");
    if (!(p->eps_rel >= 0.0) || !std::isfinite(p->eps_rel))
        return fail(PMP_ERR_INVALID, "eps_rel must be finite and >= 0");
    if (p->check_every < 1) return fail(PMP_ERR_INVALID, "check_every must be >= 1");
    if (p->adapt_every < 0 || (p->adapt_every > 0 && p->adapt_every % p->check_every != 0))
        return fail(PMP_ERR_INVALID, "adapt_every must be 0 or a multiple of check_every");
    if (p->max_iter < 0) return fail(PMP_ERR_INVALID, "max_iter must be >= 0");
    if (p->layout < PMP_LAYOUT_AUTO || p->layout > PMP_LAYOUT_BINNED)
        return fail(PMP_ERR_INVALID, "unknown layout");
    return PMP_OK;
}

pmp_status check_shape(const pmp_problem *p)
{
    if (!p) return fail(PMP_ERR_INVALID, "problem is NULL");
    if (p->m < 1 || p->n < 0) return fail(PMP_ERR_SHAPE, "m >= 1 and n >= 0 required");
    if (p->nnz < 0 || p->nnz >= (1LL << 31)) return fail(PMP_ERR_SHAPE, "nnz must be in [0, 2^31)");
    if (p->dtype != PMP_F32 && p->dtype != PMP_F64) return fail(PMP_ERR_INVALID, "unknown dtype");
    if (p->memory != PMP_MEM_HOST && p->memory != PMP_MEM_DEVICE)
        return fail(PMP_ERR_INVALID, "unknown memory kind");
    if (!(p->lo >= 0.0) || !std::isfinite(p->lo) || !(p->hi > p->lo) || std::isnan(p->hi))
        return fail(PMP_ERR_INVALID, "box must satisfy 0 <= lo < hi (lo finite)");
    if ((p->m > 0 && !p->row_ptr) || (p->nnz > 0 && !p->col_idx) || (p->m > 0 && !p->c) ||
        (p->n > 0 && (!p->w || !p->utility)))
        return fail(PMP_ERR_INVALID, "problem arrays must not be NULL");
    return PMP_OK;
}

template <typename T>
pmp_status setup_impl(pmp_handle *h, const pmp_problem *p, char *ws)
{
    const int m = p->m, n = p->n;
    const long long nnz = p->nnz;
    const Layout L = plan(m, n, nnz, sizeof(T), h->prm.layout);
    hipStream_t s = h->stream;
    Dev<T> &d = dev_of<T>(h);
    d.m = m;
    d.n = n;
    d.nnz = nnz;
    int *row_ptr = (int *)(ws + L.row_ptr);
    int *col_idx = (int *)(ws + L.col_idx);
    int *col_ptr = (int *)(ws + L.col_ptr);
    int *row_idx = (int *)(ws + L.row_idx);
    d.row_ptr = row_ptr;
    d.col_idx = col_idx;
    d.col_ptr = col_ptr;
    d.row_idx = row_idx;
    d.c = (T *)(ws + L.c);
    d.wsig = (T *)(ws + L.wsig);
    d.a = (T *)(ws + L.a);
    d.x = (T *)(ws + L.x);
    d.b = (T *)(ws + L.b);
    d.zs = (T *)(ws + L.zs);
    d.u = (T *)(ws + L.u);
    d.v = (T *)(ws + L.v);
    d.y_prev = (double *)(ws + L.y_prev);
    d.ps_prev = (double *)(ws + L.ps_prev);
    d.sblk = (int *)(ws + L.sblk);
    d.lblk = (int *)(ws + L.lblk);
    d.spart = (double *)(ws + L.spart);
    d.lpart = (double *)(ws + L.lpart);
    d.lck_beg = (int *)(ws + L.lck_beg);
    d.lck_end = (int *)(ws + L.lck_end);
    d.lr_row = (int *)(ws + L.lr_row);
    d.lr_ck = (int *)(ws + L.lr_ck);
    d.rpart = (double *)(ws + L.rpart);
    d.npart = (double *)(ws + L.npart);
    d.ctl = (Ctl *)(ws + L.ctl);
    d.hist = (HistEntry *)(ws + L.hist);
    d.lo = p->lo;
    d.hi = p->hi;
    d.alpha = h->prm.alpha;
    h->ctl = d.ctl;

    const double J = (double)nnz + (double)m;
    launch_ctl_init(d.ctl, h->prm.rho0, h->prm.eps_abs * std::sqrt(J), h->prm.eps_rel, h->prm.mu,
                    h->prm.gamma,
                    h->prm.adapt_every, s);

    // Inputs into the workspace.
    const hipMemcpyKind kind =
        p->memory == PMP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(row_ptr, p->row_ptr, ((size_t)m + 1) * 4, kind, s));
    if (nnz) HIP_TRY(hipMemcpyAsync(col_idx, p->col_idx, (size_t)nnz * 4, kind, s));
    const T *c_src = (const T *)p->c;
    const T *w_src = (const T *)p->w;
    const uint8_t *u_src = p->utility;
    if (p->memory == PMP_MEM_HOST) {
        if (m) HIP_TRY(hipMemcpyAsync((void *)d.c, p->c, (size_t)m * sizeof(T), kind, s));
        if (n) HIP_TRY(hipMemcpyAsync((void *)d.wsig, p->w, (size_t)n * sizeof(T), kind, s));
        if (n) HIP_TRY(hipMemcpyAsync(ws + L.util, p->utility, (size_t)n, kind, s));
        c_src = d.c;
        w_src = d.wsig;
        u_src = (const uint8_t *)(ws + L.util);
    }
    launch_validate_csr(row_ptr, col_idx, m, n, nnz, d.ctl, s);
    launch_check_vectors<T>(c_src, w_src, u_src, m, n, d.ctl, s);
    HIP_TRY(hipGetLastError());
    Ctl hc;
    HIP_TRY(hipMemcpyAsync(&hc, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hc.flags & ~kHasAlpha2)
        return fail(PMP_ERR_INVALID, "invalid problem: %s", flag_text(hc.flags).c_str());
    // utility codes stay on the device only when some stream is alpha = 2
    d.util = nullptr;
    if (hc.flags & kHasAlpha2) {
        if (u_src != (const uint8_t *)(ws + L.util))
            HIP_TRY(hipMemcpyAsync(ws + L.util, u_src, (size_t)n, hipMemcpyDeviceToDevice, s));
        d.util = (const uint8_t *)(ws + L.util);
    }

    // CSC pattern (setup step of the stream pass).
    launch_transpose(row_ptr, col_idx, m, n, nnz, col_ptr, row_idx, (int *)(ws + L.a), s);
    launch_check_routes(col_ptr, n, p->hi, d.ctl, s);
    launch_init_state<T>(d, c_src, w_src, u_src, s);
    HIP_TRY(hipGetLastError());

    // Workgroup tables from the two pointer arrays.
    std::vector<int> hrow((size_t)m + 1), hcol((size_t)n + 1);
    HIP_TRY(hipMemcpyAsync(hrow.data(), row_ptr, hrow.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hcol.data(), col_ptr, hcol.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hc, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hc.flags & ~kHasAlpha2)
        return fail(PMP_ERR_INVALID, "invalid problem: %s", flag_text(hc.flags).c_str());
    std::vector<int> sblk = make_blocks(hcol, n), lblk = make_blocks(hrow, m);
    d.nsb = (int)sblk.size() - 1;
    d.nlb = (int)lblk.size() - 1;
    if (d.nsb > L.nsb_max || d.nlb > L.nlb_max)
        return fail(PMP_ERR_SHAPE, "internal: block tables exceed their bound");
    HIP_TRY(hipMemcpyAsync((void *)d.sblk, sblk.data(), sblk.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((void *)d.lblk, lblk.data(), lblk.size() * 4, hipMemcpyHostToDevice, s));
    {
        // rows longer than kCap: chunks of kLongChunk nonzeros
        std::vector<int> cb, ce, lr, lck{0};
        long long maxlong = 0;
        for (int l = 0; l < m; ++l) {
            const int b = hrow[(size_t)l], e = hrow[(size_t)l + 1];
            if (e - b <= kCap) continue;
            maxlong = std::max<long long>(maxlong, e - b);
            for (int k = b; k < e; k += kLongChunk) {
                cb.push_back(k);
                ce.push_back(std::min(e, k + kLongChunk));
            }
            lr.push_back(l);
            lck.push_back((int)cb.size());
        }
        d.nlc = (int)cb.size();
        d.nlr = (int)lr.size();
        // Long rows in fixed point (FP32, finite box): with F chosen so that
        // (longest row) x hi x 2^F <= 2^62, every term and every partial sum
        // fits an int64.  A quantum 2^-F above 2^-24 (very large hi x row
        // length) would lose more than FP32 rounding: then FP64 sums are kept.
        d.fx_shift = long_row_shift(sizeof(T), maxlong, p->hi);
        d.fx_scale = std::ldexp(1.0, d.fx_shift);
        d.fx_inv = std::ldexp(1.0, -d.fx_shift);
        if (d.nlc > L.nlc_max || d.nlr > L.nlr_max)
            return fail(PMP_ERR_SHAPE, "internal: long-row tables exceed their bound");
        if (d.nlc) {
            HIP_TRY(hipMemcpyAsync((void *)d.lck_beg, cb.data(), cb.size() * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync((void *)d.lck_end, ce.data(), ce.size() * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync((void *)d.lr_row, lr.data(), lr.size() * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync((void *)d.lr_ck, lck.data(), lck.size() * 4, hipMemcpyHostToDevice, s));
        }
        HIP_TRY(hipStreamSynchronize(s));   // the host vectors go out of scope
    }
    d.binned = L.binned ? 1 : 0;
    if (L.binned) {
        // link blocks balanced by nonzeros, stream blocks by count; tile
        // offsets and local indices of the binned message layout
        BinnedPlan bp = L.bp;
        std::vector<int> lbs((size_t)L.bp.P + 1), sbs((size_t)L.bp.Q + 1);
        binned_blocks(hrow.data(), m, n, nnz, bp, lbs.data(), sbs.data());
        if (bp.P > L.bp.P || bp.Q > L.bp.Q || bp.LB > L.bp.LB || bp.SB > L.bp.SB)
            return fail(PMP_ERR_SHAPE, "internal: binned blocks exceed their bound");
        d.P = bp.P;
        d.Q = bp.Q;
        d.LB = bp.LB;
        d.SB = bp.SB;
        // stream blocks per dispatch round: one per CU when the stream blocks
        // outnumber the two per CU that are resident at once (rounds of 1/4
        // to 4 blocks per CU measured within 2% of each other on the large
        // workload, one per CU the fastest); otherwise all of them in one
        // round, so each XCD keeps a single run of consecutive blocks (split
        // rounds cost the paper-shape stream pass 6%)
        {
            int dev = 0, cus = 0;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            d.SR = d.Q <= 2 * cus ? std::max(1, d.Q) : std::max(8, cus);
        }
        d.lbs = (const int *)(ws + L.lbs);
        d.sbs = (const int *)(ws + L.sbs);
        // one byte per route length / link degree instead of two pointer
        // reads, when they all fit
        auto lengths = [&](const std::vector<int> &ptr, int count, size_t off,
                           const uint8_t *&out) -> pmp_status {
            std::vector<uint8_t> len((size_t)count);
            out = nullptr;
            for (int i = 0; i < count; ++i) {
                const int v = ptr[(size_t)i + 1] - ptr[(size_t)i];
                if (v > 255) return PMP_OK;
                len[(size_t)i] = (uint8_t)v;
            }
            HIP_TRY(hipMemcpyAsync(ws + off, len.data(), (size_t)count, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));   // len goes out of scope
            out = (const uint8_t *)(ws + off);
            return PMP_OK;
        };
        pmp_status ls = lengths(hcol, n, L.rlen, d.rlen);
        if (ls == PMP_OK) ls = lengths(hrow, m, L.dlen, d.dlen);
        if (ls != PMP_OK) return ls;
        d.mx = (T *)(ws + L.mx);
        d.mv = (T *)(ws + L.mv);
        d.lix = (const uint16_t *)(ws + L.lix);
        d.six = (const uint16_t *)(ws + L.six);
        d.ox = (const int *)(ws + L.ox);
        d.ov = (const int *)(ws + L.ov);
        d.oxq = (const int *)(ws + L.oxq);
        d.ovp = (const int *)(ws + L.ovp);
        HIP_TRY(hipMemcpyAsync((void *)d.lbs, lbs.data(), ((size_t)d.P + 1) * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void *)d.sbs, sbs.data(), ((size_t)d.Q + 1) * 4, hipMemcpyHostToDevice, s));
        if (binned_device_build_fits(bp) &&
            binned_build_scratch_ints(bp) * 4 <= (size_t)(nnz + 4) * sizeof(T)) {
            // tables built on the device; the message buffer is the scan scratch
            binned_build_device(d.row_ptr, col_idx, bp, d.lbs, (int *)d.ox, (int *)d.ov,
                                (int *)d.oxq, (int *)d.ovp, (uint16_t *)d.lix, (uint16_t *)d.six,
                                (int *)d.mx, d.fx_shift > 0, s);
        } else {
            const size_t tiles = (size_t)d.P * (size_t)d.Q + 1;
            std::vector<int> hcolidx((size_t)nnz);
            if (nnz) HIP_TRY(hipMemcpyAsync(hcolidx.data(), col_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            std::vector<int> ox(tiles), ov(tiles);
            std::vector<uint16_t> lix((size_t)nnz), six((size_t)nnz);
            binned_build_host(hrow.data(), hcolidx.data(), m, n, bp, lbs.data(), sbs.data(),
                              ox.data(), ov.data(), lix.data(), six.data(), d.fx_shift > 0);
            // each emission walks its destination offsets in its own block order
            std::vector<int> oxq(tiles - 1), ovp(tiles - 1);
            for (long long p = 0; p < d.P; ++p)
                for (long long q = 0; q < d.Q; ++q) {
                    oxq[(size_t)(q * d.P + p)] = ox[(size_t)(p * d.Q + q)];
                    ovp[(size_t)(p * d.Q + q)] = ov[(size_t)(q * d.P + p)];
                }
            HIP_TRY(hipMemcpyAsync((void *)d.ox, ox.data(), tiles * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync((void *)d.ov, ov.data(), tiles * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync((void *)d.oxq, oxq.data(), (tiles - 1) * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync((void *)d.ovp, ovp.data(), (tiles - 1) * 4, hipMemcpyHostToDevice, s));
            if (nnz) {
                HIP_TRY(hipMemcpyAsync((void *)d.lix, lix.data(), (size_t)nnz * 2, hipMemcpyHostToDevice, s));
                HIP_TRY(hipMemcpyAsync((void *)d.six, six.data(), (size_t)nnz * 2, hipMemcpyHostToDevice, s));
            }
            HIP_TRY(hipStreamSynchronize(s));   // the host tables go out of scope
        }
        if (nnz) HIP_TRY(hipMemsetAsync(d.mv, 0, (size_t)nnz * sizeof(T), s));   // v = 0 at the start
        binned_configure();
        HIP_TRY(hipStreamSynchronize(s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

// One pass of either layout.
// The stream pass; mode as for the link pass (the gather layout always
// stores x, the binned one only before and at checks).
template <typename T>
void stream_pass(const Dev<T> &d, int mode, hipStream_t s)
{
    if (d.binned) launch_bin_stream<T>(d, mode, s);
    else launch_stream_pass<T>(d, mode == kCheck, s);
}

// The link pass; a check also reduces its residual partials and decides
// (stop rule, rho balancing) right after it.
template <typename T>
void link_pass(const Dev<T> &d, int mode, long long delta, int stop, hipStream_t s)
{
    if (d.binned) launch_bin_link<T>(d, mode, s);
    else launch_link_pass<T>(d, mode, s);
    if (mode == kCheck)
        launch_check_finalize<T>(d, d.binned ? d.Q : d.nsb, d.binned ? d.P : d.nlb + d.nlr, delta,
                                 stop, s);
}

// After a check iteration: the u rescale of a balancing step, which only
// balancing iterations can need (the kernels return at once when rho did not
// change); the binned layout then also rewrites its link messages.
template <typename T>
void after_check(const Dev<T> &d, bool adapt_iteration, hipStream_t s)
{
    if (!adapt_iteration) return;
    if (d.binned) launch_bin_emit<T>(d, 1, s);
    else launch_rescale<T>(d, s);
}

// Refresh the link messages from v after v changed outside an iteration.
template <typename T>
void refresh_messages(const Dev<T> &d, hipStream_t s)
{
    if (d.binned) launch_bin_emit<T>(d, 0, s);
}

// Queue iterations [h->iter_enq + 1, h->iter_enq + k] without a stop test;
// residuals at the last one and at every balancing iteration.
template <typename T>
void enqueue_iterations(pmp_handle *h, int k, hipStream_t s)
{
    Dev<T> &d = dev_of<T>(h);
    const int adapt = h->prm.adapt_every;
    for (int i = 1; i <= k; ++i) {
        const long long it = h->iter_enq + 1;
        const bool check = i == k || (adapt > 0 && it % adapt == 0);
        const bool next_check = i < k && (i + 1 == k || (adapt > 0 && (it + 1) % adapt == 0));
        const int mode = check ? kCheck : (next_check ? kSave : kPlain);
        stream_pass<T>(d, mode, s);
        link_pass<T>(d, mode, it - h->iter_fin, 0, s);
        if (check) {
            h->iter_fin = it;
            after_check<T>(d, adapt > 0 && it % adapt == 0, s);
        }
        h->iter_enq = it;
    }
}

// One graph = check_every iterations ending in a check with the stop test.
template <typename T>
pmp_status build_graph(pmp_handle *h)
{
    Dev<T> &d = dev_of<T>(h);
    const int ce = h->prm.check_every;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 1; i <= ce; ++i) {
        const bool check = i == ce;
        const int mode = check ? kCheck : (i == ce - 1 ? kSave : kPlain);
        stream_pass<T>(d, mode, h->cap_stream);
        link_pass<T>(d, mode, ce, 1, h->cap_stream);
    }
    if (d.binned) launch_bin_emit<T>(d, 1, h->cap_stream);
    else launch_rescale<T>(d, h->cap_stream);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(h->cap_stream, &g));
    h->graph = g;
    HIP_TRY(hipGraphInstantiateWithFlags(&h->graph_exec, g, 0));
    return PMP_OK;
}

template <typename T>
pmp_status solve_impl(pmp_handle *h, pmp_result *out)
{
    hipStream_t s = h->stream;
    const int ce = h->prm.check_every;
    const long long start = h->iter_enq;
    long long budget = h->prm.max_iter;
    launch_ctl_clear_done(h->ctl, s);
    // Align chunks so that every check lands on a multiple of check_every.
    long long align = (ce - h->iter_enq % ce) % ce;
    if (align > budget) align = budget;
    if (align > 0) {
        enqueue_iterations<T>(h, (int)align, s);
        budget -= align;
    }
    HIP_TRY(hipGetLastError());
    if (!h->graph_exec) {
        pmp_status st = build_graph<T>(h);
        if (st != PMP_OK) return st;
    }
    const long long chunks = budget / ce;
    const long long leftover = budget % ce;
    bool done = false;
    long long launched = 0, waited = 0;
    while (!done && waited < chunks) {
        while (launched < chunks && launched - waited < kSlots) {
            HIP_TRY(hipGraphLaunch(h->graph_exec, s));
            const int slot = (int)(launched % kSlots);
            HIP_TRY(hipMemcpyAsync(&h->ctl_host[slot], h->ctl, sizeof(Ctl),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipEventRecord(h->ev[slot], s));
            ++launched;
        }
        const int slot = (int)(waited % kSlots);
        HIP_TRY(hipEventSynchronize(h->ev[slot]));
        ++waited;
        if (h->ctl_host[slot].done) done = true;
    }
    HIP_TRY(hipStreamSynchronize(s));
    Ctl c;
    HIP_TRY(hipMemcpy(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    h->iter_enq = h->iter_fin = c.iter;
    if (!c.done && leftover > 0) {
        enqueue_iterations<T>(h, (int)leftover, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipMemcpy(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    }
    pmp_status st = c.done ? (pmp_status)c.status : PMP_NOT_CONVERGED;
    if (out) {
        out->iterations = c.iter - start;
        out->r_norm = c.r_norm;
        out->s_norm = c.s_norm;
        out->eps_tol = c.eps_tol;
        out->rho = c.rho;
        out->status = st;
    }
    if (st == PMP_ERR_NUMERIC) return fail(st, "non-finite residual at iteration %lld", c.iter);
    return st;
}

}  // namespace

namespace {

// ---- reverse mode ----------------------------------------------------------

struct AdjLayout {
    size_t ckpt, final_state, xK, tape_x, tape_mu, A, Sbar, wbar, ext, B, Z, U, ybar, cbar;
    size_t my, ms;   // binned layout: messages of ybar and Sbar (problem precision)
    size_t part, J, total, state;
    int nck, nobj;
};

// msgs: message slots of the binned layout (0 for the gather layout)
AdjLayout adj_plan(int m, int n, long long msgs, int K, int s, size_t sz)
{
    AdjLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    L.nck = (K + s - 1) / s;
    L.nobj = (int)std::max<long long>(1, std::min<long long>(4096, ((long long)n + kBlock - 1) / kBlock));
    L.state = ((size_t)n + 3 * (size_t)m) * sz;
    L.ckpt = take((size_t)L.nck * L.state);
    L.final_state = take(L.state);
    L.xK = take((size_t)n * sz);
    L.tape_x = take((size_t)s * n * sz);
    L.tape_mu = take((size_t)s * m);
    L.A = take((size_t)n * 8);
    L.Sbar = take((size_t)n * 8);
    L.wbar = take((size_t)n * 8);
    L.ext = take((size_t)n * 8);
    L.B = take((size_t)m * 8);
    L.Z = take((size_t)m * 8);
    L.U = take((size_t)m * 8);
    L.ybar = take((size_t)m * 8);
    L.cbar = take((size_t)m * 8);
    L.part = take((size_t)L.nobj * 8);
    L.J = take(8);
    if (msgs > 0) {
        // messages in the problem's precision, with the 4 slots of padding
        // that the 4-wide FP32 loads of the accumulation may touch
        L.my = take((size_t)(msgs + 4) * sz);
        L.ms = take((size_t)(msgs + 4) * sz);
    }
    L.total = off;
    return L;
}

AdjLayout adj_plan_for(const pmp_handle *h, int K, int s)
{
    const int binned = h->dtype == PMP_F32 ? h->df.binned : h->dd.binned;
    return adj_plan(h->m, h->n, binned ? h->nnz : 0, K, s, h->dtype == PMP_F64 ? 8 : 4);
}

template <typename T>
pmp_status copy_state(pmp_handle *h, char *dst, bool save)
{
    Dev<T> &d = dev_of<T>(h);
    const size_t n = (size_t)h->n * sizeof(T), m = (size_t)h->m * sizeof(T);
    void *parts[4] = {d.a, d.b, d.zs, d.u};
    size_t sizes[4] = {n, m, m, m};
    size_t off = 0;
    for (int i = 0; i < 4; ++i) {
        if (sizes[i]) {
            if (save) HIP_TRY(hipMemcpyAsync(dst + off, parts[i], sizes[i], hipMemcpyDeviceToDevice, h->stream));
            else HIP_TRY(hipMemcpyAsync(parts[i], dst + off, sizes[i], hipMemcpyDeviceToDevice, h->stream));
        }
        off += sizes[i];
    }
    if (!save) launch_refresh_v<T>(d, h->stream);
    return PMP_OK;
}

AdjDev adj_views(char *ws, const AdjLayout &L)
{
    AdjDev a;
    a.A = (double *)(ws + L.A);
    a.Sbar = (double *)(ws + L.Sbar);
    a.wbar = (double *)(ws + L.wbar);
    a.ext = (double *)(ws + L.ext);
    a.B = (double *)(ws + L.B);
    a.Z = (double *)(ws + L.Z);
    a.U = (double *)(ws + L.U);
    a.ybar = (double *)(ws + L.ybar);
    a.cbar = (double *)(ws + L.cbar);
    return a;
}

template <typename T>
pmp_status forward_ckpt_impl(pmp_handle *h, int K, int s, char *ws, double *J)
{
    Dev<T> &d = dev_of<T>(h);
    const AdjLayout L = adj_plan_for(h, K, s);
    hipStream_t st = h->stream;
    pmp_status rc;
    launch_ctl_clear_done(h->ctl, st);
    // v from (b, u), and the binned layout's link messages from v (between
    // checks that layout keeps v in its messages only)
    launch_refresh_v<T>(d, st);
    refresh_messages<T>(d, st);
    for (int t = 1; t <= K; ++t) {
        if ((t - 1) % s == 0)
            if ((rc = copy_state<T>(h, ws + L.ckpt + (size_t)((t - 1) / s) * L.state, true)) != PMP_OK)
                return rc;
        stream_pass<T>(d, t == K ? kSave : kPlain, st);   // x^K stored
        link_pass<T>(d, kPlain, 0, 0, st);
    }
    // the K iterations count like any others (no check ran among them)
    h->iter_enq += K;
    h->iter_fin = h->iter_enq;
    launch_ctl_advance(h->ctl, K, st);
    launch_refresh_v<T>(d, st);   // v = b - u (the binned passes keep it in messages)
    if ((rc = copy_state<T>(h, ws + L.final_state, true)) != PMP_OK) return rc;
    if (h->n) HIP_TRY(hipMemcpyAsync(ws + L.xK, d.x, (size_t)h->n * sizeof(T), hipMemcpyDeviceToDevice, st));
    launch_objective<T>(d, (double *)(ws + L.part), L.nobj, (double *)(ws + L.J), st);
    HIP_TRY(hipGetLastError());
    double jv = 0.0;
    HIP_TRY(hipMemcpyAsync(&jv, ws + L.J, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (J) *J = jv;
    h->adj_ws = ws;
    h->adj_K = K;
    h->adj_s = s;
    h->adj_ready = true;
    return PMP_OK;
}

template <typename T>
pmp_status backward_impl(pmp_handle *h, T *gc, T *gw)
{
    Dev<T> &d = dev_of<T>(h);
    const int K = h->adj_K, s = h->adj_s;
    char *ws = h->adj_ws;
    const AdjLayout L = adj_plan_for(h, K, s);
    const AdjDev a = adj_views(ws, L);
    hipStream_t st = h->stream;
    pmp_status rc;
    T *tape_x = (T *)(ws + L.tape_x);
    uint8_t *tape_mu = (uint8_t *)(ws + L.tape_mu);
    T *my = (T *)(ws + L.my), *ms = (T *)(ws + L.ms);
    launch_ctl_clear_done(h->ctl, st);
    // adjoint seeds from x^K
    if (h->n) HIP_TRY(hipMemcpyAsync(d.x, ws + L.xK, (size_t)h->n * sizeof(T), hipMemcpyDeviceToDevice, st));
    launch_adj_init<T>(d, a, st);
    if (d.binned) launch_bin_adj_emit<T>(d, a, my, st);   // ybar = 0
    for (int seg = L.nck - 1; seg >= 0; --seg) {
        const int t0 = seg * s, t1 = std::min(t0 + s, K);
        if ((rc = copy_state<T>(h, ws + L.ckpt + (size_t)seg * L.state, false)) != PMP_OK) return rc;
        refresh_messages<T>(d, st);
        for (int t = t0 + 1; t <= t1; ++t) {            // recompute, recording x^t and mu^t
            // the passes of iteration t see the tape slot of x^t as their x:
            // the stream pass writes x^t there (kSave: x stored in both
            // layouts) and the gather layout's link pass reads it from there;
            // the handle's own x is restored from x^K at the end
            // and the link pass records the slack mask mu^t in its tape slot
            Dev<T> dt = d;
            if (h->n) dt.x = tape_x + (size_t)(t - t0 - 1) * h->n;
            dt.mu_out = tape_mu + (size_t)(t - t0 - 1) * h->m;
            stream_pass<T>(dt, kSave, st);
            link_pass<T>(dt, kPlain, 0, 0, st);
        }
        if (t1 < K) {   // link step of iteration t1, deferred from the later segment
            launch_adj_link_only<T>(d, a, tape_mu + (size_t)(t1 - t0 - 1) * h->m, st);
            if (d.binned) launch_bin_adj_emit<T>(d, a, my, st);
        }
        for (int t = t1; t > t0; --t) {
            const T *xt = tape_x + (size_t)(t - t0 - 1) * h->n;
            const uint8_t *mu_prev = t - 1 > t0 ? tape_mu + (size_t)(t - 2 - t0) * h->m : nullptr;
            if (d.binned) {
                launch_bin_adj_stream<T>(d, a, xt, t == K, my, ms, st);
                launch_bin_adj_link<T>(d, a, mu_prev, ms, my, st);
            } else {
                launch_adj_stream<T>(d, a, xt, t == K, st);
                launch_adj_link<T>(d, a, mu_prev, st);
            }
        }
    }
    launch_adj_out<T>(d, a, gc, gw, st);
    if ((rc = copy_state<T>(h, ws + L.final_state, false)) != PMP_OK) return rc;
    if (h->n) HIP_TRY(hipMemcpyAsync(d.x, ws + L.xK, (size_t)h->n * sizeof(T), hipMemcpyDeviceToDevice, st));
    refresh_messages<T>(d, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return PMP_OK;
}

}  // namespace

extern "C" {

pmp_status pmp_adjoint_workspace_size(pmp_handle *h, int32_t K, int32_t s, size_t *bytes)
{
    if (!h || !bytes || K < 1 || s < 1) return fail(PMP_ERR_INVALID, "bad argument");
    *bytes = adj_plan_for(h, K, s).total;
    return PMP_OK;
}

pmp_status pmp_forward_ckpt(pmp_handle *h, int32_t K, int32_t s, void *adj_workspace,
                            size_t adj_bytes, double *J)
{
    if (!h || K < 1 || s < 1) return fail(PMP_ERR_INVALID, "bad argument");
    const size_t need = adj_plan_for(h, K, s).total;
    if (!adj_workspace || adj_bytes < need)
        return fail(PMP_ERR_SHAPE, "adjoint workspace of %zu bytes needed, %zu given", need, adj_bytes);
    if ((uintptr_t)adj_workspace % kAlign) return fail(PMP_ERR_INVALID, "adjoint workspace must be 256-byte aligned");
    h->adj_ready = false;
    return h->dtype == PMP_F32 ? forward_ckpt_impl<float>(h, K, s, (char *)adj_workspace, J)
                               : forward_ckpt_impl<double>(h, K, s, (char *)adj_workspace, J);
}

pmp_status pmp_backward(pmp_handle *h, void *grad_c, void *grad_w)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    if (!h->adj_ready) return fail(PMP_ERR_STATE, "pmp_backward needs a preceding pmp_forward_ckpt");
    return h->dtype == PMP_F32 ? backward_impl<float>(h, (float *)grad_c, (float *)grad_w)
                               : backward_impl<double>(h, (double *)grad_c, (double *)grad_w);
}

pmp_status pmp_update_weights(pmp_handle *h, const void *w_new)
{
    if (!h || (!w_new && h->n)) return fail(PMP_ERR_INVALID, "NULL argument");
    if (h->n == 0) return PMP_OK;
    launch_ctl_clear_done(h->ctl, h->stream);
    if (h->dtype == PMP_F32) launch_copy_weights<float>(h->df, (const float *)w_new, h->stream);
    else launch_copy_weights<double>(h->dd, (const double *)w_new, h->stream);
    HIP_TRY(hipGetLastError());
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (c.flags & kErrWeight) return fail(PMP_ERR_INVALID, "weights must be finite and > 0");
    return PMP_OK;
}

}  // extern "C"

namespace {

template <typename T>
pmp_status time_kernels_impl(pmp_handle *h, int k, double *ms)
{
    Dev<T> &d = dev_of<T>(h);
    hipStream_t s = h->stream;
    const int adapt = h->prm.adapt_every;
    std::vector<hipEvent_t> ev(3 * (size_t)k, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ev)
                if (f) (void)hipEventDestroy(f);
            return fail(PMP_ERR_HIP, "hipEventCreate failed");
        }
    std::vector<int> is_check((size_t)k);
    launch_ctl_clear_done(h->ctl, s);
    for (int i = 1; i <= k; ++i) {
        const long long it = h->iter_enq + 1;
        const bool check = i == k || (adapt > 0 && it % adapt == 0);
        const bool next_check = i < k && (i + 1 == k || (adapt > 0 && (it + 1) % adapt == 0));
        is_check[i - 1] = check;
        const int mode = check ? kCheck : (next_check ? kSave : kPlain);
        (void)hipEventRecord(ev[3 * (i - 1)], s);
        stream_pass<T>(d, mode, s);
        (void)hipEventRecord(ev[3 * (i - 1) + 1], s);
        link_pass<T>(d, mode, it - h->iter_fin, 0, s);
        if (check) {
            h->iter_fin = it;
            after_check<T>(d, adapt > 0 && it % adapt == 0, s);
        }
        (void)hipEventRecord(ev[3 * (i - 1) + 2], s);
        h->iter_enq = it;
    }
    hipError_t e = hipStreamSynchronize(s);
    double acc[4] = {0, 0, 0, 0};
    int cnt[4] = {0, 0, 0, 0};
    for (int i = 0; e == hipSuccess && i < k; ++i) {
        float a = 0.f, b = 0.f;
        (void)hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]);
        (void)hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]);
        const int off = is_check[i] ? 2 : 0;
        acc[off] += a;
        acc[off + 1] += b;
        cnt[off] += 1;
        cnt[off + 1] += 1;
    }
    for (auto &f : ev) (void)hipEventDestroy(f);
    if (e != hipSuccess) return fail(PMP_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    for (int i = 0; i < 4; ++i) ms[i] = cnt[i] ? acc[i] / cnt[i] : 0.0;
    return PMP_OK;
}

}  // namespace

extern "C" {

pmp_status pmp_params_default(pmp_params *p)
{
    if (!p) return fail(PMP_ERR_INVALID, "params is NULL");
    p->rho0 = 1.0;
    p->alpha = 1.6;
    p->mu = 2.0;
    p->gamma = 1.1;
    p->eps_abs = 1e-4;
    p->adapt_every = 50;
    p->check_every = 10;
    p->max_iter = 100000;
    p->layout = PMP_LAYOUT_AUTO;
    p->eps_rel = 0.0;
    return PMP_OK;
}

pmp_status pmp_workspace_size(const pmp_problem *problem, const pmp_params *params,
                              size_t *bytes)
{
    if (!problem || !bytes) return fail(PMP_ERR_INVALID, "NULL argument");
    if (problem->m < 0 || problem->n < 0 || problem->nnz < 0 || problem->nnz >= (1LL << 31))
        return fail(PMP_ERR_SHAPE, "m, n >= 0 and 0 <= nnz < 2^31 required");
    const pmp_status st = check_binned_size(problem, params);
    if (st != PMP_OK) return st;
    const size_t sz = problem->dtype == PMP_F64 ? 8 : 4;
    *bytes = plan(problem->m, problem->n, problem->nnz, sz, params ? params->layout : 0).total;
    return PMP_OK;
}

pmp_status pmp_setup(const pmp_problem *problem, const pmp_params *params, void *workspace,
                     size_t workspace_bytes, void *stream, pmp_handle **out)
{
    if (!out) return fail(PMP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    pmp_status st = check_shape(problem);
    if (st != PMP_OK) return st;
    st = check_params(params);
    if (st != PMP_OK) return st;
    st = check_binned_size(problem, params);
    if (st != PMP_OK) return st;
    const size_t sz = problem->dtype == PMP_F64 ? 8 : 4;
    const Layout L = plan(problem->m, problem->n, problem->nnz, sz, params->layout);
    if (!workspace || workspace_bytes < L.total)
        return fail(PMP_ERR_SHAPE, "workspace of %zu bytes needed, %zu given", L.total,
                    workspace_bytes);
    if ((uintptr_t)workspace % kAlign)
        return fail(PMP_ERR_INVALID, "workspace must be 256-byte aligned");
    pmp_handle *h = new (std::nothrow) pmp_handle();
    if (!h) return fail(PMP_ERR_NOMEM, "handle allocation failed");
    h->m = problem->m;
    h->n = problem->n;
    h->nnz = problem->nnz;
    h->dtype = problem->dtype;
    h->prm = *params;
    h->stream = (hipStream_t)stream;
    auto cleanup = [&](pmp_status s2) {
        pmp_destroy(h);
        return s2;
    };
    if (hipGetDevice(&h->device) != hipSuccess)
        return cleanup(fail(PMP_ERR_HIP, "hipGetDevice failed"));
    // the fixed scratch of pmp_prune_noalloc on this device (looked up once)
    if (prune_static_scratch(h->device, &h->prune_scratch) != hipSuccess)
        return cleanup(fail(PMP_ERR_HIP, "hipGetSymbolAddress of the pruning scratch failed"));
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(PMP_ERR_HIP, "hipStreamCreateWithFlags failed"));
    if (hipHostMalloc((void **)&h->ctl_host, sizeof(Ctl) * kSlots, hipHostMallocDefault) !=
        hipSuccess)
        return cleanup(fail(PMP_ERR_HIP, "hipHostMalloc failed"));
    for (auto &e : h->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(PMP_ERR_HIP, "hipEventCreate failed"));
    st = problem->dtype == PMP_F32 ? setup_impl<float>(h, problem, (char *)workspace)
                                   : setup_impl<double>(h, problem, (char *)workspace);
    if (st != PMP_OK) return cleanup(st);
    *out = h;
    return PMP_OK;
}

pmp_status pmp_iterate(pmp_handle *h, int32_t k)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    if (k < 0) return fail(PMP_ERR_INVALID, "k must be >= 0");
    if (k == 0) return PMP_OK;
    launch_ctl_clear_done(h->ctl, h->stream);
    if (h->dtype == PMP_F32) enqueue_iterations<float>(h, k, h->stream);
    else enqueue_iterations<double>(h, k, h->stream);
    HIP_TRY(hipGetLastError());
    return PMP_OK;
}

pmp_status pmp_residuals(pmp_handle *h, double *r_norm, double *s_norm, int64_t *iteration)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (r_norm) *r_norm = c.r_norm;
    if (s_norm) *s_norm = c.s_norm;
    if (iteration) *iteration = c.iter;
    if (c.status == PMP_ERR_NUMERIC)
        return fail(PMP_ERR_NUMERIC, "non-finite residual at iteration %lld", c.iter);
    return PMP_OK;
}

pmp_status pmp_solve(pmp_handle *h, pmp_result *out)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    return h->dtype == PMP_F32 ? solve_impl<float>(h, out) : solve_impl<double>(h, out);
}

pmp_status pmp_get_solution(pmp_handle *h, void *x, void *lambda, void *slack)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    if (h->dtype == PMP_F32)
        launch_solution<float>(h->df, (float *)x, (float *)lambda, (float *)slack, h->stream);
    else
        launch_solution<double>(h->dd, (double *)x, (double *)lambda, (double *)slack, h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    return PMP_OK;
}

pmp_status pmp_get_path_prices(pmp_handle *h, void *pi)
{
    if (!h || !pi) return fail(PMP_ERR_INVALID, "NULL argument");
    if (h->dtype == PMP_F32)
        launch_path_prices<float>(h->df, (float *)pi, h->stream);
    else
        launch_path_prices<double>(h->dd, (double *)pi, h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    return PMP_OK;
}

pmp_status pmp_prune_workspace_size(pmp_handle *h, size_t *bytes)
{
    if (!h || !bytes) return fail(PMP_ERR_INVALID, "NULL argument");
    *bytes = prune_scratch_ints(h->m, h->n) * 4;
    return PMP_OK;
}

pmp_status pmp_prune(pmp_handle *h, const uint8_t *failed, void *workspace,
                     size_t workspace_bytes, int32_t *row_ptr, int32_t *col_idx, void *c,
                     void *w, uint8_t *utility, int32_t *link_map, int32_t *stream_map,
                     void *state, int64_t *sizes)
{
    if (!h || !failed || !workspace || !row_ptr || !c || !link_map || !state || !sizes)
        return fail(PMP_ERR_INVALID, "NULL argument");
    if ((h->nnz > 0 && !col_idx) || (h->n > 0 && (!w || !utility || !stream_map)))
        return fail(PMP_ERR_INVALID, "NULL argument");
    if (workspace_bytes < prune_scratch_ints(h->m, h->n) * 4)
        return fail(PMP_ERR_INVALID, "workspace of %zu bytes is below the %zu required",
                    workspace_bytes, prune_scratch_ints(h->m, h->n) * 4);
    long long sz[3] = {0, 0, 0};
    hipError_t e;
    if (h->dtype == PMP_F32)
        e = prune_device<float>(h->df, failed, (int *)workspace, row_ptr, col_idx, (float *)c,
                                (float *)w, utility, link_map, stream_map, (char *)state, sz,
                                h->stream);
    else
        e = prune_device<double>(h->dd, failed, (int *)workspace, row_ptr, col_idx, (double *)c,
                                 (double *)w, utility, link_map, stream_map, (char *)state, sz,
                                 h->stream);
    if (e != hipSuccess) return fail(PMP_ERR_HIP, "pruning failed: %s", hipGetErrorString(e));
    for (int i = 0; i < 3; ++i) sizes[i] = sz[i];
    return PMP_OK;
}

pmp_status pmp_prune_noalloc(pmp_handle *h, const uint8_t *failed, int32_t *row_ptr,
                             int32_t *col_idx, void *c, void *w, uint8_t *utility,
                             int32_t *link_map, int32_t *stream_map, void *state, int64_t *sizes)
{
    if (!h) return fail(PMP_ERR_INVALID, "NULL argument");
    const size_t need = prune_scratch_ints(h->m, h->n) * 4;
    if (need > kPruneStaticBytes)
        return fail(PMP_ERR_SHAPE,
                    "pmp_prune_noalloc: %zu bytes of scratch needed, the fixed maximum is %zu "
                    "(use pmp_prune with a workspace)", need, kPruneStaticBytes);
    if (!h->prune_scratch) return fail(PMP_ERR_STATE, "pruning scratch not set up");
    return pmp_prune(h, failed, h->prune_scratch, need, row_ptr, col_idx, c, w, utility,
                     link_map, stream_map, state, sizes);
}

pmp_status pmp_state_size(pmp_handle *h, size_t *bytes)
{
    if (!h || !bytes) return fail(PMP_ERR_INVALID, "NULL argument");
    const size_t sz = h->dtype == PMP_F64 ? 8 : 4;
    *bytes = ((size_t)h->n + 3 * (size_t)h->m) * sz + 16;
    return PMP_OK;
}

pmp_status pmp_get_state(pmp_handle *h, void *state)
{
    if (!h || !state) return fail(PMP_ERR_INVALID, "NULL argument");
    const size_t sz = h->dtype == PMP_F64 ? 8 : 4;
    char *p = (char *)state;
    void *a, *b, *zs, *u;
    if (h->dtype == PMP_F32) { a = h->df.a; b = h->df.b; zs = h->df.zs; u = h->df.u; }
    else { a = h->dd.a; b = h->dd.b; zs = h->dd.zs; u = h->dd.u; }
    hipStream_t s = h->stream;
    const size_t n = (size_t)h->n * sz, m = (size_t)h->m * sz;
    if (n) HIP_TRY(hipMemcpyAsync(p, a, n, hipMemcpyDeviceToDevice, s));
    if (m) {
        HIP_TRY(hipMemcpyAsync(p + n, b, m, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(p + n + m, zs, m, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(p + n + 2 * m, u, m, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(p + n + 3 * m, &h->ctl->rho, 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(p + n + 3 * m + 8, &h->ctl->iter, 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

pmp_status pmp_set_state(pmp_handle *h, const void *state)
{
    if (!h || !state) return fail(PMP_ERR_INVALID, "NULL argument");
    const size_t sz = h->dtype == PMP_F64 ? 8 : 4;
    const char *p = (const char *)state;
    void *a, *b, *zs, *u;
    if (h->dtype == PMP_F32) { a = h->df.a; b = h->df.b; zs = h->df.zs; u = h->df.u; }
    else { a = h->dd.a; b = h->dd.b; zs = h->dd.zs; u = h->dd.u; }
    hipStream_t s = h->stream;
    const size_t n = (size_t)h->n * sz, m = (size_t)h->m * sz;
    if (n) HIP_TRY(hipMemcpyAsync(a, p, n, hipMemcpyDeviceToDevice, s));
    if (m) {
        HIP_TRY(hipMemcpyAsync(b, p + n, m, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(zs, p + n + m, m, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(u, p + n + 2 * m, m, hipMemcpyDeviceToDevice, s));
    }
    double rho;
    long long it;
    HIP_TRY(hipMemcpyAsync(&rho, p + n + 3 * m, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&it, p + n + 3 * m + 8, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!(rho > 0.0) || !std::isfinite(rho)) return fail(PMP_ERR_INVALID, "state rho must be > 0");
    if (it < 0) return fail(PMP_ERR_INVALID, "state iteration must be >= 0");
    // Re-seed the control block (keeping the tolerances) and v = b - u.
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    launch_ctl_init(h->ctl, rho, c.eps_tol, c.eps_rel, c.mu, c.gamma, c.adapt_every, s);
    HIP_TRY(hipMemcpyAsync(&h->ctl->iter, &it, 8, hipMemcpyHostToDevice, s));
    if (h->dtype == PMP_F32) {
        launch_refresh_v<float>(h->df, s);
        refresh_messages<float>(h->df, s);
    } else {
        launch_refresh_v<double>(h->dd, s);
        refresh_messages<double>(h->dd, s);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    h->iter_enq = h->iter_fin = it;
    return PMP_OK;
}

pmp_status pmp_update_params(pmp_handle *h, const pmp_params *params)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    pmp_status st = check_params(params);
    if (st != PMP_OK) return st;
    if (params->alpha != h->prm.alpha || params->check_every != h->prm.check_every ||
        params->adapt_every != h->prm.adapt_every || params->layout != h->prm.layout)
        return fail(PMP_ERR_INVALID, "alpha, check_every, adapt_every and layout are fixed at setup");
    h->prm.eps_abs = params->eps_abs;
    h->prm.eps_rel = params->eps_rel;
    h->prm.mu = params->mu;
    h->prm.gamma = params->gamma;
    h->prm.max_iter = params->max_iter;
    const double J = (double)h->nnz + (double)h->m;
    launch_ctl_set_tolerances(h->ctl, params->eps_abs * std::sqrt(J), params->eps_rel, params->mu,
                              params->gamma,
                              h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    return PMP_OK;
}

pmp_status pmp_time_kernels(pmp_handle *h, int32_t k, double *ms)
{
    if (!h || !ms || k < 1) return fail(PMP_ERR_INVALID, "bad argument");
    return h->dtype == PMP_F32 ? time_kernels_impl<float>(h, k, ms)
                               : time_kernels_impl<double>(h, k, ms);
}

pmp_status pmp_history(pmp_handle *h, double *out, int32_t capacity, int32_t *count)
{
    if (!h || !count || capacity < 0 || (capacity > 0 && !out))
        return fail(PMP_ERR_INVALID, "bad argument");
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const long long avail = std::min<long long>(c.nhist, kHist);
    const int take = (int)std::min<long long>(avail, capacity);
    std::vector<HistEntry> buf((size_t)kHist);
    const HistEntry *dh = h->dtype == PMP_F32 ? h->df.hist : h->dd.hist;
    HIP_TRY(hipMemcpy(buf.data(), dh, sizeof(HistEntry) * kHist, hipMemcpyDeviceToHost));
    for (int i = 0; i < take; ++i) {        // oldest retained entry first
        const long long idx = (c.nhist - take + i) % kHist;
        out[4 * i] = (double)buf[(size_t)idx].iter;
        out[4 * i + 1] = buf[(size_t)idx].r_norm;
        out[4 * i + 2] = buf[(size_t)idx].s_norm;
        out[4 * i + 3] = buf[(size_t)idx].rho;
    }
    *count = take;
    return PMP_OK;
}

pmp_status pmp_update_capacity(pmp_handle *h, const void *c_new)
{
    if (!h || !c_new) return fail(PMP_ERR_INVALID, "NULL argument");
    if (h->dtype == PMP_F32) launch_copy_capacity<float>(h->df, (const float *)c_new, h->stream);
    else launch_copy_capacity<double>(h->dd, (const double *)c_new, h->stream);
    HIP_TRY(hipGetLastError());
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (c.flags & kErrCap) return fail(PMP_ERR_INVALID, "capacities must be finite and > 0");
    return PMP_OK;
}

pmp_status pmp_device_views(pmp_handle *h, void **x, void **u, void **a, void **b, void **zs,
                            void **v)
{
    if (!h) return fail(PMP_ERR_INVALID, "handle is NULL");
    if (h->dtype == PMP_F32) {
        if (x) *x = h->df.x;
        if (u) *u = h->df.u;
        if (a) *a = h->df.a;
        if (b) *b = h->df.b;
        if (zs) *zs = h->df.zs;
        if (v) *v = h->df.v;
    } else {
        if (x) *x = h->dd.x;
        if (u) *u = h->dd.u;
        if (a) *a = h->dd.a;
        if (b) *b = h->dd.b;
        if (zs) *zs = h->dd.zs;
        if (v) *v = h->dd.v;
    }
    return PMP_OK;
}

pmp_status pmp_get_layout(pmp_handle *h, int32_t *layout)
{
    if (!h || !layout) return fail(PMP_ERR_INVALID, "NULL argument");
    const int b = h->dtype == PMP_F32 ? h->df.binned : h->dd.binned;
    *layout = b ? PMP_LAYOUT_BINNED : PMP_LAYOUT_GATHER;
    return PMP_OK;
}

pmp_status pmp_destroy(pmp_handle *h)
{
    if (!h) return PMP_OK;
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return PMP_OK;
}

const char *pmp_status_string(pmp_status s)
{
    switch (s) {
    case PMP_OK: return "ok";
    case PMP_ERR_INVALID: return "invalid argument";
    case PMP_ERR_SHAPE: return "shape or size error";
    case PMP_ERR_NOMEM: return "out of host memory";
    case PMP_ERR_HIP: return "HIP runtime error";
    case PMP_ERR_NUMERIC: return "non-finite residual";
    case PMP_NOT_CONVERGED: return "not converged";
    case PMP_ERR_STATE: return "invalid handle state";
    }
    return "unknown status";
}

const char *pmp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
