// Internal definitions shared by the PMP host layer and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#include "pmp.h"

namespace pmp {

// Workgroup shape of the stream and link passes: one wave64 x 4.
constexpr int kBlock = 256;
// Entries of R staged in LDS per workgroup (index stream + gathered values).
// A workgroup covers at most kBlock streams (links) and at most kCap
// nonzeros, or a single longer column (row) on its own.
constexpr int kCap = 4096;
// A link whose row holds more than kCap nonzeros (a congested link) is summed
// by several workgroups, one per chunk of kLongChunk nonzeros; a second
// kernel adds the chunk sums in chunk order and runs the link update.
constexpr int kLongChunk = 8192;
// Shift F of the fixed-point long-row sums (Dev::fx_shift) of a problem with
// element size `elem`, longest long row `maxlong` (0 if none) and box upper
// bound `hi`: the largest F with maxlong x hi x 2^F <= 2^62 (so every term and
// partial sum fits an int64), at most 126.  0 (plain FP64 sums) for FP64
// problems, without long rows, with an unbounded box, or where F would fall
// below 24 (a quantum 2^-F coarser than FP32 rounding).
inline int long_row_shift(size_t elem, long long maxlong, double hi)
{
    if (elem != 4 || maxlong <= 0 || !std::isfinite(hi) || !(hi > 0.0)) return 0;
    const int F = std::min((int)std::floor(62.0 - std::log2((double)maxlong * hi)), 126);
    return F >= 24 ? F : 0;
}
// Device history ring of (iteration, ||r||, ||s||, rho), one entry per check.
constexpr int kHist = 4096;
// Threads of the kernel that reduces the residual partials of a check.
constexpr int kFinThreads = 1024;
// Workgroups of the norm pass of a check with a relative stop rule.
constexpr int kNormBlocks = 256;

// Device-resident control block.  Kernels read rho and the done flag from
// here, so a captured graph stays valid while rho changes (Section III-G
// balancing happens on the device).
struct Ctl {
    double rho;            // penalty of the next iteration
    double ratio;          // pending u rescale rho_old / rho_new (1 = none)
    double r_norm;         // ||r|| at the last check
    double s_norm;         // ||s|| at the last check
    double eps_tol;        // eps_abs sqrt(J)
    double eps_rel;        // relative part of the stop rule (0 = absolute only)
    double p_norm, z_norm, u_norm;   // ||p||, ||z||, ||rho u|| at the last check (eps_rel > 0)
    double mu, gamma;      // balancing thresholds
    long long iter;        // iterations completed at the last check
    long long nhist;       // checks recorded in the history ring
    int adapt_every;       // 0 = fixed rho
    int done;              // 1: stop rule met or numeric failure
    int status;            // pmp_status of the last check
    unsigned int arrive;   // arrival counter of the last-workgroup finalize
    unsigned int flags;    // setup validation error bits
    int pad;
};

struct HistEntry {
    long long iter;
    double r_norm, s_norm, rho;
};

// Setup validation error bits.
enum : unsigned {
    kErrRowPtr = 1u << 0,
    kErrColRange = 1u << 1,
    kErrColOrder = 1u << 2,
    kErrCap = 1u << 3,
    kErrWeight = 1u << 4,
    kErrUtility = 1u << 5,
    kErrEmptyRoute = 1u << 6,
    kHasAlpha2 = 1u << 16,   // not an error: some stream has the alpha = 2 utility
};

// Link-pass flavours: PLAIN does the PMP update only; SAVE also keeps y and
// ps for the next iteration's residual; CHECK forms per-workgroup residual
// partials against the saved values and keeps the new ones.  The check's
// finalize kernel then reduces the partials and takes the stop and rho
// decisions.
enum LinkMode : int { kPlain = 0, kSave = 1, kCheck = 2 };

// Device pointers of one instance (all inside the caller's workspace).
template <typename T>
struct Dev {
    int m, n;
    long long nnz;
    const int *row_ptr, *col_idx;   // CSR
    const int *col_ptr, *row_idx;   // CSC
    const T *c;                     // [m]
    const T *wsig;                  // [n] w for log / alpha = 2 streams, -w for linear
    const uint8_t *util;            // [n] utility codes, or NULL when no stream is alpha = 2
    T *a, *x;                       // [n]
    T *b, *zs, *u, *v;              // [m]
    double *y_prev, *ps_prev;       // [m] saved link sums / slack prox
    const int *sblk;                // [nsb+1] stream workgroup boundaries
    const int *lblk;                // [nlb+1] link workgroup boundaries
    int nsb, nlb;
    double *spart;                  // [nsb]   stream residual partials
    double *lpart;                  // [2 (nlb + nlr)] link residual partials
    int nlc, nlr;                   // chunks of long rows, long rows
    const int *lck_beg, *lck_end;   // [nlc] nonzero range of each chunk
    const int *lr_row, *lr_ck;      // [nlr], [nlr + 1] long rows and their chunks
    double *rpart;                  // [nlc] chunk sums
    double *npart;                  // [kNormBlocks * 5] partials of the norms of a check
    double lo, hi, alpha;
    // Long rows (more than kCap nonzeros, congested links) of FP32 problems
    // with a finite box are summed in fixed point: each rate x becomes the
    // integer llrint(x 2^fx_shift) and the row sum is the exact int64 sum of
    // those, times 2^-fx_shift.  Integer sums do not depend on the order of
    // the adds, so these rows come out the same in both layouts and in every
    // run.  fx_shift = 0: plain FP64 sums.
    int fx_shift;
    double fx_scale, fx_inv;        // 2^fx_shift, 2^-fx_shift
    Ctl *ctl;
    HistEntry *hist;
    // When set (reverse mode's recomputation), the link pass also writes the
    // slack-prox mask [zs - u > -c] of each link here.
    uint8_t *mu_out;
    // Binned message layout (pmp_binned.hip); P link blocks of at most LB
    // links and Q stream blocks of at most SB streams tile R into P x Q tiles.
    int binned;                     // 1: iterations use the binned kernels
    int P, Q, LB, SB;
    int SR;                         // stream blocks per dispatch round of the stream pass
    const int *lbs, *sbs;           // [P+1], [Q+1] first link / stream of each block
    const uint8_t *rlen;            // [n] route lengths when all are below 256, else NULL
    const uint8_t *dlen;            // [m] link degrees when all are below 256, else NULL
    T *mx;                          // [nnz] stream -> link messages, tiles p-major
    T *mv;                          // [nnz] link -> stream messages, tiles q-major
    const uint16_t *lix;            // [nnz] local link of each mx entry
    const uint16_t *six;            // [nnz] local stream of each mv entry
    const int *ox;                  // [P Q + 1] tile offsets in mx, p-major
    const int *ov;                  // [Q P + 1] tile offsets in mv, q-major
    const int *oxq;                 // [Q P] the offsets of ox listed q-major
    const int *ovp;                 // [P Q] the offsets of ov listed p-major
};

// Adjoint (reverse-mode) vectors, all FP64, in the adjoint workspace.
struct AdjDev {
    double *A;       // [n] adjoint of a
    double *Sbar;    // [n] adjoint of S of the current reverse iteration
    double *wbar;    // [n] dJ/dw accumulator
    double *ext;     // [n] dJ/dx^K
    double *B, *Z, *U;   // [m] adjoints of b, zs, u
    double *ybar;    // [m] adjoint of the link sums y
    double *cbar;    // [m] dJ/dc accumulator
};

// Launchers (pmp_kernels.hip).
template <typename T>
void launch_stream_pass(const Dev<T> &d, bool check, hipStream_t s);
template <typename T>
void launch_link_pass(const Dev<T> &d, int mode, hipStream_t s);
// Reduce the partials of a check (nspart stream, nlpart link workgroups) and
// take the stop / rho decisions.
template <typename T>
void launch_check_finalize(const Dev<T> &d, int nspart, int nlpart, long long delta, int stop,
                           hipStream_t s);
template <typename T>
void launch_rescale(const Dev<T> &d, hipStream_t s);
template <typename T>
void launch_refresh_v(const Dev<T> &d, hipStream_t s);
template <typename T>
void launch_zero_state(const Dev<T> &d, hipStream_t s);
template <typename T>
void launch_init_state(const Dev<T> &d, const T *c_in, const T *w_in, const uint8_t *util,
                       hipStream_t s);
template <typename T>
void launch_check_vectors(const T *c, const T *w, const uint8_t *util, int m, int n,
                          Ctl *ctl, hipStream_t s);
template <typename T>
void launch_solution(const Dev<T> &d, T *x, T *lambda, T *slack, hipStream_t s);
// Clear `bit` in ctl->flags, then set it if some v[i] is not finite and > 0.
template <typename T>
void launch_check_positive(const T *v, int count, Ctl *ctl, unsigned bit, hipStream_t s);
// c <- c_new, unless launch_check_positive (queued first) rejected c_new.
template <typename T>
void launch_copy_capacity(const Dev<T> &d, const T *c_new, hipStream_t s);
template <typename T>
void launch_path_prices(const Dev<T> &d, T *pi, hipStream_t s);

// Link failure compaction (pmp_prune.hip).  scratch holds
// prune_scratch_ints(m, n) ints; sizes receives m', n', nnz'.  Synchronises s.
size_t prune_scratch_ints(int m, int n);
// The fixed scratch of pmp_prune_noalloc: kPruneStaticBytes on every device,
// its address on `device` looked up once (with that device current) and
// kept.  All its contents are written before they are read by each call.
constexpr size_t kPruneStaticBytes = (size_t)16 << 20;
hipError_t prune_static_scratch(int device, int **ptr);
template <typename T>
hipError_t prune_device(const Dev<T> &d, const uint8_t *failed, int *scratch, int *row_ptr,
                        int *col_idx, T *c, T *w, uint8_t *util, int *link_map, int *stream_map,
                        char *state, long long sizes[3], hipStream_t s);

// Binned layout (pmp_binned.hip).
#ifndef PMP_BIN_THREADS
#define PMP_BIN_THREADS 1024
#endif
#ifndef PMP_BIN_MAX_BLOCK
#define PMP_BIN_MAX_BLOCK 10112   // two workgroups' FP64 sums fit one CU's 160 KiB LDS
#endif
constexpr int kBinThreads = PMP_BIN_THREADS;       // threads per binned workgroup
constexpr int kBinMaxBlock = PMP_BIN_MAX_BLOCK;    // links / streams per binned workgroup
// A link-side local index (lix) carries kLongBit when its link is a long row
// (more than kCap nonzeros) whose sum is formed in fixed point (Dev::fx_shift).
constexpr uint16_t kLongBit = 0x8000;
constexpr uint16_t kLocalMask = 0x7fff;
static_assert(kBinMaxBlock <= kLocalMask, "local indices must leave the top bit free");
struct BinnedPlan {
    int P, Q;     // link blocks, stream blocks
    int LB, SB;   // most links / streams in one block (LDS sums per workgroup)
};
// Bounds of the plan from the sizes alone (workspace sizing).
BinnedPlan binned_plan(int m, int n, long long nnz);
// Block boundaries lbs[P+1] of the links, balanced by nonzeros (a block
// closes once it holds the nonzero quota or its row cap), and sbs[Q+1] of
// the streams, by count (stream j is in block j / SB); sets P, Q, LB, SB of
// bp to the actual values (within the bounds of binned_plan).
void binned_blocks(const int *row_ptr, int m, int n, long long nnz, BinnedPlan &bp, int *lbs,
                   int *sbs);
// Host construction of ox, ov, lix, six from the CSR pattern and the blocks.
// With mark_long, lix entries of rows longer than kCap carry kLongBit.
void binned_build_host(const int *row_ptr, const int *col_idx, int m, int n, const BinnedPlan &bp,
                       const int *lbs, const int *sbs, int *ox, int *ov, uint16_t *lix,
                       uint16_t *six, int mark_long);
// Device construction of the same tables (ox, ov, the reordered offsets
// oxq, ovp, and lix, six) from the device CSR pattern and block starts lbs;
// inside a tile the nonzeros are grouped by link, each link's in column
// order.  Possible when the Q stream-block counters fit one workgroup's LDS
// (binned_device_build_fits); scratch holds binned_build_scratch_ints ints.
constexpr size_t kBinBuildLds = 32768;
bool binned_device_build_fits(const BinnedPlan &bp);
size_t binned_build_scratch_ints(const BinnedPlan &bp);
void binned_build_device(const int *row_ptr, const int *col_idx, const BinnedPlan &bp,
                         const int *lbs, int *ox, int *ov, int *oxq, int *ovp, uint16_t *lix,
                         uint16_t *six, int *scratch, int mark_long, hipStream_t s);
// Exclusive scan of in[n] into out[n + 1] (out[0] = 0); bsum holds
// scan_scratch_ints(n) ints.
size_t scan_scratch_ints(int n);
void launch_scan_int(const int *in, int n, int *out, int *bsum, hipStream_t s);
// mode: kPlain (x stays in the messages), kSave (x also stored, for the
// next iteration's check), kCheck (residual partials; x stored)
template <typename T>
void launch_bin_stream(const Dev<T> &d, int mode, hipStream_t s);
template <typename T>
void launch_bin_link(const Dev<T> &d, int mode, hipStream_t s);
template <typename T>
void launch_bin_emit(const Dev<T> &d, int apply, hipStream_t s);
void binned_configure();
// Reverse mode in the binned layout: my holds ybar in the v-message layout,
// ms holds Sbar in the x-message layout (the problem's precision, one per
// nonzero each, summed in FP64).
template <typename T>
void launch_bin_adj_stream(const Dev<T> &d, const AdjDev &a, const T *xt, int last,
                           const T *my, T *ms, hipStream_t s);
template <typename T>
void launch_bin_adj_link(const Dev<T> &d, const AdjDev &a, const uint8_t *mu_prev,
                         const T *ms, T *my, hipStream_t s);
template <typename T>
void launch_bin_adj_emit(const Dev<T> &d, const AdjDev &a, T *my, hipStream_t s);

// Batched solve (pmp_batch.hip): many instances concatenated block-diagonally
// into one global pattern, iterated together by one persistent kernel with
// per-instance rho, residuals, stop flags and iteration counters.
template <typename T>
struct BDev {
    Dev<T> g;                  // concatenated arrays; CSR/CSC with global indices
    int B;                     // instances
    const int *link_off;       // [B+1]
    const int *stream_off;     // [B+1]
    const double *lo, *hi;     // [B] boxes
    Ctl *ictl;                 // [B] per-instance control blocks
    HistEntry *hist;           // [B * kHist]
    int nst, nlt;              // stream / link tiles (never straddle instances)
    const int *st_seg;         // [nst+1] first stream of each tile
    const int *st_inst;        // [nst]
    const int *lt_seg;         // [nlt+1]
    const int *lt_inst;        // [nlt]
    const int *inst_st;        // [B+1] first stream tile of each instance
    const int *inst_lt;        // [B+1] first link tile of each instance
    double *st_part;           // [nst]
    double *lt_part;           // [2 nlt]
    // Link rows longer than kCap (congested links) are split into chunk tiles
    // of heavy_chunk nonzeros: lt_ck[t] = {chunk, chunks of the row} for such
    // a tile ({0, 0} otherwise), and every chunk tile of a row starts at that
    // row in lt_seg.  A chunk tile leaves its sum in lt_hsum[t] (FP64 bits,
    // or int64 in fixed point); the workgroup that counts the row's last
    // arrival in lt_hcnt[first chunk tile] adds the sums in chunk order and
    // runs the link update.
    const int2 *lt_ck;         // [nlt]
    long long *lt_hsum;        // [nlt]
    unsigned *lt_hcnt;         // [nlt]
    int heavy_chunk;
    unsigned long long spin_limit;   // polls of a barrier wait before it gives up
    const int *ifx_shift;      // [B] fixed-point shift of each instance's long rows
    const double *ifx_scale;   // [B] 2^shift
    const double *ifx_inv;     // [B] 2^-shift
    unsigned *bar;             // grid barrier: counters, generation (pmp_batch.hip)
    int *abort;                // set when a barrier wait exceeds its bound
    unsigned long long *prof;  // [grid * kBatchPhases] phase clocks, or NULL
};

// Phases of the batch kernel timed with pmp_batch_options.profile: stream
// tiles, wait at the barrier after them, link tiles, wait after them,
// finalize with its barrier, rescale with its barrier.
constexpr int kBatchPhases = 6;
constexpr int kBatchMaxGrid = 4096;   // persistent workgroups at most (8 per CU)


template <typename T>
void launch_batch(const BDev<T> &d, int grid, int max_iter, int check_every, int adapt_every,
                  hipStream_t s);
template <typename T>
int batch_grid_size(int device, int want_per_cu);
template <typename T>
void launch_batch_gather_x(const T *x, const int *pos, int n, T *out, hipStream_t s);

// Error text for the C ABI (pmp_api.hip).
pmp_status set_error(pmp_status s, const char *fmt, ...);

// Adjoint launchers (pmp_adjoint.hip).
template <typename T>
void launch_adj_stream(const Dev<T> &d, const AdjDev &a, const T *xt, int last, hipStream_t s);
template <typename T>
void launch_adj_link(const Dev<T> &d, const AdjDev &a, const uint8_t *mu_prev, hipStream_t s);
template <typename T>
void launch_adj_link_only(const Dev<T> &d, const AdjDev &a, const uint8_t *mu, hipStream_t s);
template <typename T>
void launch_objective(const Dev<T> &d, double *part, int nblocks, double *out, hipStream_t s);
template <typename T>
void launch_adj_init(const Dev<T> &d, const AdjDev &a, hipStream_t s);
template <typename T>
void launch_adj_out(const Dev<T> &d, const AdjDev &a, T *gc, T *gw, hipStream_t s);
template <typename T>
void launch_copy_weights(const Dev<T> &d, const T *w_new, hipStream_t s);

void launch_validate_csr(const int *row_ptr, const int *col_idx, int m, int n, long long nnz,
                         Ctl *ctl, hipStream_t s);
// CSR -> CSC transpose of the pattern; `tmp` holds n + 1 + scan scratch ints.
size_t transpose_scratch_ints(int n);
void launch_transpose(const int *row_ptr, const int *col_idx, int m, int n, long long nnz,
                      int *col_ptr, int *row_idx, int *tmp, hipStream_t s);
void launch_check_routes(const int *col_ptr, int n, double hi, Ctl *ctl, hipStream_t s);
void launch_ctl_init(Ctl *ctl, double rho, double eps_tol, double eps_rel, double mu,
                     double gamma, int adapt_every, hipStream_t s);
void launch_ctl_clear_done(Ctl *ctl, hipStream_t s);
// Count k iterations run without a check (ctl->iter += k).
void launch_ctl_advance(Ctl *ctl, long long k, hipStream_t s);
void launch_ctl_set_tolerances(Ctl *ctl, double eps_tol, double eps_rel, double mu, double gamma,
                               hipStream_t s);
void launch_fill_int(int *p, int value, size_t count, hipStream_t s);

}  // namespace pmp
