// Device-side building blocks shared by the PMP kernels: reductions, the
// proximal operators of Section III-E and the per-stream / per-link updates
// of the compact over-relaxed iteration (Section III-D, III-G).
#pragma once

#include "pmp_internal.h"

#include <cmath>

namespace pmp {

__device__ __forceinline__ int ld_stream(const int *p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a workgroup of NT threads in a fixed order; the result is valid in
// thread 0.  `sh` holds NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum(double v, double *sh) { return block_sum_n<kBlock>(v, sh); }

// Fixed-point term of a long row's sum (Dev::fx_shift): x 2^F rounded to an
// integer (x >= 0 and below 2^62 / (row length) after scaling, by the choice of F).
__device__ __forceinline__ long long fx_term(double x, double scale)
{
    return __double2ll_rn(x * scale);
}

// Exact int64 sum over a workgroup of NT threads (valid in thread 0); `sh`
// holds NT / 64 doubles, reused as int64.
template <int NT = kBlock>
__device__ __forceinline__ long long block_sum_ll(long long v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    long long *s = (long long *)sh;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s[wid] = v;
    __syncthreads();
    long long r = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) r += s[i];
    __syncthreads();
    return r;
}

// Stage tab[idx[i]] for i < cnt into LDS with a workgroup of NT threads.
// Every lane first loads its share of the index stream, then issues all of
// its gathers, then writes LDS, so up to kCap / NT gathers per lane are in
// flight together.
template <typename T, int NT = kBlock, int CAP = kCap>
__device__ __forceinline__ void gather_stage(const int *__restrict__ idx,
                                             const T *__restrict__ tab, T *sh, int cnt)
{
    constexpr int R = CAP / NT;
    int id[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * NT + threadIdx.x;
        id[r] = i < cnt ? ld_stream(idx + i) : -1;
    }
    T val[R];
#pragma unroll
    for (int r = 0; r < R; ++r) val[r] = id[r] >= 0 ? tab[id[r]] : T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * NT + threadIdx.x;
        if (i < cnt) sh[i] = val[r];
    }
}

// FP64 sum of sh[b..e) in a fixed order: four interleaved partial sums
// (entries b + 4i + r go to sum r), the tail into the first, then
// (s0 + s1) + (s2 + s3).  Four independent chains hide the LDS and add
// latency of one lane's run; every kernel that sums a staged run uses this
// order, so their results agree bit for bit.
template <typename T>
__device__ __forceinline__ double run_sum(const T *sh, int b, int e)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = b;
    for (; k + 3 < e; k += 4) {
        s0 += (double)sh[k];
        s1 += (double)sh[k + 1];
        s2 += (double)sh[k + 2];
        s3 += (double)sh[k + 3];
    }
    for (; k < e; ++k) s0 += (double)sh[k];
    return (s0 + s1) + (s2 + s3);
}

// Proximal operator of one traffic stream with L terminals and sum of
// arguments S (Section III-E), clipped to the box.  wsig > 0: log utility
// with weight wsig (alpha2 = false) or -w / x with weight wsig (alpha2 =
// true); wsig < 0: linear utility with weight -wsig.  For S < 0 the log root
// uses the equal form 2w / (rho (sqrt(S^2 + 4wL/rho) - S)).  The -w / x prox
// is the positive root of L x^3 - S x^2 - w / rho = 0, reached by Newton's
// method from max(S/L, 0) + (w / (rho L))^(1/3), where the cubic is
// nonnegative and convex, so the iterates decrease monotonically.
__device__ __forceinline__ double prox_stream(double S, int L, double wsig, double rho,
                                              double lo, double hi, bool alpha2 = false)
{
    if (L == 0) return hi;
    double x;
    const double dl = (double)L;
    if (alpha2) {
        const double c = wsig / rho;
        x = (S > 0.0 ? S / dl : 0.0) + cbrt(c / dl);
        for (int it = 0; it < 100; ++it) {
            const double g = (dl * x - S) * x * x - c;
            const double nx = x - g / ((3.0 * dl * x - 2.0 * S) * x);
            if (!(nx < x)) break;
            x = nx;
        }
    } else if (wsig > 0.0) {
        const double disc = sqrt(S * S + 4.0 * wsig * dl / rho);
        x = S >= 0.0 ? (S + disc) / (2.0 * dl) : 2.0 * wsig / (rho * (disc - S));
    } else {
        x = (S - wsig / rho) / dl;
    }
    return fmin(fmax(x, lo), hi);
}

// A check also screens the state it writes: a non-finite entry can leave the
// residuals finite (the box clip and the slack prox's max discard NaN), so
// it turns the partial sum into NaN, which finalize reports as
// PMP_ERR_NUMERIC.
__device__ __forceinline__ double screen(double part, double v)
{
    return isfinite(v) ? part : __builtin_nan("");
}

template <typename T>
__device__ __forceinline__ bool is_alpha2(const Dev<T> &d, int j)
{
    return d.util != nullptr && d.util[j] == PMP_UTIL_ALPHA2;
}

template <typename T, bool CHECK>
__device__ __forceinline__ double stream_update(const Dev<T> &d, int j, int L, double vsum,
                                                double rho)
{
    const double a = (double)d.a[j];
    const double S = (double)L * a + vsum;
    const T xt = (T)prox_stream(S, L, (double)d.wsig[j], rho, d.lo, d.hi, is_alpha2(d, j));
    const double xn = (double)xt;
    const T at = (T)(d.alpha * xn + (1.0 - d.alpha) * a);
    double part = 0.0;
    if (CHECK) {                       // dual residual: sum_j L_j (dx_j)^2
        const double dx = xn - (double)d.x[j];
        part = screen((double)L * dx * dx, (double)at);
    }
    d.x[j] = xt;
    d.a[j] = at;
    return part;
}

// Per-link inputs of the link update, loaded ahead of it so that the loads
// of several links can be in flight before any of their stores.
struct LinkIn {
    double c, u, b, zs;
    double yp, pp;   // saved y and ps of the previous iteration (checks only)
};

template <typename T, int MODE>
__device__ __forceinline__ LinkIn link_load(const Dev<T> &d, int l)
{
    LinkIn in{(double)d.c[l], (double)d.u[l], (double)d.b[l], (double)d.zs[l], 0.0, 0.0};
    if (MODE == kCheck) {
        in.yp = d.y_prev[l];
        in.pp = d.ps_prev[l];
    }
    return in;
}

template <typename T, int MODE, bool WRITE_V = true>
__device__ __forceinline__ double link_update_in(const Dev<T> &d, int l, int deg, double y,
                                               const LinkIn &in, double &r2, double &s2)
{
    const double c = in.c, u = in.u, b = in.b, zs = in.zs;
    const double al = d.alpha;
    const double ps = fmax(zs - u, -c);                 // slack prox
    if (d.mu_out) d.mu_out[l] = zs - u > -c ? 1 : 0;    // its branch, for reverse mode
    const double cnt = (double)deg + 1.0;               // |l| = d_l + 1
    const double pbar = (y + ps) / cnt;                 // link average
    const T bt = (T)(-al * pbar + (1.0 - al) * b);
    const T ut = (T)(u + al * pbar);
    const T zt = (T)(al * (ps - pbar) + (1.0 - al) * zs);
    d.b[l] = bt;
    d.zs[l] = zt;
    d.u[l] = ut;
    const T vt = (T)((double)bt - (double)ut);
    if (WRITE_V) d.v[l] = vt;
    if (MODE == kCheck) {
        // ||r||^2 = sum_l |l| pbar_l^2 and, with D the change since the
        // previous iteration, the link part of ||s||^2 / rho^2:
        // sum_{j on l} (Dx_j - Dpbar)^2 + (Dps - Dpbar)^2
        //   = [sum_j Dx_j^2] + d Dpbar^2 - 2 Dpbar Dy + (Dps - Dpbar)^2,
        // the bracket being added on the stream side.
        const double yp = in.yp, pp = in.pp;
        const double dpb = pbar - (yp + pp) / cnt;
        const double dy = y - yp, dps = ps - pp;
        r2 += screen(cnt * pbar * pbar, (double)bt + (double)ut + (double)zt);
        s2 += (double)deg * dpb * dpb - 2.0 * dpb * dy + (dps - dpb) * (dps - dpb);
    }
    if (MODE != kPlain) {
        d.y_prev[l] = y;
        d.ps_prev[l] = ps;
    }
    return (double)vt;
}

template <typename T, int MODE, bool WRITE_V = true>
__device__ __forceinline__ double link_update(const Dev<T> &d, int l, int deg, double y,
                                            double &r2, double &s2)
{
    return link_update_in<T, MODE, WRITE_V>(d, l, deg, y, link_load<T, MODE>(d, l), r2, s2);
}

// ---- reverse mode (one reversed iteration; see pmp_adjoint.hip) ------------

__device__ __forceinline__ void adj_link_step(const AdjDev &a, int l, int deg, double alpha,
                                          uint8_t mu)
{
    const double B = a.B[l], Z = a.Z[l], U = a.U[l];
    const double inv = 1.0 / ((double)deg + 1.0);
    const double pbb = alpha * (U - B - Z);
    const double psb = alpha * Z + pbb * inv;
    const double m1 = mu ? 1.0 : 0.0;
    a.ybar[l] = pbb * inv;
    a.cbar[l] -= (1.0 - m1) * psb;
    a.B[l] = (1.0 - alpha) * B;
    a.Z[l] = (1.0 - alpha) * Z + m1 * psb;
    a.U[l] = U - m1 * psb;
}

template <typename T>
__device__ __forceinline__ void adj_stream_step(const Dev<T> &d, const AdjDev &a, const T *xt,
                                            int j, int L, double ysum, int last, double rho)
{
    double xbar = d.alpha * a.A[j] + ysum;
    if (last) xbar += a.ext[j];
    const double x = (double)xt[j];
    const double wsig = (double)d.wsig[j];
    double sbar = 0.0;
    if (L > 0 && x > d.lo && x < d.hi) {
        double dS, dw;
        if (d.util && d.util[j] == PMP_UTIL_ALPHA2) {
            // rho L x^3 - rho S x^2 - w = 0:  dx/dS = rho x^3 / (rho L x^3 + 2w),
            // dx/dw = x / (rho L x^3 + 2w)
            const double den = rho * (double)L * x * x * x + 2.0 * wsig;
            dS = rho * x * x * x / den;
            dw = x / den;
        } else if (wsig > 0.0) {
            const double den = rho * (double)L * x * x + wsig;
            dS = rho * x * x / den;
            dw = x / den;
        } else {
            dS = 1.0 / (double)L;
            dw = 1.0 / (rho * (double)L);
        }
        sbar = xbar * dS;
        a.wbar[j] += xbar * dw;
    }
    a.A[j] = (1.0 - d.alpha) * a.A[j] + (double)L * sbar;
    a.Sbar[j] = sbar;
}

// ---- residual reduction, stop rule and rho balancing ---------------------

// Thread 0 of the check-finalize kernel: residual norms (Section III-F), the
// stop rule, and residual balancing of rho (Section III-G).  nrm (or NULL):
// sums of squares of p, z and u over all terminals, for the relative part
// of the stop rule: ||r|| < eps_abs sqrt(J) + eps_rel max(||p||, ||z||) and
// ||s|| < eps_abs sqrt(J) + eps_rel ||rho u||.
template <typename T>
__device__ void finalize(const Dev<T> &d, long long delta, int stop, double sr, double ss,
                         const double *nrm = nullptr)
{
    Ctl *c = d.ctl;
    const double rho = c->rho;
    const long long it = c->iter + delta;
    const double r = sqrt(sr);
    const double s = rho * sqrt(ss > 0.0 ? ss : (ss == ss ? 0.0 : ss));   // keeps a NaN
    double tol_r = c->eps_tol, tol_s = c->eps_tol;
    if (nrm && c->eps_rel > 0.0) {
        c->p_norm = sqrt(fmax(nrm[0], 0.0));
        c->z_norm = sqrt(fmax(nrm[1], 0.0));
        c->u_norm = rho * sqrt(fmax(nrm[2], 0.0));
        tol_r += c->eps_rel * fmax(c->p_norm, c->z_norm);
        tol_s += c->eps_rel * c->u_norm;
    }
    c->iter = it;
    c->r_norm = r;
    c->s_norm = s;
    c->ratio = 1.0;
    HistEntry &h = d.hist[c->nhist % kHist];
    h.iter = it;
    h.r_norm = r;
    h.s_norm = s;
    h.rho = rho;
    c->nhist += 1;
    if (!isfinite(r) || !isfinite(s)) {
        c->status = PMP_ERR_NUMERIC;
        c->done = 1;
    } else if (stop && r < tol_r && s < tol_s) {
        c->status = PMP_OK;
        c->done = 1;
    } else if (c->adapt_every > 0 && it % c->adapt_every == 0) {
        double rn = rho;
        if (r > c->mu * s) rn = c->gamma * rho;
        else if (s > c->mu * r) rn = rho / c->gamma;
        c->ratio = rho / rn;
        c->rho = rn;
    }
}

}  // namespace pmp
