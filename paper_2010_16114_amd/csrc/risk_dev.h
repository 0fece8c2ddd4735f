// risk_dev.h -- the risk-set sums of one ISTA step (everything that is O(n)),
// as per-workgroup device functions shared by the one-kernel-per-phase
// launches (risk.hip) and the persistent path (persist.hip).  Each function
// is the work of one workgroup of kT = 256 threads, (bx, by) its position
// in the phase's grid; LDS is passed in.
//
// For each coefficient vector b, with subjects in the order of non-increasing
// observed time (Section 5.3):
//   eta  = eta_in (+ the partial updates of the columns that changed)
//   m    = max_i eta_i;  w_k = exp(eta_k - m)                         (FP64)
//   S_k  = w_0 + ... + w_k           cumulative sum in decreasing time (FP64)
//   W_k  = S[gend(k)]                the whole tie group is at risk (Breslow, Section 6)
//   L    = sum_k delta_k (eta_k - m - log W_k)                        (FP64)
//   T_k  = sum_{k' >= k} delta_k' / W_k'   reverse cumulative sum     (FP64)
//   c_k  = T[gstart(k)];  r_k = delta_k - w_k c_k   = ((I - P) delta)_k
// r is scattered back to subject order (FP32 for the X' r pass, FP64 on
// request).  Inside cox_fit_path the last stage also forms f_k = -L +
// lambda ||beta_k||_1 and applies the lag-k stopping rule of Section 6.
//
// Five phases, each spread over many workgroups (by = b):
//   1 eta     : add the partial updates (subject order, coalesced), block maxima
//   2 scan_w  : w and its cumulative sum within each tile of sorted positions
//   3 scan_q  : tile offsets of S (every workgroup scans the tile totals itself),
//               W at the end of the tie group, log-likelihood terms, reverse
//               cumulative sum of delta/W within the tile
//   4 resid   : tile offsets of T, c at the start of the tie group, r
//   5 finish  : fixed-order sums of the tile partials; objective; stopping rule
// A tie group may straddle tiles: W and c are read through the global offsets
// of the tile that holds gend(k) / gstart(k), which the previous phase
// completed.  Every sum runs in a fixed order, so results are bit-reproducible.
#pragma once
#include <math.h>

#include "device_common.h"

namespace cox {
namespace riskdev {

constexpr int kT = 256;  // threads per workgroup of every phase
constexpr int kNW = kT / kWave;
constexpr int kSub = 4 * kT;  // positions per sub-chunk of a tile (4 per thread)

__device__ __forceinline__ bool skip_b(const RiskArgs& a, int b) { return a.use_ctl && !a.ctl.active[b]; }

// Block-wide exclusive scan of one double per thread; *total gets the block sum.
__device__ inline double block_excl_scan(double v, double* sh, double* total)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const double inc = wave_incl_scan(v, lane);
    if (lane == kWave - 1) sh[wid] = inc;
    __syncthreads();
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int q = 0; q < kNW; ++q) {
        off += q < wid ? sh[q] : 0.0;
        tot += sh[q];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ inline double block_sum(double v, double* sh)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kNW; ++q) t += sh[q];
    __syncthreads();
    return t;
}

__device__ inline double block_max(double v, double* sh)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_max(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = -INFINITY;
#pragma unroll
    for (int q = 0; q < kNW; ++q) t = fmax(t, sh[q]);
    __syncthreads();
    return t;
}

// Exclusive prefix (reverse = false) or exclusive suffix (reverse = true) of
// v[0..m) into out[0..m) (LDS), computed by the whole block in a fixed order.
__device__ inline void block_offsets(const double* __restrict__ v, int m, bool reverse, double* out, double* sh)
{
    const int per = (m + kT - 1) / kT;
    const int lo = threadIdx.x * per;
    double s = 0.0;
    for (int q = 0; q < per; ++q) {
        const int i = lo + q;
        if (i < m) s += v[reverse ? m - 1 - i : i];
    }
    double tot;
    double run = block_excl_scan(s, sh, &tot);
    for (int q = 0; q < per; ++q) {
        const int i = lo + q;
        if (i < m) {
            const int at = reverse ? m - 1 - i : i;
            out[at] = run;
            run += v[at];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void risk_eta_blk(const RiskArgs& a, int bx, int by, double* sh)
{
    const int b = by;
    if (skip_b(a, b)) return;
    const int64_t n = a.n, bo = (int64_t)b * n;
    const bool addp = a.part != nullptr && *a.nsel > 0;
    const bool copy = addp || a.eta_in_f32 || a.eta_in != a.eta;
    double m = -INFINITY;
    const int64_t i0 = (int64_t)bx * kFinElems + threadIdx.x;
#pragma unroll 4
    for (int e = 0; e < kFinElems / kT; ++e) {
        const int64_t i = i0 + (int64_t)e * kT;
        if (i >= n) break;
        double v = a.eta_in_f32 ? (double)static_cast<const float*>(a.eta_in)[bo + i]
                                : static_cast<const double*>(a.eta_in)[bo + i];
        if (addp)
            for (int c = 0; c < a.ncg; ++c) v += a.part[(int64_t)c * a.part_cstride + bo + i];
        if (copy) a.eta[bo + i] = v;
        m = fmax(m, v);
    }
    m = block_max(m, sh);
    if (threadIdx.x == 0) a.bmax[(int64_t)b * a.nfin + bx] = m;
}

__device__ __forceinline__ void risk_scan_w_blk(const RiskArgs& a, int bx, int by, double* sh)
{
    const int b = by;
    if (skip_b(a, b)) return;
    const int64_t n = a.n, bo = (int64_t)b * n;
    double m = -INFINITY;
    for (int q = threadIdx.x; q < a.nfin; q += kT) m = fmax(m, a.bmax[(int64_t)b * a.nfin + q]);
    m = block_max(m, sh);
    if (bx == 0 && threadIdx.x == 0) a.mshift[b] = m;
    const int32_t* __restrict__ perm = a.ord.perm;
    const double* __restrict__ eta = a.eta + bo;
    double* __restrict__ w = a.w + bo;
    double* __restrict__ S = a.S + bo;
    const int64_t t0 = (int64_t)bx * a.tile;
    const int64_t t1 = min(n, t0 + a.tile);
    double carry = 0.0;
    for (int64_t base = t0; base < t1; base += kSub) {
        const int64_t k0 = base + 4 * (int64_t)threadIdx.x;
        double v[4];
        double ts = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = k0 + e < t1 ? exp(eta[perm[k0 + e]] - m) : 0.0;
            ts += v[e];
        }
        double tot;
        double run = carry + block_excl_scan(ts, sh, &tot);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            run += v[e];
            if (k0 + e < t1) {
                w[k0 + e] = v[e];
                S[k0 + e] = run;
            }
        }
        carry += tot;
    }
    if (threadIdx.x == 0) a.stot[(int64_t)b * a.ntile + bx] = carry;
}

__device__ __forceinline__ void risk_scan_q_blk(const RiskArgs& a, int bx, int by, double* sh, double* pre)
{
    const int b = by;
    if (skip_b(a, b)) return;
    const int64_t n = a.n, bo = (int64_t)b * n;
    block_offsets(a.stot + (int64_t)b * a.ntile, a.ntile, false, pre, sh);
    const double m = a.mshift[b];
    const int32_t* __restrict__ perm = a.ord.perm;
    const int32_t* __restrict__ gend = a.ord.gend;
    const uint8_t* __restrict__ ev = a.ord.ev;
    const double* __restrict__ eta = a.eta + bo;
    const double* __restrict__ S = a.S + bo;
    double* __restrict__ T = a.T + bo;
    const int64_t t0 = (int64_t)bx * a.tile;
    const int64_t len = min(n, t0 + a.tile) - t0;
    double carry = 0.0, Lacc = 0.0;
    for (int64_t base = 0; base < len; base += kSub) {
        const int64_t u0 = base + 4 * (int64_t)threadIdx.x;  // distance from the tile's last position
        double v[4];
        double ts = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = 0.0;
            if (u0 + e < len) {
                const int64_t k = t0 + len - 1 - (u0 + e);
                if (ev[k]) {
                    const int64_t ge = gend[k];
                    const double W = S[ge] + pre[ge / a.tile];
                    v[e] = 1.0 / W;
                    Lacc += eta[perm[k]] - m - log(W);
                }
            }
            ts += v[e];
        }
        double tot;
        double run = carry + block_excl_scan(ts, sh, &tot);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            run += v[e];
            if (u0 + e < len) T[t0 + len - 1 - (u0 + e)] = run;
        }
        carry += tot;
    }
    Lacc = block_sum(Lacc, sh);
    if (threadIdx.x == 0) {
        a.qtot[(int64_t)b * a.ntile + bx] = carry;
        a.Lpart[(int64_t)b * a.ntile + bx] = Lacc;
    }
}

__device__ __forceinline__ void risk_resid_blk(const RiskArgs& a, int bx, int by, double* sh, double* suf)
{
    const int b = by;
    if (skip_b(a, b)) return;
    const int64_t n = a.n, bo = (int64_t)b * n;
    block_offsets(a.qtot + (int64_t)b * a.ntile, a.ntile, true, suf, sh);
    const int32_t* __restrict__ perm = a.ord.perm;
    const int32_t* __restrict__ gstart = a.ord.gstart;
    const uint8_t* __restrict__ ev = a.ord.ev;
    const double* __restrict__ w = a.w + bo;
    const double* __restrict__ T = a.T + bo;
    const int64_t ro = (int64_t)b * a.rstride;
    const int64_t t0 = (int64_t)bx * a.tile;
    const int64_t t1 = min(n, t0 + a.tile);
    double sr = 0.0;
    for (int64_t k = t0 + threadIdx.x; k < t1; k += kT) {
        const int64_t gs = gstart[k];
        const double c = T[gs] + suf[gs / a.tile];
        const double r = (ev[k] ? 1.0 : 0.0) - w[k] * c;
        const int32_t i = perm[k];
        if (a.r32) {
            const float rf = (float)r;
            a.r32[ro + i] = rf;
            sr += (double)rf;
        } else {
            sr += r;
        }
        if (a.r64) a.r64[bo + i] = r;
    }
    sr = block_sum(sr, sh);
    if (threadIdx.x == 0) a.rpart[(int64_t)b * a.ntile + bx] = sr;
}

__device__ __forceinline__ void risk_finish_blk(const RiskArgs& a, int bx, double* sh)
{
    const int b = bx;
    if (skip_b(a, b)) return;
    double L = 0.0, sr = 0.0;
    for (int q = threadIdx.x; q < a.ntile; q += kT) {
        L += a.Lpart[(int64_t)b * a.ntile + q];
        sr += a.rpart[(int64_t)b * a.ntile + q];
    }
    L = block_sum(L, sh);
    sr = block_sum(sr, sh);
    if (threadIdx.x == 0) {
        a.L[b] = L;
        a.sumr[b] = sr;
    }
    if (!a.use_ctl) return;
    const FitCtl& c = a.ctl;
    double l1 = 0.0;
    for (int q = threadIdx.x; q < c.nblk; q += kT) l1 += c.l1[(int64_t)b * c.nblk + q];
    l1 = block_sum(l1, sh);
    if (threadIdx.x == 0) {
        if (c.l1cov) l1 += c.l1cov[b];
        const double f = -L + c.lam[b] * l1;
        const int k = c.kit[b];
        double* h = c.hist + (int64_t)b * kMaxHist;
        h[k % kMaxHist] = f;
        if (c.trace) c.trace[(int64_t)b * c.trace_stride + k] = f;
        int stop = 0;
        if (!isfinite(f))
            stop = 3;
        else if (k >= c.lag && fabs(f - h[(k - c.lag) % kMaxHist]) / (fabs(f) + 1.0) < c.tol)
            stop = 1;
        else if (k >= c.max_iter)
            stop = 2;
        c.fobj[b] = f;
        if (stop) {
            c.active[b] = 0;
            c.status[b] = stop;
            c.iters[b] = k;
        } else {
            c.kit[b] = k + 1;
        }
    }
}

}  // namespace riskdev
}  // namespace cox
