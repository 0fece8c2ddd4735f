// risk.hip -- the risk-set kernel: everything of one ISTA step that is O(n).
//
// For one coefficient vector b (one workgroup of 1024 threads), with subjects in
// the order of non-increasing observed time (Section 5.3):
//   eta  = eta_in (+ the partial updates of the columns that changed)
//   m    = max_i eta_i;  w_k = exp(eta_k - m)                         (FP64)
//   S_k  = w_0 + ... + w_k           cumulative sum in decreasing time (FP64)
//   W_k  = S[gend(k)]                the whole tie group is at risk (Breslow, Section 6)
//   L    = sum_k delta_k (eta_k - m - log W_k)                        (FP64)
//   T_k  = sum_{k' >= k} delta_k' / W_k'   reverse cumulative sum     (FP64)
//   c_k  = T[gstart(k)];  r_k = delta_k - w_k c_k   = ((I - P) delta)_k
// r is scattered back to subject order (FP32 for the X' r pass, FP64 on
// request).  Inside cox_fit_path the kernel also forms f_k = -L +
// lambda ||beta_k||_1 and applies the lag-k stopping rule of Section 6.
//
// The scans are tiled: each thread owns 4 consecutive positions of a 4096-wide
// tile; a block-wide exclusive scan of the thread totals plus the running carry
// gives every prefix.  One workgroup per b keeps the order of every FP64 sum
// fixed, so results are bit-reproducible.
#include <math.h>

#include "device_common.h"

namespace cox {
namespace {

constexpr int kT = kRiskThreads;
constexpr int kEPT = 4;
constexpr int kTile = kT * kEPT;
constexpr int kNW = kT / kWave;

__device__ double block_excl_scan(double v, double* sh, double* total)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const double inc = wave_incl_scan(v, lane);
    if (lane == kWave - 1) sh[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        const double t = lane < kNW ? sh[lane] : 0.0;
        const double ti = wave_incl_scan(t, lane);
        if (lane < kNW) sh[lane] = ti - t;
        if (lane == kNW - 1) sh[kNW] = ti;
    }
    __syncthreads();
    const double res = sh[wid] + inc - v;
    *total = sh[kNW];
    __syncthreads();
    return res;
}

__device__ double block_sum(double v, double* sh)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (wid == 0) {
        double t = lane < kNW ? sh[lane] : 0.0;
        t = wave_sum(t);
        if (lane == 0) sh[kNW] = t;
    }
    __syncthreads();
    const double r = sh[kNW];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double* sh)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_max(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (wid == 0) {
        double t = lane < kNW ? sh[lane] : -INFINITY;
        t = wave_max(t);
        if (lane == 0) sh[kNW] = t;
    }
    __syncthreads();
    const double r = sh[kNW];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kT) void risk_kernel(RiskArgs a)
{
    __shared__ double sh[kNW + 1];
    const int b = blockIdx.x;
    if (a.use_ctl && !a.ctl.active[b]) return;  // uniform over the workgroup
    const int tid = threadIdx.x;
    const int64_t n = a.n;
    const int64_t bo = (int64_t)b * n;
    const int32_t* __restrict__ perm = a.ord.perm;
    const uint8_t* __restrict__ ev = a.ord.ev;

    // eta, with the partial updates added when there are any; its maximum.
    const bool addp = a.part != nullptr && *a.nsel > 0;
    double m = -INFINITY;
    for (int64_t i = tid; i < n; i += kT) {
        double e = a.eta_in_f32 ? (double)static_cast<const float*>(a.eta_in)[bo + i]
                                : static_cast<const double*>(a.eta_in)[bo + i];
        if (addp)
            for (int c = 0; c < a.ncg; ++c) e += a.part[(int64_t)c * a.part_cstride + bo + i];
        if (a.eta_out) a.eta_out[bo + i] = e;
        m = fmax(m, e);
    }
    m = block_max(m, sh);  // also orders the eta_out writes before the reads below

    const double* eta64 = a.eta_out ? a.eta_out + bo : static_cast<const double*>(a.eta_in) + bo;
    const float* eta32 = static_cast<const float*>(a.eta_in) + bo;
    const bool e32 = a.eta_out == nullptr && a.eta_in_f32;
    auto eta_at = [&](int64_t i) -> double { return e32 ? (double)eta32[i] : eta64[i]; };

    double* __restrict__ w = a.w + bo;
    double* __restrict__ S = a.S + bo;
    double* __restrict__ T = a.T + bo;

    // Cumulative sum of w in decreasing time.
    double carry = 0.0;
    for (int64_t base = 0; base < n; base += kTile) {
        const int64_t k0 = base + (int64_t)tid * kEPT;
        double v[kEPT];
        double ts = 0.0;
#pragma unroll
        for (int e = 0; e < kEPT; ++e) {
            const int64_t k = k0 + e;
            v[e] = k < n ? exp(eta_at(perm[k]) - m) : 0.0;
            ts += v[e];
        }
        double tot;
        double run = carry + block_excl_scan(ts, sh, &tot);
#pragma unroll
        for (int e = 0; e < kEPT; ++e) {
            const int64_t k = k0 + e;
            run += v[e];
            if (k < n) {
                w[k] = v[e];
                S[k] = run;
            }
        }
        carry += tot;
    }
    __syncthreads();

    // Log-likelihood terms and the reverse cumulative sum of delta / W, walking
    // positions from the last (shortest time) to the first.
    const int32_t* __restrict__ gend = a.ord.gend;
    double Lacc = 0.0;
    carry = 0.0;
    for (int64_t base = 0; base < n; base += kTile) {
        const int64_t r0 = base + (int64_t)tid * kEPT;
        double v[kEPT];
        double ts = 0.0;
#pragma unroll
        for (int e = 0; e < kEPT; ++e) {
            v[e] = 0.0;
            const int64_t kr = r0 + e;
            if (kr < n) {
                const int64_t k = n - 1 - kr;
                if (ev[k]) {
                    const double W = S[gend[k]];
                    v[e] = 1.0 / W;
                    Lacc += eta_at(perm[k]) - m - log(W);
                }
            }
            ts += v[e];
        }
        double tot;
        double run = carry + block_excl_scan(ts, sh, &tot);
#pragma unroll
        for (int e = 0; e < kEPT; ++e) {
            const int64_t kr = r0 + e;
            run += v[e];
            if (kr < n) T[n - 1 - kr] = run;
        }
        carry += tot;
    }
    __syncthreads();

    // r = delta - w * c, scattered to subject order.
    const int32_t* __restrict__ gstart = a.ord.gstart;
    const int64_t ro = (int64_t)b * a.rstride;
    double sr = 0.0;
    for (int64_t k = tid; k < n; k += kT) {
        const double c = T[gstart[k]];
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
    Lacc = block_sum(Lacc, sh);
    sr = block_sum(sr, sh);
    if (tid == 0) {
        a.L[b] = Lacc;
        a.sumr[b] = sr;
    }

    if (a.use_ctl) {
        const FitCtl& c = a.ctl;
        double l1 = 0.0;
        for (int q = tid; q < c.nblk; q += kT) l1 += c.l1[(int64_t)b * c.nblk + q];
        l1 = block_sum(l1, sh);
        if (tid == 0) {
            const double f = -Lacc + c.lam[b] * l1;
            const int k = c.kit[b];
            double* h = c.hist + (int64_t)b * kMaxHist;
            h[k % kMaxHist] = f;
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
}

}  // namespace

hipError_t launch_risk(const RiskArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(risk_kernel, dim3(a.B), dim3(kT), 0, s, a);
    return hipGetLastError();
}

}  // namespace cox
