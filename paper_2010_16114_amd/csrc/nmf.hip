// nmf.hip -- nonnegative matrix factorisation X ~ V W (Section 5.1) on one GPU,
// and its C ABI (include/nmf.h).
//
// X is m x n FP32, row-major (row i at X + i * ldx), borrowed.  The factors are
// stored as the paper's loop stores them, V' (r x m) and W (r x n), row-major,
// in FP64: they are small (r (m + n) doubles) and every product with X is
// formed and summed in FP64, so the only rounding is in the order of the sums.
//
// One iteration (Section 5.1, the loop's order):
//   W X'   (r x m)  nmf_wxt_kernel: workgroups over (256 rows of X, a split of
//                   the columns); the 256 x 32 X tile and the r x 32 W tile of a
//                   step pass through LDS into FP64 matrix-core tiles, the next
//                   step's tiles loading into registers meanwhile (with aligned
//                   rows, nmf_wxt_direct_kernel loads them straight into
//                   registers).  The split partials are added by nmf_reduce_kernel.
//   W W'   (r x r)  nmf_gram_kernel, one workgroup per entry of the upper
//                   triangle, fixed-order reduction.
//   V' <- update    nmf_update_kernel, 4 threads per column of V': the r x r
//                   product with W W', then the multiplicative update
//                   V .* (X W') ./ (V W W' + eps) or the projected step
//                   max(0, V - sigma (V W W' - X W')), sigma = 1/(2||W W'||_F^2 + eps).
//   V' X   (r x n)  nmf_vtx_kernel: workgroups over (256 columns of X, a split
//                   of the rows); a 32 x 256 X tile and the r x 32 V' tile, the
//                   same way.
//   V' V   (r x r), then the W update the same way with tau = 1/(2||V'V||_F^2 + eps).
// Both passes over X read it once each; the r x r products and the updates
// are O(r^2 (m + n)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cox.h"
#include "device_common.h"
#include "nmf.h"

namespace cox {
namespace {

constexpr int kT = 256;
constexpr int kTJ = 32;  // columns of X per LDS step of W X'
constexpr int kTI = 32;  // rows of X per LDS step of V' X

__device__ double block_sum256(double v, double* sh)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kT / kWave; ++q) s += sh[q];
    return s;
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Both passes run on the FP64 matrix cores (v_mfma_f64_16x16x4f64: D = A B + C
// with A 16 x 4, B 4 x 16, FP64 operands and accumulation).  Per lane: A holds
// (row lane % 16, k lane / 16), B holds (k lane / 16, column lane % 16), and D
// holds rows lane / 16 + 4 v, v < 4, of column lane % 16 (interleaved, unlike
// the int8 instruction's 4 (lane / 16) + v; checked on the device).  The rank
// is padded to MT tiles of 16; a wavefront owns 64 rows (or columns) of X, 4 N
// tiles.
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// part[split][a][i] = sum over the split's columns j of W[a][j] X[i][j]:
// M = a (the rank), N = i (256 rows of X per workgroup), K = j
template <int MT>
__global__ __launch_bounds__(kT) void nmf_wxt_kernel(const float* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
                                                     int r, const double* __restrict__ W, int64_t cols,
                                                     double* __restrict__ part)
{
    constexpr int R = 16 * MT;
    __shared__ float Xs[kT][kTJ + 1];
    __shared__ double Ws[R][kTJ + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kT;
    const int64_t j0 = (int64_t)blockIdx.y * cols, j1 = min(n, j0 + cols);
    v4d acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = v4d{0.0, 0.0, 0.0, 0.0};
    // the next step's tiles are loaded into registers while the current one is
    // multiplied out of LDS
    constexpr int XE = kT * kTJ / (4 * kT);
    constexpr int WE = (R * kTJ + kT - 1) / kT;
    float xr[XE][4];
    double wr[WE];
    auto fetch = [&](int64_t js) {
#pragma unroll
        for (int e = 0; e < XE; ++e) {
            const int li = threadIdx.x + kT * e;
            const int row = li / (kTJ / 4), c4 = (li % (kTJ / 4)) * 4;
            const int64_t i = i0 + row;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t j = js + c4 + q;
                xr[e][q] = (i < m && j < j1) ? X[i * ldx + j] : 0.0f;
            }
        }
#pragma unroll
        for (int e = 0; e < WE; ++e) {
            const int li = threadIdx.x + kT * e;
            const int a = li / kTJ, jj = li % kTJ;
            const int64_t j = js + jj;
            wr[e] = (li < R * kTJ && a < r && j < j1) ? W[(int64_t)a * n + j] : 0.0;
        }
    };
    if (j0 < j1) fetch(j0);
    for (int64_t js = j0; js < j1; js += kTJ) {
#pragma unroll
        for (int e = 0; e < XE; ++e) {
            const int li = threadIdx.x + kT * e;
            const int row = li / (kTJ / 4), c4 = (li % (kTJ / 4)) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) Xs[row][c4 + q] = xr[e][q];
        }
#pragma unroll
        for (int e = 0; e < WE; ++e) {
            const int li = threadIdx.x + kT * e;
            if (li < R * kTJ) Ws[li / kTJ][li % kTJ] = wr[e];
        }
        __syncthreads();
        if (js + kTJ < j1) fetch(js + kTJ);
#pragma unroll
        for (int kk = 0; kk < kTJ; kk += 4) {
            const int k = kk + (lane >> 4);
            double av[MT], bv[4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) av[mt] = Ws[mt * 16 + (lane & 15)][k];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bv[nt] = (double)Xs[wid * 64 + nt * 16 + (lane & 15)][k];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma_f64(av[mt], bv[nt], acc[mt][nt]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = mt * 16 + (lane >> 4) + 4 * v;
                const int64_t i = i0 + wid * 64 + nt * 16 + (lane & 15);
                if (a < r && i < m) part[((int64_t)blockIdx.y * r + a) * m + i] = acc[mt][nt][v];
            }
}

// part[split][a][j] = sum over the split's rows i of Vt[a][i] X[i][j]:
// M = a, N = j (256 columns of X per workgroup), K = i
template <int MT>
__global__ __launch_bounds__(kT) void nmf_vtx_kernel(const float* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
                                                     int r, const double* __restrict__ Vt, int64_t rows,
                                                     double* __restrict__ part)
{
    constexpr int R = 16 * MT;
    __shared__ float Xs[kTI][kT + 4];
    __shared__ double Vs[R][kTI + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t jb = (int64_t)blockIdx.x * kT;
    const int64_t i0 = (int64_t)blockIdx.y * rows, i1 = min(m, i0 + rows);
    v4d acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = v4d{0.0, 0.0, 0.0, 0.0};
    // the next step's tiles (kTI rows x 256 columns of X, one column per thread,
    // and the r x kTI tile of V') are loaded into registers during this one
    constexpr int VE = (R * kTI + kT - 1) / kT;
    float xr[kTI];
    double vr[VE];
    auto fetch = [&](int64_t is) {
#pragma unroll
        for (int ii = 0; ii < kTI; ++ii) {
            const int64_t i = is + ii, j = jb + threadIdx.x;
            xr[ii] = (i < i1 && j < n) ? X[i * ldx + j] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < VE; ++e) {
            const int li = threadIdx.x + kT * e;
            const int a = li / kTI, ii = li % kTI;
            const int64_t i = is + ii;
            vr[e] = (li < R * kTI && a < r && i < i1) ? Vt[(int64_t)a * m + i] : 0.0;
        }
    };
    if (i0 < i1) fetch(i0);
    for (int64_t is = i0; is < i1; is += kTI) {
#pragma unroll
        for (int ii = 0; ii < kTI; ++ii) Xs[ii][threadIdx.x] = xr[ii];
#pragma unroll
        for (int e = 0; e < VE; ++e) {
            const int li = threadIdx.x + kT * e;
            if (li < R * kTI) Vs[li / kTI][li % kTI] = vr[e];
        }
        __syncthreads();
        if (is + kTI < i1) fetch(is + kTI);
#pragma unroll
        for (int kk = 0; kk < kTI; kk += 4) {
            const int k = kk + (lane >> 4);
            double av[MT], bv[4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) av[mt] = Vs[mt * 16 + (lane & 15)][k];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bv[nt] = (double)Xs[k][wid * 64 + nt * 16 + (lane & 15)];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma_f64(av[mt], bv[nt], acc[mt][nt]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = mt * 16 + (lane >> 4) + 4 * v;
                const int64_t j = jb + wid * 64 + nt * 16 + (lane & 15);
                if (a < r && j < n) part[((int64_t)blockIdx.y * r + a) * n + j] = acc[mt][nt][v];
            }
}

// W X' with both operands loaded straight from memory into registers, no
// LDS: used when the rows of X start 16-byte aligned (X aligned, ldx a
// multiple of 4) and so do the rows of W (aligned, n even), as at the paper's
// 10,000 x 10,000; otherwise the kernel above.  Each lane loads GL
// consecutive columns, and the s-th product of a step puts column GL q + s of
// the step in k-slot q (q = lane / 16) -- one permutation shared by both
// operands, so the products pair up as in the plain sum.  The next step's
// values load while the current ones are multiplied.  (The same form of V' X,
// with 16-byte pieces of 4 columns per row, measured slower than the LDS
// kernel: 0.19 against 0.15 ms at 10,000 x 10,000, r = 20.)

// part[split][a][i] = sum over the split's columns j of W[a][j] X[i][j].  A
// wavefront owns 64 rows of X (4 N tiles) and all MT rank tiles; a step covers
// 4 GL columns; lane (c, q) reads columns js + GL q .. + GL - 1 of X row
// ib + 16 nt + c and of W row 16 mt + c.  Rows of X past m are read from row
// m - 1 (their outputs are not stored), W rows past r and columns past the
// split give 0.
template <int MT, int GL>
__global__ __launch_bounds__(kT) void nmf_wxt_direct_kernel(const float* __restrict__ X, int64_t m, int64_t n,
                                                            int64_t ldx, int r, const double* __restrict__ W,
                                                            int64_t cols, double* __restrict__ part)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, c = lane & 15, q = lane >> 4;
    const int64_t ib = (int64_t)blockIdx.x * kT + wid * 64;
    const int64_t j0 = (int64_t)blockIdx.y * cols, j1 = min(n, j0 + cols);
    const float* xr[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) xr[nt] = X + min(ib + nt * 16 + c, m - 1) * ldx;
    const double* wr[MT];
    bool wok[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int a = mt * 16 + c;
        wok[mt] = a < r;
        wr[mt] = W + (int64_t)min(a, r - 1) * n;
    }
    v4d acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = v4d{0.0, 0.0, 0.0, 0.0};
    float nx[4][GL];
    double nw[MT][GL];
    auto fetch = [&](int64_t js) {
        const int64_t j = js + GL * q;
        if (js + 4 * GL <= j1) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int e = 0; e < GL; e += 4) {
                    const float4 v = *reinterpret_cast<const float4*>(xr[nt] + j + e);
                    nx[nt][e] = v.x, nx[nt][e + 1] = v.y, nx[nt][e + 2] = v.z, nx[nt][e + 3] = v.w;
                }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int e = 0; e < GL; e += 2) {
                    const double2 v = wok[mt] ? *reinterpret_cast<const double2*>(wr[mt] + j + e) : double2{0.0, 0.0};
                    nw[mt][e] = v.x, nw[mt][e + 1] = v.y;
                }
        } else {
#pragma unroll
            for (int e = 0; e < GL; ++e) {
                const bool in = j + e < j1;
                const int64_t jc = in ? j + e : j0;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) nx[nt][e] = xr[nt][jc];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) nw[mt][e] = (in && wok[mt]) ? wr[mt][jc] : 0.0;
            }
        }
    };
    if (j0 < j1) fetch(j0);
    for (int64_t js = j0; js < j1; js += 4 * GL) {
        float cx[4][GL];
        double cw[MT][GL];
#pragma unroll
        for (int e = 0; e < GL; ++e) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) cx[nt][e] = nx[nt][e];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) cw[mt][e] = nw[mt][e];
        }
        if (js + 4 * GL < j1) fetch(js + 4 * GL);
#pragma unroll
        for (int e = 0; e < GL; ++e)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const double b = (double)cx[nt][e];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_f64(cw[mt][e], b, acc[mt][nt]);
            }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = mt * 16 + q + 4 * v;
                const int64_t i = ib + nt * 16 + c;
                if (a < r && i < m) part[((int64_t)blockIdx.y * r + a) * m + i] = acc[mt][nt][v];
            }
}

// num[t] = sum over splits of part[split][t], t < r * len, in split order
__global__ __launch_bounds__(kT) void nmf_reduce_kernel(const double* __restrict__ part, int nsplit, int64_t count,
                                                        double* __restrict__ num)
{
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < count; t += (int64_t)gridDim.x * kT) {
        double s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * count + t];
        num[t] = s;
    }
}

// G[a][b] = G[b][a] = sum_k F[a][k] F[b][k] over len, one workgroup per a <= b
__global__ __launch_bounds__(kT) void nmf_gram_kernel(const double* __restrict__ F, int r, int64_t len,
                                                      double* __restrict__ G)
{
    __shared__ double sh[kT / kWave];
    int idx = blockIdx.x, a = 0;
    while (idx >= r - a) {
        idx -= r - a;
        ++a;
    }
    const int b = a + idx;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < len; k += kT) s += F[(int64_t)a * len + k] * F[(int64_t)b * len + k];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) {
        G[a * r + b] = s;
        G[b * r + a] = s;
    }
}

// One factor's update, kUP threads per column k of F (r x len), thread p
// taking the rows a = p, p + kUP, ...:
//   num[a][k]                                (X W' or V' X, the split sums)
//   den = (G F)[a][k]                        (W W' V' or V' V W)
//   multiplicative: F <- F num / (den + eps); APG: F <- max(0, F - step (den - num)),
//   step = 1 / (2 ||G||_F^2 + eps)
// Every old value of the workgroup's columns is read before any is written.
constexpr int kUC = 64;         // columns per workgroup of the update
constexpr int kUP = kT / kUC;   // threads per column
template <int R>
__global__ __launch_bounds__(kT) void nmf_update_kernel(double* __restrict__ F, int r, int64_t len,
                                                        const double* __restrict__ num_, const double* __restrict__ G,
                                                        int algo, double eps)
{
    __shared__ double Gs[R * R];
    __shared__ double sh[kT / kWave];
    for (int q = threadIdx.x; q < R * R; q += kT) {
        const int a = q / R, b = q % R;
        Gs[q] = (a < r && b < r) ? G[a * r + b] : 0.0;
    }
    __syncthreads();
    double step = 0.0;
    if (algo == 1) {
        double s2 = 0.0;
        for (int q = threadIdx.x; q < R * R; q += kT) s2 += Gs[q] * Gs[q];
        step = 1.0 / (2.0 * block_sum256(s2, sh) + eps);
    }
    const int p = threadIdx.x / kUC;
    const int64_t k = (int64_t)blockIdx.x * kUC + threadIdx.x % kUC;
    const bool live = k < len;
    double old[R];
#pragma unroll
    for (int a = 0; a < R; ++a) old[a] = (live && a < r) ? F[(int64_t)a * len + k] : 0.0;
    __syncthreads();
    if (!live) return;
    for (int a = p; a < r; a += kUP) {
        const double num = num_[(int64_t)a * len + k];
        double den = 0.0;
#pragma unroll
        for (int b = 0; b < R; ++b) den += Gs[a * R + b] * old[b];
        // only this thread writes row a of column k, so F[a][k] is still the old value
        const double oa = F[(int64_t)a * len + k];
        F[(int64_t)a * len + k] = algo == 0 ? oa * num / (den + eps) : fmax(0.0, oa - step * (den - num));
    }
}

// out[0] = sum_a sum_k F[a][k] num[a][k]
__global__ __launch_bounds__(kT) void nmf_inner_kernel(const double* __restrict__ F, int r, int64_t len,
                                                       const double* __restrict__ num, double* __restrict__ out)
{
    __shared__ double sh[kT / kWave];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < (int64_t)r * len; t += kT) s += F[t] * num[t];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// partial sums of X_ij^2 per row block, then their sum in a fixed order
__global__ __launch_bounds__(kT) void nmf_xnorm_kernel(const float* __restrict__ X, int64_t m, int64_t n,
                                                       int64_t ldx, double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const int64_t i = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += kT) {
        const double x = X[i * ldx + j];
        s += x * x;
    }
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) part[i] = s;
}

__global__ __launch_bounds__(kT) void nmf_sum_kernel(const double* __restrict__ v, int64_t len,
                                                     double* __restrict__ out)
{
    __shared__ double sh[kT / kWave];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < len; k += kT) s += v[k];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// f = ||X||^2 - 2 <W, V'X> + <V'V, W W'>
__global__ void nmf_objective_kernel(const double* __restrict__ scal, const double* __restrict__ VtV,
                                     const double* __restrict__ WWt, int r, double* __restrict__ f)
{
    if (threadIdx.x != 0) return;
    double c = 0.0;
    for (int q = 0; q < r * r; ++q) c += VtV[q] * WWt[q];
    f[0] = scal[0] - 2.0 * scal[1] + c;
}

// The rank padded to whole 16-row matrix-core tiles.
int rpad(int r) { return (r + 15) / 16 * 16; }

inline unsigned grid_for(int64_t m) { return (unsigned)min((int64_t)8192, max((int64_t)1, (m + kT - 1) / kT)); }

}  // namespace
}  // namespace cox

using namespace cox;

struct nmf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    const float* X = nullptr;
    int64_t m = 0, n = 0, ldx = 0;
    int r = 0;
    int ns_wxt = 1, ns_vtx = 1;
    int64_t cols = 0, rows = 0;
    double *part = nullptr, *num = nullptr, *WWt = nullptr, *VtV = nullptr, *scal = nullptr, *xpart = nullptr;
    std::vector<void*> allocs;
    std::string err;
    bool timing = false;
    std::vector<hipEvent_t> tev[2];
    double tms[2] = {};
    int64_t tcount[2] = {};
};

namespace {

cox_status nfail(nmf_ctx* c, cox_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

#define NCHK(expr, what)                                                                              \
    do {                                                                                              \
        hipError_t _e = (expr);                                                                       \
        if (_e != hipSuccess) return nfail(c, COX_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

void nmf_release(nmf_ctx* c)
{
    for (int ph = 0; ph < 2; ++ph) {
        for (hipEvent_t e : c->tev[ph]) (void)hipEventDestroy(e);
        c->tev[ph].clear();
    }
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

template <class T>
bool nalloc(nmf_ctx* c, T** out, size_t count)
{
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    c->allocs.push_back(p);
    *out = static_cast<T*>(p);
    return true;
}

void nmark(nmf_ctx* c, int ph)
{
    if (!c->timing) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    (void)hipEventRecord(e, c->stream);
    c->tev[ph].push_back(e);
}

// V'X split partials and V'V of the current V'
// the rows of X and of W start 16-byte aligned: W X' loads straight from memory
bool nmf_direct(const nmf_ctx* c, const double* W)
{
    return reinterpret_cast<uintptr_t>(c->X) % 16 == 0 && c->ldx % 4 == 0 && c->n % 2 == 0 &&
           reinterpret_cast<uintptr_t>(W) % 16 == 0;
}

// columns per lane in a step of the direct W X' pass
constexpr int direct_gl(int R) { return R <= 16 ? 8 : 4; }

template <int R>
void nmf_vtx_gram(nmf_ctx* c, const double* Vt)
{
    const int r = c->r;
    const unsigned gn = (unsigned)((c->n + kT - 1) / kT);
    nmark(c, 1);
    hipLaunchKernelGGL((nmf_vtx_kernel<R / 16>), dim3(gn, c->ns_vtx), dim3(kT), 0, c->stream, c->X, c->m, c->n,
                       c->ldx, r, Vt, c->rows, c->part);
    nmark(c, 1);
    hipLaunchKernelGGL(nmf_reduce_kernel, dim3(grid_for((int64_t)r * c->n)), dim3(kT), 0, c->stream, c->part,
                       c->ns_vtx, (int64_t)r * c->n, c->num);
    hipLaunchKernelGGL(nmf_gram_kernel, dim3((unsigned)(r * (r + 1) / 2)), dim3(kT), 0, c->stream, Vt, r, c->m,
                       c->VtV);
}

template <int R>
hipError_t nmf_iteration(nmf_ctx* c, int algo, double eps, double* Vt, double* W)
{
    const int r = c->r;
    const unsigned gm = (unsigned)((c->m + kT - 1) / kT);
    nmark(c, 0);
    if (nmf_direct(c, W))
        hipLaunchKernelGGL((nmf_wxt_direct_kernel<R / 16, direct_gl(R)>), dim3(gm, c->ns_wxt), dim3(kT), 0, c->stream,
                           c->X, c->m, c->n, c->ldx, r, W, c->cols, c->part);
    else
        hipLaunchKernelGGL((nmf_wxt_kernel<R / 16>), dim3(gm, c->ns_wxt), dim3(kT), 0, c->stream, c->X, c->m, c->n,
                           c->ldx, r, W, c->cols, c->part);
    nmark(c, 0);
    hipLaunchKernelGGL(nmf_reduce_kernel, dim3(grid_for((int64_t)r * c->m)), dim3(kT), 0, c->stream, c->part,
                       c->ns_wxt, (int64_t)r * c->m, c->num);
    hipLaunchKernelGGL(nmf_gram_kernel, dim3((unsigned)(r * (r + 1) / 2)), dim3(kT), 0, c->stream, W, r, c->n,
                       c->WWt);
    hipLaunchKernelGGL((nmf_update_kernel<R>), dim3((unsigned)((c->m + kUC - 1) / kUC)), dim3(kT), 0, c->stream, Vt, r,
                       c->m, c->num, c->WWt, algo, eps);
    nmf_vtx_gram<R>(c, Vt);
    hipLaunchKernelGGL((nmf_update_kernel<R>), dim3((unsigned)((c->n + kUC - 1) / kUC)), dim3(kT), 0, c->stream, W, r,
                       c->n, c->num, c->VtV, algo, eps);
    return hipGetLastError();
}

template <int R>
hipError_t nmf_dispatch(nmf_ctx* c, int algo, double eps, double* Vt, double* W, int iters, bool vtx_only)
{
    if (vtx_only) {
        nmf_vtx_gram<R>(c, Vt);
        return hipGetLastError();
    }
    for (int k = 0; k < iters; ++k) {
        const hipError_t e = nmf_iteration<R>(c, algo, eps, Vt, W);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t nmf_dispatch_r(nmf_ctx* c, int algo, double eps, double* Vt, double* W, int iters, bool vtx_only)
{
    switch (rpad(c->r)) {
    case 16: return nmf_dispatch<16>(c, algo, eps, Vt, W, iters, vtx_only);
    case 32: return nmf_dispatch<32>(c, algo, eps, Vt, W, iters, vtx_only);
    case 48: return nmf_dispatch<48>(c, algo, eps, Vt, W, iters, vtx_only);
    default: return nmf_dispatch<64>(c, algo, eps, Vt, W, iters, vtx_only);
    }
}

}  // namespace

extern "C" {

cox_status nmf_setup(nmf_ctx** out, const float* X, int64_t m, int64_t n, int64_t ldx, int32_t r, void* hip_stream)
{
    if (!out) return COX_ERR_INVALID_ARG;
    *out = nullptr;
    if (!X || m < 1 || n < 1 || ldx < n || r < 1 || r > NMF_MAX_RANK || m >= (1LL << 31) || n >= (1LL << 31))
        return COX_ERR_INVALID_ARG;
    nmf_ctx* c = new (std::nothrow) nmf_ctx;
    if (!c) return COX_ERR_OUT_OF_MEMORY;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return COX_ERR_DEVICE;
    }
    c->X = X;
    c->m = m;
    c->n = n;
    c->ldx = ldx;
    c->r = r;
    // split the inner dimension so each pass has several workgroups per CU
    const int64_t gm = (m + kT - 1) / kT, gn = (n + kT - 1) / kT;
    c->ns_wxt = (int)std::max<int64_t>(1, std::min<int64_t>((n + kTJ - 1) / kTJ, (1024 + gm - 1) / gm));
    c->ns_vtx = (int)std::max<int64_t>(1, std::min<int64_t>((m + kTI - 1) / kTI, (1024 + gn - 1) / gn));
    c->cols = ((n + c->ns_wxt - 1) / c->ns_wxt + kTJ - 1) / kTJ * kTJ;
    c->ns_wxt = (int)((n + c->cols - 1) / c->cols);
    c->rows = ((m + c->ns_vtx - 1) / c->ns_vtx + kTI - 1) / kTI * kTI;
    c->ns_vtx = (int)((m + c->rows - 1) / c->rows);
    const size_t pmax = std::max((size_t)c->ns_wxt * r * m, (size_t)c->ns_vtx * r * n);
    if (!(nalloc(c, &c->part, pmax) && nalloc(c, &c->num, (size_t)r * std::max(m, n)) &&
          nalloc(c, &c->WWt, (size_t)r * r) && nalloc(c, &c->VtV, (size_t)r * r) &&
          nalloc(c, &c->scal, 4) && nalloc(c, &c->xpart, m))) {
        nmf_release(c);
        delete c;
        return COX_ERR_OUT_OF_MEMORY;
    }
    // ||X||_F^2 once, for the objective
    hipLaunchKernelGGL(nmf_xnorm_kernel, dim3((unsigned)m), dim3(kT), 0, c->stream, X, m, n, ldx, c->xpart);
    hipLaunchKernelGGL(nmf_sum_kernel, dim3(1), dim3(kT), 0, c->stream, c->xpart, m, c->scal);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        nmf_release(c);
        delete c;
        return COX_ERR_DEVICE;
    }
    *out = c;
    return COX_OK;
}

cox_status nmf_destroy(nmf_ctx* c)
{
    if (!c) return COX_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    nmf_release(c);
    delete c;
    return COX_OK;
}

cox_status nmf_last_error(const nmf_ctx* c, char* buf, size_t len)
{
    if (!c || !buf || len == 0) return COX_ERR_INVALID_ARG;
    const size_t k = std::min(len - 1, c->err.size());
    std::memcpy(buf, c->err.data(), k);
    buf[k] = '\0';
    return COX_OK;
}

cox_status nmf_run(nmf_ctx* c, int32_t algo, int32_t iters, double eps, double* Vt, double* W, double* obj)
{
    if (!c) return COX_ERR_INVALID_ARG;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return nfail(c, COX_ERR_DEVICE, "hipSetDevice failed");
    if ((algo != NMF_MULTIPLICATIVE && algo != NMF_APG) || iters < 0 || !(eps >= 0) || !std::isfinite(eps) || !Vt ||
        !W)
        return nfail(c, COX_ERR_INVALID_ARG, "bad nmf_run arguments");
    NCHK(nmf_dispatch_r(c, algo, eps, Vt, W, iters, false), "NMF iteration");
    if (obj) {
        const int r = c->r;
        // V'X and V'V of the final V are still in the workspace after an
        // iteration; with none, form them
        if (iters == 0) NCHK(nmf_dispatch_r(c, algo, eps, Vt, W, 0, true), "V'X");
        hipLaunchKernelGGL(nmf_inner_kernel, dim3(1), dim3(kT), 0, c->stream, W, r, c->n, c->num, c->scal + 1);
        hipLaunchKernelGGL(nmf_gram_kernel, dim3((unsigned)(r * (r + 1) / 2)), dim3(kT), 0, c->stream, W, r, c->n,
                           c->WWt);
        hipLaunchKernelGGL(nmf_objective_kernel, dim3(1), dim3(64), 0, c->stream, c->scal, c->VtV, c->WWt, r,
                           c->scal + 2);
        NCHK(hipGetLastError(), "objective");
        NCHK(hipMemcpyAsync(obj, c->scal + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream), "objective");
        NCHK(hipStreamSynchronize(c->stream), "synchronise");
        if (!std::isfinite(*obj)) return nfail(c, COX_ERR_NUMERIC, "non-finite objective");
    }
    return COX_OK;
}

cox_status nmf_timing_enable(nmf_ctx* c, int32_t enable)
{
    if (!c) return COX_ERR_INVALID_ARG;
    NCHK(hipStreamSynchronize(c->stream), "synchronise");
    for (int ph = 0; ph < 2; ++ph) {
        for (hipEvent_t e : c->tev[ph]) (void)hipEventDestroy(e);
        c->tev[ph].clear();
        c->tms[ph] = 0;
        c->tcount[ph] = 0;
    }
    c->timing = enable != 0;
    return COX_OK;
}

cox_status nmf_timing_read(nmf_ctx* c, int32_t phase, double* total_ms, int64_t* count)
{
    if (!c || phase < 0 || phase > 1 || !total_ms) return COX_ERR_INVALID_ARG;
    NCHK(hipStreamSynchronize(c->stream), "synchronise");
    auto& ev = c->tev[phase];
    for (size_t q = 0; q + 1 < ev.size(); q += 2) {
        float ms = 0;
        NCHK(hipEventElapsedTime(&ms, ev[q], ev[q + 1]), "event time");
        c->tms[phase] += ms;
        c->tcount[phase] += 1;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    *total_ms = c->tms[phase];
    if (count) *count = c->tcount[phase];
    return COX_OK;
}

}  // extern "C"
