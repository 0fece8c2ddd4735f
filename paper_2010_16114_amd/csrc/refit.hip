// refit.hip -- the unpenalised Cox refit on a chosen set of columns.
//
// Section 6 ranks the SNPs that the lasso path selects, then refits the
// unpenalised Cox model on them together with the covariates and keeps those
// whose Wald p-value passes a Bonferroni threshold.  The refit here is
// Newton's method on L over the M chosen columns, gathered into a dense FP32
// block D (n x M, column-major, rows in subject order; genotype columns
// standardised as (g - mu_j) s_j, formed in FP64 and rounded once).
//
// With w = exp(eta - max eta), r = delta - w c (the risk-set pass), and in the
// sorted order S1(k) = sum_{k' <= k} w_k' d_k' (the risk-set sums of the rows
// of D), the negative Hessian of L in the coefficients is
//     -H = sum_i w_i c_i d_i d_i'  -  sum_G n_G S1(G) S1(G)' / W(G)^2
// where the first sum runs over subjects (w_i c_i = delta_i - r_i) and the
// second over tie groups G with n_G > 0 events, read at the group's last
// sorted position (Breslow).  Both terms are Gram matrices of tall n-row
// arrays: D with row weights delta - r, and U with row sqrt(n_G) S1(G) / W(G)
// at each group end and 0 elsewhere.  They are formed from fixed-order
// partial sums in FP64.  -H is factorised by Cholesky in one workgroup; the
// Newton direction and the diagonal of (-H)^{-1} (squared standard errors)
// come from that factor.
#include "device_common.h"

namespace cox {
namespace {

constexpr int kT = 256;
constexpr int kGT = 64;     // Gram output tile (kGT x kGT)
constexpr int kGR = 32;     // rows per LDS step of the Gram kernel

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

// D[a][i] = x~(i, cols[a]) for i < n
__global__ __launch_bounds__(kT) void gather_kernel(XDesc x, const int32_t* __restrict__ cols, float* __restrict__ D,
                                                    int64_t ldd)
{
    const int a = blockIdx.y;
    const int64_t j = cols[a];
    double mu = 0.0, sc = 1.0;
    if (x.xt != XT_F32) {
        if (x.center) mu = x.center[j];
        if (x.scale) sc = x.scale[j];
    }
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < x.n; i += (int64_t)gridDim.x * kT) {
        const int64_t off = j * x.ldx + i;
        double v;
        if (x.xt == XT_F32)
            v = load_x1<XT_F32>(x.X, off);
        else if (x.xt == XT_FP8)
            v = ((double)load_x1<XT_FP8>(x.X, off) - mu) * sc;
        else
            v = ((double)load_x1<XT_I8>(x.X, off) - mu) * sc;
        D[(int64_t)a * ldd + i] = (float)v;
    }
}

// eta[i] = sum_a D[a][i] b[a]
__global__ __launch_bounds__(kT) void refit_eta_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                       const double* __restrict__ b, double* __restrict__ eta)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        double s = 0.0;
        for (int a = 0; a < M; ++a) s += (double)D[(int64_t)a * ldd + i] * b[a];
        eta[i] = s;
    }
}

// part[rb][a] = sum over row block rb of D[a][i] r[i]
__global__ __launch_bounds__(kT) void refit_xtr_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                       const double* __restrict__ r, int64_t rows,
                                                       double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const int a = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * rows, i1 = min(n, i0 + rows);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kT) s += (double)D[(int64_t)a * ldd + i] * r[i];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * M + a] = s;
}

// g[a] = sum_rb part[rb][a], in row-block order
__global__ void refit_sum_kernel(const double* __restrict__ part, int nrb, int M, double* __restrict__ g)
{
    const int a = blockIdx.x * kT + threadIdx.x;
    if (a >= M) return;
    double s = 0.0;
    for (int rb = 0; rb < nrb; ++rb) s += part[(int64_t)rb * M + a];
    g[a] = s;
}

// row weights of the first Hessian term, in subject order: wt[perm[k]] = delta - r
__global__ void hess_weight_kernel(const int32_t* __restrict__ perm, const uint8_t* __restrict__ ev,
                                   const double* __restrict__ r, int64_t n, double* __restrict__ wt)
{
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < n; k += (int64_t)gridDim.x * kT) {
        const int32_t i = perm[k];
        wt[i] = (ev[k] ? 1.0 : 0.0) - r[i];
    }
}

// S[a][k] = sum_{k' <= k} w[k'] D[a][perm[k']] in sorted order (a < M), and
// S[M][k] = sum_{k' <= k} w[k'].  One workgroup per column walks all positions
// in chunks of 4 * kT with a running carry.
__global__ __launch_bounds__(kT) void scan_cols_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                       const int32_t* __restrict__ perm, const double* __restrict__ w,
                                                       double* __restrict__ S)
{
    __shared__ double wsum[kT / kWave];
    const int a = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    double carry = 0.0;
    for (int64_t k0 = 0; k0 < n; k0 += 4 * kT) {
        // each thread takes 4 consecutive positions
        const int64_t kb = k0 + 4 * (int64_t)threadIdx.x;
        double v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t k = kb + e;
            double x = 0.0;
            if (k < n) x = a < M ? w[k] * (double)D[(int64_t)a * ldd + perm[k]] : w[k];
            v[e] = x;
        }
        v[1] += v[0];
        v[2] += v[1];
        v[3] += v[2];
        double incl = wave_incl_scan(v[3], lane);
        if (lane == kWave - 1) wsum[wid] = incl;
        __syncthreads();
        double before = carry;
        for (int q = 0; q < wid; ++q) before += wsum[q];
        double total = carry;
        for (int q = 0; q < kT / kWave; ++q) total += wsum[q];
        const double excl = before + incl - v[3];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t k = kb + e;
            if (k < n) S[(int64_t)a * n + k] = excl + v[e];
        }
        carry = total;
        __syncthreads();
    }
}

// U rows in place of S[0..M): at the last position k of a tie group with
// n_G > 0 events, U[a][k] = sqrt(n_G) S[a][k] / S[M][k]; 0 elsewhere.
__global__ void u_rows_kernel(double* __restrict__ S, int64_t n, int M, const int32_t* __restrict__ gstart,
                              const int32_t* __restrict__ gend, const uint8_t* __restrict__ ev)
{
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < n; k += (int64_t)gridDim.x * kT) {
        double f = 0.0;
        if (gend[k] == k) {
            int nev = 0;
            for (int64_t q = gstart[k]; q <= k; ++q) nev += ev[q];
            if (nev > 0) f = sqrt((double)nev) / S[(int64_t)M * n + k];
        }
        for (int a = 0; a < M; ++a) S[(int64_t)a * n + k] *= f;
    }
}

// part[chunk][a][b] = sum over the chunk's rows of wt_i A[a][i] A[b][i], for
// the 64 x 64 output tile (ta, tb), ta <= tb (upper tiles only).
template <class T>
__global__ __launch_bounds__(kT) void gram_kernel(const T* __restrict__ A, int64_t lda, int64_t n, int M,
                                                  const double* __restrict__ wt, int64_t rows, int ntile,
                                                  double* __restrict__ part)
{
    __shared__ double As[kGR][kGT + 1], Bs[kGR][kGT + 1];
    // upper-triangle tile pair from the linear index
    int idx = blockIdx.x, ta = 0;
    while (idx >= ntile - ta) {
        idx -= ntile - ta;
        ++ta;
    }
    const int tb = ta + idx;
    const int64_t r0 = (int64_t)blockIdx.y * rows, r1 = min(n, r0 + rows);
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int64_t rs = r0; rs < r1; rs += kGR) {
        // stage kGR rows x 64 columns of both tiles; consecutive threads take consecutive rows
#pragma unroll
        for (int e = 0; e < kGR * kGT / kT; ++e) {
            const int li = threadIdx.x + kT * e;
            const int rr = li % kGR, cc = li / kGR;
            const int64_t row = rs + rr;
            const int ca = ta * kGT + cc, cb = tb * kGT + cc;
            double va = 0.0, vb = 0.0;
            if (row < r1) {
                const double wv = wt ? wt[row] : 1.0;
                if (ca < M) va = (double)A[(int64_t)ca * lda + row] * wv;
                if (cb < M) vb = (double)A[(int64_t)cb * lda + row];
            }
            As[rr][cc] = va;
            Bs[rr][cc] = vb;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kGR; ++rr) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = As[rr][tr * 4 + u];
#pragma unroll
            for (int v = 0; v < 4; ++v) bv[v] = Bs[rr][tc * 4 + v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = ta * kGT + tr * 4 + u, b = tb * kGT + tc * 4 + v;
            if (a < M && b < M) part[((int64_t)blockIdx.y * M + a) * M + b] = acc[u][v];
        }
}

// H[a][b] = sum_c p1[c][a][b] - sum_c p2[c][a][b], each entry read from the
// upper tile pair that holds it (the lower ones mirror it).
__global__ void gram_reduce_kernel(const double* __restrict__ p1, const double* __restrict__ p2, int nchunk, int M,
                                   double* __restrict__ H)
{
    const int64_t mm = (int64_t)M * M;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < mm; t += (int64_t)gridDim.x * kT) {
        const int a = (int)(t / M), b = (int)(t % M);
        // the Gram kernel wrote (a, b) when tile(a) <= tile(b)
        const bool upper = a / kGT <= b / kGT;
        const int64_t at = upper ? (int64_t)a * M + b : (int64_t)b * M + a;
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += p1[c * mm + at];
        for (int c = 0; c < nchunk; ++c) s -= p2[c * mm + at];
        H[t] = s;
    }
}

// In-place Cholesky A = L L' of the symmetric positive definite M x M matrix
// (row-major; the lower triangle receives L).  One workgroup, right-looking:
// at step j the pivot column is scaled and staged in LDS, then the trailing
// lower triangle A[i][k] -= L[i][j] L[k][j] (j < k <= i) is updated with the
// pairs spread evenly over the threads, four per batch so that their loads
// overlap.  ok[0] = 1 on success, 0 when a pivot is not positive.
__global__ __launch_bounds__(kT) void chol_kernel(double* __restrict__ A, int M, int* __restrict__ ok)
{
    __shared__ double col[kMaxRefit];
    __shared__ double piv;
    __shared__ int good;
    if (threadIdx.x == 0) good = 1;
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        if (threadIdx.x == 0) {
            const double d = A[(int64_t)j * M + j];
            if (!(d > 0.0)) good = 0;
            piv = d > 0.0 ? sqrt(d) : 1.0;
            A[(int64_t)j * M + j] = piv;
        }
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < M; i += kT) {
            const double v = A[(int64_t)i * M + j] / piv;
            A[(int64_t)i * M + j] = v;
            col[i] = v;
        }
        __syncthreads();
        // pair t of the trailing triangle: row i' = the largest with i'(i'+1)/2 <= t,
        // column k' = t - i'(i'+1)/2, both offset by j + 1
        const int64_t w = M - j - 1, npair = w * (w + 1) / 2;
        for (int64_t t0 = (int64_t)threadIdx.x * 4; t0 < npair; t0 += 4 * kT) {
            int64_t at[4];
            double upd[4], cur[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t t = min(t0 + e, npair - 1);
                int64_t ii = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
                while (ii * (ii + 1) / 2 > t) --ii;
                while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
                const int64_t kk = t - ii * (ii + 1) / 2;
                const int64_t i = j + 1 + ii, k = j + 1 + kk;
                at[e] = i * M + k;
                upd[e] = col[i] * col[k];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) cur[e] = A[at[e]];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t0 + e < npair) A[at[e]] = cur[e] - upd[e];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ok[0] = good;
}

// x = (L L')^{-1} g with the factor from chol_kernel.  One workgroup.
__global__ __launch_bounds__(kT) void chol_solve_kernel(const double* __restrict__ L, int M,
                                                        const double* __restrict__ g, double* __restrict__ x)
{
    __shared__ double sh[kT / kWave];
    for (int i = 0; i < M; ++i) {  // L y = g
        double s = 0.0;
        for (int k = threadIdx.x; k < i; k += kT) s += L[(int64_t)i * M + k] * x[k];
        s = block_sum256(s, sh);
        if (threadIdx.x == 0) x[i] = (g[i] - s) / L[(int64_t)i * M + i];
        __syncthreads();
    }
    for (int i = M - 1; i >= 0; --i) {  // L' x = y
        double s = 0.0;
        for (int k = i + 1 + threadIdx.x; k < M; k += kT) s += L[(int64_t)k * M + i] * x[k];
        s = block_sum256(s, sh);
        if (threadIdx.x == 0) x[i] = (x[i] - s) / L[(int64_t)i * M + i];
        __syncthreads();
    }
}

// Wald statistics from the factor: thread a solves L y = e_a (y in
// scratch[a][.]), so ((L L')^{-1})_aa = |y|^2; se_a = its square root,
// z_a = b_a / se_a, p_a = erfc(|z_a| / sqrt 2).
__global__ void wald_kernel(const double* __restrict__ L, int M, const double* __restrict__ b,
                            double* __restrict__ scratch, double* __restrict__ se, double* __restrict__ pval)
{
    const int a = blockIdx.x * kT + threadIdx.x;
    if (a >= M) return;
    double* y = scratch + (int64_t)a * M;
    double s2 = 0.0;
    for (int i = a; i < M; ++i) {
        double t = i == a ? 1.0 : 0.0;
        for (int k = a; k < i; ++k) t -= L[(int64_t)i * M + k] * y[k];
        t /= L[(int64_t)i * M + i];
        y[i] = t;
        s2 += t * t;
    }
    const double sd = sqrt(s2);
    se[a] = sd;
    pval[a] = erfc(fabs(b[a] / sd) * 0.70710678118654752440);
}

// out = b + t d
__global__ void axpy_kernel(const double* __restrict__ b, const double* __restrict__ d, double t, int M,
                            double* __restrict__ out)
{
    const int a = blockIdx.x * kT + threadIdx.x;
    if (a < M) out[a] = b[a] + t * d[a];
}

// first sorted position with a nonzero coefficient per column: entry[j] = the
// smallest l with path[l][j] != 0 (or -1), coef[j] = |path[entry][j]|
__global__ void entry_kernel(const float* __restrict__ path, int L, int64_t ptot, int64_t p,
                             int32_t* __restrict__ entry, float* __restrict__ coef)
{
    for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < p; j += (int64_t)gridDim.x * kT) {
        int e = -1;
        float c = 0.0f;
        for (int l = 0; l < L; ++l) {
            const float v = path[(int64_t)l * ptot + j];
            if (v != 0.0f) {
                e = l;
                c = fabsf(v);
                break;
            }
        }
        entry[j] = e;
        coef[j] = c;
    }
}

inline unsigned grid_for(int64_t m) { return (unsigned)min((int64_t)8192, max((int64_t)1, (m + kT - 1) / kT)); }

}  // namespace

hipError_t launch_gather_cols(const XDesc& x, const int32_t* cols, int m, float* D, int64_t ldd, hipStream_t s)
{
    if (m < 1 || ldd < x.n) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)min((int64_t)512, (x.n + kT - 1) / kT);
    hipLaunchKernelGGL(gather_kernel, dim3(gx, m), dim3(kT), 0, s, x, cols, D, ldd);
    return hipGetLastError();
}

hipError_t launch_refit_eta(const float* D, int64_t ldd, int64_t n, int M, const double* b, double* eta, hipStream_t s)
{
    hipLaunchKernelGGL(refit_eta_kernel, dim3(grid_for(n)), dim3(kT), 0, s, D, ldd, n, M, b, eta);
    return hipGetLastError();
}

int refit_row_blocks(int64_t n) { return (int)((n + kRefitRows - 1) / kRefitRows); }

hipError_t launch_refit_grad(const float* D, int64_t ldd, int64_t n, int M, const double* r, double* part, double* g,
                             hipStream_t s)
{
    const int nrb = refit_row_blocks(n);
    hipLaunchKernelGGL(refit_xtr_kernel, dim3(nrb, M), dim3(kT), 0, s, D, ldd, n, M, r, (int64_t)kRefitRows, part);
    hipLaunchKernelGGL(refit_sum_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, part, nrb, M, g);
    return hipGetLastError();
}

int gram_chunks(int64_t n) { return (int)min((int64_t)kGramChunks, max((int64_t)1, (n + 4095) / 4096)); }

static int64_t gram_rows(int64_t n)
{
    const int nc = gram_chunks(n);
    return ((n + nc - 1) / nc + kGR - 1) / kGR * kGR;
}

hipError_t launch_refit_hessian(const float* D, int64_t ldd, int64_t n, int M, const int32_t* perm,
                                const int32_t* gstart, const int32_t* gend, const uint8_t* ev, const double* w,
                                const double* r, double* wt, double* S, double* part1, double* part2, double* H,
                                hipStream_t s)
{
    if (M < 1 || M > kMaxRefit) return hipErrorInvalidValue;
    const int ntile = (M + kGT - 1) / kGT, npair = ntile * (ntile + 1) / 2;
    const int nc = gram_chunks(n);
    const int64_t rows = gram_rows(n);
    hipLaunchKernelGGL(hess_weight_kernel, dim3(grid_for(n)), dim3(kT), 0, s, perm, ev, r, n, wt);
    hipLaunchKernelGGL((gram_kernel<float>), dim3(npair, nc), dim3(kT), 0, s, D, ldd, n, M, wt, rows, ntile, part1);
    hipLaunchKernelGGL(scan_cols_kernel, dim3(M + 1), dim3(kT), 0, s, D, ldd, n, M, perm, w, S);
    hipLaunchKernelGGL(u_rows_kernel, dim3(grid_for(n)), dim3(kT), 0, s, S, n, M, gstart, gend, ev);
    hipLaunchKernelGGL((gram_kernel<double>), dim3(npair, nc), dim3(kT), 0, s, S, n, n, M, nullptr, rows, ntile,
                       part2);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(grid_for((int64_t)M * M)), dim3(kT), 0, s, part1, part2, nc, M, H);
    return hipGetLastError();
}

hipError_t launch_chol(double* A, int M, int* ok, hipStream_t s)
{
    hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(kT), 0, s, A, M, ok);
    return hipGetLastError();
}

hipError_t launch_chol_solve(const double* L, int M, const double* g, double* x, hipStream_t s)
{
    hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(kT), 0, s, L, M, g, x);
    return hipGetLastError();
}

hipError_t launch_wald(const double* L, int M, const double* b, double* scratch, double* se, double* pval,
                       hipStream_t s)
{
    hipLaunchKernelGGL(wald_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, L, M, b, scratch, se, pval);
    return hipGetLastError();
}

hipError_t launch_axpy(const double* b, const double* d, double t, int M, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(axpy_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, b, d, t, M, out);
    return hipGetLastError();
}

hipError_t launch_entry(const float* path, int L, int64_t ptot, int64_t p, int32_t* entry, float* coef, hipStream_t s)
{
    hipLaunchKernelGGL(entry_kernel, dim3(grid_for(p)), dim3(kT), 0, s, path, L, ptot, p, entry, coef);
    return hipGetLastError();
}

}  // namespace cox
