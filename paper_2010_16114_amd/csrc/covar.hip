// covar.hip -- the dense block of covariates beside X.
//
// Section 6's application fits sex and the top principal components as
// unpenalised covariates next to the SNPs.  Those columns are real-valued, so
// they cannot share the one-byte storage of allele counts: they live in a
// dense FP32 block Z (n x q, column-major, column k at Z + k * ldz) and the
// model matrix is [X~ | Z].  The covariate coefficients take the same steps as
// those of X (Section 5.3):
//   g_Z = Z' r                                   (part of Delta = X'(I - P) delta)
//   beta_Zk <- S_{sigma lambda pf_k}(beta_Zk + sigma g_Zk)   (pf_k = 0: no threshold)
//   eta <- eta + Z (beta_Z new - beta_Z old).
//
// Z' r: workgroups over (row block of kCovRows rows, b) hold their slice of r
// in registers and write one partial sum per covariate in a fixed order; the
// epilogue adds the partials in row-block order, so results are reproducible
// bit for bit.  FP32 Z times the stored residual is formed and summed in FP64.
#include "device_common.h"

namespace cox {
namespace {

constexpr int kT = 256;
constexpr int kRowsPerThread = kCovRows / kT;
constexpr int kChunk = 8;  // covariates reduced together

inline unsigned grid_for(int64_t m) { return (unsigned)min((int64_t)8192, max((int64_t)1, (m + kT - 1) / kT)); }

__global__ __launch_bounds__(kT) void cov_xtr_part_kernel(CovArgs c, const float* __restrict__ r32,
                                                          int64_t rstride, const double* __restrict__ r64,
                                                          const int32_t* __restrict__ active)
{
    __shared__ double sh[kT / kWave][kMaxCov];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t i0 = (int64_t)blockIdx.x * kCovRows;
    double rv[kRowsPerThread];
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
        const int64_t i = i0 + threadIdx.x + (int64_t)kT * u;
        rv[u] = i < c.n ? (r32 ? (double)r32[(int64_t)b * rstride + i] : r64[(int64_t)b * c.n + i]) : 0.0;
    }
    for (int k0 = 0; k0 < c.q; k0 += kChunk) {
        double acc[kChunk];
#pragma unroll
        for (int e = 0; e < kChunk; ++e) acc[e] = 0.0;
#pragma unroll
        for (int u = 0; u < kRowsPerThread; ++u) {
            const int64_t i = i0 + threadIdx.x + (int64_t)kT * u;
            if (i >= c.n) break;
#pragma unroll
            for (int e = 0; e < kChunk; ++e)
                if (k0 + e < c.q) acc[e] += (double)c.Z[(int64_t)(k0 + e) * c.ldz + i] * rv[u];
        }
#pragma unroll
        for (int e = 0; e < kChunk; ++e) {
            const double v = wave_sum(acc[e]);
            if (lane == 0 && k0 + e < c.q) sh[wid][k0 + e] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < c.q) {
        double s = 0.0;
        for (int w = 0; w < kT / kWave; ++w) s += sh[w][threadIdx.x];
        c.part[((int64_t)b * c.nrb + blockIdx.x) * c.q + threadIdx.x] = s;
    }
}

// One wavefront per b, lane k = covariate k.
__global__ __launch_bounds__(kWave) void cov_epilogue_kernel(CovArgs c, CovStep st)
{
    const int b = blockIdx.x, k = threadIdx.x;
    const bool valid = k < c.q;
    double g = 0.0;
    if (valid)
        for (int rb = 0; rb < c.nrb; ++rb) g += c.part[((int64_t)b * c.nrb + rb) * c.q + k];
    if (st.out64 && valid) st.out64[(int64_t)b * st.ostride + k] = g;
    if (st.mode == GT_GRAD) {
        if (valid) st.out32[(int64_t)b * st.ostride + k] = (float)(-g);
        return;
    }
    if (st.mode != GT_PROX) return;
    double l1o = 0.0, l1n = 0.0;
    if (valid) {
        const int64_t at = (int64_t)b * c.q + k;
        const double f = st.pf[k];
        const double old = st.beta[at];
        double nw = old;
        if (st.active == nullptr || st.active[b]) nw = soft_threshold(old + st.step * g, f == 0.0 ? 0.0 : st.step * st.lam[b] * f);
        st.beta[at] = nw;
        st.dbeta[at] = nw - old;
        l1o = f * fabs(old);
        l1n = f * fabs(nw);
    }
    l1o = wave_sum(l1o);
    l1n = wave_sum(l1n);
    if (k == 0) {
        st.l1old[b] = l1o;
        st.l1new[b] = l1n;
    }
}

// eta_b(i) += sum_k Z(i, k) coef_b(k)
__global__ __launch_bounds__(kT) void cov_eta_kernel(CovArgs c, const double* __restrict__ coef, double* __restrict__ eta,
                                                     const int32_t* __restrict__ active)
{
    __shared__ double cb[kMaxCov];
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    if (threadIdx.x < c.q) cb[threadIdx.x] = coef[(int64_t)b * c.q + threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < c.n; i += (int64_t)gridDim.x * kT) {
        double s = 0.0;
        for (int k = 0; k < c.q; ++k) s += (double)c.Z[(int64_t)k * c.ldz + i] * cb[k];
        eta[(int64_t)b * c.n + i] += s;
    }
}

// l1[b] = sum_k pf_k |beta_bk|
__global__ __launch_bounds__(kWave) void cov_l1_kernel(const double* __restrict__ beta, const double* __restrict__ pf,
                                                       int q, double* __restrict__ l1)
{
    const int b = blockIdx.x, k = threadIdx.x;
    double v = k < q ? pf[k] * fabs(beta[(int64_t)b * q + k]) : 0.0;
    v = wave_sum(v);
    if (k == 0) l1[b] = v;
}

// [B][p + q] FP32 <-> [B][p] and [B][q] FP64
__global__ void split_coef_kernel(const float* __restrict__ in, int64_t p, int64_t q, int B, double* __restrict__ x64,
                                  double* __restrict__ z64)
{
    const int64_t pt = p + q, m = pt * B;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < m; t += (int64_t)gridDim.x * kT) {
        const int64_t b = t / pt, j = t % pt;
        if (j < p)
            x64[b * p + j] = in[t];
        else
            z64[b * q + (j - p)] = in[t];
    }
}

__global__ void merge_coef_kernel(const double* __restrict__ x64, const double* __restrict__ z64, int64_t p,
                                  int64_t q, int B, float* __restrict__ out)
{
    const int64_t pt = p + q, m = pt * B;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < m; t += (int64_t)gridDim.x * kT) {
        const int64_t b = t / pt, j = t % pt;
        out[t] = (float)(j < p ? x64[b * p + j] : z64[b * q + (j - p)]);
    }
}

// acc[0] += sum_k v_k^2 (one wavefront)
__global__ __launch_bounds__(kWave) void sqnorm_add_kernel(const double* __restrict__ v, int q, double* __restrict__ acc)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < q; k += kWave) s += v[k] * v[k];
    s = wave_sum(s);
    if (threadIdx.x == 0) acc[0] += s;
}

}  // namespace

int cov_row_blocks(int64_t n) { return (int)((n + kCovRows - 1) / kCovRows); }

hipError_t launch_cov_xtr(const CovArgs& c, const float* r32, int64_t rstride, const double* r64, int B,
                          const int32_t* active, hipStream_t s)
{
    if (c.q < 1 || c.q > kMaxCov || c.nrb != cov_row_blocks(c.n) || (r32 == nullptr) == (r64 == nullptr) ||
        (r32 && rstride < c.n))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(cov_xtr_part_kernel, dim3(c.nrb, B), dim3(kT), 0, s, c, r32, rstride, r64, active);
    return hipGetLastError();
}

hipError_t launch_cov_epilogue(const CovArgs& c, const CovStep& st, int B, hipStream_t s)
{
    if (c.q < 1 || c.q > kMaxCov) return hipErrorInvalidValue;
    if (st.mode == GT_GRAD && (st.out32 == nullptr || st.ostride < c.q)) return hipErrorInvalidValue;
    if (st.out64 && st.ostride < c.q) return hipErrorInvalidValue;
    if (st.mode == GT_PROX && (!st.beta || !st.dbeta || !st.pf || !st.lam || !st.l1old || !st.l1new))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(cov_epilogue_kernel, dim3(B), dim3(kWave), 0, s, c, st);
    return hipGetLastError();
}

hipError_t launch_cov_eta(const CovArgs& c, const double* coef, int B, double* eta, const int32_t* active,
                          hipStream_t s)
{
    if (c.q < 1 || c.q > kMaxCov) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)min((int64_t)2048, (c.n + kT - 1) / kT);
    hipLaunchKernelGGL(cov_eta_kernel, dim3(gx, B), dim3(kT), 0, s, c, coef, eta, active);
    return hipGetLastError();
}

hipError_t launch_cov_l1(const double* beta, const double* pf, int q, int B, double* l1, hipStream_t s)
{
    if (q < 1 || q > kMaxCov) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cov_l1_kernel, dim3(B), dim3(kWave), 0, s, beta, pf, q, l1);
    return hipGetLastError();
}

hipError_t launch_split_coef(const float* in, int64_t p, int64_t q, int B, double* x64, double* z64, hipStream_t s)
{
    hipLaunchKernelGGL(split_coef_kernel, dim3(grid_for((p + q) * B)), dim3(kT), 0, s, in, p, q, B, x64, z64);
    return hipGetLastError();
}

hipError_t launch_merge_coef(const double* x64, const double* z64, int64_t p, int64_t q, int B, float* out,
                             hipStream_t s)
{
    hipLaunchKernelGGL(merge_coef_kernel, dim3(grid_for((p + q) * B)), dim3(kT), 0, s, x64, z64, p, q, B, out);
    return hipGetLastError();
}

hipError_t launch_sqnorm_add(const double* v, int q, double* acc, hipStream_t s)
{
    hipLaunchKernelGGL(sqnorm_add_kernel, dim3(1), dim3(kWave), 0, s, v, q, acc);
    return hipGetLastError();
}

}  // namespace cox
