// misc.hip -- small elementwise kernels and fixed-order reductions.
//
// prox_apply is the standalone fused elementwise step of Section 5.3,
// beta <- S_{sigma lambda pf_j}(beta - sigma grad), with S the soft-thresholding
// of Section 4.2 and pf_j the column's penalty factor; nll_backward is the adjoint of the negative log partial
// likelihood with respect to eta (-(I - P) delta scaled by the incoming
// gradient).  Reductions run in one workgroup in a fixed order, so results are
// reproducible bit for bit.
#include "device_common.h"

namespace cox {
namespace {

constexpr int kT = 256;

inline unsigned grid_for(int64_t m) { return (unsigned)min((int64_t)8192, max((int64_t)1, (m + kT - 1) / kT)); }

__global__ void f32_to_f64_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) out[i] = in[i];
}

__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT)
        out[i] = (float)in[i];
}

__global__ void scale_coef_kernel(const double* __restrict__ beta, const float* __restrict__ scale,
                                  double* __restrict__ coef, int64_t p, int B)
{
    const int64_t m = p * B;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT)
        coef[i] = scale ? beta[i] * (double)scale[i % p] : beta[i];
}

// l1[b][blk] = sum over the 16 columns of GEMV^T workgroup blk of pf_j |beta_bj|, in column order.
__global__ void l1_blocks_kernel(const double* __restrict__ beta, const double* __restrict__ pf, int64_t p, int B,
                                 int nblk, double* __restrict__ l1)
{
    const int64_t m = (int64_t)nblk * B;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < m; t += (int64_t)gridDim.x * kT) {
        const int64_t b = t / nblk, blk = t % nblk;
        double s = 0.0;
        for (int c = 0; c < kGemvtCols; ++c) {
            const int64_t j = blk * kGemvtCols + c;
            if (j < p) s += (pf ? pf[j] : 1.0) * fabs(beta[b * p + j]);
        }
        l1[t] = s;
    }
}

__global__ void prox_apply_kernel(float* __restrict__ beta, const float* __restrict__ grad,
                                  const double* __restrict__ lam, const double* __restrict__ pf, double step,
                                  int64_t p, int B)
{
    const int64_t m = p * B;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) {
        const double f = pf ? pf[i % p] : 1.0;
        const double t = f == 0.0 ? 0.0 : step * lam[i / p] * f;
        beta[i] = (float)soft_threshold((double)beta[i] - step * (double)grad[i], t);
    }
}

__global__ void nll_backward_kernel(const double* __restrict__ r, const double* __restrict__ gl, int64_t n, int B,
                                    void* __restrict__ out, int out_f64)
{
    const int64_t m = n * B;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) {
        const double v = -gl[i / n] * r[i];
        if (out_f64)
            static_cast<double*>(out)[i] = v;
        else
            static_cast<float*>(out)[i] = (float)v;
    }
}

__device__ double wg_sum(double v)
{
    __shared__ double sh[kT / kWave + 1];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < kT / kWave; ++q) s += sh[q];
        sh[kT / kWave] = s;
    }
    __syncthreads();
    return sh[kT / kWave];
}

// Reductions over a long vector in two fixed-order levels: the gridDim.x
// workgroups each sum one contiguous chunk into part[blockIdx.x], then one
// workgroup adds the parts in order (part_sum_kernel).  The chunks depend only
// on the length, so the result is the same on every run.
__device__ __forceinline__ void chunk_of(int64_t m, int64_t& i0, int64_t& i1)
{
    const int64_t chunk = (m + gridDim.x - 1) / gridDim.x;
    i0 = (int64_t)blockIdx.x * chunk;
    i1 = min(m, i0 + chunk);
}

__global__ void dot_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t m,
                           double* __restrict__ part)
{
    int64_t i0, i1;
    chunk_of(m, i0, i1);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kT) s += a[i] * (b ? b[i] : 1.0);
    s = wg_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = scale * (part[0] + ... + part[nparts - 1]), nparts <= kT
__global__ void part_sum_kernel(const double* __restrict__ part, int nparts, double scale, double* __restrict__ out)
{
    double s = threadIdx.x < nparts ? part[threadIdx.x] : 0.0;
    s = wg_sum(s);
    if (threadIdx.x == 0) out[0] = scale * s;
}

__global__ void center_shift_kernel(const float* __restrict__ center, const float* __restrict__ scale,
                                    const double* __restrict__ v, int64_t p, double* __restrict__ part)
{
    int64_t j0, j1;
    chunk_of(p, j0, j1);
    double s = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kT) s += (double)center[j] * (scale ? (double)scale[j] : 1.0) * v[j];
    s = wg_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void normalize_kernel(const double* __restrict__ in, const double* __restrict__ nrm2,
                                 const float* __restrict__ scale, double* __restrict__ vout,
                                 double* __restrict__ coef, int64_t p)
{
    const double inv = 1.0 / sqrt(nrm2[0]);
    for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < p; j += (int64_t)gridDim.x * kT) {
        const double v = in[j] * inv;
        vout[j] = v;
        coef[j] = scale ? v * (double)scale[j] : v;
    }
}

__global__ void to_r32_kernel(const double* __restrict__ u, const double* __restrict__ shift,
                              float* __restrict__ r32, int64_t n, double* __restrict__ part)
{
    int64_t i0, i1;
    chunk_of(n, i0, i1);
    const double sh = shift ? shift[0] : 0.0;
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kT) {
        const float f = (float)(u[i] + sh);
        r32[i] = f;
        s += (double)f;
    }
    s = wg_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The lambdas that stopped at max_iter (status 2) go on: active again, and the
// step counter past the step whose objective was recorded last.
__global__ void resume_kernel(int32_t* __restrict__ status, int32_t* __restrict__ active, int32_t* __restrict__ kit,
                              const int32_t* __restrict__ iters, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B && status[b] == 2) {
        status[b] = 0;
        active[b] = 1;
        kit[b] = iters[b] + 1;
    }
}

// acc[0] += v[0] (one thread): running count of the columns the eta updates read.
__global__ void count_add_kernel(const int32_t* __restrict__ v, long long* __restrict__ acc) { acc[0] += v[0]; }

__global__ void rowsum_kernel(const double* __restrict__ in, int64_t m, double a, double* __restrict__ out)
{
    const int64_t b = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kT) s += in[b * m + i];
    s = wg_sum(s);
    if (threadIdx.x == 0) out[b] = a * s;
}

__global__ void fill_f64_kernel(double* __restrict__ p, double v, int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) p[i] = v;
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int32_t v, int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) p[i] = v;
}

__global__ void iota_i32_kernel(int32_t* __restrict__ p, int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) p[i] = (int32_t)i;
}

// flag[b] = 1 when some coef[b][j], j < p, is not finite (the flags cleared by
// the caller); one workgroup row per b (blockIdx.y), every writer stores 1
__global__ void nonfinite_kernel(const double* __restrict__ coef, int64_t p, int32_t* __restrict__ flag)
{
    const int b = blockIdx.y;
    bool bad = false;
    for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < p; j += (int64_t)gridDim.x * kT)
        bad |= !isfinite(coef[(int64_t)b * p + j]);
    if (bad) flag[b] = 1;
}

// eta[b][i] = NaN for every i < n of each b whose flag is set
__global__ void poison_eta_kernel(double* __restrict__ eta, int64_t n, const int32_t* __restrict__ flag)
{
    const int b = blockIdx.y;
    if (!flag[b]) return;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        eta[(int64_t)b * n + i] = __builtin_nan("");
}

// dst[b][j] = src[b][j] - q_b R, R = llrint(src[b][j] / q_b): the integer the
// eta update's quantiser takes for that entry at the same scale q_b.  One fma,
// so the remainder carries at most one rounding of 2^-53 q_b.
__global__ void coef_remainder_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t p,
                                      int64_t m, const double* __restrict__ dscale)
{
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < m; k += (int64_t)gridDim.x * kT) {
        const double q = dscale[k / p], v = src[k];
        dst[k] = fma(-q, (double)llrint(v / q), v);
    }
}

}  // namespace

#define COX_LAUNCH(kernel, grid, ...)                                        \
    do {                                                                     \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kT), 0, s, __VA_ARGS__); \
        return hipGetLastError();                                            \
    } while (0)

hipError_t launch_f32_to_f64(const float* in, double* out, int64_t m, hipStream_t s)
{
    COX_LAUNCH(f32_to_f64_kernel, grid_for(m), in, out, m);
}
hipError_t launch_f64_to_f32(const double* in, float* out, int64_t m, hipStream_t s)
{
    COX_LAUNCH(f64_to_f32_kernel, grid_for(m), in, out, m);
}
hipError_t launch_scale_coef(const double* beta, const float* scale, double* coef, int64_t p, int B, hipStream_t s)
{
    COX_LAUNCH(scale_coef_kernel, grid_for(p * B), beta, scale, coef, p, B);
}
hipError_t launch_l1_blocks(const double* beta, const double* pf, int64_t p, int B, int nblk, double* l1,
                            hipStream_t s)
{
    COX_LAUNCH(l1_blocks_kernel, grid_for((int64_t)nblk * B), beta, pf, p, B, nblk, l1);
}
hipError_t launch_prox_apply(float* beta, const float* grad, const double* lam, const double* pf, double step,
                             int64_t p, int B, hipStream_t s)
{
    COX_LAUNCH(prox_apply_kernel, grid_for(p * B), beta, grad, lam, pf, step, p, B);
}
hipError_t launch_nll_backward(const double* r64, const double* gl, int64_t n, int B, void* out, int out_f64,
                               hipStream_t s)
{
    COX_LAUNCH(nll_backward_kernel, grid_for(n * B), r64, gl, n, B, out, out_f64);
}
// workgroups of a two-level reduction over m values: about 4,096 values each, at most kRedParts
static unsigned red_parts(int64_t m) { return (unsigned)min((int64_t)kRedParts, max((int64_t)1, (m + 4095) / 4096)); }

hipError_t launch_dot(const double* a, const double* b, int64_t m, double* part, double* out, hipStream_t s)
{
    const unsigned g = red_parts(m);
    hipLaunchKernelGGL(dot_kernel, dim3(g), dim3(kT), 0, s, a, b, m, part);
    COX_LAUNCH(part_sum_kernel, 1, part, (int)g, 1.0, out);
}
hipError_t launch_center_shift(const float* center, const float* scale, const double* v, int64_t p, double* part,
                               double* out, hipStream_t s)
{
    const unsigned g = red_parts(p);
    hipLaunchKernelGGL(center_shift_kernel, dim3(g), dim3(kT), 0, s, center, scale, v, p, part);
    COX_LAUNCH(part_sum_kernel, 1, part, (int)g, -1.0, out);
}
hipError_t launch_normalize(const double* in, const double* nrm2, const float* scale, double* vout, double* coef,
                            int64_t p, hipStream_t s)
{
    COX_LAUNCH(normalize_kernel, grid_for(p), in, nrm2, scale, vout, coef, p);
}
hipError_t launch_to_r32(const double* u, const double* shift, float* r32, double* sumr, int64_t n, double* part,
                         hipStream_t s)
{
    const unsigned g = red_parts(n);
    hipLaunchKernelGGL(to_r32_kernel, dim3(g), dim3(kT), 0, s, u, shift, r32, n, part);
    COX_LAUNCH(part_sum_kernel, 1, part, (int)g, 1.0, sumr);
}
hipError_t launch_resume(int32_t* status, int32_t* active, int32_t* kit, const int32_t* iters, int B,
                         hipStream_t s)
{
    hipLaunchKernelGGL(resume_kernel, dim3(1), dim3(64), 0, s, status, active, kit, iters, B);
    return hipGetLastError();
}

hipError_t launch_count_add(const int32_t* v, long long* acc, hipStream_t s)
{
    hipLaunchKernelGGL(count_add_kernel, dim3(1), dim3(1), 0, s, v, acc);
    return hipGetLastError();
}

hipError_t launch_rowsum(const double* in, int64_t m, int B, double a, double* out, hipStream_t s)
{
    COX_LAUNCH(rowsum_kernel, B, in, m, a, out);
}
hipError_t launch_fill_f64(double* p, double v, int64_t m, hipStream_t s)
{
    COX_LAUNCH(fill_f64_kernel, grid_for(m), p, v, m);
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t m, hipStream_t s)
{
    COX_LAUNCH(fill_i32_kernel, grid_for(m), p, v, m);
}
hipError_t launch_iota_i32(int32_t* p, int64_t m, hipStream_t s)
{
    COX_LAUNCH(iota_i32_kernel, grid_for(m), p, m);
}
hipError_t launch_nonfinite(const double* coef, int64_t p, int B, int32_t* flag, hipStream_t s)
{
    if (p < 1 || B < 1) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)min((int64_t)256, (p + kT - 1) / kT);
    hipLaunchKernelGGL(nonfinite_kernel, dim3(gx, (unsigned)B), dim3(kT), 0, s, coef, p, flag);
    return hipGetLastError();
}
hipError_t launch_poison_eta(double* eta, int64_t n, int B, const int32_t* flag, hipStream_t s)
{
    if (n < 1 || B < 1) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)min((int64_t)256, (n + kT - 1) / kT);
    hipLaunchKernelGGL(poison_eta_kernel, dim3(gx, (unsigned)B), dim3(kT), 0, s, eta, n, flag);
    return hipGetLastError();
}
hipError_t launch_coef_remainder(const double* src, double* dst, int64_t p, int B, const double* dscale,
                                 hipStream_t s)
{
    if (p < 1 || B < 1) return hipErrorInvalidValue;
    COX_LAUNCH(coef_remainder_kernel, grid_for((int64_t)B * p), src, dst, p, (int64_t)B * p, dscale);
}

}  // namespace cox
