// gemv.hip -- the linear predictor eta = X~ beta (Section 5.3: w = exp(x_i' beta)).
//
// Two forms:
//  * dense: every column of X is read once.  Workgroups tile rows (1024 per
//    workgroup, 4 consecutive rows per lane) and column blocks; the
//    coefficients of the block are staged in LDS 256 at a time.  Partial sums of
//    the column blocks are written out and reduced in a fixed order by a second
//    kernel, so the result does not depend on scheduling.
//  * update: eta += X~[:, S] dcoef_S for the set S of columns whose coefficient
//    changed in the last step (the proximal step keeps most coefficients at
//    zero, so S is small and only |S| columns are read).  Partial sums of a few
//    column groups go to a buffer that the risk-set kernel adds in fixed order;
//    eta itself is held in FP64 so that the running sum tracks X~ beta exactly
//    to rounding.
// Both take per-column coefficients already multiplied by the genotype scale
// s_j; the centring term is a constant shift of eta, to which the partial
// likelihood is invariant, and is applied only where an exact X~ v is needed.
#include <type_traits>

#include "gemv_dev.h"

namespace cox {
namespace {

using namespace gemvdev;

constexpr int kColStage = 256;

template <int XT, int NB, bool VEC>
__global__ __launch_bounds__(kT) void gemv_kernel(XDesc x, const double* __restrict__ coef, int b0, int nb,
                                                  int64_t cpb, double* __restrict__ part)
{
    __shared__ double sc[NB][kColStage];
    const int64_t n = x.n, p = x.p;
    const int64_t slab0 = (int64_t)blockIdx.x * kRows;
    const int64_t jbeg = (int64_t)blockIdx.y * cpb;
    const int64_t jend = min(p, jbeg + cpb);
    double acc[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[b][e] = 0.0;

    for (int64_t jc = jbeg; jc < jend; jc += kColStage) {
        __syncthreads();
        for (int t = threadIdx.x; t < NB * kColStage; t += kT) {
            const int b = t / kColStage, q = t % kColStage;
            sc[b][q] = (b < nb && jc + q < jend) ? coef[(int64_t)(b0 + b) * p + jc + q] : 0.0;
        }
        __syncthreads();
        const int jn = (int)min((int64_t)kColStage, jend - jc);
        const int64_t r0 = VEC ? slab0 + (int64_t)threadIdx.x * 4 : 0;
        for (int t = 0; t < jn; t += 8) {
            float xv[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (t + u < jn) {
                    if (VEC) {
                        load_rows4<XT, true>(x, jc + t + u, r0, n, xv[u]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int64_t r = row_of<false>(slab0, e);
                            xv[u][e] = r < n ? load_x1<XT>(x.X, (jc + t + u) * x.ldx + r) : 0.f;
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) xv[u][e] = 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const double cf = sc[b][t + u < kColStage ? t + u : 0];
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[b][e] = fma((double)xv[u][e], cf, acc[b][e]);
                }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = row_of<VEC>(slab0, e);
            if (r < n) part[((int64_t)blockIdx.y * nb + b) * n + r] = acc[b][e];
        }
    }
}

__global__ __launch_bounds__(256) void gemv_reduce_kernel(const double* __restrict__ part, int ncb, int nb, int64_t n,
                                                          int b0, const double* __restrict__ shift,
                                                          double* __restrict__ eta)
{
    const int b = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int c = 0; c < ncb; ++c) s += part[((int64_t)c * nb + b) * n + i];
        if (shift) s += shift[b0 + b];
        eta[(int64_t)(b0 + b) * n + i] = s;
    }
}

// Dense X~ coef for one-byte X whose 16-byte runs are aligned (base and ldx
// multiples of 16): a workgroup owns 256 RPL rows (RPL = 16 or 8 per lane, so a
// wavefront reads 1 KB or 512 bytes of a column per load) and a block of
// columns, which every wavefront walks in order with kPre columns of loads in
// flight.  The coefficient of a column is the same for the whole wavefront and
// is read through the scalar cache.  Products and sums are FP64 as in
// gemv_kernel (exact products of the small counts), and partial sums of the
// column blocks are reduced in a fixed order by gemv_reduce_kernel.  RPL = 8
// serves 5..8 vectors in one pass (their 64 sums per lane fit in registers).
constexpr int kPre = 8;  // columns of loads in flight per wavefront

template <int RPL>
constexpr int rows_wg() { return RPL * kT; }

template <int XT, int NB, int RPL>
__global__ __launch_bounds__(kT) void gemv16_kernel(XDesc x, const double* __restrict__ coef, int b0, int nb,
                                                    int64_t cpb, double* __restrict__ part)
{
    static_assert(RPL == 16 || RPL == 8, "16 or 8 rows per lane");
    using run = typename std::conditional<RPL == 16, uint4, uint2>::type;
    const int64_t n = x.n, p = x.p, ldx = x.ldx;
    const int64_t r0 = (int64_t)blockIdx.x * rows_wg<RPL>() + RPL * (int64_t)threadIdx.x;
    const bool live = r0 < n;  // r0 + RPL - 1 < ldx: the run stays inside the column's allocation
    const int64_t jbeg = (int64_t)blockIdx.y * cpb;
    const int64_t jend = min(p, jbeg + cpb);
    const uint8_t* __restrict__ X = static_cast<const uint8_t*>(x.X);
    double acc[NB][RPL];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < RPL; ++e) acc[b][e] = 0.0;
    run ring[kPre];
    auto fetch = [&](int64_t j) -> run {  // X is read once per pass: streaming loads
        if (!(live && j < jend)) return run{};
        if constexpr (RPL == 16)
            return load_u4_stream(X + j * ldx + r0);
        else
            return load_u2_stream(X + j * ldx + r0);
    };
#pragma unroll
    for (int u = 0; u < kPre; ++u) ring[u] = fetch(jbeg + u);
    for (int64_t j0 = jbeg; j0 < jend; j0 += kPre) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int64_t j = j0 + u;
            const run w = ring[u];
            ring[u] = fetch(j + kPre);
            if (j >= jend) break;
            float xf[RPL];
            decode4<XT>(w.x, &xf[0]);
            decode4<XT>(w.y, &xf[4]);
            if constexpr (RPL == 16) {
                decode4<XT>(w.z, &xf[8]);
                decode4<XT>(w.w, &xf[12]);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b >= nb) break;
                const double cf = coef[(int64_t)(b0 + b) * p + j];
#pragma unroll
                for (int e = 0; e < RPL; ++e) acc[b][e] = fma((double)xf[e], cf, acc[b][e]);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;
        double* out = part + ((int64_t)blockIdx.y * nb + b) * n + r0;
#pragma unroll
        for (int e = 0; e < RPL; ++e)
            if (r0 + e < n) out[e] = acc[b][e];
    }
}

template <int XT, int NB, bool VEC>
__global__ __launch_bounds__(kT) void eta_update_kernel(XDesc x, const int32_t* __restrict__ sel,
                                                        const int32_t* __restrict__ nsel_p,
                                                        const double* __restrict__ dcoef, int b0, int nb,
                                                        double* __restrict__ part, int64_t cstride, int ncg,
                                                        const int32_t* __restrict__ active)
{
    eta_update_blk<XT, NB, VEC>(x, sel, nsel_p, dcoef, b0, nb, part, cstride, ncg, active, blockIdx.x, blockIdx.y);
}

// One workgroup per chunk of 1024 blocks of columns.  Each adds up the counts
// of the blocks before its chunk itself (a few thousand integers at most), so
// the chunks are compacted in parallel into one ascending list.
__global__ __launch_bounds__(1024) void compact_kernel(const int32_t* __restrict__ cnt,
                                                       const int32_t* __restrict__ idx, int nblk,
                                                       int32_t* __restrict__ sel, int32_t* __restrict__ nsel)
{
    constexpr int NT = 1024;
    __shared__ int sh[17];
    __shared__ int sstart[NT], scnt[NT];
    const int b0 = blockIdx.x * NT;
    int pre = 0;
    for (int k = threadIdx.x; k < b0; k += NT) pre += cnt[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = pre;
    __syncthreads();
    int carry = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) carry += sh[w];
    __syncthreads();  // the scan below reuses sh
    compact_blk<NT>(cnt, idx, nblk, sel, nsel, sh, sstart, scnt, b0, b0 + NT, carry);
}

template <int XT, int NB>
hipError_t gemv_t(const XDesc& x, const double* coef, int b0, int nb, double* part, int ncb, hipStream_t s)
{
    const int64_t cpb = (x.p + ncb - 1) / ncb;
    const dim3 grid((unsigned)((x.n + kRows - 1) / kRows), (unsigned)ncb);
    const bool vec = x.xt == XT_F32 ? x.vec16 : x.vec4;
    if (vec)
        hipLaunchKernelGGL((gemv_kernel<XT, NB, true>), grid, dim3(kT), 0, s, x, coef, b0, nb, cpb, part);
    else
        hipLaunchKernelGGL((gemv_kernel<XT, NB, false>), grid, dim3(kT), 0, s, x, coef, b0, nb, cpb, part);
    return hipGetLastError();
}

template <int XT, int NB, int RPL>
hipError_t gemv16_t(const XDesc& x, const double* coef, int b0, int nb, double* part, int ncb, hipStream_t s)
{
    const int64_t cpb = (x.p + ncb - 1) / ncb;
    const dim3 grid((unsigned)((x.n + rows_wg<RPL>() - 1) / rows_wg<RPL>()), (unsigned)ncb);
    hipLaunchKernelGGL((gemv16_kernel<XT, NB, RPL>), grid, dim3(kT), 0, s, x, coef, b0, nb, cpb, part);
    return hipGetLastError();
}

template <int XT>
hipError_t gemv_x(const XDesc& x, const double* coef, int b0, int nb, double* part, int ncb, hipStream_t s)
{
    if (nb <= 1) return gemv_t<XT, 1>(x, coef, b0, nb, part, ncb, s);
    if (nb <= 2) return gemv_t<XT, 2>(x, coef, b0, nb, part, ncb, s);
    if (nb <= 4) return gemv_t<XT, 4>(x, coef, b0, nb, part, ncb, s);
    return gemv_t<XT, 8>(x, coef, b0, nb, part, ncb, s);
}

template <int XT, int NB>
hipError_t upd_t(const XDesc& x, const int32_t* sel, const int32_t* nsel, const double* dcoef, int b0, int nb,
                 double* part, int64_t cstride, int ncg, const int32_t* active, hipStream_t s)
{
    const dim3 grid((unsigned)((x.n + kRows - 1) / kRows), (unsigned)ncg);
    const bool vec = x.xt == XT_F32 ? x.vec16 : x.vec4;
    if (vec)
        hipLaunchKernelGGL((eta_update_kernel<XT, NB, true>), grid, dim3(kT), 0, s, x, sel, nsel, dcoef, b0, nb,
                           part, cstride, ncg, active);
    else
        hipLaunchKernelGGL((eta_update_kernel<XT, NB, false>), grid, dim3(kT), 0, s, x, sel, nsel, dcoef, b0, nb,
                           part, cstride, ncg, active);
    return hipGetLastError();
}

template <int XT>
hipError_t upd_x(const XDesc& x, const int32_t* sel, const int32_t* nsel, const double* dcoef, int b0, int nb,
                 double* part, int64_t cstride, int ncg, const int32_t* active, hipStream_t s)
{
    if (nb <= 1) return upd_t<XT, 1>(x, sel, nsel, dcoef, b0, nb, part, cstride, ncg, active, s);
    if (nb <= 2) return upd_t<XT, 2>(x, sel, nsel, dcoef, b0, nb, part, cstride, ncg, active, s);
    if (nb <= 4) return upd_t<XT, 4>(x, sel, nsel, dcoef, b0, nb, part, cstride, ncg, active, s);
    return upd_t<XT, 8>(x, sel, nsel, dcoef, b0, nb, part, cstride, ncg, active, s);
}

}  // namespace

int gemv16_blocks(int64_t n, int64_t p)
{
    const int64_t slabs = (n + rows_wg<16>() - 1) / rows_wg<16>();
    return (int)max((int64_t)1, min((2048 + slabs - 1) / slabs, (p + 63) / 64));
}

hipError_t launch_gemv(const XDesc& x, const double* coef, int b0, int nb, double* part, int ncb, double* eta,
                       const double* shift, hipStream_t s)
{
    if (nb < 1 || nb > 8 || ncb < 1) return hipErrorInvalidValue;
    hipError_t e;
    if (x.xt != XT_F32 && x.vec16) {
        // up to 4 vectors: 16 rows per lane; 5..8: 8 rows per lane (their 64
        // sums per lane fit in registers), twice the workgroups over the rows,
        // so the partial buffer's size is the same.  At 400,000 x 500,000 a pass
        // for 8 vectors takes 117 ms this way (FP64 products bound it) against
        // 189 ms in the 4-row kernel
        ncb = gemv16_blocks(x.n, x.p);
        if (nb > 4) ncb = max(1, ncb / 2);
        auto run = [&](auto xt) {
            constexpr int XT = decltype(xt)::value;
            if (nb == 1) return gemv16_t<XT, 1, 16>(x, coef, b0, nb, part, ncb, s);
            if (nb == 2) return gemv16_t<XT, 2, 16>(x, coef, b0, nb, part, ncb, s);
            if (nb <= 4) return gemv16_t<XT, 4, 16>(x, coef, b0, nb, part, ncb, s);
            return gemv16_t<XT, 8, 8>(x, coef, b0, nb, part, ncb, s);
        };
        e = x.xt == XT_FP8 ? run(std::integral_constant<int, XT_FP8>{}) : run(std::integral_constant<int, XT_I8>{});
    } else {
        switch (x.xt) {
        case XT_F32: e = gemv_x<XT_F32>(x, coef, b0, nb, part, ncb, s); break;
        case XT_FP8: e = gemv_x<XT_FP8>(x, coef, b0, nb, part, ncb, s); break;
        default: e = gemv_x<XT_I8>(x, coef, b0, nb, part, ncb, s); break;
        }
    }
    if (e != hipSuccess) return e;
    const unsigned gx = (unsigned)min((int64_t)1024, (x.n + 255) / 256);
    hipLaunchKernelGGL(gemv_reduce_kernel, dim3(gx, nb), dim3(256), 0, s, part, ncb, nb, x.n, b0, shift, eta);
    return hipGetLastError();
}

hipError_t launch_eta_update(const XDesc& x, const int32_t* sel, const int32_t* nsel, const double* dcoef, int b0,
                             int nb, double* part, int64_t part_cstride, int ncg, const int32_t* active,
                             hipStream_t s)
{
    if (nb < 1 || nb > 8 || ncg < 1) return hipErrorInvalidValue;
    switch (x.xt) {
    case XT_F32: return upd_x<XT_F32>(x, sel, nsel, dcoef, b0, nb, part, part_cstride, ncg, active, s);
    case XT_FP8: return upd_x<XT_FP8>(x, sel, nsel, dcoef, b0, nb, part, part_cstride, ncg, active, s);
    default: return upd_x<XT_I8>(x, sel, nsel, dcoef, b0, nb, part, part_cstride, ncg, active, s);
    }
}

hipError_t launch_compact(const int32_t* chg_cnt, const int32_t* chg_idx, int nblk, int32_t* sel, int32_t* nsel,
                          hipStream_t s)
{
    if (nblk < 0) return hipErrorInvalidValue;
    const int nchunk = nblk > 0 ? (nblk + 1023) / 1024 : 1;
    hipLaunchKernelGGL(compact_kernel, dim3((unsigned)nchunk), dim3(1024), 0, s, chg_cnt,
                       chg_idx, nblk, sel, nsel);
    return hipGetLastError();
}

}  // namespace cox
