// gemvt.hip -- g = X~' r for a group of NB residual vectors, with the
// proximal step fused into the epilogue (Section 5.3: Delta = X'(I - P) delta,
// beta <- S_{sigma lambda}(beta + sigma Delta)).
//
// Layout: X column-major, so column j (one SNP over all subjects) is one
// contiguous run.  A workgroup of 4 wavefronts owns 16 consecutive columns, 4 per
// wavefront.  Rows are walked in chunks whose slice of r (for all NB vectors) is
// staged in LDS (32 KB); within a chunk each lane streams 16-byte loads down its
// wavefront's 4 columns (4 FP32 rows or 16 one-byte rows per load), so every
// wavefront load instruction reads 1 KB contiguous per column.  Each r value read
// from LDS serves all 4 columns.  At the end each column's 64 lane partials are
// combined by a shuffle tree.
//
// Arithmetic: FP32 X is multiplied in FP64 (exact products, FP64 sums).  One-
// byte X (allele counts) is decoded to FP32 and accumulated in FP32 within a
// chunk, chunks summed in FP64.  Genotype columns are standardised on the fly:
// g_j = s_j (sum_i g_ij r_i - mu_j sum_i r_i).
//
// Epilogue modes: RAW (write g, FP64), GRAD (write -g, FP32: the gradient of
// -L), PROX (the soft-threshold step on the FP64 iterate, with the list of
// columns whose coefficient changed and partial sums of |beta| before and
// after, for the next eta update and the objective).
#include "device_common.h"

namespace cox {
namespace {

constexpr int kCPW = kGemvtColsPerWave;
constexpr int kU = 2;  // row steps in flight per column

template <int XT>
struct RowsPerLoad {
    static constexpr int value = XT == XT_F32 ? 4 : 16;
};

template <int NB>
struct Chunk {
    static constexpr int value = 8192 / NB;  // NB * value floats = 32 KB of LDS
};

// LDS position of chunk row `row` (a multiple of 4): FP32 X reads r in natural
// order; one-byte X reads 16 consecutive rows per lane, so rows are swizzled to
// make each of the lane's four 16-byte LDS reads contiguous across lanes.
template <int XT, bool VEC>
__device__ __forceinline__ int lds_pos(int row)
{
    if constexpr (XT == XT_F32 || !VEC) {
        return row;
    } else {
        const int blk = row >> 10, within = row & 1023;
        const int lane = within >> 4, q = (within >> 2) & 3;
        return (blk << 10) | (q << 8) | (lane << 2);
    }
}

template <int XT, int NB, bool VEC>
__global__ __launch_bounds__(kGemvtThreads) void gemvt_kernel(GemvtArgs a)
{
    constexpr int RPL = RowsPerLoad<XT>::value;
    constexpr int WROWS = kWave * RPL;
    constexpr int RC = Chunk<NB>::value;
    static_assert(RC % 1024 == 0, "chunk must hold whole wave steps");
    __shared__ __attribute__((aligned(16))) float sr[NB * RC];
    __shared__ int s_flag[kGemvtCols];
    __shared__ double s_l1o[NB][kGemvtCols];
    __shared__ double s_l1n[NB][kGemvtCols];

    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int64_t blk = blockIdx.x;
    const int64_t n = a.x.n, p = a.x.p, ldx = a.x.ldx;
    const int64_t j0 = blk * kGemvtCols + (int64_t)wid * kCPW;
    const int ncols = (int)max((int64_t)0, min((int64_t)kCPW, p - j0));
    const int64_t nvec = VEC ? (n / RPL) * RPL : 0;

    double acc[kCPW][NB];
#pragma unroll
    for (int c = 0; c < kCPW; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[c][b] = 0.0;

    for (int64_t c0 = 0; c0 < n; c0 += RC) {
        __syncthreads();  // the previous chunk is consumed
        for (int t = threadIdx.x; t < NB * (RC / 4); t += kGemvtThreads) {
            const int b = t / (RC / 4);
            const int row = (t % (RC / 4)) * 4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (b < a.nb) v = load_f4(a.r32 + (int64_t)(a.b0 + b) * a.rstride + c0 + row);
            *reinterpret_cast<float4*>(&sr[b * RC + lds_pos<XT, VEC>(row)]) = v;
        }
        __syncthreads();
        if (ncols == 0) continue;

        if constexpr (VEC) {
            const int64_t v1 = min(c0 + RC, nvec);
            float accf[kCPW][NB];
#pragma unroll
            for (int c = 0; c < kCPW; ++c)
#pragma unroll
                for (int b = 0; b < NB; ++b) accf[c][b] = 0.f;
            for (int64_t rs = c0; rs < v1; rs += (int64_t)WROWS * kU) {
                uint4 xv[kCPW][kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int64_t row = rs + (int64_t)u * WROWS + (int64_t)lane * RPL;
#pragma unroll
                    for (int c = 0; c < kCPW; ++c) {
                        if (c < ncols && row < v1) {
                            const int64_t off = (j0 + c) * ldx + row;
                            xv[c][u] = XT == XT_F32 ? load_u4(static_cast<const float*>(a.x.X) + off)
                                                    : load_u4(static_cast<const uint8_t*>(a.x.X) + off);
                        } else {
                            xv[c][u] = make_uint4(0, 0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int64_t wrow = rs + (int64_t)u * WROWS;  // first row of the wave step
                    if (wrow >= v1) break;
                    const int lrow = (int)(wrow - c0);
                    if constexpr (XT == XT_F32) {
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            const float4 r4 = *reinterpret_cast<const float4*>(&sr[b * RC + lrow + lane * 4]);
                            const double r0 = r4.x, r1 = r4.y, r2 = r4.z, r3 = r4.w;
#pragma unroll
                            for (int c = 0; c < kCPW; ++c) {
                                const float4 x4 = __builtin_bit_cast(float4, xv[c][u]);
                                double s = acc[c][b];
                                s = fma((double)x4.x, r0, s);
                                s = fma((double)x4.y, r1, s);
                                s = fma((double)x4.z, r2, s);
                                s = fma((double)x4.w, r3, s);
                                acc[c][b] = s;
                            }
                        }
                    } else {
                        float xf[kCPW][16];
#pragma unroll
                        for (int c = 0; c < kCPW; ++c) {
                            decode4<XT>(xv[c][u].x, &xf[c][0]);
                            decode4<XT>(xv[c][u].y, &xf[c][4]);
                            decode4<XT>(xv[c][u].z, &xf[c][8]);
                            decode4<XT>(xv[c][u].w, &xf[c][12]);
                        }
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            float r16[16];
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const float4 r4 =
                                    *reinterpret_cast<const float4*>(&sr[b * RC + lrow + q * 256 + lane * 4]);
                                r16[4 * q + 0] = r4.x;
                                r16[4 * q + 1] = r4.y;
                                r16[4 * q + 2] = r4.z;
                                r16[4 * q + 3] = r4.w;
                            }
#pragma unroll
                            for (int c = 0; c < kCPW; ++c) {
                                float s = accf[c][b];
#pragma unroll
                                for (int e = 0; e < 16; ++e) s = fmaf(xf[c][e], r16[e], s);
                                accf[c][b] = s;
                            }
                        }
                    }
                }
            }
            if constexpr (XT != XT_F32) {
#pragma unroll
                for (int c = 0; c < kCPW; ++c)
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[c][b] += (double)accf[c][b];
            }
        } else {
            // Any alignment: one element per lane per row step, 64 rows per wavefront step.
            const int64_t c1 = min(c0 + RC, n);
            for (int64_t row = c0 + lane; row < c1; row += kWave) {
                const int lrow = (int)(row - c0);
#pragma unroll
                for (int c = 0; c < kCPW; ++c) {
                    if (c >= ncols) break;
                    const double xval = (double)load_x1<XT>(a.x.X, (j0 + c) * ldx + row);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[c][b] = fma(xval, (double)sr[b * RC + lrow], acc[c][b]);
                }
            }
        }
    }

    // Rows beyond the last whole 16-byte load (fewer than RPL of them).
    if (VEC && ncols > 0 && nvec + lane < n) {
        const int64_t row = nvec + lane;
#pragma unroll
        for (int c = 0; c < kCPW; ++c) {
            if (c >= ncols) break;
            const double xval = (double)load_x1<XT>(a.x.X, (j0 + c) * ldx + row);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < a.nb)
                    acc[c][b] = fma(xval, (double)a.r32[(int64_t)(a.b0 + b) * a.rstride + row], acc[c][b]);
        }
    }

#pragma unroll
    for (int c = 0; c < kCPW; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[c][b] = wave_sum(acc[c][b]);

    const bool geno = XT != XT_F32;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < kCPW; ++c) {
            const int cw = wid * kCPW + c;  // column within the workgroup
            const int64_t j = j0 + c;
            int changed = 0;
            const bool valid = c < ncols;
            double mu = 0.0, sc = 1.0;
            if (valid && geno) {
                if (a.x.center) mu = a.x.center[j];
                if (a.x.scale) sc = a.x.scale[j];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                double l1o = 0.0, l1n = 0.0;
                if (valid && b < a.nb) {
                    const int bb = a.b0 + b;
                    double g = acc[c][b];
                    if (geno) g = sc * (g - mu * a.sumr[bb]);
                    const int64_t at = (int64_t)bb * p + j;
                    if (a.mode == GT_RAW) {
                        a.out64[at] = g;
                    } else if (a.mode == GT_GRAD) {
                        a.out32[at] = (float)(-g);
                    } else {
                        const double old = a.beta[at];
                        double nw = old;
                        if (a.active == nullptr || a.active[bb]) nw = soft_threshold(old + a.step * g, a.step * a.lam[bb]);
                        a.beta[at] = nw;
                        const double d = nw - old;
                        a.dcoef[at] = d * (geno ? sc : 1.0);
                        changed |= d != 0.0;
                        l1o = fabs(old);
                        l1n = fabs(nw);
                    }
                }
                s_l1o[b][cw] = l1o;
                s_l1n[b][cw] = l1n;
            }
            s_flag[cw] = changed;
        }
    }
    if (a.mode != GT_PROX) return;  // uniform
    __syncthreads();
    if (threadIdx.x == 0) {
        int cnt = 0;
        for (int cw = 0; cw < kGemvtCols; ++cw) {
            const int64_t j = blk * kGemvtCols + cw;
            if (j >= p) break;
            const int f = a.first_group ? s_flag[cw] : (a.chg_flag[j] | s_flag[cw]);
            a.chg_flag[j] = f;
            if (f) a.chg_idx[blk * kGemvtCols + cnt++] = (int32_t)j;
        }
        a.chg_cnt[blk] = cnt;
    }
    if (threadIdx.x < NB && (int)threadIdx.x < a.nb) {
        const int b = threadIdx.x;
        double so = 0.0, sn = 0.0;
        for (int cw = 0; cw < kGemvtCols; ++cw) {
            so += s_l1o[b][cw];
            sn += s_l1n[b][cw];
        }
        a.l1old[(int64_t)(a.b0 + b) * a.nblk + blk] = so;
        a.l1new[(int64_t)(a.b0 + b) * a.nblk + blk] = sn;
    }
}

template <int XT, int NB>
hipError_t launch_t(const GemvtArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.x.p + kGemvtCols - 1) / kGemvtCols));
    if (a.x.vec16)
        hipLaunchKernelGGL((gemvt_kernel<XT, NB, true>), grid, dim3(kGemvtThreads), 0, s, a);
    else
        hipLaunchKernelGGL((gemvt_kernel<XT, NB, false>), grid, dim3(kGemvtThreads), 0, s, a);
    return hipGetLastError();
}

template <int XT>
hipError_t launch_x(const GemvtArgs& a, hipStream_t s)
{
    if (a.nb <= 1) return launch_t<XT, 1>(a, s);
    if (a.nb <= 2) return launch_t<XT, 2>(a, s);
    if (a.nb <= 4) return launch_t<XT, 4>(a, s);
    return launch_t<XT, 8>(a, s);
}

}  // namespace

hipError_t launch_gemvt(const GemvtArgs& a, hipStream_t s)
{
    if (a.nb < 1 || a.nb > 8) return hipErrorInvalidValue;
    switch (a.x.xt) {
    case XT_F32: return launch_x<XT_F32>(a, s);
    case XT_FP8: return launch_x<XT_FP8>(a, s);
    default: return launch_x<XT_I8>(a, s);
    }
}

}  // namespace cox
