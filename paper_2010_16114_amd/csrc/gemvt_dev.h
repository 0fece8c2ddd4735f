// gemvt_dev.h -- g = X~' r for a group of NB residual vectors, with the
// proximal step in the epilogue (Section 5.3: Delta = X'(I - P) delta,
// beta <- S_{sigma lambda}(beta + sigma Delta)).
//
// Two phases, as per-workgroup device functions shared by the launches of
// gemvt.hip and the persistent path (persist.hip).
//
// 1. Column sums.  X is column-major, so column j (one SNP over all subjects) is
//    one contiguous run.  A workgroup of 4 wavefronts owns 16 (FP32) or 64
//    (one-byte) consecutive columns and one split of the rows; rows are walked
//    in chunks whose slice of r (all NB vectors, 32 KB) is staged in LDS.  Each
//    lane streams 16-byte loads down its wavefront's columns, four columns at a
//    time (4 FP32 or 16 one-byte rows per load, so one wavefront load reads
//    1 KB contiguous per column), and every r value read from LDS serves four
//    columns.  The 64 lane partials of a column are combined by a shuffle tree
//    and written for the split.  Splitting rows gives enough workgroups to fill
//    the chip evenly.
// 2. Epilogue, one thread per column: the split partials are added in a fixed
//    order, genotype columns are standardised, g_j = s_j (sum_i g_ij r_i -
//    mu_j sum_i r_i), and the mode's output is written: RAW (g, FP64), GRAD
//    (-g, FP32: the gradient of -L) or PROX (the soft-threshold step on the FP64
//    iterate with threshold sigma lambda pf_j, pf_j the column's penalty factor,
//    the list of columns whose coefficient changed and partial sums of
//    pf_j |beta_j| before and after, for the next eta update and the objective).
//
// Arithmetic: FP32 X is multiplied in FP64 (exact products, FP64 sums).  One-
// byte X (allele counts) is decoded to FP32 and accumulated in FP32 within an
// LDS chunk; chunks and splits are summed in FP64.
#pragma once
#include "device_common.h"

namespace cox {
namespace gemvtdev {

constexpr int kU = 2;  // row steps in flight per column

template <int XT>
constexpr int rows_per_load() { return XT == XT_F32 ? 4 : 16; }

template <int XT, int NB>
constexpr int cols_per_wave() { return XT == XT_F32 ? 4 : (NB == 1 ? 16 : (NB == 2 ? 8 : 4)); }

template <int NB>
constexpr int chunk_rows() { return 8192 / NB; }  // NB * rows floats = 32 KB of LDS

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

// One workgroup of the column sums: column block bx, row split by.  sr: LDS
// of NB * chunk_rows<NB>() floats (32 KB), 16-byte aligned.
template <int XT, int NB, bool VEC>
__device__ __forceinline__ void gemvt_sums_blk(const GemvtArgs& a, int bx, int by, float* __restrict__ sr)
{
    constexpr int RPL = rows_per_load<XT>();
    constexpr int WROWS = kWave * RPL;
    constexpr int RC = chunk_rows<NB>();
    constexpr int CPW = cols_per_wave<XT, NB>();
    static_assert(RC % 1024 == 0 && kSplitRows % RC == 0, "chunk must hold whole wave steps");

    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int64_t n = a.x.n, p = a.x.p, ldx = a.x.ldx;
    const int64_t j0 = ((int64_t)bx * 4 + wid) * CPW;
    const int ncols = (int)max((int64_t)0, min((int64_t)CPW, p - j0));
    const int64_t nvec = VEC ? (n / RPL) * RPL : 0;
    const int64_t s0 = (int64_t)by * a.split_rows;
    const int64_t s1 = min(n, s0 + a.split_rows);

    double acc[CPW][NB];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[c][b] = 0.0;

    for (int64_t c0 = s0; c0 < s1; c0 += RC) {
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
            const int64_t v1 = min(min(c0 + RC, s1), nvec);
            float accf[CPW][NB];
#pragma unroll
            for (int c = 0; c < CPW; ++c)
#pragma unroll
                for (int b = 0; b < NB; ++b) accf[c][b] = 0.f;
            for (int64_t rs = c0; rs < v1; rs += (int64_t)WROWS * kU) {
#pragma unroll
                for (int cg = 0; cg < CPW; cg += 4) {
                    uint4 xv[4][kU];
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const int64_t row = rs + (int64_t)u * WROWS + (int64_t)lane * RPL;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (cg + c < ncols && row < v1) {
                                const int64_t off = (j0 + cg + c) * ldx + row;
                                xv[c][u] = XT == XT_F32 ? load_u4_stream(static_cast<const float*>(a.x.X) + off)
                                                        : load_u4_stream(static_cast<const uint8_t*>(a.x.X) + off);
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
                                for (int c = 0; c < 4; ++c) {
                                    const float4 x4 = __builtin_bit_cast(float4, xv[c][u]);
                                    double s = acc[cg + c][b];
                                    s = fma((double)x4.x, r0, s);
                                    s = fma((double)x4.y, r1, s);
                                    s = fma((double)x4.z, r2, s);
                                    s = fma((double)x4.w, r3, s);
                                    acc[cg + c][b] = s;
                                }
                            }
                        } else {
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
                                for (int c = 0; c < 4; ++c) {
                                    float xf[16];
                                    decode4<XT>(xv[c][u].x, &xf[0]);
                                    decode4<XT>(xv[c][u].y, &xf[4]);
                                    decode4<XT>(xv[c][u].z, &xf[8]);
                                    decode4<XT>(xv[c][u].w, &xf[12]);
                                    float s = accf[cg + c][b];
#pragma unroll
                                    for (int e = 0; e < 16; ++e) s = fmaf(xf[e], r16[e], s);
                                    accf[cg + c][b] = s;
                                }
                            }
                        }
                    }
                }
            }
            if constexpr (XT != XT_F32) {
#pragma unroll
                for (int c = 0; c < CPW; ++c)
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[c][b] += (double)accf[c][b];
            }
        } else {
            // Any alignment: one element per lane per row step, 64 rows per wavefront step.
            const int64_t c1 = min(c0 + RC, s1);
            for (int64_t row = c0 + lane; row < c1; row += kWave) {
                const int lrow = (int)(row - c0);
#pragma unroll
                for (int c = 0; c < CPW; ++c) {
                    if (c >= ncols) break;
                    const double xval = (double)load_x1<XT>(a.x.X, (j0 + c) * ldx + row);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[c][b] = fma(xval, (double)sr[b * RC + lrow], acc[c][b]);
                }
            }
        }
    }

    // Rows beyond the last whole 16-byte load (fewer than RPL of them), in the last split.
    if (VEC && ncols > 0 && nvec + lane < s1 && nvec + lane >= s0) {
        const int64_t row = nvec + lane;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            if (c >= ncols) break;
            const double xval = (double)load_x1<XT>(a.x.X, (j0 + c) * ldx + row);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < a.nb)
                    acc[c][b] = fma(xval, (double)a.r32[(int64_t)(a.b0 + b) * a.rstride + row], acc[c][b]);
        }
    }

#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[c][b] = wave_sum(acc[c][b]);

    if (lane == 0) {
        double* out = a.part + (int64_t)by * a.part_sstride;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            if (c >= ncols) break;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < a.nb) out[(int64_t)(a.b0 + b) * p + j0 + c] = acc[c][b];
        }
    }
}

// One workgroup of 256 threads of the epilogue, columns 256 bx ..: one thread
// per column; a 16-lane group covers one change-list block.
__device__ __forceinline__ void gemvt_epilogue_blk(const GemvtArgs& a, int bx)
{
    const int64_t p = a.x.p;
    const int64_t j = (int64_t)bx * 256 + threadIdx.x;
    const bool valid = j < p;
    const bool geno = a.x.xt != XT_F32;
    double mu = 0.0, sc = 1.0;
    if (valid && geno) {
        if (a.x.center) mu = a.x.center[j];
        if (a.x.scale) sc = a.x.scale[j];
    }
    int changed = 0;
    const int lane16 = threadIdx.x & 15;
    const int64_t blk = j / kGemvtCols;
    for (int b = 0; b < a.nb; ++b) {
        const int bb = a.b0 + b;
        const int64_t at = (int64_t)bb * p + j;
        double l1o = 0.0, l1n = 0.0;
        if (valid) {
            double g = 0.0;
            for (int s = 0; s < a.nsplit; ++s) g += a.part[(int64_t)s * a.part_sstride + at];
            if (geno) g = sc * (g - mu * a.sumr[bb]);
            if (a.mode == GT_RAW) {
                a.out64[(int64_t)bb * a.ostride + j] = g;
            } else if (a.mode == GT_GRAD) {
                a.out32[(int64_t)bb * a.ostride + j] = (float)(-g);
            } else {
                const double f = a.pf ? a.pf[j] : 1.0;  // penalty factor: 0 leaves the column unpenalised
                const double old = a.beta[at];
                double nw = old;
                if (a.active == nullptr || a.active[bb])
                    nw = soft_threshold(old + a.step * g, f == 0.0 ? 0.0 : a.step * a.lam[bb] * f);
                a.beta[at] = nw;
                const double d = nw - old;
                a.dcoef[at] = d * (geno ? sc : 1.0);
                changed |= d != 0.0;
                l1o = f * fabs(old);
                l1n = f * fabs(nw);
            }
        }
        if (a.mode == GT_PROX) {
            // sum over the 16 columns of the block, in a fixed tree order
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                l1o += __shfl_xor(l1o, o, 16);
                l1n += __shfl_xor(l1n, o, 16);
            }
            if (lane16 == 0 && (blk * kGemvtCols) < p) {
                a.l1old[(int64_t)bb * a.nblk + blk] = l1o;
                a.l1new[(int64_t)bb * a.nblk + blk] = l1n;
            }
        }
    }
    if (a.mode != GT_PROX) return;
    int f = 0;
    if (valid) {
        f = a.first_group ? changed : (a.chg_flag[j] | changed);
        a.chg_flag[j] = f;
    }
    // compact the changed columns of the block in ascending order
    const uint64_t ball = __ballot(f != 0);
    const int gshift = (threadIdx.x & (kWave - 1)) & ~15;
    const uint32_t mask = (uint32_t)((ball >> gshift) & 0xFFFFu);
    if (f) a.chg_idx[blk * kGemvtCols + __popc(mask & ((1u << lane16) - 1u))] = (int32_t)j;
    if (lane16 == 0 && (blk * kGemvtCols) < p) a.chg_cnt[blk] = __popc(mask);
}

}  // namespace gemvtdev
}  // namespace cox
