// gemv_dev.h -- the active-set eta update (Section 5.3's linear predictor,
// updated from the columns whose coefficient changed) and the compaction of
// the change list, as per-workgroup device functions shared by the launches
// of gemv.hip and the persistent path (persist.hip).
//
// eta += X~[:, S] dcoef_S for the set S of columns whose coefficient changed
// in the last step (the proximal step keeps most coefficients at zero, so S is
// small and only |S| columns are read).  Partial sums of a few column groups
// go to a buffer that the risk-set phase adds in fixed order; eta itself is
// held in FP64 so that the running sum tracks X~ beta exactly to rounding.
// The coefficients are already multiplied by the genotype scale s_j; the
// centring term is a constant shift of eta, to which the partial likelihood is
// invariant.
#pragma once
#include "device_common.h"

namespace cox {
namespace gemvdev {

constexpr int kT = kGemvThreads;
constexpr int kRows = 4 * kT;  // rows per workgroup

// Four rows of column `col` starting at row r0 (VEC: r0 % 4 == 0, 16- or 4-byte load).
template <int XT, bool VEC>
__device__ __forceinline__ void load_rows4(const XDesc& x, int64_t col, int64_t r0, int64_t n, float* o)
{
    const int64_t off = col * x.ldx + r0;
    if (VEC && r0 + 3 < n) {
        if constexpr (XT == XT_F32) {
            const float4 v = load_f4_stream(static_cast<const float*>(x.X) + off);
            o[0] = v.x;
            o[1] = v.y;
            o[2] = v.z;
            o[3] = v.w;
        } else {
            const uint32_t w =
                __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(x.X) + off));
            decode4<XT>(w, o);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = (r0 + e < n) ? load_x1<XT>(x.X, off + e) : 0.f;
    }
}

// Rows owned by this thread: VEC -> 4 consecutive rows; otherwise 4 rows 256 apart.
template <bool VEC>
__device__ __forceinline__ int64_t row_of(int64_t slab0, int e)
{
    return VEC ? slab0 + (int64_t)threadIdx.x * 4 + e : slab0 + threadIdx.x + (int64_t)kT * e;
}

// One workgroup of the eta update: row slab bx (kRows rows), column group cg.
template <int XT, int NB, bool VEC>
__device__ __forceinline__ void eta_update_blk(const XDesc& x, const int32_t* __restrict__ sel,
                                               const int32_t* __restrict__ nsel_p, const double* __restrict__ dcoef,
                                               int b0, int nb, double* __restrict__ part, int64_t cstride, int ncg,
                                               const int32_t* __restrict__ active, int bx, int cg)
{
    const int nsel = *nsel_p;
    if (nsel == 0) return;
    if (active) {
        int any = 0;
        for (int b = 0; b < nb; ++b) any |= active[b0 + b];
        if (!any) return;
    }
    const int64_t n = x.n, p = x.p;
    const int64_t slab0 = (int64_t)bx * kRows;
    const int chunk = (nsel + ncg - 1) / ncg;
    const int q0 = cg * chunk;
    const int q1 = min(nsel, q0 + chunk);
    double acc[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[b][e] = 0.0;
    const int64_t r0 = slab0 + (int64_t)threadIdx.x * 4;
    for (int q = q0; q < q1; q += 4) {
        float xv[4][4];
        int64_t jj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            jj[u] = q + u < q1 ? sel[q + u] : -1;
            if (jj[u] >= 0) {
                if (VEC) {
                    load_rows4<XT, true>(x, jj[u], r0, n, xv[u]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t r = row_of<false>(slab0, e);
                        xv[u][e] = r < n ? load_x1<XT>(x.X, jj[u] * x.ldx + r) : 0.f;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (jj[u] < 0) break;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b >= nb) break;
                const double d = dcoef[(int64_t)(b0 + b) * p + jj[u]];
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[b][e] = fma((double)xv[u][e], d, acc[b][e]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = row_of<VEC>(slab0, e);
            if (r < n) part[(int64_t)cg * cstride + (int64_t)(b0 + b) * n + r] = acc[b][e];
        }
    }
}

// Concatenates the per-block change lists in block order: sel = the idx[blk]
// entries, cnt[blk] of them, for blk = 0, 1, ...; *nsel = their number.  One
// workgroup of NT threads (a multiple of 64, at most 1024); per round of NT
// blocks each thread scans one block's count, then groups of kGemvtCols lanes
// copy whole blocks, one entry per lane.  The result does not depend on NT.
// LDS: sh[17], sstart[NT], scnt[NT].
template <int NT>
__device__ __forceinline__ void compact_blk(const int32_t* __restrict__ cnt, const int32_t* __restrict__ idx,
                                            int nblk, int32_t* __restrict__ sel, int32_t* __restrict__ nsel,
                                            int* sh, int* sstart, int* scnt, int b0 = 0, int b1 = 0x7fffffff,
                                            int carry = 0)
{
    static_assert(NT % kGemvtCols == 0 && NT % 64 == 0 && NT <= 1024 && kGemvtCols <= 64,
                  "lane groups tile the workgroup");
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int grp = threadIdx.x / kGemvtCols, q = threadIdx.x % kGemvtCols;
    // blocks [b0, min(b1, nblk)); carry = the changed columns of the blocks before b0
    const int bend = min(nblk, b1);
    for (int base = b0; base < bend; base += NT) {
        const int blk = base + threadIdx.x;
        const int c = blk < bend ? cnt[blk] : 0;
        int inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) sh[wid] = inc;
        __syncthreads();
        if (wid == 0) {
            const int t = lane < NW ? sh[lane] : 0;
            int ti = t;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(ti, o, 64);
                if (lane >= o) ti += u;
            }
            if (lane < NW) sh[lane] = ti - t;
            if (lane == NW - 1) sh[16] = ti;
        }
        __syncthreads();
        sstart[threadIdx.x] = carry + sh[wid] + inc - c;
        scnt[threadIdx.x] = c;
        const int tot = sh[16];
        __syncthreads();
        for (int bb = grp; bb < NT; bb += NT / kGemvtCols)
            if (q < scnt[bb]) sel[sstart[bb] + q] = idx[(int64_t)(base + bb) * kGemvtCols + q];
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && bend == nblk) *nsel = carry;
}

}  // namespace gemvdev
}  // namespace cox
