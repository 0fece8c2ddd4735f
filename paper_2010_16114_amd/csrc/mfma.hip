// mfma.hip -- X~' R for a batch of residual vectors on the int8 matrix cores.
//
// With B coefficient vectors the gradient pass of Section 5.3 becomes the
// skinny product G' R (p x n times n x B, K = n subjects).  Allele counts
// g in {0, 1, 2} are exact in int8.  Each residual vector r_b is quantised to
// integers R_b = round(r_b / q_b) with q_b = max_i |r_bi| / 2^22 and split into
// three signed 8-bit limbs, R = d0 + 256 d1 + 65536 d2.  Every limb product is
// then exact on v_mfma_i32_16x16x64_i8 with int32 accumulation (|sum| <=
// 2 * 128 * n < 2^31 for n < 2^22), and
//     sum_i g_ij R_bi = acc0 + 256 acc1 + 65536 acc2      (exact, int64)
// so the only rounding is that of r to 23 significant bits relative to its
// largest entry.  The raw sums q_b * sum_i g_ij R_bi go to the same epilogue
// as the vector path (centring with sum_i q_b R_bi, proximal step).
//
// Tiling: a workgroup of CW compute wavefronts owns 16 * MT * CW SNP columns
// (MT M tiles of 16 per wavefront) and all 3 * B limb columns (N tiles of
// 16), and walks K = n in stages of 64 or 128 subjects; LW more wavefronts
// stage the limb tiles.  X is read once per pass for all B vectors.  In
// mfma_xtr_split_kernel the A fragments (16 subjects of one column per lane,
// one 16-byte load) go straight to registers; in mfma_xtr_lds_kernel the
// loader wavefronts stage X through LDS too.  Several shapes of both are
// compiled; the host times them on the live data and keeps the fastest.
//
// The eta update (eta += G[:, U] D over the changed columns U, the same limb
// arithmetic with D = s * dbeta) contracts over columns, which X does not keep
// contiguous: mfma_eta_kernel and mfma_eta_split_kernel move 64-column x
// 256-subject tiles through LDS and transpose them into A fragments.
#include <type_traits>

#include "device_common.h"
#include "mfma.h"

namespace cox {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int kLimbs = 3;
constexpr int kQBits = 22;       // |R| <= 2^22 keeps the top limb within int8
constexpr int kQBits2 = 14;      // the same for two limbs (the residual's faster, coarser form)

// Allele-count bytes -> int8 counts.  FP8 E4M3 codes of 0, 1, 2 are 0x00, 0x38,
// 0x40, whose top three bits are the count itself (000, 001, 010); other codes
// are rejected before any matrix-core pass runs.
template <int XT>
__device__ __forceinline__ uint32_t counts4(uint32_t w)
{
    if constexpr (XT == XT_FP8)
        return (w >> 5) & 0x07070707u;
    else
        return w;
}

// The 16 bytes of column col from row row (row and ldx are multiples of 16, so
// the load never leaves the column's ldx bytes).  A run that starts outside
// the matrix loads from X itself.  The bytes of rows >= n are whatever the
// padding holds: the kernels make them harmless (zero limbs, or outputs that
// are never written).  The load and the decode are separate so that a
// prefetched run is only waited for where it is used.
// NT: a non-temporal (streaming) load, for runs whose cache line is consumed
// at once, so that X does not push the shared operand tiles out of L2.
template <bool NT = false>
__device__ __forceinline__ v4i load_raw(const uint8_t* __restrict__ X, int64_t col, int64_t p, int64_t ldx,
                                        int64_t row, int64_t n)
{
    const bool ok = col < p && row < n;
    const v4i* q = reinterpret_cast<const v4i*>(X + (ok ? col * ldx + row : 0));
    if constexpr (NT)
        return __builtin_nontemporal_load(q);
    else
        return *q;
}

// int8 counts of a raw run.
template <int XT>
__device__ __forceinline__ v4i decode_a(v4i raw)
{
    v4i v;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (int)counts4<XT>((uint32_t)raw[q]);
    return v;
}

// Software pipelines.  Vector-memory loads complete in issue order per
// wavefront, so a wait for one load is a wait for every older one.  Every
// global load of a stage is therefore issued PF stages before the stage runs,
// into ring slot t mod PF, and each ring is consumed in issue order: PF - 1
// stages stay in flight.  The loop bodies have no branches on data: stages
// past the end load clamped tiles whose products are skipped or zero.
//
// X~' R: the two operand streams run in different wavefronts.  CW compute
// wavefronts keep a ring of A runs only (X, from HBM); LW loader wavefronts
// move each stage's limb tile (mostly L2 hits) into LDS two stages ahead.  In
// one mixed ring every limb load waits behind the A loads issued before it;
// split, each stream drains at its own pace.  Both roles meet at one barrier
// per stage.  The limb rows of subjects >= n are zero (the quantiser writes
// them so), so the padding bytes of X that meet them add nothing.
//
// Each compute wavefront reads the limb tile's fragments from LDS one ahead of
// the MT matrix-core operations that use each.  (Reading three or five ahead,
// with scheduling barriers to keep the reads early, measured no faster.)
template <int XT, int NG, int RL, int CW, int LW, int MT, int KS, int PF, int LD = 2, bool NTX = false>
__global__ __launch_bounds__(64 * (CW + LW), (CW + LW) / 4) void mfma_xtr_split_kernel(MfmaArgs a)
{
    static_assert(PF >= 2 && LD >= 2 && PF % LD == 0, "the loaders' ring of LD slots indexes statically");
    static_assert(RL == 2 || RL == 3, "the residual comes in 2 or 3 limbs");
    constexpr int BR = 2;  // B fragments in flight
    constexpr int WCOLS = 16 * MT * CW;  // SNP columns per workgroup
    constexpr int KC = 64 * KS;
    constexpr int NT = RL * NG;         // N tiles, limb-major: tile = limb * NG + b / 16
    constexpr int NCOL = 16 * NT;
    constexpr int QC = KC / 16;
    constexpr int CHUNKS = NCOL * QC;
    constexpr int LTH = 64 * LW;
    constexpr int CPL = (CHUNKS + LTH - 1) / LTH;
    constexpr int RS = NCOL + 8;
    constexpr int NF = KS * NT;  // B fragments per stage
    __shared__ v4i sR[2][QC * RS];

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t n = a.n, p = a.p, ldx = a.ldx;
    const uint8_t* __restrict__ X = static_cast<const uint8_t*>(a.X);
    const int64_t nstage = (n + KC - 1) / KC;
    const int64_t nloop = (nstage + PF - 1) / PF * PF;

    if (wid < CW) {
        const int arow = 16 * (lane >> 4);
        const int acol = lane & 15;
        const int64_t jw = (int64_t)blockIdx.x * WCOLS + wid * (16 * MT);
        v4i acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};
        v4i Ab[PF][MT][KS];  // raw runs
        auto fetch = [&](int64_t t, v4i (&A)[MT][KS]) {
            const int64_t k0 = t * KC;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    A[mt][ks] = load_raw<NTX>(X, jw + mt * 16 + acol, p, ldx, k0 + ks * 64 + arow, n);
        };
#pragma unroll
        for (int q = 0; q < PF; ++q) fetch(q, Ab[q]);
        __syncthreads();
        for (int64_t s0 = 0; s0 < nloop; s0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int64_t t = s0 + q;
                const int buf = (int)(t & 1);
                if (t < nstage) {
                    const v4i* sb = &sR[buf][(lane >> 4) * RS + acol];
                    auto boff = [](int f) { return (f / NT) * 4 * RS + (f % NT) * 16; };
                    v4i br[BR];
#pragma unroll
                    for (int f = 0; f < BR - 1 && f < NF; ++f) br[f] = sb[boff(f)];
                    v4i A[MT];
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        if (f + BR - 1 < NF) br[(f + BR - 1) % BR] = sb[boff(f + BR - 1)];
                        if (f % NT == 0) {
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt) A[mt] = decode_a<XT>(Ab[q][mt][f / NT]);
                        }
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[mt][f % NT] =
                                __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], br[f % BR], acc[mt][f % NT], 0, 0, 0);
                    }
                }
                fetch(t + PF, Ab[q]);
                __syncthreads();
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int bq = 0; bq < NG; ++bq)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int b = bq * 16 + acol;
                    const int64_t j = jw + mt * 16 + mfma_c_row(lane, v);
                    if (j < p && b < a.B) {
                        int64_t tot = (int64_t)acc[mt][bq][v] + 256 * (int64_t)acc[mt][NG + bq][v];
                        if constexpr (RL == 3) tot += 65536 * (int64_t)acc[mt][2 * NG + bq][v];
                        a.out[(int64_t)b * p + j] = a.qscale[b] * (double)tot;
                    }
                }
    } else {
        // loader: chunk c of a stage's contiguous limb tile goes to LDS slot (c / NCOL, c % NCOL)
        const int lt = threadIdx.x - 64 * CW;
        const int8_t* rsrc[CPL];
        int rdst[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int c = (lt + LTH * u) % CHUNKS;  // a chunk index past the end repeats a valid one
            rsrc[u] = a.limbs + 16 * c;
            rdst[u] = (c / NCOL) * RS + c % NCOL;
        }
        // a ring of LD stages of limb loads: at step t the loads of stage t + LD
        // go out before stage t + 1 (loaded LD - 1 steps earlier) is written to
        // LDS, so each load has LD - 1 stage times to arrive
        v4i Rb[LD][CPL];
        auto fetch_r = [&](int64_t t, v4i (&R)[CPL]) {
            const int64_t kr = min(t, nstage - 1) * (int64_t)(16 * CHUNKS);
#pragma unroll
            for (int u = 0; u < CPL; ++u) R[u] = *reinterpret_cast<const v4i*>(rsrc[u] + kr);
        };
        auto store_r = [&](int buf, const v4i (&R)[CPL]) {
#pragma unroll
            for (int u = 0; u < CPL; ++u) sR[buf][rdst[u]] = R[u];
        };
#pragma unroll
        for (int u = 0; u < LD; ++u) fetch_r(u, Rb[u]);
        store_r(0, Rb[0]);
        __syncthreads();
        for (int64_t s0 = 0; s0 < nloop; s0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int64_t t = s0 + q;
                fetch_r(t + LD, Rb[q % LD]);
                __builtin_amdgcn_sched_barrier(0);  // keep the new loads ahead of the stores below
                store_r((int)(t & 1) ^ 1, Rb[(q + 1) % LD]);
                __syncthreads();
            }
        }
    }
}

// X~' R with both operands through LDS.  LW loader wavefronts move each
// stage's X tile (the workgroup's WCOLS columns x 16 QC subjects, decoded to
// counts) and limb tile into LDS, with LDF stages of loads in flight in
// registers; CW compute wavefronts read both from LDS and run the matrix cores,
// QC / 4 steps of 64 subjects per stage.  The loaders read a column's 16 QC
// bytes of a stage with QC adjacent lanes, so that they go out as one request
// with one address translation (QC = 8: one whole 128-byte line per column and
// stage, where QC = 4 reads each line in two halves, a stage apart); in the
// matrix-core layout that mfma_xtr_split_kernel loads directly those bytes sit
// in lanes 16 apart and go out as separate 16-byte requests.  In LDS a column
// takes 16 (QC + 1) bytes (16 of padding), so that the 16 lanes of a fragment
// read (16 consecutive columns, one 16-byte chunk each) hit distinct banks.
//
// KSPLIT > 1 splits the last, partly filled round of workgroups: each block of
// columns from a.nfull on is taken by KSPLIT workgroups, one run of consecutive
// stages each, which write their exact integer sums to a.tail for
// xtr_tail_kernel to add (integer sums: the result equals the unsplit one).
template <int XT, int NG, int RL, int CW, int LW, int MT, int LDF, bool NTX = false, int QC = 4, int KSPLIT = 1>
__global__ __launch_bounds__(64 * (CW + LW), (CW + LW) / 4) void mfma_xtr_lds_kernel(MfmaArgs a)
{
    static_assert(LDF >= 2, "the loaders' ring needs two slots");
    static_assert(RL == 2 || RL == 3, "the residual comes in 2 or 3 limbs");
    static_assert(QC == 4 || QC == 8, "stages of 64 or 128 subjects");
    constexpr int WCOLS = 16 * MT * CW;  // SNP columns per workgroup
    constexpr int NT = RL * NG;          // N tiles, limb-major: tile = limb * NG + b / 16
    constexpr int NCOL = 16 * NT;
    constexpr int SUBJ = 16 * QC;        // subjects per stage
    constexpr int CHUNKS = NCOL * QC;    // limb chunks per stage
    constexpr int XCH = WCOLS * QC;      // X chunks per stage
    constexpr int LT = 64 * LW;
    constexpr int XPT = (XCH + LT - 1) / LT;
    constexpr int RPT = (CHUNKS + LT - 1) / LT;
    constexpr int RS = NCOL + 8;         // LDS row stride of the limb tile (16-byte units)
    constexpr int XS = QC + 1;           // LDS stride of a column of the X tile (16-byte units)
    constexpr bool XALL = XCH % LT == 0, RALL = CHUNKS % LT == 0;
    __shared__ v4i sR[2][QC * RS];
    __shared__ v4i sX[2][WCOLS * XS];

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t n = a.n, p = a.p, ldx = a.ldx;
    const int64_t nstage = (n + SUBJ - 1) / SUBJ;
    int64_t blk = blockIdx.x, t0 = 0, t1 = nstage;  // block of columns, stages [t0, t1)
    int part = -1;                                  // share of a split block, or -1
    if constexpr (KSPLIT > 1) {
        if (blk >= a.nfull) {
            const int64_t v = blk - a.nfull;
            blk = a.nfull + v / KSPLIT;
            part = (int)(v % KSPLIT);
            t0 = nstage * part / KSPLIT;
            t1 = nstage * (part + 1) / KSPLIT;
        }
    }
    const int64_t nst = t1 - t0;
    const int64_t nloop = (nst + LDF - 1) / LDF * LDF;
    const int64_t j0 = blk * WCOLS;

    if (wid >= CW) {
        // loaders.  X chunk c: column c / QC of the workgroup, subjects 16 (c % QC) .. + 15 of the
        // stage; a column past p, or a chunk that starts at or after n, loads the start of X (the
        // limb rows of subjects n .. round_up(n, 256) are zero, and columns >= p are never stored).
        // t counts the workgroup's stages from t0; the ring slots and LDS buffers go by t
        const int lt = threadIdx.x - 64 * CW;
        const uint8_t* __restrict__ X = static_cast<const uint8_t*>(a.X);
        uint64_t xbase[XPT];
        int xrow[XPT], xdst[XPT];
        bool xok[XPT];
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int c = lt + LT * k;
            xok[k] = XALL || c < XCH;
            const int cc = xok[k] ? c : 0;
            const int64_t col = j0 + cc / QC;
            xbase[k] = col < p ? (uint64_t)col * (uint64_t)ldx : 0;
            xrow[k] = 16 * (cc % QC);
            xdst[k] = (cc / QC) * XS + cc % QC;
        }
        const int8_t* rsrc[RPT];
        int rdst[RPT];
        bool rok[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int c = lt + LT * k;
            rok[k] = RALL || c < CHUNKS;
            const int cc = rok[k] ? c : 0;
            rsrc[k] = a.limbs + 16 * cc;
            rdst[k] = (cc / NCOL) * RS + cc % NCOL;
        }
        v4i xr[LDF][XPT];
        v4i rr[LDF][RPT];
        auto fetch = [&](int64_t t, v4i (&xg)[XPT], v4i (&rg)[RPT]) {
#pragma unroll
            for (int k = 0; k < XPT; ++k) {
                const int64_t row = (t0 + t) * SUBJ + xrow[k];
                const v4i* src = reinterpret_cast<const v4i*>(X + (row < n ? xbase[k] + (uint64_t)row : 0));
                if (xok[k]) {
                    if constexpr (NTX)
                        xg[k] = __builtin_nontemporal_load(src);
                    else
                        xg[k] = *src;
                }
            }
            const int64_t kr = min(t0 + t, nstage - 1) * (int64_t)(16 * CHUNKS);
#pragma unroll
            for (int k = 0; k < RPT; ++k)
                if (rok[k]) rg[k] = *reinterpret_cast<const v4i*>(rsrc[k] + kr);
        };
        auto store = [&](int buf, const v4i (&xg)[XPT], const v4i (&rg)[RPT]) {
#pragma unroll
            for (int k = 0; k < XPT; ++k)
                if (xok[k]) sX[buf][xdst[k]] = decode_a<XT>(xg[k]);
#pragma unroll
            for (int k = 0; k < RPT; ++k)
                if (rok[k]) sR[buf][rdst[k]] = rg[k];
        };
#pragma unroll
        for (int q = 0; q < LDF; ++q) fetch(q, xr[q], rr[q]);
        store(0, xr[0], rr[0]);
        __syncthreads();
        for (int64_t s0 = 0; s0 < nloop; s0 += LDF) {
#pragma unroll
            for (int q = 0; q < LDF; ++q) {
                const int64_t t = s0 + q;
                fetch(t + LDF, xr[q], rr[q]);  // slot q held stage t, stored before the last barrier
                __builtin_amdgcn_sched_barrier(0);  // keep the new loads ahead of the stores below
                store((int)(t & 1) ^ 1, xr[(q + 1) % LDF], rr[(q + 1) % LDF]);
                __syncthreads();
            }
        }
        return;
    }

    // compute wavefronts
    const int acol = lane & 15;
    const int64_t jw = j0 + wid * (16 * MT);
    v4i acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};
    __syncthreads();  // the loaders' first stage is in LDS
    for (int64_t t = 0; t < nloop; ++t) {
        const int buf = (int)(t & 1);
        if (t < nst) {
#pragma unroll
            for (int h = 0; h < QC / 4; ++h) {  // 64 subjects per matrix-core step
                v4i A[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    A[mt] = sX[buf][(wid * MT * 16 + mt * 16 + acol) * XS + 4 * h + (lane >> 4)];
                const v4i* sb = &sR[buf][(4 * h + (lane >> 4)) * RS + acol];
                v4i bcur = sb[0];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    v4i bnext = bcur;
                    if (nt + 1 < NT) bnext = sb[(nt + 1) * 16];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], bcur, acc[mt][nt], 0, 0, 0);
                    bcur = bnext;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int bq = 0; bq < NG; ++bq)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = bq * 16 + acol;
                const int64_t j = jw + mt * 16 + mfma_c_row(lane, v);
                if (j < p && b < a.B) {
                    int64_t tot = (int64_t)acc[mt][bq][v] + 256 * (int64_t)acc[mt][NG + bq][v];
                    if constexpr (RL == 3) tot += 65536 * (int64_t)acc[mt][2 * NG + bq][v];
                    if (KSPLIT > 1 && part >= 0)
                        a.tail[((int64_t)part * a.B + b) * a.tail_cols + (j - a.nfull * WCOLS)] = tot;
                    else
                        a.out[(int64_t)b * p + j] = a.qscale[b] * (double)tot;
                }
            }
}

// The split blocks' sums: out[b][j0 + jj] = qscale_b (the sum over the ksplit shares).
__global__ __launch_bounds__(kT) void xtr_tail_kernel(MfmaArgs a, int ksplit, int64_t j0, int64_t ptail)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= (int64_t)a.B * ptail) return;
    const int b = (int)(i / ptail);
    const int64_t jj = i - (int64_t)b * ptail;
    long long tot = 0;
    for (int k = 0; k < ksplit; ++k) tot += a.tail[((int64_t)k * a.B + b) * a.tail_cols + jj];
    a.out[(int64_t)b * a.p + j0 + jj] = a.qscale[b] * (double)tot;
}

// Byte transpose of a 4 x 4 block: d[r] holds bytes (x_r0, x_r1, x_r2, x_r3);
// o[c] receives (x_0c, x_1c, x_2c, x_3c).  __builtin_amdgcn_perm(hi, lo, sel)
// picks byte sel_k of the 8-byte value hi:lo for result byte k.
__device__ __forceinline__ void transpose4x4(const uint32_t (&d)[4], uint32_t (&o)[4])
{
    const uint32_t lo01 = __builtin_amdgcn_perm(d[1], d[0], 0x05010400u);  // x00 x10 x01 x11
    const uint32_t hi01 = __builtin_amdgcn_perm(d[1], d[0], 0x07030602u);  // x02 x12 x03 x13
    const uint32_t lo23 = __builtin_amdgcn_perm(d[3], d[2], 0x05010400u);  // x20 x30 x21 x31
    const uint32_t hi23 = __builtin_amdgcn_perm(d[3], d[2], 0x07030602u);  // x22 x32 x23 x33
    o[0] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);                 // x00 x10 x20 x30
    o[1] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);                 // x01 x11 x21 x31
    o[2] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// eta update on the matrix cores: eta (n x B) += G[:, U] D, contracting over the
// changed columns U.  M = subjects, N = 3 * B limb columns, K = positions in U.
// A workgroup of 4 * NSPLIT wavefronts owns 256 subjects: wavefront w takes
// subjects [64 (w % 4), 64 (w % 4) + 64) and one NSPLIT-th of the b's (all
// three limbs of each).  NSPLIT = 2 fits the accumulators two wavefronts per
// SIMD; NSPLIT = 1 keeps one wavefront per SIMD with the accumulators in the
// accumulation registers, which leaves room for a deeper load ring.  G is stored with
// subjects contiguous, so each stage's 64-column x 256-subject tile passes
// through LDS: a lane reads one dword (4 consecutive subjects of a column) for
// each of its 16 columns and transposes the four 4 x 4 byte blocks in
// registers, which yields the A fragments of 4 M tiles (subject 4 r + mt of
// the wavefront's 64 is row r of tile mt).  Dword positions within a column are
// XOR-swizzled by the column's 16-group so that the four lane groups of a read
// hit distinct banks.  The column indices run one ring lap ahead of the G
// loads they address.  Each (subject, b) is owned by one lane, so eta is
// updated in place.
template <int XT, int NG, int NSPLIT, int PF, bool D8 = false, bool NTX = false>
__global__ __launch_bounds__(256 * NSPLIT, NSPLIT) void mfma_eta_kernel(MfmaEtaArgs a)
{
    static_assert(PF >= 2, "the ring needs two slots");
    static_assert(NSPLIT == 1 || NSPLIT == 2, "one or two b groups per subject block");
    constexpr int TH = 256 * NSPLIT;
    constexpr int SUB = 256;              // subjects per workgroup
    constexpr int SW = SUB / 4;           // dwords per column of the G tile
    constexpr int RB = SUB / 16;          // 16-byte chunks per column of the G tile
    constexpr int NT = kLimbs * NG;
    constexpr int NCOL = 16 * NT;
    constexpr int NGH = (NG + NSPLIT - 1) / NSPLIT;  // b groups of 16 per wavefront (a split of an odd NG repeats one)
    constexpr int GPT = 64 * RB / TH;     // 16-byte chunks of G per thread per stage
    constexpr int DCH = 4 * NCOL;         // 16-byte chunks of D per stage
    // D8: the D tile moves as 8-byte pieces, 2 DCH / TH per thread (3 at B = 64 over
    // 512 threads, where 16-byte chunks would leave half of a second chunk idle)
    constexpr int DPT = D8 ? 2 * DCH / TH : (DCH + TH - 1) / TH;
    constexpr int DS = NCOL + 8;          // LDS row stride of the D tile (16-byte units)
    static_assert(GPT * TH == 64 * RB, "G tile splits evenly");
    static_assert(!D8 || DPT * TH == 2 * DCH, "8-byte D pieces split evenly");
    using dchunk = typename std::conditional<D8, uint2, v4i>::type;
    __shared__ uint32_t sG[2][64 * SW];
    __shared__ v4i sD[2][4 * DS];
    const int nsel = *a.nsel;
    if (nsel == 0) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wsub = wid & 3, half = wid >> 2;
    const int64_t n = a.n, p = a.p, ldx = a.ldx;
    const int64_t i0 = (int64_t)blockIdx.x * SUB;
    const uint8_t* __restrict__ X = static_cast<const uint8_t*>(a.X);
    const int32_t* __restrict__ sel = a.sel;
    const int64_t nchunk = (nsel + 63) / 64;
    const int64_t nloop = (nchunk + PF - 1) / PF * PF;

    // this thread's G chunks: column position gu[k] of the stage, 16 subjects from 16 * grb[k]
    int gu[GPT], grb[GPT], gdst[GPT];
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
        const int ch = threadIdx.x + TH * k;
        gu[k] = ch / RB;
        grb[k] = ch % RB;
        gdst[k] = gu[k] * SW + ((4 * grb[k]) ^ (((gu[k] >> 4) & 3) << 4));
    }
    // D chunks: a stage's D tile is one contiguous block of DCH chunks
    // ([16-position quarter kq][limb column])
    const int8_t* dsrc[DPT];
    int ddst[DPT];  // byte offset in a D buffer
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
        if constexpr (D8) {
            const int c8 = threadIdx.x + TH * k, c = c8 >> 1;
            dsrc[k] = a.dlimbs + 8 * c8;
            ddst[k] = ((c / NCOL) * DS + c % NCOL) * 16 + 8 * (c8 & 1);
        } else {
            const int c = (threadIdx.x + TH * k) % DCH;
            dsrc[k] = a.dlimbs + 16 * c;
            ddst[k] = ((c / NCOL) * DS + c % NCOL) * 16;
        }
    }
    // this wavefront's b groups
    int bqs[NGH];
#pragma unroll
    for (int j = 0; j < NGH; ++j) bqs[j] = min(half * NGH + j, NG - 1);

    auto load_sel = [&](int64_t t, int32_t (&s)[GPT]) {
#pragma unroll
        for (int k = 0; k < GPT; ++k) s[k] = sel[min(t * 64 + gu[k], (int64_t)nsel - 1)];
    };

    v4i acc[4][kLimbs][NGH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int l = 0; l < kLimbs; ++l)
#pragma unroll
            for (int j = 0; j < NGH; ++j) acc[mt][l][j] = v4i{0, 0, 0, 0};

    v4i gr[PF][GPT];
    dchunk dr[PF][DPT];
    int32_t sr[PF][GPT];  // column indices of stage t + PF, in slot t mod PF
    auto fetch = [&](int64_t t, const int32_t (&s)[GPT], v4i (&g)[GPT], dchunk (&dd)[DPT]) {
#pragma unroll
        for (int k = 0; k < GPT; ++k) {
            const int64_t col = t * 64 + gu[k] < nsel ? (int64_t)s[k] : p;  // past the list: reads as 0
            g[k] = load_raw<NTX>(X, col, p, ldx, i0 + 16 * grb[k], n);
        }
        const int64_t kd = min(t, nchunk - 1) * (int64_t)(16 * DCH);
#pragma unroll
        for (int k = 0; k < DPT; ++k) dd[k] = *reinterpret_cast<const dchunk*>(dsrc[k] + kd);
    };
    // positions past the change list read as 0 (subjects >= n only reach
    // outputs that are never written)
    auto store = [&](int64_t t, const v4i (&g)[GPT], const dchunk (&dd)[DPT]) {
        const int buf = (int)(t & 1);
#pragma unroll
        for (int k = 0; k < GPT; ++k)
            *reinterpret_cast<v4i*>(&sG[buf][gdst[k]]) =
                t * 64 + gu[k] < nsel ? decode_a<XT>(g[k]) : v4i{0, 0, 0, 0};
        char* sd = reinterpret_cast<char*>(sD[buf]);
#pragma unroll
        for (int k = 0; k < DPT; ++k) *reinterpret_cast<dchunk*>(sd + ddst[k]) = dd[k];
    };

    {
        int32_t s0[PF][GPT];
#pragma unroll
        for (int q = 0; q < PF; ++q) load_sel(q, s0[q]);
#pragma unroll
        for (int q = 0; q < PF; ++q) load_sel(q + PF, sr[q]);
#pragma unroll
        for (int q = 0; q < PF; ++q) fetch(q, s0[q], gr[q], dr[q]);
    }
    store(0, gr[0], dr[0]);
    __syncthreads();

    const int xr = wsub * 16 + (lane & 15);  // this lane's dword (4 subjects) within a column
    const int xs = xr ^ ((lane >> 4) << 4);  // its swizzled position (the 16-group of its columns is lane / 16)
    for (int64_t c0 = 0; c0 < nloop; c0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int64_t t = c0 + q;
            const int buf = (int)(t & 1);
            v4i A[4];
            {
                uint32_t f[4][4];  // f[mt][dword of the fragment]
#pragma unroll
                for (int blk = 0; blk < 4; ++blk) {
                    uint32_t d[4], o[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) d[e] = sG[buf][(16 * (lane >> 4) + 4 * blk + e) * SW + xs];
                    transpose4x4(d, o);
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) f[mt][blk] = o[mt];
                }
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) A[mt] = v4i{(int)f[mt][0], (int)f[mt][1], (int)f[mt][2], (int)f[mt][3]};
            }
            {
                const v4i* sb = &sD[buf][(lane >> 4) * DS + (lane & 15)];
                v4i bcur = sb[bqs[0] * 16];
#pragma unroll
                for (int l = 0; l < kLimbs; ++l)
#pragma unroll
                    for (int j = 0; j < NGH; ++j) {
                        const int f = l * NGH + j + 1;  // next fragment
                        v4i bnext = bcur;
                        if (f < kLimbs * NGH) bnext = sb[((f / NGH) * NG + bqs[f % NGH]) * 16];
#pragma unroll
                        for (int mt = 0; mt < 4; ++mt)
                            acc[mt][l][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], bcur, acc[mt][l][j], 0, 0, 0);
                        bcur = bnext;
                    }
            }
            fetch(t + PF, sr[q], gr[q], dr[q]);
            load_sel(t + 2 * PF, sr[q]);
            store(t + 1, gr[(q + 1) % PF], dr[(q + 1) % PF]);
            __syncthreads();
        }
    }

#pragma unroll
    for (int j = 0; j < NGH; ++j) {
        if (half * NGH + j >= NG) continue;  // the repeated group of an odd NG
        const int b = bqs[j] * 16 + (lane & 15);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + 64 * wsub + 4 * mfma_c_row(lane, v) + mt;
                if (i < n && b < a.B && (a.active == nullptr || a.active[b])) {
                    const int64_t tot = (int64_t)acc[mt][0][j][v] + 256 * (int64_t)acc[mt][1][j][v] +
                                        65536 * (int64_t)acc[mt][2][j][v];
                    a.eta[(int64_t)b * n + i] += a.dscale[b] * (double)tot;
                }
            }
    }
}

// eta update with the two operand streams in their own wavefronts, as in the
// X~' R pass: LW loader wavefronts move each stage's G tile (decoded to int8
// counts) and D tile into LDS and keep LDF stages of loads in flight in
// registers; CW compute wavefronts only read LDS and run the matrix cores.
// One barrier per stage joins the roles.  In mfma_eta_kernel every wavefront
// waits for its own loads of the next stage before the barrier, so about one
// stage of G is in flight per workgroup; here LDF - NB + 1 are.
//   NB = 2 LDS buffers: while the compute wavefronts work on buffer t % 2, the
//   loaders fill buffer (t + 1) % 2 with stage t + 1.
//   NB = 3: the loaders fill buffer (t + 2) % 3 with stage t + 2, so stage
//   t + 1 is complete while stage t is computed, and the compute wavefronts
//   read its G fragments before their matrix-core work on stage t.
// The work is a list of units (a block of 256 subjects, a stage of 64 columns
// of the change list), block by block; workgroup w takes an equal share of
// consecutive units.  With one workgroup per block (gridDim.x = the number of
// blocks) a share is one whole block.  With fewer workgroups, one per compute
// unit, every compute unit stays busy to the end instead of the last round of
// blocks running on a few of them; a block whose units two workgroups share is
// written by neither: each stores its exact int64 partial sums (a.part, slots
// [workgroup][head, tail]) and eta_fixup_kernel adds their sum, so eta gets
// the same single update, bit for bit, as from one workgroup.
// Tile layout (XOR-swizzled dword positions) and fragment transposes are
// mfma_eta_kernel's.  CW = 4: one compute wavefront per 64 subjects with every
// b group; CW = 8: two, with half the b groups each.
template <int XT, int NG, int CW, int LW, int LDF, int NB = 2, bool NTX = false>
__global__ __launch_bounds__(64 * (CW + LW), (CW + LW) / 4) void mfma_eta_split_kernel(MfmaEtaArgs a)
{
    static_assert(CW == 4 || CW == 8, "one or two compute wavefronts per 64 subjects");
    static_assert(NB == 2 || NB == 3, "two or three LDS buffers");
    static_assert(LDF >= NB, "the loaders' ring must reach the buffer they fill");
    constexpr int AH = NB - 1;            // stages between the one computed and the one stored
    constexpr int SUB = 256;              // subjects per block
    constexpr int SW = SUB / 4;           // dwords per column of the G tile
    constexpr int RB = SUB / 16;          // 16-byte chunks per column of the G tile
    constexpr int NT = kLimbs * NG;
    constexpr int NCOL = 16 * NT;
    constexpr int NSPLIT = CW / 4;
    constexpr int NGH = (NG + NSPLIT - 1) / NSPLIT;  // b groups of 16 per compute wavefront
    constexpr int LT = 64 * LW;           // loader threads
    constexpr int GCH = 64 * RB;          // 16-byte chunks of G per stage
    constexpr int GPT = GCH / LT;
    constexpr int DCH = 4 * NCOL;         // 16-byte chunks of D per stage
    constexpr int DPT = (DCH + LT - 1) / LT;
    constexpr int DS = NCOL + 8;          // LDS row stride of the D tile (16-byte units)
    static_assert(GPT * LT == GCH, "G tile splits evenly over the loaders");
    constexpr bool DALL = DCH % LT == 0;  // every loader thread moves DPT chunks of D
    __shared__ uint32_t sG[NB][64 * SW];
    __shared__ v4i sD[NB][4 * DS];
    const int nsel = *a.nsel;
    if (nsel == 0) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t n = a.n, ldx = a.ldx;
    const int nchunk = (nsel + 63) / 64;
    // this workgroup's units: R whole blocks w, w + G, ... (the rounds in which every
    // workgroup has a block), then its share of the T blocks left over
    const int64_t nblk = (n + SUB - 1) / SUB;
    const int64_t G = gridDim.x, w = blockIdx.x;
    const int R = (int)(nblk / G);
    const int64_t T = nblk - (int64_t)R * G;
    const int64_t tu = T * nchunk, tbase = tu / G, trem = tu % G;
    const int64_t tu0 = w * tbase + min(w, trem);  // first unit of the share within the left-over blocks
    const int tlen = (int)(tbase + (w < trem ? 1 : 0));
    const int64_t tblk0 = (int64_t)R * G + tu0 / nchunk;  // the block it starts in
    const int tst0 = (int)(tu0 % nchunk);
    const int nst = R * nchunk + tlen;
    const int nloop = (nst + LDF - 1) / LDF * LDF;
    // a position in this workgroup's unit list, advanced one stage at a time:
    // r < R: stage st of block w + r G; r == R: stage st of left-over block blk
    struct Pos {
        int64_t blk;
        int st, r;
    };
    const Pos first = R > 0 ? Pos{w, 0, 0} : Pos{tblk0, tst0, R};
    auto advance = [&](Pos& q) {
        if (++q.st < nchunk) return;
        q.st = 0;
        if (q.r == R) {  // within the share of the left-over blocks
            ++q.blk;
            return;
        }
        if (++q.r < R) {  // the next round's block
            q.blk += G;
            return;
        }
        q.blk = tblk0;  // the rounds are done: the share of the left-over blocks
        q.st = tst0;
    };

    if (wid >= CW) {
        // loaders; 32-bit index arithmetic (the host launches this kernel only for ldx < 2^32)
        const int lt = threadIdx.x - 64 * CW;
        const uint8_t* __restrict__ X = static_cast<const uint8_t*>(a.X);
        const int32_t* __restrict__ sel = a.sel;
        const uint32_t ldx32 = (uint32_t)ldx;
        int gu[GPT], grow[GPT], gdst[GPT];  // column in the stage, subject in the block, LDS dword
#pragma unroll
        for (int k = 0; k < GPT; ++k) {
            const int ch = lt + LT * k;
            const int grb = ch % RB;
            gu[k] = ch / RB;
            grow[k] = 16 * grb;
            gdst[k] = gu[k] * SW + ((4 * grb) ^ (((gu[k] >> 4) & 3) << 4));
        }
        // a stage's D tile is one contiguous block of DCH chunks ([16-position quarter][limb column])
        const int8_t* dsrc[DPT];
        int ddst[DPT];  // byte offset in a D buffer
        bool dok[DPT];
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int c = lt + LT * k;
            dok[k] = DALL || c < DCH;
            const int cc = dok[k] ? c : 0;
            dsrc[k] = a.dlimbs + 16 * cc;
            ddst[k] = ((cc / NCOL) * DS + cc % NCOL) * 16;
        }
        auto load_sel = [&](const Pos& q, int32_t (&s)[GPT]) {
#pragma unroll
            for (int k = 0; k < GPT; ++k) s[k] = sel[min(q.st * 64 + gu[k], nsel - 1)];
        };
        v4i gr[LDF][GPT];
        v4i dr[LDF][DPT];
        int32_t sr[LDF][GPT];  // column indices of stage t + LDF, in slot t mod LDF
        // stage at position q.  Nothing needs zeroing: positions past the change list load
        // the clamped last column and meet D limbs that are zero there, and subjects past
        // the last one (a chunk that starts at or after n loads the start of X) reach only
        // outputs that are never written; stages past the share are never flushed
        auto fetch = [&](const Pos& q, const int32_t (&s)[GPT], v4i (&g)[GPT], v4i (&dd)[DPT]) {
            const int64_t r0 = q.blk * SUB;
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                const uint64_t off = r0 + grow[k] < n ? (uint64_t)(uint32_t)s[k] * ldx32 + (uint32_t)(r0 + grow[k]) : 0;
                const v4i* src = reinterpret_cast<const v4i*>(X + off);
                if constexpr (NTX)
                    g[k] = __builtin_nontemporal_load(src);
                else
                    g[k] = *src;
            }
            const int64_t kd = (int64_t)q.st * (16 * DCH);
#pragma unroll
            for (int k = 0; k < DPT; ++k)
                if (dok[k]) dd[k] = *reinterpret_cast<const v4i*>(dsrc[k] + kd);
        };
        auto store = [&](int buf, const v4i (&g)[GPT], const v4i (&dd)[DPT]) {
#pragma unroll
            for (int k = 0; k < GPT; ++k) *reinterpret_cast<v4i*>(&sG[buf][gdst[k]]) = decode_a<XT>(g[k]);
            char* sd = reinterpret_cast<char*>(sD[buf]);
#pragma unroll
            for (int k = 0; k < DPT; ++k)
                if (dok[k]) *reinterpret_cast<v4i*>(sd + ddst[k]) = dd[k];
        };
        Pos pf = first, ps = first;  // the stage the next fetch and the next column-index load are for
        {
            int32_t s0[LDF][GPT];
#pragma unroll
            for (int q = 0; q < LDF; ++q) {
                load_sel(ps, s0[q]);
                advance(ps);
            }
#pragma unroll
            for (int q = 0; q < LDF; ++q) {
                load_sel(ps, sr[q]);
                advance(ps);
            }
#pragma unroll
            for (int q = 0; q < LDF; ++q) {
                fetch(pf, s0[q], gr[q], dr[q]);
                advance(pf);
            }
        }
#pragma unroll
        for (int q = 0; q < AH; ++q) store(q, gr[q], dr[q]);
        __syncthreads();
        int wb = AH % NB;  // the buffer stage t + AH goes to
        for (int c0 = 0; c0 < nloop; c0 += LDF) {
#pragma unroll
            for (int q = 0; q < LDF; ++q) {
                // at step t = c0 + q: the loads of stage t + LDF go to slot q, which held stage t,
                // stored before the last barrier
                fetch(pf, sr[q], gr[q], dr[q]);
                advance(pf);
                load_sel(ps, sr[q]);
                advance(ps);
                __builtin_amdgcn_sched_barrier(0);  // keep the new loads ahead of the stores below
                store(wb, gr[(q + AH) % LDF], dr[(q + AH) % LDF]);
                wb = wb + 1 == NB ? 0 : wb + 1;
                __syncthreads();
            }
        }
        return;
    }

    // compute wavefronts
    const int wsub = wid & 3, half = wid >> 2;
    int bqs[NGH];
#pragma unroll
    for (int j = 0; j < NGH; ++j) bqs[j] = min(half * NGH + j, NG - 1);
    v4i acc[4][kLimbs][NGH];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int l = 0; l < kLimbs; ++l)
#pragma unroll
            for (int j = 0; j < NGH; ++j) acc[mt][l][j] = v4i{0, 0, 0, 0};

    const int xr = wsub * 16 + (lane & 15);  // this lane's dword (4 subjects) within a column
    const int xs = xr ^ ((lane >> 4) << 4);  // its swizzled position (the 16-group of its columns is lane / 16)
    // the A fragments of 4 M tiles from a G buffer (M tile mt is subjects 4 r + mt)
    auto read_a = [&](int buf, v4i (&A)[4]) {
        uint32_t f[4][4];  // f[mt][dword of the fragment]
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            uint32_t d[4], o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) d[e] = sG[buf][(16 * (lane >> 4) + 4 * blk + e) * SW + xs];
            transpose4x4(d, o);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) f[mt][blk] = o[mt];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) A[mt] = v4i{(int)f[mt][0], (int)f[mt][1], (int)f[mt][2], (int)f[mt][3]};
    };
    // the sums of a block's units: eta += q_b * sum, or (a left-over block, shared
    // among workgroups) the exact partial sums into this workgroup's slot
    auto flush = [&](int64_t blk, int slot) {
#pragma unroll
        for (int j = 0; j < NGH; ++j) {
            if (half * NGH + j >= NG) continue;  // the repeated group of an odd NG
            const int b = bqs[j] * 16 + (lane & 15);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 64 * wsub + 4 * mfma_c_row(lane, v) + mt;
                    const int64_t i = blk * SUB + r;
                    if (i < n && b < a.B && (a.active == nullptr || a.active[b])) {
                        const int64_t tot = (int64_t)acc[mt][0][j][v] + 256 * (int64_t)acc[mt][1][j][v] +
                                            65536 * (int64_t)acc[mt][2][j][v];
                        if (slot < 0)
                            a.eta[(int64_t)b * n + i] += a.dscale[b] * (double)tot;
                        else
                            a.part[((w * 2 + slot) * a.bpad + b) * SUB + r] = tot;
                    }
                    acc[mt][0][j][v] = acc[mt][1][j][v] = acc[mt][2][j][v] = 0;
                }
        }
    };
    // a stage's matrix-core work: every limb and b group of the D tile in buffer cb
    // against the 4 A fragments
    auto mfma_stage = [&](int cb, const v4i (&A)[4]) {
        const v4i* sb = &sD[cb][(lane >> 4) * DS + (lane & 15)];
        v4i bcur = sb[bqs[0] * 16];
#pragma unroll
        for (int l = 0; l < kLimbs; ++l)
#pragma unroll
            for (int j = 0; j < NGH; ++j) {
                const int f = l * NGH + j + 1;  // next fragment
                v4i bnext = bcur;
                if (f < kLimbs * NGH) bnext = sb[((f / NGH) * NG + bqs[f % NGH]) * 16];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    acc[mt][l][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], bcur, acc[mt][l][j], 0, 0, 0);
                bcur = bnext;
            }
    };
    __syncthreads();  // the loaders' first stages are in LDS
    v4i A[4];
    if constexpr (NB == 3) read_a(0, A);
    int cb = 0;  // the buffer of stage t
    Pos pc = first;
    for (int t = 0; t < nloop; ++t) {
        if constexpr (NB == 3) {
            // stage t + 1 is complete: issue its fragment reads first, transpose them after
            // this stage's matrix-core work
            uint32_t d[4][4];
            const int nb = cb + 1 == NB ? 0 : cb + 1;
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int e = 0; e < 4; ++e) d[blk][e] = sG[nb][(16 * (lane >> 4) + 4 * blk + e) * SW + xs];
            mfma_stage(cb, A);
            uint32_t f[4][4];  // f[mt][dword of the fragment]
#pragma unroll
            for (int blk = 0; blk < 4; ++blk) {
                uint32_t o[4];
                transpose4x4(d[blk], o);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) f[mt][blk] = o[mt];
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) A[mt] = v4i{(int)f[mt][0], (int)f[mt][1], (int)f[mt][2], (int)f[mt][3]};
        } else {
            read_a(cb, A);
            mfma_stage(cb, A);
        }
        // the last unit of a block, or of this workgroup's share of a left-over block
        if (t < nst && (pc.st == nchunk - 1 || t == nst - 1))
            flush(pc.blk, pc.r < R ? -1 : (pc.blk == tblk0 ? 0 : 1));
        advance(pc);
        cb = cb + 1 == NB ? 0 : cb + 1;
        __syncthreads();
    }
}

// The left-over blocks of mfma_eta_split_kernel (those after the last round in
// which every one of its `shares` workgroups had a whole block), one workgroup
// per block and vector b (blockIdx.y), one thread per subject: eta += q_b *
// (the sum of the partial sums of the shares that cover the block, in share
// order; a share covers at most two of them, its first in slot 0, its second
// in slot 1).
__global__ __launch_bounds__(kT) void eta_fixup_kernel(MfmaEtaArgs a, int shares)
{
    static_assert(kT == 256, "one thread per subject of a block");
    const int nsel = *a.nsel;
    if (nsel == 0) return;
    constexpr int SUB = 256;
    const int64_t n = a.n, G = shares;
    const int64_t nchunk = (nsel + 63) / 64;
    const int64_t nblk = (n + SUB - 1) / SUB;
    const int64_t R = nblk / G, T = nblk - R * G;
    const int64_t tu = T * nchunk, tbase = tu / G, trem = tu % G;
    const int64_t tb = blockIdx.x;  // left-over block
    if (tb >= T) return;
    // the share holding unit u of the left-over list
    auto share_of = [&](int64_t u) {
        const int64_t big = trem * (tbase + 1);
        return u < big ? u / (tbase + 1) : trem + (u - big) / tbase;
    };
    const int64_t wa = share_of(tb * nchunk), wb = share_of((tb + 1) * nchunk - 1);
    const int64_t blk = R * G + tb;
    const int b = blockIdx.y, r = threadIdx.x;
    const int64_t i = blk * SUB + r;
    if (i < n && (a.active == nullptr || a.active[b])) {
        int64_t tot = 0;
        for (int64_t w = wa; w <= wb; ++w) {
            const int64_t first = (w * tbase + min(w, trem)) / nchunk;  // the first left-over block of w
            const int slot = first == tb ? 0 : 1;
            tot += a.part[((w * 2 + slot) * a.bpad + b) * SUB + r];
        }
        a.eta[(int64_t)b * n + i] += a.dscale[b] * (double)tot;
    }
}

// Largest |D_b(u)| over a tile of 4096 positions of the change list.
__global__ __launch_bounds__(kT) void dmax_kernel(const double* __restrict__ dcoef, int64_t p,
                                                  const int32_t* __restrict__ sel, const int32_t* __restrict__ nsel,
                                                  double* __restrict__ part, int ntile)
{
    __shared__ double sh[kT / 64];
    const int b = blockIdx.y;
    const int m = *nsel;
    double mx = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * 4096 + threadIdx.x; u < min((int64_t)m, (int64_t)(blockIdx.x + 1) * 4096);
         u += kT)
        mx = fmax(mx, fabs(dcoef[(int64_t)b * p + sel[u]]));
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)b * ntile + blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// D limbs by position; positions nsel .. round_up(nsel, 64) - 1 are zeroed.
// Limb layout as for the residual: [u / 16][limb * bpad + b][u % 16].
__global__ __launch_bounds__(kT) void dquant_kernel(const double* __restrict__ dcoef, int64_t p,
                                                    const int32_t* __restrict__ sel, const int32_t* __restrict__ nsel,
                                                    const double* __restrict__ dmaxp, int ntile,
                                                    int8_t* __restrict__ dlimbs, int bpad,
                                                    double* __restrict__ dscale)
{
    const int b = blockIdx.y;
    const int m = *nsel;
    const int mt = (m + 4095) / 4096;
    double mx = 0.0;
    for (int t = 0; t < mt; ++t) mx = fmax(mx, dmaxp[(int64_t)b * ntile + t]);
    const double q = mx > 0.0 ? mx / (double)(1 << kQBits) : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) dscale[b] = q;
    const int64_t mpad = ((int64_t)m + 63) / 64 * 64;
    for (int64_t u = (int64_t)blockIdx.x * 4096 + threadIdx.x; u < min(mpad, (int64_t)(blockIdx.x + 1) * 4096);
         u += kT) {
        int d0 = 0, d1 = 0, d2 = 0;
        if (u < m) {
            const int R = (int)llrint(dcoef[(int64_t)b * p + sel[u]] / q);
            d0 = ((R + 128) & 255) - 128;
            const int R1 = (R - d0) >> 8;
            d1 = ((R1 + 128) & 255) - 128;
            d2 = (R1 - d1) >> 8;
        }
        int8_t* dst = dlimbs + ((u >> 4) * (3 * bpad) + b) * 16 + (u & 15);
        dst[0] = (int8_t)d0;
        dst[16 * bpad] = (int8_t)d1;
        dst[32 * bpad] = (int8_t)d2;
    }
}

// Largest |r| of each vector over a tile of 4096 subjects.
__global__ __launch_bounds__(kT) void rmax_kernel(const double* __restrict__ r, int64_t n, double* __restrict__ part,
                                                  int ntile)
{
    __shared__ double sh[kT / 64];
    const int b = blockIdx.y;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4096 + threadIdx.x; i < min(n, (int64_t)(blockIdx.x + 1) * 4096);
         i += kT)
        m = fmax(m, fabs(r[(int64_t)b * n + i]));
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)b * ntile + blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// Quantise r to nlimb int8 limbs per vector (3: |R| <= 2^22; 2: |R| <= 2^14,
// the top limb within int8 either way); exact partial sums of R.  Limb
// layout: 16-subject chunks, [i / 16][limb * bpad + b][i % 16], so that a
// stage's tile (all nlimb * bpad limb columns of KC subjects) is one
// contiguous block.  Rows n .. round_up(n, 256) - 1 are written as zeros: the X~' R
// kernel reads whole 64- or 128-subject stages, and the layout changes with
// bpad, so stale limbs from an earlier batch size must not survive there.
__global__ __launch_bounds__(kT) void quantize_kernel(const double* __restrict__ r, int64_t n,
                                                      const double* __restrict__ rmaxp, int ntile,
                                                      int8_t* __restrict__ limbs, int bpad, int nlimb,
                                                      double* __restrict__ qscale, long long* __restrict__ rsump)
{
    __shared__ long long sh[kT / 64];
    const int b = blockIdx.y;
    double mx = 0.0;
    for (int t = 0; t < ntile; ++t) mx = fmax(mx, rmaxp[(int64_t)b * ntile + t]);
    const int bits = nlimb == 2 ? kQBits2 : kQBits;
    const double q = mx > 0.0 ? mx / (double)(1 << bits) : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) qscale[b] = q;
    long long sum = 0;
    const int64_t npad = (n + 255) / 256 * 256;
    for (int64_t i = (int64_t)blockIdx.x * 4096 + threadIdx.x; i < min(npad, (int64_t)(blockIdx.x + 1) * 4096);
         i += kT) {
        const int R = i < n ? (int)llrint(r[(int64_t)b * n + i] / q) : 0;
        const int d0 = ((R + 128) & 255) - 128;
        const int R1 = (R - d0) >> 8;
        int8_t* dst = limbs + ((i >> 4) * (nlimb * bpad) + b) * 16 + (i & 15);
        dst[0] = (int8_t)d0;
        if (nlimb == 2) {
            dst[16 * bpad] = (int8_t)R1;  // |R1| <= 64 when |R| <= 2^14
        } else {
            const int d1 = ((R1 + 128) & 255) - 128;
            dst[16 * bpad] = (int8_t)d1;
            dst[32 * bpad] = (int8_t)((R1 - d1) >> 8);
        }
        sum += R;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) rsump[(int64_t)b * ntile + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// sumr_b = q_b * sum_i R_bi (the sum of the quantised residual, exact).
__global__ void rsum_kernel(const long long* __restrict__ rsump, int ntile, const double* __restrict__ qscale,
                            double* __restrict__ sumr, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    long long s = 0;
    for (int t = 0; t < ntile; ++t) s += rsump[(int64_t)b * ntile + t];
    sumr[b] = qscale[b] * (double)s;
}

// bad[0] |= 1 if any byte of the n x p matrix is not the code of 0, 1 or 2
// (16-byte loads: the matrix-core path requires a 16-byte aligned ldx).
template <int XT>
__device__ __forceinline__ bool bad4(uint32_t w)
{
    bool b = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t v = (w >> (8 * e)) & 0xff;
        b |= XT == XT_FP8 ? !(v == 0x00 || v == 0x38 || v == 0x40) : !(v <= 2);
    }
    return b;
}

template <int XT>
__global__ __launch_bounds__(kT) void geno_check_kernel(const uint8_t* __restrict__ X, int64_t n, int64_t ldx,
                                                        int* __restrict__ bad)
{
    const int64_t j = blockIdx.x;
    const uint8_t* col = X + j * ldx;
    bool b = false;
    const int64_t nv = n / 16 * 16;
    for (int64_t i = (int64_t)threadIdx.x * 16; i < nv; i += (int64_t)kT * 16) {
        const uint4 u = *reinterpret_cast<const uint4*>(col + i);
        b |= bad4<XT>(u.x) | bad4<XT>(u.y) | bad4<XT>(u.z) | bad4<XT>(u.w);
    }
    for (int64_t i = nv + threadIdx.x; i < n; i += kT) b |= bad4<XT>((uint32_t)col[i]);  // zero bytes are valid codes
    if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

template <int XT, int NG, int NSPLIT, int PF, bool D8 = false, bool NTX = false>
hipError_t launch_eta_shape(const MfmaEtaArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((mfma_eta_kernel<XT, NG, NSPLIT, PF, D8, NTX>), dim3((unsigned)((a.n + 255) / 256)),
                       dim3(256 * NSPLIT), 0, s, a);
    return hipGetLastError();
}

// SK: one workgroup per compute unit (a.sk_grid of them) sharing the blocks evenly,
// then the shared blocks' partial sums; otherwise one workgroup per block.
template <int XT, int NG, int CW, int LW, int LDF, int NB = 2, bool NTX = false, bool SK = false>
hipError_t launch_eta_split(const MfmaEtaArgs& a, hipStream_t s)
{
    if (a.ldx >= (int64_t(1) << 32)) return hipErrorInvalidValue;  // its loaders index X in 32 bits
    const int64_t nblk = (a.n + 255) / 256;
    int64_t grid = nblk;
    if (SK && a.part && a.sk_grid > 0 && a.sk_grid < nblk) grid = a.sk_grid;
    hipLaunchKernelGGL((mfma_eta_split_kernel<XT, NG, CW, LW, LDF, NB, NTX>), dim3((unsigned)grid),
                       dim3(64 * (CW + LW)), 0, s, a);
    const int64_t left = nblk % grid;  // blocks after the last whole round
    if (left > 0) hipLaunchKernelGGL(eta_fixup_kernel, dim3((unsigned)left, (unsigned)a.B), dim3(kT), 0, s, a, (int)grid);
    return hipGetLastError();
}

template <int XT, int NG>
hipError_t launch_eta_ng(const MfmaEtaArgs& a, hipStream_t s)
{
    switch (a.variant) {
    case 1: return launch_eta_shape<XT, NG, 2, 2>(a, s);
    case 2: return launch_eta_split<XT, NG, 4, 4, 3>(a, s);
    case 3: return launch_eta_split<XT, NG, 4, 4, 4>(a, s);
    case 4: return launch_eta_split<XT, NG, 8, 4, 3>(a, s);
    case 5: return launch_eta_split<XT, NG, 4, 4, 5>(a, s);
    case 6: return launch_eta_split<XT, NG, 4, 4, 3, 2, true>(a, s);
    case 7: return launch_eta_split<XT, NG, 8, 4, 3, 3>(a, s);
    case 8: return launch_eta_split<XT, NG, 4, 4, 3, 2, true, true>(a, s);
    case 9: return launch_eta_split<XT, NG, 4, 4, 3, 2, false, true>(a, s);
    case 10: return launch_eta_split<XT, NG, 4, 4, 4, 2, true, true>(a, s);
    case 11: return launch_eta_split<XT, NG, 8, 4, 3, 2, true, true>(a, s);
    case 12: return launch_eta_split<XT, NG, 4, 4, 5, 2, true, true>(a, s);
    default: return launch_eta_shape<XT, NG, 2, 2, NG == 4>(a, s);  // the 8-byte D pieces divide over 512 threads at NG = 4
    }
}

template <int XT>
hipError_t launch_eta_xt(const MfmaEtaArgs& a, hipStream_t s)
{
    switch (a.bpad / 16) {
    case 1: return launch_eta_ng<XT, 1>(a, s);
    case 2: return launch_eta_ng<XT, 2>(a, s);
    case 3: return launch_eta_ng<XT, 3>(a, s);
    default: return launch_eta_ng<XT, 4>(a, s);
    }
}

template <int XT, int NG, int RL, int CW, int LW, int MT, int KS, int PF, int LD = 2, bool NTX = false>
hipError_t launch_split(const MfmaArgs& a, hipStream_t s)
{
    constexpr int WCOLS = 16 * MT * CW;
    hipLaunchKernelGGL((mfma_xtr_split_kernel<XT, NG, RL, CW, LW, MT, KS, PF, LD, NTX>),
                       dim3((unsigned)((a.p + WCOLS - 1) / WCOLS)), dim3(64 * (CW + LW)), 0, s, a);
    return hipGetLastError();
}

template <int XT, int NG, int RL, int CW, int LW, int MT, int LDF, bool NTX = false, int QC = 4>
hipError_t launch_lds(const MfmaArgs& a, hipStream_t s)
{
    constexpr int WCOLS = 16 * MT * CW;
    hipLaunchKernelGGL((mfma_xtr_lds_kernel<XT, NG, RL, CW, LW, MT, LDF, NTX, QC>),
                       dim3((unsigned)((a.p + WCOLS - 1) / WCOLS)), dim3(64 * (CW + LW)), 0, s, a);
    return hipGetLastError();
}

// Shape 15's launch: the blocks of columns that fill whole rounds of resident
// workgroups run unsplit, and the rest (the last round's) are split KSPLIT ways.
template <int XT, int NG, int RL, int CW, int LW, int MT, int LDF, bool NTX, int QC, int KSPLIT>
hipError_t launch_lds_tail(const MfmaArgs& a, hipStream_t s)
{
    constexpr int WCOLS = 16 * MT * CW;
    const void* fn = reinterpret_cast<const void*>(&mfma_xtr_lds_kernel<XT, NG, RL, CW, LW, MT, LDF, NTX, QC, KSPLIT>);
    if (!a.tail || a.ncu < 1) return hipErrorInvalidValue;
    int per_cu = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * (CW + LW), 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int64_t nblk = (a.p + WCOLS - 1) / WCOLS, slots = (int64_t)a.ncu * per_cu;
    const int64_t ntail = nblk % slots;
    MfmaArgs b = a;
    b.nfull = nblk - ntail;
    const int64_t j0 = b.nfull * WCOLS, ptail = a.p - j0;
    if (ntail > 0 && ptail > a.tail_cols) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mfma_xtr_lds_kernel<XT, NG, RL, CW, LW, MT, LDF, NTX, QC, KSPLIT>),
                       dim3((unsigned)(b.nfull + KSPLIT * ntail)), dim3(64 * (CW + LW)), 0, s, b);
    if (ntail > 0)
        hipLaunchKernelGGL(xtr_tail_kernel, dim3((unsigned)((a.B * ptail + kT - 1) / kT)), dim3(kT), 0, s, b, KSPLIT,
                           j0, ptail);
    return hipGetLastError();
}

template <int XT, int NG, int RL>
hipError_t launch_ng(const MfmaArgs& a, hipStream_t s)
{
    switch (a.variant) {
    case 5: return launch_split<XT, NG, RL, 7, 1, 3, 1, 6, 3>(a, s);
    case 6: return launch_split<XT, NG, RL, 7, 1, 3, 1, 4, 4>(a, s);
    case 7: return launch_split<XT, NG, RL, 6, 2, 3, 1, 6, 3>(a, s);
    case 8: return launch_lds<XT, NG, RL, 4, 4, 4, 3>(a, s);
    case 9: return launch_lds<XT, NG, RL, 4, 4, 4, 4>(a, s);
    case 10: return launch_lds<XT, NG, RL, 4, 4, 4, 5>(a, s);
    case 11: return launch_lds<XT, NG, RL, 8, 4, 2, 4>(a, s);
    case 12: return launch_lds<XT, NG, RL, 8, 4, 2, 3>(a, s);
    case 13: return launch_lds<XT, NG, RL, 4, 4, 4, 2, false, 8>(a, s);
    case 14: return launch_lds<XT, NG, RL, 4, 4, 4, 2, true, 8>(a, s);
    case 15: return launch_lds_tail<XT, NG, RL, 4, 4, 4, 2, true, 8, 3>(a, s);
    case 1: return launch_split<XT, NG, RL, 7, 1, 3, 1, 4>(a, s);
    case 2: return launch_split<XT, NG, RL, 6, 2, 3, 1, 6>(a, s);
    case 3: return launch_split<XT, NG, RL, 6, 2, 3, 1, 4>(a, s);
    case 4: return launch_split<XT, NG, RL, 6, 2, 3, 2, 2>(a, s);
    default: return launch_split<XT, NG, RL, 7, 1, 3, 1, 6>(a, s);
    }
}

template <int XT, int RL>
hipError_t launch_rl(const MfmaArgs& a, hipStream_t s)
{
    switch (a.bpad / 16) {
    case 1: return launch_ng<XT, 1, RL>(a, s);
    case 2: return launch_ng<XT, 2, RL>(a, s);
    case 3: return launch_ng<XT, 3, RL>(a, s);
    default: return launch_ng<XT, 4, RL>(a, s);
    }
}

template <int XT>
hipError_t launch_xt(const MfmaArgs& a, hipStream_t s)
{
    return a.limbs_n == 2 ? launch_rl<XT, 2>(a, s) : launch_rl<XT, 3>(a, s);
}

}  // namespace

int mfma_ntile(int64_t n) { return (int)((n + 4095) / 4096); }

hipError_t launch_quantize(const double* r64, int64_t n, int B, double* rmaxp, long long* rsump, int8_t* limbs,
                           int64_t lstride, int bpad, int nlimb, double* qscale, double* sumr, hipStream_t s)
{
    if (lstride % 256 || lstride < n || bpad < B || bpad % 16 || (nlimb != 2 && nlimb != 3))
        return hipErrorInvalidValue;
    const int nt = mfma_ntile(n);
    hipLaunchKernelGGL(rmax_kernel, dim3(nt, B), dim3(kT), 0, s, r64, n, rmaxp, nt);
    hipLaunchKernelGGL(quantize_kernel, dim3(nt, B), dim3(kT), 0, s, r64, n, rmaxp, nt, limbs, bpad, nlimb, qscale,
                       rsump);
    hipLaunchKernelGGL(rsum_kernel, dim3(1), dim3(64), 0, s, rsump, nt, qscale, sumr, B);
    return hipGetLastError();
}

hipError_t launch_quantize_d(const double* dcoef, int64_t p, const int32_t* sel, const int32_t* nsel, int B,
                             double* dmaxp, int8_t* dlimbs, int64_t dstride, int bpad, double* dscale,
                             hipStream_t s)
{
    if (dstride % 64 || dstride < p || bpad < B || bpad % 16) return hipErrorInvalidValue;
    const int nt = (int)((p + 63) / 64 * 64 + 4095) / 4096;
    hipLaunchKernelGGL(dmax_kernel, dim3(nt, B), dim3(kT), 0, s, dcoef, p, sel, nsel, dmaxp, nt);
    hipLaunchKernelGGL(dquant_kernel, dim3(nt, B), dim3(kT), 0, s, dcoef, p, sel, nsel, dmaxp, nt, dlimbs, bpad,
                       dscale);
    return hipGetLastError();
}

hipError_t launch_mfma_eta(const MfmaEtaArgs& a, hipStream_t s)
{
    if (a.bpad < 16 || a.bpad > 64 || a.bpad % 16 || a.B > a.bpad || a.dstride % 64 || a.dstride < a.p)
        return hipErrorInvalidValue;
    return a.xt == XT_FP8 ? launch_eta_xt<XT_FP8>(a, s) : launch_eta_xt<XT_I8>(a, s);
}

hipError_t launch_mfma_xtr(const MfmaArgs& a, hipStream_t s)
{
    if (a.bpad < 16 || a.bpad > 64 || a.bpad % 16 || a.B > a.bpad || a.lstride % 256 || a.lstride < a.n ||
        (a.limbs_n != 2 && a.limbs_n != 3))
        return hipErrorInvalidValue;
    return a.xt == XT_FP8 ? launch_xt<XT_FP8>(a, s) : launch_xt<XT_I8>(a, s);
}

hipError_t launch_geno_check(const void* X, int xt, int64_t n, int64_t p, int64_t ldx, int* bad, hipStream_t s)
{
    if (xt == XT_FP8)
        hipLaunchKernelGGL(geno_check_kernel<XT_FP8>, dim3((unsigned)p), dim3(kT), 0, s,
                           static_cast<const uint8_t*>(X), n, ldx, bad);
    else
        hipLaunchKernelGGL(geno_check_kernel<XT_I8>, dim3((unsigned)p), dim3(kT), 0, s,
                           static_cast<const uint8_t*>(X), n, ldx, bad);
    return hipGetLastError();
}

}  // namespace cox
