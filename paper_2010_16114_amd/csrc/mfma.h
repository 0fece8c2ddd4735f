// mfma.h -- interface of the batched int8 matrix-core pass (mfma.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cox {

// Row of the 16x16 accumulator tile held by vector register v of lane `lane`
// for v_mfma_i32_16x16x64_i8 (the column is lane & 15).
__host__ __device__ constexpr int mfma_c_row(int lane, int v) { return 4 * (lane >> 4) + v; }

struct MfmaArgs {
    const void* X;          // column-major allele counts (int8 or FP8 E4M3 codes)
    int xt;                 // XT_I8 or XT_FP8
    int64_t n, p, ldx;      // ldx % 16 == 0, X 16-byte aligned
    const int8_t* limbs;    // [lstride / 16][limbs_n * bpad][16] residual limbs by 16-subject chunk,
                            // limb-major within a chunk (column limb * bpad + b); rows n .. round_up(n, 256)
                            // zero
    int64_t lstride;        // subject rows the limb buffer holds: a multiple of 256, >= n
    int bpad;               // 16, 32, 48 or 64
    int limbs_n;            // residual limbs: 3 (|R| <= 2^22) or 2 (|R| <= 2^14)
    int B;                  // vectors written (<= bpad)
    const double* qscale;   // [B] quantisation step of each vector
    double* out;            // [B][p] raw sums q_b * sum_i g_ij R_bi
    int variant;            // pipeline shape (compute + loader wavefronts, M tiles per compute
                            // wavefront, subjects per stage, stages ahead): 0 = 7+1, 3, 64, 6;
                            // 1 = 7+1, 3, 64, 4; 2 = 6+2, 3, 64, 6; 3 = 6+2, 3, 64, 4; 4 = 6+2, 3, 128, 2
                            // (limb loads two stages ahead); with limb loads three or four stages
                            // ahead: 5 = 7+1, 3, 64, 6, 3; 6 = 7+1, 3, 64, 4, 4; 7 = 6+2, 3, 64, 6, 3;
                            // X through LDS as well, loaded by the loader wavefronts (compute +
                            // loader wavefronts, M tiles, stages of loads in flight): 8 = 4+4, 4, 3;
                            // 9 = 4+4, 4, 4; 10 = 4+4, 4, 5; 11 = 8+4, 2, 4; 12 = 8+4, 2, 3; with
                            // stages of 128 subjects (a whole 128-byte line per column): 13 = 4+4, 4, 2;
                            // 14 = 13 with streaming (non-temporal) loads of X; 15 = 14 with the
                            // last, partly filled round of workgroups split three ways over subjects
    long long* tail = nullptr;  // shape 15: [3][B][tail_cols] exact sums of the split blocks
    int64_t tail_cols = 0;      // columns tail holds per (share, b): >= the split blocks' columns
    int ncu = 0;                // shape 15: compute units of the device
    int64_t nfull = 0;          // set by the launch: blocks of columns that run unsplit
};
constexpr int kMfmaVariants = 16;    // shapes of the X~' R pass
constexpr int kMfmaEtaVariants = 13;  // shapes of the eta update

// eta_b(i) += q_b * sum_{u < nsel} g(i, sel[u]) D_b(u), D in three int8 limbs.
struct MfmaEtaArgs {
    const void* X;
    int xt;
    int64_t n, p, ldx;      // ldx % 16 == 0, X 16-byte aligned
    const int32_t* sel;     // [nsel] changed columns, ascending
    const int32_t* nsel;    // device count
    const int8_t* dlimbs;   // [dstride / 16][3 * bpad][16] limbs of D by 16-position chunk of sel;
                            // positions nsel .. round_up(nsel, 64) zero
    int64_t dstride;        // positions the buffer holds: a multiple of 64, >= p
    int bpad, B;
    const double* dscale;   // [B]
    double* eta;            // [B][n] FP64, updated in place
    const int32_t* active;  // [B] or null
    int variant;            // pipeline shape.  One kernel, 8 wavefronts that load both operands,
                            // 2 stages of 64 columns ahead: 0 = D tile in 8-byte pieces when
                            // bpad = 64, 1 = in 16-byte chunks.  Loader and compute roles in separate
                            // wavefronts (compute + loader wavefronts, stages of loads in the
                            // loaders' ring, LDS buffers), one workgroup per 256 subjects:
                            // 2 = 4+4, 3, 2; 3 = 4+4, 4, 2; 4 = 8+4, 3, 2; 5 = 4+4, 5, 2;
                            // 6 = 2 with streaming loads of G; 7 = 8+4, 3, 3 (three buffers: the
                            // compute wavefronts read the next stage's fragments ahead).  The same
                            // with one workgroup per compute unit sharing the blocks evenly
                            // (sk_grid, part): 8 = 6; 9 = 2; 10 = 3 with streaming loads; 11 = 4
                            // with streaming loads; 12 = 5 with streaming loads
    long long* part;        // [sk_grid][2][bpad][256] partial sums of shared blocks (variants 8..12), or null
    int sk_grid;            // workgroups of variants 8..12: the compute units (0: one per block)
};

int mfma_ntile(int64_t n);
// D_b(u) = dcoef[b][sel[u]] -> dlimbs, dscale (per-b step max|D_b| / 2^22)
hipError_t launch_quantize_d(const double* dcoef, int64_t p, const int32_t* sel, const int32_t* nsel, int B,
                             double* dmaxp, int8_t* dlimbs, int64_t dstride, int bpad, double* dscale,
                             hipStream_t s);
hipError_t launch_mfma_eta(const MfmaEtaArgs& a, hipStream_t s);
// r64 [B][n] -> limbs, qscale [B], sumr [B] = q_b * sum_i R_bi
hipError_t launch_quantize(const double* r64, int64_t n, int B, double* rmaxp, long long* rsump, int8_t* limbs,
                           int64_t lstride, int bpad, int nlimb, double* qscale, double* sumr, hipStream_t s);
hipError_t launch_mfma_xtr(const MfmaArgs& a, hipStream_t s);
hipError_t launch_geno_check(const void* X, int xt, int64_t n, int64_t p, int64_t ldx, int* bad, hipStream_t s);

}  // namespace cox
