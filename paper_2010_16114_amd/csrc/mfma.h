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
    const int8_t* limbs;    // [3][bpad][lstride] residual limbs, zero beyond n
    int64_t lstride;        // multiple of 256
    int bpad;               // 16, 32, 48 or 64
    int B;                  // vectors written (<= bpad)
    const double* qscale;   // [B] quantisation step of each vector
    double* out;            // [B][p] raw sums q_b * sum_i g_ij R_bi
    int variant;            // pipeline shape (waves x M tiles per wave, subjects per stage, stages ahead):
                            // 0 = 4x3, 64, 8; 1 = 8x2, 64, 5; 2 = 8x2, 64, 6; 3 = 8x2, 128, 4;
                            // 4 = 8x2, 128, 3
};
constexpr int kMfmaVariants = 5;     // shapes of the X~' R pass
constexpr int kMfmaEtaVariants = 3;  // shapes of the eta update

// eta_b(i) += q_b * sum_{u < nsel} g(i, sel[u]) D_b(u), D in three int8 limbs.
struct MfmaEtaArgs {
    const void* X;
    int xt;
    int64_t n, p, ldx;      // ldx % 16 == 0, X 16-byte aligned
    const int32_t* sel;     // [nsel] changed columns, ascending
    const int32_t* nsel;    // device count
    const int8_t* dlimbs;   // [3][bpad][dstride] limbs of D by position in sel, zero past nsel
    int64_t dstride;        // multiple of 64, >= p
    int bpad, B;
    const double* dscale;   // [B]
    double* eta;            // [B][n] FP64, updated in place
    const int32_t* active;  // [B] or null
    int variant;            // stages (of 64 columns) ahead: 0 = 4, 1 = 3, 2 = 2
};

int mfma_ntile(int64_t n);
// D_b(u) = dcoef[b][sel[u]] -> dlimbs, dscale (per-b step max|D_b| / 2^22)
hipError_t launch_quantize_d(const double* dcoef, int64_t p, const int32_t* sel, const int32_t* nsel, int B,
                             double* dmaxp, int8_t* dlimbs, int64_t dstride, int bpad, double* dscale,
                             hipStream_t s);
hipError_t launch_mfma_eta(const MfmaEtaArgs& a, hipStream_t s);
// r64 [B][n] -> limbs, qscale [B], sumr [B] = q_b * sum_i R_bi
hipError_t launch_quantize(const double* r64, int64_t n, int B, double* rmaxp, long long* rsump, int8_t* limbs,
                           int64_t lstride, int bpad, double* qscale, double* sumr, hipStream_t s);
hipError_t launch_mfma_xtr(const MfmaArgs& a, hipStream_t s);
hipError_t launch_geno_check(const void* X, int xt, int64_t n, int64_t p, int64_t ldx, int* bad, hipStream_t s);

}  // namespace cox
