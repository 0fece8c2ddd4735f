// internal.h -- launch interfaces between the host runtime (api.cpp) and the
// HIP kernels of libcoxhip.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cox {

// Element storage of X.
enum XType : int { XT_F32 = 0, XT_FP8 = 1, XT_I8 = 2 };

// Geometry shared by kernels and the host.
constexpr int kGemvtThreads = 256;                  // 4 waves
constexpr int kGemvtCols = 16;                      // columns per change-list / l1 block
constexpr int kSplitRows = 8192;                    // row splits of X' r are multiples of this
constexpr int kRiskThreads = 1024;
constexpr int kUpdThreads = 256;                    // eta update: 4 rows per thread
constexpr int kUpdRows = 4 * kUpdThreads;
constexpr int kGemvThreads = 256;                   // dense GEMV
constexpr int kMaxHist = 33;                        // lag <= 32
constexpr int kCovRows = 8192;                      // rows per workgroup of Z' r
constexpr int kMaxCov = 64;                         // covariates in the dense block beside X
constexpr int kMaxRefit = 1024;                     // columns of an unpenalised refit
constexpr int kRefitRows = 8192;                    // rows per workgroup of the refit's D' r
constexpr int kGramChunks = 64;                     // most row chunks of a refit Gram term

// Read-only description of X as the kernels see it.
struct XDesc {
    const void* X;
    int xt;
    int64_t n, p, ldx;
    const float* center;  // may be null
    const float* scale;   // may be null
    int vec16;            // 16-byte loads legal: base and ldx*elem aligned to 16 bytes
    int vec4;             // 4-byte loads legal for 1-byte types
};

// Per-subject order and tie groups (sorted position k = 0 .. n-1).
struct Order {
    const int32_t* perm;    // subject at sorted position k
    const int32_t* gstart;  // first position of k's tie group
    const int32_t* gend;    // last position of k's tie group
    const uint8_t* ev;      // event indicator at sorted position k
};

// Convergence bookkeeping of cox_fit_path, one entry per b.
struct FitCtl {
    const double* lam;     // [B]
    const double* l1;      // [B][nblk] partial sums of |beta_k|
    int nblk;
    double* hist;          // [B][kMaxHist] ring of objective values
    int32_t* kit;          // [B] current step k
    int32_t* active;       // [B] 1 while b is iterating
    int32_t* iters;        // [B] steps taken at the stop
    int32_t* status;       // [B] 0 running, 1 converged, 2 max_iter, 3 non-finite
    double* fobj;          // [B] latest objective
    const double* l1cov;   // [B] penalised l1 of the covariate coefficients, or null
    int max_iter, lag;
    double tol;
    double* trace;         // [B][trace_stride] objective of every step, or null
    int64_t trace_stride;
};

struct RiskArgs {
    int64_t n;
    int B;
    Order ord;
    const void* eta_in;    // [B][n] original order; double unless eta_in_f32
    int eta_in_f32;
    double* eta;           // [B][n] FP64 eta after the partial updates are added (may equal eta_in)
    const double* part;    // [ncg][part_cstride] partial eta updates, or null
    int ncg;
    int64_t part_cstride;  // elements between column groups
    const int32_t* nsel;   // partials are added only when *nsel > 0
    double* w;             // [B][n] exp(eta - m), sorted order
    double* S;             // [B][n] cumulative sum of w within its tile, sorted order
    double* T;             // [B][n] reverse cumulative sum of delta/W within its tile
    int64_t tile;          // positions per scan tile (multiple of 1024)
    int ntile;             // ceil(n / tile) <= kMaxTiles
    int nfin;              // workgroups per b of the eta pass
    double* bmax;          // [B][nfin] partial maxima of eta
    double* mshift;        // [B] m = max eta
    double* stot;          // [B][ntile] tile totals of w
    double* qtot;          // [B][ntile] tile totals of delta/W
    double* Lpart;         // [B][ntile] tile sums of the log-likelihood terms
    double* rpart;         // [B][ntile] tile sums of r (as stored)
    float* r32;            // [B][rstride] residual, original order (nullable)
    int64_t rstride;
    double* r64;           // [B][n] residual, original order (nullable)
    double* L;             // [B] log partial likelihood
    double* sumr;          // [B] sum of the stored residual
    int use_ctl;           // 1 inside cox_fit_path
    FitCtl ctl;
};

constexpr int kMaxTiles = 4096;
constexpr int kFinElems = 512;   // eta elements per workgroup of the eta pass

enum GemvtMode : int { GT_RAW = 0, GT_GRAD = 1, GT_PROX = 2 };

struct GemvtArgs {
    XDesc x;
    const float* r32;      // [B][rstride], b-major; rows n..rstride-1 are zero
    int64_t rstride;       // multiple of kSplitRows
    double* part;          // [nsplit][Bmax][p] raw column sums of each row split
    int nsplit;
    int64_t split_rows;    // rows per split (multiple of kSplitRows)
    int64_t part_sstride;  // elements between splits (Bmax * p)
    const double* sumr;    // [B] (centring of genotype columns)
    int b0, nb;            // this launch covers b0 .. b0+nb-1 (nb <= template NB)
    int mode;
    double* out64;         // GT_RAW: [B][ostride]  X~' r (first p entries of each row)
    float* out32;          // GT_GRAD: [B][ostride]  -X~' r
    int64_t ostride;       // >= p
    // GT_PROX
    double* beta;          // [B][p] in/out
    const double* lam;     // [B]
    const double* pf;      // [p] penalty factors (threshold step * lam * pf_j), or null: all 1
    double step;
    const int32_t* active; // [B] or null (all active)
    double* dcoef;         // [B][p] (beta_new - beta_old) * scale_j
    int32_t* chg_flag;     // [p] 1 if beta_j changed for some b (ORed over launches)
    int32_t* chg_cnt;      // [nblk] changed columns per 16-column block
    int32_t* chg_idx;      // [nblk][kGemvtCols] their indices, ascending
    double* l1old;         // [B][nblk]
    double* l1new;         // [B][nblk]
    int nblk;
    int first_group;       // 1 on the launch with b0 == 0: it resets the change lists
};

// cox_fit_path as one persistent launch (persist.hip): the vector path (B <=
// 8, active-set eta update, no covariate block, 16-byte loads legal).  Each
// step runs the phases of the multi-launch form -- eta update (from the second
// step), the five risk-set phases with the stopping rule, X~' r with the
// proximal epilogue, the change-list compaction -- over a grid of co-resident
// workgroups separated by grid-wide barriers, with the same per-workgroup code
// and therefore the same arithmetic; the loop ends when every b has stopped.
struct PersistArgs {
    RiskArgs ra;           // use_ctl = 1; part = the eta partials
    GemvtArgs g;           // GT_PROX, b0 = 0, nb = B, first_group = 1
    const int32_t* sel;    // change list (compacted), device count nsel
    int32_t* sel_w;        // the same buffer, written by the compaction
    int32_t* nsel;
    const double* dcoef;   // [B][p] coefficient changes times the genotype scale
    double* part_upd;      // [ncg][Bmax][n] eta partials
    int64_t cstride;       // Bmax * n
    int ncg;
    int max_iter;
    int B;
};
// words: persist_barrier_words() device words zeroed before the launch (the
// barrier's arrival counter, abort flag -- word persist_abort_word() -- and
// generation words); limit_s: the longest wait at one barrier before the
// launch is abandoned (abort flag set to 1).  grid_out: workgroups launched
// (co-resident, from the kernel's occupancy).
int persist_barrier_words();
constexpr int persist_abort_word() { return 32; }
hipError_t launch_fit_persistent(const PersistArgs& a, unsigned long long* words, double limit_s, hipStream_t s,
                                 int* grid_out);

// Launchers (return hipError_t of the launch).
hipError_t launch_risk(const RiskArgs& a, hipStream_t s);
hipError_t launch_gemvt(const GemvtArgs& a, hipStream_t s);       // sums, then epilogue
hipError_t launch_gemvt_sums(const GemvtArgs& a, hipStream_t s);  // the row-split column sums alone
// the epilogue alone, on column sums already in a.part (nb may exceed 8)
hipError_t launch_gemvt_epilogue(const GemvtArgs& a, hipStream_t s);
// eta partials: part[cg][b][i] for b in [b0, b0+nb) from the compacted change list
hipError_t launch_eta_update(const XDesc& x, const int32_t* sel, const int32_t* nsel, const double* dcoef,
                             int b0, int nb, double* part, int64_t part_cstride, int ncg,
                             const int32_t* active, hipStream_t s);
// column blocks of the dense pass over one-byte X with 16-byte runs (the
// partial buffer must hold gemv16_blocks(n, p) * 4 * n doubles)
int gemv16_blocks(int64_t n, int64_t p);
// dense eta = X~ coef for b in [b0, b0+nb): partials over column blocks, then reduced
hipError_t launch_gemv(const XDesc& x, const double* coef, int b0, int nb, double* part, int ncb,
                       double* eta, const double* shift, hipStream_t s);
hipError_t launch_compact(const int32_t* chg_cnt, const int32_t* chg_idx, int nblk, int32_t* sel,
                          int32_t* nsel, hipStream_t s);
// misc elementwise / reductions
hipError_t launch_f32_to_f64(const float* in, double* out, int64_t m, hipStream_t s);
hipError_t launch_f64_to_f32(const double* in, float* out, int64_t m, hipStream_t s);
hipError_t launch_scale_coef(const double* beta, const float* scale, double* coef, int64_t p, int B,
                             hipStream_t s);
// l1[b][blk] = sum over the block's columns of pf_j |beta_bj| (pf null: 1)
hipError_t launch_l1_blocks(const double* beta, const double* pf, int64_t p, int B, int nblk, double* l1,
                            hipStream_t s);
// beta <- S_{step lam_b pf_j}(beta - step grad), pf null: 1
hipError_t launch_prox_apply(float* beta, const float* grad, const double* lam, const double* pf, double step,
                             int64_t p, int B, hipStream_t s);
hipError_t launch_nll_backward(const double* r64, const double* gl, int64_t n, int B, void* out, int out_f64,
                               hipStream_t s);
// Two-level reductions: part holds kRedParts doubles of scratch (contiguous
// chunks summed by separate workgroups, then added in order by one), so the
// result depends only on the length.
constexpr int kRedParts = 256;
// out[0] = sum_i a_i * (b ? b_i : 1) over m entries
hipError_t launch_dot(const double* a, const double* b, int64_t m, double* part, double* out, hipStream_t s);
// out[0] = -sum_j center_j * scale_j * v_j  (centring shift of X~ v)
hipError_t launch_center_shift(const float* center, const float* scale, const double* v, int64_t p, double* part,
                               double* out, hipStream_t s);
// out[j] = in[j] / sqrt(nrm2[0]) * (scale ? scale_j : 1) and vout[j] = in[j] / sqrt(nrm2[0])
hipError_t launch_normalize(const double* in, const double* nrm2, const float* scale, double* vout, double* coef,
                            int64_t p, hipStream_t s);
// r32[i] = (float) u[i] + shift[0]; sumr[0] = sum (double) r32[i] (part: as for launch_dot)
hipError_t launch_to_r32(const double* u, const double* shift, float* r32, double* sumr, int64_t n, double* part,
                         hipStream_t s);
// out[b] = a * sum_i in[b*m + i], one workgroup per b, fixed order
hipError_t launch_rowsum(const double* in, int64_t m, int B, double a, double* out, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t m, hipStream_t s);
// status 2 -> 0, active -> 1, kit = iters + 1 for b < B (B <= 64): a resumed fit
hipError_t launch_resume(int32_t* status, int32_t* active, int32_t* kit, const int32_t* iters, int B,
                         hipStream_t s);
// acc[0] += v[0]
hipError_t launch_count_add(const int32_t* v, long long* acc, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t m, hipStream_t s);
// p[i] = i for i < m
hipError_t launch_iota_i32(int32_t* p, int64_t m, hipStream_t s);
// flag[b] = 1 if coef[b*p + j] is not finite for some j < p (b < B; flags cleared beforehand)
hipError_t launch_nonfinite(const double* coef, int64_t p, int B, int32_t* flag, hipStream_t s);
// eta[b*n + i] = NaN for i < n, for each b < B with flag[b] set
hipError_t launch_poison_eta(double* eta, int64_t n, int B, const int32_t* flag, hipStream_t s);
// dst[b*p + j] = src[b*p + j] - dscale[b] * llrint(src[b*p + j] / dscale[b]) for b < B, j < p
// (src == dst allowed): what the eta update's D quantisation leaves of each entry
hipError_t launch_coef_remainder(const double* src, double* dst, int64_t p, int B, const double* dscale,
                                 hipStream_t s);

// ---- the dense covariate block Z beside X (covar.hip)
struct CovArgs {
    const float* Z;        // column-major n x q, column k at Z + k * ldz
    int64_t n, ldz;
    int q;                 // 1 .. kMaxCov
    int nrb;               // cov_row_blocks(n)
    double* part;          // [B][nrb][q] partial sums of Z' r
};

struct CovStep {
    int mode;              // GemvtMode
    double* out64;         // [B][ostride] g_Z, or null
    float* out32;          // GT_GRAD: [B][ostride] -g_Z
    int64_t ostride;
    // GT_PROX
    double* beta;          // [B][q] in/out
    double* dbeta;         // [B][q] new - old
    const double* lam;     // [B]
    const double* pf;      // [q]
    double step;
    const int32_t* active; // [B] or null
    double* l1old;         // [B] sum_k pf_k |beta_k| before
    double* l1new;         // [B] and after
};

int cov_row_blocks(int64_t n);
// partial sums of Z' r for b < B; the residual is r32 ([B][rstride]) or r64 ([B][n])
hipError_t launch_cov_xtr(const CovArgs& c, const float* r32, int64_t rstride, const double* r64, int B,
                          const int32_t* active, hipStream_t s);
hipError_t launch_cov_epilogue(const CovArgs& c, const CovStep& st, int B, hipStream_t s);
// eta_b += Z coef_b for b < B (coef [B][q]) unless active[b] == 0
hipError_t launch_cov_eta(const CovArgs& c, const double* coef, int B, double* eta, const int32_t* active,
                          hipStream_t s);
hipError_t launch_cov_l1(const double* beta, const double* pf, int q, int B, double* l1, hipStream_t s);
// [B][p + q] FP32 <-> [B][p] and [B][q] FP64
hipError_t launch_split_coef(const float* in, int64_t p, int64_t q, int B, double* x64, double* z64, hipStream_t s);
hipError_t launch_merge_coef(const double* x64, const double* z64, int64_t p, int64_t q, int B, float* out,
                             hipStream_t s);
// acc[0] += sum_k v_k^2
hipError_t launch_sqnorm_add(const double* v, int q, double* acc, hipStream_t s);

// ---- the unpenalised refit on chosen columns (refit.hip)
// leading dimension of the refit's tall arrays: rows rounded up to 8 (at least 8)
int64_t refit_ld(int64_t rows);
// D[a][k] = x~(perm[k], cols[a]) as FP32 for a < m, k < x.n (sorted order), 0 up
// to ldd >= refit_ld(x.n)
hipError_t launch_gather_cols(const XDesc& x, const int32_t* cols, int m, const int32_t* perm, float* D, int64_t ldd,
                              hipStream_t s);
// D[a][k] = Z[a][perm[k]] for a < q (Z column-major, ldz), 0 past n
hipError_t launch_gather_z(const float* Z, int64_t ldz, int64_t n, int q, const int32_t* perm, float* D, int64_t ldd,
                           hipStream_t s);
// eta[perm[k]] = sum_a D[a][k] b[a] over M columns
hipError_t launch_refit_eta(const float* D, int64_t ldd, int64_t n, int M, const int32_t* perm, const double* b,
                            double* eta, hipStream_t s);
int refit_row_blocks(int64_t n);
// g = D' r with r in subject order (rs [n]: r in sorted order, written;
// part: [refit_row_blocks(n)][M] scratch)
hipError_t launch_refit_grad(const float* D, int64_t ldd, int64_t n, int M, const int32_t* perm, const double* r,
                             double* rs, double* part, double* g, hipStream_t s);
// row chunks of a Gram term over `rows` rows and M columns; risk-set scan chunks
int gram_chunks(int64_t rows, int M);
int scan_chunks(int64_t n);
// H = -Hessian of L in the M coefficients (M x M, row-major) at the risk-set
// state (w sorted, r in subject order).  egidx [n]: event group of each sorted
// position that ends a tie group with events, else -1; egcnt [G]: its events.
struct RefitHess {
    const float* D;
    int64_t ldd, n;
    int M;
    const int32_t* perm;
    const uint8_t* ev;
    const double* w;
    const double* r;
    const int32_t* egidx;
    const int32_t* egcnt;
    int64_t G, ldp;
    double* wt;     // [ldd]
    double* csum;   // [M + 1][scan_chunks(n)]
    double* P;      // [M + 1][ldp], ldp >= refit_ld(G)
    double* wg;     // [ldp]
    double* part1;  // [gram_chunks(n, M)][M][M]
    double* part2;  // [gram_chunks(G, M)][M][M]
    double* H;      // [M][M]
};
hipError_t launch_refit_hessian(const RefitHess& h, hipStream_t s);
// A = L L' in place (lower triangle), ok[0] = 1 if positive definite
hipError_t launch_chol(double* A, int M, int* ok, hipStream_t s);
hipError_t launch_chol_solve(const double* L, int M, const double* g, double* x, hipStream_t s);
// se = sqrt(diag((L L')^{-1})), pval = erfc(|b / se| / sqrt 2)
hipError_t launch_wald(const double* L, int M, const double* b, double* se, double* pval, hipStream_t s);
hipError_t launch_axpy(const double* b, const double* d, double t, int M, double* out, hipStream_t s);
// entry[j] = first l with path[l][j] != 0 (-1: never), coef[j] = |path[entry[j]][j]|, j < p
hipError_t launch_entry(const float* path, int L, int64_t ptot, int64_t p, int32_t* entry, float* coef, hipStream_t s);

}  // namespace cox
