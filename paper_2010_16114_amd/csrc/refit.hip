// refit.hip -- the unpenalised Cox refit on a chosen set of columns.
//
// Section 6 ranks the SNPs that the lasso path selects, then refits the
// unpenalised Cox model on them together with the covariates and keeps those
// whose Wald p-value passes a Bonferroni threshold.  The refit here is
// Newton's method on L over the M chosen columns, gathered into a dense FP32
// block D (M columns of ldd rows, rows in the sorted order of the times,
// zero past n; genotype columns standardised as (g - mu_j) s_j, formed in FP64
// and rounded once).
//
// With w = exp(eta - max eta), r = delta - w c (the risk-set pass), and in the
// sorted order S1(k) = sum_{k' <= k} w_k' d_k' (the risk-set sums of the rows
// of D), the negative Hessian of L in the coefficients is
//     -H = sum_i w_i c_i d_i d_i'  -  sum_G n_G S1(G) S1(G)' / W(G)^2
// where the first sum runs over subjects (w_i c_i = delta_i - r_i) and the
// second over tie groups G with n_G > 0 events, read at the group's last
// sorted position (Breslow).  Both terms are Gram matrices of tall arrays: D
// with row weights delta - r, and P with one row S1(G) per event group and
// row weights n_G / W(G)^2.  They are formed on the FP64 matrix cores from
// fixed-order partial sums.  -H is factorised by a blocked Cholesky; the Newton direction
// and the diagonal of (-H)^{-1} (squared standard errors) come from blocked
// triangular solves with that factor.
#include "device_common.h"

namespace cox {
namespace {

constexpr int kT = 256;
constexpr int kGT = 64;          // Gram output tile (kGT x kGT), one 16-row band per wavefront
constexpr int kGR = 32;          // row chunks of the Gram kernel start on multiples of this
constexpr int kScanChunk = 4096; // sorted positions per workgroup of the risk-set scans
constexpr int kCB = 32;          // block size of the Cholesky factorisation and the triangular solves

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ double block_sum256(double v, double* sh)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kT / kWave; ++q) s += sh[q];
    return s;
}

// D[a][k] = x~(perm[k], cols[a]) for k < n, 0 for n <= k < ldd
__global__ __launch_bounds__(kT) void gather_kernel(XDesc x, const int32_t* __restrict__ cols,
                                                    const int32_t* __restrict__ perm, float* __restrict__ D,
                                                    int64_t ldd)
{
    const int a = blockIdx.y;
    const int64_t j = cols[a];
    double mu = 0.0, sc = 1.0;
    if (x.xt != XT_F32) {
        if (x.center) mu = x.center[j];
        if (x.scale) sc = x.scale[j];
    }
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < ldd; k += (int64_t)gridDim.x * kT) {
        double v = 0.0;
        if (k < x.n) {
            const int64_t off = j * x.ldx + perm[k];
            if (x.xt == XT_F32)
                v = load_x1<XT_F32>(x.X, off);
            else if (x.xt == XT_FP8)
                v = ((double)load_x1<XT_FP8>(x.X, off) - mu) * sc;
            else
                v = ((double)load_x1<XT_I8>(x.X, off) - mu) * sc;
        }
        D[(int64_t)a * ldd + k] = (float)v;
    }
}

// D[a][k] = Z[a][perm[k]] for k < n, 0 for n <= k < ldd (Z column-major, ldz)
__global__ __launch_bounds__(kT) void gather_z_kernel(const float* __restrict__ Z, int64_t ldz, int64_t n,
                                                      const int32_t* __restrict__ perm, float* __restrict__ D,
                                                      int64_t ldd)
{
    const int a = blockIdx.y;
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < ldd; k += (int64_t)gridDim.x * kT)
        D[(int64_t)a * ldd + k] = k < n ? Z[(int64_t)a * ldz + perm[k]] : 0.0f;
}

// eta[perm[k]] = sum_a D[a][k] b[a]  (eta in subject order)
__global__ __launch_bounds__(kT) void refit_eta_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                       const int32_t* __restrict__ perm,
                                                       const double* __restrict__ b, double* __restrict__ eta)
{
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < n; k += (int64_t)gridDim.x * kT) {
        double s = 0.0;
        for (int a = 0; a < M; ++a) s += (double)D[(int64_t)a * ldd + k] * b[a];
        eta[perm[k]] = s;
    }
}

// rs[k] = r[perm[k]]: the residuals in the sorted order
__global__ void sort_r_kernel(const int32_t* __restrict__ perm, const double* __restrict__ r, int64_t n,
                              double* __restrict__ rs)
{
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < n; k += (int64_t)gridDim.x * kT) rs[k] = r[perm[k]];
}

// part[rb][a] = sum over row block rb of D[a][k] rs[k]
__global__ __launch_bounds__(kT) void refit_xtr_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                       const double* __restrict__ rs, int64_t rows,
                                                       double* __restrict__ part)
{
    __shared__ double sh[kT / kWave];
    const int a = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * rows, i1 = min(n, i0 + rows);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kT) s += (double)D[(int64_t)a * ldd + i] * rs[i];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * M + a] = s;
}

// g[a] = sum_rb part[rb][a], in row-block order
__global__ void refit_sum_kernel(const double* __restrict__ part, int nrb, int M, double* __restrict__ g)
{
    const int a = blockIdx.x * kT + threadIdx.x;
    if (a >= M) return;
    double s = 0.0;
    for (int rb = 0; rb < nrb; ++rb) s += part[(int64_t)rb * M + a];
    g[a] = s;
}

// row weights of the first Hessian term in the sorted order: wt[k] = delta - r
// of subject perm[k] for k < n, 0 for n <= k < ldd
__global__ void hess_weight_kernel(const int32_t* __restrict__ perm, const uint8_t* __restrict__ ev,
                                   const double* __restrict__ r, int64_t n, int64_t ldd, double* __restrict__ wt)
{
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < ldd; k += (int64_t)gridDim.x * kT)
        wt[k] = k < n ? (ev[k] ? 1.0 : 0.0) - r[perm[k]] : 0.0;
}

constexpr int kScanJ = kScanChunk / (4 * kT);  // sub-blocks of 4 kT positions in a scan chunk

// v[j][e] = w[k] D[a][k] (or w[k] with Dcol null) and g[j][e] = egidx[k]
// (when egidx is given) at position k = k0 + 4 kT j + 4 t + e of thread t:
// consecutive threads read consecutive 16-byte pieces.  0 (and g = -1) at or
// past n.  k0 is a multiple of 4 kT, ldd of 8.
__device__ __forceinline__ void scan_load(const float* __restrict__ Dcol, const double* __restrict__ w,
                                          const int32_t* __restrict__ egidx, int64_t k0, int64_t n,
                                          double (*v)[4], int32_t (*g)[4])
{
#pragma unroll
    for (int j = 0; j < kScanJ; ++j) {
        const int64_t kb = k0 + 4 * kT * j + 4 * (int64_t)threadIdx.x;
        if (kb + 4 <= n) {
            const double2 x0 = *reinterpret_cast<const double2*>(w + kb);
            const double2 x1 = *reinterpret_cast<const double2*>(w + kb + 2);
            v[j][0] = x0.x, v[j][1] = x0.y, v[j][2] = x1.x, v[j][3] = x1.y;
            if (Dcol) {
                const float4 d = *reinterpret_cast<const float4*>(Dcol + kb);
                v[j][0] *= (double)d.x, v[j][1] *= (double)d.y, v[j][2] *= (double)d.z, v[j][3] *= (double)d.w;
            }
            if (egidx) {
                const int4 q = *reinterpret_cast<const int4*>(egidx + kb);
                g[j][0] = q.x, g[j][1] = q.y, g[j][2] = q.z, g[j][3] = q.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = kb + e;
                v[j][e] = k < n ? (Dcol ? w[k] * (double)Dcol[k] : w[k]) : 0.0;
                if (egidx) g[j][e] = k < n ? egidx[k] : -1;
            }
        }
    }
}

// csum[a][ch] = sum over chunk ch's sorted positions k of w[k] D[a][k] (a < M)
// or of w[k] (a == M)
__global__ __launch_bounds__(kT) void chunk_sum_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                       const double* __restrict__ w, int nch,
                                                       double* __restrict__ csum)
{
    __shared__ double sh[kT / kWave];
    const int ch = blockIdx.x, a = blockIdx.y;
    double v[kScanJ][4];
    scan_load(a < M ? D + (int64_t)a * ldd : nullptr, w, nullptr, (int64_t)ch * kScanChunk, n, v, nullptr);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kScanJ; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) s += v[j][e];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) csum[(int64_t)a * nch + ch] = s;
}

// The prefix sums at the event groups: with P_a(k) = sum_{k' <= k} w[k'] D[a][k']
// (a < M) and P_M(k) = sum_{k' <= k} w[k'] in the sorted order, P[a][g] =
// P_a(k) at the last position k of event group g (egidx[k] = g; -1 at every
// other position).  Workgroup (ch, a) scans chunk ch of column a, starting
// from the sums of the earlier chunks: each thread's 4 positions in each
// sub-block are summed in place, every sub-block is scanned across the
// wavefront, and one exchange of the wavefront totals places them.  Chunk 0
// also clears P's padding rows G .. ldp - 1.
__global__ __launch_bounds__(kT) void scan_p_kernel(const float* __restrict__ D, int64_t ldd, int64_t n, int M,
                                                    const double* __restrict__ w, const double* __restrict__ csum,
                                                    int nch, const int32_t* __restrict__ egidx, int64_t G,
                                                    int64_t ldp, double* __restrict__ P)
{
    constexpr int NW = kT / kWave;
    __shared__ double sv[kScanJ][NW], sh[NW];
    const int ch = blockIdx.x, a = blockIdx.y;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t k0 = (int64_t)ch * kScanChunk;
    double v[kScanJ][4];
    int32_t g[kScanJ][4];
    scan_load(a < M ? D + (int64_t)a * ldd : nullptr, w, egidx, k0, n, v, g);
    double cv = 0.0;
    for (int c = threadIdx.x; c < ch; c += kT) cv += csum[(int64_t)a * nch + c];
    cv = block_sum256(cv, sh);
    double* Pa = P + (int64_t)a * ldp;
    if (ch == 0 && threadIdx.x < ldp - G) Pa[G + threadIdx.x] = 0.0;
    double iv[kScanJ];
#pragma unroll
    for (int j = 0; j < kScanJ; ++j) {
#pragma unroll
        for (int e = 1; e < 4; ++e) v[j][e] += v[j][e - 1];
        iv[j] = wave_incl_scan(v[j][3], lane);
        if (lane == kWave - 1) sv[j][wid] = iv[j];
    }
    __syncthreads();
    double before = cv;  // the earlier chunks and sub-blocks
#pragma unroll
    for (int j = 0; j < kScanJ; ++j) {
        // plus the earlier wavefronts of this sub-block and the earlier lanes
        double bv = before + iv[j] - v[j][3];
        for (int q = 0; q < wid; ++q) bv += sv[j][q];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (g[j][e] >= 0) Pa[g[j][e]] = bv + v[j][e];
        for (int q = 0; q < NW; ++q) before += sv[j][q];
    }
}

// Row weights of the second Hessian term: wg[g] = n_G / W(G)^2 with W(G) =
// P[M][g], so that sum_g wg[g] P_a(g) P_b(g) = sum_G n_G S1_a S1_b / W^2; 0 on
// the padding rows G .. ldp - 1.
__global__ void event_weight_kernel(const double* __restrict__ PM, const int32_t* __restrict__ egcnt, int64_t G,
                                    int64_t ldp, double* __restrict__ wg)
{
    for (int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x; g < ldp; g += (int64_t)gridDim.x * kT) {
        double v = 0.0;
        if (g < G) {
            const double W = PM[g];
            v = (double)egcnt[g] / (W * W);
        }
        wg[g] = v;
    }
}

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// GL consecutive values at p (16-byte aligned)
template <int GL>
__device__ __forceinline__ void load_seg(const float* p, float* o)
{
#pragma unroll
    for (int e = 0; e < GL; e += 4) {
        const float4 x = *reinterpret_cast<const float4*>(p + e);
        o[e] = x.x, o[e + 1] = x.y, o[e + 2] = x.z, o[e + 3] = x.w;
    }
}
template <int GL>
__device__ __forceinline__ void load_seg(const double* p, double* o)
{
#pragma unroll
    for (int e = 0; e < GL; e += 2) {
        const double2 x = *reinterpret_cast<const double2*>(p + e);
        o[e] = x.x, o[e + 1] = x.y;
    }
}

// part[chunk][a][b] = sum over the chunk's rows k of wt_k A[a][k] A[b][k] (wt
// nullable: 1) for the 64 x 64 output tile (ta, tb), ta <= tb, on the FP64
// matrix cores (v_mfma_f64_16x16x4f64; per lane A holds (row lane % 16, k
// lane / 16), B holds (k lane / 16, column lane % 16), D holds rows
// lane / 16 + 4 v of column lane % 16).  Each of the 4 / SW wavefronts owns
// SW bands of 16 rows of the tile and its 4 blocks of 16 columns, so a
// loaded B row serves SW products; in a diagonal tile the blocks left of a
// band are not stored (the reduction reads the upper triangle).  The rows are taken in steps of 4 GL: lane l loads
// rows GL q .. GL q + GL - 1 (q = l / 16) of its column straight from
// memory, and the s-th product of a step puts row GL q + s in k-slot q -- one
// permutation of the rows, shared by both operands, so every product pairs up
// as in the plain sum.  The next step's rows are loaded while the current
// ones are multiplied.  A is column-major (lda a multiple of 8, 0 past the
// rows, wt likewise); every chunk starts on a multiple of kGR (GL = 4 or 8).
template <class T, int GL, int SW>
__global__ __launch_bounds__(256 / SW) void gram_kernel(const T* __restrict__ A, int64_t lda, int64_t n, int M,
                                                        const double* __restrict__ wt, int64_t rows, int ntile,
                                                        double* __restrict__ part)
{
    int idx = blockIdx.x, ta = 0;
    while (idx >= ntile - ta) {
        idx -= ntile - ta;
        ++ta;
    }
    const int tb = ta + idx;
    const bool diag = ta == tb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, c = lane & 15, q = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.y * rows, r1 = min(n, r0 + rows);
    // columns past M are read from column M - 1: they only reach outputs that
    // are not stored
    const T* pa[SW];
#pragma unroll
    for (int u = 0; u < SW; ++u) pa[u] = A + (int64_t)min(ta * kGT + (wv * SW + u) * 16 + c, M - 1) * lda;
    const T* pb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) pb[t] = A + (int64_t)min(tb * kGT + t * 16 + c, M - 1) * lda;
    v4d acc[SW][4];
#pragma unroll
    for (int u = 0; u < SW; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[u][t] = v4d{0.0, 0.0, 0.0, 0.0};
    T na[SW][GL], nb[4][GL];
    double nw[GL];
    // a lane's segment at or past r1 is read at r0 with weight 0 (a segment
    // that starts before r1 ends before lda: r1 <= the rows, lda >= them
    // rounded up to 8)
    auto fetch = [&](int64_t s0) {
        const int64_t k = s0 + GL * q;
        const bool in = k < r1;
        const int64_t kl = in ? k : r0;
#pragma unroll
        for (int u = 0; u < SW; ++u) load_seg<GL>(pa[u] + kl, na[u]);
#pragma unroll
        for (int t = 0; t < 4; ++t) load_seg<GL>(pb[t] + kl, nb[t]);
        if (wt)
            load_seg<GL>(wt + kl, nw);
        else
#pragma unroll
            for (int e = 0; e < GL; ++e) nw[e] = 1.0;
#pragma unroll
        for (int e = 0; e < GL; ++e) nw[e] = in ? nw[e] : 0.0;
    };
    if (r0 < r1) fetch(r0);
    for (int64_t s0 = r0; s0 < r1; s0 += 4 * GL) {
        T cak[SW][GL], cbk[4][GL];
        double cwk[GL];
#pragma unroll
        for (int e = 0; e < GL; ++e) {
            cwk[e] = nw[e];
#pragma unroll
            for (int u = 0; u < SW; ++u) cak[u][e] = na[u][e];
#pragma unroll
            for (int t = 0; t < 4; ++t) cbk[t][e] = nb[t][e];
        }
        if (s0 + 4 * GL < r1) fetch(s0 + 4 * GL);
#pragma unroll
        for (int e = 0; e < GL; ++e) {
#pragma unroll
            for (int u = 0; u < SW; ++u) {
                const double av = (double)cak[u][e] * cwk[e];
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[u][t] = mfma_f64(av, (double)cbk[t][e], acc[u][t]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < SW; ++u) {
        const int band = wv * SW + u;  // 16-row band of the tile
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (diag && t < band) continue;  // below the diagonal: the reduction reads the mirror
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = ta * kGT + band * 16 + q + 4 * v, b = tb * kGT + t * 16 + c;
                if (a < M && b < M) part[((int64_t)blockIdx.y * M + a) * M + b] = acc[u][t][v];
            }
        }
    }
}

// H[a][b] = sum_c p1[c][a'][b'] - sum_c p2[c][a'][b'] with (a', b') = (min, max)
// of (a, b): the Gram kernel writes every entry of the upper triangle.
__global__ void gram_reduce_kernel(const double* __restrict__ p1, int nc1, const double* __restrict__ p2, int nc2,
                                   int M, double* __restrict__ H)
{
    const int64_t mm = (int64_t)M * M;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < mm; t += (int64_t)gridDim.x * kT) {
        const int a = (int)(t / M), b = (int)(t % M);
        const int64_t at = a <= b ? (int64_t)a * M + b : (int64_t)b * M + a;
        double s = 0.0;
        for (int c = 0; c < nc1; ++c) s += p1[c * mm + at];
        for (int c = 0; c < nc2; ++c) s -= p2[c * mm + at];
        H[t] = s;
    }
}

// Blocked right-looking Cholesky A = L L' of the symmetric positive definite
// M x M matrix (row-major; the lower triangle receives L, the upper one is
// left as it was), in blocks of kCB.  Step J runs chol_panel_kernel, then
// chol_update_kernel on the trailing lower blocks.

// Every workgroup factorises the diagonal block J in LDS (the same arithmetic
// in each); workgroup 0 stores it and the flag, workgroup b > 0 solves block
// row J + b of the panel, X L_JJ' = A_(J+b)J.  ok[0] = 1 after the first
// step, set to 0 by any step that meets a pivot that is not positive (the
// pivot is then taken as 1 and the factorisation runs on).
__global__ __launch_bounds__(kT) void chol_panel_kernel(double* __restrict__ A, int M, int J, int* __restrict__ ok)
{
    __shared__ double Ld[kCB][kCB + 1];
    __shared__ double P[kCB][kCB + 1];
    __shared__ int good;
    const int j0 = J * kCB, bs = min(kCB, M - j0);
    for (int e = threadIdx.x; e < kCB * kCB; e += kT) {
        const int r = e / kCB, c = e % kCB;
        Ld[r][c] = (r < bs && c < bs) ? A[(int64_t)(j0 + r) * M + j0 + c] : 0.0;
    }
    if (threadIdx.x == 0) good = 1;
    __syncthreads();
    for (int j = 0; j < bs; ++j) {
        const double d = Ld[j][j];
        const double piv = d > 0.0 ? sqrt(d) : 1.0;
        __syncthreads();
        if (threadIdx.x == 0) {
            if (!(d > 0.0)) good = 0;
            Ld[j][j] = piv;
        }
        if ((int)threadIdx.x > j && (int)threadIdx.x < bs) Ld[threadIdx.x][j] /= piv;
        __syncthreads();
        for (int e = threadIdx.x; e < kCB * kCB; e += kT) {
            const int i = e / kCB, k = e % kCB;
            if (k > j && k <= i && i < bs) Ld[i][k] -= Ld[i][j] * Ld[k][j];
        }
        __syncthreads();
    }
    if (blockIdx.x == 0) {
        for (int e = threadIdx.x; e < kCB * kCB; e += kT) {
            const int r = e / kCB, c = e % kCB;
            if (r < bs && c <= r) A[(int64_t)(j0 + r) * M + j0 + c] = Ld[r][c];
        }
        if (threadIdx.x == 0) {
            if (J == 0)
                ok[0] = good;
            else if (!good)
                ok[0] = 0;
        }
        return;
    }
    // a panel block exists only below a full diagonal block (bs == kCB)
    const int i0 = (J + blockIdx.x) * kCB, rs = min(kCB, M - i0);
    for (int e = threadIdx.x; e < kCB * kCB; e += kT) {
        const int r = e / kCB, c = e % kCB;
        P[r][c] = r < rs ? A[(int64_t)(i0 + r) * M + j0 + c] : 0.0;
    }
    __syncthreads();
    if ((int)threadIdx.x < rs) {
        const int r = threadIdx.x;
        double x[kCB];
#pragma unroll
        for (int c = 0; c < kCB; ++c) {
            double s = P[r][c];
#pragma unroll
            for (int c2 = 0; c2 < c; ++c2) s -= x[c2] * Ld[c][c2];
            x[c] = s / Ld[c][c];
        }
#pragma unroll
        for (int c = 0; c < kCB; ++c) P[r][c] = x[c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCB * kCB; e += kT) {
        const int r = e / kCB, c = e % kCB;
        if (r < rs) A[(int64_t)(i0 + r) * M + j0 + c] = P[r][c];
    }
}

// A_IK -= L_IJ L_KJ' for the trailing lower blocks J < K <= I (in a diagonal
// block only on and below the diagonal); one block per workgroup.
__global__ __launch_bounds__(kT) void chol_update_kernel(double* __restrict__ A, int M, int J)
{
    __shared__ double Pi[kCB][kCB + 1], Pk[kCB][kCB + 1];
    int64_t t = blockIdx.x;
    int ii = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)ii * (ii + 1) / 2 > t) --ii;
    while ((int64_t)(ii + 1) * (ii + 2) / 2 <= t) ++ii;
    const int kk = (int)(t - (int64_t)ii * (ii + 1) / 2);
    const int I = J + 1 + ii, K = J + 1 + kk, j0 = J * kCB;
    for (int e = threadIdx.x; e < kCB * kCB; e += kT) {
        const int r = e / kCB, c = e % kCB;
        const int ri = I * kCB + r, rk = K * kCB + r;
        Pi[r][c] = ri < M ? A[(int64_t)ri * M + j0 + c] : 0.0;
        Pk[r][c] = rk < M ? A[(int64_t)rk * M + j0 + c] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x >> 3;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int qq = 0; qq < kCB; ++qq) {
        const double pi = Pi[r][qq];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += pi * Pk[(threadIdx.x & 7) + 8 * u][qq];
    }
    const int row = I * kCB + r;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int cc = (threadIdx.x & 7) + 8 * u, col = K * kCB + cc;
        if (row < M && col < M && (I != K || cc <= r)) A[(int64_t)row * M + col] -= acc[u];
    }
}

__device__ __forceinline__ double bcast(double v, int src) { return __shfl(v, src, kWave); }

// Forward substitution L y = e on rows from block I0 on (L from the blocked
// Cholesky, y in LDS ys[], whose entries below I0 kCB are not read); e is g
// (rows i) or, with g null, the unit vector at row `unit`.  Per block: the
// known part of each row's sum with 8 threads per row, then the kCB x kCB
// diagonal block in one wavefront, lane r holding row r of it in registers.
__device__ void lower_solve(const double* __restrict__ L, int M, int I0, const double* __restrict__ g, int unit,
                            double* ys, double* red)
{
    const int nb = (M + kCB - 1) / kCB;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int I = I0; I < nb; ++I) {
        const int i0 = I * kCB, rb = min(kCB, M - i0);
        {
            const int r = threadIdx.x >> 3, s = threadIdx.x & 7;
            double part = 0.0;
            if (r < rb)
                for (int k = I0 * kCB + s; k < i0; k += 8) part += L[(int64_t)(i0 + r) * M + k] * ys[k];
            part += __shfl_xor(part, 1, kWave);
            part += __shfl_xor(part, 2, kWave);
            part += __shfl_xor(part, 4, kWave);
            if (s == 0) red[r] = part;
        }
        __syncthreads();
        if (wid == 0) {
            double b = 0.0, lr[kCB];
#pragma unroll
            for (int c = 0; c < kCB; ++c) lr[c] = (lane < rb && c <= lane) ? L[(int64_t)(i0 + lane) * M + i0 + c] : 0.0;
            if (lane < rb) b = (g ? g[i0 + lane] : (i0 + lane == unit ? 1.0 : 0.0)) - red[lane];
#pragma unroll
            for (int c = 0; c < kCB; ++c) {
                if (c < rb) {
                    const double yc = bcast(b / lr[c], c);
                    if (lane > c) b -= lr[c] * yc;
                    if (lane == c) b = yc;
                }
            }
            if (lane < rb) ys[i0 + lane] = b;
        }
        __syncthreads();
    }
}

// Back substitution L' x = y in place in ys[] (all M rows), the same blocking:
// the known part of each row's sum reads row k of L across 32 columns (8
// slices of k), and lane r holds column r of the diagonal block.
__device__ void upper_solve(const double* __restrict__ L, int M, double* ys, double (*red8)[kCB])
{
    const int nb = (M + kCB - 1) / kCB;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int I = nb - 1; I >= 0; --I) {
        const int i0 = I * kCB, rb = min(kCB, M - i0), k0 = i0 + rb;
        {
            const int r = threadIdx.x & (kCB - 1), s = threadIdx.x / kCB;
            double part = 0.0;
            if (r < rb)
                for (int k = k0 + s; k < M; k += kT / kCB) part += L[(int64_t)k * M + i0 + r] * ys[k];
            red8[s][r] = part;
        }
        __syncthreads();
        if (wid == 0) {
            double b = 0.0, lc[kCB];
#pragma unroll
            for (int c = 0; c < kCB; ++c)
                lc[c] = (lane < rb && c >= lane && c < rb) ? L[(int64_t)(i0 + c) * M + i0 + lane] : 0.0;
            if (lane < rb) {
                b = ys[i0 + lane];
                for (int s = 0; s < kT / kCB; ++s) b -= red8[s][lane];
            }
#pragma unroll
            for (int c = kCB - 1; c >= 0; --c) {
                if (c < rb) {
                    const double xc = bcast(b / lc[c], c);
                    if (lane < c) b -= lc[c] * xc;
                    if (lane == c) b = xc;
                }
            }
            if (lane < rb) ys[i0 + lane] = b;
        }
        __syncthreads();
    }
}

// x = (L L')^{-1} g with the factor from the blocked Cholesky.  One workgroup.
__global__ __launch_bounds__(kT) void chol_solve_kernel(const double* __restrict__ L, int M,
                                                        const double* __restrict__ g, double* __restrict__ x)
{
    __shared__ double ys[kMaxRefit];
    __shared__ double red8[kT / kCB][kCB];
    lower_solve(L, M, 0, g, -1, ys, red8[0]);
    upper_solve(L, M, ys, red8);
    for (int k = threadIdx.x; k < M; k += kT) x[k] = ys[k];
}

// Wald statistics from the factor, one workgroup per coefficient a: L y = e_a,
// so ((L L')^{-1})_aa = |y|^2 (y_k = 0 for k < a); se_a = its square root,
// z_a = b_a / se_a, p_a = erfc(|z_a| / sqrt 2).
__global__ __launch_bounds__(kT) void wald_kernel(const double* __restrict__ L, int M, const double* __restrict__ b,
                                                  double* __restrict__ se, double* __restrict__ pval)
{
    __shared__ double ys[kMaxRefit];
    __shared__ double red[kCB];
    __shared__ double sh[kT / kWave];
    const int a = blockIdx.x;
    lower_solve(L, M, a / kCB, nullptr, a, ys, red);
    double s2 = 0.0;
    for (int k = a + threadIdx.x; k < M; k += kT) s2 += ys[k] * ys[k];
    s2 = block_sum256(s2, sh);
    if (threadIdx.x == 0) {
        const double sd = sqrt(s2);
        se[a] = sd;
        pval[a] = erfc(fabs(b[a] / sd) * 0.70710678118654752440);
    }
}

// out = b + t d
__global__ void axpy_kernel(const double* __restrict__ b, const double* __restrict__ d, double t, int M,
                            double* __restrict__ out)
{
    const int a = blockIdx.x * kT + threadIdx.x;
    if (a < M) out[a] = b[a] + t * d[a];
}

// first sorted position with a nonzero coefficient per column: entry[j] = the
// smallest l with path[l][j] != 0 (or -1), coef[j] = |path[entry][j]|
__global__ void entry_kernel(const float* __restrict__ path, int L, int64_t ptot, int64_t p,
                             int32_t* __restrict__ entry, float* __restrict__ coef)
{
    for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < p; j += (int64_t)gridDim.x * kT) {
        int e = -1;
        float c = 0.0f;
        for (int l = 0; l < L; ++l) {
            const float v = path[(int64_t)l * ptot + j];
            if (v != 0.0f) {
                e = l;
                c = fabsf(v);
                break;
            }
        }
        entry[j] = e;
        coef[j] = c;
    }
}

inline unsigned grid_for(int64_t m) { return (unsigned)min((int64_t)8192, max((int64_t)1, (m + kT - 1) / kT)); }

}  // namespace

int64_t refit_ld(int64_t rows) { return max((int64_t)8, (rows + 7) / 8 * 8); }

hipError_t launch_gather_cols(const XDesc& x, const int32_t* cols, int m, const int32_t* perm, float* D, int64_t ldd,
                              hipStream_t s)
{
    if (m < 1 || ldd < refit_ld(x.n)) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)min((int64_t)512, (ldd + kT - 1) / kT);
    hipLaunchKernelGGL(gather_kernel, dim3(gx, m), dim3(kT), 0, s, x, cols, perm, D, ldd);
    return hipGetLastError();
}

hipError_t launch_gather_z(const float* Z, int64_t ldz, int64_t n, int q, const int32_t* perm, float* D, int64_t ldd,
                           hipStream_t s)
{
    if (q < 1 || ldd < refit_ld(n)) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)min((int64_t)512, (ldd + kT - 1) / kT);
    hipLaunchKernelGGL(gather_z_kernel, dim3(gx, q), dim3(kT), 0, s, Z, ldz, n, perm, D, ldd);
    return hipGetLastError();
}

hipError_t launch_refit_eta(const float* D, int64_t ldd, int64_t n, int M, const int32_t* perm, const double* b,
                            double* eta, hipStream_t s)
{
    hipLaunchKernelGGL(refit_eta_kernel, dim3(grid_for(n)), dim3(kT), 0, s, D, ldd, n, M, perm, b, eta);
    return hipGetLastError();
}

int refit_row_blocks(int64_t n) { return (int)((n + kRefitRows - 1) / kRefitRows); }

hipError_t launch_refit_grad(const float* D, int64_t ldd, int64_t n, int M, const int32_t* perm, const double* r,
                             double* rs, double* part, double* g, hipStream_t s)
{
    const int nrb = refit_row_blocks(n);
    hipLaunchKernelGGL(sort_r_kernel, dim3(grid_for(n)), dim3(kT), 0, s, perm, r, n, rs);
    hipLaunchKernelGGL(refit_xtr_kernel, dim3(nrb, M), dim3(kT), 0, s, D, ldd, n, M, rs, (int64_t)kRefitRows, part);
    hipLaunchKernelGGL(refit_sum_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, part, nrb, M, g);
    return hipGetLastError();
}

int gram_chunks(int64_t rows, int M)
{
    const int ntile = (M + kGT - 1) / kGT, npair = ntile * (ntile + 1) / 2;
    // at most 1024 workgroups, resident in one round: the FP32 term's are one
    // wavefront at one per SIMD, the FP64 term's two at two per SIMD
    const int want = max(1, 1024 / npair);
    const int64_t cap = max((int64_t)1, rows / 1024);
    return (int)max((int64_t)1, min((int64_t)min(want, kGramChunks), cap));
}

static int64_t gram_rows(int64_t rows, int nc) { return ((rows + nc - 1) / nc + kGR - 1) / kGR * kGR; }

int scan_chunks(int64_t n) { return (int)max((int64_t)1, (n + kScanChunk - 1) / kScanChunk); }

hipError_t launch_refit_hessian(const RefitHess& h, hipStream_t s)
{
    const int M = h.M;
    if (M < 1 || M > kMaxRefit || h.ldd < refit_ld(h.n) || h.ldp < refit_ld(h.G)) return hipErrorInvalidValue;
    const int ntile = (M + kGT - 1) / kGT, npair = ntile * (ntile + 1) / 2;
    const int nc1 = gram_chunks(h.n, M), nc2 = gram_chunks(h.G, M), nch = scan_chunks(h.n);
    hipLaunchKernelGGL(hess_weight_kernel, dim3(grid_for(h.ldd)), dim3(kT), 0, s, h.perm, h.ev, h.r, h.n, h.ldd,
                       h.wt);
    hipLaunchKernelGGL((gram_kernel<float, 8, 4>), dim3(npair, nc1), dim3(kT / 4), 0, s, h.D, h.ldd, h.n, M, h.wt,
                       gram_rows(h.n, nc1), ntile, h.part1);
    hipLaunchKernelGGL(chunk_sum_kernel, dim3(nch, M + 1), dim3(kT), 0, s, h.D, h.ldd, h.n, M, h.w, nch, h.csum);
    hipLaunchKernelGGL(scan_p_kernel, dim3(nch, M + 1), dim3(kT), 0, s, h.D, h.ldd, h.n, M, h.w, h.csum, nch, h.egidx,
                       h.G, h.ldp, h.P);
    hipLaunchKernelGGL(event_weight_kernel, dim3(grid_for(h.ldp)), dim3(kT), 0, s, h.P + (int64_t)M * h.ldp, h.egcnt,
                       h.G, h.ldp, h.wg);
    hipLaunchKernelGGL((gram_kernel<double, 4, 2>), dim3(npair, nc2), dim3(kT / 2), 0, s, h.P, h.ldp, h.G, M, h.wg,
                       gram_rows(h.G, nc2), ntile, h.part2);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(grid_for((int64_t)M * M)), dim3(kT), 0, s, h.part1, nc1, h.part2,
                       nc2, M, h.H);
    return hipGetLastError();
}

hipError_t launch_chol(double* A, int M, int* ok, hipStream_t s)
{
    if (M < 1 || M > kMaxRefit) return hipErrorInvalidValue;
    const int nb = (M + kCB - 1) / kCB;
    for (int J = 0; J < nb; ++J) {
        hipLaunchKernelGGL(chol_panel_kernel, dim3(nb - J), dim3(kT), 0, s, A, M, J, ok);
        const int nt = nb - J - 1;
        if (nt > 0) hipLaunchKernelGGL(chol_update_kernel, dim3(nt * (nt + 1) / 2), dim3(kT), 0, s, A, M, J);
    }
    return hipGetLastError();
}

hipError_t launch_chol_solve(const double* L, int M, const double* g, double* x, hipStream_t s)
{
    if (M < 1 || M > kMaxRefit) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(kT), 0, s, L, M, g, x);
    return hipGetLastError();
}

hipError_t launch_wald(const double* L, int M, const double* b, double* se, double* pval, hipStream_t s)
{
    if (M < 1 || M > kMaxRefit) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wald_kernel, dim3(M), dim3(kT), 0, s, L, M, b, se, pval);
    return hipGetLastError();
}

hipError_t launch_axpy(const double* b, const double* d, double t, int M, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(axpy_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, b, d, t, M, out);
    return hipGetLastError();
}

hipError_t launch_entry(const float* path, int L, int64_t ptot, int64_t p, int32_t* entry, float* coef, hipStream_t s)
{
    hipLaunchKernelGGL(entry_kernel, dim3(grid_for(p)), dim3(kT), 0, s, path, L, ptot, p, entry, coef);
    return hipGetLastError();
}

}  // namespace cox
