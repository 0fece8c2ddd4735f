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
// Tiling: a workgroup of 8 wavefronts (two per SIMD) owns 256 SNP columns (2 M
// tiles of 16 per wavefront) and all 3 * B limb columns (N tiles of 16), and walks K = n in
// stages of 256 rows.  X is read once per pass for all B vectors.  A fragments
// (16 rows of one column per lane, one 16-byte load) stream from global memory
// one stage ahead; the stage's limb tile (3 * B columns x 256 rows) is staged in
// LDS, double buffered, laid out so that each MFMA B fragment is one 16-byte
// LDS read per lane, contiguous across lanes.
#include "device_common.h"
#include "mfma.h"

namespace cox {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int kTM = 512;         // matrix-core kernels: 8 wavefronts, two per SIMD
constexpr int kMT = 2;           // M tiles (16 rows each) per wavefront: 8 x 2 x 16 = 256
constexpr int kKS = 4;           // MFMA k-steps (64 rows each) per stage
constexpr int kKC = 64 * kKS;    // rows per stage
constexpr int kLimbs = 3;
constexpr int kQBits = 22;       // |R| <= 2^22 keeps the top limb within int8

// Allele-count bytes -> int8 counts.  FP8 E4M3 codes of 0, 1, 2 are 0x00, 0x38,
// 0x40: bit 3 marks 1 and bit 6 marks 2 (other codes are rejected beforehand).
template <int XT>
__device__ __forceinline__ uint32_t counts4(uint32_t w)
{
    if constexpr (XT == XT_FP8)
        return ((w >> 3) & 0x01010101u) | ((w >> 5) & 0x02020202u);
    else
        return w;
}

// 16 rows [row, row + 16) of column col as int8 counts; rows >= n and columns
// >= p read as 0.  Branch-free: one 16-byte load from a clamped address, then
// byte masks (row is a multiple of 16 and ldx a multiple of 16, so the load
// never leaves the column's ldx bytes).
template <int XT>
__device__ __forceinline__ v4i load_a(const uint8_t* __restrict__ X, int64_t col, int64_t p, int64_t ldx,
                                      int64_t row, int64_t n)
{
    const bool ok = col < p && row < n;
    const uint8_t* src = X + (ok ? col * ldx + row : 0);
    const uint4 u = *reinterpret_cast<const uint4*>(src);
    const int64_t valid = ok ? n - row : 0;  // bytes of this run that are inside the column
    v4i v;
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t keep = valid - 4 * q;  // bytes of dword q to keep
        const uint32_t mask = keep >= 4 ? 0xFFFFFFFFu : (keep <= 0 ? 0u : (0xFFFFFFFFu >> (8 * (4 - keep))));
        v[q] = (int)(counts4<XT>(w[q]) & mask);
    }
    return v;
}

template <int XT, int NG, int KS, int PF>
__global__ __launch_bounds__(kTM, 2) void mfma_xtr_kernel(MfmaArgs a)
{
    // KS k-steps of 64 rows per stage; loads run PF stages ahead in a register ring.
    constexpr int KC = 64 * KS;
    constexpr int NT = kLimbs * NG;  // N tiles, limb-major: tile = limb * NG + b / 16
    constexpr int NCOL = 16 * NT;
    constexpr int CHUNKS = NCOL * (KC / 16);  // 16-byte chunks of limb data per stage
    constexpr int CPT = (CHUNKS + kTM - 1) / kTM;
    __shared__ v4i sR[2][KS * 4 * NCOL];

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t n = a.n, p = a.p, ldx = a.ldx;
    const int64_t jw = (int64_t)blockIdx.x * 256 + wid * (16 * kMT);  // first column of this wavefront
    const uint8_t* __restrict__ X = static_cast<const uint8_t*>(a.X);
    const int8_t* __restrict__ limbs = a.limbs;
    const int64_t nstage = (n + KC - 1) / KC;
    const int arow = 16 * (lane >> 4);  // k offset of this lane's 16 bytes within a k-step
    const int acol = lane & 15;

    v4i acc[kMT][NT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};

    v4i Ab[PF][kMT][KS];
    v4i Rb[PF][CPT];
    auto fetch = [&](int64_t t, v4i (&A)[kMT][KS], v4i (&R)[CPT]) {
        const int64_t k0 = t * KC;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int mt = 0; mt < kMT; ++mt)
                A[mt][ks] = load_a<XT>(X, jw + mt * 16 + acol, p, ldx, k0 + ks * 64 + arow, n);
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = threadIdx.x + kTM * u;
            if (c < CHUNKS) {
                const int col = c / (KC / 16), q = c % (KC / 16);
                const int limb = col / (16 * NG), b = col % (16 * NG);
                R[u] = *reinterpret_cast<const v4i*>(limbs + ((int64_t)limb * a.bpad + b) * a.lstride + k0 + 16 * q);
            }
        }
    };
    auto store_r = [&](int buf, const v4i (&R)[CPT]) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = threadIdx.x + kTM * u;
            if (c < CHUNKS) {
                const int col = c / (KC / 16), q = c % (KC / 16);
                sR[buf][(q >> 2) * 4 * NCOL + (q & 3) * NCOL + col] = R[u];
            }
        }
    };

#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < nstage) fetch(q, Ab[q], Rb[q]);
    store_r(0, Rb[0]);
    __syncthreads();

    for (int64_t s0 = 0; s0 < nstage; s0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int64_t t = s0 + q;
            if (t < nstage) {
                v4i A[kMT][KS];
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int mt = 0; mt < kMT; ++mt) A[mt][ks] = Ab[q][mt][ks];
                if (t + PF < nstage) fetch(t + PF, Ab[q], Rb[q]);
                const int buf = (int)(t & 1);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const v4i bf = sR[buf][ks * 4 * NCOL + (lane >> 4) * NCOL + nt * 16 + acol];
#pragma unroll
                        for (int mt = 0; mt < kMT; ++mt)
                            acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt][ks], bf, acc[mt][nt], 0, 0, 0);
                    }
                }
                if (t + 1 < nstage) store_r(buf ^ 1, Rb[(q + 1) % PF]);
                __syncthreads();
            }
        }
    }

    // C of tile (mt, nt): lane holds rows mfma_c_row(lane, v), column lane & 15.
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int bq = 0; bq < NG; ++bq)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = bq * 16 + acol;
                const int64_t j = jw + mt * 16 + mfma_c_row(lane, v);
                if (j < p && b < a.B) {
                    const int64_t tot = (int64_t)acc[mt][bq][v] + 256 * (int64_t)acc[mt][NG + bq][v] +
                                        65536 * (int64_t)acc[mt][2 * NG + bq][v];
                    a.out[(int64_t)b * p + j] = a.qscale[b] * (double)tot;
                }
            }
}

// eta update on the matrix cores: eta (n x B) += G[:, U] D, contracting over the
// changed columns U.  M = subjects, N = 3 * B limb columns, K = positions in U.
// G is stored with subjects contiguous, so a 64-column x 256-row tile is staged
// in LDS (16-byte chunks, XOR-swizzled by the column's 16-group so that the
// byte gathers below hit distinct banks) and each A fragment (16 columns of one
// subject) is gathered byte by byte.  The D limb tile is staged like R above.
// Each (subject, b) is owned by one lane, so eta is updated in place.
template <int XT, int NG, int PF>
__global__ __launch_bounds__(kTM, 2) void mfma_eta_kernel(MfmaEtaArgs a)
{
    // One 64-column k-step per stage; loads run PF stages ahead in a register ring.
    constexpr int NT = kLimbs * NG;
    constexpr int NCOL = 16 * NT;
    constexpr int DCH = 4 * NCOL;  // 16-byte chunks of D per 64-column step
    constexpr int DPT = (DCH + kTM - 1) / kTM;
    constexpr int GPT = 1024 / kTM;  // 16-byte chunks of G per thread per step
    __shared__ uint4 sG[2][64 * 16];
    __shared__ v4i sD[2][DCH];
    const int nsel = *a.nsel;
    if (nsel == 0) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t n = a.n, ldx = a.ldx;
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    const uint8_t* __restrict__ X = static_cast<const uint8_t*>(a.X);
    const int nchunk = (nsel + 63) / 64;

    v4i acc[kMT][NT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};

    uint4 gr[PF][GPT];
    v4i dr[PF][DPT];
    auto fetch = [&](int c, uint4 (&g)[GPT], v4i (&dd)[DPT]) {
#pragma unroll
        for (int k = 0; k < GPT; ++k) {
            const int ch = threadIdx.x + kTM * k;
            const int u = ch >> 4, rb = ch & 15;
            const int pos = c * 64 + u;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (pos < nsel) {
                const v4i t = load_a<XT>(X, a.sel[pos], a.p, ldx, i0 + 16 * rb, n);
                v = make_uint4((uint32_t)t[0], (uint32_t)t[1], (uint32_t)t[2], (uint32_t)t[3]);
            }
            g[k] = v;
        }
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int ch = threadIdx.x + kTM * k;
            if (ch < DCH) {
                const int col = ch >> 2, kq = ch & 3;
                const int limb = col / (16 * NG), b = col % (16 * NG);
                dd[k] = *reinterpret_cast<const v4i*>(a.dlimbs + ((int64_t)limb * a.bpad + b) * a.dstride + c * 64 +
                                                      16 * kq);
            }
        }
    };
    auto store = [&](int buf, const uint4 (&g)[GPT], const v4i (&dd)[DPT]) {
#pragma unroll
        for (int k = 0; k < GPT; ++k) {
            const int ch = threadIdx.x + kTM * k;
            const int u = ch >> 4, rb = ch & 15;
            sG[buf][u * 16 + (rb ^ (u >> 4))] = g[k];
        }
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int ch = threadIdx.x + kTM * k;
            if (ch < DCH) {
                const int col = ch >> 2, kq = ch & 3;
                sD[buf][kq * NCOL + col] = dd[k];
            }
        }
    };

#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < nchunk) fetch(q, gr[q], dr[q]);
    store(0, gr[0], dr[0]);
    __syncthreads();
    for (int c0 = 0; c0 < nchunk; c0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int c = c0 + q;
            if (c < nchunk) {
                if (c + PF < nchunk) fetch(c + PF, gr[q], dr[q]);
                const int buf = c & 1;
                const uint8_t* g8 = reinterpret_cast<const uint8_t*>(sG[buf]);
                v4i A[kMT];
#pragma unroll
                for (int mt = 0; mt < kMT; ++mt) {
                    const int row = wid * (16 * kMT) + mt * 16 + (lane & 15);
                    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int u = 16 * (lane >> 4) + e;
                        const uint32_t byte = g8[u * 256 + 16 * ((row >> 4) ^ (u >> 4)) + (row & 15)];
                        w[e >> 2] |= byte << (8 * (e & 3));
                    }
                    A[mt] = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const v4i bf = sD[buf][(lane >> 4) * NCOL + nt * 16 + (lane & 15)];
#pragma unroll
                    for (int mt = 0; mt < kMT; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], bf, acc[mt][nt], 0, 0, 0);
                }
                if (c + 1 < nchunk) store(buf ^ 1, gr[(q + 1) % PF], dr[(q + 1) % PF]);
                __syncthreads();
            }
        }
    }

#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int bq = 0; bq < NG; ++bq)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = bq * 16 + (lane & 15);
                const int64_t i = i0 + wid * (16 * kMT) + mt * 16 + mfma_c_row(lane, v);
                if (i < n && b < a.B && (a.active == nullptr || a.active[b])) {
                    const int64_t tot = (int64_t)acc[mt][bq][v] + 256 * (int64_t)acc[mt][NG + bq][v] +
                                        65536 * (int64_t)acc[mt][2 * NG + bq][v];
                    a.eta[(int64_t)b * n + i] += a.dscale[b] * (double)tot;
                }
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
__global__ __launch_bounds__(kT) void dquant_kernel(const double* __restrict__ dcoef, int64_t p,
                                                    const int32_t* __restrict__ sel, const int32_t* __restrict__ nsel,
                                                    const double* __restrict__ dmaxp, int ntile,
                                                    int8_t* __restrict__ dlimbs, int64_t dstride, int bpad,
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
        dlimbs[((int64_t)0 * bpad + b) * dstride + u] = (int8_t)d0;
        dlimbs[((int64_t)1 * bpad + b) * dstride + u] = (int8_t)d1;
        dlimbs[((int64_t)2 * bpad + b) * dstride + u] = (int8_t)d2;
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

// Quantise r to three int8 limbs per vector; exact partial sums of R.
__global__ __launch_bounds__(kT) void quantize_kernel(const double* __restrict__ r, int64_t n,
                                                      const double* __restrict__ rmaxp, int ntile,
                                                      int8_t* __restrict__ limbs, int64_t lstride, int bpad,
                                                      double* __restrict__ qscale, long long* __restrict__ rsump)
{
    __shared__ long long sh[kT / 64];
    const int b = blockIdx.y;
    double mx = 0.0;
    for (int t = 0; t < ntile; ++t) mx = fmax(mx, rmaxp[(int64_t)b * ntile + t]);
    const double q = mx > 0.0 ? mx / (double)(1 << kQBits) : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) qscale[b] = q;
    long long sum = 0;
    for (int64_t i = (int64_t)blockIdx.x * 4096 + threadIdx.x; i < min(n, (int64_t)(blockIdx.x + 1) * 4096);
         i += kT) {
        const int R = (int)llrint(r[(int64_t)b * n + i] / q);
        const int d0 = ((R + 128) & 255) - 128;
        const int R1 = (R - d0) >> 8;
        const int d1 = ((R1 + 128) & 255) - 128;
        const int d2 = (R1 - d1) >> 8;
        limbs[((int64_t)0 * bpad + b) * lstride + i] = (int8_t)d0;
        limbs[((int64_t)1 * bpad + b) * lstride + i] = (int8_t)d1;
        limbs[((int64_t)2 * bpad + b) * lstride + i] = (int8_t)d2;
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

template <int XT, int NG>
hipError_t launch_eta_ng(const MfmaEtaArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.n + 255) / 256));
    switch (a.variant) {
    case 1: hipLaunchKernelGGL((mfma_eta_kernel<XT, NG, 2>), grid, dim3(kTM), 0, s, a); break;
    case 2: hipLaunchKernelGGL((mfma_eta_kernel<XT, NG, 6>), grid, dim3(kTM), 0, s, a); break;
    default: hipLaunchKernelGGL((mfma_eta_kernel<XT, NG, 4>), grid, dim3(kTM), 0, s, a); break;
    }
    return hipGetLastError();
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

template <int XT, int NG>
hipError_t launch_ng(const MfmaArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.p + 255) / 256));
    switch (a.variant) {
    case 1: hipLaunchKernelGGL((mfma_xtr_kernel<XT, NG, 4, 1>), grid, dim3(kTM), 0, s, a); break;
    case 2: hipLaunchKernelGGL((mfma_xtr_kernel<XT, NG, 2, 4>), grid, dim3(kTM), 0, s, a); break;
    default: hipLaunchKernelGGL((mfma_xtr_kernel<XT, NG, 2, 3>), grid, dim3(kTM), 0, s, a); break;
    }
    return hipGetLastError();
}

template <int XT>
hipError_t launch_xt(const MfmaArgs& a, hipStream_t s)
{
    switch (a.bpad / 16) {
    case 1: return launch_ng<XT, 1>(a, s);
    case 2: return launch_ng<XT, 2>(a, s);
    case 3: return launch_ng<XT, 3>(a, s);
    default: return launch_ng<XT, 4>(a, s);
    }
}

}  // namespace

int mfma_ntile(int64_t n) { return (int)((n + 4095) / 4096); }

hipError_t launch_quantize(const double* r64, int64_t n, int B, double* rmaxp, long long* rsump, int8_t* limbs,
                           int64_t lstride, int bpad, double* qscale, double* sumr, hipStream_t s)
{
    const int nt = mfma_ntile(n);
    hipLaunchKernelGGL(rmax_kernel, dim3(nt, B), dim3(kT), 0, s, r64, n, rmaxp, nt);
    hipLaunchKernelGGL(quantize_kernel, dim3(nt, B), dim3(kT), 0, s, r64, n, rmaxp, nt, limbs, lstride, bpad, qscale,
                       rsump);
    hipLaunchKernelGGL(rsum_kernel, dim3(1), dim3(64), 0, s, rsump, nt, qscale, sumr, B);
    return hipGetLastError();
}

hipError_t launch_quantize_d(const double* dcoef, int64_t p, const int32_t* sel, const int32_t* nsel, int B,
                             double* dmaxp, int8_t* dlimbs, int64_t dstride, int bpad, double* dscale,
                             hipStream_t s)
{
    const int nt = (int)((p + 63) / 64 * 64 + 4095) / 4096;
    hipLaunchKernelGGL(dmax_kernel, dim3(nt, B), dim3(kT), 0, s, dcoef, p, sel, nsel, dmaxp, nt);
    hipLaunchKernelGGL(dquant_kernel, dim3(nt, B), dim3(kT), 0, s, dcoef, p, sel, nsel, dmaxp, nt, dlimbs, dstride,
                       bpad, dscale);
    return hipGetLastError();
}

hipError_t launch_mfma_eta(const MfmaEtaArgs& a, hipStream_t s)
{
    if (a.bpad < 16 || a.bpad > 64 || a.bpad % 16 || a.B > a.bpad || a.dstride % 64) return hipErrorInvalidValue;
    return a.xt == XT_FP8 ? launch_eta_xt<XT_FP8>(a, s) : launch_eta_xt<XT_I8>(a, s);
}

hipError_t launch_mfma_xtr(const MfmaArgs& a, hipStream_t s)
{
    if (a.bpad < 16 || a.bpad > 64 || a.bpad % 16 || a.B > a.bpad || a.lstride % 256) return hipErrorInvalidValue;
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
