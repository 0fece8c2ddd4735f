// genhash.hip -- device generator of synthetic genotype matrices.  Input
// generation only: no step of the Cox method is computed here.
//
// Same definition, bit for bit, as genhash.c (host) and coxsim.hashgen (numpy):
//   h(i, j) = splitmix(((j << 32) | i) ^ splitmix(seed))
//   G[i, j] = [low32(h) < t_j] + [high32(h) < t_j]
// written column-major (column j at byte j*ldx) as int8 counts (fmt 0) or OCP
// FP8 E4M3 codes (fmt 1).  Also returns exact per-column counts of 1s and 2s,
// from which the host forms the standardisation constants.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t splitmix(uint64_t x) { return mix64(x + 0x9E3779B97F4A7C15ULL); }

constexpr int kThreads = 256;
constexpr int kRowsPerThread = 16;

// One workgroup per column; each thread writes 16 consecutive rows with one
// 16-byte store when the whole run is inside the column, byte stores otherwise.
__global__ __launch_bounds__(kThreads) void genotype_kernel(uint8_t* __restrict__ out, int64_t n, int64_t ldx,
                                                            uint64_t sk, const uint32_t* __restrict__ thr,
                                                            int fmt, int64_t* __restrict__ c1,
                                                            int64_t* __restrict__ c2)
{
    const int64_t j = blockIdx.x;
    const uint32_t t = thr[j];
    uint8_t* col = out + j * ldx;
    const bool aligned = ((reinterpret_cast<uintptr_t>(col) & 15) == 0);
    int cnt1 = 0, cnt2 = 0;
    for (int64_t i0 = (int64_t)threadIdx.x * kRowsPerThread; i0 < n; i0 += (int64_t)kThreads * kRowsPerThread) {
        uint8_t v[kRowsPerThread];
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
            const uint64_t i = (uint64_t)(i0 + q);
            const uint64_t h = splitmix((((uint64_t)j) << 32 | i) ^ sk);
            const int g = ((uint32_t)h < t) + ((uint32_t)(h >> 32) < t);
            const bool in = (i0 + q) < n;
            cnt1 += in && g == 1;
            cnt2 += in && g == 2;
            v[q] = fmt ? (g == 0 ? 0x00 : (g == 1 ? 0x38 : 0x40)) : (uint8_t)g;
        }
        if (aligned && i0 + kRowsPerThread <= n) {
            uint4 w;
            w.x = v[0] | (v[1] << 8) | (v[2] << 16) | ((uint32_t)v[3] << 24);
            w.y = v[4] | (v[5] << 8) | (v[6] << 16) | ((uint32_t)v[7] << 24);
            w.z = v[8] | (v[9] << 8) | (v[10] << 16) | ((uint32_t)v[11] << 24);
            w.w = v[12] | (v[13] << 8) | (v[14] << 16) | ((uint32_t)v[15] << 24);
            *reinterpret_cast<uint4*>(col + i0) = w;
        } else {
            for (int q = 0; q < kRowsPerThread && i0 + q < n; ++q) col[i0 + q] = v[q];
        }
    }
    __shared__ int s1[kThreads], s2[kThreads];
    s1[threadIdx.x] = cnt1;
    s2[threadIdx.x] = cnt2;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c1[j] = s1[0];
        c2[j] = s2[0];
    }
}

}  // namespace

extern "C" int coxsim_genotype_device(void* out, int64_t n, int64_t p, int64_t ldx, uint64_t seed,
                                      const uint32_t* thresholds_dev, int fmt, int64_t* c1_dev,
                                      int64_t* c2_dev, void* stream)
{
    if (!out || !thresholds_dev || !c1_dev || !c2_dev || n < 0 || p < 0 || ldx < n || n >= (1LL << 32) ||
        p >= (1LL << 31))
        return 1;
    if (p == 0) return 0;
    const uint64_t x = seed + 0x9E3779B97F4A7C15ULL;
    uint64_t z = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    const uint64_t sk = z ^ (z >> 31);
    hipLaunchKernelGGL(genotype_kernel, dim3((unsigned)p), dim3(kThreads), 0, (hipStream_t)stream,
                       (uint8_t*)out, n, ldx, sk, thresholds_dev, fmt, c1_dev, c2_dev);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
