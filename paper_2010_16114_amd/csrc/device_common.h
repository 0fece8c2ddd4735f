// device_common.h -- wavefront helpers and element decoding for gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace cox {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_incl_scan(double v, int lane)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        double t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Soft-thresholding S_t(x) (Section 4.2): x - t above t, x + t below -t, 0 between.
__device__ __forceinline__ double soft_threshold(double x, double t)
{
    return x > t ? x - t : (x < -t ? x + t : 0.0);
}

// ---- element decoding: 16 bytes of X -> floats

typedef float v2f __attribute__((ext_vector_type(2)));

// Four FP8 E4M3 (OCP) codes packed in a dword -> four floats (hardware convert).
__device__ __forceinline__ void fp8x4_to_f32(uint32_t w, float* o)
{
    v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
    v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    o[0] = lo.x;
    o[1] = lo.y;
    o[2] = hi.x;
    o[3] = hi.y;
}

__device__ __forceinline__ void i8x4_to_f32(uint32_t w, float* o)
{
    o[0] = (float)(int8_t)(w & 0xff);
    o[1] = (float)(int8_t)((w >> 8) & 0xff);
    o[2] = (float)(int8_t)((w >> 16) & 0xff);
    o[3] = (float)(int8_t)(w >> 24);
}

template <int XT>
__device__ __forceinline__ void decode4(uint32_t w, float* o)
{
    if constexpr (XT == XT_FP8)
        fp8x4_to_f32(w, o);
    else
        i8x4_to_f32(w, o);
}

// One element of X as float (scalar path, any alignment).
template <int XT>
__device__ __forceinline__ float load_x1(const void* X, int64_t off)
{
    if constexpr (XT == XT_F32) {
        return static_cast<const float*>(X)[off];
    } else {
        uint32_t b = static_cast<const uint8_t*>(X)[off];
        float o[4];
        decode4<XT>(b, o);
        return o[0];
    }
}

__device__ __forceinline__ float4 load_f4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ uint4 load_u4(const void* p) { return *reinterpret_cast<const uint4*>(p); }
// A streaming (non-temporal) 16-byte load, for data read once: it does not push
// what is reused (the residual chunks, the limb tiles) out of the caches.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 load_u4_stream(const void* p)
{
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 load_u2_stream(const void* p)
{
    const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float4 load_f4_stream(const float* p)
{
    const uint4 v = load_u4_stream(p);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}

}  // namespace cox
