// gemvt.hip -- the launches of X~' r with the fused proximal epilogue (the
// phases themselves are in gemvt_dev.h).
#include "gemvt_dev.h"

namespace cox {
namespace {

using namespace gemvtdev;

template <int XT, int NB, bool VEC>
__global__ __launch_bounds__(kGemvtThreads) void gemvt_sums_kernel(GemvtArgs a)
{
    __shared__ __attribute__((aligned(16))) float sr[NB * chunk_rows<NB>()];
    gemvt_sums_blk<XT, NB, VEC>(a, blockIdx.x, blockIdx.y, sr);
}

__global__ __launch_bounds__(256) void gemvt_epilogue_kernel(GemvtArgs a) { gemvt_epilogue_blk(a, blockIdx.x); }

template <int XT, int NB>
hipError_t launch_t(const GemvtArgs& a, hipStream_t s)
{
    constexpr int cols_wg = 4 * cols_per_wave<XT, NB>();
    const dim3 grid((unsigned)((a.x.p + cols_wg - 1) / cols_wg), (unsigned)a.nsplit);
    if (a.x.vec16)
        hipLaunchKernelGGL((gemvt_sums_kernel<XT, NB, true>), grid, dim3(kGemvtThreads), 0, s, a);
    else
        hipLaunchKernelGGL((gemvt_sums_kernel<XT, NB, false>), grid, dim3(kGemvtThreads), 0, s, a);
    return hipGetLastError();
}

template <int XT>
hipError_t launch_x(const GemvtArgs& a, hipStream_t s)
{
    if (a.nb <= 1) return launch_t<XT, 1>(a, s);
    if (a.nb <= 2) return launch_t<XT, 2>(a, s);
    if (a.nb <= 4) return launch_t<XT, 4>(a, s);
    return launch_t<XT, 8>(a, s);
}

}  // namespace

hipError_t launch_gemvt_epilogue(const GemvtArgs& a, hipStream_t s)
{
    if (a.nb < 1 || a.nsplit < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemvt_epilogue_kernel, dim3((unsigned)((a.x.p + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemvt_sums(const GemvtArgs& a, hipStream_t s)
{
    if (a.nb < 1 || a.nb > 8 || a.nsplit < 1 || a.split_rows % kSplitRows != 0) return hipErrorInvalidValue;
    switch (a.x.xt) {
    case XT_F32: return launch_x<XT_F32>(a, s);
    case XT_FP8: return launch_x<XT_FP8>(a, s);
    default: return launch_x<XT_I8>(a, s);
    }
}

hipError_t launch_gemvt(const GemvtArgs& a, hipStream_t s)
{
    const hipError_t e = launch_gemvt_sums(a, s);
    if (e != hipSuccess) return e;
    return launch_gemvt_epilogue(a, s);
}

}  // namespace cox
