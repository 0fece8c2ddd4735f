// risk.hip -- the risk-set sums of one ISTA step as five launches, one per
// phase (the phases themselves are in risk_dev.h).
#include "risk_dev.h"

namespace cox {
namespace {

using namespace riskdev;

__global__ __launch_bounds__(kT) void risk_eta_kernel(RiskArgs a)
{
    __shared__ double sh[kNW];
    risk_eta_blk(a, blockIdx.x, blockIdx.y, sh);
}

__global__ __launch_bounds__(kT) void risk_scan_w_kernel(RiskArgs a)
{
    __shared__ double sh[kNW];
    risk_scan_w_blk(a, blockIdx.x, blockIdx.y, sh);
}

__global__ __launch_bounds__(kT) void risk_scan_q_kernel(RiskArgs a)
{
    __shared__ double sh[kNW];
    __shared__ double pre[kMaxTiles];
    risk_scan_q_blk(a, blockIdx.x, blockIdx.y, sh, pre);
}

__global__ __launch_bounds__(kT) void risk_resid_kernel(RiskArgs a)
{
    __shared__ double sh[kNW];
    __shared__ double suf[kMaxTiles];
    risk_resid_blk(a, blockIdx.x, blockIdx.y, sh, suf);
}

__global__ __launch_bounds__(kT) void risk_finish_kernel(RiskArgs a)
{
    __shared__ double sh[kNW];
    risk_finish_blk(a, blockIdx.x, sh);
}

}  // namespace

hipError_t launch_risk(const RiskArgs& a, hipStream_t s)
{
    if (a.ntile > kMaxTiles || a.ntile < 1 || a.nfin < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(risk_eta_kernel, dim3(a.nfin, a.B), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(risk_scan_w_kernel, dim3(a.ntile, a.B), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(risk_scan_q_kernel, dim3(a.ntile, a.B), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(risk_resid_kernel, dim3(a.ntile, a.B), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(risk_finish_kernel, dim3(a.B), dim3(kT), 0, s, a);
    return hipGetLastError();
}

}  // namespace cox
