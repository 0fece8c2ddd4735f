// persist.hip -- cox_fit_path in one persistent launch: every ISTA step of
// every b of a lambda path (Section 5.3's iteration, with Section 6's lag-k
// stopping rule applied on the device) inside a single kernel.
//
// A grid of co-resident workgroups (a cooperative launch, which the runtime
// refuses when the grid cannot be resident at once) walks the steps.  Each
// phase of the one-kernel-per-phase form becomes a loop over that phase's
// workgroup positions, strided over the resident grid, running the very
// device function the phase's own kernel runs (risk_dev.h, gemvt_dev.h,
// gemv_dev.h), so every value is computed by the same code in the same order
// and the two forms agree bit for bit.  Phases are separated by grid-wide
// barriers.  After the barrier that follows the stopping rule every workgroup
// reads the same activity flags, so all leave the loop at the same step and
// every workgroup reaches every barrier.
//
// The barrier.  Every wavefront first waits until its own stores have reached
// its XCD's L2; after a workgroup barrier one thread per workgroup writes the
// L2's dirty lines back to memory (a device-scope release fence: each of the
// eight XCDs has its own L2), adds 1 to a 64-bit arrival counter and, unless
// it was the last to arrive, polls a generation word with plain device-scope
// loads (no cache invalidation per poll; the words for the eight XCDs sit on
// separate 256-byte lines so that pollers are spread over them); the last
// arrival publishes the new generation to all eight words.  The polling
// thread then takes one device-scope acquire fence (invalidating the stale
// lines of its L1 and L2) and a workgroup barrier releases the other
// wavefronts.  The wait is bounded in time: past the limit the waiting thread
// raises an abort flag that every waiter also polls, so the kernel always
// exits; the host reports the abort as a device error.
#include <hip/hip_runtime.h>

#include "gemv_dev.h"
#include "gemvt_dev.h"
#include "risk_dev.h"

namespace cox {
namespace {

constexpr int kPT = 256;  // threads per workgroup of every phase
static_assert(riskdev::kT == kPT && gemvdev::kT == kPT && kGemvtThreads == kPT, "every phase runs 256 threads");

// Device words of the barrier, each on its own 256-byte line (zero at launch).
constexpr int kBarLine = 32;  // 8-byte words per line
struct Barrier {
    unsigned long long* words;  // [0]: arrivals; [kBarLine]: abort flag; [kBarLine (2 + x)]: generation, XCD x
    unsigned long long ticks;   // wait limit in wall-clock ticks
    unsigned long long passed;  // barriers this workgroup has entered
};

// Returns true when the launch is being abandoned (a wait passed its limit).
__device__ __forceinline__ bool grid_barrier(Barrier& br, unsigned long long nwg, int* s_flag)
{
    __builtin_amdgcn_s_waitcnt(0);  // this wavefront's stores are in L2
    __syncthreads();
    br.passed += 1;
    if (threadIdx.x == 0) {
        unsigned long long* const count = br.words;
        unsigned long long* const abort = br.words + kBarLine;
        unsigned long long* const gen = br.words + kBarLine * (2 + (blockIdx.x & 7));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long old = __hip_atomic_fetch_add(count, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ab = 0;
        if (old + 1 == br.passed * nwg) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            for (int x = 0; x < 8; ++x)
                __hip_atomic_store(br.words + kBarLine * (2 + x), br.passed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < br.passed) {
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ab = 1;
                    break;
                }
                if (wall_clock64() - t0 > br.ticks) {
                    __hip_atomic_store(abort, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ab = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = ab;
    }
    __syncthreads();
    const bool ab = *s_flag != 0;
    __syncthreads();  // s_flag is read by every thread before the next barrier writes it
    return ab;
}

// Wavefronts per SIMD the kernel is compiled for: the occupancy of the
// column-sums kernel of the same (XT, NB), whose X stream dominates a step.
template <int XT, int NB>
constexpr int persist_waves()
{
    if constexpr (XT == XT_F32) return NB <= 2 ? 4 : 3;
    else return NB == 1 || NB == 4 ? 3 : 2;
}

template <int XT, int NB>
__global__ __launch_bounds__(kPT, (persist_waves<XT, NB>())) void fit_persistent_kernel(PersistArgs a, Barrier br)
{
    // LDS shared by the phases: the r chunk of the column sums (NB x
    // chunk_rows floats, 32 KB) or the tile offsets of the scans (32 KB)
    __shared__ __attribute__((aligned(16))) double big[kMaxTiles];
    __shared__ double sh[kPT / kWave];
    __shared__ int ish[17], sstart[kPT], scnt[kPT];
    __shared__ int s_flag;
    static_assert(NB * gemvtdev::chunk_rows<NB>() * sizeof(float) <= sizeof(double) * kMaxTiles, "r chunk fits");
    float* const rchunk = reinterpret_cast<float*>(big);

    const RiskArgs& ra = a.ra;
    const GemvtArgs& g = a.g;
    const int B = a.B;
    const int64_t G = gridDim.x;
    const unsigned long long nwg = gridDim.x;
    const int64_t slabs = (ra.n + gemvdev::kRows - 1) / gemvdev::kRows;
    constexpr int cols_wg = 4 * gemvtdev::cols_per_wave<XT, NB>();
    const int64_t colblk = (g.x.p + cols_wg - 1) / cols_wg;
    const int64_t nepi = (g.x.p + 255) / 256;

    for (int it = 0; it <= a.max_iter; ++it) {
        if (it > 0) {
            // eta partials of the columns that changed in the last step
            for (int64_t v = blockIdx.x; v < slabs * a.ncg; v += G) {
                gemvdev::eta_update_blk<XT, NB, true>(g.x, a.sel, a.nsel, a.dcoef, 0, B, a.part_upd, a.cstride,
                                                      a.ncg, ra.ctl.active, (int)(v % slabs), (int)(v / slabs));
                __syncthreads();
            }
            if (grid_barrier(br, nwg, &s_flag)) return;
        }
        for (int64_t v = blockIdx.x; v < (int64_t)ra.nfin * B; v += G) {
            riskdev::risk_eta_blk(ra, (int)(v % ra.nfin), (int)(v / ra.nfin), sh);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        for (int64_t v = blockIdx.x; v < (int64_t)ra.ntile * B; v += G) {
            riskdev::risk_scan_w_blk(ra, (int)(v % ra.ntile), (int)(v / ra.ntile), sh);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        for (int64_t v = blockIdx.x; v < (int64_t)ra.ntile * B; v += G) {
            riskdev::risk_scan_q_blk(ra, (int)(v % ra.ntile), (int)(v / ra.ntile), sh, big);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        for (int64_t v = blockIdx.x; v < (int64_t)ra.ntile * B; v += G) {
            riskdev::risk_resid_blk(ra, (int)(v % ra.ntile), (int)(v / ra.ntile), sh, big);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        for (int64_t v = blockIdx.x; v < B; v += G) {
            riskdev::risk_finish_blk(ra, (int)v, sh);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        // the stopping rule has run for this step: leave once no b is active
        // (every workgroup reads the same flags after the barrier)
        int any = 0;
        for (int b = 0; b < B; ++b) any |= ra.ctl.active[b];
        if (!any || it == a.max_iter) break;
        for (int64_t v = blockIdx.x; v < colblk * g.nsplit; v += G) {
            gemvtdev::gemvt_sums_blk<XT, NB, true>(g, (int)(v % colblk), (int)(v / colblk), rchunk);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        for (int64_t v = blockIdx.x; v < nepi; v += G) {
            gemvtdev::gemvt_epilogue_blk(g, (int)v);
            __syncthreads();
        }
        if (grid_barrier(br, nwg, &s_flag)) return;
        if (blockIdx.x == 0) gemvdev::compact_blk<kPT>(g.chg_cnt, g.chg_idx, g.nblk, a.sel_w, a.nsel, ish, sstart, scnt);
        if (grid_barrier(br, nwg, &s_flag)) return;
    }
}

template <int XT, int NB>
hipError_t launch_nb(const PersistArgs& a, const Barrier& br, hipStream_t s, int* grid_out)
{
    const void* fn = reinterpret_cast<const void*>(&fit_persistent_kernel<XT, NB>);
    int dev = 0, per_cu = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPT, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1 || ncu < 1) return hipErrorInvalidConfiguration;
    const int grid = per_cu * ncu;
    *grid_out = grid;
    PersistArgs args = a;
    Barrier bar = br;
    void* kargs[] = {&args, &bar};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPT), kargs, 0, s);
}

template <int XT>
hipError_t launch_xt(const PersistArgs& a, const Barrier& br, hipStream_t s, int* grid_out)
{
    if (a.B <= 1) return launch_nb<XT, 1>(a, br, s, grid_out);
    if (a.B <= 2) return launch_nb<XT, 2>(a, br, s, grid_out);
    if (a.B <= 4) return launch_nb<XT, 4>(a, br, s, grid_out);
    return launch_nb<XT, 8>(a, br, s, grid_out);
}

}  // namespace

int persist_barrier_words() { return kBarLine * 10; }

hipError_t launch_fit_persistent(const PersistArgs& a, unsigned long long* words, double limit_s, hipStream_t s,
                                 int* grid_out)
{
    if (a.B < 1 || a.B > 8 || !a.g.x.vec16 || a.ncg < 1 || a.g.nsplit < 1 || a.g.split_rows % kSplitRows != 0 ||
        a.ra.ntile > kMaxTiles || a.ra.ntile < 1 || a.ra.nfin < 1 || !words)
        return hipErrorInvalidValue;
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    if (khz <= 0) return hipErrorInvalidValue;
    const Barrier br{words, (unsigned long long)(limit_s * 1000.0 * (double)khz), 0};
    switch (a.g.x.xt) {
    case XT_F32: return launch_xt<XT_F32>(a, br, s, grid_out);
    case XT_FP8: return launch_xt<XT_FP8>(a, br, s, grid_out);
    default: return launch_xt<XT_I8>(a, br, s, grid_out);
    }
}

}  // namespace cox
