// api.cpp -- host runtime of libcoxhip: the C ABI declared in include/cox.h.
//
// The context owns the time order and tie groups (computed once on the host),
// the FP64 linear predictor, the FP64 iterate of cox_fit_path and every
// workspace buffer, all allocated in cox_setup for the largest batch and freed
// in cox_destroy.  Every entry point validates its arguments before touching
// the device, and converts every HIP failure into a status code with a message
// kept in the context.  All device work is enqueued on the context's stream.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <limits>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include <unistd.h>

#include "cox.h"
#include "internal.h"
#include "mfma.h"

using namespace cox;

constexpr int kPhases = 9;  // cox_phase values

static_assert(kMfmaVariants == COX_MFMA_VARIANTS && kMfmaEtaVariants == COX_MFMA_ETA_VARIANTS,
              "pipeline shape counts differ from the header");
static_assert(kMfmaEtaVariants <= kMfmaVariants, "tuning times of both passes share one array size");
static_assert(kMaxCov == COX_MAX_COVARIATES, "covariate limit differs from the header");
static_assert(kMaxRefit == COX_MAX_REFIT, "refit column limit differs from the header");

namespace {

constexpr int kMaxBatch = 64;
constexpr int kGroup = 8;  // coefficient vectors per VALU pass over X
constexpr int kFreeCovMaxIter = 100000;  // steps of the unpenalised covariate fit inside cox_lambda_max
constexpr double kFreeCovGtol = 1e-10;   // its stop: max |g_k| below this fraction of its value at zero
constexpr double kPersistWaitLimit = 60.0;  // seconds one grid barrier of the persistent fit may wait

int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

}  // namespace

// Device memory of cox_rank_path_noalloc: a file-scope array that every call on
// one GPU shares (each GPU holds its own copy, at its own address, until the
// process ends), so that the call allocates nothing.  It holds the entry index
// (int32) and the |coefficient| at entry (float) of up to kNoallocMaxCols
// columns.  In host code `scratch` names a host-side stand-in, never the
// device array: kernels and copies take the address hipGetSymbolAddress
// returned for the device, kept in g_scratch_addr.
constexpr int64_t kNoallocMaxCols = int64_t(1) << 21;
static_assert(kNoallocMaxCols == COX_NOALLOC_MAX_COLS, "static scratch size differs from the header");
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[8 * kNoallocMaxCols];
static std::mutex g_scratch_mu;
// device bytes the library holds (contexts and calls' own buffers), for cox_device_bytes
static std::atomic<int64_t> g_dev_bytes{0};
static void* g_scratch_addr[kNoallocMaxDevices] = {};

struct cox_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    XDesc x{};
    int64_t n = 0, p = 0;
    int Bmax = 0;
    int64_t rstride = 0;
    int nblk = 0, ncg = 0, ncb = 0;
    std::string err;
    std::vector<void*> allocs;
    std::vector<size_t> alloc_bytes;
    void* pinned = nullptr;  // small host staging buffer (page-locked)
    size_t pinned_bytes = 0;

    int32_t *perm = nullptr, *gstart = nullptr, *gend = nullptr;
    uint8_t* ev = nullptr;
    // tie groups with events: egidx[k] = g at the last sorted position k of the
    // g-th such group (-1 elsewhere), egcnt[g] = its events
    int32_t *egidx = nullptr, *egcnt = nullptr;
    int64_t n_egroups = 0;
    double *eta = nullptr, *w = nullptr, *S = nullptr, *T = nullptr, *r64 = nullptr;
    float* r32 = nullptr;
    double *part_upd = nullptr, *part_gemv = nullptr;
    int64_t tile = 0;
    int ntile = 0, nfin = 0;
    double* part_xtr = nullptr;  // [nsplit][Bmax][p] split partials of X' r
    // batched matrix-core pass (one-byte allele counts, B > kGroup)
    int8_t* limbs = nullptr;     // [3][Bmax16][rstride]
    int bpad_max = 0;
    double *qscale = nullptr, *rmaxp = nullptr;
    long long* rsump = nullptr;
    int* geno_bad = nullptr;
    int8_t* dlimbs = nullptr;    // [3][Bmax16][dstride] eta-update limbs
    int32_t *sel_all = nullptr, *nsel_all = nullptr;  // 0 .. p - 1 and p: every column, for dense passes
    int32_t* nonfin = nullptr;   // [max_batch] a dense pass's coefficient vector holds a NaN or infinity
    long long* eta_part = nullptr;  // [ncu][2][Bmax16][256] partial sums of blocks two eta workgroups share
    long long* xtr_tail = nullptr;  // [3][Bmax16][ncu * 256] X~' R sums of the split last round (shape 15)
    int ncu = 0;                 // compute units of the device
    int64_t dstride = 0;
    double *dscale = nullptr, *dmaxp = nullptr;
    int xtr_variant = -1, eta_variant = -1;  // pipeline shapes last used (-1: not tuned yet)
    float xtr_tune_ms[kMfmaVariants] = {}, eta_tune_ms[kMfmaVariants] = {};
    int xtr_by_limbs[4] = {-1, -1, -1, -1};  // X~' R shape chosen for 2 and 3 residual limbs
    float xtr_ms_by_limbs[4][kMfmaVariants] = {};
    int geno_state = -1;         // -1 unchecked, 0 counts 0/1/2 only, 1 other values
    int nsplit = 1;
    int64_t split_rows = 0;
    double *bmax = nullptr, *mshift = nullptr, *stot = nullptr, *qtot = nullptr, *Lpart = nullptr, *rpart = nullptr;
    double *beta64 = nullptr, *coef = nullptr, *dcoef = nullptr, *g64 = nullptr;
    double* red_part = nullptr;  // [kRedParts] scratch of the two-level reductions (power iteration)
    int32_t *chg_flag = nullptr, *chg_cnt = nullptr, *chg_idx = nullptr, *sel = nullptr, *nsel = nullptr;
    double *l1old = nullptr, *l1new = nullptr;
    double *L = nullptr, *sumr = nullptr, *lam = nullptr, *fobj = nullptr, *hist = nullptr, *scal = nullptr;
    int32_t *kit = nullptr, *active = nullptr, *iters = nullptr, *status = nullptr;
    // the persistent fit's grid barrier: arrival counter, abort flag, generation words
    unsigned long long* bar_words = nullptr;
    long long* col_count = nullptr;  // columns of X read by eta updates while timing is on
    int persist_grid = 0;  // workgroups of the last persistent launch
    // the state cox_fit_path left (beta64, eta, residual, stopping-rule history) and what
    // produced it, for a resumed call (warm_start = 2); any other call that uses the
    // workspace clears fit_valid
    bool fit_valid = false;
    int fit_B = 0, fit_max_iter = 0, fit_eta_mode = 0, fit_rlimbs = 3;
    int64_t fit_q = 0;
    double fit_step = 0.0;
    std::vector<double> fit_lams;
    int fwd_B = 0, fwd_f64 = 0;
    int64_t n_events = 0;
    // the dense covariate block Z beside X, and the penalty factors
    const float* Z = nullptr;
    int64_t q = 0, ldz = 0;
    int nrb = 0;
    double *cov_part = nullptr, *betaZ = nullptr, *dZ = nullptr, *gZ = nullptr;
    double *l1c_old = nullptr, *l1c_new = nullptr;
    double* pf = nullptr;         // device [p + kMaxCov]: factors of X's columns, then of the covariates
    std::vector<double> pf_host;  // [p + q]
    bool pf_x_custom = false;     // some factor of X's columns differs from 1
    // roctx ranges of the phases (always on: a profiler with marker tracing shows them)
    roctx_range_id_t rx_id[kPhases] = {};
    bool rx_open[kPhases] = {};
    // measurement: event pairs recorded around each phase while timing is on
    bool timing = false;
    std::vector<hipEvent_t> tev[kPhases];
    double tms[kPhases] = {};
    int64_t tcount[kPhases] = {};
};

namespace {

cox_status fail(cox_ctx* c, cox_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

cox_status dev_fail(cox_ctx* c, hipError_t e, const char* what)
{
    return fail(c, COX_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, what)                                \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return dev_fail(c, _e, what); \
    } while (0)

#define STCHK(expr)                        \
    do {                                   \
        cox_status _s = (expr);            \
        if (_s != COX_OK) return _s;       \
    } while (0)

// Allocation-failure injection for tests, from the environment variable
// COXHIP_FAULT: "alloc" fails every device allocation of the library; "alloc@N"
// fails only the N-th one counted from when the variable took that value (a
// value set again after the variable was unset counts from the start), so
// that the clean-up after a failure part way through cox_setup (or through a
// call's own buffers) can be exercised.
bool fault_injected(const char* what)
{
    static std::mutex mu;
    static std::string last;
    static long count = 0;
    const char* f = std::getenv("COXHIP_FAULT");
    if (!f) {
        // unset: the next value starts its count afresh, even if it is the same
        std::lock_guard<std::mutex> lock(mu);
        last.clear();
        return false;
    }
    const size_t w = std::strlen(what);
    if (std::strncmp(f, what, w) != 0) return false;
    if (f[w] == '\0') return true;
    if (f[w] != '@') return false;
    std::lock_guard<std::mutex> lock(mu);
    if (last != f) {
        last = f;
        count = 0;
    }
    return ++count == std::atol(f + w + 1);
}

template <class T>
bool dalloc(cox_ctx* c, T** out, size_t count)
{
    *out = nullptr;
    if (fault_injected("alloc")) return false;
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    c->allocs.push_back(p);
    c->alloc_bytes.push_back(bytes);
    g_dev_bytes += (int64_t)bytes;
    *out = static_cast<T*>(p);
    return true;
}

// Device buffers of one call, freed when the call returns.
struct Scratch {
    std::vector<void*> ptrs;
    int64_t bytes = 0;
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFree(p);
        g_dev_bytes -= bytes;
    }
    template <class T>
    bool get(T** out, size_t count)
    {
        *out = nullptr;
        if (fault_injected("alloc")) return false;
        void* p = nullptr;
        const size_t b = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, b) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        ptrs.push_back(p);
        bytes += (int64_t)b;
        g_dev_bytes += (int64_t)b;
        *out = static_cast<T*>(p);
        return true;
    }
};

void timing_clear(cox_ctx* c)
{
    for (int ph = 0; ph < kPhases; ++ph) {
        for (hipEvent_t e : c->tev[ph]) (void)hipEventDestroy(e);
        c->tev[ph].clear();
        c->tms[ph] = 0;
        c->tcount[ph] = 0;
    }
}

constexpr const char* kPhaseNames[kPhases] = {"cox:xtr", "cox:risk", "cox:eta", "cox:xtr_kernel", "cox:eta_kernel",
                                              "cox:covariates", "cox:refit_hessian", "cox:refit_solve",
                                              "cox:persistent"};

// Mark the begin or the end of phase ph (they alternate): a roctx range on the
// host, and while timing is on an event on the stream.
void tmark(cox_ctx* c, int ph)
{
    if (c->rx_open[ph]) {
        roctxRangeStop(c->rx_id[ph]);
    } else {
        c->rx_id[ph] = roctxRangeStartA(kPhaseNames[ph]);
    }
    c->rx_open[ph] = !c->rx_open[ph];
    if (!c->timing) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    (void)hipEventRecord(e, c->stream);
    c->tev[ph].push_back(e);
}

// A roctx range around one entry-point call.  Phase ranges left open by an
// early error return are closed with it, and their events dropped, so that
// begin and end stay paired in the next call.
struct CallRange {
    cox_ctx* c;
    CallRange(cox_ctx* ctx, const char* name) : c(ctx) { roctxRangePushA(name); }
    ~CallRange()
    {
        if (c) {
            for (int ph = 0; ph < kPhases; ++ph)
                if (c->rx_open[ph]) {
                    roctxRangeStop(c->rx_id[ph]);
                    c->rx_open[ph] = false;
                    if (c->timing && (c->tev[ph].size() & 1)) {
                        (void)hipEventDestroy(c->tev[ph].back());
                        c->tev[ph].pop_back();
                    }
                }
        }
        roctxRangePop();
    }
};

void release(cox_ctx* c)
{
    timing_clear(c);
    for (void* p : c->allocs) (void)hipFree(p);
    for (size_t b : c->alloc_bytes) g_dev_bytes -= (int64_t)b;
    c->allocs.clear();
    c->alloc_bytes.clear();
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
}

// Look up the device address of `scratch` for the context's device (which is
// current), once per device; every later call on that device uses it.
cox_status scratch_init(cox_ctx* c)
{
    if (c->device < 0 || c->device >= kNoallocMaxDevices)
        return fail(c, COX_ERR_UNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[c->device]) return COX_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(c, COX_ERR_DEVICE, std::string("static scratch lookup: ") + hipGetErrorString(e));
    }
    g_scratch_addr[c->device] = ptr;
    return COX_OK;
}

void* scratch_addr(int device)
{
    if (device < 0 || device >= kNoallocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_addr[device];
}

// Section 6's ranking of the columns a path selects: by entry (the first row
// of a decreasing-lambda path where the column is nonzero, i.e. the largest
// lambda), ties by |coef| at entry (larger first), then by index.  Writes the
// ranked columns to order[0..m) when order is not null (sorting in place, no
// allocation) and returns m, the number of entered columns.
int64_t rank_entries(const int32_t* entry, const float* coef, int64_t p, int64_t* order)
{
    int64_t m = 0;
    for (int64_t j = 0; j < p; ++j)
        if (entry[j] >= 0) {
            if (order) order[m] = j;
            ++m;
        }
    if (order)
        std::sort(order, order + m, [&](int64_t a, int64_t b) {
            if (entry[a] != entry[b]) return entry[a] < entry[b];
            if (coef[a] != coef[b]) return coef[a] > coef[b];
            return a < b;
        });
    return m;
}

cox_status check_ctx(cox_ctx* c)
{
    if (!c) return COX_ERR_INVALID_ARG;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, COX_ERR_DEVICE, "hipSetDevice failed");
    return COX_OK;
}

cox_status check_batch(cox_ctx* c, int32_t B)
{
    if (B < 1 || B > c->Bmax)
        return fail(c, COX_ERR_INVALID_ARG, "B must be in 1..max_batch (" + std::to_string(c->Bmax) + ")");
    return COX_OK;
}

cox_status check_lambdas(cox_ctx* c, const double* lambdas, int32_t B)
{
    if (!lambdas) return fail(c, COX_ERR_INVALID_ARG, "lambdas is NULL");
    for (int b = 0; b < B; ++b)
        if (!std::isfinite(lambdas[b]) || lambdas[b] < 0)
            return fail(c, COX_ERR_INVALID_ARG, "lambdas must be finite and >= 0");
    return COX_OK;
}

cox_status sync(cox_ctx* c)
{
    HIPCHK(hipStreamSynchronize(c->stream), "stream synchronize");
    return COX_OK;
}

// Copy m bytes device -> host through the pinned buffer (synchronises).
cox_status d2h(cox_ctx* c, void* host, const void* dev, size_t m)
{
    if (m <= c->pinned_bytes) {
        HIPCHK(hipMemcpyAsync(c->pinned, dev, m, hipMemcpyDeviceToHost, c->stream), "copy to host");
        STCHK(sync(c));
        std::memcpy(host, c->pinned, m);
    } else {
        HIPCHK(hipMemcpyAsync(host, dev, m, hipMemcpyDeviceToHost, c->stream), "copy to host");
        STCHK(sync(c));
    }
    return COX_OK;
}

// Copy m bytes host -> device; the host buffer may be reused on return.
cox_status h2d(cox_ctx* c, void* dev, const void* host, size_t m)
{
    if (m <= c->pinned_bytes) {
        STCHK(sync(c));  // the pinned buffer may still feed an earlier copy
        std::memcpy(c->pinned, host, m);
        HIPCHK(hipMemcpyAsync(dev, c->pinned, m, hipMemcpyHostToDevice, c->stream), "copy to device");
        STCHK(sync(c));
    } else {
        HIPCHK(hipMemcpyAsync(dev, host, m, hipMemcpyHostToDevice, c->stream), "copy to device");
        STCHK(sync(c));
    }
    return COX_OK;
}

const float* geno_scale(const cox_ctx* c) { return c->x.xt == XT_F32 ? nullptr : c->x.scale; }

// Coefficients per vector: X's p columns, then the q covariates.
int64_t ptot(const cox_ctx* c) { return c->p + c->q; }

// Penalty factors of X's columns as the kernels take them (null: all 1).
const double* pf_x(const cox_ctx* c) { return c->pf_x_custom ? c->pf : nullptr; }

CovArgs cov_args(cox_ctx* c) { return CovArgs{c->Z, c->n, c->ldz, (int)c->q, c->nrb, c->cov_part}; }

// Caller's [B][ptot] FP32 coefficients -> the FP64 iterate of X's columns (and the covariates').
cox_status load_beta(cox_ctx* c, const float* beta, int B)
{
    if (c->q)
        HIPCHK(launch_split_coef(beta, c->p, c->q, B, c->beta64, c->betaZ, c->stream), "split coefficients");
    else
        HIPCHK(launch_f32_to_f64(beta, c->beta64, (int64_t)B * c->p, c->stream), "beta to FP64");
    return COX_OK;
}

cox_status store_beta(cox_ctx* c, float* beta, int B)
{
    if (c->q)
        HIPCHK(launch_merge_coef(c->beta64, c->betaZ, c->p, c->q, B, beta, c->stream), "merge coefficients");
    else
        HIPCHK(launch_f64_to_f32(c->beta64, beta, (int64_t)B * c->p, c->stream), "beta to FP32");
    return COX_OK;
}

// eta_b += Z coef_b (no covariates: nothing)
cox_status cov_eta(cox_ctx* c, const double* coef, int B, const int32_t* active)
{
    if (!c->q) return COX_OK;
    tmark(c, COX_PHASE_COV);
    HIPCHK(launch_cov_eta(cov_args(c), coef, B, c->eta, active, c->stream), "Z beta");
    tmark(c, COX_PHASE_COV);
    return COX_OK;
}

// g_Z = Z' r from the residual the risk pass stored (FP64 when it kept one),
// then the epilogue of st (no covariates: nothing).
cox_status cov_grad(cox_ctx* c, const RiskArgs& ra, int B, const int32_t* active, const CovStep& st)
{
    if (!c->q) return COX_OK;
    const CovArgs ca = cov_args(c);
    tmark(c, COX_PHASE_COV);
    HIPCHK(launch_cov_xtr(ca, ra.r64 ? nullptr : ra.r32, c->rstride, ra.r64, B, active, c->stream), "Z' r");
    HIPCHK(launch_cov_epilogue(ca, st, B, c->stream), "Z' r epilogue");
    tmark(c, COX_PHASE_COV);
    return COX_OK;
}

CovStep cov_prox(cox_ctx* c, double step, const int32_t* active)
{
    CovStep st{};
    st.mode = GT_PROX;
    st.beta = c->betaZ;
    st.dbeta = c->dZ;
    st.lam = c->lam;
    st.pf = c->pf + c->p;
    st.step = step;
    st.active = active;
    st.l1old = c->l1c_old;
    st.l1new = c->l1c_new;
    st.ostride = c->q;
    return st;
}

cox_status dense_eta_mfma(cox_ctx* c, const double* coef, int B);
bool use_mfma(cox_ctx* c, int B);

// eta[b] = X~ coef[b] (no centring) for b < B; coef is b-major [B][p].  More
// than 8 vectors over one-byte allele counts go through the matrix cores (three
// passes over X for any B, against one FP64 pass per 8 vectors).
cox_status dense_eta(cox_ctx* c, const double* coef, int B, const double* shift)
{
    tmark(c, COX_PHASE_ETA);
    if (!shift && c->sel_all && use_mfma(c, B)) {
        const cox_status st = dense_eta_mfma(c, coef, B);
        tmark(c, COX_PHASE_ETA);
        return st;
    }
    for (int b0 = 0; b0 < B; b0 += kGroup) {
        const int nb = std::min(kGroup, B - b0);
        HIPCHK(launch_gemv(c->x, coef, b0, nb, c->part_gemv, c->ncb, c->eta, shift, c->stream), "dense X beta");
    }
    tmark(c, COX_PHASE_ETA);
    return COX_OK;
}

// ---- autotuner of the matrix-core pipeline shapes
// A shape is forced by COXHIP_MFMA_VARIANT (the X~' R pass) or COXHIP_ETA_VARIANT
// (the eta update), read from the cache file named by COXHIP_TUNE_CACHE, or
// chosen by timing every shape on the live data (one untimed launch, then the
// median of kTuneReps timed launches; a shape whose launch fails is never
// chosen) and written to that file.  The cache is one JSON object whose keys
// name the pass, the device, its architecture, the source of the kernels
// (COXHIP_SRC_HASH, set by the build) and the problem's shape; each value holds
// the chosen shape and the medians.  Entries that do not parse, name a shape
// out of range or carry another key are ignored, so an old or corrupt file
// leads to a fresh tuning, never to a wrong shape.
#ifndef COXHIP_SRC_HASH
#define COXHIP_SRC_HASH "unknown"
#endif
constexpr int kTuneReps = 3;

int forced_variant(const char* var, int count)
{
    const char* v = std::getenv(var);
    if (!v || !*v) return -1;
    const int k = std::atoi(v);
    return (k >= 0 && k < count) ? k : -1;
}

std::string tune_key(const cox_ctx* c, const char* kernel, int bpad)
{
    hipDeviceProp_t prop{};
    std::string dev = "unknown", arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        dev = prop.name;
        arch = prop.gcnArchName;
    } else {
        (void)hipGetLastError();
    }
    for (char& ch : dev)  // keep the key a plain JSON string
        if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20) ch = '_';
    for (char& ch : arch)
        if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20) ch = '_';
    std::ostringstream os;
    os << kernel << "|" << dev << "|" << arch << "|src:" << COXHIP_SRC_HASH << "|xt" << c->x.xt << "|n" << c->n
       << "|p" << c->p << "|b" << bpad;
    return os.str();
}

// One cache entry per line: "<key>": {"variant": V, "ms": [...]}
bool tune_parse_line(const std::string& line, std::string* key, int* v)
{
    const size_t a = line.find('"');
    if (a == std::string::npos) return false;
    const size_t b = line.find('"', a + 1);
    if (b == std::string::npos) return false;
    const std::string tag = "\"variant\":";
    const size_t t = line.find(tag, b);
    if (t == std::string::npos) return false;
    const char* s = line.c_str() + t + tag.size();
    char* end = nullptr;
    const long val = std::strtol(s, &end, 10);
    if (end == s) return false;
    *key = line.substr(a + 1, b - a - 1);
    *v = (int)val;
    return true;
}

int tune_cache_lookup(const std::string& key, int count)
{
    const char* path = std::getenv("COXHIP_TUNE_CACHE");
    if (!path) return -1;
    std::ifstream f(path);
    std::string line, k;
    int v = -1, found = -1;
    while (std::getline(f, line))
        if (tune_parse_line(line, &k, &v) && k == key && v >= 0 && v < count) found = v;
    return found;
}

void tune_cache_store(const std::string& key, int v, const float* ms, int count)
{
    const char* path = std::getenv("COXHIP_TUNE_CACHE");
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line, k;
        int w;
        while (std::getline(f, line)) {
            if (!tune_parse_line(line, &k, &w) || k == key) continue;
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            keep.push_back(line);
        }
    }
    std::ostringstream e;
    e << "\"" << key << "\": {\"variant\": " << v << ", \"ms\": [";
    for (int i = 0; i < count; ++i) e << (i ? ", " : "") << ms[i];
    e << "]}";
    keep.push_back(e.str());
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream o(tmp, std::ios::trunc);
        o << "{\n";
        for (size_t i = 0; i < keep.size(); ++i) o << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        o << "}\n";
        if (!o) return;
    }
    (void)std::rename(tmp.c_str(), path);
}

// Time launch(variant) -> hipError_t for each of count variants with events on
// the stream: one untimed launch, then the median of kTuneReps timed ones.
// Returns the fastest shape whose launches all succeeded (-1 if none did).
template <class F>
int autotune(cox_ctx* c, int count, F&& launch, float* ms_out)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    int best = -1;
    for (int v = 0; v < count; ++v) {
        ms_out[v] = 0.f;
        bool ok = launch(v) == hipSuccess;
        float t[kTuneReps] = {};
        for (int r = 0; ok && r < kTuneReps; ++r) {
            ok = hipEventRecord(e0, c->stream) == hipSuccess && launch(v) == hipSuccess &&
                 hipEventRecord(e1, c->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
        }
        if (!ok) {
            (void)hipGetLastError();
            continue;
        }
        std::sort(t, t + kTuneReps);
        ms_out[v] = t[kTuneReps / 2];
        if (best < 0 || ms_out[v] < ms_out[best]) best = v;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// Arguments of the matrix-core eta update over the columns sel[0 .. *nsel) for
// vectors 0 .. B - 1, D limbs and scales from launch_quantize_d.
MfmaEtaArgs mfma_eta_args(cox_ctx* c, const int32_t* sel, const int32_t* nsel, int B, const int32_t* active)
{
    MfmaEtaArgs m{c->x.X, c->x.xt, c->n, c->p, c->x.ldx, sel, nsel, c->dlimbs, c->dstride,
                  (int)round_up(B, 16), B, c->dscale, c->eta, active, 0, c->eta_part, c->ncu};
    if (const char* e = std::getenv("COXHIP_ETA_SHARES")) {
        const int v = std::atoi(e);
        if (v > 0 && v <= c->ncu) m.sk_grid = v;
    }
    return m;
}

// The eta update's pipeline shape: forced, cached, or timed once per context on
// these arguments (writing into scratch, since the update is in place).
cox_status pick_eta_variant(cox_ctx* c, MfmaEtaArgs* m)
{
    const int forced = forced_variant("COXHIP_ETA_VARIANT", kMfmaEtaVariants);
    if (forced >= 0) {
        c->eta_variant = forced;
    } else if (c->eta_variant < 0) {
        const std::string key = tune_key(c, "eta", m->bpad);
        c->eta_variant = tune_cache_lookup(key, kMfmaEtaVariants);
        if (c->eta_variant < 0) {
            MfmaEtaArgs t = *m;
            t.eta = c->w;
            c->eta_variant = autotune(
                c, kMfmaEtaVariants, [&](int v) { t.variant = v; return launch_mfma_eta(t, c->stream); },
                c->eta_tune_ms);
            if (c->eta_variant < 0) return fail(c, COX_ERR_DEVICE, "no pipeline shape of the eta update launched");
            tune_cache_store(key, c->eta_variant, c->eta_tune_ms, kMfmaEtaVariants);
        }
    }
    m->variant = c->eta_variant;
    return COX_OK;
}

// eta[b] = X coef[b] for b < B on the matrix cores (one-byte allele counts,
// B > 8), to FP64 accuracy in three passes over X.  Each pass quantises what is
// left of coef_b to integers of at most 22 bits on a per-vector scale q_b (the
// eta update's D limbs, every column selected), adds q_b X R_b to eta with
// exact integer sums, and leaves coef_b - q_b R_b (one fma) for the next pass.
// What remains after three passes is at most 2^-69 max|coef_b|.  Integer limbs
// cannot carry a NaN or an infinity, so a vector holding one gets eta = NaN,
// as the FP64 passes would give it.
cox_status dense_eta_mfma(cox_ctx* c, const double* coef, int B)
{
    const int bpad = (int)round_up(B, 16);
    HIPCHK(launch_fill_i32(c->nonfin, 0, B, c->stream), "clear flags");
    HIPCHK(launch_nonfinite(coef, c->p, B, c->nonfin, c->stream), "coefficient check");
    HIPCHK(launch_fill_f64(c->eta, 0.0, (int64_t)B * c->n, c->stream), "clear eta");
    MfmaEtaArgs m = mfma_eta_args(c, c->sel_all, c->nsel_all, B, nullptr);
    for (int k = 0; k < 3; ++k) {
        const double* src = k == 0 ? coef : c->dcoef;
        HIPCHK(launch_quantize_d(src, c->p, c->sel_all, c->nsel_all, B, c->dmaxp, c->dlimbs, c->dstride, bpad,
                                 c->dscale, c->stream),
               "quantise coefficients");
        if (k == 0) STCHK(pick_eta_variant(c, &m));
        tmark(c, COX_PHASE_ETA_KERNEL);
        HIPCHK(launch_mfma_eta(m, c->stream), "dense X beta on matrix cores");
        tmark(c, COX_PHASE_ETA_KERNEL);
        if (k < 2) HIPCHK(launch_coef_remainder(src, c->dcoef, c->p, B, c->dscale, c->stream), "coefficient remainder");
    }
    HIPCHK(launch_poison_eta(c->eta, c->n, B, c->nonfin, c->stream), "non-finite coefficients");
    return COX_OK;
}

// The matrix-core pass serves batches of more than kGroup vectors when X holds
// allele counts (checked once over the whole matrix).
bool use_mfma(cox_ctx* c, int B)
{
    if (!c->limbs || B <= kGroup) return false;
    const char* off = std::getenv("COXHIP_NO_MFMA");
    if (off && off[0] == '1') return false;
    if (c->geno_state < 0) {
        int bad = 1;
        if (launch_fill_i32(c->geno_bad, 0, 1, c->stream) == hipSuccess &&
            launch_geno_check(c->x.X, c->x.xt, c->n, c->p, c->x.ldx, c->geno_bad, c->stream) == hipSuccess &&
            hipMemcpyAsync(&bad, c->geno_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
            hipStreamSynchronize(c->stream) == hipSuccess) {
            c->geno_state = bad ? 1 : 0;
        } else {
            (void)hipGetLastError();
            return false;
        }
    }
    return c->geno_state == 0;
}

RiskArgs risk_args(cox_ctx* c, int B)
{
    RiskArgs a{};
    a.n = c->n;
    a.B = B;
    a.ord = Order{c->perm, c->gstart, c->gend, c->ev};
    a.eta_in = c->eta;
    a.eta_in_f32 = 0;
    a.eta = c->eta;
    a.part = nullptr;
    a.ncg = c->ncg;
    a.part_cstride = (int64_t)c->Bmax * c->n;
    a.nsel = c->nsel;
    a.w = c->w;
    a.S = c->S;
    a.T = c->T;
    a.tile = c->tile;
    a.ntile = c->ntile;
    a.nfin = c->nfin;
    a.bmax = c->bmax;
    a.mshift = c->mshift;
    a.stot = c->stot;
    a.qtot = c->qtot;
    a.Lpart = c->Lpart;
    a.rpart = c->rpart;
    a.r32 = c->r32;
    a.r64 = nullptr;
    a.L = c->L;
    a.sumr = c->sumr;
    a.rstride = c->rstride;
    a.use_ctl = 0;
    if (use_mfma(c, B)) {  // the matrix-core pass quantises the FP64 residual itself
        a.r32 = nullptr;
        a.r64 = c->r64;
    }
    return a;
}

GemvtArgs gemvt_args(cox_ctx* c, int mode)
{
    GemvtArgs g{};
    g.x = c->x;
    g.r32 = c->r32;
    g.rstride = c->rstride;
    g.part = c->part_xtr;
    g.nsplit = c->nsplit;
    g.split_rows = c->split_rows;
    g.part_sstride = (int64_t)c->Bmax * c->p;
    g.sumr = c->sumr;
    g.mode = mode;
    g.ostride = c->p;
    g.pf = pf_x(c);
    g.nblk = c->nblk;
    g.dcoef = c->dcoef;
    g.chg_flag = c->chg_flag;
    g.chg_cnt = c->chg_cnt;
    g.chg_idx = c->chg_idx;
    g.l1old = c->l1old;
    g.l1new = c->l1new;
    return g;
}

// X~' r for B vectors: the matrix-core pass (residual in rlimbs int8 limbs)
// when X holds allele counts and B > kGroup, else the vector pass.
cox_status run_gemvt(cox_ctx* c, GemvtArgs g, int B, int rlimbs = 3)
{
    if (use_mfma(c, B)) {
        tmark(c, COX_PHASE_XTR);
        const int bpad = (int)round_up(B, 16);
        HIPCHK(launch_quantize(c->r64, c->n, B, c->rmaxp, c->rsump, c->limbs, c->rstride, bpad, rlimbs, c->qscale,
                               c->sumr, c->stream),
               "quantise r");
        MfmaArgs m{c->x.X,   c->x.xt, c->n, c->p,      c->x.ldx,     c->limbs, c->rstride,
                   bpad,     rlimbs,  B,    c->qscale, c->part_xtr, 0};
        m.tail = c->xtr_tail;
        m.tail_cols = (int64_t)c->ncu * 256;
        m.ncu = c->ncu;
        int& chosen = c->xtr_by_limbs[rlimbs];
        const int forced = forced_variant("COXHIP_MFMA_VARIANT", kMfmaVariants);
        if (forced >= 0) {
            chosen = forced;
        } else if (chosen < 0) {
            const std::string key = tune_key(c, rlimbs == 3 ? "xtr" : "xtr2", bpad);
            chosen = tune_cache_lookup(key, kMfmaVariants);
            if (chosen < 0) {
                chosen = autotune(
                    c, kMfmaVariants, [&](int v) { m.variant = v; return launch_mfma_xtr(m, c->stream); },
                    c->xtr_ms_by_limbs[rlimbs]);
                if (chosen < 0) return fail(c, COX_ERR_DEVICE, "no pipeline shape of the X' R pass launched");
                tune_cache_store(key, chosen, c->xtr_ms_by_limbs[rlimbs], kMfmaVariants);
            }
        }
        c->xtr_variant = chosen;
        std::copy(c->xtr_ms_by_limbs[rlimbs], c->xtr_ms_by_limbs[rlimbs] + kMfmaVariants, c->xtr_tune_ms);
        m.variant = chosen;
        tmark(c, COX_PHASE_XTR_KERNEL);
        HIPCHK(launch_mfma_xtr(m, c->stream), "X' R on matrix cores");
        tmark(c, COX_PHASE_XTR_KERNEL);
        g.b0 = 0;
        g.nb = B;
        g.nsplit = 1;
        g.first_group = 1;
        HIPCHK(launch_gemvt_epilogue(g, c->stream), "X' r epilogue");
        tmark(c, COX_PHASE_XTR);
        return COX_OK;
    }
    tmark(c, COX_PHASE_XTR);
    for (int b0 = 0; b0 < B; b0 += kGroup) {
        g.b0 = b0;
        g.nb = std::min(kGroup, B - b0);
        g.first_group = b0 == 0;
        tmark(c, COX_PHASE_XTR_KERNEL);
        HIPCHK(launch_gemvt_sums(g, c->stream), "X' r");
        tmark(c, COX_PHASE_XTR_KERNEL);
        HIPCHK(launch_gemvt_epilogue(g, c->stream), "X' r epilogue");
    }
    tmark(c, COX_PHASE_XTR);
    return COX_OK;
}

// Uniform [-1, 1) start vector from SplitMix64 (Steele, Lea and Flood 2014),
// top 53 bits of each output.
void splitmix_start(uint64_t seed, std::vector<double>& v)
{
    uint64_t st = seed;
    double nv = 0.0;
    for (double& x : v) {
        uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        x = (double)(z >> 11) * 0x1.0p-52 - 1.0;
        nv += x * x;
    }
    nv = std::sqrt(nv);
    for (double& x : v) x /= nv;
}

// ||Z||_2^2 of the covariate block by power iteration (tol 1e-6, at most 1000
// steps, the SplitMix64 start of seed 95376).  Uses eta, betaZ, dZ and gZ.
cox_status opnorm2_cov(cox_ctx* c, double* s2)
{
    const int q = (int)c->q;
    std::vector<double> v(q);
    splitmix_start(95376, v);
    STCHK(h2d(c, c->betaZ, v.data(), sizeof(double) * q));
    CovStep raw{};
    raw.mode = GT_RAW;
    raw.out64 = c->gZ;
    raw.ostride = q;
    const CovArgs ca = cov_args(c);
    double est = 0.0, prev = 0.0;
    for (int it = 0; it < 1000; ++it) {
        HIPCHK(launch_fill_f64(c->eta, 0.0, c->n, c->stream), "zero");
        HIPCHK(launch_cov_eta(ca, c->betaZ, 1, c->eta, nullptr, c->stream), "Z v");
        HIPCHK(launch_dot(c->eta, c->eta, c->n, c->red_part, c->scal + 1, c->stream), "norm of Z v");
        HIPCHK(launch_cov_xtr(ca, nullptr, 0, c->eta, 1, nullptr, c->stream), "Z' u");
        HIPCHK(launch_cov_epilogue(ca, raw, 1, c->stream), "Z' u");
        HIPCHK(launch_fill_f64(c->scal + 2, 0.0, 1, c->stream), "zero");
        HIPCHK(launch_sqnorm_add(c->gZ, q, c->scal + 2, c->stream), "norm of Z' u");
        double h[2];
        STCHK(d2h(c, h, c->scal + 1, sizeof(h)));
        prev = est;
        est = h[0];
        if (!std::isfinite(est) || !std::isfinite(h[1])) return fail(c, COX_ERR_NUMERIC, "non-finite power iteration");
        if (h[1] == 0.0) break;
        HIPCHK(launch_normalize(c->gZ, c->scal + 2, nullptr, c->betaZ, c->dZ, q, c->stream), "normalise");
        if (it > 0 && std::fabs(est - prev) < 1e-6 * est) break;
    }
    *s2 = est;
    return COX_OK;
}

// The unpenalised optimum over the covariates whose penalty factor is 0, with
// every other coefficient zero: ISTA on Z alone (a penalised covariate gets an
// infinite threshold and stays at zero) with step 1/(2 ||Z||^2), until
// max_k |g_k| over the free covariates falls below kFreeCovGtol times its value
// at zero.  Leaves betaZ, eta and the risk-set state (residual ra stores) at
// that point.  eta must be zero on entry.
cox_status fit_free_covariates(cox_ctx* c, const RiskArgs& ra)
{
    const int q = (int)c->q;
    double s2 = 0.0;
    STCHK(opnorm2_cov(c, &s2));
    if (!(s2 > 0)) return fail(c, COX_ERR_NUMERIC, "the covariate block is zero");
    const double step = 1.0 / (2.0 * s2), inf = std::numeric_limits<double>::infinity();
    STCHK(h2d(c, c->lam, &inf, sizeof(double)));
    HIPCHK(launch_fill_f64(c->betaZ, 0.0, q, c->stream), "zero");
    HIPCHK(launch_fill_f64(c->eta, 0.0, c->n, c->stream), "zero");
    CovStep st = cov_prox(c, step, nullptr);
    st.out64 = c->gZ;
    std::vector<double> gz(q);
    double g0 = -1.0;
    bool done = false;
    for (int it = 0; it < kFreeCovMaxIter && !done; ++it) {
        HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
        STCHK(cov_grad(c, ra, 1, nullptr, st));  // g at beta_it, then beta_{it+1}
        STCHK(cov_eta(c, c->dZ, 1, nullptr));
        if (it % 4 == 0) {
            STCHK(d2h(c, gz.data(), c->gZ, sizeof(double) * q));
            double gm = 0.0;
            for (int k = 0; k < q; ++k)
                if (c->pf_host[c->p + k] == 0.0) gm = std::max(gm, std::fabs(gz[k]));
            if (!std::isfinite(gm)) return fail(c, COX_ERR_NUMERIC, "non-finite covariate gradient");
            if (g0 < 0) g0 = gm;
            done = gm <= kFreeCovGtol * g0;
        }
    }
    HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
    if (!done) return fail(c, COX_ERR_NOT_CONVERGED, "the unpenalised covariate fit did not converge");
    return COX_OK;
}

}  // namespace

extern "C" {

const char* cox_status_string(cox_status s)
{
    switch (s) {
    case COX_OK: return "ok";
    case COX_ERR_INVALID_ARG: return "invalid argument";
    case COX_ERR_OUT_OF_MEMORY: return "out of memory";
    case COX_ERR_DEVICE: return "device error";
    case COX_ERR_NUMERIC: return "non-finite loss or gradient";
    case COX_ERR_NOT_CONVERGED: return "maximum number of iterations reached";
    case COX_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

cox_status cox_last_error(const cox_ctx* ctx, char* buf, size_t len)
{
    if (!ctx || !buf || len == 0) return COX_ERR_INVALID_ARG;
    const size_t m = std::min(len - 1, ctx->err.size());
    std::memcpy(buf, ctx->err.data(), m);
    buf[m] = '\0';
    return COX_OK;
}

cox_status cox_setup(cox_ctx** out, const cox_matrix* X, const double* time, const int32_t* event,
                     int32_t max_batch, void* hip_stream)
{
    if (!out) return COX_ERR_INVALID_ARG;
    *out = nullptr;
    if (!X || !X->X || !time || !event) return COX_ERR_INVALID_ARG;
    if (X->xtype != COX_X_F32 && X->xtype != COX_X_FP8_E4M3 && X->xtype != COX_X_INT8) return COX_ERR_INVALID_ARG;
    if (X->n < 1 || X->p < 1 || X->n >= (1LL << 31) || X->p >= (1LL << 31) || X->ldx < X->n) return COX_ERR_INVALID_ARG;
    if (X->ldx > (int64_t(1) << 62) / X->p) return COX_ERR_INVALID_ARG;
    if (X->xtype == COX_X_F32 && (X->col_center || X->col_scale)) return COX_ERR_INVALID_ARG;
    if (max_batch < 1 || max_batch > kMaxBatch) return COX_ERR_INVALID_ARG;
    const int64_t n = X->n, p = X->p;
    int64_t nev = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(time[i])) return COX_ERR_INVALID_ARG;
        if (event[i] != 0 && event[i] != 1) return COX_ERR_INVALID_ARG;
        nev += event[i];
    }

    cox_ctx* c = new (std::nothrow) cox_ctx;
    if (!c) return COX_ERR_OUT_OF_MEMORY;
    c->n_events = nev;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return COX_ERR_DEVICE;
    }
    if (c->device < kNoallocMaxDevices && scratch_init(c) != COX_OK) {
        delete c;
        return COX_ERR_DEVICE;
    }
    c->n = n;
    c->p = p;
    c->Bmax = max_batch;
    const size_t elem = X->xtype == COX_X_F32 ? 4 : 1;
    const uintptr_t base = reinterpret_cast<uintptr_t>(X->X);
    c->x = XDesc{X->X, X->xtype, n, p, X->ldx, X->col_center, X->col_scale,
                 (int)(base % 16 == 0 && (X->ldx * (int64_t)elem) % 16 == 0),
                 (int)(base % 4 == 0 && (X->ldx * (int64_t)elem) % 4 == 0)};
    c->rstride = round_up(n, kSplitRows);
    c->nblk = (int)((p + kGemvtCols - 1) / kGemvtCols);
    const int64_t nslab = (n + kUpdRows - 1) / kUpdRows;
    c->ncg = (int)std::max<int64_t>(1, std::min<int64_t>(4, 512 / nslab));
    c->ncb = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + nslab - 1) / nslab, (p + 255) / 256));
    c->tile = 1024 * std::max<int64_t>(1, (n + 1024LL * kMaxTiles - 1) / (1024LL * kMaxTiles));
    c->ntile = (int)((n + c->tile - 1) / c->tile);
    c->nfin = (int)((n + kFinElems - 1) / kFinElems);
    c->nrb = cov_row_blocks(n);
    c->pf_host.assign(p, 1.0);
    {   // row splits of X' r: enough workgroups for several even rounds over the chip
        const int64_t cols_wg = X->xtype == COX_X_F32 ? 16 : 64;
        const int64_t wgs = (p + cols_wg - 1) / cols_wg;
        const int64_t nchunks = (n + kSplitRows - 1) / kSplitRows;
        const int64_t target = std::max<int64_t>(1, (12288 + wgs - 1) / wgs);
        const int64_t ns = std::min(nchunks, target);
        const int64_t spc = (nchunks + ns - 1) / ns;
        c->split_rows = spc * kSplitRows;
        c->nsplit = (int)((nchunks + spc - 1) / spc);
    }

    // Order by non-increasing time, stable; tie groups (Section 5.3, Section 6).
    std::vector<int32_t> perm(n), gs(n), ge(n);
    std::vector<uint8_t> evs(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return time[a] > time[b]; });
    for (int64_t k = 0; k < n;) {
        int64_t e = k;
        while (e + 1 < n && time[perm[e + 1]] == time[perm[k]]) ++e;
        for (int64_t q = k; q <= e; ++q) {
            gs[q] = (int32_t)k;
            ge[q] = (int32_t)e;
        }
        k = e + 1;
    }
    for (int64_t k = 0; k < n; ++k) evs[k] = (uint8_t)event[perm[k]];
    std::vector<int32_t> egi(n, -1), egc;
    for (int64_t k = 0; k < n; ++k) {
        if (ge[k] != k) continue;
        int32_t cnt = 0;
        for (int64_t q = gs[k]; q <= k; ++q) cnt += evs[q];
        if (cnt > 0) {
            egi[k] = (int32_t)egc.size();
            egc.push_back(cnt);
        }
    }
    c->n_egroups = (int64_t)egc.size();

    const int64_t Bn = (int64_t)max_batch * n, Bp = (int64_t)max_batch * p;
    bool ok = dalloc(c, &c->perm, n) && dalloc(c, &c->gstart, n) && dalloc(c, &c->gend, n) && dalloc(c, &c->ev, n) &&
              dalloc(c, &c->egidx, n) && dalloc(c, &c->egcnt, std::max<size_t>(1, egc.size())) &&
              dalloc(c, &c->eta, Bn) && dalloc(c, &c->w, Bn) && dalloc(c, &c->S, Bn) && dalloc(c, &c->T, Bn) &&
              dalloc(c, &c->r64, Bn) && dalloc(c, &c->r32, (size_t)max_batch * c->rstride) &&
              dalloc(c, &c->part_upd, (size_t)c->ncg * Bn) && dalloc(c, &c->part_gemv, (size_t)std::max<int64_t>((int64_t)c->ncb * kGroup, (int64_t)gemv16_blocks(n, p) * 4) * n) &&
              dalloc(c, &c->beta64, Bp) && dalloc(c, &c->coef, Bp) && dalloc(c, &c->dcoef, Bp) &&
              dalloc(c, &c->g64, Bp) && dalloc(c, &c->chg_flag, p) && dalloc(c, &c->chg_cnt, c->nblk) &&
              dalloc(c, &c->chg_idx, (size_t)c->nblk * kGemvtCols) && dalloc(c, &c->sel, p) &&
              dalloc(c, &c->nsel, 1) && dalloc(c, &c->l1old, (size_t)max_batch * c->nblk) &&
              dalloc(c, &c->l1new, (size_t)max_batch * c->nblk) && dalloc(c, &c->L, max_batch) &&
              dalloc(c, &c->sumr, max_batch) && dalloc(c, &c->lam, max_batch) && dalloc(c, &c->fobj, max_batch) &&
              dalloc(c, &c->hist, (size_t)max_batch * kMaxHist) && dalloc(c, &c->scal, 16) &&
              dalloc(c, &c->kit, max_batch) && dalloc(c, &c->active, max_batch) && dalloc(c, &c->iters, max_batch) &&
              dalloc(c, &c->status, max_batch) && dalloc(c, &c->bmax, (size_t)max_batch * c->nfin) &&
              dalloc(c, &c->mshift, max_batch) && dalloc(c, &c->stot, (size_t)max_batch * c->ntile) &&
              dalloc(c, &c->qtot, (size_t)max_batch * c->ntile) && dalloc(c, &c->Lpart, (size_t)max_batch * c->ntile) &&
              dalloc(c, &c->rpart, (size_t)max_batch * c->ntile) &&
              dalloc(c, &c->part_xtr, (size_t)c->nsplit * Bp) &&
              dalloc(c, &c->cov_part, (size_t)max_batch * cov_row_blocks(n) * kMaxCov) &&
              dalloc(c, &c->betaZ, (size_t)max_batch * kMaxCov) && dalloc(c, &c->dZ, (size_t)max_batch * kMaxCov) &&
              dalloc(c, &c->gZ, (size_t)max_batch * kMaxCov) && dalloc(c, &c->l1c_old, max_batch) &&
              dalloc(c, &c->l1c_new, max_batch) && dalloc(c, &c->pf, p + kMaxCov) &&
              dalloc(c, &c->bar_words, persist_barrier_words()) && dalloc(c, &c->col_count, 1) &&
              dalloc(c, &c->red_part, kRedParts);
    const bool mfma_able = X->xtype != COX_X_F32 && c->x.vec16 && max_batch > kGroup;
    if (ok && mfma_able) {
        c->bpad_max = (int)round_up(max_batch, 16);
        const int nt = mfma_ntile(n);
        c->dstride = round_up(p, 64);
        ok = dalloc(c, &c->limbs, (size_t)3 * c->bpad_max * c->rstride) && dalloc(c, &c->qscale, max_batch) &&
             dalloc(c, &c->rmaxp, (size_t)max_batch * nt) && dalloc(c, &c->rsump, (size_t)max_batch * nt) &&
             dalloc(c, &c->geno_bad, 1) && dalloc(c, &c->dlimbs, (size_t)3 * c->bpad_max * c->dstride) &&
             dalloc(c, &c->dscale, max_batch) && dalloc(c, &c->dmaxp, (size_t)max_batch * ((c->dstride + 4095) / 4096)) &&
             dalloc(c, &c->sel_all, p) && dalloc(c, &c->nsel_all, 1) && dalloc(c, &c->nonfin, max_batch);
        if (ok && hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
            (void)hipGetLastError();
            c->ncu = 0;
        }
        if (ok && c->ncu > 0)
            ok = dalloc(c, &c->eta_part, (size_t)c->ncu * 2 * c->bpad_max * 256) &&
                 dalloc(c, &c->xtr_tail, (size_t)3 * c->bpad_max * c->ncu * 256);
    }
    if (ok) {
        c->pinned_bytes = 64 * 1024;
        if (hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->pinned = nullptr;
            ok = false;
        }
    }
    if (!ok) {
        release(c);
        delete c;
        return COX_ERR_OUT_OF_MEMORY;
    }
    cox_status st = COX_OK;
    auto up = [&](void* d, const void* h, size_t m) {
        if (st == COX_OK && hipMemcpyAsync(d, h, m, hipMemcpyHostToDevice, c->stream) != hipSuccess) st = COX_ERR_DEVICE;
    };
    up(c->perm, perm.data(), sizeof(int32_t) * n);
    up(c->gstart, gs.data(), sizeof(int32_t) * n);
    up(c->gend, ge.data(), sizeof(int32_t) * n);
    up(c->ev, evs.data(), n);
    up(c->egidx, egi.data(), sizeof(int32_t) * n);
    if (!egc.empty()) up(c->egcnt, egc.data(), sizeof(int32_t) * egc.size());
    auto chk = [&](hipError_t e) {
        if (st == COX_OK && e != hipSuccess) st = COX_ERR_DEVICE;
    };
    chk(launch_fill_f64(reinterpret_cast<double*>(c->r32), 0.0, (int64_t)max_batch * c->rstride / 2, c->stream));
    chk(launch_fill_i32(c->chg_flag, 0, p, c->stream));
    chk(launch_fill_i32(c->nsel, 0, 1, c->stream));
    chk(launch_fill_f64(c->eta, 0.0, Bn, c->stream));
    chk(launch_fill_f64(c->pf, 1.0, p, c->stream));
    chk(launch_fill_f64(c->pf + p, 0.0, kMaxCov, c->stream));
    if (c->limbs)
        chk(launch_fill_f64(reinterpret_cast<double*>(c->limbs), 0.0, (int64_t)3 * c->bpad_max * c->rstride / 8,
                            c->stream));
    if (c->sel_all) {
        chk(launch_iota_i32(c->sel_all, p, c->stream));
        chk(launch_fill_i32(c->nsel_all, (int32_t)p, 1, c->stream));
    }
    if (st == COX_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = COX_ERR_DEVICE;
    if (st != COX_OK) {
        (void)hipGetLastError();
        release(c);
        delete c;
        return st;
    }
    *out = c;
    return COX_OK;
}

cox_status cox_destroy(cox_ctx* c)
{
    if (!c) return COX_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
    return COX_OK;
}

cox_status cox_loss_grad(cox_ctx* c, const float* beta, int32_t B, double* loss, float* grad)
{
    CallRange range(c, "cox_loss_grad");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!beta || !loss) return fail(c, COX_ERR_INVALID_ARG, "beta and loss must not be NULL");
    STCHK(check_batch(c, B));
    STCHK(load_beta(c, beta, B));
    HIPCHK(launch_scale_coef(c->beta64, geno_scale(c), c->coef, c->p, B, c->stream), "coefficients");
    STCHK(dense_eta(c, c->coef, B, nullptr));
    STCHK(cov_eta(c, c->betaZ, B, nullptr));
    RiskArgs ra = risk_args(c, B);
    if (!grad) ra.r32 = nullptr;
    HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
    if (grad) {
        GemvtArgs g = gemvt_args(c, GT_GRAD);
        g.out32 = grad;
        g.ostride = ptot(c);
        STCHK(run_gemvt(c, g, B));
        CovStep st{};
        st.mode = GT_GRAD;
        st.out32 = grad + c->p;
        st.ostride = ptot(c);
        STCHK(cov_grad(c, ra, B, nullptr, st));
    }
    std::vector<double> L(B);
    STCHK(d2h(c, L.data(), c->L, sizeof(double) * B));
    bool finite = true;
    for (int b = 0; b < B; ++b) {
        loss[b] = -L[b];
        finite = finite && std::isfinite(loss[b]);
    }
    if (!finite) return fail(c, COX_ERR_NUMERIC, "non-finite loss");
    return COX_OK;
}

cox_status cox_prox_step(cox_ctx* c, float* beta, int32_t B, const double* lambdas, double step, double* obj_before)
{
    CallRange range(c, "cox_prox_step");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!beta) return fail(c, COX_ERR_INVALID_ARG, "beta is NULL");
    STCHK(check_batch(c, B));
    STCHK(check_lambdas(c, lambdas, B));
    if (!(step > 0) || !std::isfinite(step)) return fail(c, COX_ERR_INVALID_ARG, "step must be finite and > 0");
    STCHK(h2d(c, c->lam, lambdas, sizeof(double) * B));
    STCHK(load_beta(c, beta, B));
    HIPCHK(launch_scale_coef(c->beta64, geno_scale(c), c->coef, c->p, B, c->stream), "coefficients");
    STCHK(dense_eta(c, c->coef, B, nullptr));
    STCHK(cov_eta(c, c->betaZ, B, nullptr));
    const RiskArgs ra = risk_args(c, B);
    HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
    GemvtArgs g = gemvt_args(c, GT_PROX);
    g.beta = c->beta64;
    g.lam = c->lam;
    g.step = step;
    g.active = nullptr;
    STCHK(run_gemvt(c, g, B));
    STCHK(cov_grad(c, ra, B, nullptr, cov_prox(c, step, nullptr)));
    STCHK(store_beta(c, beta, B));
    if (obj_before) {
        HIPCHK(launch_rowsum(c->l1old, c->nblk, B, 1.0, c->scal, c->stream), "l1 norm");
        std::vector<double> v(3 * B, 0.0);
        STCHK(d2h(c, v.data(), c->L, sizeof(double) * B));
        STCHK(d2h(c, v.data() + B, c->scal, sizeof(double) * B));
        if (c->q) STCHK(d2h(c, v.data() + 2 * B, c->l1c_old, sizeof(double) * B));
        bool finite = true;
        for (int b = 0; b < B; ++b) {
            obj_before[b] = -v[b] + lambdas[b] * (v[B + b] + v[2 * B + b]);
            finite = finite && std::isfinite(obj_before[b]);
        }
        if (!finite) return fail(c, COX_ERR_NUMERIC, "non-finite objective");
    }
    return COX_OK;
}

cox_status cox_prox_apply(cox_ctx* c, float* beta, const float* grad, int32_t B, const double* lambdas, double step)
{
    CallRange range(c, "cox_prox_apply");
    STCHK(check_ctx(c));
    if (!beta || !grad) return fail(c, COX_ERR_INVALID_ARG, "beta and grad must not be NULL");
    STCHK(check_batch(c, B));
    STCHK(check_lambdas(c, lambdas, B));
    if (!(step > 0) || !std::isfinite(step)) return fail(c, COX_ERR_INVALID_ARG, "step must be finite and > 0");
    STCHK(h2d(c, c->lam, lambdas, sizeof(double) * B));
    HIPCHK(launch_prox_apply(beta, grad, c->lam, (c->pf_x_custom || c->q) ? c->pf : nullptr, step, ptot(c), B,
                             c->stream),
           "soft threshold");
    return COX_OK;
}

cox_status cox_lambda_max(cox_ctx* c, double* lambda_max)
{
    CallRange range(c, "cox_lambda_max");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!lambda_max) return fail(c, COX_ERR_INVALID_ARG, "lambda_max is NULL");
    const int64_t p = c->p, q = c->q;
    for (int64_t j = 0; j < p; ++j)
        if (c->pf_host[j] == 0.0)
            return fail(c, COX_ERR_UNSUPPORTED, "lambda_max: only covariates may have a zero penalty factor");
    bool free_cov = false;
    for (int64_t k = 0; k < q; ++k) free_cov = free_cov || c->pf_host[p + k] == 0.0;
    HIPCHK(launch_fill_f64(c->eta, 0.0, c->n, c->stream), "zero eta");
    RiskArgs ra = risk_args(c, 1);
    ra.r64 = c->r64;
    cox_status conv = COX_OK;
    if (free_cov) {
        conv = fit_free_covariates(c, ra);
        if (conv != COX_OK && conv != COX_ERR_NOT_CONVERGED) return conv;
    } else {
        HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
    }
    GemvtArgs g = gemvt_args(c, GT_RAW);
    g.out64 = c->g64;
    STCHK(run_gemvt(c, g, 1));
    std::vector<double> gh(p + q);
    if (q) {
        CovStep st{};
        st.mode = GT_RAW;
        st.out64 = c->gZ;
        st.ostride = q;
        STCHK(cov_grad(c, ra, 1, nullptr, st));
        STCHK(d2h(c, gh.data() + p, c->gZ, sizeof(double) * q));
    }
    STCHK(d2h(c, gh.data(), c->g64, sizeof(double) * p));
    double mx = 0.0;
    for (int64_t j = 0; j < p + q; ++j)
        if (c->pf_host[j] > 0.0) mx = std::max(mx, std::fabs(gh[j]) / c->pf_host[j]);
    if (!std::isfinite(mx)) return fail(c, COX_ERR_NUMERIC, "non-finite gradient");
    *lambda_max = mx;
    return conv == COX_OK ? COX_OK : fail(c, conv, "the unpenalised covariate fit did not converge");
}

cox_status cox_opnorm2(cox_ctx* c, double tol, int32_t maxiter, uint64_t seed, double* s2, int32_t* iters)
{
    CallRange range(c, "cox_opnorm2");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!s2 || !(tol >= 0) || maxiter < 1) return fail(c, COX_ERR_INVALID_ARG, "bad opnorm2 arguments");
    const int q = (int)c->q;
    std::vector<double> v(ptot(c));
    splitmix_start(seed, v);
    STCHK(h2d(c, c->beta64, v.data(), sizeof(double) * c->p));
    if (q) STCHK(h2d(c, c->betaZ, v.data() + c->p, sizeof(double) * q));
    CovStep raw{};
    raw.mode = GT_RAW;
    raw.out64 = c->gZ;
    raw.ostride = q;
    const float* scale = geno_scale(c);
    const bool centred = c->x.xt != XT_F32 && c->x.center;
    HIPCHK(launch_scale_coef(c->beta64, scale, c->coef, c->p, 1, c->stream), "coefficients");
    double est = 0.0, prev = 0.0;
    int it = 0;
    while (it < maxiter) {
        if (centred)
            HIPCHK(launch_center_shift(c->x.center, scale, c->beta64, c->p, c->red_part, c->scal + 0, c->stream),
                   "shift");
        STCHK(dense_eta(c, c->coef, 1, centred ? c->scal + 0 : nullptr));
        STCHK(cov_eta(c, c->betaZ, 1, nullptr));
        HIPCHK(launch_dot(c->eta, c->eta, c->n, c->red_part, c->scal + 1, c->stream), "norm of X v");
        HIPCHK(launch_to_r32(c->eta, nullptr, c->r32, c->sumr, c->n, c->red_part, c->stream), "u to FP32");
        GemvtArgs g = gemvt_args(c, GT_RAW);
        g.out64 = c->g64;
        STCHK(run_gemvt(c, g, 1));
        HIPCHK(launch_dot(c->g64, c->g64, c->p, c->red_part, c->scal + 2, c->stream), "norm of X' u");
        if (q) {
            RiskArgs ru{};
            ru.r32 = c->r32;
            STCHK(cov_grad(c, ru, 1, nullptr, raw));
            HIPCHK(launch_sqnorm_add(c->gZ, q, c->scal + 2, c->stream), "norm of Z' u");
        }
        double h[2];
        STCHK(d2h(c, h, c->scal + 1, sizeof(h)));
        ++it;
        prev = est;
        est = h[0];
        if (!std::isfinite(est) || !std::isfinite(h[1])) return fail(c, COX_ERR_NUMERIC, "non-finite power iteration");
        if (h[1] == 0.0) break;
        HIPCHK(launch_normalize(c->g64, c->scal + 2, scale, c->beta64, c->coef, c->p, c->stream), "normalise");
        if (q) HIPCHK(launch_normalize(c->gZ, c->scal + 2, nullptr, c->betaZ, c->dZ, q, c->stream), "normalise");
        if (it > 1 && std::fabs(est - prev) < tol * est) break;
    }
    *s2 = est;
    if (iters) *iters = it;
    return COX_OK;
}

cox_status cox_fit_path(cox_ctx* c, const double* lambdas, int32_t B, const cox_fit_opts* opts_in, float* beta,
                        int32_t* iters, double* obj)
{
    CallRange range(c, "cox_fit_path");
    STCHK(check_ctx(c));
    if (!beta) return fail(c, COX_ERR_INVALID_ARG, "beta is NULL");
    STCHK(check_batch(c, B));
    STCHK(check_lambdas(c, lambdas, B));
    cox_fit_opts o{1000, 1e-5, 10, 0.0, 0, 0, 0, 0, 16, 0, nullptr};
    if (opts_in) o = *opts_in;
    if (o.max_iter < 0 || !(o.tol >= 0) || o.lag < 1 || o.lag > kMaxHist - 1 || !std::isfinite(o.step) ||
        (o.warm_start < 0 || o.warm_start > 2) || (o.eta_mode != 0 && o.eta_mode != 1) ||
        (o.persistent != 0 && o.persistent != 1) || (o.deterministic != 0 && o.deterministic != 1) ||
        (o.residual_bits != 0 && o.residual_bits != 22 && o.residual_bits != 14))
        return fail(c, COX_ERR_INVALID_ARG, "bad cox_fit_opts");
    if (o.trace && (int64_t)B * ((int64_t)o.max_iter + 1) > (int64_t(1) << 31))
        return fail(c, COX_ERR_INVALID_ARG, "trace: B * (max_iter + 1) is too large");
    if (o.persistent && (use_mfma(c, B) || B > kGroup || o.eta_mode != 0 || c->q != 0 || !c->x.vec16))
        return fail(c, COX_ERR_UNSUPPORTED,
                    "persistent = 1 serves the vector path: B <= 8 (not the batched matrix-core pass), eta_mode 0, "
                    "no covariate block, X 16-byte aligned with ldx * element size a multiple of 16");
    const int rlimbs = o.residual_bits == 14 ? 2 : 3;
    const int poll = o.poll > 0 ? o.poll : 16;
    const bool resume = o.warm_start == 2;
    if (resume) {
        if (o.persistent) return fail(c, COX_ERR_UNSUPPORTED, "resume: not served by the persistent form");
        if (!c->fit_valid)
            return fail(c, COX_ERR_INVALID_ARG, "resume: the last call on this context was not a completed fit");
        if (B != c->fit_B || !std::equal(lambdas, lambdas + B, c->fit_lams.begin()) || o.eta_mode != c->fit_eta_mode ||
            rlimbs != c->fit_rlimbs || c->q != c->fit_q || (o.step > 0 && o.step != c->fit_step) ||
            o.max_iter < c->fit_max_iter)
            return fail(c, COX_ERR_INVALID_ARG,
                        "resume: B, lambdas, step, eta_mode, residual_bits and covariates must be those of the "
                        "fit it continues, and max_iter at least its max_iter");
    }
    c->fit_valid = false;
    double step = resume ? c->fit_step : o.step;
    if (step <= 0) {
        double s2 = 0;
        STCHK(cox_opnorm2(c, 1e-6, 1000, 95376, &s2, nullptr));
        if (!(s2 > 0)) return fail(c, COX_ERR_NUMERIC, "||X||_2 is zero; no step size");
        step = 1.0 / (2.0 * s2);
    }
    STCHK(h2d(c, c->lam, lambdas, sizeof(double) * B));
    const int64_t Bp = (int64_t)B * c->p, Bn = (int64_t)B * c->n;
    const int q = (int)c->q;
    if (resume) {
        // the iterate, eta and the stopping-rule state stay as the last fit left them; the
        // lambdas that stopped at its max_iter go on from there
        HIPCHK(launch_resume(c->status, c->active, c->kit, c->iters, B, c->stream), "resume");
    } else if (o.warm_start) {
        STCHK(load_beta(c, beta, B));
        HIPCHK(launch_scale_coef(c->beta64, geno_scale(c), c->coef, c->p, B, c->stream), "coefficients");
        STCHK(dense_eta(c, c->coef, B, nullptr));
        STCHK(cov_eta(c, c->betaZ, B, nullptr));
        HIPCHK(launch_l1_blocks(c->beta64, pf_x(c), c->p, B, c->nblk, c->l1new, c->stream), "l1 blocks");
        if (q) HIPCHK(launch_cov_l1(c->betaZ, c->pf + c->p, q, B, c->l1c_new, c->stream), "covariate l1");
    } else {
        HIPCHK(launch_fill_f64(c->beta64, 0.0, Bp, c->stream), "zero beta");
        HIPCHK(launch_fill_f64(c->eta, 0.0, Bn, c->stream), "zero eta");
        HIPCHK(launch_fill_f64(c->l1new, 0.0, (int64_t)B * c->nblk, c->stream), "zero l1");
        if (q) {
            HIPCHK(launch_fill_f64(c->betaZ, 0.0, (int64_t)B * q, c->stream), "zero beta");
            HIPCHK(launch_fill_f64(c->l1c_new, 0.0, B, c->stream), "zero l1");
        }
    }
    if (!resume) {
        HIPCHK(launch_fill_i32(c->nsel, 0, 1, c->stream), "reset");
        HIPCHK(launch_fill_i32(c->kit, 0, B, c->stream), "reset");
        HIPCHK(launch_fill_i32(c->active, 1, B, c->stream), "reset");
        HIPCHK(launch_fill_i32(c->status, 0, B, c->stream), "reset");
        HIPCHK(launch_fill_i32(c->iters, 0, B, c->stream), "reset");
        HIPCHK(launch_fill_f64(c->hist, 0.0, (int64_t)B * kMaxHist, c->stream), "reset");
    }

    const bool mfma = use_mfma(c, B);
    RiskArgs ra = risk_args(c, B);
    ra.part = (o.eta_mode == 0 && !mfma) ? c->part_upd : nullptr;
    ra.use_ctl = 1;
    ra.ctl = FitCtl{c->lam, c->l1new, c->nblk, c->hist, c->kit, c->active, c->iters, c->status, c->fobj,
                    q ? c->l1c_new : nullptr, o.max_iter, o.lag, o.tol, nullptr, 0};
    Scratch call;
    const int64_t tstride = (int64_t)o.max_iter + 1;
    if (o.trace) {  // the objective of every step, written by the stopping-rule kernel
        if (!call.get(&ra.ctl.trace, (size_t)(B * tstride)))
            return fail(c, COX_ERR_OUT_OF_MEMORY, "objective trace");
        ra.ctl.trace_stride = tstride;
        HIPCHK(launch_fill_f64(ra.ctl.trace, std::numeric_limits<double>::quiet_NaN(), B * tstride, c->stream),
               "reset trace");
    }
    const CovStep cst = cov_prox(c, step, c->active);
    GemvtArgs g = gemvt_args(c, GT_PROX);
    g.beta = c->beta64;
    g.lam = c->lam;
    g.step = step;
    g.active = c->active;
    const int64_t cstride = (int64_t)c->Bmax * c->n;

    if (o.persistent) {
        PersistArgs pa{ra, g, c->sel, c->sel, c->nsel, c->dcoef, c->part_upd, cstride, c->ncg, o.max_iter, B};
        pa.g.b0 = 0;
        pa.g.nb = B;
        pa.g.first_group = 1;
        HIPCHK(launch_fill_f64(reinterpret_cast<double*>(c->bar_words), 0.0, persist_barrier_words(), c->stream),
               "reset");
        tmark(c, COX_PHASE_PERSISTENT);
        HIPCHK(launch_fit_persistent(pa, c->bar_words, kPersistWaitLimit, c->stream, &c->persist_grid),
               "persistent fit");
        tmark(c, COX_PHASE_PERSISTENT);
        unsigned long long aborted = 0;
        STCHK(d2h(c, &aborted, c->bar_words + persist_abort_word(), sizeof(aborted)));
        if (aborted)
            return fail(c, COX_ERR_DEVICE, "persistent fit: a grid barrier waited past its limit; launch abandoned");
    }
    // a resumed fit starts where the last one ended: after the risk-set pass of
    // its last step, with that step's proximal update still to take
    const int it0 = resume ? c->fit_max_iter : 0;
    for (int it = it0; it <= o.max_iter && !o.persistent; ++it) {
        const bool first_resumed = resume && it == it0;
        if (it > 0 && !first_resumed) {
            if (o.eta_mode == 0 && mfma) {
                tmark(c, COX_PHASE_ETA);
                const int bpad = (int)round_up(B, 16);
                HIPCHK(launch_quantize_d(c->dcoef, c->p, c->sel, c->nsel, B, c->dmaxp, c->dlimbs, c->dstride, bpad,
                                         c->dscale, c->stream),
                       "quantise eta update");
                MfmaEtaArgs m = mfma_eta_args(c, c->sel, c->nsel, B, c->active);
                STCHK(pick_eta_variant(c, &m));
                tmark(c, COX_PHASE_ETA_KERNEL);
                HIPCHK(launch_mfma_eta(m, c->stream), "eta update on matrix cores");
                tmark(c, COX_PHASE_ETA_KERNEL);
                tmark(c, COX_PHASE_ETA);
            } else if (o.eta_mode == 0) {
                tmark(c, COX_PHASE_ETA);
                for (int b0 = 0; b0 < B; b0 += kGroup)
                    HIPCHK(launch_eta_update(c->x, c->sel, c->nsel, c->dcoef, b0, std::min(kGroup, B - b0),
                                             c->part_upd, cstride, c->ncg, c->active, c->stream),
                           "eta update");
                tmark(c, COX_PHASE_ETA);
            } else {
                HIPCHK(launch_scale_coef(c->beta64, geno_scale(c), c->coef, c->p, B, c->stream), "coefficients");
                STCHK(dense_eta(c, c->coef, B, nullptr));
            }
            // the covariates' share: a fresh eta needs all of Z beta_Z, an updated one the change
            STCHK(cov_eta(c, o.eta_mode == 1 ? c->betaZ : c->dZ, B, o.eta_mode == 1 ? nullptr : c->active));
        }
        if (!first_resumed) {
            tmark(c, COX_PHASE_RISK);
            HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
            tmark(c, COX_PHASE_RISK);
        }
        if (it < o.max_iter) {
            STCHK(run_gemvt(c, g, B, rlimbs));
            STCHK(cov_grad(c, ra, B, c->active, cst));
            if (o.eta_mode == 0) {
                HIPCHK(launch_compact(c->chg_cnt, c->chg_idx, c->nblk, c->sel, c->nsel, c->stream), "compact");
                if (c->timing) HIPCHK(launch_count_add(c->nsel, c->col_count, c->stream), "column count");
            }
        }
        if ((it + 1) % poll == 0 && it < o.max_iter) {
            std::vector<int32_t> act(B);
            STCHK(d2h(c, act.data(), c->active, sizeof(int32_t) * B));
            if (std::all_of(act.begin(), act.end(), [](int32_t a) { return a == 0; })) break;
        }
    }
    STCHK(store_beta(c, beta, B));
    std::vector<int32_t> st(B), itv(B);
    std::vector<double> fo(B);
    STCHK(d2h(c, st.data(), c->status, sizeof(int32_t) * B));
    STCHK(d2h(c, itv.data(), c->iters, sizeof(int32_t) * B));
    STCHK(d2h(c, fo.data(), c->fobj, sizeof(double) * B));
    if (iters) std::copy(itv.begin(), itv.end(), iters);
    if (obj) std::copy(fo.begin(), fo.end(), obj);
    if (o.trace) STCHK(d2h(c, o.trace, ra.ctl.trace, sizeof(double) * (size_t)(B * tstride)));
    bool numeric = false, notconv = false;
    for (int b = 0; b < B; ++b) {
        numeric = numeric || st[b] == 3;
        notconv = notconv || st[b] == 2 || st[b] == 0;
    }
    if (numeric) return fail(c, COX_ERR_NUMERIC, "non-finite objective");
    if (!o.persistent) {
        c->fit_valid = true;
        c->fit_B = B;
        c->fit_lams.assign(lambdas, lambdas + B);
        c->fit_step = step;
        c->fit_eta_mode = o.eta_mode;
        c->fit_rlimbs = rlimbs;
        c->fit_q = c->q;
        c->fit_max_iter = o.max_iter;
    }
    if (notconv) return fail(c, COX_ERR_NOT_CONVERGED, "max_iter reached");
    return COX_OK;
}

cox_status cox_fit_sequence(cox_ctx* c, const double* lambdas, int32_t L, const cox_fit_opts* opts_in,
                            float* beta_path, int32_t* iters, double* obj)
{
    CallRange range(c, "cox_fit_sequence");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!beta_path || L < 1) return fail(c, COX_ERR_INVALID_ARG, "beta_path is NULL or L < 1");
    STCHK(check_lambdas(c, lambdas, L));
    cox_fit_opts o{1000, 1e-5, 10, 0.0, 0, 0, 0, 0, 16, 0, nullptr};
    if (opts_in) o = *opts_in;
    if (o.step <= 0) {  // one step size for the whole sequence
        double s2 = 0;
        STCHK(cox_opnorm2(c, 1e-6, 1000, 95376, &s2, nullptr));
        if (!(s2 > 0)) return fail(c, COX_ERR_NUMERIC, "||X||_2 is zero; no step size");
        o.step = 1.0 / (2.0 * s2);
    }
    const int64_t pt = ptot(c);
    bool notconv = false;
    for (int32_t l = 0; l < L; ++l) {
        float* bl = beta_path + (int64_t)l * pt;
        cox_fit_opts ol = o;
        if (o.trace) ol.trace = o.trace + (int64_t)l * ((int64_t)o.max_iter + 1);
        if (l > 0) {
            HIPCHK(hipMemcpyAsync(bl, bl - pt, sizeof(float) * pt, hipMemcpyDeviceToDevice, c->stream),
                   "previous solution");
            ol.warm_start = 1;
        }
        int32_t it = 0;
        double f = 0;
        const cox_status st = cox_fit_path(c, lambdas + l, 1, &ol, bl, &it, &f);
        if (iters) iters[l] = it;
        if (obj) obj[l] = f;
        if (st == COX_ERR_NOT_CONVERGED)
            notconv = true;
        else if (st != COX_OK)
            return st;
    }
    if (notconv) return fail(c, COX_ERR_NOT_CONVERGED, "max_iter reached for some lambda");
    return COX_OK;
}

cox_status cox_set_covariates(cox_ctx* c, const float* Z, int64_t q, int64_t ldz)
{
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (q < 0 || q > kMaxCov) return fail(c, COX_ERR_INVALID_ARG, "q must be in 0..COX_MAX_COVARIATES");
    if (q > 0 && (!Z || ldz < c->n || ldz > (int64_t(1) << 40)))
        return fail(c, COX_ERR_INVALID_ARG, "Z is NULL or ldz < n");
    STCHK(sync(c));  // work already enqueued may still read the previous block
    c->Z = q ? Z : nullptr;
    c->q = q;
    c->ldz = q ? ldz : 0;
    c->pf_host.resize(c->p + q);
    std::fill(c->pf_host.begin() + c->p, c->pf_host.end(), 0.0);
    HIPCHK(launch_fill_f64(c->pf + c->p, 0.0, kMaxCov, c->stream), "covariate penalty factors");
    STCHK(sync(c));
    return COX_OK;
}

cox_status cox_set_penalty_factors(cox_ctx* c, const double* pf)
{
    STCHK(check_ctx(c));
    c->fit_valid = false;
    const int64_t pt = ptot(c);
    std::vector<double> v(pt);
    if (pf) {
        for (int64_t j = 0; j < pt; ++j) {
            if (!std::isfinite(pf[j]) || pf[j] < 0)
                return fail(c, COX_ERR_INVALID_ARG, "penalty factors must be finite and >= 0");
            v[j] = pf[j];
        }
    } else {
        std::fill(v.begin(), v.begin() + c->p, 1.0);
        std::fill(v.begin() + c->p, v.end(), 0.0);
    }
    STCHK(sync(c));  // work already enqueued may still read the previous factors
    HIPCHK(hipMemcpyAsync(c->pf, v.data(), sizeof(double) * pt, hipMemcpyHostToDevice, c->stream),
           "penalty factors");
    STCHK(sync(c));
    c->pf_host = v;
    c->pf_x_custom = std::any_of(v.begin(), v.begin() + c->p, [](double f) { return f != 1.0; });
    return COX_OK;
}

}  // extern "C"

extern "C" {

cox_status cox_refit(cox_ctx* c, const int64_t* cols, int32_t m, const cox_refit_opts* opts_in, double* coef,
                     double* se, double* pval, double* loglik, int32_t* iters)
{
    CallRange range(c, "cox_refit");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    const int q = (int)c->q, M = m + q;
    const int64_t n = c->n;
    if (m < 0 || M < 1 || M > kMaxRefit || (m > 0 && !cols) || !coef)
        return fail(c, COX_ERR_INVALID_ARG, "refit needs 1..COX_MAX_REFIT columns (chosen + covariates) and coef");
    std::vector<int32_t> cols32(std::max(m, 1));
    for (int a = 0; a < m; ++a) {
        if (cols[a] < 0 || cols[a] >= c->p) return fail(c, COX_ERR_INVALID_ARG, "refit column out of range");
        cols32[a] = (int32_t)cols[a];
    }
    {
        std::vector<int32_t> sorted(cols32.begin(), cols32.begin() + m);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(c, COX_ERR_INVALID_ARG, "refit columns must be distinct");
    }
    cox_refit_opts o{50, 1e-8};
    if (opts_in) o = *opts_in;
    if (o.max_iter < 0 || !(o.gtol >= 0) || !std::isfinite(o.gtol))
        return fail(c, COX_ERR_INVALID_ARG, "bad cox_refit_opts");
    for (int a = 0; a < M; ++a)
        if (!std::isfinite(coef[a])) return fail(c, COX_ERR_INVALID_ARG, "coef must be finite");

    const int64_t G = c->n_egroups, ldd = refit_ld(n), ldp = refit_ld(G);
    const int nc1 = gram_chunks(n, M), nc2 = gram_chunks(G, M), nch = scan_chunks(n), nrb = refit_row_blocks(n);
    const size_t MM = (size_t)M * M;
    Scratch w;
    float* D;
    double *Pg, *wg, *wt, *rs, *csum, *p1, *p2, *H, *g, *d, *b, *bt, *gpart, *sed, *pvd;
    int32_t* colsd;
    int* okd;
    if (!(w.get(&D, (size_t)M * ldd) && w.get(&Pg, (size_t)(M + 1) * ldp) && w.get(&wg, ldp) && w.get(&wt, ldd) &&
          w.get(&rs, n) &&
          w.get(&csum, (size_t)(M + 1) * nch) && w.get(&p1, nc1 * MM) && w.get(&p2, nc2 * MM) && w.get(&H, MM) &&
          w.get(&g, M) && w.get(&d, M) && w.get(&b, M) && w.get(&bt, M) && w.get(&gpart, (size_t)nrb * M) &&
          w.get(&sed, M) && w.get(&pvd, M) && w.get(&colsd, std::max(m, 1)) && w.get(&okd, 1)))
        return fail(c, COX_ERR_OUT_OF_MEMORY, "refit workspace");

    if (m > 0) {
        STCHK(h2d(c, colsd, cols32.data(), sizeof(int32_t) * m));
        HIPCHK(launch_gather_cols(c->x, colsd, m, c->perm, D, ldd, c->stream), "gather columns");
    }
    if (q) HIPCHK(launch_gather_z(c->Z, c->ldz, n, q, c->perm, D + (size_t)m * ldd, ldd, c->stream), "gather covariates");
    STCHK(h2d(c, b, coef, sizeof(double) * M));

    RiskArgs ra = risk_args(c, 1);
    ra.r32 = nullptr;
    ra.r64 = c->r64;
    auto eval = [&](const double* bb, double* Lout) -> cox_status {
        HIPCHK(launch_refit_eta(D, ldd, n, M, c->perm, bb, c->eta, c->stream), "D b");
        HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
        STCHK(d2h(c, Lout, c->L, sizeof(double)));
        if (!std::isfinite(*Lout)) return fail(c, COX_ERR_NUMERIC, "non-finite log likelihood");
        return COX_OK;
    };
    auto hessian = [&]() -> cox_status {
        tmark(c, COX_PHASE_REFIT_HESSIAN);
        const RefitHess hs{D, ldd, n, M, c->perm, c->ev, c->w, c->r64, c->egidx, c->egcnt, G, ldp,
                           wt, csum, Pg, wg, p1, p2, H};
        HIPCHK(launch_refit_hessian(hs, c->stream), "Hessian");
        tmark(c, COX_PHASE_REFIT_HESSIAN);
        tmark(c, COX_PHASE_REFIT_SOLVE);
        HIPCHK(launch_chol(H, M, okd, c->stream), "Cholesky");
        tmark(c, COX_PHASE_REFIT_SOLVE);
        int ok = 0;
        STCHK(d2h(c, &ok, okd, sizeof(int)));
        if (!ok) return fail(c, COX_ERR_NUMERIC, "the information matrix is not positive definite");
        return COX_OK;
    };

    double L = 0.0;
    STCHK(eval(b, &L));
    std::vector<double> gh(M), dh(M);
    bool converged = false;
    int it = 0;
    for (;; ++it) {
        HIPCHK(launch_refit_grad(D, ldd, n, M, c->perm, c->r64, rs, gpart, g, c->stream), "D' r");
        STCHK(d2h(c, gh.data(), g, sizeof(double) * M));
        double gmax = 0.0;
        for (double v : gh) gmax = std::max(gmax, std::fabs(v));
        if (!std::isfinite(gmax)) return fail(c, COX_ERR_NUMERIC, "non-finite gradient");
        if (gmax <= o.gtol) {
            converged = true;
            break;
        }
        if (it >= o.max_iter) break;
        STCHK(hessian());
        tmark(c, COX_PHASE_REFIT_SOLVE);
        HIPCHK(launch_chol_solve(H, M, g, d, c->stream), "Newton direction");
        tmark(c, COX_PHASE_REFIT_SOLVE);
        STCHK(d2h(c, dh.data(), d, sizeof(double) * M));
        double gain = 0.0;
        for (int a = 0; a < M; ++a) gain += gh[a] * dh[a];
        // once the predicted gain is at the rounding level of L the full step is
        // taken unchecked; otherwise it is halved until L does not fall
        const bool pure = gain <= 1e-12 * (1.0 + std::fabs(L));
        double t = 1.0, Lt = -std::numeric_limits<double>::infinity();
        for (int half = 0; half < 60; ++half, t *= 0.5) {
            HIPCHK(launch_axpy(b, d, t, M, bt, c->stream), "trial step");
            const cox_status st = eval(bt, &Lt);
            if (st != COX_OK && st != COX_ERR_NUMERIC) return st;
            if (st == COX_OK && (Lt >= L || pure)) break;
        }
        if (!(Lt >= L) && !pure) {  // no ascent at the rounding level of L: stay
            STCHK(eval(b, &L));
            break;
        }
        std::swap(b, bt);
        L = Lt;
    }
    STCHK(hessian());
    HIPCHK(launch_wald(H, M, b, sed, pvd, c->stream), "Wald statistics");
    STCHK(d2h(c, coef, b, sizeof(double) * M));
    if (se) STCHK(d2h(c, se, sed, sizeof(double) * M));
    if (pval) STCHK(d2h(c, pval, pvd, sizeof(double) * M));
    if (loglik) *loglik = L;
    if (iters) *iters = it;
    if (!converged) return fail(c, COX_ERR_NOT_CONVERGED, "refit: gradient above gtol at the stop");
    return COX_OK;
}

cox_status cox_rank_path(cox_ctx* c, const float* path, int32_t L, int32_t* entry, float* entry_coef, int64_t* order,
                         int64_t* n_entered)
{
    CallRange range(c, "cox_rank_path");
    STCHK(check_ctx(c));
    if (!path || L < 1 || !entry) return fail(c, COX_ERR_INVALID_ARG, "rank_path needs path, L >= 1 and entry");
    const int64_t p = c->p;
    Scratch w;
    int32_t* ed;
    float* cd;
    if (!(w.get(&ed, p) && w.get(&cd, p))) return fail(c, COX_ERR_OUT_OF_MEMORY, "rank workspace");
    HIPCHK(launch_entry(path, L, ptot(c), p, ed, cd, c->stream), "entry points");
    std::vector<float> coefv(p);
    STCHK(d2h(c, entry, ed, sizeof(int32_t) * p));
    STCHK(d2h(c, coefv.data(), cd, sizeof(float) * p));
    if (entry_coef) std::copy(coefv.begin(), coefv.end(), entry_coef);
    const int64_t m = rank_entries(entry, coefv.data(), p, order);
    if (n_entered) *n_entered = m;
    return COX_OK;
}

cox_status cox_rank_path_noalloc(cox_ctx* c, const float* path, int32_t L, int32_t* entry, float* entry_coef,
                                 int64_t* order, int64_t* n_entered)
{
    CallRange range(c, "cox_rank_path_noalloc");
    STCHK(check_ctx(c));
    if (!path || L < 1 || !entry || !entry_coef)
        return fail(c, COX_ERR_INVALID_ARG, "rank_path_noalloc needs path, L >= 1, entry and entry_coef");
    const int64_t p = c->p;
    if (p > kNoallocMaxCols)
        return fail(c, COX_ERR_UNSUPPORTED, "rank_path_noalloc serves at most " + std::to_string(kNoallocMaxCols) +
                                                " columns (its static scratch); use cox_rank_path");
    unsigned char* base = static_cast<unsigned char*>(scratch_addr(c->device));
    if (!base) STCHK(scratch_init(c));
    base = static_cast<unsigned char*>(scratch_addr(c->device));
    // the entry kernel writes every one of the p entries it later reads, so the
    // previous call's contents need no clearing
    int32_t* ed = reinterpret_cast<int32_t*>(base);
    float* cd = reinterpret_cast<float*>(base + 4 * kNoallocMaxCols);
    HIPCHK(launch_entry(path, L, ptot(c), p, ed, cd, c->stream), "entry points");
    STCHK(d2h(c, entry, ed, sizeof(int32_t) * p));
    STCHK(d2h(c, entry_coef, cd, sizeof(float) * p));
    const int64_t m = rank_entries(entry, entry_coef, p, order);
    if (n_entered) *n_entered = m;
    return COX_OK;
}

cox_status cox_nll_forward(cox_ctx* c, const void* eta, int32_t eta_f64, int32_t B, double* loss)
{
    CallRange range(c, "cox_nll_forward");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!eta || !loss || (eta_f64 != 0 && eta_f64 != 1)) return fail(c, COX_ERR_INVALID_ARG, "bad nll_forward arguments");
    STCHK(check_batch(c, B));
    RiskArgs ra = risk_args(c, B);
    ra.eta_in = eta;
    ra.eta_in_f32 = !eta_f64;
    ra.r32 = nullptr;
    ra.r64 = c->r64;
    HIPCHK(launch_risk(ra, c->stream), "risk-set sums");
    HIPCHK(launch_rowsum(c->L, 1, B, -1.0, loss, c->stream), "negate");
    c->fwd_B = B;
    c->fwd_f64 = eta_f64;
    return COX_OK;
}

cox_status cox_nll_backward(cox_ctx* c, const double* grad_loss, int32_t B, void* grad_eta)
{
    CallRange range(c, "cox_nll_backward");
    STCHK(check_ctx(c));
    c->fit_valid = false;
    if (!grad_loss || !grad_eta) return fail(c, COX_ERR_INVALID_ARG, "bad nll_backward arguments");
    if (B != c->fwd_B) return fail(c, COX_ERR_INVALID_ARG, "backward needs a forward with the same B");
    HIPCHK(launch_nll_backward(c->r64, grad_loss, c->n, B, grad_eta, c->fwd_f64, c->stream), "adjoint");
    return COX_OK;
}

cox_status cox_mfma_tuning(cox_ctx* c, int32_t* xtr_variant, int32_t* eta_variant, float* xtr_ms, float* eta_ms)
{
    STCHK(check_ctx(c));
    if (xtr_variant) *xtr_variant = c->xtr_variant;
    if (eta_variant) *eta_variant = c->eta_variant;
    for (int v = 0; v < kMfmaVariants; ++v) {
        if (xtr_ms) xtr_ms[v] = c->xtr_tune_ms[v];
        if (eta_ms) eta_ms[v] = c->eta_tune_ms[v];
    }
    return COX_OK;
}

cox_status cox_timing_enable(cox_ctx* c, int32_t enable)
{
    STCHK(check_ctx(c));
    STCHK(sync(c));
    timing_clear(c);
    c->timing = enable != 0;
    HIPCHK(launch_fill_f64(reinterpret_cast<double*>(c->col_count), 0.0, 1, c->stream), "reset column count");
    return COX_OK;
}

cox_status cox_device_bytes(int64_t* bytes)
{
    if (!bytes) return COX_ERR_INVALID_ARG;
    *bytes = g_dev_bytes.load();
    return COX_OK;
}

cox_status cox_timing_columns(cox_ctx* c, int64_t* eta_columns)
{
    STCHK(check_ctx(c));
    if (!eta_columns) return fail(c, COX_ERR_INVALID_ARG, "eta_columns is NULL");
    long long v = 0;
    STCHK(d2h(c, &v, c->col_count, sizeof(v)));
    *eta_columns = (int64_t)v;
    return COX_OK;
}

cox_status cox_timing_read(cox_ctx* c, int32_t phase, double* total_ms, int64_t* count)
{
    STCHK(check_ctx(c));
    if (phase < 0 || phase >= kPhases || !total_ms) return fail(c, COX_ERR_INVALID_ARG, "bad timing_read arguments");
    STCHK(sync(c));
    auto& ev = c->tev[phase];
    for (size_t q = 0; q + 1 < ev.size(); q += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ev[q], ev[q + 1]), "event time");
        c->tms[phase] += ms;
        c->tcount[phase] += 1;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    *total_ms = c->tms[phase];
    if (count) *count = c->tcount[phase];
    return COX_OK;
}

}  // extern "C"
