// mcdc_run_noalloc: the history form of mcdc_run with every per-run device
// buffer (tally and leakage sums per batch and copy, detector sums, event
// counters, overflow flag, the persistent launch's work counter) carved
// from one file-scope device array instead of allocated, for callers that
// cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "mcdc_internal.hpp"

using namespace mcdc;

namespace {

constexpr size_t kScratchBytes = (size_t)MCDC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code the name
// stands for the host-side shadow, not the device memory: host code reaches
// the array only through the address hipGetSymbolAddress returns per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DevScratch {
    unsigned char *ptr = nullptr;     // device address of this GPU's copy of scratch
    hipEvent_t a = nullptr, b = nullptr;   // run timing
    bool ready = false;
};

std::mutex &scratch_mutex() {
    static std::mutex m;
    return m;
}
DevScratch g_scratch[kMaxDevices];

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

// Set-up on the first call on a device (that device current): the array's
// device address and the two timing events.  Later calls only look it up.
int scratch_of(int dev, DevScratch **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(MCDC_E_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> g(scratch_mutex());
    DevScratch &d = g_scratch[dev];
    if (!d.ready) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        if ((e = hipEventCreate(&d.a)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        if ((e = hipEventCreate(&d.b)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        d.ptr = (unsigned char *)ptr;
        d.ready = true;
    }
    *out = &d;
    return MCDC_OK;
}

size_t pad256(size_t b) { return (b + 255) & ~size_t(255); }

// Scratch layout of a run: [S][L][qoi sums][counters][overflow][work].
struct Layout {
    int X, XL;
    size_t off_L, off_q, off_c, off_o, off_w, total;
};

Layout layout_for(const DevProblem &P, int B, int X, int XL) {
    Layout l{};
    l.X = X;
    l.XL = XL;
    const size_t nS = (size_t)B * X * (size_t)P.tstride * sizeof(double);
    const size_t nL = (size_t)B * XL * (size_t)P.K * P.G * 6 * sizeof(double);
    l.off_L = pad256(nS);
    l.off_q = l.off_L + pad256(nL);
    l.off_c = l.off_q + 256;
    l.off_o = l.off_c + pad256(kCounters * sizeof(unsigned long long));
    l.off_w = l.off_o + 256;
    l.total = l.off_w + 256;
    return l;
}

}  // namespace

extern "C" int mcdc_run_noalloc(mcdc_problem *p, uint64_t n_histories, uint64_t seed,
                                const mcdc_run_options *opt_in, mcdc_result *out) {
    if (!p) return fail(MCDC_E_INVALID, "invalid argument: problem is NULL");
    if (!out) return fail(MCDC_E_INVALID, "invalid argument: result is NULL");
    if (n_histories == 0) return fail(MCDC_E_INVALID, "invalid argument: n_histories must be > 0");
    mcdc_run_options opt{};
    if (opt_in) opt = *opt_in;
    if (opt.algorithm != MCDC_ALG_HISTORY)
        return fail(MCDC_E_UNSUPPORTED, "mcdc_run_noalloc runs the history form only (algorithm = MCDC_ALG_HISTORY)");
    if (opt.debug_counts || opt.debug_scores || opt.profile || opt.pc_target)
        return fail(MCDC_E_UNSUPPORTED, "mcdc_run_noalloc takes no debug arrays, profile or population control");
    if (out->host_outputs)
        return fail(MCDC_E_UNSUPPORTED, "mcdc_run_noalloc writes device outputs only (host_outputs = 0)");
    const DevProblem &P = p->d;
    if (has_progeny(P))
        return fail(MCDC_E_UNSUPPORTED,
                    "mcdc_run_noalloc runs analog problems only (no weight windows, fission or implicit capture)");
    if (p->h.B > 1023) return fail(MCDC_E_UNSUPPORTED, "at most 1023 batches");

    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    DevScratch *ds = nullptr;
    int rc = scratch_of(p->device, &ds);
    if (rc) return rc;

    // tally copies as mcdc_run's history form takes them (up to 32, 256
    // leakage copies), halved until the run fits the scratch array
    const int B = (int)((uint64_t)p->h.B < n_histories ? (uint64_t)p->h.B : n_histories);
    int X = 32;
    while (X > 1 && (double)B * X * (double)P.tstride * sizeof(double) > 64.0 * 1024 * 1024) X >>= 1;
    int XL = 256;
    while (XL > 1 && (double)B * XL * P.K * P.G * 6 * sizeof(double) > 16.0 * 1024 * 1024) XL >>= 1;
    Layout l = layout_for(P, B, X, XL);
    while (l.total > kScratchBytes && (X > 1 || XL > 1)) {
        if (X >= XL && X > 1)
            X >>= 1;
        else
            XL >>= 1;
        l = layout_for(P, B, X, XL);
    }
    if (l.total > kScratchBytes)
        return fail(MCDC_E_UNSUPPORTED, "mcdc_run_noalloc: the run needs " + std::to_string(l.total) +
                                            " bytes of scratch (batches x tally), more than the " +
                                            std::to_string(kScratchBytes) + " of its static array");

    hipStream_t st = (hipStream_t)opt.stream;
    unsigned char *base = ds->ptr;
    RunArgs R{};
    R.N = n_histories;
    R.seed = seed;
    R.B = B;
    R.X = X;
    R.XL = XL;
    R.S = (double *)base;
    R.L = (double *)(base + l.off_L);
    R.qoi_sums = (double *)(base + l.off_q);
    R.counters = (unsigned long long *)(base + l.off_c);
    R.overflow = (int *)(base + l.off_o);
    R.work = (unsigned long long *)(base + l.off_w);
    R.qoi_hist = nullptr;
    R.dbg_counts = nullptr;
    R.dbg_scores = nullptr;
    R.prof = nullptr;

    if ((e = hipEventRecord(ds->a, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    // the array keeps the previous call's contents: clear all of this run's
    // part (the work counter is cleared by the launcher)
    if ((rc = launch_zero(base, l.off_w, st))) return hip_fail((hipError_t)rc, "zero fill");
    Profiler none;
    if ((rc = launch_history(p, R, 0, n_histories, 0, st, none))) return rc;
    if ((rc = fold(p, R, out, st, none))) return rc;
    if ((e = hipEventRecord(ds->b, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    Collect c{};
    if ((rc = collect_begin(p, R, out, c, st))) return rc;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, ds->a, ds->b)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    return collect_end(p, n_histories, c, out, ms);
}
