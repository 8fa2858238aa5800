// mcdc_run: buffers, kernel sequence, batch statistics and result hand-off.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "mcdc_internal.hpp"

using namespace mcdc;

namespace {

#define HIP_CHECK(call, what)                                  \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, what);       \
    } while (0)

int bad(const char *m) {
    set_error(std::string("invalid argument: ") + m);
    return MCDC_E_INVALID;
}

}  // namespace

extern "C" int mcdc_run(mcdc_problem *p, uint64_t n_histories, uint64_t seed,
                        const mcdc_run_options *opt_in, mcdc_result *out) {
    if (!p) return bad("problem is NULL");
    if (!out) return bad("result is NULL");
    if (n_histories == 0) return bad("n_histories must be > 0");
    mcdc_run_options opt{};
    if (opt_in) opt = *opt_in;
    if (opt.algorithm != MCDC_ALG_EVENT && opt.algorithm != MCDC_ALG_HISTORY)
        return bad("unknown algorithm");
    if (opt.block_size != 0 && (opt.block_size < 64 || opt.block_size > 1024 || opt.block_size % 64))
        return bad("block_size must be a multiple of 64 in [64, 1024]");
    if (opt.bank_capacity < 0) return bad("bank_capacity must be >= 0");
    if (opt.algorithm == MCDC_ALG_HISTORY && p->d.ww_center != nullptr) {
        set_error("weight windows run with the event-based algorithm only");
        return MCDC_E_UNSUPPORTED;
    }
    HIP_CHECK(hipSetDevice(p->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)opt.stream;
    const DevProblem &P = p->d;
    const uint64_t N = n_histories;
    const int B = (int)((uint64_t)p->h.B < N ? (uint64_t)p->h.B : N);
    const size_t nS = (size_t)B * P.ntally;
    const size_t nL = (size_t)B * P.K * P.G * 6;

    int rc;
    if ((rc = ensure(p->S, nS * sizeof(double)))) return rc;
    if ((rc = ensure(p->L, nL * sizeof(double)))) return rc;
    if ((rc = ensure(p->qoi_sums, 2 * sizeof(double)))) return rc;
    if ((rc = ensure(p->counters, kCounters * sizeof(unsigned long long)))) return rc;
    if ((rc = ensure(p->overflow, sizeof(int)))) return rc;

    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0), "hipEventCreate");
    HIP_CHECK(hipEventCreate(&e1), "hipEventCreate");
    HIP_CHECK(hipEventRecord(e0, st), "hipEventRecord");

    if ((rc = launch_zero(p->S.p, nS * sizeof(double), st))) return hip_fail((hipError_t)rc, "zero");
    if ((rc = launch_zero(p->L.p, nL * sizeof(double), st))) return hip_fail((hipError_t)rc, "zero");
    if ((rc = launch_zero(p->qoi_sums.p, 2 * sizeof(double), st))) return hip_fail((hipError_t)rc, "zero");
    if ((rc = launch_zero(p->counters.p, kCounters * sizeof(unsigned long long), st)))
        return hip_fail((hipError_t)rc, "zero");
    if ((rc = launch_zero(p->overflow.p, sizeof(int), st))) return hip_fail((hipError_t)rc, "zero");
    if (opt.debug_counts &&
        (rc = launch_zero(opt.debug_counts, (size_t)N * 5 * sizeof(uint32_t), st)))
        return hip_fail((hipError_t)rc, "zero");
    if (opt.debug_scores &&
        (rc = launch_zero(opt.debug_scores, (size_t)N * 2 * sizeof(double), st)))
        return hip_fail((hipError_t)rc, "zero");

    RunArgs R{};
    R.N = N;
    R.seed = seed;
    R.B = B;
    R.S = (double *)p->S.p;
    R.L = (double *)p->L.p;
    R.qoi_sums = (double *)p->qoi_sums.p;
    R.counters = (unsigned long long *)p->counters.p;
    R.dbg_counts = opt.debug_counts;
    R.dbg_scores = opt.debug_scores;
    R.overflow = (int *)p->overflow.p;
    R.qoi_hist = nullptr;

    if (opt.algorithm == MCDC_ALG_HISTORY) {
        rc = launch_history(P, R, 0, N, opt.block_size, st);
        if (rc) return hip_fail((hipError_t)rc, "history kernel launch");
    } else {
        rc = launch_event(p, R, 0, N, opt, st);
        if (rc) return rc;
    }

    // batch statistics into caller buffers (device) or staging (host outputs)
    double *mean = out->mean, *var = out->var, *raw = out->raw;
    double *lmean = out->leak_mean, *lvar = out->leak_var;
    const size_t nleak = (size_t)P.K * P.G * 6;
    if (out->host_outputs) {
        if (mean && (rc = ensure(p->mean, P.ntally * sizeof(double)))) return rc;
        if (var && (rc = ensure(p->var, P.ntally * sizeof(double)))) return rc;
        if (raw && (rc = ensure(p->raw, P.ntally * sizeof(double)))) return rc;
        if (lmean && (rc = ensure(p->leak_mean, nleak * sizeof(double)))) return rc;
        if (lvar && (rc = ensure(p->leak_var, nleak * sizeof(double)))) return rc;
        mean = mean ? (double *)p->mean.p : nullptr;
        var = var ? (double *)p->var.p : nullptr;
        raw = raw ? (double *)p->raw.p : nullptr;
        lmean = lmean ? (double *)p->leak_mean.p : nullptr;
        lvar = lvar ? (double *)p->leak_var.p : nullptr;
    }
    rc = launch_fold(P, R.S, R.L, B, N, P.bin_norm, P.time_norm, mean, var, raw, lmean, lvar, st);
    if (rc) return hip_fail((hipError_t)rc, "fold kernel launch");
    HIP_CHECK(hipEventRecord(e1, st), "hipEventRecord");

    unsigned long long cnt[kCounters];
    double qs[2];
    int ovf = 0;
    HIP_CHECK(hipMemcpyAsync(cnt, p->counters.p, sizeof(cnt), hipMemcpyDeviceToHost, st), "copy counters");
    HIP_CHECK(hipMemcpyAsync(qs, p->qoi_sums.p, sizeof(qs), hipMemcpyDeviceToHost, st), "copy detector");
    HIP_CHECK(hipMemcpyAsync(&ovf, p->overflow.p, sizeof(int), hipMemcpyDeviceToHost, st), "copy flag");
    if (out->host_outputs) {
        if (out->mean)
            HIP_CHECK(hipMemcpyAsync(out->mean, mean, P.ntally * sizeof(double), hipMemcpyDeviceToHost, st), "copy mean");
        if (out->var)
            HIP_CHECK(hipMemcpyAsync(out->var, var, P.ntally * sizeof(double), hipMemcpyDeviceToHost, st), "copy var");
        if (out->raw)
            HIP_CHECK(hipMemcpyAsync(out->raw, raw, P.ntally * sizeof(double), hipMemcpyDeviceToHost, st), "copy raw");
        if (out->leak_mean)
            HIP_CHECK(hipMemcpyAsync(out->leak_mean, lmean, nleak * sizeof(double), hipMemcpyDeviceToHost, st), "copy leak");
        if (out->leak_var)
            HIP_CHECK(hipMemcpyAsync(out->leak_var, lvar, nleak * sizeof(double), hipMemcpyDeviceToHost, st), "copy leak var");
    }
    HIP_CHECK(hipStreamSynchronize(st), "hipStreamSynchronize");
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ovf) {
        set_error("particle bank or split bank overflow");
        return MCDC_E_OVERFLOW;
    }
    for (int j = 0; j < 3; ++j) out->n_events[j] = cnt[j];
    for (int j = 0; j < 5; ++j) out->n_term[j] = cnt[3 + j];
    out->n_splits = cnt[8];
    out->qoi_sum[0] = qs[0];
    out->qoi_sum[1] = qs[1];
    const double V = p->h.qoi_volume;
    const double Nd = (double)N;
    out->qoi_mean = P.qoi_on ? qs[0] / (Nd * V) : 0.0;
    out->qoi_var = (P.qoi_on && N > 1) ? (qs[1] - qs[0] * qs[0] / Nd) / (Nd * (Nd - 1.0)) / (V * V) : 0.0;
    out->kernel_ms = ms;
    return MCDC_OK;
}
