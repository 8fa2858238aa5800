// mcdc_run and mcdc_run_batched: buffers, kernel sequence, batch statistics
// and result hand-off.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mcdc_internal.hpp"

using namespace mcdc;

namespace {
// Events are reused across profiled runs (creating one per launch costs
// more than the short kernels it would time).
std::vector<hipEvent_t> &event_pool() {
    static thread_local std::vector<hipEvent_t> pool;
    return pool;
}
hipEvent_t take_event() {
    auto &pool = event_pool();
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

hipEvent_t Profiler::take() { return take_event(); }

void Profiler::give(hipEvent_t e) { event_pool().push_back(e); }

void Profiler::begin(int c) {
    if (!wants(c)) return;
    cls = c;
    open = take_event();
    if (open) (void)hipEventRecord(open, st);
}

void Profiler::end() {
    if (!out || !open) return;
    hipEvent_t e = take_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    marks.push_back({cls, {open, e}});
    open = nullptr;
}

int Profiler::finish() {
    if (!out) return MCDC_OK;
    hipError_t err = hipStreamSynchronize(st);
    for (auto &m : marks) {
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, m.second.first, m.second.second);
        out[m.first * 4 + 0] += ms;
        out[m.first * 4 + 1] += 1.0;
        event_pool().push_back(m.second.first);
        event_pool().push_back(m.second.second);
    }
    marks.clear();
    if (err != hipSuccess) return hip_fail(err, "profile events");
    return MCDC_OK;
}

namespace {

#define HIP_CHECK(call, what)                                  \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, what);       \
    } while (0)

#define ZERO(ptr, bytes)                                                        \
    do {                                                                        \
        int r_ = launch_zero((ptr), (bytes), st);                               \
        if (r_) return hip_fail((hipError_t)r_, "zero fill");                   \
    } while (0)

int bad(const char *m) {
    set_error(std::string("invalid argument: ") + m);
    return MCDC_E_INVALID;
}

int check_options(const mcdc_run_options &opt) {
    if (opt.algorithm != MCDC_ALG_EVENT && opt.algorithm != MCDC_ALG_HISTORY) return bad("unknown algorithm");
    if (opt.block_size != 0 && (opt.block_size < 64 || opt.block_size > 1024 || opt.block_size % 64))
        return bad("block_size must be a multiple of 64 in [64, 1024]");
    if (opt.segments < 0 || opt.segments > (1 << 20)) return bad("segments must be in [0, 2^20]");
    if (opt.profile_every < 0 || opt.profile_phase < 0) return bad("profile_every and profile_phase must be >= 0");
    if (opt.bank_capacity < 0) return bad("bank_capacity must be >= 0");
    if (opt.sort_cadence < -1 || opt.sort_cadence > 64) return bad("sort_cadence must be in [-1, 64]");
    if (opt.steps_per_launch < 0 || opt.steps_per_launch > 65535) return bad("steps_per_launch must be in [0, 65535]");
    if (opt.pc_method != MCDC_PC_SPLIT && opt.pc_method != MCDC_PC_COMB)
        return bad("pc_method must be MCDC_PC_SPLIT or MCDC_PC_COMB");
    if (opt.pc_method == MCDC_PC_COMB && opt.pc_target == 0) return bad("pc_method needs pc_target");
    return MCDC_OK;
}

// Allocate and clear the per-run device buffers of a problem; fill R.
// (B_force > 0: that many batches instead of the problem's.)
int prepare(mcdc_problem *p, uint64_t N, uint64_t seed, const mcdc_run_options &opt, hipStream_t st, RunArgs &R,
            int B_force = 0) {
    const DevProblem &P = p->d;
    const int B = B_force > 0 ? B_force : (int)((uint64_t)p->h.B < N ? (uint64_t)p->h.B : N);
    // tally copies per batch: up to 32 while the copies stay within 64 MB
    // (the event form adds a step's scores from its LDS slice once per
    // workgroup when the slice fits, and needs no copies then)
    int X = 32;
    while (X > 1 && (double)B * X * (double)P.tstride * sizeof(double) > 64.0 * 1024 * 1024) X >>= 1;
    if (opt.algorithm != MCDC_ALG_HISTORY && slice_mult(P) * (int64_t)P.G * P.nts <= kLdsTallyMax) X = 1;
    const size_t nS = (size_t)B * X * P.tstride;
    // leakage copies: up to 256 within 16 MB
    int XL = 256;
    while (XL > 1 && (double)B * XL * P.K * P.G * 6 * sizeof(double) > 16.0 * 1024 * 1024) XL >>= 1;
    const size_t nL = (size_t)B * XL * P.K * P.G * 6;
    int rc;
    if ((rc = ensure(p->S, nS * sizeof(double)))) return rc;
    if ((rc = ensure(p->L, nL * sizeof(double)))) return rc;
    if ((rc = ensure(p->qoi_sums, 2 * sizeof(double)))) return rc;
    if ((rc = ensure(p->counters, kCounters * sizeof(unsigned long long)))) return rc;
    if ((rc = ensure(p->overflow, sizeof(int)))) return rc;
    if ((rc = ensure(p->prof, 2 * MCDC_PROF_CLASSES * sizeof(unsigned long long)))) return rc;
    ZERO(p->S.p, nS * sizeof(double));
    ZERO(p->L.p, nL * sizeof(double));
    ZERO(p->qoi_sums.p, 2 * sizeof(double));
    ZERO(p->counters.p, kCounters * sizeof(unsigned long long));
    ZERO(p->overflow.p, sizeof(int));
    if (opt.profile) ZERO(p->prof.p, 2 * MCDC_PROF_CLASSES * sizeof(unsigned long long));
    if (opt.debug_counts) ZERO(opt.debug_counts, (size_t)N * 5 * sizeof(uint32_t));
    if (opt.debug_scores) ZERO(opt.debug_scores, (size_t)N * 2 * sizeof(double));
    R = RunArgs{};
    R.N = N;
    R.seed = seed;
    R.B = B;
    R.X = X;
    R.XL = XL;
    R.S = (double *)p->S.p;
    R.L = (double *)p->L.p;
    R.qoi_sums = (double *)p->qoi_sums.p;
    R.counters = (unsigned long long *)p->counters.p;
    R.dbg_counts = opt.debug_counts;
    R.dbg_scores = opt.debug_scores;
    R.overflow = (int *)p->overflow.p;
    R.qoi_hist = nullptr;
    R.prof = opt.profile ? (unsigned long long *)p->prof.p : nullptr;
    return MCDC_OK;
}

}  // namespace

// Batch statistics into the caller's buffers (device) or staging buffers
// (host outputs).
int mcdc::fold(mcdc_problem *p, const RunArgs &R, mcdc_result *out, hipStream_t st, Profiler &prof) {
    const DevProblem &P = p->d;
    double *mean = out->mean, *var = out->var, *raw = out->raw;
    double *lmean = out->leak_mean, *lvar = out->leak_var;
    double *tmean = P.tc_on ? out->tc_mean : nullptr, *tvar = P.tc_on ? out->tc_var : nullptr;
    const size_t nleak = (size_t)P.K * P.G * 6;
    int rc;
    if (out->host_outputs) {
        if (tmean && (rc = ensure(p->tc_mean, P.ntally * sizeof(double)))) return rc;
        if (tvar && (rc = ensure(p->tc_var, P.ntally * sizeof(double)))) return rc;
        tmean = tmean ? (double *)p->tc_mean.p : nullptr;
        tvar = tvar ? (double *)p->tc_var.p : nullptr;
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
    prof.begin(MCDC_PROF_OTHER);
    rc = launch_fold(P, R.S, R.L, R.B, R.X, R.XL, R.N, P.bin_norm, P.time_norm, mean, var, raw, lmean, lvar, tmean,
                     tvar, st);
    prof.end();
    return rc ? hip_fail((hipError_t)rc, "fold kernel launch") : MCDC_OK;
}

// Host copies of counters, detector sums and (host) outputs.  The caller
// synchronises the stream between collect_begin and collect_end.
int mcdc::collect_begin(mcdc_problem *p, const RunArgs &R, mcdc_result *out, Collect &c, hipStream_t st) {
    const DevProblem &P = p->d;
    HIP_CHECK(hipMemcpyAsync(c.cnt, R.counters, sizeof(c.cnt), hipMemcpyDeviceToHost, st), "copy counters");
    HIP_CHECK(hipMemcpyAsync(c.qs, R.qoi_sums, sizeof(c.qs), hipMemcpyDeviceToHost, st), "copy detector");
    HIP_CHECK(hipMemcpyAsync(&c.ovf, R.overflow, sizeof(int), hipMemcpyDeviceToHost, st), "copy flag");
    if (out->host_outputs) {
        const size_t nt = P.ntally * sizeof(double), nl = (size_t)P.K * P.G * 6 * sizeof(double);
        if (out->mean) HIP_CHECK(hipMemcpyAsync(out->mean, p->mean.p, nt, hipMemcpyDeviceToHost, st), "copy mean");
        if (out->var) HIP_CHECK(hipMemcpyAsync(out->var, p->var.p, nt, hipMemcpyDeviceToHost, st), "copy var");
        if (out->raw) HIP_CHECK(hipMemcpyAsync(out->raw, p->raw.p, nt, hipMemcpyDeviceToHost, st), "copy raw");
        if (out->leak_mean)
            HIP_CHECK(hipMemcpyAsync(out->leak_mean, p->leak_mean.p, nl, hipMemcpyDeviceToHost, st), "copy leak");
        if (out->leak_var)
            HIP_CHECK(hipMemcpyAsync(out->leak_var, p->leak_var.p, nl, hipMemcpyDeviceToHost, st), "copy leak var");
        if (P.tc_on && out->tc_mean)
            HIP_CHECK(hipMemcpyAsync(out->tc_mean, p->tc_mean.p, nt, hipMemcpyDeviceToHost, st), "copy tc mean");
        if (P.tc_on && out->tc_var)
            HIP_CHECK(hipMemcpyAsync(out->tc_var, p->tc_var.p, nt, hipMemcpyDeviceToHost, st), "copy tc var");
    }
    return MCDC_OK;
}

int mcdc::collect_end(mcdc_problem *p, uint64_t N, const Collect &c, mcdc_result *out, double ms) {
    if (c.ovf) {
        static const char *what[] = {"particle bank or split bank overflow",
                                     "population control: a weight of 2^32 or more (or not a number)",
                                     "population control: more copies of a particle than its bank segment holds",
                                     "population control: a bank segment overflowed"};
        set_error(what[(c.ovf >= 1 && c.ovf <= 4) ? c.ovf - 1 : 0]);
        return MCDC_E_OVERFLOW;
    }
    for (int j = 0; j < 3; ++j) out->n_events[j] = c.cnt[j];
    for (int j = 0; j < 5; ++j) out->n_term[j] = c.cnt[3 + j];
    out->n_splits = c.cnt[8];
    out->n_fission = c.cnt[9];
    out->qoi_sum[0] = c.qs[0];
    out->qoi_sum[1] = c.qs[1];
    const double V = p->h.qoi_volume;
    const double Nd = (double)N;
    const bool q = p->d.qoi_on != 0;
    out->qoi_mean = q ? c.qs[0] / (Nd * V) : 0.0;
    out->qoi_var = (q && N > 1) ? (c.qs[1] - c.qs[0] * c.qs[0] / Nd) / (Nd * (Nd - 1.0)) / (V * V) : 0.0;
    out->kernel_ms = ms;
    return MCDC_OK;
}

namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" int mcdc_run(mcdc_problem *p, uint64_t n_histories, uint64_t seed, const mcdc_run_options *opt_in,
                        mcdc_result *out) {
    if (!p) return bad("problem is NULL");
    if (!out) return bad("result is NULL");
    if (n_histories == 0) return bad("n_histories must be > 0");
    mcdc_run_options opt{};
    if (opt_in) opt = *opt_in;
    if (opt.pc_target) {
        // population control synchronises all particles at census: event form only
        if (opt.algorithm == MCDC_ALG_AUTO) opt.algorithm = MCDC_ALG_EVENT;
        if (opt.algorithm == MCDC_ALG_HISTORY) {
            set_error("population control runs in the event form only");
            return MCDC_E_UNSUPPORTED;
        }
        if (p->d.ww_center || p->d.fission_on || p->d.qoi_on) {
            set_error("population control is not combined with weight windows, fission or a detector");
            return MCDC_E_UNSUPPORTED;
        }
        if (n_histories > (1ULL << 26) || opt.pc_target > (1ULL << 26)) {
            set_error("population control runs at most 2^26 histories per call, to at most 2^26 particles");
            return MCDC_E_UNSUPPORTED;
        }
    }
    if (opt.algorithm == MCDC_ALG_AUTO) {
        // the faster form for this problem and history count: both forms
        // run (and are timed) on the first call, the choice is kept on the
        // handle; the result is the last run's
        mcdc_run_options o = opt;
        if (p->auto_alg >= 0 && p->auto_n == n_histories) {
            o.algorithm = p->auto_alg;
            return mcdc_run(p, n_histories, seed, &o, out);
        }
        o.algorithm = MCDC_ALG_EVENT;
        int r = mcdc_run(p, n_histories, seed, &o, out);
        if (r) return r;
        const double t_event = out->kernel_ms;
        o.algorithm = MCDC_ALG_HISTORY;
        if ((r = mcdc_run(p, n_histories, seed, &o, out))) return r;
        p->auto_alg = (out->kernel_ms < t_event) ? MCDC_ALG_HISTORY : MCDC_ALG_EVENT;
        p->auto_n = n_histories;
        return MCDC_OK;
    }
    int rc = check_options(opt);
    if (rc) return rc;
    if (opt.algorithm == MCDC_ALG_EVENT && opt.block_size != 0 && opt.block_size != 256 && opt.block_size != 512 &&
        opt.block_size != 1024)
        return bad("event form: block_size must be 0, 256, 512 or 1024");
    if (opt.algorithm == MCDC_ALG_EVENT && opt.block_size && opt.block_size != 512 &&
        (has_progeny(p->d) || opt.pc_target)) {
        set_error("event form: weighted runs and population control use 512-thread workgroups");
        return MCDC_E_UNSUPPORTED;
    }
    HIP_CHECK(hipSetDevice(p->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)opt.stream;
    Profiler prof;
    prof.out = opt.profile;
    prof.mask = opt.profile_mask;
    prof.st = st;
    Events ev;
    HIP_CHECK(hipEventCreate(&ev.a), "hipEventCreate");
    HIP_CHECK(hipEventCreate(&ev.b), "hipEventCreate");
    // (the history form's split banks are allocated before the run's timed
    // region, so kernel_ms holds device time only)
    if (opt.algorithm == MCDC_ALG_HISTORY && (rc = history_reserve(p, n_histories, (uint64_t)opt.bank_capacity)))
        return rc;
    HIP_CHECK(hipEventRecord(ev.a, st), "hipEventRecord");

    RunArgs R;
    if ((rc = prepare(p, n_histories, seed, opt, st, R))) return rc;
    if (opt.algorithm == MCDC_ALG_HISTORY)
        rc = launch_history(p, R, 0, n_histories, (uint64_t)opt.bank_capacity, st, prof);
    else
        rc = launch_event(p, R, 0, n_histories, opt, st, prof);
    if (rc) return rc;
    if ((rc = fold(p, R, out, st, prof))) return rc;
    HIP_CHECK(hipEventRecord(ev.b, st), "hipEventRecord");

    Collect c{};
    if ((rc = collect_begin(p, R, out, c, st))) return rc;
    unsigned long long pc[2 * MCDC_PROF_CLASSES] = {};
    if (opt.profile) HIP_CHECK(hipMemcpyAsync(pc, p->prof.p, sizeof(pc), hipMemcpyDeviceToHost, st), "copy profile");
    HIP_CHECK(hipStreamSynchronize(st), "hipStreamSynchronize");
    if ((rc = prof.finish())) return rc;
    if (opt.profile)
        for (int k = 0; k < MCDC_PROF_CLASSES; ++k) {
            opt.profile[k * 4 + 2] += (double)pc[2 * k];
            opt.profile[k * 4 + 3] += (double)pc[2 * k + 1];
        }
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
    return collect_end(p, n_histories, c, out, ms);
}

// ---------------------------------------------------------------------------
// batched solve
// ---------------------------------------------------------------------------
namespace {

struct Tuned {
    int block, per_thread;   // history form: workgroup size, histories per thread per pull
    unsigned int seg_len;    // event form: slots per bank segment
    int step_form;           // event form: -1 one kernel per census step, 0 two-kernel step,
                             // c >= 1 two-kernel step with the queue sort every c-th step
    uint64_t tail;           // event form: problems of at most this many histories run in
                             // the history-form launch instead
    int ev_block;            // event form: workgroup size of the step kernels
};

// Launch shapes and form choices of batched solves, per batch signature,
// shared by every thread of the process (lookups and inserts locked).
std::mutex &cache_mutex() {
    static std::mutex m;
    return m;
}
std::map<std::string, Tuned> &tune_cache() {
    static std::map<std::string, Tuned> m;
    return m;
}
bool tuned_get(const std::string &sig, Tuned &t) {
    std::lock_guard<std::mutex> g(cache_mutex());
    auto it = tune_cache().find(sig);
    if (it == tune_cache().end()) return false;
    t = it->second;
    return true;
}
void tuned_put(const std::string &sig, const Tuned &t) {
    std::lock_guard<std::mutex> g(cache_mutex());
    tune_cache()[sig] = t;
}
std::map<std::string, int> &form_cache() {
    static std::map<std::string, int> m;
    return m;
}
bool form_get(const std::string &sig, int &alg) {
    std::lock_guard<std::mutex> g(cache_mutex());
    auto it = form_cache().find(sig);
    if (it == form_cache().end()) return false;
    alg = it->second;
    return true;
}
void form_put(const std::string &sig, int alg) {
    std::lock_guard<std::mutex> g(cache_mutex());
    form_cache()[sig] = alg;
}

std::string signature(mcdc_problem *const *ps, int32_t n, const uint64_t *n_hist) {
    std::string s;
    for (int j = 0; j < n; ++j) {
        const DevProblem &P = ps[j]->d;
        s += std::to_string(P.G) + "," + std::to_string(P.ncells) + "," + std::to_string(P.ntally) + "," +
             std::to_string(P.finite_mask) + "," + std::to_string(n_hist[j]) + ";";
    }
    return s;
}

struct DevMem {
    void *mem = nullptr;
    ~DevMem() {
        if (mem) (void)hipFree(mem);
    }
};

// Options of problem j of a batch: the debug arrays of a batched run hold
// every problem's histories in problem order, so problem j's records start
// after the histories of problems 0 .. j-1.
mcdc_run_options batch_opt(const mcdc_run_options &opt, const uint64_t *n_hist, int j, int alg) {
    mcdc_run_options o = opt;
    o.algorithm = alg;
    uint64_t off = 0;
    for (int k = 0; k < j; ++k) off += n_hist[k];
    if (o.debug_counts) o.debug_counts += off * 5;
    if (o.debug_scores) o.debug_scores += off * 2;
    return o;
}

// Device memory of batched runs, kept across the tuning runs of one call.
struct BatchWork {
    DevMem ev;             // event form: banks, tables, segment list
    size_t ev_bytes = 0;
    DevMem hist;           // history form: items, history offsets, work counter
    size_t hist_bytes = 0;
};

int grow(DevMem &m, size_t &have, size_t need) {
    if (need <= have) return MCDC_OK;
    if (m.mem) (void)hipFree(m.mem);
    m.mem = nullptr;
    have = 0;
    HIP_CHECK(hipMalloc(&m.mem, need), "hipMalloc(batched work)");
    have = need;
    return MCDC_OK;
}

// One batched run in configuration t: problems with more than t.tail
// histories go to the event form (all their segments in one set of banks,
// one captured graph per census step in form t.step_form), the others to
// one persistent history-form launch (workgroups of t.block threads
// pulling t.per_thread histories per thread); all_history sends every
// problem to the history launch.  Fills items[j].R for the fold and the
// device time of the run into *ms.
int batched_once(mcdc_problem *const *ps, int32_t n, const uint64_t *n_hist, const uint64_t *seeds,
                 const mcdc_run_options &opt, bool all_history, const Tuned &t, std::vector<BatchItem> &items,
                 BatchWork &wk, hipStream_t st, float *ms) {
    Events ev;
    HIP_CHECK(hipEventCreate(&ev.a), "hipEventCreate");
    HIP_CHECK(hipEventCreate(&ev.b), "hipEventCreate");
    HIP_CHECK(hipEventRecord(ev.a, st), "hipEventRecord");
    std::vector<int> E, H;
    for (int j = 0; j < n; ++j) {
        items[j] = BatchItem{};
        items[j].P = ps[j]->d;
        if (n_hist[j] == 0) continue;
        const bool in_e = !all_history && n_hist[j] > t.tail;
        (in_e ? E : H).push_back(j);
        int r = prepare(ps[j], n_hist[j], seeds[j],
                        batch_opt(opt, n_hist, j, in_e ? MCDC_ALG_EVENT : MCDC_ALG_HISTORY), st, items[j].R);
        if (r) return r;
        if (in_e && ps[j]->d.qoi_on) {
            if ((r = ensure(ps[j]->qoi_hist, n_hist[j] * sizeof(double)))) return r;
            items[j].R.qoi_hist = (double *)ps[j]->qoi_hist.p;
            ZERO(items[j].R.qoi_hist, n_hist[j] * sizeof(double));
        }
    }
    int r;
    if (!E.empty()) {
        std::vector<BatchItem> ie;
        std::vector<uint64_t> ne;
        for (int j : E) {
            ie.push_back(items[j]);
            ne.push_back(n_hist[j]);
        }
        const size_t need = event_batched_bytes(ne.data(), (int)E.size(), t.seg_len, t.step_form);
        if ((r = grow(wk.ev, wk.ev_bytes, need))) return r;
        if ((r = launch_event_batched(ie, ne.data(), t.seg_len, wk.ev.mem, wk.ev_bytes, st, t.step_form, t.ev_block)))
            return r;
        for (int j : E)
            if (ps[j]->d.qoi_on && (r = launch_qoi_reduce(items[j].R.qoi_hist, n_hist[j], items[j].R.qoi_sums, st)))
                return hip_fail((hipError_t)r, "detector reduce");
    }
    if (!H.empty()) {
        const int nh = (int)H.size();
        std::vector<BatchItem> ih;
        std::vector<uint64_t> offs(nh + 1, 0);
        int fm = -1;
        for (int k = 0; k < nh; ++k) {
            const int j = H[k];
            ih.push_back(items[j]);
            offs[k + 1] = offs[k] + n_hist[j];
            const int m = ps[j]->d.finite_mask;
            fm = (fm < 0 || fm == m) ? m : 0;
        }
        const size_t items_bytes = (sizeof(BatchItem) * n + 255) & ~size_t(255);
        const size_t offs_bytes = ((n + 1) * sizeof(uint64_t) + 255) & ~size_t(255);
        if ((r = grow(wk.hist, wk.hist_bytes, items_bytes + offs_bytes + 256))) return r;
        BatchItem *d_items = (BatchItem *)wk.hist.mem;
        uint64_t *d_offs = (uint64_t *)((char *)wk.hist.mem + items_bytes);
        unsigned long long *d_next = (unsigned long long *)((char *)wk.hist.mem + items_bytes + offs_bytes);
        HIP_CHECK(hipMemcpyAsync(d_items, ih.data(), sizeof(BatchItem) * nh, hipMemcpyHostToDevice, st),
                  "copy items");
        HIP_CHECK(hipMemcpyAsync(d_offs, offs.data(), (nh + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st),
                  "copy offsets");
        if ((r = launch_zero(d_next, sizeof(unsigned long long), st))) return hip_fail((hipError_t)r, "zero");
        if ((r = launch_batched(d_items, d_offs, nh, offs[nh], d_next, fm, t.block, t.per_thread, st))) return r;
    }
    HIP_CHECK(hipEventRecord(ev.b, st), "hipEventRecord");
    HIP_CHECK(hipEventSynchronize(ev.b), "hipEventSynchronize");
    HIP_CHECK(hipEventElapsedTime(ms, ev.a, ev.b), "hipEventElapsedTime");
    return MCDC_OK;
}

// Launch parameters of a batched solve: forced by the options, cached per
// batch signature, or tuned now by coordinate descent over timed runs of
// the whole batch.  Event form: segment length {2048, 8192, 32768, 65536}
// with one kernel per census step of 512-thread workgroups; then the
// workgroup size {256, 512, 1024}; then the census step's form (one
// kernel, two kernels, two kernels with the queue sort every 1, 2, 4 or 8
// steps); then the tail switch (problems of at most 0, 2e4 or 1e5
// histories run in the history-form launch), each at the best so far.  History form:
// workgroup {128, 256, 512} x histories per pull {1, 4, 16}.  No
// parameter changes per-history results, only tally summation order.
int batched_tuned(mcdc_problem *const *ps, int32_t n, const uint64_t *n_hist, const uint64_t *seeds,
                  const mcdc_run_options &opt, bool all_history, std::vector<BatchItem> &items, BatchWork &wk,
                  hipStream_t st, float *ms) {
    const bool two = (opt.flags & MCDC_FLAG_TWO_KERNEL_STEP) != 0;
    Tuned t{opt.block_size ? opt.block_size : 256, 4, (unsigned int)opt.bank_capacity,
            opt.sort_cadence > 0 ? opt.sort_cadence : (two ? 0 : -1), 0, opt.block_size ? opt.block_size : 512};
    const bool seg_forced = opt.bank_capacity != 0;
    const bool form_forced = opt.sort_cadence != 0 || two;
    const std::string sig = std::string(all_history ? "history:" : "event:") + std::to_string(opt.block_size) +
                            "," + std::to_string(opt.bank_capacity) + "," + std::to_string(opt.sort_cadence) + "," +
                            std::to_string(two) + ":" + signature(ps, n, n_hist);
    int rc;
    float m = 0.f;
    if (!tuned_get(sig, t)) {
        auto trial = [&](const Tuned &c, float *best, Tuned *arg) -> int {
            int r = batched_once(ps, n, n_hist, seeds, opt, all_history, c, items, wk, st, &m);
            if (r) return r;
            if (m < *best) {
                *best = m;
                *arg = c;
            }
            return MCDC_OK;
        };
        float best = 1e30f;
        if (all_history) {
            if (!opt.block_size) {
                for (int bsz : {128, 256, 512})
                    for (int pt : {1, 4, 16}) {
                        Tuned c = t;
                        c.block = bsz;
                        c.per_thread = pt;
                        if ((rc = trial(c, &best, &t))) return rc;
                    }
            }
        } else {
            Tuned base = t;
            if (!seg_forced) {
                for (unsigned int L : {2048u, 8192u, 32768u, 65536u}) {
                    Tuned c = base;
                    c.seg_len = L;
                    if ((rc = trial(c, &best, &t))) return rc;
                }
            } else {
                if ((rc = trial(t, &best, &t))) return rc;
            }
            if (!opt.block_size) {
                base = t;
                for (int bsz : {256, 1024}) {
                    Tuned c = base;
                    c.ev_block = bsz;
                    if ((rc = trial(c, &best, &t))) return rc;
                }
            }
            if (!form_forced) {
                base = t;
                for (int f : {0, 1, 2, 4, 8}) {
                    Tuned c = base;
                    c.step_form = f;
                    if ((rc = trial(c, &best, &t))) return rc;
                }
            }
            base = t;
            for (uint64_t tail : {20000ull, 100000ull}) {
                Tuned c = base;
                c.tail = tail;
                if ((rc = trial(c, &best, &t))) return rc;
            }
        }
        tuned_put(sig, t);
    }
    return batched_once(ps, n, n_hist, seeds, opt, all_history, t, items, wk, st, ms);
}

}  // namespace

// Fold and hand back every problem's results after a batched run.
int finish_batched(mcdc_problem *const *ps, int32_t n, const uint64_t *n_hist, std::vector<BatchItem> &items,
                   mcdc_result *outs, float ms, hipStream_t st) {
    int rc;
    Profiler none;
    std::vector<Collect> cs(n);
    for (int j = 0; j < n; ++j) {
        if (n_hist[j] == 0) continue;
        if ((rc = fold(ps[j], items[j].R, &outs[j], st, none))) return rc;
        if ((rc = collect_begin(ps[j], items[j].R, &outs[j], cs[j], st))) return rc;
    }
    HIP_CHECK(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (int j = 0; j < n; ++j) {
        if (n_hist[j] == 0) {
            std::memset(outs[j].n_events, 0, sizeof(outs[j].n_events));
            std::memset(outs[j].n_term, 0, sizeof(outs[j].n_term));
            outs[j].kernel_ms = ms;
            continue;
        }
        if ((rc = collect_end(ps[j], n_hist[j], cs[j], &outs[j], ms))) return rc;
    }
    return MCDC_OK;
}

extern "C" int mcdc_run_batched(mcdc_problem *const *ps, int32_t n, const uint64_t *n_hist, const uint64_t *seeds,
                                const mcdc_run_options *opt_in, mcdc_result *outs) {
    if (!ps || !n_hist || !seeds || !outs || n <= 0) return bad("NULL argument or n <= 0");
    mcdc_run_options opt{};
    if (opt_in) opt = *opt_in;
    if (opt.pc_target) {
        set_error("population control is not supported in batched solves");
        return MCDC_E_UNSUPPORTED;
    }
    if (opt.algorithm == MCDC_ALG_AUTO) {
        // the faster form for this batch signature, timed once and cached
        for (int j = 0; j < n; ++j)
            if (!ps[j]) return bad("NULL problem in batch");
        const std::string sig = signature(ps, n, n_hist);
        mcdc_run_options o = opt;
        int alg = 0;
        if (form_get(sig, alg)) {
            o.algorithm = alg;
            return mcdc_run_batched(ps, n, n_hist, seeds, &o, outs);
        }
        o.algorithm = MCDC_ALG_EVENT;
        int r = mcdc_run_batched(ps, n, n_hist, seeds, &o, outs);
        if (r) return r;
        const double t_event = outs[0].kernel_ms;
        o.algorithm = MCDC_ALG_HISTORY;
        if ((r = mcdc_run_batched(ps, n, n_hist, seeds, &o, outs))) return r;
        form_put(sig, (outs[0].kernel_ms < t_event) ? MCDC_ALG_HISTORY : MCDC_ALG_EVENT);
        return MCDC_OK;
    }
    int rc = check_options(opt);
    if (rc) return rc;
    if (opt.block_size != 0) {
        const int b = opt.block_size;
        if (opt.algorithm == MCDC_ALG_HISTORY && b != 64 && b != 128 && b != 256 && b != 512)
            return bad("batched history form: block_size must be 0, 64, 128, 256 or 512");
        if (opt.algorithm != MCDC_ALG_HISTORY && b != 256 && b != 512 && b != 1024)
            return bad("batched event form: block_size must be 0, 256, 512 or 1024");
    }
    if (opt.profile) {
        set_error("batched solves take no profile array");
        return MCDC_E_UNSUPPORTED;
    }
    if (opt.bank_capacity != 0 && (opt.bank_capacity < 256 || opt.bank_capacity > (1 << 24)))
        return bad("batched event form: bank_capacity (slots per segment) must be in [256, 2^24]");
    if (!ps[0]) return bad("NULL problem in batch");
    const int dev = ps[0]->device;
    uint64_t total = 0;
    for (int j = 0; j < n; ++j) {
        if (!ps[j]) return bad("NULL problem in batch");
        if (ps[j]->device != dev) return bad("all problems of a batch must be on one device");
        if (has_progeny(ps[j]->d)) {
            set_error("batched solves run analog (no weight windows, fission or implicit capture)");
            return MCDC_E_UNSUPPORTED;
        }
        if (ps[j]->h.B > 1023) {
            set_error("at most 1023 batches");
            return MCDC_E_UNSUPPORTED;
        }
        if (opt.algorithm != MCDC_ALG_HISTORY && (n_hist[j] > (1ULL << 28) || ps[j]->d.K > 65535)) {
            set_error("batched event form: at most 2^28 histories and 65535 time bins per problem");
            return MCDC_E_UNSUPPORTED;
        }
        for (int k = 0; k < j; ++k)
            if (ps[k] == ps[j]) return bad("a problem appears twice in the batch");
        total += n_hist[j];
    }
    if (total == 0) return bad("no histories");
    HIP_CHECK(hipSetDevice(dev), "hipSetDevice");
    hipStream_t st = (hipStream_t)opt.stream;
    std::vector<BatchItem> items(n);
    BatchWork wk;
    float ms = 0.f;
    if ((rc = batched_tuned(ps, n, n_hist, seeds, opt, opt.algorithm == MCDC_ALG_HISTORY, items, wk, st, &ms)))
        return rc;
    return finish_batched(ps, n, n_hist, items, outs, ms, st);
}

// ---------------------------------------------------------------------------
// k-eigenvalue power iteration
// ---------------------------------------------------------------------------
extern "C" int mcdc_run_eigenvalue(mcdc_problem *p, uint64_t n_per_cycle, int32_t n_inactive, int32_t n_active,
                                   uint64_t seed, const mcdc_run_options *opt_in, mcdc_result *out,
                                   double *k_cycle, uint64_t *source_hist, double *entropy) {
    if (!p) return bad("problem is NULL");
    if (!out) return bad("result is NULL");
    if (n_per_cycle == 0 || n_per_cycle > (1ULL << 30)) return bad("n_per_cycle must be in [1, 2^30]");
    if (n_inactive < 0 || n_active < 1 || n_active > 1023 || n_inactive > 100000)
        return bad("n_inactive must be >= 0 and n_active in [1, 1023]");
    mcdc_run_options opt{};
    if (opt_in) opt = *opt_in;
    if (opt.pc_target) {
        set_error("population control is not supported in eigenvalue cycles");
        return MCDC_E_UNSUPPORTED;
    }
    int rc = check_options(opt);
    if (rc) return rc;
    const DevProblem &P = p->d;
    if (!P.fission_on) return bad("the eigenvalue problem needs fission data");
    if (P.rod_on) {
        set_error("eigenvalue runs take no moving plane");
        return MCDC_E_UNSUPPORTED;
    }
    if (P.K != 1 || std::isfinite(p->h.T[1])) return bad("the eigenvalue problem is steady state: time edges [T0, inf)");
    if (P.ww_center || P.implicit || P.qoi_on || opt.debug_counts || opt.debug_scores || opt.profile) {
        set_error("eigenvalue runs take no weight windows, implicit capture, detector, debug or profile arrays");
        return MCDC_E_UNSUPPORTED;
    }
    HIP_CHECK(hipSetDevice(p->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)opt.stream;
    Events ev;
    HIP_CHECK(hipEventCreate(&ev.a), "hipEventCreate");
    HIP_CHECK(hipEventCreate(&ev.b), "hipEventCreate");
    HIP_CHECK(hipEventRecord(ev.a, st), "hipEventRecord");
    // the active cycles are the batches: N per batch in order
    const uint64_t n_tally = n_per_cycle * (uint64_t)n_active;
    RunArgs R;
    if ((rc = prepare(p, n_tally, seed, opt, st, R, n_active))) return rc;
    const int C = n_inactive + n_active;
    const size_t mb = eigen_bytes(n_per_cycle);
    const size_t mbytes = ((size_t)C * sizeof(uint64_t) + 255) & ~size_t(255);
    const size_t hbytes = (size_t)C * P.nts * sizeof(uint64_t);
    if ((rc = ensure(p->work, mb + mbytes + hbytes + 256))) return rc;
    uint64_t *m_dev = (uint64_t *)((char *)p->work.p + mb);
    unsigned long long *hist = (unsigned long long *)((char *)p->work.p + mb + mbytes);
    ZERO(hist, hbytes);
    int *no_sites = R.overflow;
    if ((rc = launch_eigen(P, R, n_per_cycle, n_inactive, n_active, seed, p->work.p, m_dev, no_sites, hist, st)))
        return rc;
    Profiler none;
    if ((rc = fold(p, R, out, st, none))) return rc;
    HIP_CHECK(hipEventRecord(ev.b, st), "hipEventRecord");
    Collect c{};
    if ((rc = collect_begin(p, R, out, c, st))) return rc;
    std::vector<uint64_t> m(C), h((size_t)C * P.nts);
    HIP_CHECK(hipMemcpyAsync(m.data(), m_dev, C * sizeof(uint64_t), hipMemcpyDeviceToHost, st), "copy sites");
    HIP_CHECK(hipMemcpyAsync(h.data(), hist, hbytes, hipMemcpyDeviceToHost, st), "copy source histogram");
    HIP_CHECK(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (c.ovf) {
        set_error("a cycle banked no fission site");
        return MCDC_E_INVALID;
    }
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
    if ((rc = collect_end(p, n_tally, c, out, ms))) return rc;
    double sum = 0.0;
    for (int j = 0; j < C; ++j) {
        const double k = (double)m[j] / (double)n_per_cycle;
        if (k_cycle) k_cycle[j] = k;
        if (j >= n_inactive) sum += k;
    }
    out->k_mean = sum / n_active;
    double acc = 0.0;
    for (int j = n_inactive; j < C; ++j) {
        const double d = (double)m[j] / (double)n_per_cycle - out->k_mean;
        acc += d * d;
    }
    out->k_std = n_active > 1 ? std::sqrt(acc / ((double)(n_active - 1) * n_active)) : 0.0;
    if (source_hist) std::memcpy(source_hist, h.data(), hbytes);
    if (entropy)
        for (int j = 0; j < C; ++j) {
            // Shannon entropy of the cycle's sites over the spatial bins
            const uint64_t *hj = h.data() + (size_t)j * P.nts;
            double tot = 0.0;
            for (int t = 0; t < P.nts; ++t) tot += (double)hj[t];
            double e = 0.0;
            for (int t = 0; t < P.nts && tot > 0.0; ++t)
                if (hj[t]) {
                    const double q = (double)hj[t] / tot;
                    e -= q * std::log2(q);
                }
            entropy[j] = e;
        }
    return MCDC_OK;
}
