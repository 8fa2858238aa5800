// History-based tracking (the paper's current algorithm, Section 2): one
// thread follows one particle from birth to death with its whole state in
// registers.  Track-length scores go straight to the per-batch tally in HBM
// through hardware FP64 atomics.
//
// With weight windows, split progeny are written to a split bank and
// tracked in further rounds (one kernel per generation) until none are
// left; a history's records and detector score then come from several
// particles and are accumulated per history with atomics.
#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

struct BlockCounters {
    unsigned int c[kCounters];
};

struct Acc {
    unsigned int n_ev[3] = {0u, 0u, 0u};
    unsigned int term_mask = 0u;
    unsigned int spawned = 0u;
    double track = 0.0, qoi = 0.0;
};

// Track one particle of history hid until it terminates; returns the
// termination code (also ORed into acc.term_mask).  Split progeny go to the
// split bank.
template <int FM, bool WW>
__device__ __forceinline__ int track(const DevProblem &P, const RunArgs &R, Particle &p, int b, uint64_t hid,
                                     Acc &acc, const SplitBank &SB) {
    double *S = R.S + (int64_t)b * P.ntally;
    int cell = cell_index(P, p.ix);
    int since = 0;
    int code = -1;
    while (code < 0) {
        if (since >= kMaxEventsPerStep) {
            code = kLost;
            break;
        }
        ++since;
        const Flight f = next_event<FM>(P, p, cell);
        if (f.d == kInf) {
            code = kLost;
            break;
        }
        const double sc = p.w * f.d;
        const int tb = P.cell_tal[cell];
        if (tb >= 0) {
            atomic_add_f64(S + ((int64_t)p.k * P.G + p.g) * P.nts + tb, sc);
            acc.track += sc;
        }
        if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) acc.qoi += sc;
        move<FM>(P, p, f);
        bool check = false;
        if (f.ev == kCensus) {
            ++acc.n_ev[0];
            since = 0;
            p.k += 1;
            if (p.k == P.K)
                code = kTime;
            else
                check = WW;
        } else if (f.ev == kSurface) {
            ++acc.n_ev[1];
            const int old_ww = WW ? P.cell_ww[cell] : 0;
            const int face = cross<FM>(P, p, crossing_mask<FM>(P, f));
            if (face >= 0) {
                atomic_add_f64(R.L + (((int64_t)b * P.K + p.k) * P.G + p.g) * 6 + face, p.w);
                code = kLeak;
            } else {
                cell = cell_index(P, p.ix);
                check = WW && (P.cell_ww[cell] != old_ww);
            }
        } else {
            ++acc.n_ev[2];
            if (!collide<FM>(P, p, f.m))
                code = kAbsorb;
            else
                check = WW;
        }
        if (WW && check) {
            int nc = 0;
            if (!ww_check(P, p, cell, nc)) {
                code = kRoulette;
            } else if (nc > 0) {
                if (!spawn_children(SB, p, nc, b, hid)) *R.overflow = 1;
                acc.spawned += (unsigned int)nc;
            }
        }
    }
    acc.term_mask |= 1u << code;
    return code;
}

template <int FM, bool WW>
__global__ void __launch_bounds__(256) k_history(DevProblem P, RunArgs R, uint64_t first, uint64_t count,
                                                 uint64_t chunk_first, SplitBank SB) {
    __shared__ BlockCounters bc;
    __shared__ double qsum[2];
    if (threadIdx.x < kCounters) bc.c[threadIdx.x] = 0u;
    if (threadIdx.x < 2) qsum[threadIdx.x] = 0.0;
    __syncthreads();

    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < count) {
        const uint64_t i = first + r;
        const int b = (int)(((i + 1) * (uint64_t)R.B - 1) / R.N);
        Particle p;
        Acc acc;
        if (!birth<FM>(P, history_stream(P, R.seed, i), p)) {
            acc.term_mask = 1u << kTime;
            atomicAdd(&bc.c[3 + kTime], 1u);
        } else {
            atomicAdd(&bc.c[3 + track<FM, WW>(P, R, p, b, i, acc, SB)], 1u);
        }
        // children of this history are tracked in later launches, so plain
        // stores here precede their atomic updates
        if (R.dbg_counts) {
            uint32_t *d = R.dbg_counts + i * 5;
            d[0] = acc.n_ev[0];
            d[1] = acc.n_ev[1];
            d[2] = acc.n_ev[2];
            d[3] = 1u + acc.spawned;
            d[4] = acc.term_mask;
        }
        if (R.dbg_scores) {
            R.dbg_scores[i * 2 + 0] = acc.track;
            R.dbg_scores[i * 2 + 1] = acc.qoi;
        }
        if (WW) {
            if (P.qoi_on) R.qoi_hist[i - chunk_first] = acc.qoi;
        } else if (P.qoi_on && acc.qoi != 0.0) {
            atomicAdd(&qsum[0], acc.qoi);
            atomicAdd(&qsum[1], acc.qoi * acc.qoi);
        }
        for (int e = 0; e < 3; ++e)
            if (acc.n_ev[e]) atomicAdd(&bc.c[e], acc.n_ev[e]);
        if (acc.spawned) atomicAdd(&bc.c[8], acc.spawned);
    }
    __syncthreads();
    if (threadIdx.x < kCounters && bc.c[threadIdx.x])
        atomicAdd(R.counters + threadIdx.x, (unsigned long long)bc.c[threadIdx.x]);
    if (!WW && P.qoi_on && threadIdx.x < 2 && qsum[threadIdx.x] != 0.0)
        atomic_add_f64(R.qoi_sums + threadIdx.x, qsum[threadIdx.x]);
    if (R.prof && threadIdx.x == 0) {
        const uint64_t lo = (uint64_t)blockIdx.x * blockDim.x;
        const uint64_t nb = (count > lo) ? ((count - lo < blockDim.x) ? count - lo : blockDim.x) : 0;
        atomicAdd(R.prof + 2 * MCDC_PROF_HISTORY, (unsigned long long)nb);
    }
}

// One generation of split progeny: each thread tracks one child to death
// and adds its records to its history with atomics.
template <int FM>
__global__ void __launch_bounds__(256) k_history_children(DevProblem P, RunArgs R, SplitBank in, unsigned int n,
                                                          uint64_t chunk_first, SplitBank out) {
    __shared__ BlockCounters bc;
    if (threadIdx.x < kCounters) bc.c[threadIdx.x] = 0u;
    __syncthreads();
    const unsigned int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        Particle p;
        int b;
        uint64_t i;
        split_load(in, r, p, b, i);
        set_inverse<FM>(P, p);
        Acc acc;
        atomicAdd(&bc.c[3 + track<FM, true>(P, R, p, b, i, acc, out)], 1u);
        if (R.dbg_counts) {
            uint32_t *d = R.dbg_counts + i * 5;
            for (int e = 0; e < 3; ++e)
                if (acc.n_ev[e]) atomicAdd(d + e, acc.n_ev[e]);
            if (acc.spawned) atomicAdd(d + 3, acc.spawned);
            atomicOr(d + 4, acc.term_mask);
        }
        if (R.dbg_scores) {
            if (acc.track != 0.0) atomic_add_f64(R.dbg_scores + i * 2, acc.track);
            if (acc.qoi != 0.0) atomic_add_f64(R.dbg_scores + i * 2 + 1, acc.qoi);
        }
        if (P.qoi_on && acc.qoi != 0.0) atomic_add_f64(R.qoi_hist + (i - chunk_first), acc.qoi);
        for (int e = 0; e < 3; ++e)
            if (acc.n_ev[e]) atomicAdd(&bc.c[e], acc.n_ev[e]);
        if (acc.spawned) atomicAdd(&bc.c[8], acc.spawned);
    }
    __syncthreads();
    if (threadIdx.x < kCounters && bc.c[threadIdx.x])
        atomicAdd(R.counters + threadIdx.x, (unsigned long long)bc.c[threadIdx.x]);
}

__global__ void k_zero_count(unsigned int *c) { *c = 0u; }

SplitBank carve_split(void *mem, unsigned int cap, unsigned int *count) {
    SplitBank B{};
    char *p = (char *)mem;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += (bytes + 255) & ~size_t(255);
        return r;
    };
    for (int a = 0; a < 3; ++a) B.x[a] = (double *)take((size_t)cap * 8);
    for (int a = 0; a < 3; ++a) B.u[a] = (double *)take((size_t)cap * 8);
    B.t = (double *)take((size_t)cap * 8);
    B.tau = (double *)take((size_t)cap * 8);
    B.w = (double *)take((size_t)cap * 8);
    B.s = (uint64_t *)take((size_t)cap * 8);
    B.ixyz = (uint32_t *)take((size_t)cap * 4);
    B.gk = (uint32_t *)take((size_t)cap * 4);
    B.hid = (uint64_t *)take((size_t)cap * 8);
    B.count = count;
    B.cap = cap;
    return B;
}

size_t split_bytes(unsigned int cap) { return (size_t)cap * (13 * 8 + 8) + 16 * 256; }

template <int FM, bool WW>
void launch_main(const DevProblem &P, const RunArgs &R, uint64_t first, uint64_t count, uint64_t chunk_first,
                 const SplitBank &SB, hipStream_t st, Profiler &prof) {
    const int bs = 256;
    const uint64_t grid = (count + bs - 1) / bs;
    launch_timed(prof, MCDC_PROF_HISTORY, k_history<FM, WW>, dim3((unsigned)grid), dim3(bs), 0u, st, P, R, first,
                 count, chunk_first, SB);
}

// Split progeny of one chunk, generation by generation, until none are left
// (the count of each generation is read back to size the next launch).
template <int FM>
int run_generations(const DevProblem &P, const RunArgs &R, SplitBank SB[2], uint64_t cfirst, hipStream_t st,
                    Profiler &prof) {
    for (int gen = 0;; ++gen) {
        unsigned int n_in = 0;
        hipError_t e = hipMemcpyAsync(&n_in, SB[gen & 1].count, sizeof(unsigned int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "split count");
        if (n_in == 0) return MCDC_OK;
        if (n_in > SB[gen & 1].cap || gen > 10000) {
            set_error("split bank overflow (weight windows split too many particles)");
            return MCDC_E_OVERFLOW;
        }
        const SplitBank &in = SB[gen & 1], &out = SB[(gen + 1) & 1];
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, out.count);
        launch_timed(prof, MCDC_PROF_HISTORY, k_history_children<FM>, dim3((n_in + 255) / 256), dim3(256), 0u, st,
                     P, R, in, n_in, cfirst, out);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "history children launch");
    }
}

template <int FM>
int run_history(mcdc_problem *pb, const RunArgs &R0, uint64_t first, uint64_t count, hipStream_t st,
                Profiler &prof) {
    const DevProblem &P = pb->d;
    const bool ww = P.ww_center != nullptr;
    RunArgs R = R0;
    // analog runs keep the detector score in registers; weight-window runs
    // assemble it per history in chunks
    const uint64_t chunk = ww ? ((count < (1ULL << 24)) ? count : (1ULL << 24)) : count;
    SplitBank SB[2]{};
    int rc;
    if (ww) {
        if ((rc = split_prepare(pb, chunk, SB))) return rc;
        if (P.qoi_on) {
            if ((rc = ensure(pb->qoi_hist, chunk * sizeof(double)))) return rc;
            R.qoi_hist = (double *)pb->qoi_hist.p;
        }
    }
    for (uint64_t c0 = 0; c0 < count; c0 += chunk) {
        const uint64_t n = (count - c0 < chunk) ? count - c0 : chunk;
        const uint64_t cfirst = first + c0;
        if (ww) split_reset(SB, st);
        if (ww)
            launch_main<FM, true>(P, R, cfirst, n, cfirst, SB[0], st, prof);
        else
            launch_main<FM, false>(P, R, cfirst, n, cfirst, SB[0], st, prof);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "history kernel launch");
        if (!ww) continue;
        if ((rc = run_generations<FM>(P, R, SB, cfirst, st, prof))) return rc;
        if (P.qoi_on && (rc = launch_qoi_reduce(R.qoi_hist, n, R.qoi_sums, st)))
            return hip_fail((hipError_t)rc, "detector reduce");
    }
    return MCDC_OK;
}

// ---------------------------------------------------------------------------
// batched solve: many problems, one persistent launch
// ---------------------------------------------------------------------------
// Workgroups pull chunks of BS * per_thread consecutive histories of the
// concatenated history ranges from one device-wide counter until none are
// left (every workgroup exits when the counter passes the total).
template <int FM, int BS>
__global__ void __launch_bounds__(BS) k_history_batched(const BatchItem *__restrict__ items,
                                                        const uint64_t *__restrict__ offs, int n_items,
                                                        uint64_t total, unsigned long long *next, int per_thread) {
    __shared__ unsigned long long base_s;
    __shared__ int j0_s;
    __shared__ unsigned int cnt[2][kCounters];
    const uint64_t chunk = (uint64_t)BS * per_thread;
    SplitBank none{};
    for (;;) {
        if (threadIdx.x == 0) {
            base_s = atomicAdd(next, (unsigned long long)chunk);
            int lo = 0, hi = n_items - 1;   // largest j with offs[j] <= base
            const uint64_t b0 = base_s;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (offs[mid] <= b0)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            j0_s = lo;
        }
        if (threadIdx.x < 2 * kCounters) (&cnt[0][0])[threadIdx.x] = 0u;
        __syncthreads();
        const uint64_t base = base_s;
        const int j0 = j0_s;
        if (base >= total) break;
        for (int m = 0; m < per_thread; ++m) {
            const uint64_t gi = base + (uint64_t)m * BS + threadIdx.x;
            if (gi >= total) break;
            int j = j0;
            while (gi >= offs[j + 1]) ++j;
            const BatchItem &it = items[j];
            const uint64_t i = gi - offs[j];
            const int b = (int)(((i + 1) * (uint64_t)it.R.B - 1) / it.R.N);
            Particle p;
            Acc acc;
            int code = kTime;
            if (birth<FM>(it.P, history_stream(it.P, it.R.seed, i), p))
                code = track<FM, false>(it.P, it.R, p, b, i, acc, none);
            const int slot = j - j0;
            if (slot < 2) {
                for (int e = 0; e < 3; ++e)
                    if (acc.n_ev[e]) atomicAdd(&cnt[slot][e], acc.n_ev[e]);
                atomicAdd(&cnt[slot][3 + code], 1u);
            } else {
                for (int e = 0; e < 3; ++e)
                    if (acc.n_ev[e]) atomicAdd(it.R.counters + e, (unsigned long long)acc.n_ev[e]);
                atomicAdd(it.R.counters + 3 + code, 1ull);
            }
            if (it.P.qoi_on && acc.qoi != 0.0) {
                atomic_add_f64(it.R.qoi_sums, acc.qoi);
                atomic_add_f64(it.R.qoi_sums + 1, acc.qoi * acc.qoi);
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * kCounters) {
            const int slot = threadIdx.x / kCounters, c = threadIdx.x % kCounters;
            const unsigned int v = cnt[slot][c];
            if (v && j0 + slot < n_items) atomicAdd(items[j0 + slot].R.counters + c, (unsigned long long)v);
        }
        __syncthreads();
    }
}

template <int FM, int BS>
int launch_batched_bs(const BatchItem *items, const uint64_t *offs, int n_items, uint64_t total,
                      unsigned long long *next, int per_thread, hipStream_t st) {
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&k_history_batched<FM, BS>),
                                                         BS, 0);
    if (e != hipSuccess) return hip_fail(e, "batched launch shape");
    if (occ < 1) occ = 1;
    hipLaunchKernelGGL((k_history_batched<FM, BS>), dim3((unsigned)(cus * occ)), dim3(BS), 0, st, items, offs, n_items,
                       total, next, per_thread);
    e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "batched launch");
}

template <int FM>
int launch_batched_fm(const BatchItem *items, const uint64_t *offs, int n_items, uint64_t total,
                      unsigned long long *next, int block, int per_thread, hipStream_t st) {
    switch (block) {
    case 64: return launch_batched_bs<FM, 64>(items, offs, n_items, total, next, per_thread, st);
    case 128: return launch_batched_bs<FM, 128>(items, offs, n_items, total, next, per_thread, st);
    case 512: return launch_batched_bs<FM, 512>(items, offs, n_items, total, next, per_thread, st);
    default: return launch_batched_bs<FM, 256>(items, offs, n_items, total, next, per_thread, st);
    }
}

}  // namespace

int launch_batched(const BatchItem *items, const uint64_t *offs, int n_items, uint64_t total,
                   unsigned long long *next, int finite_mask, int block, int per_thread, hipStream_t st) {
    if (finite_mask == 7) return launch_batched_fm<7>(items, offs, n_items, total, next, block, per_thread, st);
    if (finite_mask == 1) return launch_batched_fm<1>(items, offs, n_items, total, next, block, per_thread, st);
    return launch_batched_fm<0>(items, offs, n_items, total, next, block, per_thread, st);
}

int split_prepare(mcdc_problem *pb, uint64_t chunk, dev::SplitBank SB[2]) {
    const unsigned int cap = (unsigned int)((chunk < (1u << 22)) ? (1u << 22) : chunk);
    int rc;
    if ((rc = ensure(pb->split, 2 * split_bytes(cap) + 256))) return rc;
    if ((rc = ensure(pb->counters_split, 2 * sizeof(unsigned int)))) return rc;
    unsigned int *cnt = (unsigned int *)pb->counters_split.p;
    SB[0] = carve_split(pb->split.p, cap, cnt);
    SB[1] = carve_split((char *)pb->split.p + split_bytes(cap), cap, cnt + 1);
    return MCDC_OK;
}

void split_reset(const dev::SplitBank SB[2], hipStream_t st) {
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, SB[0].count);
}

int split_generations(mcdc_problem *pb, const RunArgs &R, dev::SplitBank SB[2], uint64_t cfirst, hipStream_t st,
                      Profiler &prof) {
    const int fm = pb->d.finite_mask;
    if (fm == 1) return run_generations<1>(pb->d, R, SB, cfirst, st, prof);
    if (fm == 7) return run_generations<7>(pb->d, R, SB, cfirst, st, prof);
    return run_generations<0>(pb->d, R, SB, cfirst, st, prof);
}

int launch_history(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count, int block, hipStream_t st,
                   Profiler &prof) {
    (void)block;
    if (count == 0) return MCDC_OK;
    if (p->h.B > 1023) {
        set_error("at most 1023 batches");
        return MCDC_E_UNSUPPORTED;
    }
    const int fm = p->d.finite_mask;
    if (fm == 1) return run_history<1>(p, R, first, count, st, prof);
    if (fm == 7) return run_history<7>(p, R, first, count, st, prof);
    return run_history<0>(p, R, first, count, st, prof);
}

}  // namespace mcdc
