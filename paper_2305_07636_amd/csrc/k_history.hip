// History-based tracking (the paper's current algorithm, Section 2): one
// thread follows one particle from birth to death with its whole state in
// registers.  Track-length scores go straight to the per-batch tally in HBM
// through hardware FP64 atomics.
//
// With weight windows, split progeny are written to a split bank and
// tracked in further rounds (one kernel per generation) until none are
// left; a history's records and detector score then come from several
// particles and are accumulated per history with atomics.
#include <chrono>
#include <thread>

#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

struct Acc {
    unsigned int n_ev[3] = {0u, 0u, 0u};
    unsigned int term_mask = 0u;
    unsigned int spawned = 0u;     // window-split progeny
    unsigned int fissioned = 0u;   // fission neutrons beyond the colliding one
    double track = 0.0, qoi = 0.0;
};

constexpr int kCollisionPending = -2;

// A lane's track-length score held back while its next scores go to the
// same tally bin (one atomic then carries their sum).
struct Held {
    double *a = nullptr;
    double v = 0.0;
    __device__ __forceinline__ void add(double *x, double w) {
        if (x == a) {
            v += w;
        } else {
            if (a) atomic_add_f64(a, v);
            a = x;
            v = w;
        }
    }
    __device__ __forceinline__ void release() {
        if (a) atomic_add_f64(a, v);
        a = nullptr;
    }
};

// Weight-window check point after an event (roulette or split).
template <bool WW>
__device__ __forceinline__ int ww_after(const DevProblem &P, const RunArgs &R, Particle &p, int cell, int b,
                                        uint64_t hid, Acc &acc, const SplitBank &SB, bool check, int code) {
    if (WW && check) {
        int nc = 0;
        if (!ww_check(P, p, cell, nc)) {
            code = kRoulette;
        } else if (nc > 0) {
            if (!spawn_children(SB, p, nc, b, hid)) *R.overflow = 1;
            acc.spawned += (unsigned int)nc;
        }
    }
    return code;
}

// The collision of a particle of history hid in material m; returns the
// termination code, or -1 while the particle lives.
template <int FM, bool WW>
__device__ __forceinline__ int hcollide(const DevProblem &P, const RunArgs &R, Particle &p, int cell, int b,
                                        uint64_t hid, Acc &acc, const SplitBank &SB, int m) {
    bool check = false;
    int code = -1;
    const int r = collide<FM, WW>(P, p, m);
    if (r == 0) {
        code = kAbsorb;
    } else if (WW && r == 3) {
        code = kRoulette;
    } else if (WW && r == 2) {
        const int n = fission<FM>(P, p, m, SB, b, hid, R.overflow);
        if (n == 0) {
            code = kAbsorb;
        } else {
            acc.fissioned += (unsigned int)(n - 1);
            check = true;
        }
    } else {
        check = WW;
    }
    return ww_after<WW>(P, R, p, cell, b, hid, acc, SB, check, code);
}

// One flight of a particle of history hid and its census or surface event;
// returns the termination code, -1 while the particle lives, or
// kCollisionPending when the flight ends in a collision (its material in
// m_coll), which hcollide then applies.  Split progeny go to the split bank.
// (slice: the workgroup's LDS copy of batch b0's track-length tally, or
// nullptr: a score of that batch goes there, any other to HBM)
template <int FM, bool WW>
__device__ __forceinline__ int hflight(const DevProblem &P, const RunArgs &R, Particle &p, int &cell, int b,
                                       uint64_t hid, Acc &acc, const SplitBank &SB, int &since, int &m_coll,
                                       Held &held, double *slice = nullptr, int b0 = -1) {
    if (since >= kMaxEventsPerStep) return kLost;
    ++since;
    const Flight f = next_event<FM>(P, p, cell);
    if (f.d == kInf) return kLost;
    const double sc = p.w * f.d;
    const int tb = P.cell_tal[cell];
    if (tb >= 0) {
        const int64_t j = ((int64_t)p.k * P.G + p.g) * P.nts + tb;
        if (slice && b == b0)
            atomicAdd(slice + j, sc);
        else
            held.add(tally_copy(P, R, b) + j, sc);
        acc.track += sc;
    }
    if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) acc.qoi += sc;
    move<FM>(P, p, f);
    bool check = false;
    int code = -1;
    if (f.ev == kCensus) {
        ++acc.n_ev[0];
        // time-crossing flux at the edge T_{k+1} the particle has reached
        if (P.tc_on && tb >= 0)
            atomic_add_f64(tally_copy(P, R, b) + P.ntally + ((int64_t)p.k * P.G + p.g) * P.nts + tb,
                           p.w * P.speed[p.g]);
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
            add_leak(P, R, b, p.k, p.g, face, p.w);
            code = kLeak;
        } else {
            cell = cell_index(P, p.ix);
            check = WW && (P.cell_ww[cell] != old_ww);
        }
    } else {
        ++acc.n_ev[2];
        m_coll = f.m;
        return kCollisionPending;
    }
    return ww_after<WW>(P, R, p, cell, b, hid, acc, SB, check, code);
}

// One flight of a particle of history hid and its event; returns the
// termination code, or -1 while the particle lives.
template <int FM, bool WW>
__device__ __forceinline__ int hstep(const DevProblem &P, const RunArgs &R, Particle &p, int &cell, int b,
                                     uint64_t hid, Acc &acc, const SplitBank &SB, int &since, Held &held) {
    int m = 0;
    const int code = hflight<FM, WW>(P, R, p, cell, b, hid, acc, SB, since, m, held);
    return code == kCollisionPending ? hcollide<FM, WW>(P, R, p, cell, b, hid, acc, SB, m) : code;
}

// A wave's persistent loop takes queued collisions only once they make up
// kCollEighths / 8 of its busy lanes (or every busy lane has one), so that
// the collision code runs for many lanes at once.  The progeny kernel
// waits for every busy lane when fission makes its collisions costly (each
// may bank neutrons) and takes them at 2/8 otherwise (measured on the
// supercritical pulse: 3/8 34.8 ms, 5/8 29.2, 8/8 26.3; on the windowed
// dog-leg: 0-2/8 1142 ms, 3/8 1173, 8/8 1684).
constexpr int kCollEighths = 3;
__device__ __forceinline__ int progeny_coll_eighths(const DevProblem &P) { return P.fission_on ? 8 : 2; }

// Track one particle of history hid until it terminates; returns the
// termination code (also ORed into acc.term_mask).
template <int FM, bool WW>
__device__ __forceinline__ int track(const DevProblem &P, const RunArgs &R, Particle &p, int b, uint64_t hid,
                                     Acc &acc, const SplitBank &SB, Held &held) {
    int cell = cell_index(P, p.ix);
    int since = 0;
    int code;
    do {
        code = hstep<FM, WW>(P, R, p, cell, b, hid, acc, SB, since, held);
    } while (code < 0);
    acc.term_mask |= 1u << code;
    return code;
}

// Per-lane totals of the persistent kernel, kept in registers (every
// index a compile-time constant) and reduced once at the end.
struct LaneTotals {
    unsigned int c[kCounters];
    double q[2];
    unsigned long long started;
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int j = 0; j < kCounters; ++j) c[j] = 0u;
        q[0] = q[1] = 0.0;
        started = 0ull;
    }
    __device__ __forceinline__ void term(int code) {
        if (code == kAbsorb)
            c[3 + kAbsorb] += 1u;
        else if (code == kLeak)
            c[3 + kLeak] += 1u;
        else if (code == kTime)
            c[3 + kTime] += 1u;
        else if (code == kLost)
            c[3 + kLost] += 1u;
        else
            c[3 + kRoulette] += 1u;
    }
};

// A history's records once its source particle has terminated (its split
// progeny, tracked in later launches, add theirs with atomics, so plain
// stores here come first).
template <bool WW>
__device__ __forceinline__ void end_history(const DevProblem &P, const RunArgs &R, const Acc &acc, int code,
                                            uint64_t i, uint64_t chunk_first, LaneTotals &lt) {
    lt.term(code);
    if (R.dbg_counts) {
        uint32_t *d = R.dbg_counts + i * 5;
        d[0] = acc.n_ev[0];
        d[1] = acc.n_ev[1];
        d[2] = acc.n_ev[2];
        d[3] = 1u + acc.spawned + acc.fissioned;
        d[4] = acc.term_mask;
    }
    if (R.dbg_scores) {
        R.dbg_scores[i * 2 + 0] = acc.track;
        R.dbg_scores[i * 2 + 1] = acc.qoi;
    }
    if (WW) {
        if (P.qoi_on) R.qoi_hist[i - chunk_first] = acc.qoi;
    } else if (P.qoi_on) {
        lt.q[0] += acc.qoi;
        lt.q[1] += acc.qoi * acc.qoi;
    }
    lt.c[0] += acc.n_ev[0];
    lt.c[1] += acc.n_ev[1];
    lt.c[2] += acc.n_ev[2];
    lt.c[8] += acc.spawned;
    lt.c[9] += acc.fissioned;
}

// Idle lanes that trigger a refill.  The histories a wave takes from the
// device-wide counter at a time scale with the job (about 16 takes per
// wave), so short histories do not serialise on that one counter.  The
// history kernel refills once half the wave is idle (each refill's loads
// then serve many lanes); the progeny kernel, whose particles end at
// scattered times and which waits on memory most of the time, refills as
// soon as a few lanes are idle.
constexpr int kRefillMin = 32, kRefillMinProgeny = 4;
// LDS budget for the persistent kernel's staged tables, and for its LDS
// slice of one batch's tally (analog runs).
constexpr int64_t kHistoryTablesMax = 40 * 1024;
constexpr int64_t kHistorySliceMax = 48 * 1024;

// Persistent history form: every wave takes chunks of consecutive histories
// [first, first + count) from a device counter; a lane whose particle has
// terminated starts the next history of the wave's chunk at once, so a
// wave is not held back by its longest history.  Every wave exits once the
// counter has passed the end and its lanes are idle.
// (LT: the flight tables are copied into LDS first; the workgroups live
// for the whole run, so the copy is paid once per workgroup.)
// (SL, analog runs whose tally of one batch fits in LDS: workgroup w takes
// the histories [w H, (w + 1) H) of the chunk, H = ceil(count / grid), its
// waves drawing chunks of them from a workgroup counter, so that they
// belong to one batch or two whenever a batch holds at least H histories;
// the track-length scores of the range's first batch b0 go to an LDS copy
// of that batch's tally (gn doubles behind the staged tables), added to HBM
// once at the end, and those of any later batch straight to HBM.)
template <int FM, bool WW, bool LT, bool SL = false>
__global__ void __launch_bounds__(256) k_history(DevProblem P0, RunArgs R, uint64_t first, uint64_t count,
                                                 uint64_t chunk_first, SplitBank SB, unsigned long long *next,
                                                 unsigned int wave_chunk, LdsTables tabs, int gn = 0) {
    __shared__ unsigned long long red[kCounters + 1];
    __shared__ double qsum[2];
    __shared__ unsigned long long wg_next;
    extern __shared__ double lds_tables[];
    if (threadIdx.x < kCounters + 1) red[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) qsum[threadIdx.x] = 0.0;
    if (threadIdx.x == 0) wg_next = 0ull;
    const DevProblem P = stage_tables<LT, 256>(P0, tabs, reinterpret_cast<char *>(lds_tables));
    // the workgroup's range and its slice
    uint64_t w_lo = 0, w_hi = count;
    int b0 = -1;
    double *slice = nullptr;
    if constexpr (SL) {
        const uint64_t H = (count + gridDim.x - 1) / gridDim.x;
        w_lo = (uint64_t)blockIdx.x * H;
        w_hi = (w_lo + H < count) ? w_lo + H : count;
        if (w_lo > count) w_lo = count;
        b0 = (int)(((first + w_lo + 1) * (uint64_t)R.B - 1) / R.N);
        slice = lds_tables + (LT ? (tabs.bytes + 15) / 16 * 2 : 0);
        for (int j = threadIdx.x; j < gn; j += 256) slice[j] = 0.0;
    }
    __syncthreads();

    uint64_t c_pos = 0, c_end = 0;   // the wave's current chunk (wave-uniform)
    uint64_t s_pos = 0;              // the stream of history first + c_pos
    bool drained = false;            // the device counter has passed the end
    LaneTotals tot;
    tot.init();
    Particle p;
    Acc acc;
    int b = 0, cell = 0, since = 0, pm = -1;   // pm: material of a queued collision, or -1
    uint64_t i = 0;
    bool busy = false;
    Held held;
    for (;;) {
        // idle lanes start the next histories of the chunk, once enough of
        // them are idle that the births run at a useful SIMD width
        uint64_t need = __ballot(!busy);
        if (__popcll(need) < kRefillMin && need != ~0ull) need = 0;
        while (need && !drained) {
            if (c_pos == c_end) {
                unsigned long long base = 0;
                if (__lane_id() == 0)
                    base = SL ? w_lo + atomicAdd(&wg_next, (unsigned long long)wave_chunk)
                              : atomicAdd(next, (unsigned long long)wave_chunk);
                base = __shfl(base, 0);
                if (base >= w_hi) {
                    drained = true;
                    break;
                }
                c_pos = base;
                c_end = (base + wave_chunk < w_hi) ? base + wave_chunk : w_hi;
                s_pos = history_stream(P, R.seed, first + c_pos);
            }
            const uint64_t avail = c_end - c_pos;
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            const uint32_t n_need = (uint32_t)__popcll(need);
            const uint32_t taken = (n_need < avail) ? n_need : (uint32_t)avail;
            if (!busy && rank < avail) {
                i = first + c_pos + rank;
                b = (int)(((i + 1) * (uint64_t)R.B - 1) / R.N);
                acc = Acc();
                ++tot.started;
                // (the stream from the wave's position in its chunk: at most
                // 64 histories ahead)
                if (birth<FM>(P, stream_skip(P, s_pos, rank), p)) {
                    cell = cell_index(P, p.ix);
                    since = 0;
                    pm = -1;
                    busy = true;
                } else {
                    acc.term_mask = 1u << kTime;
                    end_history<WW>(P, R, acc, kTime, i, chunk_first, tot);
                }
            }
            c_pos += taken;
            if (c_pos < c_end) s_pos = stream_skip(P, s_pos, taken);
            need = __ballot(!busy);
        }
        const int n_busy = __popcll(__ballot(busy));
        if (n_busy == 0) break;
        const bool pend = busy && pm >= 0;
        const int n_pend = __popcll(__ballot(pend));
        int code = -1;
        if (n_pend > 0 && (n_pend * 8 >= n_busy * kCollEighths || n_pend == n_busy) && pend) {
            code = hcollide<FM, WW>(P, R, p, cell, b, i, acc, SB, pm);
            pm = -1;
        }
        if (busy && pm < 0 && code < 0) {
            code = hflight<FM, WW>(P, R, p, cell, b, i, acc, SB, since, pm, held, slice, b0);
            if (code == kCollisionPending) code = -1;
            else pm = -1;
        }
        if (busy && code >= 0) {
            acc.term_mask |= 1u << code;
            end_history<WW>(P, R, acc, code, i, chunk_first, tot);
            busy = false;
        }
    }
    held.release();
    if constexpr (SL) {
        // the slice into batch b0's tally copy of this workgroup
        __syncthreads();
        if (b0 >= 0 && w_lo < w_hi) {
            double *dst = tally_copy(P, R, b0);
            for (int j = threadIdx.x; j < gn; j += 256)
                if (slice[j] != 0.0) atomic_add_f64(dst + j, slice[j]);
        }
    }
    // totals: wave reductions, then one atomic per counter and workgroup
#pragma unroll
    for (int j = 0; j < kCounters; ++j) {
        unsigned int v = tot.c[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (__lane_id() == 0 && v) atomicAdd(&red[j], (unsigned long long)v);
    }
    for (int o = 32; o > 0; o >>= 1) tot.started += __shfl_xor(tot.started, o);
    if (__lane_id() == 0) atomicAdd(&red[kCounters], tot.started);
    if (!WW && P.qoi_on) {
        for (int o = 32; o > 0; o >>= 1) {
            tot.q[0] += __shfl_xor(tot.q[0], o);
            tot.q[1] += __shfl_xor(tot.q[1], o);
        }
        if (__lane_id() == 0) {
            atomicAdd(&qsum[0], tot.q[0]);
            atomicAdd(&qsum[1], tot.q[1]);
        }
    }
    __syncthreads();
    if (threadIdx.x < kCounters && red[threadIdx.x]) atomicAdd(R.counters + threadIdx.x, red[threadIdx.x]);
    if (!WW && P.qoi_on && threadIdx.x < 2 && qsum[threadIdx.x] != 0.0)
        atomic_add_f64(R.qoi_sums + threadIdx.x, qsum[threadIdx.x]);
    if (R.prof && threadIdx.x == 0) atomicAdd(R.prof + 2 * MCDC_PROF_HISTORY, red[kCounters]);
}

// A progeny particle of history i has ended: its records go to the history
// with atomics (a history's progeny may run on any lane of any launch).
__device__ __forceinline__ void child_done(const DevProblem &P, const RunArgs &R, const Acc &acc, int code,
                                           uint64_t i, uint64_t chunk_first, LaneTotals &lt) {
    lt.term(code);
    if (R.dbg_counts) {
        uint32_t *d = R.dbg_counts + i * 5;
        for (int e = 0; e < 3; ++e)
            if (acc.n_ev[e]) atomicAdd(d + e, acc.n_ev[e]);
        if (acc.spawned + acc.fissioned) atomicAdd(d + 3, acc.spawned + acc.fissioned);
        atomicOr(d + 4, acc.term_mask);
    }
    if (R.dbg_scores) {
        if (acc.track != 0.0) atomic_add_f64(R.dbg_scores + i * 2, acc.track);
        if (acc.qoi != 0.0) atomic_add_f64(R.dbg_scores + i * 2 + 1, acc.qoi);
    }
    if (P.qoi_on && acc.qoi != 0.0) atomic_add_f64(R.qoi_hist + (i - chunk_first), acc.qoi);
    lt.c[0] += acc.n_ev[0];
    lt.c[1] += acc.n_ev[1];
    lt.c[2] += acc.n_ev[2];
    lt.c[8] += acc.spawned;
    lt.c[9] += acc.fissioned;
}

// One generation of progeny (window splits, fission neutrons), persistent
// like k_history: waves take chunks of the generation's entries [0, n) from
// a device counter, and a lane whose particle has ended loads the next entry
// of the wave's chunk once enough lanes are idle, so a wave is not held back
// by its longest-lived particle.  Their own progeny go to the next
// generation's bank.  (LT: flight tables in LDS.)
template <int FM, bool LT>
// (The generation's size is read here from the input bank's counter, so
// the host can queue several generations without reading it: an empty
// generation exits at once, and more progeny than the bank holds set the
// overflow flag instead of being read.)
__global__ void __launch_bounds__(256) k_history_children(DevProblem P0, RunArgs R, SplitBank in,
                                                          uint64_t chunk_first, SplitBank out,
                                                          unsigned long long *next, LdsTables tabs) {
    __shared__ unsigned long long red[kCounters];
    extern __shared__ double lds_tables[];
    const unsigned long long n_in = *in.count;
    if (n_in > in.cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *R.overflow = 1;
        return;
    }
    const unsigned long long n = n_in;
    if (n == 0) return;
    // entries per wave take: about 4 takes per wave of the grid, 64..65536
    // (measured on the supercritical pulse: 16 takes 25.2 ms, 4 takes 23.2;
    // 1 to 4 take the same time on both workloads tried)
    const unsigned long long waves = (unsigned long long)gridDim.x * (blockDim.x / 64);
    unsigned long long wcl = n / (waves * 4ull);
    wcl = (wcl < 64ull) ? 64ull : (wcl > 65536ull ? 65536ull : (wcl + 63ull) & ~63ull);
    const unsigned int wave_chunk = (unsigned int)wcl;
    if (threadIdx.x < kCounters) red[threadIdx.x] = 0ull;
    const DevProblem P = stage_tables<LT, 256>(P0, tabs, reinterpret_cast<char *>(lds_tables));
    const int coll_eighths = progeny_coll_eighths(P0);
    __syncthreads();

    uint64_t c_pos = 0, c_end = 0;   // the wave's current chunk (wave-uniform)
    bool drained = false;
    LaneTotals tot;
    tot.init();
    Particle p;
    Acc acc;
    int b = 0, cell = 0, since = 0, pm = -1;   // pm: material of a queued collision, or -1
    uint64_t i = 0;
    bool busy = false;
    Held held;
    for (;;) {
        uint64_t need = __ballot(!busy);
        if (__popcll(need) < kRefillMinProgeny && need != ~0ull) need = 0;
        while (need && !drained) {
            if (c_pos == c_end) {
                unsigned long long base = 0;
                if (__lane_id() == 0) base = atomicAdd(next, (unsigned long long)wave_chunk);
                base = __shfl(base, 0);
                if (base >= n) {
                    drained = true;
                    break;
                }
                c_pos = base;
                c_end = (base + wave_chunk < n) ? base + wave_chunk : n;
            }
            const uint64_t avail = c_end - c_pos;
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            const uint32_t n_need = (uint32_t)__popcll(need);
            if (!busy && rank < avail) {
                split_load(in, (unsigned int)(c_pos + rank), p, b, i);
                set_inverse<FM>(P, p);
                cell = cell_index(P, p.ix);
                since = 0;
                pm = -1;
                acc = Acc();
                busy = true;
            }
            c_pos += (n_need < avail) ? n_need : avail;
            need = __ballot(!busy);
        }
        const int n_busy = __popcll(__ballot(busy));
        if (n_busy == 0) break;
        const bool pend = busy && pm >= 0;
        const int n_pend = __popcll(__ballot(pend));
        int code = -1;
        if (n_pend > 0 && (n_pend * 8 >= n_busy * coll_eighths || n_pend == n_busy) && pend) {
            code = hcollide<FM, true>(P, R, p, cell, b, i, acc, out, pm);
            pm = -1;
        }
        if (busy && pm < 0 && code < 0) {
            code = hflight<FM, true>(P, R, p, cell, b, i, acc, out, since, pm, held);
            if (code == kCollisionPending) code = -1;
            else pm = -1;
        }
        if (busy && code >= 0) {
            acc.term_mask |= 1u << code;
            child_done(P, R, acc, code, i, chunk_first, tot);
            busy = false;
        }
    }
    held.release();
#pragma unroll
    for (int j = 0; j < kCounters; ++j) {
        unsigned int v = tot.c[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (__lane_id() == 0 && v) atomicAdd(&red[j], (unsigned long long)v);
    }
    __syncthreads();
    if (threadIdx.x < kCounters && red[threadIdx.x]) atomicAdd(R.counters + threadIdx.x, red[threadIdx.x]);
}

__global__ void k_zero_count(unsigned long long *c) { *c = 0ull; }
__global__ void k_zero_u64(unsigned long long *c) { *c = 0ull; }

SplitBank carve_split(void *mem, unsigned int cap, unsigned long long *count) {
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

// (nine doubles and the stream, 8 bytes each; ixyz and gk, 4 each; the
// history index, 8: 96 bytes an entry; each of the 13 arrays padded to 256)
size_t split_bytes(unsigned int cap) { return (size_t)cap * 96 + 13 * 256; }

// The persistent history kernel: as many workgroups as the GPU holds
// resident (no more than the work needs), and the work counter cleared.
template <int FM, bool WW>
int launch_main(mcdc_problem *pb, const DevProblem &P, const RunArgs &R, uint64_t first, uint64_t count,
                uint64_t chunk_first, const SplitBank &SB, hipStream_t st, Profiler &prof,
                unsigned long long *next_in = nullptr) {
    const int bs = 256;
    int rc;
    unsigned long long *next = next_in ? next_in : R.work;
    if (!next) {
        if ((rc = ensure(pb->work, 256))) return rc;
        next = (unsigned long long *)pb->work.p;
    }
    LdsTables tabs{};
    const bool lt = table_layout(P, tabs, kHistoryTablesMax);
    // analog slab runs (x the only finite axis) whose track-length tally of
    // one batch fits beside the tables score that batch in LDS (SL; the
    // time-crossing tally, if any, still goes to HBM; in 3-D problems the
    // slice's registers would cost a wave per SIMD)
    constexpr bool kSlice = FM == 1 && !WW;
    const int64_t gn64 = P.ntally;
    const bool sl = kSlice && lt && gn64 > 0 && gn64 * 8 <= kHistorySliceMax;
    const int gn = sl ? (int)gn64 : 0;
    const size_t shmem = lt ? (size_t)(tabs.bytes + 15) / 16 * 16 + (size_t)gn * 8 : 0;
    const void *kern = lt ? reinterpret_cast<const void *>(&k_history<FM, WW, true>)
                          : reinterpret_cast<const void *>(&k_history<FM, WW, false>);
    if constexpr (kSlice)
        if (sl) kern = reinterpret_cast<const void *>(&k_history<FM, WW, true, true>);
    int per_cu = 0, n_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, bs, shmem);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, pb->device);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    uint64_t grid = (uint64_t)(per_cu > 0 ? per_cu : 1) * (uint64_t)(n_cu > 0 ? n_cu : 1);
    const uint64_t waves = grid * (bs / 64);
    uint64_t wc = count / (waves * 16);
    wc = (wc < 256) ? 256 : (wc > 65536 ? 65536 : (wc + 63) & ~63ull);
    const uint64_t grid_needed = ((count + wc - 1) / wc + bs / 64 - 1) / (bs / 64);
    if (grid > grid_needed) grid = grid_needed;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, next);
    if constexpr (kSlice) {
        if (sl) {
            launch_timed(prof, MCDC_PROF_HISTORY, k_history<FM, WW, true, true>, dim3((unsigned)grid), dim3(bs),
                         (uint32_t)shmem, st, P, R, first, count, chunk_first, SB, next, (unsigned int)wc, tabs, gn);
            return MCDC_OK;
        }
    }
    if (lt)
        launch_timed(prof, MCDC_PROF_HISTORY, k_history<FM, WW, true>, dim3((unsigned)grid), dim3(bs),
                     (uint32_t)shmem, st, P, R, first, count, chunk_first, SB, next, (unsigned int)wc, tabs, 0);
    else
        launch_timed(prof, MCDC_PROF_HISTORY, k_history<FM, WW, false>, dim3((unsigned)grid), dim3(bs), 0u, st, P, R,
                     first, count, chunk_first, SB, next, (unsigned int)wc, tabs, 0);
    return MCDC_OK;
}

// Split progeny of one chunk, generation by generation, until none are left.
// Generations are queued kGensPerCheck at a time, each launch reading its
// input count on the device; the host reads the count once per batch.
constexpr int kGensPerCheck = 4;

// Launch shape of the persistent children kernel and its staged tables.
struct ChildShape {
    bool lt = false;
    LdsTables tabs{};
    size_t shmem = 0;
    uint64_t grid = 1;
};

template <int FM>
int child_shape(mcdc_problem *pb, ChildShape &cs) {
    const DevProblem &P = pb->d;
    cs.lt = table_layout(P, cs.tabs, kHistoryTablesMax);
    cs.shmem = cs.lt ? (size_t)cs.tabs.bytes : 0;
    int per_cu = 0, n_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, cs.lt ? reinterpret_cast<const void *>(&k_history_children<FM, true>)
                       : reinterpret_cast<const void *>(&k_history_children<FM, false>), 256, cs.shmem);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, pb->device);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    cs.grid = (uint64_t)(per_cu > 0 ? per_cu : 1) * (uint64_t)(n_cu > 0 ? n_cu : 1);
    return MCDC_OK;
}

// Queue generations gen .. gen + kGensPerCheck - 1 of a chunk's progeny on
// stream st (next: the children kernel's work counter of this bank pair).
template <int FM>
int queue_generations(const DevProblem &P, const RunArgs &R, const SplitBank SB[2], uint64_t cfirst, hipStream_t st,
                      Profiler &prof, int gen, unsigned long long *next, const ChildShape &cs) {
    for (int q = 0; q < kGensPerCheck; ++q, ++gen) {
        const SplitBank &in = SB[gen & 1], &out = SB[(gen + 1) & 1];
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, out.count);
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, next);
        if (cs.lt)
            launch_timed(prof, MCDC_PROF_HISTORY, k_history_children<FM, true>, dim3((unsigned)cs.grid), dim3(256),
                         (uint32_t)cs.shmem, st, P, R, in, cfirst, out, next, cs.tabs);
        else
            launch_timed(prof, MCDC_PROF_HISTORY, k_history_children<FM, false>, dim3((unsigned)cs.grid), dim3(256),
                         0u, st, P, R, in, cfirst, out, next, cs.tabs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "history children launch");
    }
    return MCDC_OK;
}

int overflow_error() {
    set_error("split bank overflow (window splits or fission made too many progeny in one generation; "
              "run fewer histories per chunk with bank_capacity)");
    return MCDC_E_OVERFLOW;
}

// Split progeny of one chunk, generation by generation, until none are
// left (the event form's weighted chunks).
template <int FM>
int run_generations(mcdc_problem *pb, const RunArgs &R, SplitBank SB[2], uint64_t cfirst, hipStream_t st,
                    Profiler &prof) {
    ChildShape cs;
    int rc;
    if ((rc = child_shape<FM>(pb, cs))) return rc;
    unsigned long long *next = (unsigned long long *)pb->counters_split.p + 2;
    for (int gen = 0;; gen += kGensPerCheck) {
        unsigned long long n_in = 0;
        hipError_t e = hipMemcpyAsync(&n_in, SB[gen & 1].count, sizeof(n_in), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "split count");
        if (n_in == 0) return MCDC_OK;
        if (n_in > SB[gen & 1].cap || gen > 10000) return overflow_error();
        if ((rc = queue_generations<FM>(pb->d, R, SB, cfirst, st, prof, gen, next, cs))) return rc;
    }
}

// Weighted chunks of the history form, kChunkStreams at a time: chunk c
// runs on one of the streams with its own split-bank pair, detector
// accumulator and work counters, so that the last, small generations of
// one chunk overlap the other chunks' histories.  The host starts a chunk
// as soon as a pair is free and queues the generations of each running
// chunk in batches, polling each batch's completion event and its copied
// count (no stream waits on another stream's progress).
// (measured against 2: 3 streams about the same, 4 streams 5 % faster on a
// windowed 1e8-history run in 48 chunks and 18 % on a 1e7-history fission
// run in 10; each stream holds two split banks of up to 2^26 entries)
constexpr int kChunkStreams = 4;
static_assert(kChunkStreams >= 1 && kChunkStreams <= kMaxChunkStreams, "chunk streams");

// The chunk streams of a weighted run of `count` histories in chunks of
// `chunk`, and the device memory they need (split banks, detector
// accumulators, work counters); allocating it twice is a no-op.
int weighted_streams(uint64_t count, uint64_t chunk) {
    const uint64_t n_chunks = (count + chunk - 1) / chunk;
    return (int)((n_chunks < (uint64_t)kChunkStreams) ? n_chunks : (uint64_t)kChunkStreams);
}
int weighted_reserve(mcdc_problem *pb, uint64_t chunk, int NS, SplitBank (*SB)[2]) {
    int rc;
    if ((rc = split_prepare_slots(pb, chunk, SB, NS))) return rc;
    if (pb->d.qoi_on && (rc = ensure(pb->qoi_hist, (size_t)NS * chunk * sizeof(double)))) return rc;
    return ensure(pb->work, (size_t)NS * 256);
}
uint64_t weighted_chunk(const DevProblem &P, uint64_t count, uint64_t chunk_opt) {
    const uint64_t cmax = chunk_opt ? chunk_opt : (P.fission_on ? kFissionChunk : kWindowChunk);
    return (count < cmax) ? count : cmax;
}

template <int FM>
int run_weighted_chunks(mcdc_problem *pb, const RunArgs &R0, uint64_t first, uint64_t count, uint64_t chunk,
                        hipStream_t st, Profiler &prof) {
    const DevProblem &P = pb->d;
    const int NS = weighted_streams(count, chunk);
    SplitBank SB[kMaxChunkStreams][2]{};
    int rc;
    if ((rc = weighted_reserve(pb, chunk, NS, SB))) return rc;
    ChildShape cs;
    if ((rc = child_shape<FM>(pb, cs))) return rc;
    hipError_t e = hipSuccess;
    for (int j = 0; j + 1 < NS && e == hipSuccess; ++j)
        if (!pb->aux_streams[j]) e = hipStreamCreateWithFlags((hipStream_t *)&pb->aux_streams[j], hipStreamNonBlocking);
    for (int j = 0; j < 2 * kMaxChunkStreams && e == hipSuccess; ++j)
        if (!pb->aux_events[j]) e = hipEventCreateWithFlags((hipEvent_t *)&pb->aux_events[j], hipEventDisableTiming);
    if (e == hipSuccess && !pb->host_counts)
        e = hipHostMalloc((void **)&pb->host_counts, kMaxChunkStreams * sizeof(unsigned long long),
                          hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "chunk streams");
    hipStream_t S[kMaxChunkStreams];
    hipEvent_t done[kMaxChunkStreams], joined[kMaxChunkStreams];
    for (int q = 0; q < kMaxChunkStreams; ++q) {
        S[q] = q == 0 ? st : (hipStream_t)pb->aux_streams[q - 1];
        done[q] = (hipEvent_t)pb->aux_events[q];
        joined[q] = (hipEvent_t)pb->aux_events[kMaxChunkStreams + q];
    }
    // the other streams start after everything queued on the caller's
    if (NS > 1) {
        e = hipEventRecord(joined[0], st);
        for (int q = 1; q < NS && e == hipSuccess; ++q) e = hipStreamWaitEvent(S[q], joined[0], 0);
        if (e != hipSuccess) return hip_fail(e, "chunk streams");
    }
    struct Slot {
        bool busy = false;
        uint64_t cfirst = 0, n = 0;
        int gen = 0;
        RunArgs R;
        unsigned long long *next_main = nullptr, *next_child = nullptr;
    } slot[kMaxChunkStreams];
    for (int q = 0; q < NS; ++q) {
        slot[q].R = R0;
        if (P.qoi_on) slot[q].R.qoi_hist = (double *)pb->qoi_hist.p + (size_t)q * chunk;
        slot[q].next_main = (unsigned long long *)((char *)pb->work.p + (size_t)q * 256);
        slot[q].next_child = (unsigned long long *)pb->counters_split.p + 3 * q + 2;
    }
    volatile unsigned long long *hc = pb->host_counts;
    // queue the next batch of a running chunk, then its count and event
    auto batch = [&](int q) -> int {
        Slot &sl = slot[q];
        int r = queue_generations<FM>(P, sl.R, SB[q], sl.cfirst, S[q], prof, sl.gen, sl.next_child, cs);
        if (r) return r;
        sl.gen += kGensPerCheck;
        hipError_t ee = hipMemcpyAsync((void *)(hc + q), SB[q][sl.gen & 1].count, sizeof(unsigned long long),
                                       hipMemcpyDeviceToHost, S[q]);
        if (ee == hipSuccess) ee = hipEventRecord(done[q], S[q]);
        return ee == hipSuccess ? MCDC_OK : hip_fail(ee, "split count");
    };
    uint64_t c0 = 0;
    for (;;) {
        bool progress = false, any = false;
        for (int q = 0; q < NS; ++q) {
            Slot &sl = slot[q];
            if (!sl.busy) {
                if (c0 >= count) continue;
                sl.cfirst = first + c0;
                sl.n = (count - c0 < chunk) ? count - c0 : chunk;
                sl.gen = 0;
                c0 += sl.n;
                split_reset(SB[q], S[q]);
                if ((rc = launch_main<FM, true>(pb, P, sl.R, sl.cfirst, sl.n, sl.cfirst, SB[q][0], S[q], prof,
                                                sl.next_main)))
                    return rc;
                e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(e, "history kernel launch");
                if ((rc = batch(q))) return rc;
                sl.busy = true;
                progress = any = true;
                continue;
            }
            any = true;
            e = hipEventQuery(done[q]);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return hip_fail(e, "split count");
            progress = true;
            const unsigned long long n_in = hc[q];
            if (n_in == 0) {
                if (P.qoi_on && (rc = launch_qoi_reduce(sl.R.qoi_hist, sl.n, sl.R.qoi_sums, S[q])))
                    return hip_fail((hipError_t)rc, "detector reduce");
                sl.busy = false;
                continue;
            }
            if (n_in > SB[q][sl.gen & 1].cap || sl.gen > 10000) return overflow_error();
            if ((rc = batch(q))) return rc;
        }
        if (!any && c0 >= count) break;
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    // the caller's stream waits for the other streams' work
    for (int q = 1; q < NS; ++q) {
        e = hipEventRecord(joined[q], S[q]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, joined[q], 0);
        if (e != hipSuccess) return hip_fail(e, "chunk streams");
    }
    return MCDC_OK;
}

template <int FM>
int run_history(mcdc_problem *pb, const RunArgs &R0, uint64_t first, uint64_t count, uint64_t chunk_opt,
                hipStream_t st, Profiler &prof) {
    const DevProblem &P = pb->d;
    const bool ww = has_progeny(P);
    // analog runs keep the detector score in registers; runs with progeny
    // (weight windows, fission) assemble it per history in chunks
    if (ww) return run_weighted_chunks<FM>(pb, R0, first, count, weighted_chunk(P, count, chunk_opt), st, prof);
    SplitBank none[2]{};
    int rc = launch_main<FM, false>(pb, P, R0, first, count, first, none[0], st, prof);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "history kernel launch");
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
    Held held;
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
                code = track<FM, false>(it.P, it.R, p, b, i, acc, none, held);
            if (it.R.dbg_counts) {
                uint32_t *d = it.R.dbg_counts + i * 5;
                d[0] = acc.n_ev[0];
                d[1] = acc.n_ev[1];
                d[2] = acc.n_ev[2];
                d[3] = 1u;
                d[4] = 1u << code;
            }
            if (it.R.dbg_scores) {
                it.R.dbg_scores[i * 2 + 0] = acc.track;
                it.R.dbg_scores[i * 2 + 1] = acc.qoi;
            }
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
    held.release();
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

// (slots: independent bank pairs, for chunks that run at the same time;
// pair q takes counters 3q, 3q + 1 and its children's work counter 3q + 2)
int split_prepare_slots(mcdc_problem *pb, uint64_t chunk, dev::SplitBank (*SB)[2], int slots) {
    // room for 32 progeny per history of the chunk in each generation (64
    // with fission; implicit capture alone makes none: the minimum), at
    // most 2^26 entries per bank (7.5 GB): 8 per history at the default
    // chunk of 2^23 histories
    const uint64_t per = pb->d.fission_on ? 64 : (pb->d.ww_center ? 32 : 0);
    const uint64_t want = per * chunk;
    const unsigned int cap = (unsigned int)((want < (1u << 22)) ? (1u << 22) : (want > (1u << 26) ? (1u << 26) : want));
    int rc;
    if (slots > kMaxChunkStreams) {
        set_error("too many chunk streams");
        return MCDC_E_INVALID;
    }
    for (int q = 0; q < slots; ++q)
        if ((rc = ensure(pb->split[q], 2 * split_bytes(cap) + 256))) return rc;
    // (two bank counters, then the children kernel's work counter)
    if ((rc = ensure(pb->counters_split, (size_t)slots * 3 * sizeof(unsigned long long)))) return rc;
    unsigned long long *cnt = (unsigned long long *)pb->counters_split.p;
    for (int q = 0; q < slots; ++q) {
        char *base = (char *)pb->split[q].p;
        SB[q][0] = carve_split(base, cap, cnt + 3 * q);
        SB[q][1] = carve_split(base + split_bytes(cap), cap, cnt + 3 * q + 1);
    }
    return MCDC_OK;
}

int split_prepare(mcdc_problem *pb, uint64_t chunk, dev::SplitBank SB[2]) {
    dev::SplitBank pair[1][2];
    const int rc = split_prepare_slots(pb, chunk, pair, 1);
    SB[0] = pair[0][0];
    SB[1] = pair[0][1];
    return rc;
}

void split_reset(const dev::SplitBank SB[2], hipStream_t st) {
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, SB[0].count);
}

int split_generations(mcdc_problem *pb, const RunArgs &R, dev::SplitBank SB[2], uint64_t cfirst, hipStream_t st,
                      Profiler &prof) {
    const int fm = pb->d.finite_mask;
    if (fm == 1) return run_generations<1>(pb, R, SB, cfirst, st, prof);
    if (fm == 7) return run_generations<7>(pb, R, SB, cfirst, st, prof);
    return run_generations<0>(pb, R, SB, cfirst, st, prof);
}

int history_reserve(mcdc_problem *p, uint64_t count, uint64_t chunk_opt) {
    if (count == 0 || !has_progeny(p->d)) return MCDC_OK;
    const uint64_t chunk = weighted_chunk(p->d, count, chunk_opt);
    SplitBank SB[kMaxChunkStreams][2]{};
    return weighted_reserve(p, chunk, weighted_streams(count, chunk), SB);
}

int launch_history(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count, uint64_t chunk,
                   hipStream_t st, Profiler &prof) {
    if (count == 0) return MCDC_OK;
    if (p->h.B > 1023) {
        set_error("at most 1023 batches");
        return MCDC_E_UNSUPPORTED;
    }
    const int fm = p->d.finite_mask;
    if (fm == 1) return run_history<1>(p, R, first, count, chunk, st, prof);
    if (fm == 7) return run_history<7>(p, R, first, count, chunk, st, prof);
    return run_history<0>(p, R, first, count, chunk, st, prof);
}

}  // namespace mcdc
