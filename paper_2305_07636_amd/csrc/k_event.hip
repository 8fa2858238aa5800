// Event-based tracking (the second algorithm mode the paper names, Section 2;
// it gives no design).  Particles live in structure-of-arrays banks in HBM
// and advance one event per kernel pass; after each pass they are sorted
// into per-event queues (census, surface, collision) built with wavefront
// ballot + mbcnt prefix sums and one atomic per wave and queue.
//
// Time is advanced census step by census step (the census grid is the tally
// time grid, Section 3).  One step is a fixed kernel sequence, so it can be
// replayed without host round trips:
//   advance(dense bank) -> surface(queue) -> collision(queue)
//   [advance(active queue) -> surface -> collision] x (iters - 1)
//   finish(active queue)
// advance moves each particle to its next event, scores the track-length
// tally and files it: census crossers are copied whole into the next step's
// dense bank, surface and collision particles stay in place and their slots
// go to the surface / collision queues; the surface and collision kernels
// append survivors to the active queue.  finish takes the few particles
// still in flight after the last iteration to their census or death in
// registers, so no step needs an unbounded number of passes.
#include <vector>

#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

constexpr int kBlock = 256;

struct Bank {
    double *x[3], *u[3], *t, *tau, *w;
    uint64_t *s;
    uint32_t *ixyz;   // ix | iy << 11 | iz << 22
    uint32_t *gk;     // g | batch << 5 | k << 15
    uint32_t *hid;    // history index within the chunk
};

// Device-resident queue counts and step index.  Every queue iteration j of
// a step has its own surface / collision / active counts, so nothing needs
// resetting between iterations; the step's counts are cleared once when the
// previous step ends.
constexpr int kMaxIters = 16;
struct Ctl {
    unsigned int n_cur, n_next;
    unsigned int n_s[kMaxIters], n_c[kMaxIters], n_a[kMaxIters];
    int step;
    int pad;
    uint64_t first;   // global index of the chunk's first history
};

// LDS-privatised tally of one census step.  Every particle scored in step
// k lies in time bin k, so a block only touches the slice [B][G][nts];
// when that fits in LDS each block accumulates it there and writes it out
// as one row of per-block partials (no global atomics, no contention on
// the few bins of a step), and one reduction per step adds the rows into
// the per-batch tally in a fixed order.
struct StepTally {
    double *partial;     // [rows][n] per-block partial slices
    uint8_t *row_used;   // [rows] 1 if the block scored anything
    int n;               // B * G * nts (0 = slice too large: global atomics)
    int row0;            // first row of this launch (launch index * grid)
};

// End of a scoring kernel: write the block's slice as its partial row.
// Contains the block barrier the counter flush needs.
__device__ __forceinline__ void flush_tally(const StepTally &T, const double *lt, bool scored) {
    const int any = __syncthreads_or(scored ? 1 : 0);
    if (T.n == 0) return;
    const int64_t row = (int64_t)T.row0 + blockIdx.x;
    if (threadIdx.x == 0) T.row_used[row] = any ? 1 : 0;
    if (!any) return;
    double *dst = T.partial + row * T.n;
    for (int j = threadIdx.x; j < T.n; j += blockDim.x) dst[j] = lt[j];
}

__device__ __forceinline__ uint32_t pack_gk(int g, int b, int k) {
    return (uint32_t)g | ((uint32_t)b << 5) | ((uint32_t)k << 15);
}
__device__ __forceinline__ uint32_t pack_ix(const int ix[3]) {
    return (uint32_t)ix[0] | ((uint32_t)ix[1] << 11) | ((uint32_t)ix[2] << 22);
}

// Wave-aggregated append: lanes with pred get consecutive slots of the
// queue behind counter, in lane order; one atomic per wave.
__device__ __forceinline__ uint32_t wave_append(bool pred, unsigned int *counter) {
    const uint64_t mask = __ballot(pred);
    const uint32_t prefix =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    uint32_t base = 0;
    if (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        if ((int)__lane_id() == leader) base = atomicAdd(counter, (unsigned int)__popcll(mask));
        base = __shfl(base, leader);
    }
    return base + prefix;
}

// Per-block event / termination counters and profile tallies (particles
// processed, algorithmic bytes requested), flushed once per block.
struct Counters {
    unsigned int c[kCounters];
    unsigned long long items, bytes;
    __device__ void init() {
        if (threadIdx.x < kCounters) c[threadIdx.x] = 0u;
        if (threadIdx.x == 0) items = bytes = 0ull;
    }
    __device__ void add(int j, unsigned int v = 1u) {
        if (v) atomicAdd(&c[j], v);
    }
    __device__ void prof(unsigned int n_items, unsigned int n_bytes) {
        if (n_items) atomicAdd(&items, (unsigned long long)n_items);
        if (n_bytes) atomicAdd(&bytes, (unsigned long long)n_bytes);
    }
    __device__ void flush(const RunArgs &R, int cls) {
        if (threadIdx.x < kCounters && c[threadIdx.x]) atomicAdd(R.counters + threadIdx.x, (unsigned long long)c[threadIdx.x]);
        if (R.prof && threadIdx.x == 0) {
            atomicAdd(R.prof + 2 * cls, items);
            atomicAdd(R.prof + 2 * cls + 1, bytes);
        }
    }
};

// Bytes of the particle state as the kernels move it (finite axes only).
template <int FM, bool WW>
__device__ __forceinline__ unsigned int nfinite(const DevProblem &P) {
    return (unsigned int)__popc((unsigned int)(FM ? FM : P.finite_mask));
}
// load_state: x, u per finite axis, t, tau, (w), ixyz, gk
template <int FM, bool WW>
__device__ __forceinline__ unsigned int load_bytes(const DevProblem &P) {
    return 16u * nfinite<FM, WW>(P) + 24u + (WW ? 8u : 0u);
}
// store_state: the whole particle (load_state fields + s + hid)
template <int FM, bool WW>
__device__ __forceinline__ unsigned int state_bytes(const DevProblem &P) {
    return load_bytes<FM, WW>(P) + 12u;
}

struct Hist {   // per-history debug / detector hooks
    uint64_t first;
    __device__ static void event(const RunArgs &R, uint64_t i, int e) {
        if (R.dbg_counts) atomicAdd(R.dbg_counts + i * 5 + e, 1u);
    }
    __device__ static void term(const RunArgs &R, uint64_t i, int code) {
        if (R.dbg_counts) atomicOr(R.dbg_counts + i * 5 + 4, 1u << code);
    }
};

template <int FM, bool WW>
__device__ __forceinline__ void load_state(const DevProblem &P, const Bank &B, uint32_t slot, Particle &p,
                                           uint32_t &gk) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            p.x[a] = B.x[a][slot];
            p.u[a] = B.u[a][slot];
        }
    }
    set_inverse<FM>(P, p);
    p.t = B.t[slot];
    p.tau = B.tau[slot];
    p.w = WW ? B.w[slot] : 1.0;
    const uint32_t c = B.ixyz[slot];
    p.ix[0] = c & 2047u;
    p.ix[1] = (c >> 11) & 2047u;
    p.ix[2] = c >> 22;
    gk = B.gk[slot];
    p.g = gk & 31u;
    p.k = gk >> 15;
}

template <int FM, bool WW>
__device__ __forceinline__ void store_state(const DevProblem &P, const Bank &B, uint32_t slot,
                                            const Particle &p, uint32_t gk, uint32_t hid) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            B.x[a][slot] = p.x[a];
            B.u[a][slot] = p.u[a];
        }
    }
    B.t[slot] = p.t;
    B.tau[slot] = p.tau;
    if (WW) B.w[slot] = p.w;
    B.s[slot] = p.s;
    B.ixyz[slot] = pack_ix(p.ix);
    B.gk[slot] = gk;
    B.hid[slot] = hid;
}

__device__ __forceinline__ uint32_t with_gk(uint32_t gk, const Particle &p) {
    return (uint32_t)p.g | (gk & (1023u << 5)) | ((uint32_t)p.k << 15);
}

// ---------------------------------------------------------------------------
// source
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_SOURCE>
__global__ void __launch_bounds__(kBlock) k_source(DevProblem P, RunArgs R, Bank cur, Ctl *ctl,
                                                   uint64_t first, uint64_t count) {
    __shared__ Counters cnt;
    cnt.init();
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < count; base += (uint64_t)gridDim.x * kBlock) {
        const uint64_t r = base + threadIdx.x;
        const bool valid = r < count;
        Particle p;
        bool alive = false;
        int b = 0;
        if (valid) {
            const uint64_t i = first + r;
            b = (int)(((i + 1) * (uint64_t)R.B - 1) / R.N);
            alive = birth<FM>(P, history_stream(P, R.seed, i), p);
            if (R.dbg_counts) R.dbg_counts[i * 5 + 3] = 1u;
            if (!alive) {
                cnt.add(3 + kTime);
                Hist::term(R, i, kTime);
            }
        }
        const uint32_t slot = wave_append(valid && alive, &ctl->n_cur);
        if (valid && alive) store_state<FM, WW>(P, cur, slot, p, pack_gk(p.g, b, p.k), (uint32_t)r);
        if (R.prof) cnt.prof(valid ? 1u : 0u, (valid && alive) ? state_bytes<FM, WW>(P) : 0u);
    }
    __syncthreads();
    cnt.flush(R, CLS);
}

// ---------------------------------------------------------------------------
// advance: one flight per particle, score, file into a queue
// ---------------------------------------------------------------------------
enum Outcome : int { kNone = 0, kToNext = 1, kToSurface = 2, kToCollision = 3 };

template <int FM, bool WW, bool DENSE, int CLS = DENSE ? MCDC_PROF_ADVANCE : MCDC_PROF_ADVANCE_Q>
__global__ void __launch_bounds__(kBlock) k_advance(DevProblem P, RunArgs R, Bank cur, Bank next, Ctl *ctl,
                                                    const uint32_t *__restrict__ aq, int it,
                                                    uint32_t *sq, uint32_t *cq, StepTally T) {
    __shared__ Counters cnt;
    const uint64_t first = ctl->first;
    extern __shared__ double lt[];
    cnt.init();
    for (int j = threadIdx.x; j < T.n; j += kBlock) lt[j] = 0.0;
    __syncthreads();
    bool scored = false;
    const unsigned int n = DENSE ? ctl->n_cur : ctl->n_a[it - 1];
    const int step = ctl->step;
    const bool per_hist = (R.dbg_counts != nullptr) || (R.dbg_scores != nullptr) || P.qoi_on;
    for (unsigned int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const unsigned int idx = base + threadIdx.x;
        const bool valid = idx < n;
        const uint32_t slot = valid ? (DENSE ? idx : aq[idx]) : 0u;
        int outcome = kNone;
        int mask = 0;
        Particle p;
        uint32_t gk = 0, hid = 0;
        if (valid) {
            load_state<FM, WW>(P, cur, slot, p, gk);
            if (per_hist) hid = cur.hid[slot];
            if (p.k > step) {
                outcome = kToNext;   // born in a later time bin: wait
            } else {
                const int cell = cell_index(P, p.ix);
                Flight f = next_event<FM>(P, p, cell);
                const uint64_t i = first + hid;
                if (f.d == kInf) {
                    cnt.add(3 + kLost);
                    if (per_hist) Hist::term(R, i, kLost);
                } else {
                    const double sc = p.w * f.d;
                    const int tb = P.cell_tal[cell];
                    const int b = (gk >> 5) & 1023u;
                    if (tb >= 0) {
                        if (T.n) {
                            atomicAdd(&lt[(b * P.G + p.g) * P.nts + tb], sc);
                            scored = true;
                        } else {
                            atomic_add_f64(R.S + (int64_t)b * P.ntally + ((int64_t)p.k * P.G + p.g) * P.nts + tb, sc);
                        }
                        if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2, sc);
                    }
                    if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) {
                        atomic_add_f64(R.qoi_hist + hid, sc);
                        if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2 + 1, sc);
                    }
                    move<FM>(P, p, f);
                    if (f.ev == kCensus) {
                        cnt.add(0);
                        if (per_hist) Hist::event(R, i, 0);
                        p.k += 1;
                        if (p.k == P.K) {
                            cnt.add(3 + kTime);
                            if (per_hist) Hist::term(R, i, kTime);
                        } else {
                            outcome = kToNext;
                        }
                    } else if (f.ev == kSurface) {
                        cnt.add(1);
                        if (per_hist) Hist::event(R, i, 1);
                        mask = crossing_mask<FM>(P, f);
                        outcome = kToSurface;
                    } else {
                        cnt.add(2);
                        if (per_hist) Hist::event(R, i, 2);
                        outcome = kToCollision;
                    }
                }
            }
        }
        const uint32_t ns = wave_append(outcome == kToNext, &ctl->n_next);
        const uint32_t ss = wave_append(outcome == kToSurface, &ctl->n_s[it]);
        const uint32_t cs = wave_append(outcome == kToCollision, &ctl->n_c[it]);
        if (outcome == kToNext) {
            p.s = cur.s[slot];
            if (!per_hist) hid = cur.hid[slot];
            store_state<FM, WW>(P, next, ns, p, with_gk(gk, p), hid);
        } else if (outcome == kToSurface || outcome == kToCollision) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (finite_axis<FM>(P, a)) cur.x[a][slot] = p.x[a];
            cur.t[slot] = p.t;
            cur.tau[slot] = p.tau;
            if (outcome == kToSurface)
                sq[ss] = slot | ((uint32_t)mask << 29);
            else
                cq[cs] = slot;
        }
        if (R.prof && valid) {
            unsigned int by = load_bytes<FM, WW>(P) + (DENSE ? 0u : 4u) + (per_hist ? 4u : 0u);
            if (outcome == kToNext)
                by += 8u + (per_hist ? 0u : 4u) + state_bytes<FM, WW>(P);
            else if (outcome != kNone)
                by += 8u * nfinite<FM, WW>(P) + 16u + 4u;
            cnt.prof(1u, by);
        }
    }
    flush_tally(T, lt, scored);
    cnt.flush(R, CLS);
}

// ---------------------------------------------------------------------------
// surface crossing and boundary conditions
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_SURFACE>
__global__ void __launch_bounds__(kBlock) k_surface(DevProblem P, RunArgs R, Bank cur, Ctl *ctl,
                                                    const uint32_t *__restrict__ sq, uint32_t *aq_out,
                                                    int it) {
    __shared__ Counters cnt;
    const uint64_t first = ctl->first;
    cnt.init();
    __syncthreads();
    const unsigned int n = ctl->n_s[it];
    for (unsigned int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const unsigned int idx = base + threadIdx.x;
        const bool valid = idx < n;
        bool alive = false;
        uint32_t slot = 0;
        Particle p;
        if (valid) {
            const uint32_t e = sq[idx];
            slot = e & 0x1FFFFFFFu;
            const int mask = (int)(e >> 29);
            uint32_t gk;
            load_state<FM, WW>(P, cur, slot, p, gk);
            const int face = cross<FM>(P, p, mask);
            if (face >= 0) {
                const int b = (gk >> 5) & 1023u;
                atomic_add_f64(R.L + (((int64_t)b * P.K + p.k) * P.G + p.g) * 6 + face, p.w);
                cnt.add(3 + kLeak);
                if (R.dbg_counts) Hist::term(R, first + cur.hid[slot], kLeak);
            } else {
                alive = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (finite_axis<FM>(P, a) && ((mask >> a) & 1)) {
                        cur.x[a][slot] = p.x[a];
                        cur.u[a][slot] = p.u[a];
                    }
                }
                cur.ixyz[slot] = pack_ix(p.ix);
            }
        }
        const uint32_t as = wave_append(alive, &ctl->n_a[it]);
        if (alive) aq_out[as] = slot;
        if (R.prof && valid) {
            unsigned int by = 4u + load_bytes<FM, WW>(P);
            if (alive) by += 16u * (unsigned int)__popc(sq[idx] >> 29) + 4u + 4u;
            cnt.prof(1u, by);
        }
    }
    __syncthreads();
    cnt.flush(R, CLS);
}

// ---------------------------------------------------------------------------
// analog collision
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_COLLISION>
__global__ void __launch_bounds__(kBlock) k_collision(DevProblem P, RunArgs R, Bank cur, Ctl *ctl,
                                                      const uint32_t *__restrict__ cq, uint32_t *aq_out,
                                                      int it) {
    __shared__ Counters cnt;
    const uint64_t first = ctl->first;
    cnt.init();
    __syncthreads();
    const unsigned int n = ctl->n_c[it];
    for (unsigned int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const unsigned int idx = base + threadIdx.x;
        const bool valid = idx < n;
        bool alive = false;
        uint32_t slot = 0;
        Particle p;
        if (valid) {
            slot = cq[idx];
            const uint32_t gk = cur.gk[slot];
            p.g = gk & 31u;
            p.s = cur.s[slot];
            const uint32_t c = cur.ixyz[slot];
            const int ix[3] = {(int)(c & 2047u), (int)((c >> 11) & 2047u), (int)(c >> 22)};
            const int m = P.cell_mat[cell_index(P, ix)];
            if (collide<FM>(P, p, m)) {
                alive = true;
                cur.s[slot] = p.s;
                cur.gk[slot] = (gk & ~31u) | (uint32_t)p.g;
                cur.tau[slot] = p.tau;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (finite_axis<FM>(P, a)) cur.u[a][slot] = p.u[a];
            } else {
                cur.s[slot] = p.s;
                cnt.add(3 + kAbsorb);
                if (R.dbg_counts) Hist::term(R, first + cur.hid[slot], kAbsorb);
            }
        }
        const uint32_t as = wave_append(alive, &ctl->n_a[it]);
        if (alive) aq_out[as] = slot;
        if (R.prof && valid)
            cnt.prof(1u, 20u + 8u + (alive ? 16u + 8u * nfinite<FM, WW>(P) + 4u : 0u));
    }
    __syncthreads();
    cnt.flush(R, CLS);
}

// ---------------------------------------------------------------------------
// finish: the particles still in flight, in registers, to census or death
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_FINISH>
__global__ void __launch_bounds__(kBlock) k_finish(DevProblem P, RunArgs R, Bank cur, Bank next, Ctl *ctl,
                                                   const uint32_t *__restrict__ aq, int it, StepTally T) {
    __shared__ Counters cnt;
    const uint64_t first = ctl->first;
    extern __shared__ double lt[];
    cnt.init();
    for (int j = threadIdx.x; j < T.n; j += kBlock) lt[j] = 0.0;
    __syncthreads();
    bool scored = false;
    const unsigned int n = ctl->n_a[it - 1];
    const bool per_hist = (R.dbg_counts != nullptr) || (R.dbg_scores != nullptr) || P.qoi_on;
    for (unsigned int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const unsigned int idx = base + threadIdx.x;
        const bool valid = idx < n;
        bool to_next = false;
        Particle p;
        uint32_t gk = 0, hid = 0;
        if (valid) {
            const uint32_t slot = aq[idx];
            load_state<FM, WW>(P, cur, slot, p, gk);
            p.s = cur.s[slot];
            hid = cur.hid[slot];
            const uint64_t i = first + hid;
            const int b = (gk >> 5) & 1023u;
            double *S = R.S + (int64_t)b * P.ntally;
            int cell = cell_index(P, p.ix);
            int since = 0;
            for (;;) {
                if (since >= kMaxEventsPerStep) {
                    cnt.add(3 + kLost);
                    if (per_hist) Hist::term(R, i, kLost);
                    break;
                }
                ++since;
                Flight f = next_event<FM>(P, p, cell);
                if (f.d == kInf) {
                    cnt.add(3 + kLost);
                    if (per_hist) Hist::term(R, i, kLost);
                    break;
                }
                const double sc = p.w * f.d;
                const int tb = P.cell_tal[cell];
                if (tb >= 0) {
                    if (T.n) {
                        atomicAdd(&lt[(b * P.G + p.g) * P.nts + tb], sc);
                        scored = true;
                    } else {
                        atomic_add_f64(S + ((int64_t)p.k * P.G + p.g) * P.nts + tb, sc);
                    }
                    if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2, sc);
                }
                if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) {
                    atomic_add_f64(R.qoi_hist + hid, sc);
                    if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2 + 1, sc);
                }
                move<FM>(P, p, f);
                if (f.ev == kCensus) {
                    cnt.add(0);
                    if (per_hist) Hist::event(R, i, 0);
                    p.k += 1;
                    if (p.k == P.K) {
                        cnt.add(3 + kTime);
                        if (per_hist) Hist::term(R, i, kTime);
                    } else {
                        to_next = true;
                    }
                    break;
                } else if (f.ev == kSurface) {
                    cnt.add(1);
                    if (per_hist) Hist::event(R, i, 1);
                    const int face = cross<FM>(P, p, crossing_mask<FM>(P, f));
                    if (face >= 0) {
                        atomic_add_f64(R.L + (((int64_t)b * P.K + p.k) * P.G + p.g) * 6 + face, p.w);
                        cnt.add(3 + kLeak);
                        if (per_hist) Hist::term(R, i, kLeak);
                        break;
                    }
                    cell = cell_index(P, p.ix);
                } else {
                    cnt.add(2);
                    if (per_hist) Hist::event(R, i, 2);
                    if (!collide<FM>(P, p, f.m)) {
                        cnt.add(3 + kAbsorb);
                        if (per_hist) Hist::term(R, i, kAbsorb);
                        break;
                    }
                }
            }
        }
        const uint32_t ns = wave_append(to_next, &ctl->n_next);
        if (to_next) store_state<FM, WW>(P, next, ns, p, with_gk(gk, p), hid);
        if (R.prof && valid)
            cnt.prof(1u, 4u + load_bytes<FM, WW>(P) + 12u + (to_next ? state_bytes<FM, WW>(P) : 0u));
    }
    flush_tally(T, lt, scored);
    cnt.flush(R, CLS);
}

// Sum the partial rows of one step into the per-batch tally: 64 columns
// per block, 4 row lanes, fixed order (deterministic).
__global__ void __launch_bounds__(256) k_tally_reduce(StepTally T, int rows, const Ctl *ctl, double *S,
                                                      int64_t ntally, int gn) {
    __shared__ double red[4][64];
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int lane = threadIdx.x >> 6;
    double acc = 0.0;
    if (col < T.n)
        for (int r = lane; r < rows; r += 4)
            if (T.row_used[r]) acc += T.partial[(int64_t)r * T.n + col];
    red[lane][threadIdx.x & 63] = acc;
    __syncthreads();
    if (lane == 0 && col < T.n) {
        const double v = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
        const int b = col / gn;
        const int rem = col - b * gn;
        S[(int64_t)b * ntally + (int64_t)ctl->step * gn + rem] += v;
    }
}

// ---------------------------------------------------------------------------
// control
// ---------------------------------------------------------------------------
__device__ __forceinline__ void clear_step(Ctl *c) {
    c->n_next = 0u;
    for (int j = 0; j < kMaxIters; ++j) c->n_s[j] = c->n_c[j] = c->n_a[j] = 0u;
}
__global__ void k_ctl_init(Ctl *c, uint64_t first) {
    c->n_cur = 0u;
    c->step = 0;
    c->first = first;
    clear_step(c);
}
// end of a step: the census bank becomes the next step's dense bank
__global__ void k_step_end(Ctl *c) {
    c->n_cur = c->n_next;
    c->step += 1;
    clear_step(c);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Layout {
    Bank bank[2];
    uint32_t *sq, *cq, *aq[2];
    Ctl *ctl;
};

size_t bank_bytes(uint64_t C) { return C * (11 * sizeof(double) + sizeof(uint64_t) + 3 * sizeof(uint32_t)); }

Layout carve(void *bank_mem, void *queue_mem, uint64_t C) {
    Layout L{};
    char *p = (char *)bank_mem;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += (bytes + 255) & ~size_t(255);
        return r;
    };
    for (int k = 0; k < 2; ++k) {
        Bank &B = L.bank[k];
        for (int a = 0; a < 3; ++a) B.x[a] = (double *)take(C * 8);
        for (int a = 0; a < 3; ++a) B.u[a] = (double *)take(C * 8);
        B.t = (double *)take(C * 8);
        B.tau = (double *)take(C * 8);
        B.w = (double *)take(C * 8);
        B.s = (uint64_t *)take(C * 8);
        B.ixyz = (uint32_t *)take(C * 4);
        B.gk = (uint32_t *)take(C * 4);
        B.hid = (uint32_t *)take(C * 4);
    }
    char *q = (char *)queue_mem;
    auto takeq = [&](size_t bytes) {
        char *r = q;
        q += (bytes + 255) & ~size_t(255);
        return r;
    };
    L.sq = (uint32_t *)takeq(C * 4);
    L.cq = (uint32_t *)takeq(C * 4);
    L.aq[0] = (uint32_t *)takeq(C * 4);
    L.aq[1] = (uint32_t *)takeq(C * 4);
    L.ctl = (Ctl *)takeq(sizeof(Ctl));
    return L;
}

size_t queue_bytes(uint64_t C) { return 4 * (((C * 4) + 255) & ~size_t(255)) + 256; }

// Captured census steps (one graph per bank parity), cached per problem and
// re-captured when any kernel argument changes.
struct StepGraphs {
    std::vector<char> key;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipStream_t cs = nullptr;
    void clear() {
        for (int q = 0; q < 2; ++q) {
            if (exec[q]) (void)hipGraphExecDestroy(exec[q]);
            if (graph[q]) (void)hipGraphDestroy(graph[q]);
            exec[q] = nullptr;
            graph[q] = nullptr;
        }
        key.clear();
    }
};

template <class T>
void key_add(std::vector<char> &k, const T &v) {
    const char *p = reinterpret_cast<const char *>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

template <int FM, bool WW>
int run_event(mcdc_problem *pb, const RunArgs &R0, uint64_t first, uint64_t count, const mcdc_run_options &opt,
              hipStream_t st, Profiler &prof) {
    const DevProblem &P = pb->d;
    uint64_t C = opt.bank_capacity ? (uint64_t)opt.bank_capacity : (uint64_t)1 << 24;
    if (C > count) C = count;
    if (C > (1ULL << 29)) C = 1ULL << 29;
    int iters = opt.event_iters > 0 ? opt.event_iters : 3;
    if (iters > kMaxIters - 1) iters = kMaxIters - 1;
    int rc;
    if ((rc = ensure(pb->bank, bank_bytes(C) * 2 + 64 * 256))) return rc;
    if ((rc = ensure(pb->queues, queue_bytes(C)))) return rc;
    if (P.qoi_on && (rc = ensure(pb->qoi_hist, C * sizeof(double)))) return rc;
    Layout L = carve(pb->bank.p, pb->queues.p, C);
    RunArgs R = R0;
    R.qoi_hist = (double *)pb->qoi_hist.p;

    // per-step tally slice in LDS when it fits (32 KB)
    const int64_t gn = (int64_t)P.G * P.nts;
    const int64_t slice = (int64_t)R.B * gn;
    const bool lds = slice <= 4096;
    const unsigned grid_max = lds ? 1024u : 2048u;
    unsigned grid = (unsigned)((C + kBlock - 1) / kBlock);
    if (grid > grid_max) grid = grid_max;
    StepTally T{};
    const int launches_per_step = iters + 1;   // advance x iters + finish
    if (lds) {
        T.n = (int)slice;
        const size_t rows = (size_t)launches_per_step * grid;
        if ((rc = ensure(pb->tally_part, rows * slice * sizeof(double) + rows + 256))) return rc;
        T.partial = (double *)pb->tally_part.p;
        T.row_used = (uint8_t *)((char *)pb->tally_part.p + rows * slice * sizeof(double));
    }
    const size_t shmem = lds ? (size_t)slice * sizeof(double) : 0;

    // the step kernels never read the seed or the history count
    RunArgs Rs = R;
    Rs.seed = 0;
    Rs.N = 0;

    auto enqueue_step = [&](int par, hipStream_t s, Profiler &pr) {
        const Bank &cur = L.bank[par];
        const Bank &nxt = L.bank[par ^ 1];
        StepTally t = T;
        int launch = 0;
        t.row0 = launch++ * (int)grid;
        pr.begin(MCDC_PROF_ADVANCE);
        hipLaunchKernelGGL((k_advance<FM, WW, true>), dim3(grid), dim3(kBlock), shmem, s, P, Rs, cur, nxt, L.ctl,
                           (const uint32_t *)nullptr, 0, L.sq, L.cq, t);
        pr.end();
        pr.begin(MCDC_PROF_SURFACE);
        hipLaunchKernelGGL((k_surface<FM, WW>), dim3(grid), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                           (const uint32_t *)L.sq, L.aq[0], 0);
        pr.end();
        pr.begin(MCDC_PROF_COLLISION);
        hipLaunchKernelGGL((k_collision<FM, WW>), dim3(grid), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                           (const uint32_t *)L.cq, L.aq[0], 0);
        pr.end();
        for (int j = 1; j < iters; ++j) {
            t.row0 = launch++ * (int)grid;
            pr.begin(MCDC_PROF_ADVANCE_Q);
            hipLaunchKernelGGL((k_advance<FM, WW, false>), dim3(grid), dim3(kBlock), shmem, s, P, Rs, cur, nxt,
                               L.ctl, (const uint32_t *)L.aq[(j - 1) & 1], j, L.sq, L.cq, t);
            pr.end();
            pr.begin(MCDC_PROF_SURFACE);
            hipLaunchKernelGGL((k_surface<FM, WW>), dim3(grid), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                               (const uint32_t *)L.sq, L.aq[j & 1], j);
            pr.end();
            pr.begin(MCDC_PROF_COLLISION);
            hipLaunchKernelGGL((k_collision<FM, WW>), dim3(grid), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                               (const uint32_t *)L.cq, L.aq[j & 1], j);
            pr.end();
        }
        t.row0 = launch++ * (int)grid;
        pr.begin(MCDC_PROF_FINISH);
        hipLaunchKernelGGL((k_finish<FM, WW>), dim3(grid), dim3(kBlock), shmem, s, P, Rs, cur, nxt, L.ctl,
                           (const uint32_t *)L.aq[(iters - 1) & 1], iters, t);
        pr.end();
        if (lds) {
            pr.begin(MCDC_PROF_OTHER);
            hipLaunchKernelGGL(k_tally_reduce, dim3((unsigned)((slice + 63) / 64)), dim3(256), 0, s, t,
                               launch * (int)grid, (const Ctl *)L.ctl, R.S, P.ntally, (int)gn);
            pr.end();
        }
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, s, L.ctl);
    };

    // replay captured steps unless a per-launch profile or per-history
    // debug output is requested (those launch eagerly)
    const bool use_graph = !(opt.flags & MCDC_FLAG_EAGER) && !opt.profile && !R.dbg_counts && !R.dbg_scores && P.K > 1;
    StepGraphs *G = nullptr;
    if (use_graph) {
        if (!pb->graph_cache) pb->graph_cache = new StepGraphs();
        G = (StepGraphs *)pb->graph_cache;
        std::vector<char> key;
        key_add(key, P);
        key_add(key, Rs);
        key_add(key, L);
        key_add(key, T);
        key_add(key, grid);
        key_add(key, iters);
        key_add(key, shmem);
        if (key != G->key) {
            G->clear();
            hipError_t e = hipSuccess;
            if (!G->cs) e = hipStreamCreateWithFlags(&G->cs, hipStreamNonBlocking);
            Profiler none;
            for (int q = 0; q < 2 && e == hipSuccess; ++q) {
                e = hipStreamBeginCapture(G->cs, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) break;
                enqueue_step(q, G->cs, none);
                e = hipStreamEndCapture(G->cs, &G->graph[q]);
                if (e == hipSuccess) e = hipGraphInstantiate(&G->exec[q], G->graph[q], nullptr, nullptr, 0);
            }
            if (e != hipSuccess) {
                G->clear();
                return hip_fail(e, "census step capture");
            }
            G->key = key;
        }
    }

    for (uint64_t c0 = 0; c0 < count; c0 += C) {
        const uint64_t n = (count - c0 < C) ? count - c0 : C;
        const uint64_t cfirst = first + c0;
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, st, L.ctl, cfirst);
        if (P.qoi_on && (rc = launch_zero(R.qoi_hist, n * sizeof(double), st))) return hip_fail((hipError_t)rc, "zero");
        unsigned sgrid = (unsigned)((n + kBlock - 1) / kBlock);
        if (sgrid > grid_max) sgrid = grid_max;
        prof.begin(MCDC_PROF_SOURCE);
        hipLaunchKernelGGL((k_source<FM, WW>), dim3(sgrid), dim3(kBlock), 0, st, P, R, L.bank[0], L.ctl, cfirst, n);
        prof.end();
        for (int step = 0; step < P.K; ++step) {
            if (G) {
                hipError_t e = hipGraphLaunch(G->exec[step & 1], st);
                if (e != hipSuccess) return hip_fail(e, "census step replay");
            } else {
                enqueue_step(step & 1, st, prof);
            }
        }
        if (P.qoi_on && (rc = launch_qoi_reduce(R.qoi_hist, n, R.qoi_sums, st)))
            return hip_fail((hipError_t)rc, "detector reduce");
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "event kernel launch");
    }
    return MCDC_OK;
}

}  // namespace

void destroy_graph_cache(mcdc_problem *p) {
    if (!p->graph_cache) return;
    StepGraphs *G = (StepGraphs *)p->graph_cache;
    G->clear();
    if (G->cs) (void)hipStreamDestroy(G->cs);
    delete G;
    p->graph_cache = nullptr;
}

int launch_event(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count,
                 const mcdc_run_options &opt, hipStream_t st, Profiler &prof) {
    const DevProblem &P = p->d;
    if (p->h.B > 1023 || P.K > 131071) {
        set_error("event form supports at most 1023 batches and 131071 time bins");
        return MCDC_E_UNSUPPORTED;
    }
    if (P.ww_center != nullptr) {
        set_error("weight windows run with the history-based algorithm");
        return MCDC_E_UNSUPPORTED;
    }
    if (P.finite_mask == 1) return run_event<1, false>(p, R, first, count, opt, st, prof);
    if (P.finite_mask == 7) return run_event<7, false>(p, R, first, count, opt, st, prof);
    return run_event<0, false>(p, R, first, count, opt, st, prof);
}

}  // namespace mcdc
