// Event-based tracking (the second algorithm mode the paper names, Section 2;
// it gives no design).  Particles live in structure-of-arrays banks in HBM
// and advance one event per kernel pass; after each pass they are sorted
// into per-event queues (census, surface, collision) built from wavefront
// ballots and mbcnt prefix counts.
//
// Segment-private pipelines.  The bank, and every queue, is cut into G
// segments of L slots, one per workgroup: workgroup b of every kernel works
// only on segment b, and a particle never leaves the segment it was born in.
// Queue appends therefore need no device-wide atomics (one LDS atomic per
// wave, no contention across the 8 XCDs), the dense census bank stays
// contiguous per segment, and each segment holds a contiguous range of
// histories, so its particles belong to at most two tally batches.
//
// Time is advanced census step by census step (the census grid is the tally
// time grid, Section 3).  One step is a fixed kernel sequence, captured once
// as a graph and replayed:
//   advance(dense bank) -> surface(queue) -> collision(queue)
//   [advance(active queue) -> surface -> collision] x (iters - 1)
//   finish(active queue) -> step end
// advance moves each particle to its next event, scores the track-length
// tally and files it: census crossers are copied whole into the next step's
// bank segment, surface and collision particles stay in place and their
// slots go to the surface / collision queues; the surface and collision
// kernels append survivors to the active queue.  finish takes the few
// particles still in flight after the last iteration to their census or
// death in registers, so no step needs an unbounded number of passes.
//
// Tally: every particle scored in step k lies in time bin k, so a
// workgroup touches only the slice [2 batches][G][nts] of the step; when that
// fits in LDS it is accumulated there and flushed with one global atomic
// per nonzero bin at the end of the kernel.
#include <vector>

#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

constexpr int kBlock = 256;
constexpr int kMaxIters = 16;
constexpr int kLdsTallyMax = 4096;   // doubles (32 KB)

struct Bank {
    double *x[3], *u[3], *t, *tau, *w;
    uint64_t *s;
    uint32_t *ixyz;   // ix | iy << 11 | iz << 22
    uint32_t *gk;     // g | batch << 5 | k << 15
    uint32_t *hid;    // history index within the chunk
};

// Per-segment fill counts of the banks and queues, plus the step index.
// Only workgroup b reads or writes the entries of segment b.
struct Ctl {
    unsigned int *n_bank;   // [2][G] particles in each segment of bank 0 / 1
    unsigned int *n_s;      // [kMaxIters][G] surface queue fill per iteration
    unsigned int *n_c;      // [kMaxIters][G] collision queue fill
    unsigned int *n_a;      // [kMaxIters][G] active queue fill
    int *seg_b0;            // [G] batch of the segment's first history
    int *step;              // current census step
    uint64_t *first;        // global index of the chunk's first history
    unsigned int G, L;      // segments (= workgroups), slots per segment
};

__device__ __forceinline__ uint32_t pack_gk(int g, int b, int k) {
    return (uint32_t)g | ((uint32_t)b << 5) | ((uint32_t)k << 15);
}
__device__ __forceinline__ uint32_t pack_ix(const int ix[3]) {
    return (uint32_t)ix[0] | ((uint32_t)ix[1] << 11) | ((uint32_t)ix[2] << 22);
}

// Lanes with pred get consecutive offsets of the workgroup-local counter
// cnt (LDS) in lane order: ballot, mbcnt prefix, one LDS atomic per wave.
__device__ __forceinline__ uint32_t block_append(bool pred, unsigned int *cnt) {
    const uint64_t mask = __ballot(pred);
    const uint32_t prefix =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    uint32_t base = 0;
    if (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        if ((int)__lane_id() == leader) base = atomicAdd(cnt, (unsigned int)__popcll(mask));
        base = __shfl(base, leader);
    }
    return base + prefix;
}

// Per-workgroup event / termination counters and profile tallies (particles
// processed, algorithmic bytes requested), flushed once per workgroup.
// Profile tallies are kept per thread in registers and summed per wave and
// workgroup only at the end of the kernel.
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
    // flush: barrier, then counters and the per-thread profile tallies
    __device__ void flush(const RunArgs &R, int cls, unsigned long long t_items, unsigned long long t_bytes) {
        if (R.prof) {
            for (int o = 32; o > 0; o >>= 1) {
                t_items += __shfl_xor(t_items, o);
                t_bytes += __shfl_xor(t_bytes, o);
            }
            if (__lane_id() == 0) {
                atomicAdd(&items, t_items);
                atomicAdd(&bytes, t_bytes);
            }
        }
        __syncthreads();
        if (threadIdx.x < kCounters && c[threadIdx.x])
            atomicAdd(R.counters + threadIdx.x, (unsigned long long)c[threadIdx.x]);
        if (R.prof && threadIdx.x == 0) {
            atomicAdd(R.prof + 2 * cls, items);
            atomicAdd(R.prof + 2 * cls + 1, bytes);
        }
    }
};

// Bytes of the particle state as the kernels move it (finite axes only).
template <int FM>
__device__ __forceinline__ unsigned int nfinite(const DevProblem &P) {
    return (unsigned int)__popc((unsigned int)(FM ? FM : P.finite_mask));
}
// load_state: x, u per finite axis, t, tau, (w), cell, g/k
template <int FM, bool WW>
__device__ __forceinline__ unsigned int load_bytes(const DevProblem &P) {
    return 16u * nfinite<FM>(P) + 24u + (WW ? 8u : 0u);
}
// store_state: the whole particle (load_state fields + RNG state + history)
template <int FM, bool WW>
__device__ __forceinline__ unsigned int state_bytes(const DevProblem &P) {
    return load_bytes<FM, WW>(P) + 12u;
}

__device__ __forceinline__ void tprof(unsigned long long &items, unsigned long long &bytes, unsigned int n_items,
                                      unsigned int n_bytes) {
    items += n_items;
    bytes += n_bytes;
}

__device__ __forceinline__ void hist_event(const RunArgs &R, uint64_t i, int e) {
    if (R.dbg_counts) atomicAdd(R.dbg_counts + i * 5 + e, 1u);
}
__device__ __forceinline__ void hist_term(const RunArgs &R, uint64_t i, int code) {
    if (R.dbg_counts) atomicOr(R.dbg_counts + i * 5 + 4, 1u << code);
}

template <int FM, bool WW>
__device__ __forceinline__ void load_state(const DevProblem &P, const Bank &B, uint32_t slot, Particle &p,
                                           uint32_t &gk) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            p.x[a] = B.x[a][slot];
            p.u[a] = B.u[a][slot];
        } else if (WW) {
            p.x[a] = 0.0;   // copied to split progeny; never used in flight
            p.u[a] = 0.0;
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

// Weight-window check point of the event kernels: roulette (returns false)
// or split, with the progeny written whole to the split bank; they are
// tracked after the chunk's census steps, generation by generation.
template <bool WW>
__device__ __forceinline__ bool ww_point(const DevProblem &P, const RunArgs &R, const SplitBank &SB, Particle &p,
                                         int cell, int b, uint64_t i, Counters &cnt) {
    if (!WW) return true;
    int nc = 0;
    if (!ww_check(P, p, cell, nc)) {
        cnt.add(3 + kRoulette);
        hist_term(R, i, kRoulette);
        return false;
    }
    if (nc > 0) {
        if (!spawn_children(SB, p, nc, b, i)) *R.overflow = 1;
        cnt.add(8, (unsigned int)nc);
        if (R.dbg_counts) atomicAdd(R.dbg_counts + i * 5 + 3, (unsigned int)nc);
    }
    return true;
}

__device__ __forceinline__ uint32_t with_gk(uint32_t gk, const Particle &p) {
    return (uint32_t)p.g | (gk & (1023u << 5)) | ((uint32_t)p.k << 15);
}

// Track-length score of one flight: into the workgroup's LDS slice when the
// particle's batch is one of the segment's two, else straight to HBM.
struct StepScore {
    double *lt;     // LDS [2][gn]
    int gn;         // G * nts of the slice (0 = no LDS slice)
    int b0;         // first batch of the segment
    bool scored;
    __device__ __forceinline__ void add(const DevProblem &P, const RunArgs &R, int b, int g, int k, int tb,
                                        double v) {
        const int rel = b - b0;
        if (gn && rel >= 0 && rel < 2) {
            atomicAdd(&lt[rel * gn + g * P.nts + tb], v);
            scored = true;
        } else {
            atomic_add_f64(R.S + (int64_t)b * P.ntally + ((int64_t)k * P.G + g) * P.nts + tb, v);
        }
    }
};

__device__ __forceinline__ void init_slice(StepScore &sc, double *lt, int gn, int b0) {
    sc.lt = lt;
    sc.gn = gn;
    sc.b0 = b0;
    sc.scored = false;
    for (int j = threadIdx.x; j < 2 * gn; j += kBlock) lt[j] = 0.0;
}

// End of a scoring kernel: add the workgroup's slice into the tally (one
// atomic per nonzero bin).  Contains the barrier the counter flush needs.
__device__ __forceinline__ void flush_slice(const DevProblem &P, const RunArgs &R, const StepScore &sc, int step) {
    const int any = __syncthreads_or(sc.scored ? 1 : 0);
    if (!sc.gn || !any) return;
    for (int j = threadIdx.x; j < 2 * sc.gn; j += kBlock) {
        const double v = sc.lt[j];
        const int b = sc.b0 + j / sc.gn;
        if (v != 0.0 && b < R.B)
            atomic_add_f64(R.S + (int64_t)b * P.ntally + (int64_t)step * sc.gn + (j % sc.gn), v);
    }
}

// ---------------------------------------------------------------------------
// source: workgroup b samples histories [b L, (b + 1) L) of the chunk
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_SOURCE>
__global__ void __launch_bounds__(kBlock) k_source(DevProblem P, RunArgs R, Bank bank, Ctl C, uint64_t count) {
    __shared__ Counters cnt;
    __shared__ unsigned int cN;
    cnt.init();
    unsigned long long p_items = 0, p_bytes = 0;
    if (threadIdx.x == 0) cN = 0u;
    const uint64_t first = *C.first;
    const unsigned int seg = blockIdx.x;
    const uint64_t lo = (uint64_t)seg * C.L;
    const uint64_t hi = (lo + C.L < count) ? lo + C.L : count;
    if (threadIdx.x == 0)
        C.seg_b0[seg] = (lo < count) ? (int)(((first + lo + 1) * (uint64_t)R.B - 1) / R.N) : 0;
    __syncthreads();
    for (uint64_t base = lo; base < hi; base += kBlock) {
        const uint64_t r = base + threadIdx.x;
        const bool valid = r < hi;
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
                hist_term(R, i, kTime);
            }
        }
        const uint32_t off = block_append(valid && alive, &cN);
        if (valid && alive) store_state<FM, WW>(P, bank, seg * C.L + off, p, pack_gk(p.g, b, p.k), (uint32_t)r);
        if (R.prof) tprof(p_items, p_bytes, valid ? 1u : 0u, (valid && alive) ? state_bytes<FM, WW>(P) : 0u);
    }
    __syncthreads();
    if (threadIdx.x == 0) C.n_bank[seg] = cN;   // bank 0
    cnt.flush(R, CLS, p_items, p_bytes);
}

// ---------------------------------------------------------------------------
// advance: one flight per particle, score, file into a queue
// ---------------------------------------------------------------------------
enum Outcome : int { kNone = 0, kToNext = 1, kToSurface = 2, kToCollision = 3 };

template <int FM, bool WW, bool DENSE, int CLS = DENSE ? MCDC_PROF_ADVANCE : MCDC_PROF_ADVANCE_Q>
__global__ void __launch_bounds__(kBlock) k_advance(DevProblem P, RunArgs R, Bank cur, Bank next, Ctl C, int par,
                                                    const uint32_t *__restrict__ aq, int it, uint32_t *sq,
                                                    uint32_t *cq, int gn, SplitBank SB) {
    __shared__ Counters cnt;
    __shared__ unsigned int cN, cS, cC;
    extern __shared__ double lt[];
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const unsigned int n = DENSE ? C.n_bank[par * C.G + seg] : C.n_a[(it - 1) * C.G + seg];
    const int step = *C.step;
    const uint64_t first = *C.first;
    cnt.init();
    unsigned long long p_items = 0, p_bytes = 0;
    if (threadIdx.x == 0) {
        cN = DENSE ? 0u : C.n_bank[(par ^ 1) * C.G + seg];
        cS = 0u;
        cC = 0u;
    }
    StepScore sc;
    init_slice(sc, lt, gn, C.seg_b0[seg]);
    __syncthreads();
    const bool per_hist = WW || (R.dbg_counts != nullptr) || (R.dbg_scores != nullptr) || P.qoi_on;
    for (unsigned int j0 = 0; j0 < n; j0 += kBlock) {
        const unsigned int idx = j0 + threadIdx.x;
        const bool valid = idx < n;
        const uint32_t slot = valid ? (DENSE ? seg0 + idx : aq[seg0 + idx]) : 0u;
        int outcome = kNone;
        int mask = 0;
        bool have_s = false;
        Particle p;
        uint32_t gk = 0, hid = 0;
        if (valid) {
            load_state<FM, WW>(P, cur, slot, p, gk);
            if (per_hist) hid = cur.hid[slot];
            if (p.k > step) {
                outcome = kToNext;   // born in a later time bin: wait
            } else {
                const int cell = cell_index(P, p.ix);
                const Flight f = next_event<FM>(P, p, cell);
                const uint64_t i = first + hid;
                if (f.d == kInf) {
                    cnt.add(3 + kLost);
                    if (per_hist) hist_term(R, i, kLost);
                } else {
                    const double v = p.w * f.d;
                    const int tb = P.cell_tal[cell];
                    const int b = (gk >> 5) & 1023u;
                    if (tb >= 0) {
                        sc.add(P, R, b, p.g, p.k, tb, v);
                        if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2, v);
                    }
                    if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) {
                        atomic_add_f64(R.qoi_hist + hid, v);
                        if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2 + 1, v);
                    }
                    move<FM>(P, p, f);
                    if (f.ev == kCensus) {
                        cnt.add(0);
                        if (per_hist) hist_event(R, i, 0);
                        p.k += 1;
                        if (p.k == P.K) {
                            cnt.add(3 + kTime);
                            if (per_hist) hist_term(R, i, kTime);
                        } else {
                            outcome = kToNext;
                            if (WW) {
                                p.s = cur.s[slot];
                                have_s = true;
                                if (!ww_point<WW>(P, R, SB, p, cell, b, i, cnt)) outcome = kNone;
                            }
                        }
                    } else if (f.ev == kSurface) {
                        cnt.add(1);
                        if (per_hist) hist_event(R, i, 1);
                        mask = crossing_mask<FM>(P, f);
                        outcome = kToSurface;
                    } else {
                        cnt.add(2);
                        if (per_hist) hist_event(R, i, 2);
                        outcome = kToCollision;
                    }
                }
            }
        }
        const uint32_t ns = block_append(outcome == kToNext, &cN);
        const uint32_t ss = block_append(outcome == kToSurface, &cS);
        const uint32_t cs = block_append(outcome == kToCollision, &cC);
        if (outcome == kToNext) {
            if (!have_s) p.s = cur.s[slot];
            if (!per_hist) hid = cur.hid[slot];
            store_state<FM, WW>(P, next, seg0 + ns, p, with_gk(gk, p), hid);
        } else if (outcome == kToSurface || outcome == kToCollision) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (finite_axis<FM>(P, a)) cur.x[a][slot] = p.x[a];
            cur.t[slot] = p.t;
            cur.tau[slot] = p.tau;
            if (outcome == kToSurface)
                sq[seg0 + ss] = slot | ((uint32_t)mask << 29);
            else
                cq[seg0 + cs] = slot;
        }
        if (R.prof && valid) {
            unsigned int by = load_bytes<FM, WW>(P) + (DENSE ? 0u : 4u) + (per_hist ? 4u : 0u);
            if (outcome == kToNext)
                by += 8u + (per_hist ? 0u : 4u) + state_bytes<FM, WW>(P);
            else if (outcome != kNone)
                by += 8u * nfinite<FM>(P) + 16u + 4u;
            tprof(p_items, p_bytes, 1u, by);
        }
    }
    flush_slice(P, R, sc, step);
    if (threadIdx.x == 0) {
        C.n_bank[(par ^ 1) * C.G + seg] = cN;
        C.n_s[it * C.G + seg] = cS;
        C.n_c[it * C.G + seg] = cC;
    }
    cnt.flush(R, CLS, p_items, p_bytes);
}

// ---------------------------------------------------------------------------
// surface crossing and boundary conditions
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_SURFACE>
__global__ void __launch_bounds__(kBlock) k_surface(DevProblem P, RunArgs R, Bank cur, Ctl C,
                                                    const uint32_t *__restrict__ sq, uint32_t *aq_out, int it,
                                                    SplitBank SB) {
    __shared__ Counters cnt;
    __shared__ unsigned int cA;
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const unsigned int n = C.n_s[it * C.G + seg];
    const uint64_t first = *C.first;
    cnt.init();
    unsigned long long p_items = 0, p_bytes = 0;
    if (threadIdx.x == 0) cA = 0u;
    __syncthreads();
    for (unsigned int j0 = 0; j0 < n; j0 += kBlock) {
        const unsigned int idx = j0 + threadIdx.x;
        const bool valid = idx < n;
        bool alive = false;
        uint32_t slot = 0;
        int mask = 0;
        Particle p;
        if (valid) {
            const uint32_t e = sq[seg0 + idx];
            slot = e & 0x1FFFFFFFu;
            mask = (int)(e >> 29);
            uint32_t gk;
            load_state<FM, WW>(P, cur, slot, p, gk);
            const int old_ww = WW ? P.cell_ww[cell_index(P, p.ix)] : 0;
            const int face = cross<FM>(P, p, mask);
            const int b = (gk >> 5) & 1023u;
            if (face >= 0) {
                atomic_add_f64(R.L + (((int64_t)b * P.K + p.k) * P.G + p.g) * 6 + face, p.w);
                cnt.add(3 + kLeak);
                if (R.dbg_counts) hist_term(R, first + cur.hid[slot], kLeak);
            } else {
                alive = true;
                if (WW) {
                    const int cell = cell_index(P, p.ix);
                    if (P.cell_ww[cell] != old_ww) {
                        p.s = cur.s[slot];
                        alive = ww_point<WW>(P, R, SB, p, cell, b, first + cur.hid[slot], cnt);
                        cur.s[slot] = p.s;
                        cur.w[slot] = p.w;
                    }
                }
            }
            if (alive) {
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
        const uint32_t as = block_append(alive, &cA);
        if (alive) aq_out[seg0 + as] = slot;
        if (R.prof && valid)
            tprof(p_items, p_bytes, 1u, 4u + load_bytes<FM, WW>(P) + (alive ? 16u * (unsigned int)__popc(mask) + 8u : 0u));
    }
    __syncthreads();
    if (threadIdx.x == 0) C.n_a[it * C.G + seg] = cA;
    cnt.flush(R, CLS, p_items, p_bytes);
}

// ---------------------------------------------------------------------------
// analog collision
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_COLLISION>
__global__ void __launch_bounds__(kBlock) k_collision(DevProblem P, RunArgs R, Bank cur, Ctl C,
                                                      const uint32_t *__restrict__ cq, uint32_t *aq_out, int it,
                                                      SplitBank SB) {
    __shared__ Counters cnt;
    __shared__ unsigned int cA;
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const unsigned int n = C.n_c[it * C.G + seg];
    const uint64_t first = *C.first;
    cnt.init();
    unsigned long long p_items = 0, p_bytes = 0;
    if (threadIdx.x == 0) cA = C.n_a[it * C.G + seg];   // after the surface kernel's appends
    __syncthreads();
    for (unsigned int j0 = 0; j0 < n; j0 += kBlock) {
        const unsigned int idx = j0 + threadIdx.x;
        const bool valid = idx < n;
        bool alive = false;
        uint32_t slot = 0;
        Particle p;
        if (valid) {
            slot = cq[seg0 + idx];
            const uint32_t gk = cur.gk[slot];
            if (WW) {
                uint32_t gk_unused;
                load_state<FM, WW>(P, cur, slot, p, gk_unused);   // whole state for split progeny
            }
            p.g = gk & 31u;
            p.s = cur.s[slot];
            const uint32_t c = cur.ixyz[slot];
            const int ix[3] = {(int)(c & 2047u), (int)((c >> 11) & 2047u), (int)(c >> 22)};
            const int cell = cell_index(P, ix);
            const int m = P.cell_mat[cell];
            if (collide<FM>(P, p, m)) {
                alive = !WW || ww_point<WW>(P, R, SB, p, cell, (gk >> 5) & 1023u, first + cur.hid[slot], cnt);
                if (alive) {
                    cur.gk[slot] = (gk & ~31u) | (uint32_t)p.g;
                    cur.tau[slot] = p.tau;
                    if (WW) cur.w[slot] = p.w;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        if (finite_axis<FM>(P, a)) cur.u[a][slot] = p.u[a];
                }
            } else {
                cnt.add(3 + kAbsorb);
                if (R.dbg_counts) hist_term(R, first + cur.hid[slot], kAbsorb);
            }
            cur.s[slot] = p.s;
        }
        const uint32_t as = block_append(alive, &cA);
        if (alive) aq_out[seg0 + as] = slot;
        if (R.prof && valid) tprof(p_items, p_bytes, 1u, 20u + 8u + (alive ? 16u + 8u * nfinite<FM>(P) + 4u : 0u));
    }
    __syncthreads();
    if (threadIdx.x == 0) C.n_a[it * C.G + seg] = cA;
    cnt.flush(R, CLS, p_items, p_bytes);
}

// ---------------------------------------------------------------------------
// finish: the particles still in flight, in registers, to census or death
// ---------------------------------------------------------------------------
template <int FM, bool WW, int CLS = MCDC_PROF_FINISH>
__global__ void __launch_bounds__(kBlock) k_finish(DevProblem P, RunArgs R, Bank cur, Bank next, Ctl C, int par,
                                                   const uint32_t *__restrict__ aq, int it, int gn, SplitBank SB) {
    __shared__ Counters cnt;
    __shared__ unsigned int cN;
    extern __shared__ double lt[];
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const unsigned int n = C.n_a[(it - 1) * C.G + seg];
    const int step = *C.step;
    const uint64_t first = *C.first;
    cnt.init();
    unsigned long long p_items = 0, p_bytes = 0;
    if (threadIdx.x == 0) cN = C.n_bank[(par ^ 1) * C.G + seg];
    StepScore sc;
    init_slice(sc, lt, gn, C.seg_b0[seg]);
    __syncthreads();
    const bool per_hist = (R.dbg_counts != nullptr) || (R.dbg_scores != nullptr) || P.qoi_on;
    for (unsigned int j0 = 0; j0 < n; j0 += kBlock) {
        const unsigned int idx = j0 + threadIdx.x;
        const bool valid = idx < n;
        bool to_next = false;
        Particle p;
        uint32_t gk = 0, hid = 0;
        if (valid) {
            const uint32_t slot = aq[seg0 + idx];
            load_state<FM, WW>(P, cur, slot, p, gk);
            p.s = cur.s[slot];
            hid = cur.hid[slot];
            const uint64_t i = first + hid;
            const int b = (gk >> 5) & 1023u;
            int cell = cell_index(P, p.ix);
            int since = 0;
            for (;;) {
                if (since >= kMaxEventsPerStep) {
                    cnt.add(3 + kLost);
                    if (per_hist) hist_term(R, i, kLost);
                    break;
                }
                ++since;
                const Flight f = next_event<FM>(P, p, cell);
                if (f.d == kInf) {
                    cnt.add(3 + kLost);
                    if (per_hist) hist_term(R, i, kLost);
                    break;
                }
                const double v = p.w * f.d;
                const int tb = P.cell_tal[cell];
                if (tb >= 0) {
                    sc.add(P, R, b, p.g, p.k, tb, v);
                    if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2, v);
                }
                if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) {
                    atomic_add_f64(R.qoi_hist + hid, v);
                    if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2 + 1, v);
                }
                move<FM>(P, p, f);
                if (f.ev == kCensus) {
                    cnt.add(0);
                    if (per_hist) hist_event(R, i, 0);
                    p.k += 1;
                    if (p.k == P.K) {
                        cnt.add(3 + kTime);
                        if (per_hist) hist_term(R, i, kTime);
                    } else {
                        to_next = ww_point<WW>(P, R, SB, p, cell, b, i, cnt);
                    }
                    break;
                } else if (f.ev == kSurface) {
                    cnt.add(1);
                    if (per_hist) hist_event(R, i, 1);
                    const int old_ww = WW ? P.cell_ww[cell] : 0;
                    const int face = cross<FM>(P, p, crossing_mask<FM>(P, f));
                    if (face >= 0) {
                        atomic_add_f64(R.L + (((int64_t)b * P.K + p.k) * P.G + p.g) * 6 + face, p.w);
                        cnt.add(3 + kLeak);
                        if (per_hist) hist_term(R, i, kLeak);
                        break;
                    }
                    cell = cell_index(P, p.ix);
                    if (WW && P.cell_ww[cell] != old_ww && !ww_point<WW>(P, R, SB, p, cell, b, i, cnt)) break;
                } else {
                    cnt.add(2);
                    if (per_hist) hist_event(R, i, 2);
                    if (!collide<FM>(P, p, f.m)) {
                        cnt.add(3 + kAbsorb);
                        if (per_hist) hist_term(R, i, kAbsorb);
                        break;
                    }
                    if (WW && !ww_point<WW>(P, R, SB, p, cell, b, i, cnt)) break;
                }
            }
        }
        const uint32_t ns = block_append(to_next, &cN);
        if (to_next) store_state<FM, WW>(P, next, seg0 + ns, p, with_gk(gk, p), hid);
        if (R.prof && valid)
            tprof(p_items, p_bytes, 1u, 4u + load_bytes<FM, WW>(P) + 12u + (to_next ? state_bytes<FM, WW>(P) : 0u));
    }
    flush_slice(P, R, sc, step);
    if (threadIdx.x == 0) C.n_bank[(par ^ 1) * C.G + seg] = cN;
    cnt.flush(R, CLS, p_items, p_bytes);
}

// ---------------------------------------------------------------------------
// control
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(Ctl C, uint64_t first) {
    *C.step = 0;
    *C.first = first;
}
__global__ void k_step_end(Ctl C) { *C.step += 1; }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Layout {
    Bank bank[2];
    uint32_t *sq, *cq, *aq[2];
    Ctl ctl;
};

size_t pad256(size_t b) { return (b + 255) & ~size_t(255); }

size_t bank_bytes(uint64_t slots) { return 10 * pad256(slots * 8) + 3 * pad256(slots * 4); }

size_t queue_bytes(uint64_t slots, unsigned int G) {
    return 4 * pad256(slots * 4) + pad256(2 * G * 4) + 3 * pad256(kMaxIters * G * 4) + pad256(G * 4) + 2 * 256;
}

Layout carve(void *bank_mem, void *queue_mem, uint64_t slots, unsigned int G, unsigned int Lseg) {
    Layout Lo{};
    char *p = (char *)bank_mem;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += pad256(bytes);
        return r;
    };
    for (int k = 0; k < 2; ++k) {
        Bank &B = Lo.bank[k];
        for (int a = 0; a < 3; ++a) B.x[a] = (double *)take(slots * 8);
        for (int a = 0; a < 3; ++a) B.u[a] = (double *)take(slots * 8);
        B.t = (double *)take(slots * 8);
        B.tau = (double *)take(slots * 8);
        B.w = (double *)take(slots * 8);
        B.s = (uint64_t *)take(slots * 8);
        B.ixyz = (uint32_t *)take(slots * 4);
        B.gk = (uint32_t *)take(slots * 4);
        B.hid = (uint32_t *)take(slots * 4);
    }
    p = (char *)queue_mem;
    Lo.sq = (uint32_t *)take(slots * 4);
    Lo.cq = (uint32_t *)take(slots * 4);
    Lo.aq[0] = (uint32_t *)take(slots * 4);
    Lo.aq[1] = (uint32_t *)take(slots * 4);
    Ctl &C = Lo.ctl;
    C.n_bank = (unsigned int *)take(2 * G * 4);
    C.n_s = (unsigned int *)take(kMaxIters * G * 4);
    C.n_c = (unsigned int *)take(kMaxIters * G * 4);
    C.n_a = (unsigned int *)take(kMaxIters * G * 4);
    C.seg_b0 = (int *)take(G * 4);
    C.step = (int *)take(64);
    C.first = (uint64_t *)take(64);
    C.G = G;
    C.L = Lseg;
    return Lo;
}

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
    if (C > (1ULL << 28)) C = 1ULL << 28;
    int iters = opt.event_iters > 0 ? opt.event_iters : 1;
    if (iters > kMaxIters - 1) iters = kMaxIters - 1;
    // per-step tally slice [2 batches][G][nts] in LDS when it fits
    const int64_t gn64 = (int64_t)P.G * P.nts;
    const int gn = (2 * gn64 <= kLdsTallyMax) ? (int)gn64 : 0;
    const size_t shmem = (size_t)2 * gn * sizeof(double);

    // segments: one per workgroup.  Auto: the advance kernel's resident
    // capacity, so its pass over the census bank is one round of workgroups
    // (a second, partly filled round would cost nearly a full one).
    unsigned int G;
    if (opt.segments > 0) {
        G = (unsigned int)opt.segments;
    } else {
        int per_cu = 0, n_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_advance<FM, WW, true>), kBlock, shmem);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, pb->device);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        G = (unsigned int)(per_cu > 0 ? per_cu : 1) * (unsigned int)(n_cu > 0 ? n_cu : 1);
    }
    const uint64_t g_need = (C + kBlock - 1) / kBlock;
    if (G > g_need) G = (unsigned int)g_need;
    if (G < 1) G = 1;
    const unsigned int Lseg = (unsigned int)((C + G - 1) / G);
    const uint64_t slots = (uint64_t)G * Lseg;
    int rc;
    if ((rc = ensure(pb->bank, bank_bytes(slots) * 2 + 64 * 256))) return rc;
    if ((rc = ensure(pb->queues, queue_bytes(slots, G)))) return rc;
    if (P.qoi_on && (rc = ensure(pb->qoi_hist, C * sizeof(double)))) return rc;
    Layout L = carve(pb->bank.p, pb->queues.p, slots, G, Lseg);
    RunArgs R = R0;
    R.qoi_hist = (double *)pb->qoi_hist.p;
    // weight windows: split progeny of a chunk go to the split bank and are
    // tracked after its census steps
    SplitBank SB[2]{};
    if (WW && (rc = split_prepare(pb, C, SB))) return rc;

    // the step kernels never read the seed or the history count
    RunArgs Rs = R;
    Rs.seed = 0;
    Rs.N = 0;

    auto enqueue_step = [&](int par, hipStream_t s, Profiler &pr) {
        const Bank &cur = L.bank[par];
        const Bank &nxt = L.bank[par ^ 1];
        pr.begin(MCDC_PROF_ADVANCE);
        hipLaunchKernelGGL((k_advance<FM, WW, true>), dim3(G), dim3(kBlock), shmem, s, P, Rs, cur, nxt, L.ctl, par,
                           (const uint32_t *)nullptr, 0, L.sq, L.cq, gn, SB[0]);
        pr.end();
        pr.begin(MCDC_PROF_SURFACE);
        hipLaunchKernelGGL((k_surface<FM, WW>), dim3(G), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                           (const uint32_t *)L.sq, L.aq[0], 0, SB[0]);
        pr.end();
        pr.begin(MCDC_PROF_COLLISION);
        hipLaunchKernelGGL((k_collision<FM, WW>), dim3(G), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                           (const uint32_t *)L.cq, L.aq[0], 0, SB[0]);
        pr.end();
        for (int j = 1; j < iters; ++j) {
            pr.begin(MCDC_PROF_ADVANCE_Q);
            hipLaunchKernelGGL((k_advance<FM, WW, false>), dim3(G), dim3(kBlock), shmem, s, P, Rs, cur, nxt, L.ctl,
                               par, (const uint32_t *)L.aq[(j - 1) & 1], j, L.sq, L.cq, gn, SB[0]);
            pr.end();
            pr.begin(MCDC_PROF_SURFACE);
            hipLaunchKernelGGL((k_surface<FM, WW>), dim3(G), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                               (const uint32_t *)L.sq, L.aq[j & 1], j, SB[0]);
            pr.end();
            pr.begin(MCDC_PROF_COLLISION);
            hipLaunchKernelGGL((k_collision<FM, WW>), dim3(G), dim3(kBlock), 0, s, P, Rs, cur, L.ctl,
                               (const uint32_t *)L.cq, L.aq[j & 1], j, SB[0]);
            pr.end();
        }
        pr.begin(MCDC_PROF_FINISH);
        hipLaunchKernelGGL((k_finish<FM, WW>), dim3(G), dim3(kBlock), shmem, s, P, Rs, cur, nxt, L.ctl, par,
                           (const uint32_t *)L.aq[(iters - 1) & 1], iters, gn, SB[0]);
        pr.end();
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, s, L.ctl);
    };

    // replay captured steps unless a per-launch profile or per-history
    // debug output is requested (those launch eagerly)
    const bool use_graph =
        !(opt.flags & MCDC_FLAG_EAGER) && !opt.profile && !R.dbg_counts && !R.dbg_scores && P.K > 1;
    StepGraphs *Gr = nullptr;
    if (use_graph) {
        if (!pb->graph_cache) pb->graph_cache = new StepGraphs();
        Gr = (StepGraphs *)pb->graph_cache;
        std::vector<char> key;
        key_add(key, P);
        key_add(key, Rs);
        key_add(key, L);
        key_add(key, gn);
        key_add(key, iters);
        key_add(key, SB[0]);
        if (key != Gr->key) {
            Gr->clear();
            hipError_t e = hipSuccess;
            if (!Gr->cs) e = hipStreamCreateWithFlags(&Gr->cs, hipStreamNonBlocking);
            Profiler none;
            for (int q = 0; q < 2 && e == hipSuccess; ++q) {
                e = hipStreamBeginCapture(Gr->cs, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) break;
                enqueue_step(q, Gr->cs, none);
                e = hipStreamEndCapture(Gr->cs, &Gr->graph[q]);
                if (e == hipSuccess) e = hipGraphInstantiate(&Gr->exec[q], Gr->graph[q], nullptr, nullptr, 0);
            }
            if (e != hipSuccess) {
                Gr->clear();
                return hip_fail(e, "census step capture");
            }
            Gr->key = key;
        }
    }

    for (uint64_t c0 = 0; c0 < count; c0 += C) {
        const uint64_t n = (count - c0 < C) ? count - c0 : C;
        const uint64_t cfirst = first + c0;
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, st, L.ctl, cfirst);
        if (P.qoi_on && (rc = launch_zero(R.qoi_hist, n * sizeof(double), st))) return hip_fail((hipError_t)rc, "zero");
        if (WW) split_reset(SB, st);
        prof.begin(MCDC_PROF_SOURCE);
        hipLaunchKernelGGL((k_source<FM, WW>), dim3(G), dim3(kBlock), 0, st, P, R, L.bank[0], L.ctl, n);
        prof.end();
        for (int step = 0; step < P.K; ++step) {
            if (Gr) {
                hipError_t e = hipGraphLaunch(Gr->exec[step & 1], st);
                if (e != hipSuccess) return hip_fail(e, "census step replay");
            } else {
                enqueue_step(step & 1, st, prof);
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "event kernel launch");
        if (WW && (rc = split_generations(pb, R, SB, cfirst, st, prof))) return rc;
        if (P.qoi_on && (rc = launch_qoi_reduce(R.qoi_hist, n, R.qoi_sums, st)))
            return hip_fail((hipError_t)rc, "detector reduce");
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

int launch_event(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count, const mcdc_run_options &opt,
                 hipStream_t st, Profiler &prof) {
    const DevProblem &P = p->d;
    if (p->h.B > 1023 || P.K > 131071) {
        set_error("event form supports at most 1023 batches and 131071 time bins");
        return MCDC_E_UNSUPPORTED;
    }
    if (P.ww_center != nullptr) {
        if (P.finite_mask == 1) return run_event<1, true>(p, R, first, count, opt, st, prof);
        if (P.finite_mask == 7) return run_event<7, true>(p, R, first, count, opt, st, prof);
        return run_event<0, true>(p, R, first, count, opt, st, prof);
    }
    if (P.finite_mask == 1) return run_event<1, false>(p, R, first, count, opt, st, prof);
    if (P.finite_mask == 7) return run_event<7, false>(p, R, first, count, opt, st, prof);
    return run_event<0, false>(p, R, first, count, opt, st, prof);
}

}  // namespace mcdc
