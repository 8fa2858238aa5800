// Event-based tracking (the second algorithm mode the paper names, Section 2;
// it gives no design).  Particles live in structure-of-arrays banks in HBM,
// in tiles of one wavefront, and time advances census step by census step
// (the census grid is the tally time grid, Section 3): the particles alive
// at the start of a step are one bank, and the census crossers of the step
// are filed into the next bank.
//
// Segment-private pipelines.  Every bank is cut into G segments of L slots,
// one per workgroup: workgroup b of every kernel works only on segment b,
// and a particle never leaves the segment it was born in (except under
// population control, whose copies are spread over all segments).  Queue
// appends therefore need no device-wide atomics (ballots, mbcnt prefix
// counts, one LDS atomic per wave; no contention across the 8 XCDs), and
// each segment holds a contiguous range of histories, so its particles
// belong to at most two tally batches (scores of any other batch go to
// HBM directly).
//
// One kernel per census step (default): the events kernel takes the step's
// bank as its work list; each lane follows its particle through its
// flights and events (surface crossing, collision) in registers until it
// reaches the census edge or dies, files census crossers whole into the
// next bank, and takes the next particle of the list at once, so a wave is
// never held back by its longest-lived particle.  The step is captured
// once per bank parity as a graph and replayed K times.  The earlier
// two-kernel form (kept behind a run flag) first moved every particle one
// flight (advance), filing it whole into census, surface or collision
// queues (the surface and collision queues share an event bank, from the
// front and from the back of each segment), and then applied the queued
// events; the single kernel saves the event bank's write and re-read.
//
// Tally: every particle scored in step k lies in time bin k, so a
// workgroup touches only the slice [2 batches][G][nts] of the step; when that
// fits in LDS it is accumulated there and flushed with one global atomic
// per nonzero bin at the end of the kernel.
//
// Tables: the read-only tables every flight consults (union planes, time
// edges, cross sections, speeds, per-cell material and tally bin) are
// copied into LDS at the start of each step kernel when they fit, so the
// dependent table lookups of a flight cost LDS latency, not cache latency.
#include <type_traits>
#include <vector>


#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

constexpr int kBlock = 512;
constexpr int kLdsTablesMax = 32 * 1024;    // bytes of staged tables
constexpr int kWave = 64;
// Wave schedule of the events kernel: idle lanes refill once at least
// kRefillMin lanes of the wave are idle; queued collisions run once they
// make up kCollEighths / 8 of the busy lanes.
// (Measured on the pulsed slab, 1e7 histories: collisions run at once,
// 7.9 ms; queued to 3/8 of the busy lanes, 6.7 ms; to 6/8, 7.7 ms.
// Thresholds on refills and queued surface crossings measured no gain.)
constexpr int kRefillMin = 1;
constexpr int kCollEighths = 3;
constexpr uint32_t kHidMask = 0x0FFFFFFFu;  // history index within a chunk (< 2^28)

// A bank of particle states in tiles of 64 slots (one wavefront): inside a
// tile every field is one contiguous run of 64 values, so a wave's access
// to a field is one contiguous run and its whole state one contiguous
// block of HBM (one DRAM stream per wave instead of one per field array).
// Fields: x, u per stored axis, t, tau, (w), RNG state (8 B each), then
// the packed cell ix | iy << 11 | iz << 22, g | batch << 5 | k << 15 |
// inside pin << 31 and
// the history index within the chunk | crossing axes << 29 (surface queue)
// (4 B each).
struct Bank {
    char *base;                // tile 0
    uint32_t tile;             // bytes per tile: 64 * bytes per particle
    uint32_t ox[3], ou[3];     // byte offset of each field's run within a tile
    uint32_t ot, otau, ow, os, oc, ogk, ohid;
};

// Field access: byte offset of slot's value in its tile's run of the field.
__device__ __forceinline__ uint64_t tile_off8(const Bank &B, uint32_t slot) {
    return (uint64_t)(slot >> 6) * B.tile + (slot & 63u) * 8u;
}
__device__ __forceinline__ uint64_t tile_off4(const Bank &B, uint32_t slot) {
    return (uint64_t)(slot >> 6) * B.tile + (slot & 63u) * 4u;
}
template <class T>
__device__ __forceinline__ T &fld(const Bank &B, uint32_t field, uint64_t off) {
    return *reinterpret_cast<T *>(B.base + field + off);
}

// Per-segment fill counts of the banks and queues, plus the step index.
// Only workgroup b reads or writes the entries of segment b.
struct Ctl {
    unsigned int *n_bank;   // [2][G] particles in each segment of bank 0 / 1
    unsigned int *n_s;      // [G] surface particles at the front of the event bank segment
    unsigned int *n_c;      // [G] collision particles at its back
    int *seg_b0;            // [G] batch of the segment's first history
    int *step;              // current census step
    uint64_t *first;        // global index of the chunk's first history
    uint64_t *seed;         // the run's seed (63 bits; the combing offsets' streams)
    unsigned long long *pc_w;  // [G][2] population control: fixed-point weight sum per segment
    unsigned long long *pc_cnt;  // [G] population control: copies made from each segment
    unsigned int G, L;      // segments (= workgroups), slots per segment
    unsigned int Lh;        // histories per segment (L, or fewer with population control)
    unsigned int ordered;   // 1: the banks keep the run's list order (births in history
                            // order, a census step keeps every particle in its slot)
};

// gk word of a bank slot whose particle ended in the census step (banks in
// list order keep their slots; a control skips these)
constexpr uint32_t kTombGk = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t pack_gk(int g, int b, int k, int inpin) {
    return (uint32_t)g | ((uint32_t)b << 5) | ((uint32_t)k << 15) | ((uint32_t)inpin << 31);
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
        base = __builtin_amdgcn_readlane(base, leader);
    }
    return base + prefix;
}

// 128-bit fixed-point weight sums with 64 fractional bits: a weight w is
// truncated to a multiple of 2^-64 and added to the accumulator (hi, lo).
// floor(w) is exact in binary64 and so is the fraction w - floor(w); the
// fraction times 2^64 (a power-of-two scaling, below 2^64) truncated to an
// integer is the low word.  False if w is 2^32 or more, negative or not a
// number.
__device__ __forceinline__ bool fixed_add(unsigned long long &hi, unsigned long long &lo, double w) {
    if (!(w >= 0.0) || !(w < 4294967296.0)) return false;
    const double whole = floor(w);
    const double frac = w - whole;
    const unsigned long long fbits = __double2ull_rz(frac * 18446744073709551616.0);
    unsigned __int128 acc = ((unsigned __int128)hi << 64) | lo;
    acc += ((unsigned __int128)(unsigned long long)whole << 64) + fbits;
    hi = (unsigned long long)(acc >> 64);
    lo = (unsigned long long)acc;
    return true;
}
__device__ __forceinline__ void fixed_merge(unsigned long long &hi, unsigned long long &lo, unsigned long long h2,
                                            unsigned long long l2) {
    unsigned __int128 acc = ((unsigned __int128)hi << 64) | lo;
    acc += ((unsigned __int128)h2 << 64) | l2;
    hi = (unsigned long long)(acc >> 64);
    lo = (unsigned long long)acc;
}

// Exclusive prefix of v over the workgroup in thread order, and the
// workgroup total (every thread calls it; wtot: LDS [BS / 64]).
template <int BS>
__device__ __forceinline__ unsigned long long block_exclusive(unsigned long long v, unsigned long long *wtot,
                                                              unsigned long long &total) {
    const int lane = (int)__lane_id(), w = (int)(threadIdx.x >> 6);
    unsigned long long x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long t = __shfl_up(x, d);
        if (lane >= d) x += t;
    }
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    unsigned long long before = 0ull, tot = 0ull;
    for (int j = 0; j < BS / 64; ++j) {
        const unsigned long long t = wtot[j];
        if (j < w) before += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

// The same for 128-bit fixed-point sums (hi, lo); wtot: LDS [BS / 64][2].
template <int BS>
__device__ __forceinline__ void block_exclusive_u128(unsigned long long hi, unsigned long long lo,
                                                     unsigned long long (*wtot)[2], unsigned long long &ehi,
                                                     unsigned long long &elo, unsigned long long &thi,
                                                     unsigned long long &tlo) {
    const int lane = (int)__lane_id(), w = (int)(threadIdx.x >> 6);
    unsigned long long xh = hi, xl = lo;
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long th = __shfl_up(xh, d), tl = __shfl_up(xl, d);
        if (lane >= d) fixed_merge(xh, xl, th, tl);
    }
    if (lane == 63) {
        wtot[w][0] = xh;
        wtot[w][1] = xl;
    }
    __syncthreads();
    unsigned long long bh = 0ull, bl = 0ull, sh = 0ull, sl = 0ull;
    for (int j = 0; j < BS / 64; ++j) {
        if (j < w) fixed_merge(bh, bl, wtot[j][0], wtot[j][1]);
        fixed_merge(sh, sl, wtot[j][0], wtot[j][1]);
    }
    __syncthreads();
    // exclusive = before + inclusive - own (exact modulo 2^128)
    unsigned __int128 e = (((unsigned __int128)bh << 64) | bl) + (((unsigned __int128)xh << 64) | xl) -
                          (((unsigned __int128)hi << 64) | lo);
    ehi = (unsigned long long)(e >> 64);
    elo = (unsigned long long)e;
    thi = sh;
    tlo = sl;
}

// Lanes with pred get consecutive offsets of the workgroup-local counter
// cnt (LDS) in thread order (every thread calls it; wtot as above).
template <int BS>
__device__ __forceinline__ uint32_t block_append_ordered(bool pred, unsigned int *cnt, unsigned long long *wtot) {
    unsigned long long tot;
    const unsigned long long ex = block_exclusive<BS>(pred ? 1ull : 0ull, wtot, tot);
    const uint32_t base = *cnt;
    __syncthreads();
    if (threadIdx.x == 0) *cnt = base + (uint32_t)tot;
    return base + (uint32_t)ex;
}

// Event / termination counters and profile tallies (particles processed,
// algorithmic bytes requested), kept per thread in registers (every index
// is a compile-time constant) and reduced per wave, then per workgroup in
// LDS, only at the end of the kernel.
struct Counters {
    unsigned int c[kCounters];
    unsigned long long items, bytes;
    __device__ __forceinline__ void init(unsigned long long *red) {
#pragma unroll
        for (int j = 0; j < kCounters; ++j) c[j] = 0u;
        items = bytes = 0ull;
        if (threadIdx.x < kCounters + 2) red[threadIdx.x] = 0ull;
    }
    __device__ __forceinline__ void add(int j, unsigned int v = 1u) { c[j] += v; }
    __device__ __forceinline__ void prof(unsigned int n_items, unsigned int n_bytes) {
        items += n_items;
        bytes += n_bytes;
    }
    // flush: barrier, then one global atomic per nonzero counter per workgroup
    __device__ void flush(const RunArgs &R, int cls, unsigned long long *red) {
#pragma unroll
        for (int j = 0; j < kCounters; ++j) {
            unsigned int v = c[j];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (__lane_id() == 0 && v) atomicAdd(&red[j], (unsigned long long)v);
        }
        if (R.prof) {
            unsigned long long a = items, b = bytes;
            for (int o = 32; o > 0; o >>= 1) {
                a += __shfl_xor(a, o);
                b += __shfl_xor(b, o);
            }
            if (__lane_id() == 0) {
                atomicAdd(&red[kCounters], a);
                atomicAdd(&red[kCounters + 1], b);
            }
        }
        __syncthreads();
        if (threadIdx.x < kCounters && red[threadIdx.x]) atomicAdd(R.counters + threadIdx.x, red[threadIdx.x]);
        if (R.prof && threadIdx.x == 0) {
            atomicAdd(R.prof + 2 * cls, red[kCounters]);
            atomicAdd(R.prof + 2 * cls + 1, red[kCounters + 1]);
        }
    }
};

// Bytes of one particle's state as the kernels move it (finite axes only):
// x, u per finite axis, t, tau, (w), RNG state, cell, g/batch/k, history.
template <int FM, bool WW>
__device__ __forceinline__ unsigned int state_bytes(const DevProblem &P) {
    const unsigned int nf = (unsigned int)__popc((unsigned int)(FM ? FM : P.finite_mask));
    return 16u * nf + 36u + (WW ? 8u : 0u);
}

__device__ __forceinline__ void hist_event(const RunArgs &R, uint64_t i, int e) {
    if (R.dbg_counts) atomicAdd(R.dbg_counts + i * 5 + e, 1u);
}
__device__ __forceinline__ void hist_term(const RunArgs &R, uint64_t i, int code) {
    if (R.dbg_counts) atomicOr(R.dbg_counts + i * 5 + 4, 1u << code);
}

template <int FM, bool WW>
__device__ __forceinline__ void load_state(const DevProblem &P, const Bank &B, uint32_t slot, Particle &p,
                                           uint32_t &gk, uint32_t &hidw) {
    const uint64_t o8 = tile_off8(B, slot), o4 = tile_off4(B, slot);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            p.x[a] = fld<double>(B, B.ox[a], o8);
            p.u[a] = fld<double>(B, B.ou[a], o8);
        } else {
            p.x[a] = 0.0;   // stays 0 in flight; copied whole to split progeny
            p.u[a] = 0.0;
        }
    }
    p.t = fld<double>(B, B.ot, o8);
    p.tau = fld<double>(B, B.otau, o8);
    p.w = WW ? fld<double>(B, B.ow, o8) : 1.0;
    p.s = fld<uint64_t>(B, B.os, o8);
    const uint32_t c = fld<uint32_t>(B, B.oc, o4);
    gk = fld<uint32_t>(B, B.ogk, o4);
    hidw = fld<uint32_t>(B, B.ohid, o4);
    set_inverse<FM>(P, p);
    p.ix[0] = c & 2047u;
    p.ix[1] = (c >> 11) & 2047u;
    p.ix[2] = c >> 22;
    p.g = gk & 31u;
    // (a slab has no pins: bit 31 stays clear)
    p.k = (FM == 1) ? (int)(gk >> 15) : (int)((gk >> 15) & 0xFFFFu);
    p.inpin = (FM == 1) ? 0 : (int)(gk >> 31);
}

// The state of one particle as loaded, before any arithmetic on it: lets
// a kernel issue the loads of its next particle before working on the
// current one.
struct RawState {
    double x[3], u[3], t, tau, w;
    uint64_t s;
    uint32_t c, gk, hidw;
};

template <int FM, bool WW>
__device__ __forceinline__ void load_raw(const DevProblem &P, const Bank &B, uint32_t slot, RawState &r) {
    const uint64_t o8 = tile_off8(B, slot), o4 = tile_off4(B, slot);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            r.x[a] = fld<double>(B, B.ox[a], o8);
            r.u[a] = fld<double>(B, B.ou[a], o8);
        }
    }
    r.t = fld<double>(B, B.ot, o8);
    r.tau = fld<double>(B, B.otau, o8);
    if (WW) r.w = fld<double>(B, B.ow, o8);
    r.s = fld<uint64_t>(B, B.os, o8);
    r.c = fld<uint32_t>(B, B.oc, o4);
    r.gk = fld<uint32_t>(B, B.ogk, o4);
    r.hidw = fld<uint32_t>(B, B.ohid, o4);
}

template <int FM, bool WW>
__device__ __forceinline__ void unpack(const DevProblem &P, const RawState &r, Particle &p) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.x[a] = finite_axis<FM>(P, a) ? r.x[a] : 0.0;
        p.u[a] = finite_axis<FM>(P, a) ? r.u[a] : 0.0;
    }
    p.t = r.t;
    p.tau = r.tau;
    p.w = WW ? r.w : 1.0;
    p.s = r.s;
    set_inverse<FM>(P, p);
    p.ix[0] = r.c & 2047u;
    p.ix[1] = (r.c >> 11) & 2047u;
    p.ix[2] = r.c >> 22;
    p.g = r.gk & 31u;
    p.k = (FM == 1) ? (int)(r.gk >> 15) : (int)((r.gk >> 15) & 0xFFFFu);
    p.inpin = (FM == 1) ? 0 : (int)(r.gk >> 31);
}

template <int FM, bool WW>
__device__ __forceinline__ void store_raw(const DevProblem &P, const Bank &B, uint32_t slot, const RawState &r) {
    const uint64_t o8 = tile_off8(B, slot), o4 = tile_off4(B, slot);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            fld<double>(B, B.ox[a], o8) = r.x[a];
            fld<double>(B, B.ou[a], o8) = r.u[a];
        }
    }
    fld<double>(B, B.ot, o8) = r.t;
    fld<double>(B, B.otau, o8) = r.tau;
    if (WW) fld<double>(B, B.ow, o8) = r.w;
    fld<uint64_t>(B, B.os, o8) = r.s;
    fld<uint32_t>(B, B.oc, o4) = r.c;
    fld<uint32_t>(B, B.ogk, o4) = r.gk;
    fld<uint32_t>(B, B.ohid, o4) = r.hidw;
}

template <int FM, bool WW>
__device__ __forceinline__ void store_state(const DevProblem &P, const Bank &B, uint32_t slot,
                                            const Particle &p, uint32_t gk, uint32_t hidw) {
    const uint64_t o8 = tile_off8(B, slot), o4 = tile_off4(B, slot);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (finite_axis<FM>(P, a)) {
            fld<double>(B, B.ox[a], o8) = p.x[a];
            fld<double>(B, B.ou[a], o8) = p.u[a];
        }
    }
    fld<double>(B, B.ot, o8) = p.t;
    fld<double>(B, B.otau, o8) = p.tau;
    if (WW) fld<double>(B, B.ow, o8) = p.w;
    fld<uint64_t>(B, B.os, o8) = p.s;
    fld<uint32_t>(B, B.oc, o4) = pack_ix(p.ix);
    fld<uint32_t>(B, B.ogk, o4) = gk;
    fld<uint32_t>(B, B.ohid, o4) = hidw;
}

__device__ __forceinline__ uint32_t with_gk(uint32_t gk, const Particle &p) {
    return (uint32_t)p.g | (gk & (1023u << 5)) | ((uint32_t)p.k << 15) | ((uint32_t)p.inpin << 31);
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

// Scores of one census step: into the workgroup's LDS slice when the
// particle's batch is one of the segment's two, else straight to HBM.  The
// slice holds [2][gn] track-length bins and, with the time-crossing tally,
// [2][gn] bins of the flux at the step's closing edge behind them.
// A score bound for HBM is held back in the lane while the lane's next
// scores go to the same bin (a collision that keeps the group, say), so
// that one atomic carries their sum.
struct StepScore {
    double *lt;     // LDS [ns][parts][2][gn]
    int gn;         // G * nts of the slice (0 = no LDS slice)
    int b0;         // first batch of the segment
    int k0, ns;     // time bins k0 .. k0 + ns - 1 of the launch's census steps
    bool scored;
    double *pa;     // HBM bin of the held-back score (nullptr: none)
    double pv;      // its value
    __device__ __forceinline__ void put(const DevProblem &P, const RunArgs &R, int part, int b, int g, int k,
                                        int tb, double v) {
        const int rel = b - b0;
        const int dk = k - k0;
        if (gn && rel >= 0 && rel < 2 && dk >= 0 && dk < ns) {
            atomicAdd(&lt[((dk * (slice_mult(P) >> 1) + part) * 2 + rel) * gn + g * P.nts + tb], v);
            scored = true;
        } else {
            double *a = tally_copy(P, R, b) + part * P.ntally + ((int64_t)k * P.G + g) * P.nts + tb;
            if (a == pa) {
                pv += v;
            } else {
                if (pa) atomic_add_f64(pa, pv);
                pa = a;
                pv = v;
            }
        }
    }
    // the held-back score to HBM
    __device__ __forceinline__ void release() {
        if (pa) atomic_add_f64(pa, pv);
        pa = nullptr;
    }
    // track length w d of a flight in time bin k
    __device__ __forceinline__ void add(const DevProblem &P, const RunArgs &R, int b, int g, int k, int tb,
                                        double v) {
        put(P, R, 0, b, g, k, tb, v);
    }
    // time-crossing score w v_g of an arrival at the edge T_{k+1}
    __device__ __forceinline__ void cross(const DevProblem &P, const RunArgs &R, int b, int g, int k, int tb,
                                          double v) {
        put(P, R, 1, b, g, k, tb, v);
    }
};

template <int BS = kBlock>
__device__ __forceinline__ void init_slice(const DevProblem &P, StepScore &sc, double *lt, int gn, int b0, int k0 = 0,
                                           int ns = 1) {
    sc.lt = lt;
    sc.gn = gn;
    sc.b0 = b0;
    sc.k0 = k0;
    sc.ns = ns;
    sc.scored = false;
    sc.pa = nullptr;
    sc.pv = 0.0;
    for (int j = threadIdx.x; j < slice_mult(P) * gn * ns; j += BS) lt[j] = 0.0;
}

// End of a scoring kernel: add the workgroup's slice into the tally (one
// atomic per nonzero bin).  Contains the barrier the counter flush needs.
template <int BS = kBlock>
__device__ __forceinline__ void flush_slice(const DevProblem &P, const RunArgs &R, StepScore &sc, int step) {
    sc.release();
    const int any = __syncthreads_or(sc.scored ? 1 : 0);
    if (!sc.gn || !any) return;
    const int per_part = 2 * sc.gn, per_step = slice_mult(P) * sc.gn;
    for (int j = threadIdx.x; j < per_step * sc.ns; j += BS) {
        const double v = sc.lt[j];
        const int dk = j / per_step, r2 = j % per_step;
        const int part = r2 / per_part, r = r2 % per_part;
        const int b = sc.b0 + r / sc.gn;
        if (v != 0.0 && b < R.B && step + dk < P.K)
            atomic_add_f64(tally_copy(P, R, b) + part * P.ntally + (int64_t)(step + dk) * sc.gn + (r % sc.gn), v);
    }
}

// Time-crossing score of a particle that has just reached the edge
// T_{k+1} (before its time bin moves on).
__device__ __forceinline__ void score_crossing(const DevProblem &P, const RunArgs &R, StepScore &sc,
                                               const Particle &p, int cell, int b) {
    if (!P.tc_on) return;
    const int tb = P.cell_tal[cell];
    if (tb >= 0) sc.cross(P, R, b, p.g, p.k, tb, p.w * P.speed[p.g]);
}

// Score one flight (tally bin and detector) before the move.
__device__ __forceinline__ void score_flight(const DevProblem &P, const RunArgs &R, StepScore &sc, const Particle &p,
                                             int cell, int b, uint64_t i, uint32_t hid, double d) {
    const double v = p.w * d;
    const int tb = P.cell_tal[cell];
    if (tb >= 0) {
        sc.add(P, R, b, p.g, p.k, tb, v);
        if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2, v);
    }
    if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) {
        atomic_add_f64(R.qoi_hist + hid, v);
        if (R.dbg_scores) atomic_add_f64(R.dbg_scores + i * 2 + 1, v);
    }
}

// ---------------------------------------------------------------------------
// source: workgroup b samples histories [b L, (b + 1) L) of the chunk
// ---------------------------------------------------------------------------
// (BAT: a batched solve; segment b belongs to problem segs[b].prob and is
// born with its histories [first, first + count), items holds every
// problem's tables and run arguments.)
template <int FM, bool WW, bool BAT, int CLS = MCDC_PROF_SOURCE, int BS = kBlock>
__global__ void __launch_bounds__(BS) k_source(DevProblem P0, RunArgs R0, Bank bank, Ctl C, uint64_t count,
                                                   const BatchItem *__restrict__ items,
                                                   const SegInfo *__restrict__ segs) {
    __shared__ unsigned long long red[kCounters + 2];
    __shared__ unsigned long long wtot[BS / 64];
    Counters cnt;
    __shared__ unsigned int cN;
    const SegInfo si = BAT ? segs[blockIdx.x] : SegInfo{0, 0u, 0u, 0u};
    const DevProblem &P = BAT ? items[si.prob].P : P0;
    const RunArgs &R = BAT ? items[si.prob].R : R0;
    cnt.init(red);
    if (threadIdx.x == 0) cN = 0u;
    const uint64_t first = *C.first;
    const unsigned int seg = blockIdx.x;
    const uint64_t lo = BAT ? (uint64_t)si.first : (uint64_t)seg * C.Lh;
    const uint64_t hi = BAT ? lo + si.count : ((lo + C.Lh < count) ? lo + C.Lh : count);
    if (threadIdx.x == 0)
        C.seg_b0[seg] = (lo < hi) ? (int)(((first + lo + 1) * (uint64_t)R.B - 1) / R.N) : 0;
    __syncthreads();
    // the thread's histories are BS apart: one full skip-ahead to the
    // first, then the map for BS histories (BS a power of two)
    constexpr int lbs = (BS == 1024) ? 10 : (BS == 512 ? 9 : (BS == 256 ? 8 : (BS == 128 ? 7 : 6)));
    static_assert((1 << lbs) == BS, "workgroup size must be a power of two");
    uint64_t s_next = history_stream(P, R.seed, first + lo + threadIdx.x);
    for (uint64_t base = lo; base < hi; base += BS) {
        const uint64_t r = base + threadIdx.x;
        const bool valid = r < hi;
        Particle p;
        bool alive = false;
        int b = 0;
        const uint64_t s0 = s_next;
        s_next = (P.skipA[lbs] * s_next + P.skipC[lbs]) & kMask63;
        if (valid) {
            const uint64_t i = first + r;
            b = (int)(((i + 1) * (uint64_t)R.B - 1) / R.N);
            alive = birth<FM>(P, s0, p);
            if (R.dbg_counts) R.dbg_counts[i * 5 + 3] = 1u;
            if (!alive) {
                cnt.add(3 + kTime);
                hist_term(R, i, kTime);
            }
        }
        // (banks in list order: the births in history order)
        const uint32_t off = (!BAT && C.ordered) ? block_append_ordered<BS>(valid && alive, &cN, wtot)
                                                 : block_append(valid && alive, &cN);
        if (valid && alive) store_state<FM, WW>(P, bank, seg * C.L + off, p, pack_gk(p.g, b, p.k, p.inpin), (uint32_t)r);
        if (R.prof) cnt.prof(valid ? 1u : 0u, (valid && alive) ? state_bytes<FM, WW>(P) : 0u);
    }
    __syncthreads();
    if (threadIdx.x == 0) C.n_bank[seg] = cN;   // bank 0
    cnt.flush(R, CLS, red);
}

// ---------------------------------------------------------------------------
// advance: one flight per particle of the bank, score, file into a queue
// ---------------------------------------------------------------------------
enum Outcome : int { kNone = 0, kToNext = 1, kToSurface = 2, kToCollision = 3 };

template <int FM, bool WW, bool LT, bool BAT, int CLS = MCDC_PROF_ADVANCE, int BS = kBlock>
__global__ void __launch_bounds__(BS) k_advance(DevProblem P0, RunArgs R0, Bank cur, Bank next, Bank ev, Ctl C,
                                                    int par, int gn0, SplitBank SB, LdsTables tabs0,
                                                    const BatchItem *__restrict__ items,
                                                    const SegInfo *__restrict__ segs) {
    const int prob = BAT ? segs[blockIdx.x].prob : 0;
    const RunArgs &R = BAT ? items[prob].R : R0;
    const int gn = BAT ? items[prob].gn : gn0;
    __shared__ unsigned long long red[kCounters + 2];
    Counters cnt;
    __shared__ unsigned int cN, cS, cC;
    extern __shared__ double lt[];
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const uint32_t seg_end = seg0 + C.L - 1;
    const unsigned int n = C.n_bank[par * C.G + seg];
    const int step = *C.step;
    const uint64_t first = *C.first;
    cnt.init(red);
    if (threadIdx.x == 0) {
        cN = 0u;
        cS = 0u;
        cC = 0u;
    }
    StepScore sc;
    const DevProblem &Pin = BAT ? items[prob].P : P0;
    init_slice<BS>(Pin, sc, lt, gn, C.seg_b0[seg], step, 1);
    const DevProblem P = stage_tables<LT, BS>(Pin, BAT ? items[prob].tabs : tabs0,
                                                  reinterpret_cast<char *>(lt + slice_mult(Pin) * gn));
    __syncthreads();
    // software pipeline: the next particle's state is in flight while the
    // current one is moved
    RawState nx;
    if (threadIdx.x < n) load_raw<FM, WW>(P, cur, seg0 + threadIdx.x, nx);
    for (unsigned int j0 = 0; j0 < n; j0 += BS) {
        const unsigned int idx = j0 + threadIdx.x;
        const bool valid = idx < n;
        int outcome = kNone;
        int mask = 0;
        Particle p;
        uint32_t gk = 0, hid = 0;
        const RawState rs = nx;
        if (idx + BS < n) load_raw<FM, WW>(P, cur, seg0 + idx + BS, nx);
        if (valid) {
            unpack<FM, WW>(P, rs, p);
            gk = rs.gk;
            hid = rs.hidw;
            if (p.k > step) {
                outcome = kToNext;   // born in a later time bin: wait
            } else {
                const int cell = cell_index(P, p.ix);
                const Flight f = next_event<FM>(P, p, cell);
                const uint64_t i = first + hid;
                if (f.d == kInf) {
                    cnt.add(3 + kLost);
                    hist_term(R, i, kLost);
                } else {
                    const int b = (gk >> 5) & 1023u;
                    score_flight(P, R, sc, p, cell, b, i, hid, f.d);
                    move<FM>(P, p, f);
                    if (f.ev == kCensus) {
                        cnt.add(0);
                        hist_event(R, i, 0);
                        score_crossing(P, R, sc, p, cell, b);
                        p.k += 1;
                        if (p.k == P.K) {
                            cnt.add(3 + kTime);
                            hist_term(R, i, kTime);
                        } else if (ww_point<WW>(P, R, SB, p, cell, b, i, cnt)) {
                            outcome = kToNext;
                        }
                    } else if (f.ev == kSurface) {
                        cnt.add(1);
                        hist_event(R, i, 1);
                        mask = crossing_mask<FM>(P, f);
                        outcome = kToSurface;
                    } else {
                        cnt.add(2);
                        hist_event(R, i, 2);
                        outcome = kToCollision;
                    }
                }
            }
        }
        const uint32_t ns = block_append(outcome == kToNext, &cN);
        const uint32_t ss = block_append(outcome == kToSurface, &cS);
        const uint32_t cs = block_append(outcome == kToCollision, &cC);
        if (outcome == kToNext)
            store_state<FM, WW>(P, next, seg0 + ns, p, with_gk(gk, p), hid);
        else if (outcome == kToSurface)
            store_state<FM, WW>(P, ev, seg0 + ss, p, gk, hid | ((uint32_t)mask << 29));
        else if (outcome == kToCollision)
            store_state<FM, WW>(P, ev, seg_end - cs, p, gk, hid);
        if (R.prof && valid)
            cnt.prof(1u, state_bytes<FM, WW>(P) * (outcome == kNone ? 1u : 2u));
    }
    flush_slice<BS>(P, R, sc, step);
    if (threadIdx.x == 0) {
        C.n_bank[(par ^ 1) * C.G + seg] = cN;
        C.n_s[seg] = cS;
        C.n_c[seg] = cC;
    }
    cnt.flush(R, CLS, red);
}

// ---------------------------------------------------------------------------
// events: apply each queued event, then the rest of the step, in registers
// ---------------------------------------------------------------------------
// One launch takes both queues of a segment as one work list (surface
// particles first, then collision particles).  A lane whose particle has
// reached its census or died takes the next item of the list at once, so
// a wave is never held back by its longest-lived particle while work is
// left.  Each item starts with its queued event; every later step of it
// is a flight to the next event and that event.  The event cap counts
// flights from the item's start.
// (STEP: the whole census step in this one kernel: the work list is the
// step's bank itself, every item starting with a flight, and particles
// born in a later time bin pass straight on to the next bank.)
// (Two-kernel step with a queue sort at this step: both queues are read
// from the front of the sorted event bank srt, surface entries first.)
// (STEP, ns > 1: census steps step .. step + ns - 1 in one launch; a
// particle that reaches the edge of one goes on into the next in
// registers.)
// (ORD: banks in list order -- the weighted one-kernel step of a combed
// run writes every particle that goes on to its own slot of the next bank
// and a tombstone word to the slot of one that ends)
template <int FM, bool WW, bool LT, bool BAT, int CLS = MCDC_PROF_EVENTS, bool STEP = false, int BS = kBlock,
          bool ORD = false>
__global__ void __launch_bounds__(BS) k_event(DevProblem P0, RunArgs R0, Bank ev, Bank next, Ctl C, int par,
                                                  int gn0, SplitBank SB, LdsTables tabs0,
                                                  const BatchItem *__restrict__ items,
                                                  const SegInfo *__restrict__ segs, Bank srt, int cadence,
                                                  int ns) {
    const int prob = BAT ? segs[blockIdx.x].prob : 0;
    const RunArgs &R = BAT ? items[prob].R : R0;
    const int gn = BAT ? items[prob].gn : gn0;
    __shared__ unsigned long long red[kCounters + 2];
    __shared__ unsigned int cN, cW;
    Counters cnt;
    extern __shared__ double lt[];
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const uint32_t seg_end = seg0 + C.L - 1;
    const int step = *C.step;
    const uint64_t first = *C.first;
    const unsigned int n_s = STEP ? 0u : C.n_s[seg];
    const unsigned int n = STEP ? C.n_bank[par * C.G + seg] : n_s + C.n_c[seg];
    const bool sorted = !STEP && cadence > 0 && step % cadence == 0;
    const Bank &bsrc = sorted ? srt : ev;
    cnt.init(red);
    if (threadIdx.x == 0) {
        cN = STEP ? 0u : C.n_bank[(par ^ 1) * C.G + seg];   // after the advance kernel's census crossers
        cW = 0u;
    }
    StepScore sc;
    const DevProblem &Pin = BAT ? items[prob].P : P0;
    const int nsl = STEP ? ns : 1;   // census steps of the LDS slice
    init_slice<BS>(Pin, sc, lt, gn, C.seg_b0[seg], step, nsl);
    const DevProblem P = stage_tables<LT, BS>(Pin, BAT ? items[prob].tabs : tabs0,
                                                  reinterpret_cast<char *>(lt + slice_mult(Pin) * gn * nsl));
    __syncthreads();

    Particle p;
    uint32_t gk = 0, hid = 0, src = 0;
    int cell = 0, b = 0, queued = kCensus, mask = 0, since = 0;
    uint64_t i = 0;
    bool busy = false, exhausted = false, waiting = false;
    constexpr bool in_place = ORD && WW && STEP && !BAT;
    for (;;) {
        // idle lanes take the next items of the work list, once enough of
        // the wave is idle (or all of it)
        const int n_idle = kWave - __popcll(__ballot(busy));
        if (!exhausted && (n_idle >= kRefillMin || n_idle == kWave)) {
            const bool need = !busy;
            const uint32_t w = block_append(need, &cW);
            if (need && w < n) {
                uint32_t hidw;
                const uint32_t at = (STEP || sorted || w < n_s) ? seg0 + w : seg_end - (w - n_s);
                if constexpr (in_place) src = at;
                load_state<FM, WW>(P, bsrc, at, p, gk, hidw);
                hid = hidw & kHidMask;
                mask = STEP ? 0 : (int)(hidw >> 29);
                queued = STEP ? kCensus : ((w < n_s) ? kSurface : kCollision);
                waiting = STEP && p.k >= step + ns;   // born after this launch's census steps
                i = first + hid;
                b = (gk >> 5) & 1023u;
                cell = cell_index(P, p.ix);
                since = 0;
                busy = true;
                if (R.prof) cnt.prof(1u, state_bytes<FM, WW>(P));
            }
            exhausted = __ballot(need && w >= n) != 0;
        }
        const int n_busy = __popcll(__ballot(busy));
        if (n_busy == 0) break;
        const bool had = in_place && busy;
        // collisions wait until a share of the busy lanes has one (or no
        // lane has anything else to do), so that the wave runs the costly
        // collision code for many lanes at once
        const bool pend = busy && queued == kCollision;
        const int n_coll = __popcll(__ballot(pend));
        const int n_fly = __popcll(__ballot(busy && queued == kCensus));
        if (n_coll > 0 && (n_coll * 8 >= n_busy * kCollEighths || n_fly == 0) && pend) {
            queued = kCensus;
            const int m = (FM == 1) ? P.cell_mat[cell] : material_of(P, p, cell);
            int r = collide<FM, WW>(P, p, m);
            if (WW && r == 2) {
                // fission: neutrons 1..n-1 to the split bank
                const int nf = fission<FM>(P, p, m, SB, b, i, R.overflow);
                if (nf > 1) {
                    cnt.add(9, (unsigned int)(nf - 1));
                    if (R.dbg_counts) atomicAdd(R.dbg_counts + i * 5 + 3, (unsigned int)(nf - 1));
                }
                r = nf > 0 ? 1 : 0;
            }
            if (r == 0) {
                cnt.add(3 + kAbsorb);
                hist_term(R, i, kAbsorb);
                busy = false;
            } else if (WW && r == 3) {
                cnt.add(3 + kRoulette);
                hist_term(R, i, kRoulette);
                busy = false;
            } else if (!ww_point<WW>(P, R, SB, p, cell, b, i, cnt)) {
                busy = false;
            }
        }
        // a flight to the next event (or the queued surface crossing), and
        // the census or surface event it ends in; a collision is queued
        bool to_next = false;
        if (STEP && busy && waiting) {
            to_next = true;
            busy = false;
            waiting = false;
        } else if (busy && queued != kCollision) {
            int evt = queued;
            bool flown = true;
            if (queued == kCensus) {
                if (since >= kMaxEventsPerStep) {
                    cnt.add(3 + kLost);
                    hist_term(R, i, kLost);
                    busy = false;
                    flown = false;
                } else {
                    ++since;
                    const Flight f = next_event<FM>(P, p, cell);
                    if (f.d == kInf) {
                        cnt.add(3 + kLost);
                        hist_term(R, i, kLost);
                        busy = false;
                        flown = false;
                    } else {
                        score_flight(P, R, sc, p, cell, b, i, hid, f.d);
                        move<FM>(P, p, f);
                        evt = f.ev;
                        if (evt == kSurface) mask = crossing_mask<FM>(P, f);
                        if (evt == kCensus)
                            cnt.add(0);
                        else if (evt == kSurface)
                            cnt.add(1);
                        else
                            cnt.add(2);
                        hist_event(R, i, evt);   // census 0, surface 1, collision 2
                    }
                }
            }
            queued = kCensus;
            if (flown) {
                if (evt == kCensus) {
                    score_crossing(P, R, sc, p, cell, b);
                    p.k += 1;
                    if (p.k == P.K) {
                        cnt.add(3 + kTime);
                        hist_term(R, i, kTime);
                        busy = false;
                    } else if (!ww_point<WW>(P, R, SB, p, cell, b, i, cnt)) {
                        busy = false;
                    } else if (STEP && p.k < step + ns) {
                        since = 0;   // on into the launch's next census step, in registers
                    } else {
                        to_next = true;
                        busy = false;
                    }
                } else if (evt == kSurface) {
                    const int old_ww = WW ? P.cell_ww[cell] : 0;
                    const int face = cross<FM>(P, p, mask);
                    if (face >= 0) {
                        add_leak(P, R, b, p.k, p.g, face, p.w);
                        cnt.add(3 + kLeak);
                        hist_term(R, i, kLeak);
                        busy = false;
                    } else {
                        cell = cell_index(P, p.ix);
                        if (WW && P.cell_ww[cell] != old_ww && !ww_point<WW>(P, R, SB, p, cell, b, i, cnt))
                            busy = false;
                    }
                } else {
                    queued = kCollision;
                }
            }
        }
        if constexpr (in_place) {
            if (to_next) {
                store_state<FM, WW>(P, next, src, p, with_gk(gk, p), hid);
                if (R.prof) cnt.prof(0u, state_bytes<FM, WW>(P));
            } else if (had && !busy) {
                fld<uint32_t>(next, next.ogk, tile_off4(next, src)) = kTombGk;
            }
        } else {
            const uint32_t slot = block_append(to_next, &cN);
            if (to_next) {
                store_state<FM, WW>(P, next, seg0 + slot, p, with_gk(gk, p), hid);
                if (R.prof) cnt.prof(0u, state_bytes<FM, WW>(P));
            }
        }
    }
    flush_slice<BS>(P, R, sc, step);
    if (threadIdx.x == 0) C.n_bank[(par ^ 1) * C.G + seg] = in_place ? n : cN;
    cnt.flush(R, CLS, red);
}

// ---------------------------------------------------------------------------
// staged census step (slab, analog): the one-kernel step with every lane
// refill served from LDS
// ---------------------------------------------------------------------------
// Each wave claims whole 64-slot tiles of its segment's bank (one LDS atomic
// per tile: segments start on a tile, so a claim of 64 items is one tile)
// and copies each into one of its two LDS buffers with direct-to-LDS loads
// (global_load_lds_dwordx4: 1 KB per instruction, no registers held), one
// tile ahead of use.  A lane that takes a new particle reads its state from
// the buffer; the wave waits for its outstanding loads (vmcnt) only when it
// first reads a buffer filled since its last wait, and for its LDS reads
// (lgkmcnt) before a buffer is refilled.  Everything else is the one-kernel
// step: flights and events in registers, census crossers filed whole into
// the next bank with wave-ballot appends.  (The compiler cannot tell the
// buffers, addressed at run time, from the kernel's other LDS data, so it
// waits for the copies in flight before every later LDS access -- table
// lookups, tally-slice atomics, appends -- and the copies overlap little:
// this form measured 3 % slower than reading refills from HBM and runs
// only on request, MCDC_FLAG_STAGED.)
constexpr uint32_t kStageTile = 3328;   // bytes of a slab tile: x, u, t, tau, s (8 B); cell, g/k, history (4 B)

typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;

// the 64-slot tile t of a segment (global, 256-B aligned) into an LDS buffer
__device__ __forceinline__ void tile_to_lds(const char *tile, char *buf) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (uint32_t off = 0; off < kStageTile; off += 1024u)
        if (off + lane * 16u < kStageTile)
            __builtin_amdgcn_global_load_lds((global_void *)(tile + off + lane * 16u), (lds_void *)(buf + off), 16, 0,
                                             0);
}
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }    // vmcnt(0)
__device__ __forceinline__ void wait_lgkm() { __builtin_amdgcn_s_waitcnt(0xC07F); }  // lgkmcnt(0)

// a slab particle's state from slot j of a staged tile (the tile's layout)
__device__ __forceinline__ void load_state_lds(const DevProblem &P, const Bank &B, const char *buf, int j, Particle &p,
                                               uint32_t &gk, uint32_t &hidw) {
    p.x[0] = *reinterpret_cast<const double *>(buf + B.ox[0] + j * 8);
    p.u[0] = *reinterpret_cast<const double *>(buf + B.ou[0] + j * 8);
    p.x[1] = p.x[2] = 0.0;
    p.u[1] = p.u[2] = 0.0;
    p.t = *reinterpret_cast<const double *>(buf + B.ot + j * 8);
    p.tau = *reinterpret_cast<const double *>(buf + B.otau + j * 8);
    p.w = 1.0;
    p.s = *reinterpret_cast<const uint64_t *>(buf + B.os + j * 8);
    const uint32_t c = *reinterpret_cast<const uint32_t *>(buf + B.oc + j * 4);
    gk = *reinterpret_cast<const uint32_t *>(buf + B.ogk + j * 4);
    hidw = *reinterpret_cast<const uint32_t *>(buf + B.ohid + j * 4);
    set_inverse<1>(P, p);
    p.ix[0] = c & 2047u;
    p.ix[1] = (c >> 11) & 2047u;
    p.ix[2] = c >> 22;
    p.g = gk & 31u;
    p.k = (int)(gk >> 15);
    p.inpin = 0;
}

template <bool LT, int BS = kBlock>
__global__ void __launch_bounds__(BS) k_event_staged(DevProblem P0, RunArgs R, Bank cur, Bank next, Ctl C, int par,
                                                     int gn, LdsTables tabs0) {
    constexpr int FM = 1;
    constexpr bool WW = false;
    __shared__ __attribute__((aligned(16))) char stage[BS / 64][2][kStageTile];
    __shared__ unsigned long long red[kCounters + 2];
    __shared__ unsigned int cN, cT;
    Counters cnt;
    extern __shared__ double lt[];
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const unsigned int n = C.n_bank[par * C.G + seg];
    const int ntiles = (int)((n + 63u) >> 6);
    const int step = *C.step;
    const uint64_t first = *C.first;
    cnt.init(red);
    if (threadIdx.x == 0) {
        cN = 0u;
        cT = 0u;
    }
    StepScore sc;
    init_slice<BS>(P0, sc, lt, gn, C.seg_b0[seg], step, 1);
    const DevProblem P = stage_tables<LT, BS>(P0, tabs0, reinterpret_cast<char *>(lt + slice_mult(P0) * gn));
    __syncthreads();

    const uint32_t lane = __lane_id();
    char *const bufs = &stage[threadIdx.x >> 6][0][0];
    const char *const seg_tiles = cur.base + (uint64_t)(seg0 >> 6) * kStageTile;
    auto claim = [&]() -> int {
        unsigned int t = 0u;
        if (lane == 0) t = atomicAdd(&cT, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        return ((int)t < ntiles) ? (int)t : -1;
    };
    auto items_of = [&](int t) -> int { return t < 0 ? 0 : (int)min(64u, n - (uint32_t)t * 64u); };
    // the wave's two buffers: ta (current, head items taken) and tb (next)
    int ta = claim();
    if (ta >= 0) tile_to_lds(seg_tiles + (uint64_t)ta * kStageTile, bufs);
    int tb = (ta >= 0) ? claim() : -1;
    if (tb >= 0) tile_to_lds(seg_tiles + (uint64_t)tb * kStageTile, bufs + kStageTile);
    int cb = 0, head = 0, na = items_of(ta), nb = items_of(tb);
    bool pa = ta >= 0, pb = tb >= 0;   // buffer filled since the wave's last vmcnt wait

    Particle p;
    uint32_t gk = 0, hid = 0;
    int cell = 0, b = 0, since = 0;
    uint64_t i = 0;
    bool busy = false, exhausted = ta < 0, waiting = false;
    for (;;) {
        // idle lanes take the next items of the staged tiles
        if (!exhausted) {
            const bool need = !busy;
            const uint64_t m = __ballot(need);
            const int k = __popcll(m);
            const int pre =
                (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const int left = na - head;
            const bool from_a = need && pre < left;
            const bool from_b = need && !from_a && pre - left < nb;
            if ((k > 0 && left > 0 && pa) || (k > left && nb > 0 && pb)) {
                wait_vm();
                pa = pb = false;
            }
            if (from_a || from_b) {
                uint32_t hidw;
                const char *buf = bufs + (from_a ? cb : (cb ^ 1)) * kStageTile;
                load_state_lds(P, cur, buf, from_a ? head + pre : pre - left, p, gk, hidw);
                hid = hidw & kHidMask;
                waiting = p.k > step;   // born in a later time bin
                i = first + hid;
                b = (gk >> 5) & 1023u;
                cell = cell_index(P, p.ix);
                since = 0;
                busy = true;
                if (R.prof) cnt.prof(1u, state_bytes<FM, WW>(P));
            }
            const int taken = min(k, left + nb);
            head += taken;
            if (head >= na) {
                // the current buffer is spent: the next one becomes current
                // and the spent one is refilled once its reads are done
                head -= na;
                ta = tb;
                na = nb;
                pa = pb;
                cb ^= 1;
                tb = (ta >= 0) ? claim() : -1;
                nb = items_of(tb);
                pb = false;
                if (tb >= 0) {
                    wait_lgkm();
                    tile_to_lds(seg_tiles + (uint64_t)tb * kStageTile, bufs + (cb ^ 1) * kStageTile);
                    pb = true;
                }
            }
            exhausted = (na - head <= 0) && tb < 0;
        }
        if (!__any(busy)) break;
        bool to_next = false;
        if (busy && waiting) {
            to_next = true;
            busy = false;
            waiting = false;
        } else if (busy) {
            if (since >= kMaxEventsPerStep) {
                cnt.add(3 + kLost);
                hist_term(R, i, kLost);
                busy = false;
            } else {
                ++since;
                const Flight f = next_event<FM>(P, p, cell);
                if (f.d == kInf) {
                    cnt.add(3 + kLost);
                    hist_term(R, i, kLost);
                    busy = false;
                } else {
                    score_flight(P, R, sc, p, cell, b, i, hid, f.d);
                    move<FM>(P, p, f);
                    const int evt = f.ev;
                    if (evt == kCensus)
                        cnt.add(0);
                    else if (evt == kSurface)
                        cnt.add(1);
                    else
                        cnt.add(2);
                    hist_event(R, i, evt);
                    if (evt == kCensus) {
                        score_crossing(P, R, sc, p, cell, b);
                        p.k += 1;
                        if (p.k == P.K) {
                            cnt.add(3 + kTime);
                            hist_term(R, i, kTime);
                        } else {
                            to_next = true;
                        }
                        busy = false;
                    } else if (evt == kSurface) {
                        const int face = cross<FM>(P, p, crossing_mask<FM>(P, f));
                        if (face >= 0) {
                            add_leak(P, R, b, p.k, p.g, face, p.w);
                            cnt.add(3 + kLeak);
                            hist_term(R, i, kLeak);
                            busy = false;
                        } else {
                            cell = cell_index(P, p.ix);
                        }
                    } else {
                        if (collide<FM, WW>(P, p, P.cell_mat[cell]) == 0) {
                            cnt.add(3 + kAbsorb);
                            hist_term(R, i, kAbsorb);
                            busy = false;
                        }
                    }
                }
            }
        }
        const uint32_t ns = block_append(to_next, &cN);
        if (to_next) {
            store_state<FM, WW>(P, next, seg0 + ns, p, with_gk(gk, p), hid);
            if (R.prof) cnt.prof(0u, state_bytes<FM, WW>(P));
        }
    }
    flush_slice<BS>(P, R, sc, step);
    if (threadIdx.x == 0) C.n_bank[(par ^ 1) * C.G + seg] = cN;
    cnt.flush(R, MCDC_PROF_EVENTS, red);
}

// ---------------------------------------------------------------------------
// queue sort (two-kernel step): each segment's surface and collision queues
// reordered by (event, material, group, cell) into the sorted event bank
// before the events kernel, at the census steps k with k mod cadence == 0
// ---------------------------------------------------------------------------
// Bucket of an entry: queue * 256 + sub (queue 0 surface, 1 collision);
// sub = (m G + g) * CB + cell * CB / ncells with CB = 256 / (M G) cell
// sub-buckets per material and group (the material and group alone when
// M G >= 256).  Per segment: a histogram of the buckets in LDS, an
// exclusive prefix over the 512 buckets, then every entry copied whole to
// the next slot of its bucket.  Entries of one bucket land in the order
// of the LDS atomics; per-history results do not depend on it (each
// particle draws from its own stream), tallies only by summation order.
constexpr int kSortBuckets = 512;

template <int FM>
__device__ __forceinline__ int sort_bucket(const DevProblem &P, uint32_t c, uint32_t gk, int queue) {
    const int ix[3] = {(int)(c & 2047u), (int)((c >> 11) & 2047u), (int)(c >> 22)};
    const int cell = cell_index(P, ix);
    const int g = (int)(gk & 31u);
    const int m = material_at(P, cell, (FM == 1) ? 0 : (int)(gk >> 31));
    const int mg = m * P.G + g;
    const int nmg = P.M * P.G;
    int sub;
    if (nmg >= 256) {
        sub = mg & 255;
    } else {
        const int cb = 256 / nmg;
        sub = mg * cb + (int)(((int64_t)cell * cb) / P.ncells);
    }
    return queue * 256 + sub;
}

template <int FM, bool WW, bool BAT, int CLS = MCDC_PROF_SORT, int BS = kBlock>
__global__ void __launch_bounds__(BS) k_sort_events(DevProblem P0, RunArgs R0, Bank ev, Bank srt, Ctl C,
                                                        int cadence, const BatchItem *__restrict__ items,
                                                        const SegInfo *__restrict__ segs) {
    const int step = *C.step;
    if (cadence <= 0 || step % cadence != 0) return;
    const int prob = BAT ? segs[blockIdx.x].prob : 0;
    const DevProblem &P = BAT ? items[prob].P : P0;
    const RunArgs &R = BAT ? items[prob].R : R0;
    __shared__ unsigned long long red[kCounters + 2];
    constexpr int PER = (kSortBuckets + BS - 1) / BS;   // buckets per thread in the prefix
    __shared__ unsigned int off[kSortBuckets];
    __shared__ unsigned int wsum[BS / 64];
    Counters cnt;
    cnt.init(red);
    const unsigned int seg = blockIdx.x;
    const uint32_t seg0 = seg * C.L;
    const uint32_t seg_end = seg0 + C.L - 1;
    const unsigned int n_s = C.n_s[seg];
    const unsigned int n = n_s + C.n_c[seg];
    for (int j = threadIdx.x; j < kSortBuckets; j += BS) off[j] = 0u;
    __syncthreads();
    for (unsigned int w = threadIdx.x; w < n; w += BS) {
        const uint32_t slot = (w < n_s) ? seg0 + w : seg_end - (w - n_s);
        const uint64_t o4 = tile_off4(ev, slot);
        atomicAdd(&off[sort_bucket<FM>(P, fld<uint32_t>(ev, ev.oc, o4), fld<uint32_t>(ev, ev.ogk, o4),
                                       w < n_s ? 0 : 1)],
                  1u);
    }
    __syncthreads();
    // exclusive prefix over the buckets: each thread sums PER consecutive
    // buckets, a prefix of those sums within each wave by shuffles, then
    // the totals of the waves before
    unsigned int mine[PER];
    unsigned int v = 0u;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = (int)threadIdx.x * PER + q;
        mine[q] = (j < kSortBuckets) ? off[j] : 0u;
        v += mine[q];
    }
    unsigned int inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned int t = __shfl_up(inc, o);
        if ((int)__lane_id() >= o) inc += t;
    }
    if (__lane_id() == 63) wsum[threadIdx.x >> 6] = inc;
    __syncthreads();
    unsigned int base = 0u;
    for (unsigned int k = 0; k < (threadIdx.x >> 6); ++k) base += wsum[k];
    base += inc - v;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = (int)threadIdx.x * PER + q;
        if (j < kSortBuckets) off[j] = base;
        base += mine[q];
    }
    __syncthreads();
    for (unsigned int w = threadIdx.x; w < n; w += BS) {
        const uint32_t slot = (w < n_s) ? seg0 + w : seg_end - (w - n_s);
        RawState r;
        load_raw<FM, WW>(P, ev, slot, r);
        const unsigned int pos = atomicAdd(&off[sort_bucket<FM>(P, r.c, r.gk, w < n_s ? 0 : 1)], 1u);
        store_raw<FM, WW>(P, srt, seg0 + pos, r);
        if (R.prof) cnt.prof(1u, 8u + 2u * state_bytes<FM, WW>(P));
    }
    cnt.flush(R, CLS, red);
}

// ---------------------------------------------------------------------------
// population control at census: splitting-roulette to a target population
// ---------------------------------------------------------------------------
// (Section 2 lists population control among the time-dependent features
// without giving a method.)  After the step kernel has filed the census
// crossers of edge T_{k+1} into the next bank, two kernels control them:
// k_pc_sum forms each segment's exact weight sum (128-bit fixed point, 64
// fractional bits, so the total does not depend on the order of the
// particles); every workgroup of the next two adds the G partial sums in
// segment order and sets w_t = W / target.  k_pc_count counts the copies
// each segment makes; k_pc_apply copies every particle of the next bank
// back into the step's input bank, spread evenly over all segments: a
// crosser as n = floor(w / w_t + xi) copies of weight w_t (copy 0 keeps the
// stream after the draw, copy j >= 1 takes child_stream(s, j)), a particle
// of a later time bin unchanged.

__device__ __forceinline__ uint32_t clock_of(uint32_t gk) { return (gk >> 15) & 0xFFFFu; }

// overflow flag values of population control (1: particle or split bank)
constexpr int kOvfWeight = 2, kOvfCopies = 3, kOvfSegment = 4;

// profile tallies of a control kernel (particles, bytes): reduced per wave,
// then per workgroup in LDS, one global atomic per workgroup and counter;
// called by every thread of the workgroup
__device__ void pc_prof(const RunArgs &R, unsigned long long items, unsigned long long bytes) {
    __shared__ unsigned long long acc[2];
    if (!R.prof) return;
    if (threadIdx.x == 0) acc[0] = acc[1] = 0ull;
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) {
        items += __shfl_xor(items, o);
        bytes += __shfl_xor(bytes, o);
    }
    if (__lane_id() == 0) {
        atomicAdd(&acc[0], items);
        atomicAdd(&acc[1], bytes);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(R.prof + 2 * MCDC_PROF_CONTROL, acc[0]);
        atomicAdd(R.prof + 2 * MCDC_PROF_CONTROL + 1, acc[1]);
    }
}

__global__ void __launch_bounds__(kBlock) k_pc_sum(RunArgs R, Bank next, Ctl C, int par) {
    __shared__ unsigned long long part[kBlock / 64][2];
    const unsigned int seg = blockIdx.x;
    const unsigned int n = C.n_bank[(par ^ 1) * C.G + seg];
    const uint32_t edge = (uint32_t)(*C.step + 1);
    const uint32_t seg0 = seg * C.L;
    unsigned long long hi = 0ull, lo = 0ull, items = 0ull, bytes = 0ull;
    bool ok = true;
    for (uint32_t r = threadIdx.x; r < n; r += kBlock) {
        const uint32_t slot = seg0 + r;
        items += 1ull;
        bytes += 4ull;
        if (clock_of(fld<uint32_t>(next, next.ogk, tile_off4(next, slot))) != edge) continue;
        bytes += 8ull;
        ok = fixed_add(hi, lo, fld<double>(next, next.ow, tile_off8(next, slot))) && ok;
    }
    pc_prof(R, items, bytes);
    if (!ok) *R.overflow = kOvfWeight;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long h2 = __shfl_xor(hi, o), l2 = __shfl_xor(lo, o);
        fixed_merge(hi, lo, h2, l2);
    }
    if (__lane_id() == 0) {
        part[threadIdx.x >> 6][0] = hi;
        part[threadIdx.x >> 6][1] = lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long H = 0ull, L = 0ull;
        for (int w = 0; w < kBlock / 64; ++w) fixed_merge(H, L, part[w][0], part[w][1]);
        C.pc_w[2 * seg] = H;
        C.pc_w[2 * seg + 1] = L;
    }
}

// Workgroup-wide sums over the segments' partials (integers, so the order
// of the additions does not matter): the fixed-point weight W, then w_t =
// W / target and whether the control acts (W > 0); with counts, also the
// copies of all segments and of the segments before `seg`.  Every thread
// returns the same values.
struct PcSums {
    double W, wt;
    int on;
    unsigned long long total, before;
};
__device__ PcSums pc_sums(const Ctl &C, uint64_t target, unsigned int seg, bool counts) {
    __shared__ unsigned long long part[kBlock / 64][4];
    __shared__ PcSums res;
    unsigned long long hi = 0ull, lo = 0ull, tot = 0ull, bef = 0ull;
    for (unsigned int j = threadIdx.x; j < C.G; j += kBlock) {
        fixed_merge(hi, lo, C.pc_w[2 * j], C.pc_w[2 * j + 1]);
        if (counts) {
            const unsigned long long c = C.pc_cnt[j];
            tot += c;
            if (j < seg) bef += c;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long h2 = __shfl_xor(hi, o), l2 = __shfl_xor(lo, o);
        fixed_merge(hi, lo, h2, l2);
        tot += __shfl_xor(tot, o);
        bef += __shfl_xor(bef, o);
    }
    if (__lane_id() == 0) {
        part[threadIdx.x >> 6][0] = hi;
        part[threadIdx.x >> 6][1] = lo;
        part[threadIdx.x >> 6][2] = tot;
        part[threadIdx.x >> 6][3] = bef;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long H = 0ull, L = 0ull, T = 0ull, Bf = 0ull;
        for (int w = 0; w < kBlock / 64; ++w) {
            fixed_merge(H, L, part[w][0], part[w][1]);
            T += part[w][2];
            Bf += part[w][3];
        }
        const double W = (double)H + ((double)(L >> 32) * 0x1p-32 + (double)(L & 0xFFFFFFFFull) * 0x1p-64);
        res.W = W;
        res.wt = W / (double)target;
        res.on = (H | L) != 0ull;
        res.total = T;
        res.before = Bf;
    }
    __syncthreads();
    return res;
}

// Copies of particle p at the control of edge `edge`: floor(w / w_t + xi)
// for a crosser (its stream advances by the draw), 1 for a particle of a
// later time bin.  More than `cap` copies: overflow, none made.
__device__ __forceinline__ uint64_t pc_copies(Particle &p, int edge, bool on, double wt, double cap,
                                              const RunArgs &R) {
    if (!on || p.k != edge) return 1ull;
    const double nr = floor(p.w / wt + rn(p.s));
    if (nr > cap) {
        *R.overflow = kOvfCopies;
        return 0ull;
    }
    return (uint64_t)nr;
}

// Pass 2: copies per segment (the draws are repeated, not kept, by pass 3).
// (it reads only the weight, stream and clock of each particle)
// (comb: the copies of each controlled particle by slot, from k_comb_teeth)
__global__ void __launch_bounds__(kBlock) k_pc_count(RunArgs R, Bank next, Ctl C, int par, uint64_t target,
                                                     const uint32_t *__restrict__ comb) {
    __shared__ unsigned long long part[kBlock / 64];
    const unsigned int seg = blockIdx.x;
    const PcSums S = pc_sums(C, target, seg, false);
    const double wt = S.wt;
    const bool on = S.on != 0;
    const double cap = (double)C.G * (double)C.L;
    const unsigned int n = C.n_bank[(par ^ 1) * C.G + seg];
    const int edge = *C.step + 1;
    const uint32_t seg0 = seg * C.L;
    unsigned long long tot = 0ull, items = 0ull;
    for (uint32_t r = threadIdx.x; r < n; r += kBlock) {
        const uint32_t slot = seg0 + r;
        items += 1ull;
        Particle p;
        const uint32_t gk = fld<uint32_t>(next, next.ogk, tile_off4(next, slot));
        if (gk == kTombGk) continue;   // ended in the census step
        p.k = (int)clock_of(gk);
        if (comb) {
            tot += (on && p.k == edge) ? (unsigned long long)comb[slot] : 1ull;
            continue;
        }
        p.w = fld<double>(next, next.ow, tile_off8(next, slot));
        p.s = fld<uint64_t>(next, next.os, tile_off8(next, slot));
        tot += pc_copies(p, edge, on, wt, cap, R);
    }
    pc_prof(R, items, 20ull * items);   // clock word, weight, stream
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0ull;
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        C.pc_cnt[seg] = t;
    }
}

// Pass 3: the copies.  Segment seg's copies take the global positions
// [sum of the earlier segments' counts, + its count), and position q goes
// to slot q mod Lq of segment q / Lq, Lq = ceil(T / G) for T copies in all:
// the controlled population is spread evenly over the segments again (a
// segment's share would otherwise drift from step to step).
// (comb: the copies by slot from k_comb_teeth, no draw: copy 0 keeps the
// stream as it is)
// (banks in list order: the copies take their positions in slot order,
// each particle's copies together, copy 0 first, so the list order holds)
template <int FM, bool ORD = false>
__global__ void __launch_bounds__(kBlock) k_pc_apply(DevProblem P, RunArgs R, Bank next, Bank cur, Ctl C, int par,
                                                     uint64_t target, const uint32_t *__restrict__ comb) {
    __shared__ unsigned long long red[kCounters + 2];
    __shared__ unsigned long long wtot[kBlock / 64];
    __shared__ unsigned int cN;
    Counters cnt;
    cnt.init(red);
    const unsigned int seg = blockIdx.x;
    if (threadIdx.x == 0) cN = 0u;
    const PcSums S = pc_sums(C, target, seg, true);
    const double wt = S.wt;
    const bool on = S.on != 0;
    const double cap = (double)C.G * (double)C.L;
    const unsigned long long T = S.total, base = S.before;
    const unsigned long long Lq = (T + C.G - 1) / C.G;   // copies per output segment
    if (threadIdx.x == 0) {
        const unsigned long long lo = (unsigned long long)seg * Lq;
        const unsigned long long cnt_out = (T > lo) ? ((T - lo < Lq) ? T - lo : Lq) : 0ull;
        C.n_bank[par * C.G + seg] = (unsigned int)((cnt_out < C.L) ? cnt_out : C.L);
        if (Lq > C.L) *R.overflow = kOvfSegment;
    }
    const unsigned int n = C.n_bank[(par ^ 1) * C.G + seg];
    const int edge = *C.step + 1;
    const uint64_t first = *C.first;
    const uint32_t seg0 = seg * C.L;
    unsigned long long run = 0ull;   // copies placed so far (banks in list order)
    for (uint32_t b0 = 0; b0 < n; b0 += kBlock) {
        const uint32_t r = b0 + threadIdx.x;
        bool valid = r < n;
        Particle p;
        uint32_t gk = 0u, hidw = 0u;
        uint64_t copies = 0ull, sf = 0ull;
        if (ORD && valid && fld<uint32_t>(next, next.ogk, tile_off4(next, seg0 + r)) == kTombGk) valid = false;
        if (valid) {
            load_state<FM, true>(P, next, seg0 + r, p, gk, hidw);
            const bool ctl = on && p.k == edge;
            copies = comb ? (ctl ? (uint64_t)comb[seg0 + r] : 1ull) : pc_copies(p, edge, on, wt, cap, R);
            if (ctl) {
                const uint64_t i = first + (hidw & kHidMask);
                if (copies == 0ull) {
                    cnt.add(3 + kRoulette);
                    hist_term(R, i, kRoulette);
                } else {
                    p.w = wt;
                    cnt.add(8, (unsigned int)(copies - 1ull));
                    if (R.dbg_counts && copies > 1ull)
                        atomicAdd(R.dbg_counts + i * 5 + 3, (unsigned int)(copies - 1ull));
                }
            }
            sf = p.s;
        }
        if constexpr (ORD) {
            // the lane's copies at its exclusive prefix of the round's copies
            unsigned long long tot;
            const unsigned long long ex = block_exclusive<kBlock>(valid ? copies : 0ull, wtot, tot);
            for (uint64_t j = 0ull; valid && j < copies; ++j) {
                const unsigned long long q = base + run + ex + j;
                const unsigned long long os = q / Lq, oslot = q - os * Lq;
                if (os < C.G && oslot < C.L) {
                    p.s = (j > 0ull) ? child_stream(sf, j) : sf;
                    store_state<FM, true>(P, cur, (uint32_t)(os * C.L + oslot), p, gk, hidw);
                } else {
                    *R.overflow = kOvfSegment;
                }
            }
            run += tot;
        } else {
            // one copy per lane and round
            uint64_t j = 0ull;
            for (;;) {
                const bool put = valid && j < copies;
                if (!__any(put)) break;
                const uint32_t off = block_append(put, &cN);
                if (put) {
                    const unsigned long long q = base + off;
                    const unsigned long long os = q / Lq, oslot = q - os * Lq;
                    if (os < C.G && oslot < C.L) {
                        p.s = (j > 0ull) ? child_stream(sf, j) : sf;
                        store_state<FM, true>(P, cur, (uint32_t)(os * C.L + oslot), p, gk, hidw);
                    } else {
                        *R.overflow = kOvfSegment;
                    }
                    ++j;
                }
            }
        }
        if (R.prof) cnt.prof(valid ? 1u : 0u, valid ? (unsigned int)((copies + 1ull) * state_bytes<FM, true>(P)) : 0u);
    }
    cnt.flush(R, MCDC_PROF_CONTROL, red);
}

// ---------------------------------------------------------------------------
// population control by combing
// ---------------------------------------------------------------------------
// (The comb takes the controlled particles in the run's list order: the
// banks keep it -- births in history order, survivors in their slots
// through a census step, copies in their parent's place -- so the order is
// slot order, segment after segment.  One workgroup per segment scans the
// 128-bit fixed-point weights of its controlled particles in slot order,
// from the exact sum of the earlier segments, and counts the teeth in each
// particle's stretch [P, P + q) of the cumulative weight.)

// teeth of the comb below the fixed-point point (hi, lo)
__device__ __forceinline__ uint32_t comb_teeth(unsigned long long hi, unsigned long long lo, double W, uint64_t M,
                                               double u) {
    const double dx = (double)hi + ((double)(lo >> 32) * 0x1p-32 + (double)(lo & 0xFFFFFFFFull) * 0x1p-64);
    const double c = ceil((dx / W) * (double)M - u);
    if (!(c > 0.0)) return 0u;
    if (c >= (double)M) return (uint32_t)M;
    return (uint32_t)c;
}

__global__ void __launch_bounds__(kBlock) k_comb_teeth(RunArgs R, Bank next, Ctl C, int par, uint64_t target,
                                                       uint32_t *copies) {
    __shared__ unsigned long long wtot[kBlock / 64][2];
    __shared__ unsigned long long part[kBlock / 64][2];
    const unsigned int seg = blockIdx.x;
    const PcSums S = pc_sums(C, target, seg, false);
    if (!S.on) return;
    // the exact weight of the segments before this one
    unsigned long long bh = 0ull, bl = 0ull;
    for (unsigned int j = threadIdx.x; j < seg; j += kBlock) fixed_merge(bh, bl, C.pc_w[2 * j], C.pc_w[2 * j + 1]);
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long h2 = __shfl_xor(bh, o), l2 = __shfl_xor(bl, o);
        fixed_merge(bh, bl, h2, l2);
    }
    if (__lane_id() == 0) {
        part[threadIdx.x >> 6][0] = bh;
        part[threadIdx.x >> 6][1] = bl;
    }
    __syncthreads();
    bh = bl = 0ull;
    for (int w = 0; w < kBlock / 64; ++w) fixed_merge(bh, bl, part[w][0], part[w][1]);
    const uint32_t edge = (uint32_t)(*C.step + 1);
    uint64_t su = child_stream(*C.seed, (1ull << 62) + edge);
    const double u = rn(su);
    const unsigned int n = C.n_bank[(par ^ 1) * C.G + seg];
    const uint32_t seg0 = seg * C.L;
    unsigned long long items = 0ull, bytes = 0ull;
    for (uint32_t b0 = 0; b0 < n; b0 += kBlock) {
        const uint32_t r = b0 + threadIdx.x;
        unsigned long long qh = 0ull, ql = 0ull;
        bool member = false;
        if (r < n) {
            items += 1ull;
            bytes += 8ull;   // clock word; weight and copy count of a member
            member = clock_of(fld<uint32_t>(next, next.ogk, tile_off4(next, seg0 + r))) == edge;
            if (member) {
                bytes += 12ull;
                fixed_add(qh, ql, fld<double>(next, next.ow, tile_off8(next, seg0 + r)));
            }
        }
        unsigned long long eh, el, th, tl;
        block_exclusive_u128<kBlock>(qh, ql, wtot, eh, el, th, tl);
        if (member) {
            unsigned long long ah = bh, al = bl;
            fixed_merge(ah, al, eh, el);
            unsigned long long zh = ah, zl = al;
            fixed_merge(zh, zl, qh, ql);
            copies[seg0 + r] = comb_teeth(zh, zl, S.W, target, u) - comb_teeth(ah, al, S.W, target, u);
        }
        fixed_merge(bh, bl, th, tl);
    }
    pc_prof(R, items, bytes);
}

// ---------------------------------------------------------------------------
// control
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(Ctl C, uint64_t first, uint64_t seed) {
    *C.step = 0;
    *C.first = first;
    *C.seed = seed & kMask63;
}
__global__ void k_step_end(Ctl C, int inc) { *C.step += inc; }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Layout {
    Bank bank[2];
    Bank ev;
    Bank srt;   // sorted event bank (queue sort on), else base == nullptr
    Ctl ctl;
};

size_t pad256(size_t b) { return (b + 255) & ~size_t(255); }

// Tile layout of a bank for the axes in fmask (all three if 0) and, with
// ww, the weight field.
Bank bank_layout(int fmask, bool ww) {
    Bank B{};
    const int axes = fmask ? fmask : 7;
    uint32_t o = 0;
    for (int a = 0; a < 3; ++a)
        if ((axes >> a) & 1) {
            B.ox[a] = o;
            o += 512;
        }
    for (int a = 0; a < 3; ++a)
        if ((axes >> a) & 1) {
            B.ou[a] = o;
            o += 512;
        }
    B.ot = o;
    o += 512;
    B.otau = o;
    o += 512;
    if (ww) {
        B.ow = o;
        o += 512;
    }
    B.os = o;
    o += 512;
    B.oc = o;
    o += 256;
    B.ogk = o;
    o += 256;
    B.ohid = o;
    o += 256;
    B.tile = o;
    return B;
}

// Bytes of one bank of `slots` slots (whole tiles).
size_t bank_bytes(uint64_t slots, int fmask, bool ww) { return ((slots + 63) / 64) * bank_layout(fmask, ww).tile; }

size_t ctl_bytes(unsigned int G) {
    return pad256(2 * G * 4) + 3 * pad256(G * 4) + 2 * 256 + pad256(G * 16) + pad256(G * 8);
}

// (banks: 3, or 4 with the sorted event bank of the queue sort)
Layout carve(void *bank_mem, void *ctl_mem, uint64_t slots, unsigned int G, unsigned int Lseg, int fmask,
             bool ww, int banks = 3) {
    Layout Lo{};
    char *p = (char *)bank_mem;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += pad256(bytes);
        return r;
    };
    for (int k = 0; k < banks; ++k) {
        Bank &B = (k < 2) ? Lo.bank[k] : (k == 2 ? Lo.ev : Lo.srt);
        B = bank_layout(fmask, ww);
        B.base = take(bank_bytes(slots, fmask, ww));
    }
    p = (char *)ctl_mem;
    Ctl &C = Lo.ctl;
    C.n_bank = (unsigned int *)take(2 * G * 4);
    C.n_s = (unsigned int *)take(G * 4);
    C.n_c = (unsigned int *)take(G * 4);
    C.seg_b0 = (int *)take(G * 4);
    C.step = (int *)take(64);
    C.first = (uint64_t *)take(64);
    C.seed = C.first + 1;
    C.pc_w = (unsigned long long *)take(G * 16);
    C.pc_cnt = (unsigned long long *)take(G * 8);
    C.G = G;
    C.L = Lseg;
    C.Lh = Lseg;
    return Lo;
}

// Captured census steps, cached per problem and re-captured when any
// kernel argument changes: one step per bank parity, and a stretch of
// consecutive steps starting at either parity (all K steps of a chunk, or
// with sampled profiling the steps between two sampled ones) so that a
// stretch costs one graph launch instead of one per step.
struct StepGraphs {
    std::vector<char> key;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec_run[2] = {nullptr, nullptr};
    hipGraph_t graph_run[2] = {nullptr, nullptr};
    hipStream_t cs = nullptr;
    void clear() {
        for (int q = 0; q < 2; ++q) {
            if (exec[q]) (void)hipGraphExecDestroy(exec[q]);
            if (graph[q]) (void)hipGraphDestroy(graph[q]);
            if (exec_run[q]) (void)hipGraphExecDestroy(exec_run[q]);
            if (graph_run[q]) (void)hipGraphDestroy(graph_run[q]);
            exec[q] = nullptr;
            graph[q] = nullptr;
            exec_run[q] = nullptr;
            graph_run[q] = nullptr;
        }
        key.clear();
    }
};

template <class T>
void key_add(std::vector<char> &k, const T &v) {
    const char *p = reinterpret_cast<const char *>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

// Workgroups (= segments) per CU when the caller leaves it open.  Each
// segment streams its own slice of every bank array, so fewer, larger
// workgroups keep fewer concurrent streams open per HBM channel: two
// 512-thread workgroups per CU (16 waves) measured fastest on both the slab
// and the lattice workloads (four 256-thread ones: 5 % slower; segment
// counts that are not a multiple of the CU count: 10-20 % slower).
constexpr int kSegmentsPerCU = 2;

// Doubles of a 1024-thread workgroup's LDS tally slice over several census
// steps (96 KiB; with the staged tables at most 128 KiB of the compute
// unit's 160 KiB).
constexpr int64_t kLdsStepsMax = 12288;

// (BS: workgroup size of the step kernels; weighted runs use kBlock)
template <int FM, bool WW, bool LT, int BS>
int run_event(mcdc_problem *pb, const RunArgs &R0, uint64_t first, uint64_t count, const mcdc_run_options &opt,
              hipStream_t st, Profiler &prof, const LdsTables &tabs) {
    const DevProblem &P = pb->d;
    // (weight-window runs take smaller chunks: their progeny of a chunk must
    // fit the split bank)
    // (population control runs the whole job as one chunk)
    const uint64_t pc = opt.pc_target;
    if (pc && !WW) {
        set_error("population control needs the weighted event form");
        return MCDC_E_UNSUPPORTED;
    }
    uint64_t C = opt.bank_capacity ? (uint64_t)opt.bank_capacity
                                   : (WW ? (P.fission_on ? kFissionChunk : kWindowChunk) : (uint64_t)1 << 24);
    if (pc) C = count;
    if (C > count) C = count;
    if (C > (1ULL << 28)) C = 1ULL << 28;

    // census steps per launch of the one-kernel step (analog only: the
    // weighted forms act between steps)
    const int cadence = opt.sort_cadence > 0 ? opt.sort_cadence : 0;
    const bool one_kernel = (opt.flags & MCDC_FLAG_TWO_KERNEL_STEP) == 0 && cadence == 0;
    const bool multi = !WW && !pc && one_kernel && !(opt.flags & MCDC_FLAG_STAGED);
    // (default: every census step of the chunk, or as many as the LDS slice
    // holds)
    int ns = opt.steps_per_launch > 0 ? opt.steps_per_launch : P.K;
    if (opt.steps_per_launch > 1 && !multi) {
        set_error("steps_per_launch > 1 needs the analog one-kernel step");
        return MCDC_E_UNSUPPORTED;
    }
    if (!multi) ns = 1;
    if (ns > P.K) ns = P.K;

    // per-step tally slice [2 batches][G][nts] in LDS when it fits (for
    // each of the launch's census steps: fewer steps per launch until it
    // does), then the staged tables
    // (a 1024-thread workgroup has its compute unit's LDS to itself, so its
    // slice of several steps may take up to kLdsStepsMax doubles)
    const int64_t gn64 = (int64_t)P.G * P.nts;
    const int gn = (slice_mult(P) * gn64 <= kLdsTallyMax) ? (int)gn64 : 0;
    const int64_t lds_max = (BS == 1024 && ns > 1) ? kLdsStepsMax : kLdsTallyMax;
    while (gn && ns > 1 && slice_mult(P) * gn64 * ns > lds_max) --ns;
    const size_t shmem = (size_t)slice_mult(P) * gn * ns * sizeof(double) + (LT ? (size_t)tabs.bytes : 0);
    const int NL = (P.K + ns - 1) / ns;   // launches per chunk
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_event<FM, WW, LT, false, MCDC_PROF_EVENTS,
                                                                                   true, BS>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return hip_fail(e, "LDS size of the multi-step launch");
    }

    // segments: one per workgroup
    unsigned int G;
    if (opt.segments > 0) {
        G = (unsigned int)opt.segments;
    } else {
        int per_cu = 0, n_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_advance<FM, WW, LT, false, MCDC_PROF_ADVANCE, BS>), BS,
            shmem > 65536 ? (size_t)65536 : shmem);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, pb->device);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        if (per_cu < 1) per_cu = 1;
        // (as many waves per CU as two 512-thread workgroups)
        const int cap = kSegmentsPerCU * kBlock / BS;
        if (per_cu > cap) per_cu = cap;
        G = (unsigned int)per_cu * (unsigned int)(n_cu > 0 ? n_cu : 1);
    }
    const uint64_t g_need = (C + BS - 1) / BS;
    if (G > g_need) G = (unsigned int)g_need;
    if (G < 1) G = 1;
    // (segments are whole tiles of 64 slots; with population control a
    // segment also holds its even share of the target population, plus a
    // tile for the control's noise)
    const unsigned int Lh = (unsigned int)(((C + G - 1) / G + 63) & ~(uint64_t)63);
    const unsigned int Lseg = pc ? Lh + (unsigned int)(((pc + G - 1) / G + 63) & ~(uint64_t)63) + 64u : Lh;
    const uint64_t slots = (uint64_t)G * Lseg;
    // queue sort at every cadence-th census step (two-kernel step only)
    const int nbanks = cadence ? 4 : 3;
    int rc;
    if ((rc = ensure(pb->bank, pad256(bank_bytes(slots, FM, WW)) * nbanks + 64 * 256))) return rc;
    if ((rc = ensure(pb->queues, ctl_bytes(G)))) return rc;
    if (P.qoi_on && (rc = ensure(pb->qoi_hist, C * sizeof(double)))) return rc;
    Layout L = carve(pb->bank.p, pb->queues.p, slots, G, Lseg, FM ? FM : P.finite_mask, WW, nbanks);
    L.ctl.Lh = Lh;
    RunArgs R = R0;
    R.qoi_hist = (double *)pb->qoi_hist.p;
    // weight windows and fission: progeny of a chunk go to the split bank and are
    // tracked after its census steps
    SplitBank SB[2]{};
    if (WW && (rc = split_prepare(pb, C, SB))) return rc;

    // population control by combing: the banks keep the run's list order
    // (births in history order, survivors in their slots, copies in their
    // parent's place), and the comb writes each controlled particle's teeth
    // per slot; the one-kernel step only
    const bool comb = pc && opt.pc_method == MCDC_PC_COMB;
    uint32_t *comb_copies = nullptr;
    if (comb) {
        if (!one_kernel) {
            set_error("combing runs the one-kernel census step (no two-kernel step or queue sort)");
            return MCDC_E_UNSUPPORTED;
        }
        if ((rc = ensure(pb->comb, pad256((size_t)slots * 4)))) return rc;
        comb_copies = (uint32_t *)pb->comb.p;
    }
    L.ctl.ordered = comb ? 1u : 0u;

    // the step kernels never read the seed or the history count; Rs is the
    // uninstrumented form the graphs capture, Rp the profiled one
    RunArgs Rs = R;
    Rs.seed = 0;
    Rs.N = 0;
    const RunArgs Rp = Rs;
    Rs.prof = nullptr;
    const int every = opt.profile_every > 1 ? opt.profile_every : 1;

    // one kernel per census step (default), or the advance / events pair
    // the slab's one-kernel step with its refills served through per-wave
    // LDS staging, when asked for (measured 3 % slower: kept for comparison)
    const bool staged = one_kernel && FM == 1 && !WW && (opt.flags & MCDC_FLAG_STAGED) != 0 &&
                        L.bank[0].tile == kStageTile;
    // (with population control the controlled particles go back into the
    // step's input bank, so every step runs on bank 0)
    auto enqueue_step = [&](int par_in, hipStream_t s, Profiler &pr, const RunArgs &Ra) {
        const int par = pc ? 0 : par_in;
        const Bank &cur = L.bank[par];
        const Bank &nxt = L.bank[par ^ 1];
        if (staged) {
            if constexpr (FM == 1 && !WW)
                launch_timed(pr, MCDC_PROF_EVENTS, k_event_staged<LT, BS>, dim3(G), dim3(BS), (uint32_t)shmem, s, P, Ra,
                             cur, nxt, L.ctl, par, gn, tabs);
        } else if (one_kernel && WW && comb) {
            if constexpr (WW)
                launch_timed(pr, MCDC_PROF_EVENTS, k_event<FM, WW, LT, false, MCDC_PROF_EVENTS, true, BS, true>,
                             dim3(G), dim3(BS), (uint32_t)shmem, s, P, Ra, cur, nxt, L.ctl, par, gn, SB[0], tabs,
                             (const BatchItem *)nullptr, (const SegInfo *)nullptr, L.srt, 0, ns);
        } else if (one_kernel) {
            launch_timed(pr, MCDC_PROF_EVENTS, k_event<FM, WW, LT, false, MCDC_PROF_EVENTS, true, BS>, dim3(G),
                         dim3(BS), (uint32_t)shmem, s, P, Ra, cur, nxt, L.ctl, par, gn, SB[0], tabs,
                         (const BatchItem *)nullptr, (const SegInfo *)nullptr, L.srt, 0, ns);
        } else {
            launch_timed(pr, MCDC_PROF_ADVANCE, k_advance<FM, WW, LT, false, MCDC_PROF_ADVANCE, BS>, dim3(G), dim3(BS),
                         (uint32_t)shmem,
                         s, P, Ra, cur, nxt, L.ev, L.ctl, par, gn, SB[0], tabs, (const BatchItem *)nullptr,
                         (const SegInfo *)nullptr);
            if (cadence)
                launch_timed(pr, MCDC_PROF_SORT, k_sort_events<FM, WW, false, MCDC_PROF_SORT, BS>, dim3(G), dim3(BS), 0u, s,
                             P, Ra,
                             L.ev, L.srt, L.ctl, cadence, (const BatchItem *)nullptr, (const SegInfo *)nullptr);
            launch_timed(pr, MCDC_PROF_EVENTS, k_event<FM, WW, LT, false, MCDC_PROF_EVENTS, false, BS>, dim3(G), dim3(BS),
                         (uint32_t)shmem, s,
                         P, Ra, L.ev, nxt, L.ctl, par, gn, SB[0], tabs, (const BatchItem *)nullptr,
                         (const SegInfo *)nullptr, L.srt, cadence, 1);
        }
        if constexpr (WW) {
            if (pc) {
                launch_timed(pr, MCDC_PROF_CONTROL, k_pc_sum, dim3(G), dim3(kBlock), 0u, s, Ra, nxt, L.ctl, par);
                if (comb)
                    launch_timed(pr, MCDC_PROF_CONTROL, k_comb_teeth, dim3(G), dim3(kBlock), 0u, s, Ra, nxt, L.ctl,
                                 par, pc, comb_copies);
                const uint32_t *cc = comb_copies;
                launch_timed(pr, MCDC_PROF_CONTROL, k_pc_count, dim3(G), dim3(kBlock), 0u, s, Ra, nxt, L.ctl, par, pc,
                             cc);
                if (comb)
                    launch_timed(pr, MCDC_PROF_CONTROL, k_pc_apply<FM, true>, dim3(G), dim3(kBlock), 0u, s, P, Ra, nxt,
                                 cur, L.ctl, par, pc, cc);
                else
                    launch_timed(pr, MCDC_PROF_CONTROL, k_pc_apply<FM>, dim3(G), dim3(kBlock), 0u, s, P, Ra, nxt, cur,
                                 L.ctl, par, pc, cc);
            }
        }
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, s, L.ctl, ns);
    };

    // replay captured steps unless per-history debug output is requested;
    // profiled steps launch eagerly
    const bool use_graph = !(opt.flags & MCDC_FLAG_EAGER) && !(opt.profile && every == 1) && !R.dbg_counts &&
                           !R.dbg_scores && NL > 1;
    StepGraphs *Gr = nullptr;
    // stretch of unsampled launches captured as one graph (none below 2)
    const int span = opt.profile ? every - 1 : NL;
    const int n_run = (span >= 2 && span <= 4096) ? (opt.profile ? 2 : 1) : 0;
    if (use_graph) {
        if (!pb->graph_cache) pb->graph_cache = new StepGraphs();
        Gr = (StepGraphs *)pb->graph_cache;
        std::vector<char> key;
        key_add(key, P);
        key_add(key, Rs);
        key_add(key, L);
        key_add(key, gn);
        key_add(key, SB[0]);
        key_add(key, tabs);
        key_add(key, LT);
        key_add(key, one_kernel);
        key_add(key, staged);
        key_add(key, cadence);
        key_add(key, ns);
        key_add(key, pc);
        key_add(key, comb_copies);
        key_add(key, span);
        key_add(key, n_run);
        if (key != Gr->key) {
            Gr->clear();
            hipError_t e = hipSuccess;
            if (!Gr->cs) e = hipStreamCreateWithFlags(&Gr->cs, hipStreamNonBlocking);
            Profiler none;
            for (int q = 0; q < 2 && e == hipSuccess; ++q) {
                e = hipStreamBeginCapture(Gr->cs, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) break;
                enqueue_step(q, Gr->cs, none, Rs);
                e = hipStreamEndCapture(Gr->cs, &Gr->graph[q]);
                if (e == hipSuccess) e = hipGraphInstantiate(&Gr->exec[q], Gr->graph[q], nullptr, nullptr, 0);
            }
            for (int q = 0; q < n_run && e == hipSuccess; ++q) {
                e = hipStreamBeginCapture(Gr->cs, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) break;
                for (int j = 0; j < span; ++j) enqueue_step((q + j) & 1, Gr->cs, none, Rs);
                e = hipStreamEndCapture(Gr->cs, &Gr->graph_run[q]);
                if (e == hipSuccess) e = hipGraphInstantiate(&Gr->exec_run[q], Gr->graph_run[q], nullptr, nullptr, 0);
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
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, st, L.ctl, cfirst, R.seed);
        if (P.qoi_on && (rc = launch_zero(R.qoi_hist, n * sizeof(double), st))) return hip_fail((hipError_t)rc, "zero");
        if (WW) split_reset(SB, st);
        launch_timed(prof, MCDC_PROF_SOURCE, k_source<FM, WW, false, MCDC_PROF_SOURCE, BS>, dim3(G), dim3(BS), 0u, st, P,
                     R, L.bank[0], L.ctl, n, (const BatchItem *)nullptr, (const SegInfo *)nullptr);
        // launch j takes census steps j ns .. j ns + ns - 1
        for (int j = 0; j < NL;) {
            const bool sampled = opt.profile && j % every == opt.profile_phase % every;
            // a whole stretch of unsampled launches from here: from the
            // first without profiling, else right after a sampled one
            const bool stretch = Gr && n_run > 0 && j + span <= NL &&
                                 (opt.profile ? j % every == (opt.profile_phase % every + 1) % every : j == 0);
            if (stretch) {
                hipError_t e = hipGraphLaunch(Gr->exec_run[(pc || n_run == 1) ? 0 : (j & 1)], st);
                if (e != hipSuccess) return hip_fail(e, "census steps replay");
                j += span;
                continue;
            }
            if (Gr && !sampled) {
                hipError_t e = hipGraphLaunch(Gr->exec[pc ? 0 : (j & 1)], st);
                if (e != hipSuccess) return hip_fail(e, "census step replay");
            } else {
                Profiler none;
                enqueue_step(j & 1, st, sampled ? prof : none, sampled ? Rp : Rs);
            }
            ++j;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "event kernel launch");
        if (WW && (rc = split_generations(pb, R, SB, cfirst, st, prof))) return rc;
        if (P.qoi_on && (rc = launch_qoi_reduce(R.qoi_hist, n, R.qoi_sums, st)))
            return hip_fail((hipError_t)rc, "detector reduce");
    }
    return MCDC_OK;
}

template <int FM, bool WW, int BS>
int run_event_bs(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count, const mcdc_run_options &opt,
                 hipStream_t st, Profiler &prof, const LdsTables &tabs, bool lt) {
    return lt ? run_event<FM, WW, true, BS>(p, R, first, count, opt, st, prof, tabs)
              : run_event<FM, WW, false, BS>(p, R, first, count, opt, st, prof, tabs);
}

// The step kernels' workgroup size: analog runs take opt.block_size 256,
// 512 or 1024 (0 = 1024: one 16-wave workgroup per CU shares one work list,
// so no wave idles while the other workgroup of its CU still has
// particles; the slab's step measured 5 % faster than with two 512-thread
// workgroups); weighted runs and population control always 512.
template <int FM, bool WW>
int run_event_lt(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count, const mcdc_run_options &opt,
                 hipStream_t st, Profiler &prof, const LdsTables &tabs, bool lt) {
    if constexpr (!WW) {
        if (opt.block_size == 256) return run_event_bs<FM, WW, 256>(p, R, first, count, opt, st, prof, tabs, lt);
        if (opt.block_size == 512) return run_event_bs<FM, WW, 512>(p, R, first, count, opt, st, prof, tabs, lt);
        return run_event_bs<FM, WW, 1024>(p, R, first, count, opt, st, prof, tabs, lt);
    }
    return run_event_bs<FM, WW, kBlock>(p, R, first, count, opt, st, prof, tabs, lt);
}

// Batched solve: every problem's segments share one set of banks; each
// census step (advance, events, step end over all segments of all
// problems) is captured once as a graph and replayed for the largest K.
// (step < 0: one kernel per census step; 0: the two-kernel step; c >= 1:
// the two-kernel step with the queue sort at every c-th census step)
template <int FM, bool LT, int BS>
int run_batched_steps(const BatchItem *d_items, const SegInfo *d_segs, unsigned int G, unsigned int Lseg, int Kmax,
                      size_t shmem, void *bank_mem, void *ctl_mem, hipStream_t st, int step_form, int ns) {
    const uint64_t slots = (uint64_t)G * Lseg;
    Layout L = carve(bank_mem, ctl_mem, slots, G, Lseg, FM, false, step_form > 0 ? 4 : 3);
    const DevProblem P0{};
    const RunArgs R0{};
    const LdsTables t0{};
    const SplitBank none{};
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, st, L.ctl, (uint64_t)0, (uint64_t)0);
    hipLaunchKernelGGL((k_source<FM, false, true, MCDC_PROF_SOURCE, BS>), dim3(G), dim3(BS), 0, st, P0, R0, L.bank[0], L.ctl,
                       (uint64_t)0, d_items, d_segs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched source launch");
    hipStream_t cs = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) break;
        if (step_form < 0) {
            hipLaunchKernelGGL((k_event<FM, false, LT, true, MCDC_PROF_EVENTS, true, BS>), dim3(G), dim3(BS), shmem,
                               cs, P0, R0, L.bank[q], L.bank[q ^ 1], L.ctl, q, 0, none, t0, d_items, d_segs, L.srt,
                               0, ns);
        } else {
            hipLaunchKernelGGL((k_advance<FM, false, LT, true, MCDC_PROF_ADVANCE, BS>), dim3(G), dim3(BS), shmem, cs, P0, R0, L.bank[q],
                               L.bank[q ^ 1], L.ev, L.ctl, q, 0, none, t0, d_items, d_segs);
            if (step_form > 0)
                hipLaunchKernelGGL((k_sort_events<FM, false, true, MCDC_PROF_SORT, BS>), dim3(G), dim3(BS), 0, cs, P0, R0, L.ev,
                                   L.srt, L.ctl, step_form, d_items, d_segs);
            hipLaunchKernelGGL((k_event<FM, false, LT, true, MCDC_PROF_EVENTS, false, BS>), dim3(G), dim3(BS), shmem, cs, P0, R0, L.ev,
                               L.bank[q ^ 1], L.ctl, q, 0, none, t0, d_items, d_segs, L.srt, step_form, 1);
        }
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, cs, L.ctl, step_form < 0 ? ns : 1);
        e = hipStreamEndCapture(cs, &graph[q]);
        if (e == hipSuccess) e = hipGraphInstantiate(&exec[q], graph[q], nullptr, nullptr, 0);
    }
    // (one-kernel form: ns census steps per launch)
    const int launches = step_form < 0 ? (Kmax + ns - 1) / ns : Kmax;
    for (int k = 0; k < launches && e == hipSuccess; ++k) e = hipGraphLaunch(exec[k & 1], st);
    hipError_t e2 = hipStreamSynchronize(st);
    for (int q = 0; q < 2; ++q) {
        if (exec[q]) (void)hipGraphExecDestroy(exec[q]);
        if (graph[q]) (void)hipGraphDestroy(graph[q]);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "batched census steps");
    if (e2 != hipSuccess) return hip_fail(e2, "batched census steps");
    return MCDC_OK;
}

struct BatchedLayout {
    size_t items_off, segs_off, ctl_off, bank_off, bytes;
    unsigned int G;
};

BatchedLayout batched_layout(const uint64_t *n_hist, int n, unsigned int Lseg, int banks) {
    BatchedLayout b{};
    uint64_t G = 0;
    for (int j = 0; j < n; ++j) G += (n_hist[j] + Lseg - 1) / Lseg;
    if (G == 0) G = 1;
    b.G = (unsigned int)G;
    b.items_off = 0;
    b.segs_off = pad256(sizeof(BatchItem) * n);
    b.ctl_off = b.segs_off + pad256(sizeof(SegInfo) * G);
    b.bank_off = b.ctl_off + ctl_bytes((unsigned int)G);
    b.bytes = b.bank_off + pad256(bank_bytes(G * Lseg, 0, false)) * banks + 64 * 256;
    return b;
}

}  // namespace

size_t event_batched_bytes(const uint64_t *n_hist, int n, unsigned int seg_len, int step_form) {
    return batched_layout(n_hist, n, seg_len, step_form > 0 ? 4 : 3).bytes;
}

int launch_event_batched(std::vector<BatchItem> &items, const uint64_t *n_hist, unsigned int seg_len, void *mem,
                         size_t mem_bytes, hipStream_t st, int step_form, int block) {
    const int n = (int)items.size();
    const BatchedLayout lay = batched_layout(n_hist, n, seg_len, step_form > 0 ? 4 : 3);
    if (lay.bytes > mem_bytes) {
        set_error("batched solve: work memory too small");
        return MCDC_E_INVALID;
    }
    // per-problem slice and table layouts; one template for all problems
    bool lt_all = true;
    int fm = -1, Kmax = 0;
    std::vector<bool> fit(n);
    for (int j = 0; j < n; ++j) {
        const DevProblem &P = items[j].P;
        fit[j] = table_layout(P, items[j].tabs, kLdsTablesMax);
        lt_all = lt_all && fit[j];
        const int64_t gn64 = (int64_t)P.G * P.nts;
        items[j].gn = (slice_mult(P) * gn64 <= kLdsTallyMax) ? (int)gn64 : 0;
        fm = (fm < 0 || fm == P.finite_mask) ? P.finite_mask : 0;
        if (P.K > Kmax) Kmax = P.K;
    }
    // one-kernel form: as many census steps per launch as every problem's
    // LDS slice holds (all of them when no slice limits it)
    int ns = 1;
    if (step_form < 0) {
        const int64_t lds_max = (block == 1024) ? kLdsStepsMax : kLdsTallyMax;
        ns = Kmax > 0 ? Kmax : 1;
        for (int j = 0; j < n; ++j)
            while (items[j].gn && ns > 1 && slice_mult(items[j].P) * (int64_t)items[j].gn * ns > lds_max) --ns;
    }
    size_t shmem = 0;
    for (int j = 0; j < n; ++j) {
        const size_t b = (size_t)slice_mult(items[j].P) * items[j].gn * ns * sizeof(double) +
                         (lt_all ? (size_t)items[j].tabs.bytes : 0);
        if (b > shmem) shmem = b;
    }
    std::vector<SegInfo> segs;
    segs.reserve(lay.G);
    for (int j = 0; j < n; ++j)
        for (uint64_t f = 0; f < n_hist[j]; f += seg_len) {
            const uint64_t c = (n_hist[j] - f < seg_len) ? n_hist[j] - f : seg_len;
            segs.push_back(SegInfo{j, (uint32_t)f, (uint32_t)c, 0u});
        }
    if (segs.empty()) segs.push_back(SegInfo{0, 0u, 0u, 0u});
    char *base = (char *)mem;
    BatchItem *d_items = (BatchItem *)(base + lay.items_off);
    SegInfo *d_segs = (SegInfo *)(base + lay.segs_off);
    hipError_t e = hipMemcpyAsync(d_items, items.data(), sizeof(BatchItem) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_segs, segs.data(), sizeof(SegInfo) * segs.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "batched tables");
    void *ctl = base + lay.ctl_off, *bank = base + lay.bank_off;
    const int sf = step_form;
    auto go = [&](auto bs_tag) -> int {
        constexpr int BS = decltype(bs_tag)::value;
        auto one = [&](auto fm_tag, auto lt_tag) -> int {
            constexpr int F = decltype(fm_tag)::value;
            constexpr bool T = decltype(lt_tag)::value;
            if (shmem > 65536) {
                hipError_t ea = hipFuncSetAttribute(
                    reinterpret_cast<const void *>(&k_event<F, false, T, true, MCDC_PROF_EVENTS, true, BS>),
                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
                if (ea != hipSuccess) return hip_fail(ea, "LDS size of the batched multi-step launch");
            }
            return run_batched_steps<F, T, BS>(d_items, d_segs, lay.G, seg_len, Kmax, shmem, bank, ctl, st, sf, ns);
        };
        using I1 = std::integral_constant<int, 1>;
        using I7 = std::integral_constant<int, 7>;
        using I0 = std::integral_constant<int, 0>;
        using BT = std::true_type;
        using BF = std::false_type;
        if (fm == 1) return lt_all ? one(I1{}, BT{}) : one(I1{}, BF{});
        if (fm == 7) return lt_all ? one(I7{}, BT{}) : one(I7{}, BF{});
        return lt_all ? one(I0{}, BT{}) : one(I0{}, BF{});
    };
    if (block == 256) return go(std::integral_constant<int, 256>{});
    if (block == 1024) return go(std::integral_constant<int, 1024>{});
    return go(std::integral_constant<int, kBlock>{});
}

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
    if (p->h.B > 1023 || P.K > 65535) {
        set_error("event form supports at most 1023 batches and 65535 time bins");
        return MCDC_E_UNSUPPORTED;
    }
    LdsTables tabs{};
    const bool lt = table_layout(P, tabs, kLdsTablesMax);
    if (has_progeny(P) || opt.pc_target) {
        if (P.finite_mask == 1) return run_event_lt<1, true>(p, R, first, count, opt, st, prof, tabs, lt);
        if (P.finite_mask == 7) return run_event_lt<7, true>(p, R, first, count, opt, st, prof, tabs, lt);
        return run_event_lt<0, true>(p, R, first, count, opt, st, prof, tabs, lt);
    }
    if (P.finite_mask == 1) return run_event_lt<1, false>(p, R, first, count, opt, st, prof, tabs, lt);
    if (P.finite_mask == 7) return run_event_lt<7, false>(p, R, first, count, opt, st, prof, tabs, lt);
    return run_event_lt<0, false>(p, R, first, count, opt, st, prof, tabs, lt);
}

}  // namespace mcdc
