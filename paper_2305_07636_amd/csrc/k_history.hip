// History-based tracking (the paper's current algorithm, Section 2): one
// thread follows one source particle from birth to death, with the whole
// particle state in registers.  Track-length scores go straight to the
// per-batch tally in HBM through hardware FP64 atomics.
#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

struct BlockCounters {
    unsigned int c[kCounters];
};

template <int FM>
__global__ void __launch_bounds__(256) k_history(DevProblem P, RunArgs R, uint64_t first,
                                                 uint64_t count) {
    __shared__ BlockCounters bc;
    __shared__ double qsum[2];
    if (threadIdx.x < kCounters) bc.c[threadIdx.x] = 0u;
    if (threadIdx.x < 2) qsum[threadIdx.x] = 0.0;
    __syncthreads();

    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned int n_ev[3] = {0u, 0u, 0u};
    unsigned int term_mask = 0u;
    if (r < count) {
        const uint64_t i = first + r;
        const int b = (int)(((i + 1) * (uint64_t)R.B - 1) / R.N);
        double *S = R.S + (int64_t)b * P.ntally;
        Particle p;
        double track = 0.0, qoi = 0.0;
        bool alive = birth<FM>(P, history_stream(P, R.seed, i), p);
        if (!alive) term_mask = 1u << kTime;
        int cell = cell_index(P, p.ix);
        int since = 0;
        while (alive) {
            if (since >= kMaxEventsPerStep) {
                term_mask = 1u << kLost;
                break;
            }
            ++since;
            Flight f = next_event<FM>(P, p, cell);
            if (f.d == kInf) {
                term_mask = 1u << kLost;
                break;
            }
            const double sc = p.w * f.d;
            const int tb = P.cell_tal[cell];
            if (tb >= 0) {
                atomic_add_f64(S + ((int64_t)p.k * P.G + p.g) * P.nts + tb, sc);
                track += sc;
            }
            if (P.qoi_on && P.cell_qoi[cell] && P.qoi_groups[p.g]) qoi += sc;
            move<FM>(P, p, f);
            if (f.ev == kCensus) {
                ++n_ev[0];
                since = 0;
                p.k += 1;
                if (p.k == P.K) {
                    term_mask = 1u << kTime;
                    alive = false;
                }
            } else if (f.ev == kSurface) {
                ++n_ev[1];
                int face = cross<FM>(P, p, f);
                if (face >= 0) {
                    atomic_add_f64(R.L + (((int64_t)b * P.K + p.k) * P.G + p.g) * 6 + face, p.w);
                    term_mask = 1u << kLeak;
                    alive = false;
                } else {
                    cell = cell_index(P, p.ix);
                }
            } else {
                ++n_ev[2];
                if (!collide<FM>(P, p, f.m)) {
                    term_mask = 1u << kAbsorb;
                    alive = false;
                }
            }
        }
        if (R.dbg_counts) {
            uint32_t *d = R.dbg_counts + i * 5;
            d[0] = n_ev[0];
            d[1] = n_ev[1];
            d[2] = n_ev[2];
            d[3] = 1u;
            d[4] = term_mask;
        }
        if (R.dbg_scores) {
            R.dbg_scores[i * 2 + 0] = track;
            R.dbg_scores[i * 2 + 1] = qoi;
        }
        if (P.qoi_on && qoi != 0.0) {
            atomicAdd(&qsum[0], qoi);
            atomicAdd(&qsum[1], qoi * qoi);
        }
        for (int e = 0; e < 3; ++e)
            if (n_ev[e]) atomicAdd(&bc.c[e], n_ev[e]);
        atomicAdd(&bc.c[3 + __builtin_ctz(term_mask)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kCounters && bc.c[threadIdx.x])
        atomicAdd(R.counters + threadIdx.x, (unsigned long long)bc.c[threadIdx.x]);
    if (P.qoi_on && threadIdx.x < 2 && qsum[threadIdx.x] != 0.0)
        atomic_add_f64(R.qoi_sums + threadIdx.x, qsum[threadIdx.x]);
}

}  // namespace

int launch_history(const DevProblem &P, const RunArgs &R, uint64_t first, uint64_t count,
                   int block, hipStream_t st) {
    (void)block;
    const int bs = 256;
    const uint64_t grid = (count + bs - 1) / bs;
    if (grid == 0) return hipSuccess;
    if (P.finite_mask == 1)
        hipLaunchKernelGGL(k_history<1>, dim3((unsigned)grid), dim3(bs), 0, st, P, R, first, count);
    else if (P.finite_mask == 7)
        hipLaunchKernelGGL(k_history<7>, dim3((unsigned)grid), dim3(bs), 0, st, P, R, first, count);
    else
        hipLaunchKernelGGL(k_history<0>, dim3((unsigned)grid), dim3(bs), 0, st, P, R, first, count);
    return (int)hipGetLastError();
}

}  // namespace mcdc
