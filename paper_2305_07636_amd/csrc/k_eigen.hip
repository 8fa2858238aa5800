// k-eigenvalue power iteration (Section 3 runs its pin-cell and core
// problems as k-eigenvalue cycles): cycles of N particles on a steady-state
// problem with fission.  One thread follows one particle of a cycle from
// birth to death with its state in registers.  A fission ends the particle
// and banks floor(nu + xi) sites at the collision point; since a particle
// fissions at most once, its sites are one record (position, cell,
// multiplicity), and an integer prefix sum over the multiplicities orders
// the cycle's M sites by (particle, site) without a sort.  Particle q of
// the next cycle is born at site floor((q + u) M / N) (a comb with offset
// u) and draws its group from the site material's fission spectrum, an
// isotropic direction and an optical depth.  k of a cycle is M / N; flux
// and leakage are tallied in the active cycles, one batch per cycle.
//
// Streams: cycle c uses s_c = SplitMix64(seed ^ c) (63 bits); particle q
// starts at s_c skipped (q + 1) strides; u is the first draw of s_c.
//
// The whole cycle loop is enqueued without host synchronisation: every
// thread of cycle c + 1 reads M from the last prefix sum of cycle c.
#include "k_common.hpp"

namespace mcdc {
namespace {

using namespace dev;

// One cycle's fission-site records, one per particle.
struct Sites {
    double *x;        // [N][3] collision point of the particle's fission
    uint32_t *ixyz;   // [N] its union cell, ix | iy << 11 | iz << 22
    uint32_t *n;      // [N] sites banked there (0: no fission) | inside pin << 31
    uint64_t *cum;    // [N] inclusive prefix sum of n
};

struct EigenCounters {
    unsigned int c[kCounters];
};

template <int FM>
__global__ void __launch_bounds__(256) k_eigen_cycle(DevProblem P, RunArgs R, uint64_t N, uint64_t seed, int cycle,
                                                     int active, int b, Sites prev, Sites cur, int *no_sites,
                                                     unsigned long long *hist) {
    __shared__ EigenCounters bc;
    if (threadIdx.x < kCounters) bc.c[threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) {
        const uint64_t sc = child_stream(seed & kMask63, (uint64_t)cycle);
        Particle p;
        bool alive = true;
        const uint64_t s0 = history_stream(P, sc, q + 1);
        if (cycle == 0) {
            alive = birth<FM>(P, s0, p);
        } else {
            const uint64_t M = prev.cum[N - 1];
            if (M == 0) {
                // the previous cycle banked no site: nothing to start from
                if (q == 0) *no_sites = 1;
                alive = false;
                p.k = 0;
            } else {
                uint64_t su = child_stream(seed & kMask63, (uint64_t)(cycle - 1));
                const double u = rn(su);
                uint64_t idx = (uint64_t)floor(((double)q + u) * (double)M / (double)N);
                if (idx >= M) idx = M - 1;
                uint64_t lo = 0, hi = N - 1;   // first record with cum > idx
                while (lo < hi) {
                    const uint64_t mid = lo + (hi - lo) / 2;
                    if (prev.cum[mid] > idx)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) p.x[a] = prev.x[lo * 3 + a];
                const uint32_t c = prev.ixyz[lo];
                p.ix[0] = c & 2047u;
                p.ix[1] = (c >> 11) & 2047u;
                p.ix[2] = c >> 22;
                p.inpin = (int)(prev.n[lo] >> 31);
                p.t = P.T[0];
                p.w = 1.0;
                p.k = 0;
                p.s = s0;
                fission_emit<FM>(P, p, material_of(P, p, cell_index(P, p.ix)));
            }
        }
        uint32_t n_sites = 0, site_pin = 0;
        int code = kTime;
        unsigned int ev[3] = {0u, 0u, 0u};
        if (alive) {
            int cell = cell_index(P, p.ix);
            int since = 0;
            double *S = active ? tally_copy(P, R, b) : nullptr;
            for (code = -1; code < 0;) {
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
                const int tb = P.cell_tal[cell];
                if (S && tb >= 0) atomic_add_f64(S + ((int64_t)p.k * P.G + p.g) * P.nts + tb, p.w * f.d);
                move<FM>(P, p, f);
                if (f.ev == kSurface) {
                    ++ev[1];
                    const int face = cross<FM>(P, p, crossing_mask<FM>(P, f));
                    if (face >= 0) {
                        if (active) add_leak(P, R, b, p.k, p.g, face, p.w);
                        code = kLeak;
                    } else {
                        cell = cell_index(P, p.ix);
                    }
                } else if (f.ev == kCollision) {
                    ++ev[2];
                    const int m = f.m;
                    const int g = p.g;
                    const int r = collide<FM, true>(P, p, m);
                    if (r == 2) {
                        // bank the sites, end the particle
                        n_sites = (uint32_t)floor(P.nu[(int64_t)m * P.G + g] + rn(p.s));
#pragma unroll
                        for (int a = 0; a < 3; ++a) cur.x[q * 3 + a] = p.x[a];
                        cur.ixyz[q] = (uint32_t)p.ix[0] | ((uint32_t)p.ix[1] << 11) | ((uint32_t)p.ix[2] << 22);
                        site_pin = (uint32_t)p.inpin;
                        // the cycle's sites per spatial tally bin (integer: exact in any order)
                        const int tb = P.cell_tal[cell];
                        if (n_sites && tb >= 0)
                            atomicAdd(hist + (int64_t)cycle * P.nts + tb, (unsigned long long)n_sites);
                        code = kAbsorb;
                    } else if (r == 0) {
                        code = kAbsorb;
                    }
                } else {
                    // a census edge is reached only on a finite last edge,
                    // which an eigenvalue problem does not have
                    ++ev[0];
                    code = kTime;
                }
            }
        }
        cur.n[q] = n_sites | (site_pin << 31);
        if (alive || cycle == 0) {
            atomicAdd(&bc.c[3 + code], 1u);
            for (int e = 0; e < 3; ++e)
                if (ev[e]) atomicAdd(&bc.c[e], ev[e]);
        }
    }
    __syncthreads();
    if (threadIdx.x < kCounters && bc.c[threadIdx.x])
        atomicAdd(R.counters + threadIdx.x, (unsigned long long)bc.c[threadIdx.x]);
}

// Inclusive prefix sum of the site counts in three passes: per block of
// 1024, over the block totals (one workgroup, in order), then the block
// offsets added back.  Integer arithmetic: the result is exact.
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(const uint32_t *__restrict__ in, uint64_t *out,
                                                            uint64_t *totals, uint64_t n) {
    __shared__ uint64_t buf[kScanBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
    buf[threadIdx.x] = (i < n) ? (uint64_t)(in[i] & 0x7FFFFFFFu) : 0ull;   // (bit 31: pin flag)
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const uint64_t v = (threadIdx.x >= (unsigned)off) ? buf[threadIdx.x - off] : 0ull;
        __syncthreads();
        buf[threadIdx.x] += v;
        __syncthreads();
    }
    if (i < n) out[i] = buf[threadIdx.x];
    if (threadIdx.x == kScanBlock - 1) totals[blockIdx.x] = buf[kScanBlock - 1];
}

__global__ void __launch_bounds__(kScanBlock) k_scan_totals(uint64_t *totals, uint64_t nb) {
    __shared__ uint64_t buf[kScanBlock];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0ull;
    __syncthreads();
    for (uint64_t base = 0; base < nb; base += kScanBlock) {
        const uint64_t i = base + threadIdx.x;
        buf[threadIdx.x] = (i < nb) ? totals[i] : 0ull;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            const uint64_t v = (threadIdx.x >= (unsigned)off) ? buf[threadIdx.x - off] : 0ull;
            __syncthreads();
            buf[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < nb) totals[i] = buf[threadIdx.x] + carry;
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[kScanBlock - 1];
        __syncthreads();
    }
}

__global__ void k_scan_add(uint64_t *out, const uint64_t *__restrict__ totals, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t blk = i / kScanBlock;
    if (i < n && blk > 0) out[i] += totals[blk - 1];
}

// M of the cycle into the per-cycle record.
__global__ void k_store_sites(const uint64_t *cum, uint64_t n, uint64_t *m_out) { *m_out = cum[n - 1]; }

size_t pad(size_t b) { return (b + 255) & ~size_t(255); }

Sites carve_sites(char *&p, uint64_t N) {
    Sites s;
    s.x = (double *)p;
    p += pad(N * 3 * sizeof(double));
    s.ixyz = (uint32_t *)p;
    p += pad(N * sizeof(uint32_t));
    s.n = (uint32_t *)p;
    p += pad(N * sizeof(uint32_t));
    s.cum = (uint64_t *)p;
    p += pad(N * sizeof(uint64_t));
    return s;
}

template <int FM>
int run_eigen(const DevProblem &P, const RunArgs &R, uint64_t N, int n_inactive, int n_active, uint64_t seed,
              void *mem, uint64_t *m_dev, int *no_sites, unsigned long long *hist, hipStream_t st) {
    char *p = (char *)mem;
    Sites s[2] = {carve_sites(p, N), carve_sites(p, N)};
    uint64_t *totals = (uint64_t *)p;
    const uint64_t nb = (N + kScanBlock - 1) / kScanBlock;
    const unsigned grid = (unsigned)((N + 255) / 256);
    for (int c = 0; c < n_inactive + n_active; ++c) {
        const Sites &prev = s[(c + 1) & 1], &cur = s[c & 1];
        const int active = c >= n_inactive;
        hipLaunchKernelGGL(k_eigen_cycle<FM>, dim3(grid), dim3(256), 0, st, P, R, N, seed, c, active,
                           active ? c - n_inactive : 0, prev, cur, no_sites, hist);
        hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanBlock), 0, st, (const uint32_t *)cur.n,
                           cur.cum, totals, N);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, st, totals, nb);
        hipLaunchKernelGGL(k_scan_add, dim3(grid), dim3(256), 0, st, cur.cum, (const uint64_t *)totals, N);
        hipLaunchKernelGGL(k_store_sites, dim3(1), dim3(1), 0, st, (const uint64_t *)cur.cum, N, m_dev + c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "eigenvalue cycle launch");
    }
    return MCDC_OK;
}

}  // namespace

size_t eigen_bytes(uint64_t N) {
    return 2 * (pad(N * 3 * sizeof(double)) + 2 * pad(N * sizeof(uint32_t)) + pad(N * sizeof(uint64_t))) +
           pad(((N + kScanBlock - 1) / kScanBlock) * sizeof(uint64_t));
}

int launch_eigen(const DevProblem &P, const RunArgs &R, uint64_t N, int n_inactive, int n_active, uint64_t seed,
                 void *mem, uint64_t *m_dev, int *no_sites, unsigned long long *hist, hipStream_t st) {
    if (P.finite_mask == 1) return run_eigen<1>(P, R, N, n_inactive, n_active, seed, mem, m_dev, no_sites, hist, st);
    if (P.finite_mask == 7) return run_eigen<7>(P, R, N, n_inactive, n_active, seed, mem, m_dev, no_sites, hist, st);
    return run_eigen<0>(P, R, N, n_inactive, n_active, seed, mem, m_dev, no_sites, hist, st);
}

}  // namespace mcdc
