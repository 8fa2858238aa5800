// Internal types of the MI355X tracker library: the compiled problem that
// kernels receive by value, the per-run arguments, and the launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mcdc.h"

namespace mcdc {

constexpr int kMaxGroups = 32;      // outgoing-group search is unrolled over this
constexpr int kCounters = 10;       // census, surface, collision; 5 terminations; splits; fission progeny
constexpr int kLdsTallyMax = 4096;  // doubles of the event form's per-step LDS tally slice
constexpr int kMaxChunkStreams = 4;   // weighted bank chunks in flight at once, at most
constexpr uint64_t kWindowChunk = 1ULL << 23;  // histories per chunk of a weight-window run
constexpr uint64_t kFissionChunk = 1ULL << 20; // histories per chunk of a run with fission
constexpr double kMaxNu = 64.0;                // largest mean number of neutrons per fission
constexpr uint64_t kStride = 152917ULL;

enum Term : int { kAbsorb = 0, kLeak = 1, kTime = 2, kLost = 3, kRoulette = 4 };

// Compiled problem: device pointers to the read-only tables plus scalars.
// Passed to every kernel by value (well under the kernel-argument limit).
struct DevProblem {
    int G, M, K;
    int nU[3];             // union planes per axis (0 = infinite axis)
    int nc[3];             // union cells per axis (1 on an infinite axis)
    int finite_mask;       // bit a set if axis a is finite
    int ncells;            // nc[0] * nc[1] * nc[2]
    int nts;               // tally spatial bins nz * ny * nx
    int64_t ntally;        // K * G * nts
    int tc_on;             // 1: time-crossing tally at the edges T_1..T_K as well
    int64_t tstride;       // doubles per tally copy: the track-length tally, then
                           // the time-crossing tally (entry k for edge T_{k+1})
    const double *U[3];    // union planes
    const int32_t *cell_mat;   // [ncells] material of each union cell
    const int32_t *cell_tal;   // [ncells] spatial tally bin, -1 outside the mesh
    const int32_t *cell_ww;    // [ncells] weight-window cell, -1 outside
    const uint8_t *cell_qoi;   // [ncells] 1 inside the detector box
    const double *sigma_t;     // [M][G]
    const double *inv_st;      // [M][G] 1 / sigma_t (0 for a void)
    const double *ps;          // [M][G] sigma_s,g / sigma_t,g
    const double *cdf;         // [M][G][G] outgoing-group CDF
    const double *speed;       // [G]
    const double *inv_v;       // [G] 1 / speed
    const double *T;           // [K + 1] census / time-bin edges
    const double *src_cdf;     // [G]
    const uint8_t *qoi_groups; // [G]
    const uint64_t *skipA;     // [64] LCG map for stride * 2^j steps: s -> A s + C
    const uint64_t *skipC;     // [64]
    const double *bin_norm;    // [nts] tally-bin volume (product of bin widths)
    const double *time_norm;   // [K] time-bin width (1 for an infinite bin)
    int bc[6];
    int src_kind, src_axis, src_mu_law;
    double src_sign;
    double src_lo[3], src_hi[3], src_t_lo, src_t_hi;
    int qoi_on;
    // weight windows
    const double *ww_center;   // [K][G][nww] or nullptr (analog)
    int nww;
    int ww_max_split;
    double ww_ratio;
    // prompt fission (fission_on = 0: none)
    int fission_on;
    const double *pf;          // [M][G] (sigma_s,g + sigma_f,g) / sigma_t,g
    const double *nu;          // [M][G] mean neutrons per fission
    const double *chi_cdf;     // [M][G] fission-spectrum CDF
    // implicit capture with weight roulette (implicit = 0: analog collisions)
    int implicit;
    double roulette_w, roulette_ws;   // threshold, survival weight
    // cylindrical pins parallel to z, per union cell (pins_on = 0: none)
    int pins_on;
    const double *pin_r2;      // [ncells] squared radius of the cell's pin, 0 = none
    const double *pin_xc;      // [ncells] its centre (the geometry cell's x-y midpoint)
    const double *pin_yc;
    const int32_t *pin_mat;    // [ncells] material inside it
    // moving plane normal to z (rod_on = 0: none; never with pins)
    int rod_on;
    const double *rod_z;       // [K + 1] heights at the time edges
    const double *rod_v;       // [K] speed in each census step
    const int32_t *rod_mat;    // [ncells] material above the plane, -1 = not a rod cell
    // quadric surfaces, one per geometry cell (quad_on = 0: none; never with
    // pins or a moving plane)
    int quad_on;
    const int32_t *quad_cell;  // [ncells] the quadric of the cell's geometry cell, -1 = none
    const double *quad_coef;   // [nq][10] A B C D E F G H J K
    const int32_t *quad_mat;   // [ncells] material on the quadric's negative side
};

// Runs whose particles make progeny (window splits, fission neutrons) or
// carry weights (implicit capture) take the kernels' weighted form: weights
// in the banks, split bank, per-history detector scores.
__host__ __device__ inline bool has_progeny(const DevProblem &P) {
    return P.ww_center != nullptr || P.fission_on != 0 || P.implicit != 0;
}

// Doubles per bin of the event form's per-step LDS slice: two batches of
// the track-length tally, and two of the time-crossing tally when it is on.
__host__ __device__ inline int slice_mult(const DevProblem &P) { return P.tc_on ? 4 : 2; }

// Per-launch arguments shared by the tracking kernels.
struct RunArgs {
    uint64_t N;          // histories in the whole run (sets the batch partition)
    uint64_t seed;       // base LCG state (masked to 63 bits)
    int B;               // batches
    int X;               // tally copies per batch (power of two): workgroup w adds into copy w mod X
    double *S;           // [B][X][tstride] raw track-length (and time-crossing) sums per batch and copy
    int XL;              // leakage copies per batch (power of two), as X
    double *L;           // [B][XL][K][G][6] leaked weight per batch and copy
    double *qoi_hist;    // [chunk] per-history detector score (WW runs) or nullptr
    double *qoi_sums;    // [2] sum x, sum x^2
    unsigned long long *counters;  // [kCounters]
    uint32_t *dbg_counts;          // [N][5] or nullptr
    double *dbg_scores;            // [N][2] or nullptr
    int *overflow;                 // set to 1 when a bank overflows
    unsigned long long *prof;      // [MCDC_PROF_CLASSES][2] particles, bytes; or nullptr
    unsigned long long *work;      // history form: the persistent launch's work counter, or
                                   // nullptr (the launcher then uses the problem's own buffer)
};

// Read-only tables the event kernels stage in LDS: byte offsets (behind
// the tally slice) and element counts per table.
enum TabId : int { kTU0, kTU1, kTU2, kTT, kTSt, kTISt, kTPs, kTCdf, kTV, kTIV, kTMat, kTTal, kTabs };
struct LdsTables {
    int off[kTabs];
    int count[kTabs];
    int bytes;
};

// One problem of a batched solve (device array element).
struct BatchItem {
    DevProblem P;
    RunArgs R;
    LdsTables tabs;   // event form: staged-table layout
    int gn;           // event form: G * nts of the LDS tally slice, 0 = none
};

// One bank segment of the batched event form: problem, and the histories
// [first, first + count) of that problem it is born with.
struct SegInfo {
    int prob;
    uint32_t first, count;
    uint32_t pad;
};

// Host-side launch profiler: HIP events around each launch of a class.
struct Profiler {
    double *out = nullptr;             // host [classes][4] or nullptr
    unsigned int mask = 0;             // classes to time (0 = all)
    hipStream_t st = nullptr;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    int cls = -1;
    hipEvent_t open = nullptr;
    bool wants(int c) const { return out && (!mask || ((mask >> c) & 1u)); }
    void begin(int c);                 // event pair around launches made in between
    void end();
    hipEvent_t take();                 // an event from the reuse pool (nullptr on failure)
    void give(hipEvent_t e);           // back to the pool
    void add(int c, hipEvent_t a, hipEvent_t b) { marks.push_back({c, {a, b}}); }
    int finish();                      // synchronise, accumulate, return events to the pool
};

// Launch a kernel; when the profiler times class cls the launch carries a
// start / stop event pair that the runtime stamps at the kernel's own start
// and end (no marker packets around the dispatch).
template <typename F, typename... Args>
void launch_timed(Profiler &pr, int cls, F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                  Args... args) {
    if (pr.wants(cls)) {
        hipEvent_t a = pr.take(), b = pr.take();
        if (a && b) {
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0u, args...);
            pr.add(cls, a, b);
            return;
        }
        if (a) pr.give(a);
        if (b) pr.give(b);
    }
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// Host-side compiled problem (owns the device blob).
struct HostProblem {
    int G = 0, M = 0, K = 0, B = 0;
    std::vector<double> U[3];
    int nc[3] = {1, 1, 1};
    int nt[3] = {1, 1, 1};     // tally bins per axis
    int nw[3] = {1, 1, 1};     // window cells per axis
    std::vector<int32_t> cell_mat, cell_tal, cell_ww;
    std::vector<uint8_t> cell_qoi;
    std::vector<double> sigma_t, inv_st, ps, cdf, speed, inv_v, T, src_cdf;
    bool fission = false;
    std::vector<double> pf, nu, chi_cdf;   // [M][G] each (fission only)
    bool pins = false;
    std::vector<double> pin_r2, pin_xc, pin_yc;   // [ncells] (pins only)
    std::vector<int32_t> pin_mat;
    bool rod = false;
    std::vector<double> rod_z, rod_v;  // [K + 1], [K] (moving plane only)
    std::vector<int32_t> rod_mat;      // [ncells]
    bool quad = false;
    std::vector<int32_t> quad_cell, quad_mat;  // [ncells] (quadrics only)
    std::vector<double> quad_coef;             // [nq][10]
    std::vector<uint8_t> qoi_groups;
    std::vector<double> bin_norm;      // [nts] V_j (product of bin widths)
    std::vector<double> time_norm;     // [K] dt_k (1 if infinite)
    double qoi_volume = 1.0;
    mcdc_problem_desc desc{};          // scalars of the descriptor
};

}  // namespace mcdc

// The opaque handle of the C ABI.
struct mcdc_problem {
    mcdc::HostProblem h;
    mcdc::DevProblem d{};
    int device = 0;
    void *blob = nullptr;          // device tables
    size_t blob_bytes = 0;
    // weight windows
    double *ww_dev = nullptr;
    std::vector<double> ww_host;
    // work buffers, grown on demand and reused across runs
    struct Buf {
        void *p = nullptr;
        size_t bytes = 0;
    };
    Buf S, L, qoi_hist, qoi_sums, counters, overflow, bank, queues, prof, counters_split, tally_part, work, comb;
    Buf split[mcdc::kMaxChunkStreams];   // each chunk stream's pair of split banks (one allocation each)
    Buf mean, var, raw, leak_mean, leak_var, tc_mean, tc_var;
    void *graph_cache = nullptr;   // captured census steps of the event form
    // weighted history-form runs: a second stream (default priority) and
    // events for overlapping bank chunks, pinned host words for their
    // generation counts
    void *aux_streams[mcdc::kMaxChunkStreams - 1] = {};   // weighted chunks: streams beside the caller's
    void *aux_events[2 * mcdc::kMaxChunkStreams] = {};   // per stream: batch done, join
    unsigned long long *host_counts = nullptr;      // [kMaxChunkStreams]
    // MCDC_ALG_AUTO: the faster form for one history count, once timed
    uint64_t auto_n = 0;
    int auto_alg = -1;
};

namespace mcdc {

void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);
int ensure(mcdc_problem::Buf &b, size_t bytes);

// launchers (return a hipError_t as int)
// Allocates beforehand the device memory a history-form run of `count`
// histories will take (the weighted runs' split banks), so that a run's
// timed region holds no allocation.
int history_reserve(mcdc_problem *p, uint64_t count, uint64_t chunk_opt);
int launch_history(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count,
                   uint64_t chunk, hipStream_t st, Profiler &prof);
int launch_event(mcdc_problem *p, const RunArgs &R, uint64_t first, uint64_t count,
                 const mcdc_run_options &opt, hipStream_t st, Profiler &prof);
// (sums the tally and leakage copies into copy 0 first, in place)
int launch_fold(const DevProblem &P, double *S, double *L, int B, int X, int XL, uint64_t N,
                const double *bin_norm_dev, const double *time_norm_dev, double *mean,
                double *var, double *raw, double *leak_mean, double *leak_var,
                double *tc_mean, double *tc_var, hipStream_t st);
int launch_zero(void *p, size_t bytes, hipStream_t st);
// Run-level steps shared by mcdc_run and its allocation-free variant
// (run.cpp): batch statistics into the result's arrays, and the host copies
// of counters and detector sums (begin before, end after the stream is
// synchronised).
struct Collect {
    unsigned long long cnt[kCounters];
    double qs[2];
    int ovf;
};
int fold(mcdc_problem *p, const RunArgs &R, mcdc_result *out, hipStream_t st, Profiler &prof);
int collect_begin(mcdc_problem *p, const RunArgs &R, mcdc_result *out, Collect &c, hipStream_t st);
int collect_end(mcdc_problem *p, uint64_t N, const Collect &c, mcdc_result *out, double ms);
void destroy_graph_cache(mcdc_problem *p);
int launch_batched(const BatchItem *items, const uint64_t *offs, int n_items, uint64_t total,
                   unsigned long long *next, int finite_mask, int block, int per_thread, hipStream_t st);
int launch_qoi_reduce(const double *qoi_hist, uint64_t n, double *qoi_sums, hipStream_t st);
// Batched event form (k_event.hip): device memory it needs for segments of
// seg_len slots, and the run itself (items hold each problem's DevProblem
// and prepared RunArgs; the launcher fills their table layouts).
// step_form < 0: one kernel per census step; 0: the two-kernel step; c >= 1:
// the two-kernel step with the queue sort at every c-th census step.
size_t event_batched_bytes(const uint64_t *n_hist, int n, unsigned int seg_len, int step_form);
// k-eigenvalue cycles (k_eigen.hip): device memory for N particles per
// cycle, and the cycle loop (M of every cycle into m_dev[cycles]; the
// sites of every cycle per spatial tally bin added into hist[cycles][nts];
// *no_sites set if a cycle banked no site).
size_t eigen_bytes(uint64_t N);
int launch_eigen(const DevProblem &P, const RunArgs &R, uint64_t N, int n_inactive, int n_active, uint64_t seed,
                 void *mem, uint64_t *m_dev, int *no_sites, unsigned long long *hist, hipStream_t st);
// (block: the step kernels' workgroup size, 256, 512 or 1024)
int launch_event_batched(std::vector<BatchItem> &items, const uint64_t *n_hist, unsigned int seg_len, void *mem,
                         size_t mem_bytes, hipStream_t st, int step_form, int block);

}  // namespace mcdc
