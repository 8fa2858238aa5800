/*
 * mcdc.h -- C ABI of the MI355X (gfx950) multigroup, time-dependent Monte
 * Carlo particle tracker.
 *
 * The operation is the fixed-source, multigroup, time-dependent neutron
 * transport the paper describes in words (Section 3): multigroup materials
 * (group-wise total cross section, isotropic scattering through a group-to-
 * group transfer matrix), a time-dependent source, time census, and
 * time-dependent mesh tallies scored with the track-length estimator of the
 * time-averaged flux (Section 3.1).  Analog tracking means uniform particle
 * weight and no variance reduction (Section 3.3).  The tracking runs in two
 * forms the paper names (Section 2): history-based (one GPU thread follows
 * one particle to its death) and event-based (the particles of a census
 * step live in a structure-of-arrays bank; by default one launch of the
 * step kernel takes every particle of a bank chunk through its events and
 * across the census edges in registers, refilling idle lanes from the
 * bank, with each wave running queued collisions for many lanes at once;
 * with fewer census steps per launch the crossers of the launch's last
 * edge go to the next bank with wave-ballot appends; with
 * MCDC_FLAG_TWO_KERNEL_STEP an advance kernel sorts the particles into
 * per-event census, surface and collision queues and an events kernel
 * works the queues, one census step at a time).
 *
 * Conventions shared by every entry point
 *  - Units are arbitrary but consistent (length, 1/length, length/time,
 *    time).  Group 0 is the fastest group.
 *  - Every array in a descriptor is copied during the call; the caller may
 *    free it afterwards.  The library never frees caller memory.
 *  - Return value: MCDC_OK (0) or a negative MCDC_E_* code; the message of
 *    the last failure on the calling thread is mcdc_last_error().
 *  - A problem handle is used by one host thread at a time.
 *  - Random numbers: each history i of a run with seed s draws from its own
 *    63-bit linear congruential stream starting at s skipped ahead by
 *    i * 152917 steps, so results depend only on (problem, N, seed), never
 *    on the algorithm, launch shape or GPU.
 */
#ifndef MCDC_H
#define MCDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCDC_ABI_VERSION 6

/* return codes */
#define MCDC_OK 0
#define MCDC_E_INVALID -1     /* bad descriptor or argument (message says which) */
#define MCDC_E_HIP -2         /* a HIP runtime call failed */
#define MCDC_E_NOMEM -3       /* device or host allocation failed */
#define MCDC_E_OVERFLOW -4    /* particle bank, queue or split bank overflowed */
#define MCDC_E_UNSUPPORTED -5 /* valid request this build does not support */

/* boundary conditions of the six domain faces x-, x+, y-, y+, z-, z+ */
#define MCDC_VACUUM 0
#define MCDC_REFLECTIVE 1

/* source kinds and angular laws of a surface source */
#define MCDC_SRC_ISOTROPIC 0 /* volume, plane or point source, isotropic */
#define MCDC_SRC_SURFACE 1   /* enters through a face with the given law */
#define MCDC_MU_BEAM 0       /* mu = 1 */
#define MCDC_MU_UNIFORM 1    /* mu uniform on (0, 1] */
#define MCDC_MU_COSINE 2     /* isotropic incident flux: pdf 2 mu */

/* tracking algorithms */
#define MCDC_ALG_EVENT 0
#define MCDC_ALG_HISTORY 1
#define MCDC_ALG_AUTO 2   /* the faster form, timed on the first call (per history count or batch signature) */

typedef struct mcdc_problem mcdc_problem;

/*
 * Problem descriptor (Section 3: fixed-source transport on box geometry
 * with multigroup physics, time-dependent source and mesh tallies).
 *
 * Materials: sigma_t[M][G] >= 0; sigma_s[M][G][G] >= 0 with row g the
 * outgoing distribution from group g (sum over g' <= sigma_t[m][g]);
 * speed[G] > 0.  A zero sigma_t is a void.
 *
 * Geometry: per axis a (x, y, z) n_planes[a] strictly increasing plane
 * positions planes[a]; n_planes[a] == 0 makes the axis infinite (a 1-D slab
 * has planes only along x).  The outermost planes bound the domain.
 * material[cz][cy][cx] gives the material of each geometry cell (cx runs
 * over n_planes[0]-1 cells, or 1 cell on an infinite axis).  bc[6] are the
 * face conditions.
 *
 * Source: src_kind ISOTROPIC samples position uniformly in the box
 * [src_lo, src_hi] (a degenerate extent is a plane or a point; ignored on
 * infinite axes) and an isotropic direction.  src_kind SURFACE places the
 * particle the same way and gives it direction cosine mu (src_mu_law)
 * about the axis src_axis, pointing along src_sign (+1 or -1), with a
 * uniform azimuth.  Emission time is uniform on [src_t_lo, src_t_hi]; the
 * group is drawn from src_group_pmf[G] (sum 1 within 1e-12).
 *
 * Tally: mesh planes per axis (0 planes = one bin spanning the axis, with
 * width factor 1), strictly increasing and inside the domain; time edges
 * T_0 < ... < T_K (T_K may be +inf; T_0 <= src_t_lo) are both the tally
 * time bins and the census grid; n_batches >= 1 contiguous batches give
 * the variance.  The tally holds the time-averaged scalar flux per source
 * particle, shape [K][G][nz][ny][nx].
 *
 * Detector (optional, qoi_enabled = 1): a box [qoi_lo, qoi_hi] and a group
 * mask qoi_group_mask[G]; its flux is tallied per history so its variance
 * is the history variance (used for the figure of merit).
 *
 * Weight-window mesh (optional): planes per axis (0 = one window cell);
 * the window centres are set with mcdc_set_weight_windows.
 *
 * Time-crossing estimator (optional, time_crossing = 1; Section 3 tallies
 * the flux on a time grid this way in its multigroup pulse verification):
 * the scalar flux at each time edge T_1 .. T_K in the tally's space and
 * group bins, estimated from every particle that reaches the edge alive
 * (score w v_g in the bin of its position at that instant), per source
 * particle and unit bin volume.  Shape [K][G][nz][ny][nx], entry k for
 * edge T_{k+1} (an infinite last edge stays 0).  0 = off.
 *
 * Prompt fission (optional; Section 3's supercritical AZURV1 adds it to
 * the pulse problem): sigma_f[M][G] >= 0 with sum_g' sigma_s + sigma_f <=
 * sigma_t, nu[M][G] in [0, 64] mean neutrons per fission, chi[M][G] >= 0
 * the fission spectrum of each material (sums to 1 within 1e-12).  All
 * three NULL: no fission.  A collision draws one number for the reaction
 * (scatter, fission, capture in that order of the cumulative
 * probabilities); a fission emits floor(nu + xi) neutrons at the collision
 * point and time, neutron 0 continuing the colliding particle, neutrons
 * j >= 1 on the SplitMix64 child streams of its state; each then draws its
 * group from chi, an isotropic direction and an optical depth.  The extra
 * neutrons are tracked like weight-window progeny (split bank, generation
 * by generation after each chunk of histories).
 *
 * Implicit capture (optional, implicit_capture = 1; Section 3 runs the
 * time-dependent dog-leg duct with it): collisions never absorb; the weight
 * is multiplied by sigma_s / sigma_t and, when it falls below roulette_w,
 * one draw keeps the particle with probability w / roulette_ws at weight
 * roulette_ws (else it ends, counted as rouletted); then the scatter draws
 * group, direction and optical depth.  0 < roulette_w <= roulette_ws; not
 * combined with fission; not in batched solves or eigenvalue runs.
 *
 * Cylindrical pins (optional; Section 3's pin cells and cores use
 * quadric-surface geometry): pin_radius[cz][cy][cx] >= 0 over the geometry
 * cells (0 = no pin) and pin_material[cz][cy][cx].  A pin is the cylinder
 * parallel to z centred on its cell's x-y midpoint, radius below half the
 * cell's x and y widths (x and y must be finite axes), filled with its own
 * material; tally, window and detector bins stay those of the box mesh.  A
 * particle carries an inside flag; the distance to the pin surface solves
 * the x-y quadratic (far root from inside, near root from outside when
 * closing in), ties go census, planes, pin, collision, and a pin crossing
 * is a surface event that crosses no plane.  Both NULL: no pins.
 *
 * Moving plane (optional; Section 3 lists time-dependent surfaces for
 * continuous object movement and runs control-rod transients with them):
 * rod_z[K + 1] are the heights of one plane normal to z at the time edges
 * T_0 .. T_K, linear in time in between (Z(t) = Z_k + v_k (t - T_k) on
 * [T_k, T_{k+1}), v_k = (Z_{k+1} - Z_k) / (T_{k+1} - T_k), 0 for an
 * infinite last edge; all finite), and rod_material[cz][cy][cx] over the
 * geometry cells is the material above the plane (-1: the cell keeps its
 * own material on both sides).  In a rod cell a particle carries an above
 * flag, set at birth and on entering a rod cell from a cell that is not one
 * (above iff z > Z(t), or z == Z(t) with the particle rising faster than
 * the plane) and kept between rod cells; the distance to the plane is
 * (Z(t) - z) / (u_z - v_k / v_g) when the two close in; ties go census,
 * planes, moving plane, collision; a crossing is a surface event that
 * crosses no plane and flips the flag.  Needs a finite z axis; not
 * combined with pins; not in eigenvalue runs.  Both NULL: none.
 *
 * Quadric surfaces (optional; Section 3 models its geometry with quadric
 * surfaces; ABI version 6): quadric_coef[cz][cy][cx][10] are the
 * coefficients A B C D E F G H J K of one second-degree surface
 *   Q(x, y, z) = A x^2 + B y^2 + C z^2 + D x y + E y z + F z x
 *                + G x + H y + J z + K
 * per geometry cell (all finite), and quadric_material[cz][cy][cx] the
 * material on its negative side (-1: the cell has none).  Along a flight
 * Q(x + d u) = a d^2 + 2 b d + c.  A particle carries an inside flag (c < 0,
 * or c == 0 with b < 0), set at birth and whenever a plane crossing lands
 * it in another geometry cell (0 where that cell has no quadric).  From
 * inside the distance is the larger root when a > 0 (discriminant clipped
 * at 0), the root (-b + sqrt(b^2 - a c)) / a when a < 0 and b > 0 with a
 * positive discriminant, -c / (2 b) when a == 0 and b > 0; from outside the
 * smaller root when a > 0, b < 0 and the discriminant is positive,
 * (-b - sqrt(b^2 - a c)) / a when a < 0 with a positive discriminant,
 * -c / (2 b) when a == 0 and b < 0; otherwise infinite; negative distances
 * clip at 0.  Ties go census, planes, quadric, collision; a quadric
 * crossing is a surface event that crosses no plane and flips the flag.
 * The surface is not clipped to its cell: the cell's planes bound it.  y or
 * z must be a finite axis (a slab takes none); not combined with pins or a
 * moving plane.  Both NULL: none.
 */
typedef struct {
    int32_t abi_version; /* MCDC_ABI_VERSION */
    int32_t n_groups;
    int32_t n_materials;
    const double *sigma_t;
    const double *sigma_s;
    const double *speed;
    int32_t n_planes[3];
    const double *planes[3];
    const int32_t *material;
    int32_t bc[6];
    int32_t src_kind;
    int32_t src_axis;
    int32_t src_sign;
    int32_t src_mu_law;
    double src_lo[3];
    double src_hi[3];
    double src_t_lo;
    double src_t_hi;
    const double *src_group_pmf;
    int32_t n_mesh_planes[3];
    const double *mesh_planes[3];
    int32_t n_time_edges;
    const double *time_edges;
    int32_t n_batches;
    int32_t qoi_enabled;
    double qoi_lo[3];
    double qoi_hi[3];
    const int32_t *qoi_group_mask;
    int32_t n_ww_planes[3];
    const double *ww_planes[3];
    int32_t time_crossing;
    const double *sigma_f;
    const double *nu;
    const double *chi;
    int32_t implicit_capture;
    double roulette_w;
    double roulette_ws;
    const double *pin_radius;
    const int32_t *pin_material;
    const double *rod_z;
    const int32_t *rod_material;
    const double *quadric_coef;
    const int32_t *quadric_material;
} mcdc_problem_desc;

/*
 * Run options (all-zero = defaults; ABI version 4 added sort_cadence and
 * the sort profile class, version 5 steps_per_launch and pc_method).
 *  algorithm      MCDC_ALG_EVENT (default), MCDC_ALG_HISTORY, or
 *                 MCDC_ALG_AUTO: mcdc_run runs both forms on its first call
 *                 for a history count (results of the history-form run)
 *                 and keeps the faster on the problem handle; batched
 *                 solves keep it per batch signature.
 *  block_size     threads per workgroup.  mcdc_run, event form: the
 *                 census-step kernels' 256, 512 or 1024 (0 = 1024; weighted
 *                 runs and population control take 512 only); the history
 *                 form always uses 256.  mcdc_run_batched: the history
 *                 form's persistent launch 64, 128, 256 or 512, the event
 *                 form's step kernels 256, 512 or 1024 (0 = autotuned).
 *  bank_capacity  event form: particles resident at once (0 = auto).  Work
 *                 is processed in chunks of this many histories.  History
 *                 form with weight windows or fission: histories per chunk
 *                 (0 = auto: 2^23, 2^20 with fission).  Each generation
 *                 of a chunk's progeny (both forms) must fit a split bank
 *                 of 32 (64 with fission) entries per history of the
 *                 chunk, at least 2^22 and at most 2^26, else the run ends
 *                 with MCDC_E_OVERFLOW.  In
 *                 mcdc_run_batched's event form: slots per bank segment.
 *  flags          bit 0 (MCDC_FLAG_EAGER): launch the event form's census
 *                 steps one kernel at a time instead of replaying the
 *                 captured step graphs (graphs are also skipped when a
 *                 profile or debug array is given).
 *                 bit 1 (MCDC_FLAG_TWO_KERNEL_STEP): event form, run each
 *                 census step as an advance kernel (one flight for every
 *                 particle, sorting them into census, surface and
 *                 collision queues) followed by an events kernel, instead
 *                 of the default single kernel that takes every particle
 *                 of the step's bank through its flights to census or
 *                 death with lane refill.  Same results; kept for
 *                 comparison.
 *                 bit 2 (MCDC_FLAG_STAGED): event form on a slab (x the
 *                 only finite axis), analog: the one-kernel step reads
 *                 each refill from tiles of the bank each wave copies into
 *                 LDS one tile ahead (direct-to-LDS loads) instead of
 *                 straight from HBM.  Same results; slower on MI355X,
 *                 kept for comparison.

 *  stream         hipStream_t to run on (NULL = the null stream).  mcdc_run
 *                 synchronises this stream before it returns.
 *  debug_counts   device array [N][5] (census, surface, collision events,
 *                 particles, termination mask per history) or NULL.
 *  debug_scores   device array [N][2] (tallied track and detector score per
 *                 history) or NULL.
 *  profile        host array [MCDC_PROF_CLASSES][4] or NULL.  When given,
 *                 each kernel launch is bracketed by HIP events on the run's
 *                 stream and row c (a MCDC_PROF_* class) receives: total
 *                 device milliseconds, launches, particles processed, and
 *                 algorithmic HBM bytes (the particle-state and queue bytes
 *                 the kernels' loads and stores request, tally atomics
 *                 excluded).  Values are added to what the array holds.
 *  profile_mask   bit c set: bracket launches of class c with events
 *                 (0 = all classes); particle and byte counts are always
 *                 gathered for every class when profile is given.
 *  profile_every, profile_phase
 *                 event form, with profile: time and count only the census
 *                 steps k with k mod profile_every == profile_phase mod
 *                 profile_every (profile_every 0 or 1 = every step); those
 *                 launch one kernel at a time, the others replay the
 *                 captured step graphs uninstrumented.  Runs with phases
 *                 0 .. profile_every-1 together sample every step once.
 *  sort_cadence   event form: 0 = the default (mcdc_run: no queue sort;
 *                 mcdc_run_batched: tuned), -1 = no queue sort.  c >= 1 (at
 *                 most 64) runs the two-kernel step and, at the census steps
 *                 k with k mod c == 0, sorts each segment's surface and
 *                 collision queues by (event, material, group, cell) into a
 *                 fourth bank before the events kernel takes them, so that
 *                 the lanes of a wave start on like events (the per-event
 *                 queues the paper's event-based mode processes, Section 2).
 *                 Same per-history results; tallies differ by summation
 *                 order only.
 *  segments       event form: bank segments, one per workgroup of every
 *                 event kernel (0 = auto: 2 per compute unit, or fewer if
 *                 the advance kernel cannot hold that many resident).
 *                 Results do not depend on it beyond summation order.
 *  pc_target      event form: population control at census (0 = off).  The
 *                 paper lists population control among the time-dependent
 *                 features (Section 2) without a method; this is
 *                 splitting-roulette to pc_target particles at every census
 *                 edge T_k, k < K, over the particles whose clock stands at
 *                 T_k (those that just crossed it and those born in bin k):
 *                 their total weight W is summed exactly (128-bit fixed
 *                 point, 64 fractional bits, each weight truncated to a
 *                 multiple of 2^-64), w_t = W / pc_target, and each of them
 *                 draws xi and goes on as n = floor(w / w_t + xi) copies of
 *                 weight w_t (copy 0 keeps the stream after the draw, copy
 *                 j >= 1 takes the child stream j of it; n = 0 counts as
 *                 rouletted, the extra copies as splits).  The run is one
 *                 bank chunk: n_histories and pc_target <= 2^26.  Not with weight
 *                 windows, fission or a detector, nor in the history form
 *                 (MCDC_E_UNSUPPORTED); MCDC_ALG_AUTO runs the event form.
 *                 The controlled particles are spread evenly over the
 *                 bank segments.  A weight of 2^32 or more, or more
 *                 copies than the banks hold (about n_histories +
 *                 pc_target), ends the run with MCDC_E_OVERFLOW.
 *  steps_per_launch
 *                 mcdc_run, event form, analog one-kernel step: census
 *                 steps s taken per launch of the step kernel (1 .. 65535;
 *                 0 = the default, all K).  With s > 1 a particle that
 *                 reaches the edge T_{k+1} inside the launch's steps
 *                 k0 .. k0+s-1 goes on into time bin k+1 in registers
 *                 instead of through the next bank, and the workgroup's
 *                 LDS slice of the tally holds all s time bins (s is
 *                 lowered until it fits: 4096 doubles, 12288 with
 *                 1024-thread workgroups).  The census edges stay where
 *                 the paper puts them (Section 2): per-history results are
 *                 the same, tallies differ by summation order only.  s > 1
 *                 with weight windows, fission, population control, a
 *                 queue sort, the two-kernel or the staged step is refused
 *                 (MCDC_E_UNSUPPORTED); those take one step per launch.
 *                 mcdc_run_batched ignores the option: its one-kernel form
 *                 takes as many steps per launch as every problem's slice
 *                 holds.  With profile, profile_every and profile_phase
 *                 count launches instead of census steps.
 *  pc_method      with pc_target: MCDC_PC_SPLIT (0, the default) for the
 *                 splitting-roulette above, or MCDC_PC_COMB (1): combing.
 *                 At each edge the same particles as above are taken in
 *                 the run's list order, which depends on nothing but the
 *                 particles' history: it starts with the births in history
 *                 order, a census step keeps every survivor in its place,
 *                 and a control replaces every particle in its place by its
 *                 copies (copy 0 first).  The comb's M = pc_target teeth sit at (u + j) W / M,
 *                 j = 0 .. M-1, with one draw u per edge from the stream
 *                 child_stream(seed, 2^62 + k) of edge T_k, and a particle
 *                 whose stretch [P, P + q) of the cumulative fixed-point
 *                 weight holds n teeth goes on as n copies of weight
 *                 w_t = W / M (copy 0 keeps the stream, copy j >= 1 takes
 *                 child stream j; n = 0 counts as rouletted).  Exactly M
 *                 particles go on at every edge.  The teeth below a point
 *                 x are ceil((X / W) M - u) with X, W the fixed-point sums
 *                 as doubles (hi + (lo >> 32) 2^-32 + (lo mod 2^32) 2^-64),
 *                 clipped to [0, M].  The banks keep the list order (the
 *                 step writes each survivor back to its own slot), so the
 *                 comb is an in-order scan of the fixed-point weights, with
 *                 no sort.  Combing runs the one-kernel step: with the
 *                 two-kernel step or a queue sort it is refused
 *                 (MCDC_E_UNSUPPORTED).
 */
#define MCDC_PC_SPLIT 0
#define MCDC_PC_COMB 1
#define MCDC_FLAG_EAGER 1
#define MCDC_FLAG_TWO_KERNEL_STEP 2
#define MCDC_FLAG_STAGED 4
#define MCDC_PROF_CLASSES 7
#define MCDC_PROF_SOURCE 0     /* event form: source sampling */
#define MCDC_PROF_ADVANCE 1    /* event form: one flight over the census bank */
#define MCDC_PROF_EVENTS 2     /* event form: surface and collision queues, on to census */
#define MCDC_PROF_HISTORY 3    /* history form (and weight-window progeny) */
#define MCDC_PROF_OTHER 4      /* fills, step counters, batch statistics */
#define MCDC_PROF_CONTROL 5    /* event form: population control at census */
#define MCDC_PROF_SORT 6       /* event form: queue sort of the two-kernel step */
typedef struct {
    int32_t algorithm;
    int32_t block_size;
    int64_t bank_capacity;
    int32_t flags;
    void *stream;
    uint32_t *debug_counts;
    double *debug_scores;
    double *profile;
    uint32_t profile_mask;
    int32_t profile_every;
    int32_t profile_phase;
    int32_t segments;
    int32_t sort_cadence;
    uint64_t pc_target;
    int32_t steps_per_launch;
    int32_t pc_method;
} mcdc_run_options;

/*
 * Results.  Array outputs are caller-allocated and are device pointers
 * (hipMalloc or a torch CUDA tensor) unless host_outputs is 1; any may be
 * NULL to skip it.  Scalars are filled on the host.
 *  mean[ntally], var[ntally]   normalised bin flux and its batch variance:
 *                              mean = sum_b S_b / (N V dt), var of the
 *                              batch means m_b = S_b / (N_b V dt).
 *  raw[ntally]                 unnormalised sum of w*d per bin.
 *  leak_mean/leak_var[K][G][6] weight leaked through each face per source
 *                              particle, and its batch variance.
 *  tc_mean[ntally], tc_var[ntally]
 *                              time-crossing flux at the time edges (problems
 *                              with time_crossing = 1; else left untouched):
 *                              mean = sum_b C_b / (N V), variance of the
 *                              batch means C_b / (N_b V).
 *  qoi_sum[2]                  detector sum x and sum x^2 over histories
 *                              (x = the history's track in the detector).
 *  qoi_mean, qoi_var           detector flux per source particle and the
 *                              variance of that mean (history variance).
 *  n_events                    census, surface and collision events.
 *  n_term                      terminations: absorbed, leaked, time cut-off,
 *                              lost (infinite flight), rouletted.
 *  n_splits                    weight-window split progeny created.
 *  n_fission                   fission neutrons beyond the colliding one
 *                              (problems with fission data).
 *  k_mean, k_std               mcdc_run_eigenvalue: k over the active cycles
 *                              and its standard error (else untouched).
 *  kernel_ms                   device time of the run (HIP events).
 */
typedef struct {
    int32_t host_outputs;
    int32_t reserved;
    double *mean;
    double *var;
    double *raw;
    double *leak_mean;
    double *leak_var;
    double qoi_sum[2];
    double qoi_mean;
    double qoi_var;
    uint64_t n_events[3];
    uint64_t n_term[5];
    uint64_t n_splits;
    double kernel_ms;
    double *tc_mean;
    double *tc_var;
    uint64_t n_fission;
    double k_mean;
    double k_std;
} mcdc_result;

/*
 * Validate a descriptor (the problem statement of Section 3: materials,
 * box geometry, source, mesh tallies) and compile it: merge geometry,
 * tally, detector and weight-window planes per axis into one union grid
 * (exact de-duplication),
 * derive the per-cell material/tally tables and the cross-section tables
 * (1/sigma_t, scattering probability, outgoing-group CDF, 1/speed), and
 * upload them to the current HIP device.  *out is owned by the caller and
 * released with mcdc_problem_destroy.  Errors: MCDC_E_INVALID (message
 * names the field), MCDC_E_NOMEM, MCDC_E_HIP.
 */
int mcdc_problem_create(const mcdc_problem_desc *desc, mcdc_problem **out);

/* Release a problem and all device memory it owns.  NULL is a no-op. */
int mcdc_problem_destroy(mcdc_problem *p);

/* Tally shape [K][G][nz][ny][nx] into shape[5]; returns the element count
 * in *ntally if ntally is not NULL. */
int mcdc_problem_tally_shape(const mcdc_problem *p, int64_t shape[5], int64_t *ntally);

/*
 * Track n_histories source particles with the given seed (Section 3
 * fixed-source transport, Section 3.1 track-length tally) and fill *out.
 * opt == NULL means defaults.  Both algorithms give the same per-history
 * event sequence for the same (problem, n_histories, seed); tallies differ
 * only by floating-point summation order.  Errors: MCDC_E_INVALID (NULL
 * problem or result, n_histories == 0, bad option), MCDC_E_OVERFLOW,
 * MCDC_E_NOMEM, MCDC_E_HIP.
 */
int mcdc_run(mcdc_problem *p, uint64_t n_histories, uint64_t seed,
             const mcdc_run_options *opt, mcdc_result *out);

/*
 * Allocation-free run, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as mcdc_run in the history form,
 * and the same kernels; every per-run device buffer (per-batch tally and
 * leakage sums and their copies, detector sums, event counters, overflow
 * flag, the persistent launch's work counter) lives in one static device
 * array of MCDC_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it
 * runs on until the process ends.  The call allocates no device memory;
 * its first call on a device looks up that GPU's copy of the array and
 * creates two timing events.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other threads, or streams not
 * synchronised with each other) race.  Each call clears the part it uses.
 * Requirements: opt->algorithm == MCDC_ALG_HISTORY; out->host_outputs == 0
 * (device output arrays); no debug arrays, profile or population control;
 * an analog problem (no weight windows, fission or implicit capture); a
 * tally that fits: batches x tally doubles x 8 bytes plus the leakage sums
 * within the array (the tally copies per batch are reduced to fit; a
 * 17 x 17 x 10 x 7-group x 20-bin tally with 32 batches, 104 MB, still
 * fits).  Otherwise MCDC_E_UNSUPPORTED with a message naming the limit;
 * other errors as mcdc_run.
 */
#define MCDC_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int mcdc_run_noalloc(mcdc_problem *p, uint64_t n_histories, uint64_t seed, const mcdc_run_options *opt,
                     mcdc_result *out);

/*
 * Batched solve: run n independent problems (any sizes, group counts and
 * history counts) together (Section 2 names both algorithm modes; the
 * batching is this library's).  Problem j runs n_hist[j] histories with
 * seed seeds[j]; outs[j] is filled exactly as mcdc_run would fill it for
 * that problem, and per-history results are identical to separate
 * mcdc_run calls (tallies differ only in summation order).
 *  MCDC_ALG_EVENT (default): every problem's histories are cut into bank
 *    segments of one length; all segments of all problems share one set of
 *    banks, and each census step is one captured graph over all of them,
 *    replayed up to the largest K.  Problems of at most a tail threshold of
 *    histories run instead in one history-form launch after it (the tail
 *    switch).  Launch parameters are forced by the options or tuned on the
 *    first call for a batch signature (problem shapes, history counts and
 *    the forcing options) and reused: the segment length (queue capacity
 *    per workgroup; opt->bank_capacity, 256..2^24, else tuned over {2048,
 *    8192, 32768, 65536}), then the step kernels' workgroup size {256,
 *    512, 1024} (opt->block_size), then the census step's form (one
 *    kernel; two kernels; two kernels with the queue sort every 1, 2, 4 or
 *    8 steps; forced by opt->sort_cadence or MCDC_FLAG_TWO_KERNEL_STEP),
 *    then the tail threshold {0, 2e4, 1e5}, each at the best of the ones
 *    before, timing whole runs of the batch.  At most 2^28 histories and 65535
 *    time bins per problem.
 *  MCDC_ALG_HISTORY: one persistent launch; a fixed grid of workgroups
 *    pulls chunks of histories from one device-wide counter over the
 *    concatenated history ranges; workgroup size and histories per pull are
 *    autotuned the same way (opt->block_size forces a workgroup size).
 *  MCDC_ALG_AUTO: the first call for a batch signature runs both forms
 *    (each tuned as above) and caches the one with the shorter run; later
 *    calls run that form only.  outs hold the results of the last run.
 * opt->debug_counts and opt->debug_scores, if given, hold every problem's
 * per-history records in problem order: problem j's history i is row
 * n_hist[0] + ... + n_hist[j-1] + i of [sum n_hist][5] and [sum n_hist][2].
 * Profiles, weight windows, fission and implicit capture are not supported
 * here (MCDC_E_UNSUPPORTED).  All problems must live on the same device.
 */
int mcdc_run_batched(mcdc_problem *const *ps, int32_t n, const uint64_t *n_hist, const uint64_t *seeds,
                     const mcdc_run_options *opt, mcdc_result *outs);

/*
 * k-eigenvalue power iteration (Section 3 solves its C5G7 pin-cell and
 * core problems as k-eigenvalue cycles; the cycle scheme here is this
 * library's): n_inactive + n_active cycles of n_per_cycle particles on a
 * steady-state problem (time edges [T0, +inf)) with fission data.  Cycle c
 * uses the stream SplitMix64(seed ^ c) (63 bits); particle q starts at it
 * skipped (q + 1) strides.  Cycle 0 starts from the problem's source.  In
 * a cycle a fission ends the particle and banks floor(nu + xi) sites at
 * the collision point; the cycle's M sites, ordered by (particle, site),
 * give the next cycle's sources by a comb: particle q starts at site
 * floor((q + u) M / n_per_cycle) with u the first draw of the cycle's
 * stream, taking its group from the site material's spectrum, an
 * isotropic direction and an optical depth.  k of a cycle = M / n_per_cycle.
 * Outputs: out->mean/var/raw and leak_mean/leak_var over the active cycles
 * (one batch per cycle; per cycle-source particle), event and termination
 * totals over all cycles, out->k_mean and out->k_std (standard error over
 * the active cycles), k of every cycle in the host array
 * k_cycle[n_inactive + n_active] (or NULL), and, as the source diagnostic,
 * the sites of every cycle per spatial tally bin in the host array
 * source_hist[n_inactive + n_active][nz][ny][nx] and their Shannon entropy
 * -sum p log2 p (bits) in entropy[n_inactive + n_active] (either may be
 * NULL; sites outside the mesh are not counted).  n_per_cycle in [1, 2^30],
 * n_active in [1, 1023].  Errors: MCDC_E_INVALID for a problem without
 * fission or not steady state, or a cycle that banks no site;
 * MCDC_E_UNSUPPORTED with weight windows, a detector, debug or profile
 * arrays.  opt->algorithm is not used (one thread per particle).
 */
int mcdc_run_eigenvalue(mcdc_problem *p, uint64_t n_per_cycle, int32_t n_inactive, int32_t n_active,
                        uint64_t seed, const mcdc_run_options *opt, mcdc_result *out, double *k_cycle,
                        uint64_t *source_hist, double *entropy);

/*
 * Set weight-window centres for later runs.  The paper runs analog only
 * (Section 3.3); weight windows are this library's variance reduction,
 * which changes the variance and never the mean.
 * centers[K][G][wz][wy][wx] over the weight-window mesh (0 = no window in
 * that cell); ratio rho > 1 sets
 * the window [2 w_c / (1 + rho), 2 rho w_c / (1 + rho)] with survival weight
 * w_c; a particle above the window splits into min(ceil(w / w_U),
 * max_split) copies.  centers == NULL returns the problem to analog
 * tracking.  The table is copied.
 */
int mcdc_set_weight_windows(mcdc_problem *p, const double *centers, double ratio,
                            int32_t max_split);

/*
 * Weight-window network (no counterpart in the paper): the learned
 * weight-window generator maps a window cell's features (x, y, z scaled to
 * [0, 1], one-hot group, scaled time, zero-padded to 8) to the log10 of an
 * importance (adjoint flux) estimate, from which window centres are formed.  Architecture: 8 -> 64 -> 64 -> 64 -> 1, tanh on the
 * hidden layers, linear output (the only supported widths).  Training is
 * FP32 on matrix cores (weighted mean-squared error, full batch, Adam with
 * beta = (0.9, 0.999), eps = 1e-8); inference rounds weights and
 * activations to bfloat16 with FP32 accumulation.
 *
 * Flat parameter layout, MCDC_MLP_PARAMS floats: W1[8][64], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4[1] (W[k][j] links
 * input k to output j).
 *
 * X[n][8], T[n] (targets), W[n] (sample weights) and Y[n] are device
 * pointers; params and grads are host pointers; stream is a hipStream_t
 * (NULL = null stream).  Each call synchronises its stream before it
 * returns.  Gradients are reduced in a fixed order, so they are
 * reproducible run to run.
 */
#define MCDC_MLP_PARAMS 8961
typedef struct mcdc_mlp mcdc_mlp;

/* widths = {8, 64, 64, 64, 1}, n_layers = 4; Xavier-uniform weights from
 * SplitMix64(seed), zero biases.  Errors: MCDC_E_UNSUPPORTED for other
 * shapes, MCDC_E_NOMEM, MCDC_E_HIP. */
int mcdc_mlp_create(const int32_t *widths, int32_t n_layers, uint64_t seed, mcdc_mlp **out);
int mcdc_mlp_destroy(mcdc_mlp *m);
/* Copy the parameters out / in (setting them also resets Adam's moments). */
int mcdc_mlp_get_params(const mcdc_mlp *m, float *params);
int mcdc_mlp_set_params(mcdc_mlp *m, const float *params);
/* Loss sum_i W_i (y_i - T_i)^2 and its gradient (host grads[MCDC_MLP_PARAMS],
 * may be NULL) at the current parameters. */
int mcdc_mlp_grad(mcdc_mlp *m, const float *X, const float *T, const float *W, int64_t n, float *loss,
                  float *grads, void *stream);
/* steps full-batch Adam steps with learning rate lr; loss_out[steps] (host,
 * may be NULL) receives the loss before each step. */
int mcdc_mlp_train(mcdc_mlp *m, const float *X, const float *T, const float *W, int64_t n, int32_t steps,
                   float lr, float *loss_out, void *stream);
/* BF16 inference: Y[i] = network(X[i]). */
int mcdc_mlp_infer(mcdc_mlp *m, const float *X, int64_t n, float *Y, void *stream);

/* Message of the last failure on the calling thread ("" if none). */
const char *mcdc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCDC_H */
