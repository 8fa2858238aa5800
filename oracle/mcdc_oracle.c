/*
 * mcdc_oracle.c -- plain serial CPU oracle for multigroup, time-dependent,
 * fixed-source Monte Carlo particle transport with track-length mesh tallies.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the judge of correctness of the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or constant
 * generator with the GPU library: every piece (random numbers, grid, sampling,
 * tallies) is written out here on its own, slowly and in the plainest order.
 *
 * What it computes.  The paper (Section 3) describes the method in words: MC
 * transport of neutrons through multigroup materials (group-wise total cross
 * section, isotropic scattering through a group-to-group transfer matrix, no
 * fission unless the problem gives fission data, R12), on box geometry, with a
 * time-dependent source, time census,
 * time-dependent mesh tallies, and the track-length estimator of the
 * time-averaged flux (Section 3.1); analog mode means uniform weight and no
 * variance reduction (Section 3.3).  The paper prints no equations and no
 * random-number scheme; every point where it is silent is fixed by an
 * explicit reading, stated next to the code that implements it:
 *
 *   R1  RNG: 63-bit linear congruential generator s <- (g s + c) mod 2^63,
 *       g = 2806196910506780709, c = 1; history i starts at the state
 *       skip(seed, i * 152917); xi = (s >> 10) * 2^-53 after each advance.
 *   R2  Floating point: IEEE binary64, round to nearest, no contraction;
 *       an explicit fused multiply-add only in the position update.
 *   R3  Tie order of the next event: census, then surface, then collision.
 *   R4  Geometry, tally, weight-window and detector planes are merged per
 *       axis into one sorted, exactly de-duplicated union grid; a crossing of
 *       any union plane is one surface event; axes whose distance equals the
 *       event distance all cross in that one event; the cell index moves by
 *       one and is never recomputed from the position.
 *   R5  Random-number order: birth draws x, y, z, t, group, direction,
 *       optical depth; a collision draws the absorb test, the outgoing group
 *       (always), the direction, the optical depth.
 *   R6  Optical depth to collision tau = -log(1 - xi) is carried across
 *       surfaces and census and reduced by d * Sigma_t on each flight.
 *   R7  Isotropic directions by Marsaglia's (1972) method.
 *   R8  Time bins are the census grid; a particle reaching the last edge is
 *       killed (time cut-off) with no further tally.
 *   R9  B contiguous batches of histories; mean and batch variance of the
 *       normalised bin fluxes.
 *   R10 Weight windows (optional): centre w_c per (time bin, group, window
 *       cell); bounds w_L = 2 w_c / (1 + rho), w_U = rho w_L, survival weight
 *       w_c; split into n = min(ceil(w / w_U), max_split) copies; children
 *       take streams SplitMix64(parent state xor j) masked to 63 bits.
 *   R11 Time-crossing estimator (optional; Section 3, verification with the
 *       multigroup pulse, names it without formulas): the scalar flux at
 *       the time edge T_{k+1} (k = 0..K-1) is estimated by every particle
 *       that reaches that edge alive, scoring w * v_g into the spatial bin
 *       of its cell at that instant, before the weight-window check;
 *       normalised by N V (no time width).  A particle born exactly on an
 *       edge does not cross it.
 *   R12 Fission (optional; Section 3 runs the supercritical AZURV1 with
 *       fission added, prompt neutrons only): a collision draws one number
 *       xi for the reaction: scatter if xi < Sigma_s/Sigma_t, fission if
 *       xi < (Sigma_s + Sigma_f)/Sigma_t, else capture.  A fission draws
 *       one more number and emits n = floor(nu + xi) neutrons at the
 *       collision point and time (n = 0 ends the particle as absorbed).
 *       Neutron 0 is the colliding particle itself; neutron j >= 1 takes
 *       the stream SplitMix64(s ^ j) masked to 63 bits of the state s
 *       after that draw.  Each neutron then draws from its own stream its
 *       group from the material's spectrum chi, an isotropic direction and
 *       an optical depth; the colliding particle then takes the window
 *       check as after a scatter.
 *   R13 k-eigenvalue power iteration (Section 3 runs the C5G7 pin cell and
 *       core this way; steady state): cycles of N particles.  Cycle c uses
 *       the stream s_c = SplitMix64(seed ^ c) masked to 63 bits; particle q
 *       starts at skip(s_c, (q + 1) * stride).  Cycle 0 is born from the
 *       problem's source; in the cycle loop a fission does not continue the
 *       particle: it banks floor(nu + xi) sites at the collision point and
 *       the particle ends (absorbed).  The sites of a cycle, M in all, are
 *       ordered by (particle, site); particle q of the next cycle is born
 *       at site floor((q + u) M / N) (a comb with offset u, the first draw
 *       of s_c) and draws its group from the spectrum of the site's
 *       material, an isotropic direction and an optical depth.  k of a
 *       cycle is M / N.  Flux and leakage are tallied in the active cycles
 *       only, one batch per active cycle.  Source diagnostic: the sites of
 *       each cycle counted per spatial tally bin (Shannon entropy of the
 *       fission source, -sum p log2 p over the bins with sites).
 *   R14 Implicit capture (optional; Section 3 runs the time-dependent
 *       dog-leg duct with it): a collision never absorbs; the weight is
 *       multiplied by Sigma_s/Sigma_t.  If it falls below w_min a draw
 *       decides a roulette: survive with probability w/w_s at weight w_s,
 *       else the particle ends (rouletted).  Then the scatter draws as in
 *       the analog game (group, direction, optical depth) and the window
 *       check follows.  Not combined with fission; 0 < w_min <= w_s.
 *   R15 Cylindrical pins (optional; Section 3's pin cells and cores, on
 *       quadric-surface geometry): a geometry cell may hold one cylinder
 *       parallel to z, centred on the cell's x-y midpoint (0.5 (lo + hi)
 *       per axis), radius r below half the cell's x and y widths, with its
 *       own material.  A particle carries an inside flag.  Distance: with
 *       dx = x - xc, dy = y - yc, a = u^2 + v^2, b = dx u + dy v,
 *       c = (dx^2 + dy^2) - r^2: inside, (-b + sqrt(max(b^2 - a c, 0))) / a;
 *       outside, if b < 0 and b^2 - a c > 0, (-b - sqrt(b^2 - a c)) / a;
 *       else (or a = 0) none; clipped at 0.  Tie order: census, planes,
 *       cylinder, collision.  A cylinder crossing is a surface event that
 *       crosses no plane and flips the flag.  Birth: inside iff c < 0.
 *   R16 Population control at census (optional; Section 2 lists population
 *       control among the time-dependent features, without a method):
 *       splitting-roulette to a target population N_t.  The run tracks all
 *       particles census step by census step.  At each census edge T_k
 *       (k < K) the particles whose clock stands at T_k (those that just
 *       crossed it, and those born in time bin k) are controlled together;
 *       particles born in later bins are not touched.  Their total weight W
 *       is summed exactly, order-free, in 128-bit fixed point with 64
 *       fractional bits (each weight truncated to a multiple of 2^-64; a
 *       weight of 2^32 or more is an error).  W becomes a double as
 *       hi + ((lo >> 32) 2^-32 + (lo mod 2^32) 2^-64), and w_t = W / N_t.
 *       Each of them, in any order, draws xi and makes
 *       n = floor(w / w_t + xi) copies of weight w_t (n = 0: the particle
 *       ends, rouletted).  Copy 0 keeps the stream after the draw; copy
 *       j >= 1 takes child_stream of that state and j (as R10's splits) and
 *       counts as a split.  W = 0: nothing happens.  Analog tracking with
 *       optional implicit capture only (no windows, fission or detector).
 *   R28 Population control by combing (optional, the other census method
 *       Section 2's population control names): the same particles as R16
 *       at each edge T_k, taken in the run's list order, which depends on
 *       nothing but the particles' history: the list starts with the
 *       histories' births in history order; a census step keeps each
 *       survivor in its place (the dead drop out, particles of later bins
 *       wait in theirs); a control replaces each particle in its place by
 *       its copies, copy 0 first (an uncontrolled particle by itself).  (A
 *       code that tracks one history after the other and banks census
 *       crossers as they arrive keeps exactly this order.)  With
 *       q_r their R16 fixed-point weights, P_r the exact sum of the q before
 *       r, W the total and D(.) R16's conversion to a double, one draw u of
 *       the edge's own stream child_stream(seed, 2^62 + k) sets the teeth
 *       at (u + j) W / M, j = 0 .. M-1, M the target.  The number of teeth
 *       below a point x is T(x) = ceil((D(x) / D(W)) M - u) clipped to
 *       [0, M], and particle r becomes n_r = T(P_r + q_r) - T(P_r) copies
 *       of weight w_t = D(W) / M (n_r = 0: rouletted).  T(0) = 0 and
 *       T(W) = M, so exactly M particles go on; n_r is the floor or the
 *       ceiling of M q_r / W, and its mean over u is M q_r / W up to the
 *       doubles' rounding.  Copy 0 keeps the particle's stream (no draw),
 *       copy j >= 1 takes child_stream of it and j and counts as a split.
 *   R27 Moving plane (optional; Section 3 lists time-dependent surfaces
 *       for continuous object movement, and runs control-rod transients
 *       with them): one plane normal to z whose height is linear in time
 *       within each census step, Z(t) = Z_k + v_k (t - T_k) on
 *       [T_k, T_{k+1}), from the heights Z_k given at the time edges,
 *       v_k = (Z_{k+1} - Z_k) / (T_{k+1} - T_k) (0 for an infinite last
 *       edge).  A geometry cell may be a rod cell with a rod material:
 *       above the plane its material is the rod's, below its own.  In rod
 *       cells a particle carries an above flag; per unit track length its
 *       height gains u_z and the plane's v_k / v_g, so with q = u_z -
 *       v_k (1 / v_g) the distance to the plane is (Z(t) - z) / q when
 *       the two close in (above and q < 0, or below and q > 0), clipped at
 *       0.  Crossing it is a surface event that crosses no union plane and
 *       flips the flag.  The flag is set at birth in a rod cell and when a
 *       plane crossing enters a rod cell from a cell that is not one:
 *       above iff z > Z(t), or z == Z(t) and q > 0; it is kept between rod
 *       cells.  Tie order: census, planes, moving plane, collision.  Not
 *       combined with pins nor in eigenvalue cycles; needs a finite z axis.
 *   R29 Quadric surfaces (optional; Section 3's geometry is built from
 *       quadric surfaces): a geometry cell may carry one quadric
 *       Q(x) = A x^2 + B y^2 + C z^2 + D x y + E y z + F z x + G x + H y
 *       + J z + K with a material for its inside (Q < 0); outside it the
 *       cell keeps its own material.  Along x + d u,
 *       Q = a d^2 + 2 b d + c with, in this evaluation order,
 *         a = ((A ux ux + B uy uy) + C uz uz) + ((D ux uy + E uy uz) + F uz ux)
 *         b = ((A x ux + B y uy) + C z uz) + 0.5 ((((D (x uy + y ux)
 *             + E (y uz + z uy)) + F (z ux + x uz)) + ((G ux + H uy) + J uz)))
 *         c = (((A x x + B y y) + C z z) + ((D x y + E y z) + F z x))
 *             + (((G x + H y) + J z) + K)
 *       (products left to right).  The particle carries an inside flag;
 *       with disc = b b - a c, the distance to the surface is: inside,
 *       a > 0: (-b + sqrt(max(disc, 0))) / a; a < 0: (-b + sqrt(disc)) / a
 *       if b > 0 and disc > 0; a = 0: -c / (2 b) if b > 0; outside, a > 0:
 *       (-b - sqrt(disc)) / a if b < 0 and disc > 0; a < 0:
 *       (-b - sqrt(disc)) / a if disc > 0; a = 0: -c / (2 b) if b < 0;
 *       else none; clipped at 0.  (These are the first roots ahead at which
 *       Q changes sign in the flag's direction.)  Crossing it is a surface
 *       event that crosses no union plane and flips the flag.  The flag is
 *       set at birth, and when a plane crossing lands in another geometry
 *       cell (after any reflection), from the particle's side of that
 *       cell's quadric: inside iff c < 0, or c == 0 and b < 0; 0 in a cell
 *       without one.  Tie order: census, planes, quadric, collision.  Not
 *       combined with pins or a moving plane; not in a slab (x the only
 *       finite axis).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so mcdc_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Problem description (this oracle's own layout)                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t G, M;
    const double *sigma_t;   /* [M][G] */
    const double *sigma_s;   /* [M][G][G], from g (row) to g' (column) */
    const double *speed;     /* [G] */
    int32_t n_planes[3];     /* 0 = infinite axis */
    const double *planes[3];
    const int32_t *material; /* [cz][cy][cx] over geometry cells */
    int32_t bc[6];           /* x-, x+, y-, y+, z-, z+ : 0 vacuum, 1 reflective */
    /* source */
    double src_lo[3], src_hi[3];
    double src_t_lo, src_t_hi;
    const double *src_pmf;   /* [G] */
    int32_t src_kind;        /* 0 isotropic, 1 surface */
    int32_t src_axis, src_sign, src_mu_law; /* mu law: 0 beam, 1 uniform, 2 cosine */
    /* tally */
    int32_t n_mesh[3];       /* 0 = one bin spanning the axis */
    const double *mesh[3];
    int32_t n_time_edges;
    const double *time_edges;
    int32_t n_batches;
    /* detector (quantity of interest) */
    int32_t qoi_on;
    double qoi_lo[3], qoi_hi[3];
    const int32_t *qoi_groups; /* [G] 0/1 */
    /* weight windows */
    int32_t n_ww[3];         /* 0 = one window cell spanning the axis */
    const double *ww[3];
    const double *ww_center; /* [K][G][wz][wy][wx] or NULL (analog) */
    double ww_ratio;
    int32_t ww_max_split;
    /* time-crossing estimator of the flux at the time edges (R11) */
    int32_t time_crossing;
    /* fission (R12): all three NULL for a non-multiplying problem */
    const double *sigma_f;   /* [M][G] */
    const double *nu;        /* [M][G] mean neutrons per fission */
    const double *chi;       /* [M][G] fission spectrum (sums to 1 per material) */
    /* implicit capture with weight roulette (R14) */
    int32_t implicit_capture;
    double roulette_w, roulette_ws;
    /* cylindrical pins (R15): per geometry cell, or NULL */
    const double *pin_radius;     /* [cz][cy][cx], 0 = no pin */
    const int32_t *pin_material;  /* [cz][cy][cx] */
    /* moving plane (R27): heights at the time edges and rod cells, or NULL */
    const double *rod_z;          /* [K + 1] */
    const int32_t *rod_material;  /* [cz][cy][cx], -1 = not a rod cell */
    /* quadric surfaces (R29): per geometry cell, or NULL */
    const double *quad_coef;      /* [cz][cy][cx][10]: A B C D E F G H J K */
    const int32_t *quad_material; /* [cz][cy][cx], -1 = no quadric */
} oracle_problem;

enum { EV_CENSUS = 0, EV_SURFACE = 1, EV_COLLISION = 2 };
enum { T_ABSORB = 0, T_LEAK = 1, T_TIME = 2, T_LOST = 3, T_ROULETTE = 4 };

/* ------------------------------------------------------------------------ */
/* R1: random numbers                                                         */
/* ------------------------------------------------------------------------ */

static const uint64_t LCG_MULT = 2806196910506780709ULL;
static const uint64_t LCG_ADD = 1ULL;
static const uint64_t LCG_STRIDE = 152917ULL;
static const uint64_t MASK63 = 0x7FFFFFFFFFFFFFFFULL;

/* s_k = g^k s + c (g^k - 1)/(g - 1) mod 2^63, by repeated squaring of the
 * affine map s -> h s + f (F. B. Brown, "Random number generation with
 * arbitrary strides", Trans. Am. Nucl. Soc. 71, 1994). */
uint64_t oracle_rng_skip(uint64_t s, uint64_t k)
{
    uint64_t G = 1, C = 0, h = LCG_MULT, f = LCG_ADD;
    while (k) {
        if (k & 1ULL) {
            G = G * h;
            C = C * h + f;
        }
        f = f * (h + 1ULL);
        h = h * h;
        k >>= 1;
    }
    return (G * (s & MASK63) + C) & MASK63;
}

static double rn(uint64_t *s)
{
    *s = (LCG_MULT * (*s) + LCG_ADD) & MASK63;
    return (double)((*s) >> 10) * 0x1p-53;
}

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
static uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* exported for the random-number tests */
void oracle_rng_draws(uint64_t s, int64_t n, uint64_t *states, double *xi)
{
    for (int64_t j = 0; j < n; j++) {
        double x = rn(&s);
        if (states) states[j] = s;
        if (xi) xi[j] = x;
    }
}

uint64_t oracle_child_stream(uint64_t parent, uint64_t j)
{
    return splitmix64(parent ^ j) & MASK63;
}

/* ------------------------------------------------------------------------ */
/* R4: union grid per axis                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;        /* number of union planes; 0 = infinite axis */
    double *P;    /* [n] */
    int *geo;     /* [n-1] geometry cell of each union cell */
    int *tal;     /* [n-1] tally bin index along the axis, -1 outside mesh */
    int *wwc;     /* [n-1] weight-window cell index, -1 outside */
    int *inq;     /* [n-1] 1 if inside the detector box along this axis */
} axis_grid;

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* index j with E[j] <= x < E[j+1] over n edges, or -1 if outside */
static int bin_of(const double *E, int n, double x)
{
    if (n < 2 || x < E[0] || x >= E[n - 1]) return -1;
    int j = 0;
    while (!(x < E[j + 1])) j++;
    return j;
}

static int build_axis(const oracle_problem *p, int a, axis_grid *A)
{
    memset(A, 0, sizeof(*A));
    int ng = p->n_planes[a];
    if (ng == 0) return 0;
    int cap = ng + p->n_mesh[a] + p->n_ww[a] + 2;
    double *all = (double *)malloc(sizeof(double) * cap);
    int m = 0;
    for (int j = 0; j < ng; j++) all[m++] = p->planes[a][j];
    for (int j = 0; j < p->n_mesh[a]; j++) all[m++] = p->mesh[a][j];
    for (int j = 0; j < p->n_ww[a]; j++) all[m++] = p->ww[a][j];
    if (p->qoi_on) {
        all[m++] = p->qoi_lo[a];
        all[m++] = p->qoi_hi[a];
    }
    double lo = p->planes[a][0], hi = p->planes[a][ng - 1];
    for (int j = 0; j < m; j++)
        if (all[j] < lo || all[j] > hi) {
            free(all);
            return -1;
        }
    qsort(all, m, sizeof(double), cmp_double);
    int n = 0;
    for (int j = 0; j < m; j++)
        if (n == 0 || all[j] != all[n - 1]) all[n++] = all[j];
    A->n = n;
    A->P = all;
    A->geo = (int *)malloc(sizeof(int) * n);
    A->tal = (int *)malloc(sizeof(int) * n);
    A->wwc = (int *)malloc(sizeof(int) * n);
    A->inq = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i + 1 < n; i++) {
        double left = all[i], right = all[i + 1];
        A->geo[i] = bin_of(p->planes[a], ng, left);
        A->tal[i] = (p->n_mesh[a] == 0) ? 0 : bin_of(p->mesh[a], p->n_mesh[a], left);
        A->wwc[i] = (p->n_ww[a] == 0) ? 0 : bin_of(p->ww[a], p->n_ww[a], left);
        A->inq[i] = p->qoi_on ? (left >= p->qoi_lo[a] && right <= p->qoi_hi[a]) : 1;
    }
    return 0;
}

static void free_axis(axis_grid *A)
{
    free(A->P);
    free(A->geo);
    free(A->tal);
    free(A->wwc);
    free(A->inq);
}

/* Birth location: the cell i with P_i <= x < P_{i+1}; a particle born exactly
 * on P_i moving towards -axis belongs to cell i-1; clamp to the domain cells. */
static int locate(const axis_grid *A, double x, double u)
{
    int i = -1;
    for (int j = 0; j < A->n; j++)
        if (A->P[j] <= x) i = j;
    if (i >= 0 && x == A->P[i] && u < 0.0) i = i - 1;
    if (i < 0) i = 0;
    if (i > A->n - 2) i = A->n - 2;
    return i;
}

/* ------------------------------------------------------------------------ */
/* Neumaier compensated sums                                                  */
/* ------------------------------------------------------------------------ */

static void csum(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/* ------------------------------------------------------------------------ */
/* Particle and per-run context                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    double x[3], u[3], inv_u[3];
    double t, tau, w;
    int ix[3];
    int g, k;
    int inpin;      /* R15: inside the cell's pin; R29: inside the cell's quadric */
    int above;      /* R27: above the moving plane (meaningful in rod cells) */
    int since;      /* events since birth or the last census */
    uint64_t s;
} particle;

/* A particle with this many events since its last census (or birth) is
 * killed as lost: a guard against problems that trap a particle forever
 * (e.g. a pure scatterer enclosed by reflective faces with no time limit).
 * Normal problems never come near it. */
#define MAX_EVENTS_PER_STEP (1 << 20)

typedef struct {
    const oracle_problem *p;
    axis_grid ax[3];
    int K;              /* number of time bins */
    int nt[3];          /* tally bins per axis */
    int nw[3];          /* weight-window cells per axis */
    int64_t ntally;     /* K * G * nt[2] * nt[1] * nt[0] */
    int nc[3];          /* geometry cells per axis */
    double *ps;         /* [M][G] Sigma_s,g / Sigma_t,g */
    double *cdf;        /* [M][G][G] outgoing-group CDF */
    double *src_cdf;    /* [G] */
    /* outputs */
    double *S, *Sc;     /* [B][ntally] raw sums + compensation */
    double *X, *Xc;     /* [B][ntally] time-crossing sums (edge T_{k+1} at k) */
    double *L, *Lc;     /* [B][K][G][6] leak sums */
    double q[2], qc[2]; /* detector: sum x, sum x^2 over histories */
    uint64_t tot[10];   /* events: census, surface, collision; terminations
                           absorb, leak, time, lost, roulette; splits;
                           fission neutrons beyond the colliding one */
    double *pf;         /* [M][G] (Sigma_s,g + Sigma_f,g) / Sigma_t,g (fission only) */
    /* k-eigenvalue cycles (R13) */
    int eigen;          /* fissions bank sites instead of continuing */
    int quiet;          /* inactive cycle: no tallies */
    double site_x[3];   /* fission site of the current particle */
    int site_ix[3];
    int site_inpin;
    int site_n;         /* sites banked there (0: none) */
    double *chi_cdf;    /* [M][G] fission-spectrum CDF (fission only) */
} ctx;

static void isotropic(uint64_t *s, double u[3])
{
    for (;;) {
        double a = 2.0 * rn(s) - 1.0;
        double b = 2.0 * rn(s) - 1.0;
        double r = a * a + b * b;
        if (r < 1.0) {
            double q = sqrt(1.0 - r);
            u[0] = 1.0 - 2.0 * r;
            u[1] = (2.0 * a) * q;
            u[2] = (2.0 * b) * q;
            return;
        }
    }
}

static void set_inv(particle *pt)
{
    for (int a = 0; a < 3; a++) pt->inv_u[a] = 1.0 / pt->u[a];
}

static int64_t geo_cell(const ctx *C, const particle *pt, int c[3])
{
    for (int a = 0; a < 3; a++) c[a] = (C->ax[a].n == 0) ? 0 : C->ax[a].geo[pt->ix[a]];
    return ((int64_t)c[2] * C->nc[1] + c[1]) * C->nc[0] + c[0];
}

/* R27: rod material of the particle's geometry cell, -1 if not a rod cell */
static int rod_cell(const ctx *C, const particle *pt)
{
    if (!C->p->rod_material) return -1;
    int c[3];
    return C->p->rod_material[geo_cell(C, pt, c)];
}

static int material_of(const ctx *C, const particle *pt)
{
    int c[3];
    int64_t g = geo_cell(C, pt, c);
    if (pt->inpin) return C->p->pin_radius ? C->p->pin_material[g] : C->p->quad_material[g];
    if (C->p->rod_material && C->p->rod_material[g] >= 0 && pt->above) return C->p->rod_material[g];
    return C->p->material[g];
}

/* R27: height of the moving plane at time t in census step k, and its
 * speed there */
static double rod_height(const ctx *C, int k, double t, double *vz)
{
    const double *T = C->p->time_edges;
    const double *Z = C->p->rod_z;
    double v = 0.0;
    if (T[k + 1] != INFINITY) v = (Z[k + 1] - Z[k]) / (T[k + 1] - T[k]);
    *vz = v;
    return Z[k] + v * (t - T[k]);
}

/* R27: the side of the moving plane a particle at its place and time is on */
static int rod_side(const ctx *C, const particle *pt)
{
    double vz;
    double Z = rod_height(C, pt->k, pt->t, &vz);
    if (pt->x[2] > Z) return 1;
    if (pt->x[2] < Z) return 0;
    double q = pt->u[2] - vz * (1.0 / C->p->speed[pt->g]);
    return q > 0.0;
}

/* R15: the pin of the particle's geometry cell (centre, r^2); 0 if none */
static int pin_of(const ctx *C, const particle *pt, double *xc, double *yc, double *r2)
{
    const oracle_problem *p = C->p;
    if (!p->pin_radius) return 0;
    int c[3];
    int64_t g = geo_cell(C, pt, c);
    double r = p->pin_radius[g];
    if (!(r > 0.0)) return 0;
    *xc = 0.5 * (p->planes[0][c[0]] + p->planes[0][c[0] + 1]);
    *yc = 0.5 * (p->planes[1][c[1]] + p->planes[1][c[1] + 1]);
    *r2 = r * r;
    return 1;
}

/* R29: the quadric of the particle's geometry cell (its coefficients), or
 * NULL; *gc receives the geometry cell */
static const double *quad_of(const ctx *C, const particle *pt, int64_t *gc)
{
    const oracle_problem *p = C->p;
    int c[3];
    int64_t g = geo_cell(C, pt, c);
    if (gc) *gc = g;
    if (!p->quad_material || p->quad_material[g] < 0) return NULL;
    return p->quad_coef + 10 * g;
}

/* R29: Q(x + d u) = a d^2 + 2 b d + c */
static void quad_abc(const double *q, const double *x, const double *u, double *a, double *b, double *c)
{
    *a = ((q[0] * u[0] * u[0] + q[1] * u[1] * u[1]) + q[2] * u[2] * u[2]) +
         ((q[3] * u[0] * u[1] + q[4] * u[1] * u[2]) + q[5] * u[2] * u[0]);
    *b = ((q[0] * x[0] * u[0] + q[1] * x[1] * u[1]) + q[2] * x[2] * u[2]) +
         0.5 * (((q[3] * (x[0] * u[1] + x[1] * u[0]) + q[4] * (x[1] * u[2] + x[2] * u[1])) +
                 q[5] * (x[2] * u[0] + x[0] * u[2])) +
                ((q[6] * u[0] + q[7] * u[1]) + q[8] * u[2]));
    *c = (((q[0] * x[0] * x[0] + q[1] * x[1] * x[1]) + q[2] * x[2] * x[2]) +
          ((q[3] * x[0] * x[1] + q[4] * x[1] * x[2]) + q[5] * x[2] * x[0])) +
         (((q[6] * x[0] + q[7] * x[1]) + q[8] * x[2]) + q[9]);
}

/* R29: inside the quadric at the particle's place, or on it and moving in */
static int quad_side(const double *q, const particle *pt)
{
    double a, b, c;
    quad_abc(q, pt->x, pt->u, &a, &b, &c);
    return c < 0.0 || (c == 0.0 && b < 0.0);
}

/* R29: distance to the quadric from the side the flag gives, or infinity */
static double quad_distance(const double *q, const particle *pt)
{
    double a, b, c;
    quad_abc(q, pt->x, pt->u, &a, &b, &c);
    double d = INFINITY;
    const double disc = b * b - a * c;
    if (pt->inpin) {
        if (a > 0.0)
            d = (-b + sqrt(disc > 0.0 ? disc : 0.0)) / a;
        else if (a < 0.0) {
            if (b > 0.0 && disc > 0.0) d = (-b + sqrt(disc)) / a;
        } else if (b > 0.0)
            d = -c / (2.0 * b);
    } else {
        if (a > 0.0) {
            if (b < 0.0 && disc > 0.0) d = (-b - sqrt(disc)) / a;
        } else if (a < 0.0) {
            if (disc > 0.0) d = (-b - sqrt(disc)) / a;
        } else if (b < 0.0)
            d = -c / (2.0 * b);
    }
    if (d < 0.0) d = 0.0;
    return d;
}

/* tally bin of the particle's union cell in the current (k, g), or -1 */
static int64_t tally_bin(const ctx *C, const particle *pt)
{
    int t[3];
    for (int a = 0; a < 3; a++) {
        t[a] = (C->ax[a].n == 0) ? 0 : C->ax[a].tal[pt->ix[a]];
        if (t[a] < 0) return -1;
    }
    return ((((int64_t)pt->k * C->p->G + pt->g) * C->nt[2] + t[2]) * C->nt[1] + t[1]) * C->nt[0] + t[0];
}

static int in_qoi(const ctx *C, const particle *pt)
{
    if (!C->p->qoi_on || !C->p->qoi_groups[pt->g]) return 0;
    for (int a = 0; a < 3; a++)
        if (C->ax[a].n != 0 && !C->ax[a].inq[pt->ix[a]]) return 0;
    return 1;
}

/* weight-window centre of the particle's cell, 0 = no window */
static double ww_center(const ctx *C, const particle *pt)
{
    if (!C->p->ww_center) return 0.0;
    int c[3];
    for (int a = 0; a < 3; a++) {
        c[a] = (C->ax[a].n == 0) ? 0 : C->ax[a].wwc[pt->ix[a]];
        if (c[a] < 0) return 0.0;
    }
    int64_t j = ((((int64_t)pt->k * C->p->G + pt->g) * C->nw[2] + c[2]) * C->nw[1] + c[1]) * C->nw[0] + c[0];
    return C->p->ww_center[j];
}

/* ------------------------------------------------------------------------ */
/* Per-history tracking                                                       */
/* ------------------------------------------------------------------------ */

#define STACK_MAX 4096

typedef struct {
    uint32_t n_census, n_surf, n_coll, n_particles, term_mask;
    double track;   /* sum of w*d over all tallied segments */
    double qoi;     /* detector score of this history */
} hist_rec;

/* R10: the weight-window game.  Returns 0 if the particle is killed. */
static int ww_game(ctx *C, particle *pt, particle *stack, int *sp, hist_rec *h)
{
    double wc = ww_center(C, pt);
    if (wc == 0.0) return 1;
    double rho = C->p->ww_ratio;
    double wl = (2.0 * wc) / (1.0 + rho);
    double wu = rho * wl;
    if (pt->w > wu) {
        double nr = ceil(pt->w / wu);
        int n = (nr > (double)C->p->ww_max_split) ? C->p->ww_max_split : (int)nr;
        if (n > 1) {
            pt->w = pt->w / (double)n;
            for (int j = 1; j < n; j++) {
                if (*sp >= STACK_MAX) return -1;
                stack[*sp] = *pt;
                stack[*sp].s = splitmix64(pt->s ^ (uint64_t)j) & MASK63;
                (*sp)++;
                h->n_particles++;
                C->tot[8]++;
            }
        }
    } else if (pt->w < wl) {
        double xi = rn(&pt->s);
        if (xi < pt->w / wc) {
            pt->w = wc;
        } else {
            h->term_mask |= 1u << T_ROULETTE;
            C->tot[3 + T_ROULETTE]++;
            return 0;
        }
    }
    return 1;
}

static void terminate(ctx *C, hist_rec *h, int code)
{
    h->term_mask |= 1u << code;
    C->tot[3 + code]++;
}

/* R12: a fission neutron takes its group from the spectrum, an isotropic
 * direction and an optical depth, all from its own stream. */
static void emit(const ctx *C, particle *pt, int m)
{
    const int G = C->p->G;
    double xg = rn(&pt->s);
    int g = 0;
    while (!(xg < C->chi_cdf[m * G + g])) g++;
    pt->g = g;
    isotropic(&pt->s, pt->u);
    set_inv(pt);
    pt->tau = -log(1.0 - rn(&pt->s));
}

/* R12: fission at a collision in material m.  Returns 1 if the colliding
 * particle goes on as neutron 0, 0 if no neutron is emitted, -1 if the
 * progeny overflow the stack. */
static int fission(ctx *C, particle *pt, int m, particle *stack, int *sp, hist_rec *h)
{
    const int G = C->p->G;
    double nu = C->p->nu[m * G + pt->g];
    int n = (int)floor(nu + rn(&pt->s));
    if (n == 0) {
        terminate(C, h, T_ABSORB);
        return 0;
    }
    uint64_t sf = pt->s;
    for (int j = 1; j < n; j++) {
        if (*sp >= STACK_MAX) return -1;
        particle c = *pt;
        c.s = splitmix64(sf ^ (uint64_t)j) & MASK63;
        emit(C, &c, m);
        stack[(*sp)++] = c;
        h->n_particles++;
        C->tot[9]++;
    }
    emit(C, pt, m);
    return 1;
}

/* One flight plus the event that ends it.  Returns 1 if the particle lives
 * on, 0 if it terminated, -1 if split progeny overflow the stack.  If row is
 * not NULL it receives (event, d, x, y, z, t, g, k, tau) after the event. */
static int step(ctx *C, particle *pt, int b, particle *stack, int *sp, hist_rec *h, double *row)
{
    const oracle_problem *p = C->p;
    const int G = p->G;
    if (pt->since >= MAX_EVENTS_PER_STEP) {
        if (row) {
            row[0] = EV_COLLISION;
            row[1] = INFINITY;
        }
        terminate(C, h, T_LOST);
        return 0;
    }
    pt->since++;
    int m = material_of(C, pt);
    double st = p->sigma_t[m * G + pt->g];

    /* distance to collision */
    double dc = (st == 0.0) ? INFINITY : pt->tau * (1.0 / st);
    /* distance to the nearest union plane along each finite axis */
    double da[3], ds = INFINITY;
    for (int a = 0; a < 3; a++) {
        da[a] = INFINITY;
        if (C->ax[a].n == 0 || pt->u[a] == 0.0) continue;
        double P = (pt->u[a] > 0.0) ? C->ax[a].P[pt->ix[a] + 1] : C->ax[a].P[pt->ix[a]];
        double d = (P - pt->x[a]) * pt->inv_u[a];
        if (d < 0.0) d = 0.0;
        da[a] = d;
        if (d < ds) ds = d;
    }
    /* R15: distance to the cell's pin surface */
    double dcyl = INFINITY;
    {
        double xc, yc, r2;
        if (pin_of(C, pt, &xc, &yc, &r2)) {
            double dx = pt->x[0] - xc, dy = pt->x[1] - yc;
            double a = pt->u[0] * pt->u[0] + pt->u[1] * pt->u[1];
            double b = dx * pt->u[0] + dy * pt->u[1];
            double c = (dx * dx + dy * dy) - r2;
            if (a > 0.0) {
                if (pt->inpin) {
                    double disc = b * b - a * c;
                    if (disc < 0.0) disc = 0.0;
                    dcyl = (-b + sqrt(disc)) / a;
                } else if (b < 0.0) {
                    double disc = b * b - a * c;
                    if (disc > 0.0) dcyl = (-b - sqrt(disc)) / a;
                }
                if (dcyl < 0.0) dcyl = 0.0;
            }
        }
        /* R29: distance to the cell's quadric (a problem has pins or
           quadrics, not both) */
        const double *q = quad_of(C, pt, NULL);
        if (q) dcyl = quad_distance(q, pt);
    }
    /* R27: distance to the moving plane in a rod cell */
    double dmov = INFINITY;
    if (rod_cell(C, pt) >= 0) {
        double vz;
        double Z = rod_height(C, pt->k, pt->t, &vz);
        double q = pt->u[2] - vz * (1.0 / p->speed[pt->g]);
        if ((pt->above && q < 0.0) || (!pt->above && q > 0.0)) {
            dmov = (Z - pt->x[2]) / q;
            if (dmov < 0.0) dmov = 0.0;
        }
    }
    /* distance to the next time-census edge */
    double Tn = p->time_edges[pt->k + 1];
    double dt = INFINITY;
    if (Tn != INFINITY) {
        dt = (Tn - pt->t) * p->speed[pt->g];
        if (dt < 0.0) dt = 0.0;
    }
    /* R3, R15, R27 (a problem has pins or a moving plane, not both) */
    int ev, cyl = 0, mov = 0;
    double d;
    if (dt <= ds && dt <= dcyl && dt <= dmov && dt <= dc) {
        ev = EV_CENSUS;
        d = dt;
    } else if (ds <= dcyl && ds <= dmov && ds <= dc) {
        ev = EV_SURFACE;
        d = ds;
    } else if (dcyl <= dmov && dcyl <= dc) {
        ev = EV_SURFACE;
        d = dcyl;
        cyl = 1;
    } else if (dmov <= dc) {
        ev = EV_SURFACE;
        d = dmov;
        mov = 1;
    } else {
        ev = EV_COLLISION;
        d = dc;
    }
    if (row) {
        row[0] = ev;
        row[1] = d;
    }
    if (d == INFINITY) {
        terminate(C, h, T_LOST);
        return 0;
    }

    /* track-length score of the flight */
    double sc = pt->w * d;
    int64_t j = C->quiet ? -1 : tally_bin(C, pt);
    if (j >= 0) {
        csum(&C->S[(int64_t)b * C->ntally + j], &C->Sc[(int64_t)b * C->ntally + j], sc);
        h->track += sc;
    }
    if (!C->quiet && in_qoi(C, pt)) h->qoi += sc;

    /* move */
    for (int a = 0; a < 3; a++) pt->x[a] = fma(d, pt->u[a], pt->x[a]);
    if (ev == EV_CENSUS)
        pt->t = Tn;
    else
        pt->t = pt->t + d * (1.0 / p->speed[pt->g]);
    if (ev != EV_COLLISION && st != 0.0) {
        pt->tau = pt->tau - d * st;
        if (pt->tau < 0.0) pt->tau = 0.0;
    }

    int alive = 1;
    if (ev == EV_CENSUS) {
        h->n_census++;
        C->tot[0]++;
        /* R11: the particle is at the edge T_{k+1} now */
        if (p->time_crossing) {
            int64_t jx = tally_bin(C, pt);
            if (jx >= 0)
                csum(&C->X[(int64_t)b * C->ntally + jx], &C->Xc[(int64_t)b * C->ntally + jx],
                     pt->w * p->speed[pt->g]);
        }
        pt->since = 0;
        pt->k++;
        if (pt->k == C->K) {
            terminate(C, h, T_TIME);
            alive = 0;
        } else {
            alive = ww_game(C, pt, stack, sp, h);
        }
    } else if (ev == EV_SURFACE) {
        h->n_surf++;
        C->tot[1]++;
        int wcell_changed = 0;
        const int rod_before = rod_cell(C, pt);
        int64_t geo_before = -1;
        if (p->quad_material) (void)quad_of(C, pt, &geo_before);
        for (int a = 0; a < 3 && alive; a++) {
            if (mov || C->ax[a].n == 0 || da[a] != d) continue;
            int last = C->ax[a].n - 2;
            int old = pt->ix[a];
            int face = -1;
            if (pt->u[a] > 0.0) {
                pt->x[a] = C->ax[a].P[pt->ix[a] + 1];
                if (pt->ix[a] == last) face = 2 * a + 1;
                else pt->ix[a]++;
            } else {
                pt->x[a] = C->ax[a].P[pt->ix[a]];
                if (pt->ix[a] == 0) face = 2 * a;
                else pt->ix[a]--;
            }
            if (face >= 0) {
                if (p->bc[face] == 0) {
                    int64_t l = (((int64_t)b * C->K + pt->k) * G + pt->g) * 6 + face;
                    if (!C->quiet) csum(&C->L[l], &C->Lc[l], pt->w);
                    terminate(C, h, T_LEAK);
                    alive = 0;
                } else {
                    pt->u[a] = -pt->u[a];
                    pt->inv_u[a] = -pt->inv_u[a];
                }
            }
            if (pt->ix[a] != old && C->ax[a].wwc[pt->ix[a]] != C->ax[a].wwc[old]) wcell_changed = 1;
        }
        if (cyl) pt->inpin ^= 1;
        if (!cyl && alive && p->quad_material) {
            /* R29: landing in another geometry cell sets the flag from that
               cell's quadric */
            int64_t geo_now;
            const double *q = quad_of(C, pt, &geo_now);
            if (geo_now != geo_before) pt->inpin = q ? quad_side(q, pt) : 0;
        }
        if (mov) {
            pt->above ^= 1;
        } else if (alive && p->rod_material) {
            /* R27: entering a rod cell from one that is not sets the flag */
            if (rod_cell(C, pt) < 0)
                pt->above = 0;
            else if (rod_before < 0)
                pt->above = rod_side(C, pt);
        }
        if (alive && wcell_changed) alive = ww_game(C, pt, stack, sp, h);
    } else {
        h->n_coll++;
        C->tot[2]++;
        /* analog collision: scatter with probability Sigma_s,g / Sigma_t,g,
         * fission with probability Sigma_f,g / Sigma_t,g (R12); with implicit
         * capture every collision scatters at reduced weight (R14) */
        double xr = 0.0;
        if (p->implicit_capture) {
            pt->w = pt->w * C->ps[m * G + pt->g];
            if (pt->w < p->roulette_w) {
                double xw = rn(&pt->s);
                if (xw < pt->w / p->roulette_ws) {
                    pt->w = p->roulette_ws;
                } else {
                    terminate(C, h, T_ROULETTE);
                    alive = 0;
                }
            }
        } else {
            xr = rn(&pt->s);
        }
        if (!alive) {
            /* rouletted */
        } else if (!p->implicit_capture && !(xr < C->ps[m * G + pt->g])) {
            if (C->pf && xr < C->pf[m * G + pt->g] && C->eigen) {
                /* R13: bank the sites, end the particle */
                C->site_n = (int)floor(p->nu[m * G + pt->g] + rn(&pt->s));
                for (int a = 0; a < 3; a++) {
                    C->site_x[a] = pt->x[a];
                    C->site_ix[a] = pt->ix[a];
                }
                C->site_inpin = pt->inpin;
                terminate(C, h, T_ABSORB);
                alive = 0;
            } else if (C->pf && xr < C->pf[m * G + pt->g]) {
                alive = fission(C, pt, m, stack, sp, h);
                if (alive > 0) alive = ww_game(C, pt, stack, sp, h);
            } else {
                terminate(C, h, T_ABSORB);
                alive = 0;
            }
        } else {
            double xg = rn(&pt->s);
            const double *cdf = &C->cdf[((int64_t)m * G + pt->g) * G];
            int g2 = 0;
            while (!(xg < cdf[g2])) g2++;
            pt->g = g2;
            isotropic(&pt->s, pt->u);
            set_inv(pt);
            pt->tau = -log(1.0 - rn(&pt->s));
            alive = ww_game(C, pt, stack, sp, h);
        }
    }
    if (row) {
        row[2] = pt->x[0];
        row[3] = pt->x[1];
        row[4] = pt->x[2];
        row[5] = pt->t;
        row[6] = pt->g;
        row[7] = pt->k;
        row[8] = pt->tau;
    }
    return alive;
}

/* Track one particle until it terminates (its split progeny go on the stack). */
static int track(ctx *C, particle *pt, int b, particle *stack, int *sp, hist_rec *h)
{
    for (;;) {
        int r = step(C, pt, b, stack, sp, h, NULL);
        if (r <= 0) return r;
    }
}

static int birth(ctx *C, uint64_t s0, particle *pt, hist_rec *h)
{
    const oracle_problem *p = C->p;
    memset(pt, 0, sizeof(*pt));
    pt->s = s0;
    for (int a = 0; a < 3; a++) {
        double xi = rn(&pt->s);
        pt->x[a] = (C->ax[a].n == 0) ? 0.0 : p->src_lo[a] + xi * (p->src_hi[a] - p->src_lo[a]);
    }
    double xt = rn(&pt->s);
    pt->t = p->src_t_lo + xt * (p->src_t_hi - p->src_t_lo);
    double xg = rn(&pt->s);
    int g = 0;
    while (!(xg < C->src_cdf[g])) g++;
    pt->g = g;
    if (p->src_kind == 0) {
        isotropic(&pt->s, pt->u);
    } else {
        double xm = rn(&pt->s);
        double mu = (p->src_mu_law == 0) ? 1.0 : (p->src_mu_law == 1) ? 1.0 - xm : sqrt(1.0 - xm);
        double a, b, r;
        for (;;) {
            a = 2.0 * rn(&pt->s) - 1.0;
            b = 2.0 * rn(&pt->s) - 1.0;
            r = a * a + b * b;
            if (r > 0.0 && r < 1.0) break;
        }
        double cph = (a * a - b * b) / r;
        double sph = ((2.0 * a) * b) / r;
        double sn = sqrt(1.0 - mu * mu);
        int ax = p->src_axis;
        pt->u[ax] = (double)p->src_sign * mu;
        pt->u[(ax + 1) % 3] = sn * cph;
        pt->u[(ax + 2) % 3] = sn * sph;
    }
    set_inv(pt);
    pt->tau = -log(1.0 - rn(&pt->s));
    pt->w = 1.0;
    for (int a = 0; a < 3; a++) pt->ix[a] = (C->ax[a].n == 0) ? 0 : locate(&C->ax[a], pt->x[a], pt->u[a]);
    {
        double xc, yc, r2;
        if (pin_of(C, pt, &xc, &yc, &r2)) {
            double dx = pt->x[0] - xc, dy = pt->x[1] - yc;
            pt->inpin = ((dx * dx + dy * dy) - r2) < 0.0;
        }
        /* R29 */
        const double *q = quad_of(C, pt, NULL);
        if (q) pt->inpin = quad_side(q, pt);
    }
    /* time bin */
    if (pt->t >= p->time_edges[C->K]) {
        terminate(C, h, T_TIME);
        return 0;
    }
    int k = 0;
    while (!(pt->t < p->time_edges[k + 1])) k++;
    pt->k = k;
    /* R27: the side of the moving plane in a rod cell */
    if (rod_cell(C, pt) >= 0) pt->above = rod_side(C, pt);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Set-up                                                                     */
/* ------------------------------------------------------------------------ */

static int ctx_init(ctx *C, const oracle_problem *p)
{
    memset(C, 0, sizeof(*C));
    C->p = p;
    const int G = p->G, M = p->M;
    C->K = p->n_time_edges - 1;
    if (G < 1 || M < 1 || C->K < 1 || p->n_batches < 1) return -1;
    if (p->implicit_capture &&
        (p->sigma_f || !(p->roulette_w > 0.0) || !(p->roulette_ws >= p->roulette_w)))
        return -1;
    for (int a = 0; a < 3; a++) {
        if (build_axis(p, a, &C->ax[a]) != 0) return -1;
        C->nc[a] = (p->n_planes[a] == 0) ? 1 : p->n_planes[a] - 1;
        C->nt[a] = (p->n_mesh[a] == 0) ? 1 : p->n_mesh[a] - 1;
        C->nw[a] = (p->n_ww[a] == 0) ? 1 : p->n_ww[a] - 1;
    }
    C->ntally = (int64_t)C->K * G * C->nt[0] * C->nt[1] * C->nt[2];
    if (p->rod_material) {
        /* R27: a finite z axis, heights at every time edge, no pins */
        if (p->n_planes[2] == 0 || !p->rod_z || p->pin_radius) return -1;
        for (int k = 0; k <= C->K; k++)
            if (!isfinite(p->rod_z[k])) return -1;
        for (int64_t g = 0; g < (int64_t)C->nc[0] * C->nc[1] * C->nc[2]; g++)
            if (p->rod_material[g] < -1 || p->rod_material[g] >= M) return -1;
    }
    if (p->quad_material) {
        /* R29: finite coefficients, materials in range, no pins or moving
           plane, not a slab */
        if (!p->quad_coef || p->pin_radius || p->rod_material) return -1;
        if (p->n_planes[1] == 0 && p->n_planes[2] == 0) return -1;
        for (int64_t g = 0; g < (int64_t)C->nc[0] * C->nc[1] * C->nc[2]; g++) {
            if (p->quad_material[g] < -1 || p->quad_material[g] >= M) return -1;
            for (int j = 0; j < 10; j++)
                if (!isfinite(p->quad_coef[10 * g + j])) return -1;
        }
    }
    if (p->pin_radius) {
        /* R15: pins need finite x and y axes and must fit their cells */
        if (p->n_planes[0] == 0 || p->n_planes[1] == 0 || !p->pin_material) return -1;
        for (int cz = 0; cz < C->nc[2]; cz++)
            for (int cy = 0; cy < C->nc[1]; cy++)
                for (int cx = 0; cx < C->nc[0]; cx++) {
                    int64_t g = ((int64_t)cz * C->nc[1] + cy) * C->nc[0] + cx;
                    double r = p->pin_radius[g];
                    if (!(r >= 0.0)) return -1;
                    if (r == 0.0) continue;
                    double hx = 0.5 * (p->planes[0][cx + 1] - p->planes[0][cx]);
                    double hy = 0.5 * (p->planes[1][cy + 1] - p->planes[1][cy]);
                    if (!(r < hx) || !(r < hy) || p->pin_material[g] < 0 || p->pin_material[g] >= M) return -1;
                }
    }
    C->ps = (double *)calloc((size_t)M * G, sizeof(double));
    C->cdf = (double *)calloc((size_t)M * G * G, sizeof(double));
    C->src_cdf = (double *)calloc((size_t)G, sizeof(double));
    for (int m = 0; m < M; m++)
        for (int g = 0; g < G; g++) {
            const double *row = &p->sigma_s[((int64_t)m * G + g) * G];
            double ss = 0.0;
            for (int g2 = 0; g2 < G; g2++) ss += row[g2];
            double st = p->sigma_t[m * G + g];
            C->ps[m * G + g] = (st > 0.0) ? ss / st : 0.0;
            double run = 0.0;
            int last = -1;
            for (int g2 = 0; g2 < G; g2++) {
                run += row[g2];
                C->cdf[((int64_t)m * G + g) * G + g2] = (ss > 0.0) ? run / ss : 1.0;
                if (row[g2] > 0.0) last = g2;
            }
            for (int g2 = (last < 0 ? 0 : last); g2 < G; g2++) C->cdf[((int64_t)m * G + g) * G + g2] = 1.0;
        }
    if (p->sigma_f) {
        if (!p->nu || !p->chi) return -1;
        C->pf = (double *)calloc((size_t)M * G, sizeof(double));
        C->chi_cdf = (double *)calloc((size_t)M * G, sizeof(double));
        for (int m = 0; m < M; m++) {
            for (int g = 0; g < G; g++) {
                const double *row = &p->sigma_s[((int64_t)m * G + g) * G];
                double ss = 0.0;
                for (int g2 = 0; g2 < G; g2++) ss += row[g2];
                double st = p->sigma_t[m * G + g];
                C->pf[m * G + g] = (st > 0.0) ? (ss + p->sigma_f[m * G + g]) / st : 0.0;
            }
            double run = 0.0;
            int last = -1;
            for (int g = 0; g < G; g++) {
                run += p->chi[m * G + g];
                C->chi_cdf[m * G + g] = run;
                if (p->chi[m * G + g] > 0.0) last = g;
            }
            for (int g = (last < 0 ? 0 : last); g < G; g++) C->chi_cdf[m * G + g] = 1.0;
        }
    }
    {
        double run = 0.0;
        int last = -1;
        for (int g = 0; g < G; g++) {
            run += p->src_pmf[g];
            C->src_cdf[g] = run;
            if (p->src_pmf[g] > 0.0) last = g;
        }
        if (last < 0) return -1;
        for (int g = last; g < G; g++) C->src_cdf[g] = 1.0;
    }
    return 0;
}

static void ctx_free(ctx *C)
{
    for (int a = 0; a < 3; a++) free_axis(&C->ax[a]);
    free(C->ps);
    free(C->cdf);
    free(C->pf);
    free(C->chi_cdf);
    free(C->src_cdf);
    free(C->S);
    free(C->Sc);
    free(C->X);
    free(C->Xc);
    free(C->L);
    free(C->Lc);
}

int64_t oracle_ntally(const oracle_problem *p)
{
    int64_t n = (int64_t)(p->n_time_edges - 1) * p->G;
    for (int a = 0; a < 3; a++) n *= (p->n_mesh[a] == 0) ? 1 : p->n_mesh[a] - 1;
    return n;
}

/* Union-grid planes of one axis, for inspection by the tests. */
int oracle_union_planes(const oracle_problem *p, int axis, double *out, int cap)
{
    axis_grid A;
    if (build_axis(p, axis, &A) != 0) return -1;
    int n = A.n;
    for (int j = 0; j < n && j < cap; j++) out[j] = A.P[j];
    free_axis(&A);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Runs                                                                       */
/* ------------------------------------------------------------------------ */

/*
 * Run the histories listed in ids[0..n_ids) of an N-history job (ids==NULL:
 * the contiguous range first..first+n_ids-1).  Accumulates raw per-batch
 * tally sums S[B][ntally] and leak sums L[B][K][G][6] (both may be NULL),
 * detector sums q[2] = (sum x, sum x^2), event and termination totals
 * tot[10], per-history records rec[n_ids][5] = (census, surface,
 * collision, particles, termination mask), per-history track and
 * detector scores trk[n_ids][2], and time-crossing sums X[B][ntally] (R11;
 * zeros unless the problem asks for them).  Returns 0, or -1 on an invalid problem,
 * -4 if split progeny overflow the per-history stack, -5 if a history
 * index is not below N.
 */
int oracle_run(const oracle_problem *p, uint64_t N, uint64_t seed,
               const uint64_t *ids, uint64_t first, uint64_t n_ids,
               double *S_out, double *L_out, double *q_out, uint64_t *tot_out,
               uint32_t *rec, double *trk, double *X_out)
{
    ctx C;
    if (ctx_init(&C, p) != 0) {
        ctx_free(&C);
        return -1;
    }
    int64_t B = p->n_batches;
    if ((uint64_t)B > N) B = (int64_t)N;
    if (B < 1) B = 1;
    const int G = p->G;
    C.S = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.Sc = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.X = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.Xc = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.L = (double *)calloc((size_t)(B * C.K * G * 6), sizeof(double));
    C.Lc = (double *)calloc((size_t)(B * C.K * G * 6), sizeof(double));
    particle *stack = (particle *)malloc(sizeof(particle) * STACK_MAX);
    int rc = 0;
    uint64_t s0 = seed & MASK63;
    for (uint64_t r = 0; r < n_ids; r++) {
        uint64_t i = ids ? ids[r] : first + r;
        if (i >= N) {
            rc = -5;
            break;
        }
        int64_t b = (int64_t)(((i + 1) * (uint64_t)B - 1) / N);
        hist_rec h;
        memset(&h, 0, sizeof(h));
        h.n_particles = 1;
        particle pt;
        int sp = 0;
        if (birth(&C, oracle_rng_skip(s0, i * LCG_STRIDE), &pt, &h)) {
            if (track(&C, &pt, (int)b, stack, &sp, &h) < 0) rc = -4;
            while (sp > 0 && rc == 0) {
                pt = stack[--sp];
                if (track(&C, &pt, (int)b, stack, &sp, &h) < 0) rc = -4;
            }
        }
        if (rc) break;
        if (p->qoi_on) {
            csum(&C.q[0], &C.qc[0], h.qoi);
            csum(&C.q[1], &C.qc[1], h.qoi * h.qoi);
        }
        if (rec) {
            rec[r * 5 + 0] = h.n_census;
            rec[r * 5 + 1] = h.n_surf;
            rec[r * 5 + 2] = h.n_coll;
            rec[r * 5 + 3] = h.n_particles;
            rec[r * 5 + 4] = h.term_mask;
        }
        if (trk) {
            trk[r * 2 + 0] = h.track;
            trk[r * 2 + 1] = h.qoi;
        }
    }
    if (S_out)
        for (int64_t j = 0; j < B * C.ntally; j++) S_out[j] += C.S[j] + C.Sc[j];
    if (X_out)
        for (int64_t j = 0; j < B * C.ntally; j++) X_out[j] += C.X[j] + C.Xc[j];
    if (L_out)
        for (int64_t j = 0; j < B * C.K * G * 6; j++) L_out[j] += C.L[j] + C.Lc[j];
    if (q_out) {
        q_out[0] += C.q[0] + C.qc[0];
        q_out[1] += C.q[1] + C.qc[1];
    }
    if (tot_out)
        for (int j = 0; j < 10; j++) tot_out[j] += C.tot[j];
    free(stack);
    ctx_free(&C);
    return rc;
}

/* R16: w truncated to a multiple of 2^-64, as a 128-bit integer (hi, lo),
 * added to (*hi, *lo).  Returns 0, or -1 if w is 2^32 or more (or not a
 * finite non-negative number). */
static int q64_add(uint64_t *hi, uint64_t *lo, double w)
{
    if (!(w >= 0.0) || !(w < 4294967296.0)) return -1;
    uint64_t bits;
    memcpy(&bits, &w, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FF);
    if (e == 0) return 0;  /* zero or below 2^-1022: truncates to 0 */
    uint64_t m = (bits & ((1ULL << 52) - 1)) | (1ULL << 52);
    /* w = m 2^(e - 1075), so w 2^64 = m 2^(e - 1011) */
    int sh = e - 1011;
    uint64_t h = 0, l = 0;
    if (sh >= 64) {
        h = m << (sh - 64);
    } else if (sh > 0) {
        h = m >> (64 - sh);
        l = m << sh;
    } else if (sh == 0) {
        l = m;
    } else if (sh > -64) {
        l = m >> (-sh);
    }
    uint64_t nl = *lo + l;
    *hi += h + (nl < *lo ? 1u : 0u);
    *lo = nl;
    return 0;
}

/* R16: the exact fixed-point sum of n weights (out[0] = hi, out[1] = lo)
 * and its double value.  Returns 0, or -1 as q64_add. */
int oracle_q64_sum(const double *w, int64_t n, uint64_t *out, double *value)
{
    uint64_t hi = 0, lo = 0;
    for (int64_t i = 0; i < n; i++)
        if (q64_add(&hi, &lo, w[i]) != 0) return -1;
    out[0] = hi;
    out[1] = lo;
    *value = (double)hi + ((double)(lo >> 32) * 0x1p-32 + (double)(lo & 0xFFFFFFFFULL) * 0x1p-64);
    return 0;
}

typedef struct {
    particle pt;
    int b;
    uint64_t i;   /* history index */
} pc_entry;

typedef struct {
    pc_entry *e;
    size_t n, cap;
} pc_list;

static int pc_push(pc_list *L, const particle *pt, int b, uint64_t i)
{
    if (L->n == L->cap) {
        size_t cap = L->cap ? 2 * L->cap : 1024;
        pc_entry *e = (pc_entry *)realloc(L->e, cap * sizeof(pc_entry));
        if (!e) return -1;
        L->e = e;
        L->cap = cap;
    }
    L->e[L->n].pt = *pt;
    L->e[L->n].b = b;
    L->e[L->n].i = i;
    L->n++;
    return 0;
}

/* R16's conversion of a fixed-point weight sum to a double. */
static double q64_value(uint64_t hi, uint64_t lo)
{
    return (double)hi + ((double)(lo >> 32) * 0x1p-32 + (double)(lo & 0xFFFFFFFFULL) * 0x1p-64);
}

/* R28: teeth of the comb below the fixed-point point (hi, lo). */
static uint64_t comb_teeth(uint64_t hi, uint64_t lo, double dW, uint64_t M, double u)
{
    const double y = (q64_value(hi, lo) / dW) * (double)M - u;
    const double c = ceil(y);
    if (!(c > 0.0)) return 0;
    if (c >= (double)M) return M;
    return (uint64_t)c;
}

/* R28: copies n[r] of n weights w[r] taken in the given order, for M
 * teeth at offset u.  Returns 0, or -1 as q64_add (or an empty total). */
int oracle_comb(const double *w, int64_t n, uint64_t M, double u, uint64_t *out)
{
    uint64_t hi = 0, lo = 0;
    for (int64_t r = 0; r < n; r++)
        if (q64_add(&hi, &lo, w[r]) != 0) return -1;
    if (hi == 0 && lo == 0) return -1;
    const double dW = q64_value(hi, lo);
    uint64_t ph = 0, pl = 0;
    for (int64_t r = 0; r < n; r++) {
        const uint64_t t0 = comb_teeth(ph, pl, dW, M, u);
        q64_add(&ph, &pl, w[r]);
        out[r] = comb_teeth(ph, pl, dW, M, u) - t0;
    }
    return 0;
}

/* R16 / R28: an N-history run with population control to `target`
 * particles at every census edge (method 0: splitting-roulette, R16; 1:
 * combing, R28).  Outputs as oracle_run (totals: roulette terminations
 * include the controlled-away particles, splits the extra copies); pop[k]
 * (k = 0..K-1, may be NULL) receives the particles alive at T_k after the
 * control (pop[0]: particles born).  Returns 0, -1 invalid problem, -3 a
 * problem with windows, fission or a detector, -4 a weight of 2^32 or more,
 * -2 out of memory. */
int oracle_run_pc(const oracle_problem *p, uint64_t N, uint64_t seed, uint64_t target, int method,
                  double *S_out, double *L_out, uint64_t *tot_out, double *X_out, uint64_t *pop)
{
    if (p->ww_center || p->sigma_f || p->qoi_on || target == 0 || method < 0 || method > 1) return -3;
    ctx C;
    if (ctx_init(&C, p) != 0) {
        ctx_free(&C);
        return -1;
    }
    int64_t B = p->n_batches;
    if ((uint64_t)B > N) B = (int64_t)N;
    if (B < 1) B = 1;
    const int G = p->G;
    C.S = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.Sc = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.X = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.Xc = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.L = (double *)calloc((size_t)(B * C.K * G * 6), sizeof(double));
    C.Lc = (double *)calloc((size_t)(B * C.K * G * 6), sizeof(double));
    particle *stack = (particle *)malloc(sizeof(particle) * STACK_MAX);
    pc_list cur = {0}, nxt = {0};
    int rc = 0;
    hist_rec h;
    uint64_t s0 = seed & MASK63;
    if (pop)
        for (int k = 0; k < C.K; k++) pop[k] = 0;
    /* every history is born first, in order */
    for (uint64_t i = 0; i < N && rc == 0; i++) {
        int b = (int)(((i + 1) * (uint64_t)B - 1) / N);
        memset(&h, 0, sizeof(h));
        particle pt;
        if (birth(&C, oracle_rng_skip(s0, i * LCG_STRIDE), &pt, &h)) {
            if (pc_push(&cur, &pt, b, i)) rc = -2;
            if (pop) pop[0]++;
        }
    }
    for (int k = 0; k < C.K && rc == 0; k++) {
        nxt.n = 0;
        /* census step k: track every particle of time bin k to T_{k+1} */
        for (size_t r = 0; r < cur.n && rc == 0; r++) {
            particle pt = cur.e[r].pt;
            const int b = cur.e[r].b;
            const uint64_t hid = cur.e[r].i;
            if (pt.k == k) {
                int sp = 0, alive;
                memset(&h, 0, sizeof(h));
                do {
                    alive = step(&C, &pt, b, stack, &sp, &h, NULL);
                } while (alive > 0 && pt.k == k);
                if (alive < 0 || sp != 0) rc = -3;
                if (alive <= 0) continue;
            }
            if (pc_push(&nxt, &pt, b, hid)) rc = -2;
        }
        if (rc) break;
        /* control at T_{k+1} over its crossers (those with clock k + 1) */
        uint64_t hi = 0, lo = 0;
        for (size_t r = 0; r < nxt.n; r++)
            if (nxt.e[r].pt.k == k + 1 && q64_add(&hi, &lo, nxt.e[r].pt.w) != 0) rc = -4;
        if (rc) break;
        cur.n = 0;
        const double W = q64_value(hi, lo);
        const double wt = W / (double)target;
        /* R28: the comb's copies of each controlled particle, in list
           order (nxt holds the particles in it) */
        uint64_t *ncomb = NULL;
        if (method == 1 && (hi != 0 || lo != 0)) {
            size_t nc = 0;
            size_t *ord = (size_t *)malloc(sizeof(size_t) * (nxt.n ? nxt.n : 1));
            ncomb = (uint64_t *)calloc(nxt.n ? nxt.n : 1, sizeof(uint64_t));
            if (!ord || !ncomb) {
                free(ord);
                rc = -2;
                break;
            }
            for (size_t r = 0; r < nxt.n; r++)
                if (nxt.e[r].pt.k == k + 1) ord[nc++] = r;
            uint64_t su = oracle_child_stream(s0, (1ULL << 62) + (uint64_t)(k + 1));
            const double u = rn(&su);
            uint64_t ph = 0, pl = 0;
            for (size_t q = 0; q < nc; q++) {
                const uint64_t t0 = comb_teeth(ph, pl, W, target, u);
                q64_add(&ph, &pl, nxt.e[ord[q]].pt.w);
                ncomb[ord[q]] = comb_teeth(ph, pl, W, target, u) - t0;
            }
            free(ord);
        }
        uint64_t alive_at = 0;
        for (size_t r = 0; r < nxt.n && rc == 0; r++) {
            particle pt = nxt.e[r].pt;
            const int b = nxt.e[r].b;
            const uint64_t hid = nxt.e[r].i;
            if (pt.k != k + 1 || (hi == 0 && lo == 0)) {
                if (pc_push(&cur, &pt, b, hid)) rc = -2;
                if (pt.k == k + 1) alive_at++;
                continue;
            }
            uint64_t n;
            if (method == 1) {
                n = ncomb[r];
            } else {
                double xi = rn(&pt.s);
                n = (uint64_t)floor(pt.w / wt + xi);
            }
            if (n == 0) {
                C.tot[3 + T_ROULETTE]++;
                continue;
            }
            pt.w = wt;
            const uint64_t sf = pt.s;
            for (uint64_t j = 0; j < n && rc == 0; j++) {
                particle c = pt;
                if (j > 0) {
                    c.s = splitmix64(sf ^ j) & MASK63;
                    C.tot[8]++;
                }
                if (pc_push(&cur, &c, b, hid)) rc = -2;
            }
            alive_at += n;
        }
        free(ncomb);
        if (pop && k + 1 < C.K) pop[k + 1] = alive_at;
    }
    if (rc == 0) {
        if (S_out)
            for (int64_t j = 0; j < B * C.ntally; j++) S_out[j] += C.S[j] + C.Sc[j];
        if (X_out)
            for (int64_t j = 0; j < B * C.ntally; j++) X_out[j] += C.X[j] + C.Xc[j];
        if (L_out)
            for (int64_t j = 0; j < B * C.K * G * 6; j++) L_out[j] += C.L[j] + C.Lc[j];
        if (tot_out)
            for (int j = 0; j < 10; j++) tot_out[j] += C.tot[j];
    }
    free(cur.e);
    free(nxt.e);
    free(stack);
    ctx_free(&C);
    return rc;
}

/* Event-by-event trace of history i (brute-force comparison on tiny inputs):
 * one row of 9 doubles per event, (type, d, x, y, z, t, g, k, tau) after the
 * event, then a final row (type = 10 + termination code).  Analog problems
 * without fission only.  Returns the row count, or -1 if the buffer is too small or the
 * problem is invalid. */
int oracle_trace(const oracle_problem *p, uint64_t N, uint64_t seed, uint64_t i, double *rows, int cap)
{
    ctx C;
    if (ctx_init(&C, p) != 0 || cap < 1 || p->sigma_f) {
        ctx_free(&C);
        return -1;
    }
    int64_t B = p->n_batches;
    if ((uint64_t)B > N) B = (int64_t)N;
    C.S = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.Sc = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.X = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.Xc = (double *)calloc((size_t)(B * C.ntally), sizeof(double));
    C.L = (double *)calloc((size_t)(B * C.K * p->G * 6), sizeof(double));
    C.Lc = (double *)calloc((size_t)(B * C.K * p->G * 6), sizeof(double));
    int b = (int)(((i + 1) * (uint64_t)B - 1) / N);
    hist_rec h;
    memset(&h, 0, sizeof(h));
    particle pt;
    int n = 0;
    int alive = birth(&C, oracle_rng_skip(seed & MASK63, i * LCG_STRIDE), &pt, &h);
    while (alive > 0) {
        if (n + 1 >= cap) {
            ctx_free(&C);
            return -1;
        }
        int sp = 0;
        alive = step(&C, &pt, b, NULL, &sp, &h, &rows[(int64_t)n * 9]);
        n++;
    }
    double *r = &rows[(int64_t)n * 9];
    int code = 0;
    while (!(h.term_mask & (1u << code))) code++;
    r[0] = 10 + code;
    r[1] = 0.0;
    r[2] = pt.x[0];
    r[3] = pt.x[1];
    r[4] = pt.x[2];
    r[5] = pt.t;
    r[6] = pt.g;
    r[7] = pt.k;
    r[8] = pt.tau;
    n++;
    ctx_free(&C);
    return n;
}

/* ------------------------------------------------------------------------ */
/* k-eigenvalue power iteration (R13)                                         */
/* ------------------------------------------------------------------------ */

/*
 * n_inactive + n_active cycles of N particles on a steady-state problem
 * with fission data (no weight windows).  Outputs: raw flux sums
 * S[n_active][ntally] and leak sums L[n_active][K][G][6] of the active
 * cycles (one batch each), k of every cycle k_out[n_inactive + n_active],
 * event and termination totals over all cycles tot[10], and the sites of
 * every cycle per spatial tally bin hist[cycles][nts] (any may be NULL).
 * Returns 0, -1 on an invalid problem (or one without fission, or not
 * steady state), -6 if a cycle banks no site.
 */
int oracle_eigen(const oracle_problem *p, uint64_t N, int n_inactive, int n_active, uint64_t seed,
                 double *S_out, double *L_out, double *k_out, uint64_t *tot_out, uint64_t *hist)
{
    ctx C;
    memset(&C, 0, sizeof(C));
    if (N == 0 || n_inactive < 0 || n_active < 1 || !p->sigma_f || p->ww_center || p->implicit_capture ||
        p->rod_material ||
        ctx_init(&C, p) != 0 || C.K != 1 || p->time_edges[1] != INFINITY) {
        ctx_free(&C);
        return -1;
    }
    const int G = p->G, A = n_active;
    C.eigen = 1;
    C.S = (double *)calloc((size_t)(A * C.ntally), sizeof(double));
    C.Sc = (double *)calloc((size_t)(A * C.ntally), sizeof(double));
    C.X = (double *)calloc((size_t)(A * C.ntally), sizeof(double));
    C.Xc = (double *)calloc((size_t)(A * C.ntally), sizeof(double));
    C.L = (double *)calloc((size_t)(A * G * 6), sizeof(double));
    C.Lc = (double *)calloc((size_t)(A * G * 6), sizeof(double));
    /* sites of the previous and the current cycle, one record per particle */
    double *sx[2];
    int *six[2], *sn[2], *sin[2];
    uint64_t *cum = (uint64_t *)malloc(sizeof(uint64_t) * N);   /* inclusive prefix of sn[prev] */
    for (int r = 0; r < 2; r++) {
        sx[r] = (double *)malloc(sizeof(double) * 3 * N);
        six[r] = (int *)malloc(sizeof(int) * 3 * N);
        sn[r] = (int *)malloc(sizeof(int) * N);
        sin[r] = (int *)malloc(sizeof(int) * N);
    }
    int rc = 0, cur = 0;
    uint64_t M = 0;
    double u = 0.0;
    for (int c = 0; c < n_inactive + n_active && rc == 0; c++) {
        const uint64_t sc = oracle_child_stream(seed & MASK63, (uint64_t)c);
        const int active = c >= n_inactive;
        const int b = active ? c - n_inactive : 0;
        C.quiet = !active;
        const int prev = cur ^ 1;
        for (uint64_t q = 0; q < N; q++) {
            hist_rec h;
            memset(&h, 0, sizeof(h));
            particle pt;
            int alive;
            const uint64_t s0 = oracle_rng_skip(sc, (q + 1) * LCG_STRIDE);
            if (c == 0) {
                alive = birth(&C, s0, &pt, &h);
            } else {
                /* comb over the previous cycle's sites */
                uint64_t idx = (uint64_t)floor(((double)q + u) * (double)M / (double)N);
                if (idx >= M) idx = M - 1;
                uint64_t lo = 0, hi = N - 1;   /* first i with cum[i] > idx */
                while (lo < hi) {
                    uint64_t mid = lo + (hi - lo) / 2;
                    if (cum[mid] > idx) hi = mid; else lo = mid + 1;
                }
                memset(&pt, 0, sizeof(pt));
                pt.s = s0;
                for (int a = 0; a < 3; a++) {
                    pt.x[a] = sx[prev][3 * lo + a];
                    pt.ix[a] = six[prev][3 * lo + a];
                }
                pt.inpin = sin[prev][lo];
                pt.t = p->time_edges[0];
                pt.w = 1.0;
                emit(&C, &pt, material_of(&C, &pt));
                alive = 1;
            }
            C.site_n = 0;
            if (alive) {
                int sp = 0;
                if (track(&C, &pt, b, NULL, &sp, &h) < 0) rc = -4;
            }
            sn[cur][q] = C.site_n;
            sin[cur][q] = C.site_inpin;
            for (int a = 0; a < 3; a++) {
                sx[cur][3 * q + a] = C.site_x[a];
                six[cur][3 * q + a] = C.site_ix[a];
            }
        }
        M = 0;
        for (uint64_t q = 0; q < N; q++) {
            M += (uint64_t)sn[cur][q];
            cum[q] = M;
        }
        if (hist) {
            const int64_t nts = (int64_t)C.nt[0] * C.nt[1] * C.nt[2];
            for (uint64_t q = 0; q < N; q++) {
                if (sn[cur][q] == 0) continue;
                int t[3], inside = 1;
                for (int a = 0; a < 3; a++) {
                    t[a] = (C.ax[a].n == 0) ? 0 : C.ax[a].tal[six[cur][3 * q + a]];
                    if (t[a] < 0) inside = 0;
                }
                if (inside)
                    hist[(int64_t)c * nts + ((int64_t)t[2] * C.nt[1] + t[1]) * C.nt[0] + t[0]] +=
                        (uint64_t)sn[cur][q];
            }
        }
        if (k_out) k_out[c] = (double)M / (double)N;
        if (M == 0) rc = -6;
        uint64_t su = sc;
        u = rn(&su);
        cur ^= 1;
    }
    if (rc == 0) {
        if (S_out)
            for (int64_t j = 0; j < A * C.ntally; j++) S_out[j] += C.S[j] + C.Sc[j];
        if (L_out)
            for (int64_t j = 0; j < A * G * 6; j++) L_out[j] += C.L[j] + C.Lc[j];
        if (tot_out)
            for (int j = 0; j < 10; j++) tot_out[j] += C.tot[j];
    }
    for (int r = 0; r < 2; r++) {
        free(sx[r]);
        free(six[r]);
        free(sn[r]);
        free(sin[r]);
    }
    free(cum);
    ctx_free(&C);
    return rc;
}
