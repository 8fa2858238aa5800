// Device building blocks of the tracker: random numbers, birth sampling,
// distances, collision physics.  Used by the history-based kernel and by
// the event-based kernels, so both forms take identical per-particle
// decisions.  All floating point is IEEE binary64 with contraction off
// (-ffp-contract=off); the only fused multiply-add is the explicit one in
// the position update.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mcdc_internal.hpp"

namespace mcdc {
namespace dev {

constexpr uint64_t kMult = 2806196910506780709ULL;   // 63-bit LCG multiplier
constexpr uint64_t kMask63 = 0x7FFFFFFFFFFFFFFFULL;
constexpr double kInf = __builtin_huge_val();
// A particle with this many events since its last census (or birth) is
// killed as lost: a guard against problems that could trap it forever.
constexpr int kMaxEventsPerStep = 1 << 20;

enum Event : int { kCensus = 0, kSurface = 1, kCollision = 2 };

// Advance the stream and return xi = (s >> 10) * 2^-53 in [0, 1 - 2^-53].
__device__ __forceinline__ double rn(uint64_t &s) {
    s = (kMult * s + 1ULL) & kMask63;
    return (double)(s >> 10) * 0x1p-53;
}

// Start of history i's stream: the base state skipped i * stride steps,
// composing the precomputed maps for stride * 2^j steps over the set bits.
__device__ __forceinline__ uint64_t history_stream(const DevProblem &P, uint64_t seed,
                                                   uint64_t i) {
    uint64_t s = seed & kMask63;
    int j = 0;
    while (i) {
        if (i & 1ULL) s = P.skipA[j] * s + P.skipC[j];
        i >>= 1;
        ++j;
    }
    return s & kMask63;
}

// The stream of the history n after the one whose stream is s (the maps
// compose: history_stream(i + n) = stream_skip(history_stream(i), n)).
__device__ __forceinline__ uint64_t stream_skip(const DevProblem &P, uint64_t s, uint64_t n) {
    int j = 0;
    while (n) {
        if (n & 1ULL) s = P.skipA[j] * s + P.skipC[j];
        n >>= 1;
        ++j;
    }
    return s & kMask63;
}

// SplitMix64 finaliser over parent ^ j (Steele, Lea & Flood, OOPSLA 2014):
// the stream of the j-th split child, masked to 63 bits.
__device__ __forceinline__ uint64_t child_stream(uint64_t parent, uint64_t j) {
    uint64_t z = (parent ^ j) + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return (z ^ (z >> 31)) & kMask63;
}

// Marsaglia (1972): isotropic unit vector from a point in the unit disk.
__device__ __forceinline__ void isotropic(uint64_t &s, double &ux, double &uy, double &uz) {
    for (;;) {
        double a = 2.0 * rn(s) - 1.0;
        double b = 2.0 * rn(s) - 1.0;
        double r = a * a + b * b;
        if (r < 1.0) {
            double q = sqrt(1.0 - r);
            ux = 1.0 - 2.0 * r;
            uy = (2.0 * a) * q;
            uz = (2.0 * b) * q;
            return;
        }
    }
}

// Register-resident particle.
struct Particle {
    double x[3], u[3], iu[3];   // position, direction, 1 / direction
    double t, tau, w;
    int ix[3];
    int g, k;
    int inpin;                  // inside the cell's cylindrical pin or quadric, or
                                // (problems with a moving plane) above the plane in a
                                // rod cell
    uint64_t s;
};

// Material of union cell `cell` for a particle with the given flag: the
// cell's, its pin's inside the pin, its quadric's on the negative side,
// its rod's above the moving plane.
__device__ __forceinline__ int material_at(const DevProblem &P, int cell, int flag) {
    if (flag) {
        if (P.pins_on) return P.pin_mat[cell];
        if (P.quad_on) return P.quad_mat[cell];
        if (P.rod_on && P.rod_mat[cell] >= 0) return P.rod_mat[cell];
    }
    return P.cell_mat[cell];
}
__device__ __forceinline__ int material_of(const DevProblem &P, const Particle &p, int cell) {
    return material_at(P, cell, p.inpin);
}

// Moving plane: height at the particle's time in its census step, and the
// rate at which the particle closes on it per unit track length when it
// rises by u_z and the plane by v_k / v_g.
__device__ __forceinline__ double rod_height(const DevProblem &P, const Particle &p) {
    return P.rod_z[p.k] + P.rod_v[p.k] * (p.t - P.T[p.k]);
}
__device__ __forceinline__ double rod_rate(const DevProblem &P, const Particle &p) {
    return p.u[2] - P.rod_v[p.k] * P.inv_v[p.g];
}
// The side of the plane the particle is on (1 above): on the plane, the
// side it moves to.
__device__ __forceinline__ int rod_side(const DevProblem &P, const Particle &p) {
    const double Z = rod_height(P, p);
    if (p.x[2] > Z) return 1;
    if (p.x[2] < Z) return 0;
    return rod_rate(P, p) > 0.0 ? 1 : 0;
}

// Quadric along the flight: Q(x + d u) = a d^2 + 2 b d + c for the
// coefficients q = A B C D E F G H J K of
// A x^2 + B y^2 + C z^2 + D x y + E y z + F z x + G x + H y + J z + K.  The
// sums are taken in one fixed order (square terms, then cross terms, then
// linear terms), so every form of the kernels rounds them alike.
struct QuadLine {
    double a, b, c;
};
__device__ __forceinline__ QuadLine quad_line(const double *q, const Particle &p) {
    const double x = p.x[0], y = p.x[1], z = p.x[2];
    const double ux = p.u[0], uy = p.u[1], uz = p.u[2];
    QuadLine l;
    l.a = ((q[0] * ux * ux + q[1] * uy * uy) + q[2] * uz * uz) + ((q[3] * ux * uy + q[4] * uy * uz) + q[5] * uz * ux);
    l.b = ((q[0] * x * ux + q[1] * y * uy) + q[2] * z * uz) +
          0.5 * (((q[3] * (x * uy + y * ux) + q[4] * (y * uz + z * uy)) + q[5] * (z * ux + x * uz)) +
                 ((q[6] * ux + q[7] * uy) + q[8] * uz));
    l.c = (((q[0] * x * x + q[1] * y * y) + q[2] * z * z) + ((q[3] * x * y + q[4] * y * z) + q[5] * z * x)) +
          (((q[6] * x + q[7] * y) + q[8] * z) + q[9]);
    return l;
}
// The side of the quadric the particle is on (1 negative): on it, the side
// it moves to.
__device__ __forceinline__ int quad_side(const double *q, const Particle &p) {
    const QuadLine l = quad_line(q, p);
    return (l.c < 0.0 || (l.c == 0.0 && l.b < 0.0)) ? 1 : 0;
}
// Distance to the quadric from the side the flag names: the root the
// flight reaches first on leaving (inside) or entering (outside), or
// infinity when it reaches none.
__device__ __forceinline__ double quad_distance(const double *q, const Particle &p) {
    const QuadLine l = quad_line(q, p);
    const double disc = l.b * l.b - l.a * l.c;
    double d = kInf;
    if (p.inpin) {
        if (l.a > 0.0)
            d = (-l.b + sqrt(disc > 0.0 ? disc : 0.0)) / l.a;
        else if (l.a < 0.0) {
            if (l.b > 0.0 && disc > 0.0) d = (-l.b + sqrt(disc)) / l.a;
        } else if (l.b > 0.0) {
            d = -l.c / (2.0 * l.b);
        }
    } else {
        if (l.a > 0.0) {
            if (l.b < 0.0 && disc > 0.0) d = (-l.b - sqrt(disc)) / l.a;
        } else if (l.a < 0.0) {
            if (disc > 0.0) d = (-l.b - sqrt(disc)) / l.a;
        } else if (l.b < 0.0) {
            d = -l.c / (2.0 * l.b);
        }
    }
    return d < 0.0 ? 0.0 : d;
}

template <int FM>
__device__ __forceinline__ bool finite_axis(const DevProblem &P, int a) {
    if constexpr (FM != 0) return (FM >> a) & 1;
    return (P.finite_mask >> a) & 1;
}

// 1 / u along the finite axes (recomputed whenever the direction changes;
// a reflection negates it, which is exact).
template <int FM>
__device__ __forceinline__ void set_inverse(const DevProblem &P, Particle &p) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (finite_axis<FM>(P, a)) p.iu[a] = 1.0 / p.u[a];
}

__device__ __forceinline__ int cell_index(const DevProblem &P, const int ix[3]) {
    return (ix[2] * P.nc[1] + ix[1]) * P.nc[0] + ix[0];
}

// Birth cell along an axis: the i with U_i <= x < U_{i+1}; born exactly on
// U_i moving towards -axis belongs to cell i-1; clamped to the domain.
__device__ __forceinline__ int locate(const double *U, int n, double x, double u) {
    int i = -1;
    for (int j = 0; j < n; ++j)
        if (U[j] <= x) i = j;
    if (i >= 0 && x == U[i] && u < 0.0) i = i - 1;
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    return i;
}

// Sample the source particle of a history (draw order: x, y, z, t, group,
// direction, optical depth).  Returns false if it is born at or after the
// last time edge (time cut-off with no events).
template <int FM>
__device__ __forceinline__ bool birth(const DevProblem &P, uint64_t s0, Particle &p) {
    p.s = s0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double xi = rn(p.s);
        p.x[a] = finite_axis<FM>(P, a) ? P.src_lo[a] + xi * (P.src_hi[a] - P.src_lo[a]) : 0.0;
    }
    double xt = rn(p.s);
    p.t = P.src_t_lo + xt * (P.src_t_hi - P.src_t_lo);
    double xg = rn(p.s);
    int g = 0;
    while (!(xg < P.src_cdf[g])) ++g;
    p.g = g;
    if (P.src_kind == MCDC_SRC_ISOTROPIC) {
        isotropic(p.s, p.u[0], p.u[1], p.u[2]);
    } else {
        double xm = rn(p.s);
        double mu = (P.src_mu_law == MCDC_MU_BEAM) ? 1.0
                    : (P.src_mu_law == MCDC_MU_UNIFORM) ? 1.0 - xm
                                                         : sqrt(1.0 - xm);
        double a, b, r;
        for (;;) {
            a = 2.0 * rn(p.s) - 1.0;
            b = 2.0 * rn(p.s) - 1.0;
            r = a * a + b * b;
            if (r > 0.0 && r < 1.0) break;
        }
        double cph = (a * a - b * b) / r;
        double sph = ((2.0 * a) * b) / r;
        double sn = sqrt(1.0 - mu * mu);
        double v0 = P.src_sign * mu, v1 = sn * cph, v2 = sn * sph;
        if (P.src_axis == 0) {
            p.u[0] = v0; p.u[1] = v1; p.u[2] = v2;
        } else if (P.src_axis == 1) {
            p.u[1] = v0; p.u[2] = v1; p.u[0] = v2;
        } else {
            p.u[2] = v0; p.u[0] = v1; p.u[1] = v2;
        }
    }
    set_inverse<FM>(P, p);
    p.tau = -log(1.0 - rn(p.s));
    p.w = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        p.ix[a] = finite_axis<FM>(P, a) ? locate(P.U[a], P.nU[a], p.x[a], p.u[a]) : 0;
    p.inpin = 0;
    if (FM != 1 && P.pins_on) {
        const int cell = cell_index(P, p.ix);
        const double r2 = P.pin_r2[cell];
        if (r2 > 0.0) {
            const double dx = p.x[0] - P.pin_xc[cell], dy = p.x[1] - P.pin_yc[cell];
            p.inpin = ((dx * dx + dy * dy) - r2) < 0.0;
        }
    }
    if (FM != 1 && P.quad_on) {
        const int qi = P.quad_cell[cell_index(P, p.ix)];
        if (qi >= 0) p.inpin = quad_side(P.quad_coef + 10 * qi, p);
    }
    if (p.t >= P.T[P.K]) {
        p.k = P.K;
        return false;
    }
    int k = 0;
    while (!(p.t < P.T[k + 1])) ++k;
    p.k = k;
    if (FM != 1 && P.rod_on && P.rod_mat[cell_index(P, p.ix)] >= 0) p.inpin = rod_side(P, p);
    return true;
}

// Distances to the next collision, union plane (per axis) and census edge;
// picks the event with the tie order census, surface, collision.
struct Flight {
    double d;
    double da[3];
    double st;
    int ev;
    int m;
};

template <int FM>
__device__ __forceinline__ Flight next_event(const DevProblem &P, const Particle &p, int cell) {
    Flight f;
    f.m = (FM != 1) ? material_of(P, p, cell) : P.cell_mat[cell];
    const int mg = f.m * P.G + p.g;
    f.st = P.sigma_t[mg];
    double dc = (f.st == 0.0) ? kInf : p.tau * P.inv_st[mg];
    double ds = kInf;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f.da[a] = kInf;
        if (!finite_axis<FM>(P, a) || p.u[a] == 0.0) continue;
        double pl = (p.u[a] > 0.0) ? P.U[a][p.ix[a] + 1] : P.U[a][p.ix[a]];
        double d = (pl - p.x[a]) * p.iu[a];
        if (d < 0.0) d = 0.0;
        f.da[a] = d;
        if (d < ds) ds = d;
    }
    // the cell's pin (x-y quadratic; a slab has none): from inside, the far
    // root; from outside, the near root if the flight closes in on the axis;
    // or, in a rod cell, the moving plane when the particle closes in on it
    double dcyl = kInf;
    if (FM != 1 && P.rod_on && P.rod_mat[cell] >= 0) {
        const double q = rod_rate(P, p);
        if ((p.inpin && q < 0.0) || (!p.inpin && q > 0.0)) {
            dcyl = (rod_height(P, p) - p.x[2]) / q;
            if (dcyl < 0.0) dcyl = 0.0;
        }
    }
    if (FM != 1 && P.pins_on) {
        const double r2 = P.pin_r2[cell];
        if (r2 > 0.0) {
            const double dx = p.x[0] - P.pin_xc[cell], dy = p.x[1] - P.pin_yc[cell];
            const double a = p.u[0] * p.u[0] + p.u[1] * p.u[1];
            const double b = dx * p.u[0] + dy * p.u[1];
            const double c = (dx * dx + dy * dy) - r2;
            if (a > 0.0) {
                if (p.inpin) {
                    double disc = b * b - a * c;
                    if (disc < 0.0) disc = 0.0;
                    dcyl = (-b + sqrt(disc)) / a;
                } else if (b < 0.0) {
                    const double disc = b * b - a * c;
                    if (disc > 0.0) dcyl = (-b - sqrt(disc)) / a;
                }
                if (dcyl < 0.0) dcyl = 0.0;
            }
        }
    }
    // the cell's quadric (a problem has pins, quadrics or a moving plane)
    if (FM != 1 && P.quad_on) {
        const int qi = P.quad_cell[cell];
        if (qi >= 0) dcyl = quad_distance(P.quad_coef + 10 * qi, p);
    }
    double Tn = P.T[p.k + 1];
    double dt = kInf;
    if (Tn != kInf) {
        dt = (Tn - p.t) * P.speed[p.g];
        if (dt < 0.0) dt = 0.0;
    }
    // tie order: census, planes, pin, quadric or moving plane, collision (a
    // crossing of one of those is a surface event that crosses no plane)
    if (dt <= ds && dt <= dcyl && dt <= dc) {
        f.ev = kCensus;
        f.d = dt;
    } else if (ds <= dcyl && ds <= dc) {
        f.ev = kSurface;
        f.d = ds;
    } else if (dcyl <= dc) {
        f.ev = kSurface;
        f.d = dcyl;
    } else {
        f.ev = kCollision;
        f.d = dc;
    }
    return f;
}

// Move along the flight (positions, time, optical depth).
template <int FM>
__device__ __forceinline__ void move(const DevProblem &P, Particle &p, const Flight &f) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (finite_axis<FM>(P, a)) p.x[a] = __builtin_fma(f.d, p.u[a], p.x[a]);
    if (f.ev == kCensus)
        p.t = P.T[p.k + 1];
    else
        p.t = p.t + f.d * P.inv_v[p.g];
    if (f.ev != kCollision && f.st != 0.0) {
        p.tau = p.tau - f.d * f.st;
        if (p.tau < 0.0) p.tau = 0.0;
    }
}

// Axes whose plane distance equals the flight: they all cross in this one
// surface event.
template <int FM>
__device__ __forceinline__ int crossing_mask(const DevProblem &P, const Flight &f) {
    int m = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (finite_axis<FM>(P, a) && f.da[a] == f.d) m |= 1 << a;
    return m;
}

// Surface crossing of the axes in mask, in axis order: snap onto the plane,
// step the cell index, reflect at a reflective face.  Returns the vacuum
// face crossed (the particle leaks; later axes are not processed), or -1.
// With a moving plane, a crossing that enters a rod cell from a cell that
// is not one sets the above flag from the particle's side of the plane;
// between rod cells the flag is kept.  With quadrics, a crossing that lands
// in another geometry cell sets the inside flag from that cell's quadric
// (0 where it has none); within a geometry cell the flag is kept.
template <int FM>
__device__ __forceinline__ int cross(const DevProblem &P, Particle &p, int mask) {
    if (FM != 1 && mask == 0) {   // the cell's pin, quadric or moving plane (a slab has none)
        p.inpin ^= 1;
        return -1;
    }
    const bool rod_before = (FM != 1 && P.rod_on) ? P.rod_mat[cell_index(P, p.ix)] >= 0 : false;
    const int quad_before = (FM != 1 && P.quad_on) ? P.quad_cell[cell_index(P, p.ix)] : -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!finite_axis<FM>(P, a) || !((mask >> a) & 1)) continue;
        // (each face's boundary condition is read with a constant index, so
        // a local copy of the problem stays in registers)
        int face = -1;
        bool vacuum = false;
        if (p.u[a] > 0.0) {
            p.x[a] = P.U[a][p.ix[a] + 1];
            if (p.ix[a] == P.nU[a] - 2) {
                face = 2 * a + 1;
                vacuum = P.bc[2 * a + 1] == MCDC_VACUUM;
            } else {
                p.ix[a] += 1;
            }
        } else {
            p.x[a] = P.U[a][p.ix[a]];
            if (p.ix[a] == 0) {
                face = 2 * a;
                vacuum = P.bc[2 * a] == MCDC_VACUUM;
            } else {
                p.ix[a] -= 1;
            }
        }
        if (face >= 0) {
            if (vacuum) return face;
            p.u[a] = -p.u[a];
            p.iu[a] = -p.iu[a];
        }
    }
    if (FM != 1 && P.rod_on) {
        if (P.rod_mat[cell_index(P, p.ix)] < 0)
            p.inpin = 0;
        else if (!rod_before)
            p.inpin = rod_side(P, p);
    }
    if (FM != 1 && P.quad_on) {
        const int qi = P.quad_cell[cell_index(P, p.ix)];
        if (qi != quad_before) p.inpin = (qi >= 0) ? quad_side(P.quad_coef + 10 * qi, p) : 0;
    }
    return -1;
}

// Collision in material m.  Analog: one draw picks the reaction: scatter
// below sigma_s / sigma_t, fission below (sigma_s + sigma_f) / sigma_t
// (FIS kernels only), else capture.  Implicit capture (FIS kernels only):
// no capture; the weight is multiplied by sigma_s / sigma_t and, below the
// roulette threshold, one draw keeps the particle with probability
// w / w_s at weight w_s.  Returns 0 on capture; 1 on a scatter, after
// which the particle has its outgoing group, a new isotropic direction and
// a new optical depth; 2 on a fission, whose neutrons fission() then
// emits; 3 when the roulette ends the particle.
template <int FM, bool FIS = false>
__device__ __forceinline__ int collide(const DevProblem &P, Particle &p, int m) {
    const int mg = m * P.G + p.g;
    if (FIS && P.implicit) {
        p.w = p.w * P.ps[mg];
        if (p.w < P.roulette_w) {
            if (rn(p.s) < p.w / P.roulette_ws)
                p.w = P.roulette_ws;
            else
                return 3;
        }
    } else {
        const double xr = rn(p.s);
        if (!(xr < P.ps[mg])) return (FIS && P.fission_on && xr < P.pf[mg]) ? 2 : 0;
    }
    double xg = rn(p.s);
    const double *cdf = P.cdf + (int64_t)mg * P.G;
    int g2 = 0;
    while (!(xg < cdf[g2])) ++g2;
    p.g = g2;
    isotropic(p.s, p.u[0], p.u[1], p.u[2]);
    set_inverse<FM>(P, p);
    p.tau = -log(1.0 - rn(p.s));
    return 1;
}

// Weight-window centre of a cell for the particle's (k, g), 0 = none.
__device__ __forceinline__ double ww_centre(const DevProblem &P, int cell, int g, int k) {
    if (P.ww_center == nullptr) return 0.0;
    int c = P.cell_ww[cell];
    if (c < 0) return 0.0;
    return P.ww_center[((int64_t)k * P.G + g) * P.nww + c];
}

// Weight-window game at a check point (after a scatter, a census, or a
// surface crossing into a new window cell).  Returns false if the particle
// loses the roulette.  On a split the particle keeps weight w / n and
// n_children = n - 1 copies are to be made, child j taking the stream
// child_stream(s, j) of the particle's current state s.
__device__ __forceinline__ bool ww_check(const DevProblem &P, Particle &p, int cell, int &n_children) {
    n_children = 0;
    const double wc = ww_centre(P, cell, p.g, p.k);
    if (wc == 0.0) return true;
    const double rho = P.ww_ratio;
    const double wl = (2.0 * wc) / (1.0 + rho);
    const double wu = rho * wl;
    if (p.w > wu) {
        const double nr = ceil(p.w / wu);
        const int n = (nr > (double)P.ww_max_split) ? P.ww_max_split : (int)nr;
        if (n > 1) {
            p.w = p.w / (double)n;
            n_children = n - 1;
        }
    } else if (p.w < wl) {
        const double xi = rn(p.s);
        if (xi < p.w / wc)
            p.w = wc;
        else
            return false;
    }
    return true;
}

// Structure-of-arrays bank of split progeny (whole particle states).
struct SplitBank {
    double *x[3], *u[3], *t, *tau, *w;
    uint64_t *s;
    uint32_t *ixyz, *gk;      // gk = g | batch << 5 | k << 15 | inside pin << 31
    uint64_t *hid;            // global history index
    unsigned long long *count;  // device counter of entries asked for (64-bit: it
                                // keeps counting past cap on overflow, never wraps)
    unsigned int cap;
};

__device__ __forceinline__ void split_store(const SplitBank &B, unsigned int slot, const Particle &p, int b,
                                            uint64_t hid) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        B.x[a][slot] = p.x[a];
        B.u[a][slot] = p.u[a];
    }
    B.t[slot] = p.t;
    B.tau[slot] = p.tau;
    B.w[slot] = p.w;
    B.s[slot] = p.s;
    B.ixyz[slot] = (uint32_t)p.ix[0] | ((uint32_t)p.ix[1] << 11) | ((uint32_t)p.ix[2] << 22);
    B.gk[slot] = (uint32_t)p.g | ((uint32_t)b << 5) | ((uint32_t)p.k << 15) | ((uint32_t)p.inpin << 31);
    B.hid[slot] = hid;
}

__device__ __forceinline__ void split_load(const SplitBank &B, unsigned int slot, Particle &p, int &b,
                                           uint64_t &hid) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.x[a] = B.x[a][slot];
        p.u[a] = B.u[a][slot];
    }
    p.t = B.t[slot];
    p.tau = B.tau[slot];
    p.w = B.w[slot];
    p.s = B.s[slot];
    const uint32_t c = B.ixyz[slot];
    p.ix[0] = c & 2047u;
    p.ix[1] = (c >> 11) & 2047u;
    p.ix[2] = c >> 22;
    const uint32_t gk = B.gk[slot];
    p.g = gk & 31u;
    b = (gk >> 5) & 1023u;
    p.k = (gk >> 15) & 0xFFFFu;
    p.inpin = (int)(gk >> 31);
    hid = B.hid[slot];
}

// A fission neutron in material m draws from its own stream its group from
// the fission spectrum, an isotropic direction and an optical depth.
template <int FM>
__device__ __forceinline__ void fission_emit(const DevProblem &P, Particle &p, int m) {
    const double xg = rn(p.s);
    const double *cdf = P.chi_cdf + (int64_t)m * P.G;
    int g = 0;
    while (!(xg < cdf[g])) ++g;
    p.g = g;
    isotropic(p.s, p.u[0], p.u[1], p.u[2]);
    set_inverse<FM>(P, p);
    p.tau = -log(1.0 - rn(p.s));
}

// Prompt fission of p (group p.g) in material m: n = floor(nu + xi)
// neutrons at the collision point and time.  Neutron j = 1..n-1 takes the
// stream child_stream(s, j) of the state s after that draw and goes whole
// to the split bank (overflow sets *overflow); neutron 0 is p itself.
// Returns n (0: p is absorbed).
template <int FM>
__device__ __forceinline__ int fission(const DevProblem &P, Particle &p, int m, const SplitBank &SB, int b,
                                       uint64_t hid, int *overflow) {
    const int n = (int)floor(P.nu[(int64_t)m * P.G + p.g] + rn(p.s));
    if (n <= 0) return 0;
    const uint64_t sf = p.s;
    if (n > 1) {
        const unsigned long long base = atomicAdd(SB.count, (unsigned long long)(n - 1));
        if (base + (unsigned long long)(n - 1) > SB.cap) {
            *overflow = 1;
        } else {
            for (int j = 1; j < n; ++j) {
                Particle c = p;
                c.s = child_stream(sf, (uint64_t)j);
                fission_emit<FM>(P, c, m);
                split_store(SB, (unsigned int)base + j - 1, c, b, hid);
            }
        }
    }
    fission_emit<FM>(P, p, m);
    return n;
}

// Append the n_children split copies of p (streams child_stream(p.s, j),
// j = 1..n_children) to the split bank.  Returns false on overflow.
__device__ __forceinline__ bool spawn_children(const SplitBank &B, const Particle &p, int n_children, int b,
                                               uint64_t hid) {
    if (n_children <= 0) return true;
    const unsigned long long base = atomicAdd(B.count, (unsigned long long)n_children);
    if (base + (unsigned long long)n_children > B.cap) return false;
    Particle c = p;
    for (int j = 1; j <= n_children; ++j) {
        c.s = child_stream(p.s, (uint64_t)j);
        split_store(B, base + j - 1, c, b, hid);
    }
    return true;
}

__device__ __forceinline__ void atomic_add_f64(double *a, double v) {
    unsafeAtomicAdd(a, v);
}

// The tally copy of batch b this workgroup adds into.  Consecutive
// workgroups go to different XCDs, so with X a multiple of 8 each copy is
// touched by one XCD's L2 only, and concurrent flights of the same batch
// spread their atomics over X addresses per bin.
// (The copy holds the track-length tally, then the time-crossing tally.)
__device__ __forceinline__ double *tally_copy(const DevProblem &P, const RunArgs &R, int b) {
    return R.S + ((int64_t)b * R.X + (int64_t)(blockIdx.x & (unsigned)(R.X - 1))) * P.tstride;
}

// Weight leaked through a face, into this workgroup's copy of the leakage
// tally (a handful of bins per batch that every leaking particle hits).
__device__ __forceinline__ void add_leak(const DevProblem &P, const RunArgs &R, int b, int k, int g, int face,
                                         double w) {
    const int64_t nl = (int64_t)P.K * P.G * 6;
    double *L = R.L + ((int64_t)b * R.XL + (int64_t)(blockIdx.x & (unsigned)(R.XL - 1))) * nl;
    atomic_add_f64(L + ((int64_t)k * P.G + g) * 6 + face, w);
}


// Read-only tables a kernel may copy into LDS at its start: union planes,
// time edges, cross sections, speeds, per-cell material and tally bin.
template <int BS, class T>
__device__ __forceinline__ const T *stage(const T *src, const LdsTables &lt, int id, char *base) {
    T *dst = reinterpret_cast<T *>(base + lt.off[id]);
    for (int j = threadIdx.x; j < lt.count[id]; j += BS) dst[j] = src[j];
    return dst;
}

// The problem as a kernel sees it: with LT every staged table is read from
// LDS at base (the copies need a barrier before use), else from P0.
template <bool LT, int BS>
__device__ __forceinline__ DevProblem stage_tables(const DevProblem &P0, const LdsTables &lt, char *base) {
    DevProblem P = P0;
    if (LT) {
        P.U[0] = stage<BS>(P0.U[0], lt, kTU0, base);
        P.U[1] = stage<BS>(P0.U[1], lt, kTU1, base);
        P.U[2] = stage<BS>(P0.U[2], lt, kTU2, base);
        P.T = stage<BS>(P0.T, lt, kTT, base);
        P.sigma_t = stage<BS>(P0.sigma_t, lt, kTSt, base);
        P.inv_st = stage<BS>(P0.inv_st, lt, kTISt, base);
        P.ps = stage<BS>(P0.ps, lt, kTPs, base);
        P.cdf = stage<BS>(P0.cdf, lt, kTCdf, base);
        P.speed = stage<BS>(P0.speed, lt, kTV, base);
        P.inv_v = stage<BS>(P0.inv_v, lt, kTIV, base);
        P.cell_mat = stage<BS>(P0.cell_mat, lt, kTMat, base);
        P.cell_tal = stage<BS>(P0.cell_tal, lt, kTTal, base);
    }
    return P;
}

}  // namespace dev

// Layout of the staged tables within `budget` bytes; false if they do not
// fit.
inline bool table_layout(const DevProblem &P, LdsTables &t, int64_t budget) {
    const int64_t mg = (int64_t)P.M * P.G;
    const int64_t cnt[kTabs] = {P.nU[0], P.nU[1], P.nU[2], P.K + 1, mg, mg, mg, mg * P.G, P.G, P.G, P.ncells, P.ncells};
    const int64_t size[kTabs] = {8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 4, 4};
    int64_t off = 0;
    for (int j = 0; j < kTabs; ++j) {
        t.off[j] = (int)off;
        t.count[j] = (int)cnt[j];
        off += (cnt[j] * size[j] + 15) & ~(int64_t)15;
        if (off > budget) return false;
    }
    t.bytes = (int)off;
    return true;
}

// Split bank of the weight-window game (k_history.hip): carve two
// generations' banks for chunks of up to `chunk` histories, clear the first
// generation's count, and track every generation of progeny of a chunk.
int split_prepare(mcdc_problem *pb, uint64_t chunk, dev::SplitBank SB[2]);
int split_prepare_slots(mcdc_problem *pb, uint64_t chunk, dev::SplitBank (*SB)[2], int slots);
void split_reset(const dev::SplitBank SB[2], hipStream_t st);
int split_generations(mcdc_problem *pb, const RunArgs &R, dev::SplitBank SB[2], uint64_t cfirst, hipStream_t st,
                      Profiler &prof);

}  // namespace mcdc
