// Problem compilation for the C ABI: validation of the descriptor, the
// per-axis union grid, the per-union-cell tables and the cross-section
// tables, uploaded once into one device allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mcdc_internal.hpp"

namespace mcdc {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return (e == hipErrorOutOfMemory) ? MCDC_E_NOMEM : MCDC_E_HIP;
}

int ensure(mcdc_problem::Buf &b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return MCDC_OK;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    b.bytes = bytes;
    return MCDC_OK;
}

namespace {

int invalid(const std::string &m) {
    set_error("invalid problem: " + m);
    return MCDC_E_INVALID;
}

bool strictly_increasing(const double *a, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    for (int i = 1; i < n; ++i)
        if (!(a[i] > a[i - 1])) return false;
    return true;
}

// index j with E[j] <= x < E[j+1], or -1 outside [E[0], E[n-1])
int bin_of(const std::vector<double> &E, double x) {
    if (E.size() < 2 || x < E.front() || x >= E.back()) return -1;
    return (int)(std::upper_bound(E.begin(), E.end(), x) - E.begin()) - 1;
}

// The LCG map for k steps, s -> A s + C (mod 2^64; callers mask to 63 bits),
// by repeated squaring of the one-step map s -> g s + 1.
void lcg_map(uint64_t k, uint64_t &A, uint64_t &C) {
    const uint64_t g = 2806196910506780709ULL;
    uint64_t a = 1, c = 0, h = g, f = 1;
    while (k) {
        if (k & 1ULL) {
            a = a * h;
            c = c * h + f;
        }
        f = f * (h + 1ULL);
        h = h * h;
        k >>= 1;
    }
    A = a;
    C = c;
}

struct Blob {
    std::vector<char> bytes;
    template <class T>
    size_t add(const std::vector<T> &v) {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + std::max<size_t>(v.size() * sizeof(T), 1));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

int compile(const mcdc_problem_desc *d, HostProblem &h) {
    if (!d) return invalid("descriptor is NULL");
    if (d->abi_version != MCDC_ABI_VERSION) return invalid("abi_version mismatch");
    const int G = d->n_groups, M = d->n_materials;
    if (G < 1 || G > kMaxGroups) return invalid("n_groups must be in [1, 32]");
    if (M < 1) return invalid("n_materials must be >= 1");
    if (!d->sigma_t || !d->sigma_s || !d->speed || !d->material || !d->src_group_pmf ||
        !d->time_edges)
        return invalid("a required array is NULL");
    h.G = G;
    h.M = M;
    h.desc = *d;

    // materials
    h.sigma_t.assign(d->sigma_t, d->sigma_t + (size_t)M * G);
    h.speed.assign(d->speed, d->speed + G);
    h.inv_st.resize((size_t)M * G);
    h.ps.resize((size_t)M * G);
    h.cdf.resize((size_t)M * G * G);
    for (int g = 0; g < G; ++g)
        if (!(h.speed[g] > 0.0) || !std::isfinite(h.speed[g])) return invalid("speed must be > 0");
    for (int m = 0; m < M; ++m)
        for (int g = 0; g < G; ++g) {
            const double st = h.sigma_t[m * G + g];
            if (!(st >= 0.0) || !std::isfinite(st)) return invalid("sigma_t must be finite and >= 0");
            const double *row = d->sigma_s + ((size_t)m * G + g) * G;
            double ss = 0.0;
            int last = -1;
            for (int g2 = 0; g2 < G; ++g2) {
                if (!(row[g2] >= 0.0) || !std::isfinite(row[g2]))
                    return invalid("sigma_s must be finite and >= 0");
                ss += row[g2];
                if (row[g2] > 0.0) last = g2;
            }
            if (ss > st * (1.0 + 1e-12)) return invalid("scattering exceeds sigma_t");
            h.inv_st[m * G + g] = (st > 0.0) ? 1.0 / st : 0.0;
            h.ps[m * G + g] = (st > 0.0) ? ss / st : 0.0;
            double run = 0.0;
            double *cdf = &h.cdf[((size_t)m * G + g) * G];
            for (int g2 = 0; g2 < G; ++g2) {
                run += row[g2];
                cdf[g2] = (ss > 0.0) ? run / ss : 1.0;
            }
            for (int g2 = (last < 0 ? 0 : last); g2 < G; ++g2) cdf[g2] = 1.0;
        }
    h.inv_v.resize(G);
    for (int g = 0; g < G; ++g) h.inv_v[g] = 1.0 / h.speed[g];

    // prompt fission (optional): reaction thresholds, nu, spectrum CDF
    const int nfis = (d->sigma_f != nullptr) + (d->nu != nullptr) + (d->chi != nullptr);
    if (nfis != 0 && nfis != 3) return invalid("fission needs sigma_f, nu and chi together");
    h.fission = nfis == 3;
    if (h.fission) {
        h.pf.resize((size_t)M * G);
        h.nu.assign(d->nu, d->nu + (size_t)M * G);
        h.chi_cdf.resize((size_t)M * G);
        for (int m = 0; m < M; ++m) {
            for (int g = 0; g < G; ++g) {
                const double st = h.sigma_t[m * G + g], sf = d->sigma_f[m * G + g], nu = h.nu[m * G + g];
                if (!(sf >= 0.0) || !std::isfinite(sf)) return invalid("sigma_f must be finite and >= 0");
                if (!(nu >= 0.0) || !(nu <= kMaxNu)) return invalid("nu must be in [0, 64]");
                const double *row = d->sigma_s + ((size_t)m * G + g) * G;
                double ss = 0.0;
                for (int g2 = 0; g2 < G; ++g2) ss += row[g2];
                if (ss + sf > st * (1.0 + 1e-12)) return invalid("scattering plus fission exceeds sigma_t");
                h.pf[m * G + g] = (st > 0.0) ? (ss + sf) / st : 0.0;
            }
            double run = 0.0;
            int last = -1;
            for (int g = 0; g < G; ++g) {
                const double c = d->chi[m * G + g];
                if (!(c >= 0.0) || !std::isfinite(c)) return invalid("chi must be finite and >= 0");
                run += c;
                h.chi_cdf[m * G + g] = run;
                if (c > 0.0) last = g;
            }
            if (last < 0 || std::fabs(run - 1.0) > 1e-12) return invalid("chi must sum to 1 for every material");
            for (int g = last; g < G; ++g) h.chi_cdf[m * G + g] = 1.0;
        }
    }

    // geometry planes and domain
    int ngc[3];
    for (int a = 0; a < 3; ++a) {
        const int n = d->n_planes[a];
        if (n == 1 || n < 0) return invalid("an axis needs 0 or >= 2 planes");
        if (n > 0 && (!d->planes[a] || !strictly_increasing(d->planes[a], n)))
            return invalid("geometry planes must be finite and strictly increasing");
        ngc[a] = (n == 0) ? 1 : n - 1;
        if (n == 0 && (d->n_mesh_planes[a] != 0 || d->n_ww_planes[a] != 0))
            return invalid("mesh or window planes given on an infinite axis");
    }
    const size_t ngeo = (size_t)ngc[0] * ngc[1] * ngc[2];
    for (size_t c = 0; c < ngeo; ++c)
        if (d->material[c] < 0 || d->material[c] >= M) return invalid("material id out of range");
    for (int f = 0; f < 6; ++f)
        if (d->bc[f] != MCDC_VACUUM && d->bc[f] != MCDC_REFLECTIVE) return invalid("bad boundary condition");

    // source
    if (d->src_kind != MCDC_SRC_ISOTROPIC && d->src_kind != MCDC_SRC_SURFACE)
        return invalid("bad source kind");
    if (d->src_kind == MCDC_SRC_SURFACE) {
        if (d->src_axis < 0 || d->src_axis > 2) return invalid("bad source axis");
        if (d->src_sign != 1 && d->src_sign != -1) return invalid("source sign must be +1 or -1");
        if (d->src_mu_law < 0 || d->src_mu_law > 2) return invalid("bad angular law");
    }
    for (int a = 0; a < 3; ++a) {
        if (d->n_planes[a] == 0) continue;
        const double lo = d->planes[a][0], hi = d->planes[a][d->n_planes[a] - 1];
        if (!(d->src_lo[a] <= d->src_hi[a]) || d->src_lo[a] < lo || d->src_hi[a] > hi)
            return invalid("source box outside the domain");
    }
    if (!(d->src_t_lo <= d->src_t_hi) || !std::isfinite(d->src_t_hi))
        return invalid("bad source time window");
    {
        double sum = 0.0;
        int last = -1;
        h.src_cdf.resize(G);
        for (int g = 0; g < G; ++g) {
            const double v = d->src_group_pmf[g];
            if (!(v >= 0.0)) return invalid("group pmf must be >= 0");
            sum += v;
            h.src_cdf[g] = sum;
            if (v > 0.0) last = g;
        }
        if (last < 0 || std::fabs(sum - 1.0) > 1e-12) return invalid("group pmf must sum to 1");
        for (int g = last; g < G; ++g) h.src_cdf[g] = 1.0;
    }

    // time grid
    const int nte = d->n_time_edges;
    if (nte < 2) return invalid("need at least 2 time edges");
    h.K = nte - 1;
    h.T.assign(d->time_edges, d->time_edges + nte);
    for (int k = 0; k < nte; ++k) {
        if (std::isnan(h.T[k]) || (k < nte - 1 && !std::isfinite(h.T[k])))
            return invalid("only the last time edge may be infinite");
        if (k > 0 && !(h.T[k] > h.T[k - 1])) return invalid("time edges must increase");
    }
    if (d->src_t_lo < h.T[0]) return invalid("source emits before the first time edge");
    if (d->n_batches < 1) return invalid("n_batches must be >= 1");
    h.B = d->n_batches;
    if (d->time_crossing != 0 && d->time_crossing != 1) return invalid("time_crossing must be 0 or 1");
    if (d->implicit_capture != 0 && d->implicit_capture != 1) return invalid("implicit_capture must be 0 or 1");
    if (d->implicit_capture) {
        if (d->sigma_f) return invalid("implicit capture is not combined with fission");
        if (!(d->roulette_w > 0.0) || !(d->roulette_ws >= d->roulette_w) || !std::isfinite(d->roulette_ws))
            return invalid("implicit capture needs 0 < roulette_w <= roulette_ws");
    }

    // tally, window and detector planes; union grid per axis
    if (d->qoi_enabled) {
        if (!d->qoi_group_mask) return invalid("detector group mask is NULL");
        h.qoi_groups.resize(G);
        for (int g = 0; g < G; ++g) h.qoi_groups[g] = d->qoi_group_mask[g] ? 1 : 0;
    } else {
        h.qoi_groups.assign(G, 0);
    }
    std::vector<int> geo_of[3], tal_of[3], ww_of[3];
    std::vector<uint8_t> q_of[3];
    std::vector<double> mesh[3];
    h.qoi_volume = 1.0;
    for (int a = 0; a < 3; ++a) {
        const int ng = d->n_planes[a];
        const int nm = d->n_mesh_planes[a];
        const int nw = d->n_ww_planes[a];
        if (nm == 1 || nm < 0 || nw == 1 || nw < 0) return invalid("mesh needs 0 or >= 2 planes");
        if (nm > 0 && (!d->mesh_planes[a] || !strictly_increasing(d->mesh_planes[a], nm)))
            return invalid("mesh planes must be strictly increasing");
        if (nw > 0 && (!d->ww_planes[a] || !strictly_increasing(d->ww_planes[a], nw)))
            return invalid("window planes must be strictly increasing");
        h.nt[a] = (nm == 0) ? 1 : nm - 1;
        h.nw[a] = (nw == 0) ? 1 : nw - 1;
        if (nm > 0) mesh[a].assign(d->mesh_planes[a], d->mesh_planes[a] + nm);
        if (ng == 0) {
            h.nc[a] = 1;
            geo_of[a] = {0};
            tal_of[a] = {0};
            ww_of[a] = {0};
            q_of[a] = {1};
            continue;
        }
        const double lo = d->planes[a][0], hi = d->planes[a][ng - 1];
        std::vector<double> all(d->planes[a], d->planes[a] + ng);
        for (int j = 0; j < nm; ++j) all.push_back(d->mesh_planes[a][j]);
        for (int j = 0; j < nw; ++j) all.push_back(d->ww_planes[a][j]);
        if (d->qoi_enabled) {
            if (!(d->qoi_lo[a] <= d->qoi_hi[a])) return invalid("detector box is inverted");
            all.push_back(d->qoi_lo[a]);
            all.push_back(d->qoi_hi[a]);
            h.qoi_volume *= d->qoi_hi[a] - d->qoi_lo[a];
        }
        for (double v : all)
            if (v < lo || v > hi) return invalid("mesh, window or detector plane outside the domain");
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        h.U[a] = all;
        const int ncell = (int)all.size() - 1;
        if (ncell > ((a == 2) ? 1023 : 2047)) {
            set_error("union grid too fine along an axis (2047 x, 2047 y, 1023 z cells at most)");
            return MCDC_E_UNSUPPORTED;
        }
        h.nc[a] = ncell;
        std::vector<double> geo(d->planes[a], d->planes[a] + ng);
        std::vector<double> ww;
        if (nw > 0) ww.assign(d->ww_planes[a], d->ww_planes[a] + nw);
        geo_of[a].resize(ncell);
        tal_of[a].resize(ncell);
        ww_of[a].resize(ncell);
        q_of[a].resize(ncell);
        for (int i = 0; i < ncell; ++i) {
            const double left = all[i], right = all[i + 1];
            geo_of[a][i] = bin_of(geo, left);
            tal_of[a][i] = (nm == 0) ? 0 : bin_of(mesh[a], left);
            ww_of[a][i] = (nw == 0) ? 0 : bin_of(ww, left);
            q_of[a][i] = d->qoi_enabled ? (left >= d->qoi_lo[a] && right <= d->qoi_hi[a]) : 1;
        }
    }
    // Union-cell, tally-bin and window-cell indices are 32-bit in the device
    // tables and kernels; a grid whose cell count exceeds that is refused
    // before anything is allocated (tally and window meshes never have more
    // cells per axis than the union grid, so one bound covers all three).
    const uint64_t ncells64 = (uint64_t)h.nc[0] * (uint64_t)h.nc[1] * (uint64_t)h.nc[2];
    if (ncells64 > (uint64_t)INT32_MAX) {
        set_error("union grid has more than 2^31 - 1 cells (" + std::to_string(h.nc[0]) + " x " +
                  std::to_string(h.nc[1]) + " x " + std::to_string(h.nc[2]) + ")");
        return MCDC_E_UNSUPPORTED;
    }
    const size_t ncells = (size_t)ncells64;
    h.cell_mat.resize(ncells);
    h.cell_tal.resize(ncells);
    h.cell_ww.resize(ncells);
    h.cell_qoi.resize(ncells);
    for (int iz = 0; iz < h.nc[2]; ++iz)
        for (int iy = 0; iy < h.nc[1]; ++iy)
            for (int ix = 0; ix < h.nc[0]; ++ix) {
                const size_t c = ((size_t)iz * h.nc[1] + iy) * h.nc[0] + ix;
                const int gx = geo_of[0][ix], gy = geo_of[1][iy], gz = geo_of[2][iz];
                h.cell_mat[c] = d->material[((size_t)gz * ngc[1] + gy) * ngc[0] + gx];
                const int tx = tal_of[0][ix], ty = tal_of[1][iy], tz = tal_of[2][iz];
                h.cell_tal[c] = (tx < 0 || ty < 0 || tz < 0) ? -1 : (tz * h.nt[1] + ty) * h.nt[0] + tx;
                const int wx = ww_of[0][ix], wy = ww_of[1][iy], wz = ww_of[2][iz];
                h.cell_ww[c] = (wx < 0 || wy < 0 || wz < 0) ? -1 : (wz * h.nw[1] + wy) * h.nw[0] + wx;
                h.cell_qoi[c] = (q_of[0][ix] && q_of[1][iy] && q_of[2][iz]) ? 1 : 0;
            }
    // cylindrical pins: per union cell, the pin of its geometry cell
    if (d->pin_radius) {
        if (!d->pin_material) return invalid("pins need pin_material");
        if (d->n_planes[0] == 0 || d->n_planes[1] == 0) return invalid("pins need finite x and y axes");
        for (size_t g = 0; g < ngeo; ++g) {
            const int gx = (int)(g % ngc[0]), gy = (int)((g / ngc[0]) % ngc[1]);
            const double r = d->pin_radius[g];
            if (!(r >= 0.0) || !std::isfinite(r)) return invalid("pin radius must be finite and >= 0");
            if (r == 0.0) continue;
            const double hx = 0.5 * (d->planes[0][gx + 1] - d->planes[0][gx]);
            const double hy = 0.5 * (d->planes[1][gy + 1] - d->planes[1][gy]);
            if (!(r < hx) || !(r < hy)) return invalid("a pin must fit inside its cell");
            if (d->pin_material[g] < 0 || d->pin_material[g] >= M) return invalid("pin material out of range");
        }
        h.pins = true;
        h.pin_r2.assign(ncells, 0.0);
        h.pin_xc.assign(ncells, 0.0);
        h.pin_yc.assign(ncells, 0.0);
        h.pin_mat.assign(ncells, 0);
        for (int iz = 0; iz < h.nc[2]; ++iz)
            for (int iy = 0; iy < h.nc[1]; ++iy)
                for (int ix = 0; ix < h.nc[0]; ++ix) {
                    const size_t c = ((size_t)iz * h.nc[1] + iy) * h.nc[0] + ix;
                    const int gx = geo_of[0][ix], gy = geo_of[1][iy], gz = geo_of[2][iz];
                    const size_t g = ((size_t)gz * ngc[1] + gy) * ngc[0] + gx;
                    const double r = d->pin_radius[g];
                    if (!(r > 0.0)) continue;
                    h.pin_r2[c] = r * r;
                    h.pin_xc[c] = 0.5 * (d->planes[0][gx] + d->planes[0][gx + 1]);
                    h.pin_yc[c] = 0.5 * (d->planes[1][gy] + d->planes[1][gy + 1]);
                    h.pin_mat[c] = d->pin_material[g];
                }
    }

    // moving plane: per union cell, the rod material of its geometry cell;
    // the plane's speed in each census step
    if (d->rod_z || d->rod_material) {
        if (!d->rod_z || !d->rod_material) return invalid("a moving plane needs rod_z and rod_material");
        if (d->pin_radius) {
            set_error("a moving plane is not combined with pins");
            return MCDC_E_UNSUPPORTED;
        }
        if (d->n_planes[2] == 0) return invalid("a moving plane needs a finite z axis");
        for (int k = 0; k <= h.K; ++k)
            if (!std::isfinite(d->rod_z[k])) return invalid("rod_z must be finite");
        for (size_t g = 0; g < ngeo; ++g)
            if (d->rod_material[g] < -1 || d->rod_material[g] >= M) return invalid("rod material out of range");
        h.rod = true;
        h.rod_z.assign(d->rod_z, d->rod_z + h.K + 1);
        h.rod_v.assign(h.K, 0.0);
        for (int k = 0; k < h.K; ++k)
            if (std::isfinite(h.T[k + 1])) h.rod_v[k] = (h.rod_z[k + 1] - h.rod_z[k]) / (h.T[k + 1] - h.T[k]);
        h.rod_mat.assign(ncells, -1);
        for (int iz = 0; iz < h.nc[2]; ++iz)
            for (int iy = 0; iy < h.nc[1]; ++iy)
                for (int ix = 0; ix < h.nc[0]; ++ix) {
                    const size_t c = ((size_t)iz * h.nc[1] + iy) * h.nc[0] + ix;
                    const int gx = geo_of[0][ix], gy = geo_of[1][iy], gz = geo_of[2][iz];
                    h.rod_mat[c] = d->rod_material[((size_t)gz * ngc[1] + gy) * ngc[0] + gx];
                }
    }

    // quadric surfaces: one table row per geometry cell that has one; per
    // union cell, the row of its geometry cell and the material inside
    if (d->quadric_coef || d->quadric_material) {
        if (!d->quadric_coef || !d->quadric_material) return invalid("quadrics need quadric_coef and quadric_material");
        if (d->pin_radius || d->rod_z || d->rod_material) {
            set_error("quadric surfaces are not combined with pins or a moving plane");
            return MCDC_E_UNSUPPORTED;
        }
        if (d->n_planes[1] == 0 && d->n_planes[2] == 0) return invalid("quadrics need a finite y or z axis");
        std::vector<int32_t> row(ngeo, -1);
        for (size_t g = 0; g < ngeo; ++g) {
            const int32_t m = d->quadric_material[g];
            if (m < -1 || m >= M) return invalid("quadric material out of range");
            for (int j = 0; j < 10; ++j)
                if (!std::isfinite(d->quadric_coef[10 * g + j])) return invalid("quadric coefficients must be finite");
            if (m < 0) continue;
            row[g] = (int32_t)(h.quad_coef.size() / 10);
            h.quad_coef.insert(h.quad_coef.end(), d->quadric_coef + 10 * g, d->quadric_coef + 10 * g + 10);
        }
        h.quad = true;
        if (h.quad_coef.empty()) h.quad_coef.assign(10, 0.0);
        h.quad_cell.assign(ncells, -1);
        h.quad_mat.assign(ncells, 0);
        for (int iz = 0; iz < h.nc[2]; ++iz)
            for (int iy = 0; iy < h.nc[1]; ++iy)
                for (int ix = 0; ix < h.nc[0]; ++ix) {
                    const size_t c = ((size_t)iz * h.nc[1] + iy) * h.nc[0] + ix;
                    const size_t g = ((size_t)geo_of[2][iz] * ngc[1] + geo_of[1][iy]) * ngc[0] + geo_of[0][ix];
                    h.quad_cell[c] = row[g];
                    if (row[g] >= 0) h.quad_mat[c] = d->quadric_material[g];
                }
    }

    // normalisation: bin volume (product of the widths of meshed axes) and
    // time-bin width (1 for an infinite bin)
    std::vector<double> wdt[3];
    for (int a = 0; a < 3; ++a) {
        if (mesh[a].empty()) {
            wdt[a] = {1.0};
        } else {
            for (size_t j = 0; j + 1 < mesh[a].size(); ++j) wdt[a].push_back(mesh[a][j + 1] - mesh[a][j]);
        }
    }
    h.bin_norm.resize((size_t)h.nt[0] * h.nt[1] * h.nt[2]);
    for (int tz = 0; tz < h.nt[2]; ++tz)
        for (int ty = 0; ty < h.nt[1]; ++ty)
            for (int tx = 0; tx < h.nt[0]; ++tx)
                h.bin_norm[((size_t)tz * h.nt[1] + ty) * h.nt[0] + tx] = (wdt[2][tz] * wdt[1][ty]) * wdt[0][tx];
    h.time_norm.resize(h.K);
    for (int k = 0; k < h.K; ++k) {
        const double dt = h.T[k + 1] - h.T[k];
        h.time_norm[k] = std::isfinite(dt) ? dt : 1.0;
    }
    return MCDC_OK;
}

int upload(mcdc_problem *p) {
    HostProblem &h = p->h;
    Blob b;
    size_t oU[3];
    for (int a = 0; a < 3; ++a) oU[a] = b.add(h.U[a]);
    const size_t o_mat = b.add(h.cell_mat), o_tal = b.add(h.cell_tal), o_ww = b.add(h.cell_ww),
                 o_q = b.add(h.cell_qoi), o_st = b.add(h.sigma_t), o_ist = b.add(h.inv_st),
                 o_ps = b.add(h.ps), o_cdf = b.add(h.cdf), o_v = b.add(h.speed),
                 o_iv = b.add(h.inv_v), o_T = b.add(h.T), o_sc = b.add(h.src_cdf),
                 o_qg = b.add(h.qoi_groups), o_bn = b.add(h.bin_norm), o_tn = b.add(h.time_norm),
                 o_pf = b.add(h.pf), o_nu = b.add(h.nu), o_chi = b.add(h.chi_cdf),
                 o_pr2 = b.add(h.pin_r2), o_pxc = b.add(h.pin_xc), o_pyc = b.add(h.pin_yc),
                 o_pm = b.add(h.pin_mat), o_rz = b.add(h.rod_z), o_rv = b.add(h.rod_v),
                 o_rm = b.add(h.rod_mat), o_qc = b.add(h.quad_cell), o_qk = b.add(h.quad_coef),
                 o_qm = b.add(h.quad_mat);
    std::vector<uint64_t> A(64), C(64);
    lcg_map(kStride, A[0], C[0]);
    for (int j = 1; j < 64; ++j) {
        A[j] = A[j - 1] * A[j - 1];
        C[j] = C[j - 1] * (A[j - 1] + 1ULL);
    }
    const size_t o_A = b.add(A), o_C = b.add(C);

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipMalloc(&p->blob, b.bytes.size());
    if (e != hipSuccess) {
        p->blob = nullptr;
        return hip_fail(e, "hipMalloc(problem tables)");
    }
    p->blob_bytes = b.bytes.size();
    e = hipMemcpy(p->blob, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(problem tables)");

    char *base = (char *)p->blob;
    DevProblem &D = p->d;
    D.G = h.G;
    D.M = h.M;
    D.K = h.K;
    D.finite_mask = 0;
    for (int a = 0; a < 3; ++a) {
        D.nU[a] = (int)h.U[a].size();
        D.nc[a] = h.nc[a];
        D.U[a] = (const double *)(base + oU[a]);
        if (D.nU[a] > 0) D.finite_mask |= 1 << a;
    }
    D.ncells = h.nc[0] * h.nc[1] * h.nc[2];
    D.nts = h.nt[0] * h.nt[1] * h.nt[2];
    D.ntally = (int64_t)h.K * h.G * D.nts;
    D.tc_on = h.desc.time_crossing ? 1 : 0;
    D.tstride = D.ntally * (1 + D.tc_on);
    D.cell_mat = (const int32_t *)(base + o_mat);
    D.cell_tal = (const int32_t *)(base + o_tal);
    D.cell_ww = (const int32_t *)(base + o_ww);
    D.cell_qoi = (const uint8_t *)(base + o_q);
    D.sigma_t = (const double *)(base + o_st);
    D.inv_st = (const double *)(base + o_ist);
    D.ps = (const double *)(base + o_ps);
    D.cdf = (const double *)(base + o_cdf);
    D.speed = (const double *)(base + o_v);
    D.inv_v = (const double *)(base + o_iv);
    D.T = (const double *)(base + o_T);
    D.src_cdf = (const double *)(base + o_sc);
    D.qoi_groups = (const uint8_t *)(base + o_qg);
    D.bin_norm = (const double *)(base + o_bn);
    D.time_norm = (const double *)(base + o_tn);
    D.skipA = (const uint64_t *)(base + o_A);
    D.skipC = (const uint64_t *)(base + o_C);
    const mcdc_problem_desc &d = h.desc;
    for (int f = 0; f < 6; ++f) D.bc[f] = d.bc[f];
    D.src_kind = d.src_kind;
    D.src_axis = d.src_axis;
    D.src_mu_law = d.src_mu_law;
    D.src_sign = (double)d.src_sign;
    for (int a = 0; a < 3; ++a) {
        D.src_lo[a] = d.src_lo[a];
        D.src_hi[a] = d.src_hi[a];
    }
    D.src_t_lo = d.src_t_lo;
    D.src_t_hi = d.src_t_hi;
    D.qoi_on = d.qoi_enabled ? 1 : 0;
    D.ww_center = nullptr;
    D.nww = h.nw[0] * h.nw[1] * h.nw[2];
    D.ww_max_split = 16;
    D.ww_ratio = 5.0;
    D.fission_on = h.fission ? 1 : 0;
    D.pins_on = h.pins ? 1 : 0;
    D.pin_r2 = h.pins ? (const double *)(base + o_pr2) : nullptr;
    D.pin_xc = h.pins ? (const double *)(base + o_pxc) : nullptr;
    D.pin_yc = h.pins ? (const double *)(base + o_pyc) : nullptr;
    D.pin_mat = h.pins ? (const int32_t *)(base + o_pm) : nullptr;
    D.rod_on = h.rod ? 1 : 0;
    D.rod_z = h.rod ? (const double *)(base + o_rz) : nullptr;
    D.rod_v = h.rod ? (const double *)(base + o_rv) : nullptr;
    D.rod_mat = h.rod ? (const int32_t *)(base + o_rm) : nullptr;
    D.quad_on = h.quad ? 1 : 0;
    D.quad_cell = h.quad ? (const int32_t *)(base + o_qc) : nullptr;
    D.quad_coef = h.quad ? (const double *)(base + o_qk) : nullptr;
    D.quad_mat = h.quad ? (const int32_t *)(base + o_qm) : nullptr;
    D.implicit = d.implicit_capture ? 1 : 0;
    D.roulette_w = d.roulette_w;
    D.roulette_ws = d.roulette_ws;
    D.pf = h.fission ? (const double *)(base + o_pf) : nullptr;
    D.nu = h.fission ? (const double *)(base + o_nu) : nullptr;
    D.chi_cdf = h.fission ? (const double *)(base + o_chi) : nullptr;
    return MCDC_OK;
}

void free_buf(mcdc_problem::Buf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

}  // namespace
}  // namespace mcdc

using namespace mcdc;

extern "C" const char *mcdc_last_error(void) { return g_last_error.c_str(); }

extern "C" int mcdc_problem_create(const mcdc_problem_desc *desc, mcdc_problem **out) {
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    mcdc_problem *p = new (std::nothrow) mcdc_problem();
    if (!p) {
        set_error("host allocation failed");
        return MCDC_E_NOMEM;
    }
    int rc = compile(desc, p->h);
    if (rc == MCDC_OK) rc = upload(p);
    if (rc != MCDC_OK) {
        mcdc_problem_destroy(p);
        return rc;
    }
    *out = p;
    return MCDC_OK;
}

extern "C" int mcdc_problem_destroy(mcdc_problem *p) {
    if (!p) return MCDC_OK;
    destroy_graph_cache(p);
    for (void *a : p->aux_streams)
        if (a) (void)hipStreamDestroy((hipStream_t)a);
    for (void *e : p->aux_events)
        if (e) (void)hipEventDestroy((hipEvent_t)e);
    if (p->host_counts) (void)hipHostFree(p->host_counts);
    if (p->blob) (void)hipFree(p->blob);
    if (p->ww_dev) (void)hipFree(p->ww_dev);
    mcdc_problem::Buf *bufs[] = {&p->S, &p->L, &p->qoi_hist, &p->qoi_sums, &p->counters,
                                 &p->overflow, &p->bank, &p->queues, &p->prof,
                                 &p->counters_split, &p->tally_part, &p->mean,
                                 &p->var, &p->raw, &p->leak_mean, &p->leak_var, &p->tc_mean, &p->tc_var, &p->work,
                                 &p->comb};
    for (auto *b : bufs) free_buf(*b);
    for (auto &b : p->split) free_buf(b);
    delete p;
    return MCDC_OK;
}

extern "C" int mcdc_problem_tally_shape(const mcdc_problem *p, int64_t shape[5], int64_t *ntally) {
    if (!p || !shape) return invalid("NULL argument");
    shape[0] = p->h.K;
    shape[1] = p->h.G;
    shape[2] = p->h.nt[2];
    shape[3] = p->h.nt[1];
    shape[4] = p->h.nt[0];
    if (ntally) *ntally = p->d.ntally;
    return MCDC_OK;
}

extern "C" int mcdc_set_weight_windows(mcdc_problem *p, const double *centers, double ratio,
                                       int32_t max_split) {
    if (!p) return invalid("problem is NULL");
    if (!centers) {
        p->d.ww_center = nullptr;
        p->ww_host.clear();
        return MCDC_OK;
    }
    if (!(ratio > 1.0) || !std::isfinite(ratio)) return invalid("window ratio must be > 1");
    if (max_split < 1 || max_split > 64) return invalid("max_split must be in [1, 64]");
    const size_t n = (size_t)p->h.K * p->h.G * p->d.nww;
    p->ww_host.assign(centers, centers + n);
    for (double v : p->ww_host)
        if (!(v >= 0.0) || !std::isfinite(v)) return invalid("window centres must be finite and >= 0");
    if (!p->ww_dev) {
        hipError_t e = hipMalloc(&p->ww_dev, n * sizeof(double));
        if (e != hipSuccess) {
            p->ww_dev = nullptr;
            return hip_fail(e, "hipMalloc(weight windows)");
        }
    }
    hipError_t e = hipMemcpy(p->ww_dev, p->ww_host.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(weight windows)");
    p->d.ww_center = p->ww_dev;
    p->d.ww_ratio = ratio;
    p->d.ww_max_split = max_split;
    return MCDC_OK;
}
