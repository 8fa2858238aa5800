"""Seeded synthetic problem generators for the multigroup time-dependent
fixed-source transport problems this project solves.

This module only *describes* problems: cross sections, plane positions,
material maps, source and tally definitions, as plain NumPy arrays in a dict.
It holds none of the transport method's arithmetic (no union grid, no derived
tables, no sampling), so that both the GPU library and the CPU oracle can be
fed from it without sharing any of their computation.

Random problem content (cross sections, material masks, problem sizes) is
drawn from SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) implemented here in plain Python integers, so
the generated problems do not depend on the NumPy version.

Problem dict schema (all floats are float64, all ints int32):

    sigma_t   [M, G]      total cross section per material and group
    sigma_s   [M, G, G]   scattering cross section, row g = from, col g' = to
    speed     [G]         particle speed per group
    planes    list of 3 arrays: geometry planes per axis (x, y, z), strictly
              increasing; an empty array means the axis is infinite
    material  [nz, ny, nx] material id of each geometry cell (an infinite
              axis has one cell)
    bc        [6]         boundary condition of the faces x-, x+, y-, y+, z-,
              z+: 0 = vacuum, 1 = reflective
    source    dict: lo[3], hi[3] (box; a degenerate extent is a point or a
              plane), t_lo, t_hi (emission time window), group_pmf[G],
              kind 'isotropic' (volume/point, isotropic) or 'surface'
              (axis, sign = direction of the inward normal, mu_law in
              'beam' | 'uniform' | 'cosine')
    tally     dict: mesh list of 3 arrays (empty = one bin spanning the
              axis), time_edges[K+1] (last may be +inf), n_batches,
              time_crossing (bool: also tally the flux at the time edges
              T_1..T_K with the time-crossing estimator)
    qoi       None or dict: lo[3], hi[3], group_mask[G]
    fission   None or dict: sigma_f[M, G], nu[M, G] (mean neutrons per
              fission), chi[M, G] (fission spectrum per material)
    implicit_capture
              None or dict: w_min (roulette threshold > 0), w_survive
              (roulette survival weight >= w_min)
    pins      None or dict: radius [nz, ny, nx] (a cylinder parallel to z
              centred in each geometry cell's x-y rectangle, 0 = none) and
              material [nz, ny, nx] (the material inside it)
    rod       None or dict: z [K+1] heights of a plane normal to z at the
              time edges (linear in time between them) and material
              [nz, ny, nx] (the material above the plane in each geometry
              cell, -1 = the cell's own material on both sides)
    quadrics  None or dict: coef [nz, ny, nx, 10] (A..K of the quadric
              A x^2 + B y^2 + C z^2 + D xy + E yz + F zx + G x + H y + J z
              + K in each geometry cell) and material [nz, ny, nx] (the
              material where it is negative, -1 = no quadric)
    ww_mesh   None or list of 3 arrays of weight-window mesh planes

The workload recipes follow the transport problems the method is exercised
on (Section 3): slab benchmarks with closed forms, a pulsed slab (the
time-dependent, AZURV1-like pulse with c < 1), a C5G7-like 17x17 lattice with
synthetic multigroup data, a batch of random lattices, and a Kobayashi-like
dog-leg duct. None of these reproduce benchmark data; all are synthetic.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1

VACUUM = 0
REFLECTIVE = 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood 2014), Python integers."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] inclusive."""
        return lo + self.next_u64() % (hi - lo + 1)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _empty():
    return np.zeros(0, dtype=np.float64)


def make_problem(sigma_t, sigma_s, speed, planes, material, bc, source, tally,
                 qoi=None, ww_mesh=None, fission=None):
    sigma_t = _f64(sigma_t)
    M, G = sigma_t.shape
    src = dict(source)
    src.setdefault("t_lo", 0.0)
    src.setdefault("t_hi", 0.0)
    src.setdefault("kind", "isotropic")
    src["lo"] = _f64(src["lo"])
    src["hi"] = _f64(src["hi"])
    src["group_pmf"] = _f64(src["group_pmf"])
    tal = dict(tally)
    tal["mesh"] = [_f64(m) for m in tal["mesh"]]
    tal["time_edges"] = _f64(tal["time_edges"])
    tal.setdefault("n_batches", 32)
    tal["time_crossing"] = bool(tal.get("time_crossing", False))
    p = {
        "sigma_t": sigma_t,
        "sigma_s": _f64(sigma_s).reshape(M, G, G),
        "speed": _f64(speed),
        "planes": [_f64(pl) for pl in planes],
        "material": np.ascontiguousarray(np.asarray(material, dtype=np.int32)),
        "bc": np.asarray(bc, dtype=np.int32),
        "source": src,
        "tally": tal,
        "qoi": None,
        "ww_mesh": None,
        "fission": None,
        "implicit_capture": None,
        "pins": None,
        "rod": None,
        "quadrics": None,
    }
    if fission is not None:
        p["fission"] = {k: _f64(fission[k]).reshape(M, G) for k in ("sigma_f", "nu", "chi")}
    if qoi is not None:
        p["qoi"] = {"lo": _f64(qoi["lo"]), "hi": _f64(qoi["hi"]),
                    "group_mask": np.asarray(qoi["group_mask"], dtype=np.int32)}
    if ww_mesh is not None:
        p["ww_mesh"] = [_f64(m) for m in ww_mesh]
    return p


# ---------------------------------------------------------------------------
# 1-D slabs
# ---------------------------------------------------------------------------

def slab(thickness=10.0, sigma_t=1.0, sigma_s=0.5, speed=1.0, n_bins=20,
         source="surface", mu_law="cosine", x_src=0.0, time_edges=None,
         bc=(VACUUM, VACUUM), n_batches=32, t_hi=0.0):
    """One-group slab x in [0, thickness], infinite in y and z.

    source='surface': surface source on the x- face, entering along +x with
    the given angular law.  source='plane': isotropic plane source at x_src.
    """
    planes = [np.array([0.0, thickness]), _empty(), _empty()]
    mesh_x = np.linspace(0.0, thickness, n_bins + 1)
    if time_edges is None:
        time_edges = np.array([0.0, math.inf])
    if source == "surface":
        src = {"kind": "surface", "axis": 0, "sign": 1, "mu_law": mu_law,
               "lo": [0.0, 0.0, 0.0], "hi": [0.0, 0.0, 0.0]}
    else:
        src = {"kind": "isotropic", "lo": [x_src, 0.0, 0.0],
               "hi": [x_src, 0.0, 0.0]}
    src.update({"group_pmf": [1.0], "t_lo": 0.0, "t_hi": t_hi})
    return make_problem(
        sigma_t=[[sigma_t]], sigma_s=[[[sigma_s]]], speed=[speed],
        planes=planes, material=np.zeros((1, 1, 1)),
        bc=[bc[0], bc[1], VACUUM, VACUUM, VACUUM, VACUUM],
        source=src,
        tally={"mesh": [mesh_x, _empty(), _empty()], "time_edges": time_edges,
               "n_batches": n_batches})


def multigroup_slab(sigma_t=(1.0, 1.5, 2.0), sigma_s=((0.3, 0.4, 0.1), (0.0, 0.6, 0.5), (0.0, 0.2, 1.2)),
                    group_pmf=(0.6, 0.3, 0.1), thickness=6.0, n_bins=24, n_batches=32):
    """Multigroup slab [0, thickness], vacuum faces, one material with the
    transfer matrix sigma_s[g][g'] (from g to g'; down- and up-scatter), lit
    at x = 0 by a cosine-law current whose group follows group_pmf; steady
    flux tallies in n_bins x-bins."""
    G = len(sigma_t)
    return make_problem(
        sigma_t=[list(sigma_t)], sigma_s=[[list(r) for r in sigma_s]], speed=[1.0] * G,
        planes=[np.array([0.0, thickness]), _empty(), _empty()], material=np.zeros((1, 1, 1)),
        bc=[VACUUM] * 6,
        source={"kind": "surface", "axis": 0, "sign": 1, "mu_law": "cosine", "lo": [0.0, 0.0, 0.0],
                "hi": [0.0, 0.0, 0.0], "group_pmf": list(group_pmf)},
        tally={"mesh": [np.linspace(0.0, thickness, n_bins + 1), _empty(), _empty()],
               "time_edges": np.array([0.0, math.inf]), "n_batches": n_batches})


def reflected_column(sigma_t=(1.0, 1.5, 2.0), sigma_s=((0.3, 0.4, 0.1), (0.0, 0.6, 0.5), (0.0, 0.2, 1.2)),
                     group_pmf=(0.6, 0.3, 0.1), side=1.26, height=8.0, n_z_bins=16, n_batches=32):
    """Box side x side x height of one material, reflective on its x and y
    faces and vacuum on z, with a uniform isotropic volume source (group
    from group_pmf): its flux depends on z alone.  Steady flux tallies in
    n_z_bins z-bins (x and y without mesh planes)."""
    G = len(sigma_t)
    return make_problem(
        sigma_t=[list(sigma_t)], sigma_s=[[list(r) for r in sigma_s]], speed=[1.0] * G,
        planes=[np.array([0.0, side]), np.array([0.0, side]), np.array([0.0, height])],
        material=np.zeros((1, 1, 1)),
        bc=[REFLECTIVE, REFLECTIVE, REFLECTIVE, REFLECTIVE, VACUUM, VACUUM],
        source={"kind": "isotropic", "lo": [0.0, 0.0, 0.0], "hi": [side, side, height],
                "group_pmf": list(group_pmf)},
        tally={"mesh": [_empty(), _empty(), np.linspace(0.0, height, n_z_bins + 1)],
               "time_edges": np.array([0.0, math.inf]), "n_batches": n_batches})


def cfg1_slab_steady(c=0.5, mu_law="cosine", n_batches=32):
    """Slab of 10 mfp, Sigma_t = 1, scattering ratio c, surface source at x=0,
    20 tally bins, steady state (one time bin [0, inf))."""
    return slab(thickness=10.0, sigma_t=1.0, sigma_s=c, n_bins=20,
                source="surface", mu_law=mu_law, n_batches=n_batches)


def cfg2_slab_pulse(c=0.9, n_batches=32):
    """Slab of 40 mfp, Sigma_t = 1, v = 1, isotropic pulse plane source at the
    centre x = 20 at t = 0; 50 spatial bins x 100 time bins over [0, 20]."""
    return slab(thickness=40.0, sigma_t=1.0, sigma_s=c, speed=1.0, n_bins=50,
                source="plane", x_src=20.0,
                time_edges=np.linspace(0.0, 20.0, 101), n_batches=n_batches)


# ---------------------------------------------------------------------------
# Multigroup box lattices
# ---------------------------------------------------------------------------

def synthetic_xs(rng: SplitMix64, n_groups: int):
    """One synthetic multigroup material: Sigma_t,g uniform in [0.2, 2.0],
    scattering ratio c_g uniform in [0.3, 0.9], downscatter-only transfer
    (row g spread over g' >= g with random weights; the last group only
    self-scatters)."""
    G = n_groups
    st = np.zeros(G)
    ss = np.zeros((G, G))
    for g in range(G):
        st[g] = rng.uniform(0.2, 2.0)
        c = rng.uniform(0.3, 0.9)
        wts = np.array([rng.uniform(0.05, 1.0) for _ in range(g, G)])
        wts = wts / wts.sum()
        ss[g, g:] = c * st[g] * wts
    return st, ss


def lattice(n=17, pitch=1.26, height=50.0, n_groups=7, n_materials=2,
            n_z_bins=10, n_time_bins=20, t_end=20.0, gen_seed=3,
            bc_xy=REFLECTIVE, bc_z=VACUUM, n_batches=32, homogeneous=False):
    """n x n box lattice of square cells of the given pitch, one geometry
    layer of the given height, materials assigned by a seeded Bernoulli(1/2)
    mask, synthetic XS, speeds v_g = G - g, a uniform volume pulse source at
    t = 0 in group 0, and a mesh tally n x n x n_z_bins x G x n_time_bins."""
    rng = SplitMix64(gen_seed)
    G = n_groups
    M = 1 if homogeneous else n_materials
    st = np.zeros((M, G))
    ss = np.zeros((M, G, G))
    for m in range(M):
        st[m], ss[m] = synthetic_xs(rng, G)
    px = np.arange(n + 1) * pitch
    pz = np.array([0.0, height])
    mat = np.zeros((1, n, n), dtype=np.int32)
    if not homogeneous:
        for j in range(n):
            for i in range(n):
                mat[0, j, i] = rng.next_u64() & 1
    speed = np.array([float(G - g) for g in range(G)])
    pmf = np.zeros(G)
    pmf[0] = 1.0
    src = {"kind": "isotropic", "lo": [px[0], px[0], pz[0]],
           "hi": [px[-1], px[-1], pz[-1]], "group_pmf": pmf,
           "t_lo": 0.0, "t_hi": 0.0}
    tally = {"mesh": [px, px, np.linspace(0.0, height, n_z_bins + 1)],
             "time_edges": np.linspace(0.0, t_end, n_time_bins + 1),
             "n_batches": n_batches}
    return make_problem(st, ss, speed, [px, px, pz], mat,
                        [bc_xy, bc_xy, bc_xy, bc_xy, bc_z, bc_z], src, tally)


def cfg3_lattice(n_batches=32):
    """17x17x1 lattice of 1.26 cells, 2 materials, 7 groups, reflective x/y,
    vacuum z (height 50); tally 17x17x10 x 7 groups x 20 time bins."""
    return lattice(n=17, gen_seed=3, n_batches=n_batches)


def cfg4_batch(n_problems=256, seed=1000):
    """Random lattices for the batched solve: n ~ U{4..32}, G ~ U{1..7},
    histories ~ round(10**(4 + 2 xi)). Returns (problems, n_histories)."""
    probs, nh = [], []
    for p in range(n_problems):
        rng = SplitMix64(seed + p)
        n = rng.randint(4, 32)
        G = rng.randint(1, 7)
        xi = rng.uniform()
        nh.append(int(round(10.0 ** (4.0 + 2.0 * xi))))
        probs.append(lattice(n=n, n_groups=G, gen_seed=seed + p + 100000))
    return probs, nh


# ---------------------------------------------------------------------------
# Deep-penetration dog-leg duct (Kobayashi-like, synthetic)
# ---------------------------------------------------------------------------

CORNER_DETECTOR = ((10.0, 7.0, 4.0), (12.0, 9.0, 6.0))   # after the first bend
LEG_A_DETECTOR = ((8.0, 1.0, 4.0), (10.0, 3.0, 6.0))     # in sight of the source


def cfg5_dogleg(n_batches=32, detector=((29.0, 7.0, 4.0), (30.0, 9.0, 6.0))):
    """Box [0,30]x[0,10]x[0,10], vacuum on all faces, 2 groups.
    Bulk: Sigma_t = (1.0, 1.5), c = (0.8, 0.6), Sigma_s[0][0] = Sigma_s[0][1]
    = 0.4, Sigma_s[1][1] = 0.9.  A 2-unit-wide low-density dog-leg channel
    (Sigma_t = 0.05, same c and transfer split) at z in [4,6]: leg A x in
    [0,12], y in [1,3]; leg B x in [10,12], y in [1,9]; leg C x in [10,30],
    y in [7,9].  Source box x in [0,1], y in [1,3], z in [4,6], group 0,
    isotropic, steady.  Detector (quantity of interest) x in [29,30],
    y in [7,9], z in [4,6] (default), both groups.  Tally and weight-window
    mesh 40 x 10 x 10 (cells 0.75 x 1 x 1)."""
    st_bulk = np.array([1.0, 1.5])
    ss_bulk = np.array([[0.4, 0.4], [0.0, 0.9]])
    scale = 0.05 / st_bulk
    st_ch = np.array([0.05, 0.05])
    ss_ch = ss_bulk * scale[:, None]
    st = np.stack([st_bulk, st_ch])
    ss = np.stack([ss_bulk, ss_ch])
    px = np.array([0.0, 10.0, 12.0, 30.0])
    py = np.array([0.0, 1.0, 3.0, 7.0, 9.0, 10.0])
    pz = np.array([0.0, 4.0, 6.0, 10.0])
    mat = np.zeros((3, 5, 3), dtype=np.int32)
    # cell index: x cells [0,10],[10,12],[12,30]; y cells [0,1],[1,3],[3,7],
    # [7,9],[9,10]; z cells [0,4],[4,6],[6,10]
    kz = 1
    mat[kz, 1, 0] = 1          # leg A, x in [0,10]
    mat[kz, 1, 1] = 1          # leg A, x in [10,12]
    mat[kz, 2, 1] = 1          # leg B, y in [3,7]
    mat[kz, 3, 1] = 1          # leg B / C corner, y in [7,9]
    mat[kz, 3, 2] = 1          # leg C, x in [12,30]
    src = {"kind": "isotropic", "lo": [0.0, 1.0, 4.0], "hi": [1.0, 3.0, 6.0],
           "group_pmf": [1.0, 0.0], "t_lo": 0.0, "t_hi": 0.0}
    mesh = [np.arange(41) * 0.75, np.arange(11) * 1.0, np.arange(11) * 1.0]
    tally = {"mesh": mesh, "time_edges": [0.0, math.inf],
             "n_batches": n_batches}
    qoi = {"lo": list(detector[0]), "hi": list(detector[1]), "group_mask": [1, 1]}
    return make_problem(st, ss, [1.0, 1.0], [px, py, pz], mat,
                        [VACUUM] * 6, src, tally, qoi=qoi, ww_mesh=mesh)


# ---------------------------------------------------------------------------
# Small problems used by closed-form checks
# ---------------------------------------------------------------------------

def reflective_box(sigma_t, sigma_s, speed, size=(2.0, 2.0, 2.0),
                   time_edges=None, n_batches=32, pulse=True, fission=None):
    """Homogeneous all-reflective box (an infinite medium), uniform volume
    source in group 0, one tally bin per axis."""
    st = _f64(sigma_t).reshape(1, -1)
    G = st.shape[1]
    planes = [np.array([0.0, s]) for s in size]
    pmf = np.zeros(G)
    pmf[0] = 1.0
    if time_edges is None:
        time_edges = [0.0, math.inf]
    src = {"kind": "isotropic", "lo": [0.0, 0.0, 0.0], "hi": list(size),
           "group_pmf": pmf, "t_lo": 0.0, "t_hi": 0.0}
    tally = {"mesh": [np.array([0.0, s]) for s in size],
             "time_edges": time_edges, "n_batches": n_batches}
    return make_problem(st, _f64(sigma_s).reshape(1, G, G), speed, planes,
                        np.zeros((1, 1, 1)), [REFLECTIVE] * 6, src, tally, fission=fission)


def pin_cell_eigen_cylinder(n_groups=7, gen_seed=9, fine=4):
    """The pin cell of pin_cell_eigen with a cylindrical fuel pin (radius
    0.54 in the 1.26-wide reflected cell) in place of the square one."""
    p = pin_cell_eigen(n_groups, gen_seed)
    planes = [np.array([0.0, 1.26]), np.array([0.0, 1.26]), _empty()]
    mesh = np.linspace(0.0, 1.26, fine + 1)
    src = dict(p["source"], lo=_f64([0.63 - 0.3, 0.63 - 0.3, 0.0]), hi=_f64([0.63 + 0.3, 0.63 + 0.3, 0.0]))
    q = make_problem(p["sigma_t"], p["sigma_s"], p["speed"], planes, np.ones((1, 1, 1), dtype=np.int32),
                     p["bc"], src, {"mesh": [mesh, mesh, _empty()], "time_edges": [0.0, math.inf],
                                    "n_batches": 8}, fission=p["fission"])
    q["pins"] = {"radius": np.array([[[0.54]]]), "material": np.zeros((1, 1, 1), dtype=np.int32)}
    return q


def pin_cell_eigen(n_groups=7, gen_seed=9, fine=3):
    """Box stand-in for a reflected pin cell (Section 3's k-eigenvalue
    performance test uses a C5G7 pin cell, whose data is not used here): a
    1.26-wide square cell, infinite in z, reflective on every side, with a
    0.84-wide square fuel region in the middle and moderator around it.
    Synthetic 7-group cross sections: fuel absorbs more and fissions in all
    groups (80 % of its absorption; nu = 2.45, chi in the two fastest
    groups), the moderator
    scatters more.  The first cycle starts from a uniform source in the
    fuel in group 0.  Flux tally on a (3 fine) x (3 fine) mesh."""
    rng = SplitMix64(gen_seed)
    G = n_groups
    st = np.zeros((2, G))
    ss = np.zeros((2, G, G))
    for m in range(2):
        st[m], ss[m] = synthetic_xs(rng, G)
    ss[1] = ss[1] * np.minimum(1.0, 0.95 * st[1][:, None] / np.maximum(ss[1].sum(axis=1, keepdims=True), 1e-300))
    sf = 0.8 * (st[0] - ss[0].sum(axis=1))      # 80 % of the fuel's absorption fissions
    chi = np.zeros(G)
    chi[0], chi[1] = 0.7, 0.3
    planes = [np.array([0.0, 0.21, 1.05, 1.26])] * 2 + [_empty()]
    mat = np.ones((1, 3, 3), dtype=np.int32)
    mat[0, 1, 1] = 0
    pmf = np.zeros(G)
    pmf[0] = 1.0
    src = {"kind": "isotropic", "lo": [0.21, 0.21, 0.0], "hi": [1.05, 1.05, 0.0], "group_pmf": pmf}
    mesh = np.concatenate([np.linspace(0.0, 0.21, fine + 1)[:-1], np.linspace(0.21, 1.05, fine + 1)[:-1],
                           np.linspace(1.05, 1.26, fine + 1)])
    tally = {"mesh": [mesh, mesh, _empty()], "time_edges": [0.0, math.inf], "n_batches": 8}
    return make_problem(st, ss, [float(G - g) for g in range(G)], planes, mat,
                        [REFLECTIVE] * 4 + [VACUUM, VACUUM], src, tally,
                        fission={"sigma_f": np.stack([sf, np.zeros(G)]), "nu": np.full((2, G), 2.45),
                                 "chi": np.stack([chi, chi])})


def beam_through_pin(y0=1.2, sigma_pin=1.5, radius=0.6, n_bins=20, mu_law="beam"):
    """A 2 x 2 (x, y) void box, infinite in z, with one purely absorbing
    pin of the given radius centred at (1, 1).  Surface source on the x-
    face at the point (0, y0), entering along +x with the given angular
    law; the particles that miss or cross the pin leak through the far
    faces.  Flux tally in n_bins x-bins."""
    planes = [np.array([0.0, 2.0]), np.array([0.0, 2.0]), _empty()]
    src = {"kind": "surface", "axis": 0, "sign": 1, "mu_law": mu_law, "lo": [0.0, y0, 0.0],
           "hi": [0.0, y0, 0.0], "group_pmf": [1.0]}
    tally = {"mesh": [np.linspace(0.0, 2.0, n_bins + 1), np.array([0.0, 2.0]), _empty()],
             "time_edges": [0.0, math.inf], "n_batches": 32}
    p = make_problem([[0.0], [sigma_pin]], [[[0.0]], [[0.0]]], [1.0], planes, np.zeros((1, 1, 1)),
                     [VACUUM] * 6, src, tally)
    p["pins"] = {"radius": np.array([[[radius]]]), "material": np.array([[[1]]], dtype=np.int32)}
    return p


def sphere_quadric(center, radius):
    """Coefficients (A..K) of the sphere |x - c|^2 - r^2."""
    cx, cy, cz = center
    return np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0, -2.0 * cx, -2.0 * cy, -2.0 * cz,
                     cx * cx + cy * cy + cz * cz - radius * radius])


def cone_quadric(apex):
    """Coefficients of the double cone (x - x0)^2 + (y - y0)^2 - (z - z0)^2
    (negative inside the two nappes along z)."""
    x0, y0, z0 = apex
    return np.array([1.0, 1.0, -1.0, 0.0, 0.0, 0.0, -2.0 * x0, -2.0 * y0, 2.0 * z0,
                     x0 * x0 + y0 * y0 - z0 * z0])


def plane_quadric(normal, offset):
    """Coefficients of the plane n . x - offset (a quadric of degree one)."""
    return np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0, normal[0], normal[1], normal[2], -offset])


def beam_through_quadric(coef, axis=0, sign=1, point=(0.0, 1.2, 0.9), sigma=1.5, n_bins=20,
                         scatter=0.0, inside_material=1):
    """A [0, 2]^3 void box (vacuum faces) whose one geometry cell carries
    the quadric `coef`, filled inside with an absorber of total cross
    section sigma (scattering ratio `scatter`).  Surface source at `point`
    on the face the beam enters through (axis, sign), entering as a beam;
    flux tally in n_bins bins along the beam axis."""
    planes = [np.array([0.0, 2.0])] * 3
    lo = list(point)
    lo[axis] = 0.0 if sign > 0 else 2.0
    src = {"kind": "surface", "axis": axis, "sign": sign, "mu_law": "beam", "lo": lo, "hi": lo,
           "group_pmf": [1.0]}
    mesh = [np.array([0.0, 2.0])] * 3
    mesh[axis] = np.linspace(0.0, 2.0, n_bins + 1)
    tally = {"mesh": mesh, "time_edges": [0.0, math.inf], "n_batches": 32}
    p = make_problem([[0.0], [sigma]], [[[0.0]], [[scatter * sigma]]], [1.0], planes,
                     np.zeros((1, 1, 1)), [VACUUM] * 6, src, tally)
    p["quadrics"] = {"coef": np.asarray(coef, dtype=np.float64).reshape(1, 1, 1, 10),
                     "material": np.array([[[inside_material]]], dtype=np.int32)}
    return p


def sphere_lattice(n=4, pitch=1.26, radius=0.5, n_layers=4, n_groups=3, gen_seed=23, n_time_bins=5, t_end=5.0,
                   bc=REFLECTIVE, n_batches=16):
    """n x n x n_layers lattice of cubic cells of the given pitch, each
    holding a spherical fuel kernel (material 0) of the given radius in
    moderator (material 1): quadric-surface geometry; synthetic cross
    sections; uniform volume pulse in group 0 at t = 0; one tally bin per
    cell."""
    rng = SplitMix64(gen_seed)
    G = n_groups
    st = np.zeros((2, G))
    ss = np.zeros((2, G, G))
    for m in range(2):
        st[m], ss[m] = synthetic_xs(rng, G)
    px = np.arange(n + 1) * pitch
    pz = np.arange(n_layers + 1) * pitch
    pmf = np.zeros(G)
    pmf[0] = 1.0
    src = {"kind": "isotropic", "lo": [0.0, 0.0, 0.0], "hi": [px[-1], px[-1], pz[-1]], "group_pmf": pmf}
    tally = {"mesh": [px, px, pz], "time_edges": np.linspace(0.0, t_end, n_time_bins + 1), "n_batches": n_batches}
    p = make_problem(st, ss, [float(G - g) for g in range(G)], [px, px, pz],
                     np.ones((n_layers, n, n), dtype=np.int32), [bc] * 6, src, tally)
    coef = np.zeros((n_layers, n, n, 10))
    for k in range(n_layers):
        for j in range(n):
            for i in range(n):
                coef[k, j, i] = sphere_quadric(((i + 0.5) * pitch, (j + 0.5) * pitch, (k + 0.5) * pitch), radius)
    p["quadrics"] = {"coef": coef, "material": np.zeros((n_layers, n, n), dtype=np.int32)}
    return p


def mixed_quadric_lattice(n=3, n_layers=2, pitch=1.26, n_groups=3, gen_seed=29, refine=2, n_time_bins=4,
                          t_end=4.0, bc=REFLECTIVE, n_batches=8):
    """n x n x n_layers lattice of cubic cells, each geometry cell holding
    one quadric drawn from: a sphere, a tilted ellipsoid (cross terms), a
    double cone, a one-sheet hyperboloid, a tilted plane, a quadric holding
    the cell's own material, or none; the inside material drawn from the
    three.  Tally mesh `refine` times finer than the cells, so particles
    cross union-cell planes inside one geometry cell (and its quadric)."""
    rng = SplitMix64(gen_seed)
    G = n_groups
    st = np.zeros((3, G))
    ss = np.zeros((3, G, G))
    for m in range(3):
        st[m], ss[m] = synthetic_xs(rng, G)
    px = np.arange(n + 1) * pitch
    pz = np.arange(n_layers + 1) * pitch
    mat = np.zeros((n_layers, n, n), dtype=np.int32)
    coef = np.zeros((n_layers, n, n, 10))
    qmat = np.full((n_layers, n, n), -1, dtype=np.int32)
    for k in range(n_layers):
        for j in range(n):
            for i in range(n):
                mat[k, j, i] = rng.randint(0, 2)
                c = np.array([(i + rng.uniform(0.3, 0.7)) * pitch, (j + rng.uniform(0.3, 0.7)) * pitch,
                              (k + rng.uniform(0.3, 0.7)) * pitch])
                kind = rng.randint(0, 6)
                r = rng.uniform(0.2, 0.5) * pitch
                if kind == 0:
                    q = sphere_quadric(c, r)
                elif kind in (1, 5):
                    # (x - c)^T S (x - c) - r^2 with S = R^T diag R: a rotated ellipsoid
                    ang = rng.uniform(0.0, math.pi)
                    ca, sa = math.cos(ang), math.sin(ang)
                    Rm = np.array([[ca, -sa, 0.0], [sa, ca, 0.0], [0.0, 0.0, 1.0]])
                    Sm = Rm.T @ np.diag([rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)]) @ Rm
                    lin = -2.0 * Sm @ c
                    q = np.array([Sm[0, 0], Sm[1, 1], Sm[2, 2], 2.0 * Sm[0, 1], 2.0 * Sm[1, 2], 2.0 * Sm[2, 0],
                                  lin[0], lin[1], lin[2], float(c @ Sm @ c) - r * r])
                elif kind == 2:
                    q = cone_quadric(c)
                elif kind == 3:
                    # one-sheet hyperboloid about z: (x-cx)^2 + (y-cy)^2 - (z-cz)^2 - r^2
                    q = cone_quadric(c)
                    q[9] -= r * r
                elif kind == 4:
                    nrm = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1)])
                    q = plane_quadric(nrm, float(nrm @ c))
                else:
                    q = sphere_quadric(c, r)
                coef[k, j, i] = q
                if kind == 6:
                    continue        # no quadric (its coefficients stay unused)
                qmat[k, j, i] = mat[k, j, i] if kind == 5 else rng.randint(0, 2)
    pmf = np.zeros(G)
    pmf[0] = 1.0
    src = {"kind": "isotropic", "lo": [0.0, 0.0, 0.0], "hi": [px[-1], px[-1], pz[-1]], "group_pmf": pmf}
    mx = np.linspace(0.0, px[-1], refine * n + 1)
    mz = np.linspace(0.0, pz[-1], refine * n_layers + 1)
    tally = {"mesh": [mx, mx, mz], "time_edges": np.linspace(0.0, t_end, n_time_bins + 1), "n_batches": n_batches}
    p = make_problem(st, ss, [float(G - g) for g in range(G)], [px, px, pz], mat, [bc] * 6, src, tally)
    p["quadrics"] = {"coef": coef, "material": qmat}
    return p


def pin_lattice(n=3, pitch=1.26, radius=0.54, height=10.0, n_groups=3, gen_seed=17, n_z_bins=4,
                n_time_bins=5, t_end=5.0, bc_xy=REFLECTIVE, bc_z=VACUUM, n_batches=16, fine=1):
    """n x n lattice of square cells of the given pitch, each holding a
    cylindrical fuel pin (material 0) of the given radius in moderator
    (material 1); synthetic cross sections; uniform volume pulse source in
    group 0 at t = 0; tally mesh fine x fine per cell in x-y, n_z_bins in z."""
    rng = SplitMix64(gen_seed)
    G = n_groups
    st = np.zeros((2, G))
    ss = np.zeros((2, G, G))
    for m in range(2):
        st[m], ss[m] = synthetic_xs(rng, G)
    px = np.arange(n + 1) * pitch
    pz = np.array([0.0, height])
    mesh_xy = np.linspace(0.0, px[-1], n * fine + 1)
    pmf = np.zeros(G)
    pmf[0] = 1.0
    src = {"kind": "isotropic", "lo": [0.0, 0.0, 0.0], "hi": [px[-1], px[-1], height], "group_pmf": pmf}
    tally = {"mesh": [mesh_xy, mesh_xy, np.linspace(0.0, height, n_z_bins + 1)],
             "time_edges": np.linspace(0.0, t_end, n_time_bins + 1), "n_batches": n_batches}
    p = make_problem(st, ss, [float(G - g) for g in range(G)], [px, px, pz], np.ones((1, n, n), dtype=np.int32),
                     [bc_xy] * 4 + [bc_z] * 2, src, tally)
    p["pins"] = {"radius": np.full((1, n, n), radius), "material": np.zeros((1, n, n), dtype=np.int32)}
    return p


def bare_slab_eigen(thickness=6.0, sigma_s=0.6, sigma_f=0.2, nu=2.5, n_bins=24):
    """One-group bare slab for the k-eigenvalue power iteration: Sigma_t = 1,
    scattering sigma_s, fission sigma_f with nu neutrons (the rest
    capture), vacuum faces, steady state; the first cycle starts from an
    isotropic plane source at the centre; flux tally in n_bins x-bins."""
    p = slab(thickness=thickness, sigma_t=1.0, sigma_s=sigma_s, n_bins=n_bins, source="plane",
             x_src=0.5 * thickness)
    p["fission"] = {"sigma_f": np.array([[sigma_f]]), "nu": np.array([[nu]]), "chi": np.array([[1.0]])}
    return p


def azurv1_supercritical(c_scatter=0.5, sigma_f=0.25, nu=2.4, n_bins=42, n_time_bins=20,
                         t_end=20.0, n_batches=32):
    """AZURV1-like supercritical pulse (Section 3 adds fission to reach
    c = 1.1): one group, Sigma_t = v = 1 (time in mean free times), an
    isotropic plane pulse at the centre of a 42-mfp slab whose faces no
    particle reaches before t = 20, scattering c_scatter, fission
    sigma_f with nu neutrons (c = c_scatter + nu sigma_f), the rest
    capture.  Flux tallies in n_bins x-bins and n_time_bins time bins with
    the time-crossing tally at the edges."""
    half = 21.0
    p = slab(thickness=2 * half, sigma_t=1.0, sigma_s=c_scatter, n_bins=n_bins, source="plane",
             x_src=half, time_edges=np.linspace(0.0, t_end, n_time_bins + 1), n_batches=n_batches)
    p["tally"]["time_crossing"] = True
    p["fission"] = {"sigma_f": np.array([[sigma_f]]), "nu": np.array([[nu]]),
                    "chi": np.array([[1.0]])}
    return p


def void_box(size=(3.0, 2.0, 1.0), n_mesh=(3, 2, 1), src_point=(0.5, 0.5, 0.5),
             time_edges=None, speed=1.0, bc=None):
    """Void (Sigma_t = 0) box with an isotropic point source: every track is
    deterministic given its direction."""
    planes = [np.array([0.0, s]) for s in size]
    mesh = [np.linspace(0.0, s, n + 1) for s, n in zip(size, n_mesh)]
    if time_edges is None:
        time_edges = [0.0, math.inf]
    src = {"kind": "isotropic", "lo": list(src_point), "hi": list(src_point),
           "group_pmf": [1.0], "t_lo": 0.0, "t_hi": 0.0}
    return make_problem([[0.0]], [[[0.0]]], [speed], planes,
                        np.zeros((1, 1, 1)), bc if bc is not None else [VACUUM] * 6,
                        src, {"mesh": mesh, "time_edges": time_edges,
                              "n_batches": 8})


def rod_beam_box(sigma_rod=0.2, length=10.0, height=10.0, t_move=10.0, void_rod=False, n_batches=16):
    """Void box [0, L] x [0, 1] x [0, H] with an absorbing rod that descends:
    the moving plane falls from z = H at t = 0 to z = 0 at t = t_move and
    rests there until t = 2 t_move; above it the box is rod (a pure
    absorber of Sigma = sigma_rod, or a second void material).  A beam
    enters the x- face at a height and time uniform over [0, H] x [0, t_move],
    speed 1: a particle at height z born at t_b is inside the rod along
    min(L, t_b + z) of its path when L = H = t_move."""
    st = [[0.0], [0.0 if void_rod else sigma_rod]]
    ss = [[[0.0]], [[0.0]]]
    planes = [np.array([0.0, length]), np.array([0.0, 1.0]), np.array([0.0, height])]
    src = {"kind": "surface", "axis": 0, "sign": 1, "mu_law": "beam", "lo": [0.0, 0.0, 0.0],
           "hi": [0.0, 1.0, height], "group_pmf": [1.0], "t_lo": 0.0, "t_hi": t_move}
    tally = {"mesh": [np.linspace(0.0, length, 6), _empty(), np.linspace(0.0, height, 6)],
             "time_edges": np.array([0.0, t_move, 2.0 * t_move]), "n_batches": n_batches}
    p = make_problem(st, ss, [1.0], planes, np.zeros((1, 1, 1)), [VACUUM] * 6, src, tally)
    p["rod"] = {"z": _f64([height, 0.0, 0.0]), "material": np.ones((1, 1, 1), dtype=np.int32)}
    return p


def rod_lattice(n=17, pitch=1.26, height=50.0, n_groups=7, gen_seed=3, rods_every=3, z_top=50.0,
                z_bottom=10.0, n_z_bins=10, n_time_bins=20, t_end=20.0, t_insert=10.0, n_batches=32):
    """The lattice workload with a bank of control rods inserted from the top
    during the transient: every rods_every-th lattice cell in x and y holds a
    rod of a third, strongly absorbing synthetic material whose tip (the
    moving plane) descends from z_top at t = 0 to z_bottom at t = t_insert
    and stays there; elsewhere the plane only bounds no material change."""
    p = lattice(n=n, pitch=pitch, height=height, n_groups=n_groups, gen_seed=gen_seed, n_z_bins=n_z_bins,
                n_time_bins=n_time_bins, t_end=t_end, n_batches=n_batches)
    rng = SplitMix64(gen_seed + 7777)
    G = n_groups
    st_r = np.array([rng.uniform(1.5, 3.0) for _ in range(G)])
    ss_r = np.zeros((G, G))
    for g in range(G):
        ss_r[g, g] = 0.1 * st_r[g]          # mostly absorbing
    p["sigma_t"] = np.ascontiguousarray(np.concatenate([p["sigma_t"], st_r[None, :]], axis=0))
    p["sigma_s"] = np.ascontiguousarray(np.concatenate([p["sigma_s"], ss_r[None, :, :]], axis=0))
    rodm = np.full((1, n, n), -1, dtype=np.int32)
    M = p["sigma_t"].shape[0]
    for j in range(n):
        for i in range(n):
            if i % rods_every == rods_every // 2 and j % rods_every == rods_every // 2:
                rodm[0, j, i] = M - 1
    te = p["tally"]["time_edges"]
    z = np.where(te < t_insert, z_top + (z_bottom - z_top) * te / t_insert, z_bottom)
    p["rod"] = {"z": _f64(z), "material": rodm}
    return p


CONFIGS = {
    "cfg1": cfg1_slab_steady,
    "cfg2": cfg2_slab_pulse,
    "cfg3": cfg3_lattice,
    "cfg5": cfg5_dogleg,
}
