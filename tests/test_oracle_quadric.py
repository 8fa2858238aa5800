"""Pins of the oracle's quadric surfaces (reading R29: one second-degree
surface per geometry cell, its negative side filled with a material of its
own) against closed forms and exact invariants.

* Beams through a purely absorbing inside in a void box: the flux along
  the beam is 1 before the first entry and is attenuated by e^{-sigma s}
  over every stretch s inside, so the track length per bin and the
  transmission follow from the roots of a d^2 + 2 b d + c on the line.
  The cases reach every root rule: a sphere (a > 0, entered and left), a
  double cone along z crossed along its axis (a < 0: the line starts
  inside, leaves, and enters again) and across it (a > 0), and a tilted
  plane (a = 0) crossed both ways.
* A quadric whose inside is the surrounding material changes nothing but
  the number of surface events: per-history collisions and terminations
  are those of the problem without it, tallies equal to rounding.
* A cylinder written as a quadric behaves as the pin of the same radius.
* Problems the reading does not cover are refused."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

Z_MAX = 4.5


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


def _inside_intervals(q, x0, u, L):
    """The stretches of [0, L] of the line x0 + s u where the quadric is
    negative (roots of a s^2 + 2 b s + c, by numpy)."""
    A, B, C, D, E, F, G, H, J, K = q
    x, y, z = x0
    ux, uy, uz = u
    a = A * ux * ux + B * uy * uy + C * uz * uz + D * ux * uy + E * uy * uz + F * uz * ux
    b = (A * x * ux + B * y * uy + C * z * uz
         + 0.5 * (D * (x * uy + y * ux) + E * (y * uz + z * uy) + F * (z * ux + x * uz) + G * ux + H * uy + J * uz))
    c = (A * x * x + B * y * y + C * z * z + D * x * y + E * y * z + F * z * x + G * x + H * y + J * z + K)
    cuts = [0.0, L]
    if a != 0.0:
        disc = b * b - a * c
        if disc > 0:
            cuts += [(-b - math.sqrt(disc)) / a, (-b + math.sqrt(disc)) / a]
    elif b != 0.0:
        cuts.append(-c / (2.0 * b))
    cuts = sorted(t for t in cuts if 0.0 <= t <= L)
    out = []
    for s0, s1 in zip(cuts[:-1], cuts[1:]):
        m = 0.5 * (s0 + s1)
        if a * m * m + 2.0 * b * m + c < 0.0 and s1 > s0:
            out.append((s0, s1))
    return out


def _beam_profile(edges, intervals, sigma):
    """Track length per source particle in each bin [e_j, e_j+1] (measured
    along the beam from its entry) when stretches inside attenuate by
    e^{-sigma s}."""
    def flux_integral(a, c):
        # integral of the surviving fraction over [a, c]
        tot, pos, att = 0.0, 0.0, 1.0
        pts = sorted({a, c, *[t for iv in intervals for t in iv if a < t < c]})
        for s0, s1 in zip(pts[:-1], pts[1:]):
            # attenuation accumulated before s0
            lost = sum(max(0.0, min(s0, hi) - lo) for lo, hi in intervals if lo < s0)
            att0 = math.exp(-sigma * lost)
            mid = 0.5 * (s0 + s1)
            inside = any(lo <= mid <= hi for lo, hi in intervals)
            if inside:
                tot += att0 * (1.0 - math.exp(-sigma * (s1 - s0))) / sigma
            else:
                tot += att0 * (s1 - s0)
        return tot

    return np.array([flux_integral(a, c) for a, c in zip(edges[:-1], edges[1:])])


def _run_beam(coef, axis, sign, point, sigma=1.5, N=40000, seed=71):
    p = w.beam_through_quadric(coef, axis=axis, sign=sign, point=point, sigma=sigma)
    res = oracle.run(p, N, seed)
    e = oracle.estimates(p, res)
    x0 = list(point)
    x0[axis] = 0.0 if sign > 0 else 2.0
    u = [0.0, 0.0, 0.0]
    u[axis] = float(sign)
    iv = _inside_intervals(coef, x0, u, 2.0)
    ell = sum(hi - lo for lo, hi in iv)
    T = math.exp(-sigma * ell)
    # transmission: the particles that leave through the far face
    face = 2 * axis + (1 if sign > 0 else 0)
    leak = e["leak_mean"][0, 0, face]
    lvar = e["leak_var"][0, 0, face]
    _check([leak], [lvar], [T])
    # every particle either crosses or is absorbed inside
    t = res["tot"].astype(np.int64)
    assert int(t[3 + oracle.T_ABSORB] + t[3 + oracle.T_LEAK]) == N
    # the flux profile along the beam (bin j of the mesh along the axis)
    edges = np.linspace(0.0, 2.0, 21)
    prof = _beam_profile(edges if sign > 0 else edges, iv, sigma)
    if sign < 0:
        prof = prof[::-1]
    mean = e["mean"].reshape(20) * 0.4     # flux density times the bin volume (0.1 x 2 x 2): track length
    var = e["var"].reshape(20) * 0.16
    _check(mean, var, prof)
    return iv


@pytest.mark.parametrize("point", [(0.0, 1.2, 0.9), (0.0, 1.0, 1.0), (0.0, 0.55, 1.1), (0.0, 1.7, 1.3)])
def test_beam_through_a_sphere(point):
    iv = _run_beam(w.sphere_quadric((1.0, 1.0, 1.0), 0.6), 0, 1, point)
    b2 = (point[1] - 1.0) ** 2 + (point[2] - 1.0) ** 2
    assert (len(iv) == 1) == (b2 < 0.36)


@pytest.mark.parametrize("point", [(0.8, 1.3, 0.0), (1.0, 1.05, 0.0)])
def test_beam_along_the_axis_of_a_double_cone(point):
    """Along +z the line starts inside the lower nappe, leaves it at
    z = 1 - r0, enters the upper one at z = 1 + r0 (a = -1 < 0)."""
    iv = _run_beam(w.cone_quadric((1.0, 1.0, 1.0)), 2, 1, point)
    r0 = math.hypot(point[0] - 1.0, point[1] - 1.0)
    assert len(iv) == 2 and abs(iv[0][1] - (1.0 - r0)) < 1e-12 and abs(iv[1][0] - (1.0 + r0)) < 1e-12


def test_beam_across_a_double_cone():
    """Along +x at height z0 the inside is |x - 1| < sqrt((z0-1)^2 - (y0-1)^2)."""
    iv = _run_beam(w.cone_quadric((1.0, 1.0, 1.0)), 0, 1, (0.0, 1.1, 1.6))
    assert len(iv) == 1


@pytest.mark.parametrize("sign", [1, -1])
def test_beam_through_a_tilted_plane(sign):
    """A degree-one quadric (a = 0): inside for x < 1.1 - 0.5 (y - 1) - 0.3 (z - 1);
    crossed from inside (+x) and from outside (-x)."""
    q = w.plane_quadric((1.0, 0.5, 0.3), 1.1 + 0.5 + 0.3)
    iv = _run_beam(q, 0, sign, (0.0, 1.4, 0.7))
    assert len(iv) == 1


def test_quadric_of_the_surrounding_material_changes_nothing():
    """A scattering box whose spheres hold the box's own material: every
    history has the same collisions and termination as without them, and
    the tallies agree to rounding; only surface events are added."""
    p = w.sphere_lattice(n=2, n_layers=2, radius=0.5, n_groups=2)
    q = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in p.items()}
    q["quadrics"] = {"coef": p["quadrics"]["coef"], "material": np.ones((2, 2, 2), dtype=np.int32)}
    q2 = dict(q)
    q2["quadrics"] = None
    N = 4000
    a = oracle.run(q, N, 9, records=True)
    b = oracle.run(q2, N, 9, records=True)
    # records: census, surface, collision, particles, termination mask
    assert np.array_equal(a["rec"][:, [0, 2, 3, 4]], b["rec"][:, [0, 2, 3, 4]])
    assert np.all(a["rec"][:, 1] >= b["rec"][:, 1])
    np.testing.assert_allclose(a["S"], b["S"], rtol=1e-11, atol=1e-14)


def test_cylinder_as_a_quadric_matches_the_pin():
    """The z-cylinder of radius 0.6 about (1, 1) as a quadric and as a pin:
    the same transmission within the statistics of both."""
    N = 40000
    pin = w.beam_through_pin(y0=1.3)
    quad = w.beam_through_pin(y0=1.3)
    quad["pins"] = None
    quad["quadrics"] = {"coef": np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0, -2.0, -2.0, 0.0, 2.0 - 0.36]).reshape(1, 1, 1, 10),
                        "material": np.array([[[1]]], dtype=np.int32)}
    ep = oracle.estimates(pin, oracle.run(pin, N, 5))
    eq = oracle.estimates(quad, oracle.run(quad, N, 5))
    T = math.exp(-1.5 * 2.0 * math.sqrt(0.36 - 0.09))
    for e in (ep, eq):
        _check([e["leak_mean"][0, 0, 1]], [e["leak_var"][0, 0, 1]], [T])


def test_quadric_validation():
    p = w.beam_through_quadric(w.sphere_quadric((1.0, 1.0, 1.0), 0.6))
    q = dict(p)
    q["pins"] = {"radius": np.array([[[0.3]]]), "material": np.array([[[1]]], dtype=np.int32)}
    with pytest.raises(Exception):
        oracle.run(q, 10, 1)
    q = dict(p)
    q["quadrics"] = {"coef": np.full((1, 1, 1, 10), np.nan), "material": np.array([[[1]]], dtype=np.int32)}
    with pytest.raises(Exception):
        oracle.run(q, 10, 1)
    q = dict(p)
    q["quadrics"] = {"coef": p["quadrics"]["coef"], "material": np.array([[[2]]], dtype=np.int32)}
    with pytest.raises(Exception):
        oracle.run(q, 10, 1)
    s = w.slab()
    s["quadrics"] = {"coef": np.zeros((1, 1, s["material"].shape[2], 10)),
                     "material": np.zeros_like(s["material"])}
    with pytest.raises(Exception):
        oracle.run(s, 10, 1)


def test_constant_quadrics_reduce_to_plain_cells():
    """A quadric with only its constant term: K < 0 is inside everywhere,
    so the run is bit for bit that of the cell filled with the inside
    material; K > 0 is inside nowhere, so it is the run without it."""
    const_in = np.array([0, 0, 0, 0, 0, 0, 0, 0, 0, -1.0])
    p = w.beam_through_quadric(const_in, scatter=0.6)
    q = w.beam_through_quadric(const_in, scatter=0.6)
    q["quadrics"] = None
    q["material"] = np.ones_like(q["material"])
    a, b = oracle.run(p, 3000, 5, records=True), oracle.run(q, 3000, 5, records=True)
    assert np.array_equal(a["rec"], b["rec"]) and np.array_equal(a["S"], b["S"])
    p = w.beam_through_quadric(-const_in, scatter=0.6)
    q = dict(p)
    q["quadrics"] = None
    a, b = oracle.run(p, 3000, 5, records=True), oracle.run(q, 3000, 5, records=True)
    assert np.array_equal(a["rec"], b["rec"]) and np.array_equal(a["S"], b["S"])


def test_tangent_beam_never_enters():
    """A beam tangent to the sphere (zero discriminant from outside) makes
    no quadric crossing: every particle leaks, with one surface event per
    mesh plane and none more."""
    p = w.beam_through_quadric(w.sphere_quadric((1.0, 1.0, 1.0), 0.6), point=(0.0, 1.6, 1.0))
    r = oracle.run(p, 2000, 7)
    t = r["tot"].astype(np.int64)
    assert int(t[3 + oracle.T_LEAK]) == 2000 and int(t[3 + oracle.T_ABSORB]) == 0
    assert int(t[1]) == 2000 * 20


@pytest.mark.parametrize("coef, point, chord", [
    # a plane quadric on the mesh plane x = 1 (the plane and the quadric tie;
    # planes go first, then the quadric at distance 0)
    (w.plane_quadric((1.0, 0.0, 0.0), 1.0), (0.0, 1.3, 0.7), 1.0),
    # a sphere touching the cell's faces, the beam along its axis: born on
    # the surface moving in
    (w.sphere_quadric((1.0, 1.0, 1.0), 1.0), (0.0, 1.0, 1.0), 2.0),
])
def test_degenerate_crossings_keep_the_transmission(coef, point, chord):
    p = w.beam_through_quadric(coef, point=point)
    r = oracle.run(p, 40000, 9)
    e = oracle.estimates(p, r)
    _check([e["leak_mean"][0, 0, 1]], [e["leak_var"][0, 0, 1]], [math.exp(-1.5 * chord)])
