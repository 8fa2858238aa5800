"""Pins of the oracle's time-crossing estimator (the flux at the time edges,
Section 3's multigroup pulse verification) against closed forms.

The estimator scores w v_g at every arrival of a particle at an edge T_j in
the spatial bin it is in, normalised by N V.  Its expectation is the scalar
flux at that instant, which is known in closed form for an infinite medium
(a matrix exponential of the multigroup balance) and for the uncollided
plane pulse.  A brute-force count over event traces pins the binning."""
import math

import numpy as np
import pytest

import oracle
import workloads as w
from refs import infinite_medium_pulse_points, plane_pulse_uncollided_point

Z_MAX = 4.5

MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1],
         [0.05, 0.6, 0.5],
         [0.0, 0.2, 1.4]]


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


def _with_crossing(p):
    p["tally"]["time_crossing"] = True
    return p


def test_time_crossing_off_by_default():
    p = w.reflective_box([1.0], [[0.5]], [1.0], time_edges=[0.0, 1.0, 2.0])
    res = oracle.run(p, 2000, 5)
    assert not res["X"].any()
    assert "tc_mean" not in oracle.estimates(p, res)


def test_infinite_medium_point_flux_multigroup():
    """phi(T_j) = V exp(-M V T_j) n0 at every edge, every group."""
    edges = np.array([0.0, 0.25, 0.5, 1.0, 2.0, 4.0])
    speed = [3.0, 2.0, 1.0]
    p = _with_crossing(w.reflective_box(MG_ST, MG_SS, speed, size=(1.0, 1.0, 2.0),
                                        time_edges=edges))
    res = oracle.run(p, 100000, 31)
    e = oracle.estimates(p, res)
    exact = infinite_medium_pulse_points(np.array(MG_ST), np.array(MG_SS), np.array(speed),
                                         edges[1:], 2.0)
    assert e["tc_mean"].shape == (5, 3, 1, 1, 1)
    _check(e["tc_mean"].ravel(), e["tc_var"].ravel(), exact.ravel())
    # the estimator is not the time-averaged one: at t = 4 the point value
    # lies below the average over [2, 4] for this decaying population
    assert (e["tc_mean"][4] < e["mean"][4]).all()


def test_infinite_medium_point_flux_one_group_decay():
    """One group, c = 0.9, Sigma_t = v = 1: phi(t) = e^{-0.1 t} (unit volume).
    The last edge is finite, so arrivals there score before the cut-off."""
    edges = np.linspace(0.0, 20.0, 11)
    p = _with_crossing(w.reflective_box([1.0], [[0.9]], [1.0], size=(1.0, 1.0, 1.0),
                                        time_edges=edges))
    res = oracle.run(p, 100000, 32)
    e = oracle.estimates(p, res)
    exact = np.exp(-0.1 * edges[1:])
    _check(e["tc_mean"].ravel(), e["tc_var"].ravel(), exact)
    # every arrival at T_K scores, and each such history ends there
    assert int(res["tot"][5]) > 0


def test_plane_pulse_uncollided_points():
    """Purely absorbing slab with a centre plane pulse: at time t the
    surviving particles (fraction e^{-t}) are spread uniformly over
    |x - 20| < t, so phi = e^{-t} / (2 t) there and 0 outside."""
    p = _with_crossing(w.cfg2_slab_pulse(c=0.0))
    res = oracle.run(p, 100000, 33)
    e = oracle.estimates(p, res)
    xe = p["tally"]["mesh"][0]
    te = p["tally"]["time_edges"]
    K = 20   # edges 0.2 .. 4.0
    exact = np.array([[plane_pulse_uncollided_point(20.0, 1.0, 1.0, xe[j], xe[j + 1], te[k + 1])
                       for j in range(50)] for k in range(K)])
    m = e["tc_mean"][:K, 0, 0, 0, :]
    v = e["tc_var"][:K, 0, 0, 0, :]
    _check(m, v, exact)
    assert (m[exact == 0] == 0).all()


def test_brute_force_from_traces():
    """Tiny 3-D lattice: the crossing sums of a few histories equal the sum
    over their traced census events of v_g in the bin found by searching the
    mesh for the position at the edge (edge index = k after the event - 1)."""
    p = _with_crossing(w.lattice(n=3, height=4.0, n_groups=3, gen_seed=7, t_end=3.0,
                                 n_time_bins=6, n_batches=1))
    N = 40
    res = oracle.run(p, N, 34)
    mesh = p["tally"]["mesh"]
    G = p["sigma_t"].shape[1]
    nt = [max(1, mesh[a].size - 1) for a in range(3)]
    X = np.zeros(res["X"].shape[1])
    n_census = 0
    for i in range(N):
        rows = oracle.trace(p, N, 34, i)
        for r in rows:
            if r[0] != 0:           # census rows only
                continue
            n_census += 1
            g, k = int(r[6]), int(r[7]) - 1
            t = [int(np.searchsorted(mesh[a], r[2 + a], side="right")) - 1 if mesh[a].size else 0
                 for a in range(3)]
            t = [min(max(t[a], 0), nt[a] - 1) for a in range(3)]
            j = ((k * G + g) * nt[2] + t[2]) * nt[1] * nt[0] + t[1] * nt[0] + t[0]
            X[j] += p["speed"][g]
    assert n_census == int(res["tot"][0]) and n_census > 0
    np.testing.assert_allclose(res["X"][0], X, rtol=1e-13, atol=0)
