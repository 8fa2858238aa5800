"""Pins of the oracle's implicit capture with weight roulette (Section 3
runs the time-dependent dog-leg duct with implicit capture) against the
same closed forms as the analog game: the technique changes the variance,
never the expectation.  Also checks what it is for: a smaller variance in
the deep bins of a scattering slab for the same number of histories."""
import math

import numpy as np

import oracle
import workloads as w
from refs import (infinite_medium_pulse_bins, infinite_medium_steady, slab_absorber_bins, sn_slab)

Z_MAX = 4.5
IC = {"w_min": 0.25, "w_survive": 1.0}

MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5], [0.0, 0.2, 1.2]]


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


def _ic(p, **kw):
    p["implicit_capture"] = dict(IC, **kw)
    return p


def test_infinite_medium_steady_one_and_multigroup():
    p = _ic(w.reflective_box([1.0], [[0.5]], [1.0], size=(2.0, 2.0, 2.0)))
    res = oracle.run(p, 100000, 41)
    e = oracle.estimates(p, res)
    _check(e["mean"], e["var"], [1.0 / (8.0 * 0.5)])
    tot = res["tot"]
    assert int(tot[3]) == 0                       # nothing is absorbed ...
    assert int(tot[7]) == 100000                  # ... every history ends in a roulette
    p = _ic(w.reflective_box(MG_ST, MG_SS, [1.0, 1.0, 1.0], size=(1.0, 2.0, 3.0)))
    res = oracle.run(p, 100000, 42)
    e = oracle.estimates(p, res)
    _check(e["mean"].ravel(), e["var"].ravel(), infinite_medium_steady(np.array(MG_ST), np.array(MG_SS), 6.0))


def test_infinite_medium_pulse_bins():
    edges = np.array([0.0, 0.25, 0.5, 1.0, 2.0, 4.0])
    speed = [3.0, 2.0, 1.0]
    p = _ic(w.reflective_box(MG_ST, MG_SS, speed, size=(1.0, 1.0, 2.0), time_edges=edges))
    res = oracle.run(p, 100000, 43)
    e = oracle.estimates(p, res)
    exact = infinite_medium_pulse_bins(np.array(MG_ST), np.array(MG_SS), np.array(speed), edges, 2.0)
    _check(e["mean"].ravel(), e["var"].ravel(), exact.ravel())


def test_scattering_slab_against_sn_with_lower_variance():
    """c = 0.5 slab lit by a cosine current: bin fluxes agree with S_N; the
    deep bins (x > 5) have a smaller batch variance than analog's with the
    same histories."""
    pa = w.cfg1_slab_steady(c=0.5, mu_law="cosine")
    pi = _ic(w.cfg1_slab_steady(c=0.5, mu_law="cosine"), w_min=0.1, w_survive=0.5)
    N = 200000
    ea = oracle.estimates(pa, oracle.run(pa, N, 44))
    ei = oracle.estimates(pi, oracle.run(pi, N, 44))
    _, _, bins = sn_slab(10.0, 1.0, 0.5, n_cells=4000, n_mu=64)
    exact = bins(pi["tally"]["mesh"][0])
    _check(ei["mean"].ravel(), ei["var"].ravel(), exact, floor=2e-5 * exact.max())
    va, vi = ea["var"].ravel()[10:], ei["var"].ravel()[10:]
    assert vi.sum() < 0.8 * va.sum(), (vi.sum(), va.sum())


def test_pure_absorber_is_uncollided():
    """c = 0: the weight drops to 0 at the first collision and the roulette
    ends the particle, so the flux is the uncollided closed form and every
    collision ends a history."""
    p = _ic(w.cfg1_slab_steady(c=0.0, mu_law="uniform"))
    res = oracle.run(p, 100000, 45)
    e = oracle.estimates(p, res)
    edges = p["tally"]["mesh"][0]
    exact = slab_absorber_bins(edges, 1.0, "uniform")
    m, v = e["mean"].ravel(), e["var"].ravel()
    ok = m > 0
    _check(m[ok], v[ok], exact[ok])
    tot = res["tot"]
    assert int(tot[2]) == int(tot[7]) and int(tot[7] + tot[4]) == 100000


def test_invalid_parameters_rejected():
    import pytest

    for bad in ({"w_min": 0.0, "w_survive": 1.0}, {"w_min": 0.5, "w_survive": 0.25}):
        p = w.reflective_box([1.0], [[0.5]], [1.0])
        p["implicit_capture"] = bad
        with pytest.raises(RuntimeError):
            oracle.run(p, 10, 1)


def test_roulette_game_collision_count():
    """Infinite medium, c = 0.5, w_min = 0.25, w_s = 1: the weight runs
    1 -> 0.5 -> 0.25 -> 0.125 and the third collision's roulette keeps the
    particle with probability 1/8 (back at weight 1).  Collisions per history
    are 3 K with K geometric (P(K = k) = (1/8)^(k-1) 7/8): mean 24/7,
    variance 9 (1/8) / (7/8)^2."""
    p = _ic(w.reflective_box([1.0], [[0.5]], [1.0], size=(2.0, 2.0, 2.0)))
    N = 100000
    res = oracle.run(p, N, 46, records=True)
    coll = res["rec"][:, 2].astype(float)
    assert (coll % 3 == 0).all()
    mean, sd = coll.mean(), math.sqrt(9.0 * 0.125 / 0.875 ** 2 / N)
    assert abs(mean - 24.0 / 7.0) < Z_MAX * sd, (mean, 24.0 / 7.0, sd)
