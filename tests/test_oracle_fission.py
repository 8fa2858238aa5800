"""Pins of the oracle's fission branch (prompt fission in time-dependent
fixed-source runs; Section 3's supercritical AZURV1) against the paper's
printed growth factor and closed forms of the multiplying infinite medium.

The balance of an infinite homogeneous medium with fission is linear:
dn/dt = -(M V) n with M = diag(Sigma_t) - Sigma_s^T - chi (nu Sigma_f)^T,
so point and time-averaged fluxes are matrix exponentials and the steady
flux of a subcritical medium is M^-1 S."""
import json
import math
import os

import numpy as np

import oracle
import workloads as w
from refs import (infinite_medium_pulse_bins, infinite_medium_pulse_points,
                  infinite_medium_steady, plane_pulse_moments)

Z_MAX = 4.5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1],
         [0.0, 0.6, 0.5],
         [0.0, 0.2, 1.2]]
MG_SF = [0.05, 0.1, 0.3]
MG_NU = [2.6, 2.5, 2.43]
MG_CHI = [0.7, 0.3, 0.0]


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


def _population(p, res):
    """Neutrons alive at each time edge per source particle (from the
    time-crossing sums, one group, v = 1) and the variance of that mean
    over batches."""
    N, B = res["N"], res["B"]
    K = p["tally"]["time_edges"].size - 1
    Nb = oracle.batch_sizes(N, B).astype(float)
    per_batch = res["X"].reshape(B, K, -1).sum(axis=2) / Nb[:, None]
    mean = res["X"].reshape(B, K, -1).sum(axis=2).sum(axis=0) / N
    var = ((per_batch - per_batch.mean(0)) ** 2).sum(0) / (B * (B - 1))
    return mean, var


def test_azurv1_supercritical_growth_matches_paper():
    """c = 0.5 + 2.4 * 0.25 = 1.1: the population grows as e^{0.1 t}, about
    7.39 times in 20 mean free times, the factor Section 3 prints."""
    with open(os.path.join(GOLDEN, "azurv1_growth.json")) as f:
        gold = json.load(f)
    p = w.azurv1_supercritical()
    res = oracle.run(p, 40000, 61)
    assert int(res["tot"][4]) == 0                  # no face is reached
    assert int(res["tot"][9]) > 0                   # fission progeny
    pop, var = _population(p, res)
    te = p["tally"]["time_edges"]
    _check(pop, var, np.exp(0.1 * te[1:]))
    # the paper's figure, to its printed precision
    assert abs(pop[-1] - gold["growth"]) <= Z_MAX * math.sqrt(var[-1]) + 0.005
    assert round(math.exp((gold["c"] - 1.0) * gold["t_mft"]), 2) == gold["growth"]


def test_azurv1_time_averaged_flux():
    """Track-length flux, space-integrated per time bin: the average of
    e^{0.1 t} over the bin."""
    p = w.azurv1_supercritical()
    N = 40000
    res = oracle.run(p, N, 62)
    B = res["B"]
    Nb = oracle.batch_sizes(N, B).astype(float)
    te = p["tally"]["time_edges"]
    dt = np.diff(te)
    S = res["S"].reshape(B, dt.size, -1).sum(axis=2)
    mean = S.sum(0) / (N * dt)
    mb = S / (Nb[:, None] * dt[None, :])
    var = ((mb - mb.mean(0)) ** 2).sum(0) / (B * (B - 1))
    exact = (np.exp(0.1 * te[1:]) - np.exp(0.1 * te[:-1])) / (0.1 * dt)
    _check(mean, var, exact)


def test_azurv1_spread_second_moment():
    """Fission neutrons leave isotropically: the second spatial moment of
    the population, int x^2 n dx, follows the closed moment system of the
    plane pulse (fine 0.1-mfp bins make the in-bin x^2 error ~1e-3)."""
    p = w.azurv1_supercritical(n_bins=420, n_time_bins=10)
    N = 40000
    res = oracle.run(p, N, 67)
    B = res["B"]
    Nb = oracle.batch_sizes(N, B).astype(float)
    xe = p["tally"]["mesh"][0]
    xc = 0.5 * (xe[1:] + xe[:-1]) - 21.0
    h = np.diff(xe)
    X = res["X"].reshape(B, 10, -1)      # raw w v sums: v = 1, per bin
    m2b = (X * (xc ** 2)[None, None, :]).sum(axis=2) / Nb[:, None]
    m2 = (X * (xc ** 2)[None, None, :]).sum(axis=2).sum(0) / N
    var = ((m2b - m2b.mean(0)) ** 2).sum(0) / (B * (B - 1))
    te = p["tally"]["time_edges"]
    exact = np.array([plane_pulse_moments(1.1, t)[1] for t in te[1:]])
    _check(m2, var, exact)
    assert (h > 0).all()
    # the moment system reduces to the uncollided spread x = mu t for c = 0
    for t in (0.5, 3.0):
        assert abs(plane_pulse_moments(0.0, t)[1] - t * t * math.exp(-t) / 3.0) < 1e-13


def test_multigroup_fission_pulse_point_and_bins():
    edges = np.array([0.0, 0.5, 1.0, 2.0, 3.0])
    speed = [3.0, 2.0, 1.0]
    fis = {"sigma_f": [MG_SF], "nu": [MG_NU], "chi": [MG_CHI]}
    p = w.reflective_box(MG_ST, MG_SS, speed, size=(1.0, 1.0, 2.0), time_edges=edges, fission=fis)
    p["tally"]["time_crossing"] = True
    res = oracle.run(p, 60000, 63)
    e = oracle.estimates(p, res)
    f = (MG_SF, MG_NU, MG_CHI)
    pts = infinite_medium_pulse_points(np.array(MG_ST), np.array(MG_SS), np.array(speed), edges[1:], 2.0, f)
    bins = infinite_medium_pulse_bins(np.array(MG_ST), np.array(MG_SS), np.array(speed), edges, 2.0, f)
    _check(e["tc_mean"].ravel(), e["tc_var"].ravel(), pts.ravel())
    _check(e["mean"].ravel(), e["var"].ravel(), bins.ravel())
    # group 2 is born only by down-scatter (chi_2 = 0): still populated
    assert (e["mean"][:, 2] > 0).all()


def test_subcritical_multiplying_medium_steady():
    """One group, c = 0.3 + 2.5 * 0.2 = 0.8: phi = S / (Sigma_t (1 - c));
    three groups against M^-1 S with the fission term."""
    p = w.reflective_box([1.0], [[0.3]], [1.0], size=(1.0, 1.0, 1.0),
                         fission={"sigma_f": [[0.2]], "nu": [[2.5]], "chi": [[1.0]]})
    res = oracle.run(p, 60000, 64)
    e = oracle.estimates(p, res)
    _check(e["mean"].ravel(), e["var"].ravel(), [1.0 / 0.2])
    sf = [0.05, 0.08, 0.2]
    fis = {"sigma_f": [sf], "nu": [MG_NU], "chi": [MG_CHI]}
    p = w.reflective_box(MG_ST, MG_SS, [1.0, 1.0, 1.0], size=(1.0, 2.0, 3.0), fission=fis)
    res = oracle.run(p, 60000, 65)
    e = oracle.estimates(p, res)
    exact = infinite_medium_steady(np.array(MG_ST), np.array(MG_SS), 6.0, (sf, MG_NU, MG_CHI))
    _check(e["mean"].ravel(), e["var"].ravel(), exact)


def test_zero_fission_data_is_the_analog_run():
    """Fission data with Sigma_f = 0 changes nothing, bit for bit."""
    a = w.cfg3_lattice()
    b = w.cfg3_lattice()
    M, G = b["sigma_t"].shape
    b["fission"] = {"sigma_f": np.zeros((M, G)), "nu": np.full((M, G), 2.5),
                    "chi": np.tile(np.eye(G)[0], (M, 1))}
    ra = oracle.run(a, 3000, 66, records=True)
    rb = oracle.run(b, 3000, 66, records=True)
    assert np.array_equal(ra["rec"], rb["rec"])
    assert np.array_equal(ra["S"], rb["S"])
    assert np.array_equal(ra["tot"], rb["tot"])
