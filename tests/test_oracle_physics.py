"""Pins of the CPU oracle against closed forms and independent solvers.

Each test names the closed form it uses.  Statistical checks compare the
oracle's mean with the exact value within Z_MAX standard deviations (fixed
seeds, so every check is deterministic); the exact variance of a Bernoulli
transmission also pins the batch-variance estimator."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w
from refs import (infinite_medium_pulse_bins, infinite_medium_steady,
                  plane_pulse_uncollided_bin, pulse_population, slab_absorber_bins,
                  slab_absorber_transmission, sn_slab, sn_slab_mg,
                  sn_slab_mg_volume)

Z_MAX = 4.5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


# --------------------------------------------------------------------------
# purely absorbing slabs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("law", ["beam", "uniform", "cosine"])
def test_absorbing_slab_flux_bins(law):
    p = w.cfg1_slab_steady(c=0.0, mu_law=law)
    res = oracle.run(p, 200000, 11)
    e = oracle.estimates(p, res)
    edges = p["tally"]["mesh"][0]
    exact = slab_absorber_bins(edges, 1.0, law)
    m, v = e["mean"].ravel(), e["var"].ravel()
    ok = m > 0
    assert ok[:10].all()
    _check(m[ok], v[ok], exact[ok])
    # nothing scatters: one termination per history, absorb or leak
    tot = res["tot"]
    assert int(tot[2]) == int(tot[3])          # every collision absorbs
    assert int(tot[3] + tot[4]) == 200000


@pytest.mark.parametrize("law", ["beam", "uniform", "cosine"])
def test_absorbing_slab_transmission_bernoulli(law):
    """Transmission through 2 mfp is Bernoulli(p): the batch variance of the
    leak tally must match p (1 - p) / N."""
    p = w.slab(thickness=2.0, sigma_t=1.0, sigma_s=0.0, n_bins=4, source="surface",
               mu_law=law, n_batches=64)
    N = 256000
    res = oracle.run(p, N, 21)
    e = oracle.estimates(p, res)
    pt = slab_absorber_transmission(2.0, 1.0, law)
    est = e["leak_mean"][0, 0, 1]
    var_exact = pt * (1 - pt) / N
    assert abs(est - pt) < Z_MAX * math.sqrt(var_exact)
    ratio = e["leak_var"][0, 0, 1] / var_exact
    # chi-square with 63 degrees of freedom: 99.99% interval ~ [0.45, 1.75]
    assert 0.45 < ratio < 1.75
    # reflection back out of x- is impossible without scattering
    assert e["leak_mean"][0, 0, 0] == 0.0


# --------------------------------------------------------------------------
# scattering slab against discrete ordinates
# --------------------------------------------------------------------------

def test_scattering_slab_against_sn():
    p = w.cfg1_slab_steady(c=0.5, mu_law="cosine")
    res = oracle.run(p, 200000, 12)
    e = oracle.estimates(p, res)
    _, _, bins = sn_slab(10.0, 1.0, 0.5, n_cells=4000, n_mu=64)
    exact = bins(p["tally"]["mesh"][0])
    m, v = e["mean"].ravel(), e["var"].ravel()
    _check(m, v, exact, floor=2e-5 * exact.max())


def test_sn_solver_reduces_to_closed_form():
    # the S_N reference itself: without scattering it is the E3 closed form
    _, _, bins = sn_slab(10.0, 1.0, 0.0, n_cells=2000, n_mu=16)
    edges = np.linspace(0, 10, 21)
    np.testing.assert_allclose(bins(edges), slab_absorber_bins(edges, 1.0, "cosine"), rtol=1e-12)


# three groups with down- and up-scatter (from g to g'), a cosine current
# spread over the groups
MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5], [0.0, 0.2, 1.2]]
MG_PMF = [0.6, 0.3, 0.1]


def test_multigroup_sn_solver_reduces_to_one_group_solves():
    """Without coupling between groups each group is the one-group solver's
    flux (its own sweep code) scaled by its share of the current; without
    scattering each is the E3 closed form."""
    edges = np.linspace(0.0, 6.0, 13)
    diag = np.diag([0.3, 0.6, 1.2])
    mg = sn_slab_mg(6.0, MG_ST, diag, MG_PMF, n_cells=1200, n_mu=32)(edges)
    for g in range(3):
        _, _, one = sn_slab(6.0, MG_ST[g], diag[g, g], n_cells=1200, n_mu=32)
        # (both iterate to 1e-12 absolute)
        np.testing.assert_allclose(mg[g], MG_PMF[g] * one(edges), rtol=1e-9, atol=1e-11)
    free = sn_slab_mg(6.0, MG_ST, np.zeros((3, 3)), MG_PMF, n_cells=1200, n_mu=16)(edges)
    for g in range(3):
        np.testing.assert_allclose(free[g], MG_PMF[g] * slab_absorber_bins(edges, MG_ST[g], "cosine"), rtol=1e-12)


def test_multigroup_slab_matches_sn():
    """Leakage, group transfer (up-scatter included) and the angular law
    together: the oracle's 3-group slab bin fluxes, group by group, agree
    with the multigroup S_N solution."""
    prob = w.multigroup_slab(MG_ST, MG_SS, MG_PMF)
    edges = prob["tally"]["mesh"][0]
    res = oracle.run(prob, 200000, 15)
    e = oracle.estimates(prob, res)
    exact = sn_slab_mg(6.0, MG_ST, MG_SS, MG_PMF, n_cells=2400, n_mu=64)(edges)
    m, v = e["mean"].reshape(3, -1), e["var"].reshape(3, -1)
    _check(m, v, exact, floor=2e-5 * exact.max())


def test_volume_source_sn_infinite_limit():
    """The volume-source solver's flux far from thick faces is the
    infinite-medium M^-1 S (M = diag(St) - Ss^T), here mid-slab in a
    60-mfp slab."""
    st, ss = np.array(MG_ST), np.array(MG_SS)
    L = 60.0
    f = sn_slab_mg_volume(L, st, ss, MG_PMF, n_cells=3000, n_mu=32)(np.array([29.0, 31.0]))[:, 0]
    inf = np.linalg.solve(np.diag(st) - ss.T, np.array(MG_PMF) / L)
    np.testing.assert_allclose(f, inf, rtol=1e-6)


def test_reflected_box_column_matches_the_z_slab():
    """A 3-D box of one material, reflective on its x and y faces and
    vacuum on z, with a uniform volume source: the flux depends on z
    alone, and integrated over the box's cross-section (the tally's x and
    y axes carry no mesh planes, so they count with width 1) it is the
    multigroup z-slab's, so the 3-D tracking with reflections, leakage and
    group transfer is pinned against multigroup S_N."""
    H, nz = 8.0, 16
    prob = w.reflected_column(MG_ST, MG_SS, MG_PMF, height=H, n_z_bins=nz)
    res = oracle.run(prob, 100000, 16)
    e = oracle.estimates(prob, res)
    exact = sn_slab_mg_volume(H, MG_ST, MG_SS, MG_PMF, n_cells=1600, n_mu=64)(np.linspace(0.0, H, nz + 1))
    m, v = e["mean"].reshape(3, -1), e["var"].reshape(3, -1)
    _check(m, v, exact, floor=2e-5 * exact.max())


def test_balance_steady_slab():
    """Every history ends exactly once; absorption + leakage = 1 in mean."""
    p = w.cfg1_slab_steady(c=0.5, mu_law="cosine")
    N = 100000
    res = oracle.run(p, N, 13)
    tot = res["tot"]
    assert int(tot[3] + tot[4] + tot[5] + tot[6]) == N
    assert int(tot[0]) == 0                    # steady state: no census
    B = res["B"]
    Nb = oracle.batch_sizes(N, B)
    dx = np.diff(p["tally"]["mesh"][0])
    sa = 0.5
    # per batch: Sigma_a * total track + leaked weight, per history
    per_batch = (sa * res["S"].sum(axis=1) + res["L"].sum(axis=(1, 2, 3))) / Nb
    mean = per_batch.mean()
    sig = per_batch.std(ddof=1) / math.sqrt(B)
    assert abs(mean - 1.0) < Z_MAX * sig
    assert dx.size == 20


# --------------------------------------------------------------------------
# infinite media (all-reflective boxes)
# --------------------------------------------------------------------------

def test_infinite_medium_steady_one_group():
    p = w.reflective_box([1.0], [[0.5]], [1.0], size=(2.0, 2.0, 2.0))
    res = oracle.run(p, 100000, 14)
    e = oracle.estimates(p, res)
    exact = 1.0 / (8.0 * 0.5)                  # S / Sigma_a
    _check(e["mean"], e["var"], [exact])
    tot = res["tot"]
    assert int(tot[4]) == 0 and int(tot[3]) == 100000


MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1],
         [0.0, 0.6, 0.5],
         [0.0, 0.2, 1.2]]       # includes up-scatter 2 -> 1 to expose a transpose


def test_infinite_medium_steady_multigroup():
    p = w.reflective_box(MG_ST, MG_SS, [1.0, 1.0, 1.0], size=(1.0, 2.0, 3.0))
    res = oracle.run(p, 100000, 15)
    e = oracle.estimates(p, res)
    exact = infinite_medium_steady(np.array(MG_ST), np.array(MG_SS), 6.0)
    _check(e["mean"].ravel(), e["var"].ravel(), exact)


def test_infinite_medium_pulse_one_group():
    edges = np.linspace(0.0, 10.0, 21)
    p = w.reflective_box([1.0], [[0.9]], [2.0], size=(1.0, 1.0, 1.0), time_edges=edges)
    res = oracle.run(p, 100000, 16)
    e = oracle.estimates(p, res)
    exact = infinite_medium_pulse_bins(np.array([1.0]), np.array([[0.9]]), np.array([2.0]),
                                       edges, 1.0)
    _check(e["mean"].ravel(), e["var"].ravel(), exact.ravel())
    # every history is absorbed or cut off at t = 10
    tot = res["tot"]
    assert int(tot[3] + tot[5]) == 100000


def test_infinite_medium_pulse_multigroup():
    edges = np.array([0.0, 0.25, 0.5, 1.0, 2.0, 4.0])
    speed = [3.0, 2.0, 1.0]
    p = w.reflective_box(MG_ST, MG_SS, speed, size=(1.0, 1.0, 2.0), time_edges=edges)
    res = oracle.run(p, 100000, 17)
    e = oracle.estimates(p, res)
    exact = infinite_medium_pulse_bins(np.array(MG_ST), np.array(MG_SS), np.array(speed),
                                       edges, 2.0)
    _check(e["mean"].ravel(), e["var"].ravel(), exact.ravel())


def test_pulse_population_law_and_paper_growth_factor():
    """Section 3 quotes a population growth of about 7.39 over 20 mean free
    times for c = 1.1; the same law exp((c - 1) t) governs the decay of the
    subcritical pulse the oracle tracks (c = 0.9)."""
    with open(os.path.join(GOLDEN, "azurv1_growth.json")) as f:
        gold = json.load(f)
    assert round(pulse_population(gold["c"], gold["t_mft"]), 2) == gold["growth"]
    # one-group infinite medium with Sigma_t = v = 1: time is in mean free times
    edges = np.linspace(0.0, 20.0, 11)
    p = w.reflective_box([1.0], [[0.9]], [1.0], size=(1.0, 1.0, 1.0), time_edges=edges)
    res = oracle.run(p, 100000, 18)
    e = oracle.estimates(p, res)
    # bin-averaged population = phi / v per unit volume (volume 1)
    exact = [(math.exp(-0.1 * a) - math.exp(-0.1 * b)) / (0.1 * (b - a))
             for a, b in zip(edges[:-1], edges[1:])]
    pops = [pulse_population(0.9, t) for t in edges]
    assert all(pops[j + 1] < exact[j] < pops[j] for j in range(10))
    _check(e["mean"].ravel(), e["var"].ravel(), exact)


# --------------------------------------------------------------------------
# pulsed slab (the 40 mfp slab with a centre pulse)
# --------------------------------------------------------------------------

def test_plane_pulse_totals_exact():
    """No particle reaches a face before t = 20 (distance 20 = v t), so the
    space-integrated flux per time bin is exactly the infinite-medium one."""
    p = w.cfg2_slab_pulse(c=0.9)
    N = 100000
    res = oracle.run(p, N, 2)
    assert int(res["tot"][4]) == 0             # no leakage
    B = res["B"]
    Nb = oracle.batch_sizes(N, B)
    dt = np.diff(p["tally"]["time_edges"])
    S = res["S"].reshape(B, 100, 50).sum(axis=2)        # raw track per time bin
    per_batch = S / (Nb[:, None] * dt[None, :])
    mean = S.sum(0) / (N * dt)
    sig = per_batch.std(axis=0, ddof=1) / math.sqrt(B)
    te = p["tally"]["time_edges"]
    sa = 0.1
    exact = (np.exp(-sa * te[:-1]) - np.exp(-sa * te[1:])) / (sa * dt)
    _check(mean, sig ** 2, exact)


def test_plane_pulse_symmetry():
    """Birth exactly on the x = 20 tally plane: mirror bins agree."""
    p = w.cfg2_slab_pulse(c=0.9)
    res = oracle.run(p, 100000, 3)
    e = oracle.estimates(p, res)
    m = e["mean"][:, 0, 0, 0, :]
    v = e["var"][:, 0, 0, 0, :]
    d = m - m[:, ::-1]
    s = np.sqrt(v + v[:, ::-1])
    assert (np.abs(d) <= Z_MAX * s + 1e-15).all()


def test_plane_pulse_uncollided_shape():
    """Purely absorbing variant: phi = e^{-St v t} / (2 t) on |x - 20| < v t."""
    p = w.cfg2_slab_pulse(c=0.0)
    res = oracle.run(p, 100000, 4)
    e = oracle.estimates(p, res)
    xe = p["tally"]["mesh"][0]
    te = p["tally"]["time_edges"]
    K = 20
    exact = np.zeros((K, 50))
    for k in range(K):
        for j in range(50):
            exact[k, j] = plane_pulse_uncollided_bin(20.0, 1.0, 1.0, xe[j], xe[j + 1],
                                                     te[k], te[k + 1]) / ((xe[j + 1] - xe[j]) * (te[k + 1] - te[k]))
    m = e["mean"][:K, 0, 0, 0, :]
    v = e["var"][:K, 0, 0, 0, :]
    _check(m, v, exact)
    assert (m[exact == 0] == 0).all()


# --------------------------------------------------------------------------
# void streaming
# --------------------------------------------------------------------------

def test_void_streaming_mean_chord():
    """Void box, isotropic point source at the centre of [0,2]^3: the scored
    track of each history is its straight exit distance; the mean over the
    sphere of directions is a fixed integral."""
    from scipy.integrate import dblquad

    p = w.void_box(size=(2.0, 2.0, 2.0), n_mesh=(2, 2, 2), src_point=(1.0, 1.0, 1.0))
    N = 50000
    res = oracle.run(p, N, 5, records=True)
    trk = res["trk"][:, 0]

    def exit_dist(phi, mu):
        s = math.sqrt(1 - mu * mu)
        u = (s * math.cos(phi), s * math.sin(phi), mu)
        return min(1.0 / abs(c) if c != 0 else math.inf for c in u)

    val, _ = dblquad(exit_dist, -1.0, 1.0, 0.0, 2 * math.pi, epsabs=1e-10)
    exact = val / (4 * math.pi)
    assert abs(trk.mean() - exact) < Z_MAX * trk.std(ddof=1) / math.sqrt(N)
    # every history leaks once, crossing at most 3 interior planes first
    rec = res["rec"]
    assert (rec[:, 2] == 0).all() and (rec[:, 1] >= 1).all() and (rec[:, 1] <= 4).all()
    assert (rec[:, 4] == 1 << oracle.T_LEAK).all()
    # the raw tally sums to the sum of the per-history tracks
    assert math.isclose(res["S"].sum(), trk.sum(), rel_tol=1e-12)


# --------------------------------------------------------------------------
# 1/sqrt(N) convergence (Section 3)
# --------------------------------------------------------------------------

def test_error_converges_as_inverse_sqrt_n():
    p = w.cfg1_slab_steady(c=0.0, mu_law="beam")
    edges = p["tally"]["mesh"][0]
    exact = slab_absorber_bins(edges, 1.0, "beam")[:8]
    Ns = [1000, 10000, 100000]
    errs = []
    for N in Ns:
        e2 = []
        for seed in range(1, 9):
            e = oracle.estimates(p, oracle.run(p, N, 1000 * seed + N))
            e2.append(np.mean((e["mean"].ravel()[:8] - exact) ** 2))
        errs.append(math.sqrt(np.mean(e2)))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert -0.65 < slope < -0.35, (slope, errs)
