"""Pins of the oracle's population control at census (reading R16:
splitting-roulette to a target population, exact fixed-point total weight).

The exact pins use void all-reflective boxes, where no random number is
used after birth, so every trajectory is fixed by its birth: a target equal
to the population leaves every particle alone (n = 1 for all), a target of
twice the population doubles every particle exactly once, and in both
cases the tallies equal the uncontrolled run's.  The statistical pin is the
pulsed plane source in a slab (the paper's AZURV1-type time-dependent
verification, Section 3), whose spatially integrated flux has a closed
form while the boundaries are out of reach."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from workloads import problems as W


def _exact_q64(ws):
    tot = 0
    for w in ws:
        tot += math.floor(Fraction(float(w)) * 2 ** 64)
    return tot >> 64, tot & (2 ** 64 - 1), tot


def test_q64_sum_is_the_exact_truncated_sum():
    rng = np.random.default_rng(5)
    ws = np.concatenate([rng.random(500), rng.random(50) * 2.0 ** 31, 10.0 ** rng.uniform(-25, -15, 50),
                         [0.0, 5e-324, 2.0 ** -64, 2.0 ** -65, 3 * 2.0 ** -66, 1.0, 2.0 ** 32 - 1]])
    (hi, lo), val = oracle.q64_sum(ws)
    ehi, elo, tot = _exact_q64(ws)
    assert (hi, lo) == (ehi, elo)
    # order-free
    (hi2, lo2), val2 = oracle.q64_sum(ws[::-1].copy())
    assert (hi2, lo2) == (hi, lo) and val2 == val
    # the double is within two roundings of the exact fixed-point value
    exact = Fraction(tot, 2 ** 64)
    assert abs(Fraction(val) - exact) <= 2 * Fraction(math.ulp(float(exact)))
    # carries across the 2^64 boundary of the low word
    (h, l), _ = oracle.q64_sum([0.75, 0.75])
    assert (h, l) == (1, 2 ** 63)


def test_q64_sum_rejects_large_weights():
    with pytest.raises(ValueError):
        oracle.q64_sum([1.0, 2.0 ** 32])
    with pytest.raises(ValueError):
        oracle.q64_sum([-1.0])


def _void_reflective(K=4, speed=1.0):
    return W.void_box(size=(2.0, 1.5, 1.0), n_mesh=(2, 3, 1), src_point=(0.3, 0.7, 0.4),
                      time_edges=list(np.linspace(0.0, 4.0, K + 1)), speed=speed,
                      bc=[W.REFLECTIVE] * 6)


def test_target_equal_to_the_population_is_the_identity():
    prob = _void_reflective()
    N = 3000
    pc = oracle.run_pc(prob, N, 7, target=N)
    an = oracle.run(prob, N, 7)
    assert list(pc["pop"]) == [N] * 4
    assert int(pc["tot"][8]) == 0 and int(pc["tot"][3 + oracle.T_ROULETTE]) == 0
    assert int(pc["tot"][3 + oracle.T_TIME]) == N
    np.testing.assert_allclose(pc["S"], an["S"], rtol=1e-13, atol=0)
    # every particle flies v dt in every bin: sum over the box = N v dt
    tot_k = pc["S"].sum(axis=0).reshape(4, -1).sum(axis=1)
    np.testing.assert_allclose(tot_k, N * 1.0 * 1.0, rtol=1e-12)


def test_twice_the_population_doubles_every_particle_once():
    prob = _void_reflective()
    N = 2000
    pc = oracle.run_pc(prob, N, 11, target=2 * N)
    an = oracle.run(prob, N, 11)
    # T_1: every weight-1 particle makes floor(2 + xi) = 2 copies of weight
    # 1/2; later edges: floor(1 + xi) = 1
    assert list(pc["pop"]) == [N, 2 * N, 2 * N, 2 * N]
    assert int(pc["tot"][8]) == N
    assert int(pc["tot"][3 + oracle.T_ROULETTE]) == 0
    assert int(pc["tot"][3 + oracle.T_TIME]) == 2 * N
    np.testing.assert_allclose(pc["S"], an["S"], rtol=1e-12, atol=0)


def test_half_the_population_roulettes_half():
    prob = _void_reflective()
    N = 4000
    pc = oracle.run_pc(prob, N, 13, target=N // 2)
    # T_1: w_t = 2, each particle survives with probability 1/2 at weight 2
    p1 = int(pc["pop"][1])
    assert abs(p1 - N / 2) < 5 * math.sqrt(N / 4)
    # particles are only rouletted or split, never lost
    born = int(pc["pop"][0])
    assert born + int(pc["tot"][8]) == int(pc["tot"][3 + oracle.T_ROULETTE]) + int(pc["tot"][3 + oracle.T_TIME])


def _slab_pulse(c=0.5, K=20):
    return W.slab(thickness=40.0, sigma_t=1.0, sigma_s=c, speed=1.0, n_bins=40, source="plane",
                  x_src=20.0, time_edges=np.linspace(0.0, 20.0, K + 1), n_batches=16)


def test_controlled_pulse_matches_the_closed_form_and_beats_analog_late():
    c, K, N = 0.5, 20, 20000
    prob = _slab_pulse(c, K)
    pc = oracle.run_pc(prob, N, 21, target=N)
    est = oracle.estimates(prob, pc)
    dx = 1.0
    integ = est["mean"].reshape(K, -1).sum(axis=1) * dx
    ivar = est["var"].reshape(K, -1).sum(axis=1) * dx * dx
    te = np.linspace(0.0, 20.0, K + 1)
    sa = 1.0 - c
    exact = (np.exp(-sa * te[:-1]) - np.exp(-sa * te[1:])) / (sa * np.diff(te))
    z = (integ - exact) / np.sqrt(ivar)
    assert np.all(np.abs(z) < 5.0), z
    # the population stays at the target (in expectation; +-5 sigma)
    pop = pc["pop"][1:].astype(np.float64)
    assert np.all(np.abs(pop - N) < 5 * math.sqrt(N)), pop
    # balance: born + splits = rouletted + absorbed + leaked + cut off
    t = pc["tot"].astype(np.int64)
    assert N + t[8] == t[3] + t[4] + t[5] + t[6] + t[7]
    # late-time relative error far below the analog run's
    an = oracle.estimates(prob, oracle.run(prob, N, 21))
    ia = an["mean"].reshape(K, -1).sum(axis=1)
    va = an["var"].reshape(K, -1).sum(axis=1)
    rel_pc = math.sqrt(ivar[-1]) / integ[-1]
    rel_an = math.sqrt(va[-1]) / ia[-1] if ia[-1] > 0 else math.inf
    assert rel_pc < rel_an / 5.0, (rel_pc, rel_an)


def test_rejects_what_it_does_not_model():
    prob = W.azurv1_supercritical()
    with pytest.raises(RuntimeError):
        oracle.run_pc(prob, 100, 1, target=100)
    with pytest.raises(RuntimeError):
        oracle.run_pc(_void_reflective(), 100, 1, target=0)


def test_later_births_wait_for_their_own_edge():
    """Births spread over all four time bins of a void reflective box,
    target N.  The first edge controls the particles of bins 0 and 1 only
    (about N/2 of weight 1, so about N/2 extra copies); a control over every
    particle alive would leave all N of weight 1 as they are (no copies)."""
    prob = _void_reflective()
    prob["source"]["t_lo"], prob["source"]["t_hi"] = 0.0, 4.0
    N = 4000
    pc = oracle.run_pc(prob, N, 17, target=N)
    an = oracle.run(prob, N, 17)
    assert int(pc["tot"][8]) > N // 4
    assert abs(int(pc["pop"][1]) - N) < 5 * math.sqrt(N)
    born = int(pc["pop"][0])
    assert born + int(pc["tot"][8]) == int(pc["tot"][3 + oracle.T_ROULETTE]) + int(pc["tot"][3 + oracle.T_TIME])
    # unbiased: the total track per time bin matches the uncontrolled run
    tk = pc["S"].sum(axis=0).reshape(4, -1).sum(axis=1)
    ta = an["S"].sum(axis=0).reshape(4, -1).sum(axis=1)
    np.testing.assert_allclose(tk, ta, rtol=0.05)


def test_steady_state_has_no_edge_to_control():
    """One time bin [0, inf): no inner census edge, so the controlled run is
    the uncontrolled one (same events, same tallies)."""
    prob = W.cfg1_slab_steady(c=0.5)
    N = 3000
    pc = oracle.run_pc(prob, N, 23, target=N // 3)
    an = oracle.run(prob, N, 23)
    assert np.array_equal(pc["tot"], an["tot"])
    np.testing.assert_allclose(pc["S"], an["S"], rtol=1e-13, atol=0)
    assert list(pc["pop"]) == [N]


def test_target_of_one_particle():
    """Target 1: every edge keeps about one particle of the whole weight; the
    run stays balanced and unbiased in expectation (a single edge: the
    expected number of survivors is exactly 1)."""
    prob = _void_reflective()
    N = 2000
    pc = oracle.run_pc(prob, N, 29, target=1)
    born = int(pc["pop"][0])
    t = pc["tot"].astype(np.int64)
    assert born + t[8] == t[3 + oracle.T_ROULETTE] + t[3 + oracle.T_TIME]
    assert all(int(x) <= 10 for x in pc["pop"][1:])
