"""Pins of the oracle's population control by combing (reading R28: the
controlled particles in the run's list order, M teeth spaced W / M at one
random offset per edge, each particle copied once per tooth in its stretch
of the cumulative fixed-point weight).

The comb itself is pinned against exact rational arithmetic: every count
is the floor or the ceiling of M q / W (q the fixed-point weight, W their
sum), the counts add up to M for every offset, and their mean over a
uniform grid of offsets is M q / W.  The runs are pinned where no
randomness is left to the control: in a purely scattering all-reflective
box every particle keeps weight 1, so a target equal to the population
must reproduce the uncontrolled run exactly (the comb keeps every stream,
unlike splitting-roulette, which draws), and a target of twice the
population must copy every particle exactly twice at the first edge.  The
pulsed plane source in an absorbing slab checks unbiasedness against its
closed form with the population held at exactly the target."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from workloads import problems as W


def _q(w):
    return math.floor(Fraction(float(w)) * 2 ** 64)


def _weights(rng, n):
    return np.concatenate([rng.random(n // 2) * 3.0, 10.0 ** rng.uniform(-9, 2, n - n // 2)])


@pytest.mark.parametrize("M", [1, 7, 100, 12345])
def test_comb_counts_are_floor_or_ceil_and_sum_to_the_target(M):
    rng = np.random.default_rng(M)
    w = _weights(rng, 300)
    q = [_q(x) for x in w]
    Wq = sum(q)
    for u in [0.0, 0.25, 0.5, 0.999999, *rng.random(20)]:
        n = oracle.comb(w, M, u).astype(np.int64)
        assert int(n.sum()) == M
        for r in range(w.size):
            e = Fraction(M * q[r], Wq)
            assert math.floor(e) <= n[r] <= math.ceil(e), (r, n[r], float(e))


def test_comb_mean_over_offsets_is_proportional_to_weight():
    rng = np.random.default_rng(3)
    w = _weights(rng, 60)
    M, grid = 37, 4096
    q = [_q(x) for x in w]
    Wq = sum(q)
    acc = np.zeros(w.size)
    for j in range(grid):
        acc += oracle.comb(w, M, (j + 0.5) / grid)
    mean = acc / grid
    exact = np.array([float(Fraction(M * qi, Wq)) for qi in q])
    assert np.max(np.abs(mean - exact)) <= 1.0 / grid + 1e-12


def test_comb_order_changes_who_but_not_how_many():
    rng = np.random.default_rng(9)
    w = _weights(rng, 100)
    a = oracle.comb(w, 50, 0.4)
    perm = rng.permutation(w.size)
    b = oracle.comb(w[perm], 50, 0.4)
    assert int(a.sum()) == int(b.sum()) == 50
    q = [_q(x) for x in w]
    Wq = sum(q)
    for r in range(w.size):
        e = Fraction(50 * q[perm[r]], Wq)
        assert math.floor(e) <= b[r] <= math.ceil(e)


def _scattering_box(K=5):
    return W.reflective_box([1.3], [[1.3]], [1.0], size=(2.0, 1.0, 1.5),
                            time_edges=list(np.linspace(0.0, 2.5, K + 1)), n_batches=8)


def test_comb_at_the_population_is_the_uncontrolled_run():
    prob = _scattering_box()
    N = 3000
    pc = oracle.run_pc(prob, N, 31, target=N, method="comb")
    an = oracle.run(prob, N, 31)
    assert list(pc["pop"]) == [N] * 5
    # the same events and terminations: no copy, no roulette, every stream kept
    assert np.array_equal(pc["tot"], an["tot"])
    np.testing.assert_allclose(pc["S"], an["S"], rtol=1e-12, atol=0)
    # splitting-roulette at the same target draws once per particle and edge,
    # so its trajectories differ (its tallies agree only statistically)
    sr = oracle.run_pc(prob, N, 31, target=N, method="split")
    assert not np.array_equal(sr["tot"][:3], an["tot"][:3])


def test_comb_at_twice_the_population_doubles_every_particle_once():
    prob = _scattering_box()
    N = 2000
    pc = oracle.run_pc(prob, N, 37, target=2 * N, method="comb")
    # T_1: 2 N teeth over N equal weights: exactly two copies each, weight 1/2;
    # later edges: 2 N particles of weight 1/2, one tooth each
    assert list(pc["pop"]) == [N] + [2 * N] * 4
    assert int(pc["tot"][8]) == N
    assert int(pc["tot"][3 + oracle.T_ROULETTE]) == 0
    assert int(pc["tot"][3 + oracle.T_TIME]) == 2 * N
    # flux per time bin: every particle flies v dt in every bin
    tot_k = pc["S"].sum(axis=0).reshape(5, -1).sum(axis=1)
    np.testing.assert_allclose(tot_k, N * 1.0 * 0.5, rtol=1e-12)


def _slab_pulse(c=0.5, K=20):
    return W.slab(thickness=40.0, sigma_t=1.0, sigma_s=c, speed=1.0, n_bins=40, source="plane",
                  x_src=20.0, time_edges=np.linspace(0.0, 20.0, K + 1), n_batches=16)


def test_combed_pulse_holds_the_target_and_matches_the_closed_form():
    c, K, N = 0.5, 20, 20000
    prob = _slab_pulse(c, K)
    pc = oracle.run_pc(prob, N, 41, target=N, method="comb")
    # exactly the target at every inner edge
    assert all(int(x) == N for x in pc["pop"][1:]), pc["pop"]
    est = oracle.estimates(prob, pc)
    integ = est["mean"].reshape(K, -1).sum(axis=1)
    ivar = est["var"].reshape(K, -1).sum(axis=1)
    te = np.linspace(0.0, 20.0, K + 1)
    sa = 1.0 - c
    exact = (np.exp(-sa * te[:-1]) - np.exp(-sa * te[1:])) / (sa * np.diff(te))
    z = (integ - exact) / np.sqrt(ivar)
    assert np.all(np.abs(z) < 5.0), z
    t = pc["tot"].astype(np.int64)
    assert N + t[8] == t[3] + t[4] + t[5] + t[6] + t[7]


def test_comb_edge_streams_differ_by_seed_and_edge():
    """The offset of each edge comes from its own stream: two seeds give
    different copies, the same seed the same run."""
    prob = _slab_pulse(0.7, K=8)
    a = oracle.run_pc(prob, 5000, 5, target=3000, method="comb")
    b = oracle.run_pc(prob, 5000, 5, target=3000, method="comb")
    c = oracle.run_pc(prob, 5000, 6, target=3000, method="comb")
    assert np.array_equal(a["tot"], b["tot"]) and np.array_equal(a["S"], b["S"])
    assert not np.array_equal(a["tot"], c["tot"])
    assert all(int(x) == 3000 for x in a["pop"][1:])


def test_comb_rejects_unknown_method():
    with pytest.raises(KeyError):
        oracle.run_pc(_slab_pulse(), 100, 1, target=100, method="combing")
