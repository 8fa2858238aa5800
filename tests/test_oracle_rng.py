"""Pins of the oracle's random-number streams against the generator's
mathematical definition (63-bit LCG, Brown's skip-ahead, SplitMix64)."""
import numpy as np
import pytest

import oracle
from refs import LCG_C, LCG_G, LCG_STRIDE, MOD, lcg_skip_closed_form, lcg_step, xi_of


def test_full_period_conditions():
    # Hull-Dobell for a power-of-two modulus: c odd and g = 1 (mod 4)
    assert LCG_C % 2 == 1
    assert LCG_G % 4 == 1


@pytest.mark.parametrize("bits", [8, 12, 16])
def test_full_period_brute_force_on_reductions(bits):
    # the generator reduced mod 2^bits must visit every residue once
    m = 1 << bits
    g, s, seen = LCG_G % m, 0, set()
    for _ in range(m):
        s = (g * s + LCG_C) % m
        seen.add(s)
    assert len(seen) == m and s == 0


@pytest.mark.parametrize("seed", [0, 1, 12345, (1 << 63) - 1, 0xDEADBEEFCAFEBABE])
@pytest.mark.parametrize("k", [0, 1, 2, 7, 1000, LCG_STRIDE, 123456789012, (1 << 62) + 3])
def test_skip_matches_closed_form(seed, k):
    assert oracle.rng_skip(seed, k) == lcg_skip_closed_form(seed % MOD, k)


def test_skip_equals_single_steps():
    s = 987654321
    ref = s
    for k in range(1, 2001):
        ref = lcg_step(ref)
        if k in (1, 2, 3, 10, 999, 2000):
            assert oracle.rng_skip(s, k) == ref


def test_skip_composes():
    s = 42
    a, b = 77777, 1234567
    assert oracle.rng_skip(oracle.rng_skip(s, a), b) == oracle.rng_skip(s, a + b)


def test_draws_and_uniforms():
    s0 = lcg_skip_closed_form(5, 3 * LCG_STRIDE)
    st, xi = oracle.rng_draws(s0, 500)
    s = s0
    for j in range(500):
        s = lcg_step(s)
        assert int(st[j]) == s
        assert xi[j] == xi_of(s)
    assert xi.min() >= 0.0 and xi.max() <= 1.0 - 2.0 ** -53


def test_uniform_moments():
    _, xi = oracle.rng_draws(1, 200000)
    assert abs(xi.mean() - 0.5) < 4 * np.sqrt(1 / 12 / xi.size)
    assert abs((xi ** 2).mean() - 1 / 3) < 4 * np.sqrt(4 / 45 / xi.size)


def test_child_stream_splitmix64_published_vector():
    # SplitMix64 seeded with 1234567: the first five outputs of the reference
    # generator (Steele, Lea & Flood 2014; Vigna's splitmix64.c); each output
    # is the finalizer applied to seed + n * 0x9E3779B97F4A7C15.
    expected = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                4593380528125082431, 16408922859458223821]
    gamma = 0x9E3779B97F4A7C15
    mask64 = (1 << 64) - 1
    for n, e in enumerate(expected):
        state = (1234567 + n * gamma) & mask64
        assert oracle.child_stream(state, 0) == e & (MOD - 1)


def test_child_streams_depend_on_lineage_only():
    p = 0x123456789ABCDEF
    kids = [oracle.child_stream(p, j) for j in range(1, 17)]
    assert len(set(kids)) == 16
    assert all(0 <= k < MOD for k in kids)
    assert kids == [oracle.child_stream(p, j) for j in range(1, 17)]
