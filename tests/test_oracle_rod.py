"""Pins of the oracle's moving plane (a plane normal to z whose height is
linear in time between the time edges; above it a rod cell holds the rod's
material): closed forms and exact per-history event counts on a beam
crossing a descending rod, and a plane at rest against the same plane as a
fixed geometry plane."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

_G, _M63, _STRIDE = 2806196910506780709, (1 << 63) - 1, 152917


def _stream_start(seed, i):
    k = i * _STRIDE
    mod = (_G - 1) << 63
    gk = pow(_G, k, mod)
    return ((gk % (1 << 63)) * (seed & _M63) + (gk - 1) // (_G - 1)) & _M63


def _draw(s):
    s = (_G * s + 1) & _M63
    return s, (s >> 10) * 2.0 ** -53


def _beam_birth(seed, i):
    """Height and time of history i's beam particle (draws x, y, z, t)."""
    s = _stream_start(seed, i)
    s, _ = _draw(s)
    s, _ = _draw(s)
    s, xz = _draw(s)
    s, xt = _draw(s)
    return 0.0 + xz * 10.0, 0.0 + xt * 10.0


def test_descending_rod_transmission_closed_form():
    """Beam along x at height z, born at t_b (both uniform on [0, 10]); the
    rod above Z(t) = 10 - t absorbs with Sigma = 0.2.  The path inside the
    rod is min(10, t_b + z), so the transmission is E exp(-Sigma min(10, s))
    with s = t_b + z triangular on [0, 20]:
    (1 - e^{-10 S}(1 + 10 S)) / (100 S^2) + e^{-10 S} / 2."""
    S = 0.2
    p = w.rod_beam_box(sigma_rod=S)
    N = 200_000
    r = oracle.run(p, N, 3)
    exact = (1.0 - math.exp(-10 * S) * (1 + 10 * S)) / (100 * S * S) + 0.5 * math.exp(-10 * S)
    e = oracle.estimates(p, r)
    leak = float(e["leak_mean"][:, 0, 1].sum())       # through x+
    sig = math.sqrt(exact * (1 - exact) / N)
    assert abs(leak - exact) < 4.0 * sig, (leak, exact, sig)
    tot = r["tot"]
    assert int(tot[3] + tot[4] + tot[5]) == N               # absorbed + leaked + cut off
    assert int(tot[5]) == 0


def test_moving_plane_crossings_exact_per_history():
    """With a void rod material the moving plane changes nothing but still
    is crossed: a particle born at height z at time t_b meets the falling
    plane iff t_b + z < 10 (it starts below it and the plane comes down to
    it before it leaves).  Its surface events are that crossing plus the
    x+ face; every crossing lies on Z(t) = 10 - t."""
    p = w.rod_beam_box(void_rod=True)
    N, seed = 500, 7
    r = oracle.run(p, N, seed, records=True)
    expect = np.array([5 + int(sum(_beam_birth(seed, i)) < 10.0) for i in range(N)])
    assert np.array_equal(r["rec"][:, 1].astype(int), expect)
    assert 0.35 < (expect == 6).mean() < 0.65
    # trace rows (event, d, x, y, z, t, g, k, tau): a surface event off the
    # union planes x = 0, 2, ..., 10 is the plane crossing, at height 10 - t
    n_seen = 0
    for i in range(0, N, 25):
        rows = oracle.trace(p, N, seed, i)
        for row in rows:
            if row[0] == 1 and abs(row[2] / 2.0 - round(row[2] / 2.0)) > 1e-9:
                assert abs(row[4] - (10.0 - row[5])) < 1e-12, (i, row)
                n_seen += 1
    assert n_seen > 5


def test_plane_at_rest_equals_fixed_geometry_plane():
    """A plane at rest at z = 4 in a scattering box with the rod material
    above it, against the same box built with a geometry plane at z = 4 and
    that material above: the tallies agree within statistics."""
    st = [[1.0], [2.0]]
    ss = [[[0.7]], [[0.4]]]
    planes = [np.array([0.0, 3.0]), np.array([0.0, 3.0]), np.array([0.0, 10.0])]
    src = {"kind": "isotropic", "lo": [0.0, 0.0, 0.0], "hi": [3.0, 3.0, 10.0], "group_pmf": [1.0],
           "t_lo": 0.0, "t_hi": 0.0}
    tally = {"mesh": [np.array([0.0, 3.0]), np.array([0.0, 3.0]), np.linspace(0.0, 10.0, 6)],
             "time_edges": np.array([0.0, 2.0, 5.0]), "n_batches": 16}
    bc = [1, 1, 1, 1, 0, 0]
    a = w.make_problem(st, ss, [1.0], planes, np.zeros((1, 1, 1)), bc, src, tally)
    a["rod"] = {"z": np.array([4.0, 4.0, 4.0]), "material": np.ones((1, 1, 1), dtype=np.int32)}
    planes_b = [planes[0], planes[1], np.array([0.0, 4.0, 10.0])]
    b = w.make_problem(st, ss, [1.0], planes_b, np.array([[[0]], [[1]]]), bc, src, tally)
    N = 100_000
    ea = oracle.estimates(a, oracle.run(a, N, 11))
    eb = oracle.estimates(b, oracle.run(b, N, 12))
    ma, mb = ea["mean"].ravel(), eb["mean"].ravel()
    s = np.sqrt(ea["var"].ravel() + eb["var"].ravel())
    ok = s > 0
    z = np.abs(ma[ok] - mb[ok]) / s[ok]
    assert ok.sum() >= 8 and z.max() < 4.5, z


def test_invalid_rod_rejected():
    p = w.rod_beam_box()
    p["rod"]["z"] = np.array([10.0, math.nan, 0.0])
    with pytest.raises(RuntimeError):
        oracle.run(p, 10, 1)
