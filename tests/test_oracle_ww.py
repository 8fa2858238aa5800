"""Pins of the oracle's weight-window game: with no windows it is the
analog game bit for bit; with windows it stays unbiased (means agree with
analog within statistics) while spreading particles toward the detector."""
import math

import numpy as np

import oracle
import workloads as w
from ww_tables import flux_table


def test_zero_table_is_analog_bit_exact():
    p = w.cfg5_dogleg()
    G = 2
    zero = np.zeros((1, G, 10, 10, 40))
    a = oracle.run(p, 3000, 5, records=True)
    b = oracle.run(p, 3000, 5, records=True, ww_center=zero)
    assert np.array_equal(a["rec"], b["rec"])
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["q"], b["q"])
    assert int(b["tot"][8]) == 0


def test_windows_unbiased_dogleg():
    p = w.cfg5_dogleg(detector=w.LEG_A_DETECTOR)
    table = flux_table(p, floor=1e-3)
    N = 20000
    a = oracle.run(p, N, 7)
    b = oracle.run(p, N, 8, ww_center=table)
    ea, eb = oracle.estimates(p, a), oracle.estimates(p, b)
    assert int(b["tot"][8]) > 0 and int(b["tot"][7]) > 0          # splits and roulettes happen
    # detector (quantity of interest): means agree within 4 sigma
    d = eb["qoi_mean"] - ea["qoi_mean"]
    s = math.sqrt(ea["qoi_var"] + eb["qoi_var"])
    assert abs(d) < 4.0 * s, (ea["qoi_mean"], eb["qoi_mean"], s)
    # tally bins with decent statistics on both sides agree within 4.5 sigma
    ma, mb = ea["mean"].ravel(), eb["mean"].ravel()
    va, vb = ea["var"].ravel(), eb["var"].ravel()
    ok = (ma > 0) & (mb > 0) & (np.sqrt(va) < 0.2 * ma) & (np.sqrt(vb) < 0.2 * mb)
    z = np.abs(ma[ok] - mb[ok]) / np.sqrt(va[ok] + vb[ok])
    # 32-batch variances are themselves uncertain by ~25%, hence 5 sigma
    assert ok.sum() > 200 and z.max() < 5.0, (ok.sum(), z.max())
    # windows shrink the detector's relative error per history
    ra = math.sqrt(ea["qoi_var"]) / ea["qoi_mean"]
    rb = math.sqrt(eb["qoi_var"]) / eb["qoi_mean"]
    assert rb < ra


def test_windows_unbiased_time_dependent():
    """Census check points: windows per time bin on the pulsed slab."""
    p = w.cfg2_slab_pulse()
    p["ww_mesh"] = [p["tally"]["mesh"][0], np.zeros(0), np.zeros(0)]
    table = flux_table(p, N=20000, floor=1e-3)
    N = 20000
    a = oracle.run(p, N, 3)
    b = oracle.run(p, N, 4, ww_center=table)
    ea, eb = oracle.estimates(p, a), oracle.estimates(p, b)
    assert int(b["tot"][8]) > 0
    te = p["tally"]["time_edges"]
    S = (eb["mean"][:, 0, 0, 0, :] * 0.8).sum(1)
    exact = (np.exp(-0.1 * te[:-1]) - np.exp(-0.1 * te[1:])) / (0.1 * np.diff(te))
    B = b["B"]
    Nb = oracle.batch_sizes(N, B)
    per_batch = b["S"].reshape(B, 100, 50).sum(2) / (Nb[:, None] * np.diff(te)[None, :])
    sig = per_batch.std(axis=0, ddof=1) / math.sqrt(B)
    assert (np.abs(S - exact) < 4.5 * sig + 1e-12).all()


# ---------------------------------------------------------------------------
# The window game on hand-built particles: a void slab [0, 2] entered by a
# beam at x = 0 (weight 1, direction +x), window cells [0, 1] (no window)
# and [1, 2] (centre w_c); the detector is the second cell.  Crossing x = 1
# is the one window check of each history, so its outcome is known by hand.
# ---------------------------------------------------------------------------

_G, _M63, _STRIDE = 2806196910506780709, (1 << 63) - 1, 152917


def _void_beam(wc_right):
    p = w.slab(thickness=2.0, sigma_t=0.0, sigma_s=0.0, n_bins=2, source="surface",
               mu_law="beam", n_batches=4)
    p["ww_mesh"] = [np.array([0.0, 1.0, 2.0]), np.zeros(0), np.zeros(0)]
    p["qoi"] = {"lo": np.array([1.0, 0.0, 0.0]), "hi": np.array([2.0, 0.0, 0.0]),
                "group_mask": np.array([1], dtype=np.int32)}
    table = np.zeros((1, 1, 1, 1, 2))
    table[..., 1] = wc_right
    return p, table


def _stream_start(seed, i):
    """LCG state after i * stride steps from the seed: the closed form
    g^k s + (g^k - 1) / (g - 1) mod 2^63 with exact integers."""
    k = i * _STRIDE
    mod = (_G - 1) << 63
    gk = pow(_G, k, mod)
    return ((gk % (1 << 63)) * (seed & _M63) + (gk - 1) // (_G - 1)) & _M63


def _draw(s):
    s = (_G * s + 1) & _M63
    return s, (s >> 10) * 2.0 ** -53


def test_ww_split_by_hand():
    """w = 1 above w_U = rho * 2 w_c / (1 + rho): rho = 5, w_c = 0.13 gives
    w_U = 0.21667, n = ceil(1 / w_U) = 5 copies of weight 0.2; each streams
    the unit width of the detector cell and leaks."""
    p, table = _void_beam(0.13)
    N = 64
    r = oracle.run(p, N, 11, records=True, ww_center=table)
    assert int(r["tot"][8]) == 4 * N                              # splits
    assert int(r["tot"][4]) == 5 * N and int(r["tot"][3]) == 0     # 5 leaks, no absorption
    assert (r["rec"][:, 3] == 5).all()                            # particles per history
    assert (r["rec"][:, 1] == 2 + 4).all()                        # parent 2 crossings, each child 1
    assert np.allclose(r["trk"][:, 1], 5 * 0.2, rtol=0, atol=4e-16)
    S = r["S"].sum(0)
    assert np.allclose(S, [N * 1.0, N * 1.0], rtol=1e-15)


def test_ww_split_capped_by_hand():
    """w_c = 0.01: w_U = 1/60, so ceil(w / w_U) is about 60, above the cap of
    16: 16 copies of weight 1/16 (exact in binary64)."""
    p, table = _void_beam(0.01)
    N = 32
    r = oracle.run(p, N, 12, records=True, ww_center=table)
    assert int(r["tot"][8]) == 15 * N
    assert (r["rec"][:, 3] == 16).all()
    assert (r["trk"][:, 1] == 1.0).all()          # 16 x 0.0625 x 1 with exact sums


def test_ww_roulette_by_hand():
    """w = 1 below w_L = 2 w_c / (1 + rho) = 10/6 with w_c = 5: one draw xi,
    survival iff xi < w / w_c = 0.2, at weight w_c = 5.  The draw is the one
    after the birth's: three position draws, time, group, mu, the azimuth's
    rejection pairs (0 < a^2 + b^2 < 1) and the optical depth; the void
    flight to x = 1 draws nothing.  Each history's outcome is computed here
    from its own stream."""
    p, table = _void_beam(5.0)
    N, seed = 400, 13
    r = oracle.run(p, N, seed, records=True, ww_center=table)
    expect = np.zeros(N)
    for i in range(N):
        s = _stream_start(seed, i)
        for _ in range(6):                       # x, y, z, t, group, mu
            s, _x = _draw(s)
        while True:                              # azimuth pair by rejection
            s, xa = _draw(s)
            s, xb = _draw(s)
            a, b = 2.0 * xa - 1.0, 2.0 * xb - 1.0
            if 0.0 < a * a + b * b < 1.0:
                break
        s, _x = _draw(s)                         # optical depth
        s, xi = _draw(s)                         # the roulette draw
        expect[i] = 5.0 if xi < 0.2 else 0.0
    assert np.array_equal(r["trk"][:, 1], expect)
    survivors = int((expect > 0).sum())
    assert int(r["tot"][7]) == N - survivors                       # rouletted
    assert int(r["tot"][4]) == survivors                           # leaked at x = 2
    assert 0.1 < survivors / N < 0.3
