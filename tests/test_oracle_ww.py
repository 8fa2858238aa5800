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
