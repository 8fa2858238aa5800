"""Pins of the oracle's cylindrical pins (quadric-surface geometry: a
cylinder parallel to z in a box cell) against closed forms:

* a beam through a purely absorbing pin in a void box: transmission
  e^{-sigma l} with the chord l = 2 sqrt(r^2 - b^2), and the track length
  in each x-bin, attenuated only along the chord;
* a cosine-law point source on the box face: the transmission is the
  angular average of e^{-sigma l(Omega)} over the 3-D chords, by quadrature;
* births inside the pin: the fraction of a uniform source that starts in
  it is pi r^2 / pitch^2;
* a pin of the surrounding material changes nothing but the event count;
* conservation: equal absorption inside and outside make the cell-averaged
  flux S / (Sigma_a V) whatever the pin does to its shape."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

Z_MAX = 4.5


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


def _beam_bins(edges, y0, sigma, r, xc=1.0, yc=1.0):
    """Track length per source particle in each x-bin of a beam along +x at
    height y0 through the pin (void outside)."""
    b = y0 - yc
    out = np.zeros(len(edges) - 1)
    if abs(b) >= r:
        return np.diff(edges)
    h = math.sqrt(r * r - b * b)
    x1, x2 = xc - h, xc + h
    T = math.exp(-sigma * (x2 - x1))
    for j, (a, c) in enumerate(zip(edges[:-1], edges[1:])):
        out[j] += max(0.0, min(c, x1) - a)                                   # before the pin
        lo, hi = max(a, x1), min(c, x2)
        if hi > lo:                                                          # inside, attenuated
            out[j] += (math.exp(-sigma * (lo - x1)) - math.exp(-sigma * (hi - x1))) / sigma
        out[j] += T * max(0.0, c - max(a, x2))                               # after the pin
    return out


@pytest.mark.parametrize("y0", [1.0, 1.4, 0.7, 0.35])
def test_beam_through_pin(y0):
    p = w.beam_through_pin(y0=y0)
    N = 40000
    res = oracle.run(p, N, 61)
    e = oracle.estimates(p, res)
    b = abs(y0 - 1.0)
    ell = 2.0 * math.sqrt(0.36 - b * b) if b < 0.6 else 0.0
    T = math.exp(-1.5 * ell)
    leak = e["leak_mean"][0, 0]
    assert abs(leak[1] - T) <= Z_MAX * math.sqrt(T * (1 - T) / N) + 1e-12
    edges = p["tally"]["mesh"][0]
    exact = _beam_bins(edges, y0, 1.5, 0.6) / (np.diff(edges) * 2.0)     # per unit x-y area
    _check(e["mean"].ravel(), e["var"].ravel(), exact, floor=1e-12)


def test_cosine_point_source_transmission_quadrature():
    y0 = 1.3
    p = w.beam_through_pin(y0=y0, mu_law="cosine")
    N = 100000
    res = oracle.run(p, N, 62)
    leak = res["L"].sum() / N
    # E[exp(-sigma l(Omega))] for mu ~ cosine law (pdf 2 mu), azimuth uniform
    nm, nphi = 1200, 1200
    mu = (np.arange(nm) + 0.5) / nm
    mu = np.sqrt(mu)                       # equal-probability points of the cosine law
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    M, PHI = np.meshgrid(mu, phi, indexing="ij")
    st = np.sqrt(1.0 - M * M)
    u, v = M, st * np.cos(PHI)
    dx, dy = 0.0 - 1.0, y0 - 1.0
    a = u * u + v * v
    bq = dx * u + dy * v
    c = dx * dx + dy * dy - 0.36
    disc = bq * bq - a * c
    hit = (bq < 0) & (disc > 0) & (a > 0)
    ell3 = np.where(hit, 2.0 * np.sqrt(np.where(hit, disc, 0.0)) / np.where(a > 0, a, 1.0), 0.0)
    T = np.exp(-1.5 * ell3).mean()
    assert abs(leak - T) <= Z_MAX * math.sqrt(T * (1 - T) / N) + 2e-5, (leak, T)


def test_births_inside_the_pin():
    """Void moderator, black pin: at t = 1e-4 only particles born outside
    the pin (and not within 1e-4 of its surface heading in) are alive."""
    p = w.pin_lattice(n=1, pitch=1.26, radius=0.54, height=1.0, n_groups=1, n_time_bins=1, t_end=1e-4,
                      bc_z=w.REFLECTIVE, n_batches=8)
    p["sigma_t"][:] = [[1e6], [0.0]]
    p["sigma_s"][:] = 0.0
    p["tally"]["time_edges"] = np.array([0.0, 1e-4, math.inf])
    N = 100000
    res = oracle.run(p, N, 63)
    alive = int(res["tot"][0])                    # census arrivals at t = 1e-4
    frac_out = 1.0 - math.pi * 0.54 ** 2 / 1.26 ** 2
    shell = 2 * math.pi * 0.54 * 1e-4 / 1.26 ** 2  # bound on the thin shell that reaches the pin
    q = alive / N
    assert abs(q - frac_out) <= Z_MAX * math.sqrt(frac_out * (1 - frac_out) / N) + shell, (q, frac_out)


def test_pin_of_the_same_material_changes_nothing():
    base = w.pin_lattice(n=2, n_groups=3, gen_seed=5, n_batches=16)
    same = w.pin_lattice(n=2, n_groups=3, gen_seed=5, n_batches=16)
    same["pins"]["material"][:] = 1                # the moderator itself
    base["pins"] = None
    N = 30000
    ea = oracle.estimates(base, oracle.run(base, N, 64))
    rb = oracle.run(same, N, 64)
    eb = oracle.estimates(same, rb)
    d = eb["mean"].ravel() - ea["mean"].ravel()
    s = np.sqrt(ea["var"].ravel() + eb["var"].ravel())
    assert (np.abs(d) <= Z_MAX * s + 1e-12).all()


def test_equal_absorption_conserves_the_cell_average():
    """One group, reflective pin cell: pin Sigma_t 2, Sigma_s 1.5; moderator
    Sigma_t 1, Sigma_s 0.5 (Sigma_a = 0.5 both): the volume-averaged flux is
    S / (Sigma_a V) = 1 / (0.5 V)."""
    p = w.pin_lattice(n=1, pitch=1.26, radius=0.5, height=1.0, n_groups=1, n_time_bins=1, t_end=1.0,
                      bc_z=w.REFLECTIVE, n_batches=16, fine=4)
    p["sigma_t"][:] = [[2.0], [1.0]]
    p["sigma_s"][:] = [[[1.5]], [[0.5]]]
    p["tally"]["time_edges"] = np.array([0.0, math.inf])
    N = 50000
    res = oracle.run(p, N, 65)
    V = 1.26 * 1.26 * 1.0
    # cell-averaged flux of each batch: its whole track length over N_b V
    B = res["B"]
    per = res["S"].reshape(B, -1).sum(axis=1) / oracle.batch_sizes(N, B) / V
    m = res["S"].sum() / (N * V)
    sig = per.std(ddof=1) / math.sqrt(B)
    assert abs(m - 1.0 / (0.5 * V)) <= Z_MAX * sig, (m, 1.0 / (0.5 * V), sig)


def test_pins_must_fit_their_cells():
    p = w.pin_lattice(n=1, radius=0.63)
    with pytest.raises(RuntimeError):
        oracle.run(p, 10, 1)
