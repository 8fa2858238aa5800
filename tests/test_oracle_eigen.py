"""Pins of the oracle's k-eigenvalue power iteration (Section 3 runs its
pin-cell and core problems as k-eigenvalue cycles) against closed forms of
the infinite medium and a deterministic transport solution of a bare slab.

Infinite homogeneous medium: every cycle-source neutron is born with the
spectrum chi, so the expected number of sites per neutron is
k = (nu Sigma_f)^T M^-1 chi with M = diag(Sigma_t) - Sigma_s^T, and the
flux per source neutron is M^-1 chi / V.  Bare slab: the discrete-ordinates
power iteration of refs.sn_slab_k (2 000 cells, S64; refinement moves k by
3e-6)."""
import math

import numpy as np
import pytest

import oracle
import workloads as w
from refs import removal_matrix, sn_slab_k

Z_MAX = 4.5

MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5], [0.0, 0.2, 1.2]]
MG_SF = [0.05, 0.1, 0.3]
MG_NU = [2.6, 2.5, 2.43]
MG_CHI = [0.7, 0.3, 0.0]


def _check(mean, var, exact, z=Z_MAX, floor=1e-12):
    mean, var, exact = map(lambda a: np.asarray(a, dtype=float).ravel(), (mean, var, exact))
    sig = np.sqrt(var)
    bad = np.abs(mean - exact) > z * sig + floor
    assert not bad.any(), (np.nonzero(bad), mean[bad], exact[bad], sig[bad])


def test_infinite_medium_one_group_k_and_flux():
    """k_inf = nu Sigma_f / Sigma_a = 2.5 x 0.2 / 0.5 = 1, phi = 1 / (Sigma_a V)."""
    p = w.reflective_box([1.0], [[0.5]], [1.0], fission={"sigma_f": [[0.2]], "nu": [[2.5]], "chi": [[1.0]]})
    r = oracle.eigen(p, 20000, 3, 30, 81)
    e = oracle.eigen_estimates(p, r)
    _check([e["k_mean"]], [e["k_std"] ** 2], [1.0])
    _check(e["mean"].ravel(), e["var"].ravel(), [1.0 / (0.5 * 8.0)])
    # 20 000 neutrons per cycle: every cycle's flux is within a few per cent,
    # so the standard error of the mean is well under 1 %
    assert (np.sqrt(e["var"]) < 0.01 * e["mean"]).all()
    assert r["k"].size == 33 and int(r["tot"][9]) == 0


def test_infinite_medium_multigroup_k_and_flux():
    fis = {"sigma_f": [MG_SF], "nu": [MG_NU], "chi": [MG_CHI]}
    p = w.reflective_box(MG_ST, MG_SS, [3.0, 2.0, 1.0], size=(1.0, 1.0, 2.0), fission=fis)
    r = oracle.eigen(p, 20000, 3, 30, 82)
    e = oracle.eigen_estimates(p, r)
    Minv_chi = np.linalg.solve(removal_matrix(MG_ST, MG_SS), MG_CHI)
    k_exact = float(np.dot(np.array(MG_NU) * MG_SF, Minv_chi))
    _check([e["k_mean"]], [e["k_std"] ** 2], [k_exact])
    _check(e["mean"].ravel(), e["var"].ravel(), Minv_chi / 2.0)
    assert (np.sqrt(e["var"]) < 0.01 * e["mean"]).all()
    # cycle 0 starts in group 0 (the problem's source), the others from chi
    Minv_e0 = np.linalg.solve(removal_matrix(MG_ST, MG_SS), [1.0, 0.0, 0.0])
    k0 = float(np.dot(np.array(MG_NU) * MG_SF, Minv_e0))
    sig_cycle = e["k_std"] * np.sqrt(r["n_active"])
    assert abs(r["k"][0] - k0) < Z_MAX * sig_cycle


def test_bare_slab_k_and_mode_shape_against_sn():
    p = w.bare_slab_eigen()
    r = oracle.eigen(p, 20000, 10, 40, 83)
    e = oracle.eigen_estimates(p, r)
    k_sn, xe, phi = sn_slab_k(6.0, 1.0, 0.6, 0.5, n_cells=2400)
    _check([e["k_mean"]], [e["k_std"] ** 2], [k_sn], floor=2e-5)
    # flux per cycle-source neutron in the 24 tally bins (0.25 mfp each)
    edges = p["tally"]["mesh"][0]
    fine = phi.reshape(24, -1).mean(axis=1)
    assert np.allclose(edges, xe[::xe.size // 24][:25])
    _check(e["mean"].ravel(), e["var"].ravel(), fine, floor=1e-4 * fine.max())
    # leakage through each face: half of what the source does not absorb
    lm = e["leak_mean"][0, 0]
    assert abs(lm[0] - lm[1]) < Z_MAX * np.sqrt(e["leak_var"][0, 0, 0] + e["leak_var"][0, 0, 1])


def test_eigen_rejects_non_steady_or_non_fissile():
    with pytest.raises(RuntimeError):
        oracle.eigen(w.cfg2_slab_pulse(), 100, 1, 2, 1)
    with pytest.raises(RuntimeError):
        oracle.eigen(w.cfg1_slab_steady(), 100, 1, 2, 1)


def test_source_entropy():
    """Sites per spatial bin: they add up to k N in every cycle; one bin
    gives entropy 0 exactly; a uniform infinite medium on a 2 x 2 x 2 mesh
    gives log2(8) = 3 bits up to the small-sample bias (8 - 1) / (2 M ln 2);
    in the bare slab the first cycle (a point source at the centre) is less
    spread than the converged source."""
    p = w.reflective_box([1.0], [[0.5]], [1.0], fission={"sigma_f": [[0.2]], "nu": [[2.5]], "chi": [[1.0]]})
    r = oracle.eigen(p, 20000, 2, 3, 84)
    assert np.array_equal(r["hist"].sum(axis=1), np.round(r["k"] * 20000).astype(np.uint64))
    assert (oracle.source_entropy(r["hist"]) == 0.0).all()          # the box has one tally bin
    for a in range(3):
        p["tally"]["mesh"][a] = np.array([0.0, 1.0, 2.0])
    r = oracle.eigen(p, 20000, 2, 3, 85)
    H = oracle.source_entropy(r["hist"])
    M = r["hist"].sum(axis=1)
    bias = 7.0 / (2.0 * M * math.log(2.0))
    assert (np.abs(H - (3.0 - bias)) < 5e-3).all(), H
    p = w.bare_slab_eigen()
    r = oracle.eigen(p, 20000, 10, 5, 86)
    H = oracle.source_entropy(r["hist"])
    assert H[0] < H[-1] - 0.5, H
