"""GPU parity of prompt fission in both forms against the oracle: the
supercritical AZURV1-like pulse, a multigroup multiplying medium, a
lattice with one fissile material, several chunks per run, the
time-crossing tally, overflow reporting, and the benchmarked-size pulse
on a sample plus the population growth at any size.  Tolerances are
stated in gpu_common."""
import math

import numpy as np
import pytest

import workloads as w
from gpu_common import compare_full, compare_sampled

ALGS = ["history", "event"]

MG_ST = [1.0, 1.5, 2.0]
MG_SS = [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5], [0.0, 0.2, 1.2]]
MG_FIS = {"sigma_f": [[0.05, 0.1, 0.3]], "nu": [[2.6, 2.5, 2.43]], "chi": [[0.7, 0.3, 0.0]]}


def fissile_lattice():
    p = w.lattice(n=5, n_groups=3, gen_seed=21, n_time_bins=6, t_end=6.0, n_batches=8)
    M, G = p["sigma_t"].shape
    st, ss = p["sigma_t"], p["sigma_s"]
    sf = np.zeros((M, G))
    # material 0 fissile: up to 60 % of what scattering leaves of sigma_t
    sf[0] = 0.6 * (st[0] - ss[0].sum(axis=1))
    p["fission"] = {"sigma_f": sf, "nu": np.full((M, G), 2.45),
                    "chi": np.tile([0.8, 0.2, 0.0], (M, 1))}
    p["tally"]["time_crossing"] = True
    return p


CASES = {
    "azurv1": (lambda: w.azurv1_supercritical(n_batches=16), 3001, 71),
    "multigroup_box": (lambda: w.reflective_box(MG_ST, MG_SS, [3.0, 2.0, 1.0], size=(1.0, 1.0, 2.0),
                                                time_edges=[0.0, 0.5, 1.0, 2.0, 3.0], fission=MG_FIS),
                       4001, 72),
    "fissile_lattice": (fissile_lattice, 3001, 73),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(CASES))
def test_fission_parity(case, alg):
    make, N, seed = CASES[case]
    print(f"[fission] {case} alg={alg} N={N}", flush=True)
    g, r, _ = compare_full(make(), N, seed, alg)
    assert g["fission"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_fission_several_chunks(alg):
    """bank_capacity 1000: four chunks of histories, each with its own
    split-bank generations."""
    print(f"[fission] chunks alg={alg}", flush=True)
    compare_full(w.azurv1_supercritical(n_batches=8), 3500, 74, alg, bank_capacity=1000)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_fission_overflow_reported(alg):
    """nu = 60 at every collision: far more neutrons in one generation than
    the split bank holds; the run reports MCDC_E_OVERFLOW and the handle
    stays usable."""
    import paper_2305_07636_amd as m

    p = w.reflective_box([1.0], [[0.0]], [1.0], time_edges=[0.0, 1.0],
                         fission={"sigma_f": [[1.0]], "nu": [[60.0]], "chi": [[1.0]]})
    h = m.mcdc_problem_create(p)
    try:
        print(f"[fission] overflow alg={alg}", flush=True)
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_run(h, 200000, 5, algorithm=alg, outputs=("mean",))
        assert ei.value.code == -4
    finally:
        h.close()
    compare_full(w.azurv1_supercritical(n_batches=8), 1001, 75, alg)


@pytest.mark.gpu
def test_fission_descriptor_validation():
    import paper_2305_07636_amd as m

    bad = [({"sigma_f": [[0.6]], "nu": [[2.0]], "chi": [[1.0]]}, "exceeds"),
           ({"sigma_f": [[0.1]], "nu": [[65.0]], "chi": [[1.0]]}, "nu"),
           ({"sigma_f": [[0.1]], "nu": [[2.0]], "chi": [[0.9]]}, "chi")]
    for fis, needle in bad:
        p = w.reflective_box([1.0], [[0.5]], [1.0], fission=fis)
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_problem_create(p)
        assert ei.value.code == -1 and needle in str(ei.value)
    p = w.reflective_box([1.0], [[0.5]], [1.0], fission={"sigma_f": [[0.1]], "nu": [[2.0]], "chi": [[1.0]]})
    with pytest.raises(m.MCDCError) as ei:
        m.mcdc_run_batched([m.mcdc_problem_create(p)], [100], [1])
    assert ei.value.code == -5


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_fission_large_pulse_sampled_and_growth(alg):
    """1e6 histories of the supercritical pulse (about 2e8 events): a
    sample of histories agrees exactly with the oracle, and the population
    at t = 20 from the time-crossing tally is e^2 = 7.39 within 4.5 sigma."""
    import paper_2305_07636_amd as m

    p = w.azurv1_supercritical()
    N = 1_000_000
    print(f"[fission] 1e6 pulse alg={alg}", flush=True)
    compare_sampled(p, N, 76, alg, n_sample=300)
    h = m.mcdc_problem_create(p)
    try:
        out = m.mcdc_run(h, N, 77, algorithm=alg, outputs=("mean", "var"))
        tc = out["tc_mean"].cpu().numpy()[:, 0, 0, 0, :]
        tv = out["tc_var"].cpu().numpy()[:, 0, 0, 0, :]
    finally:
        h.close()
    # population at the edges (v = 1, bin width 1): sum over bins; its
    # batch variance is at most (sum of bin sigmas)^2
    pop = tc.sum(axis=1)
    sig = np.sqrt(tv).sum(axis=1)
    te = p["tally"]["time_edges"]
    exact = np.exp(0.1 * te[1:])
    assert (np.abs(pop - exact) <= 4.5 * sig).all(), (pop, exact, sig)
    assert abs(pop[-1] - math.exp(2.0)) < 0.05 * math.exp(2.0)
