"""GPU parity of cylindrical pins (quadric surfaces) in both forms against
the oracle: a beam through an absorbing pin, pin lattices (pulse, implicit
capture, weight windows, time-crossing), the batched solve, k-eigenvalue
cycles of a cylindrical pin cell, and a 17 x 17 pin lattice at 1e7
histories on a sample.  Tolerances are stated in gpu_common."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import VAR_RTOL, close, compare_full, compare_sampled
from ww_tables import flux_table

ALGS = ["history", "event"]


def lattice_ic():
    p = w.pin_lattice(n=3, n_groups=3, gen_seed=23)
    p["implicit_capture"] = {"w_min": 0.25, "w_survive": 1.0}
    return p


def lattice_tc():
    p = w.pin_lattice(n=4, n_groups=2, gen_seed=24, fine=2)
    p["tally"]["time_crossing"] = True
    return p


CASES = {
    "beam_center": (lambda: w.beam_through_pin(y0=1.0), 4001, 81),
    "beam_cosine": (lambda: w.beam_through_pin(y0=1.3, mu_law="cosine"), 6007, 82),
    "lattice3": (lambda: w.pin_lattice(n=3, n_groups=3, gen_seed=22), 4001, 83),
    "lattice_ic": (lattice_ic, 3001, 84),
    "lattice_tc": (lattice_tc, 3001, 85),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(CASES))
def test_pin_parity(case, alg):
    make, N, seed = CASES[case]
    print(f"[pins] {case} alg={alg} N={N}", flush=True)
    compare_full(make(), N, seed, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_pin_lattice_with_windows(alg):
    p = w.pin_lattice(n=3, n_groups=2, gen_seed=25)
    p["ww_mesh"] = [p["tally"]["mesh"][0], p["tally"]["mesh"][1], p["tally"]["mesh"][2]]
    table = flux_table(p, N=20000, floor=1e-3)
    print(f"[pins] windows alg={alg}", flush=True)
    compare_full(p, 1501, 86, alg, ww={"centers": table, "max_split": 4})


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
def test_pin_lattices_batched(alg):
    import paper_2305_07636_amd as m

    probs = [w.pin_lattice(n=2 + j, n_groups=1 + j % 3, gen_seed=90 + j, radius=0.3 + 0.1 * j) for j in range(3)]
    nh = [1501, 777, 2003]
    seeds = [60 + j for j in range(3)]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print(f"[pins] batched alg={alg}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean",), algorithm=alg)
        for j, p in enumerate(probs):
            r = oracle.run(p, nh[j], seeds[j])
            e = oracle.estimates(p, r)
            assert np.array_equal(outs[j]["events"], r["tot"][0:3])
            close(outs[j]["mean"].cpu().numpy(), e["mean"])
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
def test_pin_cell_eigenvalue_parity():
    import paper_2305_07636_amd as m

    p = w.pin_cell_eigen_cylinder()
    h = m.mcdc_problem_create(p)
    try:
        print("[pins] eigenvalue", flush=True)
        g = m.mcdc_run_eigenvalue(h, 3001, 3, 5, 87)
        g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}
    finally:
        h.close()
    r = oracle.eigen(p, 3001, 3, 5, 87)
    e = oracle.eigen_estimates(p, r)
    assert np.array_equal(g["k"], r["k"])
    assert np.array_equal(g["events"], r["tot"][0:3])
    assert np.array_equal(g["source_hist"], r["hist"])
    close(g["mean"], e["mean"], what="flux")
    close(g["var"], e["var"], rtol=VAR_RTOL, what="flux var")


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_pin_lattice_17x17_sampled(alg):
    """17 x 17 pin lattice (radius 0.54, pitch 1.26, 7 groups), 1e7
    histories: a sample agrees exactly with the oracle."""
    p = w.pin_lattice(n=17, n_groups=7, gen_seed=3, height=50.0, n_z_bins=10, n_time_bins=20, t_end=20.0,
                      n_batches=32)
    print(f"[pins] 17x17 1e7 alg={alg}", flush=True)
    compare_sampled(p, 10_000_000, 88, alg, n_sample=1000)
