"""GPU parity of implicit capture with weight roulette in both forms
against the oracle: infinite media, the c = 0.5 slab, the census-heavy
pulsed slab (weights carried through the banks), the dog-leg duct with and
without weight windows, and the 1e8-history dog-leg on a sample.
Tolerances are stated in gpu_common."""
import numpy as np
import pytest

import workloads as w
from gpu_common import compare_full, compare_sampled
from ww_tables import flux_table

ALGS = ["history", "event"]


def _ic(p, w_min=0.25, w_survive=1.0):
    p["implicit_capture"] = {"w_min": w_min, "w_survive": w_survive}
    return p


CASES = {
    "reflective_mg": (lambda: _ic(w.reflective_box([1.0, 1.5, 2.0], [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5],
                                                                     [0.0, 0.2, 1.2]], [3.0, 2.0, 1.0],
                                                    time_edges=[0.0, 0.25, 0.5, 1.0, 2.0, 4.0])), 4099, 51),
    "slab_c05": (lambda: _ic(w.cfg1_slab_steady(c=0.5), 0.1, 0.5), 6007, 52),
    "pulse_c09": (lambda: _ic(w.cfg2_slab_pulse(c=0.9), 0.2, 0.6), 3001, 53),
    "dogleg": (lambda: _ic(w.cfg5_dogleg()), 4001, 54),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(CASES))
def test_implicit_capture_parity(case, alg):
    make, N, seed = CASES[case]
    print(f"[implicit] {case} alg={alg} N={N}", flush=True)
    g, r, _ = compare_full(make(), N, seed, alg)
    assert int(g["terms"][0]) == 0 and int(g["terms"][4]) > 0     # no absorption, roulettes


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_implicit_capture_with_windows(alg):
    p = _ic(w.cfg2_slab_pulse(), 0.05, 0.2)
    p["ww_mesh"] = [p["tally"]["mesh"][0], np.zeros(0), np.zeros(0)]
    table = flux_table(w.cfg2_slab_pulse() | {"ww_mesh": p["ww_mesh"]}, N=20000, floor=1e-3)
    print(f"[implicit] windows alg={alg}", flush=True)
    compare_full(p, 1001, 55, alg, ww={"centers": table, "max_split": 4})


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_implicit_capture_dogleg_sampled(alg):
    """1e8 dog-leg histories with implicit capture (Section 3 runs the duct
    this way): a sample agrees exactly with the oracle; every history ends
    once."""
    print(f"[implicit] dogleg 1e8 alg={alg}", flush=True)
    compare_sampled(_ic(w.cfg5_dogleg()), 100_000_000, 56, alg, n_sample=1000)
