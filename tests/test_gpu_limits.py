"""GPU parity at the library's size limits, against the oracle: 32 groups
(the largest group count), 2 047 union cells along x (the largest), 1 023
along z, 2 000 census steps, the largest batch count (1 023), bank segments
of odd sizes (the last tile of a segment part-filled), and a run split into
many bank chunks.  Tolerances are stated in gpu_common."""
import math

import numpy as np
import pytest

import workloads as w
from gpu_common import compare_full

ALGS = ["history", "event"]


def many_groups(G=32):
    rng = w.SplitMix64(401)
    st, ss = w.synthetic_xs(rng, G)
    # some up-scatter into the first groups, to use every row of the CDF
    ss[G - 1, 0] = 0.05 * st[G - 1]
    p = w.reflective_box(st, ss, [float(G - g) for g in range(G)], size=(1.0, 1.0, 1.0),
                         time_edges=[0.0, 0.5, 1.0, 2.0, math.inf])
    return p


def finest_x_slab():
    """2 047 tally bins (the union grid's limit along x)."""
    return w.slab(thickness=20.47, sigma_t=1.0, sigma_s=0.7, n_bins=2047, source="plane", x_src=10.0,
                  time_edges=np.array([0.0, 5.0, math.inf]), n_batches=16)


def finest_z_box():
    """1 023 z cells (the union grid's limit along z)."""
    p = w.pin_lattice(n=1, radius=0.3, height=10.23, n_groups=2, n_z_bins=1023, n_time_bins=1, t_end=1.0,
                      bc_z=w.VACUUM)
    p["tally"]["time_edges"] = np.array([0.0, math.inf])
    return p


def many_census_steps():
    return w.slab(thickness=10.0, sigma_t=1.0, sigma_s=0.9, n_bins=10, source="plane", x_src=5.0,
                  time_edges=np.linspace(0.0, 20.0, 2001), n_batches=8)


def max_batches():
    return w.slab(thickness=6.0, sigma_t=1.0, sigma_s=0.5, n_bins=6, source="plane", x_src=3.0,
                  time_edges=np.linspace(0.0, 4.0, 5), n_batches=1023)


CASES = {
    "groups32": (many_groups, 3001, 111, {}),
    "x_cells_2047": (finest_x_slab, 2003, 112, {}),
    "z_cells_1023": (finest_z_box, 2003, 113, {}),
    "census_2000": (many_census_steps, 1501, 114, {}),
    "batches_1023": (max_batches, 5003, 115, {}),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(CASES))
def test_limits_parity(case, alg):
    make, N, seed, kw = CASES[case]
    print(f"[limits] {case} alg={alg} N={N}", flush=True)
    compare_full(make(), N, seed, alg, **kw)


@pytest.mark.gpu
@pytest.mark.parametrize("kw", [{"segments": 13, "bank_capacity": 1000},   # capped at 2 segments of 512 slots
                                {"segments": 1},                           # one segment for the whole bank
                                {"bank_capacity": 257}])                   # 12 chunks of 257 histories (ragged tiles)
def test_event_bank_shapes(kw):
    p = w.cfg2_slab_pulse()
    print(f"[limits] event bank {kw}", flush=True)
    compare_full(p, 3001, 116, "event", **kw)


def test_union_grid_limit_rejected_on_cpu():
    """One plane too many along x is refused before any device work."""
    import ctypes as C

    from paper_2305_07636_amd import _binding as b

    p = w.slab(thickness=20.48, n_bins=2048)
    d, keep = b.make_desc(p)
    h = C.c_void_p()
    rc = b.lib().mcdc_problem_create(C.byref(d), C.byref(h))
    assert rc != 0 and "too fine" in b.lib().mcdc_last_error().decode()
