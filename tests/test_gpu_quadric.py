"""GPU parity of quadric surfaces (reading R29: one second-degree surface
per geometry cell, its negative side filled with a material of its own) in
both forms against the oracle: beams through a sphere, a double cone along
and across its axis and a tilted plane crossed both ways (with scattering
inside, so every root rule is reached from both sides), degenerate cases
(a constant quadric, a beam tangent to a sphere, a plane quadric on a
mesh plane, a sphere touching its cell's faces), sphere lattices
(pulse, implicit capture, time-crossing tally, weight windows), a lattice
of mixed quadrics (rotated ellipsoids with cross terms, cones, hyperboloids,
planes, cells without one) under a tally mesh finer than the cells, several
census steps per launch, population control, the batched solve,
k-eigenvalue cycles of a pin cell whose fuel is a cylinder written as a
quadric, and a 10 x 10 x 10 sphere lattice at 1e7 histories on a sample.
Tolerances are stated in gpu_common."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import VAR_RTOL, close, compare_full, compare_sampled, gpu_run
from ww_tables import flux_table

ALGS = ["history", "event"]


def _beam(coef, axis, sign, point):
    return lambda: w.beam_through_quadric(coef, axis=axis, sign=sign, point=point, scatter=0.6)


def _ic(p):
    p["implicit_capture"] = {"w_min": 0.25, "w_survive": 1.0}
    return p


def _tc(p):
    p["tally"]["time_crossing"] = True
    return p


CASES = {
    "beam_sphere": (_beam(w.sphere_quadric((1.0, 1.0, 1.0), 0.6), 0, 1, (0.0, 1.2, 0.9)), 4001, 91),
    "beam_cone_axis": (_beam(w.cone_quadric((1.0, 1.0, 1.0)), 2, 1, (0.8, 1.3, 0.0)), 4001, 92),
    "beam_cone_across": (_beam(w.cone_quadric((1.0, 1.0, 1.0)), 0, 1, (0.0, 1.1, 1.6)), 4001, 93),
    "beam_plane_in": (_beam(w.plane_quadric((1.0, 0.5, 0.3), 1.9), 0, 1, (0.0, 1.4, 0.7)), 3001, 94),
    "beam_plane_out": (_beam(w.plane_quadric((1.0, 0.5, 0.3), 1.9), 0, -1, (0.0, 1.4, 0.7)), 3001, 95),
    "spheres": (lambda: w.sphere_lattice(n=3, n_layers=2, n_groups=3), 4001, 96),
    "spheres_ic": (lambda: _ic(w.sphere_lattice(n=3, n_layers=2, n_groups=2, gen_seed=24)), 3001, 97),
    "spheres_tc": (lambda: _tc(w.sphere_lattice(n=2, n_layers=2, n_groups=2, gen_seed=25)), 3001, 98),
    "const_inside": (_beam(np.array([0, 0, 0, 0, 0, 0, 0, 0, 0, -1.0]), 0, 1, (0.0, 1.2, 0.9)), 3001, 106),
    "tangent": (_beam(w.sphere_quadric((1.0, 1.0, 1.0), 0.6), 0, 1, (0.0, 1.6, 1.0)), 2001, 107),
    "coincident_plane": (_beam(w.plane_quadric((1.0, 0.0, 0.0), 1.0), 0, 1, (0.0, 1.3, 0.7)), 3001, 108),
    "touching_sphere": (_beam(w.sphere_quadric((1.0, 1.0, 1.0), 1.0), 0, 1, (0.0, 1.0, 1.0)), 3001, 109),
    "mixed": (lambda: w.mixed_quadric_lattice(), 5003, 99),
    "mixed_vacuum": (lambda: w.mixed_quadric_lattice(n=4, n_layers=3, gen_seed=31, bc=w.VACUUM), 5003, 100),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(CASES))
def test_quadric_parity(case, alg):
    make, N, seed = CASES[case]
    print(f"[quadric] {case} alg={alg} N={N}", flush=True)
    compare_full(make(), N, seed, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_quadric_lattice_with_windows(alg):
    p = w.mixed_quadric_lattice(gen_seed=33)
    p["ww_mesh"] = [p["tally"]["mesh"][0], p["tally"]["mesh"][1], p["tally"]["mesh"][2]]
    table = flux_table(p, N=20000, floor=1e-3)
    print(f"[quadric] windows alg={alg}", flush=True)
    compare_full(p, 1501, 101, alg, ww={"centers": table, "max_split": 4})


@pytest.mark.gpu
@pytest.mark.parametrize("spl", [2, 5])
def test_quadric_steps_per_launch(spl):
    p = w.mixed_quadric_lattice(n=3, n_layers=2, gen_seed=35, n_time_bins=7, t_end=7.0)
    print(f"[quadric] steps_per_launch={spl}", flush=True)
    compare_full(p, 5003, 102, "event", steps_per_launch=spl)
    h = gpu_run(p, 5003, 102, "event", debug=False, steps_per_launch=spl)
    r = oracle.run(p, 5003, 102)
    assert np.array_equal(h["events"], r["tot"][0:3]) and np.array_equal(h["terms"], r["tot"][3:8])
    close(h["mean"], oracle.estimates(p, r)["mean"], what="mean (graphs)")


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["split", "comb"])
def test_quadric_population_control(method):
    p = w.sphere_lattice(n=3, n_layers=2, n_groups=2, gen_seed=26, bc=w.VACUUM)
    print(f"[quadric] population control {method}", flush=True)
    g = gpu_run(p, 4001, 103, "event", debug=False, pc_target=3000, pc_method=method)
    r = oracle.run_pc(p, 4001, 103, 3000, method=method)
    e = oracle.estimates(p, r)
    assert np.array_equal(g["events"], r["tot"][0:3]) and np.array_equal(g["terms"], r["tot"][3:8])
    assert g["splits"] == int(r["tot"][8])
    close(g["mean"], e["mean"], what="mean")
    close(g["var"], e["var"], rtol=VAR_RTOL, what="var")


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_quadric_lattices_batched(alg):
    import paper_2305_07636_amd as m

    probs = [w.sphere_lattice(n=2, n_layers=1 + j, n_groups=1 + j, gen_seed=110 + j, radius=0.3 + 0.1 * j)
             for j in range(2)] + [w.mixed_quadric_lattice(gen_seed=37)]
    nh = [1501, 777, 2003]
    seeds = [70 + j for j in range(3)]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print(f"[quadric] batched alg={alg}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean",), algorithm=alg)
        for j, p in enumerate(probs):
            r = oracle.run(p, nh[j], seeds[j])
            e = oracle.estimates(p, r)
            assert np.array_equal(outs[j]["events"], r["tot"][0:3])
            assert np.array_equal(outs[j]["terms"], r["tot"][3:8])
            close(outs[j]["mean"].cpu().numpy(), e["mean"])
    finally:
        for h in hs:
            h.close()


def _pin_cell_quadric():
    p = w.pin_cell_eigen_cylinder()
    p["pins"] = None
    c, r = 0.63, 0.54
    p["quadrics"] = {"coef": np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0, -2.0 * c, -2.0 * c, 0.0,
                                       2.0 * c * c - r * r]).reshape(1, 1, 1, 10),
                     "material": np.zeros((1, 1, 1), dtype=np.int32)}
    return p


@pytest.mark.gpu
def test_quadric_pin_cell_eigenvalue_parity():
    import paper_2305_07636_amd as m

    p = _pin_cell_quadric()
    h = m.mcdc_problem_create(p)
    try:
        print("[quadric] eigenvalue", flush=True)
        g = m.mcdc_run_eigenvalue(h, 3001, 3, 5, 104)
        g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}
    finally:
        h.close()
    r = oracle.eigen(p, 3001, 3, 5, 104)
    e = oracle.eigen_estimates(p, r)
    assert np.array_equal(g["k"], r["k"])
    assert np.array_equal(g["events"], r["tot"][0:3])
    assert np.array_equal(g["source_hist"], r["hist"])
    close(g["mean"], e["mean"], what="flux")
    close(g["var"], e["var"], rtol=VAR_RTOL, what="flux var")


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_sphere_lattice_1e7_sampled(alg):
    """10 x 10 x 10 sphere lattice (radius 0.5, pitch 1.26, 7 groups), 1e7
    histories: a sample agrees exactly with the oracle."""
    p = w.sphere_lattice(n=10, n_layers=10, n_groups=7, gen_seed=5, n_time_bins=10, t_end=10.0, n_batches=32)
    print(f"[quadric] spheres 10^3 1e7 alg={alg}", flush=True)
    compare_sampled(p, 10_000_000, 105, alg, n_sample=1000)


@pytest.mark.gpu
def test_quadric_refusals():
    import paper_2305_07636_amd as m
    from paper_2305_07636_amd._binding import MCDC_E_INVALID, MCDC_E_UNSUPPORTED

    p = w.beam_through_quadric(w.sphere_quadric((1.0, 1.0, 1.0), 0.6))
    q = dict(p)
    q["pins"] = {"radius": np.array([[[0.3]]]), "material": np.array([[[1]]], dtype=np.int32)}
    with pytest.raises(m.MCDCError) as ei:
        m.mcdc_problem_create(q)
    assert ei.value.code == MCDC_E_UNSUPPORTED
    for bad in ({"coef": np.full((1, 1, 1, 10), np.inf), "material": np.array([[[1]]], dtype=np.int32)},
                {"coef": p["quadrics"]["coef"], "material": np.array([[[2]]], dtype=np.int32)},
                {"coef": p["quadrics"]["coef"], "material": np.array([[[-2]]], dtype=np.int32)}):
        q = dict(p)
        q["quadrics"] = bad
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_problem_create(q)
        assert ei.value.code == MCDC_E_INVALID
    s = w.slab()
    s["quadrics"] = {"coef": np.zeros((1, 1, s["material"].shape[2], 10)), "material": np.zeros_like(s["material"])}
    with pytest.raises(m.MCDCError) as ei:
        m.mcdc_problem_create(s)
    assert ei.value.code == MCDC_E_INVALID
