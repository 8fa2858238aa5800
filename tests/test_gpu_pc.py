"""GPU parity of population control at census (splitting-roulette to a
target population, exact fixed-point total weight) against the oracle's
census-synchronous run: every event, termination and split count agrees
exactly and the tallies within the stated tolerances (gpu_common).  Cases:
the decaying pulsed slab (analog and implicit capture), a void reflective
box whose population doubles exactly, the same box with births spread over
its time bins (later births wait for their own edge), a steady-state
problem with no inner edge, a target of one particle, a multigroup reflective box with the
time-crossing tally, a ragged history count with a target above and below
it, both step forms; then the 1e7-history pulsed slab at full size against
the closed form of its spatially integrated flux."""
import math

import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import RTOL, VAR_RTOL, close, gpu_run


def _slab_pulse(c=0.5, K=20, batches=16):
    return w.slab(thickness=40.0, sigma_t=1.0, sigma_s=c, speed=1.0, n_bins=40, source="plane",
                  x_src=20.0, time_edges=np.linspace(0.0, 20.0, K + 1), n_batches=batches)


def _void_reflective():
    return w.void_box(size=(2.0, 1.5, 1.0), n_mesh=(2, 3, 1), src_point=(0.3, 0.7, 0.4),
                      time_edges=list(np.linspace(0.0, 4.0, 5)), bc=[w.REFLECTIVE] * 6)


def _void_spread():
    p = _void_reflective()
    p["source"]["t_lo"], p["source"]["t_hi"] = 0.0, 4.0
    return p


def _mg_box():
    p = w.reflective_box([1.0, 1.5, 2.0], [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5], [0.0, 0.2, 1.2]], [3.0, 2.0, 1.0],
                         time_edges=[0.0, 0.25, 0.5, 1.0, 2.0, 4.0])
    p["tally"]["time_crossing"] = True
    return p


def _ic(p, w_min, w_survive):
    p["implicit_capture"] = {"w_min": w_min, "w_survive": w_survive}
    return p


CASES = {
    "slab_c05": (lambda: _slab_pulse(0.5), 20000, 1.0, 61),
    "slab_c09_implicit": (lambda: _ic(_slab_pulse(0.9), 0.2, 0.6), 6007, 1.0, 62),
    "void_double": (_void_reflective, 3000, 2.0, 63),
    "mg_box_tc": (_mg_box, 4099, 1.0, 64),
    "void_spread_births": (_void_spread, 4000, 1.0, 68),
    "ragged_up": (lambda: _slab_pulse(0.7, K=13, batches=7), 12345, 1.5, 65),
    "ragged_down": (lambda: _slab_pulse(0.7, K=13, batches=7), 12345, 0.4, 66),
    "steady_no_edge": (lambda: w.cfg1_slab_steady(c=0.5), 3000, 1.0 / 3.0, 69),
    "target_one": (_void_reflective, 2000, 1.0 / 2000, 70),
}


def compare_pc(prob, N, target, seed, method="split", **kw):
    g = gpu_run(prob, N, seed, "event", debug=False, pc_target=target, pc_method=method, **kw)
    r = oracle.run_pc(prob, N, seed, target, method=method)
    e = oracle.estimates(prob, r)
    tot = r["tot"]
    assert np.array_equal(g["events"], tot[0:3]), (g["events"], tot[0:3])
    assert np.array_equal(g["terms"], tot[3:8]), (g["terms"], tot[3:8])
    assert g["splits"] == int(tot[8]), (g["splits"], int(tot[8]))
    close(g["raw"], e["raw"], what="raw")
    close(g["mean"], e["mean"], what="mean")
    close(g["var"], e["var"], rtol=VAR_RTOL, what="var")
    close(g["leak_mean"], e["leak_mean"], what="leak mean")
    close(g["leak_var"], e["leak_var"], rtol=VAR_RTOL, what="leak var")
    if prob["tally"].get("time_crossing", False):
        close(g["tc_mean"], e["tc_mean"], what="time-crossing mean")
        close(g["tc_var"], e["tc_var"], rtol=VAR_RTOL, what="time-crossing var")
    return g, r


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(CASES))
def test_population_control_parity(case):
    make, N, f, seed = CASES[case]
    target = int(round(f * N))
    print(f"[pc] {case} N={N} target={target}", flush=True)
    g, r = compare_pc(make(), N, target, seed)
    born = int(r["pop"][0])
    # balance: born + copies = every way a particle ends
    assert born + g["splits"] == int(np.sum(g["terms"]))
    if case == "void_double":
        assert g["splits"] == N and int(g["terms"][4]) == 0


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(CASES))
def test_population_control_by_combing_parity(case):
    """Combing (reading R28): the controlled particles in the run's list
    order (the banks keep it), their teeth counted from an exact 128-bit
    prefix of their fixed-point weights; every count and tally against the
    oracle's comb."""
    make, N, f, seed = CASES[case]
    target = int(round(f * N))
    print(f"[pc comb] {case} N={N} target={target}", flush=True)
    g, r = compare_pc(make(), N, target, seed, method="comb")
    born = int(r["pop"][0])
    assert born + g["splits"] == int(np.sum(g["terms"]))


@pytest.mark.gpu
def test_combing_many_copies_per_history():
    """200 histories combed to 12 000 particles at the first edge (some 60
    copies of each, written together in their parent's place), and 300
    multigroup histories to 9000: list order through every later edge."""
    print("[pc comb] 60 copies per history", flush=True)
    compare_pc(_void_reflective(), 200, 12000, 75, method="comb")
    compare_pc(_mg_box(), 300, 9000, 76, method="comb")


@pytest.mark.gpu
def test_combing_graphs_eager_and_profiled_runs_agree():
    """Combed runs replay their census steps as captured graphs; eager and
    profiled launches (every control kernel timed) give the same counts,
    and the oracle's tallies."""
    import paper_2305_07636_amd as m

    prob = _slab_pulse(0.5)
    print("[pc comb] graphs, eager, profiled", flush=True)
    g, r = compare_pc(prob, 20000, 15000, 74, method="comb")
    p = m.mcdc_problem_create(prob)
    try:
        e = m.mcdc_run(p, 20000, 74, pc_target=15000, pc_method="comb", eager=True)
        prof = np.zeros((len(m._binding.PROF_CLASSES), 4))
        f = m.mcdc_run(p, 20000, 74, pc_target=15000, pc_method="comb", profile=prof)
        # a second graph run of the same handle replays the cached graphs
        h = m.mcdc_run(p, 20000, 74, pc_target=15000, pc_method="comb")
        for o in (e, f, h):
            assert np.array_equal(o["events"], g["events"]) and np.array_equal(o["terms"], g["terms"])
            assert o["splits"] == g["splits"]
            close(o["mean"].cpu().numpy(), g["mean"], what="mean")
        ct = m._binding.PROF_CLASSES.index("control")
        assert prof[ct, 1] == 4 * 20 and prof[ct, 3] > 0   # sum, teeth, count, apply after each of 20 steps
    finally:
        p.close()


@pytest.mark.gpu
def test_combing_full_size_pulse():
    """1e7 histories of the 40-mfp pulsed slab (c = 0.9, 100 census steps)
    combed to 1e7 at every edge: the spatially integrated flux of every
    time bin matches the closed form v exp(-v Sigma_a t) averaged over the
    bin, every particle ends once, and the last bin's error is below that
    of splitting-roulette to the same population."""
    import paper_2305_07636_amd as m

    N = 10_000_000
    prob = w.cfg2_slab_pulse(c=0.9)
    print(f"[pc comb] full-size pulse N={N}", flush=True)
    p = m.mcdc_problem_create(prob)
    try:
        g = m.mcdc_run(p, N, 72, pc_target=N, pc_method="comb")
        mean = g["mean"].cpu().numpy().reshape(100, -1)
        var = g["var"].cpu().numpy().reshape(100, -1)
    finally:
        p.close()
    dx = 40.0 / 50
    integ = mean.sum(axis=1) * dx
    ivar = var.sum(axis=1) * dx * dx
    te = np.linspace(0.0, 20.0, 101)
    sa = 0.1
    exact = (np.exp(-sa * te[:-1]) - np.exp(-sa * te[1:])) / (sa * np.diff(te))
    z = (integ - exact) / np.sqrt(ivar)
    assert np.all(np.abs(z) < 5.0), z[np.abs(z) >= 5.0]
    assert N + g["splits"] == int(np.sum(g["terms"]))
    assert int(g["terms"][3]) == 0


@pytest.mark.gpu
def test_population_control_two_kernel_step():
    print("[pc] two-kernel step", flush=True)
    compare_pc(_slab_pulse(0.5), 20000, 20000, 67, two_kernel_step=True)


@pytest.mark.gpu
def test_population_control_rejections():
    import paper_2305_07636_amd as m
    from paper_2305_07636_amd._binding import MCDC_E_UNSUPPORTED

    print("[pc] rejections", flush=True)
    p = m.mcdc_problem_create(_slab_pulse(0.5))
    try:
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_run(p, 1000, 1, algorithm="history", pc_target=1000)
        assert ei.value.code == MCDC_E_UNSUPPORTED
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_run(p, (1 << 26) + 1, 1, pc_target=1000)
        assert ei.value.code == MCDC_E_UNSUPPORTED
        # combing needs a target
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_run(p, 1000, 1, pc_method="comb")
        assert ei.value.code == m._binding.MCDC_E_INVALID
        # combing runs the one-kernel step only
        for kw in (dict(two_kernel_step=True), dict(sort_cadence=2)):
            with pytest.raises(m.MCDCError) as ei:
                m.mcdc_run(p, 1000, 1, pc_target=1000, pc_method="comb", **kw)
            assert ei.value.code == MCDC_E_UNSUPPORTED, kw
        # auto picks the event form
        g = m.mcdc_run(p, 2000, 1, algorithm="auto", pc_target=2000)
        assert g["splits"] > 0
        # per-history debug counts follow each history's copies
        g = m.mcdc_run(p, 2000, 1, pc_target=2000, debug=True)
        dc = g["debug_counts"].cpu().numpy().astype(np.int64)
        assert np.array_equal(dc[:, :3].sum(axis=0), np.asarray(g["events"], dtype=np.int64))
        assert int(dc[:, 3].sum()) == 2000 + g["splits"]
    finally:
        p.close()
    q = m.mcdc_problem_create(w.azurv1_supercritical())
    try:
        with pytest.raises(m.MCDCError) as ei:
            m.mcdc_run(q, 1000, 1, pc_target=1000)
        assert ei.value.code == MCDC_E_UNSUPPORTED
    finally:
        q.close()


@pytest.mark.gpu
def test_population_control_full_size_pulse():
    """1e7 histories of the 40-mfp pulsed slab (c = 0.9, 100 census steps)
    with the population held at 1e7: the spatially integrated flux of every
    time bin matches the closed form v exp(-v Sigma_a t) averaged over the
    bin (exact while the boundaries are out of reach), every particle ends
    once, and the late-time error is below the analog run's."""
    import paper_2305_07636_amd as m

    N = 10_000_000
    prob = w.cfg2_slab_pulse(c=0.9)
    print(f"[pc] full-size pulse N={N}", flush=True)
    p = m.mcdc_problem_create(prob)
    try:
        g = m.mcdc_run(p, N, 71, pc_target=N)
        a = m.mcdc_run(p, N, 71)
        mean = g["mean"].cpu().numpy().reshape(100, -1)
        var = g["var"].cpu().numpy().reshape(100, -1)
        am = a["mean"].cpu().numpy().reshape(100, -1)
        av = a["var"].cpu().numpy().reshape(100, -1)
    finally:
        p.close()
    dx = 40.0 / 50
    integ = mean.sum(axis=1) * dx
    ivar = var.sum(axis=1) * dx * dx
    te = np.linspace(0.0, 20.0, 101)
    sa = 0.1
    exact = (np.exp(-sa * te[:-1]) - np.exp(-sa * te[1:])) / (sa * np.diff(te))
    z = (integ - exact) / np.sqrt(ivar)
    assert np.all(np.abs(z) < 5.0), z[np.abs(z) >= 5.0]
    born = N
    assert born + g["splits"] == int(np.sum(g["terms"]))
    assert int(g["terms"][3]) == 0   # nothing lost
    # late-time relative error of the integrated flux below the analog's
    rel_pc = math.sqrt(ivar[-1]) / integ[-1]
    rel_an = math.sqrt(av[-1].sum() * dx * dx) / (am[-1].sum() * dx)
    assert rel_pc < rel_an, (rel_pc, rel_an)
