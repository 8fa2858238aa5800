"""GPU parity: the HIP tracker (history- and event-based forms, through the
C ABI) against the CPU oracle on the same seeded inputs.  Tolerances are
stated in gpu_common."""
import math

import numpy as np
import pytest

import workloads as w
from gpu_common import compare_full, compare_sampled
from test_oracle_trace import tiny_lattice

ALGS = ["history", "event"]

# small cases: a few seconds of oracle time, several blocks and a ragged tail
SMALL = {
    "slab_c05_cosine": (lambda: w.cfg1_slab_steady(c=0.5, mu_law="cosine"), 20011, 1),
    "slab_c0_beam": (lambda: w.cfg1_slab_steady(c=0.0, mu_law="beam"), 20011, 11),
    "slab_c0_uniform": (lambda: w.cfg1_slab_steady(c=0.0, mu_law="uniform"), 9001, 12),
    "pulse_c09": (lambda: w.cfg2_slab_pulse(c=0.9), 12345, 2),
    "pulse_c0": (lambda: w.cfg2_slab_pulse(c=0.0), 7001, 4),
    "lattice17": (lambda: w.cfg3_lattice(), 20011, 3),
    "tiny_lattice": (tiny_lattice, 5003, 9),
    "reflective_mg": (lambda: w.reflective_box([1.0, 1.5, 2.0], [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5],
                                                                [0.0, 0.2, 1.2]], [3.0, 2.0, 1.0],
                                               time_edges=[0.0, 0.25, 0.5, 1.0, 2.0, 4.0]), 4099, 17),
    "void_box": (lambda: w.void_box(), 3001, 5),
    "slab_mg3": (lambda: w.multigroup_slab(), 6007, 18),
    "reflected_column": (lambda: w.reflected_column(), 4003, 19),
    "dogleg": (lambda: w.cfg5_dogleg(), 4001, 50),
    "census_heavy": (lambda: w.reflective_box([0.3, 0.5], [[0.1, 0.15], [0.0, 0.4]], [0.7, 1.3],
                                              time_edges=np.linspace(0.0, 9.1, 71)), 2003, 8),
    "surface_y_minus": (lambda: w.make_problem(
        [[1.0]], [[[0.6]]], [1.0], [np.array([0.0, 1.0]), np.array([0.0, 0.5, 2.0]), np.array([])],
        np.zeros((1, 2, 1)), [1, 1, 0, 0, 0, 0],
        {"kind": "surface", "axis": 1, "sign": -1, "mu_law": "cosine", "lo": [0.0, 2.0, 0.0],
         "hi": [1.0, 2.0, 0.0], "group_pmf": [1.0]},
        {"mesh": [np.array([]), np.linspace(0, 2, 9), np.array([])], "time_edges": [0.0, math.inf],
         "n_batches": 16}), 3001, 6),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(SMALL))
def test_parity_small(case, alg):
    make, N, seed = SMALL[case]
    print(f"[parity] {case} alg={alg} N={N} seed={seed}", flush=True)
    compare_full(make(), N, seed, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_parity_edge_single_history(alg):
    # one history: one batch, zero variance
    print(f"[parity] single history alg={alg}", flush=True)
    compare_full(w.cfg2_slab_pulse(), 1, 7, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_parity_edge_fewer_histories_than_batches(alg):
    print(f"[parity] N < B alg={alg}", flush=True)
    compare_full(w.cfg3_lattice(), 17, 8, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_parity_edge_born_after_cutoff(alg):
    # emission window partly beyond the last time edge: some histories end
    # at birth with zero events
    p = w.slab(thickness=4.0, sigma_t=1.0, sigma_s=0.5, n_bins=8, source="plane", x_src=2.0,
               time_edges=np.linspace(0.0, 2.0, 11), t_hi=3.0)
    print(f"[parity] born after cutoff alg={alg}", flush=True)
    g, r, _ = compare_full(p, 4001, 10, alg)
    assert int(r["tot"][5]) > 0


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_parity_full_size_pulse_sampled(alg):
    """The 1e7-history pulsed slab as benchmarked, checked on a sample."""
    print(f"[parity] pulse 1e7 sampled alg={alg}", flush=True)
    compare_sampled(w.cfg2_slab_pulse(), 10_000_000, 2, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_parity_lattice_sampled(alg):
    """The 17 x 17 lattice at its full size, 1e8 histories."""
    print(f"[parity] lattice 1e8 sampled alg={alg}", flush=True)
    compare_sampled(w.cfg3_lattice(), 100_000_000, 3, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("c", [0.5, 0.0])
def test_parity_steady_slab_full_size(alg, c):
    """The steady slab at its full size, 1e5 histories, every history
    compared (c = 0.5 and the purely absorbing variant)."""
    print(f"[parity] steady slab c={c} 1e5 alg={alg}", flush=True)
    compare_full(w.cfg1_slab_steady(c=c, mu_law="cosine"), 100_000, 1, alg)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_parity_dogleg_analog_full_size_sampled(alg):
    """The dog-leg duct analog at its full size, 1e9 histories."""
    print(f"[parity] dog-leg analog 1e9 sampled alg={alg}", flush=True)
    out = compare_sampled(w.cfg5_dogleg(), 1_000_000_000, 52, alg)
    assert out["qoi_mean"] > 0


@pytest.mark.gpu
def test_algorithms_agree_bitwise_on_counts():
    """History and event forms give the same per-history records and totals
    for the same (problem, N, seed)."""
    from gpu_common import close, gpu_run

    p = w.cfg3_lattice()
    a = gpu_run(p, 200003, 31, "history")
    b = gpu_run(p, 200003, 31, "event")
    assert np.array_equal(a["debug_counts"], b["debug_counts"])
    assert np.array_equal(a["events"], b["events"]) and np.array_equal(a["terms"], b["terms"])
    close(b["debug_scores"], a["debug_scores"])
    close(b["mean"], a["mean"])


@pytest.mark.gpu
@pytest.mark.parametrize("spl", [1, 7])
@pytest.mark.parametrize("case", ["pulse_c09", "lattice17", "census_heavy"])
def test_event_graph_replays_match_eager_and_oracle(case, spl):
    """The event form replays captured census-step graphs when no debug or
    profile output is asked for and a chunk takes more than one launch (one
    census step per launch, or seven).  Several replays, with eager runs
    and synchronisations in between, must each equal the eager result."""
    import torch

    import oracle
    import paper_2305_07636_amd as m
    from gpu_common import close

    make, N, seed = SMALL[case]
    prob = make()
    ref = oracle.run(prob, N, seed)
    e = oracle.estimates(prob, ref)
    p = m.mcdc_problem_create(prob)
    try:
        eager = m.mcdc_run(p, N, seed, algorithm="event", eager=True, steps_per_launch=spl)
        for rep in range(3):
            print(f"[graph] {case} steps/launch {spl} replay {rep}", flush=True)
            g = m.mcdc_run(p, N, seed, algorithm="event", steps_per_launch=spl)
            torch.cuda.synchronize()
            assert np.array_equal(g["events"], eager["events"]) and np.array_equal(g["terms"], eager["terms"])
            assert np.array_equal(g["events"], ref["tot"][0:3]) and np.array_equal(g["terms"], ref["tot"][3:8])
            close(g["mean"].cpu().numpy(), eager["mean"].cpu().numpy())
            close(g["mean"].cpu().numpy(), e["mean"])
            close(g["var"].cpu().numpy(), e["var"], rtol=1e-9)
            m.mcdc_run(p, 1000, seed + 1 + rep, algorithm="history")   # unrelated eager work in between
    finally:
        p.close()


@pytest.mark.gpu
@pytest.mark.parametrize("segments", [1, 7, 300])
def test_event_segment_count_does_not_change_results(segments):
    """The bank is cut into segments owned by workgroups; how many there
    are changes the schedule, never the counts or (beyond summation order)
    the tallies."""
    from gpu_common import close, gpu_run

    p = w.cfg3_lattice()
    a = gpu_run(p, 30011, 41, "event")
    import paper_2305_07636_amd as m

    print(f"[segments] {segments}", flush=True)
    h = m.mcdc_problem_create(p)
    try:
        b = m.mcdc_run(h, 30011, 41, algorithm="event", segments=segments)
    finally:
        h.close()
    assert np.array_equal(a["events"], b["events"]) and np.array_equal(a["terms"], b["terms"])
    close(b["mean"].cpu().numpy(), a["mean"])


@pytest.mark.gpu
def test_sampled_profile_mixes_graph_and_eager_steps():
    """With profile_every, sampled census steps launch eagerly between
    graph replays; results equal an uninstrumented run, only the sampled
    launches are timed and counted, and the phases 0..every-1 together
    count every launch once."""
    import paper_2305_07636_amd as m
    from gpu_common import close

    p = w.cfg2_slab_pulse()
    h = m.mcdc_problem_create(p)
    adv = m._binding.PROF_CLASSES.index("events")   # the census-step kernel
    try:
        a = m.mcdc_run(h, 200003, 21, algorithm="event")
        full = np.zeros((len(m._binding.PROF_CLASSES), 4))
        c = m.mcdc_run(h, 200003, 21, algorithm="event", profile=full, steps_per_launch=1)
        total = np.zeros_like(full)
        for phase in range(10):
            prof = np.zeros_like(full)
            b = m.mcdc_run(h, 200003, 21, algorithm="event", profile=prof, profile_classes=["events"],
                           profile_every=10, profile_phase=phase, steps_per_launch=1)
            assert prof[adv, 1] == 10 and prof[adv, 0] > 0
            assert np.array_equal(a["events"], b["events"]) and np.array_equal(a["terms"], b["terms"])
            close(b["mean"].cpu().numpy(), a["mean"].cpu().numpy())
            total += prof
    finally:
        h.close()
    assert np.array_equal(a["events"], c["events"]) and np.array_equal(a["terms"], c["terms"])
    assert full[adv, 1] == 100 and total[adv, 1] == 100
    assert total[adv, 2] == full[adv, 2] and total[adv, 3] == full[adv, 3]


TWO_KERNEL = {
    "pulse_c09": SMALL["pulse_c09"],
    "lattice17": SMALL["lattice17"],
    "dogleg": SMALL["dogleg"],
    "census_heavy": SMALL["census_heavy"],
    "pins": (lambda: w.pin_lattice(n=3, n_groups=3, gen_seed=22), 3001, 83),
}


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(TWO_KERNEL))
def test_two_kernel_step_parity(case):
    """The earlier census step (advance, then events), kept behind a flag,
    against the oracle."""
    make, N, seed = TWO_KERNEL[case]
    print(f"[parity] two-kernel step {case} N={N}", flush=True)
    compare_full(make(), N, seed, "event", two_kernel_step=True)


@pytest.mark.gpu
def test_step_forms_agree_at_full_size():
    """1e7-history pulsed slab: the one- and two-kernel census steps give the
    same event and termination totals and the same tallies to rounding."""
    import paper_2305_07636_amd as m
    from gpu_common import close

    h = m.mcdc_problem_create(w.cfg2_slab_pulse())
    try:
        print("[parity] step forms at 1e7", flush=True)
        a = m.mcdc_run(h, 10_000_000, 2, algorithm="event", outputs=("mean",))
        b = m.mcdc_run(h, 10_000_000, 2, algorithm="event", outputs=("mean",), two_kernel_step=True)
        assert np.array_equal(a["events"], b["events"]) and np.array_equal(a["terms"], b["terms"])
        close(a["mean"].cpu().numpy(), b["mean"].cpu().numpy())
    finally:
        h.close()


@pytest.mark.gpu
def test_auto_form_choice_single_problem():
    """algorithm="auto": the first call runs both forms (the result is the
    history form's) and keeps the faster; later calls with the same history
    count run that form; every result agrees with the oracle."""
    import paper_2305_07636_amd as m
    from gpu_common import close

    p = w.cfg3_lattice()
    h = m.mcdc_problem_create(p)
    try:
        print("[parity] auto form", flush=True)
        first = m.mcdc_run(h, 20011, 3, algorithm="auto", debug=True)
        second = m.mcdc_run(h, 20011, 3, algorithm="auto", debug=True)
        ev = m.mcdc_run(h, 20011, 3, algorithm="event", debug=True)
        for o in (first, second):
            assert np.array_equal(o["debug_counts"].cpu().numpy(), ev["debug_counts"].cpu().numpy())
            close(o["mean"].cpu().numpy(), ev["mean"].cpu().numpy())
    finally:
        h.close()
    import oracle
    r = oracle.run(p, 20011, 3)
    assert np.array_equal(first["events"], r["tot"][0:3])


def _slice_slab(n_bins, n_time_bins, n_batches=16):
    """Pulsed slab whose one-batch tally has n_bins x n_time_bins doubles."""
    return w.slab(thickness=40.0, sigma_t=1.0, sigma_s=0.9, speed=1.0, n_bins=n_bins, source="plane",
                  x_src=20.0, time_edges=np.linspace(0.0, 20.0, n_time_bins + 1), n_batches=n_batches)


# the history form scores an analog slab's batch in LDS when that batch's
# tally takes at most 48 KB: 64 x 96 doubles is exactly that, 65 x 96 one
# time-bin row more (scores go to HBM); one history per batch puts every
# workgroup's range across many batches
SLICE = {
    "fits": (lambda: _slice_slab(64, 96), 4001, 61),
    "over": (lambda: _slice_slab(65, 96), 4001, 62),
    "batch_per_history": (lambda: _slice_slab(50, 40, n_batches=700), 700, 63),
}


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(SLICE))
def test_history_slice_boundaries(case):
    make, N, seed = SLICE[case]
    print(f"[parity] history slice {case} N={N}", flush=True)
    compare_full(make(), N, seed, "history")
