"""Several census steps per launch of the event form's one-kernel step: a
particle that reaches the edge T_{k+1} inside the launch goes on into
time bin k+1 in registers, and each workgroup's LDS slice holds the scores
of all the launch's time bins.  The census edges are the paper's (Section
2), so every history's record and every tally bin must still match the
oracle: slab, lattice, moving plane, time-crossing tally, pins, a slice
too large for LDS (scores go to HBM atomics), launches that overrun the
last time bin, eager and graph-replayed launches, sampled profiling; the
forms it does not apply to are refused."""
import numpy as np
import pytest

import workloads as w
from gpu_common import close, compare_full, gpu_run


def _tc(p):
    p["tally"]["time_crossing"] = True
    return p


CASES = {
    # G nts = 50, 100 time bins
    "slab": (lambda: w.cfg2_slab_pulse(), 20_000),
    "slab_tc": (lambda: _tc(w.cfg2_slab_pulse(c=0.9)), 20_000),
    # 5 groups, 9 x 9 x 4 bins, 6 time bins: one step's slice is 3240
    # doubles, so only one step fits (the launch keeps one step)
    "lattice": (lambda: w.lattice(n=9, n_groups=5, gen_seed=41, n_z_bins=4, n_time_bins=6, t_end=6.0,
                                  n_batches=8), 30_000),
    # 2 groups, 4 x 4 x 2 bins, 11 time bins: several steps per slice
    "lattice_small": (lambda: w.lattice(n=4, n_groups=2, gen_seed=44, n_z_bins=2, n_time_bins=11, t_end=11.0,
                                        n_batches=8), 30_000),
    # 7 groups, 24 x 24 bins: no LDS slice at all
    "lattice_hbm": (lambda: w.lattice(n=24, n_groups=7, gen_seed=501, n_time_bins=5, t_end=5.0, n_batches=4),
                    20_000),
    "rod": (lambda: w.rod_beam_box(), 30_000),
    "pins": (lambda: w.pin_lattice(n=5, n_groups=3, gen_seed=43), 20_000),
}


@pytest.mark.gpu
@pytest.mark.parametrize("spl", [2, 3, 7, 64])
@pytest.mark.parametrize("which", list(CASES))
def test_steps_per_launch_matches_oracle(which, spl):
    make, N = CASES[which]
    prob = make()
    print(f"[multistep] {which} steps_per_launch={spl}", flush=True)
    g, r, e = compare_full(prob, N, 31, "event", steps_per_launch=spl)
    # without debug arrays the launches replay as captured graphs
    h = gpu_run(prob, N, 31, "event", debug=False, steps_per_launch=spl)
    assert np.array_equal(h["events"], r["tot"][0:3]) and np.array_equal(h["terms"], r["tot"][3:8])
    close(h["mean"], e["mean"], what="mean (graphs)")
    close(h["raw"], e["raw"], what="raw (graphs)")


@pytest.mark.gpu
def test_steps_per_launch_full_size_slab_totals_and_profile():
    """The benchmarked 1e7-history pulsed slab: the same event and
    termination totals as one step per launch, tallies equal up to
    summation order, and a sampled profile counts launches."""
    import paper_2305_07636_amd as m

    prob = w.cfg2_slab_pulse()
    p = m.mcdc_problem_create(prob)
    try:
        ref = m.mcdc_run(p, 10_000_000, 5, outputs=("raw",), steps_per_launch=1)
        for spl in (0, 1, 4, 10):
            print(f"[multistep] slab 1e7 steps_per_launch={spl}", flush=True)
            o = m.mcdc_run(p, 10_000_000, 5, outputs=("raw",), steps_per_launch=spl)
            assert np.array_equal(o["events"], ref["events"]) and np.array_equal(o["terms"], ref["terms"])
            close(o["raw"].cpu().numpy(), ref["raw"].cpu().numpy(), what=f"raw s={spl}")
        # 100 time bins in launches of 4 steps: 25 launches, 5 per phase
        ev = m._binding.PROF_CLASSES.index("events")
        full = np.zeros((len(m._binding.PROF_CLASSES), 4))
        m.mcdc_run(p, 1_000_000, 5, outputs=("raw",), steps_per_launch=4, profile=full)
        assert int(full[ev, 1]) == 25
        total = np.zeros_like(full)
        for phase in range(5):
            prof = np.zeros_like(full)
            m.mcdc_run(p, 1_000_000, 5, outputs=("raw",), steps_per_launch=4, profile=prof,
                       profile_classes=["events"], profile_every=5, profile_phase=phase)
            assert int(prof[ev, 1]) == 5 and prof[ev, 0] > 0
            total += prof
        assert total[ev, 2] == full[ev, 2] and total[ev, 3] == full[ev, 3]
    finally:
        p.close()


@pytest.mark.gpu
def test_steps_per_launch_refused_where_it_does_not_apply():
    import paper_2305_07636_amd as m
    from paper_2305_07636_amd._binding import MCDC_E_UNSUPPORTED

    prob = w.cfg2_slab_pulse()
    p = m.mcdc_problem_create(prob)
    try:
        for kw in (dict(two_kernel_step=True), dict(sort_cadence=2), dict(staged=True), dict(pc_target=10_000)):
            with pytest.raises(m.MCDCError) as ei:
                m.mcdc_run(p, 10_000, 3, steps_per_launch=2, **kw)
            assert ei.value.code == MCDC_E_UNSUPPORTED, kw
        # one step per launch is always accepted
        o = m.mcdc_run(p, 10_000, 3, steps_per_launch=1, two_kernel_step=True)
        assert int(o["terms"].sum()) == 10_000
    finally:
        p.close()
