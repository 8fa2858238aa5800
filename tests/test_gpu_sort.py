"""The event form's queue sort (two-kernel step; surface and collision
queues reordered by event, material, group and cell before the events
kernel) changes only the order in which particles are processed: every
history's record and every tally bin still match the oracle, in single
runs at several cadences and in batched solves."""
import numpy as np
import pytest

import workloads as w
from gpu_common import close, compare_full, gpu_run
from test_gpu_batched import small_batch


@pytest.mark.gpu
@pytest.mark.parametrize("cadence", [1, 3])
@pytest.mark.parametrize("which", ["lattice", "slab", "pins"])
def test_sorted_queues_match_oracle(which, cadence):
    if which == "lattice":
        prob, N = w.lattice(n=9, n_groups=5, gen_seed=41, n_z_bins=4, n_time_bins=6, t_end=6.0, n_batches=8), 30_000
    elif which == "slab":
        prob, N = w.cfg2_slab_pulse(), 20_000
    else:
        prob, N = w.pin_lattice(n=5, n_groups=3, gen_seed=43), 20_000
    print(f"[sort] {which} cadence={cadence}", flush=True)
    g, r, e = compare_full(prob, N, 17, "event", sort_cadence=cadence)
    # without debug arrays the census steps replay as captured graphs
    h = gpu_run(prob, N, 17, "event", debug=False, sort_cadence=cadence)
    assert np.array_equal(h["events"], r["tot"][0:3]) and np.array_equal(h["terms"], r["tot"][3:8])
    close(h["mean"], e["mean"], what="mean (graphs)")


@pytest.mark.gpu
@pytest.mark.parametrize("cadence", [-1, 1, 2])
def test_sorted_queues_batched_equal_separate_runs(cadence):
    import paper_2305_07636_amd as m

    probs, nh = small_batch(8, 5000)
    seeds = [400 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print(f"[sort] batched cadence={cadence}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean", "raw"), sort_cadence=cadence,
                                  two_kernel_step=(cadence == -1))
        for j, h in enumerate(hs):
            ref = m.mcdc_run(h, nh[j], seeds[j], algorithm="history", outputs=("mean", "raw"))
            assert np.array_equal(outs[j]["events"], ref["events"]), j
            assert np.array_equal(outs[j]["terms"], ref["terms"]), j
            close(outs[j]["raw"].cpu().numpy(), ref["raw"].cpu().numpy())
    finally:
        for h in hs:
            h.close()
