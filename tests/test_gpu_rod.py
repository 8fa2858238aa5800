"""The moving plane (control-rod tip whose height is linear in time within
each census step) on the GPU against the oracle: every history's record
and every tally bin in both forms on the descending-rod beam box and on a
small rodded lattice; sampled histories of the 17 x 17 rodded lattice at
1e7 histories; and a batched solve with rodded problems."""
import numpy as np
import pytest

import workloads as w
from gpu_common import close, compare_full, compare_sampled


def _small_rod_lattice():
    return w.rod_lattice(n=6, n_groups=3, gen_seed=21, rods_every=2, z_top=50.0, z_bottom=5.0, n_z_bins=5,
                         n_time_bins=8, t_end=8.0, t_insert=5.0, n_batches=8)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
@pytest.mark.parametrize("which", ["beam", "beam_void", "lattice"])
def test_moving_plane_matches_oracle(which, alg):
    if which == "beam":
        prob, N = w.rod_beam_box(), 40_000
    elif which == "beam_void":
        prob, N = w.rod_beam_box(void_rod=True), 20_000
    else:
        prob, N = _small_rod_lattice(), 40_000
    print(f"[rod] {which} {alg}", flush=True)
    compare_full(prob, N, 23, alg)


@pytest.mark.gpu
def test_moving_plane_sorted_queues_match_oracle():
    compare_full(_small_rod_lattice(), 30_000, 24, "event", sort_cadence=2)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
def test_rodded_lattice_full_size_sampled(alg):
    print(f"[rod] 17x17 rodded lattice 1e7 {alg}", flush=True)
    compare_sampled(w.rod_lattice(), 10_000_000, 25, alg, n_sample=1500, sample_seed=3)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
def test_rodded_problems_batched(alg):
    import paper_2305_07636_amd as m

    probs = [_small_rod_lattice(), w.rod_beam_box(), w.lattice(n=5, n_groups=2, gen_seed=31, n_z_bins=3,
                                                             n_time_bins=4, t_end=4.0, n_batches=8)]
    nh = [20_000, 10_000, 5_000]
    seeds = [60, 61, 62]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean", "raw"), algorithm=alg)
        for j, h in enumerate(hs):
            ref = m.mcdc_run(h, nh[j], seeds[j], algorithm="history", outputs=("mean", "raw"))
            assert np.array_equal(outs[j]["events"], ref["events"]), j
            assert np.array_equal(outs[j]["terms"], ref["terms"]), j
            close(outs[j]["raw"].cpu().numpy(), ref["raw"].cpu().numpy())
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
def test_moving_plane_refused_where_unsupported():
    import paper_2305_07636_amd as m
    from paper_2305_07636_amd._binding import MCDCError

    p = w.pin_lattice(n=2)
    p["rod"] = {"z": np.zeros(p["tally"]["time_edges"].size), "material": np.zeros((1, 2, 2), dtype=np.int32)}
    with pytest.raises(MCDCError) as ei:
        m.mcdc_problem_create(p)
    assert ei.value.code == -5
