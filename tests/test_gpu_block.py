"""The event form's census-step kernels at workgroup sizes 256, 512 and
1024 (1024 is the default of analog runs, 512 of weighted ones): every
history's record and every bin against the oracle, in the one-kernel step
and the two-kernel step with the queue sort; the batched solve with each
size forced equals separate runs."""
import numpy as np
import pytest

import workloads as w
from gpu_common import close, compare_full, gpu_run
from test_gpu_batched import small_batch


def _prob(which):
    if which == "slab":
        return w.cfg2_slab_pulse(), 20_000
    if which == "lattice":
        return w.lattice(n=7, n_groups=4, gen_seed=51, n_z_bins=4, n_time_bins=6, t_end=6.0, n_batches=8), 30_000
    return w.rod_lattice(n=6, n_groups=3, gen_seed=52, rods_every=2, z_top=50.0, z_bottom=5.0, n_z_bins=5,
                         n_time_bins=8, t_end=8.0, t_insert=5.0, n_batches=8), 20_000


@pytest.mark.gpu
@pytest.mark.parametrize("block", [256, 512])
@pytest.mark.parametrize("which", ["slab", "lattice", "rod"])
def test_block_sizes_match_oracle(which, block):
    prob, N = _prob(which)
    print(f"[block] {which} {block}", flush=True)
    g, r, e = compare_full(prob, N, 31, "event", block_size=block)
    compare_full(prob, N, 31, "event", block_size=block, sort_cadence=2)
    h = gpu_run(prob, N, 31, "event", debug=False, block_size=block)      # graph replays
    assert np.array_equal(h["events"], r["tot"][0:3]) and np.array_equal(h["terms"], r["tot"][3:8])
    close(h["mean"], e["mean"], what="mean (graphs)")


@pytest.mark.gpu
@pytest.mark.parametrize("block", [256, 1024])
def test_block_sizes_batched(block):
    import paper_2305_07636_amd as m

    probs, nh = small_batch(6, 7000)
    seeds = [500 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        for cad in (-1, 1):
            outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("raw",), block_size=block, sort_cadence=cad)
            for j, h in enumerate(hs):
                ref = m.mcdc_run(h, nh[j], seeds[j], algorithm="history", outputs=("raw",))
                assert np.array_equal(outs[j]["events"], ref["events"]), (cad, j)
                assert np.array_equal(outs[j]["terms"], ref["terms"]), (cad, j)
                close(outs[j]["raw"].cpu().numpy(), ref["raw"].cpu().numpy())
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
def test_block_size_refused_where_unsupported():
    import paper_2305_07636_amd as m
    from paper_2305_07636_amd._binding import MCDCError

    p = m.mcdc_problem_create(w.cfg2_slab_pulse())
    try:
        with pytest.raises(MCDCError):
            m.mcdc_run(p, 100, 1, algorithm="event", block_size=384)
        with pytest.raises(MCDCError):
            m.mcdc_run(p, 100, 1, algorithm="event", block_size=256, pc_target=100)
    finally:
        p.close()


@pytest.mark.gpu
@pytest.mark.parametrize("block", [256, 512, 1024])
def test_slab_step_with_and_without_staging(block):
    """The slab's one-kernel step reads its refills straight from HBM
    (default) or from tiles each wave copies into LDS (staged): both give
    the oracle's per-history records and bins."""
    for prob, N in ((w.cfg2_slab_pulse(), 20_000), (w.cfg1_slab_steady(), 20_000)):
        compare_full(prob, N, 33, "event", block_size=block)
        compare_full(prob, N, 33, "event", block_size=block, staged=True)
        g = gpu_run(prob, N, 33, "event", debug=False, block_size=block)
        h = gpu_run(prob, N, 33, "event", debug=False, block_size=block, staged=True)
        assert np.array_equal(g["events"], h["events"]) and np.array_equal(g["terms"], h["terms"])
        close(g["mean"], h["mean"], what="staged vs unstaged")
