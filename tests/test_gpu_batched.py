"""Batched solve, both forms: many uneven problems in one launch (history
form) or one set of banks with graph-replayed census steps (event form)
give, per problem, exactly what separate runs give (and what the oracle
gives)."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import close


def small_batch(n=12, seed=2000):
    probs, nh = [], []
    for j in range(n):
        rng = w.SplitMix64(seed + j)
        size = rng.randint(2, 9)
        G = rng.randint(1, 4)
        probs.append(w.lattice(n=size, n_groups=G, gen_seed=seed + j + 7, n_z_bins=3, n_time_bins=5,
                               t_end=5.0, n_batches=8))
        nh.append(int(rng.randint(300, 4000)))
    nh[3] = 1
    return probs, nh


def mixed_batch():
    """Different geometries (slab and lattices), group counts and census
    grids (K = 1, 5, 12) in one batch."""
    probs, nh = small_batch(6, 4000)
    probs.append(w.slab(thickness=6.0, sigma_t=1.0, sigma_s=0.7, n_bins=12, source="plane", x_src=3.0,
                        time_edges=np.linspace(0.0, 6.0, 13), n_batches=8))
    nh.append(5003)
    probs.append(w.cfg1_slab_steady(c=0.5, mu_law="cosine"))
    nh.append(3001)
    return probs, nh


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
@pytest.mark.parametrize("which", ["lattices", "mixed"])
def test_batched_equals_separate_runs_and_oracle(alg, which):
    import paper_2305_07636_amd as m

    probs, nh = small_batch() if which == "lattices" else mixed_batch()
    seeds = [100 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print(f"[batched] {which} alg={alg}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean", "var", "raw"), algorithm=alg)
        for j, (h, p) in enumerate(zip(hs, probs)):
            print(f"[batched] problem {j} N={nh[j]}", flush=True)
            ref = m.mcdc_run(h, nh[j], seeds[j], algorithm=alg, outputs=("mean", "var", "raw"))
            assert np.array_equal(outs[j]["events"], ref["events"])
            assert np.array_equal(outs[j]["terms"], ref["terms"])
            close(outs[j]["raw"].cpu().numpy(), ref["raw"].cpu().numpy())
            close(outs[j]["mean"].cpu().numpy(), ref["mean"].cpu().numpy())
            if j % 4 == 0:
                r = oracle.run(p, nh[j], seeds[j])
                e = oracle.estimates(p, r)
                assert np.array_equal(outs[j]["events"], r["tot"][0:3])
                close(outs[j]["mean"].cpu().numpy(), e["mean"])
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
@pytest.mark.parametrize("seg_len", [256, 1024, 8192])
def test_batched_event_segment_length_does_not_change_counts(seg_len):
    import paper_2305_07636_amd as m

    probs, nh = small_batch(6, 3000)
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        a = m.mcdc_run_batched(hs, nh, list(range(6)), seg_len=seg_len)
        b = m.mcdc_run_batched(hs, nh, list(range(6)), algorithm="history")
        for x, y in zip(a, b):
            assert np.array_equal(x["events"], y["events"]) and np.array_equal(x["terms"], y["terms"])
            close(x["mean"].cpu().numpy(), y["mean"].cpu().numpy())
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
@pytest.mark.parametrize("block", [64, 256, 512])
def test_batched_launch_shape_does_not_change_counts(block):
    import paper_2305_07636_amd as m

    probs, nh = small_batch(6, 3000)
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        a = m.mcdc_run_batched(hs, nh, list(range(6)), block_size=block, algorithm="history")
        b = m.mcdc_run_batched(hs, nh, list(range(6)), block_size=128, algorithm="history")
        for x, y in zip(a, b):
            assert np.array_equal(x["events"], y["events"]) and np.array_equal(x["terms"], y["terms"])
            close(x["mean"].cpu().numpy(), y["mean"].cpu().numpy())
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
def test_batched_auto_form_choice():
    """algorithm="auto": the first call runs both tuned forms and keeps the
    faster; every call gives the separate runs' counts."""
    import paper_2305_07636_amd as m

    probs, nh = small_batch(8, 6000)
    seeds = [300 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print("[batched] auto", flush=True)
        first = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean",), algorithm="auto")
        second = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean",), algorithm="auto")
        for j, h in enumerate(hs):
            ref = m.mcdc_run(h, nh[j], seeds[j], algorithm="history", outputs=("mean",))
            for o in (first[j], second[j]):
                assert np.array_equal(o["events"], ref["events"])
                assert np.array_equal(o["terms"], ref["terms"])
                close(o["mean"].cpu().numpy(), ref["mean"].cpu().numpy())
    finally:
        for h in hs:
            h.close()
