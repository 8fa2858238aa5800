"""Batched solves at the sizes of the 256-problem workload, against the
oracle: lattices whose per-step tally slice is too large for the event
form's LDS pre-reduction (their scores go straight to HBM atomics) in one
launch with small ones that take the LDS slice, in both forms.

* a batch of three 7-group lattices of 24, 28 and 32 cells a side at 1e5
  histories each plus three small ones: every history's record and every
  tally bin against the oracle;
* the full 256-lattice workload (4..32 cells a side, 1..7 groups, 1e4..1e6
  histories each, 5.9e7 in all): a seeded sample of histories of every
  problem against the oracle record by record, full tallies of the problems
  with at most 3e4 histories (among them 27- and 31-cell 7-group
  lattices), and for every problem the properties that hold at any size
  (each history ends exactly once, per-history counts add up to the event
  totals, per-history scored tracks add up to the tally)."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import RTOL, VAR_RTOL, close

OUTS = ("mean", "var", "raw")


def _slice_fits(prob):
    G = prob["sigma_t"].shape[1]
    nts = 1
    for m in prob["tally"]["mesh"]:
        nts *= max(1, m.size - 1)
    return 2 * G * nts <= 4096


def _large_batch():
    probs = [w.lattice(n=24, n_groups=7, gen_seed=501), w.lattice(n=28, n_groups=7, gen_seed=502),
             w.lattice(n=32, n_groups=7, gen_seed=503),
             w.lattice(n=4, n_groups=2, gen_seed=504), w.lattice(n=6, n_groups=3, gen_seed=505),
             w.lattice(n=8, n_groups=1, gen_seed=506)]
    nh = [100_000, 100_000, 100_000, 3_001, 20_000, 50_000]
    return probs, nh


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
def test_large_lattices_batched_every_history_and_bin(alg):
    import paper_2305_07636_amd as m

    probs, nh = _large_batch()
    assert [_slice_fits(p) for p in probs] == [False, False, False, True, True, True]
    seeds = [700 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print(f"[batched-large] alg={alg}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=OUTS, algorithm=alg, debug=True)
        for j, p in enumerate(probs):
            print(f"[batched-large] problem {j} N={nh[j]}", flush=True)
            o = outs[j]
            r = oracle.run(p, nh[j], seeds[j], records=True)
            e = oracle.estimates(p, r)
            dc = o["debug_counts"].cpu().numpy().astype(np.uint32)
            mism = np.nonzero((dc != r["rec"]).any(axis=1))[0]
            assert mism.size == 0, (j, mism[:10], dc[mism[:3]], r["rec"][mism[:3]])
            close(o["debug_scores"].cpu().numpy(), r["trk"], what=f"problem {j} per-history scores")
            assert np.array_equal(o["events"], r["tot"][0:3]), (j, o["events"], r["tot"][0:3])
            assert np.array_equal(o["terms"], r["tot"][3:8]), (j, o["terms"], r["tot"][3:8])
            close(o["raw"].cpu().numpy(), e["raw"], what=f"problem {j} raw")
            close(o["mean"].cpu().numpy(), e["mean"], what=f"problem {j} mean")
            close(o["var"].cpu().numpy(), e["var"], rtol=VAR_RTOL, what=f"problem {j} var")
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
def test_full_256_problem_batch_against_oracle(alg):
    import torch

    import paper_2305_07636_amd as m

    probs, nh = w.cfg4_batch()
    seeds = [2000 + j for j in range(len(probs))]
    fits = [_slice_fits(p) for p in probs]
    assert any(fits) and not all(fits)            # both tally paths in one launch
    hs = [m.mcdc_problem_create(p) for p in probs]
    rng = np.random.default_rng(4)
    n_full = 0
    try:
        print(f"[batched-256] alg={alg} histories={sum(nh)}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=OUTS, algorithm=alg, debug=True)
        for j, p in enumerate(probs):
            o, N = outs[j], nh[j]
            d = o["debug_counts"]
            # any size: each history ends exactly once, counts add up
            term = d[:, 4]
            assert int((term != 0).sum().item()) == N, j
            assert int(((term & (term - 1)) == 0).sum().item()) == N, j
            ev = d[:, :3].sum(dim=0, dtype=torch.int64).cpu().numpy()
            assert np.array_equal(ev, o["events"].astype(np.int64)), (j, ev, o["events"])
            assert int(o["terms"].sum()) == N
            trk = float(o["debug_scores"][:, 0].sum().item())
            raw = float(o["raw"].sum().item())
            assert abs(trk - raw) <= 1e-11 * abs(raw), (j, trk, raw)
            # sampled histories against the oracle, record by record
            ids = np.unique(np.concatenate([rng.integers(0, N, 8), [0, N - 1]])).astype(np.uint64)
            idx = torch.as_tensor(ids.astype(np.int64), device=d.device)
            dc = d.index_select(0, idx).cpu().numpy().astype(np.uint32)
            ds = o["debug_scores"].index_select(0, idx).cpu().numpy()
            r = oracle.run(p, N, seeds[j], ids=ids, records=True)
            mism = np.nonzero((dc != r["rec"]).any(axis=1))[0]
            assert mism.size == 0, (j, ids[mism[:5]], dc[mism[:3]], r["rec"][mism[:3]])
            close(ds, r["trk"], what=f"problem {j} sampled scores")
            # the smaller problems in full
            if N <= 30_000:
                n_full += 1
                r = oracle.run(p, N, seeds[j])
                e = oracle.estimates(p, r)
                assert np.array_equal(o["events"], r["tot"][0:3]), j
                close(o["raw"].cpu().numpy(), e["raw"], rtol=RTOL, what=f"problem {j} raw")
                close(o["mean"].cpu().numpy(), e["mean"], what=f"problem {j} mean")
                close(o["var"].cpu().numpy(), e["var"], rtol=VAR_RTOL, what=f"problem {j} var")
        print(f"[batched-256] {n_full} problems compared in full", flush=True)
        assert n_full >= 30
    finally:
        for h in hs:
            h.close()
