"""GPU parity of the time-crossing tally (flux at the time edges) in both
forms: full comparison with the oracle on small cases (LDS-slice and
global-atomic paths, eager and graph-replayed census steps, weight
windows, batched solves) and, at the benchmarked 1e7-history pulsed slab,
an exact count identity.  Tolerances are stated in gpu_common."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import close, compare_full
from ww_tables import flux_table

ALGS = ["history", "event"]


def _tc(p):
    p["tally"]["time_crossing"] = True
    return p


CASES = {
    # G nts = 50: the event form scores through its LDS slice
    "pulse_c09": (lambda: _tc(w.cfg2_slab_pulse(c=0.9)), 12345, 2),
    # multigroup infinite medium with a finite last edge (arrivals there score)
    "reflective_mg": (lambda: _tc(w.reflective_box([1.0, 1.5, 2.0], [[0.3, 0.4, 0.1], [0.0, 0.6, 0.5],
                                                                      [0.0, 0.2, 1.2]], [3.0, 2.0, 1.0],
                                                     time_edges=[0.0, 0.25, 0.5, 1.0, 2.0, 4.0])), 4099, 17),
    # G nts = 750 (slice) and 5 670 (no slice: global atomics)
    "lattice5_g3": (lambda: _tc(w.lattice(n=5, n_groups=3, gen_seed=11, n_time_bins=8, t_end=8.0,
                                          n_batches=8)), 6007, 21),
    "lattice9_g7": (lambda: _tc(w.lattice(n=9, n_groups=7, gen_seed=12, n_time_bins=6, t_end=6.0,
                                          n_batches=8)), 4001, 22),
    # steady state: the only edge is infinite, the tally stays zero
    "steady_slab": (lambda: _tc(w.cfg1_slab_steady(c=0.5)), 3001, 23),
}


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", list(CASES))
def test_time_crossing_parity(case, alg):
    make, N, seed = CASES[case]
    print(f"[tc] {case} alg={alg} N={N}", flush=True)
    g, r, e = compare_full(make(), N, seed, alg)
    if case == "steady_slab":
        assert not g["tc_mean"].any()
    else:
        assert g["tc_mean"].any()


@pytest.mark.gpu
def test_time_crossing_eager_and_segments():
    p = _tc(w.cfg2_slab_pulse(c=0.9))
    for kw in ({"eager": True}, {"segments": 7}):
        print(f"[tc] pulse event {kw}", flush=True)
        compare_full(p, 5003, 5, "event", **kw)


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_time_crossing_with_weight_windows(alg):
    """Scores use the weight on arrival, before the census window check."""
    p = _tc(w.cfg2_slab_pulse())
    p["ww_mesh"] = [p["tally"]["mesh"][0], np.zeros(0), np.zeros(0)]
    table = flux_table(p, N=20000, floor=1e-3)
    print(f"[tc] pulse windows alg={alg}", flush=True)
    g, r, _ = compare_full(p, 1001, 4, alg, ww={"centers": table, "max_split": 4})
    assert g["splits"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ["event", "history"])
def test_time_crossing_batched(alg):
    import paper_2305_07636_amd as m

    probs = [_tc(w.lattice(n=3 + j, n_groups=1 + j % 3, gen_seed=300 + j, n_z_bins=3, n_time_bins=5,
                           t_end=5.0, n_batches=8)) for j in range(4)]
    probs.append(w.lattice(n=4, n_groups=2, gen_seed=310, n_z_bins=3, n_time_bins=5, t_end=5.0,
                           n_batches=8))   # one without the tally in the same batch
    nh = [2001, 1, 3003, 777, 1500]
    seeds = [40 + j for j in range(len(probs))]
    hs = [m.mcdc_problem_create(p) for p in probs]
    try:
        print(f"[tc] batched alg={alg}", flush=True)
        outs = m.mcdc_run_batched(hs, nh, seeds, outputs=("mean", "var"), algorithm=alg)
        for j, p in enumerate(probs):
            r = oracle.run(p, nh[j], seeds[j])
            e = oracle.estimates(p, r)
            assert np.array_equal(outs[j]["events"], r["tot"][0:3])
            close(outs[j]["mean"].cpu().numpy(), e["mean"], what="mean")
            if j < 4:
                close(outs[j]["tc_mean"].cpu().numpy(), e["tc_mean"], what="tc mean")
            else:
                assert "tc_mean" not in outs[j]
    finally:
        for h in hs:
            h.close()


@pytest.mark.gpu
@pytest.mark.parametrize("alg", ALGS)
def test_time_crossing_full_size_count_identity(alg):
    """1e7-history pulsed slab (one group, v = 1, analog): the crossing sums
    over all bins and edges, times N V / v, count the census events exactly
    (every census is an arrival at an edge inside the mesh)."""
    import paper_2305_07636_amd as m

    p = _tc(w.cfg2_slab_pulse(c=0.9))
    N = 10_000_000
    h = m.mcdc_problem_create(p)
    try:
        print(f"[tc] full-size pulse alg={alg}", flush=True)
        out = m.mcdc_run(h, N, 2, algorithm=alg, outputs=("mean",))
        tc = out["tc_mean"].cpu().numpy()
    finally:
        h.close()
    V = np.diff(p["tally"]["mesh"][0])
    arrivals = (tc[:, 0, 0, 0, :] * V[None, :]).sum() * N
    n_census = int(out["events"][0])
    assert abs(arrivals - n_census) <= 1e-9 * n_census, (arrivals, n_census)
    # and each edge's arrivals are the survivors to that edge: they fall
    per_edge = (tc[:, 0, 0, 0, :] * V[None, :]).sum(axis=1) * N
    assert (np.diff(per_edge) <= 0).all()
