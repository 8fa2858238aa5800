"""mcdc_run_noalloc (the history form with its per-run buffers in a static
device array, for callers that cannot allocate) against mcdc_run's history
form on the same problem, histories and seed, through the C ABI.

Bar: event and termination totals bit-exact; tallies, leakage and detector
sums to the parity tolerance of tests/gpu_common.py (the two sum the same
terms in another order); variances to its variance tolerance.  Two calls in
a row on one GPU, the second with fewer histories and a smaller tally (the
array keeps the first call's contents, which the second must clear), then
the first problem again; and a small case against the oracle itself."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import VAR_RTOL, close

OUTS = ("mean", "var", "raw", "leak_mean", "leak_var")


def _both(p, N, seed):
    import paper_2305_07636_amd as m

    a = m.mcdc_run(p, N, seed, algorithm="history", outputs=OUTS)
    b = m.mcdc_run(p, N, seed, algorithm="history", outputs=OUTS, noalloc=True)
    return a, b


def _same(a, b, what):
    assert np.array_equal(a["events"], b["events"]), (what, a["events"], b["events"])
    assert np.array_equal(a["terms"], b["terms"]), (what, a["terms"], b["terms"])
    for k in ("raw", "mean", "leak_mean"):
        close(b[k].cpu().numpy(), a[k].cpu().numpy(), what=f"{what} {k}")
    for k in ("var", "leak_var"):
        close(b[k].cpu().numpy(), a[k].cpu().numpy(), rtol=VAR_RTOL, what=f"{what} {k}")
    close([b["qoi_sum"][0], b["qoi_sum"][1]], [a["qoi_sum"][0], a["qoi_sum"][1]], what=f"{what} detector")


@pytest.mark.gpu
def test_noalloc_matches_mcdc_run_two_calls():
    import paper_2305_07636_amd as m

    big = w.cfg3_lattice()                       # 404 600-bin tally, 32 batches
    small = w.cfg2_slab_pulse()                  # 5 000-bin tally
    pb, ps = m.mcdc_problem_create(big), m.mcdc_problem_create(small)
    try:
        print("[noalloc] lattice 1e6 histories", flush=True)
        a, b = _both(pb, 1_000_000, 3)
        _same(a, b, "lattice")
        print("[noalloc] slab 2e5 histories after the lattice", flush=True)
        a, b = _both(ps, 200_000, 4)
        _same(a, b, "slab")
        print("[noalloc] lattice 1e5 histories again", flush=True)
        a, b = _both(pb, 100_000, 5)
        _same(a, b, "lattice again")
    finally:
        pb.close()
        ps.close()


@pytest.mark.gpu
def test_noalloc_matches_oracle_small():
    import paper_2305_07636_amd as m

    prob = w.cfg1_slab_steady()
    N, seed = 20_000, 1
    r = oracle.run(prob, N, seed)
    e = oracle.estimates(prob, r)
    p = m.mcdc_problem_create(prob)
    try:
        g = m.mcdc_run(p, N, seed, algorithm="history", outputs=OUTS, noalloc=True)
    finally:
        p.close()
    assert np.array_equal(g["events"], r["tot"][0:3])
    assert np.array_equal(g["terms"], r["tot"][3:8])
    close(g["raw"].cpu().numpy(), e["raw"], what="raw")
    close(g["mean"].cpu().numpy(), e["mean"], what="mean")
    close(g["var"].cpu().numpy(), e["var"], rtol=VAR_RTOL, what="var")
    close(g["leak_mean"].cpu().numpy(), e["leak_mean"], what="leak mean")


@pytest.mark.gpu
def test_noalloc_refuses_what_it_does_not_run():
    import paper_2305_07636_amd as m
    from paper_2305_07636_amd._binding import MCDCError

    p = m.mcdc_problem_create(w.cfg2_slab_pulse())
    try:
        with pytest.raises(MCDCError) as ei:
            m.mcdc_run(p, 1000, 1, algorithm="event", noalloc=True)
        assert ei.value.code == -5 and "history form" in str(ei.value)
        with pytest.raises(MCDCError) as ei:
            m.mcdc_run(p, 1000, 1, algorithm="history", noalloc=True, debug=True)
        assert ei.value.code == -5
    finally:
        p.close()
    # a tally beyond the array: 64 x 64 x 100 cells x 7 groups x 20 time
    # bins x 32 batches x 8 bytes is about 1.5e10 bytes
    big = w.cfg3_lattice()
    big["tally"]["mesh"] = [np.linspace(0.0, 21.42, 65), np.linspace(0.0, 21.42, 65), np.linspace(0.0, 50.0, 101)]
    p = m.mcdc_problem_create(big)
    try:
        with pytest.raises(MCDCError) as ei:
            m.mcdc_run(p, 1000, 1, algorithm="history", noalloc=True)
        assert ei.value.code == -5 and "scratch" in str(ei.value)
    finally:
        p.close()
