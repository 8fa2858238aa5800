"""GPU parity of the weight-window game (split progeny in generations,
roulette) against the oracle, and the no-window limit."""
import numpy as np
import pytest

import oracle
import workloads as w
from gpu_common import compare_full, compare_sampled
from ww_tables import flux_table

WW_ALGS = ["history", "event"]


@pytest.mark.gpu
@pytest.mark.parametrize("alg", WW_ALGS)
def test_ww_zero_table_matches_analog_oracle(alg):
    p = w.cfg5_dogleg(detector=w.LEG_A_DETECTOR)
    zero = np.zeros((1, 2, 10, 10, 40))
    print(f"[ww] zero table alg={alg}", flush=True)
    g, r, _ = compare_full(p, 3001, 5, alg, ww={"centers": zero})
    assert g["splits"] == 0


@pytest.mark.gpu
@pytest.mark.parametrize("alg", WW_ALGS)
def test_ww_parity_dogleg(alg):
    p = w.cfg5_dogleg(detector=w.LEG_A_DETECTOR)
    table = flux_table(p, floor=1e-3)
    print(f"[ww] dog-leg alg={alg}", flush=True)
    g, r, _ = compare_full(p, 2001, 8, alg, ww={"centers": table})
    assert g["splits"] > 0 and int(g["terms"][4]) > 0


@pytest.mark.gpu
@pytest.mark.parametrize("alg", WW_ALGS)
def test_ww_parity_pulse_census_checks(alg):
    p = w.cfg2_slab_pulse()
    p["ww_mesh"] = [p["tally"]["mesh"][0], np.zeros(0), np.zeros(0)]
    table = flux_table(p, N=20000, floor=1e-3)
    print(f"[ww] pulse alg={alg}", flush=True)
    g, r, _ = compare_full(p, 1001, 4, alg, ww={"centers": table, "max_split": 4})
    assert g["splits"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("alg", WW_ALGS)
def test_ww_overflow_reported(alg):
    """A tiny split limit per particle cannot overflow; an impossible table
    (every cell asks for heavy splitting) runs to completion or reports
    MCDC_E_OVERFLOW, never corrupts memory."""
    import paper_2305_07636_amd as m

    p = w.cfg5_dogleg(detector=w.LEG_A_DETECTOR)
    table = np.full((1, 2, 10, 10, 40), 1e-3)
    h = m.mcdc_problem_create(p)
    try:
        m.mcdc_set_weight_windows(h, table, 5.0, 2)
        print(f"[ww] heavy splitting alg={alg}", flush=True)
        out = m.mcdc_run(h, 2000, 3, algorithm=alg)
        assert out["splits"] > 0
    except m.MCDCError as e:
        assert e.code == -4
    finally:
        h.close()


@pytest.mark.gpu
def test_ww_forms_agree_at_full_size():
    """Windowed runs of the two forms, 1e7 histories of the dog-leg duct
    in five chunks of 2^21 histories (the windows split about 64 times per
    history, more than the default chunk of 2^23 holds): the same counts,
    splits and detector sums."""
    import paper_2305_07636_amd as m
    from gpu_common import close

    p = w.cfg5_dogleg(detector=w.LEG_A_DETECTOR)
    table = flux_table(p, floor=1e-3)
    h = m.mcdc_problem_create(p)
    try:
        m.mcdc_set_weight_windows(h, table, 5.0, 16)
        a = m.mcdc_run(h, 10_000_000, 12, algorithm="history", bank_capacity=1 << 21)
        b = m.mcdc_run(h, 10_000_000, 12, algorithm="event", bank_capacity=1 << 21)
    finally:
        h.close()
    assert np.array_equal(a["events"], b["events"]) and np.array_equal(a["terms"], b["terms"])
    assert a["splits"] == b["splits"] > 0
    close(np.array(b["qoi_sum"]), np.array(a["qoi_sum"]))
    close(b["mean"].cpu().numpy(), a["mean"].cpu().numpy())


@pytest.mark.gpu
@pytest.mark.parametrize("alg", WW_ALGS)
def test_ww_dogleg_sampled_2e7(alg):
    """Windowed dog-leg at 2e7 histories (several chunks of the event form's
    bank), checked on a sample of histories (split progeny included)
    against the oracle."""
    from paper_2305_07636_amd import learned_ww as lw

    p = w.cfg5_dogleg(detector=w.LEG_A_DETECTOR)
    # importance windows from an oracle run of the adjoint problem (forward
    # flux windows multiply the population a thousandfold here)
    adj = lw.adjoint_problem(p)
    e = oracle.estimates(adj, oracle.run(adj, 20000, 77))
    phi = e["mean"].ravel()
    ok = phi > 0
    logI = np.where(ok, np.log10(np.where(ok, phi, 1.0)), -np.inf)
    table = lw.centres_from_log_importance(logI, float(np.percentile(logI[ok], 70.0)), (1, 2, 10, 10, 40))
    print(f"[ww] dog-leg 2e7 sampled alg={alg}", flush=True)
    out = compare_sampled(p, 20_000_000, 51, alg, n_sample=1000, ww={"centers": table})
    assert out["splits"] > 0
