"""Shared helpers of the GPU parity tests: run a problem through the HIP
library and through the CPU oracle on the same seeded inputs and compare.

Tolerances (written here, used by every parity test):
* per-history event counts, particle counts, termination masks and every
  event/termination total: bit-exact (integer work);
* per-history scored track and detector score, raw bin sums and bin means:
  |gpu - oracle| <= 1e-12 |oracle| + 1e-12 max|oracle| (the GPU sums the
  same IEEE terms in another order: about sqrt(n) eps relative, far below);
* batch variances: 1e-9 relative + 1e-12 of the largest variance.  The
  variance is a difference of batch means that agree to ~1e-15 relative;
  with batch means spread by ~1e-4 of the mean the difference keeps about
  1e-11 relative accuracy, and 1e-9 leaves margin for bins with few scores.
  Plus 16 eps (max |mean|)^2 absolute: the variance is formed as
  (sum of squared batch means - squared sum / B) / (B (B - 1)), whose
  cancellation leaves an error of order eps m^2 in either order of
  summation, the whole result when every batch mean is the same (a
  deterministic bin: the true variance is 0 and each side returns its
  rounding).
"""
from __future__ import annotations

import numpy as np

import oracle

RTOL = 1e-12
VAR_RTOL = 1e-9


EPS = np.finfo(np.float64).eps


def var_floor(mean):
    """Absolute tolerance of a batch variance of the given means."""
    m = np.abs(np.asarray(mean, dtype=np.float64))
    return 16.0 * EPS * (m.max() ** 2 if m.size else 0.0)


def close(gpu, ref, rtol=RTOL, what="", atol=0.0):
    gpu = np.asarray(gpu, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    scale = np.abs(ref).max() if ref.size else 0.0
    tol = rtol * np.abs(ref) + 1e-12 * scale + atol
    bad = np.abs(gpu - ref) > tol
    assert not bad.any(), (what, int(bad.sum()), np.nonzero(bad)[0][:5], gpu[bad][:5], ref[bad][:5])


def gpu_run(prob, N, seed, algorithm, debug=True, ww=None, **kw):
    import paper_2305_07636_amd as m

    p = m.mcdc_problem_create(prob)
    try:
        if ww is not None:
            m.mcdc_set_weight_windows(p, ww["centers"], ww.get("ratio", 5.0), ww.get("max_split", 16))
        out = m.mcdc_run(p, N, seed, algorithm=algorithm, debug=debug, **kw)
        host = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    finally:
        p.close()
    return host


def compare_full(prob, N, seed, algorithm, ww=None, **kw):
    """Run all N histories on both sides and compare everything."""
    g = gpu_run(prob, N, seed, algorithm, ww=ww, **kw)
    if ww is not None:
        r = oracle.run(prob, N, seed, records=True, ww_center=ww["centers"],
                       ww_ratio=ww.get("ratio", 5.0), ww_max_split=ww.get("max_split", 16))
    else:
        r = oracle.run(prob, N, seed, records=True)
    e = oracle.estimates(prob, r)
    rec = r["rec"]
    dc = g["debug_counts"].astype(np.uint32)
    mism = np.nonzero((dc != rec).any(axis=1))[0]
    assert mism.size == 0, ("per-history counts differ", mism[:10], dc[mism[:3]], rec[mism[:3]])
    close(g["debug_scores"], r["trk"], what="per-history scores")
    tot = r["tot"]
    assert np.array_equal(g["events"], tot[0:3]), (g["events"], tot[0:3])
    assert np.array_equal(g["terms"], tot[3:8]), (g["terms"], tot[3:8])
    assert g["splits"] == int(tot[8])
    assert g["fission"] == int(tot[9])
    close(g["raw"], e["raw"], what="raw")
    close(g["mean"], e["mean"], what="mean")
    close(g["var"], e["var"], rtol=VAR_RTOL, what="var", atol=var_floor(e["mean"]))
    close(g["leak_mean"], e["leak_mean"], what="leak mean")
    close(g["leak_var"], e["leak_var"], rtol=VAR_RTOL, what="leak var", atol=var_floor(e["leak_mean"]))
    if prob["tally"].get("time_crossing", False):
        close(g["tc_mean"], e["tc_mean"], what="time-crossing mean")
        close(g["tc_var"], e["tc_var"], rtol=VAR_RTOL, what="time-crossing var", atol=var_floor(e["tc_mean"]))
    else:
        assert "tc_mean" not in g
    if prob.get("qoi") is not None:
        close(g["qoi_sum"], r["q"], what="detector sums")
        close([g["qoi_mean"]], [e["qoi_mean"]], what="detector mean")
        close([g["qoi_var"]], [e["qoi_var"]], rtol=VAR_RTOL, what="detector var")
    return g, r, e


def compare_sampled(prob, N, seed, algorithm, n_sample=2000, sample_seed=0, ww=None, **kw):
    """Full-size run on the GPU; the oracle recomputes a seeded sample of
    histories one by one (skip-ahead makes each history independent) and
    their per-history records must agree exactly."""
    import torch

    import paper_2305_07636_amd as m

    rng = np.random.default_rng(sample_seed)
    ids = np.unique(np.concatenate([rng.integers(0, N, n_sample), [0, N - 1]])).astype(np.uint64)
    p = m.mcdc_problem_create(prob)
    try:
        if ww is not None:
            m.mcdc_set_weight_windows(p, ww["centers"], ww.get("ratio", 5.0), ww.get("max_split", 16))
        out = m.mcdc_run(p, N, seed, algorithm=algorithm, debug=True, **kw)
        d = out["debug_counts"]
        idx = torch.as_tensor(ids.astype(np.int64), device=d.device)
        dc = d.index_select(0, idx).cpu().numpy().astype(np.uint32)
        ds = out["debug_scores"].index_select(0, idx).cpu().numpy()
        ev_sum = d[:, :3].sum(dim=0, dtype=torch.int64).cpu().numpy()
        terms_hist = d[:, 4]
        n_term_bits = int((terms_hist != 0).sum().item())
        one_bit = int(((terms_hist & (terms_hist - 1)) == 0).sum().item())
        del d, terms_hist
        out.pop("debug_counts")
        out.pop("debug_scores")
    finally:
        p.close()
    if ww is not None:
        r = oracle.run(prob, N, seed, ids=ids, records=True, ww_center=ww["centers"],
                       ww_ratio=ww.get("ratio", 5.0), ww_max_split=ww.get("max_split", 16))
    else:
        r = oracle.run(prob, N, seed, ids=ids, records=True)
    mism = np.nonzero((dc != r["rec"]).any(axis=1))[0]
    assert mism.size == 0, ("sampled per-history counts differ", ids[mism[:10]], dc[mism[:3]], r["rec"][mism[:3]])
    close(ds, r["trk"], what="sampled per-history scores")
    # properties at any size: every history terminates (exactly once without
    # windows) and the per-history counts add up to the event totals
    if ww is None and prob.get("fission") is None:
        assert int(out["terms"].sum()) == N
        assert one_bit == N
    assert n_term_bits == N
    assert np.array_equal(ev_sum, out["events"].astype(np.int64))
    return out
