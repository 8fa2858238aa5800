"""Learned weight-window generator.

A small network maps a weight-window cell's features (scaled position,
one-hot group, scaled time) to log10 of the adjoint (importance) flux of
the problem's detector; the window centre of a cell is a reference
importance divided by the cell's importance, so particles are split as they
move toward the detector and rouletted where they matter less (see
centres_from_log_importance for the reference).  The network is trained with the
library's own FP32 matrix-core kernels on the flux tally of the adjoint
problem computed by plain (analog) batches of the same tracker, and run in
BF16; it fills in and smooths cells the pilot tally saw poorly.  Windows
only change the variance: the tracker's game is unbiased, and analog runs
stay the judge of the figure of merit.

Adjoint problem (steady state, isotropic scattering): the same geometry,
total cross sections and boundaries, the transposed group-transfer matrix,
and the detector box as a uniform volume source whose group spectrum is the
detector's group response.  Its scalar flux is the importance of the
forward problem's detector response.

All arithmetic on the transport side runs in the HIP library; this module
only builds inputs and tables from its outputs (NumPy on a few thousand
numbers).
"""
from __future__ import annotations

import copy
import math
import time

import numpy as np

from . import _binding as B


def adjoint_problem(prob: dict) -> dict:
    q = prob.get("qoi")
    if q is None or prob.get("ww_mesh") is None:
        raise ValueError("the problem needs a detector (qoi) and a weight-window mesh")
    te = prob["tally"]["time_edges"]
    if te.size != 2 or not math.isinf(te[1]):
        raise ValueError("learned windows are built for steady-state problems (one time bin [t0, inf))")
    st = prob["sigma_t"]
    ssT = np.ascontiguousarray(np.transpose(prob["sigma_s"], (0, 2, 1)))
    if (ssT.sum(axis=2) > st * (1 + 1e-12)).any():
        raise ValueError("the transposed transfer matrix exceeds sigma_t: the adjoint needs weights")
    mask = np.asarray(q["group_mask"], dtype=np.float64)
    adj = copy.deepcopy(prob)
    adj["sigma_s"] = ssT
    adj["source"] = {"kind": "isotropic", "lo": np.array(q["lo"], dtype=np.float64),
                     "hi": np.array(q["hi"], dtype=np.float64), "group_pmf": mask / mask.sum(),
                     "t_lo": float(te[0]), "t_hi": float(te[0])}
    adj["tally"] = {"mesh": [np.asarray(m, dtype=np.float64) for m in prob["ww_mesh"]],
                    "time_edges": np.array(te, dtype=np.float64),
                    "n_batches": prob["tally"]["n_batches"]}
    adj["qoi"] = None
    return adj


def cell_features(prob: dict) -> np.ndarray:
    """Features of every window cell in table order [K][G][wz][wy][wx]:
    (x, y, z) centre scaled to [0, 1] over the mesh, one-hot group, scaled
    time-bin centre, zero-padded to 8.  Returns float32 [n, 8]."""
    mesh = prob["ww_mesh"]
    G = prob["sigma_t"].shape[1]
    if 3 + G + 1 > 8:
        raise ValueError("at most 4 groups fit the 8 network inputs")
    te = prob["tally"]["time_edges"]
    K = te.size - 1
    cen = []
    for a in range(3):
        m = mesh[a]
        if m.size:
            c = 0.5 * (m[:-1] + m[1:])
            cen.append((c - m[0]) / (m[-1] - m[0]))
        else:
            cen.append(np.array([0.5]))
    tt = np.zeros(K)
    if K > 1 or math.isfinite(te[-1]):
        fin = te[np.isfinite(te)]
        tt = 0.5 * (te[:-1] + np.minimum(te[1:], fin[-1])) / max(fin[-1], 1e-300)
    nz, ny, nx = cen[2].size, cen[1].size, cen[0].size
    X = np.zeros((K, G, nz, ny, nx, 8), dtype=np.float32)
    X[..., 0] = cen[0][None, None, None, None, :]
    X[..., 1] = cen[1][None, None, None, :, None]
    X[..., 2] = cen[2][None, None, :, None, None]
    for g in range(G):
        X[:, g, ..., 3 + g] = 1.0
    X[..., 3 + G] = tt[:, None, None, None, None]
    return X.reshape(-1, 8)


def source_cells(prob: dict) -> np.ndarray:
    """Boolean [wz, wy, wx] mask of window cells overlapping the source box."""
    mesh = prob["ww_mesh"]
    src = prob["source"]
    sel = []
    for a in range(3):
        m = mesh[a]
        if not m.size:
            sel.append(np.array([True]))
            continue
        lo, hi = src["lo"][a], src["hi"][a]
        s = (m[1:] > lo) & (m[:-1] < hi)
        if lo == hi:
            s = (m[:-1] <= lo) & (m[1:] >= lo)
        sel.append(s)
    return sel[2][:, None, None] & sel[1][None, :, None] & sel[0][None, None, :]


def centres_from_log_importance(logI: np.ndarray, log_ref: float, shape, below: float = 0.0) -> np.ndarray:
    """w_c(cell) = I_ref / I(cell) on cells at most `below` decades less
    important than the reference level (there w_c > 1: particles entering
    are rouletted), 0 (no window: analog tracking) elsewhere.

    The reference is the importance at the frontier of the region the
    adjoint pilot resolved: particles coming from the source travel analog
    (weight 1) until they reach that frontier, where the window centre is 1,
    and are split as they move on toward the detector.  Source-normalised
    windows would need the importance at the source, which an analog
    adjoint pilot of a deep-penetration problem does not reach."""
    logI = np.asarray(logI, dtype=np.float64).reshape(shape)
    w = np.where(logI >= log_ref - below, 10.0 ** np.minimum(log_ref - logI, below), 0.0)
    return np.ascontiguousarray(w)


def _tally(prob: dict, n: int, seed: int, table=None, ratio: float = 5.0, max_split: int = 16):
    """Steady flux tally (mean, relative error) of a run of the tracker."""
    p = B.mcdc_problem_create(prob)
    try:
        if table is not None:
            B.mcdc_set_weight_windows(p, table, ratio, max_split)
        out = B.mcdc_run(p, n, seed, algorithm="history", outputs=("mean", "var"))
        phi = out["mean"].double().cpu().numpy().ravel()
        var = out["var"].double().cpu().numpy().ravel()
    finally:
        p.close()
    rel = np.sqrt(var) / np.where(phi > 0, phi, 1.0)
    return phi, rel


def _frontier_table(logI, ok, shape, pct):
    log_ref = float(np.percentile(logI[ok], pct))
    return centres_from_log_importance(np.where(ok, logI, -np.inf), log_ref, shape)


def learned_windows(prob: dict, n_pilot: int = 100_000_000, seed: int = 1000, steps: int = 3000,
                    lr: float = 1e-3, net_seed: int = 1, rel_max: float = 0.3, frontier_pct: float = 5.0,
                    below: float = 0.0, extrapolate: float = 1.0, normalise: str = "auto",
                    support: str = "resolved"):
    """Plain pilots -> training set -> network -> window table.

    1. forward analog pilot: the flux phi, which is the importance of the
       adjoint problem's response (the forward source region);
    2. adjoint pilot, with windows from phi (frontier-normalised, analog
       where phi is unresolved) so adjoint particles reach back to the
       source: the adjoint flux phi+, the importance of the detector;
    3. the network fits log10 phi+ on the cells the pilot resolved
       (weights 1 / (R^2 + 0.01)); BF16 inference gives a smooth log10 I;
       windows w_c = I(source) / I(cell), normalised over the source cells
       when the pilot resolved them, else at the resolved frontier.

    support: "resolved" (default) puts windows on the cells the adjoint
    pilot resolved, with the network's smoothed importance in place of the
    noisy tally, and leaves the other cells analog (no window); "all" puts
    the network's prediction on every cell.  Measured on the dog-leg duct
    (three pilot seeds, 1e8-history pilots, 1e9 windowed histories),
    "resolved" gave 8-10x the analog figure of merit against 6-9x for the
    raw tally windows, while "all" split particles deep into the thick
    walls, where the fit extrapolates, and gave 4.5-5x.

    extrapolate: decades the network's prediction may leave the range of
    the pilot's values (cells the pilot did not resolve).  normalise:
    "auto" (source if the pilot resolved the source cells, else frontier),
    "source" (the network's importance at the source cells, resolved or
    not) or "frontier".

    The pilots run with seeds `seed` (forward) and `seed + 1` (adjoint),
    returned as info["pilot_seeds"]: a run judged with these windows should
    take other seeds, so that the table does not depend on the very
    histories it is judged on.

    Returns (table [K][G][wz][wy][wx], info dict with the raw-tally table,
    the pilot seeds and timings)."""
    import torch

    adj = adjoint_problem(prob)
    shape = (1, prob["sigma_t"].shape[1]) + source_cells(prob).shape
    t0 = time.perf_counter()
    phi_f, rel_f = _tally(prob, n_pilot, seed)
    ok_f = (phi_f > 0) & (rel_f < rel_max)
    adj_table = _frontier_table(np.log10(np.where(ok_f, phi_f, 1.0)), ok_f, shape, frontier_pct)
    phi, rel = _tally(adj, n_pilot, seed + 1, table=adj_table)
    t_pilot = time.perf_counter() - t0
    X = cell_features(prob)
    ok = (phi > 0) & (rel < rel_max)
    T = np.log10(phi[ok]).astype(np.float32)
    W = (1.0 / (rel[ok] ** 2 + 0.01)).astype(np.float32)
    W /= W.sum()
    t1 = time.perf_counter()
    dev = torch.device("cuda", torch.cuda.current_device())
    Xd = torch.as_tensor(X, device=dev).contiguous()
    net = B.MLP(net_seed)
    try:
        losses = net.train(torch.as_tensor(X[ok], device=dev).contiguous(),
                           torch.as_tensor(T, device=dev), torch.as_tensor(W, device=dev), steps, lr)
        yhat = net.infer(Xd).double().cpu().numpy()
    finally:
        net.close()
    t_train = time.perf_counter() - t1
    # keep the prediction within the range the pilot saw (no runaway
    # extrapolation into cells the network never observed)
    yhat = np.clip(yhat, T.min() - extrapolate, T.max() + extrapolate)
    src = source_cells(prob)
    pmf = np.asarray(prob["source"]["group_pmf"], dtype=np.float64)
    ok5 = ok.reshape(shape)
    src_resolved = all(ok5[0, g][src].any() for g in range(shape[1]) if pmf[g] > 0)
    y5 = yhat.reshape(shape)
    use_source = normalise == "source" or (normalise == "auto" and src_resolved)
    if use_source:
        # importance of the source: spectrum-weighted mean over source cells
        I_src = sum(pmf[g] * np.mean(10.0 ** y5[0, g][src]) for g in range(shape[1]) if pmf[g] > 0)
        log_ref = float(np.log10(I_src))
    else:
        log_ref = float(np.percentile(T, frontier_pct))
    if support not in ("resolved", "all"):
        raise ValueError("support must be 'resolved' or 'all'")
    fit = np.where(ok, yhat, -np.inf) if support == "resolved" else yhat
    table = centres_from_log_importance(fit, log_ref, shape, below if use_source else 0.0)
    raw = centres_from_log_importance(np.where(ok, np.log10(np.where(ok, phi, 1.0)), -np.inf), log_ref, shape,
                                      below if use_source else 0.0)
    info = {"pilot_s": t_pilot, "train_s": t_train, "n_train": int(ok.sum()), "loss_first": float(losses[0]),
            "loss_last": float(losses[-1]), "raw_table": raw, "adjoint_flux": phi,
            "source_resolved": bool(src_resolved), "log_ref": log_ref, "pilot_seeds": (seed, seed + 1),
            "log_importance": yhat, "adjoint_rel": rel, "resolved": ok}
    return table, info


def figure_of_merit(prob: dict, n: int, seed: int, table=None, ratio: float = 5.0, max_split: int = 16,
                    algorithm: str = "history"):
    """Run n histories (analog if table is None) and return the detector
    mean, its relative error R, the tracking time T (device ms of the run)
    and FOM = 1 / (R^2 T)."""
    p = B.mcdc_problem_create(prob)
    try:
        if table is not None:
            B.mcdc_set_weight_windows(p, table, ratio, max_split)
        out = B.mcdc_run(p, n, seed, algorithm=algorithm, outputs=())
    finally:
        p.close()
    mean, var = out["qoi_mean"], out["qoi_var"]
    R = math.sqrt(var) / mean if mean > 0 else math.inf
    T = out["kernel_ms"] * 1e-3
    return {"mean": mean, "sigma": math.sqrt(var), "R": R, "T_s": T,
            "fom": 1.0 / (R * R * T) if mean > 0 else 0.0, "splits": out["splits"],
            "events": [int(x) for x in out["events"]]}
