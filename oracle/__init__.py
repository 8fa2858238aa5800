"""CPU oracle for the multigroup time-dependent Monte Carlo tracker.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library; the two share only
the seeded problem generators in ``workloads`` (problem descriptions, no
transport arithmetic).

The transport itself runs in the plain serial C file ``mcdc_oracle.c``
(built here with gcc, no contraction).  This module marshals a problem dict
into that file's own struct and applies the batch statistics (tally
normalisation, batch means and variances) in plain NumPy float64.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mcdc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

T_ABSORB, T_LEAK, T_TIME, T_LOST, T_ROULETTE = range(5)
MU_LAWS = {"beam": 0, "uniform": 1, "cosine": 2}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no floating-point contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)


class _Problem(C.Structure):
    _fields_ = [
        ("G", C.c_int32), ("M", C.c_int32),
        ("sigma_t", _DP), ("sigma_s", _DP), ("speed", _DP),
        ("n_planes", C.c_int32 * 3), ("planes", _DP * 3),
        ("material", _IP), ("bc", C.c_int32 * 6),
        ("src_lo", C.c_double * 3), ("src_hi", C.c_double * 3),
        ("src_t_lo", C.c_double), ("src_t_hi", C.c_double),
        ("src_pmf", _DP), ("src_kind", C.c_int32),
        ("src_axis", C.c_int32), ("src_sign", C.c_int32), ("src_mu_law", C.c_int32),
        ("n_mesh", C.c_int32 * 3), ("mesh", _DP * 3),
        ("n_time_edges", C.c_int32), ("time_edges", _DP),
        ("n_batches", C.c_int32),
        ("qoi_on", C.c_int32), ("qoi_lo", C.c_double * 3), ("qoi_hi", C.c_double * 3),
        ("qoi_groups", _IP),
        ("n_ww", C.c_int32 * 3), ("ww", _DP * 3),
        ("ww_center", _DP), ("ww_ratio", C.c_double), ("ww_max_split", C.c_int32),
        ("time_crossing", C.c_int32),
        ("sigma_f", _DP), ("nu", _DP), ("chi", _DP),
        ("implicit_capture", C.c_int32), ("roulette_w", C.c_double), ("roulette_ws", C.c_double),
        ("pin_radius", _DP), ("pin_material", _IP),
        ("rod_z", _DP), ("rod_material", _IP),
        ("quad_coef", _DP), ("quad_material", _IP),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.oracle_rng_skip.restype = C.c_uint64
        _lib.oracle_rng_skip.argtypes = [C.c_uint64, C.c_uint64]
        _lib.oracle_child_stream.restype = C.c_uint64
        _lib.oracle_child_stream.argtypes = [C.c_uint64, C.c_uint64]
        _lib.oracle_rng_draws.restype = None
        _lib.oracle_rng_draws.argtypes = [C.c_uint64, C.c_int64, C.c_void_p, C.c_void_p]
        _lib.oracle_ntally.restype = C.c_int64
        _lib.oracle_ntally.argtypes = [C.c_void_p]
        _lib.oracle_union_planes.restype = C.c_int
        _lib.oracle_union_planes.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        _lib.oracle_run.restype = C.c_int
        _lib.oracle_run.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p,
                                    C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        _lib.oracle_eigen.restype = C.c_int
        _lib.oracle_eigen.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_int, C.c_uint64,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.oracle_run_pc.restype = C.c_int
        _lib.oracle_run_pc.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]
        _lib.oracle_comb.restype = C.c_int
        _lib.oracle_comb.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_double, C.c_void_p]
        _lib.oracle_q64_sum.restype = C.c_int
        _lib.oracle_q64_sum.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        _lib.oracle_trace.restype = C.c_int
        _lib.oracle_trace.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64,
                                      C.c_void_p, C.c_int]
    return _lib


def _dp(a):
    return a.ctypes.data_as(_DP)


class OracleProblem:
    """A problem dict (see ``workloads.problems``) marshalled into the
    oracle's struct.  Keeps every array it points at alive."""

    def __init__(self, prob: dict, ww_center=None, ww_ratio=5.0, ww_max_split=16):
        self.prob = prob
        keep = []

        def arr(a, dt=np.float64):
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            keep.append(a)
            return a

        s = _Problem()
        st = arr(prob["sigma_t"])
        M, G = st.shape
        s.G, s.M = G, M
        s.sigma_t = _dp(st)
        s.sigma_s = _dp(arr(prob["sigma_s"]))
        s.speed = _dp(arr(prob["speed"]))
        for a in range(3):
            pl = arr(prob["planes"][a])
            s.n_planes[a] = pl.size
            s.planes[a] = _dp(pl)
        s.material = arr(prob["material"], np.int32).ctypes.data_as(_IP)
        for f in range(6):
            s.bc[f] = int(prob["bc"][f])
        src = prob["source"]
        for a in range(3):
            s.src_lo[a] = float(src["lo"][a])
            s.src_hi[a] = float(src["hi"][a])
        s.src_t_lo, s.src_t_hi = float(src["t_lo"]), float(src["t_hi"])
        s.src_pmf = _dp(arr(src["group_pmf"]))
        if src["kind"] == "surface":
            s.src_kind = 1
            s.src_axis = int(src["axis"])
            s.src_sign = int(src["sign"])
            s.src_mu_law = MU_LAWS[src["mu_law"]]
        tal = prob["tally"]
        for a in range(3):
            m = arr(tal["mesh"][a])
            s.n_mesh[a] = m.size
            s.mesh[a] = _dp(m)
        te = arr(tal["time_edges"])
        s.n_time_edges = te.size
        s.time_edges = _dp(te)
        s.n_batches = int(tal["n_batches"])
        q = prob.get("qoi")
        if q is not None:
            s.qoi_on = 1
            for a in range(3):
                s.qoi_lo[a] = float(q["lo"][a])
                s.qoi_hi[a] = float(q["hi"][a])
            s.qoi_groups = arr(q["group_mask"], np.int32).ctypes.data_as(_IP)
        ww = prob.get("ww_mesh")
        for a in range(3):
            m = arr(ww[a] if ww is not None else np.zeros(0))
            s.n_ww[a] = m.size
            s.ww[a] = _dp(m)
        if ww_center is not None:
            s.ww_center = _dp(arr(ww_center))
            s.ww_ratio = float(ww_ratio)
            s.ww_max_split = int(ww_max_split)
        s.time_crossing = 1 if tal.get("time_crossing", False) else 0
        fis = prob.get("fission")
        if fis is not None:
            s.sigma_f = _dp(arr(fis["sigma_f"]))
            s.nu = _dp(arr(fis["nu"]))
            s.chi = _dp(arr(fis["chi"]))
        ic = prob.get("implicit_capture")
        if ic is not None:
            s.implicit_capture = 1
            s.roulette_w = float(ic["w_min"])
            s.roulette_ws = float(ic["w_survive"])
        pins = prob.get("pins")
        if pins is not None:
            s.pin_radius = _dp(arr(pins["radius"]))
            s.pin_material = arr(pins["material"], np.int32).ctypes.data_as(_IP)
        rod = prob.get("rod")
        if rod is not None:
            s.rod_z = _dp(arr(rod["z"]))
            s.rod_material = arr(rod["material"], np.int32).ctypes.data_as(_IP)
        quad = prob.get("quadrics")
        if quad is not None:
            s.quad_coef = _dp(arr(quad["coef"]))
            s.quad_material = arr(quad["material"], np.int32).ctypes.data_as(_IP)
        self.time_crossing = bool(s.time_crossing)
        self.struct = s
        self._keep = keep
        self.G, self.M = G, M
        self.K = te.size - 1
        self.B = int(tal["n_batches"])
        self.ntally = lib().oracle_ntally(C.byref(s))
        self.tally_shape = (self.K, G) + tuple(
            max(1, prob["tally"]["mesh"][a].size - 1) for a in (2, 1, 0))

    def ptr(self):
        return C.byref(self.struct)


def union_planes(prob: dict, axis: int) -> np.ndarray:
    op = OracleProblem(prob)
    buf = np.zeros(4096)
    n = lib().oracle_union_planes(op.ptr(), axis, buf.ctypes.data, buf.size)
    if n < 0:
        raise ValueError("invalid planes")
    return buf[:n].copy()


def rng_skip(state: int, k: int) -> int:
    return int(lib().oracle_rng_skip(state, k))


def rng_draws(state: int, n: int):
    st = np.zeros(n, dtype=np.uint64)
    xi = np.zeros(n)
    lib().oracle_rng_draws(state, n, st.ctypes.data, xi.ctypes.data)
    return st, xi


def child_stream(parent: int, j: int) -> int:
    return int(lib().oracle_child_stream(parent, j))


def batch_sizes(N: int, B: int) -> np.ndarray:
    B = max(1, min(B, N))
    b = np.arange(B + 1, dtype=np.int64)
    edges = (b * N) // B
    return np.diff(edges)


def run(prob, N: int, seed: int, ids=None, first: int = 0, count=None,
        records: bool = False, ww_center=None, ww_ratio=5.0, ww_max_split=16):
    """Run histories of an N-history job through the oracle.

    Returns raw per-batch sums 'S' [B, ntally], time-crossing sums 'X'
    [B, ntally] (zeros unless the problem's tally asks for them), leak sums
    'L' [B, K, G, 6],
    detector sums 'q' = (sum x, sum x^2), totals 'tot' (census, surface,
    collision events; absorb, leak, time, lost, roulette terminations;
    splits; fission neutrons beyond the colliding one), and if records: per-history 'rec' [n, 5] = (census, surface,
    collision, particles, termination mask) and 'trk' [n, 2] = (scored track,
    detector score)."""
    op = prob if isinstance(prob, OracleProblem) else OracleProblem(
        prob, ww_center, ww_ratio, ww_max_split)
    B = max(1, min(op.B, N))
    if ids is not None:
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
        n = ids.size
        if n and int(ids.max()) >= N:
            raise ValueError("history ids must be below N")
    else:
        n = N - first if count is None else count
        if first < 0 or n < 0 or first + n > N:
            raise ValueError(f"histories [{first}, {first + n}) outside the {N}-history job")
    S = np.zeros((B, op.ntally))
    X = np.zeros((B, op.ntally))
    L = np.zeros((B, op.K, op.G, 6))
    q = np.zeros(2)
    tot = np.zeros(10, dtype=np.uint64)
    rec = np.zeros((n, 5), dtype=np.uint32) if records else None
    trk = np.zeros((n, 2)) if records else None
    rc = lib().oracle_run(op.ptr(), N, seed, ids.ctypes.data if ids is not None else None,
                          first, n, S.ctypes.data, L.ctypes.data, q.ctypes.data,
                          tot.ctypes.data,
                          rec.ctypes.data if records else None,
                          trk.ctypes.data if records else None,
                          X.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_run failed with code {rc}")
    out = {"S": S, "X": X, "L": L, "q": q, "tot": tot, "N": N, "B": B, "op": op}
    if records:
        out["rec"] = rec
        out["trk"] = trk
    return out


def run_pc(prob, N: int, seed: int, target: int, method: str = "split"):
    """An N-history run with population control at every census edge to
    `target` particles: splitting-roulette (method "split", the oracle's
    reading R16) or combing ("comb", R28).  Returns the dict of ``run`` (no
    detector, no records) plus 'pop' [K]: particles alive at each edge T_k
    after the control (pop[0]: born)."""
    op = prob if isinstance(prob, OracleProblem) else OracleProblem(prob)
    B = max(1, min(op.B, N))
    S = np.zeros((B, op.ntally))
    X = np.zeros((B, op.ntally))
    L = np.zeros((B, op.K, op.G, 6))
    tot = np.zeros(10, dtype=np.uint64)
    pop = np.zeros(op.K, dtype=np.uint64)
    m = {"split": 0, "comb": 1}[method]
    rc = lib().oracle_run_pc(op.ptr(), N, seed, target, m, S.ctypes.data, L.ctypes.data,
                             tot.ctypes.data, X.ctypes.data, pop.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_run_pc failed with code {rc}")
    return {"S": S, "X": X, "L": L, "q": np.zeros(2), "tot": tot, "N": N, "B": B, "op": op,
            "pop": pop}


def comb(w, M: int, u: float) -> np.ndarray:
    """R28's copies of the weights w, taken in the given order, for a comb
    of M teeth at offset u in [0, 1)."""
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    out = np.zeros(w.size, dtype=np.uint64)
    rc = lib().oracle_comb(w.ctypes.data, w.size, M, float(u), out.ctypes.data)
    if rc != 0:
        raise ValueError("weights with a zero total, or a weight of 2^32 or more")
    return out


def q64_sum(w) -> tuple:
    """The oracle's exact fixed-point weight sum (R16): ((hi, lo), value)."""
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    out = np.zeros(2, dtype=np.uint64)
    val = C.c_double(0.0)
    rc = lib().oracle_q64_sum(w.ctypes.data, w.size, out.ctypes.data, C.byref(val))
    if rc != 0:
        raise ValueError("weight of 2^32 or more, or not a finite non-negative number")
    return (int(out[0]), int(out[1])), val.value


def bin_volumes(prob) -> np.ndarray:
    """Tally-bin volume factor per (z, y, x) bin: product of the bin widths
    of the axes that carry mesh planes (1 for axes without)."""
    w = []
    for a in (2, 1, 0):
        m = prob["tally"]["mesh"][a]
        w.append(np.diff(m) if m.size else np.ones(1))
    return w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]


def time_widths(prob) -> np.ndarray:
    te = prob["tally"]["time_edges"]
    dt = np.diff(te)
    return np.where(np.isfinite(dt), dt, 1.0)


def estimates(prob, res) -> dict:
    """Normalised mean and batch variance of the bin fluxes (time-averaged
    scalar flux per source particle), of the leakage per face, and of the
    detector score.

    mean_j = sum_b S_b[j] / (N V_j dt_k); the batch mean of batch b is
    m_b = S_b / (N_b V_j dt_k); var = sum_b (m_b - mbar)^2 / (B (B - 1))."""
    op = res["op"]
    N, B = res["N"], res["B"]
    Nb = batch_sizes(N, B).astype(np.float64)
    norm = (time_widths(prob)[:, None, None, None, None] *
            bin_volumes(prob)[None, None, :, :, :] *
            np.ones((1, op.G, 1, 1, 1))).reshape(-1)
    S = res["S"]
    total = S.sum(axis=0)
    mean = total / (N * norm)
    mb = S / (Nb[:, None] * norm[None, :])
    if B > 1:
        var = ((mb - mb.mean(axis=0)) ** 2).sum(axis=0) / (B * (B - 1))
    else:
        var = np.zeros_like(mean)
    L = res["L"]
    leak_mean = L.sum(axis=0) / N
    lb = L / Nb[:, None, None, None]
    leak_var = (((lb - lb.mean(axis=0)) ** 2).sum(axis=0) / (B * (B - 1))) if B > 1 else np.zeros_like(leak_mean)
    out = {"mean": mean.reshape(op.tally_shape), "var": var.reshape(op.tally_shape),
           "raw": total.reshape(op.tally_shape),
           "leak_mean": leak_mean, "leak_var": leak_var}
    if op.time_crossing:
        # time-crossing flux at the edges T_1..T_K: sum_b X_b / (N V), no
        # time width; batch variance as for the bin fluxes
        vnorm = (bin_volumes(prob)[None, None, :, :, :] *
                 np.ones((op.K, op.G, 1, 1, 1))).reshape(-1)
        X = res["X"]
        xt = X.sum(axis=0)
        xb = X / (Nb[:, None] * vnorm[None, :])
        xvar = (((xb - xb.mean(axis=0)) ** 2).sum(axis=0) / (B * (B - 1))) if B > 1 else np.zeros_like(xt)
        out["tc_mean"] = (xt / (N * vnorm)).reshape(op.tally_shape)
        out["tc_var"] = xvar.reshape(op.tally_shape)
    q = prob.get("qoi")
    if q is not None:
        vol = 1.0
        for a in range(3):
            if prob["planes"][a].size:
                vol *= q["hi"][a] - q["lo"][a]
        sx, sxx = res["q"]
        out["qoi_mean"] = sx / (N * vol)
        out["qoi_var"] = (sxx - sx * sx / N) / (N * (N - 1)) / (vol * vol) if N > 1 else 0.0
    return out


def trace(prob, N: int, seed: int, i: int, cap: int = 100000) -> np.ndarray:
    op = OracleProblem(prob)
    rows = np.zeros((cap, 9))
    n = lib().oracle_trace(op.ptr(), N, seed, i, rows.ctypes.data, cap)
    if n < 0:
        raise RuntimeError("trace failed")
    return rows[:n].copy()


def eigen(prob, N: int, n_inactive: int, n_active: int, seed: int):
    """k-eigenvalue power iteration (reading R13 of mcdc_oracle.c): cycles of
    N particles on a steady-state problem with fission.  Returns raw flux
    sums 'S' [n_active, ntally] and leak sums 'L' [n_active, K, G, 6] of
    the active cycles (one batch each), 'k' per cycle, totals 'tot'."""
    op = prob if isinstance(prob, OracleProblem) else OracleProblem(prob)
    S = np.zeros((n_active, op.ntally))
    L = np.zeros((n_active, op.K, op.G, 6))
    k = np.zeros(n_inactive + n_active)
    tot = np.zeros(10, dtype=np.uint64)
    nts = op.ntally // (op.K * op.G)
    hist = np.zeros((n_inactive + n_active, nts), dtype=np.uint64)
    rc = lib().oracle_eigen(op.ptr(), N, n_inactive, n_active, seed, S.ctypes.data, L.ctypes.data,
                            k.ctypes.data, tot.ctypes.data, hist.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_eigen failed with code {rc}")
    return {"S": S, "L": L, "k": k, "tot": tot, "hist": hist, "N": N, "n_inactive": n_inactive,
            "n_active": n_active, "op": op}


def source_entropy(hist) -> np.ndarray:
    """Shannon entropy (bits) of each cycle's fission source over the
    spatial tally bins: -sum p log2 p over the bins with sites."""
    hist = np.asarray(hist, dtype=np.float64)
    out = np.zeros(hist.shape[0])
    for c, h in enumerate(hist):
        tot = h.sum()
        if tot > 0:
            p = h[h > 0] / tot
            out[c] = float(-(p * np.log2(p)).sum())
    return out


def eigen_estimates(prob, res) -> dict:
    """Flux per cycle-source neutron and leakage, mean over the active
    cycles and the variance of that mean across cycles; k mean over the
    active cycles and its standard error."""
    op = res["op"]
    N, A = res["N"], res["n_active"]
    norm = (bin_volumes(prob)[None, None, :, :, :] * np.ones((op.K, op.G, 1, 1, 1))).reshape(-1)
    mb = res["S"] / (N * norm[None, :])
    mean = mb.mean(axis=0)
    var = ((mb - mean) ** 2).sum(axis=0) / (A * (A - 1)) if A > 1 else np.zeros_like(mean)
    lb = res["L"] / N
    lmean = lb.mean(axis=0)
    lvar = ((lb - lmean) ** 2).sum(axis=0) / (A * (A - 1)) if A > 1 else np.zeros_like(lmean)
    ka = res["k"][res["n_inactive"]:]
    return {"mean": mean.reshape(op.tally_shape), "var": var.reshape(op.tally_shape),
            "leak_mean": lmean, "leak_var": lvar, "k_mean": float(ka.mean()),
            "k_std": float(ka.std(ddof=1) / math.sqrt(A)) if A > 1 else 0.0, "k": res["k"]}
