"""ctypes binding of libmcdc_hip.so (the C ABI in include/mcdc.h).

Argument marshalling only: every step of the transport runs in the HIP
library.  Device buffers and the stream come from PyTorch.  The library must
be built (``__graft_entry__.build()`` or ``python -m
paper_2305_07636_amd.build``); importing this module on a machine without
it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcdc_hip.so")

MCDC_ABI_VERSION = 6
MCDC_OK, MCDC_E_INVALID, MCDC_E_HIP, MCDC_E_NOMEM, MCDC_E_OVERFLOW, MCDC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
MCDC_ALG_EVENT, MCDC_ALG_HISTORY, MCDC_ALG_AUTO = 0, 1, 2
MCDC_SRC_ISOTROPIC, MCDC_SRC_SURFACE = 0, 1
MU_LAWS = {"beam": 0, "uniform": 1, "cosine": 2}

EXPORTS = ["mcdc_problem_create", "mcdc_problem_destroy", "mcdc_problem_tally_shape",
           "mcdc_run", "mcdc_run_noalloc", "mcdc_run_batched", "mcdc_run_eigenvalue", "mcdc_set_weight_windows",
           "mcdc_last_error", "mcdc_mlp_create",
           "mcdc_mlp_destroy", "mcdc_mlp_get_params", "mcdc_mlp_set_params", "mcdc_mlp_grad",
           "mcdc_mlp_train", "mcdc_mlp_infer"]

_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)


class mcdc_problem_desc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("n_groups", C.c_int32), ("n_materials", C.c_int32),
        ("sigma_t", _DP), ("sigma_s", _DP), ("speed", _DP),
        ("n_planes", C.c_int32 * 3), ("planes", _DP * 3),
        ("material", _IP), ("bc", C.c_int32 * 6),
        ("src_kind", C.c_int32), ("src_axis", C.c_int32), ("src_sign", C.c_int32),
        ("src_mu_law", C.c_int32),
        ("src_lo", C.c_double * 3), ("src_hi", C.c_double * 3),
        ("src_t_lo", C.c_double), ("src_t_hi", C.c_double),
        ("src_group_pmf", _DP),
        ("n_mesh_planes", C.c_int32 * 3), ("mesh_planes", _DP * 3),
        ("n_time_edges", C.c_int32), ("time_edges", _DP),
        ("n_batches", C.c_int32),
        ("qoi_enabled", C.c_int32), ("qoi_lo", C.c_double * 3), ("qoi_hi", C.c_double * 3),
        ("qoi_group_mask", _IP),
        ("n_ww_planes", C.c_int32 * 3), ("ww_planes", _DP * 3),
        ("time_crossing", C.c_int32),
        ("sigma_f", _DP), ("nu", _DP), ("chi", _DP),
        ("implicit_capture", C.c_int32), ("roulette_w", C.c_double), ("roulette_ws", C.c_double),
        ("pin_radius", _DP), ("pin_material", _IP),
        ("rod_z", _DP), ("rod_material", _IP),
        ("quadric_coef", _DP), ("quadric_material", _IP),
    ]


class mcdc_run_options(C.Structure):
    _fields_ = [
        ("algorithm", C.c_int32), ("block_size", C.c_int32), ("bank_capacity", C.c_int64),
        ("flags", C.c_int32), ("stream", C.c_void_p),
        ("debug_counts", C.c_void_p), ("debug_scores", C.c_void_p),
        ("profile", C.c_void_p), ("profile_mask", C.c_uint32), ("profile_every", C.c_int32), ("profile_phase", C.c_int32),
        ("segments", C.c_int32), ("sort_cadence", C.c_int32), ("pc_target", C.c_uint64),
        ("steps_per_launch", C.c_int32), ("pc_method", C.c_int32),
    ]


PROF_CLASSES = ["source", "advance", "events", "history", "other", "control", "sort"]


class mcdc_result(C.Structure):
    _fields_ = [
        ("host_outputs", C.c_int32), ("reserved", C.c_int32),
        ("mean", C.c_void_p), ("var", C.c_void_p), ("raw", C.c_void_p),
        ("leak_mean", C.c_void_p), ("leak_var", C.c_void_p),
        ("qoi_sum", C.c_double * 2), ("qoi_mean", C.c_double), ("qoi_var", C.c_double),
        ("n_events", C.c_uint64 * 3), ("n_term", C.c_uint64 * 5), ("n_splits", C.c_uint64),
        ("kernel_ms", C.c_double),
        ("tc_mean", C.c_void_p), ("tc_var", C.c_void_p),
        ("n_fission", C.c_uint64),
        ("k_mean", C.c_double), ("k_std", C.c_double),
    ]


_lib = None


def lib():
    """Load libmcdc_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (loaded the other way round, torch later finds no GPU)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        L.mcdc_problem_create.argtypes = [C.POINTER(mcdc_problem_desc), C.POINTER(C.c_void_p)]
        L.mcdc_problem_create.restype = C.c_int
        L.mcdc_problem_destroy.argtypes = [C.c_void_p]
        L.mcdc_problem_destroy.restype = C.c_int
        L.mcdc_problem_tally_shape.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.mcdc_problem_tally_shape.restype = C.c_int
        L.mcdc_run.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(mcdc_run_options),
                               C.POINTER(mcdc_result)]
        L.mcdc_run.restype = C.c_int
        L.mcdc_run_noalloc.argtypes = L.mcdc_run.argtypes
        L.mcdc_run_noalloc.restype = C.c_int
        L.mcdc_set_weight_windows.argtypes = [C.c_void_p, _DP, C.c_double, C.c_int32]
        L.mcdc_set_weight_windows.restype = C.c_int
        L.mcdc_last_error.argtypes = []
        L.mcdc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class MCDCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mcdc error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != MCDC_OK:
        raise MCDCError(rc, lib().mcdc_last_error().decode(errors="replace"))


def _dp(a):
    return a.ctypes.data_as(_DP)


def make_desc(prob: dict):
    """Marshal a problem dict (see ``workloads.problems``) into the C
    descriptor.  Returns (desc, keep-alive list)."""
    keep = []

    def arr(a, dt=np.float64):
        a = np.ascontiguousarray(np.asarray(a, dtype=dt))
        keep.append(a)
        return a

    d = mcdc_problem_desc()
    d.abi_version = MCDC_ABI_VERSION
    st = arr(prob["sigma_t"])
    M, G = st.shape
    d.n_groups, d.n_materials = G, M
    d.sigma_t = _dp(st)
    d.sigma_s = _dp(arr(prob["sigma_s"]))
    d.speed = _dp(arr(prob["speed"]))
    for a in range(3):
        pl = arr(prob["planes"][a])
        d.n_planes[a] = pl.size
        d.planes[a] = _dp(pl)
    d.material = arr(prob["material"], np.int32).ctypes.data_as(_IP)
    for f in range(6):
        d.bc[f] = int(prob["bc"][f])
    src = prob["source"]
    d.src_kind = MCDC_SRC_SURFACE if src["kind"] == "surface" else MCDC_SRC_ISOTROPIC
    if d.src_kind == MCDC_SRC_SURFACE:
        d.src_axis = int(src["axis"])
        d.src_sign = int(src["sign"])
        d.src_mu_law = MU_LAWS[src["mu_law"]]
    for a in range(3):
        d.src_lo[a] = float(src["lo"][a])
        d.src_hi[a] = float(src["hi"][a])
    d.src_t_lo, d.src_t_hi = float(src["t_lo"]), float(src["t_hi"])
    d.src_group_pmf = _dp(arr(src["group_pmf"]))
    tal = prob["tally"]
    for a in range(3):
        m = arr(tal["mesh"][a])
        d.n_mesh_planes[a] = m.size
        d.mesh_planes[a] = _dp(m)
    te = arr(tal["time_edges"])
    d.n_time_edges = te.size
    d.time_edges = _dp(te)
    d.n_batches = int(tal["n_batches"])
    q = prob.get("qoi")
    if q is not None:
        d.qoi_enabled = 1
        for a in range(3):
            d.qoi_lo[a] = float(q["lo"][a])
            d.qoi_hi[a] = float(q["hi"][a])
        d.qoi_group_mask = arr(q["group_mask"], np.int32).ctypes.data_as(_IP)
    ww = prob.get("ww_mesh")
    for a in range(3):
        m = arr(ww[a] if ww is not None else np.zeros(0))
        d.n_ww_planes[a] = m.size
        d.ww_planes[a] = _dp(m)
    d.time_crossing = 1 if prob["tally"].get("time_crossing", False) else 0
    fis = prob.get("fission")
    if fis is not None:
        d.sigma_f = _dp(arr(fis["sigma_f"]))
        d.nu = _dp(arr(fis["nu"]))
        d.chi = _dp(arr(fis["chi"]))
    ic = prob.get("implicit_capture")
    if ic is not None:
        d.implicit_capture = 1
        d.roulette_w = float(ic["w_min"])
        d.roulette_ws = float(ic["w_survive"])
    pins = prob.get("pins")
    if pins is not None:
        d.pin_radius = _dp(arr(pins["radius"]))
        d.pin_material = arr(pins["material"], np.int32).ctypes.data_as(_IP)
    rod = prob.get("rod")
    if rod is not None:
        d.rod_z = _dp(arr(rod["z"]))
        d.rod_material = arr(rod["material"], np.int32).ctypes.data_as(_IP)
    quad = prob.get("quadrics")
    if quad is not None:
        d.quadric_coef = _dp(arr(quad["coef"]))
        d.quadric_material = arr(quad["material"], np.int32).ctypes.data_as(_IP)
    return d, keep


class Problem:
    """Owning wrapper of an mcdc_problem handle."""

    def __init__(self, prob: dict):
        d, keep = make_desc(prob)
        h = C.c_void_p()
        _check(lib().mcdc_problem_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.prob = prob
        self.time_crossing = bool(prob["tally"].get("time_crossing", False))
        shape = (C.c_int64 * 5)()
        n = C.c_int64()
        _check(lib().mcdc_problem_tally_shape(h, shape, C.byref(n)))
        self.tally_shape = tuple(int(s) for s in shape)
        self.ntally = int(n.value)
        K, G = self.tally_shape[0], self.tally_shape[1]
        self.leak_shape = (K, G, 6)

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().mcdc_problem_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mcdc_problem_create(prob: dict) -> Problem:
    return Problem(prob)


def mcdc_problem_destroy(p: Problem) -> None:
    p.close()


def mcdc_problem_tally_shape(p: Problem):
    return p.tally_shape


def mcdc_set_weight_windows(p: Problem, centers, ratio: float = 5.0, max_split: int = 16) -> None:
    if centers is None:
        _check(lib().mcdc_set_weight_windows(p.handle, None, ratio, max_split))
        return
    c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64))
    _check(lib().mcdc_set_weight_windows(p.handle, _dp(c), float(ratio), int(max_split)))


def mcdc_run(p: Problem, n_histories: int, seed: int, algorithm: str = "event",
             block_size: int = 0, bank_capacity: int = 0, segments: int = 0,
             debug: bool = False, outputs=("mean", "var", "raw", "leak_mean", "leak_var"),
             profile=None, eager: bool = False, profile_classes=None, profile_every: int = 0,
             profile_phase: int = 0, two_kernel_step: bool = False, pc_target: int = 0,
             noalloc: bool = False, sort_cadence: int = 0, staged: bool = False,
             steps_per_launch: int = 0, pc_method: str = "split"):
    """Run n_histories through the GPU tracker.  Returns a dict of torch
    CUDA tensors (mean, var, raw [K, G, nz, ny, nx]; leak_mean, leak_var
    [K, G, 6]; tc_mean, tc_var [K, G, nz, ny, nx] for a problem with the
    time-crossing tally; debug_counts [N, 5] and debug_scores [N, 2] if
    debug) plus
    host scalars (events, terminations, splits, detector sums, kernel_ms).
    profile: optional float64 array [8, 4] that accumulates per kernel class
    (ms, launches, particles, algorithmic bytes).
    pc_target: population control at every census edge (splitting-roulette
    to that many particles; event form; 0 = off).
    noalloc: call mcdc_run_noalloc (history form, device outputs, no
    debug arrays or profile) instead of mcdc_run.
    steps_per_launch: census steps per launch of the event form's
    one-kernel step (analog; 0 = default).
    pc_method: "split" (splitting-roulette) or "comb" (combing) with
    pc_target."""
    import torch

    dev = torch.device("cuda", torch.cuda.current_device())
    res = mcdc_result()
    out = {}
    for name in ("mean", "var", "raw") + (("tc_mean", "tc_var") if p.time_crossing else ()):
        if name in outputs or (name.startswith("tc_") and name[3:] in outputs):
            t = torch.empty(p.tally_shape, dtype=torch.float64, device=dev)
            out[name] = t
            setattr(res, name, t.data_ptr())
    for name in ("leak_mean", "leak_var"):
        if name in outputs:
            t = torch.empty(p.leak_shape, dtype=torch.float64, device=dev)
            out[name] = t
            setattr(res, name, t.data_ptr())
    opt = mcdc_run_options()
    opt.algorithm = {"history": MCDC_ALG_HISTORY, "auto": MCDC_ALG_AUTO}.get(algorithm, MCDC_ALG_EVENT)
    opt.block_size = block_size
    opt.bank_capacity = bank_capacity
    opt.segments = segments
    opt.pc_target = pc_target
    opt.sort_cadence = sort_cadence
    opt.steps_per_launch = steps_per_launch
    opt.pc_method = {"split": 0, "comb": 1}[pc_method]
    opt.flags = (1 if eager else 0) | (2 if two_kernel_step else 0) | (4 if staged else 0)
    opt.stream = torch.cuda.current_stream(dev).cuda_stream
    if debug:
        dc = torch.empty((n_histories, 5), dtype=torch.int32, device=dev)
        ds = torch.empty((n_histories, 2), dtype=torch.float64, device=dev)
        opt.debug_counts = dc.data_ptr()
        opt.debug_scores = ds.data_ptr()
        out["debug_counts"] = dc
        out["debug_scores"] = ds
    if profile is not None:
        assert profile.dtype == np.float64 and profile.shape == (len(PROF_CLASSES), 4)
        assert profile.flags["C_CONTIGUOUS"]
        opt.profile = profile.ctypes.data
        if profile_classes:
            opt.profile_mask = sum(1 << PROF_CLASSES.index(c) for c in profile_classes)
        opt.profile_every = profile_every
        opt.profile_phase = profile_phase
    run = lib().mcdc_run_noalloc if noalloc else lib().mcdc_run
    _check(run(p.handle, int(n_histories), int(seed), C.byref(opt), C.byref(res)))
    out["events"] = np.array(res.n_events[:], dtype=np.uint64)
    out["terms"] = np.array(res.n_term[:], dtype=np.uint64)
    out["splits"] = int(res.n_splits)
    out["fission"] = int(res.n_fission)
    out["qoi_sum"] = (res.qoi_sum[0], res.qoi_sum[1])
    out["qoi_mean"] = res.qoi_mean
    out["qoi_var"] = res.qoi_var
    out["kernel_ms"] = res.kernel_ms
    return out


# ---------------------------------------------------------------------------
# weight-window network
# ---------------------------------------------------------------------------
MLP_WIDTHS = (8, 64, 64, 64, 1)
MLP_PARAMS = 8961
_mlp_ready = False


def _mlp_lib():
    global _mlp_ready
    L = lib()
    if not _mlp_ready:
        L.mcdc_mlp_create.argtypes = [C.POINTER(C.c_int32), C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]
        L.mcdc_mlp_create.restype = C.c_int
        L.mcdc_mlp_destroy.argtypes = [C.c_void_p]
        L.mcdc_mlp_destroy.restype = C.c_int
        L.mcdc_mlp_get_params.argtypes = [C.c_void_p, C.c_void_p]
        L.mcdc_mlp_get_params.restype = C.c_int
        L.mcdc_mlp_set_params.argtypes = [C.c_void_p, C.c_void_p]
        L.mcdc_mlp_set_params.restype = C.c_int
        L.mcdc_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        L.mcdc_mlp_grad.restype = C.c_int
        L.mcdc_mlp_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                     C.c_float, C.c_void_p, C.c_void_p]
        L.mcdc_mlp_train.restype = C.c_int
        L.mcdc_mlp_infer.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.mcdc_mlp_infer.restype = C.c_int
        _mlp_ready = True
    return L


def _f32_dev(t):
    import torch

    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return t.data_ptr()


class MLP:
    """Owning wrapper of an mcdc_mlp handle (device tensors in, device
    tensors out)."""

    def __init__(self, seed: int = 1):
        L = _mlp_lib()
        w = (C.c_int32 * 5)(*MLP_WIDTHS)
        h = C.c_void_p()
        _check(L.mcdc_mlp_create(w, 4, seed, C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle is not None and self.handle.value:
            _mlp_lib().mcdc_mlp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_mlp_lib().mcdc_mlp_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        assert p.size == MLP_PARAMS
        _check(_mlp_lib().mcdc_mlp_set_params(self.handle, p.ctypes.data))

    def _stream(self):
        import torch

        return torch.cuda.current_stream().cuda_stream

    def grad(self, X, T, W):
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = C.c_float()
        _check(_mlp_lib().mcdc_mlp_grad(self.handle, _f32_dev(X), _f32_dev(T), _f32_dev(W), X.shape[0],
                                        C.byref(loss), g.ctypes.data, self._stream()))
        return float(loss.value), g

    def train(self, X, T, W, steps: int, lr: float = 1e-3):
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        _check(_mlp_lib().mcdc_mlp_train(self.handle, _f32_dev(X), _f32_dev(T), _f32_dev(W), X.shape[0],
                                         steps, lr, losses.ctypes.data, self._stream()))
        return losses[:steps]

    def infer(self, X):
        import torch

        Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(_mlp_lib().mcdc_mlp_infer(self.handle, _f32_dev(X), X.shape[0], _f32_dev(Y), self._stream()))
        return Y


def mcdc_mlp_create(seed: int = 1) -> MLP:
    return MLP(seed)


def mcdc_run_batched(problems, n_hist, seeds, block_size: int = 0, outputs=("mean", "var"),
                     algorithm: str = "event", seg_len: int = 0, debug: bool = False, sort_cadence: int = 0,
                     two_kernel_step: bool = False):
    """Run many problems together: event form (shared banks, one graph per
    census step for all problems), history form (one persistent launch) or
    "auto" (both timed on the first call for a batch signature, the faster
    one cached).  Returns one result dict per problem, like mcdc_run (with
    debug: each dict's debug_counts [n, 5] and debug_scores [n, 2] are views
    of one array over all problems' histories in problem order)."""
    import torch

    L = lib()
    if not getattr(L, "_batched_ready", False):
        L.mcdc_run_batched.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_uint64),
                                       C.POINTER(C.c_uint64), C.POINTER(mcdc_run_options),
                                       C.POINTER(mcdc_result)]
        L.mcdc_run_batched.restype = C.c_int
        L._batched_ready = True
    n = len(problems)
    dev = torch.device("cuda", torch.cuda.current_device())
    hs = (C.c_void_p * n)(*[p.handle.value for p in problems])
    nh = (C.c_uint64 * n)(*[int(x) for x in n_hist])
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    res = (mcdc_result * n)()
    outs = []
    for j, p in enumerate(problems):
        o = {}
        for name in ("mean", "var", "raw") + (("tc_mean", "tc_var") if p.time_crossing else ()):
            if name in outputs or (name.startswith("tc_") and name[3:] in outputs):
                t = torch.empty(p.tally_shape, dtype=torch.float64, device=dev)
                o[name] = t
                setattr(res[j], name, t.data_ptr())
        for name in ("leak_mean", "leak_var"):
            if name in outputs:
                t = torch.empty(p.leak_shape, dtype=torch.float64, device=dev)
                o[name] = t
                setattr(res[j], name, t.data_ptr())
        outs.append(o)
    opt = mcdc_run_options()
    opt.algorithm = {"history": MCDC_ALG_HISTORY, "auto": MCDC_ALG_AUTO}.get(algorithm, MCDC_ALG_EVENT)
    opt.block_size = block_size
    opt.bank_capacity = seg_len
    opt.sort_cadence = sort_cadence
    opt.flags = 2 if two_kernel_step else 0
    opt.stream = torch.cuda.current_stream(dev).cuda_stream
    if debug:
        tot = int(sum(int(x) for x in n_hist))
        dc = torch.empty((tot, 5), dtype=torch.int32, device=dev)
        ds = torch.empty((tot, 2), dtype=torch.float64, device=dev)
        opt.debug_counts = dc.data_ptr()
        opt.debug_scores = ds.data_ptr()
        off = 0
        for j, o in enumerate(outs):
            k = int(n_hist[j])
            o["debug_counts"] = dc[off:off + k]
            o["debug_scores"] = ds[off:off + k]
            off += k
    _check(L.mcdc_run_batched(hs, n, nh, sd, C.byref(opt), res))
    for j, o in enumerate(outs):
        r = res[j]
        o["events"] = np.array(r.n_events[:], dtype=np.uint64)
        o["terms"] = np.array(r.n_term[:], dtype=np.uint64)
        o["qoi_sum"] = (r.qoi_sum[0], r.qoi_sum[1])
        o["qoi_mean"] = r.qoi_mean
        o["qoi_var"] = r.qoi_var
        o["kernel_ms"] = r.kernel_ms
    return outs


def mcdc_run_eigenvalue(p: Problem, n_per_cycle: int, n_inactive: int, n_active: int, seed: int,
                        outputs=("mean", "var", "leak_mean", "leak_var")):
    """k-eigenvalue power iteration on the GPU.  Returns a dict like
    mcdc_run (flux and leakage over the active cycles, totals over all
    cycles) plus 'k' (every cycle), 'k_mean', 'k_std', and the fission
    source per cycle: 'source_hist' (sites per spatial tally bin) and its
    Shannon 'entropy' (bits)."""
    import torch

    L = lib()
    if not getattr(L, "_eigen_ready", False):
        L.mcdc_run_eigenvalue.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, C.c_int32, C.c_uint64,
                                          C.POINTER(mcdc_run_options), C.POINTER(mcdc_result), _DP,
                                          C.c_void_p, _DP]
        L.mcdc_run_eigenvalue.restype = C.c_int
        L._eigen_ready = True
    dev = torch.device("cuda", torch.cuda.current_device())
    res = mcdc_result()
    out = {}
    for name in ("mean", "var", "raw"):
        if name in outputs:
            t = torch.empty(p.tally_shape, dtype=torch.float64, device=dev)
            out[name] = t
            setattr(res, name, t.data_ptr())
    for name in ("leak_mean", "leak_var"):
        if name in outputs:
            t = torch.empty(p.leak_shape, dtype=torch.float64, device=dev)
            out[name] = t
            setattr(res, name, t.data_ptr())
    opt = mcdc_run_options()
    opt.stream = torch.cuda.current_stream(dev).cuda_stream
    k = np.zeros(n_inactive + n_active)
    nts = p.tally_shape[2] * p.tally_shape[3] * p.tally_shape[4]
    hist = np.zeros((n_inactive + n_active, nts), dtype=np.uint64)
    ent = np.zeros(n_inactive + n_active)
    _check(L.mcdc_run_eigenvalue(p.handle, int(n_per_cycle), int(n_inactive), int(n_active), int(seed),
                                 C.byref(opt), C.byref(res), _dp(k), hist.ctypes.data, _dp(ent)))
    out["source_hist"] = hist
    out["entropy"] = ent
    out["events"] = np.array(res.n_events[:], dtype=np.uint64)
    out["terms"] = np.array(res.n_term[:], dtype=np.uint64)
    out["k"] = k
    out["k_mean"] = res.k_mean
    out["k_std"] = res.k_std
    out["kernel_ms"] = res.kernel_ms
    return out
