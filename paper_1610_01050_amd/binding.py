"""ctypes binding of the RSFT C ABI (include/rsft.h).

Argument marshalling only: every step of the hot path runs in the HIP
library. torch is used for device memory (tensors' data pointers) and
streams (the current stream's handle); no torch op touches the data.
The binding refuses to work without the built library: there is no CPU
fallback.
"""

import ctypes
import os

import numpy as np

LIB_NAME = "librsft.so"
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), LIB_NAME)

MAX_DIMS = 4
MAX_ROUNDS = 64

OK = 0
STATUS_NAMES = {
    0: "RSFT_OK", 1: "RSFT_ERROR_INVALID_ARGUMENT", 2: "RSFT_ERROR_NOT_POW2",
    3: "RSFT_ERROR_BAD_SIGMA", 4: "RSFT_ERROR_UNSUPPORTED",
    5: "RSFT_ERROR_OUT_OF_MEMORY", 6: "RSFT_ERROR_DEVICE",
    7: "RSFT_ERROR_CAPACITY", 8: "RSFT_ERROR_NOT_READY",
}
ERROR_CAPACITY = 7

C64, C128 = 0, 1
NOISE_KNOWN, NOISE_ESTIMATED = 0, 1
OPT_GRAPH, OPT_TIMING = 0, 1
OPT_FOLD_THREADS, OPT_FOLD_VEC, OPT_FOLD_NONTEMPORAL = 2, 3, 4
OPT_ESTIMATE_WORKERS = 5
OPT_VOTE_WORDS = 6
OPT_DFT_SPLIT = 7
OPT_DFT_THREADS = 8
STAGES = ("fold", "dft", "vote", "estimate")

# Every symbol include/rsft.h declares.
SYMBOLS = (
    "rsft_plan", "rsft_execute", "rsft_autotune", "rsft_execute_per_frame", "rsft_detect",
    "rsft_detection_count", "rsft_get_buckets", "rsft_get_flags",
    "rsft_vote_flags", "rsft_plan_info", "rsft_set_option", "rsft_stage_times",
    "rsft_destroy", "rsft_status_string", "rsft_last_error",
    "rsft_chebyshev_window", "rsft_flat_window", "rsft_mod_inverse",
    "rsft_stage1_probability", "rsft_draw_sigma",
    "rsft_model_workspace_size", "rsft_model_forward", "rsft_model_forward_noalloc",
    "rsft_model_backward", "rsft_refine_workspace_size", "rsft_initial_amplitudes", "rsft_refine",
    "rsft_model_residual", "rsft_execute_fold", "rsft_execute_tail",
    "rsft_design_thresholds",
)


class Params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("rounds", ctypes.c_int32),
        ("n", ctypes.c_int64 * MAX_DIMS), ("b", ctypes.c_int64 * MAX_DIMS),
        ("sigma", ctypes.POINTER(ctypes.c_int64)), ("seed", ctypes.c_uint64),
        ("window_atten_db", ctypes.c_double), ("flat_atten_db", ctypes.c_double),
        ("pfa", ctypes.c_double), ("mu", ctypes.c_int32),
        ("noise_mode", ctypes.c_int32), ("noise_var", ctypes.c_double),
        ("dtype", ctypes.c_int32), ("max_detections", ctypes.c_int32),
        ("max_batch", ctypes.c_int64), ("segments", ctypes.c_int32),
        ("reserved0", ctypes.c_int32), ("stage1_pfa", ctypes.c_double),
    ]


class Detection(ctypes.Structure):
    _fields_ = [
        ("frame", ctypes.c_int64), ("idx", ctypes.c_int64 * MAX_DIMS),
        ("votes", ctypes.c_int32), ("is_peak", ctypes.c_int32),
        ("magnitude", ctypes.c_float), ("reserved", ctypes.c_float),
        ("freq", ctypes.c_double * MAX_DIMS),
    ]


DETECTION_DTYPE = np.dtype([
    ("frame", "<i8"), ("idx", "<i8", (MAX_DIMS,)), ("votes", "<i4"),
    ("is_peak", "<i4"), ("magnitude", "<f4"), ("reserved", "<f4"),
    ("freq", "<f8", (MAX_DIMS,)),
])
assert DETECTION_DTYPE.itemsize == ctypes.sizeof(Detection)


class DesignParams(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("rounds", ctypes.c_int32),
        ("n", ctypes.c_int64 * MAX_DIMS), ("b", ctypes.c_int64 * MAX_DIMS),
        ("window_atten_db", ctypes.c_double), ("flat_atten_db", ctypes.c_double),
        ("omega_bins", ctypes.c_double * MAX_DIMS), ("sparsity", ctypes.c_double),
        ("eta_m", ctypes.c_double), ("pd", ctypes.c_double), ("pfa", ctypes.c_double),
        ("upper_bound", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("noise_var", ctypes.c_double),
    ]


class DesignResult(ctypes.Structure):
    _fields_ = [
        ("feasible", ctypes.c_int32), ("mu", ctypes.c_int32),
        ("snr_min", ctypes.c_double), ("snr_min_db", ctypes.c_double),
        ("pd_bar", ctypes.c_double), ("pfa_bar", ctypes.c_double),
        ("gamma", ctypes.c_double), ("alpha_bar", ctypes.c_double),
        ("beta_bar", ctypes.c_double), ("F", ctypes.c_double),
        ("eta_p", ctypes.c_double), ("eta_m", ctypes.c_double),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("rounds", ctypes.c_int32),
        ("mu", ctypes.c_int32), ("noise_mode", ctypes.c_int32),
        ("n", ctypes.c_int64 * MAX_DIMS), ("b", ctypes.c_int64 * MAX_DIMS),
        ("sigma", (ctypes.c_int64 * MAX_DIMS) * MAX_ROUNDS),
        ("sigma_inv", (ctypes.c_int64 * MAX_DIMS) * MAX_ROUNDS),
        ("tau", (ctypes.c_int64 * MAX_DIMS) * MAX_ROUNDS),
        ("beta", ctypes.c_double * MAX_ROUNDS),
        ("gamma", ctypes.c_double * MAX_ROUNDS),
        ("p1", ctypes.c_double), ("eta_m", ctypes.c_double),
        ("max_sparsity", ctypes.c_double),
        ("estimation_rounds", ctypes.c_uint64),
        ("fold_threads", ctypes.c_int32), ("fold_vec", ctypes.c_int32),
        ("fold_nontemporal", ctypes.c_int32), ("estimate_workers", ctypes.c_int32),
        ("vote_kernel", ctypes.c_int32), ("dft_two_pass", ctypes.c_int32),
        ("dft_threads", ctypes.c_int32),
    ]


class RsftError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_LIB = None


def load_library(path=None):
    """Load librsft.so (built by build.build_library). Raises if missing."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"RSFT HIP library not found at {p}; build it first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.rsft_plan.argtypes = [ctypes.POINTER(Params), i64, ctypes.POINTER(vp)]
    lib.rsft_execute.argtypes = [vp, vp, i64, vp]
    lib.rsft_execute_per_frame.argtypes = [vp, vp, i64, vp]
    lib.rsft_autotune.argtypes = [vp, vp, i64, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.rsft_detect.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.rsft_detection_count.argtypes = [vp, vp, ctypes.POINTER(i64)]
    lib.rsft_get_buckets.argtypes = [vp, vp, vp]
    lib.rsft_get_flags.argtypes = [vp, vp, vp]
    lib.rsft_vote_flags.argtypes = [vp, vp, vp]
    lib.rsft_plan_info.argtypes = [vp, i64, ctypes.POINTER(PlanInfo)]
    lib.rsft_set_option.argtypes = [vp, ctypes.c_int32, i64]
    lib.rsft_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(i64), ctypes.c_int32]
    lib.rsft_destroy.argtypes = [vp]
    lib.rsft_destroy.restype = None
    lib.rsft_status_string.argtypes = [ctypes.c_int]
    lib.rsft_status_string.restype = ctypes.c_char_p
    lib.rsft_last_error.argtypes = []
    lib.rsft_last_error.restype = ctypes.c_char_p
    lib.rsft_chebyshev_window.argtypes = [i64, ctypes.c_double, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.rsft_flat_window.argtypes = [i64, i64, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_double)]
    lib.rsft_mod_inverse.argtypes = [i64, i64, ctypes.POINTER(i64)]
    lib.rsft_stage1_probability.argtypes = [ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_double)]
    lib.rsft_model_workspace_size.argtypes = [vp, i64, ctypes.c_int32, ctypes.POINTER(i64)]
    lib.rsft_model_forward.argtypes = [vp, vp, vp, i64, ctypes.c_int32, vp, vp, vp]
    lib.rsft_model_forward_noalloc.argtypes = [vp, vp, vp, i64, ctypes.c_int32, vp, vp]
    lib.rsft_model_backward.argtypes = [vp, vp, i64, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    lib.rsft_refine_workspace_size.argtypes = [vp, i64, ctypes.c_int32, ctypes.POINTER(i64)]
    lib.rsft_initial_amplitudes.argtypes = [vp, vp, vp, i64, ctypes.c_int32, vp, vp, vp, vp]
    lib.rsft_refine.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_double,
                                vp, vp, vp]
    lib.rsft_model_residual.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int32, vp, vp, vp, vp]
    lib.rsft_execute_fold.argtypes = [vp, vp, i64, vp]
    lib.rsft_execute_tail.argtypes = [vp, vp]
    lib.rsft_design_thresholds.argtypes = [ctypes.POINTER(DesignParams),
                                           ctypes.POINTER(DesignResult)]
    lib.rsft_draw_sigma.argtypes = [ctypes.c_uint64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
    for name in SYMBOLS:
        if name in ("rsft_destroy", "rsft_status_string", "rsft_last_error"):
            continue
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _LIB = lib
    return lib


def _check(lib, status):
    if status != OK:
        raise RsftError(status, lib.rsft_last_error().decode(errors="replace"))


# ---- host-only design functions --------------------------------------------

def chebyshev_window(n, atten_db, periodic=False):
    lib = load_library()
    out = np.zeros(int(n), dtype=np.float64)
    _check(lib, lib.rsft_chebyshev_window(
        int(n), float(atten_db), 1 if periodic else 0,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def flat_window(n, b, atten_db):
    lib = load_library()
    out = np.zeros(2 * int(n), dtype=np.float64)
    _check(lib, lib.rsft_flat_window(int(n), int(b), float(atten_db),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out[0::2] + 1j * out[1::2]


def mod_inverse(sigma, n):
    lib = load_library()
    out = ctypes.c_int64()
    _check(lib, lib.rsft_mod_inverse(int(sigma), int(n), ctypes.byref(out)))
    return out.value


def stage1_probability(pfa, rounds, mu):
    lib = load_library()
    out = ctypes.c_double()
    _check(lib, lib.rsft_stage1_probability(float(pfa), int(rounds), int(mu),
                                            ctypes.byref(out)))
    return out.value


def draw_sigma(seed, rounds, shape):
    lib = load_library()
    n = (ctypes.c_int64 * len(shape))(*[int(v) for v in shape])
    out = (ctypes.c_int64 * (int(rounds) * len(shape)))()
    _check(lib, lib.rsft_draw_sigma(int(seed), int(rounds), len(shape), n, out))
    return np.array(list(out), dtype=np.int64).reshape(int(rounds), len(shape))


def design_thresholds(shape, buckets, rounds, sparsity, pd, pfa, omega_bins,
                      window_atten_db=60.0, flat_atten_db=-1.0, eta_m=0.0,
                      upper_bound=False, noise_var=1.0):
    """Optimal thresholds of eq. opt (rsft_design_thresholds): returns a
    dict with feasible, mu, snr_min, snr_min_db, pd_bar, pfa_bar (use as
    stage1_pfa of a plan, with mu), gamma, alpha_bar, beta_bar, F, eta_p,
    eta_m."""
    lib = load_library()
    q = DesignParams()
    q.ndim = len(shape)
    q.rounds = int(rounds)
    for d in range(len(shape)):
        q.n[d] = int(shape[d])
        q.b[d] = int(buckets[d])
        q.omega_bins[d] = float(omega_bins[d])
    q.window_atten_db = float(window_atten_db)
    q.flat_atten_db = float(flat_atten_db)
    q.sparsity = float(sparsity)
    q.eta_m = float(eta_m)
    q.pd = float(pd)
    q.pfa = float(pfa)
    q.upper_bound = 1 if upper_bound else 0
    q.noise_var = float(noise_var)
    r = DesignResult()
    _check(lib, lib.rsft_design_thresholds(ctypes.byref(q), ctypes.byref(r)))
    return {name: getattr(r, name) for name, _ in DesignResult._fields_}


# ---- plans ------------------------------------------------------------------

def _make_params(shape, buckets, rounds=3, sigma=None, seed=0, window_atten_db=60.0,
                 flat_atten_db=-1.0, pfa=1e-3, mu=0, noise_mode="known",
                 noise_var=1.0, dtype="c64", max_detections=0, max_batch=1,
                 segments=False, stage1_pfa=0.0):
    """Fill a Params struct; returns (params, keepalive) where keepalive
    holds the sigma array for the duration of rsft_plan."""
    shape = tuple(int(v) for v in shape)
    buckets = tuple(int(v) for v in buckets)
    if len(shape) != len(buckets) or not 1 <= len(shape) <= MAX_DIMS:
        raise ValueError("shape and buckets need 1..4 matching dimensions")
    p = Params()
    p.ndim = len(shape)
    p.rounds = int(rounds)
    for d in range(len(shape)):
        p.n[d] = shape[d]
        p.b[d] = buckets[d]
    keep = None
    if sigma is not None:
        sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.int64).reshape(-1))
        if sig.size != p.rounds * p.ndim:
            raise ValueError("sigma needs rounds * ndim entries")
        keep = sig
        p.sigma = sig.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    p.seed = int(seed)
    p.window_atten_db = float(window_atten_db)
    p.flat_atten_db = float(flat_atten_db)
    p.pfa = float(pfa)
    p.mu = int(mu)
    p.noise_mode = {"known": NOISE_KNOWN, "estimated": NOISE_ESTIMATED}[noise_mode]
    p.noise_var = float(noise_var)
    p.dtype = {"c64": C64, "c128": C128}[dtype]
    p.max_detections = int(max_detections)
    p.max_batch = int(max_batch)
    p.segments = int(segments)
    p.stage1_pfa = float(stage1_pfa)
    return p, keep


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """An RSFT plan (rsft_plan). Create with Plan(shape, buckets, ...) for a
    uniform batch or Plan.uneven([dict(shape=..., buckets=..., ...), ...])
    for one descriptor per frame."""

    def __init__(self, shape=None, buckets=None, _descs=None, **kw):
        self._lib = load_library()
        if _descs is None:
            _descs = [dict(shape=shape, buckets=buckets, **kw)]
        structs = []
        keep = []
        for dsc in _descs:
            p, k = _make_params(**dsc)
            structs.append(p)
            keep.append(k)
        arr = (Params * len(structs))(*structs)
        handle = ctypes.c_void_p()
        _check(self._lib, self._lib.rsft_plan(arr, len(structs), ctypes.byref(handle)))
        self._h = handle
        self.descs = [dict(d) for d in _descs]
        self.uniform = len(_descs) == 1
        self.rounds = int(_descs[0].get("rounds", 3))
        self.dtype = _descs[0].get("dtype", "c64")
        self.last_batch = None
        self._folded = None
        # input elements: per frame of a uniform plan, in all of an uneven one
        seg = self.rounds if _descs[0].get("segments") else 1
        self._elems = [int(np.prod(d["shape"])) * seg for d in self.descs]
        self._elems_total = sum(self._elems)

    @classmethod
    def uneven(cls, frames):
        return cls(_descs=list(frames))

    def _frame_buckets(self, batch):
        if self.uniform:
            return [tuple(self.descs[0]["buckets"])] * batch
        return [tuple(d["buckets"]) for d in self.descs]

    def _check_input(self, x, batch):
        import torch
        want = torch.complex64 if self.dtype == "c64" else torch.complex128
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("input must be a CUDA (HIP) torch tensor")
        if x.dtype != want:
            raise TypeError(f"input dtype must be {want}")
        if not x.is_contiguous():
            raise ValueError("input must be contiguous")
        need = self._elems[0] * int(batch) if self.uniform else self._elems_total
        if x.numel() < need:
            raise ValueError(f"input holds {x.numel()} elements, batch needs {need}")

    def execute(self, x, batch=None, stream=None):
        """Enqueue the hot path on `stream` (default: torch's current stream)."""
        if batch is None:
            batch = x.shape[0] if self.uniform else len(self.descs)
        self._check_input(x, batch)
        _check(self._lib, self._lib.rsft_execute(self._h, ctypes.c_void_p(x.data_ptr()),
                                                 int(batch), _stream_handle(stream)))
        self.last_batch = int(batch)

    def execute_fold(self, x, batch=None, stream=None):
        """Enqueue the fold stage of `x` on `stream` (rsft_execute_fold)."""
        if batch is None:
            batch = x.shape[0] if self.uniform else len(self.descs)
        self._check_input(x, batch)
        _check(self._lib, self._lib.rsft_execute_fold(self._h, ctypes.c_void_p(x.data_ptr()),
                                                      int(batch), _stream_handle(stream)))
        self._folded = int(batch)

    def execute_tail(self, stream=None):
        """Enqueue the stages after the fold for the batch last folded
        (rsft_execute_tail)."""
        _check(self._lib, self._lib.rsft_execute_tail(self._h, _stream_handle(stream)))
        self.last_batch = self._folded

    def autotune(self, x, batch=None, repeats=5, stream=None):
        """Time the launch shapes of every stage on `x` and keep the fastest
        (rsft_autotune: fold shape, DFT form and size, vote kernel, estimate
        layout; a later plan of the same signature starts from them);
        returns the fold's average duration in ms. The plan then holds the
        results of an execute of `x`."""
        if batch is None:
            batch = x.shape[0] if self.uniform else len(self.descs)
        self._check_input(x, batch)
        best = ctypes.c_double()
        _check(self._lib, self._lib.rsft_autotune(self._h, ctypes.c_void_p(x.data_ptr()), int(batch),
                                                  _stream_handle(stream), int(repeats),
                                                  ctypes.byref(best)))
        if batch > 0:
            self.last_batch = int(batch)
            self._folded = None
        return best.value

    def execute_per_frame(self, x, batch=None, stream=None):
        if batch is None:
            batch = x.shape[0] if self.uniform else len(self.descs)
        self._check_input(x, batch)
        _check(self._lib, self._lib.rsft_execute_per_frame(
            self._h, ctypes.c_void_p(x.data_ptr()), int(batch), _stream_handle(stream)))
        self.last_batch = int(batch)

    def detection_count(self, stream=None):
        out = ctypes.c_int64()
        _check(self._lib, self._lib.rsft_detection_count(self._h, _stream_handle(stream),
                                                         ctypes.byref(out)))
        return out.value

    def detect(self, capacity=None, stream=None, allow_truncation=False):
        """Synchronize and return (records, counts): records is a numpy
        structured array (DETECTION_DTYPE) sorted by (frame, cell); counts
        the exact per-frame detection counts."""
        if self.last_batch is None:
            raise RuntimeError("execute first")
        if capacity is None:
            capacity = self.detection_count(stream)
        recs = np.zeros(max(int(capacity), 1), dtype=DETECTION_DTYPE)
        counts = np.zeros(max(self.last_batch, 1), dtype=np.int64)
        written = ctypes.c_int64()
        st = self._lib.rsft_detect(self._h, _stream_handle(stream),
                                   ctypes.c_void_p(recs.ctypes.data), int(capacity),
                                   counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   ctypes.byref(written))
        if not (st == ERROR_CAPACITY and allow_truncation):
            _check(self._lib, st)
        return recs[:written.value], counts[:self.last_batch]

    def buckets(self, stream=None):
        """fhat of the last execute as a list of complex64 tensors [T, *B]."""
        import torch
        bks = self._frame_buckets(self.last_batch)
        sizes = [self.rounds * int(np.prod(b)) for b in bks]
        out = torch.empty(sum(sizes), dtype=torch.complex64, device="cuda")
        _check(self._lib, self._lib.rsft_get_buckets(self._h, ctypes.c_void_p(out.data_ptr()),
                                                     _stream_handle(stream)))
        res = []
        off = 0
        for b, sz in zip(bks, sizes):
            res.append(out[off:off + sz].view(self.rounds, *b))
            off += sz
        return res

    def flags(self, stream=None):
        """First-stage flags of the last execute: list of uint32 word tensors
        [T, ceil(B/32)] (as int32 storage)."""
        import torch
        bks = self._frame_buckets(self.last_batch)
        words = [(int(np.prod(b)) + 31) // 32 for b in bks]
        sizes = [self.rounds * w for w in words]
        out = torch.empty(sum(sizes), dtype=torch.int32, device="cuda")
        _check(self._lib, self._lib.rsft_get_flags(self._h, ctypes.c_void_p(out.data_ptr()),
                                                   _stream_handle(stream)))
        res = []
        off = 0
        for w, sz in zip(words, sizes):
            res.append(out[off:off + sz].view(self.rounds, w))
            off += sz
        return res

    def vote_flags(self, words, stream=None):
        """Redo voting and estimation from caller-supplied flag words (a
        contiguous int32 CUDA tensor in the layout of flags())."""
        _check(self._lib, self._lib.rsft_vote_flags(self._h, ctypes.c_void_p(words.data_ptr()),
                                                    _stream_handle(stream)))

    def info(self, frame=0):
        out = PlanInfo()
        _check(self._lib, self._lib.rsft_plan_info(self._h, int(frame), ctypes.byref(out)))
        D, T = out.ndim, out.rounds
        return {
            "ndim": D, "rounds": T, "mu": out.mu, "noise_mode": out.noise_mode,
            "n": [out.n[d] for d in range(D)], "b": [out.b[d] for d in range(D)],
            "sigma": np.array([[out.sigma[s][d] for d in range(D)] for s in range(T)]),
            "sigma_inv": np.array([[out.sigma_inv[s][d] for d in range(D)] for s in range(T)]),
            "tau": np.array([[out.tau[s][d] for d in range(D)] for s in range(T)]),
            "beta": np.array([out.beta[s] for s in range(T)]),
            "gamma": np.array([out.gamma[s] for s in range(T)]),
            "p1": out.p1, "eta_m": out.eta_m, "max_sparsity": out.max_sparsity,
            "estimation_rounds": [s for s in range(T) if (out.estimation_rounds >> s) & 1],
            "fold": {"threads": out.fold_threads, "vec": out.fold_vec,
                     "nontemporal": out.fold_nontemporal},
            "estimate_workers": out.estimate_workers,
            "vote_kernel": ("per_cell", "candidate_rows", "masks_32", "word_masks")[out.vote_kernel],
            "dft_two_pass": out.dft_two_pass,
            "dft_threads": out.dft_threads,
        }

    # -- bucketized forward model of complex tones (off-grid refinement) --

    def _model_args(self, freqs, amps):
        import torch
        if not (isinstance(freqs, torch.Tensor) and freqs.is_cuda and freqs.dtype == torch.float64
                and freqs.is_contiguous() and freqs.dim() == 3):
            raise TypeError("freqs must be a contiguous CUDA float64 tensor [batch, K, D]")
        if not (isinstance(amps, torch.Tensor) and amps.is_cuda and amps.dtype == torch.complex64
                and amps.is_contiguous() and tuple(amps.shape) == tuple(freqs.shape[:2])):
            raise TypeError("amps must be a contiguous CUDA complex64 tensor [batch, K]")
        batch, K, D = (int(v) for v in freqs.shape)
        if D != len(self.descs[0]["shape"]):
            raise ValueError("freqs' last dimension must be the frame dimension count")
        return batch, K

    def model_size(self, batch):
        """Complex values of a model (or bucket) array for `batch` frames."""
        return sum(self.rounds * int(np.prod(b)) for b in self._frame_buckets(batch))

    def model_workspace(self, batch, tones):
        import torch
        n = ctypes.c_int64()
        _check(self._lib, self._lib.rsft_model_workspace_size(self._h, int(batch), int(tones),
                                                              ctypes.byref(n)))
        return torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")

    def model_forward(self, freqs, amps, workspace, out=None, stream=None):
        """model_s[k] = sum_t b_t prod_d G_{s,d}(f_t)[k_d] for every frame:
        a complex64 tensor in the layout of buckets() (flat). `workspace`
        (model_workspace) receives the factors the backward call needs."""
        import torch
        batch, K = self._model_args(freqs, amps)
        if out is None:
            out = torch.empty(self.model_size(batch), dtype=torch.complex64, device="cuda")
        _check(self._lib, self._lib.rsft_model_forward(
            self._h, ctypes.c_void_p(freqs.data_ptr()), ctypes.c_void_p(amps.data_ptr()), batch, K,
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
            _stream_handle(stream)))
        return out

    @staticmethod
    def _observed_ptr(observed):
        import torch
        if observed is None:
            return 0
        if not (isinstance(observed, torch.Tensor) and observed.is_cuda
                and observed.dtype == torch.complex64 and observed.is_contiguous()):
            raise TypeError("observed must be a contiguous CUDA complex64 tensor")
        return observed.data_ptr()

    @staticmethod
    def _counts_ptr(counts, batch):
        import torch
        if counts is None:
            return 0
        if not (isinstance(counts, torch.Tensor) and counts.is_cuda and counts.dtype == torch.int32
                and counts.is_contiguous() and counts.numel() == batch):
            raise TypeError("counts must be a contiguous CUDA int32 tensor of batch elements")
        return counts.data_ptr()

    def model_residual(self, freqs, amps, workspace, observed=None, counts=None, out=None, stream=None):
        """observed - model of the first counts[f] tones of every frame
        (rsft_model_residual): a complex64 tensor in the layout of buckets()
        (flat). observed: default this plan's buckets of the last execute."""
        import torch
        batch, K = self._model_args(freqs, amps)
        if out is None:
            out = torch.empty(self.model_size(batch), dtype=torch.complex64, device="cuda")
        _check(self._lib, self._lib.rsft_model_residual(
            self._h, ctypes.c_void_p(self._observed_ptr(observed)), ctypes.c_void_p(freqs.data_ptr()),
            ctypes.c_void_p(amps.data_ptr()), batch, K, ctypes.c_void_p(self._counts_ptr(counts, batch)),
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(workspace.data_ptr()), _stream_handle(stream)))
        return out

    def model_forward_noalloc(self, freqs, amps, out, stream=None):
        """model_forward into the caller's `out` with the factors in the
        library's static scratch array (no allocation anywhere; the factors
        are not kept for a backward call)."""
        batch, K = self._model_args(freqs, amps)
        _check(self._lib, self._lib.rsft_model_forward_noalloc(
            self._h, ctypes.c_void_p(freqs.data_ptr()), ctypes.c_void_p(amps.data_ptr()), batch, K,
            ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def model_backward(self, amps, grad_model, workspace, steps=False, stream=None):
        """(grad_freqs float64 [batch, K, D], grad_amps complex64 [batch, K])
        for the output gradient grad_model (dL/dRe + j dL/dIm of the model);
        with steps=True also each tone's Gauss-Newton step (step_freqs,
        step_amps) for the loss sum |model - observed|^2, given
        grad_model = 2 (model - observed)."""
        import torch
        batch, K = int(amps.shape[0]), int(amps.shape[1])
        D = len(self.descs[0]["shape"])
        grad_model = grad_model.contiguous()
        gf = torch.empty((batch, K, D), dtype=torch.float64, device="cuda")
        ga = torch.empty((batch, K), dtype=torch.complex64, device="cuda")
        sf = torch.empty((batch, K, D), dtype=torch.float64, device="cuda") if steps else None
        sa = torch.empty((batch, K), dtype=torch.complex64, device="cuda") if steps else None
        _check(self._lib, self._lib.rsft_model_backward(
            self._h, ctypes.c_void_p(amps.data_ptr()), batch, K,
            ctypes.c_void_p(grad_model.data_ptr()), ctypes.c_void_p(gf.data_ptr()),
            ctypes.c_void_p(ga.data_ptr()), ctypes.c_void_p(sf.data_ptr() if steps else 0),
            ctypes.c_void_p(sa.data_ptr() if steps else 0), ctypes.c_void_p(workspace.data_ptr()),
            _stream_handle(stream)))
        return (gf, ga, sf, sa) if steps else (gf, ga)

    def refine_workspace(self, batch, tones):
        import torch
        n = ctypes.c_int64()
        _check(self._lib, self._lib.rsft_refine_workspace_size(self._h, int(batch), int(tones),
                                                               ctypes.byref(n)))
        return torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")

    def initial_amplitudes(self, freqs, workspace, observed=None, with_spread=False, stream=None):
        """Starting amplitudes (complex64 [batch, K]) of tones at `freqs`
        (float64 [batch, K, D]) from the observed buckets (default: this
        plan's buckets of the last execute); with_spread: also the per-round
        spread (float32 [batch, K])."""
        import torch
        if not (isinstance(freqs, torch.Tensor) and freqs.is_cuda and freqs.dtype == torch.float64
                and freqs.is_contiguous() and freqs.dim() == 3):
            raise TypeError("freqs must be a contiguous CUDA float64 tensor [batch, K, D]")
        batch, K = int(freqs.shape[0]), int(freqs.shape[1])
        amps = torch.empty((batch, K), dtype=torch.complex64, device="cuda")
        spread = torch.empty((batch, K), dtype=torch.float32, device="cuda") if with_spread else None
        obs = self._observed_ptr(observed)
        _check(self._lib, self._lib.rsft_initial_amplitudes(
            self._h, ctypes.c_void_p(obs), ctypes.c_void_p(freqs.data_ptr()), batch, K,
            ctypes.c_void_p(amps.data_ptr()), ctypes.c_void_p(spread.data_ptr() if with_spread else 0),
            ctypes.c_void_p(workspace.data_ptr()), _stream_handle(stream)))
        return (amps, spread) if with_spread else amps

    def refine(self, freqs, amps, steps, workspace, observed=None, trust_bins=0.25, loss=None,
               counts=None, stream=None):
        """rsft_refine in place on freqs (float64 [batch, K, D]) and amps
        (complex64 [batch, K]); loss: None or a float64 CUDA tensor of
        (steps + 1) * batch elements; counts: None or an int32 CUDA tensor
        [batch] of the tones taking part in each frame."""
        batch, K = self._model_args(freqs, amps)
        obs = self._observed_ptr(observed)
        lp = 0 if loss is None else loss.data_ptr()
        cp = self._counts_ptr(counts, batch)
        _check(self._lib, self._lib.rsft_refine(
            self._h, ctypes.c_void_p(obs), ctypes.c_void_p(freqs.data_ptr()),
            ctypes.c_void_p(amps.data_ptr()), batch, K, ctypes.c_void_p(cp), int(steps), float(trust_bins),
            ctypes.c_void_p(workspace.data_ptr()), ctypes.c_void_p(lp), _stream_handle(stream)))
        return freqs, amps

    def set_option(self, option, value):
        _check(self._lib, self._lib.rsft_set_option(self._h, int(option), int(value)))

    def stage_times(self, reset=True):
        """Average device ms per stage over timed executes, and the count."""
        arr = (ctypes.c_double * len(STAGES))()
        cnt = ctypes.c_int64()
        _check(self._lib, self._lib.rsft_stage_times(self._h, arr, ctypes.byref(cnt),
                                                     1 if reset else 0))
        return {name: arr[i] for i, name in enumerate(STAGES)}, cnt.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rsft_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
