"""ctypes binding of libtor.so (the C ABI declared in include/tor.h).

Argument marshalling only: every step of the Torontonian runs in the HIP
library.  If ``libtor.so`` is missing or cannot be loaded this module raises;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtor.so")

TOR_OK = 0
TOR_PENDING = 1
TOR_E_INVAL = -1
TOR_E_NOT_PD = -2
TOR_E_NUMERIC = -3
TOR_E_BUSY = -4
TOR_E_NOMEM = -5
TOR_E_DEVICE = -6
TOR_E_TIMEOUT = -7
TOR_E_UNKNOWN = -8
TOR_E_SCRATCH = -9

TOR_ACCUM_DD = 0
TOR_ACCUM_FP64 = 1

TOR_INPUT_DEVICE = 0x1
TOR_CHECK_HERMITIAN = 0x2
TOR_FORCE_COMPLEX = 0x4
TOR_FACTOR_DD = 0x8
TOR_OUTPUT_DEVICE = 0x10

TOR_CLICK_ALL_MAX_M = 32  # the most modes tor_click_all takes

# every symbol include/tor.h declares
EXPORTS = [
    "tor_default_options", "tor_create", "tor_destroy", "tor_workspace_size", "tor_eval",
    "tor_eval_batch", "tor_eval_plain", "tor_eval_partials", "tor_submit", "tor_poll",
    "tor_drain", "tor_debug_math", "tor_debug_fma_peak", "tor_strerror", "tor_autotune", "tor_tune_save", "tor_tune_load",
    "tor_serve_config", "tor_click_probs", "tor_eval_removal", "tor_eval_static", "tor_debug_fail_root",
    "tor_click_all", "tor_debug_zeta",
]

TOR_TUNE_REAL = 0x1
TOR_TUNE_COMPLEX = 0x2
TOR_TUNE_QUAD = 0x4


class tor_options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("max_n", ctypes.c_int),
        ("split_k", ctypes.c_int),
        ("waves_per_cu", ctypes.c_int),
        ("accum", ctypes.c_int),
        ("flags", ctypes.c_uint),
    ]


class tor_result(ctypes.Structure):
    _fields_ = [
        ("tor", ctypes.c_double),
        ("tor_lo", ctypes.c_double),
        ("sum_abs", ctypes.c_double),
        ("err_est", ctypes.c_double),
        ("subsets", ctypes.c_ulonglong),
        ("status", ctypes.c_int),
        ("path", ctypes.c_int),
        ("device_ms", ctypes.c_float),
        ("launches", ctypes.c_int),
    ]


# the same layout as a numpy record, to read an array of results at once
_RESULT_DTYPE = np.dtype({
    "names": [f[0] for f in tor_result._fields_],
    "formats": ["<f8", "<f8", "<f8", "<f8", "<u8", "<i4", "<i4", "<f4", "<i4"],
    "offsets": [getattr(tor_result, f[0]).offset for f in tor_result._fields_],
    "itemsize": ctypes.sizeof(tor_result),
})

_lib = None


def _torch_runtime_first():
    """torch ships its own HIP runtime under the soname libtor links against
    (libamdhip64.so.7), and whichever copy is loaded first serves the whole
    process.  torch initialised after libtor was loaded reports no GPU, while
    the other order works; so when torch is importable and sees a GPU it is
    initialised before libtor is loaded."""
    try:
        import torch
    except ImportError:
        return
    try:
        if torch.cuda.device_count() > 0:
            torch.cuda.init()
    except RuntimeError:
        pass


def load(path: str = LIB_PATH):
    """Load libtor.so and declare the signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtor.so not built at {path}; run __graft_entry__.build() or "
                          "python -m paper_2109_04528_amd.build")
    _torch_runtime_first()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.tor_default_options.argtypes = [P(tor_options)]
    lib.tor_default_options.restype = None
    lib.tor_create.argtypes = [P(ctypes.c_void_p), P(tor_options)]
    lib.tor_create.restype = ctypes.c_int
    lib.tor_destroy.argtypes = [ctypes.c_void_p]
    lib.tor_destroy.restype = None
    lib.tor_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.tor_workspace_size.restype = ctypes.c_size_t
    lib.tor_eval.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long, P(tor_result)]
    lib.tor_eval.restype = ctypes.c_int
    lib.tor_eval_static.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long, P(tor_result)]
    lib.tor_eval_static.restype = ctypes.c_int
    lib.tor_eval_batch.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_void_p),
                                   P(ctypes.c_long), P(tor_result)]
    lib.tor_eval_batch.restype = ctypes.c_int
    lib.tor_eval_plain.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long,
                                   ctypes.c_ulonglong, ctypes.c_ulonglong, P(tor_result)]
    lib.tor_eval_plain.restype = ctypes.c_int
    lib.tor_eval_partials.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long,
                                      ctypes.c_int, P(ctypes.c_int), P(ctypes.c_double), P(tor_result)]
    lib.tor_eval_partials.restype = ctypes.c_int
    lib.tor_submit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long,
                               P(ctypes.c_ulonglong)]
    lib.tor_submit.restype = ctypes.c_int
    lib.tor_poll.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong, P(tor_result)]
    lib.tor_poll.restype = ctypes.c_int
    lib.tor_drain.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.tor_drain.restype = ctypes.c_int
    lib.tor_debug_math.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]
    lib.tor_debug_math.restype = ctypes.c_int
    lib.tor_debug_fma_peak.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_float)]
    lib.tor_debug_fma_peak.restype = ctypes.c_int
    lib.tor_debug_fail_root.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int]
    lib.tor_debug_fail_root.restype = ctypes.c_int
    lib.tor_serve_config.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_longlong, ctypes.c_double,
                                     ctypes.c_int]
    lib.tor_serve_config.restype = ctypes.c_int
    lib.tor_click_probs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long, ctypes.c_int,
                                    P(ctypes.c_ulonglong), P(ctypes.c_double), ctypes.c_void_p]
    lib.tor_click_probs.restype = ctypes.c_int
    DP = P(ctypes.c_double)
    lib.tor_click_all.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long, DP, DP, DP,
                                  ctypes.c_void_p]
    lib.tor_click_all.restype = ctypes.c_int
    lib.tor_debug_zeta.argtypes = [ctypes.c_void_p, ctypes.c_int, DP, DP, DP]
    lib.tor_debug_zeta.restype = ctypes.c_int
    lib.tor_eval_removal.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long, P(tor_result)]
    lib.tor_eval_removal.restype = ctypes.c_int
    lib.tor_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    lib.tor_autotune.restype = ctypes.c_int
    lib.tor_tune_save.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    lib.tor_tune_save.restype = ctypes.c_int
    lib.tor_tune_load.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    lib.tor_tune_load.restype = ctypes.c_int
    lib.tor_strerror.argtypes = [ctypes.c_int]
    lib.tor_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


class TorError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().tor_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


@dataclass
class TorResult:
    tor: float
    tor_lo: float
    sum_abs: float
    err_est: float
    subsets: int
    status: int
    path: int
    device_ms: float
    launches: int = 1

    @property
    def value(self) -> float:
        return self.tor + self.tor_lo

    @property
    def cancellation(self) -> float:
        v = abs(self.tor)
        return float("inf") if v == 0 else self.sum_abs / v

    @classmethod
    def from_c(cls, r: tor_result) -> "TorResult":
        return cls(r.tor, r.tor_lo, r.sum_abs, r.err_est, int(r.subsets), r.status, r.path, r.device_ms,
                   r.launches)


def _results(res, cnt: int) -> List["TorResult"]:
    """TorResults of a tor_result array, read through one structured view."""
    a = np.frombuffer(res, dtype=_RESULT_DTYPE, count=cnt)
    return [TorResult(*row) for row in a.tolist()]


def _host_c128(O) -> np.ndarray:
    """Marshal O (numpy array or torch tensor) to a contiguous host complex128 array."""
    if (type(O) is np.ndarray and O.dtype == np.complex128 and O.ndim == 2 and O.flags.c_contiguous
            and O.shape[0] == O.shape[1] and O.shape[0] % 2 == 0):
        return O  # already in the form the library reads
    try:
        import torch  # noqa: F401
        if hasattr(O, "detach") and hasattr(O, "device"):
            O = O.detach()
            if O.device.type != "cpu":
                O = O.cpu()
            O = O.numpy()
    except ImportError:
        pass
    A = np.ascontiguousarray(np.asarray(O, dtype=np.complex128))
    if A.ndim != 2 or A.shape[0] != A.shape[1] or A.shape[0] % 2:
        raise ValueError("O must be a 2n x 2n matrix")
    return A


def _dev_c128(O):
    """A device matrix for a context with TOR_INPUT_DEVICE: a torch complex128
    CUDA tensor, 2n x 2n, unit column stride.  Returns (pointer, n, ld); the
    caller keeps O alive across the call."""
    if not (hasattr(O, "device") and getattr(O.device, "type", None) == "cuda"):
        raise ValueError("a context with TOR_INPUT_DEVICE takes torch CUDA tensors")
    import torch
    if O.dtype != torch.complex128 or O.dim() != 2 or O.shape[0] != O.shape[1] or O.shape[0] % 2:
        raise ValueError("O must be a 2n x 2n complex128 tensor")
    if O.shape[0] and O.stride(1) != 1:
        raise ValueError("O needs unit column stride")
    return O.data_ptr(), O.shape[0] // 2, max(O.stride(0), 1)


class Context:
    """One libtor context (device state, stream, workspace).  With
    flags & TOR_INPUT_DEVICE every matrix argument is a torch complex128 CUDA
    tensor read in place by the staging kernel; otherwise numpy arrays (or
    tensors, copied to the host)."""

    def __init__(self, device: int = 0, stream=None, max_n: int = 40, split_k: int = 0,
                 waves_per_cu: int = 0, accum: str = "dd", flags: int = 0, workspace=None):
        lib = load()
        opt = tor_options()
        lib.tor_default_options(ctypes.byref(opt))
        opt.device = device
        # a torch stream the library runs on (None: the library's own stream,
        # or a raw handle torch knows nothing of)
        self._torch_stream = stream if hasattr(stream, "wait_stream") else None
        if stream is not None:
            opt.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        if workspace is not None:  # e.g. a torch uint8 tensor on the device
            opt.workspace = ctypes.c_void_p(int(workspace.data_ptr()))
            opt.workspace_bytes = int(workspace.numel() * workspace.element_size())
            self._ws = workspace
        opt.max_n = max_n
        opt.split_k = split_k
        opt.waves_per_cu = waves_per_cu
        opt.accum = TOR_ACCUM_FP64 if accum == "fp64" else TOR_ACCUM_DD
        opt.flags = flags
        h = ctypes.c_void_p()
        rc = lib.tor_create(ctypes.byref(h), ctypes.byref(opt))
        if rc != TOR_OK:
            raise TorError(rc, "tor_create")
        self._h = h
        self._lib = lib
        self._device_in = bool(flags & TOR_INPUT_DEVICE)
        self._flags = flags
        self._device = device

    def _after_torch_writes(self, O):
        """Order the library's reads of a device tensor after the work torch
        has queued on its current stream (which may still be writing O): the
        library's stream waits for it on the device when it is a torch
        stream, else the host waits for torch's stream to finish."""
        import torch
        cur = torch.cuda.current_stream(O.device)
        if self._torch_stream is None:
            cur.synchronize()
        elif self._torch_stream != cur:
            self._torch_stream.wait_stream(cur)

    def _in(self, O):
        """(pointer, n, ld, keep-alive) of a matrix argument."""
        if self._device_in:
            ptr, n, ld = _dev_c128(O)
            if n:
                self._after_torch_writes(O)
            return (ptr if n else None), n, ld, O
        A = _host_c128(O)
        n = A.shape[0] // 2
        return (A.__array_interface__["data"][0] if n else None), n, max(2 * n, 1), A

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tor_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, O, check: bool = True) -> TorResult:
        ptr, n, ld, _keep = self._in(O)
        r = tor_result()
        rc = self._lib.tor_eval(self._h, n, ptr, ld, ctypes.byref(r))
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_eval")
        return TorResult.from_c(r)

    def eval_static(self, O, check: bool = True) -> TorResult:
        """tor_eval without any allocation (the library's static device
        array; see tor_eval_static in include/tor.h)."""
        ptr, n, ld, _keep = self._in(O)
        r = tor_result()
        rc = self._lib.tor_eval_static(self._h, n, ptr, ld, ctypes.byref(r))
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_eval_static")
        return TorResult.from_c(r)

    def eval_batch(self, Os: Sequence, check: bool = True) -> List[TorResult]:
        args = [self._in(O) for O in Os]
        cnt = len(args)
        ns = (ctypes.c_int * cnt)(*[a[1] for a in args])
        ptrs = (ctypes.c_void_p * cnt)(*[a[0] for a in args])
        lds = (ctypes.c_long * cnt)(*[a[2] for a in args])
        res = (tor_result * cnt)()
        rc = self._lib.tor_eval_batch(self._h, cnt, ns, ptrs, lds, res)
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_eval_batch")
        return _results(res, cnt)

    def eval_plain(self, O, mask_begin: int = 0, mask_end: Optional[int] = None,
                   check: bool = True) -> TorResult:
        ptr, n, ld, _keep = self._in(O)
        if mask_end is None:
            mask_end = 1 << n
        r = tor_result()
        rc = self._lib.tor_eval_plain(self._h, n, ptr, ld, mask_begin, mask_end, ctypes.byref(r))
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_eval_plain")
        return TorResult.from_c(r)

    def eval_removal(self, O, check: bool = True) -> TorResult:
        """The paper's removal-order algorithm (comparison kernel)."""
        ptr, n, ld, _keep = self._in(O)
        r = tor_result()
        rc = self._lib.tor_eval_removal(self._h, n, ptr, ld, ctypes.byref(r))
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_eval_removal")
        return TorResult.from_c(r)

    def eval_partials(self, O, k_max: int):
        ptr, n, ld, _keep = self._in(O)
        parts = np.zeros(3 * (1 << k_max), dtype=np.float64)
        k = ctypes.c_int()
        r = tor_result()
        rc = self._lib.tor_eval_partials(self._h, n, ptr, ld, k_max,
                                         ctypes.byref(k), parts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.byref(r))
        if rc != TOR_OK:
            raise TorError(rc, "tor_eval_partials")
        return k.value, parts[: 3 * (1 << k.value)].reshape(-1, 3), TorResult.from_c(r)

    def click_probs(self, O, patterns, check: bool = True):
        """Click probabilities p(S) = Tor(O_S) sqrt(det(I - O)) of an M-mode
        state for each pattern: an int bitmask (bit q = mode q clicked) or an
        iterable of clicked modes.  Returns (probs, [TorResult of O_S])."""
        ptr, M, ld, _keep = self._in(O)
        masks = []
        for p in patterns:
            if isinstance(p, (int, np.integer)):
                masks.append(int(p))
            else:
                m = 0
                for q in p:
                    m |= 1 << int(q)
                masks.append(m)
        cnt = len(masks)
        pat = (ctypes.c_ulonglong * max(cnt, 1))(*masks)
        probs = np.zeros(max(cnt, 1), dtype=np.float64)
        res = (tor_result * max(cnt, 1))()
        rc = self._lib.tor_click_probs(self._h, M, ptr, ld, cnt, pat,
                                       probs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.cast(res, ctypes.c_void_p))
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_click_probs")
        return probs[:cnt], [TorResult.from_c(res[i]) for i in range(cnt)]

    def click_all(self, O, probs: bool = True, tor: bool = False, check: bool = True):
        """Click probabilities of every pattern of the M-mode state at once
        (tor_click_all): p[S] for every bitmask S < 2^M, the subset
        determinants shared by all patterns.  Returns (probs or None,
        (tor_hi, tor_lo) or None, TorResult of the whole state)."""
        ptr, M, ld, _keep = self._in(O)
        n = 1 << M
        dp = ctypes.POINTER(ctypes.c_double)
        if self._flags & TOR_OUTPUT_DEVICE:
            # torch tensors on the context's device, written on its stream
            import torch
            dev = torch.device("cuda", self._device)
            mk = lambda: torch.empty(n, dtype=torch.float64, device=dev)
            at = lambda a: ctypes.cast(ctypes.c_void_p(a.data_ptr()), dp)
            # the new tensors' memory may still be read by work torch has
            # queued: order the library's writes after it
            cur = torch.cuda.current_stream(dev)
            if self._torch_stream is None:
                cur.synchronize()
            elif self._torch_stream != cur:
                self._torch_stream.wait_stream(cur)
        else:
            mk = lambda: np.empty(n, dtype=np.float64)
            at = lambda a: a.ctypes.data_as(dp)
        p = mk() if probs else None
        th = mk() if tor else None
        tl = mk() if tor else None
        r = tor_result()
        nul = ctypes.cast(None, dp)
        rc = self._lib.tor_click_all(self._h, M, ptr, ld,
                                     at(p) if probs else nul,
                                     at(th) if tor else nul,
                                     at(tl) if tor else nul,
                                     ctypes.cast(ctypes.byref(r), ctypes.c_void_p))
        if check and rc != TOR_OK:
            raise TorError(rc, "tor_click_all")
        return p, ((th, tl) if tor else None), TorResult.from_c(r)

    def debug_zeta(self, t):
        """The subset-sum transform of click_all on 2^nbits host doubles:
        (g_hi, g_lo) with g[S] = sum over Z subset of S of t[Z]."""
        t = np.ascontiguousarray(t, dtype=np.float64)
        nbits = int(t.size).bit_length() - 1
        if t.size != 1 << nbits:
            raise ValueError("the number of terms must be a power of two")
        gh = np.empty_like(t)
        gl = np.empty_like(t)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.tor_debug_zeta(self._h, nbits, t.ctypes.data_as(dp), gh.ctypes.data_as(dp),
                                      gl.ctypes.data_as(dp))
        if rc != TOR_OK:
            raise TorError(rc, "tor_debug_zeta")
        return gh, gl

    def submit(self, O) -> int:
        ptr, n, ld, _keep = self._in(O)
        t = ctypes.c_ulonglong()
        rc = self._lib.tor_submit(self._h, n, ptr, ld, ctypes.byref(t))
        if rc != TOR_OK:
            raise TorError(rc, "tor_submit")
        return t.value

    def poll(self, ticket: int) -> Optional[TorResult]:
        r = tor_result()
        rc = self._lib.tor_poll(self._h, ticket, ctypes.byref(r))
        if rc == TOR_PENDING:
            return None
        if rc != TOR_OK:
            raise TorError(rc, "tor_poll")
        return TorResult.from_c(r)

    def drain(self, timeout_ms: int = -1) -> None:
        rc = self._lib.tor_drain(self._h, timeout_ms)
        if rc != TOR_OK:
            raise TorError(rc, "tor_drain")

    def serve_config(self, chunk_subsets: int = 1 << 30, oldest_share: float = 0.5,
                     max_queue: int = 1 << 16, express_subsets: int = 1 << 24) -> None:
        rc = self._lib.tor_serve_config(self._h, chunk_subsets, express_subsets, oldest_share, max_queue)
        if rc != TOR_OK:
            raise TorError(rc, "tor_serve_config")

    def autotune(self, n_min: int, n_max: int, paths: int = TOR_TUNE_REAL | TOR_TUNE_COMPLEX) -> None:
        rc = self._lib.tor_autotune(self._h, n_min, n_max, paths)
        if rc != TOR_OK:
            raise TorError(rc, "tor_autotune")

    def save_tuning(self, path: str) -> None:
        rc = self._lib.tor_tune_save(self._h, path.encode())
        if rc != TOR_OK:
            raise TorError(rc, "tor_tune_save")

    def load_tuning(self, path: str) -> None:
        rc = self._lib.tor_tune_load(self._h, path.encode())
        if rc != TOR_OK:
            raise TorError(rc, "tor_tune_load")

    def debug_math(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(4 * x.size, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.tor_debug_math(self._h, x.size, x.ctypes.data_as(dp), out.ctypes.data_as(dp))
        if rc != TOR_OK:
            raise TorError(rc, "tor_debug_math")
        return out.reshape(-1, 4)

    def fma_peak(self, iters: int = 4096):
        """Measured FP64 FMA throughput of the device: (TFLOP/s, kernel ms)."""
        tf = ctypes.c_double()
        ms = ctypes.c_float()
        rc = self._lib.tor_debug_fma_peak(self._h, iters, ctypes.byref(tf), ctypes.byref(ms))
        if rc != TOR_OK:
            raise TorError(rc, "tor_debug_fma_peak")
        return tf.value, ms.value

    def debug_fail_root(self, root: int, runs: int = 1):
        """The next synchronous evaluation's first matrix: root `root` reports
        a numeric failure in its first `runs` launches (tor_debug_fail_root)."""
        rc = self._lib.tor_debug_fail_root(self._h, int(root), int(runs))
        if rc != TOR_OK:
            raise TorError(rc, "tor_debug_fail_root")


def workspace_size(max_n: int, split_k: int = 0, max_inflight: int = 1) -> int:
    return int(load().tor_workspace_size(max_n, split_k, max_inflight))
