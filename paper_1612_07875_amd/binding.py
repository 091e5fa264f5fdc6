"""ctypes binding of libdmdstream (see include/dmd_stream.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  torch provides device buffers and streams; it is imported before
the library is loaded so that both share one HIP runtime.  There is no
fallback: if the library is missing or no GPU is present, calls raise.
"""

import ctypes
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmdstream.so")

OK, W_RANK = 0, 1
E_INVAL, E_NOMEM, E_NOT_READY, E_NONFINITE, E_CONVERGENCE, E_DEVICE, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {
    0: "OK", 1: "W_RANK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_NOT_READY",
    -4: "E_NONFINITE", -5: "E_CONVERGENCE", -6: "E_DEVICE", -7: "E_UNSUPPORTED",
}

DTYPES = {"f32": 0, "f64": 1, "c64_csr": 2}
PRECISIONS = {"default": 0, "fp32": 1, "bf16x3": 2, "fp64": 3}
EIG_SOLVERS = {"default": 0, "jacobi": 1, "tridiag": 2}


class DMDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_nnz", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32), ("max_qr_iter", ctypes.c_int32), ("auto_solve", ctypes.c_int32),
        ("rcond", ctypes.c_double), ("tol", ctypes.c_double), ("warm_start", ctypes.c_int32),
        ("max_block", ctypes.c_int32), ("eig_solver", ctypes.c_int32), ("buildup", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 4),
    ]


class BatchOpts(ctypes.Structure):
    _fields_ = [("max_streams", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("reserved", ctypes.c_int32 * 8)]


class Info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int32), ("r", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("count", ctypes.c_int32), ("r_eff", ctypes.c_int32),
        ("sweeps", ctypes.c_int32), ("qr_iters", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
        ("gram_iter", ctypes.c_int32), ("proj_form", ctypes.c_int32),
    ]


class Frame(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("nnz", ctypes.c_int32), ("idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("gram_iter", ctypes.c_int32), ("proj_form", ctypes.c_int32), ("gram_us", ctypes.c_double),
                ("step_us", ctypes.c_double), ("reserved", ctypes.c_int32 * 4)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_DP = ctypes.POINTER(ctypes.c_double)
_I32P = ctypes.POINTER(ctypes.c_int32)

# exported symbol -> argument types (every function returns int unless noted)
SIGNATURES = {
    "dmd_opts_init": [ctypes.POINTER(Opts)],
    "dmd_stream_create": [_I64, _I32, _I32, ctypes.POINTER(Opts), ctypes.POINTER(_P)],
    "dmd_stream_footprint": [_I64, _I32, _I32, ctypes.POINTER(Opts), ctypes.POINTER(_I64)],
    "dmd_stream_destroy": [_P],
    "dmd_stream_sync": [_P],
    "dmd_stream_reset": [_P, _P],
    "dmd_stream_push": [_P, _P, _P],
    "dmd_stream_push_csr": [_P, _I32, _P, _P, _P],
    "dmd_stream_push_block": [_P, _P, _I64, _I32, _P],
    "dmd_stream_block_eigs": [_P, _I32P, _DP, _DP, _DP, _I64, _I32P, _I32P],
    "dmd_stream_block_modes": [_P, _P, _I64, _I64, _P],
    "dmd_stream_solve": [_P, _P],
    "dmd_stream_eigs": [_P, _DP, _DP, _DP, _I32P],
    "dmd_stream_svd": [_P, _DP, _DP, _I64, _I32P],
    "dmd_stream_atilde": [_P, _DP, _I64, _DP, _I64, _I32P],
    "dmd_stream_gram": [_P, _DP, _I64, _I32P],
    "dmd_stream_fourier_setup": [_P, _I32, _I32, _I32],
    "dmd_stream_fourier_support": [_P, _I32P, _I32, _I32P],
    "dmd_stream_push_fourier": [_P, ctypes.c_void_p, _I64, ctypes.c_void_p],
    "dmd_stream_checkpoint_bytes": [_P, ctypes.POINTER(ctypes.c_int64)],
    "dmd_stream_save": [_P, ctypes.c_void_p, _I64],
    "dmd_stream_restore": [_P, ctypes.c_void_p, _I64, ctypes.c_void_p],
    "dmd_stream_modes": [_P, _P, _I64, _P],
    "dmd_stream_pod": [_P, _P, _I64, _P],
    "dmd_stream_amplitudes": [_P, _DP, _DP, _I32P, _I32P],
    "dmd_stream_background": [_P, _P, _P, _P],
    "dmd_stream_load_window": [_P, _P, _I64, _I32, _P],
    "dmd_stream_resync": [_P, _P],
    "dmd_window_gram": [_P, _I64, _I64, _I32, _I32, _I32, _P, _I64, _P],
    "dmd_window_gram_noalloc": [_P, _I64, _I64, _I32, _I32, _I32, _P, _I64, _P],
    "dmd_stream_info": [_P, ctypes.POINTER(Info)],
    "dmd_tune": [_I64, _I32, _I32, ctypes.POINTER(Opts), ctypes.POINTER(Tuning), _P],
    "dmd_tune_lookup": [_I64, _I32, _I32, ctypes.POINTER(Opts), ctypes.POINTER(Tuning)],
    "dmd_tune_save": [ctypes.c_char_p],
    "dmd_tune_load": [ctypes.c_char_p],
    "dmd_tune_clear": [],
    "dmd_batch_opts_init": [ctypes.POINTER(BatchOpts)],
    "dmd_batch_create": [ctypes.POINTER(BatchOpts), ctypes.POINTER(_P)],
    "dmd_batch_destroy": [_P],
    "dmd_batch_attach": [_P, _P],
    "dmd_batch_detach": [_P, _P],
    "dmd_batch_tick": [_P, _I32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                       ctypes.POINTER(_I64), _P],
    "dmd_batch_tick_frames": [_P, _I32, ctypes.POINTER(_P), ctypes.POINTER(Frame), ctypes.POINTER(_P),
                              ctypes.POINTER(_I64), _P],
    "dmd_batch_info": [_P, _I32P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
    "dmd_profile_enable": [ctypes.c_int],
    "dmd_profile_reset": [],
    "dmd_profile_read": [ctypes.c_char_p, ctypes.POINTER(_I64), _DP],
}
STRING_FUNCS = ["dmd_last_error", "dmd_version"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the shared library once and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1612_07875_amd.build`")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in STRING_FUNCS:
        fn = getattr(lib, name)
        fn.argtypes = []
        fn.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().dmd_last_error().decode()


def check(rc: int) -> int:
    if rc < 0:
        raise DMDError(rc, last_error())
    return rc


def profile_enable(on: bool = True) -> None:
    check(load().dmd_profile_enable(1 if on else 0))


def profile_reset() -> None:
    check(load().dmd_profile_reset())


def profile_read(kernel: str):
    """(launches, total milliseconds) of one kernel since the last reset."""
    cnt = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    check(load().dmd_profile_read(kernel.encode(), ctypes.byref(cnt), ctypes.byref(ms)))
    return cnt.value, ms.value


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_DP)


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def make_opts(dtype: str = "f32", precision: str = "default", auto_solve: bool = True,
              rcond: Optional[float] = None, tol: float = 0.0, max_nnz: int = 0, max_sweeps: int = 0,
              max_qr_iter: int = 0, warm_start: bool = False, max_block: int = 1,
              eig_solver: str = "default", buildup: bool = False) -> Opts:
    """dmd_opts_t from keyword options (defaults from dmd_opts_init)."""
    o = Opts()
    check(load().dmd_opts_init(ctypes.byref(o)))
    o.dtype = DTYPES[dtype]
    o.precision = PRECISIONS[precision]
    o.max_nnz = max_nnz
    o.max_sweeps = max_sweeps
    o.max_qr_iter = max_qr_iter
    o.auto_solve = 1 if auto_solve else 0
    o.rcond = -1.0 if rcond is None else float(rcond)
    o.tol = float(tol)
    o.warm_start = 1 if warm_start else 0
    o.max_block = int(max_block)
    o.eig_solver = EIG_SOLVERS[eig_solver]
    o.buildup = 1 if buildup else 0
    return o


def footprint(n: int, m: int, r: int, **opts) -> int:
    """Device bytes a Stream(n, m, r, **opts) would allocate (nothing is allocated)."""
    b = ctypes.c_int64(0)
    check(load().dmd_stream_footprint(int(n), int(m), int(r), ctypes.byref(make_opts(**opts)), ctypes.byref(b)))
    return int(b.value)


def window_gram(X: torch.Tensor, precision: str = "default", out: Optional[torch.Tensor] = None,
                stream=None, noalloc: bool = False) -> torch.Tensor:
    """G = X^* X (FP64, k x k on the device) of the columns of X, given as a
    (k, n) CUDA tensor whose rows are the snapshots (column-major n x k).
    noalloc: call dmd_window_gram_noalloc (the library's fixed scratch instead
    of a stream-ordered allocation); pass `out` as well for a call that
    allocates nothing at all."""
    if not (X.is_cuda and X.dim() == 2 and X.stride(1) == 1 and X.dtype in (torch.float32, torch.float64)):
        raise ValueError("X must be a (k, n) float32/float64 CUDA tensor with unit stride along n")
    k = X.shape[0]
    if out is None:
        out = torch.empty((k, k), dtype=torch.float64, device=X.device)
    if not (out.is_cuda and out.dtype == torch.float64 and out.dim() == 2 and out.stride(1) == 1
            and out.shape[0] >= k and out.shape[1] >= k):
        raise ValueError("out must be a float64 CUDA tensor of at least k x k with unit inner stride")
    dt = DTYPES["f32"] if X.dtype == torch.float32 else DTYPES["f64"]
    # out is row-major (k, ldg): read as column-major it is G^T = G
    fn = load().dmd_window_gram_noalloc if noalloc else load().dmd_window_gram
    check(fn(X.data_ptr(), X.stride(0), X.shape[1], k, dt, PRECISIONS[precision], out.data_ptr(), out.stride(0),
             _stream_ptr(stream)))
    return out


def _tuning_dict(t: Tuning) -> dict:
    return {"gram_iter": int(t.gram_iter), "proj_form": int(t.proj_form), "gram_us": float(t.gram_us),
            "step_us": float(t.step_us)}


def tune(n: int, m: int, r: int, stream=None, **opts) -> dict:
    """Measure and record the launch shapes of streams of shape (n, m, r, **opts)
    (see dmd_tune); streams created afterwards with that shape use them."""
    t = Tuning()
    check(load().dmd_tune(int(n), int(m), int(r), ctypes.byref(make_opts(**opts)), ctypes.byref(t),
                          _stream_ptr(stream)))
    return _tuning_dict(t)


def tune_lookup(n: int, m: int, r: int, **opts) -> Optional[dict]:
    """The tuning table's entry for this shape, or None."""
    t = Tuning()
    rc = load().dmd_tune_lookup(int(n), int(m), int(r), ctypes.byref(make_opts(**opts)), ctypes.byref(t))
    if rc == E_NOT_READY:
        return None
    check(rc)
    return _tuning_dict(t)


def tune_save(path: str) -> None:
    check(load().dmd_tune_save(os.fsencode(path)))


def tune_load(path: str) -> None:
    check(load().dmd_tune_load(os.fsencode(path)))


def tune_clear() -> None:
    check(load().dmd_tune_clear())


class Stream:
    """One streaming-DMD window on the current GPU (see dmd_stream_create)."""

    def __init__(self, n: int, m: int, r: int, dtype: str = "f32", precision: str = "default",
                 auto_solve: bool = True, rcond: Optional[float] = None, tol: float = 0.0,
                 max_nnz: int = 0, max_sweeps: int = 0, max_qr_iter: int = 0, warm_start: bool = False,
                 max_block: int = 1, eig_solver: str = "default", buildup: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("libdmdstream needs a HIP GPU; none is available")
        lib = load()
        o = make_opts(dtype=dtype, precision=precision, auto_solve=auto_solve, rcond=rcond, tol=tol,
                      max_nnz=max_nnz, max_sweeps=max_sweeps, max_qr_iter=max_qr_iter, warm_start=warm_start,
                      max_block=max_block, eig_solver=eig_solver, buildup=buildup)
        h = _P()
        check(lib.dmd_stream_create(int(n), int(m), int(r), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.n, self.m, self.r = int(n), int(m), int(r)
        self.max_block = int(max_block)
        self.dtype = dtype
        self.precision = precision
        self.elem = {"f32": torch.float32, "f64": torch.float64, "c64_csr": torch.complex64}[dtype]
        wide = dtype == "f64" or precision == "fp64"
        self.mode_dtype = torch.complex128 if wide else torch.complex64
        self.pod_dtype = (torch.float64 if wide else torch.float32) if dtype != "c64_csr" else self.mode_dtype

    # ---------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            load().dmd_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def sync(self) -> int:
        return check(load().dmd_stream_sync(self._h))

    def reset(self, stream=None):
        check(load().dmd_stream_reset(self._h, _stream_ptr(stream)))

    def info(self) -> Info:
        inf = Info()
        check(load().dmd_stream_info(self._h, ctypes.byref(inf)))
        return inf

    # ---------------------------------------------------------------- ingest
    def push(self, x: torch.Tensor, stream=None) -> int:
        """x: contiguous tensor of n elements on the GPU or in host memory
        (host data is staged on the device by the library)."""
        if not (x.dtype == self.elem and x.numel() == self.n and x.is_contiguous()):
            raise ValueError(f"snapshot must be a contiguous {self.elem} tensor of {self.n} elements")
        return check(load().dmd_stream_push(self._h, x.data_ptr(), _stream_ptr(stream)))

    def push_csr(self, idx: torch.Tensor, val: torch.Tensor, stream=None) -> int:
        if not (idx.dtype == torch.int32 and val.dtype == torch.complex64
                and idx.numel() == val.numel() and idx.is_contiguous() and val.is_contiguous()):
            raise ValueError("idx must be int32 and val complex64, contiguous tensors of equal length")
        return check(load().dmd_stream_push_csr(self._h, idx.numel(), idx.data_ptr(), val.data_ptr(),
                                                _stream_ptr(stream)))

    def push_block(self, X: torch.Tensor, stream=None) -> int:
        """X: (k, n) tensor whose rows are snapshots (column-major n x k)."""
        if not (X.is_cuda and X.dtype == self.elem and X.dim() == 2 and X.shape[1] == self.n
                and X.stride(1) == 1):
            raise ValueError("X must be a (k, n) CUDA tensor with unit stride along n")
        return check(load().dmd_stream_push_block(self._h, X.data_ptr(), X.stride(0), X.shape[0],
                                                  _stream_ptr(stream)))

    def block_eigs(self):
        """Per window of the latest block push: list of (status, lambda complex128[r_eff],
        sigma float64[r_eff]); the last entry is the current window.  Also returns the
        call's own status (that of the current window)."""
        kb = self.max_block
        re = np.zeros((kb, self.r))
        im = np.zeros((kb, self.r))
        sg = np.zeros((kb, self.r))
        reff = np.zeros(kb, dtype=np.int32)
        stat = np.zeros(kb, dtype=np.int32)
        k = ctypes.c_int32(0)
        rc = check(load().dmd_stream_block_eigs(self._h, ctypes.byref(k), _dp(re), _dp(im), _dp(sg), self.r,
                                                reff.ctypes.data_as(_I32P), stat.ctypes.data_as(_I32P)))
        out = []
        for w in range(k.value):
            q = int(reff[w])
            out.append((int(stat[w]), re[w, :q] + 1j * im[w, :q], sg[w, :q].copy()))
        return out, rc

    def block_modes(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Phi of every window of the latest block push: a (max_block, r, n) tensor whose
        [w].T is window w's n x r modes (first r_eff[w] columns written)."""
        if out is None:
            out = torch.zeros((self.max_block, self.r, self.n), dtype=self.mode_dtype, device="cuda")
        if not (out.is_cuda and out.dtype == self.mode_dtype and out.dim() == 3 and out.shape[2] == self.n
                and out.shape[1] >= self.r and out.stride(2) == 1):
            raise ValueError("output must be a (k, >= r, n) CUDA tensor with unit stride along n")
        check(load().dmd_stream_block_modes(self._h, out.data_ptr(), out.stride(1), out.stride(0),
                                            _stream_ptr(stream)))
        return out

    def load_window(self, X: torch.Tensor, stream=None) -> int:
        if not (X.is_cuda and X.dtype == self.elem and X.dim() == 2 and X.shape[1] == self.n
                and X.stride(1) == 1):
            raise ValueError("X must be a (k, n) CUDA tensor with unit stride along n")
        return check(load().dmd_stream_load_window(self._h, X.data_ptr(), X.stride(0), X.shape[0],
                                                   _stream_ptr(stream)))

    def resync(self, stream=None) -> int:
        return check(load().dmd_stream_resync(self._h, _stream_ptr(stream)))

    # ---------------------------------------------------------------- small solves
    def solve(self, stream=None) -> int:
        return check(load().dmd_stream_solve(self._h, _stream_ptr(stream)))

    def eigs(self):
        """(lambda complex128[r_eff], sigma float64[r_eff], status)."""
        re = np.zeros(self.r)
        im = np.zeros(self.r)
        sg = np.zeros(self.r)
        k = ctypes.c_int32(0)
        rc = check(load().dmd_stream_eigs(self._h, _dp(re), _dp(im), _dp(sg), ctypes.byref(k)))
        k = k.value
        return re[:k] + 1j * im[:k], sg[:k], rc

    def svd(self):
        """(sigma float64[m], V[m, r_eff] (complex128 for sparse streams), status)."""
        cw = 2 if self.dtype == "c64_csr" else 1
        sg = np.zeros(self.m)
        V = np.zeros((self.r, self.m * cw))
        k = ctypes.c_int32(0)
        rc = check(load().dmd_stream_svd(self._h, _dp(sg), _dp(V), self.m, ctypes.byref(k)))
        k = k.value
        V = V[:k]
        V = (V[:, 0::2] + 1j * V[:, 1::2]) if cw == 2 else V
        return sg, np.ascontiguousarray(V.T), rc

    def atilde(self):
        """(Atilde[r_eff, r_eff], W[r_eff, r_eff] complex128, status)."""
        cw = 2 if self.dtype == "c64_csr" else 1
        At = np.zeros((self.r, self.r * cw))
        W = np.zeros((self.r, self.r * 2))
        k = ctypes.c_int32(0)
        rc = check(load().dmd_stream_atilde(self._h, _dp(At), self.r, _dp(W), self.r, ctypes.byref(k)))
        k = k.value
        At = At[:k, : k * cw]
        At = (At[:, 0::2] + 1j * At[:, 1::2]) if cw == 2 else At
        W = W[:k, : 2 * k]
        W = W[:, 0::2] + 1j * W[:, 1::2]
        return np.ascontiguousarray(At.T), np.ascontiguousarray(W.T), rc

    def gram(self) -> np.ndarray:
        """Gram of the current window in window order (count x count)."""
        cw = 2 if self.dtype == "c64_csr" else 1
        ld = self.m + 1
        G = np.zeros((ld, ld * cw))
        k = ctypes.c_int32(0)
        check(load().dmd_stream_gram(self._h, _dp(G), ld, ctypes.byref(k)))
        k = k.value
        G = G[:k, : k * cw]
        G = (G[:, 0::2] + 1j * G[:, 1::2]) if cw == 2 else G
        return np.ascontiguousarray(G.T)

    # ---------------------------------------------------------------- Fourier ingest (Sec. 3.5)
    def fourier_setup(self, height: int, width: int, nkeep: int) -> None:
        """Sparse streams: ingest height x width spatial frames as their nkeep lowest-|k| DFT coefficients."""
        check(load().dmd_stream_fourier_setup(self._h, int(height), int(width), int(nkeep)))
        self.fourier_shape = (int(height), int(width))

    def fourier_support(self) -> np.ndarray:
        k = ctypes.c_int32(0)
        check(load().dmd_stream_fourier_support(self._h, None, 0, ctypes.byref(k)))
        idx = np.zeros(k.value, dtype=np.int32)
        check(load().dmd_stream_fourier_support(self._h, idx.ctypes.data_as(_I32P), k.value, ctypes.byref(k)))
        return idx

    def push_fourier(self, frame: torch.Tensor, stream=None) -> int:
        """frame: (height, width) float32 CUDA tensor (rows may be strided)."""
        assert frame.is_cuda and frame.dtype == torch.float32 and frame.dim() == 2 and frame.stride(1) == 1
        return check(load().dmd_stream_push_fourier(self._h, ctypes.c_void_p(frame.data_ptr()),
                                                   frame.stride(0), _stream_ptr(stream)))

    # ---------------------------------------------------------------- checkpoint / resume
    def save(self) -> bytes:
        """Checkpoint of the window (snapshots, Gram, counters) as bytes."""
        lib = load()
        nb = ctypes.c_int64(0)
        check(lib.dmd_stream_checkpoint_bytes(self._h, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        check(lib.dmd_stream_save(self._h, buf, nb.value))
        return buf.raw

    def restore(self, blob: bytes, stream=None) -> int:
        """Replace the window by a checkpoint from save() of a stream of the same shape."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        return check(load().dmd_stream_restore(self._h, buf, len(blob), _stream_ptr(stream)))

    # ---------------------------------------------------------------- projections
    def modes(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Phi (n x r) on the device; the first r_eff columns are written."""
        if out is None:
            out = torch.zeros((self.r, self.n), dtype=self.mode_dtype, device="cuda").T
        self._check_out(out, self.mode_dtype)
        check(load().dmd_stream_modes(self._h, out.data_ptr(), out.stride(1), _stream_ptr(stream)))
        return out

    def pod(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """U (n x r) on the device; the first r_eff columns are written."""
        if out is None:
            out = torch.zeros((self.r, self.n), dtype=self.pod_dtype, device="cuda").T
        self._check_out(out, self.pod_dtype)
        check(load().dmd_stream_pod(self._h, out.data_ptr(), out.stride(1), _stream_ptr(stream)))
        return out

    def amplitudes(self):
        """(b complex128[r_eff], background index, status) of the latest solve."""
        re = np.zeros(self.r)
        im = np.zeros(self.r)
        idx = ctypes.c_int32(-1)
        k = ctypes.c_int32(0)
        rc = check(load().dmd_stream_amplitudes(self._h, _dp(re), _dp(im), ctypes.byref(idx), ctypes.byref(k)))
        k = k.value
        return re[:k] + 1j * im[:k], idx.value, rc

    def background(self, fg: Optional[torch.Tensor] = None, bg: Optional[torch.Tensor] = None,
                   want_bg: bool = True, stream=None):
        """Foreground and background magnitude (n values each, device) of the newest snapshot."""
        if fg is None:
            fg = torch.zeros(self.n, dtype=self.pod_dtype, device="cuda")
        if bg is None and want_bg:
            bg = torch.zeros(self.n, dtype=self.pod_dtype, device="cuda")
        for t in (fg, bg):
            if t is not None and not (t.is_cuda and t.dtype == self.pod_dtype and t.numel() == self.n
                                      and t.is_contiguous()):
                raise ValueError(f"outputs must be contiguous {self.pod_dtype} CUDA tensors of n elements")
        check(load().dmd_stream_background(self._h, fg.data_ptr(), bg.data_ptr() if bg is not None else None,
                                           _stream_ptr(stream)))
        return fg, bg

    def _check_out(self, out: torch.Tensor, dt):
        if not (out.is_cuda and out.dtype == dt and out.dim() == 2 and out.shape[0] == self.n
                and out.shape[1] >= self.r and out.stride(0) == 1):
            raise ValueError(f"output must be an (n, >= r) column-major CUDA tensor of {dt}")


class Batch:
    """Many streams advanced together (see dmd_batch_create / dmd_batch_tick)."""

    def __init__(self, max_streams: int = 256, hbm_budget: int = 0, graphs: int = 0):
        """graphs > 0 replays each tick as one HIP graph launch, keeping up to
        that many captured tick shapes."""
        if not torch.cuda.is_available():
            raise RuntimeError("libdmdstream needs a HIP GPU; none is available")
        lib = load()
        o = BatchOpts()
        check(lib.dmd_batch_opts_init(ctypes.byref(o)))
        o.max_streams = int(max_streams)
        o.hbm_budget = int(hbm_budget)
        o.graphs = int(graphs)
        h = _P()
        check(lib.dmd_batch_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.members = []

    def close(self):
        if getattr(self, "_h", None):
            load().dmd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def attach(self, s: "Stream"):
        check(load().dmd_batch_attach(self._h, s._h))
        self.members.append(s)

    def detach(self, s: "Stream"):
        check(load().dmd_batch_detach(self._h, s._h))
        self.members.remove(s)

    def info(self):
        n = ctypes.c_int32(0)
        used = ctypes.c_int64(0)
        bud = ctypes.c_int64(0)
        check(load().dmd_batch_info(self._h, ctypes.byref(n), ctypes.byref(used), ctypes.byref(bud)))
        return n.value, used.value, bud.value

    def _modes(self, streams, modes):
        k = len(streams)
        if modes is None:
            return None, None
        ms = (_P * k)(*[(o.data_ptr() if o is not None else None) for o in modes])
        lds = (_I64 * k)(*[(o.stride(1) if o is not None else 0) for o in modes])
        for s, o in zip(streams, modes):
            if o is not None:
                s._check_out(o, s.mode_dtype)
        return ms, lds

    def tick(self, streams, snapshots, modes=None, stream=None):
        """One tick of dense members: snapshots[i] is a contiguous CUDA tensor
        of streams[i].n values of the stream's dtype."""
        k = len(streams)
        hs = (_P * k)(*[s._h for s in streams])
        for s, x in zip(streams, snapshots):
            if not (x.is_cuda and x.dtype == s.elem and x.numel() == s.n and x.is_contiguous()):
                raise ValueError("snapshots must be contiguous CUDA tensors of n values of the stream's dtype")
        xs = (_P * k)(*[x.data_ptr() for x in snapshots])
        ms, lds = self._modes(streams, modes)
        return check(load().dmd_batch_tick(self._h, k, hs, xs, ms, lds, _stream_ptr(stream)))

    def tick_frames(self, streams, frames, modes=None, stream=None):
        """One tick of any members: frames[i] is a dense snapshot tensor, or for
        a sparse stream an (idx, val) pair of CUDA tensors (int32, complex64)."""
        k = len(streams)
        hs = (_P * k)(*[s._h for s in streams])
        fr = (Frame * k)()
        for i, (s, f) in enumerate(zip(streams, frames)):
            if s.elem == torch.complex64:
                idx, val = f
                if not (idx.is_cuda and val.is_cuda and idx.dtype == torch.int32 and val.dtype == torch.complex64
                        and idx.numel() == val.numel() and idx.is_contiguous() and val.is_contiguous()):
                    raise ValueError("a sparse frame is (idx int32, val complex64) contiguous CUDA tensors")
                fr[i].nnz = idx.numel()
                fr[i].idx = idx.data_ptr() if idx.numel() else None
                fr[i].val = val.data_ptr() if val.numel() else None
            else:
                if not (f.is_cuda and f.dtype == s.elem and f.numel() == s.n and f.is_contiguous()):
                    raise ValueError("a dense frame is a contiguous CUDA tensor of n values of the stream's dtype")
                fr[i].x = f.data_ptr()
        ms, lds = self._modes(streams, modes)
        return check(load().dmd_batch_tick_frames(self._h, k, hs, fr, ms, lds, _stream_ptr(stream)))
