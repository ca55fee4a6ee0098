"""Python binding of libentropy: randomized von Neumann entropy estimators
(Kontopoulou et al., arXiv:1801.01072) on MI355X.

Argument marshalling only.  Every step of every estimate runs in the gfx950
kernels of ``libentropy.so``; there is no CPU or PyTorch fallback, and
importing this package fails loudly if the library has not been built.
PyTorch supplies device memory (tensors) and streams.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

# torch first: it brings the HIP runtime that this library then shares (the
# dynamic linker resolves the library's libamdhip64 to the one already
# loaded), so both see the same devices, streams and allocations.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libentropy.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)

# ---- enums (mirror include/entropy.h) ---------------------------------------
OK, EINVAL, ENOTDENSITY, ENOMEM, EDEVICE, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
TAYLOR, CHEBYSHEV, RANDPROJ, AUTO = 0, 1, 2, 3
F64, F32, BF16X3 = 0, 1, 2
DENSE, CSR = 0, 1
STORE_F64, STORE_F32, STORE_C128, STORE_C64 = 0, 1, 2, 3
RADEMACHER, GAUSSIAN = 0, 1
FLAG_SKIP_TRACE_CHECK = 1
FLAG_AUTOTUNE = 2
FLAG_COMPLEX_POWER = 4
FLAG_CLENSHAW = 8
FLAG_CSR_GENERAL = 16
FLAG_CSR_BANDED = 32
FLAG_NORMALIZE = 64
FLAG_BATCH_STEPWISE = 128
FLAG_AUTO_RANDPROJ = 256

_METHODS = {"taylor": TAYLOR, "chebyshev": CHEBYSHEV, "randproj": RANDPROJ, "auto": AUTO}
_PRECISIONS = {"f64": F64, "f32": F32, "bf16x3": BF16X3}
_DISTS = {"rademacher": RADEMACHER, "gaussian": GAUSSIAN}
SKETCH_GAUSSIAN, SKETCH_SRHT, SKETCH_COUNT = 0, 1, 2
_SKETCHES = {"gaussian": SKETCH_GAUSSIAN, "srht": SKETCH_SRHT, "count": SKETCH_COUNT}


class EntMatrix(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("layout", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("ld", ctypes.c_int64), ("nnz", ctypes.c_int64), ("values", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class EntOptions(ctypes.Structure):
    _fields_ = [("power_iters", ctypes.c_int32), ("power_trials", ctypes.c_int32),
                ("u_factor", ctypes.c_double), ("u_fixed", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("precision", ctypes.c_int32),
                ("probe_dist", ctypes.c_int32), ("rank_k", ctypes.c_int32),
                ("sketch_width", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("sketch", ctypes.c_int32), ("trace_tol", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class EntResult(ctypes.Structure):
    _fields_ = [("entropy", ctypes.c_double), ("std_err", ctypes.c_double),
                ("p1_est", ctypes.c_double), ("u", ctypes.c_double), ("lo", ctypes.c_double),
                ("degree", ctypes.c_int32), ("probes", ctypes.c_int32),
                ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("products", ctypes.c_int32)]


class EntTiming(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("power_ms", ctypes.c_double),
                ("steps_ms", ctypes.c_double), ("step_max_ms", ctypes.c_double),
                ("epilogue_ms", ctypes.c_double), ("other_ms", ctypes.c_double),
                ("step_launches", ctypes.c_int32), ("power_launches", ctypes.c_int32),
                ("epilogue_launches", ctypes.c_int32), ("csr_band", ctypes.c_int32),
                ("steps_fused", ctypes.c_int32)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "ent_options_default": (None, [ctypes.POINTER(EntOptions)]),
    "ent_entropy_estimate": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_uint64,
                                            ctypes.POINTER(EntOptions), ctypes.POINTER(EntResult)]),
    "ent_entropy_estimate_detail": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_int32,
                                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                                   ctypes.POINTER(EntOptions),
                                                   ctypes.POINTER(EntResult), _P, _P]),
    "ent_entropy_estimate_noalloc": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_int32,
                                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                                    ctypes.POINTER(EntOptions),
                                                    ctypes.POINTER(EntResult), _P, _P]),
    "ent_power_method": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_double)]),
    "ent_chebyshev_coeffs": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P]),
    "ent_probes_for": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double]),
    "ent_degree_taylor": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "ent_degree_chebyshev": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "ent_power_trials_for": (ctypes.c_int32, [ctypes.c_double]),
    "ent_power_iters_for": (ctypes.c_int32, [ctypes.c_int64]),
    "ent_entropy_estimate_batched": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_int32,
                                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_uint64, ctypes.POINTER(EntOptions),
                                                    ctypes.POINTER(EntResult)]),
    "ent_graph_create": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.POINTER(EntOptions), ctypes.POINTER(_P)]),
    "ent_graph_launch": (ctypes.c_int, [_P, ctypes.POINTER(EntResult)]),
    "ent_graph_per_probe": (ctypes.c_int, [_P, _P]),
    "ent_graph_time_eager": (ctypes.c_int, [_P, ctypes.POINTER(EntResult), ctypes.POINTER(EntTiming)]),
    "ent_graph_tile_rows": (ctypes.c_int32, [_P]),
    "ent_graph_window_bytes": (ctypes.c_size_t, [_P]),
    "ent_graph_workspace_bytes": (ctypes.c_size_t, [_P]),
    "ent_graph_destroy": (ctypes.c_int, [_P]),
    "ent_mlp_nparams": (ctypes.c_int32, []),
    "ent_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    "ent_mlp_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "ent_mlp_train_epoch": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_int32), _P, _P,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_float, _P,
                                           ctypes.POINTER(ctypes.c_double)]),
    "ent_selector_load": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ent_selector_features": (ctypes.c_int, [ctypes.POINTER(EntMatrix), ctypes.c_uint64,
                                             ctypes.POINTER(EntOptions), _P, _P]),
    "ent_timing_enable": (ctypes.c_int, [ctypes.c_int32]),
    "ent_last_timing": (ctypes.c_int, [ctypes.POINTER(EntTiming)]),
    "ent_set_workspace_limit": (ctypes.c_int, [ctypes.c_size_t]),
    "ent_release_workspace": (ctypes.c_int, []),
    "ent_workspace_bytes": (ctypes.c_size_t, []),
    "ent_last_error": (ctypes.c_char_p, []),
    "ent_version": (ctypes.c_int32, []),
}
for _name, (_res, _args) in _SIGNATURES.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class EntropyError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status
        self.message = message


def last_error() -> str:
    return _lib.ent_last_error().decode()


def _check(status: int):
    if status != OK:
        raise EntropyError(status, last_error())


@dataclass
class Result:
    entropy: float
    std_err: float
    p1_est: float
    u: float
    lo: float
    degree: int
    probes: int
    method: int
    precision: int
    fell_back: int = 0
    products: int = 0


def _result(r: EntResult) -> Result:
    return Result(r.entropy, r.std_err, r.p1_est, r.u, r.lo, r.degree, r.probes, r.method,
                  r.precision, r.fell_back, r.products)


# ---- matrices -----------------------------------------------------------------
def _store_dtype(t) -> int:
    import torch

    if t.dtype == torch.float64:
        return STORE_F64
    if t.dtype == torch.float32:
        return STORE_F32
    if t.dtype == torch.complex128:
        return STORE_C128
    if t.dtype == torch.complex64:
        return STORE_C64
    raise TypeError(f"unsupported value dtype {t.dtype}")


def dense_matrix(R) -> EntMatrix:
    """Descriptor of a dense 2-D tensor with unit column stride (device memory,
    or host memory that the library copies to the device)."""
    if R.dim() != 2 or R.shape[0] != R.shape[1]:
        raise ValueError("R must be a square 2-D tensor")
    if R.stride(1) != 1:
        raise ValueError("R must have unit column stride (row-major)")
    return EntMatrix(R.shape[0], DENSE, _store_dtype(R), R.stride(0), 0, R.data_ptr(), None, None)


def csr_matrix(row_ptr, col_idx, values, n: int) -> EntMatrix:
    """Descriptor of a CSR matrix held in tensors (int64, int32, values), on the
    device or in host memory (copied in by the library)."""
    import torch

    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col_idx int32")
    return EntMatrix(n, CSR, _store_dtype(values), 0, values.numel(), values.data_ptr(),
                     row_ptr.data_ptr(), col_idx.data_ptr())


def as_matrix(R) -> EntMatrix:
    if isinstance(R, EntMatrix):
        return R
    if isinstance(R, tuple):
        rp, ci, val, n = R
        return csr_matrix(rp, ci, val, n)
    return dense_matrix(R)


def _stream_handle(stream):
    if stream is not None:
        return int(getattr(stream, "cuda_stream", stream))
    try:
        import torch

        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch without a device
        pass
    return None


def options(precision="f64", probe_dist="rademacher", power_iters=20, power_trials=1,
            u_factor=6.0, u_fixed=0.0, cutoff=0.0, rank_k=0, sketch_width=0, flags=0,
            trace_tol=0.0, stream=None, sketch="gaussian") -> EntOptions:
    o = EntOptions()
    _lib.ent_options_default(ctypes.byref(o))
    o.precision = _PRECISIONS.get(precision, precision)
    o.probe_dist = _DISTS.get(probe_dist, probe_dist)
    o.power_iters = power_iters
    o.power_trials = power_trials
    o.u_factor = u_factor
    o.u_fixed = u_fixed
    o.cutoff = cutoff
    o.rank_k = rank_k
    o.sketch_width = sketch_width
    o.flags = flags
    o.sketch = _SKETCHES.get(sketch, sketch)
    o.trace_tol = trace_tol
    o.stream = _stream_handle(stream)
    return o


# ---- entry points ----------------------------------------------------------------
def entropy_estimate(R, method="chebyshev", degree=30, probes=50, seed=0, **opts) -> Result:
    """One estimate of H(R) (Algorithms 1-3); see ent_entropy_estimate."""
    M = as_matrix(R)
    o = options(**opts)
    res = EntResult()
    _check(_lib.ent_entropy_estimate(ctypes.byref(M), _METHODS.get(method, method), degree, probes,
                                     seed, ctypes.byref(o), ctypes.byref(res)))
    return _result(res)


def entropy_estimate_detail(R, method="chebyshev", degree=30, probes=50, seed=0, **opts):
    """Estimate plus per-probe values h_j and the moment table (degree+1, probes)."""
    M = as_matrix(R)
    o = options(**opts)
    res = EntResult()
    meth = _METHODS.get(method, method)
    nper = opts.get("rank_k", 0) if meth == RANDPROJ else probes
    per = np.zeros(max(nper, 1), dtype=np.float64)
    mom = np.zeros((degree + 1) * probes if meth != RANDPROJ else 1, dtype=np.float64)
    _check(_lib.ent_entropy_estimate_detail(ctypes.byref(M), meth, degree, probes, seed,
                                            ctypes.byref(o), ctypes.byref(res),
                                            per.ctypes.data_as(_P), mom.ctypes.data_as(_P)))
    if meth == RANDPROJ:
        return _result(res), per[:nper], None
    return _result(res), per, mom.reshape(degree + 1, probes)


NOALLOC_SCRATCH_BYTES = 128 << 20


def entropy_estimate_noalloc(R, method="chebyshev", degree=30, probes=50, seed=0, **opts):
    """entropy_estimate_detail through the entry point that allocates no
    device memory (fixed per-device scratch; Taylor / Chebyshev only)."""
    M = as_matrix(R)
    o = options(**opts)
    res = EntResult()
    meth = _METHODS.get(method, method)
    per = np.zeros(probes, dtype=np.float64)
    mom = np.zeros((degree + 1) * probes, dtype=np.float64)
    _check(_lib.ent_entropy_estimate_noalloc(ctypes.byref(M), meth, degree, probes, seed,
                                             ctypes.byref(o), ctypes.byref(res),
                                             per.ctypes.data_as(_P), mom.ctypes.data_as(_P)))
    return _result(res), per, mom.reshape(degree + 1, probes)


def power_method(R, t=20, q=1, seed=0, stream=None) -> float:
    """Algorithm 4 with per-iteration normalisation; returns p~1."""
    M = as_matrix(R)
    v = ctypes.c_double()
    _check(_lib.ent_power_method(ctypes.byref(M), t, q, seed, _stream_handle(stream), ctypes.byref(v)))
    return v.value


def chebyshev_coeffs(lo: float, u: float, m: int) -> np.ndarray:
    a = np.zeros(m + 1, dtype=np.float64)
    _check(_lib.ent_chebyshev_coeffs(lo, u, m, a.ctypes.data_as(_P)))
    return a


def probes_for(eps: float, delta: float) -> int:
    return _lib.ent_probes_for(eps, delta)


def degree_taylor(u: float, ell: float, eps: float) -> int:
    return _lib.ent_degree_taylor(u, ell, eps)


def degree_chebyshev(u: float, ell: float, eps: float) -> int:
    return _lib.ent_degree_chebyshev(u, ell, eps)


def power_trials_for(delta: float) -> int:
    return _lib.ent_power_trials_for(delta)


def power_iters_for(n: int) -> int:
    return _lib.ent_power_iters_for(n)


def timing_enable(on: bool = True):
    """Record HIP events between launches of later estimates on this thread."""
    _check(_lib.ent_timing_enable(1 if on else 0))


def last_timing() -> dict:
    t = EntTiming()
    _check(_lib.ent_last_timing(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in EntTiming._fields_}


# ---- learned selector ---------------------------------------------------------------
def mlp_nparams() -> int:
    return _lib.ent_mlp_nparams()


def mlp_forward(params, X, stream=None):
    """Inference of the selector network on device tensors (X: count x 16 float32)."""
    import torch

    Y = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
    _check(_lib.ent_mlp_forward(params.data_ptr(), X.data_ptr(), X.shape[0], Y.data_ptr(),
                                _stream_handle(stream)))
    return Y


def mlp_grad(params, X, T, stream=None):
    """Gradient (device tensor) and value of the mean squared error."""
    import torch

    g = torch.empty_like(params)
    loss = ctypes.c_double()
    _check(_lib.ent_mlp_grad(params.data_ptr(), X.data_ptr(), T.data_ptr(), X.shape[0], g.data_ptr(),
                             ctypes.byref(loss), _stream_handle(stream)))
    return g, loss.value


class AdamState:
    """Device-resident parameters and Adam moments of the selector network."""

    def __init__(self, params):
        import torch

        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = ctypes.c_int32(0)

    def epoch(self, X, T, batch, lr, stream=None) -> float:
        loss = ctypes.c_double()
        _check(_lib.ent_mlp_train_epoch(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                        ctypes.byref(self.step), X.data_ptr(), T.data_ptr(), X.shape[0],
                                        batch, lr, _stream_handle(stream), ctypes.byref(loss)))
        return loss.value


def selector_load(params):
    """Install selector parameters (host numpy float32 array or tensor) on the current device."""
    a = np.ascontiguousarray(np.asarray(params.detach().cpu() if hasattr(params, "detach") else params,
                                        dtype=np.float32))
    _check(_lib.ent_selector_load(a.ctypes.data_as(_P), a.size))


def selector_features(R, seed=0, **opts):
    """Features of R's sketch pass and the loaded network's outputs (needs selector_load)."""
    M = as_matrix(R)
    o = options(**opts)
    f = np.zeros(16, dtype=np.float32)
    y = np.zeros(2, dtype=np.float32)
    _check(_lib.ent_selector_features(ctypes.byref(M), seed, ctypes.byref(o), f.ctypes.data_as(_P),
                                      y.ctypes.data_as(_P)))
    return f, y


# ---- batches ----------------------------------------------------------------------
def _mat_array(mats):
    arr = (EntMatrix * len(mats))()
    for i, R in enumerate(mats):
        arr[i] = as_matrix(R)
    return arr


def entropy_estimate_batched(mats, method="chebyshev", degree=40, probes=64, seed=0, **opts):
    """One synchronous run over a batch of dense matrices; matrix b uses seed + b."""
    arr = _mat_array(mats)
    o = options(**opts)
    outs = (EntResult * len(mats))()
    _check(_lib.ent_entropy_estimate_batched(arr, len(mats), _METHODS.get(method, method), degree,
                                             probes, seed, ctypes.byref(o), outs))
    return [_result(r) for r in outs]


class Graph:
    """A planned batch captured into a hipGraph (see ent_graph_create)."""

    def __init__(self, mats, method="chebyshev", degree=40, probes=64, seed=0, **opts):
        self._mats = list(mats)  # keep the tensors alive while the graph exists
        self._arr = _mat_array(self._mats)
        self.count = len(self._mats)
        self.probes = probes
        o = options(**opts)
        h = _P()
        _check(_lib.ent_graph_create(self._arr, self.count, _METHODS.get(method, method), degree,
                                     probes, seed, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def launch(self):
        outs = (EntResult * self.count)()
        _check(_lib.ent_graph_launch(self._h, outs))
        return [_result(r) for r in outs]

    def per_probe(self) -> np.ndarray:
        a = np.zeros(self.count * self.probes, dtype=np.float64)
        _check(_lib.ent_graph_per_probe(self._h, a.ctypes.data_as(_P)))
        return a.reshape(self.count, self.probes)

    def time_eager(self):
        outs = (EntResult * self.count)()
        t = EntTiming()
        _check(_lib.ent_graph_time_eager(self._h, outs, ctypes.byref(t)))
        return [_result(r) for r in outs], {f: getattr(t, f) for f, _ in EntTiming._fields_}

    @property
    def tile_rows(self) -> int:
        return _lib.ent_graph_tile_rows(self._h)

    @property
    def workspace_bytes(self) -> int:
        return _lib.ent_graph_workspace_bytes(self._h)

    @property
    def window_bytes(self) -> int:
        """Window of the persistent step schedule (0: one launch per step)."""
        return _lib.ent_graph_window_bytes(self._h)

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.ent_graph_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.destroy()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def set_workspace_limit(nbytes: int):
    _check(_lib.ent_set_workspace_limit(nbytes))


def release_workspace():
    _check(_lib.ent_release_workspace())


def workspace_bytes() -> int:
    return _lib.ent_workspace_bytes()


def version() -> int:
    return _lib.ent_version()
