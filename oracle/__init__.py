"""FP64 CPU oracle for the randomized von Neumann entropy estimators.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the
CPU-baseline leg of the benchmark are the only callers.  The GPU library never
imports, links or executes anything in this package, and this package never
imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, double precision); this module
only marshals numpy arrays through ctypes.  Each wrapper names the passage of
Kontopoulou et al. (arXiv:1801.01072) that the C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TAYLOR, CHEBYSHEV = 0, 1
RADEMACHER, GAUSSIAN = 0, 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Mat(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("ld", ctypes.c_int64),
                ("values", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p)]


class _ZMat(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("ld", ctypes.c_int64), ("values", ctypes.c_void_p)]


class _Res(ctypes.Structure):
    _fields_ = [("entropy", ctypes.c_double), ("p1_est", ctypes.c_double),
                ("u", ctypes.c_double), ("std_err", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    d, i32, i64, u32, u64 = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint32, ctypes.c_uint64)
    sig = {
        "orc_philox4x32_10": (None, [P, P, P]),
        "orc_probe_value": (d, [u64, i32, u32, i64, i64]),
        "orc_probe_vector": (None, [u64, i32, u32, i64, i64, P]),
        "orc_matvec": (None, [P, P, P]),
        "orc_power_method": (d, [P, i32, i32, u64]),
        "orc_cheb_coeffs": (None, [d, i32, P]),
        "orc_cheb_interp_coeffs": (None, [d, d, i32, i32, P]),
        "orc_cheb_eval_scalar": (d, [P, i32, d, d, d]),
        "orc_cheb_quadform": (d, [P, P, i32, d, d, P]),
        "orc_cheb_moments_forward": (None, [P, d, d, i32, P, P]),
        "orc_taylor_quadform": (d, [P, d, i32, P]),
        "orc_estimate": (ctypes.c_int, [P, i32, i32, i32, u64, i32, i32, d, i32,
                                        d, d, P, i32, P, P]),
        "orc_jacobi_eigen": (ctypes.c_int, [i64, P, P, P, d, i32]),
        "orc_entropy_from_eigs": (d, [i64, P]),
        "orc_exact_entropy": (d, [P]),
        "orc_rp_entropy_with_pi": (d, [P, P, i32, i32, P]),
        "orc_rp_entropy": (d, [P, i32, i32, u64, P]),
        "orc_rp_entropy_kind": (d, [P, i32, i32, i32, u64, P]),
        "orc_sketch_matrix": (None, [i32, u64, i64, i32, P]),
        "orc_sketch_sign": (d, [u64, i64]),
        "orc_sketch_bucket": (i32, [u64, i64, i32]),
        "orc_srht_column": (i64, [u64, i64, i64]),
        "orc_hadamard_order": (i64, [i64]),
        "orc_mlp_nparams": (i32, []),
        "orc_mlp_forward": (None, [P, i32, P, P]),
        "orc_mlp_loss_grad": (d, [P, i32, P, P, P]),
        "orc_max_threads": (i32, []),
        "orc_cutoff_nodes": (i32, [i32]),
        "orc_zmatvec": (None, [P, P, P]),
        "orc_zpower_method": (d, [P, i32, i32, u64]),
        "orc_zcheb_quadform": (d, [P, P, i32, d, d, P]),
        "orc_zcheb_moments_forward": (None, [P, d, d, i32, P, P]),
        "orc_ztaylor_quadform": (d, [P, d, i32, P]),
        "orc_zestimate": (ctypes.c_int, [P, i32, i32, i32, u64, i32, i32, d, i32,
                                         d, d, P, i32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Matrices
# --------------------------------------------------------------------------
class OMatrix:
    """Holds references to the arrays a C descriptor points at."""

    def __init__(self, dense=None, csr=None):
        if dense is not None:
            a = np.asarray(dense)
            if a.dtype not in (np.float64, np.float32):
                a = a.astype(np.float64)
            a = np.ascontiguousarray(a)
            self._keep = (a,)
            self.n = a.shape[0]
            self.s = _Mat(a.shape[0], 0, 0 if a.dtype == np.float64 else 1,
                          a.shape[1], a.ctypes.data, None, None)
        else:
            rp, ci, val, n = csr
            rp = np.ascontiguousarray(rp, dtype=np.int64)
            ci = np.ascontiguousarray(ci, dtype=np.int32)
            val = np.ascontiguousarray(val)
            if val.dtype not in (np.float64, np.float32):
                val = val.astype(np.float64)
            self._keep = (rp, ci, val)
            self.n = n
            self.s = _Mat(n, 1, 0 if val.dtype == np.float64 else 1, 0,
                          val.ctypes.data, rp.ctypes.data, ci.ctypes.data)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def as_matrix(R) -> OMatrix:
    """Dense ndarray, or a (row_ptr, col_idx, values, n) CSR tuple."""
    if isinstance(R, OMatrix):
        return R
    if isinstance(R, tuple):
        return OMatrix(csr=R)
    return OMatrix(dense=R)


# --------------------------------------------------------------------------
# Random numbers (Philox4x32-10) and probes
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter under a 2-word key (Salmon et al. 2011)."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return [int(x) for x in o]


def probe_value(seed: int, dist: int, stream: int, i: int, j: int) -> float:
    return _load().orc_probe_value(seed, dist, stream, i, j)


def probe_vector(seed: int, dist: int, stream: int, n: int, j: int) -> np.ndarray:
    g = np.empty(n, dtype=np.float64)
    _load().orc_probe_vector(seed, dist, stream, n, j, _ptr(g))
    return g


def probe_block(seed: int, dist: int, stream: int, n: int, s: int) -> np.ndarray:
    """n x s block, column j = probe j (slow: one generator call per entry)."""
    return np.stack([probe_vector(seed, dist, stream, n, j) for j in range(s)], axis=1)


# --------------------------------------------------------------------------
# Linear algebra building blocks
# --------------------------------------------------------------------------
def matvec(R, x) -> np.ndarray:
    M = as_matrix(R)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(M.n, dtype=np.float64)
    _load().orc_matvec(M.ref, _ptr(x), _ptr(y))
    return y


def power_method(R, t: int = 20, q: int = 1, seed: int = 0) -> float:
    """Algorithm 4 (Appendix A) with per-iteration normalisation."""
    M = as_matrix(R)
    return _load().orc_power_method(M.ref, t, q, seed)


def cheb_coeffs(u: float, m: int) -> np.ndarray:
    """Closed-form coefficients of Lemma 3 (Section 3)."""
    a = np.empty(m + 1, dtype=np.float64)
    _load().orc_cheb_coeffs(u, m, _ptr(a))
    return a


def cheb_interp_coeffs(lo: float, u: float, m: int, npts: int = 0) -> np.ndarray:
    """Chebyshev interpolant of x ln x on [lo, u] (lower-cutoff extension)."""
    a = np.empty(m + 1, dtype=np.float64)
    _load().orc_cheb_interp_coeffs(lo, u, m, npts, _ptr(a))
    return a


def cutoff_nodes(m: int) -> int:
    """Quadrature nodes of the estimator's lower-cutoff coefficients."""
    return _load().orc_cutoff_nodes(m)


def cheb_eval_scalar(alpha, lo: float, u: float, x: float) -> float:
    """Scalar Clenshaw recurrence (Appendix B)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    return _load().orc_cheb_eval_scalar(_ptr(a), len(a) - 1, lo, u, x)


def cheb_quadform(R, alpha, lo: float, u: float, g) -> float:
    """g^T f_m(R) g by the vector Clenshaw recurrence (Algorithm 5)."""
    M = as_matrix(R)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return _load().orc_cheb_quadform(M.ref, _ptr(a), len(a) - 1, lo, u, _ptr(g))


def cheb_moments_forward(R, lo: float, u: float, m: int, g) -> np.ndarray:
    """d_k = g^T T_k(X) g, k = 0..m, by the forward three-term recurrence."""
    M = as_matrix(R)
    g = np.ascontiguousarray(g, dtype=np.float64)
    d = np.empty(m + 1, dtype=np.float64)
    _load().orc_cheb_moments_forward(M.ref, lo, u, m, _ptr(g), _ptr(d))
    return d


def taylor_quadform(R, u: float, m: int, g) -> float:
    """sum_{k=1}^m g^T R (I - R/u)^k g / k, literally as in Algorithm 1."""
    M = as_matrix(R)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return _load().orc_taylor_quadform(M.ref, u, m, _ptr(g))


@dataclass
class Estimate:
    entropy: float
    p1_est: float
    u: float
    std_err: float
    per_probe: np.ndarray


def estimate(R, method: int, m: int, s: int, seed: int, t: int = 20, q: int = 1,
             c: float = 6.0, dist: int = RADEMACHER, lo: float = 0.0,
             u_override: float = 0.0, probes=None) -> Estimate:
    """Algorithms 1 (Taylor, method=0) and 2 (Chebyshev, method=1).

    ``probes`` selects a subset of probe indices (the mean then covers only
    those); per_probe holds h_j for each evaluated probe.
    """
    M = as_matrix(R)
    sel = None if probes is None else np.ascontiguousarray(probes, dtype=np.int32)
    cnt = s if sel is None else len(sel)
    pp = np.empty(cnt, dtype=np.float64)
    res = _Res()
    rc = _load().orc_estimate(M.ref, method, m, s, seed, t, q, c, dist, lo,
                              u_override, _ptr(sel), 0 if sel is None else len(sel),
                              _ptr(pp), ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle estimate rejected its arguments")
    return Estimate(res.entropy, res.p1_est, res.u, res.std_err, pp)


# --------------------------------------------------------------------------
# Hermitian density matrices (Section 4; Algorithms 1c and 2c)
# --------------------------------------------------------------------------
class ZMatrix:
    """A dense Hermitian matrix (complex128 or complex64 ndarray) for the C side."""

    def __init__(self, A):
        a = np.asarray(A)
        if a.dtype not in (np.complex128, np.complex64):
            a = a.astype(np.complex128)
        a = np.ascontiguousarray(a)
        self._keep = a
        self.n = a.shape[0]
        self.s = _ZMat(a.shape[0], 0 if a.dtype == np.complex128 else 1, a.shape[1], a.ctypes.data)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _zmat(R) -> ZMatrix:
    return R if isinstance(R, ZMatrix) else ZMatrix(R)


def zmatvec(R, x) -> np.ndarray:
    M = _zmat(R)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty(M.n, dtype=np.complex128)
    _load().orc_zmatvec(M.ref, _ptr(x), _ptr(y))
    return y


def zpower_method(R, t: int = 20, q: int = 1, seed: int = 0) -> float:
    """Algorithm 4 with a complex iterate (start s_i + i s_{n+i}, stream 1)."""
    return _load().orc_zpower_method(_zmat(R).ref, t, q, seed)


def zcheb_quadform(R, alpha, lo: float, u: float, g) -> float:
    """g^T Re[f_m(R)] g by the complex vector Clenshaw recurrence."""
    M = _zmat(R)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return _load().orc_zcheb_quadform(M.ref, _ptr(a), len(a) - 1, lo, u, _ptr(g))


def zcheb_moments_forward(R, lo: float, u: float, m: int, g) -> np.ndarray:
    """d_k = g^T Re[T_k(X)] g, k = 0..m."""
    M = _zmat(R)
    g = np.ascontiguousarray(g, dtype=np.float64)
    d = np.empty(m + 1, dtype=np.float64)
    _load().orc_zcheb_moments_forward(M.ref, lo, u, m, _ptr(g), _ptr(d))
    return d


def ztaylor_quadform(R, u: float, m: int, g) -> float:
    """sum_{k=1}^m g^T Re[R (I - R/u)^k] g / k (Algorithm 1c at u = 1)."""
    M = _zmat(R)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return _load().orc_ztaylor_quadform(M.ref, u, m, _ptr(g))


def zestimate(R, method: int, m: int, s: int, seed: int, t: int = 20, q: int = 1,
              c: float = 6.0, dist: int = GAUSSIAN, lo: float = 0.0,
              u_override: float = 1.0, probes=None) -> Estimate:
    """Algorithms 1c (method=0) and 2c (method=1) on Hermitian R.

    u_override = 1 is the paper's choice for Hermitian inputs; 0 runs the
    complex power method and takes u = min{1, c p~1}.
    """
    M = _zmat(R)
    sel = None if probes is None else np.ascontiguousarray(probes, dtype=np.int32)
    cnt = s if sel is None else len(sel)
    pp = np.empty(cnt, dtype=np.float64)
    res = _Res()
    rc = _load().orc_zestimate(M.ref, method, m, s, seed, t, q, c, dist, lo, u_override,
                               _ptr(sel), 0 if sel is None else len(sel), _ptr(pp),
                               ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle estimate rejected its arguments")
    return Estimate(res.entropy, res.p1_est, res.u, res.std_err, pp)


def jacobi_eigen(A, tol: float = 1e-15, max_sweeps: int = 100, vectors: bool = False):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    e = np.empty(n, dtype=np.float64)
    V = np.empty((n, n), dtype=np.float64) if vectors else None
    sweeps = _load().orc_jacobi_eigen(n, _ptr(A), _ptr(e), _ptr(V), tol, max_sweeps)
    return (e, V, sweeps) if vectors else e


def entropy_from_eigs(p) -> float:
    p = np.ascontiguousarray(p, dtype=np.float64)
    return _load().orc_entropy_from_eigs(len(p), _ptr(p))


def exact_entropy(R) -> float:
    """-sum p_i ln p_i over the Jacobi eigenvalues (eqn. (1))."""
    return _load().orc_exact_entropy(as_matrix(R).ref)


def rp_entropy_with_pi(R, Pi, k: int):
    """Algorithm 3 with a given sketch Pi (n x s)."""
    M = as_matrix(R)
    Pi = np.ascontiguousarray(Pi, dtype=np.float64)
    s = Pi.shape[1]
    sig = np.zeros(k, dtype=np.float64)
    h = _load().orc_rp_entropy_with_pi(M.ref, _ptr(Pi), s, k, _ptr(sig))
    return h, sig


SKETCH_GAUSSIAN, SKETCH_SRHT, SKETCH_COUNT = 0, 1, 2


def rp_entropy(R, s: int, k: int, seed: int, kind: int = SKETCH_GAUSSIAN):
    """Algorithm 3 with a Gaussian (kind 0), subsampled randomized Hadamard
    (1) or input-sparsity (2) sketch; see orc_sketch_matrix."""
    M = as_matrix(R)
    sig = np.zeros(k, dtype=np.float64)
    h = _load().orc_rp_entropy_kind(M.ref, kind, s, k, seed, _ptr(sig))
    return h, sig


def sketch_matrix(kind: int, seed: int, n: int, s: int) -> np.ndarray:
    """The n x s sketch Pi of Algorithm 3 for the given construction."""
    Pi = np.empty((n, s), dtype=np.float64)
    _load().orc_sketch_matrix(kind, seed, n, s, _ptr(Pi))
    return Pi


def sketch_sign(seed: int, j: int) -> float:
    return _load().orc_sketch_sign(seed, j)


def sketch_bucket(seed: int, j: int, s: int) -> int:
    return _load().orc_sketch_bucket(seed, j, s)


def srht_column(seed: int, t: int, N: int) -> int:
    return _load().orc_srht_column(seed, t, N)


def hadamard_order(n: int) -> int:
    return _load().orc_hadamard_order(n)


def mlp_nparams() -> int:
    return _load().orc_mlp_nparams()


def mlp_forward(params, X) -> np.ndarray:
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.empty((X.shape[0], 2), dtype=np.float64)
    _load().orc_mlp_forward(_ptr(P), X.shape[0], _ptr(X), _ptr(Y))
    return Y


def mlp_loss_grad(params, X, T):
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.empty_like(P)
    loss = _load().orc_mlp_loss_grad(_ptr(P), X.shape[0], _ptr(X), _ptr(T), _ptr(g))
    return loss, g


def max_threads() -> int:
    return _load().orc_max_threads()
