"""CPU oracle for the filtered precise-integration matrix exponential.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark use this package to check and time the GPU library.
The GPU library never imports it.  It wraps ``oracle_expm.c`` (plain C,
OpenMP over rows) through ctypes; see that file for the algorithm and the
paper passages each function follows.

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` (closed forms, brute force, the paper's worked
example and Tables 1-3).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_expm.c")
_LIB = os.path.join(_HERE, "liboracle_expm.so")
MAXSTEP = 256

OK, EINVAL, ENOMEM, ERANGE, ENOTCONV = 0, -1, -2, -4, -5


def build() -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("normal", C.c_int), ("filter_mode", C.c_int), ("e_r", C.c_double),
                ("max_iter", C.c_int), ("keep", C.c_int), ("norm", C.c_int),
                ("exact_ri", C.c_int), ("literal_a", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("M", C.c_int), ("N", C.c_int), ("taylor_terms", C.c_int),
                ("squarings", C.c_int), ("normal", C.c_int),
                ("a", C.c_double), ("nh", C.c_double), ("h0", C.c_double),
                ("r0", C.c_double), ("eg0", C.c_double),
                ("taylor_theta", C.c_double * MAXSTEP), ("taylor_iters", C.c_int * MAXSTEP),
                ("taylor_cand", C.c_int64 * MAXSTEP), ("taylor_kept", C.c_int64 * MAXSTEP),
                ("sq_theta", C.c_double * MAXSTEP), ("sq_normF", C.c_double * MAXSTEP),
                ("sq_budget", C.c_double * MAXSTEP), ("sq_dropped", C.c_double * MAXSTEP),
                ("sq_iters", C.c_int * MAXSTEP),
                ("sq_cand", C.c_int64 * MAXSTEP), ("sq_kept", C.c_int64 * MAXSTEP),
                ("sq_band", C.c_int64 * MAXSTEP), ("sq_ri", C.c_double * MAXSTEP)]


_lib = None
_P = C.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        lib.ora_r0.restype = C.c_double
        lib.ora_r0.argtypes = [C.c_int, C.c_double]
        lib.ora_choose_mn.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        lib.ora_filter.argtypes = [_P, C.c_int64, C.c_double, C.c_double, C.c_int,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int),
                                   C.POINTER(C.c_double), _P]
        lib.ora_expm.restype = _P
        lib.ora_expm.argtypes = [C.c_int64, _P, _P, _P, C.c_double, C.POINTER(_Opts),
                                 C.POINTER(C.c_int)]
        lib.ora_matmul.restype = _P
        lib.ora_matmul.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, C.POINTER(C.c_int)]
        lib.ora_run_nnz.restype = C.c_int64
        lib.ora_run_nnz.argtypes = [_P]
        lib.ora_run_copy.argtypes = [_P, _P, _P, _P]
        lib.ora_run_stats.argtypes = [_P, C.POINTER(_Stats)]
        lib.ora_run_inter.restype = C.c_int64
        lib.ora_run_inter.argtypes = [_P, C.c_int, C.c_int, _P, _P, _P]
        lib.ora_backward.argtypes = [_P, _P, _P]
        lib.ora_free.argtypes = [_P]
        lib.ora_threads.restype = C.c_int
        lib.ora_spmm.restype = None
        lib.ora_spmm.argtypes = [C.c_int64, _P, _P, _P, C.c_int64, _P, _P]
        lib.ora_power_norms.argtypes = [C.c_int64, _P, _P, _P, C.c_int, _P]
        lib.ora_alpha_hat.argtypes = [C.c_double, C.c_int, C.c_int, C.c_double, _P, C.c_int,
                                      C.POINTER(C.c_int64)]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr_arrays(rowptr, col, val):
    return (np.ascontiguousarray(rowptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def r0(M: int, x: float) -> float:
    """Eq. (4.5): bound on ||F0^-1 R0|| for Taylor degree M at ||H 2^-N|| = x."""
    return _load().ora_r0(int(M), float(x))


def choose_mn(norm: float, eps: float) -> tuple[int, int]:
    """Problem (4.20): (M, N) minimising M 2^N."""
    M, N = C.c_int(), C.c_int()
    st = _load().ora_choose_mn(float(norm), float(eps), C.byref(M), C.byref(N))
    if st:
        raise OracleError(st, "choose_mn")
    return M.value, N.value


def filter_values(v, eg: float, e_r: float = 0.1, max_iter: int = 64):
    """Algorithm 4.1 on a value array: returns (keep mask, theta, iterations, b)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    keep = np.zeros(v.size, dtype=np.uint8)
    th, it, b = C.c_double(), C.c_int(), C.c_double()
    st = _load().ora_filter(_ptr(v), v.size, float(eg), float(e_r), int(max_iter),
                            C.byref(th), C.byref(it), C.byref(b), _ptr(keep))
    if st:
        raise OracleError(st, "filter")
    return keep.astype(bool), th.value, it.value, b.value


def threads() -> int:
    return _load().ora_threads()


@dataclass
class Result:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    stats: dict


def _stats_dict(s: _Stats) -> dict:
    d = {k: getattr(s, k) for k in ("M", "N", "taylor_terms", "squarings", "normal",
                                    "a", "nh", "h0", "r0", "eg0")}
    T = s.taylor_terms
    Nsq = s.squarings
    d["taylor_theta"] = list(s.taylor_theta[2:T + 2])
    d["taylor_iters"] = list(s.taylor_iters[2:T + 2])
    d["taylor_cand"] = list(s.taylor_cand[2:T + 2])
    d["taylor_kept"] = list(s.taylor_kept[2:T + 2])
    for k in ("sq_theta", "sq_normF", "sq_budget", "sq_dropped", "sq_iters", "sq_cand", "sq_kept",
              "sq_ri"):
        d[k] = list(getattr(s, k)[1:Nsq + 1])
    d["sq_band"] = list(s.sq_band[0:Nsq + 1])        # l(T^_0) .. l(T^_N)
    d["theta0"] = s.sq_theta[0]                       # FPIM's threshold of T_0
    return d


class Run:
    """One oracle evaluation of Algorithm 4.2; keeps the intermediates when
    ``keep`` so that :meth:`backward` can run."""

    def __init__(self, rowptr, col, val, eps: float, *, normal: int = -1,
                 filter_mode: int = 0, e_r: float = 0.1, max_iter: int = 64, keep: bool = True,
                 norm: int = 0, exact_ri: bool = False, literal_a: bool = False):
        lib = _load()
        rp, ci, v = _csr_arrays(rowptr, col, val)
        self.n = rp.size - 1
        self._H = (rp, ci, v)
        o = _Opts(int(normal), int(filter_mode), float(e_r), int(max_iter), int(keep), int(norm),
                  int(exact_ri), int(literal_a))
        st = C.c_int()
        self._h = lib.ora_expm(self.n, _ptr(rp), _ptr(ci), _ptr(v), float(eps), C.byref(o), C.byref(st))
        if st.value:
            self.close()
            raise OracleError(st.value, "expm")

    def result(self) -> Result:
        lib = _load()
        nnz = lib.ora_run_nnz(self._h)
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        lib.ora_run_copy(self._h, _ptr(rp), _ptr(ci), _ptr(v))
        s = _Stats()
        lib.ora_run_stats(self._h, C.byref(s))
        return Result(self.n, rp, ci, v, _stats_dict(s))

    def intermediate(self, kind: str, idx: int):
        """kind 'S': filtered Taylor term S^_idx (idx >= 1); kind 'T': squaring
        iterate T^_idx (idx = 0..N).  Returns (rowptr, col, val) or None."""
        lib = _load()
        k = 0 if kind == "S" else 1
        nnz = lib.ora_run_inter(self._h, k, int(idx), None, None, None)
        if nnz < 0:
            return None
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        lib.ora_run_inter(self._h, k, int(idx), _ptr(rp), _ptr(ci), _ptr(v))
        return rp, ci, v

    def backward(self, dE) -> np.ndarray:
        """Adjoint with frozen masks: dL/d(values of H) given dL/d(values of E)."""
        lib = _load()
        dE = np.ascontiguousarray(dE, dtype=np.float64)
        dH = np.zeros(self._H[1].size, np.float64)
        st = lib.ora_backward(self._h, _ptr(dE), _ptr(dH))
        if st:
            raise OracleError(st, "backward")
        return dH

    def close(self):
        if getattr(self, "_h", None):
            _load().ora_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def expm(rowptr, col, val, eps: float, **kw) -> Result:
    """e^H for a CSR matrix by Algorithm 4.2 (no intermediates kept)."""
    kw.setdefault("keep", False)
    r = Run(rowptr, col, val, eps, **kw)
    try:
        return r.result()
    finally:
        r.close()


def matmul(n: int, A, B):
    """Plain sparse product A*B (structural pattern kept), for tests."""
    lib = _load()
    a = _csr_arrays(*A)
    b = _csr_arrays(*B)
    st = C.c_int()
    h = lib.ora_matmul(n, _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(b[0]), _ptr(b[1]), _ptr(b[2]),
                       C.byref(st))
    try:
        if st.value:
            raise OracleError(st.value, "matmul")
        nnz = lib.ora_run_nnz(h)
        rp = np.empty(n + 1, np.int64)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        lib.ora_run_copy(h, _ptr(rp), _ptr(ci), _ptr(v))
        return rp, ci, v
    finally:
        lib.ora_free(h)


def spmm(A, X) -> np.ndarray:
    """Y = A X for a CSR matrix A = (rowptr, col, val) and a dense X (n x m)."""
    lib = _load()
    rp, ci, v = _csr_arrays(*A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, m = X.shape
    Y = np.empty((n, m), np.float64)
    lib.ora_spmm(n, _ptr(rp), _ptr(ci), _ptr(v), m, _ptr(X), _ptr(Y))
    return Y


def power_norms(A, K: int) -> np.ndarray:
    """||A^k||_F for k = 1..K by plain sparse products."""
    lib = _load()
    rp, ci, v = _csr_arrays(*A)
    out = np.zeros(K, np.float64)
    st = lib.ora_power_norms(rp.size - 1, _ptr(rp), _ptr(ci), _ptr(v), int(K), _ptr(out))
    if st:
        raise OracleError(st, "power_norms")
    return out


def alpha_hat(ri: float, i: int, N: int, norm: float = 0.0, power_norms=None) -> int:
    """alpha-hat_i of Eq. (4.8) (from ||H|| = norm) or, given power_norms
    [||H^k||, k = 1..K], of Eq. (4.9)."""
    lib = _load()
    out = C.c_int64()
    if power_norms is None:
        st = lib.ora_alpha_hat(float(ri), int(i), int(N), float(norm), None, 0, C.byref(out))
    else:
        hk = np.ascontiguousarray(power_norms, dtype=np.float64)
        st = lib.ora_alpha_hat(float(ri), int(i), int(N), 0.0, _ptr(hk), hk.size, C.byref(out))
    if st:
        raise OracleError(st, "alpha_hat")
    return out.value
