"""ctypes binding of ``include/expm.h`` (argument marshalling only).

The names match the C ABI one to one.  Pointers are plain integers (device
addresses); nothing here computes anything: every step of the method runs in
the gfx950 library ``libexpm_gfx950.so``.  Loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexpm_gfx950.so")

EXPM_OK = 0
EXPM_EINVAL = -1
EXPM_ENOMEM = -2
EXPM_EHIP = -3
EXPM_ERANGE = -4
EXPM_ENOTCONV = -5
EXPM_ENOTIMPL = -6
EXPM_ESTATE = -7
EXPM_NORMAL_AUTO = -1
EXPM_FILTER_PAPER = 0
EXPM_FILTER_NONE = 1
EXPM_FILTER_FIXED_REL = 2
EXPM_NORM_FRO = 0
EXPM_NORM_ONE = 1
EXPM_MAXSTEP = 128

ERROR_NAMES = {0: "EXPM_OK", -1: "EXPM_EINVAL", -2: "EXPM_ENOMEM", -3: "EXPM_EHIP",
               -4: "EXPM_ERANGE", -5: "EXPM_ENOTCONV", -6: "EXPM_ENOTIMPL", -7: "EXPM_ESTATE"}

# Every function the header declares.
SYMBOLS = ["expm_opts_default", "expm_plan", "expm_sparse", "expm_sparse_backward",
           "expm_sparse_batched", "expm_get_stats", "expm_csr_release", "expm_free",
           "expm_last_error", "expm_r0", "expm_choose_mn", "expm_sparse_noalloc",
           "expm_analyze", "expm_spmm", "expm_propagate", "expm_power_norms", "expm_alpha_hat",
           "expm_sparse_z"]

# bytes of the static device array behind expm_sparse_noalloc (expm.h)
NOALLOC_SCRATCH_BYTES = 256 << 20


class expm_csr_cview(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("on_host", C.c_int)]


class expm_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class expm_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class expm_opts(C.Structure):
    _fields_ = [("normal", C.c_int), ("filter_mode", C.c_int), ("e_r", C.c_double),
                ("max_filter_iter", C.c_int), ("keep_checkpoints", C.c_int),
                ("checkpoint_interval", C.c_int), ("stream", C.c_void_p),
                ("allocator", C.POINTER(expm_allocator)), ("profile", C.c_int),
                ("reorder", C.c_int), ("tile_min_fill", C.c_double), ("norm", C.c_int),
                ("exact_ri", C.c_int), ("diagnostics", C.c_int), ("literal_a", C.c_int),
                ("batch_solo_n", C.c_int), ("use_symmetry", C.c_int)]


_S = EXPM_MAXSTEP


class expm_stats(C.Structure):
    _fields_ = [("status", C.c_int), ("M", C.c_int), ("N", C.c_int), ("taylor_terms", C.c_int),
                ("normal", C.c_int), ("squarings", C.c_int),
                ("a", C.c_double), ("norm_h", C.c_double), ("h0", C.c_double),
                ("r0", C.c_double), ("eg0", C.c_double),
                ("taylor_theta", C.c_double * _S), ("taylor_iters", C.c_int * _S),
                ("taylor_cand", C.c_int64 * _S), ("taylor_kept", C.c_int64 * _S),
                ("sq_theta", C.c_double * _S), ("sq_normF", C.c_double * _S),
                ("sq_budget", C.c_double * _S), ("sq_dropped", C.c_double * _S),
                ("sq_iters", C.c_int * _S),
                ("sq_cand", C.c_int64 * _S), ("sq_kept", C.c_int64 * _S),
                ("nnz_e", C.c_int64), ("peak_workspace_bytes", C.c_size_t),
                ("sq_fma", C.c_int64 * _S), ("sq_in", C.c_int64 * _S),
                ("t_sym_ms", C.c_double * _S), ("t_num_ms", C.c_double * _S),
                ("t_filter_ms", C.c_double * _S),
                ("t_taylor_ms", C.c_double), ("t_backward_ms", C.c_double),
                ("t_total_ms", C.c_double),
                ("tile_launches", C.c_int64), ("tile_ms", C.c_double),
                ("tile_flops", C.c_double), ("adj_tile_launches", C.c_int64),
                ("adj_tile_ms", C.c_double), ("sq_tiles", C.c_int * _S),
                ("sq_ri", C.c_double * _S), ("sq_band", C.c_int64 * _S),
                ("theta0", C.c_double), ("tile_bytes", C.c_double),
                ("adj_tile_flops", C.c_double), ("adj_tile_bytes", C.c_double),
                ("ordering", C.c_int), ("adj_sparse_first", C.c_int), ("symmetric", C.c_int)]

    def to_dict(self) -> dict:
        d = {k: getattr(self, k) for k in ("status", "M", "N", "taylor_terms", "normal",
                                           "squarings", "a", "norm_h", "h0", "r0", "eg0",
                                           "nnz_e", "peak_workspace_bytes", "t_taylor_ms",
                                           "t_backward_ms", "t_total_ms", "tile_launches",
                                           "tile_ms", "tile_flops", "adj_tile_launches",
                                           "adj_tile_ms", "theta0", "tile_bytes",
                                           "adj_tile_flops", "adj_tile_bytes", "ordering",
                                           "adj_sparse_first", "symmetric")}
        T, N = self.taylor_terms, self.squarings
        for k in ("taylor_theta", "taylor_iters", "taylor_cand", "taylor_kept"):
            d[k] = list(getattr(self, k)[2:T + 2])
        for k in ("sq_theta", "sq_normF", "sq_budget", "sq_dropped", "sq_iters", "sq_cand",
                  "sq_kept", "sq_fma", "sq_in", "t_sym_ms", "t_num_ms", "t_filter_ms",
                  "sq_tiles", "sq_ri"):
            d[k] = list(getattr(self, k)[1:N + 1])
        d["sq_band"] = list(self.sq_band[0:N + 1])   # l(T^_0) .. l(T^_N), -1: not computed
        return d


class expm_analysis(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("norm_h", C.c_double),
                ("norm_fro", C.c_double), ("M", C.c_int), ("N", C.c_int), ("normal", C.c_int),
                ("a", C.c_double), ("h0", C.c_double), ("r0", C.c_double), ("eg0", C.c_double)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ExpmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = C.c_void_p


def lib():
    """The loaded gfx950 library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2110_04493_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        L.expm_opts_default.argtypes = [C.POINTER(expm_opts)]
        L.expm_opts_default.restype = None
        L.expm_plan.argtypes = [C.POINTER(_P), C.POINTER(expm_opts)]
        L.expm_sparse.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_double, C.POINTER(expm_csr)]
        L.expm_sparse_z.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_double,
                                    C.POINTER(expm_csr)]
        L.expm_sparse_backward.argtypes = [_P, _P, _P]
        L.expm_sparse_batched.argtypes = [_P, C.c_int, C.POINTER(expm_csr_cview),
                                          C.POINTER(C.c_double), C.POINTER(expm_csr)]
        L.expm_get_stats.argtypes = [_P, C.POINTER(expm_stats)]
        L.expm_csr_release.argtypes = [_P, C.POINTER(expm_csr)]
        L.expm_csr_release.restype = None
        L.expm_free.argtypes = [_P]
        L.expm_free.restype = None
        L.expm_last_error.argtypes = []
        L.expm_last_error.restype = C.c_char_p
        L.expm_r0.argtypes = [C.c_int, C.c_double]
        L.expm_r0.restype = C.c_double
        L.expm_choose_mn.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int),
                                     C.POINTER(C.c_int)]
        L.expm_sparse_noalloc.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_double, _P, _P,
                                          _P, C.c_int64, C.POINTER(C.c_int64)]
        L.expm_analyze.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_double,
                                   C.POINTER(expm_analysis)]
        L.expm_spmm.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_int64, _P, C.c_int64, _P,
                                C.c_int64]
        L.expm_propagate.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_int64, _P, C.c_int, _P]
        L.expm_power_norms.argtypes = [_P, C.POINTER(expm_csr_cview), C.c_int,
                                       C.POINTER(C.c_double)]
        L.expm_alpha_hat.argtypes = [C.c_double, C.c_int, C.c_int, C.c_double,
                                     C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int64)]
        for name in SYMBOLS:
            if name not in ("expm_opts_default", "expm_csr_release", "expm_free",
                            "expm_last_error", "expm_r0"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(code: int, where: str) -> None:
    if code != EXPM_OK:
        raise ExpmError(code, where, expm_last_error())


def expm_opts_default() -> expm_opts:
    o = expm_opts()
    lib().expm_opts_default(C.byref(o))
    return o


def expm_plan(opts: expm_opts) -> int:
    h = _P()
    check(lib().expm_plan(C.byref(h), C.byref(opts)), "expm_plan")
    return h.value


def expm_sparse(plan: int, H: expm_csr_cview, eps: float) -> expm_csr:
    E = expm_csr()
    check(lib().expm_sparse(_P(plan), C.byref(H), float(eps), C.byref(E)), "expm_sparse")
    return E


def expm_sparse_z(plan: int, H: expm_csr_cview, eps: float) -> expm_csr:
    """Complex H (val: nnz (real, imaginary) pairs of doubles)."""
    E = expm_csr()
    check(lib().expm_sparse_z(_P(plan), C.byref(H), float(eps), C.byref(E)), "expm_sparse_z")
    return E


def expm_sparse_noalloc(plan: int, H: expm_csr_cview, eps: float, rowptr_ptr: int,
                        col_ptr: int, val_ptr: int, capacity: int) -> int:
    """E into caller buffers (device pointers), workspace from the library's
    static scratch; returns nnz(E).  On an error the raised ExpmError
    carries nnz(E) in .nnz_e when it was known (-1 otherwise)."""
    nnz = C.c_int64(-1)
    code = lib().expm_sparse_noalloc(_P(plan), C.byref(H), float(eps), _P(rowptr_ptr),
                                     _P(col_ptr), _P(val_ptr), int(capacity), C.byref(nnz))
    if code != EXPM_OK:
        err = ExpmError(code, "expm_sparse_noalloc", expm_last_error())
        err.nnz_e = nnz.value
        raise err
    return nnz.value


def expm_analyze(plan: int, H: expm_csr_cview, eps: float) -> dict:
    a = expm_analysis()
    check(lib().expm_analyze(_P(plan), C.byref(H), float(eps), C.byref(a)), "expm_analyze")
    return a.to_dict()


def expm_spmm(plan: int, A: expm_csr_cview, m: int, X_ptr: int, ldx: int, Y_ptr: int,
              ldy: int) -> None:
    check(lib().expm_spmm(_P(plan), C.byref(A), int(m), _P(X_ptr), int(ldx), _P(Y_ptr),
                          int(ldy)), "expm_spmm")


def expm_propagate(plan: int, E: expm_csr_cview, m: int, U0_ptr: int, steps: int,
                   U_ptr: int) -> None:
    check(lib().expm_propagate(_P(plan), C.byref(E), int(m), _P(U0_ptr), int(steps),
                               _P(U_ptr)), "expm_propagate")


def expm_power_norms(plan: int, H: expm_csr_cview, K: int) -> list:
    out = (C.c_double * max(K, 1))()
    check(lib().expm_power_norms(_P(plan), C.byref(H), int(K), out), "expm_power_norms")
    return [out[k] for k in range(K)]


def expm_alpha_hat(ri: float, i: int, N: int, norm: float = 0.0, hk=None) -> int:
    out = C.c_int64()
    if hk is None:
        code = lib().expm_alpha_hat(float(ri), int(i), int(N), float(norm), None, 0,
                                    C.byref(out))
    else:
        arr = (C.c_double * len(hk))(*[float(x) for x in hk])
        code = lib().expm_alpha_hat(float(ri), int(i), int(N), 0.0, arr, len(hk), C.byref(out))
    check(code, "expm_alpha_hat")
    return out.value


def expm_sparse_backward(plan: int, dE_ptr: int, dH_ptr: int) -> None:
    check(lib().expm_sparse_backward(_P(plan), _P(dE_ptr), _P(dH_ptr)), "expm_sparse_backward")


def expm_sparse_batched(plan: int, H: list, eps: list) -> list:
    k = len(H)
    Harr = (expm_csr_cview * max(k, 1))(*H)
    earr = (C.c_double * max(k, 1))(*[float(e) for e in eps])
    Earr = (expm_csr * max(k, 1))()
    check(lib().expm_sparse_batched(_P(plan), k, Harr, earr, Earr), "expm_sparse_batched")
    return [Earr[j] for j in range(k)]


def expm_get_stats(plan: int) -> dict:
    s = expm_stats()
    check(lib().expm_get_stats(_P(plan), C.byref(s)), "expm_get_stats")
    return s.to_dict()


def expm_csr_release(plan: int, E: expm_csr) -> None:
    lib().expm_csr_release(_P(plan), C.byref(E))


def expm_free(plan: int) -> None:
    lib().expm_free(_P(plan))


def expm_last_error() -> str:
    return lib().expm_last_error().decode()


def expm_r0(M: int, x: float) -> float:
    return lib().expm_r0(int(M), float(x))


def expm_choose_mn(norm_h: float, eps: float) -> tuple[int, int]:
    M, N = C.c_int(), C.c_int()
    check(lib().expm_choose_mn(float(norm_h), float(eps), C.byref(M), C.byref(N)),
          "expm_choose_mn")
    return M.value, N.value
