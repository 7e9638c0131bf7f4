"""CPU oracle of Algorithm 4.2 over the complex numbers.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU leg use it to
check the GPU library's complex entry point; the library never imports it.

The paper states the method for H in C^{n x n} (section 4, problem (4.20)
and Algorithm 4.2).  This module follows the same steps as the real oracle
in ``oracle_expm.c``, with complex entries:

  step 1   (M, N) by problem (4.20) at ||H||_F (the real oracle's planner);
  step 2   a = 1/(N+1) when H is normal (H H^* = H^* H), else
           min(1/(N+1), 1/||H||_F) (1/||H||_F with ``literal_a``);
  step 3   H0 = H 2^-N, S_1 = H0, S_i = filter(S_{i-1} H0 / i) against the
           absolute budget eg0 = a r0 / (M e^{2 ||H0||}) of Eq. (4.14),
           stopping at the first term that filters to empty, T_0 = sum S_i;
  step 4   N times T~ = 2T + T T (Eq. (2.7)/(4.15)) and T = filter(T~)
           against a r_i ||I + T~||_F, r_i = 2^i r0 (or Eq. (4.3));
  step 5   E = I + T_N (exact zeros not stored);
  filter   Algorithm 4.1 on the moduli |z| = sqrt(re^2 + im^2): the dropped
           set of a threshold theta is {|z| <= theta}, its norm is
           sqrt(sum |z|^2) over that set.

A sparse product is formed from four real products of the real oracle
(each keeps the structural pattern: every (i, j) reached by some
a_ik b_kj, also where the values cancel), so that a candidate keeps its
exact zeros until the filter removes them, as in the real oracle; sums of
matrices are scipy's.  Nothing else is fused or reordered.

Parity status: pinned by tests/test_oracle_complex.py (the real oracle on
real inputs, closed forms of e^{-itL} from a symmetric eigensolver,
unitarity, scipy's dense expm, the normality cases, Algorithm 4.1 against
the real oracle's filter on the moduli)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import Result, choose_mn, r0, OracleError, EINVAL, ENOTCONV, ERANGE
from . import matmul as _real_matmul

MAXSTEP = 256


def _csr(n, rowptr, col, val) -> sp.csr_matrix:
    A = sp.csr_matrix((np.asarray(val, np.complex128), np.asarray(col, np.int64),
                       np.asarray(rowptr, np.int64)), shape=(n, n))
    A.has_sorted_indices = True
    return A


def _pattern(A: sp.csr_matrix) -> sp.csr_matrix:
    P = A.copy()
    P.data = np.ones(P.nnz)
    return P


def _aligned(C: sp.csr_matrix, pattern: sp.csr_matrix) -> sp.csr_matrix:
    """The values of C on `pattern` (a superset of C's stored entries):
    zeros where C holds none."""
    pattern = pattern.tocsr()
    pattern.sort_indices()
    C = C.tocsr()
    C.sort_indices()
    n = pattern.shape[0]
    rows_p = np.repeat(np.arange(n, dtype=np.int64), np.diff(pattern.indptr))
    rows_c = np.repeat(np.arange(n, dtype=np.int64), np.diff(C.indptr))
    kp = rows_p * n + pattern.indices.astype(np.int64)
    kc = rows_c * n + C.indices.astype(np.int64)
    v = np.zeros(kp.size, np.complex128)
    pos = np.searchsorted(kp, kc)
    assert np.all(kp[pos] == kc), "product entry outside its structural pattern"
    v[pos] = C.data
    out = sp.csr_matrix((v, pattern.indices.astype(np.int64), pattern.indptr.astype(np.int64)),
                        shape=pattern.shape)
    out.has_sorted_indices = True
    return out


def matmul(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """A B with its full structural pattern (exact zeros stored), from four
    real products by the real oracle's sparse product (which keeps the
    structural pattern): (Ar + i Ai)(Br + i Bi) = (Ar Br - Ai Bi) +
    i (Ar Bi + Ai Br).  The real and imaginary parts of a matrix share its
    pattern (explicit zeros kept), so the four products share the pattern
    of A B."""
    n = A.shape[0]
    def part(X, f):
        return (X.indptr.astype(np.int64), X.indices.astype(np.int32),
                np.ascontiguousarray(f(X.data)))
    re = lambda x: x.real
    im = lambda x: x.imag
    rr = _real_matmul(n, part(A, re), part(B, re))
    ii = _real_matmul(n, part(A, im), part(B, im))
    ri = _real_matmul(n, part(A, re), part(B, im))
    ir = _real_matmul(n, part(A, im), part(B, re))
    for x in (ii, ri, ir):
        assert np.array_equal(x[0], rr[0]) and np.array_equal(x[1], rr[1])
    v = np.empty(rr[2].size, np.complex128)
    v.real = rr[2] - ii[2]
    v.imag = ri[2] + ir[2]
    out = sp.csr_matrix((v, rr[1].astype(np.int64), rr[0]), shape=A.shape)
    out.has_sorted_indices = True
    return out


def add(alpha, A: sp.csr_matrix, beta, B: sp.csr_matrix, drop_zeros: bool) -> sp.csr_matrix:
    """alpha A + beta B on the union of the patterns; with drop_zeros the
    exact zeros of the sum are removed."""
    C = _aligned(alpha * A + beta * B, _pattern(A) + _pattern(B))
    if drop_zeros:
        C.eliminate_zeros()
    return C


def modulus(v: np.ndarray) -> np.ndarray:
    """|z| = sqrt(re^2 + im^2), each step rounded once."""
    re, im = v.real, v.imag
    return np.sqrt(re * re + im * im)


def filter_values(v: np.ndarray, eg: float, e_r: float = 0.1, max_iter: int = 64):
    """Algorithm 4.1 on complex values: the first trial threshold is the
    budget eg; while the norm d of the dropped set {|z| <= theta} exceeds
    eg (1 + e_r), the threshold becomes eg / (d / theta).  Returns (keep
    mask, theta, passes, d).  eg <= 0 keeps every nonzero."""
    v = np.asarray(v, np.complex128)
    mag = modulus(v)
    if eg <= 0.0:
        return mag != 0.0, 0.0, 0, 0.0
    sq = v.real * v.real + v.imag * v.imag
    theta = eg
    it = 0
    while True:
        if it >= max_iter:
            raise OracleError(ENOTCONV, "filter")
        d = float(np.sqrt(np.sum(sq[mag <= theta])))
        it += 1
        if d <= eg * (1.0 + e_r):
            break
        theta = eg / (d / theta)
    return mag > theta, theta, it, d


def _scaled(v: np.ndarray, f) -> np.ndarray:
    """f(real part) + i f(imaginary part), each part on its own."""
    out = np.empty_like(v)
    out.real = f(v.real)
    out.imag = f(v.imag)
    return out


def _select(A: sp.csr_matrix, keep: np.ndarray) -> sp.csr_matrix:
    n = A.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.indptr))
    counts = np.bincount(rows[keep], minlength=n)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    out = sp.csr_matrix((A.data[keep], A.indices[keep].astype(np.int64), rp), shape=A.shape)
    out.has_sorted_indices = True
    return out


def is_normal(H: sp.csr_matrix, nh: float) -> int:
    """Algorithm 4.2 step 2 over C: 1 if H equals +H^* or -H^* exactly
    (Hermitian or skew-Hermitian), else 1 if ||H H^* - H^* H||_F <=
    16 u ||H||_F^2 (u = 2^-53), else 0."""
    Hs = H.conj().T.tocsr()
    Hs.sort_indices()
    same = (np.array_equal(H.indptr, Hs.indptr) and np.array_equal(H.indices, Hs.indices))
    if same and (np.array_equal(H.data, Hs.data) or np.array_equal(H.data, -Hs.data)):
        return 1
    C = add(1.0, matmul(H, Hs), -1.0, matmul(Hs, H), False)
    c = float(np.sqrt(np.sum(C.data.real ** 2 + C.data.imag ** 2)))
    return int(c <= 16.0 * 2.0 ** -53 * nh * nh)


def expm(rowptr, col, val, eps: float, *, normal: int = -1, filter_mode: int = 0,
         e_r: float = 0.1, max_iter: int = 64, exact_ri: bool = False,
         literal_a: bool = False) -> Result:
    """E ~= e^H for a complex CSR matrix by Algorithm 4.2 (filter_mode 0:
    the paper's filter, 1: none, a = 0)."""
    rowptr = np.asarray(rowptr, np.int64)
    n = rowptr.size - 1
    col = np.asarray(col, np.int32)
    val = np.asarray(val, np.complex128)
    if not (2.0 ** -60 <= eps < 1.0) or not np.all(np.isfinite(val.view(np.float64))):
        raise OracleError(EINVAL, "expm_z")
    if filter_mode not in (0, 1):
        raise OracleError(EINVAL, "expm_z filter_mode")
    H = _csr(n, rowptr, col, val)
    st = {"taylor_theta": [], "taylor_iters": [], "taylor_cand": [], "taylor_kept": [],
          "sq_theta": [], "sq_normF": [], "sq_budget": [], "sq_dropped": [], "sq_iters": [],
          "sq_cand": [], "sq_kept": [], "sq_ri": []}
    nh = float(np.sqrt(np.sum(val.real ** 2 + val.imag ** 2)))
    st["nh"] = nh
    I = sp.identity(n, dtype=np.complex128, format="csr")
    if nh == 0.0:
        st.update(M=0, N=0, normal=1, a=0.0, h0=0.0, r0=0.0, eg0=0.0, taylor_terms=0,
                  squarings=0)
        return Result(n, I.indptr.astype(np.int64), I.indices.astype(np.int32), I.data.copy(), st)
    M, N = choose_mn(nh, eps)                                  # step 1
    if N >= MAXSTEP - 1 or M >= MAXSTEP - 1:
        raise OracleError(ERANGE, "expm_z")
    nrm = normal if normal >= 0 else is_normal(H, nh)          # step 2
    a = 1.0 / (N + 1)
    if not nrm and (literal_a or 1.0 / nh < a):
        a = 1.0 / nh
    if filter_mode == 1:
        a = 0.0
    H0 = H.copy()                                              # step 3
    H0.data = _scaled(H0.data, lambda x: np.ldexp(x, -N))
    h0 = float(np.ldexp(nh, -N))
    rr0 = r0(M, h0)
    eg0 = a * rr0 / (M * np.exp(2.0 * h0))
    st.update(M=M, N=N, normal=nrm, a=a, h0=h0, r0=rr0, eg0=eg0)
    S = H0
    T = H0.copy()
    terms = 1
    for i in range(2, M + 1):
        P = matmul(S, H0)
        P.data = _scaled(P.data, lambda x: x / i)
        keep, th, it, _ = filter_values(P.data, eg0, e_r, max_iter)
        st["taylor_cand"].append(P.nnz)
        st["taylor_theta"].append(th)
        st["taylor_iters"].append(it)
        S = _select(P, keep)
        st["taylor_kept"].append(S.nnz)
        if S.nnz == 0:
            break
        terms = i
        T = add(1.0, T, 1.0, S, True)                          # T0 += S_i
    st["taylor_terms"] = terms
    # per-term lists for i = 2 .. terms + 1, as the real oracle reports them
    # (the term after the last one is zero when it was never formed)
    for k, z in (("taylor_cand", 0), ("taylor_theta", 0.0), ("taylor_iters", 0),
                 ("taylor_kept", 0)):
        st[k] = (st[k] + [z] * terms)[:terms]
    ri = rr0                                                   # step 4
    for i in range(1, N + 1):
        Tt = add(2.0, T, 1.0, matmul(T, T), False)
        ri = 2.0 * ri + ri * ri if exact_ri else float(np.ldexp(rr0, i))
        F = add(1.0, I, 1.0, Tt, False)
        nF = float(np.sqrt(np.sum(F.data.real ** 2 + F.data.imag ** 2)))
        budget = a * ri * nF
        keep, th, it, d = filter_values(Tt.data, budget, e_r, max_iter)
        T = _select(Tt, keep)
        for k, x in (("sq_ri", ri), ("sq_normF", nF), ("sq_budget", budget), ("sq_theta", th),
                     ("sq_iters", it), ("sq_dropped", d), ("sq_cand", Tt.nnz),
                     ("sq_kept", T.nnz)):
            st[k].append(x)
    st["squarings"] = N
    E = add(1.0, I, 1.0, T, True)                              # step 5
    E.sort_indices()
    return Result(n, E.indptr.astype(np.int64), E.indices.astype(np.int32), E.data.copy(), st)
