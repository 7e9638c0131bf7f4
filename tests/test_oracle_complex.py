"""Pins of the complex oracle (Algorithm 4.2 over C) against what does not
come from it:

  * real inputs: the real oracle (plain C, pinned on its own) gives the same
    E, (M, N), thresholds and counts;
  * Algorithm 4.1 on complex values equals the real oracle's Algorithm 4.1
    on their moduli (same threshold, passes and dropped norm);
  * skew-Hermitian H = -i t L (L a weighted path or grid Laplacian): the
    closed form V diag(e^{-i t lambda}) V^T from a symmetric eigensolver
    (the grid through its Kronecker factors), and E unitary;
  * Hermitian H (a magnetic Laplacian, complex phases on the edges):
    V diag(e^{lambda}) V^* from a Hermitian eigensolver, E Hermitian;
  * general complex H: scipy's dense expm within the tolerance;
  * Algorithm 4.2 step 2: normal and non-normal complex matrices are told
    apart (complex circulants are normal without being Hermitian);
  * e^{conj H} = conj(e^H) bit for bit."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from oracle import complex_expm as Z
from paper_2110_04493_amd import workloads as W


def dense(res):
    E = np.zeros((res.n, res.n), complex)
    rows = np.repeat(np.arange(res.n), np.diff(res.rowptr))
    E[rows, res.col] = res.val
    return E


def rel(A, B):
    return np.linalg.norm(A - B) / np.linalg.norm(B)


@pytest.mark.parametrize("eps,mode", [(1e-8, 0), (1e-12, 0), (1e-12, 1)])
def test_real_input_matches_real_oracle(eps, mode):
    L = W.grid_laplacian(18, 17, np.random.default_rng(2)).scaled(-0.7)
    rz = Z.expm(L.rowptr, L.col, L.val.astype(complex), eps, filter_mode=mode)
    rr = oracle.expm(L.rowptr, L.col, L.val, eps, filter_mode=mode)
    assert np.array_equal(rz.rowptr, rr.rowptr) and np.array_equal(rz.col, rr.col)
    assert np.all(rz.val.imag == 0)
    assert np.abs(rz.val.real - rr.val).max() <= 1e-15 * np.abs(rr.val).max()
    for k in ("M", "N", "normal", "taylor_terms"):
        assert rz.stats[k] == rr.stats[k], k
    for k in ("sq_kept", "sq_cand", "taylor_kept", "taylor_cand", "sq_iters", "taylor_iters"):
        assert list(rz.stats[k]) == list(rr.stats[k]), k
    for a, b in zip(rz.stats["sq_theta"], rr.stats["sq_theta"]):
        assert abs(a - b) <= 1e-12 * max(b, 1e-300)


def test_filter_equals_real_filter_on_moduli():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(5000) * np.exp(rng.uniform(-20, 0, 5000)) \
        + 1j * rng.standard_normal(5000) * np.exp(rng.uniform(-20, 0, 5000))
    mag = Z.modulus(v)
    for eg in (1e-9, 1e-6, 1e-3):
        kz, tz, iz, dz = Z.filter_values(v, eg)
        kr, tr, ir, dr = oracle.filter_values(mag, eg)
        assert iz == ir and np.array_equal(kz, kr)
        assert abs(tz - tr) <= 1e-14 * tr and abs(dz - dr) <= 1e-13 * dr


def path_laplacian(n, w):
    """Weighted path Laplacian, dense."""
    L = np.zeros((n, n))
    for k, x in enumerate(w):
        L[k, k] += x
        L[k + 1, k + 1] += x
        L[k, k + 1] -= x
        L[k + 1, k] -= x
    return L


def test_skew_hermitian_closed_form_and_unitarity():
    rng = np.random.default_rng(4)
    n, t = 120, 3.0
    L = path_laplacian(n, rng.lognormal(0, 0.3, n - 1))
    H = -1j * t * L
    r, c = np.nonzero(H)
    Hs = W.csr_from_coo(n, r, c, np.zeros(r.size))
    res = Z.expm(Hs.rowptr, Hs.col, H[Hs.rows(), Hs.col], 1e-13)
    lam, V = np.linalg.eigh(L)
    exact = (V * np.exp(-1j * t * lam)) @ V.T
    E = dense(res)
    assert res.stats["normal"] == 1
    assert rel(E, exact) <= 1e-11
    assert np.linalg.norm(E @ E.conj().T - np.eye(n)) <= 1e-11 * np.sqrt(n)


def test_skew_hermitian_grid_kronecker():
    rng = np.random.default_rng(5)
    a, b, t = 14, 11, 1.2
    L1 = path_laplacian(a, rng.lognormal(0, 0.3, a - 1))
    L2 = path_laplacian(b, rng.lognormal(0, 0.3, b - 1))
    L = np.kron(L1, np.eye(b)) + np.kron(np.eye(a), L2)
    H = -1j * t * L
    r, c = np.nonzero(H)
    Hs = W.csr_from_coo(a * b, r, c, np.zeros(r.size))
    res = Z.expm(Hs.rowptr, Hs.col, H[Hs.rows(), Hs.col], 1e-12)
    def ex(Lk):
        lam, V = np.linalg.eigh(Lk)
        return (V * np.exp(-1j * t * lam)) @ V.T
    assert rel(dense(res), np.kron(ex(L1), ex(L2))) <= 1e-10


def magnetic_laplacian(side, seed, phase=0.7):
    """Hermitian: D - A with A_jk = w e^{i phi_jk}, phi_kj = -phi_jk."""
    rng = np.random.default_rng(seed)
    e = W.grid_edges(side, side)
    w = rng.lognormal(0, 0.4, len(e))
    ph = rng.uniform(-phase, phase, len(e))
    n = side * side
    H = np.zeros((n, n), complex)
    for (j, k), x, p in zip(e, w, ph):
        H[j, k] -= x * np.exp(1j * p)
        H[k, j] -= x * np.exp(-1j * p)
        H[j, j] += x
        H[k, k] += x
    return H


def test_hermitian_closed_form():
    D = -0.4 * magnetic_laplacian(9, 6)
    r, c = np.nonzero(D)
    Hs = W.csr_from_coo(D.shape[0], r, c, np.zeros(r.size))
    res = Z.expm(Hs.rowptr, Hs.col, D[Hs.rows(), Hs.col], 1e-13)
    lam, V = np.linalg.eigh(D)
    exact = (V * np.exp(lam)) @ V.conj().T
    E = dense(res)
    assert res.stats["normal"] == 1
    assert rel(E, exact) <= 1e-11
    assert np.linalg.norm(E - E.conj().T) <= 1e-12 * np.linalg.norm(E)


@pytest.mark.parametrize("seed,scale", [(7, 0.5), (8, 3.0)])
def test_general_against_dense_expm(seed, scale):
    rng = np.random.default_rng(seed)
    A = W.random_sparse(60, 0.06, seed, kind="general", scale=scale)
    v = A.val + 1j * scale * rng.standard_normal(A.nnz)
    res = Z.expm(A.rowptr, A.col, v, 1e-13)
    D = np.zeros((60, 60), complex)
    D[A.rows(), A.col] = v
    assert res.stats["normal"] == 0
    assert rel(dense(res), sl.expm(D)) <= 1e-11


def circulant_complex(n, offsets, values):
    i = np.arange(n)
    r = np.concatenate([i for _ in offsets])
    c = np.concatenate([(i + o) % n for o in offsets])
    v = np.concatenate([np.full(n, x) for x in values])
    D = np.zeros((n, n), complex)
    np.add.at(D, (r, c), v)
    return D


@pytest.mark.parametrize("kind,expect", [("circulant", 1), ("bumped", 0), ("hermitian", 1),
                                         ("skew", 1), ("random", 0)])
def test_normality(kind, expect):
    rng = np.random.default_rng(9)
    if kind in ("circulant", "bumped"):
        D = circulant_complex(50, [0, 1, 3], [0.2 + 0.1j, 1.0 - 0.5j, 0.3j])
        if kind == "bumped":
            D[0, 1] += 1e-3
    elif kind == "hermitian":
        D = -0.3 * magnetic_laplacian(6, 10)
    elif kind == "skew":
        D = 1j * 0.3 * magnetic_laplacian(6, 11)
    else:
        D = np.where(rng.random((40, 40)) < 0.1,
                     rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40)), 0)
    r, c = np.nonzero(D)
    Hs = W.csr_from_coo(D.shape[0], r, c, np.zeros(r.size))
    res = Z.expm(Hs.rowptr, Hs.col, D[Hs.rows(), Hs.col], 1e-12)
    assert res.stats["normal"] == expect
    if kind in ("circulant", "bumped"):
        assert rel(dense(res), sl.expm(D)) <= 1e-10


def test_conjugate_symmetry():
    rng = np.random.default_rng(12)
    A = W.random_sparse(50, 0.08, 12, kind="general", scale=1.5)
    v = A.val + 1j * rng.standard_normal(A.nnz)
    r1 = Z.expm(A.rowptr, A.col, v, 1e-12)
    r2 = Z.expm(A.rowptr, A.col, np.conj(v), 1e-12)
    assert np.array_equal(r1.col, r2.col) and np.array_equal(r1.val, np.conj(r2.val))


def test_zero_and_taylor_only():
    A = W.random_sparse(30, 0.1, 13, scale=1e-3)
    v = A.val * (1 + 1j)
    res = Z.expm(A.rowptr, A.col, v, 1e-14)
    assert res.stats["N"] == 0
    D = np.zeros((30, 30), complex)
    D[A.rows(), A.col] = v
    assert rel(dense(res), sl.expm(D)) <= 1e-13
    z = Z.expm(A.rowptr, A.col, np.zeros(A.nnz, complex), 1e-12)
    assert np.array_equal(dense(z), np.eye(30))
