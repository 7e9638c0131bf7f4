"""Pins of the oracle's adjoint (frozen-mask derivative of Algorithm 4.2).

* Frechet: for L = sum(G .* e^H), dL/dH = [expm([[H^T, G], [0, H^T]])]_12,
  restricted to the stored positions of H (dense scipy expm, small n).  The
  filtered method differs from e^H by its truncation, so the match is to the
  method's accuracy.
* Finite differences of the oracle's own forward map along random
  directions on supp(H).  With the filter off (plain precise integration,
  a = 0) the map is a polynomial in H and central differences converge; with
  the paper's filter the masks may flip inside the stencil, and the check is
  looser.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2110_04493_amd import workloads as W


def frechet_grad(H: W.Csr, Gd: np.ndarray) -> np.ndarray:
    n = H.n
    D = W.to_dense(H)
    B = np.zeros((2 * n, 2 * n))
    B[:n, :n] = D.T
    B[n:, n:] = D.T
    B[:n, n:] = Gd
    F = sla.expm(B)[:n, n:]
    return F[H.rows(), H.col.astype(np.int64)]


def loss_grad_E(res, n, seed=5000, density=0.3):
    rows = np.repeat(np.arange(n), np.diff(res.rowptr))
    return W.loss_weights(rows, res.col, n, density=density, seed=seed)


def dense_G(n, seed=5000, density=0.3):
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return W.loss_weights(r.ravel(), c.ravel(), n, density=density, seed=seed).reshape(n, n)


def skew_part(H: W.Csr, g: np.ndarray) -> np.ndarray:
    D = W.to_dense(W.Csr(H.n, H.rowptr, H.col, g))
    return (D - D.T)[H.rows(), H.col.astype(np.int64)]


@pytest.mark.parametrize("kind,seed,scale", [("symmetric", 1, 1.0), ("general", 2, 0.6),
                                             ("general", 3, 2.5), ("skew", 4, 1.2)])
def test_adjoint_matches_frechet(kind, seed, scale):
    """For skew-symmetric H the odd powers have exactly zero diagonals, which
    the filter drops although their derivative across non-skew directions is
    not small; along skew directions (the tangent space of the skew matrices)
    the two derivatives agree, so skew inputs compare the skew parts."""
    n = 40
    H = W.random_sparse(n, 0.06, seed, kind=kind, scale=scale)
    r = oracle.Run(H.rowptr, H.col, H.val, 1e-14)
    res = r.result()
    dE = loss_grad_E(res, n)
    dH = r.backward(dE)
    ref = frechet_grad(H, dense_G(n))
    if kind == "skew":
        dH, ref = skew_part(H, dH), skew_part(H, ref)
    assert np.linalg.norm(dH - ref) <= 1e-8 * np.linalg.norm(ref)
    r.close()


def test_adjoint_grid_frechet():
    """2D grid heat conduction, as in the differentiation workload, at n = 144."""
    rng = np.random.default_rng(3)
    L = W.grid_laplacian(12, 12, rng)
    H = L.scaled(-5.0 / W.norm1(L))
    r = oracle.Run(H.rowptr, H.col, H.val, 1e-12)
    res = r.result()
    dH = r.backward(loss_grad_E(res, H.n, density=0.02))
    ref = frechet_grad(H, dense_G(H.n, density=0.02))
    assert np.linalg.norm(dH - ref) <= 1e-8 * np.linalg.norm(ref)
    r.close()


def _loss(H, vals, eps, G_of, **kw):
    res = oracle.expm(H.rowptr, H.col, vals, eps, **kw)
    rows = np.repeat(np.arange(H.n), np.diff(res.rowptr))
    return float(np.dot(G_of(rows, res.col), res.val))


@pytest.mark.parametrize("filter_mode,tol", [(1, 1e-7), (0, 1e-6)])
def test_adjoint_finite_differences(filter_mode, tol):
    n = 30
    H = W.random_sparse(n, 0.08, 21, kind="general", scale=1.5)
    eps = 1e-13
    G_of = lambda r, c: W.loss_weights(r, c, n, density=0.5, seed=77)
    run = oracle.Run(H.rowptr, H.col, H.val, eps, filter_mode=filter_mode)
    res = run.result()
    rows = np.repeat(np.arange(n), np.diff(res.rowptr))
    dH = run.backward(G_of(rows, res.col))
    run.close()
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.standard_normal(H.nnz)
        h = 1e-5 * np.linalg.norm(H.val) / np.linalg.norm(d)
        # keep (M, N) and a fixed: the norm changes by O(h), far from a switch
        fp = _loss(H, H.val + h * d, eps, G_of, filter_mode=filter_mode)
        fm = _loss(H, H.val - h * d, eps, G_of, filter_mode=filter_mode)
        fd = (fp - fm) / (2 * h)
        an = float(np.dot(dH, d))
        assert abs(fd - an) <= tol * (abs(an) + np.linalg.norm(dH) * np.linalg.norm(d) * 1e-3)


def test_adjoint_taylor_only_and_zero():
    """Tiny norms give N = 0 (no squaring): the adjoint is that of the
    filtered Taylor polynomial alone; H = 0 gives a zero gradient."""
    n = 20
    H = W.random_sparse(n, 0.1, 8, scale=0.01)
    r = oracle.Run(H.rowptr, H.col, H.val, 1e-14)
    res = r.result()
    assert res.stats["N"] == 0
    dH = r.backward(loss_grad_E(res, n))
    ref = frechet_grad(H, dense_G(n))
    assert np.linalg.norm(dH - ref) <= 1e-9 * np.linalg.norm(ref)
    r.close()
    Z = W.Csr(n, H.rowptr, H.col, np.zeros_like(H.val))
    r = oracle.Run(Z.rowptr, Z.col, Z.val, 1e-14)
    res = r.result()
    assert np.all(r.backward(np.ones(res.val.size)) == 0)
    r.close()
