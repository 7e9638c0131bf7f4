"""Seeded synthetic input generators.

This module builds the sparse matrices that both the GPU path and the CPU
oracle are run on.  It holds none of the exponential method's arithmetic:
only graph construction, random draws and the input scaling that defines a
workload.  Every generator returns host CSR arrays

    rowptr : int64[n+1]   col : int32[nnz]   val : float64[nnz]

with sorted, unique column indices in every row.

Workload families (the paper's heat-conduction and network-communicability
classes, section 5; the paper's own benchmark matrices are not available,
these synthetic families stand in for them):

* 1D heat conduction: ``s * tridiag(1, -2, 1)`` (section 5.2 uses this matrix).
* 2D heat conduction: graph Laplacian of a 5-point grid with lognormal or
  unit edge conductances, ``H = -tau * L``.
* Network communicability: ``H = beta * A`` with ``A`` a random symmetric
  adjacency matrix built by a configuration model.

Node numbering is natural row-major; grid edges are listed horizontal edges
first, then vertical edges, and edge conductances are drawn in that order.
Random draws use ``numpy.random.default_rng(1000 * config + instance)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Csr", "csr_from_coo", "tridiag", "grid_edges", "laplacian_from_edges",
    "grid_laplacian", "random_adjacency", "norm1", "config1", "config2",
    "config3", "config4_instance", "config4", "config5", "loss_weights",
    "random_sparse", "to_dense", "table2_matrix", "table4_matrix", "circulant",
    "perm_plus_identity", "structural_hamiltonian", "magnetic_laplacian", "schrodinger_grid",
    "complex_random",
]


@dataclass
class Csr:
    """Host CSR matrix (square)."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def scaled(self, s: float) -> "Csr":
        return Csr(self.n, self.rowptr.copy(), self.col.copy(), self.val * s, dict(self.meta))

    def rows(self) -> np.ndarray:
        """Row index of every stored entry."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.rowptr))


def csr_from_coo(n: int, r, c, v, *, sum_duplicates: bool = False, dtype=np.float64) -> Csr:
    """Sorted CSR from coordinates.  Duplicates keep the first occurrence
    unless ``sum_duplicates``.  ``dtype`` float64 or complex128."""
    r = np.asarray(r, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    v = np.asarray(v, dtype=dtype)
    key = r * n + c
    order = np.argsort(key, kind="stable")
    key = key[order]
    v = v[order]
    if key.size:
        first = np.ones(key.size, dtype=bool)
        first[1:] = key[1:] != key[:-1]
        if sum_duplicates:
            seg = np.cumsum(first) - 1
            m = int(first.sum())
            if np.iscomplexobj(v):
                v = np.bincount(seg, weights=v.real, minlength=m) \
                    + 1j * np.bincount(seg, weights=v.imag, minlength=m)
            else:
                v = np.bincount(seg, weights=v, minlength=m)
            key = key[first]
        else:
            key = key[first]
            v = v[first]
    rr = key // n
    cc = key % n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rr + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    return Csr(n, rowptr, cc.astype(np.int32), np.ascontiguousarray(v, dtype=dtype))


def to_dense(A: Csr) -> np.ndarray:
    D = np.zeros((A.n, A.n))
    D[A.rows(), A.col.astype(np.int64)] = A.val
    return D


def tridiag(n: int, lo: float, d: float, up: float, scale: float = 1.0) -> Csr:
    """``scale * tridiag(lo, d, up)`` of order n."""
    i = np.arange(n, dtype=np.int64)
    r = np.concatenate([i[1:], i, i[:-1]])
    c = np.concatenate([i[:-1], i, i[1:]])
    v = np.concatenate([np.full(n - 1, lo), np.full(n, d), np.full(n - 1, up)]) * scale
    return csr_from_coo(n, r, c, v)


def grid_edges(rows: int, cols: int, n_nodes: int | None = None):
    """Edges of a rows x cols 5-point grid, nodes numbered row-major.
    Horizontal edges first, then vertical edges.  With ``n_nodes`` only the
    first ``n_nodes`` nodes (and edges between them) are kept."""
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1)
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1)
    e = np.concatenate([h, v], axis=0)
    if n_nodes is not None:
        e = e[(e[:, 0] < n_nodes) & (e[:, 1] < n_nodes)]
    return e


def laplacian_from_edges(n: int, edges: np.ndarray, w: np.ndarray) -> Csr:
    """Weighted graph Laplacian L = D - K (diagonal = row sum of K)."""
    a, b = edges[:, 0], edges[:, 1]
    deg = np.zeros(n)
    np.add.at(deg, a, w)
    np.add.at(deg, b, w)
    r = np.concatenate([a, b, np.arange(n)])
    c = np.concatenate([b, a, np.arange(n)])
    v = np.concatenate([-w, -w, deg])
    return csr_from_coo(n, r, c, v)


def grid_laplacian(rows: int, cols: int, rng=None, sigma: float = 0.5,
                   n_nodes: int | None = None) -> Csr:
    """5-point grid Laplacian; lognormal(0, sigma) conductances if ``rng``
    is given, else unit conductances."""
    n = rows * cols if n_nodes is None else n_nodes
    e = grid_edges(rows, cols, n_nodes)
    w = np.ones(len(e)) if rng is None else rng.lognormal(0.0, sigma, len(e))
    return laplacian_from_edges(n, e, w)


def random_adjacency(n: int, rng, dmin: int = 4, dmax: int = 8) -> Csr:
    """Random symmetric weighted adjacency matrix by a configuration model:
    degrees uniform in {dmin..dmax}, stubs paired at random, self loops
    dropped, a repeated pair keeps its first weight; weights uniform in (0, 1]."""
    deg = rng.integers(dmin, dmax + 1, n)
    stubs = np.repeat(np.arange(n, dtype=np.int64), deg)
    if stubs.size % 2:
        stubs = stubs[:-1]
    rng.shuffle(stubs)
    a, b = stubs[0::2], stubs[1::2]
    w = 1.0 - rng.random(a.size)          # (0, 1]
    keep = a != b
    a, b, w = a[keep], b[keep], w[keep]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * n + hi
    _, first = np.unique(key, return_index=True)
    first = np.sort(first)
    lo, hi, w = lo[first], hi[first], w[first]
    return csr_from_coo(n, np.concatenate([lo, hi]), np.concatenate([hi, lo]),
                        np.concatenate([w, w]))


def norm1(A: Csr) -> float:
    """Max column absolute sum (used only to scale workloads)."""
    s = np.zeros(A.n)
    np.add.at(s, A.col.astype(np.int64), np.abs(A.val))
    return float(s.max()) if A.n else 0.0


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------

def config1() -> tuple[Csr, float]:
    """1D heat conduction: H = 10 * tridiag(1,-2,1), n = 1000, eps = 1e-14."""
    H = tridiag(1000, 1.0, -2.0, 1.0, 10.0)
    H.meta.update(name="tridiag_n1000", scale=10.0)
    return H, 1e-14


def config2(side: int = 300) -> tuple[Csr, float]:
    """2D heat conduction on a side x side grid (n = 90,000 at side 300),
    conductances lognormal(0, 0.5), H = -tau L with ||H||_1 = 50, eps = 1e-12."""
    rng = np.random.default_rng(2000)
    L = grid_laplacian(side, side, rng)
    tau = 50.0 / norm1(L)
    H = L.scaled(-tau)
    H.meta.update(name=f"grid{side}x{side}_lognormal", tau=tau)
    return H, 1e-12


def config3(side: int = 1448) -> tuple[Csr, float]:
    """Large 2D unit grid (n = 2,096,704 at side 1448), H = -0.5 L, eps = 1e-10."""
    L = grid_laplacian(side, side, None)
    H = L.scaled(-0.5)
    H.meta.update(name=f"grid{side}x{side}_unit", tau=0.5, side=side)
    return H, 1e-10


def config4_instance(j: int, nmin: int = 500, nmax: int = 20000) -> tuple[Csr, float]:
    """Instance j of the batched workload.  Even j: unit grid Laplacian with
    r = floor(sqrt(n)) rows, ceil(n/r) columns, first n nodes, H = -tau L,
    tau ~ U[1, 20].  Odd j: random adjacency, H = beta A, beta ~ U[0.1, 1]."""
    rng = np.random.default_rng(4000 + j)
    n = int(rng.integers(nmin, nmax + 1))
    if j % 2 == 0:
        r = int(math.isqrt(n))
        c = -(-n // r)
        tau = float(rng.uniform(1.0, 20.0))
        H = grid_laplacian(r, c, None, n_nodes=n).scaled(-tau)
        H.meta.update(name=f"grid_n{n}", tau=tau, kind="grid")
    else:
        beta = float(rng.uniform(0.1, 1.0))
        H = random_adjacency(n, rng).scaled(beta)
        H.meta.update(name=f"adjacency_n{n}", beta=beta, kind="adjacency")
    return H, 1e-12


def config4(count: int = 256, nmin: int = 500, nmax: int = 20000):
    return [config4_instance(j, nmin, nmax) for j in range(count)]


def config5(side: int = 200) -> tuple[Csr, float]:
    """Differentiation workload: side x side grid (n = 40,000 at side 200),
    conductances lognormal(0, 0.5), H = -5 L / ||L||_1, eps = 1e-12."""
    rng = np.random.default_rng(5000)
    L = grid_laplacian(side, side, rng)
    H = L.scaled(-5.0 / norm1(L))
    H.meta.update(name=f"grid{side}x{side}_lognormal_grad")
    return H, 1e-12


def table2_matrix(n: int = 10000) -> tuple[Csr, float]:
    """tridiag(1,-2,1) with eps_tol = 1e-16 (section 5.2, Tables 2 and 3)."""
    return tridiag(n, 1.0, -2.0, 1.0), 1e-16


def table4_matrix(n: int) -> Csr:
    """tridiag(-1,2,-1)/(n+1) (section 5.2, Table 4)."""
    return tridiag(n, -1.0, 2.0, -1.0, 1.0 / (n + 1))


# --------------------------------------------------------------------------
# Counter-based loss weights: G(i, j) for the loss sum(G .* E).
# --------------------------------------------------------------------------

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea and Flood, 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def loss_weights(rows, cols, n: int, density: float = 0.02, seed: int = 5000) -> np.ndarray:
    """Entries G(i, j) of a random sparse matrix with the given density and
    N(0, 1) values, evaluated at the positions (rows, cols).  G is defined
    position by position by a counter-based generator, so any support can be
    queried without forming G."""
    r = np.asarray(rows, dtype=np.uint64)
    c = np.asarray(cols, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = r * np.uint64(n) + c + (np.uint64(seed) << np.uint64(40))
    h1 = _splitmix64(key)
    h2 = _splitmix64(h1)
    h3 = _splitmix64(h2)
    scale = 2.0 ** -53
    u1 = (h1 >> np.uint64(11)).astype(np.float64) * scale
    u2 = ((h2 >> np.uint64(11)).astype(np.float64) + 1.0) * scale    # (0, 1]
    u3 = (h3 >> np.uint64(11)).astype(np.float64) * scale
    g = np.sqrt(-2.0 * np.log(u2)) * np.cos(2.0 * np.pi * u3)
    return np.where(u1 < density, g, 0.0)


def random_sparse(n: int, density: float, seed: int, kind: str = "general",
                  scale: float = 1.0, diag: bool = True) -> Csr:
    """Small random sparse test matrix: kind in general | symmetric | skew."""
    rng = np.random.default_rng(seed)
    m = max(1, int(round(density * n * n)))
    r = rng.integers(0, n, m)
    c = rng.integers(0, n, m)
    v = rng.standard_normal(m)
    if diag:
        r = np.concatenate([r, np.arange(n)])
        c = np.concatenate([c, np.arange(n)])
        v = np.concatenate([v, rng.standard_normal(n)])
    A = csr_from_coo(n, r, c, v)
    if kind == "general":
        return A.scaled(scale)
    D = to_dense(A)
    D = D + D.T if kind == "symmetric" else D - D.T
    rr, cc = np.nonzero(D)
    return csr_from_coo(n, rr, cc, D[rr, cc] * scale)


def circulant(n: int, offsets, values, bump: float = 0.0) -> Csr:
    """Sparse circulant matrix sum_k values[k] * P^offsets[k], P the cyclic
    shift (P[i, (i+1) mod n] = 1): normal and, for offsets not symmetric
    about 0, not symmetric.  ``bump`` is added to entry (0, 1), which makes
    the matrix non-normal by a controlled amount."""
    i = np.arange(n, dtype=np.int64)
    r = np.concatenate([i for _ in offsets])
    c = np.concatenate([(i + o) % n for o in offsets])
    v = np.concatenate([np.full(n, float(x)) for x in values])
    A = csr_from_coo(n, r, c, v, sum_duplicates=True)
    if bump:
        p = int(np.searchsorted(A.col[A.rowptr[0]:A.rowptr[1]], 1)) + int(A.rowptr[0])
        if p >= A.rowptr[1] or A.col[p] != 1:
            raise ValueError("entry (0, 1) must be stored to bump it")
        A.val[p] += bump
    return A


def perm_plus_identity(n: int, c: float, s: float, seed: int) -> Csr:
    """c I + s Q with Q the matrix of a random permutation without fixed
    points: normal (Q is orthogonal), not symmetric unless Q is an
    involution."""
    rng = np.random.default_rng(seed)
    while True:
        q = rng.permutation(n)
        if not np.any(q == np.arange(n)):
            break
    i = np.arange(n, dtype=np.int64)
    return csr_from_coo(n, np.concatenate([i, i]), np.concatenate([i, q]),
                        np.concatenate([np.full(n, c), np.full(n, s)]))


def structural_hamiltonian(rows: int, cols: int, dt: float, alpha: float = 0.0,
                           beta: float = 0.0, seed: int = 0, sigma: float = 0.3,
                           ground: float = 0.05) -> tuple[Csr, np.ndarray, np.ndarray]:
    """H = dt * Theta of Eq. (2.1) for a lumped mass-spring grid: masses m_i
    ~ lognormal(0, sigma) at the nodes of a rows x cols 5-point grid,
    springs of stiffness ~ lognormal(0, sigma) along its edges, and a
    grounding spring of stiffness ``ground`` at every node (so that K is
    positive definite).  Damping is Rayleigh's, C = alpha M + beta K.  The
    state is U = (a, v) (displacements, then velocities), so
        Theta = [[0, I], [-M^{-1} K, -M^{-1} C]],  n = 2 rows cols,
    and H is not normal.  Returns (H, m, K as a dense-free Csr of order
    rows cols): the masses and stiffness that define the energy norm
    U^T diag(K, M) U, which e^H preserves without damping and does not
    increase with it."""
    rng = np.random.default_rng(seed)
    m = rows * cols
    mass = rng.lognormal(0.0, sigma, m)
    e = grid_edges(rows, cols)
    K = laplacian_from_edges(m, e, rng.lognormal(0.0, sigma, len(e)))
    kd = K.val.copy()
    rr = np.repeat(np.arange(m, dtype=np.int64), np.diff(K.rowptr))
    kd[rr == K.col] += ground
    K = Csr(m, K.rowptr.copy(), K.col.copy(), kd)
    mk = kd / mass[rr]                        # M^{-1} K, row by row
    ident = np.arange(m, dtype=np.int64)
    r = np.concatenate([ident, m + rr, m + rr, m + ident])
    c = np.concatenate([m + ident, K.col.astype(np.int64), m + K.col.astype(np.int64), m + ident])
    v = np.concatenate([np.ones(m), -mk, -beta * mk, np.full(m, -alpha)])
    keep = v != 0.0
    H = csr_from_coo(2 * m, r[keep], c[keep], v[keep] * dt, sum_duplicates=True)
    return H, mass, K


# --------------------------------------------------------------------------
# Complex matrices (the method is stated for H in C^{n x n}).
# --------------------------------------------------------------------------

def magnetic_laplacian(rows: int, cols: int, seed: int = 0, sigma: float = 0.4,
                       phase: float = 0.7) -> Csr:
    """Hermitian magnetic Laplacian of a rows x cols 5-point grid: D - A with
    A_jk = w e^{i phi}, A_kj = w e^{-i phi} for each edge (j, k), weights
    w ~ lognormal(0, sigma), phases phi ~ U[-phase, phase], D the weighted
    degrees (complex128 values)."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    e = grid_edges(rows, cols)
    w = rng.lognormal(0.0, sigma, len(e))
    ph = rng.uniform(-phase, phase, len(e))
    deg = np.zeros(n)
    np.add.at(deg, e[:, 0], w)
    np.add.at(deg, e[:, 1], w)
    z = w * np.exp(1j * ph)
    return csr_from_coo(n, np.concatenate([e[:, 0], e[:, 1], np.arange(n)]),
                        np.concatenate([e[:, 1], e[:, 0], np.arange(n)]),
                        np.concatenate([-z, -np.conj(z), deg.astype(complex)]),
                        dtype=np.complex128)


def schrodinger_grid(side: int, t: float, vmax: float = 1.0, seed: int = 0) -> Csr:
    """H = -i t (L + V) for a side x side unit grid Laplacian L and a random
    potential V ~ U[0, vmax] on the diagonal: skew-Hermitian, so e^H is the
    unitary propagator of the discrete Schroedinger equation over time t."""
    rng = np.random.default_rng(seed)
    L = grid_laplacian(side, side)
    d = L.rows() == L.col
    v = L.val.astype(complex)
    v[d] += rng.uniform(0.0, vmax, side * side)
    return Csr(L.n, L.rowptr.copy(), L.col.copy(), np.ascontiguousarray(-1j * t * v))


def complex_random(n: int, density: float, seed: int, scale: float = 1.0) -> Csr:
    """Random sparse complex matrix (general, not normal): the pattern of
    random_sparse with independent N(0, scale^2) real and imaginary parts."""
    A = random_sparse(n, density, seed)
    rng = np.random.default_rng(seed + 1)
    v = scale * (rng.standard_normal(A.nnz) + 1j * rng.standard_normal(A.nnz))
    return Csr(n, A.rowptr, A.col, np.ascontiguousarray(v))
