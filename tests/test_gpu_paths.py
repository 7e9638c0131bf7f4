"""Both squaring paths (16x16 tiles on matrix cores, scalar rows) forced on
their own, with and without the locality reordering, forward and adjoint,
against the oracle.  tile_min_fill = 0 takes tiles at every squaring step,
2 never."""
import numpy as np
import pytest

from paper_2110_04493_amd import workloads as W
from _helpers import compare, final_theta, run_gpu, run_oracle
from test_gpu_adjoint import gpu_grad, oracle_grad

pytestmark = pytest.mark.gpu
TOL = 1e-11


def cases():
    rng = np.random.default_rng(11)
    L = W.grid_laplacian(33, 29, rng)                    # n not a multiple of 16
    yield "grid", L.scaled(-30.0 / W.norm1(L)), 1e-12
    yield "tridiag", W.tridiag(1000, 1.0, -2.0, 1.0, 10.0), 1e-14
    yield "general", W.random_sparse(150, 0.03, 3, kind="general", scale=1.2), 1e-12
    yield "adjacency", W.config4_instance(1, nmin=100, nmax=300)[0], 1e-12
    yield "disconnected", disconnected(), 1e-12
    yield "hub", hub(), 1e-12


def hub():
    """A grid plus one node joined to every seventh grid node: rows longer
    than the searches' fixed-width neighbour lists (eight slots) are read
    from the CSR rows instead."""
    rng = np.random.default_rng(13)
    A = W.grid_laplacian(24, 25, rng)
    m = A.n
    r = [A.rows()]
    c = [A.col.astype(np.int64)]
    v = [A.val]
    spokes = np.arange(0, m, 7)
    w = 0.05 * rng.uniform(0.5, 1.0, spokes.size)
    r += [np.full(spokes.size, m), spokes, [m]]
    c += [spokes, np.full(spokes.size, m), [m]]
    v += [w, w, [-w.sum()]]
    H = W.csr_from_coo(m + 1, np.concatenate(r), np.concatenate(c), np.concatenate(v))
    return H.scaled(-20.0 / W.norm1(H))


def disconnected():
    """Two components of different shape plus isolated nodes (empty rows)."""
    rng = np.random.default_rng(12)
    A = W.grid_laplacian(20, 23, rng).scaled(-0.4)
    B = W.tridiag(300, 1.0, -2.0, 1.0, 3.0)
    n = A.n + B.n + 5
    r = np.concatenate([A.rows(), B.rows() + A.n])
    c = np.concatenate([A.col.astype(np.int64), B.col.astype(np.int64) + A.n])
    v = np.concatenate([A.val, B.val])
    return W.csr_from_coo(n, r, c, v)


@pytest.mark.parametrize("reorder", [0, 1])
@pytest.mark.parametrize("fill", ["0", "2"])
@pytest.mark.parametrize("name,H,eps", list(cases()), ids=[c[0] for c in cases()])
def test_forward_paths(fill, reorder, name, H, eps):
    print(f"[{name} fill={fill} reorder={reorder}] n={H.n}", flush=True)
    Eg, sg = run_gpu(H, eps, reorder=reorder, tile_min_fill=float(fill))
    Eo, so = run_oracle(H, eps)
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[{name} fill={fill} reorder={reorder}] relF={rel:.2e} only={og},{oo}", flush=True)
    assert rel <= TOL and ok
    assert (sg["M"], sg["N"]) == (so["M"], so["N"])


@pytest.mark.parametrize("reorder", [0, 1])
@pytest.mark.parametrize("fill", ["0", "2"])
@pytest.mark.parametrize("name,H,eps", list(cases()), ids=[c[0] for c in cases()])
def test_adjoint_paths(fill, reorder, name, H, eps):
    print(f"[{name} fill={fill} reorder={reorder}] adjoint n={H.n}", flush=True)
    dg, _ = gpu_grad(H, eps, density=0.2, checkpoint_interval=2, reorder=reorder,
                     tile_min_fill=float(fill))
    do, _ = oracle_grad(H, eps, density=0.2)
    rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
    print(f"[{name} fill={fill} reorder={reorder}] adjoint rel={rel:.2e}", flush=True)
    assert rel <= TOL


@pytest.mark.parametrize("reorder", [0, 1])
def test_tiles_deterministic(reorder):
    H, eps = W.config5(40)
    E1, _ = run_gpu(H, eps, reorder=reorder, tile_min_fill=0.0)
    E2, _ = run_gpu(H, eps, reorder=reorder, tile_min_fill=0.0)
    assert np.array_equal(E1.col, E2.col)
    assert np.array_equal(E1.val.view(np.uint64), E2.val.view(np.uint64))


def test_reorder_matches_natural_order():
    """The permuted run returns the same E as the natural-order run up to
    rounding order (entries that flip across the threshold aside)."""
    H, eps = W.config5(60)
    Ea, sa = run_gpu(H, eps, reorder=0)
    Eb, sb = run_gpu(H, eps, reorder=1)
    rel, ok, og, oo = compare(Eb, Ea, sa["sq_theta"][-1])
    print(f"[reorder vs natural] relF={rel:.2e} only={og},{oo}", flush=True)
    assert rel <= 1e-13 and ok
    assert (sa["M"], sa["N"]) == (sb["M"], sb["N"])


def test_reorder_fills_tiles():
    """The locality ordering packs the band of a 60 x 60 grid into far fewer
    16 x 16 tiles than the natural order (every squaring on tiles; on the
    oracle's last iterate the strips need about half the tiles)."""
    H, eps = W.config5(60)
    _, sa = run_gpu(H, eps, reorder=0, tile_min_fill=0.0)
    _, sb = run_gpu(H, eps, reorder=1, tile_min_fill=0.0)
    ta, tb = sa["sq_tiles"][-1], sb["sq_tiles"][-1]   # steps 1 .. N in order
    print(f"[reorder tiles] last step: natural {ta}, ordered {tb}", flush=True)
    assert 0 < tb < 0.8 * ta


@pytest.mark.parametrize("reorder", [0, 1])
def test_adjoint_mixed_paths(reorder):
    """Fill thresholds between the two paths: the late squaring steps run on
    tiles and the early ones on scalar rows, so the adjoint hands its
    gradient from the tile steps to the row steps."""
    rng = np.random.default_rng(11)
    L = W.grid_laplacian(33, 29, rng)
    H, eps = L.scaled(-30.0 / W.norm1(L)), 1e-12
    do, _ = oracle_grad(H, eps, density=0.2)
    mixed = 0
    for fill in (0.05, 0.1, 0.15, 0.2, 0.3, 0.45):
        dg, st = gpu_grad(H, eps, density=0.2, checkpoint_interval=3, reorder=reorder,
                          tile_min_fill=fill)
        paths = [st["sq_tiles"][i] > 0 for i in range(st["N"])]
        rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
        print(f"[mixed reorder={reorder} fill={fill}] tiles per step {paths} rel={rel:.2e}",
              flush=True)
        assert rel <= TOL
        mixed += any(paths) and not all(paths)
    assert mixed > 0


@pytest.mark.parametrize("adjoint", [False, True])
def test_wide_rows_taylor_sum(adjoint):
    """A ring of 20,000 nodes in natural order: the rows of the first and
    last node span the whole index range, wider than the LDS slice of the
    multi-term Taylor sum, which then falls back to pairwise adds."""
    n = 20000
    T = W.tridiag(n, 1.0, -2.0, 1.0, 0.4)
    r = np.concatenate([T.rows(), [0, n - 1]])
    c = np.concatenate([T.col.astype(np.int64), [n - 1, 0]])
    v = np.concatenate([T.val, [0.4, 0.4]])
    H, eps = W.csr_from_coo(n, r, c, v), 1e-12
    if adjoint:
        dg, _ = gpu_grad(H, eps, density=0.05, reorder=0)
        do, _ = oracle_grad(H, eps, density=0.05)
        rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
        print(f"[wide rows] adjoint rel={rel:.2e}", flush=True)
        assert rel <= TOL
        return
    Eg, sg = run_gpu(H, eps, reorder=0)
    Eo, so = run_oracle(H, eps)
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[wide rows] M={sg['M']} N={sg['N']} terms={sg['taylor_terms']} relF={rel:.2e}",
          flush=True)
    assert rel <= TOL and ok


@pytest.mark.parametrize("adjoint", [False, True])
def test_dense_rows_taylor_sum(adjoint):
    """A random matrix whose Taylor seed has rows of several hundred
    distinct columns in a narrow window: the multi-term sum accumulates
    those rows densely, block by block."""
    H, eps = W.random_sparse(700, 0.012, 21, kind="general", scale=2.0), 1e-12
    if adjoint:
        dg, _ = gpu_grad(H, eps, density=0.05)
        do, _ = oracle_grad(H, eps, density=0.05)
        rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
        print(f"[dense rows] adjoint rel={rel:.2e}", flush=True)
        assert rel <= TOL
        return
    Eg, sg = run_gpu(H, eps)
    Eo, so = run_oracle(H, eps)
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[dense rows] M={sg['M']} N={sg['N']} terms={sg['taylor_terms']} "
          f"nnz(E)/n={Eg.nnz / H.n:.0f} relF={rel:.2e}", flush=True)
    assert rel <= TOL and ok


@pytest.mark.parametrize("adjoint", [False, True])
def test_long_column_taylor_adjoint(adjoint):
    """A ring of 1,500 nodes with one full column: every Taylor term has a
    column of about n entries, so the Taylor adjoint's inner products read
    that column from memory rather than from its LDS stage (512 entries)."""
    n = 1500
    T = W.tridiag(n, 1.0, -2.0, 1.0, 0.4)
    r = np.concatenate([T.rows(), [0, n - 1], np.arange(2, n - 1)])
    c = np.concatenate([T.col.astype(np.int64), [n - 1, 0], np.zeros(n - 3, np.int64)])
    v = np.concatenate([T.val, [0.4, 0.4], np.full(n - 3, 0.05)])
    H, eps = W.csr_from_coo(n, r, c, v), 1e-12
    assert np.count_nonzero(H.col == 0) > 512
    if adjoint:
        dg, _ = gpu_grad(H, eps, density=0.05)
        do, _ = oracle_grad(H, eps, density=0.05)
        rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
        print(f"[long column] adjoint rel={rel:.2e}", flush=True)
        assert rel <= TOL
        return
    Eg, sg = run_gpu(H, eps)
    Eo, so = run_oracle(H, eps)
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[long column] M={sg['M']} N={sg['N']} terms={sg['taylor_terms']} relF={rel:.2e}",
          flush=True)
    assert rel <= TOL and ok


def test_row_product_global_scratch():
    """A row whose accumulator does not fit the largest LDS class: a dense
    first row on a tridiagonal matrix of order 9000.  The product's row 0
    then has 9000 candidate columns, 8 * 9000 + 8 * ceil(9000 / 32) = 74,256
    bytes of accumulator and rank table, above the 65,536-byte LDS class, so
    the row products run it on global scratch.  Scalar rows only (no tiles),
    natural order."""
    n = 9000
    T = W.tridiag(n, 1.0, -2.0, 1.0, 0.5)
    rng = np.random.default_rng(77)
    r = np.concatenate([T.rows(), np.zeros(n, np.int64)])
    c = np.concatenate([T.col.astype(np.int64), np.arange(n)])
    v = np.concatenate([T.val, 1e-2 * rng.uniform(0.1, 1.0, n)])
    H = W.csr_from_coo(n, r, c, v, sum_duplicates=True)
    assert 8 * n + 8 * ((n + 31) // 32) > 65536
    Eg, sg = run_gpu(H, 1e-12, reorder=0, tile_min_fill=2.0)
    Eo, so = run_oracle(H, 1e-12)
    assert np.all(np.diff(Eo.rowptr)[:10] == n)          # dense rows reached the output
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[global scratch rows] relF={rel:.2e} only={og},{oo}", flush=True)
    assert rel <= TOL and ok
    assert (sg["M"], sg["N"]) == (so["M"], so["N"])


_WORK_ORDER_CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[2])
sys.path.insert(0, sys.argv[3])
from paper_2110_04493_amd import workloads as W
from test_gpu_adjoint import gpu_grad
from _helpers import run_gpu
H, eps = W.config5(48)
E, _ = run_gpu(H, eps, tile_min_fill=0.0)
dH, _ = gpu_grad(H, eps, density=0.2, tile_min_fill=0.0)
np.savez(sys.argv[1], col=E.col, val=E.val, dH=dH)
"""


def test_work_order_does_not_change_bits(tmp_path):
    """The tile product and adjoint kernels give every work item the same
    arithmetic wherever it runs: a child process with the work items in the
    hardware's round-robin order over the XCDs (EXPM_TILE_XCD=0) returns the
    same bits of E and dL/dH as the default per-XCD ranges."""
    import os
    import subprocess
    import sys
    H, eps = W.config5(48)
    E, _ = run_gpu(H, eps, tile_min_fill=0.0)
    dH, _ = gpu_grad(H, eps, density=0.2, tile_min_fill=0.0)
    out = tmp_path / "rr.npz"
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, EXPM_TILE_XCD="0")
    print("[work order] child with round-robin work items", flush=True)
    r = subprocess.run([sys.executable, "-c", _WORK_ORDER_CHILD, str(out), os.path.dirname(here),
                        here], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    z = np.load(out)
    assert np.array_equal(z["col"], E.col)
    assert np.array_equal(z["val"].view(np.uint64), E.val.view(np.uint64))
    assert np.array_equal(z["dH"].view(np.uint64), dH.view(np.uint64))


def grid_plus(extra):
    """A 24 x 24 grid, H = -0.5 L, plus one more node m whose entries extra(m)
    lists as (row, column, value)."""
    rng = np.random.default_rng(21)
    A = W.grid_laplacian(24, 24, rng).scaled(-0.5)
    m = A.n
    r, c, v = [A.rows()], [A.col.astype(np.int64)], [A.val]
    for i, j, x in extra(m):
        r.append([i])
        c.append([j])
        v.append([x])
    return W.csr_from_coo(m + 1, np.concatenate(r), np.concatenate(c), np.concatenate(v)), m


def diagonal_cases():
    # a node joined to the grid by 1e-7: T_N's diagonal there (about 5e-15)
    # falls under the last threshold (6.4e-15), so E takes the diagonal 1 of
    # I alone in a row that has other entries
    yield "pendant", *grid_plus(lambda m: [(m, 100, 1e-7), (100, m, 1e-7)])
    # an isolated node with h = -800: its t = e^h - 1 rounds to -1 exactly,
    # so E's diagonal there is exactly 0 and not stored
    yield "vanishing", *grid_plus(lambda m: [(m, m, -800.0)])


@pytest.mark.parametrize("reorder", [0, 1, 2])
@pytest.mark.parametrize("name,H,m", list(diagonal_cases()),
                         ids=[c[0] for c in diagonal_cases()])
def test_identity_at_the_diagonal(name, H, m, reorder):
    """E = I + T_N where T_N's diagonal is absent from a nonempty row, or
    where 1 + t is exactly zero: in the natural order, and with the
    permutation back from the locality order adding the identity on its way
    (reorder 2 forces an ordering); forward and adjoint against the oracle."""
    eps = 1e-12
    print(f"[{name} reorder={reorder}] n={H.n}", flush=True)
    Eg, sg = run_gpu(H, eps, reorder=reorder)
    Eo, so = run_oracle(H, eps)
    if reorder == 2:
        assert sg["ordering"] != 0
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[{name} reorder={reorder}] relF={rel:.2e} only={og},{oo}", flush=True)
    assert rel <= TOL and ok, (rel, og, oo)
    row = lambda E: slice(E.rowptr[m], E.rowptr[m + 1])
    if name == "pendant":
        assert Eo.col[row(Eo)][-1] == m and Eo.val[row(Eo)][-1] == 1.0
        assert Eg.col[row(Eg)][-1] == m and Eg.val[row(Eg)][-1] == 1.0
        assert Eg.rowptr[m + 1] - Eg.rowptr[m] > 1
    else:
        assert Eo.rowptr[m + 1] == Eo.rowptr[m] and Eg.rowptr[m + 1] == Eg.rowptr[m]
    dg, _ = gpu_grad(H, eps, density=0.3, reorder=reorder)
    do, _ = oracle_grad(H, eps, density=0.3)
    rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
    print(f"[{name} reorder={reorder}] adjoint rel={rel:.2e}", flush=True)
    assert rel <= TOL


def advection(side, c, seed):
    """H = -(L + A) on a side x side grid: L a grid Laplacian with lognormal
    conductances, A an upwind difference along x with weight c (unsymmetric,
    so every iterate is), scaled to ||H||_1 = 20."""
    L = W.grid_laplacian(side, side, np.random.default_rng(seed))
    node = np.arange(side * side).reshape(side, side)
    a, b = node[:, :-1].ravel(), node[:, 1:].ravel()
    r = np.concatenate([L.rows(), a, a])
    col = np.concatenate([L.col.astype(np.int64), a, b])
    v = np.concatenate([L.val, np.full(a.size, c), np.full(a.size, -c)])
    H = W.csr_from_coo(side * side, r, col, v, sum_duplicates=True).scaled(-1.0)
    return H.scaled(20.0 / W.norm1(H))


@pytest.mark.parametrize("reorder", [1, 2])
def test_ordering_unsymmetric(reorder):
    """An unsymmetric H with 2D structure under the orderings (strips, and
    the level ordering forced): the permutation back adds I to an
    unsymmetric T'_N, and the adjoint's first step reads dL/dE through its
    entry map; forward and adjoint against the oracle."""
    H = advection(40, 0.8, 33)
    eps = 1e-12
    print(f"[advection reorder={reorder}] n={H.n} nnz={H.nnz}", flush=True)
    Eg, sg = run_gpu(H, eps, reorder=reorder)
    Eo, so = run_oracle(H, eps)
    assert sg["symmetric"] == 0 and sg["ordering"] == reorder   # strips, levels
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[advection reorder={reorder}] ordering={sg['ordering']} relF={rel:.2e} "
          f"only={og},{oo} nnz={Eg.nnz}", flush=True)
    assert rel <= TOL and ok
    dg, _ = gpu_grad(H, eps, density=0.3, reorder=reorder)
    do, _ = oracle_grad(H, eps, density=0.3)
    rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
    print(f"[advection reorder={reorder}] adjoint rel={rel:.2e}", flush=True)
    assert rel <= TOL
