"""GPU parity of the options and diagnostics beyond the default method:
the 1-norm for (M, N), the exact error recurrence of Eq. (4.3), the FPIM's
fixed filter (section 2), the bandwidths of the iterates (Eq. (3.1),
Table 3), the plan of steps 1-3 before a run, host-memory inputs, the norms
of the powers of H (section 4.2), and the action E R / time stepping of
section 5.3 and Eq. (2.2).  Same bar as the forward parity tests."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2110_04493_amd import workloads as W
from _helpers import compare, final_theta, run_gpu, run_oracle, to_device
from test_gpu_forward import check_parity
from test_gpu_adjoint import gpu_grad

pytestmark = pytest.mark.gpu
TOL = 1e-11
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def grid(side, seed, norm1):
    L = W.grid_laplacian(side, side, np.random.default_rng(seed))
    return L.scaled(-norm1 / W.norm1(L))


# ------------------------------------------------ norm, error recurrence, FPIM

@pytest.mark.parametrize("name,H,eps", [
    ("general", W.random_sparse(150, 0.03, 51, kind="general", scale=1.1), 1e-12),
    ("grid", grid(45, 52, 50.0), 1e-12)], ids=["general", "grid"])
def test_norm_one(name, H, eps):
    _, sg, _, so = check_parity(H, eps, norm=1)
    assert abs(sg["norm_h"] - so["nh"]) <= 1e-14 * so["nh"]


def test_exact_error_recurrence():
    H = grid(40, 53, 30.0)
    _, sg, _, so = check_parity(H, 1e-12, exact_ri=True)
    # the same recurrence from an r0 whose ||H|| was summed in another order
    for a, b in zip(sg["sq_ri"], so["sq_ri"]):
        assert abs(a - b) <= 1e-13 * b


@pytest.mark.parametrize("fill", [-1.0, 0.0, 2.0])
def test_fpim_fixed_filter(fill):
    """The FPIM's filter on both product paths (tiles and rows): the
    thresholds come from column sums taken in another order than the
    oracle's, so the kept sets may differ only at the threshold."""
    H = grid(50, 54, 40.0)
    Eg, sg = run_gpu(H, 1e-12, filter_mode=2, tile_min_fill=fill)
    Eo, so = run_oracle(H, 1e-12, filter_mode=2)
    rel, ok, og, oo = compare(Eg, Eo, so["sq_theta"][-1])
    print(f"[fpim fill={fill}] relF={rel:.2e} only={og},{oo}", flush=True)
    assert rel <= TOL and ok
    assert abs(sg["theta0"] - so["theta0"]) <= 1e-12 * so["theta0"]
    for a, b in zip(sg["sq_theta"], so["sq_theta"]):
        assert abs(a - b) <= 1e-12 * b
    for a, b in zip(sg["sq_kept"], so["sq_kept"]):
        assert abs(a - b) <= 0.002 * b + 2


def test_fpim_config1_and_adjoint():
    """Config 1 (10 tridiag(1,-2,1), n = 1000) under the FPIM, and the
    adjoint with the FPIM's masks frozen against the oracle's."""
    H, eps = W.config1()
    check_parity(H, eps, filter_mode=2)
    G = W.grid_laplacian(24, 24, np.random.default_rng(55)).scaled(-0.3)
    dg, _ = gpu_grad(G, 1e-12, density=0.2, filter_mode=2)
    run = oracle.Run(G.rowptr, G.col, G.val, 1e-12, filter_mode=2, keep=True)
    res = run.result()
    rows = np.repeat(np.arange(G.n), np.diff(res.rowptr))
    do = run.backward(W.loss_weights(rows, res.col, G.n, density=0.2))
    run.close()
    assert np.linalg.norm(dg - do) <= TOL * np.linalg.norm(do)


def test_batched_refuses_variants():
    from paper_2110_04493_amd import api, capi
    plan = api.Plan("cuda", api.Options(filter_mode=2))
    try:
        with pytest.raises(capi.ExpmError) as e:
            plan.expm_batched([to_device(W.tridiag(20, 1.0, -2.0, 1.0))], [1e-12])
        assert e.value.code == capi.EXPM_ENOTIMPL
    finally:
        plan.close()


# ------------------------------------------------ bandwidth diagnostics (Table 3)

@pytest.mark.parametrize("reorder", [0, 1])
def test_band_diagnostics_table3(reorder):
    """l(T^_i) per squaring, in the caller's ordering whether or not the
    library reorders internally: equal to the oracle's and to Table 3 row 1
    (tridiag(1,-2,1), n = 10^4, eps_tol = 1e-16)."""
    g = json.load(open(os.path.join(GOLD, "tables23.json")))
    H, eps = W.table2_matrix(g["n"])
    _, sg = run_gpu(H, eps, diagnostics=True, reorder=reorder)
    so = run_oracle(H, eps)[1]
    assert sg["sq_band"] == so["sq_band"]
    assert sg["sq_band"][1:] == g["table3_lambda_T_hat"]


def test_band_diagnostics_grid_reordered():
    H = grid(70, 56, 30.0)
    _, sg = run_gpu(H, 1e-12, diagnostics=True, reorder=1)
    so = run_oracle(H, 1e-12)[1]
    assert sg["sq_band"] == so["sq_band"]
    _, s0 = run_gpu(H, 1e-12)
    assert s0["sq_band"] == [-1] * (s0["N"] + 1)


# ------------------------------------------------ plan before the run, host inputs

@pytest.mark.parametrize("norm", [0, 1])
def test_analyze_matches_oracle_plan(norm):
    import torch
    from paper_2110_04493_amd import api
    H = W.random_sparse(120, 0.04, 57, kind="general", scale=0.9)
    plan = api.Plan("cuda", api.Options(norm=norm))
    try:
        A = plan.analyze(*to_device(H), 1e-12)
    finally:
        plan.close()
    so = run_oracle(H, 1e-12, norm=norm)[1]
    assert (A["M"], A["N"], A["normal"], A["n"], A["nnz"]) == (so["M"], so["N"], so["normal"],
                                                                H.n, H.nnz)
    for k, ko in (("norm_h", "nh"), ("a", "a"), ("h0", "h0"), ("r0", "r0"), ("eg0", "eg0")):
        assert abs(A[k] - so[ko]) <= 1e-13 * abs(so[ko]), k


def test_analyze_keeps_adjoint_state():
    """expm_analyze between a forward and its backward leaves the backward
    intact (it works on a scratch copy of its input)."""
    import torch
    from paper_2110_04493_amd import api
    H = grid(20, 58, 10.0)
    other = W.random_sparse(60, 0.05, 59, kind="general")
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True))
    try:
        rp, ci, v = plan.expm(*to_device(H), 1e-12)
        plan.analyze(*to_device(other), 1e-10)
        rows = np.repeat(np.arange(H.n), np.diff(rp.cpu().numpy()))
        g = W.loss_weights(rows, ci.cpu().numpy(), H.n, density=0.2)
        dH = plan.backward(torch.from_numpy(g).cuda(), H.nnz).cpu().numpy()
    finally:
        plan.close()
    run = oracle.Run(H.rowptr, H.col, H.val, 1e-12, keep=True)
    res = run.result()
    rows = np.repeat(np.arange(H.n), np.diff(res.rowptr))
    do = run.backward(W.loss_weights(rows, res.col, H.n, density=0.2))
    run.close()
    assert np.linalg.norm(dH - do) <= TOL * np.linalg.norm(do)


def test_host_inputs():
    """A view of host memory (on_host = 1) gives the same E as the device
    input."""
    import ctypes
    import torch
    from paper_2110_04493_amd import api, capi
    H = grid(30, 60, 20.0)
    Ed, _ = run_gpu(H, 1e-12)
    plan = api.Plan("cuda")
    try:
        rp, ci, v = (np.ascontiguousarray(H.rowptr), np.ascontiguousarray(H.col),
                     np.ascontiguousarray(H.val))
        view = capi.expm_csr_cview(H.n, H.nnz, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 1)
        E = capi.expm_sparse(plan.handle, view, 1e-12)
        erp, eci, ev = plan._take(E)
        torch.cuda.synchronize()
        Eh = W.Csr(H.n, erp.cpu().numpy(), eci.cpu().numpy(), ev.cpu().numpy())
    finally:
        plan.close()
    assert np.array_equal(Eh.rowptr, Ed.rowptr) and np.array_equal(Eh.col, Ed.col)
    assert np.array_equal(Eh.val, Ed.val)


# ------------------------------------------------ norms of powers (Eq. 4.9)

def test_power_norms():
    import torch
    from paper_2110_04493_amd import api
    H = W.tridiag(2000, 1.0, -2.0, 1.0)
    A = W.random_sparse(200, 0.02, 61, kind="general", scale=0.5)
    plan = api.Plan("cuda")
    try:
        g1 = plan.power_norms(*to_device(H), 41)
        g2 = plan.power_norms(*to_device(A), 12)
    finally:
        plan.close()
    o1 = oracle.power_norms((H.rowptr, H.col, H.val), 41)
    o2 = oracle.power_norms((A.rowptr, A.col, A.val), 12)
    # k products deep, each entry a sum with cancellation (alternating
    # signs in the powers of tridiag(1,-2,1)) rounded in another order and
    # with fused multiply-adds on the GPU: about k u of drift at power k
    assert np.max(np.abs(np.array(g1) / o1 - 1)) <= 41 * 2 ** -53 * 1000
    assert np.max(np.abs(np.array(g2) / o2 - 1)) <= 1e-13


# ------------------------------------------------ E R and time stepping

def gpu_spmm(E, X):
    import torch
    from paper_2110_04493_amd import api
    plan = api.Plan("cuda")
    try:
        Y = plan.spmm(*to_device(E), torch.from_numpy(X).cuda())
        torch.cuda.synchronize()
        return Y.cpu().numpy()
    finally:
        plan.close()


@pytest.mark.parametrize("m", [1, 37, 64, 130])
def test_spmm_kernel(m):
    """The product kernel on identical inputs: ragged column chunks, rows
    of every length up to several hundred, empty rows, n not a multiple of
    the four rows of a workgroup."""
    rng = np.random.default_rng(62 + m)
    A = W.random_sparse(1003, 0.01, 63, kind="general")
    A.val[A.rowptr[5]:A.rowptr[6]] = 0.0
    r = np.concatenate([A.rows(), np.full(700, 17)])
    c = np.concatenate([A.col.astype(np.int64), rng.integers(0, 1003, 700)])
    v = np.concatenate([A.val, rng.standard_normal(700)])
    A = W.csr_from_coo(1003, r, c, v)
    keep = A.rows() != 40
    A = W.csr_from_coo(1003, A.rows()[keep], A.col[keep], A.val[keep])
    X = rng.standard_normal((1003, m))
    Y = gpu_spmm(A, X)
    Yo = oracle.spmm((A.rowptr, A.col, A.val), X)
    assert np.linalg.norm(Y - Yo) <= 1e-14 * np.linalg.norm(Yo)


@pytest.mark.parametrize("m", [1, 37, 64, 130])
def test_spmm_tile_kernel(m):
    """The matrix-core product on 16 x 16 tiles (taken when the entries fill
    enough of their tiles): a dense band of half-width 20 with a few empty
    rows, n = 1003 (a partial last block row), ragged column chunks."""
    rng = np.random.default_rng(70 + m)
    n = 1003
    i = np.repeat(np.arange(n), 41)
    j = i + np.tile(np.arange(-20, 21), n)
    ok = (j >= 0) & (j < n) & (i % 97 != 5)
    A = W.csr_from_coo(n, i[ok], j[ok], rng.standard_normal(int(ok.sum())))
    X = rng.standard_normal((n, m))
    Y = gpu_spmm(A, X)
    Yo = oracle.spmm((A.rowptr, A.col, A.val), X)
    assert np.linalg.norm(Y - Yo) <= 1e-14 * np.linalg.norm(Yo)


def test_action_against_oracle():
    """Section 5.3's check E R, R = rand(n, m): the GPU's E times R against
    the oracle's E times R."""
    H = grid(40, 64, 30.0)
    Eg, _ = run_gpu(H, 1e-12)
    Eo, _ = run_oracle(H, 1e-12)
    R = np.random.default_rng(65).random((H.n, 100))
    Y = gpu_spmm(Eg, R)
    Yo = oracle.spmm((Eo.rowptr, Eo.col, Eo.val), R)
    assert np.linalg.norm(Y - Yo) <= TOL * np.linalg.norm(Yo)


def test_propagate():
    """Eq. (2.2): U_k = E^k U_0 by repeated products, in place and not."""
    import torch
    from paper_2110_04493_amd import api
    H = grid(25, 66, 5.0)
    Eo, _ = run_oracle(H, 1e-12)
    U0 = np.random.default_rng(67).standard_normal((H.n, 3))
    ref = U0
    for _ in range(5):
        ref = oracle.spmm((Eo.rowptr, Eo.col, Eo.val), ref)
    plan = api.Plan("cuda")
    try:
        dev = to_device(Eo)
        U = plan.propagate(*dev, torch.from_numpy(U0).cuda(), 5).cpu().numpy()
        U1 = plan.propagate(*dev, torch.from_numpy(U0).cuda(), 1).cpu().numpy()
        U0k = plan.propagate(*dev, torch.from_numpy(U0).cuda(), 0).cpu().numpy()
    finally:
        plan.close()
    assert np.linalg.norm(U - ref) <= 1e-13 * np.linalg.norm(ref)
    assert np.linalg.norm(U1 - oracle.spmm((Eo.rowptr, Eo.col, Eo.val), U0)) <= \
        1e-13 * np.linalg.norm(U1)
    assert np.array_equal(U0k, U0)


# ------------------------------------------------ level ordering (non-mesh inputs)

def scrambled_band(n, half, seed):
    """A banded matrix (half-bandwidth `half`) with its rows and columns
    permuted at random: no 2D structure, and a wide band in its own order."""
    rng = np.random.default_rng(seed)
    i = np.repeat(np.arange(n), 2 * half + 1)
    j = i + np.tile(np.arange(-half, half + 1), n)
    ok = (j >= 0) & (j < n)
    i, j = i[ok], j[ok]
    v = rng.standard_normal(i.size)
    keep = i <= j
    i, j, v = i[keep], j[keep], v[keep]
    r = np.concatenate([i, j[i != j]])
    c = np.concatenate([j, i[i != j]])
    w = np.concatenate([v, v[i != j]])
    p = rng.permutation(n)
    return W.csr_from_coo(n, p[r], p[c], w * 0.3)


def test_level_ordering_scrambled_band():
    """A scrambled band has no 2D structure: the default takes the level
    ordering, which narrows the band (fewer tiles in the last squaring) and
    leaves the result that of the method in the given order."""
    H = scrambled_band(6000, 3, 71)
    Eg, sg = run_gpu(H, 1e-12)
    Eo, so = run_oracle(H, 1e-12)
    rel, ok, _, _ = compare(Eg, Eo, final_theta(so))
    assert rel <= TOL and ok
    assert sg["ordering"] == 2
    # on tiles at every step, the last candidate needs far fewer tiles
    Et, st = run_gpu(H, 1e-12, tile_min_fill=0.0)
    _, s0 = run_gpu(H, 1e-12, reorder=0, tile_min_fill=0.0)
    assert st["ordering"] == 2 and s0["ordering"] == 0
    rel, ok, _, _ = compare(Et, Eo, final_theta(so))
    assert rel <= TOL and ok
    print(f"[level ordering] last-step tiles {st['sq_tiles'][-1]} vs {s0['sq_tiles'][-1]} in "
          "the given order", flush=True)
    assert 4 * st["sq_tiles"][-1] < s0["sq_tiles"][-1]


def test_level_ordering_forced_on_grid():
    H = grid(65, 72, 20.0)
    Eg, sg = run_gpu(H, 1e-12, reorder=2)
    assert sg["ordering"] == 2
    Eo, so = run_oracle(H, 1e-12)
    rel, ok, _, _ = compare(Eg, Eo, final_theta(so))
    assert rel <= TOL and ok
    _, s1 = run_gpu(H, 1e-12)
    assert s1["ordering"] == 1


# ------------------------------------------------ structural Hamiltonian, literal a

@pytest.mark.parametrize("side,dt,literal", [(40, 0.5, False), (40, 0.5, True), (100, 0.5, False)])
def test_structural_hamiltonian(side, dt, literal):
    """H = dt Theta of Eq. (2.1) for a damped mass-spring grid (n = 2 side^2,
    non-normal), with both readings of the filter constant."""
    H, _, _ = W.structural_hamiltonian(side, side, dt, alpha=0.02, beta=0.01, seed=3)
    _, sg, _, so = check_parity(H, 1e-12, literal_a=literal)
    assert sg["normal"] == 0 and abs(sg["a"] - so["a"]) <= 1e-14 * so["a"]


def test_literal_a_small_norm():
    """||H||_F = 2.5: 1/||H|| exceeds 1/(N+1), so the literal reading sets a
    larger filter constant; both runs agree with the oracle."""
    H, _, _ = W.structural_hamiltonian(12, 12, 1.0, alpha=0.05, beta=0.01, seed=13)
    H = H.scaled(2.5 / np.linalg.norm(H.val))
    _, s0, _, _ = check_parity(H, 1e-12, literal_a=False)
    _, s1, _, _ = check_parity(H, 1e-12, literal_a=True)
    assert s1["a"] > s0["a"] and abs(s1["a"] * s1["norm_h"] - 1.0) <= 1e-14
