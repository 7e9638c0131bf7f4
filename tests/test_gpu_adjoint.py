"""GPU parity of the adjoint (expm_sparse_backward / ExpmFn) against the
oracle's frozen-mask adjoint: relative Frobenius error of dL/d(vals of H)
<= 1e-11 for L = sum(G .* E), G a counter-based synthetic sparse matrix."""
import numpy as np
import pytest

import oracle
from paper_2110_04493_amd import workloads as W
from _helpers import to_device

pytestmark = pytest.mark.gpu
TOL = 1e-11


def gpu_grad(H, eps, density=0.3, seed=5000, **opts):
    import torch
    from paper_2110_04493_amd import api
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True, **opts))
    try:
        rp, ci, v = plan.expm(*to_device(H), eps)
        rows = np.repeat(np.arange(H.n), np.diff(rp.cpu().numpy()))
        g = W.loss_weights(rows, ci.cpu().numpy(), H.n, density=density, seed=seed)
        dH = plan.backward(torch.from_numpy(g).cuda(), H.nnz)
        torch.cuda.synchronize()
        st = plan.stats()
    finally:
        plan.close()
    return dH.cpu().numpy(), st


def oracle_grad(H, eps, density=0.3, seed=5000, **kw):
    run = oracle.Run(H.rowptr, H.col, H.val, eps, **kw)
    res = run.result()
    rows = np.repeat(np.arange(H.n), np.diff(res.rowptr))
    dH = run.backward(W.loss_weights(rows, res.col, H.n, density=density, seed=seed))
    run.close()
    return dH, res.stats


def check(H, eps, density=0.3, **opts):
    print(f"[adjoint] n={H.n} nnz={H.nnz} eps={eps} {opts}", flush=True)
    okw = {k: v for k, v in opts.items() if k in ("filter_mode", "normal")}
    dg, sg = gpu_grad(H, eps, density, **opts)
    do, so = oracle_grad(H, eps, density, **okw)
    rel = np.linalg.norm(dg - do) / max(np.linalg.norm(do), 1e-300)
    print(f"  rel={rel:.3e} N={sg['N']} M={sg['M']} taylor={sg['taylor_terms']}", flush=True)
    assert (sg["M"], sg["N"]) == (so["M"], so["N"])
    assert rel <= TOL
    return rel, sg


@pytest.mark.parametrize("kind,seed,scale", [("general", 2, 0.6), ("general", 3, 2.5),
                                             ("symmetric", 1, 1.0), ("skew", 4, 1.2)])
def test_random_small(kind, seed, scale):
    H = W.random_sparse(40, 0.06, seed, kind=kind, scale=scale)
    check(H, 1e-14)


@pytest.mark.parametrize("ck", [-1, 0, 1, 2, 100])
def test_grid_checkpoint_intervals(ck):
    rng = np.random.default_rng(3)
    L = W.grid_laplacian(24, 24, rng)
    H = L.scaled(-5.0 / W.norm1(L))
    rel, st = check(H, 1e-12, density=0.05, checkpoint_interval=ck)
    assert st["N"] >= 3


def test_taylor_only_and_zero():
    H = W.random_sparse(20, 0.1, 8, scale=0.01)
    rel, st = check(H, 1e-14)
    assert st["N"] == 0
    Z = W.Csr(20, H.rowptr, H.col, np.zeros_like(H.val))
    dg, _ = gpu_grad(Z, 1e-14)
    assert np.all(dg == 0)


def test_filter_none():
    H = W.random_sparse(30, 0.08, 21, kind="general", scale=1.5)
    check(H, 1e-13, filter_mode=1)


def test_backward_without_checkpoints_is_an_error():
    import torch
    from paper_2110_04493_amd import api, capi
    H = W.tridiag(10, 1.0, -2.0, 1.0)
    plan = api.Plan("cuda")
    try:
        plan.expm(*to_device(H), 1e-12)
        with pytest.raises(capi.ExpmError) as e:
            plan.backward(torch.zeros(100, dtype=torch.float64, device="cuda"), H.nnz)
        assert e.value.code == capi.EXPM_ESTATE
    finally:
        plan.close()


def test_autograd_function():
    import torch
    from paper_2110_04493_amd import api
    rng = np.random.default_rng(7)
    L = W.grid_laplacian(16, 16, rng)
    H = L.scaled(-5.0 / W.norm1(L))
    crow, col, val = to_device(H)
    val = val.clone().requires_grad_(True)
    ev, erp, eci = api.ExpmFn.apply(crow, col, val, 1e-12)
    rows = np.repeat(np.arange(H.n), np.diff(erp.cpu().numpy()))
    g = torch.from_numpy(W.loss_weights(rows, eci.cpu().numpy(), H.n, density=0.2)).cuda()
    (ev * g).sum().backward()
    do, _ = oracle_grad(H, 1e-12, density=0.2)
    dg = val.grad.cpu().numpy()
    assert np.linalg.norm(dg - do) <= TOL * np.linalg.norm(do)


@pytest.mark.parametrize("ck", [0, -1])
def test_config5_reduced(ck):
    """The differentiation workload's family at 80 x 80 (n = 6,400), with
    the default checkpoints (every iterate fits) and with ceil(sqrt(N))
    checkpoints and recomputation."""
    H, eps = W.config5(80)
    check(H, eps, density=0.02, checkpoint_interval=ck)


def test_config5_full_size():
    """The differentiation workload at full size (n = 40,000)."""
    H, eps = W.config5()
    check(H, eps, density=0.02)


@pytest.mark.parametrize("density,sparse", [(0.004, 1), (0.3, 0)])
def test_sparse_incoming_gradient(density, sparse):
    """A loss on 0.4% of E's entries gives a dL/dE that is mostly exact
    zeros: the first adjoint step then runs on the rows of its nonzeros (a
    denser loss keeps the tiles); both agree with the oracle."""
    L = W.grid_laplacian(60, 60, np.random.default_rng(91))
    H = L.scaled(-30.0 / W.norm1(L))
    dg, st = gpu_grad(H, 1e-12, density=density)
    do, _ = oracle_grad(H, 1e-12, density=density)
    assert st["adj_sparse_first"] == sparse
    assert np.linalg.norm(dg - do) <= TOL * np.linalg.norm(do)
