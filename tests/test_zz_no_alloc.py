"""expm_sparse_noalloc: the forward computation with its workspace in the
library's static device scratch and E in caller buffers.  Checked through
the C ABI against expm_sparse on the same plan, to the parity bar (relative
Frobenius error over the union of supports <= 1e-11, entries in only one
support within a factor 2 of the final threshold; the two run the same
kernels in the same order, so they are expected to agree exactly), and
against the oracle; two calls in a row, the second on a smaller input."""
import numpy as np
import pytest

from paper_2110_04493_amd import workloads as W
from _helpers import compare, final_theta, run_oracle, to_device

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _noalloc(plan, H, eps, capacity):
    import torch
    from paper_2110_04493_amd import api, capi
    crow, col, val = to_device(H)
    rp = torch.full((H.n + 1,), -7, dtype=torch.int64, device="cuda")
    ci = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda")
    v = torch.empty(max(capacity, 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    nnz = capi.expm_sparse_noalloc(plan.handle, api._view(crow, col, val), eps, rp.data_ptr(),
                                   ci.data_ptr(), v.data_ptr(), capacity)
    plan.stream.synchronize()
    return W.Csr(H.n, rp.cpu().numpy(), ci[:nnz].cpu().numpy(), v[:nnz].cpu().numpy())


def _grid(side, seed, norm1=30.0):
    L = W.grid_laplacian(side, side, np.random.default_rng(seed))
    return L.scaled(-norm1 / W.norm1(L))


def test_noalloc_matches_expm_sparse_two_calls():
    import torch
    from paper_2110_04493_amd import api
    plan = api.Plan("cuda")
    try:
        # a reordered tile case (n >= 4096), then a smaller row-and-tile case
        for H, eps in [(_grid(64, 1, 10.0), 1e-12), (_grid(23, 2), 1e-12)]:
            print(f"[noalloc] n={H.n} nnz={H.nnz}", flush=True)
            rp, ci, v = plan.expm(*to_device(H), eps)
            torch.cuda.synchronize()
            Eref = W.Csr(H.n, rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy())
            sref = plan.stats()
            Ena = _noalloc(plan, H, eps, Eref.nnz + 10)
            sna = plan.stats()
            rel, ok, og, oo = compare(Ena, Eref, final_theta(sref))
            exact = (np.array_equal(Ena.rowptr, Eref.rowptr) and np.array_equal(Ena.col, Eref.col)
                     and np.array_equal(Ena.val.view(np.uint64), Eref.val.view(np.uint64)))
            print(f"[noalloc] n={H.n} vs expm_sparse relF={rel:.2e} only={og},{oo} "
                  f"bitwise={exact} workspace={sna['peak_workspace_bytes']}", flush=True)
            assert rel <= TOL and ok
            assert (sna["M"], sna["N"], sna["nnz_e"]) == (sref["M"], sref["N"], Ena.nnz)
            Eo, so = run_oracle(H, eps)
            rel, ok, _, _ = compare(Ena, Eo, final_theta(so))
            assert rel <= TOL and ok
    finally:
        plan.close()


def test_noalloc_errors():
    import torch
    from paper_2110_04493_amd import api, capi
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True))
    try:
        H, eps = _grid(20, 3), 1e-12
        # capacity too small: EXPM_ENOMEM, with nnz(E) reported
        with pytest.raises(capi.ExpmError) as e:
            _noalloc(plan, H, eps, 5)
        assert e.value.code == capi.EXPM_ENOMEM
        need = e.value.nnz_e
        assert need > 5
        E = _noalloc(plan, H, eps, need)
        assert E.nnz == need
        Eo, so = run_oracle(H, eps)
        rel, ok, _, _ = compare(E, Eo, final_theta(so))
        assert rel <= TOL and ok
        # no adjoint after a fixed-region call
        with pytest.raises(capi.ExpmError) as e:
            plan.backward(torch.zeros(need, dtype=torch.float64, device="cuda"), H.nnz)
        assert e.value.code == capi.EXPM_ESTATE
        # an input too large for the static scratch is refused up front
        n = capi.NOALLOC_SCRATCH_BYTES // 64
        D = W.Csr(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                  np.full(n, -1.0))
        with pytest.raises(capi.ExpmError) as e:
            _noalloc(plan, D, eps, n)
        assert e.value.code == capi.EXPM_ENOMEM
        assert "static scratch" in str(e.value)
    finally:
        plan.close()
