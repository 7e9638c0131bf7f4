"""GPU parity of the complex entry point (expm_sparse_z, Algorithm 4.2 over
C) against the complex oracle: relative Frobenius error over the union of
the supports <= 1e-11, entries present on one side only within a factor 2
of the final threshold, (M, N), the normality decision, the Taylor term
count and the per-step kept and candidate counts as in the real parity
tests.  At full size (n = 90,000) sampled rows are checked against the
closed form of the free Schroedinger propagator, a Kronecker product of
path propagators from a symmetric eigensolver, and against unitarity."""
import numpy as np
import pytest

from oracle import complex_expm as Z
from paper_2110_04493_amd import workloads as W
from _helpers import compare, final_theta

pytestmark = pytest.mark.gpu
TOL = 1e-11


def to_device_z(H):
    import torch
    return (torch.from_numpy(H.rowptr.astype(np.int64)).cuda(),
            torch.from_numpy(H.col.astype(np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(H.val, dtype=np.complex128)).cuda())


def run_gpu_z(H, eps, **opts):
    import torch
    from paper_2110_04493_amd import api
    plan = api.Plan("cuda", api.Options(**opts))
    try:
        rp, ci, v = plan.expm_z(*to_device_z(H), eps)
        torch.cuda.synchronize()
        st = plan.stats()
    finally:
        plan.close()
    return W.Csr(H.n, rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy()), st


def compare_z(Eg, Eo, theta):
    """compare() of the real tests on complex values: the Frobenius error
    over the union of the supports, and the one-sided entries' moduli."""
    kg, ko = W.Csr.rows(Eg) * Eg.n + Eg.col, W.Csr.rows(Eo) * Eo.n + Eo.col
    assert np.all(np.diff(kg) > 0) and np.all(np.diff(ko) > 0)
    u = np.union1d(kg, ko)
    a = np.zeros(u.size, complex)
    b = np.zeros(u.size, complex)
    a[np.searchsorted(u, kg)] = Eg.val
    b[np.searchsorted(u, ko)] = Eo.val
    rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    og = np.setdiff1d(kg, ko, assume_unique=True)
    oo = np.setdiff1d(ko, kg, assume_unique=True)
    vals = np.abs(np.concatenate([a[np.searchsorted(u, og)], b[np.searchsorted(u, oo)]]))
    ok = bool(np.all((vals >= theta / 2) & (vals <= 2 * theta))) if vals.size else True
    return rel, ok, og.size, oo.size


def check_z(H, eps, count_tol=0.002, **kw):
    print(f"[complex] n={H.n} nnz={H.nnz} eps={eps} {kw}", flush=True)
    Eg, sg = run_gpu_z(H, eps, **kw)
    okw = {k: kw[k] for k in ("filter_mode", "normal", "exact_ri", "literal_a") if k in kw}
    res = Z.expm(H.rowptr, H.col, H.val, eps, **okw)
    so = res.stats
    Eo = W.Csr(H.n, res.rowptr, res.col, res.val)
    rel, ok, og, oo = compare_z(Eg, Eo, final_theta(so))
    print(f"  relF={rel:.3e} only_gpu={og} only_oracle={oo} M,N={sg['M']},{sg['N']} "
          f"normal={sg['normal']} nnzE={Eg.nnz}/{Eo.nnz}", flush=True)
    assert (sg["M"], sg["N"]) == (so["M"], so["N"])
    assert sg["normal"] == so["normal"]
    assert sg["taylor_terms"] == so["taylor_terms"]
    assert rel <= TOL and ok
    for k in ("sq_kept", "sq_cand", "taylor_kept", "taylor_cand"):
        assert len(sg[k]) == len(so[k]), k
        for a, b in zip(sg[k], so[k]):
            assert abs(a - b) <= count_tol * b + 2, k
    assert abs(sg["a"] - so["a"]) <= 1e-14 * max(so["a"], 1e-300)
    return Eg, sg, Eo, so


def test_general_random():
    check_z(W.complex_random(150, 0.03, 61, scale=0.8), 1e-12)


def test_hermitian_magnetic_laplacian():
    _, sg, _, _ = check_z(W.magnetic_laplacian(30, 30, seed=62).scaled(-1.0), 1e-12)
    assert sg["normal"] == 1


def test_skew_hermitian_schrodinger():
    _, sg, _, _ = check_z(W.schrodinger_grid(40, 1.0, seed=63), 1e-12)
    assert sg["normal"] == 1


def test_normal_circulant_commutator():
    """Normal without being Hermitian or skew-Hermitian: the commutator test
    of step 2 decides (then a bumped copy must come out non-normal)."""
    n = 800
    i = np.arange(n)
    off = [0, 1, 3]
    vals = [0.2 + 0.1j, 1.0 - 0.5j, 0.3j]
    r = np.concatenate([i] * 3)
    c = np.concatenate([(i + o) % n for o in off])
    v = np.concatenate([np.full(n, x) for x in vals])
    H = W.csr_from_coo(n, r, c, v, dtype=np.complex128)
    _, sg, _, _ = check_z(H, 1e-12)
    assert sg["normal"] == 1
    Hb = W.Csr(n, H.rowptr, H.col, H.val.copy())
    Hb.val[1] += 1e-3     # entry (0, 1)
    _, sb, _, _ = check_z(Hb, 1e-12)
    assert sb["normal"] == 0


def test_structural_hamiltonian_complex_time():
    """Eq. (2.1)'s H at a complex time step (non-normal, complex)."""
    H, _, _ = W.structural_hamiltonian(20, 20, 0.5, alpha=0.02, beta=0.01, seed=64)
    Hz = W.Csr(H.n, H.rowptr, H.col, H.val * (1.0 + 0.4j))
    for lit in (False, True):
        _, sg, _, _ = check_z(Hz, 1e-12, literal_a=lit)
        assert sg["normal"] == 0


@pytest.mark.parametrize("opts", [{"filter_mode": 1}, {"exact_ri": True}, {"normal": 0}])
def test_options(opts):
    check_z(W.schrodinger_grid(24, 0.8, seed=65), 1e-12, **opts)


@pytest.mark.parametrize("case", ["schrodinger", "magnetic", "general"])
def test_locality_reordering(case):
    """The locality ordering forced on (reorder = 1; by default it applies
    from n = 4096): H is permuted before the method and E back after it, so
    the result is the oracle's up to rounding order."""
    if case == "schrodinger":
        H = W.schrodinger_grid(40, 1.0, seed=70)
    elif case == "magnetic":
        H = W.magnetic_laplacian(30, 30, seed=71).scaled(-1.0)
    else:
        H = W.complex_random(300, 0.02, 72, scale=0.8)
    _, sg, _, _ = check_z(H, 1e-12, reorder=1)
    if case != "general":
        assert sg["ordering"] >= 1


def test_real_input_matches_real_path():
    """Imaginary parts zero: the complex path agrees with the real one
    (rows, no reordering) entry by entry."""
    from _helpers import run_gpu
    L = W.grid_laplacian(40, 40, np.random.default_rng(66))
    H = L.scaled(-20.0 / W.norm1(L))
    Er, sr = run_gpu(H, 1e-12, tile_min_fill=2.0, reorder=0)
    Hz = W.Csr(H.n, H.rowptr, H.col, H.val.astype(complex))
    Ez, sz = run_gpu_z(Hz, 1e-12)
    assert (sz["M"], sz["N"], sz["normal"]) == (sr["M"], sr["N"], sr["normal"])
    assert np.all(Ez.val.imag == 0)
    rel, ok, _, _ = compare(W.Csr(H.n, Ez.rowptr, Ez.col, Ez.val.real), Er, final_theta(sr))
    assert rel <= 1e-13 and ok


def test_taylor_only_zero_and_empty():
    import torch
    from paper_2110_04493_amd import api
    A = W.complex_random(40, 0.1, 67, scale=1e-3)
    _, sg, _, _ = check_z(A, 1e-14)
    assert sg["N"] == 0
    Zm = W.Csr(40, A.rowptr, A.col, np.zeros(A.nnz, complex))
    Ez, _ = run_gpu_z(Zm, 1e-12)
    assert np.array_equal(Ez.col, np.arange(40)) and np.all(Ez.val == 1.0)
    plan = api.Plan("cuda")
    try:
        rp, ci, v = plan.expm_z(torch.zeros(1, dtype=torch.int64, device="cuda"),
                                torch.zeros(0, dtype=torch.int32, device="cuda"),
                                torch.zeros(0, dtype=torch.complex128, device="cuda"), 1e-12)
        assert rp.numel() == 1 and ci.numel() == 0 and v.numel() == 0
    finally:
        plan.close()


def test_long_row_global_scratch():
    """A row whose complex accumulators exceed the LDS classes (6,000
    candidate columns, 96 KB) runs in global scratch."""
    n = 6000
    rng = np.random.default_rng(68)
    r = np.concatenate([np.zeros(n, np.int64), np.arange(1, n)])
    c = np.concatenate([np.arange(n), np.arange(1, n)])
    v = np.concatenate([rng.standard_normal(n) + 1j * rng.standard_normal(n),
                        rng.uniform(-1, 1, n - 1) + 0.5j])
    H = W.csr_from_coo(n, r, c, v * 0.02, dtype=np.complex128)
    _, sg, _, _ = check_z(H, 1e-12)
    assert sg["N"] >= 1


def test_errors():
    import torch
    from paper_2110_04493_amd import api, capi
    H = W.schrodinger_grid(8, 0.5)
    dev = to_device_z(H)
    for opts, code in (({"filter_mode": 2}, capi.EXPM_ENOTIMPL), ({"norm": 1}, capi.EXPM_ENOTIMPL)):
        plan = api.Plan("cuda", api.Options(**opts))
        try:
            with pytest.raises(capi.ExpmError) as e:
                plan.expm_z(*dev, 1e-12)
            assert e.value.code == code
        finally:
            plan.close()
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True))
    try:
        plan.expm_z(*dev, 1e-12)
        with pytest.raises(capi.ExpmError) as e:
            plan.backward(torch.zeros(10, dtype=torch.float64, device="cuda"), H.nnz)
        assert e.value.code == capi.EXPM_ESTATE
        bad = dev[2].clone()
        bad[3] = complex(0.0, float("nan"))
        with pytest.raises(capi.ExpmError) as e:
            plan.expm_z(dev[0], dev[1], bad, 1e-12)
        assert e.value.code == capi.EXPM_EINVAL
    finally:
        plan.close()


def path_propagator(n, t):
    """e^{-i t L} for the unit path Laplacian of n nodes (eigh)."""
    L = np.diag(np.r_[1.0, np.full(n - 2, 2.0), 1.0]) - np.eye(n, k=1) - np.eye(n, k=-1)
    lam, V = np.linalg.eigh(L)
    return (V * np.exp(-1j * t * lam)) @ V.T


def test_full_size_free_schrodinger_sampled_rows():
    """n = 90,000: the 300 x 300 free propagator e^{-i t L} = P (x) P with P
    the path propagator; sampled rows to 1e-10 relative, unit row norms."""
    side, t = 300, 1.0
    H = W.schrodinger_grid(side, t, vmax=0.0)
    Eg, sg = run_gpu_z(H, 1e-12)
    print(f"[complex full] M={sg['M']} N={sg['N']} nnz(E)={Eg.nnz}", flush=True)
    P = path_propagator(side, t)
    rng = np.random.default_rng(69)
    for i in [0, side - 1, H.n // 2 + side // 2, H.n - 1, *rng.integers(0, H.n, 5).tolist()]:
        b, e = int(Eg.rowptr[i]), int(Eg.rowptr[i + 1])
        got = np.zeros(H.n, complex)
        got[Eg.col[b:e]] = Eg.val[b:e]
        exact = np.kron(P[i // side], P[i % side])
        rel = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        print(f"  row {i}: nnz={e - b} relF={rel:.2e} |row|-1={np.linalg.norm(got) - 1:.2e}",
              flush=True)
        assert rel <= 1e-10
        assert abs(np.linalg.norm(got) - 1.0) <= 1e-10
