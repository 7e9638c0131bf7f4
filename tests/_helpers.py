"""Shared helpers of the parity tests: run the GPU library and the oracle on
the same seeded input and compare them entry by entry."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2110_04493_amd import workloads as W


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def to_device(H: W.Csr):
    import torch
    return (torch.from_numpy(H.rowptr.astype(np.int64)).cuda(),
            torch.from_numpy(H.col.astype(np.int32)).cuda(),
            torch.from_numpy(H.val.astype(np.float64)).cuda())


def run_gpu(H: W.Csr, eps: float, **opts):
    """Returns (Csr of E, stats dict) from the gfx950 library."""
    import torch
    from paper_2110_04493_amd import api
    plan = api.Plan("cuda", api.Options(**opts))
    try:
        rp, ci, v = plan.expm(*to_device(H), eps)
        torch.cuda.synchronize()
        st = plan.stats()
    finally:
        plan.close()
    return W.Csr(H.n, rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy()), st


def run_oracle(H: W.Csr, eps: float, **kw):
    res = oracle.expm(H.rowptr, H.col, H.val, eps, **kw)
    return W.Csr(H.n, res.rowptr, res.col, res.val), res.stats


def keys(A: W.Csr) -> np.ndarray:
    return A.rows() * A.n + A.col.astype(np.int64)


def compare(E_gpu: W.Csr, E_ora: W.Csr, theta: float):
    """relative Frobenius error over the union of the supports, and whether
    every entry present in only one support lies in [theta/2, 2 theta]."""
    kg, ko = keys(E_gpu), keys(E_ora)
    for k in (kg, ko):
        assert np.all(np.diff(k) > 0), "rows must have sorted unique columns"
    u = np.union1d(kg, ko)
    a = np.zeros(u.size)
    b = np.zeros(u.size)
    a[np.searchsorted(u, kg)] = E_gpu.val
    b[np.searchsorted(u, ko)] = E_ora.val
    rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    only_g = np.setdiff1d(kg, ko, assume_unique=True)
    only_o = np.setdiff1d(ko, kg, assume_unique=True)
    vals = np.concatenate([a[np.searchsorted(u, only_g)], b[np.searchsorted(u, only_o)]])
    ok = bool(np.all((np.abs(vals) >= theta / 2) & (np.abs(vals) <= 2 * theta))) if vals.size else True
    return rel, ok, int(only_g.size), int(only_o.size)


def final_theta(stats: dict) -> float:
    if stats["N"] >= 1 and stats["sq_theta"]:
        return stats["sq_theta"][-1]
    th = stats.get("taylor_theta") or [0.0]
    return max(th) if th else 0.0
