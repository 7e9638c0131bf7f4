"""The three profiling modes give the same result; mode 1 counts the
algorithmic work and times every phase, mode 2 only times the launches of
the tile kernels (the same launches as mode 1)."""
import numpy as np
import pytest

from paper_2110_04493_amd import workloads as W
from _helpers import to_device

pytestmark = pytest.mark.gpu


def run(H, eps, profile):
    import torch
    from paper_2110_04493_amd import api
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True, profile=profile,
                                        tile_min_fill=0.0))
    try:
        rp, ci, v = plan.expm(*to_device(H), eps)
        g = torch.ones_like(v)
        dH = plan.backward(g, H.nnz)
        torch.cuda.synchronize()
        return v.cpu().numpy(), dH.cpu().numpy(), plan.stats()
    finally:
        plan.close()


def test_profile_modes():
    H, eps = W.config5(40)
    v0, d0, s0 = run(H, eps, 0)
    v1, d1, s1 = run(H, eps, 1)
    v2, d2, s2 = run(H, eps, 2)
    print(f"[profile] launches {s1['tile_launches']}/{s2['tile_launches']} "
          f"ms {s1['tile_ms']:.3f}/{s2['tile_ms']:.3f} adj {s1['adj_tile_launches']}/"
          f"{s2['adj_tile_launches']}", flush=True)
    for v, d in ((v1, d1), (v2, d2)):
        assert np.array_equal(v.view(np.uint64), v0.view(np.uint64))
        assert np.array_equal(d.view(np.uint64), d0.view(np.uint64))
    assert s0["tile_launches"] == 0 and s0["tile_ms"] == 0.0
    assert s1["tile_launches"] > 0 and s1["tile_flops"] > 0 and s1["tile_ms"] > 0
    assert s2["tile_launches"] == s1["tile_launches"]
    assert s2["adj_tile_launches"] == s1["adj_tile_launches"] > 0
    assert s2["tile_ms"] > 0 and s2["adj_tile_ms"] > 0 and s2["tile_flops"] == 0
    assert sum(s2["t_num_ms"]) == 0.0 and sum(s1["t_num_ms"]) > 0
