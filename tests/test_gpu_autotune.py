"""The autotuner returns valid options (one of the candidates it timed), and
a run with those options passes the oracle parity bar."""
import numpy as np
import pytest

from paper_2110_04493_amd import workloads as W
from _helpers import compare, final_theta, run_gpu, run_oracle, to_device

pytestmark = pytest.mark.gpu


def test_autotune_small_grid():
    from paper_2110_04493_amd import autotune
    rng = np.random.default_rng(21)
    L = W.grid_laplacian(70, 70, rng)
    H, eps = L.scaled(-20.0 / W.norm1(L)), 1e-12
    opts, times = autotune.autotune(*to_device(H), eps, fills=(0.0, 0.2, 2.0), reorders=(0, 1),
                                    with_adjoint=True, repeats=1, verbose=True)
    assert len(times) == 6 and all(t > 0 for t in times.values())
    assert (opts.tile_min_fill, opts.reorder) in times
    assert times[(opts.tile_min_fill, opts.reorder)] == min(times.values())
    Eg, _ = run_gpu(H, eps, tile_min_fill=opts.tile_min_fill, reorder=opts.reorder)
    Eo, so = run_oracle(H, eps)
    rel, ok, og, oo = compare(Eg, Eo, final_theta(so))
    print(f"[autotune] chose fill={opts.tile_min_fill} reorder={opts.reorder}; relF={rel:.2e}",
          flush=True)
    assert rel <= 1e-11 and ok
