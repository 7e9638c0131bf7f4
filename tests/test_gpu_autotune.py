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


def test_tune_cache_single_and_batched(tmp_path, monkeypatch):
    """The cache under $EXPM_TUNE_CACHE: the first input of a shape bucket
    is tuned and stored (keyed by architecture and bucket), the next one of
    the same bucket reuses the entry; the batched path takes its threshold
    from the cache, and its results pass the parity bar."""
    import json
    from paper_2110_04493_amd import api, autotune
    path = tmp_path / "tune.json"
    monkeypatch.setenv("EXPM_TUNE_CACHE", str(path))
    rng = np.random.default_rng(22)
    L = W.grid_laplacian(40, 40, rng)
    H = L.scaled(-20.0 / W.norm1(L))
    opts, cached = autotune.tuned_options(*to_device(H), 1e-12, fills=(0.0, 2.0), reorders=(0,))
    assert not cached and path.exists()
    data = json.loads(path.read_text())
    assert len(data) == 1 and next(iter(data)).startswith("gfx950/single/")
    L2 = W.grid_laplacian(40, 40, np.random.default_rng(23))      # same bucket
    H2 = L2.scaled(-20.0 / W.norm1(L2))
    opts2, cached2 = autotune.tuned_options(*to_device(H2), 1e-12, fills=(0.0, 2.0),
                                            reorders=(0,))
    assert cached2 and opts2 == opts
    mats, eps = [], []
    for j in range(6):
        A, e = W.config4_instance(j, nmin=60, nmax=300)
        mats.append(A)
        eps.append(e)
    dev = [to_device(A) for A in mats]
    bo, bc = autotune.tuned_batched_options(dev, eps, fills=(0.0, 2.0))
    assert not bc and bo.tile_min_fill in (0.0, 2.0)
    outs = api.expm_batched(dev, eps, tune=True)
    assert len(json.loads(path.read_text())) == 2
    for A, e, (rp, ci, v) in zip(mats, eps, outs):
        Eg = W.Csr(A.n, rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy())
        Eo, so = run_oracle(A, e)
        rel, ok, _, _ = compare(Eg, Eo, final_theta(so))
        assert rel <= 1e-11 and ok
