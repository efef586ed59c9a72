"""The learned coarse correction end to end on the GPU, at a small size
(fine 64 x 128, coarse 16 x 32, one coarse step = 4 fine steps): data from
the solver's own fine runs, training on the GPU, a gain over the plain
coarse solver on flows it has not seen, and the rollout evaluated against the
fine solver."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def LD():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_00814_amd import learned

    return learned


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


KW = dict(factor=4, nx=64, ny=128)


@pytest.fixture(scope="module")
def trained(LD):
    """Data from 8 fine runs, training on one-step pairs, pairs from the
    network's short corrected coarse rollouts (1-3 steps), more training on
    all of them."""
    train_data = LD.generate(list(range(8)), fine_steps=1200, n_snap=12, log=_say, unroll=3, **KW)
    assert train_data["finite"].sum() == 8
    net, hist, sin, sout, _ = LD.train(train_data, iters=800, batch=16, lr=1e-3, log=_say)
    _say(f"[learned] window losses {[round(h[1], 4) for h in hist]}")
    assert np.mean([h[1] for h in hist[-4:]]) < 0.8 * np.mean([h[1] for h in hist[:2]])
    LD.rollout_pairs(net, train_data, sin, sout, log=_say)
    assert len(train_data["pairs"]) == 4
    net, hist2, _, _, _ = LD.train(train_data, iters=600, batch=16, lr=5e-4, log=_say, net=net,
                                   scales_=(sin, sout))
    assert all(math.isfinite(h[1]) for h in hist2)
    return net, sin, sout


def test_learned_correction_small(LD, trained):
    net, sin, sout = trained
    held = LD.generate([100, 101, 102], fine_steps=1200, n_snap=12, log=_say, **KW)
    plain, corr = LD.one_step_gain(net, held, sin, sout)
    _say(f"[learned] held-out one-step mse (units of the target scale): plain {plain:.4f} network {corr:.4f}")
    assert corr < plain
    res = LD.evaluate(net, sin, sout, [100, 101], fine_steps=1200, log=_say, **KW)
    assert res["fine_finite"] == 2 and res["plain_coarse"]["finite"] == 2
    assert res["coarse_steps"] == 300 and len(res["checkpoints"]) == 4
    for k in ("plain_coarse", "learned_coarse"):
        assert math.isfinite(res[k]["mean_err_mean"]) or res[k]["finite"] < 2
        assert k in res["horizon_95pct_columns_every_case"]
    _say(f"[learned] horizons {res['horizon_95pct_columns_every_case']}, fallback "
         f"{res['learned_coarse']['fallback_to_fine']}, indicator max "
         f"{[c['learned_coarse']['indicator_rms_max'] for c in res['checkpoints']]}")


def test_fallback_to_fine_solver_fires(LD, trained):
    """The error indicator forced to fire from the host (threshold 0): every
    learned case falls back to the fine solver after the first segment, its
    result is the fine solution (no interface error) and the fine solver's
    cost is charged to the learned run."""
    net, sin, sout = trained
    res = LD.evaluate(net, sin, sout, [100, 101], fine_steps=1200, log=_say, indicator=0.0, **KW)
    lc = res["learned_coarse"]
    assert lc["fallback_to_fine"] == 2 and res["checkpoints"][0]["learned_coarse"]["fallback_to_fine"] == 2
    assert lc["mean_err_mean"] == 0.0 and lc["columns_within_1_cell"] == 1.0
    assert res["fallback_ms"] == pytest.approx(res["fine_ms"])
    assert res["speedup_vs_fine"] < 1.0
    assert res["horizon_95pct_columns_every_case"]["learned_coarse"]["fine_steps"] == res["fine_steps"]
