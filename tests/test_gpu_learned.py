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


def test_learned_correction_small(LD):
    kw = dict(factor=4, nx=64, ny=128, log=_say)
    train_data = LD.generate(list(range(8)), fine_steps=1200, n_snap=12, **kw)
    assert train_data["finite"].sum() == 8
    net, hist, sin, sout, _ = LD.train(train_data, iters=1200, batch=16, lr=1e-3, log=_say)
    _say(f"[learned] window losses {[round(h[1], 4) for h in hist]}")
    assert np.mean([h[1] for h in hist[-4:]]) < 0.8 * np.mean([h[1] for h in hist[:2]])
    held = LD.generate([100, 101, 102], fine_steps=1200, n_snap=12, **kw)
    plain, corr = LD.one_step_gain(net, held, sin, sout)
    _say(f"[learned] held-out one-step mse (units of the target scale): plain {plain:.4f} network {corr:.4f}")
    assert corr < plain
    res = LD.evaluate(net, sin, sout, [100, 101], fine_steps=1200, **kw)
    assert res["fine_finite"] == 2 and res["plain_coarse"]["finite"] == 2
    assert res["coarse_steps"] == 300 and len(res["checkpoints"]) == 4
    for k in ("plain_coarse", "learned_coarse"):
        assert math.isfinite(res[k]["mean_err_mean"]) or res[k]["finite"] < 2
