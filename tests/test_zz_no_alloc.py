"""The allocation-free fused inference entry point, gpe_cnn_infer_noalloc,
against gpe_cnn_infer with a caller-owned scratch buffer, through the
C-ABI: bitwise the same network output and corrected states on two calls
in a row, the second with a smaller batch and grid (the library's buffer
keeps the first call's contents); a batch beyond the buffer's capacity is
rejected before anything is launched."""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as C

pytestmark = pytest.mark.gpu

SCALE_IN = (0.03, 0.03, 1e-3, 1.0)
OUT_SCALE = (1e-3, 2e-3, 1e-4, 0.01)


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_00814_amd import learn

    learn.lib()
    return learn


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _states(B, H, W, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(B):
        st = {"u": r.normal(size=(H, W)) * 0.03, "v": r.normal(size=(H, W)) * 0.03,
              "p": r.normal(size=(H, W)) * 1e-3, "phi": np.tanh(r.normal(size=(H, W)) * 2)}
        st["v"][0] = 0.0
        out.append(st)
    return out


def _upload(states):
    import torch

    ts, ptrs = [], []
    for st in states:
        for k in ("u", "v", "p", "phi"):
            t = torch.tensor(np.ascontiguousarray(st[k], dtype=np.float32), device="cuda:0")
            ts.append(t)
            ptrs.append(t.data_ptr())
    return ts, torch.tensor(ptrs, dtype=torch.int64, device="cuda:0")


def test_noalloc_inference_equals_scratch_entry_point(L):
    import torch

    for call, (B, H, W) in enumerate([(5, 40, 100), (2, 16, 40)]):
        _say(f"[no-alloc] call {call}: B={B} H={H} W={W}")
        p = C.init_params(31 + call)
        p[2] = (p[2][0] * 10, p[2][1] + 0.01)
        states = _states(B, H, W, 40 + call)
        ta, taba = _upload(states)
        tb, tabb = _upload(states)
        net = L.CNN(B, H, W, act_type=L.GPE_ACT_BF16, params=L.pack_params(p))
        net.infer(taba, B, SCALE_IN, OUT_SCALE)
        out_b = torch.full_like(net.out, float("nan"))
        L.gpe_cnn_infer_noalloc(tabb.data_ptr(), net.params.data_ptr(), net.params_act.data_ptr(), B, H, W,
                                SCALE_IN, OUT_SCALE, out_b.data_ptr(), net.sid)
        net.synchronize()
        a, b = net.out.cpu().numpy(), out_b.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b)
        for q in range(4 * B):
            assert np.array_equal(ta[q].cpu().numpy(), tb[q].cpu().numpy()), q
        # the correction changed the states, and kept each state's phase mass
        assert np.max(np.abs(tb[3].cpu().numpy() - states[0]["phi"].astype(np.float32))) > 0
        for s in range(B):
            assert abs(tb[4 * s + 3].cpu().numpy().astype(np.float64).sum() - states[s]["phi"].sum()) < 1e-3


def test_noalloc_inference_rejects_batches_beyond_capacity(L):
    import torch

    from paper_2011_00814_amd import gpe as G

    # 300 x 300 tiles of 32 x 8 cells: 90,001 partial sums > 65,536
    H, W = 8 * 300, 32 * 300
    assert L.gpe_cnn_infer_scratch_bytes(1, H, W) > 65536 * 4
    dummy = torch.zeros(64, dtype=torch.float32, device="cuda:0")
    table = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    with pytest.raises(G.GpeError) as e:
        L.gpe_cnn_infer_noalloc(table.data_ptr(), dummy.data_ptr(), dummy.data_ptr(), 1, H, W, SCALE_IN, OUT_SCALE,
                                dummy.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert e.value.code == G.GPE_EWORKSPACE
