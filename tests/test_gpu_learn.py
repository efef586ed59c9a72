"""Kernels of the learned coarse correction against the CPU reference
(oracle/cnn_oracle.py), through the C-ABI: restriction, network input,
forward and backward passes in FP32 and BF16 storage, Adam, the
mass-projected correction, the interface position, and a short training
run that must reduce the loss."""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as C

pytestmark = pytest.mark.gpu


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


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _upload(states):
    """list of dicts (u, v, p, phi) -> device tensors and their pointer table."""
    import torch

    ts, ptrs = [], []
    for st in states:
        for k in ("u", "v", "p", "phi"):
            t = torch.tensor(np.ascontiguousarray(st[k], dtype=np.float32), device="cuda:0")
            ts.append(t)
            ptrs.append(t.data_ptr())
    return ts, torch.tensor(ptrs, dtype=torch.int64, device="cuda:0")


def _random_states(B, H, W, seed):
    r = _rng(seed)
    out = []
    for _ in range(B):
        st = {"u": r.normal(size=(H, W)) * 0.03, "v": r.normal(size=(H, W)) * 0.03,
              "p": r.normal(size=(H, W)) * 1e-3, "phi": np.tanh(r.normal(size=(H, W)) * 2)}
        st["v"][0] = 0.0
        out.append(st)
    return out


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


SCALE_IN = (0.03, 0.03, 1e-3, 1.0)


def _params(seed):
    p = C.init_params(seed)
    p[2] = (p[2][0] * 10, p[2][1] + 0.01)
    p[0] = (p[0][0], p[0][1] + 0.05)
    return p


def test_restrict_matches_oracle(L):
    import torch

    B, ny, nx, f = 3, 32, 16, 4
    fine = _random_states(B, ny, nx, 1)
    coarse = [{k: np.zeros((ny // f, nx // f)) for k in ("u", "v", "p", "phi")} for _ in range(B)]
    tf, tabf = _upload(fine)
    tc, tabc = _upload(coarse)
    L.gpe_restrict2d(tabf.data_ptr(), tabc.data_ptr(), B, ny, nx, f, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for b in range(B):
        ref = C.restrict(fine[b], f)
        for q, k in enumerate(("u", "v", "p", "phi")):
            got = tc[4 * b + q].cpu().numpy()
            assert np.max(np.abs(got - ref[k])) <= 1e-6 * max(1e-3, np.max(np.abs(ref[k]))), (b, k)


@pytest.mark.parametrize("act", ["fp32", "bf16"])
def test_forward_and_backward_match_oracle(L, act):
    import torch

    B, H, W = 2, 16, 8
    at = L.GPE_ACT_FP32 if act == "fp32" else L.GPE_ACT_BF16
    params = _params(3)
    net = L.CNN(B, H, W, act_type=at, params=L.pack_params(params))
    states = _random_states(B, H, W, 5)
    _, tab = _upload(states)
    net.features(tab, B, SCALE_IN)
    r = _rng(7)
    target = r.normal(size=(B, H, W, 4)) * 0.1
    net.target.copy_(torch.tensor(target.ravel(), dtype=torch.float32, device="cuda:0"))
    net.forward(B)
    net.loss(B)
    net.backward(B)
    net.synchronize()
    # the reference sees the operands the kernels read: FP32 master weights
    # in FP32 mode, the BF16-rounded copies and input in BF16 mode
    if act == "fp32":
        x0 = net.x0.cpu().numpy().astype(np.float64).reshape(B, H, W, 4)
        p_ref = params
    else:
        x0 = L.bf16_to_float(net.x0).astype(np.float64).reshape(B, H, W, 4)
        wa = L.bf16_to_float(net.params_act).astype(np.float64)
        master = L.pack_params(params).astype(np.float32).astype(np.float64)
        p_ref = [(w, b) for (w, _), (_, b) in zip(L.unpack_params(wa), L.unpack_params(master))]
    feats = np.stack([C.features(st, SCALE_IN) for st in states])
    assert np.max(np.abs(x0 - feats)) <= (1e-6 if act == "fp32" else 8e-3) * np.max(np.abs(feats))
    loss, grads, out = C.loss_and_grads(p_ref, x0, target)
    tol_out, tol_g = (1e-5, 1e-4) if act == "fp32" else (2e-2, 5e-2)
    got_out = net.out.cpu().numpy().reshape(B, H, W, 4)
    _say(f"[learn] {act} forward rel {_rel(got_out, out):.2e} loss {net.loss_buf.item():.6e} vs {loss:.6e}")
    assert _rel(got_out, out) < tol_out
    assert abs(net.loss_buf.item() - loss) <= tol_out * loss * 10
    got = L.unpack_params(net.grads.cpu().numpy())
    for layer in range(3):
        ew, eb = _rel(got[layer][0], grads[layer][0]), _rel(got[layer][1], grads[layer][1])
        _say(f"[learn] {act} layer {layer} grad rel w {ew:.2e} b {eb:.2e}")
        assert ew < tol_g and eb < tol_g, (layer, ew, eb)


@pytest.mark.parametrize("B,H,W", [(3, 16, 64), (2, 20, 50), (1, 64, 256)])
def test_fused_inference_matches_unfused_path_and_oracle(L, B, H, W):
    """gpe_cnn_infer (network input, three layers on the matrix cores with the
    activations in LDS, correction) against gpe_cnn_features + forward +
    apply with BF16 operands, and its output against the CPU reference fed
    the same BF16 operands; ragged tiles in x and y included."""
    import torch

    params = _params(21)
    states = _random_states(B, H, W, 22)
    out_scale = (1e-3, 2e-3, 1e-4, 0.01)
    ta, taba = _upload(states)
    tb, tabb = _upload(states)
    net = L.CNN(B, H, W, act_type=L.GPE_ACT_BF16, params=L.pack_params(params))
    _say(f"[learn] fused inference B={B} H={H} W={W}")
    net.features(taba, B, SCALE_IN)
    net.forward(B)
    net.apply(taba, B, out_scale)
    net.synchronize()
    ref_out = net.out.cpu().numpy().reshape(B, H, W, 4).copy()
    x0 = L.bf16_to_float(net.x0).astype(np.float64).reshape(B, H, W, 4)
    net.out.zero_()
    net.infer(tabb, B, SCALE_IN, out_scale)
    net.synchronize()
    got = net.out.cpu().numpy().reshape(B, H, W, 4)
    # the fused kernel accumulates every layer in another order (double-K
    # MFMA) and sums the phase mass per tile: FP32 rounding differences
    assert _rel(got, ref_out) < 1e-5, _rel(got, ref_out)
    for q in range(4 * B):
        a, b = ta[q].cpu().numpy(), tb[q].cpu().numpy()
        assert np.max(np.abs(a - b)) <= 1e-6 * max(1e-3, np.max(np.abs(a))), q
    wa = L.bf16_to_float(net.params_act).astype(np.float64)
    master = L.pack_params(params).astype(np.float32).astype(np.float64)
    p_ref = [(w, bb) for (w, _), (_, bb) in zip(L.unpack_params(wa), L.unpack_params(master))]
    out, _ = C.forward(p_ref, x0)  # FP64 activations: the kernels round them to BF16
    assert _rel(got, out) < 2e-2
    # the phase mass of every state is kept
    for b in range(B):
        assert abs(tb[4 * b + 3].cpu().numpy().astype(np.float64).sum() - states[b]["phi"].sum()) < 1e-3


def test_adam_matches_update_rule(L):
    import torch

    net = L.CNN(1, 4, 4, act_type=L.GPE_ACT_FP32)
    r = _rng(9)
    p0 = r.normal(size=net.n)
    net.params.copy_(torch.tensor(p0, dtype=torch.float32, device="cuda:0"))
    m = np.zeros(net.n)
    v = np.zeros(net.n)
    p = p0.astype(np.float32).astype(np.float64)
    for t in range(1, 4):
        g = r.normal(size=net.n)
        net.grads.copy_(torch.tensor(g, dtype=torch.float32, device="cuda:0"))
        net.adam(lr=1e-2)
        g = g.astype(np.float32).astype(np.float64)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        p = p - 1e-2 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    net.synchronize()
    assert np.max(np.abs(net.params.cpu().numpy() - p)) < 1e-5


def test_apply_correction_matches_oracle_and_keeps_mass(L):
    import torch

    B, H, W = 2, 12, 8
    states = _random_states(B, H, W, 11)
    ts, tab = _upload(states)
    net = L.CNN(B, H, W, act_type=L.GPE_ACT_FP32)
    out = _rng(12).normal(size=(B, H, W, 4))
    net.out.copy_(torch.tensor(out.ravel(), dtype=torch.float32, device="cuda:0"))
    scale = (1e-3, 2e-3, 1e-4, 0.01)
    net.apply(tab, B, scale)
    net.synchronize()
    for b in range(B):
        ref = C.apply_correction({k: states[b][k].astype(np.float32).astype(np.float64) for k in states[b]},
                                 out[b].astype(np.float32).astype(np.float64), scale)
        for q, k in enumerate(("u", "v", "p", "phi")):
            got = ts[4 * b + q].cpu().numpy()
            assert np.max(np.abs(got - ref[k])) < 1e-6 * max(1.0, np.max(np.abs(ref[k]))), (b, k)
        assert abs(ts[4 * b + 3].cpu().numpy().astype(np.float64).sum() - states[b]["phi"].sum()) < 1e-4
        assert np.all(ts[4 * b + 1].cpu().numpy()[0] == 0.0)


def test_interface_position_matches_oracle(L):
    import torch

    B, H, W = 3, 64, 16
    r = _rng(13)
    phis = []
    y = np.arange(H)[:, None] + 0.5
    x = np.arange(W)[None, :] + 0.5
    for b in range(B):
        y0 = H / 2 + 6 * np.cos(2 * np.pi * x / W + r.uniform(0, 6.3)) + 3 * np.sin(4 * np.pi * x / W)
        ph = np.tanh(2 * (y - y0) / 2.0)
        if b == 2:  # a detached liquid blob below the interface: top and bottom differ
            ph = np.maximum(ph, -np.tanh(2 * (np.hypot(y - 10, x - 8) - 4) / 2.0))
        phis.append(ph)
    ts = [torch.tensor(p.astype(np.float32), device="cuda:0") for p in phis]
    tab = torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device="cuda:0")
    out = torch.zeros(B * W * 2, dtype=torch.float32, device="cuda:0")
    L.gpe_interface_position(tab.data_ptr(), B, H, W, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    got = out.cpu().numpy().reshape(B, W, 2)
    for b in range(B):
        top, bot = C.interface_position(phis[b].astype(np.float32).astype(np.float64))
        assert np.allclose(got[b, :, 0], top, atol=1e-4, equal_nan=True)
        assert np.allclose(got[b, :, 1], bot, atol=1e-4, equal_nan=True)


def test_short_training_reduces_loss(L):
    """Fit the network to a fixed smooth map of its input (a learnable
    target): 400 Adam steps in BF16 must cut the loss by 4x."""
    import torch

    B, H, W = 4, 32, 16
    net = L.CNN(B, H, W, act_type=L.GPE_ACT_BF16, params=L.pack_params(C.init_params(21)))
    states = _random_states(B, H, W, 22)
    _, tab = _upload(states)
    net.features(tab, B, SCALE_IN)
    feats = np.stack([C.features(st, SCALE_IN) for st in states])
    target = 0.1 * np.tanh(np.roll(feats, 1, axis=2)[..., [1, 0, 3, 2]])
    net.target.copy_(torch.tensor(target.ravel(), dtype=torch.float32, device="cuda:0"))
    losses = []
    for it in range(400):
        net.forward(B)
        net.loss(B)
        net.backward(B)
        net.adam(lr=3e-3)
        if it % 80 == 0 or it == 399:
            losses.append(net.loss_buf.item())
    _say(f"[learn] training losses {losses}")
    assert losses[-1] < 0.25 * losses[0]
