"""Pins of the CPU reference of the learned correction (oracle/cnn_oracle.py)
against definitions written out independently: direct convolution loops,
central finite differences, conservation identities of the restriction and
exact crossings of linear profiles."""

import numpy as np

from oracle import cnn_oracle as C


def _rng(s=0):
    return np.random.Generator(np.random.PCG64(s))


def test_conv_matches_direct_loops():
    r = _rng(1)
    B, H, W, Ci, Co = 2, 5, 4, 3, 2
    x = r.normal(size=(B, H, W, Ci))
    w = r.normal(size=(Co, 3, 3, Ci))
    b = r.normal(size=Co)
    out = C.conv3x3(x, w, b)
    ref = np.zeros((B, H, W, Co))
    for bb in range(B):
        for y in range(H):
            for xx in range(W):
                for o in range(Co):
                    s = b[o]
                    for dy in (-1, 0, 1):
                        yy = y + dy
                        if not 0 <= yy < H:
                            continue
                        for dx in (-1, 0, 1):
                            x2 = (xx + dx) % W
                            for i in range(Ci):
                                s += w[o, dy + 1, dx + 1, i] * x[bb, yy, x2, i]
                    ref[bb, y, xx, o] = s
    assert np.max(np.abs(out - ref)) < 1e-12


def test_conv_gradients_match_finite_differences():
    r = _rng(2)
    B, H, W, Ci, Co = 1, 4, 3, 2, 3
    x = r.normal(size=(B, H, W, Ci))
    w = r.normal(size=(Co, 3, 3, Ci))
    b = r.normal(size=Co)
    g = r.normal(size=(B, H, W, Co))
    f = lambda xx, ww, bb: float(np.sum(g * C.conv3x3(xx, ww, bb)))  # noqa: E731
    gx = C.conv3x3_input_grad(g, w)
    gw, gb = C.conv3x3_weight_grad(g, x)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 3, 2, 1), (0, 1, 1, 0), (0, 2, 0, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * h) - gx[idx]) < 1e-7
    for idx in [(0, 0, 0, 0), (2, 1, 2, 1), (1, 2, 1, 0)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * h) - gw[idx]) < 1e-7
    e = np.zeros_like(b)
    e[1] = h
    assert abs((f(x, w, b + e) - f(x, w, b - e)) / (2 * h) - gb[1]) < 1e-7


def test_network_loss_gradient_matches_finite_differences():
    params = C.init_params(3)
    # larger last layer so the loss depends visibly on every layer
    params[2] = (params[2][0] * 10, params[2][1])
    r = _rng(4)
    x = r.normal(size=(1, 6, 5, 4))
    t = r.normal(size=(1, 6, 5, 4)) * 0.1
    loss, grads, _ = C.loss_and_grads(params, x, t)
    h = 1e-6
    for layer, idx in [(0, (3, 1, 2, 0)), (1, (7, 0, 1, 5)), (2, (2, 1, 1, 9)), (1, (0, 2, 2, 31))]:
        w, b = params[layer]
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        pp = [p if q != layer else (wp, b) for q, p in enumerate(params)]
        pm = [p if q != layer else (wm, b) for q, p in enumerate(params)]
        fd = (C.loss_and_grads(pp, x, t)[0] - C.loss_and_grads(pm, x, t)[0]) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) < 1e-7 * max(1.0, abs(fd)), (layer, idx)
    # biases of the hidden layers
    w, b = params[1]
    bp, bm = b.copy(), b.copy()
    bp[4] += h
    bm[4] -= h
    fd = (C.loss_and_grads([params[0], (w, bp), params[2]], x, t)[0]
          - C.loss_and_grads([params[0], (w, bm), params[2]], x, t)[0]) / (2 * h)
    assert abs(fd - grads[1][1][4]) < 1e-7


def test_restriction_keeps_means_and_discrete_incompressibility():
    r = _rng(5)
    ny, nx, f = 16, 12, 4
    # a discretely divergence-free face field from a stream function psi on
    # cell corners: u = psi[j+1, i] - psi[j, i], v = -(psi[j, i+1] - psi[j, i]),
    # periodic in x, psi = 0 on the bottom and top walls
    psi = np.zeros((ny + 1, nx))
    psi[1:ny] = r.normal(size=(ny - 1, nx))
    u = psi[1:] - psi[:-1]
    v = -(np.roll(psi, -1, axis=1) - psi)[:ny]
    div = (np.roll(u, -1, axis=1) - u) + (np.concatenate([v[1:], np.zeros((1, nx))]) - v)
    assert np.max(np.abs(div)) < 1e-12 and np.max(np.abs(v[0])) < 1e-15
    p = r.normal(size=(ny, nx))
    phi = np.tanh(r.normal(size=(ny, nx)))
    c = C.restrict({"u": u, "v": v, "p": p, "phi": phi}, f)
    assert c["p"].shape == (ny // f, nx // f)
    assert abs(c["p"].sum() * f * f - p.sum()) < 1e-12 and abs(c["phi"].sum() * f * f - phi.sum()) < 1e-12
    cdiv = (np.roll(c["u"], -1, axis=1) - c["u"]) + (np.concatenate([c["v"][1:], np.zeros((1, nx // f))]) - c["v"])
    assert np.max(np.abs(cdiv)) < 1e-12
    assert np.max(np.abs(c["v"][0])) < 1e-15


def test_features_and_correction():
    H, W = 6, 5
    st = {"u": np.full((H, W), 2.0), "v": np.ones((H, W)), "p": np.zeros((H, W)), "phi": np.zeros((H, W))}
    st["v"][0] = 0.0
    x = C.features(st, (2.0, 1.0, 1.0, 1.0))
    assert np.all(x[..., 0] == 1.0)
    assert np.all(x[0, :, 1] == 0.5) and np.all(x[1:-1, :, 1] == 1.0) and np.all(x[-1, :, 1] == 0.5)
    r = _rng(6)
    out = r.normal(size=(H, W, 4))
    phi0 = r.normal(size=(H, W))
    st["phi"] = phi0
    new = C.apply_correction(st, out, (1.0, 2.0, 1.0, 0.5))
    assert abs(new["phi"].sum() - phi0.sum()) < 1e-12
    assert np.all(new["v"][0] == 0.0)
    assert np.allclose(new["u"] - st["u"], out[..., 0])


def test_interface_position_exact_on_linear_profiles():
    H, W = 20, 4
    y = np.arange(H) + 0.5
    phi = np.empty((H, W))
    y0 = np.array([7.3, 10.0, 12.81, 3.5])
    for x in range(W):
        phi[:, x] = 0.1 * (y - y0[x])  # one crossing per column
    top, bot = C.interface_position(phi)
    assert np.allclose(top, y0, atol=1e-12) and np.allclose(bot, y0, atol=1e-12)
    # two crossings in a column (a finger): top and bottom differ
    c = np.where(np.abs(y - 10) < 3.2, 1.0, -1.0)
    phi2 = np.stack([c] * 2, axis=1)
    t2, b2 = C.interface_position(phi2)
    assert np.allclose(t2, 13.0) and np.allclose(b2, 7.0)
    assert np.all(np.isnan(C.interface_position(np.ones((5, 3)))[0]))
