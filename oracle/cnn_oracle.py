"""CPU reference of the learned coarse-grid correction (TEST INFRASTRUCTURE).

Plain NumPy, FP64, written for checking the HIP kernels of the learned part:
only tests/, __graft_entry__.smoke() and bench.py's CPU baseline may import it.
Nothing here is used by the product path.

What it computes (the network and its data path, not part of the paper's
method; the paper's Sec. 4 Rayleigh-Taylor set-up supplies the flows it is
trained on):

* restriction of a fine 2-D state to a grid coarser by an integer factor f:
  cell averages of p and phi over f x f cells; the x-face velocity of a coarse
  cell's low face is the mean of the f fine x-faces on that coarse face (and
  likewise for the y-face velocity);
* features of a coarse state: channels (u_c, v_c, p, phi) at cell centres,
  u_c = (u[i] + u[i+1]) / 2 with x periodic, v_c = (v[j] + v[j+1]) / 2 with the
  face above the top row equal to 0 (wall), each channel divided by its scale;
* a 3-layer network of 3 x 3 convolutions, channels 4 -> 32 -> 32 -> 4, ReLU
  after the first two; x periodic, y zero-padded (walls); arrays are NHWC
  (batch, y, x, channel), weights (C_out, 3, 3, C_in) indexed by (dy+1, dx+1);
* the loss: mean over all outputs of (out - target)^2 and its gradients;
* the correction: state += scale * out, the y-face correction on the wall
  row set to 0, the phi correction projected to zero mean (phase mass kept);
* the interface position: per column, the outermost phi = 0 crossings (the
  first sign change scanning down from the top and up from the bottom),
  linearly interpolated between cell centres (y = j + 1/2).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (4, 32, 32, 4)


def restrict(fields: dict, f: int) -> dict:
    """fields: u, v, p, phi of shape (ny, nx) -> coarse (ny/f, nx/f)."""
    p, phi, u, v = (np.asarray(fields[k], dtype=np.float64) for k in ("p", "phi", "u", "v"))
    ny, nx = p.shape
    H, W = ny // f, nx // f
    out = {}
    for k, a in (("p", p), ("phi", phi)):
        out[k] = a.reshape(H, f, W, f).mean(axis=(1, 3))
    # x-faces at coarse low faces: fine face index f*I, averaged over f rows
    out["u"] = u[:, ::f].reshape(H, f, W).mean(axis=1)
    # y-faces at coarse low faces: fine face index f*J, averaged over f columns
    out["v"] = v[::f, :].reshape(H, W, f).mean(axis=2)
    return out


def features(st: dict, scale) -> np.ndarray:
    """Coarse state -> (H, W, 4) array of (u_c, v_c, p, phi) / scale."""
    u, v, p, phi = (np.asarray(st[k], dtype=np.float64) for k in ("u", "v", "p", "phi"))
    uc = 0.5 * (u + np.roll(u, -1, axis=1))
    vn = np.concatenate([v[1:], np.zeros((1, v.shape[1]))], axis=0)
    vc = 0.5 * (v + vn)
    x = np.stack([uc, vc, p, phi], axis=-1)
    return x / np.asarray(scale, dtype=np.float64)


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x (B, H, W, Ci), w (Co, 3, 3, Ci), b (Co): out[y, x] = b + sum over
    taps of w[:, dy+1, dx+1, :] . x[y+dy, (x+dx) mod W] (zero outside 0..H-1)."""
    B, H, W, Ci = x.shape
    out = np.broadcast_to(b, (B, H, W, w.shape[0])).astype(np.float64).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            sh = np.roll(x, -dx, axis=2)            # sh[:, y, x] = x[:, y, x+dx]
            shy = np.zeros_like(sh)
            if dy == 0:
                shy = sh
            elif dy == 1:
                shy[:, :-1] = sh[:, 1:]             # row y reads y+1
            else:
                shy[:, 1:] = sh[:, :-1]             # row y reads y-1
            out += np.einsum("bhwi,oi->bhwo", shy, w[:, dy + 1, dx + 1, :])
    return out


def conv3x3_input_grad(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of sum(g * conv3x3(x)) with respect to x."""
    B, H, W, Co = g.shape
    gx = np.zeros((B, H, W, w.shape[3]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            t = np.einsum("bhwo,oi->bhwi", g, w[:, dy + 1, dx + 1, :])
            # output (y, x) read input (y+dy, x+dx): send t back there
            if dy == 0:
                ty = t
            else:
                ty = np.zeros_like(t)
                if dy == 1:
                    ty[:, 1:] = t[:, :-1]
                else:
                    ty[:, :-1] = t[:, 1:]
            gx += np.roll(ty, dx, axis=2)
    return gx


def conv3x3_weight_grad(g: np.ndarray, x: np.ndarray):
    """Gradients of sum(g * conv3x3(x)) with respect to w and b."""
    Co, Ci = g.shape[3], x.shape[3]
    gw = np.zeros((Co, 3, 3, Ci))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            sh = np.roll(x, -dx, axis=2)
            shy = np.zeros_like(sh)
            if dy == 0:
                shy = sh
            elif dy == 1:
                shy[:, :-1] = sh[:, 1:]
            else:
                shy[:, 1:] = sh[:, :-1]
            gw[:, dy + 1, dx + 1, :] = np.einsum("bhwo,bhwi->oi", g, shy)
    return gw, g.sum(axis=(0, 1, 2))


def init_params(seed: int = 0) -> list:
    """He-uniform weights, zero biases, the last layer scaled by 0.1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for layer in range(3):
        ci, co = CHANNELS[layer], CHANNELS[layer + 1]
        lim = np.sqrt(6.0 / (9 * ci))
        w = rng.uniform(-lim, lim, size=(co, 3, 3, ci))
        if layer == 2:
            w *= 0.1
        params.append((w, np.zeros(co)))
    return params


def forward(params, x):
    """Returns the output and the activations (input of every layer)."""
    acts = [x]
    h = x
    for layer, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        h = np.maximum(z, 0.0) if layer < 2 else z
        if layer < 2:
            acts.append(h)
    return h, acts


def loss_and_grads(params, x, target):
    """Mean squared error over all outputs and its gradients (w, b per layer)."""
    out, acts = forward(params, x)
    n = out.size
    loss = float(np.mean((out - target) ** 2))
    g = 2.0 * (out - target) / n
    grads = [None] * 3
    for layer in (2, 1, 0):
        w, _ = params[layer]
        grads[layer] = conv3x3_weight_grad(g, acts[layer])
        if layer > 0:
            g = conv3x3_input_grad(g, w) * (acts[layer] > 0)
    return loss, grads, out


def apply_correction(st: dict, out: np.ndarray, scale) -> dict:
    """st (coarse u, v, p, phi) += scale * out (H, W, 4); v correction 0 on
    the wall row (j = 0); phi correction minus its mean."""
    s = np.asarray(scale, dtype=np.float64)
    d = out * s
    du, dv, dp, dphi = (d[..., c] for c in range(4))
    dv = dv.copy()
    dv[0, :] = 0.0
    dphi = dphi - dphi.mean()
    return {"u": st["u"] + du, "v": st["v"] + dv, "p": st["p"] + dp, "phi": st["phi"] + dphi}


def interface_position(phi: np.ndarray):
    """phi (H, W) -> (top, bottom) heights per column: the first sign change
    of phi scanning from the top row down and from the bottom row up, linearly
    interpolated between the cell centres; NaN where the column has none."""
    H, W = phi.shape
    top = np.full(W, np.nan)
    bot = np.full(W, np.nan)
    for x in range(W):
        c = phi[:, x]
        for j in range(H - 1, 0, -1):          # pair (j-1, j), from the top
            if (c[j - 1] > 0) != (c[j] > 0):
                top[x] = (j - 1 + 0.5) + c[j - 1] / (c[j - 1] - c[j])
                break
        for j in range(0, H - 1):              # pair (j, j+1), from the bottom
            if (c[j] > 0) != (c[j + 1] > 0):
                bot[x] = (j + 0.5) + c[j] / (c[j] - c[j + 1])
                break
    return top, bot
