"""Oracle of the gamma/hadron + energy network — TEST INFRASTRUCTURE ONLY.

The paper lists gamma/hadron separation and energy reconstruction among the
products of the reconstruction (Section 4.1) without naming a method; the
reading used here is a small multilayer perceptron on per-telescope image
parameters, with plain scaled-width / scaled-length box cuts as the baseline
and fallback (see boxcut.py).

Network: 10 standardised features -> 64 -> 64 -> 64 (ReLU) -> 2 outputs
(gamma logit, log10 E/TeV).  Parameters, in this order (9154 values):
W1 [10][64], b1 [64], W2 [64][64], b2, W3 [64][64], b3, W4 [64][2], b4 [2],
with W[in][out] (a layer computes a = h @ W + b).

Mixed precision, as the kernels do it (bfloat16 storage, wide accumulation):
  forward   x16 = bf16(standardised x);  a_l = h16_{l-1} @ bf16(W_l) + b_l;
            h16_l = bf16(relu(a_l)) for l = 1..3;  out = h16_3 @ bf16(W4) + b4
  loss      L = (1/B) sum_i [ BCE(logit_i, label_i) + m_i (y_i - e_i)^2 ],
            m_i = 1 for gammas (energy is learned on gammas only)
  backward  g4 = bf16(dL/dout);  g_l = bf16((g_{l+1} @ bf16(W_{l+1})^T) * [h16_l > 0]);
            dW_l = h16_{l-1}^T @ g_l,  db_l = sum_i g_l  (wide accumulation)
  Adam      FP32 master weights, beta 0.9 / 0.999, eps 1e-8, bias-corrected.

bfloat16 rounding is round-to-nearest-even of the float32 value.  Sums here
are FP64; the kernels accumulate in FP32, so parity is to a tolerance.

Parity status: pinned by bf16 known values, a closed-form forward pass, loss
values, finite differences and the first Adam step (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 10, 64, 2
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_HID, N_OUT)), ("b4", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
FEATURES = ("log10_size", "length", "width", "cog_dist", "psi", "skewness", "kurtosis", "time_gradient",
            "leakage", "n_islands")


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    assert theta.size == N_PARAMS
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[k:k + n].reshape(shp)
        k += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed):
    """He-normal weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            p[name] = rng.normal(0.0, np.sqrt(2.0 / shp[0]), size=shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p).astype(np.float32).astype(np.float64)


def standardise(x, mean, std):
    return (np.asarray(x, np.float64) - np.asarray(mean, np.float64)) / np.asarray(std, np.float64)


def forward(theta, xs, emulate_bf16=True):
    """xs: standardised features [B][10].  Returns (out [B][2], cache)."""
    p = unpack(theta)
    q = bf16 if emulate_bf16 else (lambda v: np.asarray(v, np.float64))
    h = [q(np.asarray(xs, np.float32))]
    a = []
    for l in (1, 2, 3):
        al = h[-1] @ q(p["W%d" % l]) + p["b%d" % l]
        a.append(al)
        h.append(q(np.maximum(al, 0.0)))
    out = h[-1] @ q(p["W4"]) + p["b4"]
    return out, {"h": h, "a": a, "p": p}


def loss_and_grad_out(out, label, log10e):
    """Mean BCE on the logit + gamma-masked squared energy error, and dL/dout."""
    z, e = out[:, 0], out[:, 1]
    B = out.shape[0]
    lab = np.asarray(label, np.float64)
    m = (lab > 0.5).astype(np.float64)
    bce = np.maximum(z, 0) - z * lab + np.log1p(np.exp(-np.abs(z)))
    se = m * (e - np.asarray(log10e, np.float64)) ** 2
    L = float(np.sum(bce + se) / B)
    sig = 1.0 / (1.0 + np.exp(-z))
    g = np.stack([(sig - lab) / B, 2.0 * m * (e - np.asarray(log10e, np.float64)) / B], 1)
    return L, g


def backward(theta, cache, g_out, emulate_bf16=True):
    """Gradient of the loss w.r.t. all parameters (packed), given dL/dout."""
    p, h = cache["p"], cache["h"]
    q = bf16 if emulate_bf16 else (lambda v: np.asarray(v, np.float64))
    grads = {}
    g = q(g_out)
    grads["W4"] = h[3].T @ g
    grads["b4"] = g.sum(0)
    for l in (3, 2, 1):
        upstream = g @ q(p["W%d" % (l + 1)]).T
        relu_mask = (h[l] > 0) if emulate_bf16 else (cache["a"][l - 1] > 0)
        g = q(upstream * relu_mask)
        grads["W%d" % l] = h[l - 1].T @ g
        grads["b%d" % l] = g.sum(0)
    return pack(grads)


def layer_sums(theta, layer, h_prev):
    """One layer of the forward pass from given bf16-valued inputs h_prev
    [B][fan_in]: the pre-activation a = h_prev @ bf16(W_l) + b_l (FP64) and
    mag = |h_prev| @ |bf16(W_l)| + |b_l|, the sum of the absolute values of
    its terms.  layer 1..4 (4: the output layer, whose a is the output)."""
    p = unpack(theta)
    W = bf16(p["W%d" % layer])
    b = p["b%d" % layer]
    h = np.asarray(h_prev, np.float64)
    return h @ W + b, np.abs(h) @ np.abs(W) + np.abs(b)


def backward_sums(theta, layer, g_next):
    """The gradient that reaches the pre-activation of hidden layer l (1..3)
    from bf16-valued gradients g_next [B][fan_out] of layer l+1, before the
    ReLU mask: u = g_next @ bf16(W_{l+1})^T (FP64), and the sum of the
    absolute values of its terms."""
    p = unpack(theta)
    W = bf16(p["W%d" % (layer + 1)])
    g = np.asarray(g_next, np.float64)
    return g @ W.T, np.abs(g) @ np.abs(W).T


def loss_grad(theta, xs, label, log10e, emulate_bf16=True):
    out, cache = forward(theta, xs, emulate_bf16)
    L, g = loss_and_grad_out(out, label, log10e)
    return L, backward(theta, cache, g, emulate_bf16)


class Adam:
    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def features_from_records(rec):
    """The 10 network inputs of Hillas records (any structured array with the
    record fields): log10(size) and nine raw parameters."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.stack([np.log10(np.asarray(rec["size"], np.float64)), rec["length"], rec["width"], rec["cog_dist"],
                         rec["psi"], rec["skewness"], rec["kurtosis"], rec["time_gradient"], rec["leakage"],
                         np.asarray(rec["n_islands"], np.float64)], 1).astype(np.float64)
