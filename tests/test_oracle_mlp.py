"""Pins of the network oracle: bfloat16 rounding, closed-form forward,
loss values, finite-difference gradients and the first Adam step.  CPU only."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties to even -> 1
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0
    # 1 + 3 * 2^-8 ties between 1 + 2^-7 and 1 + 2^-6: even mantissa -> 1 + 2^-6
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    assert mlp.bf16(np.float32(1 + 2 ** -8 + 2 ** -20)) == 1 + 2 ** -7      # above the tie rounds up
    assert mlp.bf16(np.float32(-3.0)) == -3.0
    assert mlp.bf16(np.float32(0.1)) == 0.10009765625                     # 0x3DCD


def test_parameter_count():
    assert mlp.N_PARAMS == 9154


def test_forward_closed_form():
    """Weights that pass feature 0 through three ReLU layers and read it out:
    out = (relu chain of 2 x0 + 1) in the logit, 0.5 x1 in the energy."""
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["W1"][0, 0] = 2.0
    p["b1"][0] = 1.0
    p["W1"][1, 1] = 1.0
    p["W2"][0, 0] = 1.0
    p["W2"][1, 1] = 1.0
    p["W3"][0, 0] = 1.0
    p["W3"][1, 1] = 1.0
    p["W4"][0, 0] = 1.0
    p["W4"][1, 1] = 0.5
    theta = mlp.pack(p)
    x = np.zeros((3, 10))
    x[:, 0] = [0.25, -2.0, 3.0]
    x[:, 1] = [1.0, 4.0, -1.0]
    out, _ = mlp.forward(theta, x)
    assert np.allclose(out[:, 0], [1.5, 0.0, 7.0])
    assert np.allclose(out[:, 1], [0.5, 2.0, 0.0])


def test_loss_values():
    out = np.array([[0.0, 1.0], [0.0, 1.0]])
    L, g = mlp.loss_and_grad_out(out, np.array([1.0, 0.0]), np.array([3.0, 3.0]))
    # BCE at logit 0 is ln 2 for either label; the gamma adds (1 - 3)^2
    assert L == pytest.approx((2 * math.log(2) + 4.0) / 2)
    assert g[:, 0] == pytest.approx([-0.25, 0.25])
    assert g[:, 1] == pytest.approx([2 * (1.0 - 3.0) / 2, 0.0])


def test_backward_matches_finite_differences():
    """FP64 backward (no bf16 rounding) against central differences."""
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1) * 0.7
    x = rng.normal(size=(12, 10))
    lab = (rng.random(12) < 0.5).astype(float)
    y = rng.normal(size=12)
    L0, g = mlp.loss_grad(theta, x, lab, y, emulate_bf16=False)
    idx = rng.choice(mlp.N_PARAMS, 120, replace=False)
    idx = np.concatenate([idx, [0, 639, 640, 9151, 9152, 9153]])
    h = 1e-6
    num = []
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        num.append((mlp.loss_grad(tp, x, lab, y, False)[0] - mlp.loss_grad(tm, x, lab, y, False)[0]) / (2 * h))
    num = np.array(num)
    assert np.linalg.norm(num - g[idx]) <= 1e-6 * max(np.linalg.norm(num), 1e-12)


def test_bf16_backward_close_to_exact():
    """The bf16-emulated gradient is the exact one up to bfloat16 rounding."""
    rng = np.random.default_rng(2)
    theta = mlp.init_params(3)
    x = rng.normal(size=(256, 10))
    lab = (rng.random(256) < 0.3).astype(float)
    y = rng.normal(size=256)
    _, g64 = mlp.loss_grad(theta, x, lab, y, emulate_bf16=False)
    _, g16 = mlp.loss_grad(theta, x, lab, y, emulate_bf16=True)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


def test_adam_first_step_moves_by_lr_times_sign():
    opt = mlp.Adam(5, lr=1e-3)
    theta = np.zeros(5)
    g = np.array([0.3, -2.0, 1e-3, -1e-2, 5.0])
    new = opt.step(theta, g)
    assert np.allclose(new, -1e-3 * np.sign(g), rtol=1e-4)


def _record(**kw):
    dt = np.dtype([(f, "<f8") for f in ("size", "cog_x", "cog_y", "length", "width", "psi", "skewness",
                                         "kurtosis", "time_gradient", "time_intercept", "leakage", "cog_dist")]
                  + [("n_pix", "<i8"), ("n_islands", "<i8"), ("n_lowgain", "<i8"), ("flags", "<i8")])
    r = np.zeros(1, dt)
    for k, v in kw.items():
        r[k] = v
    return r


def test_features_from_records_hand_record():
    """The network input of one hand-written record, every field distinct:
    the ten columns in the documented order log10(size), length, width,
    cog distance, psi, skewness, kurtosis, time gradient, leakage, islands
    (log10(1000) = 3); fields the network does not read stay out."""
    r = _record(size=1000.0, cog_x=9.1, cog_y=9.2, length=0.11, width=0.022, psi=0.44, skewness=0.55,
                kurtosis=2.66, time_gradient=7.77, time_intercept=9.3, leakage=0.088, cog_dist=0.33,
                n_pix=91, n_islands=3, n_lowgain=94, flags=0)
    x = mlp.features_from_records(r)
    assert x.shape == (1, 10)
    assert x[0].tolist() == [3.0, 0.11, 0.022, 0.33, 0.44, 0.55, 2.66, 7.77, 0.088, 3.0]
    assert mlp.FEATURES[0] == "log10_size" and mlp.FEATURES[9] == "n_islands"


def test_features_from_records_log_size_edges():
    """log10 of the size: exact at powers of ten, -inf at 0, NaN below 0 and
    for a NaN size, so such records can never look in range."""
    sizes = [1e5, 10.0, 0.0, -5.0, float("nan")]
    r = np.concatenate([_record(size=s, length=0.1) for s in sizes])
    x = mlp.features_from_records(r)
    assert x[0, 0] == 5.0 and x[1, 0] == 1.0
    assert x[2, 0] == -math.inf
    assert math.isnan(x[3, 0]) and math.isnan(x[4, 0])
    assert np.all(x[:, 1] == 0.1)


def test_layer_sums_hand_case():
    """Layer 2 with two inputs and hand-set weights: the pre-activation and
    the magnitude sum written out (weights already bfloat16 values)."""
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["W2"][0, 0], p["W2"][1, 0], p["b2"][0] = 0.5, -2.0, 0.25
    p["W2"][0, 3], p["b2"][3] = 3.0, -1.0
    theta = mlp.pack(p)
    h = np.zeros((2, 64))
    h[0, :2] = [1.0, 0.75]
    h[1, :2] = [4.0, 0.0]
    a, mag = mlp.layer_sums(theta, 2, h)
    assert a[0, 0] == 0.5 * 1.0 - 2.0 * 0.75 + 0.25 and mag[0, 0] == 0.5 + 1.5 + 0.25
    assert a[1, 0] == 2.0 + 0.25 and mag[1, 0] == 2.25
    assert a[0, 3] == 3.0 - 1.0 and mag[0, 3] == 4.0
    assert a[1, 3] == 12.0 - 1.0 and mag[1, 3] == 13.0
    assert not np.any(a[:, [1, 2]]) and not np.any(mag[:, 4:])
    # the weights enter rounded to bfloat16: 0.1 becomes 0x3DCD
    p["W2"][0, 5] = 0.1
    a, _ = mlp.layer_sums(mlp.pack(p), 2, h)
    assert a[1, 5] == 4.0 * 0.10009765625


def test_backward_sums_hand_case():
    """Gradient reaching hidden layer 3 from the two outputs: u = g4 W4^T."""
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["W4"][7, 0], p["W4"][7, 1], p["W4"][9, 1] = 2.0, -0.5, 4.0
    g = np.array([[1.0, 2.0], [-3.0, 0.5]])
    u, mag = mlp.backward_sums(mlp.pack(p), 3, g)
    assert u[0, 7] == 2.0 - 1.0 and mag[0, 7] == 3.0
    assert u[1, 7] == -6.0 - 0.25 and mag[1, 7] == 6.25
    assert u[0, 9] == 8.0 and u[1, 9] == 2.0
    assert np.count_nonzero(u) == 4


def test_layer_sums_reproduce_the_pinned_pass():
    """Rounding each layer_sums result to bfloat16 after the ReLU, and the
    masked backward_sums, walk exactly through forward / backward (whose
    results are pinned above by the closed form and finite differences)."""
    rng = np.random.default_rng(4)
    theta = mlp.init_params(4)
    x = rng.normal(size=(50, 10))
    out, cache = mlp.forward(theta, x)
    h = mlp.bf16(x.astype(np.float32))
    for l in (1, 2, 3):
        a, mag = mlp.layer_sums(theta, l, h)
        assert np.all(mag >= np.abs(a))
        h = mlp.bf16(np.maximum(a, 0.0))
        assert np.array_equal(h, cache["h"][l])
    a, _ = mlp.layer_sums(theta, 4, h)
    assert np.array_equal(a, out)
    lab = (rng.random(50) < 0.5).astype(np.float64)
    y = rng.normal(size=50)
    _, g_out = mlp.loss_and_grad_out(out, lab, y)
    grads = mlp.unpack(mlp.backward(theta, cache, g_out))
    g = mlp.bf16(g_out)
    for l in (3, 2, 1):
        u, _ = mlp.backward_sums(theta, l, g)
        g = mlp.bf16(u * (cache["h"][l] > 0))
        assert np.allclose(grads["W%d" % l], cache["h"][l - 1].T @ g, rtol=1e-12, atol=0)


def test_bf16_bracket_holds_float32_sums_in_any_order():
    """Sums of 65 bfloat16 products plus a bias, added in float32 in random
    orders (and with truncation instead of rounding after every addition):
    the rounded result always lies in the bracket, and the bracket is a
    single value when the exact sum is far from a rounding boundary."""
    import oracle.parity as par
    rng = np.random.default_rng(17)
    n_rows, K = 400, 64
    h = mlp.bf16(np.abs(rng.normal(size=(n_rows, K))))
    w = mlp.bf16(rng.normal(size=(n_rows, K)) * 0.2)
    b = rng.normal(size=n_rows).astype(np.float32).astype(np.float64)
    terms = np.concatenate([h * w, b[:, None]], 1)          # products are exact in float32
    exact = terms.sum(1)
    mag = np.abs(terms).sum(1)
    lo, hi = par.bf16_bracket(exact, mag, K + 1, relu=True)
    assert np.all(lo <= hi)
    for trial in range(20):
        perm = rng.permutation(K + 1)
        acc = np.zeros(n_rows, np.float32)
        for k in perm:
            s = acc + terms[:, k].astype(np.float32)
            if trial % 2:       # truncate toward zero instead of rounding
                s64 = acc.astype(np.float64) + terms[:, k]
                s = np.where(np.abs(s.astype(np.float64)) > np.abs(s64), np.nextafter(s, np.float32(0)), s)
            acc = s.astype(np.float32)
        got = mlp.bf16(np.maximum(acc, 0))
        assert np.all((got >= lo) & (got <= hi)), trial
    assert np.mean(lo == hi) > 0.9
