"""Pins of the oracle's training rule (Sec. 4.3), CPU only.

- FP64 gradients against central finite differences of the loss;
- a zero learning rate returns the initialisation exactly;
- the first Adam step moves every parameter with a non-zero gradient by
  almost exactly lr against the gradient's sign (closed form of Adam's first
  bias-corrected step);
- sampling: the 8:2 split, the 2^15 filter, and the drawn set equals the
  splitmix64 threshold rule recomputed here;
- the selected network never scores below the untrained one, and training
  on a smooth field lowers the validation entropy.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2309_09778_amd import synth


def _samples(n, K, seed):
    rng = np.random.default_rng(seed)
    u = rng.integers(-50, 50, size=(n, K)).astype(np.float64)
    t = (u @ rng.normal(0, 0.5, K) + rng.normal(0, 3, n)).round()
    return u, t


@pytest.mark.parametrize("K,H", [(6, 16), (2, 8), (6, 32)])
def test_gradient_matches_finite_differences(K, H):
    rng = np.random.default_rng(K * 100 + H)
    th = rng.normal(0, 0.3, H * K + 2 * H + 1)
    u, t = _samples(64, K, 3)
    # keep pre-activations away from the kink at 0 so the loss is smooth
    loss, g = O.loss_grad(th, H, K, 0.01, u, t, 7.0, 1e-3)
    h = 1e-6
    num = np.zeros_like(th)
    for q in range(th.size):
        a, b = th.copy(), th.copy()
        a[q] += h
        b[q] -= h
        num[q] = (O.loss_grad(a, H, K, 0.01, u, t, 7.0, 1e-3)[0] -
                  O.loss_grad(b, H, K, 0.01, u, t, 7.0, 1e-3)[0]) / (2 * h)
    rel = np.abs(num - g) / np.maximum(np.abs(g), 1e-3)
    assert np.median(rel) < 1e-6 and np.max(rel) < 1e-4, (np.median(rel), np.max(rel))


def test_zero_learning_rate_returns_initialisation():
    m = O.mlp_init(3, 16, seed=4)
    th0 = O.theta_from_model(m)
    u, t = _samples(1000, 6, 9)
    for opt in (0, 1):
        th, *_ = O.train_pass(th0, 16, 6, 0.01, u, t, 5.0, 1e-4, 0.0, 256, opt)
        assert np.array_equal(th, th0)


def test_first_adam_step_closed_form():
    m = O.mlp_init(3, 8, seed=2)
    th0 = O.theta_from_model(m)
    u, t = _samples(256, 6, 1)
    _, g = O.loss_grad(th0, 8, 6, 0.01, u, t, 4.0, 0.0)
    lr = 1e-3
    th, am, av, step = O.train_pass(th0, 8, 6, 0.01, u, t, 4.0, 0.0, lr, 256, 1)
    assert step == 1
    # m_hat = g, v_hat = g^2  =>  step = lr * g / (|g| + 1e-8)
    expect = th0 - lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(th, expect, rtol=0, atol=1e-12)
    # SGD: plain gradient step
    th_s, *_ = O.train_pass(th0, 8, 6, 0.01, u, t, 4.0, 0.0, lr, 256, 0)
    assert np.allclose(th_s, th0 - lr * g, rtol=0, atol=1e-15)


def test_sampling_rule():
    x = synth.gaussian_bumps((40, 40, 40), seed=1, zero_frac=0.01)
    c = O.consts(x, 1e-2)
    p = O.transform_field(x, c)
    rho, seed = 0.1, 12345
    s = O.sample(p, c, 8, rho, seed)
    idx = s["idx"].astype(np.int64)
    # recompute the draw: U(i) = (splitmix64(seed ^ i) >> 11) 2^-53 < rho, interior points
    zz, yy, xx = np.unravel_index(idx, p.shape)
    assert np.all((zz > 0) & (yy > 0) & (xx > 0))
    for i, v in zip(idx[:300], s["is_val"][:300]):
        U = (O.splitmix64(seed ^ int(i)) >> 11) * 2.0 ** -53
        assert U < rho and (U < 0.2 * rho) == bool(v)
    frac_val = s["is_val"].mean()
    assert 0.17 < frac_val < 0.23
    assert len(idx) / ((39 ** 3) * rho) > 0.5
    # every kept stencil lies in one sign range
    vals = np.stack([p[zz - a, yy - b, xx - d] for a in (0, 1) for b in (0, 1) for d in (0, 1)], 1)
    pos = (vals > c["p_zero"]) & (vals <= c["b_sign"])
    assert np.all(pos.all(1) | (vals > c["b_sign"]).all(1))
    # inputs and targets are neighbour differences of the grid field
    i0 = idx[0]
    z, y, xq = np.unravel_index(i0, p.shape)
    n1 = int(p[z, y, xq - 1])
    assert s["t"][0] == int(p[z, y, xq]) - n1
    assert s["u"][0, 0] == int(p[z, y - 1, xq]) - n1
    assert s["u"][0, 5] == int(p[z - 1, y - 1, xq - 1]) - n1
    assert np.all(np.abs(s["u"]) < 32768) and np.all(np.abs(s["t"]) < 32768)


@pytest.mark.parametrize("kind", ["bumps", "grf"])
def test_training_rule_selects_no_worse_than_untrained(kind):
    if kind == "bumps":
        x = synth.gaussian_bumps((48, 48, 48), seed=2, zero_frac=0.01)
    else:
        x = synth.lognormal_grf((64, 64, 64), seed=1001, decades=8, neg_frac=0.1,
                                zero_frac=0.005)
    c = O.consts(x, 1e-2)
    p = O.transform_field(x, c)
    init = O.mlp_init(3, 16, seed=7)
    model, idx, ntr, nva = O.train_rule(p, c, 8, init, rho=0.1, seed=99)
    s = O.sample(p, c, 8, 0.1, 99)
    uv, tv = s["u"][s["is_val"]], s["t"][s["is_val"]]
    assert nva == len(tv) and ntr == len(s["t"]) - nva
    gain = (O.val_score(model, uv, tv) - O.val_score(init, uv, tv)) / 2.0 ** 32 / nva
    assert gain >= 0
    if kind == "grf":
        # log-normal k^-3 field: one SGD pass buys a large entropy drop
        assert idx > 0 and gain > 0.3, gain


@pytest.mark.parametrize("K,H,sigma", [(6, 16, 7.3), (6, 32, 0.37), (2, 8, 123.0)])
def test_fold_is_scale_equivariant(K, H, sigma):
    """The exported network (scale folded in: w1 / s, b1, v s, b2 s) is the
    trained one moved back to grid units: y_raw(u) = s y_scaled(u / s) for
    every u.  Any other placement of s (b1 s, w1 s, v / s, b2 unscaled)
    breaks the identity by far more than the FP32 rounding of the weights."""
    rng = np.random.default_rng(K * 1000 + H)
    th = rng.normal(0, 0.5, H * K + 2 * H + 1)
    tmpl = O.mlp_init(3 if K == 6 else 2, H, seed=1)
    m = O.model_from_theta(tmpl, th, sigma)
    u = rng.integers(-500, 501, size=(400, K)).astype(np.float32)
    y_raw, _ = O.mlp_eval_f64(m, u)
    y_scaled = O.theta_eval(th, H, K, 0.01, u, sigma)
    W, b1, v, b2 = th[:H * K].reshape(H, K), th[H * K:H * K + H], th[H * K + H:-1], th[-1]
    mag = sigma * ((np.abs(u.astype(np.float64)) / sigma @ np.abs(W).T + np.abs(b1)) @ np.abs(v)
                   + abs(b2))
    # each folded weight is one FP32 rounding away from its exact value
    tol = 2.0 ** -21 * mag
    assert np.all(np.abs(y_raw - sigma * y_scaled) <= tol)
    # and the identity is not satisfied by accident: every weight group matters
    for name in ("w1", "b1", "v"):
        bad = dict(m)
        bad[name] = (np.asarray(m[name], np.float64) * (sigma if name != "v" else 1 / sigma)
                     ).astype(np.float32)
        yb, _ = O.mlp_eval_f64(bad, u)
        assert np.max(np.abs(yb - sigma * y_scaled) / tol) > 10, name
    bad = dict(m, b2=float(np.float32(th[-1])))
    yb, _ = O.mlp_eval_f64(bad, u)
    assert np.max(np.abs(yb - sigma * y_scaled) / tol) > 10
