"""Pins of the warm-start network oracle (oracle/mlp_oracle.py).

The analytic gradients are checked against central finite differences of the
loss (plain float64, no rounding), the bfloat16 rounding against values fixed
by round-to-nearest-even, the Adam step against its closed form at the first
step, and the loss against a closed form.  A planted mistake in the
back-propagation (a missing ReLU mask) is caught by the finite differences.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as N

DIMS = (16, 32, 32, 48)


def _params(dims, seed):
    rng = np.random.default_rng(seed)
    d0, d1, d2, d3 = dims
    parts = []
    for rows, cols in ((d1, d0), (d2, d1), (d3, d2)):
        parts.append(rng.standard_normal(rows * cols) * np.sqrt(2.0 / cols))
        parts.append(0.1 * rng.standard_normal(rows))
    return np.concatenate(parts)


def _fd_gradient(params, dims, x, t, h=1e-6):
    g = np.zeros_like(params)
    for i in range(len(params)):
        p = params.copy()
        p[i] += h
        lp = N.loss_and_gradients(p, dims, x, t, rounding=False)[0]
        p[i] -= 2 * h
        lm = N.loss_and_gradients(p, dims, x, t, rounding=False)[0]
        g[i] = (lp - lm) / (2 * h)
    return g


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    params = _params(DIMS, 1)
    x = rng.standard_normal((16, DIMS[0]))
    t = rng.standard_normal((16, DIMS[3]))
    loss, g = N.loss_and_gradients(params, DIMS, x, t, rounding=False)
    gf = _fd_gradient(params, DIMS, x, t)
    assert np.max(np.abs(g - gf)) <= 1e-7 * np.max(np.abs(g)) + 1e-10
    # every block of the packed gradient is exercised
    assert np.count_nonzero(g) > 0.5 * len(g)


def test_planted_missing_relu_mask_is_caught(monkeypatch):
    rng = np.random.default_rng(4)
    params = _params(DIMS, 2)
    x = rng.standard_normal((16, DIMS[0]))
    t = rng.standard_normal((16, DIMS[3]))
    good = N.loss_and_gradients

    def bad(params, dims, x, t, rounding=True):
        # back-propagation through layer 2 without the ReLU derivative
        (W1, _), (W2, _), (W3, _) = N.unpack(params, dims)
        y, (x0, z1, h1, z2, h2) = N.forward(params, dims, x, rounding)
        B, d3 = y.shape
        dy = 2.0 * (y - t) / (B * d3)
        dz2 = dy @ W3
        dz1 = (dz2 @ W2) * (z1 > 0)
        grads = np.concatenate([(dz1.T @ x0).ravel(), dz1.sum(0), (dz2.T @ h1).ravel(),
                                dz2.sum(0), (dy.T @ h2).ravel(), dy.sum(0)])
        return float(np.mean((y - t) ** 2)), grads
    monkeypatch.setattr(N, "loss_and_gradients", bad)
    g = bad(params, DIMS, x, t, rounding=False)[1]
    monkeypatch.setattr(N, "loss_and_gradients", good)
    gf = _fd_gradient(params, DIMS, x, t)
    assert np.max(np.abs(g - gf)) > 1e-3 * np.max(np.abs(gf))


def test_bf16_round_to_nearest_even():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                        # tie, even neighbour below
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,        # tie, even neighbour above
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,
        -(one + 2.0 ** -8 + 2.0 ** -20): -(one + 2.0 ** -7),
        3.0: 3.0, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130,  # exact (subnormal float32 too)
    }
    x = np.array(list(cases.keys()))
    assert np.array_equal(N.bf16(x), np.array(list(cases.values())))


def test_loss_closed_form_zero_weights():
    d0, d1, d2, d3 = DIMS
    params = np.zeros(N.n_params(DIMS))
    (_, _), (_, _), (_, b3) = N.unpack(params, DIMS)
    b3[:] = np.linspace(-1.0, 1.0, d3)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((16, d0))
    t = rng.standard_normal((16, d3))
    loss, g = N.loss_and_gradients(params, DIMS, x, t, rounding=False)
    assert np.isclose(loss, np.mean((b3[None, :] - t) ** 2), rtol=1e-15)
    # only the output bias has a gradient: mean over the batch of 2 (b3 - t) / d3
    gb3 = g[-d3:]
    assert np.allclose(gb3, np.sum(2.0 * (b3[None, :] - t), axis=0) / (16 * d3), rtol=1e-14)
    assert np.all(g[:-d3] == 0.0)


def test_adam_first_step_closed_form():
    # at the first step m_hat = g and v_hat = g^2: each parameter moves by
    # lr * g / (|g| + eps), i.e. by lr against the sign of its gradient
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m, v = N.adam_step(p, g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # a second step with the same gradient moves by the same amount again
    p2, _, _ = N.adam_step(p1, g, m, v, 2, 0.01)
    assert np.allclose(p2 - p1, p1 - p, rtol=1e-9, atol=1e-15)


def test_rounded_gradients_close_to_exact():
    rng = np.random.default_rng(6)
    params = _params(DIMS, 3)
    x = rng.standard_normal((16, DIMS[0]))
    t = rng.standard_normal((16, DIMS[3]))
    _, g = N.loss_and_gradients(params, DIMS, x, t, rounding=False)
    _, gr = N.loss_and_gradients(params, DIMS, x, t, rounding=True)
    assert np.linalg.norm(gr - g) <= 3e-2 * np.linalg.norm(g)
    assert not np.array_equal(gr, g)
