"""Pins of the FP64 reference of the learned guess (oracle/mlp.py): the hand-written gradient
against central finite differences, BF16 rounding against the bit definition, the Adam step
against its closed form for a constant gradient, and a tiny fit that must reduce the loss."""
import numpy as np

import oracle as O
from oracle import mlp as M


def test_bf16_rounding_bits():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even gives 1; just above rounds up
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0
    assert M.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6        # tie to even (upwards)
    x = np.random.default_rng(0).standard_normal(1000)
    r = M.bf16(x)
    assert np.all(np.abs(r / x - 1) <= 2.0 ** -8)
    assert np.all(M.bf16(r) == r)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    theta = M.init(3) + 0.05 * rng.standard_normal(M.N_PARAM)
    x = rng.standard_normal((3, 40))
    t = rng.standard_normal(40)
    loss, g = M.loss_and_grad(theta, x, t, bf16_round=False)
    idx = np.concatenate([np.arange(0, 192, 7), np.arange(192, 256, 5),
                          rng.choice(np.arange(256, 4352), 60, replace=False),
                          np.arange(4352, 4481, 9), [4480]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss_and_grad(tp, x, t, False)[0] - M.loss_and_grad(tm, x, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_silu_derivative():
    a = np.linspace(-20, 20, 401)
    h = 1e-6
    fd = (M.silu(a + h) - M.silu(a - h)) / (2 * h)
    assert np.max(np.abs(fd - M.dsilu(a))) < 1e-8


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are exactly g and g^2, so every
    # step moves each parameter by lr * g / (|g| + eps)
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -7.0])
    m = v = np.zeros(5)
    for k in range(1, 6):
        theta, m, v = M.adam(theta, g, m, v, k, 0.01)
    assert np.allclose(theta, -5 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_small_fit_reduces_loss_on_oracle_labels():
    # labels: log of the oracle's root ht on conversion-batch states; a few hundred Adam steps
    # must cut the loss of a fresh network clearly (the three inputs cannot resolve L for
    # hypersonic states, where it is a difference far below their rounding, so the floor is high)
    import workloads as W
    prim = W.conversion_batch(4000, seed=31)
    cons = O.prim2cons(prim)
    w, st, _ = O.cons2prim(cons)
    ok = st == 0
    ht = np.array([O.htilde_of_theta(p / r) for p, r in zip(w[4, ok], w[0, ok])])
    f = M.features(cons[:, ok])
    mu, sd = f.mean(axis=1, keepdims=True), f.std(axis=1, keepdims=True)
    x = (f - mu) / sd
    y = np.log(ht)
    t = (y - y.mean()) / y.std()
    theta = M.init(0)
    m = v = np.zeros_like(theta)
    l0 = M.loss_and_grad(theta, x, t)[0]
    for k in range(1, 301):
        loss, g = M.loss_and_grad(theta, x, t)
        theta, m, v = M.adam(theta, g, m, v, k, 3e-3)
    assert loss < 0.7 * l0, (l0, loss)
