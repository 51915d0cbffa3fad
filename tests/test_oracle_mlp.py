"""Pins for the FP64 reference MLP: finite differences, Adam's first step in closed form,
and an affine special case with a least-squares answer."""
import numpy as np

from oracle.mlp import MLP, Adam, dsilu, precond_loss, silu


def test_silu_derivative_matches_finite_difference():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (silu(z + h) - silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - dsilu(z))) < 1e-9


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    net = MLP(7, 5, width=16, seed=1)
    X = rng.standard_normal((9, 7))
    g = rng.standard_normal((9, 4))
    gs = rng.standard_normal((9, 4))
    w = rng.standard_normal(9)

    def L():
        y, _ = net.forward(X)
        return precond_loss(y, g, gs, w, 4)[0]

    y, cache = net.forward(X)
    _, dy = precond_loss(y, g, gs, w, 4)
    grads = net.backward(cache, dy)
    h = 1e-6
    for p, gp in zip(net.params, grads):
        flat = p.reshape(-1)
        gflat = gp.reshape(-1)
        for k in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            old = flat[k]
            flat[k] = old + h
            lp = L()
            flat[k] = old - h
            lm = L()
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[k]) <= 1e-7 * max(1.0, abs(fd)), (fd, gflat[k])


def test_adam_first_step_closed_form():
    """After one step m/c1 = g and v/c2 = g^2, so p moves by lr * g / (|g| + eps)."""
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    opt = Adam(p, lr=0.01, eps=1e-8)
    p0 = p[0].copy()
    opt.step(p, g)
    assert np.allclose(p[0], p0 - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=0, atol=1e-15)


def test_training_reaches_least_squares_fit_of_affine_target():
    """A target that is an affine function of the inputs is learnt to small error."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((256, 4))
    A = rng.standard_normal((4, 2))
    T = X @ A + 0.5
    net = MLP(4, 2, width=32, seed=4)
    opt = Adam(net.params, lr=3e-3)
    for _ in range(3000):
        y, cache = net.forward(X)
        dy = (y - T) / len(X)
        opt.step(net.params, net.backward(cache, dy))
    y, _ = net.forward(X)
    assert np.sqrt(np.mean((y - T) ** 2)) < 2e-2
