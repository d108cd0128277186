"""Pins of the learned-sketch oracle (oracle/mlp_oracle.py) against facts that
do not come from its own formulas: values of the normal CDF, symmetry
identities, the loss written on n x n matrices, its exact minimisers, central
finite differences of the whole network, and Adam's first-step property."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_gelu_values_and_identities():
    x = np.array([-3.0, -1.0, -0.25, 0.0, 0.5, 1.0, 2.0])
    g = M.gelu(x)
    # gelu(1) = Phi(1), Phi(1) from the normal table; gelu(0) = 0
    assert g[5] == pytest.approx(0.8413447460685429, abs=1e-15)
    assert g[3] == 0.0
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.allclose(M.gelu(x) - M.gelu(-x), x, atol=1e-15)
    # derivative against central differences
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(x), fd, atol=1e-8)


def _orth(rng, n, k):
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return q


def test_loss_blocks_equal_dense_definition():
    rng = np.random.default_rng(1)
    n, k = 17, 4
    S = _orth(rng, n, k)
    D = np.array([5.0, 2.0, 0.7, 0.1])
    Z = rng.standard_normal((n, k))
    l_blk, _ = M.loss_and_dZ(Z, S, D)
    assert l_blk == pytest.approx(M.loss_definition(Z, S, D), rel=1e-12)


def test_loss_exact_minimisers_and_gradient():
    rng = np.random.default_rng(2)
    n, k = 13, 3
    S = _orth(rng, n, k)
    D = np.array([3.0, 1.5, 0.2])
    Q = _orth(rng, k, k)
    Zstar = (S * np.sqrt(D)) @ Q  # Z Z^T = S D S^T for every rotation Q
    l, dZ = M.loss_and_dZ(Zstar, S, D)
    assert abs(l) < 1e-13 and np.abs(dZ).max() < 1e-12
    # gradient against central differences of the dense definition
    Z = rng.standard_normal((n, k))
    _, dZ = M.loss_and_dZ(Z, S, D)
    eps = 1e-6
    fd = np.zeros_like(Z)
    for i in range(n):
        for j in range(k):
            Zp, Zm = Z.copy(), Z.copy()
            Zp[i, j] += eps
            Zm[i, j] -= eps
            fd[i, j] = (M.loss_definition(Zp, S, D) - M.loss_definition(Zm, S, D)) / (2 * eps)
    assert np.allclose(dZ, fd, rtol=1e-6, atol=1e-8)


def test_network_gradient_central_differences():
    rng = np.random.default_rng(3)
    n, h, k, B = 6, 5, 2, 3
    tot = M.dims_offsets(n, h, k)["total"]
    theta = M.he_init(rng.standard_normal(tot), n, h, k) + 0.05 * rng.standard_normal(tot)
    X = M.normalise_input(rng.standard_normal((n, B)))
    Ss = [_orth(rng, n, k) for _ in range(B)]
    Ds = [np.sort(rng.uniform(0.1, 3.0, k))[::-1] for _ in range(B)]
    loss, grad = M.loss_and_grad(theta, X, Ss, Ds, n, h, k)

    def f(t):
        Z, _ = M.forward(t, X, n, h, k)
        return sum(M.loss_definition(Z[b], Ss[b], Ds[b]) for b in range(B)) / B

    assert loss == pytest.approx(f(theta), rel=1e-12)
    eps = 1e-6
    for idx in rng.choice(tot, 40, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[idx] += eps
        tm[idx] -= eps
        fd = (f(tp) - f(tm)) / (2 * eps)
        assert grad[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), idx


def test_input_normalisation():
    b = np.array([[3.0, 0.0], [4.0, 2.0]])
    x = M.normalise_input(b)
    assert np.allclose(np.linalg.norm(x, axis=0), math.sqrt(2.0))
    assert np.allclose(x[:, 0], np.array([3.0, 4.0]) / 5.0 * math.sqrt(2.0))


def test_adam_first_steps():
    # step 1: m_hat = g, v_hat = g^2, so every parameter moves by lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    th = np.array([1.0, 1.0, 1.0])
    t1, m, v = M.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # step 2 with the same gradient: the bias-corrected moments are again g, g^2
    t2, _, _ = M.adam_step(t1, g, m, v, 2, lr=0.01)
    assert np.allclose(t2, t1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-10)


def test_he_init_scale():
    n, h, k = 64, 32, 2
    o = M.dims_offsets(n, h, k)
    z = np.random.default_rng(4).standard_normal(o["total"])
    th = M.he_init(z, n, h, k)
    W1, b1, W2, b2, W3, b3 = M.unpack(th, n, h, k)
    assert W1.var() == pytest.approx(2.0 / n, rel=0.1) and W3.var() == pytest.approx(2.0 / h, rel=0.1)
    assert not b1.any() and not b2.any() and not b3.any()
