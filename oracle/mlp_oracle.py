"""CPU FP64 oracle of the learned sketch (a small MLP that maps the control
member's right-hand side to sketch directions).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's
CPU leg, never by the library.  Plain numpy, FP64, no autograd: forward pass,
loss and the hand-derived backward pass, and Adam, each written out from its
definition so that a reader can check it line by line.

The paper trains nothing; this component and its every choice below are
readings of the learned-sketch specification:
  * input x = b_0 / ||b_0|| * sqrt(n) (the control RHS, normalised);
  * layers: h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2), o = W3 h2 + b3, with
    gelu the exact (erf) form; o (k n values) holds the k directions
    Z[:, j] = o[j n : (j + 1) n];
  * target: a Ritz pair set (S, D) of the control Hessian's A computed by the
    method (Nystrom, S orthonormal n x k, D >= 0);
  * loss: ||Z Z^T - S diag(D) S^T||_F^2 / ||D||_2^2 (Gram matching: invariant to
    rotations of Z, so only the spanned subspace and scale are learned),
    averaged over the batch;
  * He initialisation W ~ N(0, 2 / fan_in), zero biases; Adam (Kingma & Ba,
    2015) with bias correction.
Parameter vector layout (column-major matrices, one flat array):
  W1 (h x n), b1 (h), W2 (h x h), b2 (h), W3 (k n x h), b3 (k n).
"""
from __future__ import annotations

import math

import numpy as np


def dims_offsets(n: int, h: int, k: int) -> dict:
    """Offsets of W1, b1, W2, b2, W3, b3 in the flat parameter vector."""
    sizes = [("W1", h * n), ("b1", h), ("W2", h * h), ("b2", h), ("W3", k * n * h), ("b3", k * n)]
    off, out = 0, {}
    for name, s in sizes:
        out[name] = (off, s)
        off += s
    out["total"] = off
    return out


def unpack(theta: np.ndarray, n: int, h: int, k: int):
    o = dims_offsets(n, h, k)

    def get(name, shape):
        a, s = o[name]
        return theta[a:a + s].reshape(shape, order="F")

    return get("W1", (h, n)), get("b1", (h,)), get("W2", (h, h)), get("b2", (h,)), get("W3", (k * n, h)), \
        get("b3", (k * n,))


def he_init(normals: np.ndarray, n: int, h: int, k: int) -> np.ndarray:
    """Weights = standard normals * sqrt(2 / fan_in); biases 0.  `normals` holds
    one standard normal per parameter (biases' entries unused)."""
    o = dims_offsets(n, h, k)
    theta = np.zeros(o["total"])
    for name, fan_in in (("W1", n), ("W2", h), ("W3", h)):
        a, s = o[name]
        theta[a:a + s] = normals[a:a + s] * math.sqrt(2.0 / fan_in)
    return theta


def gelu(x):
    """x Phi(x), Phi the standard normal CDF (exact erf form)."""
    erf = np.vectorize(math.erf)
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    erf = np.vectorize(math.erf)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def normalise_input(b0: np.ndarray) -> np.ndarray:
    """x = b_0 / ||b_0|| sqrt(n), column by column."""
    b0 = np.atleast_2d(b0.T).T
    return b0 / np.linalg.norm(b0, axis=0) * math.sqrt(b0.shape[0])


def forward(theta, X, n, h, k):
    """X: n x B inputs.  Returns (Z list of n x k, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n, h, k)
    P1 = W1 @ X + b1[:, None]
    H1 = gelu(P1)
    P2 = W2 @ H1 + b2[:, None]
    H2 = gelu(P2)
    O = W3 @ H2 + b3[:, None]
    Z = [O[:, b].reshape((n, k), order="F") for b in range(X.shape[1])]
    return Z, (X, P1, H1, P2, H2, O)


def loss_definition(Z, S, D):
    """||Z Z^T - S diag(D) S^T||_F^2 / ||D||^2 for one sample, written out on
    the n x n matrices."""
    return np.linalg.norm(Z @ Z.T - (S * D) @ S.T) ** 2 / np.dot(D, D)


def loss_and_dZ(Z, S, D):
    """The same loss on k x k blocks (S orthonormal) and its gradient
    dL/dZ = 4 (Z (Z^T Z) - S diag(D) (S^T Z)) / ||D||^2."""
    G = Z.T @ Z
    M = S.T @ Z
    dd = np.dot(D, D)
    loss = (np.sum(G * G) - 2.0 * np.sum(D[:, None] * M * M) + dd) / dd
    dZ = 4.0 * (Z @ G - S @ (D[:, None] * M)) / dd
    return loss, dZ


def loss_and_grad(theta, X, Ss, Ds, n, h, k):
    """Mean loss over the batch and its gradient with respect to theta."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n, h, k)
    Z, (X, P1, H1, P2, H2, O) = forward(theta, X, n, h, k)
    B = X.shape[1]
    loss = 0.0
    dO = np.zeros_like(O)
    for b in range(B):
        lb, dZ = loss_and_dZ(Z[b], Ss[b], Ds[b])
        loss += lb / B
        dO[:, b] = dZ.reshape(-1, order="F") / B
    dW3 = dO @ H2.T
    db3 = dO.sum(axis=1)
    dH2 = W3.T @ dO
    dP2 = dH2 * gelu_grad(P2)
    dW2 = dP2 @ H1.T
    db2 = dP2.sum(axis=1)
    dH1 = W2.T @ dP2
    dP1 = dH1 * gelu_grad(P1)
    dW1 = dP1 @ X.T
    db1 = dP1.sum(axis=1)
    grad = np.concatenate([dW1.reshape(-1, order="F"), db1, dW2.reshape(-1, order="F"), db2,
                           dW3.reshape(-1, order="F"), db3])
    return loss, grad


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counted from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
