"""Oracle (test infrastructure): forward and backward of the learned
warm-start network and its span loss, in numpy.

The paper computes the GenEO eigenvectors from scratch in every subdomain
(Section 3.2); the learned warm start only changes where the eigensolver
starts, not what it converges to, so nothing here is pinned by the paper.
Parity unpinned against the paper: the gradients are pinned by central
finite differences (exact mode) and the loss by its closed-form properties
(zero exactly when span Y = span V for orthonormal V; invariant under
Y -> Y Q for orthogonal Q).

Network: Z1 = X W1^T + b1, H1 = relu(Z1), Z2 = H1 W2^T + b2, H2 = relu(Z2),
Y = H2 W3^T + b3; each sample's output row is reshaped to rows x k.
Loss per sample, over the masked rows: ||Y^T Y||_F^2 - 2 ||V^T Y||_F^2 + k;
the batch loss is the mean.

rounding=True reproduces the library's storage precision: inputs, weights,
hidden activations and the back-propagated signals that enter products are
rounded to BF16 (round to nearest even) and the products are accumulated in
float64 here (FP32 in the library); biases and their gradients stay exact.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def split_params(p, in_dim, hidden, R):
    """Flat parameter vector -> W1 [h x in], b1, W2 [h x h], b2, W3 [R x h], b3."""
    sizes = [hidden * in_dim, hidden, hidden * hidden, hidden, R * hidden, R]
    shapes = [(hidden, in_dim), (hidden,), (hidden, hidden), (hidden,), (R, hidden), (R,)]
    out, o = [], 0
    for s, sh in zip(sizes, shapes):
        out.append(np.asarray(p[o:o + s], dtype=np.float64).reshape(sh))
        o += s
    return out


def forward(params, X, rounding=True):
    r = bf16 if rounding else _id
    W1, b1, W2, b2, W3, b3 = params
    Xr = r(X)
    Z1 = Xr @ r(W1).T + b1
    H1 = r(np.maximum(Z1, 0.0))
    Z2 = H1 @ r(W2).T + b2
    H2 = r(np.maximum(Z2, 0.0))
    Y = H2 @ r(W3).T + b3
    return Y, (Xr, Z1, H1, Z2, H2)


def span_loss(Y, V, mask, k):
    """Mean over the batch of ||Ym^T Ym||^2 - 2 ||V^T Ym||^2 + k and dL/dY."""
    B = Y.shape[0]
    rows = mask.shape[1]
    L = 0.0
    dY = np.zeros_like(Y, dtype=np.float64)
    for s in range(B):
        m = mask[s].astype(bool)
        Ys = Y[s].reshape(rows, k) * m[:, None]
        Vs = V[s].reshape(rows, k) * m[:, None]
        G1 = Ys.T @ Ys
        G2 = Vs.T @ Ys
        L += np.sum(G1 * G1) - 2.0 * np.sum(G2 * G2) + k
        dY[s] = ((4.0 * (Ys @ G1) - 4.0 * (Vs @ G2)) * m[:, None]).ravel() / B
    return L / B, dY


def loss_and_grad(params, X, V, mask, k, rounding=True):
    """Loss and gradients [dW1, db1, dW2, db2, dW3, db3]."""
    r = bf16 if rounding else _id
    W1, b1, W2, b2, W3, b3 = params
    Y, (Xr, Z1, H1, Z2, H2) = forward(params, X, rounding)
    L, dY = span_loss(Y, V, mask, k)
    db3 = dY.sum(axis=0)
    dYr = r(dY)
    dW3 = dYr.T @ H2
    dH2 = dYr @ r(W3)
    dZ2 = dH2 * (Z2 > 0)
    db2 = dZ2.sum(axis=0)
    dZ2r = r(dZ2)
    dW2 = dZ2r.T @ H1
    dH1 = dZ2r @ r(W2)
    dZ1 = dH1 * (Z1 > 0)
    db1 = dZ1.sum(axis=0)
    dW1 = r(dZ1).T @ Xr
    return L, [dW1, db1, dW2, db2, dW3, db3]
