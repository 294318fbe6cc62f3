"""Pins of the oracle's warm-start network (no GPU): central finite
differences of the exact-mode gradients and closed-form properties of the
span loss; the BF16 rounding helper against hand-checked values."""
import numpy as np

from oracle import mlp


def _problem(seed=0, B=3, in_dim=7, h=5, rows=6, k=2):
    rng = np.random.default_rng(seed)
    R = rows * k
    params = [rng.standard_normal((h, in_dim)) * 0.5, rng.standard_normal(h) * 0.1,
              rng.standard_normal((h, h)) * 0.5, rng.standard_normal(h) * 0.1,
              rng.standard_normal((R, h)) * 0.5, rng.standard_normal(R) * 0.1]
    X = rng.standard_normal((B, in_dim))
    mask = (rng.random((B, rows)) < 0.8).astype(np.uint8)
    mask[:, :k] = 1
    V = np.zeros((B, R))
    for s in range(B):
        m = mask[s].astype(bool)
        Q, _ = np.linalg.qr(rng.standard_normal((int(m.sum()), k)))
        Vs = np.zeros((rows, k))
        Vs[m] = Q
        V[s] = Vs.ravel()
    return params, X, V, mask, k


def test_gradients_match_central_differences():
    params, X, V, mask, k = _problem()
    L, g = mlp.loss_and_grad(params, X, V, mask, k, rounding=False)
    rng = np.random.default_rng(1)
    for i, P in enumerate(params):
        for _ in range(6):
            idx = tuple(rng.integers(0, d) for d in P.shape)
            e = 1e-6
            old = P[idx]
            P[idx] = old + e
            lp, _ = mlp.loss_and_grad(params, X, V, mask, k, rounding=False)
            P[idx] = old - e
            lm, _ = mlp.loss_and_grad(params, X, V, mask, k, rounding=False)
            P[idx] = old
            fd = (lp - lm) / (2 * e)
            assert abs(fd - g[i][idx]) <= 1e-6 * max(1.0, abs(fd)), (i, idx, fd, g[i][idx])


def test_span_loss_zero_at_span_and_rotation_invariant():
    rng = np.random.default_rng(2)
    rows, k, B = 9, 3, 2
    mask = np.ones((B, rows), np.uint8)
    mask[1, 7:] = 0
    V = np.zeros((B, rows * k))
    for s in range(B):
        m = mask[s].astype(bool)
        Vs = np.zeros((rows, k))
        Vs[m] = np.linalg.qr(rng.standard_normal((int(m.sum()), k)))[0]
        V[s] = Vs.ravel()
    # Y = V Q (any orthogonal Q) plus junk on the unmasked rows: loss 0, gradient 0
    Q = np.linalg.qr(rng.standard_normal((k, k)))[0]
    Y = np.stack([(V[s].reshape(rows, k) @ Q).ravel() for s in range(B)])
    Y[1].reshape(rows, k)[7:] = 5.0
    L, dY = mlp.span_loss(Y, V, mask, k)
    assert abs(L) < 1e-12 and np.abs(dY).max() < 1e-12
    # generic Y: positive, unchanged by Y -> Y Q
    Y = rng.standard_normal((B, rows * k))
    L1, _ = mlp.span_loss(Y, V, mask, k)
    L2, _ = mlp.span_loss(np.stack([(Y[s].reshape(rows, k) @ Q).ravel() for s in range(B)]), V, mask, k)
    assert L1 > 0 and abs(L1 - L2) < 1e-10 * L1


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.140625, 1e-40])
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 ties to 1 + 2^-6
    assert np.array_equal(mlp.bf16(x)[:5], [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -3.140625])
