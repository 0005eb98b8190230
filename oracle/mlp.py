"""Reference (FP64, numpy) for the join-cardinality MLP.

TEST INFRASTRUCTURE ONLY: used by tests to check the GPU forward, backward
and BF16 inference kernels.  Network: x (8 features) scaled by 1/16 ->
dense 64 + ReLU -> dense 64 + ReLU -> dense 1; loss = mean squared error.
Parameters are one vector laid out W1[64][8] b1[64] W2[64][64] b2[64]
W3[1][64] b3[1].  Backward is written out by the chain rule:
dL/dyhat = 2 (yhat - y) / n; for a dense layer out = in W^T + b:
dW = dout^T in, db = sum_rows dout, din = dout W; ReLU passes the gradient
where its input was positive.
"""
import numpy as np

H, I = 64, 8
N_PARAMS = H * I + H + H * H + H + H + 1
IN_SCALE = 1.0 / 16.0


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * I].reshape(H, I); o += H * I
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H].reshape(1, H); o += H
    b3 = p[o:o + 1]; o += 1
    assert o == N_PARAMS
    return W1, b1, W2, b2, W3, b3


def forward(X, p):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(X, np.float64) * IN_SCALE
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0)
    yhat = (h2 @ W3.T + b3)[:, 0]
    return x, z1, h1, z2, h2, yhat


def loss(X, y, p):
    yhat = forward(X, p)[-1]
    return float(np.mean((yhat - np.asarray(y, np.float64)) ** 2))


def loss_and_grad(X, y, p):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x, z1, h1, z2, h2, yhat = forward(X, p)
    y = np.asarray(y, np.float64)
    n = len(y)
    dy = (2.0 * (yhat - y) / n)[:, None]          # n x 1
    dW3 = dy.T @ h2
    db3 = dy.sum(0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return float(np.mean((yhat - y) ** 2)), g


def bf16(a):
    """Round float32 values to BF16 (round to nearest even), kept as float32."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def forward_bf16(X, p):
    """Inference with BF16 weights and activations and FP32 accumulation."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(t, np.float32) for t in unpack(p)]
    x = bf16(np.asarray(X, np.float32) * np.float32(IN_SCALE))
    h1 = bf16(np.maximum(x @ bf16(W1).T + b1, 0))
    h2 = bf16(np.maximum(h1 @ bf16(W2).T + b2, 0))
    return (h2 @ bf16(W3).T + b3)[:, 0]
