"""CPU FP64 reference of the learned-sizing MLP (TEST INFRASTRUCTURE ONLY).

Plain numpy forward/backward of the network the GPU library trains: 22 -> H -> H -> K with ReLU
hidden layers, sigmoid outputs and mean-squared-error loss.  The flat parameter layout is
W1[H][22], b1[H], W2[H][H], b2[H], W3[K][H], b3[K].  Gradients here are written from the chain
rule directly, not from the GPU code.
"""
import numpy as np


def unpack(flat, H, K, F=22):
    flat = np.asarray(flat, dtype=np.float64)
    o = 0
    shapes = [(H, F), (H,), (H, H), (H,), (K, H), (K,)]
    out = []
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(flat[o:o + n].reshape(sh))
        o += n
    assert o == flat.size
    return out


def loss_and_grad(flat, X, Y, H, K):
    W1, b1, W2, b2, W3, b3 = unpack(flat, H, K)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    n = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3.T + b3
    yh = 1.0 / (1.0 + np.exp(-z3))
    diff = yh - Y
    loss = np.mean(diff ** 2)
    d3 = 2.0 / (n * K) * diff * yh * (1.0 - yh)
    gW3 = d3.T @ h2
    gb3 = d3.sum(0)
    d2 = (d3 @ W3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g, yh
