"""FP64 reference of the learned scheduler's network (test infrastructure only).

3-layer perceptron x[F] -> 64 -> 64 -> 3 with ReLU, parameters flattened as
W1[F][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3] (row-major, [in][out]).
Loss of a minibatch of B samples: (1/B) sum_b sum_o w[b,o] (yhat[b,o] - y[b,o])^2.
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Gradients are plain reverse-mode differentiation of the expressions above;
they are pinned against central finite differences in the test-suite.
"""

from __future__ import annotations

import numpy as np

F, H, O = 14, 64, 3
P = F * H + H + H * H + H + H * O + O


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    i = 0
    W1 = p[i:i + F * H].reshape(F, H); i += F * H
    b1 = p[i:i + H]; i += H
    W2 = p[i:i + H * H].reshape(H, H); i += H * H
    b2 = p[i:i + H]; i += H
    W3 = p[i:i + H * O].reshape(H, O); i += H * O
    b3 = p[i:i + O]; i += O
    return W1, b1, W2, b2, W3, b3


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3


def loss(p, X, Y, Wt):
    d = forward(p, X) - Y
    return float(np.sum(Wt * d * d) / X.shape[0])


def grad(p, X, Y, Wt):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    B = X.shape[0]
    a1 = X @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    out = h2 @ W3 + b3
    dout = 2.0 * Wt * (out - Y) / B
    gW3 = h2.T @ dout
    gb3 = dout.sum(axis=0)
    d2 = (dout @ W3.T) * (a2 > 0)
    gW2 = h1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (a1 > 0)
    gW1 = X.T @ d1
    gb1 = d1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
