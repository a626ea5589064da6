"""FP64 reference of the learned preconditioner correction network.

Test infrastructure only: the product path never imports this module.

The network is a per-row multilayer perceptron with two hidden layers of
width H (ReLU) and a linear output of size O:
    h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2), y = h2 W3^T + b3.
The training loss over a batch of rows is the weighted squared error
    L = sum_i w_i sum_o (y_io - t_io)^2 .
With w_i = 1 / (G * sum_{k in g(i)} |t_k|^2) (group_weights) it is the mean
over the G right-hand sides in the batch of the relative squared error of
the correction.  Gradients are written out by the chain rule; tests compare
them with central finite differences and with the device kernels (which use
the same bf16-rounded weights and inputs, upcast).
"""
import numpy as np


def init(F, H=256, O=2, seed=0):
    """He-normal hidden layers, a small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, F)) * np.sqrt(2.0 / F)
    W2 = rng.standard_normal((H, H)) * np.sqrt(2.0 / H)
    W3 = rng.standard_normal((O, H)) * np.sqrt(1.0 / H) * 0.1
    return dict(W1=W1, b1=np.zeros(H), W2=W2, b2=np.zeros(H), W3=W3, b3=np.zeros(O))


def forward(p, X):
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (a1, h1, a2, h2)


def group_weights(T, group):
    """w_i = 1 / (G * sum over row i's group of |t|^2); group[i] in 0..G-1."""
    G = int(group.max()) + 1
    den = np.bincount(group, weights=np.sum(T ** 2, axis=1), minlength=G)
    den = np.maximum(den, 1e-300)
    return (1.0 / (G * den))[group]


def loss_and_grad(p, X, T, w):
    """Loss, parameter gradients (same keys as p) and the output y."""
    y, (a1, h1, a2, h2) = forward(p, X)
    d = y - T
    L = float(np.sum(w[:, None] * d * d))
    dy = 2.0 * w[:, None] * d
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = (dy @ p["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(axis=0)
    return L, g, y


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) of every array in p, in
    place; m, v are the moment estimates, t the 1-based step."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
