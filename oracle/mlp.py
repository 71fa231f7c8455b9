"""Oracle for the RHS-cost MLP — TEST INFRASTRUCTURE ONLY.

16 -> 64 -> 64 -> 1 with ReLU, FP64.  Parameter layout as the library's:
W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3 (5313 values).
Loss: L = mean_s (y_s - t_s)^2.  Adam with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8 and bias correction (Kingma & Ba, 2015).
"""
import numpy as np

NIN, NH = 16, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", ())]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape)) if shape else 1
        out[name] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shape) if shape else float(w[o])
        o += n
    return out


def pack(p):
    return np.concatenate([np.atleast_1d(np.asarray(p[name], dtype=np.float64)).ravel() for name, _ in SIZES])


def forward(w, X):
    p = unpack(w)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (X, a1, h1, a2, h2)


def loss_and_grad(w, X, t):
    p = unpack(w)
    y, (X, a1, h1, a2, h2) = forward(w, X)
    n = X.shape[0]
    e = y - t
    L = float(np.mean(e * e))
    dy = 2.0 * e / n
    g = {"W3": h2.T @ dy, "b3": float(dy.sum())}
    dh2 = np.outer(dy, p["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return L, pack(g)


def adam_step(w, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
