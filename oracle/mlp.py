"""FP64 reference of the learned initialiser's network — TEST INFRASTRUCTURE ONLY.

A 3 -> 64 -> 64 -> 3 multilayer perceptron with tanh hidden units, loss = mean
over rows of |y - p|^2, and its exact gradient by the chain rule (textbook
backpropagation), written plainly in numpy float64.  Parameter layout:
W1[3][64] | b1[64] | W2[64][64] | b2[64] | W3[64][3] | b3[3]  (4611 values).
"""
import numpy as np

SIZES = [("W1", (3, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 3)),
         ("b3", (3,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(theta, x):
    P = unpack(theta)
    h1 = np.tanh(x @ P["W1"] + P["b1"])
    h2 = np.tanh(h1 @ P["W2"] + P["b2"])
    return h2 @ P["W3"] + P["b3"]


def loss(theta, x, p):
    e = forward(theta, x) - p
    return float(np.sum(e * e) / len(x))


def loss_and_grad(theta, x, p):
    P = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    B = len(x)
    h1 = np.tanh(x @ P["W1"] + P["b1"])
    h2 = np.tanh(h1 @ P["W2"] + P["b2"])
    y = h2 @ P["W3"] + P["b3"]
    e = y - p
    L = float(np.sum(e * e) / B)
    dy = 2.0 * e / B
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dz2 = (dy @ P["W3"].T) * (1.0 - h2 * h2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"].T) * (1.0 - h1 * h1)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(0)
    return L, pack(g)
