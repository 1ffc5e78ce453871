"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain numpy: forward pass, the masked loss and its gradient by the chain rule,
written from the definitions (a 3-layer perceptron with GELU activations in
their tanh form, 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))),
BCE-with-logits on 32 basis indicators, squared error on 32 fractions, both
masked by the input's slot mask and averaged over rows).  Used to check the
GPU's BF16 matrix-core forward and backward passes, and its optimiser step
(AdamW: Kingma and Ba's bias-corrected moments with Loshchilov and Hutter's
decoupled weight decay).
"""
import math

import numpy as np

IN, HID, OUT, SLOTS = 128, 128, 64, 32
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, OUT)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    t = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def forward(theta, X):
    p = unpack(theta)
    X = np.asarray(X, np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["W3"] + p["b3"]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, T, wf=1.0):
    p = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    T = np.asarray(T, np.float64)
    rows = X.shape[0]
    mask = X[:, 2 * SLOTS:3 * SLOTS]
    z, ind = y[:, :SLOTS], T[:, :SLOTS]
    pf, f = y[:, SLOTS:], T[:, SLOTS:]
    softplus = np.logaddexp(0.0, z)
    loss = float((mask * (softplus - ind * z + wf * (pf - f) ** 2)).sum() / rows)
    dy = np.zeros_like(y)
    dy[:, :SLOTS] = mask * (1.0 / (1.0 + np.exp(-z)) - ind) / rows
    dy[:, SLOTS:] = mask * wf * 2.0 * (pf - f) / rows
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dz2 = (dy @ p["W3"].T) * gelu_grad(z2)
    g["W2"], g["b2"] = h1.T @ dz2, dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(z1)
    g["W1"], g["b1"] = X.T @ dz1, dz1.sum(0)
    return loss, pack(g)


def init_params(seed=0):
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        d[name] = rng.normal(0.0, math.sqrt(2.0 / shape[0]), shape) if len(shape) == 2 else np.zeros(shape)
    return pack(d)


def adamw_step(w, g, m, v, t, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """Step t (from 1) of AdamW: the moments m <- b1 m + (1 - b1) g and
    v <- b2 v + (1 - b2) g^2, their bias corrections m / (1 - b1^t) and
    v / (1 - b2^t), and w <- w - lr (m_hat / (sqrt(v_hat) + eps) + wd w), the
    weight decay applied to the parameter directly rather than through the
    gradient.  Returns the new (w, m, v)."""
    w, g, m, v = (np.asarray(a, np.float64) for a in (w, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * (mh / (np.sqrt(vh) + eps) + wd * w), m, v
