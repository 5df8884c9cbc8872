"""FP64 NumPy oracle of the chi^2 surrogate MLP and of Adam.

TEST INFRASTRUCTURE ONLY.

Network: 12 -> 256 -> 256 -> 256 -> 1, SiLU(z) = z sigmoid(z) on the hidden
layers, linear output.  Parameters packed as [W1 (256x12), b1, W2 (256x256),
b2, W3 (256x256), b3, W4 (1x256), b4], weights row-major [out][in].
Backpropagation is the chain rule written out layer by layer; Adam follows
Kingma & Ba (2015), Algorithm 1, with bias-corrected moments.
"""
import numpy as np

IN, HID = 12, 256
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (1, HID)), ("b4", (1,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, s in SHAPES:
        k = int(np.prod(s))
        out[name] = p[o:o + k].reshape(s)
        o += k
    return out


def pack(d):
    return np.concatenate([d[name].reshape(-1) for name, _ in SHAPES])


def init(seed=0):
    """He-style uniform initialisation (fan-in scaling)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, s in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / s[1]) * (0.5 if name == "W4" else 1.0)
            d[name] = rng.uniform(-lim, lim, size=s)
        else:
            d[name] = np.zeros(s)
    return pack(d)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(p, x):
    """Returns y [B] and the cache (pre-activations and activations)."""
    P = unpack(p)
    z1 = x @ P["W1"].T + P["b1"]
    a1 = z1 * _sig(z1)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = z2 * _sig(z2)
    z3 = a2 @ P["W3"].T + P["b3"]
    a3 = z3 * _sig(z3)
    y = (a3 @ P["W4"].T + P["b4"])[:, 0]
    return y, (x, z1, a1, z2, a2, z3, a3)


def _dsilu(z):
    s = _sig(z)
    return s * (1 + z * (1 - s))


def backward(p, cache, dy):
    """Gradient of sum_b dy[b] y[b] with respect to every parameter."""
    P = unpack(p)
    x, z1, a1, z2, a2, z3, a3 = cache
    g = {}
    g["W4"] = dy[None, :] @ a3
    g["b4"] = np.array([dy.sum()])
    d3 = (dy[:, None] @ P["W4"]) * _dsilu(z3)
    g["W3"] = d3.T @ a2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ P["W3"]) * _dsilu(z2)
    g["W2"] = d2.T @ a1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ P["W2"]) * _dsilu(z1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return pack(g)


def mse_grad(y, t):
    """L = mean (y - t)^2 and dL/dy."""
    r = y - t
    return float(np.mean(r * r)), 2.0 * r / y.size


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
