"""CPU oracle of the per-node warm-start MLP.  TEST INFRASTRUCTURE ONLY.

The network maps 60 node features to a 12-DOF correction:
    h1 = relu(x W1 + b1)   (60 -> 128)
    h2 = relu(h1 W2 + b2)  (128 -> 128)
    y  = h2 W3 + b3        (128 -> 12)
and is trained on the squared error mean over samples of sum_k (y_k - t_k)^2.
With ``bf16=True`` every operand of a matrix product (x, h1, h2, the
weights, and in the backward pass the back-propagated errors) is rounded to
bfloat16 (round to nearest even) before the product, which is accumulated in
FP64 here; biases, losses and weight gradients stay FP64.  The gradients of
b1 and b2 are sums of the same rounded errors that enter the weight
products.  With bf16=False it
is a plain FP64 network (used for finite-difference checks).

Parameter vector layout (FP32 on the device, FP64 here), row-major:
W1[60][128], b1[128], W2[128][128], b2[128], W3[128][12], b3[12].
"""
import numpy as np

N_IN, N_H, N_OUT = 60, 128, 12
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H, N_OUT)),
          ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(a, bf16):
    return bf16_round(a) if bf16 else np.asarray(a, dtype=np.float64)


def forward(theta, x, bf16=False):
    p = unpack(theta)
    z1 = _r(x, bf16) @ _r(p["W1"], bf16) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = _r(h1, bf16) @ _r(p["W2"], bf16) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = _r(h2, bf16) @ _r(p["W3"], bf16) + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(theta, x, t, bf16=False):
    """Mean over samples of ||y - t||^2 and its gradient with respect to theta."""
    p = unpack(theta)
    y, (x, z1, h1, z2, h2) = forward(theta, x, bf16)
    n = x.shape[0]
    e = y - t
    loss = float(np.sum(e * e) / n)
    dy = 2.0 * e / n
    g = {}
    g["W3"] = _r(h2, bf16).T @ _r(dy, bf16)
    g["b3"] = dy.sum(axis=0)
    dh2 = (_r(dy, bf16) @ _r(p["W3"], bf16).T) * (z2 > 0)
    g["W2"] = _r(h1, bf16).T @ _r(dh2, bf16)
    g["b2"] = _r(dh2, bf16).sum(axis=0)
    dh1 = (_r(dh2, bf16) @ _r(p["W2"], bf16).T) * (z1 > 0)
    g["W1"] = _r(x, bf16).T @ _r(dh1, bf16)
    g["b1"] = _r(dh1, bf16).sum(axis=0)
    return loss, pack(g)


def init_params(seed=0):
    """He-uniform weights, zero biases, and a zero last layer (the untrained
    network predicts no correction)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        elif name == "W3":
            p[name] = np.zeros(shape)
        else:
            lim = np.sqrt(6.0 / shape[0])
            p[name] = rng.uniform(-lim, lim, size=shape)
    return pack(p)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
