"""FP64 reference of the learned damping / depth network (test infrastructure).

TEST INFRASTRUCTURE: the oracle the HIP MLP kernels are checked against;
only tests and the benchmark's baseline leg import it.

Network: 16 inputs -> 64 (ReLU) -> 64 (ReLU) -> 2. Output heads:
damping d = 0.9 * sigmoid(o0) in [0, 0.9], log-depth correction
delta = C_DELTA * tanh(o1). Loss: per-sample weighted squared error on
both heads, averaged over the samples:
    L = (1/N) sum_i [ m0_i (d_i - d*_i)^2 + m1_i (delta_i - delta*_i)^2 ].
Parameter vector layout (5378 values): W1[64][16], b1[64], W2[64][64],
b2[64], W3[2][64], b3[2].
"""
import numpy as np
from scipy.special import expit

N_IN, N_H, N_OUT = 16, 64, 2
C_DELTA = 2.5
D_MAX = 0.9
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed=0):
    """He-uniform weights, zero biases (a plain, reproducible start)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def forward(theta, x):
    """Heads (d, delta) and the intermediate activations."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    d = D_MAX * expit(o[:, 0])
    delta = C_DELTA * np.tanh(o[:, 1])
    return np.stack([d, delta], axis=1), dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, o=o)


def loss(theta, x, y, m):
    heads, _ = forward(theta, x)
    r = heads - np.asarray(y, dtype=np.float64)
    return float(np.mean(np.sum(np.asarray(m, dtype=np.float64) * r * r, axis=1)))


def grad(theta, x, y, m):
    """Analytic gradient of `loss` by back-propagation (chain rule written
    out layer by layer)."""
    p = unpack(theta)
    heads, a = forward(theta, x)
    n = heads.shape[0]
    m = np.asarray(m, dtype=np.float64)
    r = heads - np.asarray(y, dtype=np.float64)
    dheads = 2.0 * m * r / n
    sig = expit(a["o"][:, 0])
    th = np.tanh(a["o"][:, 1])
    do = np.stack([dheads[:, 0] * D_MAX * sig * (1.0 - sig),
                   dheads[:, 1] * C_DELTA * (1.0 - th * th)], axis=1)
    g = {}
    g["W3"] = do.T @ a["h2"]
    g["b3"] = do.sum(0)
    dh2 = do @ p["W3"]
    dz2 = dh2 * (a["z2"] > 0)
    g["W2"] = dz2.T @ a["h1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (a["z1"] > 0)
    g["W1"] = dz1.T @ a["x"]
    g["b1"] = dz1.sum(0)
    return pack(g)


def bf16_round(v):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    f = np.asarray(v, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def to_bf16_bits(v):
    f = np.asarray(v, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def forward_bf16(theta, x):
    """Heads of the network evaluated the way the BF16 inference stores its
    operands: inputs, weights, biases and both hidden activations rounded to
    bfloat16 (nearest even), all arithmetic in FP64."""
    p = unpack(bf16_round(theta))
    x = bf16_round(x)
    h1 = bf16_round(np.maximum(x @ p["W1"].T + p["b1"], 0.0))
    h2 = bf16_round(np.maximum(h1 @ p["W2"].T + p["b2"], 0.0))
    o = h2 @ p["W3"].T + p["b3"]
    return np.stack([D_MAX * expit(o[:, 0]), C_DELTA * np.tanh(o[:, 1])], axis=1)


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction (Kingma and Ba, Algorithm 1)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
