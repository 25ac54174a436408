"""Error bound of the BF16 network against the plain FP64 network.

The inference kernel rounds its inputs, weights, biases and both hidden
activations to bfloat16 (round to nearest even, 8 significant bits: relative
error at most u = 2^-8, the FP64 -> FP32 step before it included), forms
BF16 x BF16 products exactly in FP32 and sums them in FP32. To first order
the error of an output o is sum_s (d o / d v_s) delta_s over the rounding
sites s, with |delta_s| <= u |v_s|. Taking the site errors as independent
with mean zero (the probabilistic model of rounding-error analysis; Higham
and Mary, SIAM J. Sci. Comput. 2019), Hoeffding's inequality gives
|error| <= lam u sqrt(sum_s (d o / d v_s)^2 v_s^2) with probability at least
1 - 2 exp(-lam^2 / 2) per output (lam = 7: 5e-11). To that are added, as
worst cases: units whose pre-activation lies within reach of zero (a ReLU
that may switch, which the linear model misses), the FP32 sums (gamma_n =
n 2^-24 / (1 - n 2^-24) times the sum of magnitudes, doubled for the matrix
cores' unspecified order) and 5% for second-order terms. The heads d = 0.9
sigmoid(o0) and delta = 2.5 tanh(o1) take the largest slope over the
interval o +- error (mean value theorem); 1e-6 covers FP32 exp and tanh.
"""
import numpy as np
from scipy.special import expit

from oracle import mlp as omlp

U_BF16 = 2.0 ** -8 * (1 + 2.0 ** -15)


def _gamma(n):
    return 2 * n * 2.0 ** -24 / (1 - n * 2.0 ** -24)


def forward_error_bound(theta, x, lam=7.0, u=U_BF16):
    """(n, 2) bound on |heads(BF16 network) - heads(FP64 network)| per row."""
    x = np.asarray(x, dtype=np.float64)
    p = omlp.unpack(theta)
    _, a = omlp.forward(theta, x)
    W1, W2, W3, b1, b2, b3 = p["W1"], p["W2"], p["W3"], p["b1"], p["b2"], p["b3"]
    h1, h2, z1, z2, o = a["h1"], a["h2"], a["z1"], a["z2"], a["o"]
    xw1 = (x * x) @ (W1 * W1).T                 # sum_i (x_i W1_ji)^2
    hw2 = (h1 * h1) @ (W2 * W2).T               # sum_j (h1_j W2_kj)^2
    m1, m2 = (z1 > 0).astype(float), (z2 > 0).astype(float)
    # spread of the pre-activations (sites: x, W1, b1 for z1; all upstream for z2)
    s_z1 = u * np.sqrt(2 * xw1 + b1 ** 2)
    G1p = W2[None] * m1[:, None, :]             # d z2_k / d z1_j
    Gxp = G1p @ W1                              # d z2_k / d x_i
    s_z2 = u * np.sqrt(np.einsum("rki,ri->rk", Gxp ** 2, x ** 2)
                       + np.einsum("rkj,rj->rk", G1p ** 2, xw1 + b1 ** 2) + 2 * hw2 + b2 ** 2)
    # spread of the outputs
    G2 = W3[None] * m2[:, None, :]              # d o / d z2
    Gh1 = G2 @ W2                               # d o / d h1
    G1 = Gh1 * m1[:, None, :]                   # d o / d z1
    Gx = G1 @ W1                                # d o / d x
    s_o = u * np.sqrt(np.einsum("roi,ri->ro", Gx ** 2, x ** 2)
                      + np.einsum("roj,rj->ro", G1 ** 2, xw1 + b1 ** 2)
                      + np.einsum("roj,rj->ro", Gh1 ** 2, h1 ** 2)
                      + np.einsum("rok,rk->ro", G2 ** 2, hw2 + b2 ** 2)
                      + 2 * (h2 * h2) @ (W3 * W3).T + b3 ** 2)
    # ReLUs within reach of zero
    k1 = np.where(np.abs(z1) <= lam * s_z1, lam * s_z1, 0.0)
    k2 = np.where(np.abs(z2) <= lam * s_z2, lam * s_z2, 0.0)
    kink = np.einsum("roj,rj->ro", np.abs(Gh1), k1) + k2 @ np.abs(W3).T
    # FP32 sums
    a1 = _gamma(17) * (np.abs(x) @ np.abs(W1).T + np.abs(b1)) * (1 + u) ** 2
    a2 = _gamma(65) * ((h1 + lam * s_z1) @ np.abs(W2).T + np.abs(b2)) * (1 + u) ** 2
    a3 = _gamma(65) * ((h2 + lam * s_z2) @ np.abs(W3).T + np.abs(b3)) * (1 + u) ** 2
    acc = np.einsum("roj,rj->ro", np.abs(Gh1), a1) + np.einsum("rok,rk->ro", np.abs(G2), a2) + a3
    e = 1.05 * (lam * s_o + kink + acc)
    # heads: largest slope over o +- e
    r0 = np.maximum(np.abs(o[:, 0]) - e[:, 0], 0.0)
    r1 = np.maximum(np.abs(o[:, 1]) - e[:, 1], 0.0)
    slope_d = omlp.D_MAX * expit(r0) * (1 - expit(r0))
    slope_t = omlp.C_DELTA * (1 - np.tanh(r1) ** 2)
    return np.stack([slope_d * e[:, 0] + 1e-6, slope_t * e[:, 1] + 1e-6], axis=1)
