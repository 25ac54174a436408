"""Pins of the FP64 oracle MLP: analytic gradient vs central finite
differences on every parameter, head ranges, BF16 rounding vs the format's
definition."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, mlp.N_IN))
    y = np.stack([rng.uniform(0, 0.9, n), rng.normal(0, 1, n)], axis=1)
    m = rng.uniform(0.2, 1.0, (n, 2))
    return x, y, m


def test_gradient_matches_central_differences_on_every_parameter():
    theta = mlp.init_params(1) + np.random.default_rng(2).normal(0, 0.05, mlp.N_PARAMS)
    x, y, m = _data(3)
    g = mlp.grad(theta, x, y, m)
    eps = 1e-6
    fd = np.zeros_like(theta)
    for i in range(mlp.N_PARAMS):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd[i] = (mlp.loss(tp, x, y, m) - mlp.loss(tm, x, y, m)) / (2 * eps)
    scale = np.abs(fd).max()
    assert np.abs(g - fd).max() < 1e-6 * scale
    # every tensor has a non-trivial gradient (no dead block in the test)
    o = 0
    for name, shp in mlp.SHAPES:
        n = int(np.prod(shp))
        assert np.abs(g[o:o + n]).max() > 0, name
        o += n


def test_heads_are_in_range_and_zero_weight_samples_do_not_count():
    theta = mlp.init_params(4)
    x, y, m = _data(5)
    heads, _ = mlp.forward(theta * 50, x)
    assert np.all(heads[:, 0] >= 0) and np.all(heads[:, 0] <= mlp.D_MAX)
    assert np.all(np.abs(heads[:, 1]) <= mlp.C_DELTA)
    m2 = m.copy()
    m2[:10] = 0.0
    y2 = y.copy()
    y2[:10] += 100.0
    assert abs(mlp.loss(theta, x, y, m2) - mlp.loss(theta, x, y2, m2)) < 1e-12


def test_bf16_rounding_definition():
    # values exactly representable stay; halfway cases round to even
    assert mlp.bf16_round(1.0) == 1.0
    one_plus_half_ulp = np.float32(1.0 + 2.0 ** -8)          # halfway between 1 and 1+2^-7
    assert mlp.bf16_round(one_plus_half_ulp) == 1.0          # ties to even (mantissa 0)
    v = np.float32(1.0 + 3 * 2.0 ** -8)                      # halfway, odd neighbour below
    assert mlp.bf16_round(v) == 1.0 + 2 * 2.0 ** -7
    bits = mlp.to_bf16_bits([1.0, -2.0, 0.15625])
    assert list(bits) == [0x3F80, 0xC000, 0x3E20]
    assert np.allclose(mlp.from_bf16_bits(bits), [1.0, -2.0, 0.15625])


def test_bf16_forward_reduces_to_fp64_forward_on_representable_values():
    # parameters in {-1/4, 0, 1/4} and integer inputs keep every activation a
    # multiple of 1/16 below 16, which bfloat16 holds exactly (8 significant
    # bits): the emulated forward must then equal the plain one bit for bit
    rng = np.random.default_rng(7)
    theta = rng.integers(-1, 2, mlp.N_PARAMS) / 4.0
    x = rng.integers(-2, 3, (30, mlp.N_IN)).astype(float)
    _, a = mlp.forward(theta, x)
    for h in (a["h1"], a["h2"]):
        assert np.abs(h).max() < 16 and np.all((h * 16) % 1 == 0)
    assert np.array_equal(mlp.forward_bf16(theta, x), mlp.forward(theta, x)[0])
    # generic values: the emulation differs from FP64 only by rounding
    theta = mlp.init_params(3)
    x = rng.normal(size=(50, mlp.N_IN))
    diff = np.abs(mlp.forward_bf16(theta, x) - mlp.forward(theta, x)[0])
    assert 0 < diff.max() < 0.05


@pytest.mark.parametrize("where", ["input", "weight", "hidden1", "hidden2"])
def test_bf16_forward_rounds_at_each_storage_point(where):
    """Inputs, weights and both hidden activations are stored in bfloat16
    (nearest even) before they are read: a value v = 1 + 2^-9 + 2^-12, which
    bfloat16 cannot hold, placed at one storage point of a one-unit path
    reads as 1 there. Where a later rounding would hide it, the path doubles
    and shifts the value (2 v - 1 rounds up to 1 + 2^-7, 2 round(v) - 1 is 1)."""
    v = 1.0 + 2.0 ** -9 + 2.0 ** -12
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    x = np.zeros((1, mlp.N_IN))
    x[0, 0] = 1.0
    p["W1"][0, 0] = p["W2"][0, 0] = p["W3"][0, 0] = 1.0
    if where == "input":            # h1 = 2 x - 1
        x[0, 0] = v
        p["W1"][0, 0], p["b1"][0] = 2.0, -1.0
        o_fp64 = 2.0 * v - 1.0
    elif where == "weight":         # o = W3 h2
        p["W3"][0, 0] = v
        o_fp64 = v
    elif where == "hidden1":        # h1 = v, h2 = 2 h1 - 1
        p["b1"][0] = v - 1.0
        p["W2"][0, 0], p["b2"][0] = 2.0, -1.0
        o_fp64 = 2.0 * v - 1.0
    else:                           # h2 = v, o = h2
        p["b2"][0] = v - 1.0
        o_fp64 = v
    theta = mlp.pack(p)
    d_bf16 = mlp.forward_bf16(theta, x)[0, 0]
    d_fp64 = mlp.forward(theta, x)[0][0, 0]
    assert d_bf16 == mlp.D_MAX / (1.0 + np.exp(-1.0))
    assert abs(d_fp64 - mlp.D_MAX / (1.0 + np.exp(-o_fp64))) < 1e-15
    assert d_bf16 != d_fp64


def test_adam_first_step_is_signed_learning_rate():
    # at step 1 the bias-corrected moments are g and g^2: the update is
    # -lr * g / (|g| + eps), i.e. -lr * sign(g) for |g| >> eps
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert th[3] == 0.0
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps the step at lr (bias correction exact)
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for k in range(1, 6):
        th, m, v = mlp.adam_step(th, m, v, np.full(4, 2.0), k, 0.1)
    assert np.allclose(th, -0.5, rtol=1e-6)


def test_bf16_error_bound_covers_the_storage_rounding_and_is_not_vacuous():
    """The bound the GPU inference is held to (`bf16_bound`): the emulated
    BF16 forward (a realisation of the same roundings, in FP64) stays inside
    it on every row, and a bound built for a rounding 8x finer fails, so it
    is not loose by more than that factor."""
    from tests.bf16_bound import U_BF16, forward_error_bound
    rng = np.random.default_rng(21)
    for seed in (3, 4):
        theta = mlp.init_params(seed)
        p = mlp.unpack(theta)
        for b in ("b1", "b2", "b3"):
            p[b][:] = rng.normal(0, 0.3, p[b].shape)
        theta = mlp.pack(p).astype(np.float32).astype(np.float64)
        x = rng.normal(0, 1.5, (600, mlp.N_IN)).astype(np.float32).astype(np.float64)
        err = np.abs(mlp.forward_bf16(theta, x) - mlp.forward(theta, x)[0])
        assert np.all(err <= forward_error_bound(theta, x))
        assert np.any(err > forward_error_bound(theta, x, u=U_BF16 / 8))
