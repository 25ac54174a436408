"""Pins of the oracle's pairwise difference factors (heterogeneous factors,
the outlook of Sections 9-10) against what the mathematics fixes: GBP on a
tree is exact in means and covariances, loopy GBP converges to the exact
means (Section 3.2), here against a dense solve of the same quadratic
objective assembled term by term from the factors' definition (a factor
between a and b contributes (x_b - x_a - z)^T P (x_b - x_a - z) / 2)."""
import numpy as np
import pytest

import synth
from tests import dense_ref

FROZEN = dict(beta=1e30, relin_interval=10 ** 9, anneal=False)


def keyframes_only(nk, seed=3, anchor=None):
    """nk anchored keyframes, no landmarks and no measurements."""
    rng = np.random.default_rng(seed)
    kf = np.concatenate([rng.normal(0, 0.2, (nk, 3)), rng.normal(0, 1.0, (nk, 3))], 1)
    return synth.BAProblem("kf_only", synth.Camera(), kf, np.zeros((0, 3)), kf.copy(), np.zeros((0, 3)),
                           np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 2)), np.zeros((0, 2)),
                           np.zeros(0, bool), np.full(nk, 3.0) if anchor is None else anchor)


def add_pairs_dense(H, g, offset, D, a, b, z, prec):
    """The pairwise terms of the objective, by definition."""
    for i in range(len(a)):
        ia = offset + D * a[i] + np.arange(D)
        ib = offset + D * b[i] + np.arange(D)
        P = np.diag(prec[i])
        H[np.ix_(ia, ia)] += P
        H[np.ix_(ib, ib)] += P
        H[np.ix_(ia, ib)] -= P
        H[np.ix_(ib, ia)] -= P
        g[ia] -= P @ z[i]
        g[ib] += P @ z[i]


@pytest.mark.parametrize("damping", [0.0, 0.4])
def test_pose_chain_is_exact_in_means_and_covariances(oracle_mod, damping):
    nk = 5
    rng = np.random.default_rng(7)
    p = keyframes_only(nk)
    a, b = np.arange(nk - 1), np.arange(1, nk)
    z = rng.normal(0, 0.3, (nk - 1, 6))
    prec = rng.uniform(0.5, 5.0, (nk - 1, 6))
    o = oracle_mod.Oracle(p, **FROZEN)
    o.add_pairs(0, a, b, z, prec)
    H, g = dense_ref.assemble(o)
    add_pairs_dense(H, g, 0, 6, a, b, z, prec)
    mu = np.linalg.solve(H, g)
    cov = np.linalg.inv(H)
    o.iterate(300 if damping else 3 * nk, damping=damping)
    bel = o.beliefs()
    for k in range(nk):
        s = slice(6 * k, 6 * k + 6)
        assert np.abs(bel["kf_mu"][k] - mu[s]).max() < 1e-10 * max(1.0, np.abs(mu[s]).max())
        ck = np.linalg.inv(bel["kf_lam"][k])
        assert np.abs(ck - cov[s, s]).max() < 1e-9 * np.abs(cov[s, s]).max()
    # the pairs moved the means away from the anchors (the test can fail)
    assert np.abs(bel["kf_mu"] - p.kf_init).max() > 1e-2


@pytest.mark.parametrize("damping", [0.0, 0.4])
def test_loopy_pairs_with_measurements_reach_the_dense_means(oracle_mod, damping):
    """Keyframe ring and landmark pairs on top of the measurement factors of
    the circle problem, linearisation frozen: the means converge to the
    dense solve of the whole objective."""
    p = synth.make_config0(seed=0)
    rng = np.random.default_rng(11)
    nk, nl = p.n_keyframes, p.n_landmarks
    ka, kb = np.arange(nk), (np.arange(nk) + 1) % nk
    kz = p.kf_true[kb] - p.kf_true[ka] + rng.normal(0, 0.01, (nk, 6))
    kp = rng.uniform(50, 500, (nk, 6))
    la = rng.choice(nl, 20, replace=False)
    lb = (la + 1 + rng.integers(0, nl - 1, 20)) % nl
    lz = p.lm_true[lb] - p.lm_true[la] + rng.normal(0, 0.02, (20, 3))
    lp = rng.uniform(5, 50, (20, 3))
    o = oracle_mod.Oracle(p, **FROZEN)
    o.add_pairs(0, ka, kb, kz, kp)
    o.add_pairs(1, la, lb, lz, lp)
    H, g = dense_ref.assemble(o)
    add_pairs_dense(H, g, 0, 6, ka, kb, kz, kp)
    add_pairs_dense(H, g, 6 * nk, 3, la, lb, lz, lp)
    mu = np.linalg.solve(H, g)
    prev, cur = None, None
    for _ in range(400):
        o.iterate(10, damping=damping)
        bel = o.beliefs()
        cur = np.concatenate([bel["kf_mu"].ravel(), bel["lm_mu"].ravel()])
        if prev is not None and np.abs(cur - prev).max() < 1e-13:
            break
        prev = cur
    assert np.abs(cur - mu).max() / max(1.0, np.abs(mu).max()) < 1e-8
    # without the pairs the solution differs (they carry information)
    H0, g0 = dense_ref.assemble(o)
    assert np.abs(np.linalg.solve(H0, g0) - mu).max() > 1e-4


def test_pair_messages_damping_and_lambda(oracle_mod):
    """Pairwise messages are undamped for their first `undamped` updates,
    then their eta is damped; Lambda messages never depend on d."""
    p = synth.make_config0(seed=1)
    nk = p.n_keyframes
    rng = np.random.default_rng(2)
    args = (0, np.arange(nk - 1), np.arange(1, nk), rng.normal(0, 0.05, (nk - 1, 6)),
            rng.uniform(10, 100, (nk - 1, 6)))
    runs = {}
    for d in (0.0, 0.4):
        o = oracle_mod.Oracle(p, anneal=False, undamped=3)
        o.add_pairs(*args)
        hist = []
        for _ in range(6):
            o.iterate(1, damping=d)
            hist.append(o.pair_messages(0))
        runs[d] = hist
    for it in range(6):
        for key in ("a_lam", "b_lam"):
            assert np.array_equal(runs[0.0][it][key], runs[0.4][it][key])
        if it < 3:
            assert np.array_equal(runs[0.0][it]["a_eta"], runs[0.4][it]["a_eta"])
    # from the fourth update on the damped eta differs
    assert np.abs(runs[0.0][4]["b_eta"] - runs[0.4][4]["b_eta"]).max() > 1e-9


def test_bad_pairs_are_rejected(oracle_mod):
    o = oracle_mod.Oracle(synth.make_config0(seed=0))
    z, pr = np.zeros((1, 3)), np.ones((1, 3))
    for a, b, prec in (([0], [0], pr), ([0], [50], pr), ([-1], [2], pr), ([0], [1], np.zeros((1, 3)))):
        with pytest.raises(ValueError):
            o.add_pairs(1, a, b, z, prec)


# --------------------------------------------------------------------------
# odometry factors: displacement of the camera centres (kind 2)
# --------------------------------------------------------------------------

def _centre(x):
    from scipy.spatial.transform import Rotation
    return -Rotation.from_rotvec(x[:3]).as_matrix().T @ x[3:]


def test_odometry_measurement_and_jacobian(oracle_mod):
    """h = c_b - c_a against scipy's rotation, J against central
    differences of that independent h."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        xa = np.r_[rng.normal(0, 0.6, 3), rng.normal(0, 2, 3)]
        xb = np.r_[rng.normal(0, 0.6, 3), rng.normal(0, 2, 3)]
        h, J = oracle_mod.odometry(xa, xb)
        f = lambda x: _centre(x[6:]) - _centre(x[:6])  # noqa: E731
        x = np.r_[xa, xb]
        assert np.abs(h - f(x)).max() < 1e-12
        Jn = np.zeros((3, 12))
        for i in range(12):
            d = np.zeros(12)
            d[i] = 1e-6
            Jn[:, i] = (f(x + d) - f(x - d)) / 2e-6
        assert np.abs(J - Jn).max() < 1e-7 * max(1.0, np.abs(Jn).max())


def _map_by_gauss_newton(x0, anchors, a, b, z, prec, iters=100):
    """MAP of anchored keyframes plus odometry terms by dense Gauss-Newton
    with numerical Jacobians of the scipy-based centres."""
    nk = x0.shape[0]
    x = x0.copy().ravel()
    for _ in range(iters):
        H = np.diag(np.repeat(anchors, 6)).astype(float)
        g = np.repeat(anchors, 6) * (x0.ravel() - x)
        for i in range(len(a)):
            ia, ib = slice(6 * a[i], 6 * a[i] + 6), slice(6 * b[i], 6 * b[i] + 6)
            xa, xb = x[ia], x[ib]
            r = z[i] - (_centre(xb) - _centre(xa))
            J = np.zeros((3, 12))
            for k in range(6):
                d = np.zeros(6)
                d[k] = 1e-6
                J[:, k] = -(_centre(xa + d) - _centre(xa - d)) / 2e-6
                J[:, 6 + k] = (_centre(xb + d) - _centre(xb - d)) / 2e-6
            P = np.diag(prec[i])
            idx = np.r_[np.arange(6 * a[i], 6 * a[i] + 6), np.arange(6 * b[i], 6 * b[i] + 6)]
            H[np.ix_(idx, idx)] += J.T @ P @ J
            g[idx] += J.T @ P @ r
        dx = np.linalg.solve(H, g)
        x += dx
        if np.abs(dx).max() < 1e-13:
            break
    return x.reshape(nk, 6)


@pytest.mark.parametrize("damping", [0.0, 0.4])
def test_odometry_chain_reaches_the_map(oracle_mod, damping):
    """Anchored keyframes joined by odometry factors (a chain): relinearised
    at every update (hence never damped: always inside the window that
    follows a relinearisation), GBP settles at the MAP of the nonlinear
    objective, whatever the damping setting."""
    nk = 5
    rng = np.random.default_rng(9)
    p = keyframes_only(nk, seed=4, anchor=np.array([1e4, 2.0, 2.0, 2.0, 2.0]))
    a, b = np.arange(nk - 1), np.arange(1, nk)
    z = np.array([_centre(p.kf_init[j]) - _centre(p.kf_init[i]) for i, j in zip(a, b)]) \
        + rng.normal(0, 0.3, (nk - 1, 3))
    prec = rng.uniform(20.0, 200.0, (nk - 1, 3))
    o = oracle_mod.Oracle(p, **FROZEN)
    o.add_pairs(2, a, b, z, prec)
    x_map = _map_by_gauss_newton(p.kf_init, p.kf_anchor_info, a, b, z, prec)
    prev = None
    for _ in range(300):
        o.iterate(10, damping=damping)
        cur = o.beliefs()["kf_mu"]
        if prev is not None and np.abs(cur - prev).max() < 1e-13:
            break
        prev = cur
    assert np.abs(cur - x_map).max() < 1e-8 * max(1.0, np.abs(x_map).max())
    assert np.abs(x_map - p.kf_init).max() > 1e-2   # the odometry moved the poses
