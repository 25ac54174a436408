"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (scipy's rotations), finite differences, closed forms, exact
marginals on trees, the dense linearised MAP on loopy graphs, dense
Gauss-Newton, invariants, and relations between runs that follow from the
definitions (damping, incremental growth).
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from tests import dense_ref

pytestmark = []

CAM = [500.0, 500.0, 320.0, 240.0]
# a camera whose focal lengths and principal point coordinates all differ,
# so that no pin passes with one of them read for another
CAM_SKEWED = [450.0, 520.0, 300.0, 250.0]


def rand_pose_point(rng):
    w = rng.normal(0, 0.6, 3)
    t = rng.normal(0, 1.0, 3)
    R = Rotation.from_rotvec(w).as_matrix()
    # place the point in front of the camera: pick camera coords, map back
    pc = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(2, 8)])
    l = R.T @ (pc - t)
    return np.concatenate([w, t]), l


# --------------------------------------------------------------------------
# SO(3) and the measurement model (Section 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [0.0, 1e-9, 1e-6, 1e-3, 0.3, 1.5, 3.0])
def test_so3_exp_matches_scipy(oracle_mod, scale):
    rng = np.random.default_rng(1)
    for _ in range(5):
        w = rng.normal(size=3)
        w = w / np.linalg.norm(w) * scale
        R = oracle_mod.so3_exp(w)
        Rs = Rotation.from_rotvec(w).as_matrix()
        assert np.abs(R - Rs).max() < 1e-14


@pytest.mark.parametrize("scale", [1e-7, 1e-4, 0.2, 1.0, 2.5])
def test_so3_right_jacobian_fd(oracle_mod, scale):
    """Exp(w + d) = Exp(w) Exp(J_r(w) d) to first order, with Exp and Log
    taken from scipy."""
    rng = np.random.default_rng(2)
    w = rng.normal(size=3)
    w = w / np.linalg.norm(w) * scale
    Jr = oracle_mod.so3_jr(w)
    eps = 1e-6
    Rw = Rotation.from_rotvec(w)
    for i in range(3):
        d = np.zeros(3)
        d[i] = eps
        plus = (Rw.inv() * Rotation.from_rotvec(w + d)).as_rotvec()
        minus = (Rw.inv() * Rotation.from_rotvec(w - d)).as_rotvec()
        col = (plus - minus) / (2 * eps)
        assert np.abs(col - Jr[:, i]).max() < 2e-8


@pytest.mark.parametrize("cam", [CAM, CAM_SKEWED])
def test_projection_matches_library_rotation(oracle_mod, cam):
    rng = np.random.default_rng(3)
    for _ in range(20):
        x, l = rand_pose_point(rng)
        h, _, pz = oracle_mod.project(x, l, cam)
        pc = Rotation.from_rotvec(x[:3]).apply(l) + x[3:]
        assert abs(pz - pc[2]) < 1e-12
        assert np.allclose(h, [cam[0] * pc[0] / pc[2] + cam[2],
                               cam[1] * pc[1] / pc[2] + cam[3]], atol=1e-10)


@pytest.mark.parametrize("cam", [CAM, CAM_SKEWED])
def test_projection_principal_point(oracle_mod, cam):
    # identity pose: a point on the optical axis projects to (cx, cy)
    h, _, pz = oracle_mod.project(np.zeros(6), np.array([0.0, 0.0, 3.0]), cam)
    assert np.allclose(h, cam[2:4]) and pz == 3.0
    # a quarter turn about camera y sends world +x onto the optical axis
    x = np.array([0.0, -np.pi / 2, 0.0, 0.0, 0.0, 0.0])
    h, _, pz = oracle_mod.project(x, np.array([2.0, 0.0, 0.0]), cam)
    assert np.allclose(h, cam[2:4], atol=1e-9) and abs(pz - 2.0) < 1e-12
    # one unit off the axis in x (y) at depth 2 moves u (v) by fx / 2 (fy / 2)
    h, _, _ = oracle_mod.project(np.zeros(6), np.array([1.0, 0.0, 2.0]), cam)
    assert np.allclose(h, [cam[2] + cam[0] / 2, cam[3]], atol=1e-12)
    h, _, _ = oracle_mod.project(np.zeros(6), np.array([0.0, 1.0, 2.0]), cam)
    assert np.allclose(h, [cam[2], cam[3] + cam[1] / 2], atol=1e-12)


@pytest.mark.parametrize("cam", [CAM, CAM_SKEWED])
def test_jacobian_central_differences(oracle_mod, cam):
    """The 2x9 Jacobian of the measurement function (Section 4) against
    central finite differences in every coordinate, relative error < 1e-6."""
    rng = np.random.default_rng(4)
    for _ in range(25):
        x, l = rand_pose_point(rng)
        _, J, _ = oracle_mod.project(x, l, cam)
        v = np.concatenate([x, l])
        Jfd = np.zeros((2, 9))
        for i in range(9):
            e = 1e-6 * max(1.0, abs(v[i]))
            vp, vm = v.copy(), v.copy()
            vp[i] += e
            vm[i] -= e
            hp = oracle_mod.project(vp[:6], vp[6:], cam)[0]
            hm = oracle_mod.project(vm[:6], vm[6:], cam)[0]
            Jfd[:, i] = (hp - hm) / (2 * e)
        assert np.abs(J - Jfd).max() <= 1e-6 * np.abs(Jfd).max()


# --------------------------------------------------------------------------
# Huber rescaling (Section 6)
# --------------------------------------------------------------------------

def test_huber_weight_closed_form(oracle_mod):
    N = 2.0
    assert oracle_mod.huber_weight(N, N) == 1.0           # continuity
    assert oracle_mod.huber_weight(0.3, N) == 1.0
    Ms = np.linspace(2.01, 50, 200)
    w = np.array([oracle_mod.huber_weight(M, N) for M in Ms])
    # w M^2 equals the linear branch of the Huber cost 2 N M - N^2
    assert np.allclose(w * Ms ** 2, 2 * N * Ms - N * N, rtol=1e-14)
    assert np.all(np.diff(w) < 0) and np.all(w < 1) and np.all(w > 0)
    assert oracle_mod.huber_weight(100.0, 0.0) == 1.0     # disabled


# --------------------------------------------------------------------------
# linearised factor in information form (Section 4, eq. (infform))
# --------------------------------------------------------------------------

@pytest.mark.parametrize("camera", [synth.Camera(), synth.Camera(sigma=2.5),
                                    synth.Camera(*CAM_SKEWED, sigma=1.5)], ids=["unit", "sigma2.5", "skewed"])
def test_factor_information_form(oracle_mod, camera):
    """1/2 x^T Lambda x - eta^T x equals 1/2 (w/sigma^2) |J x - (J x0 + r0)|^2
    up to a constant, for the oracle's stored eta_f and Lambda_f (a pixel
    noise other than 1 keeps sigma from cancelling out; a camera whose
    intrinsics all differ checks that the oracle reads the problem's own)."""
    p = synth.make_config0(seed=3, camera=camera)
    o = oracle_mod.Oracle(p, huber_k=2.0)
    rng = np.random.default_rng(5)
    cam = [camera.fx, camera.fy, camera.cx, camera.cy]
    for f in rng.choice(p.n_factors, 12, replace=False):
        eta, lam, lin, w = o.factor(int(f))
        h, J, _ = oracle_mod.project(lin[:6], lin[6:], cam)
        r0 = p.z[f] - h
        M = np.linalg.norm(r0) / p.cam.sigma
        assert abs(w - oracle_mod.huber_weight(M, 2.0 / p.cam.sigma)) < 1e-14
        s = w / p.cam.sigma ** 2

        def e_info(x):
            return 0.5 * x @ lam @ x - eta @ x

        def e_ls(x):
            d = J @ x - (J @ lin + r0)
            return 0.5 * s * d @ d

        xs = [lin + rng.normal(0, 0.05, 9) for _ in range(4)]
        c0 = e_info(xs[0]) - e_ls(xs[0])
        for x in xs[1:]:
            assert abs((e_info(x) - e_ls(x)) - c0) < 1e-8 * max(1.0, abs(c0))
        assert np.allclose(lam, lam.T, atol=0)


def test_prior_schedule(oracle_mod):
    """Automatic priors (Section 4) and their schedule (Section 8): the
    diagonal of sum_f J_i^T Sigma^-1 J_i at the initial linearisation,
    scaled from 1 down to 1/100 geometrically over 10 iterations; the
    anchored keyframe keeps information 1e8 at its initial pose."""
    p = synth.make_config0(seed=4)
    o = oracle_mod.Oracle(p, anneal=True)
    base_k = np.zeros((p.n_keyframes, 6))
    base_l = np.zeros((p.n_landmarks, 3))
    for f in range(p.n_factors):
        k, m = p.factor_kf[f], p.factor_lm[f]
        _, J, _ = oracle_mod.project(p.kf_init[k], p.lm_init[m], CAM)
        base_k[k] += (J[:, :6] ** 2).sum(0) / p.cam.sigma ** 2
        base_l[m] += (J[:, 6:] ** 2).sum(0) / p.cam.sigma ** 2
    for t in [0, 1, 5, 10, 11, 40]:
        sc = 0.01 ** (min(t, 10) / 10)
        kd, ke, ld, le = o.prior(t)
        assert np.allclose(kd[1:], base_k[1:] * sc, rtol=1e-12)
        assert np.allclose(ld, base_l * sc, rtol=1e-12)
        assert np.all(kd[0] == 1e8)
        assert np.allclose(ke, kd * p.kf_init, rtol=1e-12)
        assert np.allclose(le, ld * p.lm_init, rtol=1e-12)
    o2 = oracle_mod.Oracle(p, anneal=False)
    kd, _, ld, _ = o2.prior(0)
    assert np.allclose(kd[1:], base_k[1:] * 0.01, rtol=1e-12)
    assert np.allclose(ld, base_l * 0.01, rtol=1e-12)


# --------------------------------------------------------------------------
# message passing: trees are exact (Section 3.2); loopy means are exact
# --------------------------------------------------------------------------

FROZEN = dict(beta=1e30, relin_interval=10 ** 9, anneal=False)


def _marginals(H, g, nk, nl):
    mu = np.linalg.solve(H, g)
    cov = np.linalg.inv(H)
    kf, lm = dense_ref.index_maps(nk, nl)
    return mu, cov, kf, lm


@pytest.mark.parametrize("shape", [(3, 0), (4, 2), (2, 3)])
def test_tree_beliefs_are_exact_marginals(oracle_mod, shape):
    p = synth.make_tree_chain(*shape)
    o = oracle_mod.Oracle(p, **FROZEN)
    H, g = dense_ref.assemble(o)
    o.iterate(4 * (p.n_keyframes + 2), damping=0.0)
    b = o.beliefs()
    mu, cov, kf, lm = _marginals(H, g, o.nk, o.nl)
    for k in range(o.nk):
        assert np.abs(b["kf_mu"][k] - mu[kf(k)]).max() < 1e-9 * max(1, np.abs(mu[kf(k)]).max())
        ck = np.linalg.inv(b["kf_lam"][k])
        assert np.abs(ck - cov[np.ix_(kf(k), kf(k))]).max() < 1e-8 * np.abs(ck).max()
    for m in range(o.nl):
        assert np.abs(b["lm_mu"][m] - mu[lm(m)]).max() < 1e-9 * max(1, np.abs(mu[lm(m)]).max())
        cm = np.linalg.inv(b["lm_lam"][m])
        assert np.abs(cm - cov[np.ix_(lm(m), lm(m))]).max() < 1e-8 * np.abs(cm).max()


@pytest.mark.parametrize("damping", [0.0, 0.4])
def test_loopy_means_equal_dense_solve(oracle_mod, damping):
    """Loopy GBP on the tiny circle problem with the linearisation frozen
    converges to the dense linearised MAP (Section 3.2)."""
    p = synth.make_config0(seed=0)
    o = oracle_mod.Oracle(p, **FROZEN)
    H, g = dense_ref.assemble(o)
    mu, cov, kf, lm = _marginals(H, g, o.nk, o.nl)
    prev = None
    for _ in range(400):
        o.iterate(10, damping=damping)
        b = o.beliefs()
        cur = np.concatenate([b["kf_mu"].ravel(), b["lm_mu"].ravel()])
        if prev is not None and np.abs(cur - prev).max() < 1e-13:
            break
        prev = cur
    err = np.abs(cur - mu).max() / max(1.0, np.abs(mu).max())
    assert err < 1e-8, err


def test_tree_covariance_only_loopy_mean(oracle_mod):
    """On a loopy graph the belief covariances are not the exact marginals
    (only the means are); this guards against a test that could not fail."""
    p = synth.make_config0(seed=0)
    o = oracle_mod.Oracle(p, **FROZEN)
    H, g = dense_ref.assemble(o)
    o.iterate(600, damping=0.0)
    b = o.beliefs()
    _, cov, kf, lm = _marginals(H, g, o.nk, o.nl)
    rel = [np.abs(np.linalg.inv(b["lm_lam"][m]) - cov[np.ix_(lm(m), lm(m))]).max()
           / np.abs(cov[np.ix_(lm(m), lm(m))]).max() for m in range(o.nl)]
    assert max(rel) > 1e-4


def test_damping_acts_on_eta_only_after_window(oracle_mod):
    """Damping (Section 5, Section 8): Lambda messages do not depend on d;
    eta messages are undamped for the first 8 updates after linearisation;
    the 9th damped update equals (1-d) new + d old, where `new` is what the
    undamped run computes from the identical state."""
    p = synth.make_config0(seed=1)
    a = oracle_mod.Oracle(p, **FROZEN)
    b = oracle_mod.Oracle(p, **FROZEN)
    hist = []
    for it in range(1, 10):
        a.iterate(1, damping=0.0)
        b.iterate(1, damping=0.4)
        ma, mb = a.messages(), b.messages()
        hist.append(ma)
        if it <= 8:
            for key in ma:
                assert np.array_equal(ma[key], mb[key]), (it, key)
        else:
            assert np.array_equal(ma["k_lam"], mb["k_lam"])
            assert np.array_equal(ma["l_lam"], mb["l_lam"])
            for key in ("k_eta", "l_eta"):
                want = 0.6 * ma[key] + 0.4 * hist[-2][key]
                assert np.allclose(mb[key], want, rtol=1e-12, atol=1e-9)
                assert not np.allclose(mb[key], ma[key], rtol=1e-6)


def test_relinearised_fixed_point_matches_gauss_newton(oracle_mod):
    """With relinearisation, the stationary GBP means are the Gauss-Newton
    fixed point of the same objective (same priors, same Huber weight rule)."""
    p = synth.make_config0(seed=2, n_lm=25)
    o = oracle_mod.Oracle(p, anneal=False, huber_k=2.0)
    priors = o.prior(0)
    prev = None
    for _ in range(150):
        o.iterate(10, damping=0.4, huber_k=2.0)
        o.relinearise(-1)
        b = o.beliefs()
        cur = np.concatenate([b["kf_mu"].ravel(), b["lm_mu"].ravel()])
        if prev is not None and np.abs(cur - prev).max() < 1e-12:
            break
        prev = cur
    x = dense_ref.gauss_newton(p, priors, 2.0, project=oracle_mod.project,
                               huber_weight=oracle_mod.huber_weight, x0=cur)
    assert np.abs(x - cur).max() < 1e-6 * max(1.0, np.abs(x).max())
    # and the fixed point is a genuine improvement on the initial estimate
    assert o.reproj()["are_all"] < 2.0


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

def test_messages_symmetric_psd_beliefs_pd(oracle_mod):
    p = synth.make_config0(seed=5)
    o = oracle_mod.Oracle(p)
    for _ in range(3):
        o.iterate(10, 0.4)
        o.relinearise(-1)
        m = o.messages()
        for key in ("k_lam", "l_lam"):
            L = m[key]
            assert np.abs(L - np.swapaxes(L, 1, 2)).max() <= 1e-9 * np.abs(L).max()
            ev = np.linalg.eigvalsh(0.5 * (L + np.swapaxes(L, 1, 2)))
            nrm = np.abs(L).max(axis=(1, 2)) + 1e-300
            assert np.all(ev.min(axis=1) >= -1e-9 * nrm)
        b = o.beliefs()
        assert np.all(np.linalg.eigvalsh(b["kf_lam"]).min(axis=1) > 0)
        assert np.all(np.linalg.eigvalsh(b["lm_lam"]).min(axis=1) > 0)


@pytest.mark.parametrize("damping,damp_lambda", [(0.0, False), (0.4, True)])
def test_noise_free_data_stays_at_truth(oracle_mod, damping, damp_lambda):
    """Noise-free measurements and a true initial estimate give r0 = 0, so
    every message is centred on the truth and the means stay there at every
    iteration whenever eta and Lambda are updated consistently."""
    p = synth.make_config0(seed=6)
    p.z = p.z_true.copy()
    o = oracle_mod.Oracle(p, kf_init=p.kf_true, lm_init=p.lm_true,
                          damp_lambda=damp_lambda)
    assert o.reproj()["are_all"] < 1e-9
    for _ in range(5):
        o.iterate(10, damping)
        o.relinearise(-1)
        b = o.beliefs()
        assert np.abs(b["kf_mu"] - p.kf_true).max() < 1e-9
        assert np.abs(b["lm_mu"] - p.lm_true).max() < 1e-9
        assert o.reproj()["are_all"] < 1e-9


def test_eta_only_damping_transient_returns_to_truth(oracle_mod):
    """Damping eta alone mixes a new Lambda with an old eta, so on noise-free
    data the means leave the truth while the Lambda messages still change,
    and return to it at the fixed point (damping does not move fixed
    points)."""
    p = synth.make_config0(seed=6)
    p.z = p.z_true.copy()
    o = oracle_mod.Oracle(p, kf_init=p.kf_true, lm_init=p.lm_true, beta=1e30,
                          relin_interval=10 ** 9)
    o.iterate(12, 0.4)
    b = o.beliefs()
    assert np.abs(b["lm_mu"] - p.lm_true).max() > 1e-8
    o.iterate(800, 0.4)
    b = o.beliefs()
    assert np.abs(b["kf_mu"] - p.kf_true).max() < 1e-9
    assert np.abs(b["lm_mu"] - p.lm_true).max() < 1e-9


@pytest.mark.parametrize("camera", [synth.Camera(), synth.Camera(sigma=2.5),
                                    synth.Camera(*CAM_SKEWED, sigma=1.5)], ids=["unit", "sigma2.5", "skewed"])
def test_reprojection_error_brute_force(oracle_mod, camera):
    """Average reprojection error (Section 9.1) recomputed with scipy; the
    robust kernel's linear regime is |r| above the threshold in pixels,
    whatever the pixel noise."""
    p = synth.make_random_walk("t", 3, 12, 150, "poisson", 0.05, camera=camera)
    o = oracle_mod.Oracle(p)
    o.iterate(15, 0.4, 2.0)
    b = o.beliefs()
    pc = (Rotation.from_rotvec(b["kf_mu"][p.factor_kf, :3]).apply(b["lm_mu"][p.factor_lm])
          + b["kf_mu"][p.factor_kf, 3:])
    hz = np.stack([camera.fx * pc[:, 0] / pc[:, 2] + camera.cx,
                   camera.fy * pc[:, 1] / pc[:, 2] + camera.cy], 1)
    valid = pc[:, 2] > 1e-3
    e = np.linalg.norm(p.z - hz, axis=1)
    r = o.reproj(p.z_true, p.inlier)
    assert r["n_valid"] == valid.sum()
    assert abs(r["are_all"] - e[valid].mean()) < 1e-10
    lin = valid & (e > 2.0)
    assert r["n_linear"] == lin.sum()
    assert abs(r["are_quadratic"] - e[valid & ~lin].mean()) < 1e-10
    eref = np.linalg.norm(p.z_true - hz, axis=1)
    assert abs(r["are_ref"] - eref[valid & p.inlier].mean()) < 1e-10
    # outlier classification (Section 9.4): linear-regime true inliers are
    # the false positives; with 5% outliers after 15 iterations both kinds
    # of linear-regime factor occur
    assert r["n_ref"] == (valid & p.inlier).sum()
    assert r["n_linear_ref"] == (lin & p.inlier).sum()
    assert 0 < r["n_linear_ref"] < r["n_linear"]


def test_reprojection_statistics_leave_out_points_behind_the_camera(oracle_mod):
    """The averages run over the points in front of their camera only, and
    the others are counted apart (brute force at the oracle's means)."""
    p = synth.make_config0(seed=7)
    for m in (0, 5):
        k = int(p.factor_kf[np.flatnonzero(p.factor_lm == m)[0]])
        R = Rotation.from_rotvec(p.kf_init[k, :3]).as_matrix()
        p.lm_init[m] = R.T @ (np.array([0.1, 0.1, -1.0]) - p.kf_init[k, 3:])
    o = oracle_mod.Oracle(p)
    b = o.beliefs()
    pc = (Rotation.from_rotvec(b["kf_mu"][p.factor_kf, :3]).apply(b["lm_mu"][p.factor_lm])
          + b["kf_mu"][p.factor_kf, 3:])
    valid = pc[:, 2] > 1e-3
    assert 0 < (~valid).sum() < len(valid)
    hz = np.stack([500 * pc[:, 0] / pc[:, 2] + 320, 500 * pc[:, 1] / pc[:, 2] + 240], 1)
    e = np.linalg.norm(p.z - hz, axis=1)
    # a threshold between the errors, so that both regimes occur (the
    # means at creation do not depend on it)
    thr = float(np.median(e[valid]))
    o = oracle_mod.Oracle(p, huber_k=thr)
    assert np.array_equal(o.beliefs()["lm_mu"], b["lm_mu"])
    r = o.reproj()
    assert r["n_invalid"] == (~valid).sum() and r["n_valid"] == valid.sum()
    assert abs(r["are_all"] - e[valid].mean()) < 1e-10
    lin = valid & (e > thr)
    assert 0 < lin.sum() < valid.sum() and r["n_linear"] == lin.sum()
    assert abs(r["are_quadratic"] - e[valid & ~lin].mean()) < 1e-10


def test_point_behind_camera_carries_no_information(oracle_mod):
    p = synth.make_config0(seed=7)
    # push landmark 0 behind keyframe 1's camera for its initial estimate
    k = int(p.factor_kf[np.flatnonzero(p.factor_lm == 0)[0]])
    R = Rotation.from_rotvec(p.kf_init[k, :3]).as_matrix()
    p.lm_init[0] = R.T @ (np.array([0.1, 0.1, -1.0]) - p.kf_init[k, 3:])
    o = oracle_mod.Oracle(p)
    fs = np.flatnonzero((p.factor_lm == 0) & (p.factor_kf == k))
    for f in fs:
        eta, lam, _, w = o.factor(int(f))
        assert w == 0.0 and not eta.any() and not lam.any()
    assert o.reproj()["n_invalid"] >= len(fs)


def test_incremental_add_of_disjoint_block_equals_joint_create(oracle_mod):
    """Growing the graph by a disconnected block at t = 0 gives exactly the
    state of creating both blocks at once (own priors, zero messages)."""
    a = synth.make_config0(seed=8, n_lm=20)
    bb = synth.make_config0(seed=9, n_lm=15)
    bb.kf_anchor_info[:] = 0.0
    bb.kf_anchor_info[0] = 1e8
    nk, nl = a.n_keyframes, a.n_landmarks
    joint = synth.BAProblem(
        "joint", a.cam, np.vstack([a.kf_true, bb.kf_true]), np.vstack([a.lm_true, bb.lm_true]),
        np.vstack([a.kf_init, bb.kf_init]), np.vstack([a.lm_init, bb.lm_init]),
        np.concatenate([a.factor_kf, bb.factor_kf + nk]).astype(np.int32),
        np.concatenate([a.factor_lm, bb.factor_lm + nl]).astype(np.int32),
        np.vstack([a.z, bb.z]), np.vstack([a.z_true, bb.z_true]),
        np.concatenate([a.inlier, bb.inlier]),
        np.concatenate([a.kf_anchor_info, bb.kf_anchor_info]))
    oj = oracle_mod.Oracle(joint)
    og = oracle_mod.Oracle(a)
    og.add(bb.kf_init, bb.lm_init, bb.factor_kf + nk, bb.factor_lm + nl, bb.z,
           kf_anchor_info=bb.kf_anchor_info)
    for _ in range(3):
        oj.iterate(7, 0.4)
        og.iterate(7, 0.4)
        x, y = oj.beliefs(), og.beliefs()
        for key in x:
            assert np.array_equal(x[key], y[key]), key
