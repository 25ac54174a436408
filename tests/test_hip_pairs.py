"""Pairwise difference factors (heterogeneous factors) on the HIP path,
through the C ABI, against the FP64 oracle (which is pinned in
tests/test_oracle_pairs.py). Tolerances as for the measurement factors:
FP64 storage 1e-8 relative on means and information, FP32 storage 1e-4."""
import numpy as np
import pytest

import synth
from tests.test_hip_parity import gbp, info_err, mean_errs, pair  # noqa: F401

pytestmark = pytest.mark.gpu


def ring_and_lm_pairs(p, seed=11, n_lm_pairs=20, kp=(50, 500), lp=(5, 50)):
    """Keyframe ring (k -> k + 1 mod Nk) and random landmark pairs, with
    measured differences near the truth."""
    rng = np.random.default_rng(seed)
    nk, nl = p.n_keyframes, p.n_landmarks
    ka, kb = np.arange(nk), (np.arange(nk) + 1) % nk
    kz = p.kf_true[kb] - p.kf_true[ka] + rng.normal(0, 0.01, (nk, 6))
    kpr = rng.uniform(*kp, (nk, 6))
    la = rng.choice(nl, n_lm_pairs, replace=False)
    lb = (la + 1 + rng.integers(0, nl - 1, n_lm_pairs)) % nl
    lz = p.lm_true[lb] - p.lm_true[la] + rng.normal(0, 0.02, (n_lm_pairs, 3))
    lpr = rng.uniform(*lp, (n_lm_pairs, 3))
    return (0, ka, kb, kz, kpr), (1, la, lb, lz, lpr)


def add_both(s, o, pairs):
    for kind, a, b, z, pr in pairs:
        s.add_pair_factors(kind, a, b, z, pr)
        o.add_pairs(kind, a, b, z, pr)


@pytest.mark.parametrize("damp_lambda", [False, True])
def test_fp64_pairs_forced_schedule_every_checkpoint(gbp, damp_lambda):
    prob = synth.make_config0(seed=0)
    s, o = pair(gbp, prob, gbp.GBP_FP64, damp_lambda=damp_lambda)
    add_both(s, o, ring_and_lm_pairs(prob))
    for it in range(12):
        s.iterate(10, 0.4, 2.0)
        o.iterate(10, 0.4, 2.0)
        g, r = s.beliefs(info=True), o.beliefs()
        assert mean_errs(g, r) < 1e-8, it
        assert info_err(g, r) < 1e-8, it
        s.relinearise(-1)
        o.relinearise(-1)
    s.close()


def test_fp64_pairs_beta_rule_and_added_later(gbp):
    """Pairs added after 15 iterations (their messages start at zero, their
    undamped window starts then), beta rule on both sides."""
    prob = synth.make_config0(seed=3)
    s, o = pair(gbp, prob, gbp.GBP_FP64)
    s.iterate(15, 0.4, 2.0)
    o.iterate(15, 0.4, 2.0)
    add_both(s, o, ring_and_lm_pairs(prob, seed=4))
    for it in range(5):
        s.iterate(20, 0.4, 2.0)
        o.iterate(20, 0.4, 2.0)
        assert mean_errs(s.beliefs(), o.beliefs()) < 1e-8, it
    s.close()


def test_keyframe_chain_without_measurements(gbp):
    """Anchored keyframes joined only by pose pairs (a tree, no landmarks,
    no measurements): GPU and oracle agree, and the pairs moved the means."""
    from tests.test_oracle_pairs import keyframes_only
    p = keyframes_only(6)
    rng = np.random.default_rng(5)
    a, b = np.arange(5), np.arange(1, 6)
    z, pr = rng.normal(0, 0.3, (5, 6)), rng.uniform(0.5, 5.0, (5, 6))
    s, o = pair(gbp, p, gbp.GBP_FP64)
    s.add_pair_factors(0, a, b, z, pr)
    o.add_pairs(0, a, b, z, pr)
    s.iterate(40, 0.4, 2.0)
    o.iterate(40, 0.4, 2.0)
    g, r = s.beliefs(info=True), o.beliefs()
    assert np.abs(g["kf_mu"] - r["kf_mu"]).max() < 1e-8 * max(1.0, np.abs(r["kf_mu"]).max())
    assert np.abs(g["kf_lam"] - r["kf_lam"]).max() < 1e-8 * np.abs(r["kf_lam"]).max()
    assert np.abs(g["kf_mu"] - p.kf_init).max() > 1e-2
    s.close()


def test_fp32_pairs_on_the_paper_scale_problem(gbp):
    prob = synth.make_config1()
    s, o = pair(gbp, prob, gbp.GBP_FP32)
    add_both(s, o, ring_and_lm_pairs(prob, n_lm_pairs=300, kp=(5, 50)))
    worst = 0.0
    for it in range(6):
        s.iterate(10, 0.4, 2.0)
        o.iterate(10, 0.4, 2.0)
        e = mean_errs(s.beliefs(), o.beliefs())
        worst = max(worst, e)
        assert e < 1e-4, (it, e)
        s.relinearise(-1)
        o.relinearise(-1)
    print(f"config1 FP32 with pairs: worst relative mean error {worst:.2e}")
    s.close()


def test_batched_pairs_equal_single_problems(gbp):
    """Pairs in a batch (caller indices problem-major) give bitwise the
    single-problem results; a problem without pairs is unaffected."""
    probs = [synth.make_config3_problem(p) for p in range(3)]
    sets = [ring_and_lm_pairs(probs[0], seed=1), None, ring_and_lm_pairs(probs[2], seed=2)]
    ko = np.cumsum([0] + [p.n_keyframes for p in probs])
    lo = np.cumsum([0] + [p.n_landmarks for p in probs])
    b = gbp.GBPSolver(probs)
    for i, ps in enumerate(sets):
        if ps is None:
            continue
        for kind, a, bb, z, pr in ps:
            off = ko[i] if kind == 0 else lo[i]
            b.add_pair_factors(kind, a + off, bb + off, z, pr)
    b.iterate(30, 0.4, 2.0)
    gb = b.beliefs()
    for i, ps in enumerate(sets):
        s = gbp.GBPSolver(probs[i])
        if ps is not None:
            for args in ps:
                s.add_pair_factors(*args)
        s.iterate(30, 0.4, 2.0)
        g = s.beliefs()
        assert np.array_equal(g["kf_mu"], gb["kf_mu"][ko[i]:ko[i + 1]]), i
        assert np.array_equal(g["lm_mu"], gb["lm_mu"][lo[i]:lo[i + 1]]), i
        s.close()
    b.close()


def test_reset_logging_and_autotune_with_pairs(gbp, tmp_path):
    prob = synth.make_config1()
    s = gbp.GBPSolver(prob)
    for args in ring_and_lm_pairs(prob, n_lm_pairs=200, kp=(5, 50)):
        s.add_pair_factors(*args)
    s.iterate(25, 0.4, 2.0)
    ref = s.beliefs()
    s.reset()                                   # pairs kept, messages zeroed
    log = s.iterate_logged(25, 0.4, 2.0, log_every=1)
    got = s.beliefs()
    for key in ref:
        assert np.array_equal(got[key], ref[key]), key
    assert log.shape == (25, 1, 5)
    # stored beliefs (no recomputation: the tuned lane count may change the
    # landmark sums' order)
    before = s.beliefs()
    s.autotune(2, str(tmp_path / "tune.txt"))   # snapshot covers the pair state
    after = s.beliefs()
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    s.iterate(5, 0.4, 2.0)
    s.close()


def test_bad_pairs_and_growth_are_rejected(gbp):
    prob = synth.make_config0(seed=0)
    s = gbp.GBPSolver(prob)
    z3, one3 = np.zeros((1, 3)), np.ones((1, 3))
    bad = [(1, [0], [0], z3, one3), (1, [0], [50], z3, one3), (1, [-1], [3], z3, one3),
           (1, [0], [1], z3, np.zeros((1, 3))), (1, [0], [1], np.full((1, 3), np.nan), one3),
           (3, [0], [1], z3, one3), (2, [0], [50], z3, one3)]
    for args in bad:
        with pytest.raises(gbp.GBPError) as e:
            s.add_pair_factors(*args)
        assert e.value.status == -1
    # a count beyond the 32-bit index limit is refused before the arrays are
    # read (the pointers below are never dereferenced)
    import ctypes as C
    lib = gbp.load_library()
    fi = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_int32))
    fd = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_double))
    for kind in (0, 1, 2):
        assert lib.gbp_add_pair_factors(s.h, kind, (1 << 30) + 1, fi, fi, fd, fd) == -1
        assert b"GBP_MAX_BATCH_ITEMS" in lib.gbp_last_error(s.h)
    s.add_pair_factors(1, [0], [1], z3, one3)
    with pytest.raises(gbp.GBPError) as e:
        s.add_keyframe(prob.kf_init[1], np.zeros((0, 3)), [], [], np.zeros((0, 2)))
    assert e.value.status == -5
    s.close()


# --------------------------------------------------------------------------
# odometry factors (camera-centre displacement, relinearised every update)
# --------------------------------------------------------------------------

def _centres(x):
    from scipy.spatial.transform import Rotation
    return np.array([-Rotation.from_rotvec(v[:3]).as_matrix().T @ v[3:] for v in x])


def odometry_ring(p, seed=3, closed=True, prec=(10, 100)):
    rng = np.random.default_rng(seed)
    nk = p.n_keyframes
    a = np.arange(nk if closed else nk - 1)
    b = (a + 1) % nk
    c = _centres(p.kf_true)
    z = c[b] - c[a] + rng.normal(0, 0.02, (len(a), 3))
    return (2, a, b, z, rng.uniform(*prec, (len(a), 3)))


@pytest.mark.parametrize("damp_lambda", [False, True])
def test_fp64_odometry_with_difference_and_landmark_pairs(gbp, damp_lambda):
    """Odometry ring plus difference factors of both kinds on the circle
    problem, forced relinearisation of the measurement factors."""
    prob = synth.make_config0(seed=0)
    s, o = pair(gbp, prob, gbp.GBP_FP64, damp_lambda=damp_lambda)
    add_both(s, o, ring_and_lm_pairs(prob) + (odometry_ring(prob),))
    for it in range(10):
        s.iterate(10, 0.4, 2.0)
        o.iterate(10, 0.4, 2.0)
        g, r = s.beliefs(info=True), o.beliefs()
        assert mean_errs(g, r) < 1e-8, it
        assert info_err(g, r) < 1e-8, it
        s.relinearise(-1)
        o.relinearise(-1)
    s.close()


def test_odometry_chain_without_measurements(gbp):
    from tests.test_oracle_pairs import keyframes_only
    p = keyframes_only(6, seed=4, anchor=np.array([1e4] + [2.0] * 5))
    rng = np.random.default_rng(2)
    a, b = np.arange(5), np.arange(1, 6)
    c = _centres(p.kf_init)
    z, pr = c[b] - c[a] + rng.normal(0, 0.3, (5, 3)), rng.uniform(20, 200, (5, 3))
    s, o = pair(gbp, p, gbp.GBP_FP64)
    s.add_pair_factors(gbp.GBP_PAIR_ODOMETRY, a, b, z, pr)
    o.add_pairs(2, a, b, z, pr)
    for it in range(4):
        s.iterate(15, 0.4, 2.0)
        o.iterate(15, 0.4, 2.0)
        g, r = s.beliefs(info=True), o.beliefs()
        assert np.abs(g["kf_mu"] - r["kf_mu"]).max() < 1e-8 * max(1.0, np.abs(r["kf_mu"]).max()), it
        assert np.abs(g["kf_lam"] - r["kf_lam"]).max() < 1e-8 * np.abs(r["kf_lam"]).max(), it
    assert np.abs(g["kf_mu"] - p.kf_init).max() > 1e-2
    s.close()


def test_fp32_odometry_on_the_paper_scale_problem(gbp):
    prob = synth.make_config1()
    s, o = pair(gbp, prob, gbp.GBP_FP32)
    add_both(s, o, (odometry_ring(prob, closed=False),))
    worst = 0.0
    for it in range(6):
        s.iterate(10, 0.4, 2.0)
        o.iterate(10, 0.4, 2.0)
        e = mean_errs(s.beliefs(), o.beliefs())
        worst = max(worst, e)
        assert e < 1e-4, (it, e)
        s.relinearise(-1)
        o.relinearise(-1)
    print(f"config1 FP32 with odometry: worst relative mean error {worst:.2e}")
    s.close()
