"""Host logic of the robustness and Huber studies (Sections 9.3 and 9.4),
no GPU: the success and classification arithmetic on hand-made logs, the
study inputs against their stated shapes, and the oracle's classification
counts on a converged problem."""
import numpy as np
import pytest

from paper_2003_03134_amd import studies


def test_first_below_is_one_based_and_zero_when_never():
    a = np.array([[3.0, 2.0, 9.0], [1.4, 1.6, 9.0], [1.0, 1.2, 9.0]])
    assert studies.first_below(a, 1.5).tolist() == [2, 3, 0]
    # equal to the target is not below it
    assert studies.first_below(np.array([[1.5]]), 1.5).tolist() == [0]


def test_classification_counts():
    # rows: 2 logged iterations, 2 trials; columns t, are_all, are_ref,
    # n_linear (all classed outliers), n_linear_ref (inliers among them)
    log = np.zeros((2, 2, 5))
    log[0, :, 3], log[0, :, 4] = [10, 6], [7, 3]   # tp = 3, 3
    log[1, :, 3], log[1, :, 4] = [4, 3], [0, 1]    # tp = 4, 2
    c = studies.classification(log, np.array([4, 5]))
    assert np.allclose(c["precision"], [6 / 16, 6 / 7])
    assert np.allclose(c["recall"], [6 / 9, 6 / 9])
    assert np.allclose(c["precision_trial0"], [0.3, 1.0])
    assert np.allclose(c["recall_trial0"], [0.75, 1.0])


def test_study_inputs_have_the_stated_shapes():
    p = studies.basin_problem("fr1desk30", 0.1, 0)
    q = studies.basin_problem("fr1desk30", 0.3, 0)
    assert p.n_keyframes == 30 and p.n_landmarks == 1390
    assert 4.0 < p.n_factors / p.n_landmarks < 5.2 and p.inlier.all()
    # same geometry and noise directions at every level, the noise scaled
    assert np.array_equal(p.z, q.z) and np.array_equal(p.kf_true, q.kf_true)
    dp = p.kf_init[1:, 3:] - p.kf_true[1:, 3:]
    dq = q.kf_init[1:, 3:] - q.kf_true[1:, 3:]
    assert np.allclose(dq, 3.0 * dp, rtol=1e-9, atol=1e-12)
    o = studies.outlier_problem(0.03, 0)
    assert o.n_keyframes == 20 and abs((~o.inlier).sum() - 0.03 * o.n_factors) <= 1


def test_oracle_outlier_classification_recall_and_precision(oracle_mod):
    """Section 9.4 (Fig. 7a): every bad association sits in the linear
    regime (recall 1), while inliers enter it only through the Gaussian
    tail: a 2-D residual of per-axis deviation sigma exceeds 2 sigma with
    probability exp(-2) = 13.5%, less once the estimate fits the noise."""
    p = studies.outlier_problem(0.03, 1)
    o = oracle_mod.Oracle(p, anneal=False)
    n_out = int((~p.inlier).sum())
    for _ in range(3):
        o.iterate(50, 0.4, 2.0)
        r = o.reproj(p.z, p.inlier)
        assert r["n_ref"] == int(p.inlier.sum())
        assert r["n_linear"] - r["n_linear_ref"] == n_out
        assert 0.05 * r["n_ref"] < r["n_linear_ref"] < 0.16 * r["n_ref"]
        assert r["are_ref"] < 1.5 < r["are_all"]
