"""Pins of the oracle's schedules: the local relinearisation rule (Section 5,
hyperparameters of Section 8), the annealed prior as the belief phase applies
it (Section 4 automatic priors, Section 8 schedule), the own clock of
variables added by incremental growth (Section 9.2) and the claim of
Section 8 that the annealed run reaches the same answer as the un-annealed
one.

Each expected value is computed here from the definitions with numpy: which
factors are due (counter and stacked 9-vector distance), the prior scale
0.01^(min(t, 10)/10) times the diagonal of sum_f J^T J / sigma^2 from the
projection Jacobians, and the belief identity "belief = prior + sum of the
incoming messages" (eqs. beliefeta, belieflambda). None of them re-runs the
oracle's own schedule code.
"""
import numpy as np
import pytest

import synth

CAM = [500.0, 500.0, 320.0, 240.0]


def _means(o):
    b = o.beliefs()
    return b["kf_mu"].copy(), b["lm_mu"].copy()


def _lin_points(o):
    return np.array([o.factor(f)[2] for f in range(o.nf)])


def _distances(p, kf_mu, lm_mu, lin):
    x = np.concatenate([kf_mu[p.factor_kf], lm_mu[p.factor_lm]], axis=1)
    return np.linalg.norm(x - lin, axis=1)


def _schedule_beta(p):
    """A beta that splits the factors: the median distance from the
    linearisation point after 10 iterations without relinearisation."""
    import oracle
    ref = oracle.Oracle(p, beta=1e30)
    ref.iterate(10, damping=0.4)
    kf, lm = _means(ref)
    return float(np.median(_distances(p, kf, lm, _lin_points(ref))))


def test_relinearisation_rule_selects_exactly_the_due_factors(oracle_mod):
    """Section 5 / Section 8: at the start of an iteration a factor is
    relinearised iff at least 10 updates have passed since its last
    linearisation and the stacked [mu_k; mu_m] lies strictly farther than
    beta from its linearisation point. A relinearised factor takes the
    current means as its new point and its counter restarts."""
    p = synth.make_config0(seed=11)
    beta = _schedule_beta(p)
    o = oracle_mod.Oracle(p, beta=beta, anneal=True)
    seen = dict(due=0, young_far=0, old_near=0, old_half=0)
    for it in range(40):
        kf, lm = _means(o)
        lin = _lin_points(o)
        cnt, _ = o.counters()
        dist = _distances(p, kf, lm, lin)
        old = cnt >= 10
        due = old & (dist > beta)
        seen["due"] += int(due.sum())
        seen["young_far"] += int((~old & (dist > beta)).sum())
        seen["old_near"] += int((old & (dist <= beta)).sum())
        seen["old_half"] += int((old & (dist > 0.5 * beta) & (dist <= beta)).sum())
        o.iterate(1, damping=0.4)
        cnt2, _ = o.counters()
        lin2 = _lin_points(o)
        x = np.concatenate([kf[p.factor_kf], lm[p.factor_lm]], axis=1)
        assert np.array_equal(cnt2, np.where(due, 1, cnt + 1)), it
        assert np.array_equal(lin2[due], x[due]), it
        assert np.array_equal(lin2[~due], lin[~due]), it
    # the run exercised every branch of the rule
    assert seen["due"] > 0 and seen["young_far"] > 0
    assert seen["old_near"] > 0 and seen["old_half"] > 0, seen


def test_no_relinearisation_before_the_interval(oracle_mod):
    """With beta = 0 every factor that moved is due as soon as it is old
    enough: nothing relinearises in iterations 1-10, and at iteration 11
    exactly the factors whose point moved do."""
    p = synth.make_config0(seed=12, n_lm=20)
    o = oracle_mod.Oracle(p, beta=0.0)
    lin0 = _lin_points(o)
    for it in range(1, 11):
        o.iterate(1, damping=0.4)
        cnt, _ = o.counters()
        assert np.all(cnt == it)
        assert np.array_equal(_lin_points(o), lin0)
    kf, lm = _means(o)
    moved = _distances(p, kf, lm, lin0) > 0.0
    assert moved.sum() > 0.9 * p.n_factors
    o.iterate(1, damping=0.4)
    cnt, _ = o.counters()
    assert np.array_equal(cnt, np.where(moved, 1, 11))


def _prior_base(p, kf_at, lm_at, factors):
    """diag(sum_f J_v^T J_v) / sigma^2 over `factors`, Jacobians taken at
    (kf_at, lm_at), Huber weight 1, floored at 1e-8 (Section 4 priors)."""
    import oracle
    bk = np.zeros((p.n_keyframes, 6))
    bl = np.zeros((p.n_landmarks, 3))
    for f in factors:
        k, m = p.factor_kf[f], p.factor_lm[f]
        _, J, pz = oracle.project(kf_at[k], lm_at[m], CAM)
        if pz > 1e-3:
            bk[k] += (J[:, :6] ** 2).sum(0) / p.cam.sigma ** 2
            bl[m] += (J[:, 6:] ** 2).sum(0) / p.cam.sigma ** 2
    return np.maximum(bk, 1e-8), np.maximum(bl, 1e-8)


def _belief_minus_messages(o, p_kf, p_lm):
    """Belief information minus the sum of the incoming factor messages: the
    prior that the belief phase applied (eq. belieflambda), with eta."""
    b = o.beliefs()
    m = o.messages()
    kl = b["kf_lam"].copy()
    ke = b["kf_eta"].copy()
    ll = b["lm_lam"].copy()
    le = b["lm_eta"].copy()
    np.subtract.at(kl, p_kf, m["k_lam"])
    np.subtract.at(ke, p_kf, m["k_eta"])
    np.subtract.at(ll, p_lm, m["l_lam"])
    np.subtract.at(le, p_lm, m["l_eta"])
    scale = (np.abs(b["kf_lam"]).max(), np.abs(b["lm_lam"]).max())
    return kl, ke, ll, le, scale


def _check_prior(kl, ke, ll, le, scale, want_kd, want_ld, kf_mean, lm_mean, sel_k, sel_l, tag):
    for k in sel_k:
        assert np.allclose(np.diag(kl[k]), want_kd[k], rtol=1e-9, atol=1e-12 * scale[0]), (tag, k)
        off = kl[k] - np.diag(np.diag(kl[k]))
        assert np.abs(off).max() <= 1e-12 * scale[0], (tag, k)
        assert np.allclose(ke[k], want_kd[k] * kf_mean[k], rtol=1e-8,
                           atol=1e-12 * scale[0] * (1 + np.abs(kf_mean[k]).max())), (tag, k)
    for m in sel_l:
        assert np.allclose(np.diag(ll[m]), want_ld[m], rtol=1e-9, atol=1e-12 * scale[1]), (tag, m)
        off = ll[m] - np.diag(np.diag(ll[m]))
        assert np.abs(off).max() <= 1e-12 * scale[1], (tag, m)
        assert np.allclose(le[m], want_ld[m] * lm_mean[m], rtol=1e-8,
                           atol=1e-12 * scale[1] * (1 + np.abs(lm_mean[m]).max())), (tag, m)


def test_belief_phase_applies_the_prior_of_the_new_clock(oracle_mod):
    """Section 8: the priors start at the scale of the Jacobian information
    and are weakened to a hundredth over 10 iterations. The belief formed in
    iteration t (t = 1, 2, ...) carries the prior at clock t:
    base * 0.01^(min(t, 10)/10), mean at the initial estimate; the anchored
    keyframe keeps 1e8 I."""
    p = synth.make_config0(seed=13, n_lm=30)
    o = oracle_mod.Oracle(p, anneal=True)
    bk, bl = _prior_base(p, p.kf_init, p.lm_init, range(p.n_factors))
    anchored = p.kf_anchor_info > 0
    for t in range(0, 13):
        if t:
            o.iterate(1, damping=0.4)
        s = 0.01 ** (min(t, 10) / 10)
        want_kd = np.where(anchored[:, None], p.kf_anchor_info[:, None], bk * s)
        kl, ke, ll, le, sc = _belief_minus_messages(o, p.factor_kf, p.factor_lm)
        _check_prior(kl, ke, ll, le, sc, want_kd, bl * s, p.kf_init, p.lm_init,
                     range(p.n_keyframes), range(p.n_landmarks), t)


def test_unannealed_prior_is_constant(oracle_mod):
    """Without annealing (the FP64 configuration) the prior is the hundredth
    from the first iteration on."""
    p = synth.make_config0(seed=14, n_lm=20)
    o = oracle_mod.Oracle(p, anneal=False)
    bk, bl = _prior_base(p, p.kf_init, p.lm_init, range(p.n_factors))
    anchored = p.kf_anchor_info > 0
    want_kd = np.where(anchored[:, None], p.kf_anchor_info[:, None], bk * 0.01)
    for t in (1, 2, 5):
        o.iterate(1 if t != 5 else 3, damping=0.4)
        kl, ke, ll, le, sc = _belief_minus_messages(o, p.factor_kf, p.factor_lm)
        _check_prior(kl, ke, ll, le, sc, want_kd, bl * 0.01, p.kf_init, p.lm_init,
                     range(p.n_keyframes), range(p.n_landmarks), t)


def test_grown_variables_run_their_own_prior_clock(oracle_mod):
    """Section 9.2 growth: a keyframe and landmarks added at t = 7 get
    automatic priors from their new factors, Jacobians at the current means
    (new variables at their initial estimates), and anneal on a clock that
    starts at 7; the variables created at t = 0 keep their own clock."""
    p = synth.make_config0(seed=15, n_lm=30)
    nk, nl = p.n_keyframes, p.n_landmarks
    new_k, new_l = nk - 1, np.arange(nl - 5, nl)
    old_f = np.flatnonzero((p.factor_kf < new_k) & (p.factor_lm < nl - 5))
    new_f = np.setdiff1d(np.arange(p.n_factors), old_f)
    base = synth.BAProblem(
        "base", p.cam, p.kf_true[:new_k], p.lm_true[:nl - 5], p.kf_init[:new_k],
        p.lm_init[:nl - 5], p.factor_kf[old_f], p.factor_lm[old_f], p.z[old_f],
        p.z_true[old_f], p.inlier[old_f], p.kf_anchor_info[:new_k])
    o = oracle_mod.Oracle(base, anneal=True)
    o.iterate(7, damping=0.4)
    kf_mu, lm_mu = _means(o)
    kf_at = np.vstack([kf_mu, p.kf_init[new_k:]])
    lm_at = np.vstack([lm_mu, p.lm_init[nl - 5:]])
    # factors in the grown problem's order: the base factors, then the new
    order = np.concatenate([old_f, new_f])
    o.add(p.kf_init[new_k:], p.lm_init[nl - 5:], p.factor_kf[new_f], p.factor_lm[new_f], p.z[new_f])
    bk_old, bl_old = _prior_base(p, p.kf_init, p.lm_init, old_f)
    bk_new, bl_new = _prior_base(p, kf_at, lm_at, new_f)
    anchored = p.kf_anchor_info > 0
    for t in range(8, 21):
        o.iterate(1, damping=0.4)
        s_old = 0.01 ** (min(t, 10) / 10)
        s_new = 0.01 ** (min(t - 7, 10) / 10)
        want_kd = np.where(anchored[:, None], p.kf_anchor_info[:, None], bk_old * s_old)
        want_kd[new_k] = bk_new[new_k] * s_new
        want_ld = bl_old * s_old
        want_ld[new_l] = bl_new[new_l] * s_new
        kl, ke, ll, le, sc = _belief_minus_messages(o, p.factor_kf[order], p.factor_lm[order])
        _check_prior(kl, ke, ll, le, sc, want_kd, want_ld, p.kf_init, p.lm_init,
                     range(nk), range(nl), t)


@pytest.mark.parametrize("seed", [16, 17])
def test_annealed_and_unannealed_runs_reach_the_same_means(oracle_mod, seed):
    """Section 8: the strong initial priors are a help for the early
    iterations, not part of the answer. With forced relinearisation every
    10 iterations the annealed and the un-annealed runs become stationary at
    the same means (both end with the priors at a hundredth)."""
    p = synth.make_config0(seed=seed, n_lm=25)
    res = []
    for anneal in (True, False):
        o = oracle_mod.Oracle(p, anneal=anneal, huber_k=2.0)
        prev = None
        for _ in range(150):
            o.iterate(10, damping=0.4, huber_k=2.0)
            o.relinearise(-1)
            kf, lm = _means(o)
            cur = np.concatenate([kf.ravel(), lm.ravel()])
            if prev is not None and np.abs(cur - prev).max() < 1e-12:
                break
            prev = cur
        res.append(cur)
    a, b = res
    assert np.abs(a - b).max() < 1e-6 * max(1.0, np.abs(b).max())
    # the two runs did differ on the way (guards a test that cannot fail)
    o1 = oracle_mod.Oracle(p, anneal=True)
    o2 = oracle_mod.Oracle(p, anneal=False)
    o1.iterate(3, damping=0.4)
    o2.iterate(3, damping=0.4)
    assert np.abs(_means(o1)[1] - _means(o2)[1]).max() > 1e-6
