"""Learned per-factor damping: training data from the method's own GBP
trajectories, training of the network on the GPU, and the weight file.

The paper damps every message with one constant and names learned
components as future work (Section 5, Section 10). Here a small network
predicts, every few iterations, a damping value per factor from 16 features
of its state (gbp_factor_features). Damping leaves the fixed points of GBP
unchanged (Section 5), so the network can only change how fast the solver
gets there.

Labels. Messages are damped on the information vector: the stored message
after an update is (1 - d) eta_new + d eta_old. In the library's measurement
space the information vector of the message to variable v is carried by
h_v = g_v + S_v J_v a_v (gbp_factor_messages), which is damped the same way
while the factor keeps its linearisation. A training run with constant
damping d0 therefore recovers the undamped update h_new = (h_1 - d0 h_0) /
(1 - d0) from two consecutive iterations, and the damping that would have
put the message closest to where it is heading, h_T, is

    d* = clamp(<h_0 - h_new, h_T - h_new> / |h_0 - h_new|^2, 0, 0.9)

over both ends of the factor (4 numbers). Under the relinearisation rule a
moving factor is relinearised every few iterations (Section 8), which
changes the space its messages live in; h_T is therefore the factor's last
message before its next relinearisation (or the end of the run), at least
two iterations after the sample. The sample counts only when the factor was
inside its damped regime and its message still moved. The second head is
trained on log(converged depth / current depth) of the landmark in the
keyframe's frame.

Everything numeric here that the solver runs (features, messages, network
training) executes in the HIP library; the host only samples factor indices,
forms the labels from exported rows and shuffles the data.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import (GBP_DAMP_ETA, GBP_DAMP_ETA_LAMBDA, GBP_FP32, GBP_FP64, GBPError, GBPSolver, MLP_FEATURES,
               MLP_PARAMS, MLPTrainer, bf16_bits)
from ._capi import GBP_ENUMERIC

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "damping_mlp.npz")
D_MAX = 0.9
C_DELTA = 2.5


# ----------------------------------------------------------------------------
# weight file
# ----------------------------------------------------------------------------

def save_weights(path: str, theta: np.ndarray, meta: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    theta = np.asarray(theta, dtype=np.float32)
    np.savez(path, theta=theta, bf16=bf16_bits(theta), meta=np.array(json.dumps(meta, sort_keys=True)))


def load_weights(path: str = DEFAULT_WEIGHTS):
    """(bf16 bit patterns, float32 master weights, metadata dict)."""
    with np.load(path, allow_pickle=False) as z:
        bf16 = z["bf16"].astype(np.uint16)
        theta = z["theta"].astype(np.float32)
        meta = json.loads(str(z["meta"]))
    if bf16.shape != (MLP_PARAMS,):
        raise ValueError(f"{path}: expected {MLP_PARAMS} parameters")
    return bf16, theta, meta


# ----------------------------------------------------------------------------
# labels
# ----------------------------------------------------------------------------

def info_vectors(rows: np.ndarray) -> np.ndarray:
    """(n, 4) h = g + S J a of both message ends from gbp_factor_messages
    rows (S = [[a b][b c]] stored as a, b, c)."""
    r = rows.astype(np.float64)

    def side(s0, g0, j0):
        a, b, c = r[:, s0], r[:, s0 + 1], r[:, s0 + 2]
        j1, j2 = r[:, j0], r[:, j0 + 1]
        return np.stack([r[:, g0] + a * j1 + b * j2, r[:, g0 + 1] + b * j1 + c * j2], axis=1)

    return np.concatenate([side(0, 3, 12), side(5, 8, 14)], axis=1)


def damping_labels(m0, m1, mT, d0, horizon, undamped=1, min_horizon=2):
    """Best damping d* per sample and its weight (0 = no label); mT is the
    message `horizon` iterations after m0 under the same linearisation."""
    h0, h1, hT = info_vectors(m0), info_vectors(m1), info_vectors(mT)
    hnew = (h1 - d0 * h0) / (1.0 - d0)
    dv = h0 - hnew
    den = np.sum(dv * dv, axis=1)
    num = np.sum(dv * (hT - hnew), axis=1)
    c0, c1 = m0[:, 10], m1[:, 10]
    valid = (c0 >= undamped) & (c1 == c0 + 1) & (horizon >= min_horizon)
    # the change must stand clear of FP32 rounding of the exported rows
    valid &= den > (1e-11 * np.sum(h0 * h0, axis=1) + 1e-30)
    valid &= np.isfinite(num) & np.isfinite(den)
    d = np.where(valid, np.clip(num / np.where(den > 0, den, 1.0), 0.0, D_MAX), 0.0)
    return d.astype(np.float32), valid.astype(np.float32)


def _rotmats(omega: np.ndarray) -> np.ndarray:
    th = np.linalg.norm(omega, axis=1)
    k = omega / np.where(th > 0, th, 1.0)[:, None]
    K = np.zeros((omega.shape[0], 3, 3))
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -k[:, 2], k[:, 1], -k[:, 0]
    K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = k[:, 2], -k[:, 1], k[:, 0]
    s, c = np.sin(th)[:, None, None], np.cos(th)[:, None, None]
    return np.eye(3)[None] + s * K + (1.0 - c) * (K @ K)


def depths(kf_mean: np.ndarray, lm_mean: np.ndarray, fkf: np.ndarray, flm: np.ndarray) -> np.ndarray:
    R = _rotmats(kf_mean[fkf, :3])
    p = np.einsum("nij,nj->ni", R, lm_mean[flm]) + kf_mean[fkf, 3:]
    return p[:, 2]


# ----------------------------------------------------------------------------
# data generation
# ----------------------------------------------------------------------------

class _Pending:
    """Factors sampled at one iteration, followed until they relinearise."""

    def __init__(self, t0, idx, x, m0, dep):
        import torch
        self.t0, self.idx, self.x, self.dep = t0, idx, x, dep
        self.m0 = m0
        self.m1 = None
        self.last = m0.clone()
        self.last_t = torch.full((m0.shape[0],), t0, dtype=torch.int32, device=m0.device)
        self.alive = torch.ones(m0.shape[0], dtype=torch.bool, device=m0.device)
        self.c0 = m0[:, 10]

    def update(self, t, rows):
        # same linearisation iff the update counter advanced every iteration
        # (counters saturate at 255: stop following before that)
        same = self.alive & (rows[:, 10] == self.c0 + float(t - self.t0)) & (self.c0 + float(t - self.t0) < 255)
        self.last[same] = rows[same]
        self.last_t[same] = t
        self.alive = same
        if t == self.t0 + 1:
            self.m1 = rows.clone()


def generate(problems, *, iters=300, every=5, frac=0.05, damping=0.4, huber_k=2.0, seed=0,
             follow=30, undamped=1, damp_mode=GBP_DAMP_ETA_LAMBDA, depth_label="converged", log=print):
    """Run plain GBP (FP32, constant damping) on a batch of problems and
    return features X (n, 16), labels Y (n, 2) and weights M (n, 2) of a
    random `frac` of the factors at every `every`-th iteration; each sample
    is followed for up to `follow` iterations for its damping label. The
    generating run damps every update but the relinearising one
    (undamped=1), so that almost every sampled update reveals its undamped
    value, and damps information and vector together (both stay
    interpolations, which keeps the run stable on large graphs; the
    information vector, and with it h, is damped linearly either way).
    depth_label: "converged" takes the depth head's label from the run's
    final beliefs, "truth" from the problems' true poses and points (a
    landmark started far from its depth can converge to a wrong depth)."""
    solver = GBPSolver(problems, precision=GBP_FP32, undamped=undamped, damp_mode=damp_mode)
    done = []
    try:
        nf = int(sum(solver.f_counts))
        kf_off = np.concatenate([[0], np.cumsum(solver.kf_counts)[:-1]])
        lm_off = np.concatenate([[0], np.cumsum(solver.lm_counts)[:-1]])
        fkf = np.concatenate([np.asarray(p.factor_kf) + o for p, o in zip(problems, kf_off)])
        flm = np.concatenate([np.asarray(p.factor_lm) + o for p, o in zip(problems, lm_off)])
        rng = np.random.default_rng(seed)
        pending = []
        for t in range(iters + 1):
            assert solver.t == t
            keep = []
            for P in pending:
                P.update(t, solver.factor_messages(P.idx))
                if t - P.t0 >= follow or t == iters:
                    done.append(P)
                else:
                    keep.append(P)
            pending = keep
            if t % every == 0 and t + 1 < iters:
                idx = np.sort(rng.choice(nf, size=max(1, int(frac * nf)), replace=False)).astype(np.int32)
                x = solver.factor_features(idx).cpu().numpy()
                m0 = solver.factor_messages(idx)
                b = solver.beliefs()
                pending.append(_Pending(t, idx, x, m0, depths(b["kf_mu"], b["lm_mu"], fkf[idx], flm[idx])))
            if t < iters:
                solver.iterate(1, damping, huber_k)
        if depth_label == "truth":
            depT_all = depths(np.concatenate([p.kf_true for p in problems]),
                              np.concatenate([p.lm_true for p in problems]), fkf, flm)
        else:
            b = solver.beliefs()
            depT_all = depths(b["kf_mu"], b["lm_mu"], fkf, flm)
    finally:
        solver.close()
    X, Y, M = [], [], []
    for P in done:
        m0, m1, mT = P.m0.cpu().numpy(), P.m1.cpu().numpy(), P.last.cpu().numpy()
        horizon = P.last_t.cpu().numpy() - P.t0
        d, wd = damping_labels(m0, m1, mT, damping, horizon, undamped=undamped)
        dep, dT = P.dep, depT_all[P.idx]
        ok = (dep > 0.05) & (dT > 0.05) & np.isfinite(dep) & np.isfinite(dT)
        delta = np.where(ok, np.clip(np.log(np.where(ok, dT, 1.0) / np.where(ok, dep, 1.0)), -C_DELTA, C_DELTA), 0.0)
        good = np.all(np.isfinite(P.x), axis=1)
        X.append(P.x[good])
        Y.append(np.stack([d, delta], axis=1)[good].astype(np.float32))
        M.append(np.stack([wd, ok.astype(np.float32)], axis=1)[good])
    X, Y, M = np.concatenate(X), np.concatenate(Y), np.concatenate(M)
    lab = M[:, 0] > 0
    log(f"[learned] {len(problems)} problems, {nf} factors, {X.shape[0]} samples, "
        f"damping labels {int(lab.sum())} (mean d* {Y[lab, 0].mean() if lab.any() else float('nan'):.3f}, "
        f"share at 0: {np.mean(Y[lab, 0] == 0.0) if lab.any() else float('nan'):.3f}, "
        f"at 0.9: {np.mean(Y[lab, 0] == D_MAX) if lab.any() else float('nan'):.3f})")
    return X, Y, M


# ----------------------------------------------------------------------------
# training
# ----------------------------------------------------------------------------

def fold_standardisation(theta: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """Parameters acting on raw features from parameters trained on
    (x - mu) / sd: W1' = W1 / sd, b1' = b1 - W1' mu."""
    th = theta.astype(np.float64).copy()
    W1 = th[:MLP_FEATURES * 64].reshape(64, MLP_FEATURES)
    b1 = th[MLP_FEATURES * 64:MLP_FEATURES * 64 + 64]
    W1n = W1 / sd[None, :]
    b1n = b1 - W1n @ mu
    th[:MLP_FEATURES * 64] = W1n.ravel()
    th[MLP_FEATURES * 64:MLP_FEATURES * 64 + 64] = b1n
    return th.astype(np.float32)


def train(X, Y, M, *, epochs=6, batch=4096, lr=2e-3, seed=0, val_frac=0.1, log=print):
    """Adam on the GPU (gbp_mlp_train_step); returns raw-feature parameters
    and a training report."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    perm = rng.permutation(n)
    n_val = max(1, int(val_frac * n))
    val, tr = perm[:n_val].astype(np.int32), perm[n_val:].astype(np.int32)
    mu = X[tr].mean(axis=0).astype(np.float64)
    sd = X[tr].std(axis=0).astype(np.float64)
    sd = np.where(sd > 1e-6, sd, 1.0)
    Xs = ((X - mu) / sd).astype(np.float32)
    tr_ = MLPTrainer(max_batch=batch, seed=seed)
    tr_.set_data(Xs, Y, M)

    def val_loss():
        tot = 0.0
        for i in range(0, n_val, batch):
            chunk = val[i:i + batch]
            _, l = tr_.gradient(chunk)
            tot += l * chunk.shape[0]
        return tot / n_val

    l0 = val_loss()
    hist = [l0]
    steps_per_epoch = max(1, tr.shape[0] // batch)
    total = epochs * steps_per_epoch
    k = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = tr[rng.permutation(tr.shape[0])]
        for s in range(steps_per_epoch):
            # cosine decay of the learning rate
            lr_k = lr * 0.5 * (1.0 + np.cos(np.pi * k / total))
            tr_.step(order[s * batch:(s + 1) * batch], lr_k)
            k += 1
        hist.append(val_loss())
        log(f"[learned] epoch {ep + 1}/{epochs}: validation loss {hist[-1]:.5f} (start {l0:.5f})")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    theta = fold_standardisation(tr_.theta_host(), mu, sd)
    report = dict(samples=int(n), train=int(tr.shape[0]), val=int(n_val), epochs=epochs, batch=batch,
                  lr=lr, steps=k, val_loss=[float(v) for v in hist], train_seconds=secs)
    return theta, report


# ----------------------------------------------------------------------------
# evaluation: time to target, plain against learned damping
# ----------------------------------------------------------------------------

def time_to_target(problem, *, weights=None, every_k=5, damping=0.4, huber_k=2.0, target=1.0,
                   max_iters=300, fallback_rise=0.5, damp_mode=GBP_DAMP_ETA, judge=False):
    """Plain (weights None) or learned GBP on one problem (FP32): the first
    iteration at which the mean error of inliers against their noise-free
    projections is <= target px, and the GPU time to get there. The full
    run is made twice: the first records the iteration graph, the second
    (after gbp_reset) is timed as one replay with the error logged on the
    device every iteration (its per-iteration time, model evaluations
    included, is `ms_per_iter`) and finds the first iteration at target.
    Then exactly that many iterations are run from the start once more to
    record their graph, and once more timed with HIP events on the solver's
    stream (`ms`: launch to the logged error of the hit, on the device).
    judge: the learned run carries its plain-GBP judge (the same problem
    with the constant damping) in the same launches, and its fallback
    compares with that run's error (gbp_set_damping_judges)."""
    import torch
    probs = [problem, problem] if judge else problem
    s = GBPSolver(probs, precision=GBP_FP32, damp_mode=damp_mode)
    try:
        n = 2 if judge else 1
        s.set_reference(np.concatenate([problem.z_true] * n), np.concatenate([problem.inlier] * n))
        if weights is not None:
            s.set_damping_model(weights, every_k=every_k, fallback_rise=fallback_rise)
            if judge:
                s.set_damping_judges([1, -1])
        s.iterate_logged(max_iters, damping, huber_k, log_every=1)
        s.reset()
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        log = s.iterate_logged(max_iters, damping, huber_k, log_every=1)
        wall = time.perf_counter() - t0
        fb = int(s.fallback_flags()[0])
        are_ref, are_all = log[:, 0, 2], log[:, 0, 1]
        hit = np.nonzero(are_ref <= target)[0]
        it = int(hit[0]) + 1 if hit.size else None
        ms_hit = None
        if it is not None:
            s.reset()
            s.iterate_logged(it, damping, huber_k, log_every=1)
            s.reset()
            s.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            again = s.iterate_logged(it, damping, huber_k, log_every=1)
            e1.record(s.stream)
            e1.synchronize()
            ms_hit = e0.elapsed_time(e1)
            if not np.array_equal(again[:, 0, 2], are_ref[:it]):
                raise RuntimeError("time_to_target: the timed rerun did not repeat the logged run")
    finally:
        s.close()
    marks = [i for i in (1, 2, 5, 10, 20, 50, 100, 200, 300, 400, 600) if i <= max_iters]
    return dict(iterations=it, ms=ms_hit,
                ms_per_iter=wall * 1e3 / max_iters, final_are_ref=float(are_ref[-1]),
                final_are_all=float(are_all[-1]), fallback=fb, max_iters=max_iters,
                damping=damping, damp_mode=int(damp_mode), judged=bool(judge),
                are_ref_at={i: round(float(are_ref[i - 1]), 4) for i in marks})


def incremental_run(stream, *, weights=None, use_depth=False, every_k=5, damping=0.4, huber_k=2.0,
                    iters_per_kf=20, depth_delay=5, target=1.0, fallback_rise=0.5, damp_mode=GBP_DAMP_ETA,
                    trace=False, precision=GBP_FP64):
    """The SLAM protocol of Section 9.2 on an incremental stream: start from
    the base problem, and for every later keyframe add it (initialised at
    the previous keyframe's current estimate) with its new landmarks and
    factors, then run `iters_per_kf` iterations. With `use_depth` the
    learned depth head moves the new landmarks (and, in the first window,
    the base problem's) `depth_delay` iterations after they join. Returns per-addition iterations to the inlier target,
    final errors and the GPU wall time of the whole run (host work for the
    additions included). FP64 factor state by default: the beliefs of a long,
    unconverged chain become too ill-conditioned for FP32 messages."""
    import torch
    full, base = stream.full, stream.base
    cap = (full.n_keyframes, full.n_landmarks, full.n_factors)
    s = GBPSolver(base, precision=precision, capacity=cap, damp_mode=damp_mode, anneal=True)
    try:
        if weights is not None:
            s.set_damping_model(weights, every_k=every_k, fallback_rise=fallback_rise)
        nb = base.n_landmarks
        step_lms = [st["lm"] for st in stream.steps]
        base_ids = sorted(set(range(full.n_landmarks)) - set(np.concatenate(step_lms).tolist()))
        user_of = {int(j): i for i, j in enumerate(base_ids)}
        # caller order of the grown factor set: the base factors, then each
        # step's factors in arrival order
        base_f = np.flatnonzero(np.isin(full.factor_lm, np.array(base_ids)))
        forder = [base_f]
        s.set_reference(full.z_true[base_f], full.inlier[base_f])
        n_lm = nb
        to_target, final_ref = [], []
        diverged_at = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if use_depth and weights is not None:
            s.iterate(depth_delay, damping, huber_k)
            s.apply_depth_model(np.arange(nb, dtype=np.int32))
            s.iterate(iters_per_kf - depth_delay, damping, huber_k)
        else:
            s.iterate(iters_per_kf, damping, huber_k)
        for st in stream.steps:
            try:
                pose = s.beliefs()["kf_mu"][st["kf"] - 1].copy()
            except GBPError as e:
                if e.status != GBP_ENUMERIC:
                    raise
                diverged_at = int(st["kf"])  # a belief lost positive definiteness
                break
            new_users = []
            for j in st["lm"]:
                user_of[int(j)] = n_lm
                new_users.append(n_lm)
                n_lm += 1
            fs = st["factors"]
            flm = np.array([user_of[int(j)] for j in full.factor_lm[fs]], dtype=np.int32)
            s.add_keyframe(pose, full.lm_init[st["lm"]], full.factor_kf[fs], flm, full.z[fs])
            forder.append(fs)
            allf = np.concatenate(forder)
            s.set_reference(full.z_true[allf], full.inlier[allf])
            if use_depth and weights is not None and new_users:
                a = s.iterate_logged(depth_delay, damping, huber_k, log_every=1)
                s.apply_depth_model(np.array(new_users, dtype=np.int32))
                b = s.iterate_logged(iters_per_kf - depth_delay, damping, huber_k, log_every=1)
                log = np.concatenate([a, b])
            else:
                log = s.iterate_logged(iters_per_kf, damping, huber_k, log_every=1)
            ref = log[:, 0, 2]
            hit = np.nonzero(ref <= target)[0]
            to_target.append(int(hit[0]) + 1 if hit.size else None)
            final_ref.append(float(ref[-1]))
        s.synchronize()
        wall = time.perf_counter() - t0
        fb = int(s.fallback_flags()[0])
        last = s.reproj() if diverged_at is None else dict(are_ref=float("nan"), are_all=float("nan"))
    finally:
        s.close()
    reached = [v for v in to_target if v is not None]
    extra = dict(final_are_ref_per_addition=[round(v, 3) for v in final_ref]) if trace else {}
    return dict(additions=len(to_target), reached=len(reached), diverged_at_keyframe=diverged_at, **extra,
                mean_iters_to_target=float(np.mean(reached)) if reached else None,
                mean_final_are_ref=float(np.mean(final_ref)), last_are_ref=float(last["are_ref"]),
                last_are_all=float(last["are_all"]), wall_s=wall, fallback=fb,
                iterations=iters_per_kf * (len(to_target) + 1))


def compare(problem, weights, *, undamped_too=False, **kw) -> dict:
    """Time to target of plain GBP as the paper runs it (damping 0.4 on the
    information vector), of the learned damping (its own error history as
    fallback rule) and of the learned damping with its plain-GBP judge in the
    same launches; with undamped_too also plain GBP undamped and with
    information and vector damped, and the learned damping under the latter.
    speedup: against the paper's plain run; speedup_vs_best_plain: against
    the fastest plain variant measured (None when a run misses the target)."""
    plain = time_to_target(problem, weights=None, **kw)
    learned = time_to_target(problem, weights=weights, **kw)
    judged = time_to_target(problem, weights=weights, judge=True, **kw)
    sp = (plain["ms"] / learned["ms"]) if plain["ms"] and learned["ms"] else None
    out = dict(plain=plain, learned=learned, learned_judged=judged, speedup=sp)
    if undamped_too:
        out["plain_undamped"] = time_to_target(problem, weights=None, **dict(kw, damping=0.0))
        out["plain_damp_both"] = time_to_target(problem, weights=None,
                                                **dict(kw, damp_mode=GBP_DAMP_ETA_LAMBDA))
        out["learned_damp_both"] = time_to_target(problem, weights=weights,
                                                  **dict(kw, damp_mode=GBP_DAMP_ETA_LAMBDA))
    plains = {k: v for k, v in out.items() if k.startswith("plain") and v["ms"]}
    if plains:
        best = min(plains, key=lambda k: plains[k]["ms"])
        out["best_plain"] = best
        out["speedup_vs_best_plain"] = (plains[best]["ms"] / learned["ms"]) if learned["ms"] else None
        out["judged_speedup_vs_best_plain"] = (plains[best]["ms"] / judged["ms"]) if judged["ms"] else None
    return out


# ----------------------------------------------------------------------------
# command line
# ----------------------------------------------------------------------------

def main(argv=None):
    import synth
    ap = argparse.ArgumentParser(description="generate GBP trajectories and train the damping network")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--problems", type=int, default=128)
    ap.add_argument("--batch-problems", type=int, default=64)
    ap.add_argument("--large", type=int, default=0, help="1000-keyframe problems added to the data")
    ap.add_argument("--mixed", type=int, default=0, help="uneven batched problems added to the data")
    ap.add_argument("--depth-init", type=int, default=0,
                    help="125-keyframe problems with landmarks started at 1 m depth added to the data")
    ap.add_argument("--eval-incremental", type=int, default=0,
                    help="also the incremental run up to this many keyframes")
    ap.add_argument("--incremental-precision", default="fp64", choices=["fp32", "fp64"],
                    help="factor state of the incremental runs")
    ap.add_argument("--incremental-seed", type=int, default=20000)
    ap.add_argument("--seed0", type=int, default=10000)
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--frac", type=float, default=0.05)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--depth-label", default="converged", choices=["converged", "truth"],
                    help="label of the depth head: the run's converged depth or the true depth")
    ap.add_argument("--eval", action="store_true", help="compare plain and learned damping instead")
    ap.add_argument("--eval-seeds", default="1,2,3,4")
    ap.add_argument("--eval-large", action="store_true", help="also the 1000-keyframe problem")
    a = ap.parse_args(argv)
    if a.eval:
        w, _, _ = load_weights(a.out)
        out = {}
        for sd in [int(v) for v in a.eval_seeds.split(",")]:
            out[f"random_walk_125kf_seed{sd}"] = compare(synth.make_config1(sd), w, undamped_too=True)
            print(json.dumps({f"seed{sd}": out[f"random_walk_125kf_seed{sd}"]}), flush=True)
        if a.eval_incremental:
            prec = GBP_FP64 if a.incremental_precision == "fp64" else GBP_FP32
            for tag, init in (("landmarks_at_1m", 1.0), ("landmarks_noisy", None)):
                st = synth.make_incremental_stream(seed=a.incremental_seed, n_kf=a.eval_incremental, init_depth=init)
                res = {"plain": incremental_run(st, precision=prec),
                       "plain_damp_both": incremental_run(st, damp_mode=GBP_DAMP_ETA_LAMBDA, precision=prec),
                       "learned_damping": incremental_run(st, weights=w, precision=prec),
                       "learned_damping_and_depth": incremental_run(st, weights=w, use_depth=True, precision=prec)}
                out[f"incremental_{tag}"] = res
                print(json.dumps({f"incremental_{tag}": res}), flush=True)
        if a.eval_large:
            out["random_walk_1000kf"] = compare(synth.make_config2(), w, max_iters=400, undamped_too=True)
            print(json.dumps({"large": out["random_walk_1000kf"]}), flush=True)
        return
    t0 = time.perf_counter()
    parts = []
    for b0 in range(0, a.problems, a.batch_problems):
        seeds = range(a.seed0 + b0, a.seed0 + min(a.problems, b0 + a.batch_problems))
        probs = [synth.make_config1(s) for s in seeds]
        parts.append(generate(probs, iters=a.iters, every=a.every, frac=a.frac, seed=b0,
                              depth_label=a.depth_label))
    for i in range(a.large):
        parts.append(generate([synth.make_config2(a.seed0 + 5000 + i)], iters=a.iters, every=a.every,
                              frac=a.frac, seed=5000 + i, depth_label=a.depth_label))
    for b0 in range(0, a.depth_init, a.batch_problems):
        probs = [synth.reinit_at_depth(synth.make_config1(a.seed0 + 9000 + i))
                 for i in range(b0, min(a.depth_init, b0 + a.batch_problems))]
        parts.append(generate(probs, iters=a.iters, every=a.every, frac=a.frac, seed=9000 + b0,
                              depth_label=a.depth_label))
    for b0 in range(0, a.mixed, a.batch_problems):
        probs = [synth.make_config3_problem(p, base_seed=a.seed0 + 7000)
                 for p in range(b0, min(a.mixed, b0 + a.batch_problems))]
        parts.append(generate(probs, iters=a.iters, every=a.every, frac=a.frac, seed=7000 + b0,
                              depth_label=a.depth_label))
    X = np.concatenate([p[0] for p in parts])
    Y = np.concatenate([p[1] for p in parts])
    M = np.concatenate([p[2] for p in parts])
    t_gen = time.perf_counter() - t0
    theta, rep = train(X, Y, M, epochs=a.epochs, lr=a.lr)
    meta = dict(problems=a.problems, seeds=[a.seed0, a.seed0 + a.problems - 1], iters=a.iters,
                every=a.every, frac=a.frac, damping=0.4, generator="125 keyframes / 1919 landmarks random walk",
                large_problems=a.large, mixed_problems=a.mixed, depth_init_problems=a.depth_init,
                depth_label=a.depth_label,
                label_mean_damping=float(Y[M[:, 0] > 0, 0].mean()), data_seconds=t_gen, **rep)
    save_weights(a.out, theta, meta)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
