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
put the message closest to its converged value h_T is

    d* = clamp(<h_0 - h_new, h_T - h_new> / |h_0 - h_new|^2, 0, 0.9)

over both ends of the factor (4 numbers). The sample counts only when the
factor was inside its damped regime, kept its linearisation from the sample
to the end of the run, and its message still moved. The second head is
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

from . import (GBP_FP32, GBPSolver, MLP_FEATURES, MLP_PARAMS, MLPTrainer, bf16_bits)

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


def damping_labels(m0, m1, mT, d0, t, T, undamped=8):
    """Best damping d* per sample and its weight (0 = no label)."""
    h0, h1, hT = info_vectors(m0), info_vectors(m1), info_vectors(mT)
    hnew = (h1 - d0 * h0) / (1.0 - d0)
    dv = h0 - hnew
    den = np.sum(dv * dv, axis=1)
    num = np.sum(dv * (hT - hnew), axis=1)
    c0, c1, cT = m0[:, 10], m1[:, 10], mT[:, 10]
    steps_left = T - (t + 1)
    valid = (c0 >= undamped) & (c0 < 254) & (c1 == c0 + 1)
    valid &= (cT == np.minimum(255, c1 + steps_left))
    valid &= den > (1e-8 * np.sum(h0 * h0, axis=1) + 1e-30)
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

def generate(problems, *, iters=300, every=5, frac=0.05, damping=0.4, huber_k=2.0, seed=0,
             log=print):
    """Run plain GBP (FP32, constant damping) on a batch of problems and
    return features X (n, 16), labels Y (n, 2) and weights M (n, 2) of a
    random `frac` of the factors at every `every`-th iteration."""
    solver = GBPSolver(problems, precision=GBP_FP32)
    try:
        nf = int(sum(solver.f_counts))
        kf_off = np.concatenate([[0], np.cumsum(solver.kf_counts)[:-1]])
        lm_off = np.concatenate([[0], np.cumsum(solver.lm_counts)[:-1]])
        fkf = np.concatenate([np.asarray(p.factor_kf) + o for p, o in zip(problems, kf_off)])
        flm = np.concatenate([np.asarray(p.factor_lm) + o for p, o in zip(problems, lm_off)])
        rng = np.random.default_rng(seed)
        recs = []
        for t in range(0, iters - every + 1, every):
            assert solver.t == t
            idx = np.sort(rng.choice(nf, size=max(1, int(frac * nf)), replace=False)).astype(np.int32)
            x = solver.factor_features(idx).cpu().numpy()
            m0 = solver.factor_messages(idx).cpu().numpy()
            b = solver.beliefs()
            dep = depths(b["kf_mu"], b["lm_mu"], fkf[idx], flm[idx])
            solver.iterate(1, damping, huber_k)
            m1 = solver.factor_messages(idx).cpu().numpy()
            solver.iterate(every - 1, damping, huber_k)
            recs.append((t, idx, x, m0, m1, dep))
        if solver.t < iters:
            solver.iterate(iters - solver.t, damping, huber_k)
        T = solver.t
        mT = solver.factor_messages(np.arange(nf, dtype=np.int32)).cpu().numpy()
        b = solver.beliefs()
        depT_all = depths(b["kf_mu"], b["lm_mu"], fkf, flm)
    finally:
        solver.close()
    X, Y, M = [], [], []
    for t, idx, x, m0, m1, dep in recs:
        d, wd = damping_labels(m0, m1, mT[idx], damping, t, T)
        dT = depT_all[idx]
        ok = (dep > 0.05) & (dT > 0.05) & np.isfinite(dep) & np.isfinite(dT)
        delta = np.where(ok, np.clip(np.log(np.where(ok, dT, 1.0) / np.where(ok, dep, 1.0)), -C_DELTA, C_DELTA), 0.0)
        good = np.all(np.isfinite(x), axis=1)
        X.append(x[good])
        Y.append(np.stack([d, delta], axis=1)[good].astype(np.float32))
        M.append(np.stack([wd, ok.astype(np.float32)], axis=1)[good])
    X, Y, M = np.concatenate(X), np.concatenate(Y), np.concatenate(M)
    log(f"[learned] {len(problems)} problems, {nf} factors, {X.shape[0]} samples, "
        f"damping labels {int(M[:, 0].sum())} (mean d* {Y[M[:, 0] > 0, 0].mean():.3f})")
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
# command line
# ----------------------------------------------------------------------------

def main(argv=None):
    import synth
    ap = argparse.ArgumentParser(description="generate GBP trajectories and train the damping network")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--problems", type=int, default=128)
    ap.add_argument("--batch-problems", type=int, default=64)
    ap.add_argument("--seed0", type=int, default=10000)
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--frac", type=float, default=0.05)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    parts = []
    for b0 in range(0, a.problems, a.batch_problems):
        seeds = range(a.seed0 + b0, a.seed0 + min(a.problems, b0 + a.batch_problems))
        probs = [synth.make_config1(s) for s in seeds]
        parts.append(generate(probs, iters=a.iters, every=a.every, frac=a.frac, seed=b0))
    X = np.concatenate([p[0] for p in parts])
    Y = np.concatenate([p[1] for p in parts])
    M = np.concatenate([p[2] for p in parts])
    t_gen = time.perf_counter() - t0
    theta, rep = train(X, Y, M, epochs=a.epochs, lr=a.lr)
    meta = dict(problems=a.problems, seeds=[a.seed0, a.seed0 + a.problems - 1], iters=a.iters,
                every=a.every, frac=a.frac, damping=0.4, generator="125 keyframes / 1919 landmarks random walk",
                label_mean_damping=float(Y[M[:, 0] > 0, 0].mean()), data_seconds=t_gen, **rep)
    save_weights(a.out, theta, meta)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
