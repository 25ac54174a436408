"""Robustness and robust-loss studies of the evaluation (Sections 9.3 and
9.4), each run as batched launches of the GPU path.

basin(): the convergence basin (Section 9.3, Fig. 5). For every keyframe
initialisation noise level, `trials` problems run as one block-diagonal
batch; a trial succeeds when its average reprojection error over all
measurements falls below 1.5 px within the iteration budget. The trials
keep their geometry and noise directions at every level (only the noise
scale changes), so the levels differ in the noise alone. Plain GBP and,
optionally, the learned damping model.

outliers(): outlier classification (Section 9.4, Fig. 7a). A measurement is
classed an outlier while it lies in the linear Huber regime; against the
generator's record of which measurements are bad this gives precision and
recall at every iteration, logged on the device with no host round trip.

huber_ablation(): the error reached with and without the Huber loss over a
range of bad-association fractions (Section 9.4, Fig. 7b).

Inputs are seeded synthetic stand-ins for the TUM sequences the paper uses:
30 keyframes with landmark counts scaled from Table 1 (fr1desk: 63
keyframes, 2913 points; fr3teddy: 125 keyframes, 1919 points) and about 4.6
observations per point, and a 20-keyframe fr1desk-sized sequence for the
outlier studies. A bad data association is a measurement replaced by a
pixel drawn uniformly over the image.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import GBPSolver, GBP_FP32

# 30-keyframe sequences of the basin study (Fig. 5)
SEQUENCES = {
    "fr1desk30": dict(n_kf=30, n_lm=1390, seed0=30000),
    "fr3teddy30": dict(n_kf=30, n_lm=460, seed0=31000),
}
# 20-keyframe fr1desk-sized sequence of the outlier studies (Fig. 7)
OUTLIER_SEQ = dict(n_kf=20, n_lm=925, seed0=32000)
TARGET_PX = 1.5


def basin_problem(seq: str, noise_m: float, trial: int):
    """Trial `trial` of sequence `seq` with keyframe camera centres perturbed
    by N(0, noise_m^2) per axis (orientations exact, landmarks N(0, 0.1 m))."""
    import synth
    q = SEQUENCES[seq]
    return synth.make_random_walk(f"{seq}_t{trial}", q["seed0"] + trial, q["n_kf"], q["n_lm"],
                                  "sparse", 0.0, min_obs=2, centre_sigma=noise_m)


def outlier_problem(frac: float, trial: int):
    import synth
    q = OUTLIER_SEQ
    return synth.make_random_walk(f"out_t{trial}", q["seed0"] + trial, q["n_kf"], q["n_lm"],
                                  "sparse", frac, min_obs=2)


def first_below(series: np.ndarray, target: float) -> np.ndarray:
    """[rows, trials] -> 1-based first row with a value < target (0: never)."""
    hit = series < target
    first = np.argmax(hit, axis=0) + 1
    return np.where(hit.any(axis=0), first, 0)


def run_batch(problems, *, iters: int, damping: float = 0.4, huber_k: float = 2.0,
              precision: int = GBP_FP32, weights=None, every_k: int = 5, fallback_rise: float = 0.5,
              reference: str | None = None, log_every: int = 1):
    """One batched run; returns the device log [iters // log_every, trials,
    5] and the wall time of the logged iterations. reference "measured"
    sets each problem's own measurements over its inliers as the reference
    (are_ref = inlier error; n_linear_ref = inliers classed outliers)."""
    import torch
    # the threshold applies from the creation-time linearisation on
    s = GBPSolver(problems, precision=precision, huber_k=huber_k)
    try:
        if reference == "measured":
            s.set_reference(np.concatenate([p.z for p in problems]),
                            np.concatenate([p.inlier for p in problems]))
        if weights is not None:
            s.set_damping_model(weights, every_k=every_k, fallback_rise=fallback_rise)
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        log = s.iterate_logged(iters, damping, huber_k, log_every=log_every)
        wall = time.perf_counter() - t0
        fb = s.fallback_flags() if weights is not None else None
    finally:
        s.close()
    return log, wall, fb


def basin(levels=(0.05, 0.1, 0.15, 0.2, 0.3, 0.4), trials: int = 100, seqs=tuple(SEQUENCES),
          iters: int = 300, learned: bool = False, precision: int = GBP_FP32, log_every: int = 5) -> list:
    """Success rate (average error < 1.5 px reached within `iters`) per
    sequence and keyframe-noise level, plain and, with learned=True, with the
    packaged damping model too."""
    weights = None
    if learned:
        from .learned import load_weights
        weights = load_weights()[0]
    out = []
    for seq in seqs:
        for sigma in levels:
            probs = [basin_problem(seq, sigma, t) for t in range(trials)]
            nf = sum(p.n_factors for p in probs)
            variants = [("plain", None)] + ([("learned", weights)] if learned else [])
            for name, w in variants:
                log, wall, fb = run_batch(probs, iters=iters, precision=precision, weights=w,
                                          log_every=log_every)
                are = log[:, :, 1]
                first = first_below(are, TARGET_PX)
                ok = first > 0
                row = dict(sequence=seq, noise_m=sigma, damping=name, trials=trials, iters=iters,
                           success=float(ok.mean()), final_success=float((are[-1] < TARGET_PX).mean()),
                           median_iters_to_target=(float(np.median(first[ok])) * log_every if ok.any() else None),
                           median_final_are=float(np.median(are[-1])), factors=int(nf),
                           wall_s=round(wall, 4), ms_per_iter=round(wall * 1e3 / iters, 4),
                           factor_updates_per_s=nf * iters / wall)
                if fb is not None:
                    row["fallback"] = int(np.asarray(fb).sum())
                out.append(row)
                print(json.dumps(row), flush=True)
    return out


def classification(log: np.ndarray, n_outliers: np.ndarray) -> dict:
    """Precision and recall of 'linear Huber regime = bad measurement' per
    logged row, summed over the batch and for its first trial alone. A row
    holds n_linear (all classed outliers) and n_linear_ref (inliers classed
    outliers), so true positives are their difference."""
    n_lin, fp = log[:, :, 3], log[:, :, 4]
    tp = n_lin - fp
    with np.errstate(invalid="ignore", divide="ignore"):
        prec_all = tp.sum(1) / n_lin.sum(1)
        rec_all = tp.sum(1) / n_outliers.sum()
        prec_0 = tp[:, 0] / n_lin[:, 0]
        rec_0 = tp[:, 0] / n_outliers[0]
    return dict(precision=prec_all, recall=rec_all, precision_trial0=prec_0, recall_trial0=rec_0,
                are_inliers=log[:, :, 2].mean(1), are_inliers_trial0=log[:, 0, 2])


def outliers(frac: float = 0.03, trials: int = 16, iters: int = 300, huber_k: float = 2.0,
             precision: int = GBP_FP32) -> dict:
    """Outlier classification over the iterations (Fig. 7a)."""
    probs = [outlier_problem(frac, t) for t in range(trials)]
    n_out = np.array([int((~p.inlier).sum()) for p in probs])
    log, wall, _ = run_batch(probs, iters=iters, huber_k=huber_k, precision=precision, reference="measured")
    c = classification(log, n_out)
    marks = [i for i in (1, 2, 5, 10, 20, 50, 100, 150, 200, 250, 300, 400, 500) if i <= iters]
    first = first_below(log[:, :, 2], TARGET_PX)
    res = dict(frac=frac, trials=trials, iters=iters, huber_k=huber_k, outliers=int(n_out.sum()),
               factors=int(sum(p.n_factors for p in probs)), wall_s=round(wall, 4),
               iters_to_inlier_are_below_1p5=[int(v) for v in first],
               at={i: dict(precision=round(float(c["precision"][i - 1]), 4),
                           recall=round(float(c["recall"][i - 1]), 4),
                           are_inliers=round(float(c["are_inliers"][i - 1]), 4)) for i in marks})
    print(json.dumps(res), flush=True)
    return res


def huber_ablation(fracs=(0.0, 0.01, 0.03, 0.05, 0.1), trials: int = 8, iters: int = 400,
                   huber_k: float = 2.0, precision: int = GBP_FP32) -> list:
    """Inlier error after `iters` iterations with the Huber loss (threshold
    huber_k px) and without it (threshold 0: every measurement quadratic),
    per bad-association fraction (Fig. 7b)."""
    out = []
    for frac in fracs:
        probs = [outlier_problem(frac, t) for t in range(trials)]
        for k in (huber_k, 0.0):
            log, wall, _ = run_batch(probs, iters=iters, huber_k=k, precision=precision,
                                     reference="measured", log_every=10)
            are = log[:, :, 2]
            fin = are[-1]
            row = dict(frac=frac, huber_k=k, trials=trials, iters=iters,
                       mean_final_are_inliers=float(np.nanmean(fin)),
                       median_final_are_inliers=float(np.nanmedian(fin)),
                       converged=float((fin < TARGET_PX).mean()), wall_s=round(wall, 4))
            out.append(row)
            print(json.dumps(row), flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="convergence-basin and Huber studies on the GPU")
    ap.add_argument("study", choices=("basin", "outliers", "huber", "all"))
    ap.add_argument("--trials", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--learned", action="store_true", help="basin: also the learned damping model")
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    a = ap.parse_args(argv)
    kw = {k: v for k, v in (("trials", a.trials), ("iters", a.iters)) if v is not None}
    res = {}
    t0 = time.perf_counter()
    if a.study in ("basin", "all"):
        res["basin"] = basin(learned=a.learned, **kw)
    if a.study in ("outliers", "all"):
        res["outliers"] = outliers(**kw)
    if a.study in ("huber", "all"):
        res["huber"] = huber_ablation(**kw)
    res["wall_s"] = time.perf_counter() - t0
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
