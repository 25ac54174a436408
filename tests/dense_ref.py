"""Dense reference solves used to pin the oracle (test helpers).

The linearised BA system is assembled densely from the oracle's linearised
factors and priors: H = sum_f P_f^T Lambda_f P_f + Lambda_p and
g = sum_f P_f^T eta_f + eta_p, with P_f selecting the factor's keyframe and
landmark blocks. Its solution H^-1 g is the MAP estimate of the linearised
problem (Section 4, eq. (residuals)); the blocks of H^-1 are the exact
marginal covariances (Section 3.2, eq. (marginal)).
"""
import numpy as np


def index_maps(nk, nl):
    kf = lambda k: np.arange(6 * k, 6 * k + 6)
    lm = lambda m: 6 * nk + np.arange(3 * m, 3 * m + 3)
    return kf, lm


def assemble(orc, t=None):
    p = orc.problem
    nk, nl, nf = orc.nk, orc.nl, orc.nf
    n = 6 * nk + 3 * nl
    H = np.zeros((n, n))
    g = np.zeros(n)
    kf, lm = index_maps(nk, nl)
    fkf, flm = p.factor_kf, p.factor_lm
    for f in range(nf):
        eta, lam, _, _ = orc.factor(f)
        idx = np.concatenate([kf(fkf[f]), lm(flm[f])])
        H[np.ix_(idx, idx)] += lam
        g[idx] += eta
    kd, ke, ld, le = orc.prior(orc.t if t is None else t)
    for k in range(nk):
        H[kf(k), kf(k)] += kd[k]
        g[kf(k)] += ke[k]
    for m in range(nl):
        H[lm(m), lm(m)] += ld[m]
        g[lm(m)] += le[m]
    return H, g


def gauss_newton(problem, priors, huber_k, zmin=1e-3, iters=200, tol=1e-13,
                 project=None, huber_weight=None, x0=None):
    """Dense Gauss-Newton on the BA objective with fixed diagonal priors and
    the Huber weight evaluated at each linearisation point (the same rule the
    GBP factors use). Returns the stacked estimate [kf (6 Nk); lm (3 Nl)]."""
    p = problem
    nk, nl = p.n_keyframes, p.n_landmarks
    kd, ke, ld, le = priors
    kf, lm = index_maps(nk, nl)
    cam = [p.cam.fx, p.cam.fy, p.cam.cx, p.cam.cy]
    s2 = p.cam.sigma ** 2
    x = np.concatenate([p.kf_init.ravel(), p.lm_init.ravel()]) if x0 is None else x0.copy()
    n = x.size
    for _ in range(iters):
        H = np.zeros((n, n))
        g = np.zeros(n)
        for f in range(p.n_factors):
            ik, il = kf(p.factor_kf[f]), lm(p.factor_lm[f])
            idx = np.concatenate([ik, il])
            h, J, pz = project(x[ik], x[il], cam)
            if not pz > zmin:
                continue
            r0 = p.z[f] - h
            M = np.linalg.norm(r0) / p.cam.sigma
            w = huber_weight(M, huber_k / p.cam.sigma)
            y = J @ x[idx] + r0
            H[np.ix_(idx, idx)] += (w / s2) * J.T @ J
            g[idx] += (w / s2) * J.T @ y
        for k in range(nk):
            H[kf(k), kf(k)] += kd[k]
            g[kf(k)] += ke[k]
        for m in range(nl):
            H[lm(m), lm(m)] += ld[m]
            g[lm(m)] += le[m]
        xn = np.linalg.solve(H, g)
        step = np.abs(xn - x).max()
        x = xn
        if step < tol:
            break
    return x
