/*
 * FP64 reference implementation of synchronous Gaussian Belief Propagation
 * for bundle adjustment (Ortiz et al., "Bundle Adjustment on a Graph
 * Processor", CVPR 2020).
 *
 * TEST INFRASTRUCTURE. This file is the oracle that the HIP library is
 * checked against. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it. It shares
 * no code, header or constant with the HIP library.
 *
 * It follows the paper's formulation literally, in absolute coordinates and
 * full information form:
 *   - factor graph and BA factorisation: Sections 3.1, 4, eqs. (factorprod),
 *     (jointprob);
 *   - measurement model h = pi(R l + t) and its linearisation to information
 *     form with the 2x9 Jacobian: Section 4, eq. (infform) and the two
 *     equations after it;
 *   - factor-to-variable messages by Schur marginalisation of the 9x9
 *     factor plus the incoming variable-to-factor message: Section 5,
 *     eqs. (factor), (messageeta), (messagelambda);
 *   - variable-to-factor messages recovered by dividing the belief by the
 *     previous factor-to-variable message: Section 5, text after
 *     eq. (belieflambda);
 *   - beliefs as prior plus the sum of incoming messages: eqs. (beliefeta),
 *     (belieflambda);
 *   - synchronous schedule, local relinearisation with threshold beta,
 *     damping of the eta message: Section 5 (text), Section 8;
 *   - Huber covariance rescaling: Section 6;
 *   - hyperparameters (beta = 0.01, at most every 10 iterations, d = 0.4,
 *     undamped for 8 iterations after relinearising, priors built from the
 *     Jacobians and weakened to a hundredth over 10 iterations): Section 8;
 *   - average reprojection error: Section 9.1;
 *   - heterogeneous factors (the outlook of Sections 9 and 10: factors from
 *     further priors and sensors in the same graph): pairwise difference
 *     factors between two keyframes or two landmarks, whose messages follow
 *     the same eqs. (messageeta), (messagelambda).
 *
 * Readings where the paper is silent (documented with the design notes):
 *   - a keyframe is x = (omega, t), world->camera, R = Exp(omega);
 *   - pinhole projection without distortion, Sigma_M = sigma^2 I;
 *   - Huber weight w = 2N/M - N^2/M^2 when M > N (N = huber_k / sigma),
 *     evaluated at the linearisation point and multiplying eta_f, Lambda_f;
 *   - relinearise when the Euclidean norm of [mu_k; mu_m] - lin_pt exceeds
 *     beta, at least `relin_interval` factor updates after the previous one;
 *   - damping acts on the eta message only (option damp_lambda: on the
 *     Lambda message as well); the first `undamped` updates after a
 *     relinearisation are undamped;
 *   - beliefs at t+1 use the messages computed in the same iteration;
 *   - automatic priors: diag(sum_f J_i^T Sigma^-1 J_i) at the initial
 *     linearisation (Huber weight 1) times a scale that goes geometrically
 *     from 1 to `weaken` over `anneal_iters` iterations (anneal on), or is
 *     `weaken` throughout (anneal off); a keyframe with an anchor
 *     information a > 0 gets the prior a*I at its initial pose instead;
 *   - the automatic prior information of a coordinate is floored at 1e-8 so
 *     that a variable without a valid factor at its initial estimate still
 *     has a proper belief;
 *   - a factor whose point lies at camera depth <= zmin at the linearisation
 *     point carries no information until it is relinearised again and is
 *     excluded from the reprojection error;
 *   - a pairwise difference factor between variables a and b of the same
 *     kind (dimension D = 6 for keyframes, 3 for landmarks) measures
 *     x_b - x_a ~ N(z, diag(p)^-1): it is linear, never relinearised, and
 *     its information form is Lambda = [P, -P; -P, P], eta = [-P z; P z]
 *     with P = diag(p); its messages are damped like a measurement factor's
 *     (eta only unless damp_lambda; undamped for its first `undamped`
 *     updates after it was added); belief sums take the measurement
 *     factors' messages first, then the pairwise ones in pair order;
 *   - an odometry factor between keyframes a and b measures the displacement
 *     of the camera centres in the world frame, c_b - c_a ~ N(z, diag(p)^-1)
 *     with c = -R(omega)^T t (3 values); it is nonlinear and is linearised
 *     at the current means at every update, then treated as a pairwise
 *     factor with information Lambda = J^T P J, eta = J^T P (z - h(x0) + J x0)
 *     over [x_a; x_b] (J the 3x12 Jacobian at x0); relinearised at every
 *     update, it never leaves the undamped window after a relinearisation,
 *     so its messages are undamped; they enter the keyframe beliefs after
 *     the difference factors'.
 *
 * Every loop runs over factors or variables in increasing index order; a
 * variable sums its incoming messages in increasing factor index order.
 * OpenMP (when enabled at compile time) parallelises those loops without
 * changing any result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KD 6 /* keyframe dimension */
#define LD 3 /* landmark dimension */
#define FD 9 /* factor dimension   */
#define PRIOR_FLOOR 1e-8

typedef struct {
    /* sizes and capacity */
    int nk, nl, nf;
    int cap_k, cap_l, cap_f;
    /* camera: fx fy cx cy sigma */
    double fx, fy, cx, cy, sigma, zmin;
    /* options */
    double beta;
    int relin_interval, undamped, anneal_iters, anneal, damp_lambda;
    double weaken, huber_k;
    int t; /* completed iterations */
    /* variables */
    double *kf_mu, *lm_mu;
    double *kf_eta, *kf_lam, *lm_eta, *lm_lam;
    double *kf_pmean, *lm_pmean, *kf_base, *lm_base, *kf_anchor;
    int *kf_t0, *lm_t0;
    /* factors */
    int *f_kf, *f_lm;
    double *z;
    double *lin, *feta, *flam, *fw;
    int *cnt;
    unsigned char *invalid;
    /* messages factor -> keyframe / landmark, and scratch copies */
    double *mk_eta, *mk_lam, *ml_eta, *ml_lam;
    double *nk_eta, *nk_lam, *nl_eta, *nl_lam;
    /* adjacency: factors of each variable, increasing factor index */
    int *k_ptr, *k_adj, *l_ptr, *l_adj;
    int adj_dirty;
    /* pairwise difference factors: kind 0 between keyframes, 1 between
     * landmarks; per factor: ends a, b, z and diagonal precision (D each),
     * update count, messages to a and b (eta D, Lambda D x D) and scratch */
    struct pairs {
        int n, cap;
        int *a, *b, *cnt;
        double *z, *p;
        double *ma_eta, *ma_lam, *mb_eta, *mb_lam;
        double *na_eta, *na_lam, *nb_eta, *nb_lam;
    } pr[3];
} oracle_t;

/* variable dimension of a pair kind (0: keyframe difference, 1: landmark
 * difference, 2: keyframe odometry) and the dimension of its measurement */
static int pair_dim(int kind) { return kind == 1 ? 3 : 6; }
static int pair_mdim(int kind) { return kind == 0 ? 6 : 3; }

/* --------------------------------------------------------------------------
 * small dense linear algebra
 * ------------------------------------------------------------------------ */

/* Solve A X = B for X (A n x n, B n x m, row-major), Gaussian elimination
 * with partial pivoting. B is overwritten with X. Returns 0 on success. */
static int solve_dense(int n, const double *A_in, double *B, int m) {
    double A[FD * FD];
    memcpy(A, A_in, sizeof(double) * n * n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(A[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > best) { best = fabs(A[r * n + c]); p = r; }
        if (best == 0.0) return -1;
        if (p != c) {
            for (int j = 0; j < n; ++j) { double t = A[c*n+j]; A[c*n+j] = A[p*n+j]; A[p*n+j] = t; }
            for (int j = 0; j < m; ++j) { double t = B[c*m+j]; B[c*m+j] = B[p*m+j]; B[p*m+j] = t; }
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            for (int j = 0; j < m; ++j) B[r * m + j] -= f * B[c * m + j];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int j = 0; j < m; ++j) {
            double s = B[c * m + j];
            for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * B[k * m + j];
            B[c * m + j] = s / A[c * n + c];
        }
    }
    return 0;
}

static void skew(const double *v, double *S) {
    S[0] = 0;     S[1] = -v[2]; S[2] = v[1];
    S[3] = v[2];  S[4] = 0;     S[5] = -v[0];
    S[6] = -v[1]; S[7] = v[0];  S[8] = 0;
}

static void mat3_mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[i*3+k] * B[k*3+j];
            C[i*3+j] = s;
        }
}

/* --------------------------------------------------------------------------
 * SO(3): exponential map (Rodrigues) and right Jacobian
 * ------------------------------------------------------------------------ */

void oracle_so3_exp(const double *w, double *R) {
    double th2 = w[0]*w[0] + w[1]*w[1] + w[2]*w[2];
    double th = sqrt(th2), a, b;
    if (th < 1e-5) { a = 1.0 - th2 / 6.0; b = 0.5 - th2 / 24.0; }
    else { a = sin(th) / th; b = (1.0 - cos(th)) / th2; }
    double W[9], W2[9];
    skew(w, W);
    mat3_mul(W, W, W2);
    for (int i = 0; i < 9; ++i) R[i] = a * W[i] + b * W2[i];
    R[0] += 1.0; R[4] += 1.0; R[8] += 1.0;
}

/* J_r(w) = I - (1-cos th)/th^2 [w]x + (th - sin th)/th^3 [w]x^2 */
void oracle_so3_jr(const double *w, double *Jr) {
    double th2 = w[0]*w[0] + w[1]*w[1] + w[2]*w[2];
    double th = sqrt(th2), b, c;
    if (th < 1e-5) { b = 0.5 - th2 / 24.0; c = 1.0 / 6.0 - th2 / 120.0; }
    else { b = (1.0 - cos(th)) / th2; c = (th - sin(th)) / (th2 * th); }
    double W[9], W2[9];
    skew(w, W);
    mat3_mul(W, W, W2);
    for (int i = 0; i < 9; ++i) Jr[i] = -b * W[i] + c * W2[i];
    Jr[0] += 1.0; Jr[4] += 1.0; Jr[8] += 1.0;
}

/* --------------------------------------------------------------------------
 * measurement model h(x, l) = pi(R l + t) and its 2x9 Jacobian
 * cam = {fx, fy, cx, cy}. Returns the camera depth p_z.
 * J (row-major 2x9) columns: d/d omega (3), d/d t (3), d/d l (3).
 * ------------------------------------------------------------------------ */

double oracle_project(const double *x, const double *l, const double *cam,
                      double *h, double *J) {
    double R[9];
    oracle_so3_exp(x, R);
    double p[3];
    for (int i = 0; i < 3; ++i)
        p[i] = R[i*3+0]*l[0] + R[i*3+1]*l[1] + R[i*3+2]*l[2] + x[3+i];
    double fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3];
    if (h) {
        h[0] = fx * p[0] / p[2] + cx;
        h[1] = fy * p[1] / p[2] + cy;
    }
    if (J) {
        /* d pi / d p */
        double D[6] = { fx / p[2], 0.0, -fx * p[0] / (p[2]*p[2]),
                        0.0, fy / p[2], -fy * p[1] / (p[2]*p[2]) };
        /* d p / d omega = -R [l]x J_r(omega) */
        double L[9], Jr[9], RL[9], Pw[9];
        skew(l, L);
        oracle_so3_jr(x, Jr);
        mat3_mul(R, L, RL);
        mat3_mul(RL, Jr, Pw);
        for (int i = 0; i < 9; ++i) Pw[i] = -Pw[i];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) {
                double sw = 0, sl = 0;
                for (int k = 0; k < 3; ++k) {
                    sw += D[r*3+k] * Pw[k*3+c];
                    sl += D[r*3+k] * R[k*3+c];
                }
                J[r*9 + c] = sw;             /* omega */
                J[r*9 + 3 + c] = D[r*3+c];   /* t: d p / d t = I */
                J[r*9 + 6 + c] = sl;         /* l: d p / d l = R */
            }
    }
    return p[2];
}

/* Huber rescaling of Section 6: the Gaussian exponent -M^2/2 is multiplied
 * by w so that it equals the Huber cost; N is the threshold in units of
 * sigma. N <= 0 disables the robust kernel. */
double oracle_huber_weight(double M, double N) {
    if (N <= 0.0 || M <= N) return 1.0;
    return 2.0 * N / M - N * N / (M * M);
}

/* --------------------------------------------------------------------------
 * state
 * ------------------------------------------------------------------------ */

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

static void build_adjacency(oracle_t *o) {
    free(o->k_ptr); free(o->k_adj); free(o->l_ptr); free(o->l_adj);
    o->k_ptr = xcalloc(o->nk + 1, sizeof(int));
    o->l_ptr = xcalloc(o->nl + 1, sizeof(int));
    o->k_adj = xcalloc(o->nf, sizeof(int));
    o->l_adj = xcalloc(o->nf, sizeof(int));
    for (int f = 0; f < o->nf; ++f) { o->k_ptr[o->f_kf[f] + 1]++; o->l_ptr[o->f_lm[f] + 1]++; }
    for (int i = 0; i < o->nk; ++i) o->k_ptr[i + 1] += o->k_ptr[i];
    for (int i = 0; i < o->nl; ++i) o->l_ptr[i + 1] += o->l_ptr[i];
    int *pk = xcalloc(o->nk, sizeof(int)), *pl = xcalloc(o->nl, sizeof(int));
    for (int f = 0; f < o->nf; ++f) {
        int k = o->f_kf[f], m = o->f_lm[f];
        o->k_adj[o->k_ptr[k] + pk[k]++] = f;
        o->l_adj[o->l_ptr[m] + pl[m]++] = f;
    }
    free(pk); free(pl);
    o->adj_dirty = 0;
}

/* Linearise factor f at the current means (Section 4, eq. (infform) and the
 * two equations that follow it; Huber rescaling of Section 6). */
static void relinearise_factor(oracle_t *o, int f, double huber_k) {
    const double *x0 = o->kf_mu + (size_t)o->f_kf[f] * KD;
    const double *l0 = o->lm_mu + (size_t)o->f_lm[f] * LD;
    double *lin = o->lin + (size_t)f * FD;
    double *eta = o->feta + (size_t)f * FD;
    double *lam = o->flam + (size_t)f * FD * FD;
    for (int i = 0; i < KD; ++i) lin[i] = x0[i];
    for (int i = 0; i < LD; ++i) lin[KD + i] = l0[i];
    double cam[4] = { o->fx, o->fy, o->cx, o->cy };
    double h[2], J[18];
    double pz = oracle_project(x0, l0, cam, h, J);
    o->cnt[f] = 0;
    if (!(pz > o->zmin)) {
        o->invalid[f] = 1;
        o->fw[f] = 0.0;
        memset(eta, 0, sizeof(double) * FD);
        memset(lam, 0, sizeof(double) * FD * FD);
        return;
    }
    o->invalid[f] = 0;
    double r0[2] = { o->z[2*f] - h[0], o->z[2*f+1] - h[1] };
    double M = sqrt(r0[0]*r0[0] + r0[1]*r0[1]) / o->sigma;
    double w = oracle_huber_weight(M, huber_k / o->sigma);
    o->fw[f] = w;
    double s = w / (o->sigma * o->sigma);   /* Sigma_M^-1 rescaled by Huber */
    /* y = J [x0; l0] + z - h(x0, l0) */
    double y[2];
    for (int r = 0; r < 2; ++r) {
        double acc = r0[r];
        for (int c = 0; c < FD; ++c) acc += J[r*9 + c] * lin[c];
        y[r] = acc;
    }
    for (int i = 0; i < FD; ++i) {
        eta[i] = s * (J[i] * y[0] + J[9 + i] * y[1]);
        for (int j = 0; j < FD; ++j)
            lam[i*FD + j] = s * (J[i] * J[j] + J[9 + i] * J[9 + j]);
    }
}

/* prior information (diagonal) and information vector of a variable at
 * iteration clock t (Section 4 auto-priors; Section 8 schedule). */
static double prior_scale(const oracle_t *o, int age) {
    if (!o->anneal || o->anneal_iters <= 0) return o->weaken;
    int a = age < o->anneal_iters ? age : o->anneal_iters;
    if (a < 0) a = 0;
    return pow(o->weaken, (double)a / (double)o->anneal_iters);
}

static void kf_prior(const oracle_t *o, int k, int t, double *lam_diag, double *eta) {
    const double *mean = o->kf_pmean + (size_t)k * KD;
    if (o->kf_anchor[k] > 0.0) {
        for (int i = 0; i < KD; ++i) lam_diag[i] = o->kf_anchor[k];
    } else {
        double sc = prior_scale(o, t - o->kf_t0[k]);
        for (int i = 0; i < KD; ++i) lam_diag[i] = o->kf_base[(size_t)k*KD + i] * sc;
    }
    for (int i = 0; i < KD; ++i) eta[i] = lam_diag[i] * mean[i];
}

static void lm_prior(const oracle_t *o, int m, int t, double *lam_diag, double *eta) {
    const double *mean = o->lm_pmean + (size_t)m * LD;
    double sc = prior_scale(o, t - o->lm_t0[m]);
    for (int i = 0; i < LD; ++i) {
        lam_diag[i] = o->lm_base[(size_t)m*LD + i] * sc;
        eta[i] = lam_diag[i] * mean[i];
    }
}

/* Belief of every variable at clock o->t: prior plus the sum of incoming
 * factor messages (eqs. (beliefeta), (belieflambda)); mean = Lambda^-1 eta.
 * Measurement-factor messages are added first (increasing factor index),
 * then the pairwise factors' (increasing pair index). */
static int update_beliefs(oracle_t *o) {
    if (o->adj_dirty) build_adjacency(o);
    int bad = 0;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < o->nk; ++k) {
        double *eta = o->kf_eta + (size_t)k * KD, *lam = o->kf_lam + (size_t)k * KD * KD;
        double pd[KD], pe[KD];
        kf_prior(o, k, o->t, pd, pe);
        for (int i = 0; i < KD; ++i) {
            eta[i] = pe[i];
            for (int j = 0; j < KD; ++j) lam[i*KD + j] = (i == j) ? pd[i] : 0.0;
        }
        for (int e = o->k_ptr[k]; e < o->k_ptr[k + 1]; ++e) {
            int f = o->k_adj[e];
            for (int i = 0; i < KD; ++i) eta[i] += o->mk_eta[(size_t)f*KD + i];
            for (int i = 0; i < KD*KD; ++i) lam[i] += o->mk_lam[(size_t)f*KD*KD + i];
        }
    }
#pragma omp parallel for schedule(static)
    for (int m = 0; m < o->nl; ++m) {
        double *eta = o->lm_eta + (size_t)m * LD, *lam = o->lm_lam + (size_t)m * LD * LD;
        double pd[LD], pe[LD];
        lm_prior(o, m, o->t, pd, pe);
        for (int i = 0; i < LD; ++i) {
            eta[i] = pe[i];
            for (int j = 0; j < LD; ++j) lam[i*LD + j] = (i == j) ? pd[i] : 0.0;
        }
        for (int e = o->l_ptr[m]; e < o->l_ptr[m + 1]; ++e) {
            int f = o->l_adj[e];
            for (int i = 0; i < LD; ++i) eta[i] += o->ml_eta[(size_t)f*LD + i];
            for (int i = 0; i < LD*LD; ++i) lam[i] += o->ml_lam[(size_t)f*LD*LD + i];
        }
    }
    for (int kind = 0; kind < 3; ++kind) {
        const struct pairs *q = &o->pr[kind];
        const int D = pair_dim(kind);
        double *veta = kind == 1 ? o->lm_eta : o->kf_eta, *vlam = kind == 1 ? o->lm_lam : o->kf_lam;
        for (int f = 0; f < q->n; ++f) {
            for (int i = 0; i < D; ++i) {
                veta[(size_t)q->a[f]*D + i] += q->ma_eta[(size_t)f*D + i];
                veta[(size_t)q->b[f]*D + i] += q->mb_eta[(size_t)f*D + i];
            }
            for (int i = 0; i < D*D; ++i) {
                vlam[(size_t)q->a[f]*D*D + i] += q->ma_lam[(size_t)f*D*D + i];
                vlam[(size_t)q->b[f]*D*D + i] += q->mb_lam[(size_t)f*D*D + i];
            }
        }
    }
#pragma omp parallel for schedule(static) reduction(+:bad)
    for (int k = 0; k < o->nk; ++k) {
        double mu[KD];
        memcpy(mu, o->kf_eta + (size_t)k * KD, sizeof mu);
        if (solve_dense(KD, o->kf_lam + (size_t)k * KD * KD, mu, 1) != 0) { bad++; continue; }
        memcpy(o->kf_mu + (size_t)k * KD, mu, sizeof mu);
    }
#pragma omp parallel for schedule(static) reduction(+:bad)
    for (int m = 0; m < o->nl; ++m) {
        double mu[LD];
        memcpy(mu, o->lm_eta + (size_t)m * LD, sizeof mu);
        if (solve_dense(LD, o->lm_lam + (size_t)m * LD * LD, mu, 1) != 0) { bad++; continue; }
        memcpy(o->lm_mu + (size_t)m * LD, mu, sizeof mu);
    }
    return bad;
}

/* Camera centre c = -R(omega)^T t of pose x = (omega, t) and its 3x6
 * Jacobian: with Exp(omega + d) ~ Exp(omega) Exp(J_r(omega) d),
 * dc/domega = [c]x J_r(omega) and dc/dt = -R^T. */
static void centre_and_jacobian(const double *x, double *c, double *Jc) {
    double R[9], Jr[9], S[9];
    oracle_so3_exp(x, R);
    oracle_so3_jr(x, Jr);
    for (int i = 0; i < 3; ++i) c[i] = -(R[0*3+i] * x[3] + R[1*3+i] * x[4] + R[2*3+i] * x[5]);
    skew(c, S);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += S[i*3+k] * Jr[k*3+j];
            Jc[i*6 + j] = s;
            Jc[i*6 + 3 + j] = -R[j*3 + i];
        }
}

/* Odometry measurement h(x_a, x_b) = c_b - c_a and its 3x12 Jacobian */
void oracle_odometry(const double *xa, const double *xb, double *h, double *J) {
    double ca[3], cb[3], Ja[18], Jb[18];
    centre_and_jacobian(xa, ca, Ja);
    centre_and_jacobian(xb, cb, Jb);
    for (int i = 0; i < 3; ++i) {
        h[i] = cb[i] - ca[i];
        if (J)
            for (int j = 0; j < 6; ++j) { J[i*12 + j] = -Ja[i*6 + j]; J[i*12 + 6 + j] = Jb[i*6 + j]; }
    }
}

/* Messages of an odometry factor (kind 2), linearised at the current means,
 * to both ends by eqs. (messageeta), (messagelambda) with the full 12x12
 * factor; damping as for the other pairs. */
static int odometry_messages(oracle_t *o, int f, double damping) {
    struct pairs *q = &o->pr[2];
    const int a = q->a[f], b = q->b[f];
    const double *xa = o->kf_mu + (size_t)a * KD, *xb = o->kf_mu + (size_t)b * KD;
    const double *z = q->z + (size_t)f * 3, *p = q->p + (size_t)f * 3;
    double h[3], J[36], L[144], e[12], r[3];
    oracle_odometry(xa, xb, h, J);
    for (int i = 0; i < 3; ++i) {
        double jx = 0.0;
        for (int j = 0; j < 6; ++j) jx += J[i*12 + j] * xa[j] + J[i*12 + 6 + j] * xb[j];
        r[i] = z[i] - h[i] + jx;
    }
    for (int u = 0; u < 12; ++u) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += J[i*12 + u] * p[i] * r[i];
        e[u] = s;
        for (int v = 0; v < 12; ++v) {
            double t = 0.0;
            for (int i = 0; i < 3; ++i) t += J[i*12 + u] * p[i] * J[i*12 + v];
            L[u*12 + v] = t;
        }
    }
    /* relinearised at every update, the factor is always inside the
     * undamped window that follows a relinearisation (Section 8) */
    const double d_eff = 0.0;
    (void)damping;
    for (int side = 0; side < 2; ++side) {
        /* side 0: message to b (marginalise a, block offset 0); side 1: to a */
        const int u = side == 0 ? a : b, ou = side == 0 ? 0 : 6, ov = side == 0 ? 6 : 0;
        const double *mu_eta = (side == 0 ? q->ma_eta : q->mb_eta) + (size_t)f * KD;
        const double *mu_lam = (side == 0 ? q->ma_lam : q->mb_lam) + (size_t)f * KD * KD;
        const double *old_eta = (side == 0 ? q->mb_eta : q->ma_eta) + (size_t)f * KD;
        const double *old_lam = (side == 0 ? q->mb_lam : q->ma_lam) + (size_t)f * KD * KD;
        double *out_eta = (side == 0 ? q->nb_eta : q->na_eta) + (size_t)f * KD;
        double *out_lam = (side == 0 ? q->nb_lam : q->na_lam) + (size_t)f * KD * KD;
        double A[KD*KD], X[KD*(KD+1)];
        for (int i = 0; i < KD; ++i) {
            for (int j = 0; j < KD; ++j) {
                A[i*KD + j] = L[(ou+i)*12 + ou + j] + o->kf_lam[(size_t)u*KD*KD + i*KD + j] - mu_lam[i*KD + j];
                X[i*(KD+1) + j] = L[(ou+i)*12 + ov + j];
            }
            X[i*(KD+1) + KD] = e[ou+i] + o->kf_eta[(size_t)u*KD + i] - mu_eta[i];
        }
        if (solve_dense(KD, A, X, KD + 1) != 0) return -1;
        for (int i = 0; i < KD; ++i) {
            double se = e[ov+i];
            for (int k = 0; k < KD; ++k) se -= L[(ov+i)*12 + ou + k] * X[k*(KD+1) + KD];
            out_eta[i] = (1.0 - d_eff) * se + d_eff * old_eta[i];
            for (int j = 0; j < KD; ++j) {
                double sl = L[(ov+i)*12 + ov + j];
                for (int k = 0; k < KD; ++k) sl -= L[(ov+i)*12 + ou + k] * X[k*(KD+1) + j];
                out_lam[i*KD + j] = o->damp_lambda ? (1.0 - d_eff) * sl + d_eff * old_lam[i*KD + j] : sl;
            }
        }
    }
    return 0;
}

/* Messages of pairwise factor f (kind: 0 keyframes, 1 landmarks) to both
 * ends, eqs. (messageeta), (messagelambda) for the factor Lambda = [P, -P;
 * -P, P], eta = [-P z; P z]: the message to one end marginalises the other
 * end's block after adding that end's variable-to-factor message (its
 * belief minus this factor's previous message to it). */
static int pair_messages(oracle_t *o, int kind, int f, double damping) {
    struct pairs *q = &o->pr[kind];
    const int D = pair_dim(kind);
    const double *veta = kind == 0 ? o->kf_eta : o->lm_eta, *vlam = kind == 0 ? o->kf_lam : o->lm_lam;
    const double *z = q->z + (size_t)f * D, *p = q->p + (size_t)f * D;
    const double d_eff = (q->cnt[f] < o->undamped) ? 0.0 : damping;
    for (int side = 0; side < 2; ++side) {
        /* side 0: message to b (marginalise a); side 1: message to a */
        const int u = side == 0 ? q->a[f] : q->b[f];
        const double *mu_eta = (side == 0 ? q->ma_eta : q->mb_eta) + (size_t)f * D;
        const double *mu_lam = (side == 0 ? q->ma_lam : q->mb_lam) + (size_t)f * D * D;
        const double *old_eta = (side == 0 ? q->mb_eta : q->ma_eta) + (size_t)f * D;
        const double *old_lam = (side == 0 ? q->mb_lam : q->ma_lam) + (size_t)f * D * D;
        double *out_eta = (side == 0 ? q->nb_eta : q->na_eta) + (size_t)f * D;
        double *out_lam = (side == 0 ? q->nb_lam : q->na_lam) + (size_t)f * D * D;
        /* factor blocks seen from the receiving end v: Lambda_vv = P,
         * Lambda_vu = -P, Lambda_uu = P, eta_v = +-P z, eta_u = -+P z */
        const double sv = side == 0 ? 1.0 : -1.0;
        double A[KD*KD], X[KD*(KD+1)];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                /* Lambda_uu + (belief_u - message_u) */
                A[r*D + c] = (r == c ? p[r] : 0.0) + vlam[(size_t)u*D*D + r*D + c] - mu_lam[r*D + c];
                X[r*(D+1) + c] = (r == c ? -p[r] : 0.0);                      /* Lambda_uv */
            }
        for (int r = 0; r < D; ++r)
            X[r*(D+1) + D] = -sv * p[r] * z[r] + veta[(size_t)u*D + r] - mu_eta[r]; /* eta_u + v_eta_u */
        if (solve_dense(D, A, X, D + 1) != 0) return -1;
        for (int r = 0; r < D; ++r) {
            /* eta_v - Lambda_vu X_eta, Lambda_vv - Lambda_vu X_Lambda */
            double se = sv * p[r] * z[r] + p[r] * X[r*(D+1) + D];
            out_eta[r] = (1.0 - d_eff) * se + d_eff * old_eta[r];
            for (int c = 0; c < D; ++c) {
                double sl = (r == c ? p[r] : 0.0) + p[r] * X[r*(D+1) + c];
                out_lam[r*D + c] = o->damp_lambda ? (1.0 - d_eff) * sl + d_eff * old_lam[r*D + c] : sl;
            }
        }
    }
    return 0;
}

/* Messages of factor f to its keyframe (block 0..5) and landmark (6..8),
 * eqs. (messageeta), (messagelambda), with the variable-to-factor message
 * recovered as belief minus the previous factor-to-variable message, and
 * eta damping with factor d_eff. Writes into the scratch message arrays. */
static int factor_messages(oracle_t *o, int f, double damping) {
    int k = o->f_kf[f], m = o->f_lm[f];
    const double *eta = o->feta + (size_t)f * FD, *lam = o->flam + (size_t)f * FD * FD;
    /* variable-to-factor messages: belief / previous factor-to-variable */
    double vk_eta[KD], vk_lam[KD*KD], vl_eta[LD], vl_lam[LD*LD];
    for (int i = 0; i < KD; ++i) vk_eta[i] = o->kf_eta[(size_t)k*KD + i] - o->mk_eta[(size_t)f*KD + i];
    for (int i = 0; i < KD*KD; ++i) vk_lam[i] = o->kf_lam[(size_t)k*KD*KD + i] - o->mk_lam[(size_t)f*KD*KD + i];
    for (int i = 0; i < LD; ++i) vl_eta[i] = o->lm_eta[(size_t)m*LD + i] - o->ml_eta[(size_t)f*LD + i];
    for (int i = 0; i < LD*LD; ++i) vl_lam[i] = o->lm_lam[(size_t)m*LD*LD + i] - o->ml_lam[(size_t)f*LD*LD + i];

    /* factor blocks: i = keyframe (0..5), j = landmark (6..8) */
    double Lkk[KD*KD], Lkm[KD*LD], Lmk[LD*KD], Lmm[LD*LD];
    for (int r = 0; r < KD; ++r) {
        for (int c = 0; c < KD; ++c) Lkk[r*KD + c] = lam[r*FD + c];
        for (int c = 0; c < LD; ++c) Lkm[r*LD + c] = lam[r*FD + KD + c];
    }
    for (int r = 0; r < LD; ++r) {
        for (int c = 0; c < KD; ++c) Lmk[r*KD + c] = lam[(KD + r)*FD + c];
        for (int c = 0; c < LD; ++c) Lmm[r*LD + c] = lam[(KD + r)*FD + KD + c];
    }

    double d_eff = (o->cnt[f] < o->undamped) ? 0.0 : damping;

    /* ---- message to the keyframe: marginalise the landmark ---- */
    {
        double A[LD*LD];
        for (int i = 0; i < LD*LD; ++i) A[i] = Lmm[i] + vl_lam[i];
        /* X = A^-1 [Lmk | eta_m + v_eta_m] */
        double X[LD*(KD+1)];
        for (int r = 0; r < LD; ++r) {
            for (int c = 0; c < KD; ++c) X[r*(KD+1) + c] = Lmk[r*KD + c];
            X[r*(KD+1) + KD] = eta[KD + r] + vl_eta[r];
        }
        if (solve_dense(LD, A, X, KD + 1) != 0) return -1;
        double *out_eta = o->nk_eta + (size_t)f * KD, *out_lam = o->nk_lam + (size_t)f * KD * KD;
        for (int r = 0; r < KD; ++r) {
            double se = eta[r];
            for (int q = 0; q < LD; ++q) se -= Lkm[r*LD + q] * X[q*(KD+1) + KD];
            out_eta[r] = (1.0 - d_eff) * se + d_eff * o->mk_eta[(size_t)f*KD + r];
            for (int c = 0; c < KD; ++c) {
                double sl = Lkk[r*KD + c];
                for (int q = 0; q < LD; ++q) sl -= Lkm[r*LD + q] * X[q*(KD+1) + c];
                out_lam[r*KD + c] = o->damp_lambda
                    ? (1.0 - d_eff) * sl + d_eff * o->mk_lam[(size_t)f*KD*KD + r*KD + c] : sl;
            }
        }
    }
    /* ---- message to the landmark: marginalise the keyframe ---- */
    {
        double B[KD*KD];
        for (int i = 0; i < KD*KD; ++i) B[i] = Lkk[i] + vk_lam[i];
        double X[KD*(LD+1)];
        for (int r = 0; r < KD; ++r) {
            for (int c = 0; c < LD; ++c) X[r*(LD+1) + c] = Lkm[r*LD + c];
            X[r*(LD+1) + LD] = eta[r] + vk_eta[r];
        }
        if (solve_dense(KD, B, X, LD + 1) != 0) return -1;
        double *out_eta = o->nl_eta + (size_t)f * LD, *out_lam = o->nl_lam + (size_t)f * LD * LD;
        for (int r = 0; r < LD; ++r) {
            double se = eta[KD + r];
            for (int q = 0; q < KD; ++q) se -= Lmk[r*KD + q] * X[q*(LD+1) + LD];
            out_eta[r] = (1.0 - d_eff) * se + d_eff * o->ml_eta[(size_t)f*LD + r];
            for (int c = 0; c < LD; ++c) {
                double sl = Lmm[r*LD + c];
                for (int q = 0; q < KD; ++q) sl -= Lmk[r*KD + q] * X[q*(LD+1) + c];
                out_lam[r*LD + c] = o->damp_lambda
                    ? (1.0 - d_eff) * sl + d_eff * o->ml_lam[(size_t)f*LD*LD + r*LD + c] : sl;
            }
        }
    }
    return 0;
}

static double dist_to_lin(const oracle_t *o, int f) {
    const double *x = o->kf_mu + (size_t)o->f_kf[f] * KD;
    const double *l = o->lm_mu + (size_t)o->f_lm[f] * LD;
    const double *lin = o->lin + (size_t)f * FD;
    double s = 0;
    for (int i = 0; i < KD; ++i) { double d = x[i] - lin[i]; s += d * d; }
    for (int i = 0; i < LD; ++i) { double d = l[i] - lin[KD + i]; s += d * d; }
    return sqrt(s);
}

/* --------------------------------------------------------------------------
 * public entry points (ctypes)
 * ------------------------------------------------------------------------ */

static int grow(oracle_t *o, int cap_k, int cap_l, int cap_f) {
#define RE(p, n, T) do { size_t cnt_ = (size_t)(n); void *q = realloc(o->p, (cnt_ ? cnt_ : 1) * sizeof(T)); if (!q) return -1; o->p = q; } while (0)
    RE(kf_mu, cap_k*KD, double); RE(kf_eta, cap_k*KD, double); RE(kf_lam, cap_k*KD*KD, double);
    RE(kf_pmean, cap_k*KD, double); RE(kf_base, cap_k*KD, double); RE(kf_anchor, cap_k, double);
    RE(kf_t0, cap_k, int);
    RE(lm_mu, cap_l*LD, double); RE(lm_eta, cap_l*LD, double); RE(lm_lam, cap_l*LD*LD, double);
    RE(lm_pmean, cap_l*LD, double); RE(lm_base, cap_l*LD, double); RE(lm_t0, cap_l, int);
    RE(f_kf, cap_f, int); RE(f_lm, cap_f, int); RE(z, cap_f*2, double);
    RE(lin, cap_f*FD, double); RE(feta, cap_f*FD, double); RE(flam, cap_f*FD*FD, double);
    RE(fw, cap_f, double); RE(cnt, cap_f, int); RE(invalid, cap_f, unsigned char);
    RE(mk_eta, cap_f*KD, double); RE(mk_lam, cap_f*KD*KD, double);
    RE(ml_eta, cap_f*LD, double); RE(ml_lam, cap_f*LD*LD, double);
    RE(nk_eta, cap_f*KD, double); RE(nk_lam, cap_f*KD*KD, double);
    RE(nl_eta, cap_f*LD, double); RE(nl_lam, cap_f*LD*LD, double);
#undef RE
    o->cap_k = cap_k; o->cap_l = cap_l; o->cap_f = cap_f;
    return 0;
}

void oracle_destroy(void *h);

/* Add factors [f0, nf) that are already stored (indices, z); linearise them
 * at the current means and zero their messages. */
static void init_new_factors(oracle_t *o, int f0) {
    for (int f = f0; f < o->nf; ++f) {
        relinearise_factor(o, f, o->huber_k);
        memset(o->mk_eta + (size_t)f*KD, 0, sizeof(double)*KD);
        memset(o->mk_lam + (size_t)f*KD*KD, 0, sizeof(double)*KD*KD);
        memset(o->ml_eta + (size_t)f*LD, 0, sizeof(double)*LD);
        memset(o->ml_lam + (size_t)f*LD*LD, 0, sizeof(double)*LD*LD);
    }
}

/* Automatic prior base of variables born at or after (k0, m0): the diagonal
 * of sum_f J_i^T Sigma_M^-1 J_i over the factors from f0 on, Huber weight 1. */
static void build_prior_base(oracle_t *o, int k0, int m0, int f0) {
    for (int k = k0; k < o->nk; ++k) for (int i = 0; i < KD; ++i) o->kf_base[(size_t)k*KD + i] = 0.0;
    for (int m = m0; m < o->nl; ++m) for (int i = 0; i < LD; ++i) o->lm_base[(size_t)m*LD + i] = 0.0;
    double cam[4] = { o->fx, o->fy, o->cx, o->cy };
    double inv_s2 = 1.0 / (o->sigma * o->sigma);
    for (int f = f0; f < o->nf; ++f) {
        int k = o->f_kf[f], m = o->f_lm[f];
        if (k < k0 && m < m0) continue;
        double J[18];
        double pz = oracle_project(o->kf_mu + (size_t)k*KD, o->lm_mu + (size_t)m*LD, cam, NULL, J);
        if (!(pz > o->zmin)) continue;
        if (k >= k0)
            for (int i = 0; i < KD; ++i)
                o->kf_base[(size_t)k*KD + i] += inv_s2 * (J[i]*J[i] + J[9+i]*J[9+i]);
        if (m >= m0)
            for (int i = 0; i < LD; ++i)
                o->lm_base[(size_t)m*LD + i] += inv_s2 * (J[KD+i]*J[KD+i] + J[9+KD+i]*J[9+KD+i]);
    }
    for (int k = k0; k < o->nk; ++k) for (int i = 0; i < KD; ++i)
        if (o->kf_base[(size_t)k*KD + i] < PRIOR_FLOOR) o->kf_base[(size_t)k*KD + i] = PRIOR_FLOOR;
    for (int m = m0; m < o->nl; ++m) for (int i = 0; i < LD; ++i)
        if (o->lm_base[(size_t)m*LD + i] < PRIOR_FLOOR) o->lm_base[(size_t)m*LD + i] = PRIOR_FLOOR;
}

/* cam = {fx, fy, cx, cy, sigma, zmin}
 * opt = {beta, relin_interval, undamped, anneal_iters, weaken, anneal, huber_k,
 *        damp_lambda} */
void *oracle_create(int nk, int nl, int nf, const int *f_kf, const int *f_lm,
                    const double *kf_init, const double *lm_init,
                    const double *kf_anchor_info, const double *z,
                    const double *cam, const double *opt) {
    oracle_t *o = calloc(1, sizeof(oracle_t));
    if (!o) return NULL;
    if (grow(o, nk, nl, nf) != 0) { oracle_destroy(o); return NULL; }
    o->nk = nk; o->nl = nl; o->nf = nf;
    o->fx = cam[0]; o->fy = cam[1]; o->cx = cam[2]; o->cy = cam[3];
    o->sigma = cam[4]; o->zmin = cam[5];
    o->beta = opt[0]; o->relin_interval = (int)opt[1]; o->undamped = (int)opt[2];
    o->anneal_iters = (int)opt[3]; o->weaken = opt[4]; o->anneal = (int)opt[5];
    o->huber_k = opt[6]; o->damp_lambda = (int)opt[7];
    o->t = 0;
    memcpy(o->f_kf, f_kf, sizeof(int) * nf);
    memcpy(o->f_lm, f_lm, sizeof(int) * nf);
    memcpy(o->z, z, sizeof(double) * 2 * nf);
    memcpy(o->kf_mu, kf_init, sizeof(double) * KD * nk);
    memcpy(o->lm_mu, lm_init, sizeof(double) * LD * nl);
    memcpy(o->kf_pmean, kf_init, sizeof(double) * KD * nk);
    memcpy(o->lm_pmean, lm_init, sizeof(double) * LD * nl);
    for (int k = 0; k < nk; ++k) { o->kf_anchor[k] = kf_anchor_info ? kf_anchor_info[k] : 0.0; o->kf_t0[k] = 0; }
    for (int m = 0; m < nl; ++m) o->lm_t0[m] = 0;
    o->adj_dirty = 1;
    build_prior_base(o, 0, 0, 0);
    init_new_factors(o, 0);
    update_beliefs(o);
    return o;
}

void oracle_destroy(void *h) {
    oracle_t *o = h;
    if (!o) return;
    void *ps[] = { o->kf_mu, o->lm_mu, o->kf_eta, o->kf_lam, o->lm_eta, o->lm_lam,
                   o->kf_pmean, o->lm_pmean, o->kf_base, o->lm_base, o->kf_anchor,
                   o->kf_t0, o->lm_t0, o->f_kf, o->f_lm, o->z, o->lin, o->feta,
                   o->flam, o->fw, o->cnt, o->invalid, o->mk_eta, o->mk_lam,
                   o->ml_eta, o->ml_lam, o->nk_eta, o->nk_lam, o->nl_eta, o->nl_lam,
                   o->k_ptr, o->k_adj, o->l_ptr, o->l_adj };
    for (size_t i = 0; i < sizeof ps / sizeof ps[0]; ++i) free(ps[i]);
    for (int kind = 0; kind < 3; ++kind) {
        struct pairs *q = &o->pr[kind];
        void *qs[] = { q->a, q->b, q->cnt, q->z, q->p, q->ma_eta, q->ma_lam, q->mb_eta,
                       q->mb_lam, q->na_eta, q->na_lam, q->nb_eta, q->nb_lam };
        for (size_t i = 0; i < sizeof qs / sizeof qs[0]; ++i) free(qs[i]);
    }
    free(o);
}

/* beta < 0: relinearise every factor; otherwise every factor whose distance
 * from its linearisation point exceeds beta. Returns the count. */
int oracle_relinearise(void *h, double beta) {
    oracle_t *o = h;
    int n = 0;
    for (int f = 0; f < o->nf; ++f)
        if (beta < 0.0 || dist_to_lin(o, f) > beta) { relinearise_factor(o, f, o->huber_k); ++n; }
    return n;
}

/* n synchronous iterations (Section 5): relinearisation phase, factor
 * phase, belief phase. Returns 0, or -1 when a solve failed. */
int oracle_iterate(void *h, int n, double damping, double huber_k) {
    oracle_t *o = h;
    o->huber_k = huber_k;
    if (o->adj_dirty) build_adjacency(o);
    for (int it = 0; it < n; ++it) {
#pragma omp parallel for schedule(static)
        for (int f = 0; f < o->nf; ++f)
            if (o->cnt[f] >= o->relin_interval && dist_to_lin(o, f) > o->beta)
                relinearise_factor(o, f, huber_k);
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(+:bad)
        for (int f = 0; f < o->nf; ++f) {
            if (factor_messages(o, f, damping) != 0) bad++;
            o->cnt[f] += 1;
        }
        for (int kind = 0; kind < 3; ++kind) {
            struct pairs *q = &o->pr[kind];
            for (int f = 0; f < q->n; ++f) {
                if ((kind == 2 ? odometry_messages(o, f, damping) : pair_messages(o, kind, f, damping)) != 0) bad++;
                q->cnt[f] += 1;
            }
            double *u;
            u = q->ma_eta; q->ma_eta = q->na_eta; q->na_eta = u;
            u = q->ma_lam; q->ma_lam = q->na_lam; q->na_lam = u;
            u = q->mb_eta; q->mb_eta = q->nb_eta; q->nb_eta = u;
            u = q->mb_lam; q->mb_lam = q->nb_lam; q->nb_lam = u;
        }
        if (bad) return -1;
        double *t;
        t = o->mk_eta; o->mk_eta = o->nk_eta; o->nk_eta = t;
        t = o->mk_lam; o->mk_lam = o->nk_lam; o->nk_lam = t;
        t = o->ml_eta; o->ml_eta = o->nl_eta; o->nl_eta = t;
        t = o->ml_lam; o->ml_lam = o->nl_lam; o->nl_lam = t;
        o->t += 1;
        if (update_beliefs(o) != 0) return -1;
    }
    return 0;
}

void oracle_beliefs(void *h, double *kf_mu, double *lm_mu, double *kf_lam,
                    double *lm_lam, double *kf_eta, double *lm_eta) {
    oracle_t *o = h;
    if (kf_mu) memcpy(kf_mu, o->kf_mu, sizeof(double) * KD * o->nk);
    if (lm_mu) memcpy(lm_mu, o->lm_mu, sizeof(double) * LD * o->nl);
    if (kf_lam) memcpy(kf_lam, o->kf_lam, sizeof(double) * KD * KD * o->nk);
    if (lm_lam) memcpy(lm_lam, o->lm_lam, sizeof(double) * LD * LD * o->nl);
    if (kf_eta) memcpy(kf_eta, o->kf_eta, sizeof(double) * KD * o->nk);
    if (lm_eta) memcpy(lm_eta, o->lm_eta, sizeof(double) * LD * o->nl);
}

/* Reprojection statistics at the current means (Section 9.1: average
 * reprojection error over the measurements; Section 9.4: a measurement is
 * classed an outlier when it lies in the linear Huber regime).
 * out = {are_all, are_quadratic, n_valid, n_quadratic, n_linear, n_invalid,
 *        are_ref, n_ref, n_linear_ref}; zref/mask optional (both or
 * neither). n_linear_ref counts the linear-regime factors inside the mask:
 * with the mask marking the true inliers, the measurements wrongly classed
 * outliers (the precision of Fig. 7a). */
void oracle_reproj(void *h, double *out, const double *zref, const unsigned char *mask) {
    oracle_t *o = h;
    double cam[4] = { o->fx, o->fy, o->cx, o->cy };
    double s_all = 0, s_q = 0, s_ref = 0;
    long n_valid = 0, n_q = 0, n_lin = 0, n_inv = 0, n_ref = 0, n_lin_ref = 0;
    double N = o->huber_k / o->sigma;
    for (int f = 0; f < o->nf; ++f) {
        double hp[2];
        double pz = oracle_project(o->kf_mu + (size_t)o->f_kf[f]*KD, o->lm_mu + (size_t)o->f_lm[f]*LD, cam, hp, NULL);
        if (!(pz > o->zmin)) { n_inv++; continue; }
        double e = hypot(o->z[2*f] - hp[0], o->z[2*f+1] - hp[1]);
        s_all += e; n_valid++;
        int lin = N > 0.0 && e / o->sigma > N;
        if (lin) n_lin++; else { s_q += e; n_q++; }
        if (zref && mask && mask[f]) {
            s_ref += hypot(zref[2*f] - hp[0], zref[2*f+1] - hp[1]); n_ref++;
            if (lin) n_lin_ref++;
        }
    }
    out[0] = n_valid ? s_all / n_valid : 0.0;
    out[1] = n_q ? s_q / n_q : 0.0;
    out[2] = (double)n_valid; out[3] = (double)n_q; out[4] = (double)n_lin; out[5] = (double)n_inv;
    out[6] = n_ref ? s_ref / n_ref : 0.0; out[7] = (double)n_ref; out[8] = (double)n_lin_ref;
}

/* linearised factor f: eta (9), Lambda (81), linearisation point (9), weight */
void oracle_factor(void *h, int f, double *eta, double *lam, double *lin, double *w) {
    oracle_t *o = h;
    if (eta) memcpy(eta, o->feta + (size_t)f*FD, sizeof(double)*FD);
    if (lam) memcpy(lam, o->flam + (size_t)f*FD*FD, sizeof(double)*FD*FD);
    if (lin) memcpy(lin, o->lin + (size_t)f*FD, sizeof(double)*FD);
    if (w) *w = o->fw[f];
}

/* priors at clock t: diagonal information and information vectors */
void oracle_prior(void *h, int t, double *kf_diag, double *kf_eta, double *lm_diag, double *lm_eta) {
    oracle_t *o = h;
    for (int k = 0; k < o->nk; ++k) kf_prior(o, k, t, kf_diag + (size_t)k*KD, kf_eta + (size_t)k*KD);
    for (int m = 0; m < o->nl; ++m) lm_prior(o, m, t, lm_diag + (size_t)m*LD, lm_eta + (size_t)m*LD);
}

/* current factor-to-variable messages */
void oracle_messages(void *h, double *k_eta, double *k_lam, double *l_eta, double *l_lam) {
    oracle_t *o = h;
    if (k_eta) memcpy(k_eta, o->mk_eta, sizeof(double)*KD*o->nf);
    if (k_lam) memcpy(k_lam, o->mk_lam, sizeof(double)*KD*KD*o->nf);
    if (l_eta) memcpy(l_eta, o->ml_eta, sizeof(double)*LD*o->nf);
    if (l_lam) memcpy(l_lam, o->ml_lam, sizeof(double)*LD*LD*o->nf);
}

/* counters and flags: t, per-factor update count and validity */
int oracle_time(void *h) { return ((oracle_t *)h)->t; }

void oracle_counters(void *h, int *cnt, unsigned char *invalid) {
    oracle_t *o = h;
    if (cnt) memcpy(cnt, o->cnt, sizeof(int) * o->nf);
    if (invalid) memcpy(invalid, o->invalid, o->nf);
}

/* Incremental growth (Section 9.2): append one keyframe with initial pose,
 * n_new_lm landmarks with initial positions and n_new_f factors (indices
 * refer to the enlarged variable sets). New factors are linearised at the
 * current means, new variables get automatic priors built from the new
 * factors and their own annealing clock; beliefs of the new variables start
 * at their priors and existing beliefs are left untouched until the next
 * belief phase. Returns 0 or -1 on bad indices / allocation failure. */
int oracle_add(void *h, int n_new_kf, const double *kf_init, const double *kf_anchor_info,
               int n_new_lm, const double *lm_init,
               int n_new_f, const int *f_kf, const int *f_lm, const double *z) {
    oracle_t *o = h;
    int nk = o->nk + n_new_kf, nl = o->nl + n_new_lm, nf = o->nf + n_new_f;
    for (int i = 0; i < n_new_f; ++i)
        if (f_kf[i] < 0 || f_kf[i] >= nk || f_lm[i] < 0 || f_lm[i] >= nl) return -1;
    if (nk > o->cap_k || nl > o->cap_l || nf > o->cap_f) {
        int ck = nk > o->cap_k ? 2 * nk : o->cap_k;
        int cl = nl > o->cap_l ? 2 * nl : o->cap_l;
        int cf = nf > o->cap_f ? 2 * nf : o->cap_f;
        if (grow(o, ck, cl, cf) != 0) return -1;
    }
    int k0 = o->nk, m0 = o->nl, f0 = o->nf;
    for (int i = 0; i < n_new_kf; ++i) {
        int k = k0 + i;
        memcpy(o->kf_mu + (size_t)k*KD, kf_init + (size_t)i*KD, sizeof(double)*KD);
        memcpy(o->kf_pmean + (size_t)k*KD, kf_init + (size_t)i*KD, sizeof(double)*KD);
        o->kf_anchor[k] = kf_anchor_info ? kf_anchor_info[i] : 0.0;
        o->kf_t0[k] = o->t;
    }
    for (int i = 0; i < n_new_lm; ++i) {
        int m = m0 + i;
        memcpy(o->lm_mu + (size_t)m*LD, lm_init + (size_t)i*LD, sizeof(double)*LD);
        memcpy(o->lm_pmean + (size_t)m*LD, lm_init + (size_t)i*LD, sizeof(double)*LD);
        o->lm_t0[m] = o->t;
    }
    for (int i = 0; i < n_new_f; ++i) {
        int f = f0 + i;
        o->f_kf[f] = f_kf[i]; o->f_lm[f] = f_lm[i];
        o->z[2*f] = z[2*i]; o->z[2*f+1] = z[2*i+1];
    }
    o->nk = nk; o->nl = nl; o->nf = nf;
    o->adj_dirty = 1;
    build_prior_base(o, k0, m0, f0);
    init_new_factors(o, f0);
    /* new variables: belief = prior at the current clock */
    for (int k = k0; k < nk; ++k) {
        double pd[KD], pe[KD];
        kf_prior(o, k, o->t, pd, pe);
        for (int i = 0; i < KD; ++i) {
            o->kf_eta[(size_t)k*KD + i] = pe[i];
            for (int j = 0; j < KD; ++j) o->kf_lam[(size_t)k*KD*KD + i*KD + j] = (i == j) ? pd[i] : 0.0;
        }
    }
    for (int m = m0; m < nl; ++m) {
        double pd[LD], pe[LD];
        lm_prior(o, m, o->t, pd, pe);
        for (int i = 0; i < LD; ++i) {
            o->lm_eta[(size_t)m*LD + i] = pe[i];
            for (int j = 0; j < LD; ++j) o->lm_lam[(size_t)m*LD*LD + i*LD + j] = (i == j) ? pd[i] : 0.0;
        }
    }
    return 0;
}

/* Append n pairwise difference factors of `kind` (0: keyframes, 1:
 * landmarks) between variables a[i] and b[i], measuring x_b - x_a ~
 * N(z[i], diag(prec[i])^-1) (D values each). Their messages start at zero
 * and enter the beliefs from the next belief phase. Returns 0, or -1 on a
 * bad index, a non-positive precision or an allocation failure. */
int oracle_add_pairs(void *h, int kind, int n, const int *a, const int *b, const double *z, const double *prec) {
    oracle_t *o = h;
    if (kind < 0 || kind > 2 || n < 0) return -1;
    const int D = pair_dim(kind), MD = pair_mdim(kind), nv = kind == 1 ? o->nl : o->nk;
    for (int i = 0; i < n; ++i) {
        if (a[i] < 0 || a[i] >= nv || b[i] < 0 || b[i] >= nv || a[i] == b[i]) return -1;
        for (int j = 0; j < MD; ++j) if (!(prec[(size_t)i*MD + j] > 0.0)) return -1;
    }
    struct pairs *q = &o->pr[kind];
    const int nn = q->n + n;
    if (nn > q->cap) {
        const int cap = 2 * nn;
        int **is[] = { &q->a, &q->b, &q->cnt };
        for (int r = 0; r < 3; ++r) {
            int *t = realloc(*is[r], sizeof(int) * cap);
            if (!t) return -1;
            *is[r] = t;
        }
        double **ds[] = { &q->z, &q->p, &q->ma_eta, &q->mb_eta, &q->na_eta, &q->nb_eta };
        for (int r = 0; r < 6; ++r) {
            double *t = realloc(*ds[r], sizeof(double) * cap * (r < 2 ? MD : D));
            if (!t) return -1;
            *ds[r] = t;
        }
        double **ls[] = { &q->ma_lam, &q->mb_lam, &q->na_lam, &q->nb_lam };
        for (int r = 0; r < 4; ++r) {
            double *t = realloc(*ls[r], sizeof(double) * cap * D * D);
            if (!t) return -1;
            *ls[r] = t;
        }
        q->cap = cap;
    }
    for (int i = 0; i < n; ++i) {
        const int f = q->n + i;
        q->a[f] = a[i]; q->b[f] = b[i]; q->cnt[f] = 0;
        memcpy(q->z + (size_t)f*MD, z + (size_t)i*MD, sizeof(double) * MD);
        memcpy(q->p + (size_t)f*MD, prec + (size_t)i*MD, sizeof(double) * MD);
        memset(q->ma_eta + (size_t)f*D, 0, sizeof(double) * D);
        memset(q->mb_eta + (size_t)f*D, 0, sizeof(double) * D);
        memset(q->ma_lam + (size_t)f*D*D, 0, sizeof(double) * D * D);
        memset(q->mb_lam + (size_t)f*D*D, 0, sizeof(double) * D * D);
    }
    q->n = nn;
    return 0;
}

/* current messages of the pairwise factors of `kind` to their a and b ends */
void oracle_pair_messages(void *h, int kind, double *a_eta, double *a_lam, double *b_eta, double *b_lam) {
    oracle_t *o = h;
    const struct pairs *q = &o->pr[kind];
    const int D = pair_dim(kind);
    if (a_eta) memcpy(a_eta, q->ma_eta, sizeof(double) * D * q->n);
    if (a_lam) memcpy(a_lam, q->ma_lam, sizeof(double) * D * D * q->n);
    if (b_eta) memcpy(b_eta, q->mb_eta, sizeof(double) * D * q->n);
    if (b_lam) memcpy(b_lam, q->mb_lam, sizeof(double) * D * D * q->n);
}

/* OpenMP threads for the following calls (results do not depend on it) */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
