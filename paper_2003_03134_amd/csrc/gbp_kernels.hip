// HIP kernels (gfx950) of the synchronous GBP bundle-adjustment sweep.
//
// Mathematical content (Ortiz et al., "Bundle Adjustment on a Graph
// Processor"):
//   - linearisation of the reprojection factor, Section 4, eq. (infform) and
//     the equations after it; Huber rescaling, Section 6;
//   - factor-to-variable messages, Section 5, eqs. (messageeta),
//     (messagelambda), with the variable-to-factor message recovered by
//     dividing the belief by the previous factor-to-variable message;
//   - beliefs, eqs. (beliefeta), (belieflambda); synchronous schedule, local
//     relinearisation, damping, Section 5 and Section 8;
//   - average reprojection error, Section 9.1.
//
// Representation. A linearised reprojection factor has information
// Lambda_f = s J^T J with a 2x9 Jacobian J = [J_k | J_m], so every message it
// sends is a Gaussian over the factor's 2-D measurement space: the message
// to variable v is Lambda = J_v^T S J_v, eta' = J_v^T g with a symmetric 2x2 S
// and a 2-vector g. The Schur complement of eqs. (messageeta) and
// (messagelambda) then reduces to 2x2 algebra: with the belief of v in
// covariance form (Sigma_v, mean offset dmu_v), the cavity (belief divided by
// the previous message, the variable-to-factor message) projected into the
// measurement space has covariance P_c and mean m_c (Woodbury identity), and
// the new message to the other variable u is
//     S_u = s (I + s P_c)^-1,   g_u = S_u (J_u x0_u' + r0 - m_c),
// i.e. the measurement with noise inflated by the cavity's projected
// uncertainty. This is the same quantity as the 9x9 Schur complement of the
// paper, evaluated without forming it.
//
// Coordinates. Every variable has a fixed anchor (its initial estimate, also
// the mean of its prior); beliefs store the mean as an FP64 offset from the
// anchor and the FP64 covariance, and information vectors are kept relative
// to the anchor, so FP32 factor state never carries absolute coordinates.
// Damping the eta message alone (the paper's choice) is not invariant to
// that change of origin; the term d (S_old - S_new) J a restores exactly the
// absolute-coordinate update.
//
// Summation order is fixed (per-landmark loops, per-keyframe lane-strided
// loops and a butterfly reduction, per-problem tree reductions): results are
// bitwise reproducible run to run. No floating-point atomics are used.

#include "gbp_internal.h"
#include "../../include/gbp.h"

#include <hip/hip_ext.h>

#include <algorithm>

namespace gbp {

// --------------------------------------------------------------------------
// small dense helpers
// --------------------------------------------------------------------------

template <int D>
__host__ __device__ constexpr int pidx(int i, int j) {
    // packed upper triangle, row-major
    return i <= j ? i * D - i * (i - 1) / 2 + (j - i) : j * D - j * (j - 1) / 2 + (i - j);
}

template <typename T, int N>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i];
}

__device__ __forceinline__ void load16(const float *__restrict__ p, float (&v)[16]) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float4 a = q[i];
        v[4 * i] = a.x; v[4 * i + 1] = a.y; v[4 * i + 2] = a.z; v[4 * i + 3] = a.w;
    }
}
__device__ __forceinline__ void load16(const double *__restrict__ p, double (&v)[16]) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int i = 0; i < 8; ++i) { double2 a = q[i]; v[2 * i] = a.x; v[2 * i + 1] = a.y; }
}
__device__ __forceinline__ void load12(const float *__restrict__ p, float (&v)[12]) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float4 a = q[i];
        v[4 * i] = a.x; v[4 * i + 1] = a.y; v[4 * i + 2] = a.z; v[4 * i + 3] = a.w;
    }
}
__device__ __forceinline__ void load12(const double *__restrict__ p, double (&v)[12]) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int i = 0; i < 6; ++i) { double2 a = q[i]; v[2 * i] = a.x; v[2 * i + 1] = a.y; }
}

template <typename TS>
__device__ __forceinline__ void load5(const TS *__restrict__ p, TS (&v)[5]) {
#pragma unroll
    for (int i = 0; i < 5; ++i) v[i] = p[i];  // 20-byte records: dword loads, coalesced across lanes
}

__device__ __forceinline__ void load4(const float *__restrict__ p, float (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void load4(const double *__restrict__ p, double (&v)[4]) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
    const double2 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

__device__ __forceinline__ void load2(const float *__restrict__ p, float (&v)[2]) {
    const float2 a = *reinterpret_cast<const float2 *>(p);
    v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void load2(const double *__restrict__ p, double (&v)[2]) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    v[0] = a.x; v[1] = a.y;
}

__device__ __forceinline__ void load8(const float *__restrict__ p, float (&v)[8]) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        float4 a = q[i];
        v[4 * i] = a.x; v[4 * i + 1] = a.y; v[4 * i + 2] = a.z; v[4 * i + 3] = a.w;
    }
}
__device__ __forceinline__ void load8(const double *__restrict__ p, double (&v)[8]) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) { double2 a = q[i]; v[2 * i] = a.x; v[2 * i + 1] = a.y; }
}

// A belief that failed (bit 0: not positive definite, bit 1: not finite):
// the batch's status word, read by the synchronising calls, and its
// problem's, read by the fallback monitor of the learned damping.
template <typename TS>
__device__ __forceinline__ void flag_failure(const Dev<TS> &d, int prob, unsigned bit) {
    atomicOr(d.status, bit);
    atomicOr(d.pstatus + prob, bit);
}

// a non-negative index kept in a record slot of the factor state's type
__device__ __forceinline__ float index_to_slot(int i, float) { return __int_as_float(i); }
__device__ __forceinline__ double index_to_slot(int i, double) { return (double)i; }
__device__ __forceinline__ int slot_to_index(float v) { return __float_as_int(v); }
__device__ __forceinline__ int slot_to_index(double v) { return (int)v; }

// Cholesky of a packed symmetric D x D matrix; returns false when a pivot is
// not positive. L is stored packed by rows of the lower triangle in `L`.
template <int D>
__device__ __forceinline__ bool chol(const double *A, double (&L)[D * (D + 1) / 2]) {
    // lower-triangle packed: row i holds L[i][0..i] at offset i(i+1)/2
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = A[pidx<D>(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * (i + 1) / 2 + i] = sqrt(s);
            } else {
                L[i * (i + 1) / 2 + j] = s / L[j * (j + 1) / 2 + j];
            }
        }
    }
    return true;
}

// Inverse (packed upper) and solution x = A^-1 b from the Cholesky factor.
template <int D>
__device__ __forceinline__ void chol_inverse_solve(const double (&L)[D * (D + 1) / 2], const double (&b)[D],
                                                   double (&inv)[D * (D + 1) / 2], double (&x)[D]) {
    // W = L^-1 (lower triangular)
    double W[D * (D + 1) / 2];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        W[i * (i + 1) / 2 + i] = 1.0 / L[i * (i + 1) / 2 + i];
#pragma unroll
        for (int j = 0; j < i; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) s += L[i * (i + 1) / 2 + k] * W[k * (k + 1) / 2 + j];
            W[i * (i + 1) / 2 + j] = -s * W[i * (i + 1) / 2 + i];
        }
    }
    // A^-1 = W^T W
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < D; ++k) s += W[k * (k + 1) / 2 + i] * W[k * (k + 1) / 2 + j];
            inv[pidx<D>(i, j)] = s;
        }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) s += inv[pidx<D>(i, j)] * b[j];
        x[i] = s;
    }
}

// a wave-uniform double moved into scalar registers
__device__ __forceinline__ double uniform_f64(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// --------------------------------------------------------------------------
// XCD-aware work mapping: workgroups are dispatched round-robin over the
// eight XCDs (each with its own L2); this bijection on [0, n) gives XCD x a
// contiguous range of work items, so neighbouring keyframes, factors and
// landmarks (which share beliefs) meet in the same L2.
// --------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int n) {
    constexpr int NX = 8;
    const int q = n / NX, r = n % NX;
    const int x = b % NX, i = b / NX;
    return x * q + (x < r ? x : r) + i;
}

// --------------------------------------------------------------------------
// measurement model h = pi(R(omega) l + t) and its 2x9 Jacobian (FP64)
// --------------------------------------------------------------------------

struct Lin {
    double J[2][9];
    double r0[2];
    double s;
    bool valid;
};

__device__ __forceinline__ void so3_exp_d(const double w[3], double R[9]) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2), a, b;
    if (th < 1e-5) { a = 1.0 - th2 / 6.0; b = 0.5 - th2 / 24.0; }
    else { a = sin(th) / th; b = (1.0 - cos(th)) / th2; }
    // R = I + a [w]x + b [w]x^2,   [w]x^2 = w w^T - |w|^2 I
    R[0] = 1.0 + b * (w[0] * w[0] - th2);
    R[4] = 1.0 + b * (w[1] * w[1] - th2);
    R[8] = 1.0 + b * (w[2] * w[2] - th2);
    R[1] = -a * w[2] + b * w[0] * w[1];
    R[3] = a * w[2] + b * w[0] * w[1];
    R[2] = a * w[1] + b * w[0] * w[2];
    R[6] = -a * w[1] + b * w[0] * w[2];
    R[5] = -a * w[0] + b * w[1] * w[2];
    R[7] = a * w[0] + b * w[1] * w[2];
}

// right Jacobian of SO(3): I - (1-cos)/th^2 [w]x + (th - sin)/th^3 [w]x^2
__device__ __forceinline__ void so3_jr_d(const double w[3], double Jr[9]) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2), b, c;
    if (th < 1e-5) { b = 0.5 - th2 / 24.0; c = 1.0 / 6.0 - th2 / 120.0; }
    else { b = (1.0 - cos(th)) / th2; c = (th - sin(th)) / (th2 * th); }
    Jr[0] = 1.0 + c * (w[0] * w[0] - th2);
    Jr[4] = 1.0 + c * (w[1] * w[1] - th2);
    Jr[8] = 1.0 + c * (w[2] * w[2] - th2);
    Jr[1] = b * w[2] + c * w[0] * w[1];
    Jr[3] = -b * w[2] + c * w[0] * w[1];
    Jr[2] = -b * w[1] + c * w[0] * w[2];
    Jr[6] = b * w[1] + c * w[0] * w[2];
    Jr[5] = b * w[0] + c * w[1] * w[2];
    Jr[7] = -b * w[0] + c * w[1] * w[2];
}

// Linearise h at (x, l) against measurement z (Section 4); Huber weight w at
// the linearisation point (Section 6) folded into s = w / sigma^2.
__device__ __forceinline__ void linearise(const double x[6], const double l[3], const double z[2],
                                          const ProbParams &pp, double huber_k, Lin &out) {
    double R[9];
    so3_exp_d(x, R);
    double p[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = R[3 * i] * l[0] + R[3 * i + 1] * l[1] + R[3 * i + 2] * l[2] + x[3 + i];
    if (!(p[2] > pp.zmin)) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 9; ++c) out.J[r][c] = 0.0;
        out.r0[0] = out.r0[1] = 0.0;
        out.s = 0.0;
        out.valid = false;
        return;
    }
    double iz = 1.0 / p[2];
    double D[2][3] = {{pp.fx * iz, 0.0, -pp.fx * p[0] * iz * iz}, {0.0, pp.fy * iz, -pp.fy * p[1] * iz * iz}};
    double h0 = pp.fx * p[0] * iz + pp.cx, h1 = pp.fy * p[1] * iz + pp.cy;
    out.r0[0] = z[0] - h0;
    out.r0[1] = z[1] - h1;
    double M = sqrt(out.r0[0] * out.r0[0] + out.r0[1] * out.r0[1]) / pp.sigma;
    double N = huber_k / pp.sigma;
    double w = (N <= 0.0 || M <= N) ? 1.0 : 2.0 * N / M - N * N / (M * M);
    out.s = w * pp.inv_s2;
    out.valid = true;
    // K = R [l]x ; d p / d omega = -K J_r
    double K[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        K[3 * i + 0] = R[3 * i + 1] * l[2] - R[3 * i + 2] * l[1];
        K[3 * i + 1] = -R[3 * i + 0] * l[2] + R[3 * i + 2] * l[0];
        K[3 * i + 2] = R[3 * i + 0] * l[1] - R[3 * i + 1] * l[0];
    }
    double Jr[9];
    so3_jr_d(x, Jr);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        double DK[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) DK[c] = D[r][0] * K[c] + D[r][1] * K[3 + c] + D[r][2] * K[6 + c];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            out.J[r][c] = -(DK[0] * Jr[c] + DK[1] * Jr[3 + c] + DK[2] * Jr[6 + c]);
            out.J[r][3 + c] = D[r][c];
            out.J[r][6 + c] = D[r][0] * R[c] + D[r][1] * R[3 + c] + D[r][2] * R[6 + c];
        }
    }
}

// --------------------------------------------------------------------------
// 2x2 measurement-space marginalisation
// --------------------------------------------------------------------------

// Structural zeros of a factor's Jacobian block (D = 6: the keyframe block,
// whose d h / d t is [[fx/pz, 0, .], [0, fy/pz, .]]; D = 3: none).
template <int D>
__device__ __forceinline__ constexpr bool jac_zero(int r, int c) {
    return D == 6 && ((r == 0 && c == 4) || (r == 1 && c == 3));
}

// Cavity of one variable (its belief divided by this factor's previous
// message S_o, g_o expressed with Jacobian Jo) projected through the
// factor's current Jacobian Jn, its mean relative to the anchor:
//   Pc = Jn Sigma_c Jn^T,  mc = Jn dmu_c.
template <int D>
__device__ __forceinline__ void cavity(const double (&Jo)[2][D], const double (&Jn)[2][D], bool relin,
                                       const double *__restrict__ cov, const double (&dmu)[D], double Sa,
                                       double Sb, double Sc, double g0, double g1, double &Pa, double &Pb,
                                       double &Pc, double &m0, double &m1) {
    double A0[D], A1[D];  // Sigma Jo^T
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double c = cov[pidx<D>(i, j)];
            s0 += c * Jo[0][j];
            s1 += c * Jo[1][j];
        }
        A0[i] = s0;
        A1[i] = s1;
    }
    double poa = 0, pob = 0, poc = 0, jd0 = 0, jd1 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        poa += Jo[0][i] * A0[i];
        pob += Jo[0][i] * A1[i];
        poc += Jo[1][i] * A1[i];
        jd0 += Jo[0][i] * dmu[i];
        jd1 += Jo[1][i] * dmu[i];
    }
    double t00, t01, t10, t11, pna, pnb, pnc, jn0 = 0, jn1 = 0;
    if (relin) {
        t00 = t01 = t10 = t11 = 0.0;
        double B0[D], B1[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            t00 += Jn[0][i] * A0[i];
            t01 += Jn[0][i] * A1[i];
            t10 += Jn[1][i] * A0[i];
            t11 += Jn[1][i] * A1[i];
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double c = cov[pidx<D>(i, j)];
                s0 += c * Jn[0][j];
                s1 += c * Jn[1][j];
            }
            B0[i] = s0;
            B1[i] = s1;
        }
        pna = pnb = pnc = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            pna += Jn[0][i] * B0[i];
            pnb += Jn[0][i] * B1[i];
            pnc += Jn[1][i] * B1[i];
            jn0 += Jn[0][i] * dmu[i];
            jn1 += Jn[1][i] * dmu[i];
        }
    } else {
        t00 = poa; t01 = pob; t10 = pob; t11 = poc;
        pna = poa; pnb = pob; pnc = poc;
        jn0 = jd0;
        jn1 = jd1;
    }
    // M = (I - S Po)^-1
    double e00 = 1.0 - (Sa * poa + Sb * pob), e01 = -(Sa * pob + Sb * poc);
    double e10 = -(Sb * poa + Sc * pob), e11 = 1.0 - (Sb * pob + Sc * poc);
    double idet = 1.0 / (e00 * e11 - e01 * e10);
    double m00 = e11 * idet, m01 = -e01 * idet, m10 = -e10 * idet, m11 = e00 * idet;
    // G = M S (symmetric in exact arithmetic)
    double G00 = m00 * Sa + m01 * Sb, G01 = m00 * Sb + m01 * Sc;
    double G10 = m10 * Sa + m11 * Sb, G11 = m10 * Sb + m11 * Sc;
    double Gs = 0.5 * (G01 + G10);
    // h = M (S Jo dmu - g)
    double v0 = Sa * jd0 + Sb * jd1 - g0, v1 = Sb * jd0 + Sc * jd1 - g1;
    double h0 = m00 * v0 + m01 * v1, h1 = m10 * v0 + m11 * v1;
    // Pc = Pn + T G T^T
    double u00 = t00 * G00 + t01 * Gs, u01 = t00 * Gs + t01 * G11;
    double u10 = t10 * G00 + t11 * Gs, u11 = t10 * Gs + t11 * G11;
    Pa = pna + u00 * t00 + u01 * t01;
    Pb = pnb + 0.5 * ((u00 * t10 + u01 * t11) + (u10 * t00 + u11 * t01));
    Pc = pnc + u10 * t10 + u11 * t11;
    m0 = jn0 + t00 * h0 + t01 * h1;
    m1 = jn1 + t10 * h0 + t11 * h1;
}

// Hot-path cavity (the factor's Jacobian is unchanged since the previous
// message): Po = J Sigma J^T evaluated as a quadratic form over the packed
// covariance, so each covariance entry is used once as it arrives.
template <int D>
__device__ __forceinline__ void cavity_same_j(const double (&J)[2][D], const double *__restrict__ cov,
                                              const double (&dmu)[D], double Sa, double Sb, double Sc,
                                              double g0, double g1, double &Pa, double &Pb, double &Pc,
                                              double &m0, double &m1) {
    // Po = J Sigma J^T, one row of Sigma J^T at a time (products with the
    // structural zeros of the keyframe Jacobian are skipped)
    double poa = 0, pob = 0, poc = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double w = cov[pidx<D>(i, j)];
            if (!jac_zero<D>(0, j)) a0 += w * J[0][j];
            if (!jac_zero<D>(1, j)) a1 += w * J[1][j];
        }
        if (!jac_zero<D>(0, i)) poa += J[0][i] * a0;
        if (!jac_zero<D>(1, i)) {
            pob += J[1][i] * a0;
            poc += J[1][i] * a1;
        }
    }
    double jd0 = 0, jd1 = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (!jac_zero<D>(0, i)) jd0 += J[0][i] * dmu[i];
        if (!jac_zero<D>(1, i)) jd1 += J[1][i] * dmu[i];
    }
    // M = (I - S Po)^-1 ; G = M S ; h = M (S J dmu - g)
    double e00 = 1.0 - (Sa * poa + Sb * pob), e01 = -(Sa * pob + Sb * poc);
    double e10 = -(Sb * poa + Sc * pob), e11 = 1.0 - (Sb * pob + Sc * poc);
    double idet = 1.0 / (e00 * e11 - e01 * e10);
    double m00 = e11 * idet, m01 = -e01 * idet, m10 = -e10 * idet, m11 = e00 * idet;
    double G00 = m00 * Sa + m01 * Sb, G11 = m10 * Sb + m11 * Sc;
    double Gs = 0.5 * ((m00 * Sb + m01 * Sc) + (m10 * Sa + m11 * Sb));
    double v0 = Sa * jd0 + Sb * jd1 - g0, v1 = Sb * jd0 + Sc * jd1 - g1;
    double h0 = m00 * v0 + m01 * v1, h1 = m10 * v0 + m11 * v1;
    // Pc = Po + Po G Po ; mc = J dmu + Po h
    double u00 = poa * G00 + pob * Gs, u01 = poa * Gs + pob * G11;
    double u10 = pob * G00 + poc * Gs, u11 = pob * Gs + poc * G11;
    Pa = poa + u00 * poa + u01 * pob;
    Pb = pob + 0.5 * ((u00 * pob + u01 * poc) + (u10 * poa + u11 * pob));
    Pc = poc + u10 * pob + u11 * poc;
    m0 = jd0 + poa * h0 + pob * h1;
    m1 = jd1 + pob * h0 + poc * h1;
}

// --------------------------------------------------------------------------
// factor phase
// --------------------------------------------------------------------------
//
// One iteration runs k_check (relinearisation check; due factors go to a
// queue per residual block), k_relin (queued factors relinearise and send
// their messages), k_factor_kf (one workgroup per keyframe: every other
// factor of the keyframe sends its messages, then the keyframe's message sums
// are formed in the same kernel) and k_belief_lm (landmark beliefs, with the
// keyframe solves of those sums in its first workgroups). When the residual
// statistics are logged, k_reproj_block also runs the next iteration's check
// and k_relin reduces the statistics, so a logged iteration is four launches.
// Factors are stored sorted by keyframe, so a workgroup's keyframe belief is
// a uniform (scalar) load and its factor records are contiguous.

// One factor's message update (Section 5). RELIN = true relinearises first
// (Section 4) and forms the cavity through both the old and the new
// Jacobian. k and bk are the factor's keyframe and its current belief.
// `stage` (may be null) receives the keyframe-side Jacobian and the new
// stored message for the keyframe belief reduction. fd_on: whether the
// learned per-factor damping applies (its problem has not fallen back); -1:
// look it up for this factor. m_in: the factor's landmark (RELIN); prob, pend_k: its
// problem and the Huber threshold of host-requested relinearisations (read
// by RELIN only, which needs them).
template <typename TS, bool RELIN>
__device__ __forceinline__ void factor_body(const Dev<TS> &d, const IterOpts &o, const int f, const int k,
                                            const int m_in, const double *__restrict__ bk,
                                            const double *__restrict__ ak, TS *__restrict__ stage,
                                            const int fd_on = -1, const int prob = -1,
                                            const double pend_k = 0.0) {
    TS ar[AREC], kr[KREC], lr[LREC], km[KMSG], mm[MMSG];
    load2(d.arec + (size_t)f * AREC, ar);
    load12(d.krec + (size_t)f * KREC, kr);
    // the relinearising caller has the landmark from its queue entry; the
    // keyframe kernel takes it from the keyframe-side record
    const int m = RELIN ? m_in : slot_to_index(kr[11]);
    load5(d.kmsg + (size_t)f * KMSG, km);
    load8(d.lrec + (size_t)f * LREC, lr);
    load5(d.mmsg + (size_t)f * MMSG, mm);
    int c = d.cnt[f];
    const uint8_t fl = d.flags[f];
    const bool use_fd = fd_on < 0 ? (d.fdamp && !d.fallback[d.kf_prob[k]]) : fd_on > 0;
    const float fd = use_fd ? d.fdamp[f] : -1.f;  // issued with the record loads

    const double *bm = d.lm_bel + (size_t)m * LBEL;
    double dmk[6], dmm[3];
#pragma unroll
    for (int i = 0; i < 6; ++i) dmk[i] = bk[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) dmm[i] = bm[i];

    constexpr bool relin = RELIN;

    // current (old) Jacobian blocks
    double Jko[2][6], Jmo[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { Jko[r][i] = (double)kr[3 * r + i]; Jmo[r][i] = (double)lr[3 * r + i]; }
    }
    Jko[0][3] = (double)kr[6]; Jko[0][4] = 0.0; Jko[0][5] = (double)kr[8];
    Jko[1][3] = 0.0; Jko[1][4] = (double)kr[7]; Jko[1][5] = (double)kr[9];
    // linearised residual at the anchors, rho = r0 + J_k d0_k + J_m d0_m
    // (d0: the linearisation point relative to the anchors), and J a of both
    // blocks (the keyframe's from its anchor ak, the landmark's stored)
    double rho0 = (double)ar[0], rho1 = (double)ar[1];
    double s = (double)kr[10];
    double jak0 = 0.0, jak1 = 0.0, jam0 = (double)lr[6], jam1 = (double)lr[7];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (!jac_zero<6>(0, i)) jak0 += Jko[0][i] * ak[i];
        if (!jac_zero<6>(1, i)) jak1 += Jko[1][i] * ak[i];
    }
    const double Ska = km[0], Skb = km[1], Skc = km[2], gk0 = km[3], gk1 = km[4];
    const double Sma = mm[0], Smb = mm[1], Smc = mm[2], gm0 = mm[3], gm1 = mm[4];

    double Jkn[2][6], Jmn[2][3];
    uint8_t nfl = (uint8_t)((fl & ~FLAG_PENDING) | (RELIN ? FLAG_DONE : 0));
    if constexpr (RELIN) {
        const ProbParams pp = d.prob[prob];
        const double hk = (fl & FLAG_PENDING) ? pend_k : o.huber_k;
        double x[6], l[3], zz[2] = {d.z[2 * (size_t)f], d.z[2 * (size_t)f + 1]};
#pragma unroll
        for (int i = 0; i < 6; ++i) x[i] = ak[i] + dmk[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) l[i] = bm[LANC + i] + dmm[i];
        Lin L;
        linearise(x, l, zz, pp, hk, L);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int i = 0; i < 6; ++i) Jkn[r][i] = L.J[r][i];
#pragma unroll
            for (int i = 0; i < 3; ++i) Jmn[r][i] = L.J[r][6 + i];
        }
        s = L.s;
        nfl = L.valid ? (uint8_t)(nfl & ~FLAG_INVALID) : (uint8_t)(nfl | FLAG_INVALID);
        // the new linearisation point is the current mean: d0 = dmu
        rho0 = L.r0[0];
        rho1 = L.r0[1];
#pragma unroll
        for (int i = 0; i < 6; ++i) { rho0 += Jkn[0][i] * dmk[i]; rho1 += Jkn[1][i] * dmk[i]; }
#pragma unroll
        for (int i = 0; i < 3; ++i) { rho0 += Jmn[0][i] * dmm[i]; rho1 += Jmn[1][i] * dmm[i]; }
        jak0 = jak1 = jam0 = jam1 = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            jak0 += Jkn[0][i] * ak[i];
            jak1 += Jkn[1][i] * ak[i];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double a = bm[LANC + i];
            jam0 += Jmn[0][i] * a;
            jam1 += Jmn[1][i] * a;
        }
        c = 0;
    } else {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int i = 0; i < 6; ++i) Jkn[r][i] = Jko[r][i];
#pragma unroll
            for (int i = 0; i < 3; ++i) Jmn[r][i] = Jmo[r][i];
        }
    }

    // cavities of both variables in the factor's measurement space, their
    // means relative to the anchors: m = J dmu_c
    double Pka, Pkb, Pkc, mk0, mk1, Pma, Pmb, Pmc, mm0, mm1;
    if constexpr (RELIN) {
        cavity<6>(Jko, Jkn, relin, bk + 6, dmk, Ska, Skb, Skc, gk0, gk1, Pka, Pkb, Pkc, mk0, mk1);
        cavity<3>(Jmo, Jmn, relin, bm + 3, dmm, Sma, Smb, Smc, gm0, gm1, Pma, Pmb, Pmc, mm0, mm1);
    } else {
        cavity_same_j<3>(Jmo, bm + 3, dmm, Sma, Smb, Smc, gm0, gm1, Pma, Pmb, Pmc, mm0, mm1);
        cavity_same_j<6>(Jko, bk + 6, dmk, Ska, Skb, Skc, gk0, gk1, Pka, Pkb, Pkc, mk0, mk1);
    }

    // new messages: to the landmark through the keyframe cavity and back;
    // the measurement predicted from the other variable's cavity leaves the
    // residual rho - m in the message's anchor-relative coordinates
    double nSm_a, nSm_b, nSm_c, ngm0, ngm1, nSk_a, nSk_b, nSk_c, ngk0, ngk1;
    {
        double qa = 1.0 + s * Pka, qb = s * Pkb, qc = 1.0 + s * Pkc;
        double f0 = s / (qa * qc - qb * qb);
        nSm_a = f0 * qc; nSm_b = -f0 * qb; nSm_c = f0 * qa;
        const double u0 = rho0 - mk0, u1 = rho1 - mk1;
        ngm0 = nSm_a * u0 + nSm_b * u1;
        ngm1 = nSm_b * u0 + nSm_c * u1;
    }
    {
        double qa = 1.0 + s * Pma, qb = s * Pmb, qc = 1.0 + s * Pmc;
        double f0 = s / (qa * qc - qb * qb);
        nSk_a = f0 * qc; nSk_b = -f0 * qb; nSk_c = f0 * qa;
        const double u0 = rho0 - mm0, u1 = rho1 - mm1;
        ngk0 = nSk_a * u0 + nSk_b * u1;
        ngk1 = nSk_b * u0 + nSk_c * u1;
    }

    // damping (Section 5; undamped window of Section 8)
    // (per-factor value from the learned model unless its problem fell back;
    // a negative value means none has been evaluated yet)
    double dd = o.damping;
    if (c < o.undamped) dd = 0.0;
    else if (fd >= 0.f) dd = (double)fd;
    double oSk_a, oSk_b, oSk_c, ogk0, ogk1, oSm_a, oSm_b, oSm_c, ogm0, ogm1;
    if (o.damp_mode == 1) {
        oSk_a = (1 - dd) * nSk_a + dd * Ska; oSk_b = (1 - dd) * nSk_b + dd * Skb; oSk_c = (1 - dd) * nSk_c + dd * Skc;
        oSm_a = (1 - dd) * nSm_a + dd * Sma; oSm_b = (1 - dd) * nSm_b + dd * Smb; oSm_c = (1 - dd) * nSm_c + dd * Smc;
        ogk0 = (1 - dd) * ngk0 + dd * gk0; ogk1 = (1 - dd) * ngk1 + dd * gk1;
        ogm0 = (1 - dd) * ngm0 + dd * gm0; ogm1 = (1 - dd) * ngm1 + dd * gm1;
    } else {
        oSk_a = nSk_a; oSk_b = nSk_b; oSk_c = nSk_c;
        oSm_a = nSm_a; oSm_b = nSm_b; oSm_c = nSm_c;
        // absolute eta damped, Lambda not: anchor-relative correction
        ogk0 = (1 - dd) * ngk0 + dd * gk0 + dd * ((Ska - nSk_a) * jak0 + (Skb - nSk_b) * jak1);
        ogk1 = (1 - dd) * ngk1 + dd * gk1 + dd * ((Skb - nSk_b) * jak0 + (Skc - nSk_c) * jak1);
        ogm0 = (1 - dd) * ngm0 + dd * gm0 + dd * ((Sma - nSm_a) * jam0 + (Smb - nSm_b) * jam1);
        ogm1 = (1 - dd) * ngm1 + dd * gm1 + dd * ((Smb - nSm_b) * jam0 + (Smc - nSm_c) * jam1);
    }

    TS *kw = d.krec + (size_t)f * KREC;
    TS *lw = d.lrec + (size_t)f * LREC;
    TS *mw = d.kmsg + (size_t)f * KMSG;  // dense: full-line writes
    mw[0] = (TS)oSk_a; mw[1] = (TS)oSk_b; mw[2] = (TS)oSk_c; mw[3] = (TS)ogk0; mw[4] = (TS)ogk1;
    TS *nw = d.mmsg + (size_t)f * MMSG;  // dense: full-line writes
    nw[0] = (TS)oSm_a; nw[1] = (TS)oSm_b; nw[2] = (TS)oSm_c; nw[3] = (TS)ogm0; nw[4] = (TS)ogm1;
    if constexpr (RELIN) {
        TS *aw = d.arec + (size_t)f * AREC;
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int i = 0; i < 3; ++i) { kw[3 * r + i] = (TS)Jkn[r][i]; lw[3 * r + i] = (TS)Jmn[r][i]; }
        kw[6] = (TS)Jkn[0][3]; kw[7] = (TS)Jkn[1][4]; kw[8] = (TS)Jkn[0][5]; kw[9] = (TS)Jkn[1][5];
        kw[10] = (TS)s;
        TS *dw = d.drec + (size_t)f * DREC;
        aw[0] = (TS)rho0; aw[1] = (TS)rho1;
        lw[6] = (TS)jam0; lw[7] = (TS)jam1;
#pragma unroll
        for (int i = 0; i < 6; ++i) dw[i] = (TS)dmk[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) dw[6 + i] = (TS)dmm[i];
    }
    d.cnt[f] = (uint8_t)(c + 1 > 255 ? 255 : c + 1);
    if constexpr (RELIN) d.flags[f] = nfl;
    if (stage) {
        // keyframe-side Jacobian and the stored (rounded) message, for the
        // keyframe belief reduction
#pragma unroll
        for (int i = 0; i < 6; ++i) { stage[i] = (TS)Jkn[0][i]; stage[6 + i] = (TS)Jkn[1][i]; }
        stage[12] = (TS)oSk_a; stage[13] = (TS)oSk_b; stage[14] = (TS)oSk_c;
        stage[15] = (TS)ogk0; stage[16] = (TS)ogk1; stage[17] = (TS)0;
    }
}

// Relinearisation check (Section 5, Section 8): a pending request, or at
// least `interval` updates since the last linearisation and the stacked means
// farther than beta from the linearisation point (strictly). fl, cf: the
// factor's flags and update counter; dm: the landmark's mean offset. The
// linearisation point and the keyframe mean are read only for factors old
// enough to be checked.
template <typename TS>
__device__ __forceinline__ bool check_due(const Dev<TS> &d, const IterOpts &o, const int f, const int k,
                                          const uint8_t fl, const int cf, const double dm[3]) {
    bool need = (fl & FLAG_PENDING) != 0;
    const bool old_enough = (cf >= o.interval) & !need;
    if (old_enough) {
        const double *bk = d.kf_bel + (size_t)k * KBEL;
        const TS *dr = d.drec + (size_t)f * DREC;
        double dist2 = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) { double e = bk[i] - (double)dr[i]; dist2 += e * e; }
#pragma unroll
        for (int i = 0; i < 3; ++i) { double e = dm[i] - (double)dr[6 + i]; dist2 += e * e; }
        need = dist2 > o.beta2;
    }
    return need;
}

// The due factors of residual block b (RTHREADS threads, all calling) go to
// the block's own queue segment (wave ballots and a prefix over the block's
// waves: no atomics).
template <typename TS>
__device__ __forceinline__ void queue_due(const Dev<TS> &d, const int b, const int f, const int k, const int m,
                                          const bool need) {
    __shared__ int wcount[RTHREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(need);
    if (lane == 0) wcount[wave] = __popcll(mask);
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < RTHREADS / 64; ++w) {
        base += w < wave ? wcount[w] : 0;
        tot += wcount[w];
    }
    if (need) d.relin_queue[(size_t)b * RBLK + base + __popcll(mask & ((1ull << lane) - 1ull))] = RelinEntry{f, k, m, 0};
    if (threadIdx.x == 0) d.relin_qcount[b] = tot;
}

// Standalone check over the residual blocks (one factor per thread); also
// advances the clock.
template <typename TS>
__global__ __launch_bounds__(RTHREADS) void k_check(Dev<TS> d, IterOpts o) {
    static_assert(RPL == 1, "one factor per thread per residual block");
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int f = d.rblk_start[b] + (int)threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.t_dev[0] = d.t_dev[0] + 1;
    bool need = false;
    int k = 0, m = 0;
    if (f < d.rblk_start[b + 1]) {
        k = d.f_kf[f];
        m = d.f_lm[f];
        const uint8_t fl = d.flags[f];
        const int cf = d.cnt[f];
        const double *bm = d.lm_bel + (size_t)m * LBEL;
        const double dm[3] = {bm[0], bm[1], bm[2]};
        need = check_due(d, o, f, k, fl, cf, dm);
    }
    queue_due(d, b, f, k, m, need);
}

// Tuning load for the relinearisation kernel: every stride-th factor of each
// residual block goes to the block's queue segment, as the check queues due
// factors (stride 11: about the share due per iteration at steady state).
template <typename TS>
__global__ __launch_bounds__(RTHREADS) void k_queue_every(Dev<TS> d, int stride) {
    const int b = blockIdx.x;
    const int f = d.rblk_start[b] + (int)threadIdx.x;
    const bool in = f < d.rblk_start[b + 1];
    queue_due(d, b, f, in ? d.f_kf[f] : 0, in ? d.f_lm[f] : 0, in && (int)threadIdx.x % stride == 0);
}

// One problem's residual statistics from its blocks' partials (64 threads):
// lane l adds blocks l, l + 64, ... in order, then a butterfly adds the lanes
// (a fixed order: deterministic). Writes the 8 sums to out (if set) and a log
// row {t, are_all, are_ref, n_linear, n_linear_ref} (if set), t being the
// clock plus t_off.
__device__ __forceinline__ void reduce_problem(const double *part, const int *prob_blk, const int p, double *out,
                                               double *log_row, const int *t_dev, const int t_off) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = prob_blk[p] + (int)threadIdx.x; b < prob_blk[p + 1]; b += 64)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] += part[8 * (size_t)b + i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    if (threadIdx.x != 0) return;
    if (out)
#pragma unroll
        for (int i = 0; i < 8; ++i) out[8 * (size_t)p + i] = acc[i];
    if (log_row) {
        double *r = log_row + GBP_LOG_COLS * (size_t)p;
        r[0] = (double)(t_dev[0] + t_off);
        r[1] = acc[3] > 0 ? acc[0] / acc[3] : 0.0;
        r[2] = acc[7] > 0 ? acc[2] / acc[7] : 0.0;
        r[3] = acc[5];
        r[4] = acc[4];
    }
}

// One pairwise difference factor between variables a and b of dimension D
// (keyframes: 6, landmarks: 3), measuring x_b - x_a ~ N(z, diag(p)^-1):
// both messages by eqs. (messageeta), (messagelambda). The factor is
// Lambda = [P, -P; -P, P], eta = [-P z; P z] (anchor-relative: z minus the
// anchors' difference); the message to v marginalises the other end u after
// adding u's variable-to-factor message (u's belief in information form,
// stored by the belief kernels, minus this factor's previous message to u):
// S = P + Lambda_c, message Lambda = P - P S^-1 P, eta = +-P z + P S^-1 (eta_c
// -+ P z). Damped like a measurement factor's messages (eta only in absolute
// coordinates, or both; undamped for the first `undamped` updates).
template <typename TS, int D>
__device__ void pair_update(const Dev<TS> &d, const IterOpts &o, const int kind, const int i) {
    constexpr int T = D * (D + 1) / 2, MS = pair_msg_doubles(D);
    const int a = d.pair_ab[kind][2 * i], b = d.pair_ab[kind][2 * i + 1];
    const double *zp = d.pair_zp[kind] + 2 * D * (size_t)i;
    // anchors: keyframes' own array (stride 6), landmarks' in their belief
    // records (stride LBEL)
    const double *anc = kind == 0 ? d.kf_anchor : d.lm_bel + LANC;
    const int AS = kind == 0 ? 6 : LBEL;
    const double *bi = kind == 0 ? d.kf_binfo : d.lm_binfo;
    const int BI = kind == 0 ? KBI : LBI;
    double *msg = d.pair_msg[kind] + MS * (size_t)i;
    double zr[D], P[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        zr[j] = zp[j] - (anc[(size_t)AS * b + j] - anc[(size_t)AS * a + j]);
        P[j] = zp[D + j];
    }
    const int c = d.pair_cnt[kind][i];
    const double dd = c < o.undamped ? 0.0 : o.damping;
    double out[2][D + T];  // new messages to b (side 0) and to a (side 1)
    bool ok = true;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int u = side == 0 ? a : b, v = side == 0 ? b : a;
        const double sv = side == 0 ? 1.0 : -1.0;
        const double *mu = msg + (side == 0 ? 0 : D + T);   // old message to u
        const double *mv = msg + (side == 0 ? D + T : 0);   // old message to v
        const double *bu = bi + (size_t)BI * u;
        double S[T], rhs[D];
#pragma unroll
        for (int q = 0; q < T; ++q) S[q] = bu[q] - mu[D + q];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            S[pidx<D>(j, j)] += P[j];
            rhs[j] = -sv * P[j] * zr[j] + bu[T + j] - mu[j];
        }
        double L[T], inv[T], x[D];
        if (!chol<D>(S, L)) { ok = false; break; }
        chol_inverse_solve<D>(L, rhs, inv, x);
        double *w = out[side];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int q = r; q < D; ++q) w[D + pidx<D>(r, q)] = (r == q ? P[r] : 0.0) - P[r] * inv[pidx<D>(r, q)] * P[q];
#pragma unroll
        for (int r = 0; r < D; ++r) w[r] = sv * P[r] * zr[r] + P[r] * x[r];
        if (o.damp_mode == 1) {
#pragma unroll
            for (int q = 0; q < D + T; ++q) w[q] = (1.0 - dd) * w[q] + dd * mv[q];
        } else {
            // eta damped in absolute coordinates: anchor-relative correction
            double corr[D];
#pragma unroll
            for (int r = 0; r < D; ++r) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < D; ++q) t += (mv[D + pidx<D>(r, q)] - w[D + pidx<D>(r, q)]) * anc[(size_t)AS * v + q];
                corr[r] = t;
            }
#pragma unroll
            for (int r = 0; r < D; ++r) w[r] = (1.0 - dd) * w[r] + dd * mv[r] + dd * corr[r];
        }
    }
    if (!ok) { flag_failure(d, kind == 0 ? d.kf_prob[a] : d.lm_prob[a], 1u); return; }
#pragma unroll
    for (int q = 0; q < D + T; ++q) {
        msg[D + T + q] = out[0][q];  // to b
        msg[q] = out[1][q];          // to a
    }
    d.pair_cnt[kind][i] = c < (1 << 30) ? c + 1 : c;
}

// Camera centre c = -R(omega)^T t of pose x and dc/dx (3x6, row-major):
// dc/domega = [c]x J_r(omega) (from Exp(omega + e) ~ Exp(omega) Exp(J_r e)),
// dc/dt = -R^T.
__device__ __forceinline__ void centre_jacobian(const double x[6], double c[3], double Jc[18]) {
    double R[9], Jr[9];
    so3_exp_d(x, R);
    so3_jr_d(x, Jr);
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = -(R[i] * x[3] + R[3 + i] * x[4] + R[6 + i] * x[5]);
    const double S[9] = {0.0, -c[2], c[1], c[2], 0.0, -c[0], -c[1], c[0], 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Jc[6 * i + j] = S[3 * i] * Jr[j] + S[3 * i + 1] * Jr[3 + j] + S[3 * i + 2] * Jr[6 + j];
            Jc[6 * i + 3 + j] = -R[3 * j + i];
        }
}

// Odometry factor between keyframes a and b: c_b - c_a ~ N(z, diag(p)^-1)
// (3 values), linearised at the current means at every update (so always
// inside the undamped window that follows a relinearisation: undamped).
// With J = [J_a | J_b] = [-dc_a/dx | dc_b/dx] and r = z - h(x0) + J d0
// (d0: the mean offsets from the anchors), the factor is Lambda = J^T P J,
// eta = J^T P r. The message to v marginalises u: S = J_u^T P J_u + Lambda_c,
// y = S^-1 (J_u^T P r + eta_c), Q = J_u S^-1 J_u^T; message Lambda =
// J_v^T (P - P Q P) J_v, eta = J_v^T (P r - P J_u y).
template <typename TS>
__device__ void odometry_update(const Dev<TS> &d, const int i) {
    constexpr int T = 21, MS = pair_msg_doubles(6);
    const int a = d.pair_ab[0][2 * i], b = d.pair_ab[0][2 * i + 1];
    const double *zp = d.pair_zp[0] + 12 * (size_t)i;
    double *msg = d.pair_msg[0] + MS * (size_t)i;
    double xa[6], xb[6], ca[3], cb[3], Ja[18], Jb[18];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        xa[j] = d.kf_anchor[6 * (size_t)a + j] + d.kf_bel[KBEL * (size_t)a + j];
        xb[j] = d.kf_anchor[6 * (size_t)b + j] + d.kf_bel[KBEL * (size_t)b + j];
    }
    centre_jacobian(xa, ca, Ja);
    centre_jacobian(xb, cb, Jb);
    double r[3], P[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double jd = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            jd += -Ja[6 * q + j] * d.kf_bel[KBEL * (size_t)a + j] + Jb[6 * q + j] * d.kf_bel[KBEL * (size_t)b + j];
        r[q] = zp[q] - (cb[q] - ca[q]) + jd;
        P[q] = zp[6 + q];
    }
    double out[2][6 + T];
    bool ok = true;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        // side 0: message to b (u = a, J_u = -Ja); side 1: message to a
        const int u = side == 0 ? a : b;
        const double su = side == 0 ? -1.0 : 1.0, sv = -su;
        const double *Ju = side == 0 ? Ja : Jb, *Jv = side == 0 ? Jb : Ja;
        const double *mu = msg + (side == 0 ? 0 : 6 + T);  // old message to u
        const double *bu = d.kf_binfo + (size_t)KBI * u;
        double S[T], rhs[6];
#pragma unroll
        for (int x = 0; x < 6; ++x) {
#pragma unroll
            for (int y = x; y < 6; ++y) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) t += Ju[6 * q + x] * P[q] * Ju[6 * q + y];  // signs cancel
                S[pidx<6>(x, y)] = t + bu[pidx<6>(x, y)] - mu[6 + pidx<6>(x, y)];
            }
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) t += su * Ju[6 * q + x] * P[q] * r[q];
            rhs[x] = t + bu[21 + x] - mu[x];
        }
        double L[T], inv[T], y[6];
        if (!chol<6>(S, L)) { ok = false; break; }
        chol_inverse_solve<6>(L, rhs, inv, y);
        // Q = J_u S^-1 J_u^T (the signs of J_u cancel), core = P - P Q P
        double core[6], ce[3];
        double JS[3][6];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int x = 0; x < 6; ++x) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < 6; ++w) t += Ju[6 * q + w] * inv[pidx<6>(w, x)];
                JS[q][x] = t;
            }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
#pragma unroll
            for (int s2 = q; s2 < 3; ++s2) {
                double t = 0.0;
#pragma unroll
                for (int x = 0; x < 6; ++x) t += JS[q][x] * Ju[6 * s2 + x];
                core[pidx<3>(q, s2)] = (q == s2 ? P[q] : 0.0) - P[q] * t * P[s2];
            }
            double t = 0.0;
#pragma unroll
            for (int x = 0; x < 6; ++x) t += su * Ju[6 * q + x] * y[x];
            ce[q] = P[q] * r[q] - P[q] * t;
        }
        double *w = out[side];
#pragma unroll
        for (int x = 0; x < 6; ++x) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) t += sv * Jv[6 * q + x] * ce[q];
            w[x] = t;
#pragma unroll
            for (int y2 = x; y2 < 6; ++y2) {
                double s3 = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int q2 = 0; q2 < 3; ++q2) s3 += Jv[6 * q + x] * core[pidx<3>(q, q2)] * Jv[6 * q2 + y2];
                w[6 + pidx<6>(x, y2)] = s3;
            }
        }
    }
    if (!ok) { flag_failure(d, d.kf_prob[a], 1u); return; }
#pragma unroll
    for (int q = 0; q < 6 + T; ++q) {
        msg[6 + T + q] = out[0][q];  // to b
        msg[q] = out[1][q];          // to a
    }
    d.pair_cnt[0][i] = d.pair_cnt[0][i] + 1;
}

// Pairwise factors, one per thread (keyframe pairs first). A kernel of its
// own, launched only while pairs exist: inside the relinearisation launch
// its registers halved that kernel's occupancy.
template <typename TS>
__global__ __launch_bounds__(128) void k_pairs(Dev<TS> d, IterOpts o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.n_pair[0]) {
        if (d.pair_type0[i] == 1) odometry_update<TS>(d, i);
        else pair_update<TS, 6>(d, o, 0, i);
    } else if (i < d.n_pair[0] + d.n_pair[1]) {
        pair_update<TS, 3>(d, o, 1, i - d.n_pair[0]);
    }
}

// Queue segments of the residual blocks: their due factors relinearise and
// send (marked done). A workgroup of two waves takes G consecutive segments
// (tuned; 2 on the 256-problem batch): a segment holds ~22 due factors in
// most iterations, but up to its 256 when a cohort of factors comes due
// together. The workgroups past the segments' (np of them when statistics
// are pending, else none: the launch's grid decides) reduce the residual
// statistics of the previous iteration's fused residual pass (whose check
// advanced the clock: t_off -1) into log_row.
constexpr int RELIN_BS = 128;
constexpr int RELIN_GROUP_MAX = 16;  // queue segments per relinearisation workgroup, at most

// (two waves per SIMD at 252 registers; held to three waves it spills, and
// was slower)
template <typename TS>
__global__ __launch_bounds__(RELIN_BS) __attribute__((amdgpu_waves_per_eu(2))) void k_relin(Dev<TS> d, IterOpts o,
                                                                                            int nseg,
                                                                                            double *log_row) {
    const int G = d.relin_group;
    const int nwg = (nseg + G - 1) / G;
    if ((int)blockIdx.x >= nwg) {
        if (threadIdx.x >= 64) return;  // one wave per problem
        reduce_problem(d.rblk_part, d.prob_rblk, (int)blockIdx.x - nwg, nullptr, log_row, d.t_dev, -1);
        return;
    }
    const double pend_k = d.pending_k[0];
    // G consecutive segments per workgroup, their entries dealt to the lanes
    // in order (entry i of the group: segment g with pre[g] <= i < pre[g+1]);
    // G = 1: one segment, whose problem is the workgroup's
    __shared__ int pre[RELIN_GROUP_MAX + 1];
    const int b0 = (G == 1 ? xcd_remap(blockIdx.x, nseg) : xcd_remap(blockIdx.x, nwg) * G);
    const int gn = min(G, nseg - b0);
    if ((int)threadIdx.x < gn) pre[threadIdx.x + 1] = d.relin_qcount[b0 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int g = 1; g <= gn; ++g) pre[g] += pre[g - 1];
    }
    __syncthreads();
    const int total = pre[gn];
    for (int i = threadIdx.x; i < total; i += RELIN_BS) {
        int g = 0;
        while (g + 1 < gn && pre[g + 1] <= i) ++g;
        const int b = b0 + g;
        // a residual block lies in one problem: its parameters and learned-
        // damping switch hold for all of the block's entries
        const int prob = d.rblk_prob[b];
        const int fd_on = (d.fdamp && !d.fallback[prob]) ? 1 : 0;
        const RelinEntry q = d.relin_queue[(size_t)b * RBLK + (i - pre[g])];
        factor_body<TS, true>(d, o, q.f, q.k, q.m, d.kf_bel + (size_t)q.k * KBEL, d.kf_anchor + 6 * (size_t)q.k,
                              nullptr, fd_on, prob, pend_k);
    }
}

// factors relinearised in the last iteration: sum of the queue segments
__global__ __launch_bounds__(256) void k_relin_total(const int *qcount, int nb, unsigned long long *out) {
    __shared__ unsigned long long sh[256];
    unsigned long long s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += (unsigned long long)qcount[b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

__device__ __forceinline__ double prior_scale(const IterOpts &o, int age) {
    int a = age < 0 ? 0 : (age > o.anneal_iters ? o.anneal_iters : age);
    return o.scale[a];
}

// Keyframe belief (eqs. (beliefeta), (belieflambda)) from the summed
// messages (21 packed information entries, 6 information-vector entries,
// anchor-relative) plus the prior at the current clock; FP64 Cholesky,
// covariance and mean offset; absolute pose for the residual phase.
template <typename TS>
__device__ void kf_solve(const Dev<TS> &d, const IterOpts &o, const int k, const double *sums, const int readout) {
    double A[21], e[6];
#pragma unroll
    for (int i = 0; i < 21; ++i) A[i] = sums[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) e[i] = sums[21 + i];
    const double pinfo = d.kf_pinfo[k];
    if (pinfo > 0.0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) A[pidx<6>(i, i)] += pinfo;
    } else {
        const double sc = prior_scale(o, d.t_dev[0] - d.kf_t0[k]);
#pragma unroll
        for (int i = 0; i < 6; ++i) A[pidx<6>(i, i)] += d.kf_pbase[6 * (size_t)k + i] * sc;
    }
    if (d.kf_binfo) {
        // pairwise factors' messages, then the belief in information form
        // for the next pairwise update
        for (int q = d.kp_row[k]; q < d.kp_row[k + 1]; ++q) {
            const int ent = d.kp_ent[q];
            const double *m = d.pair_msg[0] + pair_msg_doubles(6) * (size_t)(ent >> 1) + (ent & 1) * 27;
#pragma unroll
            for (int i = 0; i < 6; ++i) e[i] += m[i];
#pragma unroll
            for (int i = 0; i < 21; ++i) A[i] += m[6 + i];
        }
        double *bi = d.kf_binfo + KBI * (size_t)k;
#pragma unroll
        for (int i = 0; i < 21; ++i) bi[i] = A[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) bi[21 + i] = e[i];
    }
    if (readout) {
        double *out = d.kf_info + 36 * (size_t)k;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < 6; ++j) out[6 * i + j] = A[pidx<6>(i, j)];
    }
    double L[21], inv[21], x[6];
    if (!chol<6>(A, L)) { flag_failure(d, d.kf_prob[k], 1u); return; }
    chol_inverse_solve<6>(L, e, inv, x);
    bool fin = true;
#pragma unroll
    for (int i = 0; i < 6; ++i) fin = fin && isfinite(x[i]);
    if (!fin) { flag_failure(d, d.kf_prob[k], 2u); return; }
    double *b = d.kf_bel + (size_t)k * KBEL;
#pragma unroll
    for (int i = 0; i < 6; ++i) b[i] = x[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) b[6 + i] = inv[i];
    double w[6], R[9];
#pragma unroll
    for (int i = 0; i < 6; ++i) w[i] = d.kf_anchor[6 * (size_t)k + i] + x[i];
    so3_exp_d(w, R);
    double *ps = d.kf_pose + 12 * (size_t)k;
#pragma unroll
    for (int i = 0; i < 9; ++i) ps[i] = R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) ps[9 + i] = w[3 + i];
}

// Contribution of one factor's keyframe-side message to the keyframe belief
// (eqs. (beliefeta), (belieflambda)): J^T S J (21 packed) and J^T g (6).
template <typename TS>
__device__ __forceinline__ void kf_contrib(const TS *row, TS *c) {
    double J0[6], J1[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) { J0[i] = (double)row[i]; J1[i] = (double)row[6 + i]; }
    const double Sa = row[12], Sb = row[13], Sc = row[14], g0 = row[15], g1 = row[16];
    // (the keyframe Jacobian's structural zeros drop out exactly)
    double SJ0[6], SJ1[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        SJ0[j] = jac_zero<6>(0, j) ? Sb * J1[j] : jac_zero<6>(1, j) ? Sa * J0[j] : Sa * J0[j] + Sb * J1[j];
        SJ1[j] = jac_zero<6>(0, j) ? Sc * J1[j] : jac_zero<6>(1, j) ? Sb * J0[j] : Sb * J0[j] + Sc * J1[j];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = i; j < 6; ++j)
            c[pidx<6>(i, j)] = (TS)(jac_zero<6>(0, i)   ? J1[i] * SJ1[j]
                                    : jac_zero<6>(1, i) ? J0[i] * SJ0[j]
                                                        : J0[i] * SJ0[j] + J1[i] * SJ1[j]);
        c[21 + i] = (TS)(jac_zero<6>(0, i) ? J1[i] * g1 : jac_zero<6>(1, i) ? J0[i] * g0 : J0[i] * g0 + J1[i] * g1);
    }
}

// One workgroup per keyframe. MODE 0: every factor of the keyframe not
// relinearised this iteration sends its messages, then the keyframe's
// message sums (information and information vector) are formed; MODE 1:
// sums only (creation, read-out). k_kf_solve turns the sums into beliefs.
// Each lane forms its factor's 27 contributions and writes them, rounded to
// the factor-state precision, to a padded LDS row; 27 x G lanes then add
// interleaved rows column by column in FP64 and the G partials are added in
// group order (fixed order, no cross-lane shuffles).
// FP32 factor state: four waves per SIMD (126 registers, no spill). The
// target once held the kernel, then at 137 registers, to 128 with a 12-byte
// spill, 4% faster than three waves; it now keeps a change from silently
// costing a wave. (No target for FP64 factor state, which cannot reach it.)
template <typename TS, int BS>
constexpr int kf_waves_per_eu() { return sizeof(TS) == 4 ? 4 : 1; }

template <typename TS, int BS, int MODE>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(kf_waves_per_eu<TS, BS>()))) void k_factor_kf(
    Dev<TS> d, IterOpts o) {
    constexpr int G = BS / 32;     // row groups in the column sums
    constexpr int RS = 29;         // padded row stride (elements) against bank conflicts
    __shared__ TS red[BS * RS];
    __shared__ double part[G][28];
    // slot -> keyframe, its factor range and problem (per-XCD runs; k = -1:
    // no keyframe)
    const KfSlot sl = d.kf_slot[blockIdx.x];
    const int k = sl.k;
    if (k < 0) return;
    const int tid = threadIdx.x;
    const int e0 = sl.e0, e1 = sl.e1;
    // the keyframe's belief is the same for every lane: broadcast it into
    // scalar registers (loaded per lane, the compiler would keep 54 vector
    // registers for it, since it cannot rule out that the record stores
    // alias the belief array)
    double kb[27], ka[6];
#pragma unroll
    for (int i = 0; i < 27; ++i) kb[i] = uniform_f64(d.kf_bel[(size_t)k * KBEL + i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) ka[i] = uniform_f64(d.kf_anchor[6 * (size_t)k + i]);
    const double *bk = kb;
    // learned damping: on unless absent or the keyframe's problem fell back
    // (the same for the whole workgroup)
    const int fd_on = (d.fdamp && !d.fallback[sl.prob]) ? 1 : 0;
    const int col = tid % 27, grp = tid / 27;
    double acc = 0.0;
    for (int base = e0; base < e1; base += BS) {
        const int f = base + tid;
        TS row[18];
#pragma unroll
        for (int i = 0; i < 18; ++i) row[i] = (TS)0;
        if (f < e1) {
            const uint8_t fl = d.flags[f];
            if (MODE == 0 && !(fl & FLAG_DONE)) {
                factor_body<TS, false>(d, o, f, k, -1, bk, ka, row, fd_on);
            } else {
                TS kr[KREC], km[KMSG];
                load12(d.krec + (size_t)f * KREC, kr);
                load5(d.kmsg + (size_t)f * KMSG, km);
                row[0] = kr[0]; row[1] = kr[1]; row[2] = kr[2]; row[3] = kr[6]; row[5] = kr[8];
                row[6] = kr[3]; row[7] = kr[4]; row[8] = kr[5]; row[10] = kr[7]; row[11] = kr[9];
                row[12] = km[0]; row[13] = km[1]; row[14] = km[2]; row[15] = km[3]; row[16] = km[4];
                if (MODE == 0) d.flags[f] = (uint8_t)(fl & ~FLAG_DONE);
            }
        }
        kf_contrib<TS>(row, red + tid * RS);
        __syncthreads();
        if (grp < G) {
            // rows grp, grp + G, ... in order; a fixed trip count lets the
            // LDS reads go out together instead of one round trip per row
            static_assert(BS % G == 0, "whole rows per group");
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < BS / G; ++r) s += (double)red[(grp + r * G) * RS + col];
            part[grp][col] = s;
        }
        __syncthreads();
        if (tid < 27)
#pragma unroll
            for (int g = 0; g < G; ++g) acc += part[g][tid];
        __syncthreads();
    }
    if (tid < 27) d.kf_sums[32 * (size_t)k + tid] = acc;
}

// one thread per keyframe: belief from the summed messages (k_factor_kf)
template <typename TS>
__global__ __launch_bounds__(64) void k_kf_solve(Dev<TS> d, IterOpts o, int readout) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.nk) return;
    double s[27];
    const double *src = d.kf_sums + 32 * (size_t)k;
#pragma unroll
    for (int i = 0; i < 27; ++i) s[i] = src[i];
    kf_solve<TS>(d, o, k, s, readout);
}

// --------------------------------------------------------------------------
// features of the learned damping / depth network (one row of 16 per factor)
// --------------------------------------------------------------------------
//
// 0 residual at the linearisation point / Huber threshold, 1 Huber weight,
// 2 log(1 + residual / sigma), 3 updates since the last linearisation / 10,
// 4 log(1 + distance from the linearisation point / beta), 5-6 relative
// change of the keyframe- and landmark-side message vectors since the last
// evaluation, 7 relative change of the landmark-side message information,
// 8 cosine between the last two landmark-side message changes, 9 log(depth /
// 5 m), 10-11 log degrees of landmark and keyframe, 12 log trace of the
// landmark covariance / 10, 13 cosine between the last two keyframe-side
// message changes, 14 iteration / 300, 15 log(1 + predicted pixel shift of
// the landmark since linearisation). `hist` keeps FHIST values per factor
// between evaluations: g_k (2), g_m (2), tr S_m, last change of g_m (2),
// valid flag, last change of g_k (2), pad (2).
// a feature row: FP32 (export) or BF16 bits (the in-loop network input,
// rounded to nearest even as the network would round it)
__device__ __forceinline__ void store_features(float *__restrict__ p, const float (&x)[NFEAT]) {
    float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int i = 0; i < NFEAT / 4; ++i) q[i] = make_float4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
}
__device__ __forceinline__ void store_features(uint16_t *__restrict__ p, const float (&x)[NFEAT]) {
    uint32_t w[NFEAT / 2];
#pragma unroll
    for (int i = 0; i < NFEAT / 2; ++i) {
        const uint32_t lo = __builtin_bit_cast(uint16_t, (__bf16)x[2 * i]);
        const uint32_t hi = __builtin_bit_cast(uint16_t, (__bf16)x[2 * i + 1]);
        w[i] = lo | (hi << 16);
    }
    uint4 *q = reinterpret_cast<uint4 *>(p);
    q[0] = make_uint4(w[0], w[1], w[2], w[3]);
    q[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

template <typename TS, typename FT>
__global__ __launch_bounds__(256) void k_features(Dev<TS> d, IterOpts o, FT *__restrict__ feat,
                                                  float *__restrict__ hist, double huber_k) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.nf) return;
    const int k = d.f_kf[f], m = d.f_lm[f];
    TS kr[KREC], lr[LREC], ar[AREC], dr[DREC], km[KMSG], mm[MMSG];
    load12(d.krec + (size_t)f * KREC, kr);
    load5(d.kmsg + (size_t)f * KMSG, km);
    load8(d.lrec + (size_t)f * LREC, lr);
    load5(d.mmsg + (size_t)f * MMSG, mm);
    load2(d.arec + (size_t)f * AREC, ar);
    load12(d.drec + (size_t)f * DREC, dr);
    const ProbParams pp = d.prob[d.kf_prob[k]];
    const double *bk = d.kf_bel + (size_t)k * KBEL, *bm = d.lm_bel + (size_t)m * LBEL;
    // residual at the linearisation point: r0 = rho - J_k d0_k - J_m d0_m
    double r00 = (double)ar[0], r01 = (double)ar[1];
    for (int i = 0; i < 3; ++i) {
        r00 -= (double)kr[i] * dr[i] + (double)lr[i] * dr[6 + i];
        r01 -= (double)kr[3 + i] * dr[i] + (double)lr[3 + i] * dr[6 + i];
    }
    r00 -= (double)kr[6] * dr[3] + (double)kr[8] * dr[5];
    r01 -= (double)kr[7] * dr[4] + (double)kr[9] * dr[5];
    const double M0 = sqrt(r00 * r00 + r01 * r01) / pp.sigma;
    const double N = huber_k / pp.sigma;
    double dist2 = 0.0;
    for (int i = 0; i < 6; ++i) { double e = bk[i] - (double)dr[i]; dist2 += e * e; }
    for (int i = 0; i < 3; ++i) { double e = bm[i] - (double)dr[6 + i]; dist2 += e * e; }
    double ju0 = 0, ju1 = 0;
    for (int i = 0; i < 3; ++i) {
        const double e = bm[i] - (double)dr[6 + i];
        ju0 += (double)lr[i] * e;
        ju1 += (double)lr[3 + i] * e;
    }
    const float gk0 = km[3], gk1 = km[4], gm0 = mm[3], gm1 = mm[4], trS = (float)mm[0] + (float)mm[2];
    float *h = hist + FHIST * (size_t)f;
    const bool have = h[7] > 0.5f;
    const float dk0 = gk0 - h[0], dk1 = gk1 - h[1], dm0 = gm0 - h[2], dm1 = gm1 - h[3];
    const float nk = sqrtf(gk0 * gk0 + gk1 * gk1), nkp = sqrtf(h[0] * h[0] + h[1] * h[1]);
    const float nm = sqrtf(gm0 * gm0 + gm1 * gm1), nmp = sqrtf(h[2] * h[2] + h[3] * h[3]);
    const float ndm = sqrtf(dm0 * dm0 + dm1 * dm1), ndmp = sqrtf(h[5] * h[5] + h[6] * h[6]);
    const float ndk = sqrtf(dk0 * dk0 + dk1 * dk1), ndkp = sqrtf(h[8] * h[8] + h[9] * h[9]);
    float x[NFEAT];
    x[0] = N > 0.0 ? (float)fmin(M0 / N, 10.0) : 0.f;
    x[1] = (float)((double)kr[10] / pp.inv_s2);
    x[2] = (float)log1p(M0);
    x[3] = fminf((float)d.cnt[f], 30.f) / 10.f;
    x[4] = (float)log1p(sqrt(dist2) / sqrt(o.beta2 > 0.0 ? o.beta2 : 1e-4));
    x[5] = have ? sqrtf(dk0 * dk0 + dk1 * dk1) / (nk + nkp + 1e-6f) : 0.f;
    x[6] = have ? ndm / (nm + nmp + 1e-6f) : 0.f;
    x[7] = have ? fabsf(trS - h[4]) / (fabsf(trS) + fabsf(h[4]) + 1e-12f) : 0.f;
    x[8] = have ? (dm0 * h[5] + dm1 * h[6]) / (ndm * ndmp + 1e-12f) : 0.f;
    const double a0 = (double)kr[6];
    x[9] = a0 > 0.0 ? (float)log(pp.fx / a0 / 5.0) : 0.f;
    x[10] = logf((float)(d.lm_row[m + 1] - d.lm_row[m]));
    x[11] = logf((float)(d.kf_row[k + 1] - d.kf_row[k]));
    const double trc = bm[3 + pidx<3>(0, 0)] + bm[3 + pidx<3>(1, 1)] + bm[3 + pidx<3>(2, 2)];
    x[12] = (float)fmin(fmax(log(trc > 0.0 ? trc : 1e-30), -30.0), 10.0) / 10.f;
    x[13] = have ? (dk0 * h[8] + dk1 * h[9]) / (ndk * ndkp + 1e-12f) : 0.f;
    x[14] = fminf((float)d.t_dev[0], 300.f) / 300.f;
    x[15] = (float)log1p(sqrt(ju0 * ju0 + ju1 * ju1));
    store_features(feat + NFEAT * (size_t)f, x);
    h[0] = gk0; h[1] = gk1; h[2] = gm0; h[3] = gm1; h[4] = trS;
    h[5] = have ? dm0 : 0.f; h[6] = have ? dm1 : 0.f; h[7] = 1.f;
    h[8] = have ? dk0 : 0.f; h[9] = have ? dk1 : 0.f;
}

__global__ void k_fill_f32(float *p, float v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// dst row i = src row u2i[idx[i]] (width w); an index outside [0, nf) gives a
// row of NaN
__global__ void k_gather_rows(const float *__restrict__ src, float *__restrict__ dst, const int *__restrict__ idx,
                              const int *__restrict__ u2i, int nf, int n, int w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int u = idx[i];
    if (u < 0 || u >= nf) {
        for (int c = 0; c < w; ++c) dst[(size_t)i * w + c] = __int_as_float(0x7fc00000);
        return;
    }
    const int j = u2i[u];
    for (int c = 0; c < w; ++c) dst[(size_t)i * w + c] = src[(size_t)j * w + c];
}

// per-factor messages and counters: S_k (3), g_k (2), S_m (3), g_m (2),
// updates since linearisation, flags, J_k a_k (2), J_m a_m (2)
template <typename TS>
__global__ void k_export_messages(Dev<TS> d, const int *__restrict__ idx, const int *__restrict__ u2i, int n,
                                  float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *o = out + MSG_W * (size_t)i;
    const int u = idx[i];
    if (u < 0 || u >= d.nf) {
        for (int c = 0; c < MSG_W; ++c) o[c] = __int_as_float(0x7fc00000);
        return;
    }
    const int f = u2i[u];
    const TS *kr = d.krec + (size_t)f * KREC, *lr = d.lrec + (size_t)f * LREC;
    const TS *km = d.kmsg + (size_t)f * KMSG;
    for (int c = 0; c < 5; ++c) o[c] = (float)km[c];
    const TS *mm = d.mmsg + (size_t)f * MMSG;
    for (int c = 0; c < 5; ++c) o[5 + c] = (float)mm[c];
    o[10] = (float)d.cnt[f];
    o[11] = (float)d.flags[f];
    // J_k anchor_k from the keyframe-side Jacobian and the keyframe's anchor
    const int k = d.f_kf[f];
    const double *ak = d.kf_anchor + 6 * (size_t)k;
    double ja0 = 0.0, ja1 = 0.0;
    for (int i = 0; i < 3; ++i) {
        ja0 += (double)kr[i] * ak[i];
        ja1 += (double)kr[3 + i] * ak[i];
    }
    ja0 += (double)kr[6] * ak[3] + (double)kr[8] * ak[5];
    ja1 += (double)kr[7] * ak[4] + (double)kr[9] * ak[5];
    o[12] = (float)ja0; o[13] = (float)ja1;
    o[14] = (float)lr[6]; o[15] = (float)lr[7];
}

// --------------------------------------------------------------------------
// linearise new factors at the current means (creation / growth)
// --------------------------------------------------------------------------

template <typename TS>
__global__ __launch_bounds__(256) void k_linearise(Dev<TS> d, int f0, int f1, double huber_k, const int *list) {
    const int i = f0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f1) return;
    const int f = list ? list[i] : i;
    const int k = d.f_kf[f], m = d.f_lm[f];
    const ProbParams pp = d.prob[d.kf_prob[k]];
    double x[6], l[3], dmk[6], dmm[3], zz[2] = {d.z[2 * (size_t)f], d.z[2 * (size_t)f + 1]};
#pragma unroll
    for (int i = 0; i < 6; ++i) { dmk[i] = d.kf_bel[(size_t)k * KBEL + i]; x[i] = d.kf_anchor[6 * (size_t)k + i] + dmk[i]; }
#pragma unroll
    for (int i = 0; i < 3; ++i) { dmm[i] = d.lm_bel[(size_t)m * LBEL + i]; l[i] = d.lm_bel[(size_t)m * LBEL + LANC + i] + dmm[i]; }
    Lin L;
    linearise(x, l, zz, pp, huber_k, L);
    TS *kw = d.krec + (size_t)f * KREC, *lw = d.lrec + (size_t)f * LREC, *aw = d.arec + (size_t)f * AREC;
    TS *dw = d.drec + (size_t)f * DREC;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i) { kw[3 * r + i] = (TS)L.J[r][i]; lw[3 * r + i] = (TS)L.J[r][6 + i]; }
    kw[6] = (TS)L.J[0][3]; kw[7] = (TS)L.J[1][4]; kw[8] = (TS)L.J[0][5]; kw[9] = (TS)L.J[1][5];
    kw[10] = (TS)L.s;
    kw[11] = index_to_slot(m, TS(0));
    TS *mw = d.kmsg + (size_t)f * KMSG;
#pragma unroll
    for (int i = 0; i < KMSG; ++i) mw[i] = (TS)0;
    TS *nw = d.mmsg + (size_t)f * MMSG;
#pragma unroll
    for (int i = 0; i < MMSG; ++i) nw[i] = (TS)0;
    // rho = r0 + J (x0 - anchor) with the linearisation point at the means
    double rho0 = L.r0[0], rho1 = L.r0[1];
#pragma unroll
    for (int i = 0; i < 6; ++i) { rho0 += L.J[0][i] * dmk[i]; rho1 += L.J[1][i] * dmk[i]; dw[i] = (TS)dmk[i]; }
#pragma unroll
    for (int i = 0; i < 3; ++i) { rho0 += L.J[0][6 + i] * dmm[i]; rho1 += L.J[1][6 + i] * dmm[i]; dw[6 + i] = (TS)dmm[i]; }
#pragma unroll
    for (int i = 9; i < DREC; ++i) dw[i] = (TS)0;
    aw[0] = (TS)rho0; aw[1] = (TS)rho1;
    double jam0 = 0, jam1 = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double a = d.lm_bel[(size_t)m * LBEL + LANC + i];
        jam0 += L.J[0][6 + i] * a;
        jam1 += L.J[1][6 + i] * a;
    }
    lw[6] = (TS)jam0; lw[7] = (TS)jam1;
    d.cnt[f] = 0;
    d.flags[f] = L.valid ? 0 : FLAG_INVALID;
}

// --------------------------------------------------------------------------
// automatic priors: diag(sum_f J_v^T Sigma^-1 J_v) at the initial
// linearisation (Section 4), floored so that every belief is proper
// --------------------------------------------------------------------------

constexpr double PRIOR_FLOOR = 1e-8;

template <typename TS>
__global__ __launch_bounds__(256) void k_prior_kf(Dev<TS> d, int k0) {
    const int k = k0 + ((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= d.nk) return;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int f = d.kf_row[k] + lane; f < d.kf_row[k + 1]; f += 64) {
        const TS *r = d.krec + (size_t)f * KREC;
        double j00 = r[0], j01 = r[1], j02 = r[2], j10 = r[3], j11 = r[4], j12 = r[5];
        double a0 = r[6], a1 = r[7], b0 = r[8], b1 = r[9];
        acc[0] += j00 * j00 + j10 * j10;
        acc[1] += j01 * j01 + j11 * j11;
        acc[2] += j02 * j02 + j12 * j12;
        acc[3] += a0 * a0;
        acc[4] += a1 * a1;
        acc[5] += b0 * b0 + b1 * b1;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    if (lane == 0) {
        const double is2 = d.prob[d.kf_prob[k]].inv_s2;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            double v = acc[i] * is2;
            d.kf_pbase[6 * (size_t)k + i] = v < PRIOR_FLOOR ? PRIOR_FLOOR : v;
        }
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void k_prior_lm(Dev<TS> d, int m0) {
    const int m = m0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.nl) return;
    double acc[3] = {0, 0, 0};
    for (int e = d.lm_row[m]; e < d.lm_row[m + 1]; ++e) {
        const TS *r = d.lrec + (size_t)d.lm_edge[e] * LREC;
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i] += (double)r[i] * (double)r[i] + (double)r[3 + i] * (double)r[3 + i];
    }
    const double is2 = d.prob[d.lm_prob[m]].inv_s2;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double v = acc[i] * is2;
        d.lm_pbase[3 * (size_t)m + i] = v < PRIOR_FLOOR ? PRIOR_FLOOR : v;
    }
}

// --------------------------------------------------------------------------
// belief phase (eqs. (beliefeta), (belieflambda)): prior at the current
// clock plus the sum of incoming messages, then covariance and mean offset
// --------------------------------------------------------------------------


// one factor's message to its landmark, J^T S J and J^T g with the message
// in measurement space (S packed 2x2, g), added to the landmark's sums
template <typename TS>
__device__ __forceinline__ void lm_edge_add(double A[6], double e[3], const TS *r, const TS *mr) {
    double J0[3] = {r[0], r[1], r[2]}, J1[3] = {r[3], r[4], r[5]};
    double Sa = mr[0], Sb = mr[1], Sc = mr[2], g0 = mr[3], g1 = mr[4];
    double SJ0[3], SJ1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) { SJ0[j] = Sa * J0[j] + Sb * J1[j]; SJ1[j] = Sb * J0[j] + Sc * J1[j]; }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = i; j < 3; ++j) A[pidx<3>(i, j)] += J0[i] * SJ0[j] + J1[i] * SJ1[j];
        e[i] += J0[i] * g0 + J1[i] * g1;
    }
}

constexpr int BEL_UNR = 2;   // landmark edges in flight per lane

template <typename TS, int LANES, bool WITH_KF>
__global__ __launch_bounds__(256) void k_belief_lm(Dev<TS> d, IterOpts o, int readout, int nkb) {
    // WITH_KF: the first nkb workgroups turn the keyframe message sums into
    // keyframe beliefs (one thread per keyframe, as k_kf_solve), overlapping
    // that short serial solve with the landmark beliefs, which do not depend
    // on it.
    int bid = blockIdx.x, nb = gridDim.x;
    if constexpr (WITH_KF) {
        if (bid < nkb) {
            const int k = bid * blockDim.x + threadIdx.x;
            if (k < d.nk) {
                double sm[27];
                const double *src = d.kf_sums + 32 * (size_t)k;
#pragma unroll
                for (int i = 0; i < 27; ++i) sm[i] = src[i];
                kf_solve<TS>(d, o, k, sm, 0);
            }
            return;
        }
        bid -= nkb;
        nb -= nkb;
    }
    // LANES lanes per landmark: lane q of a group sums edges q, q + LANES,
    // ... (in order), then the group adds its partial sums with a fixed
    // butterfly; every lane of the group ends with the same sums
    const int gid = xcd_remap(bid, nb) * blockDim.x + threadIdx.x;
    const int m = gid / LANES, q = gid % LANES;
    const bool live = m < d.nl;
    double A[6] = {0, 0, 0, 0, 0, 0}, e[3] = {0, 0, 0};
    if (live) {
        // the edge gathers are a chain of two dependent loads (edge index,
        // then records): BEL_UNR edges' records are requested before the
        // first is used, and added in edge order as in the one-edge tail
        const int e1 = d.lm_row[m + 1];
        int ei = d.lm_row[m] + q;
        for (; ei + (BEL_UNR - 1) * LANES < e1; ei += BEL_UNR * LANES) {
            int fe[BEL_UNR];
#pragma unroll
            for (int u = 0; u < BEL_UNR; ++u) fe[u] = d.lm_edge[ei + u * LANES];
            TS r[BEL_UNR][LREC], mr[BEL_UNR][MMSG];
#pragma unroll
            for (int u = 0; u < BEL_UNR; ++u) {
                load8(d.lrec + (size_t)fe[u] * LREC, r[u]);
                load5(d.mmsg + (size_t)fe[u] * MMSG, mr[u]);
            }
#pragma unroll
            for (int u = 0; u < BEL_UNR; ++u) lm_edge_add(A, e, r[u], mr[u]);
        }
        for (; ei < e1; ei += LANES) {
            const int fe = d.lm_edge[ei];
            TS r[LREC], mr[MMSG];
            load8(d.lrec + (size_t)fe * LREC, r);
            load5(d.mmsg + (size_t)fe * MMSG, mr);
            lm_edge_add(A, e, r, mr);
        }
    }
#pragma unroll
    for (int off = 1; off < LANES; off <<= 1) {
#pragma unroll
        for (int i = 0; i < 6; ++i) A[i] += __shfl_xor(A[i], off, 64);
#pragma unroll
        for (int i = 0; i < 3; ++i) e[i] += __shfl_xor(e[i], off, 64);
    }
    if (!live || q != 0) return;
    const int t = d.t_dev[0];
    const double sc = prior_scale(o, t - d.lm_t0[m]);
    A[pidx<3>(0, 0)] += d.lm_pbase[3 * (size_t)m] * sc;
    A[pidx<3>(1, 1)] += d.lm_pbase[3 * (size_t)m + 1] * sc;
    A[pidx<3>(2, 2)] += d.lm_pbase[3 * (size_t)m + 2] * sc;
    if (d.lm_binfo) {
        for (int q = d.lp_row[m]; q < d.lp_row[m + 1]; ++q) {
            const int ent = d.lp_ent[q];
            const double *pm = d.pair_msg[1] + pair_msg_doubles(3) * (size_t)(ent >> 1) + (ent & 1) * 9;
#pragma unroll
            for (int i = 0; i < 3; ++i) e[i] += pm[i];
#pragma unroll
            for (int i = 0; i < 6; ++i) A[i] += pm[3 + i];
        }
        double *bi = d.lm_binfo + LBI * (size_t)m;
#pragma unroll
        for (int i = 0; i < 6; ++i) bi[i] = A[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) bi[6 + i] = e[i];
    }
    if (readout) {
        double *out = d.lm_info + 9 * (size_t)m;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) out[3 * i + j] = A[pidx<3>(i, j)];
    }
    double L[6], inv[6], x[3];
    if (!chol<3>(A, L)) { flag_failure(d, d.lm_prob[m], 1u); return; }
    chol_inverse_solve<3>(L, e, inv, x);
    bool fin = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) fin = fin && isfinite(x[i]);
    if (!fin) { flag_failure(d, d.lm_prob[m], 2u); return; }
    double *b = d.lm_bel + (size_t)m * LBEL;
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = x[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) b[3 + i] = inv[i];
}

// --------------------------------------------------------------------------
// relinearisation requests (explicit call): mark and count
// --------------------------------------------------------------------------

template <typename TS>
__global__ __launch_bounds__(256) void k_flag_relin(Dev<TS> d, double beta, int *count) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.nf) return;
    bool sel = beta < 0.0;
    // a factor already marked takes the current means as its linearisation
    // point, so its distance is zero: only beta < 0 selects it again
    if (!sel && !(d.flags[f] & FLAG_PENDING)) {
        const int k = d.f_kf[f], m = d.f_lm[f];
        const TS *dr = d.drec + (size_t)f * DREC;
        double dist2 = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) { double e = d.kf_bel[(size_t)k * KBEL + i] - (double)dr[i]; dist2 += e * e; }
#pragma unroll
        for (int i = 0; i < 3; ++i) { double e = d.lm_bel[(size_t)m * LBEL + i] - (double)dr[6 + i]; dist2 += e * e; }
        sel = sqrt(dist2) > beta;
    }
    if (sel) {
        d.flags[f] = d.flags[f] | FLAG_PENDING;
        atomicAdd(count, 1);
    }
}

// --------------------------------------------------------------------------
// reprojection statistics (Section 9.1, Section 9.4 outlier classes)
// --------------------------------------------------------------------------

// Per-block partial statistics over the factor range of one block (blocks
// never straddle problems): {sum_all, sum_quad, sum_ref, n_valid, n_lin_ref,
// n_lin, n_inv, n_ref}. Each lane takes the block's factors tid, tid + 256,
// ... in order; the wave adds its three error sums with a butterfly and
// counts its flags with ballots, then the four waves are added in order (a
// fixed order: deterministic). CHECK: the same pass also runs the next
// iteration's relinearisation check on the updated beliefs (sharing the
// factor's indices and landmark mean) and advances the clock, so the next
// iteration needs no separate check.
template <typename TS, bool CHECK>
__global__ __launch_bounds__(RTHREADS) void k_reproj_block(Dev<TS> d, IterOpts o, double huber_k,
                                                           const TS *zref, const uint8_t *mask) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int f0 = d.rblk_start[b], f1 = d.rblk_start[b + 1];
    const ProbParams pp = d.prob[d.rblk_prob[b]];
    const double N = huber_k / pp.sigma;
    if (CHECK && blockIdx.x == 0 && threadIdx.x == 0) d.t_dev[0] = d.t_dev[0] + 1;
    double s_all = 0.0, s_quad = 0.0, s_ref = 0.0;
    int c_valid = 0, c_lin_ref = 0, c_lin = 0, c_inv = 0, c_ref = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool need = false;
    int fq = f0, kq = 0, mq = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int f = f0 + r * RTHREADS + (int)threadIdx.x;
        bool valid = false, lin = false, inv = false, ref = false;
        if (f < f1) {
            // two rounds of loads: first the factor's own words (coalesced),
            // then the gathers they index; the linearisation point and the
            // keyframe mean are fetched only for factors old enough to be
            // checked
            const int k = d.f_kf[f], m = d.f_lm[f];
            const double z0 = d.z[2 * (size_t)f], z1 = d.z[2 * (size_t)f + 1];
            // the mask byte is read from the flags when there is no
            // reference (uniform choice, no branch to wait in)
            const uint32_t want_ref = (zref ? mask : d.flags)[f];
            double zr0 = 0.0, zr1 = 0.0;
            if (zref) {
                zr0 = (double)zref[2 * (size_t)f];
                zr1 = (double)zref[2 * (size_t)f + 1];
            }
            uint8_t fl = 0;
            int cf = 0;
            if (CHECK) {
                fl = d.flags[f];
                cf = d.cnt[f];
            }
            const double *ps = d.kf_pose + 12 * (size_t)k;
            double P[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) P[i] = ps[i];
            const double *bm = d.lm_bel + (size_t)m * LBEL;
            double dm[3], l[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                dm[i] = bm[i];
                l[i] = bm[LANC + i] + dm[i];
            }
            if (CHECK) {
                need = check_due(d, o, f, k, fl, cf, dm);
                fq = f;
                kq = k;
                mq = m;
            }
            double p[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) p[i] = P[3 * i] * l[0] + P[3 * i + 1] * l[1] + P[3 * i + 2] * l[2] + P[9 + i];
            // a point at or behind the depth limit is counted invalid; its
            // projection is formed with a harmless depth and discarded
            inv = !(p[2] > pp.zmin);
            const double pz = inv ? 1.0 : p[2];
            const double h0 = pp.fx * p[0] / pz + pp.cx, h1 = pp.fy * p[1] / pz + pp.cy;
            const double e = hypot(z0 - h0, z1 - h1);
            if (!inv) {
                valid = true;
                s_all += e;
                lin = N > 0.0 && e / pp.sigma > N;
                if (!lin) s_quad += e;
            }
            if (zref) {
                const double er = hypot(zr0 - h0, zr1 - h1);
                if (!inv && want_ref != 0) {
                    s_ref += er;
                    ref = true;
                }
            }
        }
        c_valid += __popcll(__ballot(valid));
        c_lin += __popcll(__ballot(lin));
        c_inv += __popcll(__ballot(inv));
        c_ref += __popcll(__ballot(ref));
        c_lin_ref += __popcll(__ballot(lin && ref));
    }
    if constexpr (CHECK) {
        static_assert(RPL == 1, "the fused check takes one factor per thread");
        queue_due(d, b, fq, kq, mq, need);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s_all += __shfl_xor(s_all, off, 64);
        s_quad += __shfl_xor(s_quad, off, 64);
        s_ref += __shfl_xor(s_ref, off, 64);
    }
    __shared__ double sh[RTHREADS / 64][8];
    if (lane == 0) {
        sh[wave][0] = s_all; sh[wave][1] = s_quad; sh[wave][2] = s_ref; sh[wave][3] = (double)c_valid;
        sh[wave][4] = (double)c_lin_ref; sh[wave][5] = (double)c_lin; sh[wave][6] = (double)c_inv;
        sh[wave][7] = (double)c_ref;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < RTHREADS / 64; ++w) s += sh[w][threadIdx.x];
        d.rblk_part[8 * (size_t)b + threadIdx.x] = s;
    }
}

// one wave per problem (reduce_problem)
__global__ __launch_bounds__(64) void k_reproj_reduce(const double *part, const int *prob_blk, int np,
                                                      double *out, double *log_row, const int *t_dev, int t_off) {
    if ((int)blockIdx.x >= np) return;
    reduce_problem(part, prob_blk, (int)blockIdx.x, out, log_row, t_dev, t_off);
}

__global__ void k_tick(int *t_dev) { t_dev[0] = t_dev[0] + 1; }

// Learned depth: landmark lms[i] moves along the ray from the camera centre
// of its newest observing keyframe (the keyframe of its last factor, factors
// being keyframe-major) to c + exp(mean depth head over its factors) (l - c);
// its prior mean (the anchor) moves with it and its mean offset is cleared.
template <typename TS>
__global__ void k_depth_move(Dev<TS> d, const int *__restrict__ lms, int n, const float *__restrict__ delta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = lms[i];
    const int e0 = d.lm_row[m], e1 = d.lm_row[m + 1];
    if (e1 <= e0) return;
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) acc += (double)delta[d.lm_edge[e]];
    const double scale = exp(acc / (double)(e1 - e0));
    const int k = d.f_kf[d.lm_edge[e1 - 1]];
    const double *ps = d.kf_pose + 12 * (size_t)k;
    double c[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) c[j] = -(ps[j] * ps[9] + ps[3 + j] * ps[10] + ps[6 + j] * ps[11]);
    double *bm = d.lm_bel + (size_t)m * LBEL;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double l = bm[LANC + j] + bm[j];
        bm[LANC + j] = c[j] + scale * (l - c[j]);
        bm[j] = 0.0;
    }
}

// Fallback monitor of the learned damping, one thread per problem: the
// problem switches to the plain constant damping for good once its mean
// reprojection error exceeds (1 + rise) times the best seen so far, or is not
// finite, or a belief failed.
// Fallback monitor of the learned damping (one thread per problem), run at
// every model evaluation on the previous iteration's mean reprojection
// errors: a problem whose judge is plain GBP (judge[p] = j >= 0: problem j
// of the batch runs the same problem with the constant damping) goes back to
// the constant damping for good when its error exceeds (1 + rise) x the
// judge's at the same iteration; without a judge (-1) the reference is the
// best error the problem itself has reached; a judge (-2) always runs the
// constant damping. A non-finite error or a failed belief of the problem
// (its own status word) also switches it.
__global__ void k_monitor(const double *are_out, int np, double rise, double *best, int *fallback,
                          const unsigned *pstatus, const int *judge) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int j = judge[p];
    if (j == -2) { fallback[p] = 1; return; }
    auto mean_err = [&](int q) {
        const double n = are_out[8 * (size_t)q + 3];
        return n > 0.0 ? are_out[8 * (size_t)q] / n : 0.0;
    };
    const double are = mean_err(p);
    const double ref = j >= 0 ? mean_err(j) : best[p];
    if (!isfinite(are) || pstatus[p] != 0u || are > (1.0 + rise) * ref) fallback[p] = 1;
    if (are < best[p]) best[p] = are;
}

// --------------------------------------------------------------------------
// factor-state permutation (incremental growth keeps factors landmark-sorted)
// --------------------------------------------------------------------------

template <typename T, int W>
__global__ __launch_bounds__(256) void k_gather(const T *src, T *dst, const int *perm, int n, T fresh) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    if (j < 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) dst[(size_t)i * W + w] = fresh;
        return;
    }
#pragma unroll
    for (int w = 0; w < W; ++w) dst[(size_t)i * W + w] = src[(size_t)j * W + w];
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

static inline int blocks(long n, int b) { return (int)((n + b - 1) / b); }

template <typename TS>
void launch_linearise(const Dev<TS> &d, int f0, int f1, double huber_k, const int *list, hipStream_t s) {
    if (f1 > f0)
        hipLaunchKernelGGL(k_linearise<TS>, dim3(blocks(f1 - f0, 256)), dim3(256), 0, s, d, f0, f1, huber_k, list);
}

template <typename TS>
void launch_prior_base(const Dev<TS> &d, int k0, int m0, hipStream_t s) {
    if (d.nk > k0) hipLaunchKernelGGL(k_prior_kf<TS>, dim3(blocks((long)(d.nk - k0) * 64, 256)), dim3(256), 0, s, d, k0);
    if (d.nl > m0) hipLaunchKernelGGL(k_prior_lm<TS>, dim3(blocks(d.nl - m0, 256)), dim3(256), 0, s, d, m0);
}

// With events, the keyframe kernel is launched through the HIP runtime's
// extension that records ev0 / ev1 at the kernel's own start and end.
template <typename TS, int MODE>
static void launch_kf(const Dev<TS> &d, const IterOpts &o, int block, int readout, hipStream_t s,
                      hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool solve = true) {
    const dim3 g(d.n_kf_slots);
    auto go = [&](auto kern, int bs) {
        if (ev0)
            hipExtLaunchKernelGGL(kern, g, dim3(bs), 0, s, ev0, ev1, 0, d, o);
        else
            hipLaunchKernelGGL(kern, g, dim3(bs), 0, s, d, o);
    };
    switch (block) {
        case 64: go(k_factor_kf<TS, 64, MODE>, 64); break;
        case 256: go(k_factor_kf<TS, 256, MODE>, 256); break;
        default: go(k_factor_kf<TS, 128, MODE>, 128); break;
    }
    if (solve) hipLaunchKernelGGL(k_kf_solve<TS>, dim3(blocks(d.nk, 64)), dim3(64), 0, s, d, o, readout);
}

template <typename TS>
void launch_check(const Dev<TS> &d, const IterOpts &o, hipStream_t s) {
    if (d.n_rblk > 0)
        hipLaunchKernelGGL(k_check<TS>, dim3(d.n_rblk), dim3(RTHREADS), 0, s, d, o);
    else
        hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, d.t_dev);  // the clock still advances
}

template <typename TS>
void launch_relin(const Dev<TS> &d, const IterOpts &o, hipStream_t s, double *pending_log_row) {
    const int nred = pending_log_row ? d.np : 0;
    const int g = (d.n_rblk + d.relin_group - 1) / d.relin_group + nred;
    if (g > 0) hipLaunchKernelGGL(k_relin<TS>, dim3(g), dim3(RELIN_BS), 0, s, d, o, d.n_rblk, pending_log_row);
    // pairwise factors: they read the previous iteration's beliefs and
    // their own messages only, like the relinearised factors
    const int np = d.n_pair[0] + d.n_pair[1];
    if (np > 0) hipLaunchKernelGGL(k_pairs<TS>, dim3(blocks(np, 128)), dim3(128), 0, s, d, o);
}

template <typename TS>
void launch_queue_every(const Dev<TS> &d, int stride, hipStream_t s) {
    if (d.n_rblk > 0) hipLaunchKernelGGL(k_queue_every<TS>, dim3(d.n_rblk), dim3(RTHREADS), 0, s, d, stride);
}

void launch_relin_total(const int *qcount, int nb, unsigned long long *out, hipStream_t s) {
    hipLaunchKernelGGL(k_relin_total, dim3(1), dim3(256), 0, s, qcount, nb, out);
}

template <typename TS>
void launch_factor_kf(const Dev<TS> &d, const IterOpts &o, int block, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1, bool solve) {
    launch_kf<TS, 0>(d, o, block, 0, s, ev0, ev1, solve);
}

template <typename TS>
void launch_belief_lm(const Dev<TS> &d, const IterOpts &o, int readout, int block, hipStream_t s, bool with_kf) {
    const int nkb = with_kf ? blocks(d.nk, block) : 0;
    const int nlb = d.nl > 0 ? blocks((long)d.nl * d.lm_lanes, block) : 0;
    if (nkb + nlb == 0) return;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(nkb + nlb), dim3(block), 0, s, d, o, readout, nkb); };
    switch (d.lm_lanes) {
        case 2: with_kf ? go(k_belief_lm<TS, 2, true>) : go(k_belief_lm<TS, 2, false>); break;
        case 8: with_kf ? go(k_belief_lm<TS, 8, true>) : go(k_belief_lm<TS, 8, false>); break;
        default: with_kf ? go(k_belief_lm<TS, 4, true>) : go(k_belief_lm<TS, 4, false>); break;
    }
}

template <typename TS>
void launch_belief_kf(const Dev<TS> &d, const IterOpts &o, int readout, int block, hipStream_t s) {
    launch_kf<TS, 1>(d, o, block, readout, s);
}

template <typename TS>
void launch_flag_relin(const Dev<TS> &d, double beta, int *count, hipStream_t s) {
    if (d.nf > 0) hipLaunchKernelGGL(k_flag_relin<TS>, dim3(blocks(d.nf, 256)), dim3(256), 0, s, d, beta, count);
}

template <typename TS>
void launch_reproj(const Dev<TS> &d, const IterOpts &o, double huber_k, const TS *zref, const uint8_t *mask,
                   double *log_row, hipStream_t s) {
    if (d.n_rblk > 0)
        hipLaunchKernelGGL((k_reproj_block<TS, false>), dim3(d.n_rblk), dim3(RTHREADS), 0, s, d, o, huber_k, zref,
                           mask);
    hipLaunchKernelGGL(k_reproj_reduce, dim3(d.np), dim3(64), 0, s, (const double *)d.rblk_part,
                       d.prob_rblk, d.np, d.are_out, log_row, (const int *)d.t_dev, 0);
}

template <typename TS>
void launch_reproj_check(const Dev<TS> &d, const IterOpts &o, double huber_k, const TS *zref,
                         const uint8_t *mask, hipStream_t s) {
    if (d.n_rblk > 0)
        hipLaunchKernelGGL((k_reproj_block<TS, true>), dim3(d.n_rblk), dim3(RTHREADS), 0, s, d, o, huber_k, zref,
                           mask);
    else
        hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, d.t_dev);
}

template <typename TS>
void launch_permute_factors(const Dev<TS> &d, const int *perm, int nf, void *scratch, float *fdamp, float *hist,
                            hipStream_t s) {
    // gather every per-factor array through `perm` (new index -> old index,
    // -1 for a fresh slot) via the scratch buffer, then copy back
    const int b = blocks(nf > 0 ? nf : 1, 256);
    auto run = [&](auto *arr, auto fresh, int w) {
        using T = decltype(fresh);
        T *tmp = (T *)scratch;
        switch (w) {
            case 1: hipLaunchKernelGGL((k_gather<T, 1>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            case 2: hipLaunchKernelGGL((k_gather<T, 2>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            case 4: hipLaunchKernelGGL((k_gather<T, 4>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            case 5: hipLaunchKernelGGL((k_gather<T, 5>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            case 8: hipLaunchKernelGGL((k_gather<T, 8>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            case 12: hipLaunchKernelGGL((k_gather<T, 12>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            case 16: hipLaunchKernelGGL((k_gather<T, 16>), dim3(b), dim3(256), 0, s, (const T *)arr, tmp, perm, nf, fresh); break;
            default: return;
        }
        (void)hipMemcpyAsync(arr, tmp, sizeof(T) * (size_t)w * nf, hipMemcpyDeviceToDevice, s);
    };
    static_assert(KREC == 12 && KMSG == 5 && LREC == 8 && MMSG == 5 && AREC == 2 && DREC == 12,
                  "every record width needs its gather below");
    run(d.krec, TS(0), KREC);
    run(d.kmsg, TS(0), KMSG);
    run(d.lrec, TS(0), LREC);
    run(d.mmsg, TS(0), MMSG);
    run(d.arec, TS(0), AREC);
    run(d.drec, TS(0), DREC);
    run(d.cnt, uint8_t(0), 1);
    run(d.flags, uint8_t(0), 1);
    if (fdamp) run(fdamp, -1.f, 1);  // fresh factors: constant damping until the next evaluation
    static_assert(FHIST == 12, "history rows are gathered with the width-12 gather");
    if (hist) run(hist, 0.f, FHIST);
}

template <typename TS>
void launch_features(const Dev<TS> &d, const IterOpts &o, float *feat, float *hist, double huber_k, hipStream_t s) {
    if (d.nf > 0)
        hipLaunchKernelGGL((k_features<TS, float>), dim3(blocks(d.nf, 256)), dim3(256), 0, s, d, o, feat, hist, huber_k);
}
template <typename TS>
void launch_features_bf16(const Dev<TS> &d, const IterOpts &o, uint16_t *feat, float *hist, double huber_k,
                          hipStream_t s) {
    if (d.nf > 0)
        hipLaunchKernelGGL((k_features<TS, uint16_t>), dim3(blocks(d.nf, 256)), dim3(256), 0, s, d, o, feat, hist,
                           huber_k);
}

template <typename TS>
void launch_export_messages(const Dev<TS> &d, const int *idx, const int *u2i, int n, float *out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_export_messages<TS>, dim3(blocks(n, 256)), dim3(256), 0, s, d, idx, u2i, n, out);
}

template <typename TS>
void launch_depth_move(const Dev<TS> &d, const int *lms, int n, const float *delta, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_depth_move<TS>, dim3(blocks(n, 64)), dim3(64), 0, s, d, lms, n, delta);
}

void launch_monitor(const double *are_out, int np, double rise, double *best, int *fallback, const unsigned *pstatus,
                    const int *judge, hipStream_t s) {
    if (np > 0)
        hipLaunchKernelGGL(k_monitor, dim3(blocks(np, 256)), dim3(256), 0, s, are_out, np, rise, best, fallback,
                           pstatus, judge);
}

void launch_fill_f32(float *p, float v, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_f32, dim3(blocks(n, 256)), dim3(256), 0, s, p, v, n);
}

void launch_gather_rows(const float *src, float *dst, const int *idx, const int *u2i, int nf, int n, int w,
                        hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather_rows, dim3(blocks(n, 256)), dim3(256), 0, s, src, dst, idx, u2i, nf, n, w);
}

void launch_tick(int *t_dev, hipStream_t s) { hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, t_dev); }

#define GBP_INSTANTIATE(TS)                                                                                        \
    template void launch_linearise<TS>(const Dev<TS> &, int, int, double, const int *, hipStream_t);               \
    template void launch_prior_base<TS>(const Dev<TS> &, int, int, hipStream_t);                                   \
    template void launch_check<TS>(const Dev<TS> &, const IterOpts &, hipStream_t);                                \
    template void launch_relin<TS>(const Dev<TS> &, const IterOpts &, hipStream_t, double *);                      \
    template void launch_queue_every<TS>(const Dev<TS> &, int, hipStream_t);                                       \
    template void launch_factor_kf<TS>(const Dev<TS> &, const IterOpts &, int, hipStream_t, hipEvent_t,            \
                                       hipEvent_t, bool);                                                        \
    template void launch_belief_lm<TS>(const Dev<TS> &, const IterOpts &, int, int, hipStream_t, bool);            \
    template void launch_belief_kf<TS>(const Dev<TS> &, const IterOpts &, int, int, hipStream_t);                  \
    template void launch_flag_relin<TS>(const Dev<TS> &, double, int *, hipStream_t);                              \
    template void launch_reproj<TS>(const Dev<TS> &, const IterOpts &, double, const TS *, const uint8_t *,        \
                                    double *, hipStream_t);                                                       \
    template void launch_reproj_check<TS>(const Dev<TS> &, const IterOpts &, double, const TS *,                   \
                                          const uint8_t *, hipStream_t);                                          \
    template void launch_permute_factors<TS>(const Dev<TS> &, const int *, int, void *, float *, float *,         \
                                             hipStream_t);              \
    template void launch_depth_move<TS>(const Dev<TS> &, const int *, int, const float *, hipStream_t);            \
    template void launch_features<TS>(const Dev<TS> &, const IterOpts &, float *, float *, double, hipStream_t);  \
    template void launch_features_bf16<TS>(const Dev<TS> &, const IterOpts &, uint16_t *, float *, double,        \
                                           hipStream_t);                                                          \
    template void launch_export_messages<TS>(const Dev<TS> &, const int *, const int *, int, float *, hipStream_t);

GBP_INSTANTIATE(float)
GBP_INSTANTIATE(double)

}  // namespace gbp
