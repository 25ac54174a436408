// Internal declarations shared by the kernel and runtime translation units
// of the GBP library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbp {

constexpr int KREC = 12;  // keyframe-side Jacobian record per factor (see layout below)
constexpr int KMSG = 5;   // message to the keyframe (dense, rewritten every iteration)
constexpr int LREC = 8;   // landmark-side Jacobian record per factor
constexpr int MMSG = 5;   // message to the landmark (dense, rewritten every iteration)
constexpr int AREC = 2;   // factor-private record read by the message update
constexpr int DREC = 12;  // factor's linearisation point (check, features)
constexpr int KBEL = 32;  // doubles per keyframe belief: dmu 6, cov 21 (packed), pad
constexpr int LBEL = 16;  // doubles per landmark belief: dmu 3, cov 6 (packed), anchor 3, pad to 128 B
constexpr int LANC = 9;   // offset of the landmark's anchor (prior mean) in its belief record
constexpr int MAX_ANNEAL = 64;
constexpr int RTHREADS = 256;          // threads of a residual-phase block
constexpr int RPL = 1;                 // factors per lane in the residual phase (more: slower, latency-bound)
constexpr int RBLK = RTHREADS * RPL;   // factors per residual-phase block
constexpr int LM_LANES = 4;  // default lanes per landmark in the landmark belief kernel
constexpr int NFEAT = 16;   // learned-model features per factor
constexpr int FHIST = 12;   // floats of per-factor feature history
constexpr int MSG_W = 16;   // floats per exported factor-message row
// pairwise difference factors: D = 6 (keyframes) or 3 (landmarks); per pair
// the messages to a and to b, each eta (D) then Lambda (packed, D(D+1)/2)
constexpr int pair_msg_doubles(int D) { return 2 * (D + D * (D + 1) / 2); }
constexpr int KBI = 32;     // doubles of keyframe belief information: Lambda packed (21), eta (6), pad
constexpr int LBI = 12;     // doubles of landmark belief information: Lambda packed (6), eta (3), pad

// keyframe-side record (TS = float | double), one per factor:
//   [0..5]  d h / d omega (2x3, row-major)
//   [6]     fx / pz   [7] fy / pz   [8] -fx px / pz^2   [9] -fy py / pz^2
//           (d h / d t = [[6], 0, [8]; 0, [7], [9]])
//   [10]    s = w / sigma^2   [11] the factor's landmark index (its bit pattern
//           in FP32 state, its value in FP64 state; fixed for the factor's
//           lifetime, so the keyframe kernel needs no separate index stream)
// message to the keyframe (its own dense array, so that the rewrite every
// iteration covers whole cache lines):
//   [0..2] S (a, b, c) = [[a b][b c]]   [3..4] g (anchor-relative information
//          vector in the factor's 2-D measurement space)
// landmark-side record: [0..5] J_m (2x3), [6..7] J_m anchor_m (read by the
// message update with the Jacobian; the landmark belief kernel reads the
// Jacobian only); message to the landmark (dense array): [0..2] S, [3..4] g
// factor-private record:
//   [0..1]  rho = z - h(x0) + J_k (x0_k - anchor_k) + J_m (x0_m - anchor_m),
//           the linearised residual at the anchors: the message update needs
//           the residual and the linearisation point only in this sum
// (J_k anchor_k is formed where it is needed, from the keyframe's anchor,
// which a keyframe-kernel workgroup holds in scalar registers)
// linearisation-point record: [0..5] x0_k - anchor_k, [6..8] x0_m - anchor_m, pad

struct ProbParams {
    double fx, fy, cx, cy, sigma, inv_s2, zmin, pad;
};

// Device view of one problem set (a single problem or a batch).
// one workgroup of the keyframe kernel: its keyframe (-1: none), the
// keyframe's factor range and its problem, read in one load
struct alignas(16) KfSlot {
    int k, e0, e1, prob;
};

// one queued relinearisation: the factor and its two variables (so that the
// relinearising kernel gathers the beliefs in the same round of loads as the
// factor's records)
struct alignas(16) RelinEntry {
    int f, k, m, pad;
};

template <typename TS>
struct Dev {
    int nk, nl, nf, np;
    // variables
    const double *kf_anchor;              // absolute initial estimate (prior mean)
    // landmark anchors live in the landmarks' belief records (LANC), so that
    // a gather of a landmark's mean and anchor touches one 128-B line; they
    // are moved only by the learned depth
    double *kf_pbase, *lm_pbase;          // automatic prior information (diag)
    const double *kf_pinfo;               // anchor prior information (0: automatic)
    const int *kf_t0, *lm_t0;             // iteration at which the variable was born
    const int *kf_prob, *lm_prob;
    double *kf_bel, *lm_bel;              // beliefs (KBEL / LBEL doubles)
    double *kf_info, *lm_info;            // full information for read-out
    // graph
    const int *f_kf, *f_lm;
    const int *kf_row;                    // factors of keyframe k: [kf_row[k], kf_row[k+1])
    const KfSlot *kf_slot;                // work of each keyframe-kernel workgroup
    int n_kf_slots;                       // workgroups of the keyframe kernel
    int lm_lanes;                         // lanes per landmark in the landmark belief kernel (2, 4, 8)
    int relin_group;                      // relinearisation queue segments per workgroup (1..16)
    const int *lm_row, *lm_edge;          // factors of each landmark (CSR, increasing)
    const int *f_row_prob;                // first factor of each problem (np + 1)
    // factor state
    const double *z;
    TS *krec, *kmsg, *lrec, *mmsg, *arec, *drec;
    uint8_t *cnt, *flags;
    float *fdamp;                         // per-factor damping (learned model) or null
    const int *fallback;                  // per problem: 1 = learned damping switched off
    // parameters
    const ProbParams *prob;
    int *t_dev;                           // iteration clock
    unsigned *status;                     // bit 0: non-PD belief, bit 1: non-finite
    unsigned *pstatus;                    // the same bits per problem (np)
    double *pending_k;                    // Huber threshold for requested relinearisations
    RelinEntry *relin_queue;              // factors due for relinearisation, RBLK per residual block
    int *relin_qcount;                    // queue entries of each residual block
    double *kf_sums;                      // per keyframe: 21 information + 6 vector sums (32)
    double *kf_pose;                      // absolute R (9) and t (3) of each keyframe mean
    // residual phase: blocks of at most RBLK factors inside one problem
    int n_rblk;
    const int *rblk_start;                // first factor of each block (n_rblk + 1)
    const int *rblk_prob;                 // problem of each block
    const int *prob_rblk;                 // first block of each problem (np + 1)
    double *rblk_part;                    // per-block partial statistics (8 doubles)
    double *are_out;                      // per-problem statistics (8 doubles)
    // pairwise difference factors (kind 0: keyframes, kind 1: landmarks),
    // FP64, messages relative to the variables' anchors
    int n_pair[2];
    const int *pair_ab[2];                // ends a, b of each pair
    const int *pair_type0;                // keyframe pairs: 0 difference, 1 odometry (camera centres)
    const double *pair_zp[2];             // measured x_b - x_a (D) and diagonal precision (D)
    int *pair_cnt[2];                     // updates since the pair was added
    double *pair_msg[2];                  // pair_msg_doubles(D) per pair
    const int *kp_row, *kp_ent;           // pair ends of each keyframe (CSR; entry 2 pair + side)
    const int *lp_row, *lp_ent;           // pair ends of each landmark
    double *kf_binfo, *lm_binfo;          // belief information (KBI / LBI) while pairs of that kind exist
};

struct IterOpts {
    double beta2;
    int interval, undamped, damp_mode, anneal_iters;
    double damping, huber_k;
    double scale[MAX_ANNEAL + 1];  // prior scale by age 0..anneal_iters (last = steady)
};

enum : uint8_t { FLAG_PENDING = 1, FLAG_INVALID = 2, FLAG_DONE = 4 };

// launchers (gbp_kernels.hip); all asynchronous on `s`
template <typename TS> void launch_linearise(const Dev<TS> &d, int f0, int f1, double huber_k, const int *list,
                                             hipStream_t s);
template <typename TS> void launch_prior_base(const Dev<TS> &d, int k0, int m0, hipStream_t s);
template <typename TS> void launch_check(const Dev<TS> &d, const IterOpts &o, hipStream_t s);
// pending_log_row: also reduce the statistics of a preceding launch_reproj_check
template <typename TS> void launch_relin(const Dev<TS> &d, const IterOpts &o, hipStream_t s,
                                         double *pending_log_row = nullptr);
void launch_relin_total(const int *qcount, int nb, unsigned long long *out, hipStream_t s);
// tuning: queue every stride-th factor of each residual block for relinearisation
template <typename TS> void launch_queue_every(const Dev<TS> &d, int stride, hipStream_t s);
// solve = false leaves the keyframe solve to launch_belief_lm(..., with_kf = true)
template <typename TS> void launch_factor_kf(const Dev<TS> &d, const IterOpts &o, int block, hipStream_t s,
                                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool solve = true);
template <typename TS> void launch_belief_lm(const Dev<TS> &d, const IterOpts &o, int readout, int block, hipStream_t s,
                                             bool with_kf = false);
template <typename TS> void launch_belief_kf(const Dev<TS> &d, const IterOpts &o, int readout, int block, hipStream_t s);
template <typename TS> void launch_flag_relin(const Dev<TS> &d, double beta, int *count, hipStream_t s);
template <typename TS> void launch_reproj(const Dev<TS> &d, const IterOpts &o, double huber_k, const TS *zref,
                                          const uint8_t *mask, double *log_row, hipStream_t s);
// residual partials of every block plus the next iteration's check (the
// statistics are reduced by the next launch_relin)
template <typename TS> void launch_reproj_check(const Dev<TS> &d, const IterOpts &o, double huber_k,
                                                const TS *zref, const uint8_t *mask, hipStream_t s);
template <typename TS> void launch_permute_factors(const Dev<TS> &d, const int *perm, int nf,
                                                   void *scratch, float *fdamp, float *hist, hipStream_t s);
template <typename TS> void launch_features(const Dev<TS> &d, const IterOpts &o, float *feat, float *hist,
                                            double huber_k, hipStream_t s);
// the same features as BF16 bits, for the network inside the iteration
template <typename TS> void launch_features_bf16(const Dev<TS> &d, const IterOpts &o, uint16_t *feat, float *hist,
                                                 double huber_k, hipStream_t s);
template <typename TS> void launch_export_messages(const Dev<TS> &d, const int *idx, const int *u2i, int n, float *out,
                                                   hipStream_t s);
void launch_fill_f32(float *p, float v, int n, hipStream_t s);
void launch_gather_rows(const float *src, float *dst, const int *idx, const int *u2i, int nf, int n, int w,
                        hipStream_t s);
void launch_monitor(const double *are_out, int np, double rise, double *best, int *fallback, const unsigned *pstatus,
                    const int *judge, hipStream_t s);
template <typename TS> void launch_depth_move(const Dev<TS> &d, const int *lms, int n, const float *delta,
                                              hipStream_t s);
void launch_tick(int *t_dev, hipStream_t s);

}  // namespace gbp
