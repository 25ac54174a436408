// Host runtime and C ABI of the GBP bundle-adjustment library.
//
// Graph build (the paper's "predetermined" exchange schedule, Section 7,
// becomes a fixed memory layout): within each problem, landmarks are ordered
// by their first observing keyframe, factors by keyframe and then landmark
// (so a keyframe's factors are contiguous and one workgroup owns them), and
// each landmark gets a CSR list of its factors in increasing factor order. A batch is the block-diagonal
// concatenation of its problems. Every buffer is carved from one device
// workspace (caller-provided, e.g. a torch allocation, or allocated here).
// Iterations are recorded once per (n, damping, Huber threshold) into a HIP
// graph and replayed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/gbp.h"
#include "gbp_internal.h"
#include "gbp_mlp.h"

using namespace gbp;

namespace {

struct GraphEntry {
    int n;
    double damping, huber;
    int log_every;
    int phase;  // clock modulo the model period (learned damping), else -1
    hipGraphExec_t exec;
};

// error text of calls that have no problem handle (the MLP entry points)
thread_local std::string g_err;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct gbp_problem {
    int precision = GBP_FP32;
    gbp_options opt{};
    int np = 0, nk = 0, nl = 0, nf = 0;
    int cap_k = 0, cap_l = 0, cap_f = 0;
    // internal <-> caller ordering
    std::vector<int> lm_int2user, f_int2user;
    std::vector<int> kf_off, lm_off, f_off;  // internal offsets per problem
    // host mirrors needed to rebuild the layout on growth
    std::vector<int> h_fkf, h_flm, h_kf_row, h_lm_row, h_lm_edge;
    std::vector<double> h_z, h_kf_anchor, h_lm_anchor;
    std::vector<double> h_lm_anchor0;  // landmark anchors at creation (the learned depth moves anchors)
    std::vector<int> h_first_obs;  // first observing keyframe of each internal landmark
    // device
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Dev<float> df{};
    Dev<double> dd{};
    int *d_count = nullptr;
    unsigned long long *d_total = nullptr;
    void *d_zref = nullptr;   // reference pixels in the factor-state precision
    uint8_t *d_mask = nullptr;
    bool has_ref = false;
    int *d_perm = nullptr;
    void *d_scratch = nullptr;
    double *d_log = nullptr;
    size_t log_cap = 0;
    IterOpts iopt{};
    double huber_k = 2.0;
    int t = 0;
    std::vector<GraphEntry> graphs;
    bool use_graph = true;
    int blk_lm = 256, blk_kf = 128;
    // keyframe solves in the first workgroups of the landmark-belief launch
    // (1) or in a launch of their own after the keyframe kernel (0): tuned
    int kf_fused = 1;
    // learned damping (one allocation, made on first use)
    float *fdamp_buf = nullptr;    // per-factor damping, in the workspace
    void *learn_mem = nullptr;
    float *d_feat = nullptr;       // [cap_f][16] features
    float *d_hist = nullptr;       // [cap_f][12] feature history
    float *d_delta = nullptr;      // [cap_f] log-depth head
    uint16_t *d_w = nullptr;       // network weights (BF16 bits)
    int *d_u2i = nullptr;          // caller factor index -> internal slot
    int *d_lms = nullptr;          // [cap_l] landmark list (learned depth)
    int *d_fallback = nullptr;     // [np]
    int *d_judge = nullptr;        // [np] judge of each problem (monitor), -1 none, -2 is a judge
    std::vector<int> h_judge;      // host copy (empty: no judges)
    double *d_best = nullptr;      // [np] best mean reprojection error seen
    bool learned = false;
    bool grown = false;            // gbp_add_keyframe was called
    // pairwise difference factors (kind 0 keyframes, 1 landmarks): host
    // mirrors in internal indices, and one device allocation for their
    // state, their variables' pair lists and the belief information
    std::vector<int> h_pair_ab[2];
    std::vector<double> h_pair_zp[2];
    std::vector<int> h_pair_type0;  // keyframe pairs: 0 difference, 1 odometry
    void *pair_mem = nullptr;
    size_t pair_state_bytes = 0;   // leading bytes that hold messages and counts
    int every_k = 5;
    double fb_rise = 0.1;
    std::string err;
    bool broken = false;
};

namespace {

gbp_status fail(gbp_problem *p, gbp_status st, const std::string &msg) {
    if (p) p->err = msg;
    return st;
}

#define HIP_TRY(p, call)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((p), GBP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Workspace layout: one entry per device array.
struct Layout {
    size_t total = 0;
    std::vector<std::pair<void **, size_t>> items;
    void add(void **ptr, size_t bytes) {
        items.push_back({ptr, total});
        total += align_up(bytes ? bytes : 1);
    }
};

// Landmark anchors live in the landmark belief records (offset LANC, stride
// LBEL doubles). A strided copy of 24-byte rows from pageable host memory
// goes row by row (about 2.3 s for 269,085 landmarks), so whole records move
// in one contiguous copy instead. put: records m0 .. m0 + n - 1 become zero
// with the anchor in place (every caller writes them when they are new or
// just cleared); get: the records come back whole and the anchors are taken
// out on the host. Both synchronise the stream (their host staging is local).
gbp_status put_lm_anchors(gbp_problem *p, double *lm_bel, int m0, int n, const double *src, hipStream_t s) {
    if (n <= 0) return GBP_OK;
    std::vector<double> rec((size_t)n * LBEL, 0.0);
    for (size_t m = 0; m < (size_t)n; ++m)
        for (int c = 0; c < 3; ++c) rec[m * LBEL + LANC + c] = src[3 * m + c];
    HIP_TRY(p, hipMemcpyAsync(lm_bel + (size_t)m0 * LBEL, rec.data(), rec.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    return GBP_OK;
}

gbp_status get_lm_anchors(gbp_problem *p, const double *lm_bel, int n, double *dst, hipStream_t s) {
    if (n <= 0) return GBP_OK;
    std::vector<double> rec((size_t)n * LBEL);
    HIP_TRY(p, hipMemcpyAsync(rec.data(), lm_bel, rec.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    for (size_t m = 0; m < (size_t)n; ++m)
        for (int c = 0; c < 3; ++c) dst[3 * m + c] = rec[m * LBEL + LANC + c];
    return GBP_OK;
}

template <typename TS>
void plan(gbp_problem *p, Dev<TS> &d, Layout &L) {
    const size_t K = p->cap_k, M = p->cap_l, F = p->cap_f, P = p->np;
    L.add((void **)&d.kf_anchor, K * 6 * 8);
    L.add((void **)&d.kf_pbase, K * 6 * 8);
    L.add((void **)&d.lm_pbase, M * 3 * 8);
    L.add((void **)&d.kf_pinfo, K * 8);
    L.add((void **)&d.kf_t0, K * 4);
    L.add((void **)&d.lm_t0, M * 4);
    L.add((void **)&d.kf_prob, K * 4);
    L.add((void **)&d.lm_prob, M * 4);
    L.add((void **)&d.kf_bel, K * KBEL * 8);
    L.add((void **)&d.lm_bel, M * LBEL * 8);
    L.add((void **)&d.kf_info, K * 36 * 8);
    L.add((void **)&d.lm_info, M * 9 * 8);
    L.add((void **)&d.f_kf, F * 4);
    L.add((void **)&d.f_lm, F * 4);
    L.add((void **)&d.kf_row, (K + 1) * 4);
    L.add((void **)&d.kf_slot, (8 * K + 1) * sizeof(KfSlot));  // at most 8 slots per keyframe (runs of unequal length)
    L.add((void **)&d.lm_edge, F * 4);
    L.add((void **)&d.lm_row, (M + 1) * 4);
    L.add((void **)&d.f_row_prob, (P + 1) * 4);
    L.add((void **)&d.z, F * 2 * 8);
    L.add((void **)&d.krec, F * KREC * sizeof(TS));
    L.add((void **)&d.kmsg, F * KMSG * sizeof(TS));
    L.add((void **)&d.lrec, F * LREC * sizeof(TS));
    L.add((void **)&d.mmsg, F * MMSG * sizeof(TS));
    L.add((void **)&d.arec, F * AREC * sizeof(TS));
    L.add((void **)&d.drec, F * DREC * sizeof(TS));
    L.add((void **)&d.cnt, F);
    L.add((void **)&d.flags, F);
    L.add((void **)&d.fdamp, F * 4);
    L.add((void **)&d.prob, P * sizeof(ProbParams));
    L.add((void **)&d.t_dev, 4);
    L.add((void **)&d.status, 4);
    L.add((void **)&d.pstatus, P * 4);
    L.add((void **)&d.pending_k, 8);
    // relinearisation queue: one segment per residual block (F / RBLK + P + 1)
    L.add((void **)&d.relin_queue, (F / RBLK + P + 1) * RBLK * sizeof(RelinEntry));
    L.add((void **)&d.relin_qcount, (F / RBLK + P + 1) * 4);
    L.add((void **)&d.kf_sums, K * 32 * 8);
    L.add((void **)&p->d_total, 8);
    L.add((void **)&d.kf_pose, K * 12 * 8);
    const size_t RB = F / RBLK + P + 1;
    L.add((void **)&d.rblk_start, (RB + 1) * 4);
    L.add((void **)&d.rblk_prob, RB * 4);
    L.add((void **)&d.prob_rblk, (P + 1) * 4);
    L.add((void **)&d.rblk_part, RB * 8 * 8);
    L.add((void **)&d.are_out, P * 8 * 8);
    L.add((void **)&p->d_count, 4);
    L.add((void **)&p->d_zref, F * 2 * 8);
    L.add((void **)&p->d_mask, F);
    L.add((void **)&p->d_perm, F * 4);
    L.add((void **)&p->d_scratch, F * 16 * 8);
}

void default_opts(gbp_options *o) {
    std::memset(o, 0, sizeof(*o));
    o->precision = GBP_FP32;
    o->damp_mode = GBP_DAMP_ETA;
    o->beta = 0.01;
    o->relin_min_interval = 10;
    o->undamped_after_relin = 8;
    o->anneal = 1;
    o->prior_anneal_iters = 10;
    o->prior_weaken = 0.01;
    o->huber_k = 2.0;
    o->zmin = 1e-3;
}

gbp_status check_opts(const gbp_options *o, std::string &msg) {
    if (o->precision != GBP_FP32 && o->precision != GBP_FP64) { msg = "precision must be GBP_FP32 or GBP_FP64"; return GBP_EINVAL; }
    if (o->damp_mode != GBP_DAMP_ETA && o->damp_mode != GBP_DAMP_ETA_LAMBDA) { msg = "bad damp_mode"; return GBP_EINVAL; }
    if (o->undamped_after_relin < 1) { msg = "undamped_after_relin must be >= 1"; return GBP_EINVAL; }
    if (o->relin_min_interval < 0 || o->relin_min_interval > 250) { msg = "relin_min_interval must be in [0, 250]"; return GBP_EINVAL; }
    if (o->prior_anneal_iters < 0 || o->prior_anneal_iters > MAX_ANNEAL) { msg = "prior_anneal_iters must be in [0, 64]"; return GBP_EINVAL; }
    if (!(o->prior_weaken > 0.0) || !(o->beta >= 0.0)) { msg = "prior_weaken must be > 0 and beta >= 0"; return GBP_EINVAL; }
    return GBP_OK;
}

// Sizes of a batch before any of its arrays is read: each graph's sizes,
// then the totals (capacities included) against GBP_MAX_BATCH_ITEMS, so
// that every index and every 2 x index fits 32 bits.
gbp_status check_totals(int n, const gbp_graph *gs, const gbp_options &o, std::string &msg) {
    long long nk = 0, nl = 0, nf = 0;
    for (int i = 0; i < n; ++i) {
        if (gs[i].n_keyframes < 1 || gs[i].n_landmarks < 0 || gs[i].n_factors < 0) {
            msg = "problem " + std::to_string(i) + ": bad sizes";
            return GBP_EINVAL;
        }
        nk += gs[i].n_keyframes;
        nl += gs[i].n_landmarks;
        nf += gs[i].n_factors;
    }
    nk = std::max(nk, (long long)o.max_keyframes);
    nl = std::max(nl, (long long)o.max_landmarks);
    nf = std::max(nf, (long long)o.max_factors);
    if (nk > GBP_MAX_BATCH_ITEMS || nl > GBP_MAX_BATCH_ITEMS || nf > GBP_MAX_BATCH_ITEMS) {
        msg = "batch too large: " + std::to_string(nk) + " keyframes, " + std::to_string(nl) + " landmarks, " +
              std::to_string(nf) + " factors (at most " + std::to_string(GBP_MAX_BATCH_ITEMS) + " each)";
        return GBP_EINVAL;
    }
    return GBP_OK;
}

gbp_status check_graph(const gbp_graph *g, const gbp_measurements *m, const gbp_camera *c, std::string &msg) {
    if (!g || !m || !c) { msg = "null argument"; return GBP_EINVAL; }
    if (g->n_keyframes < 1 || g->n_landmarks < 0 || g->n_factors < 0) { msg = "bad sizes"; return GBP_EINVAL; }
    if (g->n_factors > 0 && (!g->factor_kf || !g->factor_lm || !m->z)) { msg = "null factor arrays"; return GBP_EINVAL; }
    if (!g->kf_init || (g->n_landmarks > 0 && !g->lm_init)) { msg = "null initial estimate"; return GBP_EINVAL; }
    if (!(c->sigma_px > 0.0) || !(c->fx > 0.0) || !(c->fy > 0.0)) { msg = "bad camera"; return GBP_EINVAL; }
    for (int f = 0; f < g->n_factors; ++f) {
        if (g->factor_kf[f] < 0 || g->factor_kf[f] >= g->n_keyframes || g->factor_lm[f] < 0 ||
            g->factor_lm[f] >= g->n_landmarks) {
            msg = "factor " + std::to_string(f) + " has an out-of-range variable index";
            return GBP_EINVAL;
        }
        if (!std::isfinite(m->z[2 * f]) || !std::isfinite(m->z[2 * f + 1])) {
            msg = "factor " + std::to_string(f) + " has a non-finite measurement";
            return GBP_EINVAL;
        }
    }
    for (long i = 0; i < 6L * g->n_keyframes; ++i)
        if (!std::isfinite(g->kf_init[i])) { msg = "non-finite keyframe initial estimate"; return GBP_EINVAL; }
    for (long i = 0; i < 3L * g->n_landmarks; ++i)
        if (!std::isfinite(g->lm_init[i])) { msg = "non-finite landmark initial estimate"; return GBP_EINVAL; }
    return GBP_OK;
}

void fill_iopt(gbp_problem *p) {
    IterOpts &o = p->iopt;
    o.beta2 = p->opt.beta * p->opt.beta;
    o.interval = p->opt.relin_min_interval;
    o.undamped = p->opt.undamped_after_relin;
    o.damp_mode = p->opt.damp_mode;
    const int T = p->opt.anneal ? p->opt.prior_anneal_iters : 0;
    o.anneal_iters = T;
    for (int a = 0; a <= MAX_ANNEAL; ++a) o.scale[a] = p->opt.prior_weaken;
    if (T > 0)
        for (int a = 0; a <= T; ++a) o.scale[a] = std::pow(p->opt.prior_weaken, (double)a / (double)T);
}

template <typename TS>
Dev<TS> &dev(gbp_problem *p);
template <>
Dev<float> &dev<float>(gbp_problem *p) { return p->df; }
template <>
Dev<double> &dev<double>(gbp_problem *p) { return p->dd; }

// landmark anchors live in the landmark belief records (offset LANC,
// stride LBEL): strided copies to and from a packed [n][3] host array
gbp_status put_lm_anchors(gbp_problem *p, double *lm_bel, int m0, int n, const double *src, hipStream_t s);
gbp_status get_lm_anchors(gbp_problem *p, const double *lm_bel, int n, double *dst, hipStream_t s);

// Build the internal ordering of the whole (possibly batched) graph.
void build_order(gbp_problem *p, int n, const gbp_graph *gs, const gbp_measurements *ms,
                 std::vector<int> &fkf, std::vector<int> &flm, std::vector<double> &z) {
    p->kf_off.assign(n + 1, 0);
    p->lm_off.assign(n + 1, 0);
    p->f_off.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        p->kf_off[i + 1] = p->kf_off[i] + gs[i].n_keyframes;
        p->lm_off[i + 1] = p->lm_off[i] + gs[i].n_landmarks;
        p->f_off[i + 1] = p->f_off[i] + gs[i].n_factors;
    }
    p->nk = p->kf_off[n];
    p->nl = p->lm_off[n];
    p->nf = p->f_off[n];
    p->lm_int2user.resize(p->nl);
    p->f_int2user.resize(p->nf);
    p->h_first_obs.assign(p->nl, 0);
    fkf.resize(p->nf);
    flm.resize(p->nf);
    z.resize(2 * (size_t)p->nf);
    for (int i = 0; i < n; ++i) {
        const gbp_graph &g = gs[i];
        const int K0 = p->kf_off[i], M0 = p->lm_off[i], F0 = p->f_off[i];
        // landmarks ordered by first observing keyframe (locality of the
        // keyframe-side gathers), ties by caller index
        std::vector<int> first(g.n_landmarks, g.n_keyframes);
        for (int f = 0; f < g.n_factors; ++f) first[g.factor_lm[f]] = std::min(first[g.factor_lm[f]], g.factor_kf[f]);
        std::vector<int> lorder(g.n_landmarks);
        std::iota(lorder.begin(), lorder.end(), 0);
        std::stable_sort(lorder.begin(), lorder.end(), [&](int a, int b) { return first[a] < first[b]; });
        std::vector<int> lrank(g.n_landmarks);
        for (int r = 0; r < g.n_landmarks; ++r) {
            lrank[lorder[r]] = r;
            p->lm_int2user[M0 + r] = M0 + lorder[r];
            p->h_first_obs[M0 + r] = first[lorder[r]];
        }
        std::vector<int> forder(g.n_factors);
        std::iota(forder.begin(), forder.end(), 0);
        std::stable_sort(forder.begin(), forder.end(), [&](int a, int b) {
            if (g.factor_kf[a] != g.factor_kf[b]) return g.factor_kf[a] < g.factor_kf[b];
            return lrank[g.factor_lm[a]] < lrank[g.factor_lm[b]];
        });
        for (int r = 0; r < g.n_factors; ++r) {
            int f = forder[r];
            p->f_int2user[F0 + r] = F0 + f;
            fkf[F0 + r] = K0 + g.factor_kf[f];
            flm[F0 + r] = M0 + lrank[g.factor_lm[f]];
            z[2 * (size_t)(F0 + r)] = ms[i].z[2 * f];
            z[2 * (size_t)(F0 + r) + 1] = ms[i].z[2 * f + 1];
        }
    }
}

void build_csr(gbp_problem *p) {
    const int nk = p->nk, nl = p->nl, nf = p->nf;
    p->h_kf_row.assign(nk + 1, 0);
    p->h_lm_row.assign(nl + 1, 0);
    for (int f = 0; f < nf; ++f) {
        p->h_kf_row[p->h_fkf[f] + 1]++;
        p->h_lm_row[p->h_flm[f] + 1]++;
    }
    for (int k = 0; k < nk; ++k) p->h_kf_row[k + 1] += p->h_kf_row[k];
    for (int m = 0; m < nl; ++m) p->h_lm_row[m + 1] += p->h_lm_row[m];
    p->h_lm_edge.assign(nf, 0);
    std::vector<int> fill(nl, 0);
    for (int f = 0; f < nf; ++f) {
        int m = p->h_flm[f];
        p->h_lm_edge[p->h_lm_row[m] + fill[m]++] = f;
    }
}

// Workgroup order of the keyframe kernel. Workgroups are dispatched
// round-robin over the eight XCDs, so slot b runs on XCD b % 8. The
// keyframes, in index order (problems concatenated), are cut into eight
// contiguous runs of about equal work (factor chunks of the workgroup size),
// one per XCD, which keeps keyframes that share landmarks in one L2. Within
// a run the problems with the largest keyframes go first, so the long
// workgroups start early, and each problem's keyframes stay together
// (largest first), so the landmarks they share are fetched while still in
// L2. Slots past the end of a shorter run hold -1 (the workgroup exits).
std::vector<int> kf_order(const gbp_problem *p) {
    constexpr int NX = 8;
    const int nk = p->nk;
    std::vector<double> w(nk);
    double total = 0.0;
    for (int k = 0; k < nk; ++k) {
        const int n = p->h_kf_row[k + 1] - p->h_kf_row[k];
        w[k] = (double)((n + 63) / 64) + 0.25;  // chunks plus a per-workgroup cost
        total += w[k];
    }
    std::vector<std::vector<int>> run(NX);
    double acc = 0.0;
    for (int k = 0; k < nk; ++k) {
        int x = (int)(acc * NX / (total > 0.0 ? total : 1.0));
        if (x >= NX) x = NX - 1;
        run[x].push_back(k);
        acc += w[k];
    }
    // each keyframe's problem and each problem's largest keyframe
    std::vector<int> kp(nk, 0);
    for (int i = 0; i + 1 < (int)p->kf_off.size(); ++i)
        for (int k = p->kf_off[i]; k < p->kf_off[i + 1]; ++k) kp[k] = i;
    std::vector<double> pw(p->kf_off.size(), 0.0);
    for (int k = 0; k < nk; ++k) pw[kp[k]] = std::max(pw[kp[k]], w[k]);
    size_t len = 0;
    for (auto &r : run) {
        std::stable_sort(r.begin(), r.end(), [&](int a, int b) {
            if (pw[kp[a]] != pw[kp[b]]) return pw[kp[a]] > pw[kp[b]];
            if (kp[a] != kp[b]) return kp[a] < kp[b];
            return w[a] > w[b];
        });
        len = std::max(len, r.size());
    }
    std::vector<int> order(len * NX, -1);
    for (int x = 0; x < NX; ++x)
        for (size_t i = 0; i < run[x].size(); ++i) order[i * NX + x] = run[x][i];
    return order;
}

// the keyframe kernel's slots: keyframe, factor range and problem per
// workgroup, in the order above
std::vector<KfSlot> kf_slots(const gbp_problem *p) {
    const std::vector<int> order = kf_order(p);
    std::vector<int> kp(p->nk, 0);
    for (int i = 0; i + 1 < (int)p->kf_off.size(); ++i)
        for (int k = p->kf_off[i]; k < p->kf_off[i + 1]; ++k) kp[k] = i;
    std::vector<KfSlot> slots(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
        const int k = order[i];
        slots[i] = k < 0 ? KfSlot{-1, 0, 0, 0} : KfSlot{k, p->h_kf_row[k], p->h_kf_row[k + 1], kp[k]};
    }
    return slots;
}

void destroy_graphs(gbp_problem *p) {
    for (auto &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    p->graphs.clear();
}

// residual-phase blocks: chunks of RBLK factors that stay inside a problem
template <typename TS>
gbp_status upload_rblk(gbp_problem *p) {
    Dev<TS> &d = dev<TS>(p);
    const int n = p->np;
    std::vector<int> bstart, bprob, pblk(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        pblk[i] = (int)bprob.size();
        for (int f = p->f_off[i]; f < p->f_off[i + 1]; f += RBLK) {
            bstart.push_back(f);
            bprob.push_back(i);
        }
    }
    pblk[n] = (int)bprob.size();
    bstart.push_back(p->nf);
    d.n_rblk = (int)bprob.size();
    HIP_TRY(p, hipMemcpyAsync((void *)d.rblk_start, bstart.data(), bstart.size() * 4, hipMemcpyHostToDevice, p->stream));
    if (!bprob.empty())
        HIP_TRY(p, hipMemcpyAsync((void *)d.rblk_prob, bprob.data(), bprob.size() * 4, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipMemcpyAsync((void *)d.prob_rblk, pblk.data(), pblk.size() * 4, hipMemcpyHostToDevice, p->stream));
    // rblk arrays are sized for the capacity: F / RBLK + P + 1 blocks
    return GBP_OK;
}

template <typename TS>
gbp_status upload_and_init(gbp_problem *p, const gbp_graph *gs, const gbp_camera *cams, int n) {
    gbp_status st_rb;
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    const int nk = p->nk, nl = p->nl, nf = p->nf;
    d.nk = nk; d.nl = nl; d.nf = nf; d.np = n;
    // per-variable host arrays
    std::vector<double> kf_anchor(6 * (size_t)nk), lm_anchor(3 * (size_t)nl), kf_pinfo(nk, 0.0);
    std::vector<int> kf_prob(nk), lm_prob(nl), zero_k(nk, 0), zero_l(nl, 0);
    std::vector<ProbParams> pp(n);
    for (int i = 0; i < n; ++i) {
        const gbp_graph &g = gs[i];
        for (int k = 0; k < g.n_keyframes; ++k) {
            int K = p->kf_off[i] + k;
            for (int c = 0; c < 6; ++c) kf_anchor[6 * (size_t)K + c] = g.kf_init[6 * (size_t)k + c];
            kf_pinfo[K] = g.kf_anchor_info ? g.kf_anchor_info[k] : 0.0;
            kf_prob[K] = i;
        }
        for (int r = 0; r < g.n_landmarks; ++r) {
            int M = p->lm_off[i] + r;
            int u = p->lm_int2user[M] - p->lm_off[i];
            for (int c = 0; c < 3; ++c) lm_anchor[3 * (size_t)M + c] = g.lm_init[3 * (size_t)u + c];
            lm_prob[M] = i;
        }
        const gbp_camera &c = cams[i];
        pp[i] = ProbParams{c.fx, c.fy, c.cx, c.cy, c.sigma_px, 1.0 / (c.sigma_px * c.sigma_px), p->opt.zmin, 0.0};
    }
    p->h_kf_anchor = kf_anchor;
    p->h_lm_anchor = lm_anchor;
    p->h_lm_anchor0 = lm_anchor;
#define UP(dst, src, bytes) HIP_TRY(p, hipMemcpyAsync((void *)(dst), (const void *)(src), (bytes), hipMemcpyHostToDevice, s))
    UP(d.kf_anchor, kf_anchor.data(), kf_anchor.size() * 8);
    // (landmark anchors go into the belief records after they are cleared)
    UP(d.kf_pinfo, kf_pinfo.data(), kf_pinfo.size() * 8);
    UP(d.kf_prob, kf_prob.data(), kf_prob.size() * 4);
    UP(d.lm_prob, lm_prob.data(), lm_prob.size() * 4);
    UP(d.kf_t0, zero_k.data(), zero_k.size() * 4);
    UP(d.lm_t0, zero_l.data(), zero_l.size() * 4);
    UP(d.prob, pp.data(), pp.size() * sizeof(ProbParams));
    UP(d.f_kf, p->h_fkf.data(), (size_t)nf * 4);
    UP(d.f_lm, p->h_flm.data(), (size_t)nf * 4);
    UP(d.kf_row, p->h_kf_row.data(), (size_t)(nk + 1) * 4);
    const std::vector<KfSlot> slots = kf_slots(p);
    d.n_kf_slots = (int)slots.size();
    if (!slots.empty()) UP(d.kf_slot, slots.data(), slots.size() * sizeof(KfSlot));
    UP(d.lm_edge, p->h_lm_edge.data(), (size_t)nf * 4);
    UP(d.lm_row, p->h_lm_row.data(), (size_t)(nl + 1) * 4);
    std::vector<int> frp(p->f_off.begin(), p->f_off.end());
    UP(d.f_row_prob, frp.data(), frp.size() * 4);
    st_rb = upload_rblk<TS>(p);
    if (st_rb != GBP_OK) return st_rb;
    UP(d.z, p->h_z.data(), (size_t)nf * 2 * 8);
    HIP_TRY(p, hipMemsetAsync(d.kf_bel, 0, (size_t)p->cap_k * KBEL * 8, s));
    HIP_TRY(p, hipMemsetAsync(d.lm_bel, 0, (size_t)p->cap_l * LBEL * 8, s));
    {
        gbp_status sa = put_lm_anchors(p, d.lm_bel, 0, p->nl, p->h_lm_anchor.data(), s);
        if (sa != GBP_OK) return sa;
    }
    HIP_TRY(p, hipMemsetAsync(d.t_dev, 0, 4, s));
    HIP_TRY(p, hipMemsetAsync(d.status, 0, 4, s));
    HIP_TRY(p, hipMemsetAsync(d.pstatus, 0, (size_t)p->np * 4, s));
    HIP_TRY(p, hipMemsetAsync(d.relin_qcount, 0, ((size_t)p->cap_f / RBLK + p->np + 1) * 4, s));
    HIP_TRY(p, hipMemcpyAsync(d.pending_k, &p->huber_k, 8, hipMemcpyHostToDevice, s));
#undef UP
    p->fdamp_buf = d.fdamp;
    d.lm_lanes = LM_LANES;
    d.relin_group = 2;  // untuned default (measured fastest on the 256-problem batch)
    d.fdamp = nullptr;
    d.fallback = nullptr;
    // initial linearisation at the initial estimate, automatic priors,
    // beliefs = priors at clock 0
    launch_linearise<TS>(d, 0, nf, p->huber_k, nullptr, s);
    launch_prior_base<TS>(d, 0, 0, s);
    launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s);
    launch_belief_kf<TS>(d, p->iopt, 0, p->blk_kf, s);
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipStreamSynchronize(s));
    return GBP_OK;
}

gbp_status create_impl(int n, const gbp_graph *gs, const gbp_camera *cams, const gbp_measurements *ms,
                       const gbp_options *opt_in, gbp_problem **out) {
    if (!out) return GBP_EINVAL;
    *out = nullptr;
    auto *p = new (std::nothrow) gbp_problem();
    if (!p) return GBP_ENOMEM;
    *out = p;
    gbp_options opt;
    if (opt_in) opt = *opt_in; else default_opts(&opt);
    p->opt = opt;
    std::string msg;
    gbp_status st = check_opts(&opt, msg);
    if (st != GBP_OK) { p->broken = true; return fail(p, st, msg); }
    if (n < 1 || !gs || !cams || !ms) { p->broken = true; return fail(p, GBP_EINVAL, "need n >= 1 problems"); }
    st = check_totals(n, gs, opt, msg);
    if (st != GBP_OK) { p->broken = true; return fail(p, st, msg); }
    for (int i = 0; i < n; ++i) {
        st = check_graph(&gs[i], &ms[i], &cams[i], msg);
        if (st != GBP_OK) { p->broken = true; return fail(p, st, "problem " + std::to_string(i) + ": " + msg); }
    }
    if (n > 1 && (opt.max_keyframes || opt.max_landmarks || opt.max_factors)) {
        p->broken = true;
        return fail(p, GBP_EINVAL, "growth capacity is only supported for a single problem");
    }
    p->precision = opt.precision;
    p->np = n;
    p->huber_k = opt.huber_k;
    if (const char *e = std::getenv("GBP_NO_GRAPH")) p->use_graph = !(e[0] == '1');
    if (const char *e = std::getenv("GBP_KF_BLOCK")) p->blk_kf = std::atoi(e);
    fill_iopt(p);
    build_order(p, n, gs, ms, p->h_fkf, p->h_flm, p->h_z);
    build_csr(p);
    p->cap_k = std::max(p->nk, (int)opt.max_keyframes);
    p->cap_l = std::max(p->nl, (int)opt.max_landmarks);
    p->cap_f = std::max(p->nf, (int)opt.max_factors);
    Layout L;
    if (p->precision == GBP_FP32) plan<float>(p, p->df, L); else plan<double>(p, p->dd, L);
    if (opt.workspace) {
        if (opt.workspace_bytes < L.total) {
            p->broken = true;
            return fail(p, GBP_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
        }
        p->ws = opt.workspace;
        p->own_ws = false;
    } else {
        hipError_t e = hipMalloc(&p->ws, L.total);
        if (e != hipSuccess) { p->broken = true; return fail(p, GBP_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)); }
        p->own_ws = true;
    }
    p->ws_bytes = L.total;
    for (auto &it : L.items) *it.first = (char *)p->ws + it.second;
    if (opt.stream) {
        p->stream = (hipStream_t)opt.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { p->broken = true; return fail(p, GBP_EDEVICE, "hipStreamCreate failed"); }
        p->own_stream = true;
    }
    st = p->precision == GBP_FP32 ? upload_and_init<float>(p, gs, cams, n) : upload_and_init<double>(p, gs, cams, n);
    if (st != GBP_OK) p->broken = true;
    return st;
}

// Model evaluation of the learned damping (every `every_k` iterations of the
// clock, before the iteration): per-problem reprojection error and the
// fallback monitor, then features and the network, which writes the
// per-factor damping used by the next factor phases.
template <typename TS>
void record_model(gbp_problem *p, hipStream_t s, bool stats_fresh) {
    Dev<TS> &d = dev<TS>(p);
    // the monitor's per-problem statistics: the previous iteration's logged
    // residual pass left them in are_out at the same beliefs, else compute
    if (!stats_fresh) launch_reproj<TS>(d, p->iopt, p->huber_k, nullptr, nullptr, nullptr, s);
    launch_monitor(d.are_out, p->np, p->fb_rise, p->d_best, p->d_fallback, d.pstatus, p->d_judge, s);
    launch_features_bf16<TS>(d, p->iopt, (uint16_t *)p->d_feat, p->d_hist, p->huber_k, s);
    launch_mlp_infer_bf16((const uint16_t *)p->d_feat, d.nf, p->d_w, d.fdamp, p->d_delta, s);
}

template <typename TS>
gbp_status record_iterations(gbp_problem *p, int n, int log_every, double *log_base) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    const TS *zref = p->has_ref ? (const TS *)p->d_zref : nullptr;
    const uint8_t *mask = p->has_ref ? p->d_mask : nullptr;
    auto model_at = [&](int i) { return p->learned && (p->t + i) % p->every_k == 0; };
    // A logged iteration followed by another (with no model evaluation in
    // between) runs the next iteration's relinearisation check inside its
    // residual pass, and the next relinearisation launch reduces the
    // residual statistics: two launches fewer per logged iteration.
    bool checked = false, stats_fresh = false;
    double *pending_row = nullptr;
    for (int i = 0; i < n; ++i) {
        if (model_at(i)) record_model<TS>(p, s, stats_fresh);
        stats_fresh = false;
        if (!checked) launch_check<TS>(d, p->iopt, s);
        launch_relin<TS>(d, p->iopt, s, pending_row);
        checked = false;
        pending_row = nullptr;
        launch_factor_kf<TS>(d, p->iopt, p->blk_kf, s, nullptr, nullptr, !p->kf_fused);
        launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s, p->kf_fused != 0);
        if (log_every > 0 && (i + 1) % log_every == 0) {
            double *row = log_base + (size_t)((i + 1) / log_every - 1) * p->np * GBP_LOG_COLS;
            if (i + 1 < n && !model_at(i + 1)) {
                launch_reproj_check<TS>(d, p->iopt, p->huber_k, zref, mask, s);
                checked = true;
                pending_row = row;
            } else {
                launch_reproj<TS>(d, p->iopt, p->huber_k, zref, mask, row, s);
                stats_fresh = true;
            }
        }
    }
    return GBP_OK;
}

template <typename TS>
gbp_status iterate_impl(gbp_problem *p, int n, double damping, double huber_k, int log_every, double *log_base) {
    p->iopt.damping = damping;
    p->iopt.huber_k = huber_k;
    p->huber_k = huber_k;
    if (n <= 0) return GBP_OK;
    hipStream_t s = p->stream;
    if (p->use_graph) {
        const int phase = p->learned ? p->t % p->every_k : -1;
        GraphEntry *hit = nullptr;
        for (auto &g : p->graphs)
            if (g.n == n && g.damping == damping && g.huber == huber_k && g.log_every == log_every && g.phase == phase)
                hit = &g;
        if (!hit) {
            if (p->graphs.size() >= 8) destroy_graphs(p);
            hipGraph_t graph;
            HIP_TRY(p, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            record_iterations<TS>(p, n, log_every, log_base);
            hipError_t le = hipGetLastError();
            hipError_t ce = hipStreamEndCapture(s, &graph);
            if (le != hipSuccess || ce != hipSuccess)
                return fail(p, GBP_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce != hipSuccess ? ce : le));
            hipGraphExec_t exec;
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(p, GBP_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
            p->graphs.push_back(GraphEntry{n, damping, huber_k, log_every, phase, exec});
            hit = &p->graphs.back();
        }
        HIP_TRY(p, hipGraphLaunch(hit->exec, s));
    } else {
        record_iterations<TS>(p, n, log_every, log_base);
        HIP_TRY(p, hipGetLastError());
    }
    p->t += n;
    return GBP_OK;
}

template <typename TS>
gbp_status phase_times_impl(gbp_problem *p, int n, double damping, double huber_k, double *ms) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    p->iopt.damping = damping;
    p->iopt.huber_k = huber_k;
    p->huber_k = huber_k;
    // all events are recorded back to back on the stream and read after one
    // synchronisation, so queue-empty launch latency is not counted
    constexpr int NPH = 5;
    std::vector<hipEvent_t> ev(NPH * (size_t)n + 1), kev(2 * (size_t)n);
    for (auto &e : ev) HIP_TRY(p, hipEventCreate(&e));
    for (auto &e : kev) HIP_TRY(p, hipEventCreate(&e));
    HIP_TRY(p, hipEventRecord(ev[0], s));
    for (int i = 0; i < n; ++i) {
        launch_check<TS>(d, p->iopt, s);
        HIP_TRY(p, hipEventRecord(ev[NPH * i + 1], s));
        launch_relin<TS>(d, p->iopt, s);
        HIP_TRY(p, hipEventRecord(ev[NPH * i + 2], s));
        launch_factor_kf<TS>(d, p->iopt, p->blk_kf, s, kev[2 * i], kev[2 * i + 1]);
        HIP_TRY(p, hipEventRecord(ev[NPH * i + 3], s));
        launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s);
        HIP_TRY(p, hipEventRecord(ev[NPH * i + 4], s));
        launch_reproj<TS>(d, p->iopt, p->huber_k, p->has_ref ? (const TS *)p->d_zref : nullptr,
                          p->has_ref ? p->d_mask : nullptr, nullptr, s);
        HIP_TRY(p, hipEventRecord(ev[NPH * i + 5], s));
    }
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipEventSynchronize(ev.back()));
    double acc[NPH + 1] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
        for (int q = 0; q < NPH; ++q) {
            float t = 0.f;
            HIP_TRY(p, hipEventElapsedTime(&t, ev[NPH * i + q], ev[NPH * i + q + 1]));
            acc[q] += t;
        }
        float t = 0.f;
        HIP_TRY(p, hipEventElapsedTime(&t, kev[2 * i], kev[2 * i + 1]));
        acc[NPH] += t;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (auto &e : kev) (void)hipEventDestroy(e);
    for (int q = 0; q <= NPH; ++q) ms[q] = acc[q] / n;
    p->t += n;
    return GBP_OK;
}

template <typename TS>
gbp_status time_config(gbp_problem *p, int n, double *ms) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    hipEvent_t a, b;
    HIP_TRY(p, hipEventCreate(&a));
    HIP_TRY(p, hipEventCreate(&b));
    HIP_TRY(p, hipEventRecord(a, s));
    for (int i = 0; i < n; ++i) {
        launch_check<TS>(d, p->iopt, s);
        launch_relin<TS>(d, p->iopt, s);
        launch_factor_kf<TS>(d, p->iopt, p->blk_kf, s, nullptr, nullptr, !p->kf_fused);
        launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s, p->kf_fused != 0);
    }
    HIP_TRY(p, hipEventRecord(b, s));
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipEventSynchronize(b));
    float t = 0.f;
    HIP_TRY(p, hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / n;
    return GBP_OK;
}

std::string tune_key(gbp_problem *p) {
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    auto lg = [](long v) { int b = 0; while (v > 1) { v >>= 1; ++b; } return b; };
    std::ostringstream os;
    os << arch.substr(0, arch.find(':')) << "/p" << p->precision << "/f" << lg(p->nf) << "/k" << lg(p->nk) << "/l"
       << lg(p->nl);
    return os.str();
}

// a whole token as a decimal integer (no trailing characters)
static bool parse_int(const std::string &t, int &v) {
    if (t.empty()) return false;
    char *end = nullptr;
    const long x = std::strtol(t.c_str(), &end, 10);
    if (*end != '\0' || x < INT32_MIN || x > INT32_MAX) return false;
    v = (int)x;
    return true;
}

// Tuning cache, a text file of one line per key: key, keyframe-kernel
// size, landmark-kernel size, lanes per landmark, relinearisation segments
// per workgroup, keyframe solves in the landmark launch (1) or apart (0),
// iteration ms.
bool cache_lookup(const char *path, const std::string &key, int &kb, int &lb, int &ll, int &rg, int &fu) {
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream is(line);
        std::vector<std::string> tok;
        for (std::string t; is >> t;) tok.push_back(t);
        // key, five integers, the time: entries of an older format (fewer
        // fields) do not match
        int a = 0, b = 0, c = 0, e = 0, g = -1;
        if (tok.size() != 7 || tok[0] != key || !parse_int(tok[1], a) || !parse_int(tok[2], b) ||
            !parse_int(tok[3], c) || !parse_int(tok[4], e) || !parse_int(tok[5], g))
            continue;
        if (e >= 1 && e <= 16 && (c == 2 || c == 4 || c == 8) && (g == 0 || g == 1) &&
            (a == 64 || a == 128 || a == 256) && (b == 64 || b == 128 || b == 256)) {
            kb = a; lb = b; ll = c; rg = e; fu = g;
            return true;
        }
    }
    return false;
}

void cache_store(const char *path, const std::string &key, int kb, int lb, int ll, int rg, int fu, double ms) {
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << kb << " " << lb << " " << ll << " " << rg << " " << fu << " " << ms << "\n";
}

// n launches of the relinearisation kernel on a synthetic queue (every 11th
// factor of each residual block)
template <typename TS>
gbp_status time_relin(gbp_problem *p, int n, double *ms) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    hipEvent_t a, b;
    HIP_TRY(p, hipEventCreate(&a));
    HIP_TRY(p, hipEventCreate(&b));
    HIP_TRY(p, hipEventRecord(a, s));
    for (int i = 0; i < n; ++i) {
        launch_queue_every<TS>(d, 11, s);
        launch_relin<TS>(d, p->iopt, s);
    }
    HIP_TRY(p, hipEventRecord(b, s));
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipEventSynchronize(b));
    float t = 0.f;
    HIP_TRY(p, hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / n;
    return GBP_OK;
}

// Autotuner: the workgroup sizes of the keyframe kernel and of the landmark
// belief kernel (3 x 3, with 4 lanes per landmark), then the lanes per
// landmark (2 / 4 / 8) with the chosen sizes, then whether the keyframe
// solves run inside the landmark-belief launch or in their own, then the
// queue segments per relinearisation workgroup (1 / 2 / 4) on a synthetic
// steady-state queue; each candidate runs n iterations (or relinearisation
// launches) from a snapshot of the workspace, which is restored after it.
template <typename TS>
gbp_status autotune_impl(gbp_problem *p, int n, const char *cache_path, int32_t *chosen) {
    Dev<TS> &d = dev<TS>(p);
    const std::string key = tune_key(p);
    int kb = 0, lb = 0, ll = 0, rg = 0, fu = 1;
    if (cache_lookup(cache_path, key, kb, lb, ll, rg, fu)) {
        p->blk_kf = kb;
        p->blk_lm = lb;
        d.lm_lanes = ll;
        d.relin_group = rg;
        p->kf_fused = fu;
    } else {
        void *snap = nullptr, *psnap = nullptr;
        HIP_TRY(p, hipMalloc(&snap, p->ws_bytes));
        HIP_TRY(p, hipMemcpyAsync(snap, p->ws, p->ws_bytes, hipMemcpyDeviceToDevice, p->stream));
        if (p->pair_mem) {
            HIP_TRY(p, hipMalloc(&psnap, p->pair_state_bytes));
            HIP_TRY(p, hipMemcpyAsync(psnap, p->pair_mem, p->pair_state_bytes, hipMemcpyDeviceToDevice, p->stream));
        }
        double best = 1e30;
        int bk = p->blk_kf, bl = p->blk_lm, bll = 4, bfu = 1;
        auto trial = [&](int x, int y, int z, int f) -> gbp_status {
            p->blk_kf = x;
            p->blk_lm = y;
            d.lm_lanes = z;
            p->kf_fused = f;
            double ms = 0;
            gbp_status st = time_config<TS>(p, n, &ms);
            if (st != GBP_OK) return st;
            HIP_TRY(p, hipMemcpyAsync(p->ws, snap, p->ws_bytes, hipMemcpyDeviceToDevice, p->stream));
            if (psnap)
                HIP_TRY(p, hipMemcpyAsync(p->pair_mem, psnap, p->pair_state_bytes, hipMemcpyDeviceToDevice, p->stream));
            if (ms < best) { best = ms; bk = x; bl = y; bll = z; bfu = f; }
            return GBP_OK;
        };
        gbp_status st = GBP_OK;
        for (int x : {64, 128, 256})
            for (int y : {64, 128, 256})
                if (st == GBP_OK) st = trial(x, y, 4, 1);
        const int bk0 = bk, bl0 = bl;
        for (int z : {2, 8})
            if (st == GBP_OK) st = trial(bk0, bl0, z, 1);
        if (st == GBP_OK) st = trial(bk, bl, bll, 0);
        p->kf_fused = bfu;
        double best_r = 1e30;
        int brg = d.relin_group;
        for (int g : {1, 2, 4}) {
            if (st != GBP_OK) break;
            d.relin_group = g;
            double ms = 0;
            st = time_relin<TS>(p, n, &ms);
            if (st != GBP_OK) break;
            HIP_TRY(p, hipMemcpyAsync(p->ws, snap, p->ws_bytes, hipMemcpyDeviceToDevice, p->stream));
            if (psnap)
                HIP_TRY(p, hipMemcpyAsync(p->pair_mem, psnap, p->pair_state_bytes, hipMemcpyDeviceToDevice, p->stream));
            if (ms < best_r) { best_r = ms; brg = g; }
        }
        HIP_TRY(p, hipStreamSynchronize(p->stream));
        (void)hipFree(snap);
        if (psnap) (void)hipFree(psnap);
        if (st != GBP_OK) return st;
        p->blk_kf = bk;
        p->blk_lm = bl;
        d.lm_lanes = bll;
        d.relin_group = brg;
        p->kf_fused = bfu;
        cache_store(cache_path, key, bk, bl, bll, brg, bfu, best);
    }
    destroy_graphs(p);
    if (chosen) {
        chosen[0] = p->blk_kf; chosen[1] = p->blk_lm; chosen[2] = d.lm_lanes; chosen[3] = d.relin_group;
        chosen[4] = p->kf_fused;
    }
    return GBP_OK;
}

// caller factor index -> internal slot, on the device
gbp_status upload_u2i(gbp_problem *p) {
    std::vector<int> u2i(p->nf);
    for (int i = 0; i < p->nf; ++i) u2i[p->f_int2user[i]] = i;
    HIP_TRY(p, hipMemcpyAsync(p->d_u2i, u2i.data(), (size_t)p->nf * 4, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return GBP_OK;
}

// Buffers of the learned damping (features, history, heads, weights, index
// map, monitor state), sized by the factor capacity: one device allocation
// of about 116 bytes per factor, owned by the problem.
gbp_status ensure_learn_mem(gbp_problem *p) {
    if (p->learn_mem) return GBP_OK;
    Layout L;
    const size_t F = p->cap_f, P = p->np;
    L.add((void **)&p->d_feat, F * NFEAT * 4);
    L.add((void **)&p->d_hist, F * FHIST * 4);
    L.add((void **)&p->d_delta, F * 4);
    L.add((void **)&p->d_w, MLP_NPARAMS * 2);
    L.add((void **)&p->d_u2i, F * 4);
    L.add((void **)&p->d_lms, (size_t)p->cap_l * 4);
    L.add((void **)&p->d_fallback, P * 4);
    L.add((void **)&p->d_judge, P * 4);
    L.add((void **)&p->d_best, P * 8);
    void *mem = nullptr;
    if (hipMalloc(&mem, L.total) != hipSuccess) return fail(p, GBP_ENOMEM, "cannot allocate the learned-model buffers");
    p->learn_mem = mem;
    for (auto &it : L.items) *it.first = (char *)mem + it.second;
    hipStream_t s = p->stream;
    HIP_TRY(p, hipMemsetAsync(p->d_hist, 0, F * FHIST * 4, s));
    HIP_TRY(p, hipMemsetAsync(p->d_fallback, 0, P * 4, s));
    p->h_judge.assign(P, -1);
    HIP_TRY(p, hipMemcpyAsync(p->d_judge, p->h_judge.data(), P * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    std::vector<double> inf(P, HUGE_VAL);
    HIP_TRY(p, hipMemcpyAsync(p->d_best, inf.data(), P * 8, hipMemcpyHostToDevice, s));
    launch_fill_f32(p->fdamp_buf, -1.f, (int)F, s);
    HIP_TRY(p, hipGetLastError());
    return upload_u2i(p);
}

// Incremental growth (Section 9.2) of a single problem. Factor state is kept
// keyframe-major, so the factor arrays are permuted on the device (old slots
// gathered, new slots zeroed) and the index arrays rebuilt; new factors are
// linearised at the current means, new variables get automatic priors from
// their factors and their own annealing clock, and beliefs are re-formed
// (existing ones only gain the new factors' zero messages).
template <typename TS>
gbp_status add_impl(gbp_problem *p, const double *pose, int n_new_lm, const double *lm_init, int n_new_f,
                    const int32_t *f_kf, const int32_t *f_lm, const double *z) {
    if (p->np != 1) return fail(p, GBP_ESTATE, "incremental growth needs a single (non-batched) problem");
    if (n_new_lm < 0 || n_new_f < 0 || (n_new_lm > 0 && !lm_init) || (n_new_f > 0 && (!f_kf || !f_lm || !z)))
        return fail(p, GBP_EINVAL, "bad growth arguments");
    const int nk0 = p->nk, nl0 = p->nl, nf0 = p->nf;
    // sums in 64 bits: a count near INT32_MAX must fail the capacity test,
    // not wrap below it
    if ((long long)nk0 + (pose ? 1 : 0) > p->cap_k || (long long)nl0 + n_new_lm > p->cap_l ||
        (long long)nf0 + n_new_f > p->cap_f)
        return fail(p, GBP_ENOMEM, "growth exceeds the capacity set at creation (max_keyframes/landmarks/factors)");
    const int nk1 = nk0 + (pose ? 1 : 0), nl1 = nl0 + n_new_lm, nf1 = nf0 + n_new_f;
    for (int i = 0; i < n_new_f; ++i) {
        if (f_kf[i] < 0 || f_kf[i] >= nk1 || f_lm[i] < 0 || f_lm[i] >= nl1)
            return fail(p, GBP_EINVAL, "new factor " + std::to_string(i) + " has an out-of-range variable index");
        if (!std::isfinite(z[2 * i]) || !std::isfinite(z[2 * i + 1]))
            return fail(p, GBP_EINVAL, "new factor " + std::to_string(i) + " has a non-finite measurement");
    }
    if (pose)
        for (int c = 0; c < 6; ++c)
            if (!std::isfinite(pose[c])) return fail(p, GBP_EINVAL, "non-finite keyframe pose");
    for (long i = 0; i < 3L * n_new_lm; ++i)
        if (!std::isfinite(lm_init[i])) return fail(p, GBP_EINVAL, "non-finite landmark position");
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    // caller landmark index -> internal index (new landmarks are appended)
    std::vector<int> lm_user2int(nl1);
    for (int m = 0; m < nl0; ++m) lm_user2int[p->lm_int2user[m]] = m;
    for (int j = 0; j < n_new_lm; ++j) lm_user2int[nl0 + j] = nl0 + j;
    // all factors (old: internal order; new appended), then keyframe-major order
    std::vector<int> fk(nf1), fl(nf1), src(nf1), user(nf1);
    std::vector<double> zz(2 * (size_t)nf1);
    for (int f = 0; f < nf0; ++f) {
        fk[f] = p->h_fkf[f]; fl[f] = p->h_flm[f]; src[f] = f; user[f] = p->f_int2user[f];
        zz[2 * f] = p->h_z[2 * f]; zz[2 * f + 1] = p->h_z[2 * f + 1];
    }
    for (int i = 0; i < n_new_f; ++i) {
        const int f = nf0 + i;
        fk[f] = f_kf[i]; fl[f] = lm_user2int[f_lm[i]]; src[f] = -1; user[f] = nf0 + i;
        zz[2 * (size_t)f] = z[2 * i]; zz[2 * (size_t)f + 1] = z[2 * i + 1];
    }
    std::vector<int> order(nf1);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (fk[x] != fk[y]) return fk[x] < fk[y];
        return fl[x] < fl[y];
    });
    std::vector<int> perm(nf1), fresh;
    p->h_fkf.resize(nf1); p->h_flm.resize(nf1); p->h_z.resize(2 * (size_t)nf1); p->f_int2user.resize(nf1);
    for (int r = 0; r < nf1; ++r) {
        const int f = order[r];
        perm[r] = src[f];
        if (src[f] < 0) fresh.push_back(r);
        p->h_fkf[r] = fk[f]; p->h_flm[r] = fl[f]; p->f_int2user[r] = user[f];
        p->h_z[2 * (size_t)r] = zz[2 * (size_t)f]; p->h_z[2 * (size_t)r + 1] = zz[2 * (size_t)f + 1];
    }
    p->nk = nk1; p->nl = nl1; p->nf = nf1;
    p->grown = true;
    p->has_ref = false;  // the reference covered the old factor set
    p->kf_off = {0, nk1}; p->lm_off = {0, nl1}; p->f_off = {0, nf1};
    for (int j = 0; j < n_new_lm; ++j) p->lm_int2user.push_back(nl0 + j);
    build_csr(p);
    // new variables: anchors (initial estimates), clocks, problem index
    if (pose) p->h_kf_anchor.insert(p->h_kf_anchor.end(), pose, pose + 6);
    p->h_lm_anchor.insert(p->h_lm_anchor.end(), lm_init, lm_init + 3 * (size_t)n_new_lm);
#define UP(dst, srcp, bytes) HIP_TRY(p, hipMemcpyAsync((void *)(dst), (const void *)(srcp), (bytes), hipMemcpyHostToDevice, s))
    std::vector<int> tk(nk1 - nk0, p->t), tl(n_new_lm, p->t), zk(nk1 - nk0, 0), zl(n_new_lm, 0);
    std::vector<double> pk(nk1 - nk0, 0.0);
    if (pose) {
        UP(d.kf_anchor + 6 * (size_t)nk0, pose, 6 * 8);
        UP(d.kf_pinfo + nk0, pk.data(), 8);
        UP(d.kf_t0 + nk0, tk.data(), 4);
        UP(d.kf_prob + nk0, zk.data(), 4);
        HIP_TRY(p, hipMemsetAsync(d.kf_bel + (size_t)nk0 * KBEL, 0, KBEL * 8, s));
    }
    if (n_new_lm) {
        UP(d.lm_t0 + nl0, tl.data(), 4 * (size_t)n_new_lm);
        UP(d.lm_prob + nl0, zl.data(), 4 * (size_t)n_new_lm);
        HIP_TRY(p, hipMemsetAsync(d.lm_bel + (size_t)nl0 * LBEL, 0, (size_t)n_new_lm * LBEL * 8, s));
        gbp_status sa = put_lm_anchors(p, d.lm_bel, nl0, n_new_lm, lm_init, s);
        if (sa != GBP_OK) return sa;
    }
    // permute the device factor state into the new order
    UP(p->d_perm, perm.data(), (size_t)nf1 * 4);
    launch_permute_factors<TS>(d, p->d_perm, nf1, p->d_scratch, p->learn_mem ? p->fdamp_buf : nullptr,
                               p->d_hist, s);
    UP(d.f_kf, p->h_fkf.data(), (size_t)nf1 * 4);
    UP(d.f_lm, p->h_flm.data(), (size_t)nf1 * 4);
    UP(d.z, p->h_z.data(), (size_t)nf1 * 2 * 8);
    UP(d.kf_row, p->h_kf_row.data(), (size_t)(nk1 + 1) * 4);
    const std::vector<KfSlot> kslots = kf_slots(p);
    d.n_kf_slots = (int)kslots.size();
    UP(d.kf_slot, kslots.data(), kslots.size() * sizeof(KfSlot));
    UP(d.lm_row, p->h_lm_row.data(), (size_t)(nl1 + 1) * 4);
    UP(d.lm_edge, p->h_lm_edge.data(), (size_t)nf1 * 4);
    std::vector<int> frp = {0, nf1};
    UP(d.f_row_prob, frp.data(), 8);
    d.nk = nk1; d.nl = nl1; d.nf = nf1;
    gbp_status st = upload_rblk<TS>(p);
    if (st != GBP_OK) return st;
    // new factors: linearise at the current means (their slots are scattered)
    if (!fresh.empty()) {
        UP(p->d_perm, fresh.data(), fresh.size() * 4);
        launch_linearise<TS>(d, 0, (int)fresh.size(), p->huber_k, p->d_perm, s);
    }
#undef UP
    launch_prior_base<TS>(d, nk0, nl0, s);
    launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s);
    launch_belief_kf<TS>(d, p->iopt, 0, p->blk_kf, s);
    HIP_TRY(p, hipGetLastError());
    if (p->learn_mem) {
        // the fallback monitor restarts: the new factors raise the error
        st = upload_u2i(p);
        if (st != GBP_OK) return st;
        const double inf = HUGE_VAL;
        HIP_TRY(p, hipMemcpyAsync(p->d_best, &inf, 8, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(p, hipStreamSynchronize(s));
    destroy_graphs(p);
    return GBP_OK;
}

template <typename TS>
gbp_status features_impl(gbp_problem *p, const int32_t *idx, int n, float *out) {
    gbp_status st = ensure_learn_mem(p);
    if (st != GBP_OK) return st;
    Dev<TS> &d = dev<TS>(p);
    launch_features<TS>(d, p->iopt, p->d_feat, p->d_hist, p->huber_k, p->stream);
    launch_gather_rows(p->d_feat, out, idx, p->d_u2i, p->nf, n, NFEAT, p->stream);
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return GBP_OK;
}

template <typename TS>
gbp_status messages_impl(gbp_problem *p, const int32_t *idx, int n, float *out) {
    gbp_status st = ensure_learn_mem(p);
    if (st != GBP_OK) return st;
    launch_export_messages<TS>(dev<TS>(p), idx, p->d_u2i, n, out, p->stream);
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return GBP_OK;
}

// Learned depth for the listed (internal) landmarks: a fresh evaluation of
// the network, the move along the ray, then every factor of a moved
// landmark relinearised at the new position with zero messages, and the
// beliefs re-formed.
template <typename TS>
gbp_status depth_impl(gbp_problem *p, const std::vector<int> &lms) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    std::vector<int> fl;
    for (int m : lms)
        for (int e = p->h_lm_row[m]; e < p->h_lm_row[m + 1]; ++e) fl.push_back(p->h_lm_edge[e]);
    std::sort(fl.begin(), fl.end());
    if (!lms.empty())
        HIP_TRY(p, hipMemcpyAsync(p->d_lms, lms.data(), lms.size() * 4, hipMemcpyHostToDevice, s));
    if (!fl.empty())
        HIP_TRY(p, hipMemcpyAsync(p->d_perm, fl.data(), fl.size() * 4, hipMemcpyHostToDevice, s));
    launch_features_bf16<TS>(d, p->iopt, (uint16_t *)p->d_feat, p->d_hist, p->huber_k, s);
    launch_mlp_infer_bf16((const uint16_t *)p->d_feat, d.nf, p->d_w, d.fdamp, p->d_delta, s);
    launch_depth_move<TS>(d, p->d_lms, (int)lms.size(), p->d_delta, s);
    launch_linearise<TS>(d, 0, (int)fl.size(), p->huber_k, p->d_perm, s);
    launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s);
    launch_belief_kf<TS>(d, p->iopt, 0, p->blk_kf, s);
    HIP_TRY(p, hipGetLastError());
    // the host mirror of the anchors (absolute means = anchor + offset)
    {
        gbp_status sa = get_lm_anchors(p, d.lm_bel, p->nl, p->h_lm_anchor.data(), s);
        if (sa != GBP_OK) return sa;
    }
    HIP_TRY(p, hipStreamSynchronize(s));
    return GBP_OK;
}

// Every problem back on the learned damping, except the plain-GBP judges
// (they run the constant damping throughout).
gbp_status reset_fallback(gbp_problem *p) {
    std::vector<int> fb(p->np, 0);
    for (int i = 0; i < p->np && i < (int)p->h_judge.size(); ++i) fb[i] = p->h_judge[i] == -2 ? 1 : 0;
    HIP_TRY(p, hipMemcpyAsync(p->d_fallback, fb.data(), (size_t)p->np * 4, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return GBP_OK;
}

gbp_status set_model_impl(gbp_problem *p, const uint16_t *w, int every_k, double rise) {
    destroy_graphs(p);
    if (!w) {
        p->learned = false;
        p->df.fdamp = nullptr; p->dd.fdamp = nullptr;
        p->df.fallback = nullptr; p->dd.fallback = nullptr;
        return GBP_OK;
    }
    gbp_status st = ensure_learn_mem(p);
    if (st != GBP_OK) return st;
    hipStream_t s = p->stream;
    HIP_TRY(p, hipMemcpyAsync(p->d_w, w, MLP_NPARAMS * 2, hipMemcpyHostToDevice, s));
    st = reset_fallback(p);
    if (st != GBP_OK) return st;
    std::vector<double> inf(p->np, HUGE_VAL);
    HIP_TRY(p, hipMemcpyAsync(p->d_best, inf.data(), (size_t)p->np * 8, hipMemcpyHostToDevice, s));
    launch_fill_f32(p->fdamp_buf, -1.f, p->cap_f, s);
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipStreamSynchronize(s));
    p->learned = true;
    p->every_k = every_k;
    p->fb_rise = rise > -1.0 ? rise : HUGE_VAL;
    p->df.fdamp = p->fdamp_buf; p->dd.fdamp = p->fdamp_buf;
    p->df.fallback = p->d_fallback; p->dd.fallback = p->d_fallback;
    return GBP_OK;
}

// Pairwise difference factors: append n of `kind` (indices already
// internal), rebuild the device allocation (messages and counts of the
// existing pairs are kept, the new ones start at zero), rebuild the pair
// lists of the variables, and recompute the beliefs so that the belief
// information the pair update reads exists before the next iteration.
template <typename TS>
gbp_status pairs_impl(gbp_problem *p, int kind, const std::vector<int> &ab, const std::vector<double> &zp,
                      int type) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    HIP_TRY(p, hipStreamSynchronize(s));
    const int n_old[2] = {d.n_pair[0], d.n_pair[1]};
    p->h_pair_ab[kind].insert(p->h_pair_ab[kind].end(), ab.begin(), ab.end());
    p->h_pair_zp[kind].insert(p->h_pair_zp[kind].end(), zp.begin(), zp.end());
    if (kind == 0) p->h_pair_type0.insert(p->h_pair_type0.end(), ab.size() / 2, type);
    const int n[2] = {(int)p->h_pair_ab[0].size() / 2, (int)p->h_pair_ab[1].size() / 2};
    const int Ds[2] = {6, 3};
    // layout: messages and counts first (the state that reset clears and
    // the autotuner snapshots), then the constant data
    Layout L;
    double *msg[2];
    int *cnt[2], *abd[2];
    double *zpd[2];
    for (int k = 0; k < 2; ++k) L.add((void **)&msg[k], (size_t)n[k] * pair_msg_doubles(Ds[k]) * 8);
    for (int k = 0; k < 2; ++k) L.add((void **)&cnt[k], (size_t)n[k] * 4);
    const size_t state_bytes = L.total;
    for (int k = 0; k < 2; ++k) {
        L.add((void **)&abd[k], (size_t)n[k] * 2 * 4);
        L.add((void **)&zpd[k], (size_t)n[k] * 2 * Ds[k] * 8);
    }
    int *typed = nullptr;
    L.add((void **)&typed, (size_t)n[0] * 4);
    // pair lists: entry 2 i + side (side 0: end a, 1: end b), increasing i
    std::vector<int> row[2], ent[2];
    const int nv[2] = {p->nk, p->nl};
    for (int k = 0; k < 2; ++k) {
        row[k].assign(nv[k] + 1, 0);
        for (int i = 0; i < n[k]; ++i)
            for (int side = 0; side < 2; ++side) row[k][p->h_pair_ab[k][2 * i + side] + 1]++;
        for (int v = 0; v < nv[k]; ++v) row[k][v + 1] += row[k][v];
        ent[k].resize(2 * (size_t)n[k]);
        std::vector<int> fill(row[k].begin(), row[k].end() - 1);
        for (int i = 0; i < n[k]; ++i)
            for (int side = 0; side < 2; ++side) ent[k][fill[p->h_pair_ab[k][2 * i + side]]++] = 2 * i + side;
    }
    int *rowd[2], *entd[2];
    for (int k = 0; k < 2; ++k) {
        L.add((void **)&rowd[k], (size_t)(nv[k] + 1) * 4);
        L.add((void **)&entd[k], ent[k].size() * 4 + 4);
    }
    double *kbi = nullptr, *lbi = nullptr;
    if (n[0] > 0) L.add((void **)&kbi, (size_t)p->cap_k * KBI * 8);
    if (n[1] > 0) L.add((void **)&lbi, (size_t)p->cap_l * LBI * 8);
    void *mem = nullptr;
    if (hipMalloc(&mem, L.total) != hipSuccess) return fail(p, GBP_ENOMEM, "cannot allocate the pairwise factors");
    for (auto &it : L.items) *it.first = (char *)mem + it.second;
    HIP_TRY(p, hipMemsetAsync(mem, 0, state_bytes, s));
    if (n[0] > 0)
        HIP_TRY(p, hipMemcpyAsync(typed, p->h_pair_type0.data(), (size_t)n[0] * 4, hipMemcpyHostToDevice, s));
    for (int k = 0; k < 2; ++k) {
        if (n_old[k] > 0) {
            HIP_TRY(p, hipMemcpyAsync(msg[k], d.pair_msg[k], (size_t)n_old[k] * pair_msg_doubles(Ds[k]) * 8,
                                      hipMemcpyDeviceToDevice, s));
            HIP_TRY(p, hipMemcpyAsync(cnt[k], d.pair_cnt[k], (size_t)n_old[k] * 4, hipMemcpyDeviceToDevice, s));
        }
        if (n[k] > 0) {
            HIP_TRY(p, hipMemcpyAsync(abd[k], p->h_pair_ab[k].data(), p->h_pair_ab[k].size() * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(p, hipMemcpyAsync(zpd[k], p->h_pair_zp[k].data(), p->h_pair_zp[k].size() * 8, hipMemcpyHostToDevice, s));
        }
        HIP_TRY(p, hipMemcpyAsync(rowd[k], row[k].data(), row[k].size() * 4, hipMemcpyHostToDevice, s));
        if (!ent[k].empty())
            HIP_TRY(p, hipMemcpyAsync(entd[k], ent[k].data(), ent[k].size() * 4, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(p, hipStreamSynchronize(s));
    if (p->pair_mem) (void)hipFree(p->pair_mem);
    p->pair_mem = mem;
    p->pair_state_bytes = state_bytes;
    for (int k = 0; k < 2; ++k) {
        d.n_pair[k] = n[k];
        d.pair_ab[k] = abd[k];
        d.pair_zp[k] = zpd[k];
        d.pair_cnt[k] = cnt[k];
        d.pair_msg[k] = msg[k];
    }
    d.pair_type0 = typed;
    d.kp_row = rowd[0]; d.kp_ent = entd[0];
    d.lp_row = rowd[1]; d.lp_ent = entd[1];
    d.kf_binfo = kbi;
    d.lm_binfo = lbi;
    destroy_graphs(p);
    // beliefs again from the current messages (the new pairs' are zero):
    // the same beliefs, now with their information form stored
    launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s);
    launch_belief_kf<TS>(d, p->iopt, 0, p->blk_kf, s);
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipStreamSynchronize(s));
    return GBP_OK;
}

// Back to the state right after creation (initial linearisation, zero
// messages, beliefs = priors at clock 0); buffers, recorded graphs, the
// reference and the damping model stay.
template <typename TS>
gbp_status reset_impl(gbp_problem *p) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    p->huber_k = p->opt.huber_k;
    p->iopt.huber_k = p->opt.huber_k;
    p->h_lm_anchor = p->h_lm_anchor0;
    HIP_TRY(p, hipMemsetAsync(d.kf_bel, 0, (size_t)p->cap_k * KBEL * 8, s));
    HIP_TRY(p, hipMemsetAsync(d.lm_bel, 0, (size_t)p->cap_l * LBEL * 8, s));
    {
        gbp_status sa = put_lm_anchors(p, d.lm_bel, 0, p->nl, p->h_lm_anchor.data(), s);
        if (sa != GBP_OK) return sa;
    }
    HIP_TRY(p, hipMemsetAsync(d.t_dev, 0, 4, s));
    HIP_TRY(p, hipMemsetAsync(d.status, 0, 4, s));
    HIP_TRY(p, hipMemsetAsync(d.pstatus, 0, (size_t)p->np * 4, s));
    HIP_TRY(p, hipMemsetAsync(d.relin_qcount, 0, ((size_t)p->cap_f / RBLK + p->np + 1) * 4, s));
    HIP_TRY(p, hipMemcpyAsync(d.pending_k, &p->huber_k, 8, hipMemcpyHostToDevice, s));
    if (p->pair_mem) HIP_TRY(p, hipMemsetAsync(p->pair_mem, 0, p->pair_state_bytes, s));  // pair messages, counts
    launch_linearise<TS>(d, 0, p->nf, p->huber_k, nullptr, s);
    launch_prior_base<TS>(d, 0, 0, s);
    launch_belief_lm<TS>(d, p->iopt, 0, p->blk_lm, s);
    launch_belief_kf<TS>(d, p->iopt, 0, p->blk_kf, s);
    if (p->learn_mem) {
        HIP_TRY(p, hipMemsetAsync(p->d_hist, 0, (size_t)p->cap_f * FHIST * 4, s));
        gbp_status sf = reset_fallback(p);
        if (sf != GBP_OK) return sf;
        std::vector<double> inf(p->np, HUGE_VAL);
        HIP_TRY(p, hipMemcpyAsync(p->d_best, inf.data(), (size_t)p->np * 8, hipMemcpyHostToDevice, s));
        launch_fill_f32(p->fdamp_buf, -1.f, p->cap_f, s);
    }
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, hipStreamSynchronize(s));
    p->t = 0;
    return GBP_OK;
}

gbp_status check_live(gbp_problem *p) {
    if (!p) return GBP_EINVAL;
    if (p->broken) return fail(p, GBP_ESTATE, "problem creation failed: " + p->err);
    return GBP_OK;
}

template <typename TS>
gbp_status status_check(gbp_problem *p) {
    unsigned st = 0;
    HIP_TRY(p, hipMemcpyAsync(&st, dev<TS>(p).status, 4, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (st) {
        HIP_TRY(p, hipMemsetAsync(dev<TS>(p).status, 0, 4, p->stream));
        return fail(p, GBP_ENUMERIC, st & 1 ? "a belief information matrix was not positive definite"
                                            : "a belief mean was not finite");
    }
    return GBP_OK;
}

template <typename TS>
gbp_status beliefs_impl(gbp_problem *p, double *kf_mean, double *lm_mean, double *kf_info, double *lm_info) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    const int readout = (kf_info || lm_info) ? 1 : 0;
    if (readout) {
        launch_belief_lm<TS>(d, p->iopt, 1, p->blk_lm, s);
        launch_belief_kf<TS>(d, p->iopt, 1, p->blk_kf, s);
        HIP_TRY(p, hipGetLastError());
    }
    std::vector<double> kb((size_t)p->nk * KBEL), lb((size_t)p->nl * LBEL), ki, li;
    HIP_TRY(p, hipMemcpyAsync(kb.data(), d.kf_bel, kb.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipMemcpyAsync(lb.data(), d.lm_bel, lb.size() * 8, hipMemcpyDeviceToHost, s));
    if (kf_info) { ki.resize((size_t)p->nk * 36); HIP_TRY(p, hipMemcpyAsync(ki.data(), d.kf_info, ki.size() * 8, hipMemcpyDeviceToHost, s)); }
    if (lm_info) { li.resize((size_t)p->nl * 9); HIP_TRY(p, hipMemcpyAsync(li.data(), d.lm_info, li.size() * 8, hipMemcpyDeviceToHost, s)); }
    gbp_status st = status_check<TS>(p);
    for (int k = 0; k < p->nk; ++k) {
        if (kf_mean)
            for (int c = 0; c < 6; ++c) kf_mean[6 * (size_t)k + c] = p->h_kf_anchor[6 * (size_t)k + c] + kb[(size_t)k * KBEL + c];
        if (kf_info) std::memcpy(kf_info + 36 * (size_t)k, ki.data() + 36 * (size_t)k, 36 * 8);
    }
    for (int m = 0; m < p->nl; ++m) {
        int u = p->lm_int2user[m];
        if (lm_mean)
            for (int c = 0; c < 3; ++c) lm_mean[3 * (size_t)u + c] = p->h_lm_anchor[3 * (size_t)m + c] + lb[(size_t)m * LBEL + c];
        if (lm_info) std::memcpy(lm_info + 9 * (size_t)u, li.data() + 9 * (size_t)m, 9 * 8);
    }
    return st;
}

template <typename TS>
gbp_status reproj_impl(gbp_problem *p, std::vector<double> &sums) {
    Dev<TS> &d = dev<TS>(p);
    launch_reproj<TS>(d, p->iopt, p->huber_k, p->has_ref ? (const TS *)p->d_zref : nullptr,
                      p->has_ref ? p->d_mask : nullptr, nullptr,
                      p->stream);
    HIP_TRY(p, hipGetLastError());
    sums.resize((size_t)p->np * 8);
    HIP_TRY(p, hipMemcpyAsync(sums.data(), d.are_out, sums.size() * 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return GBP_OK;
}

void sums_to_stats(const double *s, gbp_reproj *o) {
    o->are_all = s[3] > 0 ? s[0] / s[3] : 0.0;
    const double nq = s[3] - s[5];  // valid factors in the quadratic regime
    o->are_quadratic = nq > 0 ? s[1] / nq : 0.0;
    o->are_ref = s[7] > 0 ? s[2] / s[7] : 0.0;
    o->n_valid = (int64_t)s[3];
    o->n_quadratic = (int64_t)nq;
    o->n_linear = (int64_t)s[5];
    o->n_invalid = (int64_t)s[6];
    o->n_ref = (int64_t)s[7];
    o->n_linear_ref = (int64_t)s[4];
}

template <typename TS>
gbp_status relin_impl(gbp_problem *p, double beta, int32_t *n_relin) {
    Dev<TS> &d = dev<TS>(p);
    hipStream_t s = p->stream;
    HIP_TRY(p, hipMemcpyAsync(d.pending_k, &p->huber_k, 8, hipMemcpyHostToDevice, s));
    HIP_TRY(p, hipMemsetAsync(p->d_count, 0, 4, s));
    launch_flag_relin<TS>(d, beta, p->d_count, s);
    HIP_TRY(p, hipGetLastError());
    int cnt = 0;
    HIP_TRY(p, hipMemcpyAsync(&cnt, p->d_count, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    if (n_relin) *n_relin = cnt;
    return GBP_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

void gbp_default_options(gbp_options *opt) {
    if (opt) default_opts(opt);
}

gbp_status gbp_workspace_bytes(int32_t n, const gbp_graph *gs, const gbp_options *opt_in, size_t *bytes) {
    if (!bytes || n < 1 || !gs) return GBP_EINVAL;
    gbp_options opt;
    if (opt_in) opt = *opt_in; else default_opts(&opt);
    std::string msg;
    if (check_totals(n, gs, opt, msg) != GBP_OK) {
        g_err = "gbp_workspace_bytes: " + msg;
        return GBP_EINVAL;
    }
    gbp_problem tmp;
    tmp.np = n;
    long nk = 0, nl = 0, nf = 0;
    for (int i = 0; i < n; ++i) { nk += gs[i].n_keyframes; nl += gs[i].n_landmarks; nf += gs[i].n_factors; }
    tmp.cap_k = (int)std::max(nk, (long)opt.max_keyframes);
    tmp.cap_l = (int)std::max(nl, (long)opt.max_landmarks);
    tmp.cap_f = (int)std::max(nf, (long)opt.max_factors);
    Layout L;
    if (opt.precision == GBP_FP64) plan<double>(&tmp, tmp.dd, L); else plan<float>(&tmp, tmp.df, L);
    *bytes = L.total;
    return GBP_OK;
}

gbp_status gbp_create(const gbp_graph *graph, const gbp_camera *camera, const gbp_measurements *meas,
                      const gbp_options *opt, gbp_problem **out) {
    return create_impl(1, graph, camera, meas, opt, out);
}

gbp_status gbp_create_batch(int32_t n, const gbp_graph *graphs, const gbp_camera *cameras,
                            const gbp_measurements *meas, const gbp_options *opt, gbp_problem **out) {
    return create_impl(n, graphs, cameras, meas, opt, out);
}

gbp_status gbp_relinearise(gbp_problem *p, double beta, int32_t *n_relin) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (std::isnan(beta)) return fail(p, GBP_EINVAL, "gbp_relinearise: beta is NaN");
    return p->precision == GBP_FP32 ? relin_impl<float>(p, beta, n_relin) : relin_impl<double>(p, beta, n_relin);
}

gbp_status gbp_iterate(gbp_problem *p, int32_t n, double damping, double huber_k) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (n < 0 || !(damping >= 0.0 && damping < 1.0) || !std::isfinite(huber_k))
        return fail(p, GBP_EINVAL, "need n >= 0, 0 <= damping < 1, finite huber_k");
    return p->precision == GBP_FP32 ? iterate_impl<float>(p, n, damping, huber_k, 0, nullptr)
                                    : iterate_impl<double>(p, n, damping, huber_k, 0, nullptr);
}

gbp_status gbp_iterate_logged(gbp_problem *p, int32_t n, double damping, double huber_k, int32_t log_every,
                              double *log_out) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (n < 0 || log_every < 1 || !log_out || !(damping >= 0.0 && damping < 1.0) || !std::isfinite(huber_k))
        return fail(p, GBP_EINVAL, "need n >= 0, log_every >= 1, a log buffer, 0 <= damping < 1 and finite huber_k");
    const size_t rows = (size_t)(n / log_every);
    const size_t bytes = std::max<size_t>(rows, 1) * p->np * GBP_LOG_COLS * 8;
    if (bytes > p->log_cap) {
        destroy_graphs(p);  // graphs may reference the old log buffer
        if (p->d_log) (void)hipFree(p->d_log);
        p->d_log = nullptr;
        HIP_TRY(p, hipMalloc(&p->d_log, bytes));
        p->log_cap = bytes;
    }
    st = p->precision == GBP_FP32 ? iterate_impl<float>(p, n, damping, huber_k, log_every, p->d_log)
                                  : iterate_impl<double>(p, n, damping, huber_k, log_every, p->d_log);
    if (st != GBP_OK) return st;
    if (rows) HIP_TRY(p, hipMemcpyAsync(log_out, p->d_log, rows * p->np * GBP_LOG_COLS * 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return GBP_OK;
}

gbp_status gbp_beliefs(gbp_problem *p, double *kf_mean, double *lm_mean, double *kf_info, double *lm_info) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    return p->precision == GBP_FP32 ? beliefs_impl<float>(p, kf_mean, lm_mean, kf_info, lm_info)
                                    : beliefs_impl<double>(p, kf_mean, lm_mean, kf_info, lm_info);
}

gbp_status gbp_reproj_stats(gbp_problem *p, int32_t problem_index, gbp_reproj *out) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (!out || problem_index < -1 || problem_index >= p->np) return fail(p, GBP_EINVAL, "bad problem index");
    std::vector<double> sums;
    st = p->precision == GBP_FP32 ? reproj_impl<float>(p, sums) : reproj_impl<double>(p, sums);
    if (st != GBP_OK) return st;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < p->np; ++i) {
        if (problem_index >= 0 && i != problem_index) continue;
        for (int c = 0; c < 8; ++c) acc[c] += sums[8 * (size_t)i + c];
    }
    sums_to_stats(acc, out);
    return GBP_OK;
}

gbp_status gbp_reproj_error(gbp_problem *p, double *are_all, double *are_inlier_quadratic, int32_t *n_linear_regime) {
    gbp_reproj r;
    gbp_status st = gbp_reproj_stats(p, -1, &r);
    if (st != GBP_OK) return st;
    if (are_all) *are_all = r.are_all;
    if (are_inlier_quadratic) *are_inlier_quadratic = r.are_quadratic;
    if (n_linear_regime) *n_linear_regime = (int32_t)r.n_linear;
    return GBP_OK;
}

gbp_status gbp_set_reference(gbp_problem *p, const double *z_ref, const uint8_t *mask) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (!z_ref || !mask) {
        p->has_ref = false;
        destroy_graphs(p);
        return GBP_OK;
    }
    std::vector<double> zr(2 * (size_t)p->nf);
    std::vector<uint8_t> mk(p->nf);
    for (int f = 0; f < p->nf; ++f) {
        int u = p->f_int2user[f];
        zr[2 * (size_t)f] = z_ref[2 * (size_t)u];
        zr[2 * (size_t)f + 1] = z_ref[2 * (size_t)u + 1];
        mk[f] = mask[u] ? 1 : 0;
    }
    // in the factor-state precision (used for statistics only: in FP32 the
    // rounding is below 1e-4 px for pixels under 2048)
    std::vector<float> zf;
    if (p->precision == GBP_FP32) zf.assign(zr.begin(), zr.end());
    if (p->precision == GBP_FP32)
        HIP_TRY(p, hipMemcpyAsync(p->d_zref, zf.data(), zf.size() * 4, hipMemcpyHostToDevice, p->stream));
    else
        HIP_TRY(p, hipMemcpyAsync(p->d_zref, zr.data(), zr.size() * 8, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipMemcpyAsync(p->d_mask, mk.data(), mk.size(), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (!p->has_ref) destroy_graphs(p);
    p->has_ref = true;
    return GBP_OK;
}

gbp_status gbp_add_pair_factors(gbp_problem *p, int32_t kind, int32_t n, const int32_t *a, const int32_t *b,
                                const double *z, const double *precision) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (kind != GBP_PAIR_KEYFRAMES && kind != GBP_PAIR_LANDMARKS && kind != GBP_PAIR_ODOMETRY)
        return fail(p, GBP_EINVAL,
                    "gbp_add_pair_factors: kind must be GBP_PAIR_KEYFRAMES, GBP_PAIR_LANDMARKS or GBP_PAIR_ODOMETRY");
    if (n < 0 || (n > 0 && (!a || !b || !z || !precision)))
        return fail(p, GBP_EINVAL, "gbp_add_pair_factors: need n >= 0 and the four arrays");
    if (p->grown) return fail(p, GBP_ESTATE, "gbp_add_pair_factors: the problem has grown since creation");
    if (n == 0) return GBP_OK;
    if ((long long)p->h_pair_ab[kind == GBP_PAIR_LANDMARKS ? 1 : 0].size() / 2 + n > GBP_MAX_BATCH_ITEMS)
        return fail(p, GBP_EINVAL, "gbp_add_pair_factors: more than GBP_MAX_BATCH_ITEMS pair factors of one kind of "
                                   "variable");
    // odometry factors live with the keyframe pairs (D = 6 storage, 3 values
    // measured, the rest zero)
    const bool kfk = kind != GBP_PAIR_LANDMARKS;
    const int D = kfk ? 6 : 3, MD = kind == GBP_PAIR_LANDMARKS ? 3 : (kind == GBP_PAIR_ODOMETRY ? 3 : 6);
    const int nv = kfk ? p->nk : p->nl;
    std::vector<int> u2i(nv);
    for (int i = 0; i < nv; ++i) u2i[kfk ? i : p->lm_int2user[i]] = i;
    std::vector<int> ab(2 * (size_t)n);
    std::vector<double> zp(2 * (size_t)D * n, 0.0);
    for (int i = 0; i < n; ++i) {
        if (a[i] < 0 || a[i] >= nv || b[i] < 0 || b[i] >= nv || a[i] == b[i])
            return fail(p, GBP_EINVAL, "gbp_add_pair_factors: variable index out of range or a == b");
        ab[2 * (size_t)i] = u2i[a[i]];
        ab[2 * (size_t)i + 1] = u2i[b[i]];
        for (int j = 0; j < MD; ++j) {
            const double zz = z[(size_t)MD * i + j], pr = precision[(size_t)MD * i + j];
            if (!std::isfinite(zz) || !(pr > 0.0) || !std::isfinite(pr))
                return fail(p, GBP_EINVAL, "gbp_add_pair_factors: z must be finite and precisions positive");
            zp[2 * (size_t)D * i + j] = zz;
            zp[2 * (size_t)D * i + D + j] = pr;
        }
    }
    const int store = kfk ? 0 : 1, type = kind == GBP_PAIR_ODOMETRY ? 1 : 0;
    return p->precision == GBP_FP32 ? pairs_impl<float>(p, store, ab, zp, type)
                                    : pairs_impl<double>(p, store, ab, zp, type);
}

gbp_status gbp_add_keyframe(gbp_problem *p, const double pose[6], int32_t n_new_lm, const double *lm_init,
                            int32_t n_new_f, const int32_t *f_kf, const int32_t *f_lm, const double *z) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (p->pair_mem)
        return fail(p, GBP_ESTATE, "gbp_add_keyframe: problems with pairwise factors do not grow");
    return p->precision == GBP_FP32 ? add_impl<float>(p, pose, n_new_lm, lm_init, n_new_f, f_kf, f_lm, z)
                                    : add_impl<double>(p, pose, n_new_lm, lm_init, n_new_f, f_kf, f_lm, z);
}

gbp_status gbp_set_damping_model(gbp_problem *p, const uint16_t *weights, int32_t every_k, double fallback_rise) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (weights && (every_k < 1 || every_k > 1000 || std::isnan(fallback_rise)))
        return fail(p, GBP_EINVAL, "need 1 <= every_k <= 1000 and a fallback_rise that is not NaN");
    return set_model_impl(p, weights, every_k, fallback_rise);
}

gbp_status gbp_set_damping_judges(gbp_problem *p, const int32_t *judge_of) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (!p->learned) return fail(p, GBP_ESTATE, "set a damping model first");
    std::vector<int> dj(p->np, -1);
    if (judge_of) {
        for (int i = 0; i < p->np; ++i) {
            const int j = judge_of[i];
            if (j == -1) continue;
            if (j < 0 || j >= p->np || j == i || judge_of[j] != -1)
                return fail(p, GBP_EINVAL, "judge of problem " + std::to_string(i) +
                                               " must be another problem of the batch that has no judge itself");
            dj[i] = j;
        }
        for (int i = 0; i < p->np; ++i)
            if (judge_of[i] >= 0) dj[judge_of[i]] = -2;
    }
    p->h_judge = dj;
    HIP_TRY(p, hipMemcpyAsync(p->d_judge, dj.data(), (size_t)p->np * 4, hipMemcpyHostToDevice, p->stream));
    return reset_fallback(p);
}

gbp_status gbp_reset(gbp_problem *p) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (p->grown) return fail(p, GBP_ESTATE, "gbp_reset: the problem has grown since creation");
    return p->precision == GBP_FP32 ? reset_impl<float>(p) : reset_impl<double>(p);
}

gbp_status gbp_apply_depth_model(gbp_problem *p, const int32_t *landmarks, int32_t n) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (!p->learned) return fail(p, GBP_ESTATE, "gbp_apply_depth_model: set a damping/depth model first");
    if (!p->h_pair_ab[1].empty())
        return fail(p, GBP_ESTATE, "gbp_apply_depth_model: landmarks with pairwise factors cannot be moved");
    if (n < 0 || (n > 0 && !landmarks)) return fail(p, GBP_EINVAL, "gbp_apply_depth_model: need n >= 0 and landmarks");
    std::vector<int> u2i(p->nl);
    for (int i = 0; i < p->nl; ++i) u2i[p->lm_int2user[i]] = i;
    std::vector<char> seen(p->nl, 0);
    std::vector<int> lms;
    for (int i = 0; i < n; ++i) {
        const int u = landmarks[i];
        if (u < 0 || u >= p->nl) return fail(p, GBP_EINVAL, "gbp_apply_depth_model: landmark index out of range");
        if (!seen[u]) { seen[u] = 1; lms.push_back(u2i[u]); }
    }
    return p->precision == GBP_FP32 ? depth_impl<float>(p, lms) : depth_impl<double>(p, lms);
}

gbp_status gbp_fallback_flags(gbp_problem *p, int32_t *flags) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (!flags) return fail(p, GBP_EINVAL, "flags is null");
    if (!p->learn_mem) {
        for (int i = 0; i < p->np; ++i) flags[i] = 0;
        return GBP_OK;
    }
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    HIP_TRY(p, hipMemcpy(flags, p->d_fallback, (size_t)p->np * 4, hipMemcpyDeviceToHost));
    return GBP_OK;
}

gbp_status gbp_factor_features(gbp_problem *p, const int32_t *idx, int32_t n, float *out) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (n < 0 || (n > 0 && (!idx || !out))) return fail(p, GBP_EINVAL, "need n >= 0 and device idx/out");
    return p->precision == GBP_FP32 ? features_impl<float>(p, idx, n, out) : features_impl<double>(p, idx, n, out);
}

gbp_status gbp_factor_messages(gbp_problem *p, const int32_t *idx, int32_t n, float *out) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (n < 0 || (n > 0 && (!idx || !out))) return fail(p, GBP_EINVAL, "need n >= 0 and device idx/out");
    return p->precision == GBP_FP32 ? messages_impl<float>(p, idx, n, out) : messages_impl<double>(p, idx, n, out);
}

gbp_status gbp_mlp_infer(const uint16_t *weights, const float *x, int32_t n, float *d_out, float *delta_out,
                         void *stream) {
    if (n < 0 || (n > 0 && (!weights || !x || !d_out))) {
        g_err = "gbp_mlp_infer: need n >= 0 and device weights, x and d_out";
        return GBP_EINVAL;
    }
    if ((uintptr_t)x % 16 != 0) {
        g_err = "gbp_mlp_infer: x must be 16-byte aligned (rows are read as 16-byte vectors)";
        return GBP_EINVAL;
    }
    if (n == 0) return GBP_OK;
    launch_mlp_infer(x, n, weights, d_out, delta_out, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { g_err = std::string("gbp_mlp_infer: ") + hipGetErrorString(e); return GBP_EDEVICE; }
    return GBP_OK;
}

gbp_status gbp_mlp_infer_bf16(const uint16_t *weights, const uint16_t *x_bf16, int32_t n, float *d_out,
                              float *delta_out, void *stream) {
    if (n < 0 || (n > 0 && (!weights || !x_bf16 || !d_out))) {
        g_err = "gbp_mlp_infer_bf16: need n >= 0 and device weights, x and d_out";
        return GBP_EINVAL;
    }
    if ((uintptr_t)x_bf16 % 16 != 0) {
        g_err = "gbp_mlp_infer_bf16: x_bf16 must be 16-byte aligned (rows are read as 16-byte vectors)";
        return GBP_EINVAL;
    }
    if (n == 0) return GBP_OK;
    launch_mlp_infer_bf16(x_bf16, n, weights, d_out, delta_out, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { g_err = std::string("gbp_mlp_infer_bf16: ") + hipGetErrorString(e); return GBP_EDEVICE; }
    return GBP_OK;
}

gbp_status gbp_mlp_train_workspace_bytes(int32_t max_batch, size_t *bytes) {
    if (max_batch < 1 || !bytes) { g_err = "gbp_mlp_train_workspace_bytes: need max_batch >= 1"; return GBP_EINVAL; }
    *bytes = (size_t)mlp_partial_blocks(max_batch) * (MLP_NPARAMS + 1) * 4 + 256;
    return GBP_OK;
}

gbp_status gbp_mlp_train_step(const float *x, const float *y, const float *mask, int32_t n_rows,
                              const int32_t *batch_idx, int32_t n_batch, float *theta, float *adam_m, float *adam_v,
                              uint16_t *weights_bf16, float lr, int32_t step, float *grad_out, float *loss_out,
                              void *workspace, size_t workspace_bytes, void *stream) {
    size_t need = 0;
    if (n_batch < 1 || n_rows < 0 || !x || !y || !mask || !batch_idx || !theta || !grad_out || !loss_out ||
        !workspace || step < 0 || (step > 0 && (!adam_m || !adam_v || !weights_bf16 || !(lr > 0.f)))) {
        g_err = "gbp_mlp_train_step: bad arguments";
        return GBP_EINVAL;
    }
    gbp_mlp_train_workspace_bytes(n_batch, &need);
    if (workspace_bytes < need) {
        g_err = "gbp_mlp_train_step: workspace too small (" + std::to_string(need) + " bytes needed)";
        return GBP_EINVAL;
    }
    const int nb = mlp_partial_blocks(n_batch);
    float *part_grad = (float *)workspace;
    float *part_loss = part_grad + (size_t)nb * MLP_NPARAMS;
    launch_mlp_train_step(x, y, mask, n_rows, batch_idx, n_batch, theta, adam_m, adam_v, grad_out, part_grad,
                          part_loss, loss_out, weights_bf16, lr, step, step > 0, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { g_err = std::string("gbp_mlp_train_step: ") + hipGetErrorString(e); return GBP_EDEVICE; }
    return GBP_OK;
}

gbp_status gbp_mlp_train_step_static(const float *x, const float *y, const float *mask, int32_t n_rows,
                                     const int32_t *batch_idx, int32_t n_batch, float *theta, float *adam_m,
                                     float *adam_v, uint16_t *weights_bf16, float lr, int32_t step, float *grad_out,
                                     float *loss_out, void *stream) {
    if (n_batch < 1 || n_rows < 0 || !x || !y || !mask || !batch_idx || !theta || !grad_out || !loss_out ||
        step < 0 || (step > 0 && (!adam_m || !adam_v || !weights_bf16 || !(lr > 0.f)))) {
        g_err = "gbp_mlp_train_step_static: bad arguments";
        return GBP_EINVAL;
    }
    if (n_batch > MLP_STATIC_MAX_BATCH) {
        g_err = "gbp_mlp_train_step_static: batch of " + std::to_string(n_batch) + " exceeds the fixed scratch (at most " +
                std::to_string(MLP_STATIC_MAX_BATCH) + " samples)";
        return GBP_EINVAL;
    }
    if (stream) {
        int cur = -1, sdev = -1;
        if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess ||
            cur != sdev) {
            g_err = "gbp_mlp_train_step_static: the stream must belong to the current device";
            return GBP_EINVAL;
        }
    }
    float *scr = nullptr;
    size_t floats = 0;
    hipError_t e = mlp_static_scratch(&scr, &floats);
    if (e != hipSuccess) {
        g_err = std::string("gbp_mlp_train_step_static: scratch address: ") + hipGetErrorString(e);
        return GBP_EDEVICE;
    }
    const int nb = mlp_partial_blocks(n_batch);
    if ((size_t)nb * (MLP_NPARAMS + 1) > floats) {
        g_err = "gbp_mlp_train_step_static: scratch too small";
        return GBP_EINVAL;
    }
    // every partial the reduction reads is written by this call's first
    // kernel: nothing left by an earlier call needs clearing
    float *part_grad = scr;
    float *part_loss = part_grad + (size_t)nb * MLP_NPARAMS;
    launch_mlp_train_step(x, y, mask, n_rows, batch_idx, n_batch, theta, adam_m, adam_v, grad_out, part_grad,
                          part_loss, loss_out, weights_bf16, lr, step, step > 0, (hipStream_t)stream);
    e = hipGetLastError();
    if (e != hipSuccess) { g_err = std::string("gbp_mlp_train_step_static: ") + hipGetErrorString(e); return GBP_EDEVICE; }
    return GBP_OK;
}

gbp_status gbp_phase_times(gbp_problem *p, int32_t n, double damping, double huber_k, double *ms_out) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (n < 1 || !ms_out || !(damping >= 0.0 && damping < 1.0) || !std::isfinite(huber_k))
        return fail(p, GBP_EINVAL, "need n >= 1, ms_out, 0 <= damping < 1 and finite huber_k");
    return p->precision == GBP_FP32 ? phase_times_impl<float>(p, n, damping, huber_k, ms_out)
                                    : phase_times_impl<double>(p, n, damping, huber_k, ms_out);
}

gbp_status gbp_counters(gbp_problem *p, int64_t *relinearisations) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    const int *qc = p->precision == GBP_FP32 ? p->df.relin_qcount : p->dd.relin_qcount;
    const int nb = p->precision == GBP_FP32 ? p->df.n_rblk : p->dd.n_rblk;
    launch_relin_total(qc, nb, p->d_total, p->stream);
    HIP_TRY(p, hipGetLastError());
    unsigned long long v = 0;
    HIP_TRY(p, hipMemcpyAsync(&v, p->d_total, 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    if (relinearisations) *relinearisations = (int64_t)v;
    return GBP_OK;
}

gbp_status gbp_autotune(gbp_problem *p, int32_t n_iters, const char *cache_path, int32_t *chosen) {
    gbp_status st = check_live(p);
    if (st != GBP_OK) return st;
    if (n_iters < 1) return fail(p, GBP_EINVAL, "need n_iters >= 1");
    return p->precision == GBP_FP32 ? autotune_impl<float>(p, n_iters, cache_path, chosen)
                                    : autotune_impl<double>(p, n_iters, cache_path, chosen);
}

gbp_status gbp_sizes(const gbp_problem *p, int32_t *nk, int32_t *nl, int32_t *nf, int32_t *np, int32_t *t) {
    if (!p) return GBP_EINVAL;
    if (nk) *nk = p->nk;
    if (nl) *nl = p->nl;
    if (nf) *nf = p->nf;
    if (np) *np = p->np;
    if (t) *t = p->t;
    return GBP_OK;
}

const char *gbp_last_error(const gbp_problem *p) {
    if (!p) return g_err.empty() ? "null problem" : g_err.c_str();
    return p->err.c_str();
}

void gbp_destroy(gbp_problem *p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    destroy_graphs(p);
    if (p->d_log) (void)hipFree(p->d_log);
    if (p->learn_mem) (void)hipFree(p->learn_mem);
    if (p->pair_mem) (void)hipFree(p->pair_mem);
    if (p->own_ws && p->ws) (void)hipFree(p->ws);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

}  // extern "C"
