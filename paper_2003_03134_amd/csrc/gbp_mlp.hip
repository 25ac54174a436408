// Learned damping / depth network: 16 -> 64 (ReLU) -> 64 (ReLU) -> 2, BF16
// weights and activations, FP32 accumulation.
//
// Heads: damping d = 0.9 sigmoid(o0) (per factor, used by the factor phase
// in place of the constant damping), log-depth correction
// delta = 2.5 tanh(o1). Parameter blob (5378 values, BF16 bits for inference,
// FP32 for training): W1[64][16], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
//
// Inference (k_mlp_infer) is the only dense contraction on the path: layers 1
// and 2 run on the matrix cores with v_mfma_f32_32x32x16_bf16 (32 rows per
// tile, computed transposed so activations stay in registers); the 64 -> 2
// head is a per-lane dot product.
// Training (k_mlp_train_block, k_mlp_reduce, k_adam) evaluates the same
// BF16-rounded forward pass per sample and back-propagates in FP32; block
// partial gradients are summed in a fixed order, so training is
// deterministic.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "gbp_mlp.h"

namespace gbp {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int O_W1 = 0, O_B1 = O_W1 + MLP_H * MLP_IN, O_W2 = O_B1 + MLP_H, O_B2 = O_W2 + MLP_H * MLP_H,
              O_W3 = O_B2 + MLP_H, O_B3 = O_W3 + MLP_OUT * MLP_H;
static_assert(O_B3 + MLP_OUT == MLP_NPARAMS, "parameter layout");

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ void heads(float o0, float o1, float &d, float &delta) {
    d = MLP_DMAX / (1.0f + expf(-o0));
    delta = MLP_CDELTA * tanhf(o1);
}

// --------------------------------------------------------------------------
// inference: persistent waves over tiles of 32 rows
// --------------------------------------------------------------------------
//
// Each layer is computed transposed, H^T = W X^T, with
// v_mfma_f32_32x32x16_bf16: the weights are the A operand (lane l: row l % 32,
// k slots 8 (l / 32) + 0..7) and stay in registers for the kernel's life; the
// activations of 32 rows are the B operand (lane l: column = row l % 32 of
// the tile, same k slots). The accumulator of a 32x32 tile holds, in lane l
// and entry q, hidden unit 8 (q / 4) + 4 (l / 32) + q % 4 of row l % 32: the
// 8 entries 8 c .. 8 c + 7 of one lane are exactly the 8 k slots the next
// layer's B operand needs from that lane, once that layer's A operand (the
// weight columns) is taken in the same hidden-unit order (hid() below). So
// activations never leave registers and need no transpose through LDS. The
// 64 -> 2 head is a per-lane dot product over the lane's 32 hidden units plus
// one exchange between the two lane halves.

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ __bf16 bf_bits(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// hidden unit held by k slot j (0..7) of k-step kk (0..3) in lane half hh,
// i.e. accumulator entry 8 (kk % 2) + j of hidden block kk / 2
__device__ __forceinline__ int hid(int kk, int hh, int j) {
    return 32 * (kk >> 1) + 8 * (2 * (kk & 1) + (j >> 2)) + 4 * hh + (j & 3);
}

constexpr int INFER_WAVES_MAX = 2048;  // 256 CUs x 8 waves
constexpr int INFER_AHEAD = 4;         // tiles whose features a wave has in flight

// One tile's features in the layer-1 B operand layout (row tile * 32 + r,
// features 8 hh .. 8 hh + 7), loaded raw so that the load stays in flight
// until the tile is computed, then converted to BF16 (round to nearest even)
// at use. Rows past n read as zeros without a load.
struct RawF32 { float4 u, v; };
struct RawBF16 { uint4 u; };

__device__ __forceinline__ RawF32 load_raw(const float *__restrict__ X, int n, int tile, int r, int hh) {
    const int row = tile * 32 + r;
    RawF32 x{make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f)};
    if (row < n) {
        const float4 *xp = reinterpret_cast<const float4 *>(X + (size_t)row * MLP_IN + 8 * hh);
        x.u = xp[0];
        x.v = xp[1];
    }
    return x;
}

// the same from features already stored as BF16 bits
__device__ __forceinline__ RawBF16 load_raw(const uint16_t *__restrict__ X, int n, int tile, int r, int hh) {
    const int row = tile * 32 + r;
    RawBF16 x{make_uint4(0u, 0u, 0u, 0u)};
    if (row < n) x.u = *reinterpret_cast<const uint4 *>(X + (size_t)row * MLP_IN + 8 * hh);
    return x;
}

__device__ __forceinline__ bf16x8_t to_operand(const RawF32 &r) {
    bf16x8_t x;
    x[0] = (__bf16)r.u.x; x[1] = (__bf16)r.u.y; x[2] = (__bf16)r.u.z; x[3] = (__bf16)r.u.w;
    x[4] = (__bf16)r.v.x; x[5] = (__bf16)r.v.y; x[6] = (__bf16)r.v.z; x[7] = (__bf16)r.v.w;
    return x;
}
__device__ __forceinline__ bf16x8_t to_operand(const RawBF16 &r) { return __builtin_bit_cast(bf16x8_t, r.u); }

// relu(acc + bias) of one 32x32 accumulator, rounded to BF16, as two B
// operands
__device__ __forceinline__ void relu_operands(const f32x16_t &acc, const f32x16_t &bias, bf16x8_t &lo,
                                              bf16x8_t &hi) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        lo[q] = (__bf16)fmaxf(acc[q] + bias[q], 0.f);
        hi[q] = (__bf16)fmaxf(acc[8 + q] + bias[8 + q], 0.f);
    }
}

template <typename TX>
__global__ __launch_bounds__(256) void k_mlp_infer(const TX *__restrict__ X, int n,
                                                   const uint16_t *__restrict__ P, float *__restrict__ out_d,
                                                   float *__restrict__ out_delta) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hh = lane >> 5, r = lane & 31;
    // weights as A operands; the head's two output rows padded to 32 with
    // zeros so that it runs on the matrix cores as well
    bf16x8_t w1[2], w2[2][4], w3[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 8; ++j) w1[mt][j] = bf_bits(P[O_W1 + (32 * mt + r) * MLP_IN + 8 * hh + j]);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int j = 0; j < 8; ++j) w2[mt][kk][j] = bf_bits(P[O_W2 + (32 * mt + r) * MLP_H + hid(kk, hh, j)]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int j = 0; j < 8; ++j) w3[kk][j] = bf_bits(r < MLP_OUT ? P[O_W3 + r * MLP_H + hid(kk, hh, j)] : 0);
    // biases (LDS), added to the finished sums as in the reference order
    // (sum first, then bias): entry q of hidden block mt is unit
    // 32 mt + 8 (q / 4) + 4 hh + q % 4, four consecutive units per float4
    __shared__ float4 sb[2][MLP_H / 4];
    if (tid < MLP_H) reinterpret_cast<float *>(sb[0])[tid] = bf2f(P[O_B1 + tid]);
    else if (tid < 2 * MLP_H) reinterpret_cast<float *>(sb[1])[tid - MLP_H] = bf2f(P[O_B2 + tid - MLP_H]);
    const float b30 = bf2f(P[O_B3]), b31 = bf2f(P[O_B3 + 1]);
    __syncthreads();
    auto bias = [&](int layer, int mt) {
        f32x16_t acc;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const float4 v = sb[layer][8 * mt + 2 * a + hh];
            acc[4 * a] = v.x; acc[4 * a + 1] = v.y; acc[4 * a + 2] = v.z; acc[4 * a + 3] = v.w;
        }
        return acc;
    };

    const int ntiles = (n + 31) / 32;
    const int stride = gridDim.x * (blockDim.x / 64);
    const int first = blockIdx.x * (blockDim.x / 64) + wave;
    // the features of the wave's next INFER_AHEAD tiles are in flight while
    // one computes (a ring of registers, rotated by unrolling; rows past n
    // read as zeros without a load)
    decltype(load_raw(X, n, 0, r, hh)) ring[INFER_AHEAD];
#pragma unroll
    for (int u = 0; u < INFER_AHEAD; ++u) ring[u] = load_raw(X, n, first + u * stride, r, hh);
    for (int t0 = first; t0 < ntiles; t0 += INFER_AHEAD * stride)
#pragma unroll
    for (int u = 0; u < INFER_AHEAD; ++u) {
        const int tile = t0 + u * stride;
        if (tile >= ntiles) break;
        const bf16x8_t x = to_operand(ring[u]);
        ring[u] = load_raw(X, n, tile + INFER_AHEAD * stride, r, hh);
        // layer 1: H1^T = relu(W1 X^T + b1)
        bf16x8_t h1[4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const f32x16_t zero = {0};
            const f32x16_t acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[mt], x, zero, 0, 0, 0);
            relu_operands(acc, bias(0, mt), h1[2 * mt], h1[2 * mt + 1]);
        }
        // layer 2: H2^T = relu(W2 H1^T + b2)
        bf16x8_t h2[4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            f32x16_t acc = {0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2[mt][kk], h1[kk], acc, 0, 0, 0);
            relu_operands(acc, bias(1, mt), h2[2 * mt], h2[2 * mt + 1]);
        }
        // head: O^T = W3 H2^T (rows 0 and 1 land in lanes 0..31), then b3
        f32x16_t o = {0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w3[kk], h2[kk], o, 0, 0, 0);
        const int row = tile * 32 + r;
        if (hh == 0 && row < n) {
            float d, delta;
            heads(o[0] + b30, o[1] + b31, d, delta);
            out_d[row] = d;
            if (out_delta) out_delta[row] = delta;
        }
    }
}

// --------------------------------------------------------------------------
// training
// --------------------------------------------------------------------------

constexpr int SB = 32;  // samples per training workgroup

// Per workgroup: forward (BF16-rounded weights, inputs and hidden
// activations, FP32 sums) and back-propagation for SB samples, then the
// workgroup's partial gradient of every parameter (sum over its samples in
// sample order) and its partial loss. Loss per sample: m0 (d - y0)^2 +
// m1 (delta - y1)^2, divided by the batch size. Activations live in LDS; the
// ReLU derivative is read from the stored activation (positive iff the
// pre-activation is positive).
__global__ __launch_bounds__(256) void k_mlp_train_block(const float *__restrict__ X, const float *__restrict__ Y,
                                                         const float *__restrict__ M, int n_rows,
                                                         const int *__restrict__ idx, int n_batch, const float *__restrict__ theta,
                                                         float *__restrict__ part_grad, float *__restrict__ part_loss) {
    __shared__ float w[MLP_NPARAMS];
    // rows padded by one word: the lanes of a wave read one column of 8
    // samples' rows, which unpadded rows of 64 floats would put on one LDS
    // bank
    __shared__ float sx[SB][MLP_IN + 1], sh1[SB][MLP_H + 1], sh2[SB][MLP_H + 1], sd1[SB][MLP_H + 1],
        sd2[SB][MLP_H + 1], sdo[SB][2];
    __shared__ float sl[SB], so[SB][2];
    const int tid = threadIdx.x;
    for (int i = tid; i < MLP_NPARAMS; i += 256) w[i] = bfround(theta[i]);
    // 8 lanes per sample: lane r of sample s owns hidden units 8 r .. 8 r + 7
    // of every layer and evaluates each of their dot products in full, in
    // index order (the same sums as one lane per sample)
    static_assert(SB * 8 == 256, "8 lanes per sample");
    const int s = tid >> 3, r = tid & 7, u0 = 8 * r;
    // samples past the batch or with an index outside [0, n_rows) count as
    // zero-weight samples
    const int g = blockIdx.x * SB + s;
    const int src0 = g < n_batch ? idx[g] : -1;
    const bool live = src0 >= 0 && src0 < n_rows;
    const int src = live ? src0 : 0;
#pragma unroll
    for (int j = 2 * r; j < 2 * r + 2; ++j) sx[s][j] = live ? bfround(X[(size_t)src * MLP_IN + j]) : 0.f;
    __syncthreads();
    for (int i = u0; i < u0 + 8; ++i) {
        float a = w[O_B1 + i];
#pragma unroll
        for (int j = 0; j < MLP_IN; ++j) a += w[O_W1 + i * MLP_IN + j] * sx[s][j];
        sh1[s][i] = bfround(a > 0.f ? a : 0.f);
    }
    __syncthreads();
    for (int i = u0; i < u0 + 8; ++i) {
        float a = w[O_B2 + i];
        for (int j = 0; j < MLP_H; ++j) a += w[O_W2 + i * MLP_H + j] * sh1[s][j];
        sh2[s][i] = bfround(a > 0.f ? a : 0.f);
    }
    __syncthreads();
    if (r < 2) {
        float o = w[O_B3 + r];
        for (int j = 0; j < MLP_H; ++j) o += w[O_W3 + r * MLP_H + j] * sh2[s][j];
        so[s][r] = o;
    }
    __syncthreads();
    if (r == 0) {
        float d, delta;
        heads(so[s][0], so[s][1], d, delta);
        float m0 = 0.f, m1 = 0.f, y0 = 0.f, y1 = 0.f;
        if (live) {
            m0 = M[2 * (size_t)src]; m1 = M[2 * (size_t)src + 1];
            y0 = Y[2 * (size_t)src]; y1 = Y[2 * (size_t)src + 1];
        }
        const float r0 = d - y0, r1 = delta - y1;
        sl[s] = (m0 * r0 * r0 + m1 * r1 * r1) / (float)n_batch;
        const float sig = d / MLP_DMAX, th = delta / MLP_CDELTA;
        sdo[s][0] = 2.f * m0 * r0 / (float)n_batch * MLP_DMAX * sig * (1.f - sig);
        sdo[s][1] = 2.f * m1 * r1 / (float)n_batch * MLP_CDELTA * (1.f - th * th);
    }
    __syncthreads();
    for (int i = u0; i < u0 + 8; ++i) {
        const float dh = sdo[s][0] * w[O_W3 + i] + sdo[s][1] * w[O_W3 + MLP_H + i];
        sd2[s][i] = sh2[s][i] > 0.f ? dh : 0.f;
    }
    __syncthreads();
    for (int jj = u0; jj < u0 + 8; ++jj) {
        float dh = 0.f;
        for (int i = 0; i < MLP_H; ++i) dh += sd2[s][i] * w[O_W2 + i * MLP_H + jj];
        sd1[s][jj] = sh1[s][jj] > 0.f ? dh : 0.f;
    }
    __syncthreads();
    float *pg = part_grad + (size_t)blockIdx.x * MLP_NPARAMS;
    for (int e = tid; e < MLP_NPARAMS; e += 256) {
        float a = 0.f;
        if (e < O_B1) {
            const int i = e / MLP_IN, j = e % MLP_IN;
            for (int q = 0; q < SB; ++q) a += sd1[q][i] * sx[q][j];
        } else if (e < O_W2) {
            const int i = e - O_B1;
            for (int q = 0; q < SB; ++q) a += sd1[q][i];
        } else if (e < O_B2) {
            const int i = (e - O_W2) / MLP_H, j = (e - O_W2) % MLP_H;
            for (int q = 0; q < SB; ++q) a += sd2[q][i] * sh1[q][j];
        } else if (e < O_W3) {
            const int i = e - O_B2;
            for (int q = 0; q < SB; ++q) a += sd2[q][i];
        } else if (e < O_B3) {
            const int i = (e - O_W3) / MLP_H, j = (e - O_W3) % MLP_H;
            for (int q = 0; q < SB; ++q) a += sdo[q][i] * sh2[q][j];
        } else {
            const int i = e - O_B3;
            for (int q = 0; q < SB; ++q) a += sdo[q][i];
        }
        pg[e] = a;
    }
    if (tid == 0) {
        float a = 0.f;
        for (int q = 0; q < SB; ++q) a += sl[q];
        part_loss[blockIdx.x] = a;
    }
}

// Sum of the workgroups' partial gradients: each workgroup takes 64
// parameters, its 4 waves sum consecutive quarters of the partials in
// workgroup order and the quarters are added in order (a fixed order:
// deterministic). The last workgroup sums the partial losses in order.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ part_grad,
                                                    const float *__restrict__ part_loss, int nb,
                                                    float *__restrict__ grad, float *__restrict__ loss) {
    const int nchunk = (MLP_NPARAMS + 63) / 64;
    if ((int)blockIdx.x == nchunk) {
        if (threadIdx.x == 0) {
            float a = 0.f;
            for (int b = 0; b < nb; ++b) a += part_loss[b];
            loss[0] = a;
        }
        return;
    }
    __shared__ float q[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int b0 = (nb * wave) / 4, b1 = (nb * (wave + 1)) / 4;
    float a = 0.f;
    if (e < MLP_NPARAMS)
        for (int b = b0; b < b1; ++b) a += part_grad[(size_t)b * MLP_NPARAMS + e];
    q[wave][lane] = a;
    __syncthreads();
    if (threadIdx.x < 64 && e < MLP_NPARAMS) grad[e] = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
}

// Adam with bias correction on FP32 master weights; writes the BF16 copy
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ theta, float *__restrict__ m1,
                                              float *__restrict__ m2, const float *__restrict__ g, float lr,
                                              float beta1, float beta2, float eps, int step,
                                              uint16_t *__restrict__ bf16) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MLP_NPARAMS) return;
    const float ge = g[e];
    const float a = beta1 * m1[e] + (1.f - beta1) * ge;
    const float b = beta2 * m2[e] + (1.f - beta2) * ge * ge;
    m1[e] = a;
    m2[e] = b;
    const float ah = a / (1.f - powf(beta1, (float)step)), bh = b / (1.f - powf(beta2, (float)step));
    const float t = theta[e] - lr * ah / (sqrtf(bh) + eps);
    theta[e] = t;
    bf16[e] = f2bf(t);
}

__global__ void k_to_bf16(const float *__restrict__ theta, uint16_t *__restrict__ out, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = f2bf(theta[e]);
}

void launch_mlp_infer(const float *X, int n, const uint16_t *P, float *out_d, float *out_delta, hipStream_t s) {
    if (n > 0) {
        const int waves = std::min((n + 31) / 32, INFER_WAVES_MAX);
        hipLaunchKernelGGL(k_mlp_infer<float>, dim3((waves + 3) / 4), dim3(256), 0, s, X, n, P, out_d, out_delta);
    }
}
void launch_mlp_infer_bf16(const uint16_t *X, int n, const uint16_t *P, float *out_d, float *out_delta,
                           hipStream_t s) {
    if (n > 0) {
        const int waves = std::min((n + 31) / 32, INFER_WAVES_MAX);
        hipLaunchKernelGGL(k_mlp_infer<uint16_t>, dim3((waves + 3) / 4), dim3(256), 0, s, X, n, P, out_d, out_delta);
    }
}

void launch_mlp_train_step(const float *X, const float *Y, const float *M, int n_rows, const int *idx, int n_batch,
                           float *theta, float *m1, float *m2, float *grad, float *part_grad, float *part_loss,
                           float *loss, uint16_t *bf16, float lr, int step, bool update, hipStream_t s) {
    const int nb = (n_batch + SB - 1) / SB;
    hipLaunchKernelGGL(k_mlp_train_block, dim3(nb), dim3(256), 0, s, X, Y, M, n_rows, idx, n_batch, (const float *)theta,
                       part_grad, part_loss);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAMS + 63) / 64 + 1), dim3(256), 0, s, (const float *)part_grad,
                       (const float *)part_loss, nb, grad, loss);
    if (update)
        hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, s, theta, m1, m2,
                           (const float *)grad, lr, 0.9f, 0.999f, 1e-8f, step, bf16);
}

void launch_to_bf16(const float *theta, uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, s, theta, out, MLP_NPARAMS);
}

int mlp_partial_blocks(int n_batch) { return (n_batch + SB - 1) / SB; }

// Fixed device scratch of the allocation-free training step: the partial
// gradients and partial losses of up to MLP_STATIC_MAX_BATCH samples. Each
// GPU the library runs on holds one copy for the life of the process. In host
// code the array's name is not a device address: its address on a device is
// looked up once per device (with that device current) and kept.
constexpr size_t MLP_SCRATCH_FLOATS =
    (size_t)((MLP_STATIC_MAX_BATCH + SB - 1) / SB) * (MLP_NPARAMS + 1);
static __device__ __align__(256) float scratch[MLP_SCRATCH_FLOATS];

static std::mutex g_scratch_mu;
static float *g_scratch_ptr[MLP_MAX_DEVICES];

hipError_t mlp_static_scratch(float **ptr, size_t *floats) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MLP_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (float *)p;
    }
    *ptr = g_scratch_ptr[dev];
    *floats = MLP_SCRATCH_FLOATS;
    return hipSuccess;
}

}  // namespace gbp
