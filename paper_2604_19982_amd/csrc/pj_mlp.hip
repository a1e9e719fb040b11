// pj_mlp.hip -- the LoD-skip network: 16 -> 64 -> 64 -> 4, ReLU, softmax.
//
// Weights are used in BF16 (rounded from FP32 master copies, round to
// nearest even) and every product is accumulated in FP32.  Training runs
// three kernels per batch: per-sample forward + backpropagation to the
// pre-activations (one thread per sample, weights staged in LDS), weight
// gradients as batch reductions (one thread per parameter, no atomics, so the
// result does not depend on scheduling), and Adam on the FP32 masters.
// Parameter layout: W1[16][64] b1[64] W2[64][64] b2[64] W3[64][4] b3[4].
#include "pj_internal.h"

namespace pj {

constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_IN * MLP_H;
constexpr int OFF_W2 = OFF_B1 + MLP_H;
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_H * MLP_OUT;
static_assert(OFF_B3 + MLP_OUT == MLP_NPARAM, "layout");

__device__ __forceinline__ float bf16_round(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// stage the BF16-rounded parameters in LDS
__device__ __forceinline__ void stage(const float *params, float *w)
{
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) w[i] = bf16_round(params[i]);
    __syncthreads();
}

// forward of one sample; keeps z1, z2 (pre-activations) and logits
__device__ __forceinline__ void forward1(const float *w, const float *x, float *z1, float *z2, float *lg)
{
    for (int j = 0; j < MLP_H; ++j) {
        float a = w[OFF_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) a = fmaf(x[i], w[OFF_W1 + i * MLP_H + j], a);
        z1[j] = a;
    }
    for (int j = 0; j < MLP_H; ++j) {
        float a = w[OFF_B2 + j];
        for (int i = 0; i < MLP_H; ++i) a = fmaf(fmaxf(z1[i], 0.0f), w[OFF_W2 + i * MLP_H + j], a);
        z2[j] = a;
    }
    for (int j = 0; j < MLP_OUT; ++j) {
        float a = w[OFF_B3 + j];
        for (int i = 0; i < MLP_H; ++i) a = fmaf(fmaxf(z2[i], 0.0f), w[OFF_W3 + i * MLP_OUT + j], a);
        lg[j] = a;
    }
}

// per sample: forward, loss, and gradients w.r.t. z3 (logits), z2, z1
__global__ __launch_bounds__(128) void k_mlp_fwd_bwd(const float *params, const float *x, const int32_t *y, int n,
                                                     float inv_batch, float *logits, float *loss_per, float *a1,
                                                     float *a2, float *g1, float *g2, float *g3)
{
    __shared__ float w[MLP_NPARAM];
    stage(params, w);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float xs[MLP_IN], z1[MLP_H], z2[MLP_H], lg[MLP_OUT];
    for (int i = 0; i < MLP_IN; ++i) xs[i] = x[(int64_t)b * MLP_IN + i];
    forward1(w, xs, z1, z2, lg);
    for (int j = 0; j < MLP_OUT; ++j) logits[(int64_t)b * MLP_OUT + j] = lg[j];
    if (!y) return;
    float m = fmaxf(fmaxf(lg[0], lg[1]), fmaxf(lg[2], lg[3]));
    float e[MLP_OUT], se = 0.0f;
    for (int j = 0; j < MLP_OUT; ++j) {
        e[j] = expf(lg[j] - m);
        se += e[j];
    }
    const int lab = y[b];
    loss_per[b] = -(lg[lab] - m - logf(se));
    float d3[MLP_OUT];
    for (int j = 0; j < MLP_OUT; ++j) d3[j] = (e[j] / se - (j == lab ? 1.0f : 0.0f)) * inv_batch;
    float d2[MLP_H];
    for (int i = 0; i < MLP_H; ++i) {
        float a = 0.0f;
        for (int j = 0; j < MLP_OUT; ++j) a = fmaf(d3[j], w[OFF_W3 + i * MLP_OUT + j], a);
        d2[i] = z2[i] > 0.0f ? a : 0.0f;
    }
    for (int i = 0; i < MLP_H; ++i) {
        float a = 0.0f;
        for (int j = 0; j < MLP_H; ++j) a = fmaf(d2[j], w[OFF_W2 + i * MLP_H + j], a);
        g1[(int64_t)b * MLP_H + i] = z1[i] > 0.0f ? a : 0.0f;
        a1[(int64_t)b * MLP_H + i] = fmaxf(z1[i], 0.0f);
        a2[(int64_t)b * MLP_H + i] = fmaxf(z2[i], 0.0f);
        g2[(int64_t)b * MLP_H + i] = d2[i];
    }
    for (int j = 0; j < MLP_OUT; ++j) g3[(int64_t)b * MLP_OUT + j] = d3[j];
}

// one thread per parameter: sum over the batch of (input activation x
// output gradient), or of the output gradient for a bias
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float *x, const float *a1, const float *a2,
                                                   const float *g1, const float *g2, const float *g3, int n,
                                                   float *grads)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float *in = nullptr;
    const float *g = nullptr;
    int nin = 0, nout = 0, i = 0, j = 0;
    if (p < OFF_B1) {
        in = x; g = g1; nin = MLP_IN; nout = MLP_H; i = (p - OFF_W1) / MLP_H; j = (p - OFF_W1) % MLP_H;
    } else if (p < OFF_W2) {
        g = g1; nout = MLP_H; j = p - OFF_B1;
    } else if (p < OFF_B2) {
        in = a1; g = g2; nin = MLP_H; nout = MLP_H; i = (p - OFF_W2) / MLP_H; j = (p - OFF_W2) % MLP_H;
    } else if (p < OFF_W3) {
        g = g2; nout = MLP_H; j = p - OFF_B2;
    } else if (p < OFF_B3) {
        in = a2; g = g3; nin = MLP_H; nout = MLP_OUT; i = (p - OFF_W3) / MLP_OUT; j = (p - OFF_W3) % MLP_OUT;
    } else {
        g = g3; nout = MLP_OUT; j = p - OFF_B3;
    }
    float acc = 0.0f;
    for (int b = 0; b < n; ++b) {
        const float gv = g[(int64_t)b * nout + j];
        acc = in ? fmaf(in[(int64_t)b * nin + i], gv, acc) : acc + gv;
    }
    grads[p] = acc;
}

hipError_t launch_mlp_fwd_bwd(const float *params, const float *x, const int32_t *y, int n, float *logits,
                              float *loss_per, float *grads, float *scratch, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    float *a1 = scratch, *a2 = a1 + (int64_t)n * MLP_H, *g1 = a2 + (int64_t)n * MLP_H, *g2 = g1 + (int64_t)n * MLP_H,
          *g3 = g2 + (int64_t)n * MLP_H;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((n + 127) / 128), dim3(128), 0, st, params, x, y, n, 1.0f / n, logits,
                       loss_per, a1, a2, g1, g2, g3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !y) return e;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, x, a1, a2, g1, g2, g3, n, grads);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *params, float *m, float *v, const float *grads, float lr,
                                                  float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float g = grads[p];
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

hipError_t launch_mlp_adam(float *params, float *m, float *v, const float *grads, int step, float lr, float b1,
                           float b2, float eps, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, params, m, v, grads, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

// Inference.  The 16 features of a candidate pair, computed as the logged
// ones are (FP64, rounded once): log1p of its lower bound, of tau and of its
// upper bound, where tau sits between the bounds, and per LoD l log1p of the
// two objects' max hd and max ph summed and log2(n_r * n_s) / 16.  The first
// LoD to refine is chosen to minimise the expected facet-pair work
// C(s) = c_s + sum_{l>s} c_l P(y >= l), c_l = sqrt(n_r n_s) at LoD l (a pair
// is assumed to resolve at s when its label is <= s).
// Feature q of a candidate (computed by lane q of its wave): the same
// expressions as the logged features, in FP64 rounded once.
__device__ __forceinline__ float pair_feature(const FeatSide &R, const FeatSide &S, const StartIn &c, int q)
{
    if (q == 0) return (float)log1p(fmax(c.lb, 0.0));
    if (q == 1) return (float)log1p(c.tau);
    if (q == 2) return (float)log1p(fmax(c.ub, 0.0));
    if (q == 3) return (float)fmin(1.0, fmax(0.0, (c.tau - c.lb) / fmax(c.ub - c.lb, 1e-9)));
    const int l = (q - 4) / 3, m = (q - 4) % 3;
    const int lr = min(l, R.L - 1);
    const float2 a = R.lodmax[(int64_t)c.r * R.L + lr], b = S.lodmax[(int64_t)c.s * S.L + lr];
    if (m == 0) return (float)log1p((double)a.x + b.x);
    if (m == 1) return (float)log1p((double)a.y + b.y);
    const double nr = R.tcnt[(int64_t)c.r * R.L + lr], ns = S.tcnt[(int64_t)c.s * S.L + lr];
    return (float)(log2(fmax(nr * ns, 1.0)) / 16.0);
}

// One wave per candidate (a workgroup's four waves stride over them, the
// BF16 weights staged once per workgroup): lane q < 16 computes feature q,
// lane j of 64 hidden unit j of each layer (its inputs broadcast from LDS,
// summed in the same order as the training kernels), lanes 0..3 the logits,
// lane 0 the choice.
__global__ __launch_bounds__(256) void k_mlp_start(const float *params, const float *norm, FeatSide R, FeatSide S,
                                                   const StartIn *in, int n, int32_t *start)
{
    __shared__ float w[MLP_NPARAM];
    __shared__ float act[4][MLP_H + MLP_IN];
    stage(params, w);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float *xs = act[wv] + MLP_H;  // features, then the hidden activations in act[wv][0..63]
    float *hs = act[wv];
    // every wave runs the same iterations (the barriers are workgroup-wide);
    // a wave past the end computes on a copy of the last candidate and stores
    // nothing
    for (int b0 = blockIdx.x * 4; b0 < n; b0 += gridDim.x * 4) {
        const int b = b0 + wv;
        const StartIn c = in[min(b, n - 1)];
        if (lane < MLP_IN) xs[lane] = (pair_feature(R, S, c, lane) - norm[lane]) / norm[MLP_IN + lane];
        float cost = 0.0f;  // lane l < 4: the work of LoD l
        if (lane < MLP_OUT) {
            const int lr = min(lane, R.L - 1);
            cost = (float)sqrt((double)R.tcnt[(int64_t)c.r * R.L + lr] * (double)S.tcnt[(int64_t)c.s * S.L + lr]);
        }
        __syncthreads();
        float a = w[OFF_B1 + lane];
        for (int i = 0; i < MLP_IN; ++i) a = fmaf(xs[i], w[OFF_W1 + i * MLP_H + lane], a);
        __syncthreads();
        hs[lane] = fmaxf(a, 0.0f);
        __syncthreads();
        a = w[OFF_B2 + lane];
        for (int i = 0; i < MLP_H; ++i) a = fmaf(hs[i], w[OFF_W2 + i * MLP_H + lane], a);
        __syncthreads();
        hs[lane] = fmaxf(a, 0.0f);
        __syncthreads();
        float lg = 0.0f;
        if (lane < MLP_OUT) {
            lg = w[OFF_B3 + lane];
            for (int i = 0; i < MLP_H; ++i) lg = fmaf(hs[i], w[OFF_W3 + i * MLP_OUT + lane], lg);
        }
        // logits and costs to lane 0
        float L4[MLP_OUT], C4[MLP_OUT];
        for (int j = 0; j < MLP_OUT; ++j) {
            L4[j] = __shfl(lg, j, 64);
            C4[j] = __shfl(cost, j, 64);
        }
        if (lane == 0 && b < n) {
            const float m = fmaxf(fmaxf(L4[0], L4[1]), fmaxf(L4[2], L4[3]));
            float e[MLP_OUT], se = 0.0f;
            for (int j = 0; j < MLP_OUT; ++j) {
                e[j] = expf(L4[j] - m);
                se += e[j];
            }
            float tail[MLP_OUT + 1];  // tail[l] = P(y >= l)
            tail[MLP_OUT] = 0.0f;
            for (int j = MLP_OUT - 1; j >= 0; --j) tail[j] = tail[j + 1] + e[j] / se;
            const int nl = min(R.L, MLP_OUT);
            int best = 0;
            float bc = 3.4e38f;
            for (int s0 = 0; s0 < nl; ++s0) {
                float cc = C4[s0];
                for (int l = s0 + 1; l < nl; ++l) cc += C4[l] * tail[l];
                if (cc < bc) {
                    bc = cc;
                    best = s0;
                }
            }
            start[b] = best;
        }
        __syncthreads();
    }
}

hipError_t launch_mlp_start(const float *params, const float *norm, FeatSide R, FeatSide S, const StartIn *in, int n,
                            int32_t *start, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(((int64_t)n + 3) / 4, 4096);
    hipLaunchKernelGGL(k_mlp_start, dim3(blocks), dim3(256), 0, st, params, norm, R, S, in, n, start);
    return hipGetLastError();
}

}  // namespace pj
