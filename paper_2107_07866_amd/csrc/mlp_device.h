// Surrogate networks of the learned form: layout and the per-lane float32
// evaluation shared by the training kernels and the run-away fix-up kernels.
//
// Network: t = (x - c) s;  h1 = silu(W1 t + b1);  h2 = silu(W2 h1 + b2);
// y = w3 . h2 + b3;  g = y_shift + y_scale y;  g' = y_scale s dy/dt.
// Parameter vector: W1[H], b1[H], W2[H][H] (row = output unit), b2[H], w3[H], b3.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace misa {

constexpr int MLP_H = 32;
constexpr int MLP_NP = MLP_H * (MLP_H + 4) + 1;
constexpr int OFF_W1 = 0, OFF_B1 = MLP_H, OFF_W2 = 2 * MLP_H, OFF_B2 = 2 * MLP_H + MLP_H * MLP_H,
              OFF_W3 = 3 * MLP_H + MLP_H * MLP_H, OFF_B3 = 4 * MLP_H + MLP_H * MLP_H;

// One network as the kernels read it.
struct MlpNet {
    const float *p = nullptr;  // MLP_NP weights (float32 holding bfloat16 values on a lattice)
    float c = 0.f, s = 0.f;    // t = (x - c) s
    float y_shift = 0.f, y_scale = 0.f;
    float x_lo = 0.f, x_hi = -1.f;  // served range (empty: always the table)
};

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Normalised output y(t) and dy/dt of a network, one input per lane, float32.
template <bool kTan>
__device__ __forceinline__ void mlp_lane(const float *__restrict__ p, float t, float &y, float &dy) {
    float h1[MLP_H], d1[MLP_H];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) {
        const float w = p[OFF_W1 + k];
        const float z = w * t + p[OFF_B1 + k];
        const float sg = sigm(z);
        h1[k] = z * sg;
        if (kTan) d1[k] = (sg + h1[k] * (1.0f - sg)) * w;
    }
    float yy = p[OFF_B3], dd = 0.0f;
    for (int n = 0; n < MLP_H; ++n) {
        const float *w2 = p + OFF_W2 + n * MLP_H;
        float z = p[OFF_B2 + n], dz = 0.0f;
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) {
            z += w2[k] * h1[k];
            if (kTan) dz += w2[k] * d1[k];
        }
        const float sg = sigm(z);
        const float h = z * sg;
        yy += p[OFF_W3 + n] * h;
        if (kTan) dd += p[OFF_W3 + n] * (sg + h * (1.0f - sg)) * dz;
    }
    y = yy;
    dy = dd;
}

__device__ __forceinline__ bool mlp_serves(const MlpNet &m, float x) { return x >= m.x_lo && x <= m.x_hi; }

// g(x) and g'(x) in physical units.
__device__ __forceinline__ void mlp_eval_lane(const MlpNet &m, float x, float &g, float &dg) {
    float y, dy;
    mlp_lane<true>(m.p, (x - m.c) * m.s, y, dy);
    g = m.y_shift + m.y_scale * y;
    dg = m.y_scale * m.s * dy;
}

// ---------------------------------------------------------------------------
// Training jobs (filled on the host, read by the kernels).

constexpr int GRAD_SAMPLES = 64;  // samples per block of the gradient kernel
constexpr int GRAD_SPLIT = 4;                           // lanes per sample
constexpr int GRAD_THREADS = GRAD_SAMPLES * GRAD_SPLIT;  // threads per block of the gradient kernel
constexpr int GRAD_UNITS = MLP_H / GRAD_SPLIT;           // hidden units per lane

struct GradJob {
    const float *p;        // weights used by the forward pass
    float c, s;            // input scaling
    float y_shift, y_scale;
    const double *x;       // sample inputs
    int64_t n;             // samples available
    // Sobolev mode (cval == nullptr): targets, and a random mini-batch
    const double *y, *dy;
    float lam;
    uint64_t seed, step;
    int64_t batch;         // samples this call
    // coefficient mode: cval[i], cder[i] for sample i = 0 .. n-1 in order
    const double *cval, *cder;
    float *part;           // [blocks][MLP_NP]
    double *loss_part;     // [blocks] (Sobolev mode)
};

// One network's share of a fused fit iteration (k_fit_step).
struct FitStep {
    GradJob J;                     // the gradient job of blocks 0 .. nblk1 - 1 (all of them if nblk1 = 0)
    GradJob J2;                    // blocks nblk1 ..: a second job whose partials follow J's
    int nblk1;
    float *w, *m, *v, *q;          // float32 master weights, Adam moments, bfloat16 copy
    double bc1, bc2;               // Adam bias corrections of this step
    int32_t *ticket;               // blocks finished in this launch (zero between launches)
    double *loss_hist;             // the iteration's summed loss (J.loss_part) goes to loss_hist[slot] if slot >= 0
    int slot;
};

struct FitSteps {
    FitStep s[3];
    int nnet;
    double lr;
};

struct FmJob {
    MlpNet nf, np;              // forward weights (training copies)
    const double *r, *dhat, *fpj, *fpi, *fref;
    int64_t n_env;
    const int32_t *envs;        // mini-batch: environment ids
    int nb;
    double inv_norm;            // 1 / (nb <|f_ref|^2>)
    double *x_out;              // [nb][MISA_FM_SLOTS] pair distances of the batch (0 = none)
    double *cf, *cp;            // [nb][MISA_FM_SLOTS] coefficients of dy/dt of f and phi
    double *loss_part;          // [nb]
};

hipError_t launch_mlp_eval(hipStream_t st, int path, const MlpNet &m, const uint16_t *w2b, const double *x,
                           int64_t n, double *y, double *dy);
hipError_t launch_grad(hipStream_t st, const GradJob &J, int nblk);
hipError_t launch_fit_step(hipStream_t st, const FitSteps &F, int nblk);
hipError_t launch_grad_sum(hipStream_t st, const float *part, int nblk, double *grad);
hipError_t launch_adam(hipStream_t st, float *w, float *m, float *v, const double *grad, float *q, double lr,
                       int64_t step);
hipError_t launch_round_weights(hipStream_t st, const float *w, float *q, uint16_t *w2b);
hipError_t launch_fm(hipStream_t st, const FmJob &J, uint64_t seed, uint64_t step, int32_t *envs);
hipError_t launch_fm_norm(hipStream_t st, const double *fref, int64_t n, double *out);
hipError_t launch_sum_into(hipStream_t st, const double *a, int n, double *out, int slot);

}  // namespace misa
