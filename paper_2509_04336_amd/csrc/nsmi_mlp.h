// Surrogate network buffers and drivers (see nsmi_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsmi_device.h"

namespace nsmi {

// The activation silu(z) = z sigmoid(z) in FP32, written once for every
// network pass (training, prediction and the in-walk screen) so all of them
// compute the same values: sigmoid with the hardware exponential and the
// hardware reciprocal (about 1 ulp each; the activations are rounded to BF16
// afterwards).
__device__ __forceinline__ float mlp_sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float mlp_silu(float z) { return z * mlp_sigmoid(z); }

constexpr int MLP_IN = 11;    // inputs: the unit-cube point, zero padded
constexpr int MLP_KIN = 32;   // inputs padded to one MFMA k-step
constexpr int MLP_H = 256;    // hidden width (three hidden layers)
constexpr int64_t MLP_OFF_W1 = 0;
constexpr int64_t MLP_OFF_B1 = MLP_OFF_W1 + (int64_t)MLP_H * MLP_IN;
constexpr int64_t MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int64_t MLP_OFF_B2 = MLP_OFF_W2 + (int64_t)MLP_H * MLP_H;
constexpr int64_t MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int64_t MLP_OFF_B3 = MLP_OFF_W3 + (int64_t)MLP_H * MLP_H;
constexpr int64_t MLP_OFF_W4 = MLP_OFF_B3 + MLP_H;
constexpr int64_t MLP_OFF_B4 = MLP_OFF_W4 + MLP_H;
constexpr int64_t MLP_NPARAM = MLP_OFF_B4 + 1;  // 134913
// Weight-gradient products contract over the batch rows (K up to max_rows):
// they are split over at most MLP_SPLITK workgroup slices of K.
constexpr int MLP_SPLITK = 32;

// Device buffers of one network and its training workspace for batches of
// up to max_rows rows (a multiple of 32).
struct MlpBuffers {
    int64_t max_rows = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // fp32 master, grad, Adam
    __bf16 *W1p = nullptr, *W1T = nullptr, *W2 = nullptr, *W3 = nullptr, *W2T = nullptr, *W3T = nullptr;
    __bf16 *X = nullptr, *XT = nullptr;
    float *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
    __bf16 *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *h1T = nullptr, *h2T = nullptr, *h3T = nullptr;
    // back-propagated deltas: two row-major buffers, and the feature-major
    // deltas of layers 3, 2, 1 at dT, dT + max_rows MLP_H, dT + 2 max_rows MLP_H
    __bf16 *d = nullptr, *d2 = nullptr, *dT = nullptr;
    float *gtmp = nullptr, *y = nullptr, *dy = nullptr, *t = nullptr;
    double *stats = nullptr, *loss = nullptr;
    double *sq = nullptr;  // squared error of each training row (0 on padding rows)
    float *in_mu = nullptr, *in_isig = nullptr;  // input standardisation [MLP_KIN]
    // split-K partial products of the weight gradients of layers 3, 2, 1:
    // three regions of [MLP_SPLITK][MLP_H][MLP_H]
    float *ws = nullptr;
    double mu = 0.0, sig = 1.0, clip = -1e300;  // target normalisation
    double top = HUGE_VAL;                      // log-gap transform when finite
};

// Training target of a log-likelihood y before standardisation: max(y, clip),
// or with a finite top the log-gap z = -log(top - max(y, clip)), which spreads
// the values just below top (where the screen decides) and compresses the
// far tail.  Gaps are floored at 1e-12.
__host__ __device__ inline double target_z(double y, double clip, double top)
{
    double v = y > clip ? y : clip;
    if (top < HUGE_VAL) {
        double g = top - v;
        v = -log(g > 1e-12 ? g : 1e-12);
    }
    return v;
}

// Inverse of target_z for a de-standardised network output z.
__host__ __device__ inline double target_from_z(double z, double top)
{
    return top < HUGE_VAL ? top - exp(-z) : z;
}

hipError_t mlp_refresh_weights(MlpBuffers &B, hipStream_t s);
hipError_t mlp_init_params(MlpBuffers &B, uint64_t seed, hipStream_t s);
hipError_t mlp_forward(MlpBuffers &B, const double *u, int ndim, int64_t n, double *out,
                       hipStream_t s);
hipError_t mlp_loss_grad(MlpBuffers &B, const double *u, int ndim, const double *y, int64_t n,
                         hipStream_t s);
hipError_t mlp_target_stats(MlpBuffers &B, const double *y, int64_t n, hipStream_t s);
hipError_t mlp_input_stats(MlpBuffers &B, const double *u, int ndim, int64_t n, hipStream_t s);
hipError_t mlp_train_step(MlpBuffers &B, const double *u, const double *y, int ndim, int64_t n_src,
                          int64_t batch, uint64_t seed, int64_t step, float lr, hipStream_t s);

}  // namespace nsmi
