// mlp.hpp -- sizes, parameter layout and scratch of the warm-start network.
#pragma once

#include <hip/hip_runtime.h>

namespace turret {

constexpr int kMlpIn = 16, kMlpH = 64, kMlpOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 5443
constexpr int kMlpSlice = 256;                 // samples per weight-gradient partial sum

// Warm-start features of marker k, each a 3-vector over the marker's scale
// s_k = |h0(t)| + |h(t-1)|: the plain start h0(t) = U - I[u*], the previous
// step's final h(t-1), the last change of the final h, h(t-1) - h(t-2), and
// the change of the plain start, h0(t) - h0(t-1) (the changes are formed in
// FP64 before they are scaled: as differences of two FP16 operands of
// similar size they would keep only a few bits); then the normal n and the
// marker's area dS.  The network predicts the change of h from h(t-1), over
// s_k.
constexpr int kFeatH0 = 0, kFeatHPrev = 3, kFeatDH = 6, kFeatDH0 = 9, kFeatNormal = 12, kFeatArea = 15;

// Per-sample training scratch, [field][sample] layout (n samples).
struct MlpScratch {
    float *a1, *a2, *d1, *d2;   // activations and SiLU derivatives, 64 fields each
    float *dz1, *dz2;           // back-propagated pre-activation gradients, 64 fields each
    float *dy;                  // output errors / n, 3 fields
    float *part;                // weight-gradient partial sums [slices][params]
    float *loss_part;           // loss partial sums per block
};

struct DevPtrs;
hipError_t launch_mlp_forward(const _Float16 *th16, const float *X, int n, float *Y, hipStream_t s);
hipError_t launch_mlp_warm_start(const _Float16 *th16, const DevPtrs &p, int Mtot, hipStream_t s);
hipError_t launch_mlp_grad(const _Float16 *th16, const float *X, const float *T, int n, const MlpScratch &sc,
                           float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *th32, _Float16 *th16, float *m, float *v, const float *g, float lr, int step,
                           hipStream_t s);
hipError_t launch_mlp_round(const float *th32, _Float16 *th16, hipStream_t s);

}  // namespace turret
