// mlp.hpp -- sizes, parameter layout and scratch of the warm-start network.
#pragma once

#include <hip/hip_runtime.h>

namespace turret {

constexpr int kMlpIn = 12, kMlpH = 64, kMlpOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 5187
constexpr int kMlpSlice = 256;                 // samples per weight-gradient partial sum

// The marker velocity feature is scaled by 1 / 0.02, the largest lattice
// terminal velocity of the cases, so it is O(1); the force-like features
// and the output are taken over a per-marker scale instead.
constexpr double kFeatScale = 50.0;
// Features kFeatHPrev .. kFeatHPrev + 2 are the previous step's final h over
// the marker's scale; a zero network output starts from them.
constexpr int kFeatHPrev = 9;

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
