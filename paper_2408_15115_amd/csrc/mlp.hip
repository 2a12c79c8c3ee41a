// mlp.hip -- the warm-start network of the learned IBM form: a
// 16 -> 64 -> 64 -> 3 multilayer perceptron with SiLU hidden activations,
// FP16 weights and FP32 accumulation; inference for every marker, and
// training (per-sample forward/backward, deterministic weight-gradient sums,
// Adam) on samples the solver produced.
//
// Parameter layout (flat): W1[64][16] b1[64] W2[64][64] b2[64] W3[3][64] b3[3].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"
#include "mlp.hpp"

namespace turret {

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }
// The same with the hardware reciprocal (about 1 ulp), for FP16-operand inference.
__device__ __forceinline__ float sigmoid_fast(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// Weights: FP16 in HBM, widened once per workgroup into LDS.
__device__ __forceinline__ void load_weights(const _Float16 *__restrict__ th16, float *w)
{
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = (float)th16[i];
    __syncthreads();
}

// Forward pass of one sample; optionally keeps a1, a2, silu'(z1), silu'(z2).
__device__ __forceinline__ void mlp_forward_one(const float *w, const float x[kMlpIn], float y[kMlpOut],
                                                float *a1o, float *a2o, float *d1o, float *d2o, int stride)
{
    const float *W1 = w + kOffW1, *b1 = w + kOffB1, *W2 = w + kOffW2, *b2 = w + kOffB2, *W3 = w + kOffW3,
                *b3 = w + kOffB3;
    float a1[kMlpH];
#pragma unroll
    for (int o = 0; o < kMlpH; o++) {
        float z = b1[o];
#pragma unroll
        for (int i = 0; i < kMlpIn; i++) z = fmaf(W1[o * kMlpIn + i], x[i], z);
        const float s = sigmoidf(z);
        a1[o] = z * s;
        if (a1o) {
            a1o[o * stride] = a1[o];
            d1o[o * stride] = s + z * s * (1.0f - s);
        }
    }
    float y0 = b3[0], y1 = b3[1], y2 = b3[2];
    for (int o = 0; o < kMlpH; o++) {
        float z = b2[o];
#pragma unroll
        for (int i = 0; i < kMlpH; i++) z = fmaf(W2[o * kMlpH + i], a1[i], z);
        const float s = sigmoidf(z);
        const float a = z * s;
        if (a2o) {
            a2o[o * stride] = a;
            d2o[o * stride] = s + z * s * (1.0f - s);
        }
        y0 = fmaf(W3[o], a, y0);
        y1 = fmaf(W3[kMlpH + o], a, y1);
        y2 = fmaf(W3[2 * kMlpH + o], a, y2);
    }
    y[0] = y0;
    y[1] = y1;
    y[2] = y2;
}

// ------------------------------------------------ inference on the matrix cores
// Inference runs on v_mfma_f32_16x16x16_f16: FP16 weights and activations,
// FP32 accumulation, SiLU in FP32.  A wavefront takes 16 samples at a time as
// the 16 columns of D = W X: for each layer the weights are the A operand
// (rows = output neurons, 16 per chunk) and the previous layer's activations
// the B operand (k = input neurons, 16 per step).  Lane l of the wave holds
// B[k][j] and D[i][j] for sample j = l % 16 and k, i = 4 (l / 16) + e
// (e = 0..3), so a layer's output chunk c is, as it stands in the registers,
// the next layer's operand for input step c.  The weights stay in registers
// while the wave strides over sample tiles.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kInSteps = (kMlpIn + 15) / 16;   // 16-wide input steps of layer 1 (zero padded)
constexpr int kHChunks = kMlpH / 16;
static_assert(kMlpH % 16 == 0 && kMlpOut <= 4, "layer sizes of the matrix-core inference");
static_assert(kMlpIn % 4 == 0 && kOffW2 % 4 == 0 && kOffB1 % 4 == 0 && kOffB2 % 4 == 0 && kOffW3 % 4 == 0,
              "8-byte aligned parameter blocks for the vector loads");

struct MlpRegs {
    half4_t w1[kHChunks][kInSteps], w2[kHChunks][kHChunks], w3[kHChunks];
    float b1[kHChunks][4], b2[kHChunks][4], b3[4];
};

// Four consecutive FP16 parameters starting at a multiple of 4 (one 8-byte load).
__device__ __forceinline__ half4_t load_half4(const _Float16 *th, int at)
{
    return *reinterpret_cast<const half4_t *>(th + at);
}

// The FP16 parameters, staged once per 256-thread workgroup in LDS with
// 16-byte copies (the parameter buffer extends to a 256-byte boundary, past
// the rounding up to 8 values).  Every load of a thread is issued before the
// first store, so the staging waits for one memory latency, not one per
// round of copies; the plain copy is padded to whole rounds (the padding
// holds repeats of the last vector) so that no store is conditional.
//
// W1 and W2 are also laid out in LDS as the register image of their A
// operands: slot (matrix, mc, kc) holds, for lanes l = 0..63 in a row, the 4
// values W[16 mc + l % 16][16 kc + 4 (l / 16) + 0..3], so that a wave takes
// each operand with one conflict-free 8-byte read per lane.  (Read straight
// from the row-major copy, the 16 rows of a W2 operand lie 128 bytes apart
// and fall into the same LDS banks.)  W3 and the biases are read from the
// plain copy, where lanes that share an address get it broadcast.
constexpr int kMlpParams8 = (kMlpParams + 7) / 8 * 8;
constexpr int kStageVecs = kMlpParams8 / 8;
constexpr int kStageRounds = (kStageVecs + 255) / 256;
constexpr int kStageHalves = kStageRounds * 256 * 8;
constexpr int kImgW1 = 0;                              // slot of (mc, kc): kImgW1 + mc kInSteps + kc
constexpr int kImgW2 = kHChunks * kInSteps;            // slot of (mc, kc): kImgW2 + mc kHChunks + kc
constexpr int kImgSlots = kImgW2 + kHChunks * kHChunks;
static_assert(kOffW2 % 8 == 0 && kOffB1 % 8 == 0 && kOffB2 % 8 == 0,
              "16-byte parameter vectors never straddle W1 / W2 and the next block");

struct MlpLds {
    _Float16 raw[kStageHalves];
    half4_t img[kImgSlots * 64];
};

// Places W[o][c..c+3] (c a multiple of 4) of a matrix with `steps` 16-wide
// column steps into its operand slot.
__device__ __forceinline__ void img_put(half4_t *img, int base, int steps, int o, int c, half4_t v)
{
    img[(base + (o >> 4) * steps + (c >> 4)) * 64 + (o & 15) + 16 * ((c & 15) >> 2)] = v;
}

__device__ inline void mlp_stage(const _Float16 *__restrict__ th, MlpLds &L)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(th);
    uint4 *dst = reinterpret_cast<uint4 *>(L.raw);
    uint4 v[kStageRounds];
#pragma unroll
    for (int j = 0; j < kStageRounds; j++) v[j] = src[std::min((int)threadIdx.x + 256 * j, kStageVecs - 1)];
#pragma unroll
    for (int j = 0; j < kStageRounds; j++) {
        const int i = (int)threadIdx.x + 256 * j, h = 8 * i;
        dst[i] = v[j];
        const half4_t lo = __builtin_bit_cast(half4_t, make_uint2(v[j].x, v[j].y)),
                      hi = __builtin_bit_cast(half4_t, make_uint2(v[j].z, v[j].w));
        if (h < kOffB1) {
            const int o = (h - kOffW1) / kMlpIn, c = (h - kOffW1) % kMlpIn;
            img_put(L.img, kImgW1, kInSteps, o, c, lo);
            img_put(L.img, kImgW1, kInSteps, o, c + 4, hi);
        } else if (h >= kOffW2 && h < kOffB2) {
            const int o = (h - kOffW2) / kMlpH, c = (h - kOffW2) % kMlpH;
            img_put(L.img, kImgW2, kHChunks, o, c, lo);
            img_put(L.img, kImgW2, kHChunks, o, c + 4, hi);
        }
    }
    __syncthreads();
}

__device__ inline void mlp_load_regs(const MlpLds &L, MlpRegs &R)
{
    const _Float16 *th = L.raw;
    const int l = threadIdx.x & 63, r = l & 15, kq = (l >> 4) * 4;
    const _Float16 zero = (_Float16)0.0f;
#pragma unroll
    for (int mc = 0; mc < kHChunks; mc++) {
#pragma unroll
        for (int kc = 0; kc < kInSteps; kc++) R.w1[mc][kc] = L.img[(kImgW1 + mc * kInSteps + kc) * 64 + l];
#pragma unroll
        for (int kc = 0; kc < kHChunks; kc++) R.w2[mc][kc] = L.img[(kImgW2 + mc * kHChunks + kc) * 64 + l];
        // biases of the D rows this lane holds
        const half4_t b1 = load_half4(th, kOffB1 + 16 * mc + kq), b2 = load_half4(th, kOffB2 + 16 * mc + kq);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            R.b1[mc][e] = (float)b1[e];
            R.b2[mc][e] = (float)b2[e];
        }
    }
#pragma unroll
    for (int kc = 0; kc < kHChunks; kc++) {
        const half4_t w = load_half4(th, kOffW3 + (r < kMlpOut ? r : 0) * kMlpH + 16 * kc + kq);
        const half4_t z = {zero, zero, zero, zero};
        R.w3[kc] = r < kMlpOut ? w : z;
    }
#pragma unroll
    for (int e = 0; e < 4; e++) R.b3[e] = kq + e < kMlpOut ? (float)th[kOffB3 + kq + e] : 0.0f;
}

__device__ __forceinline__ float4_t mfma16(half4_t a, half4_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// One tile of 16 samples: x holds this lane's B operand of layer 1; the
// result holds, in lanes 0..15, outputs 0..kMlpOut-1 of sample l.  The bias
// is the accumulator's initial value, so the matrix cores add it.  SiLU is
// the tile's main cost: two quarter-rate transcendentals (exp, reciprocal)
// per hidden value.
__device__ inline float4_t mlp_tile(const MlpRegs &R, const half4_t x[kInSteps])
{
    half4_t a1[kHChunks], a2[kHChunks];
#pragma unroll
    for (int mc = 0; mc < kHChunks; mc++) {
        float4_t d = {R.b1[mc][0], R.b1[mc][1], R.b1[mc][2], R.b1[mc][3]};
#pragma unroll
        for (int kc = 0; kc < kInSteps; kc++) d = mfma16(R.w1[mc][kc], x[kc], d);
#pragma unroll
        for (int e = 0; e < 4; e++) a1[mc][e] = (_Float16)(d[e] * sigmoid_fast(d[e]));
    }
#pragma unroll
    for (int mc = 0; mc < kHChunks; mc++) {
        float4_t d = {R.b2[mc][0], R.b2[mc][1], R.b2[mc][2], R.b2[mc][3]};
#pragma unroll
        for (int kc = 0; kc < kHChunks; kc++) d = mfma16(R.w2[mc][kc], a1[kc], d);
#pragma unroll
        for (int e = 0; e < 4; e++) a2[mc][e] = (_Float16)(d[e] * sigmoid_fast(d[e]));
    }
    float4_t y = {R.b3[0], R.b3[1], R.b3[2], R.b3[3]};
#pragma unroll
    for (int kc = 0; kc < kHChunks; kc++) y = mfma16(R.w3[kc], a2[kc], y);
    return y;
}

// This lane's layer-1 operand for sample s of an n x kMlpIn FP32 array
// (zeros past n): four consecutive features per input step, one 16-byte
// load each.  The loads and the conversion to FP16 are split so that a
// wave can issue the next tile's loads before it works on the current tile.
static_assert(kMlpIn % 16 == 0, "one 16-byte feature load per lane and input step");
struct MlpRaw {
    float4 v[kInSteps];
};

__device__ inline MlpRaw mlp_load(const float *__restrict__ X, int s, int n)
{
    const int kq = ((threadIdx.x & 63) >> 4) * 4;
    MlpRaw r;
#pragma unroll
    for (int kc = 0; kc < kInSteps; kc++) {
        r.v[kc] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (s < n) r.v[kc] = *reinterpret_cast<const float4 *>(X + (long long)s * kMlpIn + 16 * kc + kq);
    }
    return r;
}

__device__ inline void mlp_convert(const MlpRaw &r, half4_t x[kInSteps])
{
#pragma unroll
    for (int kc = 0; kc < kInSteps; kc++) {
        x[kc][0] = (_Float16)r.v[kc].x;
        x[kc][1] = (_Float16)r.v[kc].y;
        x[kc][2] = (_Float16)r.v[kc].z;
        x[kc][3] = (_Float16)r.v[kc].w;
    }
}

// Tiles a wave takes per round.  Their features are loaded together, those
// of the first round before the weights are staged (both latencies overlap),
// those of the next round while the wave works on the current one.
constexpr int kMlpRound = 2;

// The inference loop shared by the two kernels: every wave strides over
// 16-sample tiles (the loop bounds are the same for the whole wave); epi(s,
// x, R) finishes sample s of this lane from its layer-1 operand x.
template <class Epi>
__device__ inline void mlp_stream(const _Float16 *__restrict__ th16, MlpLds &wsh, const float *__restrict__ X,
                                  int n, Epi &&epi)
{
    const int l = threadIdx.x & 63;
    const int wave = (int)(blockIdx.x * 4 + (threadIdx.x >> 6)), nwaves = (int)(gridDim.x * 4);   // 256 threads
    const int stride = 16 * nwaves;
    MlpRaw buf[kMlpRound];
#pragma unroll
    for (int j = 0; j < kMlpRound; j++) buf[j] = mlp_load(X, 16 * wave + j * stride + (l & 15), n);
    mlp_stage(th16, wsh);
    MlpRegs R;
    mlp_load_regs(wsh, R);
    for (int base = 16 * wave; base < n; base += kMlpRound * stride) {
#pragma unroll
        for (int j = 0; j < kMlpRound; j++) {
            const int s0 = base + j * stride;
            if (s0 >= n) break;
            half4_t x[kInSteps];
            mlp_convert(buf[j], x);
            buf[j] = mlp_load(X, s0 + kMlpRound * stride + (l & 15), n);   // the next round's tile j
            epi(s0 + (l & 15), x, R);
        }
    }
}

// Inference on caller arrays: X (n x kMlpIn) -> Y (n x 3).
__global__ void __launch_bounds__(256) k_mlp_forward(const _Float16 *__restrict__ th16, const float *__restrict__ X,
                                                     int n, float *__restrict__ Y)
{
    __shared__ __align__(16) MlpLds wsh;
    const int l = threadIdx.x & 63;
    mlp_stream(th16, wsh, X, n, [&](int s, const half4_t *x, const MlpRegs &R) {
        const float4_t y = mlp_tile(R, x);
        if (l < 16 && s < n)
#pragma unroll
            for (int j = 0; j < kMlpOut; j++) Y[(long long)s * kMlpOut + j] = y[j];
    });
}

// Warm start inside the IBM coupling: the network predicts, over the
// marker's feature scale s_k, the change of h from the previous step's final
// value: h = s_k (h(t-1) / s_k + MLP(features_k)), for every marker of an
// unmasked case; it becomes the first increment to spread.  A zero network
// starts from h(t-1), the control start.
__global__ void __launch_bounds__(256) k_mlp_warm_start(const _Float16 *__restrict__ th16, DevPtrs p, int Mtot)
{
    __shared__ __align__(16) MlpLds wsh;
    const int l = threadIdx.x & 63;
    mlp_stream(th16, wsh, p.feat, Mtot, [&](int k, const half4_t *x, const MlpRegs &R) {
        // the epilogue's operands, loaded before the matrix work
        bool live = false;
        float hp[3] = {0.0f, 0.0f, 0.0f};
        double hs = 0.0;
        if (l < 16 && k < Mtot) {
            live = p.body[p.mcase[k]].err == 0;
#pragma unroll
            for (int a = 0; a < 3; a++) hp[a] = p.feat[(long long)kMlpIn * k + kFeatHPrev + a];
            hs = p.hs[k];
        }
        const float4_t y = mlp_tile(R, x);
        if (live)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                p.hk[3 * k + a] = 0.0;
                p.dh[3 * k + a] = ((double)hp[a] + (double)y[a]) * hs;
            }
    });
}

// Training, pass 1: forward of every sample, keeping the activations and
// SiLU derivatives (scratch, layout [field][sample]), dY = (Y - T)/N and the
// per-block loss partial 1/(2N) sum |Y - T|^2.
__global__ void __launch_bounds__(256) k_mlp_fwd_train(const _Float16 *__restrict__ th16, const float *__restrict__ X,
                                                       const float *__restrict__ Tg, int n, MlpScratch sc)
{
    __shared__ float w[kMlpParams];
    __shared__ float red[256];
    load_weights(th16, w);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (s < n) {
        float x[kMlpIn], y[kMlpOut];
#pragma unroll
        for (int i = 0; i < kMlpIn; i++) x[i] = X[(long long)s * kMlpIn + i];
        mlp_forward_one(w, x, y, sc.a1 + s, sc.a2 + s, sc.d1 + s, sc.d2 + s, n);
#pragma unroll
        for (int j = 0; j < kMlpOut; j++) {
            const float e = y[j] - Tg[(long long)s * kMlpOut + j];
            sc.dy[j * n + s] = e / (float)n;
            l += e * e;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc.loss_part[blockIdx.x] = red[0] * 0.5f / (float)n;
}

// Training, pass 2: back-propagate dY to dz2 = (W3^T dY) silu'(z2) and
// dz1 = (W2^T dz2) silu'(z1) per sample.
__global__ void __launch_bounds__(256) k_mlp_bwd_train(const _Float16 *__restrict__ th16, int n, MlpScratch sc)
{
    __shared__ float w[kMlpParams];
    load_weights(th16, w);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float *W2 = w + kOffW2, *W3 = w + kOffW3;
    const float dy0 = sc.dy[s], dy1 = sc.dy[n + s], dy2 = sc.dy[2 * n + s];
    float dz2[kMlpH];
#pragma unroll
    for (int o = 0; o < kMlpH; o++) {
        const float g = W3[o] * dy0 + W3[kMlpH + o] * dy1 + W3[2 * kMlpH + o] * dy2;
        dz2[o] = g * sc.d2[o * n + s];
        sc.dz2[o * n + s] = dz2[o];
    }
    for (int i = 0; i < kMlpH; i++) {
        float g = 0.0f;
#pragma unroll
        for (int o = 0; o < kMlpH; o++) g = fmaf(W2[o * kMlpH + i], dz2[o], g);
        sc.dz1[i * n + s] = g * sc.d1[i * n + s];
    }
}

// Training, pass 3: weight gradients as sums over samples of outer products,
// one thread per parameter per slice of samples (partial[slice][param]); the
// sums over slices are taken in a fixed order by k_mlp_reduce, so the
// gradient is bitwise reproducible.
__global__ void __launch_bounds__(256) k_mlp_wgrad(const float *__restrict__ X, int n, int slice, MlpScratch sc)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const int s0 = blockIdx.y * slice, s1 = min(n, s0 + slice);
    const float *u = nullptr, *v = nullptr;   // gradient = sum_s u[s] * v[s]
    int vstride = 0;
    const float *vX = nullptr;
    int xi = 0;
    if (p < kOffB1) {                 // W1[o][i] = sum dz1[o] x[i]
        const int o = p / kMlpIn;
        xi = p - o * kMlpIn;
        u = sc.dz1 + (long long)o * n;
        vX = X;
    } else if (p < kOffW2) {          // b1[o] = sum dz1[o]
        u = sc.dz1 + (long long)(p - kOffB1) * n;
    } else if (p < kOffB2) {          // W2[o][i] = sum dz2[o] a1[i]
        const int q = p - kOffW2, o = q / kMlpH, i = q - o * kMlpH;
        u = sc.dz2 + (long long)o * n;
        v = sc.a1 + (long long)i * n;
        vstride = 1;
    } else if (p < kOffW3) {          // b2[o] = sum dz2[o]
        u = sc.dz2 + (long long)(p - kOffB2) * n;
    } else if (p < kOffB3) {          // W3[j][i] = sum dy[j] a2[i]
        const int q = p - kOffW3, j = q / kMlpH, i = q - j * kMlpH;
        u = sc.dy + (long long)j * n;
        v = sc.a2 + (long long)i * n;
        vstride = 1;
    } else {                          // b3[j] = sum dy[j]
        u = sc.dy + (long long)(p - kOffB3) * n;
    }
    float acc = 0.0f;
    if (vX) {
        for (int s = s0; s < s1; s++) acc = fmaf(u[s], vX[(long long)s * kMlpIn + xi], acc);
    } else if (vstride) {
        for (int s = s0; s < s1; s++) acc = fmaf(u[s], v[s], acc);
    } else {
        for (int s = s0; s < s1; s++) acc += u[s];
    }
    sc.part[(long long)blockIdx.y * kMlpParams + p] = acc;
}

__global__ void __launch_bounds__(256) k_mlp_reduce(int nslices, int nloss, MlpScratch sc, float *__restrict__ grad,
                                                    float *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        float g = 0.0f;
        for (int k = 0; k < nslices; k++) g += sc.part[(long long)k * kMlpParams + p];
        grad[p] = g;
    }
    if (p == 0 && loss) {
        float l = 0.0f;
        for (int k = 0; k < nloss; k++) l += sc.loss_part[k];
        *loss = l;
    }
}

// Adam (Kingma & Ba): FP32 master weights and moments; the FP16 copy used by
// the forward passes is refreshed (round to nearest even).
__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ th32, _Float16 *__restrict__ th16,
                                                  float *__restrict__ m, float *__restrict__ v,
                                                  const float *__restrict__ g, float lr, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.0f - b1) * g[p];
    const float vv = b2 * v[p] + (1.0f - b2) * g[p] * g[p];
    m[p] = mm;
    v[p] = vv;
    const float t = th32[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    th32[p] = t;
    th16[p] = (_Float16)t;
}

__global__ void k_mlp_round(const float *__restrict__ th32, _Float16 *__restrict__ th16)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) th16[p] = (_Float16)th32[p];
}

// ------------------------------------------------------------ launchers
// Workgroups of 4 waves for the matrix-core inference: one wave per 16-sample
// tile up to 2048 waves (2 per SIMD), which then stride.  Over the 161,818
// markers of the 64-case batch this takes 9.1 us; 1024 and 4096 waves were
// slower, and 8192 waves much slower (each workgroup stages the weights).
static dim3 infer_grid(int n)
{
    const int tiles = (n + 15) / 16;
    return dim3((unsigned)std::max(1, (std::min(tiles, 2048) + 3) / 4));
}

hipError_t launch_mlp_forward(const _Float16 *th16, const float *X, int n, float *Y, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, infer_grid(n), dim3(256), 0, s, th16, X, n, Y);
    return hipGetLastError();
}

hipError_t launch_mlp_warm_start(const _Float16 *th16, const DevPtrs &p, int Mtot, hipStream_t s)
{
    if (Mtot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_warm_start, infer_grid(Mtot), dim3(256), 0, s, th16, p, Mtot);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const _Float16 *th16, const float *X, const float *Tg, int n, const MlpScratch &sc,
                           float *grad, float *loss, hipStream_t s)
{
    const int nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_mlp_fwd_train, dim3(nb), dim3(256), 0, s, th16, X, Tg, n, sc);
    hipLaunchKernelGGL(k_mlp_bwd_train, dim3(nb), dim3(256), 0, s, th16, n, sc);
    const int slices = (n + kMlpSlice - 1) / kMlpSlice;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((kMlpParams + 255) / 256, slices), dim3(256), 0, s, X, n, kMlpSlice, sc);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, slices, nb, sc, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *th32, _Float16 *th16, float *m, float *v, const float *g, float lr, int step,
                           hipStream_t s)
{
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, th32, th16, m, v, g, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_round(const float *th32, _Float16 *th16, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_round, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, th32, th16);
    return hipGetLastError();
}

}  // namespace turret
