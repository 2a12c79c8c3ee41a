// lattice.hpp -- D3Q27 constants, population storage codecs and the
// separable Hermite-basis collision used by the gfx950 kernels.
//
// The recursive-regularized collision of arXiv 2408.15115 (Sec. 2.1, App. A)
// is evaluated here in the tensor-product Hermite basis of D3Q27: with the
// one-dimensional normalized Hermite polynomials
//     e0(xi) = 1,  e1(xi) = xi / cs^2,  e2(xi) = (xi^2 - cs^2) / (2 cs^4),
// every population set supported by the lattice is
//     f_i = w_i * sum_m A_m e_mx(xi_x) e_my(xi_y) e_mz(xi_z),   m in {0,1,2}^3,
// where A_m is the Hermite coefficient of multi-index m.  The post-collision
// state of App. A has
//     A_000 = rho,  A_a = rho u~_a,
//     A_m   = rho u~^m + (1 - 1/tau) a1_m          (|m| >= 2),
// with u~ = u + tau h (Sec. 2.2 forced rule) and a1_m the App. A coefficients,
// which for D3Q27 multi-indices equal  (1/2) P1 : grad_u grad_u (u^m)
// (each index pair of the string contributes P1 times the remaining u's).
// Populations are kept as deviations g_i = f_i - w_i, so A_000 is replaced by
// rho - 1 and no O(1) cancellation ever happens in FP32.
//
// Both directions of the change of basis factor into three passes of
// 3-point transforms along x, y and z (81 multiply-adds each way), instead
// of the 27 x 27 dense sums of the printed formulas.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace turret {

constexpr int Q = 27;
constexpr float CS2 = 1.0f / 3.0f;

__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wq(int i) { return w1d(cx(i)) * w1d(cy(i)) * w1d(cz(i)); }
// direction with xi_z reversed (specular wall) and fully reversed (bounce-back)
__host__ __device__ constexpr int mirror_z(int i) { return 9 * (-cz(i) + 1) + 3 * (cy(i) + 1) + (cx(i) + 1); }
__host__ __device__ constexpr int opposite(int i) { return 26 - i; }

// FP16/BF16 storage keeps s_i * g_i with the power of two
// s_i = 2^(14 + 2 |xi_i|^2), the first power of two at or above 4096 / w_i:
// g_i / w_i is O(|u|), so stored magnitudes sit well inside the FP16 normal
// range (|g_i / w_i| up to 13.49 in every direction) and the rest state is
// exactly 0.  A power of two makes the scaling itself exact in FP32 in both
// directions, so the only rounding is the store's.  Mirror and opposite
// directions share |xi_i|, so wall rules never change the scale.
__host__ __device__ constexpr int scale_exp(int i) { return 14 + 2 * (cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i)); }
__host__ __device__ constexpr double store_scale(int i) { return (double)(1ull << scale_exp(i)); }

enum { BC_PERIODIC = 0, BC_FREESLIP = 1, BC_NOSLIP = 2, BC_PRESSURE = 3 };
enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2, ST_MOM = 3 };

// ------------------------------------------------------------------ codecs
struct CodecF32 {
    using T = float;
    template <int I> __device__ static inline float dec(T v) { return v; }
    template <int I> __device__ static inline T enc(float g) { return g; }
};

struct CodecF16 {
    using T = _Float16;
    template <int I> __device__ static inline float dec(T v)
    {
        return (float)v * (float)(1.0 / store_scale(I));
    }
    template <int I> __device__ static inline T enc(float g)
    {
        return (_Float16)(g * (float)store_scale(I));   // v_cvt_f16_f32: round to nearest even
    }
};

struct CodecBF16 {
    using T = uint16_t;
    template <int I> __device__ static inline float dec(T v)
    {
        return __uint_as_float((uint32_t)v << 16) * (float)(1.0 / store_scale(I));
    }
    template <int I> __device__ static inline T enc(float g)
    {
        uint32_t u = __float_as_uint(g * (float)store_scale(I));
        if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40u);   // keep NaN a NaN
        u += 0x7fffu + ((u >> 16) & 1u);                                        // round to nearest even
        return (T)(u >> 16);
    }
};

// ------------------------------------------------------- compile-time loop
template <int I, int N> struct Unroll {
    template <class F> __device__ static inline void run(F &&f)
    {
        f(std::integral_constant<int, I>{});
        Unroll<I + 1, N>::run(f);
    }
};
template <int N> struct Unroll<N, N> {
    template <class F> __device__ static inline void run(F &&) {}
};

// ---------------------------------------------------------- raw moments
// Sums of g, xi g and xi xi g over the 27 directions, as three passes of
// 3-point sums (x, then y, then z).
struct Moments {
    float r1;                 // sum g = rho - 1
    float j[3];               // sum xi g = rho u
    float pxx, pyy, pzz, pxy, pxz, pyz;   // sum xi xi g
};

__device__ inline Moments raw_moments(const float g[Q])
{
    float s0[9], s1[9], s2[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        float a = g[3 * k], b = g[3 * k + 1], c = g[3 * k + 2];
        s0[k] = a + b + c;
        s1[k] = c - a;
        s2[k] = c + a;
    }
    float t00[3], t10[3], t20[3], t01[3], t02[3], t11[3];
#pragma unroll
    for (int kz = 0; kz < 3; kz++) {
        int r = 3 * kz;
        t00[kz] = s0[r] + s0[r + 1] + s0[r + 2];
        t10[kz] = s1[r] + s1[r + 1] + s1[r + 2];
        t20[kz] = s2[r] + s2[r + 1] + s2[r + 2];
        t01[kz] = s0[r + 2] - s0[r];
        t02[kz] = s0[r + 2] + s0[r];
        t11[kz] = s1[r + 2] - s1[r];
    }
    Moments m;
    m.r1 = t00[0] + t00[1] + t00[2];
    m.j[0] = t10[0] + t10[1] + t10[2];
    m.j[1] = t01[0] + t01[1] + t01[2];
    m.j[2] = t00[2] - t00[0];
    m.pxx = t20[0] + t20[1] + t20[2];
    m.pyy = t02[0] + t02[1] + t02[2];
    m.pzz = t00[2] + t00[0];
    m.pxy = t11[0] + t11[1] + t11[2];
    m.pxz = t10[2] - t10[0];
    m.pyz = t01[2] - t01[0];
    return m;
}

// Macroscopic state and the off-equilibrium second moment
//   P1 = sum xi xi (f - f0(rho,u)) = Pi' - cs^2 (rho - 1) I - rho u u,
// with Pi' = sum xi xi g (the weights carry cs^2 I).
struct Macro {
    float r1, rho, u[3];
    float P[3][3];
};

__device__ inline Macro macro(const Moments &m)
{
    Macro o;
    o.r1 = m.r1;
    o.rho = 1.0f + m.r1;
    float inv = 1.0f / o.rho;
#pragma unroll
    for (int a = 0; a < 3; a++) o.u[a] = m.j[a] * inv;
    float iso = CS2 * m.r1;
    o.P[0][0] = m.pxx - iso - m.j[0] * o.u[0];
    o.P[1][1] = m.pyy - iso - m.j[1] * o.u[1];
    o.P[2][2] = m.pzz - iso - m.j[2] * o.u[2];
    o.P[0][1] = o.P[1][0] = m.pxy - m.j[0] * o.u[1];
    o.P[0][2] = o.P[2][0] = m.pxz - m.j[0] * o.u[2];
    o.P[1][2] = o.P[2][1] = m.pyz - m.j[1] * o.u[2];
    return o;
}

// u^k for k in {0,1,2} per axis
struct Pow3 {
    float p[3][3];
    __device__ inline Pow3(const float u[3])
    {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            p[a][0] = 1.0f;
            p[a][1] = u[a];
            p[a][2] = u[a] * u[a];
        }
    }
    __device__ inline float mono(int mx, int my, int mz) const { return p[0][mx] * p[1][my] * p[2][mz]; }
};

// Hermite coefficients A_m (index m = mx + 3 my + 9 mz) of the collided state
// for equilibrium velocity ue (u or u + tau h), off-equilibrium built from
// P1 and u, relaxation factor om = 1 - 1/tau.
__device__ inline void post_collision_coeffs(const Macro &M, const float ue[3], float om, float A[Q])
{
    Pow3 pe(ue), pu(M.u);
#pragma unroll
    for (int m = 0; m < Q; m++) {
        const int mv[3] = {m % 3, (m / 3) % 3, m / 9};
        const int ord = mv[0] + mv[1] + mv[2];
        if (ord == 0) {
            A[m] = M.r1;
            continue;
        }
        float eq = M.rho * pe.mono(mv[0], mv[1], mv[2]);
        if (ord == 1) {
            A[m] = eq;
            continue;
        }
        // a1_m = sum over index pairs of P1 times the remaining u's
        float a1 = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (mv[a] == 2) {
                int r[3] = {mv[0], mv[1], mv[2]};
                r[a] -= 2;
                a1 += M.P[a][a] * pu.mono(r[0], r[1], r[2]);
            }
#pragma unroll
            for (int b = a + 1; b < 3; b++) {
                if (mv[a] && mv[b]) {
                    int r[3] = {mv[0], mv[1], mv[2]};
                    r[a] -= 1;
                    r[b] -= 1;
                    a1 += (float)(mv[a] * mv[b]) * M.P[a][b] * pu.mono(r[0], r[1], r[2]);
                }
            }
        }
        A[m] = eq + om * a1;
    }
}

// Difference of equilibria f0(rho, u + du) - f0(rho, u) in the Hermite basis.
__device__ inline void shift_coeffs(float rho, const float u[3], const float us[3], float A[Q])
{
    Pow3 ps(us), pu(u);
#pragma unroll
    for (int m = 0; m < Q; m++) {
        const int mx = m % 3, my = (m / 3) % 3, mz = m / 9;
        A[m] = (m == 0) ? 0.0f : rho * (ps.mono(mx, my, mz) - pu.mono(mx, my, mz));
    }
}

// Hermite coefficients -> populations (deviation form): three 3-point passes
// with e0 = 1, e1(-1,0,1) = (-3, 0, 3), e2(-1,0,1) = (3, -1.5, 3), then w_i.
__device__ inline void hermite_to_populations(const float A[Q], float out[Q])
{
    float T1[Q];   // [mx + 3 my + 9 kz]
#pragma unroll
    for (int k = 0; k < 9; k++) {
        float a0 = A[k], a1 = A[k + 9], a2 = A[k + 18];
        float s = a0 + 3.0f * a2;
        T1[k] = s - 3.0f * a1;
        T1[k + 9] = a0 - 1.5f * a2;
        T1[k + 18] = s + 3.0f * a1;
    }
    float T2[Q];   // [mx + 3 ky + 9 kz]
#pragma unroll
    for (int kz = 0; kz < 3; kz++)
#pragma unroll
        for (int mx = 0; mx < 3; mx++) {
            int b = mx + 9 * kz;
            float a0 = T1[b], a1 = T1[b + 3], a2 = T1[b + 6];
            float s = a0 + 3.0f * a2;
            T2[b] = s - 3.0f * a1;
            T2[b + 3] = a0 - 1.5f * a2;
            T2[b + 6] = s + 3.0f * a1;
        }
#pragma unroll
    for (int r = 0; r < 9; r++) {      // r = ky + 3 kz
        int b = 3 * r;
        float a0 = T2[b], a1 = T2[b + 1], a2 = T2[b + 2];
        float s = a0 + 3.0f * a2;
        out[b] = s - 3.0f * a1;
        out[b + 1] = a0 - 1.5f * a2;
        out[b + 2] = s + 3.0f * a1;
    }
#pragma unroll
    for (int i = 0; i < Q; i++) out[i] *= (float)wq(i);
}

// Relaxation time at physical height z: tau0 below the sponge, rising
// linearly to 1 on the top row inside it (Sec. 2.5).
// Periodic wrap of an index into [0, n).
__device__ inline int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ inline float tau_at(float tau0, int nz, int sponge, int z)
{
    if (sponge < 2) return tau0;
    int zs = nz - sponge;
    if (z < zs) return tau0;
    return tau0 + (1.0f - tau0) * (float)(z - zs) / (float)(nz - 1 - zs);
}

}  // namespace turret
