// stream_collide19.hip -- the fused pull-streaming + collision kernel on the
// D3Q19 lattice, the lattice the paper sets its D3Q27 choice against for
// stability (arXiv 2408.15115, Sec. 2.1).  Fluid-only contexts, FP32
// deviation storage, periodic in x, y and z; one thread per cell over the same
// tile table and SoA layout [19][nz][ny][nx] as the D3Q27 kernel.
//
// Velocities: {-1, 0, 1}^3 with |xi|^2 <= 2, in the D3Q27 order
// 9 (xi_z + 1) + 3 (xi_y + 1) + (xi_x + 1) with the corners left out; weights
// 1/3, 1/18, 1/36; cs^2 = 1/3.
//
// Model (the App. A construction on the Hermite polynomials D3Q19 carries):
// orders 0..2 in full; at third order the pairs (H_xxy, H_yzz),
// (H_yyz, H_xxz), (H_zzx, H_xyy), which are not orthogonal on these
// velocities, enter through their sum S and difference D (orthogonal, lattice
// norms 2 cs^6 and 6 cs^6); no fourth order.  The third-order coefficients
// are rho u_a u_a u_b (equilibrium) and, for the regularized non-equilibrium
// part, the recursion a_aab = P1_aa u_b + 2 u_a P1_ab.
// COLL 0: recursive regularized, f0 + (1 - 1/tau) f1; COLL 1: BGK.
#include "internal.hpp"

namespace turret {
namespace q19 {

constexpr int N = 19;
struct Vel {
    int x[N], y[N], z[N];
    float w[N];
};
constexpr Vel make_vel()
{
    Vel v{};
    int j = 0;
    for (int z = -1; z <= 1; z++)
        for (int y = -1; y <= 1; y++)
            for (int x = -1; x <= 1; x++) {
                const int n = x * x + y * y + z * z;
                if (n == 3) continue;
                v.x[j] = x;
                v.y[j] = y;
                v.z[j] = z;
                v.w[j] = n == 0 ? 1.0f / 3.0f : (n == 1 ? 1.0f / 18.0f : 1.0f / 36.0f);
                j++;
            }
    return v;
}
constexpr Vel V = make_vel();
constexpr float CS2 = 1.0f / 3.0f;

__device__ __forceinline__ int wrap(int v, int n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

}  // namespace q19

// Per cell, with j = sum xi g (= rho u) and the constants 1/cs^2 = 3,
// 1/(2 cs^4) = 4.5 folded in, both models write
//   out_i = w_i [dr - C0 + 3 xi.j + xi xi : Q + sum_pairs (k1 H_1 + k2 H_2)]
// RR:  Q = 4.5 (rho uu + om P1),  C0 = 1.5 (rho u^2 + om tr P1), and the
//      third-order pair coefficients of a = a0 + om a1; BGK: the equilibrium
//      alone (om = 0), then out = geq + om (g - geq).
// The moments on S and D, (a_1 + a_2) / (2 cs^6) and (a_1 - a_2) / (6 cs^6),
// recombine on H_1 and H_2 as k1 = 18 a_1 + 9 a_2, k2 = 9 a_1 + 18 a_2.
template <int COLL>
__global__ void __launch_bounds__(256) k_stream_collide19(const float *__restrict__ src, float *__restrict__ dst,
                                                          const CaseDev *__restrict__ cases, BodyDev *__restrict__ body,
                                                          const Tile *__restrict__ tiles)
{
    using namespace q19;
    const Tile tl = tiles[blockIdx.x];
    const CaseDev &cd = cases[tl.c];
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int cell = tl.first + (int)threadIdx.x;
    if (body[tl.c].err != 0 || cell >= (int)cd.cells) return;
    const int z0 = body[tl.c].z0;
    const int x = cell % nx, t2 = cell / nx, y = t2 % ny, z = t2 / ny;
    // periodic neighbours; physical row z sits in ring slot (z + z0) mod nz
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    int zc = z + z0;
    if (zc >= nz) zc -= nz;
    const int zlo = zc == 0 ? nz - 1 : zc - 1, zhi = zc == nz - 1 ? 0 : zc + 1;
    const int rowc = zc * ny, rowlo = zlo * ny, rowhi = zhi * ny;
    const float *s = src + cd.pop_off;
    const long long plane = cd.plane;
    float g[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int sx = V.x[i] == 1 ? xm : (V.x[i] == -1 ? xp : x);
        const int sy = V.y[i] == 1 ? ym : (V.y[i] == -1 ? yp : y);
        const int sr = V.z[i] == 1 ? rowlo : (V.z[i] == -1 ? rowhi : rowc);
        g[i] = s[(long long)i * plane + ((sr + sy) * nx + sx)];
    }
    // moments of the deviations g = f - w
    float dr = 0.0f, j[3] = {0.0f, 0.0f, 0.0f}, Pg[3][3] = {};
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int xi[3] = {V.x[i], V.y[i], V.z[i]};
        dr += g[i];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (xi[a] != 0) j[a] += xi[a] > 0 ? g[i] : -g[i];
#pragma unroll
            for (int b = a; b < 3; b++)
                if (xi[a] * xi[b] != 0) Pg[a][b] += xi[a] * xi[b] > 0 ? g[i] : -g[i];
        }
    }
    const float rho = 1.0f + dr, inv = 1.0f / rho;
    const float u[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
    const float u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const bool bad = !(fabsf(dr) < 1.0f) || !(u2 < 0.25f);
    const unsigned long long m = __ballot(bad);
    if (m != 0ull && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) atomicOr(&body[tl.c].err, 4);
    const float tau = cd.tau0, om = 1.0f - 1.0f / tau;
    // rho u_a u_b = j_a u_b; P1 = sum xi xi g - rho uu - dr cs^2 I (sum xi xi w = cs^2 I)
    float ruu[3][3], P1[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = a; b < 3; b++) {
            ruu[a][b] = ruu[b][a] = j[a] * u[b];
            P1[a][b] = P1[b][a] = Pg[a][b] - j[a] * u[b] - (a == b ? dr * CS2 : 0.0f);
        }
    const float omr = COLL == 1 ? 0.0f : om;   // weight of the non-equilibrium part in out
    float Qm[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) Qm[a][b] = 4.5f * (ruu[a][b] + omr * P1[a][b]);
    const float C0 = 1.5f * (ruu[0][0] + ruu[1][1] + ruu[2][2] + omr * (P1[0][0] + P1[1][1] + P1[2][2]));
    // third-order pairs (a, a, b) / (b, c, c): a0 = rho u u u, a1 from the recursion
    constexpr int PA[3] = {0, 1, 2}, PB[3] = {1, 2, 0}, PC[3] = {2, 0, 1};
    float k1[3], k2[3];
#pragma unroll
    for (int p = 0; p < 3; p++) {
        const int a = PA[p], b = PB[p], c = PC[p];
        float a1 = ruu[a][a] * u[b], a2 = ruu[c][c] * u[b];
        if constexpr (COLL != 1) {
            a1 += om * (P1[a][a] * u[b] + 2.0f * u[a] * P1[a][b]);
            a2 += om * (2.0f * u[c] * P1[b][c] + u[b] * P1[c][c]);
        }
        k1[p] = 18.0f * a1 + 9.0f * a2;
        k2[p] = 9.0f * a1 + 18.0f * a2;
    }
    const float base = dr - C0;
    float out[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int xi[3] = {V.x[i], V.y[i], V.z[i]};
        float v = base;
#pragma unroll
        for (int a = 0; a < 3; a++)
            if (xi[a] != 0) v += xi[a] > 0 ? 3.0f * j[a] : -3.0f * j[a];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++)
                if (xi[a] * xi[b] != 0) v += xi[a] * xi[b] > 0 ? Qm[a][b] : -Qm[a][b];
#pragma unroll
        for (int p = 0; p < 3; p++) {
            const int a = PA[p], b = PB[p], c = PC[p];
            // H_1 = xi_b (xi_a^2 - cs^2), H_2 = xi_b (xi_c^2 - cs^2): constants
            if (xi[b] != 0) {
                const float h1 = (float)xi[b] * ((float)(xi[a] * xi[a]) - CS2);
                const float h2 = (float)xi[b] * ((float)(xi[c] * xi[c]) - CS2);
                v += h1 * k1[p] + h2 * k2[p];
            }
        }
        const float eq = V.w[i] * v;
        if constexpr (COLL == 1)
            out[i] = eq + om * (g[i] - eq);
        else
            out[i] = eq;
    }
    float *d = dst + cd.pop_off + (rowc + y) * nx + x;
#pragma unroll
    for (int i = 0; i < N; i++) __builtin_nontemporal_store(out[i], &d[(long long)i * plane]);
}

hipError_t launch_stream_collide19(const void *src, void *dst, const DevPtrs &p, int ntiles, int block,
                                   int collision, hipStream_t s)
{
    if (collision == 1)
        hipLaunchKernelGGL(k_stream_collide19<1>, dim3(ntiles), dim3(block), 0, s, (const float *)src, (float *)dst,
                           p.cases, p.body, p.tiles);
    else
        hipLaunchKernelGGL(k_stream_collide19<0>, dim3(ntiles), dim3(block), 0, s, (const float *)src, (float *)dst,
                           p.cases, p.body, p.tiles);
    return hipGetLastError();
}

}  // namespace turret
