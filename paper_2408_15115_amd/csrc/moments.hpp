// moments.hpp -- device helpers of moment storage (arXiv 2408.15115, App. A
// and Sec. 2.2), shared by the z-marching step and the coupling kernels.
//
// A cell stores m = (rho - 1, rho u, (1 - 1/tau) P1): the regularized
// post-collision state C = f0(rho, u) + (1 - 1/tau) f1(P1, u).  A cell that
// carried an immersed force in the last step holds the forced state of
// Sec. 2.2 instead, C + f0(rho, u + tau h) - f0(rho, u) (in the
// momentum-exact variant less the first-order term (tau - 1) rho h); its
// shift is kept beside the moments in the forcing box of its case:
// (Delta = tau h, lambda) with lambda = 1, or 1 / tau in the momentum-exact
// variant.  In Hermite coefficients the forced state is
//   A_m = rho (u + Delta)^m + a1_m(P, u),  A_e_a = rho (u_a + lambda Delta_a).
#pragma once
#include "internal.hpp"
#include "lattice.hpp"

namespace turret {
namespace mom {

// Hermite coefficients of the stored state with the cell's shift sh
// ({0, 0, 0, 1} for a cell without one: then exactly the unforced state).
__device__ __forceinline__ void state_coeffs(const float m[10], const float sh[4], float A[Q])
{
    Macro M;
    M.r1 = m[0];
    M.rho = 1.0f + m[0];
    const float inv = 1.0f / M.rho;
    M.u[0] = m[1] * inv;
    M.u[1] = m[2] * inv;
    M.u[2] = m[3] * inv;
    M.P[0][0] = m[4];
    M.P[1][1] = m[5];
    M.P[2][2] = m[6];
    M.P[0][1] = M.P[1][0] = m[7];
    M.P[0][2] = M.P[2][0] = m[8];
    M.P[1][2] = M.P[2][1] = m[9];
    const float ue[3] = {M.u[0] + sh[0], M.u[1] + sh[1], M.u[2] + sh[2]};
    post_collision_coeffs(M, ue, 1.0f, A);
    const float k = M.rho * (1.0f - sh[3]);
    A[1] -= k * sh[0];
    A[3] -= k * sh[1];
    A[9] -= k * sh[2];
}

// Deviations C - w of the 27 collided populations.
__device__ __forceinline__ void expand(const float m[10], const float sh[4], float out[Q])
{
    float A[Q];
    state_coeffs(m, sh, A);
    hermite_to_populations(A, out);
}

// Collide: raw moments of the pulled deviations -> the stored post-collision state.
__device__ __forceinline__ void collide_to_moments(const Moments &rm, float om, float m[10], bool &bad)
{
    const Macro M = macro(rm);
    const float u2 = M.u[0] * M.u[0] + M.u[1] * M.u[1] + M.u[2] * M.u[2];
    bad = !(fabsf(M.r1) < 1.0f) || !(u2 < 0.25f);
    m[0] = M.r1;
    m[1] = rm.j[0];
    m[2] = rm.j[1];
    m[3] = rm.j[2];
    m[4] = om * M.P[0][0];
    m[5] = om * M.P[1][1];
    m[6] = om * M.P[2][2];
    m[7] = om * M.P[0][1];
    m[8] = om * M.P[0][2];
    m[9] = om * M.P[1][2];
}

// The forcing box of a case: the particle region of the step that wrote it,
// origin in (x, y, ring slot) coordinates, edge L; shifts as [4][L^3].
struct ShiftBox {
    int o[3], L, valid;
    const float *d;
    long long L3;
};

__device__ __forceinline__ ShiftBox shift_box(const DevPtrs &p, const CaseDev &cd, const BodyDev &B)
{
    ShiftBox s;
    s.valid = B.dvalid && cd.M > 0;
    s.L = cd.L;
    s.L3 = (long long)cd.L * cd.L * cd.L;
    s.o[0] = B.dorg[0];
    s.o[1] = B.dorg[1];
    s.o[2] = B.dorg[2];
    s.d = p.dsh + cd.reg_off * 4;
    return s;
}

// The shift of the cell at (x, y, ring slot zs) into sh; sh = {0, 0, 0, 1}
// and false where there is none.
__device__ __forceinline__ bool shift_at(const ShiftBox &s, int nx, int ny, int nz, int x, int y, int zs, float sh[4])
{
    sh[0] = sh[1] = sh[2] = 0.0f;
    sh[3] = 1.0f;
    if (!s.valid) return false;
    int a = x - s.o[0], b = y - s.o[1], c = zs - s.o[2];
    a = a < 0 ? a + nx : a;
    b = b < 0 ? b + ny : b;
    c = c < 0 ? c + nz : c;
    if (a >= s.L || b >= s.L || c >= s.L) return false;
    const long long q = ((long long)c * s.L + b) * s.L + a;
    sh[0] = s.d[q];
    sh[1] = s.d[s.L3 + q];
    sh[2] = s.d[2 * s.L3 + q];
    sh[3] = s.d[3 * s.L3 + q];
    return sh[0] != 0.0f || sh[1] != 0.0f || sh[2] != 0.0f;
}

}  // namespace mom
}  // namespace turret
