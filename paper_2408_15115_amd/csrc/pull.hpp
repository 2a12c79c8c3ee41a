// pull.hpp -- pull streaming with the boundary rules of the domain
// (arXiv 2408.15115, Sec. 2.1 and Sec. 2.5), shared by the lattice kernel and
// the particle-region gather.
#pragma once
#include "internal.hpp"
#include "lattice.hpp"

namespace turret {

// ------------------------------------------------------------------ pull
// The 27 populations arriving at cell (x, y, z): g_i = C_i(x - xi_i) from the
// previous post-collision buffer.  x, y periodic; at the z walls the missing
// population comes from specular reflection (free-slip: C_{mirror_z(i)} of the
// lateral neighbour in the same row), bounce-back (no-slip: C_{opposite(i)}
// of the cell itself) or anti-bounce-back at density 1 (constant pressure:
// f_i = -C_{opposite(i)} + 2 w_i, i.e. g_i = -g^C_{opposite(i)} in deviation
// form); periodic z wraps.  A no-slip wall may move in x at uw_lo / uw_hi:
// bounce-back then adds the wall's momentum, 6 w_i rho0 (xi_i . u_w) with
// rho0 = 1.  Physical row z sits in ring slot (z + z0) mod nz.
template <class CD>
__device__ inline void pull(const typename CD::T *__restrict__ src, long long plane, int nx, int ny, int nz,
                            int z0, int bc_lo, int bc_hi, float uw_lo, float uw_hi, int x, int y, int z, float g[Q])
{
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    int zc = z + z0;
    if (zc >= nz) zc -= nz;
    const int zlo = zc == 0 ? nz - 1 : zc - 1;
    const int zhi = zc == nz - 1 ? 0 : zc + 1;
    const bool wlo = (z == 0) && bc_lo != BC_PERIODIC;
    const bool whi = (z == nz - 1) && bc_hi != BC_PERIODIC;
    const int rowc = zc * ny, rowlo = zlo * ny, rowhi = zhi * ny;
    Unroll<0, Q>::run([&](auto I) {
        constexpr int i = decltype(I)::value;
        int sx = cx(i) == 1 ? xm : (cx(i) == -1 ? xp : x);
        int sy = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
        int srow = cz(i) == 1 ? rowlo : (cz(i) == -1 ? rowhi : rowc);
        int dir = i;
        bool neg = false;
        float add = 0.0f;
        if constexpr (cz(i) != 0) {
            const bool wall = cz(i) == 1 ? wlo : whi;
            const int bc = cz(i) == 1 ? bc_lo : bc_hi;
            if (wall) {
                srow = rowc;
                if (bc == BC_FREESLIP) {
                    dir = mirror_z(i);
                } else {
                    dir = opposite(i);
                    sx = x;
                    sy = y;
                    neg = bc == BC_PRESSURE;
                    if constexpr (cx(i) != 0)
                        if (bc == BC_NOSLIP) add = (float)(6.0 * wq(i) * cx(i)) * (cz(i) == 1 ? uw_lo : uw_hi);
                }
            }
        }
        const float v = CD::template dec<i>(src[(long long)dir * plane + (long long)((srow + sy) * nx + sx)]);
        g[i] = (neg ? -v : v) + add;
    });
}

}  // namespace turret
