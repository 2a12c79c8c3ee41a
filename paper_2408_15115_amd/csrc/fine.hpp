// fine.hpp -- the full-precision box of the reduced-precision storage forms.
//
// With FP16 or BF16 population storage, each case with a body can keep a box
// of cells around it in FP32: the particle region of the coupling (the cells
// the stress, the interpolations and the forcing touch) plus a one-cell rim,
// so that every population those cells pull also comes from the box.  The
// rest of the lattice stays in the reduced-precision store, which always
// holds the rounding of every cell's value (also inside the box), so cells
// outside the box read exactly what a pure FP16/BF16 run would.
//
// Each population buffer has its own box: origin fo[buffer] (physical cell
// coordinates, x and y unwrapped and taken modulo the box size, z not
// wrapped), valid once a step has written it; edges LB[3] per case, the
// region edge plus two cells, at most the case's own size per axis.  Layout
// [27][LBz][LBy][LBx] FP32 per case at fine_off of each box buffer.
#pragma once
#include "internal.hpp"
#include "lattice.hpp"

namespace turret {

__device__ inline int wrap_mod(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

// Box slot of physical cell (x, y, z) for the box with origin fo, or -1.
__device__ inline int fine_slot(const CaseDev &cd, const int fo[3], int x, int y, int z)
{
    const int kx = wrap_mod(x - fo[0], cd.nx), ky = wrap_mod(y - fo[1], cd.ny), kz = z - fo[2];
    if (kx >= cd.LB[0] || ky >= cd.LB[1] || kz < 0 || kz >= cd.LB[2]) return -1;
    return (kz * cd.LB[1] + ky) * cd.LB[0] + kx;
}

__device__ inline long long fine_plane(const CaseDev &cd) { return (long long)cd.LB[0] * cd.LB[1] * cd.LB[2]; }

// The pull of pull.hpp in physical coordinates, with every read taken from
// the source buffer's box (FP32) where the source cell lies in it and from
// the reduced-precision store elsewhere.  fsrc == nullptr reads the store
// only.  The cell's place in the source box is found once; a source's is
// then that place minus xi (one wrap at the periodic x / y edges), so no
// division runs per population.
template <class CD>
__device__ inline void pull_fine(const typename CD::T *__restrict__ src, const float *__restrict__ fsrc,
                                 const CaseDev &cd, int z0, const int fo[3], int x, int y, int z, float g[Q])
{
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int LBx = cd.LB[0], LBy = cd.LB[1], LBz = cd.LB[2];
    const long long plane = cd.plane, fplane = fine_plane(cd);
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    const bool wlo = (z == 0) && cd.bc_lo != BC_PERIODIC;
    const bool whi = (z == nz - 1) && cd.bc_hi != BC_PERIODIC;
    // the cell in the source box (x, y modulo the case; z may lie outside)
    const int bx = fsrc ? wrap_mod(x - fo[0], nx) : 0, by = fsrc ? wrap_mod(y - fo[1], ny) : 0;
    const int bz = z - fo[2];
    Unroll<0, Q>::run([&](auto I) {
        constexpr int i = decltype(I)::value;
        int sx = cx(i) == 1 ? xm : (cx(i) == -1 ? xp : x);
        int sy = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
        int sz = cz(i) == 1 ? zm : (cz(i) == -1 ? zp : z);
        int kx = bx - cx(i), ky = by - cy(i), kz = bz - cz(i);
        int dir = i;
        bool neg = false;
        float add = 0.0f;
        if constexpr (cz(i) != 0) {
            const bool wall = cz(i) == 1 ? wlo : whi;
            const int bc = cz(i) == 1 ? cd.bc_lo : cd.bc_hi;
            if (wall) {
                sz = z;
                kz = bz;
                if (bc == BC_FREESLIP) {
                    dir = mirror_z(i);
                } else {
                    dir = opposite(i);
                    sx = x;
                    sy = y;
                    kx = bx;
                    ky = by;
                    neg = bc == BC_PRESSURE;
                    if constexpr (cx(i) != 0)
                        if (bc == BC_NOSLIP) add = (float)(6.0 * wq(i) * cx(i)) * (cz(i) == 1 ? cd.uw_lo : cd.uw_hi);
                }
            }
        }
        // periodic x / y: one wrap at the case's edge
        kx = kx < 0 ? kx + nx : (kx >= nx ? kx - nx : kx);
        ky = ky < 0 ? ky + ny : (ky >= ny ? ky - ny : ky);
        if (cz(i) != 0 && sz != z + (cz(i) == 1 ? -1 : 1) && sz != z) kz = sz - fo[2];   // periodic z wrap
        float v;
        if (fsrc && kx < LBx && ky < LBy && kz >= 0 && kz < LBz) {
            v = fsrc[(long long)dir * fplane + (kz * LBy + ky) * LBx + kx];
        } else {
            int zc = sz + z0;
            if (zc >= nz) zc -= nz;
            // mirror and opposite directions share the storage scale of i
            v = CD::template dec<i>(src[(long long)dir * plane + (long long)((zc * ny + sy) * nx + sx)]);
        }
        g[i] = (neg ? -v : v) + add;
    });
}

}  // namespace turret
