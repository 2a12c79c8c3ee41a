// moments.hip -- moment-space storage of the D3Q27 recursive-regularized
// step (arXiv 2408.15115, App. A): the collided populations are
// C = f0(rho, u) + (1 - 1/tau) f1(P1, u), a function of rho, u and the
// off-equilibrium stress P1 alone, so a cell's post-collision state is fully
// given by ten numbers.  Stored per cell (FP32, SoA [10][nz][ny][nx]):
//   m0 = rho - 1,  m1..3 = rho u,  m4..9 = (1 - 1/tau) P1 as xx, yy, zz, xy, xz, yz.
// The step reads 40 bytes and writes 40 bytes per cell instead of 27 + 27
// populations.  Periodic in x and y; z periodic or bounded by the walls of the
// lattice kernel (free-slip, no-slip at rest or moving in x, constant
// pressure).  Cells forced in the last step carry their equilibrium shift in
// the forcing box of their case (moments.hpp); the expansion applies it.
//
// The step marches in z.  A workgroup owns a column of MX x MY cells and a
// chunk of LZ output planes.  For each plane it expands the stored moments of
// the (MX + 2) x (MY + 2) halo into all 27 collided populations (the
// regularized reconstruction) in LDS; each output cell adds the populations it
// pulls from that plane into partial moment sums of three output planes, and
// the plane whose sums are complete collides and is stored.  The next plane's
// moments are loaded before the gather so that the HBM reads overlap it.
#include "internal.hpp"
#include "lattice.hpp"
#include "moments.hpp"

namespace turret {

namespace mom {
#ifndef TURRET_MOM_TILE
#define TURRET_MOM_TILE 32, 13, 32, 512
#endif
// x, y extent of a column tile; z planes per chunk; threads per workgroup
constexpr int kTile[4] = {TURRET_MOM_TILE};
constexpr int MX = kTile[0], MY = kTile[1], LZ = kTile[2];
constexpr int HX = MX + 2, HY = MY + 2, NH = HX * HY;   // halo cells, one per thread
constexpr int kBlock = kTile[3];
static_assert(NH <= kBlock && MX * MY <= kBlock, "tile does not fit the workgroup");

__device__ __forceinline__ int wrap1(int v, int n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Partial raw moments of the nine pulled populations with xi_z = CZ (from
// one source plane) added into acc (r1, j, pxx, pyy, pzz, pxy, pxz, pyz).
template <int CZ>
__device__ __forceinline__ void add_group(const float (*L)[NH], int ix, int iy, float acc[10])
{
    float s0 = 0.0f, sx = 0.0f, sy = 0.0f, sxx = 0.0f, syy = 0.0f, sxy = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const int ex = k % 3 - 1, ey = k / 3 - 1;
        const float v = L[9 * (CZ + 1) + k][(iy + 1 - ey) * HX + (ix + 1 - ex)];
        s0 += v;
        if (ex != 0) {
            sx += ex > 0 ? v : -v;
            sxx += v;
        }
        if (ey != 0) {
            sy += ey > 0 ? v : -v;
            syy += v;
        }
        if (ex * ey != 0) sxy += ex * ey > 0 ? v : -v;
    }
    acc[0] += s0;
    acc[1] += sx;
    acc[2] += sy;
    acc[4] += sxx;
    acc[5] += syy;
    acc[7] += sxy;
    if (CZ != 0) {
        acc[3] += CZ > 0 ? s0 : -s0;
        acc[6] += s0;
        acc[8] += CZ > 0 ? sx : -sx;
        acc[9] += CZ > 0 ? sy : -sy;
    }
}
// The nine populations with xi_z = CZ that a z wall supplies to its boundary
// row (CZ = +1 at the bottom, -1 at the top), from the plane of that row:
// free-slip, the mirrored direction (xi_z reversed) of the lateral
// neighbour; no-slip, the opposite direction of the cell itself plus the
// moving wall's momentum 6 w_i xi_x u_w; constant pressure, the opposite
// direction of the cell itself with its sign reversed (deviation form).
template <int CZ>
__device__ __forceinline__ void add_wall(const float (*L)[NH], int bc, float uw, int ix, int iy, float acc[10])
{
    float s0 = 0.0f, sx = 0.0f, sy = 0.0f, sxx = 0.0f, syy = 0.0f, sxy = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const int ex = k % 3 - 1, ey = k / 3 - 1;
        const int i = 9 * (CZ + 1) + k;
        float v;
        if (bc == BC_FREESLIP) {
            v = L[9 * (1 - CZ) + k][(iy + 1 - ey) * HX + (ix + 1 - ex)];
        } else {
            v = L[Q - 1 - i][(iy + 1) * HX + (ix + 1)];
            if (bc == BC_PRESSURE) v = -v;
            else if (ex != 0) v += (float)(6.0 * wq(i) * ex) * uw;
        }
        s0 += v;
        if (ex != 0) {
            sx += ex > 0 ? v : -v;
            sxx += v;
        }
        if (ey != 0) {
            sy += ey > 0 ? v : -v;
            syy += v;
        }
        if (ex * ey != 0) sxy += ex * ey > 0 ? v : -v;
    }
    acc[0] += s0;
    acc[1] += sx;
    acc[2] += sy;
    acc[4] += sxx;
    acc[5] += syy;
    acc[7] += sxy;
    acc[3] += CZ > 0 ? s0 : -s0;
    acc[6] += s0;
    acc[8] += CZ > 0 ? sx : -sx;
    acc[9] += CZ > 0 ? sy : -sy;
}
}  // namespace mom

// Tile t of a case: x fastest, then y, then the z chunk.  Workgroups are
// spread over the 8 XCDs round-robin; block b takes table entry
// (b mod 8) * ceil(n / 8) + b / 8, so that each XCD's L2 serves a contiguous
// run of neighbouring tiles and their shared halo rows.
//
// Pull: output plane o takes population i from plane o - xi_z.  So the plane
// z just expanded feeds three outputs: its xi_z = -1 group completes plane
// z - 1, its xi_z = 0 group goes to plane z, its xi_z = +1 group starts plane
// z + 1.  Raw moments are linear in the populations, so each output cell
// keeps partial moment sums for planes z - 1, z and z + 1 in registers and
// only the newest expanded plane is held in LDS.
__global__ void __launch_bounds__(mom::kBlock) k_moment_step(const float *__restrict__ src, float *__restrict__ dst,
                                                             DevPtrs p, int ntiles)
{
    using namespace mom;
    const CaseDev *__restrict__ cases = p.cases;
    BodyDev *__restrict__ body = p.body;
    const Tile *__restrict__ tiles = p.tiles;
    const int b = blockIdx.x;
    const int ti = (b & 7) * ((ntiles + 7) >> 3) + (b >> 3);
    if (ti >= ntiles) return;
    const Tile tl = tiles[ti];
    const CaseDev &cd = cases[tl.c];
    if (body[tl.c].err != 0) return;
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int ntx = (nx + MX - 1) / MX, nty = (ny + MY - 1) / MY;
    const int x0 = (tl.first % ntx) * MX, y0 = ((tl.first / ntx) % nty) * MY, zs = (tl.first / (ntx * nty)) * LZ;
    const int ze = min(zs + LZ, nz);
    const long long plane = cd.plane;
    const float *s = src + cd.pop_off;
    float *d = dst + cd.pop_off;

    __shared__ float L[Q][NH];   // the 27 collided populations of the newest plane

    const int t = threadIdx.x;
    const bool halo = t < NH;
    // halo coordinates may pass the box more than once when it is narrower than the tile
    const int gx = ((x0 - 1 + t % HX) % nx + nx) % nx, gy = ((y0 - 1 + t / HX) % ny + ny) % ny;
    const int hoff = gy * nx + gx;
    const int ix = t % MX, iy = t / MX;
    const bool out = t < MX * MY && x0 + ix < nx && y0 + iy < ny;

    // z walls: planes -1 and nz exist only when z is periodic; physical
    // plane z is stored in ring slot (z + z0) mod nz
    const bool wlo = cd.bc_lo != BC_PERIODIC, whi = cd.bc_hi != BC_PERIODIC;
    const int z0 = body[tl.c].z0;
    auto exists = [&](int z) { return (z >= 0 || !wlo) && (z < nz || !whi); };
    auto slot = [&](int z) { return wrap1(wrap1(z, nz) + z0, nz); };
    const ShiftBox sb = shift_box(p, cd, body[tl.c]);   // forcing shifts of the last correction
    float m[10];
    if (halo && exists(zs - 1)) {
        const float *sp = s + (long long)slot(zs - 1) * ny * nx + hoff;
#pragma unroll
        for (int c = 0; c < 10; c++) m[c] = sp[c * plane];
    }
    float a[10], bq[10], cq[10];   // partial raw moments of output planes z - 1, z, z + 1
#pragma unroll
    for (int c = 0; c < 10; c++) a[c] = bq[c] = cq[c] = 0.0f;
    for (int z = zs - 1; z <= ze; z++) {
        const bool have = exists(z);   // the same for the whole workgroup
        if (halo && have) {
            float c[Q], sh[4];
            (void)shift_at(sb, nx, ny, nz, gx, gy, slot(z), sh);
            expand(m, sh, c);
#pragma unroll
            for (int i = 0; i < Q; i++) L[i][t] = c[i];
        }
        if (halo && z < ze && exists(z + 1)) {   // prefetch plane z + 1
            const float *sp = s + (long long)slot(z + 1) * ny * nx + hoff;
#pragma unroll
            for (int c2 = 0; c2 < 10; c2++) m[c2] = sp[c2 * plane];
        }
        __syncthreads();
        if (out) {
            if (have) {
                add_group<-1>(L, ix, iy, a);
                add_group<0>(L, ix, iy, bq);
                add_group<1>(L, ix, iy, cq);
                if (z == 0 && wlo) add_wall<1>(L, cd.bc_lo, cd.uw_lo, ix, iy, bq);
                if (z == nz - 1 && whi) add_wall<-1>(L, cd.bc_hi, cd.uw_hi, ix, iy, bq);
            }
            if (z - 1 >= zs) {   // plane z - 1 is complete
                const int zo = z - 1;
                Moments rm;
                rm.r1 = a[0];
                rm.j[0] = a[1];
                rm.j[1] = a[2];
                rm.j[2] = a[3];
                rm.pxx = a[4];
                rm.pyy = a[5];
                rm.pzz = a[6];
                rm.pxy = a[7];
                rm.pxz = a[8];
                rm.pyz = a[9];
                const float om = 1.0f - 1.0f / tau_at(cd.tau0, nz, cd.sponge, zo);
                float mo[10];
                bool bad;
                collide_to_moments(rm, om, mo, bad);
                const unsigned long long bm = __ballot(bad);
                if (bm != 0ull && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)bm) - 1)
                    atomicOr(&body[tl.c].err, 4);
                float *dp = d + ((long long)slot(zo) * ny + (y0 + iy)) * nx + (x0 + ix);
#pragma unroll
                for (int c = 0; c < 10; c++) __builtin_nontemporal_store(mo[c], &dp[c * plane]);
            }
        }
#pragma unroll
        for (int c = 0; c < 10; c++) {
            a[c] = bq[c];
            bq[c] = cq[c];
            cq[c] = 0.0f;
        }
        __syncthreads();
    }
}

// Moments (and forcing shifts) -> population deviations of case c, layout
// [27][plane] in the ring order of the storage.
__global__ void __launch_bounds__(256) k_moments_expand(const float *__restrict__ src, float *__restrict__ dst,
                                                        DevPtrs p, int c)
{
    const CaseDev cd = p.cases[c];
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= cd.cells) return;
    const long long plane = cd.plane;
    const int x = (int)(i % cd.nx), y = (int)((i / cd.nx) % cd.ny), zs = (int)(i / ((long long)cd.nx * cd.ny));
    const mom::ShiftBox sb = mom::shift_box(p, cd, p.body[c]);
    float m[10], sh[4], out[Q];
#pragma unroll
    for (int k = 0; k < 10; k++) m[k] = src[k * plane + i];
    (void)mom::shift_at(sb, cd.nx, cd.ny, cd.nz, x, y, zs, sh);
    mom::expand(m, sh, out);
#pragma unroll
    for (int k = 0; k < Q; k++) dst[k * plane + i] = out[k];
}

// Population deviations of post-collision states -> stored moments: rho - 1,
// rho u and the off-equilibrium stress about f0(rho, u).  Exact for
// regularized states; any other state is replaced by its regularized part.
__global__ void __launch_bounds__(256) k_moments_project(const float *__restrict__ src, float *__restrict__ dst,
                                                         long long plane, long long cells)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= cells) return;
    float g[Q], m[10];
#pragma unroll
    for (int k = 0; k < Q; k++) g[k] = src[k * plane + i];
    bool bad;
    mom::collide_to_moments(raw_moments(g), 1.0f, m, bad);
#pragma unroll
    for (int k = 0; k < 10; k++) dst[k * plane + i] = m[k];
}

int moment_tiles(int nx, int ny, int nz)
{
    return ((nx + mom::MX - 1) / mom::MX) * ((ny + mom::MY - 1) / mom::MY) * ((nz + mom::LZ - 1) / mom::LZ);
}

hipError_t launch_moment_step(const void *src, void *dst, const DevPtrs &p, int ntiles, hipStream_t s)
{
    const int grid = (ntiles + 7) / 8 * 8;
    hipLaunchKernelGGL(k_moment_step, dim3(grid), dim3(mom::kBlock), 0, s, (const float *)src, (float *)dst, p, ntiles);
    return hipGetLastError();
}

hipError_t launch_moments_expand(const float *src, float *dst, const DevPtrs &p, int c, hipStream_t s)
{
    CaseDev cd;
    hipError_t e = hipMemcpy(&cd, p.cases + c, sizeof cd, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    const long long grid = (cd.cells + 255) / 256;
    hipLaunchKernelGGL(k_moments_expand, dim3((unsigned)grid), dim3(256), 0, s, src, dst, p, c);
    return hipGetLastError();
}

hipError_t launch_moments_expand_n(const float *src, float *dst, const DevPtrs &p, int c, long long cells,
                                   hipStream_t s)
{
    const long long grid = (cells + 255) / 256;
    hipLaunchKernelGGL(k_moments_expand, dim3((unsigned)grid), dim3(256), 0, s, src, dst, p, c);
    return hipGetLastError();
}

hipError_t launch_moments_project(const float *src, float *dst, long long plane, long long cells, hipStream_t s)
{
    const long long grid = (cells + 255) / 256;
    hipLaunchKernelGGL(k_moments_project, dim3((unsigned)grid), dim3(256), 0, s, src, dst, plane, cells);
    return hipGetLastError();
}

}  // namespace turret
